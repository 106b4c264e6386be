// Launchers of the sparse-FFT device passes (k_sfft.hip).  dt is an mr1l_dtype, kt a KType.
#pragma once

#include "common.h"
#include "mr1l.h"

namespace mr1l {

void sf_planted_w1d(const int32_t* hf, int64_t s, int d, const void* c, const double* anchors, const int* comp,
                    int njobs, void* w, hipStream_t st);
void sf_planted_1d(int dt, const int32_t* hf, int64_t s, const void* w, const int* comp, int njobs, int64_t K,
                   const uint64_t* keys, double sigma, void* y, hipStream_t st);
void sf_planted_wlat(int dt, const int32_t* hf, int64_t s, int d, int t, const void* c, const double* anchors, int nrep,
                     void* w, hipStream_t st);
void sf_add_noise(int dt, void* y, int64_t len, int nrep, const uint64_t* keys, double sigma, hipStream_t st);
void sf_nodes_lattice(const int64_t* M, const int64_t* off, const int64_t* z, int L, int64_t maxM, int t, int d,
                      const double* anchors, double* nodes, const int* col, hipStream_t st);
void sf_nodes_1d(int64_t K, int tc, int d, const double* anchors, double* nodes, const int* col, hipStream_t st);
void sf_select(int dt, const void* coeffs, int64_t n, int64_t n_rhs, double delta, int64_t s, uint8_t* flags,
               int rhs_per_group, int64_t flags_stride, hipStream_t st);
void sf_compact(const uint8_t* flags, int64_t n, int32_t* idx, int64_t* count, hipStream_t st);
void sf_product(int kt, const void* P, int64_t n1, const int32_t* Q, int64_t n2, int t, void* J, hipStream_t st);
void sf_gather_rows(int kt, const void* J, int64_t nJ, int t, const int32_t* idx, int64_t m, void* out, hipStream_t st);
void sf_flags_to_values(const int32_t* idx, int64_t m, int32_t lo, int32_t* vals, hipStream_t st);
void sf_values_to_k(int kt, const int32_t* v, int64_t m, void* out, hipStream_t st);
void sf_gather_coeffs(int dt, const void* c, const int32_t* idx, int64_t m, void* out, hipStream_t st);
void sf_soa_to_rows(int kt, const void* f, int64_t m, int d, int32_t* rows, hipStream_t st);

}  // namespace mr1l
