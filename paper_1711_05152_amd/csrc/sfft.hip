// Alg. 3 (dimension-incremental sparse FFT on multiple rank-1 lattices): placeholder until the
// driver lands.
#include "runtime.h"

using namespace mr1l;

extern "C" mr1l_status sfft_detect(int d, const int32_t* lo, const int32_t* hi, sfft_sampler_fn sampler, void* user,
                                   const sfft_planted* planted, const sfft_params* params, int64_t cap,
                                   int64_t* n_out, int32_t* freqs_out, double* coeffs_out, sfft_stats* stats,
                                   int device) {
    (void)d; (void)lo; (void)hi; (void)sampler; (void)user; (void)planted; (void)params; (void)cap;
    (void)n_out; (void)freqs_out; (void)coeffs_out; (void)stats; (void)device;
    set_error("sfft_detect is not built yet");
    return MR1L_ERR_UNSUPPORTED;
}
