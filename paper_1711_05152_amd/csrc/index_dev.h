// Device helpers for exact residues k . z mod M and alias-bitmap lookups.
#pragma once

#include "common.h"

namespace mr1l {

template <typename K>
__device__ __forceinline__ int64_t dot_kz(const K* __restrict__ f, int64_t nf, int d, int64_t g,
                                          const int64_t* __restrict__ z) {
    // components loaded in groups of 8 so that their loads are in flight together
    int64_t s = 0;
    int c = 0;
    for (; c + 8 <= d; c += 8) {
        int64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = (int64_t)f[(c + u) * nf + g];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u] * z[c + u];
    }
    for (; c < d; ++c) s += (int64_t)f[c * nf + g] * z[c];
    return s;
}

// floor-mod for |s| < 2^52 (plan-checked): quotient estimate in double, off by at most one.
__device__ __forceinline__ int64_t mod_fast(int64_t s, int64_t M, double invM) {
    const int64_t q = (int64_t)floor((double)s * invM);
    int64_t r = s - q * M;
    if (r < 0) r += M;
    if (r >= M) r -= M;
    return r;
}
__device__ __forceinline__ int64_t mod_exact(int64_t s, int64_t M) {
    const int64_t r = s % M;
    return r < 0 ? r + M : r;
}

template <typename K>
__device__ __forceinline__ int64_t residue(const TxArgs& a, const LatDesc& D, int64_t g) {
    const int64_t s = dot_kz<K>((const K*)a.fv.f, a.fv.nf, a.fv.d, g, a.z + D.zoff);
    return a.fast_mod ? mod_fast(s, D.M, D.invM) : mod_exact(s, D.M);
}

__device__ __forceinline__ int find_tx(const int64_t* __restrict__ pre, int n, int64_t g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ bool is_multi(const uint32_t* __restrict__ bm, const LatDesc& D, int64_t r) {
    return (bm[D.bm_off + D.bm_words + (r >> 5)] >> (r & 31)) & 1u;
}

}  // namespace mr1l
