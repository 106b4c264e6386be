// Device passes of the dimension-incremental sparse FFT (Alg. 3) around the mr1l transform:
//  * the built-in black box: a planted sparse polynomial sampled along 1-D lines
//    (x'_1, .., l/K_t, .., x'_d) and, through the Fourier-matrix synthesis of the transform
//    library, along the lattice nodes with appended anchors; complex Gaussian noise from a
//    counter-based stream (Box-Muller, noise model of Sec. 5.2);
//  * explicit nodes for a caller-supplied black box;
//  * "(up to) s largest |p~| >= delta" selection (radix select on the IEEE bit pattern of
//    |p~|^2 computed without fused multiply-add, ties by ascending position), OR-ed into flags
//    (the union over detection iterations);
//  * stream compaction of flags, the candidate product J_t = I^(1..t-1) x I^(t), row gathers.
#include "common.h"
#include "sfft_dev.h"

namespace mr1l {

// ---- counter-based random numbers (SplitMix64 output function on a counter) -----------------------
__device__ __forceinline__ uint64_t d_mix64(uint64_t x) {
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}
__device__ __forceinline__ double d_uniform01(uint64_t key, uint64_t c) {
    return (double)(d_mix64(key + 0x9E3779B97F4A7C15ull * (c + 1)) >> 11) * 0x1.0p-53;
}
// sigma/sqrt(2) * sqrt(-2 ln(1-u1)) * e^{2 pi i u2}, u1, u2 = draws 2g and 2g+1
__device__ __forceinline__ cx<double> d_noise(uint64_t key, uint64_t g, double sigma) {
    const double u1 = d_uniform01(key, 2 * g);
    const double u2 = d_uniform01(key, 2 * g + 1);
    const double rad = sqrt(-2.0 * log1p(-u1)) * (sigma * 0.70710678118654752440);
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    return {rad * c, rad * s};
}

// e^{2 pi i x} for a double x
__device__ __forceinline__ cx<double> d_cis2pi(double x) {
    double s, c;
    sincospi(2.0 * (x - floor(x)), &s, &c);
    return {c, s};
}

// ---- planted black box -----------------------------------------------------------------------------
// w[q][h] = c_h e^{2 pi i sum_{comp != tc} h_comp x'_comp} for 1-D job q (component tc = comp[q])
__global__ void k_planted_w1d(const int32_t* __restrict__ hf, int64_t s, int d, const cx<double>* __restrict__ c,
                              const double* __restrict__ anchors, const int* __restrict__ comp, int njobs,
                              cx<double>* w) {
    const int q = blockIdx.y;
    const int tc = comp[q];
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < s; h += (int64_t)gridDim.x * blockDim.x) {
        double ph = 0.0;
        for (int k = 0; k < d; ++k)
            if (k != tc) ph += (double)hf[(int64_t)k * s + h] * anchors[(int64_t)q * d + k];
        const cx<double> e = d_cis2pi(ph);
        w[(int64_t)q * s + h] = cmul(c[h], e);
    }
}

// y[q][l] = sum_h w[q][h] e^{2 pi i ((h_tc l) mod K)/K} + noise(kind 0, key[q], l)
template <typename T>
__global__ void k_planted_1d(const int32_t* __restrict__ hf, int64_t s, const cx<double>* __restrict__ w,
                             const int* __restrict__ comp, int64_t K, const uint64_t* __restrict__ keys, double sigma,
                             cx<T>* y) {
    const int q = blockIdx.y;
    const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (l >= K) return;
    const int32_t* ht = hf + (int64_t)comp[q] * s;
    const cx<double>* wq = w + (int64_t)q * s;
    cx<double> acc = {0.0, 0.0};
    for (int64_t h = 0; h < s; ++h) {
        int64_t qq = ((int64_t)ht[h] * l) % K;
        if (qq < 0) qq += K;
        double sn, cs;
        sincospi(2.0 * (double)qq / (double)K, &sn, &cs);
        acc = acc + cmul(wq[h], cx<double>{cs, sn});
    }
    if (sigma > 0.0) acc = acc + d_noise(keys[q], (uint64_t)l, sigma);
    y[(int64_t)q * K + l] = make_cx<T>((T)acc.x, (T)acc.y);
}

// The same values for K <= kPlanted1dMaxK, one workgroup per job q: the phase of term h at point l
// depends only on m = h_tc mod K, so the terms are first summed per class, B[m] = sum of w[q][h]
// over h with h_tc = m mod K (ascending h), then y[q][l] = sum_m B[m] e^{2 pi i ((m l) mod K)/K}
// (ascending m): K^2 phases instead of s K.
constexpr int64_t kPlanted1dMaxK = 2048;   // B in LDS: 32 KiB
template <typename T>
__global__ __launch_bounds__(256) void k_planted_1d_bins(const int32_t* __restrict__ hf, int64_t s,
                                                         const cx<double>* __restrict__ w,
                                                         const int* __restrict__ comp, int64_t K,
                                                         const uint64_t* __restrict__ keys, double sigma, cx<T>* y) {
    __shared__ cx<double> B[kPlanted1dMaxK];
    const int q = blockIdx.x;
    const int kk = (int)K;
    const int32_t* ht = hf + (int64_t)comp[q] * s;
    const cx<double>* wq = w + (int64_t)q * s;
    for (int m = threadIdx.x; m < kk; m += blockDim.x) {
        cx<double> acc = {0.0, 0.0};
        for (int64_t h = 0; h < s; ++h) {
            int r = ht[h] % kk;
            if (r < 0) r += kk;
            if (r == m) acc = acc + wq[h];
        }
        B[m] = acc;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < kk; l += blockDim.x) {
        cx<double> acc = {0.0, 0.0};
        for (int m = 0; m < kk; ++m) {
            const int qq = (int)(((int64_t)m * l) % kk);
            double sn, cs;
            sincospi(2.0 * (double)qq / (double)kk, &sn, &cs);
            acc = acc + cmul(B[m], cx<double>{cs, sn});
        }
        if (sigma > 0.0) acc = acc + d_noise(keys[q], (uint64_t)l, sigma);
        y[(int64_t)q * K + l] = make_cx<T>((T)acc.x, (T)acc.y);
    }
}

// w[i][h] = c_h e^{2 pi i sum_{comp >= t} h_comp x~_comp^(i)}  (coefficients of the synthesis)
template <typename T>
__global__ void k_planted_wlat(const int32_t* __restrict__ hf, int64_t s, int d, int t, const cx<double>* __restrict__ c,
                               const double* __restrict__ anchors, cx<T>* w) {
    const int i = blockIdx.y;
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < s; h += (int64_t)gridDim.x * blockDim.x) {
        double ph = 0.0;
        for (int k = t; k < d; ++k) ph += (double)hf[(int64_t)k * s + h] * anchors[(int64_t)i * d + k];
        const cx<double> v = cmul(c[h], d_cis2pi(ph));
        w[(int64_t)i * s + h] = make_cx<T>((T)v.x, (T)v.y);
    }
}

template <typename T>
__global__ void k_add_noise(cx<T>* y, int64_t len, const uint64_t* __restrict__ keys, double sigma) {
    const int i = blockIdx.y;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < len; g += (int64_t)gridDim.x * blockDim.x) {
        const cx<double> e = d_noise(keys[i], (uint64_t)g, sigma);
        cx<T>& v = y[(int64_t)i * len + g];
        v = make_cx<T>((T)((double)v.x + e.x), (T)((double)v.y + e.y));
    }
}

// ---- explicit nodes for a caller-supplied black box -------------------------------------------------
// lattice nodes (j z_l mod M_l)/M_l in components < t, anchors in components >= t
// col: NULL, or the column of the node array that holds processing component k (component
// order of the caller's black box)
__global__ void k_nodes_lattice(const int64_t* __restrict__ M, const int64_t* __restrict__ off, const int64_t* __restrict__ z,
                                int L, int t, int d, const double* __restrict__ anchors, double* nodes,
                                const int* __restrict__ col) {
    const int l = blockIdx.y;
    const int64_t Ml = M[l];
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < Ml; j += (int64_t)gridDim.x * blockDim.x) {
        double* x = nodes + (off[l] + j) * d;
        for (int k = 0; k < d; ++k) {
            double v;
            if (k < t) {
                const int64_t q = (j * z[(int64_t)l * t + k]) % Ml;   // j, z < M < 2^23
                v = (double)q / (double)Ml;
            } else {
                v = anchors[k];
            }
            x[col ? col[k] : k] = v;
        }
    }
}

// 1-D line: anchors everywhere, component tc = l / K
__global__ void k_nodes_1d(int64_t K, int tc, int d, const double* __restrict__ anchors, double* nodes,
                           const int* __restrict__ col) {
    const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (l >= K) return;
    for (int k = 0; k < d; ++k) nodes[l * d + (col ? col[k] : k)] = (k == tc) ? (double)l / (double)K : anchors[k];
}

// ---- selection -------------------------------------------------------------------------------------
constexpr int kSelThreads = 1024;

// key = bits(|v|^2) | 2^63 when |v|^2 >= delta^2 (|v|^2 = re*re + im*im in double, no contraction)
template <typename T>
__device__ __forceinline__ uint64_t sel_key(cx<T> v, double delta2) {
    const double re = (double)v.x, im = (double)v.y;
    const double m = __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im));
    return m >= delta2 ? ((uint64_t)__double_as_longlong(m) | (1ull << 63)) : 0ull;
}

__device__ __forceinline__ unsigned int block_sum_u32(unsigned int v, unsigned int* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kSelThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const unsigned int r = sh[0];
    __syncthreads();
    return r;
}

// inclusive scan over the workgroup: within each wavefront by shuffles, then over the 16 wave
// totals by the first wavefront (sh: at least kSelThreads / 64 entries; free again on return)
__device__ __forceinline__ unsigned int block_scan_u32(unsigned int v, unsigned int* sh) {
    constexpr int kWaves = kSelThreads / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    if (wv == 0) {
        unsigned int t = lane < kWaves ? sh[lane] : 0u;
#pragma unroll
        for (int off = 1; off < kWaves; off <<= 1) {
            const unsigned int y = __shfl_up(t, off);
            if (lane >= off) t += y;
        }
        if (lane < kWaves) sh[lane] = t;
    }
    __syncthreads();
    const unsigned int r = x + (wv > 0 ? sh[wv - 1] : 0u);
    __syncthreads();
    return r;
}

// fn(k, key) for this thread's positions k = threadIdx.x + j kSelThreads, with the loads of
// kSelUnroll positions in flight together
constexpr int kSelUnroll = 8;
template <typename T, typename F>
__device__ __forceinline__ void for_keys(const cx<T>* __restrict__ c, int64_t n, double delta2, F&& fn) {
    int64_t k = threadIdx.x;
    for (; k + (int64_t)(kSelUnroll - 1) * kSelThreads < n; k += (int64_t)kSelUnroll * kSelThreads) {
        cx<T> v[kSelUnroll];
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) v[u] = c[k + (int64_t)u * kSelThreads];
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) fn(k + (int64_t)u * kSelThreads, sel_key(v[u], delta2));
    }
    for (; k < n; k += kSelThreads) fn(k, sel_key(c[k], delta2));
}

// One workgroup per right-hand side: flags[(rhs / rhs_per_group) * flags_stride + k] |= selected.
template <typename T>
__global__ __launch_bounds__(kSelThreads) void k_select(const cx<T>* __restrict__ coeffs, int64_t n, double delta2,
                                                        int64_t s, uint8_t* flags, int rhs_per_group,
                                                        int64_t flags_stride) {
    __shared__ unsigned int sh[kSelThreads];
    __shared__ unsigned int hist[256];
    __shared__ uint64_t sel_prefix;
    __shared__ int64_t sel_remaining;
    __shared__ int64_t sel_equal;   // keys equal to the s-th largest (after the last pass)
    const int64_t rhs = blockIdx.x;
    const cx<T>* c = coeffs + rhs * n;
    uint8_t* f = flags + (rhs / rhs_per_group) * flags_stride;
    unsigned int local = 0;
    for_keys(c, n, delta2, [&](int64_t, uint64_t key) { local += key != 0; });
    const int64_t eligible = block_sum_u32(local, sh);
    if (eligible <= s) {
        for_keys(c, n, delta2, [&](int64_t k, uint64_t key) {
            if (key) f[k] = 1;
        });
        return;
    }
    // radix select of the s-th largest key, 8 bits per pass from the top
    if (threadIdx.x == 0) {
        sel_prefix = 0;
        sel_remaining = s;
    }
    __syncthreads();
    for (int pass = 7; pass >= 0; --pass) {
        for (int b = threadIdx.x; b < 256; b += kSelThreads) hist[b] = 0;
        __syncthreads();
        const uint64_t prefix = sel_prefix;
        const uint64_t hi_mask = pass == 7 ? 0ull : (~0ull << (8 * (pass + 1)));
        for_keys(c, n, delta2, [&](int64_t, uint64_t key) {
            if ((key & hi_mask) == (prefix & hi_mask)) atomicAdd(&hist[(key >> (8 * pass)) & 255], 1u);
        });
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t rem = sel_remaining, cum = 0;
            int b = 255;
            for (; b > 0; --b) {
                if (cum + hist[b] >= rem) break;
                cum += hist[b];
            }
            sel_remaining = rem - cum;
            sel_prefix = prefix | ((uint64_t)b << (8 * pass));
            if (pass == 0) sel_equal = hist[b];
        }
        __syncthreads();
    }
    const uint64_t kstar = sel_prefix;
    const int64_t need_eq = sel_remaining;   // how many keys equal to kstar to take, lowest positions first
    if (need_eq == sel_equal) {   // every key equal to kstar is taken: no ranking among them
        for_keys(c, n, delta2, [&](int64_t k, uint64_t key) {
            if (key >= kstar) f[k] = 1;
        });
        return;
    }
    int64_t taken = 0;
    for (int64_t k0 = 0; k0 < n; k0 += kSelThreads) {
        const int64_t k = k0 + threadIdx.x;
        uint64_t key = 0;
        if (k < n) key = sel_key(c[k], delta2);
        const unsigned int eq = (k < n && key == kstar) ? 1u : 0u;
        const unsigned int incl = block_scan_u32(eq, sh);
        if (k < n && (key > kstar || (eq && taken + (int64_t)incl <= need_eq))) f[k] = 1;
        // total of this chunk
        if (threadIdx.x == kSelThreads - 1) sh[0] = incl;
        __syncthreads();
        taken += sh[0];
        __syncthreads();
    }
}

// indices of nonzero flags, ascending; *count = their number (one workgroup; each thread takes 16
// consecutive flags per pass, so a pass covers 16384 flags with one block scan)
constexpr int kCompactPer = 16;
__global__ __launch_bounds__(kSelThreads) void k_compact(const uint8_t* __restrict__ flags, int64_t n, int32_t* idx,
                                                         int64_t* count) {
    __shared__ unsigned int sh[kSelThreads];
    int64_t base = 0;
    const bool vec = ((uintptr_t)flags & 15) == 0;   // 16 flags per 16-byte load
    for (int64_t k0 = 0; k0 < n; k0 += (int64_t)kSelThreads * kCompactPer) {
        const int64_t kb = k0 + (int64_t)threadIdx.x * kCompactPer;
        unsigned int bits = 0;
        if (vec && kb + kCompactPer <= n) {
            const uint4 q = *(const uint4*)(flags + kb);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int i = 0; i < kCompactPer; ++i)
                if ((w[i >> 2] >> (8 * (i & 3))) & 0xffu) bits |= 1u << i;
        } else {
#pragma unroll
            for (int i = 0; i < kCompactPer; ++i)
                if (kb + i < n && flags[kb + i]) bits |= 1u << i;
        }
        const unsigned int c = __popc(bits);
        const unsigned int incl = block_scan_u32(c, sh);
        int64_t pos = base + incl - c;
#pragma unroll
        for (int i = 0; i < kCompactPer; ++i)
            if ((bits >> i) & 1u) idx[pos++] = (int32_t)(kb + i);
        if (threadIdx.x == kSelThreads - 1) sh[0] = incl;
        __syncthreads();
        base += sh[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base;
}

// J[c][a n2 + b] = P[c][a] (c < t-1), J[t-1][a n2 + b] = Q[b]   (lexicographic order kept)
template <typename K>
__global__ void k_product(const K* __restrict__ P, int64_t n1, const int32_t* __restrict__ Q, int64_t n2, int t,
                          K* J) {
    const int64_t nJ = n1 * n2;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nJ; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = j / n2, b = j - a * n2;
        for (int c = 0; c < t - 1; ++c) J[(int64_t)c * nJ + j] = P[(int64_t)c * n1 + a];
        J[(int64_t)(t - 1) * nJ + j] = (K)Q[b];
    }
}

template <typename K>
__global__ void k_gather_rows(const K* __restrict__ J, int64_t nJ, int t, const int32_t* __restrict__ idx, int64_t m,
                              K* out) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        for (int c = 0; c < t; ++c) out[(int64_t)c * m + j] = J[(int64_t)c * nJ + idx[j]];
}

// I^(t) values from 1-D flags: value lo + position
__global__ void k_flags_to_values(const int32_t* __restrict__ idx, int64_t m, int32_t lo, int32_t* vals) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        vals[j] = lo + idx[j];
}

template <typename K>
__global__ void k_values_to_k(const int32_t* __restrict__ v, int64_t m, K* out) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        out[j] = (K)v[j];
}

template <typename T>
__global__ void k_gather_coeffs(const cx<T>* __restrict__ c, const int32_t* __restrict__ idx, int64_t m, cx<double>* out) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const cx<T> v = c[idx[j]];
        out[j] = {(double)v.x, (double)v.y};
    }
}

template <typename K>
__global__ void k_soa_to_rows(const K* __restrict__ f, int64_t m, int d, int32_t* rows) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        for (int c = 0; c < d; ++c) rows[j * d + c] = (int32_t)f[(int64_t)c * m + j];
}

// ---- launchers -------------------------------------------------------------------------------------
static inline dim3 g1(int64_t n, unsigned y = 1) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return dim3((unsigned)b, y);
}

void sf_planted_w1d(const int32_t* hf, int64_t s, int d, const void* c, const double* anchors, const int* comp,
                    int njobs, void* w, hipStream_t st) {
    hipLaunchKernelGGL(k_planted_w1d, g1(s, njobs), dim3(256), 0, st, hf, s, d, (const cx<double>*)c, anchors, comp,
                       njobs, (cx<double>*)w);
}

void sf_planted_1d(int dt, const int32_t* hf, int64_t s, const void* w, const int* comp, int njobs, int64_t K,
                   const uint64_t* keys, double sigma, void* y, hipStream_t st) {
    if (K <= kPlanted1dMaxK && s > K) {   // per-class sums first
        if (dt == MR1L_C128)
            hipLaunchKernelGGL(k_planted_1d_bins<double>, dim3((unsigned)njobs), dim3(256), 0, st, hf, s,
                               (const cx<double>*)w, comp, K, keys, sigma, (cx<double>*)y);
        else
            hipLaunchKernelGGL(k_planted_1d_bins<float>, dim3((unsigned)njobs), dim3(256), 0, st, hf, s,
                               (const cx<double>*)w, comp, K, keys, sigma, (cx<float>*)y);
        return;
    }
    const dim3 grid((unsigned)((K + 255) / 256), (unsigned)njobs);
    if (dt == MR1L_C128)
        hipLaunchKernelGGL(k_planted_1d<double>, grid, dim3(256), 0, st, hf, s, (const cx<double>*)w, comp, K, keys,
                           sigma, (cx<double>*)y);
    else
        hipLaunchKernelGGL(k_planted_1d<float>, grid, dim3(256), 0, st, hf, s, (const cx<double>*)w, comp, K, keys,
                           sigma, (cx<float>*)y);
}

void sf_planted_wlat(int dt, const int32_t* hf, int64_t s, int d, int t, const void* c, const double* anchors, int nrep,
                     void* w, hipStream_t st) {
    if (dt == MR1L_C128)
        hipLaunchKernelGGL(k_planted_wlat<double>, g1(s, nrep), dim3(256), 0, st, hf, s, d, t, (const cx<double>*)c,
                           anchors, (cx<double>*)w);
    else
        hipLaunchKernelGGL(k_planted_wlat<float>, g1(s, nrep), dim3(256), 0, st, hf, s, d, t, (const cx<double>*)c,
                           anchors, (cx<float>*)w);
}

void sf_add_noise(int dt, void* y, int64_t len, int nrep, const uint64_t* keys, double sigma, hipStream_t st) {
    if (dt == MR1L_C128)
        hipLaunchKernelGGL(k_add_noise<double>, g1(len, nrep), dim3(256), 0, st, (cx<double>*)y, len, keys, sigma);
    else
        hipLaunchKernelGGL(k_add_noise<float>, g1(len, nrep), dim3(256), 0, st, (cx<float>*)y, len, keys, sigma);
}

void sf_nodes_lattice(const int64_t* M, const int64_t* off, const int64_t* z, int L, int64_t maxM, int t, int d,
                      const double* anchors, double* nodes, const int* col, hipStream_t st) {
    hipLaunchKernelGGL(k_nodes_lattice, g1(maxM, L), dim3(256), 0, st, M, off, z, L, t, d, anchors, nodes, col);
}

void sf_nodes_1d(int64_t K, int tc, int d, const double* anchors, double* nodes, const int* col, hipStream_t st) {
    hipLaunchKernelGGL(k_nodes_1d, g1(K), dim3(256), 0, st, K, tc, d, anchors, nodes, col);
}

void sf_select(int dt, const void* coeffs, int64_t n, int64_t n_rhs, double delta, int64_t s, uint8_t* flags,
               int rhs_per_group, int64_t flags_stride, hipStream_t st) {
    if (n == 0 || n_rhs == 0) return;
    const double d2 = delta * delta;
    if (dt == MR1L_C128)
        hipLaunchKernelGGL(k_select<double>, dim3((unsigned)n_rhs), dim3(kSelThreads), 0, st,
                           (const cx<double>*)coeffs, n, d2, s, flags, rhs_per_group, flags_stride);
    else
        hipLaunchKernelGGL(k_select<float>, dim3((unsigned)n_rhs), dim3(kSelThreads), 0, st,
                           (const cx<float>*)coeffs, n, d2, s, flags, rhs_per_group, flags_stride);
}

void sf_compact(const uint8_t* flags, int64_t n, int32_t* idx, int64_t* count, hipStream_t st) {
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(kSelThreads), 0, st, flags, n, idx, count);
}

void sf_product(int kt, const void* P, int64_t n1, const int32_t* Q, int64_t n2, int t, void* J, hipStream_t st) {
    const dim3 grid = g1(n1 * n2);
    if (kt == K_I8) hipLaunchKernelGGL(k_product<int8_t>, grid, dim3(256), 0, st, (const int8_t*)P, n1, Q, n2, t, (int8_t*)J);
    else if (kt == K_I16)
        hipLaunchKernelGGL(k_product<int16_t>, grid, dim3(256), 0, st, (const int16_t*)P, n1, Q, n2, t, (int16_t*)J);
    else hipLaunchKernelGGL(k_product<int32_t>, grid, dim3(256), 0, st, (const int32_t*)P, n1, Q, n2, t, (int32_t*)J);
}

void sf_gather_rows(int kt, const void* J, int64_t nJ, int t, const int32_t* idx, int64_t m, void* out, hipStream_t st) {
    const dim3 grid = g1(m);
    if (kt == K_I8)
        hipLaunchKernelGGL(k_gather_rows<int8_t>, grid, dim3(256), 0, st, (const int8_t*)J, nJ, t, idx, m, (int8_t*)out);
    else if (kt == K_I16)
        hipLaunchKernelGGL(k_gather_rows<int16_t>, grid, dim3(256), 0, st, (const int16_t*)J, nJ, t, idx, m,
                           (int16_t*)out);
    else
        hipLaunchKernelGGL(k_gather_rows<int32_t>, grid, dim3(256), 0, st, (const int32_t*)J, nJ, t, idx, m,
                           (int32_t*)out);
}

void sf_flags_to_values(const int32_t* idx, int64_t m, int32_t lo, int32_t* vals, hipStream_t st) {
    hipLaunchKernelGGL(k_flags_to_values, g1(m), dim3(256), 0, st, idx, m, lo, vals);
}

void sf_values_to_k(int kt, const int32_t* v, int64_t m, void* out, hipStream_t st) {
    if (kt == K_I8) hipLaunchKernelGGL(k_values_to_k<int8_t>, g1(m), dim3(256), 0, st, v, m, (int8_t*)out);
    else if (kt == K_I16) hipLaunchKernelGGL(k_values_to_k<int16_t>, g1(m), dim3(256), 0, st, v, m, (int16_t*)out);
    else hipLaunchKernelGGL(k_values_to_k<int32_t>, g1(m), dim3(256), 0, st, v, m, (int32_t*)out);
}

void sf_gather_coeffs(int dt, const void* c, const int32_t* idx, int64_t m, void* out, hipStream_t st) {
    if (dt == MR1L_C128)
        hipLaunchKernelGGL(k_gather_coeffs<double>, g1(m), dim3(256), 0, st, (const cx<double>*)c, idx, m,
                           (cx<double>*)out);
    else
        hipLaunchKernelGGL(k_gather_coeffs<float>, g1(m), dim3(256), 0, st, (const cx<float>*)c, idx, m,
                           (cx<double>*)out);
}

void sf_soa_to_rows(int kt, const void* f, int64_t m, int d, int32_t* rows, hipStream_t st) {
    if (kt == K_I8) hipLaunchKernelGGL(k_soa_to_rows<int8_t>, g1(m), dim3(256), 0, st, (const int8_t*)f, m, d, rows);
    else if (kt == K_I16)
        hipLaunchKernelGGL(k_soa_to_rows<int16_t>, g1(m), dim3(256), 0, st, (const int16_t*)f, m, d, rows);
    else hipLaunchKernelGGL(k_soa_to_rows<int32_t>, g1(m), dim3(256), 0, st, (const int32_t*)f, m, d, rows);
}

}  // namespace mr1l
