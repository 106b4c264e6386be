// Prime-length DFTs of the rank-1 lattice FFT (Alg. 2, "rank-1 lattice FFT": one 1-D DFT of
// length M_l per lattice) via Bluestein's chirp-z identity
//     jm = (j^2 + m^2 - (m - j)^2) / 2,
//     X[m] = e^{s i pi m^2/M} sum_j (x[j] e^{s i pi j^2/M}) e^{-s i pi (m-j)^2/M},
// i.e. a cyclic convolution of length N = 2^lgN >= 2M - 1 computed with power-of-two FFTs.
// Chirp phases are reduced exactly in integers (j^2 mod 2M) before sin/cos.
//
// Two code paths:
//  * one-block path (N <= 4096): one workgroup holds the whole convolution in LDS;
//  * four-step path: N = N1 * N2; stage 1 = chirp + zero-pad + column DFTs of length N1 + twiddles,
//    stage 2 = row DFTs of length N2, multiplication by the filter spectrum, inverse row DFTs,
//    stage 3 = inverse twiddles + inverse column DFTs + output chirp.  Stage 2 is where forward
//    and inverse transforms meet, so the filter spectrum is stored in that stage's layout and the
//    intermediate never needs a transpose.
// All in-LDS DFTs are Stockham radix-8 (+ one radix-2/4 stage) with twiddles from a table.
#include <map>
#include <mutex>
#include <cmath>
#include <vector>

#include "common.h"

namespace mr1l {

// ---- twiddle tables --------------------------------------------------------------------------------
// tw[m] = e^{-2 pi i m/4096} (m < 4096), tw[4096 + m] = e^{-2 pi i m/2^24} (m < 4096).
static std::mutex g_tw_mu;
static std::map<std::pair<int, int>, void*> g_tw;

static void host_cispi2(long double num, long double den, double* c, double* s) {
    // e^{-2 pi i num/den} with the angle folded to the first octant for accuracy
    long double a = 2.0L * 3.14159265358979323846264338327950288L * num / den;
    *c = (double)cosl(a);
    *s = (double)-sinl(a);
}

template <typename T>
const cx<T>* twiddles(int device) {
    std::lock_guard<std::mutex> lk(g_tw_mu);
    auto key = std::make_pair(device, (int)sizeof(T));
    auto it = g_tw.find(key);
    if (it != g_tw.end()) return (const cx<T>*)it->second;
    std::vector<cx<T>> h(8192);
    for (int m = 0; m < 4096; ++m) {
        double c, s;
        // exact values at multiples of pi/2
        if (m % 1024 == 0) {
            const int q = m / 1024;
            c = (q == 0) ? 1.0 : (q == 2 ? -1.0 : 0.0);
            s = (q == 1) ? -1.0 : (q == 3 ? 1.0 : 0.0);
        } else {
            host_cispi2(m, 4096.0L, &c, &s);
        }
        h[m] = make_cx<T>((T)c, (T)s);
        host_cispi2(m, 16777216.0L, &c, &s);
        h[4096 + m] = make_cx<T>((T)c, (T)s);
    }
    void* d = nullptr;
    if (hipMalloc(&d, h.size() * sizeof(cx<T>)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(cx<T>), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    g_tw[key] = d;
    return (const cx<T>*)d;
}
template const cx<float>* twiddles<float>(int);
template const cx<double>* twiddles<double>(int);

// e^{i pi x}
template <typename T> __device__ __forceinline__ cx<T> cispi(double x);
template <> __device__ __forceinline__ cx<float> cispi<float>(double x) {
    float s, c;
    sincospif((float)x, &s, &c);
    return {c, s};
}
template <> __device__ __forceinline__ cx<double> cispi<double>(double x) {
    double s, c;
    sincospi(x, &s, &c);
    return {c, s};
}

// e^{-2 pi i e / 2^lgN} for 0 <= e < 2^lgN <= 2^24; the argument -2e/2^lgN is exact in T.
template <typename T>
__device__ __forceinline__ cx<T> tw_pow2(uint32_t e, int lgN) {
    T s, c;
    const T x = -(T)e * (T)ldexp(1.0, 1 - lgN);
    if constexpr (sizeof(T) == 4) sincospif(x, &s, &c);
    else sincospi(x, &s, &c);
    return {c, s};
}

// (n^2 mod 2M) as an integer-valued double: every intermediate is an integer below 2^53 for
// n < 2^23, so the remainder is exact after at most one correction of the quotient estimate.
__device__ __forceinline__ double sq_mod_2M(int64_t n, int64_t M, double inv2M) {
    const double nn = (double)n * (double)n;
    const double m2 = 2.0 * (double)M;
    double q = nn - m2 * floor(nn * inv2M);
    if (q < 0.0) q += m2;
    else if (q >= m2) q -= m2;
    return q;
}

// e^{sign i pi (n^2 mod 2M)/M}
template <typename T>
__device__ __forceinline__ cx<T> chirp(int64_t n, int64_t M, double invM, int sign) {
    return cispi<T>((double)sign * (sq_mod_2M(n, M, 0.5 * invM) * invM));
}

// LDS index with one pad slot after every 8 elements: strided Stockham writes and column loads
// then spread over the banks instead of piling onto a few.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }
template <int ELEMS> struct Padded { static constexpr int v = ELEMS + (ELEMS >> 3) + 64; };

// ---- in-register DFTs ------------------------------------------------------------------------------
template <typename T, int SIGN>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {  // a * (SIGN i)
    return SIGN < 0 ? cx<T>{a.y, -a.x} : cx<T>{-a.y, a.x};
}

template <typename T, int R, int SIGN> struct Dft;
template <typename T, int SIGN> struct Dft<T, 2, SIGN> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        const cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};
template <typename T, int SIGN> struct Dft<T, 4, SIGN> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        const cx<T> a0 = v[0] + v[2], a1 = v[0] - v[2], a2 = v[1] + v[3];
        const cx<T> a3 = mul_si<T, SIGN>(v[1] - v[3]);
        v[0] = a0 + a2;
        v[2] = a0 - a2;
        v[1] = a1 + a3;
        v[3] = a1 - a3;
    }
};
template <typename T, int SIGN> struct Dft<T, 8, SIGN> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        cx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cx<T> o[4] = {v[1], v[3], v[5], v[7]};
        Dft<T, 4, SIGN>::run(e);
        Dft<T, 4, SIGN>::run(o);
        const T c = (T)0.707106781186547524400844362104849039;
        const T sg = (T)SIGN;
        const cx<T> t1 = {c * (o[1].x - sg * o[1].y), c * (o[1].y + sg * o[1].x)};
        const cx<T> t2 = mul_si<T, SIGN>(o[2]);
        const cx<T> t3 = {c * (-o[3].x - sg * o[3].y), c * (sg * o[3].x - o[3].y)};
        v[0] = e[0] + o[0];
        v[4] = e[0] - o[0];
        v[1] = e[1] + t1;
        v[5] = e[1] - t1;
        v[2] = e[2] + t2;
        v[6] = e[2] - t2;
        v[3] = e[3] + t3;
        v[7] = e[3] - t3;
    }
};

template <int R> struct Lg;
template <> struct Lg<2> { static constexpr int v = 1; };
template <> struct Lg<4> { static constexpr int v = 2; };
template <> struct Lg<8> { static constexpr int v = 3; };

// One Stockham radix-R stage over nseq sequences of length 2^lgN stored at buf[b*S + e].
// Ns = 2^lgNs is the length of the sub-transforms already done.  Every thread holds E values.
template <typename T, int E, int R, int SIGN>
__device__ __forceinline__ void fft_stage(cx<T>* buf, int lgN, int nseq, int S, int lgNs,
                                          const cx<T>* __restrict__ tw) {
    constexpr int NB = E / R;
    constexpr int LR = Lg<R>::v;
    const int lgNb = lgN - LR;
    const int nbf = 1 << lgNb;
    const int total = nbf * nseq;
    cx<T> v[NB][R];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int g = threadIdx.x + u * kThreads;
        if (g < total) {
            const int b = g >> lgNb, j = g & (nbf - 1);
            const int base = b * S + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = buf[pidx(base + (r << lgNb))];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int g = threadIdx.x + u * kThreads;
        if (g < total) {
            const int b = g >> lgNb, j = g & (nbf - 1);
            const int k = j & ((1 << lgNs) - 1);
            if (lgNs > 0) {
                const int step = k << (kTwLg - lgNs - LR);   // w_{Ns R}^{k} = tw[k 4096/(Ns R)]
                // powers w^r from table values w, w^2, w^4 (exact entries) and at most two products
                cx<T> w[R];
                w[1] = tw[step];
                if (R >= 4) {
                    w[2] = tw[2 * step];
                    w[3] = cmul(w[1], w[2]);
                }
                if (R >= 8) {
                    w[4] = tw[4 * step];
                    w[5] = cmul(w[1], w[4]);
                    w[6] = cmul(w[2], w[4]);
                    w[7] = cmul(w[3], w[4]);
                }
#pragma unroll
                for (int r = 1; r < R; ++r) v[u][r] = SIGN < 0 ? cmul(v[u][r], w[r]) : cmulc(v[u][r], w[r]);
            }
            Dft<T, R, SIGN>::run(v[u]);
            const int base = b * S + ((j - k) << LR) + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[pidx(base + (r << lgNs))] = v[u][r];
        }
    }
    __syncthreads();
}

// In-LDS DFT (SIGN -1: e^{-2 pi i nk/N}, +1: e^{+...}, unnormalized) of nseq sequences.
// Requires nseq * 2^lgN <= kThreads * E.  Output in natural order.
template <typename T, int E, int SIGN>
__device__ __forceinline__ void lds_fft(cx<T>* buf, int lgN, int nseq, int S, const cx<T>* __restrict__ tw) {
    int lgNs = 0;
    const int rem = lgN % 3;
    if (rem == 1) {
        fft_stage<T, E, 2, SIGN>(buf, lgN, nseq, S, 0, tw);
        lgNs = 1;
    } else if (rem == 2) {
        fft_stage<T, E, 4, SIGN>(buf, lgN, nseq, S, 0, tw);
        lgNs = 2;
    }
    while (lgNs < lgN) {
        fft_stage<T, E, 8, SIGN>(buf, lgN, nseq, S, lgNs, tw);
        lgNs += 3;
    }
}

__device__ __forceinline__ int find_seg(const int* __restrict__ pre, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---- four-step stage 1 -----------------------------------------------------------------------------
// SRC 0: x = samples * chirp, 1: x = work (bins) * chirp, 2: x = work as is (all N entries).
template <typename T, int SRC>
__global__ __launch_bounds__(kThreads) void k_p1(TxArgs a, const cx<T>* __restrict__ src, int64_t src_stride,
                                                 cx<T>* work, int sign, const cx<T>* __restrict__ tw) {
    constexpr int LGE = TileElems<T>::lg;
    constexpr int E = (1 << LGE) / kThreads;
    __shared__ cx<T> lds[Padded<(1 << LGE) + 256>::v];
    const int i = find_seg(a.tile0_col, a.nlarge + 1, blockIdx.x);
    const LatDesc D = a.desc[a.large[i]];
    const int lgN1 = D.lgN1, lgN2 = D.lgN2;
    const int lgC = min(lgN2, LGE - lgN1);
    const int C = 1 << lgC, N1 = 1 << lgN1;
    const int c0 = (blockIdx.x - a.tile0_col[i]) << lgC;
    const int S = N1 + 1;
    const int64_t rhs = blockIdx.y;
    const cx<T>* in = src + rhs * src_stride + (SRC == 0 ? D.samp_off : D.work_off);
    cx<T>* w = work + rhs * a.work_stride + D.work_off;
    const int64_t nvalid = (SRC == 2) ? ((int64_t)1 << D.lgN) : D.M;
    const int total = N1 << lgC;
    for (int e = threadIdx.x; e < total; e += kThreads) {
        const int col = e & (C - 1), n1 = e >> lgC;
        const int64_t n = ((int64_t)n1 << lgN2) + c0 + col;
        cx<T> v = {(T)0, (T)0};
        if (n < nvalid) {
            v = in[n];
            if (SRC != 2) v = cmul(v, chirp<T>(n, D.M, D.invM, sign));
        }
        lds[pidx(col * S + n1)] = v;
    }
    __syncthreads();
    lds_fft<T, E, -1>(lds, lgN1, C, S, tw);
    {
        // this thread's column n2 is fixed and k1 advances by kThreads/C: w_N^{n2 k1} by recurrence
        const int col = threadIdx.x & (C - 1), n2 = c0 + col;
        const int dk = kThreads >> lgC;
        cx<T> wk = tw_pow2<T>((uint32_t)(n2 * (threadIdx.x >> lgC)), D.lgN);
        const cx<T> ws = tw_pow2<T>((uint32_t)((n2 * dk) & ((1 << D.lgN) - 1)), D.lgN);
        for (int e = threadIdx.x; e < total; e += kThreads) {
            const int k1 = e >> lgC;
            w[((int64_t)k1 << lgN2) + n2] = cmul(lds[pidx(col * S + k1)], wk);
            wk = cmul(wk, ws);
        }
    }
}

// ---- four-step stage 2 -----------------------------------------------------------------------------
// CONV: row DFT, multiply by the filter (conjugated for sign +1), inverse row DFT; else row DFT only.
template <typename T, bool CONV>
__global__ __launch_bounds__(kThreads) void k_p2(TxArgs a, cx<T>* work, const cx<T>* __restrict__ filt, int sign,
                                                 const cx<T>* __restrict__ tw) {
    constexpr int LGE = TileElems<T>::lg;
    constexpr int E = (1 << LGE) / kThreads;
    __shared__ cx<T> lds[Padded<(1 << LGE)>::v];
    const int i = find_seg(a.tile0_row, a.nlarge + 1, blockIdx.x);
    const LatDesc D = a.desc[a.large[i]];
    const int lgN1 = D.lgN1, lgN2 = D.lgN2;
    const int lgR = min(lgN1, LGE - lgN2);
    const int r0 = (blockIdx.x - a.tile0_row[i]) << lgR;
    const int64_t rhs = blockIdx.y;
    cx<T>* w = work + rhs * a.work_stride + D.work_off + ((int64_t)r0 << lgN2);
    const int total = 1 << (lgR + lgN2);
    for (int e = threadIdx.x; e < total; e += kThreads) lds[pidx(e)] = w[e];
    __syncthreads();
    lds_fft<T, E, -1>(lds, lgN2, 1 << lgR, 1 << lgN2, tw);
    if (CONV) {
        const cx<T>* f = filt + D.filt_off + ((int64_t)r0 << lgN2);
        for (int e = threadIdx.x; e < total; e += kThreads)
            lds[pidx(e)] = sign < 0 ? cmul(lds[pidx(e)], f[e]) : cmulc(lds[pidx(e)], f[e]);
        __syncthreads();
        lds_fft<T, E, +1>(lds, lgN2, 1 << lgR, 1 << lgN2, tw);
    }
    for (int e = threadIdx.x; e < total; e += kThreads) w[e] = lds[pidx(e)];
}

// ---- four-step stage 3 -----------------------------------------------------------------------------
template <typename T, bool TO_SAMPLES>
__global__ __launch_bounds__(kThreads) void k_p3(TxArgs a, cx<T>* work, cx<T>* dst, int64_t dst_stride, int sign,
                                                 int scale_by_invM, const cx<T>* __restrict__ tw) {
    constexpr int LGE = TileElems<T>::lg;
    constexpr int E = (1 << LGE) / kThreads;
    __shared__ cx<T> lds[Padded<(1 << LGE) + 256>::v];
    const int i = find_seg(a.tile0_col, a.nlarge + 1, blockIdx.x);
    const LatDesc D = a.desc[a.large[i]];
    const int lgN1 = D.lgN1, lgN2 = D.lgN2;
    const int lgC = min(lgN2, LGE - lgN1);
    const int C = 1 << lgC, N1 = 1 << lgN1;
    const int c0 = (blockIdx.x - a.tile0_col[i]) << lgC;
    const int S = N1 + 1;
    const int64_t rhs = blockIdx.y;
    cx<T>* w = work + rhs * a.work_stride + D.work_off;
    const int total = N1 << lgC;
    {
        const int col = threadIdx.x & (C - 1), n2 = c0 + col;
        const int dk = kThreads >> lgC;
        cx<T> wk = tw_pow2<T>((uint32_t)(n2 * (threadIdx.x >> lgC)), D.lgN);
        const cx<T> ws = tw_pow2<T>((uint32_t)((n2 * dk) & ((1 << D.lgN) - 1)), D.lgN);
        for (int e = threadIdx.x; e < total; e += kThreads) {
            const int k1 = e >> lgC;
            lds[pidx(col * S + k1)] = cmulc(w[((int64_t)k1 << lgN2) + n2], wk);
            wk = cmul(wk, ws);
        }
    }
    __syncthreads();
    lds_fft<T, E, +1>(lds, lgN1, C, S, tw);
    cx<T>* out = TO_SAMPLES ? dst + rhs * dst_stride + D.samp_off : w;
    const T sc = scale_by_invM ? (T)D.invM : (T)1;
    for (int e = threadIdx.x; e < total; e += kThreads) {
        const int col = e & (C - 1), n1 = e >> lgC;
        const int64_t n = ((int64_t)n1 << lgN2) + c0 + col;
        if (n < D.M) out[n] = cscale(cmul(lds[pidx(col * S + n1)], chirp<T>(n, D.M, D.invM, sign)), sc);
    }
}

// ---- one-block Bluestein ---------------------------------------------------------------------------
template <typename T, bool SRC_SAMPLES, bool TO_SAMPLES>
__global__ __launch_bounds__(kThreads) void k_small(TxArgs a, const cx<T>* __restrict__ src, int64_t src_stride,
                                                    cx<T>* work, const cx<T>* __restrict__ filt, cx<T>* dst,
                                                    int64_t dst_stride, int sign, int scale_by_invM,
                                                    const cx<T>* __restrict__ tw) {
    constexpr int E = (1 << kSmallMaxLg) / kThreads;
    __shared__ cx<T> lds[Padded<(1 << kSmallMaxLg)>::v];
    const LatDesc D = a.desc[a.small[blockIdx.x]];
    const int64_t rhs = blockIdx.y;
    const int N = 1 << D.lgN;
    const cx<T>* in = src + rhs * src_stride + (SRC_SAMPLES ? D.samp_off : D.work_off);
    for (int n = threadIdx.x; n < N; n += kThreads) {
        cx<T> v = {(T)0, (T)0};
        if (n < D.M) v = cmul(in[n], chirp<T>(n, D.M, D.invM, sign));
        lds[pidx(n)] = v;
    }
    __syncthreads();
    lds_fft<T, E, -1>(lds, D.lgN, 1, N, tw);
    const cx<T>* f = filt + D.filt_off;
    for (int n = threadIdx.x; n < N; n += kThreads) lds[pidx(n)] = sign < 0 ? cmul(lds[pidx(n)], f[n]) : cmulc(lds[pidx(n)], f[n]);
    __syncthreads();
    lds_fft<T, E, +1>(lds, D.lgN, 1, N, tw);
    cx<T>* out = TO_SAMPLES ? dst + rhs * dst_stride + D.samp_off : work + rhs * a.work_stride + D.work_off;
    const T sc = scale_by_invM ? (T)D.invM : (T)1;
    for (int n = threadIdx.x; n < D.M; n += kThreads)
        out[n] = cscale(cmul(lds[pidx(n)], chirp<T>(n, D.M, D.invM, sign)), sc);
}

// plain in-place forward DFT of the whole region (filter construction, one-block lattices)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_small_dft(TxArgs a, cx<T>* work, const cx<T>* __restrict__ tw) {
    constexpr int E = (1 << kSmallMaxLg) / kThreads;
    __shared__ cx<T> lds[Padded<(1 << kSmallMaxLg)>::v];
    const LatDesc D = a.desc[a.small[blockIdx.x]];
    const int N = 1 << D.lgN;
    cx<T>* w = work + D.work_off;
    for (int n = threadIdx.x; n < N; n += kThreads) lds[pidx(n)] = w[n];
    __syncthreads();
    lds_fft<T, E, -1>(lds, D.lgN, 1, N, tw);
    for (int n = threadIdx.x; n < N; n += kThreads) w[n] = lds[pidx(n)];
}

// b_l[n] = e^{+i pi n^2/M} for 0 <= n < M and at N - n for 0 < n < M, zero elsewhere (double)
__global__ void k_filter_fill(const LatDesc* __restrict__ desc, int L, cx<double>* tmp) {
    const int l = blockIdx.y;
    const LatDesc D = desc[l];
    const int64_t N = (int64_t)1 << D.lgN;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        int64_t m = -1;
        if (n < D.M) m = n;
        else if (N - n < D.M) m = N - n;
        cx<double> v = {0.0, 0.0};
        if (m >= 0) {
            v = cispi<double>(sq_mod_2M(m, D.M, 0.5 * D.invM) * D.invM);
        }
        tmp[D.work_off + n] = v;
    }
}

template <typename T>
__global__ void k_filter_store(const LatDesc* __restrict__ desc, const cx<double>* __restrict__ tmp, cx<T>* filt) {
    const int l = blockIdx.y;
    const LatDesc D = desc[l];
    const int64_t N = (int64_t)1 << D.lgN;
    const double sc = 1.0 / (double)N;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const cx<double> v = tmp[D.work_off + n];
        filt[D.filt_off + n] = make_cx<T>((T)(v.x * sc), (T)(v.y * sc));
    }
}

// ---- launchers -------------------------------------------------------------------------------------
template <typename T>
void launch_bluestein_small(const TxArgs& a, const cx<T>* src, int64_t src_stride, bool src_is_samples,
                            cx<T>* work, const cx<T>* filt, cx<T>* dst, int64_t dst_stride, bool dst_is_samples,
                            int sign, bool scale_by_invM, hipStream_t s) {
    if (a.nsmall == 0 || a.n_rhs == 0) return;
    int dev = 0;
    hipGetDevice(&dev);
    const cx<T>* tw = twiddles<T>(dev);
    dim3 grid(a.nsmall, (unsigned)a.n_rhs);
    if (src_is_samples && !dst_is_samples)
        hipLaunchKernelGGL((k_small<T, true, false>), grid, dim3(kThreads), 0, s, a, src, src_stride, work, filt, dst,
                           dst_stride, sign, (int)scale_by_invM, tw);
    else if (!src_is_samples && dst_is_samples)
        hipLaunchKernelGGL((k_small<T, false, true>), grid, dim3(kThreads), 0, s, a, src, src_stride, work, filt, dst,
                           dst_stride, sign, (int)scale_by_invM, tw);
    else if (src_is_samples && dst_is_samples)
        hipLaunchKernelGGL((k_small<T, true, true>), grid, dim3(kThreads), 0, s, a, src, src_stride, work, filt, dst,
                           dst_stride, sign, (int)scale_by_invM, tw);
    else
        hipLaunchKernelGGL((k_small<T, false, false>), grid, dim3(kThreads), 0, s, a, src, src_stride, work, filt,
                           dst, dst_stride, sign, (int)scale_by_invM, tw);
}

template <typename T>
void launch_p1(const TxArgs& a, const cx<T>* src, int64_t src_stride, bool src_is_samples, cx<T>* work, int sign,
               hipStream_t s) {
    if (a.nlarge == 0 || a.n_rhs == 0) return;
    int dev = 0;
    hipGetDevice(&dev);
    const cx<T>* tw = twiddles<T>(dev);
    dim3 grid(a.tiles_col, (unsigned)a.n_rhs);
    if (src_is_samples)
        hipLaunchKernelGGL((k_p1<T, 0>), grid, dim3(kThreads), 0, s, a, src, src_stride, work, sign, tw);
    else
        hipLaunchKernelGGL((k_p1<T, 1>), grid, dim3(kThreads), 0, s, a, src, src_stride, work, sign, tw);
}

template <typename T>
void launch_p2(const TxArgs& a, cx<T>* work, const cx<T>* filt, int sign, hipStream_t s) {
    if (a.nlarge == 0 || a.n_rhs == 0) return;
    int dev = 0;
    hipGetDevice(&dev);
    const cx<T>* tw = twiddles<T>(dev);
    dim3 grid(a.tiles_row, (unsigned)a.n_rhs);
    hipLaunchKernelGGL((k_p2<T, true>), grid, dim3(kThreads), 0, s, a, work, filt, sign, tw);
}

template <typename T>
void launch_p3(const TxArgs& a, cx<T>* work, cx<T>* dst, int64_t dst_stride, bool dst_is_samples, int sign,
               bool scale_by_invM, hipStream_t s) {
    if (a.nlarge == 0 || a.n_rhs == 0) return;
    int dev = 0;
    hipGetDevice(&dev);
    const cx<T>* tw = twiddles<T>(dev);
    dim3 grid(a.tiles_col, (unsigned)a.n_rhs);
    if (dst_is_samples)
        hipLaunchKernelGGL((k_p3<T, true>), grid, dim3(kThreads), 0, s, a, work, dst, dst_stride, sign,
                           (int)scale_by_invM, tw);
    else
        hipLaunchKernelGGL((k_p3<T, false>), grid, dim3(kThreads), 0, s, a, work, dst, dst_stride, sign,
                           (int)scale_by_invM, tw);
}

#define MR1L_INST_FFT(T)                                                                                           \
    template void launch_bluestein_small<T>(const TxArgs&, const cx<T>*, int64_t, bool, cx<T>*, const cx<T>*,      \
                                            cx<T>*, int64_t, bool, int, bool, hipStream_t);                      \
    template void launch_p1<T>(const TxArgs&, const cx<T>*, int64_t, bool, cx<T>*, int, hipStream_t);             \
    template void launch_p2<T>(const TxArgs&, cx<T>*, const cx<T>*, int, hipStream_t);                            \
    template void launch_p3<T>(const TxArgs&, cx<T>*, cx<T>*, int64_t, bool, int, bool, hipStream_t);
MR1L_INST_FFT(float)
MR1L_INST_FFT(double)

// Filter spectra for every lattice of a plan (synchronous on s).  The double-precision DFT of
// b_l reuses the four-step stages 1-2 (or the one-block DFT) on a temporary buffer laid out like
// the work area (work_off, length 2^lgN).
template <typename T>
void build_filters(const LatDesc* hdesc, int L, const LatDesc* ddesc, cx<T>* filt, int64_t filt_total,
                   int device, hipStream_t s) {
    if (L == 0) return;
    (void)filt_total;
    int64_t tot = 0;
    int maxlg = 0;
    std::vector<int> smalls, larges, t0c, t0r;
    int tc = 0, tr = 0;
    for (int l = 0; l < L; ++l) {
        tot = std::max<int64_t>(tot, hdesc[l].work_off + ((int64_t)1 << hdesc[l].lgN));
        maxlg = std::max(maxlg, hdesc[l].lgN);
        if (hdesc[l].small) {
            smalls.push_back(l);
        } else {
            larges.push_back(l);
            constexpr int LGE = TileElems<double>::lg;
            const int lgC = std::min(hdesc[l].lgN2, LGE - hdesc[l].lgN1);
            const int lgR = std::min(hdesc[l].lgN1, LGE - hdesc[l].lgN2);
            t0c.push_back(tc);
            t0r.push_back(tr);
            tc += 1 << (hdesc[l].lgN2 - lgC);
            tr += 1 << (hdesc[l].lgN1 - lgR);
        }
    }
    t0c.push_back(tc);
    t0r.push_back(tr);
    cx<double>* tmp = nullptr;
    int* dsm = nullptr;
    int* dlg = nullptr;
    int* dt0c = nullptr;
    int* dt0r = nullptr;
    hipMalloc(&tmp, tot * sizeof(cx<double>));
    hipMalloc(&dsm, (smalls.size() + 1) * sizeof(int));
    hipMalloc(&dlg, (larges.size() + 1) * sizeof(int));
    hipMalloc(&dt0c, t0c.size() * sizeof(int));
    hipMalloc(&dt0r, t0r.size() * sizeof(int));
    if (!smalls.empty()) hipMemcpy(dsm, smalls.data(), smalls.size() * sizeof(int), hipMemcpyHostToDevice);
    if (!larges.empty()) hipMemcpy(dlg, larges.data(), larges.size() * sizeof(int), hipMemcpyHostToDevice);
    hipMemcpy(dt0c, t0c.data(), t0c.size() * sizeof(int), hipMemcpyHostToDevice);
    hipMemcpy(dt0r, t0r.data(), t0r.size() * sizeof(int), hipMemcpyHostToDevice);

    TxArgs a{};
    a.desc = ddesc;
    a.L = L;
    a.n_rhs = 1;
    a.work_stride = 0;
    a.large = dlg;
    a.tile0_col = dt0c;
    a.tile0_row = dt0r;
    a.nlarge = (int)larges.size();
    a.tiles_col = tc;
    a.tiles_row = tr;
    a.small = dsm;
    a.nsmall = (int)smalls.size();
    const cx<double>* tw = twiddles<double>(device);

    const int blocks = std::max(1, std::min(1024, (int)(((int64_t)1 << maxlg) / 256)));
    hipLaunchKernelGGL(k_filter_fill, dim3(blocks, L), dim3(256), 0, s, ddesc, L, tmp);
    if (a.nsmall) hipLaunchKernelGGL(k_small_dft<double>, dim3(a.nsmall), dim3(kThreads), 0, s, a, tmp, tw);
    if (a.nlarge) {
        hipLaunchKernelGGL((k_p1<double, 2>), dim3(tc, 1), dim3(kThreads), 0, s, a, (const cx<double>*)tmp,
                           (int64_t)0, tmp, -1, tw);
        hipLaunchKernelGGL((k_p2<double, false>), dim3(tr, 1), dim3(kThreads), 0, s, a, tmp,
                           (const cx<double>*)nullptr, -1, tw);
    }
    hipLaunchKernelGGL((k_filter_store<T>), dim3(blocks, L), dim3(256), 0, s, ddesc, (const cx<double>*)tmp, filt);
    hipStreamSynchronize(s);
    hipFree(tmp);
    hipFree(dsm);
    hipFree(dlg);
    hipFree(dt0c);
    hipFree(dt0r);
}
template void build_filters<float>(const LatDesc*, int, const LatDesc*, cx<float>*, int64_t, int, hipStream_t);
template void build_filters<double>(const LatDesc*, int, const LatDesc*, cx<double>*, int64_t, int, hipStream_t);

}  // namespace mr1l
