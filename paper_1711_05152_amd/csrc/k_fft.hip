// Prime-length DFTs of the rank-1 lattice FFT (Alg. 2, "rank-1 lattice FFT": one 1-D DFT of
// length M_l per lattice) via Bluestein's chirp-z identity
//     jm = (j^2 + m^2 - (m - j)^2) / 2,
//     X[m] = e^{s i pi m^2/M} sum_j (x[j] e^{s i pi j^2/M}) e^{-s i pi (m-j)^2/M},
// i.e. a cyclic convolution of length N >= 2M - 1: N = 2^lgN, or N = 3 * 2^lgN where that is shorter
// (the factor 3 then sits in the rows of stage 2, below).  Chirp phases are reduced exactly in
// integers (j^2 mod 2M) before sin/cos.
//
// Two code paths:
//  * one-block path (N <= 4096): one workgroup holds the whole convolution in LDS;
//  * four-step path: N = N1 * N2; stage 1 = chirp + zero-pad + column DFTs of length N1 + twiddles,
//    stage 2 = row DFTs of length N2, multiplication by the filter spectrum, inverse row DFTs,
//    stage 3 = inverse twiddles + inverse column DFTs + output chirp.  Stage 2 is where forward
//    and inverse transforms meet, so the filter spectrum is stored in that stage's layout and the
//    intermediate never needs a transpose.
// The tile DFTs of the four-step path are Stockham stages of radix up to 16 whose first and last
// stages work on registers (only the exchanges between stages go through LDS); the one-block path
// uses radix-8 stages in LDS.  Stage twiddles come from a table; single-precision chirps and
// four-step twiddles from a 256-entry LDS table plus a small-angle rotation.  Every length is a
// compile-time constant: lattices are grouped by convolution length and each group is launched
// with kernels specialised for its sizes.
#include <map>
#include <mutex>
#include <type_traits>
#include <cmath>
#include <vector>

#include "common.h"
#include "index_dev.h"
#include "runtime.h"

namespace mr1l {

// ---- twiddle tables --------------------------------------------------------------------------------
// tw[m] = e^{-2 pi i m/4096} (m < 4096), tw[4096 + m] = e^{-2 pi i m/2^24} (m < 4096),
// tw[kTw3Off + m] = e^{-2 pi i m/(3 * 2^11)} (m < 2^11: the radix-3 twiddles of rows of 3 * 2^k points).
constexpr int kTw3Off = 8192, kTw3Lg = 11;
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
    std::vector<cx<T>> h(kTw3Off + (1 << kTw3Lg));
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
    for (int m = 0; m < (1 << kTw3Lg); ++m) {
        double c, s;
        host_cispi2(m, 3.0L * (1 << kTw3Lg), &c, &s);
        h[kTw3Off + m] = make_cx<T>((T)c, (T)s);
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

// Single precision phases: e^{-2 pi i (idx/256)} from a 256-entry table in LDS times e^{-i th}
// for a residual angle |th| <= pi/256, with cos th = 1 - th^2/2 and sin th = th (1 - th^2/6)
// (dropped terms below 1e-9).  The integer part of the phase is reduced exactly before th is
// formed, so the result is accurate to a few ulp at any index.
constexpr int kPhLg = 8;
template <typename T> struct PhaseTab { static constexpr int n = sizeof(T) == 4 ? (1 << kPhLg) : 1; };

// ph[m] = e^{-2 pi i m/256} (every thread of the workgroup takes part; a barrier must follow)
template <typename T>
__device__ __forceinline__ void phase_fill(cx<T>* ph) {
    if constexpr (sizeof(T) == 4) {
        for (int m = threadIdx.x; m < (1 << kPhLg); m += blockDim.x) {
            float sn, c;
            sincospif(-(float)m * (2.0f / (1 << kPhLg)), &sn, &c);   // exact argument
            ph[m] = {c, sn};
        }
    }
}

__device__ __forceinline__ cx<float> tw_rot(const cx<float>* ph, int idx, float th) {
    const cx<float> t = ph[idx & ((1 << kPhLg) - 1)];
    const float t2 = th * th;
    const float c = fmaf(-0.5f, t2, 1.0f);
    const float sn = th * fmaf(-t2, 1.0f / 6.0f, 1.0f);
    return {t.x * c + t.y * sn, t.y * c - t.x * sn};
}

// e^{-2 pi i e / 2^lgN} for 0 <= e < 2^lgN <= 2^24 (ph: the LDS phase table, single precision)
template <typename T>
__device__ __forceinline__ cx<T> tw_pow2(uint32_t e, int lgN, const cx<T>* ph) {
    if constexpr (sizeof(T) == 4) {
        if (lgN <= kPhLg) return ph[e << (kPhLg - lgN)];
        const int sh = lgN - kPhLg;
        const uint32_t idx = (e + (1u << (sh - 1))) >> sh;
        const int rem = (int)e - (int)(idx << sh);
        return tw_rot(ph, (int)idx, (float)rem * (float)(6.283185307179586 / (double)(1 << lgN)));
    } else {
        T s, c;
        const T x = -(T)e * (T)ldexp(1.0, 1 - lgN);   // exact
        sincospi(x, &s, &c);
        return {c, s};
    }
}

// e^{-2 pi i e / (3 * 2^lgN)} for 0 <= e < 3 * 2^lgN: the numerator is exact, the division by 3 one
// rounding in double, then the same table + small-angle rotation (single) or sincospi (double)
template <typename T>
__device__ __forceinline__ cx<T> tw_n3(uint32_t e, int lgN, const cx<T>* ph) {
    if constexpr (sizeof(T) == 4) {
        const double tau = ldexp((double)e, kPhLg - lgN) * (1.0 / 3.0);   // turns of 1/256
        const double id = rint(tau);
        return tw_rot(ph, (int)id, (float)(tau - id) * (float)(6.283185307179586 / (1 << kPhLg)));
    } else {
        T s, c;
        sincospi(-ldexp((double)e, 1 - lgN) / 3.0, &s, &c);
        return {c, s};
    }
}

// e^{-2 pi i e / N} for the four-step length N = F3 * 2^lgN
template <typename T, int F3>
__device__ __forceinline__ cx<T> tw_len(uint32_t e, int lgN, const cx<T>* ph) {
    if constexpr (F3 == 1) return tw_pow2<T>(e, lgN, ph);
    else return tw_n3<T>(e, lgN, ph);
}

// e^{sign i pi (n^2 mod 2M)/M}
template <typename T>
__device__ __forceinline__ cx<T> chirp(int64_t n, int64_t M, double invM, int sign, const cx<T>* ph) {
    const double q = sq_mod_2M(n, M, 0.5 * invM);
    if constexpr (sizeof(T) == 4) {
        // e^{sign i pi q/M} = e^{-2 pi i tau/256}, tau = -sign q 128/M
        const double tau = (double)(-sign) * q * ((double)(1 << (kPhLg - 1)) * invM);
        const double id = rint(tau);
        return tw_rot(ph, (int)id, (float)(tau - id) * (float)(6.283185307179586 / (1 << kPhLg)));
    } else {
        return cispi<T>((double)sign * (q * invM));
    }
}

// bin m of lattice D holds exactly one frequency: seen and not multi in the alias bitmaps
__device__ __forceinline__ bool owned_bin(const uint32_t* __restrict__ bm, const LatDesc& D, int64_t m) {
    const uint32_t s = bm[D.bm_off + (m >> 5)], x = bm[D.bm_off + D.bm_words + (m >> 5)];
    return ((s & ~x) >> (m & 31)) & 1u;
}

// LDS index with one pad slot after every 8 elements: strided Stockham writes and column loads
// then spread over the banks instead of piling onto a few.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }
template <int ELEMS> struct Padded { static constexpr int v = ELEMS + (ELEMS >> 3) + 64; };

// Column rotation of the four-step tiles that touch the sample vector.  Lattice offsets in the
// samples are arbitrary, so a tile's C columns n2 = c0 .. c0+C-1 of a row would straddle 128-byte
// lines.  Stage 1 (forward) and stage 3 (adjoint) instead take the columns
// n2 = (c0 + col - rot) mod N2, rot = (sample address of n = 0, in elements) mod AL, whose samples
// are line-aligned, and the work area holds column n2 at position (n2 + rot) mod N2, so their
// work-area accesses stay aligned as well; stage 2 undoes (forward) or applies (adjoint) the
// rotation when it loads or stores a row.  rot_base is the sample pointer in elements mod 1024.
// Tiles of stages 1 and 3 (column DFTs): 2^TLG elements = C columns of N1 = 2^LGN1 values, 16 per
// thread.  The default 4096-element tile leaves C = 4096 / N1 columns, i.e. row segments shorter
// than a 128-byte line once N1 > 256 (fp32) or N1 > 512 (fp64); such lengths take a tile of C =
// 128 B / element columns instead, as far as LDS allows (2^14 fp32 / 2^13 fp64 elements, 148 KiB),
// run by 1024 or 512 threads.  Stage 2 has row tiles of its own (RowTile).
template <typename T, int LGN, int LG1>
struct ColTile {
    static constexpr int LGN1 = LG1;
    static constexpr int LINE_LG = sizeof(T) == 4 ? 4 : 3;        // log2(128 B / element)
    static constexpr int MAX_LG = sizeof(T) == 4 ? 14 : 13;
    static constexpr int WANT = LGN1 + LINE_LG;
    static constexpr int TLG = WANT < kTileLg ? kTileLg : (WANT > MAX_LG ? MAX_LG : WANT);
    static constexpr int LGC = TLG - LGN1, C = 1 << LGC;
    static constexpr int NT = (1 << TLG) / 16;                     // threads: 16 values each
    // tiles whose row pieces make up one 128-byte line (1 while a tile's rows are whole lines)
    static constexpr int G = LGC < LINE_LG ? (1 << (LINE_LG - LGC)) : 1;
};

// Tile of workgroup b (of nb).  Workgroups are dispatched to the eight XCDs in turn, so b, b + 8,
// ..., b + 8 (G - 1) share an XCD and start close together: they take the G tiles whose row pieces
// share 128-byte lines, which each XCD's L2 then fetches once.  A permutation of the tiles (the
// last nb mod 8G workgroups keep their own index).
template <int G>
__device__ __forceinline__ int line_tile(int b, int nb) {
    if constexpr (G == 1) {
        return b;
    } else {
        const int full = nb / (8 * G) * (8 * G);
        if (b >= full) return b;
        const int r = b % (8 * G);
        return (b - r) + (r % 8) * G + r / 8;
    }
}

template <typename T, int LGN, int LG1>
struct Rot {
    static constexpr int C = ColTile<T, LGN, LG1>::C;
    static constexpr int AL = C < (int)(128 / sizeof(cx<T>)) ? C : (int)(128 / sizeof(cx<T>));
    __device__ static int of(int rot_base, int64_t rhs, int64_t stride, int64_t samp_off) {
        return (int)(((int64_t)rot_base + rhs * stride + samp_off) & (AL - 1));
    }
};

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


// x * e^{SIGN 2 pi i E/16} for a compile-time E
template <typename T, int SIGN, int E>
__device__ __forceinline__ cx<T> rot16(cx<T> x) {
    constexpr int e = E & 15;
    if constexpr (e == 0) return x;
    else if constexpr (e == 4) return mul_si<T, SIGN>(x);
    else if constexpr (e == 8) return cx<T>{-x.x, -x.y};
    else if constexpr (e == 12) return mul_si<T, -SIGN>(x);
    else {
        // cos and sin of 2 pi e / 16
        constexpr double C1 = 0.923879532511286756128183189396788933, S1 = 0.382683432365089771728459984030398866;
        constexpr double C2 = 0.707106781186547524400844362104849039;
        constexpr double cs[16] = {1, C1, C2, S1, 0, -S1, -C2, -C1, -1, -C1, -C2, -S1, 0, S1, C2, C1};
        constexpr double sn[16] = {0, S1, C2, C1, 1, C1, C2, S1, 0, -S1, -C2, -C1, -1, -C1, -C2, -S1};
        const T wc = (T)cs[e], ws = (T)(SIGN * sn[e]);
        return {x.x * wc - x.y * ws, x.x * ws + x.y * wc};
    }
}

// radix 16 as 4 x 4: DFT-4 over the residues mod 4, twiddles w16^{m k1}, DFT-4 across
template <typename T, int SIGN> struct Dft<T, 16, SIGN> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        cx<T> a[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int q = 0; q < 4; ++q) a[m][q] = v[m + 4 * q];
            Dft<T, 4, SIGN>::run(a[m]);
        }
        a[1][1] = rot16<T, SIGN, 1>(a[1][1]);
        a[1][2] = rot16<T, SIGN, 2>(a[1][2]);
        a[1][3] = rot16<T, SIGN, 3>(a[1][3]);
        a[2][1] = rot16<T, SIGN, 2>(a[2][1]);
        a[2][2] = rot16<T, SIGN, 4>(a[2][2]);
        a[2][3] = rot16<T, SIGN, 6>(a[2][3]);
        a[3][1] = rot16<T, SIGN, 3>(a[3][1]);
        a[3][2] = rot16<T, SIGN, 6>(a[3][2]);
        a[3][3] = rot16<T, SIGN, 9>(a[3][3]);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            Dft<T, 4, SIGN>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
        }
    }
};

// ---- Stockham stages with compile-time sizes -------------------------------------------------------
// NSEQ sequences of length 2^LGN stored at buf[pidx(b*S + e)].  2^LGNS is the length of the
// sub-transforms already done; this stage has radix 2^LR.
template <typename T, int LGN, int NSEQ, int S, int SIGN, int LGNS, int LR>
__device__ __forceinline__ void stage_ct(cx<T>* buf, const cx<T>* __restrict__ tw) {
    constexpr int R = 1 << LR;
    constexpr int LGNB = LGN - LR;
    constexpr int NBF = 1 << LGNB;            // butterflies per sequence
    constexpr int TOTAL = NBF * NSEQ;
    constexpr int NB = (TOTAL + kThreads - 1) / kThreads;
    constexpr bool FULL = (TOTAL % kThreads) == 0;
    cx<T> v[NB][R];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int g = threadIdx.x + u * kThreads;
        if (FULL || g < TOTAL) {
            const int b = g >> LGNB, j = g & (NBF - 1);
            const int base = b * S + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = buf[pidx(base + (r << LGNB))];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int g = threadIdx.x + u * kThreads;
        if (FULL || g < TOTAL) {
            const int b = g >> LGNB, j = g & (NBF - 1);
            const int k = j & ((1 << LGNS) - 1);
            if constexpr (LGNS > 0) {
                const int step = k << (kTwLg - LGNS - LR);   // w_{Ns R}^{k} = tw[k 4096/(Ns R)]
                // powers w^r from the exact table values w, w^2, w^4 and at most two products
                cx<T> w[R];
                w[1] = tw[step];
                if constexpr (R >= 4) {
                    w[2] = tw[2 * step];
                    w[3] = cmul(w[1], w[2]);
                }
                if constexpr (R >= 8) {
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
            for (int r = 0; r < R; ++r) buf[pidx(base + (r << LGNS))] = v[u][r];
        }
    }
    __syncthreads();
}

// In-LDS DFT (SIGN -1: e^{-2 pi i nk/N}, +1: e^{+...}, unnormalized), natural order in and out.
template <typename T, int LGN, int NSEQ, int S, int SIGN, int LGNS = 0>
__device__ __forceinline__ void fft_ct(cx<T>* buf, const cx<T>* __restrict__ tw) {
    if constexpr (LGNS < LGN) {
        constexpr int LR = (LGNS == 0 && (LGN % 3) != 0) ? (LGN % 3) : 3;
        stage_ct<T, LGN, NSEQ, S, SIGN, LGNS, LR>(buf, tw);
        fft_ct<T, LGN, NSEQ, S, SIGN, LGNS + LR>(buf, tw);
    }
}

// ---- register-resident FFTs for the four-step tiles ------------------------------------------------
// A tile holds NSEQ sequences of 2^LGN values (NSEQ * 2^LGN = 2048 or 4096): every thread owns 16
// values of each stage (8 under radix orders 4 / 5).  The first stage takes its inputs from registers (the caller loads them from
// global memory in that stage's order) and the last stage leaves its outputs in registers (the
// caller stores them), so only the exchanges between stages go through LDS.  The radix schedule
// (REMF: the radix order of stage_lr in common.h) distributes the bits over the stages; which
// schedule a stage-2 length uses is one of the choices of the autotuner.

constexpr int kVals = (1 << kTileLg) / kThreads;   // values per thread (16)

// butterfly u of this thread in a stage with 2^LGNB butterflies per sequence: (sequence b, index j).
// BF: sequence index fastest across threads (column tiles), else j fastest (row tiles).
template <int LGNB, int NSEQ, bool BF, int NT = kThreads>
__device__ __forceinline__ void bfly(int u, int& b, int& j) {
    const int g = threadIdx.x + u * NT;
    if constexpr (BF) {
        b = g & (NSEQ - 1);
        j = g / NSEQ;
    } else {
        b = g >> LGNB;
        j = g & ((1 << LGNB) - 1);
    }
}

// twiddles and radix-2^LR DFTs of stage I on the registers
template <typename T, int LGN, int NSEQ, int SIGN, int REMF, int I, bool BF, int NT = kThreads>
__device__ __forceinline__ void stage_compute(cx<T>* v, const cx<T>* __restrict__ tw) {
    constexpr int LR = stage_lr(LGN, I, REMF), R = 1 << LR;
    constexpr int LGNS = stage_lgns(LGN, I, REMF);
    constexpr int LGNB = LGN - LR;
    constexpr int NB = (1 << ord_lgv(REMF)) / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        int b, j;
        bfly<LGNB, NSEQ, BF, NT>(u, b, j);
        cx<T>* x = v + u * R;
        if constexpr (LGNS > 0) {
            const int k = j & ((1 << LGNS) - 1);
            const int step = k << (kTwLg - LGNS - LR);
            // w, w^2, w^4, w^8 from the table and the other powers as products; in double precision
            // the even powers are squares of w instead (one 16-byte load per butterfly: complex128
            // standalone step 0.208 -> 0.205 ms; in single precision the loads measured faster)
            constexpr bool SQ = sizeof(T) == 8;
            cx<T> w[R];
            w[1] = tw[step];
            if constexpr (R >= 4) {
                w[2] = SQ ? cmul(w[1], w[1]) : tw[2 * step];
                w[3] = cmul(w[1], w[2]);
            }
            if constexpr (R >= 8) {
                w[4] = SQ ? cmul(w[2], w[2]) : tw[4 * step];
                w[5] = cmul(w[1], w[4]);
                w[6] = cmul(w[2], w[4]);
                w[7] = cmul(w[3], w[4]);
            }
            if constexpr (R >= 16) {
                w[8] = SQ ? cmul(w[4], w[4]) : tw[8 * step];
#pragma unroll
                for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) x[r] = SIGN < 0 ? cmul(x[r], w[r]) : cmulc(x[r], w[r]);
        }
        Dft<T, R, SIGN>::run(x);
    }
}

// outputs of stage I -> LDS
template <typename T, int LGN, int NSEQ, int S, int REMF, int I, bool BF, int NT = kThreads>
__device__ __forceinline__ void stage_store(cx<T>* buf, const cx<T>* v) {
    constexpr int LR = stage_lr(LGN, I, REMF), R = 1 << LR;
    constexpr int LGNS = stage_lgns(LGN, I, REMF);
    constexpr int LGNB = LGN - LR;
    constexpr int NB = (1 << ord_lgv(REMF)) / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        int b, j;
        bfly<LGNB, NSEQ, BF, NT>(u, b, j);
        const int k = j & ((1 << LGNS) - 1);
        const int base = b * S + ((j - k) << LR) + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[pidx(base + (r << LGNS))] = v[u * R + r];
    }
}

// inputs of stage I <- LDS
template <typename T, int LGN, int NSEQ, int S, int REMF, int I, bool BF, int NT = kThreads>
__device__ __forceinline__ void stage_load(const cx<T>* buf, cx<T>* v) {
    constexpr int LR = stage_lr(LGN, I, REMF), R = 1 << LR;
    constexpr int LGNB = LGN - LR;
    constexpr int NB = (1 << ord_lgv(REMF)) / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        int b, j;
        bfly<LGNB, NSEQ, BF, NT>(u, b, j);
        const int base = b * S + j;
#pragma unroll
        for (int r = 0; r < R; ++r) v[u * R + r] = buf[pidx(base + (r << LGNB))];
    }
}

// stages I..last; stage I's inputs are in v (mapping BF0 for I = 0, else j-fast); the last stage
// uses mapping BFL.  On return v holds the last stage's outputs and all LDS reads are done.
template <typename T, int LGN, int NSEQ, int S, int SIGN, int REMF, bool BF0, bool BFL, int NT = kThreads, int I = 0>
__device__ __forceinline__ void fft_regs(cx<T>* buf, cx<T>* v, const cx<T>* __restrict__ tw) {
    constexpr int NS = n_stages(LGN, REMF);
    constexpr bool BFI = (I == NS - 1) ? BFL : (I == 0 ? BF0 : false);
    stage_compute<T, LGN, NSEQ, SIGN, REMF, I, BFI, NT>(v, tw);
    if constexpr (I + 1 < NS) {
        constexpr bool BFN = (I + 1 == NS - 1) ? BFL : false;
        stage_store<T, LGN, NSEQ, S, REMF, I, BFI, NT>(buf, v);
        __syncthreads();
        stage_load<T, LGN, NSEQ, S, REMF, I + 1, BFN, NT>(buf, v);
        __syncthreads();
        fft_regs<T, LGN, NSEQ, S, SIGN, REMF, BF0, BFL, NT, I + 1>(buf, v, tw);
    }
}

// ---- four-step stage 1 -----------------------------------------------------------------------------
// One tile = C columns of the N1 x N2 arrangement (N = F3 * 2^LGN, N1 = 2^LGN1, N2 = F3 * 2^LGN2);
// tiles per lattice N / 2^TLG.
// SRC 0: x = samples * chirp, 1: x = work (bins) * chirp, 2: x = work as is (all N entries),
// 3: x = work (bins) * chirp where the alias bitmaps mark the bin as holding exactly one frequency,
// else 0 (the adjoint's scatter writes only those bins).
template <typename T, int LGN, int LG1, int SRC, int F3 = 1>
__global__ __launch_bounds__((ColTile<T, LGN, LG1>::NT)) void k_p1(TxArgs a, const int* __restrict__ lat,
                                                            const cx<T>* __restrict__ src, int64_t src_stride,
                                                            cx<T>* work, int sign, const cx<T>* __restrict__ tw,
                                                            int rot_base) {
    using CT = ColTile<T, LGN, LG1>;
    constexpr int LGN1 = CT::LGN1, LGN2 = LGN - LGN1;
    constexpr int LGC = CT::LGC, C = CT::C, N1 = 1 << LGN1, NT = CT::NT;
    constexpr int S = N1 + 1;
    constexpr int TPL = F3 << (LGN - CT::TLG);   // tiles per lattice
    constexpr int N2 = F3 << LGN2;
    constexpr int NS = n_stages(LGN1);
    constexpr int LR0 = stage_lr(LGN1, 0, true), R0 = 1 << LR0, LGNB0 = LGN1 - LR0;
    constexpr int LRL = stage_lr(LGN1, NS - 1, true), RL = 1 << LRL, LGNBL = LGN1 - LRL;
    __shared__ cx<T> lds[Padded<(1 << CT::TLG) + C>::v];
    __shared__ cx<T> ph[PhaseTab<T>::n];
    phase_fill<T>(ph);
    __syncthreads();
    const int tb = line_tile<CT::G>((int)blockIdx.x, (int)gridDim.x);
    const int li = tb / TPL;
    const int c0 = (tb - li * TPL) << LGC;
    const LatDesc D = a.desc[lat[li]];
    const int64_t rhs = blockIdx.y;
    const cx<T>* in = src + rhs * src_stride + (SRC == 0 ? D.samp_off : D.work_off);
    cx<T>* w = work + rhs * a.work_stride + D.work_off;
    const int64_t nvalid = (SRC == 2) ? ((int64_t)F3 << LGN) : D.M;
    const int rot = SRC == 0 ? Rot<T, LGN, LG1>::of(rot_base, rhs, src_stride, D.samp_off) : 0;
    // column n2 of tile column col: (c0 + col - rot) mod N2, c0 + col < N2 and rot < C
    auto colv = [&](int col) -> int {
        const int x = c0 + col - rot;
        return x < 0 ? x + N2 : x;
    };
    cx<T> v[kVals];
#pragma unroll
    for (int u = 0; u < kVals / R0; ++u) {
        int col, j;
        bfly<LGNB0, C, true, NT>(u, col, j);
        const int n2 = colv(col);
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int64_t n = (int64_t)(j + (r << LGNB0)) * N2 + n2;
            cx<T> x = {(T)0, (T)0};
            if (n < nvalid) {
                x = in[n];
                if (SRC != 2) x = cmul(x, chirp<T>(n, D.M, D.invM, sign, ph));
                if (SRC == 3 && !owned_bin(a.bitmaps, D, n)) x = {(T)0, (T)0};
            }
            v[u * R0 + r] = x;
        }
    }
    fft_regs<T, LGN1, C, S, -1, true, true, true, NT>(lds, v, tw);
    // outputs: column n2, k1 = j + r N1/RL; times w_N^{n2 k1}, stored at k1 N2 + (n2 + rot) mod N2
#pragma unroll
    for (int u = 0; u < kVals / RL; ++u) {
        int col, j;
        bfly<LGNBL, C, true, NT>(u, col, j);
        const int n2 = colv(col);
        // n2 j and n2 2^LGNBL are below N (n2 < N2, j and 2^LGNBL below N1)
        cx<T> wk = tw_len<T, F3>((uint32_t)(n2 * j), LGN, ph);
        const cx<T> ws = tw_len<T, F3>((uint32_t)(n2 << LGNBL), LGN, ph);
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int k1 = j + (r << LGNBL);
            w[(int64_t)k1 * N2 + c0 + col] = cmul(v[u * RL + r], wk);
            wk = cmul(wk, ws);
        }
    }
}

// ---- four-step stage 2 -----------------------------------------------------------------------------
// Row tiles: 2^TLG elements = 2^(TLG - LGN2) rows, at least two (a mirror pair) while LGN2 < 12,
// run by NT threads of 2^LGV values (16, or 8 with twice the threads).  Rows of up to 2^10 points take 2048-element tiles: workgroups
// of two waves instead of four, so each barrier holds fewer waves and the loads of some workgroups
// on a CU overlap the arithmetic of others (the same waves per CU either way).
template <int LGN, int LG1, int BIG = 0, int LGV = 4>
struct RowTile {
    static constexpr int LGN2 = LGN - LG1;
    static constexpr int TLG = (BIG || LGN2 + 1 > kP2TileLg) ? kTileLg : kP2TileLg;
    static constexpr int NT = (1 << TLG) >> LGV;
    static_assert(TLG >= LGN2 && TLG <= kTileLg, "row tile");
};

// One tile = 2^(TLG - LGN2) rows.  CONV: row DFT, multiply by the filter (conjugated for sign +1),
// inverse row DFT (the forward's last stage and the inverse's first stage have the same radix and
// hold the same elements, so the product never leaves the registers); else row DFT only.
template <typename T, int LGN, int LG1, bool CONV, int V = 0>
__global__ __launch_bounds__((RowTile<LGN, LG1, (V >> 1) & 1, (V & 4) ? 3 : 4>::NT))
void k_p2(TxArgs a, const int* __restrict__ lat, cx<T>* work, const cx<T>* __restrict__ filt, int sign,
          const cx<T>* __restrict__ tw, int rot_in_base, int rot_out_base) {
    using RT = RowTile<LGN, LG1, (V >> 1) & 1, (V & 4) ? 3 : 4>;
    // forward / inverse radix orders
    constexpr int OF = (V & 4) ? 5 : ((V & 1) ? 3 : 1), OI = (V & 4) ? 4 : ((V & 1) ? 2 : 0);
    constexpr int VPT = 1 << ord_lgv(OF);
    constexpr int LGN1 = LG1, LGN2 = LGN - LGN1, NT = RT::NT;
    constexpr int LGR = RT::TLG - LGN2, ROWS = 1 << LGR, N2 = 1 << LGN2, N1 = 1 << LGN1;
    constexpr int TPL_LG = LGN - RT::TLG;
    constexpr int LR0 = stage_lr(LGN2, 0, OF), R0 = 1 << LR0, LGNB0 = LGN2 - LR0;
    constexpr int NSI = n_stages(LGN2, OF);
    constexpr int LRM = stage_lr(LGN2, NSI - 1, OF), RM = 1 << LRM;   // forward last = inverse first
    constexpr int LGNBM = LGN2 - LRM;
    constexpr int LRL = stage_lr(LGN2, NSI - 1, OI), RL = 1 << LRL, LGNBL = LGN2 - LRL;
    static_assert(stage_lr(LGN2, 0, OI) == LRM, "the forward's last and the inverse's first stage must match");
    __shared__ cx<T> lds[Padded<(1 << RT::TLG)>::v];
    const int li = blockIdx.x >> TPL_LG;
    const int t = blockIdx.x & ((1 << TPL_LG) - 1);
    const LatDesc D = a.desc[lat[li]];
    const int64_t rhs = blockIdx.y;
    cx<T>* w = work + rhs * a.work_stride + D.work_off;
    // rotation of the rows as stored by stage 1 / as stage 3 reads them (rot_*_base < 0: none)
    const int rin = rot_in_base < 0 ? 0 : Rot<T, LGN, LG1>::of(rot_in_base, rhs, a.samp_stride, D.samp_off);
    const int rout = rot_out_base < 0 ? 0 : Rot<T, LGN, LG1>::of(rot_out_base, rhs, a.samp_stride, D.samp_off);
    // Rows of the tile: ROWS/2 mirror pairs (p, N1 - p) of the [k1][k2] layout, pair 0 being
    // (0, N1/2).  The filter spectrum is even (B[k] = B[N - k]), i.e. B[k1][k2] = B[N1-k1][N2-1-k2]
    // for 0 < k1 < N1, so the second row of a pair reads its partner's filter values (the same
    // lines, reversed) and the tile fetches half of the filter bytes.
    constexpr int H = ROWS > 1 ? ROWS / 2 : 1;
    auto prow = [&](int b) -> int {
        if constexpr (ROWS == 1) return t;
        const int p = t * H + (b & (H - 1));
        return b < H ? p : (p == 0 ? N1 / 2 : N1 - p);
    };
    cx<T> v[VPT];
#pragma unroll
    for (int u = 0; u < VPT / R0; ++u) {
        int b, j;
        bfly<LGNB0, ROWS, false, NT>(u, b, j);
        const cx<T>* src = w + ((int64_t)prow(b) << LGN2);
#pragma unroll
        for (int r = 0; r < R0; ++r) v[u * R0 + r] = src[(j + (r << LGNB0) + rin) & (N2 - 1)];
    }
    fft_regs<T, LGN2, ROWS, N2, -1, OF, false, false, NT>(lds, v, tw);
    if constexpr (CONV) {
        const cx<T>* f = filt + D.filt_off;
#pragma unroll
        for (int u = 0; u < VPT / RM; ++u) {
            int b, j;
            bfly<LGNBM, ROWS, false, NT>(u, b, j);
            const int p = t * H + (b & (H - 1));
            const bool mirror = ROWS > 1 && b >= H && p != 0;
            const cx<T>* fr = f + ((int64_t)(mirror ? p : prow(b)) << LGN2);
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                const int c = j + (r << LGNBM);
                const cx<T> fv = fr[mirror ? N2 - 1 - c : c];
                v[u * RM + r] = sign < 0 ? cmul(v[u * RM + r], fv) : cmulc(v[u * RM + r], fv);
            }
        }
        fft_regs<T, LGN2, ROWS, N2, +1, OI, false, false, NT>(lds, v, tw);
#pragma unroll
        for (int u = 0; u < VPT / RL; ++u) {
            int b, j;
            bfly<LGNBL, ROWS, false, NT>(u, b, j);
            cx<T>* dstp = w + ((int64_t)prow(b) << LGN2);
#pragma unroll
            for (int r = 0; r < RL; ++r) dstp[(j + (r << LGNBL) + rout) & (N2 - 1)] = v[u * RL + r];
        }
    } else {
#pragma unroll
        for (int u = 0; u < VPT / RM; ++u) {
            int b, j;
            bfly<LGNBM, ROWS, false, NT>(u, b, j);
            cx<T>* dstp = w + ((int64_t)prow(b) << LGN2);
#pragma unroll
            for (int r = 0; r < RM; ++r) dstp[j + (r << LGNBM)] = v[u * RM + r];
        }
    }
}

// ---- stage 2 for N = 3 * 2^LGN ---------------------------------------------------------------------
// Rows of N2 = 3Q points, Q = 2^LGN2.  Decimation in time by 3: the row DFT is three Q-point DFTs
// Y_s of x[3m + s] (register tile DFTs over the 3 ROWS sequences of a tile, loaded straight from
// the row) and one radix-3 pass,
//   X[k + tQ] = sum_s e^{-2 pi i s k/(3Q)} Y_s[k] e^{-2 pi i s t/3}      (k < Q, t < 3),
// done in LDS together with the filter product and the inverse radix-3 pass; the inverse Q-point
// DFTs then leave x[3m + s] in registers for the store.  A tile holds 3 * 2^TLG3 elements: ROWS =
// 2^(TLG3 - LGN2) rows, mirror pairs as in stage 2 above.
template <int LGN, int LG1>
struct RowTile3 {
    static constexpr int LGN2 = LGN - LG1;
    static constexpr int TLG3 = LGN2 > 10 ? LGN2 : 10;
    static constexpr int ELEMS = 3 << TLG3;
    static constexpr int NT = ELEMS / 16;
    static_assert(LGN2 >= 4 && LGN2 <= 11 && NT <= 1024, "row tile of stage 2 for N = 3 * 2^LGN");
};

// 3-point DFT with e^{SIGN 2 pi i/3}
template <typename T, int SIGN>
__device__ __forceinline__ void dft3(cx<T> y0, cx<T> y1, cx<T> y2, cx<T>& x0, cx<T>& x1, cx<T>& x2) {
    const T h = (T)0.866025403784438646763723170752936183;   // sqrt(3)/2
    const cx<T> p = y1 + y2, q = y1 - y2;
    const cx<T> m = {y0.x - (T)0.5 * p.x, y0.y - (T)0.5 * p.y};
    const cx<T> r = mul_si<T, SIGN>(cx<T>{h * q.x, h * q.y});   // SIGN i (sqrt(3)/2) (y1 - y2)
    x0 = y0 + p;
    x1 = m + r;
    x2 = m - r;
}

template <typename T, int LGN, int LG1, bool CONV>
__global__ __launch_bounds__((RowTile3<LGN, LG1>::NT)) void k_p2r3(TxArgs a, const int* __restrict__ lat, cx<T>* work,
                                                            const cx<T>* __restrict__ filt, int sign,
                                                            const cx<T>* __restrict__ tw, int rot_in_base,
                                                            int rot_out_base) {
    using RT = RowTile3<LGN, LG1>;
    constexpr int OF = 1, OI = 0;
    constexpr int LGQ = RT::LGN2, Q = 1 << LGQ, N2 = 3 * Q, N1 = 1 << LG1, NT = RT::NT;
    constexpr int LGR = RT::TLG3 - LGQ, ROWS = 1 << LGR, NSEQ = 3 * ROWS;
    constexpr int TPL_LG = LGN - RT::TLG3;   // tiles per lattice: N / (3 * 2^TLG3)
    constexpr int LR0 = stage_lr(LGQ, 0, OF), R0 = 1 << LR0, LGNB0 = LGQ - LR0;
    constexpr int NSF = n_stages(LGQ, OF), NSI = n_stages(LGQ, OI);
    constexpr int LRL = stage_lr(LGQ, NSI - 1, OI), RL = 1 << LRL, LGNBL = LGQ - LRL;
    constexpr int NTRI = (ROWS * Q + NT - 1) / NT;   // radix-3 points per thread (16/3 rounded up)
    __shared__ cx<T> lds[Padded<RT::ELEMS>::v];
    const int li = blockIdx.x >> TPL_LG;
    const int t = blockIdx.x & ((1 << TPL_LG) - 1);
    const LatDesc D = a.desc[lat[li]];
    const int64_t rhs = blockIdx.y;
    cx<T>* w = work + rhs * a.work_stride + D.work_off;
    const int rin = rot_in_base < 0 ? 0 : Rot<T, LGN, LG1>::of(rot_in_base, rhs, a.samp_stride, D.samp_off);
    const int rout = rot_out_base < 0 ? 0 : Rot<T, LGN, LG1>::of(rot_out_base, rhs, a.samp_stride, D.samp_off);
    constexpr int H = ROWS > 1 ? ROWS / 2 : 1;
    auto prow = [&](int row) -> int {
        if constexpr (ROWS == 1) return t;
        const int p = t * H + (row & (H - 1));
        return row < H ? p : (p == 0 ? N1 / 2 : N1 - p);
    };
    // sequence b = s ROWS + row: x[3m + s] of tile row `row`, m < Q (stage 1's rotation undone)
    cx<T> v[16];
#pragma unroll
    for (int u = 0; u < 16 / R0; ++u) {
        int b, j;
        bfly<LGNB0, NSEQ, false, NT>(u, b, j);
        const int sres = b >> LGR, row = b & (ROWS - 1);
        const cx<T>* src = w + (int64_t)prow(row) * N2;
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int e = 3 * (j + (r << LGNB0)) + sres + rin;   // < 2 N2
            v[u * R0 + r] = src[e >= N2 ? e - N2 : e];
        }
    }
    fft_regs<T, LGQ, NSEQ, Q, -1, OF, false, false, NT>(lds, v, tw);
    // every LDS read of the DFTs is done (fft_regs ends with a barrier after its last load)
    stage_store<T, LGQ, NSEQ, Q, OF, NSF - 1, false, NT>(lds, v);   // Y_s[k] at (s ROWS + row) Q + k
    __syncthreads();
    const cx<T>* f = CONV ? filt + D.filt_off : nullptr;
#pragma unroll
    for (int kk = 0; kk < NTRI; ++kk) {
        const int e = threadIdx.x + kk * NT;
        if (e >= ROWS * Q) break;
        const int row = e >> LGQ, k = e & (Q - 1);
        const int i0 = pidx(row * Q + k), i1 = pidx((ROWS + row) * Q + k), i2 = pidx((2 * ROWS + row) * Q + k);
        const cx<T> w1 = tw[kTw3Off + (k << (kTw3Lg - LGQ))];   // e^{-2 pi i k/(3Q)}
        const cx<T> w2 = cmul(w1, w1);
        cx<T> x0, x1, x2;
        dft3<T, -1>(lds[i0], cmul(lds[i1], w1), cmul(lds[i2], w2), x0, x1, x2);
        if constexpr (CONV) {
            // filter B[k1][k2] = B[N1 - k1][N2 - 1 - k2] (0 < k1 < N1): a mirror row reads its partner's
            const int p = ROWS > 1 ? t * H + (row & (H - 1)) : t;
            const bool mirror = ROWS > 1 && row >= H && p != 0;
            const cx<T>* fr = f + (int64_t)(mirror ? p : prow(row)) * N2;
            const cx<T> f0 = fr[mirror ? N2 - 1 - k : k];
            const cx<T> f1 = fr[mirror ? N2 - 1 - (k + Q) : k + Q];
            const cx<T> f2 = fr[mirror ? N2 - 1 - (k + 2 * Q) : k + 2 * Q];
            x0 = sign < 0 ? cmul(x0, f0) : cmulc(x0, f0);
            x1 = sign < 0 ? cmul(x1, f1) : cmulc(x1, f1);
            x2 = sign < 0 ? cmul(x2, f2) : cmulc(x2, f2);
            cx<T> z0, z1, z2;
            dft3<T, +1>(x0, x1, x2, z0, z1, z2);
            lds[i0] = z0;
            lds[i1] = cmulc(z1, w1);
            lds[i2] = cmulc(z2, w2);
        } else {
            // forward row DFT only (filter construction): natural order, no rotation
            cx<T>* dstp = w + (int64_t)prow(row) * N2;
            dstp[k] = x0;
            dstp[k + Q] = x1;
            dstp[k + 2 * Q] = x2;
        }
    }
    if constexpr (CONV) {
        __syncthreads();
        stage_load<T, LGQ, NSEQ, Q, OI, 0, false, NT>(lds, v);
        __syncthreads();
        fft_regs<T, LGQ, NSEQ, Q, +1, OI, false, false, NT>(lds, v, tw);
#pragma unroll
        for (int u = 0; u < 16 / RL; ++u) {
            int b, j;
            bfly<LGNBL, NSEQ, false, NT>(u, b, j);
            const int sres = b >> LGR, row = b & (ROWS - 1);
            cx<T>* dstp = w + (int64_t)prow(row) * N2;
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int e = 3 * (j + (r << LGNBL)) + sres + rout;
                dstp[e >= N2 ? e - N2 : e] = v[u * RL + r];
            }
        }
    }
}

// ---- four-step stage 3 -----------------------------------------------------------------------------
template <typename T, int LGN, int LG1, bool TO_SAMPLES, int F3 = 1>
__global__ __launch_bounds__((ColTile<T, LGN, LG1>::NT)) void k_p3(TxArgs a, const int* __restrict__ lat, cx<T>* work,
                                                            cx<T>* dst, int64_t dst_stride, int sign,
                                                            int scale_by_invM, const cx<T>* __restrict__ tw,
                                                            int rot_base) {
    using CT = ColTile<T, LGN, LG1>;
    constexpr int LGN1 = CT::LGN1, LGN2 = LGN - LGN1;
    constexpr int LGC = CT::LGC, C = CT::C, N1 = 1 << LGN1, NT = CT::NT;
    constexpr int S = N1 + 1;
    constexpr int TPL = F3 << (LGN - CT::TLG);   // tiles per lattice
    constexpr int N2 = F3 << LGN2;
    constexpr int NS = n_stages(LGN1);
    constexpr int LR0 = stage_lr(LGN1, 0, false), R0 = 1 << LR0, LGNB0 = LGN1 - LR0;
    constexpr int LRL = stage_lr(LGN1, NS - 1, false), RL = 1 << LRL, LGNBL = LGN1 - LRL;
    __shared__ cx<T> lds[Padded<(1 << CT::TLG) + C>::v];
    __shared__ cx<T> ph[PhaseTab<T>::n];
    phase_fill<T>(ph);
    __syncthreads();
    const int tb = line_tile<CT::G>((int)blockIdx.x, (int)gridDim.x);
    const int li = tb / TPL;
    const int c0 = (tb - li * TPL) << LGC;
    const LatDesc D = a.desc[lat[li]];
    const int64_t rhs = blockIdx.y;
    cx<T>* w = work + rhs * a.work_stride + D.work_off;
    const int rot = TO_SAMPLES ? Rot<T, LGN, LG1>::of(rot_base, rhs, dst_stride, D.samp_off) : 0;
    auto colv = [&](int col) -> int {
        const int x = c0 + col - rot;
        return x < 0 ? x + N2 : x;
    };
    cx<T> v[kVals];
#pragma unroll
    for (int u = 0; u < kVals / R0; ++u) {
        int col, j;
        bfly<LGNB0, C, true, NT>(u, col, j);
        const int n2 = colv(col);
        cx<T> wk = tw_len<T, F3>((uint32_t)(n2 * j), LGN, ph);
        const cx<T> ws = tw_len<T, F3>((uint32_t)(n2 << LGNB0), LGN, ph);
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k1 = j + (r << LGNB0);
            v[u * R0 + r] = cmulc(w[(int64_t)k1 * N2 + c0 + col], wk);
            wk = cmul(wk, ws);
        }
    }
    fft_regs<T, LGN1, C, S, +1, false, true, true, NT>(lds, v, tw);
    cx<T>* out = TO_SAMPLES ? dst + rhs * dst_stride + D.samp_off : w;
    const T sc = scale_by_invM ? (T)D.invM : (T)1;
    // the inverse column DFTs read all of the tile before any thread writes (fft_regs ends with a
    // barrier after its last LDS read), so writing the outputs in place is safe
#pragma unroll
    for (int u = 0; u < kVals / RL; ++u) {
        int col, j;
        bfly<LGNBL, C, true, NT>(u, col, j);
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int n1 = j + (r << LGNBL);
            const int64_t n = (int64_t)n1 * N2 + colv(col);
            if (n < D.M) out[n] = cscale(cmul(v[u * RL + r], chirp<T>(n, D.M, D.invM, sign, ph)), sc);
        }
    }
}

// ---- one-block Bluestein ---------------------------------------------------------------------------
template <typename T, int LGN, bool SRC_SAMPLES, bool TO_SAMPLES>
__global__ __launch_bounds__(kThreads) void k_small(TxArgs a, const int* __restrict__ lat,
                                                    const cx<T>* __restrict__ src, int64_t src_stride, cx<T>* work,
                                                    const cx<T>* __restrict__ filt, cx<T>* dst, int64_t dst_stride,
                                                    int sign, int scale_by_invM, int mask_bins,
                                                    const cx<T>* __restrict__ tw) {
    constexpr int N = 1 << LGN;
    __shared__ cx<T> lds[Padded<N>::v];
    __shared__ cx<T> ph[PhaseTab<T>::n];
    phase_fill<T>(ph);
    __syncthreads();
    const LatDesc D = a.desc[lat[blockIdx.x]];
    const int64_t rhs = blockIdx.y;
    const cx<T>* in = src + rhs * src_stride + (SRC_SAMPLES ? D.samp_off : D.work_off);
    for (int n = threadIdx.x; n < N; n += kThreads) {
        cx<T> v = {(T)0, (T)0};
        if (n < D.M) v = cmul(in[n], chirp<T>(n, D.M, D.invM, sign, ph));
        if (!SRC_SAMPLES && mask_bins && n < D.M && !owned_bin(a.bitmaps, D, n)) v = {(T)0, (T)0};
        lds[pidx(n)] = v;
    }
    __syncthreads();
    fft_ct<T, LGN, 1, N, -1>(lds, tw);
    const cx<T>* f = filt + D.filt_off;
    for (int n = threadIdx.x; n < N; n += kThreads)
        lds[pidx(n)] = sign < 0 ? cmul(lds[pidx(n)], f[n]) : cmulc(lds[pidx(n)], f[n]);
    __syncthreads();
    fft_ct<T, LGN, 1, N, +1>(lds, tw);
    cx<T>* out = TO_SAMPLES ? dst + rhs * dst_stride + D.samp_off : work + rhs * a.work_stride + D.work_off;
    const T sc = scale_by_invM ? (T)D.invM : (T)1;
    for (int n = threadIdx.x; n < D.M; n += kThreads)
        out[n] = cscale(cmul(lds[pidx(n)], chirp<T>(n, D.M, D.invM, sign, ph)), sc);
}

// plain in-place forward DFT of a whole region (filter construction on the one-block path)
template <int LGN>
__global__ __launch_bounds__(kThreads) void k_small_dft(TxArgs a, const int* __restrict__ lat, cx<double>* work,
                                                        const cx<double>* __restrict__ tw) {
    constexpr int N = 1 << LGN;
    __shared__ cx<double> lds[Padded<N>::v];
    const LatDesc D = a.desc[lat[blockIdx.x]];
    cx<double>* w = work + D.work_off;
    for (int n = threadIdx.x; n < N; n += kThreads) lds[pidx(n)] = w[n];
    __syncthreads();
    fft_ct<double, LGN, 1, N, -1>(lds, tw);
    for (int n = threadIdx.x; n < N; n += kThreads) w[n] = lds[pidx(n)];
}

// b_l[n] = e^{+i pi n^2/M} for 0 <= n < M and at N - n for 0 < n < M, zero elsewhere (double);
// N = bl_len, a power of two or 3 * 2^lgN
__global__ void k_filter_fill(const LatDesc* __restrict__ desc, int L, cx<double>* tmp) {
    const int l = blockIdx.y;
    const LatDesc D = desc[l];
    const int64_t N = bl_len(D);
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        int64_t m = -1;
        if (n < D.M) m = n;
        else if (N - n < D.M) m = N - n;
        cx<double> v = {0.0, 0.0};
        if (m >= 0) v = cispi<double>(sq_mod_2M(m, D.M, 0.5 * D.invM) * D.invM);
        tmp[D.work_off + n] = v;
    }
}

template <typename T>
__global__ void k_filter_store(const LatDesc* __restrict__ desc, const cx<double>* __restrict__ tmp, cx<T>* filt) {
    const int l = blockIdx.y;
    const LatDesc D = desc[l];
    const int64_t N = bl_len(D);
    const double sc = 1.0 / (double)N;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const cx<double> v = tmp[D.work_off + n];
        filt[D.filt_off + n] = make_cx<T>((T)(v.x * sc), (T)(v.y * sc));
    }
}

// ---- dispatch over compile-time sizes --------------------------------------------------------------
template <int LO, int HI, typename F>
__device__ __forceinline__ void with_lg_dev(int lg, F&& f) {
    if constexpr (LO <= HI) {
        if (lg == LO) f(std::integral_constant<int, LO>{});
        else with_lg_dev<LO + 1, HI>(lg, f);
    }
}

// f(std::integral_constant<int, lg>) for lg in [LO, HI]
template <int LO, int HI, typename F>
static void with_lg(int lg, F&& f) {
    if constexpr (LO <= HI) {
        if (lg == LO) f(std::integral_constant<int, LO>{});
        else with_lg<LO + 1, HI>(lg, f);
    }
}

// four-step kernels for (2^lgN, split lg1): f(LG, LG1) with both as integral constants; lg1 must
// be a compiled split (split_compiled), which plans guarantee
template <typename F>
static void with_split(int lgN, int lg1, F&& f) {
    with_lg<kSmallMaxLg + 1, kMaxLgN>(lgN, [&](auto LG) {
        constexpr int lg = decltype(LG)::value;
        constexpr int r = split_lgN1(lg);
        if (lg1 == r) f(LG, std::integral_constant<int, r>{});
        if constexpr (split_compiled(lg, r - 1))
            if (lg1 == r - 1) f(LG, std::integral_constant<int, r - 1>{});
        if constexpr (split_compiled(lg, r + 1))
            if (lg1 == r + 1) f(LG, std::integral_constant<int, r + 1>{});
    });
}

// kernels for N = 3 * 2^lgN: f(LG, LG1) with the one compiled split
template <typename F>
static void with_len3(int lgN, F&& f) {
    with_lg<kMinLg3, kMaxLg3>(lgN, [&](auto LG) {
        constexpr int lg = decltype(LG)::value;
        f(LG, std::integral_constant<int, split3_lgN1(lg)>{});
    });
}

template <typename T>
void launch_bluestein_small(const TxArgs& a, const FftGroup& g, const cx<T>* src, int64_t src_stride,
                            bool src_is_samples, cx<T>* work, const cx<T>* filt, cx<T>* dst, int64_t dst_stride,
                            bool dst_is_samples, int sign, bool scale_by_invM, bool mask_bins, hipStream_t s) {
    if (g.nlat == 0 || a.n_rhs == 0) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const cx<T>* tw = twiddles<T>(dev);
    const dim3 grid(g.nlat, (unsigned)a.n_rhs);
    with_lg<0, kSmallMaxLg>(g.lgN, [&](auto LG) {
        constexpr int lg = decltype(LG)::value;
        if (src_is_samples && !dst_is_samples)
            hipLaunchKernelGGL((k_small<T, lg, true, false>), grid, dim3(kThreads), 0, s, a, g.lat, src, src_stride,
                               work, filt, dst, dst_stride, sign, (int)scale_by_invM, 0, tw);
        else
            hipLaunchKernelGGL((k_small<T, lg, false, true>), grid, dim3(kThreads), 0, s, a, g.lat, src, src_stride,
                               work, filt, dst, dst_stride, sign, (int)scale_by_invM, (int)mask_bins, tw);
    });
}

template <typename T>
void launch_p1(const TxArgs& a, const FftGroup& g, const cx<T>* src, int64_t src_stride, bool src_is_samples,
               cx<T>* work, int sign, bool mask_bins, hipStream_t s) {
    const int rb = (int)(((uintptr_t)src / sizeof(cx<T>)) & 1023);
    if (g.nlat == 0 || a.n_rhs == 0) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const cx<T>* tw = twiddles<T>(dev);
    auto go = [&](auto LG, auto LG1c, auto F3c) {
        constexpr int lg = decltype(LG)::value, l1 = decltype(LG1c)::value, f3 = decltype(F3c)::value;
        using CT = ColTile<T, lg, l1>;
        const dim3 grid((unsigned)((g.nlat * f3) << (lg - CT::TLG)), (unsigned)a.n_rhs), block(CT::NT);
        if (src_is_samples)
            hipLaunchKernelGGL((k_p1<T, lg, l1, 0, f3>), grid, block, 0, s, a, g.lat, src, src_stride, work, sign, tw,
                               rb);
        else if (mask_bins)
            hipLaunchKernelGGL((k_p1<T, lg, l1, 3, f3>), grid, block, 0, s, a, g.lat, src, src_stride, work, sign, tw,
                               0);
        else
            hipLaunchKernelGGL((k_p1<T, lg, l1, 1, f3>), grid, block, 0, s, a, g.lat, src, src_stride, work, sign, tw,
                               0);
    };
    if (g.n3)
        with_len3(g.lgN, [&](auto LG, auto LG1c) { go(LG, LG1c, std::integral_constant<int, 3>{}); });
    else
        with_split(g.lgN, g.lg1, [&](auto LG, auto LG1c) { go(LG, LG1c, std::integral_constant<int, 1>{}); });
}

template <typename T>
void launch_p2(const TxArgs& a, const FftGroup& g, cx<T>* work, const cx<T>* filt, int sign, const cx<T>* rot_in,
               const cx<T>* rot_out, hipStream_t s) {
    const int ri = rot_in ? (int)(((uintptr_t)rot_in / sizeof(cx<T>)) & 1023) : -1;
    const int ro = rot_out ? (int)(((uintptr_t)rot_out / sizeof(cx<T>)) & 1023) : -1;
    if (g.nlat == 0 || a.n_rhs == 0) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const cx<T>* tw = twiddles<T>(dev);
    if (g.n3) {
        with_len3(g.lgN, [&](auto LG, auto LG1c) {
            constexpr int lg = decltype(LG)::value, l1 = decltype(LG1c)::value;
            using RT = RowTile3<lg, l1>;
            const dim3 grid((unsigned)(g.nlat << (lg - RT::TLG3)), (unsigned)a.n_rhs);
            hipLaunchKernelGGL((k_p2r3<T, lg, l1, true>), grid, dim3(RT::NT), 0, s, a, g.lat, work, filt, sign, tw,
                               ri, ro);
        });
        return;
    }
    with_split(g.lgN, g.lg1, [&](auto LG, auto LG1c) {
        constexpr int lg = decltype(LG)::value, l1 = decltype(LG1c)::value;
        auto go = [&](auto Vc) {
            constexpr int V = decltype(Vc)::value;
            if constexpr (p2_variant_compiled(lg, l1, V)) {
                using RT = RowTile<lg, l1, (V >> 1) & 1, (V & 4) ? 3 : 4>;
                const dim3 grid((unsigned)(g.nlat << (lg - RT::TLG)), (unsigned)a.n_rhs);
                hipLaunchKernelGGL((k_p2<T, lg, l1, true, V>), grid, dim3(RT::NT), 0, s, a, g.lat, work, filt, sign,
                                   tw, ri, ro);
            }
        };
        switch (p2_variant_compiled(lg, l1, g.p2v) ? g.p2v : 0) {
            case 1: go(std::integral_constant<int, 1>{}); break;
            case 2: go(std::integral_constant<int, 2>{}); break;
            case 3: go(std::integral_constant<int, 3>{}); break;
            case 4: go(std::integral_constant<int, 4>{}); break;
            case 6: go(std::integral_constant<int, 6>{}); break;
            default: go(std::integral_constant<int, 0>{}); break;
        }
    });
}

template <typename T>
void launch_p3(const TxArgs& a, const FftGroup& g, cx<T>* work, cx<T>* dst, int64_t dst_stride, bool dst_is_samples,
               int sign, bool scale_by_invM, hipStream_t s) {
    const int rb = dst_is_samples ? (int)(((uintptr_t)dst / sizeof(cx<T>)) & 1023) : 0;
    if (g.nlat == 0 || a.n_rhs == 0) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const cx<T>* tw = twiddles<T>(dev);
    auto go = [&](auto LG, auto LG1c, auto F3c) {
        constexpr int lg = decltype(LG)::value, l1 = decltype(LG1c)::value, f3 = decltype(F3c)::value;
        using CT = ColTile<T, lg, l1>;
        const dim3 grid((unsigned)((g.nlat * f3) << (lg - CT::TLG)), (unsigned)a.n_rhs), block(CT::NT);
        if (dst_is_samples)
            hipLaunchKernelGGL((k_p3<T, lg, l1, true, f3>), grid, block, 0, s, a, g.lat, work, dst, dst_stride, sign,
                               (int)scale_by_invM, tw, rb);
        else
            hipLaunchKernelGGL((k_p3<T, lg, l1, false, f3>), grid, block, 0, s, a, g.lat, work, dst, dst_stride,
                               sign, (int)scale_by_invM, tw, 0);
    };
    if (g.n3)
        with_len3(g.lgN, [&](auto LG, auto LG1c) { go(LG, LG1c, std::integral_constant<int, 3>{}); });
    else
        with_split(g.lgN, g.lg1, [&](auto LG, auto LG1c) { go(LG, LG1c, std::integral_constant<int, 1>{}); });
}

#define MR1L_INST_FFT(T)                                                                                           \
    template void launch_bluestein_small<T>(const TxArgs&, const FftGroup&, const cx<T>*, int64_t, bool, cx<T>*,   \
                                            const cx<T>*, cx<T>*, int64_t, bool, int, bool, bool, hipStream_t);  \
    template void launch_p1<T>(const TxArgs&, const FftGroup&, const cx<T>*, int64_t, bool, cx<T>*, int, bool,    \
                               hipStream_t);                                                                      \
    template void launch_p2<T>(const TxArgs&, const FftGroup&, cx<T>*, const cx<T>*, int, const cx<T>*,          \
                               const cx<T>*, hipStream_t);           \
    template void launch_p3<T>(const TxArgs&, const FftGroup&, cx<T>*, cx<T>*, int64_t, bool, int, bool,          \
                               hipStream_t);
MR1L_INST_FFT(float)
MR1L_INST_FFT(double)

// ---- persistent small-transform kernel (batched plans) ---------------------------------------------
// LDS of one workgroup: the Bluestein buffer (one-block path, up to 2^kSmallMaxLg points), the
// single-precision phase table, per frequency its residue in the current lattice, its running sum
// and its counter, and the alias bitmaps of the current lattice (at most 2^(kSmallMaxLg-1) bins).
template <typename T>
struct FusedLds {
    static constexpr int kBuf = Padded<(1 << kSmallMaxLg)>::v;
    static constexpr int kWords = (1 << (kSmallMaxLg - 1)) / 32;
    cx<T> buf[kBuf];
    cx<T> ph[PhaseTab<T>::n];
    cx<T> acc[kFusedTxMaxN];
    int32_t res[kFusedTxMaxN];
    uint8_t cnt[kFusedTxMaxN];
    uint32_t seen[kWords], multi[kWords];
    int next;
};

// residues of the transform's frequencies in lattice D into L.res and the lattice's 2-bit alias
// counts into L.seen / L.multi (same integers as the index pass); ends with a barrier
template <typename T, typename K>
__device__ void fused_alias(const TxArgs& a, const TxDesc& t, const LatDesc& D, FusedLds<T>& L) {
    const int words = (int)D.bm_words;
    for (int w = threadIdx.x; w < words; w += kThreads) {
        L.seen[w] = 0u;
        L.multi[w] = 0u;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < (int)t.fn; k += kThreads) {
        const int r = (int)residue<K>(a, D, t.foff + k);
        L.res[k] = r;
        const uint32_t old = atomicOr(&L.seen[r >> 5], 1u << (r & 31));
        if ((old >> (r & 31)) & 1u) atomicOr(&L.multi[r >> 5], 1u << (r & 31));
    }
    __syncthreads();
}

// the one-block Bluestein of k_small on L.buf, which holds the chirped, zero-padded input:
// forward DFT, filter, inverse DFT; ends with a barrier
template <typename T, int LGN>
__device__ void fused_conv(cx<T>* buf, const cx<T>* __restrict__ f, int sign, const cx<T>* __restrict__ tw) {
    constexpr int N = 1 << LGN;
    fft_ct<T, LGN, 1, N, -1>(buf, tw);
    for (int n = threadIdx.x; n < N; n += kThreads)
        buf[pidx(n)] = sign < 0 ? cmul(buf[pidx(n)], f[n]) : cmulc(buf[pidx(n)], f[n]);
    __syncthreads();
    fft_ct<T, LGN, 1, N, +1>(buf, tw);
}

template <typename T>
__device__ void fused_conv_any(int lgN, cx<T>* buf, const cx<T>* __restrict__ f, int sign,
                               const cx<T>* __restrict__ tw) {
    with_lg_dev<0, kSmallMaxLg>(lgN, [&](auto LG) { fused_conv<T, decltype(LG)::value>(buf, f, sign, tw); });
}

// FORWARD: c_k = (1/counter_k) sum over ascending l with k in I_l of DFT(y_l)[r_l(k)] / M_l.
// Adjoint: y_l = (1/M_l) IDFT(bins_l), bins_l[r_l(k)] = c_k / counter_k for k in I_l.  Every
// floating-point operation is the one the stage sweep does for the same transform (k_small, then
// the gather's ascending sum and division, or the scatter's division, then k_small), so the two
// paths give the same bits.
template <typename T, typename K, bool FORWARD>
__global__ __launch_bounds__(kThreads) void k_fused_small(TxArgs a, const int* __restrict__ list, int nlist,
                                                         int* queue, const cx<T>* __restrict__ src, cx<T>* dst,
                                                         const cx<T>* __restrict__ filt,
                                                         const cx<T>* __restrict__ tw) {
    extern __shared__ __align__(16) char fused_raw[];
    FusedLds<T>& L = *reinterpret_cast<FusedLds<T>*>(fused_raw);
    phase_fill<T>(L.ph);
    for (;;) {
        if (threadIdx.x == 0) L.next = atomicAdd(&queue[0], 1);
        __syncthreads();
        const int b = L.next;
        __syncthreads();
        if (b >= nlist) break;
        const TxDesc t = a.tx[list[b]];
        const int fn = (int)t.fn;
        for (int k = threadIdx.x; k < fn; k += kThreads) {
            L.acc[k] = {(T)0, (T)0};
            L.cnt[k] = 0;
        }
        if (!FORWARD) {
            // counter_k over every lattice first
            for (int j = 0; j < t.nlat; ++j) {
                const LatDesc D = a.desc[t.lat0 + j];
                fused_alias<T, K>(a, t, D, L);
                for (int k = threadIdx.x; k < fn; k += kThreads) {
                    const int r = L.res[k];
                    if (!((L.multi[r >> 5] >> (r & 31)) & 1u)) ++L.cnt[k];
                }
                __syncthreads();
            }
        }
        for (int j = 0; j < t.nlat; ++j) {
            const LatDesc D = a.desc[t.lat0 + j];
            const int N = 1 << D.lgN;
            fused_alias<T, K>(a, t, D, L);
            if (FORWARD) {
                const cx<T>* in = src + D.samp_off;
                for (int n = threadIdx.x; n < N; n += kThreads) {
                    cx<T> v = {(T)0, (T)0};
                    if (n < D.M) v = cmul(in[n], chirp<T>(n, D.M, D.invM, -1, L.ph));
                    L.buf[pidx(n)] = v;
                }
            } else {
                for (int n = threadIdx.x; n < N; n += kThreads) L.buf[pidx(n)] = {(T)0, (T)0};
                __syncthreads();
                // bins of the frequencies in I_l: c_k / counter_k
                for (int k = threadIdx.x; k < fn; k += kThreads) {
                    const int r = L.res[k];
                    if (!((L.multi[r >> 5] >> (r & 31)) & 1u)) {
                        const cx<T> c = src[t.foff + k];
                        L.buf[pidx(r)] = {c.x / (T)L.cnt[k], c.y / (T)L.cnt[k]};
                    }
                }
                __syncthreads();
                for (int n = threadIdx.x; n < D.M; n += kThreads) {
                    const bool own = ((L.seen[n >> 5] & ~L.multi[n >> 5]) >> (n & 31)) & 1u;
                    L.buf[pidx(n)] = own ? cmul(L.buf[pidx(n)], chirp<T>(n, D.M, D.invM, +1, L.ph)) : cx<T>{(T)0, (T)0};
                }
            }
            __syncthreads();
            fused_conv_any<T>(D.lgN, L.buf, filt + D.filt_off, FORWARD ? -1 : +1, tw);
            if (FORWARD) {
                // DFT bins (chirp, 1/M) in place, then the ascending-l sum of the frequencies in I_l
                for (int n = threadIdx.x; n < D.M; n += kThreads)
                    L.buf[pidx(n)] = cscale(cmul(L.buf[pidx(n)], chirp<T>(n, D.M, D.invM, -1, L.ph)), (T)D.invM);
                __syncthreads();
                for (int k = threadIdx.x; k < fn; k += kThreads) {
                    const int r = L.res[k];
                    if (!((L.multi[r >> 5] >> (r & 31)) & 1u)) {
                        L.acc[k] = L.acc[k] + L.buf[pidx(r)];
                        ++L.cnt[k];
                    }
                }
            } else {
                cx<T>* out = dst + D.samp_off;
                for (int n = threadIdx.x; n < D.M; n += kThreads)
                    out[n] = cscale(cmul(L.buf[pidx(n)], chirp<T>(n, D.M, D.invM, +1, L.ph)), (T)D.invM);
            }
            __syncthreads();
        }
        if (FORWARD)
            for (int k = threadIdx.x; k < fn; k += kThreads) {
                const int c = L.cnt[k];
                dst[t.foff + k] = c ? cx<T>{L.acc[k].x / (T)c, L.acc[k].y / (T)c} : cx<T>{(T)0, (T)0};
            }
        __syncthreads();
    }
    // the last workgroup out empties the queue for the next launch: every workgroup's last fetch
    // returned before it counted itself done
    if (threadIdx.x == 0 && atomicAdd(&queue[1], 1) == (int)gridDim.x - 1) {
        atomicExch(&queue[0], 0);
        atomicExch(&queue[1], 0);
    }
}

template <typename T>
void launch_fused_small(const TxArgs& a, const int* list, int nlist, int* queue, const cx<T>* src, cx<T>* dst,
                        const cx<T>* filt, bool forward, hipStream_t s) {
    if (nlist == 0) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const cx<T>* tw = twiddles<T>(dev);
    const size_t lds = sizeof(FusedLds<T>);
    const int per_cu = std::max(1, (int)((160u * 1024u) / lds));
    const dim3 grid((unsigned)std::min(nlist, 256 * per_cu));
    auto go = [&](auto Kc) {
        using K = decltype(Kc);
        if (forward)
            hipLaunchKernelGGL((k_fused_small<T, K, true>), grid, dim3(kThreads), lds, s, a, list, nlist, queue, src,
                               dst, filt, tw);
        else
            hipLaunchKernelGGL((k_fused_small<T, K, false>), grid, dim3(kThreads), lds, s, a, list, nlist, queue, src,
                               dst, filt, tw);
    };
    switch (a.fv.ktype) {
        case K_I8: go(int8_t{}); break;
        case K_I16: go(int16_t{}); break;
        default: go(int32_t{}); break;
    }
}
template void launch_fused_small<float>(const TxArgs&, const int*, int, int*, const cx<float>*, cx<float>*,
                                        const cx<float>*, bool, hipStream_t);
template void launch_fused_small<double>(const TxArgs&, const int*, int, int*, const cx<double>*, cx<double>*,
                                         const cx<double>*, bool, hipStream_t);

// Filter spectra for every lattice of a plan (synchronous on s).  The double-precision DFT of
// b_l reuses the stage-1/stage-2 kernels (or the one-block DFT) on a temporary buffer laid out
// like the work area; the four-step split is the one the plan's own stage 2 reads.
template <typename T>
hipError_t build_filters(const LatDesc* hdesc, int L, const LatDesc* ddesc, const std::vector<FftGroup>& groups,
                         cx<T>* filt, int device, hipStream_t s) {
    if (L == 0) return hipSuccess;
    int64_t tot = 0;
    int maxlg = 0;
    for (int l = 0; l < L; ++l) {
        tot = std::max<int64_t>(tot, hdesc[l].work_off + bl_len(hdesc[l]));
        maxlg = std::max(maxlg, hdesc[l].lgN);
    }
    DevMem tmpm;
    hipError_t e = tmpm.alloc((size_t)tot * sizeof(cx<double>));
    if (e != hipSuccess) return e;
    cx<double>* tmp = tmpm.as<cx<double>>();
    TxArgs a{};
    a.desc = ddesc;
    a.L = L;
    a.n_rhs = 1;
    a.work_stride = 0;
    const cx<double>* tw = twiddles<double>(device);
    const int blocks = std::max(1, std::min(1024, (int)(((int64_t)1 << maxlg) / 256)));
    hipLaunchKernelGGL(k_filter_fill, dim3(blocks, L), dim3(256), 0, s, ddesc, L, tmp);
    for (const FftGroup& g : groups) {
        if (g.small) {
            with_lg<0, kSmallMaxLg>(g.lgN, [&](auto LG) {
                hipLaunchKernelGGL((k_small_dft<decltype(LG)::value>), dim3(g.nlat), dim3(kThreads), 0, s, a, g.lat,
                                   tmp, tw);
            });
        } else if (g.n3) {
            with_len3(g.lgN, [&](auto LG, auto LG1c) {
                constexpr int lg = decltype(LG)::value, l1 = decltype(LG1c)::value;
                using CT = ColTile<double, lg, l1>;
                using RT = RowTile3<lg, l1>;
                const dim3 grid1((unsigned)((g.nlat * 3) << (lg - CT::TLG)), 1);
                const dim3 grid((unsigned)(g.nlat << (lg - RT::TLG3)), 1);
                hipLaunchKernelGGL((k_p1<double, lg, l1, 2, 3>), grid1, dim3(CT::NT), 0, s, a, g.lat,
                                   (const cx<double>*)tmp, (int64_t)0, tmp, -1, tw, 0);
                hipLaunchKernelGGL((k_p2r3<double, lg, l1, false>), grid, dim3(RT::NT), 0, s, a, g.lat, tmp,
                                   (const cx<double>*)nullptr, -1, tw, -1, -1);
            });
        } else {
            with_split(g.lgN, g.lg1, [&](auto LG, auto LG1c) {
                constexpr int lg = decltype(LG)::value, l1 = decltype(LG1c)::value;
                using CT = ColTile<double, lg, l1>;
                using RT = RowTile<lg, l1>;
                const dim3 grid1((unsigned)(g.nlat << (lg - CT::TLG)), 1);
                const dim3 grid((unsigned)(g.nlat << (lg - RT::TLG)), 1);
                hipLaunchKernelGGL((k_p1<double, lg, l1, 2>), grid1, dim3(CT::NT), 0, s, a, g.lat,
                                   (const cx<double>*)tmp, (int64_t)0, tmp, -1, tw, 0);
                hipLaunchKernelGGL((k_p2<double, lg, l1, false>), grid, dim3(RT::NT), 0, s, a, g.lat, tmp,
                                   (const cx<double>*)nullptr, -1, tw, -1, -1);
            });
        }
    }
    hipLaunchKernelGGL((k_filter_store<T>), dim3(blocks, L), dim3(256), 0, s, ddesc, (const cx<double>*)tmp, filt);
    return hipStreamSynchronize(s);
}
template hipError_t build_filters<float>(const LatDesc*, int, const LatDesc*, const std::vector<FftGroup>&, cx<float>*, int,
                                   hipStream_t);
template hipError_t build_filters<double>(const LatDesc*, int, const LatDesc*, const std::vector<FftGroup>&, cx<double>*,
                                    int, hipStream_t);

}  // namespace mr1l
