// Built-in test function of Sec. 5.3: weighted sums of tensor products of periodic B-splines
// N_m(x) = C_m sum_k sinc(pi k/m)^m (-1)^k e^{2 pi i k x}, ||N_m||_{L2(T)} = 1.
//
// Point values use N_m(x) = C_m m B_m(m (x mod 1)), B_m the cardinal B-spline of order m on
// [0, m] (the series above is the 1-periodisation of B_m(m .) scaled by C_m m).  B_m(u) on the
// unit interval [i, i+1) holding u comes from the Cox-de Boor recursion in the local coordinate
// v = u - i: every step is a convex combination, so no cancellation occurs.
//
// The sampler runs on the device, one thread per node; the Fourier coefficients, the norm and the
// relative L2 error of Sec. 5.3 are host computations on the parameters alone.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "common.h"
#include "runtime.h"

namespace mr1l {
namespace {

constexpr int kBsMaxD = SFFT_MAX_D;

struct BsArgs {
    int T, d;
    double scale[SFFT_BSPLINE_MAX_ORDER + 1];   // C_m m
    double w[SFFT_BSPLINE_MAX_TERMS];
    int8_t m[SFFT_BSPLINE_MAX_TERMS][kBsMaxD];
};

// B_m at u = i + v, 0 <= i < m, 0 <= v < 1.  After the step to order k + 1 the array holds the
// k + 1 basis functions of that order that are nonzero on [i, i+1), the last one starting at i:
// entry q becomes ((k - q + v) entry[q-1] + (q + 1 - v) entry[q]) / k.  B_m is entry m - 1 - i.
template <int M>
__device__ inline double cardinal(int i, double v) {
    double b[M];
    b[0] = 1.0;
#pragma unroll
    for (int k = 1; k < M; ++k) {
        const double inv = 1.0 / k;
        double prev = 0.0;
#pragma unroll
        for (int q = 0; q <= k; ++q) {
            const double cur = q < k ? b[q] : 0.0;
            b[q] = ((k - q + v) * prev + (q + 1 - v) * cur) * inv;
            prev = cur;
        }
    }
    double out = 0.0;
#pragma unroll
    for (int q = 0; q < M; ++q)
        if (q == M - 1 - i) out = b[q];
    return out;
}

// B_m(m x) for x in [0, 1)
__device__ __forceinline__ double bspline_at(int m, double x) {
    const double u = m * (x - floor(x));
    int i = (int)u;
    i = i < 0 ? 0 : (i >= m ? m - 1 : i);
    const double v = u - i;
    switch (m) {
        case 1: return cardinal<1>(i, v);
        case 2: return cardinal<2>(i, v);
        case 3: return cardinal<3>(i, v);
        case 4: return cardinal<4>(i, v);
        case 5: return cardinal<5>(i, v);
        case 6: return cardinal<6>(i, v);
        case 7: return cardinal<7>(i, v);
        case 8: return cardinal<8>(i, v);
        case 9: return cardinal<9>(i, v);
        case 10: return cardinal<10>(i, v);
        case 11: return cardinal<11>(i, v);
        case 12: return cardinal<12>(i, v);
        default: return 0.0;
    }
}

// one thread per node; the node's coordinates are re-read per product (cache hits)
template <typename T>
__global__ __launch_bounds__(256) void k_bspline(BsArgs a, int64_t n, const double* __restrict__ nodes,
                                                 cx<T>* __restrict__ out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double* x = nodes + j * a.d;
    double v = 0.0;
    for (int t = 0; t < a.T; ++t) {
        double p = a.w[t];
        for (int c = 0; c < a.d; ++c) {
            const int m = a.m[t][c];
            if (m > 0) p *= a.scale[m] * bspline_at(m, x[c]);
        }
        v += p;
    }
    out[j] = cx<T>{(T)v, (T)0};
}

// Host: B_M(u) at integer u = i (v = 0) by the same recursion
double cardinal_host(int M, int i) {
    std::vector<double> b(M, 0.0);
    b[0] = 1.0;
    for (int k = 1; k < M; ++k) {
        double prev = 0.0;
        for (int q = 0; q <= k; ++q) {
            const double cur = q < k ? b[q] : 0.0;
            b[q] = ((k - q) * prev + (q + 1) * cur) / k;
            prev = cur;
        }
    }
    return b[M - 1 - i];
}

// C_m from ||N_m|| = 1: C_m^-2 = sum_k sinc(pi k/m)^(2m) = m B_2m(m) (Poisson summation of the
// autocorrelation of B_m, which is B_2m)
double norm_const(int m) { return 1.0 / std::sqrt(m * cardinal_host(2 * m, m)); }

// N^_m(k) = C_m sinc(pi k/m)^m (-1)^k
double n_hat(int m, int64_t k) {
    const double cm = norm_const(m);
    if (k == 0) return cm;
    if (k % m == 0) return 0.0;
    const int64_t kr = ((k % (2 * m)) + 2 * m) % (2 * m);        // sin(pi k/m) has period 2m in k
    const double s = std::sin(M_PI * (double)kr / m) / (M_PI * (double)k / m);
    return cm * std::pow(s, m) * ((k & 1) ? -1.0 : 1.0);
}

// <N_m1, N_m2> on T (0 stands for the constant 1)
double inner(int m1, int m2) {
    if (m1 == 0 && m2 == 0) return 1.0;
    if (m1 == 0 || m2 == 0) return norm_const(m1 ? m1 : m2);
    if (m1 == m2) return 1.0;
    double s = 0.0;
    for (int64_t k = 100000; k >= 1; --k) s += n_hat(m1, k) * n_hat(m2, k);
    return n_hat(m1, 0) * n_hat(m2, 0) + 2.0 * s;
}

mr1l_status check_desc(const sfft_bspline* f, int d) {
    if (!f || f->terms < 1 || f->terms > SFFT_BSPLINE_MAX_TERMS || f->d < 1 || f->d > kBsMaxD || !f->orders ||
        (d >= 0 && d != f->d) || (f->dtype != MR1L_C64 && f->dtype != MR1L_C128)) {
        set_error("invalid sfft_bspline description");
        return MR1L_ERR_ARG;
    }
    for (int i = 0; i < f->terms * f->d; ++i)
        if (f->orders[i] < 0 || f->orders[i] > SFFT_BSPLINE_MAX_ORDER) {
            set_error("B-spline orders must lie in 0.." + std::to_string(SFFT_BSPLINE_MAX_ORDER));
            return MR1L_ERR_ARG;
        }
    return MR1L_OK;
}

double weight(const sfft_bspline* f, int t) { return f->weights ? f->weights[t] : 1.0; }

}  // namespace
}  // namespace mr1l

using namespace mr1l;

extern "C" int sfft_sample_bspline(void* user, int d, int64_t n_nodes, const double* nodes_dev, void* values_dev,
                                   void* stream) {
    try {
        const sfft_bspline* f = (const sfft_bspline*)user;
        if (check_desc(f, d) != MR1L_OK) return 1;
        if (n_nodes < 0 || (n_nodes > 0 && (!nodes_dev || !values_dev))) {
            set_error("invalid nodes or values for the B-spline sampler");
            return 1;
        }
        if (n_nodes == 0) return 0;
        BsArgs a{};
        a.T = f->terms;
        a.d = f->d;
        for (int m = 1; m <= SFFT_BSPLINE_MAX_ORDER; ++m) a.scale[m] = norm_const(m) * m;
        for (int t = 0; t < a.T; ++t) {
            a.w[t] = weight(f, t);
            for (int c = 0; c < a.d; ++c) a.m[t][c] = (int8_t)f->orders[t * a.d + c];
        }
        const int64_t blocks = (n_nodes + 255) / 256;
        if (blocks > 0x7fffffffLL) {
            set_error("too many nodes for one sampler call");
            return 1;
        }
        hipStream_t st = (hipStream_t)stream;
        if (f->dtype == MR1L_C128)
            hipLaunchKernelGGL(k_bspline<double>, dim3((unsigned)blocks), dim3(256), 0, st, a, n_nodes, nodes_dev,
                               (cx<double>*)values_dev);
        else
            hipLaunchKernelGGL(k_bspline<float>, dim3((unsigned)blocks), dim3(256), 0, st, a, n_nodes, nodes_dev,
                               (cx<float>*)values_dev);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error(std::string("B-spline sampler launch: ") + hipGetErrorString(e));
            return 1;
        }
        return 0;
    } catch (const std::exception& e) {
        set_error(e.what());
        return 1;
    }
}

extern "C" mr1l_status sfft_bspline_coeffs(const sfft_bspline* f, int64_t n, const int32_t* freqs, double* coeffs) {
    try {
        clear_error();
        if (check_desc(f, -1) != MR1L_OK) return MR1L_ERR_ARG;
        if (n < 0 || (n > 0 && (!freqs || !coeffs))) {
            set_error("invalid arguments to sfft_bspline_coeffs");
            return MR1L_ERR_ARG;
        }
        const int d = f->d;
        for (int64_t i = 0; i < n; ++i) {
            double v = 0.0;
            for (int t = 0; t < f->terms; ++t) {
                double p = weight(f, t);
                for (int c = 0; c < d && p != 0.0; ++c) {
                    const int m = f->orders[t * d + c];
                    const int64_t k = freqs[i * d + c];
                    p *= m > 0 ? n_hat(m, k) : (k == 0 ? 1.0 : 0.0);
                }
                v += p;
            }
            coeffs[2 * i] = v;
            coeffs[2 * i + 1] = 0.0;
        }
        return MR1L_OK;
    } catch (const std::exception& e) {
        set_error(e.what());
        return MR1L_ERR_ARG;
    }
}

extern "C" mr1l_status sfft_bspline_l2_error(const sfft_bspline* f, int64_t n, const int32_t* freqs,
                                             const double* coeffs, double* rel_err, double* norm2) {
    try {
        clear_error();
        if (check_desc(f, -1) != MR1L_OK) return MR1L_ERR_ARG;
        if (n < 0 || (n > 0 && (!freqs || !coeffs)) || !rel_err) {
            set_error("invalid arguments to sfft_bspline_l2_error");
            return MR1L_ERR_ARG;
        }
        const int d = f->d;
        double nf2 = 0.0;
        for (int a = 0; a < f->terms; ++a)
            for (int b = 0; b < f->terms; ++b) {
                double p = weight(f, a) * weight(f, b);
                for (int c = 0; c < d; ++c) p *= inner(f->orders[a * d + c], f->orders[b * d + c]);
                nf2 += p;
            }
        std::vector<double> fh((size_t)std::max<int64_t>(1, n) * 2);
        const mr1l_status rc = sfft_bspline_coeffs(f, n, freqs, fh.data());
        if (rc != MR1L_OK) return rc;
        double kept = 0.0, err = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double re = coeffs[2 * i] - fh[2 * i], im = coeffs[2 * i + 1];
            kept += fh[2 * i] * fh[2 * i];
            err += re * re + im * im;
        }
        const double e2 = nf2 - kept + err;
        *rel_err = std::sqrt((e2 > 0.0 ? e2 : 0.0) / nf2);
        if (norm2) *norm2 = nf2;
        return MR1L_OK;
    } catch (const std::exception& e) {
        set_error(e.what());
        return MR1L_ERR_ARG;
    }
}
