// Weighted least-squares residual on the stacked lattices of a plan: the sample-domain loss of a
// fit y ~ A c through the Fourier matrix A of Sec. 2.1,
//     loss = 1/2 sum_rhs sum_l (1/M_l) sum_j |s_l[j] - y_l[j]|^2,
// and its gradient with respect to s, (1/M_l)(s_l[j] - y_l[j]), in one pass over s and y.  The
// loss is summed in double in a fixed order (block tree sums, then one ordered pass over the block
// partials), so it is deterministic.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "common.h"
#include "runtime.h"

// Block partials of the allocation-free variant (mr1l_lsq_residual_noalloc): one array per GPU for
// the life of the process, shared by every call on that GPU (calls that overlap on one GPU race for
// it).  Host code uses the device address hipGetSymbolAddress returns for the current device, never
// the array's name.
constexpr long long kLsqScratchDoubles = 1LL << 17;   // 1 MiB: 64 L n_rhs <= 131072
static __device__ __align__(256) double scratch[kLsqScratchDoubles];

namespace mr1l {
namespace {

constexpr int kLsqThreads = 256;
constexpr int kLsqBlocksPerLat = 64;
constexpr int kLsqSumThreads = 1024;

// grid (kLsqBlocksPerLat, L, n_rhs); s and grad may alias
template <typename T>
__global__ __launch_bounds__(kLsqThreads) void k_lsq(const LatDesc* __restrict__ desc, int64_t stride,
                                                     const cx<T>* s, const cx<T>* __restrict__ y,
                                                     const double* __restrict__ scale, cx<T>* grad,
                                                     double* __restrict__ part) {
    __shared__ double sh[kLsqThreads];
    const int l = blockIdx.y;
    const int64_t rhs = blockIdx.z;
    const LatDesc D = desc[l];
    const int64_t base = rhs * stride + D.samp_off;
    const double gw = scale ? scale[0] * D.invM : D.invM;
    double acc = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)kLsqThreads + threadIdx.x; j < D.M;
         j += (int64_t)gridDim.x * kLsqThreads) {
        const cx<T> a = s[base + j], b = y[base + j];
        const double re = (double)a.x - (double)b.x, im = (double)a.y - (double)b.y;
        acc += re * re + im * im;
        if (grad) grad[base + j] = cx<T>{(T)(gw * re), (T)(gw * im)};
    }
    if (!part) return;
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kLsqThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[(rhs * gridDim.y + l) * (int64_t)gridDim.x + blockIdx.x] = 0.5 * D.invM * sh[0];
}

// one block: thread t sums partials t, t + 1024, ... in order, then a tree over the threads
__global__ __launch_bounds__(kLsqSumThreads) void k_lsq_sum(const double* __restrict__ part, int64_t n,
                                                            double* __restrict__ loss) {
    __shared__ double sh[kLsqSumThreads];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kLsqSumThreads) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kLsqSumThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = sh[0];
}

// the two kernels with the block partials in ``part`` (64 L n_rhs doubles, every one written by
// k_lsq before k_lsq_sum reads it, so nothing needs clearing)
template <typename T>
mr1l_status launch_lsq(Plan* P, const void* s, const void* y, const double* scale, void* grad, double* loss,
                       double* part, hipStream_t st) {
    const int64_t nparts = (int64_t)kLsqBlocksPerLat * P->L * P->n_rhs;
    if (P->L > 0 && P->n_rhs > 0 && (grad || loss))
        hipLaunchKernelGGL(k_lsq<T>, dim3(kLsqBlocksPerLat, P->L, (unsigned)P->n_rhs), dim3(kLsqThreads), 0, st,
                           P->desc.as<LatDesc>(), P->sum_M, (const cx<T>*)s, (const cx<T>*)y, scale, (cx<T>*)grad,
                           loss ? part : nullptr);
    if (loss)
        hipLaunchKernelGGL(k_lsq_sum, dim3(1), dim3(kLsqSumThreads), 0, st, (const double*)part,
                           P->L > 0 && P->n_rhs > 0 ? nparts : (int64_t)0, loss);
    MR1L_HIP_TRY(hipGetLastError());
    return MR1L_OK;
}

template <typename T>
mr1l_status run_lsq(Plan* P, const void* s, const void* y, const double* scale, void* grad, double* loss,
                    hipStream_t st) {
    const int64_t nparts = (int64_t)kLsqBlocksPerLat * P->L * P->n_rhs;
    if (loss && nparts > 0 && P->lsq_part.bytes < (size_t)nparts * sizeof(double))
        MR1L_HIP_TRY(P->lsq_part.alloc((size_t)nparts * sizeof(double)));
    return launch_lsq<T>(P, s, y, scale, grad, loss, P->lsq_part.as<double>(), st);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// address of this device's array (looked up once per device; the device must be current)
mr1l_status scratch_for(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("mr1l_lsq_residual_noalloc: device index beyond 63");
        return MR1L_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return MR1L_ERR_HIP;
        }
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MR1L_OK;
}

}  // namespace
}  // namespace mr1l

using namespace mr1l;

extern "C" mr1l_status mr1l_lsq_residual_noalloc(mr1l_plan_t plan, const void* s, const void* y,
                                                 const double* scale, void* grad, double* loss, void* stream) {
    try {
        clear_error();
        Plan* P = (Plan*)plan;
        if (!P || ((!s || !y) && P->sum_M * P->n_rhs > 0)) {
            set_error("invalid argument to mr1l_lsq_residual_noalloc");
            return MR1L_ERR_ARG;
        }
        const int64_t nparts = (int64_t)kLsqBlocksPerLat * P->L * P->n_rhs;
        if (loss && nparts > kLsqScratchDoubles) {
            set_error("mr1l_lsq_residual_noalloc: the loss needs 64 L n_rhs = " + std::to_string(nparts) +
                      " block partials, more than the 131072 of its fixed buffer (use mr1l_lsq_residual)");
            return MR1L_ERR_UNSUPPORTED;
        }
        MR1L_HIP_TRY(hipSetDevice(P->device));
        double* part = nullptr;
        const mr1l_status st0 = scratch_for(P->device, &part);
        if (st0 != MR1L_OK) return st0;
        hipStream_t st = (hipStream_t)stream;
        return P->dtype == MR1L_C128 ? launch_lsq<double>(P, s, y, scale, grad, loss, part, st)
                                     : launch_lsq<float>(P, s, y, scale, grad, loss, part, st);
    } catch (const std::exception& e) {
        set_error(e.what());
        return MR1L_ERR_ARG;
    }
}

extern "C" mr1l_status mr1l_lsq_residual(mr1l_plan_t plan, const void* s, const void* y, const double* scale,
                                         void* grad, double* loss, void* stream) {
    try {
        clear_error();
        Plan* P = (Plan*)plan;
        if (!P || ((!s || !y) && P->sum_M * P->n_rhs > 0)) {
            set_error("invalid argument to mr1l_lsq_residual");
            return MR1L_ERR_ARG;
        }
        MR1L_HIP_TRY(hipSetDevice(P->device));
        hipStream_t st = (hipStream_t)stream;
        return P->dtype == MR1L_C128 ? run_lsq<double>(P, s, y, scale, grad, loss, st)
                                     : run_lsq<float>(P, s, y, scale, grad, loss, st);
    } catch (const std::exception& e) {
        set_error(e.what());
        return MR1L_ERR_ARG;
    }
}
