// Integer and data-movement passes of the multiple rank-1 lattice FFT (Alg. 2):
//  * residues r_l(k) = k . z_l mod M_l in exact int64 arithmetic (Alg. 1/2, definition of I_l),
//  * the alias histogram of every lattice as a 2-bit saturating count per bin, kept in two
//    bitmaps (seen, multi) updated with global atomic OR; k is in I_l iff its bin is not "multi",
//  * the gather of Alg. 2 (c_k = average over the lattices where k is unaliased, ascending l),
//  * the scatter of the adjoint (bins[r_l(k)] = c_k / counter_k, or summed for the Fourier
//    matrix), and an export of the integer results.
// One thread per frequency; frequencies are stored component-major so every component load is
// coalesced.  Plans with several independent transforms find their transform by binary search.
#include "common.h"
#include "index_dev.h"

namespace mr1l {

__global__ void k_clear_u32(uint32_t* p, int64_t words) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <typename K>
__global__ __launch_bounds__(256) void k_residue_hist(TxArgs a) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = a.tx[a.ntx == 1 ? 0 : find_tx(a.tx_foff, a.ntx + 1, g)];
        for (int l = t.lat0; l < t.lat0 + t.nlat; ++l) {
            const LatDesc D = a.desc[l];
            const int64_t r = residue<K>(a, D, g);
            uint32_t* seen = a.bitmaps + D.bm_off + (r >> 5);
            const uint32_t bit = 1u << (r & 31);
            const uint32_t old = atomicOr(seen, bit);
            if (old & bit) atomicOr(seen + D.bm_words, bit);
        }
    }
}

constexpr int kRB = 4;  // right-hand sides per thread in gather/scatter

template <typename T, typename K, bool EVAL>
__global__ __launch_bounds__(256) void k_gather(TxArgs a, const cx<T>* __restrict__ work, cx<T>* coeffs) {
    const int64_t rhs0 = (int64_t)blockIdx.y * kRB;
    const int nr = (int)min((int64_t)kRB, a.n_rhs - rhs0);
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = a.tx[a.ntx == 1 ? 0 : find_tx(a.tx_foff, a.ntx + 1, g)];
        cx<T> acc[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j) acc[j] = {(T)0, (T)0};
        int cnt = 0;
        for (int l = t.lat0; l < t.lat0 + t.nlat; ++l) {
            const LatDesc D = a.desc[l];
            const int64_t r = residue<K>(a, D, g);
            if (!EVAL) {
                if (is_multi(a.bitmaps, D, r)) continue;
                ++cnt;
            }
            const cx<T>* src = work + rhs0 * a.work_stride + D.work_off + r;
#pragma unroll
            for (int j = 0; j < kRB; ++j)
                if (j < nr) acc[j] = acc[j] + src[j * a.work_stride];
        }
#pragma unroll
        for (int j = 0; j < kRB; ++j) {
            if (j < nr) {
                cx<T> v = acc[j];
                if (!EVAL) v = cnt ? cx<T>{v.x / (T)cnt, v.y / (T)cnt} : cx<T>{(T)0, (T)0};
                coeffs[(rhs0 + j) * a.n + g] = v;
            }
        }
    }
}

// zero the first M_l entries (the DFT bins) of every lattice's work region
template <typename T>
__global__ void k_clear_bins(TxArgs a, cx<T>* work) {
    const int l = blockIdx.y;
    const int64_t rhs = blockIdx.z;
    const LatDesc D = a.desc[l];
    cx<T>* w = work + rhs * a.work_stride + D.work_off;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < D.M; m += (int64_t)gridDim.x * blockDim.x)
        w[m] = {(T)0, (T)0};
}

template <typename T, typename K, bool EVAL>
__global__ __launch_bounds__(256) void k_scatter(TxArgs a, const cx<T>* __restrict__ coeffs, cx<T>* work) {
    const int64_t rhs0 = (int64_t)blockIdx.y * kRB;
    const int nr = (int)min((int64_t)kRB, a.n_rhs - rhs0);
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = a.tx[a.ntx == 1 ? 0 : find_tx(a.tx_foff, a.ntx + 1, g)];
        int cnt = 0;
        if (!EVAL) {
            for (int l = t.lat0; l < t.lat0 + t.nlat; ++l) {
                const LatDesc D = a.desc[l];
                if (!is_multi(a.bitmaps, D, residue<K>(a, D, g))) ++cnt;
            }
            if (cnt == 0) continue;
        }
        cx<T> v[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j) {
            v[j] = {(T)0, (T)0};
            if (j < nr) {
                v[j] = coeffs[(rhs0 + j) * a.n + g];
                if (!EVAL) v[j] = {v[j].x / (T)cnt, v[j].y / (T)cnt};
            }
        }
        for (int l = t.lat0; l < t.lat0 + t.nlat; ++l) {
            const LatDesc D = a.desc[l];
            const int64_t r = residue<K>(a, D, g);
            if (!EVAL && is_multi(a.bitmaps, D, r)) continue;
            cx<T>* dst = work + rhs0 * a.work_stride + D.work_off + r;
#pragma unroll
            for (int j = 0; j < kRB; ++j) {
                if (j < nr) {
                    if (EVAL) {
                        atomicAdd(&dst[j * a.work_stride].x, v[j].x);
                        atomicAdd(&dst[j * a.work_stride].y, v[j].y);
                    } else {
                        dst[j * a.work_stride] = v[j];
                    }
                }
            }
        }
    }
}

template <typename K>
__global__ __launch_bounds__(256) void k_alias_export(TxArgs a, int64_t* res, uint8_t* uniq, uint8_t* counter) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = a.tx[a.ntx == 1 ? 0 : find_tx(a.tx_foff, a.ntx + 1, g)];
        int cnt = 0;
        for (int l = t.lat0; l < t.lat0 + t.nlat; ++l) {
            const LatDesc D = a.desc[l];
            const int64_t r = residue<K>(a, D, g);
            const bool u = !is_multi(a.bitmaps, D, r);
            cnt += u;
            const int64_t o = (int64_t)(l - t.lat0) * a.n + g;
            if (res) res[o] = r;
            if (uniq) uniq[o] = (uint8_t)u;
        }
        if (counter) counter[g] = (uint8_t)min(cnt, 255);
    }
}

// ---- launchers -------------------------------------------------------------------------------------
static inline int grid_for(int64_t n, int threads = 256, int cap = 8192) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

template <typename T>
void launch_clear_u32(uint32_t* p, int64_t words, hipStream_t s) {
    if (words <= 0) return;
    hipLaunchKernelGGL(k_clear_u32, dim3(grid_for(words)), dim3(256), 0, s, p, words);
}

template <typename T>
void launch_residue_hist(const TxArgs& a, hipStream_t s) {
    if (a.n == 0) return;
    const dim3 grid(grid_for(a.n));
    switch (a.fv.ktype) {
        case K_I8: hipLaunchKernelGGL(k_residue_hist<int8_t>, grid, dim3(256), 0, s, a); break;
        case K_I16: hipLaunchKernelGGL(k_residue_hist<int16_t>, grid, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(k_residue_hist<int32_t>, grid, dim3(256), 0, s, a); break;
    }
}

template <typename T, typename K>
static void gather_k(const TxArgs& a, const cx<T>* work, cx<T>* coeffs, bool eval, hipStream_t s) {
    const dim3 grid(grid_for(a.n), (unsigned)((a.n_rhs + kRB - 1) / kRB));
    if (eval) hipLaunchKernelGGL((k_gather<T, K, true>), grid, dim3(256), 0, s, a, work, coeffs);
    else hipLaunchKernelGGL((k_gather<T, K, false>), grid, dim3(256), 0, s, a, work, coeffs);
}

template <typename T>
void launch_gather(const TxArgs& a, const cx<T>* work, cx<T>* coeffs, bool eval, hipStream_t s) {
    if (a.n == 0 || a.n_rhs == 0) return;
    switch (a.fv.ktype) {
        case K_I8: gather_k<T, int8_t>(a, work, coeffs, eval, s); break;
        case K_I16: gather_k<T, int16_t>(a, work, coeffs, eval, s); break;
        default: gather_k<T, int32_t>(a, work, coeffs, eval, s); break;
    }
}

template <typename T>
void launch_clear_bins(const TxArgs& a, cx<T>* work, hipStream_t s) {
    if (a.L == 0 || a.n_rhs == 0) return;
    hipLaunchKernelGGL((k_clear_bins<T>), dim3(64, a.L, (unsigned)a.n_rhs), dim3(256), 0, s, a, work);
}

template <typename T, typename K>
static void scatter_k(const TxArgs& a, const cx<T>* coeffs, cx<T>* work, bool eval, hipStream_t s) {
    const dim3 grid(grid_for(a.n), (unsigned)((a.n_rhs + kRB - 1) / kRB));
    if (eval) hipLaunchKernelGGL((k_scatter<T, K, true>), grid, dim3(256), 0, s, a, coeffs, work);
    else hipLaunchKernelGGL((k_scatter<T, K, false>), grid, dim3(256), 0, s, a, coeffs, work);
}

template <typename T>
void launch_scatter(const TxArgs& a, const cx<T>* coeffs, cx<T>* work, bool eval, hipStream_t s) {
    if (a.n == 0 || a.n_rhs == 0) return;
    switch (a.fv.ktype) {
        case K_I8: scatter_k<T, int8_t>(a, coeffs, work, eval, s); break;
        case K_I16: scatter_k<T, int16_t>(a, coeffs, work, eval, s); break;
        default: scatter_k<T, int32_t>(a, coeffs, work, eval, s); break;
    }
}

void launch_alias_export(const TxArgs& a, int64_t* res, uint8_t* uniq, uint8_t* counter, hipStream_t s) {
    if (a.n == 0) return;
    const dim3 grid(grid_for(a.n));
    switch (a.fv.ktype) {
        case K_I8: hipLaunchKernelGGL(k_alias_export<int8_t>, grid, dim3(256), 0, s, a, res, uniq, counter); break;
        case K_I16: hipLaunchKernelGGL(k_alias_export<int16_t>, grid, dim3(256), 0, s, a, res, uniq, counter); break;
        default: hipLaunchKernelGGL(k_alias_export<int32_t>, grid, dim3(256), 0, s, a, res, uniq, counter); break;
    }
}

#define MR1L_INST_INDEX(T)                                                                                   \
    template void launch_clear_u32<T>(uint32_t*, int64_t, hipStream_t);                                     \
    template void launch_residue_hist<T>(const TxArgs&, hipStream_t);                                       \
    template void launch_gather<T>(const TxArgs&, const cx<T>*, cx<T>*, bool, hipStream_t);                 \
    template void launch_clear_bins<T>(const TxArgs&, cx<T>*, hipStream_t);                                 \
    template void launch_scatter<T>(const TxArgs&, const cx<T>*, cx<T>*, bool, hipStream_t);
MR1L_INST_INDEX(float)
MR1L_INST_INDEX(double)

}  // namespace mr1l
