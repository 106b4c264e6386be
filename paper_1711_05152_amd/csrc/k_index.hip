// Integer and data-movement passes of the multiple rank-1 lattice FFT (Alg. 2):
//  * residues r_l(k) = k . z_l mod M_l in exact int64 arithmetic (Alg. 1/2, definition of I_l),
//    stored as int32 (r < M_l < 2^23) once per call and reused by every later pass;
//  * the alias histogram of every lattice as a 2-bit saturating count per bin, kept in two bitmaps
//    (seen, multi).  Each workgroup owns a range of bins of one lattice, builds its part of the
//    bitmaps in LDS with LDS atomics while streaming that lattice's residues, and writes its words
//    out whole, so no global atomics are needed.  k is in I_l iff its bin is not "multi";
//  * the gather of Alg. 2 (c_k = average over the lattices where k is unaliased, ascending l),
//  * the scatter of the adjoint (bins[r_l(k)] = c_k / counter_k, or summed for the Fourier
//    matrix), and an export of the integer results.
// Frequencies are stored component-major so every component load is coalesced.  Plans with
// several independent transforms find a frequency's transform by binary search.
#include "common.h"
#include "index_dev.h"

namespace mr1l {

__global__ void k_clear_u32(uint32_t* p, int64_t words) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// The transform a frequency belongs to.  SINGLE plans have one transform, so the lattice loop
// bounds and descriptor addresses are uniform across the wavefront (scalar loads).
template <bool SINGLE>
__device__ __forceinline__ TxDesc get_tx(const TxArgs& a, int64_t g) {
    if (SINGLE) return TxDesc{0, a.n, 0, a.L};
    return a.tx[find_tx(a.tx_foff, a.ntx + 1, g)];
}

// one thread per (frequency, lattice slot): blockIdx.y is the slot within the transform
template <typename K, bool SINGLE>
__global__ __launch_bounds__(256) void k_residues(TxArgs a) {
    const int j = blockIdx.y;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        if (j < t.nlat) a.res32[(int64_t)j * a.n + g] = (int32_t)residue<K>(a, a.desc[t.lat0 + j], g);
    }
}

constexpr int kHistThreads = 1024;
constexpr int kHistUnroll = 16;

__global__ __launch_bounds__(kHistThreads) void k_hist_lds(TxArgs a) {
    __shared__ uint32_t seen[kHistMaxBins / 32];
    __shared__ uint32_t multi[kHistMaxBins / 32];
    const HistTile h = a.hist[blockIdx.x];
    const LatDesc D = a.desc[h.l];
    const TxDesc t = a.tx[h.tx];
    const int words = (h.m1 - h.m0 + 31) >> 5;
    const uint32_t span = (uint32_t)(h.m1 - h.m0);
    for (int w = threadIdx.x; w < words; w += kHistThreads) {
        seen[w] = 0u;
        multi[w] = 0u;
    }
    __syncthreads();
    const int32_t* r = a.res32 + (int64_t)(h.l - t.lat0) * a.n + t.foff;
    const int64_t last = t.fn - 1;
    for (int64_t k0 = threadIdx.x; k0 < t.fn; k0 += kHistThreads * kHistUnroll) {
        // straight-line loads (clamped addresses) so that all of them are in flight together
        int32_t v[kHistUnroll];
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) v[u] = r[min(k0 + (int64_t)u * kHistThreads, last)];
        uint32_t rr[kHistUnroll], old[kHistUnroll];
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) {
            rr[u] = (k0 + (int64_t)u * kHistThreads <= last) ? (uint32_t)(v[u] - h.m0) : span;
            old[u] = rr[u] < span ? atomicOr(&seen[rr[u] >> 5], 1u << (rr[u] & 31)) : 0u;
        }
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u)
            if (rr[u] < span && ((old[u] >> (rr[u] & 31)) & 1u)) atomicOr(&multi[rr[u] >> 5], 1u << (rr[u] & 31));
    }
    __syncthreads();
    uint32_t* gs = a.bitmaps + D.bm_off + (h.m0 >> 5);
    for (int w = threadIdx.x; w < words; w += kHistThreads) {
        gs[w] = seen[w];
        gs[D.bm_words + w] = multi[w];
    }
}

constexpr int kRB = 4;  // right-hand sides per thread in gather/scatter
constexpr int kLC = 8;  // lattices whose loads are issued together

// unaliased flags of lattices j0 .. j0+kLC-1 for frequency g; residues returned in r
template <bool SINGLE>
__device__ __forceinline__ uint32_t unaliased_chunk(const TxArgs& a, const TxDesc& t, int j0, int64_t g,
                                                    int32_t* r) {
    const int jl = t.nlat - 1;
#pragma unroll
    for (int u = 0; u < kLC; ++u) r[u] = a.res32[(int64_t)min(j0 + u, jl) * a.n + g];
    uint32_t w[kLC];
#pragma unroll
    for (int u = 0; u < kLC; ++u) {
        const LatDesc& D = a.desc[t.lat0 + min(j0 + u, jl)];
        w[u] = a.bitmaps[D.bm_off + D.bm_words + (r[u] >> 5)];
    }
#pragma unroll
    for (int u = 0; u < kLC; ++u)
        if (j0 + u > jl) w[u] = 0xffffffffu;
    uint32_t mask = 0;
#pragma unroll
    for (int u = 0; u < kLC; ++u) mask |= (((w[u] >> (r[u] & 31)) & 1u) ^ 1u) << u;
    return mask;
}

template <typename T, bool EVAL, bool SINGLE>
__global__ __launch_bounds__(256) void k_gather(TxArgs a, const cx<T>* __restrict__ work, cx<T>* coeffs) {
    const int64_t rhs0 = (int64_t)blockIdx.y * kRB;
    const int nr = (int)min((int64_t)kRB, a.n_rhs - rhs0);
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        cx<T> acc[kRB];
#pragma unroll
        for (int q = 0; q < kRB; ++q) acc[q] = {(T)0, (T)0};
        int cnt = 0;
        for (int j0 = 0; j0 < t.nlat; j0 += kLC) {
            int32_t r[kLC];
            uint32_t use;
            if (EVAL) {
#pragma unroll
                for (int u = 0; u < kLC; ++u) r[u] = a.res32[(int64_t)min(j0 + u, t.nlat - 1) * a.n + g];
                use = (t.nlat - j0 >= kLC) ? 0xffu : ((1u << (t.nlat - j0)) - 1u);
            } else {
                use = unaliased_chunk<SINGLE>(a, t, j0, g, r);
                if (t.nlat - j0 < kLC) use &= (1u << (t.nlat - j0)) - 1u;
                cnt += __popc(use);
            }
            cx<T> v[kLC][kRB];
#pragma unroll
            for (int u = 0; u < kLC; ++u) {
                if ((use >> u) & 1u) {
                    const cx<T>* src = work + rhs0 * a.work_stride + a.desc[t.lat0 + j0 + u].work_off + r[u];
#pragma unroll
                    for (int q = 0; q < kRB; ++q)
                        if (q < nr) v[u][q] = src[q * a.work_stride];
                }
            }
#pragma unroll
            for (int u = 0; u < kLC; ++u)   // ascending l
                if ((use >> u) & 1u) {
#pragma unroll
                    for (int q = 0; q < kRB; ++q)
                        if (q < nr) acc[q] = acc[q] + v[u][q];
                }
        }
#pragma unroll
        for (int q = 0; q < kRB; ++q) {
            if (q < nr) {
                cx<T> v = acc[q];
                if (!EVAL) v = cnt ? cx<T>{v.x / (T)cnt, v.y / (T)cnt} : cx<T>{(T)0, (T)0};
                coeffs[(rhs0 + q) * a.n + g] = v;
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

template <typename T, bool EVAL, bool SINGLE>
__global__ __launch_bounds__(256) void k_scatter(TxArgs a, const cx<T>* __restrict__ coeffs, cx<T>* work) {
    const int64_t rhs0 = (int64_t)blockIdx.y * kRB;
    const int nr = (int)min((int64_t)kRB, a.n_rhs - rhs0);
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        cx<T> v[kRB];
#pragma unroll
        for (int q = 0; q < kRB; ++q) v[q] = (q < nr) ? coeffs[(rhs0 + q) * a.n + g] : cx<T>{(T)0, (T)0};
        if (EVAL) {
            for (int j = 0; j < t.nlat; ++j) {
                const int64_t r = a.res32[(int64_t)j * a.n + g];
                cx<T>* dst = work + rhs0 * a.work_stride + a.desc[t.lat0 + j].work_off + r;
#pragma unroll
                for (int q = 0; q < kRB; ++q)
                    if (q < nr) {
                        atomicAdd(&dst[q * a.work_stride].x, v[q].x);
                        atomicAdd(&dst[q * a.work_stride].y, v[q].y);
                    }
            }
            continue;
        }
        // counter_k over all lattices, keeping the first chunk's flags and residues
        int cnt = 0;
        for (int j0 = 0; j0 < t.nlat; j0 += kLC) {
            int32_t r[kLC];
            uint32_t use = unaliased_chunk<SINGLE>(a, t, j0, g, r);
            if (t.nlat - j0 < kLC) use &= (1u << (t.nlat - j0)) - 1u;
            cnt += __popc(use);
        }
        if (cnt == 0) continue;
#pragma unroll
        for (int q = 0; q < kRB; ++q) v[q] = {v[q].x / (T)cnt, v[q].y / (T)cnt};
        for (int j0 = 0; j0 < t.nlat; j0 += kLC) {
            int32_t r[kLC];
            uint32_t use = unaliased_chunk<SINGLE>(a, t, j0, g, r);
            if (t.nlat - j0 < kLC) use &= (1u << (t.nlat - j0)) - 1u;
#pragma unroll
            for (int u = 0; u < kLC; ++u)
                if ((use >> u) & 1u) {
                    cx<T>* dst = work + rhs0 * a.work_stride + a.desc[t.lat0 + j0 + u].work_off + r[u];
#pragma unroll
                    for (int q = 0; q < kRB; ++q)
                        if (q < nr) dst[q * a.work_stride] = v[q];
                }
        }
    }
}

__global__ __launch_bounds__(256) void k_alias_export(TxArgs a, int64_t* res, uint8_t* uniq, uint8_t* counter) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = a.tx[a.ntx == 1 ? 0 : find_tx(a.tx_foff, a.ntx + 1, g)];
        int cnt = 0;
        for (int j = 0; j < t.nlat; ++j) {
            const LatDesc D = a.desc[t.lat0 + j];
            const int64_t r = a.res32[(int64_t)j * a.n + g];
            const bool u = !is_multi(a.bitmaps, D, r);
            cnt += u;
            const int64_t o = (int64_t)j * a.n + g;
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

void launch_clear_u32(uint32_t* p, int64_t words, hipStream_t s) {
    if (words <= 0) return;
    hipLaunchKernelGGL(k_clear_u32, dim3(grid_for(words)), dim3(256), 0, s, p, words);
}

void launch_alias(const TxArgs& a, bool histogram, hipStream_t s) {
    if (a.n == 0 || a.L == 0) return;
    const dim3 grid(grid_for(a.n, 256, 65535), (unsigned)a.max_nlat);
    const bool single = a.ntx == 1;
    switch (a.fv.ktype) {
        case K_I8:
            if (single) hipLaunchKernelGGL((k_residues<int8_t, true>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((k_residues<int8_t, false>), grid, dim3(256), 0, s, a);
            break;
        case K_I16:
            if (single) hipLaunchKernelGGL((k_residues<int16_t, true>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((k_residues<int16_t, false>), grid, dim3(256), 0, s, a);
            break;
        default:
            if (single) hipLaunchKernelGGL((k_residues<int32_t, true>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((k_residues<int32_t, false>), grid, dim3(256), 0, s, a);
            break;
    }
    if (histogram) hipLaunchKernelGGL(k_hist_lds, dim3(a.nhist), dim3(kHistThreads), 0, s, a);
}

template <typename T>
void launch_gather(const TxArgs& a, const cx<T>* work, cx<T>* coeffs, bool eval, hipStream_t s) {
    if (a.n == 0 || a.n_rhs == 0) return;
    const dim3 grid(grid_for(a.n), (unsigned)((a.n_rhs + kRB - 1) / kRB));
    const bool single = a.ntx == 1;
    if (eval && single) hipLaunchKernelGGL((k_gather<T, true, true>), grid, dim3(256), 0, s, a, work, coeffs);
    else if (eval) hipLaunchKernelGGL((k_gather<T, true, false>), grid, dim3(256), 0, s, a, work, coeffs);
    else if (single) hipLaunchKernelGGL((k_gather<T, false, true>), grid, dim3(256), 0, s, a, work, coeffs);
    else hipLaunchKernelGGL((k_gather<T, false, false>), grid, dim3(256), 0, s, a, work, coeffs);
}

template <typename T>
void launch_clear_bins(const TxArgs& a, cx<T>* work, hipStream_t s) {
    if (a.L == 0 || a.n_rhs == 0) return;
    hipLaunchKernelGGL((k_clear_bins<T>), dim3(64, a.L, (unsigned)a.n_rhs), dim3(256), 0, s, a, work);
}

template <typename T>
void launch_scatter(const TxArgs& a, const cx<T>* coeffs, cx<T>* work, bool eval, hipStream_t s) {
    if (a.n == 0 || a.n_rhs == 0) return;
    const dim3 grid(grid_for(a.n), (unsigned)((a.n_rhs + kRB - 1) / kRB));
    const bool single = a.ntx == 1;
    if (eval && single) hipLaunchKernelGGL((k_scatter<T, true, true>), grid, dim3(256), 0, s, a, coeffs, work);
    else if (eval) hipLaunchKernelGGL((k_scatter<T, true, false>), grid, dim3(256), 0, s, a, coeffs, work);
    else if (single) hipLaunchKernelGGL((k_scatter<T, false, true>), grid, dim3(256), 0, s, a, coeffs, work);
    else hipLaunchKernelGGL((k_scatter<T, false, false>), grid, dim3(256), 0, s, a, coeffs, work);
}

void launch_alias_export(const TxArgs& a, int64_t* res, uint8_t* uniq, uint8_t* counter, hipStream_t s) {
    if (a.n == 0) return;
    hipLaunchKernelGGL(k_alias_export, dim3(grid_for(a.n)), dim3(256), 0, s, a, res, uniq, counter);
}

#define MR1L_INST_INDEX(T)                                                                                   \
    template void launch_gather<T>(const TxArgs&, const cx<T>*, cx<T>*, bool, hipStream_t);                 \
    template void launch_clear_bins<T>(const TxArgs&, cx<T>*, hipStream_t);                                 \
    template void launch_scatter<T>(const TxArgs&, const cx<T>*, cx<T>*, bool, hipStream_t);
MR1L_INST_INDEX(float)
MR1L_INST_INDEX(double)

}  // namespace mr1l
