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

#include <algorithm>
#include <climits>
#include <type_traits>

namespace mr1l {

__global__ void k_clear_u32(uint32_t* p, int64_t words) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// The transform a frequency belongs to.  SINGLE plans have one transform, so the lattice loop
// bounds and descriptor addresses are uniform across the wavefront (scalar loads).
template <bool SINGLE>
__device__ __forceinline__ TxDesc get_tx(const TxArgs& a, int64_t g) {
    if (SINGLE) return TxDesc{0, a.n, 0, a.L, 0, 0};
    return a.tx[find_tx(a.tx_foff, a.ntx + 1, g)];
}

// one thread per (frequency, lattice slot): blockIdx.y is the slot within the transform
template <typename K, bool SINGLE>
__global__ __launch_bounds__(256) void k_residues(TxArgs a) {
    const int j = blockIdx.y;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        if (j < t.nlat) a.res32[(int64_t)j * a.rs + g] = (int32_t)residue<K>(a, a.desc[t.lat0 + j], g);
    }
}

// 32-bit path: one thread per (frequency, group of kResLat lattice slots), its d components loaded
// once into registers.  Products of 24-bit operands wrap modulo 2^32, which is exact because the
// plan checked |k . z| < 2^31; the quotient estimate in double is off by at most one and the
// remainder s - qM is exact in double.  z rows are zero-padded to DP entries, so components past
// d (loaded from the clamped address of the last one) contribute nothing and every load is
// unconditional (all of them in flight together).
constexpr int kResLat = 4;
template <typename K, int DP, bool SINGLE>
__global__ __launch_bounds__(256) void k_residues_narrow(TxArgs a) {
    const K* __restrict__ f = (const K*)a.fv.f;
    const int dl = a.fv.d - 1;
    const int j0 = blockIdx.y * kResLat;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        if (j0 >= t.nlat) continue;
        int kv[DP];
#pragma unroll
        for (int c = 0; c < DP; ++c) kv[c] = (int)(f + (int64_t)min(c, dl) * a.fv.nf)[(uint32_t)g];
#pragma unroll
        for (int jj = 0; jj < kResLat; ++jj) {
            const int j = j0 + jj;
            if (j >= t.nlat) break;
            const int l = t.lat0 + j;
            const int32_t* __restrict__ zz = a.z32 + (int64_t)l * a.zrow;
            int s = 0;
#pragma unroll
            for (int c = 0; c < DP; ++c) s = __mul24(kv[c], zz[c]) + s;
            const int M = (int)a.desc[l].M;
            const double q = floor((double)s * a.desc[l].invM);
            int r = (int)fma(-q, (double)M, (double)s);
            r += r < 0 ? M : 0;
            r -= r >= M ? M : 0;
            a.res32[(int64_t)j * a.rs + g] = r;
        }
    }
}

// r = k . z mod M on the 32-bit path; zr is z_l padded with zeros to DP entries, so components
// past d (loaded from the clamped address of the last one) contribute nothing and every load is
// unconditional (all of them in flight together).  g < 2^31 (plan-checked), so the component
// loads take a uniform base and a 32-bit offset.
template <typename K, int DP>
__device__ __forceinline__ int residue_narrow(const TxArgs& a, const int* zr, int M, double invM, uint32_t g) {
    const K* __restrict__ f = (const K*)a.fv.f;
    const int dl = a.fv.d - 1;
    int kv[DP];
#pragma unroll
    for (int c = 0; c < DP; ++c) kv[c] = (int)(f + (int64_t)min(c, dl) * a.fv.nf)[g];
    int s = 0;
#pragma unroll
    for (int c = 0; c < DP; ++c) s = __mul24(kv[c], zr[c]) + s;
    const double q = floor((double)s * invM);
    int r = (int)fma(-q, (double)M, (double)s);
    r += r < 0 ? M : 0;
    r -= r >= M ? M : 0;
    return r;
}

// Fused residues + alias histogram (Alg. 2, definition of I_l): one workgroup per ResTile computes
// r_l(k) for its chunk of frequencies, stores them, and counts them into LDS bitmaps covering all
// bins of lattice l (2-bit saturating counts: seen, multi); the partial bitmaps are written out
// whole and combined by k_hist_merge.


template <typename K, int DP>
__global__ __launch_bounds__(kResThreads) void k_res_hist(TxArgs a) {
    extern __shared__ uint32_t rh_lds[];
    const ResTile rt = a.rtiles[blockIdx.x];
    const LatDesc D = a.desc[rt.l];
    const TxDesc t = a.tx[rt.tx];
    const int j = rt.l - t.lat0;
    const int words = (int)D.bm_words;
    uint32_t* seen = rh_lds;
    uint32_t* multi = rh_lds + a.rt_words;
    for (int w = threadIdx.x; w < words; w += kResThreads) {
        seen[w] = 0u;
        multi[w] = 0u;
    }
    __syncthreads();
    int32_t* res = a.res32 + (int64_t)j * a.rs;
    const int64_t last = rt.k1 - 1;
    constexpr int DZ = DP > 0 ? DP : 1;
    int zr[DZ];
#pragma unroll
    for (int c = 0; c < DZ; ++c) zr[c] = DP > 0 ? a.z32[(int64_t)rt.l * a.zrow + c] : 0;
    const int M = (int)D.M;
    constexpr int kResUnroll = res_unroll(DP);
    for (int64_t kb = rt.k0 + threadIdx.x; kb < rt.k1; kb += kResThreads * kResUnroll) {
        int r[kResUnroll];
#pragma unroll
        for (int u = 0; u < kResUnroll; ++u) {
            const int64_t g = min(kb + (int64_t)u * kResThreads, last);   // clamped: loads stay in range
            if (DP > 0) r[u] = residue_narrow<K, DZ>(a, zr, M, D.invM, (uint32_t)g);
            else r[u] = (int)residue<K>(a, D, g);
        }
        uint32_t old[kResUnroll];
#pragma unroll
        for (int u = 0; u < kResUnroll; ++u) {
            const int64_t g = kb + (int64_t)u * kResThreads;
            old[u] = 0u;
            if (g <= last) {
                res[(uint32_t)g] = r[u];
                old[u] = atomicOr(&seen[r[u] >> 5], 1u << (r[u] & 31));
            }
        }
#pragma unroll
        for (int u = 0; u < kResUnroll; ++u)
            if ((old[u] >> (r[u] & 31)) & 1u) atomicOr(&multi[r[u] >> 5], 1u << (r[u] & 31));
    }
    __syncthreads();
    uint32_t* p = a.part + rt.part;
    for (int w = threadIdx.x; w < words; w += kResThreads) {
        p[w] = seen[w];
        p[words + w] = multi[w];
    }
}

// bitmaps of lattice blockIdx.y from its partial bitmaps (consecutive, 2 bm_words apart): multi =
// some partial multi, or seen in two partials.  (A last-arriving-workgroup merge inside the fused
// kernel needs an agent-scope release per workgroup, i.e. an L2 writeback each, which costs more
// than this separate launch.)
__global__ __launch_bounds__(256) void k_hist_merge(TxArgs a) {
    const LatDesc D = a.desc[blockIdx.y];
    const int64_t words = D.bm_words;
    const uint32_t* p0 = a.part + a.rtiles[D.rt0].part;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < words; w += (int64_t)gridDim.x * blockDim.x) {
        uint32_t sa = 0u, ma = 0u;
        // all partials of a chunk in flight together (addresses clamped to the last partial, whose
        // repeats are not counted)
        constexpr int kMergeChunk = 16;
        for (int i = 0; i < D.rtn; i += kMergeChunk) {
            uint32_t ps[kMergeChunk], pm[kMergeChunk];
#pragma unroll
            for (int u = 0; u < kMergeChunk; ++u) {
                const int64_t t = min(i + u, D.rtn - 1);
                ps[u] = p0[t * 2 * words + w];
                pm[u] = p0[t * 2 * words + words + w];
            }
#pragma unroll
            for (int u = 0; u < kMergeChunk; ++u) {
                if (i + u < D.rtn) {
                    ma |= pm[u] | (sa & ps[u]);
                    sa |= ps[u];
                }
            }
        }
        a.bitmaps[D.bm_off + w] = sa;
        a.bitmaps[D.bm_off + words + w] = ma;
    }
}

constexpr int kHistThreads = 1024;
constexpr int kHistVec = 4;   // 16-byte residue loads in flight per thread and iteration

// Alias histogram of one bin range [m0, m1) of lattice l (Alg. 2, definition of I_l): the
// workgroup streams all residues of the lattice (16-byte loads; the row is 16-byte aligned) and
// counts those in its range into LDS bitmaps (2-bit saturating counts: seen, multi), then writes
// its words out whole.  Ranges of one lattice sit on workgroup slots of the same XCD, so the
// residue row is fetched into one L2 only.
__device__ __forceinline__ void hist_count(uint32_t* seen, uint32_t* multi, int32_t v, int32_t m0, uint32_t span,
                                           uint32_t& old, uint32_t& rr) {
    rr = (uint32_t)(v - m0);
    old = rr < span ? atomicOr(&seen[rr >> 5], 1u << (rr & 31)) : 0u;
}
__device__ __forceinline__ void hist_multi(uint32_t* multi, uint32_t old, uint32_t rr) {
    if ((old >> (rr & 31)) & 1u) atomicOr(&multi[rr >> 5], 1u << (rr & 31));
}

// LDS: seen[hist_words] then multi[hist_words] (dynamic)
__global__ __launch_bounds__(kHistThreads) void k_hist_lds(TxArgs a) {
    extern __shared__ uint32_t hist_lds[];
    const HistTile h = a.hist[blockIdx.x];
    if (h.l < 0) return;
    uint32_t* seen = hist_lds;
    uint32_t* multi = hist_lds + a.hist_words;
    const LatDesc D = a.desc[h.l];
    const TxDesc t = a.tx[h.tx];
    const int words = (h.m1 - h.m0 + 31) >> 5;
    const uint32_t span = (uint32_t)(h.m1 - h.m0);
    for (int w = threadIdx.x; w < words; w += kHistThreads) {
        seen[w] = 0u;
        multi[w] = 0u;
    }
    __syncthreads();
    const int32_t* row = a.res32 + (int64_t)(h.l - t.lat0) * a.rs;
    const int64_t k0 = t.foff, k1 = t.foff + t.fn;
    const int64_t a0 = std::min<int64_t>((k0 + 3) & ~(int64_t)3, k1);
    const int64_t a1 = std::max<int64_t>(a0, k1 & ~(int64_t)3);
    // unaligned head [k0, a0) and tail [a1, k1): at most 3 residues each
    if (threadIdx.x < a0 - k0 || threadIdx.x < k1 - a1) {
        uint32_t o0 = 0, r0 = span, o1 = 0, r1 = span;
        if (threadIdx.x < a0 - k0) hist_count(seen, multi, row[k0 + threadIdx.x], h.m0, span, o0, r0);
        if (threadIdx.x < k1 - a1) hist_count(seen, multi, row[a1 + threadIdx.x], h.m0, span, o1, r1);
        if (r0 < span) hist_multi(multi, o0, r0);
        if (r1 < span) hist_multi(multi, o1, r1);
    }
    const int4* v4 = (const int4*)(row + a0);
    const int64_t nv = (a1 - a0) >> 2;
    for (int64_t i = threadIdx.x; i < nv; i += kHistThreads * kHistVec) {
        int4 q[kHistVec];
#pragma unroll
        for (int u = 0; u < kHistVec; ++u) q[u] = v4[std::min<int64_t>(i + u * kHistThreads, nv - 1)];   // clamped
        uint32_t old[4 * kHistVec], rr[4 * kHistVec];
#pragma unroll
        for (int u = 0; u < kHistVec; ++u) {
            const bool ok = i + u * kHistThreads < nv;
            const int32_t e[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                rr[4 * u + c] = span;
                old[4 * u + c] = 0u;
                if (ok) hist_count(seen, multi, e[c], h.m0, span, old[4 * u + c], rr[4 * u + c]);
            }
        }
#pragma unroll
        for (int u = 0; u < 4 * kHistVec; ++u)
            if (rr[u] < span) hist_multi(multi, old[u], rr[u]);
    }
    __syncthreads();
    uint32_t* gs = a.bitmaps + D.bm_off + (h.m0 >> 5);
    for (int w = threadIdx.x; w < words; w += kHistThreads) {
        gs[w] = seen[w];
        gs[D.bm_words + w] = multi[w];
    }
}

constexpr int kRB = 4;  // right-hand sides per thread in gather/scatter with several right-hand sides

// unaliased flags of lattice slots j0 .. j0+LC-1 for frequency g (bit u set: k in I_l); residues in r.
// All LC residue loads, then all LC bitmap loads, are issued together.
template <int LC>
__device__ __forceinline__ uint32_t unaliased_chunk(const TxArgs& a, const TxDesc& t, int j0, int64_t g,
                                                    int32_t* r) {
    const int jl = t.nlat - 1;
#pragma unroll
    for (int u = 0; u < LC; ++u) r[u] = a.res32[(int64_t)min(j0 + u, jl) * a.rs + g];
    uint32_t w[LC];
#pragma unroll
    for (int u = 0; u < LC; ++u) {
        const LatDesc& D = a.desc[t.lat0 + min(j0 + u, jl)];
        w[u] = a.bitmaps[D.bm_off + D.bm_words + (r[u] >> 5)];
    }
    uint32_t mask = 0;
#pragma unroll
    for (int u = 0; u < LC; ++u)
        if (j0 + u <= jl) mask |= (((w[u] >> (r[u] & 31)) & 1u) ^ 1u) << u;
    return mask;
}

// lattice slots handled per chunk: all 16 loads in flight for one right-hand side, 8 for kRB
template <int RB> struct GatherChunk { static constexpr int v = RB == 1 ? 16 : 8; };

template <typename T, bool EVAL, bool SINGLE, int RB>
__global__ __launch_bounds__(256) void k_gather(TxArgs a, const cx<T>* __restrict__ work, cx<T>* coeffs) {
    constexpr int LC = GatherChunk<RB>::v;
    const int64_t rhs0 = (int64_t)blockIdx.y * RB;
    const int nr = (int)min((int64_t)RB, a.n_rhs - rhs0);
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        if (t.in_block) continue;   // the persistent small-transform kernel writes these
        cx<T> acc[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[q] = {(T)0, (T)0};
        int cnt = 0;
        for (int j0 = 0; j0 < t.nlat; j0 += LC) {
            int32_t r[LC];
            uint32_t use;
            if (EVAL) {
#pragma unroll
                for (int u = 0; u < LC; ++u) r[u] = a.res32[(int64_t)min(j0 + u, t.nlat - 1) * a.rs + g];
                use = (t.nlat - j0 >= LC) ? (uint32_t)((1ull << LC) - 1) : ((1u << (t.nlat - j0)) - 1u);
            } else {
                use = unaliased_chunk<LC>(a, t, j0, g, r);
                cnt += __popc(use);
            }
            cx<T> v[LC][RB];
#pragma unroll
            for (int u = 0; u < LC; ++u) {
                if ((use >> u) & 1u) {
                    const cx<T>* src = work + rhs0 * a.work_stride + a.desc[t.lat0 + j0 + u].work_off + r[u];
#pragma unroll
                    for (int q = 0; q < RB; ++q)
                        if (q < nr) v[u][q] = src[q * a.work_stride];
                }
            }
#pragma unroll
            for (int u = 0; u < LC; ++u)   // ascending l
                if ((use >> u) & 1u) {
#pragma unroll
                    for (int q = 0; q < RB; ++q)
                        if (q < nr) acc[q] = acc[q] + v[u][q];
                }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            if (q < nr) {
                cx<T> v = acc[q];
                if (!EVAL) v = cnt ? cx<T>{v.x / (T)cnt, v.y / (T)cnt} : cx<T>{(T)0, (T)0};
                coeffs[(rhs0 + q) * a.n + g] = v;
            }
        }
    }
}

// Single right-hand side: kSplit lanes per frequency share its lattice slots (lane s takes slots
// s, s + kSplit, ...), so eight times as many threads keep the random residue, bitmap and bin
// accesses in flight.  The gather's lane 0 adds the values in ascending slot order, fetching them
// from the other lanes by shuffles: the same order and rounding as one thread walking all slots.
constexpr int kSplit = 8;
constexpr int kSplitSlots = 2;   // slots per lane per pass (16 lattice slots of a frequency)

// transform of frequency g for a group of kSplit lanes: lane 0 of the group searches, the others
// take its answer (the binary search over the transform offsets is the slow part for many
// transforms)
template <bool SINGLE>
__device__ __forceinline__ TxDesc split_tx(const TxArgs& a, int64_t g, int sub, int lead) {
    if (SINGLE) return TxDesc{0, a.n, 0, a.L, 0, 0};
    int ti = 0;
    if (sub == 0) ti = find_tx(a.tx_foff, a.ntx + 1, g);
    ti = __shfl(ti, lead);
    return a.tx[ti];
}

// loads of the residues and alias words of slots j0 + u kSplit + sub (clamped to the last slot)
__device__ __forceinline__ void split_slots(const TxArgs& a, const TxDesc& t, int j0, int sub, int64_t g,
                                            int32_t* r, uint32_t* w) {
#pragma unroll
    for (int u = 0; u < kSplitSlots; ++u) r[u] = a.res32[(int64_t)min(j0 + u * kSplit + sub, t.nlat - 1) * a.rs + g];
#pragma unroll
    for (int u = 0; u < kSplitSlots; ++u) {
        const LatDesc& D = a.desc[t.lat0 + min(j0 + u * kSplit + sub, t.nlat - 1)];
        w[u] = a.bitmaps[D.bm_off + D.bm_words + (r[u] >> 5)];
    }
}

template <typename T, bool SINGLE>
__global__ __launch_bounds__(256) void k_gather_split(TxArgs a, const cx<T>* __restrict__ work,
                                                      cx<T>* coeffs) {
    const int sub = threadIdx.x & (kSplit - 1);
    const int lead = (int)(threadIdx.x & 63) & ~(kSplit - 1);      // lane of sub 0 in the wave
    const int64_t stride = ((int64_t)gridDim.x * blockDim.x) / kSplit;
    for (int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kSplit; g < a.n; g += stride) {
        const TxDesc t = split_tx<SINGLE>(a, g, sub, lead);
        if (t.in_block) continue;   // the persistent small-transform kernel writes these
        cx<T> acc = {(T)0, (T)0};
        int cnt = 0;
        for (int j0 = 0; j0 < t.nlat; j0 += kSplit * kSplitSlots) {
            int32_t r[kSplitSlots];
            uint32_t w[kSplitSlots];
            split_slots(a, t, j0, sub, g, r, w);
            cx<T> v[kSplitSlots];
            int own[kSplitSlots];
#pragma unroll
            for (int u = 0; u < kSplitSlots; ++u) {
                const int j = j0 + u * kSplit + sub;
                own[u] = j < t.nlat && !((w[u] >> (r[u] & 31)) & 1u);
                v[u] = own[u] ? work[a.desc[t.lat0 + j].work_off + r[u]] : cx<T>{(T)0, (T)0};
            }
#pragma unroll
            for (int u = 0; u < kSplitSlots; ++u) {
#pragma unroll
                for (int q = 0; q < kSplit; ++q) {   // slot j0 + u kSplit + q, ascending
                    const T vx = __shfl(v[u].x, lead + q);
                    const T vy = __shfl(v[u].y, lead + q);
                    const int o = __shfl(own[u], lead + q);
                    if (o) {
                        acc = acc + cx<T>{vx, vy};
                        ++cnt;
                    }
                }
            }
        }
        if (sub == 0) coeffs[g] = cnt ? cx<T>{acc.x / (T)cnt, acc.y / (T)cnt} : cx<T>{(T)0, (T)0};
    }
}

template <typename T, bool SINGLE>
__global__ __launch_bounds__(256) void k_scatter_split(TxArgs a, const cx<T>* __restrict__ coeffs, cx<T>* work) {
    constexpr int SPAN = kSplit * kSplitSlots;
    const int sub = threadIdx.x & (kSplit - 1);
    const int lead = (int)(threadIdx.x & 63) & ~(kSplit - 1);      // lane of sub 0 in the wave
    const int64_t stride = ((int64_t)gridDim.x * blockDim.x) / kSplit;
    for (int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kSplit; g < a.n; g += stride) {
        const TxDesc t = split_tx<SINGLE>(a, g, sub, lead);
        if (t.nlat == 0 || t.in_block) continue;
        const cx<T> c = coeffs[g];
        // counter_k over all slots (the first pass's slots are kept for the writes)
        int32_t r[kSplitSlots];
        uint32_t w[kSplitSlots];
        split_slots(a, t, 0, sub, g, r, w);
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < kSplitSlots; ++u) cnt += (u * kSplit + sub < t.nlat) && !((w[u] >> (r[u] & 31)) & 1u);
        for (int j0 = SPAN; j0 < t.nlat; j0 += SPAN) {
            int32_t rx[kSplitSlots];
            uint32_t wx[kSplitSlots];
            split_slots(a, t, j0, sub, g, rx, wx);
#pragma unroll
            for (int u = 0; u < kSplitSlots; ++u)
                cnt += (j0 + u * kSplit + sub < t.nlat) && !((wx[u] >> (rx[u] & 31)) & 1u);
        }
#pragma unroll
        for (int m = 1; m < kSplit; m <<= 1) cnt += __shfl_xor(cnt, m);
        if (cnt == 0) continue;
        const cx<T> v = {c.x / (T)cnt, c.y / (T)cnt};
        for (int j0 = 0; j0 < t.nlat; j0 += SPAN) {
            if (j0 > 0) split_slots(a, t, j0, sub, g, r, w);
#pragma unroll
            for (int u = 0; u < kSplitSlots; ++u) {
                const int j = j0 + u * kSplit + sub;
                if (j < t.nlat && !((w[u] >> (r[u] & 31)) & 1u)) work[a.desc[t.lat0 + j].work_off + r[u]] = v;
            }
        }
    }
}

// zero the first M_l entries (the DFT bins) of every lattice's work region (Fourier-matrix
// adjoint, which accumulates into the bins)
template <typename T>
__global__ void k_clear_bins(TxArgs a, cx<T>* work) {
    const int l = blockIdx.y;
    const int64_t rhs = blockIdx.z;
    const LatDesc D = a.desc[l];
    cx<T>* w = work + rhs * a.work_stride + D.work_off;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < D.M; m += (int64_t)gridDim.x * blockDim.x)
        w[m] = {(T)0, (T)0};
}

// Fourier-matrix adjoint: bins[r_l(k)] += c_k over every lattice, one thread per (lattice slot,
// frequency) pair (slot u / n of frequency u mod n), so that few frequencies still keep many
// residue loads and atomics in flight
template <typename T, bool SINGLE, int RB>
__global__ __launch_bounds__(256) void k_scatter_eval(TxArgs a, const cx<T>* __restrict__ coeffs, cx<T>* work) {
    const int64_t rhs0 = (int64_t)blockIdx.y * RB;
    const int nr = (int)min((int64_t)RB, a.n_rhs - rhs0);
    const int64_t pairs = a.n * (int64_t)a.max_nlat;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < pairs; u += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(u / a.n);
        const int64_t g = u - (int64_t)j * a.n;
        const TxDesc t = get_tx<SINGLE>(a, g);
        if (j >= t.nlat) continue;
        const int64_t r = a.res32[(int64_t)j * a.rs + g];
        cx<T> v[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) v[q] = (q < nr) ? coeffs[(rhs0 + q) * a.n + g] : cx<T>{(T)0, (T)0};
        cx<T>* dst = work + rhs0 * a.work_stride + a.desc[t.lat0 + j].work_off + r;
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (q < nr) {
                atomicAdd(&dst[q * a.work_stride].x, v[q].x);
                atomicAdd(&dst[q * a.work_stride].y, v[q].y);
            }
    }
}

// Adjoint of Alg. 2: bins[r_l(k)] = c_k / counter_k for every lattice where k is unaliased.  Only
// unaliased bins are written; the bins that stay stale (empty or shared) are masked out by stage 1
// of the Bluestein transform through the same alias bitmaps, so no clearing pass is needed.
template <typename T, bool SINGLE, int RB>
__global__ __launch_bounds__(256) void k_scatter(TxArgs a, const cx<T>* __restrict__ coeffs, cx<T>* work) {
    constexpr int LC = GatherChunk<RB>::v;
    const int64_t rhs0 = (int64_t)blockIdx.y * RB;
    const int nr = (int)min((int64_t)RB, a.n_rhs - rhs0);
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        cx<T> v[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) v[q] = (q < nr) ? coeffs[(rhs0 + q) * a.n + g] : cx<T>{(T)0, (T)0};
        if (t.nlat == 0 || t.in_block) continue;
        int32_t r[LC];
        uint32_t use = unaliased_chunk<LC>(a, t, 0, g, r);
        int cnt = __popc(use);
        for (int j0 = LC; j0 < t.nlat; j0 += LC) {   // counter_k over the remaining lattices
            int32_t rx[LC];
            cnt += __popc(unaliased_chunk<LC>(a, t, j0, g, rx));
        }
        if (cnt == 0) continue;
#pragma unroll
        for (int q = 0; q < RB; ++q) v[q] = {v[q].x / (T)cnt, v[q].y / (T)cnt};
        for (int j0 = 0; j0 < t.nlat; j0 += LC) {
            if (j0 > 0) use = unaliased_chunk<LC>(a, t, j0, g, r);
#pragma unroll
            for (int u = 0; u < LC; ++u)
                if ((use >> u) & 1u) {
                    cx<T>* dst = work + rhs0 * a.work_stride + a.desc[t.lat0 + j0 + u].work_off + r[u];
#pragma unroll
                    for (int q = 0; q < RB; ++q)
                        if (q < nr) dst[q * a.work_stride] = v[q];
                }
        }
    }
}

// ---- Fourier-matrix adjoint by counting sort --------------------------------------------------------
// bins_l[m] = sum over k with r_l(k) = m of c_k (synthesis A c on the lattices, Sec. 2.1): the pairs
// (k, l) are counted per bin, the counts scanned, the pairs placed in bin order, each bin's list put
// in ascending k (when the bin holds <= kBinSort of them; once per sort, not per right-hand-side
// chunk), and one thread per bin adds its frequencies' coefficients in list order, so every bin is
// written exactly once and the result does not depend on scheduling.
constexpr int kBinSort = 16;

template <bool SINGLE>
__global__ __launch_bounds__(256) void k_bin_count(TxArgs a) {
    const int j = blockIdx.y;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        if (j >= t.nlat) continue;
        const int32_t r = a.res32[(int64_t)j * a.rs + g];
        atomicAdd(&a.bcnt[a.desc[t.lat0 + j].samp_off + r], 1);
    }
}

// exclusive scan of 1024 values held one per thread (64-wide waves, then across the 16 waves)
__device__ __forceinline__ int block_excl_scan_1024(int v, int* lds16, int& total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds16[wv] = x;
    __syncthreads();
    int wbase = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        const int ws = lds16[w];
        if (w < wv) wbase += ws;
        tot += ws;
    }
    __syncthreads();
    total = tot;
    return wbase + x - v;
}

// chunk-local exclusive scans of the counts and chunk totals
__global__ __launch_bounds__(1024) void k_bin_scan(TxArgs a) {
    __shared__ int wsum[16];
    const int64_t c0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * (kScanChunk / 1024);
    int v[kScanChunk / 1024], run = 0;
#pragma unroll
    for (int i = 0; i < kScanChunk / 1024; ++i) {
        v[i] = c0 + i < a.nbins ? a.bcnt[c0 + i] : 0;
        run += v[i];
    }
    int total;
    int ex = block_excl_scan_1024(run, wsum, total);
#pragma unroll
    for (int i = 0; i < kScanChunk / 1024; ++i) {
        if (c0 + i < a.nbins) a.bloc[c0 + i] = ex;
        ex += v[i];
    }
    if (threadIdx.x == 0) a.bbase[blockIdx.x] = total;
}

// exclusive scan of the chunk totals in place (one workgroup)
__global__ __launch_bounds__(1024) void k_bin_scan_bases(TxArgs a, int nchunks) {
    __shared__ int wsum[16];
    int carry = 0;
    for (int c0 = 0; c0 < nchunks; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const int v = i < nchunks ? a.bbase[i] : 0;
        int total;
        const int ex = block_excl_scan_1024(v, wsum, total);
        if (i < nchunks) a.bbase[i] = carry + ex;
        carry += total;
    }
}

__device__ __forceinline__ int bin_offset(const TxArgs& a, int64_t b) {
    return a.bloc[b] + a.bbase[b / kScanChunk];
}

template <bool SINGLE>
__global__ __launch_bounds__(256) void k_bin_place(TxArgs a) {
    const int j = blockIdx.y;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        if (j >= t.nlat) continue;
        const LatDesc& D = a.desc[t.lat0 + j];
        const int64_t b = D.samp_off + a.res32[(int64_t)j * a.rs + g];
        const int pos = bin_offset(a, b) - bin_offset(a, D.samp_off) + atomicSub(&a.bcnt[b], 1) - 1;
        a.perm[(int64_t)j * a.rs + t.foff + pos] = (int32_t)g;
    }
}

// list of bin m (one thread per bin of lattice blockIdx.y) in ascending k: bins of up to four
// frequencies (almost all of them when the bins outnumber the frequencies) by a sorting network in
// registers, up to kBinSort by insertion, larger ones stay in placement order
__global__ __launch_bounds__(256) void k_bin_order(TxArgs a) {
    const int l = blockIdx.y;
    const LatDesc D = a.desc[l];
    const TxDesc t = a.tx[D.tx];
    const int j = l - t.lat0;
    const int base = bin_offset(a, D.samp_off);
    int32_t* pm = a.perm + (int64_t)j * a.rs + t.foff;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < D.M; m += (int64_t)gridDim.x * blockDim.x) {
        const int beg = bin_offset(a, D.samp_off + m) - base;
        const int end = m + 1 < D.M ? bin_offset(a, D.samp_off + m + 1) - base : (int)t.fn;
        const int cnt = end - beg;
        if (cnt <= 1 || cnt > kBinSort) continue;
        if (cnt <= 4) {
            int x[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) x[i] = i < cnt ? pm[beg + i] : INT_MAX;
            auto cx2 = [](int& u, int& v) {
                const int lo = min(u, v), hi = max(u, v);
                u = lo;
                v = hi;
            };
            cx2(x[0], x[1]);
            cx2(x[2], x[3]);
            cx2(x[0], x[2]);
            cx2(x[1], x[3]);
            cx2(x[1], x[2]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (i < cnt) pm[beg + i] = x[i];
            continue;
        }
        int ks[kBinSort];
        for (int i = 0; i < cnt; ++i) {   // insertion sort: ascending k
            const int k = pm[beg + i];
            int q = i;
            while (q > 0 && ks[q - 1] > k) {
                ks[q] = ks[q - 1];
                --q;
            }
            ks[q] = k;
        }
        for (int i = 0; i < cnt; ++i) pm[beg + i] = ks[i];
    }
}

// one thread per bin m of lattice blockIdx.y, every right-hand side of the chunk, RB of them at a
// time: the RB coefficient loads of one frequency are independent, so they are in flight together
// (each right-hand side adds the bin's frequencies in list order)
template <typename T, int RB>
__global__ __launch_bounds__(256) void k_bin_sum(TxArgs a, const cx<T>* __restrict__ coeffs, cx<T>* work) {
    const int l = blockIdx.y;
    const LatDesc D = a.desc[l];
    const TxDesc t = a.tx[D.tx];
    const int j = l - t.lat0;
    const int base = bin_offset(a, D.samp_off);
    const int32_t* pm = a.perm + (int64_t)j * a.rs + t.foff;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < D.M; m += (int64_t)gridDim.x * blockDim.x) {
        const int beg = bin_offset(a, D.samp_off + m) - base;
        const int end = m + 1 < D.M ? bin_offset(a, D.samp_off + m + 1) - base : (int)t.fn;
        const int cnt = end - beg;
        constexpr int KH = 2;   // leading frequencies of the list held in registers
        int kh[KH];
#pragma unroll
        for (int i = 0; i < KH; ++i) kh[i] = i < cnt ? pm[beg + i] : 0;
        for (int64_t rhs0 = 0; rhs0 < a.n_rhs; rhs0 += RB) {
            const int nr = (int)min((int64_t)RB, a.n_rhs - rhs0);
            const cx<T>* cr = coeffs + rhs0 * a.n;
            cx<T> acc[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) acc[q] = {(T)0, (T)0};
#pragma unroll
            for (int i = 0; i < KH; ++i) {
                if (i < cnt) {
                    cx<T> v[RB];
#pragma unroll
                    for (int q = 0; q < RB; ++q)
                        if (q < nr) v[q] = cr[q * a.n + kh[i]];
#pragma unroll
                    for (int q = 0; q < RB; ++q)
                        if (q < nr) acc[q] = acc[q] + v[q];
                }
            }
            for (int i = KH; i < cnt; ++i) {
                const int k = pm[beg + i];
                cx<T> v[RB];
#pragma unroll
                for (int q = 0; q < RB; ++q)
                    if (q < nr) v[q] = cr[q * a.n + k];
#pragma unroll
                for (int q = 0; q < RB; ++q)
                    if (q < nr) acc[q] = acc[q] + v[q];
            }
            cx<T>* wr = work + rhs0 * a.work_stride + D.work_off + m;
#pragma unroll
            for (int q = 0; q < RB; ++q)
                if (q < nr) wr[q * a.work_stride] = acc[q];
        }
    }
}

// ---- right-hand-side interleaving ------------------------------------------------------------------
// With several right-hand sides, the gather's random bin reads and the bin sums' random coefficient
// reads would fetch one line per right-hand side.  A block of RB right-hand sides is first copied
// into 64-byte slots (RB values of one bin, or of one coefficient, side by side; coalesced on both
// sides), so that one random access fetches the whole block in one line.  The sums run in the same
// order as in the plain kernels, so the results are bit-identical.
template <typename T>
struct alignas(64) RhsSlot {
    static constexpr int RB = 64 / (int)sizeof(cx<T>);
    cx<T> v[RB];
};

// bins m < M_l of lattice blockIdx.y, right-hand sides [0, nr) of work -> slot samp_off_l + m
template <typename T>
__global__ __launch_bounds__(256) void k_bins_ilv(TxArgs a, const cx<T>* __restrict__ work, RhsSlot<T>* out, int nr) {
    const LatDesc D = a.desc[blockIdx.y];
    if (a.tx[D.tx].in_block) return;   // written by the persistent small-transform kernel
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < D.M; m += (int64_t)gridDim.x * blockDim.x) {
        RhsSlot<T> v;
#pragma unroll
        for (int q = 0; q < RhsSlot<T>::RB; ++q)
            v.v[q] = q < nr ? work[q * a.work_stride + D.work_off + m] : cx<T>{(T)0, (T)0};
        out[D.samp_off + m] = v;
    }
}

// coefficients g < n, right-hand sides [0, nr) -> slot g
template <typename T>
__global__ __launch_bounds__(256) void k_coef_ilv(TxArgs a, const cx<T>* __restrict__ coeffs, RhsSlot<T>* out, int nr) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        RhsSlot<T> v;
#pragma unroll
        for (int q = 0; q < RhsSlot<T>::RB; ++q) v.v[q] = q < nr ? coeffs[q * a.n + g] : cx<T>{(T)0, (T)0};
        out[g] = v;
    }
}

// k_gather over interleaved bins: one thread per frequency, nr <= RB right-hand sides
template <typename T, bool EVAL, bool SINGLE>
__global__ __launch_bounds__(256) void k_gather_ilv(TxArgs a, const RhsSlot<T>* __restrict__ bins, cx<T>* coeffs,
                                                    int nr) {
    constexpr int RB = RhsSlot<T>::RB;
    constexpr int LC = 4;   // lattice slots in flight
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = get_tx<SINGLE>(a, g);
        if (t.in_block) continue;
        cx<T> acc[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[q] = {(T)0, (T)0};
        int cnt = 0;
        for (int j0 = 0; j0 < t.nlat; j0 += LC) {
            int32_t r[LC];
            uint32_t use;
            if (EVAL) {
#pragma unroll
                for (int u = 0; u < LC; ++u) r[u] = a.res32[(int64_t)min(j0 + u, t.nlat - 1) * a.rs + g];
                use = (t.nlat - j0 >= LC) ? (uint32_t)((1u << LC) - 1) : ((1u << (t.nlat - j0)) - 1u);
            } else {
                use = unaliased_chunk<LC>(a, t, j0, g, r);
                cnt += __popc(use);
            }
            RhsSlot<T> v[LC];
#pragma unroll
            for (int u = 0; u < LC; ++u)
                if ((use >> u) & 1u) v[u] = bins[a.desc[t.lat0 + j0 + u].samp_off + r[u]];
#pragma unroll
            for (int u = 0; u < LC; ++u)   // ascending l
                if ((use >> u) & 1u) {
#pragma unroll
                    for (int q = 0; q < RB; ++q) acc[q] = acc[q] + v[u].v[q];
                }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            if (q < nr) {
                cx<T> v = acc[q];
                if (!EVAL) v = cnt ? cx<T>{v.x / (T)cnt, v.y / (T)cnt} : cx<T>{(T)0, (T)0};
                coeffs[q * a.n + g] = v;
            }
        }
    }
}

// k_bin_sum over interleaved coefficients: one thread per bin, nr <= RB right-hand sides
template <typename T>
__global__ __launch_bounds__(256) void k_bin_sum_ilv(TxArgs a, const RhsSlot<T>* __restrict__ cs, cx<T>* work, int nr) {
    constexpr int RB = RhsSlot<T>::RB;
    const int l = blockIdx.y;
    const LatDesc D = a.desc[l];
    const TxDesc t = a.tx[D.tx];
    const int j = l - t.lat0;
    const int base = bin_offset(a, D.samp_off);
    const int32_t* pm = a.perm + (int64_t)j * a.rs + t.foff;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < D.M; m += (int64_t)gridDim.x * blockDim.x) {
        const int beg = bin_offset(a, D.samp_off + m) - base;
        const int end = m + 1 < D.M ? bin_offset(a, D.samp_off + m + 1) - base : (int)t.fn;
        const int cnt = end - beg;
        cx<T> acc[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[q] = {(T)0, (T)0};
        for (int i0 = 0; i0 < cnt; i0 += 2) {   // two slots in flight
            RhsSlot<T> v[2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (i0 + u < cnt) v[u] = cs[pm[beg + i0 + u]];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (i0 + u < cnt) {
#pragma unroll
                    for (int q = 0; q < RB; ++q) acc[q] = acc[q] + v[u].v[q];
                }
        }
        cx<T>* wr = work + D.work_off + m;
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (q < nr) wr[q * a.work_stride] = acc[q];
    }
}

__global__ __launch_bounds__(256) void k_alias_export(TxArgs a, int64_t* res, uint8_t* uniq, uint8_t* counter) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        const TxDesc t = a.tx[a.ntx == 1 ? 0 : find_tx(a.tx_foff, a.ntx + 1, g)];
        int cnt = 0;
        for (int j = 0; j < t.nlat; ++j) {
            const LatDesc D = a.desc[t.lat0 + j];
            const int64_t r = a.res32[(int64_t)j * a.rs + g];
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

template <int DP, typename K>
static void launch_res_narrow(const TxArgs& a, hipStream_t s) {
    const dim3 grid(grid_for(a.n, 256, 65535), (unsigned)((a.max_nlat + kResLat - 1) / kResLat));
    if (a.ntx == 1) hipLaunchKernelGGL((k_residues_narrow<K, DP, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_residues_narrow<K, DP, false>), grid, dim3(256), 0, s, a);
}

template <typename K>
static void launch_res(const TxArgs& a, hipStream_t s) {
    if (a.narrow) {
        if (a.zpad == 8) launch_res_narrow<8, K>(a, s);
        else if (a.zpad == 12) launch_res_narrow<12, K>(a, s);
        else if (a.zpad == 16) launch_res_narrow<16, K>(a, s);
        else if (a.zpad == 24) launch_res_narrow<24, K>(a, s);
        else launch_res_narrow<32, K>(a, s);
        return;
    }
    const dim3 grid(grid_for(a.n, 256, 65535), (unsigned)a.max_nlat);
    if (a.ntx == 1) hipLaunchKernelGGL((k_residues<K, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_residues<K, false>), grid, dim3(256), 0, s, a);
}

template <typename K, int DP>
static void launch_res_hist_k(const TxArgs& a, hipStream_t s) {
    const size_t lds = 2 * (size_t)a.rt_words * sizeof(uint32_t);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_res_hist<K, DP>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_res_hist<K, DP>), dim3(a.nrt), dim3(kResThreads), lds, s, a);
}

template <typename K>
static void launch_res_hist(const TxArgs& a, hipStream_t s) {
    if (!a.narrow) launch_res_hist_k<K, 0>(a, s);
    else if (a.zpad == 8) launch_res_hist_k<K, 8>(a, s);
    else if (a.zpad == 12) launch_res_hist_k<K, 12>(a, s);
    else if (a.zpad == 16) launch_res_hist_k<K, 16>(a, s);
    else if (a.zpad == 24) launch_res_hist_k<K, 24>(a, s);
    else launch_res_hist_k<K, 32>(a, s);
}

void launch_alias(const TxArgs& a, bool histogram, hipStream_t s) {
    if (a.n == 0 || a.L == 0) return;
    if (histogram && a.fused) {
        switch (a.fv.ktype) {
            case K_I8: launch_res_hist<int8_t>(a, s); break;
            case K_I16: launch_res_hist<int16_t>(a, s); break;
            default: launch_res_hist<int32_t>(a, s); break;
        }
        const unsigned gx = (unsigned)std::max(1, std::min(64, (a.rt_words + 255) / 256));
        hipLaunchKernelGGL(k_hist_merge, dim3(gx, (unsigned)a.L), dim3(256), 0, s, a);
        return;
    }
    switch (a.fv.ktype) {
        case K_I8: launch_res<int8_t>(a, s); break;
        case K_I16: launch_res<int16_t>(a, s); break;
        default: launch_res<int32_t>(a, s); break;
    }
    if (histogram)
        hipLaunchKernelGGL(k_hist_lds, dim3(a.nhist), dim3(kHistThreads), 2 * a.hist_words * sizeof(uint32_t), s, a);
}

// The lane-split gather/scatter read each residue row in 32-byte pieces (a wavefront covers 8
// frequencies); that pays while the residue rows stay in cache and costs HBM traffic beyond
// (measured: 18.6 million frequencies of 512 transforms, 5.6 / 7.4 ms split against ~4 ms).
static inline bool split_pays(const TxArgs& a) { return a.n * (int64_t)a.max_nlat * 4 <= ((int64_t)64 << 20); }

template <typename T>
void launch_gather(const TxArgs& a, const cx<T>* work, cx<T>* coeffs, bool eval, hipStream_t s) {
    if (a.n == 0 || a.n_rhs == 0) return;
    const bool single = a.ntx == 1;
    if (a.n_rhs > 1 && a.ilv_bins) {
        constexpr int RB = RhsSlot<T>::RB;
        RhsSlot<T>* buf = (RhsSlot<T>*)a.ilv;
        for (int64_t r0 = 0; r0 < a.n_rhs; r0 += RB) {
            const int nr = (int)std::min<int64_t>(RB, a.n_rhs - r0);
            hipLaunchKernelGGL((k_bins_ilv<T>), dim3(grid_for(a.max_M, 256, 65535), (unsigned)a.L), dim3(256), 0, s, a,
                               work + r0 * a.work_stride, buf, nr);
            cx<T>* cr = coeffs + r0 * a.n;
            const dim3 grid(grid_for(a.n));
            if (eval && single) hipLaunchKernelGGL((k_gather_ilv<T, true, true>), grid, dim3(256), 0, s, a, buf, cr, nr);
            else if (eval) hipLaunchKernelGGL((k_gather_ilv<T, true, false>), grid, dim3(256), 0, s, a, buf, cr, nr);
            else if (single) hipLaunchKernelGGL((k_gather_ilv<T, false, true>), grid, dim3(256), 0, s, a, buf, cr, nr);
            else hipLaunchKernelGGL((k_gather_ilv<T, false, false>), grid, dim3(256), 0, s, a, buf, cr, nr);
        }
        return;
    }
    auto go = [&](auto RBc) {
        constexpr int RB = decltype(RBc)::value;
        const dim3 grid(grid_for(a.n), (unsigned)((a.n_rhs + RB - 1) / RB));
        if (eval && single) hipLaunchKernelGGL((k_gather<T, true, true, RB>), grid, dim3(256), 0, s, a, work, coeffs);
        else if (eval) hipLaunchKernelGGL((k_gather<T, true, false, RB>), grid, dim3(256), 0, s, a, work, coeffs);
        else if (RB == 1 && split_pays(a)) {
            const dim3 g4(grid_for(a.n * kSplit));
            if (single) hipLaunchKernelGGL((k_gather_split<T, true>), g4, dim3(256), 0, s, a, work, coeffs);
            else hipLaunchKernelGGL((k_gather_split<T, false>), g4, dim3(256), 0, s, a, work, coeffs);
        }
        else if (single) hipLaunchKernelGGL((k_gather<T, false, true, RB>), grid, dim3(256), 0, s, a, work, coeffs);
        else hipLaunchKernelGGL((k_gather<T, false, false, RB>), grid, dim3(256), 0, s, a, work, coeffs);
    };
    if (a.n_rhs == 1) go(std::integral_constant<int, 1>{});
    else go(std::integral_constant<int, kRB>{});
}

template <typename T>
void launch_clear_bins(const TxArgs& a, cx<T>* work, hipStream_t s) {
    if (a.L == 0 || a.n_rhs == 0) return;
    hipLaunchKernelGGL((k_clear_bins<T>), dim3(64, a.L, (unsigned)a.n_rhs), dim3(256), 0, s, a, work);
}

template <typename T>
void launch_scatter(const TxArgs& a, const cx<T>* coeffs, cx<T>* work, bool eval, hipStream_t s) {
    if (a.n == 0 || a.n_rhs == 0) return;
    const bool single = a.ntx == 1;
    auto go = [&](auto RBc) {
        constexpr int RB = decltype(RBc)::value;
        const dim3 grid(grid_for(a.n), (unsigned)((a.n_rhs + RB - 1) / RB));
        const dim3 gpair(grid_for(a.n * (int64_t)a.max_nlat), grid.y);
        if (eval && single) hipLaunchKernelGGL((k_scatter_eval<T, true, RB>), gpair, dim3(256), 0, s, a, coeffs, work);
        else if (eval) hipLaunchKernelGGL((k_scatter_eval<T, false, RB>), gpair, dim3(256), 0, s, a, coeffs, work);
        else if (RB == 1 && split_pays(a)) {
            const dim3 g4(grid_for(a.n * kSplit));
            if (single) hipLaunchKernelGGL((k_scatter_split<T, true>), g4, dim3(256), 0, s, a, coeffs, work);
            else hipLaunchKernelGGL((k_scatter_split<T, false>), g4, dim3(256), 0, s, a, coeffs, work);
        }
        else if (single) hipLaunchKernelGGL((k_scatter<T, true, RB>), grid, dim3(256), 0, s, a, coeffs, work);
        else hipLaunchKernelGGL((k_scatter<T, false, RB>), grid, dim3(256), 0, s, a, coeffs, work);
    };
    if (a.n_rhs == 1) go(std::integral_constant<int, 1>{});
    else go(std::integral_constant<int, kRB>{});
}

void launch_bin_sort(const TxArgs& a, hipStream_t s) {
    if (a.n == 0 || a.L == 0 || a.nbins == 0) return;
    const dim3 grid(grid_for(a.n, 256, 65535), (unsigned)a.max_nlat);
    if (a.ntx == 1) hipLaunchKernelGGL((k_bin_count<true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_bin_count<false>), grid, dim3(256), 0, s, a);
    const int nchunks = (int)((a.nbins + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_bin_scan, dim3(nchunks), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_bin_scan_bases, dim3(1), dim3(1024), 0, s, a, nchunks);
    if (a.ntx == 1) hipLaunchKernelGGL((k_bin_place<true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_bin_place<false>), grid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_bin_order, dim3(grid_for(a.max_M, 256, 65535), (unsigned)a.L), dim3(256), 0, s, a);
}

template <typename T>
void launch_bin_sum(const TxArgs& a, const cx<T>* coeffs, cx<T>* work, hipStream_t s) {
    if (a.L == 0 || a.n_rhs == 0) return;
    const dim3 grid(grid_for(a.max_M, 256, 65535), (unsigned)a.L);
    if (a.n_rhs > 1 && a.ilv_coef) {
        constexpr int RB = RhsSlot<T>::RB;
        RhsSlot<T>* buf = (RhsSlot<T>*)a.ilv;
        for (int64_t r0 = 0; r0 < a.n_rhs; r0 += RB) {
            const int nr = (int)std::min<int64_t>(RB, a.n_rhs - r0);
            if (a.n > 0)
                hipLaunchKernelGGL((k_coef_ilv<T>), dim3(grid_for(a.n)), dim3(256), 0, s, a, coeffs + r0 * a.n, buf, nr);
            hipLaunchKernelGGL((k_bin_sum_ilv<T>), grid, dim3(256), 0, s, a, buf, work + r0 * a.work_stride, nr);
        }
        return;
    }
    if (a.n_rhs == 1) hipLaunchKernelGGL((k_bin_sum<T, 1>), grid, dim3(256), 0, s, a, coeffs, work);
    else if (a.n_rhs <= 4) hipLaunchKernelGGL((k_bin_sum<T, 4>), grid, dim3(256), 0, s, a, coeffs, work);
    else hipLaunchKernelGGL((k_bin_sum<T, 8>), grid, dim3(256), 0, s, a, coeffs, work);
}
template void launch_bin_sum<float>(const TxArgs&, const cx<float>*, cx<float>*, hipStream_t);
template void launch_bin_sum<double>(const TxArgs&, const cx<double>*, cx<double>*, hipStream_t);

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
