// Alg. 1: reconstructing multiple rank-1 lattices with pairwise distinct prime sizes, plus the
// repetition of Alg. 3 step 2b (at most b calls, the last one kept if none covers I).
//
// Host side: L_max and lambda (Alg. 1 first two steps), the prime sizes p > lambda of P^I found by
// trial division with a cached table of small primes, and the random generating vectors
// (SplitMix64 Z stream keyed by (t, call, L)).  Device side, for rounds of up to sixteen trial
// lattices: the residues of all frequencies and the alias bitmaps of every lattice of the round
// (LDS bitmaps per chunk of frequencies plus a merge; global atomics for lattices above 2^19
// bins), then one pass that extends the running union of the unaliased sets and counts the
// covered frequencies after each lattice of the round, and one device-to-host copy of those counts
// (the stopping test of Alg. 1, applied lattice by lattice on the host).  The construction variant
// with redraws keeps one lattice per round.
#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "index_dev.h"
#include "runtime.h"

namespace mr1l {

template <typename K>
__global__ __launch_bounds__(256) void k_trial_hist(const K* __restrict__ f, int64_t nf, int d, int64_t n,
                                                    const int64_t* __restrict__ z, int64_t M, double invM, int fast,
                                                    uint32_t* bm, int64_t words) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = dot_kz<K>(f, nf, d, g, z);
        const int64_t r = fast ? mod_fast(s, M, invM) : mod_exact(s, M);
        const uint32_t bit = 1u << (r & 31);
        const uint32_t old = atomicOr(bm + (r >> 5), bit);
        if (old & bit) atomicOr(bm + words + (r >> 5), bit);
    }
}

template <typename K>
__global__ __launch_bounds__(256) void k_trial_cover(const K* __restrict__ f, int64_t nf, int d, int64_t n,
                                                     const int64_t* __restrict__ z, int64_t M, double invM, int fast,
                                                     const uint32_t* __restrict__ bm, int64_t words, uint8_t* covered,
                                                     unsigned long long* count) {
    __shared__ unsigned int part[256];
    unsigned int local = 0;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        if (covered[g]) {
            ++local;
            continue;
        }
        const int64_t s = dot_kz<K>(f, nf, d, g, z);
        const int64_t r = fast ? mod_fast(s, M, invM) : mod_exact(s, M);
        if (!((bm[words + (r >> 5)] >> (r & 31)) & 1u)) {
            covered[g] = 1;
            ++local;
        }
    }
    part[threadIdx.x] = local;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(count, (unsigned long long)part[0]);
}

// Batched trials (Alg. 1 itself): lattices i = 0..nk-1 of a round, generating vectors z[i][d],
// sizes M[i]; bitmaps of lattice i at bm + i * 2 * wstride (seen, then multi at + wstride).
constexpr int kSpec = 16;
struct TrialRound {
    int64_t M[kSpec];
    double invM[kSpec];
    int nk;
};

// grid (blocks, nk): alias bitmaps of every lattice of the round
template <typename K>
__global__ __launch_bounds__(256) void k_trial_hist_round(const K* __restrict__ f, int64_t nf, int d, int64_t n,
                                                          const int64_t* __restrict__ z, TrialRound tr, int fast,
                                                          uint32_t* bm, int64_t wstride) {
    const int i = blockIdx.y;
    const int64_t M = tr.M[i];
    uint32_t* b = bm + (int64_t)i * 2 * wstride;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = dot_kz<K>(f, nf, d, g, z + (int64_t)i * d);
        const int64_t r = fast ? mod_fast(s, M, tr.invM[i]) : mod_exact(s, M);
        const uint32_t bit = 1u << (r & 31);
        const uint32_t old = atomicOr(b + (r >> 5), bit);
        if (old & bit) atomicOr(b + wstride + (r >> 5), bit);
    }
}

// LDS form of the round's histograms (lattices of at most kTrialLdsWords bitmap words): one
// workgroup per (chunk of frequencies, lattice i) counts its residues into LDS bitmaps over all
// bins of the lattice and writes them out whole as a partial (lattice i, chunk c at
// part + (i chunks + c) 2 wstride); k_trial_merge_round combines the partials of every lattice
// (multi = some partial multi, or seen in two partials).  No global atomics, and the bitmaps need
// no clearing.
constexpr int kTrialThreads = 1024;
constexpr int64_t kTrialLdsWords = (int64_t)1 << 14;   // 2 x 64 KiB of LDS: up to 2^19 bins

template <typename K>
__global__ __launch_bounds__(kTrialThreads) void k_trial_hist_lds(const K* __restrict__ f, int64_t nf, int d,
                                                                  int64_t n, const int64_t* __restrict__ z,
                                                                  TrialRound tr, int fast, int64_t chunk,
                                                                  uint32_t* part, int64_t wstride) {
    extern __shared__ uint32_t th_lds[];
    const int i = blockIdx.y;
    const int64_t M = tr.M[i];
    const int words = (int)((M + 31) / 32);
    uint32_t* seen = th_lds;
    uint32_t* multi = th_lds + wstride;
    for (int w = threadIdx.x; w < words; w += kTrialThreads) {
        seen[w] = 0u;
        multi[w] = 0u;
    }
    __syncthreads();
    const int64_t g0 = (int64_t)blockIdx.x * chunk;
    const int64_t g1 = min(n, g0 + chunk);
    for (int64_t g = g0 + threadIdx.x; g < g1; g += kTrialThreads) {
        const int64_t s = dot_kz<K>(f, nf, d, g, z + (int64_t)i * d);
        const int64_t r = fast ? mod_fast(s, M, tr.invM[i]) : mod_exact(s, M);
        const uint32_t bit = 1u << (r & 31);
        const uint32_t old = atomicOr(&seen[r >> 5], bit);
        if (old & bit) atomicOr(&multi[r >> 5], bit);
    }
    __syncthreads();
    uint32_t* p = part + ((int64_t)i * gridDim.x + blockIdx.x) * 2 * wstride;
    for (int w = threadIdx.x; w < words; w += kTrialThreads) {
        p[w] = seen[w];
        p[wstride + w] = multi[w];
    }
}

// bitmaps of lattice blockIdx.y of the round (at bm + i 2 wstride) from its nchunks partials
__global__ __launch_bounds__(256) void k_trial_merge_round(const uint32_t* __restrict__ part, int nchunks,
                                                           TrialRound tr, uint32_t* bm, int64_t wstride) {
    constexpr int kChunk = 16;   // partials whose loads are in flight together
    const int i = blockIdx.y;
    const int64_t words = (tr.M[i] + 31) / 32;
    const uint32_t* p0 = part + (int64_t)i * nchunks * 2 * wstride;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < words; w += (int64_t)gridDim.x * blockDim.x) {
        uint32_t sa = 0u, ma = 0u;
        for (int c0 = 0; c0 < nchunks; c0 += kChunk) {
            uint32_t ps[kChunk], pm[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const int64_t c = min(c0 + u, nchunks - 1);   // clamped; repeats are not counted
                ps[u] = p0[c * 2 * wstride + w];
                pm[u] = p0[c * 2 * wstride + wstride + w];
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                if (c0 + u < nchunks) {
                    ma |= pm[u] | (sa & ps[u]);
                    sa |= ps[u];
                }
            }
        }
        bm[(int64_t)i * 2 * wstride + w] = sa;
        bm[(int64_t)i * 2 * wstride + wstride + w] = ma;
    }
}

// one pass over the frequencies: counts[i] = number covered once lattices 0..i of the round are
// added to the running union; covered becomes the union with all nk lattices
template <typename K>
__global__ __launch_bounds__(256) void k_trial_cover_round(const K* __restrict__ f, int64_t nf, int d, int64_t n,
                                                           const int64_t* __restrict__ z, TrialRound tr, int fast,
                                                           const uint32_t* __restrict__ bm, int64_t wstride,
                                                           uint8_t* covered, unsigned long long* counts) {
    __shared__ unsigned int part[kSpec][256];
    unsigned int local[kSpec];
#pragma unroll
    for (int i = 0; i < kSpec; ++i) local[i] = 0;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        int first = covered[g] ? 0 : kSpec;   // first lattice of the round after which g is covered
        if (first) {
            for (int i = 0; i < tr.nk; ++i) {
                const int64_t s = dot_kz<K>(f, nf, d, g, z + (int64_t)i * d);
                const int64_t r = fast ? mod_fast(s, tr.M[i], tr.invM[i]) : mod_exact(s, tr.M[i]);
                if (!((bm[(int64_t)i * 2 * wstride + wstride + (r >> 5)] >> (r & 31)) & 1u)) {
                    first = i;
                    break;
                }
            }
            if (first < tr.nk) covered[g] = 1;
        }
#pragma unroll
        for (int i = 0; i < kSpec; ++i) local[i] += first <= i;
    }
#pragma unroll
    for (int i = 0; i < kSpec; ++i) part[i][threadIdx.x] = local[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int i = 0; i < kSpec; ++i) part[i][threadIdx.x] += part[i][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < kSpec && (int)threadIdx.x < tr.nk) atomicAdd(counts + threadIdx.x, (unsigned long long)part[threadIdx.x][0]);
}

// any pair a < b with k_a = k_b componentwise mod p  ->  *found = 1
template <typename K>
__global__ void k_pairs_congruent(const K* __restrict__ f, int64_t nf, int d, int64_t n, int64_t p, int* found) {
    const int64_t pairs = n * (n - 1) / 2;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < pairs; q += (int64_t)gridDim.x * blockDim.x) {
        // row a of the strictly upper triangle: q = a n - a(a+1)/2 + (b - a - 1)
        int64_t a = (int64_t)((2.0 * n - 1.0 - sqrt((2.0 * n - 1.0) * (2.0 * n - 1.0) - 8.0 * (double)q)) / 2.0);
        if (a < 0) a = 0;
        while (a > 0 && a * n - a * (a + 1) / 2 > q) --a;
        while ((a + 1) * n - (a + 1) * (a + 2) / 2 <= q) ++a;
        const int64_t b = q - (a * n - a * (a + 1) / 2) + a + 1;
        bool same = true;
        for (int c = 0; c < d && same; ++c) {
            int64_t diff = (int64_t)f[c * nf + a] - (int64_t)f[c * nf + b];
            same = (diff % p) == 0;
        }
        if (same) atomicOr(found, 1);
    }
}

// ---- host helpers ----------------------------------------------------------------------------------
int64_t lmax_rule(int64_t n, double c, double gamma) { return host::lmax_rule(n, c, gamma); }

template <typename K>
static mr1l_status congruent_pair_exists(const void* f, int64_t nf, int d, int64_t n, int64_t p, bool* out,
                                         hipStream_t s) {
    DevMem flag;
    MR1L_HIP_TRY(flag.alloc(sizeof(int)));
    MR1L_HIP_TRY(hipMemsetAsync(flag.p, 0, sizeof(int), s));
    const int64_t pairs = n * (n - 1) / 2;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(16384, (pairs + 255) / 256));
    hipLaunchKernelGGL(k_pairs_congruent<K>, dim3(blocks), dim3(256), 0, s, (const K*)f, nf, d, n, p,
                       flag.as<int>());
    MR1L_HIP_TRY(hipGetLastError());
    int h = 0;
    MR1L_HIP_TRY(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    MR1L_HIP_TRY(hipStreamSynchronize(s));
    *out = h != 0;
    return MR1L_OK;
}

template <typename K>
static mr1l_status construct_t(int d, int64_t n, const void* f, int64_t maxabs, int64_t expansion, double c,
                               double gamma, int b, int redraw, uint64_t seed, int64_t t, hipStream_t s,
                               ConstructResult* out) {
    out->M.clear();
    out->z.clear();
    out->calls = 0;
    out->uncovered = 0;
    out->redraws = 0;
    if (n == 0) return MR1L_OK;
    const int64_t L_max = lmax_rule(n, c, gamma);
    const double lambda = c * (double)(n - 1);

    // P^I_{lambda, L_max}: the L_max smallest primes p > lambda with k -> k mod p injective on I
    std::vector<int64_t> primes;
    mr1l_status inj_status = MR1L_OK;
    auto injective = [&](int64_t p) -> int {
        if (p > expansion) return 1;   // distinct rows stay distinct modulo p
        if (n > 65536) {
            set_error("prime-size injectivity check needs |I| <= 65536 when lambda < expansion of I");
            inj_status = MR1L_ERR_UNSUPPORTED;
            return -1;
        }
        bool clash = false;
        inj_status = congruent_pair_exists<K>(f, n, d, n, p, &clash, s);
        return inj_status != MR1L_OK ? -1 : (clash ? 0 : 1);
    };
    if (host::prime_sizes(lambda, L_max, injective, primes) < 0) return inj_status;
    const int64_t maxM = primes.back();
    if (maxM >= ((int64_t)1 << 31)) {
        set_error("lattice sizes beyond 2^31 are not supported");
        return MR1L_ERR_UNSUPPORTED;
    }
    const long double bound = (long double)d * maxabs * maxM;
    if (bound >= 0x1.0p62L) {
        set_error("d * max|k| * max M >= 2^62");
        return MR1L_ERR_OVERFLOW;
    }
    const int fast = bound < 0x1.0p52L;

    DevMem bm, covered, count, zdev;
    const int64_t words = (maxM + 31) / 32;
    MR1L_HIP_TRY(bm.alloc(2 * words * sizeof(uint32_t)));
    MR1L_HIP_TRY(covered.alloc((size_t)n));
    MR1L_HIP_TRY(count.alloc(sizeof(unsigned long long)));
    MR1L_HIP_TRY(zdev.alloc((size_t)d * sizeof(int64_t)));
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256));

    if (redraw == 0) {
        // Alg. 1 itself: lattices L, L+1, ... are tried kSpec at a time with one host
        // synchronisation.  Each draw depends only on its own stream key (t, call, L) and the
        // coverage after every lattice is recorded, so keeping the lattices up to the first that
        // completes the coverage (the later ones are discarded) is exactly the sequential result.
        // one buffer per round, cleared by one memset: the kSpec coverage counts, then the alias
        // bitmaps of the round's lattices
        DevMem zk_dev, round, part;
        MR1L_HIP_TRY(zk_dev.alloc((size_t)kSpec * d * sizeof(int64_t)));
        MR1L_HIP_TRY(round.alloc((size_t)kSpec * sizeof(unsigned long long) + (size_t)kSpec * 2 * words * sizeof(uint32_t)));
        unsigned long long* counts = round.as<unsigned long long>();
        uint32_t* bmr = (uint32_t*)(counts + kSpec);
        // LDS histograms where the bitmaps fit: chunks of at least 4096 frequencies, about 256
        // workgroups per round
        const bool lds = words <= kTrialLdsWords;
        int chunks = 1;
        int64_t chunk = n;
        const size_t lds_bytes = 2 * (size_t)words * sizeof(uint32_t);
        if (lds) {
            chunks = (int)std::min<int64_t>(std::max<int64_t>(1, (n + 4095) / 4096), std::max(1, 256 / kSpec));
            chunk = (n + chunks - 1) / chunks;
            MR1L_HIP_TRY(part.alloc((size_t)kSpec * chunks * 2 * words * sizeof(uint32_t)));
            if (lds_bytes > 65536)
                MR1L_HIP_TRY(hipFuncSetAttribute((const void*)k_trial_hist_lds<K>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
        }
        const unsigned merge_x = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (words + 255) / 256));
        std::vector<int64_t> zk((size_t)kSpec * d);
        unsigned long long hc[kSpec];
        for (int call = 0; call < std::max(1, b); ++call) {
            out->M.clear();
            out->z.clear();
            out->calls = call + 1;
            MR1L_HIP_TRY(hipMemsetAsync(covered.p, 0, (size_t)n, s));
            unsigned long long ncov = 0;
            bool done = false;
            for (int64_t L = 1; L <= L_max && !done; L += kSpec) {
                TrialRound tr{};
                tr.nk = (int)std::min<int64_t>(kSpec, L_max - L + 1);
                for (int i = 0; i < tr.nk; ++i) {
                    const int64_t M = primes[L + i - 1];
                    tr.M[i] = M;
                    tr.invM[i] = 1.0 / (double)M;
                    const uint64_t key = Rng::key(seed, {Rng::Z, t, call, L + i});
                    uint64_t ctr = 0;
                    for (int c = 0; c < d; ++c) zk[(size_t)i * d + c] = (int64_t)Rng::uniform_int(key, &ctr, (uint64_t)M);
                }
                MR1L_HIP_TRY(hipMemcpyAsync(zk_dev.p, zk.data(), (size_t)tr.nk * d * sizeof(int64_t),
                                            hipMemcpyHostToDevice, s));
                if (lds) {
                    MR1L_HIP_TRY(hipMemsetAsync(round.p, 0, (size_t)kSpec * sizeof(unsigned long long), s));
                    hipLaunchKernelGGL(k_trial_hist_lds<K>, dim3(chunks, tr.nk), dim3(kTrialThreads), lds_bytes, s,
                                       (const K*)f, n, d, n, zk_dev.as<int64_t>(), tr, fast, chunk, part.as<uint32_t>(),
                                       words);
                    hipLaunchKernelGGL(k_trial_merge_round, dim3(merge_x, tr.nk), dim3(256), 0, s,
                                       (const uint32_t*)part.p, chunks, tr, bmr, words);
                } else {
                    MR1L_HIP_TRY(hipMemsetAsync(round.p, 0, (size_t)kSpec * sizeof(unsigned long long) +
                                                                (size_t)tr.nk * 2 * words * sizeof(uint32_t), s));
                    hipLaunchKernelGGL(k_trial_hist_round<K>, dim3(blocks, tr.nk), dim3(256), 0, s, (const K*)f, n, d,
                                       n, zk_dev.as<int64_t>(), tr, fast, bmr, words);
                }
                hipLaunchKernelGGL(k_trial_cover_round<K>, dim3(blocks), dim3(256), 0, s, (const K*)f, n, d, n,
                                   zk_dev.as<int64_t>(), tr, fast, (const uint32_t*)bmr, words,
                                   covered.as<uint8_t>(), counts);
                MR1L_HIP_TRY(hipGetLastError());
                MR1L_HIP_TRY(hipMemcpyAsync(hc, counts, (size_t)tr.nk * sizeof(unsigned long long),
                                            hipMemcpyDeviceToHost, s));
                MR1L_HIP_TRY(hipStreamSynchronize(s));
                for (int i = 0; i < tr.nk; ++i) {
                    out->M.push_back(primes[L + i - 1]);
                    out->z.insert(out->z.end(), zk.begin() + (size_t)i * d, zk.begin() + (size_t)(i + 1) * d);
                    ncov = hc[i];
                    if ((int64_t)ncov == n) {
                        done = true;
                        break;
                    }
                }
            }
            out->uncovered = n - (int64_t)ncov;
            if (out->uncovered == 0) break;
        }
        return MR1L_OK;
    }

    std::vector<int64_t> zl(d);
    for (int call = 0; call < std::max(1, b); ++call) {
        out->M.clear();
        out->z.clear();
        out->calls = call + 1;
        MR1L_HIP_TRY(hipMemsetAsync(covered.p, 0, (size_t)n, s));
        unsigned long long ncov = 0;
        for (int64_t L = 1; L <= L_max; ++L) {
            const int64_t M = primes[L - 1];
            const unsigned long long before = ncov;
            for (int a = 0;; ++a) {
                // draw a = 0: the Z stream of Alg. 1; a >= 1: redraws of the variant
                const uint64_t key = a == 0 ? Rng::key(seed, {Rng::Z, t, call, L})
                                            : Rng::key(seed, {Rng::ZREDRAW, t, call, L, a});
                uint64_t ctr = 0;
                for (int i = 0; i < d; ++i) zl[i] = (int64_t)Rng::uniform_int(key, &ctr, (uint64_t)M);
                const int64_t w = (M + 31) / 32;
                MR1L_HIP_TRY(hipMemcpyAsync(zdev.p, zl.data(), d * sizeof(int64_t), hipMemcpyHostToDevice, s));
                MR1L_HIP_TRY(hipMemsetAsync(bm.p, 0, 2 * w * sizeof(uint32_t), s));
                MR1L_HIP_TRY(hipMemsetAsync(count.p, 0, sizeof(unsigned long long), s));
                hipLaunchKernelGGL(k_trial_hist<K>, dim3(blocks), dim3(256), 0, s, (const K*)f, n, d, n,
                                   zdev.as<int64_t>(), M, 1.0 / (double)M, fast, bm.as<uint32_t>(), w);
                // covered only grows by this lattice's unaliased frequencies; a lattice that adds
                // none leaves it unchanged, so a rejected draw needs no undo
                hipLaunchKernelGGL(k_trial_cover<K>, dim3(blocks), dim3(256), 0, s, (const K*)f, n, d, n,
                                   zdev.as<int64_t>(), M, 1.0 / (double)M, fast, (const uint32_t*)bm.p, w,
                                   covered.as<uint8_t>(), count.as<unsigned long long>());
                MR1L_HIP_TRY(hipGetLastError());
                MR1L_HIP_TRY(hipMemcpyAsync(&ncov, count.p, sizeof(ncov), hipMemcpyDeviceToHost, s));
                MR1L_HIP_TRY(hipStreamSynchronize(s));
                if (ncov > before || a >= redraw) break;
                ++out->redraws;
            }
            out->M.push_back(M);
            out->z.insert(out->z.end(), zl.begin(), zl.end());
            if ((int64_t)ncov == n) break;
        }
        out->uncovered = n - (int64_t)ncov;
        if (out->uncovered == 0) break;
    }
    return MR1L_OK;
}

mr1l_status construct_lattices(int d, int64_t n, const int32_t* host_freqs, const void* dev_freqs, int ktype,
                               int64_t maxabs, int64_t expansion, double c, double gamma, int b, int redraw,
                               uint64_t seed, int64_t t, int device, hipStream_t s, ConstructResult* out) {
    MR1L_HIP_TRY(hipSetDevice(device));
    DevMem packed;
    const void* f = dev_freqs;
    if (host_freqs) {
        maxabs = 0;
        expansion = 0;
        for (int c0 = 0; c0 < d; ++c0) {
            int64_t lo = INT64_MAX, hi = INT64_MIN;
            for (int64_t g = 0; g < n; ++g) {
                const int64_t v = host_freqs[g * d + c0];
                lo = std::min(lo, v);
                hi = std::max(hi, v);
                maxabs = std::max<int64_t>(maxabs, std::llabs(v));
            }
            if (n) expansion = std::max(expansion, hi - lo);
        }
        ktype = K_I32;
        std::vector<int32_t> soa((size_t)n * d);
        for (int64_t g = 0; g < n; ++g)
            for (int c0 = 0; c0 < d; ++c0) soa[(size_t)c0 * n + g] = host_freqs[g * d + c0];
        MR1L_HIP_TRY(packed.upload(soa.data(), soa.size() * sizeof(int32_t)));
        f = packed.p;
    }
    switch (ktype) {
        case K_I8: return construct_t<int8_t>(d, n, f, maxabs, expansion, c, gamma, b, redraw, seed, t, s, out);
        case K_I16: return construct_t<int16_t>(d, n, f, maxabs, expansion, c, gamma, b, redraw, seed, t, s, out);
        default: return construct_t<int32_t>(d, n, f, maxabs, expansion, c, gamma, b, redraw, seed, t, s, out);
    }
}

}  // namespace mr1l

using namespace mr1l;

extern "C" mr1l_status mr1l_construct(int d, int64_t n, const int32_t* freqs, double c, double gamma, int b,
                                      int redraw, uint64_t seed, int64_t t, int L_cap, int* L_out, int64_t* M,
                                      int64_t* z, int* calls, int64_t* n_uncovered, int device) {
    try {
        clear_error();
        if (d < 1 || d > 64 || n < 0 || (n > 0 && !freqs) || !(c > 1.0) || !(gamma > 0.0 && gamma < 1.0) || b < 1 ||
            redraw < 0 || !L_out || L_cap < 0 || (L_cap > 0 && (!M || !z))) {
            set_error("invalid argument to mr1l_construct");
            return MR1L_ERR_ARG;
        }
        ConstructResult r;
        mr1l_status st = construct_lattices(d, n, freqs, nullptr, K_I32, 0, 0, c, gamma, b, redraw, seed, t,
                                            device, nullptr, &r);
        if (st != MR1L_OK) return st;
        const int L = (int)r.M.size();
        *L_out = L;
        if (calls) *calls = r.calls;
        if (n_uncovered) *n_uncovered = r.uncovered;
        if (L > L_cap) {
            set_error("L_cap too small: need " + std::to_string(L));
            return MR1L_ERR_ARG;
        }
        std::copy(r.M.begin(), r.M.end(), M);
        std::copy(r.z.begin(), r.z.end(), z);
        return r.uncovered ? MR1L_WARN_UNCOVERED : MR1L_OK;
    } catch (const std::exception& e) {
        set_error(e.what());
        return MR1L_ERR_ARG;
    }
}
