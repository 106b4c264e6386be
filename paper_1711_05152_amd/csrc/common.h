// Internal declarations shared by the HIP kernels and the host runtime of libmr1l.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace mr1l {

// ---- complex arithmetic ---------------------------------------------------------------------------
template <typename T>
struct cx {
    T x, y;
};

template <typename T>
__host__ __device__ inline cx<T> make_cx(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ inline cx<T> cmul(cx<T> a, cx<T> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename T>
__device__ inline cx<T> cmulc(cx<T> a, cx<T> b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }  // a * conj(b)
template <typename T>
__device__ inline cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ inline cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }

// e^{i pi x} from an exactly representable argument (x given in double).
__device__ inline void sincospi_d(double x, double* s, double* c) { sincospi(x, s, c); }

// ---- lattice descriptors ---------------------------------------------------------------------------
// One entry per rank-1 lattice of a transform.  All offsets are in elements.
struct LatDesc {
    int64_t M;         // lattice size M_l
    int64_t samp_off;  // first sample of lattice l inside one right-hand side
    int64_t work_off;  // first element of its Bluestein work region (length N, bl_len) per rhs
    int64_t filt_off;  // first element of its filter spectrum (length N)
    int64_t bm_off;    // first 32-bit word of its alias bitmaps: seen [bm_words] then multi [bm_words]
    int64_t bm_words;  // ceil(M / 32)
    int64_t zoff;      // first component of z_l in the generating-vector table
    double invM;       // 1 / M
    int32_t lgN;       // Bluestein length N = 2^lgN, or 3 * 2^lgN when n3, N >= 2M - 1
    int32_t lgN1;      // four-step split: N = 2^lgN1 * N2, N2 = 2^lgN2 or 3 * 2^lgN2 (lgN1 = 0 on
    int32_t lgN2;      //   the one-block path)
    int32_t small;     // 1: the whole Bluestein convolution runs in one workgroup
    int32_t rt0;       // fused residue/histogram pass: first ResTile of this lattice
    int32_t rtn;       //   and their number
    int32_t tx;        // transform the lattice belongs to
    int32_t n3;        // 1: N = 3 * 2^lgN (the factor 3 sits in the stage-2 rows)
};
__host__ __device__ inline int64_t bl_len(const LatDesc& D) { return (int64_t)(D.n3 ? 3 : 1) << D.lgN; }

// One entry per independent transform of a plan (a plain plan has one; a batched plan many).
// Its frequencies are [foff, foff + fn) of the plan's frequency table and of every coefficient
// vector; its lattices are [lat0, lat0 + nlat) of the descriptor table.
struct TxDesc {
    int64_t foff;
    int64_t fn;
    int32_t lat0;
    int32_t nlat;
    int32_t in_block;  // 1: the persistent small-transform kernel does this transform's forward and
    int32_t pad_;      //    adjoint in one workgroup; the FFT stages, the gather and the scatter skip it
};

// One workgroup of the alias-histogram pass: lattice l, bins [m0, m1) (multiples of 32 except
// possibly m1 = M), of transform tx.
struct HistTile {
    int32_t l;
    int32_t tx;
    int32_t m0;
    int32_t m1;
};
constexpr int kHistMaxBins = 1 << 18;   // 2 x 2^18 bits = 64 KiB of LDS bitmaps per workgroup

// One workgroup of the fused residue + alias-histogram pass: frequencies [k0, k1) of transform tx
// against lattice l, counted into LDS bitmaps over all M_l bins; the workgroup's partial bitmaps
// (seen then multi, bm_words each) go to word offset part of the partial-bitmap area.
struct ResTile {
    int64_t k0, k1, part;
    int32_t l, tx;
};
constexpr int kFusedMaxWords = 1 << 14;   // bitmaps of up to 2^19 bins (2 x 64 KiB of LDS)
constexpr int kResThreads = 1024;         // threads of a fused-pass workgroup
// residues per thread and iteration of the fused pass for padded width DP (0: 64-bit path), all
// their component loads in flight together within the 128 VGPRs of a 1024-thread workgroup; a
// ResTile holds kResThreads * res_unroll(DP) frequencies, one iteration
__host__ __device__ constexpr int res_unroll(int dp) {
    return dp == 0 ? 4 : (dp <= 8 ? 8 : (dp <= 12 ? 6 : (dp <= 16 ? 4 : 2)));
}

// Frequencies are kept component-major (structure of arrays) in the narrowest signed integer
// type that holds them.
enum KType { K_I8 = 0, K_I16 = 1, K_I32 = 2 };

constexpr int kThreads = 256;      // threads per workgroup of every FFT kernel
constexpr int kSmallMaxLg = 12;    // one-block Bluestein up to 2^12 points
constexpr int kMaxLgN = 24;        // largest Bluestein length 2^24 (M_l < 2^23)
constexpr int kTwLg = 12;          // twiddle table e^{-2 pi i m / 4096}, m < 4096
constexpr int kTileLg = 12;        // elements of one four-step tile (fp32 32 KiB, fp64 64 KiB of LDS)

// Four-step split 2^lgN = 2^lgN1 * 2^lgN2 for lgN > kSmallMaxLg: rows of stage 2 at most 2^12
// long, and at least 16 columns per stage-1/3 tile so every column segment spans >= 128 bytes.
__host__ __device__ constexpr int split_lgN1(int lgN) {
    return (lgN - kTileLg) > ((lgN / 2) < (kTileLg - 4) ? (lgN / 2) : (kTileLg - 4))
               ? (lgN - kTileLg)
               : ((lgN / 2) < (kTileLg - 4) ? (lgN / 2) : (kTileLg - 4));
}

// Splits compiled for each length: the rule above and its neighbours lgN1 - 1 and lgN1 + 1 where
// both factors have 2^4 .. 2^12 points (stage-2 rows fit one tile).  Plans take the split of
// their Bluestein lengths from the measured schedule table (fft_schedule.hip, mr1l_fft_split).
__host__ __device__ constexpr bool split_ok(int lgN, int lgN1) {
    return lgN1 >= 4 && lgN - lgN1 >= 4 && lgN1 <= kTileLg && lgN - lgN1 <= kTileLg;
}
__host__ __device__ constexpr bool split_compiled(int lgN, int lgN1) {
    return lgN > kSmallMaxLg && lgN <= kMaxLgN && split_ok(lgN, lgN1) && lgN1 >= split_lgN1(lgN) - 1 &&
           lgN1 <= split_lgN1(lgN) + 1;
}
int fft_split(int dtype, int lgN);   // split plans of this dtype use for Bluestein length 2^lgN

// Bluestein lengths N = 3 * 2^lgN (lgN in [kMinLg3, kMaxLg3]) take the place of 2^(lgN + 2) for the
// lattices of a transform in that class when all of them have 2M - 1 <= N (in large transforms:
// each lattice that does): 25 % fewer points.  Their split puts the factor 3 into the stage-2 rows,
// N = 2^lgN1 * 3 * 2^(lgN - lgN1), with one compiled split per length: rows of at most 3 * 2^10
// points (3 * 2^11-point rows left two workgroups per CU in stage 2) and at least 16 columns per
// stage-1/3 tile where the length allows.
constexpr int kMinLg3 = 12, kMaxLg3 = 22;
constexpr int kGroupStreams = 3;   // extra streams of a plan for concurrent Bluestein groups
__host__ __device__ constexpr int split3_lgN1(int lgN) {
    return (lgN - 10) > ((lgN + 1) / 2 < 8 ? (lgN + 1) / 2 : 8) ? (lgN - 10) : ((lgN + 1) / 2 < 8 ? (lgN + 1) / 2 : 8);
}
// plans of this dtype created now may turn the power-of-two class 2^lg into 3 * 2^(lg - 2)
bool fft_smooth_class(int dtype, int lg);

// Radix schedules of the register-resident tile DFTs (stage i of a 2^lgn-point DFT has radix
// 2^stage_lr(lgn, i, ord)).  Every thread holds 2^ord_lgv(ord) values of a tile: 16 (radix up to
// 16, ceil(lgn/4) stages) or 8 (radix up to 8, ceil(lgn/3) stages, twice the threads);
//   ord 0 / 1  16 values, bits spread evenly, radices descending (0) or ascending (1);
//   ord 2 / 3  16 values, radix 16 in every stage but one, which takes the remaining bits, last (2)
//              or first (3);
//   ord 4 / 5  8 values, bits spread evenly, descending (4) or ascending (5).
// A forward DFT with an ascending order and an inverse with the matching descending one meet at
// stages of the same radix (1024 = 8 8 16 | 16 8 8, 4 16 16 | 16 16 4, or 4 4 8 8 | 8 8 4 4).
constexpr int ord_lgv(int ord) { return ord >= 4 ? 3 : 4; }
constexpr int n_stages(int lgn, int ord = 0) { return (lgn + ord_lgv(ord) - 1) / ord_lgv(ord); }
constexpr int stage_lr(int lgn, int i, int ord) {
    if (ord == 2 || ord == 3) {
        const int rem = lgn - 4 * (n_stages(lgn, ord) - 1);
        return i == (ord == 3 ? 0 : n_stages(lgn, ord) - 1) ? rem : 4;
    }
    const int ns = n_stages(lgn, ord);
    return (ord == 1 || ord == 5) ? (i >= ns - lgn % ns ? lgn / ns + 1 : lgn / ns)
                                  : (i < lgn % ns ? lgn / ns + 1 : lgn / ns);
}
constexpr int stage_lgns(int lgn, int i, int ord) {
    int s = 0;
    for (int k = 0; k < i; ++k) s += stage_lr(lgn, k, ord);
    return s;
}
// the radix-16-major schedule gives different radices than the even one for this length
constexpr bool schedules_differ(int lgn) {
    for (int i = 0; i < n_stages(lgn, 1); ++i)
        if (stage_lr(lgn, i, 1) != stage_lr(lgn, i, 3)) return true;
    return false;
}

// Stage 2 takes 2048-element tiles for rows of up to 2^10 points, else 4096.  Its variants, which
// the autotuner chooses from per length: bit 0, radix orders 3 / 2 instead of 1 / 0 for the forward
// / inverse row DFTs; bit 1, 4096-element tiles also for the shorter rows; bit 2, 8 values per
// thread (orders 5 / 4, twice the threads per tile; not combined with bit 0).  A variant is
// compiled only where it changes the kernel.
constexpr int kP2TileLg = 11;
constexpr bool p2_variant_compiled(int lgN, int lg1, int v) {
    return v >= 0 && v <= 6 && !((v & 4) && (v & 1)) && (!(v & 1) || schedules_differ(lgN - lg1)) &&
           (!(v & 2) || lgN - lg1 + 1 <= kP2TileLg);
}
constexpr int kP2Variants = 7;
int fft_p2_variant(int dtype, int lgN, int lg1);   // the variant plans use for that length and split

// Lattices sharing one Bluestein length, launched together with kernels specialised for it.
struct FftGroup {
    int lgN;
    int n3;           // 1: length 3 * 2^lgN
    int lg1;          // four-step split N = 2^lg1 * N / 2^lg1 (0 on the one-block path)
    int p2v;          // stage-2 variant (radix schedule, tile size) the autotuner chose
    int small;        // one-block path (lgN <= kSmallMaxLg)
    int nlat;
    const int* lat;   // device [nlat] lattice indices
};

// ---- launchers (defined in the .hip files) ---------------------------------------------------------
struct FreqView {
    const void* f;   // component-major [d][nf]
    int ktype;
    int d;
    int64_t nf;      // stride between components
};

// Transform launch context shared by the stage launchers.
struct TxArgs {
    const LatDesc* desc;      // device [L]
    int L;
    const TxDesc* tx;         // device [ntx]
    const int64_t* tx_foff;   // device [ntx + 1] frequency prefix sums (binary search)
    int ntx;
    int max_nlat;             // largest lattice count of one transform
    const int64_t* z;         // device generating vectors
    FreqView fv;
    int64_t n;                // frequencies of all transforms = coefficients per rhs
    int64_t n_rhs;
    int64_t samp_stride;      // elements per rhs in the sample vector
    int64_t work_stride;      // elements per rhs in the work area
    uint32_t* bitmaps;        // device alias bitmaps
    int64_t bm_total;         // words of all bitmaps
    int32_t* res32;           // device residues [max_nlat][rs] (slot = lattice index within its transform)
    int64_t rs;               // row stride of res32: n rounded up to a multiple of 4 (16-byte rows)
    const HistTile* hist;     // device [nhist] (l = -1: idle slot of the XCD-interleaved order)
    int nhist;
    int hist_words;           // largest bitmap words of one tile (LDS per bitmap)
    // fused residue + histogram pass (every lattice has at most kFusedMaxWords bitmap words)
    bool fused;
    const ResTile* rtiles;    // device [nrt]
    int nrt;
    int rt_words;             // largest bm_words over the lattices (LDS per bitmap)
    uint32_t* part;           // partial bitmaps of every ResTile
    // Fourier-matrix adjoint by counting sort (bsort): per bin (lattice-major like the samples)
    // the number of frequencies it receives (zero between calls), chunk-local exclusive scans and
    // chunk bases of the concatenated counts, and per lattice slot the frequencies ordered by bin
    bool bsort;
    int32_t* bcnt;            // [sum_M]
    int32_t* bloc;            // [sum_M]
    int32_t* bbase;           // [ceil(sum_M / kScanChunk)]
    int32_t* perm;            // [max_nlat][rs]
    int64_t nbins;            // sum_M
    int64_t max_M;            // largest lattice size
    // right-hand-side interleaving buffer of max(n, sum_M) 64-byte slots (null: not used), and
    // whether the gather (bins) and the bin sums (coefficients) go through it
    void* ilv;
    bool ilv_bins, ilv_coef;
    bool fast_mod;            // residues may use the fp64 quotient estimate
    // 32-bit residue path: |k . z| < 2^31 for every frequency and lattice, |k_c| < 2^23 and d <= 32;
    // z32 holds the reduced generators as int32 rows padded with zeros
    bool narrow;
    int zpad;                 // 8, 12, 16, 24 or 32: components the residue kernels multiply
    int zrow;                 // row stride of z32 (16 or 32)
    const int32_t* z32;
};

// Interleaving a pass's right-hand sides pays where its random reads leave the caches: the
// gather's bins beyond the 256 MB Infinity Cache (inside it the copy costs more than the reads it
// saves), the bin sums' coefficients beyond a 4 MB L2.
constexpr int64_t kIlvBinBytes = (int64_t)1 << 28;
constexpr int64_t kIlvCoefBytes = (int64_t)1 << 22;

template <typename T> const cx<T>* twiddles(int device);   // e^{-2 pi i m/4096}, m < 4096

void launch_clear_u32(uint32_t* p, int64_t words, hipStream_t s);
// residues of every (lattice, frequency) into res32, then (if histogram) the per-lattice 2-bit
// alias histograms (LDS atomics, one workgroup per HistTile) written to the global bitmaps
void launch_alias(const TxArgs& a, bool histogram, hipStream_t s);
template <typename T>
void launch_gather(const TxArgs& a, const cx<T>* work, cx<T>* coeffs, bool eval, hipStream_t s);
template <typename T>
void launch_clear_bins(const TxArgs& a, cx<T>* work, hipStream_t s);   // Fourier-matrix adjoint only
template <typename T>
void launch_scatter(const TxArgs& a, const cx<T>* coeffs, cx<T>* work, bool eval, hipStream_t s);
constexpr int kScanChunk = 8192;   // bins per workgroup of the counting-sort scan
// counting sort of every (frequency, lattice) pair by bin (needs the residues); then, per rhs
// chunk, bins[m] = sum of c_k over the frequencies in bin m (Fourier-matrix adjoint, no atomics)
void launch_bin_sort(const TxArgs& a, hipStream_t s);
template <typename T>
void launch_bin_sum(const TxArgs& a, const cx<T>* coeffs, cx<T>* work, hipStream_t s);
void launch_alias_export(const TxArgs& a, int64_t* res, uint8_t* uniq, uint8_t* counter, hipStream_t s);

// Bluestein stages for one group of lattices.  sign = -1: DFT with e^{-2 pi i jm/M} (forward),
// +1: with e^{+...} (adjoint).  src: samples, or the bins already in the work area.
template <typename T>
void launch_bluestein_small(const TxArgs& a, const FftGroup& g, const cx<T>* src, int64_t src_stride,
                            bool src_is_samples, cx<T>* work, const cx<T>* filt, cx<T>* dst, int64_t dst_stride,
                            bool dst_is_samples, int sign, bool scale_by_invM, bool mask_bins, hipStream_t s);
// mask_bins: the bins in the work area are valid only where the alias bitmaps mark them as holding
// exactly one frequency (adjoint of Alg. 2); the others are read as zero
template <typename T>
void launch_p1(const TxArgs& a, const FftGroup& g, const cx<T>* src, int64_t src_stride, bool src_is_samples,
               cx<T>* work, int sign, bool mask_bins, hipStream_t s);
// rot_in / rot_out: the sample vector whose column rotation the rows carry when loaded (forward,
// after stage 1 read samples) or must carry when stored (adjoint, before stage 3 writes samples);
// NULL for none
template <typename T>
void launch_p2(const TxArgs& a, const FftGroup& g, cx<T>* work, const cx<T>* filt, int sign, const cx<T>* rot_in,
               const cx<T>* rot_out, hipStream_t s);
template <typename T>
void launch_p3(const TxArgs& a, const FftGroup& g, cx<T>* work, cx<T>* dst, int64_t dst_stride, bool dst_is_samples,
               int sign, bool scale_by_invM, hipStream_t s);

// Persistent small-transform kernel of batched plans (Alg. 2 and its adjoint, weights of Alg. 2):
// one workgroup takes a whole transform from a work queue (list[0 .. nlist), transforms whose
// lattices all have one-block Bluestein lengths and at most kFusedTxMaxN frequencies), computes
// residues and alias bitmaps in LDS, runs each lattice's prime-length DFT in LDS and averages
// (forward) or scatters and transforms back (adjoint), and takes the next transform until the queue
// is empty.  queue: two device ints, zero before the launch and zero again after it (the last
// workgroup to finish resets them), so a captured graph can replay the launch.
constexpr int kFusedTxMaxN = 2048;
template <typename T>
void launch_fused_small(const TxArgs& a, const int* list, int nlist, int* queue, const cx<T>* src, cx<T>* dst,
                        const cx<T>* filt, bool forward, hipStream_t s);

// Filter spectra: filt_l = DFT_{2^lgN}(b_l) / 2^lgN with b_l[n] = e^{+i pi n^2 / M_l} for |n| < M_l
// (wrapped), stored in the layout stage 2 reads (natural order on the one-block path,
// [k1][k2] = B[k1 + N1 k2] on the four-step path).
template <typename T>
hipError_t build_filters(const LatDesc* hdesc, int L, const LatDesc* ddesc, const std::vector<FftGroup>& groups,
                         cx<T>* filt, int device, hipStream_t s);

}  // namespace mr1l
