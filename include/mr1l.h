/*
 * mr1l.h -- C ABI of the MI355X multiple rank-1 lattice FFT and the dimension-incremental sparse
 * FFT built on it (Kaemmerer, Potts, Volkmer, "High-dimensional sparse FFT based on sampling along
 * multiple rank-1 lattices", arXiv 1711.05152).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Frequencies are int32 rows k in Z^d, row-major [n][d], host memory.
 * - A multiple rank-1 lattice is L pairs (M_l, z_l), M_l >= 1, z_l in Z^d (any integers; they are
 *   reduced modulo M_l).  Its samples are stored lattice after lattice: lattice l owns entries
 *   [off_l, off_l + M_l) of a vector of length sum_l M_l, and entry j of that slice is the value
 *   at the node (j z_l / M_l) mod 1 (definition of Lambda(z, M), Sec. 2.1).
 * - Complex data are interleaved (re, im) pairs: MR1L_C64 = two floats, MR1L_C128 = two doubles.
 *   Multi right-hand-side data are [n_rhs][...] with the rhs index slowest.
 * - Device pointers are HIP device memory on the plan's device; ``stream`` is a hipStream_t (or
 *   NULL for the default stream).  Transform calls only enqueue work on that stream and return;
 *   they never synchronize.  The caller owns every buffer passed in.
 * - Every entry point returns a status and never aborts.  Arguments are validated before any
 *   work is enqueued; on error nothing is launched and mr1l_last_error() describes the problem
 *   (thread-local, valid until the next call on the same thread).
 * - A plan is bound to one device and must not be used by two host threads at once; calls on
 *   one plan must be ordered on one stream (the plan owns one scratch area).
 */
#ifndef MR1L_H
#define MR1L_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mr1l_status {
    MR1L_OK = 0,
    MR1L_ERR_ARG = 1,          /* invalid argument (sizes, pointers, duplicate frequencies ...) */
    MR1L_ERR_OVERFLOW = 2,     /* d * max|k| * max M_l >= 2^62 (exact int64 residues)         */
    MR1L_ERR_NOMEM = 3,        /* device or host allocation failed                              */
    MR1L_ERR_HIP = 4,          /* a HIP runtime call or kernel launch failed                    */
    MR1L_ERR_CALLBACK = 5,     /* the user sampler returned non-zero                            */
    MR1L_ERR_UNSUPPORTED = 6,  /* valid but outside this build's limits (e.g. M_l >= 2^23)      */
    MR1L_WARN_UNCOVERED = 16   /* result defined, but some frequency lies in no I_l            */
} mr1l_status;

typedef enum mr1l_dtype { MR1L_C64 = 0, MR1L_C128 = 1 } mr1l_dtype;

/* Weighting of the transform pair.
 * MR1L_W_PAPER -- Alg. 2 (inverse multiple rank-1 lattice FFT):
 *   forward  c_k = (1/counter_k) sum_{l: k in I_l} (1/M_l) sum_j y_l[j] e^{-2 pi i j (k.z_l)/M_l}
 *            with I_l = { k in I : no h != k in I has h.z_l = k.z_l (mod M_l) } and
 *            counter_k = #{l : k in I_l};  c_k = 0 when counter_k = 0.
 *   adjoint  y_l[j] = (1/M_l) sum_{k in I_l} (c_k/counter_k) e^{+2 pi i j (k.z_l)/M_l}
 *            (the exact adjoint of the forward map).
 * MR1L_W_EVAL -- the Fourier matrix A(X, I) = (e^{2 pi i k.x})_{x in X, k in I} of Sec. 2.1 on the
 *   stacked lattice nodes:  adjoint computes y = A c (synthesis, every k, colliding residues
 *   summed), forward computes A^* y = sum_l DFT_{M_l}(y_l)[k.z_l mod M_l] (no 1/M_l, every l). */
typedef enum mr1l_weights { MR1L_W_PAPER = 0, MR1L_W_EVAL = 1 } mr1l_weights;

typedef struct mr1l_plan_s* mr1l_plan_t;

/* Build a transform plan (Alg. 2, inputs I and Lambda; Sec. 2.1 for the lattice definition).
 *   d, n        dimension (1..64) and number of frequencies (n >= 0)
 *   freqs       host int32 [n][d], pairwise distinct rows (checked)
 *   L, M, z     host int64 [L] lattice sizes (1 <= M_l < 2^23) and [L][d] generating vectors
 *   dtype       precision of samples, coefficients and arithmetic
 *   weights     MR1L_W_PAPER or MR1L_W_EVAL (see above)
 *   n_rhs       number of right-hand sides transformed per call (>= 1)
 *   device      HIP device index the plan lives on
 *   out         receives the plan; released with mr1l_destroy
 * The plan allocates its device scratch (packed frequencies, alias bitmaps, Bluestein filter
 * spectra, work area) and computes the filter spectra on the device; it synchronizes the device
 * before returning.  Residues are exact: the int64 dot products k.z_l never overflow because the
 * plan rejects d * max|k| * max M_l >= 2^62 (MR1L_ERR_OVERFLOW; unreachable with int32 k,
 * d <= 64 and M_l < 2^23).  Errors: MR1L_ERR_ARG (bad sizes/pointers, duplicate rows),
 * MR1L_ERR_OVERFLOW, MR1L_ERR_UNSUPPORTED (M_l >= 2^23), MR1L_ERR_NOMEM, MR1L_ERR_HIP.
 * The Bluestein work area is bounded (4 GiB); larger n_rhs are processed in chunks of
 * right-hand sides within one call. */
mr1l_status mr1l_plan(int d, int64_t n, const int32_t* freqs, int L, const int64_t* M,
                      const int64_t* z, mr1l_dtype dtype, mr1l_weights weights, int64_t n_rhs,
                      int device, mr1l_plan_t* out);

/* Batched plan: n_tx independent transforms in one plan (each with its own frequency set and its
 * own lattices, Alg. 2 applied to each), executed by the same few kernel launches per call.
 *   n         host int64 [n_tx]: frequencies of transform b
 *   freqs     host int32 [sum n][d]: the frequency sets one after another
 *   L         host int32 [n_tx]: lattices of transform b
 *   M, z      host int64 [sum L] and [sum L][d]: the lattices one transform after another
 * Samples of one right-hand side are all lattices of all transforms one after another
 * (transform-major); coefficients are all frequencies one after another.  Everything else as in
 * mr1l_plan; mr1l_forward / mr1l_adjoint / mr1l_alias / mr1l_info accept batched plans (the alias
 * export uses rows [j][sum n] for the j-th lattice of each frequency's own transform). */
mr1l_status mr1l_plan_batched(int d, int n_tx, const int64_t* n, const int32_t* freqs, const int32_t* L,
                              const int64_t* M, const int64_t* z, mr1l_dtype dtype, mr1l_weights weights,
                              int64_t n_rhs, int device, mr1l_plan_t* out);

/* Forward transform (Alg. 2; the residues k.z_l mod M_l, the alias histograms, the prime-length
 * DFTs and the gather are all recomputed on every call).
 *   samples  device [n_rhs][sum_l M_l] complex (read only)
 *   coeffs   device [n_rhs][n] complex (written)
 * Asynchronous on ``stream``. */
mr1l_status mr1l_forward(mr1l_plan_t plan, const void* samples, void* coeffs, void* stream);

/* Adjoint transform (the adjoint of the forward map, see mr1l_weights).
 *   coeffs   device [n_rhs][n] complex (read only)
 *   samples  device [n_rhs][sum_l M_l] complex (written)
 * Asynchronous on ``stream``. */
mr1l_status mr1l_adjoint(mr1l_plan_t plan, const void* coeffs, void* samples, void* stream);

/* Integer outputs of the residue and alias-histogram passes (Alg. 1 and Alg. 2, definition of
 * I_l and counter), for inspection and exact comparison.  Any output may be NULL.
 *   residues   device int64 [L][n]: k.z_l mod M_l in [0, M_l)
 *   unaliased  device uint8 [L][n]: 1 iff k is in I_l
 *   counter    device uint8 [n]: #{l : k in I_l} (saturates at 255)
 * Asynchronous on ``stream``. */
mr1l_status mr1l_alias(mr1l_plan_t plan, int64_t* residues, uint8_t* unaliased, uint8_t* counter,
                       void* stream);

/* Host-side facts about the plan (synchronous).  Any output may be NULL.
 *   sample_offsets  host int64 [L+1]: off_l, off_L = sum_l M_l
 *   n_uncovered     number of frequencies with counter 0 (reading of Alg. 2 for that case: c_k = 0)
 *   fft_lengths     host int64 [L]: Bluestein convolution length used for lattice l */
mr1l_status mr1l_info(mr1l_plan_t plan, int64_t* sample_offsets, int64_t* n_uncovered,
                      int64_t* fft_lengths);

/* Weighted least-squares residual on the plan's stacked lattices: for samples s = A c (the
 * Fourier matrix of Sec. 2.1, a plan with weights MR1L_W_EVAL) and data y,
 *     loss = 1/2 sum_rhs sum_l (1/M_l) sum_j |s_l[j] - y_l[j]|^2
 *     grad = scale * (1/M_l) (s_l[j] - y_l[j])      (gradient of loss with respect to s)
 * computed in one pass over s and y (any weighting of the plan; only its lattice sizes are used).
 *   s, y    device [n_rhs][sum_l M_l] complex of the plan's dtype (read only; grad may alias s)
 *   scale   optional device double [1] multiplying grad (NULL: 1)
 *   grad    optional device [n_rhs][sum_l M_l] complex (written)
 *   loss    optional device double [1] (written; summed in double in a fixed order)
 * Asynchronous on ``stream``; the first call with a loss allocates the plan's buffer of block
 * partials (64 L n_rhs doubles), later calls allocate nothing.  Errors: MR1L_ERR_ARG for a NULL
 * plan or NULL s / y with samples present. */
mr1l_status mr1l_lsq_residual(mr1l_plan_t plan, const void* s, const void* y, const double* scale, void* grad,
                              double* loss, void* stream);

/* Allocation-free mr1l_lsq_residual, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving or training loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and results as mr1l_lsq_residual (bit-identical), but the block partials of the loss live
 * in one fixed device array per GPU (1 MiB, held until the process ends, looked up on the first call
 * on each device) instead of a plan buffer: no call allocates or frees anything.  Limit: with a loss
 * requested, 64 L n_rhs <= 131072 (else MR1L_ERR_UNSUPPORTED and nothing is launched).  Every call
 * on one GPU uses that GPU's array: calls that overlap on one GPU (different streams or host
 * threads without ordering between them) race and must not be issued.  Errors: MR1L_ERR_ARG as for
 * mr1l_lsq_residual, MR1L_ERR_HIP when the array's address cannot be obtained. */
mr1l_status mr1l_lsq_residual_noalloc(mr1l_plan_t plan, const void* s, const void* y, const double* scale,
                                      void* grad, double* loss, void* stream);

/* Plan-cached index work.  The residues r_l(k) and the alias bitmaps of Alg. 2 depend only on I
 * and the lattices, not on the samples or coefficients.  By default every forward and adjoint call
 * recomputes them (Alg. 2 as stated).  With enable = 1 the next call computes them once and later
 * calls reuse them; enable = 0 restores recomputation.  Host-side state, not ordered with
 * streams: a HIP graph captured while caching is on contains no index kernels.
 * Errors: MR1L_ERR_ARG for a NULL plan. */
mr1l_status mr1l_cache_alias(mr1l_plan_t plan, int enable);

/* Four-step schedule of the Bluestein FFTs.  A prime-length DFT runs as a power-of-two FFT of
 * length 2^lgN split as 2^lgN1 columns by 2^(lgN - lgN1) rows; every length from 2^13 to 2^24 has
 * the rule's split and its neighbours compiled, and the built-in table (measured on MI355X by
 * paper_1711_05152_amd/tune_fft.py) picks one.  This call sets the split plans of ``dtype`` use
 * for 2^lgN from now on (lgN1 > 0), restores the table's choice (lgN1 < 0) or only queries
 * (lgN1 = 0); ``current`` (optional) receives the split in effect.  Plans read the schedule when
 * they are created.  Errors: MR1L_ERR_ARG for a length outside 13..24 or a split not compiled. */
mr1l_status mr1l_fft_split(mr1l_dtype dtype, int lgN, int lgN1, int* current);

/* Variant of stage 2 of the four-step Bluestein FFT (row DFTs, filter, inverse row DFTs) for
 * length 2^lgN: bit 0 selects the radix schedule (radix 16 in every stage but one instead of the
 * bits spread evenly over the stages, e.g. 4 16 16 instead of 8 8 16 for 1024-point rows), bit 1
 * 4096-element row tiles instead of 2048 for rows of up to 2^10 points, bit 2 eight values per
 * thread instead of 16 (radices up to 8, e.g. 4 4 8 8, twice the threads; never with bit 0).  The
 * built-in table (measured by paper_1711_05152_amd/tune_fft.py together with the split) picks one
 * per precision and length.  variant 0..6 sets it for plans of ``dtype`` created from now on (it
 * must be compiled for the length and the split in effect), -1 only queries, -2 restores the
 * table's choice; ``current`` (optional) receives the variant in effect.  Errors: MR1L_ERR_ARG for
 * a length outside 13..24, a variant outside 0..6 or one not compiled for the length and split. */
mr1l_status mr1l_fft_p2_variant(mr1l_dtype dtype, int lgN, int variant, int* current);

/* Bound of a plan's Bluestein work area (the intermediate of the prime-length DFTs, one region of
 * sum_l N_l complex values per right-hand side).  Plans created from now on process
 * floor(max_bytes / region bytes) right-hand sides per pass over the lattices (at least one) and
 * loop over the passes within each call; results do not depend on the bound.  max_bytes > 0 sets
 * it (process-wide), < 0 restores the default of 4 GiB, 0 only queries; ``current`` (optional)
 * receives the bound in effect.  Never fails. */
mr1l_status mr1l_work_limit(int64_t max_bytes, int64_t* current);

/* Persistent in-block kernel of batched plans.  With enable = 1 (the default), a batched plan with
 * the weights of Alg. 2 and one right-hand side runs every transform whose lattices all have a
 * Bluestein length of at most 2^12 and that has at most 2048 frequencies in one persistent launch:
 * each workgroup takes a whole transform (residues, alias counts, prime-length DFTs, average or
 * scatter) from a work queue until none is left; the other transforms take the stage sweep.
 * Results are the same bits either way.  enable = 0 sends every transform to the stage sweep,
 * < 0 only queries; ``current`` (optional) receives the setting.  Plans read it when they are
 * created.  Never fails. */
mr1l_status mr1l_batch_inblock(int enable, int* current);

/* Right-hand sides side by side.  With several right-hand sides per pass, the forward's gather
 * (Alg. 2's average, or the Fourier-matrix weights' sum over the lattices) reads one random bin
 * per frequency, lattice and right-hand side, and the Fourier-matrix adjoint one random
 * coefficient per frequency, lattice and right-hand side.  Interleaving copies a block of 8
 * (complex64) or 4 (complex128) right-hand sides into 64-byte slots first, bins (forward) or
 * coefficients (adjoint), so that one random read fetches the whole block; the sums keep their
 * order, so results are the same bits either way.  mode 1 (the default) interleaves where the
 * pass's random reads leave the caches: bins of at least 256 MB per pass (sum M x right-hand sides
 * x element size), coefficients of at least 4 MB; 2 interleaves every pass of several right-hand
 * sides, 0 none; < 0 only queries.  ``current`` (optional) receives the mode.  Plans read it when
 * they are created and then hold a buffer of max(n, sum M) x 64 bytes (only while that is within
 * the work-area bound of mr1l_work_limit).  Errors: MR1L_ERR_ARG for a mode above 2. */
mr1l_status mr1l_rhs_interleave(int mode, int* current);

/* Bluestein lengths with a factor 3.  The convolution length of a lattice of size M must be at
 * least 2M - 1 (the chirp-z form of its prime-length DFT, Alg. 2's one-dimensional DFTs).  The
 * lattices of a transform whose power-of-two length would be 2^(k+2), 2^12 <= 2^k <= 2^22, may
 * take N = 3 * 2^k instead (25 % fewer points) when every one of them fits, 3 * 2^k >= 2M - 1; a
 * class whose lattices do not all fit keeps 2^(k+2) for all of them (two lengths in one class cost
 * more launches than the smaller one saves), except in a transform of at least 2^25 power-of-two
 * points times right-hand sides, where every lattice that fits takes 3 * 2^k.  The choice is per
 * transform, so a transform of a batched plan takes the lengths (and gives the bits) of its own
 * plan with the same number of right-hand sides.  mode 1 (the default) does so for the classes where the
 * autotuner (paper_1711_05152_amd/tune_fft.py) measured the factor-3 length faster, 2 for every
 * class, 0 never; < 0 only queries.  ``current`` (optional) receives the mode.  Plans read it when
 * they are created; results agree to rounding either way.  Errors: MR1L_ERR_ARG for a mode above 2. */
mr1l_status mr1l_fft_smooth(int mode, int* current);

/* Device-memory cache.  Every device buffer of the library (plan work areas, sparse-FFT steps)
 * comes from a per-device cache of size-classed blocks: a released block stays mapped and serves
 * later requests of its class, because allocating and freeing multi-GB regions through the driver
 * costs up to seconds per call once device memory has been churned.  Idle bytes per device are
 * capped (default: a quarter of the device's memory); a request that finds the device full
 * empties the cache and retries.
 *   device          device whose cache is addressed
 *   max_idle_bytes  new cap (0 disables caching); < 0 keeps the current cap
 *   released        optional out: bytes returned to the driver by this call
 * Returns every idle block of the device to the driver (after a device-wide synchronisation) and
 * then applies the cap.  The library also keeps the Bluestein filter spectra of recent plans per
 * device (at most 1 GiB, spectra up to 64 MiB; a plan whose lattice sizes all hit copies them
 * instead of recomputing); this call drops them too.  Errors: MR1L_ERR_ARG for an invalid device. */
mr1l_status mr1l_memory_cache(int device, int64_t max_idle_bytes, int64_t* released);

/* Release a plan and its device memory (NULL is accepted). */
mr1l_status mr1l_destroy(mr1l_plan_t plan);

/* Per-stage device timing.  While enabled, every forward/adjoint call records HIP events on its
 * stream around each kernel stage; mr1l_timing_read returns the summed milliseconds and launch
 * counts per stage and resets them (it synchronizes the events it reads).
 *   names      optional host array of MR1L_NSTAGES C strings receiving the stage names */
#define MR1L_NSTAGES 8
mr1l_status mr1l_timing_enable(mr1l_plan_t plan, int enable);
mr1l_status mr1l_timing_read(mr1l_plan_t plan, double* ms_sum, int64_t* launches,
                             const char** names);

/* Alg. 1: randomized construction of a reconstructing multiple rank-1 lattice with pairwise
 * distinct prime sizes, called until every k lies in some I_l, at most b calls (Alg. 3 step 2b).
 *   d, n, freqs   host int32 [n][d] frequency set (distinct rows)
 *   c, gamma      oversampling factor c > 1 and failure-probability bound 0 < gamma < 1
 *   b             maximal number of Alg. 1 calls (>= 1); the last call is kept if none covers I
 *   redraw        0: Alg. 1 as stated.  > 0: the earlier construction Alg. 1 modifies (remark
 *                 after Alg. 1): while Lambda(z_L, M_L) reconstructs no frequency not yet covered,
 *                 z_L is drawn again, at most redraw times (stream fields (t, call, L, a))
 *   seed, t       key of the generating-vector stream (SplitMix64, fields (t, call, L))
 *   L_cap         capacity of M and z (L_max = ceil(c^2/(c-1)^2 (ln n - ln gamma)/2) suffices)
 *   L_out         number of lattices returned
 *   M, z          host int64 [L_cap] sizes and [L_cap][d] generating vectors
 *   calls         number of Alg. 1 calls made
 *   n_uncovered   frequencies in no I_l (0 on success)
 *   device        device the residue/alias passes run on (synchronous)
 * Returns MR1L_WARN_UNCOVERED when b calls did not cover I (outputs still valid). */
mr1l_status mr1l_construct(int d, int64_t n, const int32_t* freqs, double c, double gamma, int b,
                           int redraw, uint64_t seed, int64_t t, int L_cap, int* L_out, int64_t* M,
                           int64_t* z, int* calls, int64_t* n_uncovered, int device);

/* ---- dimension-incremental sparse FFT (Alg. 3) ------------------------------------------------ */

/* Black box p(x) given by the caller: fill values_dev[j] = p(nodes_dev[j]) for j < n_nodes.
 * nodes_dev is device double [n_nodes][d] with coordinates in [0,1); values_dev is device complex
 * in the run's dtype.  Enqueue on ``stream`` or finish before returning; return 0 on success. */
typedef int (*sfft_sampler_fn)(void* user, int d, int64_t n_nodes, const double* nodes_dev,
                               void* values_dev, void* stream);

/* Built-in black box: a planted sparse polynomial p(x) = sum_h c_h e^{2 pi i h.x} plus complex
 * Gaussian noise eta = sigma/sqrt(2) (N(0,1) + i N(0,1)) on every sample (noise model of Sec. 5.2),
 * drawn from a counter-based stream keyed by noise_seed. */
typedef struct sfft_planted {
    int64_t s;               /* number of terms                                  */
    const int32_t* freqs;    /* host int32 [s][d]                                */
    const double* coeffs;    /* host double [s][2] (re, im)                      */
    double sigma;            /* noise level (0 = exact samples)                  */
    uint64_t noise_seed;
} sfft_planted;

/* Built-in test function of Sec. 5.3: f(x) = sum_tau w_tau prod_c N_{m(tau,c)}(x_c), a weighted sum
 * of tensor products of the periodic B-splines
 *     N_m(x) = C_m sum_{k in Z} sinc(pi k/m)^m (-1)^k e^{2 pi i k x},  ||N_m||_{L2(T)} = 1,
 * (factor 1 where the order is 0).  The test function on T^10 of Sec. 5.3 has three terms: order 2 on
 * components 1, 3, 8, order 4 on 2, 5, 6, 10 and order 6 on 4, 7, 9 (1-based), all weights 1. */
#define SFFT_BSPLINE_MAX_TERMS 8
#define SFFT_BSPLINE_MAX_ORDER 12
typedef struct sfft_bspline {
    int terms;               /* number of products, 1..SFFT_BSPLINE_MAX_TERMS    */
    int d;                   /* dimension, 1..SFFT_MAX_D                         */
    const int32_t* orders;   /* host int32 [terms][d]: order m (0..12) of the
                                factor of component c in product tau, 0 = none    */
    const double* weights;   /* host double [terms], or NULL for all ones        */
    mr1l_dtype dtype;        /* complex type of the values the sampler writes    */
} sfft_bspline;

/* Sampler of the built-in test function (signature of sfft_sampler_fn; pass it to sfft_detect with
 * user = a const sfft_bspline*).  Writes values_dev[j] = (f(nodes_dev[j]), 0) for j < n_nodes with
 * one kernel enqueued on ``stream`` (a hipStream_t, NULL for the default stream); nodes may lie
 * anywhere on R^d (taken mod 1).  Allocates nothing.  Returns 0, or 1 for an invalid description
 * (orders outside 0..12, d not matching) or a failed launch (mr1l_last_error() tells which). */
int sfft_sample_bspline(void* user, int d, int64_t n_nodes, const double* nodes_dev, void* values_dev,
                        void* stream);

/* Fourier coefficients f^_k = sum_tau w_tau prod_c g^_{tau,c}(k_c) of the test function (Sec. 5.3),
 * g^ = N^_m for a factor N_m, the indicator of k_c = 0 for a factor 1.
 *   freqs   host int32 [n][d];   coeffs  host double [n][2] (re, im; im is 0).  Host only. */
mr1l_status sfft_bspline_coeffs(const sfft_bspline* f, int64_t n, const int32_t* freqs, double* coeffs);

/* Relative L2(T^d) approximation error of p = sum_{k in I} p~_k e^{2 pi i k.x}, I = rows of freqs
 * (Sec. 5.3, by Parseval):
 *   ||f - p|| / ||f|| = sqrt(||f||^2 - sum_I |f^_k|^2 + sum_I |p~_k - f^_k|^2) / ||f||.
 *   freqs   host int32 [n][d] (distinct);  coeffs  host double [n][2];  rel_err  out;
 *   norm2   optional out, ||f||^2.  Host only. */
mr1l_status sfft_bspline_l2_error(const sfft_bspline* f, int64_t n, const int32_t* freqs, const double* coeffs,
                                  double* rel_err, double* norm2);

typedef struct sfft_params {
    double delta;            /* absolute threshold                               */
    int64_t s;               /* sparsity of the output                           */
    int64_t s_local;         /* sparsity of intermediate steps (0: use s)        */
    int r;                   /* detection iterations                             */
    int b;                   /* maximal Alg. 1 calls per step                    */
    uint64_t seed;           /* key of the generating-vector and anchor streams  */
    mr1l_dtype dtype;        /* precision of the transforms                      */
    double c, gamma;         /* Alg. 1 parameters (0 selects 2 and 1/2)          */
    int zero_anchors;        /* 1: anchors fixed to 0 (r = 1 mode of Sec. 3.1)   */
    int plain;               /* 1: one transform call per repetition (no batching
                                of repetitions / 1-D lines as right-hand sides)  */
    int redraw;              /* construction variant of step 2b (see
                                mr1l_construct); 0: Alg. 1                       */
    const int32_t* order;    /* NULL, or host int32 [d]: a permutation; step t
                                works on component order[t-1] (any component
                                order may be used).  Stream keys follow the step;
                                output rows hold the original components, listed
                                lexicographically in the processing order        */
    double delta_1d;         /* threshold of the 1-D detections (steps 1 and 2a);
                                0: delta.  The threshold-based truncation of
                                Sec. 5.3 uses delta / 10 there                   */
} sfft_params;

#define SFFT_MAX_D 64
typedef struct sfft_stats {
    int d;
    int64_t n_It[SFFT_MAX_D];      /* |I^(t)|                                          */
    int64_t n_J[SFFT_MAX_D];       /* |J_t| = |I^(1..t-1) x I^(t)| (t >= 2)           */
    int64_t n_detected[SFFT_MAX_D];/* |I^(1..t)|                                       */
    int32_t L[SFFT_MAX_D];         /* lattices used at step t                          */
    int64_t sumM[SFFT_MAX_D];      /* sum of their sizes                               */
    int32_t calls[SFFT_MAX_D];     /* Alg. 1 calls at step t                           */
    int32_t redraws[SFFT_MAX_D];   /* generating vectors drawn again (redraw variant)  */
    int64_t uncovered[SFFT_MAX_D]; /* frequencies of J_t in no I_l after the last call */
    int64_t samples;               /* distinct nodes: sum r K_t + sum r~ (1 - L + sum M) */
    int64_t samples_full;          /* values drawn (every lattice sampled in full)     */
    double ms_sampling, ms_transform, ms_construct, ms_select, ms_total;
} sfft_stats;

/* Alg. 3 on the box search space Gamma = [lo_1, hi_1] x ... x [lo_d, hi_d].
 *   d, lo, hi      host int32 [d] box corners (lo <= hi, hi - lo < 2^20)
 *   sampler, user  caller's black box (used when planted == NULL)
 *   planted        built-in black box (takes precedence over sampler when not NULL)
 *   params         thresholds, sparsities, r, b, seed, dtype
 *   cap            capacity of freqs_out / coeffs_out
 *   n_out          number of detected frequencies (<= min(s, |Gamma|)); if it exceeds cap only
 *                  the first cap are written and MR1L_ERR_ARG is returned
 *   freqs_out      host int32 [cap][d], lexicographically ascending
 *   coeffs_out     host double [cap][2] coefficients from the final transform
 *   stats          optional per-step statistics
 * Synchronous.  Returns MR1L_WARN_UNCOVERED when some step kept a non-reconstructing lattice. */
mr1l_status sfft_detect(int d, const int32_t* lo, const int32_t* hi, sfft_sampler_fn sampler,
                        void* user, const sfft_planted* planted, const sfft_params* params,
                        int64_t cap, int64_t* n_out, int32_t* freqs_out, double* coeffs_out,
                        sfft_stats* stats, int device);

/* Thread-local description of the last error (empty string when none). */
const char* mr1l_last_error(void);

/* Library version string. */
const char* mr1l_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MR1L_H */
