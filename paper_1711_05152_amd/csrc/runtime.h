// Host runtime of libmr1l: device buffers, error reporting, plans, random streams.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "common.h"
#include "host_logic.h"
#include "mr1l.h"

namespace mr1l {

// thread-local error text behind mr1l_last_error()
void set_error(const std::string& msg);
void clear_error();

#define MR1L_HIP_TRY(expr)                                                                           \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            ::mr1l::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                    \
            return e_ == hipErrorOutOfMemory ? MR1L_ERR_NOMEM : MR1L_ERR_HIP;                        \
        }                                                                                            \
    } while (0)

// Spectra kept across plans (plan.hip); mr1l_memory_cache drops a device's entries.
void filter_cache_clear(int dev);

// Caching device allocator (pool.hip): every DevMem goes through it.
hipError_t pool_alloc(void** p, size_t bytes, int* dev, size_t* block);
void pool_free(void* p, size_t block, int dev);

// Owning device allocation (size-classed, cached per device; see pool.hip).
struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;    // requested
    size_t block = 0;    // size of the cached block behind p (>= bytes)
    int dev = -1;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    DevMem(DevMem&& o) noexcept : p(o.p), bytes(o.bytes), block(o.block), dev(o.dev) {
        o.p = nullptr;
        o.bytes = o.block = 0;
        o.dev = -1;
    }
    DevMem& operator=(DevMem&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            block = o.block;
            dev = o.dev;
            o.p = nullptr;
            o.bytes = o.block = 0;
            o.dev = -1;
        }
        return *this;
    }
    ~DevMem() { release(); }
    void release() {
        if (p) pool_free(p, block, dev);
        p = nullptr;
        bytes = block = 0;
        dev = -1;
    }
    hipError_t alloc(size_t b) {
        release();
        if (b == 0) return hipSuccess;
        hipError_t e = pool_alloc(&p, b, &dev, &block);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    hipError_t upload(const void* h, size_t b) {
        hipError_t e = alloc(b);
        if (e != hipSuccess || b == 0) return e;
        return hipMemcpy(p, h, b, hipMemcpyHostToDevice);
    }
    template <typename U> U* as() const { return (U*)p; }
};

// Segment copies in one launch per 16 segments: src and dst in device memory or in pinned,
// device-accessible host memory, any alignment (16-byte moves where both ends allow).
struct CopySeg {
    const void* src;
    void* dst;
    uint64_t bytes;
};
hipError_t copy_segments(const CopySeg* segs, int n, hipStream_t st);

// Small host tables (descriptors, generating vectors, tile lists) on their way to the device: each
// add() allocates the device buffer and appends the bytes to a host list; flush() copies the list
// into a pinned, device-accessible buffer owned by the calling thread (one per slot) and queues one
// copy kernel that moves every table from there to its device buffer (one launch instead of one
// copy call per table), ordered before the kernels that read them.  A flush first waits for the
// copy of the slot's previous flush (an event), so the pinned bytes outlive their copy; a caller
// that destroys the stream it flushed on settles the slot first.  The device buffers must not be
// released before the copy has run (the stream is synchronised before they go out of scope).
struct TableStager {
    enum Slot { PLAN = 0, DRIVER = 1 };
    explicit TableStager(Slot s) : slot(s) {}
    hipError_t add(DevMem& dst, const void* src, size_t bytes);
    hipError_t flush(hipStream_t st);
    // wait for the copies of the slot's last flush on this thread (before their stream goes away)
    static hipError_t settle(Slot slot);
    Slot slot;
    struct Item { DevMem* dst; size_t off, bytes; };
    std::vector<Item> items;
    std::vector<char> host;
};

// Counter-based SplitMix64 streams of the method's random draws (host_logic.h).
using host::Rng;

// Bound of a plan's Bluestein work area in bytes (process-wide, mr1l_work_limit; default 4 GiB).
int64_t work_limit_bytes();
// Whether batched plans run their small transforms in the persistent in-block kernel
// (process-wide, mr1l_batch_inblock; default on).
bool batch_inblock_enabled();
// Right-hand-side interleaving of the gather and the bin sums (process-wide, mr1l_rhs_interleave):
// 0 never, 1 where the pass's random reads leave the caches (default), 2 for every pass of
// several right-hand sides.
int rhs_interleave_mode();

// Description of the transforms a plan holds.  A plain plan has one transform; a batched plan
// stacks several independent ones (own frequencies, own lattices).
struct PlanSpec {
    int d = 0;
    mr1l_dtype dtype = MR1L_C64;
    mr1l_weights weights = MR1L_W_PAPER;
    int64_t n_rhs = 1;
    int device = 0;
    // frequencies: either host int32 [n][d] or device component-major packed data
    const int32_t* host_freqs = nullptr;
    const void* dev_freqs = nullptr;   // component-major [d][n] of type ktype (not owned)
    int dev_ktype = K_I32;
    int64_t dev_maxabs = 0;            // max |k| of the device frequencies
    bool check_distinct = true;
    int64_t max_work_bytes = work_limit_bytes();   // bound of the Bluestein work area (rhs chunking)
    // reuse the filter spectra of a plan with the same lattice sizes (same order) and dtype
    const struct Plan* share_filters = nullptr;
    // set-up work (table copies, filter spectra) goes to ``stream``; with sync the device is
    // synchronised before plan_create returns (the public entry points), without it the plan may
    // only be used on ``stream`` (the sparse-FFT driver's own plans)
    hipStream_t stream = nullptr;
    bool sync = true;
    // transforms
    std::vector<int64_t> tx_n;         // frequencies per transform
    std::vector<int32_t> tx_L;         // lattices per transform
    std::vector<int64_t> M;            // all lattice sizes, transform after transform
    std::vector<int64_t> z;            // [sum L][d]
};

struct Plan {
    int device = 0;
    int d = 0;
    int64_t n = 0;
    int L = 0;
    mr1l_dtype dtype = MR1L_C64;
    mr1l_weights weights = MR1L_W_PAPER;
    int64_t n_rhs = 1;
    int64_t rhs_chunk = 1;             // right-hand sides per pass through the work area
    std::vector<LatDesc> hdesc;
    std::vector<TxDesc> htx;
    std::vector<int64_t> samp_off;     // [L + 1]
    int64_t sum_M = 0;
    int64_t work_stride = 0;
    int64_t filt_total = 0;
    int64_t bm_total = 0;
    DevMem freqs, desc, tx, tx_foff, z, z32, bitmaps, filt, work, grp_lat, res32, hist, rtiles, part, bcnt, bloc, bbase, perm,
        ilv;
    DevMem lsq_part;                   // block partials of mr1l_lsq_residual (allocated on first use)
    std::vector<FftGroup> groups;   // lattices grouped by Bluestein length (filter construction)
    std::vector<FftGroup> sweep;    // the same without the lattices of in-block transforms
    DevMem sweep_lat;                  // lattice lists of the sweep groups
    DevMem inblock, queue;             // in-block transforms (largest first) and their work queue
    int n_inblock = 0;
    hipStream_t side = nullptr;        // the in-block launch runs here, beside the stage sweep
    hipEvent_t fork = nullptr, join = nullptr;
    // four-step groups after the first run their stage pipelines (stage 1 -> 2 -> 3) on streams of
    // their own, from a per-device pool, forked after the index pass and joined before the gather
    std::vector<hipStream_t> gstream;
    std::vector<hipEvent_t> gdone;
    hipEvent_t gstart = nullptr;
    void* filt_ptr = nullptr;          // filt.p, or the filters of the plan shared at creation
    TxArgs args{};
    // plan-cached index work: residues and bitmaps valid from an earlier call
    bool cache_alias = false;
    bool alias_valid = false;
    bool sort_valid = false;           // counting sort of the Fourier-matrix adjoint, same rule
    // per-stage timing
    bool timing = false;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> free_events;
    double ms_sum[MR1L_NSTAGES] = {0};
    int64_t launches[MR1L_NSTAGES] = {0};
    ~Plan();
};

mr1l_status plan_create(const PlanSpec& spec, Plan** out);
mr1l_status plan_forward(Plan* p, const void* samples, void* coeffs, hipStream_t s);
mr1l_status plan_adjoint(Plan* p, const void* coeffs, void* samples, hipStream_t s);
mr1l_status plan_alias(Plan* p, int64_t* res, uint8_t* uniq, uint8_t* counter, hipStream_t s);

// Alg. 1 (+ repetition, Alg. 3 step 2b) on device-resident or host frequencies.
// redraw > 0: the construction variant that draws z_L again (at most redraw times) while the
// lattice reconstructs no frequency not yet covered
struct ConstructResult {
    std::vector<int64_t> M, z;
    int calls = 0;
    int64_t uncovered = 0;
    int64_t redraws = 0;
};
mr1l_status construct_lattices(int d, int64_t n, const int32_t* host_freqs, const void* dev_freqs, int ktype,
                               int64_t maxabs, int64_t expansion, double c, double gamma, int b, int redraw,
                               uint64_t seed, int64_t t, int device, hipStream_t s, ConstructResult* out);

}  // namespace mr1l
