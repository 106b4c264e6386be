// Schedule of the four-step Bluestein FFT: which compiled split each length uses.  The built-in
// table is the one the tuning script measured (fft_schedule_table.h); mr1l_fft_split overrides an
// entry for the process (the tuner itself times every candidate that way).  Plans read the
// schedule when they are created, and so they read the bound of their work area
// (mr1l_work_limit), which decides how many right-hand sides one pass over the lattices holds.
#include <hip/hip_runtime.h>

#include <atomic>

#include "common.h"
#include "fft_schedule_table.h"
#include "runtime.h"

namespace mr1l {
namespace {
std::atomic<int> g_override[2][kMaxLgN + 1];
std::atomic<int> g_p2_override[2][kMaxLgN + 1];
struct InitOverrides {
    InitOverrides() {
        for (auto& row : g_override)
            for (auto& v : row) v.store(-1);
        for (auto& row : g_p2_override)
            for (auto& v : row) v.store(-1);
    }
} g_init_overrides;

constexpr int64_t kDefaultWorkLimit = (int64_t)4 << 30;
std::atomic<int64_t> g_work_limit{kDefaultWorkLimit};
std::atomic<int> g_inblock{1};
std::atomic<int> g_smooth{1};
std::atomic<int> g_interleave{1};

int table_split(int dt, int lgN) {
    const int t = kTunedSplit[dt][lgN];
    return split_compiled(lgN, t) ? t : split_lgN1(lgN);
}
}  // namespace

int fft_split(int dtype, int lgN) {
    const int dt = dtype == MR1L_C128 ? 1 : 0;
    if (lgN <= kSmallMaxLg || lgN > kMaxLgN) return split_lgN1(lgN);
    const int o = g_override[dt][lgN].load();
    return o >= 0 ? o : table_split(dt, lgN);
}

int fft_p2_variant(int dtype, int lgN, int lg1) {
    const int dt = dtype == MR1L_C128 ? 1 : 0;
    if (lgN <= kSmallMaxLg || lgN > kMaxLgN) return 0;
    const int o = g_p2_override[dt][lgN].load();
    const int v = o >= 0 ? o : kTunedP2[dt][lgN];
    return p2_variant_compiled(lgN, lg1, v) ? v : 0;
}

int64_t work_limit_bytes() { return g_work_limit.load(); }
bool batch_inblock_enabled() { return g_inblock.load() != 0; }
int rhs_interleave_mode() { return g_interleave.load(); }
bool fft_smooth_class(int dtype, int lg) {
    const int m = g_smooth.load();
    if (lg < kMinLg3 + 2 || lg > kMaxLg3 + 2) return false;
    return m == 2 || (m == 1 && kTunedSmooth[dtype == MR1L_C128 ? 1 : 0][lg] == 1);
}

}  // namespace mr1l

using namespace mr1l;

extern "C" mr1l_status mr1l_work_limit(int64_t max_bytes, int64_t* current) {
    clear_error();
    if (max_bytes > 0) g_work_limit.store(max_bytes);
    else if (max_bytes < 0) g_work_limit.store(kDefaultWorkLimit);
    if (current) *current = g_work_limit.load();
    return MR1L_OK;
}

extern "C" mr1l_status mr1l_batch_inblock(int enable, int* current) {
    clear_error();
    if (enable >= 0) g_inblock.store(enable ? 1 : 0);
    if (current) *current = g_inblock.load();
    return MR1L_OK;
}

extern "C" mr1l_status mr1l_rhs_interleave(int mode, int* current) {
    clear_error();
    if (mode > 2) {
        set_error("mr1l_rhs_interleave: mode 0 (never), 1 (by size) or 2 (every pass of several right-hand sides)");
        return MR1L_ERR_ARG;
    }
    if (mode >= 0) g_interleave.store(mode);
    if (current) *current = g_interleave.load();
    return MR1L_OK;
}

extern "C" mr1l_status mr1l_fft_smooth(int enable, int* current) {
    clear_error();
    if (enable > 2) {
        set_error("mr1l_fft_smooth: mode 0 (powers of two), 1 (measured table) or 2 (every class)");
        return MR1L_ERR_ARG;
    }
    if (enable >= 0) g_smooth.store(enable);
    if (current) *current = g_smooth.load();
    return MR1L_OK;
}

extern "C" mr1l_status mr1l_fft_p2_variant(mr1l_dtype dtype, int lgN, int variant, int* current) {
    clear_error();
    if ((dtype != MR1L_C64 && dtype != MR1L_C128) || lgN <= kSmallMaxLg || lgN > kMaxLgN || variant >= kP2Variants) {
        set_error("mr1l_fft_p2_variant: dtype, length (2^13 .. 2^24) or variant (0 .. 6) out of range");
        return MR1L_ERR_ARG;
    }
    const int dt = dtype == MR1L_C128 ? 1 : 0;
    if (variant >= 0) {
        if (!p2_variant_compiled(lgN, fft_split(dtype, lgN), variant)) {
            set_error("mr1l_fft_p2_variant: variant not compiled for this length and its current split");
            return MR1L_ERR_ARG;
        }
        g_p2_override[dt][lgN].store(variant);
    } else if (variant < -1) {
        g_p2_override[dt][lgN].store(-1);
    }
    if (current) *current = fft_p2_variant(dtype, lgN, fft_split(dtype, lgN));
    return MR1L_OK;
}

extern "C" mr1l_status mr1l_fft_split(mr1l_dtype dtype, int lgN, int lgN1, int* current) {
    clear_error();
    if ((dtype != MR1L_C64 && dtype != MR1L_C128) || lgN <= kSmallMaxLg || lgN > kMaxLgN) {
        set_error("mr1l_fft_split: dtype or length outside the four-step range 2^13 .. 2^24");
        return MR1L_ERR_ARG;
    }
    const int dt = dtype == MR1L_C128 ? 1 : 0;
    if (lgN1 > 0) {
        if (!split_compiled(lgN, lgN1)) {
            set_error("mr1l_fft_split: split not compiled for this length (rule +- 1, factors 2^4 .. 2^12)");
            return MR1L_ERR_ARG;
        }
        g_override[dt][lgN].store(lgN1);
    } else if (lgN1 < 0) {
        g_override[dt][lgN].store(-1);
    }
    if (current) *current = fft_split(dtype, lgN);
    return MR1L_OK;
}
