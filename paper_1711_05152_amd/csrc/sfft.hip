// Alg. 3: dimension-incremental sparse FFT on multiple rank-1 lattices ("MLFFT").
//
// Host control flow in the paper's order; every data-parallel step runs on the device:
//   steps 1/2a  1-D projections of all components up front (they only depend on their own random
//               anchors): black-box samples on the lines, one mr1l transform with L = 1, M = K_t,
//               z = 1 (the DFT of length K_t with the factor 1/K_t), selection of the (up to)
//               s_local largest |p~| >= delta per repetition, union over repetitions;
//   step 2b     J_t = I^(1..t-1) x I^(t) built on the device; Alg. 1 with c = 2, gamma = 1/2,
//               repeated up to b calls (construct.hip);
//   steps 2c-e  r~ repetitions as right-hand sides of one transform: black-box samples on the
//               lattice nodes with anchors appended (built-in planted polynomial: Fourier-matrix
//               synthesis on the same lattices; or the caller's sampler on explicit nodes),
//               forward transform (Alg. 2), selection of the (up to) s~ largest |p~| >= delta,
//               union, compaction into I^(1..t);
//   step 3      I^(1..d) and the coefficients of the final transform.
// Random draws (generating vectors, anchors) use the SplitMix64 streams of runtime.h keyed by
// (purpose, t, i): ANCHOR1D anchors for the 1-D lines, ANCHOR for the lattice steps.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "runtime.h"
#include "sfft_dev.h"

namespace mr1l {

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); }

struct PlanGuard {
    Plan* p = nullptr;
    ~PlanGuard() { delete p; }
};

int ktype_for(int64_t maxabs) { return maxabs <= 127 ? K_I8 : (maxabs <= 32767 ? K_I16 : K_I32); }
size_t ksize(int kt) { return kt == K_I8 ? 1 : (kt == K_I16 ? 2 : 4); }

struct Ctx {
    int d;
    const int32_t* lo;
    const int32_t* hi;
    sfft_sampler_fn sampler;
    void* user;
    const sfft_planted* planted;
    sfft_params prm;
    int device;
    hipStream_t st;
    sfft_stats* stats;
    int kt;                 // packed type of candidate frequencies
    int64_t box_maxabs;
    // planted black box on the device
    DevMem hf;              // int32 [d][s]
    DevMem hc;              // complex double [s]
    int64_t s_pl = 0;
    int64_t pl_maxabs = 0;
    // component order: step t works on component order[t]; the box and the planted frequencies
    // are held in processing order, caller nodes are written in the caller's columns
    std::vector<int> order;
    std::vector<int32_t> plo, phi;
    DevMem dcol;
};

mr1l_status sync_check(hipStream_t st) {
    MR1L_HIP_TRY(hipGetLastError());
    MR1L_HIP_TRY(hipStreamSynchronize(st));
    return MR1L_OK;
}

#define TRY(x)                                  \
    do {                                        \
        mr1l_status st_ = (x);                  \
        if (st_ != MR1L_OK) return st_;         \
    } while (0)

// ---- steps 1 and 2a ------------------------------------------------------------------------------
// For every component t (1-based) returns I^(t) on the device (ascending values) and its size;
// for d = 1 also the coefficients of the last repetition at I^(1).
mr1l_status detect_1d(Ctx& C, std::vector<DevMem>& It, std::vector<int64_t>& nIt, DevMem* c1, int64_t* n1out) {
    const int d = C.d, r = C.prm.r;
    const size_t csz = C.prm.dtype == MR1L_C128 ? 16 : 8;
    std::map<std::pair<int32_t, int32_t>, std::vector<int>> groups;
    for (int t = 1; t <= d; ++t) groups[{C.lo[t - 1], C.hi[t - 1]}].push_back(t);
    It.resize(d + 1);
    nIt.assign(d + 1, 0);
    for (auto& kv : groups) {
        const int32_t lo = kv.first.first, hi = kv.first.second;
        const std::vector<int>& ts = kv.second;
        const int64_t K = (int64_t)hi - lo + 1;
        const int njobs = (int)ts.size() * r;
        auto t0 = clk::now();
        std::vector<int32_t> f1(K);
        for (int64_t k = 0; k < K; ++k) f1[k] = (int32_t)(lo + k);
        PlanSpec sp;
        sp.d = 1;
        sp.dtype = C.prm.dtype;
        sp.weights = MR1L_W_PAPER;
        const int per_call = C.prm.plain ? 1 : njobs;
        sp.n_rhs = per_call;
        sp.device = C.device;
        sp.host_freqs = f1.data();
        sp.check_distinct = false;
        sp.tx_n = {K};
        sp.tx_L = {1};
        sp.M = {K};
        sp.z = {1};
        PlanGuard pg;
        TRY(plan_create(sp, &pg.p));
        if (C.stats) C.stats->ms_construct += ms_since(t0);

        // anchors, components and noise keys per job q = (index of t in the group) * r + (i - 1)
        std::vector<double> anchors((size_t)njobs * d, 0.0);
        std::vector<int> comp(njobs);
        std::vector<uint64_t> keys(njobs);
        for (size_t a = 0; a < ts.size(); ++a)
            for (int i = 1; i <= r; ++i) {
                const int q = (int)a * r + (i - 1);
                comp[q] = ts[a] - 1;
                const uint64_t key = Rng::key(C.prm.seed, {Rng::ANCHOR1D, ts[a], i});
                if (!C.prm.zero_anchors)
                    for (int c = 0; c < d; ++c) anchors[(size_t)q * d + c] = Rng::uniform01(key, c);
                keys[q] = C.planted ? Rng::key(C.planted->noise_seed, {Rng::NOISE, 0, ts[a], i}) : 0;
            }
        t0 = clk::now();
        DevMem dA, dComp, dKeys, y, w, coeffs, flags, idx, cnt;
        {
            TableStager stg(TableStager::DRIVER);
            MR1L_HIP_TRY(stg.add(dA, anchors.data(), anchors.size() * sizeof(double)));
            MR1L_HIP_TRY(stg.add(dComp, comp.data(), comp.size() * sizeof(int)));
            MR1L_HIP_TRY(stg.add(dKeys, keys.data(), keys.size() * sizeof(uint64_t)));
            MR1L_HIP_TRY(stg.flush(C.st));
        }
        MR1L_HIP_TRY(y.alloc((size_t)njobs * K * csz));
        if (C.planted) {
            MR1L_HIP_TRY(w.alloc((size_t)njobs * std::max<int64_t>(1, C.s_pl) * 16));
            if (C.s_pl > 0) {
                sf_planted_w1d(C.hf.as<int32_t>(), C.s_pl, d, C.hc.p, dA.as<double>(), dComp.as<int>(), njobs, w.p,
                               C.st);
            }
            sf_planted_1d(C.prm.dtype, C.hf.as<int32_t>(), C.s_pl, w.p, dComp.as<int>(), njobs, K, dKeys.as<uint64_t>(),
                          C.planted->sigma, y.p, C.st);
        } else {
            DevMem nodes;
            MR1L_HIP_TRY(nodes.alloc((size_t)K * d * sizeof(double)));
            for (int q = 0; q < njobs; ++q) {
                sf_nodes_1d(K, comp[q], d, dA.as<double>() + (size_t)q * d, nodes.as<double>(),
                            C.dcol.p ? C.dcol.as<int>() : nullptr, C.st);
                if (C.sampler(C.user, d, K, nodes.as<double>(), (char*)y.p + (size_t)q * K * csz, C.st) != 0) {
                    set_error("sampler callback returned an error");
                    return MR1L_ERR_CALLBACK;
                }
            }
        }
        TRY(sync_check(C.st));
        if (C.stats) C.stats->ms_sampling += ms_since(t0);

        t0 = clk::now();
        MR1L_HIP_TRY(coeffs.alloc((size_t)njobs * K * csz));
        for (int q0 = 0; q0 < njobs; q0 += per_call)
            TRY(plan_forward(pg.p, (const char*)y.p + (size_t)q0 * K * csz, (char*)coeffs.p + (size_t)q0 * K * csz,
                             C.st));
        TRY(sync_check(C.st));
        if (C.stats) C.stats->ms_transform += ms_since(t0);

        t0 = clk::now();
        MR1L_HIP_TRY(flags.alloc((size_t)ts.size() * K));
        MR1L_HIP_TRY(hipMemsetAsync(flags.p, 0, (size_t)ts.size() * K, C.st));
        sf_select(C.prm.dtype, coeffs.p, K, njobs, C.prm.delta_1d, C.prm.s_local, flags.as<uint8_t>(), r, K, C.st);
        MR1L_HIP_TRY(idx.alloc((size_t)K * sizeof(int32_t)));
        MR1L_HIP_TRY(cnt.alloc(sizeof(int64_t)));
        for (size_t a = 0; a < ts.size(); ++a) {
            const int t = ts[a];
            sf_compact(flags.as<uint8_t>() + a * K, K, idx.as<int32_t>(), cnt.as<int64_t>(), C.st);
            int64_t m = 0;
            MR1L_HIP_TRY(hipMemcpyAsync(&m, cnt.p, sizeof(int64_t), hipMemcpyDeviceToHost, C.st));
            TRY(sync_check(C.st));
            nIt[t] = m;
            MR1L_HIP_TRY(It[t].alloc((size_t)std::max<int64_t>(1, m) * sizeof(int32_t)));
            if (m) sf_flags_to_values(idx.as<int32_t>(), m, lo, It[t].as<int32_t>(), C.st);
            if (C.stats) C.stats->n_It[t - 1] = m;
            if (C.stats) {
                C.stats->samples += (int64_t)r * K;
                C.stats->samples_full += (int64_t)r * K;
            }
            if (t == 1 && d == 1 && m > 0) {
                // d = 1: the coefficients of the last repetition at I^(1)
                MR1L_HIP_TRY(c1->alloc((size_t)m * 16));
                const int q = (int)a * r + (r - 1);
                sf_gather_coeffs(C.prm.dtype, (const char*)coeffs.p + (size_t)q * K * csz, idx.as<int32_t>(), m, c1->p,
                                 C.st);
                *n1out = m;
            }
        }
        TRY(sync_check(C.st));
        if (C.stats) C.stats->ms_select += ms_since(t0);
    }
    return MR1L_OK;
}

mr1l_status run(Ctx& C, int64_t cap, int64_t* n_out, int32_t* freqs_out, double* coeffs_out, bool* uncovered_any) {
    const int d = C.d;
    const int r = C.prm.r;
    const size_t csz = C.prm.dtype == MR1L_C128 ? 16 : 8;
    const size_t ks = ksize(C.kt);
    *n_out = 0;
    *uncovered_any = false;

    std::vector<DevMem> It;
    std::vector<int64_t> nIt;
    DevMem c1;
    int64_t n1 = 0;
    TRY(detect_1d(C, It, nIt, &c1, &n1));

    // I^(1..1) = I^(1)
    DevMem prev;
    int64_t nprev = nIt[1];
    MR1L_HIP_TRY(prev.alloc((size_t)std::max<int64_t>(1, nprev) * ks));
    if (nprev) sf_values_to_k(C.kt, It[1].as<int32_t>(), nprev, prev.p, C.st);
    if (C.stats) C.stats->n_detected[0] = nprev;
    DevMem final_coeffs;
    int64_t nfinal = 0;
    if (d == 1) {
        final_coeffs = std::move(c1);
        nfinal = n1;
    }

    for (int t = 2; t <= d && nprev > 0; ++t) {
        const int64_t n2 = nIt[t];
        const int64_t nJ = nprev * n2;
        if (C.stats) C.stats->n_J[t - 1] = nJ;
        if (nJ == 0) {
            nprev = 0;
            break;
        }
        auto t0 = clk::now();
        DevMem J;
        MR1L_HIP_TRY(J.alloc((size_t)nJ * t * ks));
        sf_product(C.kt, prev.p, nprev, It[t].as<int32_t>(), n2, t, J.p, C.st);
        TRY(sync_check(C.st));
        if (C.stats) C.stats->ms_select += ms_since(t0);

        // step 2b: Alg. 1, repeated up to b calls
        t0 = clk::now();
        int64_t expansion = 0;
        for (int c = 0; c < t; ++c) expansion = std::max<int64_t>(expansion, (int64_t)C.hi[c] - C.lo[c]);
        ConstructResult cr;
        TRY(construct_lattices(t, nJ, nullptr, J.p, C.kt, C.box_maxabs, expansion, C.prm.c, C.prm.gamma, C.prm.b,
                               C.prm.redraw, C.prm.seed, t, C.device, C.st, &cr));
        if (C.stats) C.stats->redraws[t - 1] = (int32_t)cr.redraws;
        const int L = (int)cr.M.size();
        int64_t sumM = 0;
        for (int64_t m : cr.M) sumM += m;
        if (cr.uncovered) *uncovered_any = true;
        const int rt = t < d ? r : 1;
        const int64_t st_ = t < d ? C.prm.s_local : C.prm.s;
        const int per_call = C.prm.plain ? 1 : rt;
        PlanSpec sp;
        sp.d = t;
        sp.dtype = C.prm.dtype;
        sp.weights = MR1L_W_PAPER;
        sp.n_rhs = per_call;
        sp.device = C.device;
        sp.dev_freqs = J.p;
        sp.dev_ktype = C.kt;
        sp.dev_maxabs = C.box_maxabs;
        sp.check_distinct = false;
        sp.tx_n = {nJ};
        sp.tx_L = {L};
        sp.M = cr.M;
        sp.z = cr.z;
        sp.stream = C.st;   // set up on the driver's stream, without a device-wide wait
        sp.sync = false;
        if (C.stats) {
            C.stats->L[t - 1] = L;
            C.stats->sumM[t - 1] = sumM;
            C.stats->calls[t - 1] = cr.calls;
            C.stats->uncovered[t - 1] = cr.uncovered;
            C.stats->ms_construct += ms_since(t0);
        }

        // steps 2c-e: r~ repetitions as right-hand sides
        std::vector<double> anchors((size_t)rt * d, 0.0);
        std::vector<uint64_t> keys(rt);
        for (int i = 1; i <= rt; ++i) {
            const uint64_t key = Rng::key(C.prm.seed, {Rng::ANCHOR, t, i});
            if (!C.prm.zero_anchors)
                for (int c = t; c < d; ++c) anchors[(size_t)(i - 1) * d + c] = Rng::uniform01(key, c);
            keys[i - 1] = C.planted ? Rng::key(C.planted->noise_seed, {Rng::NOISE, 1, t, i}) : 0;
        }
        t0 = clk::now();
        DevMem dA, dKeys, y;
        {
            TableStager stg(TableStager::DRIVER);
            MR1L_HIP_TRY(stg.add(dA, anchors.data(), anchors.size() * sizeof(double)));
            MR1L_HIP_TRY(stg.add(dKeys, keys.data(), keys.size() * sizeof(uint64_t)));
            MR1L_HIP_TRY(stg.flush(C.st));
        }
        MR1L_HIP_TRY(y.alloc((size_t)rt * std::max<int64_t>(1, sumM) * csz));
        // the sampling plan (built-in black box) is created first, with the lattices' filter
        // spectra; the transform plan shares them and is set up while the device samples, so it
        // must not outlive the sampling plan (declared before it)
        PlanGuard pP;
        if (C.planted) {
            if (C.s_pl > 0) {
                PlanSpec pp;
                pp.d = t;
                pp.dtype = C.prm.dtype;
                pp.weights = MR1L_W_EVAL;
                pp.n_rhs = per_call;
                pp.device = C.device;
                pp.dev_freqs = C.hf.p;           // first t components of [d][s]
                pp.dev_ktype = K_I32;
                pp.dev_maxabs = C.pl_maxabs;
                pp.check_distinct = false;
                pp.tx_n = {C.s_pl};
                pp.tx_L = {L};
                pp.M = cr.M;
                pp.z = cr.z;
                pp.stream = C.st;
                pp.sync = false;
                TRY(plan_create(pp, &pP.p));
                DevMem w;
                MR1L_HIP_TRY(w.alloc((size_t)rt * C.s_pl * csz));
                sf_planted_wlat(C.prm.dtype, C.hf.as<int32_t>(), C.s_pl, d, t, C.hc.p, dA.as<double>(), rt, w.p, C.st);
                for (int i0 = 0; i0 < rt; i0 += per_call)
                    TRY(plan_adjoint(pP.p, (const char*)w.p + (size_t)i0 * C.s_pl * csz,
                                     (char*)y.p + (size_t)i0 * sumM * csz, C.st));
            } else {
                MR1L_HIP_TRY(hipMemsetAsync(y.p, 0, (size_t)rt * sumM * csz, C.st));
            }
            if (C.planted->sigma > 0.0) sf_add_noise(C.prm.dtype, y.p, sumM, rt, dKeys.as<uint64_t>(), C.planted->sigma, C.st);
        } else {
            DevMem nodes, dM, dOff, dZ;
            std::vector<int64_t> off(L + 1, 0);
            for (int l = 0; l < L; ++l) off[l + 1] = off[l] + cr.M[l];
            MR1L_HIP_TRY(nodes.alloc((size_t)sumM * d * sizeof(double)));
            {
                TableStager stg(TableStager::DRIVER);
                MR1L_HIP_TRY(stg.add(dM, cr.M.data(), L * sizeof(int64_t)));
                MR1L_HIP_TRY(stg.add(dOff, off.data(), off.size() * sizeof(int64_t)));
                MR1L_HIP_TRY(stg.add(dZ, cr.z.data(), cr.z.size() * sizeof(int64_t)));
                MR1L_HIP_TRY(stg.flush(C.st));
            }
            const int64_t maxM = *std::max_element(cr.M.begin(), cr.M.end());
            for (int i = 0; i < rt; ++i) {
                sf_nodes_lattice(dM.as<int64_t>(), dOff.as<int64_t>(), dZ.as<int64_t>(), L, maxM, t, d,
                                 dA.as<double>() + (size_t)i * d, nodes.as<double>(),
                                 C.dcol.p ? C.dcol.as<int>() : nullptr, C.st);
                if (C.sampler(C.user, d, sumM, nodes.as<double>(), (char*)y.p + (size_t)i * sumM * csz, C.st) != 0) {
                    set_error("sampler callback returned an error");
                    return MR1L_ERR_CALLBACK;
                }
            }
        }
        // the transform plan, set up on the host while the device samples; its host time counts
        // as construction
        const auto tp = clk::now();
        sp.share_filters = pP.p;
        PlanGuard pJ;
        TRY(plan_create(sp, &pJ.p));
        const double ms_plan = ms_since(tp);
        TRY(sync_check(C.st));
        if (C.stats) {
            C.stats->ms_construct += ms_plan;
            C.stats->ms_sampling += ms_since(t0) - ms_plan;
            C.stats->samples += (int64_t)rt * (1 - L + sumM);
            C.stats->samples_full += (int64_t)rt * sumM;
        }

        t0 = clk::now();
        DevMem coeffs;
        MR1L_HIP_TRY(coeffs.alloc((size_t)rt * nJ * csz));
        for (int i0 = 0; i0 < rt; i0 += per_call)
            TRY(plan_forward(pJ.p, (const char*)y.p + (size_t)i0 * sumM * csz, (char*)coeffs.p + (size_t)i0 * nJ * csz,
                             C.st));
        TRY(sync_check(C.st));
        if (C.stats) C.stats->ms_transform += ms_since(t0);

        t0 = clk::now();
        DevMem flags, idx, cnt, next;
        MR1L_HIP_TRY(flags.alloc((size_t)nJ));
        MR1L_HIP_TRY(hipMemsetAsync(flags.p, 0, (size_t)nJ, C.st));
        sf_select(C.prm.dtype, coeffs.p, nJ, rt, C.prm.delta, st_, flags.as<uint8_t>(), rt, 0, C.st);
        MR1L_HIP_TRY(idx.alloc((size_t)nJ * sizeof(int32_t)));
        MR1L_HIP_TRY(cnt.alloc(sizeof(int64_t)));
        sf_compact(flags.as<uint8_t>(), nJ, idx.as<int32_t>(), cnt.as<int64_t>(), C.st);
        int64_t m = 0;
        MR1L_HIP_TRY(hipMemcpyAsync(&m, cnt.p, sizeof(int64_t), hipMemcpyDeviceToHost, C.st));
        TRY(sync_check(C.st));
        MR1L_HIP_TRY(next.alloc((size_t)std::max<int64_t>(1, m) * t * ks));
        if (m) sf_gather_rows(C.kt, J.p, nJ, t, idx.as<int32_t>(), m, next.p, C.st);
        if (t == d && m) {
            MR1L_HIP_TRY(final_coeffs.alloc((size_t)m * 16));
            sf_gather_coeffs(C.prm.dtype, coeffs.p, idx.as<int32_t>(), m, final_coeffs.p, C.st);
            nfinal = m;
        }
        TRY(sync_check(C.st));
        prev = std::move(next);
        nprev = m;
        if (C.stats) {
            C.stats->n_detected[t - 1] = m;
            C.stats->ms_select += ms_since(t0);
        }
    }

    if (nprev == 0) return MR1L_OK;
    *n_out = nprev;
    const int64_t w = std::min(nprev, cap);
    if (w > 0) {
        DevMem rows;
        MR1L_HIP_TRY(rows.alloc((size_t)nprev * d * sizeof(int32_t)));
        sf_soa_to_rows(C.kt, prev.p, nprev, d, rows.as<int32_t>(), C.st);
        TRY(sync_check(C.st));
        MR1L_HIP_TRY(hipMemcpy(freqs_out, rows.p, (size_t)w * d * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (!C.order.empty()) {   // processing order -> the caller's components (rows keep their order)
            std::vector<int32_t> row(d);
            for (int64_t g = 0; g < w; ++g) {
                for (int c = 0; c < d; ++c) row[C.order[c]] = freqs_out[g * d + c];
                std::copy(row.begin(), row.end(), freqs_out + g * d);
            }
        }
        if (nfinal == nprev) MR1L_HIP_TRY(hipMemcpy(coeffs_out, final_coeffs.p, (size_t)w * 16, hipMemcpyDeviceToHost));
    }
    if (nprev > cap) {
        set_error("capacity too small: " + std::to_string(nprev) + " frequencies detected");
        return MR1L_ERR_ARG;
    }
    return MR1L_OK;
}

}  // namespace
}  // namespace mr1l

using namespace mr1l;

extern "C" mr1l_status sfft_detect(int d, const int32_t* lo, const int32_t* hi, sfft_sampler_fn sampler, void* user,
                                   const sfft_planted* planted, const sfft_params* params, int64_t cap,
                                   int64_t* n_out, int32_t* freqs_out, double* coeffs_out, sfft_stats* stats,
                                   int device) {
    try {
        clear_error();
        if (d < 1 || d > SFFT_MAX_D || !lo || !hi || !params || !n_out || cap < 0 ||
            (cap > 0 && (!freqs_out || !coeffs_out)) || (!planted && !sampler)) {
            set_error("invalid argument to sfft_detect");
            return MR1L_ERR_ARG;
        }
        int64_t box_maxabs = 0;
        for (int t = 0; t < d; ++t) {
            if (lo[t] > hi[t] || (int64_t)hi[t] - lo[t] >= (1 << 20)) {
                set_error("box component " + std::to_string(t) + " must satisfy lo <= hi and hi - lo < 2^20");
                return MR1L_ERR_ARG;
            }
            box_maxabs = std::max<int64_t>(box_maxabs, std::max(std::llabs(lo[t]), std::llabs(hi[t])));
        }
        sfft_params prm = *params;
        std::vector<int> order;
        if (prm.order) {
            std::vector<int> seen(d, 0);
            bool ident = true;
            for (int t = 0; t < d; ++t) {
                const int o = prm.order[t];
                if (o < 0 || o >= d || seen[o]++) {
                    set_error("order must be a permutation of 0..d-1");
                    return MR1L_ERR_ARG;
                }
                ident = ident && o == t;
            }
            if (!ident) order.assign(prm.order, prm.order + d);
        }
        if (prm.redraw < 0) {
            set_error("redraw must be >= 0");
            return MR1L_ERR_ARG;
        }
        if (prm.s_local <= 0) prm.s_local = prm.s;
        if (prm.delta_1d == 0.0) prm.delta_1d = prm.delta;
        if (prm.c <= 0.0) prm.c = 2.0;
        if (prm.gamma <= 0.0) prm.gamma = 0.5;
        if (!(prm.delta >= 0.0) || !(prm.delta_1d >= 0.0) || prm.s < 1 || prm.r < 1 || prm.b < 1 || !(prm.c > 1.0) || !(prm.gamma < 1.0) ||
            (prm.dtype != MR1L_C64 && prm.dtype != MR1L_C128)) {
            set_error("invalid sfft_params");
            return MR1L_ERR_ARG;
        }
        if (planted && (planted->s < 0 || (planted->s > 0 && (!planted->freqs || !planted->coeffs)) ||
                        !(planted->sigma >= 0.0))) {
            set_error("invalid planted polynomial");
            return MR1L_ERR_ARG;
        }
        MR1L_HIP_TRY(hipSetDevice(device));
        Ctx C{};
        C.d = d;
        C.lo = lo;
        C.hi = hi;
        if (!order.empty()) {
            C.order = order;
            C.plo.resize(d);
            C.phi.resize(d);
            for (int t = 0; t < d; ++t) {
                C.plo[t] = lo[order[t]];
                C.phi[t] = hi[order[t]];
            }
            C.lo = C.plo.data();
            C.hi = C.phi.data();
            if (sampler && !planted) MR1L_HIP_TRY(C.dcol.upload(order.data(), order.size() * sizeof(int)));
        }
        C.sampler = sampler;
        C.user = user;
        C.planted = planted;
        C.prm = prm;
        C.device = device;
        C.stats = stats;
        C.kt = ktype_for(box_maxabs);
        C.box_maxabs = box_maxabs;
        if (stats) {
            *stats = sfft_stats{};
            stats->d = d;
        }
        if (planted) {
            const int64_t s = planted->s;
            C.s_pl = s;
            std::vector<int32_t> soa((size_t)std::max<int64_t>(1, s) * d);
            for (int64_t h = 0; h < s; ++h)
                for (int c = 0; c < d; ++c) {
                    const int oc = C.order.empty() ? c : C.order[c];   // processing component c
                    soa[(size_t)c * s + h] = planted->freqs[h * d + oc];
                    C.pl_maxabs = std::max<int64_t>(C.pl_maxabs, std::llabs(planted->freqs[h * d + oc]));
                }
            MR1L_HIP_TRY(C.hf.upload(soa.data(), soa.size() * sizeof(int32_t)));
            MR1L_HIP_TRY(C.hc.upload(planted->coeffs, (size_t)std::max<int64_t>(1, s) * 16));
        }
        hipStream_t st = nullptr;
        MR1L_HIP_TRY(hipStreamCreate(&st));
        C.st = st;
        auto t0 = std::chrono::steady_clock::now();
        bool unc = false;
        mr1l_status res = run(C, cap, n_out, freqs_out, coeffs_out, &unc);
        hipStreamSynchronize(st);
        (void)TableStager::settle(TableStager::DRIVER);   // its last copies ran on st
        hipStreamDestroy(st);
        if (stats) stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (res == MR1L_OK && unc) res = MR1L_WARN_UNCOVERED;
        return res;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return MR1L_ERR_NOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return MR1L_ERR_ARG;
    }
}
