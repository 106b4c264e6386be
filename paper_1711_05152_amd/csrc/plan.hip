// Plans and the transform entry points of libmr1l (Alg. 2 and its adjoint).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <tuple>
#include <numeric>
#include <string>

#include "runtime.h"

namespace mr1l {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

static const char* kStageNames[MR1L_NSTAGES] = {"alias_hist", "bluestein_small", "bluestein_p1", "bluestein_p2",
                                                "bluestein_p3", "gather",        "scatter",      "inblock_small"};

// Group streams from this many Bluestein points on: the 512-transform batch (about 2^30 points)
// gains 2 % from them, while its transforms planned one by one (up to 2^24 points each) lose 8 %
// to the fork and join of every call.
constexpr int64_t kGroupStreamMinPoints = (int64_t)1 << 25;
constexpr int64_t kSplitClassMinPoints = kGroupStreamMinPoints;

// Streams for the concurrent group pipelines, kept per device between plans (plans of the sparse
// FFT come and go at every step; creating streams each time would cost more than the transforms).
// Every stream is created with the default priority.
namespace {
std::mutex g_gs_mu;
std::map<int, std::vector<hipStream_t>> g_gs_free;

hipError_t take_group_streams(int dev, int k, std::vector<hipStream_t>& out) {
    std::lock_guard<std::mutex> lk(g_gs_mu);
    auto& f = g_gs_free[dev];
    while ((int)out.size() < k) {
        if (!f.empty()) {
            out.push_back(f.back());
            f.pop_back();
            continue;
        }
        hipStream_t st;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        out.push_back(st);
    }
    return hipSuccess;
}

void give_group_streams(int dev, std::vector<hipStream_t>& st) {
    for (hipStream_t x : st) (void)hipStreamSynchronize(x);
    std::lock_guard<std::mutex> lk(g_gs_mu);
    auto& f = g_gs_free[dev];
    f.insert(f.end(), st.begin(), st.end());
    st.clear();
}
}  // namespace

Plan::~Plan() {
    if (side) {
        (void)hipStreamSynchronize(side);
        (void)hipStreamDestroy(side);
    }
    if (fork) hipEventDestroy(fork);
    if (join) hipEventDestroy(join);
    if (!gstream.empty()) give_group_streams(device, gstream);
    for (auto e : gdone) hipEventDestroy(e);
    if (gstart) hipEventDestroy(gstart);

    for (auto& r : pending) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : free_events) hipEventDestroy(e);
}

static int ceil_lg(int64_t v) {
    int lg = 0;
    while (((int64_t)1 << lg) < v) ++lg;
    return lg;
}


static mr1l_status check_distinct_rows(const int32_t* f, int64_t n, int d) {
    int64_t a = 0, b = 0;
    if (host::find_equal_rows(f, n, d, &a, &b)) {
        set_error("frequency rows " + std::to_string(a) + " and " + std::to_string(b) + " are equal");
        return MR1L_ERR_ARG;
    }
    return MR1L_OK;
}

template <typename K>
static void pack_soa(const int32_t* f, int64_t n, int d, std::vector<char>& out) {
    out.resize((size_t)n * d * sizeof(K));
    K* o = (K*)out.data();
    for (int64_t g = 0; g < n; ++g)
        for (int c = 0; c < d; ++c) o[(size_t)c * n + g] = (K)f[g * d + c];
}

// Filter spectra of earlier plans, per device: the spectrum of a lattice depends only on (M, the
// Bluestein length, the four-step split, the precision), and the steps of Alg. 3 and repeated
// solves meet the same prime sizes again.  Spectra up to 64 MiB are kept, at most 1 GiB per
// device, least recently used out first; mr1l_memory_cache empties the device's entries.
namespace {
struct FiltKey {
    int dev, dtype, lgN, n3, lgN1;
    int64_t M;
    bool operator<(const FiltKey& o) const {
        return std::tie(dev, dtype, lgN, n3, lgN1, M) < std::tie(o.dev, o.dtype, o.lgN, o.n3, o.lgN1, o.M);
    }
};
struct FiltEntry {
    DevMem buf;
    uint64_t used = 0;
};
constexpr size_t kFiltEntryMax = (size_t)64 << 20;
constexpr size_t kFiltCacheMax = (size_t)1 << 30;
// never destroyed: entries hand their blocks back to the allocator, which must outlive them
std::mutex& fc_mutex() {
    static std::mutex* m = new std::mutex;
    return *m;
}
std::map<FiltKey, FiltEntry>& fc_map() {
    static auto* m = new std::map<FiltKey, FiltEntry>;
    return *m;
}
size_t g_fc_bytes = 0;
uint64_t g_fc_clock = 0;
}  // namespace

void filter_cache_clear(int dev) {
    std::lock_guard<std::mutex> lk(fc_mutex());
    auto& m = fc_map();
    for (auto it = m.begin(); it != m.end();) {
        if (it->first.dev == dev) {
            g_fc_bytes -= it->second.buf.bytes;
            it = m.erase(it);
        } else {
            ++it;
        }
    }
}

// copy every lattice's spectrum from the cache, or (any missing) build them all and remember the
// missing ones; on the stream of the plan's set-up.  New cache entries are complete before this
// returns (plans on other streams may copy from them at once).
template <typename T>
static hipError_t plan_filters(Plan* P, const TxArgs& a, int device, hipStream_t st) {
    const int L = P->L;
    cx<T>* filt = (cx<T>*)P->filt_ptr;
    std::vector<int> miss;
    {
        std::lock_guard<std::mutex> lk(fc_mutex());
        auto& m = fc_map();
        std::vector<std::pair<const FiltEntry*, int>> hits;
        for (int l = 0; l < L; ++l) {
            const LatDesc& D = P->hdesc[l];
            auto it = m.find(FiltKey{device, (int)P->dtype, D.lgN, D.n3, D.lgN1, D.M});
            if (it == m.end()) miss.push_back(l);
            else hits.push_back({&it->second, l});
        }
        if (miss.empty()) {
            std::vector<CopySeg> segs;
            for (auto& h : hits) {
                const LatDesc& D = P->hdesc[h.second];
                segs.push_back(CopySeg{h.first->buf.p, filt + D.filt_off, (uint64_t)bl_len(D) * sizeof(cx<T>)});
                const_cast<FiltEntry*>(h.first)->used = ++g_fc_clock;
            }
            return copy_segments(segs.data(), (int)segs.size(), st);
        }
    }
    hipError_t e = build_filters<T>(P->hdesc.data(), L, a.desc, P->groups, filt, device, st);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(fc_mutex());
    auto& m = fc_map();
    for (int l : miss) {
        const LatDesc& D = P->hdesc[l];
        const size_t bytes = (size_t)bl_len(D) * sizeof(cx<T>);
        const FiltKey key{device, (int)P->dtype, D.lgN, D.n3, D.lgN1, D.M};
        if (bytes > kFiltEntryMax || m.count(key)) continue;
        FiltEntry ent;
        if (ent.buf.alloc(bytes) != hipSuccess) {
            (void)hipGetLastError();
            break;   // no room: the cache is an optimisation only
        }
        e = hipMemcpyAsync(ent.buf.p, filt + D.filt_off, bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        ent.used = ++g_fc_clock;
        g_fc_bytes += bytes;
        m.emplace(key, std::move(ent));
        while (g_fc_bytes > kFiltCacheMax) {
            auto old = m.begin();
            for (auto it = m.begin(); it != m.end(); ++it)
                if (it->second.used < old->second.used) old = it;
            g_fc_bytes -= old->second.buf.bytes;
            m.erase(old);
        }
    }
    // the entries' copies are queued on st: done before another stream may read them
    return miss.empty() ? hipSuccess : hipStreamSynchronize(st);
}

template <typename T>
static mr1l_status plan_create_t(const PlanSpec& sp, Plan** out) {
    auto P = new Plan();
    std::unique_ptr<Plan> guard(P);
    P->device = sp.device;
    P->d = sp.d;
    P->dtype = sp.dtype;
    P->weights = sp.weights;
    P->n_rhs = sp.n_rhs;
    const int d = sp.d;
    const int ntx = (int)sp.tx_n.size();
    int64_t n = 0;
    int L = 0;
    for (int i = 0; i < ntx; ++i) {
        n += sp.tx_n[i];
        L += sp.tx_L[i];
    }
    P->n = n;
    P->L = L;
    MR1L_HIP_TRY(hipSetDevice(sp.device));
    TableStager stg(TableStager::PLAN);   // host tables -> device, flushed before the first kernel

    // ---- frequencies ----
    int64_t maxabs = 0;
    int ktype = K_I32;
    if (sp.host_freqs) {
        for (int64_t i = 0; i < n * d; ++i) maxabs = std::max<int64_t>(maxabs, std::llabs((int64_t)sp.host_freqs[i]));
        if (sp.check_distinct) {
            int64_t off = 0;
            for (int i = 0; i < ntx; ++i) {
                mr1l_status st = check_distinct_rows(sp.host_freqs + off * d, sp.tx_n[i], d);
                if (st != MR1L_OK) return st;
                off += sp.tx_n[i];
            }
        }
        ktype = maxabs <= 127 ? K_I8 : (maxabs <= 32767 ? K_I16 : K_I32);
        std::vector<char> packed;
        if (ktype == K_I8) pack_soa<int8_t>(sp.host_freqs, n, d, packed);
        else if (ktype == K_I16) pack_soa<int16_t>(sp.host_freqs, n, d, packed);
        else pack_soa<int32_t>(sp.host_freqs, n, d, packed);
        MR1L_HIP_TRY(stg.add(P->freqs, packed.data(), packed.size()));
        P->args.fv.f = P->freqs.p;
    } else {
        ktype = sp.dev_ktype;
        maxabs = sp.dev_maxabs;
        P->args.fv.f = sp.dev_freqs;
    }
    P->args.fv.ktype = ktype;
    P->args.fv.d = d;
    P->args.fv.nf = n;

    // ---- lattices ----
    int64_t maxM = 1;
    std::vector<int64_t> zred((size_t)L * d);
    for (int l = 0; l < L; ++l) {
        const int64_t M = sp.M[l];
        if (M < 1) {
            set_error("lattice size M must be >= 1");
            return MR1L_ERR_ARG;
        }
        if (M >= ((int64_t)1 << 23)) {
            set_error("lattice size " + std::to_string(M) + " exceeds the supported maximum 2^23 - 1");
            return MR1L_ERR_UNSUPPORTED;
        }
        maxM = std::max(maxM, M);
        for (int c = 0; c < d; ++c) {
            int64_t v = sp.z[(size_t)l * d + c] % M;
            if (v < 0) v += M;
            zred[(size_t)l * d + c] = v;
        }
    }
    const long double bound = (long double)d * (long double)maxabs * (long double)maxM;
    if (bound >= 0x1.0p62L) {
        set_error("d * max|k| * max M >= 2^62: residues would overflow int64");
        return MR1L_ERR_OVERFLOW;
    }
    P->args.fast_mod = bound < 0x1.0p52L;
    P->args.narrow = d <= 32 && maxabs < ((int64_t)1 << 23) && bound < 0x1.0p31L && n < ((int64_t)1 << 31);
    if (P->args.narrow) {
        const int zp = d <= 8 ? 8 : d <= 12 ? 12 : d <= 16 ? 16 : d <= 24 ? 24 : 32;
        const int zrow = zp <= 16 ? 16 : 32;   // row stride of the table, >= every kernel's width
        std::vector<int32_t> z32((size_t)std::max(1, L) * zrow, 0);
        for (int l = 0; l < L; ++l)
            for (int c = 0; c < d; ++c) z32[(size_t)l * zrow + c] = (int32_t)zred[(size_t)l * d + c];
        MR1L_HIP_TRY(stg.add(P->z32, z32.data(), z32.size() * sizeof(int32_t)));
        P->args.zpad = zp;
        P->args.zrow = zrow;
        P->args.z32 = P->z32.as<int32_t>();
    }

    P->hdesc.resize(L);
    P->samp_off.assign(L + 1, 0);
    int64_t woff = 0, bmoff = 0;
    std::map<int, std::vector<int>> by_len;   // Bluestein length (2 lgN + n3) -> lattices
    // A power-of-two class 2^lg turns into 3 * 2^(lg - 2) only when every lattice of the transform in
    // it fits (2M - 1 <= 3 * 2^(lg - 2)): a class split over two lengths runs twice the launches,
    // each with half the tiles, which costs more on the GPU than the 25 % fewer points save.  The
    // choice is per transform, so that a transform of a batched plan gets the bits of its own plan.
    std::vector<int> lat_tx(L);
    for (int i = 0, l = 0; i < ntx; ++i)
        for (int k = 0; k < sp.tx_L[i]; ++k) lat_tx[l++] = i;
    // A large transform (at least 2^25 power-of-two points times right-hand sides) splits a class:
    // its launches carry enough tiles that two lengths on two streams cost nothing extra, so every
    // lattice that fits takes the factor-3 length.
    std::vector<int64_t> tx_pts(ntx, 0);
    for (int l = 0; l < L; ++l) tx_pts[lat_tx[l]] += (int64_t)1 << ceil_lg(2 * sp.M[l] - 1);
    std::set<std::pair<int, int>> no3;   // (transform, class) with a lattice above 3 * 2^(lg - 2)
    for (int l = 0; l < L; ++l) {
        const int lg = ceil_lg(2 * sp.M[l] - 1);
        if (tx_pts[lat_tx[l]] * sp.n_rhs >= kSplitClassMinPoints) continue;
        if (lg - 2 >= kMinLg3 && lg - 2 <= kMaxLg3 && (3LL << (lg - 2)) < 2 * sp.M[l] - 1) no3.insert({lat_tx[l], lg});
    }
    for (int l = 0; l < L; ++l) {
        LatDesc& D = P->hdesc[l];
        D.M = sp.M[l];
        D.invM = 1.0 / (double)D.M;
        D.samp_off = P->samp_off[l];
        P->samp_off[l + 1] = P->samp_off[l] + D.M;
        D.lgN = ceil_lg(2 * D.M - 1);
        D.n3 = 0;
        if (fft_smooth_class(sp.dtype, D.lgN) && !no3.count({lat_tx[l], D.lgN}) &&
            (3LL << (D.lgN - 2)) >= 2 * D.M - 1) {
            D.lgN -= 2;   // N = 3 * 2^(lgN - 2) < 2^lgN still covers 2M - 1
            D.n3 = 1;
        }
        D.small = !D.n3 && D.lgN <= kSmallMaxLg;
        D.lgN1 = D.small ? 0 : (D.n3 ? split3_lgN1(D.lgN) : fft_split(sp.dtype, D.lgN));
        D.lgN2 = D.lgN - D.lgN1;
        D.work_off = woff;
        D.filt_off = woff;
        woff += bl_len(D);
        D.bm_words = (D.M + 31) / 32;
        D.bm_off = bmoff;
        bmoff += 2 * D.bm_words;
        D.zoff = (int64_t)l * d;
        by_len[2 * D.lgN + D.n3].push_back(l);
    }
    P->sum_M = P->samp_off[L];
    P->work_stride = woff;
    P->filt_total = woff;
    P->bm_total = bmoff;

    P->htx.resize(ntx);
    std::vector<int64_t> foff(ntx + 1, 0);
    int lat = 0, max_nlat = 0;
    for (int i = 0; i < ntx; ++i) {
        P->htx[i].foff = foff[i];
        P->htx[i].fn = sp.tx_n[i];
        P->htx[i].lat0 = lat;
        P->htx[i].nlat = sp.tx_L[i];
        foff[i + 1] = foff[i] + sp.tx_n[i];
        lat += sp.tx_L[i];
        max_nlat = std::max(max_nlat, sp.tx_L[i]);
    }

    for (int i = 0; i < ntx; ++i)
        for (int l = P->htx[i].lat0; l < P->htx[i].lat0 + P->htx[i].nlat; ++l) P->hdesc[l].tx = i;
    // transforms of a batched plan (Alg. 2 weights, one right-hand side) whose lattices all take
    // the one-block Bluestein path and whose frequencies fit one workgroup's LDS run whole in the
    // persistent in-block kernel, largest first so that the queue drains evenly
    std::vector<int> inblock;
    if (ntx > 1 && sp.weights == MR1L_W_PAPER && sp.n_rhs == 1 && batch_inblock_enabled()) {
        for (int i = 0; i < ntx; ++i) {
            TxDesc& t = P->htx[i];
            bool ok = t.nlat >= 1 && t.fn >= 1 && t.fn <= kFusedTxMaxN;
            for (int l = t.lat0; ok && l < t.lat0 + t.nlat; ++l) ok = P->hdesc[l].small;
            if (ok) {
                t.in_block = 1;
                inblock.push_back(i);
            }
        }
        std::stable_sort(inblock.begin(), inblock.end(), [&](int x, int y) {
            return P->htx[x].fn * P->htx[x].nlat > P->htx[y].fn * P->htx[y].nlat;
        });
    }
    P->n_inblock = (int)inblock.size();
    if (P->n_inblock > 0) {
        MR1L_HIP_TRY(stg.add(P->inblock, inblock.data(), inblock.size() * sizeof(int)));
        const int zero[2] = {0, 0};
        MR1L_HIP_TRY(stg.add(P->queue, zero, sizeof(zero)));
        // default priority, like every stream of the library
        MR1L_HIP_TRY(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking));
        MR1L_HIP_TRY(hipEventCreateWithFlags(&P->fork, hipEventDisableTiming));
        MR1L_HIP_TRY(hipEventCreateWithFlags(&P->join, hipEventDisableTiming));
    }
    MR1L_HIP_TRY(stg.add(P->tx, P->htx.data(), P->htx.size() * sizeof(TxDesc)));
    MR1L_HIP_TRY(stg.add(P->tx_foff, foff.data(), foff.size() * sizeof(int64_t)));
    MR1L_HIP_TRY(stg.add(P->z, zred.data(), zred.size() * sizeof(int64_t)));
    {
        std::vector<int> ids;
        std::vector<std::pair<int, int>> spans;   // (2 lgN + n3, first index)
        for (auto& kv : by_len) {
            spans.push_back({kv.first, (int)ids.size()});
            ids.insert(ids.end(), kv.second.begin(), kv.second.end());
        }
        MR1L_HIP_TRY(stg.add(P->grp_lat, ids.data(), ids.size() * sizeof(int)));
        for (size_t i = 0; i < spans.size(); ++i) {
            FftGroup g;
            g.lgN = spans[i].first >> 1;
            g.n3 = spans[i].first & 1;
            g.small = !g.n3 && g.lgN <= kSmallMaxLg;
            g.lg1 = P->hdesc[by_len[spans[i].first][0]].lgN1;
            g.p2v = (g.small || g.n3) ? 0 : fft_p2_variant(sp.dtype, g.lgN, g.lg1);
            g.nlat = (int)by_len[spans[i].first].size();
            g.lat = P->grp_lat.as<int>() + spans[i].second;
            P->groups.push_back(g);
        }
        // execution groups: the lattices of in-block transforms are done by the persistent kernel
        if (P->n_inblock == 0) {
            P->sweep = P->groups;
        } else {
            std::vector<int> sids;
            std::vector<std::pair<const FftGroup*, std::pair<int, int>>> sspans;
            for (size_t i = 0; i < spans.size(); ++i) {
                const int first = (int)sids.size();
                for (int l : by_len[spans[i].first])
                    if (!P->htx[P->hdesc[l].tx].in_block) sids.push_back(l);
                if ((int)sids.size() > first) sspans.push_back({&P->groups[i], {first, (int)sids.size() - first}});
            }
            if (!sids.empty()) MR1L_HIP_TRY(stg.add(P->sweep_lat, sids.data(), sids.size() * sizeof(int)));
            for (auto& sg : sspans) {
                FftGroup g = *sg.first;
                g.nlat = sg.second.second;
                g.lat = P->sweep_lat.as<int>() + sg.second.first;
                P->sweep.push_back(g);
            }
        }
        // only where the groups carry enough work (kGroupStreamMinPoints)
        int n4 = 0;
        int64_t pts = 0;
        for (const FftGroup& g : P->sweep) n4 += !g.small;
        for (int l = 0; l < L; ++l)
            if (!P->hdesc[l].small && !P->htx[P->hdesc[l].tx].in_block) pts += bl_len(P->hdesc[l]);
        if (n4 >= 2 && pts * sp.n_rhs >= kGroupStreamMinPoints) {
            const int k = std::min(n4 - 1, kGroupStreams);
            MR1L_HIP_TRY(take_group_streams(P->device, k, P->gstream));
            MR1L_HIP_TRY(hipEventCreateWithFlags(&P->gstart, hipEventDisableTiming));
            P->gdone.assign(k, nullptr);
            for (auto& e : P->gdone) MR1L_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
    }
    // alias-histogram tiles: every lattice's bins split into ranges of <= 2^18 bins (multiples of
    // 32), enough of them that a few hundred workgroups run.  Every tile streams all residues of its
    // lattice, so with >= 8 lattices the tiles of lattice l are placed on workgroup slots
    // b = l (mod 8): workgroups are dealt to the 8 XCDs round-robin, so each lattice's residues are
    // then read into one XCD's L2 only (idle slots pad uneven groups).
    std::vector<HistTile> tiles;
    int hist_words = 1;
    {
        const int rpl = std::max(1, std::min(16, (256 + L - 1) / std::max(1, L)));
        std::vector<std::vector<HistTile>> byx(L >= 8 ? 8 : 1);
        int txi = 0;
        for (int l = 0; l < L; ++l) {
            while (txi + 1 < ntx && l >= P->htx[txi].lat0 + P->htx[txi].nlat) ++txi;
            const int64_t M = P->hdesc[l].M;
            int64_t nr = std::max<int64_t>((M + kHistMaxBins - 1) / kHistMaxBins, rpl);
            nr = std::min<int64_t>(nr, (M + 31) / 32);
            int64_t step = ((M + nr - 1) / nr + 31) / 32 * 32;
            hist_words = std::max<int>(hist_words, (int)(step / 32));
            for (int64_t m0 = 0; m0 < M; m0 += step)
                byx[l % byx.size()].push_back(HistTile{l, txi, (int32_t)m0, (int32_t)std::min(M, m0 + step)});
        }
        size_t most = 0;
        for (auto& v : byx) most = std::max(most, v.size());
        for (size_t i = 0; i < most; ++i)
            for (auto& v : byx) tiles.push_back(i < v.size() ? v[i] : HistTile{-1, 0, 0, 0});
    }
    MR1L_HIP_TRY(stg.add(P->hist, tiles.data(), tiles.size() * sizeof(HistTile)));
    // fused residue + histogram tiles: each lattice's frequencies split into chunks of one
    // workgroup iteration, each counted over all bins of the lattice in LDS
    bool fused = L > 0 && n < ((int64_t)1 << 31);   // 32-bit frequency offsets inside the kernel
    int rt_words = 1;
    for (int l = 0; l < L; ++l) fused = fused && P->hdesc[l].bm_words <= kFusedMaxWords;
    std::vector<ResTile> rtiles;
    int64_t part_words = 0;
    if (fused) {
        int txi = 0;
        for (int l = 0; l < L; ++l) {
            while (txi + 1 < ntx && l >= P->htx[txi].lat0 + P->htx[txi].nlat) ++txi;
            LatDesc& D = P->hdesc[l];
            const int64_t fn = P->htx[txi].fn, words = D.bm_words;
            rt_words = std::max<int>(rt_words, (int)words);
            const int64_t ch = (int64_t)kResThreads * res_unroll(P->args.narrow ? P->args.zpad : 0);
            D.rt0 = (int32_t)rtiles.size();
            for (int64_t k0 = 0; k0 < fn; k0 += ch) {
                rtiles.push_back(ResTile{P->htx[txi].foff + k0, P->htx[txi].foff + std::min(fn, k0 + ch), part_words,
                                         l, txi});
                part_words += 2 * words;
            }
            if (fn == 0) {   // one empty tile still clears the bitmaps
                rtiles.push_back(ResTile{P->htx[txi].foff, P->htx[txi].foff, part_words, l, txi});
                part_words += 2 * words;
            }
            D.rtn = (int32_t)rtiles.size() - D.rt0;
        }
        MR1L_HIP_TRY(stg.add(P->rtiles, rtiles.data(), rtiles.size() * sizeof(ResTile)));
        MR1L_HIP_TRY(P->part.alloc((size_t)std::max<int64_t>(1, part_words) * sizeof(uint32_t)));
    }
    const int64_t rstride = (n + 3) / 4 * 4;
    MR1L_HIP_TRY(P->res32.alloc((size_t)std::max<int64_t>(4, (int64_t)max_nlat * rstride) * sizeof(int32_t)));
    MR1L_HIP_TRY(P->bitmaps.alloc((size_t)std::max<int64_t>(1, P->bm_total) * sizeof(uint32_t)));
    const Plan* sh = sp.share_filters;
    if (sh) {
        bool same = sh->dtype == sp.dtype && sh->L == L;
        for (int l = 0; same && l < L; ++l)
            same = sh->hdesc[l].M == P->hdesc[l].M && sh->hdesc[l].lgN == P->hdesc[l].lgN &&
                   sh->hdesc[l].n3 == P->hdesc[l].n3 && sh->hdesc[l].lgN1 == P->hdesc[l].lgN1;
        if (!same) {
            set_error("share_filters: lattice sizes, four-step splits or dtype differ");
            return MR1L_ERR_ARG;
        }
        P->filt_ptr = sh->filt_ptr;
    } else {
        MR1L_HIP_TRY(P->filt.alloc((size_t)std::max<int64_t>(1, P->filt_total) * sizeof(cx<T>)));
        P->filt_ptr = P->filt.p;
    }
    {
        const int64_t per_rhs = std::max<int64_t>(1, P->work_stride) * (int64_t)sizeof(cx<T>);
        P->rhs_chunk = std::max<int64_t>(1, std::min<int64_t>(P->n_rhs, sp.max_work_bytes / per_rhs));
    }
    MR1L_HIP_TRY(P->work.alloc((size_t)std::max<int64_t>(1, P->work_stride * P->rhs_chunk) * sizeof(cx<T>)));
    // Fourier-matrix adjoint by counting sort: every bin is summed by one thread in ascending k,
    // so the synthesis is bit-reproducible from run to run (floating-point atomics are kept only for
    // plans beyond the sort's 32-bit positions)
    P->args.bsort = sp.weights == MR1L_W_EVAL && (int64_t)n * max_nlat < ((int64_t)1 << 31) &&
                    P->sum_M < ((int64_t)1 << 31);
    if (P->args.bsort) {
        const int64_t nchunks = (P->sum_M + kScanChunk - 1) / kScanChunk;
        MR1L_HIP_TRY(P->bcnt.alloc((size_t)P->sum_M * sizeof(int32_t)));
        MR1L_HIP_TRY(hipMemsetAsync(P->bcnt.p, 0, (size_t)P->sum_M * sizeof(int32_t), sp.stream));
        MR1L_HIP_TRY(P->bloc.alloc((size_t)P->sum_M * sizeof(int32_t)));
        MR1L_HIP_TRY(P->bbase.alloc((size_t)std::max<int64_t>(1, nchunks) * sizeof(int32_t)));
        MR1L_HIP_TRY(P->perm.alloc((size_t)std::max<int64_t>(4, (int64_t)max_nlat * rstride) * sizeof(int32_t)));
        P->args.bcnt = P->bcnt.as<int32_t>();
        P->args.bloc = P->bloc.as<int32_t>();
        P->args.bbase = P->bbase.as<int32_t>();
        P->args.perm = P->perm.as<int32_t>();
    }
    // right-hand-side interleaving for the gather and the bin sums of passes with several
    // right-hand sides: 64 bytes per bin or coefficient, within the work-area bound
    P->args.ilv = nullptr;
    P->args.ilv_bins = P->args.ilv_coef = false;
    {
        const int mode = rhs_interleave_mode();
        const int64_t pass = P->rhs_chunk * (int64_t)sizeof(cx<T>);
        if (mode > 0 && P->rhs_chunk > 1 && std::max<int64_t>(n, P->sum_M) <= sp.max_work_bytes / 64) {
            P->args.ilv_bins = mode == 2 || P->sum_M * pass >= kIlvBinBytes;
            P->args.ilv_coef = P->args.bsort && (mode == 2 || (int64_t)n * pass >= kIlvCoefBytes);
        }
        if (P->args.ilv_bins || P->args.ilv_coef) {
            MR1L_HIP_TRY(P->ilv.alloc((size_t)std::max<int64_t>(n, P->sum_M) * 64));
            P->args.ilv = P->ilv.p;
        }
    }
    P->args.nbins = P->sum_M;
    P->args.max_M = maxM;

    TxArgs& a = P->args;
    a.desc = P->desc.as<LatDesc>();
    a.L = L;
    a.tx = P->tx.as<TxDesc>();
    a.tx_foff = P->tx_foff.as<int64_t>();
    a.ntx = ntx;
    a.max_nlat = max_nlat;
    a.z = P->z.as<int64_t>();
    a.n = n;
    a.n_rhs = P->rhs_chunk;
    a.samp_stride = P->sum_M;
    a.work_stride = P->work_stride;
    a.bitmaps = P->bitmaps.as<uint32_t>();
    a.bm_total = P->bm_total;
    a.res32 = P->res32.as<int32_t>();
    a.rs = rstride;
    a.hist = P->hist.as<HistTile>();
    a.nhist = (int)tiles.size();
    a.hist_words = hist_words;
    a.fused = fused;
    a.rtiles = P->rtiles.as<ResTile>();
    a.nrt = (int)rtiles.size();
    a.rt_words = rt_words;
    a.part = P->part.as<uint32_t>();

    // lattice descriptors as complete (fused-pass tiles included), then every staged table
    MR1L_HIP_TRY(stg.add(P->desc, P->hdesc.data(), P->hdesc.size() * sizeof(LatDesc)));
    a.desc = P->desc.as<LatDesc>();
    MR1L_HIP_TRY(stg.flush(sp.stream));
    if (!twiddles<T>(sp.device) || !twiddles<double>(sp.device)) {
        set_error("could not allocate twiddle tables");
        return MR1L_ERR_NOMEM;
    }
    if (!sh) MR1L_HIP_TRY(plan_filters<T>(P, a, sp.device, sp.stream));
    MR1L_HIP_TRY(hipGetLastError());
    if (sp.sync) MR1L_HIP_TRY(hipDeviceSynchronize());
    *out = guard.release();
    return MR1L_OK;
}

mr1l_status plan_create(const PlanSpec& sp, Plan** out) {
    if (sp.d < 1 || sp.d > 64) {
        set_error("d must be in 1..64");
        return MR1L_ERR_ARG;
    }
    if (sp.n_rhs < 1) {
        set_error("n_rhs must be >= 1");
        return MR1L_ERR_ARG;
    }
    if (sp.tx_n.size() != sp.tx_L.size() || sp.tx_n.empty()) {
        set_error("inconsistent transform description");
        return MR1L_ERR_ARG;
    }
    return sp.dtype == MR1L_C128 ? plan_create_t<double>(sp, out) : plan_create_t<float>(sp, out);
}

// ---- stage timing ----------------------------------------------------------------------------------
struct StageTimer {
    Plan* p;
    hipStream_t s;
    int stage = -1;
    hipEvent_t a = nullptr;
    StageTimer(Plan* p_, hipStream_t s_) : p(p_), s(s_) {}
    hipEvent_t get() {
        if (!p->free_events.empty()) {
            hipEvent_t e = p->free_events.back();
            p->free_events.pop_back();
            return e;
        }
        hipEvent_t e;
        hipEventCreate(&e);
        return e;
    }
    void begin(int st) {
        if (!p->timing) return;
        stage = st;
        a = get();
        hipEventRecord(a, s);
    }
    void end() {
        if (!p->timing || stage < 0) return;
        hipEvent_t b = get();
        hipEventRecord(b, s);
        p->pending.push_back({stage, a, b});
        stage = -1;
    }
};

// residues (and, for Alg. 2's weights, the alias bitmaps) of every lattice, unless cached
static void index_pass(Plan* p, bool eval, StageTimer& tm, hipStream_t s) {
    if (p->cache_alias && p->alias_valid) return;
    tm.begin(0);
    launch_alias(p->args, !eval, s);
    tm.end();
    p->alias_valid = p->cache_alias;
}

// Fork the in-block launch onto the plan's side stream after the work already queued on s (the
// caller joins with p->join before returning).  With stage timing on, the launch is timed on the
// side stream.
template <typename T>
static hipError_t inblock_begin(Plan* p, const cx<T>* src, cx<T>* dst, bool forward, hipStream_t s) {
    if (p->n_inblock == 0) return hipSuccess;
    hipError_t e = hipEventRecord(p->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->fork, 0);
    if (e != hipSuccess) return e;
    StageTimer tm(p, p->side);
    tm.begin(7);
    launch_fused_small<T>(p->args, p->inblock.as<int>(), p->n_inblock, p->queue.as<int>(), src, dst,
                          (const cx<T>*)p->filt_ptr, forward, p->side);
    tm.end();
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(p->join, p->side);
    return e;
}

// The four-step groups of one pass: the first on s, the others round-robin on the plan's group
// streams, which wait for everything queued on s so far and are waited for by s at the end.  Each
// group touches only its own lattices' work regions, filters and samples.  With stage timing on,
// everything stays on s so that the per-stage events bracket single launches.
struct GroupFork {
    Plan* p;
    hipStream_t s;
    int k = 0;
    bool on = false;
    GroupFork(Plan* p_, hipStream_t s_) : p(p_), s(s_) {}
    hipError_t begin() {
        on = !p->gstream.empty() && !p->timing;
        if (!on) return hipSuccess;
        hipError_t e = hipEventRecord(p->gstart, s);
        for (size_t i = 0; e == hipSuccess && i < p->gstream.size(); ++i) e = hipStreamWaitEvent(p->gstream[i], p->gstart, 0);
        return e;
    }
    hipStream_t next() {
        if (!on) return s;
        const int i = k++;
        return i == 0 ? s : p->gstream[(i - 1) % p->gstream.size()];
    }
    hipError_t end() {
        if (!on) return hipSuccess;
        hipError_t e = hipSuccess;
        for (size_t i = 0; e == hipSuccess && i < p->gstream.size(); ++i) {
            e = hipEventRecord(p->gdone[i], p->gstream[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, p->gdone[i], 0);
        }
        return e;
    }
};

// A group's stage pipeline runs in pieces (a lattice range times a right-hand-side range) whose
// Bluestein work regions together stay within a share of the 256 MB Infinity Cache, so that stage
// 2 reads what stage 1 wrote, and stage 3 what stage 2 wrote, from there instead of from HBM.
// Groups whose regions fit anyway run as one piece, and so do passes of one right-hand side (a
// batch of transforms: the many short launches there slowed the eager call beside the in-block
// kernel and gained nothing).
constexpr int64_t kPieceCacheBytes = (int64_t)192 << 20;
struct Piece {
    int l0, nl;
    int64_t q0, nq;
};
template <typename T>
static void group_pieces(const FftGroup& g, int64_t nrhs, int conc, std::vector<Piece>& out) {
    out.clear();
    const int64_t region = ((int64_t)(g.n3 ? 3 : 1) << g.lgN) * (int64_t)sizeof(cx<T>);
    const int64_t k = std::max<int64_t>(1, kPieceCacheBytes / std::max(1, conc) / region);   // regions per piece
    if (nrhs == 1 || (int64_t)g.nlat * nrhs <= 2 * k) {
        out.push_back(Piece{0, g.nlat, 0, nrhs});
        return;
    }
    if (nrhs >= k) {   // one lattice, its right-hand sides in even parts of at most k
        const int64_t parts = (nrhs + k - 1) / k, per = (nrhs + parts - 1) / parts;
        for (int l = 0; l < g.nlat; ++l)
            for (int64_t q = 0; q < nrhs; q += per) out.push_back(Piece{l, 1, q, std::min(per, nrhs - q)});
    } else {           // every right-hand side, lattices in even parts of at most k / nrhs
        const int most = (int)std::max<int64_t>(1, k / nrhs);
        const int parts = (g.nlat + most - 1) / most, per = (g.nlat + parts - 1) / parts;
        for (int l = 0; l < g.nlat; l += per) out.push_back(Piece{l, std::min(per, g.nlat - l), 0, nrhs});
    }
}

// stage pipelines running at once: the caller's stream plus the group streams in use
static int concurrent_pipelines(const Plan* p, const GroupFork& gf) {
    if (!gf.on) return 1;
    int n4 = 0;
    for (const FftGroup& g : p->sweep) n4 += !g.small;
    return std::max(1, std::min(n4, (int)p->gstream.size() + 1));
}

template <typename T>
static mr1l_status forward_t(Plan* p, const cx<T>* y, cx<T>* c, hipStream_t s) {
    const bool eval = p->weights == MR1L_W_EVAL;
    cx<T>* work = p->work.as<cx<T>>();
    const cx<T>* filt = (const cx<T>*)p->filt_ptr;
    StageTimer tm(p, s);
    std::vector<Piece> pieces;
    // small transforms of a batch, whole, in one persistent launch on the side stream, beside the
    // stage sweep of the others (they share no data)
    MR1L_HIP_TRY(inblock_begin<T>(p, y, c, true, s));
    index_pass(p, eval, tm, s);
    for (int64_t r0 = 0; r0 < p->n_rhs; r0 += p->rhs_chunk) {
        TxArgs a = p->args;
        a.n_rhs = std::min(p->rhs_chunk, p->n_rhs - r0);
        const cx<T>* yc = y + r0 * a.samp_stride;
        cx<T>* cc = c + r0 * a.n;
        GroupFork gf(p, s);
        MR1L_HIP_TRY(gf.begin());
        for (const FftGroup& g : p->sweep) {
            if (g.small) {
                tm.begin(1);
                launch_bluestein_small<T>(a, g, yc, a.samp_stride, true, work, filt, work, a.work_stride, false, -1,
                                          !eval, false, s);
                tm.end();
                continue;
            }
            const hipStream_t gs = gf.next();
            group_pieces<T>(g, a.n_rhs, concurrent_pipelines(p, gf), pieces);
            for (const Piece& pc : pieces) {
                TxArgs b = a;
                b.n_rhs = pc.nq;
                FftGroup h = g;
                h.lat = g.lat + pc.l0;
                h.nlat = pc.nl;
                const cx<T>* yq = yc + pc.q0 * a.samp_stride;
                cx<T>* wq = work + pc.q0 * a.work_stride;
                tm.begin(2);
                launch_p1<T>(b, h, yq, a.samp_stride, true, wq, -1, false, gs);
                tm.end();
                tm.begin(3);
                launch_p2<T>(b, h, wq, filt, -1, yq, nullptr, gs);
                tm.end();
                tm.begin(4);
                launch_p3<T>(b, h, wq, wq, a.work_stride, false, -1, !eval, gs);
                tm.end();
            }
        }
        MR1L_HIP_TRY(gf.end());
        tm.begin(5);
        launch_gather<T>(a, work, cc, eval, s);
        tm.end();
    }
    if (p->n_inblock > 0) MR1L_HIP_TRY(hipStreamWaitEvent(s, p->join, 0));
    MR1L_HIP_TRY(hipGetLastError());
    return MR1L_OK;
}

template <typename T>
static mr1l_status adjoint_t(Plan* p, const cx<T>* c, cx<T>* y, hipStream_t s) {
    const bool eval = p->weights == MR1L_W_EVAL;
    cx<T>* work = p->work.as<cx<T>>();
    const cx<T>* filt = (const cx<T>*)p->filt_ptr;
    StageTimer tm(p, s);
    std::vector<Piece> pieces;
    MR1L_HIP_TRY(inblock_begin<T>(p, c, y, false, s));
    index_pass(p, eval, tm, s);
    if (eval && p->args.bsort && !(p->cache_alias && p->sort_valid)) {
        tm.begin(0);
        launch_bin_sort(p->args, s);
        tm.end();
        p->sort_valid = p->cache_alias;
    }
    for (int64_t r0 = 0; r0 < p->n_rhs; r0 += p->rhs_chunk) {
        TxArgs a = p->args;
        a.n_rhs = std::min(p->rhs_chunk, p->n_rhs - r0);
        const cx<T>* cc = c + r0 * a.n;
        cx<T>* yc = y + r0 * a.samp_stride;
        tm.begin(6);
        if (eval && a.bsort) {
            launch_bin_sum<T>(a, cc, work, s);
        } else {
            if (eval) launch_clear_bins<T>(a, work, s);
            launch_scatter<T>(a, cc, work, eval, s);
        }
        tm.end();
        GroupFork gf(p, s);
        MR1L_HIP_TRY(gf.begin());
        for (const FftGroup& g : p->sweep) {
            if (g.small) {
                tm.begin(1);
                launch_bluestein_small<T>(a, g, work, a.work_stride, false, work, filt, yc, a.samp_stride, true, +1,
                                          !eval, !eval, s);
                tm.end();
                continue;
            }
            const hipStream_t gs = gf.next();
            group_pieces<T>(g, a.n_rhs, concurrent_pipelines(p, gf), pieces);
            for (const Piece& pc : pieces) {
                TxArgs b = a;
                b.n_rhs = pc.nq;
                FftGroup h = g;
                h.lat = g.lat + pc.l0;
                h.nlat = pc.nl;
                cx<T>* yq = yc + pc.q0 * a.samp_stride;
                cx<T>* wq = work + pc.q0 * a.work_stride;
                tm.begin(2);
                launch_p1<T>(b, h, wq, a.work_stride, false, wq, +1, !eval, gs);
                tm.end();
                tm.begin(3);
                launch_p2<T>(b, h, wq, filt, +1, nullptr, yq, gs);
                tm.end();
                tm.begin(4);
                launch_p3<T>(b, h, wq, yq, a.samp_stride, true, +1, !eval, gs);
                tm.end();
            }
        }
        MR1L_HIP_TRY(gf.end());
    }
    if (p->n_inblock > 0) MR1L_HIP_TRY(hipStreamWaitEvent(s, p->join, 0));
    MR1L_HIP_TRY(hipGetLastError());
    return MR1L_OK;
}

mr1l_status plan_forward(Plan* p, const void* samples, void* coeffs, hipStream_t s) {
    if (p->dtype == MR1L_C128) return forward_t<double>(p, (const cx<double>*)samples, (cx<double>*)coeffs, s);
    return forward_t<float>(p, (const cx<float>*)samples, (cx<float>*)coeffs, s);
}

mr1l_status plan_adjoint(Plan* p, const void* coeffs, void* samples, hipStream_t s) {
    if (p->dtype == MR1L_C128) return adjoint_t<double>(p, (const cx<double>*)coeffs, (cx<double>*)samples, s);
    return adjoint_t<float>(p, (const cx<float>*)coeffs, (cx<float>*)samples, s);
}

mr1l_status plan_alias(Plan* p, int64_t* res, uint8_t* uniq, uint8_t* counter, hipStream_t s) {
    launch_alias(p->args, true, s);
    p->alias_valid = p->cache_alias;
    launch_alias_export(p->args, res, uniq, counter, s);
    MR1L_HIP_TRY(hipGetLastError());
    return MR1L_OK;
}

}  // namespace mr1l

using namespace mr1l;

#define MR1L_GUARD_BEGIN try {
#define MR1L_GUARD_END                                  \
    }                                                   \
    catch (const std::bad_alloc&) {                     \
        set_error("host allocation failed");            \
        return MR1L_ERR_NOMEM;                          \
    }                                                   \
    catch (const std::exception& ex) {                  \
        set_error(ex.what());                           \
        return MR1L_ERR_ARG;                            \
    }

extern "C" {

const char* mr1l_last_error(void) { return g_err.c_str(); }
const char* mr1l_version(void) { return "mr1l 0.1 (gfx950)"; }

mr1l_status mr1l_plan(int d, int64_t n, const int32_t* freqs, int L, const int64_t* M, const int64_t* z,
                      mr1l_dtype dtype, mr1l_weights weights, int64_t n_rhs, int device, mr1l_plan_t* out) {
    MR1L_GUARD_BEGIN
    clear_error();
    if (!out || n < 0 || L < 0 || (n > 0 && !freqs) || (L > 0 && (!M || !z)) ||
        (dtype != MR1L_C64 && dtype != MR1L_C128) || (weights != MR1L_W_PAPER && weights != MR1L_W_EVAL)) {
        set_error("invalid argument to mr1l_plan");
        return MR1L_ERR_ARG;
    }
    PlanSpec sp;
    sp.d = d;
    sp.dtype = dtype;
    sp.weights = weights;
    sp.n_rhs = n_rhs;
    sp.device = device;
    sp.host_freqs = freqs;
    sp.tx_n = {n};
    sp.tx_L = {L};
    sp.M.assign(M, M + L);
    sp.z.assign(z, z + (size_t)L * (d > 0 ? d : 0));
    Plan* p = nullptr;
    mr1l_status st = plan_create(sp, &p);
    if (st == MR1L_OK) *out = (mr1l_plan_t)p;
    return st;
    MR1L_GUARD_END
}

mr1l_status mr1l_plan_batched(int d, int n_tx, const int64_t* n, const int32_t* freqs, const int32_t* L,
                              const int64_t* M, const int64_t* z, mr1l_dtype dtype, mr1l_weights weights,
                              int64_t n_rhs, int device, mr1l_plan_t* out) {
    MR1L_GUARD_BEGIN
    clear_error();
    if (!out || n_tx < 1 || !n || !L || (dtype != MR1L_C64 && dtype != MR1L_C128) ||
        (weights != MR1L_W_PAPER && weights != MR1L_W_EVAL) || d < 1 || d > 64) {
        set_error("invalid argument to mr1l_plan_batched");
        return MR1L_ERR_ARG;
    }
    int64_t ntot = 0, Ltot = 0;
    for (int i = 0; i < n_tx; ++i) {
        if (n[i] < 0 || L[i] < 0) {
            set_error("negative size in mr1l_plan_batched");
            return MR1L_ERR_ARG;
        }
        ntot += n[i];
        Ltot += L[i];
    }
    if ((ntot > 0 && !freqs) || (Ltot > 0 && (!M || !z))) {
        set_error("null array in mr1l_plan_batched");
        return MR1L_ERR_ARG;
    }
    PlanSpec sp;
    sp.d = d;
    sp.dtype = dtype;
    sp.weights = weights;
    sp.n_rhs = n_rhs;
    sp.device = device;
    sp.host_freqs = freqs;
    sp.tx_n.assign(n, n + n_tx);
    sp.tx_L.assign(L, L + n_tx);
    sp.M.assign(M, M + Ltot);
    sp.z.assign(z, z + (size_t)Ltot * d);
    Plan* p = nullptr;
    mr1l_status st = plan_create(sp, &p);
    if (st == MR1L_OK) *out = (mr1l_plan_t)p;
    return st;
    MR1L_GUARD_END
}

mr1l_status mr1l_forward(mr1l_plan_t plan, const void* samples, void* coeffs, void* stream) {
    MR1L_GUARD_BEGIN
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || (p->sum_M > 0 && !samples) || (p->n > 0 && !coeffs)) {
        set_error("invalid argument to mr1l_forward");
        return MR1L_ERR_ARG;
    }
    MR1L_HIP_TRY(hipSetDevice(p->device));
    return plan_forward(p, samples, coeffs, (hipStream_t)stream);
    MR1L_GUARD_END
}

mr1l_status mr1l_adjoint(mr1l_plan_t plan, const void* coeffs, void* samples, void* stream) {
    MR1L_GUARD_BEGIN
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || (p->sum_M > 0 && !samples) || (p->n > 0 && !coeffs)) {
        set_error("invalid argument to mr1l_adjoint");
        return MR1L_ERR_ARG;
    }
    MR1L_HIP_TRY(hipSetDevice(p->device));
    return plan_adjoint(p, coeffs, samples, (hipStream_t)stream);
    MR1L_GUARD_END
}

mr1l_status mr1l_alias(mr1l_plan_t plan, int64_t* residues, uint8_t* unaliased, uint8_t* counter, void* stream) {
    MR1L_GUARD_BEGIN
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p) {
        set_error("null plan");
        return MR1L_ERR_ARG;
    }
    MR1L_HIP_TRY(hipSetDevice(p->device));
    return plan_alias(p, residues, unaliased, counter, (hipStream_t)stream);
    MR1L_GUARD_END
}

mr1l_status mr1l_info(mr1l_plan_t plan, int64_t* sample_offsets, int64_t* n_uncovered, int64_t* fft_lengths) {
    MR1L_GUARD_BEGIN
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p) {
        set_error("null plan");
        return MR1L_ERR_ARG;
    }
    if (sample_offsets) std::copy(p->samp_off.begin(), p->samp_off.end(), sample_offsets);
    if (fft_lengths)
        for (int l = 0; l < p->L; ++l) fft_lengths[l] = bl_len(p->hdesc[l]);
    if (n_uncovered) {
        MR1L_HIP_TRY(hipSetDevice(p->device));
        DevMem cnt;
        MR1L_HIP_TRY(cnt.alloc((size_t)std::max<int64_t>(1, p->n)));
        mr1l_status st = plan_alias(p, nullptr, nullptr, cnt.as<uint8_t>(), nullptr);
        if (st != MR1L_OK) return st;
        std::vector<uint8_t> h((size_t)p->n);
        if (p->n) MR1L_HIP_TRY(hipMemcpy(h.data(), cnt.p, (size_t)p->n, hipMemcpyDeviceToHost));
        int64_t u = 0;
        for (uint8_t v : h) u += (v == 0);
        *n_uncovered = u;
    }
    return MR1L_OK;
    MR1L_GUARD_END
}

mr1l_status mr1l_cache_alias(mr1l_plan_t plan, int enable) {
    clear_error();
    if (!plan) {
        set_error("plan is NULL");
        return MR1L_ERR_ARG;
    }
    Plan* p = (Plan*)plan;
    p->cache_alias = enable != 0;
    p->alias_valid = false;
    p->sort_valid = false;
    return MR1L_OK;
}

mr1l_status mr1l_destroy(mr1l_plan_t plan) {
    if (!plan) return MR1L_OK;
    Plan* p = (Plan*)plan;
    hipSetDevice(p->device);
    delete p;
    return MR1L_OK;
}

mr1l_status mr1l_timing_enable(mr1l_plan_t plan, int enable) {
    Plan* p = (Plan*)plan;
    if (!p) return MR1L_ERR_ARG;
    p->timing = enable != 0;
    return MR1L_OK;
}

mr1l_status mr1l_timing_read(mr1l_plan_t plan, double* ms_sum, int64_t* launches, const char** names) {
    MR1L_GUARD_BEGIN
    Plan* p = (Plan*)plan;
    if (!p) return MR1L_ERR_ARG;
    MR1L_HIP_TRY(hipSetDevice(p->device));
    for (auto& r : p->pending) {
        MR1L_HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.f;
        MR1L_HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        p->ms_sum[r.stage] += ms;
        p->launches[r.stage] += 1;
        p->free_events.push_back(r.a);
        p->free_events.push_back(r.b);
    }
    p->pending.clear();
    for (int i = 0; i < MR1L_NSTAGES; ++i) {
        if (ms_sum) ms_sum[i] = p->ms_sum[i];
        if (launches) launches[i] = p->launches[i];
        if (names) names[i] = kStageNames[i];
        p->ms_sum[i] = 0;
        p->launches[i] = 0;
    }
    return MR1L_OK;
    MR1L_GUARD_END
}

}  // extern "C"
