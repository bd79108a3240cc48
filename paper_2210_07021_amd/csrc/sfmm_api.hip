// Host driver of libsfmm and its C ABI (include/sfmm.h).  All device work
// is ordered on the caller's stream; the plan reads back only a few counts
// (per tree level and per walk round) to size the next step.
#include "../../include/sfmm.h"
#include "common.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace sfmm;

namespace {
thread_local std::string g_last_error;

// pinned host scratch for the counts read back during planning
struct Pinned {
    int* p = nullptr;
    Pinned() { SFMM_HIP(hipHostMalloc((void**)&p, 64 * sizeof(int), hipHostMallocDefault)); }
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
};

// ---- stage timing (sfmm_profile_*)
enum Stage {
    S_SRC = 0, S_TREE, S_GEOM, S_WALK, S_LISTS, S_TGT, S_P2M, S_M2M, S_M2L, S_L2L, S_L2P, S_P2P, S_M2P, S_COUNT
};
std::atomic<int> g_prof_on{0};
thread_local bool g_capturing = false;  // no stage timing while a graph is recorded
std::mutex g_prof_mu;
double g_prof_ms[S_COUNT];
long long g_prof_calls[S_COUNT];

// Records (stage, start, stop) events on one stream during one API call;
// flush() waits for the stream and adds the elapsed times to the totals.
struct Profiler {
    hipStream_t s;
    bool on;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    // allowed = false: no events at all (the no-allocation entry point)
    explicit Profiler(hipStream_t st, bool allowed = true)
        : s(st), on(allowed && g_prof_on.load() != 0 && !g_capturing) {}
    int begin(int stage) {
        if (!on) return -1;
        Rec r{stage, nullptr, nullptr};
        SFMM_HIP(hipEventCreate(&r.a));
        SFMM_HIP(hipEventCreate(&r.b));
        SFMM_HIP(hipEventRecord(r.a, s));
        recs.push_back(r);
        return (int)recs.size() - 1;
    }
    void end(int id) {
        if (id >= 0) SFMM_HIP(hipEventRecord(recs[id].b, s));
    }
    void flush() {
        if (!on || recs.empty()) return;
        SFMM_HIP(hipStreamSynchronize(s));
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (auto& r : recs) {
            float ms = 0.f;
            SFMM_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            g_prof_ms[r.stage] += ms;
            g_prof_calls[r.stage] += 1;
        }
        release();
    }
    void release() {
        for (auto& r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        recs.clear();
    }
    ~Profiler() { release(); }
};

struct StageScope {
    Profiler& p;
    int id;
    StageScope(Profiler& pr, int stage) : p(pr), id(pr.begin(stage)) {}
    ~StageScope() { p.end(id); }
};

int bits_for(int64_t v) {
    int b = 1;
    while (b < 63 && ((int64_t)1 << b) <= v) ++b;
    return b;
}
}  // namespace

struct sfmm_plan_impl {
    sfmm_options opt{};
    int p = 0;
    int64_t N = 0, M = 0;
    double q_total = 0.0;
    // sources, sorted by key: (x, y, z, q) records
    DVec<double4> spt;
    DVec<uint32_t> sperm;
    DVec<uint64_t> skeys;
    // boxes, ordered by (level, pixel)
    int nbox = 0;
    std::vector<int> lvl_start;
    DVec<int> level, first, count, parent, child0;
    DVec<uint64_t> pixel;
    DVec<double> cen, rad, gdd;
    // interaction lists in CSR form by target box
    int n_m2l = 0, n_p2p = 0;
    DVec<int> m2l_off, m2l_src, p2p_off, p2p_src, m2l_order;
    int n_m2l_fp64 = 0;  // the first n_m2l_fp64 boxes of m2l_order take the FP64 M2L
    // targets, sorted by key
    DVec<double> tx, ty, tz;
    DVec<uint32_t> tperm;
    DVec<uint64_t> tkeys;
    DVec<int> tleaf, tfirst, tcount;
    mutable int ntl = -1;  // leaves with targets and direct-sum work (counted when the statistics ask)
    // direct-act lists split into direct sums and multipole evaluations
    NearLists nl;
    WorkItems near_items, far_items;
    mutable long long n_p2p_pairs = -1, n_m2p_evals = -1;  // summed on the first stats request
    // expansions
    DVec<double> mult, local;
    DVec<double> zrec;  // one zero record (lanes past the end of an FMM-act list)
    DVec<float> multf;  // precision tier: FP32 A-blocks of the multipoles
    DVec<double> hess_part;  // partial slots of 8 doubles (sfmm_execute_hessian)
    // per-pair order policies
    DVec<int> m2l_ent;        // target box of every FMM-act entry (per-pair order policies)
    DVec<int> p2p_ent;        // target box of every direct-act entry (until the near-field split)
    DVec<float> mlp_w;        // order network (learned policy)
    DVec<float4> decay;       // per-box multipole decay features
    DVec<uint8_t> m2l_ord;    // order of every FMM act (last execute)
    DVec<int> ord_off, ord_src;  // FMM acts split by order
    // sum of p'^2 over the FMM acts of the last execute; -1: still in osq_dev
    mutable long long m2l_order_sq = 0;
    DVec<long long> osq_dev;
    bool executed = false;
    // judge of the per-pair order policies (first execute of the plan)
    bool judged = false, judge_failed = false;
    int judge_S = 0;
    DVec<int> judge_pos;       // the judge's targets (caller order)
    DVec<double4> judge_tsel;  // their unit vectors
    DVec<double> judge_part;   // their direct sum per source chunk (computed by the plan)
    bool judge_ready = false;
    double judge_psi = -1.0, judge_alpha = -1.0;
    std::unique_ptr<Pinned> pin;
    // recorded at the end of every sfmm_plan / sfmm_execute on the caller's
    // stream (not while a graph is recorded): sfmm_destroy waits for it
    hipEvent_t done = nullptr;
    void mark_done(hipStream_t s) {
        if (g_capturing) return;
        if (!done) SFMM_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        SFMM_HIP(hipEventRecord(done, s));
    }
    // host reads of the plan's buffers start after its last call's work
    void wait() const {
        if (done) SFMM_HIP(hipEventSynchronize(done));
    }
    ~sfmm_plan_impl() {
        if (done) (void)hipEventDestroy(done);
    }

    FmmCtx ctx() const {
        FmmCtx c;
        c.p = p;
        c.cen = cen.data();
        c.rad = rad.data();
        c.level = level.data();
        c.first = first.data();
        c.count = count.data();
        c.parent = parent.data();
        c.child0 = child0.data();
        c.spt = spt.data();
        c.mult = mult.data();
        c.local = local.data();
        c.zrec = zrec.data();
        c.npm_sigma = opt.npm_sigma;
        return c;
    }
};

namespace {

int read_int(const int* dev, sfmm_plan_impl& P, hipStream_t s) {
    SFMM_HIP(hipMemcpyAsync(P.pin->p, dev, sizeof(int), hipMemcpyDeviceToHost, s));
    SFMM_HIP(hipStreamSynchronize(s));
    return P.pin->p[0];
}

void validate(const sfmm_options& o) {
    auto bad = [](const std::string& m) { throw Error(ST_INVALID_ARG, m); };
    if (o.order < 0 || o.order > kMaxOrder) bad("order must be in [0, 64]");
    if (o.order == 0 && !(o.tolerance >= 1e-15 && o.tolerance <= 1e-1)) bad("tolerance must be in [1e-15, 1e-1]");
    if (o.leaf_size < 1) bad("leaf_size must be >= 1");
    if (!(o.c_s > 0.0) || !std::isfinite(o.c_s)) bad("c_s must be positive");
    if (!(o.c_t > 0.0 && o.c_t < 1.0)) bad("c_t must be in (0, 1)");
    if (o.max_level < 0 || o.max_level > 29) bad("max_level must be in [0, 29]");
    if (o.precision != SFMM_FP64 && o.precision != SFMM_FP32_MIXED) bad("unknown precision");
    if (o.psi_gauge != SFMM_GAUGE_ZERO_MEAN && o.psi_gauge != SFMM_GAUGE_RAW) bad("unknown psi_gauge");
    if (o.order_policy != SFMM_ORDER_FIXED && o.order_policy != SFMM_ORDER_BOUND &&
        o.order_policy != SFMM_ORDER_LEARNED)
        bad("unknown order_policy");
    if (o.order_policy == SFMM_ORDER_LEARNED && !o.mlp_weights) bad("the learned order policy needs mlp_weights");
    if (o.near_segment != 0 && (o.near_segment < 8 || o.near_segment > 4096)) bad("near_segment must be 0 or in [8, 4096]");
    if (o.far_segment != 0 && (o.far_segment < 8 || o.far_segment > 4096)) bad("far_segment must be 0 or in [8, 4096]");
    if (o.judge_targets > 4096) bad("judge_targets must be at most 4096");
    if (!(o.npm_sigma >= 0.0 && o.npm_sigma <= 0.5)) bad("npm_sigma must be in [0, 0.5]");
}

// Sort points by key and keep the permutation; outputs resized here: the
// sorted points as (x, y, z, q) records (sources, rec != nullptr) or as three
// coordinate arrays (targets).
// Keys, records in caller order and the identity permutation; throws on
// non-finite points or points off the unit sphere.
void prepare_checked(const double* in, const double* q_in, int64_t n, DVec<double4>& u, DVec<uint64_t>& keys,
                     DVec<uint32_t>& perm, sfmm_plan_impl& P, hipStream_t s, const char* what) {
    DVec<int> err;
    err.resize(1);
    fill_i32(err.data(), 1, 0, s);
    prepare_points(in, q_in, n, u.data(), keys.data(), perm.data(), err.data(), s);
    const int e = read_int(err.data(), P, s);
    if (e & 1) throw Error(ST_INVALID_ARG, std::string(what) + ": non-finite coordinates");
    if (e & 2) throw Error(ST_INVALID_ARG, std::string(what) + ": points off the unit sphere by more than 1e-6");
}

// Sources: keys, sort by key, records (x, y, z, q) in key order.
void sort_points(const double* in, const double* q_in, int64_t n, DVec<double4>& rec, DVec<uint32_t>& perm,
                 DVec<uint64_t>& keys, sfmm_plan_impl& P, hipStream_t s, const char* what) {
    rec.resize(n);
    perm.resize(n);
    keys.resize(n);
    if (n == 0) return;
    DVec<double4> u;
    u.resize(n);
    prepare_checked(in, q_in, n, u, keys, perm, P, s, what);
    radix_sort_u64(keys.data(), perm.data(), n, 62, s);
    gather_records(perm.data(), n, u.data(), rec.data(), s);
}

constexpr int kTreeBatch = 8;  // queued levels between two read-backs

// Levels with a host read of the split count after each: the arrays grow as
// needed.
void build_levels_exact(sfmm_plan_impl& P, int m, hipStream_t s) {
    tree_base_level(P.skeys.data(), P.N, P.level.data(), P.pixel.data(), P.first.data(), P.count.data(),
                    P.parent.data(), P.child0.data(), s);
    P.lvl_start.assign({0, 12});
    DVec<int> flag, off, tot;
    tot.resize(1);
    const int wave_level = tree_wave_level();
    for (int L = 0;; ++L) {
        const int b0 = P.lvl_start[L], b1 = P.lvl_start[L + 1], nb = b1 - b0;
        flag.resize(nb);
        off.resize(nb);
        tree_split_flags(b0, nb, P.level.data(), P.count.data(), m, P.opt.max_level, flag.data(), s);
        scan_excl_i32(flag.data(), off.data(), nb, tot.data(), s);
        const int nsplit = read_int(tot.data(), P, s);
        if (nsplit == 0) break;
        const size_t need = (size_t)b1 + 4 * (size_t)nsplit;
        if (need > 0x7fffffff) throw Error(ST_INVALID_ARG, "tree too large");
        P.level.grow(need, s);
        P.pixel.grow(need, s);
        P.first.grow(need, s);
        P.count.grow(need, s);
        P.parent.grow(need, s);
        P.child0.grow(need, s);
        tree_make_children(b0, nb, b1, flag.data(), off.data(), P.skeys.data(), P.level.data(), P.pixel.data(),
                           P.first.data(), P.count.data(), P.parent.data(), P.child0.data(), wave_level, s);
        P.lvl_start.push_back((int)need);
    }
}

// Levels queued kTreeBatch at a time with the level bounds on the device;
// false when the children of some level would pass cap boxes (nothing of
// the partial build is kept then).
bool build_levels_queued(sfmm_plan_impl& P, int m, int cap, hipStream_t s) {
    constexpr int kLs = 32;  // level bounds ls[0 .. max_level + 2]
    DVec<int> ls, ctl, ccnt, wpre;
    ls.resize(kLs);
    ctl.resize(1);
    const int nch = (cap + kTreeChunk - 1) / kTreeChunk;
    ccnt.resize(nch);
    wpre.resize(cap);
    const int grid = std::min(nch, 1024);
    const int cgrid = 2048;  // 8192 waves
    tree_base_level(P.skeys.data(), P.N, P.level.data(), P.pixel.data(), P.first.data(), P.count.data(),
                    P.parent.data(), P.child0.data(), s);
    tree_init_queued(ls.data(), kLs, ctl.data(), s);
    const int lmax = P.opt.max_level;
    const int wave_level = tree_wave_level();
    int* h = P.pin->p;
    for (int L = 0;;) {
        const int Lend = std::min(L + kTreeBatch, lmax + 1);
        for (; L < Lend; ++L)
            tree_level_queued(ls.data(), L, ccnt.data(), wpre.data(), grid, cgrid, cap, ctl.data(), m,
                              L < lmax ? 1 : 0, P.skeys.data(), P.level.data(), P.pixel.data(), P.first.data(), P.count.data(),
                              P.parent.data(), P.child0.data(), wave_level, s);
        SFMM_HIP(hipMemcpyAsync(h, ls.data(), sizeof(int) * kLs, hipMemcpyDeviceToHost, s));
        SFMM_HIP(hipMemcpyAsync(h + kLs, ctl.data(), sizeof(int), hipMemcpyDeviceToHost, s));
        SFMM_HIP(hipStreamSynchronize(s));
        if (h[kLs]) return false;
        // the first level that split nothing ends the tree
        for (int z = 0; z < L; ++z) {
            if (h[z + 2] == h[z + 1]) {
                P.lvl_start.assign(h, h + z + 2);
                return true;
            }
        }
        if (L > lmax) throw Error(ST_INTERNAL, "tree levels did not terminate");
    }
}

void build_tree(sfmm_plan_impl& P, hipStream_t s, Profiler& prof) {
    const int stage_tree = prof.begin(S_TREE);
    const int m = P.opt.leaf_size;
    size_t cap = 12 + 8 * (size_t)(P.N / std::max(1, m)) + 64;
    // SFMM_TREE_CAP (boxes) overrides the capacity of the queued levels:
    // tests use it to drive the fallback
    if (const char* forced = std::getenv("SFMM_TREE_CAP")) cap = std::max<size_t>(12, std::strtoull(forced, nullptr, 10));
    cap = std::min<size_t>(cap, 0x7fffffff);
    P.level.resize(cap);
    P.pixel.resize(cap);
    P.first.resize(cap);
    P.count.resize(cap);
    P.parent.resize(cap);
    P.child0.resize(cap);
    if (!build_levels_queued(P, m, (int)cap, s)) build_levels_exact(P, m, s);
    prof.end(stage_tree);
    P.nbox = P.lvl_start.back();
    P.cen.resize(4 * (size_t)P.nbox);
    P.rad.resize(P.nbox);
    P.gdd.resize(8 * (size_t)P.nbox);
    StageScope st(prof, S_GEOM);
    box_geometry(P.nbox, P.level.data(), P.pixel.data(), P.cen.data(), P.rad.data(), P.gdd.data(), s);
}

// Stable sort on the target field only: within one target the pairs keep the
// walk's (deterministic) emission order.
void sort_pairs_to_csr(DVec<uint64_t>& pairs, int np, int nbox, DVec<int>& off, DVec<int>& src, DVec<int>* ent,
                       hipStream_t s) {
    off.resize((size_t)nbox + 1);
    src.resize(std::max(np, 1));
    DVec<int> tgt_own;
    DVec<int>& tgt = ent ? *ent : tgt_own;
    tgt.resize(std::max(np, 1));
    if (np > 1) {  // the last pass writes the sources and targets themselves
        DVec<uint64_t> alt;
        alt.resize(np);
        radix_sort_u64_pp(pairs.data(), nullptr, alt.data(), nullptr, np, 32 + bits_for(nbox), s, 32, nullptr,
                          reinterpret_cast<uint32_t*>(src.data()), reinterpret_cast<uint32_t*>(tgt.data()));
    } else {
        pair_split(pairs.data(), np, src.data(), tgt.data(), s);
    }
    csr_offsets(tgt.data(), np, nbox, off.data(), s);
}

// Capacities of the queued walk, as multiples of the box count: the largest
// needs seen so far in this process (x 1.25), at least the defaults.
std::mutex g_walk_mu;
double g_walk_ratio[3] = {24.0, 40.0, 40.0};  // frontier, M2L, P2P pairs per box

constexpr int kWalkBatch = 8;        // rounds queued between two read-backs
constexpr int kWalkMaxRounds = 64;   // a round raises level(S) + level(T): at most 2 x 29 + 1 rounds
constexpr int kWalkGrid = 8192;      // workgroups of a queued round (each takes chunks in turn)

// The frontier form of Algorithm 1.  Queued mode: rounds run back to back on
// the device with fixed capacities, the host reading the frontier size every
// kWalkBatch rounds; a round that would overflow ends the walk with
// *overflow set.  Exact mode: the host reads each round's totals and grows
// every buffer before the emit.  Both produce the same lists.
bool walk(sfmm_plan_impl& P, const WalkCtx& w, bool exact, DVec<uint64_t>& m2l, DVec<uint64_t>& p2p, int* n_m2l,
          int* n_p2p, hipStream_t s) {
    // Algorithm 1 starts at INTERACTION(root, root): root is not a leaf and
    // equals itself, so the first round is every pair of its 12 children
    std::vector<int2> f0;
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) f0.push_back(make_int2(i, j));
    const int n0 = (int)f0.size();
    // SFMM_WALK_RATIO (pairs per box, all three capacities, no lower bound)
    // overrides the capacities: tests use it to drive the overflow path
    const char* forced = std::getenv("SFMM_WALK_RATIO");
    WalkCaps cap;
    {
        std::lock_guard<std::mutex> lk(g_walk_mu);
        const double lo = forced ? 1.0 : 65536.0;
        auto c = [&](double r) { return (int)std::min(2.0e9, std::max(lo, r * P.nbox)); };
        const double f = forced ? std::atof(forced) : 0.0;
        cap.frontier = exact ? n0 : c(forced ? f : g_walk_ratio[0]);
        cap.m2l = exact ? 1 : c(forced ? f : g_walk_ratio[1]);
        cap.p2p = exact ? 1 : c(forced ? f : g_walk_ratio[2]);
    }
    DVec<int2> F, G;
    F.resize(std::max(cap.frontier, n0));
    G.resize(cap.frontier);
    m2l.resize(cap.m2l);
    p2p.resize(cap.p2p);
    DVec<uint8_t> action;
    DVec<int> ctot, coff, tot, rs;
    tot.resize(3);
    rs.resize(4 * (kWalkMaxRounds + 1) + 1);
    int* overflow = rs.data() + 4 * (kWalkMaxRounds + 1);
    fill_i32(rs.data(), 4 * (kWalkMaxRounds + 1) + 1, 0, s);
    const int st0[3] = {n0, 0, 0};
    SFMM_HIP(hipMemcpyAsync(rs.data(), st0, sizeof(st0), hipMemcpyHostToDevice, s));
    SFMM_HIP(hipMemcpyAsync(F.data(), f0.data(), f0.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    int n = n0, rounds = 0;
    int nch = walk_chunks(exact ? n0 : cap.frontier);
    action.resize(exact ? n0 : cap.frontier);
    ctot.resize(3 * (size_t)nch);
    coff.resize(3 * (size_t)nch);
    for (int r = 0; r < kWalkMaxRounds; ++r) {
        const int* st = rs.data() + 4 * r;
        int* st_next = rs.data() + 4 * (r + 1);
        if (exact) {
            nch = walk_chunks(n);
            action.resize(std::max(n, 1));
            ctot.resize(3 * (size_t)nch);
            coff.resize(3 * (size_t)nch);
            const int grid = std::min(kWalkGrid, nch);
            walk_round_scan(F.data(), st, w, action.data(), ctot.data(), coff.data(), nch, tot.data(), grid, s);
            SFMM_HIP(hipMemcpyAsync(P.pin->p, tot.data(), 3 * sizeof(int), hipMemcpyDeviceToHost, s));
            SFMM_HIP(hipMemcpyAsync(P.pin->p + 3, st, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
            SFMM_HIP(hipStreamSynchronize(s));
            const int nc = P.pin->p[0], am = P.pin->p[1], ap = P.pin->p[2];
            const int64_t em = (int64_t)P.pin->p[4] + am, ep = (int64_t)P.pin->p[5] + ap;
            if (em > 0x7fffffff || ep > 0x7fffffff) throw Error(ST_INVALID_ARG, "interaction lists too large");
            m2l.grow((size_t)std::max<int64_t>(em, 1), s);
            p2p.grow((size_t)std::max<int64_t>(ep, 1), s);
            G.resize(std::max(nc, 1));
            cap.frontier = std::max(nc, 1);
            cap.m2l = (int)m2l.n;
            cap.p2p = (int)p2p.n;
            walk_round_emit(F.data(), st, w, action.data(), coff.data(), nch, tot.data(), cap, G.data(), m2l.data(),
                            p2p.data(), st_next, overflow, grid, s);
            n = nc;
        } else {
            walk_round_scan(F.data(), st, w, action.data(), ctot.data(), coff.data(), nch, tot.data(), kWalkGrid, s);
            walk_round_emit(F.data(), st, w, action.data(), coff.data(), nch, tot.data(), cap, G.data(), m2l.data(),
                            p2p.data(), st_next, overflow, kWalkGrid, s);
            if ((r + 1) % kWalkBatch == 0) {
                SFMM_HIP(hipMemcpyAsync(P.pin->p, st_next, sizeof(int), hipMemcpyDeviceToHost, s));
                SFMM_HIP(hipStreamSynchronize(s));
                n = P.pin->p[0];
            }
        }
        std::swap(F.p, G.p);
        std::swap(F.n, G.n);
        std::swap(F.cap, G.cap);
        rounds = r + 1;
        if (n == 0) break;
    }
    std::vector<int> h(4 * (kWalkMaxRounds + 1) + 1);
    SFMM_HIP(hipMemcpyAsync(h.data(), rs.data(), h.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    SFMM_HIP(hipStreamSynchronize(s));
    if (h.back()) return false;  // overflow: the lists are incomplete
    if (h[4 * rounds] != 0) throw Error(ST_INTERNAL, "the interaction walk did not end");
    *n_m2l = h[4 * rounds + 1];
    *n_p2p = h[4 * rounds + 2];
    int fmax = 0;
    for (int r = 0; r <= rounds; ++r) fmax = std::max(fmax, h[4 * r]);
    if (!forced) {
        std::lock_guard<std::mutex> lk(g_walk_mu);
        const double nb = std::max(1, P.nbox);
        g_walk_ratio[0] = std::max(g_walk_ratio[0], 1.25 * fmax / nb);
        g_walk_ratio[1] = std::max(g_walk_ratio[1], 1.25 * *n_m2l / nb);
        g_walk_ratio[2] = std::max(g_walk_ratio[2], 1.25 * *n_p2p / nb);
    }
    return true;
}

void build_lists(sfmm_plan_impl& P, hipStream_t s, Profiler& prof) {
    const int stage_walk = prof.begin(S_WALK);
    DVec<double4> geo, ttrig;
    DVec<double2> strig;
    DVec<int2> cc;
    DVec<double> dtrig;
    geo.resize(std::max(P.nbox, 1));
    strig.resize(std::max(P.nbox, 1));
    ttrig.resize(std::max(P.nbox, 1));
    cc.resize(std::max(P.nbox, 1));
    dtrig.resize(kWalkDtrig * (size_t)std::max(P.nbox, 1));
    walk_boxes(P.nbox, P.cen.data(), P.rad.data(), P.gdd.data(), P.child0.data(), P.count.data(), P.opt.c_s,
               P.opt.c_t, P.opt.npm_sigma, geo.data(), strig.data(), ttrig.data(), cc.data(), dtrig.data(), s);
    WalkCtx w;
    w.child0 = P.child0.data();
    w.count = P.count.data();
    w.geo = geo.data();
    w.strig = strig.data();
    w.ttrig = ttrig.data();
    w.cc = cc.data();
    w.gdd = P.gdd.data();
    w.dtrig = dtrig.data();
    w.c_s = P.opt.c_s;
    w.c_t = P.opt.c_t;
    w.sigma = P.opt.npm_sigma;
    DVec<uint64_t> m2l, p2p;
    int n_m2l = 0, n_p2p = 0;
    if (!walk(P, w, false, m2l, p2p, &n_m2l, &n_p2p, s) && !walk(P, w, true, m2l, p2p, &n_m2l, &n_p2p, s))
        throw Error(ST_INTERNAL, "the interaction walk overflowed its exactly sized buffers");
    prof.end(stage_walk);
    StageScope st(prof, S_LISTS);
    P.n_m2l = n_m2l;
    P.n_p2p = n_p2p;
    m2l.grow(std::max(n_m2l, 1), s);
    p2p.grow(std::max(n_p2p, 1), s);
    // target box of every entry: the per-pair order policies need it for the
    // FMM acts, the near-field split for the direct acts
    const bool ent = P.opt.order_policy != SFMM_ORDER_FIXED;
    sort_pairs_to_csr(m2l, n_m2l, P.nbox, P.m2l_off, P.m2l_src, ent ? &P.m2l_ent : nullptr, s);
    sort_pairs_to_csr(p2p, n_p2p, P.nbox, P.p2p_off, P.p2p_src, &P.p2p_ent, s);
    // M2L work order: target boxes with the most team rounds first, so the
    // lanes of a wave carry the same work
    DVec<uint64_t> k;
    DVec<uint32_t> v;
    k.resize(P.nbox);
    v.resize(P.nbox);
    // precision tier: boxes of the coarse levels first (they stay FP64)
    const bool tier = P.opt.precision == SFMM_FP32_MIXED;
    int lc = 29;
    if (tier) {
        // SFMM_FP32_COARSE_LEVEL overrides the last FP64 level (-1: none), for
        // tuning it and for tests
        const char* v = std::getenv("SFMM_FP32_COARSE_LEVEL");
        lc = v ? (int)std::max(-1L, std::min(29L, std::strtol(v, nullptr, 10))) : kFp32CoarseLevel;
    }
    const int nlev = (int)P.lvl_start.size() - 1;
    P.n_m2l_fp64 = tier ? P.lvl_start[std::min(lc + 1, nlev)] : P.nbox;
    m2l_order_keys(P.m2l_off.data(), P.level.data(), lc, m2l_team_width(P.n_m2l_fp64), kM2LTeamF32, P.nbox, k.data(),
                   v.data(), s);
    radix_sort_u64(k.data(), v.data(), P.nbox, 16, s);
    P.m2l_order.resize(P.nbox);
    SFMM_HIP(hipMemcpyAsync(P.m2l_order.data(), v.data(), sizeof(int) * P.nbox, hipMemcpyDeviceToDevice, s));
}

// Boxes that have items: the items minus the extra segments of split boxes
int count_boxes(const WorkItems& w, hipStream_t s) {
    if (w.nred == 0) return w.n;
    std::vector<int4> r(w.nred);
    SFMM_HIP(hipMemcpyAsync(r.data(), w.red.data(), sizeof(int4) * w.nred, hipMemcpyDeviceToHost, s));
    SFMM_HIP(hipStreamSynchronize(s));
    int extra = 0;
    for (const int4& x : r) extra += x.y - 1;
    return w.n - extra;
}

// Targets: keys (kept in caller order), leaf box of each, and the plan order
// = a stable sort by leaf box (a leaf's targets form one run, in caller
// order; nothing downstream needs key order within a leaf).
void build_targets(sfmm_plan_impl& P, const double* tgt, hipStream_t s) {
    const int64_t M = P.M;
    P.tx.resize(M);
    P.ty.resize(M);
    P.tz.resize(M);
    P.tperm.resize(M);
    P.tkeys.resize(M);
    P.tleaf.resize(std::max<int64_t>(M, 1));
    P.tfirst.resize(P.nbox);
    P.tcount.resize(P.nbox);
    fill_i32(P.tfirst.data(), P.nbox, 0, s);
    fill_i32(P.tcount.data(), P.nbox, 0, s);
    if (M > 0) {
        DVec<double4> u;
        DVec<uint64_t> leaf, leaf2;
        DVec<uint32_t> perm2;
        u.resize(M);
        leaf.resize(M);
        leaf2.resize(M);
        perm2.resize(M);
        prepare_checked(tgt, nullptr, M, u, P.tkeys, P.tperm, P, s, "targets");
        locate_targets(P.tkeys.data(), M, P.child0.data(), P.level.data(), leaf.data(), s);
        uint32_t* pv = nullptr;
        const uint64_t* ls = radix_sort_u64_pp(leaf.data(), P.tperm.data(), leaf2.data(), perm2.data(), M,
                                               bits_for(P.nbox), s, 0, &pv);
        if (pv != P.tperm.data()) {
            std::swap(P.tperm.p, perm2.p);
            std::swap(P.tperm.n, perm2.n);
            std::swap(P.tperm.cap, perm2.cap);
        }
        gather_targets(P.tperm.data(), ls, M, u.data(), P.tx.data(), P.ty.data(), P.tz.data(), P.tleaf.data(), s);
    }
    target_ranges(P.tleaf.data(), M, P.nbox, P.tfirst.data(), P.tcount.data(), s);
    near_split(P.ctx(), P.p2p_off.data(), P.p2p_src.data(), P.p2p_ent.data(), P.nbox, P.n_p2p, P.tfirst.data(),
               P.tcount.data(), P.tx.data(), P.ty.data(), P.tz.data(), P.nl, s);
    P.p2p_ent.reset();  // stream-ordered pool: later work on this stream may reuse it
    const int segn = P.opt.near_segment > 0 ? P.opt.near_segment : kSegNear;
    const int segf = P.opt.far_segment > 0 ? P.opt.far_segment : kSegFar;
    build_items2(P.nl.near_off.data(), P.nl.near_src.data(), P.count.data(), segn, P.near_items,
                 P.nl.far_off.data(), P.nl.far_src.data(), nullptr, segf, P.far_items, P.tcount.data(), P.nbox, s);
    P.ntl = -1;  // counted by the statistics: a read-back the plan itself does not need
}

// Order from a tolerance, by a measured calibration at the default MACs
// (c_s = 2, c_t = 0.5).  kOrderCal[k] is the largest relative L2 error of
// the deflection (the slower output to converge; psi is ~100 times smaller)
// at order p = 8 + 2k, over every target of uniform-1e4 (leaf sizes 16, 32,
// 64), clustered-5e4 (16, 32, 64), clustered-1e6 (16, 32, 64) and
// clustered-1e7 (32, 56), each order against the same plan at order 48
// (itself ~1e-14 from the direct sum).  clustered-1e6 is the worst sky at
// every order: its tail targets, on the corners of deep leaves next to
// massive clumps, set the norm.  The order is the smallest p whose error,
// interpolated log-linearly in p (end slopes outside 8..44), is at most a
// quarter of the tolerance.
constexpr double kOrderCal[] = {3.48e-4, 8.80e-5,  2.29e-5,  6.12e-6,  1.69e-6,  4.82e-7,  1.44e-7,
                                4.48e-8, 1.46e-8,  4.90e-9,  1.70e-9,  6.03e-10, 2.19e-10, 8.11e-11,
                                3.04e-11, 1.15e-11, 4.40e-12, 1.66e-12, 5.97e-13};
constexpr int kOrderCalN = sizeof(kOrderCal) / sizeof(kOrderCal[0]);
constexpr int kOrderCalP0 = 8, kOrderCalStep = 2;
constexpr double kOrderMarginFactor = 4.0;

}  // namespace

double sfmm::order_calibrated_error(int p) {
    const double x = (double)(p - kOrderCalP0) / kOrderCalStep;
    const int k = std::min(kOrderCalN - 2, std::max(0, (int)std::floor(x)));
    const double t = x - k;
    return std::exp(std::log(kOrderCal[k]) + t * (std::log(kOrderCal[k + 1]) - std::log(kOrderCal[k])));
}

namespace {

// Odd orders are rounded up to the next even one: measured on clustered-1e7,
// the M2L kernel at an odd order runs ~15 % slower per flop than at the even
// orders around it (36: 2.93 ms, 37: 3.60 ms, 38: 3.25 ms), so the next even
// order costs less and is more accurate.
int order_for_tolerance(double tol) {
    for (int p = 4; p < kMaxTolOrder; ++p)
        if (order_calibrated_error(p) * kOrderMarginFactor <= tol) return p + (p & 1);
    return kMaxTolOrder;
}

sfmm_status fail(const Error& e) {
    g_last_error = e.what();
    return (sfmm_status)e.status;
}

template <typename S, typename D>
void copy_widen(D* dst, const S* dev, size_t n) {
    if (!dst || n == 0) return;
    std::vector<S> h(n);
    SFMM_HIP(hipMemcpy(h.data(), dev, sizeof(S) * n, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < n; ++i) dst[i] = (D)h[i];
}

void export_csr(const DVec<int>& off, const DVec<int>& src, int nbox, int np, int64_t* s_out, int64_t* t_out) {
    std::vector<int> o(nbox + 1), s(std::max(np, 1));
    SFMM_HIP(hipMemcpy(o.data(), off.data(), sizeof(int) * (nbox + 1), hipMemcpyDeviceToHost));
    if (np) SFMM_HIP(hipMemcpy(s.data(), src.data(), sizeof(int) * np, hipMemcpyDeviceToHost));
    for (int t = 0; t < nbox; ++t) {
        // canonical order within a target: ascending source box
        std::sort(s.begin() + o[t], s.begin() + o[t + 1]);
        for (int k = o[t]; k < o[t + 1]; ++k) {
            if (s_out) s_out[k] = s[k];
            if (t_out) t_out[k] = t;
        }
    }
}

void check_finite(const float* a, int64_t n, const char* what) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) throw Error(ST_INVALID_ARG, std::string(what) + " holds a non-finite value");
}

}  // namespace

// A batch of plans (shells) executed together; the work of sfmm_execute on
// all of them is recorded once in a HIP graph and replayed as one launch.
// host threads (each with its own stream) that plan the shells of a batch
constexpr int kBatchPlanStreams = 4;

struct sfmm_batch_impl {
    std::vector<sfmm_plan_impl*> plans;
    hipStream_t own = nullptr;  // used when the caller passes the null stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double*> g_psi, g_defl;  // outputs the graph was recorded with
    hipStream_t g_stream = nullptr;
    bool capturable = true;
    hipEvent_t done = nullptr;  // end of the last sfmm_batch_execute
    // worker streams (from planning) and the shells each runs, largest first;
    // the fork and join events order them after and before the caller's stream
    std::vector<hipStream_t> ws;
    std::vector<std::vector<int>> groups;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    void drop_graph() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~sfmm_batch_impl() {
        if (done) (void)hipEventSynchronize(done);
        drop_graph();
        for (auto w : ws) (void)hipStreamSynchronize(w);
        for (auto* p : plans) sfmm_destroy(p);
        if (done) (void)hipEventDestroy(done);
        if (fork) (void)hipEventDestroy(fork);
        for (auto e : join) (void)hipEventDestroy(e);
        for (auto w : ws) (void)hipStreamDestroy(w);
        if (own) hipStreamDestroy(own);
    }
};

// Scratch of one execute taken from outside the plan (the no-allocation
// entry point): the partial slots of both near-field work item sets and the
// FP32 copy of the multipole A-blocks.
struct ExecScratch {
    double* near_part;
    double* far_part;
    float* multf;
};

// Bytes of ExecScratch a plan needs (each part 256-byte aligned).
size_t exec_scratch_bytes(const sfmm_plan_impl& P, size_t* off_far = nullptr, size_t* off_multf = nullptr) {
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t near = al(sizeof(double) * 4 * (size_t)std::max(P.near_items.nslot, 1));
    const size_t far = al(sizeof(double) * 4 * (size_t)std::max(P.far_items.nslot, 1));
    const bool tier = P.n_m2l_fp64 < P.nbox;
    const size_t mf = tier ? al(sizeof(float) * 2 * (size_t)P.p * (size_t)P.nbox) : 0;
    if (off_far) *off_far = near;
    if (off_multf) *off_multf = near + far;
    return near + far + mf;
}

// The five stages of Sec. 3.7 on a plan; xs = null: the plan's own buffers.
// fixed: every FMM act at the plan order whatever the order policy.
// hess [3][M] (may be null): also the Hessian of Sec. 2.2.
void execute_impl(sfmm_plan_impl& P, double* psi, double* defl, hipStream_t s, const ExecScratch* xs, bool fixed,
                  double* hess = nullptr) {
    // raw gauge: without the share Q_tot/(4pi); near-particle model: the
    // constant of the smoothed particles' potential
    const double shift = ((P.opt.psi_gauge == SFMM_GAUGE_RAW) ? -P.q_total : 0.0) * 0.079577471545947667884 +
                         P.q_total * 0.079577471545947667884 * npm_constant(P.opt.npm_sigma);
    if (P.N == 0) {
        fill_f64(psi, P.M, 0.0, s);
        fill_f64(defl, 3 * P.M, 0.0, s);
        if (hess) fill_f64(hess, 3 * P.M, 0.0, s);
        return;
    }
    // every multipole record is written by Lemma 1 (leaves) or Lemma 2
    // (split boxes), every local record by the first M2L pass
    const FmmCtx c = P.ctx();
    const int nlev = (int)P.lvl_start.size() - 1;
    Profiler prof(s, xs == nullptr);
    // up-pass: Lemma 1 on leaves, Lemma 2 from the deepest split level up
    {
        StageScope st(prof, S_P2M);
        fmm_p2m(c, P.nbox, s);
    }
    {
        StageScope st(prof, S_M2M);
        for (int L = nlev - 2; L >= 0; --L)
            fmm_m2m(c, P.lvl_start[L], P.lvl_start[L + 1] - P.lvl_start[L], s);
    }
    // FMM acts: Lemma 3
    {
        StageScope st(prof, S_M2L);
        const bool tier = P.n_m2l_fp64 < P.nbox;
        float* multf = xs ? xs->multf : nullptr;
        if (tier) {
            if (!xs) {
                P.multf.resize((size_t)P.nbox * 2 * P.p);
                multf = P.multf.data();
            }
            mult_to_f32(c, P.nbox, multf, s);
        }
        // one pass per order: (order, CSR offsets, sources); the first pass
        // writes the local records, later ones add to them
        auto m2l_pass = [&](int p, bool acc, const int* off, const int* src) {
            fmm_m2l(c, p, acc, P.m2l_order.data(), P.n_m2l_fp64, off, src, s);
            if (tier)
                fmm_m2l_f32(c, p, acc, multf, P.m2l_order.data() + P.n_m2l_fp64,
                            P.nbox - P.n_m2l_fp64, off, src, s);
        };
        if (fixed || P.opt.order_policy == SFMM_ORDER_FIXED || P.n_m2l == 0) {
            m2l_pass(P.p, false, P.m2l_off.data(), P.m2l_src.data());
            P.m2l_order_sq = (long long)P.n_m2l * P.p * P.p;
        } else {
            const double kt = SFMM_ORDER_KAPPA * P.opt.tolerance;
            P.m2l_ord.resize(P.n_m2l);
            if (P.opt.order_policy == SFMM_ORDER_BOUND) {
                order_bound(c, P.m2l_ent.data(), P.m2l_src.data(), P.n_m2l, kt, P.m2l_ord.data(), s);
            } else {
                P.decay.resize(P.nbox);
                order_box_decay(c, P.nbox, P.decay.data(), s);
                order_mlp(c, P.m2l_ent.data(), P.m2l_src.data(), P.decay.data(), kt, nullptr, P.n_m2l,
                          P.mlp_w.data(), P.p, kOrderMargin, P.m2l_ord.data(), nullptr, s);
            }
            P.osq_dev.resize(1);
            order_split(P.m2l_off.data(), P.m2l_src.data(), P.m2l_ord.data(), P.nbox, P.n_m2l, P.p, P.ord_off,
                        P.ord_src, P.osq_dev.data(), s);
            P.m2l_order_sq = -1;
            // class q holds the orders in (4q, 4q + 4]; the top class the plan
            // order.  In the precision tier every box runs all its classes in
            // one launch, each pair's monopole part completed inside its
            // class; the FP64 path takes one pass per class and the monopole
            // parts from one pass afterwards
            const bool tail_in_pass = tier && m2l_f32_tail_supported(P.p);
            if (tail_in_pass) {
                // the precision tier: its FP64 and its FP32 boxes each take
                // every class in one launch, monopole parts included
                fmm_m2l_f64_classes(c, P.m2l_order.data(), P.n_m2l_fp64, P.ord_off.data(), P.ord_src.data(),
                                    P.nbox, s);
                fmm_m2l_f32_classes(c, multf, P.m2l_order.data() + P.n_m2l_fp64, P.nbox - P.n_m2l_fp64,
                                    P.ord_off.data(), P.ord_src.data(), P.nbox, s);
            } else {
                for (int q = 0; q < (P.p + kOrderStep - 1) / kOrderStep; ++q) {
                    const int pq = std::min((q + 1) * kOrderStep, P.p);
                    m2l_pass(pq, q > 0, P.ord_off.data() + (size_t)q * P.nbox, P.ord_src.data());
                }
                m2l_qtail(c, P.m2l_off.data(), P.m2l_src.data(), P.m2l_ord.data(), P.nbox, s);
            }
        }
    }
    // down-pass: Lemma 4 from level 1 down
    {
        StageScope st(prof, S_L2L);
        for (int L = 1; L < nlev; ++L) fmm_l2l(c, P.lvl_start[L], P.lvl_start[L + 1] - P.lvl_start[L], s);
    }
    // far field at the targets, then the direct acts
    {
        StageScope st(prof, S_L2P);
        fmm_l2p(c, P.tx.data(), P.ty.data(), P.tz.data(), P.tleaf.data(), P.tperm.data(), P.M, shift, psi,
                defl, P.M, s, hess);
    }
    // the Hessian's partial slots hold 8 doubles instead of 4
    double* far_part = xs ? xs->far_part : nullptr;
    double* near_part = xs ? xs->near_part : nullptr;
    if (hess) {
        P.hess_part.resize(8 * ((size_t)std::max(P.far_items.nslot, 1) + (size_t)std::max(P.near_items.nslot, 1)));
        far_part = P.hess_part.data();
        near_part = P.hess_part.data() + 8 * (size_t)std::max(P.far_items.nslot, 1);
    }
    {
        StageScope st(prof, S_M2P);
        fmm_m2p(c, P.far_items, P.nl.far_src.data(), P.tfirst.data(), P.tcount.data(), P.tx.data(),
                P.ty.data(), P.tz.data(), P.tperm.data(), psi, defl, P.M, s, far_part, hess);
    }
    {
        StageScope st(prof, S_P2P);
        fmm_p2p(c, P.opt.precision == SFMM_FP32_MIXED, P.near_items, P.nl.near_src.data(), P.tfirst.data(),
                P.tcount.data(), P.tx.data(), P.ty.data(), P.tz.data(), P.tperm.data(), psi, defl, P.M, s,
                near_part, hess);
    }
    prof.flush();
}

constexpr int kJudgeDefault = 32;

// The judge's S targets: distinct caller-order positions from a
// counter-based generator (splitmix64), seeded by the plan's sizes
std::vector<int> judge_positions(int64_t N, int64_t M, int S) {
    std::vector<int> pos;
    std::vector<char> taken((size_t)M, 0);
    for (uint64_t i = 0; (int)pos.size() < S; ++i) {
        uint64_t z = 0x2210070210ULL + (uint64_t)N * 0x9e3779b97f4a7c15ULL + 0x9e3779b97f4a7c15ULL * (i + 1);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        const int64_t j = (int64_t)(z % (uint64_t)M);
        if (!taken[j]) {
            taken[j] = 1;
            pos.push_back((int)j);
        }
    }
    return pos;
}

// Second streams for the judge's direct sum during planning: created on
// first use per device (non-blocking, default priority) and kept for the
// life of the process; a plan takes one and gives it back when it ends.
struct SideStream {
    int dev = -1;
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_side_mu;
std::vector<SideStream*> g_side_free;

SideStream* side_acquire() {
    int dev = 0;
    SFMM_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_side_mu);
        for (size_t k = 0; k < g_side_free.size(); ++k)
            if (g_side_free[k]->dev == dev) {
                SideStream* w = g_side_free[k];
                g_side_free.erase(g_side_free.begin() + k);
                return w;
            }
    }
    std::unique_ptr<SideStream> w(new SideStream());
    w->dev = dev;
    SFMM_HIP(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
    SFMM_HIP(hipEventCreateWithFlags(&w->fork, hipEventDisableTiming));
    SFMM_HIP(hipEventCreateWithFlags(&w->join, hipEventDisableTiming));
    return w.release();
}

// Holds a plan's second stream: end() makes the plan's stream wait for the
// judge's sum; the destructor (also on an error inside the plan) waits for
// the second stream before the plan's buffers can go, and returns it.
struct JudgeOverlap {
    SideStream* w = nullptr;
    void end(hipStream_t s) {
        if (w) SFMM_HIP(hipStreamWaitEvent(s, w->join, 0));
    }
    ~JudgeOverlap() {
        if (!w) return;
        (void)hipStreamSynchronize(w->stream);
        std::lock_guard<std::mutex> lk(g_side_mu);
        g_side_free.push_back(w);
    }
};

// Plan-time half of the judge (per-pair order policies): its targets, and
// their direct sum over the sorted sources on a second stream beside the
// rest of the plan.
void judge_start(sfmm_plan_impl& P, const double* tgt, JudgeOverlap& ov, hipStream_t s) {
    const int S = (int)std::min<int64_t>(P.M, P.opt.judge_targets > 0 ? P.opt.judge_targets : kJudgeDefault);
    P.judge_S = S;
    if (S <= 0) return;
    const std::vector<int> pos = judge_positions(P.N, P.M, S);
    P.judge_pos.resize(S);
    P.judge_tsel.resize(S);
    P.judge_part.resize(judge_part_doubles(P.N, S));
    SFMM_HIP(hipMemcpyAsync(P.judge_pos.data(), pos.data(), sizeof(int) * S, hipMemcpyHostToDevice, s));
    judge_targets(P.judge_pos.data(), S, tgt, P.M, P.judge_tsel.data(), s);
    ov.w = side_acquire();
    SFMM_HIP(hipEventRecord(ov.w->fork, s));
    SFMM_HIP(hipStreamWaitEvent(ov.w->stream, ov.w->fork, 0));
    judge_sum(P.spt.data(), P.N, P.judge_tsel.data(), S, P.judge_part.data(), ov.w->stream);
    SFMM_HIP(hipEventRecord(ov.w->join, ov.w->stream));
    P.judge_ready = true;
}

// The judge: psi and alpha of the last execute at the plan's S judge
// targets against their direct sum; sets P.judge_psi / judge_alpha
// (relative L2 errors).
void run_judge(sfmm_plan_impl& P, const double* psi, const double* defl, hipStream_t s) {
    const int S = P.judge_S;
    if (S <= 0) {
        P.judge_psi = P.judge_alpha = 0.0;
        return;
    }
    if (!P.judge_ready) throw Error(ST_INTERNAL, "the judge's direct sum was not started by the plan");
    DVec<double> ref, got;
    ref.resize(4 * (size_t)S);
    got.resize(4 * (size_t)S);
    const double shift = (P.opt.psi_gauge == SFMM_GAUGE_RAW) ? 0.0 : P.q_total * 0.079577471545947667884;
    judge_outputs(P.judge_pos.data(), S, P.judge_tsel.data(), P.judge_part.data(), P.N, shift, psi, defl, P.M,
                  ref.data(), got.data(), s);
    std::vector<double> hr(4 * (size_t)S), hg(4 * (size_t)S);
    SFMM_HIP(hipMemcpyAsync(hr.data(), ref.data(), sizeof(double) * 4 * S, hipMemcpyDeviceToHost, s));
    SFMM_HIP(hipMemcpyAsync(hg.data(), got.data(), sizeof(double) * 4 * S, hipMemcpyDeviceToHost, s));
    SFMM_HIP(hipStreamSynchronize(s));
    double dp = 0, rp = 0, da = 0, ra = 0;
    for (int k = 0; k < S; ++k) {
        dp += (hg[4 * k] - hr[4 * k]) * (hg[4 * k] - hr[4 * k]);
        rp += hr[4 * k] * hr[4 * k];
        for (int c = 1; c < 4; ++c) {
            da += (hg[4 * k + c] - hr[4 * k + c]) * (hg[4 * k + c] - hr[4 * k + c]);
            ra += hr[4 * k + c] * hr[4 * k + c];
        }
    }
    P.judge_psi = rp > 0 ? std::sqrt(dp / rp) : std::sqrt(dp);
    P.judge_alpha = ra > 0 ? std::sqrt(da / ra) : std::sqrt(da);
}

// ---- no-allocation execute (sfmm_execute_noalloc)
// Its scratch lives in this file-scope device array: each GPU the library
// runs on holds its own copy for the life of the process.  Host code never
// uses the array's name as an address (on the host it is only a stand-in for
// the symbol): the device address is looked up once per device and kept.
constexpr size_t kNoallocScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
unsigned char* noalloc_scratch() {
    int dev = 0;
    SFMM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(ST_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            throw Error(ST_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    return (unsigned char*)g_scratch_ptr[dev];
}

extern "C" {

void sfmm_default_options(sfmm_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->order = 0;
    opt->tolerance = 1e-10;
    opt->leaf_size = 64;
    opt->c_s = 2.0;
    opt->c_t = 0.5;
    opt->max_level = 29;
    opt->precision = SFMM_FP64;
    opt->psi_gauge = SFMM_GAUGE_ZERO_MEAN;
}

int32_t sfmm_order_for_tolerance(double tol) { return order_for_tolerance(tol); }

sfmm_status sfmm_plan(const double* src, const double* q, int64_t N, const double* tgt, int64_t M,
                      const sfmm_options* opt, void* stream, sfmm_plan_t* out) {
    if (out) *out = nullptr;
    try {
        if (!out) throw Error(ST_INVALID_ARG, "out is NULL");
        if (N < 0 || M < 0 || N > 0x7fffffff || M > 0x7fffffff)
            throw Error(ST_INVALID_ARG, "N and M must be in [0, 2^31 - 1]");
        if (N > 0 && (!src || !q)) throw Error(ST_INVALID_ARG, "src or q is NULL");
        if (M > 0 && !tgt) throw Error(ST_INVALID_ARG, "tgt is NULL");
        sfmm_options o;
        if (opt) o = *opt;
        else sfmm_default_options(&o);
        validate(o);
        hipStream_t s = (hipStream_t)stream;
        PoolStream ps(s);
        std::unique_ptr<sfmm_plan_impl> P(new sfmm_plan_impl());
        JudgeOverlap ov;  // after P: on any exit it waits for the judge's stream before P goes
        P->pin.reset(new Pinned());
        P->opt = o;
        P->p = o.order > 0 ? o.order : order_for_tolerance(o.tolerance);
        P->N = N;
        P->M = M;
        Profiler prof(s);
        {
            StageScope st(prof, S_SRC);
            sort_points(src, q, N, P->spt, P->sperm, P->skeys, *P, s, "sources");
        }
        if (N > 0) {
            DVec<double> qt;
            qt.resize(1);
            sum_f64(q, N, qt.data(), s);  // the caller's charges, contiguous
            SFMM_HIP(hipMemcpyAsync(&P->q_total, qt.data(), sizeof(double), hipMemcpyDeviceToHost, s));
            SFMM_HIP(hipStreamSynchronize(s));
        }
        // per-pair order policies: the judge's direct sum needs only the
        // sorted sources, so it runs beside the tree, the walk and the targets
        if (o.order_policy != SFMM_ORDER_FIXED && o.judge_targets >= 0 && M > 0) judge_start(*P, tgt, ov, s);
        build_tree(*P, s, prof);
        build_lists(*P, s, prof);
        {
            StageScope st(prof, S_TGT);
            build_targets(*P, tgt, s);
        }
        if (o.order_policy == SFMM_ORDER_LEARNED) {
            P->mlp_w.resize(kMlpWeights);
            SFMM_HIP(hipMemcpyAsync(P->mlp_w.data(), o.mlp_weights, sizeof(float) * kMlpWeights,
                                    hipMemcpyHostToDevice, s));
        }
        P->opt.mlp_weights = nullptr;  // not kept: the caller owns it
        prof.flush();
        const size_t ne = (size_t)P->nbox * (2 * P->p + 2);
        P->mult.resize(ne);
        P->local.resize(ne);
        P->zrec.resize(2 * (size_t)P->p + 2);
        fill_f64(P->zrec.data(), 2 * (size_t)P->p + 2, 0.0, s);
        ov.end(s);
        SFMM_HIP(hipStreamSynchronize(s));
        P->mark_done(s);
        *out = P.release();
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SFMM_ERR_INTERNAL;
    }
}

sfmm_status sfmm_execute(sfmm_plan_t plan, double* psi, double* defl, void* stream) {
    try {
        if (!plan) throw Error(ST_INVALID_ARG, "plan is NULL");
        sfmm_plan_impl& P = *plan;
        if (P.M == 0) return SFMM_OK;
        if (!psi || !defl) throw Error(ST_INVALID_ARG, "psi or defl is NULL");
        hipStream_t s = (hipStream_t)stream;
        PoolStream ps(s, g_capturing);
        const bool policy = P.opt.order_policy != SFMM_ORDER_FIXED && P.N > 0;
        const bool fallen = policy && P.judge_failed && !P.opt.no_fallback;
        execute_impl(P, psi, defl, s, nullptr, fallen);
        if (policy && !P.judged && P.opt.judge_targets >= 0) {
            if (g_capturing) throw Error(ST_INVALID_ARG, "a per-pair order policy cannot be judged during capture");
            run_judge(P, psi, defl, s);
            P.judged = true;
            P.judge_failed = !(P.judge_psi <= P.opt.tolerance && P.judge_alpha <= P.opt.tolerance);
            if (P.judge_failed && !P.opt.no_fallback) execute_impl(P, psi, defl, s, nullptr, true);
        }
        P.executed = true;
        P.mark_done(s);
        if (policy && P.judge_failed && P.opt.no_fallback) {
            char m[160];
            std::snprintf(m, sizeof(m), "order policy failed its judge: relative L2 error psi %.3e alpha %.3e > %.1e",
                          P.judge_psi, P.judge_alpha, P.opt.tolerance);
            throw Error(ST_TOL, m);
        }
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SFMM_ERR_INTERNAL;
    }
}

sfmm_status sfmm_execute_hessian(sfmm_plan_t plan, double* psi, double* defl, double* hess, void* stream) {
    try {
        if (!plan) throw Error(ST_INVALID_ARG, "plan is NULL");
        sfmm_plan_impl& P = *plan;
        if (P.M == 0) return SFMM_OK;
        if (!psi || !defl || !hess) throw Error(ST_INVALID_ARG, "psi, defl or hess is NULL");
        hipStream_t s = (hipStream_t)stream;
        PoolStream ps(s, g_capturing);
        // the per-pair order policies run as in sfmm_execute, including the
        // fallback verdict of an earlier judge
        const bool policy = P.opt.order_policy != SFMM_ORDER_FIXED && P.N > 0;
        const bool fallen = policy && P.judge_failed && !P.opt.no_fallback;
        execute_impl(P, psi, defl, s, nullptr, fallen, hess);
        if (policy && !P.judged && P.opt.judge_targets >= 0) {
            if (g_capturing) throw Error(ST_INVALID_ARG, "a per-pair order policy cannot be judged during capture");
            run_judge(P, psi, defl, s);
            P.judged = true;
            P.judge_failed = !(P.judge_psi <= P.opt.tolerance && P.judge_alpha <= P.opt.tolerance);
            if (P.judge_failed && !P.opt.no_fallback) execute_impl(P, psi, defl, s, nullptr, true, hess);
        }
        P.executed = true;
        P.mark_done(s);
        if (policy && P.judge_failed && P.opt.no_fallback)
            throw Error(ST_TOL, "order policy failed its judge (see sfmm_stats)");
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SFMM_ERR_INTERNAL;
    }
}

sfmm_status sfmm_lensing(const double* hess, int64_t M, double* out, void* stream) {
    try {
        if (M < 0) throw Error(ST_INVALID_ARG, "M must be >= 0");
        if (M > 0 && (!hess || !out)) throw Error(ST_INVALID_ARG, "hess or out is NULL");
        lensing_from_hessian(hess, M, out, (hipStream_t)stream);
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_raytrace(int32_t nlayer, const double* const* src, const double* const* q, const int64_t* N,
                          const double* weight, double* rays, int64_t M, double* dist, const sfmm_options* opt,
                          void* stream) {
    try {
        if (nlayer < 1 || nlayer > 4096) throw Error(ST_INVALID_ARG, "nlayer must be in [1, 4096]");
        if (!src || !q || !N || !weight) throw Error(ST_INVALID_ARG, "NULL array");
        if (M < 0 || M > 0x7fffffff) throw Error(ST_INVALID_ARG, "M must be in [0, 2^31 - 1]");
        for (int i = 0; i < nlayer; ++i)
            if (!std::isfinite(weight[i])) throw Error(ST_INVALID_ARG, "layer weights must be finite");
        if (M == 0) return SFMM_OK;
        if (!rays) throw Error(ST_INVALID_ARG, "rays is NULL");
        hipStream_t s = (hipStream_t)stream;
        PoolStream ps(s);
        DVec<double> psi, defl, hess;
        psi.resize(M);
        defl.resize(3 * (size_t)M);
        if (dist) {
            hess.resize(3 * (size_t)M);
            ray_identity(dist, M, s);
        }
        for (int i = 0; i < nlayer; ++i) {
            // the layer's plan has the rays' current positions as targets
            sfmm_plan_t p = nullptr;
            sfmm_status st = sfmm_plan(src[i], q[i], N[i], rays, M, opt, stream, &p);
            if (st != SFMM_OK) return st;
            st = dist ? sfmm_execute_hessian(p, psi.data(), defl.data(), hess.data(), stream)
                      : sfmm_execute(p, psi.data(), defl.data(), stream);
            sfmm_destroy(p);
            if (st != SFMM_OK) return st;
            ray_step(rays, defl.data(), dist ? hess.data() : nullptr, weight[i], M, dist, s);
        }
        SFMM_HIP(hipStreamSynchronize(s));
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SFMM_ERR_INTERNAL;
    }
}

sfmm_status sfmm_execute_noalloc(sfmm_plan_t plan, double* psi, double* defl, void* stream) {
    try {
        if (!plan) throw Error(ST_INVALID_ARG, "plan is NULL");
        sfmm_plan_impl& P = *plan;
        if (P.opt.order_policy != SFMM_ORDER_FIXED)
            throw Error(ST_INVALID_ARG, "sfmm_execute_noalloc needs the fixed order policy");
        if (P.M == 0) return SFMM_OK;
        if (!psi || !defl) throw Error(ST_INVALID_ARG, "psi or defl is NULL");
        size_t off_far = 0, off_mf = 0;
        const size_t need = exec_scratch_bytes(P, &off_far, &off_mf);
        if (need > kNoallocScratchBytes)
            throw Error(ST_INVALID_ARG, "plan needs " + std::to_string(need) +
                                            " bytes of execute scratch; sfmm_execute_noalloc has " +
                                            std::to_string(kNoallocScratchBytes));
        unsigned char* base = noalloc_scratch();
        ExecScratch xs{(double*)base, (double*)(base + off_far), (float*)(base + off_mf)};
        hipStream_t s = (hipStream_t)stream;
        PoolStream ps(s, g_capturing);
        execute_impl(P, psi, defl, s, &xs, true);
        P.executed = true;
        if (P.done && !g_capturing) SFMM_HIP(hipEventRecord(P.done, s));
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SFMM_ERR_INTERNAL;
    }
}

sfmm_status sfmm_stats_get(sfmm_plan_t plan, sfmm_stats* out) {
    // (the exact direct-act pair count is computed here, outside planning)
    if (!plan || !out) {
        g_last_error = "plan or out is NULL";
        return SFMM_ERR_INVALID_ARG;
    }
    try {
        PoolStream ps(nullptr);
        const sfmm_plan_impl& P = *plan;
        P.wait();
        std::memset(out, 0, sizeof(*out));
        out->n_sources = P.N;
        out->n_targets = P.M;
        out->n_boxes = P.nbox;
        out->n_levels = (int64_t)P.lvl_start.size() - 1;
        std::vector<int> c0(P.nbox);
        if (P.nbox) SFMM_HIP(hipMemcpy(c0.data(), P.child0.data(), sizeof(int) * P.nbox, hipMemcpyDeviceToHost));
        out->n_leaves = std::count_if(c0.begin(), c0.end(), [](int v) { return v < 0; });
        out->n_m2l = P.n_m2l;
        out->n_p2p = P.n_p2p;
        if (P.ntl < 0) P.ntl = count_boxes(P.near_items, nullptr);
        out->n_target_leaves = P.ntl;
        if (P.n_p2p_pairs < 0 && P.nbox > 0) {
            DVec<long long> w, tot;
            w.resize(2 * (size_t)P.nbox);
            tot.resize(2);
            near_work(P.count.data(), P.nl, P.tcount.data(), P.nbox, w.data(), w.data() + P.nbox, nullptr);
            sum_i64(w.data(), P.nbox, tot.data(), nullptr);
            sum_i64(w.data() + P.nbox, P.nbox, tot.data() + 1, nullptr);
            long long h[2];
            SFMM_HIP(hipMemcpy(h, tot.data(), sizeof(h), hipMemcpyDeviceToHost));
            P.n_p2p_pairs = h[0];
            P.n_m2p_evals = h[1];
        }
        out->n_p2p_pairs = P.n_p2p_pairs < 0 ? 0 : P.n_p2p_pairs;
        out->n_m2p_evals = P.n_m2p_evals < 0 ? 0 : P.n_m2p_evals;
        if (P.executed && P.m2l_order_sq < 0)
            SFMM_HIP(hipMemcpy(&P.m2l_order_sq, P.osq_dev.data(), sizeof(long long), hipMemcpyDeviceToHost));
        out->m2l_order_sq = P.executed ? P.m2l_order_sq : 0;
        out->order = P.p;
        out->leaf_size = P.opt.leaf_size;
        out->q_total = P.q_total;
        out->execute_scratch_bytes = (int64_t)exec_scratch_bytes(P);
        out->judge_psi = P.judged ? P.judge_psi : -1.0;
        out->judge_alpha = P.judged ? P.judge_alpha : -1.0;
        out->judge_targets = P.judged ? P.judge_S : 0;
        out->fell_back = (P.judge_failed && !P.opt.no_fallback) ? 1 : 0;
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_export_boxes(sfmm_plan_t plan, int32_t* level, int64_t* pixel, int64_t* first, int64_t* count,
                              int64_t* parent, int64_t* child0, double* centre, double* radius) {
    try {
        if (!plan) throw Error(ST_INVALID_ARG, "plan is NULL");
        const sfmm_plan_impl& P = *plan;
        P.wait();
        const size_t nb = P.nbox;
        copy_widen(level, P.level.data(), nb);
        copy_widen(pixel, P.pixel.data(), nb);
        copy_widen(first, P.first.data(), nb);
        copy_widen(count, P.count.data(), nb);
        copy_widen(parent, P.parent.data(), nb);
        copy_widen(child0, P.child0.data(), nb);
        copy_widen(radius, P.rad.data(), nb);
        if (centre && nb) {
            std::vector<double> h(4 * nb);
            SFMM_HIP(hipMemcpy(h.data(), P.cen.data(), sizeof(double) * 4 * nb, hipMemcpyDeviceToHost));
            for (size_t b = 0; b < nb; ++b)
                for (int k = 0; k < 3; ++k) centre[k * nb + b] = h[4 * b + k];
        }
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_export_lists(sfmm_plan_t plan, int64_t* m2l_src, int64_t* m2l_tgt, int64_t* p2p_src,
                              int64_t* p2p_tgt) {
    try {
        if (!plan) throw Error(ST_INVALID_ARG, "plan is NULL");
        const sfmm_plan_impl& P = *plan;
        P.wait();
        export_csr(P.m2l_off, P.m2l_src, P.nbox, P.n_m2l, m2l_src, m2l_tgt);
        export_csr(P.p2p_off, P.p2p_src, P.nbox, P.n_p2p, p2p_src, p2p_tgt);
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_export_keys(sfmm_plan_t plan, uint64_t* src_keys, int64_t* src_perm, uint64_t* tgt_keys,
                             int64_t* tgt_perm, int64_t* tgt_leaf) {
    try {
        if (!plan) throw Error(ST_INVALID_ARG, "plan is NULL");
        const sfmm_plan_impl& P = *plan;
        P.wait();
        copy_widen(src_keys, P.skeys.data(), P.N);
        copy_widen(src_perm, P.sperm.data(), P.N);
        copy_widen(tgt_perm, P.tperm.data(), P.M);
        if (tgt_keys && P.M > 0) {  // the keys are kept in caller order
            std::vector<uint64_t> k(P.M);
            SFMM_HIP(hipMemcpy(k.data(), P.tkeys.data(), sizeof(uint64_t) * P.M, hipMemcpyDeviceToHost));
            std::vector<uint32_t> pm(P.M);
            SFMM_HIP(hipMemcpy(pm.data(), P.tperm.data(), sizeof(uint32_t) * P.M, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < P.M; ++i) tgt_keys[i] = k[pm[i]];
        }
        copy_widen(tgt_leaf, P.tleaf.data(), P.M);
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_export_work(sfmm_plan_t plan, int64_t* tgt_count, int64_t* pairs, int64_t* evals) {
    try {
        PoolStream ps(nullptr);
        if (!plan) throw Error(ST_INVALID_ARG, "plan is NULL");
        const sfmm_plan_impl& P = *plan;
        P.wait();
        if (P.N == 0 || P.nbox == 0) return SFMM_OK;
        copy_widen(tgt_count, P.tcount.data(), P.nbox);
        DVec<long long> w;
        w.resize(2 * (size_t)P.nbox);
        near_work(P.count.data(), P.nl, P.tcount.data(), P.nbox, w.data(), w.data() + P.nbox, nullptr);
        copy_widen(pairs, w.data(), P.nbox);
        copy_widen(evals, w.data() + P.nbox, P.nbox);
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_export_expansions(sfmm_plan_t plan, double* multipole, double* local) {
    try {
        PoolStream ps(nullptr);
        if (!plan) throw Error(ST_INVALID_ARG, "plan is NULL");
        const sfmm_plan_impl& P = *plan;
        P.wait();
        if (!P.executed) throw Error(ST_INVALID_ARG, "plan has not been executed");
        const int p = P.p, w = 2 * p + 2;
        const size_t nb = P.nbox;
        std::vector<double> cen(4 * nb);
        SFMM_HIP(hipMemcpy(cen.data(), P.cen.data(), sizeof(double) * 4 * nb, hipMemcpyDeviceToHost));
        auto unscale = [&](const DVec<double>& dev, double* out, bool is_local) {
            if (!out) return;
            SFMM_HIP(hipMemcpy(out, dev.data(), sizeof(double) * w * nb, hipMemcpyDeviceToHost));
            for (size_t b = 0; b < nb; ++b) {
                double* e = out + b * w;
                const double rho = cen[4 * b + 3];
                e[0] -= e[1];  // the zero-mean gauge share carried in C
                double f = 1.0;
                for (int l = 1; l <= p; ++l) {
                    f *= rho;
                    const double s = is_local ? 1.0 / f : f;
                    e[2 * l] *= s;
                    e[2 * l + 1] *= s;
                }
            }
        };
        unscale(P.mult, multipole, false);
        unscale(P.local, local, true);
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_order_samples(sfmm_plan_t plan, int64_t n, uint64_t seed, float* features, float* labels,
                               int64_t* pairs) {
    try {
        PoolStream ps(nullptr);
        if (!plan) throw Error(ST_INVALID_ARG, "plan is NULL");
        if (n < 0 || n > 0x7fffffff) throw Error(ST_INVALID_ARG, "n must be in [0, 2^31 - 1]");
        if (n > 0 && (!features || !labels)) throw Error(ST_INVALID_ARG, "features or labels is NULL");
        sfmm_plan_impl& P = *plan;
        P.wait();
        if (!P.executed) throw Error(ST_INVALID_ARG, "plan has not been executed");
        if (n == 0) return SFMM_OK;
        if (P.n_m2l == 0) throw Error(ST_INVALID_ARG, "plan has no FMM acts");
        hipStream_t s = nullptr;
        if (P.m2l_ent.n < (size_t)P.n_m2l) {
            P.m2l_ent.resize(P.n_m2l);
            entry_box(P.m2l_off.data(), P.nbox, P.n_m2l, P.m2l_ent.data(), s);
        }
        // pairs drawn with a counter-based generator (splitmix64)
        std::vector<int> idx(n);
        for (int64_t i = 0; i < n; ++i) {
            uint64_t z = seed + 0x9e3779b97f4a7c15ULL * (uint64_t)(i + 1);
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
            z ^= z >> 31;
            idx[i] = (int)(z % (uint64_t)P.n_m2l);
        }
        DVec<int> didx;
        DVec<float> feat, lab;
        didx.resize(n);
        feat.resize((size_t)n * kMlpIn);
        lab.resize(n);
        SFMM_HIP(hipMemcpy(didx.data(), idx.data(), sizeof(int) * n, hipMemcpyHostToDevice));
        const FmmCtx c = P.ctx();
        const double kt = SFMM_ORDER_KAPPA * P.opt.tolerance;
        P.decay.resize(P.nbox);
        order_box_decay(c, P.nbox, P.decay.data(), s);
        order_features(c, P.m2l_ent.data(), P.m2l_src.data(), didx.data(), n, P.decay.data(), kt, feat.data(), s);
        order_labels(c, P.m2l_ent.data(), P.m2l_src.data(), didx.data(), (int)n, kt, lab.data(), s);
        SFMM_HIP(hipMemcpy(features, feat.data(), sizeof(float) * n * kMlpIn, hipMemcpyDeviceToHost));
        SFMM_HIP(hipMemcpy(labels, lab.data(), sizeof(float) * n, hipMemcpyDeviceToHost));
        if (pairs) {
            std::vector<int> ent(P.n_m2l), src(P.n_m2l);
            SFMM_HIP(hipMemcpy(ent.data(), P.m2l_ent.data(), sizeof(int) * P.n_m2l, hipMemcpyDeviceToHost));
            SFMM_HIP(hipMemcpy(src.data(), P.m2l_src.data(), sizeof(int) * P.n_m2l, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n; ++i) {
                pairs[2 * i] = ent[idx[i]];
                pairs[2 * i + 1] = src[idx[i]];
            }
        }
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

void sfmm_mlp_init(uint64_t seed, float* weights) {
    if (!weights) return;
    // He-normal weights (Box-Muller on splitmix64), zero biases
    uint64_t st = seed;
    auto next = [&]() {
        uint64_t z = (st += 0x9e3779b97f4a7c15ULL);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    auto gauss = [&]() { return std::sqrt(-2.0 * std::log(next())) * std::cos(6.283185307179586 * next()); };
    float* w = weights;
    const int H = kMlpHidden, I = kMlpIn;
    for (int k = 0; k < H * I; ++k) *w++ = (float)(gauss() * std::sqrt(2.0 / I));
    for (int k = 0; k < H; ++k) *w++ = 0.0f;
    for (int k = 0; k < H * H; ++k) *w++ = (float)(gauss() * std::sqrt(2.0 / H));
    for (int k = 0; k < H; ++k) *w++ = 0.0f;
    for (int k = 0; k < H; ++k) *w++ = (float)(gauss() * std::sqrt(1.0 / H));
    *w++ = 0.0f;
}

sfmm_status sfmm_mlp_grad(const float* weights, const float* features, const float* labels, int64_t n,
                          float* grad, float* loss) {
    try {
        PoolStream ps(nullptr);
        if (n < 0 || n > (1 << 26)) throw Error(ST_INVALID_ARG, "n must be in [0, 2^26]");
        if (!weights || !grad || (n > 0 && (!features || !labels)))
            throw Error(ST_INVALID_ARG, "NULL buffer");
        check_finite(weights, kMlpWeights, "weights");
        check_finite(features, n * kMlpIn, "features");
        check_finite(labels, n, "labels");
        DVec<float> w, f, l, rec, g;
        w.resize(kMlpWeights);
        g.resize(kMlpWeights + 1);
        f.resize(std::max<int64_t>(n, 1) * kMlpIn);
        l.resize(std::max<int64_t>(n, 1));
        rec.resize(std::max<int64_t>(n, 1) * mlp_record_floats());
        SFMM_HIP(hipMemcpy(w.data(), weights, sizeof(float) * kMlpWeights, hipMemcpyHostToDevice));
        fill_f32(g.data(), kMlpWeights + 1, 0.0f, nullptr);
        if (n > 0) {
            SFMM_HIP(hipMemcpy(f.data(), features, sizeof(float) * n * kMlpIn, hipMemcpyHostToDevice));
            SFMM_HIP(hipMemcpy(l.data(), labels, sizeof(float) * n, hipMemcpyHostToDevice));
            mlp_grad(w.data(), f.data(), l.data(), (int)n, rec.data(), g.data(), nullptr);
        }
        std::vector<float> h(kMlpWeights + 1);
        SFMM_HIP(hipMemcpy(h.data(), g.data(), sizeof(float) * (kMlpWeights + 1), hipMemcpyDeviceToHost));
        std::memcpy(grad, h.data(), sizeof(float) * kMlpWeights);
        if (loss) *loss = h[kMlpWeights];
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_mlp_train(const float* features, const float* labels, int64_t n, int32_t epochs, int32_t batch,
                           float lr, uint64_t seed, float* weights, float* epoch_loss) {
    try {
        PoolStream ps(nullptr);
        if (n < 0 || n > (1 << 26)) throw Error(ST_INVALID_ARG, "n must be in [0, 2^26]");
        if (batch < 1 || epochs < 0 || !(lr > 0.0f)) throw Error(ST_INVALID_ARG, "batch, epochs or lr out of range");
        if (!weights || (n > 0 && (!features || !labels))) throw Error(ST_INVALID_ARG, "NULL buffer");
        check_finite(weights, kMlpWeights, "weights");
        check_finite(features, n * kMlpIn, "features");
        check_finite(labels, n, "labels");
        if (n == 0 || epochs == 0) return SFMM_OK;
        const int B = (int)std::min<int64_t>(batch, n);
        DVec<float> w, m, v, g, f, l, rec;
        w.resize(kMlpWeights);
        m.resize(kMlpWeights);
        v.resize(kMlpWeights);
        g.resize(kMlpWeights + 1);
        f.resize((size_t)n * kMlpIn);
        l.resize(n);
        rec.resize((size_t)B * mlp_record_floats());
        SFMM_HIP(hipMemcpy(w.data(), weights, sizeof(float) * kMlpWeights, hipMemcpyHostToDevice));
        fill_f32(m.data(), kMlpWeights, 0.0f, nullptr);
        fill_f32(v.data(), kMlpWeights, 0.0f, nullptr);
        // shuffled copies per epoch (Fisher-Yates on splitmix64)
        std::vector<int64_t> perm(n);
        std::vector<float> fs((size_t)n * kMlpIn), ls(n);
        uint64_t st = seed ^ 0x5bd1e995ULL;
        auto next = [&]() {
            uint64_t z = (st += 0x9e3779b97f4a7c15ULL);
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
            return z ^ (z >> 31);
        };
        int step = 0;
        std::vector<float> hl(kMlpWeights + 1);
        for (int ep = 0; ep < epochs; ++ep) {
            for (int64_t i = 0; i < n; ++i) perm[i] = i;
            for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[next() % (uint64_t)(i + 1)]);
            for (int64_t i = 0; i < n; ++i) {
                std::memcpy(&fs[i * kMlpIn], &features[perm[i] * kMlpIn], sizeof(float) * kMlpIn);
                ls[i] = labels[perm[i]];
            }
            SFMM_HIP(hipMemcpy(f.data(), fs.data(), sizeof(float) * n * kMlpIn, hipMemcpyHostToDevice));
            SFMM_HIP(hipMemcpy(l.data(), ls.data(), sizeof(float) * n, hipMemcpyHostToDevice));
            double ep_loss = 0.0;
            int nb = 0;
            for (int64_t b0 = 0; b0 + B <= n; b0 += B) {
                mlp_grad(w.data(), f.data() + b0 * kMlpIn, l.data() + b0, B, rec.data(), g.data(), nullptr);
                mlp_adam(w.data(), m.data(), v.data(), g.data(), lr, ++step, nullptr);
                if (epoch_loss) {
                    float lv;
                    SFMM_HIP(hipMemcpy(&lv, g.data() + kMlpWeights, sizeof(float), hipMemcpyDeviceToHost));
                    ep_loss += lv;
                    ++nb;
                }
            }
            if (epoch_loss) epoch_loss[ep] = nb ? (float)(ep_loss / nb) : 0.0f;
        }
        SFMM_HIP(hipMemcpy(weights, w.data(), sizeof(float) * kMlpWeights, hipMemcpyDeviceToHost));
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_mlp_forward(const float* weights, const float* features, int64_t n, int32_t bf16, float* y) {
    try {
        PoolStream ps(nullptr);
        if (n < 0 || n > (1 << 26)) throw Error(ST_INVALID_ARG, "n must be in [0, 2^26]");
        if (!weights || (n > 0 && (!features || !y))) throw Error(ST_INVALID_ARG, "NULL buffer");
        if (n == 0) return SFMM_OK;
        DVec<float> w, f, out;
        w.resize(kMlpWeights);
        f.resize((size_t)n * kMlpIn);
        out.resize(n);
        SFMM_HIP(hipMemcpy(w.data(), weights, sizeof(float) * kMlpWeights, hipMemcpyHostToDevice));
        SFMM_HIP(hipMemcpy(f.data(), features, sizeof(float) * n * kMlpIn, hipMemcpyHostToDevice));
        if (bf16) {
            FmmCtx c{};
            order_mlp(c, nullptr, nullptr, nullptr, 1.0, f.data(), n, w.data(), kMaxOrder, 0.0f, nullptr, out.data(),
                      nullptr);
        } else {
            mlp_forward_f32(w.data(), f.data(), (int)n, out.data(), nullptr);
        }
        SFMM_HIP(hipMemcpy(y, out.data(), sizeof(float) * n, hipMemcpyDeviceToHost));
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

sfmm_status sfmm_batch_plan(int32_t nshell, const double* const* src, const double* const* q, const int64_t* N,
                            const double* const* tgt, const int64_t* M, const sfmm_options* opt, void* stream,
                            sfmm_batch_t* out) {
    if (out) *out = nullptr;
    try {
        if (!out) throw Error(ST_INVALID_ARG, "out is NULL");
        if (nshell < 1 || nshell > 4096) throw Error(ST_INVALID_ARG, "nshell must be in [1, 4096]");
        if (!src || !q || !N || !tgt || !M) throw Error(ST_INVALID_ARG, "NULL array");
        std::unique_ptr<sfmm_batch_impl> B(new sfmm_batch_impl());
        hipStream_t s = (hipStream_t)stream;
        PoolStream ps(s);
        if (!s) SFMM_HIP(hipStreamCreateWithFlags(&B->own, hipStreamNonBlocking));
        B->plans.assign(nshell, nullptr);
        const int nw = std::min(nshell, kBatchPlanStreams);
        if (nw <= 1) {
            const sfmm_status st = sfmm_plan(src[0], q[0], N[0], tgt[0], M[0], opt, stream, &B->plans[0]);
            if (st != SFMM_OK) return st;
        } else {
            // The plans read sizes back on the host between their kernels; with
            // one host thread and one stream per worker, one shell's kernels fill
            // the GPU while another's host waits.  Shells go to workers largest
            // first, each to the least loaded (by N log N); the workers' streams
            // start after the caller's stream (the inputs may be written there)
            // and are waited for before this call returns.
            std::vector<hipStream_t>& ws = B->ws;
            ws.assign(nw, nullptr);
            hipEvent_t ready = nullptr;
            auto cleanup = [&]() {  // the streams stay with the batch (its destructor frees them)
                for (auto w : ws)
                    if (w) (void)hipStreamSynchronize(w);
                if (ready) (void)hipEventDestroy(ready);
            };
            try {
                SFMM_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
                SFMM_HIP(hipEventRecord(ready, s));
                for (auto& w : ws) {
                    SFMM_HIP(hipStreamCreateWithFlags(&w, hipStreamNonBlocking));
                    SFMM_HIP(hipStreamWaitEvent(w, ready, 0));
                }
            } catch (...) {
                cleanup();
                throw;
            }
            std::vector<int> idx(nshell);
            for (int i = 0; i < nshell; ++i) idx[i] = i;
            std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return N[a] > N[b]; });
            std::vector<std::vector<int>> mine(nw);
            std::vector<double> load(nw, 0.0);
            for (int i : idx) {
                const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                mine[w].push_back(i);
                load[w] += (double)std::max<int64_t>(N[i], 1) * std::log2((double)std::max<int64_t>(N[i], 2));
            }
            std::vector<sfmm_status> st(nw, SFMM_OK);
            std::vector<std::string> msg(nw);
            std::vector<std::thread> th;
            for (int w = 0; w < nw; ++w)
                th.emplace_back([&, w]() {
                    for (int i : mine[w]) {
                        st[w] = sfmm_plan(src[i], q[i], N[i], tgt[i], M[i], opt, ws[w], &B->plans[i]);
                        if (st[w] != SFMM_OK) {
                            msg[w] = g_last_error;
                            return;
                        }
                    }
                });
            for (auto& t : th) t.join();
            cleanup();
            for (int w = 0; w < nw; ++w)
                if (st[w] != SFMM_OK) throw Error(st[w], msg[w]);
            B->groups = std::move(mine);
            SFMM_HIP(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming));
            B->join.assign(nw, nullptr);
            for (auto& e : B->join) SFMM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        // the per-order split of the bound and learned policies reads sizes
        // on the host between kernels: those batches run without a graph
        B->capturable = !opt || opt->order_policy == SFMM_ORDER_FIXED;
        *out = B.release();
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SFMM_ERR_INTERNAL;
    }
}

sfmm_status sfmm_batch_plan_at(sfmm_batch_t batch, int32_t i, sfmm_plan_t* out) {
    if (!batch || !out || i < 0 || i >= (int32_t)batch->plans.size()) {
        g_last_error = "batch, out or index out of range";
        return SFMM_ERR_INVALID_ARG;
    }
    *out = batch->plans[i];
    return SFMM_OK;
}

sfmm_status sfmm_batch_execute(sfmm_batch_t batch, double* const* psi, double* const* defl, void* stream) {
    try {
        if (!batch || !psi || !defl) throw Error(ST_INVALID_ARG, "batch, psi or defl is NULL");
        sfmm_batch_impl& B = *batch;
        const size_t n = B.plans.size();
        hipStream_t caller = (hipStream_t)stream;
        hipStream_t s = caller ? caller : B.own;
        if (!s) throw Error(ST_INVALID_ARG, "the batch was planned with a stream: pass a stream");
        auto run_all = [&]() {
            for (size_t i = 0; i < n; ++i) {
                const sfmm_status st = sfmm_execute(B.plans[i], psi[i], defl[i], s);
                if (st != SFMM_OK) throw Error(st, g_last_error);
            }
        };
        // the shells spread over the worker streams, forked from and joined
        // back into s (recorded, this makes parallel branches of the graph):
        // one shell's latency-bound stretches (the coarse levels of Lemmas 2
        // and 4) overlap another's kernels
        auto run_par = [&]() {
            if (B.ws.empty()) return run_all();
            SFMM_HIP(hipEventRecord(B.fork, s));
            for (size_t w = 0; w < B.ws.size(); ++w) {
                SFMM_HIP(hipStreamWaitEvent(B.ws[w], B.fork, 0));
                for (int i : B.groups[w]) {
                    const sfmm_status st = sfmm_execute(B.plans[i], psi[i], defl[i], B.ws[w]);
                    if (st != SFMM_OK) throw Error(st, g_last_error);
                }
                SFMM_HIP(hipEventRecord(B.join[w], B.ws[w]));
                SFMM_HIP(hipStreamWaitEvent(s, B.join[w], 0));
            }
        };
        bool same = B.exec && B.g_stream == s;
        for (size_t i = 0; same && i < n; ++i) same = B.g_psi[i] == psi[i] && B.g_defl[i] == defl[i];
        if (same) {
            SFMM_HIP(hipGraphLaunch(B.exec, s));
        } else if (!B.capturable) {
            run_all();
        } else {
            B.drop_graph();
            // one direct pass (sizes every buffer a pass needs), then the same
            // pass recorded in a graph, which this call also launches
            run_par();
            SFMM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            g_capturing = true;
            try {
                run_par();
            } catch (...) {
                g_capturing = false;
                hipGraph_t g = nullptr;
                hipStreamEndCapture(s, &g);
                if (g) hipGraphDestroy(g);
                throw;
            }
            g_capturing = false;
            SFMM_HIP(hipStreamEndCapture(s, &B.graph));
            SFMM_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
            B.g_psi.assign(psi, psi + n);
            B.g_defl.assign(defl, defl + n);
            B.g_stream = s;
            SFMM_HIP(hipGraphLaunch(B.exec, s));
        }
        if (!B.done) SFMM_HIP(hipEventCreateWithFlags(&B.done, hipEventDisableTiming));
        SFMM_HIP(hipEventRecord(B.done, s));
        if (!caller) SFMM_HIP(hipStreamSynchronize(s));
        return SFMM_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SFMM_ERR_INTERNAL;
    }
}

void sfmm_batch_destroy(sfmm_batch_t batch) {
    if (!batch) return;
    PoolStream ps(nullptr, false, true);  // the destructor waits for the batch's work
    delete batch;
}

void sfmm_destroy(sfmm_plan_t plan) {
    if (!plan) return;
    // wait for the plan's last call, then its blocks may serve any stream
    if (plan->done) (void)hipEventSynchronize(plan->done);
    PoolStream ps(nullptr, false, true);
    delete plan;
}

// Global-basis helpers (Sec. 3.6): host arithmetic only, no device work.
sfmm_status sfmm_thetaphi_to_xyz(const double* theta, const double* phi, int64_t n, double* xyz) {
    if (n < 0 || (n > 0 && (!theta || !phi || !xyz))) {
        g_last_error = "thetaphi_to_xyz: n < 0 or a NULL buffer";
        return SFMM_ERR_INVALID_ARG;
    }
    for (int64_t i = 0; i < n; ++i) {
        const double st = std::sin(theta[i]);
        xyz[i] = st * std::cos(phi[i]);
        xyz[n + i] = st * std::sin(phi[i]);
        xyz[2 * n + i] = std::cos(theta[i]);
    }
    return SFMM_OK;
}

sfmm_status sfmm_defl_to_thetaphi(const double* xyz, const double* defl, const double* phi, int64_t n,
                                  double* out) {
    if (n < 0 || (n > 0 && (!xyz || !defl || !out))) {
        g_last_error = "defl_to_thetaphi: n < 0 or a NULL buffer";
        return SFMM_ERR_INVALID_ARG;
    }
    for (int64_t i = 0; i < n; ++i) {
        const double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
        const double ax = defl[i], ay = defl[n + i], az = defl[2 * n + i];
        const double rho = std::hypot(x, y);
        double et[3], ep[3];
        if (rho > 0.0) {
            const double c = x / rho, s = y / rho, ct = z / std::sqrt(rho * rho + z * z);
            const double st = rho / std::sqrt(rho * rho + z * z);
            et[0] = ct * c; et[1] = ct * s; et[2] = -st;
            ep[0] = -s; ep[1] = c; ep[2] = 0.0;
        } else {  // exact pole: the limit along the meridian phi
            const double f = phi ? phi[i] : 0.0, c = std::cos(f), s = std::sin(f);
            const double sg = z < 0.0 ? -1.0 : 1.0;
            et[0] = sg * c; et[1] = sg * s; et[2] = 0.0;
            ep[0] = -s; ep[1] = c; ep[2] = 0.0;
        }
        out[i] = ax * et[0] + ay * et[1] + az * et[2];
        out[n + i] = ax * ep[0] + ay * ep[1] + az * ep[2];
    }
    return SFMM_OK;
}

const char* sfmm_status_string(sfmm_status s) {
    switch (s) {
        case SFMM_OK: return "ok";
        case SFMM_ERR_INVALID_ARG: return "invalid argument";
        case SFMM_ERR_OUT_OF_MEMORY: return "out of device memory";
        case SFMM_ERR_HIP: return "HIP error";
        case SFMM_ERR_TOLERANCE_NOT_MET: return "tolerance not met";
        case SFMM_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char* sfmm_last_error(void) { return g_last_error.c_str(); }

void sfmm_profile_enable(int32_t on) { g_prof_on.store(on ? 1 : 0); }

void sfmm_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int i = 0; i < S_COUNT; ++i) {
        g_prof_ms[i] = 0.0;
        g_prof_calls[i] = 0;
    }
}

void sfmm_profile_read(double* ms, int64_t* calls) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int i = 0; i < S_COUNT; ++i) {
        if (ms) ms[i] = g_prof_ms[i];
        if (calls) calls[i] = g_prof_calls[i];
    }
}

}  // extern "C"
