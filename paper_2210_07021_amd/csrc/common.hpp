// Internal plumbing of libsfmm: error handling, the device memory pool,
// device vectors, and the launch wrappers that the host driver calls.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace sfmm {

// A failure anywhere below the C ABI is thrown as one of these and turned
// into a status code + message at the boundary.
struct Error : std::runtime_error {
    int status;
    Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

enum { ST_OK = 0, ST_INVALID_ARG = 1, ST_OOM = 2, ST_HIP = 3, ST_TOL = 4, ST_INTERNAL = 5 };

#define SFMM_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::sfmm::Error(::sfmm::ST_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

#define SFMM_LAUNCH_CHECK() SFMM_HIP(hipGetLastError())

// Caching device allocator: freed blocks are kept per size class and device
// and reused, so steady-state planning does no hipMalloc.  A freed block is
// reused only once the work queued before its release has finished, or by
// work on the same stream (stream order covers it): every API call names its
// stream with a PoolStream scope (capturing: a graph is being recorded on
// it; idle: the caller has already waited for all work that used the blocks
// freed in this scope), and the end of the scope records one event for all
// blocks freed in it.
void* pool_alloc(size_t bytes);
void pool_free(void* p);
void pool_release_all();
struct PoolStream {
    void* saved;  // the enclosing scope, restored at the end
    explicit PoolStream(hipStream_t s, bool capturing = false, bool idle = false);
    ~PoolStream();
    PoolStream(const PoolStream&) = delete;
    PoolStream& operator=(const PoolStream&) = delete;
};
// The reuse rule, exposed for host-side tests: a cached block freed on
// stream b.s (with a pending event when has_event, completed when
// event_done) may serve an allocation on stream `s` of device `dev`.
struct PoolBlockState {
    int dev;
    hipStream_t s;
    bool has_event, event_done;
};
inline bool pool_reusable(const PoolBlockState& b, hipStream_t s, int dev) {
    if (b.dev != dev) return false;
    if (!b.has_event) return true;  // released after its users were waited for
    return b.s == s || b.event_done;
}

template <typename T>
struct DVec {
    T* p = nullptr;
    size_t n = 0, cap = 0;
    DVec() = default;
    DVec(const DVec&) = delete;
    DVec& operator=(const DVec&) = delete;
    ~DVec() { reset(); }
    void reset() {
        if (p) pool_free(p);
        p = nullptr;
        n = cap = 0;
    }
    // resize without keeping contents
    void resize(size_t m) {
        if (m > cap) {
            reset();
            cap = m + m / 4 + 64;
            p = (T*)pool_alloc(cap * sizeof(T));
        }
        n = m;
    }
    // grow keeping contents (stream-ordered copy)
    void grow(size_t m, hipStream_t s) {
        if (m > cap) {
            size_t c2 = m + m / 2 + 64;
            T* q = (T*)pool_alloc(c2 * sizeof(T));
            if (p && n) SFMM_HIP(hipMemcpyAsync(q, p, n * sizeof(T), hipMemcpyDeviceToDevice, s));
            if (p) {
                // the pool may hand this block out again: make the copy finish first
                SFMM_HIP(hipStreamSynchronize(s));
                pool_free(p);
            }
            p = q;
            cap = c2;
        }
        n = m;
    }
    T* data() const { return p; }
    size_t size() const { return n; }
};

constexpr int kMaxOrder = 64;
// the tolerance map stops here: beyond it FP64 rounding, not truncation,
// sets the error (an explicit order may still go to kMaxOrder)
constexpr int kMaxTolOrder = 48;
// the order policy's measured error at order p (relative L2 of the
// deflection, worst over the calibration skies; the tolerance that gives
// order p is 4 times this)
double order_calibrated_error(int p);
// per-pair order policies: orders are multiples of kOrderStep; the order
// network maps kMlpIn features through two kMlpHidden ReLU layers to one
// output (kMlpWeights floats: W1, b1, W2, b2, w3, b3)
constexpr int kOrderStep = 4;
// the network predicts (order - kOrderCenter) / kOrderScale; kOrderMargin
// orders are added before rounding up
constexpr float kOrderCenter = 16.0f, kOrderScale = 8.0f, kOrderMargin = 2.0f;
constexpr int kMlpIn = 8, kMlpHidden = 64;
constexpr int kMlpWeights = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;

// every order 1..kMaxOrder is a template instance; SFMM_DISPATCH(p, X) runs
// X(P) for the runtime order p
#define SFMM_ORDERS(X)                                                                             \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) \
    X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32) X(33) \
    X(34) X(35) X(36) X(37) X(38) X(39) X(40) X(41) X(42) X(43) X(44) X(45) X(46) X(47) X(48) X(49) \
    X(50) X(51) X(52) X(53) X(54) X(55) X(56) X(57) X(58) X(59) X(60) X(61) X(62) X(63) X(64)

#define SFMM_DISPATCH(p, LAUNCH)                                                   \
    switch (p) {                                                                   \
        SFMM_ORDERS(LAUNCH)                                                        \
        default: throw Error(ST_INVALID_ARG, "expansion order out of range");     \
    }

// ---------------------------------------------------------------- utilities
void fill_f64(double* p, size_t n, double v, hipStream_t s);
void fill_f32(float* p, size_t n, float v, hipStream_t s);
void fill_i32(int* p, size_t n, int v, hipStream_t s);
// exclusive scan of n ints; the total goes to *total (device)
void scan_excl_i32(const int* in, int* out, int64_t n, int* total, hipStream_t s);
// three scans of n ints in one set of launches; total[0..2] their totals
void scan3_excl_i32(const int* in0, const int* in1, const int* in2, int* out0, int* out1, int* out2, int64_t n,
                    int* total, hipStream_t s);
// stable LSD radix sort of (key, value) pairs on key bits [begin_bit, bits)
void radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s, int begin_bit = 0);
// The same sort, ping-ponging between the caller's buffers (kalt / valt hold
// n elements; valt may be null when vals is): returns the buffer holding the
// sorted keys, *vout (if not null) the one holding the values.  With lo_out
// and hi_out (n elements each, n > 1 and bits > begin_bit), the last pass
// writes the sorted keys' low and high 32-bit halves there instead, and the
// returned buffer does not hold them.
uint64_t* radix_sort_u64_pp(uint64_t* keys, uint32_t* vals, uint64_t* kalt, uint32_t* valt, int64_t n, int bits,
                            hipStream_t s, int begin_bit, uint32_t** vout, uint32_t* lo_out = nullptr,
                            uint32_t* hi_out = nullptr);
void sum_f64(const double* x, int64_t n, double* out, hipStream_t s, int stride = 1);  // sum of x[i * stride]
void sum_i64(const long long* x, int64_t n, long long* out, hipStream_t s);

// ---------------------------------------------------------------- tree
// Copy [3][n] planes, check they are unit vectors (err bit 1: non-finite,
// bit 2: off the sphere by more than 1e-6), renormalise ones off by more
// than 1e-14, and compute their order-29 keys.
void prepare_points(const double* in, const double* q /*nullable*/, int64_t n, double4* u /*[n] x,y,z,q*/,
                    uint64_t* keys, uint32_t* idx, int* err, hipStream_t s);
void gather_targets(const uint32_t* idx, const uint64_t* leaf_sorted, int64_t n, const double4* u, double* ox,
                    double* oy, double* oz, int* leaf, hipStream_t s);
void gather_records(const uint32_t* idx, int64_t n, const double4* u, double4* out, hipStream_t s);
void tree_base_level(const uint64_t* keys, int64_t n, int* level, uint64_t* pixel, int* first, int* count,
                     int* parent, int* child0, hipStream_t s);
void tree_split_flags(int b0, int nb, const int* level, const int* count, int m, int max_level, int* flag,
                      hipStream_t s);
void tree_make_children(int b0, int nb, int child_base, const int* flag, const int* off, const uint64_t* keys,
                        int* level, uint64_t* pixel, int* first, int* count, int* parent, int* child0,
                        int wave_level, hipStream_t s);
void box_geometry(int nb, const int* level, const uint64_t* pixel, double* cen /*[nb][4]: x,y,z,rho*/,
                  double* rad, double* gdd /*[nb][8]*/, hipStream_t s);
void locate_targets(const uint64_t* keys, int64_t m, const int* child0, const int* level, uint64_t* leaf,
                    hipStream_t s);
// Queued tree levels (device-resident level bounds ls, chunk counts ccnt of
// at least ceil(cap / kTreeChunk) entries, per-box ranks wpre of cap
// entries, overflow flag ctl[0]).
constexpr int kTreeChunk = 1024;
// levels below wave_level boxes take a wave per box, larger ones a lane per
// box; kWaveLevel is the default (SFMM_WAVE_LEVEL overrides it, for tests)
constexpr int kWaveLevel = 65536;
int tree_wave_level();
void tree_init_queued(int* ls, int nls, int* ctl, hipStream_t s);
void tree_level_queued(int* ls, int L, int* ccnt, int* wpre, int grid, int cgrid, int cap, int* ctl, int m,
                       int split_ok, const uint64_t* keys, int* level, uint64_t* pixel, int* first, int* count,
                       int* parent, int* child0, int wave_level, hipStream_t s);
void target_ranges(const int* leaf, int64_t m, int nbox, int* tfirst, int* tcount, hipStream_t s);
void flag_nonzero(const int* count, int n, int* flag, hipStream_t s);
void compact_index(const int* flag, const int* off, int n, int* out, hipStream_t s);

// walk
struct WalkCtx {
    const int* child0;
    const int* count;
    const double4* geo;    // [nb] FP64 centre x, y, z and radius R
    const double2* strig;  // [nb] cos, sin of c_s R
    const double4* ttrig;  // [nb] cos, sin of R and of R / c_t
    const int2* cc;        // [nb] child0, count
    const double* gdd;     // [nb][8] double-double centre and radius
    const double* dtrig;   // [nb][kWalkDtrig] double-double cos, sin of the protected radius P, of R and
                           // of R / c_t, then P itself
    double c_s, c_t;
    double sigma;          // near-particle model radius: the protected radius is max(c_s R, R + sigma)
};
constexpr int kWalkDtrig = 14;
// the walk's per-box records (geo, cc) from the box table
void walk_boxes(int nb, const double* cen, const double* rad, const double* gdd, const int* child0, const int* count,
                double c_s, double c_t, double sigma, double4* geo, double2* strig, double4* ttrig, int2* cc,
                double* dtrig, hipStream_t s);
// Lanes per target box of the FP64 team M2L over n boxes: two
// (k_m2l_team2) when two-lane teams still fill the chip (two waves per SIMD
// on 256 CUs: 131072 lanes), four (k_m2l_team) below that; and of the
// precision tier's FP32 team M2L (k_m2l_team_f32).
constexpr int64_t kM2LTeam2MinBoxes = 65536;
inline int m2l_team_width(int64_t n) { return n >= kM2LTeam2MinBoxes ? 2 : 4; }
constexpr int kM2LTeamF32 = 4;
// M2L order: boxes of levels <= lc first, then the others; most team rounds
// first within each part, a round being tw_coarse pairs for the first part
// and tw_fine for the second (16-bit keys, ties in table order)
// One walk round in three launches (classify + per-chunk scans, scan of the
// chunk totals into tot[3]: children pairs, M2L pairs, P2P pairs; emit),
// sized on the device: st = {frontier size, M2L base, P2P base} of this
// round, st_next those of the next (written by the emit).  The per-round
// scratch (action [n], toff [3][tstride], ctot/coff [3][cstride]) must hold
// the round's n; cap bounds the next frontier and the two lists, and a round
// whose output would not fit writes nothing, sets *overflow and ends the walk.
struct WalkCaps {
    int frontier, m2l, p2p;
};
int walk_chunks(int n);  // chunks of a round of n pairs (at least 1)
void walk_round_scan(const int2* F, const int* st, const WalkCtx& w, uint8_t* action, int* ctot, int* coff,
                     int cstride, int* tot, int grid, hipStream_t s);
void walk_round_emit(const int2* F, const int* st, const WalkCtx& w, const uint8_t* action, const int* coff,
                     int cstride, const int* tot, const WalkCaps& cap, int2* Fnext, uint64_t* m2l, uint64_t* p2p,
                     int* st_next, int* overflow, int grid, hipStream_t s);
void m2l_order_keys(const int* off, const int* level, int lc, int tw_coarse, int tw_fine, int nbox, uint64_t* keys,
                    uint32_t* vals, hipStream_t s);
// precision tier: M2L into boxes of levels <= kFp32CoarseLevel stays FP64
// (the large contributions of coarse boxes nearly cancel on smooth skies,
// which FP32 rounding would show)
constexpr int kFp32CoarseLevel = 6;
// pairs (target << 32 | source) sorted by target -> CSR offsets and sources
// source and target box of every entry from sorted (target << 32 | source)
// keys, and CSR offsets from the sorted targets
void pair_split(const uint64_t* sorted, int np, int* src, int* tgt, hipStream_t s);
void csr_offsets(const int* tgt, int np, int nbox, int* off, hipStream_t s);
// sort keys (8 bits) putting the boxes with the most work first, in
// power-of-two buckets; flag the boxes that have any
void work_order_keys(const long long* work, int n, uint64_t* keys, uint32_t* vals, int* flag, hipStream_t s);
// ---------------------------------------------------------------- fmm
struct FmmCtx {
    int p;
    const double* cen;   // [nb][4] x, y, z, rho
    const double* rad;   // [nb] box radius R
    const int* level;
    const int* first;
    const int* count;
    const int* parent;
    const int* child0;
    const double4* spt;  // sources sorted by key: x, y, z, q
    double* mult;        // [nb][2p+2]
    double* local;       // [nb][2p+2]
    const double* zrec;  // [2p+2] zeros
    double npm_sigma;    // near-particle model radius (0: point masses)
};
// Near-particle model (Epanechnikov profile of radius sigma): with u =
// |d|^2/4 and t = sin^2(sigma/2), the interior potential is (q/4pi)(log t -
// I(u/t)), I(v) = integral_v^1 (2 - v' - t)/(1 - v' t) dv'
// = sum_k t^k [(2 - t)(1 - v^(k+1))/(k+1) - (1 - v^(k+2))/(k+2)], and the
// potential of every particle carries the constant (q/4pi) c(t), c = t (J -
// 1), J = sum_k t^k [(2 - t)/(k + 2) - 1/(k + 3)] (so that it integrates to
// -q over the sphere like a point mass's).  npm_constant(sigma) = c(t).
double npm_constant(double sigma);
struct NpmK {
    double t, inv_t, four_t, ln4t, a2;  // a2 = ((1 - t)/t)^2 / 16
    int nterms;                         // terms of the series for I
};
NpmK npm_params(double sigma);
void fmm_p2m(const FmmCtx& c, int nb, hipStream_t s);
void fmm_m2m(const FmmCtx& c, int b0, int nb, hipStream_t s);
// M2L at order p <= c.p over the boxes order[0..n) (order may be null: box
// i); acc_in adds to the local records instead of overwriting them
void fmm_m2l(const FmmCtx& c, int p, bool acc_in, const int* order, int n, const int* off, const int* src,
             hipStream_t s);
// precision tier: FP32 copy of the multipole A-blocks ([nbox][2 c.p]), and
// M2L with FP32 A-block arithmetic (p, acc_in, order as fmm_m2l)
void mult_to_f32(const FmmCtx& c, int nbox, float* multf, hipStream_t s);
void fmm_m2l_f32(const FmmCtx& c, int p, bool acc_in, const float* multf, const int* order, int n, const int* off,
                 const int* src, hipStream_t s);
// record orders (5..24) at which the precision tier runs the order classes
// of a per-pair order policy with each pair's monopole part completed up to
// c.p inside the class (fmm_m2l_f32_classes)
bool m2l_f32_tail_supported(int p);
// the precision tier's boxes of a per-pair order policy: every order class
// of every box in one launch (boff: class-major CSR over nbox boxes)
void fmm_m2l_f32_classes(const FmmCtx& c, const float* multf, const int* order, int n, const int* boff,
                         const int* bsrc, int nbox, hipStream_t s);
// and its FP64 boxes (the coarse levels), likewise in one launch
void fmm_m2l_f64_classes(const FmmCtx& c, const int* order, int n, const int* boff, const int* bsrc, int nbox,
                         hipStream_t s);
void fmm_l2l(const FmmCtx& c, int b0, int nb, hipStream_t s);
// (kappa - kappa_bar, gamma_1, gamma_2, mu) [4][m] from the Hessian [3][m]
void lensing_from_hessian(const double* hess, int64_t m, double* out, hipStream_t s);
// hess [3][m_out] (may be null): also the Hessian of Sec. 2.2 in the
// targets' e_theta, e_phi basis (written, like psi and defl)
void fmm_l2p(const FmmCtx& c, const double* tx, const double* ty, const double* tz, const int* tleaf,
             const uint32_t* tperm, int64_t m, double psi_shift, double* psi, double* defl, int64_t m_out,
             hipStream_t s, double* hess = nullptr);
// Direct-act lists split into the leaves summed particle by particle (near)
// and those taken through their multipole expansion (far), both in CSR form
// by target box, with the work each box gives the two kernels.
struct NearLists {
    DVec<int> near_off, near_src, far_off, far_src;  // the src arrays hold np entries' room
};
void near_split(const FmmCtx& c, const int* off, const int* src, const int* ent_t, int nbox, int np,
                const int* tfirst, const int* tcount, const double* tx, const double* ty, const double* tz,
                NearLists& out, hipStream_t s);
// Near-field work items: segment [y, z) of box x's list, results to the
// outputs (w < 0) or to partial slots w .. w + tcount[x] - 1; reduce records
// (box, segments, first slot) for the boxes cut into several segments.
struct WorkItems {
    DVec<int4> items, red;
    DVec<double> part;  // [nslot][4]
    int n = 0, nred = 0, nslot = 0;
};
constexpr int kSegNear = 128;  // close leaves per direct-sum item
constexpr int kSegFar = 128;   // close leaves per expansion item
// Work items of two lists of the same boxes (a and b; seg close leaves per
// item), with one read-back of the totals; count == nullptr: work counted
// per entry instead of per particle
void build_items2(const int* off_a, const int* src_a, const int* count_a, int seg_a, WorkItems& out_a,
                  const int* off_b, const int* src_b, const int* count_b, int seg_b, WorkItems& out_b,
                  const int* tcount, int nbox, hipStream_t s);
// per box: pairs[b] = targets x particles of the near leaves, evals[b] =
// targets x far leaves
void near_work(const int* count, const NearLists& nl, const int* tcount, int nbox, long long* pairs,
               long long* evals, hipStream_t s);
// fp32: the precision tier's pair arithmetic (two-float coordinates, FP32
// log / reciprocal, FP64 sums per tile)
// part: the partial slots of the split boxes ([w.nslot][4] doubles), or
// null for the work items' own buffer w.part.  hess (may be null): also add
// the Hessian of Sec. 2.2 to hess [3][m_out]; part then has [w.nslot][8]
// doubles and may not be null.
void fmm_p2p(const FmmCtx& c, bool fp32, const WorkItems& w, const int* src, const int* tfirst,
             const int* tcount, const double* tx, const double* ty, const double* tz, const uint32_t* tperm,
             double* psi, double* defl, int64_t m_out, hipStream_t s, double* part = nullptr,
             double* hess = nullptr);
void fmm_m2p(const FmmCtx& c, const WorkItems& w, const int* src, const int* tfirst, const int* tcount,
             const double* tx, const double* ty, const double* tz, const uint32_t* tperm, double* psi,
             double* defl, int64_t m_out, hipStream_t s, double* part = nullptr, double* hess = nullptr);

// ---------------------------------------------------------------- multi-plane rays
// A = identity [4][m]; one layer's step of the rays [3][m] by -w defl (along
// great circles) and, with dist [4][m] (may be null), A <- T (I - w H) A
void ray_identity(double* dist, int64_t m, hipStream_t s);
void ray_step(double* rays, const double* defl, const double* hess, double w, int64_t m, double* dist,
              hipStream_t s);

// ---------------------------------------------------------------- judge
// Direct sum at S targets of the caller (caller-order positions pos[S]) over
// the n sorted sources, FP64 with compensated sums, in three steps:
// judge_targets gathers the targets from the caller's tgt [3][m] (unit
// vectors as the plan makes them) into tsel [S]; judge_sum writes the
// per-chunk sums part [judge_part_doubles] (it needs only the sorted sources,
// so the plan runs it beside its own later stages); judge_outputs gives ref
// [S][4] = (psi + shift, alpha x, y, z) from part and got [S][4] = the
// library's outputs psi/defl (caller order, m targets) there.
size_t judge_part_doubles(int64_t n, int S);
void judge_targets(const int* pos, int S, const double* tgt, int64_t m, double4* tsel, hipStream_t s);
void judge_sum(const double4* spt, int64_t n, const double4* tsel, int S, double* part, hipStream_t s);
void judge_outputs(const int* pos, int S, const double4* tsel, const double* part, int64_t n, double shift,
                   const double* psi, const double* defl, int64_t m, double* ref, double* got, hipStream_t s);

// ---------------------------------------------------------------- order policies
void entry_box(const int* off, int nbox, int np, int* ent_t, hipStream_t s);
void order_box_decay(const FmmCtx& c, int nbox, float4* decay, hipStream_t s);
void order_features(const FmmCtx& c, const int* ent_t, const int* src, const int* idx, int64_t n,
                    const float4* decay, double kappa_tol, float* feat, hipStream_t s);
void order_bound(const FmmCtx& c, const int* ent_t, const int* src, int np, double kappa_tol, uint8_t* ord,
                 hipStream_t s);
// feat null: the features of pairs 0..n) are computed in place from (c, ent_t, src, decay, kappa_tol)
void order_mlp(const FmmCtx& c, const int* ent_t, const int* src, const float4* decay, double kappa_tol,
               const float* feat, int64_t n, const float* w, int pmax, float margin, uint8_t* ord, float* y,
               hipStream_t s);
// monopole part of the local coefficients above each pair's order (pairs in
// the full CSR off/src with their orders ord)
void m2l_qtail(const FmmCtx& c, const int* off, const int* src, const uint8_t* ord, int nbox, hipStream_t s);
void order_labels(const FmmCtx& c, const int* ent_t, const int* src, const int* idx, int n, double kappa_tol,
                  float* label, hipStream_t s);
// split pairs by order into CSR lists boff + q nbox over bsrc, class q
// holding the orders in (q kOrderStep, (q + 1) kOrderStep], q < ceil(pmax /
// kOrderStep); the sum of the orders squared goes to osq (device)
void order_split(const int* off, const int* src, const uint8_t* ord, int nbox, int np, int pmax,
                 DVec<int>& boff, DVec<int>& bsrc, long long* osq, hipStream_t s);
void mlp_grad(const float* w, const float* feat, const float* label, int n, float* rec, float* grad, hipStream_t s);
void mlp_adam(float* w, float* m, float* v, const float* grad, float lr, int step, hipStream_t s);
void mlp_forward_f32(const float* w, const float* feat, int n, float* y, hipStream_t s);
size_t mlp_record_floats();

}  // namespace sfmm
