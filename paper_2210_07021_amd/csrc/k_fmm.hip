// The numeric passes of the sFMM (Sec. 3.2-3.3, 3.6): Lemma 1 on leaves,
// Lemma 2 up the tree, Lemma 3 over the FMM-act lists, Lemma 4 down the
// tree, and the local expansion at each target.  One lane owns one box (or
// one target) and holds its order-P coefficients in registers; P is a
// template parameter so every loop over l unrolls.
#include "common.hpp"
#include "expand.hpp"

namespace sfmm {

// Sum of a double over the four lanes of a quad (lanes 4i .. 4i + 3), every
// lane getting the sum: two butterfly steps with DPP quad permutations
// (lane exchanges inside the VALU, no LDS), (v0 + v1) + (v2 + v3) on every
// lane of the quad.
// Every lane of a quad is active wherever these are called (a team's four
// lanes run the same iterations), so no lane reads a disabled one and the
// bound-control form needs no old value (no extra register move).
template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
    const int hi2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi2, lo2);
}
__device__ __forceinline__ double pair_sum(double v) {
    return v + dpp_quad<0xB1>(v);  // quad_perm [1, 0, 3, 2]: lane ^ 1
}
__device__ __forceinline__ double quad_sum(double v) {
    v += dpp_quad<0xB1>(v);     // quad_perm [1, 0, 3, 2]: lane ^ 1
    return v + dpp_quad<0x4E>(v);  // quad_perm [2, 3, 0, 1]: lane ^ 2
}

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1); }

__device__ __forceinline__ Frame box_frame(const double* cen, int b, double* rho) {
    const double* c = cen + 4 * (size_t)b;
    *rho = c[3];
    return make_frame(c[0], c[1], c[2]);
}

// Lemma 1 on every leaf (an empty leaf gets a zero record: with the split
// boxes written by k_m2m, every record is written and needs no clearing)
template <int P>
__global__ void __launch_bounds__(128) k_p2m(FmmCtx c, int nb) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb || c.child0[b] >= 0) return;
    if (c.count[b] == 0) {
        double* out = c.mult + (size_t)b * (2 * P + 2);
        for (int k = 0; k < 2 * P + 2; ++k) out[k] = 0.0;
        return;
    }
    double rho;
    const Frame f = box_frame(c.cen, b, &rho);
    const double inv_rho = 1.0 / rho;
    P2MAcc<P> a;
    p2m_init<P>(a);
    const int i0 = c.first[b], i1 = i0 + c.count[b];
    for (int i = i0; i < i1; ++i) {
        const double4 v = c.spt[i];
        p2m_add<P>(a, f, inv_rho, v.x, v.y, v.z, v.w);
    }
    p2m_finish<P>(a, c.mult + (size_t)b * (2 * P + 2));
}

// Lemma 2: every split box of one level gathers its 4 children.  Four
// consecutive lanes per box, lane 4i + k translating child k (an empty child
// has a zero record); each output entry is summed over the four lanes by two
// lane exchanges, (c0 + c1) + (c2 + c3), as it is formed, and lane 4i writes
// it.
template <int P>
__global__ void __launch_bounds__(128) k_m2m(FmmCtx c, int b0, int nb) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 2, kc = gid & 3;
    if (i >= nb) return;  // the four lanes of a box leave together
    const int b = b0 + i;
    const int ch0 = c.child0[b];
    if (ch0 < 0) return;
    const int ch = ch0 + kc;
    double rho_t, rho_s;
    const Frame ft = box_frame(c.cen, b, &rho_t);
    const Frame fs = box_frame(c.cen, ch, &rho_s);
    const TransGeom G = trans_geom<kM2M>(fs, rho_s, ft, rho_t);
    const double* in = c.mult + (size_t)ch * (2 * P + 2);
    double* out = c.mult + (size_t)b * (2 * P + 2);
    translate_emit<P>([&](int k) { return in[k]; }, G, [&](int k, double v) {
        const double s = quad_sum(v);
        if (kc == 0) out[k] = s;
    });
}

// Lemma 3 with four lanes per target box (a team): in each round lane r of
// the team translates entry k0 + 4 round + r of the box's list (a zero
// record past the end); every output entry is summed over the team by two
// lane exchanges as it is formed and added by the lane that owns it (entry
// k by lane k mod 4), so no lane holds the whole accumulator and two waves
// fit on a SIMD.
// Lemma 3 with four lanes per target box (a team): in each round lane r of
// the team translates entry k0 + 4 round + r of the box's list (a zero
// record past the end).  Every output entry is summed over the team as it
// is formed (quad_sum); the accumulator is shared out: lane r owns entries
// 2 + 4q + r (slot q) and, for r < 2, entry r (slot NG), in LDS.  The sums
// of entries 2 + 4q .. 5 + 4q are held until the group is complete and then
// each lane adds its own with one LDS add (single writer per slot, so the
// sums keep their round order).  No lane holds the whole accumulator: two
// waves fit on a SIMD.  Target boxes are taken in `order` (most rounds
// first, so the teams of a wave carry the same work).  P is the order of the
// translation, c.p that of the records (P <= c.p: a per-pair order policy
// runs one pass per order with the pairs of that order, adding to the
// records' first 2P + 2 entries, acc_in = true; a first pass, acc_in =
// false, writes whole records).
template <int P>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2)))
k_m2l_team(FmmCtx c, const int* order, int n, const int* off, const int* src, bool acc_in) {
    constexpr int EW = 2 * P + 2, NG = (2 * P + 3) / 4, NA = NG + 1;
    __shared__ double sacc[NA * 128];
    double* acc = sacc + threadIdx.x;  // slot q at acc[q * 128]
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 2, r = gid & 3;
    if (i >= n) return;  // the four lanes of a team leave together
    const int t = order ? order[i] : i;
    const int k0 = off[t], k1 = off[t + 1];
    const size_t ew = 2 * (size_t)c.p + 2;
    double* out = c.local + (size_t)t * ew;
    if (k0 == k1) {
        if (!acc_in)
            for (size_t k = r; k < ew; k += 4) out[k] = 0.0;
        return;
    }
    auto entry = [&](int q) { return q < NG ? 2 + 4 * q + r : r; };  // entry held in slot q (r < 2 for slot NG)
    for (int q = 0; q < NA; ++q) {
        const int e = entry(q);
        acc[q * 128] = (acc_in && e < EW && (q < NG || r < 2)) ? out[e] : 0.0;
    }
    double rho_t;
    const Frame ft = box_frame(c.cen, t, &rho_t);
    for (int kb = k0; kb < k1; kb += 4) {
        const int k = kb + r;
        const bool live = k < k1;
        const int s = live ? src[k] : src[k0];
        double rho_s;
        const Frame fs = box_frame(c.cen, s, &rho_s);
        const TransGeom G = trans_geom<kM2L>(fs, rho_s, ft, rho_t);
        const double* in = live ? c.mult + (size_t)s * ew : c.zrec;
        double pend[4], cq[2];
        translate_emit<P>([&](int e) { return in[e]; }, G, [&](int e, double v) {
            const double sum = quad_sum(v);
            if (e < 2) {
                cq[e] = sum;
                return;
            }
            const int j = (e - 2) & 3;
            pend[j] = sum;
            if (j == 3 || e == EW - 1) {  // group complete: lane r adds entry 2 + 4q + r
                const double mine = r == 0 ? pend[0] : r == 1 ? pend[1] : r == 2 ? pend[2] : pend[3];
                if (j == 3 || r <= j)  // a partial last group holds entries up to lane j's
                    __hip_atomic_fetch_add(acc + ((e - 2) >> 2) * 128, mine, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        });
        if (r < 2) __hip_atomic_fetch_add(acc + NG * 128, r == 0 ? cq[0] : cq[1], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    for (int q = 0; q < NA; ++q) {
        const int e = entry(q);
        if (e < EW && (q < NG || r < 2)) out[e] = acc[q * 128];
    }
    if (!acc_in)
        for (size_t k = EW + r; k < ew; k += 4) out[k] = 0.0;
}

// Lemma 3 with two lanes per target box (a team): in each round lane r of
// the team translates entry k0 + 2 round + r of the box's list (a zero
// record past the end).  Every output entry is summed over the team as it
// is formed (one DPP exchange and an add, pair_sum); the accumulator is
// shared out: lane r owns entries 2 + 2q + r (slot q) and entry r (slot
// NG), in LDS.  The sums of entries 2 + 2q and 3 + 2q are held until both
// are formed and then each lane adds its own with one LDS add (single
// writer per slot, so the sums keep their round order).  No lane holds the
// whole accumulator: two waves fit on a SIMD.  Against k_m2l_team (four
// lanes, two DPP steps a sum, lists padded to rounds of four) this runs ~7 %
// faster at p = 38 with fewer spilled registers, when there are enough boxes
// to fill the chip with half as many lanes (m2l_team_width).  Order, P and
// acc_in as in k_m2l_team.
template <int P>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2)))
k_m2l_team2(FmmCtx c, const int* order, int n, const int* off, const int* src, bool acc_in) {
    constexpr int EW = 2 * P + 2, NG = P, NA = NG + 1;
    __shared__ double sacc[NA * 128];
    double* acc = sacc + threadIdx.x;  // slot q at acc[q * 128]
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 1, r = gid & 1;
    if (i >= n) return;  // the two lanes of a team leave together
    const int t = order ? order[i] : i;
    const int k0 = off[t], k1 = off[t + 1];
    const size_t ew = 2 * (size_t)c.p + 2;
    double* out = c.local + (size_t)t * ew;
    if (k0 == k1) {
        if (!acc_in)
            for (size_t k = r; k < ew; k += 2) out[k] = 0.0;
        return;
    }
    auto entry = [&](int q) { return q < NG ? 2 + 2 * q + r : r; };  // entry held in slot q
    for (int q = 0; q < NA; ++q) acc[q * 128] = acc_in ? out[entry(q)] : 0.0;
    double rho_t;
    const Frame ft = box_frame(c.cen, t, &rho_t);
    for (int kb = k0; kb < k1; kb += 2) {
        const int k = kb + r;
        const bool live = k < k1;
        const int s = live ? src[k] : src[k0];
        double rho_s;
        const Frame fs = box_frame(c.cen, s, &rho_s);
        const TransGeom G = trans_geom<kM2L>(fs, rho_s, ft, rho_t);
        const double* in = live ? c.mult + (size_t)s * ew : c.zrec;
        double pend[2];
        translate_emit<P>([&](int e) { return in[e]; }, G, [&](int e, double v) {
            const double sum = pair_sum(v);
            pend[e & 1] = sum;
            if (e & 1)  // entries e - 1, e complete: lane r adds entry e - 1 + r
                __hip_atomic_fetch_add(acc + (e < 2 ? NG : (e - 2) >> 1) * 128, r == 0 ? pend[0] : pend[1],
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        });
    }
    for (int q = 0; q < NA; ++q) out[entry(q)] = acc[q * 128];
    if (!acc_in)
        for (size_t k = EW + r; k < ew; k += 2) out[k] = 0.0;
}

// Precision tier: FP32 copy of every multipole A-block, [nb][2p]
__global__ void k_mult_to_f32(const double* __restrict__ mult, int p, int nb, float* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nb * 2 * p) return;
    const int64_t b = i / (2 * p), k = i - b * (2 * p);
    out[i] = (float)mult[b * (2 * p + 2) + 2 + k];
}

// Precision tier Lemma 3 with four lanes per target box, as k_m2l_team: in
// each round lane r of the team translates entry k0 + 4 round + r of the
// box's list.  The translation runs in FP32 on the FP32 A-block copy
// (multf); each lane adds its results into FP64 running sums held in
// registers (the FP32 working vector leaves room for them), and at the end
// the team's four sums of every entry are added by two DPP lane exchanges
// and written by the lane that owns the entry (entry k by lane k mod 4).
// C and Q stay FP64.  P and acc_in as in k_m2l_team.
template <int P>
__global__ void __launch_bounds__(128) k_m2l_team_f32(FmmCtx c, const float* __restrict__ multf, const int* order,
                                                     int n, const int* off, const int* src, bool acc_in) {
    static_assert(kM2LTeamF32 == 4, "the sums below are over quads");
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 2, r = gid & 3;
    if (i >= n) return;  // the four lanes of a team leave together
    const int t = order ? order[i] : i;
    const int k0 = off[t], k1 = off[t + 1];
    const size_t ew = 2 * (size_t)c.p + 2, fw = 2 * (size_t)c.p;
    double* out = c.local + (size_t)t * ew;
    if (k0 == k1) {
        if (!acc_in)
            for (size_t k = r; k < ew; k += 4) out[k] = 0.0;
        return;
    }
    double rho_t;
    const Frame ft = box_frame(c.cen, t, &rho_t);
    double acc[2 * P + 2];  // C, Q, then the A-block
#pragma unroll
    for (int k = 0; k < 2 * P + 2; ++k) acc[k] = 0.0;
    for (int k = k0 + r; k < k1; k += 4) {
        const int s = src[k];
        double rho_s;
        const Frame fs = box_frame(c.cen, s, &rho_s);
        const TransGeom G = trans_geom<kM2L>(fs, rho_s, ft, rho_t);
        const double* e = c.mult + (size_t)s * ew;
        translate_add_f32_d<P>(multf + (size_t)s * fw, e[0], e[1], G, acc + 2, acc);
    }
#pragma unroll
    for (int k = 0; k < 2 * P + 2; ++k) {
        const double v = quad_sum(acc[k]);
        if ((k & 3) == r) out[k] = acc_in ? out[k] + v : v;
    }
    if (!acc_in)
        for (size_t k = 2 * P + 2 + r; k < ew; k += 4) out[k] = 0.0;  // a first pass below the record order
}

// Precision tier Lemma 3 for a per-pair order policy in one launch: the
// pairs of every target box come split by order class (class q holds the
// orders in (4q, 4q + 4], the top class the record order PO; boff is the
// class-major CSR of order_split), and each team runs its box's classes one
// after another, the pairs of class q translated at order min(4q + 4, PO)
// with their monopole part completed up to PO, all into the same FP64
// running sums.  Against one launch per class this reads and writes every
// local record once and launches once.  Writes whole records (no acc_in).
template <int PO, int Q>
__device__ __forceinline__ void m2l_f32_class(const FmmCtx& c, const float* __restrict__ multf, const Frame& ft,
                                              double rho_t, const int* boff, const int* bsrc, int nbox, int t,
                                              int r, double* acc) {
    constexpr int P = (Q + 1) * kOrderStep < PO ? (Q + 1) * kOrderStep : PO;
    const size_t ew = 2 * (size_t)c.p + 2, fw = 2 * (size_t)c.p;
    const int k1 = boff[(size_t)Q * nbox + t + 1];
    for (int k = boff[(size_t)Q * nbox + t] + r; k < k1; k += 4) {
        const int s = bsrc[k];
        double rho_s;
        const Frame fs = box_frame(c.cen, s, &rho_s);
        const TransGeom G = trans_geom<kM2L>(fs, rho_s, ft, rho_t);
        const double* e = c.mult + (size_t)s * ew;
        translate_add_f32_d<P, PO>(multf + (size_t)s * fw, e[0], e[1], G, acc + 2, acc);
    }
    if constexpr (P < PO) m2l_f32_class<PO, Q + 1>(c, multf, ft, rho_t, boff, bsrc, nbox, t, r, acc);
}

template <int PO>
__global__ void __launch_bounds__(128) k_m2l_team_f32_classes(FmmCtx c, const float* __restrict__ multf,
                                                              const int* order, int n, const int* boff,
                                                              const int* bsrc, int nbox) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 2, r = gid & 3;
    if (i >= n) return;  // the four lanes of a team leave together
    const int t = order[i];
    double* out = c.local + (size_t)t * (2 * (size_t)c.p + 2);
    double rho_t;
    const Frame ft = box_frame(c.cen, t, &rho_t);
    double acc[2 * PO + 2];  // C, Q, then the A-block
#pragma unroll
    for (int k = 0; k < 2 * PO + 2; ++k) acc[k] = 0.0;
    m2l_f32_class<PO, 0>(c, multf, ft, rho_t, boff, bsrc, nbox, t, r, acc);
#pragma unroll
    for (int k = 0; k < 2 * PO + 2; ++k) {
        const double v = quad_sum(acc[k]);
        if ((k & 3) == r) out[k] = v;
    }
}

void fmm_m2l_f32_classes(const FmmCtx& c, const float* multf, const int* order, int n, const int* boff,
                         const int* bsrc, int nbox, hipStream_t s) {
    if (n <= 0) return;
    if (!m2l_f32_tail_supported(c.p)) throw Error(ST_INTERNAL, "record order outside the per-pair order M2L instances");
    const unsigned g = nblk(kM2LTeamF32 * (int64_t)n, 128);
    switch (c.p) {
#define C_(PO) case PO: k_m2l_team_f32_classes<PO><<<g, 128, 0, s>>>(c, multf, order, n, boff, bsrc, nbox); break;
        C_(5) C_(6) C_(7) C_(8) C_(9) C_(10) C_(11) C_(12) C_(13) C_(14)
        C_(15) C_(16) C_(17) C_(18) C_(19) C_(20) C_(21) C_(22) C_(23) C_(24)
#undef C_
        default: throw Error(ST_INTERNAL, "record order outside the per-pair order M2L instances");
    }
    SFMM_LAUNCH_CHECK();
}

// The FP64 boxes of the precision tier (its coarse levels) under a per-pair
// order policy, every order class in one launch: four lanes per box, each
// lane holding the box's whole accumulator in registers (two waves per SIMD
// at the tier's orders), running the box's classes one after another (class
// q at order min(4q + 4, PO), each pair's monopole part completed to PO), the
// four sums of every entry added across the quad at the end.  Writes whole
// records.
template <int PO, int Q>
__device__ __forceinline__ void m2l_f64_class(const FmmCtx& c, const Frame& ft, double rho_t, const int* boff,
                                              const int* bsrc, int nbox, int t, int r, double* acc) {
    constexpr int P = (Q + 1) * kOrderStep < PO ? (Q + 1) * kOrderStep : PO;
    const size_t ew = 2 * (size_t)c.p + 2;
    const int k1 = boff[(size_t)Q * nbox + t + 1];
    for (int k = boff[(size_t)Q * nbox + t] + r; k < k1; k += 4) {
        const int s = bsrc[k];
        double rho_s;
        const Frame fs = box_frame(c.cen, s, &rho_s);
        const TransGeom G = trans_geom<kM2L>(fs, rho_s, ft, rho_t);
        translate_add_po<P, PO>(c.mult + (size_t)s * ew, G, acc);
    }
    if constexpr (P < PO) m2l_f64_class<PO, Q + 1>(c, ft, rho_t, boff, bsrc, nbox, t, r, acc);
}

template <int PO>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2)))
k_m2l_team_f64_classes(FmmCtx c, const int* order, int n, const int* boff, const int* bsrc, int nbox) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = gid >> 2, r = gid & 3;
    if (i >= n) return;  // the four lanes of a team leave together
    const int t = order[i];
    double* out = c.local + (size_t)t * (2 * (size_t)c.p + 2);
    double rho_t;
    const Frame ft = box_frame(c.cen, t, &rho_t);
    double acc[2 * PO + 2];
#pragma unroll
    for (int k = 0; k < 2 * PO + 2; ++k) acc[k] = 0.0;
    m2l_f64_class<PO, 0>(c, ft, rho_t, boff, bsrc, nbox, t, r, acc);
#pragma unroll
    for (int k = 0; k < 2 * PO + 2; ++k) {
        const double v = quad_sum(acc[k]);
        if ((k & 3) == r) out[k] = v;
    }
}

void fmm_m2l_f64_classes(const FmmCtx& c, const int* order, int n, const int* boff, const int* bsrc, int nbox,
                         hipStream_t s) {
    if (n <= 0) return;
    const unsigned g = nblk(4 * (int64_t)n, 128);
    switch (c.p) {
#define C_(PO) case PO: k_m2l_team_f64_classes<PO><<<g, 128, 0, s>>>(c, order, n, boff, bsrc, nbox); break;
        C_(5) C_(6) C_(7) C_(8) C_(9) C_(10) C_(11) C_(12) C_(13) C_(14)
        C_(15) C_(16) C_(17) C_(18) C_(19) C_(20) C_(21) C_(22) C_(23) C_(24)
#undef C_
        default: throw Error(ST_INTERNAL, "record order outside the per-pair order M2L instances");
    }
    SFMM_LAUNCH_CHECK();
}

// Lemma 4: every box of one level takes its parent's local expansion
template <int P>
__global__ void __launch_bounds__(128) k_l2l(FmmCtx c, int b0, int nb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int b = b0 + i;
    const int par = c.parent[b];
    double rho_t, rho_s;
    const Frame ft = box_frame(c.cen, b, &rho_t);
    const Frame fs = box_frame(c.cen, par, &rho_s);
    double* loc = c.local + (size_t)b * (2 * P + 2);
    double acc[2 * P + 2];
#pragma unroll
    for (int k = 0; k < 2 * P + 2; ++k) acc[k] = loc[k];
    const TransGeom G = trans_geom<kL2L>(fs, rho_s, ft, rho_t);
    translate_add<P>(c.local + (size_t)par * (2 * P + 2), G, acc);
#pragma unroll
    for (int k = 0; k < 2 * P + 2; ++k) loc[k] = acc[k];
}

// Local expansion at each target (sorted by leaf); writes psi and alpha in
// the caller's target order
template <int P>
__global__ void __launch_bounds__(128) k_l2p(FmmCtx c, const double* tx, const double* ty, const double* tz,
                                            const int* tleaf, const uint32_t* tperm, int64_t m, double psi_shift,
                                            double* psi, double* defl, int64_t m_out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int L = tleaf[i];
    double rho;
    const Frame f = box_frame(c.cen, L, &rho);
    double p, ax, ay, az;
    l2p_eval<P>(c.local + (size_t)L * (2 * P + 2), f, rho, tx[i], ty[i], tz[i], &p, &ax, &ay, &az);
    const int64_t o = tperm[i];
    psi[o] = p + psi_shift;
    defl[o] = ax;
    defl[m_out + o] = ay;
    defl[2 * m_out + o] = az;
}

// k_l2p that also writes the local expansion's Hessian (Sec. 2.2) to hess
// [3][m_out] (H_tt, H_tp, H_pp in the target's e_theta, e_phi)
template <int P>
__global__ void __launch_bounds__(128) k_l2p_hess(FmmCtx c, const double* tx, const double* ty, const double* tz,
                                                 const int* tleaf, const uint32_t* tperm, int64_t m,
                                                 double psi_shift, double* psi, double* defl, double* hess,
                                                 int64_t m_out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int L = tleaf[i];
    double rho;
    const Frame f = box_frame(c.cen, L, &rho);
    const double nx = tx[i], ny = ty[i], nz = tz[i];
    double et[3], ep[3];
    target_basis(nx, ny, nz, et, ep);
    double p, ax, ay, az, h[3];
    l2p_eval_hess<P>(c.local + (size_t)L * (2 * P + 2), f, rho, nx, ny, nz, et, ep, &p, &ax, &ay, &az, h);
    const int64_t o = tperm[i];
    psi[o] = p + psi_shift;
    defl[o] = ax;
    defl[m_out + o] = ay;
    defl[2 * m_out + o] = az;
    hess[o] = h[0];
    hess[m_out + o] = h[1];
    hess[2 * m_out + o] = h[2];
}

void fmm_p2m(const FmmCtx& c, int nb, hipStream_t s) {
    if (nb <= 0) return;
#define L_(P) case P: k_p2m<P><<<nblk(nb, 128), 128, 0, s>>>(c, nb); break;
    SFMM_DISPATCH(c.p, L_)
#undef L_
    SFMM_LAUNCH_CHECK();
}

void fmm_m2m(const FmmCtx& c, int b0, int nb, hipStream_t s) {
    if (nb <= 0) return;
#define L_(P) case P: k_m2m<P><<<nblk(4 * (int64_t)nb, 128), 128, 0, s>>>(c, b0, nb); break;
    SFMM_DISPATCH(c.p, L_)
#undef L_
    SFMM_LAUNCH_CHECK();
}

void fmm_m2l(const FmmCtx& c, int p, bool acc_in, const int* order, int n, const int* off, const int* src,
             hipStream_t s) {
    if (n <= 0) return;
    if (p < 1 || p > c.p) throw Error(ST_INTERNAL, "M2L order above the record order");
    if (m2l_team_width(n) == 2) {
#define L_(P) case P: k_m2l_team2<P><<<nblk(2 * (int64_t)n, 128), 128, 0, s>>>(c, order, n, off, src, acc_in); break;
        SFMM_DISPATCH(p, L_)
#undef L_
    } else {
#define L_(P) case P: k_m2l_team<P><<<nblk(4 * (int64_t)n, 128), 128, 0, s>>>(c, order, n, off, src, acc_in); break;
        SFMM_DISPATCH(p, L_)
#undef L_
    }
    SFMM_LAUNCH_CHECK();
}

void mult_to_f32(const FmmCtx& c, int nbox, float* multf, hipStream_t s) {
    if (nbox <= 0) return;
    k_mult_to_f32<<<nblk((int64_t)nbox * 2 * c.p, 256), 256, 0, s>>>(c.mult, c.p, nbox, multf);
    SFMM_LAUNCH_CHECK();
}

void fmm_m2l_f32(const FmmCtx& c, int p, bool acc_in, const float* multf, const int* order, int n, const int* off,
                 const int* src, hipStream_t s) {
    if (n <= 0) return;
    if (p < 1 || p > c.p) throw Error(ST_INTERNAL, "M2L order above the record order");
#define L_(P)                                                                                                  \
    case P:                                                                                                    \
        k_m2l_team_f32<P><<<nblk(kM2LTeamF32 * (int64_t)n, 128), 128, 0, s>>>(c, multf, order, n, off, src, acc_in);   \
        break;
    SFMM_DISPATCH(p, L_)
#undef L_
    SFMM_LAUNCH_CHECK();
}

bool m2l_f32_tail_supported(int p) { return p >= 5 && p <= 24; }


void fmm_l2l(const FmmCtx& c, int b0, int nb, hipStream_t s) {
    if (nb <= 0) return;
#define L_(P) case P: k_l2l<P><<<nblk(nb, 128), 128, 0, s>>>(c, b0, nb); break;
    SFMM_DISPATCH(c.p, L_)
#undef L_
    SFMM_LAUNCH_CHECK();
}

void fmm_l2p(const FmmCtx& c, const double* tx, const double* ty, const double* tz, const int* tleaf,
             const uint32_t* tperm, int64_t m, double psi_shift, double* psi, double* defl, int64_t m_out,
             hipStream_t s, double* hess) {
    if (m <= 0) return;
#define L_(P)                                                                                         \
    case P:                                                                                           \
        if (hess)                                                                                     \
            k_l2p_hess<P><<<nblk(m, 128), 128, 0, s>>>(c, tx, ty, tz, tleaf, tperm, m, psi_shift, psi, \
                                                       defl, hess, m_out);                            \
        else                                                                                          \
            k_l2p<P><<<nblk(m, 128), 128, 0, s>>>(c, tx, ty, tz, tleaf, tperm, m, psi_shift, psi, defl, \
                                                  m_out);                                             \
        break;
    SFMM_DISPATCH(c.p, L_)
#undef L_
    SFMM_LAUNCH_CHECK();
}

// Convergence, shear and magnification from the Hessian (Eq. GAM_DEF and
// the magnification of Sec. 2.2): out [4][m] = (kappa - kappa_bar, gamma_1,
// gamma_2, mu) from hess [3][m] = (H_11, H_12, H_22).
__global__ void k_lensing(const double* __restrict__ hess, int64_t m, double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double h11 = hess[i], h12 = hess[m + i], h22 = hess[2 * m + i];
    const double kk = h11 + h22, g1 = 0.5 * (h11 - h22), g2 = h12;
    const double a = 1.0 - 0.5 * kk;
    out[i] = kk;
    out[m + i] = g1;
    out[2 * m + i] = g2;
    out[3 * m + i] = 1.0 / (a * a - g1 * g1 - g2 * g2);
}

void lensing_from_hessian(const double* hess, int64_t m, double* out, hipStream_t s) {
    if (m <= 0) return;
    k_lensing<<<nblk(m, 256), 256, 0, s>>>(hess, m, out);
    SFMM_LAUNCH_CHECK();
}

}  // namespace sfmm
