// Near field (the direct acts of Sec. 3.3-3.4): for every target in a leaf T,
// the sum of the Green's function and its tangent gradient over the particles
// of T's close leaves.
//
// At planning time each direct-act list is split in two (near_split):
//   * a close leaf S whose centre is more than R_S / x from every target of
//     T (and that holds enough particles for it to pay) is taken through its
//     own multipole expansion (Lemma 1) at each target: k_m2p.  By Eq.
//     MUL_ERR the truncation there is below (Q~/2pi) x^(p+1)/((p+1)(1-x));
//     x is at most 1/3 and makes x^(p+1) at most 1e-4 times the tolerance of
//     order p (m2p_ratio).  The split is only made for p >= 12 and for leaves
//     with at least p/4 + 2 particles.  Big leaves of sparse regions next to
//     dense clumps are where it matters: their targets otherwise meet every
//     particle of the clump directly.
//   * every other close leaf is summed particle by particle: k_p2p.
//
// k_p2p: one 64-wide wavefront (a 64-thread workgroup) owns one target leaf
// and takes its targets in groups of ng <= 64.  The lanes form ng teams of
// L = floor(64 / ng) lanes, team t owning target t of the group.  The close
// leaves' particle ranges are concatenated into one flat index space (wave
// prefix sum of their counts); each tile of 128 particles is decoded once
// (binary search by lane shuffles) and staged in LDS, and lane r of a team
// takes particles r, r + L, ... of the tile.  The four partial sums stay in
// registers across all tiles; at the end of the group the team's lanes are
// summed in a fixed order through LDS.  No floating-point atomics: the
// result is bitwise reproducible.
//
// Load balance: a leaf of a sparse region next to a dense clump can have
// thousands of close leaves (every clump leaf fails the MAC against a big
// leaf).  Each leaf's two lists are cut into segments of at most kSegNear /
// kSegFar entries; a workgroup takes one (leaf, segment) item, items are
// launched heaviest first, and a leaf cut into several segments writes its
// per-segment results to a partial buffer that k_near_reduce adds up in
// segment order (so the result stays bitwise reproducible).
//
// Per pair, with d = n_t - n_s, psi gets (q/4pi)(log(|d|^2/4) + 1) (Eq.
// GRE_FUN plus the zero-mean share) and alpha gets (q/2pi) d/|d|^2, projected
// on the tangent plane once per target.  A particle at exactly the target
// position keeps only its q/(4pi).  Per target only four sums are kept:
//   S = sum q log|d|^2   (log 4 in place of the log for a coincident particle)
//   V = sum q d/|d|^2    (d = 0 there, so nothing is added)
// and with Q_near = sum q over the summed leaves (from their Lemma 1 Q),
//   4 pi psi_near = S + (1 - log 4) Q_near.
#include "common.hpp"
#include <algorithm>
#include <cmath>
#include <type_traits>
#include "expand.hpp"

namespace sfmm {

constexpr int kTile = 128;  // particles staged in LDS per tile

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kM2PMinOrder = 12;
// A close leaf S is evaluated through its Lemma 1 expansion at the targets
// of T when every target is beyond ratio R_S from its centre, ratio = 1 / x
// with the truncation term x^(p+1) at most 1e-4 tau_p (tau_p: the tolerance
// that gives order p by the order policy, 4 times its calibrated error), and
// at least 3: ratio 3 down to p = 21, 3.2 at p = 18, 4.2 at p = 12.  And when S holds at
// least p/4 + 2 particles (measured at p = 36: lower ratios or a higher count
// move more work than they save).
double m2p_ratio(int p) {
    const double tau = 4.0 * order_calibrated_error(p);
    const double x = std::min(1.0 / 3.0, std::pow(1e-4 * tau, 1.0 / (p + 1)));
    return 1.0 / x;
}
int m2p_min_count(int p) { return (p + 8 + 3) / 4; }  // ceil(p/4 + 2)

// ------------------------------------------------------------ list split
// Target box of every direct-act entry: the last box whose list starts at
// or before it (empty boxes share their start with the next one)
__global__ void k_entry_box(const int* __restrict__ off, int nbox, int np, int* __restrict__ ent_t) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    int lo = 0, hi = nbox - 1;  // off[lo] <= k always holds (off[0] = 0)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    ent_t[k] = lo;
}

// flag[k] = 1 when entry k goes to the direct sum, 2 when it goes to the
// multipole evaluation, 0 when its target box holds no target; bnear / bfar
// count each block's entries of the two kinds.
constexpr int kNearBlk = 256;
__global__ void __launch_bounds__(kNearBlk) k_near_flags(FmmCtx c, const int* __restrict__ ent_t,
                                                         const int* __restrict__ src, int np,
                                                         const int* __restrict__ tfirst,
                                                         const int* __restrict__ tcount,
                                                         const double* __restrict__ tx,
                                                         const double* __restrict__ ty,
                                                         const double* __restrict__ tz, double ratio, int min_count,
                                                         uint8_t* __restrict__ flag, int* __restrict__ bnear,
                                                         int* __restrict__ bfar) {
    __shared__ int wn[kNearBlk / 64], wf[kNearBlk / 64];
    const int k = blockIdx.x * kNearBlk + threadIdx.x;
    bool is_near = false, is_far = false;
    if (k < np) {
        const int T = ent_t[k], S = src[k];
        const int nt = tcount[T];
        if (nt > 0 && c.p >= kM2PMinOrder && c.count[S] >= min_count) {
            // beyond every particle's profile too (near-particle model)
            const double a = fmax(ratio * c.rad[S], c.rad[S] + c.npm_sigma);
            if (a < 3.0) {
                const double* cs = c.cen + 4 * (size_t)S;
                const double* ct = c.cen + 4 * (size_t)T;
                // whole box T beyond a + R_T (every point of a box lies within R of its centre)
                const double b = a + c.rad[T];
                const double ex = cs[0] - ct[0], ey = cs[1] - ct[1], ez = cs[2] - ct[2];
                const double d2 = ex * ex + ey * ey + ez * ez;
                const double hb = 2.0 * sin(0.5 * b);
                if (b < 3.0 && d2 > hb * hb * (1.0 + 1e-12)) {
                    is_far = true;
                } else {
                    const double h = 2.0 * sin(0.5 * a);
                    const double thr = h * h;
                    is_far = true;
                    const int t0 = tfirst[T];
                    for (int i = t0; i < t0 + nt; ++i) {
                        const double dx = tx[i] - cs[0], dy = ty[i] - cs[1], dz = tz[i] - cs[2];
                        if (!(dx * dx + dy * dy + dz * dz > thr)) {
                            is_far = false;
                            break;
                        }
                    }
                }
            }
        }
        is_near = nt > 0 && !is_far;
        flag[k] = (uint8_t)((is_near ? 1 : 0) | (is_far ? 2 : 0));
    }
    const uint64_t mn = __ballot(is_near), mf = __ballot(is_far);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        wn[wave] = __popcll(mn);
        wf[wave] = __popcll(mf);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int sn = 0, sf = 0;
        for (int w = 0; w < kNearBlk / 64; ++w) {
            sn += wn[w];
            sf += wf[w];
        }
        bnear[blockIdx.x] = sn;
        bfar[blockIdx.x] = sf;
    }
}

// Entry k's place in the near and far lists: its block's base (scan of the
// block counts) plus the entries of its kind before it in the block.  The
// first entry of each target box also records the two places, which become
// the box's CSR offsets.
__global__ void __launch_bounds__(kNearBlk) k_near_scatter(const int* __restrict__ src,
                                                           const int* __restrict__ ent_t, int np,
                                                           const uint8_t* __restrict__ flag,
                                                           const int* __restrict__ bnoff,
                                                           const int* __restrict__ bfoff, int* __restrict__ near_src,
                                                           int* __restrict__ far_src, int* __restrict__ first_near,
                                                           int* __restrict__ first_far) {
    __shared__ int wn[kNearBlk / 64], wf[kNearBlk / 64];
    const int k = blockIdx.x * kNearBlk + threadIdx.x;
    const int f = k < np ? flag[k] : 0;
    const uint64_t mn = __ballot(f & 1), mf = __ballot(f & 2);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        wn[wave] = __popcll(mn);
        wf[wave] = __popcll(mf);
    }
    __syncthreads();
    if (k >= np) return;
    int pn = bnoff[blockIdx.x], pf = bfoff[blockIdx.x];
    for (int w = 0; w < wave; ++w) {
        pn += wn[w];
        pf += wf[w];
    }
    const uint64_t lt = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    pn += __popcll(mn & lt);
    pf += __popcll(mf & lt);
    if (f & 1) near_src[pn] = src[k];
    if (f & 2) far_src[pf] = src[k];
    const int T = ent_t[k];
    if (k == 0 || ent_t[k - 1] != T) {
        first_near[T] = pn;
        first_far[T] = pf;
    }
}

// CSR offsets of the two lists: box b starts where the entry off[b] of the
// full list (the first entry of the first non-empty box >= b) would land.
__global__ void k_near_offsets(const int* __restrict__ off, const int* __restrict__ ent_t, int nbox, int np,
                               const int* __restrict__ first_near, const int* __restrict__ ntot,
                               const int* __restrict__ first_far, const int* __restrict__ ftot,
                               int* __restrict__ near_off, int* __restrict__ far_off) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nbox) return;
    const int k = off[b];
    near_off[b] = k < np ? first_near[ent_t[k]] : *ntot;
    far_off[b] = k < np ? first_far[ent_t[k]] : *ftot;
}

// Work of each box: pairs[T] = tcount[T] * (particles of the near leaves),
// evals[T] = tcount[T] * (far leaves)
__global__ void k_near_work(const int* __restrict__ count, const int* __restrict__ near_off,
                            const int* __restrict__ near_src, const int* __restrict__ far_off,
                            const int* __restrict__ tcount, int nbox, long long* __restrict__ pairs,
                            long long* __restrict__ evals) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    long long ns = 0;
    for (int k = near_off[b]; k < near_off[b + 1]; ++k) ns += count[near_src[k]];
    pairs[b] = ns * (long long)tcount[b];
    evals[b] = (long long)(far_off[b + 1] - far_off[b]) * (long long)tcount[b];
}

void entry_box(const int* off, int nbox, int np, int* ent_t, hipStream_t s) {
    if (np <= 0 || nbox <= 0) return;
    k_entry_box<<<nblk(np, 256), 256, 0, s>>>(off, nbox, np, ent_t);
    SFMM_LAUNCH_CHECK();
}

void near_split(const FmmCtx& c, const int* off, const int* src, const int* ent_t, int nbox, int np,
                const int* tfirst, const int* tcount, const double* tx, const double* ty, const double* tz,
                NearLists& out, hipStream_t s) {
    out.near_off.resize(nbox + 1);
    out.far_off.resize(nbox + 1);
    // every entry goes to at most one of the two lists, so np bounds both:
    // no read-back of the totals (which stay on the device for the offsets)
    out.near_src.resize(std::max(np, 1));
    out.far_src.resize(std::max(np, 1));
    if (nbox <= 0) return;
    const int nb = std::max((np + kNearBlk - 1) / kNearBlk, 1);
    DVec<uint8_t> flag;
    DVec<int> bnear, bfar, bnoff, bfoff, first_near, first_far, tot;
    flag.resize(std::max(np, 1));
    bnear.resize(nb);
    bfar.resize(nb);
    bnoff.resize(nb);
    bfoff.resize(nb);
    first_near.resize(nbox);
    first_far.resize(nbox);
    tot.resize(2);
    fill_i32(tot.data(), 2, 0, s);
    if (np > 0) {
        k_near_flags<<<nb, kNearBlk, 0, s>>>(c, ent_t, src, np, tfirst, tcount, tx, ty, tz, m2p_ratio(c.p),
                                             m2p_min_count(c.p), flag.data(), bnear.data(), bfar.data());
        SFMM_LAUNCH_CHECK();
        scan_excl_i32(bnear.data(), bnoff.data(), nb, tot.data(), s);
        scan_excl_i32(bfar.data(), bfoff.data(), nb, tot.data() + 1, s);
    }
    if (np > 0) {
        k_near_scatter<<<nb, kNearBlk, 0, s>>>(src, ent_t, np, flag.data(), bnoff.data(), bfoff.data(),
                                               out.near_src.data(), out.far_src.data(), first_near.data(),
                                               first_far.data());
        SFMM_LAUNCH_CHECK();
    }
    k_near_offsets<<<nblk(nbox + 1, 256), 256, 0, s>>>(off, ent_t, nbox, np, first_near.data(), tot.data(),
                                                       first_far.data(), tot.data() + 1, out.near_off.data(),
                                                       out.far_off.data());
    SFMM_LAUNCH_CHECK();
}

void near_work(const int* count, const NearLists& nl, const int* tcount, int nbox, long long* pairs,
               long long* evals, hipStream_t s) {
    if (nbox <= 0) return;
    k_near_work<<<nblk(nbox, 256), 256, 0, s>>>(count, nl.near_off.data(), nl.near_src.data(), nl.far_off.data(),
                                                tcount, nbox, pairs, evals);
    SFMM_LAUNCH_CHECK();
}

// ------------------------------------------------------------ work items
// Per box b with targets and a non-empty list: nseg = ceil(K / seg) items;
// boxes cut into several items get nseg * tcount partial slots.
__global__ void k_seg_count(const int* __restrict__ off, const int* __restrict__ tcount, int nbox, int seg,
                            int* __restrict__ nseg, int* __restrict__ nslot, int* __restrict__ multi) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    const int K = off[b + 1] - off[b];
    const int ns = (tcount[b] > 0 && K > 0) ? (K + seg - 1) / seg : 0;
    nseg[b] = ns;
    nslot[b] = ns > 1 ? ns * tcount[b] : 0;
    multi[b] = ns > 1 ? 1 : 0;
}

// Items (box, first entry, end entry, partial slot base or -1) and the
// reduce records (box, nseg, base) of the boxes cut into several segments
__global__ void k_seg_emit(const int* __restrict__ off, const int* __restrict__ tcount, int nbox, int seg,
                           const int* __restrict__ nseg, const int* __restrict__ item_off,
                           const int* __restrict__ slot_off, const int* __restrict__ red_off,
                           int4* __restrict__ items, int4* __restrict__ red) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    const int ns = nseg[b];
    if (ns == 0) return;
    const int nt = tcount[b];
    for (int sg = 0; sg < ns; ++sg) {
        const int kb = off[b] + sg * seg, ke = min(kb + seg, off[b + 1]);
        items[item_off[b] + sg] = make_int4(b, kb, ke, ns > 1 ? slot_off[b] + sg * nt : -1);
    }
    if (ns > 1) red[red_off[b]] = make_int4(b, ns, slot_off[b], 0);
}

// Sort key of each item: leading zeros of its work, targets x particles (or
// targets x entries when count is null); heaviest power-of-two bucket first
// (one wave per item: its lanes sum the particle counts of the segment)
__global__ void k_item_keys(const int4* __restrict__ items, int n, const int* __restrict__ src,
                            const int* __restrict__ count, const int* __restrict__ tcount,
                            uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int i = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;  // uniform across the wave
    const int4 it = items[i];
    long long w = 0;
    if (count) {
        long long part = 0;
        for (int k = it.y + lane; k < it.z; k += 64) part += count[src[k]];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        w = part;
    } else {
        w = it.z - it.y;
    }
    if (lane != 0) return;
    w *= tcount[it.x];
    keys[i] = (w > 0) ? (uint64_t)__clzll((unsigned long long)w) : 255ULL;
    vals[i] = (uint32_t)i;
}

__global__ void k_gather_items(const int4* __restrict__ in, const uint32_t* __restrict__ idx, int n,
                               int4* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[idx[i]];
}

namespace {
// The two halves of building one list's work items around the read-back of
// its three totals (items, partial slots, reduce records), so that two lists
// can share one read-back.
struct ItemCounts {
    DVec<int> nseg, nslot, multi, item_off, slot_off, red_off;
};

void items_count(const int* off, const int* tcount, int nbox, int seg, ItemCounts& t, int* tot, hipStream_t s) {
    t.nseg.resize(nbox);
    t.nslot.resize(nbox);
    t.multi.resize(nbox);
    t.item_off.resize(nbox);
    t.slot_off.resize(nbox);
    t.red_off.resize(nbox);
    k_seg_count<<<nblk(nbox, 256), 256, 0, s>>>(off, tcount, nbox, seg, t.nseg.data(), t.nslot.data(),
                                                t.multi.data());
    SFMM_LAUNCH_CHECK();
    scan3_excl_i32(t.nseg.data(), t.nslot.data(), t.multi.data(), t.item_off.data(), t.slot_off.data(),
                   t.red_off.data(), nbox, tot, s);
}

void items_emit(const int* off, const int* src, const int* count, const int* tcount, int nbox, int seg,
                const ItemCounts& t, const int* h, WorkItems& out, hipStream_t s) {
    out.n = h[0];
    out.nslot = h[1];
    out.nred = h[2];
    out.items.resize(std::max(out.n, 1));
    out.red.resize(std::max(out.nred, 1));
    out.part.resize(4 * (size_t)std::max(out.nslot, 1));
    if (out.n == 0) return;
    DVec<int4> raw;
    DVec<uint64_t> keys;
    DVec<uint32_t> vals;
    raw.resize(out.n);
    keys.resize(out.n);
    vals.resize(out.n);
    k_seg_emit<<<nblk(nbox, 256), 256, 0, s>>>(off, tcount, nbox, seg, t.nseg.data(), t.item_off.data(),
                                               t.slot_off.data(), t.red_off.data(), raw.data(), out.red.data());
    SFMM_LAUNCH_CHECK();
    k_item_keys<<<nblk(64 * (int64_t)out.n, 256), 256, 0, s>>>(raw.data(), out.n, src, count, tcount, keys.data(),
                                                             vals.data());
    SFMM_LAUNCH_CHECK();
    radix_sort_u64(keys.data(), vals.data(), out.n, 8, s);
    k_gather_items<<<nblk(out.n, 256), 256, 0, s>>>(raw.data(), vals.data(), out.n, out.items.data());
    SFMM_LAUNCH_CHECK();
}
}  // namespace

void build_items2(const int* off_a, const int* src_a, const int* count_a, int seg_a, WorkItems& out_a,
                  const int* off_b, const int* src_b, const int* count_b, int seg_b, WorkItems& out_b,
                  const int* tcount, int nbox, hipStream_t s) {
    out_a.n = out_a.nred = out_a.nslot = 0;
    out_b.n = out_b.nred = out_b.nslot = 0;
    if (nbox <= 0) return;
    ItemCounts ta, tb;
    DVec<int> tot;
    tot.resize(6);
    items_count(off_a, tcount, nbox, seg_a, ta, tot.data(), s);
    items_count(off_b, tcount, nbox, seg_b, tb, tot.data() + 3, s);
    int h[6];
    SFMM_HIP(hipMemcpyAsync(h, tot.data(), sizeof(h), hipMemcpyDeviceToHost, s));
    SFMM_HIP(hipStreamSynchronize(s));
    items_emit(off_a, src_a, count_a, tcount, nbox, seg_a, ta, h, out_a, s);
    items_emit(off_b, src_b, count_b, tcount, nbox, seg_b, tb, h + 3, out_b, s);
}

// Adds the per-segment results of every box cut into several items, in
// segment order: one workgroup per box, lanes over its targets.
template <bool HESS>
__global__ void __launch_bounds__(64) k_near_reduce(const int4* __restrict__ red, const int* __restrict__ tfirst,
                                                   const int* __restrict__ tcount,
                                                   const uint32_t* __restrict__ tperm,
                                                   const double* __restrict__ part, double* __restrict__ psi,
                                                   double* __restrict__ defl, double* __restrict__ hess,
                                                   int64_t m_out) {
    constexpr int NV = HESS ? 7 : 4, ST = HESS ? 8 : 4;
    const int4 r = red[blockIdx.x];
    const int T = r.x, ns = r.y, base = r.z;
    const int t0 = tfirst[T], nt = tcount[T];
    for (int t = threadIdx.x; t < nt; t += 64) {
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = 0.0;
        for (int sg = 0; sg < ns; ++sg) {
            const double* q = part + ST * ((size_t)base + (size_t)sg * nt + t);
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] += q[k];
        }
        const int64_t o = tperm[t0 + t];
        psi[o] += v[0];
        defl[o] += v[1];
        defl[m_out + o] += v[2];
        defl[2 * m_out + o] += v[3];
        if constexpr (HESS) {
            hess[o] += v[4];
            hess[m_out + o] += v[5];
            hess[2 * m_out + o] += v[6];
        }
    }
}

// psi and alpha contributions of one target: straight to the outputs, or to
// its slot of the partial buffer
__device__ __forceinline__ void emit_target(int slot, int64_t o, double ps, double a0, double a1, double a2,
                                            double* __restrict__ part, double* __restrict__ psi,
                                            double* __restrict__ defl, int64_t m_out) {
    if (slot < 0) {
        psi[o] += ps;
        defl[o] += a0;
        defl[m_out + o] += a1;
        defl[2 * m_out + o] += a2;
    } else {
        double* q = part + 4 * (size_t)slot;
        q[0] = ps;
        q[1] = a0;
        q[2] = a1;
        q[3] = a2;
    }
}

// the same with the Hessian h[3] (slots of 8 doubles)
__device__ __forceinline__ void emit_target_hess(int slot, int64_t o, double ps, double a0, double a1, double a2,
                                                 const double* h, double* __restrict__ part,
                                                 double* __restrict__ psi, double* __restrict__ defl,
                                                 double* __restrict__ hess, int64_t m_out) {
    if (slot < 0) {
        psi[o] += ps;
        defl[o] += a0;
        defl[m_out + o] += a1;
        defl[2 * m_out + o] += a2;
        hess[o] += h[0];
        hess[m_out + o] += h[1];
        hess[2 * m_out + o] += h[2];
    } else {
        double* q = part + 8 * (size_t)slot;
        q[0] = ps;
        q[1] = a0;
        q[2] = a1;
        q[3] = a2;
        q[4] = h[0];
        q[5] = h[1];
        q[6] = h[2];
    }
}

// ------------------------------------------------------------ direct sums
// Pair terms of one lane over one LDS tile.  FP64: coordinates as stored.
// FP32 (precision tier): every coordinate is a two-float pair hi + lo
// (hi = float(x), lo = float(x - hi)), so d = (t_hi - s_hi) + (t_lo - s_lo)
// keeps ~1e-7 relative accuracy for close points where plain FP32 positions
// would lose all digits of d; log and reciprocal are the hardware FP32
// instructions, and each tile's FP32 partial sums (at most 256 terms) are
// added to FP64 running sums.  The log terms, all of one sign, are summed
// with Kahan compensation; the deflection terms largely cancel and are not.
struct TileF64 {
    double4 p[kTile];
};
struct TileF32 {
    float4 hi[kTile];  // x, y, z, q
    float4 lo[kTile];  // x, y, z low parts
};

__device__ __forceinline__ void tile_store(TileF64& t, int k, double4 v) { t.p[k] = v; }
__device__ __forceinline__ void tile_store(TileF32& t, int k, double4 v) {
    const float xh = (float)v.x, yh = (float)v.y, zh = (float)v.z;
    t.hi[k] = make_float4(xh, yh, zh, (float)v.w);
    t.lo[k] = make_float4((float)(v.x - (double)xh), (float)(v.y - (double)yh), (float)(v.z - (double)zh), 0.0f);
}

// Near-particle model inside a profile (u = |d|^2/4 < t): log(4u) of the
// point mass is replaced by log(4t) - I(u/t) and the deflection weight q/|d|^2
// by (q/4)(2/t - v/t - 1)/(1 - u) (both finite at u = 0); see NpmK.
template <typename R>
__device__ __forceinline__ R npm_interior_log(R v, R t, R ln4t, int nterms) {
    // I(v) = sum_k t^k [(2 - t)(1 - v^(k+1))/(k+1) - (1 - v^(k+2))/(k+2)]
    R sum = 0, tk = 1, vk1 = v, vk2 = v * v;
    for (int k = 0; k < nterms; ++k) {
        sum += tk * ((2 - t) * (1 - vk1) / (R)(k + 1) - (1 - vk2) / (R)(k + 2));
        tk *= t;
        vk1 *= v;
        vk2 *= v;
    }
    return ln4t - sum;
}

template <bool NPM>
__device__ __forceinline__ void tile_pairs(const TileF64& t, const double2* ltab, const LogPoly& lk, const NpmK& nk,
                                           int r, int L, int tn, double ax, double ay, double az, double& p0,
                                           double& p1, double& p2, double& p3) {
    for (int j = r; j < tn; j += L) {
        const double4 sp = t.p[j];
        const double dx = ax - sp.x, dy = ay - sp.y, dz = az - sp.z;
        // |d|^2 of two distinct unit vectors is >= ~1e-32: zero only for
        // coincident points, which take |d|^2 = 4 instead (log 4, and d = 0
        // zeroes their deflection): both have a zero low word, so only the
        // high word is switched (no branch: every lane takes the same path)
        const double d2r = dx * dx + dy * dy + dz * dz;
        const double d2 = __hiloint2double(d2r == 0.0 ? 0x40100000 : __double2hiint(d2r), __double2loint(d2r));
        double lg, i0;
        log_recip_tab(d2, ltab, lk, &lg, &i0);
        double wi = sp.w * i0;
        if constexpr (NPM) {
            if (d2r < nk.four_t) {
                const double u = 0.25 * d2r, v = u * nk.inv_t;
                lg = npm_interior_log(v, nk.t, nk.ln4t, nk.nterms);
                wi = sp.w * 0.25 * (2.0 * nk.inv_t - v * nk.inv_t - 1.0) / (1.0 - u);
            }
        }
        p0 = fma(sp.w, lg, p0);
        p1 = fma(wi, dx, p1);
        p2 = fma(wi, dy, p2);
        p3 = fma(wi, dz, p3);
    }
}

template <bool NPM>
__device__ __forceinline__ void tile_pairs(const TileF32& t, const double2*, const LogPoly&, const NpmK& nk, int r,
                                           int L, int tn, double ax, double ay, double az, double& p0, double& p1,
                                           double& p2, double& p3) {
    const float axh = (float)ax, ayh = (float)ay, azh = (float)az;
    const float axl = (float)(ax - (double)axh), ayl = (float)(ay - (double)ayh), azl = (float)(az - (double)azh);
    constexpr float kLn2f = 0.693147180559945309f, kLog4f = 1.38629436111989061f;
    float f0 = 0.0f, c0 = 0.0f, f1 = 0.0f, f2 = 0.0f, f3 = 0.0f;
    for (int j = r; j < tn; j += L) {
        const float4 h = t.hi[j], l = t.lo[j];
        const float dx = (axh - h.x) + (axl - l.x);
        const float dy = (ayh - h.y) + (ayl - l.y);
        const float dz = (azh - h.z) + (azl - l.z);
        const float d2 = dx * dx + dy * dy + dz * dz;
        const bool coinc = d2 == 0.0f;
        const float r2 = coinc ? 1.0f : d2;
        float lg = coinc ? kLog4f : __builtin_amdgcn_logf(r2) * kLn2f;
        float wi = h.w * __builtin_amdgcn_rcpf(r2);
        if constexpr (NPM) {
            if (d2 < (float)nk.four_t) {
                const float u = 0.25f * d2, v = u * (float)nk.inv_t;
                lg = npm_interior_log(v, (float)nk.t, (float)nk.ln4t, nk.nterms);
                wi = h.w * 0.25f * (2.0f * (float)nk.inv_t - v * (float)nk.inv_t - 1.0f) / (1.0f - u);
            }
        }
        // the log terms all have one sign and grow the sum to ~100 times
        // each: Kahan-compensated (c0 carries the lost low part)
        const float y = fmaf(h.w, lg, -c0);
        const float tt = f0 + y;
        c0 = (tt - f0) - y;
        f0 = tt;
        f1 = fmaf(wi, dx, f1);
        f2 = fmaf(wi, dy, f2);
        f3 = fmaf(wi, dz, f3);
    }
    p0 += (double)f0 - (double)c0;
    p1 += (double)f1;
    p2 += (double)f2;
    p3 += (double)f3;
}

// Pair terms with the Hessian of Sec. 2.2: per source, in the target's
// basis e_a, e_b (et, ep), H_ab = (q/2pi) [delta_ab (1 - n.d)/|d|^2 - 2 (e_a.d)
// (e_b.d)/|d|^4]; the lane sums hd = sum q (1 - n.d)/|d|^2 and h_ab = sum q
// (e_a.d)(e_b.d)/|d|^4 (coincident points add nothing).
template <bool NPM>
__device__ __forceinline__ void tile_pairs_hess(const TileF64& t, const double2* ltab, const LogPoly& lk,
                                                const NpmK& nk, int r, int L, int tn, double ax, double ay, double az,
                                                const double* et, const double* ep, double* acc) {
    for (int j = r; j < tn; j += L) {
        const double4 sp = t.p[j];
        const double dx = ax - sp.x, dy = ay - sp.y, dz = az - sp.z;
        const double d2r = dx * dx + dy * dy + dz * dz;
        const double d2 = __hiloint2double(d2r == 0.0 ? 0x40100000 : __double2hiint(d2r), __double2loint(d2r));
        double lg, i0;
        log_recip_tab(d2, ltab, lk, &lg, &i0);
        double wi = sp.w * i0;
        double wm = d2r == 0.0 ? 0.0 : wi;
        double w2 = wm * i0;
        if constexpr (NPM) {
            if (d2r < nk.four_t) {
                const double u = 0.25 * d2r, v = u * nk.inv_t, omu = 1.0 - u;
                lg = npm_interior_log(v, nk.t, nk.ln4t, nk.nterms);
                wi = sp.w * 0.25 * (2.0 * nk.inv_t - v * nk.inv_t - 1.0) / omu;
                wm = wi;
                w2 = sp.w * nk.a2 / (omu * omu);
            }
        }
        acc[0] = fma(sp.w, lg, acc[0]);
        acc[1] = fma(wi, dx, acc[1]);
        acc[2] = fma(wi, dy, acc[2]);
        acc[3] = fma(wi, dz, acc[3]);
        const double nd = ax * dx + ay * dy + az * dz;
        const double da = et[0] * dx + et[1] * dy + et[2] * dz;
        const double db = ep[0] * dx + ep[1] * dy + ep[2] * dz;
        acc[4] = fma(-nd, wm, acc[4] + wm);
        acc[5] = fma(w2 * da, da, acc[5]);
        acc[6] = fma(w2 * da, db, acc[6]);
        acc[7] = fma(w2 * db, db, acc[7]);
    }
}

template <bool NPM>
__device__ __forceinline__ void tile_pairs_hess(const TileF32& t, const double2*, const LogPoly&, const NpmK& nk,
                                                int r, int L, int tn, double ax, double ay, double az,
                                                const double* et, const double* ep, double* acc) {
    const float axh = (float)ax, ayh = (float)ay, azh = (float)az;
    const float axl = (float)(ax - (double)axh), ayl = (float)(ay - (double)ayh), azl = (float)(az - (double)azh);
    const float etf[3] = {(float)et[0], (float)et[1], (float)et[2]};
    const float epf[3] = {(float)ep[0], (float)ep[1], (float)ep[2]};
    constexpr float kLn2f = 0.693147180559945309f, kLog4f = 1.38629436111989061f;
    float f[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, c0 = 0.0f;
    for (int j = r; j < tn; j += L) {
        const float4 h = t.hi[j], l = t.lo[j];
        const float dx = (axh - h.x) + (axl - l.x);
        const float dy = (ayh - h.y) + (ayl - l.y);
        const float dz = (azh - h.z) + (azl - l.z);
        const float d2 = dx * dx + dy * dy + dz * dz;
        const bool coinc = d2 == 0.0f;
        const float r2 = coinc ? 1.0f : d2;
        float lg = coinc ? kLog4f : __builtin_amdgcn_logf(r2) * kLn2f;
        const float i0 = __builtin_amdgcn_rcpf(r2);
        float wi = h.w * i0;
        float wm = coinc ? 0.0f : wi;
        float w2 = wm * i0;
        if constexpr (NPM) {
            if (d2 < (float)nk.four_t) {
                const float u = 0.25f * d2, v = u * (float)nk.inv_t, omu = 1.0f - u;
                lg = npm_interior_log(v, (float)nk.t, (float)nk.ln4t, nk.nterms);
                wi = h.w * 0.25f * (2.0f * (float)nk.inv_t - v * (float)nk.inv_t - 1.0f) / omu;
                wm = wi;
                w2 = h.w * (float)nk.a2 / (omu * omu);
            }
        }
        const float y = fmaf(h.w, lg, -c0);  // Kahan-compensated log terms, as in tile_pairs
        const float tt = f[0] + y;
        c0 = (tt - f[0]) - y;
        f[0] = tt;
        f[1] = fmaf(wi, dx, f[1]);
        f[2] = fmaf(wi, dy, f[2]);
        f[3] = fmaf(wi, dz, f[3]);
        // 1 - n.d = 1 - |d|^2/2 for unit vectors (n.d = |d|^2 / 2)
        const float da = etf[0] * dx + etf[1] * dy + etf[2] * dz;
        const float db = epf[0] * dx + epf[1] * dy + epf[2] * dz;
        f[4] = fmaf(-0.5f * d2, wm, f[4] + wm);
        f[5] = fmaf(w2 * da, da, f[5]);
        f[6] = fmaf(w2 * da, db, f[6]);
        f[7] = fmaf(w2 * db, db, f[7]);
    }
    acc[0] += (double)f[0] - (double)c0;
#pragma unroll
    for (int k = 1; k < 8; ++k) acc[k] += (double)f[k];
}

template <class Tile, bool HESS, bool NPM>
__global__ void __launch_bounds__(64) k_p2p(FmmCtx c, const int4* __restrict__ items,
                                           const int* __restrict__ src, const int* __restrict__ tfirst,
                                           const int* __restrict__ tcount, const double* __restrict__ tx,
                                           const double* __restrict__ ty, const double* __restrict__ tz,
                                           const uint32_t* __restrict__ tperm, double* __restrict__ psi,
                                           double* __restrict__ defl, int64_t m_out, double* __restrict__ part,
                                           LogPoly lk, double* __restrict__ hess, NpmK nk) {
    // the tile and the end-of-group reduction share one LDS block (fewer
    // bytes per wave, more waves per CU)
    constexpr int NR = HESS ? 8 : 4;  // sums per lane: psi, alpha (and hd, h_tt, h_tp, h_pp)
    constexpr size_t kSm = sizeof(Tile) > NR * 64 * sizeof(double) ? sizeof(Tile) : NR * 64 * sizeof(double);
    __shared__ __align__(16) unsigned char sm[kSm];
    Tile& tile = *reinterpret_cast<Tile*>(sm);
    double(*red)[64] = reinterpret_cast<double(*)[64]>(sm);
    const int lane = threadIdx.x;
    // the FP64 pair loop's log table (made before the first tile's barrier)
    __shared__ double2 ltab[std::is_same<Tile, TileF64>::value ? kLogTab : 1];
    if constexpr (std::is_same<Tile, TileF64>::value) {
        for (int j = lane; j < kLogTab; j += 64) ltab[j] = log_tab_entry(j);
    }
    const int4 item = items[blockIdx.x];
    const int T = item.x;
    const int k0 = item.y, K = item.z - item.y;
    const int t0 = tfirst[T], nt = tcount[T];
    const int ew = 2 * c.p + 2;
    const double4* __restrict__ spt = c.spt;

    for (int tg = 0; tg < nt; tg += 64) {
        const int ng = min(64, nt - tg);
        const int g0 = t0 + tg;
        const int L = 64 / ng;  // lanes per target
        const int team = lane / L, r = lane - team * L;
        const bool active = team < ng;
        const int my = g0 + (active ? team : 0);
        const double ax = tx[my], ay = ty[my], az = tz[my];
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;  // S, V partials of this lane
        double qnear = 0.0;                              // lane partials of Q_near
        double hacc[HESS ? 8 : 1] = {};                  // HESS: psi, alpha, hd, h_ab partials
        double et[3], ep[3];
        if constexpr (HESS) target_basis(ax, ay, az, et, ep);
        for (int kc = 0; kc < K; kc += 64) {
            const int kk = min(64, K - kc);
            int cnt = 0, fst = 0;
            if (lane < kk) {
                const int S = src[k0 + kc + lane];
                cnt = c.count[S];
                fst = c.first[S];
                qnear += c.mult[(size_t)S * ew + 1] * (4.0 * M_PI);
            }
            // inclusive wave scan of the counts
            int incl = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            const int excl = (lane < kk) ? incl - cnt : 0x7fffffff;
            const int total = __shfl(incl, 63, 64);
            for (int s0 = 0; s0 < total; s0 += kTile) {
                const int tn = min(kTile, total - s0);
                __syncthreads();  // previous tile fully consumed
#pragma unroll
                for (int j = 0; j < kTile / 64; ++j) {
                    const int f = s0 + j * 64 + lane;
                    // entry e: the last one whose start is <= f
                    int e = 0;
#pragma unroll
                    for (int step = 32; step > 0; step >>= 1) {
                        const int cand = e + step;
                        const int v = __shfl(excl, cand, 64);
                        if (v <= f) e = cand;
                    }
                    const int base = __shfl(fst, e, 64) - __shfl(excl, e, 64);
                    if (f < total) {
                        const int i = base + f;
                        tile_store(tile, j * 64 + lane, spt[i]);
                    }
                }
                __syncthreads();
                if (active) {
                    if constexpr (HESS) tile_pairs_hess<NPM>(tile, ltab, lk, nk, r, L, tn, ax, ay, az, et, ep, hacc);
                    else tile_pairs<NPM>(tile, ltab, lk, nk, r, L, tn, ax, ay, az, p0, p1, p2, p3);
                }
            }
        }
        const double qn = wave_sum(qnear);
        if constexpr (HESS) {
            p0 = hacc[0];
            p1 = hacc[1];
            p2 = hacc[2];
            p3 = hacc[3];
        }
        __syncthreads();  // the last tile fully consumed before red overwrites it
        red[0][lane] = p0;
        red[1][lane] = p1;
        red[2][lane] = p2;
        red[3][lane] = p3;
        if constexpr (HESS) {
#pragma unroll
            for (int q = 4; q < 8; ++q) red[q][lane] = hacc[q];
        }
        __syncthreads();
        if (lane < ng) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            double sh[4] = {0.0, 0.0, 0.0, 0.0};
            for (int j = lane * L; j < lane * L + L; ++j) {
                s0 += red[0][j];
                s1 += red[1][j];
                s2 += red[2][j];
                s3 += red[3][j];
                if constexpr (HESS) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) sh[q] += red[4 + q][j];
                }
            }
            const int me = g0 + lane;
            const double mx = tx[me], myy = ty[me], mz = tz[me];
            const double il = 1.0 / sqrt(mx * mx + myy * myy + mz * mz);
            const double ux = mx * il, uy = myy * il, uz = mz * il;
            const double vr = ux * s1 + uy * s2 + uz * s3;
            if constexpr (HESS) {
                const double h[3] = {(sh[0] - 2.0 * sh[1]) * kInv2Pi, -2.0 * sh[2] * kInv2Pi,
                                     (sh[0] - 2.0 * sh[3]) * kInv2Pi};
                emit_target_hess(item.w < 0 ? -1 : item.w + tg + lane, tperm[me],
                                 (s0 + (1.0 - kLog4) * qn) * kInv4Pi, (s1 - ux * vr) * kInv2Pi,
                                 (s2 - uy * vr) * kInv2Pi, (s3 - uz * vr) * kInv2Pi, h, part, psi, defl, hess, m_out);
            } else {
                emit_target(item.w < 0 ? -1 : item.w + tg + lane, tperm[me], (s0 + (1.0 - kLog4) * qn) * kInv4Pi,
                            (s1 - ux * vr) * kInv2Pi, (s2 - uy * vr) * kInv2Pi, (s3 - uz * vr) * kInv2Pi, part, psi,
                            defl, m_out);
            }
        }
        __syncthreads();  // red is reused by the next group
    }
}

// ------------------------------------------------------------ multipole evaluations
// One 64-wide workgroup per target leaf with far entries, targets in groups
// of ng <= 64 and lanes in teams of L = floor(64 / ng) as in k_p2p.  The far
// leaves are taken kChunkF at a time: their expansion records and frames
// are loaded once into LDS (coalesced: each record is contiguous), then
// lane r of team t evaluates leaves r, r + L, ... of the chunk at target t.
// The team's partial sums are added in a fixed order at the end of the
// group.
constexpr int kChunkF = 16;

template <int P, bool HESS>
__global__ void __launch_bounds__(64) k_m2p(FmmCtx c, const int4* __restrict__ items,
                                           const int* __restrict__ src, const int* __restrict__ tfirst,
                                           const int* __restrict__ tcount, const double* __restrict__ tx,
                                           const double* __restrict__ ty, const double* __restrict__ tz,
                                           const uint32_t* __restrict__ tperm, double* __restrict__ psi,
                                           double* __restrict__ defl, int64_t m_out, double* __restrict__ part,
                                           double* __restrict__ hess) {
    constexpr int EW = 2 * P + 2;
    // the staged records double as the end-of-group reduction buffer
    static_assert(kChunkF * (2 * kM2PMinOrder + 2) >= 4 * 64, "reduction fits the record buffer");
    __shared__ __align__(16) double coef[kChunkF * EW];
    __shared__ double frm[kChunkF][10];  // c, e_theta, e_phi, rho
    double(*red)[64] = reinterpret_cast<double(*)[64]>(coef);
    __shared__ double redh[HESS ? 3 : 1][64];  // the Hessian's partials
    const int lane = threadIdx.x;
    const int4 item = items[blockIdx.x];
    const int T = item.x;
    const int k0 = item.y, K = item.z - item.y;
    const int t0 = tfirst[T], nt = tcount[T];
    for (int tg = 0; tg < nt; tg += 64) {
        const int ng = min(64, nt - tg);
        const int g0 = t0 + tg;
        const int L = 64 / ng;
        const int team = lane / L, r = lane - team * L;
        const bool active = team < ng;
        const int my = g0 + (active ? team : 0);
        const double nx = tx[my], ny = ty[my], nz = tz[my];
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
        double hs[3] = {0.0, 0.0, 0.0};
        double et[3], ep[3];
        if constexpr (HESS) target_basis(nx, ny, nz, et, ep);
        for (int kc = 0; kc < K; kc += kChunkF) {
            const int cf = min(kChunkF, K - kc);
            __syncthreads();  // previous chunk fully consumed
            // records are EW = 2P + 2 doubles (16-byte aligned): copied as
            // double2, P + 1 per record
#pragma unroll 4
            for (int idx = lane; idx < cf * (P + 1); idx += 64) {
                const int f = idx / (P + 1), e = idx - f * (P + 1);
                reinterpret_cast<double2*>(coef)[idx] =
                    reinterpret_cast<const double2*>(c.mult + (size_t)src[k0 + kc + f] * EW)[e];
            }
            if (lane < cf) {
                const double* cs = c.cen + 4 * (size_t)src[k0 + kc + lane];
                const Frame fr = make_frame(cs[0], cs[1], cs[2]);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    frm[lane][d] = fr.c[d];
                    frm[lane][3 + d] = fr.et[d];
                    frm[lane][6 + d] = fr.ep[d];
                }
                frm[lane][9] = cs[3];
            }
            __syncthreads();
            if (active) {
                for (int j = r; j < cf; j += L) {
                    Frame fr;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        fr.c[d] = frm[j][d];
                        fr.et[d] = frm[j][3 + d];
                        fr.ep[d] = frm[j][6 + d];
                    }
                    double ps, ax, ay, az;
                    if constexpr (HESS) {
                        double h[3];
                        m2p_eval_hess<P>(coef + j * EW, fr, frm[j][9], nx, ny, nz, et, ep, &ps, &ax, &ay, &az, h);
                        hs[0] += h[0];
                        hs[1] += h[1];
                        hs[2] += h[2];
                    } else {
                        m2p_eval<P>(coef + j * EW, fr, frm[j][9], nx, ny, nz, &ps, &ax, &ay, &az);
                    }
                    p0 += ps;
                    p1 += ax;
                    p2 += ay;
                    p3 += az;
                }
            }
        }
        __syncthreads();  // the last chunk fully consumed before red overwrites it
        red[0][lane] = p0;
        red[1][lane] = p1;
        red[2][lane] = p2;
        red[3][lane] = p3;
        if constexpr (HESS) {
            redh[0][lane] = hs[0];
            redh[1][lane] = hs[1];
            redh[2][lane] = hs[2];
        }
        __syncthreads();
        if (lane < ng) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            double h[3] = {0.0, 0.0, 0.0};
            for (int j = lane * L; j < lane * L + L; ++j) {
                s0 += red[0][j];
                s1 += red[1][j];
                s2 += red[2][j];
                s3 += red[3][j];
                if constexpr (HESS) {
                    h[0] += redh[0][j];
                    h[1] += redh[1][j];
                    h[2] += redh[2][j];
                }
            }
            if constexpr (HESS)
                emit_target_hess(item.w < 0 ? -1 : item.w + tg + lane, tperm[g0 + lane], s0, s1, s2, s3, h, part,
                                 psi, defl, hess, m_out);
            else
                emit_target(item.w < 0 ? -1 : item.w + tg + lane, tperm[g0 + lane], s0, s1, s2, s3, part, psi,
                            defl, m_out);
        }
        __syncthreads();  // red is reused by the next group
    }
}

void reduce_items(const WorkItems& w, const int* tfirst, const int* tcount, const uint32_t* tperm, double* psi,
                  double* defl, int64_t m_out, double* part, hipStream_t s, double* hess) {
    if (w.nred <= 0) return;
    if (hess)
        k_near_reduce<true><<<(unsigned)w.nred, 64, 0, s>>>(w.red.data(), tfirst, tcount, tperm, part, psi, defl,
                                                            hess, m_out);
    else
        k_near_reduce<false><<<(unsigned)w.nred, 64, 0, s>>>(w.red.data(), tfirst, tcount, tperm, part, psi, defl,
                                                             nullptr, m_out);
    SFMM_LAUNCH_CHECK();
}

void fmm_p2p(const FmmCtx& c, bool fp32, const WorkItems& w, const int* src, const int* tfirst,
             const int* tcount, const double* tx, const double* ty, const double* tz, const uint32_t* tperm,
             double* psi, double* defl, int64_t m_out, hipStream_t s, double* part, double* hess) {
    if (w.n <= 0) return;
    if (hess && !part && w.nred > 0) throw Error(ST_INTERNAL, "the Hessian needs partial slots of 8 doubles");
    if (!part) part = w.part.data();
    const NpmK nk = npm_params(c.npm_sigma);
    const bool npm = c.npm_sigma > 0.0;
#define P2P_(T, H, N)                                                                                          \
    k_p2p<T, H, N><<<(unsigned)w.n, 64, 0, s>>>(c, w.items.data(), src, tfirst, tcount, tx, ty, tz, tperm, psi, \
                                                defl, m_out, part, kLogPoly, hess, nk)
#define P2P_N(T, H)              \
    if (npm) P2P_(T, H, true);   \
    else P2P_(T, H, false)
    if (fp32) {
        if (hess) P2P_N(TileF32, true);
        else P2P_N(TileF32, false);
    } else {
        if (hess) P2P_N(TileF64, true);
        else P2P_N(TileF64, false);
    }
#undef P2P_N
#undef P2P_
    SFMM_LAUNCH_CHECK();
    reduce_items(w, tfirst, tcount, tperm, psi, defl, m_out, part, s, hess);
}

void fmm_m2p(const FmmCtx& c, const WorkItems& w, const int* src, const int* tfirst, const int* tcount,
             const double* tx, const double* ty, const double* tz, const uint32_t* tperm, double* psi,
             double* defl, int64_t m_out, hipStream_t s, double* part, double* hess) {
    if (w.n <= 0 || c.p < kM2PMinOrder) return;
    if (hess && !part && w.nred > 0) throw Error(ST_INTERNAL, "the Hessian needs partial slots of 8 doubles");
    if (!part) part = w.part.data();
#define L_(P)                                                                                                 \
    case P:                                                                                                   \
        if (hess)                                                                                             \
            k_m2p<P, true><<<(unsigned)w.n, 64, 0, s>>>(c, w.items.data(), src, tfirst, tcount, tx, ty, tz,  \
                                                        tperm, psi, defl, m_out, part, hess);                 \
        else                                                                                                  \
            k_m2p<P, false><<<(unsigned)w.n, 64, 0, s>>>(c, w.items.data(), src, tfirst, tcount, tx, ty, tz, \
                                                         tperm, psi, defl, m_out, part, nullptr);             \
        break;
    SFMM_DISPATCH(c.p, L_)
#undef L_
    SFMM_LAUNCH_CHECK();
    reduce_items(w, tfirst, tcount, tperm, psi, defl, m_out, part, s, hess);
}

double npm_constant(double sigma) {
    if (!(sigma > 0.0)) return 0.0;
    const double st = std::sin(0.5 * sigma), t = st * st;
    double J = 0.0, tk = 1.0;
    for (int k = 0; k < 200 && tk > 1e-18; ++k, tk *= t) J += tk * ((2.0 - t) / (k + 2) - 1.0 / (k + 3));
    return t * (J - 1.0);
}

NpmK npm_params(double sigma) {
    NpmK k{};
    if (!(sigma > 0.0)) return k;
    const double st = std::sin(0.5 * sigma);
    k.t = st * st;
    k.inv_t = 1.0 / k.t;
    k.four_t = 4.0 * k.t;
    k.ln4t = std::log(4.0 * k.t);
    const double a = (1.0 - k.t) / k.t;
    k.a2 = a * a / 16.0;
    // terms of the series for I until t^k < 2^-56 (v <= 1)
    k.nterms = 1;
    for (double tk = k.t; tk >= 0x1p-56 && k.nterms < 64; tk *= k.t) ++k.nterms;
    return k;
}

}  // namespace sfmm
