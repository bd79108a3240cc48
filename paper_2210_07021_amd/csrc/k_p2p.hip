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
// at least 3: ratio 3 down to p = 23, 3.4 at p = 18, 4.5 at p = 12.  And when S holds at
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
            const double a = ratio * c.rad[S];
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
    out.n_near = out.n_far = 0;
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
    int h[2] = {0, 0};
    SFMM_HIP(hipMemcpyAsync(h, tot.data(), sizeof(h), hipMemcpyDeviceToHost, s));
    SFMM_HIP(hipStreamSynchronize(s));
    out.n_near = h[0];
    out.n_far = h[1];
    out.near_src.resize(std::max(h[0], 1));
    out.far_src.resize(std::max(h[1], 1));
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
    SFMM_HIP(hipStreamSynchronize(s));  // the temporaries are released on return
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

void build_items(const int* off, const int* src, const int* count, const int* tcount, int nbox, int seg,
                 WorkItems& out, hipStream_t s) {
    out.n = out.nred = 0;
    out.nslot = 0;
    if (nbox <= 0) return;
    DVec<int> nseg, nslot, multi, item_off, slot_off, red_off, tot;
    nseg.resize(nbox);
    nslot.resize(nbox);
    multi.resize(nbox);
    item_off.resize(nbox);
    slot_off.resize(nbox);
    red_off.resize(nbox);
    tot.resize(3);
    k_seg_count<<<nblk(nbox, 256), 256, 0, s>>>(off, tcount, nbox, seg, nseg.data(), nslot.data(), multi.data());
    SFMM_LAUNCH_CHECK();
    scan3_excl_i32(nseg.data(), nslot.data(), multi.data(), item_off.data(), slot_off.data(), red_off.data(), nbox,
                   tot.data(), s);
    int h[3];
    SFMM_HIP(hipMemcpyAsync(h, tot.data(), sizeof(h), hipMemcpyDeviceToHost, s));
    SFMM_HIP(hipStreamSynchronize(s));
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
    k_seg_emit<<<nblk(nbox, 256), 256, 0, s>>>(off, tcount, nbox, seg, nseg.data(), item_off.data(),
                                               slot_off.data(), red_off.data(), raw.data(), out.red.data());
    SFMM_LAUNCH_CHECK();
    k_item_keys<<<nblk(64 * (int64_t)out.n, 256), 256, 0, s>>>(raw.data(), out.n, src, count, tcount, keys.data(),
                                                             vals.data());
    SFMM_LAUNCH_CHECK();
    radix_sort_u64(keys.data(), vals.data(), out.n, 8, s);
    k_gather_items<<<nblk(out.n, 256), 256, 0, s>>>(raw.data(), vals.data(), out.n, out.items.data());
    SFMM_LAUNCH_CHECK();
    SFMM_HIP(hipStreamSynchronize(s));  // the temporaries are released on return
}

// Adds the per-segment results of every box cut into several items, in
// segment order: one workgroup per box, lanes over its targets.
__global__ void __launch_bounds__(64) k_near_reduce(const int4* __restrict__ red, const int* __restrict__ tfirst,
                                                   const int* __restrict__ tcount,
                                                   const uint32_t* __restrict__ tperm,
                                                   const double* __restrict__ part, double* __restrict__ psi,
                                                   double* __restrict__ defl, int64_t m_out) {
    const int4 r = red[blockIdx.x];
    const int T = r.x, ns = r.y, base = r.z;
    const int t0 = tfirst[T], nt = tcount[T];
    for (int t = threadIdx.x; t < nt; t += 64) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int sg = 0; sg < ns; ++sg) {
            const double* q = part + 4 * ((size_t)base + (size_t)sg * nt + t);
            s0 += q[0];
            s1 += q[1];
            s2 += q[2];
            s3 += q[3];
        }
        const int64_t o = tperm[t0 + t];
        psi[o] += s0;
        defl[o] += s1;
        defl[m_out + o] += s2;
        defl[2 * m_out + o] += s3;
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

// ------------------------------------------------------------ direct sums
// Pair terms of one lane over one LDS tile.  FP64: coordinates as stored.
// FP32 (precision tier): every coordinate is a two-float pair hi + lo
// (hi = float(x), lo = float(x - hi)), so d = (t_hi - s_hi) + (t_lo - s_lo)
// keeps ~1e-7 relative accuracy for close points where plain FP32 positions
// would lose all digits of d; log and reciprocal are the hardware FP32
// instructions, and each tile's FP32 partial sums (at most 256 terms) are
// added to FP64 running sums.
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

__device__ __forceinline__ void tile_pairs(const TileF64& t, const double2* ltab, const LogPoly& lk, int r, int L,
                                           int tn, double ax, double ay, double az, double& p0, double& p1, double& p2,
                                           double& p3) {
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
        const double wi = sp.w * i0;
        p0 = fma(sp.w, lg, p0);
        p1 = fma(wi, dx, p1);
        p2 = fma(wi, dy, p2);
        p3 = fma(wi, dz, p3);
    }
}

__device__ __forceinline__ void tile_pairs(const TileF32& t, const double2*, const LogPoly&, int r, int L, int tn,
                                           double ax, double ay, double az, double& p0, double& p1, double& p2,
                                           double& p3) {
    const float axh = (float)ax, ayh = (float)ay, azh = (float)az;
    const float axl = (float)(ax - (double)axh), ayl = (float)(ay - (double)ayh), azl = (float)(az - (double)azh);
    constexpr float kLn2f = 0.693147180559945309f, kLog4f = 1.38629436111989061f;
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f, f3 = 0.0f;
    for (int j = r; j < tn; j += L) {
        const float4 h = t.hi[j], l = t.lo[j];
        const float dx = (axh - h.x) + (axl - l.x);
        const float dy = (ayh - h.y) + (ayl - l.y);
        const float dz = (azh - h.z) + (azl - l.z);
        const float d2 = dx * dx + dy * dy + dz * dz;
        const bool coinc = d2 == 0.0f;
        const float r2 = coinc ? 1.0f : d2;
        const float lg = coinc ? kLog4f : __builtin_amdgcn_logf(r2) * kLn2f;
        const float wi = h.w * __builtin_amdgcn_rcpf(r2);
        f0 = fmaf(h.w, lg, f0);
        f1 = fmaf(wi, dx, f1);
        f2 = fmaf(wi, dy, f2);
        f3 = fmaf(wi, dz, f3);
    }
    p0 += (double)f0;
    p1 += (double)f1;
    p2 += (double)f2;
    p3 += (double)f3;
}

template <class Tile>
__global__ void __launch_bounds__(64) k_p2p(FmmCtx c, const int4* __restrict__ items,
                                           const int* __restrict__ src, const int* __restrict__ tfirst,
                                           const int* __restrict__ tcount, const double* __restrict__ tx,
                                           const double* __restrict__ ty, const double* __restrict__ tz,
                                           const uint32_t* __restrict__ tperm, double* __restrict__ psi,
                                           double* __restrict__ defl, int64_t m_out, double* __restrict__ part,
                                           LogPoly lk) {
    // the tile and the end-of-group reduction share one LDS block (fewer
    // bytes per wave, more waves per CU)
    constexpr size_t kSm = sizeof(Tile) > 4 * 64 * sizeof(double) ? sizeof(Tile) : 4 * 64 * sizeof(double);
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
                if (active) tile_pairs(tile, ltab, lk, r, L, tn, ax, ay, az, p0, p1, p2, p3);
            }
        }
        const double qn = wave_sum(qnear);
        __syncthreads();  // the last tile fully consumed before red overwrites it
        red[0][lane] = p0;
        red[1][lane] = p1;
        red[2][lane] = p2;
        red[3][lane] = p3;
        __syncthreads();
        if (lane < ng) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            for (int j = lane * L; j < lane * L + L; ++j) {
                s0 += red[0][j];
                s1 += red[1][j];
                s2 += red[2][j];
                s3 += red[3][j];
            }
            const int me = g0 + lane;
            const double mx = tx[me], myy = ty[me], mz = tz[me];
            const double il = 1.0 / sqrt(mx * mx + myy * myy + mz * mz);
            const double ux = mx * il, uy = myy * il, uz = mz * il;
            const double vr = ux * s1 + uy * s2 + uz * s3;
            emit_target(item.w < 0 ? -1 : item.w + tg + lane, tperm[me], (s0 + (1.0 - kLog4) * qn) * kInv4Pi,
                        (s1 - ux * vr) * kInv2Pi, (s2 - uy * vr) * kInv2Pi, (s3 - uz * vr) * kInv2Pi, part, psi,
                        defl, m_out);
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

template <int P>
__global__ void __launch_bounds__(64) k_m2p(FmmCtx c, const int4* __restrict__ items,
                                           const int* __restrict__ src, const int* __restrict__ tfirst,
                                           const int* __restrict__ tcount, const double* __restrict__ tx,
                                           const double* __restrict__ ty, const double* __restrict__ tz,
                                           const uint32_t* __restrict__ tperm, double* __restrict__ psi,
                                           double* __restrict__ defl, int64_t m_out, double* __restrict__ part) {
    constexpr int EW = 2 * P + 2;
    // the staged records double as the end-of-group reduction buffer
    static_assert(kChunkF * (2 * kM2PMinOrder + 2) >= 4 * 64, "reduction fits the record buffer");
    __shared__ __align__(16) double coef[kChunkF * EW];
    __shared__ double frm[kChunkF][10];  // c, e_theta, e_phi, rho
    double(*red)[64] = reinterpret_cast<double(*)[64]>(coef);
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
                    m2p_eval<P>(coef + j * EW, fr, frm[j][9], nx, ny, nz, &ps, &ax, &ay, &az);
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
        __syncthreads();
        if (lane < ng) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            for (int j = lane * L; j < lane * L + L; ++j) {
                s0 += red[0][j];
                s1 += red[1][j];
                s2 += red[2][j];
                s3 += red[3][j];
            }
            emit_target(item.w < 0 ? -1 : item.w + tg + lane, tperm[g0 + lane], s0, s1, s2, s3, part, psi, defl,
                        m_out);
        }
        __syncthreads();  // red is reused by the next group
    }
}

void reduce_items(const WorkItems& w, const int* tfirst, const int* tcount, const uint32_t* tperm, double* psi,
                  double* defl, int64_t m_out, double* part, hipStream_t s) {
    if (w.nred <= 0) return;
    k_near_reduce<<<(unsigned)w.nred, 64, 0, s>>>(w.red.data(), tfirst, tcount, tperm, part, psi, defl, m_out);
    SFMM_LAUNCH_CHECK();
}

void fmm_p2p(const FmmCtx& c, bool fp32, const WorkItems& w, const int* src, const int* tfirst,
             const int* tcount, const double* tx, const double* ty, const double* tz, const uint32_t* tperm,
             double* psi, double* defl, int64_t m_out, hipStream_t s, double* part) {
    if (w.n <= 0) return;
    if (!part) part = w.part.data();
    if (fp32)
        k_p2p<TileF32><<<(unsigned)w.n, 64, 0, s>>>(c, w.items.data(), src, tfirst, tcount, tx, ty, tz, tperm, psi,
                                                    defl, m_out, part, kLogPoly);
    else
        k_p2p<TileF64><<<(unsigned)w.n, 64, 0, s>>>(c, w.items.data(), src, tfirst, tcount, tx, ty, tz, tperm, psi,
                                                    defl, m_out, part, kLogPoly);
    SFMM_LAUNCH_CHECK();
    reduce_items(w, tfirst, tcount, tperm, psi, defl, m_out, part, s);
}

void fmm_m2p(const FmmCtx& c, const WorkItems& w, const int* src, const int* tfirst, const int* tcount,
             const double* tx, const double* ty, const double* tz, const uint32_t* tperm, double* psi,
             double* defl, int64_t m_out, hipStream_t s, double* part) {
    if (w.n <= 0 || c.p < kM2PMinOrder) return;
    if (!part) part = w.part.data();
#define L_(P)                                                                                             \
    case P:                                                                                               \
        k_m2p<P><<<(unsigned)w.n, 64, 0, s>>>(c, w.items.data(), src, tfirst, tcount, tx, ty, tz, tperm, psi, \
                                              defl, m_out, part);                                         \
        break;
    SFMM_DISPATCH(c.p, L_)
#undef L_
    SFMM_LAUNCH_CHECK();
    reduce_items(w, tfirst, tcount, tperm, psi, defl, m_out, part, s);
}

}  // namespace sfmm
