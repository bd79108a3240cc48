// Tree build on the GPU: order-29 HEALPix keys (Sec. 3.1), the adaptive
// quasi-quad-tree level by level, box geometry (Sec. 3.5), target location
// (Sec. 3.7), and the frontier form of Algorithm 1 (Sec. 3.4).
#include "common.hpp"
#include "geom.hpp"

#include <algorithm>
#include <cstdlib>

namespace sfmm {

static unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1); }

// ------------------------------------------------------------------ points
// Unit vectors, keys and identity permutation of n points given as [3][n];
// each point is written as one 32-byte record (x, y, z, q) so that the
// gather after the key sort moves one aligned record per point (q = 0 when
// the points carry no charge).
__global__ void k_prepare_points(const double* in, const double* q, int64_t n, double4* u, uint64_t* keys,
                                 uint32_t* idx, int* err) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = in[i], b = in[n + i], c = in[2 * n + i];
    const double r2 = a * a + b * b + c * c;
    int e = 0;
    if (!(isfinite(a) && isfinite(b) && isfinite(c))) e |= 1;
    else if (!(fabs(r2 - 1.0) <= 2e-6)) e |= 2;
    if (e) {
        atomicOr(err, e);
        a = 0.0; b = 0.0; c = 1.0;
    } else if (fabs(r2 - 1.0) > 1e-14) {
        const double inv = 1.0 / sqrt(r2);
        a *= inv; b *= inv; c *= inv;
    }
    u[i] = make_double4(a, b, c, q ? q[i] : 0.0);
    keys[i] = key29(a, b, c);
    idx[i] = (uint32_t)i;
}

void prepare_points(const double* in, const double* q, int64_t n, double4* u, uint64_t* keys, uint32_t* idx,
                    int* err, hipStream_t s) {
    if (n <= 0) return;
    k_prepare_points<<<nblocks(n, 256), 256, 0, s>>>(in, q, n, u, keys, idx, err);
    SFMM_LAUNCH_CHECK();
}

// Targets in plan order: coordinates (SoA) and leaf box of the target at
// each position, from the leaf-sorted (leaf, index) pairs.
__global__ void k_gather_targets(const uint32_t* idx, const uint64_t* leaf_sorted, int64_t n,
                                 const double4* __restrict__ u, double* ox, double* oy, double* oz, int* leaf) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 v = u[idx[i]];
    ox[i] = v.x;
    oy[i] = v.y;
    oz[i] = v.z;
    leaf[i] = (int)leaf_sorted[i];
}

void gather_targets(const uint32_t* idx, const uint64_t* leaf_sorted, int64_t n, const double4* u, double* ox,
                    double* oy, double* oz, int* leaf, hipStream_t s) {
    if (n <= 0) return;
    k_gather_targets<<<nblocks(n, 256), 256, 0, s>>>(idx, leaf_sorted, n, u, ox, oy, oz, leaf);
    SFMM_LAUNCH_CHECK();
}

__global__ void k_gather_records(const uint32_t* idx, int64_t n, const double4* __restrict__ u, double4* out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = u[idx[i]];
}

void gather_records(const uint32_t* idx, int64_t n, const double4* u, double4* out, hipStream_t s) {
    if (n <= 0) return;
    k_gather_records<<<nblocks(n, 256), 256, 0, s>>>(idx, n, u, out);
    SFMM_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ levels
__device__ int lower_bound_u64(const uint64_t* a, int lo, int hi, uint64_t v) {
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void k_base_level(const uint64_t* keys, int n, int* level, uint64_t* pixel, int* first, int* count,
                             int* parent, int* child0) {
    const int f = threadIdx.x;
    if (f >= 12) return;
    const int a = lower_bound_u64(keys, 0, n, (uint64_t)f << (2 * kOrder));
    const int b = lower_bound_u64(keys, 0, n, (uint64_t)(f + 1) << (2 * kOrder));
    level[f] = 0;
    pixel[f] = (uint64_t)f;
    first[f] = a;
    count[f] = b - a;
    parent[f] = -1;
    child0[f] = -1;
}

void tree_base_level(const uint64_t* keys, int64_t n, int* level, uint64_t* pixel, int* first, int* count,
                     int* parent, int* child0, hipStream_t s) {
    k_base_level<<<1, 64, 0, s>>>(keys, (int)n, level, pixel, first, count, parent, child0);
    SFMM_LAUNCH_CHECK();
}

__global__ void k_split_flags(int b0, int nb, const int* level, const int* count, int m, int max_level, int* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int b = b0 + i;
    flag[i] = (count[b] > m && level[b] < max_level) ? 1 : 0;
}

void tree_split_flags(int b0, int nb, const int* level, const int* count, int m, int max_level, int* flag,
                      hipStream_t s) {
    k_split_flags<<<nblocks(nb, 256), 256, 0, s>>>(b0, nb, level, count, m, max_level, flag);
    SFMM_LAUNCH_CHECK();
}

// The four children of box b (pixel p at level L) when it splits (slot >= 0:
// the split box's index among its level's split boxes, children at
// child_base + 4 slot): each child's point range is cut from the parent's
// sorted keys; child0[b] = -1 when it does not split.
__device__ void children_thread(int b, int slot, int child_base, const uint64_t* __restrict__ keys, int* level,
                                uint64_t* pixel, int* first, int* count, int* parent, int* child0) {
    if (slot < 0) {
        child0[b] = -1;
        return;
    }
    const int c0 = child_base + 4 * slot;
    child0[b] = c0;
    const int L = level[b] + 1;
    const int shift = 2 * (kOrder - L);
    const int end = first[b] + count[b];
    int lo = first[b];
    for (int c = 0; c < 4; ++c) {
        const uint64_t pix = pixel[b] * 4 + (uint64_t)c;
        const int e = (c == 3) ? end : lower_bound_u64(keys, lo, end, (pix + 1) << shift);
        level[c0 + c] = L;
        pixel[c0 + c] = pix;
        first[c0 + c] = lo;
        count[c0 + c] = e - lo;
        parent[c0 + c] = b;
        child0[c0 + c] = -1;
        lo = e;
    }
}

__global__ void k_make_children(int b0, int nb, int child_base, const int* flag, const int* off,
                                const uint64_t* keys, int* level, uint64_t* pixel, int* first, int* count,
                                int* parent, int* child0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    children_thread(b0 + i, flag[i] ? off[i] : -1, child_base, keys, level, pixel, first, count, parent, child0);
}

// First index in [lo, hi) whose key is >= v (hi when none), found by the 64
// lanes of a wave together: each step tests 64 evenly spaced keys of the
// range and keeps the gap where the predicate turns true, so a range of n
// keys takes about log(n) / log(65) dependent loads.  Every lane returns the
// same index (the loop is uniform across the wave).
__device__ int wave_lower_bound_u64(const uint64_t* __restrict__ a, int lo, int hi, uint64_t v) {
    const int lane = threadIdx.x & 63;
    while (hi > lo) {
        const int n = hi - lo;
        if (n <= 64) {
            const bool p = lane < n && a[lo + lane] >= v;
            const uint64_t m = __ballot(p);
            return m ? lo + (int)__ffsll((unsigned long long)m) - 1 : hi;
        }
        const int q = lo + (int)(((int64_t)(lane + 1) * n) / 65);  // in [lo, hi)
        const uint64_t m = __ballot(a[q] >= v);
        const int j = m ? (int)__ffsll((unsigned long long)m) - 1 : 64;
        const int qprev = j > 0 ? __shfl(q, j - 1, 64) : lo - 1;
        const int qj = j < 64 ? __shfl(q, j, 64) : hi;
        lo = qprev + 1;
        hi = qj;
    }
    return lo;
}

// children_thread with the whole wave on one box (levels of few, large
// boxes); b and slot are uniform across the wave.
__device__ void children_wave(int b, int slot, int child_base, const uint64_t* __restrict__ keys, int* level,
                              uint64_t* pixel, int* first, int* count, int* parent, int* child0) {
    const int lane = threadIdx.x & 63;
    if (slot < 0) {
        if (lane == 0) child0[b] = -1;
        return;
    }
    const int c0 = child_base + 4 * slot;
    const int L = level[b] + 1;
    const int shift = 2 * (kOrder - L);
    const int end = first[b] + count[b];
    const int f0 = first[b];
    const uint64_t pb = pixel[b] * 4;
    const int e0 = wave_lower_bound_u64(keys, f0, end, (pb + 1) << shift);
    const int e1 = wave_lower_bound_u64(keys, e0, end, (pb + 2) << shift);
    const int e2 = wave_lower_bound_u64(keys, e1, end, (pb + 3) << shift);
    if (lane < 4) {
        const int c = lane;
        const int st = c == 0 ? f0 : c == 1 ? e0 : c == 2 ? e1 : e2;
        const int en = c == 0 ? e0 : c == 1 ? e1 : c == 2 ? e2 : end;
        level[c0 + c] = L;
        pixel[c0 + c] = pb + (uint64_t)c;
        first[c0 + c] = st;
        count[c0 + c] = en - st;
        parent[c0 + c] = b;
        child0[c0 + c] = -1;
    }
    if (lane == 0) child0[b] = c0;
}

// k_make_children with one wave per box
__global__ void k_make_children_wave(int b0, int nb, int child_base, const int* flag, const int* off,
                                     const uint64_t* keys, int* level, uint64_t* pixel, int* first, int* count,
                                     int* parent, int* child0) {
    const int i = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    if (i >= nb) return;  // uniform across the wave
    children_wave(b0 + i, flag[i] ? off[i] : -1, child_base, keys, level, pixel, first, count, parent, child0);
}

void tree_make_children(int b0, int nb, int child_base, const int* flag, const int* off, const uint64_t* keys,
                        int* level, uint64_t* pixel, int* first, int* count, int* parent, int* child0,
                        int wave_level, hipStream_t s) {
    if (nb <= 0) return;
    if (nb < wave_level) {
        k_make_children_wave<<<nblocks((int64_t)nb * 64, 256), 256, 0, s>>>(b0, nb, child_base, flag, off, keys,
                                                                           level, pixel, first, count, parent,
                                                                           child0);
    } else {
        k_make_children<<<nblocks(nb, 256), 256, 0, s>>>(b0, nb, child_base, flag, off, keys, level, pixel, first,
                                                        count, parent, child0);
    }
    SFMM_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ queued levels
// The same level loop with the level bounds in device memory (ls[L] ..
// ls[L+1] - 1 are level L's boxes), so levels run back to back without a
// read-back each: per level, split counts per chunk of kTreeChunk boxes,
// then the children (which also set ls[L+2], or the overflow flag ctl[0]
// when the children would pass the capacity): two launches per level.
constexpr int kTreeThreads = 256;
constexpr int kTreePer = kTreeChunk / kTreeThreads;

__device__ int tree_block_excl(int v, int* sh, int* total) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kTreeThreads / 64; ++w) {
        const int ws = sh[w];
        before += (w < wv) ? ws : 0;
        all += ws;
    }
    *total = all;
    __syncthreads();
    return before + x - v;
}

__global__ void k_tree_init(int* ls, int nls, int* ctl) {
    const int t = threadIdx.x;
    if (t < nls) ls[t] = (t == 0) ? 0 : 12;
    if (t == 0) ctl[0] = 0;
}

// Per chunk: the split count, and for each box its rank among the chunk's
// split boxes (wpre, -1 when it does not split).
__global__ void __launch_bounds__(kTreeThreads) k_tree_count(const int* ls, int L, const int* count, int m,
                                                              int split_ok, int* ccnt, int* wpre) {
    __shared__ int sh[kTreeThreads / 64];
    const int b0 = ls[L], nb = ls[L + 1] - b0;
    const int nch = (nb + kTreeChunk - 1) / kTreeChunk;
    for (int j = blockIdx.x; j < nch; j += gridDim.x) {
        const int i0 = j * kTreeChunk + threadIdx.x * kTreePer;
        int f[kTreePer], c = 0;
#pragma unroll
        for (int q = 0; q < kTreePer; ++q) {
            f[q] = (split_ok && i0 + q < nb && count[b0 + i0 + q] > m) ? 1 : 0;
            c += f[q];
        }
        int tot;
        int e = tree_block_excl(c, sh, &tot);
#pragma unroll
        for (int q = 0; q < kTreePer; ++q) {
            if (i0 + q < nb) wpre[i0 + q] = f[q] ? e : -1;
            e += f[q];
        }
        if (threadIdx.x == 0) ccnt[j] = tot;
    }
}

// Sum of ccnt[0 .. n) by the whole wave (every lane returns it).
__device__ int wave_sum_prefix(const int* ccnt, int n) {
    const int lane = threadIdx.x & 63;
    int sum = 0;
    for (int k = lane; k < n; k += 64) sum += ccnt[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    return sum;
}

// Children of every box of the level: a wave per box on levels of fewer
// than wave_level boxes, else a lane per box (grid-stride either way).  A
// split box's slot is the split count of the chunks before its own (summed
// here from the per-chunk counts) plus its rank in its chunk.  The first
// wave of workgroup 0 sums all chunks: the next level's bounds ls[L+2], or
// the overflow flag when the children would pass cap boxes (boxes whose
// children would not fit write none; the caller then rebuilds the tree).
__global__ void __launch_bounds__(kTreeThreads) k_tree_children(int* ls, int L, const int* ccnt, const int* wpre,
                                                                 int* ctl, int cap, const uint64_t* __restrict__ keys,
                                                                 int* level, uint64_t* pixel, int* first, int* count,
                                                                 int* parent, int* child0, int wave_level) {
    if (ctl[0]) {  // an earlier level overflowed: this one stays empty
        if (blockIdx.x == 0 && threadIdx.x == 0) ls[L + 2] = ls[L + 1];
        return;
    }
    const int b0 = ls[L], nb = ls[L + 1] - b0, child_base = ls[L + 1];
    const int nch = (nb + kTreeChunk - 1) / kTreeChunk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (blockIdx.x == 0 && wave == 0) {
        const int tot = wave_sum_prefix(ccnt, nch);
        if (lane == 0) {
            const int64_t need = (int64_t)child_base + 4 * (int64_t)tot;
            if (need > cap) {
                ctl[0] = 1;
                ls[L + 2] = ls[L + 1];
            } else {
                ls[L + 2] = (int)need;
            }
        }
    }
    const int nw = gridDim.x * (kTreeThreads / 64);
    if (nb < wave_level) {
        for (int i = blockIdx.x * (kTreeThreads / 64) + wave; i < nb; i += nw) {
            const int r = wpre[i];
            const int pre = wave_sum_prefix(ccnt, i / kTreeChunk);
            int slot = r >= 0 ? pre + r : -1;
            if (slot >= 0 && (int64_t)child_base + 4 * (int64_t)slot + 4 > cap) continue;  // overflow
            children_wave(b0 + i, slot, child_base, keys, level, pixel, first, count, parent, child0);
        }
    } else {
        // a wave takes 64 consecutive boxes, which span at most two chunks
        for (int base = (blockIdx.x * (kTreeThreads / 64) + wave) * 64; base < nb; base += nw * 64) {
            const int c0 = base / kTreeChunk;
            const int pre0 = wave_sum_prefix(ccnt, c0);
            const int i = base + lane;
            if (i >= nb) continue;
            const int pre = (i / kTreeChunk == c0) ? pre0 : pre0 + ccnt[c0];
            const int r = wpre[i];
            const int slot = r >= 0 ? pre + r : -1;
            if (slot >= 0 && (int64_t)child_base + 4 * (int64_t)slot + 4 > cap) continue;  // overflow
            children_thread(b0 + i, slot, child_base, keys, level, pixel, first, count, parent, child0);
        }
    }
}

int tree_wave_level() {
    const char* v = std::getenv("SFMM_WAVE_LEVEL");
    if (!v) return kWaveLevel;
    const long w = std::strtol(v, nullptr, 10);
    return (int)std::max(0L, std::min(w, 0x7fffffffL));
}

void tree_init_queued(int* ls, int nls, int* ctl, hipStream_t s) {
    k_tree_init<<<1, 64, 0, s>>>(ls, nls, ctl);
    SFMM_LAUNCH_CHECK();
}

void tree_level_queued(int* ls, int L, int* ccnt, int* wpre, int grid, int cgrid, int cap, int* ctl, int m,
                       int split_ok, const uint64_t* keys, int* level, uint64_t* pixel, int* first, int* count,
                       int* parent, int* child0, int wave_level, hipStream_t s) {
    k_tree_count<<<grid, kTreeThreads, 0, s>>>(ls, L, count, m, split_ok, ccnt, wpre);
    SFMM_LAUNCH_CHECK();
    k_tree_children<<<cgrid, kTreeThreads, 0, s>>>(ls, L, ccnt, wpre, ctl, cap, keys, level, pixel, first, count,
                                                   parent, child0, wave_level);
    SFMM_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ geometry
__global__ void k_box_geometry(int nb, const int* level, const uint64_t* pixel, double* cen, double* rad,
                               double* gdd) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const BoxGeomDD g = box_geometry(level[b], pixel[b]);
    cen[4 * b + 0] = g.c[0].hi;
    cen[4 * b + 1] = g.c[1].hi;
    cen[4 * b + 2] = g.c[2].hi;
    cen[4 * b + 3] = tan(0.5 * g.r.hi);  // coefficient scale rho
    rad[b] = g.r.hi;
    double* o = gdd + 8 * b;
    o[0] = g.c[0].hi; o[1] = g.c[0].lo;
    o[2] = g.c[1].hi; o[3] = g.c[1].lo;
    o[4] = g.c[2].hi; o[5] = g.c[2].lo;
    o[6] = g.r.hi;    o[7] = g.r.lo;
}

void box_geometry(int nb, const int* level, const uint64_t* pixel, double* cen, double* rad, double* gdd,
                  hipStream_t s) {
    if (nb <= 0) return;
    k_box_geometry<<<nblocks(nb, 128), 128, 0, s>>>(nb, level, pixel, cen, rad, gdd);
    SFMM_LAUNCH_CHECK();
}

// Protected radius of a source box (Sec. 3.5): c_s R, widened to R + sigma
// under the near-particle model so that a particle's whole profile lies
// inside it.  FP64 and double-double forms.
__device__ __forceinline__ double protected_radius(double r, double c_s, double sigma) {
    const double p = c_s * r;
    return (sigma > 0.0 && r + sigma > p) ? r + sigma : p;
}

__global__ void k_walk_boxes(int nb, const double* cen, const double* rad, const double* gdd, const int* child0,
                             const int* count, double c_s, double c_t, double sigma, double4* geo, double2* strig,
                             double4* ttrig, int2* cc, double* dtrig) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const double r = rad[b];
    geo[b] = make_double4(cen[4 * b], cen[4 * b + 1], cen[4 * b + 2], r);
    double s1, c1, s2, c2, s3, c3;
    sincos(protected_radius(r, c_s, sigma), &s1, &c1);
    sincos(r, &s2, &c2);
    sincos(r / c_t, &s3, &c3);
    strig[b] = make_double2(c1, s1);
    ttrig[b] = make_double4(c2, s2, c3, s3);
    cc[b] = make_int2(child0[b], count[b]);
    // double-double tables for the exact decisions of near-ties
    const dd R = {gdd[8 * (size_t)b + 6], gdd[8 * (size_t)b + 7]};
    const bool widen = sigma > 0.0 && r + sigma > c_s * r;
    const dd prot = widen ? dd_add(R, dd_from(sigma)) : dd_mul_d(R, c_s);
    const dd ang[3] = {prot, R, dd_div(R, dd_from(c_t))};
    double* o = dtrig + kWalkDtrig * (size_t)b;
    o[12] = prot.hi;
    o[13] = prot.lo;
    for (int k = 0; k < 3; ++k) {
        dd sn, cs;
        dd_sincos(ang[k], &sn, &cs);
        o[4 * k + 0] = cs.hi;
        o[4 * k + 1] = cs.lo;
        o[4 * k + 2] = sn.hi;
        o[4 * k + 3] = sn.lo;
    }
}

void walk_boxes(int nb, const double* cen, const double* rad, const double* gdd, const int* child0, const int* count,
                double c_s, double c_t, double sigma, double4* geo, double2* strig, double4* ttrig, int2* cc,
                double* dtrig, hipStream_t s) {
    if (nb <= 0) return;
    k_walk_boxes<<<nblocks(nb, 128), 128, 0, s>>>(nb, cen, rad, gdd, child0, count, c_s, c_t, sigma, geo, strig, ttrig,
                                                  cc, dtrig);
    SFMM_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ targets
// Leaf box of each target from its key (any order of the targets), as the
// 64-bit sort key of the target order.
__global__ void k_locate(const uint64_t* keys, int64_t m, const int* child0, const int* level, uint64_t* leaf) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint64_t k = keys[i];
    int b = (int)(k >> (2 * kOrder));
    while (child0[b] >= 0) {
        const int L = level[b] + 1;
        b = child0[b] + (int)((k >> (2 * (kOrder - L))) & 3);
    }
    leaf[i] = (uint64_t)b;
}

void locate_targets(const uint64_t* keys, int64_t m, const int* child0, const int* level, uint64_t* leaf,
                    hipStream_t s) {
    if (m <= 0) return;
    k_locate<<<nblocks(m, 256), 256, 0, s>>>(keys, m, child0, level, leaf);
    SFMM_LAUNCH_CHECK();
}

// Targets in plan order: each leaf's targets form one run.  The run's first target
// writes tfirst, its last one the end index into tcount; k_range_counts turns
// the end into a count (tcount starts at 0, so empty leaves stay 0).
__global__ void k_target_ranges(const int* leaf, int64_t m, int* tfirst, int* tcount) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int b = leaf[i];
    if (i == 0 || leaf[i - 1] != b) tfirst[b] = (int)i;
    if (i == m - 1 || leaf[i + 1] != b) tcount[b] = (int)(i + 1);
}

__global__ void k_range_counts(const int* tfirst, int nbox, int* tcount) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbox && tcount[b] > 0) tcount[b] -= tfirst[b];
}

void target_ranges(const int* leaf, int64_t m, int nbox, int* tfirst, int* tcount, hipStream_t s) {
    if (m <= 0) return;
    k_target_ranges<<<nblocks(m, 256), 256, 0, s>>>(leaf, m, tfirst, tcount);
    SFMM_LAUNCH_CHECK();
    k_range_counts<<<nblocks(nbox, 256), 256, 0, s>>>(tfirst, nbox, tcount);
    SFMM_LAUNCH_CHECK();
}

__global__ void k_flag_nonzero(const int* count, int n, int* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = count[i] > 0 ? 1 : 0;
}

void flag_nonzero(const int* count, int n, int* flag, hipStream_t s) {
    if (n <= 0) return;
    k_flag_nonzero<<<nblocks(n, 256), 256, 0, s>>>(count, n, flag);
    SFMM_LAUNCH_CHECK();
}

__global__ void k_compact_index(const int* flag, const int* off, int n, int* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) out[off[i]] = i;
}

void compact_index(const int* flag, const int* off, int n, int* out, hipStream_t s) {
    if (n <= 0) return;
    k_compact_index<<<nblocks(n, 256), 256, 0, s>>>(flag, off, n, out);
    SFMM_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ walk
// Frontier form of Algorithm 1.  Each frontier pair (S, T) takes exactly
// one branch of INTERACTION(B_S, B_T); its recursive calls become the next
// frontier.  A source box without particles contributes nothing (it is a
// leaf, so no recursion is lost) and is dropped.
enum : uint8_t { A_NONE = 0, A_M2L = 1, A_P2P = 2, A_SPLIT_S = 3, A_SPLIT_T = 4, A_SPLIT_SELF = 5 };

// One round of the walk in three launches, sized on the device: the round's
// frontier size and output bases sit in st[0..2] (written by the previous
// round's emit), so rounds can be queued without reading anything back.  The
// pairs are taken in chunks of kWalkChunk, chunk c by workgroup c mod grid,
// in kWalkItems passes of kWalkThreads consecutive pairs (lane order = pair
// order).  k_walk_classify writes each pair's action and the chunk's three
// totals (children pairs, M2L pairs, P2P pairs); k_walk_chunk_scan scans the
// chunk totals; k_walk_emit scans the chunk's actions again and writes every
// output at its place in pair order, consecutive lanes to consecutive slots
// (so the lists come out in the same order as a scan over single pairs).
constexpr int kWalkItems = 4, kWalkThreads = 256, kWalkChunk = kWalkItems * kWalkThreads;

__device__ __forceinline__ int walk_nchild(uint8_t a) {
    return (a == A_SPLIT_S || a == A_SPLIT_T) ? 4 : (a == A_SPLIT_SELF ? 16 : 0);
}

// walk_action with the FP64 filters only: A_TIE where a double-double
// decision is needed (a MAC margin or a radius difference near zero)
constexpr uint8_t A_TIE = 7;
__device__ __forceinline__ uint8_t walk_action_fast(const WalkCtx& w, int s, int t) {
    const int2 bs = w.cc[s];
    if (bs.y == 0) return A_NONE;
    if (s == t) return (bs.x < 0) ? A_P2P : A_SPLIT_SELF;
    const int2 bt = w.cc[t];
    const double4 gs = w.geo[s], gt = w.geo[t];
    const double rs = gs.w, rt = gt.w;
    const int f = mac_far_filter_trig(gs.x, gs.y, gs.z, gt.x, gt.y, gt.z, protected_radius(rs, w.c_s, w.sigma), rt,
                                      w.strig[s], w.ttrig[t], 1.0, w.c_t);
    if (f > 0) return A_M2L;
    if (f == 0) return A_TIE;
    const bool sl = bs.x < 0, tl = bt.x < 0;
    if (!sl && !tl) {
        const double diff = rs - rt;
        if (!(fabs(diff) > 1e-13 * (rs + rt))) return A_TIE;
        return diff > 0.0 ? A_SPLIT_S : A_SPLIT_T;
    }
    if (!sl) return A_SPLIT_S;
    if (!tl) return A_SPLIT_T;
    return A_P2P;
}

// walk_action_fast's A_TIE cases decided exactly (double-double)
__device__ uint8_t walk_action_tie(const WalkCtx& w, int s, int t) {
    const int2 bs = w.cc[s], bt = w.cc[t];
    const double4 gs4 = w.geo[s], gt4 = w.geo[t];
    const double* a = w.gdd + 8 * (size_t)s;
    const double* b = w.gdd + 8 * (size_t)t;
    int f = mac_far_filter_trig(gs4.x, gs4.y, gs4.z, gt4.x, gt4.y, gt4.z, protected_radius(gs4.w, w.c_s, w.sigma),
                                gt4.w, w.strig[s], w.ttrig[t], 1.0, w.c_t);
    if (f == 0) {
        const dd csd[3] = {{a[0], a[1]}, {a[2], a[3]}, {a[4], a[5]}};
        const dd ctd[3] = {{b[0], b[1]}, {b[2], b[3]}, {b[4], b[5]}};
        const double* ta = w.dtrig + kWalkDtrig * (size_t)s;
        const double* tb = w.dtrig + kWalkDtrig * (size_t)t;
        const dd ts[2] = {{ta[0], ta[1]}, {ta[2], ta[3]}};
        const dd tt[4] = {{tb[4], tb[5]}, {tb[6], tb[7]}, {tb[8], tb[9]}, {tb[10], tb[11]}};
        f = mac_far_dd_trig(csd, ctd, dd{ta[12], ta[13]}, dd{b[6], b[7]}, ts, tt, 1.0, w.c_t) ? 1 : -1;
    }
    if (f > 0) return A_M2L;
    const bool sl = bs.x < 0, tl = bt.x < 0;
    if (!sl && !tl) return radius_greater(a[6], b[6], dd{a[6], a[7]}, dd{b[6], b[7]}) ? A_SPLIT_S : A_SPLIT_T;
    if (!sl) return A_SPLIT_S;
    if (!tl) return A_SPLIT_T;
    return A_P2P;
}

// Three counts of a thread summed over the workgroup (kWalkThreads):
// exclusive prefix in thread order (ex) and total (all).
__device__ __forceinline__ void walk_block_scan3(const int c[3], int (*sh)[kWalkThreads / 64], int ex[3], int all[3]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        x[j] = c[j];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x[j], o, 64);
            if (lane >= o) x[j] += y;
        }
        if (lane == 63) sh[j][wv] = x[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        int before = 0, tot = 0;
#pragma unroll
        for (int v = 0; v < kWalkThreads / 64; ++v) {
            before += v < wv ? sh[j][v] : 0;
            tot += sh[j][v];
        }
        ex[j] = before + x[j] - c[j];
        all[j] = tot;
    }
    __syncthreads();  // sh is reused by the caller
}

// Classification of each chunk: FP64 decisions first; the near-ties of the
// chunk are gathered in LDS and decided exactly by consecutive threads (no
// wave runs that code for one lane); then the chunk's three totals.
__global__ void __launch_bounds__(kWalkThreads) k_walk_classify(const int2* __restrict__ F, const int* __restrict__ st,
                                                                WalkCtx w, uint8_t* __restrict__ action,
                                                                int* __restrict__ ctot, int cstride) {
    __shared__ int sh[3][kWalkThreads / 64];
    __shared__ int ntie;
    __shared__ short tie_at[kWalkChunk];
    __shared__ uint8_t tie_act[kWalkChunk];
    const int n = st[0];
    const int nchunk = (n + kWalkChunk - 1) / kWalkChunk;
    for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        const int k0 = ch * kWalkChunk;
        if (threadIdx.x == 0) ntie = 0;
        __syncthreads();
        uint8_t act[kWalkItems];
#pragma unroll
        for (int i = 0; i < kWalkItems; ++i) {
            const int li = i * kWalkThreads + threadIdx.x;
            act[i] = A_NONE;
            if (k0 + li < n) {
                const int2 f = F[k0 + li];
                act[i] = walk_action_fast(w, f.x, f.y);
                if (act[i] == A_TIE) tie_at[atomicAdd(&ntie, 1)] = (short)li;
            }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < ntie; j += kWalkThreads) {
            const int li = tie_at[j];
            const int2 f = F[k0 + li];
            tie_act[li] = walk_action_tie(w, f.x, f.y);
        }
        __syncthreads();
        int c[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < kWalkItems; ++i) {
            const int li = i * kWalkThreads + threadIdx.x;
            if (k0 + li < n) {
                const uint8_t a = act[i] == A_TIE ? tie_act[li] : act[i];
                action[k0 + li] = a;
                c[0] += walk_nchild(a);
                c[1] += a == A_M2L;
                c[2] += a == A_P2P;
            }
        }
        int ex[3], all[3];
        walk_block_scan3(c, sh, ex, all);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < 3; ++j) ctot[(size_t)j * cstride + ch] = all[j];
        }
        // sh, ntie and the tie lists are reused by the next chunk (the scan
        // ends with a barrier)
    }
}

// exclusive scans of the three chunk-total arrays (one workgroup of
// kChunkScanThreads each, in pieces of that size with a running carry);
// tot[j] = the total of array j
constexpr int kChunkScanThreads = 1024;
__global__ void __launch_bounds__(kChunkScanThreads) k_walk_chunk_scan(const int* __restrict__ st,
                                                                       const int* __restrict__ ctot, int cstride,
                                                                       int* __restrict__ coff, int* __restrict__ tot) {
    constexpr int kWaves = kChunkScanThreads / 64;
    __shared__ int sh[kWaves];
    const int n = st[0];
    const int nchunk = (n + kWalkChunk - 1) / kWalkChunk;
    const int j = blockIdx.x;
    const int* in = ctot + (size_t)j * cstride;
    int* out = coff + (size_t)j * cstride;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int carry = 0;
    for (int c0 = 0; c0 < nchunk; c0 += kChunkScanThreads) {
        const int i = c0 + threadIdx.x;
        const int v = i < nchunk ? in[i] : 0;
        int x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) sh[wv] = x;
        __syncthreads();
        int before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            before += q < wv ? sh[q] : 0;
            all += sh[q];
        }
        if (i < nchunk) out[i] = carry + before + x - v;
        carry += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[j] = carry;
}

__device__ uint64_t pair_key(int s, int t) { return ((uint64_t)(uint32_t)t << 32) | (uint32_t)s; }

// Emit of one round.  The next frontier (tot[0] pairs) and the lists'
// new ends are checked against the capacities first: when anything would not
// fit, nothing is written, *overflow is set and the next round is empty (the
// caller then runs the walk again with room to spare).  Otherwise workgroup 0
// writes the next round's st (frontier size, M2L and P2P bases).
__global__ void __launch_bounds__(kWalkThreads) k_walk_emit(const int2* __restrict__ F, const int* __restrict__ st,
                                                            WalkCtx w, const uint8_t* __restrict__ action,
                                                            const int* __restrict__ coff, int cstride,
                                                            const int* __restrict__ tot, WalkCaps cap,
                                                            int2* __restrict__ Fnext, uint64_t* __restrict__ m2l,
                                                            uint64_t* __restrict__ p2p, int* __restrict__ st_next,
                                                            int* __restrict__ overflow) {
    __shared__ int sh[3][kWalkThreads / 64];
    const int n = st[0], bm = st[1], bp = st[2];
    const int nc = tot[0], am = tot[1], ap = tot[2];
    const bool fits = nc <= cap.frontier && (int64_t)bm + am <= cap.m2l && (int64_t)bp + ap <= cap.p2p;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (fits) {
            st_next[0] = nc;
            st_next[1] = bm + am;
            st_next[2] = bp + ap;
        } else {
            *overflow = 1;
            st_next[0] = 0;
            st_next[1] = bm;
            st_next[2] = bp;
        }
    }
    if (!fits) return;
    const int nchunk = (n + kWalkChunk - 1) / kWalkChunk;
    for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        const int k0 = ch * kWalkChunk;
        int oc = coff[ch];
        int om = bm + coff[(size_t)cstride + ch];
        int op = bp + coff[2 * (size_t)cstride + ch];
        for (int i = 0; i < kWalkItems && k0 + i * kWalkThreads < n; ++i) {  // uniform across the workgroup
            const int k = k0 + i * kWalkThreads + threadIdx.x;
            const uint8_t a = k < n ? action[k] : A_NONE;
            const int c[3] = {walk_nchild(a), a == A_M2L, a == A_P2P};
            int ex[3], all[3];
            walk_block_scan3(c, sh, ex, all);
            if (a != A_NONE) {
                const int s = F[k].x, t = F[k].y;
                int2* out = Fnext + oc + ex[0];
                switch (a) {
                    case A_M2L: m2l[om + ex[1]] = pair_key(s, t); break;
                    case A_P2P: p2p[op + ex[2]] = pair_key(s, t); break;
                    case A_SPLIT_S:
                        for (int q = 0; q < 4; ++q) out[q] = make_int2(w.cc[s].x + q, t);
                        break;
                    case A_SPLIT_T:
                        for (int q = 0; q < 4; ++q) out[q] = make_int2(s, w.cc[t].x + q);
                        break;
                    case A_SPLIT_SELF:
                        for (int q = 0; q < 4; ++q)
                            for (int r = 0; r < 4; ++r) out[4 * q + r] = make_int2(w.cc[s].x + q, w.cc[s].x + r);
                        break;
                    default: break;
                }
            }
            oc += all[0];
            om += all[1];
            op += all[2];
        }
    }
}

int walk_chunks(int n) {
    const int nchunk = (n + kWalkChunk - 1) / kWalkChunk;
    return nchunk > 0 ? nchunk : 1;
}

void walk_round_scan(const int2* F, const int* st, const WalkCtx& w, uint8_t* action, int* ctot, int* coff,
                     int cstride, int* tot, int grid, hipStream_t s) {
    k_walk_classify<<<grid, kWalkThreads, 0, s>>>(F, st, w, action, ctot, cstride);
    SFMM_LAUNCH_CHECK();
    k_walk_chunk_scan<<<3, kChunkScanThreads, 0, s>>>(st, ctot, cstride, coff, tot);
    SFMM_LAUNCH_CHECK();
}

void walk_round_emit(const int2* F, const int* st, const WalkCtx& w, const uint8_t* action, const int* coff,
                     int cstride, const int* tot, const WalkCaps& cap, int2* Fnext, uint64_t* m2l, uint64_t* p2p,
                     int* st_next, int* overflow, int grid, hipStream_t s) {
    k_walk_emit<<<grid, kWalkThreads, 0, s>>>(F, st, w, action, coff, cstride, tot, cap, Fnext, m2l, p2p, st_next,
                                             overflow);
    SFMM_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ lists
// CSR offsets from the entries' target boxes in sorted order: off[b] = the
// first entry whose target is >= b
__global__ void k_csr_offsets(const int* tgt, int np, int nbox, int* off) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nbox) return;
    int lo = 0, hi = np;
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (tgt[mid] < b) lo = mid + 1;
        else hi = mid;
    }
    off[b] = lo;
}

// source and target box of every entry from the sorted pair keys
__global__ void k_pair_split(const uint64_t* sorted, int np, int* src, int* tgt) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const uint64_t v = sorted[k];
    src[k] = (int)(uint32_t)(v & 0xffffffffULL);
    tgt[k] = (int)(uint32_t)(v >> 32);
}

void pair_split(const uint64_t* sorted, int np, int* src, int* tgt, hipStream_t s) {
    if (np <= 0) return;
    k_pair_split<<<nblocks(np, 256), 256, 0, s>>>(sorted, np, src, tgt);
    SFMM_LAUNCH_CHECK();
}

void csr_offsets(const int* tgt, int np, int nbox, int* off, hipStream_t s) {
    k_csr_offsets<<<nblocks(nbox + 1, 256), 256, 0, s>>>(tgt, np, nbox, off);
    SFMM_LAUNCH_CHECK();
}

// M2L order keys: boxes of levels <= lc first (bit 15 clear), then the rest;
// most team rounds (tw_coarse or tw_fine pairs a round) first within each
// part, so the teams of a wave run the same number of rounds.  The sort is
// stable: boxes of one round count keep their index order, which is level by
// level in key order, so the teams of a workgroup are mostly neighbours
// sharing sources in the cache (3 % less M2L time than ordering by exact
// list length).
__global__ void k_m2l_order_keys(const int* off, const int* level, int lc, int tw_coarse, int tw_fine, int nbox,
                                 uint64_t* keys, uint32_t* vals) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    const bool fine = level[b] > lc;
    const int tw = fine ? tw_fine : tw_coarse;
    const uint32_t rounds = (uint32_t)(off[b + 1] - off[b] + tw - 1) / (uint32_t)tw;
    keys[b] = ((uint64_t)fine << 15) | (uint64_t)(0x7fffu - (rounds < 0x7fffu ? rounds : 0x7fffu));
    vals[b] = (uint32_t)b;
}

void m2l_order_keys(const int* off, const int* level, int lc, int tw_coarse, int tw_fine, int nbox, uint64_t* keys,
                    uint32_t* vals, hipStream_t s) {
    if (nbox <= 0) return;
    k_m2l_order_keys<<<nblocks(nbox, 256), 256, 0, s>>>(off, level, lc, tw_coarse, tw_fine, nbox, keys, vals);
    SFMM_LAUNCH_CHECK();
}

__global__ void k_work_order_keys(const long long* work, int n, uint64_t* keys, uint32_t* vals, int* flag) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const unsigned long long v = (unsigned long long)work[b];
    keys[b] = (v == 0) ? 255ULL : (uint64_t)__clzll(v);
    vals[b] = (uint32_t)b;
    flag[b] = v > 0 ? 1 : 0;
}

void work_order_keys(const long long* work, int n, uint64_t* keys, uint32_t* vals, int* flag, hipStream_t s) {
    if (n <= 0) return;
    k_work_order_keys<<<nblocks(n, 256), 256, 0, s>>>(work, n, keys, vals, flag);
    SFMM_LAUNCH_CHECK();
}

}  // namespace sfmm
