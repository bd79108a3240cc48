// Near field (the direct acts of Sec. 3.3-3.4): for every target in a leaf,
// the sum of the Green's function and its tangent gradient over the particles
// of the leaf's close boxes.
//
// One 64-wide wavefront (a 64-thread workgroup) owns one target leaf and
// takes its targets in groups of up to 64, lane t owning target t of the
// group.  The close leaves' particle ranges are concatenated into one flat
// index space (wave prefix sum of their counts); each tile of 256 particles
// is decoded once (binary search by lane shuffles) and staged in LDS, then
// every target of the group streams over the tile with the lanes splitting
// the particles, and a butterfly reduction hands the four partial sums to
// the target's lane.  No floating-point atomics: the result is bitwise
// reproducible.
//
// Per pair, with d = n_t - n_s, psi gets (q/4pi)(log(|d|^2/4) + 1) (Eq.
// GRE_FUN plus the zero-mean share) and alpha gets (q/2pi) d/|d|^2, projected
// on the tangent plane once per target.  A particle at exactly the target
// position keeps only its q/(4pi).  Per target and chunk only four sums are
// kept:
//   S = sum q log|d|^2   (log 4 in place of the log for a coincident particle)
//   V = sum q d/|d|^2    (d = 0 there, so nothing is added)
// and with Q_near = sum q over the summed leaves (from their Lemma 1 Q),
//   4 pi psi_near = S + (1 - log 4) Q_near.
//
// A close leaf S whose centre is more than 3 R_S from every target of the
// current chunk is not summed particle by particle: its own multipole
// expansion (Lemma 1) is evaluated at those targets instead.  By Eq. MUL_ERR
// the truncation error there is below (Q~/2pi) x^(p+1)/((p+1)(1-x)) with
// x ~ 1/3, i.e. under 1e-15 Q~ for p >= 28; this is done only for p >= 12
// and for leaves holding at least p/4 + 2 particles (below that the direct
// sum is cheaper).  Big leaves of sparse regions next to dense clumps are
// where it matters: their targets otherwise meet every particle of the
// clump directly.
#include "common.hpp"
#include "expand.hpp"

namespace sfmm {

constexpr int kTile = 256;  // particles staged in LDS per tile

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kM2PMinOrder = 12;
constexpr double kM2PRatio = 3.0;  // target beyond 3 R_S from the leaf centre

// Entry (close leaf) S is taken by its multipole expansion for a target group
// when it is full enough for that to pay (the expansion costs ~p/4 direct
// pairs) and every target of the group lies beyond kM2PRatio R_S of its
// centre (chord > 2 sin(3R/2)).  Both kernels below evaluate this same test.
__device__ __forceinline__ bool leaf_far(const FmmCtx& c, int S, int cnt, const double* __restrict__ tx,
                                         const double* __restrict__ ty, const double* __restrict__ tz,
                                         int g0, int ng) {
    if (c.p < kM2PMinOrder || 4 * cnt < c.p + 8) return false;
    const double a = kM2PRatio * c.rad[S];
    if (a >= 3.0) return false;
    const double h = 2.0 * sin(0.5 * a);
    const double thr = h * h;
    const double* cs = c.cen + 4 * (size_t)S;
    for (int t = 0; t < ng; ++t) {
        const int it = g0 + t;
        const double dx = tx[it] - cs[0], dy = ty[it] - cs[1], dz = tz[it] - cs[2];
        if (!(dx * dx + dy * dy + dz * dz > thr)) return false;
    }
    return true;
}

// Direct sums over the close leaves that are not taken by their expansion.
__global__ void __launch_bounds__(64) k_p2p(FmmCtx c, const int* __restrict__ tleaves, int ntl,
                                           const int* __restrict__ off, const int* __restrict__ src,
                                           const int* __restrict__ tfirst, const int* __restrict__ tcount,
                                           const double* __restrict__ tx, const double* __restrict__ ty,
                                           const double* __restrict__ tz, const uint32_t* __restrict__ tperm,
                                           double* __restrict__ psi, double* __restrict__ defl, int64_t m_out) {
    __shared__ double4 tile[kTile];
    const int lane = threadIdx.x;
    const int T = tleaves[blockIdx.x];
    const int k0 = off[T], K = off[T + 1] - k0;
    const int t0 = tfirst[T], nt = tcount[T];
    const int ew = 2 * c.p + 2;
    const double* __restrict__ sx = c.sx;
    const double* __restrict__ sy = c.sy;
    const double* __restrict__ sz = c.sz;
    const double* __restrict__ sq = c.sq;

    for (int tg = 0; tg < nt; tg += 64) {
        const int ng = min(64, nt - tg);
        const int g0 = t0 + tg;
        double own0 = 0.0, own1 = 0.0, own2 = 0.0, own3 = 0.0;  // S, V of this lane's target
        double qnear = 0.0;                                      // lane partials of Q_near
        for (int kc = 0; kc < K; kc += 64) {
            const int kk = min(64, K - kc);
            int cnt = 0, fst = 0;
            if (lane < kk) {
                const int S = src[k0 + kc + lane];
                cnt = c.count[S];
                fst = c.first[S];
                if (leaf_far(c, S, cnt, tx, ty, tz, g0, ng)) cnt = 0;
                else if (cnt > 0) qnear += c.mult[(size_t)S * ew + 1] * (4.0 * M_PI);
            }
            // inclusive wave scan of the counts left for direct summation
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
                        tile[j * 64 + lane] = make_double4(sx[i], sy[i], sz[i], sq[i]);
                    }
                }
                __syncthreads();
                for (int t = 0; t < ng; ++t) {
                    const int it = g0 + t;
                    const double ax = tx[it], ay = ty[it], az = tz[it];
                    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
                    for (int j = lane; j < tn; j += 64) {
                        const double4 sp = tile[j];
                        const double dx = ax - sp.x, dy = ay - sp.y, dz = az - sp.z;
                        const bool coinc = (dx == 0.0) & (dy == 0.0) & (dz == 0.0);
                        const double r2 = coinc ? 1.0 : dx * dx + dy * dy + dz * dz;
                        const double lg = coinc ? kLog4 : log_f64(r2);
                        const double wi = sp.w * recip(r2);
                        p0 = fma(sp.w, lg, p0);
                        p1 = fma(wi, dx, p1);
                        p2 = fma(wi, dy, p2);
                        p3 = fma(wi, dz, p3);
                    }
                    p0 = wave_sum(p0);
                    p1 = wave_sum(p1);
                    p2 = wave_sum(p2);
                    p3 = wave_sum(p3);
                    if (lane == t) {
                        own0 += p0;
                        own1 += p1;
                        own2 += p2;
                        own3 += p3;
                    }
                }
            }
        }
        const double qn = wave_sum(qnear);
        if (lane < ng) {
            const int my = g0 + lane;
            const double mx = tx[my], myy = ty[my], mz = tz[my];
            const int64_t o = tperm[my];
            psi[o] += (own0 + (1.0 - kLog4) * qn) * kInv4Pi;
            const double il = 1.0 / sqrt(mx * mx + myy * myy + mz * mz);
            const double ux = mx * il, uy = myy * il, uz = mz * il;
            const double vr = ux * own1 + uy * own2 + uz * own3;
            defl[o] += (own1 - ux * vr) * kInv2Pi;
            defl[m_out + o] += (own2 - uy * vr) * kInv2Pi;
            defl[2 * m_out + o] += (own3 - uz * vr) * kInv2Pi;
        }
    }
}

// Close leaves taken by their multipole expansion (Lemma 1).  The far leaves
// of a 64-entry chunk are compacted into LDS; the lanes split into ng groups
// of L (L the largest power of two <= 64/ng), group t evaluating every
// L-th far leaf at target t; a butterfly over the group sums them, and the
// group's first lane adds the sum to target t's slot (one writer per slot,
// fixed order: bitwise reproducible).
__global__ void __launch_bounds__(64) k_m2p(FmmCtx c, const int* __restrict__ tleaves, int ntl,
                                           const int* __restrict__ off, const int* __restrict__ src,
                                           const int* __restrict__ tfirst, const int* __restrict__ tcount,
                                           const double* __restrict__ tx, const double* __restrict__ ty,
                                           const double* __restrict__ tz, const uint32_t* __restrict__ tperm,
                                           double* __restrict__ psi, double* __restrict__ defl, int64_t m_out) {
    __shared__ int far_s[64];
    __shared__ double sums[64][4];
    const int lane = threadIdx.x;
    const int T = tleaves[blockIdx.x];
    const int k0 = off[T], K = off[T + 1] - k0;
    const int t0 = tfirst[T], nt = tcount[T];
    const int ew = 2 * c.p + 2;
    for (int tg = 0; tg < nt; tg += 64) {
        const int ng = min(64, nt - tg);
        const int g0 = t0 + tg;
        int L = 1;
        while (L * 2 * ng <= 64) L *= 2;
        const int gt = lane / L, sub = lane % L;  // target of this lane's group, rank in the group
        const bool active = gt < ng;
        const int my = g0 + (active ? gt : 0);
        const double mx = tx[my], myy = ty[my], mz = tz[my];
        sums[lane][0] = sums[lane][1] = sums[lane][2] = sums[lane][3] = 0.0;
        bool any = false;
        for (int kc = 0; kc < K; kc += 64) {
            const int kk = min(64, K - kc);
            int S = -1;
            bool far = false;
            if (lane < kk) {
                S = src[k0 + kc + lane];
                far = leaf_far(c, S, c.count[S], tx, ty, tz, g0, ng);
            }
            const uint64_t fm = __ballot(far);
            if (fm == 0) continue;
            any = true;
            const int nfar = __popcll(fm);
            __syncthreads();  // previous chunk's far list fully read
            if (far) far_s[__popcll(fm & ((1ULL << lane) - 1))] = S;
            __syncthreads();
            double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
            if (active) {
                for (int e = sub; e < nfar; e += L) {
                    const int Se = far_s[e];
                    const double* cs = c.cen + 4 * (size_t)Se;
                    const Frame fs = make_frame(cs[0], cs[1], cs[2]);
                    double ps, ax, ay, az;
                    m2p_eval(c.mult + (size_t)Se * ew, c.p, fs, cs[3], mx, myy, mz, &ps, &ax, &ay, &az);
                    p0 += ps;
                    p1 += ax;
                    p2 += ay;
                    p3 += az;
                }
            }
            for (int o = L >> 1; o > 0; o >>= 1) {
                p0 += __shfl_xor(p0, o, 64);
                p1 += __shfl_xor(p1, o, 64);
                p2 += __shfl_xor(p2, o, 64);
                p3 += __shfl_xor(p3, o, 64);
            }
            if (active && sub == 0) {
                sums[gt][0] += p0;
                sums[gt][1] += p1;
                sums[gt][2] += p2;
                sums[gt][3] += p3;
            }
        }
        __syncthreads();
        if (any && lane < ng) {
            const int64_t o = tperm[g0 + lane];
            psi[o] += sums[lane][0];
            defl[o] += sums[lane][1];
            defl[m_out + o] += sums[lane][2];
            defl[2 * m_out + o] += sums[lane][3];
        }
        __syncthreads();
    }
}

// Work actually done by the two kernels above, per target leaf: particle-
// target pairs summed directly and (target, leaf) multipole evaluations.
// Same grouping and the same far test, one lane per target leaf.
__global__ void k_near_work(FmmCtx c, const int* __restrict__ tleaves, int ntl, const int* __restrict__ off,
                            const int* __restrict__ src, const int* __restrict__ tfirst,
                            const int* __restrict__ tcount, const double* __restrict__ tx,
                            const double* __restrict__ ty, const double* __restrict__ tz, long long* pairs,
                            long long* evals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntl) return;
    const int T = tleaves[i];
    long long np = 0, ne = 0;
    for (int tg = 0; tg < tcount[T]; tg += 64) {
        const int ng = min(64, tcount[T] - tg);
        const int g0 = tfirst[T] + tg;
        for (int k = off[T]; k < off[T + 1]; ++k) {
            const int S = src[k];
            const int cnt = c.count[S];
            if (leaf_far(c, S, cnt, tx, ty, tz, g0, ng)) ne += ng;
            else np += (long long)ng * cnt;
        }
    }
    pairs[i] = np;
    evals[i] = ne;
}

void near_work(const FmmCtx& c, const int* tleaves, int ntl, const int* off, const int* src, const int* tfirst,
               const int* tcount, const double* tx, const double* ty, const double* tz, long long* pairs,
               long long* evals, hipStream_t s) {
    if (ntl <= 0) return;
    k_near_work<<<(unsigned)((ntl + 127) / 128), 128, 0, s>>>(c, tleaves, ntl, off, src, tfirst, tcount, tx, ty,
                                                              tz, pairs, evals);
    SFMM_LAUNCH_CHECK();
}

void fmm_p2p(const FmmCtx& c, const int* tleaves, int ntl, const int* off, const int* src, const int* tfirst,
             const int* tcount, const double* tx, const double* ty, const double* tz, const uint32_t* tperm,
             double* psi, double* defl, int64_t m_out, hipStream_t s) {
    if (ntl <= 0) return;
    k_p2p<<<(unsigned)ntl, 64, 0, s>>>(c, tleaves, ntl, off, src, tfirst, tcount, tx, ty, tz, tperm, psi, defl,
                                       m_out);
    SFMM_LAUNCH_CHECK();
}

void fmm_m2p(const FmmCtx& c, const int* tleaves, int ntl, const int* off, const int* src, const int* tfirst,
             const int* tcount, const double* tx, const double* ty, const double* tz, const uint32_t* tperm,
             double* psi, double* defl, int64_t m_out, hipStream_t s) {
    if (ntl <= 0 || c.p < kM2PMinOrder) return;
    k_m2p<<<(unsigned)ntl, 64, 0, s>>>(c, tleaves, ntl, off, src, tfirst, tcount, tx, ty, tz, tperm, psi, defl,
                                       m_out);
    SFMM_LAUNCH_CHECK();
}

}  // namespace sfmm
