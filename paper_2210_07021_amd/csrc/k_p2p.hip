// Near field (the direct acts of Sec. 3.3-3.4): for every target in a leaf,
// the sum of the Green's function and its tangent gradient over the particles
// of the leaf's close boxes.
//
// One 64-wide wavefront owns one target leaf.  The close boxes' particle
// ranges are concatenated into one flat index space (wave prefix sum of
// their counts, binary search by lane shuffles), so every lane holds real
// work however small the leaves are.  Each lane keeps U particles in
// registers and applies them to TB targets at a time; the per-target partial
// sums are reduced across the wave by butterfly shuffles at the end.  No
// floating-point atomics: the result is bitwise reproducible.
//
// Per pair, with d = n_t - n_s:
//   psi   += (q/4pi) (log(|d|^2/4) + 1)      (Eq. GRE_FUN + zero-mean share)
//   alpha += (q/2pi) d/|d|^2                 (projected on the tangent plane
//                                             once per target)
// and a particle at exactly the target position keeps only its q/(4pi).
//
// A close leaf S whose centre is more than 3 R_S from every target of the
// current chunk is not summed particle by particle: its own multipole
// expansion (Lemma 1) is evaluated at those targets instead.  By Eq. MUL_ERR
// the truncation error there is below (Q~/2pi) x^(p+1)/((p+1)(1-x)) with
// x ~ 1/3, i.e. under 1e-15 Q~ for p >= 28; this is done only for p >= 12
// and for leaves holding at least p/4 + 2 particles (below that the direct
// sum is cheaper).
// Big leaves of sparse regions next to dense clumps are where it matters:
// their targets otherwise meet every particle of the clump directly.
#include "common.hpp"
#include "expand.hpp"

namespace sfmm {

constexpr int kTB = 8;  // targets per pass
constexpr int kU = 4;   // particles per lane per tile

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// 1/x for x > 0 normal: hardware estimate, two Newton steps (full precision)
__device__ __forceinline__ double rcp_f64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

constexpr int kM2PMinOrder = 12;
constexpr double kM2PRatio = 3.0;  // target beyond 3 R_S from the leaf centre

__global__ void __launch_bounds__(256) k_p2p(FmmCtx c, const int* tleaves, int ntl, const int* off, const int* src,
                                            const int* tfirst, const int* tcount, const double* tx,
                                            const double* ty, const double* tz, const uint32_t* tperm,
                                            double* psi, double* defl, int64_t m_out) {
    const int wv = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (wv >= ntl) return;  // uniform per wave
    const int T = tleaves[wv];
    const int k0 = off[T], K = off[T + 1] - k0;
    const int t0 = tfirst[T], nt = tcount[T];
    const bool use_m2p = c.p >= kM2PMinOrder;
    const int ew = 2 * c.p + 2;

    for (int tb = 0; tb < nt; tb += kTB) {
        const int ntb = min(kTB, nt - tb);
        double acc[kTB][6];
#pragma unroll
        for (int t = 0; t < kTB; ++t)
#pragma unroll
            for (int v = 0; v < 6; ++v) acc[t][v] = 0.0;
        double txs[kTB], tys[kTB], tzs[kTB];
#pragma unroll
        for (int t = 0; t < kTB; ++t) {
            const int it = t0 + tb + min(t, ntb - 1);
            txs[t] = tx[it];
            tys[t] = ty[it];
            tzs[t] = tz[it];
        }
        for (int kc = 0; kc < K; kc += 64) {
            const int kk = min(64, K - kc);
            int cnt = 0, fst = 0, S = -1;
            bool far = false;
            if (lane < kk) {
                S = src[k0 + kc + lane];
                cnt = c.count[S];
                fst = c.first[S];
                // the expansion costs ~p/4 direct pairs: only worth it for fuller leaves
                if (use_m2p && 4 * cnt >= c.p + 8) {
                    // far from every target of the chunk: chord > 2 sin(3R/2)
                    const double a = kM2PRatio * c.rad[S];
                    if (a < 3.0) {
                        const double h = 2.0 * sin(0.5 * a);
                        const double thr = h * h;
                        const double* cs = c.cen + 4 * (size_t)S;
                        far = true;
                        for (int t = 0; t < ntb; ++t) {
                            const double dx = txs[t] - cs[0], dy = tys[t] - cs[1], dz = tzs[t] - cs[2];
                            far = far && (dx * dx + dy * dy + dz * dz > thr);
                        }
                    }
                }
            }
            if (far) {
                // multipole of S at each target of the chunk
                const double* cs = c.cen + 4 * (size_t)S;
                const Frame fs = make_frame(cs[0], cs[1], cs[2]);
                const double* e = c.mult + (size_t)S * ew;
                for (int t = 0; t < ntb; ++t) {
                    double ps, ax, ay, az;
                    m2p_eval(e, c.p, fs, cs[3], txs[t], tys[t], tzs[t], &ps, &ax, &ay, &az);
#pragma unroll
                    for (int tt = 0; tt < kTB; ++tt) {
                        if (tt == t) {
                            acc[tt][0] += ps * (4.0 * M_PI);
                            acc[tt][3] += ax * (2.0 * M_PI);
                            acc[tt][4] += ay * (2.0 * M_PI);
                            acc[tt][5] += az * (2.0 * M_PI);
                        }
                    }
                }
                cnt = 0;
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
            for (int f0 = 0; f0 < total; f0 += 64 * kU) {
                double px[kU], py[kU], pz[kU], pq[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int f = f0 + u * 64 + lane;
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
                        px[u] = c.sx[i];
                        py[u] = c.sy[i];
                        pz[u] = c.sz[i];
                        pq[u] = c.sq[i];
                    } else {
                        px[u] = 0.0;
                        py[u] = 0.0;
                        pz[u] = 0.0;
                        pq[u] = 0.0;
                    }
                }
#pragma unroll
                for (int t = 0; t < kTB; ++t) {
                    if (t >= ntb) break;
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        const double dx = txs[t] - px[u], dy = tys[t] - py[u], dz = tzs[t] - pz[u];
                        const bool coinc = (dx == 0.0) && (dy == 0.0) && (dz == 0.0);
                        const double r2 = coinc ? 1.0 : dx * dx + dy * dy + dz * dz;
                        const double w = coinc ? 0.0 : pq[u];
                        const double lg = log(r2);
                        const double wi = w * rcp_f64(r2);
                        acc[t][0] = fma(w, lg, acc[t][0]);
                        acc[t][1] += w;
                        acc[t][2] += coinc ? pq[u] : 0.0;
                        acc[t][3] = fma(wi, dx, acc[t][3]);
                        acc[t][4] = fma(wi, dy, acc[t][4]);
                        acc[t][5] = fma(wi, dz, acc[t][5]);
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < kTB; ++t) {
            if (t >= ntb) break;
            double v[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) v[k] = wave_sum(acc[t][k]);
            if (lane == t) {
                const int it = t0 + tb + t;
                const int64_t o = tperm[it];
                psi[o] += (v[0] + (1.0 - kLog4) * v[1] + v[2]) * kInv4Pi;
                const double nx = txs[t], ny = tys[t], nz = tzs[t];
                const double il = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
                const double ux = nx * il, uy = ny * il, uz = nz * il;
                const double vr = ux * v[3] + uy * v[4] + uz * v[5];
                defl[o] += (v[3] - ux * vr) * kInv2Pi;
                defl[m_out + o] += (v[4] - uy * vr) * kInv2Pi;
                defl[2 * m_out + o] += (v[5] - uz * vr) * kInv2Pi;
            }
        }
    }
}

void fmm_p2p(const FmmCtx& c, const int* tleaves, int ntl, const int* off, const int* src, const int* tfirst,
             const int* tcount, const double* tx, const double* ty, const double* tz, const uint32_t* tperm,
             double* psi, double* defl, int64_t m_out, hipStream_t s) {
    if (ntl <= 0) return;
    const unsigned blocks = (unsigned)((ntl + 3) / 4);
    k_p2p<<<blocks, 256, 0, s>>>(c, tleaves, ntl, off, src, tfirst, tcount, tx, ty, tz, tperm, psi, defl, m_out);
    SFMM_LAUNCH_CHECK();
}

}  // namespace sfmm
