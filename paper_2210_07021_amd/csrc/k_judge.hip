// The judge of the per-pair order policies: the direct sum of Eq. SUM and
// Eq. ALP_PSI (the paper's "PPM" of Sec. 4.1) at a seeded subset of the
// targets, over every source, on the GPU.  The bound and learned policies
// pick each FMM act's order from a criterion that only estimates its error;
// after an execute with either, the library compares its output at these
// targets with the direct sum and falls back to the fixed order when the
// relative L2 error of psi or alpha exceeds the tolerance.
//
// Layout: each workgroup takes a chunk of kJudgeChunk sorted sources, staged
// through LDS 256 at a time; a target is owned by `lanes` threads (256 over
// the targets per pass, at least 4) that split the chunk's sources; per chunk
// and target the four sums (psi, alpha x, y, z) are Neumaier-compensated,
// combined over the lanes, and written as (sum, compensation) pairs.  A
// second kernel adds the chunks in double-double in a fixed order, so the
// result is exact to rounding of the final sum and bitwise reproducible.  The
// log and reciprocal are the pair loop's table-driven ones (log_recip_tab: a
// few 1e-16 absolute, the reciprocal correctly rounded on every input
// measured), far below the tolerances the judge checks.
#include "common.hpp"
#include "expand.hpp"

namespace sfmm {

namespace {
constexpr int kJudgeThreads = 256;
constexpr int kJudgeChunk = 4096;

__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
}

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// part [nchunk][S][8]: (psi, c, ax, c, ay, c, az, c) of chunk j for target t.
// Thread (target t, lane r of `lanes`) takes sources r, r + lanes, ... of the
// chunk, so all threads work whatever S; the lanes' compensated sums of a
// target are then combined in lane order (deterministic).
__global__ void __launch_bounds__(kJudgeThreads) k_judge_chunks(const double4* __restrict__ spt, int n,
                                                                 const double4* __restrict__ tsel, int S,
                                                                 int lanes, LogPoly lk, double* __restrict__ part) {
    __shared__ double4 tile[kJudgeThreads];
    __shared__ double red[kJudgeThreads][8];
    __shared__ double2 ltab[kLogTab];
    for (int j = threadIdx.x; j < kLogTab; j += kJudgeThreads) ltab[j] = log_tab_entry(j);
    const int tpb = kJudgeThreads / lanes;  // targets per pass
    const int j = blockIdx.x;
    const int s0 = j * kJudgeChunk, s1 = min(n, s0 + kJudgeChunk);
    const int tl = threadIdx.x / lanes, r = threadIdx.x % lanes;
    for (int t0 = 0; t0 < S; t0 += tpb) {
        const int t = t0 + tl;
        const double4 tp = t < S ? tsel[t] : make_double4(1.0, 0.0, 0.0, 0.0);
        double sp = 0, cp = 0, sx = 0, cx = 0, sy = 0, cy = 0, sz = 0, cz = 0;
        for (int b = s0; b < s1; b += kJudgeThreads) {
            __syncthreads();
            if (b + threadIdx.x < s1) tile[threadIdx.x] = spt[b + threadIdx.x];
            __syncthreads();
            const int nb = min(kJudgeThreads, s1 - b);
            for (int k = r; k < nb; k += lanes) {
                const double4 sr = tile[k];
                const double dx = tp.x - sr.x, dy = tp.y - sr.y, dz = tp.z - sr.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) continue;  // a source at the target itself is left out
                double lg, inv;  // log(r2 / 4) and 4 / r2
                log_recip_tab(0.25 * r2, ltab, lk, &lg, &inv);
                neumaier(sp, cp, sr.w * kInv4Pi * lg);
                const double f = sr.w * (0.25 * kInv2Pi) * inv;
                neumaier(sx, cx, f * dx);
                neumaier(sy, cy, f * dy);
                neumaier(sz, cz, f * dz);
            }
        }
        double* my = red[threadIdx.x];
        my[0] = sp; my[1] = cp; my[2] = sx; my[3] = cx;
        my[4] = sy; my[5] = cy; my[6] = sz; my[7] = cz;
        __syncthreads();
        if (r == 0 && t < S) {
            double o[8];
            for (int q = 0; q < 4; ++q) {  // lane 0's sum, then lanes 1.. added in order (two-sum)
                double hi = red[threadIdx.x][2 * q], lo = red[threadIdx.x][2 * q + 1];
                for (int l = 1; l < lanes; ++l) {
                    double sum, e;
                    two_sum(hi, red[threadIdx.x + l][2 * q], sum, e);
                    lo += e + red[threadIdx.x + l][2 * q + 1];
                    hi = sum;
                }
                o[2 * q] = hi;
                o[2 * q + 1] = lo;
            }
            double* out = part + ((size_t)j * S + t) * 8;
            for (int q = 0; q < 8; ++q) out[q] = o[q];
        }
    }
}

// out [S][4]: psi (+ shift) and the tangent projection of alpha, from the
// chunk sums in double-double: one 64-lane workgroup per target, lane l
// adding chunks l, l + 64, ... in order, then the lanes' double-double sums
// combined in a fixed butterfly order (bitwise reproducible).
__device__ __forceinline__ void dd_add_into(double& hi, double& lo, double h2, double l2) {
    double s, e;
    two_sum(hi, h2, s, e);
    lo += e + l2;
    hi = s;
}

__global__ void __launch_bounds__(64) k_judge_finish(const double* __restrict__ part, int nchunk,
                                                     const double4* __restrict__ tsel, int S, double shift,
                                                     double* __restrict__ out) {
    const int t = blockIdx.x, lane = threadIdx.x;
    double hi[4] = {0, 0, 0, 0}, lo[4] = {0, 0, 0, 0};
    for (int j = lane; j < nchunk; j += 64) {
        const double* o = part + ((size_t)j * S + t) * 8;
        for (int k = 0; k < 4; ++k) dd_add_into(hi[k], lo[k], o[2 * k], o[2 * k + 1]);
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1)
        for (int k = 0; k < 4; ++k) {
            const double h2 = __shfl_xor(hi[k], m, 64), l2 = __shfl_xor(lo[k], m, 64);
            // both lanes of a pair add the same two values in the same order
            double a = hi[k], b = lo[k], c2 = h2, d2 = l2;
            if (lane & m) {
                a = h2;
                b = l2;
                c2 = hi[k];
                d2 = lo[k];
            }
            dd_add_into(a, b, c2, d2);
            hi[k] = a;
            lo[k] = b;
        }
    if (lane != 0) return;
    double v[4];
    for (int k = 0; k < 4; ++k) v[k] = hi[k] + lo[k];
    const double4 tp = tsel[t];
    const double nd = tp.x * v[1] + tp.y * v[2] + tp.z * v[3];
    out[4 * t + 0] = v[0] + shift;
    out[4 * t + 1] = v[1] - nd * tp.x;
    out[4 * t + 2] = v[2] - nd * tp.y;
    out[4 * t + 3] = v[3] - nd * tp.z;
}

// The subset: caller-order target positions pos[k] -> their coordinates,
// unit vectors exactly as the plan makes them (renormalised when off the
// sphere by more than 1e-14)
__global__ void k_judge_gather_tgt(const int* __restrict__ pos, int S, const double* __restrict__ tgt, int64_t m,
                                   double4* __restrict__ tsel) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S) return;
    const int64_t j = pos[k];
    double a = tgt[j], b = tgt[m + j], c = tgt[2 * m + j];
    const double r2 = a * a + b * b + c * c;
    if (fabs(r2 - 1.0) > 1e-14) {
        const double inv = 1.0 / sqrt(r2);
        a *= inv;
        b *= inv;
        c *= inv;
    }
    tsel[k] = make_double4(a, b, c, 0.0);
}

// the library's outputs (caller order) at the subset
__global__ void k_judge_gather_out(const int* __restrict__ pos, int S, const double* __restrict__ psi,
                                   const double* __restrict__ defl, int64_t m, double* __restrict__ got) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S) return;
    const int64_t i = pos[k];
    got[4 * k + 0] = psi[i];
    got[4 * k + 1] = defl[i];
    got[4 * k + 2] = defl[m + i];
    got[4 * k + 3] = defl[2 * m + i];
}
}  // namespace

size_t judge_part_doubles(int64_t n, int S) {
    const int64_t nchunk = (n + kJudgeChunk - 1) / kJudgeChunk;
    return (size_t)std::max<int64_t>(nchunk, 1) * (size_t)S * 8;
}

void judge_targets(const int* pos, int S, const double* tgt, int64_t m, double4* tsel, hipStream_t s) {
    if (S <= 0) return;
    k_judge_gather_tgt<<<(S + 255) / 256, 256, 0, s>>>(pos, S, tgt, m, tsel);
    SFMM_LAUNCH_CHECK();
}

void judge_sum(const double4* spt, int64_t n, const double4* tsel, int S, double* part, hipStream_t s) {
    if (S <= 0) return;
    if (n <= 0) {
        fill_f64(part, (size_t)S * 8, 0.0, s);
        return;
    }
    const int nchunk = (int)((n + kJudgeChunk - 1) / kJudgeChunk);
    int tpb = 64;  // targets per pass: the smallest power of two >= S, at most 64
    while (tpb > 1 && tpb / 2 >= S) tpb /= 2;
    k_judge_chunks<<<nchunk, kJudgeThreads, 0, s>>>(spt, (int)n, tsel, S, kJudgeThreads / tpb, kLogPoly, part);
    SFMM_LAUNCH_CHECK();
}

void judge_outputs(const int* pos, int S, const double4* tsel, const double* part, int64_t n, double shift,
                   const double* psi, const double* defl, int64_t m, double* ref, double* got, hipStream_t s) {
    if (S <= 0) return;
    k_judge_gather_out<<<(S + 255) / 256, 256, 0, s>>>(pos, S, psi, defl, m, got);
    SFMM_LAUNCH_CHECK();
    const int nchunk = (int)std::max<int64_t>((n + kJudgeChunk - 1) / kJudgeChunk, 1);
    k_judge_finish<<<S, 64, 0, s>>>(part, nchunk, tsel, S, shift, ref);
    SFMM_LAUNCH_CHECK();
}

}  // namespace sfmm
