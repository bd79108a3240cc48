// Per-interaction truncation order for the FMM acts (Lemma 3).
//
// The plan order p (from the tolerance) is what the worst pair needs.  A
// pair whose boxes are well separated converges faster: with the factorised
// translation of k_m2l its terms fall like x^n, x = a + b (a = rho_T cot(T/2),
// b = rho_S cot(T/2); exactly antipodal centres, where a = b = 0, converge
// like g^n, g = rho_T rho_S: x = max(a + b, sqrt g)).  A pair at order p' < p
// keeps its monopole part exact
// (the -(Q/l) a^l terms of the local coefficients for every l <= p, added by
// k_m2l_qtail: on smooth skies these large terms cancel between pairs, so
// they must not be cut) and truncates the multipole part: the source's
// A_1..A_p' in, the local coefficients up to p' out.  Its error is of the
// order of
//     W_S x^(p'+1) (p'+1) / (1 - x),   W_S = sum_l |Ah_l| (scaled multipole),
// the shape of Eq. MUL_ERR with W_S in place of Q~ and the extra p'+1 of a
// gradient.  Two policies pick p' per pair from the criterion
// e(p') <= kappa tol W_S:
//   * bound:   the smallest p' (multiple of kOrderStep) whose bound above
//              meets it;
//   * learned: a 3 x 64 MLP that maps per-pair features to p', trained on
//              labels that the FP64 translation itself produces: the exact
//              e(p') = sum_l l |A'_l(p) - A'_l(p')| over the local
//              coefficients (scaled by rho_T^l) of the pair.
// Pairs are then split per target box into one list per order (a stable
// counting split), and the M2L runs once per order over its lists, adding
// into the local records.
#include "common.hpp"
#include "expand.hpp"

namespace sfmm {

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1); }

// ------------------------------------------------------------ features
// log10 |A_l| / |Q| of a source multipole at l = 1, 4, 8, 16 (scaled
// coefficients; orders above p repeat the last one), clamped to [-40, 5]
__global__ void k_box_decay(const double* __restrict__ mult, int p, int nb, float4* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const double* e = mult + (size_t)b * (2 * p + 2);
    const double q = fabs(e[1]) + 1e-300;
    float v[4];
    const int ls[4] = {1, 4, 8, 16};
    for (int k = 0; k < 4; ++k) {
        const int l = ls[k] < p ? ls[k] : p;
        const double m = sqrt(e[2 * l] * e[2 * l] + e[2 * l + 1] * e[2 * l + 1]);
        double lg = log10(m / q + 1e-40);
        lg = lg < -40.0 ? -40.0 : (lg > 5.0 ? 5.0 : lg);
        v[k] = (float)lg;
    }
    out[b] = make_float4(v[0], v[1], v[2], v[3]);
}

// Shift parameters a, b of the pair's factorised Lemma 3 and its convergence
// ratio x = max(a + b, sqrt(g)): the terms of the translated coefficients
// fall like (a + b)^n, and like g^n through the diagonal, which alone is
// left for exactly antipodal centres (a = b = 0, g = rho_T rho_S); for any
// other pair sqrt(g) <= (a + b) / 2.  Same formulas as trans_geom<kM2L>,
// without the phases and the log.
__device__ __forceinline__ double pair_ratio(const FmmCtx& c, int t, int s, double* a, double* b) {
    const double* ct = c.cen + 4 * (size_t)t;
    const double* cs = c.cen + 4 * (size_t)s;
    const double dx = ct[0] - cs[0], dy = ct[1] - cs[1], dz = ct[2] - cs[2];
    const double sx = ct[0] + cs[0], sy = ct[1] + cs[1], sz = ct[2] + cs[2];
    const double dif2 = dx * dx + dy * dy + dz * dz, sum2 = sx * sx + sy * sy + sz * sz;
    const double cc = sum2 < 1e-24 ? 0.0 : sqrt(sum2 / dif2);  // cot(T/2); 0 for antipodes
    *a = cc * ct[3];
    *b = cc * cs[3];
    const double g = ct[3] * cs[3] * (1.0 + cc * cc);
    return fmax(*a + *b, sqrt(g));
}

// Features of pair k (target ent_t[k], source src[k]), kMlpIn floats:
// x, a/x, log10(kappa tol)/16, the source's four decay values / 8, level_T / 29
__device__ __forceinline__ void pair_feature_vec(const FmmCtx& c, int t, int s, const float4* __restrict__ decay,
                                                 float ltol, float* f) {
    double a, b;
    const double x = pair_ratio(c, t, s, &a, &b);
    const float4 d = decay[s];
    f[0] = (float)x;
    f[1] = a + b > 0.0 ? (float)(a / (a + b)) : 0.5f;  // a + b = 0: exactly antipodal base pixels
    f[2] = ltol / 16.0f;
    f[3] = d.x / 8.0f;
    f[4] = d.y / 8.0f;
    f[5] = d.z / 8.0f;
    f[6] = d.w / 8.0f;
    f[7] = (float)c.level[t] / 29.0f;
}

__global__ void k_pair_features(FmmCtx c, const int* __restrict__ ent_t, const int* __restrict__ src,
                                const int* __restrict__ idx, int64_t n, const float4* __restrict__ decay,
                                float ltol, float* __restrict__ feat) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k = idx ? idx[i] : i;
    pair_feature_vec(c, ent_t[k], src[k], decay, ltol, feat + i * kMlpIn);
}

// ------------------------------------------------------------ bound policy
__device__ __forceinline__ int round_order(int p, int pmax) {
    int q = ((p + kOrderStep - 1) / kOrderStep) * kOrderStep;
    q = q < kOrderStep ? kOrderStep : q;
    return q > pmax ? pmax : q;
}

__global__ void k_order_bound(FmmCtx c, const int* __restrict__ ent_t, const int* __restrict__ src, int np,
                              double eps, int pmax, uint8_t* __restrict__ ord) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    double a, b;
    const double x = pair_ratio(c, ent_t[k], src[k], &a, &b);
    int p = pmax;
    if (x < 1.0) {
        double xp = x;  // x^(q+1) for q = 0, 1, ...
        for (int q = 1; q <= pmax; ++q) {
            xp *= x;
            if (xp * (q + 1) / (1.0 - x) <= eps) {
                p = q;
                break;
            }
        }
    }
    ord[k] = (uint8_t)round_order(p, pmax);
}

// ------------------------------------------------------------ learned policy
// MLP: h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3, with
// the weights in one array (layout in sfmm.h).  Inference rounds weights,
// inputs and hidden activations to bfloat16 (the network's storage format)
// and accumulates in FP32.
__device__ __forceinline__ float bf16_round(float v) {
    // round to nearest even (v_cvt_pk_bf16_f32 on gfx950) and back
    return (float)(__bf16)v;
}

// The network runs on the bf16 matrix cores (v_mfma_f32_32x32x8bf16_1k,
// D[32x32] += A[32x8] B[8x32], FP32 accumulate), one wave per tile of 32
// pairs, activations kept transposed ([hidden unit][pair]):
//   * A operands are weights (rows = output units, k = input units): lane l
//     holds A[l % 32][4 (l / 32) + r], r = 0..3;
//   * B operands are activations (k = input units, columns = pairs): lane l
//     holds B[4 (l / 32) + r][l % 32];
//   * D: lane l holds D[8 g + 4 (l / 32) + r][l % 32] in element 4 g + r.
// So the D fragment of a 32-unit block of layer 1 is, group g by group g,
// exactly the B operand of layer 2's k-step covering units 8 g .. 8 g + 7 of
// that block: no data moves between the layers.  Layer 3 is a dot product
// over the 32 units a lane holds, completed with its partner lane l ^ 32.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short bf16_bits(float v) { return __builtin_bit_cast(short, (__bf16)v); }

__global__ void __launch_bounds__(256) k_order_mlp(FmmCtx c, const int* __restrict__ ent_t,
                                                   const int* __restrict__ src, const float4* __restrict__ decay,
                                                   float ltol, const float* __restrict__ feat, int64_t n,
                                                   const float* __restrict__ w, int pmax, float margin,
                                                   uint8_t* __restrict__ ord, float* __restrict__ yout) {
    constexpr int H = kMlpHidden, I = kMlpIn;
    const float* W1 = w;
    const float* B1 = W1 + H * I;
    const float* W2 = B1 + H;
    const float* B2 = W2 + H * H;
    const float* W3 = B2 + H;
    __shared__ float sb1[H], sb2[H], sw3[H + 1];
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        sb1[i] = bf16_round(B1[i]);
        sb2[i] = bf16_round(B2[i]);
        sw3[i] = bf16_round(W3[i]);
    }
    if (threadIdx.x == 0) sw3[H] = bf16_round(W3[H]);
    __syncthreads();
    const int lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
    // weight fragments, held for every tile of this wave
    bf16x4 a1[2], a2[2][8];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) a1[rb][r] = bf16_bits(W1[(32 * rb + col) * I + 4 * half + r]);
#pragma unroll
    for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int st = 0; st < 8; ++st)
#pragma unroll
            for (int r = 0; r < 4; ++r) a2[ob][st][r] = bf16_bits(W2[(32 * ob + col) * H + 8 * st + 4 * half + r]);
    // 64 pairs per wave and step: lane l computes the features of pair l of
    // the step once, and the two tiles of 32 pairs take the halves they lack
    // from the partner lane l ^ 32
    const int64_t nsteps = (n + 63) / 64;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t step = wave; step < nsteps; step += nwaves) {
        float f[I];
        {
            const int64_t k = step * 64 + lane;
            if (k < n) {
                if (feat) {
#pragma unroll
                    for (int j = 0; j < I; ++j) f[j] = feat[k * I + j];
                } else {
                    pair_feature_vec(c, ent_t[k], src[k], decay, ltol, f);
                }
            } else {
#pragma unroll
                for (int j = 0; j < I; ++j) f[j] = 0.0f;
            }
        }
        float fx[I];
#pragma unroll
        for (int j = 0; j < I; ++j) fx[j] = __shfl_xor(f[j], 32, 64);
#pragma unroll
        for (int tile = 0; tile < 2; ++tile) {
            // B operand of the tile: lane (col, half) holds inputs 4 half ..
            // 4 half + 3 of pair 32 tile + col (own when half == tile)
            bf16x4 b0;
#pragma unroll
            for (int r = 0; r < 4; ++r) b0[r] = bf16_bits(half == tile ? f[4 * half + r] : fx[4 * half + r]);
            // layer 1 -> layer 2 operands
            bf16x4 b1[8];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                f32x16 d = {};
                d = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[rb], b0, d, 0, 0, 0);
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float v = d[4 * g + r] + sb1[32 * rb + 8 * g + 4 * half + r];
                        b1[4 * rb + g][r] = bf16_bits(v > 0.0f ? v : 0.0f);
                    }
            }
            // layer 2, layer 3
            float y = 0.0f;
#pragma unroll
            for (int ob = 0; ob < 2; ++ob) {
                f32x16 d = {};
#pragma unroll
                for (int st = 0; st < 8; ++st)
                    d = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a2[ob][st], b1[st], d, 0, 0, 0);
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int u = 32 * ob + 8 * g + 4 * half + r;
                        const float v = d[4 * g + r] + sb2[u];
                        y = fmaf(sw3[u], bf16_round(v > 0.0f ? v : 0.0f), y);
                    }
            }
            y += __shfl_xor(y, 32, 64);
            y += sw3[H];
            const int64_t k = step * 64 + 32 * tile + col;
            if (half == tile && k < n) {
                if (yout) yout[k] = y;
                if (ord) {
                    const float pf = kOrderCenter + kOrderScale * y + margin;
                    const int p = pf >= (float)pmax ? pmax : (pf <= 1.0f ? 1 : (int)ceilf(pf));
                    ord[k] = (uint8_t)round_order(p, pmax);
                }
            }
        }
    }
}

// ------------------------------------------------------------ labels
// Lemma 3 at a run-time order pc: the multipole part from A_1..A_pc into
// the local coefficients 1..pc, the monopole part into all coefficients up
// to pmax (what the per-order passes plus k_m2l_qtail compute), in the same
// factorised arithmetic as translate_add; out has 2 pmax + 2 entries.
__device__ void translate_rt(const double* in, const TransGeom& G, int pc, int pmax, double* out) {
    double ar[kMaxOrder + 1], ai[kMaxOrder + 1];
    const double C = in[0], Q = in[1];
    ar[0] = ai[0] = 0.0;
    cplx pw = G.ph1;
    for (int l = 1; l <= pc; ++l) {
        const cplx v = cmul(pw, cplx{in[2 * l], in[2 * l + 1]});
        ar[l] = v.re;
        ai[l] = v.im;
        pw = cmul(pw, G.ph1);
    }
    for (int i = 0; i < pc; ++i)
        for (int j = pc - 1; j >= i; --j) {
            ar[j] = fma(G.b, ar[j + 1], ar[j]);
            ai[j] = fma(G.b, ai[j + 1], ai[j]);
        }
    const double u0 = ar[0];
    double gn = G.g;
    for (int l = 1; l <= pc; ++l) {
        ar[l] *= gn;
        ai[l] *= gn;
        gn *= G.g;
    }
    for (int i = pc - 2; i >= 0; --i)
        for (int j = i; j <= pc - 2; ++j) {
            ar[j + 2] = fma(G.a, ar[j + 1], ar[j + 2]);
            ai[j + 2] = fma(G.a, ai[j + 1], ai[j + 2]);
        }
    cplx pw2 = G.ph2;
    double an = G.a;
    for (int l = 1; l <= pmax; ++l) {
        const cplx v = {(l <= pc ? ar[l] : 0.0) - Q * (1.0 / l) * an, l <= pc ? ai[l] : 0.0};
        const cplx o = cmul(pw2, v);
        out[2 * l] = o.re;
        out[2 * l + 1] = o.im;
        pw2 = cmul(pw2, G.ph2);
        an *= G.a;
    }
    out[0] = C + Q * G.clog + 2.0 * u0;
    out[1] = Q;
}

// label[i] = smallest p' (multiple of kOrderStep, at most p) with
// sum_l l |A'_l(p) - A'_l(p')| <= eps W_S for pair idx[i]; scratch holds
// 2 (2p + 2) doubles per lane
__global__ void k_order_labels(FmmCtx c, const int* __restrict__ ent_t, const int* __restrict__ src,
                               const int* __restrict__ idx, int n, double eps, double* __restrict__ scratch,
                               float* __restrict__ label) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = idx[i];
    const int t = ent_t[k], s = src[k];
    const int p = c.p;
    const size_t ew = 2 * (size_t)p + 2;
    const double* ct = c.cen + 4 * (size_t)t;
    const double* cs = c.cen + 4 * (size_t)s;
    const Frame ft = make_frame(ct[0], ct[1], ct[2]);
    const Frame fs = make_frame(cs[0], cs[1], cs[2]);
    const TransGeom G = trans_geom<kM2L>(fs, cs[3], ft, ct[3]);
    const double* in = c.mult + (size_t)s * ew;
    double ws = 0.0;
    for (int l = 1; l <= p; ++l) ws += sqrt(in[2 * l] * in[2 * l] + in[2 * l + 1] * in[2 * l + 1]);
    double* full = scratch + (size_t)i * 2 * ew;
    double* tr = full + ew;
    translate_rt(in, G, p, p, full);
    const double lim = eps * ws;
    int best = p;
    for (int pc = kOrderStep; pc < p; pc += kOrderStep) {
        translate_rt(in, G, pc, p, tr);
        double e = 0.0;
        for (int l = 1; l <= p; ++l) {
            const double dr = full[2 * l] - tr[2 * l], di = full[2 * l + 1] - tr[2 * l + 1];
            e += l * sqrt(dr * dr + di * di);
        }
        if (e <= lim) {
            best = pc;
            break;
        }
    }
    label[i] = (float)best;
}

// Sum over the four lanes of a quad (lanes 4i .. 4i + 3), every lane getting
// (v0 + v1) + (v2 + v3): DPP quad permutations (all four lanes active).
template <int CTRL>
__device__ __forceinline__ double tail_dpp(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double tail_quad_sum(double v) {
    v += tail_dpp<0xB1>(v);        // lane ^ 1
    return v + tail_dpp<0x4E>(v);  // lane ^ 2
}

// The monopole part of the local coefficients above each pair's order:
// A'_l += e^(-i l phi_S^(T)) (-(Q/l) a^l) for ord < l <= p (c.p).  Four
// lanes per target box (lane r takes entries r, r + 4, ... of its list),
// their sums added across the quad in a fixed order and written by the lane
// that owns the entry (entry l by lane l mod 4), once per record.
template <int P>
__global__ void __launch_bounds__(128) k_m2l_qtail(FmmCtx c, const int* __restrict__ off,
                                                  const int* __restrict__ src, const uint8_t* __restrict__ ord,
                                                  int nbox) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = gid >> 2, r = gid & 3;
    if (t >= nbox) return;  // the four lanes of a box leave together
    const int k0 = off[t], k1 = off[t + 1];
    bool any = false;
    for (int k = k0 + r; k < k1; k += 4) any |= ord[k] < P;
    // every lane of the quad takes the same branch
    any = tail_quad_sum(any ? 1.0 : 0.0) > 0.0;
    if (!any) return;
    const double* ct = c.cen + 4 * (size_t)t;
    const Frame ft = make_frame(ct[0], ct[1], ct[2]);
    double acc[2 * P];
#pragma unroll
    for (int l = 0; l < 2 * P; ++l) acc[l] = 0.0;
    for (int k = k0 + r; k < k1; k += 4) {
        const int lo = ord[k];
        if (lo >= P) continue;
        const int s = src[k];
        const double* cs = c.cen + 4 * (size_t)s;
        // a = rho_T cot(T/2) and the output phase conj(e2) of trans_geom<kM2L>
        const double dx = ft.c[0] - cs[0], dy = ft.c[1] - cs[1], dz = ft.c[2] - cs[2];
        const double sx = ft.c[0] + cs[0], sy = ft.c[1] + cs[1], sz = ft.c[2] + cs[2];
        const double dif2 = dx * dx + dy * dy + dz * dz, sum2 = sx * sx + sy * sy + sz * sz;
        double u2, v2;
        if (sum2 < 1e-24) {
            const Frame fs = make_frame(cs[0], cs[1], cs[2]);
            u2 = fs.et[0] * ft.et[0] + fs.et[1] * ft.et[1] + fs.et[2] * ft.et[2];
            v2 = fs.et[0] * ft.ep[0] + fs.et[1] * ft.ep[1] + fs.et[2] * ft.ep[2];
        } else {
            u2 = -(dx * ft.et[0] + dy * ft.et[1] + dz * ft.et[2]);
            v2 = -(dx * ft.ep[0] + dy * ft.ep[1] + dz * ft.ep[2]);
        }
        const double r2 = 1.0 / sqrt(u2 * u2 + v2 * v2);
        const cplx ph2 = {u2 * r2, -v2 * r2};
        const double a = (sum2 < 1e-24 ? 0.0 : sqrt(sum2 / dif2)) * ct[3];
        const double Q = c.mult[(size_t)s * (2 * P + 2) + 1];
        cplx pw2 = ph2;
        double an = a;
#pragma unroll
        for (int l = 1; l <= P; ++l) {
            if (l > lo) {
                const double v = -Q * (1.0 / l) * an;
                acc[2 * l - 2] = fma(pw2.re, v, acc[2 * l - 2]);
                acc[2 * l - 1] = fma(pw2.im, v, acc[2 * l - 1]);
            }
            pw2 = cmul(pw2, ph2);
            an *= a;
        }
    }
    double* out = c.local + (size_t)t * (2 * P + 2);
#pragma unroll
    for (int l = 0; l < 2 * P; ++l) {
        const double v = tail_quad_sum(acc[l]);
        if ((l & 3) == r) out[2 + l] += v;
    }
}

// ------------------------------------------------------------ split by order
// cnt[q * nbox + T] = pairs of T in order class q: orders in
// (q kOrderStep, (q + 1) kOrderStep] (the top class holds the plan order p,
// which need not be a multiple of kOrderStep); the per-class counters of
// each lane live in LDS ([q][lane]), not in scratch
constexpr int kMaxQ = (kMaxOrder + kOrderStep - 1) / kOrderStep;
__device__ __forceinline__ int order_class(int o) { return (o + kOrderStep - 1) / kOrderStep - 1; }
__global__ void __launch_bounds__(256) k_order_count(const int* __restrict__ off, const uint8_t* __restrict__ ord,
                                                     int nbox, int nq, int* __restrict__ cnt,
                                                     long long* __restrict__ psq) {
    __shared__ int c[kMaxQ][256];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int q = 0; q < nq; ++q) c[q][threadIdx.x] = 0;
    if (t >= nbox) return;
    long long sq = 0;  // sum of p'^2 over the box's pairs (M2L work against p^2)
    for (int k = off[t]; k < off[t + 1]; ++k) {
        const int o = ord[k];
        ++c[order_class(o)][threadIdx.x];
        sq += o * o;
    }
    for (int q = 0; q < nq; ++q) cnt[(size_t)q * nbox + t] = c[q][threadIdx.x];
    psq[t] = sq;
}

// stable scatter of each box's entries into the list of their order; boff
// is the exclusive scan of cnt (so the lists of order q are the CSR boff +
// q nbox, with absolute offsets into bsrc).  A wave per box: the lanes take
// 64 consecutive entries at a time, and an entry's rank among the earlier
// entries of its class is the count of lower lanes of the same class (a
// ballot per class) plus those of the earlier groups.
__global__ void __launch_bounds__(256) k_order_scatter(const int* __restrict__ off, const int* __restrict__ src,
                                                       const uint8_t* __restrict__ ord, int nbox, int nq,
                                                       const int* __restrict__ boff, int* __restrict__ bsrc) {
    const int t = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    if (t >= nbox) return;  // the whole wave leaves together
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1;
    int base[kMaxQ];  // unrolled over every class so that it stays in registers
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q) base[q] = q < nq ? boff[(size_t)q * nbox + t] : 0;
    const int k1 = off[t + 1];
    for (int k0 = off[t]; k0 < k1; k0 += 64) {
        const int k = k0 + lane;
        const bool live = k < k1;
        const int mine = live ? order_class(ord[k]) : -1;
        int slot = 0;
#pragma unroll
        for (int q = 0; q < kMaxQ; ++q) {
            if (q >= nq) break;
            const uint64_t m = __ballot(mine == q);
            if (mine == q) slot = base[q] + __popcll(m & below);
            base[q] += __popcll(m);
        }
        if (live) bsrc[slot] = src[k];
    }
}

// ------------------------------------------------------------ host side
void order_box_decay(const FmmCtx& c, int nbox, float4* decay, hipStream_t s) {
    if (nbox <= 0) return;
    k_box_decay<<<nblk(nbox, 256), 256, 0, s>>>(c.mult, c.p, nbox, decay);
    SFMM_LAUNCH_CHECK();
}

void order_features(const FmmCtx& c, const int* ent_t, const int* src, const int* idx, int64_t n,
                    const float4* decay, double kappa_tol, float* feat, hipStream_t s) {
    if (n <= 0) return;
    k_pair_features<<<nblk(n, 256), 256, 0, s>>>(c, ent_t, src, idx, n, decay, (float)log10(kappa_tol), feat);
    SFMM_LAUNCH_CHECK();
}

void order_bound(const FmmCtx& c, const int* ent_t, const int* src, int np, double kappa_tol, uint8_t* ord,
                 hipStream_t s) {
    if (np <= 0) return;
    k_order_bound<<<nblk(np, 256), 256, 0, s>>>(c, ent_t, src, np, kappa_tol, c.p, ord);
    SFMM_LAUNCH_CHECK();
}

void order_mlp(const FmmCtx& c, const int* ent_t, const int* src, const float4* decay, double kappa_tol,
               const float* feat, int64_t n, const float* w, int pmax, float margin, uint8_t* ord, float* y,
               hipStream_t s) {
    if (n <= 0) return;
    // one wave per 64 pairs, a few steps per wave
    const int64_t waves = std::min<int64_t>((n + 63) / 64, 4096 * 4);
    k_order_mlp<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(c, ent_t, src, decay, (float)log10(kappa_tol), feat, n,
                                                            w, pmax, margin, ord, y);
    SFMM_LAUNCH_CHECK();
}

void m2l_qtail(const FmmCtx& c, const int* off, const int* src, const uint8_t* ord, int nbox, hipStream_t s) {
    if (nbox <= 0) return;
#define L_(P) case P: k_m2l_qtail<P><<<nblk(4 * (int64_t)nbox, 128), 128, 0, s>>>(c, off, src, ord, nbox); break;
    SFMM_DISPATCH(c.p, L_)
#undef L_
    SFMM_LAUNCH_CHECK();
}

void order_labels(const FmmCtx& c, const int* ent_t, const int* src, const int* idx, int n, double kappa_tol,
                  float* label, hipStream_t s) {
    if (n <= 0) return;
    DVec<double> scratch;
    scratch.resize((size_t)n * 2 * (2 * c.p + 2));
    k_order_labels<<<nblk(n, 64), 64, 0, s>>>(c, ent_t, src, idx, n, kappa_tol, scratch.data(), label);
    SFMM_LAUNCH_CHECK();
    SFMM_HIP(hipStreamSynchronize(s));
}

void order_split(const int* off, const int* src, const uint8_t* ord, int nbox, int np, int pmax,
                 DVec<int>& boff, DVec<int>& bsrc, long long* osq, hipStream_t s) {
    const int nq = (pmax + kOrderStep - 1) / kOrderStep;
    if (nq > kMaxQ) throw Error(ST_INTERNAL, "more order classes than the split holds");
    DVec<int> cnt;
    DVec<long long> psq;
    cnt.resize((size_t)nq * nbox);
    psq.resize(std::max(nbox, 1));
    boff.resize((size_t)nq * nbox + 1);
    bsrc.resize(std::max(np, 1));
    k_order_count<<<nblk(nbox, 256), 256, 0, s>>>(off, ord, nbox, nq, cnt.data(), psq.data());
    SFMM_LAUNCH_CHECK();
    scan_excl_i32(cnt.data(), boff.data(), (int64_t)nq * nbox, boff.data() + (size_t)nq * nbox, s);
    k_order_scatter<<<nblk(64 * (int64_t)nbox, 256), 256, 0, s>>>(off, src, ord, nbox, nq, boff.data(), bsrc.data());
    SFMM_LAUNCH_CHECK();
    sum_i64(psq.data(), nbox, osq, s);  // left on the device: read when the statistics ask
}

}  // namespace sfmm
