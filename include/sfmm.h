/*
 * libsfmm -- the spherical Fast Multipole Method (sFMM) of Suo, Kang, Wei &
 * Li (arXiv:2210.07021) on one AMD MI355X (gfx950).
 *
 * Problem (Sec. 3.1 Eq. SUM, Sec. 2.1 Eq. GRE_FUN, Eq. ALP_PSI, Eq.
 * STAND_CONDITION): N point masses q_j at unit vectors n_j; at M target unit
 * vectors n evaluate
 *     psi(n)   = sum_j q_j G(n, n_j),  G = (1/4pi) log((1 - n.n_j)/2),
 *     alpha(n) = grad psi(n), the covariant gradient on the sphere,
 * with psi in the zero-mean gauge of Eq. STAND_CONDITION (Q_tot/(4pi) added,
 * since G integrates to -1 over the sphere) unless SFMM_GAUGE_RAW is asked
 * for.  A source at exactly a target's position (bitwise) is left out of that
 * target's sum, keeping only its share of the gauge constant.
 *
 * Method: the adaptive HEALPix quasi-quad-tree of Sec. 3.1 (leaf cap m,
 * depth <= 29), Lemma 1 on leaves and Lemma 2 up the tree (Sec. 3.2), the
 * dual tree walk of Algorithm 1 (Sec. 3.4) with the MACs of Sec. 3.5 (c_s,
 * c_t), Lemma 3 on every FMM-act pair and Lemma 4 down the tree (Sec. 3.3),
 * the local expansion plus the direct sum over the close boxes at each
 * target (Sec. 3.6).
 *
 * Conventions for every call:
 *   - Point sets are device pointers to three FP64 planes [3][count]:
 *     x[0..count), y[0..count), z[0..count).  Masses are a device FP64 [N].
 *   - Outputs are caller-owned device buffers, FP64, in the caller's target
 *     order: psi [M], defl [3][M] (global Cartesian components of the tangent
 *     vector alpha).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call is ordered on it; host-visible results (stats, exports) are
 *     complete when the call returns.
 *   - Errors: every call returns an sfmm_status; on failure
 *     sfmm_last_error() holds a message for the calling thread.  No
 *     exception crosses this boundary.  A plan is not thread-safe.
 */
#ifndef SFMM_H
#define SFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfmm_plan_impl* sfmm_plan_t;
typedef struct sfmm_batch_impl* sfmm_batch_t;

typedef enum {
    SFMM_OK = 0,
    SFMM_ERR_INVALID_ARG = 1,       /* bad size, option or input values      */
    SFMM_ERR_OUT_OF_MEMORY = 2,     /* device allocation failed               */
    SFMM_ERR_HIP = 3,               /* a HIP runtime call or kernel failed    */
    SFMM_ERR_TOLERANCE_NOT_MET = 4, /* a per-pair order policy failed its
                                       judge and the fallback is disabled     */
    SFMM_ERR_INTERNAL = 5
} sfmm_status;

enum { SFMM_GAUGE_ZERO_MEAN = 0, SFMM_GAUGE_RAW = 1 };
/* SFMM_FP64: every step in FP64.  SFMM_FP32_MIXED: the precision tier -- the
 * pair sums of the near field and the M2L coefficient arithmetic in FP32
 * (two-float coordinates, per-tile FP64 sums), everything else (keys, tree,
 * P2M, M2M, L2L, L2P, C and Q of every expansion, the final sums) in FP64.
 * Meant for tolerances of 1e-6 and above; outputs are FP64 in both modes. */
enum { SFMM_FP64 = 0, SFMM_FP32_MIXED = 1 };

/* Order of each FMM act (Lemma 3 pair).  FIXED: every pair at the plan order
 * p.  Otherwise a pair at order p' < p translates its multipole part at p'
 * (A_1..A_p' of the source in, local coefficients 1..p' out) and its
 * monopole part at p.  BOUND: p' = the smallest multiple of 4 (or p) with
 * x^(p'+1) (p'+1) / (1 - x) <= SFMM_ORDER_KAPPA tolerance (the form of
 * Eq. MUL_ERR for the pair's convergence ratio x, relative to the source's
 * multipole strength W_S = sum_l |A_l| rho_S^-l).  LEARNED: p' predicted by
 * the order network (weights in sfmm_options.mlp_weights) for the same
 * criterion measured exactly; see sfmm_order_samples / sfmm_mlp_train.
 * Per-pair orders are multiples of 4 or the plan order p itself. */
enum { SFMM_ORDER_FIXED = 0, SFMM_ORDER_BOUND = 1, SFMM_ORDER_LEARNED = 2 };
#define SFMM_ORDER_KAPPA 0.1

/* The order network: kMlpIn = 8 features -> 64 ReLU -> 64 ReLU -> 1.  Weight
 * array of SFMM_MLP_WEIGHTS floats, in this order: W1 [64][8] (row = hidden
 * unit), b1 [64], W2 [64][64], b2 [64], w3 [64], b3.  Features of a pair
 * (target box T, source box S; a, b the shift parameters of the factorised
 * Lemma 3 translation, g its diagonal ratio, x = max(a + b, sqrt g)): x,
 * a/(a + b) (1/2 when a + b = 0), log10(kappa tol)/16, then
 * log10(|A_l| / |Q|)/8 of S's scaled multipole at l = 1, 4, 8, 16, and
 * level(T)/29.  The output y predicts (order - 16) / 8; the learned policy
 * uses the order ceil(16 + 8 y + 2) rounded up to a multiple of 4, at most p. */
#define SFMM_MLP_IN 8
#define SFMM_MLP_HIDDEN 64
#define SFMM_MLP_WEIGHTS (64 * 8 + 64 + 64 * 64 + 64 + 64 + 1)

typedef struct {
    int32_t order;      /* truncation order p of Eq. MUL_ERR, 1..64; 0 = pick p
                           from `tolerance`                                   */
    double tolerance;   /* target relative L2 error of psi and of alpha when
                           order == 0; in [1e-15, 1e-1]                       */
    int32_t leaf_size;  /* m of Sec. 3.1: a box holding more than m particles
                           is split; >= 1                                     */
    double c_s;         /* MAC1 constant of Sec. 3.5 (default 2)              */
    double c_t;         /* MAC2 constant of Sec. 3.5 (default 0.5)            */
    int32_t max_level;  /* maximum depth r_max of Sec. 3.1, 0..29 (default 29) */
    int32_t precision;  /* SFMM_FP64 (default) or SFMM_FP32_MIXED              */
    int32_t psi_gauge;  /* SFMM_GAUGE_ZERO_MEAN (default) or SFMM_GAUGE_RAW   */
    int32_t order_policy;      /* SFMM_ORDER_FIXED (default), _BOUND, _LEARNED */
    const float* mlp_weights;  /* host, SFMM_MLP_WEIGHTS floats; read (copied)
                                  by sfmm_plan when order_policy is LEARNED  */
    int32_t near_segment;      /* close leaves per near-field work item: direct
                                  sums (0 = 128); 8..4096                     */
    int32_t far_segment;       /* the same for the multipole evaluations     */
    int32_t judge_targets;     /* per-pair order policies: targets of the
                                  judge's direct sum (0 = 32; < 0: no judge);
                                  at most 4096                               */
    int32_t no_fallback;       /* nonzero: a failed judge returns
                                  SFMM_ERR_TOLERANCE_NOT_MET instead of
                                  rerunning at the fixed order               */
    double npm_sigma;          /* near-particle model (Sec. 3.1 NPM, Sec. 4.2
                                  Eq. KERNEL): every source is a generalised
                                  Epanechnikov profile of this angular radius
                                  (radians, in [0, 0.5]; 0 = point masses)  */
} sfmm_options;

typedef struct {
    int64_t n_sources, n_targets;
    int64_t n_boxes, n_leaves, n_levels;
    int64_t n_m2l, n_p2p;           /* FMM-act and direct-act pairs            */
    int64_t n_target_leaves;        /* leaves with targets and direct-sum work */
    int64_t n_p2p_pairs;            /* particle-target pairs summed directly    */
    int64_t n_m2p_evals;            /* (target, close leaf) pairs evaluated by
                                       the leaf's multipole expansion instead  */
    int32_t order, leaf_size;
    double q_total;                 /* sum of the masses                        */
    int64_t m2l_order_sq;           /* sum over the FMM acts of (their order)^2
                                       in the last sfmm_execute (the M2L work
                                       relative to one order-1 act); 0 before */
    double judge_psi, judge_alpha;  /* relative L2 error of psi and alpha of the
                                       per-pair order policy at the judge's
                                       targets against their direct sum; -1
                                       before the judge ran (fixed order, no
                                       judge, or not executed)                */
    int32_t judge_targets;          /* targets the judge summed directly      */
    int32_t fell_back;              /* 1: the judge failed and the plan runs at
                                       the fixed order                        */
    int64_t execute_scratch_bytes;  /* device scratch one execute of this plan
                                       uses beyond the plan's own arrays (see
                                       sfmm_execute_noalloc)                  */
} sfmm_stats;

/* Near-particle model (npm_sigma = sigma > 0; Sec. 3.1 NPM, Sec. 4.2 Eq.
 * KERNEL): every source is the mass distribution W(theta) = [1 -
 * sin^2(theta/2)/sin^2(sigma/2)] / (2 pi sin^2(sigma/2)) (theta <= sigma),
 * and psi, alpha (and the Hessian) are those of the smoothed particles: the
 * solution of Laplacian psi = sum_j q_j W_j - Q_tot/(4pi) in the zero-mean
 * gauge.  Outside sigma a particle deflects as a point mass; its potential
 * differs from the point mass's by a constant; inside, the interior
 * solution applies, and a source at the target itself contributes its
 * finite central value (no exclusion).  The expansions stay exact: the
 * protected zone of Sec. 3.5 around a source box is max(c_s R_S, R_S +
 * sigma), so no FMM act or expansion evaluation has a target inside a
 * particle.  The deflection inside differs from the printed Eq.
 * KERNEL_ALPHA (whose normalisation is -2 pi times this one's) by
 * O(sin^2(sigma/2)) relative: that formula leaves out the background term
 * -q/(4pi) inside the particle. */

/* Fill *opt with the defaults: order 0 with tolerance 1e-10, leaf_size 64,
 * c_s 2, c_t 0.5, max_level 29, FP64, zero-mean gauge, point masses. */
void sfmm_default_options(sfmm_options* opt);

/* Build a plan: keys, sorting, the tree (Sec. 3.1), box geometry (Sec. 3.5),
 * the interaction lists of Algorithm 1 (Sec. 3.4) and the target-to-leaf map
 * (Sec. 3.7).  src [3][N], q [N], tgt [3][M] are device buffers; they are
 * copied (and sorted), so the caller may reuse them once the stream has
 * passed this call.  N = 0 is allowed (all outputs are zero); M = 0 is
 * allowed (execute does nothing).
 * Errors: SFMM_ERR_INVALID_ARG for N or M negative or above 2^31 - 1, null
 * pointers with a nonzero size, options out of range, non-finite input
 * coordinates or points off the unit sphere by more than 1e-6 (points off by
 * more than 1e-14 are renormalised). */
sfmm_status sfmm_plan(const double* src, const double* q, int64_t N, const double* tgt, int64_t M,
                      const sfmm_options* opt, void* stream, sfmm_plan_t* out);

/* Run the five stages of Sec. 3.7 for a plan: psi [M] and defl [3][M]
 * (device, caller-owned, caller's target order) are overwritten.
 * With the bound or learned order policy the first execute of a plan is
 * judged: psi and alpha at a seeded subset of judge_targets targets are
 * compared with the library's own GPU direct sum of Eq. SUM / Eq. ALP_PSI
 * (FP64, compensated sums, every source); if the relative L2 error of
 * either exceeds the tolerance the plan falls back to the fixed order p for
 * this and every later execute (the outputs are recomputed), or, with
 * no_fallback set, the call returns SFMM_ERR_TOLERANCE_NOT_MET (the outputs
 * hold the policy's result; later executes return the same status).  The
 * verdict is kept with the plan: the orders a policy picks depend only on
 * the plan's inputs.  sfmm_stats reports the judge's errors. */
sfmm_status sfmm_execute(sfmm_plan_t plan, double* psi, double* defl, void* stream);

/* sfmm_execute that also returns the Hessian of psi (Sec. 2.2, the matrix H
 * of Eq. GAM_DEF): hess [3][M] (device, caller-owned, caller's target order)
 * receives H_11 = d^2 psi/d theta^2, H_12 = d/d theta ((1/sin theta) d psi /
 * d phi) and H_22 = (1/sin^2 theta) d^2 psi/d phi^2 + cot theta d psi/d theta
 * in the basis e_theta, e_phi of each target (at an exact pole the limit at
 * phi = 0).  From the same expansions (Sec. 3.6): the local and multipole
 * forms' second derivatives in their stereographic coordinate, and the
 * direct sum's pair terms.  Convergence, shear and magnification follow as
 * kappa - kappa_bar = H_11 + H_22, gamma_1 = (H_11 - H_22)/2, gamma_2 =
 * H_12, mu = 1/det(I - H) (sfmm_lensing).  Errors as sfmm_execute. */
sfmm_status sfmm_execute_hessian(sfmm_plan_t plan, double* psi, double* defl, double* hess, void* stream);

/* Lensing quantities of Sec. 2.2 from a Hessian: out [4][M] (device) =
 * (kappa - kappa_bar, gamma_1, gamma_2, mu) with kappa - kappa_bar = tr H
 * (Eq. GAM_DEF), gamma_1 = (H_11 - H_22)/2, gamma_2 = H_12 and mu =
 * 1/((1 - (kappa - kappa_bar)/2)^2 - gamma_1^2 - gamma_2^2); hess [3][M]
 * (device) as written by sfmm_execute_hessian.  Stream-ordered.  Errors:
 * SFMM_ERR_INVALID_ARG for M < 0 or NULL buffers with M > 0. */
sfmm_status sfmm_lensing(const double* hess, int64_t M, double* out, void* stream);

/* Multi-plane backtracking through nlayer lensing layers (Sec. 2.1, Eq.
 * DIS_PRO): rays [3][M] (device unit vectors) enter layer 0 at their
 * observed positions theta_0 and, layer by layer, move to theta_{i+1} =
 * theta_i - weight[i] alpha_i(theta_i), alpha_i the deflection of layer i's
 * masses (src[i] [3][N[i]], q[i] [N[i]], device; as in sfmm_plan) at the
 * rays' current positions; weight[i] (host) is f_K(r_s - r_i) / f_K(r_s) for
 * the source distance r_s.  The step follows the great circle (the ray moves
 * by |w alpha| in the direction of -alpha).  On return rays holds theta_n.
 * dist [4][M] (device, may be NULL): the distortion matrix A = d theta_n /
 * d theta_0, (A_11, A_12, A_21, A_22) in the e_theta, e_phi bases of theta_0
 * (columns) and theta_n (rows), propagated with each layer's Hessian (Sec.
 * 2.2) to first order in the step: A <- T (I - w H) A, T the parallel
 * transport along the step.  Every layer is planned and executed with *opt
 * (the same rules and errors as sfmm_plan / sfmm_execute); the call returns
 * when the work on `stream` is done.  Errors: nlayer outside [1, 4096],
 * non-finite weights, NULL arrays, M outside [0, 2^31 - 1]. */
sfmm_status sfmm_raytrace(int32_t nlayer, const double* const* src, const double* const* q, const int64_t* N,
                          const double* weight, double* rays, int64_t M, double* dist, const sfmm_options* opt,
                          void* stream);

/* sfmm_execute without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, same kernels and the same results,
 * bitwise, as sfmm_execute; the execute's scratch (partial sums of the near
 * field's split boxes, the FP32 copy of the multipoles in the precision tier)
 * lives in a static device array of 256 MiB per GPU that the library holds
 * until the process ends, instead of memory the plan or the call allocates.
 * No hipMalloc, hipFree or allocating routine is called (the plan itself was
 * allocated by sfmm_plan).  Every call on one GPU shares that array: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller.  Errors: SFMM_ERR_INVALID_ARG for a plan with a
 * per-pair order policy (its order split allocates) or one whose scratch
 * (sfmm_stats.execute_scratch_bytes) exceeds 256 MiB; otherwise as
 * sfmm_execute. */
sfmm_status sfmm_execute_noalloc(sfmm_plan_t plan, double* psi, double* defl, void* stream);

/* Batches: several independent spheres (lensing shells, Sec. 2.1: one
 * Poisson problem per layer) planned together and executed as one unit.
 * sfmm_batch_plan: sfmm_plan on each of the nshell (src[i], q[i], N[i],
 *   tgt[i], M[i]) with the same options; the batch owns the plans.  The shells
 *   are planned by up to four host threads, each with a stream of the batch
 *   that starts after the work already on `stream` (largest shells first,
 *   each to the least loaded thread); the call returns when every plan is
 *   complete.  With the null stream the batch creates a stream of its own
 *   for sfmm_batch_execute.
 * sfmm_batch_execute: psi[i] [M[i]] and defl[i] [3][M[i]] for every shell.
 *   The shells run on the batch's streams, forked from and joined back into
 *   `stream`, so that one shell's latency-bound stretches overlap another's
 *   kernels.  The first call (and any call with other output pointers or
 *   another stream) runs every shell once directly, records the same work in
 *   a HIP graph (the streams become its parallel branches) and launches it;
 *   later calls replay the graph: one launch for all shells.  Batches with the bound or learned order policy are run directly
 *   every time (their per-order split reads sizes on the host).  With the
 *   null stream the call returns when the work is done.
 * sfmm_batch_plan_at: the plan of shell i, owned by the batch (never to be
 *   destroyed by the caller; it may be executed directly, ordered with the
 *   batch's own calls).
 * Errors: as sfmm_plan / sfmm_execute; nshell outside [1, 4096]. */
sfmm_status sfmm_batch_plan(int32_t nshell, const double* const* src, const double* const* q, const int64_t* N,
                            const double* const* tgt, const int64_t* M, const sfmm_options* opt, void* stream,
                            sfmm_batch_t* out);
sfmm_status sfmm_batch_execute(sfmm_batch_t batch, double* const* psi, double* const* defl, void* stream);
sfmm_status sfmm_batch_plan_at(sfmm_batch_t batch, int32_t i, sfmm_plan_t* out);
void sfmm_batch_destroy(sfmm_batch_t batch);

/* Sizes of a plan. */
sfmm_status sfmm_stats_get(sfmm_plan_t plan, sfmm_stats* out);

/* Host copies of the tree for comparisons, in the library's box order
 * (level, then pixel).  Buffers are host memory of the sizes in sfmm_stats:
 *   level, pixel, first, count, parent, child0: [n_boxes] (child0 = -1 for a
 *   leaf, parent = -1 at level 0); centre [3][n_boxes]; radius [n_boxes]
 *   (radians).  Any pointer may be NULL to skip that array. */
sfmm_status sfmm_export_boxes(sfmm_plan_t plan, int32_t* level, int64_t* pixel, int64_t* first,
                              int64_t* count, int64_t* parent, int64_t* child0, double* centre,
                              double* radius);

/* Host copies of the interaction lists, sorted by (target box, source box):
 * m2l_src/m2l_tgt [n_m2l] and p2p_src/p2p_tgt [n_p2p].  Source boxes without
 * particles are left out of both lists (they contribute nothing). */
sfmm_status sfmm_export_lists(sfmm_plan_t plan, int64_t* m2l_src, int64_t* m2l_tgt, int64_t* p2p_src,
                              int64_t* p2p_tgt);

/* Host copies of the order-29 keys: src_keys [N] ascending with src_perm
 * [N] the caller index of each; for the targets in plan order (grouped by
 * leaf box, ascending box index, caller order within a leaf) tgt_perm [M]
 * the caller index, tgt_keys [M] the key and tgt_leaf [M] the leaf box of
 * each. */
sfmm_status sfmm_export_keys(sfmm_plan_t plan, uint64_t* src_keys, int64_t* src_perm, uint64_t* tgt_keys,
                             int64_t* tgt_perm, int64_t* tgt_leaf);

/* Host copies of the per-box near-field work, [n_boxes] each: tgt_count the
 * targets located in the box, pairs the particle-target pairs its targets
 * sum directly, evals the (target, close leaf) pairs taken through the
 * leaf's multipole expansion instead.  For load-balance diagnostics; any
 * pointer may be NULL. */
sfmm_status sfmm_export_work(sfmm_plan_t plan, int64_t* tgt_count, int64_t* pairs, int64_t* evals);

/* Host copies of the expansions after sfmm_execute, in the paper's
 * normalisation (Lemma 1: psi = C + Q log(1 -+ cos) + 2 Re sum A_l z^(-+l)):
 * multipole and local are [n_boxes][2p+2] = (C, Q, Re A_1, Im A_1, ...,
 * Re A_p, Im A_p).  C is reported without the zero-mean gauge share. */
sfmm_status sfmm_export_expansions(sfmm_plan_t plan, double* multipole, double* local);

/* Training data for the order network, from an executed plan: n FMM-act
 * pairs drawn with the seed (uniformly, with replacement), their features
 * [n][SFMM_MLP_IN] and their labels [n]: the smallest multiple of 4 (<= the
 * plan order p) for which the pair's Lemma 3 translation truncated at that
 * order (multipole part; monopole part kept at p) differs from the order-p
 * translation by sum_l l |dA'_l| <= SFMM_ORDER_KAPPA tolerance W_S (scaled
 * local coefficients, FP64).  Host buffers.  Errors: plan not executed, n < 0,
 * NULL buffers with n > 0. */
sfmm_status sfmm_order_samples(sfmm_plan_t plan, int64_t n, uint64_t seed, float* features, float* labels,
                               int64_t* pairs /* [n][2] (target box, source box), may be NULL */);

/* Order network, all host buffers.
 * sfmm_mlp_init: He-initialised weights from the seed.
 * sfmm_mlp_train: Adam (lr), `epochs` passes over the n samples in shuffled
 *   minibatches of `batch`, loss per sample w r^2 (r = prediction - label,
 *   w = 4 for r < 0, else 1); weights are read and overwritten; epoch_loss
 *   [epochs] (may be NULL) receives the mean loss of each epoch.
 * sfmm_mlp_forward: y [n] = network(features); bf16 != 0 rounds weights and
 *   activations to bfloat16 as the learned policy does, else FP32.
 * sfmm_mlp_grad: gradient [SFMM_MLP_WEIGHTS] and value of the mean loss over
 *   the n samples (FP32 network).
 * Errors: n < 0 or NULL buffers with n > 0, batch < 1, epochs < 0. */
void sfmm_mlp_init(uint64_t seed, float* weights);
sfmm_status sfmm_mlp_train(const float* features, const float* labels, int64_t n, int32_t epochs, int32_t batch,
                           float lr, uint64_t seed, float* weights, float* epoch_loss);
sfmm_status sfmm_mlp_forward(const float* weights, const float* features, int64_t n, int32_t bf16, float* y);
sfmm_status sfmm_mlp_grad(const float* weights, const float* features, const float* labels, int64_t n,
                          float* grad, float* loss);

/* Global-basis helpers (Sec. 3.6: the global components of the deflection
 * follow from its tangent vector by a change of coordinates).  Host buffers,
 * host arithmetic; no device work.
 * sfmm_thetaphi_to_xyz: xyz [3][n] = (sin t cos p, sin t sin p, cos t) for
 *   colatitudes theta [n] and longitudes phi [n] (radians): the unit vectors
 *   that sfmm_plan takes.
 * sfmm_defl_to_thetaphi: out [2][n] = (alpha_theta, alpha_phi), the
 *   components of the tangent vectors defl [3][n] (as sfmm_execute writes
 *   them) at the unit vectors xyz [3][n] in the local basis e_theta = (cos t
 *   cos p, cos t sin p, -sin t), e_phi = (-sin p, cos p, 0), so that
 *   alpha_theta = d psi/d theta and alpha_phi = (1/sin t) d psi/d phi.  At an
 *   exact pole (x = y = 0) the basis is its limit along the meridian phi[i];
 *   phi may be NULL (then phi = 0 there).
 * Errors: SFMM_ERR_INVALID_ARG for n < 0 or NULL buffers with n > 0. */
sfmm_status sfmm_thetaphi_to_xyz(const double* theta, const double* phi, int64_t n, double* xyz);
sfmm_status sfmm_defl_to_thetaphi(const double* xyz, const double* defl, const double* phi, int64_t n,
                                  double* out);

void sfmm_destroy(sfmm_plan_t plan);
const char* sfmm_status_string(sfmm_status s);
const char* sfmm_last_error(void);

/* Order p that reaches the relative tolerance tol (the policy used when
 * opt->order == 0). */
int32_t sfmm_order_for_tolerance(double tol);

/* Stage timing.  While enabled, every sfmm_plan / sfmm_execute brackets each
 * stage with HIP events on the caller's stream and, at the end of the call,
 * synchronises the stream and adds the elapsed times to process-wide
 * per-stage totals.  Stages (indices into the arrays of sfmm_profile_read):
 *   0 source keys+sort, 1 tree levels, 2 box geometry, 3 walk (Algorithm 1),
 *   4 list sort/CSR, 5 target keys+sort+locate and the split of the
 *   direct-act lists into direct sums and expansions, 6 P2M, 7 M2M (all levels),
 *   8 M2L, 9 L2L (all levels), 10 L2P, 11 P2P (direct part of the close
 *   leaves), 12 close leaves evaluated by their multipole expansion.
 * ms[SFMM_NUM_STAGES] receives the summed milliseconds and calls[] the number
 * of times each stage ran; both are host arrays and may be NULL. */
#define SFMM_NUM_STAGES 13
void sfmm_profile_enable(int32_t on);
void sfmm_profile_reset(void);
void sfmm_profile_read(double* ms, int64_t* calls);

#ifdef __cplusplus
}
#endif
#endif
