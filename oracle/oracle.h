/*
 * CPU oracle for the spherical FMM (sFMM) of Suo, Kang, Wei & Li,
 * "The spherical Fast Multipole Method (sFMM) for Gravitational Lensing
 * Simulation" (arXiv:2210.07021).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain FP64 reference
 * that the GPU path is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product library
 * never does, and it shares no code, header, table or helper with the GPU
 * sources.
 *
 * Conventions (all arrays are plain host memory owned by the caller):
 *   - points are unit vectors stored as three planes, [3][n]: x[0..n), y[0..n),
 *     z[0..n);
 *   - the Green's function is G = (1/4pi) log((1 - n.n')/2), Sec. 2.1 Eq. GRE_FUN,
 *     evaluated as (1/4pi) log(|n - n'|^2 / 4), which is the same number for
 *     unit vectors and does not cancel for close points;
 *   - the zero-mean gauge of Sec. 2.1 Eq. STAND_CONDITION adds Q_tot/(4 pi) to
 *     Eq. SUM, because the sphere integral of G is -1;
 *   - a source at exactly the target position (bitwise) is left out of the sum
 *     (the point kernel is singular there and the paper only treats it through
 *     its near-particle model).
 */
#ifndef SFMM_ORACLE_H
#define SFMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Gauges for psi: 0 = zero mean over the sphere (Eq. STAND_CONDITION),
 * 1 = Eq. SUM exactly as printed. */
enum { ORACLE_GAUGE_ZERO_MEAN = 0, ORACLE_GAUGE_RAW = 1 };

/* Direct sum (the paper's "PPM", Sec. 4.1): psi (Eq. SUM) and
 * alpha = grad psi (Eq. ALP_PSI) at m targets from n point masses, FP64 with
 * Neumaier-compensated accumulation, OpenMP over targets.
 * defl is [3][m] and holds the global Cartesian components of the tangent
 * vector alpha.  nthreads <= 0 uses the OpenMP default. */
void oracle_direct(const double* src, const double* q, int64_t n,
                   const double* tgt, int64_t m, int gauge,
                   double* psi, double* defl, int nthreads);

/* Hessian of psi (Sec. 2.2) in the basis e_theta, e_phi at each target:
 * hess [3][m] = (H_11, H_12, H_22); coincident sources left out. */
void oracle_hessian(const double* src, const double* q, int64_t n, const double* tgt, int64_t m,
                    double* hess, int nthreads);

/* Sources as near-particle-model profiles of radius sigma (Sec. 3.1 NPM,
 * Eq. KERNEL): psi [m], defl [3][m] and, if hess is not NULL, hess [3][m]. */
void oracle_npm(const double* src, const double* q, int64_t n, const double* tgt, int64_t m, double sigma,
                int gauge, double* psi, double* defl, double* hess, int nthreads);

/* HEALPix nested pixel index at the given order (nside = 2^order) of the
 * unit vector (x, y, z); the sphere division of Sec. 3.1.  Evaluated in quad
 * precision, i.e. the exact-arithmetic pixel of the FP64 input. */
int64_t oracle_key(double x, double y, double z, int order);

/* Point of pixel (order, pix) at fractional face coordinates (fx, fy) in
 * [0,1]^2; (0.5, 0.5) is the pixel centre, the four corners are its
 * vertices.  Quad-precision value rounded to FP64. */
void oracle_pix_point(int order, int64_t pix, double fx, double fy,
                      double* out3);

/* Angular radius of the smallest circle about the pixel centre that covers
 * the pixel (Sec. 3.5): the largest angular distance to its four vertices. */
double oracle_box_radius(int order, int64_t pix);

/* Angular distance between two unit vectors. */
double oracle_angdist(const double* a, const double* b);

/* Adaptive quasi-quad-tree of Sec. 3.1: 12 base boxes, every box holding
 * more than m particles is split into its 4 HEALPix children, down to
 * max_level.  Boxes come out ordered by (level, pixel).
 *   keys[n], perm[n]   sorted order-29 keys and the source index of each
 *   level..radius      box table of capacity cap (centre is [3][cap])
 * Returns the number of boxes, or -1 when cap is too small. */
int64_t oracle_tree(const double* src, int64_t n, int m, int max_level,
                    uint64_t* keys, int64_t* perm, int64_t cap,
                    int32_t* level, int64_t* pixel, int64_t* first,
                    int64_t* count, int64_t* parent, int64_t* child0,
                    double* centre, double* radius);

/* Algorithm 1 (Sec. 3.4) from (root, root) with the two MACs of Sec. 3.5,
 * over a box table given by (level, pixel, child0); the geometry is
 * recomputed in quad precision from the box identities.  Emits FMM-act pairs
 * (source box, target box) and direct-act pairs (source leaf, target leaf) in
 * recursion order.  Returns 0, or -1 when a capacity is too small (the counts
 * then hold the sizes needed).  min_margin receives the smallest relative
 * distance |a-b|/(|a|+|b|) of any MAC test from its threshold among those
 * that are not exact ties (relative distance above 1e-24); exact ties are
 * decided "not far" by a relative guard of 1e-20. */
int oracle_walk(int64_t nbox, const int32_t* level, const int64_t* pixel,
                const int64_t* child0, double c_s, double c_t,
                int64_t cap_m2l, int64_t* m2l_src, int64_t* m2l_tgt,
                int64_t* n_m2l, int64_t cap_p2p, int64_t* p2p_src,
                int64_t* p2p_tgt, int64_t* n_p2p, double* min_margin);

/* Leaf box holding each target, found by descending from its base box with
 * the target's own key (Sec. 3.7, last step of the overview). */
void oracle_locate(const double* tgt, int64_t m, const int64_t* child0,
                   const int32_t* level, int64_t* leaf_of_target,
                   uint64_t* tgt_keys);

#ifdef __cplusplus
}
#endif
#endif
