/* Oracle-internal quad-precision geometry shared by healpix.c and tree.c.
 * TEST INFRASTRUCTURE ONLY. */
#ifndef SFMM_ORACLE_GEOM_H
#define SFMM_ORACLE_GEOM_H
#include "oracle.h"

void oracle_pix_point_q(int order, int64_t pix, double fx, double fy,
                        __float128* out3);
__float128 oracle_angdist_q(const __float128* a, const __float128* b);
__float128 oracle_box_radius_q(int order, int64_t pix);

#endif
