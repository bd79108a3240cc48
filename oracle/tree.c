/*
 * Oracle: the adaptive quasi-quad-tree (Sec. 3.1), the dual tree walk of
 * Algorithm 1 (Sec. 3.4) with the acceptance criteria of Sec. 3.5, and the
 * target-to-leaf descent (Sec. 3.7).  TEST INFRASTRUCTURE ONLY.
 *
 * Readings taken where the paper is silent:
 *   - base boxes are level 0 (nside = 2^level), so the maximum depth 29 of
 *     Sec. 3.1 is HEALPix order 29;
 *   - a box splits when it holds more than m particles and is above the
 *     maximum depth; all 4 children are created, empty ones included, and a
 *     box at the maximum depth may hold more than m particles;
 *   - box centre = HEALPix pixel centre, box radius = largest angular
 *     distance from it to the pixel's vertices, box distance = angular
 *     distance of centres;
 *   - both MAC inequalities are strict as printed.  HEALPix geometry makes
 *     exact equality common (a vertex shared by two diagonal neighbours is
 *     the geodesic midpoint of their centres, so R_T = d/2 exactly), and at
 *     deep levels flat-limit ties are broken only by curvature terms far
 *     below FP64 resolution.  Geometry is therefore evaluated in quad
 *     precision from the exact box identity (level, pixel), and each side of
 *     an inequality must exceed the other by a relative 1e-20 of d:
 *     configurations equal in exact arithmetic are then "not far", as the
 *     strict inequality says;
 *   - the radius comparison of Algorithm 1 likewise treats radii within a
 *     relative 1e-20 of each other as equal (congruent boxes), so ties split
 *     the target box, as the printed else-branch does;
 *   - a leaf paired with itself direct-acts on itself (Algorithm 1 does
 *     nothing there, which would lose the particles' own leaf).
 */
#include "oracle_geom.h"
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>

#define ORACLE_ORDER 29
#define RADIUS_TIE 1e-20Q
#define MAC_TIE 1e-20Q

typedef struct {
    uint64_t key;
    int64_t idx;
} keyidx_t;

static int cmp_keyidx(const void* a, const void* b) {
    const keyidx_t* x = (const keyidx_t*)a;
    const keyidx_t* y = (const keyidx_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

/* first position in keys[lo, hi) with keys[i] >= v */
static int64_t lower_bound(const uint64_t* keys, int64_t lo, int64_t hi,
                           uint64_t v) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

int64_t oracle_tree(const double* src, int64_t n, int m, int max_level,
                    uint64_t* keys, int64_t* perm, int64_t cap,
                    int32_t* level, int64_t* pixel, int64_t* first,
                    int64_t* count, int64_t* parent, int64_t* child0,
                    double* centre, double* radius) {
    keyidx_t* ki = (keyidx_t*)malloc(sizeof(keyidx_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) {
        ki[j].key = (uint64_t)oracle_key(src[j], src[n + j], src[2 * n + j],
                                         ORACLE_ORDER);
        ki[j].idx = j;
    }
    qsort(ki, (size_t)n, sizeof(keyidx_t), cmp_keyidx);
    for (int64_t j = 0; j < n; ++j) {
        keys[j] = ki[j].key;
        perm[j] = ki[j].idx;
    }
    free(ki);

    /* Step 1: the 12 base boxes.  Step 2-3: split breadth first, which
     * leaves the table ordered by (level, pixel). */
    if (cap < 12) return -1;
    int64_t nbox = 0;
    for (int f = 0; f < 12; ++f) {
        const uint64_t lo = (uint64_t)f << (2 * ORACLE_ORDER);
        const uint64_t hi = (uint64_t)(f + 1) << (2 * ORACLE_ORDER);
        const int64_t a = lower_bound(keys, 0, n, lo);
        const int64_t b = lower_bound(keys, a, n, hi);
        level[nbox] = 0;
        pixel[nbox] = f;
        first[nbox] = a;
        count[nbox] = b - a;
        parent[nbox] = -1;
        child0[nbox] = -1;
        ++nbox;
    }
    for (int64_t b = 0; b < nbox; ++b) {
        if (count[b] > m && level[b] < max_level) {
            const int L = level[b] + 1;
            const int shift = 2 * (ORACLE_ORDER - L);
            if (nbox + 4 > cap) return -1;
            child0[b] = nbox;
            int64_t lo = first[b];
            const int64_t end = first[b] + count[b];
            for (int c = 0; c < 4; ++c) {
                const int64_t pix = pixel[b] * 4 + c;
                const uint64_t hi = (uint64_t)(pix + 1) << shift;
                const int64_t e = lower_bound(keys, lo, end, hi);
                level[nbox] = L;
                pixel[nbox] = pix;
                first[nbox] = lo;
                count[nbox] = e - lo;
                parent[nbox] = b;
                child0[nbox] = -1;
                ++nbox;
                lo = e;
            }
        }
    }
    for (int64_t b = 0; b < nbox; ++b) {
        double c[3];
        oracle_pix_point(level[b], pixel[b], 0.5, 0.5, c);
        centre[b] = c[0];
        centre[cap + b] = c[1];
        centre[2 * cap + b] = c[2];
        radius[b] = oracle_box_radius(level[b], pixel[b]);
    }
    return nbox;
}

typedef struct {
    const int64_t* child0;
    const __float128* centre; /* [nbox][3] */
    const __float128* radius;
    __float128 c_s, c_t;
    int64_t cap_m2l, cap_p2p;
    int64_t *m2l_s, *m2l_t, *p2p_s, *p2p_t;
    int64_t n_m2l, n_p2p;
    double min_margin;
} walk_t;

#define ROOT (-1)

static int is_leaf(const walk_t* w, int64_t b) {
    return b != ROOT && w->child0[b] < 0;
}

static int n_children(const walk_t* w, int64_t b) {
    (void)w;
    return b == ROOT ? 12 : 4;
}

static int64_t child(const walk_t* w, int64_t b, int i) {
    return b == ROOT ? i : w->child0[b] + i;
}

/* Track the closest genuine decision: relative margins below 1e-24 are
 * exact-arithmetic ties (quad rounding noise) and are decided by the guard;
 * anything else must sit well clear of the guard. */
static void note_margin(walk_t* w, __float128 lhs, __float128 rhs) {
    const __float128 den = fabsq(lhs) + fabsq(rhs);
    if (den > 0) {
        const double r = (double)(fabsq(lhs - rhs) / den);
        if (r > 1e-24 && r < w->min_margin) w->min_margin = r;
    }
}

/* "B_T is far from B_S": both MACs of Sec. 3.5, strict. */
static int is_far(walk_t* w, int64_t s, int64_t t) {
    const __float128 d = oracle_angdist_q(w->centre + 3 * s, w->centre + 3 * t);
    const __float128 rs = w->radius[s], rt = w->radius[t];
    note_margin(w, d, rt + w->c_s * rs);
    note_margin(w, rt, w->c_t * d);
    return (d - rt - w->c_s * rs > MAC_TIE * d) && (w->c_t * d - rt > MAC_TIE * d);
}

static void emit(int64_t* cnt, int64_t cap, int64_t* as, int64_t* at,
                 int64_t s, int64_t t) {
    if (*cnt < cap) {
        as[*cnt] = s;
        at[*cnt] = t;
    }
    ++*cnt;
}

static void interaction(walk_t* w, int64_t s, int64_t t) {
    if (s == t) {
        if (!is_leaf(w, s)) {
            for (int i = 0; i < n_children(w, s); ++i)
                for (int j = 0; j < n_children(w, s); ++j)
                    interaction(w, child(w, s, i), child(w, s, j));
        } else {
            emit(&w->n_p2p, w->cap_p2p, w->p2p_s, w->p2p_t, s, s);
        }
        return;
    }
    if (is_far(w, s, t)) {
        emit(&w->n_m2l, w->cap_m2l, w->m2l_s, w->m2l_t, s, t);
        return;
    }
    const int sl = is_leaf(w, s), tl = is_leaf(w, t);
    if (!sl && !tl) {
        if (w->radius[s] > w->radius[t] * (1 + RADIUS_TIE)) {
            for (int i = 0; i < 4; ++i) interaction(w, child(w, s, i), t);
        } else {
            for (int j = 0; j < 4; ++j) interaction(w, s, child(w, t, j));
        }
    } else if (!sl) {
        for (int i = 0; i < 4; ++i) interaction(w, child(w, s, i), t);
    } else if (!tl) {
        for (int j = 0; j < 4; ++j) interaction(w, s, child(w, t, j));
    } else {
        emit(&w->n_p2p, w->cap_p2p, w->p2p_s, w->p2p_t, s, t);
    }
}

int oracle_walk(int64_t nbox, const int32_t* level, const int64_t* pixel,
                const int64_t* child0, double c_s, double c_t,
                int64_t cap_m2l, int64_t* m2l_src, int64_t* m2l_tgt,
                int64_t* n_m2l, int64_t cap_p2p, int64_t* p2p_src,
                int64_t* p2p_tgt, int64_t* n_p2p, double* min_margin) {
    __float128* cen = (__float128*)malloc(sizeof(__float128) * 3 * (size_t)(nbox > 0 ? nbox : 1));
    __float128* rad = (__float128*)malloc(sizeof(__float128) * (size_t)(nbox > 0 ? nbox : 1));
    for (int64_t b = 0; b < nbox; ++b) {
        oracle_pix_point_q(level[b], pixel[b], 0.5, 0.5, cen + 3 * b);
        rad[b] = oracle_box_radius_q(level[b], pixel[b]);
    }
    walk_t w;
    w.child0 = child0;
    w.centre = cen;
    w.radius = rad;
    w.c_s = c_s;
    w.c_t = c_t;
    w.cap_m2l = cap_m2l;
    w.cap_p2p = cap_p2p;
    w.m2l_s = m2l_src;
    w.m2l_t = m2l_tgt;
    w.p2p_s = p2p_src;
    w.p2p_t = p2p_tgt;
    w.n_m2l = 0;
    w.n_p2p = 0;
    w.min_margin = INFINITY;
    interaction(&w, ROOT, ROOT);
    free(cen);
    free(rad);
    *n_m2l = w.n_m2l;
    *n_p2p = w.n_p2p;
    *min_margin = w.min_margin;
    return (w.n_m2l > cap_m2l || w.n_p2p > cap_p2p) ? -1 : 0;
}

void oracle_locate(const double* tgt, int64_t m, const int64_t* child0,
                   const int32_t* level, int64_t* leaf_of_target,
                   uint64_t* tgt_keys) {
    for (int64_t i = 0; i < m; ++i) {
        const uint64_t key = (uint64_t)oracle_key(tgt[i], tgt[m + i],
                                                  tgt[2 * m + i], ORACLE_ORDER);
        tgt_keys[i] = key;
        int64_t b = (int64_t)(key >> (2 * ORACLE_ORDER)); /* base box id */
        while (child0[b] >= 0) {
            const int L = level[b] + 1;
            const int c = (int)((key >> (2 * (ORACLE_ORDER - L))) & 3);
            b = child0[b] + c;
        }
        leaf_of_target[i] = b;
    }
}
