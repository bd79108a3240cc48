"""CPU oracle for the spherical FMM (arXiv:2210.07021).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never loads it and shares no code with it.

Contents
--------
* ``direct``      plain FP64 direct sum of Eq. SUM / Eq. ALP_PSI (C, OpenMP,
                  Neumaier-compensated), the paper's "PPM" of Sec. 4.1.
* ``hessian``     the same direct sum of the Hessian H of Sec. 2.2 (Eq.
                  GAM_DEF); ``lensing`` turns H into kappa, gamma, mu.
* ``npm``         psi, alpha, H with every source a near-particle-model
                  profile (Eq. KERNEL) of radius sigma.
* ``key`` / ``pix_point`` / ``box_radius``  HEALPix nested geometry (C).
* ``tree`` / ``walk`` / ``locate``  the sphere division of Sec. 3.1,
                  Algorithm 1 of Sec. 3.4 with the MACs of Sec. 3.5 (C).
* ``lemmas``      Lemmas 1-4 of Sec. 3.1-3.3 as printed, and the local
                  evaluation of Sec. 3.6, in numpy FP64.
* ``raytrace``    multi-plane backtracking across layers (Eq. DIS_PRO) with
                  the distortion matrix, on the direct sums above.
* ``nfw``         the analytic NFW halo of Sec. 4.3 (Eq. NFW and its shear),
                  the reference of the sampling-noise experiment.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["direct.c", "healpix.c", "tree.c"]
_HEADERS = ["oracle.h", "oracle_geom.h"]

GAUGE_ZERO_MEAN = 0
GAUGE_RAW = 1


def build(force: bool = True) -> str:
    """Compile the oracle's C sources into ``oracle/liboracle.so``.

    Plain gcc, FP64, no fused multiply-adds (-ffp-contract=off), OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        srcs = [os.path.join(_HERE, s) for s in _SOURCES]
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-o", tmp] + srcs + ["-lquadmath", "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_direct.argtypes = [P, P, i64, P, i64, ctypes.c_int, P, P, ctypes.c_int]
        lib.oracle_direct.restype = None
        lib.oracle_hessian.argtypes = [P, P, i64, P, i64, P, ctypes.c_int]
        lib.oracle_hessian.restype = None
        lib.oracle_npm.argtypes = [P, P, i64, P, i64, ctypes.c_double, ctypes.c_int, P, P, P, ctypes.c_int]
        lib.oracle_npm.restype = None
        lib.oracle_key.argtypes = [ctypes.c_double] * 3 + [ctypes.c_int]
        lib.oracle_key.restype = i64
        lib.oracle_pix_point.argtypes = [ctypes.c_int, i64, ctypes.c_double, ctypes.c_double, P]
        lib.oracle_pix_point.restype = None
        lib.oracle_box_radius.argtypes = [ctypes.c_int, i64]
        lib.oracle_box_radius.restype = ctypes.c_double
        lib.oracle_angdist.argtypes = [P, P]
        lib.oracle_angdist.restype = ctypes.c_double
        lib.oracle_tree.argtypes = [P, i64, ctypes.c_int, ctypes.c_int, P, P, i64,
                                    P, P, P, P, P, P, P, P]
        lib.oracle_tree.restype = i64
        lib.oracle_walk.argtypes = [i64, P, P, P, ctypes.c_double, ctypes.c_double,
                                    i64, P, P, P, i64, P, P, P, P]  # level, pixel, child0
        lib.oracle_walk.restype = ctypes.c_int
        lib.oracle_locate.argtypes = [P, i64, P, P, P, P]
        lib.oracle_locate.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _planes(x, name):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != 2 or x.shape[0] != 3:
        raise ValueError(f"{name} must have shape (3, n)")
    return x


def direct(src, q, tgt, gauge: int = GAUGE_ZERO_MEAN, nthreads: int = 0):
    """Direct sum: (psi[m], defl[3, m]) at targets ``tgt`` (3, m) from sources
    ``src`` (3, n) with masses ``q`` (n,).  Eq. SUM with Eq. GRE_FUN, the
    zero-mean gauge of Eq. STAND_CONDITION by default, alpha = grad psi
    (Eq. ALP_PSI) as a global Cartesian tangent vector."""
    lib = _load()
    src = _planes(src, "src")
    tgt = _planes(tgt, "tgt")
    q = np.ascontiguousarray(q, dtype=np.float64)
    n, m = src.shape[1], tgt.shape[1]
    if q.shape != (n,):
        raise ValueError("q must have shape (n,)")
    psi = np.zeros(m)
    defl = np.zeros((3, m))
    if m:
        lib.oracle_direct(_ptr(src), _ptr(q), n, _ptr(tgt), m, int(gauge),
                          _ptr(psi), _ptr(defl), int(nthreads))
    return psi, defl


def hessian(src, q, tgt, nthreads: int = 0):
    """Hessian of psi (Sec. 2.2, the matrix H of Eq. GAM_DEF) at targets
    ``tgt`` (3, m): (3, m) array (H_11, H_12, H_22) in the basis e_theta,
    e_phi of each target (phi = 0 at an exact pole)."""
    lib = _load()
    src = _planes(src, "src")
    tgt = _planes(tgt, "tgt")
    q = np.ascontiguousarray(q, dtype=np.float64)
    n, m = src.shape[1], tgt.shape[1]
    if q.shape != (n,):
        raise ValueError("q must have shape (n,)")
    hess = np.zeros((3, m))
    if m:
        lib.oracle_hessian(_ptr(src), _ptr(q), n, _ptr(tgt), m, _ptr(hess), int(nthreads))
    return hess


def npm(src, q, tgt, sigma: float, gauge: int = GAUGE_ZERO_MEAN, with_hessian: bool = True,
        nthreads: int = 0):
    """Direct sum with every source a near-particle-model profile of radius
    sigma (Sec. 3.1 NPM, Sec. 4.2 Eq. KERNEL): (psi (m,), defl (3, m), hess
    (3, m) or None)."""
    lib = _load()
    src = _planes(src, "src")
    tgt = _planes(tgt, "tgt")
    q = np.ascontiguousarray(q, dtype=np.float64)
    n, m = src.shape[1], tgt.shape[1]
    psi = np.zeros(m)
    defl = np.zeros((3, m))
    hess = np.zeros((3, m)) if with_hessian else None
    if m:
        lib.oracle_npm(_ptr(src), _ptr(q), n, _ptr(tgt), m, float(sigma), int(gauge), _ptr(psi), _ptr(defl),
                       _ptr(hess) if with_hessian else None, int(nthreads))
    return psi, defl, hess


def lensing(hess):
    """Convergence, shear and magnification from H (Eq. GAM_DEF and the
    magnification of Sec. 2.2): kappa - kappa_bar = tr H, gamma_1 =
    (H_11 - H_22)/2, gamma_2 = H_12, mu = 1/det(I - H).  Returns (4, m)."""
    h11, h12, h22 = np.asarray(hess)
    kk = h11 + h22
    g1 = 0.5 * (h11 - h22)
    g2 = h12
    mu = 1.0 / ((1.0 - 0.5 * kk) ** 2 - g1 * g1 - g2 * g2)
    return np.stack([kk, g1, g2, mu])


def key(x, y, z, order: int = 29) -> int:
    """HEALPix nested index of the unit vector (x, y, z) at ``order``."""
    return int(_load().oracle_key(float(x), float(y), float(z), int(order)))


def keys(pts, order: int = 29) -> np.ndarray:
    pts = _planes(pts, "pts")
    lib = _load()
    return np.array([lib.oracle_key(pts[0, i], pts[1, i], pts[2, i], order)
                     for i in range(pts.shape[1])], dtype=np.int64)


def pix_point(order: int, pix: int, fx: float = 0.5, fy: float = 0.5) -> np.ndarray:
    out = np.zeros(3)
    _load().oracle_pix_point(int(order), int(pix), float(fx), float(fy), _ptr(out))
    return out


def box_radius(order: int, pix: int) -> float:
    return float(_load().oracle_box_radius(int(order), int(pix)))


def angdist(a, b) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return float(_load().oracle_angdist(_ptr(a), _ptr(b)))


class Tree:
    """Box table of the adaptive tree, ordered by (level, pixel)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    @property
    def nbox(self) -> int:
        return len(self.level)

    def is_leaf(self) -> np.ndarray:
        return self.child0 < 0


def tree(src, m: int, max_level: int = 29) -> Tree:
    """Sphere division of Sec. 3.1 over the sources ``src`` (3, n)."""
    lib = _load()
    src = _planes(src, "src")
    n = src.shape[1]
    keys_out = np.zeros(n, dtype=np.uint64)
    perm = np.zeros(n, dtype=np.int64)
    cap = max(64, 4 * (n // max(m, 1)) + 64)
    while True:
        level = np.zeros(cap, dtype=np.int32)
        pixel = np.zeros(cap, dtype=np.int64)
        first = np.zeros(cap, dtype=np.int64)
        count = np.zeros(cap, dtype=np.int64)
        parent = np.zeros(cap, dtype=np.int64)
        child0 = np.zeros(cap, dtype=np.int64)
        centre = np.zeros((3, cap))
        radius = np.zeros(cap)
        nb = lib.oracle_tree(_ptr(src), n, int(m), int(max_level), _ptr(keys_out), _ptr(perm),
                             cap, _ptr(level), _ptr(pixel), _ptr(first), _ptr(count),
                             _ptr(parent), _ptr(child0), _ptr(centre), _ptr(radius))
        if nb >= 0:
            break
        cap *= 2
    return Tree(level=level[:nb].copy(), pixel=pixel[:nb].copy(), first=first[:nb].copy(),
                count=count[:nb].copy(), parent=parent[:nb].copy(), child0=child0[:nb].copy(),
                centre=np.ascontiguousarray(centre[:, :nb]), radius=radius[:nb].copy(),
                keys=keys_out, perm=perm, m=int(m), max_level=int(max_level))


def walk(t: Tree, c_s: float = 2.0, c_t: float = 0.5):
    """Algorithm 1 from (root, root).  Returns (m2l (k, 2), p2p (k, 2),
    min_margin) with columns (source box, target box), in recursion order."""
    lib = _load()
    nb = t.nbox
    cap_m, cap_p = 64 * nb + 1024, 16 * nb + 1024
    while True:
        ms = np.zeros(cap_m, dtype=np.int64)
        mt = np.zeros(cap_m, dtype=np.int64)
        ps = np.zeros(cap_p, dtype=np.int64)
        pt = np.zeros(cap_p, dtype=np.int64)
        nm = ctypes.c_int64(0)
        npp = ctypes.c_int64(0)
        mm = ctypes.c_double(0.0)
        rc = lib.oracle_walk(nb, _ptr(t.level), _ptr(t.pixel), _ptr(t.child0),
                             float(c_s), float(c_t), cap_m, _ptr(ms), _ptr(mt),
                             ctypes.byref(nm), cap_p, _ptr(ps), _ptr(pt), ctypes.byref(npp),
                             ctypes.byref(mm))
        if rc == 0:
            break
        cap_m = max(cap_m, nm.value + 16)
        cap_p = max(cap_p, npp.value + 16)
    m2l = np.stack([ms[:nm.value], mt[:nm.value]], axis=1)
    p2p = np.stack([ps[:npp.value], pt[:npp.value]], axis=1)
    return m2l, p2p, mm.value


def locate(t: Tree, tgt):
    """Leaf box of every target (3, m) and the targets' order-29 keys."""
    lib = _load()
    tgt = _planes(tgt, "tgt")
    m = tgt.shape[1]
    leaf = np.zeros(m, dtype=np.int64)
    k = np.zeros(m, dtype=np.uint64)
    if m:
        lib.oracle_locate(_ptr(tgt), m, _ptr(t.child0), _ptr(t.level), _ptr(leaf), _ptr(k))
    return leaf, k
