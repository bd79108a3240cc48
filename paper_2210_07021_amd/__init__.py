"""Python binding of libsfmm, the spherical FMM (arXiv:2210.07021) on MI355X.

Argument marshalling only: every step of the computation runs in the HIP
library ``libsfmm.so`` (built in-tree by ``paper_2210_07021_amd.build``).
PyTorch provides device memory and the stream.  The names follow the C ABI in
``include/sfmm.h``; :class:`Plan` is a small convenience wrapper.

There is no fallback: importing works without the library, but any call
raises if ``libsfmm.so`` has not been built or no GPU is present.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfmm.so")

SFMM_OK = 0
SFMM_ERR_INVALID_ARG = 1
SFMM_ERR_TOLERANCE_NOT_MET = 4
SFMM_GAUGE_ZERO_MEAN = 0
SFMM_GAUGE_RAW = 1
SFMM_FP64 = 0
SFMM_FP32_MIXED = 1
SFMM_ORDER_FIXED = 0
SFMM_ORDER_BOUND = 1
SFMM_ORDER_LEARNED = 2
MLP_IN = 8
MLP_HIDDEN = 64
MLP_WEIGHTS = MLP_HIDDEN * MLP_IN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1


class SfmmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"sfmm status {status}: {message}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("tolerance", ctypes.c_double),
        ("leaf_size", ctypes.c_int32),
        ("c_s", ctypes.c_double),
        ("c_t", ctypes.c_double),
        ("max_level", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("psi_gauge", ctypes.c_int32),
        ("order_policy", ctypes.c_int32),
        ("mlp_weights", ctypes.c_void_p),
        ("near_segment", ctypes.c_int32),
        ("far_segment", ctypes.c_int32),
        ("judge_targets", ctypes.c_int32),
        ("no_fallback", ctypes.c_int32),
        ("npm_sigma", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_sources", ctypes.c_int64),
        ("n_targets", ctypes.c_int64),
        ("n_boxes", ctypes.c_int64),
        ("n_leaves", ctypes.c_int64),
        ("n_levels", ctypes.c_int64),
        ("n_m2l", ctypes.c_int64),
        ("n_p2p", ctypes.c_int64),
        ("n_target_leaves", ctypes.c_int64),
        ("n_p2p_pairs", ctypes.c_int64),
        ("n_m2p_evals", ctypes.c_int64),
        ("order", ctypes.c_int32),
        ("leaf_size", ctypes.c_int32),
        ("q_total", ctypes.c_double),
        ("m2l_order_sq", ctypes.c_int64),
        ("judge_psi", ctypes.c_double),
        ("judge_alpha", ctypes.c_double),
        ("judge_targets", ctypes.c_int32),
        ("fell_back", ctypes.c_int32),
        ("execute_scratch_bytes", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every exported symbol of include/sfmm.h with its ctypes signature
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
SIGNATURES = {
    "sfmm_default_options": (None, [ctypes.POINTER(Options)]),
    "sfmm_plan": (ctypes.c_int, [_P, _P, _I64, _P, _I64, ctypes.POINTER(Options), _P, ctypes.POINTER(_P)]),
    "sfmm_execute": (ctypes.c_int, [_P, _P, _P, _P]),
    "sfmm_execute_noalloc": (ctypes.c_int, [_P, _P, _P, _P]),
    "sfmm_execute_hessian": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "sfmm_lensing": (ctypes.c_int, [_P, _I64, _P, _P]),
    "sfmm_thetaphi_to_xyz": (ctypes.c_int, [_P, _P, _I64, _P]),
    "sfmm_defl_to_thetaphi": (ctypes.c_int, [_P, _P, _P, _I64, _P]),
    "sfmm_raytrace": (ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P, _P, _I64, _P, ctypes.POINTER(Options), _P]),
    "sfmm_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(Stats)]),
    "sfmm_export_boxes": (ctypes.c_int, [_P] * 9),
    "sfmm_export_lists": (ctypes.c_int, [_P] * 5),
    "sfmm_export_keys": (ctypes.c_int, [_P] * 6),
    "sfmm_export_work": (ctypes.c_int, [_P] * 4),
    "sfmm_export_expansions": (ctypes.c_int, [_P] * 3),
    "sfmm_batch_plan": (ctypes.c_int, [ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.POINTER(Options), _P,
                                       ctypes.POINTER(_P)]),
    "sfmm_batch_execute": (ctypes.c_int, [_P, _P, _P, _P]),
    "sfmm_batch_plan_at": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(_P)]),
    "sfmm_batch_destroy": (None, [_P]),
    "sfmm_order_samples": (ctypes.c_int, [_P, _I64, ctypes.c_uint64, _P, _P, _P]),
    "sfmm_mlp_init": (None, [ctypes.c_uint64, _P]),
    "sfmm_mlp_train": (ctypes.c_int, [_P, _P, _I64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                      ctypes.c_uint64, _P, _P]),
    "sfmm_mlp_forward": (ctypes.c_int, [_P, _P, _I64, ctypes.c_int32, _P]),
    "sfmm_mlp_grad": (ctypes.c_int, [_P, _P, _P, _I64, _P, _P]),
    "sfmm_destroy": (None, [_P]),
    "sfmm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sfmm_last_error": (ctypes.c_char_p, []),
    "sfmm_order_for_tolerance": (ctypes.c_int32, [ctypes.c_double]),
    "sfmm_profile_enable": (None, [ctypes.c_int32]),
    "sfmm_profile_reset": (None, []),
    "sfmm_profile_read": (None, [_P, _P]),
}

NUM_STAGES = 13
STAGES = ["src_keys_sort", "tree", "geometry", "walk", "lists", "targets",
          "p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "m2p"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsfmm.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is None:
        # torch carries its own HIP runtime; the two share the device only when
        # torch's is up first (device tensors are passed to this library)
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        if not os.path.exists(path):
            raise RuntimeError(f"libsfmm.so not found at {path}: build it with "
                               "`python -m paper_2210_07021_amd.build` (no fallback exists)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != SFMM_OK:
        lib = load_library()
        raise SfmmError(status, lib.sfmm_last_error().decode(errors="replace"))


def default_options(**overrides) -> Options:
    opt = Options()
    load_library().sfmm_default_options(ctypes.byref(opt))
    for k, v in overrides.items():
        if not hasattr(opt, k):
            raise TypeError(f"unknown option {k!r}")
        setattr(opt, k, v)
    return opt


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def mlp_init(seed: int = 0) -> np.ndarray:
    """He-initialised order-network weights (sfmm_mlp_init)."""
    w = np.zeros(MLP_WEIGHTS, np.float32)
    load_library().sfmm_mlp_init(ctypes.c_uint64(seed), w.ctypes.data_as(_P))
    return w


def mlp_train(features, labels, weights, epochs=20, batch=1024, lr=1e-3, seed=0):
    """Train the order network on the GPU (sfmm_mlp_train); returns (weights,
    mean loss per epoch)."""
    f = _f32(features)
    l = _f32(labels)
    n = l.shape[0]
    if f.shape != (n, MLP_IN):
        raise ValueError("features must be [n][8]")
    w = _f32(weights, (MLP_WEIGHTS,)).copy()
    loss = np.zeros(max(epochs, 1), np.float32)
    _check(load_library().sfmm_mlp_train(f.ctypes.data_as(_P), l.ctypes.data_as(_P), n, epochs, batch,
                                         ctypes.c_float(lr), ctypes.c_uint64(seed), w.ctypes.data_as(_P),
                                         loss.ctypes.data_as(_P)))
    return w, loss[:epochs]


def mlp_forward(weights, features, bf16=False) -> np.ndarray:
    f = _f32(features)
    w = _f32(weights, (MLP_WEIGHTS,))
    y = np.zeros(f.shape[0], np.float32)
    _check(load_library().sfmm_mlp_forward(w.ctypes.data_as(_P), f.ctypes.data_as(_P), f.shape[0],
                                           1 if bf16 else 0, y.ctypes.data_as(_P)))
    return y


def mlp_grad(weights, features, labels):
    """Gradient of the mean training loss and the loss (sfmm_mlp_grad)."""
    f = _f32(features)
    l = _f32(labels)
    w = _f32(weights, (MLP_WEIGHTS,))
    g = np.zeros(MLP_WEIGHTS, np.float32)
    loss = ctypes.c_float()
    _check(load_library().sfmm_mlp_grad(w.ctypes.data_as(_P), f.ctypes.data_as(_P), l.ctypes.data_as(_P),
                                        l.shape[0], g.ctypes.data_as(_P), ctypes.byref(loss)))
    return g, float(loss.value)


def lensing(hess, stream=None):
    """(kappa - kappa_bar, gamma_1, gamma_2, mu) (4, M) on the GPU from a
    Hessian (3, M) of Plan.execute_hessian (sfmm_lensing)."""
    import torch
    hess = hess.contiguous()
    m = int(hess.shape[1])
    out = torch.empty((4, m), dtype=torch.float64, device=hess.device)
    _check(load_library().sfmm_lensing(ctypes.c_void_p(hess.data_ptr() if m else 0), m,
                                       ctypes.c_void_p(out.data_ptr() if m else 0), _stream_handle(stream)))
    return out


def _host_f64(a, shape0=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape0 is not None and (a.ndim != 2 or a.shape[0] != shape0):
        raise ValueError(f"expected an array of shape ({shape0}, n)")
    return a


def thetaphi_to_xyz(theta, phi):
    """Unit vectors (3, n) of colatitudes and longitudes (radians), host numpy
    (sfmm_thetaphi_to_xyz)."""
    t, f = _host_f64(theta).ravel(), _host_f64(phi).ravel()
    if t.shape != f.shape:
        raise ValueError("theta and phi differ in length")
    out = np.empty((3, t.size))
    _check(load_library().sfmm_thetaphi_to_xyz(t.ctypes.data, f.ctypes.data, t.size, out.ctypes.data))
    return out


def defl_to_thetaphi(xyz, defl, phi=None):
    """(alpha_theta, alpha_phi) (2, n) of tangent vectors defl (3, n) at unit
    vectors xyz (3, n), host numpy; phi (n,) fixes the basis at exact poles
    (sfmm_defl_to_thetaphi)."""
    x, d = _host_f64(xyz, 3), _host_f64(defl, 3)
    if x.shape != d.shape:
        raise ValueError("xyz and defl differ in shape")
    n = x.shape[1]
    f = None if phi is None else _host_f64(phi).ravel()
    if f is not None and f.size != n:
        raise ValueError("phi has the wrong length")
    out = np.empty((2, n))
    _check(load_library().sfmm_defl_to_thetaphi(x.ctypes.data, d.ctypes.data, None if f is None else f.ctypes.data,
                                                 n, out.ctypes.data))
    return out


def raytrace(layers, weights, rays, distortion=True, **options):
    """Multi-plane backtracking (sfmm_raytrace): layers = [(src (3, N_i), q
    (N_i,)), ...], weights = f_K(r_s - r_i) / f_K(r_s) per layer, rays (3, M)
    the observed positions.  Returns (final rays (3, M), distortion matrix
    (4, M) or None) as CUDA float64 tensors."""
    import torch
    lib = load_library()
    n = len(layers)
    if n == 0 or len(weights) != n:
        raise ValueError("need one weight per layer and at least one layer")
    srcs = [_dev_planes(x[0], "src") for x in layers]
    qs = [_dev_planes(x[1], "q") for x in layers]
    r = _dev_planes(rays, "rays").clone()
    m = int(r.shape[1])
    dist = torch.empty((4, m), dtype=torch.float64, device="cuda") if distortion else None
    arr = lambda xs: (ctypes.c_void_p * n)(*[x.data_ptr() if x.numel() else 0 for x in xs])
    ps, qq = arr(srcs), arr(qs)
    Ns = (ctypes.c_int64 * n)(*[int(x.shape[1]) for x in srcs])
    ws = (ctypes.c_double * n)(*[float(w) for w in weights])
    weights_ = options.pop("mlp_weights", None)
    opt = default_options(**options)
    if weights_ is not None:
        keep = _f32(weights_, (MLP_WEIGHTS,))
        opt.mlp_weights = keep.ctypes.data
    _check(lib.sfmm_raytrace(n, ps, qq, Ns, ws, ctypes.c_void_p(r.data_ptr() if m else 0), m,
                             ctypes.c_void_p(dist.data_ptr() if (dist is not None and m) else 0),
                             ctypes.byref(opt), _stream_handle()))
    return r, dist


def order_for_tolerance(tol: float) -> int:
    return int(load_library().sfmm_order_for_tolerance(float(tol)))


def profile_enable(on: bool = True):
    load_library().sfmm_profile_enable(1 if on else 0)


def profile_reset():
    load_library().sfmm_profile_reset()


def profile_read() -> dict:
    """Per-stage {name: (total ms, calls)} accumulated while enabled."""
    ms = np.zeros(NUM_STAGES)
    calls = np.zeros(NUM_STAGES, np.int64)
    load_library().sfmm_profile_read(ms.ctypes.data_as(_P), calls.ctypes.data_as(_P))
    return {n: (float(ms[i]), int(calls[i])) for i, n in enumerate(STAGES)}


def _dev_planes(x, name):
    import torch
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64)
    if x.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not x.is_cuda:
        x = x.to("cuda")
    return x.contiguous()


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A planned sFMM evaluation: sources (3, N), masses (N,), targets (3, M),
    as torch CUDA float64 tensors (or host arrays, copied to the device)."""

    def __init__(self, src, q, tgt, stream=None, **options):
        import torch
        self._lib = load_library()
        self.src = _dev_planes(src, "src")
        self.q = _dev_planes(q, "q")
        self.tgt = _dev_planes(tgt, "tgt")
        if self.src.dim() != 2 or self.src.shape[0] != 3 or self.tgt.dim() != 2 or self.tgt.shape[0] != 3:
            raise ValueError("src and tgt must have shape (3, n)")
        if self.q.shape != (self.src.shape[1],):
            raise ValueError("q must have shape (N,)")
        self.N = int(self.src.shape[1])
        self.M = int(self.tgt.shape[1])
        weights = options.pop("mlp_weights", None)
        self.options = default_options(**options)
        if weights is not None:
            # read by sfmm_plan only; kept alive until then
            self._mlp_weights = _f32(weights, (MLP_WEIGHTS,))
            self.options.mlp_weights = self._mlp_weights.ctypes.data
        self._stream = stream
        self._h = ctypes.c_void_p()
        _check(self._lib.sfmm_plan(
            ctypes.c_void_p(self.src.data_ptr() if self.N else 0),
            ctypes.c_void_p(self.q.data_ptr() if self.N else 0), self.N,
            ctypes.c_void_p(self.tgt.data_ptr() if self.M else 0), self.M,
            ctypes.byref(self.options), _stream_handle(stream), ctypes.byref(self._h)))
        self._torch = torch

    def execute(self, psi=None, defl=None, stream=None):
        """Returns (psi (M,), defl (3, M)) as CUDA float64 tensors."""
        t = self._torch
        if psi is None:
            psi = t.empty(self.M, dtype=t.float64, device="cuda")
        if defl is None:
            defl = t.empty((3, self.M), dtype=t.float64, device="cuda")
        _check(self._lib.sfmm_execute(self._h, ctypes.c_void_p(psi.data_ptr() if self.M else 0),
                                      ctypes.c_void_p(defl.data_ptr() if self.M else 0),
                                      _stream_handle(stream if stream is not None else self._stream)))
        return psi, defl

    def execute_hessian(self, psi=None, defl=None, hess=None, stream=None):
        """Returns (psi (M,), defl (3, M), hess (3, M)): hess = (H_11, H_12,
        H_22) of Sec. 2.2 in each target's e_theta, e_phi basis."""
        t = self._torch
        if psi is None:
            psi = t.empty(self.M, dtype=t.float64, device="cuda")
        if defl is None:
            defl = t.empty((3, self.M), dtype=t.float64, device="cuda")
        if hess is None:
            hess = t.empty((3, self.M), dtype=t.float64, device="cuda")
        _check(self._lib.sfmm_execute_hessian(self._h, ctypes.c_void_p(psi.data_ptr() if self.M else 0),
                                              ctypes.c_void_p(defl.data_ptr() if self.M else 0),
                                              ctypes.c_void_p(hess.data_ptr() if self.M else 0),
                                              _stream_handle(stream if stream is not None else self._stream)))
        return psi, defl, hess

    def stats(self) -> dict:
        s = Stats()
        _check(self._lib.sfmm_stats_get(self._h, ctypes.byref(s)))
        return s.as_dict()

    def export_boxes(self) -> dict:
        nb = self.stats()["n_boxes"]
        out = dict(level=np.zeros(nb, np.int32), pixel=np.zeros(nb, np.int64), first=np.zeros(nb, np.int64),
                   count=np.zeros(nb, np.int64), parent=np.zeros(nb, np.int64), child0=np.zeros(nb, np.int64),
                   centre=np.zeros((3, nb)), radius=np.zeros(nb))
        _check(self._lib.sfmm_export_boxes(self._h, *[a.ctypes.data_as(_P) for a in out.values()]))
        return out

    def export_lists(self):
        st = self.stats()
        m2l = np.zeros((2, st["n_m2l"]), np.int64)
        p2p = np.zeros((2, st["n_p2p"]), np.int64)
        _check(self._lib.sfmm_export_lists(self._h, m2l[0].ctypes.data_as(_P), m2l[1].ctypes.data_as(_P),
                                           p2p[0].ctypes.data_as(_P), p2p[1].ctypes.data_as(_P)))
        return m2l.T.copy(), p2p.T.copy()

    def export_keys(self) -> dict:
        out = dict(src_keys=np.zeros(self.N, np.uint64), src_perm=np.zeros(self.N, np.int64),
                   tgt_keys=np.zeros(self.M, np.uint64), tgt_perm=np.zeros(self.M, np.int64),
                   tgt_leaf=np.zeros(self.M, np.int64))
        _check(self._lib.sfmm_export_keys(self._h, *[a.ctypes.data_as(_P) for a in out.values()]))
        return out

    def order_samples(self, n: int, seed: int = 0, with_pairs: bool = False):
        """Features [n][8] and exact order labels [n] of n sampled FMM acts of
        this executed plan (sfmm_order_samples), and their (target, source)
        boxes [n][2] if asked."""
        f = np.zeros((n, MLP_IN), np.float32)
        l = np.zeros(n, np.float32)
        pr = np.zeros((n, 2), np.int64)
        _check(self._lib.sfmm_order_samples(self._h, n, ctypes.c_uint64(seed), f.ctypes.data_as(_P),
                                            l.ctypes.data_as(_P), pr.ctypes.data_as(_P) if with_pairs else None))
        return (f, l, pr) if with_pairs else (f, l)

    def export_work(self) -> dict:
        nb = self.stats()["n_boxes"]
        out = dict(tgt_count=np.zeros(nb, np.int64), pairs=np.zeros(nb, np.int64), evals=np.zeros(nb, np.int64))
        _check(self._lib.sfmm_export_work(self._h, *[a.ctypes.data_as(_P) for a in out.values()]))
        return out

    def export_expansions(self):
        st = self.stats()
        w = 2 * st["order"] + 2
        mult = np.zeros((st["n_boxes"], w))
        loc = np.zeros((st["n_boxes"], w))
        _check(self._lib.sfmm_export_expansions(self._h, mult.ctypes.data_as(_P), loc.ctypes.data_as(_P)))
        return mult, loc

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.sfmm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sfmm(src, q, tgt, **options):
    """One-shot evaluation: plan + execute; returns (psi, defl) on the GPU."""
    p = Plan(src, q, tgt, **options)
    try:
        return p.execute()
    finally:
        p.close()


class _PlanView(Plan):
    """A plan owned by a Batch (stats and exports only)."""

    def __init__(self, batch, i):
        self._lib = batch._lib
        self._h = ctypes.c_void_p()
        _check(self._lib.sfmm_batch_plan_at(batch._h, i, ctypes.byref(self._h)))
        self.N, self.M = batch.N[i], batch.M[i]
        self._torch = batch._torch
        self._stream = None

    def close(self):
        self._h = ctypes.c_void_p()  # the batch owns it


class Batch:
    """Several independent spheres (shells) planned together; execute() runs
    all of them, replaying a recorded HIP graph after the first call
    (sfmm_batch_plan / sfmm_batch_execute)."""

    def __init__(self, srcs, qs, tgts, **options):
        import torch
        self._lib = load_library()
        self._torch = torch
        n = len(srcs)
        if not (len(qs) == len(tgts) == n) or n == 0:
            raise ValueError("need as many masses and target sets as source sets (>= 1)")
        self.src = [_dev_planes(x, "src") for x in srcs]
        self.q = [_dev_planes(x, "q") for x in qs]
        self.tgt = [_dev_planes(x, "tgt") for x in tgts]
        self.N = [int(x.shape[1]) for x in self.src]
        self.M = [int(x.shape[1]) for x in self.tgt]
        weights = options.pop("mlp_weights", None)
        self.options = default_options(**options)
        if weights is not None:
            self._mlp_weights = _f32(weights, (MLP_WEIGHTS,))
            self.options.mlp_weights = self._mlp_weights.ctypes.data
        arr = lambda xs: (ctypes.c_void_p * n)(*[x.data_ptr() if x.numel() else 0 for x in xs])
        self._ptrs = (arr(self.src), arr(self.q), arr(self.tgt))
        Ns = (ctypes.c_int64 * n)(*self.N)
        Ms = (ctypes.c_int64 * n)(*self.M)
        self._h = ctypes.c_void_p()
        _check(self._lib.sfmm_batch_plan(n, self._ptrs[0], self._ptrs[1], Ns, self._ptrs[2], Ms,
                                         ctypes.byref(self.options), None, ctypes.byref(self._h)))
        self.n = n

    def execute(self, psi=None, defl=None):
        """Returns lists of psi (M_i,) and defl (3, M_i) CUDA float64 tensors;
        pass the same output tensors again to replay the recorded graph."""
        t = self._torch
        if psi is None:
            psi = [t.empty(m, dtype=t.float64, device="cuda") for m in self.M]
        if defl is None:
            defl = [t.empty((3, m), dtype=t.float64, device="cuda") for m in self.M]
        pp = (ctypes.c_void_p * self.n)(*[x.data_ptr() for x in psi])
        dp = (ctypes.c_void_p * self.n)(*[x.data_ptr() for x in defl])
        t.cuda.synchronize()  # inputs written by torch are visible to the batch's stream
        _check(self._lib.sfmm_batch_execute(self._h, pp, dp, None))
        return psi, defl

    def plan(self, i: int) -> Plan:
        return _PlanView(self, i)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.sfmm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

