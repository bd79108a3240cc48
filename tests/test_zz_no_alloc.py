"""The no-allocation execute (sfmm_execute_noalloc) against sfmm_execute,
through the C ABI: bitwise the same psi and alpha, on two plans in a row, the
second smaller, so the shared static scratch carries the first call's
contents into the second."""
import ctypes

import numpy as np
import pytest

from paper_2210_07021_amd import skies

pytestmark = pytest.mark.gpu


def _plan(lib, sf, src, q, tgt, **opt):
    import torch
    o = sf.default_options(**opt)
    h = ctypes.c_void_p()
    st = lib.sfmm_plan(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(q.data_ptr()), src.shape[1],
                       ctypes.c_void_p(tgt.data_ptr()), tgt.shape[1], ctypes.byref(o),
                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
    assert st == 0, lib.sfmm_last_error()
    return h


def _exec(lib, fn, h, M):
    import torch
    psi = torch.full((M,), float("nan"), dtype=torch.float64, device="cuda")
    defl = torch.full((3, M), float("nan"), dtype=torch.float64, device="cuda")
    st = getattr(lib, fn)(h, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(defl.data_ptr()),
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.sfmm_last_error()
    torch.cuda.synchronize()
    return psi.cpu().numpy(), defl.cpu().numpy()


def _case(n, nside, seed, scale_clumps):
    import torch
    rng = skies.rng_for(seed)
    src = skies.clustered(n, rng, n_clumps=scale_clumps)
    q = skies.masses_lognormal(n, rng)
    tgt = np.concatenate([skies.grid(nside), src[:, :1000]], axis=1)
    return torch.from_numpy(src).cuda(), torch.from_numpy(q).cuda(), torch.from_numpy(tgt).cuda()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32-mixed"])
def test_noalloc_execute_matches_execute(precision):
    import torch
    import paper_2210_07021_amd as sf
    lib = sf.load_library()
    # two plans in a row, the second smaller (fewer boxes, targets and slots)
    for n, nside, seed in ((200000, 64, 400), (30000, 16, 401)):
        src, q, tgt = _case(n, nside, seed, max(20, n // 500))
        M = tgt.shape[1]
        h = _plan(lib, sf, src, q, tgt, tolerance=1e-10 if precision == 0 else 1e-6, leaf_size=24,
                  precision=precision, near_segment=16, far_segment=16)
        stats = sf.Stats()
        assert lib.sfmm_stats_get(h, ctypes.byref(stats)) == 0
        print(f"[noalloc] N={n} M={M} precision {precision}: scratch {stats.execute_scratch_bytes} bytes",
              flush=True)
        assert 0 < stats.execute_scratch_bytes <= 256 << 20
        a_psi, a_defl = _exec(lib, "sfmm_execute", h, M)
        b_psi, b_defl = _exec(lib, "sfmm_execute_noalloc", h, M)
        c_psi, c_defl = _exec(lib, "sfmm_execute_noalloc", h, M)  # again: stale scratch contents
        assert np.isfinite(a_psi).all() and np.isfinite(a_defl).all()
        assert np.array_equal(a_psi, b_psi) and np.array_equal(a_defl, b_defl)
        assert np.array_equal(a_psi, c_psi) and np.array_equal(a_defl, c_defl)
        lib.sfmm_destroy(h)


def test_noalloc_rejects_order_policies():
    import paper_2210_07021_amd as sf
    lib = sf.load_library()
    src, q, tgt = _case(5000, 8, 402, 20)
    h = _plan(lib, sf, src, q, tgt, tolerance=1e-6, leaf_size=16, order_policy=sf.SFMM_ORDER_BOUND)
    import torch
    psi = torch.empty(tgt.shape[1], dtype=torch.float64, device="cuda")
    defl = torch.empty((3, tgt.shape[1]), dtype=torch.float64, device="cuda")
    st = lib.sfmm_execute_noalloc(h, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(defl.data_ptr()), None)
    assert st == 1  # SFMM_ERR_INVALID_ARG
    assert b"fixed order" in lib.sfmm_last_error()
    lib.sfmm_destroy(h)
