"""GPU parity of the precision tier (SFMM_FP32_MIXED) against the CPU oracle.

The tier runs the near-field pair sums and the M2L coefficient arithmetic in
FP32 (two-float coordinates, FP64 sums per tile, FP64 C and Q, FP64 M2L on
the coarse levels) and is meant for tolerances of 1e-6 on clustered skies.
Its error against the FP64 direct sum is gated at rel-L2 <= 1e-6 (psi and
alpha), at tolerance 1e-6 and at tolerance 1e-10 (where FP32 arithmetic, not
truncation, sets it).  On a uniform sky of equal masses the zero-mean psi is
small next to its ~13m near-field log terms, all of one sign: their FP32
sums are Kahan-compensated, which brings that case under 1e-6 too.
"""
import numpy as np
import pytest

import oracle
from paper_2210_07021_amd import skies
from parity_util import check

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(src, q, tgt, **opt):
    import torch
    import paper_2210_07021_amd as sf
    sf.load_library()
    plan = sf.Plan(src, q, tgt, **opt)
    psi, defl = plan.execute()
    torch.cuda.synchronize()
    st = plan.stats()
    plan.close()
    return st, psi.cpu().numpy(), defl.cpu().numpy()


def _cases():
    src, q, tgt = skies.workload("uniform-1e4")
    yield "uniform-1e4", src, q, tgt, np.arange(tgt.shape[1])
    rng = skies.rng_for(102)
    s2 = skies.clustered(50000, rng, n_clumps=100)
    q2 = skies.masses_lognormal(50000, rng)
    t2 = np.concatenate([skies.grid(32), s2[:, :2000]], axis=1)
    yield "clustered-5e4", s2, q2, t2, np.arange(t2.shape[1])


@pytest.mark.parametrize("case", ["uniform-1e4", "clustered-5e4"])
def test_fp32_mixed_at_1e6(case, oracle_lib):
    import paper_2210_07021_amd as sf
    name, src, q, tgt, idx = next(c for c in _cases() if c[0] == case)
    ref_p, ref_a = oracle.direct(src, q, tgt)
    bound = 1e-6
    for m in (64, 16):
        st, psi, defl = _run(src, q, tgt, tolerance=1e-6, leaf_size=m, precision=sf.SFMM_FP32_MIXED)
        check(f"fp32 {name} m={m} tol 1e-6 p={st['order']}", psi, defl, ref_p, ref_a, bound)


@pytest.mark.parametrize("case", ["uniform-1e4", "clustered-5e4"])
def test_fp32_mixed_error_stated_at_1e10(case, oracle_lib):
    """At tolerance 1e-10 the tier is limited by FP32 arithmetic: its error is
    gated as at 1e-6; the FP64 path meets 1e-10 on the same input."""
    import paper_2210_07021_amd as sf
    name, src, q, tgt, idx = next(c for c in _cases() if c[0] == case)
    ref_p, ref_a = oracle.direct(src, q, tgt)
    bound = 1e-6
    st, psi, defl = _run(src, q, tgt, tolerance=1e-10, leaf_size=32, precision=sf.SFMM_FP32_MIXED)
    check(f"fp32 {name} tol 1e-10 p={st['order']}", psi, defl, ref_p, ref_a, bound)
    st, psi, defl = _run(src, q, tgt, tolerance=1e-10, leaf_size=32)
    check(f"fp64 {name} tol 1e-10 p={st['order']}", psi, defl, ref_p, ref_a, 1e-10)


def test_fp32_mixed_clustered_1e6_sampled(oracle_lib):
    import paper_2210_07021_amd as sf
    src, q, tgt = skies.workload("clustered-1e6")
    idx = np.random.default_rng(skies.BASE_SEED + 1001).choice(tgt.shape[1], 1000, replace=False)
    ref_p, ref_a = oracle.direct(src, q, tgt[:, idx])
    st, psi, defl = _run(src, q, tgt, tolerance=1e-6, leaf_size=32, precision=sf.SFMM_FP32_MIXED)
    check(f"fp32 clustered-1e6 tol 1e-6 p={st['order']}", psi[idx], defl[:, idx], ref_p, ref_a, 1e-6)


def test_fp32_mixed_reproducible_and_coincident(oracle_lib):
    import paper_2210_07021_amd as sf
    rng = skies.rng_for(108)
    base = skies.uniform(400, rng)
    src = np.concatenate([base, base[:, :50]], axis=1)
    q = skies.masses_lognormal(src.shape[1], rng)
    tgt = np.concatenate([base[:, :100], skies.uniform(200, rng)], axis=1)
    ref_p, ref_a = oracle.direct(src, q, tgt)
    _, p1, d1 = _run(src, q, tgt, tolerance=1e-6, leaf_size=4, precision=sf.SFMM_FP32_MIXED)
    _, p2, d2 = _run(src, q, tgt, tolerance=1e-6, leaf_size=4, precision=sf.SFMM_FP32_MIXED)
    assert np.array_equal(p1, p2) and np.array_equal(d1, d2)
    check("fp32 coincident", p1, d1, ref_p, ref_a, 1e-6)


@pytest.mark.parametrize("lc", ["-1", "2"])
def test_fp32_mixed_coarse_level_override(lc, oracle_lib, monkeypatch):
    """The tier's last FP64 level moved (SFMM_FP32_COARSE_LEVEL): with no FP64
    level at all the FP64 pass has no boxes and the FP32 pass writes every
    local record; the result still meets 1e-6 on both skies."""
    import paper_2210_07021_amd as sf
    monkeypatch.setenv("SFMM_FP32_COARSE_LEVEL", lc)
    for name, src, q, tgt, _ in _cases():
        ref_p, ref_a = oracle.direct(src, q, tgt)
        st, psi, defl = _run(src, q, tgt, tolerance=1e-6, leaf_size=32, precision=sf.SFMM_FP32_MIXED)
        check(f"fp32 {name} last FP64 level {lc}", psi, defl, ref_p, ref_a, 1e-6)
