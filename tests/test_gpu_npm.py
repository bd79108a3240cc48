"""GPU near-particle model (npm_sigma; Sec. 3.1 NPM, Sec. 4.2 Eq. KERNEL)
against the oracle's direct sum over smoothed particles: psi, alpha and the
Hessian, with the particle radius sigma = beta sqrt(4 pi / N) of the paper's
tests (beta = 2 and 5), targets on the grid and on the sources themselves
(the interior centre values); sigma = 0 is bitwise the point-mass plan."""
import numpy as np
import pytest

import oracle
from paper_2210_07021_amd import skies
from parity_util import check, errors

pytestmark = pytest.mark.gpu


def _sf():
    import paper_2210_07021_amd as sf
    sf.load_library()
    return sf


def _case(name):
    if name == "uniform-1e4":
        return skies.workload("uniform-1e4")
    rng = skies.rng_for(102)
    s2 = skies.clustered(50000, rng, n_clumps=100)
    q2 = skies.masses_lognormal(50000, rng)
    t2 = np.concatenate([skies.grid(32), s2[:, :2000]], axis=1)
    return s2, q2, t2


@pytest.mark.parametrize("name,beta", [("uniform-1e4", 2.0), ("clustered-5e4", 5.0)])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32-mixed"])
def test_npm_matches_oracle(name, beta, precision, oracle_lib):
    import torch
    sf = _sf()
    src, q, tgt = _case(name)
    sigma = beta * np.sqrt(4 * np.pi / src.shape[1])
    tol = 1e-10 if precision == 0 else 1e-6
    plan = sf.Plan(src, q, tgt, tolerance=tol, leaf_size=32, precision=precision, npm_sigma=sigma)
    psi, defl, hess = plan.execute_hessian()
    torch.cuda.synchronize()
    st = plan.stats()
    plan.close()
    psi, defl, hess = psi.cpu().numpy(), defl.cpu().numpy(), hess.cpu().numpy()
    rp, ra, rh = oracle.npm(src, q, tgt, sigma)
    check(f"npm {name} sigma {sigma:.4f} precision {precision} p={st['order']}", psi, defl, rp, ra, tol)
    _, eh, _, wh = errors(hess, hess, rh, rh)
    gate = 100 * tol if precision == 0 else 1e-4
    print(f"[npm] {name}: H rel-L2 {eh:.3e}, worst target {wh:.3e}", flush=True)
    assert eh <= gate and wh <= 100 * gate


def test_npm_zero_is_the_point_mass_plan(oracle_lib):
    import torch
    sf = _sf()
    src, q, tgt = _case("uniform-1e4")
    a = sf.Plan(src, q, tgt, tolerance=1e-8, leaf_size=32)
    b = sf.Plan(src, q, tgt, tolerance=1e-8, leaf_size=32, npm_sigma=0.0)
    pa, da = a.execute()
    pb, db = b.execute()
    torch.cuda.synchronize()
    assert torch.equal(pa, pb) and torch.equal(da, db)
    ma, pa2 = a.export_lists()
    mb, pb2 = b.export_lists()
    assert np.array_equal(ma, mb) and np.array_equal(pa2, pb2)
    a.close()
    b.close()


def test_npm_sigma_rejected_out_of_range(oracle_lib):
    sf = _sf()
    src, q, tgt = _case("uniform-1e4")
    for bad in (-0.01, 0.6, float("nan")):
        with pytest.raises(sf.SfmmError) as e:
            sf.Plan(src[:, :100], q[:100], tgt[:, :10], order=8, npm_sigma=bad)
        assert e.value.status == 1
