"""GPU tests of batched shells (sfmm_batch_plan / sfmm_batch_execute).

A batch must give, shell by shell, bitwise the result of the shell's own
plan; the HIP graph recorded on the first execute is replayed several times
with other eager GPU work and synchronisations in between, and every replay
is checked against the eager result."""
import numpy as np
import pytest

import oracle
from paper_2210_07021_amd import skies
from parity_util import check

pytestmark = pytest.mark.gpu


def _sf():
    import paper_2210_07021_amd as sf
    sf.load_library()
    return sf


def _shells():
    return skies.shells(n_shell=5, n_min=3e3, n_max=4e4, nside=16)


def _single(src, q, tgt, **opt):
    import torch
    sf = _sf()
    plan = sf.Plan(src, q, tgt, **opt)
    psi, defl = plan.execute()
    torch.cuda.synchronize()
    plan.close()
    return psi.cpu().numpy(), defl.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32-mixed"])
def test_batch_equals_single_plans_and_replays(precision, oracle_lib):
    import torch
    sf = _sf()
    sh = _shells()
    tol = 1e-8 if precision == 0 else 1e-6
    opt = dict(tolerance=tol, leaf_size=16, precision=precision)
    ref = [_single(*x, **opt) for x in sh]
    b = sf.Batch([x[0] for x in sh], [x[1] for x in sh], [x[2] for x in sh], **opt)
    psi, defl = b.execute()  # direct pass, graph recorded and launched
    torch.cuda.synchronize()
    for i in range(len(sh)):
        assert np.array_equal(psi[i].cpu().numpy(), ref[i][0]) and np.array_equal(defl[i].cpu().numpy(), ref[i][1])
    # replays of the graph, with other eager work between them
    for rep in range(3):
        for x in psi + defl:
            x.fill_(float("nan"))
        torch.cuda.synchronize()
        other = _single(*sh[rep % len(sh)], **opt)  # an unrelated plan on the GPU
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        b.execute(psi, defl)
        torch.cuda.synchronize()
        for i in range(len(sh)):
            assert np.array_equal(psi[i].cpu().numpy(), ref[i][0]), (rep, i)
            assert np.array_equal(defl[i].cpu().numpy(), ref[i][1]), (rep, i)
        assert np.isfinite(junk) and np.isfinite(other[0]).all()
    # new output buffers: recorded again
    psi2, defl2 = b.execute()
    torch.cuda.synchronize()
    assert all(np.array_equal(psi2[i].cpu().numpy(), ref[i][0]) for i in range(len(sh)))
    # one shell against the direct sum
    src, q, tgt = sh[0]
    rp, ra = oracle.direct(src, q, tgt)
    check(f"batch shell 0 precision {precision}", psi2[0].cpu().numpy(), defl2[0].cpu().numpy(), rp, ra, tol)
    st = b.plan(2).stats()
    assert st["n_sources"] == sh[2][0].shape[1]
    b.close()


def test_batch_with_bound_policy_runs_directly(oracle_lib):
    import torch
    sf = _sf()
    sh = _shells()[:3]
    opt = dict(tolerance=1e-8, leaf_size=16, order_policy=sf.SFMM_ORDER_BOUND)
    ref = [_single(*x, **opt) for x in sh]
    b = sf.Batch([x[0] for x in sh], [x[1] for x in sh], [x[2] for x in sh], **opt)
    for _ in range(2):
        psi, defl = b.execute()
        torch.cuda.synchronize()
        for i in range(len(sh)):
            assert np.array_equal(psi[i].cpu().numpy(), ref[i][0])
    b.close()


def test_autotune_picks_a_valid_fast_configuration(oracle_lib, tmp_path):
    sf = _sf()
    from paper_2210_07021_amd import tune
    rng = skies.rng_for(120)
    src = skies.clustered(60000, rng, n_clumps=120)
    q = skies.masses_lognormal(60000, rng)
    tgt = skies.grid(32)
    cache = str(tmp_path / "tune.json")
    best, t_best, table = tune.autotune(src, q, tgt, tolerance=1e-8, leaf_sizes=(16, 32, 64),
                                        segments=(64, 256), repeats=1, cache=cache)
    times = [t for _, t in table]
    print(f"[tune] best {best} {t_best * 1e3:.2f} ms of {len(table)} candidates, "
          f"range {min(times) * 1e3:.2f}..{max(times) * 1e3:.2f} ms", flush=True)
    # leaf sizes, then one order above the tolerance's, then 2 x 2 segments
    assert t_best == min(times) and len(table) == 3 + 1 + 4
    assert all(o.get("order", sf.order_for_tolerance(1e-8)) >= sf.order_for_tolerance(1e-8) for o, _ in table)
    # the cached result comes back without timing
    again, t_again, table2 = tune.autotune(src, q, tgt, tolerance=1e-8, leaf_sizes=(16, 32, 64),
                                           segments=(64, 256), repeats=1, cache=cache)
    assert again == best and t_again == t_best and table2 == []
    psi, defl = _single(src, q, tgt, **best)
    rp, ra = oracle.direct(src, q, tgt[:, ::9])
    check("autotuned", psi[::9], defl[:, ::9], rp, ra, 1e-8)


def test_batch_plan_error_in_one_shell(oracle_lib):
    """A shell with a point off the sphere fails its plan on a worker thread:
    the batch call reports that error (invalid argument, with the message),
    the other workers' plans are released, and a valid batch planned next
    still equals its shells' own plans."""
    import torch
    sf = _sf()
    sh = _shells() + _shells()[:2]
    srcs = [x[0].copy() for x in sh]
    srcs[4][:, 7] *= 1.01  # off the unit sphere by more than the accepted 1e-6
    with pytest.raises(sf.SfmmError) as e:
        sf.Batch(srcs, [x[1] for x in sh], [x[2] for x in sh], tolerance=1e-8, leaf_size=16)
    assert e.value.status == 1 and "sphere" in str(e.value).lower()
    opt = dict(tolerance=1e-8, leaf_size=16)
    b = sf.Batch([x[0] for x in sh], [x[1] for x in sh], [x[2] for x in sh], **opt)
    psi, defl = b.execute()
    torch.cuda.synchronize()
    for i in (0, 4, 6):
        rp, ra = _single(*sh[i], **opt)
        assert np.array_equal(psi[i].cpu().numpy(), rp) and np.array_equal(defl[i].cpu().numpy(), ra)
    b.close()


def test_batch_with_an_empty_shell(oracle_lib):
    """A shell without masses plans and executes like any other (its psi and
    alpha are zero), also inside the recorded graph and its replays."""
    import torch
    sf = _sf()
    sh = _shells()[:3]
    empty = (np.zeros((3, 0)), np.zeros(0), sh[1][2])
    shells = [sh[0], empty, sh[2]]
    opt = dict(tolerance=1e-8, leaf_size=16)
    b = sf.Batch([x[0] for x in shells], [x[1] for x in shells], [x[2] for x in shells], **opt)
    for rep in range(2):  # direct pass + recording, then a replay
        psi, defl = (b.execute() if rep == 0 else b.execute(psi, defl))
        torch.cuda.synchronize()
        assert not psi[1].abs().max().item() and not defl[1].abs().max().item()
        for i in (0, 2):
            rp, ra = _single(*shells[i], **opt)
            assert np.array_equal(psi[i].cpu().numpy(), rp) and np.array_equal(defl[i].cpu().numpy(), ra)
    b.close()
