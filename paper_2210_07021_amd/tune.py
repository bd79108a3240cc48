"""Autotuning of the free parameters of a plan: the leaf size m (Sec. 3.1)
and the work-item sizes of the near field (close leaves per direct-sum item
and per multipole-evaluation item).  The order follows from the tolerance and
is not a free parameter; every candidate meets the same tolerance.

Candidates are timed on the given sky (plan + execute, one untimed warm-up,
the best of `repeats`), and the fastest is returned with the table."""
from __future__ import annotations

import itertools
import time


def autotune(src, q, tgt, tolerance: float = 1e-10, precision: int = 0,
             leaf_sizes=(16, 24, 32, 40, 48, 56, 64, 80), segments=(64, 128, 256), repeats: int = 2, **fixed):
    import torch
    from . import Plan
    src = torch.as_tensor(src, dtype=torch.float64).cuda() if not isinstance(src, torch.Tensor) else src
    q = torch.as_tensor(q, dtype=torch.float64).cuda() if not isinstance(q, torch.Tensor) else q
    tgt = torch.as_tensor(tgt, dtype=torch.float64).cuda() if not isinstance(tgt, torch.Tensor) else tgt
    psi = torch.empty(tgt.shape[1], dtype=torch.float64, device="cuda")
    defl = torch.empty((3, tgt.shape[1]), dtype=torch.float64, device="cuda")

    def step(opts):
        plan = Plan(src, q, tgt, **opts)
        plan.execute(psi, defl)
        plan.close()

    table = []
    # leaf size first (default segments), then the segments at the best leaf size
    best = None
    for m in leaf_sizes:
        opts = dict(fixed, tolerance=tolerance, precision=precision, leaf_size=m)
        table.append((opts, _time(step, opts, repeats)))
    best = min(table, key=lambda r: r[1])[0]
    for sn, sfar in itertools.product(segments, segments):
        opts = dict(best, near_segment=sn, far_segment=sfar)
        table.append((opts, _time(step, opts, repeats)))
    best_opts, best_t = min(table, key=lambda r: r[1])
    return best_opts, best_t, table


def _time(step, opts, repeats):
    import torch
    step(opts)
    torch.cuda.synchronize()
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        step(opts)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return min(ts)
