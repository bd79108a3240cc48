"""Autotuning of the free parameters of a plan: the leaf size m (Sec. 3.1),
the expansion order at or above the one the tolerance needs (Eq. MUL_ERR),
and the work-item sizes of the near field (close leaves per direct-sum item
and per multipole-evaluation item, the tile shapes of the pair sums).  Every
candidate meets the same tolerance: the order map is monotone, so an order
above the tolerance's order only trades far-field work for a larger share of
close leaves taken through their expansions.

Candidates are timed on the given sky (plan + execute, one untimed warm-up,
the best of `repeats`), and the fastest is returned with the table.  With a
`cache` path the result is kept in a JSON file under a key of the GPU, the
problem's size class and the options, and a later call with the same key
returns it without timing (the tuning survives the process)."""
from __future__ import annotations

import itertools
import json
import math
import os
import time


def autotune(src, q, tgt, tolerance: float = 1e-10, precision: int = 0,
             leaf_sizes=(16, 24, 32, 40, 48, 56, 64, 80), segments=(64, 128, 256), orders=None,
             repeats: int = 2, cache: str | None = None, **fixed):
    """Returns (options, seconds, table).  orders: candidate orders (None:
    the tolerance's own order and that plus two); a cached result comes back
    with an empty table."""
    import torch
    from . import Plan, order_for_tolerance
    src = torch.as_tensor(src, dtype=torch.float64).cuda() if not isinstance(src, torch.Tensor) else src
    q = torch.as_tensor(q, dtype=torch.float64).cuda() if not isinstance(q, torch.Tensor) else q
    tgt = torch.as_tensor(tgt, dtype=torch.float64).cuda() if not isinstance(tgt, torch.Tensor) else tgt
    key = None
    if cache is not None:
        key = cache_key(torch.cuda.get_device_name(src.device), src.shape[1], tgt.shape[1], tolerance, precision,
                        fixed)
        hit = cache_load(cache, key)
        if hit is not None:
            return hit["options"], hit["seconds"], []
    psi = torch.empty(tgt.shape[1], dtype=torch.float64, device=src.device)
    defl = torch.empty((3, tgt.shape[1]), dtype=torch.float64, device=src.device)

    def step(opts):
        plan = Plan(src, q, tgt, **opts)
        plan.execute(psi, defl)
        plan.close()

    p0 = order_for_tolerance(tolerance)
    if orders is None:
        orders = (p0, min(p0 + 2, 48))
    orders = sorted({int(p) for p in orders if p >= p0})
    if not orders:
        raise ValueError(f"every candidate order is below {p0}, the order the tolerance needs")
    table = []
    # leaf size first (the tolerance's order, default segments), then the
    # orders at the best leaf size, then the segments at the best of those
    for m in leaf_sizes:
        opts = dict(fixed, tolerance=tolerance, precision=precision, leaf_size=m)
        table.append((opts, _time(step, opts, repeats)))
    best = min(table, key=lambda r: r[1])[0]
    for p in orders[1:]:
        opts = dict(best, order=p)
        table.append((opts, _time(step, opts, repeats)))
    best = min(table, key=lambda r: r[1])[0]
    for sn, sfar in itertools.product(segments, segments):
        opts = dict(best, near_segment=sn, far_segment=sfar)
        table.append((opts, _time(step, opts, repeats)))
    best_opts, best_t = min(table, key=lambda r: r[1])
    if cache is not None:
        cache_store(cache, key, {"options": best_opts, "seconds": best_t})
    return best_opts, best_t, table


def cache_key(device: str, n: int, m: int, tolerance: float, precision: int, fixed: dict) -> str:
    """Key of a tuning result: the GPU's name, N and M rounded to a quarter
    decade (size class), the tolerance, the precision mode and any fixed
    options."""
    def cls(x):
        return "0" if x <= 0 else f"{round(4 * math.log10(x)) / 4:.2f}"
    extra = ",".join(f"{k}={fixed[k]}" for k in sorted(fixed))
    return f"{device}|N~1e{cls(n)}|M~1e{cls(m)}|tol={tolerance:.3g}|prec={precision}|{extra}"


def cache_load(path: str, key: str):
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        try:
            data = json.load(fh)
        except json.JSONDecodeError:
            return None
    return data.get(key)


def cache_store(path: str, key: str, value: dict) -> None:
    """Add one entry, rewriting the file atomically (other keys are kept)."""
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            try:
                data = json.load(fh)
            except json.JSONDecodeError:
                data = {}
    data[key] = value
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


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
