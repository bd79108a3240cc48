"""Error measures shared by the GPU parity tests.

Every comparison with the oracle reports two numbers per output:
* the relative L2 error ||x - x_ref|| / ||x_ref|| over the target set (the
  gate of the method's tolerance), and
* the worst single target, max_i |x_i - x_ref,i| / rms(x_ref) (for the
  deflection |.| is the 3-vector norm), so that a few bad targets cannot
  hide inside a norm over many good ones.

The worst-target gate is WORST_FACTOR times the tolerance: the error of the
truncated expansions is largest at targets on the corners of deep leaves
(HEALPix grid targets sit on the vertices of every deeper pixel) and at
targets next to dense clumps, a few dozen times the mean square error
there, and a wrong near-field term or a missed box shows up as an error of
order one at its target, far above this bound.
"""
import numpy as np

WORST_FACTOR = 100.0


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def worst(a, b):
    """max_i |a_i - b_i| / rms(b): rows of (3, M) arrays are 3-vectors."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim == 2:
        d = np.linalg.norm(a - b, axis=0)
        r = np.sqrt(np.mean(np.sum(b * b, axis=0)))
    else:
        d = np.abs(a - b)
        r = np.sqrt(np.mean(b * b))
    return float(d.max() / r)


def errors(psi, defl, ref_p, ref_a):
    """(rel-L2 psi, rel-L2 alpha, worst psi, worst alpha)."""
    return rel_l2(psi, ref_p), rel_l2(defl, ref_a), worst(psi, ref_p), worst(defl, ref_a)


def check(name, psi, defl, ref_p, ref_a, tol, worst_tol=None, say=print):
    """Gate psi and alpha at rel-L2 <= tol and worst target <= worst_tol
    (WORST_FACTOR * tol by default); returns the four numbers."""
    ep, ea, wp, wa = errors(psi, defl, ref_p, ref_a)
    wt = WORST_FACTOR * tol if worst_tol is None else worst_tol
    say(f"[{name}] rel-L2 psi {ep:.3e} alpha {ea:.3e}; worst target psi {wp:.3e} alpha {wa:.3e} "
        f"(gates {tol:.0e} / {wt:.0e})")
    assert np.isfinite(psi).all() and np.isfinite(defl).all()
    assert ep <= tol and ea <= tol, (ep, ea)
    assert wp <= wt and wa <= wt, (wp, wa)
    return ep, ea, wp, wa
