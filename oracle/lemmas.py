"""Lemmas 1-4 of the sFMM paper as printed, in plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Every routine follows the paper's own notation: a box centre P carries the
local spherical system K_P whose zenith is e_r(P) and whose azimuth reference
is e_theta(P) (Sec. 3.1); a point there has coordinates (theta^(P), phi^(P))
and the base function is z^l = tan^l(theta/2) e^{i l phi}.

* ``p2m``  Lemma 1 (Sec. 3.1): multipole expansion of point masses.
* ``m2m``  Lemma 2 (Sec. 3.2): translation of a multipole expansion.
* ``m2l``  Lemma 3 (Sec. 3.3): multipole -> local expansion.
* ``l2l``  Lemma 4 (Sec. 3.3): translation of a local expansion.
* ``eval_multipole`` / ``eval_local``  the expansions themselves; the local
  one also returns alpha from the e_theta formula of Sec. 3.6 together with
  the e_phi component (1/sin theta) d/dphi of the same series.
* ``tmat``  T_{ll'} of Lemma 2 / Lemma 3, summed term by term as printed.
* ``sfmm``  the five stages of Sec. 3.7 assembled over the oracle tree and the
  Algorithm 1 lists, with these lemmas and a direct near-field sum.

Expansions are (C, Q, A) with A[l-1] = A_l, l = 1..p (complex).
"""
from __future__ import annotations

from math import comb

import numpy as np

FOUR_PI = 4.0 * np.pi


def frame(c):
    """(e_theta, e_phi, e_r) at the point c: the axes of K_P, Sec. 3.1."""
    c = np.asarray(c, dtype=np.float64)
    theta = np.arccos(np.clip(c[2], -1.0, 1.0))
    phi = np.arctan2(c[1], c[0])
    e_r = np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
    e_t = np.array([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), -np.sin(theta)])
    e_p = np.array([-np.sin(phi), np.cos(phi), 0.0])
    return e_t, e_p, e_r


def local_coords(c, pts):
    """(theta^(P), phi^(P)) of points pts (3, k) in the system K_P of centre c."""
    e_t, e_p, e_r = frame(c)
    pts = np.asarray(pts, dtype=np.float64).reshape(3, -1)
    x = e_t @ pts
    y = e_p @ pts
    z = e_r @ pts
    theta = np.arctan2(np.hypot(x, y), z)
    phi = np.arctan2(y, x)
    return theta, phi


def zpow(theta, phi, l):
    """z^l(theta, phi) = tan^l(theta/2) e^{i l phi}."""
    return np.tan(theta / 2.0) ** l * np.exp(1j * l * phi)


def tmat(x: float, p: int) -> np.ndarray:
    """T_{ll'}(x) = sum_{n=1}^{min(l,l')} C(l-1,n-1) C(l',n) x^{l+l'-2n} (1+x^2)^n,
    l, l' = 1..p (Lemma 2; Lemma 3 uses it with x = cot(theta/2))."""
    T = np.zeros((p, p))
    for l in range(1, p + 1):
        for lp in range(1, p + 1):
            s = 0.0
            for n in range(1, min(l, lp) + 1):
                s += comb(l - 1, n - 1) * comb(lp, n) * x ** (l + lp - 2 * n) * (1.0 + x * x) ** n
            T[l - 1, lp - 1] = s
    return T


def p2m(c, pts, q, p: int):
    """Lemma 1: C = (1/4pi) sum 2 q_i log cos(theta_i/2) - Q log 2,
    Q = (1/4pi) sum q_i, A_l = -(1/4pi)(1/l) sum q_i z^l(theta_i, phi_i)."""
    q = np.asarray(q, dtype=np.float64)
    theta, phi = local_coords(c, pts)
    Q = q.sum() / FOUR_PI
    C = (2.0 * q * np.log(np.cos(theta / 2.0))).sum() / FOUR_PI - Q * np.log(2.0)
    A = np.array([-(q * zpow(theta, phi, l)).sum() / (FOUR_PI * l) for l in range(1, p + 1)])
    return C, Q, A


def _pair_geometry(cS, cT):
    """theta^(S)_T, phi^(S)_T (T's centre seen from K_S) and phi^(T)_S.

    HEALPix is symmetric under n -> -n, so exactly antipodal box centres occur
    (base faces 0 and 10, 4 and 6, ...).  There the two azimuths are each
    undefined but the lemmas have a limit: take the geodesic that leaves S
    along e_theta(S) (phi^(S)_T = 0); it arrives at T heading away from S, so
    S lies along e_theta(S) seen from T."""
    th, ph_TS = local_coords(cS, np.asarray(cT).reshape(3, 1))
    if np.pi - th[0] < 1e-9:
        e_t, _, _ = frame(cS)
        f_t, f_p, _ = frame(cT)
        return float(th[0]), 0.0, float(np.arctan2(e_t @ f_p, e_t @ f_t))
    _, ph_ST = local_coords(cT, np.asarray(cS).reshape(3, 1))
    return float(th[0]), float(ph_TS[0]), float(ph_ST[0])


def m2m(expn, cS, cT):
    """Lemma 2: the multipole expansion about S re-expanded about T."""
    C, Q, A = expn
    p = len(A)
    th, ph_TS, ph_ST = _pair_geometry(cS, cT)
    t = np.tan(th / 2.0)
    ls = np.arange(1, p + 1)
    src = (-1.0) ** ls * np.exp(-1j * ls * ph_TS) * A
    C2 = C + 2.0 * Q * np.log(np.cos(th / 2.0)) + 2.0 * np.real((src * t ** ls).sum())
    T = tmat(t, p)
    A2 = (-(Q / ls) * t ** ls + T @ src) * np.exp(1j * ls * ph_ST)
    return C2, Q, A2


def m2l(expn, cS, cT):
    """Lemma 3: the multipole expansion about S converted to a local
    expansion about T."""
    C, Q, A = expn
    p = len(A)
    th, ph_TS, ph_ST = _pair_geometry(cS, cT)
    c = 1.0 / np.tan(th / 2.0)
    ls = np.arange(1, p + 1)
    src = np.exp(-1j * ls * ph_TS) * A
    C2 = C + 2.0 * Q * np.log(np.sin(th / 2.0)) + 2.0 * np.real((src * c ** ls).sum())
    T = tmat(c, p)
    A2 = (-(Q / ls) * c ** ls + T @ src) * np.exp(-1j * ls * ph_ST)
    return C2, Q, A2


def l2l(expn, cS, cT):
    """Lemma 4: the local expansion about S re-expanded about T."""
    C, Q, A = expn
    p = len(A)
    th, ph_TS, ph_ST = _pair_geometry(cS, cT)
    t = np.tan(th / 2.0)
    ls = np.arange(1, p + 1)
    src = np.exp(1j * ls * ph_TS) * A
    C2 = C + 2.0 * Q * np.log(np.cos(th / 2.0)) + 2.0 * np.real((src * t ** ls).sum())
    T = tmat(t, p)
    A2 = (-1.0) ** ls * (-(Q / ls) * t ** ls + T @ src) * np.exp(-1j * ls * ph_ST)
    return C2, Q, A2


def eval_multipole(expn, c, pts):
    """psi = C + Q log(1 - cos theta) + 2 Re sum A_l / z^l (Lemma 1)."""
    C, Q, A = expn
    theta, phi = local_coords(c, pts)
    s = np.zeros(theta.shape, dtype=complex)
    for l in range(1, len(A) + 1):
        s += A[l - 1] / zpow(theta, phi, l)
    return C + Q * np.log(1.0 - np.cos(theta)) + 2.0 * np.real(s)


def eval_local(expn, c, pts):
    """Local expansion at points pts (3, k) about centre c (Sec. 3.6):
    psi = C + Q log(1 + cos theta) + 2 Re sum A_l z^l,
    alpha_theta = -Q tan(theta/2) + 2 Re sum (l / sin theta) A_l z^l,
    alpha_phi   = (1/sin theta) d psi/d phi = 2 Re sum (i l / sin theta) A_l z^l.
    Returns (psi (k,), alpha (3, k)) with alpha in global Cartesian axes."""
    C, Q, A = expn
    theta, phi = local_coords(c, pts)
    s = np.zeros(theta.shape, dtype=complex)
    da = np.zeros(theta.shape, dtype=complex)
    for l in range(1, len(A) + 1):
        zl = zpow(theta, phi, l)
        s += A[l - 1] * zl
        da += l * A[l - 1] * zl
    psi = C + Q * np.log(1.0 + np.cos(theta)) + 2.0 * np.real(s)
    a_th = -Q * np.tan(theta / 2.0) + 2.0 * np.real(da) / np.sin(theta)
    a_ph = 2.0 * np.real(1j * da) / np.sin(theta)
    e_t, e_p, e_r = frame(c)
    # unit vectors e_theta, e_phi of K_P at each point, in global axes
    ut = (np.outer(e_t, np.cos(theta) * np.cos(phi)) + np.outer(e_p, np.cos(theta) * np.sin(phi))
          - np.outer(e_r, np.sin(theta)))
    up = -np.outer(e_t, np.sin(phi)) + np.outer(e_p, np.cos(phi))
    return psi, ut * a_th + up * a_ph


def sfmm(src, q, tgt, p: int, m: int, c_s: float = 2.0, c_t: float = 0.5,
         max_level: int = 29):
    """The sFMM of Sec. 3.7 on the CPU: division (Sec. 3.1), Lemma 1 on the
    leaves and Lemma 2 up the tree (Sec. 3.2), Algorithm 1 with Lemma 3 for
    every FMM-act pair (Sec. 3.3-3.5), Lemma 4 down the tree, and at each
    target its leaf's local expansion plus the direct sum over the leaf's
    close boxes (Sec. 3.6).  psi is in the zero-mean gauge (Eq.
    STAND_CONDITION: Q_tot/(4pi) added).  Slow; for small inputs only.

    Returns dict(psi, defl, tree, m2l, p2p, multipole, local, leaf)."""
    from . import direct, locate, tree as build_tree, walk, GAUGE_RAW

    src = np.ascontiguousarray(src, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    tgt = np.ascontiguousarray(tgt, dtype=np.float64)
    t = build_tree(src, m, max_level)
    m2l_pairs, p2p_pairs, _ = walk(t, c_s, c_t)
    nb = t.nbox
    centres = t.centre
    zero = (0.0, 0.0, np.zeros(p, dtype=complex))
    mult = [zero] * nb
    # up-pass: Lemma 1 on leaves, Lemma 2 from the deepest level up
    for b in np.argsort(-t.level, kind="stable"):
        if t.child0[b] < 0:
            idx = t.perm[t.first[b]:t.first[b] + t.count[b]]
            if len(idx):
                mult[b] = p2m(centres[:, b], src[:, idx], q[idx], p)
        else:
            C, Q, A = 0.0, 0.0, np.zeros(p, dtype=complex)
            for k in range(4):
                ch = t.child0[b] + k
                if t.count[ch] == 0:
                    continue
                c2, q2, a2 = m2m(mult[ch], centres[:, ch], centres[:, b])
                C, Q, A = C + c2, Q + q2, A + a2
            mult[b] = (C, Q, A)
    # FMM-act (Lemma 3) into each target box's local expansion
    loc = [zero] * nb
    for s, tb in m2l_pairs:
        if t.count[s] == 0:
            continue
        c2, q2, a2 = m2l(mult[s], centres[:, s], centres[:, tb])
        C, Q, A = loc[tb]
        loc[tb] = (C + c2, Q + q2, A + a2)
    # down-pass: Lemma 4 from level 0 down
    for b in np.argsort(t.level, kind="stable"):
        if t.child0[b] >= 0:
            for k in range(4):
                ch = t.child0[b] + k
                c2, q2, a2 = l2l(loc[b], centres[:, b], centres[:, ch])
                C, Q, A = loc[ch]
                loc[ch] = (C + c2, Q + q2, A + a2)
    leaf, _ = locate(t, tgt)
    M = tgt.shape[1]
    psi = np.zeros(M)
    defl = np.zeros((3, M))
    near = {}
    for s, tb in p2p_pairs:
        near.setdefault(int(tb), []).append(int(s))
    for i in range(M):
        L = int(leaf[i])
        pt = tgt[:, i:i + 1]
        ps, al = eval_local(loc[L], centres[:, L], pt)
        idx = np.concatenate([t.perm[t.first[s]:t.first[s] + t.count[s]] for s in near.get(L, [])]
                             + [np.zeros(0, dtype=np.int64)])
        pn, an = direct(src[:, idx], q[idx], pt, gauge=GAUGE_RAW, nthreads=1)
        psi[i] = ps[0] + pn[0]
        defl[:, i] = al[:, 0] + an[:, 0]
    psi += q.sum() / FOUR_PI
    return dict(psi=psi, defl=defl, tree=t, m2l=m2l_pairs, p2p=p2p_pairs,
                multipole=mult, local=loc, leaf=leaf)
