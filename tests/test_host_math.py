"""The library's device math compiled for the host (tests/host_math.cpp, the
same headers as the HIP kernels): double-double sin/cos, the pair loop's
log and reciprocal, and the walk's angle-free MAC filter, against
references computed here in higher precision."""
import os
import random
import shutil
import subprocess
from decimal import Decimal, getcontext

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def host_math(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("host_math") / "host_math")
    cmd = [HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
           os.path.join(HERE, "host_math.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(exe, mode, text=""):
    r = subprocess.run([exe, mode], input=text, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return r.stdout.split("\n")


def _sin_cos(h, l):
    # Taylor series at 70 digits (|x| <= 8 here); the argument h + l is
    # formed at that precision too
    getcontext().prec = 70
    x = Decimal(h) + Decimal(l)
    s = c = Decimal(0)
    term, k = Decimal(1), 0
    while k < 120:
        if k % 4 == 0:
            c += term
        elif k % 4 == 1:
            s += term
        elif k % 4 == 2:
            c -= term
        else:
            s -= term
        k += 1
        term = term * x / k
    return s, c


def test_dd_sincos_is_double_double_accurate(host_math):
    rng = random.Random(7)
    xs = [(h, rng.uniform(-1, 1) * abs(h) * 1e-17) for h in
          [rng.uniform(-7, 7) for _ in range(400)] + [rng.uniform(-1e-3, 1e-3) for _ in range(100)]]
    xs += [(1.5707963267948966, 6.123233995736766e-17), (3.141592653589793, 1.2246467991473532e-16), (0.0, 0.0)]
    out = _run(host_math, "sincos", "".join(f"{h.hex()} {l.hex()}\n" for h, l in xs))
    worst = 0.0
    for (h, l), line in zip(xs, out):
        v = [Decimal(float.fromhex(t)) for t in line.split()]
        s, c = _sin_cos(h, l)
        worst = max(worst, float(abs(v[0] + v[1] - s)), float(abs(v[2] + v[3] - c)))
    assert worst < 1e-31, worst


def _atan2(y, x):
    # 70 digits: atan of the smaller ratio by its Taylor series after halving
    # the argument (atan z = 2 atan(z / (1 + sqrt(1 + z^2)))) until it is small
    getcontext().prec = 70
    pi = Decimal("3.141592653589793238462643383279502884197169399375105820974944592307816")
    def atan(z):
        k = 0
        while abs(z) > Decimal("0.01"):
            z = z / (1 + (1 + z * z).sqrt())
            k += 1
        s, t, n = Decimal(0), z, 1
        while abs(t) > Decimal(10) ** -75:
            s += t / n
            t = -t * z * z
            n += 2
        return s * (2 ** k)
    if x > 0:
        return atan(y / x)
    if x < 0:
        return atan(y / x) + (pi if y >= 0 else -pi)
    return pi / 2 if y > 0 else -pi / 2


def test_dd_atan2_is_double_double_accurate(host_math):
    rng = random.Random(13)
    cases = []
    for _ in range(300):
        y, x = rng.uniform(-1, 1), rng.uniform(-1, 1)
        cases.append((y, rng.uniform(-1, 1) * abs(y) * 1e-17, x, rng.uniform(-1, 1) * abs(x) * 1e-17))
    cases += [(1e-9, 0.0, 1.0, 0.0), (1.0, 0.0, -1e-12, 0.0), (-0.5, 1e-18, -0.5, -1e-18), (0.7, 0.0, 0.7, 0.0)]
    out = _run(host_math, "atan2", "".join(f"{a.hex()} {b.hex()} {c.hex()} {d.hex()}\n" for a, b, c, d in cases))
    worst = 0.0
    for (a, b, c, d), line in zip(cases, out):
        v = [Decimal(float.fromhex(t)) for t in line.split()]
        getcontext().prec = 70
        ref = _atan2(Decimal(a) + Decimal(b), Decimal(c) + Decimal(d))
        worst = max(worst, float(abs(v[0] + v[1] - ref)))
    assert worst < 1e-30, worst


def test_pair_log_and_reciprocal_within_a_few_ulp(host_math):
    """The pair loop's table log: its error is absolute (the sums it feeds
    need no relative bound near x = 1), so it is measured in ulps of
    max(1, |log x|); the reciprocal in ulps of 1/x."""
    import math
    getcontext().prec = 40
    rng = random.Random(11)
    xs = [rng.uniform(0, 4) for _ in range(3000)] + [10 ** rng.uniform(-33, 0.6) for _ in range(3000)]
    xs += [rng.uniform(0.99, 1.01) for _ in range(300)]
    # both ends of every table bucket
    xs += [0.5 + j / 256 for j in range(128)] + [0.5 + (j + 1) / 256 - 2 ** -53 for j in range(128)]
    xs += [1.0, 2.0, 4.0, 0.5, 1e-32, 0.7071067811865476, 1.4142135623730951]
    out = _run(host_math, "log", "".join(x.hex() + "\n" for x in xs))
    wl = wi = 0.0
    for x, line in zip(xs, out):
        lg, inv = (float.fromhex(t) for t in line.split())
        el, ei = Decimal(x).ln(), 1 / Decimal(x)
        wl = max(wl, float(abs(Decimal(lg) - el)) / math.ulp(max(1.0, abs(float(el)))))
        wi = max(wi, float(abs(Decimal(inv) - ei)) / math.ulp(abs(float(ei))))
    assert wl < 4 and wi < 3, (wl, wi)


def test_angle_free_mac_filter_never_contradicts_the_angle(host_math):
    fields = _run(host_math, "mac")[0].split()
    n, decided, undecided, wrong, tie_checked, tie_wrong, tie_disagree = (int(t) for t in fields)
    assert wrong == 0 and tie_wrong == 0 and tie_disagree == 0
    # the samples reach both regimes, and many near-ties are settled by long double
    assert decided > n // 2 and undecided > n // 10 and tie_checked > n // 20


def test_pool_reuse_rule(host_math):
    """The device pool hands a cached block out again only when that cannot
    race with work still queued on it: same device, and either the block was
    released after its users were waited for (no event), or the allocation is
    on the stream that released it (stream order), or the event recorded at
    the release has completed."""
    cases = [
        # dev, free stream, has event, event done, alloc stream, alloc dev -> reuse
        ((0, 1, 1, 0, 1, 0), 1),   # same stream, work pending: stream order covers it
        ((0, 1, 1, 0, 2, 0), 0),   # other stream, work pending: not yet
        ((0, 1, 1, 1, 2, 0), 1),   # other stream, event completed
        ((0, 0, 1, 0, 0, 0), 1),   # null stream on both sides
        ((0, 0, 1, 0, 3, 0), 0),   # freed on the null stream, pending, other stream
        ((0, 5, 0, 0, 7, 0), 1),   # released after a wait (sfmm_destroy): any stream
        ((1, 1, 0, 0, 1, 0), 0),   # another device's block is never handed out
        ((1, 1, 1, 1, 1, 1), 1),
    ]
    out = _run(host_math, "pool", "\n".join(" ".join(map(str, c)) for c, _ in cases) + "\n")
    got = [int(x) for x in out if x.strip()]
    assert got == [w for _, w in cases]


def test_expansion_hessians_are_derivatives_of_the_deflection(host_math):
    """The Hessian of the local (L2P) and multipole (M2P) expansions at a
    point, from the conformal-metric formulas, equals the covariant
    derivative of the same expansion's deflection (central differences
    along great circles), for random coefficients and frames."""
    out = _run(host_math, "hess")
    loc, mul = (float(x) for x in out[0].split())
    assert loc < 1e-6 and mul < 1e-6, (loc, mul)
