"""Pins the oracle to facts that do not come from the oracle itself: values
derived by hand, closed forms, exact arithmetic, invariants and library
routines. CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")

X0, Y0, D = -2.0, -1.5, 3.0 / 1024.0


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- escape-time
def test_escape_hand_derived_points():
    g = _gold("escape_points.json")
    gr = g["grid"]
    for mi in (16, 256, 1000):
        for p in g["points"]:
            want = mi if p["count"] == "max_iter" else p["count"]
            got = O.escape_pixel(p["r"], p["c"], gr["x0"], gr["y0"], gr["dx"], gr["dy"], mi)
            assert got == want, (p, mi)


def _exact_count(cr: Fraction, ci: Fraction, max_iter: int):
    """Escape count in exact rational arithmetic; also the smallest distance
    of |z_n|^2 to 4 seen, so near-ties can be skipped."""
    zr = zi = Fraction(0)
    closest = None
    n = 0
    while n < max_iter:
        m = zr * zr + zi * zi
        dist = abs(m - 4)
        closest = dist if closest is None else min(closest, dist)
        if m > 4:
            break
        zr, zi = zr * zr - zi * zi + cr, 2 * zr * zi + ci
        n += 1
    return n, closest


def test_escape_matches_exact_rational_arithmetic():
    rng = np.random.default_rng(7)
    mi = 9
    checked = 0
    for _ in range(400):
        r, c = int(rng.integers(0, 1024)), int(rng.integers(0, 1024))
        cr = Fraction(-2) + Fraction(c * 3, 1024)
        ci = Fraction(-3, 2) + Fraction(r * 3, 1024)
        want, closest = _exact_count(cr, ci, mi)
        if closest is not None and closest < Fraction(1, 10**3):
            continue
        assert O.escape_pixel(r, c, X0, Y0, D, D, mi) == want, (r, c)
        checked += 1
    assert checked > 300


def test_escape_conjugate_symmetry_bitwise():
    img = O.escape(1024, 1024, X0, Y0, D, D, 256)
    # row r has ci = -1.5 + r*3/1024, row 1024 - r has -ci exactly
    assert np.array_equal(img[1:], img[1:][::-1])


def test_escape_max_iter_monotone():
    a = O.escape(256, 256, X0, Y0, 4 * D, 4 * D, 40)
    b = O.escape(256, 256, X0, Y0, 4 * D, 4 * D, 300)
    assert np.array_equal(a, np.minimum(b, 40))
    assert a.min() >= 1


def test_escape_area_estimate():
    # The Mandelbrot set has area about 1.5066; pixels still bounded after
    # 256 steps over-cover it slightly.
    img = O.escape(1024, 1024, X0, Y0, D, D, 256)
    area = float((img == 256).mean()) * 9.0
    assert 1.50 < area < 1.58


# ------------------------------------------------------------------- blur
def test_gauss_weights_closed_form():
    w = O.gauss5_weights(1.0).reshape(5, 5).astype(np.float64)
    s1 = 1 + 2 * math.exp(-0.5) + 2 * math.exp(-2.0)
    assert abs(w[2, 2] - 1.0 / (s1 * s1)) <= 2 ** -24 * w[2, 2]
    assert np.array_equal(w, w.T) and np.array_equal(w, w[::-1]) and np.array_equal(w, w[:, ::-1])
    assert abs(w[2, 3] / w[2, 2] - math.exp(-0.5)) < 1e-6
    assert abs(w[0, 0] / w[2, 2] - math.exp(-4.0)) < 1e-6
    assert abs(w.sum() - 1.0) < 1e-6


def test_blur_impulse_gives_mirrored_weights():
    rng = np.random.default_rng(3)
    wt = rng.random(25).astype(np.float32)  # asymmetric on purpose
    img = np.zeros((11, 13), np.float32)
    img[5, 6] = 1.0
    out = O.blur5(img, wt)
    W = wt.reshape(5, 5)
    for a in range(-2, 3):
        for b in range(-2, 3):
            assert out[5 + a, 6 + b] == W[2 - a, 2 - b]
    mask = np.ones_like(out, bool)
    mask[3:8, 4:9] = False
    assert np.all(out[mask] == 0)


def test_blur_clamp_corner():
    wt = O.gauss5_weights(1.0)
    W = wt.reshape(5, 5)
    img = np.zeros((7, 9), np.float32)
    img[0, 0] = 1.0
    out = O.blur5(img, wt)
    # fma(w, 1, acc) is a plain FP32 addition; taps with dy, dx in {-2,-1,0}
    # all clamp onto (0, 0); the others add exact zeros.
    acc = np.float32(0)
    for dy in (-2, -1, 0):
        for dx in (-2, -1, 0):
            acc = np.float32(acc + W[dy + 2, dx + 2])
    assert out[0, 0] == acc


def test_blur_constant_image():
    wt = O.gauss5_weights(1.0)
    img = np.full((9, 10), 0.37, np.float32)
    out = O.blur5(img, wt)
    assert np.all(out == out[4, 4])
    assert abs(float(out[0, 0]) - 0.37) < 1e-6


def test_blur_matches_library_correlation():
    from scipy import ndimage
    rng = np.random.default_rng(11)
    img = rng.random((37, 53)).astype(np.float32)
    wt = O.gauss5_weights(1.0)
    out = O.blur5(img, wt).astype(np.float64)
    ref = ndimage.correlate(img.astype(np.float64), wt.reshape(5, 5).astype(np.float64), mode="nearest")
    bound = 25 * 2 ** -24 * ndimage.correlate(np.abs(img).astype(np.float64),
                                                np.abs(wt.reshape(5, 5)).astype(np.float64), mode="nearest")
    assert np.all(np.abs(out - ref) <= bound)


def test_blur_power_of_two_scaling_bitwise():
    rng = np.random.default_rng(5)
    img = rng.random((20, 21)).astype(np.float32)
    wt = O.gauss5_weights(1.0)
    assert np.array_equal(O.blur5(img * np.float32(4), wt), O.blur5(img, wt) * np.float32(4))


# ----------------------------------------------------------------- n-body
def test_rsqrt_lomont_accuracy():
    xs = np.logspace(-7, 4, 4001)
    worst = max(abs(float(O.rsqrt_lomont(float(np.float32(x)))) * math.sqrt(float(np.float32(x))) - 1.0)
                for x in xs)
    # three Newton steps from Lomont's estimate leave only FP32 rounding
    assert worst < 4 * 2 ** -24


def _bits(v) -> int:
    return int(np.float32(v).view(np.uint32))


def test_rsqrt_lomont_integer_estimate_bits():
    """Lomont (2003), first estimate: the float whose bits are 0x5f375a86
    minus the input's bits shifted right by one. Worked by hand:
    1.0 = 0x3f800000 -> 0x5f375a86 - 0x1fc00000 = 0x3f775a86;
    2.0 = 0x40000000 -> - 0x20000000 = 0x3f375a86;
    0.5 = 0x3f000000 -> - 0x1f800000 = 0x3fb75a86;
    4.0 = 0x40800000 -> - 0x20400000 = 0x3ef75a86;
    1.5 = 0x3fc00000 -> - 0x1fe00000 = 0x3f575a86;
    the bit shifted out is dropped: 0x3f800001 gives the estimate of 1.0.
    Another constant (0x5f3759df, say) fails every line."""
    want = {1.0: 0x3F775A86, 2.0: 0x3F375A86, 0.5: 0x3FB75A86, 4.0: 0x3EF75A86, 1.5: 0x3F575A86}
    for x, b in want.items():
        assert _bits(O.rsqrt_lomont_estimate(x)) == b, (x, hex(_bits(O.rsqrt_lomont_estimate(x))))
    x1 = float(np.uint32(0x3F800001).view(np.float32))
    assert _bits(O.rsqrt_lomont_estimate(x1)) == 0x3F775A86


def test_rsqrt_newton_step_by_hand():
    """One step y <- y (1.5 - (x/2) y^2) on exactly representable values:
    x = 1, y = 0.5: t = 0.25, u = 1.5 - 0.125 = 1.375, y' = 0.6875;
    x = 1, y = 0.75: t = 0.5625, u = 1.5 - 0.28125 = 1.21875, y' = 0.9140625;
    the exact roots are fixed points: x = 4, y = 0.5 and x = 1, y = 1."""
    assert O.rsqrt_newton(0.5, 0.5) == np.float32(0.6875)
    assert O.rsqrt_newton(0.5, 0.75) == np.float32(0.9140625)
    assert O.rsqrt_newton(2.0, 0.5) == np.float32(0.5)
    assert O.rsqrt_newton(0.5, 1.0) == np.float32(1.0)


def test_rsqrt_lomont_is_estimate_then_three_steps():
    for x in (1e-6, 0.37, 1.0, 2.0, 3.3, 1234.5):
        xf = np.float32(x)
        hx = float(np.float32(0.5) * xf)
        y = O.rsqrt_lomont_estimate(float(xf))
        for _ in range(3):
            y = O.rsqrt_newton(hx, float(y))
        assert _bits(O.rsqrt_lomont(float(xf))) == _bits(y), x


def test_rsqrt_lomont_first_estimate_and_scaling():
    # 1/sqrt(4x) is exactly half of 1/sqrt(x) through the bit estimate and Newton steps
    for x in (0.3, 1.7, 123.0, 1e-5):
        assert O.rsqrt_lomont(4 * x) == np.float32(O.rsqrt_lomont(x) / 2)
    assert abs(float(O.rsqrt_lomont(1.0)) - 1.0) < 2 ** -23


def test_nbody_two_body_closed_form():
    pos = np.array([[0.1, 0.2, 0.3, 1.25], [0.7, -0.1, 0.5, 0.75]], np.float32)
    eps2 = 1e-6
    for strict in (True, False):
        a = O.nbody_acc(pos, eps2, strict)
        for i, j in ((0, 1), (1, 0)):
            d = pos[j, :3].astype(np.float64) - pos[i, :3].astype(np.float64)
            want = float(pos[j, 3]) * d / (d @ d + eps2) ** 1.5
            assert np.allclose(a[i, :3], want, rtol=2e-6, atol=0)
            assert a[i, 3] == 0


def test_nbody_scaling_bitwise():
    from paper_1805_02755_amd.synth import nbody_bodies
    pos = nbody_bodies(96, seed=9)
    eps2 = np.float32(1e-6)
    for strict in (True, False):
        base = O.nbody_acc(pos, float(eps2), strict)
        p2 = pos.copy()
        p2[:, 3] *= 2
        assert np.array_equal(O.nbody_acc(p2, float(eps2), strict), base * 2)
        p3 = pos.copy()
        p3[:, :3] *= 2
        assert np.array_equal(O.nbody_acc(p3, float(eps2 * 4), strict), base / 4)


def test_nbody_tiny_vs_fp64_brute_force():
    from paper_1805_02755_amd.synth import nbody_bodies
    pos = nbody_bodies(64, seed=21)
    eps2 = 1e-3
    ref = O.nbody_acc_f64(pos, eps2)
    # independent brute force in the test, FP64
    p = pos.astype(np.float64)
    d = p[None, :, :3] - p[:, None, :3]
    r2 = (d ** 2).sum(-1) + eps2
    terms = p[None, :, 3, None] * d / r2[..., None] ** 1.5
    bf = terms.sum(1)
    assert np.allclose(ref, bf, rtol=1e-12, atol=1e-12)
    scale = np.linalg.norm(terms, axis=-1).sum(1)
    for strict in (True, False):
        a = O.nbody_acc(pos, eps2, strict)[:, :3].astype(np.float64)
        err = np.linalg.norm(a - bf, axis=-1)
        assert np.all(err <= 1e-5 * scale)


def test_nbody_momentum_conservation():
    from paper_1805_02755_amd.synth import nbody_bodies
    pos = nbody_bodies(256, seed=4)
    a = O.nbody_acc(pos, 1e-6, True)[:, :3].astype(np.float64)
    m = pos[:, 3].astype(np.float64)
    tot = (m[:, None] * a).sum(0)
    mag = (m[:, None] * np.abs(a)).sum(0)
    assert np.all(np.abs(tot) <= 1e-5 * mag)


def test_nbody_self_term_is_zero():
    pos = np.array([[0.5, 0.5, 0.5, 1.0]], np.float32)
    assert np.array_equal(O.nbody_acc(pos, 1e-6, True), np.zeros((1, 4), np.float32))


# ------------------------------------------- n-body integration step
def _bodies_and_velocities(n, seed):
    from paper_1805_02755_amd.synth import nbody_bodies, nbody_velocities
    return nbody_bodies(n, seed=seed), nbody_velocities(n, seed=seed)


def test_nbody_step_zero_dt_is_identity():
    pos, vel = _bodies_and_velocities(40, 3)
    for strict in (True, False):
        po, vo = O.nbody_step(pos, vel, 1e-6, 0.0, strict)
        assert np.array_equal(po, pos) and np.array_equal(vo, vel)


def test_nbody_step_single_body_exact():
    """One body feels no force: it moves in a straight line. With values
    whose products and sums are exact in FP32 the result is exact."""
    pos = np.array([[1.0, 2.0, 3.0, 5.0]], np.float32)
    vel = np.array([[2.0, -4.0, 0.5, 7.0]], np.float32)
    po, vo = O.nbody_step(pos, vel, 1e-6, 0.25, True)
    assert np.array_equal(po, np.array([[1.5, 1.0, 3.125, 5.0]], np.float32))
    assert np.array_equal(vo, vel)


def test_nbody_step_massless_bodies_drift():
    """Massless bodies exert no force: velocities are unchanged bit for bit and
    positions advance by v dt (two roundings from the FP64 value)."""
    pos, vel = _bodies_and_velocities(64, 8)
    pos[:, 3] = 0.0
    dt = 0.01
    po, vo = O.nbody_step(pos, vel, 1e-6, dt, True)
    assert np.array_equal(vo, vel)
    exact = pos[:, :3].astype(np.float64) + vel[:, :3].astype(np.float64) * dt
    assert np.all(np.abs(po[:, :3] - exact) <= 2 * np.spacing(np.abs(exact).astype(np.float32)))


def test_nbody_step_follows_the_acceleration():
    """v' - v = a dt and x' - x = v dt + a dt^2/2 against the (separately
    pinned) acceleration, in FP64 within the few roundings of each update."""
    pos, vel = _bodies_and_velocities(128, 12)
    dt, eps2 = 0.003, 1e-6
    a = O.nbody_acc(pos, eps2, True)[:, :3].astype(np.float64)
    po, vo = O.nbody_step(pos, vel, eps2, dt, True)
    v = vel[:, :3].astype(np.float64)
    x = pos[:, :3].astype(np.float64)
    v_ref = v + a * dt
    x_ref = x + v * dt + a * (dt * dt / 2)
    tol_v = 2 * np.spacing(np.abs(v_ref).astype(np.float32)) + 1e-7 * np.abs(a * dt)
    tol_x = 3 * np.spacing(np.abs(x_ref).astype(np.float32)) + 1e-7 * np.abs(a * dt * dt)
    assert np.all(np.abs(vo[:, :3] - v_ref) <= tol_v)
    assert np.all(np.abs(po[:, :3] - x_ref) <= tol_x)
    assert np.array_equal(po[:, 3], pos[:, 3]) and np.array_equal(vo[:, 3], vel[:, 3])


def test_nbody_step_conserves_momentum():
    pos, vel = _bodies_and_velocities(200, 5)
    m = pos[:, 3].astype(np.float64)
    dt = 0.01
    po, vo = O.nbody_step(pos, vel, 1e-6, dt, True)
    before = (m[:, None] * vel[:, :3]).sum(0)
    after = (m[:, None] * vo[:, :3].astype(np.float64)).sum(0)
    a = O.nbody_acc(pos, 1e-6, True)[:, :3].astype(np.float64)
    scale = (m[:, None] * np.abs(a)).sum(0) * dt + (m[:, None] * np.abs(vel[:, :3])).sum(0) * 1e-6
    assert np.all(np.abs(after - before) <= 1e-4 * scale)


def test_nbody_step_two_body_circular_orbit():
    """Two unit masses at distance 1 on a circular orbit about their centre
    (speed sqrt(1/2) each): a quarter period of small steps keeps them at
    distance 1 and turns the line between them by 90 degrees."""
    r = 0.5
    vc = np.sqrt(1.0 / (4.0 * r))
    pos = np.array([[-r, 0, 0, 1], [r, 0, 0, 1]], np.float32)
    vel = np.array([[0, -vc, 0, 0], [0, vc, 0, 0]], np.float32)
    period = 2 * np.pi * r / vc
    steps = 1000
    dt = np.float32(period / 4 / steps)
    for _ in range(steps):
        pos, vel = O.nbody_step(pos, vel, 1e-12, float(dt), True)
    d = pos[1, :3].astype(np.float64) - pos[0, :3].astype(np.float64)
    assert abs(np.linalg.norm(d) - 1.0) < 0.01
    angle = np.degrees(np.arctan2(d[1], d[0]))
    assert abs(angle - 90.0) < 2.0


# ------------------------------------------------------ binomial options
BIN_SIGMA, BIN_RATE, BIN_T, BIN_X, BIN_N = 0.3, 0.05, 1.0, 100.0, 254


def _black_scholes_call(S, X, sigma, r, T):
    from math import erf, exp, log, sqrt
    nd = lambda x: 0.5 * (1.0 + erf(x / sqrt(2.0)))
    d1 = (log(S / X) + (r + 0.5 * sigma * sigma) * T) / (sigma * sqrt(T))
    return S * nd(d1) - X * exp(-r * T) * nd(d1 - sigma * sqrt(T))


def test_binomial_converges_to_black_scholes():
    """254 steps of the tree are within a few cents of the closed form (the
    tree's error is of order 1/N)."""
    f, pu, pd = O.binomial_table(BIN_N, BIN_SIGMA, BIN_RATE, BIN_T)
    for S in (60.0, 80.0, 100.0, 120.0, 140.0):
        c = float(O.binomial_price(S, BIN_X, BIN_N, f, pu, pd))
        assert abs(c - _black_scholes_call(S, BIN_X, BIN_SIGMA, BIN_RATE, BIN_T)) < 0.05, S


def test_binomial_one_step_closed_form():
    import math
    sigma, r, T, S, X = 0.25, 0.04, 0.5, 105.0, 100.0
    f, pu, pd = O.binomial_table(1, sigma, r, T)
    u = math.exp(sigma * math.sqrt(T))
    d = 1 / u
    p = (math.exp(r * T) - d) / (u - d)
    ref = math.exp(-r * T) * (p * max(S * u - X, 0) + (1 - p) * max(S * d - X, 0))
    assert abs(float(O.binomial_price(S, X, 1, f, pu, pd)) - ref) <= 1e-5 * ref


def test_binomial_table_symmetry():
    import math
    f, pu, pd = O.binomial_table(BIN_N, BIN_SIGMA, BIN_RATE, BIN_T)
    assert f[BIN_N // 2] == np.float32(1.0)
    prod = f.astype(np.float64) * f[::-1].astype(np.float64)
    assert np.all(np.abs(prod - 1.0) <= 4 * 2.0 ** -24)
    assert abs(float(pu) + float(pd) - math.exp(-BIN_RATE * BIN_T / BIN_N)) <= 2 * 2.0 ** -24


def test_binomial_bounds_and_monotonicity():
    import math
    f, pu, pd = O.binomial_table(BIN_N, BIN_SIGMA, BIN_RATE, BIN_T)
    spots = np.linspace(1.0, 300.0, 120).astype(np.float32)
    c = O.binomial(spots, BIN_X, BIN_N, f, pu, pd).astype(np.float64)
    lower = np.maximum(spots - BIN_X * math.exp(-BIN_RATE * BIN_T), 0.0)
    assert np.all(c >= lower - 1e-3) and np.all(c <= spots)
    assert np.all(np.diff(c) >= 0)
    # no leaf is in the money below X / f_N: the price is exactly zero
    assert O.binomial_price(0.5, BIN_X, BIN_N, f, pu, pd) == 0.0


# -------------------------------------------------------------- schedulers
def test_static_listing_example():
    g = _gold("static_listing_example.json")
    for key in ("static", "static_rev"):
        got = O.static_plan(g["G"], g["props"], g[key]["order"])
        assert got == [tuple(r) for r in g[key]["ranges"]]


def test_static_bands_equal_split():
    # 1024 rows, 8 bands of 128; device 0 takes 7/8, device 1 placed first
    got = O.static_plan(1024, [0.875], [1, 0], n_bands=8)
    assert got == [(128, 1024), (0, 128)]
    # every device gets at least one band
    got = O.static_plan(1024, [0.999], [0, 1], n_bands=8)
    assert got == [(0, 896), (896, 1024)]
    assert O.static_plan(1024, [0.5], [0, 1], n_bands=1) is None


def test_static_plan_partitions():
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = int(rng.integers(1, 5))
        G = int(rng.integers(n, 5000))
        props = list(rng.dirichlet(np.ones(n))[: n - 1])
        order = list(rng.permutation(n))
        plan = O.static_plan(G, props, order)
        cov = O.coverage(G, [(b, e - b) for b, e in plan])
        assert cov.ok
        # spatial order follows the delivery order
        starts = [plan[d][0] for d in order]
        assert starts == sorted(starts)


def test_hguided_golden_vector():
    g = _gold("hguided_vector.json")
    seq = O.hguided_sequence(g["G"], g["P"], g["k"], g["min"], [i % 2 for i in range(1000)])
    assert [[d, s] for d, _, s in seq] == g["packages"]
    assert O.coverage(g["G"], [(b, s) for _, b, s in seq]).ok


def test_hguided_sizes_shrink_and_respect_minimum():
    rng = np.random.default_rng(2)
    for _ in range(100):
        n = int(rng.integers(1, 4))
        P = [int(x) for x in rng.integers(1, 1000, n)]
        mins = [int(x) for x in rng.integers(1, 20, n)]
        G = int(rng.integers(1, 100000))
        req = [int(x) for x in rng.integers(0, n, 100000)]
        seq = O.hguided_sequence(G, P, int(rng.integers(1, 5)), mins, req)
        assert O.coverage(G, [(b, s) for _, b, s in seq]).ok
        last = {}
        for idx, (d, _, s) in enumerate(seq):
            if idx + 1 < len(seq):
                assert s >= mins[d]
            if d in last:
                assert s <= last[d]
            last[d] = s


def test_dynamic_equal_packages_with_short_tail():
    seq = O.dynamic_sequence(1000, 64, [0, 1] * 100)
    sizes = [s for _, _, s in seq]
    assert sizes[:-1] == [64] * 15 and sizes[-1] == 1000 - 15 * 64
    assert O.dynamic_package_for_count(1000, 50) == 20
    assert O.dynamic_package_for_count(1001, 50) == 21


# ------------------------------------------------------------------ metrics
def test_metrics_closed_forms():
    assert O.overhead_pct(1.028, 1.0) == pytest.approx(2.8)
    assert O.balance([2.0, 2.0, 2.0]) == 1.0
    assert O.balance([1.0, 4.0]) == 0.25
    # two devices: both readings of the S_max formula give 1 + T_fast / T_slow
    t1, t2 = 0.5, 3.0
    assert O.s_max([t1, t2]) == pytest.approx(1 + t1 / t2)
    assert O.s_max([t1, t2]) == pytest.approx((t1 + t2) / max(t1, t2))
    assert O.efficiency(1.1, O.s_max([t1, t2])) == pytest.approx(1.1 / (1 + t1 / t2))
