"""Pins of the oracle's cell geometry (volume, interface area, plane constant,
face-flux region) against exact rational arithmetic, closed forms and brute-force
sub-cell sampling. The geometry is the cube cut by the plane m.x = alpha of
section 3.2 (eq. plane_m) and c = f(alpha, m) of section 3.3.2."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import exact


def _rand_rational_normal(rng, zeros=0):
    comps = [Fr(int(rng.integers(1, 40)), int(rng.integers(1, 40))) * int(rng.choice([-1, 1]))
             for _ in range(3)]
    for i in rng.choice(3, size=zeros, replace=False):
        comps[i] = Fr(0)
    s = sum(abs(v) for v in comps)
    return [v / s for v in comps]


@pytest.mark.parametrize("zeros", [0, 1, 2])
def test_volume_matches_exact_rational(orc, zeros):
    rng = np.random.default_rng(11 + zeros)
    worst = 0.0
    for _ in range(400):
        m = _rand_rational_normal(rng, zeros)
        lo = sum(min(v, 0) for v in m)
        hi = sum(max(v, 0) for v in m)
        a = lo + (hi - lo) * Fr(int(rng.integers(0, 1001)), 1000)
        ref = exact.volume(m, a)
        got = orc.volume([float(v) for v in m], float(a))
        # the float inputs differ from the rationals by rounding; bound that effect
        # by |dV/dalpha| * (|alpha| + 1) * 2^-52
        slope = float(exact.dvolume(m, a))
        tol = 2e-16 + 4 * slope * 2.3e-16
        worst = max(worst, abs(got - float(ref)) - tol)
        assert abs(got - float(ref)) <= tol, (m, a, got, float(ref))


def test_volume_special_cases(orc):
    # a plane normal to x: the liquid is the slab x <= alpha
    for a in np.linspace(-0.2, 1.2, 57):
        assert orc.volume([1, 0, 0], a) == pytest.approx(min(max(a, 0.0), 1.0), abs=2e-16)
        assert orc.volume([-1, 0, 0], a) == pytest.approx(min(max(a + 1.0, 0.0), 1.0), abs=2e-16)
    # body diagonal: a corner tetrahedron of volume alpha^3 / (6 m1 m2 m3) = 4.5 alpha^3
    t = 1.0 / 3.0
    for a in np.linspace(0.0, t, 23):
        assert orc.volume([t, t, t], a) == pytest.approx(4.5 * a ** 3, rel=1e-14, abs=1e-17)
    # 2D: a corner triangle alpha^2 / (2 m1 m2)
    for a in np.linspace(0.0, 0.3, 13):
        assert orc.volume([0.3, 0.7, 0.0], a) == pytest.approx(a * a / (2 * 0.3 * 0.7),
                                                               rel=1e-14, abs=1e-17)


def test_volume_complement_and_bounds(orc):
    rng = np.random.default_rng(5)
    for _ in range(500):
        m = rng.normal(size=3)
        m /= np.abs(m).sum()
        a = rng.uniform(-1.1, 1.1)
        v = orc.volume(m, a)
        assert 0.0 <= v <= 1.0
        # {m.x <= a} and {(-m).x <= -a} split the cube
        assert v + orc.volume(-m, -a) == pytest.approx(1.0, abs=1e-15)


def test_volume_brute_force_bracket(orc):
    """Sub-cell counting with a rigorous bracket: sub-cells entirely inside give a
    lower bound, those not entirely outside an upper bound."""
    rng = np.random.default_rng(7)
    n = 48
    ax = (np.arange(n) + 0.0) / n
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    for _ in range(12):
        m = rng.normal(size=3)
        m /= np.abs(m).sum()
        lo = np.minimum(m, 0).sum()
        a = lo + rng.uniform(0.05, 0.95) * (np.abs(m).sum())
        # min and max of m.x over each sub-cube
        base = m[0] * X + m[1] * Y + m[2] * Z
        mn = base + np.minimum(m, 0).sum() / n
        mx = base + np.maximum(m, 0).sum() / n
        inside = np.count_nonzero(mx <= a) / n ** 3
        touched = np.count_nonzero(mn < a) / n ** 3
        v = orc.volume(m, a)
        assert inside - 1e-15 <= v <= touched + 1e-15


def test_area_matches_exact_derivative(orc):
    rng = np.random.default_rng(3)
    for zeros in (0, 1, 2):
        for _ in range(150):
            m = _rand_rational_normal(rng, zeros)
            lo = sum(min(v, 0) for v in m)
            hi = sum(max(v, 0) for v in m)
            a = lo + (hi - lo) * Fr(int(rng.integers(1, 1000)), 1000)
            mf = [float(v) for v in m]
            ref = float(exact.dvolume(m, a)) * math.sqrt(sum(v * v for v in mf))
            assert orc.area(mf, float(a)) == pytest.approx(ref, rel=1e-12, abs=1e-13)
    # closed forms: a face-parallel cut has unit area, the 2D diagonal cut through the
    # centre has length sqrt(2), the body-diagonal cut through the centre is a regular
    # hexagon of side sqrt(2)/2 (area 3*sqrt(3)/4)
    assert orc.area([1, 0, 0], 0.4) == pytest.approx(1.0, abs=1e-15)
    assert orc.area([0.5, 0.5, 0], 0.5) == pytest.approx(math.sqrt(2.0), abs=1e-15)
    t = 1.0 / 3.0
    assert orc.area([t, t, t], 0.5) == pytest.approx(3 * math.sqrt(3) / 4, abs=1e-14)


def test_alpha_round_trip(orc):
    rng = np.random.default_rng(9)
    m = rng.normal(size=(3000, 3))
    m[:1000, 2] = 0.0           # 2D normals
    m[1000:1200, 1:] = 0.0      # axis-aligned
    m /= np.abs(m).sum(axis=1, keepdims=True)
    c = np.concatenate([rng.uniform(1e-12, 1 - 1e-12, 2000),
                        10.0 ** rng.uniform(-12, -1, 500),
                        1 - 10.0 ** rng.uniform(-12, -1, 500)])
    a = orc.alpha_n(m, c)
    v = orc.volume_n(m, a)
    assert np.max(np.abs(v - c)) <= 4.5e-16
    lo = np.minimum(m, 0).sum(axis=1)
    hi = np.maximum(m, 0).sum(axis=1)
    assert np.all(a >= lo) and np.all(a <= hi)
    # alpha(V(alpha)) recovers alpha to within the volume's rounding / slope
    a0 = lo + rng.uniform(0.02, 0.98, len(lo)) * (hi - lo)
    v0 = orc.volume_n(m, a0)
    a1 = orc.alpha_n(m, v0)
    slope = orc.area_n(m, a0) / np.linalg.norm(m, axis=1)
    assert np.all(np.abs(a1 - a0) <= 1e-15 / np.maximum(slope, 1e-3) + 1e-15)


def _corner_alpha_exact(m, v):
    """Plane constant of an interface cutting off the corner of volume v (tetrahedral
    regime of the reflected frame), to 50 digits: a^3 / (6 m1 m2 m3) = v."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    mr = [abs(Decimal(float(x))) for x in m]
    a = (Decimal(6) * mr[0] * mr[1] * mr[2] * Decimal(float(v))) ** (Decimal(1) / Decimal(3))
    return a, sum(mr), sum(-Decimal(float(x)) for x in m if x < 0)


def _check_alpha_near_empty_and_full(alpha_n):
    """alpha to rounding of alpha itself (not of the volume) when the interface cuts off
    a small corner: c = v (liquid corner) and c = 1 - v (gas corner), v in [1e-14, 1e-6]."""
    rng = np.random.default_rng(31)
    m = rng.uniform(0.15, 1.0, size=(300, 3)) * rng.choice([-1.0, 1.0], size=(300, 3))
    m /= np.abs(m).sum(axis=1, keepdims=True)
    v = 10.0 ** rng.uniform(-14, -6, 300)
    for full in (False, True):
        c = 1.0 - v if full else v
        got = alpha_n(m, c)
        for i in range(len(v)):
            # 1 - c is exact for c in [1/2, 1]: the gas corner has exactly the volume 1 - c
            vv = (1.0 - c[i]) if full else c[i]
            a, S, shift = _corner_alpha_exact(m[i], vv)
            want = (S - a if full else a) - shift
            assert abs(got[i] - float(want)) <= 4.5e-16, (full, m[i], v[i], got[i], float(want))


def test_alpha_near_empty_and_full_cells(orc):
    """The plane constant of a nearly empty or nearly full cell is fixed exactly by the
    corner volume; step 2 moves such planes by a sizeable fraction of a cell, so an error
    in alpha there is carried into the new fraction at full weight."""
    _check_alpha_near_empty_and_full(orc.alpha_n)


def test_alpha_pin_catches_direct_inversion_near_full(tmp_path):
    """A copy of the oracle that inverts V = c directly also above one half (no
    complement) misses the corner's plane by about 1e-16 over the corner's area."""
    import oracle_mutants
    lib = oracle_mutants.build(tmp_path, [("    if (c > 0.5) return (S - bisect_alpha(m, 1.0 - c)) - shift;\n", "")])
    with pytest.raises(AssertionError):
        _check_alpha_near_empty_and_full(oracle_mutants.alpha_n_fn(lib))


def test_slab_bounds_additivity_and_planes(orc):
    rng = np.random.default_rng(21)
    for _ in range(400):
        m = rng.normal(size=3)
        if rng.uniform() < 0.3:
            m[rng.integers(0, 3)] = 0.0
        m /= np.abs(m).sum()
        c = rng.uniform(0.01, 0.99)
        a = orc.alpha_of(m, c)
        axis = int(rng.integers(0, 3))
        L = rng.uniform(0.0, 0.5)
        right = orc.slab(m, a, axis, L)    # region x_axis in [1-L, 1]
        left = orc.slab(m, a, axis, -L)    # region x_axis in [0, L]
        for F in (right, left):
            assert max(0.0, c - 1.0 + L) - 1e-15 <= F <= min(L, c) + 1e-15
        # the two complementary regions of one cell add up to its fraction
        rest = orc.slab(m, a, axis, -(1.0 - L))  # x_axis in [0, 1-L]
        assert right + rest == pytest.approx(c, abs=2e-15)
    # face-parallel interface: the liquid part of [1-L, 1] is [1-L, alpha]
    for a in (0.1, 0.55, 0.9):
        for L in (0.2, 0.5):
            assert orc.slab([1, 0, 0], a, 0, L) == pytest.approx(max(0.0, a - (1 - L)), abs=1e-16)
            assert orc.slab([1, 0, 0], a, 0, -L) == pytest.approx(min(a, L), abs=1e-16)
            # the same interface seen by a transverse sweep: the region is a full slab
            assert orc.slab([1, 0, 0], a, 1, L) == pytest.approx(L * a, abs=1e-16)


def test_slab_brute_force_bracket(orc):
    rng = np.random.default_rng(33)
    n = 40
    ax = (np.arange(n) + 0.0) / n
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    P = [X, Y, Z]
    for _ in range(10):
        m = rng.normal(size=3)
        m /= np.abs(m).sum()
        a = orc.alpha_of(m, rng.uniform(0.1, 0.9))
        axis = int(rng.integers(0, 3))
        L = rng.uniform(0.1, 0.5)
        sgn = rng.choice([-1.0, 1.0])
        base = m[0] * X + m[1] * Y + m[2] * Z
        mn = base + np.minimum(m, 0).sum() / n
        mx = base + np.maximum(m, 0).sum() / n
        lo_a = P[axis]
        hi_a = P[axis] + 1.0 / n
        if sgn > 0:
            full = lo_a >= 1 - L
            part = hi_a > 1 - L
        else:
            full = hi_a <= L
            part = lo_a < L
        inside = np.count_nonzero(full & (mx <= a)) / n ** 3
        touched = np.count_nonzero(part & (mn < a)) / n ** 3
        F = orc.slab(m, a, axis, sgn * L)
        assert inside - 1e-15 <= F <= touched + 1e-15
