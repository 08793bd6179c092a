"""Pins of the oracle's stencils: the interface normal (Youngs and the mixed
Youngs-centred selection named in section 3.2) on exact planar blocks, and the
WENO5 face temperature of section 3.4.1 (Jiang-Shu) by exactness, convergence
order and non-oscillation.

The mixed Youngs-centred selection (method 1) is pinned by what the exact geometry
fixes: on shallow planes the centred columns bracket the interface and are exact, so
method 1 must return them; on a 45 degree line through the block off its centre
Youngs' gradient is exact by the x-y symmetry while the columns do not bracket the
line, so method 1 must return Youngs; over random exact planes it must return the
more accurate of the two candidates nearly always. A copy of the oracle with the
selection inverted fails each of these pins."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import exact
import oracle_mutants


def _unit1(n):
    n = np.asarray(n, dtype=float)
    return n / np.abs(n).sum()


@pytest.mark.parametrize("method", [0, 1, 2])
def test_normal_axis_aligned_planes(orc, method):
    for axis in range(3):
        for sgn in (1, -1):
            n = [0, 0, 0]
            n[axis] = sgn
            for off in ("0.3", "0.71"):
                x0 = [0.5, 0.5, 0.5]
                x0[axis] = float(off)
                blk = exact.plane_block(n, x0)
                m = orc.normal(blk, method)
                assert np.array_equal(m, np.asarray(n, dtype=float)), (axis, sgn, m)


def test_normal_body_diagonal(orc):
    for signs in [(1, 1, 1), (1, -1, 1), (-1, -1, 1), (-1, 1, -1)]:
        blk = exact.plane_block(signs, [0.5, 0.5, 0.5])
        for method in (0, 1):
            m = orc.normal(blk, method)
            assert np.allclose(m, np.asarray(signs) / 3.0, atol=1e-15, rtol=0)


@pytest.mark.parametrize("nd", [2, 3])
def test_centred_columns_exact_on_shallow_planes(orc, nd):
    """With the dominant axis d and transverse slopes below 1/2, every 3-cell column
    along d contains the interface, so the column heights are exact and the
    centred-columns normal reproduces the plane."""
    rng = np.random.default_rng(4 + nd)
    for _ in range(60):
        d = int(rng.integers(0, 3)) if nd == 3 else int(rng.integers(0, 2))
        n = np.zeros(3)
        n[d] = rng.choice([-1.0, 1.0])
        for t in range(3):
            if t != d and (nd == 3 or t != 2):
                n[t] = rng.uniform(-0.45, 0.45)
        n = [float(v) for v in n]
        x0 = [0.5, 0.5, 0.5]
        x0[d] = rng.uniform(0.3, 0.7)
        blk = exact.plane_block(n, x0, nd=nd)
        for method in (2, 1):
            m = orc.normal(blk, method)
            assert np.allclose(m, _unit1(n), atol=2e-15, rtol=0), (method, n, m)
            if nd == 2:
                assert m[2] == 0.0


def _angle(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    cs = float(a @ b) / (np.linalg.norm(a) * np.linalg.norm(b))
    return math.acos(max(-1.0, min(1.0, cs)))


def _shallow_blocks(nd, count, seed):
    """Exact blocks of planes whose transverse slopes (relative to the dominant axis)
    are below 1/2, so that every 3-cell column along that axis brackets the plane."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = int(rng.integers(0, 3)) if nd == 3 else int(rng.integers(0, 2))
        n = np.zeros(3)
        n[d] = rng.choice([-1.0, 1.0])
        for t in range(3):
            if t != d and (nd == 3 or t != 2):
                n[t] = rng.uniform(-0.45, 0.45)
        x0 = [0.5, 0.5, 0.5]
        x0[d] = rng.uniform(0.3, 0.7)
        n = [float(v) for v in n]
        out.append((exact.plane_block(n, x0, nd=nd), n))
    return out


def _diagonal_blocks():
    """Exact blocks of 45 degree planes (two components of the normal of equal
    magnitude, the third zero) through points off the block's centre along the first
    of the two axes; (block, exact normal with |n|_1 = 1)."""
    out = []
    for a, b in ((0, 1), (1, 2), (0, 2)):
        for sa, sb in ((1, 1), (1, -1), (-1, -1)):
            for k in (1, 3, 5, 11, 13, 15):
                n = [0, 0, 0]
                n[a], n[b] = sa, sb
                x0 = [Fr(1, 2)] * 3
                x0[a] = Fr(k, 16)
                nd = 2 if 2 not in (a, b) else 3
                out.append((exact.plane_block(n, x0, nd=nd), _unit1(n)))
    return out


def _random_blocks(count, seed):
    """Exact blocks of random planes (normal and point on a 1/64 lattice) whose
    central cell is mixed; (block, exact normal)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = np.round(rng.normal(size=3) * 64) / 64
        if not np.any(n):
            continue
        x0 = np.round(rng.uniform(0.2, 0.8, size=3) * 64) / 64
        blk = exact.plane_block([float(v) for v in n], [float(v) for v in x0])
        if 1e-12 < blk[1, 1, 1] < 1 - 1e-12:
            out.append((blk, n))
    return out


def _check_myc_shallow(normal):
    for nd in (2, 3):
        for blk, n in _shallow_blocks(nd, 40, 40 + nd):
            m = normal(blk, 1)
            assert np.allclose(m, _unit1(n), atol=2e-15, rtol=0), ("shallow", n, m)


def _check_myc_diagonal(normal):
    for blk, n in _diagonal_blocks():
        m0, m1, m2 = normal(blk, 0), normal(blk, 1), normal(blk, 2)
        # Youngs is exact here (x-y symmetry of the block), the columns are not
        assert np.array_equal(m0, n), ("youngs", n, m0)
        assert np.max(np.abs(m2 - n)) > 1e-4, ("columns", n, m2)
        assert np.array_equal(m1, m0), ("diagonal", n, m1)


def _myc_pick_rate(normal, blocks):
    """Fraction of the blocks (those where Youngs' and the centred-columns normal differ
    in accuracy by more than 1e-9 rad) on which method 1 returns the more accurate of
    the two; also checks that method 1 always returns one of them."""
    better = decided = 0
    for blk, n in blocks:
        m0, m1, m2 = normal(blk, 0), normal(blk, 1), normal(blk, 2)
        assert np.array_equal(m1, m0) or np.array_equal(m1, m2)
        e0, e2 = _angle(m0, n), _angle(m2, n)
        if abs(e0 - e2) <= 1e-9:
            continue
        decided += 1
        better += np.array_equal(m1, m0 if e0 < e2 else m2)
    return better / decided, decided


@pytest.fixture(scope="module")
def random_plane_blocks():
    return _random_blocks(600, 61)


def test_myc_falls_back_to_youngs_on_diagonal_planes(orc):
    """On 45 degree planes through the block off its centre the 3-cell columns do not
    bracket the plane (their heights are clipped), which flattens the centred-columns
    candidate: its own component exceeds every component of Youngs' normal, and the
    mixed selection must return Youngs, which the block's symmetry makes exact."""
    _check_myc_diagonal(orc.normal)


def test_myc_picks_the_more_accurate_candidate(orc, random_plane_blocks):
    rate, decided = _myc_pick_rate(orc.normal, random_plane_blocks)
    assert decided >= 500
    assert rate >= 0.95, rate


def _check_myc_tie_band(normal):
    """Along the family of planes n = (1, s, 0) through (1/16, 1/2, 1/2) the selection
    switches from the centred columns to Youngs where the columns' own component
    overtakes Youngs' largest one. Just inside the band (0 < own - max|m_Youngs| <=
    1e-12) the columns are kept, just outside it Youngs is taken."""
    x0 = [Fr(1, 16), Fr(1, 2), Fr(1, 2)]

    def gap(s):
        blk = exact.plane_block([1.0, s, 0.0], x0, nd=2)
        m0, m2 = normal(blk, 0), normal(blk, 2)
        return np.max(np.abs(m2)) - np.max(np.abs(m0)), blk, m0, m2

    lo, hi = 13 / 16, 14 / 16
    assert gap(lo)[0] < 0 and gap(hi)[0] > 1e-6

    def find(target):
        a, b = lo, hi
        for _ in range(200):
            mid = 0.5 * (a + b)
            g = gap(mid)[0]
            if abs(g - target) <= 0.4 * target:
                return mid
            if g < target:
                a = mid
            else:
                b = mid
        raise RuntimeError("no plane with the requested gap")

    g, blk, m0, m2 = gap(find(5e-13))
    assert 0 < g <= 1e-12 and not np.array_equal(m0, m2)
    assert np.array_equal(normal(blk, 1), m2), "inside the tie band"
    g, blk, m0, m2 = gap(find(1e-10))
    assert g > 1e-12
    assert np.array_equal(normal(blk, 1), m0), "outside the tie band"


def test_myc_exact_on_shallow_planes(orc):
    _check_myc_shallow(orc.normal)


def test_myc_tie_band(orc):
    """Candidates within 1e-12 of each other count as equal (the reading that keeps
    1e-16 input differences from switching formulas)."""
    _check_myc_tie_band(orc.normal)


def test_myc_tie_band_pin_catches_a_missing_band(tmp_path):
    lib = oracle_mutants.build(tmp_path, [("if (best_own > ymax + NORMAL_TIE) {", "if (best_own > ymax) {")])
    with pytest.raises(AssertionError, match="inside the tie band"):
        _check_myc_tie_band(oracle_mutants.normal_fn(lib))


def test_myc_pins_catch_an_inverted_selection(tmp_path, random_plane_blocks):
    """The same pins on a copy of the oracle whose selection test is inverted (Youngs
    taken exactly where the centred columns should be): each pin fails."""
    lib = oracle_mutants.build(tmp_path, [("if (best_own > ymax + NORMAL_TIE) {",
                                           "if (!(best_own > ymax + NORMAL_TIE)) {")])
    normal = oracle_mutants.normal_fn(lib)
    with pytest.raises(AssertionError):
        _check_myc_shallow(normal)
    with pytest.raises(AssertionError):
        _check_myc_diagonal(normal)
    rate, _ = _myc_pick_rate(normal, random_plane_blocks)
    assert rate < 0.5, rate


def test_normal_orientation_and_symmetry(orc):
    rng = np.random.default_rng(8)
    for _ in range(100):
        blk = rng.uniform(0, 1, size=(3, 3, 3))
        for method in (0, 1):
            m = orc.normal(blk, method)
            assert abs(np.abs(m).sum() - 1.0) < 1e-15
            # reflecting the block along x reflects the normal
            mr = orc.normal(blk[:, :, ::-1], method)
            assert np.allclose(mr * np.array([-1, 1, 1]), m, atol=1e-15)
            # swapping x and y swaps the components
            ms = orc.normal(np.transpose(blk, (0, 2, 1)), method)
            if method == 0:
                assert np.allclose(ms[[1, 0, 2]], m, atol=1e-15)
    # liquid below (small z) makes the normal point to +z, i.e. from liquid to gas
    blk = exact.plane_block([0.1, -0.2, 1.0], [0.5, 0.5, 0.6])
    assert orc.normal(blk, 1)[2] > 0
    # a uniform block has no gradient: the documented fallback (1, 0, 0)
    assert np.array_equal(orc.normal(np.full(27, 0.4), 1), [1.0, 0.0, 0.0])


def test_youngs_exact_on_linear_fields(orc):
    """On a linearly varying block c = c0 + g.o every weighted central difference
    equals twice the slope, so Youngs' normal is exactly -g/|g|_1: checks the sign
    convention (m along -grad c) and that all three axes use the same weights."""
    rng = np.random.default_rng(12)
    o = np.array([[(dx, dy, dz) for dx in (-1, 0, 1)] for dz in (-1, 0, 1) for dy in (-1, 0, 1)])
    o = o.reshape(3, 3, 3, 3)
    for _ in range(100):
        # power-of-two slopes keep every difference exact
        g = rng.integers(-8, 9, size=3) / 64.0
        if not np.any(g):
            continue
        blk = 0.5 + o[..., 0] * g[0] + o[..., 1] * g[1] + o[..., 2] * g[2]
        m = orc.normal(blk, 0)
        assert np.array_equal(m, -g / np.abs(g).sum()), (g, m)


def test_weno5_exact_on_constants_and_quadratics(orc):
    for v in (0.0, 1.0, -3.25, 7.5e3):
        assert orc.weno5([v] * 5) == pytest.approx(v, rel=4e-16, abs=1e-300)
    # cell averages of a quadratic: each candidate stencil reproduces the face value,
    # so the face value is exact whatever the nonlinear weights are
    rng = np.random.default_rng(2)
    for _ in range(50):
        a, b, cq = rng.normal(size=3)
        avg = [a * ((i + 1) ** 3 - i ** 3) / 3 + b * ((i + 1) ** 2 - i ** 2) / 2 + cq
               for i in range(-2, 3)]
        xf = 1.0
        assert orc.weno5(avg) == pytest.approx(a * xf * xf + b * xf + cq, abs=1e-13)


def test_weno5_fifth_order_on_smooth_data(orc):
    errs = []
    for n in (20, 40, 80):
        h = 1.0 / n
        e = 0.0
        for i in range(n):
            # cell averages of sin(2 pi x) on cells i-2..i+2; face at x_{i+1/2} = (i+1) h
            avg = [(math.cos(2 * math.pi * (j) * h) - math.cos(2 * math.pi * (j + 1) * h)) /
                   (2 * math.pi * h) for j in range(i - 2, i + 3)]
            e = max(e, abs(orc.weno5(avg, 1e-6) - math.sin(2 * math.pi * (i + 1) * h)))
        errs.append(e)
    r1 = errs[0] / errs[1]
    r2 = errs[1] / errs[2]
    assert r2 > 2 ** 4.5 and r1 > 2 ** 3.5, errs


def test_weno5_non_oscillatory_at_a_jump(orc):
    # the only smooth candidate (the leftmost) dominates the face value
    assert abs(orc.weno5([0, 0, 0, 1, 1])) < 1e-10
    assert abs(orc.weno5([1, 1, 1, 0, 0]) - 1.0) < 1e-10
    rng = np.random.default_rng(4)
    for _ in range(200):
        v = np.where(np.arange(5) < rng.integers(1, 5), rng.uniform(0, 1), rng.uniform(2, 3))
        f = orc.weno5(v)
        assert v.min() - 1e-12 <= f <= v.max() + 1e-12
