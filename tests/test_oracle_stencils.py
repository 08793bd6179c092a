"""Pins of the oracle's stencils: the interface normal (Youngs and the mixed
Youngs-centred selection named in section 3.2) on exact planar blocks, and the
WENO5 face temperature of section 3.4.1 (Jiang-Shu) by exactness, convergence
order and non-oscillation."""
import math

import numpy as np
import pytest

import exact


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
        m = orc.normal(blk, 2)
        assert np.allclose(m, _unit1(n), atol=2e-15, rtol=0), (n, m)
        if nd == 2:
            assert m[2] == 0.0


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
