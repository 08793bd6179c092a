"""Pins of the oracle's implicit energy diffusion with the interface temperature imposed
(section 3.4.2, eqs. T_diff_disc and mod_branchesT).

* Without an interface (one phase, periodic) the step is the backward-Euler heat
  equation with the 7-point Laplacian, whose solution the discrete Fourier transform
  gives in closed form.
* The height-function distance is exact for planes, tilted ones included: the column
  sum of the fractions is the interface position at the column's centre line.
* The irregular stencil of eq. T_diff_disc is exact for a profile that is linear (zero)
  or quadratic (2 b k) in the normal direction on each side and equals T_Gamma at a
  planar interface.
* Maximum principle: the new temperatures stay within the old ones and T_Gamma.
* Steady limit: a very long step drives every node towards T_Gamma (every phase region
  touches the interface; outflow walls are adiabatic).
* Mirror symmetry of a centred sphere.
* The solve is backward Euler with that (pinned) operator at every node, also where a
  one-cell film puts the interface on both sides of a node."""
import numpy as np
import pytest

import oracle
from oracle import diffusion as D
from paper_2001_03477_amd import workloads as W


def _cfg(shape, ndim, bc, cp=(2.5, 0.25)):
    return oracle.Config(shape=shape, h=1.0 / shape[2], ndim=ndim, bc=bc, cp_l=cp[0], cp_g=cp[1])


@pytest.mark.parametrize("ndim", [2, 3])
def test_single_phase_is_the_fourier_solution(ndim):
    shape = (1, 10, 12) if ndim == 2 else (6, 8, 10)
    h = 1.0 / shape[2]
    T = np.random.default_rng(1).uniform(0.0, 1.0, size=shape)
    c = np.ones(shape)
    cfg = _cfg(shape, ndim, (0, 0, 0))
    k_l, dt = 0.7, 3e-3
    got = D.diffuse(cfg, c, T, dt, k_l, 0.1, 0.5)
    a = dt * k_l / cfg.cp_l
    lam = np.zeros(shape)
    for ax, n in enumerate(shape):
        if ndim == 2 and ax == 0:
            continue
        kk = np.arange(n).reshape([-1 if i == ax else 1 for i in range(3)])
        lam = lam + 4.0 / h ** 2 * np.sin(np.pi * kk / n) ** 2
    want = np.real(np.fft.ifftn(np.fft.fftn(T) / (1.0 + a * lam)))
    assert np.max(np.abs(got - want)) <= 1e-13


def test_height_distance_exact_for_planes():
    """A tilted front x = x0 + s y in 2D (outflow): every node with a neighbour of the
    other phase along x gets theta = its distance along x to the front (capped)."""
    nx, ny = 24, 12
    shape = (1, ny, nx)
    h = 1.0 / nx
    for x0, s, liquid_left in ((9.37, 0.23, True), (10.6, -0.31, False)):
        c = W.line_fraction_field(shape, h, x0 * h, s)
        if not liquid_left:
            c = 1.0 - c
        checked = 0
        for j in range(ny):
            for i in range(nx - 1):
                a, b = (0, j, i), (0, j, i + 1)
                if (c[a] >= 0.5) == (c[b] >= 0.5):
                    continue
                xg = x0 + s * (j + 0.5)  # front at this row's centre line (cell units)
                for node, step in ((a, 1), (b, -1)):
                    got = D.theta(c, (1, 1, 0), node, 0, step)
                    exact = abs(xg - (node[2] + 0.5))
                    assert got == pytest.approx(min(max(exact, 1e-3), 1.0), abs=1e-13), (j, i, step)
                    checked += 1
        assert checked >= 2 * ny


def _planar(shape, xg, liquid_left=True):
    nz, ny, nx = shape
    c = np.zeros(shape)
    for i in range(nx):
        left = min(max(xg - i, 0.0), 1.0)
        c[:, :, i] = left if liquid_left else 1.0 - left
    return c


@pytest.mark.parametrize("liquid_left", [True, False])
def test_stencil_exact_for_linear_and_quadratic_profiles(liquid_left):
    shape = (3, 4, 20)
    h = 1.0 / shape[2]
    xg_cells = 9.3
    c = _planar(shape, xg_cells, liquid_left)
    cfg = _cfg(shape, 3, (1, 0, 0))
    k_l, k_g, Tg = 0.7, 0.07, 1.0
    x = (np.arange(shape[2]) + 0.5) * h
    xg = xg_cells * h
    liquid = c >= 0.5
    interior = np.zeros(shape, dtype=bool)
    interior[:, :, 1:-1] = True  # the outflow walls are adiabatic: not linear there
    for gl, gg, b in ((1.3, -0.4, 0.0), (0.6, 2.0, 5.0)):
        T = np.where(liquid, Tg + gl * (x - xg) + b * (x - xg) ** 2, Tg + gg * (x - xg) + b * (x - xg) ** 2)
        L = D.apply_operator(cfg, c, T, k_l, k_g, Tg)
        want = np.where(liquid, 2 * b * k_l, 2 * b * k_g)
        assert np.max(np.abs(L[interior] - want[interior])) <= 1e-9 * max(1.0, 2 * b * k_l), (gl, gg, b)


def test_maximum_principle_and_steady_limit():
    wl = W.random_drops_3d(n=14, ndrops=3, seed=61, rmin=1.5, rmax=3.5)
    T = np.random.default_rng(61).uniform(0.2, 0.8, size=wl.shape)
    for bc in ((0, 0, 0), (1, 1, 1)):
        cfg = _cfg(wl.shape, 3, bc)
        out = D.diffuse(cfg, wl.c, T, 2e-3, 0.07, 0.007, 0.5)
        assert out.min() >= 0.2 - 1e-14 and out.max() <= 0.8 + 1e-14
        assert np.max(np.abs(out - T)) > 1e-4  # it did diffuse
        steady = D.diffuse(cfg, wl.c, T, 1e9, 0.07, 0.007, 0.5)
        assert np.max(np.abs(steady - 0.5)) <= 1e-6


def test_sphere_mirror_symmetry():
    n = 12
    c = W.sphere_fraction((n, n, n), 1.0 / n, [np.array([0.5, 0.5, 0.5])], [0.27])
    x = (np.arange(n) + 0.5) / n
    T = 0.3 + (x[None, None, :] - 0.5) ** 2 + 0.5 * (x[None, :, None] - 0.5) ** 2 + 0.0 * x[:, None, None]
    cfg = _cfg(c.shape, 3, (0, 0, 0))
    out = D.diffuse(cfg, c, T, 1e-2, 0.07, 0.007, 1.0)
    assert np.max(np.abs(out - out[:, :, ::-1])) <= 1e-13
    assert np.max(np.abs(out - out[::-1, :, :])) <= 1e-13


def test_step_is_backward_euler_with_the_pinned_operator():
    """The solve's T^{n+1} satisfies C_p (T^{n+1} - T) / dt = apply_operator(T^{n+1}) at
    every node (C_p of the node's phase), on drops with both boundary types and a thin
    film whose nodes see the interface on both sides."""
    wl = W.random_drops_3d(n=14, ndrops=3, seed=62, rmin=1.5, rmax=3.5)
    T = np.random.default_rng(62).uniform(0.2, 0.8, size=wl.shape)
    film = np.zeros((1, 6, 16))
    film[:, :, 7] = 0.8  # one liquid cell thick: interface on both sides of its nodes
    cases = [(wl.c, T, (0, 0, 0), 3), (wl.c, T, (1, 1, 1), 3),
             (film, np.random.default_rng(63).uniform(0.2, 0.8, size=film.shape), (1, 0, 0), 2)]
    for c, T0, bc, ndim in cases:
        cfg = _cfg(c.shape, ndim, bc)
        dt, k_l, k_g, Tg = 3e-3, 0.07, 0.007, 0.5
        out = D.diffuse(cfg, c, T0, dt, k_l, k_g, Tg)
        C = np.where(c >= 0.5, cfg.cp_l, cfg.cp_g)
        lhs = C * (out - T0) / dt
        rhs = D.apply_operator(cfg, c, out, k_l, k_g, Tg)
        assert np.max(np.abs(lhs - rhs)) <= 1e-9 * np.max(np.abs(rhs)), bc
