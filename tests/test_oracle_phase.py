"""Pins of the oracle's step 2 (section 3.3.2: interface shift for the phase-change
source, capping, and the capped motion carried into the neighbours the interface
moves into) and the latent energy correction (section 3.4.1): exact motion of planar
fronts of any orientation, exact bookkeeping, and the paper's 2D evaporating
droplet with u = 0 (section 4.2) against R(t) = R0 - m'' t."""
from fractions import Fraction as Fr
import json
import math
import os

import numpy as np
import pytest

import exact
from paper_2001_03477_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _front(nx, xg, liquid_left=True, shape=(3, 3)):
    """Fractions of a plane x = xg (cell units) with the liquid on one side."""
    i = np.arange(nx)
    c = np.clip(xg - i, 0.0, 1.0) if liquid_left else np.clip(i + 1 - xg, 0.0, 1.0)
    return np.broadcast_to(c, shape + (nx,)).copy()


@pytest.mark.parametrize("mdot,liquid_left", [(0.37, True), (-0.37, True), (0.37, False)])
def test_planar_front_moves_exactly(orc, mdot, liquid_left):
    """A face-parallel front with constant m'' and no flow moves m'' dt / rho_l per step,
    also when it crosses cell faces (the capped remainder goes to the next cell)."""
    nx, h, dt, rho = 16, 1.0 / 16, 0.01, 2.0
    shift = mdot * dt / rho / h           # cell units per step (0.02960...)
    xg = 8.43
    c = _front(nx, xg, liquid_left)
    cfg = orc.Config(shape=c.shape, h=h, ndim=3, bc=(1, 0, 0), rho_l=rho, cp_l=5.0, cp_g=2.0,
                     T_gamma=1.5)
    e = 1.5 * (5.0 * c + 2.0 * (1 - c))
    md = np.full(c.shape, mdot)
    zero_u = np.zeros((3, 3, nx + 1))
    zero_v = np.zeros((3, 4, nx))
    zero_w = np.zeros((4, 3, nx))
    for n in range(1, 40):
        c, e, st = orc.step(cfg, c, e, zero_u, zero_v, zero_w, md, dt, 1.0, n)
        # evaporation moves the front into the liquid
        xg_n = xg - n * shift if liquid_left else xg + n * shift
        ref = _front(nx, xg_n, liquid_left)
        assert np.max(np.abs(c - ref)) < 1e-13 * n, n
        # T stays at T_Gamma: the latent correction keeps e = C_p(c) T_Gamma
        assert np.max(np.abs(e - 1.5 * (5.0 * c + 2.0 * (1 - c)))) < 1e-13 * n


def _plane_grid(nvec, x0, shape, nd):
    nz, ny, nx = shape
    out = np.zeros(shape)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                o = (i, j, 0 if nd == 2 else k)
                a = sum(Fr(nvec[q]) * (Fr(x0[q]) - o[q]) for q in range(3))
                out[k, j, i] = float(exact.volume(nvec, a))
    return out


@pytest.mark.parametrize("case", ["diag2d", "shallow2d", "oblique3d"])
def test_oblique_front_moves_exactly(orc, case):
    """Oblique planar fronts move exactly along their normal, also across cell
    corners: the neighbour that the moving plane enters takes the swept volume."""
    # the plane is not periodic: its kink at the wrapped boundary spreads at most two
    # cells per step (the neighbours' planes use 3x3x3 blocks), so only the cells
    # farther than 2 * steps + 2 from the boundary are compared
    steps = 4
    if case == "diag2d":
        shape, nd, nvec, x0, method = (1, 28, 28), 2, [1, 1, 0], [Fr(141, 10), Fr(14), 0], 1
    elif case == "shallow2d":
        shape, nd, nvec, x0, method = (1, 28, 28), 2, [Fr(1, 4), 1, 0], [Fr(14), Fr(139, 10), 0], 2
    else:
        steps = 3
        shape, nd, nvec, x0, method = (20, 20, 20), 3, [1, 1, 1], [Fr(10), Fr(10), Fr(97, 10)], 1
    mg = 2 * steps + 2
    norm = math.sqrt(sum(float(v) ** 2 for v in nvec))
    h, rho, mdot = 1.0 / shape[2], 1.0, 0.5
    dt = 0.37 * h / mdot                 # 0.37 cells per step along the normal
    c = _plane_grid(nvec, x0, shape, nd)
    cfg = orc.Config(shape=shape, h=h, ndim=nd, bc=(0, 0, 0), rho_l=rho, normal=method)
    md = np.full(shape, mdot)
    dist = 0.0
    for n in range(steps):
        c, _, _ = orc.phase_change(cfg, c, c.copy(), md, dt)
        dist += mdot * dt / rho / h
        # move the plane by dist along -n: n.(x - x0) <= -dist |n|
        shifted = [Fr(x0[q]) - Fr(dist) * Fr(float(nvec[q]) / norm) for q in range(3)]
        ref = _plane_grid(nvec, shifted, shape, nd)
        inner = np.s_[:, mg:-mg, mg:-mg] if nd == 2 else np.s_[mg:-mg, mg:-mg, mg:-mg]
        assert np.max(np.abs(c[inner] - ref[inner])) < 1e-12, (case, n)


def test_phase_change_bookkeeping(orc):
    """vol_phase is exactly the change of sum(c) in step 2, and the energy change is
    (C_pl - C_pg) T_Gamma times it, cell by cell."""
    wl = W.random_drops_3d(n=16, ndrops=4, seed=23, rmin=1.5, rmax=3.0)
    cfg = orc.Config(shape=wl.shape, h=wl.h, ndim=3, bc=(0, 0, 0), cp_l=wl.cp_l, cp_g=wl.cp_g,
                     rho_l=1.0, T_gamma=0.7)
    rng = np.random.default_rng(0)
    md = rng.uniform(-0.5, 1.0, size=wl.shape)
    for dt in (0.002, 0.02):
        c1, e1, acc = orc.phase_change(cfg, wl.c, wl.e, md, dt)
        dc = c1 - wl.c
        assert math.fsum(dc.ravel()) == pytest.approx(acc[0], abs=1e-14)
        assert np.allclose(e1 - wl.e, dc * (wl.cp_l - wl.cp_g) * 0.7, rtol=0, atol=1e-11)
        assert c1.min() >= 0.0 and c1.max() <= 1.0
        # only mixed cells and their face neighbours change
        mixed = (wl.c > 1e-12) & (wl.c < 1 - 1e-12)
        near = mixed.copy()
        for ax in range(3):
            near |= np.roll(mixed, 1, axis=ax) | np.roll(mixed, -1, axis=ax)
        assert np.all(dc[~near] == 0.0)
    # with one sign of m'' everywhere, evaporation only removes and condensation only adds
    for sgn in (1.0, -1.0):
        c1, _, _ = orc.phase_change(cfg, wl.c, wl.e, sgn * np.abs(md), 0.02)
        assert np.all(sgn * (c1 - wl.c) <= 0.0)


def test_phase_change_small_shift_matches_area_times_distance(orc):
    """For a small shift the removed volume is the interface area times the distance,
    i.e. the source term of step 2 (m''/rho_l) dt A_Gamma / V per mixed cell."""
    wl = W.random_drops_3d(n=16, ndrops=3, seed=29, rmin=2.5, rmax=4.0)
    cfg = orc.Config(shape=wl.shape, h=wl.h, ndim=3, bc=(0, 0, 0), rho_l=1.0)
    md = np.full(wl.shape, 1.0)
    dts = (1e-5, 2e-5)
    removed = []
    for dt in dts:
        c1, _, acc = orc.phase_change(cfg, wl.c, wl.e, md, dt)
        removed.append(-acc[0])
    # sum of A_i * |dd| over mixed cells, with A from the reconstruction, is linear in dt;
    # the realised removal matches it to second order
    r = removed[1] / removed[0]
    assert r == pytest.approx(2.0, rel=1e-4)
    # total interface area (cell units) ~ 4 pi R^2 / h^2 summed over the drops
    area_est = removed[0] / (1e-5 / wl.h)
    assert area_est > 0


@pytest.mark.parametrize("n", [32, 64])
def test_evaporating_droplet_2d_volume_law(orc, n):
    """Section 4.2 with u = 0 (the flow solver is outside the advection step): the
    droplet area follows pi (R0 - m'' t)^2 to first order in h."""
    gold = json.load(open(os.path.join(GOLDEN, "evaporating_droplet_2d.json")))
    R0, mdot = gold["R0"], gold["mdot"]
    dt = gold["dt"][gold["grids"].index(n)]
    h = 1.0 / n
    shape = (1, n, n)
    c = W.sphere_fraction(shape, h, [[0.5, 0.5, 0.0]], [R0], sub=16, nd=2)
    e = c.copy()
    cfg = orc.Config(shape=shape, h=h, ndim=2, bc=(1, 1, 0), rho_l=1.0)
    u = np.zeros((1, n, n + 1))
    v = np.zeros((1, n + 1, n))
    md = np.full(shape, mdot)
    t_end = 1.0
    steps = int(round(t_end / dt))
    errs = []
    for k in range(steps):
        c, e, st = orc.step(cfg, c, e, u, v, None, md, dt, 1.0, k)
        if (k + 1) % (steps // 4) == 0:
            t = (k + 1) * dt
            area = c.sum() * h * h
            ref = math.pi * (R0 - mdot * t) ** 2
            errs.append(abs(area - ref) / ref)
    # first order in h: below 1 % at n = 32 and halving with each refinement
    assert max(errs) < 0.008 * 32 / n, errs


def test_water_heat_capacity_ratio_matches_text():
    """Table 1: C_pl / C_pg for saturated water is the ~3200 quoted in section 3.4.1."""
    w = json.load(open(os.path.join(GOLDEN, "water_properties.json")))
    ratio = w["liquid"]["Cp_kJ_per_m3K"] / w["gas"]["Cp_kJ_per_m3K"]
    assert ratio == pytest.approx(w["stated_ratio_Cpl_over_Cpg"], rel=0.02)
    assert w["liquid"]["rho"] * w["liquid"]["cp_kJ_per_kgK"] == pytest.approx(
        w["liquid"]["Cp_kJ_per_m3K"], rel=0.001)
