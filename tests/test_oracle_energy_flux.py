"""Pins of the oracle's non-conservative energy flux (section 3.4.1, eq.
disc_et_adv_noncons), the approximation the paper compares the conservative flux of
eq. disc_et_adv against: the face carries lambda T_f and each cell scales the
difference of its two faces by its own heat capacity.

* Equal phase heat capacities: both fluxes are C_p lambda T_f, so the two modes agree
  to round-off for any fractions.
* Linear temperature in pure cells: WENO5 reproduces a linear profile exactly at the
  faces, so one sweep reduces to the closed form
  e' = e - C_p(c) (lam_R T(x_R) - lam_L T(x_L)) + e_c (lam_R - lam_L).
* Uniform temperature and uniform velocity: the non-conservative update leaves e
  unchanged in every cell, while the volume moves, so the temperature of interface
  cells drifts; the conservative flux keeps the temperature uniform instead.
* The fractions do not depend on the energy flux."""
import math

import numpy as np

from paper_2001_03477_amd import workloads as W


def _cfg(orc, wl, **kw):
    args = dict(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal)
    args.update(kw)
    return orc.Config(**args)


def _steps(orc, cfg, wl, n, mdot=None):
    c, e = wl.c, wl.e
    for k in range(n):
        c, e, st = orc.step(cfg, c, e, wl.u, wl.v, wl.w, mdot, wl.dt, 1.0, k)
    return c, e, st


def test_equal_heat_capacities_make_the_fluxes_agree(orc):
    wl = W.random_drops_3d(n=16, ndrops=4, seed=81, rmin=1.5, rmax=3.0)
    wl.cp_l = wl.cp_g = 2.5
    wl.e = 2.5 * np.random.default_rng(81).uniform(0.2, 1.0, size=wl.shape)
    for bc in ((0, 0, 0), (1, 1, 1)):
        c0, e0, _ = _steps(orc, _cfg(orc, wl, bc=bc), wl, 2)
        c1, e1, _ = _steps(orc, _cfg(orc, wl, bc=bc, energy_flux=1), wl, 2)
        assert np.array_equal(c0, c1)
        assert np.max(np.abs(e1 - e0)) <= 1e-14 * np.max(np.abs(e0))


def test_linear_temperature_in_pure_cells_is_the_closed_form(orc):
    """One x sweep of a row of pure cells (liquid and gas blocks) with T linear in x and
    a non-uniform face velocity; cells at least three from a boundary see exact WENO5
    face temperatures."""
    n = 40
    h = 1.0 / n
    shape = (1, 1, n)
    c = np.zeros(shape)
    c[..., 8:20] = 1.0
    c[..., 27:33] = 1.0
    xc = (np.arange(n) + 0.5) * h
    T = 0.3 + 2.0 * xc
    cp_l, cp_g = 4.0, 0.5
    cp = cp_l * c + cp_g * (1 - c)
    e = cp * T[None, None, :]
    xf = np.arange(n + 1) * h
    lam = 0.2 + 0.1 * np.sin(2 * np.pi * xf)          # face CFL numbers, all positive
    u = np.broadcast_to(lam, (1, 1, n + 1)).copy()
    cfg = orc.Config(shape=shape, h=h, ndim=2, bc=(1, 1, 1), cp_l=cp_l, cp_g=cp_g, energy_flux=1)
    cc, ec = orc.prologue(cfg, c, e)
    c1, e1, _ = orc.sweep(cfg, 0, c, e, cc, ec, u, 1.0)
    Tf = 0.3 + 2.0 * xf
    i = np.arange(3, n - 3)
    expect = (e[0, 0, i] - cp[0, 0, i] * (lam[i + 1] * Tf[i + 1] - lam[i] * Tf[i])
              + ec[0, 0, i] * (lam[i + 1] - lam[i]))
    assert np.max(np.abs(e1[0, 0, i] - expect)) <= 1e-13 * np.max(np.abs(e))
    # and the conservative flux differs where the upwind heat capacity differs
    cfg0 = orc.Config(shape=shape, h=h, ndim=2, bc=(1, 1, 1), cp_l=cp_l, cp_g=cp_g)
    _, e0, _ = orc.sweep(cfg0, 0, c, e, cc, ec, u, 1.0)
    assert np.max(np.abs(e0[0, 0, i] - e1[0, 0, i])) > 1e-3 * np.max(np.abs(e))


def test_uniform_temperature_and_velocity_leave_the_energy_unchanged(orc):
    """One sweep with a uniform temperature and a uniform face velocity: the
    non-conservative update keeps e in every cell while the volume moves, so the
    temperature of the cells the interface moved through drifts; the conservative
    flux keeps the temperature uniform."""
    n = 16
    wl = W.random_drops_3d(n=n, ndrops=4, seed=82, rmin=1.5, rmax=3.0, cp=(4039.0, 1.248))
    T0 = 0.75
    e = (wl.cp_l * wl.c + wl.cp_g * (1 - wl.c)) * T0
    u = np.full((n, n, n + 1), 0.24)
    for mode in (1, 0):
        cfg = _cfg(orc, wl, energy_flux=mode)
        cc, ec = orc.prologue(cfg, wl.c, e)
        c1, e1, _ = orc.sweep(cfg, 0, wl.c, e, cc, ec, u, 1.0)
        T1 = e1 / (wl.cp_l * c1 + wl.cp_g * (1 - c1))
        moved = np.abs(c1 - wl.c) > 1e-3
        assert moved.any()
        if mode == 1:
            # cells clipped into [0, 1] (round-off of the fluxes) end at exactly 0 or 1
            # and have their energy adjusted; every other cell keeps e exactly
            kept = (c1 == wl.c) | ((c1 > 0.0) & (c1 < 1.0))
            assert kept.mean() > 0.99
            assert np.array_equal(e1[kept], e[kept])
            assert np.max(np.abs(T1[moved] - T0)) > 0.1 * T0
        else:
            assert np.max(np.abs(T1 - T0)) <= 1e-13 * T0


def test_nonconservative_flux_does_not_conserve_energy(orc):
    """Periodic, divergence-free: the conservative flux keeps the total energy to
    round-off (net of the dilatation and clip terms), the non-conservative one does not
    when the heat capacities differ."""
    wl = W.random_drops_3d(n=16, ndrops=4, seed=83, rmin=1.5, rmax=3.0, cp=(4039.0, 1.248))
    hv = wl.h ** 3
    e_tot0 = math.fsum(wl.e.ravel()) * hv
    res = {}
    for mode in (0, 1):
        cfg = _cfg(orc, wl, energy_flux=mode)
        c, e, prev, r = wl.c, wl.e, e_tot0, 0.0
        for k in range(2):
            c, e, st = orc.step(cfg, c, e, wl.u, wl.v, wl.w, None, wl.dt, 1.0, k)
            r += st["energy"] - prev - (-st["energy_bnd_out"] + st["energy_src"] + st["energy_clip"])
            prev = st["energy"]
        res[mode] = abs(r) / abs(e_tot0)
    assert res[0] <= 1e-13
    assert res[1] > 1e-6
