"""Pins of the oracle's Lagrangian-explicit sweeps (the method of Li, also called CIAM,
which section 3.3 names beside the Weymouth-Yue scheme it builds on), kept as an
ablation of the conservative split.

A Lagrangian-explicit sweep moves every point of a cell with the face velocity
interpolated linearly between the cell's two faces, so the cell is stretched by
s = 1 + (lam_R - lam_L) and its plane stays a plane. What that fixes:

* A plane moved by a velocity that is linear along the sweep axis lands exactly where
  the linear map puts it, in every cell (the interpolation is exact), for an
  axis-aligned plane and for a tilted one whose centred-column normal is exact. The
  Weymouth-Yue sweep does not reproduce this compressible motion.
* The pieces that the mapped cells leave in a cell tile it, so the fractions stay in
  [0, 1] with no clipping beyond round-off.
* A uniform temperature stays uniform (the energy flux carries the same liquid and gas
  volumes as the volume flux).
* A uniform velocity stretches nothing: the sweep is the Weymouth-Yue sweep.
* In a periodic divergence-free field the volume changes by the dilatation terms
  sum c (lam_R - lam_L), which do not cancel over the sweeps of a step: the scheme is
  not conservative, unlike the frozen c_c of the Weymouth-Yue split."""
import math

import numpy as np

from paper_2001_03477_amd import workloads as W


def _linear_setup(n, ny, slope, x_gamma, a_lam, x0):
    """2D grid n x ny, outflow; liquid left of the line x = x_gamma + slope y; face CFL
    numbers lam(x) = a_lam (x - x0) / h along x, none along y."""
    h = 1.0 / n
    shape = (1, ny, n)
    c = W.line_fraction_field(shape, h, x_gamma, slope)
    xf = np.arange(n + 1) * h
    lam = a_lam * (xf - x0) / h
    u = np.broadcast_to(lam, (1, ny, n + 1)).copy()
    return h, shape, c, u


def _mapped_fractions(h, shape, x_gamma, slope, a_lam, x0):
    """Exact fractions after the displacement lam(x) h = a_lam (x - x0): the line
    x = x_gamma + slope y goes to x = x_gamma + a_lam (x_gamma - x0) + slope (1 + a_lam) y."""
    k = 1.0 + a_lam
    xg = x_gamma + a_lam * (x_gamma - x0)
    return W.line_fraction_field(shape, h, xg, slope * k)


def _sweep(orc, cfg, c, e, u, axis=0):
    cc, ec = orc.prologue(cfg, c, e)
    return orc.sweep(cfg, axis, c, e, cc, ec, u, 1.0)


def test_plane_under_linear_velocity_is_exact(orc):
    """Axis-aligned and tilted planes, stretching (a > 0) and compressing (a < 0)
    fields, centred-column normals (exact for these planes away from the outflow rows
    y = 0 and y = ny - 1, whose ghost copies bend a tilted plane: those rows are not
    compared)."""
    n, ny = 32, 12
    for slope, a_lam, x0 in ((0.0, 0.3, 0.4), (0.0, -0.3, 0.5), (0.2, 0.25, 0.45), (-0.15, -0.35, 0.55)):
        a = a_lam * (1.0 / n)  # lam = a (x - x0) / h spans about +-0.15 over the box
        x_gamma = 0.431 if slope == 0.0 else 0.40
        h, shape, c, u = _linear_setup(n, ny, slope, x_gamma, a, x0)
        assert np.max(np.abs(u)) <= 0.5
        e = 1.0 + c
        cfg = orc.Config(shape=shape, h=h, ndim=2, bc=(1, 1, 1), normal=2, split=1)
        c1, _, st = _sweep(orc, cfg, c, e, u)
        want = _mapped_fractions(h, shape, x_gamma, slope, a, x0)
        rows = slice(1, ny - 1)
        assert np.max(np.abs(c1[:, rows] - want[:, rows])) <= 1e-14, (slope, a_lam)
        assert abs(st[0]) <= 1e-15  # clipped volume (cell units)
        # the Weymouth-Yue sweep moves the same plane differently
        cfg_wy = orc.Config(shape=shape, h=h, ndim=2, bc=(1, 1, 1), normal=2, split=0)
        c0, _, _ = _sweep(orc, cfg_wy, c, e, u)
        assert np.max(np.abs(c0[:, rows] - want[:, rows])) > 1e-4


def test_fractions_stay_bounded_without_clipping(orc):
    """Drops in a random divergence-free field at CFL 0.45, both normals, periodic and
    outflow: every sweep keeps c in [0, 1] up to round-off."""
    wl = W.random_drops_3d(n=16, ndrops=5, seed=71, cfl=0.45, rmin=1.5, rmax=3.5)
    for normal in (0, 1):
        for bc in ((0, 0, 0), (1, 1, 1)):
            cfg = orc.Config(shape=wl.shape, h=wl.h, ndim=3, bc=bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                             normal=normal, split=1)
            c, e = wl.c, wl.e
            for k in range(3):
                c, e, st = orc.step(cfg, c, e, wl.u, wl.v, wl.w, None, wl.dt, 1.0, k)
                assert abs(st["vol_clip"]) <= 1e-13 * wl.h ** 3, (normal, bc, k)


def test_uniform_temperature_stays_uniform(orc):
    wl = W.random_drops_3d(n=16, ndrops=5, seed=72, rmin=1.5, rmax=3.5, cp=(4039.0, 1.248))
    T0 = 0.625
    for bc in ((0, 0, 0), (1, 0, 1)):
        cfg = orc.Config(shape=wl.shape, h=wl.h, ndim=3, bc=bc, cp_l=wl.cp_l, cp_g=wl.cp_g, split=1)
        c, e = wl.c, (wl.cp_l * wl.c + wl.cp_g * (1 - wl.c)) * T0
        for k in range(2):
            c, e, _ = orc.step(cfg, c, e, wl.u, wl.v, wl.w, None, wl.dt, 1.0, k)
        T = e / (wl.cp_l * c + wl.cp_g * (1 - c))
        assert np.max(np.abs(T - T0)) <= 1e-12 * T0, bc


def test_uniform_velocity_is_the_weymouth_yue_sweep(orc):
    wl = W.random_drops_3d(n=16, ndrops=4, seed=73, rmin=1.5, rmax=3.5)
    n = 16
    u = np.full((n, n, n + 1), 0.21)
    v = np.full((n, n + 1, n), -0.17)
    w = np.full((n + 1, n, n), 0.08)
    res = []
    for split in (0, 1):
        cfg = orc.Config(shape=wl.shape, h=wl.h, ndim=3, cp_l=wl.cp_l, cp_g=wl.cp_g, split=split)
        res.append(orc.step(cfg, wl.c, wl.e, u, v, w, None, 1.0, 1.0, 0)[:2])
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


def test_volume_change_is_the_dilatation_term(orc):
    """Periodic, discretely divergence-free: the step's volume change equals its
    dilatation terms (no boundary, no clip); for the Lagrangian-explicit sweeps they add
    up to a visible change, for the Weymouth-Yue split to round-off."""
    wl = W.random_drops_3d(n=16, ndrops=5, seed=74, cfl=0.4, rmin=1.5, rmax=3.5)
    hv = wl.h ** 3
    v0 = math.fsum(wl.c.ravel()) * hv
    change = {}
    for split in (0, 1):
        cfg = orc.Config(shape=wl.shape, h=wl.h, ndim=3, cp_l=wl.cp_l, cp_g=wl.cp_g, split=split)
        c, e, st = orc.step(cfg, wl.c, wl.e, wl.u, wl.v, wl.w, None, wl.dt, 1.0, 0)
        dv = st["vol"] - v0
        assert abs(dv - (st["vol_src"] + st["vol_clip"])) <= 1e-14 * v0
        change[split] = abs(dv) / v0
    assert change[0] <= 1e-14
    assert change[1] > 1e-7
