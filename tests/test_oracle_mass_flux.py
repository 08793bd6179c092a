"""Pins of the oracle's mass-transfer rate from the PLIC reconstruction (section 3.2).

* A planar interface whose reconstruction is exact (shallow planes with centred
  columns): every first and second pure neighbour's distance to the selected plane is
  the exact node-to-plane distance, to machine precision (the paper's first check of
  the distance calculation).
* The same plane with a temperature linear in the distance on each side: every pure
  neighbour's gradient is the phase's slope, so every mixed cell gets the closed form
  m'' = (k_g G_g + k_l G_l) / h_fg.
* A uniform temperature at T_Gamma gives m'' = 0.
* Spheres: the relative distance error over the first and second pure neighbours
  falls with the mesh size (the paper's droplet convergence check, at first to second
  order)."""
import numpy as np
import pytest

import exact
from paper_2001_03477_amd import workloads as W


def _plane_fractions(n_vec, x0, shape, nd=3):
    """Exact fractions of n.(x - x0) <= 0 (liquid side), cell units."""
    nz, ny, nx = shape
    out = np.zeros(shape)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                o = (i, j, 0 if nd == 2 else k)
                a = sum(n_vec[q] * (x0[q] - o[q]) for q in range(3))
                out[k, j, i] = float(exact.volume(n_vec, a))
    return out


def _node_signed_distance(n_vec, x0, shape, nd):
    """n.(x_node - x0) / |n|_2 at every cell centre (cell units; > 0 on the gas side)."""
    nz, ny, nx = shape
    n = np.asarray([float(v) for v in n_vec])
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    if nd == 2:
        z = np.zeros_like(z)
    s = n[0] * (x - float(x0[0])) + n[1] * (y - float(x0[1])) + n[2] * (z - float(x0[2]))
    return s / np.linalg.norm(n)


# Centred columns reproduce a plane exactly when every 3-cell column of the blocks
# brackets it: with transverse slopes s1, s2 (dominant component 1), |s1| + |s2| plus
# the larger of them at most 1.
PLANES = {
    "3d": ((16, 16, 16), 3, ["3/10", "-1/5", 1], ["8", "8", "77/10"]),
    "3d-x": ((14, 14, 14), 3, [1, "1/4", "-1/5"], ["71/10", "7", "7"]),
    "2d": ((1, 24, 24), 2, ["-7/20", 1, 0], ["12", "123/10", "0"]),
}


def _plane_case(key):
    from fractions import Fraction as Fr
    shape, nd, nv, x0 = PLANES[key]
    nv = [Fr(v) for v in nv]
    x0 = [Fr(v) for v in x0]
    return shape, nd, nv, x0


def _interior(shape, nd, margin):
    nz, ny, nx = shape
    m = np.zeros(shape, dtype=bool)
    if nd == 2:
        m[:, margin:ny - margin, margin:nx - margin] = True
    else:
        m[margin:nz - margin, margin:ny - margin, margin:nx - margin] = True
    return m


@pytest.mark.parametrize("key", sorted(PLANES))
def test_plane_distances_are_exact(orc, key):
    shape, nd, nv, x0 = _plane_case(key)
    n = shape[-1]
    h = 1.0 / n
    c = _plane_fractions(nv, x0, shape, nd)
    cfg = orc.Config(shape=shape, h=h, ndim=nd, bc=(1, 1, 1), normal=2)
    T = np.ones(shape)
    _, dist = orc.mass_flux(cfg, c, T, 1.0, 1.0, 1.0)
    s = _node_signed_distance(nv, x0, shape, nd)
    # cells whose 5x5(x5) block and the blocks' 3x3x3 reconstructions stay away from
    # the outflow ghost layers
    sel = _interior(shape, nd, 3) & ~np.isnan(dist)
    assert sel.sum() > 50
    err = np.abs(dist[sel] - np.abs(s[sel]) * h)
    assert err.max() <= 1e-14, err.max()
    # exactly the pure cells within two cells of a mixed cell have a distance
    mixed = (c > 1e-12) & (c < 1 - 1e-12)
    near = np.zeros(shape, dtype=bool)
    r = range(-2, 3)
    for oz in (r if nd == 3 else [0]):
        for oy in r:
            for ox in r:
                near |= np.roll(mixed, (oz, oy, ox), axis=(0, 1, 2))
    inner = _interior(shape, nd, 3)
    assert np.array_equal((~np.isnan(dist))[inner], (near & ~mixed)[inner])


@pytest.mark.parametrize("key", sorted(PLANES))
def test_linear_temperature_gives_the_closed_form_mass_flux(orc, key):
    shape, nd, nv, x0 = _plane_case(key)
    n = shape[-1]
    h = 1.0 / n
    c = _plane_fractions(nv, x0, shape, nd)
    s = _node_signed_distance(nv, x0, shape, nd) * h
    T_g, G_l, G_g = 1.5, 3.0, 7.0
    k_l, k_g, h_fg = 0.6, 0.025, 2.0
    T = np.where(s > 0, T_g + G_g * s, T_g - G_l * s)  # phase-outward slopes
    cfg = orc.Config(shape=shape, h=h, ndim=nd, bc=(1, 1, 1), normal=2, T_gamma=T_g)
    mdot, _ = orc.mass_flux(cfg, c, T, k_l, k_g, h_fg)
    mixed = (c > 1e-12) & (c < 1 - 1e-12)
    sel = _interior(shape, nd, 5) & mixed
    assert sel.sum() > 10
    expect = (k_g * G_g + k_l * G_l) / h_fg
    assert np.max(np.abs(mdot[sel] - expect)) <= 1e-12 * expect
    assert np.all(mdot[~mixed] == 0.0)


def test_saturated_temperature_gives_zero(orc):
    wl = W.random_drops_3d(n=20, ndrops=4, seed=91, rmin=2.0, rmax=4.0)
    cfg = orc.Config(shape=wl.shape, h=wl.h, ndim=3, bc=(0, 0, 0), T_gamma=0.8)
    mdot, dist = orc.mass_flux(cfg, wl.c, np.full(wl.shape, 0.8), 0.6, 0.02, 10.0)
    assert np.all(mdot == 0.0)
    # a node of the 5x5x5 block is at most 2.5 sqrt(3) from the mixed cell's origin, and
    # the plane at most sqrt(3) from it
    assert np.nanmin(dist) > 0.0 and np.nanmax(dist) <= 3.5 * np.sqrt(3.0) * wl.h


def test_sphere_distance_error_converges(orc):
    """Spheres of radius 0.25 + delta (|delta| <= h) at (0.5, 0.5, 0.5) + delta:
    relative error |d^h - d| / R0 over the first and second pure neighbours, max and L2,
    averaged over a few seeded droplets per mesh."""
    rng = np.random.default_rng(17)
    l2s, maxs = [], []
    for n in (16, 32, 64):
        h = 1.0 / n
        shape = (n, n, n)
        el2, emax = [], []
        for _ in range(3):
            d = rng.uniform(-h, h, 4)
            R0 = 0.25 + d[0]
            x0 = 0.5 + d[1:]
            c = W.sphere_fraction(shape, h, [x0], [R0], sub=16)
            cfg = orc.Config(shape=shape, h=h, ndim=3, bc=(1, 1, 1), normal=1)
            _, dist = orc.mass_flux(cfg, c, np.ones(shape), 1.0, 1.0, 1.0)
            z, y, x = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
            r = np.sqrt((x * h - x0[0]) ** 2 + (y * h - x0[1]) ** 2 + (z * h - x0[2]) ** 2)
            ok = ~np.isnan(dist)
            e = np.abs(dist[ok] - np.abs(r[ok] - R0)) / R0
            el2.append(np.sqrt(np.mean(e ** 2)))
            emax.append(e.max())
        l2s.append(np.mean(el2))
        maxs.append(np.mean(emax))
    rates = np.log2(np.asarray(l2s[:-1]) / np.asarray(l2s[1:]))
    assert np.all(rates > 0.9), (l2s, rates)
    assert maxs[2] < maxs[0], maxs
