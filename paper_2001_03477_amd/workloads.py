"""Seeded synthetic inputs for the advection step: volume fractions of spheres
and circles, per-phase temperatures, and MAC face velocities that are discretely
divergence-free to round-off.

This module holds none of the method's arithmetic (no plane reconstruction, no
fluxes): it only draws inputs. Face velocities are face-averaged velocities
u_f = (1/h^2) * circulation of a vector potential A around the face (Stokes), with
each edge integral of A evaluated once in closed form and shared by the four
faces that meet at that edge, so every cell's net outflow cancels to round-off.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

# --------------------------------------------------------------------------- shapes


def sphere_fraction(shape, h, centres, radii, inside_liquid=True, sub=8, nd=3):
    """Volume fraction of the union of spheres (discs when nd == 2) sampled with
    sub^nd points per cell, only in cells whose centre lies within the half cell
    diagonal of a sphere surface; other cells are 0 or 1. With inside_liquid=False
    the spheres are gas (bubbles) in a liquid."""
    nz, ny, nx = shape
    centres = np.atleast_2d(np.asarray(centres, dtype=float))
    radii = np.atleast_1d(np.asarray(radii, dtype=float))
    inside = np.zeros(shape, dtype=bool)
    frac = np.zeros(shape)
    near = np.zeros(shape, dtype=bool)
    half_diag = 0.5 * h * math.sqrt(nd) * 1.0000001
    zc = (np.arange(nz) + 0.5) * h if nd == 3 else np.array([0.0])
    yc = (np.arange(ny) + 0.5) * h
    xc = (np.arange(nx) + 0.5) * h
    for cen, r in zip(centres, radii):
        # bounding box of the cells that can be touched
        lo = np.floor((cen - r) / h - 1).astype(int)
        hi = np.ceil((cen + r) / h + 1).astype(int)
        xs = np.arange(max(lo[0], 0), min(hi[0], nx))
        ys = np.arange(max(lo[1], 0), min(hi[1], ny))
        zs = np.arange(max(lo[2], 0), min(hi[2], nz)) if nd == 3 else np.array([0])
        if len(xs) == 0 or len(ys) == 0 or len(zs) == 0:
            continue
        Z, Y, X = np.meshgrid(zc[zs], yc[ys], xc[xs], indexing="ij")
        dz = (Z - cen[2]) if nd == 3 else 0.0
        d = np.sqrt((X - cen[0]) ** 2 + (Y - cen[1]) ** 2 + dz ** 2) - r
        sl = np.ix_(zs, ys, xs)
        inside[sl] |= d <= -half_diag
        near[sl] |= np.abs(d) < half_diag
    # sample the cells near a surface against all spheres
    idx = np.argwhere(near & ~inside)
    if len(idx):
        s = (np.arange(sub) + 0.5) / sub
        if nd == 3:
            SZ, SY, SX = np.meshgrid(s, s, s, indexing="ij")
        else:
            SY, SX = np.meshgrid(s, s, indexing="ij")
            SZ = np.full_like(SX, 0.5)
        SX, SY, SZ = SX.ravel(), SY.ravel(), SZ.ravel()
        chunk = 4096
        for b in range(0, len(idx), chunk):
            blk = idx[b:b + chunk]
            px = (blk[:, 2:3] + SX[None, :]) * h
            py = (blk[:, 1:2] + SY[None, :]) * h
            pz = (blk[:, 0:1] + SZ[None, :]) * h
            hit = np.zeros(px.shape, dtype=bool)
            for cen, r in zip(centres, radii):
                # cheap reject by distance of the cell centre
                cx = (blk[:, 2] + 0.5) * h - cen[0]
                cy = (blk[:, 1] + 0.5) * h - cen[1]
                cz = ((blk[:, 0] + 0.5) * h - cen[2]) if nd == 3 else 0.0 * cx
                close = np.sqrt(cx * cx + cy * cy + cz * cz) < r + half_diag
                if not np.any(close):
                    continue
                rows = np.nonzero(close)[0]
                dzz = (pz[rows] - cen[2]) if nd == 3 else 0.0
                hit[rows] |= ((px[rows] - cen[0]) ** 2 + (py[rows] - cen[1]) ** 2 +
                              dzz ** 2) <= r * r
            frac[blk[:, 0], blk[:, 1], blk[:, 2]] = hit.mean(axis=1)
    frac[inside] = 1.0
    return frac if inside_liquid else 1.0 - frac


# --------------------------------------------------------------------------- velocities


@dataclass
class EdgePotential:
    """A vector potential given by its closed-form line integrals along grid edges:
    ex(x0, x1, y, z) = int_{x0}^{x1} A_x dx, ey(x, y0, y1, z), ez(x, y, z0, z1)
    (numpy-broadcastable). Missing components are zero."""
    ex: Optional[Callable] = None
    ey: Optional[Callable] = None
    ez: Optional[Callable] = None


def mac_velocity(pot: EdgePotential, shape, h, nd=3, periodic=True):
    """Face-averaged MAC velocities (u [nz][ny][nx+1], v [nz][ny+1][nx],
    w [nz+1][ny][nx]) of curl A. In 2D (nd == 2) only A_z matters and w is None.
    With periodic=True the last node of each axis is evaluated at coordinate 0, so the
    two boundary faces of a periodic axis carry bitwise identical velocities."""
    nz, ny, nx = shape

    def nodes(n):
        idx = np.arange(n + 1)
        return (idx % n if periodic else idx) * h

    xn, yn, zn = nodes(nx), nodes(ny), nodes(nz)
    if nd == 2:
        # 2D: u = d(psi)/dy, v = -d(psi)/dx with psi = A_z; the "edge" integrals of
        # A_z along z over a unit depth are psi values at the nodes
        Y, X = np.meshgrid(yn, xn, indexing="ij")
        psi = pot.ez(X, Y, 0.0, 1.0) if pot.ez is not None else np.zeros_like(X)
        u = (psi[1:, :] - psi[:-1, :]) / h        # [ny][nx+1]
        v = -(psi[:, 1:] - psi[:, :-1]) / h       # [ny+1][nx]
        return u[None, :, :].copy(), v[None, :, :].copy(), None

    def grid(a, b, c):
        return np.meshgrid(a, b, c, indexing="ij")  # (z, y, x) order of arguments

    # E_x on x-edges: [nz+1][ny+1][nx]
    Z, Y, X0 = grid(zn, yn, xn[:-1])
    Ex = pot.ex(X0, X0 + h, Y, Z) if pot.ex is not None else np.zeros(X0.shape)
    # E_y on y-edges: [nz+1][ny][nx+1]
    Z, Y0, X = grid(zn, yn[:-1], xn)
    Ey = pot.ey(X, Y0, Y0 + h, Z) if pot.ey is not None else np.zeros(X.shape)
    # E_z on z-edges: [nz][ny+1][nx+1]
    Z0, Y, X = grid(zn[:-1], yn, xn)
    Ez = pot.ez(X, Y, Z0, Z0 + h) if pot.ez is not None else np.zeros(X.shape)
    h2 = h * h
    # x-faces (normal +x): circulation y -> z
    u = ((Ey[:-1, :, :] + Ez[:, 1:, :]) - (Ey[1:, :, :] + Ez[:, :-1, :])) / h2
    # y-faces (normal +y): circulation z -> x
    v = ((Ez[:, :, :-1] + Ex[1:, :, :]) - (Ez[:, :, 1:] + Ex[:-1, :, :])) / h2
    # z-faces (normal +z): circulation x -> y
    w = ((Ex[:, :-1, :] + Ey[:, :, 1:]) - (Ex[:, 1:, :] + Ey[:, :, :-1])) / h2
    return np.ascontiguousarray(u), np.ascontiguousarray(v), np.ascontiguousarray(w)


def leveque_potential() -> EdgePotential:
    """LeVeque's 3D deformation field u = 2 sin^2(pi x) sin(2 pi y) sin(2 pi z),
    v = -sin(2 pi x) sin^2(pi y) sin(2 pi z), w = -sin(2 pi x) sin(2 pi y) sin^2(pi z)
    as the curl of A = (0, -sin^2(pi x) sin(2 pi y) sin^2(pi z) / pi,
    sin^2(pi x) sin^2(pi y) sin(2 pi z) / pi)."""
    pi = math.pi
    s2 = lambda t: np.sin(pi * t) ** 2  # noqa: E731

    def ey(x, y0, y1, z):
        return s2(x) * s2(z) * (np.cos(2 * pi * y1) - np.cos(2 * pi * y0)) / (2 * pi * pi)

    def ez(x, y, z0, z1):
        return -s2(x) * s2(y) * (np.cos(2 * pi * z1) - np.cos(2 * pi * z0)) / (2 * pi * pi)

    return EdgePotential(None, ey, ez)


def fourier_potential(rng, nmodes=8, kmax=4, nd=3) -> EdgePotential:
    """A = sum_j a_j sin(2 pi k_j.x + phi_j) with integer k_j in [-kmax, kmax]^3 \\ {0},
    a_j ~ N(0, I), phi_j ~ U[0, 2 pi): periodic on the unit cube. In 2D only A_z (a
    stream function) with k_z = 0."""
    ks, amps, phis = [], [], []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if nd == 2:
            k[2] = 0
        if not np.any(k):
            continue
        ks.append(k.astype(float))
        a = rng.normal(size=3)
        if nd == 2:
            a[:2] = 0.0
        amps.append(a)
        phis.append(rng.uniform(0, 2 * math.pi))
    tp = 2 * math.pi

    def line(comp, axis):
        def f(*args):
            # args: the coordinates with the integration axis given as (t0, t1)
            if axis == 0:
                x0, x1, y, z = args
            elif axis == 1:
                x, y0, y1, z = args
            else:
                x, y, z0, z1 = args
            tot = 0.0
            for k, a, ph in zip(ks, amps, phis):
                if a[comp] == 0.0:
                    continue
                if axis == 0:
                    base = tp * (k[1] * y + k[2] * z) + ph
                    lo, hi, kk = x0, x1, k[0]
                elif axis == 1:
                    base = tp * (k[0] * x + k[2] * z) + ph
                    lo, hi, kk = y0, y1, k[1]
                else:
                    base = tp * (k[0] * x + k[1] * y) + ph
                    lo, hi, kk = z0, z1, k[2]
                if kk != 0.0:
                    val = (np.cos(tp * kk * lo + base) - np.cos(tp * kk * hi + base)) / (tp * kk)
                else:
                    val = (hi - lo) * np.sin(base)
                tot = tot + a[comp] * val
            return tot
        return f

    return EdgePotential(line(0, 0), line(1, 1), line(2, 2))


def max_abs_face(u, v, w=None) -> float:
    m = max(float(np.max(np.abs(u))), float(np.max(np.abs(v))))
    if w is not None:
        m = max(m, float(np.max(np.abs(w))))
    return m


# --------------------------------------------------------------------------- configurations


@dataclass
class Workload:
    name: str
    shape: tuple           # (nz, ny, nx)
    h: float
    ndim: int
    bc: tuple              # per axis x, y, z: 0 periodic, 1 outflow
    cp_l: float
    cp_g: float
    rho_l: float
    T_gamma: float
    c: np.ndarray
    e: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: Optional[np.ndarray]
    mdot: Optional[np.ndarray]
    dt: float
    steps: int
    normal: int = 1
    u_scale: Callable = field(default=lambda n: 1.0)

    @property
    def ncells(self) -> int:
        return int(np.prod(self.shape))


def energy_from_phase_temperatures(c, T_l, T_g, cp_l, cp_g):
    """e = C_p T for a cell holding liquid at T_l and gas at T_g:
    e = c C_pl T_l + (1 - c) C_pg T_g."""
    return c * cp_l * T_l + (1.0 - c) * cp_g * T_g


def circle_2d(n=64, seed=0) -> Workload:
    """2D 64x64 unit box: circle R = 0.2 at (0.5, 0.5), 16x16 sub-cell sampling,
    uniform velocity (1, 0.5), CFL 0.25 on |u| = 1, 100 steps; T = 1 in the liquid and
    0 in the gas plus 0.1 x; rho c_p 4.2e6 (liquid) and 1.2e3 (gas); m'' = 0.01."""
    h = 1.0 / n
    shape = (1, n, n)
    c = sphere_fraction(shape, h, [[0.5, 0.5, 0.0]], [0.2], sub=16, nd=2)
    x = (np.arange(n) + 0.5) * h
    X = np.broadcast_to(x[None, None, :], shape)
    cp_l, cp_g = 4.2e6, 1.2e3
    e = energy_from_phase_temperatures(c, 1.0 + 0.1 * X, 0.1 * X, cp_l, cp_g)
    u = np.full((1, n, n + 1), 1.0)
    v = np.full((1, n + 1, n), 0.5)
    dt = 0.25 * h / 1.0
    mdot = np.full(shape, 0.01)
    return Workload("circle2d_64", shape, h, 2, (0, 0, 0), cp_l, cp_g, 1.0, 1.0, c, e, u, v,
                    None, mdot, dt, 100)


def leveque_3d(n=128, seed=1, period=3.0, cfl=0.3) -> Workload:
    """3D n^3 LeVeque deformation: sphere R = 0.15 at (0.35, 0.35, 0.35), period T = 3,
    CFL 0.3 on the largest face velocity; per-phase temperatures uniform in [0, 1]
    (seeded); rho c_p 1000 : 1; m'' = 0 (no phase change)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    shape = (n, n, n)
    c = sphere_fraction(shape, h, [[0.35, 0.35, 0.35]], [0.15], sub=8, nd=3)
    cp_l, cp_g = 1000.0, 1.0
    T_l = rng.uniform(0.0, 1.0, size=shape)
    T_g = rng.uniform(0.0, 1.0, size=shape)
    e = energy_from_phase_temperatures(c, T_l, T_g, cp_l, cp_g)
    u, v, w = mac_velocity(leveque_potential(), shape, h, periodic=False)
    umax = max_abs_face(u, v, w)
    dt = cfl * h / umax
    steps = int(round(period / dt))

    def u_scale(step):
        return math.cos(math.pi * (step + 0.5) * dt / period)

    return Workload(f"leveque3d_{n}", shape, h, 3, (1, 1, 1), cp_l, cp_g, 1.0, 1.0, c, e, u, v,
                    w, None, dt, steps, u_scale=u_scale)


def random_drops_3d(n=32, ndrops=6, seed=3, cfl=0.3, rmin=2.0, rmax=5.0, cp=(4039.0, 1.248),
                    nmodes=8, mdot=None, nd=3) -> Workload:
    """Periodic box with seeded non-overlapping droplets (radii in cells in
    [rmin, rmax]) in a random periodic divergence-free Fourier velocity scaled to the
    given CFL; per-phase temperatures uniform in [0, 1]. Used by the tests at small n."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    shape = (n, n, n) if nd == 3 else (1, n, n)
    centres, radii = [], []
    tries = 0
    while len(centres) < ndrops and tries < 10000:
        tries += 1
        r = rng.uniform(rmin, rmax) * h
        p = rng.uniform(0, 1, size=3)
        if nd == 2:
            p[2] = 0.0
        # keep the drops away from the box faces so that no drop wraps around
        if np.any(p[:nd] - r < 2 * h) or np.any(p[:nd] + r > 1 - 2 * h):
            continue
        ok = all(np.linalg.norm(p - q) > r + s + 2 * h for q, s in zip(centres, radii))
        if ok:
            centres.append(p)
            radii.append(r)
    c = sphere_fraction(shape, h, centres, radii, sub=8, nd=nd)
    cp_l, cp_g = cp
    T_l = rng.uniform(0, 1, size=shape)
    T_g = rng.uniform(0, 1, size=shape)
    e = energy_from_phase_temperatures(c, T_l, T_g, cp_l, cp_g)
    u, v, w = mac_velocity(fourier_potential(rng, nmodes=nmodes, nd=nd), shape, h, nd=nd)
    umax = max_abs_face(u, v, w)
    dt = cfl * h / umax
    md = None if mdot is None else np.full(shape, float(mdot))
    return Workload(f"drops{nd}d_{n}", shape, h, nd, (0, 0, 0), cp_l, cp_g, 1.0, 1.0, c, e, u, v,
                    w, md, dt, 10)
