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


def sphere_fraction(shape, h, centres, radii, inside_liquid=True, sub=8, nd=3, disjoint=False):
    """Volume fraction of the union of spheres (discs when nd == 2) sampled with
    sub^nd points per cell, only in cells whose centre lies within the half cell
    diagonal of a sphere surface; other cells are 0 or 1. With inside_liquid=False
    the spheres are gas (bubbles) in a liquid. disjoint=True promises that the
    spheres' surfaces are more than a cell diagonal apart, so that every sampled cell
    is sampled against its own sphere only (much faster for many spheres)."""
    if disjoint:
        return _disjoint_sphere_fraction(shape, h, centres, radii, inside_liquid, sub, nd)
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


def line_fraction(xl, yl, h, x_at_y0, slope):
    """Exact area fraction of the square [xl, xl+h] x [yl, yl+h] left of the line
    x = x_at_y0 + slope * y: the mean over y of clamp(x_line(y) - xl, 0, h) / h. The
    integrand is piecewise linear with kinks where it reaches 0 or h, so the trapezoid
    rule is exact between the kinks."""
    def g(y):
        return min(max(x_at_y0 + slope * y - xl, 0.0), h)

    knots = {yl, yl + h}
    if slope != 0.0:
        for level in (0.0, h):
            yk = (xl + level - x_at_y0) / slope
            if yl < yk < yl + h:
                knots.add(yk)
    ks = sorted(knots)
    area = sum(0.5 * (g(a) + g(b)) * (b - a) for a, b in zip(ks[:-1], ks[1:]))
    return min(max(area / (h * h), 0.0), 1.0)  # rounding of the sum may step past 0 or 1


def line_fraction_field(shape, h, x_at_y0, slope):
    """Fractions of a 2D grid (shape (1, ny, nx)) of the region left of the line
    x = x_at_y0 + slope * y."""
    _, ny, nx = shape
    out = np.zeros(shape)
    for j in range(ny):
        for i in range(nx):
            out[0, j, i] = line_fraction(i * h, j * h, h, x_at_y0, slope)
    return out


def _disjoint_sphere_fraction(shape, h, centres, radii, inside_liquid, sub, nd):
    import torch  # multithreaded sampling on the host
    nz, ny, nx = shape
    frac = np.zeros(shape)
    half_diag = 0.5 * h * math.sqrt(nd) * 1.0000001
    cells, owner = [], []
    for j, (cen, r) in enumerate(zip(np.atleast_2d(centres), np.atleast_1d(radii))):
        lo = np.floor((cen - r) / h - 1).astype(int)
        hi = np.ceil((cen + r) / h + 1).astype(int)
        xs = np.arange(max(lo[0], 0), min(hi[0], nx))
        ys = np.arange(max(lo[1], 0), min(hi[1], ny))
        zs = np.arange(max(lo[2], 0), min(hi[2], nz)) if nd == 3 else np.array([0])
        if len(xs) == 0 or len(ys) == 0 or len(zs) == 0:
            continue
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        dz = ((Z + 0.5) * h - cen[2]) if nd == 3 else 0.0
        d = np.sqrt(((X + 0.5) * h - cen[0]) ** 2 + ((Y + 0.5) * h - cen[1]) ** 2 + dz ** 2) - r
        ins = d <= -half_diag
        frac[Z[ins], Y[ins], X[ins]] = 1.0
        near = np.abs(d) < half_diag
        cells.append(np.stack([Z[near], Y[near], X[near]], axis=1))
        owner.append(np.full(int(near.sum()), j))
    if cells:
        cells = np.concatenate(cells)
        owner = np.concatenate(owner)
        cen = np.atleast_2d(centres)[owner]
        rad = np.atleast_1d(radii)[owner]
        s = torch.from_numpy((np.arange(sub) + 0.5) / sub * h)
        for b in range(0, len(cells), 65536):
            blk = torch.from_numpy(cells[b:b + 65536])
            cb = torch.from_numpy(cen[b:b + 65536])
            rb = torch.from_numpy(rad[b:b + 65536])
            # offsets of the sample points from the sphere centre, per axis
            dx = (blk[:, 2:3] * h + s[None, :]) - cb[:, 0:1]
            dy = (blk[:, 1:2] * h + s[None, :]) - cb[:, 1:2]
            if nd == 3:
                dz = (blk[:, 0:1] * h + s[None, :]) - cb[:, 2:3]
                d2 = (dz * dz)[:, :, None, None] + (dy * dy)[:, None, :, None] + (dx * dx)[:, None, None, :]
            else:
                d2 = (dy * dy)[:, :, None] + (dx * dx)[:, None, :]
            hit = (d2 <= (rb * rb).reshape([-1] + [1] * (d2.dim() - 1))).to(torch.float64)
            f = hit.reshape(hit.shape[0], -1).mean(dim=1).numpy()
            cc = cells[b:b + 65536]
            frac[cc[:, 0], cc[:, 1], cc[:, 2]] = f
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


def fourier_modes(rng, nmodes=8, kmax=4, nd=3):
    """Integer wave vectors k_j in [-kmax, kmax]^3 \\ {0}, amplitudes a_j ~ N(0, I) and
    phases phi_j ~ U[0, 2 pi) of A = sum_j a_j sin(2 pi k_j.x + phi_j) (drawn in the
    same order as fourier_potential)."""
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
    return ks, amps, phis


def fourier_mac_velocity(ks, amps, phis, shape, h, lengths=None):
    """3D periodic MAC velocities of curl A for A = sum_j a_j sin(2 pi k_j.x + phi_j),
    like mac_velocity(fourier_potential(...)) but with the edge integrals evaluated
    separably: the integral of sin(2 pi k.x + phi) along an edge of length h in
    direction d is h sinc(k_d h) sin(2 pi k.x_mid + phi) with x_mid the edge midpoint,
    and sin(a + b + c) over the grid is built from 1D factors, so a 512^3 field takes
    seconds. Node coordinates wrap (the last node is at 0), so the two boundary faces
    of every axis are bitwise equal. With lengths = (Lx, Ly, Lz) the box is periodic
    with those lengths (cells of side h, n_a h = L_a) and the wave vectors are k_a / L_a."""
    nz, ny, nx = shape
    tp = 2.0 * math.pi
    if lengths is None:
        lengths = (1.0, 1.0, 1.0)
    ks = [np.array([k[0] / lengths[0], k[1] / lengths[1], k[2] / lengths[2]]) for k in ks]

    def coords(n, mid):
        idx = np.arange(n if mid else n + 1)
        if mid:
            return (idx + 0.5) * h
        return (idx % n) * h

    import torch  # multithreaded elementwise products on the host

    def edge_integral(comp, axis):
        # the grid of edges along `axis`: midpoints along it, nodes across
        zc = coords(nz, axis == 2)
        yc = coords(ny, axis == 1)
        xc = coords(nx, axis == 0)
        out = torch.zeros((len(zc), len(yc), len(xc)), dtype=torch.float64)
        for k, a, ph in zip(ks, amps, phis):
            if a[comp] == 0.0:
                continue
            kd = k[axis]
            fac = h if kd == 0.0 else math.sin(math.pi * kd * h) / (math.pi * kd)
            ax = tp * k[0] * xc
            bc = (tp * k[1] * yc)[None, :] + (tp * k[2] * zc + ph)[:, None]
            sbc = torch.from_numpy((a[comp] * fac) * np.sin(bc))[:, :, None]
            cbc = torch.from_numpy((a[comp] * fac) * np.cos(bc))[:, :, None]
            ca = torch.from_numpy(np.cos(ax))[None, None, :]
            sa = torch.from_numpy(np.sin(ax))[None, None, :]
            out.addcmul_(sbc, ca)
            out.addcmul_(cbc, sa)
        return out

    Ex = edge_integral(0, 0)  # [nz+1][ny+1][nx]
    Ey = edge_integral(1, 1)  # [nz+1][ny][nx+1]
    Ez = edge_integral(2, 2)  # [nz][ny+1][nx+1]
    h2 = h * h
    u = ((Ey[:-1, :, :] + Ez[:, 1:, :]) - (Ey[1:, :, :] + Ez[:, :-1, :])) / h2
    v = ((Ez[:, :, :-1] + Ex[1:, :, :]) - (Ez[:, :, 1:] + Ex[:-1, :, :])) / h2
    w = ((Ex[:, :-1, :] + Ey[:, :, 1:]) - (Ex[:, 1:, :] + Ey[:, :, :-1])) / h2
    return (np.ascontiguousarray(u.numpy()), np.ascontiguousarray(v.numpy()),
            np.ascontiguousarray(w.numpy()))


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


def periodic_drops(rng, n, ndrops, rmin, rmax, gap, max_tries=1000000):
    """Rejection-placed spheres in the periodic unit cube: radii uniform in
    [rmin, rmax] cells, surfaces at least `gap` cells apart in the minimum-image
    distance. Returns (centres [k, 3], radii [k]) in domain units."""
    h = 1.0 / n
    cen = np.zeros((ndrops, 3))
    rad = np.zeros(ndrops)
    k = 0
    tries = 0
    r = rng.uniform(rmin, rmax) * h  # each radius is drawn once, positions are retried
    while k < ndrops and tries < max_tries:
        tries += 1
        p = rng.uniform(0.0, 1.0, size=3)
        if k:
            d = p[None, :] - cen[:k]
            d -= np.round(d)
            dist = np.sqrt(np.sum(d * d, axis=1))
            if np.any(dist < r + rad[:k] + gap * h):
                continue
        cen[k] = p
        rad[k] = r
        k += 1
        r = rng.uniform(rmin, rmax) * h
    return cen[:k], rad[:k]


def periodic_images(centres, radii):
    """The spheres plus their periodic images that reach into the unit cube."""
    out_c, out_r = [], []
    for p, r in zip(centres, radii):
        shifts = [[0.0] if (p[a] - r > 0.0 and p[a] + r < 1.0) else [-1.0, 0.0, 1.0] for a in range(3)]
        for sx in shifts[0]:
            for sy in shifts[1]:
                for sz in shifts[2]:
                    q = p + np.array([sx, sy, sz])
                    if np.all(q + r > 0.0) and np.all(q - r < 1.0):
                        out_c.append(q)
                        out_r.append(r)
    return np.array(out_c), np.array(out_r)


def droplets_3d(n=512, ndrops=2000, seed=4, cfl=0.3, rmin=4.0, rmax=16.0, gap=2.0, nmodes=8,
                kmax=4, cp=(4.039e6, 1.248e3)) -> Workload:
    """3D n^3 periodic box with `ndrops` seeded droplets (radii uniform in [rmin, rmax]
    cells, surfaces at least `gap` cells apart in the periodic distance), a random
    divergence-free Fourier velocity (nmodes modes with integer wave vectors in
    [-kmax, kmax]^3) scaled so that the largest face velocity is 1, dt = 0.3 h, random
    per-phase temperatures, water-like volumetric heat capacities, m'' = 0."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    shape = (n, n, n)
    centres, radii = periodic_drops(rng, n, ndrops, rmin, rmax, gap)
    ic, ir = periodic_images(centres, radii)
    c = sphere_fraction(shape, h, ic, ir, sub=8, nd=3, disjoint=True)
    cp_l, cp_g = cp
    T_l = rng.uniform(0.0, 1.0, size=shape)
    T_g = rng.uniform(0.0, 1.0, size=shape)
    e = energy_from_phase_temperatures(c, T_l, T_g, cp_l, cp_g)
    del T_l, T_g
    ks, amps, phis = fourier_modes(rng, nmodes, kmax, 3)
    u, v, w = fourier_mac_velocity(ks, amps, phis, shape, h)
    s = 1.0 / max_abs_face(u, v, w)
    u *= s
    v *= s
    w *= s
    dt = cfl * h
    return Workload(f"droplets3d_{n}", shape, h, 3, (0, 0, 0), cp_l, cp_g, 1.0, 1.0, c, e, u, v, w,
                    None, dt, 10)


def rect_solid_angle(x0, y1, y2, z1, z2):
    """Signed solid angle of the rectangle {x = x0, y in [y1, y2], z in [z1, z2]} seen
    from the origin, positive when x0 > 0 (the flux of the unit point source
    r / (4 pi |r|^3) through it in +x, times 4 pi)."""
    def F(y, z):
        return np.arctan(y * z / (x0 * np.sqrt(x0 * x0 + y * y + z * z)))
    return F(y2, z2) - F(y1, z2) - F(y2, z1) + F(y1, z1)


def bubble_3d(n=256, R=0.1, u0=0.05, smooth=0.8, cfl=0.3, rho_l=2.5, cp_l=6.25, cp_g=0.25,
              k_l=0.07, h_fg=100.0, T_sat=1.0, T_inf=3.0, delta_T=0.05) -> Workload:
    """3D n^3 expanding vapour bubble: a vapour sphere of radius R at the box centre in
    liquid, outflow on all axes. Outside the ball r < smooth R the velocity is the
    point source u = u0 R^2 / r^2 r^, whose face fluxes are exact (u0 R^2 times the
    face's solid angle), so every cell outside the ball is discretely divergence-free;
    inside the ball (pure vapour) u = u0 R^2 r / R_s^3 at the face centres, a source
    the step reports. T = T_sat inside the bubble and a linear ramp to T_inf over
    delta_T outside; m'' = k_l (T_inf - T_sat) / (delta_T h_fg) in every cell (applied
    in mixed cells); properties of the paper's bubble case. CFL 0.3 on the largest
    face velocity."""
    h = 1.0 / n
    shape = (n, n, n)
    ctr = 0.5
    c = sphere_fraction(shape, h, [[ctr, ctr, ctr]], [R], inside_liquid=False, sub=8, nd=3)
    # temperature at the cell centres
    xc = (np.arange(n) + 0.5) * h - ctr
    r = np.sqrt(xc[:, None, None] ** 2 + xc[None, :, None] ** 2 + xc[None, None, :] ** 2)
    T = np.clip(T_sat + (T_inf - T_sat) * (r - R) / delta_T, T_sat, T_inf)
    del r
    e = energy_from_phase_temperatures(c, T, T, cp_l, cp_g)
    # face velocities
    Rs = smooth * R
    q = u0 * R * R
    xf = np.arange(n + 1) * h - ctr     # face positions
    xlo = np.arange(n) * h - ctr        # cell lower corners
    xhi = xlo + h
    xm = xlo + 0.5 * h                  # cell centres

    def axis_faces(axis):
        # face grid [nz][ny][nx] with the sweep axis extended by one
        a = xf[:, None, None]           # face coordinate along axis
        b1, b2, bm = xlo[None, :, None], xhi[None, :, None], xm[None, :, None]
        c1, c2, cm = xlo[None, None, :], xhi[None, None, :], xm[None, None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            om = rect_solid_angle(a, b1, b2, c1, c2)
        flux = q * om / (h * h)
        rf = np.sqrt(a * a + bm * bm + cm * cm)
        lin = q * a / Rs ** 3
        vel = np.where(rf >= Rs, flux, lin)
        vel = np.where(a == 0.0, 0.0, vel)
        # vel is indexed [axis][t1][t2]; move the axis to its MAC position
        if axis == 0:      # [x][y][z] -> [z][y][x]
            return np.ascontiguousarray(np.transpose(vel, (2, 1, 0)))
        if axis == 1:      # [y][x][z] -> [z][y][x]
            return np.ascontiguousarray(np.transpose(vel, (2, 0, 1)))
        return np.ascontiguousarray(vel)  # [z][y][x]

    u = axis_faces(0)
    v = axis_faces(1)
    w = axis_faces(2)
    umax = max_abs_face(u, v, w)
    dt = cfl * h / umax
    mdot = np.full(shape, k_l * (T_inf - T_sat) / (delta_T * h_fg))
    return Workload(f"bubble3d_{n}", shape, h, 3, (1, 1, 1), cp_l, cp_g, rho_l, T_sat, c, e, u, v, w,
                    mdot, dt, 10)


def wide_mixed_3d(nx=1100, ny=16, nz=4, seed=53) -> Workload:
    """A box whose rows are longer than one 512-cell x range of the x sweep (three ranges
    at nx = 1100, the last one ragged), every cell mixed (c uniform in [0.05, 0.95], e
    from per-phase temperatures 0.7 and 0.3 at water-like heat capacities), in a periodic
    divergence-free Fourier velocity (6 modes) at CFL 0.3."""
    rng = np.random.default_rng(seed)
    shape, h = (nz, ny, nx), 1.0 / nx
    c = rng.uniform(0.05, 0.95, size=shape)
    cp_l, cp_g = 4039.0, 1.248
    e = energy_from_phase_temperatures(c, 0.7, 0.3, cp_l, cp_g)
    ks, amps, phis = fourier_modes(rng, 6, 3, 3)
    u, v, w = fourier_mac_velocity(ks, amps, phis, shape, h, lengths=(nx * h, ny * h, nz * h))
    dt = 0.3 * h / max_abs_face(u, v, w)
    return Workload(f"wide_mixed_{nx}x{ny}x{nz}", shape, h, 3, (0, 0, 0), cp_l, cp_g, 1.0, 1.0, c, e, u, v, w,
                    None, dt, 2)


def batch_domains(nd=64, seed=5, smin=32, smax=160, cfl=0.3, cp=(1000.0, 1.0)):
    """nd independent periodic 3D domains with sides uniform in [smin, smax] cells per
    axis (cubic cells of side 1/nx), each holding one drop (liquid sphere) or bubble
    (gas sphere), 50/50, of radius uniform in [0.15, 0.3] times the shortest side, at a
    random position, in its own random periodic Fourier velocity (4 to 8 modes) scaled
    to CFL 0.3 with its own dt; random per-phase temperatures; rho c_p 1000 : 1,
    m'' = 0."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nd):
        nx, ny, nz = (int(v) for v in rng.integers(smin, smax + 1, size=3))
        h = 1.0 / nx
        shape = (nz, ny, nx)
        L = (nx * h, ny * h, nz * h)
        r = rng.uniform(0.15, 0.3) * min(nx, ny, nz) * h
        centre = np.array([rng.uniform(0, L[0]), rng.uniform(0, L[1]), rng.uniform(0, L[2])])
        drop = bool(rng.integers(0, 2))
        # the sphere and its periodic images that reach into the box
        cs, rs = [], []
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                for sz in (-1, 0, 1):
                    q = centre + np.array([sx * L[0], sy * L[1], sz * L[2]])
                    if np.all(q + r > 0) and np.all(q - r < np.array(L)):
                        cs.append(q)
                        rs.append(r)
        c = sphere_fraction(shape, h, np.array(cs), np.array(rs), inside_liquid=drop, sub=8, nd=3,
                            disjoint=True)
        cp_l, cp_g = cp
        T_l = rng.uniform(0, 1, size=shape)
        T_g = rng.uniform(0, 1, size=shape)
        e = energy_from_phase_temperatures(c, T_l, T_g, cp_l, cp_g)
        ks, amps, phis = fourier_modes(rng, int(rng.integers(4, 9)), 4, 3)
        u, v, w = fourier_mac_velocity(ks, amps, phis, shape, h, lengths=L)
        umax = max_abs_face(u, v, w)
        dt = cfl * h / umax
        out.append(Workload(f"batch{i}_{nx}x{ny}x{nz}", shape, h, 3, (0, 0, 0), cp_l, cp_g, 1.0, 1.0,
                            c, e, u, v, w, None, dt, 10))
    return out
