"""PCVOF ORACLE -- test infrastructure, not part of the product.

Liquid-velocity extension of section 3.3.1 (eqs. press_inv and the velocity
correction that follows it), written plainly in numpy with a sparse direct solve
(scipy). Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may load it. It shares no code with the HIP library; the plane geometry comes from
the C oracle (or_normal, or_alpha, or_area).

The step, in the paper's order:
1. A sub-domain around the interface: the mixed cells and the gas cells that are
   first and second neighbours of the interface. Faces between a sub-domain cell and
   a liquid cell are no-slip walls (no correction flux); the faces between the second
   and the third gas neighbours are free-flow faces with a fixed pressure.
2. On it, the Poisson problem div[(dt / rho) grad p~] = m'' (1/rho_g - 1/rho_l) delta_Gamma
   (eq. press_inv), with delta_Gamma = A_Gamma / V the interface area per cell volume.
3. The correction u~ = -(dt / rho) grad p~ on the faces of the sub-domain (zero
   elsewhere), and u_l = u + u~ (divergence-free where u carried the phase-change
   source).

Readings (the paper is silent on them):
* Neighbours are face neighbours: a gas cell is a k-th neighbour when its shortest
  path of face steps through gas cells to a mixed cell has k steps.
* rho at a face is the mean of the two cells' rho(c) = rho_l c + rho_g (1 - c); a cell
  beyond an outflow boundary is a copy of the boundary cell.
* The interface of a mixed cell is its PLIC plane (the normal method of the step and
  alpha from c), A_Gamma its area.
* Periodic axes wrap. At an outflow boundary the face of a sub-domain cell is a
  free-flow face (fixed pressure) like the faces to the third gas neighbours.
* dt and h cancel: with phi = dt p~ / h the problem reads
  sum over non-wall faces of (phi_j - phi_i) / rho_f = S_i a_i per sub-domain cell,
  with S = m'' (1/rho_g - 1/rho_l), a the plane area in cell units, phi = 0 on the
  fixed-pressure side, and u~_f = -(phi_R - phi_L) / rho_f.
* A part of the sub-domain with no fixed-pressure face (a gas pocket enclosed by
  liquid with fewer than three gas layers) makes the problem singular: without a
  source there, phi = 0 in it; with one, the extension is refused.
"""
from __future__ import annotations

import numpy as np

LIQUID, FAR = -1, 100  # labels: 0 mixed, 1..3 gas layers, FAR other gas


def _neighbour(shape, bc, ndim, idx, axis, step):
    """Index of the face neighbour of cell idx (z, y, x) along axis (0 = x) in
    direction step, or None beyond an outflow boundary."""
    q = list(idx)
    k = 2 - axis  # array position of the axis in (z, y, x)
    n = shape[k]
    q[k] += step
    if 0 <= q[k] < n:
        return tuple(q)
    if bc[axis] == 0:
        q[k] %= n
        return tuple(q)
    return None


def labels(c, bc, ndim, eps=1e-12):
    """0 for mixed cells, -1 liquid, 1..3 for the gas layers, FAR beyond."""
    lab = np.full(c.shape, FAR, dtype=np.int64)
    lab[c >= 1.0 - eps] = LIQUID
    lab[(c > eps) & (c < 1.0 - eps)] = 0
    for k in (1, 2, 3):
        prev = lab == k - 1
        new = lab.copy()
        for idx in zip(*np.nonzero(lab == FAR)):
            for axis in range(ndim):
                for step in (-1, 1):
                    j = _neighbour(c.shape, bc, ndim, idx, axis, step)
                    if j is not None and prev[j]:
                        new[idx] = k
        lab = new
    return lab


def plane_area(orc, cfg, c, idx):
    """Area (cell units) of the PLIC plane of the mixed cell idx, reconstructed from
    its 3x3x3 block like the sweeps do."""
    nz, ny, nx = c.shape
    z, y, x = idx
    c27 = np.empty(27)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                q = [z + dz, y + dy, x + dx]
                for k, n in enumerate((nz, ny, nx)):
                    axis = 2 - k
                    if cfg.ndim == 2 and axis == 2:
                        q[k] = 0
                    elif cfg.bc[axis] == 0:
                        q[k] %= n
                    else:
                        q[k] = min(max(q[k], 0), n - 1)
                c27[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] = c[tuple(q)]
    m = orc.normal(c27, cfg.normal)
    alpha = orc.alpha_of(m, c[idx])
    return orc.area(m, alpha)


def extend_velocity(cfg, c, u, v, w, mdot, rho_g):
    """Returns (u_l, v_l, w_l, corrections (du, dv, dw), labels, phi) for the
    liquid-velocity extension of the fractions c with mass flux mdot; face arrays in
    the MAC layouts u [nz][ny][nx+1], v [nz][ny+1][nx], w [nz+1][ny][nx] (w None in 2D)."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as csg
    import scipy.sparse.linalg as spla

    import oracle as orc

    c = np.asarray(c, dtype=np.float64)
    mdot = np.asarray(mdot, dtype=np.float64)
    rho_l = cfg.rho_l
    bc, ndim = cfg.bc, cfg.ndim
    lab = labels(c, bc, ndim, cfg.eps_mixed)
    rho = rho_l * c + rho_g * (1.0 - c)
    cells = [tuple(i) for i in np.argwhere((lab >= 0) & (lab <= 2))]
    index = {cell: k for k, cell in enumerate(cells)}
    S = 1.0 / rho_g - 1.0 / rho_l

    rows, cols, vals = [], [], []
    b = np.zeros(len(cells))
    has_fixed = np.zeros(len(cells), dtype=bool)
    for k, cell in enumerate(cells):
        diag = 0.0
        for axis in range(ndim):
            for step in (-1, 1):
                j = _neighbour(c.shape, bc, ndim, cell, axis, step)
                if j is None:  # outflow boundary: fixed pressure, ghost = copy
                    diag -= 1.0 / rho[cell]
                    has_fixed[k] = True
                    continue
                if lab[j] == LIQUID:
                    continue  # wall
                coef = 1.0 / (0.5 * (rho[cell] + rho[j]))
                diag -= coef
                if j in index:
                    rows.append(k)
                    cols.append(index[j])
                    vals.append(coef)
                else:  # third gas neighbour: fixed pressure
                    has_fixed[k] = True
        rows.append(k)
        cols.append(k)
        vals.append(diag)
        if lab[cell] == 0 and mdot[cell] != 0.0:
            b[k] = mdot[cell] * S * plane_area(orc, cfg, c, cell)
    n = len(cells)
    phi_u = np.zeros(n)
    if n:
        A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
        # a connected part of the sub-domain without a fixed-pressure face has a
        # solution only without a source (then phi = 0 there); with one it is refused
        ncomp, comp = csg.connected_components(A, directed=False)
        active = np.zeros(n, dtype=bool)
        for q in range(ncomp):
            part = comp == q
            if has_fixed[part].any():
                active |= part
            elif np.any(b[part] != 0.0):
                raise ValueError("a part of the extension sub-domain with a source has no fixed-pressure face")
        if active.any():
            idx = np.nonzero(active)[0]
            phi_u[idx] = spla.spsolve(A[idx][:, idx].tocsc(), b[idx])
    phi = np.zeros(c.shape)
    for k, cell in enumerate(cells):
        phi[cell] = phi_u[k]

    def corrections(axis):
        nz, ny, nx = c.shape
        shape = [nz, ny, nx]
        shape[2 - axis] += 1
        du = np.zeros(shape)
        n_ax = c.shape[2 - axis]
        for fidx in np.ndindex(*shape):
            f = fidx[2 - axis]
            if bc[axis] == 0 and f == n_ax:
                continue  # the periodic copy of face 0, set below
            R = list(fidx)
            L = list(fidx)
            L[2 - axis] = f - 1
            Rc = tuple(R) if f < n_ax else None
            if f >= 1:
                Lc = tuple(L)
            elif bc[axis] == 0:
                L[2 - axis] = n_ax - 1
                Lc = tuple(L)
            else:
                Lc = None
            if Rc is None and bc[axis] == 0:
                R[2 - axis] = 0
                Rc = tuple(R)
            inL = Lc is not None and 0 <= lab[Lc] <= 2
            inR = Rc is not None and 0 <= lab[Rc] <= 2
            if not (inL or inR):
                continue
            if (Lc is not None and lab[Lc] == LIQUID) or (Rc is not None and lab[Rc] == LIQUID):
                continue  # wall
            rL = rho[Lc] if Lc is not None else rho[Rc]
            rR = rho[Rc] if Rc is not None else rho[Lc]
            pL = phi[Lc] if inL else 0.0
            pR = phi[Rc] if inR else 0.0
            du[fidx] = -(pR - pL) / (0.5 * (rL + rR))
        if bc[axis] == 0:
            sl_last = [slice(None)] * 3
            sl_first = [slice(None)] * 3
            sl_last[2 - axis] = n_ax
            sl_first[2 - axis] = 0
            du[tuple(sl_last)] = du[tuple(sl_first)]
        return du

    du = corrections(0)
    dv = corrections(1)
    dw = corrections(2) if ndim == 3 else None
    ul = np.asarray(u, dtype=np.float64) + du
    vl = np.asarray(v, dtype=np.float64) + dv
    wl = None if ndim == 2 else np.asarray(w, dtype=np.float64) + dw
    return ul, vl, wl, (du, dv, dw), lab, phi
