"""PCVOF ORACLE -- test infrastructure, not part of the product.

Implicit energy diffusion with the interface temperature imposed (section 3.4.2, eqs.
T_diff_disc and mod_branchesT), written plainly in numpy with a sparse direct solve
(scipy). Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
load it. It shares no code with the HIP library.

The step, in the paper's order:
1. The phase of a node: liquid when c >= 1/2, gas otherwise. Each phase is solved with
   its own constant properties (conductivity k_p, volumetric heat capacity C_p).
2. Between two face neighbours of the same phase the gradient is the plain difference
   over h. Towards a neighbour of the other phase the interface is a boundary at
   distance theta from the node, with T = T_Gamma there: the gradient is
   (T_Gamma - T_i) / theta, and the node's control width along that axis becomes
   (h + theta) / 2 (both sides irregular: (theta_L + theta_R) / 2).
3. Backward Euler: C_p (T^{n+1} - T*) / dt = k_p sum over axes of
   (G_R - G_L) / W, with the gradients G taken at T^{n+1}.

Readings (the paper is silent on them):
* theta from the height function: the column of six cells along the axis centred on
  the face (three on the node's side, three on the neighbour's). When its outer cell on
  the node's side is pure in the node's phase and its outer cell on the other side is
  pure in the other phase, the interface lies sum(f) cells from the outer face on the
  node's side (f the node phase's indicator: c, or 1 - c), and theta = (sum f - 5/2) h
  (the node sits 5/2 cells from that face). Otherwise (no height in that direction) the
  paper uses a plane in the staggered volume between the two nodes; the reading here is
  the plane where the linear interpolation of f between the two nodes crosses 1/2:
  theta = h (f_i - 1/2) / (f_i - f_j).
* theta is capped to [eps_theta h, h] with eps_theta = 1e-3 (the paper's value).
* Domain boundaries: periodic axes wrap; outflow boundaries are adiabatic (zero
  gradient), matching the zero-gradient ghosts of the advection; cells beyond them are
  copies for the height columns.
* "Pure" uses the mixed-cell threshold eps < c < 1 - eps of the step.
* The step returns T^{n+1}; the energy of a cell is then C_p(c) T^{n+1} with the
  one-fluid C_p(c) of the advection.
"""
from __future__ import annotations

import numpy as np

EPS_THETA = 1e-3


def _cell(shape, bc, idx, axis, off):
    """Index of the cell off steps along axis from idx: periodic wrap, outflow copy
    (clamped); None only is never returned (columns use copies)."""
    q = list(idx)
    k = 2 - axis
    n = shape[k]
    q[k] += off
    if q[k] < 0 or q[k] >= n:
        if bc[axis] == 0:
            q[k] %= n
        else:
            q[k] = min(max(q[k], 0), n - 1)
    return tuple(q)


def _neighbour(shape, bc, idx, axis, step):
    """Face neighbour, or None beyond an outflow boundary."""
    q = list(idx)
    k = 2 - axis
    n = shape[k]
    q[k] += step
    if 0 <= q[k] < n:
        return tuple(q)
    if bc[axis] == 0:
        q[k] %= n
        return tuple(q)
    return None


def theta(c, bc, idx, axis, step, eps_mixed=1e-12, eps_theta=EPS_THETA):
    """Distance (cell units) from node idx to the interface towards its face neighbour
    along axis in direction step (which is in the other phase)."""
    liquid = c[idx] >= 0.5

    def f(cell):
        return c[cell] if liquid else 1.0 - c[cell]

    col = [_cell(c.shape, bc, idx, axis, o * step) for o in (-2, -1, 0, 1, 2, 3)]
    near, far = f(col[0]), f(col[5])
    if near >= 1.0 - eps_mixed and far <= eps_mixed:
        t = sum(f(q) for q in col) - 2.5
    else:
        j = _neighbour(c.shape, bc, idx, axis, step)
        fi, fj = f(idx), f(j)
        t = (fi - 0.5) / (fi - fj)
    return min(max(t, eps_theta), 1.0)


def _stencil(cfg, c, idx, k_l, k_g):
    """Per axis: list of (neighbour or None, weight on (T_nb - T_i), interface distance
    or None, control width) pieces of the operator at node idx, in cell units (h = 1)."""
    liquid = c[idx] >= 0.5
    out = []
    for axis in range(cfg.ndim):
        sides = []
        for step in (-1, 1):
            j = _neighbour(c.shape, cfg.bc, idx, axis, step)
            if j is None:
                sides.append(("wall", None, 1.0))
            elif (c[j] >= 0.5) == liquid:
                sides.append(("node", j, 1.0))
            else:
                t = theta(c, cfg.bc, idx, axis, step, cfg.eps_mixed)
                sides.append(("gamma", None, t))
        width = 0.5 * (sides[0][2] + sides[1][2])
        out.append((sides, width))
    return out


def operator_at(cfg, c, T, idx, k_l, k_g, T_gamma):
    """(1/V) integral of div(k grad T) at node idx by eq. T_diff_disc with the gradients
    of eq. mod_branchesT (physical units, h = cfg.h)."""
    h = cfg.h
    k = k_l if c[idx] >= 0.5 else k_g
    acc = 0.0
    for sides, width in _stencil(cfg, c, idx, k_l, k_g):
        grads = []
        for sgn, (kind, j, w) in zip((-1, 1), sides):
            if kind == "wall":
                g = 0.0
            elif kind == "node":
                g = (T[j] - T[idx]) / h if sgn > 0 else (T[idx] - T[j]) / h
            else:
                g = (T_gamma - T[idx]) / (w * h) if sgn > 0 else (T[idx] - T_gamma) / (w * h)
            grads.append(g)
        acc += (grads[1] - grads[0]) / (width * h)
    return k * acc


def apply_operator(cfg, c, T, k_l, k_g, T_gamma):
    """operator_at at every node."""
    L = np.zeros(c.shape)
    for idx in np.ndindex(*c.shape):
        L[idx] = operator_at(cfg, c, T, idx, k_l, k_g, T_gamma)
    return L


def diffuse(cfg, c, T, dt, k_l, k_g, T_gamma, return_rhs=False):
    """One backward-Euler diffusion step: returns T^{n+1} with
    C_p (T^{n+1} - T) / dt = apply_operator(T^{n+1}) node by node (C_p and k of the
    node's phase); with return_rhs, (T^{n+1}, b) with b the right-hand side of the
    assembled system (T* and the T_Gamma terms)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    c = np.asarray(c, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    h = cfg.h
    n = c.size
    index = {idx: q for q, idx in enumerate(np.ndindex(*c.shape))}
    rows, cols, vals = [], [], []
    b = np.empty(n)
    for idx, q in index.items():
        liquid = c[idx] >= 0.5
        k, C = (k_l, cfg.cp_l) if liquid else (k_g, cfg.cp_g)
        a = dt * k / C
        diag = 1.0
        rhs = T[idx]
        for sides, width in _stencil(cfg, c, idx, k_l, k_g):
            for kind, j, w in sides:
                if kind == "wall":
                    continue
                coef = a / (width * h * w * h)
                diag += coef
                if kind == "node":
                    rows.append(q)
                    cols.append(index[j])
                    vals.append(-coef)
                else:
                    rhs += coef * T_gamma
        rows.append(q)
        cols.append(q)
        vals.append(diag)
        b[q] = rhs
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    x = spla.spsolve(A.tocsc(), b).reshape(c.shape)
    return (x, b.reshape(c.shape)) if return_rhs else x
