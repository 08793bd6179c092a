"""Windows cut out of a full-size input for checking one step against the oracle:
after one step a cell depends only on cells within 7 of it, so a 32^3 window whose
cut edges are treated as outflow boundaries reproduces the full-domain step on its
inner 16^3 cells (on every side that is cut; sides on an outflow boundary of the
domain are exact)."""
import numpy as np

WIN = 32
MARGIN = 8


def window_index(start, n, periodic):
    """Cell indices of a window starting at `start` (periodic: wrapped; outflow: the
    window is shifted inside the domain)."""
    if periodic:
        return (start + np.arange(WIN)) % n, (start + np.arange(WIN + 1)) % n
    s = min(max(start, 0), n - WIN)
    return s + np.arange(WIN), s + np.arange(WIN + 1)


def cut(wl, z0, y0, x0):
    """The window's inputs and which window sides are cut (not a domain boundary)."""
    nz, ny, nx = wl.shape
    per = [b == 0 for b in wl.bc]
    xi, xf = window_index(x0, nx, per[0])
    yi, yf = window_index(y0, ny, per[1])
    zi, zf = window_index(z0, nz, per[2])
    c = wl.c[np.ix_(zi, yi, xi)]
    e = wl.e[np.ix_(zi, yi, xi)]
    u = wl.u[np.ix_(zi, yi, xf)]
    v = wl.v[np.ix_(zi, yf, xi)]
    w = wl.w[np.ix_(zf, yi, xi)]
    md = None if wl.mdot is None else wl.mdot[np.ix_(zi, yi, xi)]
    # a side is exact only where the window ends on an outflow boundary of the domain
    exact = []
    for idx, n, p in ((xi, nx, per[0]), (yi, ny, per[1]), (zi, nz, per[2])):
        exact.append((not p and idx[0] == 0, not p and idx[-1] == n - 1))
    return (zi, yi, xi), c, e, u, v, w, md, exact


def inner(exact_lo, exact_hi):
    lo = 0 if exact_lo else MARGIN
    hi = WIN if exact_hi else WIN - MARGIN
    return slice(lo, hi)



def window_oracle_step(oracle, wl, z0, y0, x0, step_index):
    """The oracle's step on the window at (z0, y0, x0) and the index sets / inner slices
    that locate its trusted cells in the full domain."""
    idx, c, e, u, v, w, md, exact = cut(wl, z0, y0, x0)
    cfg = oracle.Config(shape=(WIN, WIN, WIN), h=wl.h, ndim=3, bc=(1, 1, 1), cp_l=wl.cp_l,
                        cp_g=wl.cp_g, rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal)
    co, eo, _ = oracle.step(cfg, c, e, u, v, w, md, wl.dt, wl.u_scale(step_index), step_index)
    sl = (inner(*exact[2]), inner(*exact[1]), inner(*exact[0]))
    return idx, sl, co, eo


def pick_windows(wl, k, seed):
    """k windows centred on seeded mixed cells, plus the two corner windows."""
    rng = np.random.default_rng(seed)
    mixed = np.argwhere((wl.c > 1e-12) & (wl.c < 1 - 1e-12))
    pick = mixed[rng.choice(len(mixed), size=k, replace=False)]
    out = [tuple(int(p) - WIN // 2 for p in q) for q in pick]
    out.append((0, 0, 0))
    out.append(tuple(int(s) - WIN for s in wl.shape))
    return out
