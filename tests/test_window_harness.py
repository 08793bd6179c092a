"""The windowed check used for full-size parity: the oracle's step on a 32^3 window cut
out of a larger input equals the oracle's full-domain step on the window's trusted
inner cells, bitwise (periodic droplets with a rotated sweep order, and the outflow
bubble with phase change, including windows on the domain boundary)."""
import numpy as np
import pytest

import oracle
from paper_2001_03477_amd import workloads as W
from windows import pick_windows, window_oracle_step


@pytest.mark.parametrize("case", ["droplets", "bubble"])
def test_window_step_equals_full_domain_step(case):
    if case == "droplets":
        wl = W.droplets_3d(48, ndrops=12, rmin=2.0, rmax=5.0, seed=7)
        step_index = 1
    else:
        wl = W.bubble_3d(48, R=0.2)
        step_index = 2
    cfg = oracle.Config(shape=wl.shape, h=wl.h, ndim=3, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                        rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal)
    cf, ef, _ = oracle.step(cfg, wl.c, wl.e, wl.u, wl.v, wl.w, wl.mdot, wl.dt,
                            wl.u_scale(step_index), step_index)
    for (z0, y0, x0) in pick_windows(wl, 3, 5):
        (zi, yi, xi), sl, co, eo = window_oracle_step(oracle, wl, z0, y0, x0, step_index)
        assert np.array_equal(cf[np.ix_(zi, yi, xi)][sl], co[sl])
        assert np.array_equal(ef[np.ix_(zi, yi, xi)][sl], eo[sl])
