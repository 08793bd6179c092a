"""GPU parity at full size: one whole step of the 256^3 expanding bubble (with phase
change) and of the 512^3 field of 2000 droplets, run by the library on the full
domain, checked against the FP64 oracle on sampled 32^3 windows (inner 16^3 cells;
the window method is checked against full-domain oracle steps in
test_window_harness.py)."""
import numpy as np
import pytest

import oracle
from paper_2001_03477_amd import workloads as W
from windows import pick_windows, window_oracle_step

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def pc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_03477_amd import pcvof
    pcvof.lib()
    return pcvof


def _check_windows(pc, wl, step_index, windows):
    spec = pc.DomainSpec(shape=wl.shape, h=wl.h, ndim=3, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                         rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal)
    d = pc.Domain(spec)
    d.set_vof(wl.c)
    d.set_energy(wl.e)
    d.set_velocity(wl.u, wl.v, wl.w)
    if wl.mdot is not None:
        d.set_mass_flux(wl.mdot)
    d.step_index = step_index
    d.step(wl.dt, wl.u_scale(step_index))
    c_gpu = d.vof().cpu().numpy()
    e_gpu = d.energy().cpu().numpy()
    del d
    escale = float(np.max(np.abs(wl.e)))
    for (z0, y0, x0) in windows:
        (zi, yi, xi), sl, co, eo = window_oracle_step(oracle, wl, z0, y0, x0, step_index)
        got_c = c_gpu[np.ix_(zi, yi, xi)][sl]
        got_e = e_gpu[np.ix_(zi, yi, xi)][sl]
        err_c = np.max(np.abs(got_c - co[sl]))
        err_e = np.max(np.abs(got_e - eo[sl]))
        assert err_c <= TOL * max(1.0, float(np.max(np.abs(co[sl])))), \
            f"{wl.name} window {(z0, y0, x0)}: c error {err_c:.3e}"
        assert err_e <= TOL * max(escale, float(np.max(np.abs(eo[sl])))), \
            f"{wl.name} window {(z0, y0, x0)}: e error {err_e:.3e}"


@pytest.mark.timeout(600)
@pytest.mark.parametrize("step_index", [0, 1])
def test_bubble_256_full_step_windows(pc, step_index):
    wl = W.bubble_3d(256)
    _check_windows(pc, wl, step_index, pick_windows(wl, 6, 10 + step_index))


@pytest.mark.timeout(600)
def test_droplets_512_full_step_windows(pc):
    wl = W.droplets_3d(512)
    _check_windows(pc, wl, 2, pick_windows(wl, 8, 20))
