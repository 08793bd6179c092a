"""The pieces of the paper's time step composed in its order, on the GPU through the
C-ABI and in the oracle: the liquid-velocity extension of the one-fluid velocity
(section 3.3.1), the advection step with phase change (sections 3.3 and 3.4.1) on the
extended velocity, and the implicit energy diffusion (section 3.4.2), for three steps
(the mass flux is given: its GPU computation is switched off).

The chain checks that the states handed from stage to stage (stored velocity,
fractions, energies) are the ones the next stage expects, at the suite's 1e-12: the
fractions absolutely, the temperatures relative to max |T| (measured 1e-15 and 8e-15
over three steps; the two solves contribute at about rel_tol = 1e-13 times their
conditioning)."""
import numpy as np
import pytest

import oracle
from oracle import diffusion as D
from oracle import extension as X
from paper_2001_03477_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_03477_amd import pcvof
    pcvof.lib()
    return pcvof


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1)])
def test_extension_advection_diffusion_chain(pc, bc):
    wl = W.random_drops_3d(n=20, ndrops=3, seed=181, cfl=0.2, rmin=2.5, rmax=4.5)
    rng = np.random.default_rng(181)
    mdot = rng.uniform(0.0, 0.03, size=wl.shape)  # keeps u + u~ within the CFL limit
    rho_l, rho_g, k_l, k_g, Tg = 2.5, 0.25, 0.07, 0.007, 0.5
    cp = (2.5, 0.25)
    T0 = rng.uniform(0.3, 0.7, size=wl.shape)
    e0 = (cp[0] * wl.c + cp[1] * (1 - wl.c)) * T0
    spec = pc.DomainSpec(shape=wl.shape, h=wl.h, ndim=3, bc=bc, cp_l=cp[0], cp_g=cp[1], rho_l=rho_l, T_gamma=Tg)
    cfg = oracle.Config(shape=wl.shape, h=wl.h, ndim=3, bc=bc, cp_l=cp[0], cp_g=cp[1], rho_l=rho_l, T_gamma=Tg)
    d = pc.Domain(spec)
    d.set_vof(wl.c)
    d.set_energy(e0)
    c, e = wl.c, e0
    for n in range(3):
        # the one-fluid velocity of each step is the generated field; the extension
        # turns it into the liquid velocity of this step's fractions
        d.set_velocity(wl.u, wl.v, wl.w)
        d.set_mass_flux(mdot)
        d.extend_velocity(rho_g)
        d.step(wl.dt, 1.0)
        d.diffuse(wl.dt, k_l, k_g)
        ul, vl, wl_, *_ = X.extend_velocity(cfg, c, wl.u, wl.v, wl.w, mdot, rho_g)
        c, e, _ = oracle.step(cfg, c, e, ul, vl, wl_, mdot, wl.dt, 1.0, n)
        T = e / (cp[0] * c + cp[1] * (1 - c))
        T = D.diffuse(cfg, c, T, wl.dt, k_l, k_g, Tg)
        e = (cp[0] * c + cp[1] * (1 - c)) * T
        cg = d.vof().cpu().numpy()
        eg = d.energy().cpu().numpy()
        Tgpu = eg / (cp[0] * cg + cp[1] * (1 - cg))
        ec = np.max(np.abs(cg - c))
        eT = np.max(np.abs(Tgpu - T)) / np.max(np.abs(T))
        print(f"bc {bc} step {n}: max |c - ref| {ec:.2e}, max |T - ref| / max |T| {eT:.2e}")
        assert ec <= 1e-12 and eT <= 1e-12
