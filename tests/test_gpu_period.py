"""One period of the 3D LeVeque deformation (the C2 field: sphere R = 0.15 at (0.35, 0.35,
0.35) in a walled unit box, time scale cos(pi t / T), T = 3, CFL 0.3). The flow reverses at
T / 2, so the exact field after T is the initial one. Properties checked at 32^3, 64^3 and
128^3 on the FP64 path: the volume is conserved to round-off over the whole period (walls
with no normal flow, discretely divergence-free faces), the fractions stay in [0, 1], and the
L1 shape error sum |c(T) - c(0)| h^3 falls at each refinement (the method converges on this
field); the mixed-precision path lands within 1% of the FP64 error at 64^3."""
import math

import numpy as np
import pytest

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


def _period(pc, wl, precision="fp64"):
    spec = pc.DomainSpec(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                         normal=wl.normal, precision=precision)
    d = pc.Domain(spec)
    d.set_vof(wl.c)
    d.set_energy(wl.e)
    d.set_velocity(wl.u, wl.v, wl.w)
    d.steps(wl.steps, wl.dt, u_scale=[wl.u_scale(k) for k in range(wl.steps)])
    c = d.vof().cpu().numpy()
    d.close()
    hv = wl.h ** 3
    v0 = math.fsum(wl.c.ravel().tolist()) * hv
    v1 = math.fsum(c.ravel().tolist()) * hv
    l1 = math.fsum(np.abs(c - wl.c).ravel().tolist()) * hv
    return c, l1, (v1 - v0) / v0


@pytest.mark.timeout(600)
def test_leveque_period_converges_and_conserves(pc):
    errs = {}
    for n in (32, 64, 128):
        wl = W.leveque_3d(n)
        assert abs(wl.steps * wl.dt - 3.0) < wl.dt
        c, l1, dv = _period(pc, wl)
        assert abs(dv) <= 1e-13, f"{n}^3: volume change {dv:.3e}"
        assert c.min() >= 0.0 and c.max() <= 1.0
        errs[n] = l1
    print("L1 shape error after one period:", {n: f"{e:.3e}" for n, e in errs.items()})
    assert errs[64] < errs[32] and errs[128] < errs[64], errs


def test_leveque_period_mixed_precision(pc):
    wl = W.leveque_3d(64)
    _, l1, _ = _period(pc, wl)
    _, l1m, dvm = _period(pc, wl, "mixed")
    assert abs(dvm) <= 1e-6
    assert abs(l1m - l1) <= 0.01 * l1, (l1, l1m)
