"""GPU parity of the Lagrangian-explicit sweeps (the method of Li, CIAM, which section
3.3 names beside the Weymouth-Yue split; kept as an ablation): the library through the
C-ABI against the FP64 oracle in the same mode, per cell within 1e-12 (fractions
absolute, energies relative to max |e|), on single sweeps, on steps over several tiles
with ragged tails and phase change, on a plane under a velocity linear along the sweep
(whose exact result is known), and in the mixed-precision mode."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_03477_amd import workloads as W

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


def _assert_close(got, ref, scale, what):
    err = float(np.max(np.abs(got - ref)))
    bound = TOL * max(scale, float(np.max(np.abs(ref))))
    assert err <= bound, f"{what}: max error {err:.3e} > {bound:.3e}"


def _specs(pc, wl, bc=None, precision="fp64", normal=None):
    args = dict(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc if bc is None else bc, cp_l=wl.cp_l,
                cp_g=wl.cp_g, rho_l=wl.rho_l, T_gamma=wl.T_gamma,
                normal=wl.normal if normal is None else normal)
    spec = pc.DomainSpec(**args, precision=precision, split="le")
    cfg = oracle.Config(**args, split=1)
    return spec, cfg


def _domain(pc, spec, c, e, u, v, w, mdot=None):
    d = pc.Domain(spec)
    d.set_vof(c)
    d.set_energy(e)
    d.set_velocity(u, v, w)
    if mdot is not None:
        d.set_mass_flux(mdot)
    return d


SWEEP_CASES = {
    "drops3d-periodic": lambda: W.random_drops_3d(n=24, ndrops=5, seed=141, cfl=0.45, rmin=1.5, rmax=4.0),
    "drops3d-ragged": lambda: W.random_drops_3d(n=21, ndrops=4, seed=142, cfl=0.45, rmin=1.5, rmax=3.5),
    "circle2d": lambda: W.circle_2d(64),
}


@pytest.mark.parametrize("case", sorted(SWEEP_CASES))
@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_le_single_sweep_parity(pc, case, bc):
    wl = SWEEP_CASES[case]()
    bcs = (0, 0, 0) if bc == "periodic" else (1, 1, 1)
    spec, cfg = _specs(pc, wl, bc=bcs)
    kfac = wl.dt / wl.h
    cc, ec = oracle.prologue(cfg, wl.c, wl.e)
    vel = (wl.u, wl.v, wl.w)
    hv = wl.h ** wl.ndim
    for axis in range(wl.ndim):
        d = _domain(pc, spec, wl.c, wl.e, wl.u, wl.v, wl.w)
        d.begin_step()
        d.sweep(axis, wl.dt, 1.0)
        st = d.end_step()
        c_ref, e_ref, acc = oracle.sweep(cfg, axis, wl.c, wl.e, cc, ec, vel[axis], kfac)
        _assert_close(d.vof().cpu().numpy(), c_ref, 1.0, f"{case} axis {axis} c")
        _assert_close(d.energy().cpu().numpy(), e_ref, 0.0, f"{case} axis {axis} e")
        assert st["vol_src"] == pytest.approx(acc[4] * hv, abs=1e-13)
        assert st["energy_src"] == pytest.approx(acc[5] * hv, abs=1e-12 * abs(st["energy"]))
        assert st["vol_bnd_out"] == pytest.approx(acc[2] * hv, abs=1e-13)
        assert abs(st["vol_clip"]) <= 1e-15  # bounded without clipping


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 1)])
def test_le_steps_over_many_tiles(pc, bc):
    """70^3 drops (two x segments and several y / z chunks, all with ragged tails),
    three steps with the sweep order rotating, phase change on the outflow domain."""
    wl = W.random_drops_3d(n=70, ndrops=12, seed=143, cfl=0.4, rmin=2.0, rmax=6.0)
    mdot = None
    if bc != (0, 0, 0):
        mdot = np.random.default_rng(143).uniform(-0.3, 0.8, size=wl.shape)
    spec, cfg = _specs(pc, wl, bc=bc)
    d = _domain(pc, spec, wl.c, wl.e, wl.u, wl.v, wl.w, mdot)
    c, e = wl.c, wl.e
    for n in range(3):
        st = d.step(wl.dt, 1.0, stats=True)
        c, e, st_ref = oracle.step(cfg, c, e, wl.u, wl.v, wl.w, mdot, wl.dt, 1.0, n)
        _assert_close(d.vof().cpu().numpy(), c, 1.0, f"step {n} c")
        _assert_close(d.energy().cpu().numpy(), e, 0.0, f"step {n} e")
        for k in ("vol", "energy"):
            assert st[k] == pytest.approx(st_ref[k], rel=1e-12)
        for k in ("vol_src", "vol_clip", "vol_bnd_out", "vol_phase"):
            assert st[k] == pytest.approx(st_ref[k], abs=1e-13)


def test_le_plane_under_linear_velocity_is_exact(pc):
    """A tilted plane in a velocity linear along x: one x sweep of the library puts it
    exactly where the linear map does (rows next to the outflow walls in y, whose ghost
    copies bend the plane, are not compared)."""
    n, ny = 96, 40
    h = 1.0 / n
    shape = (1, ny, n)
    slope, x_gamma, a, x0 = 0.2, 0.40, 0.25 / n, 0.45
    c = W.line_fraction_field(shape, h, x_gamma, slope)
    e = 1.0 + 3.0 * c
    xf = np.arange(n + 1) * h
    u = np.broadcast_to(a * (xf - x0) / h, (1, ny, n + 1)).copy()  # CFL numbers (dt = h)
    v = np.zeros((1, ny + 1, n))
    wl = W.Workload("stretch2d", shape, h, 2, (1, 1, 1), 1.0, 1.0, 1.0, 1.0, c, e, u, v, None, None, h, 1)
    spec, _ = _specs(pc, wl, normal=2)
    d = _domain(pc, spec, c, e, u, v, None)
    d.begin_step()
    d.sweep(0, h, 1.0)
    d.end_step()
    got = d.vof().cpu().numpy()
    want = W.line_fraction_field(shape, h, x_gamma + a * (x_gamma - x0), slope * (1.0 + a))
    rows = slice(1, ny - 1)
    assert np.max(np.abs(got[:, rows] - want[:, rows])) <= 1e-14


def test_le_mixed_precision(pc):
    """Mixed precision in the Lagrangian-explicit mode against the FP64 oracle in the
    same mode: L1 and max errors of the fractions at the level of the conservative mode,
    and the volume bookkeeping identity to round-off."""
    wl = W.random_drops_3d(n=32, ndrops=5, seed=144, rmin=2.0, rmax=5.0)
    spec, cfg = _specs(pc, wl, precision="mixed")
    d = _domain(pc, spec, wl.c, wl.e, wl.u, wl.v, wl.w)
    c, e = wl.c, wl.e
    vol = math.fsum(wl.c.ravel()) * wl.h ** 3
    for k in range(6):
        st = d.step(wl.dt, 1.0, stats=True)
        c, e, _ = oracle.step(cfg, c, e, wl.u, wl.v, wl.w, None, wl.dt, 1.0, k)
        expect = -st["vol_bnd_out"] + st["vol_src"] + st["vol_clip"] + st["vol_phase"]
        assert abs(st["vol"] - vol - expect) <= 1e-12 * vol
        vol = st["vol"]
    got = d.vof().cpu().numpy()
    err = np.abs(got - c)
    assert err.max() <= 1e-4 and err.sum() / c.sum() <= 1e-6
    assert got.min() >= 0.0 and got.max() <= 1.0


def test_le_volume_drift_against_the_conservative_split(pc):
    """Periodic divergence-free flow: the Weymouth-Yue split keeps the volume to
    round-off, the Lagrangian-explicit sweeps change it by their dilatation terms (as
    the oracle does)."""
    wl = W.random_drops_3d(n=32, ndrops=6, seed=145, cfl=0.4, rmin=2.0, rmax=5.0)
    v0 = math.fsum(wl.c.ravel()) * wl.h ** 3
    drift = {}
    for split in ("wy", "le"):
        spec = pc.DomainSpec(shape=wl.shape, h=wl.h, ndim=3, cp_l=wl.cp_l, cp_g=wl.cp_g, split=split)
        d = _domain(pc, spec, wl.c, wl.e, wl.u, wl.v, wl.w)
        for k in range(4):
            st = d.step(wl.dt, 1.0, stats=True)
        drift[split] = abs(st["vol"] - v0) / v0
    assert drift["wy"] <= 1e-13
    assert drift["le"] > 1e-7


def test_le_full_size_leveque128(pc):
    """The configuration of the benchmark's split ablation: the 128^3 LeVeque field, one
    full Lagrangian-explicit step, every cell compared with the oracle, with the oracle's
    dilatation term and total volume."""
    wl = W.leveque_3d(128)
    spec, cfg = _specs(pc, wl)
    d = _domain(pc, spec, wl.c, wl.e, wl.u, wl.v, wl.w)
    st = d.step(wl.dt, wl.u_scale(0), stats=True)
    c, e, st_ref = oracle.step(cfg, wl.c, wl.e, wl.u, wl.v, wl.w, None, wl.dt, wl.u_scale(0), 0)
    _assert_close(d.vof().cpu().numpy(), c, 1.0, "c")
    _assert_close(d.energy().cpu().numpy(), e, 0.0, "e")
    assert st["vol_src"] == pytest.approx(st_ref["vol_src"], abs=1e-13)
    assert st["vol"] == pytest.approx(st_ref["vol"], rel=1e-13)
