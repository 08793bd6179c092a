"""GPU parity: the HIP library (through the C-ABI) against the FP64 oracle on the
same seeded inputs. Bar: |x_gpu - x_oracle| <= 1e-12 max(|x_oracle|, s) per cell
with s = 1 for the volume fraction and s = max|e| for the energy."""
import math

import numpy as np
import pytest

import oracle
from paper_2001_03477_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def pc(torch_cuda):
    from paper_2001_03477_amd import pcvof
    pcvof.lib()
    return pcvof


def _assert_close(got, ref, scale, what):
    err = np.max(np.abs(got - ref)) if got.size else 0.0
    bound = TOL * max(scale, float(np.max(np.abs(ref))) if ref.size else 0.0)
    assert err <= bound, f"{what}: max error {err:.3e} > {bound:.3e}"


def _specs(pc, wl, **kw):
    args = dict(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal)
    args.update(kw)
    o_args = {k: v for k, v in args.items()}
    spec = pc.DomainSpec(**args)
    cfg = oracle.Config(**o_args)
    return spec, cfg


def _domain(pc, spec, wl, mdot=None):
    d = pc.Domain(spec)
    d.set_vof(wl.c)
    d.set_energy(wl.e)
    d.set_velocity(wl.u, wl.v, wl.w)
    if mdot is not None:
        d.set_mass_flux(mdot)
    return d


# ------------------------------------------------------------------ geometry kernels
def test_geometry_kernels_match_oracle(pc, torch_cuda):
    torch = torch_cuda
    rng = np.random.default_rng(0)
    n = 20000
    m = rng.normal(size=(n, 3))
    m[:3000, 2] = 0.0
    m[3000:4000, 1:] = 0.0
    m[4000:5000, 0] = 1e-9 * rng.normal(size=1000)
    m /= np.abs(m).sum(1, keepdims=True)
    lo, hi = np.minimum(m, 0).sum(1), np.maximum(m, 0).sum(1)
    a = lo + rng.uniform(-0.05, 1.05, n) * (hi - lo)
    dm = torch.tensor(m, device="cuda")
    v = pc.geom_volume(dm, torch.tensor(a, device="cuda")).cpu().numpy()
    assert np.max(np.abs(v - oracle.volume_n(m, a))) <= 2e-15
    c = np.concatenate([rng.uniform(1e-12, 1 - 1e-12, n - 4000), 10 ** rng.uniform(-12, -1, 2000),
                        1 - 10 ** rng.uniform(-12, -1, 2000)])
    al = pc.geom_alpha(dm, torch.tensor(c, device="cuda")).cpu().numpy()
    assert np.max(np.abs(oracle.volume_n(m, al) - c)) <= 2e-15
    assert np.all(al >= lo - 1e-15) and np.all(al <= hi + 1e-15)
    axis = rng.integers(0, 3, n).astype(np.int32)
    lam = rng.uniform(-0.5, 0.5, n)
    ra = oracle.alpha_n(m, c)
    sl = pc.geom_slab(dm, torch.tensor(ra, device="cuda"), torch.tensor(axis, device="cuda"),
                      torch.tensor(lam, device="cuda")).cpu().numpy()
    assert np.max(np.abs(sl - oracle.slab_n(m, ra, axis, lam))) <= 2e-15
    c27 = rng.uniform(0, 1, (4000, 27))
    c27[:1000] = np.round(c27[:1000])
    c27[1000:1500] = W.sphere_fraction((3, 3, 3), 1.0, [[1.3, 1.6, 1.4]], [1.1]).reshape(1, 27)
    for method in (0, 1, 2):
        g = pc.geom_normal(torch.tensor(c27, device="cuda"), method).cpu().numpy()
        ref = np.array([oracle.normal(c27[i], method) for i in range(len(c27))])
        assert np.array_equal(g, ref), f"normal method {method} differs"
    vv = rng.uniform(-1, 2, (5000, 5))
    vv[:500] = 1.5
    w = pc.geom_weno5(torch.tensor(vv, device="cuda"), 1e-6).cpu().numpy()
    ref = np.array([oracle.weno5(vv[i]) for i in range(len(vv))])
    assert np.max(np.abs(w - ref)) <= 4e-15


# ------------------------------------------------------------------ single sweeps
SWEEP_CASES = {
    "drops3d-periodic": lambda: W.random_drops_3d(n=24, ndrops=5, seed=41, rmin=1.5, rmax=4.0),
    "drops3d-ragged": lambda: W.random_drops_3d(n=21, ndrops=4, seed=42, rmin=1.5, rmax=3.5),
    "circle2d": lambda: W.circle_2d(64),
}


@pytest.mark.parametrize("case", sorted(SWEEP_CASES))
@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_single_sweep_parity(pc, case, bc):
    wl = SWEEP_CASES[case]()
    bcs = (0, 0, 0) if bc == "periodic" else (1, 1, 1)
    spec, cfg = _specs(pc, wl, bc=bcs)
    kfac = wl.dt / wl.h
    cc, ec = oracle.prologue(cfg, wl.c, wl.e)
    vel = (wl.u, wl.v, wl.w)
    for axis in range(wl.ndim):
        d = _domain(pc, spec, wl)
        d.begin_step()
        d.sweep(axis, wl.dt, 1.0)
        st = d.end_step()
        c_ref, e_ref, acc = oracle.sweep(cfg, axis, wl.c, wl.e, cc, ec, vel[axis], kfac)
        _assert_close(d.vof().cpu().numpy(), c_ref, 1.0, f"{case} axis {axis} c")
        _assert_close(d.energy().cpu().numpy(), e_ref, 0.0, f"{case} axis {axis} e")
        hv = wl.h ** wl.ndim
        assert st["vol_src"] == pytest.approx(acc[4] * hv, abs=1e-13)
        assert st["vol_bnd_out"] == pytest.approx(acc[2] * hv, abs=1e-13)
        assert st["vol"] == pytest.approx(math.fsum(c_ref.ravel()) * hv, rel=1e-13)


# ------------------------------------------------------------------ full steps
def test_step_parity_with_phase_change(pc):
    wl = W.random_drops_3d(n=24, ndrops=5, seed=43, rmin=2.0, rmax=4.0, mdot=0.4)
    rng = np.random.default_rng(3)
    mdot = rng.uniform(-0.3, 0.8, size=wl.shape)
    for bcs in ((0, 0, 0), (1, 0, 1)):
        spec, cfg = _specs(pc, wl, bc=bcs, T_gamma=0.6)
        d = _domain(pc, spec, wl, mdot)
        c, e = wl.c, wl.e
        for n in range(3):
            st = d.step(wl.dt, 1.0, stats=True)
            c, e, st_ref = oracle.step(cfg, c, e, wl.u, wl.v, wl.w, mdot, wl.dt, 1.0, n)
            _assert_close(d.vof().cpu().numpy(), c, 1.0, f"step {n} c")
            _assert_close(d.energy().cpu().numpy(), e, 0.0, f"step {n} e")
            for k in ("vol", "energy"):
                assert st[k] == pytest.approx(st_ref[k], rel=1e-12)
            for k in ("vol_phase", "vol_src", "vol_clip", "vol_bnd_out"):
                assert st[k] == pytest.approx(st_ref[k], abs=1e-13)
            assert st["energy_phase"] == pytest.approx(st_ref["energy_phase"],
                                                       abs=1e-12 * abs(st_ref["energy"]))
            assert st["max_cfl"] == st_ref["max_cfl"]
        assert d.step_index == 3


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 1)])
def test_nonconservative_energy_flux_parity(pc, bc):
    """The ablation mode of section 3.4.1 (eq. disc_et_adv_noncons) with water-like heat
    capacities: three steps, with phase change on the outflow domain."""
    wl = W.random_drops_3d(n=24, ndrops=5, seed=45, rmin=2.0, rmax=4.0, cp=(4039.0, 1.248))
    mdot = None
    if bc != (0, 0, 0):
        mdot = np.random.default_rng(4).uniform(-0.3, 0.8, size=wl.shape)
    spec, cfg = _specs(pc, wl, bc=bc)
    spec.energy_flux = "nonconservative"
    cfg.energy_flux = 1
    d = _domain(pc, spec, wl, mdot)
    c, e = wl.c, wl.e
    for n in range(3):
        st = d.step(wl.dt, 1.0, stats=True)
        c, e, st_ref = oracle.step(cfg, c, e, wl.u, wl.v, wl.w, mdot, wl.dt, 1.0, n)
        _assert_close(d.vof().cpu().numpy(), c, 1.0, f"step {n} c")
        _assert_close(d.energy().cpu().numpy(), e, 0.0, f"step {n} e")
        assert st["energy"] == pytest.approx(st_ref["energy"], rel=1e-12)
        assert st["energy_bnd_out"] == pytest.approx(st_ref["energy_bnd_out"], abs=1e-12 * abs(st_ref["energy"]))


def test_circle2d_trajectory_parity(pc):
    """The 2D 64x64 circle (uniform velocity (1, 0.5), CFL 0.25, m'' = 0.01): all 100
    steps from identical inputs."""
    wl = W.circle_2d(64)
    spec, cfg = _specs(pc, wl)
    d = _domain(pc, spec, wl, wl.mdot)
    c, e = wl.c, wl.e
    for n in range(wl.steps):
        d.step(wl.dt, 1.0)
        c, e, _ = oracle.step(cfg, c, e, wl.u, wl.v, None, wl.mdot, wl.dt, 1.0, n)
        if n % 10 == 9 or n == wl.steps - 1:
            _assert_close(d.vof().cpu().numpy(), c, 1.0, f"step {n} c")
            _assert_close(d.energy().cpu().numpy(), e, 0.0, f"step {n} e")


def test_leveque_trajectory_parity_small(pc):
    """LeVeque deformation at 32^3 with the time-dependent scale cos(pi t / T)."""
    wl = W.leveque_3d(32)
    spec, cfg = _specs(pc, wl)
    d = _domain(pc, spec, wl)
    c, e = wl.c, wl.e
    for n in range(12):
        s = wl.u_scale(n)
        d.step(wl.dt, s)
        c, e, _ = oracle.step(cfg, c, e, wl.u, wl.v, wl.w, None, wl.dt, s, n)
    _assert_close(d.vof().cpu().numpy(), c, 1.0, "c")
    _assert_close(d.energy().cpu().numpy(), e, 0.0, "e")


def test_leveque_full_size_single_step(pc):
    """The 128^3 LeVeque workload: one full step, every cell compared."""
    wl = W.leveque_3d(128)
    spec, cfg = _specs(pc, wl)
    d = _domain(pc, spec, wl)
    st = d.step(wl.dt, wl.u_scale(0), stats=True)
    c, e, st_ref = oracle.step(cfg, wl.c, wl.e, wl.u, wl.v, wl.w, None, wl.dt, wl.u_scale(0), 0)
    _assert_close(d.vof().cpu().numpy(), c, 1.0, "c")
    _assert_close(d.energy().cpu().numpy(), e, 0.0, "e")
    assert st["vol"] == pytest.approx(st_ref["vol"], rel=1e-13)
    assert st["energy"] == pytest.approx(st_ref["energy"], rel=1e-13)


@pytest.mark.parametrize("normal", [0, 1, 2])
def test_normal_methods_and_sweep_orders(pc, normal):
    wl = W.random_drops_3d(n=20, ndrops=4, seed=44, rmin=1.5, rmax=3.5)
    spec, cfg = _specs(pc, wl, normal=normal, bc=(0, 1, 0))
    d = _domain(pc, spec, wl)
    d.step_index = 4  # order y, z, x
    d.step(wl.dt, -0.7)
    c, e, _ = oracle.step(cfg, wl.c, wl.e, wl.u, wl.v, wl.w, None, wl.dt, -0.7, 4)
    _assert_close(d.vof().cpu().numpy(), c, 1.0, "c")
    _assert_close(d.energy().cpu().numpy(), e, 0.0, "e")


# ------------------------------------------------------------------ edge cases
def test_degenerate_grids(pc):
    rng = np.random.default_rng(5)
    # a single cell line in 3D, a 1-cell-wide 2D strip and a grid smaller than a block
    for shape, nd in (((1, 1, 9), 3), ((1, 1, 7), 2), ((3, 5, 4), 3), ((1, 5, 130), 2)):
        c = np.clip(rng.uniform(-0.5, 1.5, size=shape), 0, 1)
        e = rng.uniform(0.5, 2.0, size=shape)
        nz, ny, nx = shape
        u = np.full((nz, ny, nx + 1), 0.3)
        v = np.full((nz, ny + 1, nx), -0.2)
        w = np.full((nz + 1, ny, nx), 0.1) if nd == 3 else None
        wl = W.Workload("tiny", shape, 1.0 / nx, nd, (0, 0, 0), 3.0, 1.0, 1.0, 1.0, c, e, u, v, w,
                        None, 1.0 / nx, 1)
        spec, cfg = _specs(pc, wl)
        d = _domain(pc, spec, wl)
        d.step(wl.dt, 1.0)
        cr, er, _ = oracle.step(cfg, c, e, u, v, w, None, wl.dt, 1.0, 0)
        _assert_close(d.vof().cpu().numpy(), cr, 1.0, f"{shape} c")
        _assert_close(d.energy().cpu().numpy(), er, 0.0, f"{shape} e")


def test_zero_velocity_and_zero_dt_leave_the_state_unchanged(pc):
    wl = W.random_drops_3d(n=16, ndrops=3, seed=45, rmin=1.5, rmax=3.0)
    spec, _ = _specs(pc, wl)
    d = _domain(pc, spec, wl)
    d.step(0.0, 1.0)
    d.step(wl.dt, 0.0)
    assert np.array_equal(d.vof().cpu().numpy(), wl.c)
    assert np.array_equal(d.energy().cpu().numpy(), wl.e)


def test_errors_are_reported(pc, torch_cuda):
    wl = W.random_drops_3d(n=12, ndrops=2, seed=46, rmin=1.5, rmax=2.5)
    spec, _ = _specs(pc, wl)
    d = pc.Domain(spec)
    with pytest.raises(pc.PcvofError) as ex:
        d.step(wl.dt)
    assert ex.value.code == -7
    bad = wl.c.copy()
    bad[0, 0, 0] = 1.5
    with pytest.raises(pc.PcvofError) as ex:
        d.set_vof(bad)
    assert ex.value.code == -4
    bad[0, 0, 0] = np.nan
    with pytest.raises(pc.PcvofError) as ex:
        d.set_vof(bad)
    assert ex.value.code == -3
    d.set_vof(wl.c)
    d.set_energy(wl.e)
    u = wl.u.copy()
    u[0, 0, -1] += 1.0  # periodic faces must agree
    with pytest.raises(pc.PcvofError) as ex:
        d.set_velocity(u, wl.v, wl.w)
    assert ex.value.code == -1
    d.set_velocity(wl.u, wl.v, wl.w)
    with pytest.raises(pc.PcvofError) as ex:
        d.step(wl.dt * 2.0)  # CFL 0.6 > 0.5
    assert ex.value.code == -2
    with pytest.raises(pc.PcvofError) as ex:
        d.phase_change(wl.dt)
    assert ex.value.code == -7
    d.step(wl.dt)  # still usable


def test_runs_are_bitwise_reproducible_and_resumable(pc):
    wl = W.random_drops_3d(n=20, ndrops=4, seed=47, rmin=1.5, rmax=3.5, mdot=0.2)
    spec, _ = _specs(pc, wl)
    runs = []
    for _ in range(2):
        d = _domain(pc, spec, wl, wl.mdot)
        for _ in range(4):
            d.step(wl.dt)
        runs.append((d.vof().cpu().numpy(), d.energy().cpu().numpy()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    # checkpoint after 2 steps, resume in a fresh domain
    d = _domain(pc, spec, wl, wl.mdot)
    d.step(wl.dt)
    d.step(wl.dt)
    ck = (d.vof().clone(), d.energy().clone(), d.step_index)
    r = pc.Domain(spec)
    r.set_vof(ck[0])
    r.set_energy(ck[1])
    r.set_velocity(wl.u, wl.v, wl.w)
    r.set_mass_flux(wl.mdot)
    r.step_index = ck[2]
    r.step(wl.dt)
    r.step(wl.dt)
    assert np.array_equal(r.vof().cpu().numpy(), runs[0][0])
    assert np.array_equal(r.energy().cpu().numpy(), runs[0][1])


def test_temperature_round_trip(pc):
    wl = W.random_drops_3d(n=12, ndrops=2, seed=48, rmin=1.5, rmax=2.5)
    spec, _ = _specs(pc, wl)
    d = pc.Domain(spec)
    d.set_vof(wl.c)
    T = np.random.default_rng(1).uniform(0.5, 3.0, size=wl.shape)
    d.set_temperature(T)
    cp = wl.cp_l * wl.c + wl.cp_g * (1 - wl.c)
    assert np.array_equal(d.energy().cpu().numpy(), cp * T)
    assert np.max(np.abs(d.temperature().cpu().numpy() - T)) <= 4e-16 * 3.0


def test_profiling_times_the_selected_classes(pc):
    wl = W.random_drops_3d(n=16, ndrops=3, seed=49, rmin=1.5, rmax=3.0)
    spec, _ = _specs(pc, wl)
    d = _domain(pc, spec, wl)
    d.set_profiling(["sweep_x", "checksum"])
    d.steps(3, wl.dt)
    p = d.profile()
    assert p["sweep_x"]["launches"] == 3 and p["checksum"]["launches"] == 3
    assert all(p[k]["launches"] == 0 for k in ("sweep_y", "sweep_z", "phase"))
    assert p["sweep_x"]["ms"] > 0.0
    d.set_profiling(True)
    d.steps(2, wl.dt)
    p = d.profile()
    assert p["sweep_x"]["launches"] == 2 and p["sweep_y"]["launches"] == 2
    d.set_profiling(False)
    d.step(wl.dt)
    assert d.profile()["sweep_z"]["launches"] == 2  # kept, not accumulated
    with pytest.raises(pc.PcvofError) as ex:
        pc.check(pc.lib().pcvof_set_profiling(d._h, 1 << 5))
    assert ex.value.code == -1


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1)])
def test_wide_rows_every_cell_mixed(pc, bc):
    """Rows of 1100 cells split into several x ranges (first faces inside a row, a ragged
    last range, the chunk past a range's end), every face with a mixed donor."""
    wl = W.wide_mixed_3d()
    wl.bc = bc
    spec, cfg = _specs(pc, wl)
    d = _domain(pc, spec, wl)
    c, e = wl.c, wl.e
    for k in range(2):
        d.step(wl.dt)
        c, e, _ = oracle.step(cfg, c, e, wl.u, wl.v, wl.w, None, wl.dt, 1.0, k)
    _assert_close(d.vof().cpu().numpy(), c, 1.0, "c")
    _assert_close(d.energy().cpu().numpy(), e, float(np.max(np.abs(wl.e))), "e")


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1)])
def test_every_cell_mixed(pc, bc):
    """A field where every cell is mixed: every face needs the donor geometry, which
    overflows the sweep blocks' LDS flux tables into the global face array."""
    rng = np.random.default_rng(51)
    wl = W.random_drops_3d(n=40, ndrops=3, seed=52, rmin=2.0, rmax=4.0)
    wl.bc = bc
    wl.c = rng.uniform(0.05, 0.95, size=wl.shape)
    wl.e = wl.c * wl.cp_l * 0.7 + (1 - wl.c) * wl.cp_g * 0.3
    spec, cfg = _specs(pc, wl)
    d = _domain(pc, spec, wl)
    c, e = wl.c, wl.e
    for k in range(2):
        d.step(wl.dt)
        c, e, _ = oracle.step(cfg, c, e, wl.u, wl.v, wl.w, None, wl.dt, 1.0, k)
    _assert_close(d.vof().cpu().numpy(), c, 1.0, "c")
    _assert_close(d.energy().cpu().numpy(), e, float(np.max(np.abs(wl.e))), "e")
