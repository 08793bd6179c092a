"""Batched domains: one fused launch per sweep over the tiles of many domains (and the
captured-graph replay of those launches) computes, tile by tile, what the
single-domain launches compute, so the fields must equal the single-domain results
bitwise; the first domains are also checked against the FP64 oracle."""
import numpy as np
import pytest

import oracle
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


def _spec(pc, wl, precision="fp64"):
    return pc.DomainSpec(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                         rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal, precision=precision)


def _fill(d, wl):
    d.set_vof(wl.c)
    d.set_energy(wl.e)
    d.set_velocity(wl.u, wl.v, wl.w)
    if wl.mdot is not None:
        d.set_mass_flux(wl.mdot)


def _workloads():
    wls = W.batch_domains(nd=4, seed=71, smin=20, smax=44)
    # an outflow domain with phase change and one more periodic drop field
    extra = W.random_drops_3d(n=24, ndrops=3, seed=72, rmin=2.0, rmax=4.0, mdot=0.2)
    extra.bc = (1, 0, 1)
    wls.append(extra)
    wls.append(W.random_drops_3d(n=28, ndrops=4, seed=73, rmin=2.0, rmax=5.0))
    return wls


def _singles(pc, wls, steps, precision="fp64"):
    out = []
    for wl in wls:
        d = pc.Domain(_spec(pc, wl, precision))
        _fill(d, wl)
        st = None
        for _ in range(steps):
            st = d.step(wl.dt, stats=True)
        out.append((d.vof().cpu().numpy(), d.energy().cpu().numpy(), st))
    return out


def _batch(pc, wls, precision="fp64"):
    b = pc.Batch([_spec(pc, wl, precision) for wl in wls])
    for d, wl in zip(b.domains, wls):
        _fill(d, wl)
    return b


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_single_domains(pc, use_graph):
    wls = _workloads()
    if use_graph:  # graphs are used when no domain has a mass flux
        wls = [wl for wl in wls if wl.mdot is None]
    steps = 7  # more than one cycle of sweep orders and buffer parities
    ref = _singles(pc, wls, steps)
    b = _batch(pc, wls)
    dts = [wl.dt for wl in wls]
    st = None
    for _ in range(steps):
        st = b.step(dts, use_graph=use_graph, stats=True)
    for i, (d, (c, e, s)) in enumerate(zip(b.domains, ref)):
        assert np.array_equal(d.vof().cpu().numpy(), c), f"domain {i}: c differs"
        assert np.array_equal(d.energy().cpu().numpy(), e), f"domain {i}: e differs"
        for k in ("vol", "energy", "vol_clip", "vol_src", "vol_phase"):
            assert st[i][k] == s[k], f"domain {i}: {k}"
    assert b.step_index == steps
    b.close()


def test_batch_first_domains_match_oracle(pc):
    wls = _workloads()[:2]
    b = _batch(pc, wls)
    steps = 3
    for _ in range(steps):
        b.step([wl.dt for wl in wls])
    for d, wl in zip(b.domains, wls):
        cfg = oracle.Config(shape=wl.shape, h=wl.h, ndim=3, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                            rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal)
        c, e = wl.c, wl.e
        for k in range(steps):
            c, e, _ = oracle.step(cfg, c, e, wl.u, wl.v, wl.w, wl.mdot, wl.dt, 1.0, k)
        assert np.max(np.abs(d.vof().cpu().numpy() - c)) <= 1e-12
        assert np.max(np.abs(d.energy().cpu().numpy() - e)) <= 1e-12 * np.max(np.abs(wl.e))
    b.close()


@pytest.mark.parametrize("chunk", [(0, 8), (1, 16), (2, 32), (4, 64), (8, 0)])
def test_batch_tile_choices_give_the_same_fields(pc, chunk):
    """Rows per x wavefront and y / z column chunks (0: the single-domain rules)."""
    wls = _workloads()
    ref = _singles(pc, wls, 3)
    b = _batch(pc, wls)
    b.set_tiles(chunk=[chunk[0], chunk[1], chunk[1]])
    for _ in range(3):
        b.step([wl.dt for wl in wls], use_graph=True)
    for d, (c, e, _) in zip(b.domains, ref):
        assert np.array_equal(d.vof().cpu().numpy(), c)
        assert np.array_equal(d.energy().cpu().numpy(), e)
    b.close()


def test_batch_long_x_ranges_overflow_the_flux_tables(pc):
    """Eight rows per x wavefront over 512-cell ranges of an all-mixed 1100-cell-wide
    domain list about 4,100 faces per wavefront, far past the x sweep's LDS flux table,
    and 8-cell y / z columns list about 580 per wavefront, past theirs: the fluxes go
    through the global face array. The fields must equal the single-domain runs
    (one-row, 64-cell x ranges there; that path is checked against the oracle)."""
    wls = [W.wide_mixed_3d(), _workloads()[0]]
    ref = _singles(pc, wls, 3)
    b = _batch(pc, wls)
    b.set_tiles(chunk=[8, 8, 8])
    for _ in range(3):
        b.step([wl.dt for wl in wls])
    for d, (c, e, _) in zip(b.domains, ref):
        assert np.array_equal(d.vof().cpu().numpy(), c)
        assert np.array_equal(d.energy().cpu().numpy(), e)
    b.close()


def test_batch_autotune_keeps_the_state(pc):
    wls = _workloads()
    ref = _singles(pc, wls, 2)
    b = _batch(pc, wls)
    b.step([wl.dt for wl in wls])
    chosen = b.autotune([wl.dt for wl in wls], reps=2)
    assert chosen["chunk"][0] in (0, 1, 2, 4, 8) and all(c in (0, 8, 16, 32, 64) for c in chosen["chunk"][1:])
    b.step([wl.dt for wl in wls], use_graph=True)
    for d, (c, e, _) in zip(b.domains, ref):
        assert np.array_equal(d.vof().cpu().numpy(), c)
        assert np.array_equal(d.energy().cpu().numpy(), e)
    b.close()


def test_batch_mixed_precision_equals_single_mixed(pc):
    wls = _workloads()
    wls = [wl for wl in wls if wl.mdot is None]
    ref = _singles(pc, wls, 4, precision="mixed")
    b = _batch(pc, wls, precision="mixed")
    for _ in range(4):
        b.step([wl.dt for wl in wls], use_graph=True)
    for d, (c, e, _) in zip(b.domains, ref):
        assert np.array_equal(d.vof().cpu().numpy(), c)
        assert np.array_equal(d.energy().cpu().numpy(), e)
    b.close()


def test_batch_errors(pc):
    wls = _workloads()[:3]
    b = _batch(pc, wls)
    dts = [wl.dt for wl in wls]
    with pytest.raises(pc.PcvofError) as ex:
        b.step([dts[0] * 10.0] + dts[1:])  # CFL
    assert ex.value.code == -2
    b.domains[1].step(dts[1])  # stepping a view on its own breaks the lockstep
    with pytest.raises(pc.PcvofError) as ex:
        b.step(dts)
    assert ex.value.code == -7
    with pytest.raises(pc.PcvofError) as ex:
        b.set_tiles(chunk=[0, 12, 16])
    assert ex.value.code == -1
    with pytest.raises(pc.PcvofError) as ex:
        b.set_tiles(chunk=[16, 0, 0])  # at most 8 rows per x wavefront
    assert ex.value.code == -1
    with pytest.raises(pc.PcvofError):
        pc.Batch([_spec(pc, wls[0]), _spec(pc, wls[1], "mixed")])  # mixed precisions
    b.close()
