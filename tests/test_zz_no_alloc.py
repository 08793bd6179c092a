"""The diffusion entry point that allocates nothing (pcvof_diffuse_static) against
pcvof_diffuse with a caller's workspace, through the C-ABI: two calls in a row on the
library's static scratch, the second on a smaller domain (the scratch then still holds
the first call's data), each within the parity bar of the diffusion tests (1e-12 of
max |T|) of the workspace call on the same inputs; and a domain too large for the
scratch is refused before anything runs."""
import numpy as np
import pytest

from paper_2001_03477_amd import workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def pc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_03477_amd import pcvof
    pcvof.lib()
    return pcvof


def _domain(pc, wl, bc, T_gamma=0.7):
    spec = pc.DomainSpec(shape=wl.shape, h=wl.h, ndim=3, bc=bc, cp_l=2.5, cp_g=0.25, T_gamma=T_gamma)
    d = pc.Domain(spec)
    d.set_vof(wl.c)
    rng = np.random.default_rng(11)
    T = 0.5 + rng.uniform(0.0, 1.0, size=wl.shape)
    d.set_energy((2.5 * wl.c + 0.25 * (1.0 - wl.c)) * T)
    return d


def _pair(pc, wl, bc, dt, k_l, k_g):
    ref = _domain(pc, wl, bc)
    info_ref, T_ref = ref.diffuse(dt, k_l, k_g, temperature=True)
    got = _domain(pc, wl, bc)
    info, T = got.diffuse_static(dt, k_l, k_g, temperature=True)
    T_ref, T = T_ref.cpu().numpy(), T.cpu().numpy()
    e_ref, e = ref.energy().cpu().numpy(), got.energy().cpu().numpy()
    scale = float(np.max(np.abs(T_ref)))
    assert np.max(np.abs(T - T_ref)) <= REL * scale
    assert np.max(np.abs(e - e_ref)) <= REL * float(np.max(np.abs(e_ref)))
    assert info["iterations"] == info_ref["iterations"] and info["iterations"] > 5
    return np.array_equal(T, T_ref)


def test_static_diffusion_matches_the_workspace_call_twice(pc):
    big = W.random_drops_3d(n=40, ndrops=6, seed=61, rmin=2.0, rmax=6.0)
    small = W.random_drops_3d(n=22, ndrops=3, seed=62, rmin=2.0, rmax=4.0)
    same1 = _pair(pc, big, (1, 1, 1), 2e-3, 0.7, 0.1)
    same2 = _pair(pc, small, (0, 0, 0), 3e-3, 0.5, 0.05)
    print(f"bitwise equal to the workspace call: {same1}, {same2}")


def test_static_diffusion_refuses_a_domain_beyond_its_scratch(pc):
    n = 130  # about 2.2 million cells, above the 256 MiB scratch
    spec = pc.DomainSpec(shape=(n, n, n), h=1.0 / n, cp_l=2.5, cp_g=0.25)
    d = pc.Domain(spec)
    c = np.zeros((n, n, n))
    c[:, :, : n // 2] = 1.0
    d.set_vof(c)
    d.set_energy(np.ones((n, n, n)))
    assert pc.lib().pcvof_diffusion_workspace_bytes(d._h) > (256 << 20)
    with pytest.raises(pc.PcvofError) as ex:
        d.diffuse_static(1e-3, 0.5, 0.05)
    assert ex.value.code == -5
    assert np.array_equal(d.energy().cpu().numpy(), np.ones((n, n, n)))
