"""The library's mass-transfer-rate kernels (section 3.2, massflux.hip) executed on the
host: g++ compiles the unchanged kernel source with a stand-in for the HIP runtime
header (tests/host_kernels/) and AddressSanitizer / UBSan, and runs every kernel over the
exact launch grid the library uses (ceil(nx/64) x ceil(ny/4) x nz blocks of 64 x 4), on
the inputs of the GPU mass-flux tests, each buffer in an allocation of exactly the size
the library's workspace gives it.

These kernels are switched off on the GPU: their first GPU run, in an earlier state of
the sources that was not kept, ended in a memory fault whose cause was never found.
This test shows on the CPU that the kept kernel bodies stay inside every buffer on
those inputs and agree with the oracle (m'' within 1e-12 of its largest value, the
same cells with a distance, distances within 1e-12 h)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2001_03477_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host_kernels")


def _temperatures(wl, seed, T_gamma):
    """The temperature fields of the GPU mass-flux tests (smooth and random parts)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = wl.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return T_gamma + 0.3 * np.sin(0.4 * x + 0.2 * y) + 0.2 * np.cos(0.3 * z) + 0.05 * rng.uniform(-1, 1, wl.shape)


def _cases():
    out = []
    for bc in [(0, 0, 0), (1, 1, 1), (0, 1, 0)]:
        out.append((W.random_drops_3d(n=28, ndrops=6, seed=93, rmin=1.5, rmax=5.0), bc, 1, 1.2, 0,
                    (0.6, 0.025, 2.3)))
    for normal in (0, 2):
        out.append((W.random_drops_3d(n=23, ndrops=4, seed=94, rmin=1.5, rmax=4.0), (1, 0, 1), normal, 1.2, 1,
                    (0.6, 0.025, 2.3)))
    out.append((W.circle_2d(64), (0, 0, 0), 1, 1.2, 2, (0.6, 0.025, 2.3)))
    out.append((W.random_drops_3d(n=24, ndrops=5, seed=95, rmin=2.0, rmax=4.0), (0, 0, 0), 1, 0.9, 3,
                (0.6, 0.025, 2.3e3)))
    return out


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path_factory.mktemp("mf") / "mass_flux_harness")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-ffp-contract=off", "-w", f"-I{SRC}", "-o", exe, os.path.join(SRC, "mass_flux_harness.cpp"),
                    "-lm"], check=True)
    return exe


@pytest.mark.parametrize("k", range(7))
def test_mass_flux_kernels_on_the_host(harness, tmp_path, k):
    wl, bc, normal, T_gamma, seed, kk = _cases()[k]
    T = _temperatures(wl, seed, T_gamma)
    e = (wl.cp_l * wl.c + wl.cp_g * (1.0 - wl.c)) * T
    nz, ny, nx = wl.shape
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as fh:
        fh.write(np.array([wl.ndim, nx, ny, nz, *bc, normal], dtype=np.int32).tobytes())
        fh.write(np.array([wl.cp_l, wl.cp_g, T_gamma, wl.h, *kk, 0.0]).tobytes())
        fh.write(np.ascontiguousarray(wl.c, dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(e, dtype=np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([harness, str(fin), str(fout)], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    out = np.fromfile(fout, dtype=np.float64)
    md, dist = out[: wl.c.size].reshape(wl.shape), out[wl.c.size:].reshape(wl.shape)
    cfg = oracle.Config(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=bc, cp_l=wl.cp_l, cp_g=wl.cp_g, T_gamma=T_gamma,
                        normal=normal)
    md_ref, dist_ref = oracle.mass_flux(cfg, wl.c, e / (wl.cp_l * wl.c + wl.cp_g * (1.0 - wl.c)), *kk)
    assert np.array_equal(np.isnan(dist), np.isnan(dist_ref))
    ok = ~np.isnan(dist_ref)
    assert ok.sum() > 0
    assert np.max(np.abs(dist[ok] - dist_ref[ok])) <= 1e-12 * wl.h
    assert np.max(np.abs(md - md_ref)) <= 1e-12 * max(float(np.max(np.abs(md_ref))), 1e-300)
