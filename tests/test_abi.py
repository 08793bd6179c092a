"""The C-ABI library loads and exports every entry point include/pcvof.h declares,
and its host-side argument checks behave as documented (no GPU calls)."""
import ctypes as C
import os
import re

import pytest

from paper_2001_03477_amd import pcvof

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pcvof.h")).read()
    return sorted(set(re.findall(r"\b(pcvof_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = pcvof.lib()
    names = _declared()
    assert len(names) >= 20
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(pcvof.EXPORTS)


def _spec(**kw):
    base = dict(shape=(8, 12, 20), h=0.05, ndim=3, bc=(0, 1, 0), cp_l=4.0, cp_g=1.0)
    base.update(kw)
    return pcvof.DomainSpec(**base)


def test_workspace_bytes_and_validation():
    n = pcvof.workspace_bytes(_spec())
    cells = 8 * 12 * 20
    assert n >= cells * (4 + 1 + 5 + 1) * 8  # state, frozen fields, mass flux, reconstruction
    assert n % 256 == 0
    with pytest.raises(pcvof.PcvofError):
        pcvof.workspace_bytes(_spec(ndim=2))                 # 2D needs nz == 1
    with pytest.raises(pcvof.PcvofError):
        pcvof.workspace_bytes(_spec(h=-1.0))
    with pytest.raises(pcvof.PcvofError):
        pcvof.workspace_bytes(_spec(cp_g=0.0))
    with pytest.raises(pcvof.PcvofError):
        pcvof.workspace_bytes(_spec(normal=7))
    with pytest.raises(pcvof.PcvofError):
        pcvof.workspace_bytes(_spec(bc=(0, 2, 0)))
    n2 = pcvof.workspace_bytes(_spec(shape=(1, 33, 65), ndim=2))
    assert n2 > 33 * 65 * 8
    # mixed precision stores e_c and the face velocities in single precision
    nm = pcvof.workspace_bytes(_spec(precision="mixed"))
    faces = 8 * 12 * 21 + 8 * 13 * 20 + 9 * 12 * 20
    assert n - nm >= 4 * (cells + faces) - 4 * 256  # buffers are 256-byte aligned
    spec = _spec()
    p = spec.params()
    p.precision = 2
    assert pcvof.lib().pcvof_workspace_bytes(C.byref(spec.grid()), C.byref(p)) == 0


def test_create_checks_workspace_without_touching_the_device():
    L = pcvof.lib()
    spec = _spec()
    g, p = spec.grid(), spec.params()
    need = pcvof.workspace_bytes(spec)
    h = C.c_void_p()
    assert L.pcvof_create(C.byref(g), C.byref(p), None, need, None, C.byref(h)) == -5
    assert b"null" in L.pcvof_last_error()
    # misaligned and undersized workspaces are rejected before any device access
    assert L.pcvof_create(C.byref(g), C.byref(p), 0x1008, need, None, C.byref(h)) == -5
    assert L.pcvof_create(C.byref(g), C.byref(p), 0x10000, need - 1, None, C.byref(h)) == -5
    assert b"needs" in L.pcvof_last_error()
    assert L.pcvof_create(C.byref(g), C.byref(p), 0x10000, need, None, None) == -1
    # a valid create only records the pointers; stepping before the fields are set is a
    # state error, reported without a launch
    assert L.pcvof_create(C.byref(g), C.byref(p), 0x10000, need, None, C.byref(h)) == 0
    assert L.pcvof_begin_step(h) == -7
    assert L.pcvof_advect_step(h, C.c_double(0.1), C.c_double(1.0), None) == -7
    assert L.pcvof_sweep(h, 0, C.c_double(0.1), C.c_double(1.0)) == -7
    st = C.c_long(-1)
    assert L.pcvof_get_step(h, C.byref(st)) == 0 and st.value == 0
    assert L.pcvof_set_step(h, 5) == 0
    assert L.pcvof_get_step(h, C.byref(st)) == 0 and st.value == 5
    assert L.pcvof_set_step(h, -1) == -1
    assert L.pcvof_set_vof(h, None, 1) == -1
    assert L.pcvof_set_mass_flux(h, None, 1) == 0   # NULL switches step 2 off
    assert L.pcvof_destroy(h) == 0


def test_geometry_entry_points_reject_bad_arguments():
    L = pcvof.lib()
    assert L.pcvof_geom_volume(0, None, None, None, None) == 0      # empty batch: nothing to do
    assert L.pcvof_geom_volume(-1, None, None, None, None) == -1
    assert L.pcvof_geom_volume(4, None, None, None, None) == -1
    assert L.pcvof_geom_normal(4, 0x1000, 9, 0x2000, None) == -1
