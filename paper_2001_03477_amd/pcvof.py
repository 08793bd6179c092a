"""Python binding of the pcvof C-ABI (include/pcvof.h): argument marshalling only.

Every step of the advection runs in the HIP library ``libpcvof.so``; torch provides
the device workspace and the stream. Loading fails loudly when the library is
missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcvof.so")

PCVOF_MEM_HOST, PCVOF_MEM_DEVICE = 0, 1
BC_PERIODIC, BC_OUTFLOW = 0, 1
NORMAL_YOUNGS, NORMAL_MYC, NORMAL_CC = 0, 1, 2

STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_CFL", -3: "ERR_NONFINITE", -4: "ERR_BOUNDS",
          -5: "ERR_WORKSPACE", -6: "ERR_HIP", -7: "ERR_STATE"}

EXPORTS = (
    "pcvof_workspace_bytes", "pcvof_create", "pcvof_destroy", "pcvof_set_vof", "pcvof_set_energy",
    "pcvof_set_temperature", "pcvof_set_velocity", "pcvof_set_mass_flux", "pcvof_advect_step",
    "pcvof_begin_step", "pcvof_sweep", "pcvof_phase_change", "pcvof_end_step", "pcvof_get_vof",
    "pcvof_get_energy", "pcvof_get_temperature", "pcvof_get_step", "pcvof_set_step",
    "pcvof_last_error", "pcvof_geom_volume", "pcvof_geom_alpha", "pcvof_geom_slab",
    "pcvof_geom_normal", "pcvof_geom_weno5", "pcvof_advect_steps", "pcvof_set_profiling",
    "pcvof_get_profile", "pcvof_batch_workspace_bytes", "pcvof_batch_create", "pcvof_batch_destroy",
    "pcvof_batch_domain", "pcvof_batch_advect_step", "pcvof_batch_get_step", "pcvof_batch_set_tiles",
    "pcvof_batch_get_tiles", "pcvof_batch_autotune", "pcvof_compute_mass_flux",
    "pcvof_extension_workspace_bytes", "pcvof_extend_velocity", "pcvof_diffusion_workspace_bytes",
    "pcvof_diffuse", "pcvof_diffuse_static",
)

PROF_NAMES = ("sweep_x", "sweep_y", "sweep_z", "phase", "checksum")


class PcvofError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("h", C.c_double), ("bc", C.c_int * 3)]


class Params(C.Structure):
    _fields_ = [("cp_l", C.c_double), ("cp_g", C.c_double), ("rho_l", C.c_double),
                ("T_gamma", C.c_double), ("eps_mixed", C.c_double), ("weno_eps", C.c_double),
                ("cfl_max", C.c_double), ("normal", C.c_int), ("precision", C.c_int),
                ("energy_flux", C.c_int), ("split", C.c_int)]


STAT_NAMES = ("vol", "energy", "vol_clip", "energy_clip", "vol_phase", "energy_phase",
              "vol_bnd_out", "energy_bnd_out", "vol_src", "energy_src", "max_cfl")


class Stats(C.Structure):
    _fields_ = [(n, C.c_double) for n in STAT_NAMES]

    def as_dict(self):
        return {n: getattr(self, n) for n in STAT_NAMES}


class ExtInfo(C.Structure):
    _fields_ = [("unknowns", C.c_long), ("iterations", C.c_int), ("rel_residual", C.c_double)]

    def as_dict(self):
        return {"unknowns": self.unknowns, "iterations": self.iterations, "rel_residual": self.rel_residual}


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * len(PROF_NAMES)), ("launches", C.c_long * len(PROF_NAMES))]

    def as_dict(self):
        return {n: {"ms": self.ms[i], "launches": self.launches[i]} for i, n in enumerate(PROF_NAMES)}


_lib = None
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2001_03477_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        L.pcvof_workspace_bytes.restype = C.c_size_t
        L.pcvof_workspace_bytes.argtypes = [C.POINTER(Grid), C.POINTER(Params)]
        L.pcvof_create.argtypes = [C.POINTER(Grid), C.POINTER(Params), _vp, C.c_size_t, _vp,
                                   C.POINTER(_vp)]
        L.pcvof_destroy.argtypes = [_vp]
        for nm in ("pcvof_set_vof", "pcvof_set_energy", "pcvof_set_temperature",
                   "pcvof_set_mass_flux", "pcvof_get_vof", "pcvof_get_energy",
                   "pcvof_get_temperature"):
            getattr(L, nm).argtypes = [_vp, _vp, C.c_int]
        L.pcvof_set_velocity.argtypes = [_vp, _vp, _vp, _vp, C.c_int]
        L.pcvof_advect_step.argtypes = [_vp, C.c_double, C.c_double, C.POINTER(Stats)]
        L.pcvof_begin_step.argtypes = [_vp]
        L.pcvof_sweep.argtypes = [_vp, C.c_int, C.c_double, C.c_double]
        L.pcvof_phase_change.argtypes = [_vp, C.c_double]
        L.pcvof_end_step.argtypes = [_vp, C.POINTER(Stats)]
        L.pcvof_get_step.argtypes = [_vp, C.POINTER(C.c_long)]
        L.pcvof_set_step.argtypes = [_vp, C.c_long]
        L.pcvof_last_error.restype = C.c_char_p
        L.pcvof_last_error.argtypes = []
        L.pcvof_geom_volume.argtypes = [C.c_int, _vp, _vp, _vp, _vp]
        L.pcvof_geom_alpha.argtypes = [C.c_int, _vp, _vp, _vp, _vp]
        L.pcvof_geom_slab.argtypes = [C.c_int, _vp, _vp, _vp, _vp, _vp, _vp]
        L.pcvof_geom_normal.argtypes = [C.c_int, _vp, C.c_int, _vp, _vp]
        L.pcvof_geom_weno5.argtypes = [C.c_int, _vp, C.c_double, _vp, _vp]
        L.pcvof_advect_steps.argtypes = [_vp, C.c_int, C.c_double, _vp, C.POINTER(Stats)]
        L.pcvof_set_profiling.argtypes = [_vp, C.c_int]
        L.pcvof_get_profile.argtypes = [_vp, C.POINTER(Profile)]
        L.pcvof_batch_workspace_bytes.restype = C.c_size_t
        L.pcvof_batch_workspace_bytes.argtypes = [C.c_int, C.POINTER(Grid), C.POINTER(Params)]
        L.pcvof_batch_create.argtypes = [C.c_int, C.POINTER(Grid), C.POINTER(Params), _vp, C.c_size_t,
                                         _vp, C.POINTER(_vp)]
        L.pcvof_batch_destroy.argtypes = [_vp]
        L.pcvof_batch_domain.argtypes = [_vp, C.c_int, C.POINTER(_vp)]
        L.pcvof_batch_advect_step.argtypes = [_vp, _vp, C.c_int, _vp]
        L.pcvof_batch_get_step.argtypes = [_vp, C.POINTER(C.c_long)]
        L.pcvof_batch_set_tiles.argtypes = [_vp, _vp]
        L.pcvof_batch_get_tiles.argtypes = [_vp, _vp, _vp]
        L.pcvof_batch_autotune.argtypes = [_vp, _vp, C.c_int, _vp]
        L.pcvof_compute_mass_flux.argtypes = [_vp, C.c_double, C.c_double, C.c_double, _vp, _vp, C.c_int]
        L.pcvof_extension_workspace_bytes.restype = C.c_size_t
        L.pcvof_extension_workspace_bytes.argtypes = [_vp]
        L.pcvof_extend_velocity.argtypes = [_vp, C.c_double, C.c_double, C.c_int, _vp, C.c_size_t, _vp, _vp,
                                            _vp, C.c_int, C.POINTER(ExtInfo)]
        L.pcvof_diffusion_workspace_bytes.restype = C.c_size_t
        L.pcvof_diffusion_workspace_bytes.argtypes = [_vp]
        L.pcvof_diffuse.argtypes = [_vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, _vp, C.c_size_t,
                                    _vp, C.c_int, C.POINTER(ExtInfo)]
        L.pcvof_diffuse_static.argtypes = [_vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, _vp,
                                           C.c_int, C.POINTER(ExtInfo)]
        for nm in EXPORTS:
            f = getattr(L, nm)
            if nm not in ("pcvof_workspace_bytes", "pcvof_last_error", "pcvof_batch_workspace_bytes",
                          "pcvof_extension_workspace_bytes", "pcvof_diffusion_workspace_bytes"):
                f.restype = C.c_int
        _lib = L
    return _lib


def check(rc: int):
    if rc != 0:
        raise PcvofError(rc, lib().pcvof_last_error().decode())


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


PRECISIONS = {"fp64": 0, "mixed": 1}
ENERGY_FLUXES = {"conservative": 0, "nonconservative": 1}  # section 3.4.1: eq. disc_et_adv / disc_et_adv_noncons
SPLITS = {"wy": 0, "le": 1}  # section 3.3: Weymouth-Yue split / Lagrangian-explicit sweeps of Li (CIAM)


@dataclass
class DomainSpec:
    shape: tuple              # (nz, ny, nx); nz == 1 for 2D
    h: float
    ndim: int = 3
    bc: tuple = (0, 0, 0)     # per axis x, y, z
    cp_l: float = 1.0
    cp_g: float = 1.0
    rho_l: float = 1.0
    T_gamma: float = 1.0
    eps_mixed: float = 1e-12
    weno_eps: float = 1e-6
    cfl_max: float = 0.5
    normal: int = NORMAL_MYC
    precision: str = "fp64"   # "fp64" or "mixed"
    energy_flux: str = "conservative"  # or "nonconservative" (ablation)
    split: str = "wy"         # Weymouth-Yue, or "le": Lagrangian-explicit sweeps of Li (ablation)

    def grid(self) -> Grid:
        nz, ny, nx = self.shape
        g = Grid(self.ndim, nx, ny, nz, self.h)
        for a in range(3):
            g.bc[a] = int(self.bc[a])
        return g

    def params(self) -> Params:
        return Params(self.cp_l, self.cp_g, self.rho_l, self.T_gamma, self.eps_mixed,
                      self.weno_eps, self.cfl_max, int(self.normal), PRECISIONS[self.precision],
                      ENERGY_FLUXES[self.energy_flux], SPLITS[self.split])


def workspace_bytes(spec: DomainSpec) -> int:
    g, p = spec.grid(), spec.params()
    n = lib().pcvof_workspace_bytes(C.byref(g), C.byref(p))
    if n == 0:
        raise PcvofError(-1, "invalid grid or params")
    return int(n)


class Domain:
    """One advected domain bound to a torch-owned device workspace and stream."""

    def __init__(self, spec: DomainSpec, device="cuda", stream=None):
        import torch
        self.spec = spec
        self.device = torch.device(device)
        nbytes = workspace_bytes(spec)
        # torch's caching allocator returns 256-byte (or better) aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream
        self._h = _vp()
        g, p = spec.grid(), spec.params()
        check(lib().pcvof_create(C.byref(g), C.byref(p), self.workspace.data_ptr(), nbytes,
                                 _stream_ptr(stream), C.byref(self._h)))

    # -- helpers
    @property
    def ncell(self) -> int:
        return int(np.prod(self.spec.shape))

    def _dev(self, a):
        import torch
        t = torch.as_tensor(a, dtype=torch.float64)
        if t.device != self.device:
            t = t.to(self.device)
        return t.contiguous()

    def _set(self, fn, a):
        if a is None:
            check(fn(self._h, None, PCVOF_MEM_DEVICE))
            return
        t = self._dev(a)
        check(fn(self._h, t.data_ptr(), PCVOF_MEM_DEVICE))
        self._keep = t  # keep alive until the asynchronous copy has been enqueued and run

    def set_vof(self, c):
        self._set(lib().pcvof_set_vof, c)

    def set_energy(self, e):
        self._set(lib().pcvof_set_energy, e)

    def set_temperature(self, T):
        self._set(lib().pcvof_set_temperature, T)

    def set_mass_flux(self, mdot):
        self._set(lib().pcvof_set_mass_flux, mdot)

    def set_velocity(self, u, v, w=None):
        tu, tv = self._dev(u), self._dev(v)
        tw = self._dev(w) if w is not None else None
        check(lib().pcvof_set_velocity(self._h, tu.data_ptr(), tv.data_ptr(),
                                       tw.data_ptr() if tw is not None else None,
                                       PCVOF_MEM_DEVICE))
        self._keep = (tu, tv, tw)

    def _get(self, fn):
        import torch
        out = torch.empty(self.spec.shape, dtype=torch.float64, device=self.device)
        check(fn(self._h, out.data_ptr(), PCVOF_MEM_DEVICE))
        return out

    def vof(self):
        return self._get(lib().pcvof_get_vof)

    def energy(self):
        return self._get(lib().pcvof_get_energy)

    def temperature(self):
        return self._get(lib().pcvof_get_temperature)

    def extend_velocity(self, rho_g: float, rel_tol: float = 1e-13, max_iter: int = 5000,
                        corrections: bool = False):
        """Liquid-velocity extension (section 3.3.1): the stored velocity becomes
        u + u~. Returns (info dict, (du, dv, dw) device tensors or None)."""
        import torch
        nbytes = lib().pcvof_extension_workspace_bytes(self._h)
        ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=self.device)
        outs = [None, None, None]
        if corrections:
            nz, ny, nx = self.spec.shape
            shapes = [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]
            for a in range(self.spec.ndim):
                outs[a] = torch.empty(shapes[a], dtype=torch.float64, device=self.device)
        info = ExtInfo()
        check(lib().pcvof_extend_velocity(self._h, float(rho_g), float(rel_tol), int(max_iter), ws.data_ptr(),
                                          int(nbytes), *[o.data_ptr() if o is not None else None for o in outs],
                                          PCVOF_MEM_DEVICE, C.byref(info)))
        return info.as_dict(), (tuple(outs) if corrections else None)

    def diffuse(self, dt: float, k_l: float, k_g: float, rel_tol: float = 1e-13, max_iter: int = 5000,
                temperature: bool = False):
        """Implicit energy diffusion with T_Gamma at the interface (section 3.4.2): the
        energy becomes C_p(c) T^{n+1}. Returns (info dict, T^{n+1} device tensor or None)."""
        import torch
        nbytes = lib().pcvof_diffusion_workspace_bytes(self._h)
        ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=self.device)
        T = torch.empty(self.spec.shape, dtype=torch.float64, device=self.device) if temperature else None
        info = ExtInfo()
        check(lib().pcvof_diffuse(self._h, float(dt), float(k_l), float(k_g), float(rel_tol), int(max_iter),
                                  ws.data_ptr(), int(nbytes), T.data_ptr() if T is not None else None,
                                  PCVOF_MEM_DEVICE, C.byref(info)))
        return info.as_dict(), T

    def diffuse_static(self, dt: float, k_l: float, k_g: float, rel_tol: float = 1e-13, max_iter: int = 5000,
                       temperature: bool = False):
        """pcvof_diffuse_static: the same diffusion step as diffuse(), with the library's
        static device scratch instead of a workspace (nothing is allocated for it)."""
        import torch
        T = torch.empty(self.spec.shape, dtype=torch.float64, device=self.device) if temperature else None
        info = ExtInfo()
        check(lib().pcvof_diffuse_static(self._h, float(dt), float(k_l), float(k_g), float(rel_tol), int(max_iter),
                                         T.data_ptr() if T is not None else None, PCVOF_MEM_DEVICE,
                                         C.byref(info)))
        return info.as_dict(), T

    def compute_mass_flux(self, k_l: float, k_g: float, h_fg: float, distances: bool = False):
        """m'' from the PLIC reconstruction of the current state (section 3.2); it becomes
        the domain's mass flux. Returns (mdot, dist or None) as device tensors."""
        import torch
        md = torch.empty(self.spec.shape, dtype=torch.float64, device=self.device)
        dist = torch.empty_like(md) if distances else None
        check(lib().pcvof_compute_mass_flux(self._h, float(k_l), float(k_g), float(h_fg), md.data_ptr(),
                                            dist.data_ptr() if dist is not None else None,
                                            PCVOF_MEM_DEVICE))
        return md, dist

    # -- stepping
    def step(self, dt: float, u_scale: float = 1.0, stats: bool = False):
        st = Stats() if stats else None
        check(lib().pcvof_advect_step(self._h, float(dt), float(u_scale),
                                      C.byref(st) if st is not None else None))
        return st.as_dict() if st is not None else None

    def steps(self, n: int, dt: float, u_scale=None, stats: bool = False):
        """n steps from one host call; u_scale is None or a sequence of n scales."""
        st = Stats() if stats else None
        arr = None
        if u_scale is not None:
            arr = np.ascontiguousarray(np.asarray(u_scale, dtype=np.float64))
            assert arr.shape == (n,)
        check(lib().pcvof_advect_steps(self._h, int(n), float(dt),
                                       arr.ctypes.data if arr is not None else None,
                                       C.byref(st) if st is not None else None))
        return st.as_dict() if st is not None else None

    def set_profiling(self, on=True):
        """Times the kernels of the selected classes with HIP events: True = every class,
        False = off, or an iterable of class names from PROF_NAMES."""
        if on is True:
            mask = (1 << len(PROF_NAMES)) - 1
        elif on is False or on is None:
            mask = 0
        else:
            mask = 0
            for name in on:
                mask |= 1 << PROF_NAMES.index(name)
        check(lib().pcvof_set_profiling(self._h, mask))

    def profile(self):
        p = Profile()
        check(lib().pcvof_get_profile(self._h, C.byref(p)))
        return p.as_dict()

    def begin_step(self):
        check(lib().pcvof_begin_step(self._h))

    def sweep(self, axis: int, dt: float, u_scale: float = 1.0):
        check(lib().pcvof_sweep(self._h, int(axis), float(dt), float(u_scale)))

    def phase_change(self, dt: float):
        check(lib().pcvof_phase_change(self._h, float(dt)))

    def end_step(self, stats: bool = True):
        st = Stats() if stats else None
        check(lib().pcvof_end_step(self._h, C.byref(st) if st is not None else None))
        return st.as_dict() if st is not None else None

    @property
    def step_index(self) -> int:
        v = C.c_long()
        check(lib().pcvof_get_step(self._h, C.byref(v)))
        return v.value

    @step_index.setter
    def step_index(self, n: int):
        check(lib().pcvof_set_step(self._h, int(n)))

    @classmethod
    def _view(cls, spec: DomainSpec, handle, device, stream):
        """A domain owned by a Batch (no workspace or lifetime of its own)."""
        import torch
        d = cls.__new__(cls)
        d.spec = spec
        d.device = torch.device(device)
        d.workspace = None
        d.stream = stream
        d._h = handle
        d._view_of = True
        return d

    def close(self):
        if self._h and not getattr(self, "_view_of", False):
            check(lib().pcvof_destroy(self._h))
        self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent domains advected together: one fused launch per direction sweep
    over the tiles of all domains, optionally replayed from captured HIP graphs."""

    def __init__(self, specs, device="cuda", stream=None):
        import torch
        self.specs = list(specs)
        nd = len(self.specs)
        grids = (Grid * nd)(*[s.grid() for s in self.specs])
        params = (Params * nd)(*[s.params() for s in self.specs])
        nbytes = int(lib().pcvof_batch_workspace_bytes(nd, grids, params))
        if nbytes == 0:
            raise PcvofError(-1, "invalid grids or params, or domains differ in ndim or precision")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self._b = _vp()
        check(lib().pcvof_batch_create(nd, grids, params, self.workspace.data_ptr(), nbytes,
                                       _stream_ptr(stream), C.byref(self._b)))
        self.domains = []
        for i, s in enumerate(self.specs):
            h = _vp()
            check(lib().pcvof_batch_domain(self._b, i, C.byref(h)))
            self.domains.append(Domain._view(s, h, device, stream))

    def step(self, dt, use_graph: bool = False, stats: bool = False):
        """One step of every domain with its own dt (sequence of len(domains))."""
        arr = np.ascontiguousarray(np.asarray(dt, dtype=np.float64))
        assert arr.shape == (len(self.domains),)
        st = (Stats * len(self.domains))() if stats else None
        check(lib().pcvof_batch_advect_step(self._b, arr.ctypes.data, 1 if use_graph else 0,
                                            C.cast(st, _vp) if st is not None else None))
        return [x.as_dict() for x in st] if st is not None else None

    @property
    def step_index(self) -> int:
        v = C.c_long()
        check(lib().pcvof_batch_get_step(self._b, C.byref(v)))
        return v.value

    def set_tiles(self, chunk):
        """Rows per x wavefront chunk[0] in (0, 1, 2, 4, 8) and column chunk of the y / z sweeps
        chunk[1], chunk[2] in (0, 8, 16, 32, 64); 0 keeps each domain's single-domain rule."""
        ch = (C.c_int * 3)(*chunk)
        check(lib().pcvof_batch_set_tiles(self._b, C.cast(ch, _vp)))

    def tiles(self):
        ch, nt = (C.c_int * 3)(), (C.c_int * 3)()
        check(lib().pcvof_batch_get_tiles(self._b, C.cast(ch, _vp), C.cast(nt, _vp)))
        return {"chunk": list(ch), "ntiles": list(nt)}

    def autotune(self, dt, reps: int = 3):
        arr = np.ascontiguousarray(np.asarray(dt, dtype=np.float64))
        ch = (C.c_int * 3)()
        check(lib().pcvof_batch_autotune(self._b, arr.ctypes.data, int(reps), C.cast(ch, _vp)))
        return {"chunk": list(ch)}

    def close(self):
        for d in getattr(self, "domains", []):
            d._h = _vp()
        if getattr(self, "_b", None):
            check(lib().pcvof_batch_destroy(self._b))
            self._b = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ batched geometry
def geom_volume(m, alpha):
    import torch
    out = torch.empty_like(alpha)
    check(lib().pcvof_geom_volume(alpha.numel(), m.data_ptr(), alpha.data_ptr(), out.data_ptr(),
                                  _stream_ptr()))
    return out


def geom_alpha(m, c):
    import torch
    out = torch.empty_like(c)
    check(lib().pcvof_geom_alpha(c.numel(), m.data_ptr(), c.data_ptr(), out.data_ptr(),
                                 _stream_ptr()))
    return out


def geom_slab(m, alpha, axis, lam):
    import torch
    out = torch.empty_like(alpha)
    check(lib().pcvof_geom_slab(alpha.numel(), m.data_ptr(), alpha.data_ptr(), axis.data_ptr(),
                                lam.data_ptr(), out.data_ptr(), _stream_ptr()))
    return out


def geom_normal(c27, method: int):
    import torch
    n = c27.shape[0]
    out = torch.empty((n, 3), dtype=torch.float64, device=c27.device)
    check(lib().pcvof_geom_normal(n, c27.data_ptr(), int(method), out.data_ptr(), _stream_ptr()))
    return out


def geom_weno5(v, eps: float = 1e-6):
    import torch
    n = v.shape[0]
    out = torch.empty(n, dtype=torch.float64, device=v.device)
    check(lib().pcvof_geom_weno5(n, v.data_ptr(), float(eps), out.data_ptr(), _stream_ptr()))
    return out
