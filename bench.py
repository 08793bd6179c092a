"""Benchmark of the advection step on one MI355X.

Workload (default): the 3D 512^3 periodic box with 2000 seeded droplets (radii 4-16
cells), a divergence-free random Fourier velocity at CFL 0.3, per-phase random
temperatures, the water heat-capacity ratio, m'' = 0, FP64. A step is the whole hot
path: prologue, three direction sweeps (geometric VOF fluxes + conservative WENO5
energy fluxes), checksums.

Prints one JSON line: whole-job cell-updates/s of the FP64 path over the timed steps
(inputs already resident in HBM), the roofline of the dominant kernel (the sweep;
algorithmic bytes per launch over its average duration, measured with HIP events on
the library's stream over as many steps again, right after the timed ones), the same
run in the mixed-precision mode (rate, speedup, roofline, volume drift and difference
from the FP64 fractions), the 128^3 LeVeque (with its shape error after one period of
the deformation) and 256^3 bubble workloads (with phase change, the liquid-velocity
extension and the energy diffusion) as extra keys with the energy-flux and split
ablations, and the oracle timed on the host's cores on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "VOF+energy advect cell-updates/s (FP64 vs mixed), % HBM peak, volume drift"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one sweep (FP64): per cell read c, e, e_c (8 each) and the
# dilatation flag c_c (1), write c, e (8 each); plus 8 per face velocity read. The
# first sweep of a step writes c_c and e_c instead of reading them (same count).
SWEEP_BYTES_PER_CELL = 8 + 8 + 8 + 1 + 8 + 8
SWEEP_BYTES_PER_FACE = 8
# mixed precision: e_c (4) and the face velocity (4) in single precision
SWEEP_BYTES_PER_CELL_MIXED = 8 + 8 + 4 + 1 + 8 + 8
SWEEP_BYTES_PER_FACE_MIXED = 4
CHECKED_STEPS = 20  # untimed steps with checksums for the bookkeeping residue


def workload(name):
    from paper_2001_03477_amd import workloads as W
    if name == "leveque128":
        return W.leveque_3d(128)
    if name == "leveque256":
        return W.leveque_3d(256)
    if name == "circle2d":
        return W.circle_2d(64)
    if name == "bubble256":
        return W.bubble_3d(256)
    if name == "droplets512":
        return W.droplets_3d(512)
    if name == "batch64":
        return W.batch_domains(64)
    raise SystemExit(f"unknown workload {name}")


def W_max_face(wl):
    from paper_2001_03477_amd import workloads as W
    return W.max_abs_face(wl.u, wl.v, wl.w)


def sweep_bytes(wl, axis, mixed=False):
    nz, ny, nx = wl.shape
    faces = [nz * ny * (nx + 1), nz * (ny + 1) * nx, (nz + 1) * ny * nx][axis]
    if mixed:
        return SWEEP_BYTES_PER_CELL_MIXED * wl.ncells + SWEEP_BYTES_PER_FACE_MIXED * faces
    return SWEEP_BYTES_PER_CELL * wl.ncells + SWEEP_BYTES_PER_FACE * faces


def recorded_traffic(wl, sweep_n, mixed=False):
    """HBM bytes per sweep launch (average over the axes, weighted like the timing) from
    the committed counter summary of this workload, or None when there is none, it does
    not cover the precision, or the sweep kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"sweep_{wl.name}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_json: "):
                rec = json.loads(line[len("traffic_json: "):])
    from paper_2001_03477_amd.profsum import sweep_source_hash
    if rec is None or rec.get("source_hash") != sweep_source_hash():
        return None
    per_axis = rec.get("bytes_per_launch_mixed" if mixed else "bytes_per_launch")
    if per_axis is None or any(per_axis[a] is None for a in range(wl.ndim)):
        return None
    tot = sum(per_axis[a] * sweep_n[a] for a in range(wl.ndim))
    return float(tot / sweep_n.sum())


def copy_bandwidth(torch, mib=1024, reps=10):
    """GB/s of a device-to-device copy of mib MiB (bytes read + written per second), a
    measured reference beside the specified peak."""
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        y.copy_(x)
    t1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 8 * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def run(pcvof, torch, wl, precision, steps, warmup, scales):
    """warmup + steps steps of the workload in the given precision: the timed steps
    bracketed by events on the stream, the sweep kernels timed by the library's events,
    the relative change of the total volume over the run and the final volume
    fraction."""
    spec = pcvof.DomainSpec(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc, cp_l=wl.cp_l,
                            cp_g=wl.cp_g, rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal,
                            precision=precision)
    stream = torch.cuda.current_stream()
    dom = pcvof.Domain(spec, stream=stream)
    dom.set_vof(wl.c)
    dom.set_energy(wl.e)
    dom.set_velocity(wl.u, wl.v, wl.w)
    if wl.mdot is not None:
        dom.set_mass_flux(wl.mdot)
    hv = wl.h ** wl.ndim
    vol0 = float(dom.vof().sum()) * hv
    dom.steps(warmup, wl.dt, scales[:warmup])
    torch.cuda.synchronize()
    # the timed steps: events on the stream around them, nothing inside
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record(stream)
    dom.steps(steps, wl.dt, scales[warmup:warmup + steps])
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    # sweep kernel durations: the same number of steps again, with HIP events recorded
    # by the library around each sweep launch on the stream the kernels run on (the
    # events add time between launches, so they are kept out of the timed steps)
    dom.set_profiling(["sweep_x", "sweep_y", "sweep_z"][:wl.ndim])
    dom.steps(steps, wl.dt, scales[warmup + steps:])
    prof = dom.profile()
    dom.set_profiling(False)
    sweep_ms = np.array([prof[f"sweep_{a}"]["ms"] for a in "xyz"[:wl.ndim]])
    sweep_n = np.array([prof[f"sweep_{a}"]["launches"] for a in "xyz"[:wl.ndim]])
    mixed = precision == "mixed"
    sweep_b = sum(sweep_bytes(wl, a, mixed) * sweep_n[a] for a in range(wl.ndim))
    # checked steps (untimed, with checksums): the change of total volume and energy net
    # of the reported boundary, source, clip and phase-change terms
    k0 = warmup + 2 * steps
    st = dom.step(wl.dt, wl.u_scale(k0), stats=True)
    v_prev, e_prev, e0 = st["vol"], st["energy"], abs(st["energy"])
    v_res = e_res = 0.0
    for k in range(CHECKED_STEPS):
        st = dom.step(wl.dt, wl.u_scale(k0 + 1 + k), stats=True)
        v_res += st["vol"] - v_prev - (-st["vol_bnd_out"] + st["vol_src"] + st["vol_clip"] + st["vol_phase"])
        e_res += st["energy"] - e_prev - (-st["energy_bnd_out"] + st["energy_src"] + st["energy_clip"]
                                          + st["energy_phase"])
        v_prev, e_prev = st["vol"], st["energy"]
    vol1 = st["vol"]
    c_final = dom.vof().cpu().numpy()
    del dom
    torch.cuda.empty_cache()
    return {"total_ms": total_ms, "sweep_ms": sweep_ms, "sweep_n": sweep_n, "prof": prof,
            "sweep_bytes": sweep_b, "volume_drift": abs(vol1 - vol0) / vol0,
            "unexplained": {"steps": CHECKED_STEPS, "volume": abs(v_res) / vol0, "energy": abs(e_res) / e0},
            "c_final": c_final}


def run_batch(pcvof, torch, wls, precision, steps, warmup, use_graph, autotune):
    """warmup + steps batched steps of all domains; returns the timed ms, the tile
    choice, the volume drift (summed over domains) and the final fractions."""
    specs = [pcvof.DomainSpec(shape=wl.shape, h=wl.h, ndim=3, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                              rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal, precision=precision)
             for wl in wls]
    b = pcvof.Batch(specs)
    for d, wl in zip(b.domains, wls):
        d.set_vof(wl.c)
        d.set_energy(wl.e)
        d.set_velocity(wl.u, wl.v, wl.w)
    dts = [wl.dt for wl in wls]
    vol0 = sum(float(d.vof().sum()) * wl.h ** 3 for d, wl in zip(b.domains, wls))
    tiles = b.autotune(dts, reps=3) if autotune else b.tiles()
    for _ in range(warmup):
        b.step(dts, use_graph=use_graph)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        b.step(dts, use_graph=use_graph)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    st = b.step(dts, use_graph=use_graph, stats=True)
    vol1 = sum(x["vol"] for x in st)
    finals = [d.vof().cpu().numpy() for d in b.domains]
    b.close()
    torch.cuda.empty_cache()
    return {"total_ms": ms, "tiles": {"chunk": tiles["chunk"]},
            "volume_drift": abs(vol1 - vol0) / vol0, "finals": finals}


def run_per_domain(pcvof, torch, wls, steps, warmup):
    """The same steps as one single-domain FP64 step call per domain (the domains in
    turn, each with its own launches)."""
    doms = []
    for wl in wls:
        spec = pcvof.DomainSpec(shape=wl.shape, h=wl.h, ndim=3, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                                rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal)
        d = pcvof.Domain(spec)
        d.set_vof(wl.c)
        d.set_energy(wl.e)
        d.set_velocity(wl.u, wl.v, wl.w)
        doms.append(d)
    for _ in range(warmup):
        for d, wl in zip(doms, wls):
            d.step(wl.dt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        for d, wl in zip(doms, wls):
            d.step(wl.dt)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    for d, wl in zip(doms, wls):  # the step the batched runs take with checksums
        d.step(wl.dt)
    finals = [d.vof().cpu().numpy() for d in doms]
    for d in doms:
        d.close()
    torch.cuda.empty_cache()
    return {"total_ms": ms, "finals": finals}


def bench_batch(args, pcvof, torch):
    wls = workload("batch64")
    ncells = sum(wl.ncells for wl in wls)
    # algorithmic bytes of the three sweeps of a step, summed over the domains
    step_bytes = sum(sweep_bytes(wl, a) for wl in wls for a in range(3))
    step_bytes_mx = sum(sweep_bytes(wl, a, True) for wl in wls for a in range(3))
    per = run_per_domain(pcvof, torch, wls, args.steps, args.warmup)
    b64 = run_batch(pcvof, torch, wls, "fp64", args.steps, args.warmup, use_graph=True, autotune=True)
    b64_plain = run_batch(pcvof, torch, wls, "fp64", args.steps, args.warmup, use_graph=False, autotune=False)
    bmx = run_batch(pcvof, torch, wls, "mixed", args.steps, args.warmup, use_graph=True, autotune=True)
    same = all(np.array_equal(a, c) for a, c in zip(per["finals"], b64["finals"]))
    dmx = [np.abs(a - c) for a, c in zip(bmx["finals"], b64["finals"])]
    rate = lambda r: ncells * args.steps / (r["total_ms"] * 1e-3)  # noqa: E731
    value = rate(b64)
    ms_step = b64["total_ms"] / args.steps
    achieved = step_bytes / (ms_step * 1e-3) / 1e9
    mx_ms = bmx["total_ms"] / args.steps
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch of {len(wls)} domains (sides 32-160, {ncells} cells)",
                   "ndomains": len(wls), "cells": ncells, "bc": "periodic", "cfl": 0.3, "normal": "MYC",
                   "mdot": "off", "precision": "fp64", "launch": "fused sweep launches, graph replay, autotuned chunks",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "batched sweeps (bytes of the three sweeps over the whole step time)",
                     "bytes_per_cell": SWEEP_BYTES_PER_CELL + SWEEP_BYTES_PER_FACE},
        "tiles": b64["tiles"],
        "volume_drift": b64["volume_drift"],
        "per_domain_fp64": {"value": rate(per), "ms_per_step": per["total_ms"] / args.steps,
                            "fields_equal_to_batched": same},
        "batched_fp64_no_graph": {"value": rate(b64_plain), "ms_per_step": b64_plain["total_ms"] / args.steps},
        "mixed": {"value": rate(bmx), "ms_per_step": mx_ms, "speedup_vs_fp64": rate(bmx) / value,
                  "speedup_vs_per_domain_fp64": rate(bmx) / rate(per), "tiles": bmx["tiles"],
                  "roofline": {"achieved": step_bytes_mx / (mx_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                               "frac": step_bytes_mx / (mx_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
                  "volume_drift": bmx["volume_drift"],
                  "c_vs_fp64": {"max_abs": float(max(x.max() for x in dmx)),
                                "l1_rel": float(sum(x.sum() for x in dmx) /
                                                sum(np.abs(c).sum() for c in b64["finals"]))}},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wls[0])
    print(json.dumps(out), flush=True)


def energy_flux_ablation(pcvof, torch, steps=10, timed_steps=50):
    """Conservative (eq. disc_et_adv) against non-conservative (eq. disc_et_adv_noncons)
    energy fluxes of section 3.4.1 at the water heat-capacity ratio of about 3240: 30
    seeded droplets in a 128^3 periodic box under a random divergence-free velocity,
    with a uniform temperature T0 = 1, which the exact solution keeps. Per mode: the
    largest temperature error after `steps` steps (everywhere and in interface cells),
    the change of total energy net of the reported boundary, dilatation and clip terms,
    and the throughput of `timed_steps` more steps. The error is taken after a few steps
    because WENO5 face values in a single explicit stage amplify high-wavenumber
    round-off (about 6% per sweep at CFL 0.3 for the linear weights): without the
    paper's diffusion step, the round-off of any run grows to visible levels after a few
    tens of steps."""
    from paper_2001_03477_amd import workloads as W
    wl = W.droplets_3d(128, ndrops=30, seed=9, rmin=4.0, rmax=12.0)
    T0 = 1.0
    wl.e = (wl.cp_l * wl.c + wl.cp_g * (1.0 - wl.c)) * T0
    hv = wl.h ** 3
    e_tot0 = math.fsum(wl.e.ravel().tolist()) * hv
    out = {"workload": "droplets3d_128: 30 drops, C_pl/C_pg = 4.039e6/1.248e3, uniform T",
           "steps": steps, "timed_steps": timed_steps}
    for mode in ("conservative", "nonconservative"):
        spec = pcvof.DomainSpec(shape=wl.shape, h=wl.h, ndim=3, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                                energy_flux=mode)
        d = pcvof.Domain(spec)
        d.set_vof(wl.c)
        d.set_energy(wl.e)
        d.set_velocity(wl.u, wl.v, wl.w)
        prev, res = e_tot0, 0.0
        for _ in range(steps):
            st = d.step(wl.dt, 1.0, stats=True)
            res += st["energy"] - prev - (-st["energy_bnd_out"] + st["energy_src"] + st["energy_clip"]
                                          + st["energy_phase"])
            prev = st["energy"]
        T = d.temperature().cpu().numpy()
        c = d.vof().cpu().numpy()
        iface = (c > 0.01) & (c < 0.99)
        err = np.abs(T - T0) / T0
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(timed_steps):
            d.step(wl.dt, 1.0)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out[mode] = {"T_max_rel_err": float(err.max()), "T_max_rel_err_interface": float(err[iface].max()),
                     "T_mean_rel_err_interface": float(err[iface].mean()),
                     "energy_change_net_of_reported_terms_rel": abs(res) / abs(e_tot0),
                     "value": wl.ncells * timed_steps / (ms * 1e-3), "unit": "cell-updates/s"}
        del d
        torch.cuda.empty_cache()
    return out


def split_ablation(pcvof, torch, wl, steps=200, timed_steps=50):
    """Weymouth-Yue split (the scheme the paper builds on) against the Lagrangian-
    explicit sweeps of Li (CIAM), which section 3.3 names as the other scheme, on the
    benchmark's LeVeque deformation field: the relative change of total volume and
    energy after `steps` steps (walls with no normal flow: the exact change is zero),
    the volume clipped into [0, 1] on the way, and the throughput of `timed_steps`
    more steps."""
    hv = wl.h ** wl.ndim
    v0 = math.fsum(wl.c.ravel().tolist()) * hv
    e0 = math.fsum(wl.e.ravel().tolist()) * hv
    out = {"workload": wl.name, "steps": steps, "timed_steps": timed_steps}
    for split in ("wy", "le"):
        spec = pcvof.DomainSpec(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                                normal=wl.normal, split=split)
        d = pcvof.Domain(spec)
        d.set_vof(wl.c)
        d.set_energy(wl.e)
        d.set_velocity(wl.u, wl.v, wl.w)
        clip = 0.0
        for k in range(steps):
            st = d.step(wl.dt, wl.u_scale(k), stats=True)
            clip += abs(st["vol_clip"])
        c = d.vof().cpu().numpy()
        stream = torch.cuda.current_stream()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for k in range(timed_steps):
            d.step(wl.dt, wl.u_scale(steps + k))
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        out[split] = {"vol_change_rel": (st["vol"] - v0) / v0, "energy_change_rel": (st["energy"] - e0) / e0,
                      "vol_clipped_rel": clip / v0, "c_min": float(c.min()), "c_max": float(c.max()),
                      "value": wl.ncells * timed_steps / (ms * 1e-3), "unit": "cell-updates/s"}
        del d
        torch.cuda.empty_cache()
    return out


def period_shape_error(pcvof, torch, wl):
    """One period T of the LeVeque deformation (its time scale cos(pi t / T) reverses the
    flow at T / 2, so the exact field after T is the initial one): the L1 shape error
    sum |c(T) - c(0)| h^3, also relative to the initial volume, the relative volume change
    and the time of the wl.steps steps, for the FP64 and mixed-precision paths."""
    hv = wl.h ** wl.ndim
    v0 = math.fsum(wl.c.ravel().tolist()) * hv
    scales = [wl.u_scale(k) for k in range(wl.steps)]
    out = {"workload": wl.name, "steps": wl.steps, "period": round(wl.steps * wl.dt, 6)}
    for prec in ("fp64", "mixed"):
        spec = pcvof.DomainSpec(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                                normal=wl.normal, precision=prec)
        d = pcvof.Domain(spec)
        d.set_vof(wl.c)
        d.set_energy(wl.e)
        d.set_velocity(wl.u, wl.v, wl.w)
        stream = torch.cuda.current_stream()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        d.steps(wl.steps, wl.dt, u_scale=scales)
        t1.record(stream)
        torch.cuda.synchronize()
        c = d.vof().cpu().numpy()
        l1 = math.fsum(np.abs(c - wl.c).ravel().tolist()) * hv
        v1 = math.fsum(c.ravel().tolist()) * hv
        out[prec] = {"l1": l1, "l1_rel": l1 / v0, "vol_change_rel": (v1 - v0) / v0,
                     "ms": t0.elapsed_time(t1)}
        del d
        torch.cuda.empty_cache()
    return out


def extension_timing(pcvof, torch, wl, rho_g, calls=5):
    """The liquid-velocity extension (section 3.3.1) on the workload's fractions and
    mass flux: wall time per pcvof_extend_velocity call (labels, compaction, assembly,
    conjugate gradients with their host convergence checks, face corrections), median
    of `calls` calls after one untimed call, with the solver's unknowns, iterations and
    final relative residual. Not part of the advection step that `value` times."""
    spec = pcvof.DomainSpec(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                            rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal)
    d = pcvof.Domain(spec)
    d.set_vof(wl.c)
    d.set_energy(wl.e)
    d.set_velocity(wl.u, wl.v, wl.w)
    d.set_mass_flux(wl.mdot)
    info, _ = d.extend_velocity(rho_g)
    times = []
    for _ in range(calls):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info, _ = d.extend_velocity(rho_g)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    del d
    torch.cuda.empty_cache()
    return {"ms": float(np.median(times)), "rho_g": rho_g, **info, "rel_tol": 1e-13}


def diffusion_timing(pcvof, torch, wl, k_l, k_g, calls=5):
    """The implicit energy diffusion (section 3.4.2) on the workload's state: wall time
    per pcvof_diffuse call (assembly with the height-function distances, BiCGSTAB with
    its host convergence checks, the energy written back), median of `calls` calls after
    one untimed call, with the iterations and final relative residual. Not part of the
    advection step that `value` times."""
    spec = pcvof.DomainSpec(shape=wl.shape, h=wl.h, ndim=wl.ndim, bc=wl.bc, cp_l=wl.cp_l, cp_g=wl.cp_g,
                            rho_l=wl.rho_l, T_gamma=wl.T_gamma, normal=wl.normal)
    d = pcvof.Domain(spec)
    d.set_vof(wl.c)
    d.set_energy(wl.e)
    info, _ = d.diffuse(wl.dt, k_l, k_g)
    times = []
    for _ in range(calls):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info, _ = d.diffuse(wl.dt, k_l, k_g)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    del d
    torch.cuda.empty_cache()
    return {"ms": float(np.median(times)), "k_l": k_l, "k_g": k_g, "dt": wl.dt, **info, "rel_tol": 1e-13}


def _subbox(wl, z0, y0, x0, side):
    """The inputs of the side^3 sub-box of the workload with corner (z0, y0, x0), as
    contiguous arrays (fractions, energies, face velocities, mass flux)."""
    sz, sy, sx = (min(side, n) for n in wl.shape)
    zs, ys, xs = slice(z0, z0 + sz), slice(y0, y0 + sy), slice(x0, x0 + sx)
    c = np.ascontiguousarray(wl.c[zs, ys, xs])
    e = np.ascontiguousarray(wl.e[zs, ys, xs])
    u = np.ascontiguousarray(wl.u[zs, ys, x0:x0 + sx + 1])
    v = np.ascontiguousarray(wl.v[zs, y0:y0 + sy + 1, xs])
    w = None if wl.w is None else np.ascontiguousarray(wl.w[z0:z0 + sz + 1, ys, xs])
    md = None if wl.mdot is None else np.ascontiguousarray(wl.mdot[zs, ys, xs])
    return c, e, u, v, w, md


def _oracle_steps(job):
    """Whole oracle steps of one sub-box until the budget is used (at least one step):
    (cells, steps, seconds). Runs in a worker process of its own."""
    import oracle
    c, e, u, v, w, md, cfg_kw, dt, scales, budget_s = job
    cfg = oracle.Config(**cfg_kw)
    t0 = time.perf_counter()
    n = 0
    while True:
        c, e, _ = oracle.step(cfg, c, e, u, v, w, md, dt, scales[n % len(scales)], n)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return int(c.size), n, el


def _host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(wl, budget_s=10.0, side=128, max_workers=16):
    """The oracle on the host, two runs on the same inputs: one thread on the leading
    side^3 sub-box of the workload (the whole workload if it is smaller), and one
    process per available core (at most max_workers, the host share of one GPU), each
    stepping its own side^3 sub-box. Sub-boxes of a larger domain have outflow sides;
    they are independent, so the all-core rate is the sum of the workers' rates."""
    import concurrent.futures as cf
    import multiprocessing as mp
    model, avail = _host_cpu()
    nz, ny, nx = wl.shape
    sub = max(wl.shape) > side
    cfg_kw = dict(shape=tuple(min(side, n) for n in wl.shape), h=wl.h, ndim=wl.ndim,
                  bc=(1, 1, 1) if sub else tuple(wl.bc), cp_l=wl.cp_l, cp_g=wl.cp_g, rho_l=wl.rho_l,
                  T_gamma=wl.T_gamma, normal=wl.normal)
    scales = [wl.u_scale(k) for k in range(64)]
    corners = [(z, y, x) for z in range(0, nz, side) for y in range(0, ny, side) for x in range(0, nx, side)
               if z + side <= max(nz, side) and y + side <= max(ny, side) and x + side <= max(nx, side)]
    one = _oracle_steps((*_subbox(wl, *corners[0], side), cfg_kw, wl.dt, scales, budget_s))
    nw = max(1, min(avail, max_workers, len(corners)))
    jobs = [(*_subbox(wl, *corners[k % len(corners)], side), cfg_kw, wl.dt, scales, budget_s) for k in range(nw)]
    with cf.ProcessPoolExecutor(max_workers=nw, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_steps, jobs))
    rate1 = one[0] * one[1] / one[2]
    rate_n = sum(cells * n / el for cells, n, el in res)
    shape = "x".join(str(v) for v in cfg_kw["shape"][::-1])
    what = f"{shape} sub-box(es) of the {wl.name} workload (outflow sides)" if sub else f"the {wl.name} workload"
    return {"value": rate_n, "unit": "cell-updates/s", "cores": nw, "kind": "oracle",
            "sample": (f"{sum(n for _, n, _ in res)} full steps over {nw} independent {what}, one process per "
                       f"core, about {budget_s:.0f} s each"),
            "cpu_model": model, "cores_available": avail,
            "single_thread": {"value": rate1, "cores": 1, "steps": one[1], "seconds": round(one[2], 2),
                              "sample": (f"{one[1]} full steps of the leading {shape} sub-box" if sub
                                         else f"{one[1]} full steps of the {wl.name} workload")}}


def sweep_duration(wl, r, steps, mixed=False):
    """The sweeps' average launch duration, as the tighter of two upper bounds measured
    with HIP events on the library's stream: the event pair recorded with each sweep
    launch (which adds the events' own cost, several µs per launch), and the timed region
    divided by its sweep launches (which adds the step's other kernels and the gaps
    between launches). Algorithmic bytes per launch: the mean over the axes."""
    pairs = float(r["sweep_ms"].sum() / r["sweep_n"].sum())
    region = r["total_ms"] / (steps * wl.ndim)
    per_launch = sum(sweep_bytes(wl, a, mixed) for a in range(wl.ndim)) / wl.ndim
    best = min(pairs, region)
    return {"avg_launch_ms": best, "source": "timed region" if best == region else "event pairs",
            "event_pairs_ms": pairs, "timed_region_ms": region, "bytes_per_launch": per_launch}


def bench_workload(args, pcvof, torch, wl, copy_gbs, mixed=True):
    """FP64 (and mixed-precision) runs of one single-domain workload: the fields of the
    JSON line for it."""
    scales = np.array([wl.u_scale(k) for k in range(args.warmup + 2 * args.steps)])
    r64 = run(pcvof, torch, wl, "fp64", args.steps, args.warmup, scales)
    c64 = r64.pop("c_final")
    torch.cuda.synchronize()
    rmx = run(pcvof, torch, wl, "mixed", args.steps, args.warmup, scales) if mixed else None
    total_ms, sweep_ms, sweep_n, prof = r64["total_ms"], r64["sweep_ms"], r64["sweep_n"], r64["prof"]
    dur = sweep_duration(wl, r64, args.steps)
    avg_sweep_ms = dur["avg_launch_ms"]
    achieved = dur["bytes_per_launch"] / (avg_sweep_ms * 1e-3) / 1e9
    value = wl.ncells * args.steps / (total_ms * 1e-3)
    out = {
        "value": value,
        "unit": "cell-updates/s",
        "ms_per_step": total_ms / args.steps,
        "config": {"workload": wl.name, "grid": list(wl.shape[::-1]), "ndim": wl.ndim,
                   "bc": "outflow" if wl.bc[0] else "periodic", "cfl": round(W_max_face(wl) * wl.dt / wl.h, 4),
                   "normal": "MYC", "mdot": "on" if wl.mdot is not None else "off", "precision": "fp64",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(wl, sweep_n),
                     "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
                     "kernel": "k_sweep_x / k_sweep_t<1> / k_sweep_t<2>",
                     "avg_launch_ms": avg_sweep_ms, "duration_from": dur["source"],
                     "avg_launch_ms_event_pairs": dur["event_pairs_ms"],
                     "avg_launch_ms_timed_region": dur["timed_region_ms"],
                     "per_axis_ms": [float(t / n) for t, n in zip(sweep_ms, sweep_n)],
                     "bytes_per_cell": SWEEP_BYTES_PER_CELL + SWEEP_BYTES_PER_FACE},
        "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in prof.items() if v["launches"]},
        "volume_drift": r64["volume_drift"],
        "drift_net_of_reported_terms": r64["unexplained"],
    }
    if rmx is not None:
        cmx = rmx.pop("c_final")
        dc = np.abs(cmx - c64)
        mx_value = wl.ncells * args.steps / (rmx["total_ms"] * 1e-3)
        mdur = sweep_duration(wl, rmx, args.steps, mixed=True)
        mx_achieved = mdur["bytes_per_launch"] / (mdur["avg_launch_ms"] * 1e-3) / 1e9
        out["mixed"] = {
            "value": mx_value, "unit": "cell-updates/s", "ms_per_step": rmx["total_ms"] / args.steps,
            "speedup_vs_fp64": mx_value / value, "dtype": "f64 state, f32 geometry and storage",
            "per_axis_ms": [float(t / n) for t, n in zip(rmx["sweep_ms"], rmx["sweep_n"])],
            "roofline": {"bound": "hbm", "achieved": mx_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": mx_achieved / HBM_PEAK_GBS, "duration_from": mdur["source"],
                         "traffic": recorded_traffic(wl, rmx["sweep_n"], mixed=True),
                         "bytes_per_cell": SWEEP_BYTES_PER_CELL_MIXED + SWEEP_BYTES_PER_FACE_MIXED},
            "volume_drift": rmx["volume_drift"],
            "drift_net_of_reported_terms": rmx["unexplained"],
            "c_vs_fp64": {"max_abs": float(dc.max()), "l1_rel": float(dc.sum() / np.abs(c64).sum())},
        }
    return out


# extra single-domain workloads of the default line (name for workload(), key)
EXTRA_WORKLOADS = (("leveque128", "leveque3d_128"), ("bubble256", "bubble3d_256"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="droplets512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64-only", action="store_true", help="skip the mixed-precision run")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the energy-flux and split-scheme ablations")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra workloads (128^3 LeVeque, 256^3 bubble) of the default line")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device, a kernel of known traffic "
                         "for scaling the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the advection step of one domain is measured on "
              "one MI355X; sharding over several GPUs is designed but not implemented",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2001_03477_amd import pcvof
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibration_copy_mib > 0:
        n = args.calibration_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    copy_gbs = None if args.calibration_copy_mib > 0 else copy_bandwidth(torch)
    if args.workload == "batch64":
        bench_batch(args, pcvof, torch)
        return
    wl = workload(args.workload)
    print(f"bench: {wl.name}, {args.warmup} + {args.steps} steps", file=sys.stderr, flush=True)
    res = bench_workload(args, pcvof, torch, wl, copy_gbs, mixed=not args.fp64_only)
    out = {"metric": METRIC, "value": res.pop("value"), "unit": res.pop("unit"), "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", **res}
    default_line = args.workload == "droplets512"
    if default_line and not args.no_extra:
        extra = {}
        for name, key in EXTRA_WORKLOADS:
            xw = workload(name)
            print(f"bench: extra workload {xw.name}", file=sys.stderr, flush=True)
            r = bench_workload(args, pcvof, torch, xw, copy_gbs, mixed=not args.fp64_only)
            keep = {k: r[k] for k in ("value", "unit", "ms_per_step", "config", "kernel_ms_per_step",
                                      "volume_drift", "drift_net_of_reported_terms")}
            keep["roofline"] = {k: r["roofline"][k] for k in ("achieved", "frac", "traffic", "avg_launch_ms",
                                                              "per_axis_ms")}
            if "mixed" in r:
                keep["mixed"] = {k: r["mixed"][k] for k in ("value", "ms_per_step", "speedup_vs_fp64",
                                                            "volume_drift", "c_vs_fp64")}
            if name == "leveque128":
                keep["period_shape_error"] = period_shape_error(pcvof, torch, xw)
            if name == "bubble256":
                # vapour density and conductivities of the paper's superheated-bubble case
                keep["extension"] = extension_timing(pcvof, torch, xw, 0.25)
                keep["diffusion"] = diffusion_timing(pcvof, torch, xw, 0.07, 0.007)
            extra[key] = keep
            if name == "leveque128" and not args.no_ablation:
                print("bench: ablations", file=sys.stderr, flush=True)
                out["energy_flux_ablation"] = energy_flux_ablation(pcvof, torch)
                out["split_ablation"] = split_ablation(pcvof, torch, xw)
            del xw
        out["other_workloads"] = extra
    elif args.workload == "leveque128" and not args.no_ablation:
        out["energy_flux_ablation"] = energy_flux_ablation(pcvof, torch)
        out["split_ablation"] = split_ablation(pcvof, torch, wl)
    if args.workload.startswith("leveque"):
        out["period_shape_error"] = period_shape_error(pcvof, torch, wl)
    if args.workload == "bubble256":
        out["extension"] = extension_timing(pcvof, torch, wl, 0.25)
        out["diffusion"] = diffusion_timing(pcvof, torch, wl, 0.07, 0.007)
    if not args.no_cpu_baseline:
        print("bench: oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
