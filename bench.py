#!/usr/bin/env python3
"""Throughput of the coupled HLBM step on one MI355X.

One step = momentum exchange -> Newton-Euler -> particle binning -> fused
collide/stream with the HLBM coupling (all of the hot path), over the whole
lattice.  MLUPS = cells x steps / (wall time x 1e6), inputs resident in HBM,
timed with torch.cuda.synchronize() on both sides of exactly K steps.

The default workload is hindered384: 384^3 cells with walls in z, 11 265
mixed particles (spheres, rounded cubes, 2:1 spheroids) of r_eq ~ U[4, 8] at
solid fraction 0.2, tau 0.55, density ratio 2.5, FP32 populations -- the
largest single-GPU configuration of the hindered-settling workloads.

Prints one JSON line.  Besides the throughput it carries:
  roofline      -- the collide-and-stream kernel's algorithmic HBM bytes per
                   launch (2 x 19 populations x bytes each, per cell) divided
                   by its mean HIP-event duration over the timed region,
                   against the 8 TB/s HBM peak; next to it the coupled step's
                   fraction: MLUPS x 38 x bytes per population over 8 TB/s;
  errors_vs_fp64 -- this precision against the FP64 form of the same
                   workload from rest (untimed runs): velocity L2-relative
                   and max |rho - rho_ref| at the end, time-averaged
                   per-particle force RMS-relative over particles, settling
                   velocity (mean U_z over particles, over the last 10 % of
                   the steps) relative;
  cpu_baseline  -- the FP64 CPU oracle on a bounded sample of the workload;
  segments      -- the K timed steps as 5 equal consecutive segments (stream
                   events between them, no host synchronisation): ms per step
                   of each and their median.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled HLBM MLUPS + % HBM roofline, FP32/learned vs FP64 at ≤1% force err"
HBM_PEAK_GBS = 8000.0
POP_BYTES = {"fp64": 8, "fp32": 4, "fp16s": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16s": "f32 (f16 storage)"}
DEFAULT_PRECISION = {"spheres128": "fp32", "sphere32": "fp64", "mixed256": "fp16s",
                     "mixed256_learned": "fp16s", "hindered384": "fp32", "hindered384b": "fp32",
                     "meshes128": "fp32", "meshes128_learned": "fp32"}
# surrogate training settings for the learned-indicator workload
TRAIN = dict(samples=1_000_000, holdout=100_000, iterations=30000, batch=8192, lr=1e-2, lr_final=1e-5,
             band=0.1, clip=0.25, band_share=0.8, gate_rms=0.05, gate_max=0.5)


def make_sim(H, W, wl, precision, coupling="hlbm"):
    """A context for the workload; for a learned workload the non-spherical
    families present are trained first (outside any timed region)."""
    import numpy as np
    learned = bool(getattr(wl, "learned", False))
    mesh = bool(len(wl.particles)) and bool(np.any(wl.particles["shape"] == W.MESH))
    rmax = 0.0
    if learned or mesh:
        rmax = max(W.circumradius(int(s), p) for s, p in zip(wl.particles["shape"], wl.particles["param"]))
    sim = H.Simulation(wl.n, wl.bc, wl.tau, precision, max_particles=len(wl.particles),
                       gravity=wl.gravity, eps=wl.eps, rho_f=wl.rho_f,
                       learned_max_circumradius=rmax + 0.01 if (learned or mesh) else 0.0,
                       learned_samples=1_100_000 if learned else 0,
                       max_mesh_triangles=len(W.MESH_UNIT[1]) if mesh else 0, coupling=coupling)
    if mesh:
        sim.set_mesh(*W.MESH_UNIT)
    reports = {}
    if learned:
        for s in (W.ROUNDED_CUBE, W.SPHEROID, W.MESH):
            sel = wl.particles["shape"] == s
            if not np.any(sel):
                continue
            prm = wl.particles["param"][np.argmax(sel)]
            sim.mlp_set_params(s, W.mlp_init_params(7 + s))
            reports[W.SHAPE_NAMES[s]] = sim.train_indicator(
                s, prm[:2], ref_circumradius=W.circumradius(s, prm), **TRAIN)
    sim.set_particles(wl.particles)
    return sim, reports


def kernel_source_hash() -> str:
    """Hash of the sources the lattice (collide) kernel is built from."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2312_14172_amd", "csrc")
    for name in ("hlbm_device.h", "hlbm_tile.h", "hlbm_lattice.hip"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, precision: str):
    """HBM bytes per collide launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"collide_{workload}_{precision}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and line.startswith("    "):
                k, v = line.split("=", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return int(rec["hbm_bytes_per_launch"]) if "hbm_bytes_per_launch" in rec else None


def errors_vs_fp64(H, wl, precision, steps, every, coupling="hlbm", contact=None):
    """This precision against the FP64 plain form (exact indicator) of the
    same workload from rest: velocity L2-relative and max |rho - rho_ref|
    after `steps`, the per-particle force averaged over samples every `every`
    steps (RMS-relative over particles) and the settling velocity (mean U_z
    over particles, averaged over the samples of the last 10 % of the
    steps)."""
    import numpy as np
    import torch
    from paper_2312_14172_amd import workloads as W
    res = {}
    nsamp = steps // every
    last = max(1, nsamp // 10)
    for prec in (precision, "fp64"):
        if prec == "fp64":
            mesh = bool(np.any(wl.particles["shape"] == W.MESH))
            rmax = max(W.circumradius(int(s), p) for s, p in zip(wl.particles["shape"], wl.particles["param"]))
            sim = H.Simulation(wl.n, wl.bc, wl.tau, prec, max_particles=len(wl.particles),
                               gravity=wl.gravity, eps=wl.eps, rho_f=wl.rho_f,
                               learned_max_circumradius=rmax + 0.01 if mesh else 0.0,
                               max_mesh_triangles=len(W.MESH_UNIT[1]) if mesh else 0, coupling=coupling)
            if mesh:
                sim.set_mesh(*W.MESH_UNIT)
            sim.set_particles(wl.particles)
        else:
            sim, _ = make_sim(H, W, wl, prec, coupling)
        if contact:
            sim.set_contact(*contact)
        acc = np.zeros((len(wl.particles), 3))
        vz = []
        for k in range(nsamp):
            sim.step(every)
            F, _, st = sim.get_forces()
            acc += F
            if k >= nsamp - last:
                vz.append(float(np.mean(st["vel"][:, 2])))
        fl = sim.get_fields(H.FIELD_RHO | H.FIELD_U)
        torch.cuda.synchronize()
        res[prec] = dict(F=acc / nsamp, vz=float(np.mean(vz)), rho=fl["rho"], u=fl["u"])
        sim.close()
        del sim, fl
    a, r = res[precision], res["fp64"]
    err_F = float(np.sqrt(np.mean(np.sum((a["F"] - r["F"]) ** 2, axis=1))) /
                  np.sqrt(np.mean(np.sum(r["F"] ** 2, axis=1))))
    err_u = float(np.linalg.norm(a["u"] - r["u"]) / np.linalg.norm(r["u"]))
    err_rho = float(np.max(np.abs(a["rho"] - r["rho"])))
    err_vz = abs(a["vz"] - r["vz"]) / max(abs(r["vz"]), 1e-300)
    return {"velocity_l2rel": float(f"{err_u:.4g}"), "density_maxabs": float(f"{err_rho:.4g}"),
            "force_rms_rel": float(f"{err_F:.4g}"), "settling_velocity_rel": float(f"{err_vz:.4g}"),
            "run": f"{steps} steps from rest, forces sampled every {every}, settling velocity over the last "
                   f"{last * every} steps"}


def cpu_baseline(wl, target_s=12.0, contact=None):
    """The FP64 oracle as it stands, on a bounded number of steps of the same
    workload (with the same contact, if any), all host cores (OpenMP): steps
    are timed one at a time until about target_s seconds have passed (at
    least one, at most 200)."""
    from oracle import oracle as orc
    o = orc.Oracle(wl.n, wl.bc, wl.tau, eps=wl.eps, rho_f=wl.rho_f, gravity=wl.gravity, contact=contact)
    P = o.to_parts(wl.particles)
    f = o.equilibrium()
    steps, dt = 0, 0.0
    while steps < 200 and (steps == 0 or dt < target_s):
        t0 = time.perf_counter()
        o.run(P, f, 1)
        dt += time.perf_counter() - t0
        steps += 1
    return {"value": round(wl.ncells * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": int(o.num_threads()), "kind": "oracle",
            "sample": f"{wl.name}: the first {steps} FP64 step(s) from rest of the full workload, {dt:.1f} s"}


def copy_calibration(nbytes=1 << 31, reps=3):
    """A plain device copy of known size, for scaling HBM counters."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="hindered384", choices=sorted(DEFAULT_PRECISION))
    ap.add_argument("--precision", default=None, choices=sorted(POP_BYTES))
    ap.add_argument("--coupling", default="hlbm", choices=("hlbm", "psm"),
                    help="exact-difference source (hlbm) or partially saturated collision (psm)")
    ap.add_argument("--check-steps", type=int, default=1000,
                    help="steps of the untimed runs compared with FP64")
    ap.add_argument("--contact", type=float, nargs=3, default=None, metavar=("RANGE", "K", "KW"),
                    help="turn on the contact repulsion (range in cells, pair and wall stiffness); the "
                         "oracle's node contact is slow, so --no-cpu-baseline suits large workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-force-check", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 2 GiB device copy (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path is single-GPU by design)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2312_14172_amd import hlbm as H
    from paper_2312_14172_amd import workloads as W

    torch.cuda.set_device(0)
    precision = args.precision or DEFAULT_PRECISION[args.workload]
    wl = W.get(args.workload)
    print(f"[bench] {wl.name}: {wl.n} cells, {len(wl.particles)} particles, {precision}, "
          f"phi={wl.solid_fraction:.3f}", file=sys.stderr, flush=True)
    H.lib()
    sim, train_reports = make_sim(H, W, wl, precision, args.coupling)
    if args.contact:
        sim.set_contact(*args.contact)
    sim.step(args.warmup)
    sim.get_forces()            # synchronises and reports kernel errors
    torch.cuda.synchronize()

    sim.profile_begin()
    # the K steps run as 5 equal segments between stream events (no host
    # synchronisation inside the timed region), for a median over segments
    nseg = 5 if args.steps >= 5 and args.steps % 5 == 0 else 1
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(nseg + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record()
    for k in range(nseg):
        sim.step(args.steps // nseg)
        marks[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    seg_ms = [marks[k].elapsed_time(marks[k + 1]) / (args.steps // nseg) for k in range(nseg)]
    collide_ms, launches = sim.profile_end()
    sim.get_forces()            # surfaces any kernel-raised error of the timed steps
    dt = t1 - t0
    mlups = wl.ncells * args.steps / dt / 1e6
    print(f"[bench] timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)

    alg_bytes = 2 * 19 * POP_BYTES[precision] * wl.ncells
    per_launch_s = collide_ms / max(launches, 1) / 1e3
    achieved = alg_bytes / per_launch_s / 1e9
    traffic = load_traffic(wl.name, precision)
    step_bytes = 2 * 19 * POP_BYTES[precision] * wl.ncells * args.steps
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"k_collide<{precision}>",
                "kernel_ms": round(per_launch_s * 1e3, 5),
                "bytes_per_launch": alg_bytes,
                "coupled_step_frac": round(step_bytes / dt / 1e9 / HBM_PEAK_GBS, 4),
                "coupled_step_note": "MLUPS x 38 x bytes per population / 8 TB/s: the whole step "
                                     "(all kernels) against the lattice's algorithmic traffic"}
    sim.close()

    if args.copy_calibration:
        copy_calibration()

    extra = {}
    if not args.no_force_check and precision != "fp64" and len(wl.particles):
        print(f"[bench] errors against FP64: {args.check_steps} steps per precision", file=sys.stderr, flush=True)
        extra["errors_vs_fp64"] = errors_vs_fp64(H, wl, precision, args.check_steps, 10, args.coupling,
                                                 args.contact)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, contact=args.contact)

    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[precision], "data": "synthetic",
        "config": {"workload": wl.name, "lattice": list(wl.n), "bc": list(wl.bc),
                   "particles": int(len(wl.particles)), "solid_fraction": round(wl.solid_fraction, 4),
                   "tau": wl.tau, "storage": precision, "coupling": args.coupling, "contact": args.contact,
                   "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu,
        "segments": {"count": nseg, "steps_each": args.steps // nseg,
                     "ms_per_step": [round(v, 5) for v in seg_ms],
                     "median_ms_per_step": round(float(np.median(seg_ms)), 5),
                     "median_mlups": round(wl.ncells / (float(np.median(seg_ms)) * 1e-3) / 1e6, 2)},
    }
    out.update(extra)
    if train_reports:
        out["learned_indicator"] = {k: {kk: (float(f"{vv:.4g}") if isinstance(vv, float) else vv)
                                        for kk, vv in v.items()} for k, v in train_reports.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
