"""Benchmark of the particle step (interpolate, rotate, Boris push, zig-zag
deposit, and the per-cell sort every 5 steps of the 3D box, every 20 of the
axisymmetric workloads) on one MI355X.

Default workload: 3D Cartesian 128^3 periodic box, two species with 16
particles per cell each (67,108,864 particles), Maxwell-Juttner theta=1 with a
0.3c drift, B0 = 1 z plus 32 seeded plane waves (synthetic, seeded inputs).

Prints one JSON line: ns per particle per step of the FP32 library (value),
the FP64 form beside it, the roofline of the fused particle-step kernel
(algorithmic HBM bytes per launch over its HIP-event duration, and the
calibrated counter traffic of the committed profile while it matches the
sources), the axisymmetric workloads, a particle-count sweep, the
checkpointed adjoint with the reverse-step kernel's roofline, the field
solver's kernels, and the FP64 CPU reference timed on a bounded sample of
the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def algorithmic_bytes_per_particle(dim, prec, ncells, nparticles, has_phi=False):
    """Minimum HBM traffic of one particle step: the particle SoA read (cell,
    offsets, u, w, phi) and written (cell, offsets, u, phi), the fields read
    once per cell and the current read-modify-written once per cell."""
    b = 4 if prec == "f32" else 8
    ob = 4 if prec == "f32" else 8  # FP32 build: 32-bit fixed-point offsets
    rd = 4 + dim * ob + 3 * b + b + (b if has_phi else 0)
    wr = 4 + dim * ob + 3 * b + (b if has_phi else 0)
    grid = (6 * b + 2 * 3 * b) * ncells / nparticles
    return rd + wr + grid


def measured_traffic(kernel_key, sort_every):
    """HBM bytes per launch of the push kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None once the kernel's sources or the
    workload generator differ from the ones the counters were taken on, or
    the sort cadence differs."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel_key}_hbm_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if int(kv["sort_every"]) != int(sort_every):
            return None
        h = hashlib.sha256()
        for f in kv["kernel_sources"].split():
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != kv["kernel_sources_sha256"]:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def run_gpu(wl, prec, steps, warmup, log, repeats=5):
    """warmup untimed steps, then `repeats` timed runs of exactly `steps`
    steps each (HIP events on the library's stream, synchronized around each
    run); the reported figures are those of the median run."""
    import torch

    from paper_2511_17710_amd import picstep as P
    t0 = time.time()
    ctx = P.from_workload(wl, prec=prec, sort_every=wl.sort_every)
    dt = ctx.timestep_from_cfl(wl.cfl)
    torch.cuda.synchronize()
    log(f"[bench] {wl.name} {prec}: loaded {wl.nparticles} particles in {time.time() - t0:.1f}s, "
        f"dt={dt:.6g}")
    ctx.push_deposit(dt, warmup)
    torch.cuda.synchronize()
    s = ctx.stream
    n = wl.nparticles
    runs = []
    for _ in range(repeats):
        ctx.timing_enable(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        ctx.push_deposit(dt, steps)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        tm = ctx.timing_read()
        ctx.timing_enable(False)
        runs.append(dict(ms=ms, push_ms_avg=tm["push_ms"] / max(tm["push_launches"], 1),
                         push_launches=tm["push_launches"], sort_ms_total=tm["sort_ms"],
                         sort_calls=tm["sort_calls"],
                         global_deposits_per_block=round(
                             tm["push_global_particles"] / max(tm["push_blocks"], 1), 5)))
    med = sorted(runs, key=lambda r: r["ms"])[len(runs) // 2]
    res = dict(ms_per_step=med["ms"] / steps, ns_per_particle_step=med["ms"] * 1e6 / (n * steps),
               push_ms_avg=med["push_ms_avg"], push_launches=med["push_launches"],
               sort_ms_total=med["sort_ms_total"], sort_calls=med["sort_calls"],
               global_deposits_per_block=med["global_deposits_per_block"],
               repeats_ns_per_particle_step=[round(r["ms"] * 1e6 / (n * steps), 5) for r in runs])
    log(f"[bench] {wl.name} {prec}: {res}")
    del ctx
    torch.cuda.empty_cache()
    return res


def kernel_roofline_meta(meta, prec, r):
    """Algorithmic bytes of one launch of the fused step kernel over its
    average HIP-event duration, against the HBM peak."""
    n = meta["particles"]
    bpp = algorithmic_bytes_per_particle(meta["dim"], prec, meta["ncells"], n,
                                         meta["geom"] != "cart")
    ach = bpp * n / (r["push_ms_avg"] * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach / HBM_PEAK_GBS, 4), bytes_per_particle=round(bpp, 3),
                kernel_ms_avg=round(r["push_ms_avg"], 4))


def kernel_roofline(wl, prec, r):
    return kernel_roofline_meta(dict(particles=wl.nparticles, dim=wl.dim, geom=wl.geom,
                                     ncells=int(np.prod(wl.n[:wl.dim]))), prec, r)


def particle_sweep(wl, fractions, steps, warmup, log):
    """FP32 per-particle cost at fixed grid and fields for a random subset of
    every species (the particle-count dependence of the paper's Sec. 4)."""
    import copy
    rng = np.random.default_rng(4)
    out = []
    for f in fractions:
        sub = copy.copy(wl)
        sub.species = []
        for sp in wl.species:
            n = sp["cell"].shape[0]
            k = max(1, int(round(f * n)))
            pick = np.sort(rng.choice(n, size=k, replace=False)) if k < n else np.arange(n)
            sub.species.append({key: (v[pick] if isinstance(v, np.ndarray) else v)
                                for key, v in sp.items()})
        r = run_gpu(sub, "f32", steps, warmup, log, repeats=3)
        out.append(dict(fraction=f, particles=sub.nparticles,
                        ns_per_particle_step=round(r["ns_per_particle_step"], 5),
                        push_ms_avg=round(r["push_ms_avg"], 4)))
    return out


def adjoint_kernel_bytes_per_particle(dim, prec, ncells, nparticles):
    """Minimum HBM traffic of one reverse-step kernel launch per particle:
    the stored state read (cell, offsets, u, w), the momentum and offset
    adjoints read and written, the fields read and dL/d(fields)
    read-modify-written once per cell (dL/dJ, read on the last step only, is
    left out)."""
    b = 4 if prec == "f32" else 8
    state = 4 + dim * b + 3 * b + b
    lam = 2 * (3 * b + dim * b)
    grid = (6 * b + 2 * 6 * b) * ncells / nparticles
    return state + lam + grid


def run_adjoint(prec, log, name="cart3d_64_adj"):
    """Checkpointed forward (K steps, state every m, sorts at the workload's
    cadence inside the map) and the hand-written reverse sweep of
    L = sum(W * J_K) on the 3D Cartesian 64^3 workload."""
    import torch

    from paper_2511_17710_amd import picstep as P
    from paper_2511_17710_amd import workloads as W
    wl = W.by_name(name)
    K, m = wl.K, wl.ckpt_every
    ctx = P.from_workload(wl, prec=prec)  # the workload's sort cadence, inside the map
    dt = ctx.timestep_from_cfl(wl.cfl)
    lamJ = torch.from_numpy(wl.W).to(device="cuda", dtype=ctx.dtype)
    ctx.forward_checkpointed(dt, 2, 1)  # warm-up
    ctx.backward(dt, 2, 1, lamJ)
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    s = ctx.stream
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record(s)
    ctx.forward_checkpointed(dt, K, m)
    e[1].record(s)
    dEB, du0 = ctx.backward(dt, K, m, lamJ)
    e[2].record(s)
    torch.cuda.synchronize()
    tm = ctx.timing_read()
    n = wl.nparticles
    kms = tm["adjoint_ms"] / max(tm["adjoint_launches"], 1)
    bpp = adjoint_kernel_bytes_per_particle(wl.dim, prec, int(np.prod(wl.n[:wl.dim])), n)
    ach = bpp * n / (kms * 1e-3) / 1e9
    res = dict(workload=wl.name, particles=n, K=K, checkpoint_every=m, sort_every=wl.sort_every,
               forward_ns_per_particle_step=e[0].elapsed_time(e[1]) * 1e6 / (n * K),
               backward_ns_per_particle_step=e[1].elapsed_time(e[2]) * 1e6 / (n * K),
               adjoint_kernel_ms_avg=kms,
               roofline=dict(kernel="k_adjoint<0,3,%s>" % ("float" if prec == "f32" else "double"),
                             bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=round(ach / HBM_PEAK_GBS, 4), bytes_per_particle=round(bpp, 3)),
               grad_norm=float(dEB.double().norm()))
    log(f"[bench] adjoint {prec}: {res}")
    del ctx
    torch.cuda.empty_cache()
    return res


def run_fields(name, prec, log, calls=20):
    """The field solver on a workload's grid: Faraday (advance B), Ampere
    (advance E with the current) and one pass of the current filter, each
    timed over `calls` launches with HIP events on the library's stream;
    algorithmic bytes per updated lattice point: Faraday reads E and B and
    writes B (9 values), Ampere reads B, J and E and writes E (12), a filter
    pass reads and writes J (6)."""
    import torch

    from paper_2511_17710_amd import picstep as P
    from paper_2511_17710_amd import workloads as W
    wl = W.by_name(name)
    ctx = P.from_workload(wl, prec=prec)
    dt = ctx.timestep_from_cfl(wl.cfl)
    ctx.push_deposit(dt, 1)  # a current to filter and to couple
    b = 4 if prec == "f32" else 8
    n = list(wl.n[:wl.dim])
    pts = int(np.prod([v + (1 if wl.geom != "cart" else 0) for v in n]))
    s = ctx.stream
    ops = (("faraday", lambda: ctx.fields_advance_b(0.5 * dt), 9),
           ("ampere", lambda: ctx.fields_advance_e(dt), 12),
           ("filter", lambda: ctx.current_filter(1), 6))
    res = dict(workload=wl.name, updated_points=pts)
    for tag, fn, vals in ops:
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(calls):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / calls
        ach = vals * b * pts / (ms * 1e-3) / 1e9
        res[tag] = dict(ms=round(ms, 4), bytes_per_point=vals * b, achieved=round(ach, 1),
                        peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4))
    log(f"[bench] fields {name} {prec}: {res}")
    del ctx
    torch.cuda.empty_cache()
    return res


def cpu_baseline(wl, sample_per_species, steps, log):
    """FP64 CPU reference (single thread) on the first particles of each species."""
    from oracle import oracle as O
    g = O.make_grid(wl.geom, wl.dim, wl.n, wl.lo, wl.hi, r0=wl.r0, vartheta=wl.vartheta,
                    periodic=wl.periodic, rho0=wl.rho0)
    EB = O.fields_from_tetrad(g, wl.fields_tetrad, wl.fields_includes_ghosts)
    dt = O.dt_from_cfl(g, wl.cfl)
    sub = []
    for s in wl.species:
        k = min(sample_per_species, s["cell"].shape[0])
        sub.append({key: (v[:k] if isinstance(v, np.ndarray) else v) for key, v in s.items()})
    n = sum(x["cell"].shape[0] for x in sub)
    t0 = time.perf_counter()
    O.run(g, dt, steps, EB, sub, sort_every=wl.sort_every)
    el = time.perf_counter() - t0
    log(f"[bench] cpu reference: {n} particles x {steps} steps in {el:.1f}s")
    return dict(value=el * 1e9 / (n * steps), unit="ns/particle/step", cores=1, kind="oracle",
                sample=f"first {sample_per_species} particles of each of the 2 species of "
                       f"{wl.name} ({n} particles) x {steps} steps incl. the step-0 sort, "
                       f"FP64, single thread, host {os.uname().machine} nproc={os.cpu_count()}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--workload", default="cart3d_128")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--skip-adjoint", action="store_true")
    ap.add_argument("--skip-axisymmetric", action="store_true",
                    help="leave out the 1024x512 and 2048x1024 axisymmetric rows")
    ap.add_argument("--skip-fields", action="store_true",
                    help="leave out the field-solver rows")
    ap.add_argument("--skip-sweep", action="store_true",
                    help="leave out the particle-count sweep on the default grid")
    ap.add_argument("--sort-every", type=int, default=None,
                    help="override the workload's sort cadence (steps)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs the particle step on one GPU only; "
                                   "multi-GPU domain decomposition is a design note, not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    import torch

    from paper_2511_17710_amd import workloads as W
    t0 = time.time()
    wl = W.by_name(args.workload)
    if args.sort_every is not None:
        wl.sort_every = args.sort_every
    log(f"[bench] inputs {wl.name}: {wl.nparticles} particles in {time.time() - t0:.1f}s")

    if args.calib_copy_mb:
        nb = args.calib_copy_mb << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mb} MiB done")

    r32 = run_gpu(wl, "f32", args.steps, args.warmup, log, args.repeats)
    r64 = None if args.skip_fp64 else run_gpu(wl, "f64", args.steps, args.warmup, log,
                                              args.repeats)
    sweep = None
    if not args.skip_sweep and wl.name == "cart3d_128":
        sweep = particle_sweep(wl, (0.01, 0.03, 0.1, 0.3), args.steps, args.warmup, log)
    cpu = None if args.skip_cpu else cpu_baseline(wl, args.cpu_sample, args.cpu_steps, log)
    meta = dict(name=wl.name, dim=wl.dim, geom=wl.geom, grid=list(wl.n[:wl.dim]),
                ncells=int(np.prod(wl.n[:wl.dim])), particles=wl.nparticles,
                species=len(wl.species), sort_every=wl.sort_every, cfl=wl.cfl)
    del wl  # release the default workload's host arrays before the next ones
    axi = {}
    if not args.skip_axisymmetric and args.workload == "cart3d_128":
        for name in ("qsph_1024x512", "qsph_2048x1024"):
            w2 = W.by_name(name)
            row = {"particles": w2.nparticles, "grid": list(w2.n[:w2.dim]),
                   "sort_every": w2.sort_every}
            for prec in (("f32",) if args.skip_fp64 else ("f32", "f64")):
                r = run_gpu(w2, prec, args.steps, args.warmup, log, args.repeats)
                row[prec] = dict(ns_per_particle_step=round(r["ns_per_particle_step"], 5),
                                 ms_per_step=round(r["ms_per_step"], 4),
                                 repeats_ns_per_particle_step=r["repeats_ns_per_particle_step"],
                                 roofline=kernel_roofline(w2, prec, r))
            if "f64" in row:
                row["fp32_vs_fp64_speedup"] = round(
                    row["f64"]["ns_per_particle_step"] / row["f32"]["ns_per_particle_step"], 3)
            axi[name] = row
            del w2
    adj = None
    if not args.skip_adjoint:
        adj = {p: run_adjoint(p, log) for p in (("f32",) if args.skip_fp64 else ("f32", "f64"))}
    fields = None
    if not args.skip_fields and args.workload == "cart3d_128":
        precs = ("f32",) if args.skip_fp64 else ("f32", "f64")
        fields = {name: {p: run_fields(name, p, log) for p in precs}
                  for name in ("cart3d_128", "qsph_2048x1024")}
    emit(args, meta, dict(r32=r32, r64=r64, sweep=sweep, cpu=cpu, axi=axi, adj=adj,
                          fields=fields))


def emit(args, meta, f):
    r32, r64 = f["r32"], f["r64"]
    n = meta["particles"]
    roof = kernel_roofline_meta(meta, "f32", r32)
    traffic = (measured_traffic(f"k_push_{meta['name']}", meta["sort_every"])
               if meta["name"] == "cart3d_128" else None)
    roof.update({"traffic": traffic,
                 "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                 "traffic_GBs": (round(traffic / (r32["push_ms_avg"] * 1e-3) / 1e9, 1)
                                 if traffic else None),
                 "kernel": "k_push<%d,%d,float,false,false>" % (
                     {"cart": 0, "sph": 1, "qsph": 2}[meta["geom"]], meta["dim"])})
    out = {
        "metric": "ns/particle/step push+deposit (fwd, adjoint) FP32 vs FP64; HBM GB/s vs peak",
        "value": round(r32["ns_per_particle_step"], 5),
        "unit": "ns/particle/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": meta["name"], "grid": meta["grid"], "particles": n,
                   "species": meta["species"], "sort_every": meta["sort_every"],
                   "cfl": meta["cfl"], "offsets": "u32 fixed point (f32 build)",
                   "repeats": args.repeats, "value_is": "median of the repeats"},
        "roofline": roof,
        "fp32": r32,
    }
    if r64:
        r64["roofline"] = kernel_roofline_meta(meta, "f64", r64)
        out["fp64"] = r64
        out["fp32_vs_fp64_speedup"] = round(r64["ns_per_particle_step"] / r32["ns_per_particle_step"], 3)
    if f["axi"]:
        out["axisymmetric"] = f["axi"]
    if f["sweep"]:
        out["particle_sweep_fp32"] = f["sweep"] + [dict(fraction=1.0, particles=n,
                                                        ns_per_particle_step=round(r32["ns_per_particle_step"], 5),
                                                        push_ms_avg=round(r32["push_ms_avg"], 4))]
    if f["adj"]:
        out["adjoint"] = f["adj"]
    if f.get("fields"):
        out["field_solver"] = f["fields"]
    if f["cpu"]:
        out["cpu_baseline"] = f["cpu"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
