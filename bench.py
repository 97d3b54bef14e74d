#!/usr/bin/env python
"""Benchmark of one coupled lattice-Boltzmann + DEM step on one MI355X.

Workload (default): large 3D bulk suspension, 256^3 D3Q19 lattice, Lees-Edwards simple
shear at 1e-4, bidisperse spheres of radii 4.5/6.3 (1:1) at volume fraction 0.55, i.e.
12,914 spheres, seeded synthetic packing; FP32 populations (FP64 particles).

Prints one JSON line: whole-step throughput in MLUPS (all lattice nodes per second); the
roofline of the lattice update (with spheres one kernel, k_lattice: the boundary links
and their forces, then pull-stream and collision of the same brick; timed with HIP events on
the simulation's stream) against the algorithmic bytes of the fluid nodes; the same with FP16 storage of the
populations; the FP64 CPU oracle timed on the host's cores (20 steps of this workload on
every thread, one step on one thread, and the small configurations); and the serving
comparison: the same mixed requests served one at a time by the plain loop and by the
batched server (jobs per hour, p50/p99 latency).
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

METRIC = "MLUPS & % HBM roofline; batched jobs/hr + p99 latency vs plain loop"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per fluid node update: 19 populations read + 19 written + owner word
BYTES_PER_FLUID = {"fp64": 38 * 8 + 4, "fp32": 38 * 4 + 4, "fp16store": 38 * 2 + 4}
PREC = {"fp64": 0, "fp32": 1, "fp16store": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16store": "f32 (f16 storage)"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def workload(name):
    from paper_1904_02929_amd import synth
    if name == "large3d":
        w = synth.bulk3d(256, 0.55, 1e-4, seed=1)
        return w, "large_3d_bulk_256cube_phi0.55"
    if name == "bulk96":
        w = synth.bulk3d(96, 0.55, 1e-3, seed=1)
        return w, "bulk_3d_96cube_phi0.55"
    if name == "walls256":
        w = synth.walled3d(256, 0.50, 1e-4, seed=1)
        return w, "walled_3d_256cube_phi0.50"
    if name == "empty256":
        from paper_1904_02929_amd.synth import Workload
        import numpy as np
        w = Workload("empty256", (256, 256, 256), np.zeros((0, 3)), np.zeros((0, 3)),
                     np.zeros((0, 3)), np.zeros(0), dict(shear_kind=1, gamma_dot=1e-4))
        return w, "pure_fluid_256cube"
    raise SystemExit("unknown workload " + name)


def traffic_for(kernel_key, src_hash):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source."""
    path = os.path.join(ROOT, "profiles", kernel_key + "_hbm_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_sha256") != src_hash:
        return None
    return d.get("bytes_per_launch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Thread count for oracles created from now on (the oracle takes omp_get_max_threads
    when it is created)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def _time_oracle(w, steps):
    import numpy as np
    from oracle import oracle as O
    p = O.make_params(lx=w.box[0], ly=w.box[1], lz=w.box[2], **w.params)
    t0 = time.perf_counter()
    o = O.Oracle(p, w.pos, w.vel, w.omega, w.radius, wall=w.wall)
    t1 = time.perf_counter()
    rc = o.step(steps)
    t2 = time.perf_counter()
    nodes = float(np.prod(w.box))
    return {"mlups": nodes * steps / (t2 - t1) / 1e6, "s_per_step": (t2 - t1) / steps,
            "setup_s": t1 - t0, "threads": int(o.s.nthreads), "status": int(rc)}


def cpu_baseline(w, steps):
    """The FP64 oracle on the host: `steps` steps of the benchmark workload on every thread
    (the reported value), one step of it on one thread, and a few steps of the small
    configurations (single sphere 32^3 FP64; 3D bulk 96^3 at phi 0.55; quasi-2D monolayer
    256 x 256 x 10 at area fraction 0.78)."""
    from paper_1904_02929_amd import synth
    ncpu = os.cpu_count()
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = ncpu
    full = _time_oracle(w, steps)
    small = {}
    for key, wl, n in (("single_sphere_32cube", synth.single_sphere(32, 4.5, 1e-4), 50),
                       ("bulk_3d_96cube_phi0.55", synth.bulk3d(96, 0.55, 1e-3, seed=1), 10),
                       ("monolayer_256x256x10_phi0.78", synth.monolayer(256, 10, 0.78, seed=1), 20)):
        r = _time_oracle(wl, n)
        small[key] = {"mlups": round(r["mlups"], 3), "s_per_step": round(r["s_per_step"], 5), "steps": n}
    one = None
    if _omp_threads(1):
        r = _time_oracle(w, 1)
        one = {"mlups": round(r["mlups"], 3), "s_per_step": round(r["s_per_step"], 3),
               "threads": r["threads"]}
        _omp_threads(full["threads"])
    return {
        "value": round(full["mlups"], 3),
        "unit": "MLUPS",
        "cores": full["threads"],
        "kind": "oracle",
        "sample": "%d steps of the same workload measured (FP64, all lattice nodes), after a "
                  "%.1f s set-up; %.3f s per step; status %d" % (steps, full["setup_s"],
                                                                full["s_per_step"], full["status"]),
        "cpu_model": _cpu_model(),
        "nproc": ncpu,
        "cpus_available": avail,
        "one_thread": one,
        "small_configs": small,
    }


def lattice_run(susp, torch, w, args, precision, steps, warmup):
    """Steps the workload with one storage precision; returns the timing of the whole step
    and of the two lattice kernels."""
    import numpy as np
    kw = dict(w.params)
    if args.brick:
        kw["brick_y"], kw["brick_z"] = (int(v) for v in args.brick.lower().split("x"))
    p = susp.make_params(w.box, radius=w.radius, pos=w.pos, vel=w.vel, omega=w.omega,
                         precision=PREC[precision], contact_bins=args.contact_bins, wall=w.wall,
                         lub_implicit=args.lub_implicit, n_sub=args.n_sub,
                         collision=1 if args.collision == "multi" else 0, tau_bulk=0.75, tau_ghost=1.0,
                         **kw)
    sim = susp.Simulation(p)
    stream = sim.stream
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.profile(True)
    sim.profile_read_parts()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    rc = sim.step(steps, check=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    links_ms, stream_ms, k_n = sim.profile_read_parts()
    sim.profile(False)
    own = sim.lists(susp.LIST_OWNER)
    n_fluid = int((own == -1).sum())
    health = sim.health()
    sim.close()
    nodes = int(np.prod(w.box))
    k_links = links_ms / max(1, k_n)
    k_stream = stream_ms / max(1, k_n)
    alg = n_fluid * BYTES_PER_FLUID[precision]
    return {"ms": ms, "rc": int(rc), "nodes": nodes, "n_fluid": n_fluid, "k_links_ms": k_links,
            "k_stream_ms": k_stream, "alg_bytes": alg, "n_sub": int(p.n_sub), "health": health,
            "mlups": nodes * steps / (ms / 1e3) / 1e6}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=sorted(PREC))
    ap.add_argument("--workload", default="large3d", choices=["large3d", "bulk96", "walls256", "empty256"])
    ap.add_argument("--collision", default="bgk", choices=["bgk", "multi"],
                    help="eq. 5 as BGK, or the multi-eigenvalue operator (tau_bulk 0.75, "
                         "tau_ghost 1: ghost modes projected out)")
    ap.add_argument("--lub-implicit", type=int, default=0,
                    help="Jacobi sweeps of the implicit squeeze lubrication per substep (0: explicit)")
    ap.add_argument("--n-sub", type=int, default=8, help="DEM substeps per lattice step")
    ap.add_argument("--brick", default="",
                    help="stream brick BYxBZ (e.g. 8x8; 4x4 fuses the link and stream kernels); "
                         "default: the library's choice")
    ap.add_argument("--contact-bins", type=int, default=0,
                    help="also sample the contact statistics every step in this many bins")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp16-line", action="store_true",
                    help="skip the second run of the workload with FP16 storage")
    ap.add_argument("--serve-jobs", type=int, default=64,
                    help="requests in the serving comparison (0: skip it)")
    ap.add_argument("--serve-steps", type=int, default=1000, help="lattice steps per request")
    ap.add_argument("--serve-budget-gib", type=float, default=32.0,
                    help="HBM budget of the batched server (GiB)")
    ap.add_argument("--serve-mode", default="lockstep", choices=["lockstep", "streams"],
                    help="batched server: lockstep runs with one launch per kernel over all jobs, "
                         "or one stream per job")
    ap.add_argument("--mix-probe", action="store_true",
                    help="only time the serving mix (--serve-jobs requests, 24 if 0): every job alone "
                         "against one lockstep step of all of them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device-to-device copy of 1 GiB five times (the "
                         "reference kernel for scaling the HBM byte counters)")
    args = ap.parse_args()
    if args.serve_mode == "streams":
        # one stream per job: give them their own hardware queues (read by the HIP runtime when
        # it starts, so set before torch is imported; 32 measured best of 8, 16, 32).  The
        # lockstep server keeps the runtime's default: with 32 queues its launches took ~15x
        # longer on the host and its runs twice as long.
        os.environ["GPU_MAX_HW_QUEUES"] = "32"
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the lattice would shard "
              "into z-slabs with halo planes exchanged over RCCL). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1904_02929_amd import susp

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": src.numel() * 4,
                          "copy_bytes_written_per_launch": src.numel() * 4, "launches": 5}))
        return
    if args.mix_probe:
        from paper_1904_02929_amd import serve
        print(json.dumps(serve.lockstep_probe(n_jobs=args.serve_jobs or 24, log=log)))
        return
    t = time.perf_counter()
    w, wname = workload(args.workload)
    log("workload %s: box %s, %d spheres (%.1f s to generate)" % (wname, w.box, w.n, time.perf_counter() - t))
    r = lattice_run(susp, torch, w, args, args.precision, args.steps, args.warmup)
    log("timed %d steps in %.1f ms (status %d)" % (args.steps, r["ms"], r["rc"]))
    alt = None
    if not args.no_fp16_line and args.precision == "fp32":
        r16 = lattice_run(susp, torch, w, args, "fp16store", args.steps, args.warmup)
        log("FP16 storage: %d steps in %.1f ms (status %d)" % (args.steps, r16["ms"], r16["rc"]))
        lat16 = r16["k_links_ms"] + r16["k_stream_ms"]
        alt = {
            "precision": "fp16store",
            "dtype": DTYPE["fp16store"],
            "value": round(r16["mlups"], 2),
            "unit": "MLUPS",
            "ms_per_step": round(r16["ms"] / args.steps, 5),
            "lattice_ms": round(lat16, 5),
            "lattice_frac": round(r16["alg_bytes"] / (lat16 / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "status": r16["rc"],
        }
    per_step = r["ms"] / args.steps
    lat_ms = r["k_links_ms"] + r["k_stream_ms"]
    achieved = r["alg_bytes"] / (lat_ms / 1e3) / 1e9
    with open(os.path.join(ROOT, "paper_1904_02929_amd", "csrc", "fluid.hip"), "rb") as fh:
        src_hash = hashlib.sha256(fh.read()).hexdigest()
    kernel_key = "lattice_%s_%s%s" % (wname, args.precision, "_multi" if args.collision == "multi" else "")
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on %d steps" % args.cpu_steps)
        cpu = cpu_baseline(w, args.cpu_steps)
    serving = None
    if args.serve_jobs > 0:
        from paper_1904_02929_amd import serve
        log("serving %d requests of %d steps: plain loop, then the batched server"
            % (args.serve_jobs, args.serve_steps))
        serving = serve.serve_benchmark(n_jobs=args.serve_jobs, steps=args.serve_steps, log=log,
                                        mode=args.serve_mode, budget=int(args.serve_budget_gib * (1 << 30)))
        serving["workload"] = ("mixed requests: half quasi-2D monolayers L x L x 10 (L 128-384, "
                               "area fraction 0.70-0.80, oscillatory), half 3D bulk L^3 "
                               "(L 64-128, phi 0.50-0.56, simple shear); Poisson arrivals at "
                               "jobs / (0.25 x plain-loop time); FP32")

    coll = "BGK" if args.collision == "bgk" else "multi-eigenvalue"
    # with spheres and the default 64 x 4 x 4 bricks one kernel (k_lattice) does both parts and
    # the stream events enclose nothing
    fused = r["k_stream_ms"] < 0.02 * max(r["k_links_ms"], 1e-9)
    kname = ("k_lattice (link list, bounce-back and link forces, then pull-stream and %s collision of "
             "the same 64x4x4 brick)" % coll) if fused else (
             "lattice update: k_links (link list, bounce-back, link forces) + k_stream "
             "(pull-stream, %s collision)" % coll)
    out = {
        "metric": METRIC,
        "value": round(r["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {
            "workload": wname,
            "lattice": list(w.box),
            "spheres": int(w.n),
            "radii": [4.5, 6.3] if w.n else [],
            "phi": (0.50 if args.workload == "walls256" else 0.55) if w.n else 0.0,
            "boundary": "walls" if w.params.get("boundary") == 1 else "lees-edwards",
            "shear_rate": w.params.get("gamma_dot"),
            "precision": args.precision,
            "n_sub": r["n_sub"],
            "lub_implicit": int(args.lub_implicit),
            "collision": args.collision,
            "contact_bins": int(args.contact_bins),
            "status": r["rc"],
        },
        "fluid_mlups": round(r["n_fluid"] * args.steps / (r["ms"] / 1e3) / 1e6, 2),
        "particle_steps_per_s": round(w.n * args.steps / (r["ms"] / 1e3), 1),
        "roofline": {
            "kernel": kname,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_for(kernel_key, src_hash),
            "avg_kernel_ms": round(lat_ms, 5),
            "algorithmic_bytes_per_launch": int(r["alg_bytes"]),
            "bytes_per_fluid_node": BYTES_PER_FLUID[args.precision],
            "fluid_nodes": r["n_fluid"],
            "parts": None if fused else {
                "k_links_ms": round(r["k_links_ms"], 5),
                "k_stream_ms": round(r["k_stream_ms"], 5),
                "k_stream_frac": round(r["alg_bytes"] / (r["k_stream_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            },
        },
        "fp16_storage": alt,
        "health": {"fast_node_steps": r["health"][0], "max_u_over_cs": round(r["health"][1], 4),
                   "mass_drift": r["health"][2]},
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
