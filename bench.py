"""Benchmark: geodesic distance solves on a 10.5M-vertex mesh on one MI355X.

Workload: the level-10 icosphere (10,485,762 vertices, 20,971,520 faces)
radially displaced by a seeded sum of 8 real spherical harmonics of degree
<= 16 (r = 1 + 0.05 S/max|S|), one seeded source, t = hbar^2, edge-projected
gradient formulation.  One step = one whole solve through the C ABI
(breadth-first sets, FP64 diffusion sweeps to convergence, normalisation,
edge ADMM to convergence, compensated integration), with the mesh resident
in HBM before timing starts.

Prints one JSON line.  `value` = solves per second; the roofline object is
for the dominant kernel, its average duration measured with HIP events on
the solve's stream during the timed steps; `cpu_baseline` times the CPU
oracle on a bounded sample (two smaller meshes of the same family, levels 7
and 8) and scales it to the workload with the growth measured between them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "ms/solve + HBM GB/s on 10M-vert mesh; batched queries/s, p50/p99 at ≤1e-3 err"


def _mesh(level: int, cache_dir: str | None):
    import meshgen
    name = f"bumpy{level}"
    path = os.path.join(cache_dir, f"{name}.npz") if cache_dir else None
    if path and os.path.exists(path):
        z = np.load(path)
        return z["v"], z["f"], z["s"]
    if level in (9, 10, 12):
        v, f, s = meshgen.config_mesh(name)
    else:
        v, f = meshgen.icosphere(level)
        v = meshgen.harmonic_displacement(v, seed=3)
        s = meshgen.random_sources(v.shape[0], 1, seed=104)
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        np.savez(path, v=v, f=f, s=s)
    return v, f, s


def _measured_traffic(kernel: str, per: str = "launch"):
    """HBM bytes per launch (or per diffusion pass, one launch per tile
    colour) of `kernel` from the committed rocprofv3 PMC record
    (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB
    copy), or None when the kernel's source changed since then."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["src"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["src_sha256"]:
        return None
    return rec.get("bytes_per_" + per)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(levels, full_nv: int):
    """The oracle as it stands (FP64 banded-LU diffusion, edge-form Poisson by
    multigrid CG, single-threaded scipy) timed on this host on displaced
    icospheres of two smaller levels.  The value is solves/s of the full
    workload, from the larger level's measured time and the growth exponent
    measured between the two levels, T ~ V^k (k >= 1)."""
    from oracle import pipeline
    times, sizes = [], []
    for lvl in levels:
        v, f, s = _mesh(lvl, None)
        t0 = time.perf_counter()
        pipeline.heat_method(v, f, s, form="edge", diffusion_route="bands")
        times.append(time.perf_counter() - t0)
        sizes.append(v.shape[0])
        print(f"[bench] oracle level {lvl} ({v.shape[0]} vertices): {times[-1]:.2f} s", file=sys.stderr, flush=True)
    k = max(1.0, float(np.log(times[-1] / times[0]) / np.log(sizes[-1] / sizes[0]))) if len(levels) > 1 else 1.0
    full_s = times[-1] * (full_nv / sizes[-1]) ** k
    return {"value": 1.0 / full_s, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus_available": len(os.sched_getaffinity(0)),
            "sample": (f"one full oracle solve (banded-LU FP64 diffusion, edge Poisson by multigrid CG, one "
                       f"thread) on displaced icospheres of levels {', '.join(map(str, levels))} "
                       f"({', '.join(map(str, sizes))} vertices): "
                       f"{', '.join(f'{x:.2f}' for x in times)} s; scaled to {full_nv} vertices as "
                       f"T ~ V^{k:.2f} from the two measured points"),
            "measured_s": dict(zip(map(str, levels), times)), "growth_exponent": k}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=10)
    ap.add_argument("--form", default="edge", choices=["edge", "face"])
    ap.add_argument("--cache", default=os.environ.get("HGEO_MESH_CACHE", "/tmp/hgeo_mesh_cache"))
    ap.add_argument("--cpu-sample-levels", default="7,8",
                    help="icosphere levels the oracle is timed on for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default diffusion schedule instead of tuning it on the first query")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch measurement (256 small meshes in one solve)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving measurement (Poisson stream over a pool of resident meshes)")
    ap.add_argument("--admm-block", type=int, default=0,
                    help="edge-form ADMM iterations per launch (hg_opts.admm_block; 0 = auto)")
    ap.add_argument("--serve-levels", default="4-8")
    ap.add_argument("--serve-queries", type=int, default=100)
    ap.add_argument("--serve-rate", type=float, default=1.5,
                    help="offered load as a multiple of the plain path's saturation rate")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run 5 device-to-device copies of 1 GiB (scale for PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solve is a single-GPU kernel pipeline "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1812_06060_amd as hg
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_calib:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "copies": 5}))
        return

    t0 = time.perf_counter()
    v, f, src = _mesh(args.level, args.cache)
    t_gen = time.perf_counter() - t0
    print(f"[bench] mesh level {args.level}: V={v.shape[0]} F={f.shape[0]} generated in {t_gen:.1f}s",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    mesh = hg.Mesh(v, f)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    print(f"[bench] mesh_create {t_create:.2f}s hbar={mesh.hbar:.4e}", file=sys.stderr, flush=True)
    opts = hg.default_opts(formulation=args.form, admm_block=args.admm_block)
    out = torch.empty(mesh.nv, dtype=torch.float32, device="cuda")
    tune = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tune = mesh.autotune(src, 0.0, opts)
        ch = tune["candidates"][tune["chosen"]]
        def label(c):
            return {1: "jacobi", 2: f"tiles/{c['inner_sweeps']}",
                    3: f"overlap{c.get('overlap_rings', 0)}-tiles/{c['inner_sweeps']}"}.get(c["schedule"], "?")
        print(f"[bench] autotune ({time.perf_counter() - t0:.1f}s): " +
              ", ".join(f"{label(c)}={c['ms']:.0f}ms ({c['passes']} passes)" for c in tune["candidates"]) +
              f" -> {label(ch)}", file=sys.stderr, flush=True)
        if tune["admm"]:
            print("[bench] autotune ADMM block: " +
                  ", ".join(f"{a['block']}={a['us_per_iteration']:.1f}us/it" for a in tune["admm"]) +
                  f" -> {tune['admm'][tune['admm_chosen']]['block']}", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        _, info = mesh.solve(src, 0.0, opts, out=out)
        print(f"[bench] warmup {i}: {info.ms_total:.1f} ms sweeps={info.sweeps} admm={info.admm_iters}",
              file=sys.stderr, flush=True)

    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, info = mesh.solve(src, 0.0, opts, out=out)
        infos.append(info)
        print(f"[bench] step {i}: {info.ms_total:.1f} ms (bfs {info.ms_bfs:.1f} diff {info.ms_diffusion:.1f} "
              f"norm {info.ms_normalize:.2f} admm {info.ms_admm:.1f} int {info.ms_integrate:.2f}) "
              f"sweeps={info.sweeps} admm={info.admm_iters}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per = 1000.0 * wall / args.steps

    # dominant kernel: the one with the larger share of device time
    diff_ms = float(np.mean([i.ms_pass_kernel * i.passes for i in infos]))
    admm_ms = float(np.mean([i.ms_admm_kernel * i.admm_launches for i in infos]))
    block = infos[-1].admm_block
    if diff_ms >= admm_ms:
        name = "diffusion pass"
        kms = float(np.mean([i.ms_pass_kernel for i in infos]))
        kbytes = infos[-1].bytes_pass_kernel
    else:
        name = (f"{args.form} ADMM launch ({block} iterations over LDS tiles)" if block > 1
                else f"{args.form} ADMM iteration")
        kms = float(np.mean([i.ms_admm_kernel for i in infos]))
        kbytes = infos[-1].bytes_admm_kernel
    achieved = kbytes / (kms * 1e-3) / 1e9
    if name == "diffusion pass":
        kname = "k_patch_pass"
    elif args.form == "face":
        kname = "k_admm_face"
    else:
        kname = "k_admm_edge_tiled" if block > 1 else "k_admm_edge"
    traffic = _measured_traffic(kname, "pass" if kname == "k_patch_pass" else "launch")
    last = infos[-1]
    result = {
        "metric": METRIC,
        "value": 1000.0 / ms_per,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 diffusion / f32 ADMM+integration",
        "data": "synthetic",
        "config": {"workload": f"displaced icosphere L{args.level} ({mesh.nv} vertices, {mesh.nf} faces), "
                               f"1 source, t=hbar^2, {args.form} form, tol_u={opts.tol_u:g}, "
                               f"tol_admm={opts.tol_admm:g}",
                   "sweeps": last.sweeps, "admm_iters": last.admm_iters, "admm_block": last.admm_block,
                   "admm_launches": last.admm_launches, "bfs_depth": last.bfs_depth,
                   "stage_ms": {"bfs": last.ms_bfs, "diffusion": last.ms_diffusion,
                                "normalize": last.ms_normalize, "admm": last.ms_admm,
                                "integrate": last.ms_integrate},
                   "mesh_create_s": t_create,
                   "diffusion_schedule": (None if tune is None else
                                          tune["candidates"][tune["chosen"]]),
                   "hbm_bytes_per_vertex": (mesh.stats["mesh_bytes"] + last.workspace_bytes) / mesh.nv,
                   "mesh_bytes": mesh.stats["mesh_bytes"], "query_workspace_bytes": last.workspace_bytes},
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_kernel_ms": kms, "alg_bytes_per_launch": int(kbytes)},
        # the blocked edge ADMM runs several iterations per launch: its time per
        # iteration against the HBM time of one iteration per launch (49 B per
        # face read and written once at 8 TB/s)
        "admm_per_iteration": (None if args.form != "edge" else {
            "iterations_per_launch": block,
            "us": 1e3 * float(np.mean([i.ms_admm_kernel * i.admm_launches / i.admm_iters for i in infos])),
            "single_iteration_hbm_bound_us": 49.0 * mesh.nf / (HBM_PEAK_GBS * 1e9) * 1e6}),
        "alg_hbm_gbs_whole_solve": last.bytes_alg / (last.ms_total * 1e-3) / 1e9,
    }
    mesh.close()
    del out
    if not args.no_batch:
        from paper_1812_06060_amd import batch_bench
        print("[bench] batch of 256 small meshes ...", file=sys.stderr, flush=True)
        result["batch"] = batch_bench.run(256, args.form, log=lambda m: print(m, file=sys.stderr, flush=True))
    if not args.no_serving:
        from paper_1812_06060_amd import serving_bench
        lo, hi = (int(x) for x in args.serve_levels.split("-"))
        print("[bench] serving ...", file=sys.stderr, flush=True)
        result["serving"] = serving_bench.run((lo, hi), 32, args.serve_queries, 16, args.serve_rate, 4,
                                              log=lambda m: print(m, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline([int(x) for x in args.cpu_sample_levels.split(",")], v.shape[0])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
