"""Benchmark: recursive spectral bisection of an 8M-element hex mesh into 4096
parts on one MI355X.

Workload: 256 x 256 x 128 hex box with 10% of the elements removed in
spherical clusters and vertex ids randomly renumbered onto 64-bit values
(7,549,747 elements), partitioned into 4096 parts by batched RSB with the
mixed-precision Lanczos solver.  Inputs are resident in HBM (torch tensors)
before the timed region; one step is one whole partition: dual graph, then
12 levels of components, Lanczos, split and compaction.

Prints one JSON line.  value = Lanczos iterations per second, counting one
iteration per batched Lanczos step (one launch sequence over all subgraphs
of a level); ms_per_step = time to the 4096-way partition.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Lanczos iters/s + SpMV HBM GB/s; time to 4096-way RSB at matched edge cut"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "box256x256x128-clustered10-renum-4096": dict(nparts=4096),
    "box256x256x64-holes3-1024": dict(nparts=1024),
    "box128x128x64-holes5-2": dict(nparts=2),
}


def make_mesh(name):
    import meshgen as mg
    if name.startswith("box256x256x128"):
        return mg.box256x128_clustered10()
    if name.startswith("box256x256x64"):
        return mg.box256_holes3()
    if name.startswith("box128x128x64"):
        return mg.box128_holes5()
    raise ValueError(name)


def cpu_baseline(mesh, seconds_target=20.0):
    """The CPU oracle on a bounded sample of the workload: one Lanczos cycle
    (m = 100) on the dual graph of a sub-box of the same mesh (its first
    elements in lexicographic order), scaled to iterations/s on the full
    mesh by the element ratio (the work per iteration is linear in n)."""
    import numpy as np

    import oracle
    frac = 1.0 / 64.0
    n_sample = max(2, int(mesh.nelem * frac))
    ids = mesh.ids[:n_sample]
    rp, col, w = oracle.dual_graph(ids)
    t0 = time.perf_counter()
    st, lam, y, info = oracle.fiedler_csr(rp, col, w, np.arange(n_sample), lanczos_m=100,
                                          max_restarts=0, tol=1e-12)
    dt = time.perf_counter() - t0
    steps = 100
    iters_per_s_sample = steps / dt
    return {"value": iters_per_s_sample * n_sample / mesh.nelem, "unit": "Lanczos iterations/s",
            "cores": 1, "kind": "oracle",
            "sample": (f"one 100-step Lanczos cycle (FP64, full reorthogonalisation) on the dual "
                       f"graph of the first {n_sample} elements of the same mesh, {dt:.1f} s; "
                       f"scaled by {n_sample}/{mesh.nelem} elements"),
            "cpu": platform.processor() or platform.machine()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="box256x256x128-clustered10-renum-4096",
                    choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--tol", type=float, default=1e-2)
    ap.add_argument("--m", type=int, default=100)
    ap.add_argument("--max-restarts", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", type=int, default=0)
    ap.add_argument("--unbatched", action="store_true")
    ap.add_argument("--rows-per-thread", type=int, default=0, choices=[0, 2, 4, 8])
    ap.add_argument("--autotune", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--autotune-cache", default=None)
    ap.add_argument("--no-profile", action="store_true",
                    help="time the steps with graph replay and no kernel timing (no roofline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2606_14659_amd as rsb

    wl = WORKLOADS[args.workload]
    mesh = make_mesh(args.workload)
    print(f"[bench] {args.workload}: {mesh.nelem} elements", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    ids = torch.as_tensor(mesh.ids).cuda()
    part = torch.empty(mesh.nelem, dtype=torch.int32, device="cuda")
    opts = dict(precision=args.precision, tol=args.tol, lanczos_m=args.m,
                max_restarts=args.max_restarts, verbose=args.verbose,
                batched=0 if args.unbatched else 1, rows_per_thread=args.rows_per_thread,
                autotune=args.autotune)
    if args.autotune_cache:
        opts["autotune_cache"] = args.autotune_cache

    def one_step(profile):
        o = rsb.make_opts(True, profile=1 if profile else 0, **opts)
        st = rsb.Stats()
        st.struct_size = rsb.C.sizeof(rsb.Stats)
        code = rsb.lib().rsb_partition(mesh.nelem, mesh.nv, rsb.C.c_void_p(ids.data_ptr()),
                                       wl["nparts"], rsb.C.byref(o),
                                       rsb.C.c_void_p(part.data_ptr()), rsb.C.byref(st))
        rsb._check(code, "rsb_partition")
        return code, st.as_dict()

    for i in range(args.warmup):
        code, st = one_step(False)
        print(f"[bench] warmup {i}: {st['ms_total']:.0f} ms, status {code}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_steps = 0
    kern_ms = kern_bytes = 0.0
    kern_launches = 0
    last = None
    for i in range(args.steps):
        code, st = one_step(not args.no_profile)
        total_steps += st["level_steps"]
        kern_ms += st["kernel_ms"]
        kern_bytes += st["kernel_bytes"]
        kern_launches += st["kernel_launches"]
        last = (code, st)
        print(f"[bench] step {i}: {st['ms_total']:.0f} ms, {st['level_steps']} level-steps, "
              f"status {code}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    code, st = last
    sizes = np.bincount(part.cpu().numpy(), minlength=wl["nparts"])
    achieved = kern_bytes / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": total_steps / dt,
        "unit": "Lanczos iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "elements": mesh.nelem, "nparts": wl["nparts"],
                   "precision": args.precision, "lanczos_m": args.m, "tol": args.tol,
                   "max_restarts": args.max_restarts, "graph": "weighted vertex-shared",
                   "batched": not args.unbatched},
        "time_to_partition_ms": dt * 1e3 / args.steps,
        "edge_cut": st["edge_cut"],
        "cut_pairs": st["cut_pairs"],
        "max_neighbors": st["max_neighbors"],
        "avg_neighbors": st["avg_neighbors"],
        "part_sizes": [int(sizes.min()), int(sizes.max())],
        "status": code,
        "not_converged_segments": st["not_converged"],
        "level_steps_per_partition": st["level_steps"],
        "ms_graph": st["ms_graph"],
        "ms_solve": st["ms_solve"],
        "ms_split": st["ms_split"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": (f"k_lz_project (SpMV + projection, Lanczos steps j>=3), "
                                f"{st['tile_rows']}-row tiles at level 0"),
                     "launches": kern_launches,
                     "avg_us": kern_ms * 1e3 / max(kern_launches, 1)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
