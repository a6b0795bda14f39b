"""Writes config_goldens.json: the oracle's results on the full-size benchmark
meshes, which the full-size GPU tests and bench.py compare against.

Calls only the oracle (oracle/) and the seeded mesh generators (meshgen/).
Nothing here reads a GPU result.  The oracle is FP64 throughout and its
element loops use fixed-order sums, so the numbers do not depend on the
thread count.

What is computed (paper Sec. 4 eigenproblem, Sec. 6 restarted Lanczos,
Alg. 1 recursion):
  c2            128x128x64 box, 5% uniform holes: lambda_2 by thick-restart
                Lanczos to ||L y - rho y|| <= 1e-10 rho.
  c3_level0     256x256x64 box, 3% uniform holes: lambda_2 of the whole mesh
                (the first bisection of the 1024-way partition), 1e-8.
  c3_rsb1024    the same mesh into 1024 parts, every bisection to 1e-6.
  c5a_level0    256x256x128 box, 10% clustered holes, renumbered ids: lambda_2
                of the whole mesh, 1e-8.
  c5a_rsb4096   the same mesh into 4096 parts, every bisection to 1e-6.
  c5b_rsb16     four meshes of the 64-mesh batch (the smallest, index 0, the
                median and the largest) into 16 parts each, 1e-6.
Every solve is thick-restart Lanczos (cycles of 40 steps keeping 8 Ritz
pairs) with the warm start of child subgraphs from the parent's second Ritz
vector, the settings the partitioner's benchmark uses, at tight tolerances
and a restart cap (400) that the tolerances never reach.

Usage:  python tests/golden/make_config_goldens.py [--threads N] [names...]
(the default is every entry; existing entries of other names are kept).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import meshgen as mg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "config_goldens.json")
SOLVER = dict(lanczos_m=40, lanczos_keep=8, warm_start=1, max_restarts=400)


def _c5b_sample():
    meshes = mg.batch64()
    sizes = np.array([m.nelem for m in meshes])
    order = np.argsort(sizes, kind="stable")
    picks = sorted({int(order[0]), 0, int(order[len(order) // 2]), int(order[-1])})
    return meshes, picks


def fiedler_entry(mesh_name, mesh, tol):
    t0 = time.perf_counter()
    st, lam, y, info = oracle.fiedler(mesh.ids, tol=tol, **SOLVER)
    dt = time.perf_counter() - t0
    return {"mesh": mesh_name, "elements": int(mesh.nelem), "solver": dict(SOLVER, tol=tol),
            "status": int(st), "lambda2": lam, "residual": info["residual"],
            "cycles": info["cycles"], "matvecs": info["matvecs"], "seconds": round(dt, 1)}


def partition_entry(mesh_name, mesh, nparts, tol):
    t0 = time.perf_counter()
    st, part, info = oracle.partition(mesh.ids, nparts, tol=tol, **SOLVER)
    dt = time.perf_counter() - t0
    m = oracle.metrics(mesh.ids, part, nparts)
    return {"mesh": mesh_name, "elements": int(mesh.nelem), "nparts": nparts,
            "solver": dict(SOLVER, tol=tol), "status": int(st),
            "edge_cut": m["weighted_cut"], "cut_pairs": int(m["cut_pairs"]),
            "max_neighbors": int(m["max_neighbors"]), "avg_neighbors": m["avg_neighbors"],
            "part_sizes": [int(m["min_size"]), int(m["max_size"])],
            "cycles": info["cycles"], "matvecs": info["matvecs"], "seconds": round(dt, 1)}


def c5b_entry():
    meshes, picks = _c5b_sample()
    out = {"mesh": "batch64 (64 boxes, log-uniform 1e4..5e5 elements, 3% holes)", "nparts": 16,
           "meshes": {}}
    for b in picks:
        e = partition_entry(f"batch64[{b}]", meshes[b], 16, 1e-6)
        out["meshes"][str(b)] = e
        print(f"  c5b mesh {b}: {e['elements']} elements, cut {e['edge_cut']:.0f}, "
              f"{e['seconds']} s", flush=True)
    return out


ENTRIES = {
    "c2": lambda: fiedler_entry("box128x128x64 holes5", mg.box128_holes5(), 1e-10),
    "c5b_rsb16": c5b_entry,
    "c3_level0": lambda: fiedler_entry("box256x256x64 holes3", mg.box256_holes3(), 1e-8),
    "c3_rsb1024": lambda: partition_entry("box256x256x64 holes3", mg.box256_holes3(), 1024, 1e-6),
    "c5a_level0": lambda: fiedler_entry("box256x256x128 clustered10 renumbered",
                                        mg.box256x128_clustered10(), 1e-8),
    "c5a_rsb4096": lambda: partition_entry("box256x256x128 clustered10 renumbered",
                                           mg.box256x128_clustered10(), 4096, 1e-6),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("names", nargs="*")
    a = ap.parse_args()
    names = a.names or list(ENTRIES)
    oracle.build(force=True)
    nthr = oracle.set_threads(a.threads)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_about"] = ("Oracle results (FP64, plain CPU implementation) on the full-size "
                      "benchmark meshes; written by tests/golden/make_config_goldens.py, which "
                      "calls only oracle/ and meshgen/.")
    for name in names:
        print(f"[golden] {name} ({nthr} threads)", flush=True)
        entry = ENTRIES[name]()
        data[name] = entry
        print(f"[golden] {name}: {json.dumps(entry)[:400]}", flush=True)
        with open(OUT + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
            fh.write("\n")
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
