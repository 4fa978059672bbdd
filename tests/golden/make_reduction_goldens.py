"""Writes the oracle's end-to-end reduction results for the benchmark
workloads at their full sizes: for each workload and vector storage, the
oracle's multilevel reduction (FP64, bfloat16 rounding emulated where the
storage is bfloat16) for 5 vector seeds, and the first 10 nontrivial
eigenvalues of each reduced Laplacian (Sec. 5, Fig. 5: the reduced graph
should keep the first eigenvalues).  The GPU tests gate the library's own
reduction of the same graph against these values.

Calls only the oracle and the seeded input generators.  Usage (from the
repository root):  python tests/golden/make_reduction_goldens.py [key ...]
Output: tests/golden/reduction_<key>.txt
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from workloads import graphs as W  # noqa: E402

# vector seeds: the workload's own seed first, then four more
SEED_STEP = 1000
N_SEEDS = 5
CASES = {
    # key: vector storages (the colouring order is the workload's own)
    "chunglu434k": ("f32", "bf16"),
    "knn200k": ("f32",),
    "gmm70k": ("f32",),
    "grid256": ("bf16",),
}


def graph_digest(g) -> str:
    h = hashlib.sha256()
    for a in (g.row_ptr.astype(np.int32), g.col.astype(np.int32), g.w.astype(np.float32)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def vec_seeds(wl):
    return [wl.vec_seed + SEED_STEP * s for s in range(N_SEEDS)]


def run(key, threads):
    storages = CASES[key]
    wl = W.WORKLOADS[key]
    ldf = wl.ldf
    t0 = time.time()
    g = W.build_graph(key)
    print(f"{key}: graph n={g.n} nnz={g.nnz} in {time.time() - t0:.0f} s", flush=True)
    given = getattr(g, "colours", None) if key == "grid256" else None
    lines = [
        f"# Oracle reduction of the {key} workload ({wl.description}),",
        f"# K={wl.K}, {wl.sweeps} Gauss-Seidel sweeps, ratio {wl.ratio!r},",
        f"# colour seed {wl.colour_seed}, "
        + ("largest-degree-first greedy colouring" if ldf else
           ("the prescribed parity colouring on level 0, greedy below" if given is not None
            else "greedy colouring")) + ";",
        "# first 10 nontrivial Laplacian eigenvalues of each reduced graph (Sec. 5, Fig. 5).",
        "# Written by tests/golden/make_reduction_goldens.py (oracle only).",
        f"graph {g.n} {g.nnz} {graph_digest(g)}",
    ]
    w64 = g.w.astype(np.float64)
    for st in storages:
        for vs in vec_seeds(wl):
            t = time.time()
            with O.threads(threads):
                r = O.reduce(g.n, g.row_ptr, g.col, w64, wl.K, wl.sweeps, wl.ratio, vs,
                             wl.colour_seed, colours=given,
                             n_colours=(g.n_colours if given is not None else 0),
                             bf16=(st == "bf16"), fp32_coarse=True, largest_degree_first=ldf)
            lam = O.laplacian_eigs(r.n_coarse, r.row_ptr, r.col, r.w, 10)
            lv = ",".join(str(l.n) for l in r.levels)
            lines.append(f"{st} {vs} {r.n_coarse} {len(r.col)} {lv} "
                         + " ".join(repr(float(x)) for x in lam))
            print(f"  {st} seed {vs}: {r.n_coarse} nodes, levels {lv}, "
                  f"{time.time() - t:.0f} s", flush=True)
    path = os.path.join(ROOT, "tests", "golden", f"reduction_{key}.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {path}", flush=True)


def load(key):
    """Parsed golden file: (n, nnz, digest), {(storage, seed): (n_c, nnz_c,
    levels, eigenvalues)}."""
    path = os.path.join(ROOT, "tests", "golden", f"reduction_{key}.txt")
    graph, rows = None, {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            if p[0] == "graph":
                graph = (int(p[1]), int(p[2]), p[3])
            else:
                rows[(p[0], int(p[1]))] = (int(p[2]), int(p[3]),
                                           [int(x) for x in p[4].split(",")],
                                           np.array([float(x) for x in p[5:]]))
    return graph, rows


if __name__ == "__main__":
    keys = sys.argv[1:] or list(CASES)
    thr = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    for k in keys:
        run(k, thr)
