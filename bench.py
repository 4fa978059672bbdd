"""Benchmark of the Phase A reduction hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = one full graph_reduce (gr_reduce) of the workload graph, already
resident in device memory: per level greedy colouring, colour-major relabel,
test-vector init, Gauss-Seidel sweeps, affinity + strongest neighbour,
aggregation and the Galerkin collapse, until the target size.  Prints ONE
JSON line on stdout (progress goes to stderr).

headline = the largest single-GPU configuration: the 256^3 grid (16.8M
        nodes, 100M entries, K = 32 bfloat16-stored vectors, FP32 arithmetic,
        parity colouring), reduced 170x.
value = smoothing work of the step (sum over levels of nnz * K * sweeps)
        divided by the measured step time.
roofline = the Gauss-Seidel colour-step kernels: compulsory bytes per colour
        step (CSR rows, one read and one write of each updated vector row)
        over their HIP-event durations, against the 8 TB/s HBM peak.
eig_error_vs_fp64 = the reduced graph's first 10 nontrivial eigenvalues
        (FP64 on the GPU) against those of the FP64 oracle's reduction of
        the same graph with the same seeds, stored in tests/golden/ by a
        script that calls only the oracle; also in units of the gate
        max(1e-4 lambda, half the oracle's range over 5 vector seeds).
cpu_baseline = the FP64 reference oracle on one Gauss-Seidel sweep over the
        full headline graph, on one host thread and on all of them.
secondary = the same measurement on the other configurations: the power-law
        graph (float32 and bfloat16 storage), the 200k-point kNN graph and
        the 70k-point Gaussian-mixture kNN graph.
extras = pieces outside the timed step: the GS backward, Rayleigh-quotient
        gradients, Alg. 1, the multilevel eigensolver (Alg. 5), Phase B and
        the two branches of Alg. 2, the data restriction of Alg. 6.
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
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))

HBM_PEAK_GBS = 8000.0

# The paper's only reduction timing at this scale (Table 2, coPapersCiteseer,
# the scale of the power-law workload): context, not a target.
PAPER_REFERENCE = {
    "table": "Table 2", "graph": "coPapersCiteseer", "nodes": 4.3e5, "edges": 1.6e7,
    "reduced_nodes": 1.3e4, "T_reduction_s": 16.41,
    "scope": "whole reduction: Phase B (sparsification and edge scaling) then Phase A, "
             "the dense flow",
    "hardware": "one core of a 2.67 GHz 12-core CPU, 48 GB DRAM, 64-bit RHEL 6.0",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


SECONDARY = "chunglu434k,chunglu434k:bf16,knn200k,gmm70k"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid256")
    ap.add_argument("--dtype", default=None, help="f32 or bf16 vector storage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eig", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the pieces outside the timed step")
    ap.add_argument("--secondary", default=SECONDARY,
                    help="comma-separated workloads (key or key:dtype) measured the "
                         "same way ('' for none)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (for "
                         "calibrating rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU "
              f"path (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        calibrate_copy()
        return

    from paper_1812_08942_amd import graphreduce as G

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    G.load()
    res, keep = run_workload(G, args.workload, args.dtype, args.steps, args.warmup)
    result = {
        "metric": "smoothing nnz*K*sweeps/s + affinity edges/s; % HBM peak; "
                  "eig error vs FP64",
        "value": res["value"],
        "unit": "nnz*K*sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "storage": res["storage"],
        "data": "synthetic",
    }
    result.update({k: v for k, v in res.items() if k not in result})
    result["paper_reference"] = PAPER_REFERENCE
    result["copy_bandwidth"] = copy_bandwidth()
    result["roofline"]["frac_of_copy"] = (result["roofline"]["achieved"]
                                          / result["copy_bandwidth"]["GB_per_s"])
    g, wl, r, dg = keep
    if not args.no_eig:
        result.update(eig_report(G, r, args.workload, res["storage"]))
    if not args.no_extras:
        result["extras"] = headline_extras(G, keep)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(g, wl)
    del keep, g, dg, r
    result["secondary"] = {}
    for item in [x for x in args.secondary.split(",") if x]:
        key, _, dt = item.partition(":")
        sec, keep2 = run_workload(G, key, dt or None, args.steps, args.warmup)
        entry = {k: sec[k] for k in ("value", "ms_per_step", "storage", "config", "levels",
                                     "smooth_only_rate", "affinity_edges_per_s",
                                     "phase_ms_per_step", "roofline")}
        if not args.no_eig:
            entry.update(eig_report(G, keep2[2], key, sec["storage"]))
        if not args.no_extras and key == "chunglu434k" and sec["storage"] == "f32":
            entry["extras"] = extras_report(G, keep2)
        if not args.no_extras and key == "gmm70k":
            entry["extras"] = {"alg2_sparse_branch": alg2_report(G, keep2, dense=False)}
        result["secondary"][item] = entry
        del keep2
    print(json.dumps(result), flush=True)


def run_workload(G, key, dtype, steps, warmup, g=None):
    """Times `steps` full reductions of workload `key` (after `warmup`),
    then the same steps with the library's event profiler on."""
    import torch

    from workloads import graphs as W

    wl = W.WORKLOADS[key]
    dtype = dtype or wl.dtype
    ldf = wl.ldf
    if g is None:
        t0 = time.time()
        g = W.build_graph(key)
        log(f"graph {g.name}: n={g.n} nnz={g.nnz} built in {time.time() - t0:.1f}s")
    dev = "cuda:0"
    dg = G.DeviceGraph.from_numpy(g.row_ptr, g.col, g.w, dev)
    colours = torch.from_numpy(g.colours).to(dev) if g.colours is not None else None
    code = G.vec_dtype_code(dtype)
    ws = G.workspace(g.n, g.nnz, wl.K, code, dev)
    G.gr_validate(dg, ws)
    out = (torch.empty(g.n, dtype=torch.int32, device=dev),
           torch.empty(g.n + 1, dtype=torch.int32, device=dev),
           torch.empty(g.nnz, dtype=torch.int32, device=dev),
           torch.empty(g.nnz, dtype=torch.float32, device=dev))

    def step():
        return G.gr_reduce(dg, wl.K, wl.sweeps, wl.ratio, wl.vec_seed,
                           wl.colour_seed, dtype=code, colours=colours,
                           n_colours=g.n_colours,
                           largest_degree_first=ldf, ws=ws, out=out)

    for i in range(warmup):
        r = step()
        torch.cuda.synchronize()
        log(f"{key} warmup {i + 1}/{warmup}: levels={r.levels} "
            f"n_coarse={r.coarse.n}")
    # headline: K steps with nothing but the steps on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    log(f"{key} timed {steps} steps: {ms:.3f} ms/step, levels {r.levels}, "
        f"colours {r.level_colours}")
    # breakdown: the same K steps again with the library's HIP-event
    # profiler on (events on the library stream around every phase and
    # every colour step); it adds a little time, so it is reported apart
    G.gr_profile_start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms_prof = (time.perf_counter() - t0) * 1e3 / steps
    prof = G.gr_profile_stop()
    log(f"{key} profiled {steps} steps: {ms_prof:.3f} ms/step")

    work = sum(nz * wl.K * wl.sweeps for nz in r.level_nnz)
    sm = prof["smooth"]
    achieved = sm["bytes"] / (sm["ms"] * 1e-3) / 1e9 if sm["ms"] > 0 else 0.0
    avg_us = sm["ms"] * 1e3 / max(1, sm["launches"])
    aff = prof["affinity"]
    edges = sum(nz // 2 for nz in r.level_nnz) * steps
    res = {
        "value": work / (ms / 1e3),
        "ms_per_step": ms,
        "storage": dtype,
        "config": {"workload": key, "description": wl.description,
                   "n": g.n, "nnz": g.nnz, "K": wl.K, "sweeps": wl.sweeps,
                   "ratio": wl.ratio, "vec_storage": dtype,
                   "colouring": "prescribed" if colours is not None else
                   ("greedy-ldf" if ldf else "greedy"),
                   "parallelism": "single GPU"},
        "levels": {"n": r.level_n, "nnz": r.level_nnz,
                   "colours": r.level_colours, "n_coarse": r.coarse.n,
                   "nnz_coarse": r.coarse.nnz},
        "smooth_only_rate": work * steps / (sm["ms"] * 1e-3) if sm["ms"] else 0.0,
        "affinity_edges_per_s": edges / (aff["ms"] * 1e-3) if aff["ms"] else 0.0,
        "phase_ms_per_step": {k: round(v["ms"] / steps, 4) for k, v in prof.items()},
        "profiled_ms_per_step": ms_prof,
        "roofline": {
            "bound": "hbm",
            "kernel": "Gauss-Seidel colour step (k_gs_step)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(key, dtype),
            "avg_launch_us": avg_us,
            "bytes_per_launch": sm["bytes"] / max(1, sm["launches"]),
            "launches_per_step": sm["launches"] / steps,
        },
    }
    return res, (g, wl, r, dg)


def eig_report(G, r, key, storage):
    """First 10 nontrivial eigenvalues of the reduced Laplacian, in FP64 on
    the GPU, with lambda_i / lambda_2 (the normalised eigenvalues whose
    preservation the paper plots, Fig. 5), and their error against the FP64
    oracle's reduction of the same graph with the same seeds (the stored
    values of tests/golden/reduction_<key>.txt)."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, rep = G.gr_laplacian_eigs(r.coarse, 10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"reduced-graph eigenvalues in {dt * 1e3:.1f} ms: {rep}")
    out = {"eig_reduced": [float(x) for x in lam],
           "eig_reduced_normalised": [float(x / lam[0]) for x in lam],
           "eig_ms": dt * 1e3, "eig_solver": rep}
    try:
        import make_reduction_goldens as GOLD
        from workloads import graphs as W

        (_, _, _), rows = GOLD.load(key)
        seed0 = GOLD.vec_seeds(W.WORKLOADS[key])[0]
        L = np.array([v[3] for (st, _), v in rows.items() if st == storage])
        ref = rows[(storage, seed0)][3]
        gate = np.maximum(1e-4 * ref, 0.5 * (L.max(0) - L.min(0)))
        err = np.abs(lam - ref)
        out["eig_error_vs_fp64"] = {
            "oracle": f"tests/golden/reduction_{key}.txt ({storage}, vector seed {seed0})",
            "eig_oracle": [float(x) for x in ref],
            "max_rel": float(np.max(err / ref)),
            "max_over_gate": float(np.max(err / gate)),
            "seed_range_rel": float(np.max((L.max(0) - L.min(0)) / ref)),
            # against the oracle's spread over its seeds: inside the seeds'
            # envelope widened by one range (the full-size grid's gate), and
            # the largest deviation from the seeds' mean in their standard
            # deviations
            "within_seed_envelope": bool(np.all(
                (lam >= L.min(0) - (L.max(0) - L.min(0))) &
                (lam <= L.max(0) + (L.max(0) - L.min(0))))),
            "max_abs_z": float(np.max(np.abs(lam - L.mean(0)) / L.std(0, ddof=1))),
            "oracle_n_coarse": rows[(storage, seed0)][0]}
        if storage == "bf16" and ("f32", seed0) in rows:
            # the storage format's cost: bfloat16 run against the FP32 oracle
            L32 = np.array([v[3] for (st, _), v in rows.items() if st == "f32"])
            ref32 = rows[("f32", seed0)][3]
            gate32 = np.maximum(1e-4 * ref32, 0.5 * (L32.max(0) - L32.min(0)))
            out["eig_error_vs_fp64"]["vs_f32_oracle_max_rel"] = float(
                np.max(np.abs(lam - ref32) / ref32))
            out["eig_error_vs_fp64"]["vs_f32_oracle_max_over_gate"] = float(
                np.max(np.abs(lam - ref32) / gate32))
    except (OSError, KeyError) as e:
        out["eig_error_vs_fp64"] = {"error": repr(e)}
    return out


def _timed(fn, reps):
    """Mean wall time (ms) of `reps` calls after one warm-up, device idle at
    both ends."""
    import torch

    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3, out


def vjp_report(G, dg, el, colours, nc, K, S, dtype):
    """Wall time of the GS backward (A8) with stored and with recomputed
    sweep states: random X0 of `dtype` and float32 cotangent."""
    import torch

    dev = dg.row_ptr.device
    X0 = G.gr_init_vectors(dg.n, K, 2, dtype, device=dev)
    gen = torch.Generator(device=dev).manual_seed(3)
    cot = torch.randn(dg.n, K, generator=gen, device=dev)
    out = {"n": dg.n, "nnz": dg.nnz, "K": K, "sweeps": S, "colours": int(nc),
           "states": dtype}
    for mode, store in (("stored_states", True), ("recomputed_states", False)):
        ms, _ = _timed(lambda: G.gr_smooth_vjp(dg, el, colours, nc, X0, cot, S, store), 3)
        out[mode] = {"ms": ms, "nnz_K_sweeps_per_s": dg.nnz * K * S / (ms * 1e-3)}
        log(f"GS backward ({mode}, {dtype} states): {ms:.2f} ms")
    return out


def extras_report(G, keep):
    """Pieces outside the timed step on the power-law graph:
    * the Gauss-Seidel backward pass (vector-Jacobian product) on the full
      graph, K and sweeps of the workload, with the sweep states stored and
      with them recomputed from X0;
    * Rayleigh quotients of 10 vectors and their edge gradients on the
      reduced graph (random FP64 vectors and edge weights: timing only);
    * Alg. 1 edge scaling of a spanning sparsifier P of the reduced graph G
      (maximum spanning forest plus the heaviest 10% of the other edges);
    * the multilevel eigensolver (Alg. 5) on the reduction's hierarchy;
    * Phase B on the reduced graph, and Alg. 2 forced into its dense branch
      (Phase B on the full graph first, as the paper ran coPapersCiteseer);
    * the data restriction of Alg. 6 through the reduction's final map.
    A failure is reported in place of the figures."""
    import torch

    from workloads import graphs as W

    g, wl, r, dg = keep
    out = {"restrict_mean": restrict_report(G, r.agg, r.coarse.n)}
    try:
        K, S = wl.K, wl.sweeps
        el = G.gr_edge_list(dg)
        colours, nc = G.gr_colour_greedy(dg, 1, wl.ldf)
        out["gs_vjp"] = vjp_report(G, dg, el, colours, nc, K, S, "f32")
        del el
    except Exception as e:  # keep the headline figures
        out["gs_vjp"] = {"error": repr(e)}
    try:
        cg = r.coarse
        elr = G.gr_edge_list(cg)
        dev = cg.row_ptr.device
        gen = torch.Generator(device=dev).manual_seed(4)
        wE = torch.rand(elr.E, generator=gen, device=dev, dtype=torch.float64) + 0.5
        U = torch.randn(cg.n, 10, generator=gen, device=dev, dtype=torch.float64)
        gR = torch.ones(10, dtype=torch.float64, device=dev)

        def rq():
            R, den = G.gr_rq_forward(elr, wE, U)
            return G.gr_rq_backward(elr, U, R, den, gR)

        ms, _ = _timed(rq, 5)
        out["rq_forward_backward"] = {"ms": ms, "n": cg.n, "edges": elr.E, "vectors": 10}
        log(f"Rayleigh quotients + gradients: {ms:.3f} ms")
        # Alg. 1 on a spanning sparsifier of the reduced graph
        w_entries = cg.w.to(torch.float64)
        w_edge = torch.zeros(elr.E, dtype=torch.float64, device=dev)
        w_edge[elr.edge_of_entry.long()] = w_entries
        eu, ev, we = (elr.eu.cpu().numpy(), elr.ev.cpu().numpy(), w_edge.cpu().numpy())
        keepP = W.spanning_sparsifier(cg.n, eu, ev, we, 0.1)
        pg = W.csr_from_edges(cg.n, eu[keepP], ev[keepP], we[keepP])
        dP = G.DeviceGraph.from_numpy(pg.row_ptr, pg.col, pg.w, dev)
        pel = G.gr_edge_list(dP)
        wP = torch.from_numpy(we[keepP].copy()).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = G.gr_sgd_scale(cg, dP, pel, wP, k_max=20)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out["sgd_scale"] = {"ms": ms, "n": cg.n, "edges_G": elr.E, "edges_P": int(keepP.size),
                            "iterations": rep["iterations"],
                            "lambda_n_first_last": [rep["lambda_n"][0], rep["lambda_n"][-1]],
                            "cg_iterations_max": rep["cg_iterations_max"]}
        log(f"Alg. 1: {ms:.1f} ms, {rep['iterations']} iterations")
    except Exception as e:
        out.setdefault("rq_forward_backward", {"error": repr(e)})
        out["sgd_scale"] = {"error": repr(e)}
    out["multilevel_eigs"] = multilevel_report(G, keep)
    out["phase_b_reduced"] = phase_b_report(G, r.coarse)
    out["alg2_dense_branch"] = alg2_report(G, keep, dense=True)
    return out


def multilevel_report(G, keep, k=10):
    """Alg. 5 on the reduction's hierarchy: wall time, and the Ritz values of
    the refined vectors on the fine graph against the fine eigenvalues (the
    direct FP64 solve), with 0 and 4 Jacobi steps per level."""
    import torch

    g, wl, r, dg = keep
    try:
        red = G.gr_reduce(dg, wl.K, wl.sweeps, wl.ratio, wl.vec_seed, wl.colour_seed,
                          largest_degree_first=wl.ldf, keep_hierarchy=True)
        h = red.hierarchy
        t0 = time.perf_counter()
        lam_f, rep_f = G.gr_laplacian_eigs(dg, k)
        torch.cuda.synchronize()
        direct_ms = (time.perf_counter() - t0) * 1e3
        out = {"levels": h.n, "k": k, "direct_eigs_ms": direct_ms,
               "eig_fine": [float(x) for x in lam_f]}
        for iters in (0, 4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam_c, U, rep = G.gr_multilevel_eigs(dg, h, k, iters=iters)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            # Ritz values of span(U) on the fine Laplacian (FP64 on the GPU)
            LU = laplacian_apply_gpu(dg, U)
            H = (U.T @ LU).cpu().numpy()
            ritz = np.linalg.eigvalsh((H + H.T) / 2)
            out[f"jacobi_{iters}"] = {"ms": ms, "ritz_over_lambda_minus_1": [
                float(x) for x in ritz / lam_f - 1], "coarsest_lambda": [float(x) for x in lam_c]}
            log(f"multilevel eigensolver ({iters} Jacobi steps): {ms:.1f} ms, Ritz/lambda-1 max "
                f"{np.max(ritz / lam_f - 1):.3f}")
        return out
    except Exception as e:
        return {"error": repr(e)}


def laplacian_apply_gpu(dg, U):
    """L U for the graph's Laplacian, float64 on the device (torch sparse;
    measurement only)."""
    import torch

    n = dg.n
    rows = torch.repeat_interleave(torch.arange(n, device=U.device),
                                   (dg.row_ptr[1:] - dg.row_ptr[:-1]).long())
    A = torch.sparse_coo_tensor(torch.stack([rows, dg.col.long()]), dg.w.double(), (n, n))
    d = torch.zeros(n, dtype=torch.float64, device=U.device).index_add_(0, rows, dg.w.double())
    return d[:, None] * U - torch.sparse.mm(A, U)


def phase_b_report(G, cg):
    """Phase B (tree + 5 rounds of 2% of n) on the reduced graph."""
    import torch

    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flags, _, rep = G.gr_sparsify(cg, rounds=5, add_frac=0.02)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        log(f"Phase B on the reduced graph: {ms:.1f} ms, {rep}")
        return {"ms": ms, "n": cg.n, "edges_G": cg.nnz // 2, **rep}
    except Exception as e:
        return {"error": repr(e)}


def alg2_report(G, keep, dense):
    """Alg. 2 on the workload graph.  dense=True forces the dense branch
    (gamma_max below the graph's density): Phase B and Alg. 1 on the full
    graph, then Phase A on the scaled sparsifier; dense=False keeps the
    sparse branch (Phase A, then Phase B and Alg. 1 on R).  Reports the wall
    time and the first 10 nontrivial eigenvalues of S against those of the
    plain Phase A reduction R (relative), and, in the sparse branch, of the
    unscaled sparsifier P too: the accuracy the edge scaling buys."""
    import torch

    g, wl, r, dg = keep
    try:
        gamma = (g.nnz // 2) / g.n
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = G.gr_spectral_reduce(dg, wl.K, wl.sweeps, wl.ratio, wl.vec_seed, wl.colour_seed,
                                   largest_degree_first=wl.ldf,
                                   gamma_max=(0.5 * gamma if dense else 40.0),
                                   sparsify=dict(rounds=5, add_frac=0.02, cg_max_iter=1000,
                                                 cg_tol=1e-10),
                                   scaling=dict(k_max=20, cg_max_iter=1000, cg_tol=1e-10))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        lam_S, _ = G.gr_laplacian_eigs(out.S, 10)
        lam_R, _ = G.gr_laplacian_eigs(r.coarse, 10)
        rep = {"ms": ms, "dense_branch": out.dense, "gamma": out.gamma, "n_S": out.S.n,
               "edges_S": out.S.nnz // 2, "edges_R": r.coarse.nnz // 2,
               "sparsify": out.sparsify,
               "scaling": {"iterations": out.scaling["iterations"],
                           "lambda_n_first_last": out.scaling["lambda_n"][:1]
                           + out.scaling["lambda_n"][-1:]},
               "eig_S": [float(x) for x in lam_S], "eig_R": [float(x) for x in lam_R],
               "eig_S_vs_R_max_rel": float(np.max(np.abs(lam_S - lam_R) / lam_R)),
               # the normalised eigenvalues lambda_i / lambda_2 of Fig. 5
               "eig_S_vs_R_normalised_max_rel": float(np.max(np.abs(
                   lam_S / lam_S[0] - lam_R / lam_R[0]) / (lam_R / lam_R[0])))}
        if not dense:
            # the same sparsifier of R without the edge scaling
            flags, _, _ = G.gr_sparsify(r.coarse, rounds=5, add_frac=0.02, cg_max_iter=1000,
                                        cg_tol=1e-10)
            P, _ = G.gr_subgraph(r.coarse, flags)
            lam_P, _ = G.gr_laplacian_eigs(P, 10)
            rep["eig_P_unscaled"] = [float(x) for x in lam_P]
            rep["eig_P_vs_R_max_rel"] = float(np.max(np.abs(lam_P - lam_R) / lam_R))
            rep["eig_P_vs_R_normalised_max_rel"] = float(np.max(np.abs(
                lam_P / lam_P[0] - lam_R / lam_R[0]) / (lam_R / lam_R[0])))
        log(f"Alg. 2 ({'dense' if dense else 'sparse'} branch): {ms:.1f} ms, S {out.S.n} nodes "
            f"{out.S.nnz // 2} edges, eig S vs R {rep['eig_S_vs_R_max_rel']:.3f}")
        return rep
    except Exception as e:
        return {"error": repr(e)}


def restrict_report(G, agg, n_coarse, d=64):
    """Wall time of the data restriction of Alg. 6 (F_R = H_G^R F, the mean
    of F over each aggregate) through the reduction's final map, for random
    float32 data of d columns; bytes = one read of F and one write of F_R."""
    import torch

    try:
        n = agg.numel()
        gen = torch.Generator(device=agg.device).manual_seed(5)
        F = torch.randn(n, d, generator=gen, device=agg.device)
        ms, _ = _timed(lambda: G.gr_restrict_mean(agg, n_coarse, F), 5)
        gbs = (n * d * 4 + n_coarse * d * 4 + n * 4) / (ms * 1e-3) / 1e9
        log(f"data restriction ({n} x {d} -> {n_coarse}): {ms:.3f} ms")
        return {"ms": ms, "n": n, "n_coarse": int(n_coarse), "d": d,
                "compulsory_GB_per_s": gbs}
    except Exception as e:  # keep the other figures
        return {"error": repr(e)}


def headline_extras(G, keep):
    """The GS backward on the headline workload, in its own configuration
    (vector storage type, K, sweeps; its colouring when it prescribes one),
    and the data restriction through its final map."""
    import torch

    g, wl, r, dg = keep
    out = {"restrict_mean": restrict_report(G, r.agg, r.coarse.n)}
    try:
        el = G.gr_edge_list(dg)
        if g.colours is not None:
            colours = torch.from_numpy(g.colours).to(dg.row_ptr.device)
            nc = g.n_colours
        else:
            colours, nc = G.gr_colour_greedy(dg, 1, wl.ldf)
        out["gs_vjp"] = vjp_report(G, dg, el, colours, nc, wl.K, wl.sweeps, wl.dtype)
    except Exception as e:  # keep the other figures
        out["gs_vjp"] = {"error": repr(e)}
    return out


COPY_BYTES = 1 << 30


def calibrate_copy():
    """Three device-to-device copies of exactly 1 GiB: rocprofv3 counters
    read on these give the scale from counter units to bytes."""
    import torch

    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 3}), flush=True)


def copy_bandwidth(copies=5):
    """What a plain device-to-device copy of 1 GiB reaches (bytes read plus
    bytes written over its event-measured time): the memory system's
    practical rate, as context for the roofline fraction.  Outside the timed
    steps; the copies run on torch's current stream, where the events are."""
    import torch

    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(2):
        dst.copy_(src)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(copies):
        dst.copy_(src)
    t1.record()
    t1.synchronize()
    ms = t0.elapsed_time(t1) / copies
    del src, dst
    return {"GB_per_s": 2 * COPY_BYTES / (ms * 1e-3) / 1e9, "ms_per_copy": ms,
            "bytes_per_copy": COPY_BYTES, "copies": copies,
            "kind": "device-to-device copy, read + write bytes"}


GS_SECTION = "// ----------------------------------------------------------- GS colour step"


def kernel_source_digest():
    """Digest of the GS kernel's source: its section of gr_phase_a.hip (to
    the end of the file) and the shared device helpers.  A traffic figure
    taken for another version of the kernel is not reported."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_1812_08942_amd", "csrc")
    with open(os.path.join(csrc, "gr_phase_a.hip"), "rb") as f:
        text = f.read()
    at = text.find(GS_SECTION.encode())
    if at < 0:
        raise RuntimeError("GS section marker not found in gr_phase_a.hip")
    with open(os.path.join(csrc, "gr_device.hpp"), "rb") as f:
        helpers = f.read()
    return hashlib.sha256(text[at:] + helpers).hexdigest()


def measured_traffic(workload, dtype):
    """HBM bytes per GS colour-step launch from the committed rocprofv3
    counter summary of this workload, or None when there is none for the
    current kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_gs_step_{workload}_{dtype}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(g, wl):
    """The FP64 oracle on a bounded sample of the headline workload: one
    Gauss-Seidel sweep (of the step's five) over the full graph, with the
    level-0 colouring and the storage rounding of the GPU run, on one host
    thread and on every thread the host offers this process."""
    from oracle import oracle as O

    w64 = g.w.astype(np.float64)
    if g.colours is not None:
        c, nc = g.colours, g.n_colours
    else:
        c, nc = O.colour_greedy(g.n, g.row_ptr, g.col, O.level_seed(wl.colour_seed, 0), wl.ldf)
    X = O.init_vectors(g.n, wl.K, O.level_seed(wl.vec_seed, 0))
    nthr = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    runs = {}
    for t in (1, nthr):
        with O.threads(t):
            t0 = time.perf_counter()
            O.smooth(g.n, g.row_ptr, g.col, w64, c, nc, X, 1, bf16=(wl.dtype == "bf16"))
            runs[t] = time.perf_counter() - t0
        log(f"cpu baseline, {t} thread(s): {runs[t]:.1f} s")
    work = g.nnz * wl.K
    return {"value": work / runs[1], "unit": "nnz*K*sweeps/s", "cores": 1, "kind": "oracle",
            "sample": f"one Gauss-Seidel sweep (of {wl.sweeps}) over the full {g.name} graph "
                      f"(n={g.n}, nnz={g.nnz}, K={wl.K}, {wl.dtype} rounding), FP64: "
                      f"{runs[1]:.1f} s on 1 thread, {runs[nthr]:.1f} s on {nthr}",
            "threads": {"cores": nthr, "value": work / runs[nthr]},
            "host_cpu": host_cpu()}


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
