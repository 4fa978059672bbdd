"""Benchmark of the Phase A reduction hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = one full graph_reduce (gr_reduce) of the workload graph, already
resident in device memory: per level greedy colouring, colour-major relabel,
test-vector init, Gauss-Seidel sweeps, affinity + strongest neighbour,
aggregation and the Galerkin collapse, until the target size.  Prints ONE
JSON line on stdout (progress goes to stderr).

value = smoothing work of the step (sum over levels of nnz * K * sweeps)
        divided by the measured step time.
roofline = the Gauss-Seidel colour-step kernels: compulsory bytes per colour
        step (CSR rows, one read and one write of each updated vector row)
        over their HIP-event durations, against the 8 TB/s HBM peak.
cpu_baseline = the FP64 reference oracle (one host thread) on level-0
        smoothing + affinity of the same graph, in the same unit.
bf16 = the headline workload again with bfloat16 vector storage, with its
        reduced graph's eigenvalues against the float32 run's.
secondary = the same measurement on a second workload (default: the 256^3
        grid with bfloat16 vectors, whose colour steps are large enough to
        be bandwidth-bound); --secondary '' skips it.
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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chunglu434k")
    ap.add_argument("--dtype", default=None, help="f32 or bf16 vector storage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eig", action="store_true")
    ap.add_argument("--eig-original", action="store_true",
                    help="also the original graph's eigenvalues (slow)")
    ap.add_argument("--random-priority", action="store_true",
                    help="greedy colouring with hashed priorities instead of "
                         "largest-degree-first")
    ap.add_argument("--no-bf16-compare", action="store_true",
                    help="skip the bfloat16-storage run of the headline workload")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the timings of the differentiable pieces (GS "
                         "backward, Rayleigh-quotient gradients, Alg. 1)")
    ap.add_argument("--secondary", default="grid256",
                    help="second workload measured the same way ('' for none)")
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
    args.ldf = not args.random_priority
    res, keep = run_workload(G, args.workload, args.dtype, args.steps,
                             args.warmup, args.ldf)
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
    g, wl, r, dg = keep
    if not args.no_eig:
        result.update(eig_report(G, r, args.eig_original, dg))
    if not args.no_extras:
        result["extras"] = extras_report(G, wl, dg, r, args.ldf)
    if (not args.no_bf16_compare and res["storage"] == "f32" and wl.K % 8 == 0):
        # the same workload with bfloat16 vector storage (FP32 arithmetic)
        lam32 = np.array(result["eig_reduced"]) if "eig_reduced" in result else None
        del r
        b16, keep16 = run_workload(G, args.workload, "bf16", args.steps, args.warmup,
                                   args.ldf, g=g)
        entry = {k: b16[k] for k in ("value", "ms_per_step", "levels", "phase_ms_per_step",
                                     "smooth_only_rate", "roofline")}
        if lam32 is not None:
            lam16, _ = G.gr_laplacian_eigs(keep16[2].coarse, 10)
            entry["eig_reduced"] = [float(x) for x in lam16]
            entry["eig_rel_diff_vs_f32"] = float(np.max(np.abs(lam16 - lam32) / lam32))
        result["bf16"] = entry
        del keep16
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(g, wl)
    del keep, g, dg
    if args.secondary and args.secondary != args.workload:
        # the same measurement on a second workload whose colour steps are
        # large enough to be bandwidth-bound (reported next to the headline)
        sec, keep2 = run_workload(G, args.secondary, None, args.steps,
                                  args.warmup, args.ldf)
        result["secondary"] = {k: sec[k] for k in (
            "value", "ms_per_step", "storage", "config", "levels",
            "smooth_only_rate", "affinity_edges_per_s", "phase_ms_per_step",
            "roofline")}
        if not args.no_extras:
            result["secondary"]["extras"] = secondary_extras(G, keep2)
        del keep2
    print(json.dumps(result), flush=True)


def run_workload(G, key, dtype, steps, warmup, ldf, g=None):
    """Times `steps` full reductions of workload `key` (after `warmup`),
    then the same steps with the library's event profiler on."""
    import torch

    from workloads import graphs as W

    wl = W.WORKLOADS[key]
    dtype = dtype or wl.dtype
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


def eig_report(G, r, eig_original, dg):
    """First 10 nontrivial eigenvalues of the reduced Laplacian, in FP64 on
    the GPU (Chebyshev-filtered subspace iteration), with lambda_i / lambda_2
    (the normalised eigenvalues whose preservation the paper plots, Fig. 5);
    optionally the same for the original graph."""
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
    if eig_original:
        t0 = time.perf_counter()
        lo, rep0 = G.gr_laplacian_eigs(dg, 10)
        torch.cuda.synchronize()
        log(f"original-graph eigenvalues in {time.perf_counter() - t0:.1f} s: {rep0}")
        out["eig_original"] = [float(x) for x in lo]
        out["eig_original_normalised"] = [float(x / lo[0]) for x in lo]
        out["eig_normalised_rel_err"] = float(np.max(
            np.abs(lam / lam[0] - lo / lo[0]) / (lo / lo[0])))
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


def extras_report(G, wl, dg, r, ldf):
    """Timings of the differentiable pieces on the headline workload:
    * the Gauss-Seidel backward pass (vector-Jacobian product) on the full
      graph, K and sweeps of the workload, with the sweep states stored and
      with them recomputed from X0;
    * Rayleigh quotients of 10 vectors and their edge gradients on the
      reduced graph (random FP64 vectors and edge weights: timing only);
    * Alg. 1 edge scaling of a spanning sparsifier P of the reduced graph G
      (maximum spanning forest plus the heaviest 10% of the other edges);
    * the data restriction of Alg. 6 through the reduction's final map.
    A failure is reported in place of the figures."""
    import torch

    from workloads import graphs as W

    out = {"restrict_mean": restrict_report(G, r.agg, r.coarse.n)}
    try:
        K, S = wl.K, wl.sweeps
        el = G.gr_edge_list(dg)
        colours, nc = G.gr_colour_greedy(dg, 1, ldf)
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
        keep = W.spanning_sparsifier(cg.n, eu, ev, we, 0.1)
        pg = W.csr_from_edges(cg.n, eu[keep], ev[keep], we[keep])
        dP = G.DeviceGraph.from_numpy(pg.row_ptr, pg.col, pg.w, dev)
        pel = G.gr_edge_list(dP)
        wP = torch.from_numpy(we[keep].copy()).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = G.gr_sgd_scale(cg, dP, pel, wP, k_max=20)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out["sgd_scale"] = {"ms": ms, "n": cg.n, "edges_G": elr.E, "edges_P": int(keep.size),
                            "iterations": rep["iterations"],
                            "lambda_n_first_last": [rep["lambda_n"][0], rep["lambda_n"][-1]],
                            "cg_iterations_max": rep["cg_iterations_max"]}
        log(f"Alg. 1: {ms:.1f} ms, {rep['iterations']} iterations")
    except Exception as e:
        out.setdefault("rq_forward_backward", {"error": repr(e)})
        out["sgd_scale"] = {"error": repr(e)}
    return out


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


def secondary_extras(G, keep):
    """The GS backward on the second workload, in its own configuration
    (vector storage type, K, sweeps; its colouring when it prescribes one)."""
    import torch

    g, wl, r, dg = keep
    try:
        el = G.gr_edge_list(dg)
        if g.colours is not None:
            colours = torch.from_numpy(g.colours).to(dg.row_ptr.device)
            nc = g.n_colours
        else:
            colours, nc = G.gr_colour_greedy(dg, 1, True)
        return {"gs_vjp": vjp_report(G, dg, el, colours, nc, wl.K, wl.sweeps, wl.dtype),
                "restrict_mean": restrict_report(G, r.agg, r.coarse.n)}
    except Exception as e:  # keep the other figures
        return {"gs_vjp": {"error": repr(e)}}


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
    """Oracle (FP64, one host thread) smoothing + affinity on the level-0
    graph with the level-0 colouring of the GPU run."""
    from oracle import oracle as O

    w64 = g.w.astype(np.float64)
    if g.colours is not None:
        c, nc = g.colours, g.n_colours
    else:
        c, nc = O.colour_greedy(g.n, g.row_ptr, g.col,
                                O.level_seed(wl.colour_seed, 0))
    X = O.init_vectors(g.n, wl.K, O.level_seed(wl.vec_seed, 0))
    t0 = time.perf_counter()
    X = O.smooth(g.n, g.row_ptr, g.col, w64, c, nc, X, wl.sweeps)
    O.affinity(g.n, g.row_ptr, g.col, X)
    dt = time.perf_counter() - t0
    log(f"cpu baseline: {dt:.1f}s")
    return {"value": g.nnz * wl.K * wl.sweeps / dt, "unit": "nnz*K*sweeps/s",
            "cores": 1, "kind": "oracle",
            "sample": f"level-0 smoothing ({wl.sweeps} sweeps) + affinity of "
                      f"the full {g.name} graph (n={g.n}, nnz={g.nnz}), FP64, "
                      f"{dt:.1f} s"}


if __name__ == "__main__":
    main()
