"""Benchmark of the DEC steady-diffusion hot path on one MI355X.

One step = the whole path over one synthetic input already resident in
HBM: topology from the tets, *1 with per-edge conductivity and crack cuts,
assembly of L = d0^T *1 d0, boundary data, PCG solve to 1e-10 relative
residual, flux and effective conductivity.

Default workload: unit cube, 128^3 Kuhn cells (2,146,689 vertices,
12,582,912 tets, 14,827,904 edges), lognormal kappa (sigma 1, seed 1), 200
penny cracks (seed 2), T = 1 / 0 on the faces x = 0 / 1, FP64 Jacobi PCG.

value: algorithmic bytes of the operator product L p, CSR definition over
L's static pattern (nnz (8+4) + 4 (V+1) + 2 V 8 with nnz = V + 2E), for every
PCG iteration in the timed steps, divided by the timed wall time (so the
whole step -- setup, vector updates, reductions -- is in the denominator).
roofline.achieved: the bytes the SpMV kernel actually streams per launch
(the same CSR definition over the entries it stores: the static pattern
without the edges of exactly zero dual area, whose products are -0 and
leave every sum unchanged) over its mean launch duration, timed with HIP
events on the solver's stream during the timed steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 128] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBPS = 8000.0
METRIC = "PCG SpMV GB/s (% of HBM peak); solves/sec + p99 latency, mixed vs FP64"


def spmv_bytes(V, nnz, s_v):
    return nnz * (s_v + 4) + 4 * (V + 1) + 2 * V * s_v


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sell_fp64_kuhn{n}_traffic.txt")
DUAL_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sell_diff_fp64_kuhn{n}_tets_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2104_05999_amd", "csrc", f) for f in ("sell.h", "common.h")]


def _variant(st):
    """The product variant the autotuner chose for a solve (from its stats)."""
    return {"unroll": st["spmv_unroll"], "nontemporal": st["spmv_nontemporal"], "col_bytes": st["spmv_col_bytes"],
            "band": st["spmv_band"], "columns_first": st["spmv_order"]}


def measured_traffic(n, path=TRAFFIC_FILE):
    """HBM bytes per SpMV launch from the committed counter summary of this mesh size, or None when
    there is none or the kernel sources changed since the counters were taken."""
    import hashlib

    path = path.format(n=n)
    if not os.path.exists(path):
        return None
    kv = dict(ln.strip().split("=", 1) for ln in open(path) if "=" in ln and not ln.startswith("#"))
    h = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()
    if kv.get("source_sha256") != h:
        return None
    return int(kv["traffic_bytes_per_launch"])


def make_inputs(n, dev, sigma=1.0, kseed=1, n_cracks=200, cseed=2):
    import torch

    c = W.kuhn_counts(n)
    xyz, tets = W.kuhn_cube(n, device=dev)
    kappa = torch.as_tensor(W.lognormal_kappa(c["E"], sigma, kseed), device=dev)
    cracks = torch.as_tensor(W.penny_cracks(n_cracks, cseed), device=dev)
    bt, bv, side = W.x_sides(n)
    return dict(n=n, xyz=xyz, tets=tets, kappa=kappa, cracks=cracks, bt=torch.as_tensor(bt, device=dev),
                bv=torch.as_tensor(bv, device=dev), side=torch.as_tensor(side, device=dev))


def run_step(ctx, inp, precision=0, precond=0, profile=1, tol=1e-10):
    """One pass of the hot path; returns (stats, flux, mesh counts)."""
    mesh = ctx.mesh(inp["xyz"], inp["tets"])
    mesh.hodge1(inp["kappa"], inp["cracks"], want_cut=False, want_star=False)
    mesh.assemble()
    npin, _ = mesh.apply_bc(inp["bt"], inp["bv"], want_rhs=False)
    T, st, rc = mesh.solve(tol=tol, precision=precision, precond=precond, profile=profile)
    f = mesh.flux(T, inp["side"])
    counts = dict(V=mesh.V, T=mesh.T, E=mesh.E, nnz=mesh.nnz, n_pinned=npin)
    mesh.close()
    return st, f, counts, rc


GOLDEN = os.path.join(ROOT, "tests", "golden", "kuhn128_lognormal1_cracks200")


def precision_preconditioner_table(ctx, inp, n):
    """FP64 and mixed precision, Jacobi and FSAI, on the same system (outside the timed steps); with
    the stored reference solution of this workload, the sampled error against it."""
    import torch

    import paper_2104_05999_amd as dec

    ref = None
    if n == 128 and os.path.exists(GOLDEN + ".npz"):
        meta = json.load(open(GOLDEN + ".json"))
        arr = np.load(GOLDEN + ".npz")
        ref = (meta, torch.as_tensor(arr["vertex_sample"], device=inp["xyz"].device), arr["x_sample"])
    mesh = ctx.mesh(inp["xyz"], inp["tets"])
    mesh.hodge1(inp["kappa"], inp["cracks"], want_cut=False, want_star=False)
    mesh.assemble()
    mesh.apply_bc(inp["bt"], inp["bv"], want_rhs=False)
    table = {}
    for pname, prec in (("fp64", dec.DEC_PREC_FP64), ("mixed", dec.DEC_PREC_MIXED)):
        for cname, pc in (("jacobi", dec.DEC_PRECOND_JACOBI), ("fsai", dec.DEC_PRECOND_FSAI)):
            mesh.solve(tol=1e-10, precision=prec, precond=pc)  # factor setup and tuning outside the timing
            T, st, rc = mesh.solve(tol=1e-10, precision=prec, precond=pc)
            f = mesh.flux(T, inp["side"])
            row = {"solve_ms": round(st["solve_ms"], 3), "iterations": st["iterations"],
                   "outer": st["outer_iterations"], "rel_residual": st["rel_residual"], "status": rc,
                   "fp64_fallback": st["fp64_fallback"], "k_eff": f["k_eff"]}
            if ref is not None:
                meta, vs, xs = ref
                # ||x_S - x*_S||_2 / ||x*_S||_2 on the stored 65,536-vertex sample, beside the same
                # measure of the oracle's own solve stopped at the same tolerance
                row["sampled_error_vs_reference"] = float(np.linalg.norm(T[vs].cpu().numpy() - xs) / np.linalg.norm(xs))
                # the oracle's FP64 Jacobi PCG, or its FP64 refinement around FP32 Jacobi PCG, at 1e-10
                key = "ir_sample_error_vs_ref" if pname == "mixed" else "loose_sample_error_vs_ref"
                row["oracle_same_method_sampled_error"] = meta.get(key)
                row["k_eff_rel_error"] = abs(f["k_eff"] - meta["k_eff"]) / meta["k_eff"]
            table[f"{pname}_{cname}"] = row
    mesh.close()
    base = table["fp64_jacobi"]["solve_ms"]
    table["speedup_vs_fp64_jacobi"] = {k: round(base / v["solve_ms"], 3) for k, v in table.items() if k != "fp64_jacobi"}
    return table


def make_serve_inputs(count, dev, seed=3, rate=0.0):
    """The serving stream: n ~ U{24..96}, 0..400 cracks, kappa sigma 0.5; meshes shared per n."""
    import torch

    trace = W.serving_trace(count, seed, rate)
    meshes, reqs = {}, []
    for spec in trace:
        n = spec.n
        if n not in meshes:
            xyz, tets = W.kuhn_cube(n, device=dev)
            bt, bv, side = W.x_sides(n)
            meshes[n] = dict(xyz=xyz, tets=tets, bc_type=torch.as_tensor(bt, device=dev),
                             bc_value=torch.as_tensor(bv, device=dev), side=torch.as_tensor(side, device=dev))
        r = dict(meshes[n])
        E = W.kuhn_counts(n)["E"]
        r["kappa"] = torch.as_tensor(W.lognormal_kappa(E, 0.5, spec.kappa_seed), device=dev)
        if spec.n_cracks:
            r["cracks"] = torch.as_tensor(W.penny_cracks(spec.n_cracks, spec.crack_seed), device=dev)
        r["T_out"] = torch.empty(r["xyz"].shape[0], dtype=torch.float64, device=dev)
        r["n"] = n
        reqs.append(r)
    return trace, reqs


def _percentiles(lat_s):
    a = np.sort(np.asarray(lat_s)) * 1e3
    return {"p50_ms": round(float(np.percentile(a, 50)), 3), "p99_ms": round(float(np.percentile(a, 99)), 3),
            "mean_ms": round(float(a.mean()), 3)}


def serve_fp64_sequential(ctx, reqs, arrivals):
    """Plain FP64 Jacobi PCG, one request at a time in arrival order (the unbatched baseline)."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, keff, iters = [], [], 0
    for q, r in enumerate(reqs):
        wait = arrivals[q] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        mesh = ctx.mesh(r["xyz"], r["tets"])
        mesh.hodge1(r["kappa"], r.get("cracks"), want_cut=False, want_star=False)
        mesh.assemble()
        mesh.apply_bc(r["bc_type"], r["bc_value"], want_rhs=False)
        T, st, rc = mesh.solve(T=r["T_out"], tol=1e-10)
        f = mesh.flux(T, r["side"])
        mesh.close()
        iters += st["iterations"]
        keff.append(f["k_eff"])
        lat.append(time.perf_counter() - t0 - arrivals[q])
    total = time.perf_counter() - t0
    return {"solves_per_sec": round(len(reqs) / (total - arrivals[0]), 3), **_percentiles(lat),
            "seconds": round(total, 3), "iterations": iters}, keff


def serve_batched(ctx, reqs, arrivals, precision, budget=32 << 30, max_slots=96, chunk=24):
    """The server: requests submitted at their arrival time, stepped until all are done."""
    import torch

    import paper_2104_05999_amd as dec

    srv = dec.Server(ctx, budget, precision=precision, max_slots=max_slots, chunk=chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt, done, lat, keff, steps, peak = 0, 0, [0.0] * len(reqs), [0.0] * len(reqs), 0, 0
    inner = outer = 0
    status_bad = 0
    while done < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrivals[nxt] <= now:
            srv.submit(reqs[nxt], user_tag=nxt)
            nxt += 1
        active, pending = srv.step()
        steps += 1
        peak = max(peak, active)
        for res in srv.poll():
            q = res["user_tag"]
            lat[q] = time.perf_counter() - t0 - arrivals[q]
            keff[q] = res["k_eff"]
            inner += res["inner_iterations"]
            outer += res["outer_iterations"]
            status_bad += res["status"] != 0
            done += 1
        if active == 0 and pending == 0 and nxt < len(reqs):
            wait = arrivals[nxt] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
    total = time.perf_counter() - t0
    bs = srv.stats()
    srv.close()
    achieved = bs["batch_bytes"] / (bs["batch_ms"] / 1e3) / 1e9 if bs["batch_ms"] > 0 else 0.0
    # the batched iterations (SpMV + p.q, update, close of every resident system) against HBM peak
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "batch_ms": round(bs["batch_ms"], 3),
            "batch_bytes": bs["batch_bytes"], "system_iterations": bs["batch_iterations"],
            "variant": bs["variant_fp32" if precision == 1 else "variant_fp64"]}
    return {"solves_per_sec": round(len(reqs) / (total - arrivals[0]), 3), **_percentiles(lat),
            "seconds": round(total, 3), "steps": steps, "peak_resident": peak, "inner_iterations": inner,
            "outer_iterations": outer, "failed": status_bad, "batched_iterations_roofline": roof,
            "host_ms": {k: round(v, 1) for k, v in bs["host_ms"].items()}}, keff


SERVE_GOLDEN = os.path.join(ROOT, "tests", "golden", "serve512_every16")


def stream_oracle_errors(reqs, keff, mixed):
    """Errors of the results now in the requests' T_out against the stored oracle values of requests
    0, 16, ..., 496 (||x_S - x*_S||_2 / ||x*_S||_2 on each request's vertex sample), beside the same
    measure of the oracle's own 1e-10 solves (FP64 Jacobi PCG; with `mixed`, the larger of that and
    its FP64 refinement around FP32 Jacobi PCG); None without the stored values or for another stream."""
    import torch

    if not os.path.exists(SERVE_GOLDEN + ".npz") or len(reqs) != 512:
        return None
    meta = json.load(open(SERVE_GOLDEN + ".json"))
    arr = np.load(SERVE_GOLDEN + ".npz")

    def ref_error(r):  # FP64: the oracle's FP64 PCG; mixed: the larger of its two errors at 1e-10
        return max(r["loose_sample_error_vs_ref"], r["ir_sample_error_vs_ref"]) if mixed else r["loose_sample_error_vs_ref"]

    worst, worst_ratio, worst_k, rows = 0.0, 0.0, 0.0, 0
    for r in meta["requests"]:
        q = r["index"]
        worst_k = max(worst_k, abs(keff[q] - r["k_eff"]) / r["k_eff"])
        T = reqs[q]["T_out"]
        vs = torch.as_tensor(arr[f"vertex_sample_{q}"], device=T.device)
        xs = arr[f"x_sample_{q}"]
        e = float(np.linalg.norm(T[vs].cpu().numpy() - xs) / np.linalg.norm(xs))
        worst = max(worst, e)
        worst_ratio = max(worst_ratio, e / ref_error(r))
        rows += 1
    return {"requests_checked": rows, "worst_sampled_error_vs_reference": worst,
            "worst_ratio_to_oracle_tol_solve_error": round(worst_ratio, 3), "worst_k_eff_rel_error": worst_k,
            "oracle_tol_solve_worst_sampled_error": max(ref_error(r) for r in meta["requests"])}


def serving_benchmark(ctx, dev, count):
    """Saturated throughput (all requests queued at t = 0) and latency under Poisson arrivals at
    0.8 x the FP64 baseline's saturated rate, plain FP64 one-at-a-time vs mixed batched (and, saturated,
    the same server in FP64)."""
    import paper_2104_05999_amd as dec

    trace, reqs = make_serve_inputs(count, dev)
    zero = [0.0] * count
    print(f"[bench] serving: {count} requests generated", file=sys.stderr, flush=True)
    f64_sat, k64 = serve_fp64_sequential(ctx, reqs, zero)
    print(f"[bench] serving fp64 saturated: {f64_sat}", file=sys.stderr, flush=True)
    f64_err = stream_oracle_errors(reqs, k64, False)
    mix_sat, kmix = serve_batched(ctx, reqs, zero, dec.DEC_PREC_MIXED)
    mix_err = stream_oracle_errors(reqs, kmix, True)
    print(f"[bench] serving mixed saturated: {mix_sat}", file=sys.stderr, flush=True)
    # the same server in FP64: separates what batching gives from what FP32 inner solves give
    b64_sat, kb64 = serve_batched(ctx, reqs, zero, dec.DEC_PREC_FP64)
    print(f"[bench] serving fp64 batched saturated: {b64_sat}", file=sys.stderr, flush=True)
    rate = 0.8 * f64_sat["solves_per_sec"]
    arrivals = [spec.arrival_s for spec in W.serving_trace(count, 3, rate)]
    f64_poi, _ = serve_fp64_sequential(ctx, reqs, arrivals)
    mix_poi, _ = serve_batched(ctx, reqs, arrivals, dec.DEC_PREC_MIXED)
    print(f"[bench] serving poisson: fp64 {f64_poi} mixed {mix_poi}", file=sys.stderr, flush=True)
    dk = max(abs(a - b) / abs(b) for a, b in zip(kmix, k64))
    ns = [spec.n for spec in trace]
    return {
        "workload": f"{count} requests, Kuhn n ~ U{{24..96}} (mean V {int(np.mean([(n + 1) ** 3 for n in ns]))}), "
                    "0-400 penny cracks, lognormal kappa sigma 0.5, tol 1e-10",
        "fp64_sequential": {"saturated": f64_sat, "poisson": f64_poi},
        "mixed_batched": {"saturated": mix_sat, "poisson": mix_poi},
        "fp64_batched": {"saturated": b64_sat},
        "poisson_rate_per_s": round(rate, 3),
        "speedup_saturated_solves_per_sec": round(mix_sat["solves_per_sec"] / f64_sat["solves_per_sec"], 3),
        "speedup_mixed_vs_fp64_batched": round(mix_sat["solves_per_sec"] / b64_sat["solves_per_sec"], 3),
        "max_rel_keff_diff_fp64_batched_vs_sequential": max(abs(a - b) / abs(b) for a, b in zip(kb64, k64)),
        "max_rel_keff_diff_mixed_vs_fp64": dk,
        "oracle_errors": {"fp64_sequential": f64_err, "mixed_batched": mix_err},
    }


def crack_growth(ctx, dev, n=256, steps=51, n_discs=1000, seed=4):
    """Crack growth: discs grown by 2% per step, each solve warm-started from the previous step;
    FP64 and mixed-precision chains on the same mesh.  Returns the k_eff curves and wall times."""
    import torch

    xyz, tets = W.kuhn_cube(n, device=dev)
    c = W.kuhn_counts(n)
    kappa = torch.as_tensor(W.lognormal_kappa(c["E"], 1.0, 1), device=dev)
    bt, bv, side = (torch.as_tensor(a, device=dev) for a in W.x_sides(n))
    discs = W.penny_cracks(n_discs, seed)
    grown = [torch.as_tensor(W.grown_radii(discs, s), device=dev) for s in range(steps)]
    t0 = time.perf_counter()
    mesh = ctx.mesh(xyz, tets)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    out = {"workload": f"kuhn{n}_growth_{n_discs}discs_{steps}steps", "V": mesh.V, "E": mesh.E,
           "topology_s": round(setup_s, 3)}
    for name, prec in (("fp64", 0), ("mixed", 1)):
        T = torch.zeros(mesh.V, dtype=torch.float64, device=dev)
        curve, iters, cuts, status, step_ms = [], [], [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            ts = time.perf_counter()
            cut, _ = mesh.hodge1(kappa, grown[s], want_star=False)
            mesh.assemble()
            mesh.apply_bc(bt, bv, want_rhs=False)
            T, st, rc = mesh.solve(T=T, tol=1e-10, precision=prec, warm_start=1, check=False)
            f = mesh.flux(T, side)
            curve.append(f["k_eff"])
            iters.append(st["iterations"])
            cuts.append(int(cut.sum()))
            status.append(rc)
            step_ms.append(round(1e3 * (time.perf_counter() - ts), 2))
            print(f"[bench] growth {name} step {s}: k_eff {f['k_eff']:.9f} its {st['iterations']} "
                  f"rc {rc} {step_ms[-1]} ms", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        out[name] = {"seconds": round(time.perf_counter() - t0, 3), "k_eff": curve, "iterations": iters,
                     "status": status, "step_ms": step_ms}
        out["n_cut"] = cuts
    out["mixed_vs_fp64_speedup"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 3)
    out["max_abs_keff_diff"] = max(abs(a - b) for a, b in zip(out["fp64"]["k_eff"], out["mixed"]["k_eff"]))
    mesh.close()
    return out


def _cracking_path(ctx, dev, n, order=None, max_steps=100000):
    """One cracking process on a homogeneous Kuhn n^3 cube, on ctx's stream: crack a face per step
    (largest flux density, or the next of `order`), re-solve, until k_eff <= 1e-12 of its start.
    Every step: conductivity with the new zero, *1, assembly, boundary data, a warm-started FP64
    solve to 1e-10, flux (and, deterministic, the largest-flux-density face)."""
    import torch

    with torch.cuda.stream(ctx.stream):
        xyz, tets = W.kuhn_cube(n, device=dev)
        bt, bv, side = (torch.as_tensor(a, device=dev) for a in W.x_sides(n))
        mesh = ctx.mesh(xyz, tets)
        kappa = torch.ones(mesh.E, dtype=torch.float64, device=dev)
        _, star = mesh.hodge1(kappa, want_cut=False)
        n_faces = int((star != 0).sum())
        T, ks, steps = None, [], 0
        t0 = time.perf_counter()
        while True:
            mesh.hodge1(kappa, want_cut=False, want_star=False)
            mesh.assemble()
            mesh.apply_bc(bt, bv, want_rhs=False)
            T, st, rc = mesh.solve(T=T, tol=1e-10, warm_start=T is not None, check=False)
            k = mesh.flux(T, side)["k_eff"]
            ks.append(k)
            if rc != 0 or k <= 1e-12 * ks[0] or steps >= max_steps:
                break
            if order is None:
                e, _ = mesh.max_flux_edge(T)
            else:
                e = int(order[steps]) if steps < len(order) else -1
            if e < 0:
                break
            kappa[e] = 0.0
            steps += 1
        torch.cuda.current_stream().synchronize()
        sec = time.perf_counter() - t0
        mesh.close()
    return {"steps": steps, "faces": n_faces, "D_n_at_separation": steps / n_faces, "seconds": round(sec, 3),
            "steps_per_sec": round((steps + 1) / sec, 1), "status": rc,
            "k_eff_curve": [round(ks[i], 6) for i in range(0, len(ks), max(1, len(ks) // 40))]}


def _faces_of(ctx, dev, n):
    import torch

    xyz, tets = W.kuhn_cube(n)
    probe = ctx.mesh(torch.as_tensor(xyz, device=dev), torch.as_tensor(tets, device=dev))
    _, star = probe.hodge1(torch.ones(probe.E, dtype=torch.float64, device=dev), want_cut=False)
    ids = torch.nonzero(star != 0).flatten().cpu().numpy()
    probe.close()
    return ids


def _parallel_paths(dev, n, orders, threads):
    """Monte Carlo paths driven from `threads` host threads, each with its own context on its own
    stream (the library's calls release the interpreter lock), so the paths' small kernels overlap."""
    import threading

    import torch

    import paper_2104_05999_amd as dec

    ctxs = [dec.Context(dev, stream=torch.cuda.Stream(dev)) for _ in range(threads)]
    out = [None] * len(orders)
    errors = []

    def worker(tid):
        try:
            for i in range(tid, len(orders), threads):
                out[i] = _cracking_path(ctxs[tid], dev, n, order=orders[i])
                print(f"[bench] cracking n={n} stochastic path {i}: {out[i]['steps']} cracks, "
                      f"{out[i]['seconds']:.2f} s", file=sys.stderr, flush=True)
        except Exception as exc:  # reported after the join
            errors.append(exc)

    t0 = time.perf_counter()
    th = [threading.Thread(target=worker, args=(t,)) for t in range(threads)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    if errors:
        raise errors[0]
    return out, wall


def served_paths(ctx, dev, n, orders, precision=1, max_slots=128, chunk=8, budget=8 << 30, max_steps=None):
    """Monte Carlo cracking paths as served requests: every step of every path is one request to one
    server (one more face cracked, warm-started from the path's last temperature), all on the topology,
    geometry and pattern of one prepared mesh; a path submits its next step when its result arrives,
    until the domain stops conducting (k_eff <= 1e-12 of its start).  Returns per path the k_eff after
    every step, and the wall time, the steps and the server's batch counters."""
    import torch

    import paper_2104_05999_amd as dec

    xyz, tets = W.kuhn_cube(n, device=dev)
    bt, bv, side = (torch.as_tensor(a, device=dev) for a in W.x_sides(n))
    base = ctx.mesh(xyz, tets)
    base.hodge1(torch.ones(base.E, dtype=torch.float64, device=dev), want_cut=False, want_star=False)
    base.assemble()
    paths = [{"kappa": torch.ones(base.E, dtype=torch.float64, device=dev),
              "T": [torch.zeros(base.V, dtype=torch.float64, device=dev) for _ in range(2)], "step": 0, "ks": [],
              "its": 0} for _ in orders]
    srv = dec.Server(ctx, budget, precision=precision, max_slots=max_slots, chunk=chunk, tol=1e-10)

    def submit(i):
        p, k = paths[i], paths[i]["step"]
        req = {"mesh": base, "kappa": p["kappa"], "bc_type": bt, "bc_value": bv, "side": side, "T_out": p["T"][k % 2]}
        if k > 0:
            req["T0"] = p["T"][(k - 1) % 2]
        srv.submit(req, user_tag=i)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(len(orders)):
        submit(i)
    active, status = len(orders), 0
    while active:
        srv.step()
        for res in srv.poll():
            i = res["user_tag"]
            p = paths[i]
            p["ks"].append(res["k_eff"])
            p["its"] += res["inner_iterations"]
            status = status or res["status"]
            limit = len(orders[i]) if max_steps is None else min(max_steps, len(orders[i]))
            if res["status"] != 0 or res["k_eff"] <= 1e-12 * p["ks"][0] or p["step"] >= limit:
                active -= 1
                continue
            p["kappa"][int(orders[i][p["step"]])] = 0.0
            p["step"] += 1
            submit(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    counters = srv.stats()
    srv.close()
    base.close()
    return {"ks": [p["ks"] for p in paths], "steps": [p["step"] for p in paths],
            "inner_iterations": sum(p["its"] for p in paths), "wall_seconds": wall, "status": status,
            "batch": counters}


def cracking_processes(ctx, dev, n_det=(16, 24), n_mc=(8, 16), paths=8, threads=8, seed=7, served_n=8,
                       served_paths_count=100):
    """Section 3's cracking processes on homogeneous Kuhn cubes: the deterministic one (crack the
    face of largest flux density) on each n_det^3 (24^3 has 45,000 faces, the size of the paper's
    mesh), and `paths` Monte Carlo paths (faces in seeded random orders) on each n_mc^3, run
    concurrently from `threads` host threads, each until the domain stops conducting."""
    out = {"deterministic": [], "stochastic": []}
    for n in n_det:
        r = _cracking_path(ctx, dev, n)
        print(f"[bench] cracking n={n} deterministic: {r['steps']} cracks, D_n {r['D_n_at_separation']:.4f}, "
              f"{r['seconds']:.2f} s", file=sys.stderr, flush=True)
        out["deterministic"].append({"workload": f"kuhn{n}_homogeneous", **r})
    for n in n_mc:
        rng = np.random.Generator(np.random.PCG64(seed))
        faces = _faces_of(ctx, dev, n)
        orders = [rng.permutation(faces) for _ in range(paths)]
        mc, wall = _parallel_paths(dev, n, orders, threads)
        dn = [p["D_n_at_separation"] for p in mc]
        steps = sum(p["steps"] + 1 for p in mc)
        out["stochastic"].append({
            "workload": f"kuhn{n}_homogeneous_{paths}paths_seed{seed}", "paths": paths, "threads": threads,
            "faces": mc[0]["faces"],
            "D_n_at_separation": {"mean": round(float(np.mean(dn)), 4), "min": round(min(dn), 4),
                                  "max": round(max(dn), 4)},
            "steps": steps, "wall_seconds": round(wall, 3), "steps_per_sec": round(steps / wall, 1),
            "k_eff_curve_path0": mc[0]["k_eff_curve"]})
    # the Monte Carlo paths as served requests (one request per step, warm-started, mixed precision)
    n = served_n
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    faces = _faces_of(ctx, dev, n)
    orders = [rng.permutation(faces) for _ in range(served_paths_count)]
    r = served_paths(ctx, dev, n, orders)
    nf = len(faces)
    dn = [st / nf for st in r["steps"]]
    grid = np.linspace(0.0, 0.8, 17)
    curves = np.full((len(orders), len(grid)), np.nan)
    for i, ks in enumerate(r["ks"]):  # k_eff / k_eff(0) at D_n = grid (0 beyond separation)
        d = np.arange(len(ks)) / nf
        rel = np.asarray(ks) / ks[0]
        curves[i] = np.interp(grid, d, rel, right=0.0)
    steps = sum(len(ks) for ks in r["ks"])
    print(f"[bench] cracking n={n}: {len(orders)} served paths, {steps} requests in {r['wall_seconds']:.1f} s",
          file=sys.stderr, flush=True)
    out["stochastic_served"] = {
        "workload": f"kuhn{n}_homogeneous_{len(orders)}paths_seed{seed + 1}", "paths": len(orders), "faces": nf,
        "how": "one request per step to one mixed-precision server, warm-started from the path's last T, "
               "topology copied from one prepared mesh",
        "requests": steps, "wall_seconds": round(r["wall_seconds"], 3),
        "steps_per_sec": round(steps / r["wall_seconds"], 1), "inner_iterations": r["inner_iterations"],
        "status": r["status"],
        "D_n_at_separation": {"mean": round(float(np.mean(dn)), 4), "min": round(min(dn), 4), "max": round(max(dn), 4),
                              "all": [round(x, 4) for x in dn]},
        "k_eff_vs_D_n": {"D_n": [round(float(g), 3) for g in grid],
                         "mean": [round(float(v), 5) for v in curves.mean(axis=0)],
                         "min": [round(float(v), 5) for v in curves.min(axis=0)],
                         "max": [round(float(v), 5) for v in curves.max(axis=0)]}}
    return out


def dual_inputs(n, dev, sigma=1.0, kseed=1, n_cracks=200, cseed=2, order=None, ctx=None):
    """The tet-unknown workload: the default recipe with the conductivity on the faces (per face of
    the lattice numbering; with `order`, the mesh is renumbered first and the faces follow)."""
    import torch

    xyz, tets = W.kuhn_cube(n, device=dev)
    if order:
        xyz, tets, _, _ = ctx.reorder(xyz, tets, order)
    F = W.kuhn_counts(n)["F"]
    bt, bv, side = (torch.as_tensor(a, device=dev) for a in W.x_sides(n))
    return dict(n=n, xyz=xyz, tets=tets, kappa=torch.as_tensor(W.lognormal_kappa(F, sigma, kseed), device=dev),
                cracks=torch.as_tensor(W.penny_cracks(n_cracks, cseed), device=dev), bt=bt, bv=bv, side=side)


def dual_step(ctx, inp, profile=8, tol=1e-10):
    """Topology, tet system (faces, limited Hodge entries, cuts, Dirichlet faces, blocks), block-Jacobi
    PCG to tol in the A-norm, flux; returns (stats, flux, info, build_ms)."""
    import torch

    t0 = time.perf_counter()
    mesh = ctx.mesh(inp["xyz"], inp["tets"])
    d = mesh.dual(inp["bt"], inp["bv"], inp["side"], inp["kappa"], inp["cracks"])
    mesh.close()
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - t0)
    T, st, rc = d.solve(tol=tol, profile=profile, check=False)
    f = d.flux(T)
    info = dict(d.info(), V=d.V, nnz=d.nnz, n_pinned=d.n_pinned, status=rc)
    d.close()
    return st, f, info, build_ms


def dual_cpu_baseline(n=20):
    """The oracle on the tet-unknown path (faces, geometry, cuts, Schur system, direct solve, flux) on an
    n^3 instance of the same recipe, single-threaded: tets per second."""
    from threadpoolctl import threadpool_limits

    from oracle import dual as D

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        xyz, tets = W.kuhn_cube(n)
        F = W.kuhn_counts(n)["F"]
        bt, bv, side = W.x_sides(n)
        s = D.dual_system(xyz, tets, bt, bv, side, kappa=W.lognormal_kappa(F, 1.0, 1), cracks=W.penny_cracks(200, 2))
        D.flux(D.solve(s), s)
        dt = time.perf_counter() - t0
    return {"value": len(tets) / dt, "unit": "tets/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle tet-unknown path on the {n}^3 instance of the same recipe ({len(tets)} tets, "
                      f"sparse LU for the solve) in {dt:.1f} s", "seconds": dt}


def dual_benchmark(ctx, dev, n, steps, warmup, cpu=True, order=None):
    import torch

    inp = dual_inputs(n, dev, order=order, ctx=ctx)
    for _ in range(warmup):
        st, f, info, bms = dual_step(ctx, inp)
        print(f"[bench] dual warmup: build {bms:.1f} ms, {st['iterations']} its, {st['solve_ms']:.1f} ms solve",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [dual_step(ctx, inp) for _ in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st, f, info, bms = runs[-1]
    launches = sum(r[0]["spmv_launches"] for r in runs)
    spmv_ms = sum(r[0]["spmv_ms"] for r in runs)
    per = st["spmv_bytes"]
    out = {"metric": "tet-unknown system (eq. 11-13): tets/s through topology, build, solve, flux",
           "value": round(info["V"] * steps / elapsed, 1), "unit": "tets/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(1e3 * elapsed / steps, 3), "higher_is_better": True,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"kuhn{n}_face_lognormal1_cracks200_fp64_block_energy"
                                  + (f"_{order}_numbering" if order else ""), "n": n, "tets": info["V"],
                      "faces": info["faces"], "limited": info["limited"], "blocks": info["blocks"],
                      "max_block": info["max_block"], "nnz": info["nnz"], "tol": 1e-10,
                      "stopping": "A-norm error estimate (Hestenes-Stiefel, window 16)"},
           "build_ms": round(bms, 3), "solve_ms": round(st["solve_ms"], 3), "pcg_iterations": st["iterations"],
           "error_estimate": st["rel_residual"], "plain_residual": st["plain_residual"], "k_eff": f["k_eff"],
           "q_in": f["q_in"], "q_out": f["q_out"], "n_pinned": info["n_pinned"], "status": info["status"]}
    if launches:
        achieved = per * launches / (spmv_ms / 1e3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBPS, 4),
                           "traffic": measured_traffic(n, DUAL_TRAFFIC_FILE),
                           "kernel": "k_sell<double, MODE_DOT, difference form> (tet system SpMV + p.Ap partials)",
                           "bytes_per_launch": per, "mean_launch_us": round(1e3 * spmv_ms / launches, 3),
                           "launches": launches, "variant": _variant(st)}
    if cpu:
        out["cpu_baseline"] = dual_cpu_baseline()
    return out


def _max_tet_volume(xyz, tets):
    p = xyz[tets.astype(np.int64)]
    return float(np.abs(np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]),
                                  p[:, 3] - p[:, 0])).max() / 6.0)


def _verify_mesh(ctx, dev, xyz, tets, tol=1e-12, dual=True):
    """The pristine cube (Section 3.1): T = 1 / 0 on x = 0 / 1, kappa = 1, both unknown placements;
    eq. 15 RMS errors against 1 - x, k_eff, limited faces."""
    import torch

    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    bt, bv, side = (t(a) for a in W.x_faces(xyz))
    m = ctx.mesh(t(xyz), t(tets))
    _, star = m.hodge1(want_cut=False)
    m.assemble()
    m.apply_bc(bt, bv, want_rhs=False)
    Tv, sv, rcv = m.solve(tol=tol, check=False)
    fv = m.flux(Tv, side)
    # negative circumcentric dual areas (random Delaunay meshes) make the vertex operator indefinite:
    # the solve then breaks down and has no error to report
    vert = {"negative_dual_areas": int((star < 0).sum()), "iterations": sv["iterations"], "status": rcv}
    if rcv == 0:
        vert.update(rms=m.rms_error(Tv), k_eff=fv["k_eff"])
    row = {"V": m.V, "T": m.T, "max_tet_volume": _max_tet_volume(xyz, tets), "vertex": vert}
    if not dual:
        m.close()
        return row
    d = m.dual(bt, bv, side)
    Tt, st, rct = d.solve(tol=tol, check=False)
    ft = d.flux(Tt)
    info = d.info()
    row["tets"] = {"rms": m.rms_error(Tt), "k_eff": ft["k_eff"], "iterations": st["iterations"], "status": rct,
                   "limited_fraction": info["limited"] / info["faces"], "blocks": info["blocks"]}
    d.close()
    m.close()
    return row


def _spmv_rate(ctx, dev, xyz, tets, steps=2):
    """Mean SpMV launch time and rate (profiled solves) of the vertex path on this numbering."""
    import torch

    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    bt, bv, _ = (t(a) for a in W.x_faces(xyz))
    m = ctx.mesh(t(xyz), t(tets))
    m.hodge1(want_cut=False, want_star=False)
    m.assemble()
    m.apply_bc(bt, bv, want_rhs=False)
    m.solve(tol=1e-10, profile=8)  # tuning outside the timing
    ms = launches = 0
    solve = []
    for _ in range(steps):
        _, st, _ = m.solve(tol=1e-10, profile=8)
        ms += st["spmv_ms"]
        launches += st["spmv_launches"]
        solve.append(st["solve_ms"])
    per = st["spmv_bytes"]
    m.close()
    us = 1e3 * ms / launches
    return {"spmv_us": round(us, 3), "GBps": round(per / (us * 1e-6) / 1e9, 1), "solve_ms": round(min(solve), 3),
            "iterations": st["iterations"]}


def meshes_benchmark(ctx, dev, kuhn=(8, 16, 32, 64), lattice=(8, 16, 24, 32, 48), delaunay=(2000, 8000, 32000, 128000),
                     shuffle_n=128):
    """General meshes: the eq. 15 convergence study over Kuhn cubes and Delaunay meshes of random
    points (the TetGen stand-in), and the SpMV on a scrambled numbering before and after the
    spatial numbering of Section 2.2."""
    import torch

    out = {"metric": "eq. 15 RMS error vs max tet volume; SpMV GB/s before / after spatial numbering",
           "n_gpus": 1, "data": "synthetic", "convergence": {"kuhn": [], "kuhn_jittered": [], "delaunay_lattice": [], "delaunay": []}}
    for n in kuhn:
        xyz, tets = W.kuhn_cube(n)
        out["convergence"]["kuhn"].append({"n": n, **_verify_mesh(ctx, dev, xyz, tets)})
        print(f"[bench] kuhn {n}: {out['convergence']['kuhn'][-1]}", file=sys.stderr, flush=True)
        # interior nodes moved by up to 0.15 h: not Delaunay, so only the vertex unknowns apply
        xj = W.jitter_interior(xyz, n, 0.15, n)
        row = _verify_mesh(ctx, dev, xj, tets, dual=False)
        out["convergence"]["kuhn_jittered"].append({"n": n, **row})
        print(f"[bench] kuhn {n} jittered: {row}", file=sys.stderr, flush=True)
    for n in lattice:
        t0 = time.perf_counter()
        xyz, tets = W.delaunay_lattice(n, 0.2, 3)
        gen = time.perf_counter() - t0
        row = {"n": n, "mesh_s": round(gen, 1), **_verify_mesh(ctx, dev, xyz, tets)}
        out["convergence"]["delaunay_lattice"].append(row)
        print(f"[bench] delaunay lattice {n}: {row}", file=sys.stderr, flush=True)
    for npts in delaunay:
        t0 = time.perf_counter()
        xyz, tets = W.delaunay_cube(npts, int(2 * npts ** (2.0 / 3.0)), 1)
        gen = time.perf_counter() - t0
        xr, tr, _, _ = ctx.reorder(torch.as_tensor(xyz, device=dev), torch.as_tensor(tets, device=dev))
        row = {"points": npts, "mesh_s": round(gen, 1),
               **_verify_mesh(ctx, dev, xr.cpu().numpy(), tr.cpu().numpy())}
        out["convergence"]["delaunay"].append(row)
        print(f"[bench] delaunay {npts}: {row}", file=sys.stderr, flush=True)
    # numbering: a Kuhn cube with scrambled vertex and tet numbers (a mesh file in no useful order)
    xyz, tets = W.kuhn_cube(shuffle_n)
    rng = np.random.Generator(np.random.PCG64(5))
    p = rng.permutation(len(xyz))
    xs = np.ascontiguousarray(xyz[np.argsort(p)])
    ts = np.ascontiguousarray(p[tets][rng.permutation(len(tets))].astype(np.int32))
    before = _spmv_rate(ctx, dev, xs, ts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xr, tr, _, _ = ctx.reorder(torch.as_tensor(xs, device=dev), torch.as_tensor(ts, device=dev))
    torch.cuda.synchronize()
    reorder_ms = 1e3 * (time.perf_counter() - t0)
    after = _spmv_rate(ctx, dev, xr.cpu().numpy(), tr.cpu().numpy())
    xm, tm, _, _ = ctx.reorder(torch.as_tensor(xs, device=dev), torch.as_tensor(ts, device=dev), "morton")
    morton = _spmv_rate(ctx, dev, xm.cpu().numpy(), tm.cpu().numpy())
    out["numbering"] = {"workload": f"kuhn{shuffle_n}_homogeneous_scrambled_numbering", "scrambled": before,
                        "spatial": after, "morton": morton, "reorder_ms": round(reorder_ms, 3),
                        "spmv_speedup": round(before["spmv_us"] / after["spmv_us"], 2)}
    print(f"[bench] numbering: {out['numbering']}", file=sys.stderr, flush=True)
    return out


def cpu_baseline(n=80):
    """The oracle, single-threaded, on the full path of a smaller instance of the same recipe."""
    from threadpoolctl import threadpool_limits

    import oracle as O

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        xyz, tets = W.kuhn_cube(n)
        V = len(xyz)
        E = O.edges_of(tets, V)
        kap = W.lognormal_kappa(len(E), 1.0, 1)
        cut = O.crack_cut(xyz, E, W.penny_cracks(200, 2))
        star = O.hodge1(xyz, tets, E, kappa=kap, cut=cut)
        L, _ = O.assemble(V, E, star)
        bt, bv, side = W.x_sides(n)
        A, b, _ = O.apply_bc(L, bt, bv, E, star)
        res = O.pcg(A, b, precond="jacobi", tol=1e-10)
        O.flux_effective_conductivity(res.x, E, star, side)
        dt = time.perf_counter() - t0
    byts = res.iterations * spmv_bytes(V, L.nnz, 8)
    return {
        "value": byts / dt / 1e9,
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle full path (topology..flux, FP64 Jacobi PCG to 1e-10) on the {n}^3 instance of the "
                   f"same recipe: {res.iterations} iterations x {spmv_bytes(V, L.nnz, 8)/1e6:.1f} MB SpMV "
                   f"bytes in {dt:.1f} s"),
        "seconds": dt,
    }


def spmv_roofline(st, n, kernel="k_sell<double, MODE_DOT> (sliced-ELL SpMV + p.Ap partials)"):
    """The roofline object of a profiled solve's SpMV launches (HIP events on the solve stream)."""
    per, launches, ms = st["spmv_bytes"], st["spmv_launches"], st["spmv_ms"]
    achieved = per * launches / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(n), "kernel": kernel,
            "bytes_per_launch": per, "mean_launch_us": round(1e3 * ms / launches, 3), "launches": launches}


def roofline_256(ctx, dev, profile=8):
    """The dominant kernel where its working set cannot stay in the 256 MB Infinity Cache: the same
    recipe (lognormal kappa sigma 1 seed 1, 200 penny cracks seed 2, T = 1 / 0 on x = 0 / 1) on the
    256^3 Kuhn cube (16,974,593 vertices), one warm-up solve (tuning) and one profiled FP64 Jacobi
    solve to 1e-10; measured outside the timed steps."""
    inp = make_inputs(256, dev)
    mesh = ctx.mesh(inp["xyz"], inp["tets"])
    mesh.hodge1(inp["kappa"], inp["cracks"], want_cut=False, want_star=False)
    mesh.assemble()
    mesh.apply_bc(inp["bt"], inp["bv"], want_rhs=False)
    mesh.solve(tol=1e-10)
    T, st, rc = mesh.solve(tol=1e-10, profile=profile)
    out = spmv_roofline(st, 256)
    out.update({"workload": "kuhn256_lognormal1_cracks200_fp64_jacobi", "V": mesh.V, "spmv_nnz": st["spmv_nnz"],
                "pcg_iterations": st["iterations"], "solve_ms": round(st["solve_ms"], 3), "status": rc,
                "column_bytes": st["spmv_col_bytes"], "variant": _variant(st)})
    mesh.close()
    del inp
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--precond", choices=["jacobi", "fsai"], default="jacobi")
    ap.add_argument("--no-profile", action="store_true", help="time without per-SpMV events")
    ap.add_argument("--profile-every", type=int, default=8,
                    help="carry HIP events on every k-th SpMV launch of the timed solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--copy-probe-mib", type=int, default=0, help="also run a plain device copy of this size")
    ap.add_argument("--serve-requests", type=int, default=512, help="serving stream length (0: skip)")
    ap.add_argument("--no-roofline-256", dest="roofline_256", action="store_false",
                    help="skip the SpMV roofline on the 256^3 mesh (outside the timed steps)")
    ap.add_argument("--cracking", action="store_true",
                    help="instead of the default line: the deterministic and Monte Carlo cracking processes")
    ap.add_argument("--growth-n", type=int, default=256)
    ap.add_argument("--growth-steps", type=int, default=51)
    ap.add_argument("--dual", action="store_true",
                    help="instead of the default line: the tet-unknown system (temperature per tet, flux per face)")
    ap.add_argument("--dual-n", type=int, default=128)
    ap.add_argument("--dual-order", choices=["lexicographic", "morton"], default=None,
                    help="renumber the tet workload first (dec_reorder)")
    ap.add_argument("--meshes", action="store_true",
                    help="instead of the default line: eq. 15 convergence study and the spatial numbering")
    ap.add_argument("--crack-growth", action="store_true",
                    help="instead of the default line: the 256^3 crack-growth chains (FP64 and mixed)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2104_05999_amd as dec

    dev = torch.device("cuda:0")
    ctx = dec.Context(dev)
    if args.cracking:
        print(json.dumps({"metric": "cracking processes: k_eff vs damage D_n, steps/s", "n_gpus": 1,
                          "data": "synthetic", **cracking_processes(ctx, dev)}))
        return
    if args.meshes:
        print(json.dumps(meshes_benchmark(ctx, dev)))
        return
    if args.dual:
        print(json.dumps(dual_benchmark(ctx, dev, args.dual_n, args.steps, args.warmup, not args.no_cpu_baseline,
                                        args.dual_order)))
        return
    if args.crack_growth:
        print(json.dumps({"metric": "crack growth k_eff(step), mixed vs FP64 wall time", "n_gpus": 1,
                          "data": "synthetic", **crack_growth(ctx, dev, n=args.growth_n, steps=args.growth_steps)}))
        return
    inp = make_inputs(args.n, dev)
    precond = dec.DEC_PRECOND_FSAI if args.precond == "fsai" else dec.DEC_PRECOND_JACOBI
    profile = 0 if args.no_profile else args.profile_every
    print(f"[bench] n={args.n} warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        st, f, counts, rc = run_step(ctx, inp, precond=precond, profile=profile)
        print(f"[bench] warmup: {st['iterations']} its, {st['solve_ms']:.1f} ms solve", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for _ in range(args.steps):
        steps.append(run_step(ctx, inp, precond=precond, profile=profile))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    iters = sum(s[0]["iterations"] for s in steps)
    per = steps[0][0]["spmv_bytes"]
    spmv_ms = sum(s[0]["spmv_ms"] for s in steps)
    launches = sum(s[0]["spmv_launches"] for s in steps)
    st, f, counts, rc = steps[-1]
    per_static = spmv_bytes(counts["V"], counts["nnz"], 8)
    value = iters * per_static / elapsed / 1e9
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"kuhn{args.n}_lognormal1_cracks200_fp64_{args.precond}",
                   "n": args.n, "V": counts["V"], "T": counts["T"], "E": counts["E"], "nnz": counts["nnz"],
                   "spmv_nnz": st["spmv_nnz"],
                   "spmv_pattern": ("full static pattern" if st["spmv_nnz"] == counts["nnz"] else
                                    "static pattern without the edges of zero dual area (bit-identical products)"),
                   "tol": 1e-10, "parallelism": "single GPU"},
        "value_bytes_per_iteration": per_static,
        "solves_per_sec": round(args.steps / elapsed, 4),
        "pcg_iterations": st["iterations"],
        "rel_residual": st["rel_residual"],
        "k_eff": f["k_eff"],
        "q_in": f["q_in"],
        "q_out": f["q_out"],
        "n_pinned": counts["n_pinned"],
        "solve_ms": round(st["solve_ms"], 3),
        "status": rc,
    }
    if launches:
        agg = {"spmv_bytes": per, "spmv_launches": launches, "spmv_ms": spmv_ms}
        out["roofline"] = spmv_roofline(agg, args.n)
        out["roofline"]["column_bytes"] = st["spmv_col_bytes"]
        out["roofline"]["variant"] = _variant(st)
    if args.roofline_256 and profile:
        out["roofline_256"] = roofline_256(ctx, dev, profile)
        print(f"[bench] roofline_256: {out['roofline_256']}", file=sys.stderr, flush=True)
    if not args.no_extras:
        out["mixed_vs_fp64"] = precision_preconditioner_table(ctx, inp, args.n)
    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        a = torch.empty(nb // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        out["copy_probe"] = {"bytes": 2 * nb, "GBps": round(10 * 2 * nb / (e0.elapsed_time(e1) / 1e3) / 1e9, 1)}
    if args.serve_requests > 0:
        out["serving"] = serving_benchmark(ctx, dev, args.serve_requests)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
