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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--precond", choices=["jacobi", "fsai"], default="jacobi")
    ap.add_argument("--no-profile", action="store_true", help="time without per-SpMV events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--copy-probe-mib", type=int, default=0, help="also run a plain device copy of this size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2104_05999_amd as dec

    dev = torch.device("cuda:0")
    ctx = dec.Context(dev)
    inp = make_inputs(args.n, dev)
    precond = dec.DEC_PRECOND_FSAI if args.precond == "fsai" else dec.DEC_PRECOND_JACOBI
    profile = 0 if args.no_profile else 1
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
        achieved = per * launches / (spmv_ms / 1e3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                           "kernel": "k_sell<double, MODE_DOT> (sliced-ELL SpMV + p.Ap partials)",
                           "bytes_per_launch": per, "mean_launch_us": round(1e3 * spmv_ms / launches, 3),
                           "launches": launches}
    if not args.no_extras:
        # mixed precision on the same input (FP32 PCG inside FP64 refinement), outside the timed steps
        stm, fm, _, rcm = run_step(ctx, inp, precision=dec.DEC_PREC_MIXED, precond=precond, profile=0)
        st6, f6, _, rc6 = run_step(ctx, inp, precision=dec.DEC_PREC_FP64, precond=precond, profile=0)
        out["mixed_vs_fp64"] = {
            "fp64_solve_ms": round(st6["solve_ms"], 3), "fp64_iterations": st6["iterations"],
            "mixed_solve_ms": round(stm["solve_ms"], 3), "mixed_inner_iterations": stm["iterations"],
            "mixed_outer": stm["outer_iterations"], "mixed_rel_residual": stm["rel_residual"],
            "mixed_fp64_fallback": stm["fp64_fallback"],
            "speedup": round(st6["solve_ms"] / stm["solve_ms"], 3) if stm["solve_ms"] else None,
            "k_eff_mixed": fm["k_eff"], "k_eff_fp64": f6["k_eff"],
        }
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
