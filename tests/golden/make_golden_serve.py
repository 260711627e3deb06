"""Stored expected values of the serving parity tests (calls only the oracle).

Workload "serve512_every16": the 512-request serving stream (seed 3: Kuhn
cubes n ~ U{24..96}, 0..400 penny cracks, kappa = exp(0.5 Z) per edge, T = 1
/ 0 on x = 0 / 1), requests q = 0, 16, 32, ..., 496.  For each: its n and
crack count, the pinned count, the reference solution x* (oracle Jacobi PCG
to 1e-14 relative residual or stagnation) on a seeded sample S of up to 4096
vertices with the norms of x* and x*_S, k_eff / Q_in / Q_out / energy at x*,
and the error on S (||x_S - x*_S||_2 / ||x*_S||_2) and the true relative
residual of the oracle's own solves stopped at 1e-10: Jacobi PCG in FP64, and
FP64 iterative refinement around FP32 Jacobi PCG (inner tolerance 1e-5,
adaptive final inner tolerance), the mixed-precision method.

    python tests/golden/make_golden_serve.py [workers]    (minutes of CPU)
"""
import json
import multiprocessing
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

COUNT, SEED, EVERY, SAMPLE = 512, 3, 16, 4096


def one(spec):
    t0 = time.time()
    n = spec.n
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    kappa = W.lognormal_kappa(len(E), 0.5, spec.kappa_seed)
    cracks = W.penny_cracks(spec.n_cracks, spec.crack_seed) if spec.n_cracks else np.zeros((0, 7))
    cut = O.crack_cut(xyz, E, cracks)
    star = O.hodge1(xyz, tets, E, kappa=kappa, cut=cut)
    L, _ = O.assemble(V, E, star)
    bt, bv, side = W.x_sides(n)
    A, b, pinned = O.apply_bc(L, bt, bv, E, star)
    ref = O.pcg(A, b, precond="jacobi", tol=1e-14, stagnation=50)
    loose = O.pcg(A, b, precond="jacobi", tol=1e-10)
    x_ir, _, _, ir_res = O.iterative_refinement(A, b, tol=1e-10, inner_tol=1e-5, precond="jacobi",
                                                adaptive_final=True)
    f = O.flux_effective_conductivity(ref.x, E, star, side)
    rng = np.random.Generator(np.random.PCG64(5000 + spec.index))
    vs = np.sort(rng.choice(V, size=min(V, SAMPLE), replace=False))
    x_s = ref.x[vs]
    meta = {"index": spec.index, "n": n, "n_cracks": spec.n_cracks, "V": int(V), "n_cut": int(cut.sum()),
            "n_pinned": int(pinned.sum()), "x_norm": float(np.linalg.norm(ref.x)),
            "x_sample_norm": float(np.linalg.norm(x_s)), "ref_iterations": int(ref.iterations),
            "ref_rel_residual": float(ref.rel_residual), "loose_iterations": int(loose.iterations), "loose_rel_residual": float(loose.rel_residual),
            "loose_sample_error_vs_ref": float(np.linalg.norm(loose.x[vs] - x_s) / np.linalg.norm(x_s)),
            "ir_rel_residual": float(ir_res),
            "ir_sample_error_vs_ref": float(np.linalg.norm(x_ir[vs] - x_s) / np.linalg.norm(x_s)),
            "k_eff": f["k_eff"], "q_in": f["q_in"], "q_out": f["q_out"], "energy": f["energy"],
            "seconds": time.time() - t0}
    print(f"request {spec.index}: n={n} cracks={spec.n_cracks} {meta['ref_iterations']} its "
          f"k_eff={meta['k_eff']:.12f} ({meta['seconds']:.0f}s)", flush=True)
    return meta, vs, x_s


def main(workers=4):
    trace = W.serving_trace(COUNT, SEED, 0.0)
    picked = [spec for spec in trace if spec.index % EVERY == 0]
    # largest first, so the pool's last tasks are short
    order = sorted(picked, key=lambda s: -s.n)
    with multiprocessing.Pool(workers) as pool:
        results = pool.map(one, order, chunksize=1)
    results.sort(key=lambda r: r[0]["index"])
    arrays = {}
    for meta, vs, x_s in results:
        arrays[f"vertex_sample_{meta['index']}"] = vs.astype(np.int64)
        arrays[f"x_sample_{meta['index']}"] = x_s
    np.savez_compressed(os.path.join(HERE, "serve512_every16.npz"), **arrays)
    out = {"workload": "serve512_every16", "count": COUNT, "seed": SEED, "every": EVERY,
           "requests": [r[0] for r in results]}
    with open(os.path.join(HERE, "serve512_every16.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 4)
