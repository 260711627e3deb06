"""Stored expected values of the crack-growth parity tests (calls only the oracle).

Workload "growth64": the 256^3 crack-growth recipe's 1000 penny discs (seed 4,
radius U[0.02, 0.08]) on a 64^3 Kuhn replica, radii multiplied by 1.02 per
step, kappa = exp(Z) (sigma 1, seed 1), T = 1 / 0 on x = 0 / 1.  For steps
s in STEPS: cut and pinned counts, the reference solution x* (oracle PCG to
1e-14 or stagnation) on a seeded sample S of 65,536 vertices with its norms,
k_eff, Q_in, Q_out, and the error on S (||x_S - x*_S||_2 / ||x*_S||_2) of
the oracle's own solve stopped at 1e-10; the full cut-edge sets of the first
and last step.  The reference
solve stops at 1e-14 relative residual or when 3000 iterations bring no new
best residual (conjugate gradients plateau for long stretches on the
near-percolating late steps).

    python tests/golden/make_golden_growth.py      (minutes of CPU)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

N = 64
STEPS = (0, 10, 20, 30, 40, 50)


def main():
    t0 = time.time()
    xyz, tets = W.kuhn_cube(N)
    V = len(xyz)
    E = O.edges_of(tets, V)
    kappa = W.lognormal_kappa(len(E), 1.0, 1)
    discs = W.penny_cracks(1000, 4)
    bt, bv, side = W.x_sides(N)
    rng = np.random.Generator(np.random.PCG64(777))
    v_sample = np.sort(rng.choice(V, size=65536, replace=False))
    meta = {"workload": "growth64", "n": N, "V": int(V), "E": int(len(E)), "steps": {}}
    arrays = {"vertex_sample": v_sample}
    for s in STEPS:
        cut = O.crack_cut(xyz, E, W.grown_radii(discs, s))
        star = O.hodge1(xyz, tets, E, kappa=kappa, cut=cut)
        A, b, pinned = O.apply_bc(O.assemble(V, E, star)[0], bt, bv, E, star)
        # CG plateaus for long stretches near percolation: a wide stagnation window
        ref = O.pcg(A, b, precond="jacobi", tol=1e-14, stagnation=3000, max_iters=200000)
        loose = O.pcg(A, b, precond="jacobi", tol=1e-10, max_iters=200000)
        f = O.flux_effective_conductivity(ref.x, E, star, side)
        x_s = ref.x[v_sample]
        meta["steps"][str(s)] = {"n_cut": int(cut.sum()), "n_pinned": int(pinned.sum()),
                                 "x_norm": float(np.linalg.norm(ref.x)), "x_sample_norm": float(np.linalg.norm(x_s)),
                                 "loose_sample_error_vs_ref": float(np.linalg.norm(loose.x[v_sample] - x_s)
                                                                    / np.linalg.norm(x_s)),
                                 "loose_iterations": int(loose.iterations), "ref_iterations": int(ref.iterations),
                                 "ref_rel_residual": float(ref.rel_residual), "k_eff": f["k_eff"],
                                 "q_in": f["q_in"], "q_out": f["q_out"], "energy": f["energy"]}
        arrays[f"x_sample_{s}"] = x_s
        if s in (STEPS[0], STEPS[-1]):
            arrays[f"cut_edges_{s}"] = np.nonzero(cut)[0].astype(np.int32)
        print(f"[{time.time()-t0:.0f}s] step {s}: {meta['steps'][str(s)]}", flush=True)
    meta["seconds"] = time.time() - t0
    np.savez_compressed(os.path.join(HERE, "growth64.npz"), **arrays)
    with open(os.path.join(HERE, "growth64.json"), "w") as fh:
        json.dump(meta, fh, indent=1)


if __name__ == "__main__":
    main()
