"""Writes tests/golden/mol10_q4_24.json: the oracle's forward solve, loss, adjoint and
gradient on the full 857,375-node mesh of the 10-electron model molecule (Q4, 24^3 cells,
[-12, 12]^3), with the oracle's own timings on this host.

Calls only oracle/ and the seeded input generators of synth/ (no library code).

Inputs: u = v*/2 (half of the known XC potential, so that v = v_fixed + u is not the
fixed potential alone); target density rho_data = the closed-form model density of the
molecule (each site's charge as a normalised Gaussian of 1 bohr), evaluated at the nodes.

Oracle steps (the forward problem of Eq. 19, the density and loss of Eqs. 1 and 4, the
adjoint of Eqs. 7, 10 and 20, the gradient of Eq. 22):
  eigsh on the Kronecker operator (7 lowest pairs, tol 1e-13), the density of the 5
  occupied orbitals, the loss, the projected right-hand sides, projected CG to a
  relative residual of 1e-12 per column, and g_b = sum_i psi_bi q_bi.

What is stored (the full fields are 857,375 numbers each, too large for a text fixture):
  - eigenvalues, loss, electron count, ||g||_2;
  - 16 sketches d_k . g with seeded standard-normal d_k (synth.random_block(N_f, 16, 7702)):
    for any error e, E[(d_k . e)^2] = ||e||^2, so they estimate ||g_test - g||_2;
  - rho and g at 1,200 nodes: 1,000 drawn with probability proportional to W_a rho_a
    (seeded, with replacement; their probabilities stored for an importance-sampled
    estimate of the density L1 error sum_a W_a |rho_test,a - rho_a|), and 200 uniform.

Run: python tests/golden/make_mol10_q4_24.py   (about 5 minutes on 8 cores)
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fe, ks  # noqa: E402
from synth import random_block, workload  # noqa: E402

OUT = os.path.join(HERE, "mol10_q4_24.json")
SKETCH_SEED = 7702
SAMPLE_SEED = 7703


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def blas_threads() -> int | None:
    try:
        from threadpoolctl import threadpool_info
        return max((i.get("num_threads") or 0) for i in threadpool_info()) or None
    except Exception:
        return None


def main():
    wl = workload(2)
    om = fe.mesh3d(wl.p, wl.n, wl.half_width)
    X = om.coords()
    W = om.weights()
    v = wl.v_fixed(X) + 0.5 * wl.v_xc_target(X)
    rho_d = wl.model_density(X)
    occ = ks.occupations(wl.n_elec)
    k = occ.size

    t0 = time.perf_counter()
    fw = ks.forward(om, v, k + 2, tol=1e-13)
    t1 = time.perf_counter()
    psi = fw.psi[:, :k]
    rho = ks.density(psi, occ, W)
    loss = ks.loss(rho, rho_d, W)
    B = ks.adjoint_rhs(psi, occ, rho, rho_d)
    t2 = time.perf_counter()
    Q = ks.adjoint_cg(om, v, psi, fw.eps[:k], B, rtol=1e-12)
    t3 = time.perf_counter()
    g = ks.gradient(psi, Q)
    t4 = time.perf_counter()
    print(f"forward {t1 - t0:.1f} s, density/loss/rhs {t2 - t1:.1f} s, adjoint {t3 - t2:.1f} s, "
          f"gradient {t4 - t3:.2f} s; eps {fw.eps}", flush=True)

    D = random_block(om.n_free, 16, SKETCH_SEED)
    sketches = (D.T @ g).tolist()
    rng = np.random.default_rng(SAMPLE_SEED)
    p = W * rho / np.sum(W * rho)
    imp = rng.choice(om.n_free, size=1000, replace=True, p=p)
    uni = rng.choice(om.n_free, size=200, replace=False)
    out = {
        "what": "oracle forward/adjoint/gradient on the mol10-q4-24 mesh; see make_mol10_q4_24.py",
        "workload": wl.name, "p": wl.p, "n": wl.n, "half_width": wl.half_width, "n_free": int(om.n_free),
        "n_elec": wl.n_elec, "u": "0.5 * v_xc_target", "rho_data": "model_density(width=1.0)",
        "eig": fw.eps.tolist(), "loss": loss, "electrons": float(np.sum(W * rho)),
        "grad_norm2": float(np.linalg.norm(g)), "grad_sum": float(np.sum(g)),
        "sketch_seed": SKETCH_SEED, "grad_sketches": sketches,
        "importance_nodes": imp.tolist(), "importance_prob": p[imp].tolist(),
        "importance_rho": rho[imp].tolist(), "importance_grad": g[imp].tolist(),
        "uniform_nodes": uni.tolist(), "uniform_rho": rho[uni].tolist(), "uniform_grad": g[uni].tolist(),
        "oracle_seconds": {"forward_eigsh": t1 - t0, "density_loss_rhs": t2 - t1, "adjoint_cg": t3 - t2,
                           "gradient": t4 - t3, "gradient_iteration": t4 - t0},
        "host": {"cpu_model": cpu_model(), "logical_cpus": os.cpu_count(), "blas_threads": blas_threads()},
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
