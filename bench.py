"""Benchmark of the inverse-DFT hot path on one MI355X.

A step is one gradient iteration of the inverse loop: the forward Chebyshev-
filtered eigensolve (warm-started from the previous iterate's orbitals), the
density/loss/adjoint right-hand side, the batched MINRES adjoint solve, the
gradient (all behind the autograd Function), and the potential update. Three
paths run the same steps to the same tolerances (every adjoint column held to
the same Euclidean residual bar):
  f64    the plain FP64 GPU path (diagonal MINRES preconditioner);
  f64d   FP64 with the adjoint's preconditioner deflated by the block's buffer
         Ritz vectors (the same algorithm as the mixed path, in FP64 only);
  mixed  the mixed-precision path (FP32 Chebyshev filter with FP64
         Rayleigh-Ritz, reductions and the deflated adjoint; orbitals
         recomputed in backward instead of stored).
`value` is the mixed path's gradient iterations per second, timed over --steps
steps after --warmup; the two comparison paths are timed over
min(--steps, --compare-steps) steps after min(--warmup, 2), which keeps the
run to a few minutes (their per-step cost is flat over the loop: the same
ChFSI pass and MINRES counts step after step).

The roofline object is for the dominant kernel of the timed region, the
operator apply in the precision that takes the most time: every launch is
timed by HIP events on its own stream (fe_apply_timing), and its algorithmic
bytes (X read once, Y written once, v read once) are divided by the summed
duration. Its HBM traffic comes from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of
this same command, scaled by what the counters read for fe_axpby over 2^27
doubles (launched at start-up as the reference), stored under profiles/ with
the hash of the kernel source they were taken on; it is null when the kernel
source has changed since. The same fe_axpby, timed by HIP events, gives the
bandwidth a plain streaming kernel reaches (roofline.measured_copy_GBps),
reported beside the 8 TB/s spec peak.

minres_sweeps reports the adjoint's three fused row sweeps (passes A, B, C of
one MINRES iteration) over the head path's timed steps, each launch timed by
HIP events (fe_sweep_timing_read) against its algorithmic bytes; one iteration
streams N s (3 k0 + 16 k) + 8 N bytes (k0 orbitals, k active columns).

With --kT T (Ha) the same loop runs at finite temperature: Fermi-Dirac
occupations with mu from the electron count, every orbital above the occupation
cut in the density and the adjoint, and the in-span part of the adjoint functions
(Eqs. 4, 5, 8, 9). The block is widened by 4 columns and the eigensolver converges
all but the last 4 Ritz pairs; the included count is reported in `config`.

With --vxc-h H the XC potential lives on its own linear mesh (Eq. 14): uniform cells of
H bohr on the inner cube [-L/2, L/2]^3, growing by 1.4 towards the box; the loop
optimises its vertex values (v = v_fixed + P u, gradient P^T g), and the two transfer
kernels are timed on their own as well.

With --graded H the orbitals live on a graded tensor mesh (Fig. 6, Sec. 4): cells of H
bohr on the inner cube [-L/2, L/2]^3, growing by 1.35 towards the box (for workload 5
and H = 0.6: 36 cells per axis, 5.7 M free nodes, against 40 cells of 0.8 bohr and
7.9 M nodes for the uniform mesh).

With --mapped A the orbitals live on the mapped mesh of amplitude A (the workload's uniform
mesh with its nodes moved by a smooth map of the box: curved cells, every cell its own dense
element matrix, applied as batched MFMA cell products with gather and scatter, Sec. 3.2.3).
The roofline then covers that apply, whose algorithmic bytes include the per-cell matrices;
it is bound by HBM while its arithmetic intensity is below the FP64 ridge and by the FP64
matrix cores above it.

With --coldstart the script measures the forward eigensolve alone from a random block instead of
the inverse loop: FP64 throughout, FP32 -> FP64 and bf16 -> FP32 -> FP64 (FE_BF16), each to the
same tolerance, with every stage's passes, time and error against the FP64 solve (eigenvalues,
density L1, residual) after it; it prints one JSON object.

With --frontend the set-up also times the physics front end on the target density: the
Hartree potential by the finite-element Poisson solve and the initial guess of Eq. 25
(LB94 exchange + PW92 correlation, Fermi-Amaldi tail).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 5] [--kT 0] [--vxc-h 0] [--graded 0]
                       [--frontend]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def apply_timing(api, mesh, v, nv, prec, reps=20):
    """Average ks_apply duration (ms) from HIP events on the launch stream."""
    import torch
    dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[prec]
    X = torch.randn(mesh.n_free, nv, device=v.device, dtype=torch.float32).to(dt)
    Y = torch.empty_like(X)
    for _ in range(3):
        api.ks_apply(mesh, v, X, Y, prec=prec)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        api.ks_apply(mesh, v, X, Y, prec=prec)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    s = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    algo_bytes = 2 * mesh.n_free * nv * s + mesh.n_free * 8
    if getattr(mesh, "mapped_amp", None) is not None:   # the per-cell matrices stream once per apply
        npc = mesh.nodes_per_cell
        algo_bytes += mesh.n_cells * ((npc + 15) // 16) * ((npc + 3) // 4) * 64 * s
    del X, Y
    return ms, algo_bytes


def host_cpu():
    """(CPU model, BLAS threads the oracle's dense products use) of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads") or 0) for i in threadpool_info()) or threads
    except Exception:
        pass
    return model, threads


def kernel_source_hash():
    """Hash of the operator kernels' sources (the sum-factorised apply and the mapped-mesh cell
    products): the stored counter readings belong to it."""
    import hashlib
    h = hashlib.sha256()
    for name in ("apply.hip", "mapped.hip"):
        path = os.path.join(ROOT, "paper_2510_10529_amd", "csrc", name)
        if os.path.exists(path):
            h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(prec, workload_name, deflate=0):
    """HBM bytes per launch of ks_apply in prec on this workload, from the rocprofv3 counter
    summary under profiles/ (FETCH_SIZE x fetch scale + WRITE_SIZE x write scale, KiB per
    dispatch), or None when there is none for the current kernel source. The launch mix (and so
    the average) depends on the adjoint's deflation, which is part of the key."""
    path = os.path.join(ROOT, "profiles", "ks_apply_traffic.txt")
    if not os.path.exists(path):
        return None
    want = kernel_source_hash()
    for line in open(path):
        f = dict(kv.split("=", 1) for kv in line.split() if "=" in kv)
        if (f.get("workload") == workload_name and f.get("prec") == prec and f.get("src") == want
                and int(f.get("deflate", "0")) == deflate):
            return 1024.0 * (float(f["fetch_kib"]) * float(f["fetch_scale"]) +
                             float(f["write_kib"]) * float(f["write_scale"]))
    return None


def coldstart(api, mesh, W, v, X0, nocc, wl, args):
    """Forward eigensolve from a random block: FP64, FP32 -> FP64 and bf16 -> FP32 -> FP64, with each
    stage's passes, seconds and errors against the FP64 solve."""
    import torch
    tol, deg = 1e-10, wl.cheb_degree
    zeros = torch.zeros(mesh.n_free, dtype=torch.float64, device=v.device)

    def solve(prec, maxpass=400):
        X = X0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = api.ks_eigensolve(mesh, v, X, nocc, deg, tol, maxpass, prec=prec, switch_tol=1e-4)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rho, _, _ = api.loss_grad(mesh, X[:, :nocc].contiguous(), [2.0] * nocc, zeros, want_B=False)
        return r, el, rho

    ref, t_ref, rho_ref = solve("f64")
    out = {"workload": wl.name, "n_free": mesh.n_free, "nocc": nocc, "block": X0.shape[1], "cheb_degree": deg,
           "tol": tol, "fp64": {"passes": ref.passes, "seconds": t_ref}}
    log(f"coldstart FP64: {ref.passes} passes, {t_ref:.2f} s")
    for prec in ("f32", "bf16"):
        full, t_full, _ = solve(prec)
        stages = []
        done = 0
        names = ("bf16", "f32", "f64")
        for k, n in enumerate(full.stage_passes):
            if n == 0:
                continue
            done += n
            r, el, rho = solve(prec, maxpass=done)
            eig_err = max(abs(a - b) for a, b in zip(r.eig[:nocc], ref.eig[:nocc]))
            l1 = float((W * (rho - rho_ref).abs()).sum())
            stages.append({"stage": names[k], "passes": n, "seconds_cumulative": el, "eig_err_Ha": eig_err,
                           "density_L1": l1, "max_residual": max(r.res[:nocc])})
            log(f"coldstart {prec}: after {names[k]} ({n} passes, {el:.2f} s): eig err {eig_err:.2e} Ha, "
                f"density L1 {l1:.2e}, residual {max(r.res[:nocc]):.2e}")
        out[prec] = {"passes": full.passes, "seconds": t_full, "stage_passes": full.stage_passes,
                     "speedup_vs_fp64": t_ref / t_full, "stages": stages}
    print(json.dumps(out), flush=True)


def run_path(api, inv, mesh, v_fixed, rho_d, n_elec, X0, opts, steps, warmup, step_len, vxc=None):
    import torch
    prob = inv.InverseProblem(mesh, v_fixed, rho_d, n_elec, X0, opts, vxc=vxc)
    u = prob.zeros_u()
    losses = []

    def one_step(u):
        ur = u.detach().clone().requires_grad_(True)
        loss = inv.InvDFTLoss.apply(ur, prob)
        loss.backward()
        g = ur.grad.detach()
        gmax = float(g.abs().max())          # scalar read-back for the step length only
        if gmax > 0:
            api.axpby(-step_len / gmax, g, 1.0, u)
        return float(loss.detach()), g

    g_first = None                      # the gradient at u = 0: the same point on every path
    for w in range(warmup):
        l, g = one_step(u)
        if g_first is None:
            g_first = g.clone()
        log(f"  warmup {w}: loss {l:.6e}  passes {prob.stats.passes[-1]}  minres {prob.stats.adj_iters[-1]}")
    prob.stats = inv.Stats()
    torch.cuda.synchronize()
    api.apply_timing(True)             # HIP events around every operator launch of the timed steps
    t0 = time.perf_counter()
    for k in range(steps):
        l, g = one_step(u)
        losses.append(l)
        if g_first is None:
            g_first = g.clone()
        log(f"  step {k}: loss {l:.6e}  passes {prob.stats.passes[-1]}  minres {prob.stats.adj_iters[-1]}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    api.apply_timing(False)
    timing = {p: api.apply_timing_read(p) for p in ("f64", "f32")}      # (launches, ms, bytes, columns)
    timing.update({f"minres_{q}": api.sweep_timing_read(q) for q in "ABC"})
    return elapsed, losses, g_first, prob, timing


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paths", default="mixed,f64,f64d",
                    help="paths to time; the first is the head path whose rate is `value`")
    ap.add_argument("--compare-steps", type=int, default=6,
                    help="timed steps of every path after the first (at most --steps)")
    ap.add_argument("--apply-only", action="store_true",
                    help="only time ks_apply on the workload mesh (used for kernel profiles)")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--kT", type=float, default=0.0, help="k_B T in Ha (0: zero temperature)")
    ap.add_argument("--switch-tol", type=float, default=3e-4,
                    help="mixed path: FP32 filter passes while the largest occupied residual is above this")
    ap.add_argument("--deflate", type=int, default=-1,
                    help="Ritz vectors above the orbitals that deflate the adjoint's preconditioner on the mixed "
                         "and f64d paths (default: the block's buffer columns; 0: off). The f64 path always keeps "
                         "the diagonal preconditioner.")
    ap.add_argument("--degree", type=int, default=0,
                    help="Chebyshev filter degree (default: the workload's)")
    ap.add_argument("--deflate-split", action="store_true",
                    help="let the deflation go beyond 64 columns of [Psi U] (separate sweeps for the rest); by "
                         "default the driver deflates with at most 64 - (included orbitals) vectors")
    ap.add_argument("--buffer", type=int, default=-1,
                    help="ChFSI buffer columns above the occupied ones (default: the workload's max(4, 0.2 N_occ), "
                         "with the block rounded up to a multiple of 8 columns, at most 64, at zero temperature)")
    ap.add_argument("--coldstart", action="store_true",
                    help="time the eigensolve from a random block in FP64, FP32 and bf16 stages (no inverse loop)")
    ap.add_argument("--frontend", action="store_true",
                    help="time the Hartree solve and the initial guess on the target density")
    ap.add_argument("--graded", type=float, default=0.0,
                    help="inner cell size of a graded orbital mesh (0: the workload's uniform mesh)")
    ap.add_argument("--mapped", type=float, default=None,
                    help="amplitude of the smooth map of a mapped orbital mesh (per-cell dense matrices)")
    ap.add_argument("--vxc-h", type=float, default=0.0,
                    help="cell size of the linear XC mesh on the inner cube (0: nodal XC potential)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_10529_amd import api
    from paper_2510_10529_amd import inverse as inv
    from synth import random_block, vxc_vertices, workload

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    wl = workload(args.config)
    if args.degree > 0:
        wl = dataclasses.replace(wl, cheb_degree=args.degree)
    log(f"workload {wl.name}: p={wl.p} n={wl.n} L={wl.half_width} N_e={wl.n_elec}")
    breaks = vxc_vertices(wl.half_width, args.graded, 0.5 * wl.half_width, 1.35) if args.graded > 0 else None
    if args.mapped is not None and (breaks is not None or args.vxc_h > 0 or args.frontend):
        print("--mapped does not combine with --graded, --vxc-h or --frontend", file=sys.stderr)
        sys.exit(2)
    mesh = api.Mesh(wl.p, wl.n, wl.half_width, breaks=breaks, mapped_amp=args.mapped)
    xyz, W = mesh.nodes()
    xyz_h = xyz.cpu().numpy()
    del xyz
    v_fixed = torch.tensor(wl.v_fixed(xyz_h), device=dev)
    v_star = torch.tensor(wl.v_xc_target(xyz_h), device=dev)
    del xyz_h
    kT = args.kT
    nocc, nv = wl.n_occ, wl.n_occ + (wl.n_buf if args.buffer < 0 else args.buffer)
    if args.buffer < 0 and kT <= 0:
        # whole 8-column chunks of the FP64 apply, and more Ritz vectors to deflate the adjoint
        nv = max(nv, min(64, (nv + 7) // 8 * 8))
    nconv = nocc
    if kT > 0:
        nv += 4
        nconv = nv - 4
    wname = wl.name if kT <= 0 else f"{wl.name}-kT{kT:g}"
    if args.graded > 0:
        wname += f"-graded{args.graded:g}"
    if args.mapped is not None:
        wname += f"-mapped{args.mapped:g}"
    if args.vxc_h > 0:
        wname += f"-vxc{args.vxc_h:g}"
    log(f"N_f={mesh.n_free} nocc={nocc} nv={nv}" + (f" kT={kT} converged={nconv}" if kT > 0 else ""))
    # a plain streaming kernel of known size, the reference for scaling the HBM byte
    # counters of profiled runs: fe_axpby over 2^27 doubles reads 2 GiB and writes 1 GiB
    xa = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    ya = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    for _ in range(2):
        api.axpby(1.0, xa, 1.0, ya)
    # the same kernel timed: the bandwidth a plain streaming kernel reaches, beside the 8 TB/s spec
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        api.axpby(1.0, xa, 1.0, ya)
    ev1.record()
    ev1.synchronize()
    copy_gbs = 10 * 3 * 8 * (1 << 27) / (ev0.elapsed_time(ev1) * 1e6)
    log(f"fe_axpby over 2^27 doubles: {copy_gbs:.0f} GB/s")
    del xa, ya
    if args.apply_only:
        out = {}
        for prec, cols in (("f64", nocc), ("f32", nv), ("bf16", nv)):
            ms, b = apply_timing(api, mesh, v_fixed, cols, prec, reps=args.reps)
            out[f"ks_apply_{prec}"] = {"columns": cols, "ms": ms, "algorithmic_bytes": b,
                                       "GBps": b / ms / 1e6, "hbm_frac": b / ms / 1e6 / HBM_PEAK_GBS}
            log(f"ks_apply {prec} nv={cols}: {ms:.3f} ms, {b / ms / 1e6:.0f} GB/s")
        print(json.dumps({"workload": wl.name, "n_free": mesh.n_free, **out}), flush=True)
        return
    X0 = torch.tensor(random_block(mesh.n_free, nv, 1000 + args.config), device=dev)
    if args.coldstart:
        coldstart(api, mesh, W, v_fixed + v_star, X0, nocc, wl, args)
        return

    # target density rho_data = rho(v_fixed + v*) (untimed set-up)
    t0 = time.perf_counter()
    if kT > 0:
        # at the same temperature, through the driver (occupations from fermi_occupations)
        tp = inv.InverseProblem(mesh, v_fixed, torch.zeros_like(v_fixed), wl.n_elec, X0,
                                inv.SolverOptions(degree=wl.cheb_degree, tol_eig=1e-9, maxpass=400, kT=kT,
                                                  n_states=nconv, filter_prec="f32", switch_tol=1e-4))
        tp.set_potential(v_star)
        tp.eigensolve(1e-9)
        rho_d, _, _ = tp.loss_and_rhs(tp.psi())
        target_passes, target_incl = tp.stats.passes[-1], tp.state.n
        del tp
    else:
        v_t = v_fixed + v_star
        Xt = X0.clone()
        r = api.ks_eigensolve(mesh, v_t, Xt, nocc, wl.cheb_degree, 1e-9, 400, prec="f32", switch_tol=1e-4)
        rho_d, _, _ = api.loss_grad(mesh, Xt[:, :nocc].contiguous(), [2.0] * nocc, torch.zeros_like(v_t),
                                    want_B=False)
        target_passes = r.passes
        del Xt, v_t
    # warm start for the inverse loop: orbitals of v_fixed (u = 0)
    Xw = X0.clone()
    api.ks_eigensolve(mesh, v_fixed, Xw, nconv, wl.cheb_degree, 1e-9, 400, prec="f32", switch_tol=1e-4)
    torch.cuda.synchronize()
    log(f"set-up (target density + initial orbitals) {time.perf_counter() - t0:.1f} s, "
        f"target passes {target_passes}" + (f", {target_incl} orbitals enter" if kT > 0 else ""))
    del X0

    fe_info = {}
    if args.frontend:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v_h, pres = api.poisson_solve(mesh, rho_d, sigma=1.0, tol=1e-10)
        t1 = time.perf_counter()
        v_init = api.xc_initial_guess(mesh, rho_d, v_h, float(wl.n_elec), exchange="lb94")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fe_info = {"hartree_s": t1 - t0, "hartree_cg_iters": pres.iters, "hartree_relres": pres.relres,
                   "hartree_charge": pres.charge, "initial_guess_ms": 1000 * (t2 - t1)}
        log(f"front end: Hartree {t1 - t0:.2f} s ({pres.iters} CG iterations, charge {pres.charge:.10f}), "
            f"initial guess {1000 * (t2 - t1):.2f} ms")
        del v_h, v_init

    vxc = None
    vxc_info = {}
    if args.vxc_h > 0:
        tv = vxc_vertices(wl.half_width, args.vxc_h, 0.5 * wl.half_width, 1.4)
        vxc = api.VxcMesh(mesh, tv, tv, tv)
        log(f"linear XC mesh: {tv.size} vertices per axis, {vxc.n_vertices} unknowns")
        # the two transfer kernels alone (HIP events on the current stream)
        ut = torch.randn(vxc.n_vertices, dtype=torch.float64, device=dev)
        vt_ = torch.empty_like(v_fixed)
        ft = torch.empty_like(ut)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for _ in range(3):
            vxc.prolong(ut, base=v_fixed, out=vt_)
            vxc.restrict(vt_, out=ft)
        reps = 20
        ev[0].record()
        for _ in range(reps):
            vxc.prolong(ut, base=v_fixed, out=vt_)
        ev[1].record()
        for _ in range(reps):
            vxc.restrict(vt_, out=ft)
        ev[2].record()
        ev[2].synchronize()
        ms_p, ms_r = ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps
        nb_p = 16 * mesh.n_free + 8 * vxc.n_vertices      # base read, v written, u read once
        nb_r = 8 * mesh.n_free + 8 * vxc.n_vertices       # g read once, f written
        vxc_info = {"vxc_vertices": vxc.n_vertices, "vxc_prolong_ms": ms_p, "vxc_prolong_GBps": nb_p / ms_p / 1e6,
                    "vxc_restrict_ms": ms_r, "vxc_restrict_GBps": nb_r / ms_r / 1e6}
        log(f"vxc prolong {ms_p:.3f} ms ({nb_p / ms_p / 1e6:.0f} GB/s), restrict {ms_r:.3f} ms "
            f"({nb_r / ms_r / 1e6:.0f} GB/s)")
        del ut, vt_, ft

    step_len = 0.01
    results = {}
    common = dict(degree=wl.cheb_degree, tol_eig=1e-9, tol_adj=1e-10, maxpass=100, maxit_adj=20000)
    deflate = nv - nocc if args.deflate < 0 else args.deflate
    if kT > 0:
        common.update(kT=kT, n_states=nconv)
    paths = {
        "f64": inv.SolverOptions(**common, filter_prec="f64", adjoint_prec="f64", recompute=False),
        "f64d": inv.SolverOptions(**common, filter_prec="f64", adjoint_prec="f64", recompute=False,
                                  deflate=deflate, deflate_split=args.deflate_split),
        "mixed": inv.SolverOptions(**common, filter_prec="f32", adjoint_prec="f64", switch_tol=args.switch_tol,
                                   recompute=True, deflate=deflate, deflate_split=args.deflate_split),
    }
    order = args.paths.split(",")
    for k, name in enumerate(order):
        steps = args.steps if k == 0 else max(1, min(args.steps, args.compare_steps))
        warm = args.warmup if k == 0 else min(args.warmup, 2)
        log(f"path {name}: {warm} warmup + {steps} timed steps")
        el, losses, g0, prob, timing = run_path(api, inv, mesh, v_fixed, rho_d, wl.n_elec, Xw, paths[name],
                                                steps, warm, step_len, vxc)
        results[name] = dict(elapsed=el, steps=steps, losses=losses, g0=g0, stats=prob.stats, timing=timing,
                             n_incl=prob.state.n)
        for p_, (n_, ms_, b_, _c) in timing.items():
            if n_:
                log(f"  {'ks_apply ' if p_ in ('f64', 'f32') else ''}{p_}: {n_} launches, {ms_:.1f} ms, "
                    f"{b_ / ms_ / 1e6:.0f} GB/s")
        log(f"path {name}: {steps / el:.4f} iters/s  forward {prob.stats.t_forward / steps:.2f} s/step  "
            f"adjoint {prob.stats.t_adjoint / steps:.2f} s/step")
        del prob

    head_name = order[0]
    head = results[head_name]
    ips = args.steps / head["elapsed"]
    out_extra = {}
    # every path's first gradient is taken at u = 0 from the same start block: equal accuracy
    # means these agree to the gradient tolerance
    for name in order[1:]:
        r = results[name]
        ipsx = r["steps"] / r["elapsed"]
        key = {"f64": "fp64_path", "f64d": "fp64_deflated_path", "mixed": "mixed_path"}[name]
        out_extra[f"{key}_iters_per_s"] = ipsx
        out_extra[f"speedup_vs_{key}"] = ips / ipsx
        gh, gx = head["g0"], r["g0"]
        out_extra[f"grad_rel_diff_{head_name}_vs_{name}"] = float(
            torch.linalg.vector_norm(gh - gx) / torch.linalg.vector_norm(gx))
    out_extra["seconds_per_step"] = {
        name: {"forward": r["stats"].t_forward / r["steps"], "adjoint": r["stats"].t_adjoint / r["steps"],
               "total": r["elapsed"] / r["steps"],
               "chfsi_passes": sum(r["stats"].passes) / max(1, len(r["stats"].passes)),
               "minres_iters": sum(r["stats"].adj_iters) / max(1, len(r["stats"].adj_iters))}
        for name, r in results.items()}

    # apply alone at the two fixed block widths (context; HIP events on the launch stream)
    ms32, b32 = apply_timing(api, mesh, v_fixed, nv, "f32")
    ms64, b64 = apply_timing(api, mesh, v_fixed, nocc, "f64")
    gbs32 = b32 / ms32 / 1e6
    gbs64 = b64 / ms64 / 1e6
    log(f"ks_apply f32 nv={nv}: {ms32:.3f} ms {gbs32:.0f} GB/s ; f64 nv={nocc}: {ms64:.3f} ms {gbs64:.0f} GB/s")

    # dominant kernel of the head path's timed steps: the apply precision with the most time
    tim = {p: head["timing"][p] for p in ("f64", "f32")}
    dom = max(tim, key=lambda p: tim[p][1])
    n_l, ms_l, b_l, c_l = tim[dom]
    achieved = b_l / ms_l / 1e6                       # GB/s = (bytes per launch) / (ms per launch)
    traffic = read_traffic(dom, wname, deflate if head_name in ("mixed", "f64d") else 0)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": f"ks_apply_{dom}", "launches": n_l, "ms_per_launch": ms_l / n_l,
                "algorithmic_bytes_per_launch": b_l / n_l,
                "measured_copy_GBps": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs}
    # the MINRES row sweeps of the head path's timed steps (HIP events around each pass)
    sweeps = {}
    for q in "ABC":
        n_q, ms_q, b_q, c_q = head["timing"][f"minres_{q}"]
        if n_q:
            sweeps[q] = {"launches": n_q, "ms_per_launch": ms_q / n_q, "GBps": b_q / ms_q / 1e6,
                         "mean_columns": c_q / n_q, "ms_total_per_step": ms_q / head["steps"]}
    if sweeps:
        tot_ms = sum(head["timing"][f"minres_{q}"][1] for q in "ABC")
        tot_b = sum(head["timing"][f"minres_{q}"][2] for q in "ABC")
        sweeps["bytes_per_iteration"] = "N s (3 k0 + 16 k) + 8 N"
        sweeps["GBps_all_passes"] = tot_b / tot_ms / 1e6
    if args.mapped is not None:
        # dense cell products: 2 n_c n_p^2 flops per column of each launch
        s_b = 8 if dom == "f64" else 4
        kb = mesh.n_cells * ((mesh.nodes_per_cell + 15) // 16) * ((mesh.nodes_per_cell + 3) // 4) * 64 * s_b
        nv_mean = c_l / n_l
        flops = 2.0 * mesh.n_cells * mesh.nodes_per_cell ** 2 * nv_mean
        ai = flops / (b_l / n_l)
        roofline.update({"kernel": f"ks_apply_mapped_{dom}", "arithmetic_intensity": ai,
                         "mean_columns": nv_mean, "matrix_bytes_per_launch": kb})
        if ai > FP64_MFMA_TFLOPS * 1e3 / HBM_PEAK_GBS:
            tf = flops / (ms_l / n_l) / 1e9
            roofline.update({"bound": "mfma", "achieved": tf, "peak": FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                             "frac": tf / FP64_MFMA_TFLOPS})
    st = head["stats"]
    applies = None
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import fe as ofe
        rng = np.random.default_rng(5)
        ncol = head["n_incl"]                      # the orbital block the head path carries
        if args.mapped is None:
            log("cpu baseline: one oracle Kronecker apply of the orbital block on the full mesh")
            om = ofe.mesh3d(wl.p, wl.n, wl.half_width) if breaks is None else ofe.mesh3d_graded(wl.p, breaks)
            Xc = rng.standard_normal((om.n_free, ncol))
            vc = v_fixed.cpu().numpy()
            t0 = time.perf_counter()
            ofe.hamiltonian_apply(om, vc, Xc)
            t_apply = time.perf_counter() - t0
            what = f"one FP64 oracle Kronecker apply of the {ncol}-column block on the {om.n_free}-node mesh"
        else:
            # the oracle's assembled operator on a 4^3-cell mapped mesh of the same order and cell
            # size, timed per cell and scaled to the workload's cell count
            from oracle import mapped as omapped
            nsm = 4
            om = omapped.mapped_mesh(wl.p, nsm, wl.half_width * nsm / wl.n, args.mapped)
            Xc = rng.standard_normal((om.n_free, ncol))
            vc = rng.uniform(-1, 1, om.n_free)
            Kc = om.kinetic_csr()
            t0 = time.perf_counter()
            for _ in range(5):
                Kc @ Xc + vc[:, None] * Xc
            t_apply = (time.perf_counter() - t0) / 5 * mesh.n_cells / nsm ** 3
            what = (f"the oracle's assembled FP64 operator on a {nsm}^3-cell mapped mesh ({om.n_free} nodes, "
                    f"{ncol} columns), scaled by cells to the {mesh.n_cells}-cell mesh")
        del Xc
        # applies per gradient iteration of the measured GPU path: filter passes x degree + MINRES iterations
        passes = sum(st.passes) / max(1, len(st.passes)) * (st.n_forward / max(1, head["steps"]))
        applies = passes * (wl.cheb_degree + 1) + sum(st.adj_iters) / max(1, len(st.adj_iters)) + 2
        model, threads = host_cpu()
        cpu = {"value": 1.0 / (t_apply * applies), "unit": "grad_iter/s", "cores": threads,
               "kind": "oracle", "cpu_model": model, "logical_cpus": os.cpu_count(),
               "sample": (f"{what} ({t_apply:.1f} s), scaled by {applies:.0f} applies per gradient iteration "
                          f"(the GPU path's measured filter passes x degree + MINRES iterations)")}
        gpath = os.path.join(ROOT, "tests", "golden", "mol10_q4_24.json")
        if os.path.exists(gpath):            # the oracle's own method, timed where the fixture was written
            g = json.load(open(gpath))
            cpu["oracle_full_method"] = {"workload": g["workload"], "n_free": g["n_free"],
                                         "seconds_per_gradient_iteration": g["oracle_seconds"]["gradient_iteration"],
                                         "method": "eigsh (tol 1e-13) + projected CG (rtol 1e-12)",
                                         "host": g["host"]}

    line = {
        "metric": "ks_apply GB/s (% roofline) + inverse-DFT gradient iters/s vs FP64 GPU path",
        "value": ips,
        "unit": "grad_iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * head["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_name == "mixed" else "f64",
        "data": "synthetic (seeded model molecule; target density from a known potential)",
        "config": {"workload": wname, "p": wl.p, "cells_per_dim": mesh.n, "half_width": wl.half_width,
                   "n_free": mesh.n_free, "electrons": wl.n_elec, "block": nv, "cheb_degree": wl.cheb_degree,
                   **({"kT": kT, "converged": nconv, "orbitals_included": head["n_incl"]} if kT > 0 else {}),
                   **({"vxc_h": args.vxc_h, "vxc_vertices": vxc.n_vertices} if vxc is not None else {}),
                   **({"graded_inner_h": args.graded, "growth": 1.35} if args.graded > 0 else {}),
                   **({"mapped_amp": args.mapped, "cells": mesh.n_cells} if args.mapped is not None else {}),
                   **({"adjoint_deflation": deflate} if head_name in ("mixed", "f64d") and deflate > 0 else {})},
        "ks_apply_GBps_f32": gbs32,
        "ks_apply_GBps_f64": gbs64,
        "ks_apply_ms_f32": ms32,
        "ks_apply_ms_f64": ms64,
        **out_extra,
        **vxc_info,
        **fe_info,
        "roofline": roofline,
        "minres_sweeps": sweeps,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
