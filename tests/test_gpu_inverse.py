"""The differentiation path at full size (workload mol20-q4-32: p = 4, 32^3 cells,
2,048,383 free nodes, 10 orbitals; needs an MI355X).

The gradient of the autograd Function is checked by central differences on 16 seeded
directions (h = 1e-5), then 30 L-BFGS steps run from u = 0 through the autograd
adjoint. The target density is the density of the known potential v_fixed + v*, so the
loss must fall and the recovered potential must move towards v*.
"""
import functools
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import random_block, random_directions, workload  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(f"[inverse] {msg}", file=sys.stderr, flush=True)


@functools.lru_cache(maxsize=None)
def _problem():
    from paper_2510_10529_amd import api
    from paper_2510_10529_amd import inverse as inv
    wl = workload(3)
    m = api.Mesh(wl.p, wl.n, wl.half_width)
    xyz, _ = m.nodes()
    xh = xyz.cpu().numpy()
    del xyz
    vf = torch.tensor(wl.v_fixed(xh), device=DEV)
    vs = torch.tensor(wl.v_xc_target(xh), device=DEV)
    nocc, nv = wl.n_occ, wl.n_occ + wl.n_buf
    X = torch.tensor(random_block(m.n_free, nv, 1003), device=DEV)
    r = api.ks_eigensolve(m, vf + vs, X, nocc, wl.cheb_degree, 1e-10, 400)
    assert r.status == 0, r
    rho_d, _, _ = api.loss_grad(m, X[:, :nocc].contiguous(), [2.0] * nocc, torch.zeros_like(vf), want_B=False)
    X0 = torch.tensor(random_block(m.n_free, nv, 2003), device=DEV)
    r0 = api.ks_eigensolve(m, vf, X0, nocc, wl.cheb_degree, 1e-10, 400)
    assert r0.status == 0, r0
    opts = inv.SolverOptions(degree=wl.cheb_degree, tol_eig=1e-10, tol_adj=1e-10)
    return wl, m, vf, vs, rho_d, inv.InverseProblem(m, vf, rho_d, wl.n_elec, X0, opts)


def test_gradient_central_differences_16_directions():
    from paper_2510_10529_amd import inverse as inv
    wl, m, vf, vs, rho_d, prob = _problem()
    u0 = torch.zeros_like(vf)
    ur = u0.clone().requires_grad_(True)
    loss = inv.InvDFTLoss.apply(ur, prob)
    loss.backward()
    g = ur.grad.detach()
    h = 1e-5
    worst = 0.0
    prob.opts.tol_eig = 1e-11             # loss values accurate well below h^2
    try:
        for d in random_directions(m.n_free, 16, 3003):
            dt = torch.tensor(d, device=DEV)
            lp, _ = prob.evaluate(u0 + h * dt, want_grad=False)
            lm, _ = prob.evaluate(u0 - h * dt, want_grad=False)
            fd = (lp - lm) / (2 * h)
            gd = float((g * dt).sum())
            worst = max(worst, abs(gd - fd) / abs(fd))
    finally:
        prob.opts.tol_eig = 1e-10
    _say(f"central differences, 16 directions: worst relative difference {worst:.2e}")
    assert worst <= 1e-5


def test_lbfgs_30_steps_recovers_towards_known_potential():
    from paper_2510_10529_amd import inverse as inv
    wl, m, vf, vs, rho_d, prob = _problem()
    mask = rho_d >= 1e-3

    def rms(u):
        # the density does not see a constant shift of the potential: compare up to the mean
        d = (u - vs)[mask]
        d = d - d.mean()
        return float(torch.sqrt((d * d).mean()))

    u0 = torch.zeros_like(vf)
    uT, losses = inv.lbfgs(prob, u0, maxiter=30)
    _say(f"L-BFGS 30 steps: loss {losses[0]:.3e} -> {losses[-1]:.3e}; "
         f"RMS(u - v*) over rho_d >= 1e-3: {rms(u0):.3e} -> {rms(uT):.3e} Ha")
    assert all(np.isfinite(losses))
    assert all(b <= a for a, b in zip(losses, losses[1:]))      # Armijo steps only
    assert losses[-1] <= 1e-2 * losses[0]
    assert rms(uT) < 0.78 * rms(u0)          # measured 0.747 (7.64e-2 -> 5.71e-2 Ha)


def test_lbfgs_30_steps_on_a_linear_xc_mesh():
    """With v_xc on the paper's linear mesh (Eq. 14; uniform 0.5 bohr cells on the inner cube,
    growing by 1.4 outwards) the density constrains far fewer unknowns, and the same 30 steps
    move the potential much further towards v*: measured 7.64e-2 -> 4.01e-2 Ha over rho_d >= 1e-3
    and 8.02e-2 -> 2.19e-2 Ha over rho_d >= 1e-2."""
    from paper_2510_10529_amd import api
    from paper_2510_10529_amd import inverse as inv
    from synth import vxc_vertices
    wl, m, vf, vs, rho_d, prob0 = _problem()
    tv = vxc_vertices(wl.half_width, 0.5, 0.5 * wl.half_width, 1.4)
    vm = api.VxcMesh(m, tv, tv, tv)
    prob = inv.InverseProblem(m, vf, rho_d, wl.n_elec, prob0.X, prob0.opts, vxc=vm)
    zero = torch.zeros_like(vf)

    def rms(uv, tau):
        mask = rho_d >= tau
        d = (vm.prolong(uv, base=zero) - vs)[mask]
        d = d - d.mean()
        return float(torch.sqrt((d * d).mean()))

    u0 = prob.zeros_u()
    uT, losses = inv.lbfgs(prob, u0, maxiter=30)
    _say(f"L-BFGS 30 steps on the linear mesh ({vm.n_vertices} vertices): loss {losses[0]:.3e} -> {losses[-1]:.3e}; "
         f"RMS over rho_d >= 1e-3 {rms(u0, 1e-3):.3e} -> {rms(uT, 1e-3):.3e}, "
         f">= 1e-2 {rms(u0, 1e-2):.3e} -> {rms(uT, 1e-2):.3e} Ha")
    assert all(b <= a for a, b in zip(losses, losses[1:]))
    assert rms(uT, 1e-3) < 0.6 * rms(u0, 1e-3)
    assert rms(uT, 1e-2) < 0.35 * rms(u0, 1e-2)
