"""GPU checks against closed forms and of the driver's far-field mask and adaptive tolerances
(needs an MI355X).

* Harmonic trap v = r^2/2 on the Q5 mesh with 16 cells a side of [-8, 8]^3 (493,039 free
  nodes): the eigenvalues approach n + 3/2 (ground state 3/2, first shell 5/2 three-fold;
  the 1-D discretisation errors of this mesh are about 1e-8 and 2e-7, so the 3-D levels
  are within 1e-7 and 1e-6), and the first shell is exactly degenerate because the mesh
  has the cube's symmetry.
* The far-field treatment of Sec. 3.1.2: the gradient is zero where rho_data < tau_BC,
  in loss_grad and through the autograd driver, against the oracle's masked gradient.
* The adaptive tolerances of Table 1: t_eig = e_L2^2 / c_eig and t_ad = e_L2^2 / c_ad,
  with e_L2^2 = L the loss of the last forward solve; the gradient they give stays within
  the accuracy those tolerances allow of the oracle's.
"""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fe, ks  # noqa: E402
from synth import random_block, workload  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def test_harmonic_trap_closed_form_q5_16_cells():
    from paper_2510_10529_amd import api
    p, n, L = 5, 16, 8.0
    m = api.Mesh(p, n, L)
    assert m.n_free == 79 ** 3
    xyz, _ = m.nodes()
    v = 0.5 * (xyz * xyz).sum(dim=1)
    nocc, nv = 4, 14
    X = _t(random_block(m.n_free, nv, 21))
    r = api.ks_eigensolve(m, v.contiguous(), X, nocc, 30, 1e-10, 400)
    assert r.status == 0, r
    assert max(r.res[:nocc]) <= 1e-10
    e = np.array(r.eig[:nocc])
    assert abs(e[0] - 1.5) <= 1e-7, e[0] - 1.5
    assert np.abs(e[1:] - 2.5).max() <= 1e-6, e[1:] - 2.5
    assert np.ptp(e[1:]) <= 1e-10, np.ptp(e[1:])
    m.close()


# ---------------------------------------------------------------- far field (tau_BC)
@functools.lru_cache(maxsize=None)
def _cfg1():
    from paper_2510_10529_amd import api
    wl = workload(1)
    om = fe.mesh3d(wl.p, wl.n, wl.half_width)
    X = om.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    rho_d, _ = ks.target_density(om, vf + vs, wl.n_elec)
    u = 0.4 * np.sin(X[:, 0]) * np.exp(-0.05 * np.sum(X * X, axis=1))
    m = api.Mesh(wl.p, wl.n, wl.half_width)
    return wl, om, vf, vs, rho_d, u, m


@pytest.mark.parametrize("tau", [1e-7, 1e-6])
def test_loss_grad_far_field_mask(tau):
    from paper_2510_10529_amd import api
    wl, om, vf, vs, rho_d, u, m = _cfg1()
    ev = ks.evaluate(om, vf + u, rho_d, wl.n_elec, method="bordered", extra=4, tau_bc=tau)
    masked = rho_d < tau
    assert 0.05 < masked.mean() < 0.95                     # the mask is not trivial here
    nv = wl.n_occ + wl.n_buf
    X = _t(random_block(om.n_free, nv, 1))
    v = _t(vf + u)
    r = api.ks_eigensolve(m, v, X, wl.n_occ, wl.cheb_degree, 1e-11, 300)
    assert r.status == 0, r
    k = wl.n_occ
    Psi = X[:, :k].contiguous()
    rho, B, loss = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d))
    Q, ar = api.adjoint_solve(m, v, Psi, r.eig[:k], B, tol=1e-12, maxit=4000)
    assert ar.status == 0, ar
    g = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d), Q=Q, tau_bc=tau).cpu().numpy()
    g0 = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d), Q=Q).cpu().numpy()
    assert np.all(g[masked] == 0.0)
    np.testing.assert_array_equal(g[~masked], g0[~masked])   # the mask changes nothing else
    rel = np.linalg.norm(g - ev.grad) / np.linalg.norm(ev.grad)
    assert rel <= 1e-6, rel
    np.testing.assert_array_equal(ev.grad[masked], 0.0)


def test_autograd_far_field_mask():
    from paper_2510_10529_amd import inverse
    wl, om, vf, vs, rho_d, u, m = _cfg1()
    tau = 1e-6
    ev = ks.evaluate(om, vf + u, rho_d, wl.n_elec, method="bordered", extra=4, tau_bc=tau)
    nv = wl.n_occ + wl.n_buf
    prob = inverse.InverseProblem(m, _t(vf), _t(rho_d), wl.n_elec, _t(random_block(om.n_free, nv, 4)),
                                  inverse.SolverOptions(degree=wl.cheb_degree, tol_eig=1e-11, tol_adj=1e-11,
                                                        tau_bc=tau))
    ut = _t(u).requires_grad_(True)
    loss = inverse.InvDFTLoss.apply(ut, prob)
    loss.backward()
    g = ut.grad.cpu().numpy()
    assert abs(float(loss.detach()) - ev.loss) <= 1e-8 * ev.loss
    assert np.all(g[rho_d < tau] == 0.0)
    assert np.linalg.norm(g - ev.grad) / np.linalg.norm(ev.grad) <= 1e-6


# ----------------------------------------------------------- adaptive tolerances
def test_adaptive_tolerances_follow_the_loss():
    """t_eig = L / c_eig and t_ad = L / c_ad (Table 1's defaults c_eig = 1e2, c_ad = 1e5), L the loss
    of the last forward solve, capped by the fixed tolerances. The eigensolver meets t_eig, each
    adjoint column t_ad (Euclidean, to the stop test's factor), and the gradient agrees with the
    oracle's to what these tolerances allow: an orbital residual t gives density errors of order
    t / gap against |rho - rho_data| ~ sqrt(L), so the relative error is of order t_eig / sqrt(L)."""
    from paper_2510_10529_amd import api, inverse
    wl, om, vf, vs, rho_d, _, m = _cfg1()
    u = 0.97 * vs                                            # close to the target: L ~ 1.7e-6
    ev = ks.evaluate(om, vf + u, rho_d, wl.n_elec, method="bordered", extra=4)
    nv = wl.n_occ + wl.n_buf
    opts = inverse.SolverOptions(degree=wl.cheb_degree, tol_eig=1e-4, tol_adj=1e-4, adaptive=True)
    prob = inverse.InverseProblem(m, _t(vf), _t(rho_d), wl.n_elec, _t(random_block(om.n_free, nv, 4)), opts)
    assert prob.tolerances() == (1e-4, 1e-4)                   # no loss yet: the fixed caps
    loss0, _ = prob.evaluate(_t(u), want_grad=False)
    assert abs(loss0 - ev.loss) <= 0.1 * ev.loss
    t_eig, t_ad = prob.tolerances()
    assert t_eig == pytest.approx(loss0 / 1e2, rel=1e-15)
    assert t_ad == pytest.approx(loss0 / 1e5, rel=1e-15)
    assert 1e-12 < t_ad < t_eig < 1e-4                        # neither clamp is active
    loss, g = prob.evaluate(_t(u))                             # runs with t_eig and t_ad
    g = g.cpu().numpy()
    k = wl.n_occ
    assert prob.stats.passes[-1] >= 1                          # the tighter t_eig needed more passes
    v = _t(vf + u)
    Psi = prob.psi()
    X = prob.X.clone()
    r = api.rayleigh_ritz(m, v, X)
    assert max(r[1][:k]) <= 1.01 * t_eig
    rho, B, _ = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d))
    Q, ar = api.adjoint_solve(m, v, Psi, prob.eig[:k], B, tol=t_ad, maxit=4000)
    assert max(ar.relres) <= 5 * t_ad, (ar.relres, t_ad)
    assert abs(loss - ev.loss) <= 10 * t_eig / np.sqrt(ev.loss) * ev.loss
    rel = np.linalg.norm(g - ev.grad) / np.linalg.norm(ev.grad)
    assert rel <= max(1e-6, 50 * (t_eig + t_ad) / np.sqrt(ev.loss)), (rel, t_eig)
