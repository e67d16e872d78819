"""GPU tests of the mixed-precision paths and the autograd/L-BFGS driver (needs an MI355X)."""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fe, ks  # noqa: E402
from synth import random_block, random_directions, workload  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@functools.lru_cache(maxsize=None)
def _small():
    """Workload-2 molecule on a small Q4 mesh: oracle rho_data, potential and gradient."""
    from paper_2510_10529_amd import api
    wl = workload(2, p=4, n=6, half_width=7.0)
    om = fe.mesh3d(wl.p, wl.n, wl.half_width)
    X = om.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    rho_d, _ = ks.target_density(om, vf + vs, wl.n_elec)
    u = 0.3 * vs + 0.1 * np.exp(-np.sum((X - 0.5) ** 2, axis=1))
    ev = ks.evaluate(om, vf + u, rho_d, wl.n_elec, method="cg", extra=4)
    m = api.Mesh(wl.p, wl.n, wl.half_width)
    return wl, om, vf, vs, rho_d, u, ev, m


def _forward(prec):
    from paper_2510_10529_amd import api
    wl, om, vf, vs, rho_d, u, ev, m = _small()
    nv = wl.n_occ + wl.n_buf
    X = _t(random_block(om.n_free, nv, 3))
    v = _t(vf + u)
    r = api.ks_eigensolve(m, v, X, wl.n_occ, 20, 1e-10, 300, prec=prec, switch_tol=1e-4)
    return v, X, r


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_forward_precisions_reach_fp64_accuracy(prec):
    wl, om, vf, vs, rho_d, u, ev, m = _small()
    v, X, r = _forward(prec)
    assert r.status == 0, r
    k = wl.n_occ
    np.testing.assert_allclose(r.eig[:k], ev.eps[:k], atol=1e-8)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_precisions_match_oracle_gradient(prec):
    from paper_2510_10529_amd import api
    wl, om, vf, vs, rho_d, u, ev, m = _small()
    v, X, r = _forward("f64")
    k = wl.n_occ
    Psi = X[:, :k].contiguous()
    rho, B, loss = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d))
    Q, ar = api.adjoint_solve(m, v, Psi, r.eig[:k], B, tol=1e-10, maxit=20000, prec=prec)
    assert ar.status == 0, ar
    assert max(ar.relres) <= 2e-10, ar.relres   # the Euclidean bar of the solve
    g = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d), Q=Q).cpu().numpy()
    rel = np.linalg.norm(g - ev.grad) / np.linalg.norm(ev.grad)
    assert rel <= 1e-6, rel


def test_autograd_function_matches_fd():
    """dL/du from InvDFTLoss.backward against central differences of the GPU loss (h = 1e-5)."""
    from paper_2510_10529_amd import api, inverse
    wl, om, vf, vs, rho_d, u, ev, m = _small()
    nv = wl.n_occ + wl.n_buf
    prob = inverse.InverseProblem(m, _t(vf), _t(rho_d), wl.n_elec, _t(random_block(om.n_free, nv, 4)),
                                  inverse.SolverOptions(degree=20, tol_eig=1e-11, tol_adj=1e-11, recompute=True))
    ut = _t(u).requires_grad_(True)
    loss = inverse.InvDFTLoss.apply(ut, prob)
    loss.backward()
    g = ut.grad.cpu().numpy()
    np.testing.assert_allclose(float(loss), ev.loss, rtol=1e-8)
    assert np.linalg.norm(g - ev.grad) / np.linalg.norm(ev.grad) < 1e-6
    h = 1e-5
    for d in random_directions(om.n_free, 3, 11):
        lp, _ = prob.evaluate(_t(u + h * d), want_grad=False)
        lm, _ = prob.evaluate(_t(u - h * d), want_grad=False)
        fd = (lp - lm) / (2 * h)
        assert abs(g @ d - fd) <= 1e-5 * abs(fd) + 1e-12, (g @ d, fd)


def test_lbfgs_decreases_loss():
    from paper_2510_10529_amd import inverse
    wl, om, vf, vs, rho_d, u, ev, m = _small()
    nv = wl.n_occ + wl.n_buf
    prob = inverse.InverseProblem(m, _t(vf), _t(rho_d), wl.n_elec, _t(random_block(om.n_free, nv, 5)),
                                  inverse.SolverOptions(degree=20, tol_eig=1e-10, tol_adj=1e-10))
    u0 = torch.zeros(om.n_free, dtype=torch.float64, device=DEV)
    uT, losses = inverse.lbfgs(prob, u0, maxiter=6)
    assert losses[-1] < 0.2 * losses[0], losses
    assert all(np.isfinite(losses))


def test_degenerate_gap_status():
    """A harmonic trap with 4 electrons puts the Fermi level inside the exactly degenerate shell."""
    from paper_2510_10529_amd import _lib, api
    m = api.Mesh(3, 4, 5.0)
    om = fe.mesh3d(3, 4, 5.0)
    X = om.coords()
    v = _t(0.5 * np.sum(X * X, axis=1))
    Xb = _t(random_block(om.n_free, 8, 6))
    r = api.ks_eigensolve(m, v, Xb, 2, 16, 1e-9, 200)
    assert r.status == _lib.FE_EGAP


@functools.lru_cache(maxsize=None)
def _twenty_electrons():
    """Workload-3 molecule (20 electrons, 10 adjoint columns) on a small Q4 mesh."""
    from paper_2510_10529_amd import api
    wl = workload(3, p=4, n=6, half_width=8.0)
    om = fe.mesh3d(wl.p, wl.n, wl.half_width)
    X = om.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    rho_d, _ = ks.target_density(om, vf + vs, wl.n_elec)
    u = 0.5 * vs
    ev = ks.evaluate(om, vf + u, rho_d, wl.n_elec, method="cg", extra=4)
    return wl, om, vf, rho_d, u, ev, api.Mesh(wl.p, wl.n, wl.half_width)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_column_compaction_matches_oracle(prec):
    """Ten adjoint columns converge at different rates, so converged columns are dropped
    from the batch mid-solve; the gradient must still match the oracle's."""
    from paper_2510_10529_amd import api
    wl, om, vf, rho_d, u, ev, m = _twenty_electrons()
    k = wl.n_occ
    assert k >= 8
    X = _t(random_block(om.n_free, k + wl.n_buf, 8))
    v = _t(vf + u)
    r = api.ks_eigensolve(m, v, X, k, 20, 1e-10, 300)
    assert r.status == 0, r
    Psi = X[:, :k].contiguous()
    rho, B, loss = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d))
    Q, ar = api.adjoint_solve(m, v, Psi, r.eig[:k], B, tol=1e-10, maxit=20000, prec=prec)
    assert ar.status == 0, ar
    assert max(ar.relres) <= 2e-10, ar.relres   # the Euclidean bar of the solve
    assert len(set(ar.iters)) > 1          # columns did converge at different iterations
    g = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d), Q=Q).cpu().numpy()
    rel = np.linalg.norm(g - ev.grad) / np.linalg.norm(ev.grad)
    assert rel <= 1e-6, rel
