"""GPU parity of every C-ABI call against the FP64 oracle (needs an MI355X).

Sizes span several workgroup tiles with ragged tails (cell counts that are not a
multiple of the tile edge, column counts that are not a multiple of the column
chunk) and several z-segments per launch.
"""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import chfsi, fe, ks  # noqa: E402
from synth import random_block, workload  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _api():
    from paper_2510_10529_amd import api
    return api


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@functools.lru_cache(maxsize=None)
def _mesh_pair(p, n, L):
    return _api().Mesh(p, n, L), fe.mesh3d(p, n, L)


def _potential(cfg, om):
    wl = workload(cfg, p=om.m1.p, n=om.m1.n, half_width=om.m1.L)
    X = om.coords()
    return wl, wl.v_fixed(X), wl.v_xc_target(X)


# ------------------------------------------------------------------ mesh tables
@pytest.mark.parametrize("p,n,L", [(1, 5, 2.0), (2, 6, 6.0), (4, 3, 5.0), (5, 3, 4.0), (8, 2, 3.0)])
def test_mesh_tables(p, n, L):
    m, om = _mesh_pair(p, n, L)
    assert m.n_free == om.n_free
    xyz, w = m.nodes()
    np.testing.assert_allclose(xyz.cpu().numpy(), om.coords(), atol=1e-13)
    np.testing.assert_allclose(w.cpu().numpy(), om.weights(), rtol=1e-13)
    np.testing.assert_allclose(m.kinetic_diag().cpu().numpy(), fe.kinetic_diag(om), rtol=1e-12)
    eb = fe.element_bound(p, 2 * L / n)
    if p <= 5:
        assert abs(m.kin_bound - eb) <= 1e-11 * eb
    else:
        assert m.kin_bound >= eb * (1 - 1e-12)


# --------------------------------------------------------------------- ks_apply
APPLY_CASES = [
    (1, 9, 3.0, 3), (2, 6, 4.0, 5), (2, 13, 8.0, 4), (3, 5, 4.0, 9), (4, 5, 5.0, 11),
    (5, 5, 5.0, 8), (5, 3, 4.0, 17), (6, 3, 4.0, 3), (7, 2, 3.0, 2), (8, 3, 4.0, 1),
]


@pytest.mark.parametrize("p,n,L,nv", APPLY_CASES)
def test_ks_apply_f64(p, n, L, nv):
    api = _api()
    m, om = _mesh_pair(p, n, L)
    wl, vf, vs = _potential(2, om)
    v = vf + vs
    X = random_block(om.n_free, nv, 100 + p)
    shift = np.linspace(-1.0, 2.0, nv)
    ref = fe.hamiltonian_apply(om, v, X) - X * shift[None, :]
    Y = api.ks_apply(m, _t(v), _t(X), shift=list(shift)).cpu().numpy()
    scale = np.abs(ref).max()
    np.testing.assert_allclose(Y, ref, rtol=0, atol=2e-14 * scale * (p + 1))


@pytest.mark.parametrize("p,n,L,nv", [(2, 6, 4.0, 5), (4, 5, 5.0, 20), (5, 5, 5.0, 17)])
def test_ks_apply_f32(p, n, L, nv):
    api = _api()
    m, om = _mesh_pair(p, n, L)
    wl, vf, vs = _potential(2, om)
    v = vf + vs
    X = random_block(om.n_free, nv, 200 + p).astype(np.float32)
    ref = fe.hamiltonian_apply(om, v, X.astype(np.float64))
    Xt = torch.tensor(X, device=DEV)
    Y = api.ks_apply(m, _t(v), Xt, prec="f32").cpu().numpy().astype(np.float64)
    # FP32 storage and arithmetic: error ~ eps32 * (sum of |terms|) ~ eps32 * lambda_max * |x|
    scale = np.abs(ref).max()
    assert np.abs(Y - ref).max() <= 2e-5 * scale


def test_ks_apply_bitwise_reproducible():
    api = _api()
    m, om = _mesh_pair(5, 5, 5.0)
    wl, vf, vs = _potential(3, om)
    v = _t(vf + vs)
    X = _t(random_block(om.n_free, 13, 5))
    Y1 = api.ks_apply(m, v, X)
    Y2 = api.ks_apply(m, v, X)
    assert torch.equal(Y1, Y2)


def test_kinetic_closed_form_on_gpu():
    """u~^T (K~/2) u~ = 1024 L^13 / 225 for u = prod (L^2 - x^2) (p >= 2)."""
    api = _api()
    for p, n, L in [(2, 6, 3.0), (5, 3, 2.0)]:
        m, om = _mesh_pair(p, n, L)
        X = om.coords()
        u = np.sqrt(om.weights()) * np.prod(L * L - X * X, axis=1)
        Y = api.ks_apply(m, _t(np.zeros(om.n_free)), _t(u[:, None])).cpu().numpy()[:, 0]
        assert abs(u @ Y / (1024 * L ** 13 / 225) - 1) < 1e-12


# --------------------------------------------------------------- filter and RR
def test_cheb_filter_matches_oracle():
    api = _api()
    m, om = _mesh_pair(3, 5, 5.0)
    wl, vf, vs = _potential(2, om)
    v = vf + vs
    X = random_block(om.n_free, 9, 11)
    a, b, a0 = 5.0, fe.element_bound(3, 2.0) + v.max(), v.min() - 1.0
    ref = chfsi.filter_apply(lambda Z: fe.hamiltonian_apply(om, v, Z), X, 7, a, b, a0)
    Xt = _t(X)
    api.cheb_filter(m, _t(v), 7, a, b, a0, Xt)
    np.testing.assert_allclose(Xt.cpu().numpy(), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_rayleigh_ritz_matches_oracle():
    api = _api()
    m, om = _mesh_pair(4, 4, 5.0)
    wl, vf, vs = _potential(2, om)
    v = vf + vs
    X = random_block(om.n_free, 12, 12)
    w_ref, _, res_ref = chfsi.rayleigh_ritz(lambda Z: fe.hamiltonian_apply(om, v, Z), X)
    Xt = _t(X)
    eig, res = api.rayleigh_ritz(m, _t(v), Xt)
    np.testing.assert_allclose(eig, w_ref, rtol=1e-11, atol=1e-10)
    np.testing.assert_allclose(res, res_ref, rtol=1e-8)
    Psi = Xt.cpu().numpy()
    np.testing.assert_allclose(Psi.T @ Psi, np.eye(12), atol=1e-11)


# ------------------------------------------------------- config-1 end to end
@functools.lru_cache(maxsize=None)
def _cfg1_oracle():
    wl = workload(1)
    om = fe.mesh3d(wl.p, wl.n, wl.half_width)
    X = om.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    rho_d, _ = ks.target_density(om, vf + vs, wl.n_elec)
    u = 0.4 * np.sin(X[:, 0]) * np.exp(-0.05 * np.sum(X * X, axis=1))
    ev = ks.evaluate(om, vf + u, rho_d, wl.n_elec, method="bordered", extra=4)
    return wl, om, vf, vs, rho_d, u, ev


@functools.lru_cache(maxsize=None)
def _cfg1_gpu_forward():
    api = _api()
    wl, om, vf, vs, rho_d, u, ev = _cfg1_oracle()
    m, _ = _mesh_pair(wl.p, wl.n, wl.half_width)
    nv = wl.n_occ + wl.n_buf
    X = _t(random_block(om.n_free, nv, 1))
    v = _t(vf + u)
    r = api.ks_eigensolve(m, v, X, wl.n_occ, wl.cheb_degree, 1e-10, 300)
    return m, v, X, r


def test_cfg1_eigenvalues_and_density():
    api = _api()
    wl, om, vf, vs, rho_d, u, ev = _cfg1_oracle()
    m, v, X, r = _cfg1_gpu_forward()
    assert r.status == 0, r
    k = wl.n_occ
    assert max(r.res[:k]) <= 1e-10
    np.testing.assert_allclose(r.eig[:k], ev.eps[:k], rtol=0, atol=1e-8)
    Psi = X[:, :k].contiguous()
    rho, B, loss = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d))
    W = om.weights()
    l1 = np.sum(W * np.abs(rho.cpu().numpy() - ev.rho))
    assert l1 <= 1e-7, l1
    assert abs(np.sum(W * rho.cpu().numpy()) - wl.n_elec) < 1e-10
    assert abs(loss - ev.loss) <= 1e-7 * ev.loss


def test_cfg1_loss_grad_phase1_on_oracle_orbitals():
    """loss_grad on the oracle's own orbitals: rho, L and B element by element."""
    api = _api()
    wl, om, vf, vs, rho_d, u, ev = _cfg1_oracle()
    m, _ = _mesh_pair(wl.p, wl.n, wl.half_width)
    k = wl.n_occ
    psi = ev.psi[:, :k]
    occ = ks.occupations(wl.n_elec)
    rho, B, loss = api.loss_grad(m, _t(psi), list(occ), _t(rho_d))
    np.testing.assert_allclose(rho.cpu().numpy(), ks.density(psi, occ, om.weights()), rtol=1e-13, atol=1e-16)
    Bref = ks.adjoint_rhs(psi, occ, ks.density(psi, occ, om.weights()), rho_d)
    np.testing.assert_allclose(B.cpu().numpy(), Bref, rtol=0, atol=1e-12 * np.abs(Bref).max())
    assert abs(loss - ks.loss(ks.density(psi, occ, om.weights()), rho_d, om.weights())) <= 1e-12 * loss


def test_cfg1_adjoint_and_gradient():
    api = _api()
    wl, om, vf, vs, rho_d, u, ev = _cfg1_oracle()
    m, v, X, r = _cfg1_gpu_forward()
    k = wl.n_occ
    Psi = X[:, :k].contiguous()
    rho, B, loss = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d))
    Q, ar = api.adjoint_solve(m, v, Psi, r.eig[:k], B, tol=1e-12, maxit=4000)
    assert ar.status == 0, ar
    assert max(ar.relres) < 1e-9, ar.relres
    Qn = Q.cpu().numpy()
    np.testing.assert_allclose(Psi.cpu().numpy().T @ Qn, 0, atol=1e-10 * np.abs(Qn).max())
    g = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d), Q=Q).cpu().numpy()
    rel = np.linalg.norm(g - ev.grad) / np.linalg.norm(ev.grad)
    assert rel <= 1e-6, rel
    assert abs(g.sum()) <= 1e-8 * np.abs(g).sum()      # gauge invariance


def test_adjoint_noconv_status():
    api = _api()
    from paper_2510_10529_amd import _lib
    wl, om, vf, vs, rho_d, u, ev = _cfg1_oracle()
    m, v, X, r = _cfg1_gpu_forward()
    k = wl.n_occ
    Psi = X[:, :k].contiguous()
    rho, B, loss = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d))
    Q, ar = api.adjoint_solve(m, v, Psi, r.eig[:k], B, tol=1e-14, maxit=1)
    assert ar.status == _lib.FE_ENOCONV
    assert all(i == 1 for i in ar.iters)


def test_bf16_is_refused_where_not_supported():
    """FE_BF16 blocks are taken by the apply, the filter and the eigensolver only."""
    from paper_2510_10529_amd import _lib
    api = _api()
    m, om = _mesh_pair(2, 6, 4.0)
    k = 4
    Psi = torch.zeros((om.n_free, k), dtype=torch.float64, device=DEV)
    v = torch.zeros(om.n_free, dtype=torch.float64, device=DEV)
    with pytest.raises(_lib.FEError) as e:
        api.adjoint_solve(m, v, Psi, [0.0] * k, Psi.clone(), prec="bf16", work=torch.empty(1 << 20, dtype=torch.uint8,
                                                                                         device=DEV))
    assert e.value.status == _lib.FE_EINVAL
