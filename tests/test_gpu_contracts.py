"""GPU tests of the C ABI's contracts (needs an MI355X): blocks with a row pitch ld larger than
their column count, and the adjoint solves' iteration budget and Euclidean residual bar."""
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


@functools.lru_cache(maxsize=None)
def _small():
    from paper_2510_10529_amd import api
    wl = workload(2, p=4, n=6, half_width=7.0)
    om = fe.mesh3d(wl.p, wl.n, wl.half_width)
    X = om.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    rho_d, _ = ks.target_density(om, vf + vs, wl.n_elec)
    u = 0.3 * vs
    m = api.Mesh(wl.p, wl.n, wl.half_width)
    return wl, om, vf, rho_d, u, m


def _padded(X, pad):
    """The same columns in a block with row pitch X.shape[1] + pad (padding filled with NaN)."""
    Xp = torch.full((X.shape[0], X.shape[1] + pad), float("nan"), dtype=X.dtype, device=X.device)
    Xp[:, :X.shape[1]] = X
    return Xp


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_eigensolve_with_row_pitch(prec):
    """ld = nv + 8: the same Ritz values, residuals and vectors as ld = nv (the work blocks follow
    ld, sized by fe_workspace_bytes(op, ld)), and the padding columns are never read."""
    from paper_2510_10529_amd import api
    wl, om, vf, rho_d, u, m = _small()
    nv = wl.n_occ + wl.n_buf
    X0 = _t(random_block(om.n_free, nv, 3))
    v = _t(vf + u)
    Xa = X0.clone()
    ra = api.ks_eigensolve(m, v, Xa, wl.n_occ, 20, 1e-10, 300, prec=prec, switch_tol=1e-4)
    Xb = _padded(X0, 8)
    rb = api.ks_eigensolve(m, v, Xb, wl.n_occ, 20, 1e-10, 300, prec=prec, switch_tol=1e-4, nv=nv)
    assert ra.status == 0 and rb.status == 0
    assert ra.passes == rb.passes
    np.testing.assert_allclose(rb.eig, ra.eig, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Xb[:, :nv].cpu().numpy(), Xa.cpu().numpy(), rtol=0, atol=1e-10)


def test_filter_and_rayleigh_ritz_with_row_pitch():
    from paper_2510_10529_amd import api
    wl, om, vf, rho_d, u, m = _small()
    nv = 9
    X0 = _t(random_block(om.n_free, nv, 5))
    v = _t(vf + u)
    Xa, Xb = X0.clone(), _padded(X0, 7)
    api.cheb_filter(m, v, 12, 0.5, m.kin_bound + float(v.max()), -3.0, Xa)
    api.cheb_filter(m, v, 12, 0.5, m.kin_bound + float(v.max()), -3.0, Xb, nv=nv)
    np.testing.assert_array_equal(Xb[:, :nv].cpu().numpy(), Xa.cpu().numpy())   # same kernels, same order
    assert torch.isnan(Xb[:, nv:]).all()
    ea, resa = api.rayleigh_ritz(m, v, Xa)
    eb, resb = api.rayleigh_ritz(m, v, Xb, nv=nv)
    np.testing.assert_allclose(eb, ea, rtol=1e-13)
    np.testing.assert_allclose(Xb[:, :nv].cpu().numpy(), Xa.cpu().numpy(), rtol=0, atol=1e-12)


# ----------------------------------------------------------- adjoint budget and bar
def _adjoint_inputs():
    from paper_2510_10529_amd import api
    wl, om, vf, rho_d, u, m = _small()
    nv = wl.n_occ + wl.n_buf
    X = _t(random_block(om.n_free, nv, 3))
    v = _t(vf + u)
    r = api.ks_eigensolve(m, v, X, wl.n_occ, 20, 1e-11, 300)
    k = wl.n_occ
    Psi = X[:, :k].contiguous()
    rho, B, loss = api.loss_grad(m, Psi, [2.0] * k, _t(rho_d))
    U = X[:, k:].contiguous()
    return m, v, Psi, r.eig[:k], B, U, r.eig[k:]


@pytest.mark.parametrize("deflated", [False, True])
def test_adjoint_euclidean_bar_and_budget(deflated):
    """Converged: every column meets ||b - A q|| <= 2 tol ||b||. With one iteration less than the
    converged solve used (first solve and refinement together), FE_ENOCONV, and no column ran
    more than maxit iterations."""
    from paper_2510_10529_amd import _lib, api
    m, v, Psi, eps, B, U, theta = _adjoint_inputs()
    kw = dict(U=U, theta=theta) if deflated else {}
    tol = 1e-10
    Q, ar = api.adjoint_solve(m, v, Psi, eps, B, tol=tol, maxit=20000, **kw)
    assert ar.status == _lib.FE_OK, ar
    assert max(ar.relres) <= 2 * tol, ar.relres
    total = max(ar.iters)
    Q2, ar2 = api.adjoint_solve(m, v, Psi, eps, B, tol=tol, maxit=total - 1, **kw)
    assert ar2.status == _lib.FE_ENOCONV, ar2
    assert max(ar2.iters) <= total - 1


@pytest.mark.parametrize("n", [0, 1, 2, 7, 1029, (1 << 20) + 3])
@pytest.mark.parametrize("offset", [0, 1])
def test_axpby_lengths_and_alignment(n, offset):
    """fe_axpby (y = alpha x + beta y) on 16-byte pieces where both arrays allow it, element by
    element otherwise: every length, odd tails and 8-byte-aligned views give the plain result and
    leave the neighbouring element alone. alpha and beta are powers of two, so the products are
    exact and the result is one rounding of the sum, with or without a fused multiply-add."""
    from paper_2510_10529_amd import api
    g = torch.Generator().manual_seed(n + offset)
    xb = torch.randn(n + 1, generator=g, dtype=torch.float64)
    yb = torch.randn(n + 1, generator=g, dtype=torch.float64)
    want = yb.clone()
    want[offset:offset + n] = 0.5 * xb[offset:offset + n] - 2.0 * yb[offset:offset + n]
    xd, yd = xb.to(DEV), yb.to(DEV)
    api.axpby(0.5, xd[offset:offset + n], -2.0, yd[offset:offset + n])
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), want.numpy())
