"""GPU parity of blocks wider than 64 columns (needs an MI355X): 80 occupied orbitals in a
96-column block on a small mesh. Rayleigh-Ritz and the eigensolve rotate in 64 x 64 tiles, the
projection works in 64-column groups, and the adjoint solves its 80 shifts in two groups
against all 80 orbitals (the first 64 inside the fused MINRES sweeps, the other 16 by separate
projection sweeps). Every result is checked against the oracle on the same inputs."""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import chfsi, fe, ks  # noqa: E402
from synth import random_block  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
P, NCELL, HALF = 4, 4, 6.0      # 3375 free nodes
NOCC, NV = 80, 96


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _potential(xyz):
    """A smooth potential without symmetry: a shallow well plus seeded Gaussian bumps and dips,
    so that no two of the lowest eigenvalues are degenerate."""
    rng = np.random.default_rng(80)
    r2 = np.sum(xyz ** 2, axis=1)
    v = 0.02 * r2 - 1.0
    for _ in range(12):
        c = rng.uniform(-4.0, 4.0, 3)
        a = rng.uniform(-1.5, 1.0)
        s = rng.uniform(0.8, 2.0)
        v += a * np.exp(-np.sum((xyz - c) ** 2, axis=1) / (2 * s * s))
    return v


@functools.lru_cache(maxsize=None)
def _oracle():
    """The whole spectrum of H~ on the small mesh (dense), the 80-orbital density and a target
    density; ev.eps and ev.psi hold every eigenpair."""
    om = fe.mesh3d(P, NCELL, HALF)
    v = _potential(om.coords())
    ev = ks.forward(om, v, om.n_free, dense=True)
    occ = np.full(NOCC, 2.0)
    W = om.weights()
    psi = ev.psi[:, :NOCC]
    rho = ks.density(psi, occ, W)
    # target density of a perturbed potential, so that the loss and B are not zero
    vd = v + 0.05 * np.sin(om.coords()[:, 0])
    evd = ks.forward(om, vd, NOCC, dense=True)
    rho_d = ks.density(evd.psi, occ, W)
    return om, v, ev, occ, psi, rho, rho_d


@functools.lru_cache(maxsize=None)
def _mesh():
    from paper_2510_10529_amd import api
    return api.Mesh(P, NCELL, HALF)


def test_oracle_gap_at_80():
    """Precondition of the cases below: the 80th and 81st eigenvalues are apart."""
    _, _, ev, *_ = _oracle()
    assert ev.eps[NOCC] - ev.eps[NOCC - 1] > 1e-3
    assert np.min(np.diff(ev.eps[:NV])) > 1e-6


def test_rayleigh_ritz_96_columns():
    from paper_2510_10529_amd import api
    om, v, *_ = _oracle()
    m = _mesh()
    Y = random_block(om.n_free, NV, 96)
    X = _t(Y)
    eig, res = api.rayleigh_ritz(m, _t(v), X)
    w, Psi, R = chfsi.rayleigh_ritz(lambda Z: fe.hamiltonian_apply(om, v, Z), Y)
    np.testing.assert_allclose(eig, w, rtol=0, atol=1e-10 * np.abs(w).max())
    np.testing.assert_allclose(res, R, rtol=1e-8, atol=1e-10 * np.abs(R).max())
    # Ritz vectors up to sign, and orthonormal
    Xn = X.cpu().numpy()
    sgn = np.sign(np.sum(Xn * Psi, axis=0))
    np.testing.assert_allclose(Xn * sgn[None, :], Psi, rtol=0, atol=1e-8)
    np.testing.assert_allclose(Xn.T @ Xn, np.eye(NV), rtol=0, atol=1e-12)


def test_rayleigh_ritz_96_columns_with_row_pitch():
    """The wide rotation goes through a second block; padding columns stay untouched."""
    from paper_2510_10529_amd import api
    om, v, *_ = _oracle()
    m = _mesh()
    Y = random_block(om.n_free, NV, 97)
    Xa = _t(Y)
    ea, ra = api.rayleigh_ritz(m, _t(v), Xa)
    Xb = torch.full((om.n_free, NV + 8), float("nan"), dtype=torch.float64, device=DEV)
    Xb[:, :NV] = _t(Y)
    eb, rb = api.rayleigh_ritz(m, _t(v), Xb, nv=NV)
    np.testing.assert_allclose(eb, ea, rtol=0, atol=1e-12 * max(abs(x) for x in ea))
    np.testing.assert_allclose(Xb[:, :NV].cpu().numpy(), Xa.cpu().numpy(), rtol=0, atol=1e-10)
    assert torch.isnan(Xb[:, NV:]).all()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_eigensolve_80_of_96(prec):
    from paper_2510_10529_amd import api
    om, v, ev, *_ = _oracle()
    m = _mesh()
    X = _t(random_block(om.n_free, NV, 80))
    r = api.ks_eigensolve(m, _t(v), X, NOCC, 20, 1e-10, 400, prec=prec, switch_tol=1e-4)
    assert r.status == 0, r
    assert max(r.res[:NOCC]) <= 1e-10
    np.testing.assert_allclose(r.eig[:NOCC], ev.eps[:NOCC], rtol=0, atol=1e-8)
    Xn = X.cpu().numpy()[:, :NOCC]
    # the occupied subspace: projector distance to the oracle's
    Po = ev.psi[:, :NOCC]
    assert np.linalg.norm(Xn @ (Xn.T @ Po) - Po) <= 1e-6


def test_loss_grad_80_orbitals():
    """rho, L and B = -(I - Psi Psi^T) R element by element; B's projection runs in two groups."""
    from paper_2510_10529_amd import api
    om, v, ev, occ, psi, rho, rho_d = _oracle()
    m = _mesh()
    r, B, loss = api.loss_grad(m, _t(psi), list(occ), _t(rho_d))
    W = om.weights()
    np.testing.assert_allclose(r.cpu().numpy(), rho, rtol=1e-13, atol=1e-16)
    Bref = ks.adjoint_rhs(psi, occ, rho, rho_d)
    np.testing.assert_allclose(B.cpu().numpy(), Bref, rtol=0, atol=1e-12 * np.abs(Bref).max())
    assert abs(loss - ks.loss(rho, rho_d, W)) <= 1e-12 * loss
    np.testing.assert_allclose(psi.T @ B.cpu().numpy(), 0, atol=1e-12 * np.abs(Bref).max())


def test_adjoint_80_shifts_in_two_groups():
    """(H~ - eps_i) q_i = b_i with Psi^T q_i = 0 for 80 shifts against 80 orbitals, against the
    oracle's sum over all unoccupied states (exact here: the whole spectrum is known): the
    solution, its orthogonality, the true residual of every column and the gradient."""
    from paper_2510_10529_amd import api
    om, v, ev, occ, psi, rho, rho_d = _oracle()
    m = _mesh()
    eps = ev.eps[:NOCC]
    Bref = ks.adjoint_rhs(psi, occ, rho, rho_d)
    H = fe.hamiltonian_csr(om, v)
    Rr = 4.0 * (rho - rho_d)[:, None] * psi * occ[None, :]
    Qref = ks.adjoint_sum_over_states(ev.eps, ev.psi, NOCC, Rr)
    Psi = _t(psi)
    Q, ar = api.adjoint_solve(m, _t(v), Psi, list(eps), _t(Bref), tol=1e-12, maxit=6000)
    assert ar.status == 0, ar
    assert len(ar.iters) == NOCC and min(ar.iters) >= 1
    assert max(ar.relres) <= 2e-12, max(ar.relres)
    Qn = Q.cpu().numpy()
    np.testing.assert_allclose(psi.T @ Qn, 0, atol=1e-10 * np.abs(Qn).max())
    # true residual on the host, column by column
    R = Bref - (H @ Qn - Qn * eps[None, :])
    R -= psi @ (psi.T @ R)
    rel = np.linalg.norm(R, axis=0) / np.linalg.norm(Bref, axis=0)
    assert rel.max() <= 3e-12, rel.max()
    err = np.linalg.norm(Qn - Qref, axis=0) / np.linalg.norm(Qref, axis=0)
    assert err.max() <= 1e-8, err.max()
    g = api.loss_grad(m, Psi, list(occ), _t(rho_d), Q=Q).cpu().numpy()
    gref = ks.gradient(psi, Qref)
    assert np.linalg.norm(g - gref) <= 1e-9 * np.linalg.norm(gref)


def test_adjoint_groups_match_64_column_solves():
    """Reversing the column order puts every shift in another group and another position (the
    last 16 columns first): the same systems, so the same solutions to the solve tolerance."""
    from paper_2510_10529_amd import api
    om, v, ev, occ, psi, rho, rho_d = _oracle()
    m = _mesh()
    eps = ev.eps[:NOCC]
    Bref = ks.adjoint_rhs(psi, occ, rho, rho_d)
    Psi = _t(psi)
    Q, ar = api.adjoint_solve(m, _t(v), Psi, list(eps), _t(Bref), tol=1e-12, maxit=6000)
    # reversed column order: other groups, same systems
    perm = np.arange(NOCC)[::-1].copy()
    Q2, ar2 = api.adjoint_solve(m, _t(v), Psi, list(eps[perm]), _t(Bref[:, perm]), tol=1e-12, maxit=6000)
    assert ar.status == 0 and ar2.status == 0
    Qa, Qb = Q.cpu().numpy(), Q2.cpu().numpy()[:, np.argsort(perm)]
    d = np.linalg.norm(Qa - Qb, axis=0) / np.linalg.norm(Qa, axis=0)
    assert d.max() <= 1e-9, d.max()


def test_adjoint_along_psi_80_orbitals():
    """Finite temperature with 80 included orbitals: the in-span part Q <- Q + Psi C (a tiled
    accumulating rotation) and C from M = 2 Psi^T diag(rho - rho_d) Psi, with the oracle's Fermi
    occupancies: C_ij = (f_i - f_j) / (eps_i - eps_j) M_ij off the diagonal and
    C_ii = f'_i (M_ii - etabar), etabar = sum f'_i M_ii / sum f'_i."""
    from oracle import thermal as th
    from paper_2510_10529_amd import api
    om, v, ev, occ, psi, rho, rho_d = _oracle()
    m = _mesh()
    eps = ev.eps[:NOCC]
    kT, ne = 0.01, 150.0
    mu = th.chemical_potential(ev.eps[:NV], ne, kT)
    f = th.occupancy(eps, mu, kT)
    fp = th.occupancy_deps(eps, mu, kT)
    rho_t = ks.density(psi, f, om.weights())
    Q0 = random_block(om.n_free, NOCC, 81)
    Q = _t(Q0)
    eta, C = api.adjoint_along_psi(m, _t(psi), list(eps), mu, kT, _t(rho_t), _t(rho_d), Q)
    C = np.array(C).reshape(NOCC, NOCC)
    np.testing.assert_allclose(Q.cpu().numpy() - Q0, psi @ C, rtol=0, atol=1e-12 * max(1.0, np.abs(psi @ C).max()))
    M = 2.0 * psi.T @ ((rho_t - rho_d)[:, None] * psi)
    de = eps[:, None] - eps[None, :]
    off = ~np.eye(NOCC, dtype=bool) & (np.abs(de) > 1e-3)
    dd = (f[:, None] - f[None, :]) / np.where(off, de, 1.0)
    scale = np.abs(C).max()
    np.testing.assert_allclose(C[off], (dd * M)[off], rtol=0, atol=1e-9 * scale)
    etabar = np.sum(fp * np.diag(M)) / np.sum(fp)
    np.testing.assert_allclose(np.diag(C), fp * (np.diag(M) - etabar), rtol=0, atol=1e-9 * scale)


@pytest.mark.parametrize("nv", [100, 131])
def test_uniform_apply_wide_blocks(nv):
    """The sum-factorised apply over 13 and 17 column chunks (FP64 8-column chunks, FP32 16),
    with per-column shifts, against the oracle's Kronecker apply."""
    from paper_2510_10529_amd import api
    om, v, *_ = _oracle()
    m = _mesh()
    X = random_block(om.n_free, nv, nv)
    shift = np.linspace(-1.0, 2.0, nv)
    ref = fe.hamiltonian_apply(om, v, X) - X * shift[None, :]
    Y = api.ks_apply(m, _t(v), _t(X), shift=list(shift)).cpu().numpy()
    scale = np.abs(ref).max()
    np.testing.assert_allclose(Y, ref, rtol=0, atol=2e-14 * scale * (P + 1))
    X32 = X.astype(np.float32)
    ref32 = fe.hamiltonian_apply(om, v, X32.astype(np.float64))
    Y32 = api.ks_apply(m, _t(v), torch.tensor(X32, device=DEV), prec="f32").cpu().numpy().astype(np.float64)
    assert np.abs(Y32 - ref32).max() <= 2e-5 * np.abs(ref32).max()


@pytest.mark.parametrize("nv", [70, 130])
def test_mapped_apply_wide_blocks(nv):
    """The mapped mesh's cell products stream the matrices once per 64 columns: 2 and 3 passes."""
    from oracle import mapped
    from paper_2510_10529_amd import api
    m = api.Mesh(3, 3, 3.0, mapped_amp=0.2)
    om = mapped.mapped_mesh(3, 3, 3.0, 0.2)
    X = random_block(om.n_free, nv, 7 * nv)
    v = np.random.default_rng(nv).uniform(-2, 2, om.n_free)
    shift = np.linspace(-1.0, 1.0, nv)
    ref = fe.hamiltonian_csr(om, v) @ X - X * shift[None, :]
    Y = api.ks_apply(m, torch.tensor(v, device=DEV), torch.tensor(X, device=DEV), shift=shift)
    err = np.abs(Y.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-13, err


def test_deflated_split_beyond_64_columns():
    """50 shifts deflated with 30 vectors: V = [Psi U] has 80 columns, so the fused sweeps take
    the first 64 and the last 16 deflation vectors go through their own Gram and update sweeps.
    Same system, so the same solution as the oracle's; fewer iterations than with 14 vectors
    (which fit the fused block)."""
    from paper_2510_10529_amd import api
    om, v, ev, occ, psi, rho, rho_d = _oracle()
    m = _mesh()
    k, nb = 50, 30
    W = om.weights()
    occ50 = np.full(k, 2.0)
    psi50 = ev.psi[:, :k]
    eps = ev.eps[:k]
    rho50 = ks.density(psi50, occ50, W)
    B = ks.adjoint_rhs(psi50, occ50, rho50, rho_d)
    Rr = 4.0 * (rho50 - rho_d)[:, None] * psi50 * occ50[None, :]
    Qref = ks.adjoint_sum_over_states(ev.eps, ev.psi, k, Rr)
    Psi = _t(psi50)
    res = {}
    for n in (14, nb):
        Q, ar = api.adjoint_solve(m, _t(v), Psi, list(eps), _t(B), tol=1e-12, maxit=6000,
                                  U=_t(ev.psi[:, k:k + n]), theta=list(ev.eps[k:k + n]))
        assert ar.status == 0, (n, ar)
        assert max(ar.relres) <= 2e-12, (n, max(ar.relres))
        Qn = Q.cpu().numpy()
        np.testing.assert_allclose(psi50.T @ Qn, 0, atol=1e-10 * np.abs(Qn).max())
        err = np.linalg.norm(Qn - Qref, axis=0) / np.linalg.norm(Qref, axis=0)
        assert err.max() <= 1e-8, (n, err.max())
        res[n] = max(ar.iters)
    assert res[nb] < res[14], res


def test_wide_refusals():
    """FP32-inner adjoint solves and deflation keep their 64-orbital limits."""
    from paper_2510_10529_amd import _lib, api
    om, v, ev, occ, psi, rho, rho_d = _oracle()
    m = _mesh()
    B = _t(ks.adjoint_rhs(psi, occ, rho, rho_d))
    with pytest.raises(_lib.FEError) as e:
        api.adjoint_solve(m, _t(v), _t(psi), list(ev.eps[:NOCC]), B, prec="f32")
    assert e.value.status == _lib.FE_EINVAL
    with pytest.raises(_lib.FEError) as e:
        api.adjoint_solve(m, _t(v), _t(psi), list(ev.eps[:NOCC]), B, U=_t(ev.psi[:, NOCC:NOCC + 8]),
                          theta=list(ev.eps[NOCC:NOCC + 8]))
    assert e.value.status == _lib.FE_EINVAL       # more than 64 orbitals with deflation
