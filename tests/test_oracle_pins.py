"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test pins one part of the oracle to something other than itself: closed-form
integrals, textbook quadrature values, exact eigenvalues of the harmonic trap,
discrete identities, brute-force finite differences, and independent solvers.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from numpy.polynomial import chebyshev as npcheb

from oracle import chfsi, fe, ks
from synth import workload


# ------------------------------------------------------------------ P1 tables
@pytest.mark.parametrize("p", range(1, 9))
def test_gll_gauss_exactness(p):
    xi, w = fe.gll_nodes_weights(p)
    assert np.all(np.diff(xi) > 0)
    assert abs(w.sum() - 2.0) < 1e-14
    np.testing.assert_allclose(xi, -xi[::-1], atol=1e-15)
    for k in range(0, 2 * p):                    # GLL exact to degree 2p-1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14
    if p >= 1:                                    # and not beyond (degree 2p)
        assert abs(np.dot(w, xi ** (2 * p)) - 2.0 / (2 * p + 1)) > 1e-6
    xg, wg = fe.gauss_nodes_weights(p + 1)
    for k in range(0, 2 * p + 2):                # Gauss (p+1 points) exact to 2p+1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(wg, xg ** k) - exact) < 1e-14


def test_gll_textbook_values():
    # roots of P_p' by hand: P_2' = 3x; P_3' = (15x^2 - 3)/2; P_4' = (35x^3 - 15x)/2
    xi, w = fe.gll_nodes_weights(2)
    np.testing.assert_allclose(xi, [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    xi, w = fe.gll_nodes_weights(3)
    np.testing.assert_allclose(xi, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    xi, w = fe.gll_nodes_weights(4)
    np.testing.assert_allclose(xi, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


# ------------------------------------------------------------ P2 ref. matrices
@pytest.mark.parametrize("p", range(1, 9))
def test_reference_matrices_closed_form(p):
    Kh, Mh, xi, _ = fe.reference_matrices(p)
    np.testing.assert_allclose(Kh, Kh.T, atol=1e-13)
    np.testing.assert_allclose(Mh, Mh.T, atol=1e-15)
    np.testing.assert_allclose(Kh.sum(axis=1), 0.0, atol=1e-12)      # constants: zero energy
    assert abs(Mh.sum() - 2.0) < 1e-13
    for k in range(0, p + 1):
        q = xi ** k
        mass = 2.0 / (2 * k + 1)
        stiff = 0.0 if k == 0 else 2.0 * k * k / (2 * k - 1)
        assert abs(q @ Mh @ q - mass) < 1e-13 * max(1.0, mass)
        assert abs(q @ Kh @ q - stiff) < 1e-12 * max(1.0, stiff)
    # cross term: int (x^j)'(x^k)' for j=1, k=p (odd/even parity)
    if p >= 2:
        a, b = xi ** 1, xi ** 2
        assert abs(a @ Kh @ b) < 1e-13            # int 1 * 2x = 0


# ------------------------------------------------------- P3 3-D closed form
@pytest.mark.parametrize("p,n,L", [(2, 3, 3.0), (3, 2, 2.0), (4, 3, 1.5), (5, 2, 3.0)])
def test_kinetic_closed_form(p, n, L):
    """u = prod_d (L^2 - x_d^2) lies in Q_p (p >= 2) and vanishes on the boundary:
    u~^T (K~/2) u~ = (1/2) int |grad u|^2 = 1024 L^13 / 225 exactly."""
    m = fe.mesh3d(p, n, L)
    X = m.coords()
    W = m.weights()
    u = np.prod(L * L - X * X, axis=1)
    ut = np.sqrt(W) * u
    exact = 1024.0 * L ** 13 / 225.0
    assert abs(ut @ (fe.kinetic_csr(m) @ ut) / exact - 1) < 1e-12
    assert abs(ut @ fe.kinetic_apply(m, ut) / exact - 1) < 1e-12
    if p >= 3:   # GLL quadrature exact for the degree-4 integrand
        assert abs(np.sum(W * u * u) / (16.0 * L ** 5 / 15.0) ** 3 - 1) < 1e-12


def test_coordinates_and_weights():
    p, n, L = 4, 3, 2.5
    m = fe.mesh3d(p, n, L)
    # total GLL weight of the full box (with boundary nodes) is the volume
    m1 = m.m1
    assert abs(m1.W1.sum() + 2 * (m1.h / 2) * fe.gll_nodes_weights(p)[1][0] - 2 * L) < 1e-13
    X = m.coords()
    assert X.shape == (m.n_free, 3)
    # x fastest: consecutive indices step in x
    assert X[1, 0] > X[0, 0] and X[1, 1] == X[0, 1]
    assert np.all(np.abs(X) < L)
    # element vertices sit at -L + e h
    np.testing.assert_allclose(m1.x_all[::p], -L + m1.h * np.arange(n + 1), atol=1e-14)


# ----------------------------------------------------------- P4/P5 operators
def test_symmetry_and_two_applies_agree():
    wl = workload(2, p=4, n=3, half_width=4.0)
    m = fe.mesh3d(wl.p, wl.n, wl.half_width)
    v = wl.v_fixed(m.coords()) + wl.v_xc_target(m.coords())
    rng = np.random.default_rng(3)
    X = rng.standard_normal((m.n_free, 5))
    H = fe.hamiltonian_csr(m, v)
    assert abs(H - H.T).max() < 1e-12 * abs(H).max()
    Yk = fe.hamiltonian_apply(m, v, X)
    np.testing.assert_allclose(Yk, H @ X, rtol=0, atol=1e-13 * np.abs(Yk).max())
    x, y = X[:, 0], X[:, 1]
    assert abs(x @ fe.hamiltonian_apply(m, v, y) - y @ fe.hamiltonian_apply(m, v, x)) < 1e-12 * np.abs(Yk).max()
    np.testing.assert_allclose(fe.kinetic_diag(m), fe.kinetic_csr(m).diagonal(), rtol=1e-13)


@pytest.mark.parametrize("p,n,L", [(4, 3, 4.0), (5, 2, 3.0), (2, 4, 5.0)])
def test_sampled_rows_match_assembled_operator(p, n, L):
    """Row-by-row evaluation (used to check full-size runs on sampled nodes) against the
    assembled CSR operator and the Kronecker apply, on every row of small meshes."""
    wl = workload(2, p=p, n=n, half_width=L)
    m = fe.mesh3d(wl.p, wl.n, wl.half_width)
    v = wl.v_fixed(m.coords()) + wl.v_xc_target(m.coords())
    rng = np.random.default_rng(11)
    X = rng.standard_normal((m.n_free, 4))
    shift = rng.standard_normal(4)
    ref = fe.hamiltonian_csr(m, v) @ X - X * shift[None, :]
    rows = np.arange(m.n_free)
    got = fe.hamiltonian_rows(m, v, X, rows, shift=shift)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    got2 = fe.hamiltonian_rows(m, v, X, rows[::7])
    np.testing.assert_allclose(got2, fe.hamiltonian_apply(m, v, X)[::7], rtol=0, atol=1e-12 * np.abs(ref).max())


# ------------------------------------------------------------ P6 Fried bound
@pytest.mark.parametrize("p,h", [(5, 0.8), (4, 0.75), (2, 4.0 / 3.0)])
@pytest.mark.parametrize("n", [2, 3])
def test_fried_bound(p, h, n):
    m = fe.mesh3d(p, n, n * h / 2.0)
    lam = np.linalg.eigvalsh(fe.kinetic_csr(m).toarray()).max()
    b = fe.element_bound(p, h)
    assert lam <= b
    assert lam >= 0.7 * b       # and not vacuous


# --------------------------------------------------------- P7 harmonic trap
@pytest.mark.slow
def test_harmonic_oscillator_eigenvalues():
    """v = r^2/2: eigenvalues n + 3/2 with multiplicities 1, 3, ... (exact 3-fold
    degeneracy of the first excited shell on a cube-symmetric mesh)."""
    errs = []
    for p in (4, 5):
        m = fe.mesh3d(p, 6, 5.0)
        X = m.coords()
        fw = ks.forward(m, 0.5 * np.sum(X * X, axis=1), 8, tol=1e-11)
        e = fw.eps
        errs.append(max(abs(e[0] - 1.5), np.max(np.abs(e[1:4] - 2.5))))
        assert np.ptp(e[1:4]) < 1e-10
        assert e[4] > 3.4
    assert errs[1] < 2e-5            # Q5, h = 5/3
    assert errs[0] < 1e-3            # Q4
    assert errs[1] < errs[0] / 10    # p-convergence


# ----------------------------------------------- P8/P9 forward, count, RR
def _small_system(seed_cfg=2, p=2, n=3, L=4.0):
    wl = workload(seed_cfg, p=p, n=n, half_width=L)
    m = fe.mesh3d(wl.p, wl.n, wl.half_width)
    X = m.coords()
    return wl, m, wl.v_fixed(X), wl.v_xc_target(X)


def test_forward_orthonormal_and_count():
    wl, m, vf, vs = _small_system(p=4, n=3, L=5.0)
    v = vf + vs
    fd = ks.forward(m, v, wl.n_occ + 2, dense=True)
    fl = ks.forward(m, v, wl.n_occ + 2, dense=False, tol=1e-14)
    np.testing.assert_allclose(fd.eps, fl.eps, atol=1e-10)
    np.testing.assert_allclose(fd.psi.T @ fd.psi, np.eye(fd.psi.shape[1]), atol=1e-12)
    H = fe.hamiltonian_csr(m, v)
    R = H @ fd.psi - fd.psi * fd.eps[None, :]
    assert np.abs(R).max() < 1e-10
    occ = ks.occupations(wl.n_elec)
    rho = ks.density(fd.psi, occ, m.weights())
    assert abs(ks.electron_count(rho, m.weights()) - wl.n_elec) < 1e-12 * wl.n_elec
    assert np.all(rho >= 0)


def test_rayleigh_ritz_exact_subspace():
    wl, m, vf, vs = _small_system(p=3, n=3, L=4.0)
    v = vf + vs
    H = fe.hamiltonian_csr(m, v).toarray()
    e, V = np.linalg.eigh(H)
    rng = np.random.default_rng(1)
    Y = V[:, :6] @ rng.standard_normal((6, 6))          # a skewed basis of an invariant subspace
    w, Psi, res = chfsi.rayleigh_ritz(lambda Z: H @ Z, Y)
    np.testing.assert_allclose(w, e[:6], atol=1e-10)
    assert res.max() < 1e-9
    np.testing.assert_allclose(Psi.T @ Psi, np.eye(6), atol=1e-10)


# --------------------------------------------------------------- P10 filter
def test_chebyshev_T_matches_numpy():
    x = np.linspace(-3, 3, 61)
    for m in (0, 1, 2, 7, 12):
        c = np.zeros(m + 1)
        c[m] = 1
        np.testing.assert_allclose(chfsi.cheb_T(m, x), npcheb.chebval(x, c), rtol=1e-12, atol=1e-12)


def test_chebyshev_filter_on_eigenvectors():
    wl, m, vf, vs = _small_system(p=3, n=3, L=4.0)
    v = vf + vs
    H = fe.hamiltonian_csr(m, v).toarray()
    e, V = np.linalg.eigh(H)
    a, b, a0 = e[8], e[-1] * 1.01, e[0]
    deg = 9
    Y = chfsi.filter_apply(lambda Z: H @ Z, V[:, :12], deg, a, b, a0)
    expect = V[:, :12] * chfsi.filter_scalar(deg, a, b, a0, e[:12])[None, :]
    np.testing.assert_allclose(Y, expect, rtol=0, atol=1e-12 * np.abs(expect).max())
    # the wanted end is amplified, the damped interval stays below 1/T_m
    f = chfsi.filter_scalar(deg, a, b, a0, e)
    assert abs(f[0] - 1) < 1e-12 and np.all(np.abs(f[9:]) <= np.abs(f[8]) + 1e-15)


# --------------------------------------------------- P11/P12 adjoint, gradient
def _grad_setup():
    wl, m, vf, vs = _small_system(cfg := 2, p=2, n=3, L=4.0)
    rho_d, _ = ks.target_density(m, vf + vs, wl.n_elec)
    u = 0.5 * np.sin(m.coords()[:, 0]) + 0.05     # away from the target
    return wl, m, vf, vs, rho_d, u


def test_adjoint_three_solvers_agree():
    wl, m, vf, vs, rho_d, u = _grad_setup()
    v = vf + u
    occ = ks.occupations(wl.n_elec)
    H = fe.hamiltonian_csr(m, v)
    e, V = np.linalg.eigh(H.toarray())
    k = occ.size
    psi = V[:, :k]
    rho = ks.density(psi, occ, m.weights())
    R = 4.0 * (rho - rho_d)[:, None] * psi * occ[None, :]
    B = ks.adjoint_rhs(psi, occ, rho, rho_d)
    np.testing.assert_allclose(psi.T @ B, 0, atol=1e-13 * np.abs(B).max())
    Q1 = ks.adjoint_sum_over_states(e, V, k, R)
    Q2 = ks.adjoint_bordered(H, psi, e[:k], B)
    Q3 = ks.adjoint_cg(m, v, psi, e[:k], B)
    scale = np.abs(Q1).max()
    np.testing.assert_allclose(Q2, Q1, atol=1e-10 * scale)
    np.testing.assert_allclose(Q3, Q1, atol=1e-9 * scale)
    np.testing.assert_allclose(psi.T @ Q2, 0, atol=1e-12 * scale)
    # residual of the adjoint equation on the complement
    Hd = H.toarray()
    for i in range(k):
        r = (Hd - e[i] * np.eye(m.n_free)) @ Q2[:, i] - B[:, i]
        assert np.abs(r).max() < 1e-10 * np.abs(B).max()


def test_gradient_brute_force_fd_all_nodes():
    wl, m, vf, vs, rho_d, u = _grad_setup()
    ev = ks.evaluate(m, vf + u, rho_d, wl.n_elec, method="sos")
    # central differences with one Richardson step: O(h^4) truncation
    h = 2e-3
    fd = np.empty(m.n_free)
    for b in range(m.n_free):
        d = np.zeros(m.n_free)
        d[b] = 1.0
        d1 = ks.fd_directional(m, vf + u, rho_d, wl.n_elec, d, h)
        d2 = ks.fd_directional(m, vf + u, rho_d, wl.n_elec, d, h / 2)
        fd[b] = (4.0 * d2 - d1) / 3.0
    np.testing.assert_allclose(ev.grad, fd, rtol=0, atol=1e-8 * np.abs(fd).max())
    for meth in ("bordered", "cg"):
        ev2 = ks.evaluate(m, vf + u, rho_d, wl.n_elec, method=meth)
        np.testing.assert_allclose(ev2.grad, ev.grad, atol=1e-9 * np.abs(ev.grad).max())


def test_gradient_gauge_and_target():
    wl, m, vf, vs, rho_d, u = _grad_setup()
    ev = ks.evaluate(m, vf + u, rho_d, wl.n_elec, method="sos")
    # a constant shift of v leaves rho unchanged: sum_b g_b = 0
    assert abs(ev.grad.sum()) < 1e-12 * np.abs(ev.grad).sum()
    # at the known potential, L = 0 and g = 0
    ev0 = ks.evaluate(m, vf + vs, rho_d, wl.n_elec, method="sos")
    assert ev0.loss < 1e-25
    assert np.abs(ev0.grad).max() < 1e-12


def test_shift_covariance():
    wl, m, vf, vs, rho_d, u = _grad_setup()
    e1 = ks.evaluate(m, vf + u, rho_d, wl.n_elec, method="sos")
    e2 = ks.evaluate(m, vf + u + 0.37, rho_d, wl.n_elec, method="sos")
    np.testing.assert_allclose(e2.eps, e1.eps + 0.37, atol=1e-12)
    np.testing.assert_allclose(e2.rho, e1.rho, atol=1e-12)
    np.testing.assert_allclose(e2.grad, e1.grad, atol=1e-11 * np.abs(e1.grad).max())


def test_degenerate_rotation_invariance():
    """Harmonic trap: 4 occupied orbitals = 1 + exactly degenerate triplet.
    Rotating the triplet leaves rho, the adjoint RHS span and g unchanged (Sec. 2)."""
    m = fe.mesh3d(3, 2, 4.0)
    X = m.coords()
    v = 0.5 * np.sum(X * X, axis=1)
    rng = np.random.default_rng(5)
    rho_d = ks.density(ks.forward(m, v + 0.1 * np.exp(-np.sum((X - 0.3) ** 2, axis=1)), 4, dense=True).psi,
                       ks.occupations(8), m.weights())
    H = fe.hamiltonian_csr(m, v)
    e, V = np.linalg.eigh(H.toarray())
    assert np.ptp(e[1:4]) < 1e-12 and e[4] - e[3] > 0.1
    occ = ks.occupations(8)
    psi = V[:, :4]
    Qr, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    psi_r = psi.copy()
    psi_r[:, 1:4] = psi[:, 1:4] @ Qr
    out = []
    for P in (psi, psi_r):
        rho = ks.density(P, occ, m.weights())
        B = ks.adjoint_rhs(P, occ, rho, rho_d)
        Q = ks.adjoint_bordered(H, P, e[:4], B)
        out.append((rho, ks.gradient(P, Q)))
    np.testing.assert_allclose(out[1][0], out[0][0], atol=1e-13)
    np.testing.assert_allclose(out[1][1], out[0][1], atol=1e-10 * np.abs(out[0][1]).max())


def test_tau_bc_mask():
    g = np.array([1.0, 2.0, 3.0])
    rd = np.array([1e-3, 1e-8, 1.0])
    np.testing.assert_array_equal(ks.mask_gradient(g, rd, 1e-6), [1.0, 0.0, 3.0])
    np.testing.assert_array_equal(ks.mask_gradient(g, rd, 0.0), g)
