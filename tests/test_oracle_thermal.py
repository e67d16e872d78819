"""Pins of the finite-temperature oracle (Eqs. 4, 5, 7-10) against what the
mathematics fixes independently of it (CPU only):

* the chemical potential in closed form for a symmetric pair and a single
  degenerate level;
* the zero-temperature limit, which must reproduce the pinned T -> 0 oracle;
* brute-force central differences of L(v) at every node, with mu solved anew
  at each potential;
* the Daleckii-Krein derivative of the matrix function f(H~) over the full
  spectrum, a route that solves no adjoint equation and forms no eta;
* an open shell on an exactly degenerate level: invariance of the gradient
  under rotations of the block, covariance of the adjoint functions;
* electron count, gauge (constant shift), and zero gradient at the target.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.special import expit

from oracle import fe, ks, thermal as th
from synth import workload


def _system(p=2, n=3, L=4.0, cfg=2):
    wl = workload(cfg, p=p, n=n, half_width=L)
    m = fe.mesh3d(p, n, L)
    X = m.coords()
    return wl, m, X, wl.v_fixed(X), wl.v_xc_target(X)


# --------------------------------------------------------- occupancy and mu
def test_chemical_potential_symmetric_pair():
    # f(0) + f(1) = 2 exactly when mu = 1/2: s phi(-x) + s phi(x) = s. (At kT << 1 the sum is
    # flat to the last bit across the gap, so only temperatures where it moves are asked.)
    for kT in (0.1, 0.3, 2.0):
        mu = th.chemical_potential(np.array([0.0, 1.0]), 2.0, kT)
        assert abs(mu - 0.5) <= 4e-16


def test_chemical_potential_degenerate_level():
    # one g-fold level holding N_e electrons: f = N_e / g, mu = eps + kT ln(f / (s - f))
    eps = np.full(6, -0.7)
    for ne, s in ((2.0, 2.0), (5.0, 2.0), (1.0, 1.0)):
        kT = 0.02
        mu = th.chemical_potential(eps, ne, kT, s)
        f = ne / eps.size
        assert abs(mu - (-0.7 + kT * np.log(f / (s - f)))) < 1e-14
        np.testing.assert_allclose(th.occupancy(eps, mu, kT, s), f, rtol=1e-14)
    with pytest.raises(ValueError):
        th.chemical_potential(eps, 12.0, 0.02, 2.0)


def test_occupancy_derivative():
    e = np.linspace(-1, 1, 41)
    for kT in (0.01, 0.1):
        def cd(h):
            return (th.occupancy(e + h, 0.1, kT) - th.occupancy(e - h, 0.1, kT)) / (2 * h)
        h = 1e-3 * kT
        fd = (4.0 * cd(h / 2) - cd(h)) / 3.0       # Richardson: O(h^4) truncation
        np.testing.assert_allclose(th.occupancy_deps(e, 0.1, kT), fd, rtol=1e-9, atol=1e-9 / kT)


def test_electron_count():
    wl, m, X, vf, vs = _system()
    eps, psi, mu, occ = th.states(m, vf + vs, wl.n_elec, 0.05)
    rho = ks.density(psi, occ, m.weights())
    assert abs(ks.electron_count(rho, m.weights()) - wl.n_elec) < 1e-12 * wl.n_elec
    assert abs(occ.sum() - wl.n_elec) < 1e-12 * wl.n_elec


# --------------------------------------------------------------- gradient
def _setup(kT, cfg=2):
    wl, m, X, vf, vs = _system(cfg=cfg)
    rho_d = th.target_density(m, vf + vs, wl.n_elec, kT)
    u = 0.5 * np.sin(X[:, 0]) + 0.05
    return wl, m, vf, vs, rho_d, u


def test_zero_temperature_limit():
    """Gap ~0.65 Ha at the Fermi level, kT = 2e-3: occupations are 0/2 to e^-160."""
    wl, m, X, vf, vs = _system()
    rho_d, _ = ks.target_density(m, vf + vs, wl.n_elec)
    u = 0.5 * np.sin(X[:, 0]) + 0.05
    g0 = ks.evaluate(m, vf + u, rho_d, wl.n_elec, method="sos").grad
    g1 = th.evaluate(m, vf + u, rho_d, wl.n_elec, 2e-3).grad
    np.testing.assert_allclose(g1, g0, rtol=0, atol=1e-12 * np.abs(g0).max())


@pytest.mark.parametrize("kT", [0.02, 0.1])
def test_gradient_brute_force_fd_all_nodes(kT):
    wl, m, vf, vs, rho_d, u = _setup(kT)
    ev = th.evaluate(m, vf + u, rho_d, wl.n_elec, kT)
    h = 2e-3
    fd = np.empty(m.n_free)
    for b in range(m.n_free):
        d = np.zeros(m.n_free)
        d[b] = 1.0
        d1 = th.fd_directional(m, vf + u, rho_d, wl.n_elec, kT, d, h)
        d2 = th.fd_directional(m, vf + u, rho_d, wl.n_elec, kT, d, h / 2)
        fd[b] = (4.0 * d2 - d1) / 3.0           # Richardson: O(h^4) truncation
    np.testing.assert_allclose(ev.grad, fd, rtol=0, atol=1e-8 * np.abs(fd).max())


@pytest.mark.parametrize("kT,smax", [(0.05, 2.0), (0.2, 2.0), (0.05, 1.0)])
def test_gradient_matches_daleckii_krein(kT, smax):
    """dL = sum_a G_a d[f(H~)]_aa with G = -2 (rho_d - rho), and, over the full spectrum,
    d f(H~) = Psi (F o Psi^T dH Psi) Psi^T - dmu Psi diag(f') Psi^T, F_ij = (f_i - f_j)/(e_i - e_j)
    (F_ii = f'_i), dmu = sum f'_i de_i / sum f'_i fixed by the electron count."""
    wl, m, X, vf, vs = _system()
    ne = wl.n_elec if smax == 2.0 else wl.n_elec // 2
    rho_d = th.target_density(m, vf + vs, ne, kT, smax=smax)
    v = vf + 0.5 * np.sin(X[:, 0]) + 0.05
    ev = th.evaluate(m, v, rho_d, ne, kT, smax=smax)
    e, V = sla.eigh(fe.hamiltonian_csr(m, v).toarray())
    mu = th.chemical_potential(e, ne, kT, smax)
    phi = expit(-(e - mu) / kT)
    f, fp = smax * phi, -smax * phi * (1 - phi) / kT
    rho = (V ** 2 @ f) / m.weights()
    G = -2.0 * (rho_d - rho)
    M = V.T @ (G[:, None] * V)
    de = e[:, None] - e[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        F = np.where(np.abs(de) > 1e-9, (f[:, None] - f[None, :]) / de, 0.5 * (fp[:, None] + fp[None, :]))
    g = np.einsum("bi,ij,bj->b", V, F * M, V) - (fp @ np.diag(M)) / fp.sum() * (V ** 2 @ fp)
    np.testing.assert_allclose(ev.grad, g, rtol=0, atol=1e-10 * np.abs(g).max())


def test_adjoint_equations_hold():
    """Every block: (H~ - eps_k) P_k equals Eq. 7's right-hand side, Psi_k^T P_k equals Eq. 8's."""
    kT = 0.05
    wl, m, vf, vs, rho_d, u = _setup(kT)
    v = vf + u
    ev = th.evaluate(m, v, rho_d, wl.n_elec, kT)
    H = fe.hamiltonian_csr(m, v)
    delta = rho_d - ev.rho
    for b in th.degenerate_blocks(ev.eps):
        ek = ev.eps[b].mean()
        fk = th.occupancy(ek, ev.mu, kT)
        dk = th.occupancy_deps(ek, ev.mu, kT)
        Pk, Sk = ev.P[:, b], ev.psi[:, b]
        S = Sk.T @ (delta[:, None] * Sk)
        rhs = 4.0 * fk * delta[:, None] * Sk - Sk @ (4.0 * fk * S)
        res = H @ Pk - ek * Pk - rhs
        assert np.abs(res).max() < 1e-9 * np.abs(rhs).max()
        np.testing.assert_allclose(Sk.T @ Pk, dk * (-2.0 * S + ev.eta * np.eye(b.size)),
                                   atol=1e-11 * np.abs(Pk).max())


def test_gauge_and_target():
    kT = 0.05
    wl, m, vf, vs, rho_d, u = _setup(kT)
    e1 = th.evaluate(m, vf + u, rho_d, wl.n_elec, kT)
    e2 = th.evaluate(m, vf + u + 0.37, rho_d, wl.n_elec, kT)
    assert abs(e2.mu - e1.mu - 0.37) < 1e-12
    np.testing.assert_allclose(e2.rho, e1.rho, atol=1e-12)
    np.testing.assert_allclose(e2.grad, e1.grad, atol=1e-10 * np.abs(e1.grad).max())
    assert abs(e1.grad.sum()) < 1e-11 * np.abs(e1.grad).sum()
    e0 = th.evaluate(m, vf + vs, rho_d, wl.n_elec, kT)
    assert e0.loss < 1e-25 and np.abs(e0.grad).max() < 1e-12


def test_lanczos_states_match_full_spectrum():
    kT = 0.02
    wl, m, X, vf, vs = _system(p=4, n=3, L=5.0)
    rho_d = th.target_density(m, vf + vs, wl.n_elec, kT)
    v = vf + 0.5 * np.sin(X[:, 0]) + 0.05
    full = th.evaluate(m, v, rho_d, wl.n_elec, kT)
    lz = th.evaluate(m, v, rho_d, wl.n_elec, kT, n_states=full.eps.size + 4)
    assert lz.eps.size == full.eps.size
    np.testing.assert_allclose(lz.grad, full.grad, atol=1e-9 * np.abs(full.grad).max())


# -------------------------------------------------- degenerate open shell
def _open_shell():
    """Harmonic trap on a symmetric mesh: 1 + exactly degenerate triplet. Four electrons put
    two in the triplet (f = 2/3 each at low T): an ensemble density, not a single determinant."""
    m = fe.mesh3d(3, 2, 4.0)
    X = m.coords()
    v = 0.5 * np.sum(X * X, axis=1)
    kT = 0.01
    vt = v + 0.1 * np.exp(-np.sum((X - 0.3) ** 2, axis=1))
    rho_d = th.target_density(m, vt, 4.0, kT)
    return m, X, v, kT, rho_d


def test_open_shell_fd_and_rotation_invariance():
    m, X, v, kT, rho_d = _open_shell()
    ev = th.evaluate(m, v, rho_d, 4.0, kT)
    assert ev.eps.size == 4 and np.ptp(ev.eps[1:4]) < 1e-12       # the next shell is ~1 Ha up: empty
    np.testing.assert_allclose(ev.occ[1:4], 2.0 / 3.0, rtol=1e-12)
    rng = np.random.default_rng(7)
    for _ in range(3):
        d = rng.standard_normal(m.n_free)
        d1 = th.fd_directional(m, v, rho_d, 4.0, kT, d, 2e-4)   # h << kT
        d2 = th.fd_directional(m, v, rho_d, 4.0, kT, d, 1e-4)
        fd = (4 * d2 - d1) / 3
        assert abs(ev.grad @ d - fd) < 1e-7 * abs(fd)
    # a rotated block gives the same gradient and rotated adjoint functions
    Qr, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    psi_r = ev.psi.copy()
    psi_r[:, 1:4] = ev.psi[:, 1:4] @ Qr
    H = fe.hamiltonian_csr(m, v)
    P_r, eta_r = th.adjoint(H, psi_r, ev.eps, kT, ev.mu, ev.rho, rho_d)
    np.testing.assert_allclose(P_r[:, 1:4], ev.P[:, 1:4] @ Qr, atol=1e-10 * np.abs(ev.P).max())
    np.testing.assert_allclose(th.gradient(psi_r, P_r), ev.grad, atol=1e-11 * np.abs(ev.grad).max())
    assert abs(eta_r - ev.eta) < 1e-12 * abs(ev.eta)
