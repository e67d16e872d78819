"""Pins of the mapped-mesh oracle (per-cell dense element matrices; CPU only).

Each pin is fixed by something other than the oracle's own formulas:
  * with the identity map the mapped mesh is the uniform mesh, whose operator is pinned
    separately (closed-form energies, exact quadrature): the two agree to rounding;
  * on an affinely sheared box the field u = prod (L^2 - xi_d^2) of the reference
    coordinates has the closed-form energy |det A| tr(A^{-1} A^{-T}) (8 L^3/3)(16 L^5/15)^2,
    and the lumped mass sums to the sheared volume |det A| (2L)^3;
  * the patch test: on the smoothly warped mesh every linear field c . x + d is annihilated
    at every free node (its integral of grad N_a is a boundary term that vanishes), to
    rounding, because the stiffness quadrature integrates that polynomial exactly;
  * the harmonic trap v = r^2/2 on the warped mesh: eigenvalues converge to 3/2, 5/2 as the
    order rises (the PDE does not see the map);
  * Fried's element bound is above the largest eigenvalue.
Planted mistakes (an under-integrated stiffness, a transposed Jacobian in the metric, a
lumped mass without the volume factor) must fail a pin. (The shear's energy cannot see a
transposed Jacobian: only the trace of the metric enters it; the patch test does.)
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import fe, mapped


def _shear():
    return np.array([[1.0, 0.3, 0.0], [0.0, 1.0, -0.2], [0.1, 0.0, 0.9]])


def _sheared(p, n, L):
    A = _shear()
    return mapped.MappedMesh(p, n, L, lambda xi: xi @ A.T), A


@pytest.mark.parametrize("p,n", [(2, 3), (4, 2)])
def test_identity_map_is_the_uniform_mesh(p, n):
    L = 3.0
    m = mapped.mapped_mesh(p, n, L, 0.0)
    u = fe.mesh3d(p, n, L)
    K0 = fe.kinetic_csr(u).toarray()
    Km = m.kinetic_csr().toarray()
    assert np.abs(Km - K0).max() <= 1e-13 * np.abs(K0).max()
    assert np.allclose(m.weights(), u.weights(), rtol=1e-14, atol=0)
    assert np.allclose(m.coords(), u.coords(), rtol=0, atol=1e-14)


def _shear_energy_ratio(p=2, n=2, L=1.5):
    m, A = _sheared(p, n, L)
    ref = np.linalg.solve(A, m.coords().T).T            # reference coordinates of the free nodes
    u = np.prod(L * L - ref * ref, axis=1)
    E = u @ (m.K @ u)
    Ai = np.linalg.inv(A)
    exact = abs(np.linalg.det(A)) * np.trace(Ai @ Ai.T) * (8 * L ** 3 / 3) * (16 * L ** 5 / 15) ** 2
    return E / exact, m, A


@pytest.mark.parametrize("p", [2, 3])
def test_affine_shear_closed_form_energy_and_volume(p):
    r, m, A = _shear_energy_ratio(p=p)
    assert abs(r - 1.0) <= 1e-13
    assert abs(m.W_all.sum() / (abs(np.linalg.det(A)) * (2 * 1.5) ** 3) - 1.0) <= 1e-14


def _patch_residual(p, n=2, L=2.0, amp=0.2):
    m = mapped.mapped_mesh(p, n, L, amp)
    c = np.array([0.3, -1.1, 0.7])
    u = m.x_all @ c + 0.4
    r = (m.K_all @ u)[m.free_idx]
    return float(np.abs(r).max() / (np.abs(m.K_all).max() * np.abs(u).max()))


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_patch_test_linear_fields(p):
    assert _patch_residual(p) <= 1e-13


def test_operator_symmetric_positive_and_bounded():
    m = mapped.mapped_mesh(3, 2, 2.0, 0.2)
    H = m.kinetic_csr().toarray()
    assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()
    w = sla.eigvalsh(H)
    assert w[0] > 0
    b = m.element_bound()
    assert w[-1] <= b <= 2.0 * w[-1]


def _ho_errors(p, n=4, L=6.0, amp=0.15):
    m = mapped.mapped_mesh(p, n, L, amp)
    X = m.coords()
    H = fe.hamiltonian_csr(m, 0.5 * np.sum(X * X, axis=1))
    w = spla.eigsh(H, k=4, which="SA", tol=1e-12)[0]
    return np.sort(w) - np.array([1.5, 2.5, 2.5, 2.5])


@pytest.mark.slow
def test_harmonic_trap_converges_on_the_warped_mesh():
    """Cells of 3 bohr: the lowest level's error falls by about ten per order (measured
    2.0e-2, 1.6e-3 at p = 4, 5), the split triplet's from 4.9e-2 to 3.2e-3."""
    e4, e5 = (np.abs(_ho_errors(p)) for p in (4, 5))
    assert e5[0] < 0.2 * e4[0] and e5[1:].max() < 0.2 * e4[1:].max()
    assert e5[0] < 3e-3 and e5.max() < 5e-3


def test_mutation_under_integrated_stiffness_fails_the_patch_test(monkeypatch):
    monkeypatch.setattr(mapped, "quad_points", lambda p: p + 1)
    assert _patch_residual(4) > 1e-8


def test_mutation_transposed_jacobian_fails_the_pins(monkeypatch):
    orig = mapped.metric
    monkeypatch.setattr(mapped, "metric", lambda J: orig(np.swapaxes(J, -1, -2)))
    assert _patch_residual(3) > 1e-8


def test_mutation_mass_without_jacobian_fails_the_volume(monkeypatch):
    m_ok, A = _sheared(2, 2, 1.5)
    vol = abs(np.linalg.det(A)) * 3.0 ** 3
    assert abs(m_ok.W_all.sum() / vol - 1) < 1e-14
    monkeypatch.setattr(mapped, "node_volume", lambda J: np.ones(J.shape[:-2]))
    m_bad, _ = _sheared(2, 2, 1.5)
    assert abs(m_bad.W_all.sum() / vol - 1) > 1e-3


def test_gradient_on_the_warped_mesh_by_central_differences():
    """The chain (forward, density, loss, adjoint, gradient) needs nothing of the tensor
    structure: on a warped mesh the gradient matches central differences of the loss."""
    from oracle import ks
    from synth import workload
    wl = workload(2, p=2, n=3, half_width=4.0)
    m = mapped.mapped_mesh(2, 3, 4.0, 0.2)
    X = m.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    rho_d, _ = ks.target_density(m, vf + vs, wl.n_elec)
    u = 0.5 * np.sin(X[:, 0])
    ev = ks.evaluate(m, vf + u, rho_d, wl.n_elec, method="bordered")
    d = np.random.default_rng(3).standard_normal(m.n_free)
    fd = ks.fd_directional(m, vf + u, rho_d, wl.n_elec, d, 1e-4)
    assert abs(ev.grad @ d - fd) <= 1e-7 * abs(fd)
