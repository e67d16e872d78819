"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case patches one plausible slip into the oracle (a dropped factor, a
transposed Kronecker factor, a flipped sign, a missing weight) and checks that
the pin meant for it fails. This guards the pins themselves.
"""
import numpy as np
import pytest

from oracle import fe, ks
from synth import workload


def _kinetic_energy_ratio(p=3, n=2, L=2.0):
    m = fe.mesh3d(p, n, L)
    X = m.coords()
    u = np.prod(L * L - X * X, axis=1)
    ut = np.sqrt(m.weights()) * u
    return ut @ fe.kinetic_apply(m, ut) / (1024.0 * L ** 13 / 225.0)


def test_pin_catches_dropped_half(monkeypatch):
    assert abs(_kinetic_energy_ratio() - 1) < 1e-12
    orig = fe.kinetic_apply
    monkeypatch.setattr(fe, "kinetic_apply", lambda m, X: 2.0 * orig(m, X))
    assert abs(_kinetic_energy_ratio() - 1) > 0.5


def test_pin_catches_transposed_factor(monkeypatch):
    """One term with its stiffness factor on y instead of x."""
    def bad(mesh, X):
        m = mesh.m1
        n1 = mesh.n1
        s = 1.0 / np.sqrt(m.W1)
        Ks = s[:, None] * m.K1 * s[None, :]
        Ms = s[:, None] * m.Mc * s[None, :]
        T = X.reshape(n1, n1, n1, -1)
        t1 = fe._along(Ms, fe._along(Ks, fe._along(Ms, T, 2), 1), 0)   # slip: was x
        t2 = fe._along(Ms, fe._along(Ks, fe._along(Ms, T, 2), 1), 0)
        t3 = fe._along(Ks, fe._along(Ms, fe._along(Ms, T, 2), 1), 0)
        return (0.5 * (t1 + t2 + t3)).reshape(X.shape)

    m = fe.mesh3d(3, 2, 2.0)
    X = np.random.default_rng(0).standard_normal((m.n_free, 2))
    good = fe.kinetic_csr(m) @ X
    assert np.abs(fe.kinetic_apply(m, X) - good).max() < 1e-12 * np.abs(good).max()
    assert np.abs(bad(m, X) - good).max() > 1e-3 * np.abs(good).max()


def _grad_fd_mismatch():
    wl = workload(2, p=2, n=3, half_width=4.0)
    m = fe.mesh3d(2, 3, 4.0)
    X = m.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    rho_d, _ = ks.target_density(m, vf + vs, wl.n_elec)
    u = 0.5 * np.sin(X[:, 0])
    ev = ks.evaluate(m, vf + u, rho_d, wl.n_elec, method="bordered")
    d = np.random.default_rng(1).standard_normal(m.n_free)
    fd = ks.fd_directional(m, vf + u, rho_d, wl.n_elec, d, 1e-4)
    return abs(ev.grad @ d - fd) / abs(fd)


def test_pin_catches_adjoint_sign(monkeypatch):
    assert _grad_fd_mismatch() < 1e-6
    orig = ks.adjoint_rhs
    monkeypatch.setattr(ks, "adjoint_rhs", lambda *a: -orig(*a))
    assert _grad_fd_mismatch() > 0.5


def test_pin_catches_missing_weight(monkeypatch):
    wl = workload(2, p=3, n=2, half_width=4.0)
    m = fe.mesh3d(3, 2, 4.0)
    X = m.coords()
    fw = ks.forward(m, wl.v_fixed(X), wl.n_occ, dense=True)
    occ = ks.occupations(wl.n_elec)
    W = m.weights()
    assert abs(ks.electron_count(ks.density(fw.psi, occ, W), W) - wl.n_elec) < 1e-12
    monkeypatch.setattr(ks, "density", lambda psi, occ, W: psi[:, :occ.size] ** 2 @ occ)
    assert abs(ks.electron_count(ks.density(fw.psi, occ, W), W) - wl.n_elec) > 1e-3


# ------------------------------------------------ finite temperature (Eqs. 7-9)
def _thermal_fd_mismatch(kT=0.05):
    from oracle import thermal as th
    wl = workload(2, p=2, n=3, half_width=4.0)
    m = fe.mesh3d(2, 3, 4.0)
    X = m.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    rho_d = th.target_density(m, vf + vs, wl.n_elec, kT)
    v = vf + 0.5 * np.sin(X[:, 0]) + 0.05
    ev = th.evaluate(m, v, rho_d, wl.n_elec, kT)
    d = np.random.default_rng(3).standard_normal(m.n_free)
    fd = th.fd_directional(m, v, rho_d, wl.n_elec, kT, d, 1e-4)
    return abs(ev.grad @ d - fd) / abs(fd)


def test_thermal_pin_catches_dropped_eta(monkeypatch):
    from oracle import thermal as th
    assert _thermal_fd_mismatch() < 1e-5
    monkeypatch.setattr(th, "eta", lambda *a: 0.0)
    assert _thermal_fd_mismatch() > 1e-3


def test_thermal_pin_catches_dropped_overlap_term(monkeypatch):
    """P_k without its component along Psi_k (Eq. 8), as at zero temperature."""
    from oracle import thermal as th
    monkeypatch.setattr(th, "overlap", lambda S, dfde, et: np.zeros_like(S))
    assert _thermal_fd_mismatch() > 1e-3


def test_thermal_pin_catches_wrong_sign_in_overlap(monkeypatch):
    from oracle import thermal as th
    monkeypatch.setattr(th, "overlap", lambda S, dfde, et: dfde * (2.0 * S + et * np.eye(S.shape[0])))
    assert _thermal_fd_mismatch() > 1e-3


def test_thermal_check_catches_wrong_multiplier(monkeypatch):
    """A slip in D_k + D_k^T leaves Eq. 7's right-hand side with a component along its
    block; the oracle refuses it rather than letting the bordered solve hide it."""
    from oracle import thermal as th
    monkeypatch.setattr(th, "d_plus_dt", lambda S, fk: 2.0 * S * fk)
    with pytest.raises(RuntimeError):
        _thermal_fd_mismatch()


def test_thermal_pin_catches_occupancy_without_spin_factor(monkeypatch):
    """Occupancy f in [0, 1] while its derivative still carries the factor s = 2."""
    from oracle import thermal as th
    orig = th.occupancy
    monkeypatch.setattr(th, "occupancy", lambda e, mu, kT, smax=2.0: orig(e, mu, kT, 1.0))
    assert _thermal_fd_mismatch() > 1e-3


# ------------------------------------------------------- linear v_xc mesh (Eq. 14)
def test_vxc_pin_catches_swapped_hat_weights(monkeypatch):
    from oracle import vxcmesh as vm
    from synth import vxc_vertices

    def mismatch():
        m = fe.mesh3d(3, 2, 3.0)
        t = vxc_vertices(3.0, 0.8, 1.5, 1.5)
        P = vm.prolongation(m, t, t, t)
        V = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
        return np.abs(P @ (1.0 + V[:, 0] - 2 * V[:, 2]) - (1.0 + m.coords()[:, 0] - 2 * m.coords()[:, 2])).max()

    assert mismatch() < 1e-12
    orig = vm.hat_weights
    monkeypatch.setattr(vm, "hat_weights", lambda t, x: [(c, 1.0 - w) for c, w in orig(t, x)])
    assert mismatch() > 1e-2
