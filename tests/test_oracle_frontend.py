"""Pins of the physics front end: the Hartree solve and the initial guess (Eq. 25; CPU only).

Hartree (-lap v_H = 4 pi rho on the orbital mesh):
* a manufactured solution u = prod (L^2 - x_i^2), which every order-p space with p >= 3
  holds and whose lumped right-hand side is then exact, is reproduced to rounding;
* two Gaussian charges: the split-off monopole leaves an error that shrinks with the
  mesh (discretisation only), while solving without the split keeps the box's error.
Initial guess:
* the Slater potential is the derivative of the exchange energy density -(3/4)(3/pi)^{1/3} rho^{4/3};
* the PW92 potential is the derivative of rho e_c(r_s), by central differences;
* e_c(r_s) follows the exact high-density form A ln r_s + const with A = (1 - ln 2)/pi^2;
* f = rho/(rho + tau) blends v_0 into the Fermi-Amaldi tail -v_H / N_e.
"""
import numpy as np
import pytest

from oracle import fe, hartree as hr, xcinit as xc


@pytest.mark.parametrize("p,n,L", [(3, 3, 2.0), (4, 2, 1.5), (5, 2, 2.5)])
def test_poisson_manufactured_solution(p, n, L):
    m = fe.mesh3d(p, n, L)
    X = m.coords()
    a = L * L - X * X
    u = np.prod(a, axis=1)
    f = 2 * (a[:, 1] * a[:, 2] + a[:, 0] * a[:, 2] + a[:, 0] * a[:, 1])       # -lap u
    phi, Q, c = hr.hartree(m, f / (4 * np.pi), 0.0)
    assert np.abs(phi - u).max() <= 1e-12 * np.abs(u).max()


def test_poisson_gaussian_charges_with_monopole_split():
    errs = []
    for n in (6, 8):
        m = fe.mesh3d(4, n, 8.0)
        X = m.coords()
        c0 = np.array([0.3, -0.2, 0.1])
        c1 = c0 + np.array([1.0, 0.5, 0.0])
        rho = 3.0 * hr.gaussian(X, c0, 0.8) + 0.5 * hr.gaussian(X, c1, 0.6)
        exact = 3.0 * hr.gaussian_potential(X, c0, 0.8) + 0.5 * hr.gaussian_potential(X, c1, 0.6)
        inner = np.max(np.abs(X), axis=1) < 4.0
        phi, Q, c = hr.hartree(m, rho, 1.0)
        errs.append(np.abs(phi - exact)[inner].max())
        phi0, _, _ = hr.hartree(m, rho, 0.0)
        assert np.abs(phi0 - exact)[inner].max() > 0.3          # the box's zero values, unsplit
        assert abs(Q - 3.5) < 5e-3
    assert errs[1] < errs[0] / 4 and errs[1] < 5e-3, errs


def test_slater_is_derivative_of_exchange_energy():
    rho = np.logspace(-6, 2, 41)
    e = lambda r: -0.75 * np.cbrt(3.0 / np.pi) * r ** (4.0 / 3.0)
    h = 1e-4 * rho
    fd = (e(rho + h) - e(rho - h)) / (2 * h)
    np.testing.assert_allclose(xc.slater_exchange(rho), fd, rtol=1e-7)


def test_pw92_potential_is_derivative_of_energy_density():
    rho = np.logspace(-6, 2, 41)

    def E(r):
        rs = np.cbrt(3.0 / (4.0 * np.pi * r))
        return r * xc.pw92_energy(rs)
    h = 1e-4 * rho
    fd = (E(rho + h) - E(rho - h)) / (2 * h)
    np.testing.assert_allclose(xc.pw92_potential(rho), fd, rtol=1e-6)


def test_pw92_high_density_limit():
    A = (1 - np.log(2)) / np.pi ** 2
    rs = np.array([1e-6, 1e-5])
    ec = xc.pw92_energy(rs)
    assert abs((ec[1] - ec[0]) / np.log(10.0) - A) < 1e-4 * A      # slope of e_c in ln r_s
    assert abs(xc.PW92["A"] - A) < 1e-6


def test_initial_guess_blend():
    rho = np.array([0.0, 1e-8, 1e-2, 10.0])
    vh = np.array([2.0, 2.0, 3.0, 5.0])
    v = xc.initial_guess(rho, vh, 10.0, tau=1e-2, alpha=1.0)
    assert v[0] == -0.2                                          # empty: pure Fermi-Amaldi
    f = rho / (rho + 1e-2)
    v0 = xc.slater_exchange(rho) + xc.pw92_potential(rho)
    np.testing.assert_allclose(v, f * v0 - (1 - f) * vh / 10.0, rtol=1e-14)
    assert abs(v[3] - v0[3]) < 1e-2 * abs(v0[3])                   # dense: v_0
