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


@pytest.mark.parametrize("p", [2, 3, 5])
def test_nodal_gradient_exact_for_interpolated_polynomials(p):
    """A field of degree <= p per axis that vanishes on the box is its own interpolant: the
    recovered gradient is exact, also at vertices shared by two cells (both one-sided values
    agree) and on graded cells."""
    from synth import vxc_vertices
    a = (lambda t: 4 - t * t, lambda t: -2 * t)                    # degree 2, zero at +-2
    b = (lambda t: (4 - t * t) * (1 + t), lambda t: -2 * t * (1 + t) + (4 - t * t))   # degree 3
    for m in (fe.mesh3d(p, 3, 2.0), fe.mesh3d_graded(p, vxc_vertices(2.0, 0.5, 0.6, 1.8))):
        X = m.coords()
        fx, fy, fz = a, (b if p >= 3 else a), (b if p >= 3 else a)
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        f = fx[0](x) * fy[0](y) * fz[0](z)
        g = np.stack([fx[1](x) * fy[0](y) * fz[0](z), fx[0](x) * fy[1](y) * fz[0](z),
                      fx[0](x) * fy[0](y) * fz[1](z)], axis=1)
        np.testing.assert_allclose(fe.nodal_gradient(m, f), g, rtol=0, atol=1e-11 * np.abs(g).max())


def test_lb94_decays_as_minus_one_over_r():
    """For an exponential density the LB94 potential tends to -1/r (its design property)."""
    # rho = e^{-a r} / pi: x_s = a rho_s^{-1/3}, and for large x the correction tends to
    # -(a/3) / ln(2 x_s), so r v -> -(a r/3) / (a r/3 + ln(2a) + ln(2 pi)/3) -> -1 (slowly)
    a = 2.0
    r = np.array([10.0, 15.0, 20.0, 30.0])
    rho = np.exp(-a * r) / np.pi
    v = xc.lb94_exchange(rho, a * rho)
    asym = -(a * r / 3) / (a * r / 3 + np.log(2 * a) + np.log(2 * np.pi) / 3)
    np.testing.assert_allclose(v * r, asym, rtol=0.02)
    assert np.all(np.diff(v * r) < 0) and v[-1] * r[-1] < -0.9
    # and it is the Slater potential minus a non-negative correction
    rho2 = np.logspace(-6, 1, 20)
    assert np.all(xc.lb94_exchange(rho2, 0.3 * rho2) <= xc.slater_exchange(rho2) + 1e-15)
    np.testing.assert_allclose(xc.lb94_exchange(rho2, 0 * rho2), xc.slater_exchange(rho2), rtol=1e-15)


# ------------------------------------------------------------- PW92 constants
# The PW92 fit (Perdew and Wang, Phys. Rev. B 45, 13244 (1992)) is built on the limits of the
# uniform electron gas, which fix every one of its six constants:
#   high density  e_c = c0 ln r_s - c1 + O(r_s ln r_s), c0 = (1 - ln 2)/pi^2 (exact), c1 = 0.046644,
#                 and no r_s^{1/2} term: b1 = e^{-c1/(2 c0)} / (2 c0), b2 = 2 c0 b1^2;
#   low density   e_c = -d0 / r_s + d1 / r_s^{3/2} + ..., d0 = a1/b4 = 0.4335, d1 = a1 b3 / b4^2 = 1.4408.
# c1, d0 and d1 are the published expansion coefficients; their printed digits set the tolerances.
PW92_C1, PW92_D0, PW92_D1 = 0.046644, 0.4335, 1.4408


def _pw92_relations(P):
    """Relative misfit of each defining relation for a parameter set P."""
    c0 = (1 - np.log(2)) / np.pi ** 2
    return {
        "A": (abs(P["A"] / c0 - 1), 2e-5),
        "b1": (abs(P["b1"] * 2 * P["A"] / np.exp(-PW92_C1 / (2 * P["A"])) - 1), 2e-5),
        "b2": (abs(P["b2"] / (2 * P["A"] * P["b1"] ** 2) - 1), 2e-5),
        "d0": (abs(P["a1"] / P["b4"] / PW92_D0 - 1), 2e-4),
        "d1": (abs(P["a1"] * P["b3"] / P["b4"] ** 2 / PW92_D1 - 1), 1e-4),
    }


def test_pw92_constants_from_electron_gas_limits():
    for name, (err, tol) in _pw92_relations(xc.PW92).items():
        assert err < tol, (name, err)


def test_pw92_energy_has_both_limits():
    """The coded e_c (not just its constants) follows both expansions."""
    rs = np.array([1e-9, 1e-10])
    lead = xc.pw92_energy(rs) - xc.PW92["A"] * np.log(rs)       # -> -c1 (A itself is pinned above)
    np.testing.assert_allclose(lead, -PW92_C1, rtol=3e-5)
    rs = np.array([1e6, 4e6])
    e = xc.pw92_energy(rs)
    np.testing.assert_allclose(-e * rs, PW92_D0 - PW92_D1 / np.sqrt(rs), rtol=3e-4)


def test_pw92_one_digit_slip_is_caught():
    """Changing any one constant in its fourth significant digit breaks a relation."""
    for key in xc.PW92:
        bad = dict(xc.PW92)
        v = bad[key]
        bad[key] = v + 10.0 ** (np.floor(np.log10(abs(v))) - 3)
        misfit = _pw92_relations(bad)
        assert any(err >= tol for err, tol in misfit.values()), key
