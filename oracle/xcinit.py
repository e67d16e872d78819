"""The initial guess for v_xc (Eq. 25) from a target density (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

    v_init = f v_0 + (1 - f) alpha v_FA,    f = rho / (rho + tau),   v_FA = -v_H / N_e,
    v_0 = v_x + v_c^PW92                                           (Eq. 25 and the line after)

with v_x the Slater (local-density) exchange potential of the spin-unpolarised gas,
    v_x = -(3 rho / pi)^{1/3}     (the derivative of rho e_x, e_x = -(3/4)(3 rho / pi)^{1/3}),
and the Perdew-Wang 1992 correlation of the unpolarised gas, r_s = (3 / (4 pi rho))^{1/3},
    e_c(r_s) = -2A (1 + a1 r_s) ln(1 + 1 / (2A (b1 r_s^{1/2} + b2 r_s + b3 r_s^{3/2} + b4 r_s^2))),
    v_c = e_c - (r_s / 3) de_c/dr_s.
The paper names PW92 for v_0 of Eq. 25 but prints none of its parameters; the values below are the
published unpolarised-gas parameters of J. P. Perdew and Y. Wang, Phys. Rev. B 45, 13244 (1992):
A = 0.031091, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294 (exponent p = 1).
The fit is built to reproduce the limits of the electron gas: the high-density expansion
e_c = A ln r_s - c1 + O(r_s ln r_s) with A = (1 - ln 2)/pi^2 and c1 = 0.046644, with no
r_s^{1/2} term (so b1 = e^{-c1/2A}/2A and b2 = 2 A b1^2), and the low-density expansion
e_c = -d0/r_s + d1/r_s^{3/2} with d0 = a1/b4 = 0.4335 and d1 = a1 b3/b4^2 = 1.4408. The tests
pin every constant by these relations.
LB94 exchange (van Leeuwen and Baerends 1994, the paper's recommended choice) uses the published
beta = 0.05; its design property, the -1/r tail, does not depend on beta, so beta is unpinned.
Densities below 1e-30 are treated as empty (v_x = v_c = 0 there).
"""
from __future__ import annotations

import numpy as np

PW92 = dict(A=0.031091, a1=0.21370, b1=7.5957, b2=3.5876, b3=1.6382, b4=0.49294)
RHO_MIN = 1e-30


def slater_exchange(rho: np.ndarray) -> np.ndarray:
    r = np.maximum(rho, 0.0)
    return np.where(r > RHO_MIN, -np.cbrt(3.0 * r / np.pi), 0.0)


def pw92_energy(rs: np.ndarray) -> np.ndarray:
    """Correlation energy per electron e_c(r_s) of the unpolarised gas."""
    P = PW92
    q = 2 * P["A"] * (P["b1"] * np.sqrt(rs) + P["b2"] * rs + P["b3"] * rs ** 1.5 + P["b4"] * rs ** 2)
    return -2 * P["A"] * (1 + P["a1"] * rs) * np.log1p(1.0 / q)


def pw92_potential(rho: np.ndarray) -> np.ndarray:
    """v_c = d(rho e_c)/d rho = e_c - (r_s/3) de_c/dr_s, the derivative written out."""
    P = PW92
    r = np.maximum(rho, RHO_MIN)
    rs = np.cbrt(3.0 / (4.0 * np.pi * r))
    s = np.sqrt(rs)
    q = 2 * P["A"] * (P["b1"] * s + P["b2"] * rs + P["b3"] * rs * s + P["b4"] * rs * rs)
    dq = P["A"] * (P["b1"] / s + 2 * P["b2"] + 3 * P["b3"] * s + 4 * P["b4"] * rs)
    lg = np.log1p(1.0 / q)
    ec = -2 * P["A"] * (1 + P["a1"] * rs) * lg
    dec = -2 * P["A"] * P["a1"] * lg + 2 * P["A"] * (1 + P["a1"] * rs) * dq / (q * q + q)
    return np.where(rho > RHO_MIN, ec - rs / 3.0 * dec, 0.0)


LB94_BETA = 0.05


def lb94_exchange(rho: np.ndarray, grad_norm: np.ndarray) -> np.ndarray:
    """van Leeuwen-Baerends exchange of the unpolarised gas, per spin density rho_s = rho / 2:
    v_x = v_x^LDA(rho) - beta rho_s^{1/3} x^2 / (1 + 3 beta x asinh x), x = |grad rho_s| / rho_s^{4/3}."""
    r = np.maximum(rho, 0.0)
    ok = r > RHO_MIN
    rs = np.where(ok, 0.5 * r, 1.0)
    x = np.where(ok, 0.5 * grad_norm / rs ** (4.0 / 3.0), 0.0)
    corr = LB94_BETA * np.cbrt(rs) * x * x / (1.0 + 3.0 * LB94_BETA * x * np.arcsinh(x))
    return np.where(ok, slater_exchange(rho) - corr, 0.0)


def initial_guess(rho: np.ndarray, v_h: np.ndarray, n_elec: float, tau: float = 1e-2,
                  alpha: float = 1.0, grad_norm: np.ndarray | None = None) -> np.ndarray:
    """Eq. 25 with v_0 = Slater exchange + PW92 correlation, or LB94 exchange + PW92 when the
    density's gradient norm is given."""
    f = rho / (rho + tau)
    vx = slater_exchange(rho) if grad_norm is None else lb94_exchange(rho, grad_norm)
    v0 = vx + pw92_potential(rho)
    return f * v0 + (1.0 - f) * alpha * (-v_h / n_elec)
