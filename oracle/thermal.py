"""Finite temperature: Fermi-Dirac occupancy and the adjoint with fractional
occupations and degenerate blocks (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2, taken in the paper's order, in the standard-form coefficients
psi~ = W^{1/2} psi (Eq. 19) with w = 1 and GLL quadrature, so that an integral
int g psi_i psi_j becomes sum_a g_a psi~_{a,i} psi~_{a,j}:

* occupancy f(eps) = s / (1 + exp((eps - mu) / k_B T)) (Eq. 4's Fermi-Dirac
  matrix; s = 2 for the spin-restricted reading used throughout, s = 1 is the
  paper's literal per-orbital occupancy), mu fixed by sum_i f_i = N_e (Eq. 5);
* density rho_a = sum_i f_i psi~_{a,i}^2 / W_a (Eq. 4), loss (Eq. 1);
* eigenvalues grouped into degenerate blocks Psi_k (m_k columns, one
  eigenvalue eps_k), f(E_k) = f(eps_k) I;
* eta from Eq. 9, D_k + D_k^T from the closed form that follows Eq. 9 (the one
  obtained by multiplying Eq. 7 by Psi_k^T), the adjoint of Eq. 7 solved on
  the complement of the block's own orbitals only (Sec. 3.2.2: the operator
  (H~ - eps_k) is singular on Psi_k and the right-hand side is orthogonal to
  it), plus the component along Psi_k given by Eq. 8;
* gradient delta L / delta v_b = sum_k tr(P_k^T Psi_k)_b (Eq. 10, nodal).

Unlike the zero-temperature module, every state with a non-negligible
occupation enters, and the adjoint of one block keeps its components along the
other blocks: the per-block solve is a sparse LU of the system bordered by that
block alone.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import expit

from . import fe, ks


def occupancy(eps: np.ndarray, mu: float, kT: float, smax: float = 2.0) -> np.ndarray:
    """f(eps) = s / (1 + exp((eps - mu) / k_B T)) (Fermi-Dirac, Eq. 4)."""
    return smax * expit(-(np.asarray(eps, dtype=np.float64) - mu) / kT)


def occupancy_deps(eps: np.ndarray, mu: float, kT: float, smax: float = 2.0) -> np.ndarray:
    """d f / d eps = -s phi (1 - phi) / k_B T with phi = f / s; d f / d mu is its negative."""
    phi = expit(-(np.asarray(eps, dtype=np.float64) - mu) / kT)
    return -smax * phi * (1.0 - phi) / kT


def chemical_potential(eps: np.ndarray, n_elec: float, kT: float, smax: float = 2.0) -> float:
    """mu with sum_i f(eps_i) = N_e (Eq. 5), by bisection to the last bit.

    sum_i f is increasing in mu, so the bracket [min eps - 60 kT, max eps + 60 kT]
    contains the root whenever 0 < N_e < s * len(eps).
    """
    eps = np.asarray(eps, dtype=np.float64)
    if not 0.0 < n_elec < smax * eps.size:
        raise ValueError("N_e must lie strictly between 0 and s times the number of states")
    lo, hi = eps.min() - 60.0 * kT, eps.max() + 60.0 * kT
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if occupancy(eps, mid, kT, smax).sum() < n_elec:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def degenerate_blocks(eps: np.ndarray, tol: float = 1e-8) -> list[np.ndarray]:
    """Index sets of eigenvalues that agree to within ``tol`` (the blocks Psi_k of Sec. 2)."""
    blocks, start = [], 0
    for i in range(1, eps.size + 1):
        if i == eps.size or eps[i] - eps[i - 1] > tol:
            blocks.append(np.arange(start, i))
            start = i
    return blocks


def states(mesh: fe.Mesh3D, v: np.ndarray, n_elec: float, kT: float, *, smax: float = 2.0,
           n_states: int | None = None, cut: float = 1e-14, tol: float = 1e-13) -> tuple:
    """The lowest eigenpairs, mu and f, keeping every state with f_i > cut * s.

    With ``n_states`` None the whole spectrum is taken (dense); otherwise that many
    Lanczos eigenpairs, and the highest must be empty to within ``cut``.
    """
    n = mesh.n_free
    if n_states is None or n_states >= n:
        eps, psi = sla.eigh(fe.hamiltonian_csr(mesh, v).toarray())
    else:
        fw = ks.forward(mesh, v, n_states, tol=tol)
        eps, psi = fw.eps, fw.psi
    mu = chemical_potential(eps, n_elec, kT, smax)
    occ = occupancy(eps, mu, kT, smax)
    keep = int(np.count_nonzero(occ > cut * smax))
    if n_states is not None and n_states < n and keep >= n_states:
        raise ValueError("the highest computed state is occupied: compute more states")
    while keep < eps.size and eps[keep] - eps[keep - 1] <= 1e-8:
        keep += 1                  # never split a degenerate block
    return eps[:keep], psi[:, :keep], mu, occ[:keep]


def eta(blocks, eps_blk, dfde_blk, psi: np.ndarray, delta: np.ndarray) -> float:
    """eta of Eq. 9: eta sum_k m_k df_k/dmu = 2 sum_k df_k/dmu int (rho_d - rho) tr(Psi_k^T Psi_k).

    d f/d mu = -d f/d eps. When no state lies within reach of mu both sides vanish
    (the T -> 0 case) and eta does not enter the gradient; 0 is returned.
    """
    num = den = 0.0
    for b, dfde in zip(blocks, dfde_blk):
        dfdmu = -dfde
        den += b.size * dfdmu
        num += 2.0 * dfdmu * float(np.sum(delta[:, None] * psi[:, b] ** 2))
    return num / den if den != 0.0 else 0.0


def d_plus_dt(S: np.ndarray, fk: float) -> np.ndarray:
    """D_k + D_k^T = 4 [int (rho_d - rho) Psi_k^T Psi_k] f(E_k) (the closed form after Eq. 9)."""
    return 4.0 * S * fk


def overlap(S: np.ndarray, dfde: float, et: float) -> np.ndarray:
    """int Psi_k^T P_k = df_k/deps [-2 int (rho_d - rho) Psi_k^T Psi_k + eta I] (Eq. 8)."""
    return dfde * (-2.0 * S + et * np.eye(S.shape[0]))


def adjoint(H: sp.spmatrix, psi: np.ndarray, eps: np.ndarray, kT: float, mu: float, rho: np.ndarray,
            rho_data: np.ndarray, *, smax: float = 2.0, deg_tol: float = 1e-8) -> tuple:
    """P~ = [P~_1 | ... | P~_M] for all kept blocks (Eqs. 7, 8, 9, Sec. 3.2.2). Returns (P, eta).

    For block k with eigenvalue eps_k and occupancy f_k:
      D_k + D_k^T = 4 [Psi_k^T diag(rho_d - rho) Psi_k] f_k                 (after Eq. 9)
      (H~ - eps_k) P_perp = 4 (rho_d - rho) Psi_k f_k - Psi_k (D_k + D_k^T),
          Psi_k^T P_perp = 0                                               (Eq. 7)
      d_k = df_k/deps [-2 Psi_k^T diag(rho_d - rho) Psi_k + eta I]          (Eq. 8)
      P_k = P_perp + Psi_k d_k                                             (Sec. 3.2.2)
    """
    n = psi.shape[0]
    delta = rho_data - rho
    blocks = degenerate_blocks(eps, deg_tol)
    eps_blk = [float(eps[b].mean()) for b in blocks]
    f_blk = [float(occupancy(e, mu, kT, smax)) for e in eps_blk]
    dfde_blk = [float(occupancy_deps(e, mu, kT, smax)) for e in eps_blk]
    et = eta(blocks, eps_blk, dfde_blk, psi, delta)
    P = np.zeros_like(psi)
    for b, ek, fk, dk in zip(blocks, eps_blk, f_blk, dfde_blk):
        Pk = psi[:, b]
        S = Pk.T @ (delta[:, None] * Pk)                   # int (rho_d - rho) Psi_k^T Psi_k
        DDt = d_plus_dt(S, fk)
        rhs = 4.0 * delta[:, None] * Pk * fk - Pk @ DDt
        if np.abs(Pk.T @ rhs).max() > 1e-9 * max(np.abs(rhs).max(), 1e-300):
            raise RuntimeError("Eq. 7's right-hand side is not orthogonal to its block")
        Bk = sp.csr_matrix(Pk)
        A = sp.bmat([[H - ek * sp.identity(n), Bk], [Bk.T, None]], format="csc")
        lu = spla.splu(A)
        Pperp = np.empty_like(Pk)
        for c in range(b.size):
            Pperp[:, c] = lu.solve(np.concatenate([rhs[:, c], np.zeros(b.size)]))[:n]
        P[:, b] = Pperp + Pk @ overlap(S, dk, et)
    return P, et


def gradient(psi: np.ndarray, P: np.ndarray) -> np.ndarray:
    """delta L / delta v_b = sum_k tr(P_k^T Psi_k) at node b (Eq. 10 with the collocated potential)."""
    return np.sum(psi * P, axis=1)


@dataclass
class Evaluation:
    eps: np.ndarray
    psi: np.ndarray
    mu: float
    occ: np.ndarray
    rho: np.ndarray
    loss: float
    grad: np.ndarray | None
    P: np.ndarray | None
    eta: float | None


def evaluate(mesh: fe.Mesh3D, v: np.ndarray, rho_data: np.ndarray, n_elec: float, kT: float, *,
             smax: float = 2.0, n_states: int | None = None, want_grad: bool = True,
             cut: float = 1e-14) -> Evaluation:
    """L(v) and delta L / delta v at finite temperature (Eqs. 1, 4, 5, 7-10)."""
    eps, psi, mu, occ = states(mesh, v, n_elec, kT, smax=smax, n_states=n_states, cut=cut)
    W = mesh.weights()
    rho = ks.density(psi, occ, W)
    L = ks.loss(rho, rho_data, W)
    if not want_grad:
        return Evaluation(eps, psi, mu, occ, rho, L, None, None, None)
    P, et = adjoint(fe.hamiltonian_csr(mesh, v), psi, eps, kT, mu, rho, rho_data, smax=smax)
    return Evaluation(eps, psi, mu, occ, rho, L, gradient(psi, P), P, et)


def target_density(mesh: fe.Mesh3D, v_star: np.ndarray, n_elec: float, kT: float, *, smax: float = 2.0,
                   n_states: int | None = None) -> np.ndarray:
    """rho_data = rho(v*) at the same temperature (the validation recipe of Sec. 5.1)."""
    eps, psi, mu, occ = states(mesh, v_star, n_elec, kT, smax=smax, n_states=n_states)
    return ks.density(psi, occ, mesh.weights())


def fd_directional(mesh: fe.Mesh3D, v: np.ndarray, rho_data: np.ndarray, n_elec: float, kT: float,
                   d: np.ndarray, h: float = 1e-5, *, smax: float = 2.0,
                   n_states: int | None = None) -> float:
    """Central difference of L along d, with mu solved again at each potential."""
    lp = evaluate(mesh, v + h * d, rho_data, n_elec, kT, smax=smax, n_states=n_states, want_grad=False).loss
    lm = evaluate(mesh, v - h * d, rho_data, n_elec, kT, smax=smax, n_states=n_states, want_grad=False).loss
    return (lp - lm) / (2.0 * h)
