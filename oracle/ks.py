"""Forward Kohn-Sham solve, density, loss, adjoint and gradient (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Zero-temperature, spin-restricted reading of Sec. 2: the N_occ = N_e/2 lowest
orbitals carry f_i = 2 (Eq. 5 with the Fermi-Dirac occupancy at T -> 0), the
density is rho_a = sum_i f_i psi~_{a,i}^2 / W_a (Eq. 4 in the standard-form
coefficients psi~ = W^{1/2} psi of Eq. 19), and the loss is
L = sum_a W_a (rho_data,a - rho_a)^2 (Eq. 1 with w = 1, GLL quadrature).

Adjoint (Eqs. 7, 10, 18, 20 and the null-space treatment of Sec. 3.2.2): with
r~_i = 4 f_i (rho - rho_data) * psi~_i and P = I - Psi~ Psi~^T (all occupied
orbitals), q_i solves (H~ - eps_i) q_i = -P r~_i with Psi~^T q_i = 0, and the
gradient of L with respect to the nodal potential is g_b = sum_i psi~_{b,i} q_{b,i}
(Eqs. 11, 22 with the potential collocated at the nodes).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe


@dataclass
class Forward:
    eps: np.ndarray      # (k,) ascending eigenvalues
    psi: np.ndarray      # (N_f, k) orthonormal standard-form eigenvectors


def operator(mesh: fe.Mesh3D, v: np.ndarray, use_csr: bool | None = None):
    """H~ as CSR (small meshes) or as a Kronecker LinearOperator (any mesh)."""
    n = mesh.n_free
    if use_csr is None:
        use_csr = n <= 20000
    if use_csr:
        return fe.hamiltonian_csr(mesh, v)
    vv = np.asarray(v, dtype=np.float64)

    def mv(x):
        return fe.hamiltonian_apply(mesh, vv, x.reshape(n, -1)).reshape(x.shape)

    return spla.LinearOperator((n, n), matvec=mv, matmat=lambda X: fe.hamiltonian_apply(mesh, vv, X),
                               dtype=np.float64)


def forward(mesh: fe.Mesh3D, v: np.ndarray, k: int, *, dense: bool | None = None,
            tol: float = 1e-13, v0: np.ndarray | None = None) -> Forward:
    """Lowest k eigenpairs of H~ (Eq. 19).

    Dense ``scipy.linalg.eigh`` on small meshes, Lanczos ``eigsh`` otherwise.
    """
    n = mesh.n_free
    if dense is None:
        dense = n <= 3000
    if dense:
        H = fe.hamiltonian_csr(mesh, v).toarray()
        w, V = sla.eigh(H, subset_by_index=[0, k - 1])
        return Forward(eps=w, psi=V)
    A = operator(mesh, v)
    ncv = min(n - 1, max(2 * k + 20, 40))
    w, V = spla.eigsh(A, k=k, which="SA", tol=tol, ncv=ncv, v0=v0, maxiter=200000)
    order = np.argsort(w)
    return Forward(eps=w[order], psi=V[:, order])


def occupations(n_elec: int) -> np.ndarray:
    """f_i = 2 for the N_e/2 lowest orbitals (T -> 0, spin-restricted)."""
    return np.full(n_elec // 2, 2.0)


def density(psi: np.ndarray, occ: np.ndarray, W: np.ndarray) -> np.ndarray:
    """rho_a = sum_i f_i psi~_{a,i}^2 / W_a (Eq. 4)."""
    k = occ.size
    return (psi[:, :k] ** 2 @ occ) / W


def electron_count(rho: np.ndarray, W: np.ndarray) -> float:
    """int rho by GLL quadrature, sum_a W_a rho_a (Eq. 5)."""
    return float(np.sum(W * rho))


def loss(rho: np.ndarray, rho_data: np.ndarray, W: np.ndarray) -> float:
    """L = int (rho_data - rho)^2 (Eq. 1, w = 1) by GLL quadrature."""
    d = rho_data - rho
    return float(np.sum(W * d * d))


def adjoint_rhs(psi_occ: np.ndarray, occ: np.ndarray, rho: np.ndarray,
                rho_data: np.ndarray) -> np.ndarray:
    """b_i = -(I - Psi~ Psi~^T) r~_i, r~_i = 4 f_i (rho - rho_data) psi~_i.

    Eq. 7 in standard form (Eq. 20): the right-hand side 4 f (rho_data - rho) psi
    minus its component along the occupied orbitals (Eq. 10).
    """
    R = 4.0 * (rho - rho_data)[:, None] * psi_occ * occ[None, :]
    return -(R - psi_occ @ (psi_occ.T @ R))


def adjoint_bordered(H: sp.spmatrix, psi_occ: np.ndarray, eps: np.ndarray,
                     B: np.ndarray) -> np.ndarray:
    """Direct solve of [[H~ - eps_i, Psi~], [Psi~^T, 0]] [q_i; d] = [b_i; 0] by sparse LU."""
    n, k = psi_occ.shape
    Q = np.zeros_like(B)
    Ps = sp.csr_matrix(psi_occ)
    for i in range(B.shape[1]):
        A = sp.bmat([[H - eps[i] * sp.identity(n), Ps], [Ps.T, None]], format="csc")
        rhs = np.concatenate([B[:, i], np.zeros(k)])
        Q[:, i] = spla.splu(A).solve(rhs)[:n]
    return Q


def adjoint_sum_over_states(eps_all: np.ndarray, psi_all: np.ndarray, n_occ: int,
                            R: np.ndarray) -> np.ndarray:
    """First-order perturbation theory: q_i = sum_{a > N_occ} psi~_a (psi~_a^T r~_i) / (eps_i - eps_a).

    ``R`` holds the unprojected r~_i; only unoccupied states enter.
    """
    U = psi_all[:, n_occ:]
    Q = np.zeros((psi_all.shape[0], n_occ))
    for i in range(n_occ):
        c = (U.T @ R[:, i]) / (eps_all[i] - eps_all[n_occ:])
        Q[:, i] = U @ c
    return Q


def adjoint_cg(mesh: fe.Mesh3D, v: np.ndarray, psi_occ: np.ndarray, eps: np.ndarray,
               B: np.ndarray, rtol: float = 1e-12, maxiter: int = 100000) -> np.ndarray:
    """Conjugate gradients on P (H~ - eps_i) P q = b_i (SPD on the complement of Psi~)."""
    n = mesh.n_free
    Q = np.zeros_like(B)

    def proj(x):
        return x - psi_occ @ (psi_occ.T @ x)

    for i in range(B.shape[1]):
        ei = eps[i]

        def mv(x, ei=ei):
            y = proj(x)
            return proj(fe.hamiltonian_apply(mesh, v, y) - ei * y)

        A = spla.LinearOperator((n, n), matvec=mv, dtype=np.float64)
        q, info = spla.cg(A, B[:, i], rtol=rtol, atol=0.0, maxiter=maxiter)
        if info != 0:
            raise RuntimeError(f"oracle CG did not converge for column {i} (info={info})")
        Q[:, i] = proj(q)
    return Q


def gradient(psi_occ: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """g_b = sum_i psi~_{b,i} q_{b,i} (Eqs. 11, 22 with the collocated potential)."""
    return np.sum(psi_occ * Q, axis=1)


def mask_gradient(g: np.ndarray, rho_data: np.ndarray, tau_bc: float) -> np.ndarray:
    """Zero the update where rho_data < tau_BC (Sec. 3.1.2, far-field treatment)."""
    if tau_bc <= 0:
        return g
    out = g.copy()
    out[rho_data < tau_bc] = 0.0
    return out


@dataclass
class Evaluation:
    eps: np.ndarray
    psi: np.ndarray
    rho: np.ndarray
    loss: float
    grad: np.ndarray | None
    Q: np.ndarray | None


def evaluate(mesh: fe.Mesh3D, v: np.ndarray, rho_data: np.ndarray, n_elec: int, *,
             want_grad: bool = True, method: str = "auto", tau_bc: float = 0.0,
             extra: int = 2, tol: float = 1e-13) -> Evaluation:
    """L(v) and dL/dv at the potential v = v_fixed + u (Eqs. 1, 4, 7, 11).

    method: "sos" (full dense spectrum, sum over states), "bordered" (sparse LU
    of the bordered system), "cg" (projected CG), or "auto".
    """
    occ = occupations(n_elec)
    k = occ.size
    W = mesh.weights()
    n = mesh.n_free
    if method == "auto":
        method = "sos" if n <= 3000 else ("bordered" if n <= 20000 else "cg")
    if method == "sos":
        H = fe.hamiltonian_csr(mesh, v).toarray()
        eps_all, psi_all = sla.eigh(H)
        fw = Forward(eps=eps_all[:k + extra], psi=psi_all[:, :k + extra])
    else:
        fw = forward(mesh, v, k + extra, tol=tol)
    psi = fw.psi[:, :k]
    rho = density(psi, occ, W)
    L = loss(rho, rho_data, W)
    if not want_grad:
        return Evaluation(fw.eps, fw.psi, rho, L, None, None)
    if method == "sos":
        R = 4.0 * (rho - rho_data)[:, None] * psi * occ[None, :]
        Q = adjoint_sum_over_states(eps_all, psi_all, k, R)
    elif method == "bordered":
        B = adjoint_rhs(psi, occ, rho, rho_data)
        Q = adjoint_bordered(fe.hamiltonian_csr(mesh, v), psi, fw.eps[:k], B)
    else:
        B = adjoint_rhs(psi, occ, rho, rho_data)
        Q = adjoint_cg(mesh, v, psi, fw.eps[:k], B)
    g = mask_gradient(gradient(psi, Q), rho_data, tau_bc)
    return Evaluation(fw.eps, fw.psi, rho, L, g, Q)


def target_density(mesh: fe.Mesh3D, v_star: np.ndarray, n_elec: int, tol: float = 1e-13):
    """rho_data = rho(v*): the density of the known potential (validation recipe, Sec. 5.1)."""
    occ = occupations(n_elec)
    fw = forward(mesh, v_star, occ.size + 2, tol=tol)
    return density(fw.psi[:, :occ.size], occ, mesh.weights()), fw


def loss_only(mesh: fe.Mesh3D, v: np.ndarray, rho_data: np.ndarray, n_elec: int,
              dense: bool | None = None) -> float:
    occ = occupations(n_elec)
    fw = forward(mesh, v, occ.size, dense=dense)
    return loss(density(fw.psi, occ, mesh.weights()), rho_data, mesh.weights())


def fd_directional(mesh: fe.Mesh3D, v: np.ndarray, rho_data: np.ndarray, n_elec: int,
                   d: np.ndarray, h: float = 1e-5) -> float:
    """Central difference (L(v + h d) - L(v - h d)) / (2 h)."""
    lp = loss_only(mesh, v + h * d, rho_data, n_elec)
    lm = loss_only(mesh, v - h * d, rho_data, n_elec)
    return (lp - lm) / (2.0 * h)
