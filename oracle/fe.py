"""Spectral finite elements and the standard-form Kohn-Sham operator (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Discretisation (the paper's Sec. 3.1.1 and Sec. 3.2.1, with the readings listed
in the design notes):

* Domain [-L, L]^3, n cells per axis of width h = 2L/n, tensor-product Lagrange
  basis of order p (Eq. 12) on Gauss-Lobatto-Legendre (GLL) nodes (the spectral
  elements of Sec. 3.2.1).
* 1-D global node g in [0, p n] sits at x_g = -L + h (e + (xi_j + 1)/2) with
  g = e p + j. Homogeneous Dirichlet: nodes g = 0 and g = p n are removed.
  Free node index a = (gx-1) + n1 ((gy-1) + n1 (gz-1)), n1 = p n - 1 (x fastest).
* Stiffness of Eq. 17 integrated exactly ((p+1)-point Gauss-Legendre), so
  K = K1 (x) Mc (x) Mc + Mc (x) K1 (x) Mc + Mc (x) Mc (x) K1 with the 1-D
  assembled stiffness K1 and consistent mass Mc.
* Overlap M lumped by GLL quadrature (Sec. 3.2.1): M = W = diag(W_a),
  W_a = W1(gx) W1(gy) W1(gz).
* Potential collocated at the GLL nodes: M_v = diag(W_a v_a).
* Standard form (Eq. 19): H~ = W^{-1/2} (K/2 + M_v) W^{-1/2} = K~/2 + diag(v),
  K~ = W^{-1/2} K W^{-1/2}.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg


# --------------------------------------------------------------------------- 1-D
def gll_nodes_weights(p: int):
    """GLL nodes and weights on [-1, 1] (Sec. 3.2.1, spectral elements).

    Nodes: -1, the p-1 roots of P_p', +1. Weights: 2 / (p (p+1) P_p(xi)^2).
    """
    cp = np.zeros(p + 1)
    cp[p] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(cp))) if p >= 2 else np.zeros(0)
    xi = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (p * (p + 1) * npleg.legval(xi, cp) ** 2)
    return xi, w


def gauss_nodes_weights(m: int):
    """m-point Gauss-Legendre rule on [-1, 1] (exact for degree <= 2m-1)."""
    return npleg.leggauss(m)


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[q, i] = N_i(x_q) for the Lagrange polynomials on ``nodes`` (Eq. 12).

    Written straight from the product formula N_i(x) = prod_{j != i} (x - x_j)/(x_i - x_j).
    """
    k = len(nodes)
    out = np.ones((len(x), k))
    for i in range(k):
        for j in range(k):
            if j != i:
                out[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return out


def lagrange_derivs(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[q, i] = N_i'(x_q): the product rule applied to Eq. 12."""
    k = len(nodes)
    out = np.zeros((len(x), k))
    for i in range(k):
        for m in range(k):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(k):
                if j != i and j != m:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            out[:, i] += term
    return out


def reference_matrices(p: int):
    """Reference K^_ij = int N_i' N_j' and M^_ij = int N_i N_j on [-1, 1] (Eq. 17).

    Both integrals by (p+1)-point Gauss-Legendre, exact for the degree-2p
    integrands. Returns (K^, M^, GLL nodes, GLL weights).
    """
    xi, wg = gll_nodes_weights(p)
    xq, wq = gauss_nodes_weights(p + 1)
    Nv = lagrange_values(xi, xq)
    Nd = lagrange_derivs(xi, xq)
    Kh = (Nd * wq[:, None]).T @ Nd
    Mh = (Nv * wq[:, None]).T @ Nv
    return Kh, Mh, xi, wg


@dataclass
class Mesh1D:
    """1-D assembled operators on the free nodes (size n1 = p n - 1)."""
    p: int
    n: int
    L: float
    h: float
    x: np.ndarray        # free-node coordinates
    K1: np.ndarray       # assembled stiffness, free-free block
    Mc: np.ndarray       # assembled consistent mass, free-free block
    W1: np.ndarray       # assembled GLL-lumped mass (diagonal)
    x_all: np.ndarray    # all node coordinates (0..pn)


def mesh1d(p: int, n: int, L: float, breaks: np.ndarray | None = None) -> Mesh1D:
    """Assemble the 1-D operators: K1 = sum_e (2/h_e) K^, Mc = sum_e (h_e/2) M^,
    W1 = sum_e (h_e/2) w^ over the n elements, then drop the two Dirichlet ends.

    Uniform cells of h = 2L/n on [-L, L], or, with ``breaks`` (n + 1 increasing cell
    boundaries), the graded mesh they define (cell e of width h_e = breaks[e+1] - breaks[e]);
    ``h`` is then the smallest width and L half the extent.
    """
    if breaks is None:
        t = -L + (2.0 * L / n) * np.arange(n + 1)
        hs = np.full(n, 2.0 * L / n)          # exactly 2L/n: differences of t would differ in the last bits
    else:
        t = np.asarray(breaks, dtype=np.float64)
        n = t.size - 1
        L = 0.5 * (t[-1] - t[0])
        hs = np.diff(t)
    Kh, Mh, xi, wg = reference_matrices(p)
    N = p * n + 1
    K = np.zeros((N, N))
    M = np.zeros((N, N))
    W = np.zeros(N)
    x = np.zeros(N)
    for e in range(n):
        h = hs[e]
        idx = e * p + np.arange(p + 1)
        K[np.ix_(idx, idx)] += (2.0 / h) * Kh
        M[np.ix_(idx, idx)] += (h / 2.0) * Mh
        W[idx] += (h / 2.0) * wg
        x[idx] = -L + h * (e + (xi + 1.0) / 2.0) if breaks is None else t[e] + h * (xi + 1.0) / 2.0
    f = slice(1, N - 1)
    return Mesh1D(p=p, n=n, L=L, h=float(hs.min()), x=x[f].copy(), K1=K[f, f].copy(), Mc=M[f, f].copy(),
                  W1=W[f].copy(), x_all=x)


# --------------------------------------------------------------------------- 3-D
@dataclass
class Mesh3D:
    m1: Mesh1D

    @property
    def n1(self) -> int:
        return self.m1.x.size

    @property
    def n_free(self) -> int:
        return self.n1 ** 3

    def coords(self) -> np.ndarray:
        """Free-node coordinates, (N_f, 3), x fastest."""
        x = self.m1.x
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def weights(self) -> np.ndarray:
        """Lumped mass W_a = W1(gx) W1(gy) W1(gz) at the free nodes."""
        w = self.m1.W1
        return np.kron(w, np.kron(w, w))


def mesh3d(p: int, n: int, L: float) -> Mesh3D:
    return Mesh3D(mesh1d(p, n, L))


def mesh3d_graded(p: int, breaks: np.ndarray) -> Mesh3D:
    """The tensor product of one graded 1-D mesh on every axis (cells of different widths;
    the Kronecker form of K holds because every cell is a product of 1-D cells)."""
    return Mesh3D(mesh1d(p, 0, 0.0, breaks=breaks))


def kinetic_csr(mesh: Mesh3D) -> sp.csr_matrix:
    """Assembled K~/2 = (1/2) W^{-1/2} K W^{-1/2} as CSR (Eqs. 17, 19).

    K = kron(Mc, kron(Mc, K1)) + kron(Mc, kron(K1, Mc)) + kron(K1, kron(Mc, Mc));
    the last Kronecker factor acts on x (x fastest).
    """
    if hasattr(mesh, "kinetic_csr"):                 # a mesh with its own per-cell matrices
        return mesh.kinetic_csr()
    m = mesh.m1
    K1 = sp.csr_matrix(m.K1)
    Mc = sp.csr_matrix(m.Mc)
    K = (sp.kron(Mc, sp.kron(Mc, K1)) + sp.kron(Mc, sp.kron(K1, Mc))
         + sp.kron(K1, sp.kron(Mc, Mc)))
    s = 1.0 / np.sqrt(mesh.weights())
    D = sp.diags(s)
    return (0.5 * (D @ K @ D)).tocsr()


def hamiltonian_csr(mesh: Mesh3D, v: np.ndarray) -> sp.csr_matrix:
    """H~ = K~/2 + diag(v) (Eq. 19 with the collocated potential)."""
    return (kinetic_csr(mesh) + sp.diags(np.asarray(v, dtype=np.float64))).tocsr()


def _along(A: np.ndarray, T: np.ndarray, axis: int) -> np.ndarray:
    """Apply the 1-D matrix A along grid axis ``axis`` of T[z, y, x, j]."""
    return np.moveaxis(np.tensordot(A, T, axes=([1], [axis])), 0, axis)


def kinetic_apply(mesh: Mesh3D, X: np.ndarray) -> np.ndarray:
    """(K~/2) X by Kronecker-factored 1-D applies, independent of the CSR path.

    X is (N_f, nv), node-major. Each of the three terms of K is applied as three
    1-D products along z, y, x of the W1^{-1/2}-scaled 1-D matrices.
    """
    if hasattr(mesh, "kinetic_csr"):                 # per-cell matrices: the assembled operator
        return mesh.kinetic_csr() @ np.asarray(X, dtype=np.float64)
    m = mesh.m1
    n1 = mesh.n1
    s = 1.0 / np.sqrt(m.W1)
    Ks = s[:, None] * m.K1 * s[None, :]
    Ms = s[:, None] * m.Mc * s[None, :]
    X2 = np.asarray(X, dtype=np.float64)
    squeeze = X2.ndim == 1
    if squeeze:
        X2 = X2[:, None]
    T = X2.reshape(n1, n1, n1, X2.shape[1])          # [z, y, x, j]
    t1 = _along(Ms, _along(Ms, _along(Ks, T, 2), 1), 0)
    t2 = _along(Ms, _along(Ks, _along(Ms, T, 2), 1), 0)
    t3 = _along(Ks, _along(Ms, _along(Ms, T, 2), 1), 0)
    out = (0.5 * (t1 + t2 + t3)).reshape(X2.shape)
    return out[:, 0] if squeeze else out


def hamiltonian_apply(mesh: Mesh3D, v: np.ndarray, X: np.ndarray) -> np.ndarray:
    """H~ X = (K~/2) X + v * X (Eq. 19), Kronecker path."""
    X = np.asarray(X, dtype=np.float64)
    vx = v[:, None] * X if X.ndim == 2 else v * X
    return kinetic_apply(mesh, X) + vx


def hamiltonian_rows(mesh: Mesh3D, v: np.ndarray, X: np.ndarray, rows, shift=None) -> np.ndarray:
    """Selected rows of (H~ - diag(shift)) X, each from its own definition (Eq. 19):

        (K~ X)_a = sum_b [Ks(ax,bx) Ms(ay,by) Ms(az,bz) + Ms(ax,bx) Ks(ay,by) Ms(az,bz)
                          + Ms(ax,bx) Ms(ay,by) Ks(az,bz)] X_b,

    with Ks, Ms the W1^{-1/2}-scaled assembled 1-D stiffness and consistent mass, and
    (H~ X)_a = (K~ X)_a / 2 + v_a X_a. Only the nodes b inside the 1-D bands of a enter,
    so a row costs O((2p+1)^3 nv) whatever the mesh size: this is how large meshes are
    checked on sampled outputs. rows: free-node indices; shift: nv per-column shifts.
    """
    m = mesh.m1
    n1 = mesh.n1
    s = 1.0 / np.sqrt(m.W1)
    Ks = s[:, None] * m.K1 * s[None, :]
    Ms = s[:, None] * m.Mc * s[None, :]
    X = np.asarray(X)
    nv = X.shape[1]
    T = X.reshape(n1, n1, n1, nv)                    # [z, y, x, j], a view
    rows = np.asarray(rows, dtype=np.int64)
    out = np.empty((rows.size, nv))
    for r, a in enumerate(rows):
        ax, ay, az = a % n1, (a // n1) % n1, a // (n1 * n1)
        band = [np.nonzero((Ks[c] != 0) | (Ms[c] != 0))[0] for c in (ax, ay, az)]
        bx, by, bz = band
        blk = T[np.ix_(bz, by, bx)].astype(np.float64)    # (nz, ny, nx, nv)
        kx, mx = Ks[ax, bx], Ms[ax, bx]
        ky, my = Ks[ay, by], Ms[ay, by]
        kz, mz = Ks[az, bz], Ms[az, bz]
        kin = (np.einsum("z,y,x,zyxj->j", mz, my, kx, blk) + np.einsum("z,y,x,zyxj->j", mz, ky, mx, blk)
               + np.einsum("z,y,x,zyxj->j", kz, my, mx, blk))
        xa = T[az, ay, ax].astype(np.float64)
        out[r] = 0.5 * kin + v[a] * xa
        if shift is not None:
            out[r] -= np.asarray(shift, dtype=np.float64) * xa
    return out


def derivative_1d(mesh: Mesh3D) -> np.ndarray:
    """D1 (n1 x n1): the derivative of the order-p interpolant at the free 1-D nodes, from the
    Lagrange derivatives of each cell (Eq. 12) with the two one-sided values averaged at a
    vertex shared by two cells; the Dirichlet end values are 0."""
    m = mesh.m1
    p, n = m.p, m.n
    xi, _ = gll_nodes_weights(p)
    Dh = lagrange_derivs(xi, xi)                      # Dh[j, k] = N_k'(xi_j)
    N = p * n + 1
    hs = np.diff(m.x_all[::p])                        # cell widths from the vertex coordinates
    D = np.zeros((N, N))
    cnt = np.zeros(N)
    for e in range(n):
        idx = e * p + np.arange(p + 1)
        D[np.ix_(idx, idx)] += (2.0 / hs[e]) * Dh
        cnt[idx] += 1
    D /= cnt[:, None]
    return D[1:N - 1, 1:N - 1].copy()


def nodal_gradient(mesh: Mesh3D, f: np.ndarray) -> np.ndarray:
    """(N_f, 3) gradient of a nodal field at the free nodes, axis by axis with derivative_1d."""
    n1 = mesh.n1
    D = derivative_1d(mesh)
    T = np.asarray(f, dtype=np.float64).reshape(n1, n1, n1)      # [z, y, x]
    gx = np.einsum("ik,zyk->zyi", D, T)
    gy = np.einsum("ik,zkx->zix", D, T)
    gz = np.einsum("ik,kyx->iyx", D, T)
    return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)


def kinetic_diag(mesh: Mesh3D) -> np.ndarray:
    """Diagonal of K~/2: the preconditioner of Sec. 3.2.2 (inverse diagonal of the
    kinetic, i.e. negative-Laplacian, part)."""
    if hasattr(mesh, "kinetic_diag"):
        return mesh.kinetic_diag()
    m = mesh.m1
    kd = np.diag(m.K1) / m.W1
    md = np.diag(m.Mc) / m.W1
    t = np.kron(md, np.kron(md, kd)) + np.kron(md, np.kron(kd, md)) + np.kron(kd, np.kron(md, md))
    return 0.5 * t


def element_bound(p: int, h: float) -> float:
    """Fried's element eigenvalue bound for K~/2 (Fried 1972).

    lambda_max(K, W) <= max_e lambda_max(K_e, W_e), with K_e the element stiffness
    and W_e the element's own GLL-lumped mass. On the uniform mesh every element
    is the same, so the bound is (1/2) lambda_max(W_e^{-1/2} K_e W_e^{-1/2}).
    """
    Kh, Mh, _, wg = reference_matrices(p)
    Ke1 = (2.0 / h) * Kh
    Me1 = (h / 2.0) * Mh
    We1 = (h / 2.0) * wg
    Ke = np.kron(Me1, np.kron(Me1, Ke1)) + np.kron(Me1, np.kron(Ke1, Me1)) + np.kron(Ke1, np.kron(Me1, Me1))
    We = np.kron(We1, np.kron(We1, We1))
    s = 1.0 / np.sqrt(We)
    return 0.5 * float(np.linalg.eigvalsh(s[:, None] * Ke * s[None, :]).max())
