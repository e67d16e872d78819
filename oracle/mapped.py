"""Spectral elements on a smoothly mapped hexahedral mesh: every cell its own dense
element stiffness (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's orbital meshes are adaptive and unstructured in the cell sizes (Sec. 3.2.3,
Sec. 4, Fig. 6), so every cell carries its own element matrix and the operator is a
batched product of dense per-cell matrices with gather and scatter (Sec. 3.2.3). Cells
whose shape is not a product of 1-D intervals need exactly that. This module builds such
a mesh by mapping the uniform mesh of [-L, L]^3 through a smooth map Phi of the box onto
itself and computes the per-cell matrices from their definition:

* Geometry (isoparametric): the nodes are Phi of the uniform mesh's GLL nodes (Eq. 12's
  tensor basis on the reference cell [-1, 1]^3), and a cell's shape is the order-p
  interpolant of its node coordinates, x(xi) = sum_a x_a N_a(xi).
* Stiffness (Eq. 17): K_e(a, b) = int_cell grad N_a . grad N_b dx
  = sum_q w_q grad^N_a(q)^T G(q) grad^N_b(q), G = |det J| J^{-1} J^{-T}, J = dx/dxi,
  by Gauss-Legendre quadrature with q_K = ceil((3p + 1)/2) points per axis. With that
  many points the quadrature of grad N_a . c |det J| (a polynomial) is exact, so the
  discrete operator annihilates every linear field at every free node (the patch test).
* Overlap lumped by GLL quadrature at the nodes (Sec. 3.2.1): W_a = sum over the cells
  holding a of w^_i w^_j w^_k |det J(node)|.
* Standard form (Eq. 19): H~ = (1/2) W^{-1/2} K W^{-1/2} + diag(v) on the free nodes
  (homogeneous Dirichlet on the box faces), the same node numbering as the uniform mesh.

The map used by the library's mapped meshes (``warp``) moves every coordinate by a
product of sines that vanishes on the faces it must keep:
  Phi_d(xi) = xi_d + amp (L / pi) sin(pi xi_d / L) sin(pi xi_{d+1} / L), d + 1 cyclic,
which maps each face of the box into itself. Other maps (an affine shear for the closed
form) can be passed as a callable.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import fe


def warp(xi: np.ndarray, L: float, amp: float) -> np.ndarray:
    """Phi of the module docstring at points xi (N x 3)."""
    xi = np.asarray(xi, dtype=np.float64)
    s = np.sin(np.pi * xi / L)
    out = xi.copy()
    for d in range(3):
        out[:, d] += amp * (L / np.pi) * s[:, d] * s[:, (d + 1) % 3]
    return out


def metric(J: np.ndarray) -> np.ndarray:
    """G = |det J| J^{-1} J^{-T} for Jacobians J[..., c, d] = dx_c / dxi_d: with it,
    grad N_a . grad N_b |det J| = grad^N_a^T G grad^N_b (chain rule, grad = J^{-T} grad^)."""
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("mapped mesh: a cell is inverted (det J <= 0 at a quadrature point)")
    Jinv = np.linalg.inv(J)                            # [..., d, c] = dxi_d / dx_c
    return np.einsum("...dc,...fc->...df", Jinv, Jinv) * det[..., None, None]


def node_volume(J: np.ndarray) -> np.ndarray:
    """|det J|: the volume factor of the GLL quadrature weight at a node."""
    return np.abs(np.linalg.det(J))


def quad_points(p: int) -> int:
    """Gauss points per axis for the element stiffness: ceil((3p + 1)/2)."""
    return int(math.ceil((3 * p + 1) / 2.0))


class MappedMesh:
    """Order-p cells of the uniform n^3 mesh of [-L, L]^3, mapped by ``phi``."""

    def __init__(self, p: int, n: int, L: float, phi):
        self.p, self.n, self.L = p, n, float(L)
        m1 = fe.mesh1d(p, n, L)
        t = m1.x_all                                  # reference 1-D node coordinates, pn + 1
        N = p * n + 1
        Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
        ref = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)     # all nodes, x fastest
        self.x_all = phi(ref)                          # (N^3, 3) physical node coordinates
        self.N = N
        P1 = p + 1
        g = np.arange(N)
        free1 = (g >= 1) & (g <= N - 2)
        self.free_all = np.kron(free1, np.kron(free1, free1)).astype(bool)  # over all nodes, x fastest
        self.n1 = N - 2
        # local node (i, j, k) of cell (ex, ey, ez) -> global node, x fastest in both
        loc = np.arange(P1)
        li, lj, lk = np.meshgrid(loc, loc, loc, indexing="ij")
        li, lj, lk = lk.ravel(), lj.ravel(), li.ravel()  # local index a = i + P1 (j + P1 k)
        cells = []
        for ez in range(n):
            for ey in range(n):
                for ex in range(n):
                    gx, gy, gz = ex * p + li, ey * p + lj, ez * p + lk
                    cells.append(gx + N * (gy + N * gz))
        self.cell_nodes = np.array(cells)              # (n^3, P1^3), cell index x fastest
        self._build()

    # ------------------------------------------------------------------ tables
    def _build(self):
        p = self.p
        P1 = p + 1
        xi, wg = fe.gll_nodes_weights(p)
        q = quad_points(p)
        xq, wq = fe.gauss_nodes_weights(q)
        B = fe.lagrange_values(xi, xq)                 # B[q, i] = N_i(x_q)
        D = fe.lagrange_derivs(xi, xq)                 # D[q, i] = N_i'(x_q)
        # reference gradients of the P1^3 basis functions at the q^3 points (rows qz, qy, qx)
        G = np.stack([np.kron(B, np.kron(B, D)), np.kron(B, np.kron(D, B)), np.kron(D, np.kron(B, B))])
        w3 = np.kron(wq, np.kron(wq, wq))
        Xe = self.x_all[self.cell_nodes]                # (n_c, n_p, 3)
        J = np.einsum("dqa,eac->eqcd", G, Xe)          # J[e, q, c, d] = dx_c / dxi_d
        Gm = metric(J)                                 # (n_c, q^3, 3, 3)
        # K_e(a, b) = sum_q w_q sum_{d,f} G[d, q, a] Gm[e, q, d, f] G[f, q, b], as two batched products
        T = np.matmul(Gm, np.transpose(G, (1, 0, 2))[None])          # (n_c, q^3, 3, n_p): Gm grad^N_b
        Gw = (G * w3[None, :, None]).transpose(1, 0, 2).reshape(-1, G.shape[2])   # rows (q, d)
        self.Ke = np.matmul(Gw.T[None], T.reshape(T.shape[0], -1, T.shape[3]))   # (n_c, n_p, n_p)
        # lumped mass: |det J| at the GLL nodes (the interpolant's derivative there)
        Dg = fe.lagrange_derivs(xi, xi)                # Dg[j, i] = N_i'(xi_j)
        I = np.eye(P1)
        Gg = np.stack([np.kron(I, np.kron(I, Dg)), np.kron(I, np.kron(Dg, I)), np.kron(Dg, np.kron(I, I))])
        Jg = np.einsum("dqa,eac->eqcd", Gg, Xe)
        self.We = np.kron(wg, np.kron(wg, wg))[None, :] * node_volume(Jg)   # (n_c, n_p) element lumped mass
        W_all = np.zeros(self.N ** 3)
        np.add.at(W_all, self.cell_nodes.ravel(), self.We.ravel())
        self.W_all = W_all
        # assembled stiffness over all nodes
        nc, npc = self.cell_nodes.shape
        rows = np.repeat(self.cell_nodes, npc, axis=1).ravel()
        cols = np.tile(self.cell_nodes, (1, npc)).ravel()
        self.K_all = sp.csr_matrix((self.Ke.ravel(), (rows, cols)), shape=(self.N ** 3, self.N ** 3))
        f = np.nonzero(self.free_all)[0]
        self.free_idx = f
        self.K = self.K_all[f][:, f].tocsr()
        self._W = W_all[f]

    # ------------------------------------------------------------- interface
    @property
    def n_free(self) -> int:
        return self.free_idx.size

    def coords(self) -> np.ndarray:
        """Free-node coordinates (N_f, 3), x fastest (the uniform mesh's numbering)."""
        return self.x_all[self.free_idx]

    def weights(self) -> np.ndarray:
        return self._W

    def kinetic_csr(self) -> sp.csr_matrix:
        """K~/2 = (1/2) W^{-1/2} K W^{-1/2} on the free nodes (Eq. 19)."""
        s = sp.diags(1.0 / np.sqrt(self._W))
        return (0.5 * (s @ self.K @ s)).tocsr()

    def kinetic_diag(self) -> np.ndarray:
        """diag(K~/2): the MINRES preconditioner's diagonal (Sec. 3.2.2)."""
        return 0.5 * self.K.diagonal() / self._W

    def element_bound(self) -> float:
        """max over cells of (1/2) lambda_max(W_e^{-1/2} K_e W_e^{-1/2}) with the cell's own
        lumped mass W_e (Fried 1972): an upper bound of lambda_max(K~/2)."""
        best = 0.0
        for Ke, We in zip(self.Ke, self.We):
            s = 1.0 / np.sqrt(We)
            best = max(best, float(np.linalg.eigvalsh(s[:, None] * Ke * s[None, :]).max()))
        return 0.5 * best

    def scaled_cell_matrices(self) -> np.ndarray:
        """K~_e = (1/2) W^{-1/2} K_e W^{-1/2} with the assembled W at the cell's nodes
        (zero rows and columns at Dirichlet nodes): the dense per-cell matrices of Sec. 3.2.3
        whose gathered products, scattered and summed, give K~/2 on the free nodes."""
        s = np.where(self.free_all, 1.0 / np.sqrt(np.where(self.W_all > 0, self.W_all, 1.0)), 0.0)
        sc = s[self.cell_nodes]                        # (n_c, n_p)
        return 0.5 * sc[:, :, None] * self.Ke * sc[:, None, :]


def mapped_mesh(p: int, n: int, L: float, amp: float) -> MappedMesh:
    """The library's mapped mesh: the uniform mesh warped by ``warp`` with amplitude amp."""
    return MappedMesh(p, n, L, lambda xi: warp(xi, L, amp))
