"""Inverse-DFT driver: the loss L(u) as a torch.autograd.Function whose backward
is the adjoint solve, and an L-BFGS loop on the nodal XC potential u (Eq. 21).

Forward (Sec. 3.2.2): v = v_fixed + u; Chebyshev-filtered subspace iteration to
the residual tolerance; density, loss and adjoint right-hand side (Eqs. 1, 4, 7).
Backward: optionally recompute the orbitals (from the warm-start block, so they
need not be kept between forward and backward), solve the adjoint equations by
batched projected MINRES (Eq. 20) and form g_b = sum_i psi_{b,i} q_{b,i} (Eq. 22).

XC potential on its own linear mesh (a VxcMesh, Eq. 14): u holds its vertex values,
v = v_fixed + P u, and the gradient is P^T g (Eq. 22's integral against the linear
hat functions, by the orbital mesh's quadrature).

Finite temperature (kT > 0): the occupations are Fermi-Dirac with mu from the
electron count (Eqs. 4, 5); every orbital with f_i above a cut enters the density
and the adjoint, and the adjoint functions gain their component along the included
orbitals (Eqs. 8, 9) before the gradient of Eq. 10 is formed.

Every operation on device vectors is a call into libinvdft.so; torch supplies the
buffers and the stream.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import torch

from . import _lib as L
from . import api


@dataclass
class SolverOptions:
    degree: int = 40                 # Chebyshev filter degree
    tol_eig: float = 1e-9            # max residual of the occupied Ritz pairs
    tol_adj: float = 1e-10           # relative residual of every adjoint column
    maxpass: int = 200
    maxit_adj: int = 20000
    filter_prec: str = "f64"         # "f64" | "f32"
    adjoint_prec: str = "f64"        # "f64" | "f32" (FP32 MINRES + FP64 refinement)
    switch_tol: float = 1e-4         # reduced-precision filter until the residual is below this
    recompute: bool = False          # recompute orbitals in backward instead of keeping them
    tau_bc: float = 0.0
    adaptive: bool = False           # t_eig = e_L2^2 / c_eig, t_ad = e_L2^2 / c_ad (Table 1 defaults)
    c_eig: float = 1e2
    c_ad: float = 1e5
    kT: float = 0.0                  # k_B T in Ha; 0 = doubly occupied lowest N_e/2 orbitals
    smax: float = 2.0                # occupancy of a full orbital (spin-restricted)
    n_states: int = 0                # finite T: Ritz pairs to converge (0 = block width - 4)
    occ_cut: float = 1e-12           # finite T: orbitals with f_i <= occ_cut * smax are left out
    deflate: int = 0                 # FP64 adjoint: Ritz vectors above the included orbitals that
                                     # deflate its preconditioner (0 = plain diagonal preconditioner)
    deflate_split: bool = False      # also deflate beyond 64 columns of [Psi U] (separate sweeps:
                                     # fewer MINRES iterations, each dearer); else at most 64 - n


@dataclass
class OccState:
    """Occupations of one forward solve: the first n orbitals enter."""
    n: int
    occ: list
    eig: list
    mu: float | None = None          # None at T = 0
    U: object = None                 # deflation block of the adjoint (N_f x nb copy) or None
    theta: list | None = None        # its Ritz values


@dataclass
class Stats:
    passes: list = field(default_factory=list)
    adj_iters: list = field(default_factory=list)
    t_forward: float = 0.0
    t_adjoint: float = 0.0
    n_forward: int = 0
    n_backward: int = 0


class InverseProblem:
    """One inverse-DFT problem on one GPU: mesh, fixed potential, target density."""

    def __init__(self, mesh: api.Mesh, v_fixed: torch.Tensor, rho_data: torch.Tensor, n_elec: int,
                 X0: torch.Tensor, opts: SolverOptions | None = None, vxc: api.VxcMesh | None = None):
        self.mesh = mesh
        self.vxc = vxc                         # None: u is nodal on the orbital mesh
        self.v_fixed = v_fixed
        self.rho_data = rho_data
        self.n_elec = n_elec
        self.opts = opts or SolverOptions()
        self.nv = X0.shape[1]
        o = self.opts
        if o.kT > 0:
            self.nconv = o.n_states or self.nv - 4     # Ritz pairs the eigensolver converges
            if not 0 < self.nconv < self.nv:
                raise ValueError("finite temperature needs 0 < n_states < block width")
        else:
            if n_elec != int(n_elec):
                raise ValueError("zero temperature needs an integer electron count")
            self.nconv = int(n_elec) // 2
        self.nocc = self.nconv                 # widest block of orbitals that can enter
        n0 = int(n_elec) // 2                  # placeholder until the first eigensolve
        self.state = OccState(n0, [2.0] * n0, [])
        self.X = X0.clone()                    # FP64 warm-start block (Ritz vectors)
        self.v = torch.empty_like(v_fixed)
        self.eig = None
        self.stats = Stats()
        dev = X0.device
        self.work_eig = api._work(mesh.workspace_bytes(L.FE_OP_EIGENSOLVE, self.nv, o.filter_prec), dev)
        if o.deflate > 0:
            if o.adjoint_prec != "f64":
                raise ValueError("the deflated adjoint solve is FP64 only")
            # deflation with at most 64 orbitals and 64 deflation vectors; the plain solve (more
            # orbitals, or no deflation vector clearing the shifts) in the same buffer
            need = mesh.workspace_bytes(L.FE_OP_ADJOINT_SOLVE, self.nocc, "f64")
            if self.nocc <= 64:
                need = max(need, mesh.workspace_bytes(L.FE_OP_ADJOINT_DEFLATED,
                                                      self.nocc + min(64, o.deflate), "f64"))
            self.work_adj = api._work(need, dev)
        else:
            self.work_adj = api._work(mesh.workspace_bytes(L.FE_OP_ADJOINT_SOLVE, self.nocc, o.adjoint_prec), dev)
        self.work_lg = api._work(mesh.workspace_bytes(L.FE_OP_LOSS_GRAD, self.nocc), dev)
        self.work_ap = (api._work(mesh.workspace_bytes(L.FE_OP_ALONG_PSI, self.nocc), dev) if o.kT > 0 else None)
        self.last_loss = None

    # ------------------------------------------------------------------ pieces
    def set_potential(self, u: torch.Tensor):
        if self.vxc is not None:
            self.vxc.prolong(u, base=self.v_fixed, out=self.v)     # v = v_fixed + P u
            return
        self.v.copy_(self.v_fixed)                  # device copy
        api.axpby(1.0, u, 1.0, self.v)              # v = v_fixed + u

    def zeros_u(self):
        """A zero potential update in the unknowns u lives in."""
        n = self.vxc.n_vertices if self.vxc is not None else self.mesh.n_free
        return torch.zeros(n, dtype=torch.float64, device=self.v_fixed.device)

    def tolerances(self):
        o = self.opts
        if o.adaptive and self.last_loss is not None:
            e2 = self.last_loss
            return max(min(o.tol_eig, e2 / o.c_eig), 1e-12), max(min(o.tol_adj, e2 / o.c_ad), 1e-13)
        return o.tol_eig, o.tol_adj

    def eigensolve(self, tol_eig):
        o = self.opts
        t0 = time.perf_counter()
        r = api.ks_eigensolve(self.mesh, self.v, self.X, self.nconv, o.degree, tol_eig, o.maxpass,
                              prec=o.filter_prec, switch_tol=o.switch_tol, work=self.work_eig)
        # at finite temperature the eigensolver's gap test at nconv has no meaning
        ok = (L.FE_OK, L.FE_EGAP) if o.kT > 0 else (L.FE_OK,)
        if r.status not in ok:
            raise L.FEError(r.status, "ks_eigensolve")
        self.eig = r.eig
        if o.kT > 0:
            oc = api.fermi_occupations(r.eig[:self.nconv], self.n_elec, o.kT, o.smax, o.occ_cut)
            self.state = OccState(oc.n_incl, oc.occ[:oc.n_incl], r.eig[:oc.n_incl], oc.mu)
        else:
            self.state = OccState(self.nconv, [2.0] * self.nconv, r.eig[:self.nconv])
        if o.deflate > 0:
            self._deflation_block(r.eig)
        torch.cuda.current_stream().synchronize()
        self.stats.t_forward += time.perf_counter() - t0
        self.stats.passes.append(r.passes)
        self.stats.n_forward += 1
        return r

    def _deflation_block(self, eig):
        """The Ritz pairs above the included orbitals whose values clear every shift: a copy,
        so that the next eigensolve may overwrite the block before the adjoint runs."""
        st = self.state
        top = max(st.eig)
        j0 = st.n
        while j0 < self.nv and eig[j0] <= top + 1e-8 * max(1.0, abs(top)):
            j0 += 1                                  # degenerate with an included orbital
        nb = min(self.opts.deflate, self.nv - j0, 64 if self.opts.deflate_split else 64 - st.n)
        if nb >= 1 and st.n <= 64:
            st.U = self.X[:, j0:j0 + nb].contiguous()
            st.theta = list(eig[j0:j0 + nb])

    def psi(self):
        return self.X[:, :self.state.n].contiguous()

    def loss_and_rhs(self, Psi):
        rho, B, loss = api.loss_grad(self.mesh, Psi, self.state.occ, self.rho_data, work=self.work_lg)
        self.last_loss = loss
        return rho, B, loss

    def gradient(self, Psi, B, rho=None, state: OccState | None = None):
        """dL/du from the orbitals, the adjoint right-hand sides and (finite T) the density."""
        o = self.opts
        st = state or self.state
        _, tol_adj = self.tolerances()
        t0 = time.perf_counter()
        Q, ar = api.adjoint_solve(self.mesh, self.v, Psi, st.eig, B, tol=tol_adj,
                                  maxit=o.maxit_adj, prec=o.adjoint_prec, work=self.work_adj,
                                  U=st.U, theta=st.theta)
        if o.kT > 0:
            api.adjoint_along_psi(self.mesh, Psi, st.eig, st.mu, o.kT, rho, self.rho_data, Q, smax=o.smax,
                                  work=self.work_ap)
        g = api.loss_grad(self.mesh, Psi, st.occ, self.rho_data, Q=Q, tau_bc=o.tau_bc, work=self.work_lg)
        if self.vxc is not None:
            g = self.vxc.restrict(g)                                 # f = P^T g
        torch.cuda.current_stream().synchronize()
        self.stats.t_adjoint += time.perf_counter() - t0
        self.stats.adj_iters.append(max(ar.iters))
        self.stats.n_backward += 1
        if ar.status != L.FE_OK:
            raise L.FEError(ar.status, "adjoint_solve")
        return g

    def evaluate(self, u: torch.Tensor, want_grad=True):
        """L(u) and dL/du, without autograd."""
        self.set_potential(u)
        tol_eig, _ = self.tolerances()
        self.eigensolve(tol_eig)
        Psi = self.psi()
        rho, B, loss = self.loss_and_rhs(Psi)
        if not want_grad:
            return loss, None
        return loss, self.gradient(Psi, B, rho)


class InvDFTLoss(torch.autograd.Function):
    """L(u) with the adjoint solve as its hand-written backward (Eqs. 7, 11, 20, 22)."""

    @staticmethod
    def forward(ctx, u, prob: InverseProblem):
        prob.set_potential(u)
        tol_eig, _ = prob.tolerances()
        prob.eigensolve(tol_eig)
        Psi = prob.psi()
        rho, B, loss = prob.loss_and_rhs(Psi)
        ctx.prob = prob
        ctx.state = prob.state
        if prob.opts.recompute:
            ctx.save_for_backward(u)               # orbitals are recomputed in backward
        else:
            ctx.save_for_backward(u, Psi, B, rho)
        return torch.tensor(loss, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(ctx, gL):
        prob = ctx.prob
        if prob.opts.recompute:
            (u,) = ctx.saved_tensors
            prob.set_potential(u)
            tol_eig, _ = prob.tolerances()
            prob.eigensolve(tol_eig)             # warm block is already converged: ~1 pass
            Psi = prob.psi()
            rho, B, _ = prob.loss_and_rhs(Psi)
            state = prob.state
        else:
            u, Psi, B, rho = ctx.saved_tensors
            state = ctx.state
        g = prob.gradient(Psi, B, rho, state)
        api.axpby(0.0, g, float(gL), g)            # g <- gL * g
        return g, None


def lbfgs(prob: InverseProblem, u0: torch.Tensor, maxiter: int = 30, history: int = 10,
          callback=None, use_autograd: bool = True):
    """L-BFGS (Nocedal 1980; Eq. 21) with Armijo backtracking, on device vectors.

    The two-loop recursion and every vector update run through fe_dot / fe_axpby.
    Returns (u, list of losses).
    """
    work = api._work(65536, u0.device)
    u = u0.clone()

    def fg(x):
        if use_autograd:
            xr = x.detach().clone().requires_grad_(True)
            loss = InvDFTLoss.apply(xr, prob)
            loss.backward()
            return float(loss), xr.grad.detach()
        return prob.evaluate(x)

    f, g = fg(u)
    S, Yh, RHO = [], [], []
    losses = [f]
    d = torch.empty_like(u)
    u_new = torch.empty_like(u)
    for it in range(maxiter):
        # two-loop recursion: d = -H g
        d.copy_(g)
        alphas = []
        for s, y, rho in zip(reversed(S), reversed(Yh), reversed(RHO)):
            a = rho * api.dot(s, d, work)
            api.axpby(-a, y, 1.0, d)
            alphas.append(a)
        if S:
            gamma = api.dot(S[-1], Yh[-1], work) / api.dot(Yh[-1], Yh[-1], work)
        else:
            gamma = 1.0 / math.sqrt(max(api.dot(g, g, work), 1e-300))
        api.axpby(0.0, d, gamma, d)
        for (s, y, rho), a in zip(zip(S, Yh, RHO), reversed(alphas)):
            b = rho * api.dot(y, d, work)
            api.axpby(a - b, s, 1.0, d)
        api.axpby(0.0, d, -1.0, d)
        gd = api.dot(g, d, work)
        if gd >= 0:                                 # not a descent direction: restart
            S.clear(); Yh.clear(); RHO.clear()
            d.copy_(g)
            api.axpby(0.0, d, -1.0 / math.sqrt(max(api.dot(g, g, work), 1e-300)), d)
            gd = api.dot(g, d, work)
        step = 1.0
        for _ in range(20):
            u_new.copy_(u)
            api.axpby(step, d, 1.0, u_new)
            f_new, g_new = fg(u_new)
            if f_new <= f + 1e-4 * step * gd:
                break
            step *= 0.5
        s = u_new.clone()
        api.axpby(-1.0, u, 1.0, s)
        y = g_new.clone()
        api.axpby(-1.0, g, 1.0, y)
        sy = api.dot(s, y, work)
        if sy > 1e-300:
            S.append(s); Yh.append(y); RHO.append(1.0 / sy)
            if len(S) > history:
                S.pop(0); Yh.pop(0); RHO.pop(0)
        u.copy_(u_new)
        f, g = f_new, g_new
        losses.append(f)
        if callback:
            callback(it, f, u)
    return u, losses
