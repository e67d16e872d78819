"""Thin torch-facing binding of the C ABI (argument marshalling only).

Tensors supply device memory; the current torch stream is passed to every call.
Every computation runs in libinvdft.so; nothing here touches tensor values.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

PREC = {"f64": L.FE_F64, "f32": L.FE_F32, "bf16": L.FE_BF16}
DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}   # bf16: torch's bfloat16 storage


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _host_doubles(vals):
    if vals is None:
        return None
    arr = (C.c_double * len(vals))(*[float(x) for x in vals])
    return arr


def _work(nbytes: int, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Mesh:
    """Spectral-element mesh of [-L, L]^3 with n^3 cells of order p (device tables)."""

    def __init__(self, p: int, n: int, half_width: float, breaks=None, mapped_amp=None):
        """Uniform cells of 2 half_width / n on [-half_width, half_width]^3, or, with ``breaks``
        (n + 1 increasing cell boundaries, the same on every axis), the graded mesh they define,
        or, with ``mapped_amp``, the uniform mesh's nodes moved by the smooth map of the box
        with that amplitude (curved cells, each with its own dense element matrix)."""
        lib = L.load()
        h = C.c_void_p()
        self.mapped_amp = mapped_amp
        if mapped_amp is not None:
            L.check(lib.fe_mesh_create_mapped(int(p), int(n), float(half_width), float(mapped_amp), C.byref(h)),
                    "fe_mesh_create_mapped")
        elif breaks is None:
            L.check(lib.fe_mesh_create(int(p), int(n), float(half_width), C.byref(h)), "fe_mesh_create")
        else:
            breaks = [float(b) for b in breaks]
            n = len(breaks) - 1
            half_width = 0.5 * (breaks[-1] - breaks[0])
            L.check(lib.fe_mesh_create_graded(int(p), n, _host_doubles(breaks), C.byref(h)), "fe_mesh_create_graded")
        self.breaks = breaks
        self._h = h
        self.p, self.n, self.half_width = int(p), int(n), float(half_width)
        nf, nc, npc, kb = C.c_int64(), C.c_int64(), C.c_int(), C.c_double()
        L.check(lib.fe_mesh_info(h, C.byref(nf), C.byref(nc), C.byref(npc), C.byref(kb)), "fe_mesh_info")
        self.n_free, self.n_cells, self.nodes_per_cell, self.kin_bound = nf.value, nc.value, npc.value, kb.value
        self.device = torch.device("cuda", torch.cuda.current_device())

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            L.load().fe_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nodes(self):
        xyz = torch.empty((self.n_free, 3), dtype=torch.float64, device=self.device)
        w = torch.empty(self.n_free, dtype=torch.float64, device=self.device)
        L.check(L.load().fe_mesh_nodes(self._h, _ptr(xyz), _ptr(w), _stream()), "fe_mesh_nodes")
        return xyz, w

    def kinetic_diag(self):
        d = torch.empty(self.n_free, dtype=torch.float64, device=self.device)
        L.check(L.load().fe_mesh_kinetic_diag(self._h, _ptr(d), _stream()), "fe_mesh_kinetic_diag")
        return d

    def workspace_bytes(self, op: int, nv: int, prec: str = "f64") -> int:
        return int(L.load().fe_workspace_bytes(self._h, op, nv, PREC[prec]))


class VxcMesh:
    """Linear tensor mesh of the XC potential (Eq. 14) and its transfer to a Mesh's nodes."""

    def __init__(self, mesh: Mesh, tx, ty=None, tz=None):
        ty = tx if ty is None else ty
        tz = tx if tz is None else tz
        self.vertices = [list(map(float, t)) for t in (tx, ty, tz)]
        h = C.c_void_p()
        ms = [len(t) - 1 for t in self.vertices]
        L.check(L.load().vxc_mesh_create(mesh.handle, ms[0], _host_doubles(self.vertices[0]), ms[1],
                                         _host_doubles(self.vertices[1]), ms[2], _host_doubles(self.vertices[2]),
                                         C.byref(h)), "vxc_mesh_create")
        self._h = h
        self.mesh = mesh
        nv = C.c_int64()
        per = (C.c_int * 3)()
        L.check(L.load().vxc_mesh_info(h, C.byref(nv), per), "vxc_mesh_info")
        self.n_vertices = nv.value
        self.shape = tuple(per)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            L.load().vxc_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prolong(self, u, base=None, out=None):
        """v = base + P u on the orbital nodes."""
        if out is None:
            out = torch.empty(self.mesh.n_free, dtype=torch.float64, device=u.device)
        L.check(L.load().vxc_prolong(self._h, _ptr(u), _ptr(base), _ptr(out), _stream()), "vxc_prolong")
        return out

    def restrict(self, g, out=None):
        """f = P^T g on the vertices."""
        if out is None:
            out = torch.empty(self.n_vertices, dtype=torch.float64, device=g.device)
        L.check(L.load().vxc_restrict(self._h, _ptr(g), _ptr(out), _stream()), "vxc_restrict")
        return out


def ks_apply(mesh: Mesh, v, X, Y=None, shift=None, prec: str = "f64"):
    """Y = H~ X - X diag(shift) (one call of the C ABI)."""
    nv = X.shape[1]
    if Y is None:
        Y = torch.empty_like(X)
    sh = _host_doubles(shift)
    L.check(L.load().ks_apply(mesh.handle, _ptr(v), sh, _ptr(X), _ptr(Y), nv, nv, PREC[prec], _stream()),
            "ks_apply")
    return Y


def cheb_filter(mesh: Mesh, v, degree: int, a: float, b: float, a0: float, X, prec: str = "f64", work=None,
                nv=None):
    """Filters the first nv columns (default: all) of X, whose row pitch is X.shape[1]."""
    ld = X.shape[1]
    nv = ld if nv is None else int(nv)
    if work is None:
        work = _work(mesh.workspace_bytes(L.FE_OP_CHEB_FILTER, ld, prec), X.device)
    L.check(L.load().cheb_filter(mesh.handle, _ptr(v), int(degree), float(a), float(b), float(a0), _ptr(X), nv, ld,
                                 PREC[prec], _ptr(work), _stream()), "cheb_filter")
    return X


def rayleigh_ritz(mesh: Mesh, v, X, work=None, nv=None):
    """Rayleigh-Ritz on the first nv columns (default: all) of X, whose row pitch is X.shape[1]."""
    ld = X.shape[1]
    nv = ld if nv is None else int(nv)
    if work is None:
        work = _work(mesh.workspace_bytes(L.FE_OP_RAYLEIGH_RITZ, ld), X.device)
    eig = (C.c_double * nv)()
    res = (C.c_double * nv)()
    L.check(L.load().rayleigh_ritz(mesh.handle, _ptr(v), _ptr(X), eig, res, nv, ld, _ptr(work), _stream()),
            "rayleigh_ritz")
    return list(eig), list(res)


@dataclass
class EigResult:
    eig: list
    res: list
    passes: int
    status: int
    stage_passes: tuple = (0, 0, 0)      # passes in bf16, FP32, FP64


def ks_eigensolve(mesh: Mesh, v, X, nocc: int, degree: int, tol: float, maxpass: int, prec: str = "f64",
                  switch_tol: float = 1e-5, work=None, allow=(L.FE_ENOCONV, L.FE_EGAP), nv=None) -> EigResult:
    """ChFSI on the first nv columns (default: all) of X, whose row pitch is X.shape[1]."""
    ld = X.shape[1]
    nv = ld if nv is None else int(nv)
    if work is None:
        work = _work(mesh.workspace_bytes(L.FE_OP_EIGENSOLVE, ld, prec), X.device)
    eig = (C.c_double * nv)()
    res = (C.c_double * nv)()
    passes = C.c_int()
    stages = (C.c_int * 3)()
    st = L.load().ks_eigensolve(mesh.handle, _ptr(v), _ptr(X), nv, ld, int(nocc), int(degree), float(tol),
                                int(maxpass), PREC[prec], float(switch_tol), eig, res, C.byref(passes), stages,
                                _ptr(work), _stream())
    L.check(st, "ks_eigensolve", allow=allow)
    return EigResult(list(eig), list(res), passes.value, st, tuple(stages))


@dataclass
class AdjResult:
    iters: list
    relres: list
    status: int


def adjoint_solve(mesh: Mesh, v, Psi, eps, B, Q=None, tol: float = 1e-10, maxit: int = 5000, prec: str = "f64",
                  work=None, allow=(L.FE_ENOCONV,), U=None, theta=None) -> tuple:
    """MINRES adjoint solve; with U (N_f x nbuf) and theta (nbuf values above every shift)
    the deflated preconditioner of ``adjoint_solve_deflated`` is used (FP64 only)."""
    k = Psi.shape[1]
    if Q is None:
        Q = torch.empty_like(B)
    its = (C.c_int * k)()
    rel = (C.c_double * k)()
    if U is not None:
        if prec != "f64":
            raise ValueError("the deflated adjoint solve is FP64 only")
        nb = U.shape[1]
        if work is None:
            work = _work(mesh.workspace_bytes(L.FE_OP_ADJOINT_DEFLATED, k + nb, "f64"), Psi.device)
        st = L.load().adjoint_solve_deflated(mesh.handle, _ptr(v), _ptr(Psi), _host_doubles(eps), k, _ptr(U),
                                             _host_doubles(theta), nb, _ptr(B), _ptr(Q), float(tol), int(maxit), its,
                                             rel, _ptr(work), _stream())
        L.check(st, "adjoint_solve_deflated", allow=allow)
        return Q, AdjResult(list(its), list(rel), st)
    if work is None:
        work = _work(mesh.workspace_bytes(L.FE_OP_ADJOINT_SOLVE, k, prec), Psi.device)
    st = L.load().adjoint_solve(mesh.handle, _ptr(v), _ptr(Psi), _host_doubles(eps), k, _ptr(B), _ptr(Q),
                                float(tol), int(maxit), its, rel, PREC[prec], _ptr(work), _stream())
    L.check(st, "adjoint_solve", allow=allow)
    return Q, AdjResult(list(its), list(rel), st)


def loss_grad(mesh: Mesh, Psi, occ, rho_data, Q=None, tau_bc: float = 0.0, want_rho=True, want_B=True,
              work=None):
    """Phase 1 (Q is None): returns (rho, B, loss). Phase 2: returns grad."""
    k = Psi.shape[1]
    dev = Psi.device
    if work is None:
        work = _work(mesh.workspace_bytes(L.FE_OP_LOSS_GRAD, k), dev)
    lib = L.load()
    occ_h = _host_doubles(occ)
    if Q is None:
        rho = torch.empty(mesh.n_free, dtype=torch.float64, device=dev) if want_rho else None
        B = torch.empty_like(Psi) if want_B else None
        loss = C.c_double()
        L.check(lib.loss_grad(mesh.handle, _ptr(Psi), occ_h, k, _ptr(rho_data), None, 0.0, _ptr(rho), _ptr(B), None,
                              C.byref(loss), _ptr(work), _stream()), "loss_grad")
        return rho, B, loss.value
    g = torch.empty(mesh.n_free, dtype=torch.float64, device=dev)
    L.check(lib.loss_grad(mesh.handle, _ptr(Psi), occ_h, k, _ptr(rho_data), _ptr(Q), float(tau_bc), None, None,
                          _ptr(g), None, _ptr(work), _stream()), "loss_grad")
    return g


def dot(x, y, work=None) -> float:
    if work is None:
        work = _work(65536, x.device)
    out = C.c_double()
    L.check(L.load().fe_dot(_ptr(x), _ptr(y), x.numel(), C.byref(out), _ptr(work), _stream()), "fe_dot")
    return out.value


def axpby(alpha: float, x, beta: float, y):
    L.check(L.load().fe_axpby(float(alpha), _ptr(x), float(beta), _ptr(y), x.numel(), _stream()), "fe_axpby")
    return y


def apply_timing(enable: bool):
    """Start (True: clears the record) or stop recording HIP-event timings of every operator apply."""
    L.check(L.load().fe_apply_timing(1 if enable else 0), "fe_apply_timing")


def apply_timing_read(prec: str = "f64"):
    """(launches, total ms, total algorithmic bytes, total columns) of the recorded applies in
    precision prec."""
    n, ms, b = C.c_int64(), C.c_double(), C.c_double()
    cols = C.c_double()
    L.check(L.load().fe_apply_timing_read(PREC[prec], C.byref(n), C.byref(ms), C.byref(b), C.byref(cols)),
            "fe_apply_timing_read")
    return n.value, ms.value, b.value, cols.value


def sweep_timing_read(pass_: str = "A"):
    """(launches, total ms, total algorithmic bytes, total active columns) of the recorded MINRES
    passes A, B or C."""
    n, ms, b, cols = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
    L.check(L.load().fe_sweep_timing_read("ABC".index(pass_), C.byref(n), C.byref(ms), C.byref(b), C.byref(cols)),
            "fe_sweep_timing_read")
    return n.value, ms.value, b.value, cols.value


@dataclass
class Occupations:
    occ: list
    dfde: list
    mu: float
    n_incl: int
    status: int


def fermi_occupations(eig, n_elec: float, kT: float, smax: float = 2.0, occ_cut: float = 1e-12,
                      allow=()) -> Occupations:
    """Fermi-Dirac occupations of the given eigenvalues and mu from the electron count (host call)."""
    n = len(eig)
    occ = (C.c_double * n)()
    dfde = (C.c_double * n)()
    mu = C.c_double()
    ninc = C.c_int()
    st = L.load().fermi_occupations(_host_doubles(eig), n, float(n_elec), float(kT), float(smax), float(occ_cut),
                                    occ, dfde, C.byref(mu), C.byref(ninc))
    L.check(st, "fermi_occupations", allow=allow)
    return Occupations(list(occ), list(dfde), mu.value, ninc.value, st)


def adjoint_along_psi(mesh: Mesh, Psi, eps, mu: float, kT: float, rho, rho_data, Q, smax: float = 2.0,
                      work=None):
    """Q <- Q + Psi C (the in-span part of the finite-temperature adjoint). Returns (eta, C as a list)."""
    n = Psi.shape[1]
    if work is None:
        work = _work(mesh.workspace_bytes(L.FE_OP_ALONG_PSI, n), Psi.device)
    eta = C.c_double()
    Ch = (C.c_double * (n * n))()
    L.check(L.load().adjoint_along_psi(mesh.handle, _ptr(Psi), n, _host_doubles(eps), float(mu), float(kT),
                                       float(smax), _ptr(rho), _ptr(rho_data), _ptr(Q), C.byref(eta), Ch,
                                       _ptr(work), _stream()), "adjoint_along_psi")
    return eta.value, list(Ch)


@dataclass
class PoissonResult:
    iters: int
    relres: float
    charge: float
    status: int


def poisson_solve(mesh: Mesh, rho, sigma: float = 1.0, tol: float = 1e-12, maxit: int = 20000, phi=None,
                  work=None, allow=()) -> tuple:
    """Hartree potential of rho on the mesh's free nodes (monopole split off with width sigma)."""
    if phi is None:
        phi = torch.empty_like(rho)
    if work is None:
        work = _work(mesh.workspace_bytes(L.FE_OP_POISSON, 1), rho.device)
    it, rel, q = C.c_int(), C.c_double(), C.c_double()
    st = L.load().poisson_solve(mesh.handle, _ptr(rho), float(sigma), _ptr(phi), float(tol), int(maxit),
                                C.byref(it), C.byref(rel), C.byref(q), _ptr(work), _stream())
    L.check(st, "poisson_solve", allow=allow)
    return phi, PoissonResult(it.value, rel.value, q.value, st)


def xc_initial_guess(mesh: Mesh, rho, v_h, n_elec: float, tau: float = 1e-2, alpha: float = 1.0,
                     exchange: str = "lb94", out=None):
    """Eq. 25: (Slater or LB94) exchange + PW92 correlation, Fermi-Amaldi tail."""
    if out is None:
        out = torch.empty_like(rho)
    ex = {"slater": L.FE_XC_SLATER, "lb94": L.FE_XC_LB94}[exchange]
    work = _work(8 * mesh.n, rho.device) if ex == L.FE_XC_LB94 else None
    L.check(L.load().xc_initial_guess(mesh.handle, _ptr(rho), _ptr(v_h), float(n_elec), float(tau), float(alpha), ex,
                                      _ptr(out), _ptr(work), _stream()), "xc_initial_guess")
    return out
