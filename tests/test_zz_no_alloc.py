"""loss_grad_noalloc (fixed device scratch, no allocation) against loss_grad (caller's work buffer).

Both run the same kernels over the same inputs, so every output must agree bit for bit.
Two calls in a row, the second on a smaller mesh and fewer columns, so that the second one
runs over what the first left in the shared scratch array.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2510_10529_amd import _lib as L
from paper_2510_10529_amd import api
from synth import random_block

pytestmark = pytest.mark.gpu


def _inputs(mesh, nocc, seed):
    dev = torch.device("cuda", 0)
    Psi = torch.tensor(random_block(mesh.n_free, nocc, seed) * 0.05, device=dev)
    rng = np.random.default_rng(seed + 1)
    rho_d = torch.tensor(rng.uniform(0.0, 0.2, mesh.n_free), device=dev)
    Q = torch.tensor(random_block(mesh.n_free, nocc, seed + 2), device=dev)
    occ = [2.0] * (nocc - 1) + [1.25]
    return Psi, rho_d, Q, occ


def _run_both(mesh, nocc, seed, tau_bc):
    lib = L.load()
    Psi, rho_d, Q, occ = _inputs(mesh, nocc, seed)
    occ_h = api._host_doubles(occ)
    st = api._stream()
    work = api._work(mesh.workspace_bytes(L.FE_OP_LOSS_GRAD, nocc), Psi.device)
    out = {}
    for name in ("ref", "noalloc"):
        rho = torch.full((mesh.n_free,), np.nan, dtype=torch.float64, device=Psi.device)
        B = torch.full_like(Psi, np.nan)
        g = torch.full((mesh.n_free,), np.nan, dtype=torch.float64, device=Psi.device)
        loss1, loss2 = C.c_double(), C.c_double()
        if name == "ref":
            s1 = lib.loss_grad(mesh.handle, api._ptr(Psi), occ_h, nocc, api._ptr(rho_d), None, 0.0, api._ptr(rho),
                               api._ptr(B), None, C.byref(loss1), api._ptr(work), st)
            s2 = lib.loss_grad(mesh.handle, api._ptr(Psi), occ_h, nocc, api._ptr(rho_d), api._ptr(Q), tau_bc,
                               api._ptr(rho), None, api._ptr(g), C.byref(loss2), api._ptr(work), st)
        else:
            s1 = lib.loss_grad_noalloc(mesh.handle, api._ptr(Psi), occ_h, nocc, api._ptr(rho_d), None, 0.0,
                                       api._ptr(rho), api._ptr(B), None, C.byref(loss1), st)
            s2 = lib.loss_grad_noalloc(mesh.handle, api._ptr(Psi), occ_h, nocc, api._ptr(rho_d), api._ptr(Q), tau_bc,
                                       api._ptr(rho), None, api._ptr(g), C.byref(loss2), st)
        assert s1 == L.FE_OK and s2 == L.FE_OK, (name, s1, s2, lib.fe_last_error())
        torch.cuda.synchronize()
        out[name] = (rho.cpu(), B.cpu(), g.cpu(), loss1.value, loss2.value)
    return out


def _check_equal(out):
    ref, na = out["ref"], out["noalloc"]
    for k, what in enumerate(("rho", "B", "grad")):
        assert torch.isfinite(ref[k]).all(), what
        assert torch.equal(ref[k], na[k]), (what, float((ref[k] - na[k]).abs().max()))
    assert ref[3] == na[3] and ref[4] == na[4], (ref[3:], na[3:])
    assert ref[3] > 0.0


def test_noalloc_matches_loss_grad_twice_second_smaller():
    torch.cuda.set_device(0)
    print("case: p=4 n=24 nocc=50 (857,375 nodes), then p=2 n=5 nocc=5", flush=True)
    big = api.Mesh(4, 24, 12.0)
    out = _run_both(big, 50, 11, tau_bc=0.05)
    _check_equal(out)
    assert (out["ref"][2] == 0).any()  # the far-field mask was active
    big.close()
    small = api.Mesh(2, 5, 4.0)
    _check_equal(_run_both(small, 5, 23, tau_bc=0.0))
    small.close()


def test_noalloc_rejects_what_it_cannot_do():
    torch.cuda.set_device(0)
    lib = L.load()
    mesh = api.Mesh(2, 4, 3.0)
    Psi, rho_d, Q, occ = _inputs(mesh, 4, 5)
    occ_h = api._host_doubles(occ)
    B = torch.empty_like(Psi)
    # phase 1 without a density output: this variant has no buffer of its own for it
    st = lib.loss_grad_noalloc(mesh.handle, api._ptr(Psi), occ_h, 4, api._ptr(rho_d), None, 0.0, None,
                               api._ptr(B), None, None, api._stream())
    assert st == L.FE_EINVAL and b"needs rho" in lib.fe_last_error()
    st = lib.loss_grad_noalloc(mesh.handle, api._ptr(Psi), api._host_doubles([2.0] * 65), 65, api._ptr(rho_d), None,
                               0.0, None, None, None, None, api._stream())
    assert st == L.FE_EINVAL
    # the fixed array covers the widest block on the largest mesh the gram partials can use
    need = mesh.workspace_bytes(L.FE_OP_LOSS_GRAD, 64) - 8 * mesh.n_free
    assert lib.loss_grad_noalloc_max_bytes() >= need
    mesh.close()
