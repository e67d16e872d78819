"""Mapped meshes (per-cell dense element matrices) against the oracle (needs an MI355X).

The library builds every cell's matrix on the device and applies the operator as batched
dense cell products with gather and scatter (Sec. 3.2.3); the oracle assembles the same
matrices in NumPy (oracle/mapped.py, pinned by the patch test, a closed-form energy on a
sheared box and the identity map). Checked here:
  * node coordinates, lumped weights, the kinetic diagonal and Fried's bound, p = 1..5;
  * ks_apply in FP64 (1e-13 relative: dense products in FP64) and FP32 (2e-6: FP32
    storage of the matrices and the block, FP64 accumulation) for p = 1..5 and ragged
    column counts, with per-column shifts; bitwise reproducibility;
  * the identity map against the uniform mesh's sum-factorised kernel;
  * the chain eigensolve -> density -> loss -> adjoint -> gradient against the oracle's
    dense solve and bordered adjoint (eigenvalues 1e-8 Ha, density L1 1e-7, gradient 1e-6);
  * the calls that do not take mapped meshes refuse them.
"""
import ctypes as C
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fe, ks, mapped  # noqa: E402
from synth import random_block, workload  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
AMP = 0.2


@functools.lru_cache(maxsize=8)
def _pair(p, n, L, amp=AMP):
    from paper_2510_10529_amd import api
    return api.Mesh(p, n, L, mapped_amp=amp), mapped.mapped_mesh(p, n, L, amp)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_mesh_tables(p):
    from paper_2510_10529_amd import api  # noqa: F401
    n = 4 if p <= 2 else 2
    m, om = _pair(p, n, 3.0)
    assert m.n_free == om.n_free
    xyz, W = m.nodes()
    assert np.abs(xyz.cpu().numpy() - om.coords()).max() <= 1e-13
    assert np.abs(W.cpu().numpy() / om.weights() - 1).max() <= 1e-12
    kd = m.kinetic_diag().cpu().numpy()
    assert np.abs(kd / om.kinetic_diag() - 1).max() <= 1e-12
    H = om.kinetic_csr().toarray()
    lmax = np.linalg.eigvalsh(H)[-1]
    assert lmax <= m.kin_bound <= 3.0 * lmax


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("nv", [5, 21, 37])
def test_apply_matches_oracle(p, nv):
    from paper_2510_10529_amd import api
    n = 4 if p <= 2 else 3
    m, om = _pair(p, n, 3.0)
    X = random_block(om.n_free, nv, 10 * p + nv)
    v = np.random.default_rng(p).uniform(-2, 2, om.n_free)
    shift = np.linspace(-1.0, 1.0, nv)
    ref = fe.hamiltonian_csr(om, v) @ X - X * shift[None, :]
    vd = torch.tensor(v, device=DEV)
    Y = api.ks_apply(m, vd, torch.tensor(X, device=DEV), shift=shift)
    err = np.abs(Y.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-13, err
    Y2 = api.ks_apply(m, vd, torch.tensor(X, device=DEV), shift=shift)
    assert torch.equal(Y, Y2)
    Y32 = api.ks_apply(m, vd, torch.tensor(X, dtype=torch.float32, device=DEV), shift=shift, prec="f32")
    err32 = np.abs(Y32.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err32 <= 2e-6, err32


@pytest.mark.parametrize("p,nv", [(2, 7), (4, 21)])
def test_chebyshev_filter_matches_oracle(p, nv):
    """The filter's Chebyshev steps read the previous block Z (beta Z); on a mapped mesh the
    first parity class holding a node adds it with the diagonal term. Degree 6 against the
    oracle's recurrence on the assembled operator."""
    from oracle import chfsi
    from paper_2510_10529_amd import api
    n = 4 if p <= 2 else 3
    m, om = _pair(p, n, 3.0)
    X = random_block(om.n_free, nv, 31 * p + nv)
    v = np.random.default_rng(p + 7).uniform(-2, 2, om.n_free)
    H = fe.hamiltonian_csr(om, v)
    lam = np.linalg.eigvalsh(H.toarray())
    a0, b = lam[0] - 0.1, lam[-1] + 0.1
    a = lam[min(nv, lam.size - 1)]
    ref = chfsi.filter_apply(lambda Z: H @ Z, X, 6, a, b, a0)
    Xd = torch.tensor(X, device=DEV)
    api.cheb_filter(m, torch.tensor(v, device=DEV), 6, a, b, a0, Xd)
    err = np.abs(Xd.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-11, err


def test_identity_map_equals_uniform_kernel():
    from paper_2510_10529_amd import api
    m0 = api.Mesh(4, 3, 3.0, mapped_amp=0.0)
    mu = api.Mesh(4, 3, 3.0)
    X = torch.tensor(random_block(mu.n_free, 12, 3), device=DEV)
    v = torch.tensor(np.random.default_rng(4).uniform(-1, 1, mu.n_free), device=DEV)
    Ya, Yb = api.ks_apply(m0, v, X), api.ks_apply(mu, v, X)
    assert float((Ya - Yb).abs().max() / Yb.abs().max()) <= 1e-13
    m0.close()
    mu.close()


def test_chain_against_oracle():
    from paper_2510_10529_amd import api
    p, n, L = 3, 5, 6.0
    wl = workload(2, p=p, n=n, half_width=L)
    m, om = _pair(p, n, L)
    Xc = om.coords()
    vf, vs = wl.v_fixed(Xc), wl.v_xc_target(Xc)
    rho_d, _ = ks.target_density(om, vf + vs, wl.n_elec)
    u = 0.5 * vs
    ev = ks.evaluate(om, vf + u, rho_d, wl.n_elec, method="bordered")
    nocc = wl.n_occ
    nv = nocc + 4
    v = torch.tensor(vf + u, device=DEV)
    Xb = torch.tensor(random_block(om.n_free, nv, 17), device=DEV)
    r = api.ks_eigensolve(m, v, Xb, nocc, 20, 1e-11, 400)
    assert r.status == 0, r
    de = np.max(np.abs(np.array(r.eig[:nocc]) - ev.eps[:nocc]))
    assert de <= 1e-8, de
    Psi = Xb[:, :nocc].contiguous()
    occ = [2.0] * nocc
    rd = torch.tensor(rho_d, device=DEV)
    rho, B, loss = api.loss_grad(m, Psi, occ, rd)
    W = om.weights()
    assert np.sum(W * np.abs(rho.cpu().numpy() - ev.rho)) <= 1e-7
    assert abs(loss - ev.loss) <= 1e-8 * ev.loss
    Q, ar = api.adjoint_solve(m, v, Psi, r.eig[:nocc], B, tol=1e-12, maxit=5000)
    g = api.loss_grad(m, Psi, occ, rd, Q=Q).cpu().numpy()
    rel = np.linalg.norm(g - ev.grad) / np.linalg.norm(ev.grad)
    assert rel <= 1e-6, rel
    Pq = (Psi.T @ Q).abs().max().item()
    assert Pq <= 1e-12 * float(Q.abs().max())


def test_calls_without_mapped_support_refuse():
    from paper_2510_10529_amd import _lib as L
    from paper_2510_10529_amd import api
    m, _ = _pair(2, 4, 3.0)
    rho = torch.ones(m.n_free, dtype=torch.float64, device=DEV)
    with pytest.raises(L.FEError, match="mapped"):
        api.poisson_solve(m, rho, sigma=1.0, tol=1e-8)
    lib = L.load()
    h = C.c_void_p()
    assert lib.fe_mesh_create_mapped(6, 2, 1.0, 0.1, C.byref(h)) == L.FE_EINVAL
    assert lib.fe_mesh_create_mapped(2, 2, 1.0, 1.5, C.byref(h)) == L.FE_EINVAL
