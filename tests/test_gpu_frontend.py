"""GPU parity of the physics front end (needs an MI355X): the Hartree potential by the
finite-element Poisson solve and the initial guess of Eq. 25, against the oracle.

* a manufactured solution u = prod (L^2 - x_i^2) that the order-p space holds exactly
  (p >= 3) is reproduced by the conjugate-gradient solve;
* two Gaussian charges on the ho-q2-12 mesh, with the monopole split off, against the
  oracle's direct sparse solve of the same discrete problem;
* the initial guess node by node against the oracle's formulas, from empty to dense, with
  Slater and with LB94 exchange (through the nodal gradient, on uniform and graded cells);
* at full size, the target density of mol100-q5-40 (7,880,599 nodes): the charge, the
  solver's residual, the discrete equation on sampled rows evaluated one by one from the
  oracle's Kronecker rows and the closed-form Gaussian, and the far field ~ Q / r.
"""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fe, hartree as hr, xcinit as xc  # noqa: E402
from synth import random_block, workload  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _say(msg):
    print(f"[frontend] {msg}", file=sys.stderr, flush=True)


@pytest.mark.parametrize("p,n,L", [(3, 4, 2.0), (4, 3, 1.5), (5, 3, 2.5)])
def test_poisson_manufactured_solution(p, n, L):
    from paper_2510_10529_amd import api
    m, om = api.Mesh(p, n, L), fe.mesh3d(p, n, L)
    X = om.coords()
    a = L * L - X * X
    u = np.prod(a, axis=1)
    f = 2 * (a[:, 1] * a[:, 2] + a[:, 0] * a[:, 2] + a[:, 0] * a[:, 1])
    phi, res = api.poisson_solve(m, _t(f / (4 * np.pi)), sigma=0.0, tol=1e-13)
    assert res.status == 0 and res.relres <= 1e-13
    assert np.abs(phi.cpu().numpy() - u).max() <= 1e-10 * np.abs(u).max()


def test_poisson_gaussian_charges_against_oracle():
    from paper_2510_10529_amd import api
    wl = workload(1)
    m, om = api.Mesh(wl.p, wl.n, wl.half_width), fe.mesh3d(wl.p, wl.n, wl.half_width)
    X = om.coords()
    c0 = np.array([0.3, -0.2, 0.1])
    rho = 3.0 * hr.gaussian(X, c0, 0.8) + 0.5 * hr.gaussian(X, c0 + np.array([1.0, 0.5, 0.0]), 0.6)
    ref, Q, c = hr.hartree(om, rho, 1.0)
    phi, res = api.poisson_solve(m, _t(rho), sigma=1.0, tol=1e-13)
    assert res.status == 0
    assert abs(res.charge - Q) <= 1e-13 * Q
    got = phi.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("graded", [False, True])
def test_initial_guess_against_oracle(graded):
    """Slater and LB94 on a density with empty, tiny and dense nodes; LB94 through the nodal
    gradient of the order-p interpolant (uniform and graded cells)."""
    from paper_2510_10529_amd import api
    from synth import vxc_vertices
    if graded:
        t = vxc_vertices(8.0, 1.0, 3.0, 1.6)
        m, om = api.Mesh(3, 0, 0.0, breaks=t), fe.mesh3d_graded(3, t)
    else:
        m, om = api.Mesh(3, 8, 8.0), fe.mesh3d(3, 8, 8.0)
    X = om.coords()
    rng = np.random.default_rng(12)
    rho = 5.0 * np.exp(-0.5 * np.sum((X - 0.3) ** 2, axis=1)) + 0.5 * np.exp(-2 * np.sum((X + 1) ** 2, axis=1))
    rho[rng.integers(0, om.n_free, 50)] = 0.0
    vh = rng.uniform(0.0, 20.0, om.n_free)
    grad = np.linalg.norm(fe.nodal_gradient(om, rho), axis=1)
    for ex, gn in (("slater", None), ("lb94", grad)):
        for tau, alpha in ((1e-2, 1.0), (1e-3, 0.25)):
            got = api.xc_initial_guess(m, _t(rho), _t(vh), 100.0, tau=tau, alpha=alpha, exchange=ex).cpu().numpy()
            ref = xc.initial_guess(rho, vh, 100.0, tau=tau, alpha=alpha, grad_norm=gn)
            np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-13)


def test_hartree_full_size():
    from paper_2510_10529_amd import api
    wl = workload(5)
    m, om = api.Mesh(wl.p, wl.n, wl.half_width), fe.mesh3d(wl.p, wl.n, wl.half_width)
    X = om.coords()
    v = _t(wl.v_fixed(X) + wl.v_xc_target(X))
    nocc, nv = wl.n_occ, wl.n_occ + wl.n_buf
    Xb = _t(random_block(om.n_free, nv, 1005))
    r = api.ks_eigensolve(m, v, Xb, nocc, wl.cheb_degree, 1e-9, 400, prec="f32", switch_tol=1e-4)
    assert r.status == 0, r
    rho, _, _ = api.loss_grad(m, Xb[:, :nocc].contiguous(), [2.0] * nocc, torch.zeros_like(v), want_B=False)
    del Xb
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, res = api.poisson_solve(m, rho, sigma=1.0, tol=1e-10)
    dt = time.perf_counter() - t0
    _say(f"Hartree solve at {om.n_free} nodes: {res.iters} CG iterations, relres {res.relres:.2e}, "
         f"{dt:.2f} s, charge {res.charge:.12f}")
    assert res.status == 0
    assert abs(res.charge - wl.n_elec) <= 1e-9 * wl.n_elec
    rh, ph = rho.cpu().numpy(), phi.cpu().numpy()
    W = om.weights()
    Q = float(W @ rh)
    c = (W * rh) @ X / Q
    # the discrete equation on sampled rows: (K~/2) W^{1/2} (phi - phi_G) = 2 pi W^{1/2} (rho - Q g)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([rng.integers(0, om.n_free, 400), [0, om.n_free // 2, om.n_free - 1]]))
    phit = np.sqrt(W) * (ph - Q * hr.gaussian_potential(X, c, 1.0))
    lhs = fe.hamiltonian_rows(om, np.zeros(om.n_free), phit[:, None], rows)[:, 0]
    b = 2 * np.pi * np.sqrt(W) * (rh - Q * hr.gaussian(X, c, 1.0))
    assert np.abs(lhs - b[rows]).max() <= 1e-7 * np.abs(b).max()
    # far field: the potential of 100 electrons near the box faces is ~ Q / |r - c|
    far = np.max(np.abs(X), axis=1) > 0.9 * wl.half_width
    ratio = ph[far] * np.linalg.norm(X[far] - c, axis=1) / Q
    _say(f"far field: phi |r - c| / Q in [{ratio.min():.4f}, {ratio.max():.4f}]")
    assert ratio.min() > 0.97 and ratio.max() < 1.03
    vi = api.xc_initial_guess(m, rho, phi, float(wl.n_elec), exchange="lb94").cpu().numpy()
    gn = np.linalg.norm(fe.nodal_gradient(om, rh), axis=1)
    sel = rows
    np.testing.assert_allclose(vi[sel], xc.initial_guess(rh[sel], ph[sel], float(wl.n_elec), grad_norm=gn[sel]),
                               rtol=1e-10, atol=1e-13)
