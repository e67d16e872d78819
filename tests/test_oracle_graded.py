"""Pins of the oracle on graded tensor meshes (cells of different widths along each axis;
CPU only). What the mathematics fixes, independently of the assembly:

* 1-D: for u = L^2 - x^2 (inside every order-p space, p >= 2, on any cells) integration by
  parts gives (K1 u)_i = int u' N_i' = 2 int N_i = 2 W1_i, the GLL weight being the exact
  integral of N_i;
* 3-D: the energy of u = prod (L^2 - x_i^2) is 1024 L^13 / 225 on any such mesh;
* the harmonic trap's eigenvalues (n + 3/2) are approached as the central cells shrink;
* Fried's bound with the smallest cell still bounds the spectrum of K~/2.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fe
from synth import vxc_vertices


def _breaks(L, h, inner, growth):
    return vxc_vertices(L, h, inner, growth)


@pytest.mark.parametrize("p,L,h,inner,growth", [(2, 3.0, 0.5, 1.0, 1.7), (4, 4.0, 0.7, 2.0, 1.5),
                                                (5, 3.0, 0.4, 1.2, 1.9), (3, 5.0, 0.9, 5.0, 1.0)])
def test_1d_stiffness_on_quadratic(p, L, h, inner, growth):
    m1 = fe.mesh1d(p, 0, 0.0, breaks=_breaks(L, h, inner, growth))
    u = L * L - m1.x ** 2
    np.testing.assert_allclose(m1.K1 @ u, 2.0 * m1.W1, rtol=1e-12, atol=1e-12 * m1.W1.max())


@pytest.mark.parametrize("p,L,h,inner,growth", [(2, 2.0, 0.45, 0.9, 1.6), (3, 2.5, 0.6, 1.2, 1.5),
                                                (4, 2.0, 0.5, 0.5, 2.0)])
def test_3d_energy_closed_form(p, L, h, inner, growth):
    t = _breaks(L, h, inner, growth)
    assert np.ptp(np.diff(t)) > 0.1                   # the mesh really is graded
    m = fe.mesh3d_graded(p, t)
    X = m.coords()
    u = np.prod(L * L - X * X, axis=1)
    ut = np.sqrt(m.weights()) * u
    e = ut @ fe.kinetic_apply(m, ut)
    assert abs(e / (1024.0 * L ** 13 / 225.0) - 1.0) < 1e-12
    # the Kronecker apply and the assembled operator agree
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((m.n_free, 3))
    np.testing.assert_allclose(fe.kinetic_apply(m, Y), fe.kinetic_csr(m) @ Y, rtol=0, atol=1e-11)


def test_harmonic_trap_on_graded_meshes():
    """Refining the central cells moves the lowest levels towards 3/2, 5/2."""
    errs = []
    for h in (1.2, 0.6):
        t = _breaks(5.0, h, 2.4, 1.6)
        m = fe.mesh3d_graded(3, t)
        X = m.coords()
        H = fe.hamiltonian_csr(m, 0.5 * np.sum(X * X, axis=1))
        w = np.sort(spla.eigsh(H, k=8, which="SA", tol=1e-12, ncv=48)[0])[:4]   # k > 4: Lanczos sees every copy
        errs.append(np.abs(w - np.array([1.5, 2.5, 2.5, 2.5])).max())
        assert np.ptp(w[1:]) < 1e-9                   # the triplet stays exactly degenerate
    assert errs[1] < errs[0] / 8 and errs[1] < 1e-4, errs


def test_fried_bound_with_smallest_cell():
    t = _breaks(3.0, 0.5, 1.0, 1.8)
    m = fe.mesh3d_graded(3, t)
    lmax = spla.eigsh(fe.kinetic_csr(m), k=1, which="LA", tol=1e-10)[0][0]     # kinetic_csr is K~/2
    b = fe.element_bound(3, np.diff(t).min())
    assert lmax <= b * (1 + 1e-12)
    assert lmax >= 0.7 * b          # and not vacuous (0.93 b on this mesh)
