"""Pins of the linear-mesh XC potential and its transfer (Eq. 14, Eq. 22; CPU only):

* P reproduces every trilinear function exactly (the span of the Q1 hat functions),
  and 1 in particular (partition of unity); weights are non-negative, at most 8 a row;
* the transpose is the adjoint: <P u, g> = <u, P^T g>;
* brute-force central differences of L(v_fixed + P u) with respect to every
  linear-mesh unknown equal P^T g, g the pinned nodal gradient of the orbital mesh.
"""
import numpy as np
import pytest

from oracle import fe, ks, vxcmesh as vm
from synth import vxc_vertices, workload


def _trilinear(X, c):
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z + c[6] * x * z + c[7] * x * y * z


@pytest.mark.parametrize("p,n,L,hv,inner", [(2, 3, 4.0, 0.7, 2.0), (4, 2, 3.0, 0.4, 3.5), (3, 3, 5.0, 1.3, 1.0)])
def test_prolongation_exact_on_trilinear_fields(p, n, L, hv, inner):
    m = fe.mesh3d(p, n, L)
    tx = vxc_vertices(L, hv, inner, 1.5)
    ty = vxc_vertices(L, hv * 1.3, inner, 1.4)
    tz = vxc_vertices(L, hv * 0.8, inner, 1.6)
    P = vm.prolongation(m, tx, ty, tz)
    V = np.stack(np.meshgrid(tx, ty, tz, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    c = np.random.default_rng(4).standard_normal(8)
    np.testing.assert_allclose(P @ _trilinear(V, c), _trilinear(m.coords(), c), rtol=0, atol=1e-12)
    np.testing.assert_allclose(P @ np.ones(P.shape[1]), 1.0, rtol=0, atol=1e-14)
    assert P.data.min() >= 0 and np.diff(P.indptr).max() <= 8


def test_prolongation_is_not_exact_beyond_trilinear():
    """x^2 is outside the span: the pin above can fail."""
    m = fe.mesh3d(3, 2, 3.0)
    t = vxc_vertices(3.0, 0.9, 3.0, 1.5)
    P = vm.prolongation(m, t, t, t)
    V = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    assert np.abs(P @ V[:, 0] ** 2 - m.coords()[:, 0] ** 2).max() > 1e-3


def test_transpose_is_the_adjoint():
    m = fe.mesh3d(3, 3, 4.0)
    t = vxc_vertices(4.0, 0.6, 2.0, 1.5)
    P = vm.prolongation(m, t, t, t)
    rng = np.random.default_rng(8)
    u, g = rng.standard_normal(P.shape[1]), rng.standard_normal(P.shape[0])
    assert abs((P @ u) @ g - u @ (P.T @ g)) < 1e-12 * np.abs(u).sum() * np.abs(g).max()


def test_gradient_brute_force_fd_every_vertex():
    wl = workload(2, p=2, n=3, half_width=4.0)
    m = fe.mesh3d(2, 3, 4.0)
    X = m.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    rho_d, _ = ks.target_density(m, vf + vs, wl.n_elec)
    t = vxc_vertices(4.0, 1.5, 1.5, 1.6)
    P = vm.prolongation(m, t, t, t)
    u = 0.3 * np.sin(np.arange(P.shape[1]) * 0.7)
    loss, f, _ = vm.evaluate(m, vf, P, u, rho_d, wl.n_elec, method="sos")
    h = 1e-3
    fd = np.empty(P.shape[1])
    for b in range(P.shape[1]):
        e = np.zeros(P.shape[1])
        e[b] = 1.0

        def cd(s):
            lp = vm.evaluate(m, vf, P, u + s * e, rho_d, wl.n_elec, method="sos", want_grad=False)[0]
            lm = vm.evaluate(m, vf, P, u - s * e, rho_d, wl.n_elec, method="sos", want_grad=False)[0]
            return (lp - lm) / (2 * s)
        fd[b] = (4 * cd(h / 2) - cd(h)) / 3
    np.testing.assert_allclose(f, fd, rtol=0, atol=1e-8 * np.abs(fd).max())
