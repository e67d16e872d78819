"""The extensions together through the autograd driver (needs an MI355X): a graded orbital
mesh, finite temperature with fractional occupations, and the XC potential on its own
linear mesh, against the oracle composed the same way (thermal oracle on the graded mesh,
then the transpose of the linear-mesh prolongation). Then a few L-BFGS steps.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fe, thermal as th, vxcmesh as vm  # noqa: E402
from synth import random_block, vxc_vertices, workload  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _problem():
    from paper_2510_10529_amd import api
    from paper_2510_10529_amd import inverse as inv
    wl = workload(1)
    t = vxc_vertices(8.0, 1.0, 3.0, 1.6)                       # graded orbital cells
    m, om = api.Mesh(2, 0, 0.0, breaks=t), fe.mesh3d_graded(2, t)
    tv = vxc_vertices(8.0, 0.8, 3.2, 1.5)                      # linear XC mesh
    P = vm.prolongation(om, tv, tv, tv)
    X = om.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    ne, kT = 10.0, 0.02
    rho_d = th.target_density(om, vf + vs, ne, kT, n_states=16)
    u = 0.1 * np.cos(0.4 * np.arange(P.shape[1]))
    opts = inv.SolverOptions(degree=wl.cheb_degree, tol_eig=1e-10, tol_adj=1e-12, kT=kT, n_states=12)
    V = api.VxcMesh(m, tv, tv, tv)
    prob = inv.InverseProblem(m, _t(vf), _t(rho_d), ne, _t(random_block(om.n_free, 16, 21)), opts, vxc=V)
    return om, P, vf, rho_d, ne, kT, u, prob


def test_graded_thermal_linear_mesh_gradient():
    from paper_2510_10529_amd import inverse as inv
    om, P, vf, rho_d, ne, kT, u, prob = _problem()
    ev = th.evaluate(om, vf + P @ u, rho_d, ne, kT, n_states=16)
    f_ref = P.T @ ev.grad
    ur = _t(u).requires_grad_(True)
    loss = inv.InvDFTLoss.apply(ur, prob)
    loss.backward()
    assert abs(float(loss) - ev.loss) <= 1e-7 * ev.loss
    f = ur.grad.cpu().numpy()
    rel = np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref)
    assert rel <= 1e-6, rel
    assert np.any((ev.occ > 0.05) & (ev.occ < 1.95))


def test_graded_thermal_linear_mesh_lbfgs_descends():
    from paper_2510_10529_amd import inverse as inv
    om, P, vf, rho_d, ne, kT, u, prob = _problem()
    uT, losses = inv.lbfgs(prob, _t(u), maxiter=5)
    assert all(np.isfinite(losses))
    assert all(b <= a for a, b in zip(losses, losses[1:]))
    assert losses[-1] < 0.5 * losses[0]
