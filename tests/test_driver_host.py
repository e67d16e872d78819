"""Host logic of the driver (CPU only): which Ritz pairs deflate the adjoint's preconditioner."""
import pytest

torch = pytest.importorskip("torch")


def _prob(n, eig_incl, nv, deflate):
    from paper_2510_10529_amd import inverse as inv
    p = inv.InverseProblem.__new__(inv.InverseProblem)      # no mesh or device needed here
    p.opts = inv.SolverOptions(deflate=deflate)
    p.nv = nv
    p.X = torch.arange(5 * nv, dtype=torch.float64).reshape(5, nv)
    p.state = inv.OccState(n, [2.0] * n, eig_incl)
    return p


def test_deflation_block_skips_degenerate_partners():
    p = _prob(3, [-1.0, -0.5, -0.2], 8, 4)
    eig = [-1.0, -0.5, -0.2, -0.2 + 1e-12, 0.1, 0.2, 0.3, 0.4]
    p._deflation_block(eig)
    assert p.state.theta == [0.1, 0.2, 0.3, 0.4]
    assert torch.equal(p.state.U, p.X[:, 4:8])
    assert p.state.U.is_contiguous()
    p.X.zero_()                                              # a copy: the next eigensolve may overwrite X
    assert p.state.U.abs().sum() > 0


def test_deflation_block_limits():
    p = _prob(3, [-1.0, -0.5, -0.2], 8, 10)                 # more asked than the block holds
    p._deflation_block([-1.0, -0.5, -0.2, 0.0, 0.1, 0.2, 0.3, 0.4])
    assert len(p.state.theta) == 5
    p = _prob(62, [float(i) for i in range(62)], 64, 10)   # nocc + nbuf <= 64
    p._deflation_block([float(i) for i in range(64)])
    assert len(p.state.theta) == 2
    p = _prob(3, [-1.0, -0.5, -0.2], 4, 4)                  # nothing above the included orbitals
    p._deflation_block([-1.0, -0.5, -0.2, -0.2])
    assert p.state.U is None and p.state.theta is None
