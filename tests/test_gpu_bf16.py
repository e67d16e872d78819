"""FE_BF16 blocks against the oracle (needs an MI355X).

bf16 storage, FP32 arithmetic, round to nearest even on store. The oracle works in FP64 on
the exact values of the bf16 inputs, so the bars come from the arithmetic:
  * ks_apply: every output is the FP64 result rounded to bf16, up to the FP32 accumulation
    error (about 1e-6 of the result). At least 99.5 % of the outputs must equal the oracle's
    FP64 result rounded to nearest even, and every other one must be a neighbouring bf16
    value; truncation instead of rounding would miss about half of them.
  * cheb_filter: each of the m steps rounds the block to bf16 (unit roundoff 2^-8), so the
    result is held to m 2^-7 of the block's largest entry.
  * ks_eigensolve from a random start in bf16 -> FP32 -> FP64 stages reaches the FP64
    tolerance and the oracle's eigenvalues (1e-8 Ha) and density (L1 1e-7).
"""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import chfsi, fe, ks  # noqa: E402
from synth import random_block, workload  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@functools.lru_cache(maxsize=None)
def _pair(p, n, L, graded=False):
    from paper_2510_10529_amd import api
    if graded:
        t = np.cumsum(np.r_[0.0, np.linspace(0.6, 1.4, n)])
        t = t - 0.5 * t[-1]
        return api.Mesh(p, n, L, breaks=t), fe.mesh3d_graded(p, t)
    return api.Mesh(p, n, L), fe.mesh3d(p, n, L)


def _bf16(a):
    """torch bfloat16 tensor (round to nearest even) and the exact FP64 values it holds."""
    t = torch.tensor(np.ascontiguousarray(a), dtype=torch.float32).to(torch.bfloat16)
    return t, t.double().numpy()


def _neighbours(gpu_bits, ref_bits):
    """bf16 values one step apart: their bit patterns (same sign) differ by one."""
    return (np.abs(gpu_bits.astype(np.int32) - ref_bits.astype(np.int32)) <= 1)


@pytest.mark.parametrize("p,n,graded", [(1, 6, False), (2, 5, False), (4, 3, False), (5, 3, False),
                                        (8, 2, False), (3, 4, True), (5, 3, True)])
@pytest.mark.parametrize("nv", [7, 24])
def test_apply_rounds_to_nearest_even(p, n, graded, nv):
    from paper_2510_10529_amd import api
    m, om = _pair(p, n, 4.0, graded)
    Xb, X = _bf16(random_block(om.n_free, nv, 31 * p + nv))
    v = np.random.default_rng(p).uniform(-2, 2, om.n_free)
    shift = np.linspace(-0.5, 0.5, nv)
    ref = fe.hamiltonian_csr(om, v) @ X - X * shift[None, :]
    Yb = api.ks_apply(m, torch.tensor(v, device=DEV), Xb.to(DEV), shift=shift, prec="bf16")
    assert Yb.dtype == torch.bfloat16
    got = Yb.cpu()
    ref_b = torch.tensor(ref, dtype=torch.float32).to(torch.bfloat16)
    gb, rb = got.view(torch.int16).numpy(), ref_b.view(torch.int16).numpy()
    same = np.mean(gb == rb)
    assert same >= 0.995, same
    # where a bf16 step (|ref| 2^-7) is far above the FP32 accumulation error (about 1e-6 of the
    # largest output), the result is the rounded value or its neighbour; smaller outputs come from
    # cancellation and are held by the absolute term of the bound below
    big = np.abs(ref) >= 1e-3 * np.abs(ref).max()
    assert np.all(_neighbours(gb, rb)[big]), "more than one bf16 step"
    err = np.abs(got.double().numpy() - ref)
    assert np.all(err <= 2.0 ** -7 * np.abs(ref) + 1e-5 * np.abs(ref).max())


def test_cheb_filter_bf16():
    from paper_2510_10529_amd import api
    m, om = _pair(3, 5, 5.0)
    wl = workload(2, p=3, n=5, half_width=5.0)
    Xc = om.coords()
    v = wl.v_fixed(Xc) + wl.v_xc_target(Xc)
    Xb, X = _bf16(random_block(om.n_free, 16, 12))
    deg = 6
    a, b, a0 = 5.0, fe.element_bound(3, 2.0) + v.max(), v.min() - 1.0
    ref = chfsi.filter_apply(lambda Z: fe.hamiltonian_apply(om, v, Z), X, deg, a, b, a0)
    Xt = Xb.to(DEV)
    api.cheb_filter(m, torch.tensor(v, device=DEV), deg, a, b, a0, Xt, prec="bf16")
    err = np.abs(Xt.double().cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"[bf16] filter degree {deg}: max error {err:.2e} of the largest entry", flush=True)
    assert err <= deg * 2.0 ** -7, err
    assert err > 1e-6            # the block was rounded to bf16 (not computed wider)


def test_eigensolve_stages_reach_fp64_accuracy():
    from paper_2510_10529_amd import api
    wl = workload(1)
    m, om = _pair(wl.p, wl.n, wl.half_width)
    X = om.coords()
    vf, vs = wl.v_fixed(X), wl.v_xc_target(X)
    v = vf + 0.5 * vs
    ev = ks.evaluate(om, v, np.zeros(om.n_free), wl.n_elec, want_grad=False, method="auto")
    nocc = wl.n_occ
    nv = nocc + 8
    vt = torch.tensor(v, device=DEV)
    Xb = torch.tensor(random_block(om.n_free, nv, 77), device=DEV)
    r = api.ks_eigensolve(m, vt, Xb, nocc, wl.cheb_degree, 1e-10, 400, prec="bf16", switch_tol=1e-4)
    assert r.status == 0, r
    nb, n32, n64 = r.stage_passes
    assert nb >= 1 and n32 >= 1 and n64 >= 1, r.stage_passes
    assert nb + n32 + n64 == r.passes
    assert np.max(np.abs(np.array(r.eig[:nocc]) - ev.eps[:nocc])) <= 1e-8
    rho, _, _ = api.loss_grad(m, Xb[:, :nocc].contiguous(), [2.0] * nocc,
                              torch.zeros(om.n_free, dtype=torch.float64, device=DEV), want_B=False)
    assert np.sum(om.weights() * np.abs(rho.cpu().numpy() - ev.rho)) <= 1e-7


def test_bf16_refused_on_mapped_meshes():
    from paper_2510_10529_amd import _lib
    from paper_2510_10529_amd import api
    m = api.Mesh(2, 3, 3.0, mapped_amp=0.1)
    X = torch.zeros((m.n_free, 8), dtype=torch.bfloat16, device=DEV)
    v = torch.zeros(m.n_free, dtype=torch.float64, device=DEV)
    with pytest.raises(_lib.FEError) as e:
        api.ks_apply(m, v, X, prec="bf16")
    assert e.value.status == _lib.FE_EINVAL
    m.close()
