"""Seeded synthetic workloads for the inverse-DFT hot path.

This module is shared by the FP64 oracle, the tests and the benchmark. It holds
no arithmetic of the method itself (no finite elements, no eigensolver, no
adjoint): it only draws the parameters of the model molecules and evaluates the
resulting analytic potentials at points that the caller supplies.

The paper inverts densities of real molecules (Sec. 5: Ne, BH, H2O, ortho-benzyne,
LiH, CH2 and the water decamer). Those densities come from quantum-chemistry
data that is not available here, so each workload below is a model system of
the same structure: nuclei as softened Coulomb sites (the nuclear potential of
the Kohn-Sham Hamiltonian, Sec. 2, Eq. 2), a known "exact" XC potential made of
Gaussians, and a target density that the caller computes from that potential
(the validation recipe of Sec. 5.1: invert a density whose potential is known).

Draw order with ``numpy.random.default_rng(1000 + cfg)``:
(1) sites, (2) charges, (3) Gaussian centres, (4) amplitudes, (5) widths.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "workload", "random_block", "random_directions", "CONFIGS"]


@dataclass(frozen=True)
class Workload:
    """One model system plus its mesh parameters.

    p: FE order; n: cells per axis; half_width: the box is [-L, L]^3 (bohr);
    n_elec: electron count (spin-restricted, all orbitals doubly occupied);
    kind: "ho" (harmonic trap 0.5*omega^2 r^2) or "coulomb" (softened sites).
    """
    cfg: int
    name: str
    p: int
    n: int
    half_width: float
    n_elec: int
    kind: str
    omega: float = 1.0
    soft: float = 0.5
    sites: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    charges: np.ndarray = field(default_factory=lambda: np.zeros(0))
    g_centres: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    g_amps: np.ndarray = field(default_factory=lambda: np.zeros(0))
    g_widths: np.ndarray = field(default_factory=lambda: np.zeros(0))
    cheb_degree: int = 20

    @property
    def n_occ(self) -> int:
        return self.n_elec // 2

    @property
    def n_buf(self) -> int:
        return max(4, int(np.ceil(0.2 * self.n_occ)))

    def v_fixed(self, xyz: np.ndarray) -> np.ndarray:
        """Fixed part of the potential at points xyz (N x 3), in Hartree."""
        xyz = np.asarray(xyz, dtype=np.float64)
        if self.kind == "ho":
            return 0.5 * self.omega ** 2 * np.sum(xyz * xyz, axis=1)
        v = np.zeros(xyz.shape[0])
        for r0, z in zip(self.sites, self.charges):
            d2 = np.sum((xyz - r0) ** 2, axis=1)
            v -= z / np.sqrt(d2 + self.soft ** 2)
        return v

    def model_density(self, xyz: np.ndarray, width: float = 1.0) -> np.ndarray:
        """A closed-form molecule-like target density at points xyz: every site carries
        its charge in electrons as a normalised 3-D Gaussian of standard deviation
        ``width`` (bohr), so the density is localised at the sites, decays fast and
        integrates to the electron count over all space. Used where a target that both
        sides evaluate pointwise is needed instead of the density of a potential."""
        xyz = np.asarray(xyz, dtype=np.float64)
        rho = np.zeros(xyz.shape[0])
        norm = (2.0 * np.pi * width * width) ** -1.5
        for r0, z in zip(self.sites, self.charges):
            d2 = np.sum((xyz - r0) ** 2, axis=1)
            rho += z * norm * np.exp(-d2 / (2.0 * width * width))
        return rho

    def v_xc_target(self, xyz: np.ndarray) -> np.ndarray:
        """The known XC potential v* (sum of Gaussians) at points xyz."""
        xyz = np.asarray(xyz, dtype=np.float64)
        v = np.zeros(xyz.shape[0])
        for c, a, s in zip(self.g_centres, self.g_amps, self.g_widths):
            d2 = np.sum((xyz - c) ** 2, axis=1)
            v += a * np.exp(-d2 / (2.0 * s * s))
        return v


def _in_ball(rng: np.random.Generator, k: int, radius: float) -> np.ndarray:
    d = rng.standard_normal((k, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.random(k) ** (1.0 / 3.0)
    return d * r[:, None]


def _charges(rng: np.random.Generator, k: int, total: float) -> np.ndarray:
    z = rng.uniform(0.5, 1.5, size=k)
    return total * z / z.sum()


# (p, n, L, N_e, kind, n_sites, site_region, n_gauss, gauss_region, cheb_degree)
CONFIGS = {
    1: dict(name="ho-q2-12", p=2, n=12, L=8.0, ne=8, kind="ho", sites=0,
            region=None, ng=3, gregion=("ball", 2.0), deg=12),
    2: dict(name="mol10-q4-24", p=4, n=24, L=12.0, ne=10, kind="coulomb", sites=3,
            region=("ball", 2.0), ng=4, gregion=("ball", 2.0), deg=30),
    3: dict(name="mol20-q4-32", p=4, n=32, L=12.0, ne=20, kind="coulomb", sites=6,
            region=("ball", 3.0), ng=6, gregion=("ball", 3.0), deg=30),
    4: dict(name="mol50-q5-36", p=5, n=36, L=14.0, ne=50, kind="coulomb", sites=12,
            region=("ball", 4.0), ng=8, gregion=("ball", 4.0), deg=40),
    5: dict(name="mol100-q5-40", p=5, n=40, L=16.0, ne=100, kind="coulomb", sites=20,
            region=("ellipsoid", (6.0, 4.0, 3.0)), ng=10,
            gregion=("ellipsoid", (6.0, 4.0, 3.0)), deg=40),
}


def _region_points(rng, k, region):
    kind, size = region
    if kind == "ball":
        return _in_ball(rng, k, size)
    axes = np.asarray(size, dtype=np.float64)
    return _in_ball(rng, k, 1.0) * axes[None, :]


def workload(cfg: int, *, p: int | None = None, n: int | None = None,
             half_width: float | None = None) -> Workload:
    """The seeded model system of workload ``cfg`` (1..5).

    ``p``, ``n`` and ``half_width`` override the mesh while keeping the same
    physical system; tests use that to run a workload's potential on small meshes.
    """
    c = CONFIGS[cfg]
    rng = np.random.default_rng(1000 + cfg)
    sites = np.zeros((0, 3))
    charges = np.zeros(0)
    if c["sites"]:
        sites = _region_points(rng, c["sites"], c["region"])          # (1)
        charges = _charges(rng, c["sites"], float(c["ne"]))            # (2)
    ng = c["ng"]
    centres = _region_points(rng, ng, c["gregion"])                    # (3)
    amps = rng.uniform(-0.3, 0.3, size=ng)                             # (4)
    widths = rng.uniform(0.5, 1.5, size=ng)                            # (5)
    return Workload(cfg=cfg, name=c["name"], p=p or c["p"], n=n or c["n"],
                    half_width=half_width or c["L"], n_elec=c["ne"], kind=c["kind"],
                    sites=sites, charges=charges, g_centres=centres, g_amps=amps,
                    g_widths=widths, cheb_degree=c["deg"])


def random_block(n_rows: int, n_cols: int, seed: int) -> np.ndarray:
    """Seeded standard-normal block (n_rows x n_cols, row-major), FP64.

    Used as the random start of the subspace iteration and as random operands in
    parity tests; the random numbers are drawn here and passed in as inputs.
    """
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_rows, n_cols))


def random_directions(n_rows: int, k: int, seed: int) -> np.ndarray:
    """k seeded directions d ~ N(0,1) per node, each scaled to max-norm 1."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((k, n_rows))
    d /= np.max(np.abs(d), axis=1, keepdims=True)
    return d


def vxc_vertices(L: float, h_v: float, inner: float, growth: float = 1.5) -> np.ndarray:
    """1-D vertex list of the linear mesh for the XC potential on [-L, L]: uniform cells of
    size h_v on [-inner, inner] (the inner cuboid), then cells growing by `growth` towards
    the boundary (the outer cuboid), the last one ending at +-L (a sliver is merged into
    its neighbour). Symmetric about 0. Mesh parameters are inputs, shared by both sides."""
    n_in = max(1, int(round(min(inner, L) / h_v)))
    if n_in * h_v >= L:
        n = max(1, int(round(L / h_v)))
        return np.linspace(-L, L, 2 * n + 1)
    right = [n_in * h_v]
    h = h_v
    while right[-1] < L:
        h *= growth
        right.append(right[-1] + h)
    right[-1] = L
    if len(right) > 2 and right[-1] - right[-2] < 0.5 * (right[-2] - right[-3]):
        right.pop(-2)
    core = np.linspace(-n_in * h_v, n_in * h_v, 2 * n_in + 1)
    right = np.array(right[1:])
    return np.concatenate([-right[::-1], core, right])
