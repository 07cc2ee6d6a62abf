"""Seeded synthetic inputs shared by the HIP path's tests and the oracle's tests.

This module holds input generators only: clustered point catalogues, marks and
analytic test fields.  It contains none of the estimator's arithmetic, so both
sides can consume the same inputs without sharing any of the method.

Catalogues follow a Neyman-Scott (Thomas) process: parents uniform in the
periodic box, a fixed number of Gaussian-displaced children per parent,
wrapped into [0, L).  Positions are returned as float32, the type the library
consumes.  All draws use numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_BASE = 2607_0000


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _wrap_f32(pos64: np.ndarray, box_L: float) -> np.ndarray:
    """Wrap float64 positions into [0, L) and round to float32 inside [0, L)."""
    pos = np.mod(pos64, box_L).astype(np.float32)
    # rounding to float32 can land exactly on L; fold it back to 0
    pos[pos >= np.float32(box_L)] = 0.0
    return pos


def neyman_scott(n_parents: int, n_children: int, sigma: float, box_L: float,
                 seed: int, sigma_z: float = 0.0) -> np.ndarray:
    """Clustered catalogue: float32 [n_parents*n_children, 3] in [0, L)."""
    rng = _rng(seed)
    parents = rng.uniform(0.0, box_L, size=(n_parents, 3))
    pos = np.repeat(parents, n_children, axis=0)
    pos += sigma * rng.standard_normal(size=pos.shape)
    if sigma_z > 0.0:
        pos[:, 2] += sigma_z * rng.standard_normal(size=pos.shape[0])
    return _wrap_f32(pos, box_L)


def uniform_points(n_pts: int, box_L: float, seed: int) -> np.ndarray:
    """Poisson (iid uniform) catalogue: float32 [n_pts, 3] in [0, L)."""
    rng = _rng(seed)
    return _wrap_f32(rng.uniform(0.0, box_L, size=(n_pts, 3)), box_L)


def lognormal_marks(n_pts: int, seed: int, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    """iid log-normal marks exp(N(mu, sigma^2)) as float32 [n_pts]."""
    rng = _rng(seed + 7919)
    return np.exp(mu + sigma * rng.standard_normal(n_pts)).astype(np.float32)


def cosine_field(n: int, waves, amps=None) -> np.ndarray:
    """Real field sum_j A_j cos(2 pi n_j . l / N) on an N^3 grid (float64 [N,N,N]).

    ``waves`` is a list of integer 3-vectors n_j.  Used for closed-form checks.
    """
    idx = np.arange(n, dtype=np.float64)
    lx, ly, lz = np.meshgrid(idx, idx, idx, indexing="ij")
    out = np.zeros((n, n, n))
    if amps is None:
        amps = [1.0] * len(waves)
    for a, w in zip(amps, waves):
        out += a * np.cos(2.0 * np.pi * (w[0] * lx + w[1] * ly + w[2] * lz) / n)
    return out


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: catalogue recipe, grid and statistics."""
    name: str
    box_L: float
    n_parents: int
    n_children: int
    sigma: float
    n_grid: int
    sigma_z: float = 0.0
    marks: bool = False
    seed: int = SEED_BASE

    @property
    def n_pts(self) -> int:
        return self.n_parents * self.n_children

    def catalogue(self):
        pos = neyman_scott(self.n_parents, self.n_children, self.sigma, self.box_L,
                           self.seed, self.sigma_z)
        w = lognormal_marks(pos.shape[0], self.seed) if self.marks else None
        return pos, w


# The five workloads.  Bin edges are linear throughout.
WORKLOADS = {
    # 2e4 points, L=250, 64^3, 20-bin 2PCF over [5, 50], FP64
    "ns64_fp64": Workload("ns64_fp64", 250.0, 400, 50, 2.0, 64, seed=SEED_BASE + 1),
    # 2e6 points, L=1000, 256^3, redshift-space z displacement sigma_z=4
    "ns256_rsd": Workload("ns256_rsd", 1000.0, 20_000, 100, 3.0, 256, sigma_z=4.0,
                          seed=SEED_BASE + 2),
    # 1e7 marked points, L=1000, 512^3: 3PCF l<=10 x 20 bins plus a 40-bin 2PCF
    "ns512_3pcf": Workload("ns512_3pcf", 1000.0, 100_000, 100, 3.0, 512, marks=True,
                           seed=SEED_BASE + 3),
    # 1e8 marked points, L=2000, 1024^3: marked 2PCF + counts-in-cells moments
    "ns1024_cic": Workload("ns1024_cic", 2000.0, 1_000_000, 100, 3.0, 1024, marks=True,
                           seed=SEED_BASE + 4),
}

EDGES = {
    "ns64_fp64": np.linspace(5.0, 50.0, 21),
    "ns256_rsd": np.linspace(2.0, 200.0, 41),
    "ns256_rsd_ell": np.linspace(2.0, 200.0, 31),
    "ns512_3pcf": np.linspace(10.0, 150.0, 21),
    "ns512_2pcf": np.linspace(2.0, 200.0, 41),
    "ns1024_cic": np.linspace(2.0, 200.0, 41),
}

# counts-in-cells radii: geometric from 4 to 32 Mpc/h, 8 values
CIC_RADII = 4.0 * 2.0 ** (3.0 * np.arange(8) / 7.0)

# DD(s, mu) with ring binning windows on the 256^3 redshift-space workload:
# 46 separations x 51 orientations, thin double rings at the bin centres
# (r_perp = s sqrt(1 - mu^2), r_par = s mu), s in 4 Mpc/h bins over [2, 186],
# mu in equal bins over [0, 1].
SMU_S_EDGES = np.linspace(2.0, 186.0, 47)
SMU_N_MU = 51


def smu_rings(s_edges=SMU_S_EDGES, n_mu: int = SMU_N_MU) -> list:
    """Window specs ("ring", r_perp, r_par), s-major, for every (s, mu) bin."""
    s = 0.5 * (np.asarray(s_edges[1:]) + np.asarray(s_edges[:-1]))
    mu = (np.arange(n_mu) + 0.5) / n_mu
    return [("ring", float(si * np.sqrt(1.0 - m * m)), float(si * m)) for si in s for m in mu]
