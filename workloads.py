"""Seeded synthetic workloads for the deforming-box pair-force path.

This module is shared by the tests, the benchmark and the smoke check.  It
holds only workload *definitions*: random draws (fractional positions, jitter,
replica sizes, flows, rates, strain times, momenta), fixed constants that the
workload descriptions name (densities, cut-offs, flow matrices, the lattice
automorphisms and the initial bases built from their eigenvectors), and the
linear map that turns fractional coordinates into Cartesian positions for a
basis the *caller* supplies.  It contains none of the method's arithmetic: no
lattice evolution or reduction, no cell binning, no distances or forces.  Both
the FP64 oracle and the GPU library compute those on their own.

Random numbers use numpy's PCG64 generator with a fixed seed per workload
and replica.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# ---------------------------------------------------------------------------
# potentials: Lennard-Jones form truncated at r_c; WCA is the purely repulsive
# truncation at the LJ minimum 2^(1/6) sigma.  Energies are shifted to zero at
# the cut-off (WCA's "+epsilon").  Units: epsilon = sigma = m = 1.
# ---------------------------------------------------------------------------
WCA_RC = 2.0 ** (1.0 / 6.0)
LJ_RC = 2.5


@dataclasses.dataclass(frozen=True)
class Potential:
    eps: float = 1.0
    sigma: float = 1.0
    rc: float = WCA_RC
    shift: int = 1  # 1: energy shifted to zero at r_c

    @property
    def name(self) -> str:
        return "wca" if abs(self.rc - WCA_RC) < 1e-12 else f"lj{self.rc:g}"


WCA = Potential(rc=WCA_RC)
LJ25 = Potential(rc=LJ_RC)

# ---------------------------------------------------------------------------
# lattice automorphisms (boundary-condition data)
# ---------------------------------------------------------------------------
# Planar elongation (Kraynik-Reinelt): the symmetric matrix whose eigenvectors
# give the initial basis, and the automorphism that the basis returns to after
# one period.  With Q's columns ordered by eigenvalue (golden ratio squared ->
# x, its inverse -> y, 1 -> z) and det Q = +1, L0^-1 exp(T A) L0 equals KR_M.
KR_S = np.array([[2, -1, 0], [-1, 1, 0], [0, 0, 1]], dtype=np.int32)
KR_M = np.array([[2, 1, 0], [1, 1, 0], [0, 0, 1]], dtype=np.int32)
KR_LAMBDA = (3.0 + math.sqrt(5.0)) / 2.0

# Generalised KR pair for 3D diagonal flows: two commuting symmetric
# unimodular matrices with independent log-eigenvalue vectors.
GKR_M1 = np.array([[1, -1, 0], [-1, 2, -1], [0, -1, 2]], dtype=np.int32)
GKR_M2 = ((GKR_M1 - np.eye(3, dtype=np.int32)) @ (GKR_M1 - np.eye(3, dtype=np.int32))).astype(np.int32)
# Lees-Edwards automorphism of planar shear (Sec. 2.2)
LE_M = np.array([[1, -1, 0], [0, 1, 0], [0, 0, 1]], dtype=np.int32)

FLOWS = ("planar", "uniaxial", "biaxial")


def flow_matrix(kind: str, rate: float) -> np.ndarray:
    """Traceless velocity-gradient matrix A of the background flow u = A x:
    diagonal for the elongational flows, A[0][1] = rate for planar shear."""
    if kind == "shear":
        A = np.zeros((3, 3))
        A[0, 1] = rate
        return A
    d = {"planar": (1.0, -1.0, 0.0),
         "uniaxial": (1.0, -0.5, -0.5),
         "biaxial": (0.5, 0.5, -1.0),
         "none": (0.0, 0.0, 0.0)}[kind]
    return np.diag(np.asarray(d, dtype=np.float64) * rate)


def _sorted_eigvecs(S: np.ndarray, order_values=None) -> np.ndarray:
    w, V = np.linalg.eigh(np.asarray(S, dtype=np.float64))
    if order_values is None:
        idx = np.argsort(-w)
    else:
        idx = [int(np.argmin(np.abs(w - v))) for v in order_values]
    V = V[:, idx].copy()
    if np.linalg.det(V) < 0:
        V[:, 2] *= -1.0
    return V


def kr_initial_basis(side: float) -> np.ndarray:
    """L0 = side * Q, Q's columns the unit eigenvectors of KR_S (ordered as above)."""
    Q = _sorted_eigvecs(KR_S, (KR_LAMBDA, 1.0 / KR_LAMBDA, 1.0))
    return side * Q


def gkr_initial_basis(side: float) -> np.ndarray:
    """L0 = side * V^T, V's columns the unit eigenvectors of GKR_M1, eigenvalues descending."""
    V = _sorted_eigvecs(GKR_M1)
    return side * V.T


def nominal_period(kind: str, rate: float) -> float:
    """Strain time after which the stretched lattice first coincides with itself
    (planar) or reaches the first remap scale (3D flows): log of the leading
    automorphism eigenvalue divided by the rate."""
    if kind == "planar":
        return math.log(KR_LAMBDA) / rate
    if kind == "shear":
        return 1.0 / rate
    lam1 = float(np.max(np.linalg.eigvalsh(GKR_M1.astype(np.float64))))
    return math.log(lam1) / rate


# ---------------------------------------------------------------------------
# a single box
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Box:
    name: str
    L0: np.ndarray            # 3x3, columns are the basis vectors
    A: np.ndarray             # 3x3 flow matrix
    t: float                  # strain time
    automorphisms: List[np.ndarray]   # [] (none), [M] (KR) or [M1, M2] (gKR)
    pot: Potential
    frac: np.ndarray          # N x 3 fractional coordinates in [0,1)
    jitter: Optional[np.ndarray] = None  # N x 3 Cartesian displacement or None
    flow: str = "none"
    rate: float = 0.0
    period: float = 0.0
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.frac.shape[0])

    def aut_array(self) -> Optional[np.ndarray]:
        """Automorphisms packed as int32[18] (M1 then M2, row-major); None if none."""
        if not self.automorphisms:
            return None
        out = np.zeros(18, dtype=np.int32)
        for k, M in enumerate(self.automorphisms):
            out[9 * k: 9 * k + 9] = np.asarray(M, dtype=np.int32).reshape(9)
        return out

    def positions(self, L: np.ndarray) -> np.ndarray:
        """Cartesian positions x = L s (+ jitter) for a basis L supplied by the caller."""
        x = self.frac @ np.asarray(L, dtype=np.float64).T
        if self.jitter is not None:
            x = x + self.jitter
        return np.ascontiguousarray(x)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def make_box(flow: str, rate: float, n: int, *, density: Optional[float] = None,
             side: Optional[float] = None, pot: Potential = WCA, t: Optional[float] = None,
             t_frac: Optional[float] = None, seed: int = 0, name: str = "box",
             grid: Optional[int] = None, jitter_sigma: float = 0.0) -> Box:
    """A box of n particles with initial side `side` (or (n/density)^(1/3)).

    flow in {"planar", "uniaxial", "biaxial", "shear", "none"}; planar uses
    the KR basis and automorphism, uniaxial/biaxial the generalised-KR pair,
    shear an axis-aligned cube with the Lees-Edwards automorphism, "none" an
    axis-aligned cube with no remapping.  The strain time is `t`, or
    `t_frac` times the nominal period.  Positions are uniform fractional
    coordinates, or a grid of grid^3 sites at (i+1/2)/grid plus Gaussian
    Cartesian jitter.
    """
    if side is None:
        side = (n / density) ** (1.0 / 3.0)
    g = _rng(seed)
    if grid is not None:
        ax = (np.arange(grid, dtype=np.float64) + 0.5) / grid
        c, b, a = np.meshgrid(ax, ax, ax, indexing="ij")
        frac = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)
        perm = g.permutation(frac.shape[0])
        frac = np.ascontiguousarray(frac[perm])
        n = frac.shape[0]
    else:
        frac = g.random((n, 3))
    jit = None
    if jitter_sigma > 0.0:
        jit = g.normal(0.0, jitter_sigma, size=(n, 3))
    A = flow_matrix(flow, rate)
    if flow == "planar":
        L0 = kr_initial_basis(side)
        auts = [KR_M.copy()]
    elif flow in ("uniaxial", "biaxial"):
        L0 = gkr_initial_basis(side)
        auts = [GKR_M1.copy(), GKR_M2.copy()]
    elif flow == "shear":
        L0 = np.eye(3) * side
        auts = [LE_M.copy()]
    else:
        L0 = np.eye(3) * side
        auts = []
    period = nominal_period(flow, rate) if flow != "none" and rate > 0 else 0.0
    if t is None:
        t = (t_frac or 0.0) * period
    return Box(name=name, L0=L0, A=A, t=float(t), automorphisms=auts, pot=pot, frac=frac,
               jitter=jit, flow=flow, rate=rate, period=period, seed=seed)


# ---------------------------------------------------------------------------
# the benchmark workloads
# ---------------------------------------------------------------------------
def wca_planar_4096(seed_offset: int = 0) -> Box:
    """4,096 WCA particles, rho = 0.8442, planar elongation (rate 0.1), t = T/2, uniform."""
    return make_box("planar", 0.1, 4096, density=0.8442, pot=WCA, t_frac=0.5,
                    seed=1000 + seed_offset, name="wca_planar_4096")


def lj_uniaxial_strain(k: int = 32, n: int = 1 << 20) -> Box:
    """1,048,576 LJ (r_c = 2.5) particles, rho = 0.8, uniaxial (rate 0.5), uniform.

    Strain sweep t_k = k T / 64, k = 0..63, with the fractional coordinates fixed
    (the configuration is carried affinely by the flow)."""
    return make_box("uniaxial", 0.5, n, density=0.8, pot=LJ25, t_frac=k / 64.0,
                    seed=2000, name=f"lj_uniaxial_{n}_k{k}")


def lj_biaxial_grid(grid: int = 256) -> Box:
    """16,777,216 LJ particles, rho = 0.8, biaxial (rate 0.2), t = T/2; grid + 0.05 jitter."""
    n = grid ** 3
    return make_box("biaxial", 0.2, n, density=0.8, pot=LJ25, t_frac=0.5, seed=3000,
                    name=f"lj_biaxial_{n}", grid=grid, jitter_sigma=0.05)


def wca_replica_batch(replicas: int = 512, n_lo: int = 2048, n_hi: int = 65536) -> List[Box]:
    """512 WCA replicas (rho = 0.8442), N log-uniform in [n_lo, n_hi], random flow,
    rate uniform in [0.01, 1], t uniform in [0, T)."""
    out = []
    for r in range(replicas):
        g = _rng(4000 + r)
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        flow = FLOWS[int(g.integers(0, 3))]
        rate = float(g.uniform(0.01, 1.0))
        tf = float(g.uniform(0.0, 1.0))
        out.append(make_box(flow, rate, n, density=0.8442, pot=WCA, t_frac=tf,
                            seed=40000 + r, name=f"rep{r}_{flow}"))
    return out


def lj_sllod_batch(replicas: int = 64, n_lo: int = 262144, n_hi: int = 2097152) -> List[Box]:
    """64 LJ replicas (rho = 0.8), N log-uniform in [n_lo, n_hi] rounded to the
    nearest cube g^3, mixed flows, rate uniform in [0.05, 0.5], starting at
    t = 0 from a g^3 grid of sites with 0.05 Gaussian jitter (uniform random
    sites overlap and would blow up under dynamics)."""
    out = []
    for r in range(replicas):
        g = _rng(5000 + r)
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        side = max(2, int(round(n ** (1.0 / 3.0))))
        flow = FLOWS[int(g.integers(0, 3))]
        rate = float(g.uniform(0.05, 0.5))
        out.append(make_box(flow, rate, side ** 3, density=0.8, pot=LJ25, t=0.0,
                            seed=50000 + r, name=f"nemd{r}_{flow}", grid=side, jitter_sigma=0.05))
    return out


def maxwell_momenta(n: int, temperature: float, seed: int, mass: float = 1.0) -> np.ndarray:
    """Gaussian peculiar momenta at temperature T* with zero total momentum."""
    g = _rng(seed)
    p = g.normal(0.0, math.sqrt(temperature * mass), size=(n, 3))
    p -= p.mean(axis=0, keepdims=True)
    return p


def random_unimodular(seed: int, steps: int = 6) -> np.ndarray:
    """A random integer 3x3 matrix with determinant 1 (product of elementary shears)."""
    g = _rng(seed)
    M = np.eye(3, dtype=np.int64)
    for _ in range(steps):
        i, j = g.choice(3, size=2, replace=False)
        E = np.eye(3, dtype=np.int64)
        E[i, j] = int(g.choice([-1, 1]))
        M = M @ E
    return M.astype(np.int32)


def random_rotation(seed: int) -> np.ndarray:
    g = _rng(seed)
    Qm, Rm = np.linalg.qr(g.normal(size=(3, 3)))
    Qm = Qm @ np.diag(np.sign(np.diag(Rm)))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] *= -1
    return Qm
