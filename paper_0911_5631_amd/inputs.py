"""Seeded synthetic inputs for soft-sphere molecular dynamics.

This module only *generates inputs*: lattice starts, random velocity
directions, jittered (off-lattice) states and the named workloads.  It holds
none of the method's arithmetic (no cells, lists, forces or integration), so
both the HIP path and the CPU oracle can consume what it produces.

Conventions (reduced units, sigma = epsilon = m = 1):

* The periodic region is the cube [-L/2, L/2)^3 centred at the origin, with
  L = (N / rho)^(1/3) (the paper's edge formula for a lattice start).
* Positions and velocities are float64 arrays of shape (N, 3).
* Initial velocities have magnitude sqrt(3 T) in uniformly random directions,
  then the mean is subtracted so the centre of mass is at rest (the paper's
  initial state).  No rescaling follows the mean subtraction.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional

import numpy as np

#: Soft-sphere cutoff 2^(1/6): the minimum of the Lennard-Jones potential.
RC_SOFT_SPHERE = 2.0 ** (1.0 / 6.0)

# fcc basis in units of the cubic lattice constant.
_FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])


def box_edge(n_atoms: int, rho: float) -> float:
    """Edge L of the cubic region holding ``n_atoms`` at number density rho."""
    return (n_atoms / rho) ** (1.0 / 3.0)


def fcc_lattice(n_cells: int, rho: float):
    """fcc start: ``n_cells``^3 cubic unit cells of 4 atoms each.

    Atom k sits at a*(n + basis + 1/4) - L/2 with a = L/n_cells; the 1/4
    offset keeps every atom away from cell faces and from the region edge.
    Atoms are numbered with x fastest, then y, then z, then the basis index
    varying fastest of all.  Returns (pos (N,3) float64, L).
    """
    n = 4 * n_cells ** 3
    L = box_edge(n, rho)
    a = L / n_cells
    g = np.arange(n_cells, dtype=np.float64)
    iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
    origin = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    pos = (origin[:, None, :] + _FCC_BASIS[None, :, :] + 0.25).reshape(-1, 3)
    pos = pos * a - 0.5 * L
    return np.ascontiguousarray(pos), L


def sc_lattice(n_edge: int, rho: float):
    """Simple-cubic start of edge ``n_edge`` (the paper's own initial state).

    Atom k sits at a*(n + 1/2) - L/2 with a = L/n_edge.  Returns (pos, L).
    """
    n = n_edge ** 3
    L = box_edge(n, rho)
    a = L / n_edge
    g = np.arange(n_edge, dtype=np.float64)
    iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
    pos = (np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1) + 0.5) * a - 0.5 * L
    return np.ascontiguousarray(pos), L


def random_velocities(n_atoms: int, temperature: float, seed: int) -> np.ndarray:
    """Velocities of magnitude sqrt(3T), uniform random directions, zero mean.

    Directions: z ~ U[-1, 1], phi ~ U[0, 2pi) from a seeded PCG64 stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cz = rng.uniform(-1.0, 1.0, n_atoms)
    phi = rng.uniform(0.0, 2.0 * math.pi, n_atoms)
    s = np.sqrt(1.0 - cz * cz)
    vel = np.stack([s * np.cos(phi), s * np.sin(phi), cz], axis=1) * math.sqrt(3.0 * temperature)
    vel -= vel.mean(axis=0, keepdims=True)
    return np.ascontiguousarray(vel)


def jitter(pos: np.ndarray, L: float, amplitude: float, seed: int) -> np.ndarray:
    """Displace every coordinate by U[-amplitude, amplitude], then fold the
    result into [-L/2, L/2) (an off-lattice state with non-zero forces)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = pos + rng.uniform(-amplitude, amplitude, pos.shape)
    out = out - L * np.floor(out / L + 0.5)
    out[out >= 0.5 * L] -= L
    return np.ascontiguousarray(out)


def shuffled(pos: np.ndarray, vel: np.ndarray, seed: int):
    """The same atoms in a seeded random storage order."""
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(pos))
    return np.ascontiguousarray(pos[perm]), np.ascontiguousarray(vel[perm])


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class System:
    """One soft-sphere system ready to hand to either implementation."""
    name: str
    pos: np.ndarray
    vel: np.ndarray
    box: float
    rho: float
    temperature: float
    dt: float
    shell: float          # neighbour shell delta; 0 => cell-list-only mode
    steps: int
    precision: str        # "fp32" (FP32 forces, FP64 state) or "fp64"
    seed: int

    @property
    def n(self) -> int:
        return len(self.pos)


def fcc_system(name: str, n_cells: int, rho: float, temperature: float, *,
               dt: float = 0.005, shell: float = 0.4, steps: int = 1000,
               precision: str = "fp32", seed: int = 0) -> System:
    pos, L = fcc_lattice(n_cells, rho)
    vel = random_velocities(len(pos), temperature, seed)
    return System(name, pos, vel, L, rho, temperature, dt, shell, steps, precision, seed)


def sp_small_cells() -> System:
    """N = 2048 (fcc 8^3 x 4), rho 0.8, T 1, dt 0.005, 1000 steps, cell list
    only (no neighbour shell), FP64 throughout."""
    return fcc_system("sp_2048_cells_fp64", 8, 0.8, 1.0, shell=0.0, steps=1000,
                      precision="fp64", seed=1)


def sp_256k() -> System:
    """N = 256 000 (fcc 40^3 x 4), rho 0.8, T 1, shell 0.4, 10 000 steps,
    FP32 forces with FP64 positions and velocities."""
    return fcc_system("sp_256000_nebr_fp32", 40, 0.8, 1.0, shell=0.4, steps=10000,
                      precision="fp32", seed=2)


def system_s(shell: float = 0.6, seed: int = 6, n_edge: int = 48) -> System:
    """The paper's system S (Secs. 5.1 and 5.3): simple cubic start of edge 48 (110 592
    atoms), rho 0.8, T 1, dt 0.005, FP32 forces; shell 0.6 unless given (the
    Table 5 runs vary it).  2000 steps: the Sec. 5.1 equilibration (adjustment
    every 20 steps for 500) and the block of steps 1001-2000 of Table 4."""
    pos, L = sc_lattice(n_edge, 0.8)
    vel = random_velocities(len(pos), 1.0, seed)
    return System(f"system_S_{len(pos)}_shell{shell}", pos, vel, L, 0.8, 1.0, 0.005, shell,
                  2000, "fp32", seed)


def binary_wca(sig_aa: float = 1.0, sig_bb: float = 1.2, eps_ab: float = 1.5):
    """Pair tables of a soft-sphere (WCA) binary mixture: sigma_ab the mean of
    the two diameters, epsilon 1 for like pairs and eps_ab for unlike ones,
    cutoff 2^(1/6) sigma_ab and shift epsilon_ab (so u(r_c) = 0).  Returns
    (epsilon, sigma, r_cut, shift), each 2 x 2."""
    sab = 0.5 * (sig_aa + sig_bb)
    sig = np.array([[sig_aa, sab], [sab, sig_bb]])
    eps = np.array([[1.0, eps_ab], [eps_ab, 1.0]])
    return eps, sig, RC_SOFT_SPHERE * sig, eps.copy()


def mixture_256k(seed: int = 9):
    """N = 256 000 (fcc 40^3 x 4) at rho 0.75, T 1, shell 0.4: half the atoms
    (seeded random choice) of species B, the binary_wca() tables.  Returns
    (System, species)."""
    sys_ = fcc_system("binary_wca_256000", 40, 0.75, 1.0, shell=0.4, steps=2000,
                      precision="fp32", seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    species = (rng.permutation(sys_.n) < sys_.n // 2).astype(np.int32)
    return sys_, species


def sp_4m() -> System:
    """N = 4 000 000 (fcc 100^3 x 4), rho 0.8, T 1, shell 0.4, 2000 steps."""
    return fcc_system("sp_4000000_nebr_fp32", 100, 0.8, 1.0, shell=0.4, steps=2000,
                      precision="fp32", seed=3)


def sp_33m() -> System:
    """N = 33 461 708 (fcc 203^3 x 4: the largest fcc start under the 25-bit
    storage index, 2^25 - 1 atoms), rho 0.8, T 1, shell 0.4, 500 steps."""
    return fcc_system("sp_33461708_nebr_fp32", 203, 0.8, 1.0, shell=0.4, steps=500,
                      precision="fp32", seed=4)


def _replica_seed(seed: int, index: int) -> int:
    # SplitMix64-style mixing of (seed, index) into an independent stream seed.
    z = (seed * 0x9E3779B97F4A7C15 + (index + 1) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


def replica_batch(n_replicas: int = 256, k_lo: int = 6, k_hi: int = 20, steps: int = 5000,
                  seed: int = 4, shell: float = 0.4) -> List[System]:
    """Independent replicas of uneven size: N = 4 k^3 with k ~ U{k_lo..k_hi},
    rho ~ U[0.7, 0.9], T ~ U[0.8, 1.5], dt 0.005, FP32 forces / FP64 state."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(n_replicas):
        k = int(rng.integers(k_lo, k_hi + 1))
        rho = float(rng.uniform(0.7, 0.9))
        T = float(rng.uniform(0.8, 1.5))
        out.append(fcc_system(f"replica{r}", k, rho, T, shell=shell, steps=steps,
                              precision="fp32", seed=_replica_seed(seed, r)))
    return out


@dataclasses.dataclass
class Request:
    """One served request: its arrival time and the parameters of its system.
    The positions and velocities are generated only when asked for (a trace of
    requests up to 5e5 atoms each stays small until admission)."""
    arrival: float        # seconds after the stream starts
    name: str
    n_cells: int          # fcc unit cells per edge: N = 4 n_cells^3
    rho: float
    temperature: float
    steps: int
    seed: int
    shell: float = 0.4

    @property
    def n(self) -> int:
        return 4 * self.n_cells ** 3

    def system(self) -> System:
        return fcc_system(self.name, self.n_cells, self.rho, self.temperature,
                          shell=self.shell, steps=self.steps, precision="fp32", seed=self.seed)


def served_stream(n_requests: int = 256, rate: float = 50.0, k_lo: int = 6, k_hi: int = 50,
                  steps_lo: int = 1000, steps_hi: int = 20000, seed: int = 5,
                  shell: float = 0.4) -> List[Request]:
    """Poisson arrivals (mean ``rate`` per second) of systems N = 4 k^3,
    k ~ U{k_lo..k_hi}, rho ~ U[0.7, 0.9], T ~ U[0.8, 1.5], steps ~
    U{steps_lo..steps_hi}.  A finite trace of ``n_requests``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for r in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        k = int(rng.integers(k_lo, k_hi + 1))
        rho = float(rng.uniform(0.7, 0.9))
        T = float(rng.uniform(0.8, 1.5))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        out.append(Request(t, f"request{r}", k, rho, T, steps, _replica_seed(seed, r), shell))
    return out
