"""Python wrapper of the FP64 CPU oracle (``md_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the library product.  It
shares no code with the HIP path; the only thing both sides take from a
common module is the seeded input generator.

Arrays follow the input generator's convention: positions, velocities and
forces are float64 (N, 3), atoms in the caller's order, region
[-L/2, L/2)^3.  Soft-sphere potential: r_c = 2^(1/6), energy shift +1.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "md_oracle.c")
_LIB = os.path.join(_HERE, "libmd_oracle.so")

RC_SP = 2.0 ** (1.0 / 6.0)
TRACE_FIELDS = ("ke", "pe", "virial", "vmax2", "n_pairs", "rebuilt")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, strict IEEE)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("L", C.c_double), ("rc", C.c_double), ("shell", C.c_double),
                ("dt", C.c_double), ("ushift", C.c_double), ("G", C.c_int32),
                ("cell_only", C.c_int32), ("check_missed", C.c_int32), ("pad", C.c_int32)]


MAXSP = 4


class _Mix(C.Structure):
    _fields_ = [("ns", C.c_int32), ("pad", C.c_int32), ("sp", C.POINTER(C.c_int32)),
                ("eps", C.c_double * 16), ("sig2", C.c_double * 16), ("rc2", C.c_double * 16),
                ("shift", C.c_double * 16)]


class Mixture:
    """Species of the atoms and, per species pair (a, b), epsilon, sigma,
    cutoff and the energy shift added inside it (n_species x n_species,
    symmetric).  The pair energy is Eq. (1) in units of sigma_ab, eps_ab."""

    def __init__(self, species, epsilon, sigma, r_cut, shift):
        self.species = np.ascontiguousarray(species, dtype=np.int32)
        self.epsilon = np.asarray(epsilon, dtype=np.float64)
        self.sigma = np.asarray(sigma, dtype=np.float64)
        self.r_cut = np.asarray(r_cut, dtype=np.float64)
        self.shift = np.asarray(shift, dtype=np.float64)
        self.n_species = self.epsilon.shape[0]

    def struct(self) -> "_Mix":
        m = _Mix()
        m.ns = self.n_species
        m.sp = self.species.ctypes.data_as(C.POINTER(C.c_int32))
        for a in range(self.n_species):
            for b in range(self.n_species):
                k = a * MAXSP + b
                m.eps[k] = self.epsilon[a, b]
                m.sig2[k] = self.sigma[a, b] * self.sigma[a, b]
                m.rc2[k] = self.r_cut[a, b] * self.r_cut[a, b]
                m.shift[k] = self.shift[a, b]
        return m

    @property
    def max_cut(self) -> float:
        return float(self.r_cut.max())


def _mix_arg(mix):
    return C.byref(mix.struct()) if mix is not None else None


class _State(C.Structure):
    _fields_ = [("disp", C.c_double), ("step", C.c_int64), ("n_rebuilds", C.c_int64),
                ("n_missed", C.c_int64), ("rebuild", C.c_int32), ("pad", C.c_int32)]


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)
_I8 = C.POINTER(C.c_int8)


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.or_cells_per_edge.restype = C.c_int
        L.or_cells_per_edge.argtypes = [C.c_double, C.c_double, C.c_int]
        L.or_pair_potential.argtypes = [C.c_double, C.c_double, C.c_double, _D, _D]
        L.or_wrap.argtypes = [C.c_int64, _D, _D, _D, C.c_double]
        L.or_cell_ids.argtypes = [C.c_int64, _D, _D, _D, C.c_double, C.c_int, _I32]
        L.or_layers_reorder.restype = C.c_int
        L.or_layers_reorder.argtypes = [C.c_int64, _I32, C.c_int, _I32, _I64, _I64, _I32]
        for name in ("or_pairs_cells",):
            getattr(L, name).restype = C.c_int64
            getattr(L, name).argtypes = [C.c_int64, _D, _D, _D, C.c_double, C.c_int, C.c_double,
                                         C.c_int64, _I32, _I32, _I8]
        L.or_pairs_brute.restype = C.c_int64
        L.or_pairs_brute.argtypes = [C.c_int64, _D, _D, _D, C.c_double, C.c_double, C.c_int64,
                                     _I32, _I32, _I8]
        _M = C.POINTER(_Mix)
        L.or_forces_pairs.argtypes = [C.c_int64, _D, _D, _D, C.c_double, C.c_int64, _I32, _I32,
                                      _I8, C.c_double, C.c_double, _D, _D, _D, _D, _D, _D, _M]
        L.or_forces_cells.restype = C.c_int
        L.or_forces_cells.argtypes = [C.c_int64, _D, _D, _D, C.c_double, C.c_int, C.c_double,
                                      C.c_double, _D, _D, _D, _D, _D, _D, _M]
        L.or_forces_brute.argtypes = [C.c_int64, _D, _D, _D, C.c_double, C.c_double, C.c_double,
                                      _D, _D, _D, _D, _D, _D, _M]
        L.or_sim_set_mix.restype = C.c_int
        L.or_sim_set_mix.argtypes = [C.c_void_p, _M]
        L.or_force_on_atoms.argtypes = [C.c_int64, _D, _D, _D, C.c_double, C.c_double, C.c_double,
                                        C.c_int64, _I64, _D, _D, _D, _D, _D, _I32]
        L.or_neighbors_of_atom.restype = C.c_int64
        L.or_neighbors_of_atom.argtypes = [C.c_int64, _D, _D, _D, C.c_double, C.c_double,
                                           C.c_int64, C.c_int64, _I32]
        L.or_sim_new.restype = C.c_void_p
        L.or_sim_new.argtypes = [C.c_int64, _D, _D, C.POINTER(_Params), _D, C.POINTER(C.c_int)]
        L.or_sim_run.restype = C.c_int
        L.or_sim_run.argtypes = [C.c_void_p, C.c_int64, _D]
        L.or_sim_get.argtypes = [C.c_void_p, _D, _D, _D, C.POINTER(_State)]
        L.or_sim_pairs.restype = C.c_int64
        L.or_sim_pairs.argtypes = [C.c_void_p, C.c_int64, _I32, _I32, _I8]
        L.or_sim_free.argtypes = [C.c_void_p]
        L.or_sim_adjust_temp.restype = C.c_double
        L.or_sim_adjust_temp.argtypes = [C.c_void_p, C.c_double]
        _lib = L
    return _lib


def _p(a, t=_D):
    return a.ctypes.data_as(t)


def _soa(pos):
    pos = np.asarray(pos, dtype=np.float64)
    return [np.ascontiguousarray(pos[:, a]) for a in range(3)]


# --------------------------------------------------------------------------
# Geometry, potential, cells
# --------------------------------------------------------------------------

def cells_per_edge(L: float, rn: float, even: bool = False) -> int:
    """floor(L / r_n), or its even floor (the cell counts of Tables 1 and 5)."""
    return int(lib().or_cells_per_edge(L, rn, int(even)))


def pair_potential(r: float, rc: float = RC_SP, ushift: float = 1.0) -> Tuple[float, float]:
    """(u(r), -du/dr) for one separation; zero at and beyond r_c."""
    u, fr = C.c_double(), C.c_double()
    lib().or_pair_potential(r, rc, ushift, C.byref(u), C.byref(fr))
    return u.value, fr.value


def wrap(pos: np.ndarray, L: float) -> np.ndarray:
    x, y, z = _soa(pos)
    lib().or_wrap(len(x), _p(x), _p(y), _p(z), L)
    return np.stack([x, y, z], axis=1)


def cell_ids(pos: np.ndarray, L: float, G: int) -> np.ndarray:
    x, y, z = _soa(pos)
    cell = np.empty(len(x), dtype=np.int32)
    lib().or_cell_ids(len(x), _p(x), _p(y), _p(z), L, G, _p(cell, _I32))
    return cell


def layers_reorder(cell: np.ndarray, G: int):
    """Layer assignment and the cell-order reorder scan.

    Returns (layer[n], order[n], cell_start[G^3 + 1], n_layers)."""
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    n = len(cell)
    layer = np.empty(n, dtype=np.int32)
    order = np.empty(n, dtype=np.int64)
    cs = np.empty(G ** 3 + 1, dtype=np.int64)
    nl = C.c_int32()
    rc = lib().or_layers_reorder(n, _p(cell, _I32), G, _p(layer, _I32), _p(order, _I64),
                                 _p(cs, _I64), C.byref(nl))
    if rc != 0:
        raise MemoryError("oracle layers_reorder failed: %d" % rc)
    return layer, order, cs, nl.value


# --------------------------------------------------------------------------
# Pair lists
# --------------------------------------------------------------------------

def _pairs(fn, n, *args, cap=None):
    cap = cap if cap is not None else 16 * n + 64
    while True:
        pi = np.empty(max(cap, 1), dtype=np.int32)
        pj = np.empty(max(cap, 1), dtype=np.int32)
        img = np.empty((max(cap, 1), 3), dtype=np.int8)
        m = fn(*args, cap, _p(pi, _I32), _p(pj, _I32), _p(img, _I8))
        if m < 0:
            raise ValueError("oracle pair enumeration failed: %d" % m)
        if m <= cap:
            return pi[:m].copy(), pj[:m].copy(), img[:m].copy()
        cap = int(m)


def pairs_cells(pos, L, G, rn):
    """Half list (i', i'', image of i'') with r^2 < r_n^2, 14-cell traversal."""
    x, y, z = _soa(pos)
    return _pairs(lib().or_pairs_cells, len(x), len(x), _p(x), _p(y), _p(z), L, G, rn)


def pairs_brute(pos, L, rn):
    """All i < j over all 27 images with r^2 < r_n^2."""
    x, y, z = _soa(pos)
    return _pairs(lib().or_pairs_brute, len(x), len(x), _p(x), _p(y), _p(z), L, rn)


def pair_set(pi, pj):
    """Unordered pair set {(min, max)} as a sorted (M, 2) int64 array."""
    a = np.minimum(pi, pj).astype(np.int64)
    b = np.maximum(pi, pj).astype(np.int64)
    key = np.unique(a * (1 << 32) + b)
    return np.stack([key >> 32, key & 0xFFFFFFFF], axis=1)


# --------------------------------------------------------------------------
# Forces
# --------------------------------------------------------------------------

@dataclass
class Forces:
    force: np.ndarray     # (N, 3)
    u_atom: np.ndarray    # per-atom pair-energy sums (each pair on both atoms)
    w_atom: np.ndarray    # per-atom virial sums (each pair on both atoms)
    pe: float             # U = sum over pairs of u
    virial: float         # W = sum over pairs of f r^2
    n_inter: int          # pairs inside r_c


def _forces_out(n):
    return [np.empty(n) for _ in range(5)], np.empty(3)


def forces_pairs(pos, L, pi, pj, img, rc=RC_SP, ushift=1.0, mix=None) -> Forces:
    x, y, z = _soa(pos)
    n = len(x)
    (fx, fy, fz, ua, wa), out = _forces_out(n)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    img = np.ascontiguousarray(img, dtype=np.int8)
    lib().or_forces_pairs(n, _p(x), _p(y), _p(z), L, len(pi), _p(pi, _I32), _p(pj, _I32),
                          _p(img, _I8), mix.max_cut if mix is not None else rc, ushift,
                          _p(fx), _p(fy), _p(fz), _p(ua), _p(wa), _p(out), _mix_arg(mix))
    return Forces(np.stack([fx, fy, fz], axis=1), ua, wa, out[0], out[1], int(out[2]))


def forces_cells(pos, L, G, rc=RC_SP, ushift=1.0, mix=None) -> Forces:
    x, y, z = _soa(pos)
    n = len(x)
    (fx, fy, fz, ua, wa), out = _forces_out(n)
    rcode = lib().or_forces_cells(n, _p(x), _p(y), _p(z), L, G,
                                  mix.max_cut if mix is not None else rc, ushift, _p(fx),
                                  _p(fy), _p(fz), _p(ua), _p(wa), _p(out), _mix_arg(mix))
    if rcode != 0:
        raise ValueError("oracle forces_cells failed: %d" % rcode)
    return Forces(np.stack([fx, fy, fz], axis=1), ua, wa, out[0], out[1], int(out[2]))


def forces_brute(pos, L, rc=RC_SP, ushift=1.0, mix=None) -> Forces:
    x, y, z = _soa(pos)
    n = len(x)
    (fx, fy, fz, ua, wa), out = _forces_out(n)
    lib().or_forces_brute(n, _p(x), _p(y), _p(z), L, mix.max_cut if mix is not None else rc,
                          ushift, _p(fx), _p(fy), _p(fz), _p(ua), _p(wa), _p(out),
                          _mix_arg(mix))
    return Forces(np.stack([fx, fy, fz], axis=1), ua, wa, out[0], out[1], int(out[2]))


def force_on_atoms(pos, L, idx, rc=RC_SP, ushift=1.0):
    """Per-atom force, u, w and interacting-pair count of atoms ``idx``, each
    summed on its own over every other atom (minimum image)."""
    x, y, z = _soa(pos)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    k = len(idx)
    fx, fy, fz, u, w = (np.empty(k) for _ in range(5))
    cnt = np.empty(k, dtype=np.int32)
    lib().or_force_on_atoms(len(x), _p(x), _p(y), _p(z), L, rc, ushift, k, _p(idx, _I64),
                            _p(fx), _p(fy), _p(fz), _p(u), _p(w), _p(cnt, _I32))
    return np.stack([fx, fy, fz], axis=1), u, w, cnt


def neighbors_of_atom(pos, L, rn, i, _soa_cache=None):
    """Sorted indices j != i with r^2 < r_n^2 (minimum image)."""
    x, y, z = _soa_cache if _soa_cache is not None else _soa(pos)
    cap = 256
    while True:
        out = np.empty(cap, dtype=np.int32)
        m = lib().or_neighbors_of_atom(len(x), _p(x), _p(y), _p(z), L, rn, int(i), cap,
                                       _p(out, _I32))
        if m <= cap:
            return out[:m].copy()
        cap = int(m)


# --------------------------------------------------------------------------
# The MD loop
# --------------------------------------------------------------------------

class Sim:
    """Oracle trajectory: step 0 at construction, then ``run(n)`` steps.

    ``trace`` rows hold (ke, pe, virial, vmax2, n_pairs, rebuilt) per step,
    as totals (not per atom)."""

    def __init__(self, pos, vel, L, *, shell=0.4, dt=0.005, rc=RC_SP, ushift=1.0,
                 even_cells=False, check_missed=False):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        self.n = len(pos)
        cell_only = shell == 0.0
        G = cells_per_edge(L, rc + shell, even_cells)
        self.G = G
        self.L = L
        self._p = _Params(L, rc, shell, dt, ushift, G, int(cell_only), int(check_missed), 0)
        rec = np.zeros(6)
        err = C.c_int()
        self._h = lib().or_sim_new(self.n, _p(pos), _p(vel), C.byref(self._p), _p(rec),
                                   C.byref(err))
        if not self._h:
            raise ValueError("oracle sim creation failed: %d" % err.value)
        self.start = rec

    def run(self, nsteps: int) -> np.ndarray:
        trace = np.zeros((max(nsteps, 1), 6))
        rc = lib().or_sim_run(self._h, nsteps, _p(trace))
        if rc != 0:
            raise RuntimeError("oracle run failed: %d" % rc)
        return trace[:nsteps]

    def state(self):
        pos = np.empty((self.n, 3))
        vel = np.empty((self.n, 3))
        frc = np.empty((self.n, 3))
        st = _State()
        lib().or_sim_get(self._h, _p(pos), _p(vel), _p(frc), C.byref(st))
        return pos, vel, frc, st

    def pairs(self):
        cap = 16 * self.n + 64
        while True:
            pi = np.empty(cap, dtype=np.int32)
            pj = np.empty(cap, dtype=np.int32)
            img = np.empty((cap, 3), dtype=np.int8)
            m = lib().or_sim_pairs(self._h, cap, _p(pi, _I32), _p(pj, _I32), _p(img, _I8))
            if m <= cap:
                return pi[:m].copy(), pj[:m].copy(), img[:m].copy()
            cap = int(m)

    def set_species(self, mix: "Mixture") -> None:
        """Several species (the pair cutoffs at most this Sim's rc); the
        forces of the current state are evaluated again."""
        self._mix = mix
        rc = lib().or_sim_set_mix(self._h, C.byref(mix.struct()))
        if rc != 0:
            raise ValueError("oracle set_species failed: %d" % rc)

    def adjust_temp(self, temperature: float) -> float:
        """Step (f): scale the velocities to sum v^2 = 3 (N - 1) T; returns
        the factor."""
        return float(lib().or_sim_adjust_temp(self._h, float(temperature)))

    def equilibrate_run(self, nsteps: int, temperature: float, equil_steps: int = 500,
                        interval: int = 20) -> np.ndarray:
        """``run`` with the equilibration of Sec. 5.1 folded in: after step k
        (absolute count) with k <= equil_steps and k a multiple of interval,
        the velocities are adjusted to T.  Properties of step k in the trace
        are those of (e), before the adjustment."""
        out = []
        done = int(self.state()[3].step)
        end = done + nsteps
        while done < end:
            nxt = end
            if done < equil_steps:
                nxt = min(end, (done // interval + 1) * interval)
            out.append(self.run(nxt - done))
            done = nxt
            if done <= equil_steps and done % interval == 0:
                self.adjust_temp(temperature)
        return np.concatenate(out) if out else np.zeros((0, len(TRACE_FIELDS)))

    def close(self):
        if getattr(self, "_h", None):
            lib().or_sim_free(self._h)
            self._h = None

    def __del__(self):
        self.close()


def block_means(trace: np.ndarray, n_atoms: int, first: int, last: int) -> dict:
    """Means over steps first..last (1-based, inclusive) of a trace that starts
    at step 1: per-atom kinetic, potential and total energy and virial, and
    the mean neighbour-list length per atom (twice the pairs per atom, the
    quantity the paper tabulates as neighbours per atom).  Sec. 5.1 averages
    properties over blocks of 1000 steps."""
    rows = trace[first - 1:last]
    ke = rows[:, 0].mean() / n_atoms
    pe = rows[:, 1].mean() / n_atoms
    return {"steps": len(rows), "ke_per_atom": ke, "pe_per_atom": pe,
            "etot_per_atom": ke + pe, "virial_per_atom": rows[:, 2].mean() / n_atoms,
            "nebr_per_atom": 2.0 * rows[:, 4].mean() / n_atoms}
