"""Python binding of the soft-sphere MD library (argument marshalling only).

The functions below carry the C ABI's names (md_create, md_bin_cells,
md_build_nebr, md_forces, md_step, md_props, ...) and the classes System and
Batch wrap the same calls.  Every step of the method runs in the gfx950
library; this module only converts numpy arrays to pointers.  PyTorch
provides device memory (its caching allocator, through the library's
allocator hook) and the stream the work is ordered on.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Tuple

import numpy as np

from . import _lib as L
from ._lib import MDError, check, lib

RC_SOFT_SPHERE = 2.0 ** (1.0 / 6.0)

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)


def _dptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_D)


def _rows(a, n: int, name: str) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n, 3):
        raise ValueError(f"{name} must have shape ({n}, 3), got {a.shape}")
    return a


class TorchAllocator:
    """md_allocator backed by torch's CUDA caching allocator on one device/stream."""

    def __init__(self, device: Optional[int] = None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required: torch.cuda is not available")
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self._torch = torch

        def _alloc(nbytes, _ctx):
            try:
                return self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                                self.stream)
            except Exception:  # noqa: BLE001 - out of memory reported as NULL
                return None

        def _free(ptr, _ctx):
            # during interpreter shutdown torch may already be torn down; the
            # process then returns the memory anyway
            cuda = getattr(self._torch, "cuda", None)
            if ptr and cuda is not None and getattr(cuda, "caching_allocator_delete", None):
                cuda.caching_allocator_delete(ptr)

        self._alloc_cb = L.ALLOC_FN(_alloc)
        self._free_cb = L.FREE_FN(_free)
        self.struct = L.md_allocator(self._alloc_cb, self._free_cb, None)

    @property
    def stream_handle(self) -> int:
        return int(self.stream.cuda_stream)


def make_params(n_atoms: int, box: float, *, r_cut: float = RC_SOFT_SPHERE, shell: float = 0.4,
                dt: float = 0.005, precision: str = "fp32", nebr_cap: int = 0,
                cell_cap: int = 0, even_cells: bool = False,
                trace: bool = False, reorder: bool = True,
                reorder_interval: int = 0, window: bool = True) -> L.md_params:
    prec = {"fp32": L.MD_FORCE_FP32, "fp64": L.MD_FORCE_FP64}[precision]
    flags = ((L.MD_EVEN_CELLS if even_cells else 0) | (L.MD_TRACE_PROPS if trace else 0) |
             (0 if reorder else L.MD_NO_REORDER) | (0 if window else L.MD_NO_WINDOW))
    return L.md_params(int(n_atoms), float(box), float(r_cut), float(shell), float(dt), prec,
                       int(nebr_cap), int(cell_cap), flags, int(reorder_interval))


def _trace_array(rows) -> np.ndarray:
    """md_trace_t rows as a structured array (step, ke, pe, virial, vmax)."""
    out = np.empty(len(rows), dtype=[("step", np.int64), ("ke", np.float64),
                                     ("pe", np.float64), ("virial", np.float64),
                                     ("vmax", np.float64)])
    for k, r in enumerate(rows):
        out[k] = (r.step, r.ke, r.pe, r.virial, r.vmax)
    return out


def md_cells_per_edge(params: L.md_params) -> int:
    g = C.c_int32()
    check(lib().md_cells_per_edge(C.byref(params), C.byref(g)), "md_cells_per_edge")
    return g.value


def md_query_bytes(params: L.md_params) -> int:
    b = C.c_size_t()
    check(lib().md_query_bytes(C.byref(params), C.byref(b)), "md_query_bytes")
    return b.value


def _props_dict(p: L.md_props_t) -> Dict[str, float]:
    return {name: getattr(p, name) for name, _ in L.md_props_t._fields_}


def _launch_dict(cfg: L.md_launch_t) -> Dict[str, int]:
    return {name: getattr(cfg, name) for name, _ in L.md_launch_t._fields_}


class System:
    """One periodic soft-sphere system resident on the GPU (md_create)."""

    def __init__(self, pos, vel, box: float, *, allocator: str = "torch", stream=None,
                 **params):
        pos = np.asarray(pos, dtype=np.float64)
        n = len(pos)
        self.n = n
        self.params = make_params(n, box, **params)
        pos = _rows(pos, n, "pos")
        vel = _rows(vel, n, "vel")
        self._alloc = None
        stream_handle = None
        if allocator == "torch":
            self._alloc = TorchAllocator(stream=stream)
            stream_handle = self._alloc.stream_handle
        elif allocator is not None and allocator != "hip":
            raise ValueError("allocator must be 'torch', 'hip' or None")
        h = C.c_void_p()
        alloc_ptr = C.byref(self._alloc.struct) if self._alloc else None
        check(lib().md_create(C.byref(self.params), _dptr(pos), _dptr(vel), alloc_ptr,
                              stream_handle, C.byref(h)), "md_create")
        self._h = h

    # -- the method's steps ----------------------------------------------
    def bin_cells(self) -> None:
        check(lib().md_bin_cells(self._h), "md_bin_cells")

    def build_nebr(self) -> None:
        check(lib().md_build_nebr(self._h), "md_build_nebr")

    def forces(self) -> None:
        check(lib().md_forces(self._h), "md_forces")

    def step(self, n_steps: int) -> None:
        check(lib().md_step(self._h, int(n_steps)), "md_step")

    def props(self) -> Dict[str, float]:
        p = L.md_props_t()
        check(lib().md_props(self._h, C.byref(p)), "md_props")
        return _props_dict(p)

    def set_species(self, species, epsilon, sigma, r_cut, shift) -> None:
        """Several species: per-atom species (original order) and per species
        pair epsilon, sigma, cutoff and energy shift (n x n, symmetric)."""
        species = np.ascontiguousarray(species, dtype=np.int32)
        if species.shape != (self.n,):
            raise ValueError("species must have one entry per atom")
        tabs = [np.ascontiguousarray(t, dtype=np.float64) for t in (epsilon, sigma, r_cut, shift)]
        ns = tabs[0].shape[0]
        if any(t.shape != (ns, ns) for t in tabs):
            raise ValueError("pair tables must be n_species x n_species")
        check(lib().md_set_species(self._h, ns, species.ctypes.data_as(_I32),
                                   *[_dptr(t) for t in tabs]), "md_set_species")

    def adjust_temp(self, temperature: float) -> None:
        """Step (f): scale the velocities to sum v^2 = 3 (N - 1) T (async)."""
        check(lib().md_adjust_temp(self._h, float(temperature)), "md_adjust_temp")

    def equilibrate_run(self, n_steps: int, temperature: float, equil_steps: int = 500,
                        interval: int = 20) -> None:
        """md_step with the equilibration of Sec. 5.1 folded in: after every
        step k (absolute count) with k <= equil_steps and k a multiple of
        interval, md_adjust_temp(temperature).  One synchronisation to read
        the step count; the rest is enqueued."""
        done = int(self.props()["step"])
        end = done + int(n_steps)
        while done < end:
            nxt = end
            if done < equil_steps:
                nxt = min(end, (done // interval + 1) * interval)
            self.step(nxt - done)
            done = nxt
            if done <= equil_steps and done % interval == 0:
                self.adjust_temp(temperature)

    def block_begin(self) -> None:
        check(lib().md_block_begin(self._h), "md_block_begin")

    def block_end(self) -> Dict[str, float]:
        b = L.md_block_t()
        check(lib().md_block_end(self._h, C.byref(b)), "md_block_end")
        return {name: getattr(b, name) for name, _ in L.md_block_t._fields_}

    # -- state access (original atom order) --------------------------------
    def get_state(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray, int]:
        pos = np.empty((self.n, 3))
        vel = np.empty((self.n, 3))
        frc = np.empty((self.n, 3))
        step = C.c_int64()
        check(lib().md_get_state(self._h, _dptr(pos), _dptr(vel), _dptr(frc), C.byref(step)),
              "md_get_state")
        return pos, vel, frc, step.value

    def atom_energies(self) -> Tuple[np.ndarray, np.ndarray]:
        u = np.empty(self.n)
        w = np.empty(self.n)
        check(lib().md_get_atom_energies(self._h, _dptr(u), _dptr(w)), "md_get_atom_energies")
        return u, w

    def set_state(self, pos, vel) -> None:
        pos = _rows(pos, self.n, "pos")
        vel = _rows(vel, self.n, "vel")
        check(lib().md_set_state(self._h, _dptr(pos), _dptr(vel)), "md_set_state")

    def cells(self) -> np.ndarray:
        c = np.empty(self.n, dtype=np.int32)
        check(lib().md_get_cells(self._h, c.ctypes.data_as(_I32)), "md_get_cells")
        return c

    def bins(self) -> Tuple[np.ndarray, np.ndarray]:
        G = md_cells_per_edge(self.params)
        order = np.empty(self.n, dtype=np.int32)
        cs = np.empty(G ** 3 + 1, dtype=np.int32)
        check(lib().md_get_bins(self._h, order.ctypes.data_as(_I32), cs.ctypes.data_as(_I32)),
              "md_get_bins")
        return order, cs

    def pairs(self) -> Tuple[np.ndarray, np.ndarray]:
        n = C.c_int64()
        check(lib().md_get_pairs(self._h, 0, None, None, C.byref(n)), "md_get_pairs")
        cap = n.value
        pi = np.empty(max(cap, 1), dtype=np.int32)
        pj = np.empty(max(cap, 1), dtype=np.int32)
        check(lib().md_get_pairs(self._h, cap, pi.ctypes.data_as(_I32), pj.ctypes.data_as(_I32),
                                 C.byref(n)), "md_get_pairs")
        return pi[:n.value], pj[:n.value]

    def newton3_ab(self, variant="full", reps: int = 1, noalloc: bool = False) -> Dict[str, object]:
        """Neighbour-list A/B at the held state: variant "full" (one thread
        per atom), "half" (Newton's third law, reactions by atomics) or
        "cells" (the cell-centric build; a bool selects half / full):
        forces (original order), mean build and force kernel times (ms), list
        entries.  noalloc: the entry point that allocates no device memory
        (md_newton3_ab_noalloc)."""
        if isinstance(variant, bool):
            variant = "half" if variant else "full"
        f = np.empty((self.n, 3))
        b = C.c_double()
        t = C.c_double()
        k = C.c_int64()
        fn = lib().md_newton3_ab_noalloc if noalloc else lib().md_newton3_ab
        check(fn(self._h, L.AB_VARIANTS[variant], int(reps), _dptr(f), C.byref(b), C.byref(t),
                 C.byref(k)), "md_newton3_ab_noalloc" if noalloc else "md_newton3_ab")
        return {"force": f, "build_ms": b.value, "force_ms": t.value, "n_entries": k.value}

    def ab_pairs(self, variant: str = "full") -> Tuple[np.ndarray, np.ndarray]:
        """The A/B list of ``variant`` built at the held state, as (i, j)
        original indices (md_ab_pairs)."""
        n = C.c_int64()
        v = L.AB_VARIANTS[variant]
        check(lib().md_ab_pairs(self._h, v, 0, None, None, C.byref(n)), "md_ab_pairs")
        cap = n.value
        pi = np.empty(max(cap, 1), dtype=np.int32)
        pj = np.empty(max(cap, 1), dtype=np.int32)
        check(lib().md_ab_pairs(self._h, v, cap, pi.ctypes.data_as(_I32), pj.ctypes.data_as(_I32),
                                C.byref(n)), "md_ab_pairs")
        return pi[:n.value], pj[:n.value]

    # -- measurement ---------------------------------------------------------
    def profile(self, enable: bool) -> None:
        check(lib().md_profile(self._h, 1 if enable else 0), "md_profile")

    def kernel_time(self) -> Tuple[int, float]:
        k = C.c_int64()
        ms = C.c_double()
        check(lib().md_kernel_time(self._h, C.byref(k), C.byref(ms)), "md_kernel_time")
        return k.value, ms.value

    def configure(self, steps_per_run: int = 0, grid: int = 0, sort_grid: int = 0,
                  sort_split: int = 0, tile_order: int = 0) -> Dict[str, int]:
        """Launch configuration of later steps (changes no arithmetic); 0 asks
        for the library's choice.  Returns the configuration in use."""
        cfg = L.md_launch_t(int(steps_per_run), int(grid), int(sort_grid), int(sort_split),
                            int(tile_order))
        check(lib().md_configure(self._h, C.byref(cfg)), "md_configure")
        return _launch_dict(cfg)

    def trace(self, first_step: int, count: int) -> np.ndarray:
        """Per-step KE, PE, virial and max |v| of steps first_step ..
        first_step + count - 1 (created with trace=True)."""
        rows = (L.md_trace_t * max(int(count), 1))()
        check(lib().md_get_trace(self._h, int(first_step), int(count), rows), "md_get_trace")
        return _trace_array(rows[:int(count)])

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().md_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many independent systems advanced by the same kernel launches."""

    def __init__(self, hbm_budget: int, max_slots: int, steps_per_run: int = 64, *,
                 allocator: str = "torch", stream=None):
        self._alloc = TorchAllocator(stream=stream) if allocator == "torch" else None
        h = C.c_void_p()
        check(lib().md_batch_create(int(hbm_budget), int(max_slots), int(steps_per_run),
                                    C.byref(self._alloc.struct) if self._alloc else None,
                                    self._alloc.stream_handle if self._alloc else None,
                                    C.byref(h)), "md_batch_create")
        self._h = h
        self.max_slots = max_slots
        self.steps_per_run = int(steps_per_run)
        self.n_of = {}

    def admit(self, pos, vel, box: float, n_steps: int, **params) -> int:
        """Slot of the admitted system, or raises MDError (MD_ERR_OOM /
        MD_ERR_NO_SLOT mean: try again later)."""
        pos = np.asarray(pos, dtype=np.float64)
        n = len(pos)
        prm = make_params(n, box, **params)
        slot = C.c_int32()
        check(lib().md_batch_admit(self._h, C.byref(prm), _dptr(_rows(pos, n, "pos")),
                                   _dptr(_rows(vel, n, "vel")), int(n_steps), C.byref(slot)),
              "md_batch_admit")
        self.n_of[slot.value] = n
        return slot.value

    def try_admit(self, pos, vel, box: float, n_steps: int, **params) -> Optional[int]:
        try:
            return self.admit(pos, vel, box, n_steps, **params)
        except MDError as e:
            if e.code in (-3, -9):
                return None
            raise

    def configure(self, steps_per_run: int = 0, grid: int = 0, sort_grid: int = 0,
                  sort_split: int = 0, tile_order: int = 0) -> Dict[str, int]:
        """Launch configuration of later runs (changes no arithmetic); 0 asks
        for the library's choice.  Returns the configuration in use."""
        cfg = L.md_launch_t(int(steps_per_run), int(grid), int(sort_grid), int(sort_split),
                            int(tile_order))
        check(lib().md_batch_configure(self._h, C.byref(cfg)), "md_batch_configure")
        self.steps_per_run = cfg.steps_per_run
        return _launch_dict(cfg)

    def run(self) -> None:
        check(lib().md_batch_run(self._h), "md_batch_run")

    def poll(self):
        done = np.empty(self.max_slots, dtype=np.int32)
        k = C.c_int32()
        check(lib().md_batch_poll(self._h, done.ctypes.data_as(_I32), self.max_slots, C.byref(k)),
              "md_batch_poll")
        return [int(s) for s in done[:k.value]]

    def props(self, slot: int) -> Dict[str, float]:
        p = L.md_props_t()
        check(lib().md_batch_props(self._h, int(slot), C.byref(p)), "md_batch_props")
        return _props_dict(p)

    def get_state(self, slot: int):
        n = self.n_of[slot]
        pos = np.empty((n, 3))
        vel = np.empty((n, 3))
        step = C.c_int64()
        check(lib().md_batch_get_state(self._h, int(slot), _dptr(pos), _dptr(vel),
                                       C.byref(step)), "md_batch_get_state")
        return pos, vel, step.value

    def trace(self, slot: int, first_step: int, count: int) -> np.ndarray:
        rows = (L.md_trace_t * max(int(count), 1))()
        check(lib().md_batch_get_trace(self._h, int(slot), int(first_step), int(count), rows),
              "md_batch_get_trace")
        return _trace_array(rows[:int(count)])

    def release(self, slot: int) -> None:
        check(lib().md_batch_release(self._h, int(slot)), "md_batch_release")
        self.n_of.pop(slot, None)

    def usage(self) -> Tuple[int, int]:
        b = C.c_size_t()
        k = C.c_int32()
        check(lib().md_batch_usage(self._h, C.byref(b), C.byref(k)), "md_batch_usage")
        return b.value, k.value

    def progress(self) -> Tuple[int, int, int]:
        """(atom-steps completed by the admitted systems, systems still
        running, fewest steps any running system still has to go)."""
        a = C.c_int64()
        k = C.c_int32()
        r = C.c_int64()
        check(lib().md_batch_progress(self._h, C.byref(a), C.byref(k), C.byref(r)),
              "md_batch_progress")
        return a.value, k.value, r.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().md_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


# ---------------------------------------------------------------------------
# Function forms with the C ABI's names
# ---------------------------------------------------------------------------

def md_create(pos, vel, box: float, **params) -> System:
    return System(pos, vel, box, **params)


def md_bin_cells(s: System) -> None:
    s.bin_cells()


def md_build_nebr(s: System) -> None:
    s.build_nebr()


def md_forces(s: System) -> None:
    s.forces()


def md_step(s: System, n_steps: int) -> None:
    s.step(n_steps)


def md_props(s: System) -> Dict[str, float]:
    return s.props()


def md_get_state(s: System):
    return s.get_state()


def md_set_state(s: System, pos, vel) -> None:
    s.set_state(pos, vel)


def md_get_cells(s: System) -> np.ndarray:
    return s.cells()


def md_get_bins(s: System):
    return s.bins()


def md_get_pairs(s: System):
    return s.pairs()


def md_destroy(s: System) -> None:
    s.close()
