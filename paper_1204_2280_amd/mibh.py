"""Thin ctypes binding of libmibh.so (include/mibh.h).

Argument marshalling only: every step of the force computation runs in the
library's HIP kernels.  PyTorch provides device memory (the workspace and the
caller's tensors) and the stream.  The functions keep the C names without the
``mibh_`` prefix; ``Context`` bundles a context handle with its workspace.

Importing this module does not touch the GPU; loading the library happens on
first use and raises ImportError when libmibh.so has not been built (there is
no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmibh.so")

PLAIN, KAHAN, KAHAN_TERM = 0, 1, 2
EXPORTS = {
    "keys": 0, "perm": 1, "cells": 2, "groups": 3, "counts": 4, "multipoles": 5, "delta": 6,
    "mac": 7, "quad": 8, "spos": 9, "features": 10, "predictions": 11, "queue": 12, "lside": 13,
}
ORDER_MORTON, ORDER_ESTIMATOR, ORDER_EXACT = 0, 1, 2


class BlockParams(C.Structure):
    _fields_ = [("dt_max", C.c_float), ("max_level", C.c_int32), ("eta", C.c_float), ("eps", C.c_float),
                ("rebuild_tol", C.c_float)]


class BlockStats(C.Structure):
    _fields_ = [("substeps", C.c_int64), ("rebuilds", C.c_int64), ("active_updates", C.c_int64),
                ("groups_walked", C.c_int64)]
MLP_FEATURES, MLP_PARAMS = 8, 4801
STAGES = ("sorting", "moving", "tree_construction", "multipoles", "mac_prep", "walk")
STATUS = {0: "MIBH_OK", -1: "MIBH_EINVAL", -2: "MIBH_ENOMEM", -3: "MIBH_EHIP", -4: "MIBH_ESTATE",
          -5: "MIBH_EOVERFLOW", -6: "MIBH_ENONFINITE"}


class MibhError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("ncrit", C.c_int32), ("group_cap", C.c_int32), ("eps2", C.c_float), ("G", C.c_float),
                ("precision", C.c_int32), ("walk_waves", C.c_int32), ("pc_cap", C.c_int32),
                ("pp_cap", C.c_int32), ("max_systems", C.c_int32), ("anchor_up", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("ncells", C.c_int64), ("ngroups", C.c_int64), ("nleaves", C.c_int64),
                ("depth", C.c_int32), ("root_k", C.c_int32), ("nsys", C.c_int32), ("sum_pc", C.c_uint64),
                ("sum_pp", C.c_uint64), ("flags", C.c_uint32), ("anchors", C.c_uint32),
                ("anchor_fallbacks", C.c_uint32)]


_lib = None


def lib():
    """The loaded library; ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1204_2280_amd.build.build()")
        # torch carries a HIP runtime of its own (soname libamdhip64.so) beside the
        # system one this library links (libamdhip64.so.7).  Loaded before torch's
        # runtime had started, the library's runtime found no device; so torch's
        # starts first (on a machine without a GPU this only returns False).
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, i64, st = C.c_void_p, C.c_int64, C.c_int
        L.mibh_default_params.argtypes = [C.POINTER(Params)]
        L.mibh_default_params.restype = None
        L.mibh_workspace_bytes.argtypes = [i64, C.POINTER(Params)]
        L.mibh_workspace_bytes.restype = C.c_size_t
        L.mibh_create.argtypes = [C.POINTER(Params), i64, P, C.c_size_t, P, C.POINTER(P)]
        L.mibh_destroy.argtypes = [P]
        L.mibh_build_tree.argtypes = [P, P, P, i64]
        L.mibh_build_tree_batch.argtypes = [P, P, P, P, C.c_int]
        L.mibh_graph_capture.argtypes = [P, P, P, P, C.c_int, C.c_float, P, P]
        L.mibh_graph_launch.argtypes = [P]
        L.mibh_set_stream.argtypes = [P, P]
        L.mibh_compute_multipoles.argtypes = [P]
        L.mibh_compute_forces.argtypes = [P, C.c_float, P, P]
        L.mibh_forces.argtypes = [P, P, P, i64, C.c_float, P, P]
        L.mibh_sync.argtypes = [P]
        L.mibh_stats.argtypes = [P, C.POINTER(Stats)]
        L.mibh_energy.argtypes = [P, P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.mibh_export_bytes.argtypes = [P, C.c_int, C.POINTER(C.c_size_t)]
        L.mibh_export.argtypes = [P, C.c_int, P, C.c_size_t]
        for f in ("mibh_create", "mibh_destroy", "mibh_build_tree", "mibh_build_tree_batch",
                  "mibh_graph_capture", "mibh_graph_launch", "mibh_set_stream", "mibh_compute_multipoles",
                  "mibh_compute_forces", "mibh_forces", "mibh_sync", "mibh_stats", "mibh_energy",
                  "mibh_export_bytes", "mibh_export"):
            getattr(L, f).restype = st
        L.mibh_refit.argtypes = [P, P, P]
        L.mibh_refit.restype = st
        L.mibh_compute_forces_active.argtypes = [P, C.c_float, P, P, P]
        L.mibh_compute_forces_active.restype = st
        L.mibh_kick_drift.argtypes = [P, P, P, P, i64, C.c_float, C.c_float]
        L.mibh_leapfrog.argtypes = [P, P, P, P, i64, C.c_float, C.c_float, C.c_int, C.c_int, P, P, P, C.c_int,
                                    C.POINTER(C.c_int)]
        L.mibh_kick_drift.restype = st
        L.mibh_block_run.argtypes = [P, P, P, P, i64, C.c_float, C.POINTER(BlockParams), C.c_int, P, P, P,
                                     C.POINTER(BlockStats), P, C.c_int, C.POINTER(C.c_int)]
        L.mibh_block_run.restype = st
        L.mibh_neighbor_count.argtypes = [P, P, P]
        L.mibh_neighbor_list.argtypes = [P, P, P, P, P, i64, C.POINTER(i64)]
        L.mibh_sph_density.argtypes = [P, P, P, P]
        for f in ("mibh_neighbor_count", "mibh_neighbor_list", "mibh_sph_density"):
            getattr(L, f).restype = st
        L.mibh_leapfrog.restype = st
        L.mibh_group_features.argtypes = [P, C.c_float, P]
        L.mibh_set_queue_order.argtypes = [P, C.c_int, P]
        L.mibh_mlp_forward.argtypes = [P, P, i64, P, P]
        L.mibh_mlp_scratch_bytes.argtypes = [C.c_int]
        L.mibh_mlp_scratch_bytes.restype = C.c_size_t
        L.mibh_mlp_gradient.argtypes = [P, P, P, P, C.c_int, P, P, P, C.c_size_t, P]
        L.mibh_mlp_adam.argtypes = [P, P, P, P, P, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, P]
        for f in ("mibh_group_features", "mibh_set_queue_order", "mibh_mlp_forward", "mibh_mlp_gradient",
                  "mibh_mlp_adam"):
            getattr(L, f).restype = st
        L.mibh_forces_static.argtypes = [P, P, i64, C.c_float, P, P, P]
        L.mibh_forces_static.restype = st
        L.mibh_static_bytes.argtypes = []
        L.mibh_static_bytes.restype = C.c_size_t
        L.mibh_static_n_max.argtypes = []
        L.mibh_static_n_max.restype = i64
        L.mibh_fma_probe.argtypes = [P, C.c_int32, C.c_int32, C.c_float, C.c_float, P]
        L.mibh_fma_probe.restype = st
        L.mibh_profile_begin.argtypes = [P, C.c_int]
        L.mibh_profile_read.argtypes = [P, P, C.c_int, C.POINTER(C.c_int)]
        L.mibh_profile_begin.restype = st
        L.mibh_profile_read.restype = st
        L.mibh_status_string.argtypes = [st]
        L.mibh_status_string.restype = C.c_char_p
        L.mibh_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise MibhError(status, lib().mibh_last_error().decode(errors="replace"))


def default_params(**overrides) -> Params:
    p = Params()
    lib().mibh_default_params(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def workspace_bytes(n_max: int, params: Params | None = None) -> int:
    return int(lib().mibh_workspace_bytes(n_max, None if params is None else C.byref(params)))


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else None


def _require(t, dtype, shape_tail, device, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on {device}")
    if tuple(t.shape[1:]) != shape_tail:
        raise ValueError(f"{name} has shape {tuple(t.shape)}")


def forces_static(pos, mass, theta: float, acc, pot, stream=None):
    """mibh_forces_static: the force step on the library's static workspace
    (n <= static_n_max(), default parameters).  pos [n,3], mass [n], acc [n,3]
    and pot [n] are caller-allocated float32 tensors on the current device;
    the call enqueues on `stream` (default: the current stream) and allocates
    nothing."""
    import torch
    dev = pos.device
    n = int(mass.shape[0])
    for t, name, tail in ((pos, "pos", (3,)), (acc, "acc", (3,))):
        _require(t, torch.float32, tail, dev, name)
    for t, name in ((mass, "mass"), (pot, "pot")):
        _require(t, torch.float32, (), dev, name)
    if pos.shape[0] != n or acc.shape[0] != n or pot.shape[0] != n:
        raise ValueError("pos, mass, acc and pot sizes differ")
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        _check(lib().mibh_forces_static(pos.data_ptr(), mass.data_ptr(), n, float(theta), acc.data_ptr(),
                                        pot.data_ptr(), s.cuda_stream))
    return acc, pot


def static_n_max() -> int:
    return int(lib().mibh_static_n_max())


class Context:
    """A library context with its workspace (a torch uint8 tensor) and stream."""

    def __init__(self, n_max: int, params: Params | None = None, device=None, stream=None, **overrides):
        import torch
        dev = torch.device(device if device is not None else "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.params = params if params is not None else default_params(**overrides)
        nbytes = workspace_bytes(n_max, self.params)
        if nbytes == 0:
            raise MibhError(-1, "invalid n_max or parameters")
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            h = C.c_void_p()
            _check(lib().mibh_create(C.byref(self.params), n_max, aligned, nbytes, self.stream.cuda_stream,
                                     C.byref(h)))
        self.handle = h
        self.n_max = n_max
        self.n = 0
        self._keep = ()

    def close(self):
        if getattr(self, "handle", None):
            lib().mibh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- the C entry points -------------------------------------------------
    def build_tree(self, pos, mass):
        import torch
        n = int(mass.shape[0]) if mass.dim() == 1 else -1
        _require(pos, torch.float32, (3,), self.device, "pos")
        _require(mass, torch.float32, (), self.device, "mass")
        if pos.shape[0] != n:
            raise ValueError("pos and mass sizes differ")
        with torch.cuda.device(self.device):
            _check(lib().mibh_build_tree(self.handle, pos.data_ptr(), mass.data_ptr(), n))
        self.n = n
        self._keep = (pos, mass)

    def build_tree_batch(self, pos, mass, offsets):
        """Independent systems: system s = rows offsets[s]:offsets[s+1] (host ints)."""
        import numpy as np
        import torch
        _require(pos, torch.float32, (3,), self.device, "pos")
        _require(mass, torch.float32, (), self.device, "mass")
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        nsys = len(off) - 1
        if nsys < 1 or off[-1] != pos.shape[0] or mass.shape[0] != pos.shape[0]:
            raise ValueError("offsets must run from 0 to the number of particles")
        with torch.cuda.device(self.device):
            _check(lib().mibh_build_tree_batch(self.handle, pos.data_ptr(), mass.data_ptr(), off.ctypes.data, nsys))
        self.n = int(off[-1])
        self._keep = (pos, mass)

    def forces_batch(self, pos, mass, offsets, theta: float, acc=None, pot=None):
        self.build_tree_batch(pos, mass, offsets)
        self.compute_multipoles()
        return self.compute_forces(theta, acc, pot)

    def set_stream(self, stream):
        _check(lib().mibh_set_stream(self.handle, stream.cuda_stream))
        self.stream = stream

    def graph_capture(self, pos, mass, offsets, theta: float, acc, pot):
        """Captures one whole step into a HIP graph (see mibh_graph_capture)."""
        import numpy as np
        import torch
        for t, name, tail in ((pos, "pos", (3,)), (acc, "acc", (3,))):
            _require(t, torch.float32, tail, self.device, name)
        for t, name in ((mass, "mass"), (pot, "pot")):
            _require(t, torch.float32, (), self.device, name)
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        with torch.cuda.device(self.device):
            _check(lib().mibh_graph_capture(self.handle, pos.data_ptr(), mass.data_ptr(), off.ctypes.data,
                                            len(off) - 1, float(theta), acc.data_ptr(), pot.data_ptr()))
        self._graph_keep = (pos, mass, acc, pot)

    def graph_launch(self):
        _check(lib().mibh_graph_launch(self.handle))
        self.n = int(self._graph_keep[0].shape[0])
        self._out = self._graph_keep[2:]

    def compute_multipoles(self):
        _check(lib().mibh_compute_multipoles(self.handle))

    def compute_forces(self, theta: float, acc=None, pot=None):
        import torch
        if acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float32, device=self.device)
        if pot is None:
            pot = torch.empty((self.n,), dtype=torch.float32, device=self.device)
        _require(acc, torch.float32, (3,), self.device, "acc")
        _require(pot, torch.float32, (), self.device, "pot")
        if acc.shape[0] != self.n or pot.shape[0] != self.n:
            raise ValueError("output sizes differ from the tree's particle count")
        with torch.cuda.device(self.device):
            _check(lib().mibh_compute_forces(self.handle, float(theta), acc.data_ptr(), pot.data_ptr()))
        self._out = (acc, pot)
        return acc, pot

    def refit(self, pos, mass):
        """New positions and masses for the particles of the last build (same n, input order):
        the tree is kept, the particles are moved into its order again; call compute_multipoles next."""
        import torch
        _require(pos, torch.float32, (3,), self.device, "pos")
        _require(mass, torch.float32, (), self.device, "mass")
        if pos.shape[0] != self.n or mass.shape[0] != self.n:
            raise ValueError("refit needs the particle count of the last build")
        with torch.cuda.device(self.device):
            _check(lib().mibh_refit(self.handle, pos.data_ptr(), mass.data_ptr()))
        self._keep = (pos, mass)

    def compute_forces_active(self, theta: float, active, acc, pot):
        """Forces for the groups holding a particle with active[i] != 0 (uint8 or bool [n] device
        tensor); acc/pot entries of the other groups' particles are left as they are."""
        import torch
        if active.dtype == torch.bool:
            active = active.view(torch.uint8)
        _require(active, torch.uint8, (), self.device, "active")
        _require(acc, torch.float32, (3,), self.device, "acc")
        _require(pot, torch.float32, (), self.device, "pot")
        if active.shape[0] != self.n or acc.shape[0] != self.n or pot.shape[0] != self.n:
            raise ValueError("sizes differ from the tree's particle count")
        with torch.cuda.device(self.device):
            _check(lib().mibh_compute_forces_active(self.handle, float(theta), active.data_ptr(), acc.data_ptr(),
                                                    pot.data_ptr()))
        self._out = (acc, pot, active)
        return acc, pot

    def forces(self, pos, mass, theta: float, acc=None, pot=None):
        self.build_tree(pos, mass)
        self.compute_multipoles()
        return self.compute_forces(theta, acc, pot)

    def kick_drift(self, pos, vel, acc, dt_kick: float, dt_drift: float):
        """vel += dt_kick * acc, then pos += dt_drift * vel (in place, float32 [n, 3] device tensors)."""
        import torch
        for t, name in ((pos, "pos"), (vel, "vel"), (acc, "acc")):
            _require(t, torch.float32, (3,), self.device, name)
        if not (pos.shape[0] == vel.shape[0] == acc.shape[0]):
            raise ValueError("pos, vel and acc sizes differ")
        with torch.cuda.device(self.device):
            _check(lib().mibh_kick_drift(self.handle, pos.data_ptr(), vel.data_ptr(), acc.data_ptr(),
                                         int(pos.shape[0]), float(dt_kick), float(dt_drift)))

    def leapfrog(self, pos, vel, mass, theta: float, dt: float, nsteps: int, log_every: int = 0,
                 acc=None, pot=None):
        """nsteps kick-drift-kick steps with shared time step dt (pos and vel updated in place).
        Returns (acc, pot, log): the forces at the final positions and the float64 energy log,
        rows (t, T, W) at step 0 and every log_every steps (empty when log_every == 0)."""
        import numpy as np
        import torch
        n = int(mass.shape[0])
        _require(pos, torch.float32, (3,), self.device, "pos")
        _require(vel, torch.float32, (3,), self.device, "vel")
        _require(mass, torch.float32, (), self.device, "mass")
        if pos.shape[0] != n or vel.shape[0] != n:
            raise ValueError("pos, vel and mass sizes differ")
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float32, device=self.device)
        if pot is None:
            pot = torch.empty((n,), dtype=torch.float32, device=self.device)
        cap = int(nsteps) // int(log_every) + 1 if log_every > 0 else 0
        log = np.zeros((max(cap, 1), 3), dtype=np.float64)
        nlog = C.c_int(0)
        with torch.cuda.device(self.device):
            _check(lib().mibh_leapfrog(self.handle, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), n,
                                       float(theta), float(dt), int(nsteps), int(log_every), acc.data_ptr(),
                                       pot.data_ptr(), log.ctypes.data, cap, C.byref(nlog)))
        self.n = n
        self._keep = (pos, mass)
        self._out = (acc, pot)
        return acc, pot, log[:nlog.value]

    def block_run(self, pos, vel, mass, theta: float, dt_max: float, max_level: int, eta: float, eps: float,
                  nbig: int, rebuild_tol: float = 0.25, log: bool = True, acc=None, pot=None, levels=None):
        """nbig block-time-step steps of dt_max (pos and vel updated in place, synchronised on return).
        Returns (acc, pot, levels uint8 [n], stats dict, energy log rows (t, T, W) per dt_max)."""
        import numpy as np
        import torch
        n = int(mass.shape[0])
        _require(pos, torch.float32, (3,), self.device, "pos")
        _require(vel, torch.float32, (3,), self.device, "vel")
        _require(mass, torch.float32, (), self.device, "mass")
        if pos.shape[0] != n or vel.shape[0] != n:
            raise ValueError("pos, vel and mass sizes differ")
        acc = torch.empty((n, 3), dtype=torch.float32, device=self.device) if acc is None else acc
        pot = torch.empty((n,), dtype=torch.float32, device=self.device) if pot is None else pot
        levels = torch.empty((n,), dtype=torch.uint8, device=self.device) if levels is None else levels
        bp = BlockParams(float(dt_max), int(max_level), float(eta), float(eps), float(rebuild_tol))
        stats = BlockStats()
        rows = np.zeros((int(nbig) + 1, 3), dtype=np.float64)
        nlog = C.c_int(0)
        with torch.cuda.device(self.device):
            _check(lib().mibh_block_run(self.handle, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), n,
                                        float(theta), C.byref(bp), int(nbig), acc.data_ptr(), pot.data_ptr(),
                                        levels.data_ptr(), C.byref(stats),
                                        rows.ctypes.data if log else None, rows.shape[0], C.byref(nlog)))
        self.n = n
        self._keep = (pos, mass)
        self._out = (acc, pot)
        return acc, pot, levels, {f: getattr(stats, f) for f, _ in BlockStats._fields_}, rows[:nlog.value]

    def _radius(self, r, name):
        import torch
        _require(r, torch.float32, (), self.device, name)
        if r.shape[0] != self.n:
            raise ValueError(f"{name} needs one value per particle of the tree")

    def neighbor_count(self, radius):
        """Neighbours of each particle within radius[i] (itself included), uint32 [n] as int32 tensor."""
        import torch
        self._radius(radius, "radius")
        count = torch.empty((self.n,), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().mibh_neighbor_count(self.handle, radius.data_ptr(), count.data_ptr()))
        return count

    def neighbor_list(self, radius, capacity=None):
        """(counts, offsets [n+1], indices): the neighbours of particle i are
        indices[offsets[i]:offsets[i+1]] (input indices, unordered).  With capacity None the
        list is sized from the counts (two passes)."""
        import torch
        self._radius(radius, "radius")
        count = torch.empty((self.n,), dtype=torch.int32, device=self.device)
        offset = torch.empty((self.n + 1,), dtype=torch.int32, device=self.device)
        total = C.c_int64(0)
        if capacity is None:
            with torch.cuda.device(self.device):
                st = lib().mibh_neighbor_list(self.handle, radius.data_ptr(), count.data_ptr(), offset.data_ptr(),
                                              None, 0, C.byref(total))
            if st not in (0, -5):
                _check(st)
            capacity = total.value
        index = torch.empty((max(int(capacity), 1),), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().mibh_neighbor_list(self.handle, radius.data_ptr(), count.data_ptr(), offset.data_ptr(),
                                            index.data_ptr(), int(capacity), C.byref(total)))
        return count, offset, index[:total.value]

    def sph_density(self, h):
        """(rho float32 [n], neighbour counts within 2 h) with the cubic-spline kernel."""
        import torch
        self._radius(h, "h")
        rho = torch.empty((self.n,), dtype=torch.float32, device=self.device)
        count = torch.empty((self.n,), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().mibh_sph_density(self.handle, h.data_ptr(), rho.data_ptr(), count.data_ptr()))
        return rho, count

    def sync(self):
        _check(lib().mibh_sync(self.handle))

    def stats(self) -> dict:
        s = Stats()
        _check(lib().mibh_stats(self.handle, C.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def energy(self, vel=None):
        T, W = C.c_double(), C.c_double()
        _check(lib().mibh_energy(self.handle, _ptr(vel), C.byref(T), C.byref(W)))
        return T.value, W.value

    def group_features(self, theta: float):
        """Work-estimator features of the current tree's groups, float32 [ngroups, 8]."""
        _check(lib().mibh_group_features(self.handle, float(theta), None))
        return self.export("features")

    def set_queue_order(self, mode: int, w16=None):
        """Order of the walk's group queue: ORDER_MORTON, ORDER_ESTIMATOR (float16 weights, heaviest
        predicted work first) or ORDER_EXACT (heaviest work of the previous walk of the same tree first)."""
        _check(lib().mibh_set_queue_order(self.handle, int(mode), None if w16 is None else w16.data_ptr()))
        self._est = w16

    def profile_begin(self, max_steps: int):
        """Record stage events for the next max_steps steps."""
        _check(lib().mibh_profile_begin(self.handle, max_steps))
        self._prof_max = max_steps

    def profile_read(self):
        """Per-step stage times in ms: list of dicts keyed by STAGES (synchronises)."""
        import numpy as np
        ms = np.zeros((self._prof_max, len(STAGES)), dtype=np.float32)
        ns = C.c_int()
        _check(lib().mibh_profile_read(self.handle, ms.ctypes.data, self._prof_max, C.byref(ns)))
        return [dict(zip(STAGES, map(float, ms[k]))) for k in range(ns.value)]

    def export(self, what: str):
        """Copy of an internal array as a torch tensor on the device."""
        import torch
        code = EXPORTS[what]
        nb = C.c_size_t()
        _check(lib().mibh_export_bytes(self.handle, code, C.byref(nb)))
        buf = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=self.device)
        _check(lib().mibh_export(self.handle, code, buf.data_ptr(), buf.numel()))
        buf = buf[:nb.value]
        view = {"keys": (torch.int64, (-1,)), "perm": (torch.int32, (-1,)), "cells": (torch.int32, (-1, 4)),
                "groups": (torch.int32, (-1, 2)), "counts": (torch.int32, (-1, 2)),
                "multipoles": (torch.float64, (-1, 10)), "delta": (torch.float64, (-1,)),
                "mac": (torch.float32, (-1, 4)), "quad": (torch.float32, (-1, 8)),
                "spos": (torch.float32, (-1, 4)), "features": (torch.float32, (-1, MLP_FEATURES)),
                "predictions": (torch.float32, (-1,)), "queue": (torch.int32, (-1,)),
                "lside": (torch.float64, (-1,))}[what]
        return buf.view(view[0]).reshape(view[1])


def _stream_ptr(t):
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def fma_probe(out, blocks: int, iters: int, a: float = 0.5, b: float = 2.0 ** -12):
    """Launches the float32 fused multiply-add probe on the current stream:
    `blocks` waves, 32 accumulators per lane, `iters` updates v <- fma(a, b, v);
    out is float32 [blocks * 64 * 32] on the GPU."""
    if out.numel() < blocks * 2048:
        raise ValueError("out holds fewer than 2048 floats per block")
    _check(lib().mibh_fma_probe(out.data_ptr(), int(blocks), int(iters), float(a), float(b), _stream_ptr(out)))
    return out


def mlp_forward(w16, x, y=None):
    """y = MLP(x) for x float32 [rows, 8] with float16 weights [4801]."""
    import torch
    rows = int(x.shape[0])
    if y is None:
        y = torch.empty(rows, dtype=torch.float32, device=x.device)
    _check(lib().mibh_mlp_forward(w16.data_ptr(), x.data_ptr(), rows, y.data_ptr(), _stream_ptr(x)))
    return y


def mlp_gradient(w16, x, t, idx, grad=None, loss=None, scratch=None):
    """Gradient of the batch mean squared error; returns (grad float32 [4801], loss float32 [1])."""
    import torch
    dev = x.device
    batch = int(idx.shape[0])
    if grad is None:
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    nb = int(lib().mibh_mlp_scratch_bytes(batch))
    if scratch is None or scratch.numel() < nb:
        scratch = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check(lib().mibh_mlp_gradient(w16.data_ptr(), x.data_ptr(), t.data_ptr(), idx.data_ptr(), batch,
                                   grad.data_ptr(), loss.data_ptr(), scratch.data_ptr(), scratch.numel(),
                                   _stream_ptr(x)))
    return grad, loss


def mlp_adam(w32, w16, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().mibh_mlp_adam(w32.data_ptr(), w16.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                               int(step), float(lr), float(beta1), float(beta2), float(eps), _stream_ptr(w32)))


@dataclass
class Decoded:
    """Host-side numpy views of exported integer arrays, decoded to the oracle's fields."""

    @staticmethod
    def cells(t):
        import numpy as np
        a = t.cpu().numpy().view(np.uint32).reshape(-1, 4)
        return {"first": a[:, 0].astype(np.int64), "count": a[:, 1].astype(np.int64),
                "child_first": a[:, 2].astype(np.int64), "level": ((a[:, 3] >> 8) & 255).astype(np.int32),
                "nchild": (a[:, 3] & 255).astype(np.int32), "system": (a[:, 3] >> 16).astype(np.int32)}

    @staticmethod
    def groups(t):
        import numpy as np
        a = t.cpu().numpy().view(np.uint32).reshape(-1, 2)
        return {"first": a[:, 0].astype(np.int64), "count": (a[:, 1] & 255).astype(np.int64),
                "level": ((a[:, 1] >> 8) & 255).astype(np.int32), "system": (a[:, 1] >> 16).astype(np.int32)}
