"""Float64 CPU oracle for the Barnes-Hut force step (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU library neither imports nor links it and
shares no code with it.  The arithmetic lives in ``bh_oracle.c`` (plain C,
float64, explicit fma only); this file only builds it with gcc and wraps it
with ctypes.

Steps (in the order the paper's Results section lists the parts of a step):
root cube and Morton keys, stable sort, moving, tree construction, groups,
multipole moments, MAC data, group walk, back to input order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall",
             "-shared", "-fPIC"]


def build(force: bool = False) -> str:
    """Compile bh_oracle.c into liboracle.so (always when force=True)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


SAN_LIB = os.path.join(_HERE, "liboracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]


def build_sanitized() -> str:
    """Compile bh_oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer
    into liboracle_san.so (same arithmetic flags as the normal build, one
    thread team per OpenMP region as before).  Load it through MIBH_ORACLE_SO
    with the ASan runtime preloaded; see ``sanitizer_env``."""
    flags = [f for f in GCC_FLAGS if f != "-O2"] + SAN_FLAGS
    tmp = SAN_LIB + ".tmp"
    subprocess.run(["gcc", *flags, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def sanitizer_env(base=None) -> dict:
    """Environment for a child Python process that runs the oracle from the
    sanitizer build: the ASan runtime preloaded (it must come first), leak
    checks off (the interpreter keeps its allocations until exit), any report
    fatal."""
    env = dict(os.environ if base is None else base)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], check=True, capture_output=True,
                          text=True).stdout.strip()
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["MIBH_ORACLE_SO"] = SAN_LIB
    return env


_lib = None


def lib():
    global _lib
    if _lib is None:
        alt = os.environ.get("MIBH_ORACLE_SO")  # an altered build: mutation checks, sanitizers
        if not alt:
            build()
        L = C.CDLL(alt or _LIB)
        P = C.c_void_p
        i64 = C.c_int64
        L.orc_new.restype = P
        L.orc_free.argtypes = [P]
        L.orc_build.argtypes = [P, P, P, i64, C.c_int, C.c_int]
        L.orc_build.restype = C.c_int
        L.orc_mac_prep.argtypes = [P, C.c_float]
        L.orc_mac_prep.restype = C.c_int
        L.orc_walk.argtypes = [P, C.c_float, C.c_double, C.c_double, i64, i64, C.c_int]
        L.orc_walk.restype = C.c_int
        L.orc_refit.argtypes = [P, P, P]
        L.orc_refit.restype = C.c_int
        L.orc_walk_list.argtypes = [P, C.c_float, C.c_double, C.c_double, P, i64, C.c_int]
        L.orc_walk_list.restype = C.c_int
        L.orc_group_lists.argtypes = [P, i64, P, i64, P, i64, P, P]
        L.orc_group_lists.restype = C.c_int
        L.orc_unsort.argtypes = [P]
        L.orc_direct.argtypes = [P, P, i64, P, i64, C.c_double, C.c_double, P, P, C.c_int]
        L.orc_direct.restype = C.c_int
        L.orc_energy.argtypes = [P, P, P, i64, P, P]
        L.orc_key.argtypes = [P, P, C.c_int]
        L.orc_key.restype = C.c_uint64
        L.orc_root_cube.argtypes = [P, i64, P, P]
        L.orc_root_cube.restype = C.c_int
        for name in ("orc_n", "orc_ncells", "orc_ngroups"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = i64
        L.orc_k.argtypes = [P]
        L.orc_k.restype = C.c_int
        L.orc_num_threads.restype = C.c_int
        for name in ("orc_lo", "orc_keys", "orc_perm", "orc_level", "orc_first", "orc_count",
                     "orc_child_first", "orc_nchild", "orc_parent", "orc_gfirst", "orc_gcount",
                     "orc_gcell", "orc_glevel", "orc_M", "orc_com", "orc_S", "orc_Q", "orc_delta",
                     "orc_bmin", "orc_bmax", "orc_lside",
                     "orc_com32", "orc_r2open", "orc_n_pc", "orc_n_pp", "orc_sacc", "orc_spot",
                     "orc_acc", "orc_pot"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = P
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f32(a, shape_last=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


class Tree:
    """One oracle tree over a particle set: build(), then walk(theta)."""

    def __init__(self, pos, mass, ncrit: int = 16, gcap: int = 64):
        self._pos = _f32(pos).reshape(-1, 3)
        self._mass = _f32(mass).reshape(-1)
        if self._pos.shape[0] != self._mass.shape[0]:
            raise ValueError("pos and mass sizes differ")
        self.n = int(self._mass.shape[0])
        L = lib()
        self._t = L.orc_new()
        st = L.orc_build(self._t, _ptr(self._pos), _ptr(self._mass), self.n, ncrit, gcap)
        if st != 0:
            L.orc_free(self._t)
            self._t = None
            raise OracleError(f"orc_build failed with status {st}")
        self.ncrit, self.gcap = ncrit, gcap
        self.ncells = int(L.orc_ncells(self._t))
        self.ngroups = int(L.orc_ngroups(self._t))
        self.k = int(L.orc_k(self._t))
        self.theta = None

    def __del__(self):
        if getattr(self, "_t", None) is not None and _lib is not None:
            _lib.orc_free(self._t)
            self._t = None

    def _arr(self, name, dtype, count):
        p = getattr(lib(), name)(self._t)
        if count == 0:
            return np.zeros(0, dtype=dtype)
        buf = (C.c_char * (count * np.dtype(dtype).itemsize)).from_address(p)
        return np.frombuffer(buf, dtype=dtype, count=count).copy()

    # artefacts of the build
    @property
    def lo(self):
        return self._arr("orc_lo", np.float32, 3)

    @property
    def keys(self):
        return self._arr("orc_keys", np.uint64, self.n)

    @property
    def perm(self):
        return self._arr("orc_perm", np.int64, self.n)

    def cells(self):
        nc = self.ncells
        return {
            "level": self._arr("orc_level", np.int32, nc),
            "first": self._arr("orc_first", np.int64, nc),
            "count": self._arr("orc_count", np.int64, nc),
            "child_first": self._arr("orc_child_first", np.int64, nc),
            "nchild": self._arr("orc_nchild", np.int32, nc),
            "parent": self._arr("orc_parent", np.int64, nc),
        }

    def groups(self):
        ng = self.ngroups
        return {
            "first": self._arr("orc_gfirst", np.int64, ng),
            "count": self._arr("orc_gcount", np.int64, ng),
            "cell": self._arr("orc_gcell", np.int64, ng),
            "level": self._arr("orc_glevel", np.int32, ng),
        }

    def multipoles(self):
        nc = self.ncells
        return {
            "M": self._arr("orc_M", np.float64, nc),
            "com": self._arr("orc_com", np.float64, 3 * nc).reshape(nc, 3),
            "S": self._arr("orc_S", np.float64, 6 * nc).reshape(nc, 6),
            "Q": self._arr("orc_Q", np.float64, 6 * nc).reshape(nc, 6),
            "delta": self._arr("orc_delta", np.float64, nc),
            "bmin": self._arr("orc_bmin", np.float32, 3 * nc).reshape(nc, 3),
            "bmax": self._arr("orc_bmax", np.float32, 3 * nc).reshape(nc, 3),
            "lside": self._arr("orc_lside", np.float64, nc),
        }

    def refit(self, pos, mass):
        """New positions and masses (input order) for the same particles; the
        sorted order, cells and groups stay, the multipoles are recomputed."""
        self._pos = _f32(pos).reshape(-1, 3)
        self._mass = _f32(mass).reshape(-1)
        if self._pos.shape[0] != self.n or self._mass.shape[0] != self.n:
            raise ValueError("refit needs the same number of particles")
        st = lib().orc_refit(self._t, _ptr(self._pos), _ptr(self._mass))
        if st != 0:
            raise OracleError(f"orc_refit failed with status {st}")

    def walk_groups(self, theta: float, groups, eps2: float = 0.0, G: float = 1.0, nthreads: int = 0):
        """Walk only the listed groups; the other groups' results are left as they were."""
        gl = np.ascontiguousarray(groups, dtype=np.int64)
        st = lib().orc_walk_list(self._t, C.c_float(theta), eps2, G, _ptr(gl), gl.shape[0], nthreads)
        if st != 0:
            raise OracleError(f"orc_walk_list failed with status {st}")
        self.theta = theta
        lib().orc_unsort(self._t)

    def mac_prep(self, theta: float):
        st = lib().orc_mac_prep(self._t, C.c_float(theta))
        if st != 0:
            raise OracleError(f"orc_mac_prep failed with status {st}")
        nc = self.ncells
        return {
            "com32": self._arr("orc_com32", np.float32, 3 * nc).reshape(nc, 3),
            "r2open": self._arr("orc_r2open", np.float32, nc),
        }

    def walk(self, theta: float = 0.75, eps2: float = 0.0, G: float = 1.0,
             groups=None, nthreads: int = 0):
        """Walk all groups (or the range ``groups=(begin, end)``)."""
        gb, ge = (0, self.ngroups) if groups is None else groups
        st = lib().orc_walk(self._t, C.c_float(theta), eps2, G, gb, ge, nthreads)
        if st != 0:
            raise OracleError(f"orc_walk failed with status {st}")
        self.theta = theta
        lib().orc_unsort(self._t)

    def counts(self):
        ng = self.ngroups
        return self._arr("orc_n_pc", np.int64, ng), self._arr("orc_n_pp", np.int64, ng)

    def forces(self):
        """(acc f64[n,3], pot f64[n]) in input order, after walk()."""
        return (self._arr("orc_acc", np.float64, 3 * self.n).reshape(self.n, 3),
                self._arr("orc_pot", np.float64, self.n))

    def sorted_forces(self):
        return (self._arr("orc_sacc", np.float64, 3 * self.n).reshape(self.n, 3),
                self._arr("orc_spot", np.float64, self.n))

    def group_lists(self, g: int, theta: float):
        """(accepted cells, opened leaves) of group g for this theta."""
        self.mac_prep(theta)
        cap = self.ncells
        pc = np.zeros(cap, dtype=np.int64)
        pp = np.zeros(cap, dtype=np.int64)
        npc = C.c_int64(0)
        npp = C.c_int64(0)
        st = lib().orc_group_lists(self._t, g, _ptr(pc), cap, _ptr(pp), cap,
                                   C.byref(npc), C.byref(npp))
        if st != 0:
            raise OracleError(f"orc_group_lists failed with status {st}")
        return pc[:npc.value].copy(), pp[:npp.value].copy()


def key(x, lo, k: int) -> int:
    """Morton key of one point (float32 triple) for the root cube (lo, 2^k)."""
    xa = np.ascontiguousarray(x, dtype=np.float32)
    la = np.ascontiguousarray(lo, dtype=np.float32)
    return int(lib().orc_key(_ptr(xa), _ptr(la), k))


def root_cube(pos):
    p = _f32(pos).reshape(-1, 3)
    lo = np.zeros(3, dtype=np.float32)
    k = C.c_int(0)
    st = lib().orc_root_cube(_ptr(p), p.shape[0], _ptr(lo), C.byref(k))
    if st != 0:
        raise OracleError(f"orc_root_cube failed with status {st}")
    return lo, k.value


def direct(pos, mass, targets=None, eps2: float = 0.0, G: float = 1.0, nthreads: int = 0):
    """Float64 direct summation for the target indices (all when None)."""
    p = _f32(pos).reshape(-1, 3)
    m = _f32(mass).reshape(-1)
    n = p.shape[0]
    if targets is None:
        t = None
        nt = n
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        nt = t.shape[0]
    acc = np.zeros((nt, 3), dtype=np.float64)
    pot = np.zeros(nt, dtype=np.float64)
    lib().orc_direct(_ptr(p), _ptr(m), n, None if t is None else _ptr(t), nt, eps2, G,
                     _ptr(acc), _ptr(pot), nthreads)
    return acc, pot


def energy(mass, pot, vel=None):
    """(T, W) in float64: W = 1/2 sum m phi, T = 1/2 sum m v^2."""
    m = _f32(mass).reshape(-1)
    p = np.ascontiguousarray(pot, dtype=np.float64)
    v = None if vel is None else _f32(vel).reshape(-1, 3)
    T = C.c_double(0)
    W = C.c_double(0)
    lib().orc_energy(_ptr(m), _ptr(p), None if v is None else _ptr(v), m.shape[0],
                     C.byref(T), C.byref(W))
    return T.value, W.value


def num_threads() -> int:
    return int(lib().orc_num_threads())
