"""Plain FP64 CPU oracle of the BSS-QMC sweep -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps ``liborc.so`` (built from ``bss_oracle.c``
by :func:`build`) with ctypes and shares no code with the GPU library.

The oracle follows the paper's statement of the problem: the Hubbard model of
eq. (1), the Trotter product of eq. (2), the Ising-field determinant sum of
eq. (3) and its Monte Carlo summation (Sec. 2), with the BSS update, wrap and
UDV stabilisation of the literature the paper cites.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bss_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

_lib = None


def build() -> str:
    """Compile the oracle with gcc (FP64, OpenMP over chains)."""
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wextra", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrcStats(ctypes.Structure):
    _fields_ = [("proposals", ctypes.c_int64), ("accepted", ctypes.c_int64),
                ("drift_max", ctypes.c_double), ("drift_sum", ctypes.c_double),
                ("drift_count", ctypes.c_int64), ("logw", ctypes.c_double),
                ("sign", ctypes.c_int), ("error", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        u64, i32, dbl, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_draw.argtypes = [u64] * 5
        L.orc_draw.restype = u64
        L.orc_hopping.argtypes = [i32, dbl, vp]
        L.orc_expm.argtypes = [i32, vp, dbl, vp]
        L.orc_hs_lambda.argtypes = [dbl, dbl]
        L.orc_hs_lambda.restype = dbl
        L.orc_create.argtypes = [i32, dbl, dbl, dbl, dbl, u64, i32, i32, i32]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        for nm in ("orc_N", "orc_Lambda", "orc_slice"):
            getattr(L, nm).argtypes = [vp]
            getattr(L, nm).restype = i32
        L.orc_sweep_index.argtypes = [vp]
        L.orc_sweep_index.restype = ctypes.c_int64
        L.orc_lambda.argtypes = [vp]
        L.orc_lambda.restype = dbl
        L.orc_get_Em.argtypes = [vp, vp]
        L.orc_get_Ep.argtypes = [vp, vp]
        L.orc_get_field.argtypes = [vp, vp]
        L.orc_set_field.argtypes = [vp, vp]
        L.orc_get_green.argtypes = [vp, i32, vp]
        L.orc_set_green.argtypes = [vp, i32, vp]
        L.orc_step_slices.argtypes = [vp, i32, vp, vp]
        L.orc_step_slices.restype = i32
        L.orc_ratio.argtypes = [vp, i32, i32, P(dbl), P(dbl)]
        L.orc_accept_update.argtypes = [vp, i32, i32]
        L.orc_wrap.argtypes = [vp, i32]
        L.orc_bmat.argtypes = [vp, vp, i32, i32, vp]
        L.orc_fresh_green.argtypes = [vp, vp, i32, i32, vp]
        L.orc_log_det_M.argtypes = [vp, vp, i32, P(dbl), P(i32)]
        L.orc_gtau0.argtypes = [vp, vp, i32, i32, vp]
        L.orc_measure.argtypes = [vp, P(dbl), vp]
        L.orc_get_stats.argtypes = [vp, P(OrcStats)]
        L.orc_run_chains.argtypes = [i32, dbl, dbl, dbl, dbl, u64, i32, i32, i32, i32, i32, P(i32)]
        L.orc_run_chains.restype = dbl
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(counter, key) -> np.ndarray:
    """Philox4x64-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw(k0, k1, s, pos, tag) -> int:
    return int(lib().orc_draw(k0, k1, s, pos, tag))


def hopping(L: int, t: float) -> np.ndarray:
    K = np.zeros((L * L, L * L))
    lib().orc_hopping(L, t, _ptr(K))
    return K


def expm(A: np.ndarray, s: float) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.zeros_like(A)
    lib().orc_expm(A.shape[0], _ptr(A), s, _ptr(out))
    return out


def hs_lambda(U: float, dtau: float) -> float:
    return float(lib().orc_hs_lambda(U, dtau))


class Chain:
    """One Markov chain of one (L, U, t, beta, dtau) instance.

    RNG key = (seed + chain, inst); the field is drawn at creation and the
    equal-time Green function at tau = 0 is computed from scratch.
    """

    def __init__(self, L, U, t, beta, dtau, seed, inst=0, chain=0, n_stab=4):
        self._h = lib().orc_create(L, U, t, beta, dtau, seed, inst, chain, n_stab)
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self.L = L
        self.N = lib().orc_N(self._h)
        self.Lam = lib().orc_Lambda(self._h)
        self.n_stab = n_stab

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    # --- state -----------------------------------------------------------
    @property
    def slice(self) -> int:
        return lib().orc_slice(self._h)

    @property
    def sweep_index(self) -> int:
        return lib().orc_sweep_index(self._h)

    @property
    def lam(self) -> float:
        return lib().orc_lambda(self._h)

    def Em(self):
        out = np.zeros((self.N, self.N))
        lib().orc_get_Em(self._h, _ptr(out))
        return out

    def Ep(self):
        out = np.zeros((self.N, self.N))
        lib().orc_get_Ep(self._h, _ptr(out))
        return out

    def field(self) -> np.ndarray:
        out = np.zeros((self.Lam, self.N), dtype=np.int8)
        lib().orc_get_field(self._h, _ptr(out))
        return out

    def set_field(self, f):
        f = np.ascontiguousarray(f, dtype=np.int8).reshape(self.Lam, self.N)
        lib().orc_set_field(self._h, _ptr(f))

    def green(self, spin: int) -> np.ndarray:
        out = np.zeros((self.N, self.N))
        lib().orc_get_green(self._h, spin, _ptr(out))
        return out

    def set_green(self, spin: int, G):
        G = np.ascontiguousarray(G, dtype=np.float64)
        lib().orc_set_green(self._h, spin, _ptr(G))

    def stats(self) -> dict:
        s = OrcStats()
        lib().orc_get_stats(self._h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in OrcStats._fields_}

    # --- sweep -----------------------------------------------------------
    def step_slices(self, n: int, forced=None, record: bool = False):
        """Advance n slices; returns the accept trace (uint8 per proposal) if
        `record`, with `forced` (uint8 per proposal) replacing the test."""
        total = n * self.N
        fp = None
        if forced is not None:
            forced = np.ascontiguousarray(forced, dtype=np.uint8)
            assert forced.size >= total
            fp = _ptr(forced)
        tr = np.zeros(total, dtype=np.uint8) if record else None
        rc = lib().orc_step_slices(self._h, n, fp, _ptr(tr) if record else None)
        if rc != 0:
            raise FloatingPointError("oracle met a non-positive or non-finite ratio")
        return tr

    def sweep(self, n: int = 1, forced=None, record: bool = False):
        return self.step_slices(n * self.Lam, forced, record)

    def ratio(self, l: int, i: int):
        a, b = ctypes.c_double(), ctypes.c_double()
        lib().orc_ratio(self._h, l, i, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def accept_update(self, l: int, i: int):
        lib().orc_accept_update(self._h, l, i)

    def wrap(self, l: int):
        lib().orc_wrap(self._h, l)

    # --- pure functions of a field --------------------------------------
    def _field_arg(self, field):
        if field is None:
            field = self.field()
        return np.ascontiguousarray(field, dtype=np.int8).reshape(self.Lam, self.N)

    def bmat(self, l: int, spin: int, field=None):
        f = self._field_arg(field)
        out = np.zeros((self.N, self.N))
        lib().orc_bmat(self._h, _ptr(f), l, spin, _ptr(out))
        return out

    def fresh_green(self, l: int, spin: int, field=None):
        f = self._field_arg(field)
        out = np.zeros((self.N, self.N))
        lib().orc_fresh_green(self._h, _ptr(f), l, spin, _ptr(out))
        return out

    def log_det_M(self, spin: int, field=None):
        f = self._field_arg(field)
        la, sg = ctypes.c_double(), ctypes.c_int()
        lib().orc_log_det_M(self._h, _ptr(f), spin, ctypes.byref(la), ctypes.byref(sg))
        return la.value, sg.value

    def gtau0(self, l: int, spin: int, field=None):
        f = self._field_arg(field)
        out = np.zeros((self.N, self.N))
        lib().orc_gtau0(self._h, _ptr(f), l, spin, _ptr(out))
        return out

    def measure(self):
        """(double occupancy, G(tau_l, k) [Lambda+1, N]) of the current field."""
        d = ctypes.c_double()
        gtk = np.zeros((self.Lam + 1, self.N))
        lib().orc_measure(self._h, ctypes.byref(d), _ptr(gtk))
        return d.value, gtk


def run_chains(L, U, t, beta, dtau, seed, n_chains, n_stab, n_sweeps, n_threads=0, n_warm=0):
    """Time n_sweeps sweeps of n_chains chains (OpenMP over chains) after
    n_warm untimed sweeps.  Returns (seconds, threads used)."""
    used = ctypes.c_int()
    sec = lib().orc_run_chains(L, U, t, beta, dtau, seed, n_chains, n_stab, n_warm, n_sweeps,
                               n_threads, ctypes.byref(used))
    if sec < 0:
        raise ValueError("oracle rejected the parameters")
    return sec, used.value
