"""Python binding of the MI355X BSS-QMC sweep library (libbssqmc.so).

Argument marshalling only: every step of the sweep runs in the library's
gfx950 kernels behind the C ABI of ``include/bssqmc.h``.  PyTorch supplies
the device memory (a workspace tensor) and the HIP stream.  There is no CPU
fallback: if the library is missing or no GPU is present, the calls fail.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbssqmc.so")

BSS_OK, BSS_E_INVALID_ARG, BSS_E_UNSUPPORTED, BSS_E_OUT_OF_MEMORY, BSS_E_DEVICE, BSS_E_NUMERICAL, BSS_E_STATE = range(7)
PREC = {"fp64": 0, "mixed": 1}
FLAG_RECORD_TRACE, FLAG_REPLAY_TRACE, FLAG_NO_GRAPH, FLAG_PROFILE = 0x1, 0x2, 0x4, 0x8
FLAG_KRONECKER_HOPPING = 0x10

# every entry point declared in include/bssqmc.h
EXPORTS = [
    "bss_options_default", "bss_create", "bss_create_batch", "bss_workspace_size", "bss_sweep",
    "bss_step_slices", "bss_measure_gtau_k", "bss_measure_double_occ", "bss_measure_spin_corr", "bss_reset_measurements", "bss_reset_stats", "bss_synchronize",
    "bss_get_green", "bss_get_field", "bss_set_field", "bss_set_trace", "bss_get_trace",
    "bss_get_stats", "bss_save", "bss_load", "bss_destroy", "bss_status_string", "bss_last_error",
    "bss_get_profile", "bss_reset_profile", "bss_autotune", "bss_debug_set_green", "bss_green_from_field",
    "bss_green_from_field_noalloc", "bss_green_from_field_noalloc_limit",
    "bss_trotter_extrapolate", "bss_matsubara", "bss_dyson", "bss_finite_size_extrapolate",
    "bss_correlation_length", "bss_mem_spectrum", "bss_mem_green",
]


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32), ("delay_k", ctypes.c_int32),
                ("n_stab", ctypes.c_int32), ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("flags", ctypes.c_uint32), ("drift_abort", ctypes.c_double),
                ("trace_sweeps", ctypes.c_int32), ("fp32_slices", ctypes.c_int32),
                ("fp32_drift_target", ctypes.c_double), ("fp32_adapt_sweeps", ctypes.c_int32)]


class Instance(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("U", ctypes.c_double), ("t", ctypes.c_double), ("beta", ctypes.c_double),
                ("dtau", ctypes.c_double), ("seed", ctypes.c_uint64), ("n_chains", ctypes.c_int32),
                ("delay_k", ctypes.c_int32), ("n_stab", ctypes.c_int32)]


def _instance(d: dict) -> Instance:
    """bss_instance from a dict (L, U, t, beta, dtau, seed, n_chains and the
    optional per-instance delay_k, n_stab)."""
    return Instance(int(d["L"]), float(d["U"]), float(d.get("t", 0.25)), float(d["beta"]), float(d["dtau"]),
                    int(d["seed"]), int(d["n_chains"]), int(d.get("delay_k", 0)), int(d.get("n_stab", 0)))


class Stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("proposals", ctypes.c_int64), ("accepted", ctypes.c_int64),
                ("drift_max", ctypes.c_double), ("drift_mean", ctypes.c_double), ("logw", ctypes.c_double),
                ("sign", ctypes.c_int32), ("n_chains", ctypes.c_int32), ("N", ctypes.c_int32),
                ("Lambda", ctypes.c_int32), ("delay_k", ctypes.c_int32), ("n_stab", ctypes.c_int32),
                ("fp32_slices", ctypes.c_int32), ("drift_rel_max", ctypes.c_double),
                ("drift_rel_mean", ctypes.c_double), ("sweep_graph", ctypes.c_int32), ("shards", ctypes.c_int32),
                ("fp32_fraction", ctypes.c_double), ("fp32_rejected", ctypes.c_int64),
                ("fp32_fused", ctypes.c_int32), ("fp32_settled", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("delay_k", ctypes.c_int32), ("n_stab", ctypes.c_int32),
                ("fp32_slices", ctypes.c_int32), ("met_bound", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("ms_per_sweep", ctypes.c_double), ("drift_rel_max", ctypes.c_double)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class BssError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load libbssqmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1504_05090_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl, u64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_uint64, ctypes.c_size_t)
        P = ctypes.POINTER
        L.bss_options_default.argtypes = [P(Options)]
        L.bss_options_default.restype = None
        L.bss_create.argtypes = [i32, dbl, dbl, dbl, dbl, u64, i32, P(Options), P(vp)]
        L.bss_create_batch.argtypes = [P(Instance), i32, P(Options), P(vp)]
        L.bss_workspace_size.argtypes = [P(Instance), i32, P(Options), P(sz)]
        L.bss_sweep.argtypes = [vp, i32, i32]
        L.bss_step_slices.argtypes = [vp, i32]
        L.bss_measure_gtau_k.argtypes = [vp, i32, vp, vp, i64]
        L.bss_measure_double_occ.argtypes = [vp, i32, P(dbl), P(dbl)]
        L.bss_measure_spin_corr.argtypes = [vp, i32, vp, vp, i64]
        L.bss_reset_measurements.argtypes = [vp]
        L.bss_reset_stats.argtypes = [vp]
        L.bss_synchronize.argtypes = [vp]
        L.bss_get_green.argtypes = [vp, i32, i32, i32, vp]
        L.bss_get_field.argtypes = [vp, i32, i32, vp]
        L.bss_set_field.argtypes = [vp, i32, i32, vp]
        L.bss_set_trace.argtypes = [vp, i32, vp, i32]
        L.bss_get_trace.argtypes = [vp, i32, vp, i32]
        L.bss_get_stats.argtypes = [vp, i32, P(Stats)]
        L.bss_save.argtypes = [vp, vp, P(sz)]
        L.bss_load.argtypes = [vp, vp, sz]
        L.bss_get_profile.argtypes = [vp, P(KernelTime), i32, P(i32)]
        L.bss_reset_profile.argtypes = [vp]
        L.bss_autotune.argtypes = [P(Instance), P(Options), dbl, i32, i32, P(TuneResult)]
        L.bss_debug_set_green.argtypes = [vp, i32, i32, i32, i32, i32, dbl]
        L.bss_green_from_field.argtypes = [i32, dbl, dbl, dbl, dbl, i32, i32, vp, vp, vp]
        L.bss_green_from_field_noalloc.argtypes = [i32, dbl, dbl, dbl, dbl, i32, i32, vp, vp, vp]
        L.bss_green_from_field_noalloc_limit.argtypes = []
        L.bss_trotter_extrapolate.argtypes = [i32, vp, dbl, vp, i32, i32, vp, vp]
        L.bss_matsubara.argtypes = [i32, vp, vp, dbl, i32, vp]
        L.bss_dyson.argtypes = [i32, dbl, dbl, dbl, vp, vp]
        L.bss_finite_size_extrapolate.argtypes = [i32, vp, i32, vp, vp, vp, vp, vp]
        L.bss_correlation_length.argtypes = [i32, vp, P(dbl), P(dbl)]
        L.bss_mem_spectrum.argtypes = [i32, vp, vp, vp, dbl, i32, vp, vp, dbl, vp, P(dbl), P(dbl)]
        L.bss_mem_green.argtypes = [dbl, i32, vp, vp, i32, vp, vp]
        L.bss_green_from_field_noalloc_limit.restype = sz
        L.bss_destroy.argtypes = [vp]
        L.bss_destroy.restype = None
        L.bss_status_string.argtypes = [i32]
        L.bss_status_string.restype = ctypes.c_char_p
        L.bss_last_error.argtypes = [vp]
        L.bss_last_error.restype = ctypes.c_char_p
        for nm in EXPORTS:
            f = getattr(L, nm)
            if nm not in ("bss_options_default", "bss_destroy", "bss_status_string", "bss_last_error",
                          "bss_green_from_field_noalloc_limit"):
                f.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_options(precision="fp64", delay_k=0, n_stab=0, flags=0, trace_sweeps=0, drift_abort=None,
                 stream=None, workspace=None, workspace_bytes=0, fp32_slices=0, fp32_drift_target=0.0,
                 fp32_adapt_sweeps=0) -> Options:
    """bss_options from the library's defaults; drift_abort=None keeps the
    library's default."""
    o = Options()
    lib().bss_options_default(ctypes.byref(o))
    o.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    o.delay_k, o.n_stab, o.flags = delay_k, n_stab, flags
    o.trace_sweeps = trace_sweeps
    if drift_abort is not None:
        o.drift_abort = drift_abort
    o.fp32_slices = fp32_slices
    o.fp32_drift_target = fp32_drift_target
    o.fp32_adapt_sweeps = fp32_adapt_sweeps
    o.stream = stream
    o.workspace = workspace
    o.workspace_bytes = workspace_bytes
    return o


class Context:
    """A batch of (L, U, t, beta, dtau) instances with their Markov chains.

    instances: list of dicts with keys L, U, t, beta, dtau, seed, n_chains.
    Device memory is one torch uint8 tensor; work runs on torch's current
    stream of cuda:0 unless `stream` (a torch.cuda.Stream) is given.
    """

    def __init__(self, instances, precision="fp64", delay_k=0, n_stab=0, flags=0, trace_sweeps=0,
                 drift_abort=None, stream=None, fp32_slices=0, fp32_drift_target=0.0, fp32_adapt_sweeps=0):
        import torch  # device memory and streams only

        if not torch.cuda.is_available():
            raise BssError(BSS_E_DEVICE, "no GPU visible: the BSS-QMC library runs on gfx950 only")
        self._torch = torch
        L = lib()
        arr = (Instance * len(instances))()
        for n, d in enumerate(instances):
            arr[n] = _instance(d)
        self._inst = arr
        self.n_inst = len(instances)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        opt = make_options(precision, delay_k, n_stab, flags, trace_sweeps, drift_abort,
                           stream=self._stream.cuda_stream, fp32_slices=fp32_slices,
                           fp32_drift_target=fp32_drift_target, fp32_adapt_sweeps=fp32_adapt_sweeps)
        nbytes = ctypes.c_size_t()
        self._check(L.bss_workspace_size(arr, len(instances), ctypes.byref(opt), ctypes.byref(nbytes)),
                    "bss_workspace_size")
        self._ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
        opt.workspace = self._ws.data_ptr()
        opt.workspace_bytes = int(nbytes.value)
        h = ctypes.c_void_p()
        self._check(L.bss_create_batch(arr, len(instances), ctypes.byref(opt), ctypes.byref(h)), "bss_create_batch")
        self._h = h
        self._params = []
        for n in range(self.n_inst):
            st = self.stats(n)
            self._params.append(dict(N=st["N"], Lambda=st["Lambda"], delay_k=st["delay_k"], n_stab=st["n_stab"],
                                     fp32_slices=st["fp32_slices"], n_chains=st["n_chains"],
                                     L=int(instances[n]["L"])))

    # ------------------------------------------------------------------
    def _check(self, status, what):
        if status != BSS_OK:
            msg = ""
            h = getattr(self, "_h", None)
            if h:
                msg = (lib().bss_last_error(h) or b"").decode()
            raise BssError(status, f"{what}: {lib().bss_status_string(status).decode()} {msg}".strip())

    def params(self, inst=0) -> dict:
        return dict(self._params[inst])

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().bss_destroy(h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def sweep(self, n=1, measure=False):
        self._check(lib().bss_sweep(self._h, n, 1 if measure else 0), "bss_sweep")

    def step_slices(self, n):
        self._check(lib().bss_step_slices(self._h, n), "bss_step_slices")

    def synchronize(self):
        """Wait for the context's work (on its own stream or the caller's)."""
        self._check(lib().bss_synchronize(self._h), "bss_synchronize")

    def green(self, inst=0, chain=0, spin=0) -> np.ndarray:
        N = self._params[inst]["N"]
        out = np.zeros((N, N))
        self._check(lib().bss_get_green(self._h, inst, chain, spin, _ptr(out)), "bss_get_green")
        return out

    def field(self, inst=0, chain=0) -> np.ndarray:
        p = self._params[inst]
        out = np.zeros((p["Lambda"], p["N"]), dtype=np.int8)
        self._check(lib().bss_get_field(self._h, inst, chain, _ptr(out)), "bss_get_field")
        return out

    def set_field(self, field, inst=0, chain=0):
        f = np.ascontiguousarray(field, dtype=np.int8)
        self._check(lib().bss_set_field(self._h, inst, chain, _ptr(f)), "bss_set_field")

    def set_trace(self, accept, n_sweeps, inst=0):
        a = np.ascontiguousarray(accept, dtype=np.uint8)
        p = self._params[inst]
        assert a.size == n_sweeps * p["n_chains"] * p["Lambda"] * p["N"]
        self._check(lib().bss_set_trace(self._h, inst, _ptr(a), n_sweeps), "bss_set_trace")

    def get_trace(self, n_sweeps, inst=0) -> np.ndarray:
        p = self._params[inst]
        a = np.zeros(n_sweeps * p["n_chains"] * p["Lambda"] * p["N"], dtype=np.uint8)
        self._check(lib().bss_get_trace(self._h, inst, _ptr(a), n_sweeps), "bss_get_trace")
        return a.reshape(n_sweeps, p["n_chains"], p["Lambda"], p["N"])

    def debug_set_green(self, value, inst=0, chain=0, spin=0, i=0, j=0):
        """Overwrite one element of a chain's current G (failure-handling tests)."""
        self._check(lib().bss_debug_set_green(self._h, inst, chain, spin, i, j, float(value)),
                    "bss_debug_set_green")

    def stats(self, inst=0) -> dict:
        s = Stats()
        self._check(lib().bss_get_stats(self._h, inst, ctypes.byref(s)), "bss_get_stats")
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def gtau_k(self, inst=0):
        p = self._params[inst]
        n = (p["Lambda"] + 1) * p["N"]
        mean, err = np.zeros(n), np.zeros(n)
        self._check(lib().bss_measure_gtau_k(self._h, inst, _ptr(mean), _ptr(err), n), "bss_measure_gtau_k")
        return mean.reshape(p["Lambda"] + 1, p["N"]), err.reshape(p["Lambda"] + 1, p["N"])

    def double_occ(self, inst=0):
        m, e = ctypes.c_double(), ctypes.c_double()
        self._check(lib().bss_measure_double_occ(self._h, inst, ctypes.byref(m), ctypes.byref(e)),
                    "bss_measure_double_occ")
        return m.value, e.value

    def spin_corr(self, inst=0):
        n = self._params[inst]["N"]
        mean, err = np.zeros(n), np.zeros(n)
        self._check(lib().bss_measure_spin_corr(self._h, inst, _ptr(mean), _ptr(err), n), "bss_measure_spin_corr")
        return mean, err

    def reset_measurements(self):
        self._check(lib().bss_reset_measurements(self._h), "bss_reset_measurements")

    def reset_stats(self):
        self._check(lib().bss_reset_stats(self._h), "bss_reset_stats")

    def profile(self) -> dict:
        """{kernel family: (launches, total ms)} under FLAG_PROFILE."""
        arr = (KernelTime * 16)()
        n = ctypes.c_int32()
        self._check(lib().bss_get_profile(self._h, arr, 16, ctypes.byref(n)), "bss_get_profile")
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(n.value, 16))}

    def reset_profile(self):
        self._check(lib().bss_reset_profile(self._h), "bss_reset_profile")

    def save(self) -> bytes:
        n = ctypes.c_size_t()
        self._check(lib().bss_save(self._h, None, ctypes.byref(n)), "bss_save")
        buf = ctypes.create_string_buffer(n.value)
        self._check(lib().bss_save(self._h, buf, ctypes.byref(n)), "bss_save")
        return buf.raw[: n.value]

    def load(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        self._check(lib().bss_load(self._h, buf, len(data)), "bss_load")


def green_from_field(L, U, t, beta, dtau, n_stab, l, field, out=None, stream=None, noalloc=False):
    """bss_green_from_field: G of both spins at the start of slice l for a
    field.  `field` is a torch int8 device tensor [Lambda, N]; `out` (optional)
    a torch float64 device tensor [2, N, N], returned.  noalloc: the variant
    with the library's static scratch (bss_green_from_field_noalloc), which
    allocates nothing and does not synchronise."""
    import torch  # device memory and streams only

    N = L * L
    assert field.is_cuda and field.dtype == torch.int8 and field.is_contiguous() and field.shape[-1] == N
    if out is None:
        out = torch.empty((2, N, N), dtype=torch.float64, device=field.device)
    assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() == 2 * N * N
    s = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    fn = lib().bss_green_from_field_noalloc if noalloc else lib().bss_green_from_field
    st = fn(int(L), float(U), float(t), float(beta), float(dtau), int(n_stab), int(l), field.data_ptr(),
            out.data_ptr(), s)
    if st != BSS_OK:
        raise BssError(st, f"{fn.__name__}: {lib().bss_status_string(st).decode()}")
    return out


def autotune(instance: dict, precision="fp64", drift_bound=1e-6, warmup_sweeps=4, trial_sweeps=2, flags=0) -> dict:
    """Pick delay_k, n_stab and fp32_slices for one instance by timing trial
    sweeps under a relative wrap-drift bound (bss_autotune)."""
    import torch  # the trial contexts run on the current device

    if not torch.cuda.is_available():
        raise BssError(BSS_E_DEVICE, "no GPU visible: the BSS-QMC library runs on gfx950 only")
    d = instance
    inst = _instance(d)
    opt = make_options(precision, flags=flags)
    res = TuneResult()
    st = lib().bss_autotune(ctypes.byref(inst), ctypes.byref(opt), float(drift_bound), int(warmup_sweeps),
                            int(trial_sweeps), ctypes.byref(res))
    if st != BSS_OK:
        raise BssError(st, f"bss_autotune: {lib().bss_status_string(st).decode()}")
    out = {f: getattr(res, f) for f, _ in TuneResult._fields_}
    out["precision"] = "mixed" if res.precision == PREC["mixed"] else "fp64"
    return out


# ---------------------------------------------------------------------------
# analysis of the sweep's output (host code of the library)

def _host_check(st, what):
    if st != BSS_OK:
        raise BssError(st, f"{what}: {lib().bss_status_string(st).decode()}")


def trotter_extrapolate(dtaus, Gs, beta, tau_out):
    """bss_trotter_extrapolate: Gs[a] [Lambda_a + 1, n_cols] on the slice grid
    of dtaus[a]; returns [len(tau_out), n_cols] at dtau -> 0."""
    arrs = [np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(len(G), -1)) for G in Gs]
    n_cols = arrs[0].shape[1]
    assert all(a.shape[1] == n_cols for a in arrs)
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    dt = np.ascontiguousarray(dtaus, dtype=np.float64)
    to = np.ascontiguousarray(tau_out, dtype=np.float64)
    out = np.zeros((len(to), n_cols))
    _host_check(lib().bss_trotter_extrapolate(len(arrs), _ptr(dt), float(beta), ptrs, n_cols, len(to), _ptr(to),
                                              _ptr(out)), "bss_trotter_extrapolate")
    return out


def matsubara(tau, G, beta, n_freq):
    """bss_matsubara: complex G(i w_n), n = 0..n_freq-1."""
    t = np.ascontiguousarray(tau, dtype=np.float64)
    g = np.ascontiguousarray(G, dtype=np.float64)
    out = np.zeros(2 * n_freq)
    _host_check(lib().bss_matsubara(len(t), _ptr(t), _ptr(g), float(beta), n_freq, _ptr(out)), "bss_matsubara")
    return out[0::2] + 1j * out[1::2]


def dyson(beta, eps_k, mu, G_iw):
    """bss_dyson: Sigma_k(i w_n) from complex G_k(i w_n)."""
    g = np.ascontiguousarray(np.stack([np.real(G_iw), np.imag(G_iw)], axis=1).ravel())
    out = np.zeros_like(g)
    _host_check(lib().bss_dyson(len(G_iw), float(beta), float(eps_k), float(mu), _ptr(g), _ptr(out)), "bss_dyson")
    return out[0::2] + 1j * out[1::2]


def finite_size_extrapolate(Ls, values):
    """bss_finite_size_extrapolate over real values [len(Ls), n]; returns
    (value, err, lin, quad), each [n]."""
    Larr = np.ascontiguousarray(Ls, dtype=np.int32)
    v = np.ascontiguousarray(np.asarray(values, dtype=np.float64).reshape(len(Ls), -1))
    n = v.shape[1]
    outs = [np.zeros(n) for _ in range(4)]
    _host_check(lib().bss_finite_size_extrapolate(len(Larr), _ptr(Larr), n, _ptr(v), *[_ptr(o) for o in outs]),
                "bss_finite_size_extrapolate")
    return tuple(outs)


def correlation_length(L, C):
    """bss_correlation_length: (xi, amplitude) of a spin correlation C[r]."""
    c = np.ascontiguousarray(C, dtype=np.float64)
    xi, A = ctypes.c_double(), ctypes.c_double()
    _host_check(lib().bss_correlation_length(int(L), _ptr(c), ctypes.byref(xi), ctypes.byref(A)),
                "bss_correlation_length")
    return xi.value, A.value


def mem_spectrum(tau, G, sigma, beta, omega, model, alpha=None):
    """bss_mem_spectrum: (A on omega, alpha, chi^2); alpha None = historic."""
    t, g, sg = (np.ascontiguousarray(x, dtype=np.float64) for x in (tau, G, sigma))
    w, m = (np.ascontiguousarray(x, dtype=np.float64) for x in (omega, model))
    if not (len(t) == len(g) == len(sg)) or len(w) != len(m):
        raise ValueError("tau, G, sigma and omega, model must have matching lengths")
    A = np.zeros(len(w))
    a, c = ctypes.c_double(), ctypes.c_double()
    _host_check(lib().bss_mem_spectrum(len(t), _ptr(t), _ptr(g), _ptr(sg), float(beta), len(w), _ptr(w), _ptr(m),
                                       0.0 if alpha is None else float(alpha), _ptr(A), ctypes.byref(a),
                                       ctypes.byref(c)), "bss_mem_spectrum")
    return A, a.value, c.value


def mem_green(beta, omega, A, tau):
    """bss_mem_green: eq. (4) of the spectrum A on omega at the points tau."""
    w, a, t = (np.ascontiguousarray(x, dtype=np.float64) for x in (omega, A, tau))
    if len(w) != len(a):
        raise ValueError("omega and A must have the same length")
    out = np.zeros(len(t))
    _host_check(lib().bss_mem_green(float(beta), len(w), _ptr(w), _ptr(a), len(t), _ptr(t), _ptr(out)),
                "bss_mem_green")
    return out
