"""ctypes binding of libsoft.so (include/soft.h), argument marshalling only.

Every simulation step runs in the library's HIP kernels; this module only
turns Python values and torch tensors into the C ABI's pointers and sizes.
Loading fails loudly when the built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsoft.so")

SOFT_OK, SOFT_EINVAL, SOFT_EPARSE, SOFT_ECAPACITY, SOFT_EDEVICE, SOFT_ESTATE, SOFT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PASSED, DISCARDED, OVERFLOW, NUMERIC = 0, 1, 2, 3
NO_ABORT = 0xFFFFFFFF

ERROR_NAMES = {SOFT_EINVAL: "EINVAL", SOFT_EPARSE: "EPARSE", SOFT_ECAPACITY: "ECAPACITY",
               SOFT_EDEVICE: "EDEVICE", SOFT_ESTATE: "ESTATE", SOFT_EUNSUPPORTED: "EUNSUPPORTED"}

# Every function declared in include/soft.h.
EXPORTS = ("soft_create", "soft_destroy", "soft_last_error", "soft_load_circuit", "soft_load_noise",
           "soft_set_rng", "soft_set_uniforms", "soft_set_precision", "soft_set_prune", "soft_set_caps",
           "soft_autotune", "soft_set_keep", "soft_run", "soft_read_counters", "soft_read_coeffs",
           "soft_read_tableau", "soft_circuit_info", "soft_launch_shape", "soft_set_trace", "soft_read_trace",
           "soft_load_mixture", "soft_read_variant_counters", "soft_variant_info", "soft_set_tile_memory",
           "soft_run_list", "soft_set_speculation", "soft_set_noise_mode", "soft_graph_info", "soft_run_noalloc",
           "soft_set_shared_prefix", "soft_set_deferred_t")


class SoftError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (ERROR_NAMES.get(code, str(code)), msg))
        self.code = code


class soft_noise(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("p1", "p2", "p_idle", "p_meas", "p_reset", "p_mpp")]


class soft_counters(ctypes.Structure):
    _fields_ = [("shots", ctypes.c_uint64), ("passed", ctypes.c_uint64), ("discarded", ctypes.c_uint64),
                ("overflow", ctypes.c_uint64), ("numeric", ctypes.c_uint64), ("logical_errors", ctypes.c_uint64),
                ("entries_t", ctypes.c_uint64), ("entries_m", ctypes.c_uint64), ("noise_slots", ctypes.c_uint64),
                ("events", ctypes.c_uint64), ("support_hist", ctypes.c_uint64 * 16), ("max_norm_dev", ctypes.c_double),
                ("restarts", ctypes.c_uint64), ("prefix_shots", ctypes.c_uint64),
                ("redo_shots", ctypes.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsoft.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError("libsoft.so is not built (run __graft_entry__.build()); no fallback exists")
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one; loading torch first makes libsoft bind to that single runtime, so
    # torch tensors, streams and the sampler's kernels share one HIP context.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "soft_create": (I, [ctypes.POINTER(P), I]),
        "soft_destroy": (None, [P]),
        "soft_last_error": (ctypes.c_char_p, [P]),
        "soft_load_circuit": (I, [P, ctypes.c_char_p, ctypes.c_size_t]),
        "soft_load_noise": (I, [P, ctypes.POINTER(soft_noise)]),
        "soft_set_rng": (I, [P, U64]),
        "soft_set_uniforms": (I, [P, P, U64, U32, U32]),
        "soft_set_precision": (I, [P, I]),
        "soft_set_prune": (I, [P, ctypes.c_double]),
        "soft_set_caps": (I, [P, U32, U32, U32, U32]),
        "soft_autotune": (I, [P, U64, P]),
        "soft_set_keep": (I, [P, U64, U32]),
        "soft_run": (I, [P, U64, U64, P, P, P, P, P]),
        "soft_run_noalloc": (I, [P, U64, U64, P, P, P, P, P]),
        "soft_read_counters": (I, [P, ctypes.POINTER(soft_counters)]),
        "soft_read_coeffs": (I, [P, U64, P, P, P, U32, ctypes.POINTER(U32)]),
        "soft_read_tableau": (I, [P, U64, P, P, P]),
        "soft_circuit_info": (I, [P, P]),
        "soft_launch_shape": (I, [P, P]),
        "soft_set_trace": (I, [P, U64, U32]),
        "soft_read_trace": (I, [P, U32, P, P, P, P, P, P, P, U32, ctypes.POINTER(U32)]),
        "soft_load_mixture": (I, [P, U32, P, P, P, P]),
        "soft_read_variant_counters": (I, [P, U32, ctypes.POINTER(soft_counters)]),
        "soft_variant_info": (I, [P, U32, P]),
        "soft_set_tile_memory": (I, [P, I]),
        "soft_run_list": (I, [P, P, U64, P, P, P, P, P]),
        "soft_set_speculation": (I, [P, I]),
        "soft_set_noise_mode": (I, [P, I]),
        "soft_set_shared_prefix": (I, [P, I]),
        "soft_set_deferred_t": (I, [P, I]),
        "soft_graph_info": (I, [P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(t):
    """Device or host pointer of a torch tensor / numpy array, or None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ctypes.c_void_p(t.data_ptr())
    return t.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))


class Context:
    """One soft_ctx (one GPU).  Methods mirror the soft_* calls."""

    def __init__(self, device: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        rc = self._lib.soft_create(ctypes.byref(h), device)
        if rc != SOFT_OK:
            raise SoftError(rc, (self._lib.soft_last_error(None) or b"").decode())
        self._h = h
        self.device = device
        self._ends = None  # shot ranges of a loaded mixture

    def close(self):
        if getattr(self, "_h", None):
            self._lib.soft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != SOFT_OK:
            raise SoftError(rc, (self._lib.soft_last_error(self._h) or b"").decode())

    # --- configuration -------------------------------------------------------
    def load_circuit(self, text: str):
        b = text.encode()
        self._check(self._lib.soft_load_circuit(self._h, b, len(b)))
        self._ends = None

    def load_mixture(self, texts, models, shot_ends):
        """Variant v = (texts[v], models[v] as a dict of soft_noise fields)
        owns the global shots [shot_ends[v-1], shot_ends[v])."""
        import numpy as np
        n = len(texts)
        if not (len(models) == n == len(shot_ends)):
            raise ValueError("texts, models and shot_ends differ in length")
        bufs = [t.encode() for t in texts]
        tarr = (ctypes.c_char_p * n)(*bufs)
        larr = (ctypes.c_size_t * n)(*[len(b) for b in bufs])
        marr = (soft_noise * n)(*[soft_noise(*(float(m.get(k, 0.0)) for k, _ in soft_noise._fields_)) for m in models])
        ends = np.ascontiguousarray(shot_ends, dtype=np.uint64)
        self._check(self._lib.soft_load_mixture(self._h, n, ctypes.cast(tarr, ctypes.c_void_p),
                                                ctypes.cast(larr, ctypes.c_void_p), ctypes.cast(marr, ctypes.c_void_p),
                                                _ptr(ends)))
        self._ends = [int(x) for x in ends]

    def variant_of(self, shot: int) -> int:
        if self._ends is None:
            return 0
        for v, e in enumerate(self._ends):
            if shot < e:
                return v
        raise ValueError("shot beyond the mixture's ranges")

    def load_noise(self, p1=0.0, p2=0.0, p_idle=0.0, p_meas=0.0, p_reset=0.0, p_mpp=0.0):
        m = soft_noise(p1, p2, p_idle, p_meas, p_reset, p_mpp)
        self._check(self._lib.soft_load_noise(self._h, ctypes.byref(m)))

    def set_rng(self, seed: int):
        self._check(self._lib.soft_set_rng(self._h, seed))

    def set_uniforms(self, words_dev, n_shots: int = 0, noise_slots: int = 0, meas_slots: int = 0):
        self._check(self._lib.soft_set_uniforms(self._h, _ptr(words_dev), n_shots, noise_slots, meas_slots))

    def set_precision(self, bits: int):
        self._check(self._lib.soft_set_precision(self._h, bits))

    def set_prune(self, tau: float):
        self._check(self._lib.soft_set_prune(self._h, tau))

    def set_caps(self, support_cap=0, waves_per_block=0, blocks_per_cu=0, grab=0):
        self._check(self._lib.soft_set_caps(self._h, support_cap, waves_per_block, blocks_per_cu, grab))

    def set_speculation(self, on: bool):
        """Run the speculative (span-truncating) event lists first (default)."""
        self._check(self._lib.soft_set_speculation(self._h, 1 if on else 0))

    def set_shared_prefix(self, on: bool):
        """Start each shot at the last checkpoint of the noiseless trajectory
        before its first noise hit (default on; results are the same either
        way)."""
        self._check(self._lib.soft_set_shared_prefix(self._h, 1 if on else 0))

    def set_deferred_t(self, on: bool):
        """Skip T runs whose coefficients no event needs before the shot ends
        (default on; a shot that needs them applies the run when it does, with
        the signs the run saw; a kept shot that ends with a run skipped runs
        again with every run applied)."""
        self._check(self._lib.soft_set_deferred_t(self._h, 1 if on else 0))

    def set_noise_mode(self, mode: int):
        """0: one word per noise location (default); 1: gap sampling."""
        self._check(self._lib.soft_set_noise_mode(self._h, mode))

    def set_tile_memory(self, mode: int, lds_log2: int = 0):
        """0 automatic, 1 LDS, 2 device memory (HBM), 3 split (the low
        2^lds_log2 entries in LDS, the rest in HBM; 0 = default / autotuned)."""
        self._check(self._lib.soft_set_tile_memory(self._h, int(mode) | (int(lds_log2) << 8)))

    def set_keep(self, shot_lo: int, count: int):
        self._check(self._lib.soft_set_keep(self._h, shot_lo, count))

    def autotune(self, sample_shots: int, stream=None):
        self._check(self._lib.soft_autotune(self._h, sample_shots, _stream_handle(stream)))

    # --- running -------------------------------------------------------------
    def run(self, shot0: int, n_shots: int, outcomes=None, status=None, abort_op=None, obs=None, stream=None):
        """Asynchronous on `stream`; tensors must be uint32/int32 CUDA tensors
        of the documented shapes (outcomes [record_words, n_shots])."""
        self._check(self._lib.soft_run(self._h, shot0, n_shots, _ptr(outcomes), _ptr(status), _ptr(abort_op),
                                       _ptr(obs), _stream_handle(stream)))

    def run_noalloc(self, shot0: int, n_shots: int, outcomes=None, status=None, abort_op=None, obs=None,
                    stream=None):
        """soft_run_noalloc: as run(), allocating nothing (counters, cursor and
        device-memory tiles in the library's static per-GPU scratch)."""
        self._check(self._lib.soft_run_noalloc(self._h, shot0, n_shots, _ptr(outcomes), _ptr(status),
                                               _ptr(abort_op), _ptr(obs), _stream_handle(stream)))

    def run_list(self, shots, outcomes=None, status=None, abort_op=None, obs=None, stream=None):
        """Sample the global shot indices in `shots` (an int64 CUDA tensor);
        row i of every output belongs to shots[i].  Asynchronous on `stream`."""
        self._check(self._lib.soft_run_list(self._h, _ptr(shots), int(shots.numel()), _ptr(outcomes), _ptr(status),
                                            _ptr(abort_op), _ptr(obs), _stream_handle(stream)))

    def counters(self, variant: int | None = None) -> dict:
        """Aggregates of the last run (of one variant's shots if given)."""
        c = soft_counters()
        if variant is None:
            self._check(self._lib.soft_read_counters(self._h, ctypes.byref(c)))
        else:
            self._check(self._lib.soft_read_variant_counters(self._h, variant, ctypes.byref(c)))
        out = {f: getattr(c, f) for f, _ in soft_counters._fields_ if f != "support_hist"}
        out["support_hist"] = list(c.support_hist)
        return out

    def read_coeffs(self, shot: int, cap: int = 1 << 16) -> dict:
        import numpy as np
        al = np.zeros(cap, dtype=np.uint64)
        re = np.zeros(cap, dtype=np.float64)
        im = np.zeros(cap, dtype=np.float64)
        cnt = ctypes.c_uint32(0)
        self._check(self._lib.soft_read_coeffs(self._h, shot, _ptr(al), _ptr(re), _ptr(im), cap, ctypes.byref(cnt)))
        k = min(cnt.value, cap)
        return {int(al[i]): complex(re[i], im[i]) for i in range(k)}

    def read_tableau(self, shot: int):
        import numpy as np
        n = self.info(self.variant_of(shot))["qubits"]
        x = np.zeros(2 * n, dtype=np.uint64)
        z = np.zeros(2 * n, dtype=np.uint64)
        r = np.zeros(2 * n, dtype=np.uint8)
        self._check(self._lib.soft_read_tableau(self._h, shot, _ptr(x), _ptr(z), _ptr(r)))
        return x, z, r

    def set_trace(self, shot: int, steps: int):
        self._check(self._lib.soft_set_trace(self._h, shot, steps))
        self._trace_shot = shot

    def read_trace(self, step: int, cap: int = 1 << 16):
        """State after event `step` of the traced shot: None if not reached,
        else a dict with op, status, k, norm2, final, tableau and coeffs."""
        import numpy as np
        n = self.info(self.variant_of(getattr(self, "_trace_shot", 0)))["qubits"]
        info = np.zeros(6, dtype=np.uint64)
        x = np.zeros(2 * n, dtype=np.uint64)
        z = np.zeros(2 * n, dtype=np.uint64)
        r = np.zeros(2 * n, dtype=np.uint8)
        al = np.zeros(cap, dtype=np.uint64)
        re = np.zeros(cap, dtype=np.float64)
        im = np.zeros(cap, dtype=np.float64)
        cnt = ctypes.c_uint32(0)
        self._check(self._lib.soft_read_trace(self._h, step, _ptr(info), _ptr(x), _ptr(z), _ptr(r), _ptr(al),
                                              _ptr(re), _ptr(im), cap, ctypes.byref(cnt)))
        if not info[0]:
            return None
        k = min(cnt.value, cap)
        return {"op": int(info[1]), "status": int(info[2]), "k": int(info[3]),
                "norm2": float(np.array([info[4]], dtype=np.uint64).view(np.float64)[0]),
                "final": bool(info[5]), "x": x, "z": z, "r": r,
                "coeffs": {int(al[i]): complex(re[i], im[i]) for i in range(k)}}

    def info(self, variant: int | None = None) -> dict:
        """Facts about the circuit (largest over a mixture's variants), or
        about one variant."""
        import numpy as np
        a = np.zeros(8, dtype=np.uint64)
        if variant is None:
            self._check(self._lib.soft_circuit_info(self._h, _ptr(a)))
        else:
            self._check(self._lib.soft_variant_info(self._h, variant, _ptr(a)))
        keys = ("qubits", "records", "noise_slots", "meas_slots", "observables", "events", "k_max", "record_words")
        return {k: int(v) for k, v in zip(keys, a)}

    def graph_info(self) -> dict:
        """Graph instantiations and launches of this context so far."""
        import numpy as np
        a = np.zeros(2, dtype=np.uint64)
        self._check(self._lib.soft_graph_info(self._h, _ptr(a)))
        return {"instantiations": int(a[0]), "launches": int(a[1])}

    def launch_shape(self) -> dict:
        import numpy as np
        a = np.zeros(5, dtype=np.uint32)
        self._check(self._lib.soft_launch_shape(self._h, _ptr(a)))
        return dict(zip(("waves_per_block", "blocks_per_cu", "grab", "lds_bytes_per_wave", "tiles_in_memory"),
                        (int(x) for x in a)))


def sample(ctx: Context, shot0: int, n_shots: int, stream=None):
    """Allocate output tensors on the context's GPU, run, and return them."""
    import torch
    dev = torch.device("cuda", ctx.device)
    nw = max(ctx.info()["record_words"], 1)
    outcomes = torch.zeros((nw, n_shots), dtype=torch.int32, device=dev)
    status = torch.zeros(n_shots, dtype=torch.int32, device=dev)
    abort_op = torch.zeros(n_shots, dtype=torch.int32, device=dev)
    obs = torch.zeros(n_shots, dtype=torch.int32, device=dev)
    ctx.run(shot0, n_shots, outcomes, status, abort_op, obs, stream=stream)
    return outcomes, status, abort_op, obs
