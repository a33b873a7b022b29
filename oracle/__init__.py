"""Python view of the CPU FP64 oracle (test infrastructure only).

The oracle is a plain C++ generalized-stabilizer simulator (``oracle.cpp``)
that checks the GPU sampler.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the product library
never does, and nothing here touches the product library.

``build()`` compiles ``liboracle.so`` next to this file with g++.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PASSED, DISCARDED, OVERFLOW, NUMERIC = 0, 1, 2, 3
NO_ABORT = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no GPU toolchain involved)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
               "-Wall", "-Wextra", "-o", tmp, os.path.join(HERE, "oracle.cpp")]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Noise(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("p1", "p2", "p_idle", "p_meas", "p_reset", "p_mpp")]


class _ShotInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_uint32), ("abort_op", ctypes.c_uint32),
                ("obs", ctypes.c_uint32), ("max_support", ctypes.c_uint32),
                ("t_entries", ctypes.c_uint64), ("t_phase_entries", ctypes.c_uint64),
                ("m_entries", ctypes.c_uint64), ("noise_slots", ctypes.c_uint64),
                ("events", ctypes.c_uint64), ("norm2", ctypes.c_double), ("noise_words", ctypes.c_uint64),
                ("m_out_entries", ctypes.c_uint64), ("m_pairs", ctypes.c_uint64),
                ("t_phase_flips", ctypes.c_uint64), ("meas_words", ctypes.c_uint64),
                ("shared", ctypes.c_uint64 * 10)]

WORK_KEYS = ("t_entries", "t_phase_entries", "m_entries", "noise_slots", "events", "noise_words",
             "m_out_entries", "m_pairs", "t_phase_flips", "meas_words")


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_compile.restype = P
        lib.oracle_compile.argtypes = [ctypes.c_char_p, ctypes.POINTER(_Noise), ctypes.c_char_p, ctypes.c_int]
        lib.oracle_free.argtypes = [P]
        lib.oracle_counts.argtypes = [P, P]
        lib.oracle_shot.restype = ctypes.c_int
        lib.oracle_shot.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, P, ctypes.c_double, ctypes.c_uint32,
                                    P, ctypes.POINTER(_ShotInfo), P, P, P, P, P, P, ctypes.c_uint32, P, P]
        lib.oracle_batch.restype = ctypes.c_int
        lib.oracle_batch.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, P, ctypes.c_double,
                                     ctypes.c_uint32, ctypes.c_int, P, P, P, P, P, P, P]
        lib.oracle_set_noise_mode.restype = ctypes.c_int
        lib.oracle_set_noise_mode.argtypes = [P, ctypes.c_int]
        lib.oracle_philox.argtypes = [P, P, P]
        lib.oracle_pauli_mul.argtypes = [P, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key):
    """One Philox4x32-10 block: 4 counter words, 2 key words -> 4 words."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def pauli_mul(a, b):
    """(x, z, e) * (x, z, e) -> (x, z, e) with e the exponent of i."""
    lib = _load()
    A = np.array(a, dtype=np.uint64)
    B = np.array(b, dtype=np.uint64)
    out = np.zeros(3, dtype=np.uint64)
    lib.oracle_pauli_mul(_ptr(A), _ptr(B), _ptr(out))
    return int(out[0]), int(out[1]), int(out[2])


@dataclass
class ShotResult:
    record: list          # measurement record bits
    status: int
    abort_op: int
    obs: int
    max_support: int
    tab_x: np.ndarray     # uint64 [2n]: destabilizer rows then stabilizer rows
    tab_z: np.ndarray
    tab_r: np.ndarray     # uint8 [2n]
    coeffs: dict          # alpha -> complex
    p0: np.ndarray        # P(outcome +1) per measurement slot
    work: dict
    norm2: float
    shared_work: dict     # the part of `work` done on the noiseless trajectory all shots share


class Circuit:
    """A parsed and noise-lowered circuit held by the oracle."""

    def __init__(self, text: str, noise: dict | None = None, noise_mode: int = 0):
        lib = _load()
        nz = _Noise(**(noise or {}))
        err = ctypes.create_string_buffer(512)
        h = lib.oracle_compile(text.encode(), ctypes.byref(nz), err, 512)
        if not h:
            raise ValueError("oracle parse error: " + err.value.decode())
        self._h = h
        counts = np.zeros(7, dtype=np.uint64)
        lib.oracle_counts(h, _ptr(counts))
        (self.n_qubits, self.n_ops, self.n_records, self.n_noise_slots,
         self.n_meas_slots, self.n_observables, self.n_lowered) = (int(x) for x in counts)
        if lib.oracle_set_noise_mode(h, int(noise_mode)) != 0:
            raise ValueError(f"bad noise mode {noise_mode}")
        self.noise_mode = int(noise_mode)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_free(h)
            self._h = None

    @property
    def words_per_shot(self) -> int:
        return self.n_noise_slots + self.n_meas_slots

    def shot(self, seed: int, shot: int, words=None, tau: float = 1e-12, cap: int = 0xFFFFFFFF,
             coeff_cap: int = 1 << 16) -> ShotResult:
        lib = _load()
        n = self.n_qubits
        rec = np.zeros(max(1, (self.n_records + 31) // 32), dtype=np.uint32)
        info = _ShotInfo()
        tx = np.zeros(2 * n, dtype=np.uint64)
        tz = np.zeros(2 * n, dtype=np.uint64)
        tr = np.zeros(2 * n, dtype=np.uint8)
        al = np.zeros(coeff_cap, dtype=np.uint64)
        re = np.zeros(coeff_cap, dtype=np.float64)
        im = np.zeros(coeff_cap, dtype=np.float64)
        nc = ctypes.c_uint32(0)
        p0 = np.full(max(1, self.n_meas_slots), np.nan)
        w = None
        if words is not None:
            w = np.ascontiguousarray(words, dtype=np.uint32)
            if w.size != self.words_per_shot:
                raise ValueError("explicit words: expected %d" % self.words_per_shot)
        rc = lib.oracle_shot(self._h, seed, shot, _ptr(w), tau, cap, _ptr(rec), ctypes.byref(info),
                             _ptr(tx), _ptr(tz), _ptr(tr), _ptr(al), _ptr(re), _ptr(im), coeff_cap,
                             ctypes.byref(nc), _ptr(p0))
        if rc != 0:
            raise RuntimeError("oracle_shot failed")
        k = min(nc.value, coeff_cap)
        bits = [int((rec[i >> 5] >> (i & 31)) & 1) for i in range(self.n_records)]
        coeffs = {int(al[i]): complex(re[i], im[i]) for i in range(k)}
        work = {f: int(getattr(info, f)) for f in WORK_KEYS}
        shared = dict(zip(WORK_KEYS, (int(x) for x in info.shared)))
        return ShotResult(bits, info.status, info.abort_op, info.obs, info.max_support, tx, tz, tr,
                          coeffs, p0[: self.n_meas_slots], work, info.norm2, shared)

    def batch(self, seed: int, shot0: int, n: int, words=None, tau: float = 1e-12,
              cap: int = 0xFFFFFFFF, threads: int | None = None) -> dict:
        lib = _load()
        if threads is None:
            threads = max(1, min(len(os.sched_getaffinity(0)), 16))
        nw = (self.n_records + 31) // 32
        outcomes = np.zeros((max(nw, 1), n), dtype=np.uint32)
        status = np.zeros(n, dtype=np.uint32)
        abort_op = np.zeros(n, dtype=np.uint32)
        obs = np.zeros(n, dtype=np.uint32)
        maxs = np.zeros(n, dtype=np.uint32)
        work = np.zeros(len(WORK_KEYS), dtype=np.uint64)
        shared = np.zeros(len(WORK_KEYS), dtype=np.uint64)
        w = None
        if words is not None:
            w = np.ascontiguousarray(words, dtype=np.uint32)
            if w.shape != (n, self.words_per_shot):
                raise ValueError("explicit words: expected shape (%d, %d)" % (n, self.words_per_shot))
        rc = lib.oracle_batch(self._h, seed, shot0, n, _ptr(w), tau, cap, threads, _ptr(outcomes),
                              _ptr(status), _ptr(abort_op), _ptr(obs), _ptr(maxs), _ptr(work), _ptr(shared))
        if rc != 0:
            raise RuntimeError("oracle_batch failed")
        return {"outcomes": outcomes[:nw], "status": status, "abort_op": abort_op, "obs": obs,
                "max_support": maxs, "threads": threads,
                "work": dict(zip(WORK_KEYS, (int(x) for x in work))),
                "shared_work": dict(zip(WORK_KEYS, (int(x) for x in shared)))}
