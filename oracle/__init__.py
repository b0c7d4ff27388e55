"""Plain FP64 CPU oracle of the aliasing-filter sparse FFT (test infrastructure).

TEST INFRASTRUCTURE ONLY.  The test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only code that may import this
package.  It shares no code with the GPU library: the C source beside this
file is compiled with gcc into ``oracle/_build/liborc.so`` and driven through
ctypes.  Every function of the C file cites the passage of the paper (Li,
Jiang & Chen 2020) that it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sfft_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liborc.so")

EXACT, NOISY = 0, 1
TREE, FFAST = 0, 1
ZERO, SINGLE, MULTI, DOUBLE = 0, 1, 2, 3
OK, PARTIAL = 0, 1

MAX_ROUNDS = 16
MAX_STAGES = 8
MAX_LEVELS = 64
MAX_STARTS = 64


class Cfg(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("K", ctypes.c_int64),
        ("kind", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("R", ctypes.c_int32), ("D", ctypes.c_int32),
        ("B0", ctypes.c_int64),
        ("stageB", ctypes.c_int64 * MAX_STAGES),
        ("sigma", ctypes.c_uint64 * MAX_ROUNDS),
        ("shift", ctypes.c_uint64 * MAX_ROUNDS),
        ("max_levels", ctypes.c_int32), ("window", ctypes.c_int32),
        ("max_peel_rounds", ctypes.c_int32),
        ("eps0", ctypes.c_double), ("eps1", ctypes.c_double),
        ("zero_k", ctypes.c_double), ("single_k", ctypes.c_double),
        ("noise_var", ctypes.c_double),
        ("mpp", ctypes.c_int32),
        ("rf_iters", ctypes.c_int32), ("rf_m", ctypes.c_int32),
        ("rf_off", ctypes.c_uint64 * MAX_ROUNDS),
        ("n_starts", ctypes.c_int32),
        ("start_f", ctypes.c_int64 * MAX_STARTS),
    ]


class Trace(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("n_zero", ctypes.c_int32 * MAX_LEVELS),
        ("n_single", ctypes.c_int32 * MAX_LEVELS),
        ("n_multi", ctypes.c_int32 * MAX_LEVELS),
        ("occupied", ctypes.c_int32 * MAX_LEVELS),
        ("ident", ctypes.c_int32 * MAX_LEVELS),
        ("samples", ctypes.c_int64),
        ("sref2", ctypes.c_double), ("noise_var", ctypes.c_double),
        ("n_found", ctypes.c_int64),
        ("order", ctypes.c_int64 * 4096),
        ("n_double", ctypes.c_int32 * MAX_LEVELS),
    ]


def build(force: bool = False, extra_flags: tuple = (), out: str | None = None) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    out = out or _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "sfft_oracle.h"))):
        os.makedirs(os.path.dirname(out), exist_ok=True)
        tmp = f"{out}.{os.getpid()}.tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
               *extra_flags, "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)   # atomic: parallel test workers never see a partial file
    return out


_libs: dict = {}


def lib(path: str | None = None):
    path = path or _LIB
    if path not in _libs:
        if path == _LIB:
            build()
        L = ctypes.CDLL(path)
        L.orc_config.argtypes = [ctypes.POINTER(Cfg), ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                 ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
        L.orc_config.restype = ctypes.c_int
        L.orc_config_stages.argtypes = [ctypes.POINTER(Cfg), ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.c_int32, ctypes.c_int32]
        L.orc_config_stages.restype = ctypes.c_int
        L.orc_splitmix64_next.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        L.orc_splitmix64_next.restype = ctypes.c_uint64
        L.orc_draw_starts.argtypes = [ctypes.POINTER(Cfg), ctypes.c_uint64, ctypes.c_int32]
        L.orc_draw_starts.restype = ctypes.c_int
        L.orc_set_rffast.argtypes = [ctypes.POINTER(Cfg), ctypes.c_uint64, ctypes.c_int32,
                                     ctypes.c_int32]
        L.orc_set_rffast.restype = ctypes.c_int
        L.orc_kay_phase.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.orc_kay_phase.restype = ctypes.c_double
        L.orc_bin.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        L.orc_bin.restype = None
        L.orc_level0.argtypes = [ctypes.POINTER(Cfg), ctypes.c_void_p, ctypes.c_void_p]
        L.orc_level0.restype = ctypes.c_int
        L.orc_classify_tree.argtypes = [ctypes.POINTER(Cfg), ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
        L.orc_classify_tree.restype = ctypes.c_int32
        L.orc_estimate_noise.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double]
        L.orc_estimate_noise.restype = ctypes.c_double
        L.orc_solve.argtypes = [ctypes.POINTER(Cfg), ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.POINTER(Trace)]
        L.orc_solve.restype = ctypes.c_int64
        _libs[path] = L
    return _libs[path]


def config(N, K, stages, delays, seed=0, mode=EXACT, B0=0, identity_round0=False,
           stageB=None, libpath=None, **overrides) -> Cfg:
    """Plan of the oracle: its own factoring and its own SplitMix64 draws."""
    L = lib(libpath)
    c = Cfg()
    if stageB is not None:
        arr = (ctypes.c_int64 * len(stageB))(*stageB)
        rc = L.orc_config_stages(ctypes.byref(c), N, K, len(stageB), arr, delays, mode)
    else:
        rc = L.orc_config(ctypes.byref(c), N, K, stages, delays, seed, mode, B0,
                          1 if identity_round0 else 0)
    if rc != 0:
        raise ValueError(f"oracle config rejected (rc={rc}) N={N} K={K} stages={stages} "
                         f"delays={delays} mode={mode} B0={B0}")
    if "rffast" in overrides:
        C, m = overrides.pop("rffast")
        if L.orc_set_rffast(ctypes.byref(c), seed, int(C), int(m)) != 0:
            raise ValueError("R-FFAST delay set rejected")
    for k, v in overrides.items():
        if k == "start_f":
            c.n_starts = len(v)
            for i, f in enumerate(v):
                c.start_f[i] = int(f)
            continue
        if k == "peel_starts":
            if L.orc_draw_starts(ctypes.byref(c), seed, int(v)) != 0:
                raise ValueError("too many start frequencies")
            continue
        setattr(c, k, v)
    return c


def _as_c64(x):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex64))
    return x


def bin_value(x, N, B, sigma, tau, h, libpath=None) -> complex:
    x = _as_c64(x)
    out = np.zeros(2, dtype=np.float64)
    lib(libpath).orc_bin(x.ctypes.data, N, B, sigma, tau, h, out.ctypes.data)
    return complex(out[0], out[1])


def level0(cfg: Cfg, x, libpath=None) -> np.ndarray:
    """Level-0 class table: tree -> (B0, R*D); FFAST -> (sum B_j, D)."""
    x = _as_c64(x)
    if cfg.kind == TREE:
        rows, n = cfg.B0, cfg.R * cfg.D
    else:
        rows, n = sum(cfg.stageB[j] for j in range(cfg.R)), cfg.D
    out = np.zeros((rows, n), dtype=np.complex128)
    lib(libpath).orc_level0(ctypes.byref(cfg), x.ctypes.data, out.ctypes.data)
    return out


def solve(cfg: Cfg, x, libpath=None):
    """Full solve; returns (idx[K], val[K] complex128, count, trace)."""
    x = _as_c64(x)
    if x.shape[0] != cfg.N:
        raise ValueError("signal length does not match the plan")
    idx = np.zeros(cfg.K, dtype=np.int64)
    val = np.zeros(cfg.K, dtype=np.complex128)
    tr = Trace()
    cnt = lib(libpath).orc_solve(ctypes.byref(cfg), x.ctypes.data, idx.ctypes.data,
                                 val.ctypes.data, ctypes.byref(tr))
    return idx, val, int(cnt), tr


def classify_tree(cfg: Cfg, Y, cls: int, B: int, sref2: float = 0.0, noise_var: float = 0.0,
                  libpath=None):
    """Decision rule alone on one tree class vector Y (R*D complex values):
    returns (class code, position, value)."""
    Y = np.ascontiguousarray(np.asarray(Y, dtype=np.complex128))
    if Y.shape != (cfg.R * cfg.D,):
        raise ValueError("class vector must hold R*D values")
    f = ctypes.c_int64(0)
    a = np.zeros(2, dtype=np.float64)
    code = lib(libpath).orc_classify_tree(ctypes.byref(cfg), Y.ctypes.data, int(cls), int(B),
                                          float(sref2), float(noise_var), ctypes.byref(f),
                                          a.ctypes.data)
    return int(code), int(f.value), complex(a[0], a[1])


def estimate_noise(pw, phi: float, libpath=None) -> float:
    """Noise variance estimate from values B |yhat|^2 and the expected
    noise-only fraction phi of the entries."""
    pw = np.array(pw, dtype=np.float64)  # a copy: the oracle sorts in place
    return float(lib(libpath).orc_estimate_noise(pw.ctypes.data, len(pw), float(phi)))


def kay_phase(y, libpath=None) -> float:
    """Kay's weighted phase-difference estimate of m samples (Eq. 21-22)."""
    y = np.ascontiguousarray(np.asarray(y, dtype=np.complex128))
    return float(lib(libpath).orc_kay_phase(y.ctypes.data, len(y)))


def splitmix64(seed: int, count: int, libpath=None):
    st = ctypes.c_uint64(seed)
    L = lib(libpath)
    return [int(L.orc_splitmix64_next(ctypes.byref(st))) for _ in range(count)]
