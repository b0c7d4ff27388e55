"""Python binding of libsfft (aliasing-filter sparse FFT on MI355X / gfx950).

Argument marshalling only: every step of a solve runs in the HIP kernels of
``csrc/``; torch supplies device memory and streams.  Importing this package
raises if the compiled library is missing -- there is no CPU fallback.

    import torch, paper_2011_05749_amd as sfft
    plan = sfft.Plan(N=2**22, K=1024, stages=4, delays=2, seed=1, B0=2048)
    idx, val, count = plan.exec(x)            # x: complex64 cuda tensor [N]
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libsfft.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libsfft.so not found at {LIB_PATH}: build it with "
        "`python paper_2011_05749_amd/build.py` (hipcc, gfx950); there is no fallback")

# torch is loaded first so that the library's libamdhip64.so.7 dependency binds
# to the HIP runtime torch already holds: a process must not carry two HIP/HSA
# runtimes (torch's and /opt/rocm's), which would each open the device and not
# know the other's allocations.
import torch  # noqa: E402,F401  (device memory and streams come from torch)

_lib = ctypes.CDLL(LIB_PATH)

MAX_ROUNDS = 16
MAX_STAGES = 8
MAX_PEEL_STARTS = 64
EXACT, NOISY = 0, 1
KIND_TREE, KIND_FFAST = 0, 1
STATUS_OK, STATUS_PARTIAL = 0, 1
BATCH_NO_GRAPH = 1
ERRORS = {0: "ok", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "ENOMEM", -4: "EDEVICE", -5: "ETOOBIG"}
NOALLOC_SCRATCH_MIB = 64


class Params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("K", ctypes.c_int64),
        ("stages", ctypes.c_int32), ("delays", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("mode", ctypes.c_int32),
        ("B0", ctypes.c_int64),
        ("max_levels", ctypes.c_int32), ("window", ctypes.c_int32),
        ("identity_round0", ctypes.c_int32), ("nstage_B", ctypes.c_int32),
        ("stage_B", ctypes.c_int64 * MAX_STAGES),
        ("max_peel_rounds", ctypes.c_int32), ("jump_L", ctypes.c_int32),
        ("eps0", ctypes.c_double), ("eps1", ctypes.c_double),
        ("zero_k", ctypes.c_double), ("single_k", ctypes.c_double),
        ("noise_var", ctypes.c_double),
        ("mpp", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("rf_iters", ctypes.c_int32), ("rf_m", ctypes.c_int32),
        ("peel_starts", ctypes.c_int32),
        ("peel_start_f", ctypes.c_int64 * MAX_PEEL_STARTS),
        ("l1_resolve", ctypes.c_int32),
        ("sample_format", ctypes.c_int32),
        ("fft_tile_lg", ctypes.c_int32), ("gather_unroll", ctypes.c_int32),
        ("col_form", ctypes.c_int32), ("enum_share", ctypes.c_int32),
        ("l0_spread", ctypes.c_int32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("K", ctypes.c_int64),
        ("kind", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("R", ctypes.c_int32), ("D", ctypes.c_int32),
        ("B0", ctypes.c_int64),
        ("max_levels", ctypes.c_int32), ("window", ctypes.c_int32),
        ("stage_B", ctypes.c_int64 * MAX_STAGES),
        ("sigma", ctypes.c_uint64 * MAX_ROUNDS),
        ("shift", ctypes.c_uint64 * MAX_ROUNDS),
        ("eps0", ctypes.c_double), ("eps1", ctypes.c_double),
        ("zero_k", ctypes.c_double), ("single_k", ctypes.c_double),
        ("noise_var", ctypes.c_double),
        ("max_peel_rounds", ctypes.c_int32), ("jump_L", ctypes.c_int32),
        ("found_cap", ctypes.c_int32), ("multi_cap", ctypes.c_int32),
        ("mpp", ctypes.c_int32),
        ("peel_starts", ctypes.c_int32),
        ("peel_start_f", ctypes.c_int64 * MAX_PEEL_STARTS),
        ("rf_iters", ctypes.c_int32), ("rf_m", ctypes.c_int32),
        ("rf_off", ctypes.c_uint64 * MAX_ROUNDS),
        ("precision", ctypes.c_int32),
        ("l1_resolve", ctypes.c_int32),
        ("sample_format", ctypes.c_int32),
        ("fft_tile_lg", ctypes.c_int32), ("gather_unroll", ctypes.c_int32),
        ("col_form", ctypes.c_int32), ("enum_share", ctypes.c_int32),
        ("l0_spread", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int64), ("status", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("samples", ctypes.c_int64), ("found", ctypes.c_int64),
        ("noise_var", ctypes.c_double), ("sref2", ctypes.c_double),
        ("level_mask", ctypes.c_uint64), ("ident", ctypes.c_int64),
        ("h2d_bytes", ctypes.c_int64),
    ]


class Workspace(ctypes.Structure):
    _fields_ = [
        ("bytes", ctypes.c_int64), ("y0", ctypes.c_int64), ("fst", ctypes.c_int64),
        ("found", ctypes.c_int64), ("multi", ctypes.c_int64), ("multi_vec", ctypes.c_int64),
        ("jacc", ctypes.c_int64), ("jcol", ctypes.c_int64),
        ("nmax", ctypes.c_int32), ("jstride", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("nsig", ctypes.c_int32),
    ]


class WorkspaceSignal(ctypes.Structure):
    _fields_ = [
        ("y0_off", ctypes.c_int64), ("fst_off", ctypes.c_int64), ("found_off", ctypes.c_int64),
        ("multi_off", ctypes.c_int64), ("jcol_off", ctypes.c_int64),
        ("found_cap", ctypes.c_int32), ("multi_cap", ctypes.c_int32), ("n", ctypes.c_int32),
        ("l1", ctypes.c_int32), ("jump_L", ctypes.c_int32), ("col_rows", ctypes.c_int32),
    ]


class ServerParams(ctypes.Structure):
    _fields_ = [("hbm_bytes", ctypes.c_int64), ("lanes", ctypes.c_int32),
                ("max_batch", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("release_ns", ctypes.c_int64), ("launch_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("batch", ctypes.c_int32), ("lane", ctypes.c_int32),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32)]


KERNEL_NAMES = {0: "k_reset", 1: "k_level0", 2: "k_sched", 3: "k_expand_fft",
                4: "k_expand_direct", 5: "k_children", 6: "k_finalize", 7: "k_jump_pass",
                8: "k_jump_resolve", 9: "k_col_pass", 10: "k_col_resolve",
                11: "k_col_deep"}

_vp = ctypes.c_void_p
_lib.sfft_params_init.argtypes = [ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
_lib.sfft_params_init.restype = None
_lib.sfft_plan.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                           ctypes.c_uint64]
_lib.sfft_plan.restype = _vp
_lib.sfft_plan_ex.argtypes = [ctypes.POINTER(Params)]
_lib.sfft_plan_ex.restype = _vp
_lib.sfft_plan_info.argtypes = [_vp, ctypes.POINTER(PlanInfo)]
_lib.sfft_plan_info.restype = ctypes.c_int32
_lib.sfft_destroy.argtypes = [_vp]
_lib.sfft_destroy.restype = None
_lib.sfft_exec.argtypes = [_vp, _vp, _vp, _vp]
_lib.sfft_exec.restype = ctypes.c_int64
_lib.sfft_exec_host.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(Stats)]
_lib.sfft_exec_host.restype = ctypes.c_int64
_lib.sfft_exec_async.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.sfft_exec_async.restype = ctypes.c_int32
_lib.sfft_exec_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.sfft_exec_noalloc.restype = ctypes.c_int32
_lib.sfft_exec_batch.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp]
_lib.sfft_exec_batch.restype = ctypes.c_int32
_lib.sfft_exec_batch_ex.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp,
                                    ctypes.c_int32]
_lib.sfft_exec_batch_ex.restype = ctypes.c_int32
_lib.sfft_exec_batch_profile.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp,
                                         ctypes.c_int32]
_lib.sfft_exec_batch_profile.restype = ctypes.c_int32
_lib.sfft_bucketize.argtypes = [_vp, _vp, _vp]
_lib.sfft_bucketize.restype = ctypes.c_int32
_lib.sfft_exec_stats.argtypes = [_vp, ctypes.POINTER(Stats)]
_lib.sfft_exec_stats.restype = ctypes.c_int32
_lib.sfft_batch_stats.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Stats)]
_lib.sfft_batch_stats.restype = ctypes.c_int32
_lib.sfft_workspace.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(Workspace), _vp]
_lib.sfft_workspace.restype = ctypes.c_int32
_lib.sfft_server_params_init.argtypes = [ctypes.POINTER(ServerParams)]
_lib.sfft_server_params_init.restype = None
_lib.sfft_server_create.argtypes = [ctypes.POINTER(ServerParams)]
_lib.sfft_server_create.restype = _vp
_lib.sfft_server_clock_ns.argtypes = []
_lib.sfft_server_clock_ns.restype = ctypes.c_int64
_lib.sfft_server_submit_many.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.sfft_server_submit_many.restype = ctypes.c_int32
_lib.sfft_server_submit.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int64]
_lib.sfft_server_submit.restype = ctypes.c_int64
_lib.sfft_server_requests.argtypes = [_vp, ctypes.c_int64, ctypes.c_int32, _vp]
_lib.sfft_server_requests.restype = ctypes.c_int32
_lib.sfft_server_wait.argtypes = [_vp, ctypes.c_int64]
_lib.sfft_server_wait.restype = ctypes.c_int32
_lib.sfft_server_drain.argtypes = [_vp]
_lib.sfft_server_drain.restype = ctypes.c_int32
_lib.sfft_server_destroy.argtypes = [_vp]
_lib.sfft_server_destroy.restype = None
_lib.sfft_pack_fp16.argtypes = [_vp, ctypes.c_int64, _vp, _vp]
_lib.sfft_pack_fp16.restype = ctypes.c_int32
_lib.sfft_release_batches.argtypes = []
_lib.sfft_release_batches.restype = None
_lib.sfft_last_error.argtypes = []
_lib.sfft_last_error.restype = ctypes.c_int32
_lib.sfft_strerror.argtypes = [ctypes.c_int32]
_lib.sfft_strerror.restype = ctypes.c_char_p

EXPORTS = ["sfft_params_init", "sfft_plan", "sfft_plan_ex", "sfft_plan_info", "sfft_destroy",
           "sfft_exec", "sfft_exec_host", "sfft_exec_async", "sfft_exec_batch", "sfft_exec_batch_ex",
           "sfft_exec_batch_profile",
           "sfft_bucketize", "sfft_exec_stats", "sfft_batch_stats", "sfft_release_batches",
           "sfft_workspace", "sfft_exec_noalloc", "sfft_server_params_init", "sfft_server_create",
           "sfft_server_clock_ns", "sfft_server_submit_many", "sfft_server_submit",
           "sfft_server_requests", "sfft_server_wait", "sfft_server_drain", "sfft_server_destroy",
           "sfft_pack_fp16",
           "sfft_last_error", "sfft_strerror"]


class SfftError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = int(code)
        msg = _lib.sfft_strerror(self.code).decode()
        super().__init__(f"{what}: {ERRORS.get(self.code, self.code)} ({msg})")


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise SfftError(rc, what)
    return rc


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


F16_HEADER_BYTES = 16
SAMPLES_C64, SAMPLES_F16 = 0, 1


def _sig_ptr(plan, x, what="x"):
    """Device pointer of a signal in the plan's sample format: complex64[N],
    or the packed FP16 form (uint8[16 + 4 N], see pack_fp16)."""
    if plan.info.sample_format == SAMPLES_F16:
        return _dev_ptr(x, "uint8", F16_HEADER_BYTES + 4 * plan.N, what)
    return _dev_ptr(x, "complex64", plan.N, what)


def pack_fp16(x, out=None, stream=None):
    """Packed FP16 form of a complex64 device signal (sfft_pack_fp16): uint8
    tensor of 16 + 4 N bytes (header with the power-of-two scale, then
    binary16 pairs)."""
    import torch
    n = x.numel()
    if out is None:
        out = torch.empty(F16_HEADER_BYTES + 4 * n, dtype=torch.uint8, device=x.device)
    _check(_lib.sfft_pack_fp16(_dev_ptr(x, "complex64", n, "x"), n,
                               _dev_ptr(out, "uint8", F16_HEADER_BYTES + 4 * n, "out"),
                               _stream_handle(stream)), "sfft_pack_fp16")
    return out


def _dev_ptr(t, dtype_name, n=None, what="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise SfftError(-1, f"{what} must be a device tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise SfftError(-1, f"{what} must be {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise SfftError(-1, f"{what} must be contiguous")
    if n is not None and t.numel() < n:
        raise SfftError(-1, f"{what} holds {t.numel()} < {n} elements")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """An sfft plan (immutable).  Keyword parameters map onto sfft_params_t:
    mode ('exact'|'noisy' or 0|1), B0, max_levels, window, identity_round0,
    stage_B (explicit co-prime FFAST stages), max_peel_rounds, jump_L, eps0, eps1,
    zero_k, single_k, noise_var, mpp (2 = two-ton moment preserving solve), peel_starts
    (FFAST packet-erasure schedule: number of drawn start frequencies) or peel_start_f
    (explicit start frequencies), rf_iters and rf_m (FFAST R-FFAST delay set and
    singleton estimator), precision (0: FP64 decisions, 1: FP32), l1_resolve (1:
    level-1 column pass when the shape allows, 0: off)."""

    def __init__(self, N: int, K: int, stages: int, delays: int, seed: int = 0, **kw):
        p = Params()
        _lib.sfft_params_init(ctypes.byref(p), N, K, stages, delays, seed)
        for k, v in kw.items():
            if k == "mode":
                v = {"exact": EXACT, "noisy": NOISY}.get(v, v)
            if k == "stage_B":
                p.nstage_B = len(v)
                for j, b in enumerate(v):
                    p.stage_B[j] = int(b)
                continue
            if k == "peel_start_f":
                p.peel_starts = len(v)
                for j, f in enumerate(v):
                    p.peel_start_f[j] = int(f)
                continue
            if not hasattr(p, k):
                raise TypeError(f"unknown plan parameter {k}")
            setattr(p, k, v)
        self.params = p
        h = _lib.sfft_plan_ex(ctypes.byref(p))
        if not h:
            raise SfftError(_lib.sfft_last_error(), "sfft_plan_ex")
        self._h = ctypes.c_void_p(h)
        inf = PlanInfo()
        _check(_lib.sfft_plan_info(self._h, ctypes.byref(inf)), "sfft_plan_info")
        self.info = inf
        self.N, self.K = int(inf.N), int(inf.K)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.sfft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n_meas(self) -> int:
        return self.info.R * self.info.D if self.info.kind == KIND_TREE else self.info.D

    def exec(self, x, out_idx=None, out_val=None):
        """Synchronous solve: returns (idx int64[K], val complex64[K], count)."""
        import torch
        xp = _sig_ptr(self, x)
        if out_idx is None:
            out_idx = torch.empty(self.K, dtype=torch.int64, device=x.device)
        if out_val is None:
            out_val = torch.empty(self.K, dtype=torch.complex64, device=x.device)
        ip = _dev_ptr(out_idx, "int64", self.K, "out_idx")
        vp = _dev_ptr(out_val, "complex64", self.K, "out_val")
        cnt = _check(_lib.sfft_exec(self._h, xp, ip, vp), "sfft_exec")
        return out_idx, out_val, int(cnt)

    def exec_host(self, x):
        """Solve of a host-resident signal (numpy complex64[N]); only the samples
        the solve reads are copied to the device.  Returns (idx int64[K],
        val complex64[K], count, stats) as numpy arrays and a dict."""
        import numpy as np
        x = np.ascontiguousarray(x, dtype=np.complex64)
        if x.shape != (self.N,):
            raise SfftError(-1, f"x must be complex64[{self.N}]")
        idx = np.empty(self.K, dtype=np.int64)
        val = np.empty(self.K, dtype=np.complex64)
        st = Stats()
        cnt = _check(_lib.sfft_exec_host(self._h, x.ctypes.data, idx.ctypes.data, val.ctypes.data,
                                         ctypes.byref(st)), "sfft_exec_host")
        return idx, val, int(cnt), {f: getattr(st, f) for f, _ in Stats._fields_}

    def exec_async(self, x, out_idx, out_val, d_count, d_status, stream=None):
        _check(_lib.sfft_exec_async(
            self._h, _sig_ptr(self, x),
            _dev_ptr(out_idx, "int64", self.K, "out_idx"),
            _dev_ptr(out_val, "complex64", self.K, "out_val"),
            _dev_ptr(d_count, "int64", 1, "d_count"), _dev_ptr(d_status, "int32", 1, "d_status"),
            _stream_handle(stream)), "sfft_exec_async")

    def exec_noalloc(self, x, out_idx, out_val, d_count, d_status, stream=None):
        """sfft_exec_noalloc: as exec_async, with the workspace in the library's
        static device scratch (no device allocation)."""
        _check(_lib.sfft_exec_noalloc(
            self._h, _sig_ptr(self, x),
            _dev_ptr(out_idx, "int64", self.K, "out_idx"),
            _dev_ptr(out_val, "complex64", self.K, "out_val"),
            _dev_ptr(d_count, "int64", 1, "d_count"), _dev_ptr(d_status, "int32", 1, "d_status"),
            _stream_handle(stream)), "sfft_exec_noalloc")

    def bucketize(self, x):
        """Level-0 class vectors (complex64): tree (B0, R*D); FFAST (sum B_j, D)."""
        import torch
        inf = self.info
        if inf.kind == KIND_TREE:
            shape = (int(inf.B0), int(inf.R * inf.D))
        else:
            shape = (int(sum(inf.stage_B[j] for j in range(inf.R))), int(inf.D))
        out = torch.empty(shape, dtype=torch.complex64, device=x.device)
        _check(_lib.sfft_bucketize(self._h, _sig_ptr(self, x),
                                   _dev_ptr(out, "complex64", None, "out")), "sfft_bucketize")
        return out

    def stats(self) -> dict:
        s = Stats()
        _check(_lib.sfft_exec_stats(self._h, ctypes.byref(s)), "sfft_exec_stats")
        return {f: getattr(s, f) for f, _ in Stats._fields_}


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[p.value if isinstance(p, ctypes.c_void_p) else p
                                          for p in ptrs])
    return arr


class Batch:
    """Pre-marshalled arguments of sfft_exec_batch for a fixed list of plans and
    buffers (so that the timed call does no Python-side allocation)."""

    def __init__(self, plans, xs, idxs=None, vals=None):
        import torch
        n = len(plans)
        if n < 1 or len(xs) != n:
            raise SfftError(-1, "Batch needs one signal per plan")
        dev = xs[0].device
        self.plans = list(plans)
        self.xs = list(xs)
        self.idxs = idxs if idxs is not None else [
            torch.empty(p.K, dtype=torch.int64, device=dev) for p in plans]
        self.vals = vals if vals is not None else [
            torch.empty(p.K, dtype=torch.complex64, device=dev) for p in plans]
        self.counts = torch.zeros(n, dtype=torch.int64, device=dev)
        self.status = torch.zeros(n, dtype=torch.int32, device=dev)
        self._plans = _ptr_array([p.handle for p in plans])
        self._xs = _ptr_array([_sig_ptr(p, x) for p, x in zip(plans, self.xs)])
        self._idx = _ptr_array([_dev_ptr(t, "int64", p.K, "idx") for p, t in zip(plans, self.idxs)])
        self._val = _ptr_array([_dev_ptr(t, "complex64", p.K, "val")
                                for p, t in zip(plans, self.vals)])
        self._cnt = _dev_ptr(self.counts, "int64", n, "counts")
        self._st = _dev_ptr(self.status, "int32", n, "status")
        self.n = n

    def run(self, graph: bool = True, stream=None):
        _check(_lib.sfft_exec_batch_ex(self._plans, self._xs, self._idx, self._val, self._cnt,
                                       self._st, self.n, _stream_handle(stream),
                                       0 if graph else BATCH_NO_GRAPH), "sfft_exec_batch")

    def profile(self, cap: int = 4096):
        """Eager run with a HIP event after every launch: list of
        (kernel name, level, milliseconds) in launch order."""
        ms = (ctypes.c_float * cap)()
        ids = (ctypes.c_int32 * cap)()
        n = _check(_lib.sfft_exec_batch_profile(self._plans, self._xs, self._idx, self._val,
                                                self._cnt, self._st, self.n, ms, ids, cap),
                   "sfft_exec_batch_profile")
        return [(KERNEL_NAMES.get(ids[i] & 255, str(ids[i] & 255)), ids[i] >> 8, float(ms[i]))
                for i in range(n)]

    def stats(self, i: int) -> dict:
        s = Stats()
        _check(_lib.sfft_batch_stats(self._plans, self.n, i, ctypes.byref(s)), "sfft_batch_stats")
        return {f: getattr(s, f) for f, _ in Stats._fields_}


def exec_batch(plans, xs, graph: bool = True, stream=None):
    """One batched solve; returns the Batch holding idxs, vals, counts, status."""
    b = Batch(plans, xs)
    b.run(graph=graph, stream=stream)
    return b


def workspace(plans):
    """Device workspace of a batch of these plans (host-only; no device call):
    (arena sizes as a dict, one dict of offsets per signal)."""
    n = len(plans)
    w = Workspace()
    sig = (WorkspaceSignal * n)()
    _check(_lib.sfft_workspace(_ptr_array([p.handle for p in plans]), n, ctypes.byref(w),
                               ctypes.cast(sig, ctypes.c_void_p)), "sfft_workspace")
    return ({f: getattr(w, f) for f, _ in Workspace._fields_},
            [{f: getattr(x, f) for f, _ in WorkspaceSignal._fields_} for x in sig])


class Server:
    """Serving loop (sfft_server_*): continuous batching of independent solves
    with admission by HBM footprint.  submit() queues requests with release
    times on the server clock (clock_ns()); requests() returns their times."""

    def __init__(self, hbm_bytes: int = 8 << 30, lanes: int = 2, max_batch: int = 256):
        p = ServerParams()
        _lib.sfft_server_params_init(ctypes.byref(p))
        p.hbm_bytes, p.lanes, p.max_batch = int(hbm_bytes), int(lanes), int(max_batch)
        h = _lib.sfft_server_create(ctypes.byref(p))
        if not h:
            raise SfftError(_lib.sfft_last_error(), "sfft_server_create")
        self._h = ctypes.c_void_p(h)
        self._keep = []

    @staticmethod
    def clock_ns() -> int:
        return int(_lib.sfft_server_clock_ns())

    def submit(self, plans, xs, idxs, vals, counts, status, release_ns=None):
        """Queue len(plans) requests; counts / status are device int64 / int32
        tensors with one entry per request.  Returns the first ticket."""
        import numpy as np
        n = len(plans)
        rel = None
        if release_ns is not None:
            rel = np.ascontiguousarray(np.asarray(release_ns, dtype=np.int64))
            assert rel.shape == (n,)
        tk = np.zeros(n, dtype=np.int64)
        args = (_ptr_array([p.handle for p in plans]),
                _ptr_array([_sig_ptr(p, x) for p, x in zip(plans, xs)]),
                _ptr_array([_dev_ptr(t, "int64", p.K, "idx") for p, t in zip(plans, idxs)]),
                _ptr_array([_dev_ptr(t, "complex64", p.K, "val") for p, t in zip(plans, vals)]))
        _check(_lib.sfft_server_submit_many(
            self._h, n, *args, _dev_ptr(counts, "int64", n, "counts"),
            _dev_ptr(status, "int32", n, "status"),
            ctypes.c_void_p(rel.ctypes.data) if rel is not None else None,
            ctypes.c_void_p(tk.ctypes.data)), "sfft_server_submit_many")
        self._keep.append((plans, xs, idxs, vals, counts, status))
        return int(tk[0])

    def requests(self, first: int, n: int):
        """dict of numpy arrays: release_ns, launch_ns, done_ns, batch, lane, status."""
        import numpy as np
        arr = (Request * n)()
        _check(_lib.sfft_server_requests(self._h, first, n, arr), "sfft_server_requests")
        return {f: np.array([getattr(r, f) for r in arr]) for f, _ in Request._fields_ if f != "pad"}

    def wait(self, ticket: int):
        _check(_lib.sfft_server_wait(self._h, ticket), "sfft_server_wait")

    def drain(self):
        _check(_lib.sfft_server_drain(self._h), "sfft_server_drain")

    def close(self):
        if getattr(self, "_h", None):
            _lib.sfft_server_destroy(self._h)
            self._h = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def release_batches():
    _lib.sfft_release_batches()
