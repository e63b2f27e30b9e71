"""Python binding of libsfft (ctypes).  Argument marshalling only.

The names mirror the C ABI of include/sfft.h: sfft_plan_create,
sfft_plan_destroy, sfft_recover, sfft_recover_static, sfft_static_scratch_slots,
sfft_export_bucket_features, sfft_sample_lines, sfft_dft,
sfft_plan_max_prime, sfft_plan_num_sets, sfft_autotune, sfft_last_error,
sfft_version (and the classifier kernels sfft_mlp_forward / _grad / _train).
PyTorch provides device memory and the current stream; every step of the
recovery runs in the HIP kernels of libsfft.so.  Loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfft.so")

SFFT_OK, SFFT_NOT_CONVERGED, SFFT_RESIDUAL_NONZERO = 0, 1, 2
SFFT_RESIDUAL_SPECTRUM, SFFT_RESIDUAL_SAMPLES = 0, 1
SFFT_EINVAL, SFFT_ERANGE, SFFT_ENOMEM, SFFT_EDEVICE = -1, -2, -3, -4
SFFT_PRIME_PAPER, SFFT_PRIME_SMOOTH = 0, 1
SFFT_FP64, SFFT_FP32 = 0, 1
SFFT_CLS_PLAIN, SFFT_CLS_MLP = 0, 1
SFFT_TRACE_W = 8
SFFT_FFT_RADIX24_HEAD, SFFT_FFT_RADIX8_HEAD = 1, 2
SFFT_MLP_PARAMS = 4866
SFFT_MLP_FEATURES = 8

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ERANGE", -3: "ENOMEM",
                -4: "EDEVICE"}


class sfft_params(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("d1", ctypes.c_int32), ("N", ctypes.c_int64),
        ("k_max", ctypes.c_int32), ("c", ctypes.c_double), ("prime_rule", ctypes.c_int32),
        ("p_min", ctypes.c_int32), ("ladder_K", ctypes.c_int32), ("tau", ctypes.c_double),
        ("tau_noise", ctypes.c_double), ("eta", ctypes.c_double),
        ("max_rounds", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("robust", ctypes.c_int32), ("classifier", ctypes.c_int32),
        ("mlp_weights", ctypes.c_void_p), ("mlp_threshold", ctypes.c_double),
        ("feature_scale", ctypes.c_double),
        ("verify", ctypes.c_int32),
        ("verify_eta", ctypes.c_double),
        ("residual", ctypes.c_int32),
        ("sched_nt", ctypes.c_int32 * 4),
        ("sched_fft", ctypes.c_int32),
        ("sched_dft_batch", ctypes.c_int32),
        ("blocks", ctypes.POINTER(ctypes.c_int32)),
        ("n_blocks", ctypes.c_int32),
        ("order", ctypes.POINTER(ctypes.c_int32)),
        ("tilt", ctypes.c_int32),
        ("tilt_a", ctypes.c_int32), ("tilt_b", ctypes.c_int32), ("tilt_c", ctypes.c_int32),
        ("split_groups", ctypes.c_int32),
    ]


class sfft_tune_entry(ctypes.Structure):
    _fields_ = [
        ("c", ctypes.c_double), ("sched_nt", ctypes.c_int32 * 4), ("sched_fft", ctypes.c_int32),
        ("sched_dft_batch", ctypes.c_int32), ("status", ctypes.c_int32),
        ("exact", ctypes.c_int32), ("ms", ctypes.c_double),
    ]


class sfft_signal_batch(ctypes.Structure):
    _fields_ = [
        ("B", ctypes.c_int32), ("mode_off", ctypes.c_void_p), ("freqs", ctypes.c_void_p),
        ("coeffs", ctypes.c_void_p), ("k", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
        ("seed", ctypes.c_uint64),
    ]


class sfft_outputs(ctypes.Structure):
    _fields_ = [
        ("freqs", ctypes.c_void_p), ("coeffs", ctypes.c_void_p), ("k_found", ctypes.c_void_p),
        ("status", ctypes.c_void_p), ("rounds", ctypes.c_void_p), ("samples", ctypes.c_void_p),
        ("trace", ctypes.c_void_p), ("feat", ctypes.c_void_p), ("label", ctypes.c_void_p),
        ("feat_meta", ctypes.c_void_p), ("feat_count", ctypes.c_void_p),
        ("feat_cap", ctypes.c_int64),
        ("phase", ctypes.c_void_p),
    ]


class SfftError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libsfft.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.sfft_plan_create.argtypes = [ctypes.POINTER(sfft_params), i32, ctypes.POINTER(vp)]
        L.sfft_plan_create.restype = i32
        L.sfft_plan_destroy.argtypes = [vp]
        L.sfft_plan_destroy.restype = i32
        L.sfft_recover.argtypes = [vp, ctypes.POINTER(sfft_signal_batch),
                                   ctypes.POINTER(sfft_outputs), vp]
        L.sfft_recover.restype = i32
        L.sfft_recover_static.argtypes = [vp, ctypes.POINTER(sfft_signal_batch),
                                          ctypes.POINTER(sfft_outputs), vp]
        L.sfft_recover_static.restype = i32
        L.sfft_static_scratch_slots.argtypes = [vp]
        L.sfft_static_scratch_slots.restype = i32
        L.sfft_export_bucket_features.argtypes = [vp, ctypes.POINTER(sfft_signal_batch), vp, vp,
                                                  vp, i64, vp, vp]
        L.sfft_export_bucket_features.restype = i32
        L.sfft_sample_lines.argtypes = [vp, ctypes.POINTER(sfft_signal_batch), i32, i32, i32,
                                        vp, vp, vp, vp, vp]
        L.sfft_sample_lines.restype = i32
        L.sfft_dft.argtypes = [vp, vp, i32, i32, vp]
        L.sfft_dft.restype = i32
        L.sfft_plan_max_prime.argtypes = [vp]
        L.sfft_plan_max_prime.restype = i32
        L.sfft_plan_num_sets.argtypes = [vp]
        L.sfft_plan_num_sets.restype = i32
        L.sfft_last_error.argtypes = []
        L.sfft_last_error.restype = ctypes.c_char_p
        L.sfft_version.argtypes = []
        L.sfft_version.restype = i32
        L.sfft_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.sfft_mlp_forward.restype = i32
        L.sfft_mlp_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.sfft_mlp_grad.restype = i32
        L.sfft_mlp_train.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_double,
                                     ctypes.c_uint64, vp, vp]
        L.sfft_mlp_train.restype = i32
        L.sfft_autotune.argtypes = [ctypes.POINTER(sfft_params), ctypes.POINTER(sfft_signal_batch),
                                    ctypes.POINTER(ctypes.c_double), i32, i32, i32,
                                    ctypes.POINTER(sfft_tune_entry), i32,
                                    ctypes.POINTER(i32), vp]
        L.sfft_autotune.restype = i32
        L.sfft_session_create.argtypes = [vp, i32, vp, vp, ctypes.POINTER(vp)]
        L.sfft_session_create.restype = i32
        L.sfft_session_destroy.argtypes = [vp]
        L.sfft_session_destroy.restype = i32
        L.sfft_session_request.argtypes = [vp, vp, vp, vp]
        L.sfft_session_request.restype = i32
        L.sfft_session_points.argtypes = [vp, vp, vp]
        L.sfft_session_points.restype = i32
        L.sfft_session_feed.argtypes = [vp, vp, vp]
        L.sfft_session_feed.restype = i32
        L.sfft_session_finish.argtypes = [vp, ctypes.POINTER(sfft_outputs), vp]
        L.sfft_session_finish.restype = i32
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Function names declared in include/sfft.h."""
    hdr = os.path.join(os.path.dirname(_HERE), "include", "sfft.h")
    text = open(hdr).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\*]+\s+)+\**(sfft_\w+)\s*\(", text, re.M)))


def sfft_last_error() -> str:
    return lib().sfft_last_error().decode()


def sfft_version() -> int:
    return int(lib().sfft_version())


def _check(st: int, where: str):
    if st != SFFT_OK:
        raise SfftError(st, where, sfft_last_error())


@dataclass
class Params:
    """Mirror of sfft_params with the paper's defaults (c = 5, one eps shift per axis)."""
    d: int
    N: int
    k_max: int
    d1: int = 1
    c: float = 5.0
    prime_rule: int = SFFT_PRIME_PAPER
    p_min: int = 0
    ladder_K: int = 1
    tau: float = 0.0
    tau_noise: float = 0.0
    eta: float = 1e-3
    max_rounds: int = 64
    precision: int = SFFT_FP32
    robust: int = 0
    classifier: int = SFFT_CLS_PLAIN
    mlp_weights: object = None      # device tensor of SFFT_MLP_PARAMS bfloat16 values
    mlp_threshold: float = 0.5
    feature_scale: float = 0.0
    verify: int = 0
    verify_eta: float = 0.0
    residual: int = 0               # SFFT_RESIDUAL_SPECTRUM
    sched_nt: tuple = (0, 0, 0, 0)  # kernel schedules; 0 = built-in choice
    sched_fft: int = 0
    sched_dft_batch: int = 0
    blocks: tuple | None = None     # general partition: block sizes (sum d); None = d1
    order: tuple | None = None      # coordinate order (a permutation of 0..d-1)
    tilt: int = 0                   # 1: 2D tilting (d = 2); tilt_abc (0, 0, 0) = plan's triple
    tilt_abc: tuple = (0, 0, 0)
    split_groups: int = 0           # work-groups per signal: 0 automatic, 1 one, 2..16

    def to_c(self) -> sfft_params:
        c = sfft_params(self.d, self.d1, self.N, self.k_max, self.c, self.prime_rule,
                        self.p_min, self.ladder_K, self.tau, self.tau_noise, self.eta,
                        self.max_rounds, self.precision, self.robust, self.classifier,
                        _ptr(self.mlp_weights), self.mlp_threshold, self.feature_scale,
                        self.verify, self.verify_eta, self.residual,
                        (ctypes.c_int32 * 4)(*[int(v) for v in self.sched_nt]),
                        self.sched_fft, self.sched_dft_batch)
        # the arrays live as long as the returned structure (sfft_plan_create copies them)
        if self.blocks is not None:
            c._blocks = (ctypes.c_int32 * len(self.blocks))(*[int(v) for v in self.blocks])
            c.blocks = ctypes.cast(c._blocks, ctypes.POINTER(ctypes.c_int32))
            c.n_blocks = len(self.blocks)
        if self.order is not None:
            c._order = (ctypes.c_int32 * len(self.order))(*[int(v) for v in self.order])
            c.order = ctypes.cast(c._order, ctypes.POINTER(ctypes.c_int32))
        c.tilt = int(self.tilt)
        c.tilt_a, c.tilt_b, c.tilt_c = (int(v) for v in self.tilt_abc)
        c.split_groups = int(self.split_groups)
        return c


class Plan:
    def __init__(self, handle: int, params: Params, max_batch: int):
        self.handle = ctypes.c_void_p(handle)
        self.params = params
        self.max_batch = max_batch

    @property
    def max_prime(self) -> int:
        return sfft_plan_max_prime(self)

    @property
    def num_sets(self) -> int:
        return sfft_plan_num_sets(self)

    def close(self):
        if self.handle:
            sfft_plan_destroy(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sfft_plan_create(params: Params, max_batch: int = 1) -> Plan:
    h = ctypes.c_void_p()
    p = params.to_c()
    _check(lib().sfft_plan_create(ctypes.byref(p), int(max_batch), ctypes.byref(h)),
           "sfft_plan_create")
    return Plan(h.value, params, max_batch)


def sfft_plan_destroy(plan: Plan):
    if plan.handle:
        _check(lib().sfft_plan_destroy(plan.handle), "sfft_plan_destroy")
        plan.handle = ctypes.c_void_p()


def sfft_plan_max_prime(plan: Plan) -> int:
    return int(lib().sfft_plan_max_prime(plan.handle))


def sfft_plan_num_sets(plan: Plan) -> int:
    return int(lib().sfft_plan_num_sets(plan.handle))


# ------------------------------------------------------------- device data --

def _torch():
    import torch
    return torch


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> int | None:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else stream


class DeviceBatch:
    """Device copies of a planted batch (workloads.PlantedBatch or equivalent arrays)."""

    def __init__(self, freqs, coeffs, mode_off, k, sigma, seed: int, device="cuda"):
        torch = _torch()
        c = np.asarray(coeffs, dtype=np.complex128)
        self.freqs = torch.as_tensor(np.ascontiguousarray(freqs, dtype=np.int64), device=device)
        self.coeffs = torch.as_tensor(np.ascontiguousarray(np.stack([c.real, c.imag], -1)),
                                      device=device)
        self.mode_off = torch.as_tensor(np.asarray(mode_off, dtype=np.int64), device=device)
        self.k = torch.as_tensor(np.asarray(k, dtype=np.int32), device=device)
        self.sigma = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
        self.seed = int(seed)
        self.B = int(self.k.shape[0])

    @classmethod
    def from_planted(cls, pb, device="cuda"):
        return cls(pb.freqs, pb.coeffs, pb.mode_off, pb.k, pb.sigma, pb.seed, device)

    def to_c(self) -> sfft_signal_batch:
        return sfft_signal_batch(self.B, _ptr(self.mode_off), _ptr(self.freqs),
                                 _ptr(self.coeffs), _ptr(self.k), _ptr(self.sigma),
                                 self.seed & 0xFFFFFFFFFFFFFFFF)


def alloc_outputs(plan: Plan, B: int, trace: bool = True, device="cuda",
                  export_cap: int = 0, phase: bool = False) -> dict:
    torch = _torch()
    P = plan.params
    if export_cap > 0:
        exp = dict(
            feat=torch.zeros((export_cap, SFFT_MLP_FEATURES), dtype=torch.float32, device=device),
            label=torch.zeros(export_cap, dtype=torch.uint8, device=device),
            feat_meta=torch.zeros((export_cap, 4), dtype=torch.int32, device=device),
            feat_count=torch.zeros(1, dtype=torch.int64, device=device))
    else:
        exp = dict(feat=None, label=None, feat_meta=None, feat_count=None)
    out = dict(**exp,
        freqs=torch.zeros((B, P.k_max, P.d), dtype=torch.int64, device=device),
        coeffs=torch.zeros((B, P.k_max, 2), dtype=torch.float64, device=device),
        k_found=torch.zeros(B, dtype=torch.int32, device=device),
        status=torch.zeros(B, dtype=torch.int32, device=device),
        rounds=torch.zeros(B, dtype=torch.int32, device=device),
        samples=torch.zeros(B, dtype=torch.int64, device=device),
        trace=(torch.zeros((B, P.max_rounds, SFFT_TRACE_W), dtype=torch.int32, device=device)
               if trace else None),
        phase=(torch.zeros((B, P.max_rounds, SFFT_TRACE_W), dtype=torch.int64, device=device)
               if phase else None),
    )
    return out


def sfft_recover(plan: Plan, batch: DeviceBatch, out: dict | None = None, stream=None) -> dict:
    if out is None:
        out = alloc_outputs(plan, batch.B)
    cap = int(out["feat"].shape[0]) if out.get("feat") is not None else 0
    o = sfft_outputs(_ptr(out["freqs"]), _ptr(out["coeffs"]), _ptr(out["k_found"]),
                     _ptr(out["status"]), _ptr(out.get("rounds")), _ptr(out.get("samples")),
                     _ptr(out.get("trace")), _ptr(out.get("feat")), _ptr(out.get("label")),
                     _ptr(out.get("feat_meta")), _ptr(out.get("feat_count")), cap,
                     _ptr(out.get("phase")))
    b = batch.to_c()
    _check(lib().sfft_recover(plan.handle, ctypes.byref(b), ctypes.byref(o), _stream(stream)),
           "sfft_recover")
    return out


def sfft_recover_static(plan: Plan, batch: DeviceBatch, out: dict | None = None,
                        stream=None) -> dict:
    """sfft_recover with the library's fixed device scratch instead of the plan's
    workspace (no device allocation by the library; overlapping calls on one device
    race)."""
    if out is None:
        out = alloc_outputs(plan, batch.B)
    o = sfft_outputs(_ptr(out["freqs"]), _ptr(out["coeffs"]), _ptr(out["k_found"]),
                     _ptr(out["status"]), _ptr(out.get("rounds")), _ptr(out.get("samples")),
                     _ptr(out.get("trace")), None, None, None, None, 0, _ptr(out.get("phase")))
    b = batch.to_c()
    _check(lib().sfft_recover_static(plan.handle, ctypes.byref(b), ctypes.byref(o),
                                     _stream(stream)), "sfft_recover_static")
    return out


def sfft_static_scratch_slots(plan: Plan) -> int:
    return int(lib().sfft_static_scratch_slots(plan.handle))


def sfft_export_bucket_features(plan: Plan, batch: DeviceBatch, cap: int, out: dict | None = None,
                                stream=None) -> dict:
    """Bucket features of every candidate of every round (the classifier's training
    data): dict of feat [cap, 8] float32, label [cap] uint8, feat_meta [cap, 4] int32 and
    feat_count [1] int64 device tensors; records past cap are counted, not written."""
    torch = _torch()
    if out is None:
        dev = batch.k.device
        out = dict(feat=torch.zeros((cap, SFFT_MLP_FEATURES), dtype=torch.float32, device=dev),
                   label=torch.zeros(cap, dtype=torch.uint8, device=dev),
                   feat_meta=torch.zeros((cap, 4), dtype=torch.int32, device=dev),
                   feat_count=torch.zeros(1, dtype=torch.int64, device=dev))
    b = batch.to_c()
    _check(lib().sfft_export_bucket_features(plan.handle, ctypes.byref(b), _ptr(out["feat"]),
                                             _ptr(out["label"]), _ptr(out["feat_meta"]),
                                             int(out["feat"].shape[0]), _ptr(out["feat_count"]),
                                             _stream(stream)), "sfft_export_bucket_features")
    return out


class Session:
    """Caller-supplied samples (the sfft_session_* calls of the C ABI): the caller
    evaluates its signal on the lines each round asks for.

        s = Session(plan, k)              # k: sparsity per signal
        while True:
            p, m = s.request()            # host arrays; p[b] == 0: signal b is done
            if not p.any(): break
            t = s.points()                # [B, S+1, max_prime, d] float64 on the device
            s.feed(f(t))                  # complex [B, S+1, max_prime], the plan's precision
        out = s.finish()                  # as sfft_recover

    m[b] >= 1 is the unwrapped axis of an ordinary round; m[b] = -q marks a
    verification round, whose one line (set 0 of t and of the samples) is
    t_h = (h/p) U v with v_n = q^(n-1) mod p.
    """

    def __init__(self, plan: Plan, k, stream=None):
        torch = _torch()
        self.plan = plan
        self.k = torch.as_tensor(k, dtype=torch.int32, device="cuda").reshape(-1).contiguous()
        self.B = int(self.k.shape[0])
        self.stream = stream
        self._req = torch.zeros((2, self.B), dtype=torch.int32, device="cuda")
        h = ctypes.c_void_p()
        self._after_current()
        _check(lib().sfft_session_create(plan.handle, self.B, _ptr(self.k), _stream(stream),
                                         ctypes.byref(h)), "sfft_session_create")
        self.handle = h
        self._before_current(self.k, self._req)

    def _side(self) -> bool:
        """True when the session runs on a stream other than torch's current one."""
        return (self.stream is not None and hasattr(self.stream, "wait_stream")
                and self.stream != _torch().cuda.current_stream())

    def _after_current(self):
        """Order the session's stream after torch's current one (tensors made there)."""
        if self._side():
            self.stream.wait_stream(_torch().cuda.current_stream())

    def _before_current(self, *tensors):
        """After a launch on a side stream: order torch's current stream after it (so
        that what the launch wrote is seen there) and tell the caching allocator that
        the side stream uses these tensors (made on the current stream)."""
        if self._side():
            _torch().cuda.current_stream().wait_stream(self.stream)
            for t in tensors:
                if t is not None:
                    t.record_stream(self.stream)

    def request(self):
        self._after_current()
        _check(lib().sfft_session_request(self.handle, _ptr(self._req[0]), _ptr(self._req[1]),
                                          _stream(self.stream)), "sfft_session_request")
        (self.stream if self.stream is not None else _torch().cuda.current_stream()).synchronize()
        r = self._req.cpu().numpy()
        return r[0].copy(), r[1].copy()

    def points(self, t=None):
        torch = _torch()
        P = self.plan.params
        if t is None:
            t = torch.zeros((self.B, self.plan.num_sets, self.plan.max_prime, P.d),
                            dtype=torch.float64, device="cuda")
        self._after_current()
        _check(lib().sfft_session_points(self.handle, _ptr(t), _stream(self.stream)),
               "sfft_session_points")
        self._before_current(t)
        return t

    def feed(self, samples):
        torch = _torch()
        dt = torch.complex64 if self.plan.params.precision == SFFT_FP32 else torch.complex128
        want = (self.B, self.plan.num_sets, self.plan.max_prime)
        if tuple(samples.shape) != want or samples.dtype != dt or not samples.is_contiguous():
            raise ValueError(f"samples must be a contiguous {dt} tensor of shape {want}")
        self._after_current()
        _check(lib().sfft_session_feed(self.handle, _ptr(samples), _stream(self.stream)),
               "sfft_session_feed")
        self._before_current(samples)

    def finish(self, out: dict | None = None) -> dict:
        if out is None:
            out = alloc_outputs(self.plan, self.B)
        o = sfft_outputs(_ptr(out["freqs"]), _ptr(out["coeffs"]), _ptr(out["k_found"]),
                         _ptr(out["status"]), _ptr(out.get("rounds")), _ptr(out.get("samples")),
                         _ptr(out.get("trace")), None, None, None, None, 0, None)
        self._after_current()
        _check(lib().sfft_session_finish(self.handle, ctypes.byref(o), _stream(self.stream)),
               "sfft_session_finish")
        self._before_current(*[v for v in out.values() if hasattr(v, "record_stream")])
        return out

    def close(self):
        if self.handle:
            lib().sfft_session_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sfft_sample_lines(plan: Plan, batch: DeviceBatch, round_i: int, p: int, m: int,
                      res_off=None, res_y=None, res_coeffs=None, V=None, stream=None):
    """Samples of one round: complex tensor [B, S+1, p] of the plan's precision."""
    torch = _torch()
    S1 = plan.num_sets
    if V is None:
        dt = torch.complex64 if plan.params.precision == SFFT_FP32 else torch.complex128
        V = torch.zeros((batch.B, S1, p), dtype=dt, device=batch.k.device)
    b = batch.to_c()
    _check(lib().sfft_sample_lines(plan.handle, ctypes.byref(b), int(round_i), int(p), int(m),
                                   _ptr(res_off), _ptr(res_y), _ptr(res_coeffs), _ptr(V),
                                   _stream(stream)), "sfft_sample_lines")
    return V


def sfft_dft(plan: Plan, data, stream=None):
    """In-place DFT of each row of a contiguous complex tensor [count, p]."""
    count, p = int(data.shape[0]), int(data.shape[1])
    _check(lib().sfft_dft(plan.handle, _ptr(data), count, p, _stream(stream)), "sfft_dft")
    return data


def sfft_autotune(params: Params, batch: DeviceBatch, c_values=(), warmup: int = 1,
                  steps: int = 3, stream=None):
    """Measure candidate c values and kernel schedules on `batch` (sfft_autotune of
    the C ABI).  Returns the winning Params (a copy of `params` with c and the
    sched_* fields replaced) and the list of measured candidates as dicts."""
    import dataclasses
    p = params.to_c()
    cs = (ctypes.c_double * max(1, len(c_values)))(*[float(c) for c in c_values])
    cap = 256
    log = (sfft_tune_entry * cap)()
    n = ctypes.c_int32(0)
    b = batch.to_c()
    _check(lib().sfft_autotune(ctypes.byref(p), ctypes.byref(b), cs, len(c_values), int(warmup),
                               int(steps), log, cap, ctypes.byref(n), _stream(stream)),
           "sfft_autotune")
    best = dataclasses.replace(params, c=float(p.c), sched_nt=tuple(int(v) for v in p.sched_nt),
                               sched_fft=int(p.sched_fft), sched_dft_batch=int(p.sched_dft_batch))
    entries = [dict(c=e.c, sched_nt=tuple(int(v) for v in e.sched_nt), sched_fft=e.sched_fft,
                    sched_dft_batch=e.sched_dft_batch, status=e.status, exact=e.exact, ms=e.ms)
               for e in log[:min(n.value, cap)]]
    return best, entries


def sfft_mlp_forward(w, x, prob=None, stream=None):
    """Probability of one mode for each feature row (x: float32 [n, 8] device)."""
    torch = _torch()
    n = int(x.shape[0])
    if prob is None:
        prob = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(lib().sfft_mlp_forward(_ptr(w), _ptr(x), n, _ptr(prob), _stream(stream)),
           "sfft_mlp_forward")
    return prob


def sfft_mlp_grad(w, x, y, stream=None):
    """(loss tensor [1], gradient tensor [SFFT_MLP_PARAMS]) of the mean cross-entropy."""
    torch = _torch()
    grad = torch.empty(SFFT_MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().sfft_mlp_grad(_ptr(w), _ptr(x), _ptr(y), int(x.shape[0]), _ptr(grad),
                               _ptr(loss), _stream(stream)), "sfft_mlp_grad")
    return loss, grad


def sfft_mlp_train(w, x, y, epochs: int, batch: int, lr: float, seed: int = 1, stream=None):
    """Train in place (w: bfloat16 [SFFT_MLP_PARAMS] device); returns per-epoch losses."""
    torch = _torch()
    hist = torch.zeros(epochs, dtype=torch.float32, device=x.device)
    _check(lib().sfft_mlp_train(_ptr(w), _ptr(x), _ptr(y), int(x.shape[0]), int(epochs),
                                int(batch), float(lr), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                _ptr(hist), _stream(stream)), "sfft_mlp_train")
    return hist


def outputs_to_host(out: dict) -> dict:
    """numpy copies; coefficients as complex128."""
    h = {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}
    h["coeffs"] = h["coeffs"][..., 0] + 1j * h["coeffs"][..., 1]
    return h
