"""Thin ctypes binding of libldpc.so (C ABI in include/ldpc.h).

Argument marshalling only: every step of decoding runs in the library's HIP
kernels.  PyTorch provides device memory (tensors) and streams.  If the
library is not built, loading raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldpc.so")

LDPC_OK = 0
LDPC_EINVAL = -1
LDPC_ENOMEM = -2
LDPC_EDEVICE = -3
LDPC_EUNSUPPORTED = -4
LDPC_EWORKSPACE = -5
MAX_ROW_DEGREE = 16

EXPORTS = (
    "ldpc_code_create", "ldpc_code_destroy", "ldpc_code_info", "ldpc_decode_opts_init",
    "ldpc_workspace_bytes", "ldpc_decode_batch", "ldpc_syndrome", "ldpc_status_string",
    "ldpc_last_error", "ldpc_reconciliation_llr", "ldpc_reconciliation_message",
    "ldpc_engine_create", "ldpc_engine_destroy", "ldpc_engine_request_bytes", "ldpc_engine_submit",
    "ldpc_engine_step", "ldpc_engine_poll", "ldpc_decode_schedule", "ldpc_decode_batch_noalloc",
)
NOALLOC_SCRATCH_BYTES = 64 << 20

SCHEDULE_AUTO, SCHEDULE_LAUNCHES, SCHEDULE_RESIDENT, SCHEDULE_SPLIT = 0, 1, 2, 3
_SCHEDULES = {"auto": SCHEDULE_AUTO, "launches": SCHEDULE_LAUNCHES, "resident": SCHEDULE_RESIDENT,
              "split": SCHEDULE_SPLIT}


class LdpcError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({_status_text(status)}): {detail}")
        self.status = status


class CodeInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("m", ctypes.c_int32), ("Z", ctypes.c_int32),
        ("mb", ctypes.c_int32), ("nb", ctypes.c_int32), ("blocks", ctypes.c_int32),
        ("edges", ctypes.c_int64), ("state_edges", ctypes.c_int64),
        ("core_cols", ctypes.c_int32), ("deg1_cols", ctypes.c_int32),
        ("deg0_cols", ctypes.c_int32), ("max_row_degree", ctypes.c_int32),
        ("owned_edges", ctypes.c_int64), ("owner_groups", ctypes.c_int32),
    ]


class DecodeOpts(ctypes.Structure):
    _fields_ = [
        ("early_stop", ctypes.c_int32), ("check_from_iter", ctypes.c_int32),
        ("msg_fp16", ctypes.c_int32), ("checks_per_thread", ctypes.c_int32),
        ("llr_out", ctypes.c_void_p),
        ("timing_events", ctypes.POINTER(ctypes.c_void_p)), ("n_timing_events", ctypes.c_int32),
        ("schedule", ctypes.c_int32), ("streams", ctypes.c_int32), ("graphs", ctypes.c_int32),
    ]


class EngineConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
        ("msg_fp16", ctypes.c_int32), ("early_stop", ctypes.c_int32),
        ("checks_per_thread", ctypes.c_int32), ("stream", ctypes.c_void_p),
        ("max_step_edges", ctypes.c_int64),
    ]


_lib = None
_lock = threading.Lock()


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libldpc.so once; raise if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(
                f"{path} is missing: build the HIP decoder first (__graft_entry__.build())")
        lib = ctypes.CDLL(path)
        P, I32 = ctypes.c_void_p, ctypes.c_int32
        lib.ldpc_code_create.restype = ctypes.c_int
        lib.ldpc_code_create.argtypes = [I32, I32, P, I32, ctypes.POINTER(P)]
        lib.ldpc_code_destroy.restype = None
        lib.ldpc_code_destroy.argtypes = [P]
        lib.ldpc_code_info.restype = ctypes.c_int
        lib.ldpc_code_info.argtypes = [P, ctypes.POINTER(CodeInfo)]
        lib.ldpc_decode_opts_init.restype = None
        lib.ldpc_decode_opts_init.argtypes = [ctypes.POINTER(DecodeOpts)]
        lib.ldpc_workspace_bytes.restype = ctypes.c_size_t
        lib.ldpc_workspace_bytes.argtypes = [P, I32, I32, ctypes.POINTER(DecodeOpts)]
        lib.ldpc_decode_batch.restype = ctypes.c_int
        lib.ldpc_decode_batch.argtypes = [P, I32, P, P, I32, P, P, P,
                                          ctypes.POINTER(DecodeOpts), P, ctypes.c_size_t, P]
        lib.ldpc_decode_batch_noalloc.restype = ctypes.c_int
        lib.ldpc_decode_batch_noalloc.argtypes = [P, I32, P, P, I32, P, P, P,
                                                  ctypes.POINTER(DecodeOpts), P]
        lib.ldpc_decode_schedule.restype = ctypes.c_int
        lib.ldpc_decode_schedule.argtypes = [P, I32, ctypes.POINTER(DecodeOpts), ctypes.POINTER(I32)]
        lib.ldpc_syndrome.restype = ctypes.c_int
        lib.ldpc_syndrome.argtypes = [P, I32, P, P, P]
        lib.ldpc_status_string.restype = ctypes.c_char_p
        lib.ldpc_status_string.argtypes = [ctypes.c_int]
        lib.ldpc_last_error.restype = ctypes.c_char_p
        lib.ldpc_last_error.argtypes = []
        lib.ldpc_reconciliation_llr.restype = ctypes.c_int
        lib.ldpc_reconciliation_llr.argtypes = [I32, I32, I32, P, P, ctypes.c_float, P, P]
        lib.ldpc_reconciliation_message.restype = ctypes.c_int
        lib.ldpc_reconciliation_message.argtypes = [I32, I32, I32, P, P, P, P]
        lib.ldpc_engine_create.restype = ctypes.c_int
        lib.ldpc_engine_create.argtypes = [ctypes.POINTER(EngineConfig), ctypes.POINTER(P)]
        lib.ldpc_engine_destroy.restype = None
        lib.ldpc_engine_destroy.argtypes = [P]
        lib.ldpc_engine_request_bytes.restype = ctypes.c_size_t
        lib.ldpc_engine_request_bytes.argtypes = [P, I32, I32, I32]
        lib.ldpc_engine_submit.restype = ctypes.c_int
        lib.ldpc_engine_submit.argtypes = [P, P, I32, P, P, I32, P, P, P,
                                           ctypes.POINTER(ctypes.c_int64)]
        lib.ldpc_engine_step.restype = ctypes.c_int
        lib.ldpc_engine_step.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
        lib.ldpc_engine_poll.restype = ctypes.c_int
        lib.ldpc_engine_poll.argtypes = [P, ctypes.POINTER(ctypes.c_int64), I32, ctypes.POINTER(I32)]
        _lib = lib
        return lib


def _status_text(status: int) -> str:
    return load().ldpc_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != LDPC_OK:
        raise LdpcError(status, where, load().ldpc_last_error().decode())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_opts(early_stop=True, check_from_iter=0, msg_fp16=False, llr_out_ptr=None,
              timing_events=None, checks_per_thread=0, schedule="auto",
              streams=0, graphs=0) -> DecodeOpts:
    o = DecodeOpts()
    load().ldpc_decode_opts_init(ctypes.byref(o))
    o.checks_per_thread = int(checks_per_thread)
    o.streams = int(streams)
    o.graphs = int(graphs)
    o.schedule = _SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    o.early_stop = int(bool(early_stop))
    o.check_from_iter = int(check_from_iter)
    o.msg_fp16 = int(bool(msg_fp16))
    o.llr_out = llr_out_ptr
    if timing_events is not None:
        o.timing_events = timing_events
        o.n_timing_events = len(timing_events)
    return o


class Code:
    """A QC code on the current HIP device (ldpc_code_create)."""

    def __init__(self, base, Z: int):
        lib = load()
        b = np.ascontiguousarray(np.asarray(base), dtype=np.int32)
        if b.ndim != 2:
            raise ValueError("base must be a 2-D matrix")
        self.base = b
        h = ctypes.c_void_p()
        st = lib.ldpc_code_create(b.shape[0], b.shape[1], b.ctypes.data_as(ctypes.c_void_p),
                                  int(Z), ctypes.byref(h))
        _check(st, "ldpc_code_create")
        self._h = h
        info = CodeInfo()
        _check(lib.ldpc_code_info(h, ctypes.byref(info)), "ldpc_code_info")
        self.info = {k: getattr(info, k) for k, _ in CodeInfo._fields_}
        self.n, self.m, self.Z = info.n, info.m, info.Z

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ldpc_code_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, F: int, max_iters: int, msg_fp16=False, want_llr=False) -> int:
        o = make_opts(msg_fp16=msg_fp16, llr_out_ptr=1 if want_llr else None)
        return int(load().ldpc_workspace_bytes(self._h, int(F), int(max_iters), ctypes.byref(o)))

    def alloc_workspace(self, F, max_iters, msg_fp16=False, want_llr=False, device=None):
        import torch
        nbytes = self.workspace_bytes(F, max_iters, msg_fp16, want_llr)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
        off = (-ws.data_ptr()) % 256
        return ws[off:off + nbytes]

    def schedule(self, F=1, msg_fp16=False, want_llr=False, timing=False, schedule="auto") -> str:
        """The schedule ("launches", "resident" or "split") a decode of F frames with these
        options runs on."""
        o = make_opts(msg_fp16=msg_fp16, schedule=schedule)
        if want_llr:
            o.llr_out = ctypes.c_void_p(1)  # only tested for null
        if timing:
            o.timing_events = (ctypes.c_void_p * 1)()
            o.n_timing_events = 1
        out = ctypes.c_int32()
        _check(load().ldpc_decode_schedule(self._h, int(F), ctypes.byref(o), ctypes.byref(out)),
               "ldpc_decode_schedule")
        return {SCHEDULE_LAUNCHES: "launches", SCHEDULE_RESIDENT: "resident",
                SCHEDULE_SPLIT: "split"}[out.value]

    def decode(self, llr, syndrome, max_iters: int, early_stop=True, check_from_iter=0,
               msg_fp16=False, want_llr=False, workspace=None, out=None, stream=None,
               timing_events=None, checks_per_thread=0, schedule="auto", streams=0, graphs=0):
        """Decode frames llr [F][n] float32 / syndrome [F][m] uint8 (CUDA tensors).

        Returns (bits uint8 [F][n], iters int32 [F], converged uint8 [F], L or None),
        all CUDA tensors, valid once ``stream`` (default: current) is synchronised.
        ``streams``: 0 library choice, 1 one stream, 2 two halves of the frames on
        two streams (per-iteration launches; as ldpc_decode_opts.streams).
        ``graphs``: 0 replay repeated identical calls from a captured graph, 1
        never (as ldpc_decode_opts.graphs).
        """
        import torch
        if llr.dtype != torch.float32 or syndrome.dtype != torch.uint8:
            raise TypeError("llr must be float32 and syndrome uint8")
        if not (llr.is_cuda and syndrome.is_cuda):
            raise TypeError("llr and syndrome must be device tensors")
        if llr.dim() != 2 or llr.shape[1] != self.n or syndrome.shape != (llr.shape[0], self.m):
            raise ValueError("expected llr [F][n] and syndrome [F][m]")
        llr = llr.contiguous()
        syndrome = syndrome.contiguous()
        F = llr.shape[0]
        dev = llr.device
        if out is None:
            bits = torch.empty((F, self.n), dtype=torch.uint8, device=dev)
            iters = torch.empty(F, dtype=torch.int32, device=dev)
            conv = torch.empty(F, dtype=torch.uint8, device=dev)
            L = torch.empty((F, self.n), dtype=torch.float32, device=dev) if want_llr else None
        else:
            bits, iters, conv, L = out
        if workspace is None:
            workspace = self.alloc_workspace(F, max_iters, msg_fp16, want_llr, dev)
        opts = make_opts(early_stop, check_from_iter, msg_fp16,
                         L.data_ptr() if L is not None else None, timing_events,
                         checks_per_thread, schedule, streams, graphs)
        st = load().ldpc_decode_batch(
            self._h, F, llr.data_ptr(), syndrome.data_ptr(), int(max_iters),
            bits.data_ptr(), iters.data_ptr(), conv.data_ptr(), ctypes.byref(opts),
            workspace.data_ptr(), workspace.numel(), _stream_handle(stream))
        _check(st, "ldpc_decode_batch")
        return bits, iters, conv, L

    def decode_noalloc(self, llr, syndrome, max_iters: int, early_stop=True, check_from_iter=0,
                       msg_fp16=False, out=None, stream=None, checks_per_thread=0,
                       schedule="auto", streams=0):
        """ldpc_decode_batch_noalloc: as ``decode`` (no posteriors), with the decode
        state in the library's fixed per-device scratch region instead of a
        workspace.  ``out`` = (bits, iters, converged) preallocated tensors, else
        they are allocated here (the library call itself allocates nothing)."""
        import torch
        if llr.dtype != torch.float32 or syndrome.dtype != torch.uint8:
            raise TypeError("llr must be float32 and syndrome uint8")
        if not (llr.is_cuda and syndrome.is_cuda):
            raise TypeError("llr and syndrome must be device tensors")
        if llr.dim() != 2 or llr.shape[1] != self.n or syndrome.shape != (llr.shape[0], self.m):
            raise ValueError("expected llr [F][n] and syndrome [F][m]")
        llr = llr.contiguous()
        syndrome = syndrome.contiguous()
        F = llr.shape[0]
        if out is None:
            out = (torch.empty((F, self.n), dtype=torch.uint8, device=llr.device),
                   torch.empty(F, dtype=torch.int32, device=llr.device),
                   torch.empty(F, dtype=torch.uint8, device=llr.device))
        bits, iters, conv = out[:3]
        opts = make_opts(early_stop, check_from_iter, msg_fp16, None, None, checks_per_thread,
                         schedule, streams)
        st = load().ldpc_decode_batch_noalloc(
            self._h, F, llr.data_ptr(), syndrome.data_ptr(), int(max_iters), bits.data_ptr(),
            iters.data_ptr(), conv.data_ptr(), ctypes.byref(opts), _stream_handle(stream))
        _check(st, "ldpc_decode_batch_noalloc")
        return bits, iters, conv

    def syndrome(self, bits, stream=None):
        """H x mod 2 for uint8 words [F][n] (CUDA tensor) -> uint8 [F][m]."""
        import torch
        if bits.dtype != torch.uint8 or not bits.is_cuda or bits.dim() != 2 or bits.shape[1] != self.n:
            raise ValueError("expected a uint8 device tensor [F][n]")
        bits = bits.contiguous()
        syn = torch.empty((bits.shape[0], self.m), dtype=torch.uint8, device=bits.device)
        st = load().ldpc_syndrome(self._h, bits.shape[0], bits.data_ptr(), syn.data_ptr(),
                                  _stream_handle(stream))
        _check(st, "ldpc_syndrome")
        return syn


def padded_length(n: int, d: int) -> int:
    """Samples per frame of d-dimensional reconciliation: d * ceil(n / d)."""
    return d * ((n + d - 1) // d)


def reconciliation_llr(x, m, n: int, sigma2: float, d: int = 8, out=None, stream=None):
    """Channel LLRs [F][n] from Alice's samples x and Bob's message m ([F][n_d] float32)."""
    import torch
    if x.dtype != torch.float32 or m.dtype != torch.float32 or x.shape != m.shape or x.dim() != 2:
        raise ValueError("x and m must be float32 device tensors of one shape [F][n_d]")
    if x.shape[1] != padded_length(n, d):
        raise ValueError("frames must hold d * ceil(n / d) samples")
    x, m = x.contiguous(), m.contiguous()
    if out is None:
        out = torch.empty((x.shape[0], n), dtype=torch.float32, device=x.device)
    st = load().ldpc_reconciliation_llr(d, x.shape[0], n, x.data_ptr(), m.data_ptr(),
                                        float(sigma2), out.data_ptr(), _stream_handle(stream))
    _check(st, "ldpc_reconciliation_llr")
    return out


def reconciliation_message(bits, y, d: int = 8, out=None, stream=None):
    """Bob's message M = U Y per d-tuple from key bits [F][n] and samples y [F][n_d]."""
    import torch
    F, n = bits.shape
    if bits.dtype != torch.uint8 or y.dtype != torch.float32 or y.shape != (F, padded_length(n, d)):
        raise ValueError("bits uint8 [F][n] and y float32 [F][d*ceil(n/d)] expected")
    bits, y = bits.contiguous(), y.contiguous()
    if out is None:
        out = torch.empty_like(y)
    st = load().ldpc_reconciliation_message(d, F, n, bits.data_ptr(), y.data_ptr(), out.data_ptr(),
                                            _stream_handle(stream))
    _check(st, "ldpc_reconciliation_message")
    return out


class Engine:
    """Multi-request engine (ldpc_engine_*): continuous batching of decode requests.

    ``submit`` queues a request and returns its ticket; ``step`` runs one engine
    step (retire, admit, one iteration of every active request); ``poll``
    returns the tickets whose outputs are complete.  The engine keeps every
    submitted tensor alive until its ticket is reported.
    """

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, msg_fp16=False,
                 early_stop=True, stream=None, checks_per_thread=0, max_step_edges=0):
        import torch
        lib = load()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cfg = EngineConfig(int(hbm_budget_bytes), int(max_slots), int(bool(msg_fp16)),
                           int(bool(early_stop)), int(checks_per_thread), self.stream.cuda_stream,
                           int(max_step_edges))
        h = ctypes.c_void_p()
        _check(lib.ldpc_engine_create(ctypes.byref(cfg), ctypes.byref(h)), "ldpc_engine_create")
        self._h = h
        self.msg_fp16 = bool(msg_fp16)
        self._live = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ldpc_engine_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def request_bytes(self, code: "Code", F: int, max_iters: int) -> int:
        return int(load().ldpc_engine_request_bytes(code.handle, int(F), int(max_iters),
                                                    int(self.msg_fp16)))

    def submit(self, code: "Code", llr, syndrome, max_iters: int) -> int:
        import torch
        if llr.dtype != torch.float32 or syndrome.dtype != torch.uint8 or llr.dim() != 2:
            raise TypeError("llr float32 [F][n] and syndrome uint8 [F][m] device tensors expected")
        if llr.shape[1] != code.n or syndrome.shape != (llr.shape[0], code.m):
            raise ValueError("frame shapes do not match the code")
        llr, syndrome = llr.contiguous(), syndrome.contiguous()
        F = llr.shape[0]
        bits = torch.empty((F, code.n), dtype=torch.uint8, device=llr.device)
        iters = torch.empty(F, dtype=torch.int32, device=llr.device)
        conv = torch.empty(F, dtype=torch.uint8, device=llr.device)
        t = ctypes.c_int64()
        st = load().ldpc_engine_submit(self._h, code.handle, F, llr.data_ptr(), syndrome.data_ptr(),
                                       int(max_iters), bits.data_ptr(), iters.data_ptr(),
                                       conv.data_ptr(), ctypes.byref(t))
        _check(st, "ldpc_engine_submit")
        self._live[t.value] = (code, llr, syndrome, bits, iters, conv)
        return t.value

    def step(self):
        a, q = ctypes.c_int32(), ctypes.c_int32()
        _check(load().ldpc_engine_step(self._h, ctypes.byref(a), ctypes.byref(q)),
               "ldpc_engine_step")
        return a.value, q.value

    def poll(self, capacity: int = 64):
        buf = (ctypes.c_int64 * capacity)()
        n = ctypes.c_int32()
        _check(load().ldpc_engine_poll(self._h, buf, capacity, ctypes.byref(n)), "ldpc_engine_poll")
        return [buf[i] for i in range(n.value)]

    def result(self, ticket: int):
        """(bits, iters, converged) tensors of a reported ticket; releases them."""
        code, llr, syn, bits, iters, conv = self._live.pop(ticket)
        return bits, iters, conv

    def pending(self) -> int:
        return len(self._live)

    def drain(self, tickets, max_steps: int = 1_000_000):
        """Step until every ticket in ``tickets`` is reported; returns {ticket: outputs}."""
        import torch
        want = set(tickets)
        out = {}
        for _ in range(max_steps):
            for t in self.poll():
                if t in want:
                    out[t] = self.result(t)
            if len(out) == len(want):
                return out
            active, queued = self.step()
            if active == 0 and queued == 0:
                torch.cuda.current_stream().synchronize()
        raise RuntimeError("engine did not finish within max_steps")
