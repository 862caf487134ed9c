#!/usr/bin/env python3
"""Raw decoded throughput of the HIP sum-product decoder on one MI355X.

Workload: the rate-0.02 QC multi-edge template (6 core columns, 144 degree-1
columns, 3 type-1 and 144 type-2 base rows) lifted by Z = 6667
(n = 1,000,050), 8 synthetic BIAWGN frames at SNR -15.4 dB, at most 100
iterations with early stop.  A step is one ldpc_decode_batch call over the
8 frames (the whole hot path: check pass, variable pass, syndrome check and
early stop, every iteration).  Raw Mbit/s = frames * n / decode time, the
paper's K_raw (Sec. IV-A) over a batch of frames.

Prints one JSON line.  Extra keys: FP16-message throughput, per-call latency
p50/p99, frame error rate, the roofline of the dominant kernel (HIP events
around every check and variable pass), and the FP64 oracle timed on the host.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "raw decoded Mbit/s, n=1e6 R=0.02, 100 iters; p99 latency; FP16 vs FP32 msgs"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
PAPER_KRAW_MBPS = 1.72       # GTX 1080, q=21 QC code, Table II (context only)

# HBM traffic of the steady check pass per frame, at 8 frames (cache-resident)
# and 32 frames (HBM-resident), from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, divided by the dispatch's frames: a decode of
# F frames without per-pass events runs two dispatches of F/2 frames per pass,
# one per stream), each scaled by what the counter reads for a 1 GiB device
# copy (FETCH_SIZE reads 0.5 GiB, WRITE_SIZE 1 GiB: factors 2.0 and 1.0).  The
# figures hold only for the kernel sources they were taken on; any change to
# them makes the fingerprint differ and they are reported as null.
KERNEL_SOURCES = ("internal.h", "passes.h", "decoder.hip")
MEASURED_SOURCES = "75f4283625162032"
MEASURED_TRAFFIC = {
    "check_pass_F8": {"fetch_kib": 6544.0, "write_kib": 8409.0, "fetch_scale": 2.0,
                      "write_scale": 1.0},
    "check_pass_F32": {"fetch_kib": 6492.2, "write_kib": 8412.2, "fetch_scale": 2.0,
                       "write_scale": 1.0},
}
# Instruction counts of the steady check pass per frame (rocprofv3 --pmc
# SQ_INSTS_VALU, SQ_INSTS_VALU_TRANS_F32, SQ_INSTS_SALU per dispatch, divided by
# the dispatch's frames): wave64 instructions, transcendentals included in VALU.
MEASURED_ISSUE = {
    "check_pass_fp32": {"valu": 915688, "trans": 100008, "salu": 479873},
    "check_pass_fp16": {"valu": 996973, "trans": 100008, "salu": 488585},
}
# VALU issue ceiling: 256 CUs x 4 SIMDs, each issuing one wave64 VALU
# instruction every 4 cycles, at 2.4 GHz = 614.4 G wave-instructions/s.  A
# transcendental (exp2, log2, rcp) takes two issue slots on CDNA4 (half the
# FP32 rate).  The scalar unit issues one instruction per CU and cycle, the
# same 614.4 G/s.
VALU_ISSUE_PEAK = 256 * 2.4e9
TRANS_SLOTS = 2.0


def kernel_fingerprint() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1702_07740_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, F: int):
    """HBM bytes of `kernel` for F frames from the counters, or None if stale."""
    m = MEASURED_TRAFFIC.get(f"{kernel}_F{F}")
    if m is None or MEASURED_SOURCES != kernel_fingerprint():
        return None
    return F * 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])


def issue_ceiling(kernel: str, F: int, avg_ms: float):
    """The instruction-issue ceiling of `kernel` for F frames: issue slots
    (VALU, transcendentals counted twice) over the VALU issue peak, and the
    scalar instructions over the same rate.  None if the counters are stale."""
    m = MEASURED_ISSUE.get(kernel)
    if m is None or MEASURED_SOURCES != kernel_fingerprint():
        return None
    slots = F * (m["valu"] + (TRANS_SLOTS - 1.0) * m["trans"])
    valu_ms = slots / VALU_ISSUE_PEAK * 1e3
    salu_ms = F * m["salu"] / VALU_ISSUE_PEAK * 1e3
    ms = max(valu_ms, salu_ms)
    return {"valu_wave_instr": F * m["valu"], "trans_wave_instr": F * m["trans"],
            "salu_wave_instr": F * m["salu"], "issue_slots": slots,
            "peak_G_per_s": VALU_ISSUE_PEAK / 1e9, "valu_min_ms": valu_ms, "salu_min_ms": salu_ms,
            "min_ms": ms, "frac": ms / avg_ms}


class HipEvents:
    """hipEvent_t handles through the HIP runtime torch already loaded."""

    def __init__(self, count: int):
        self.lib = ctypes.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.arr = (ctypes.c_void_p * count)()
        for i in range(count):
            ev = ctypes.c_void_p()
            rc = self.lib.hipEventCreate(ctypes.byref(ev))
            if rc != 0:
                raise RuntimeError(f"hipEventCreate failed: {rc}")
            self.arr[i] = ev
        self.count = count

    def elapsed_ms(self, i: int, j: int) -> float:
        ms = ctypes.c_float()
        rc = self.lib.hipEventElapsedTime(ctypes.byref(ms), self.arr[i], self.arr[j])
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return ms.value

    def close(self):
        for i in range(self.count):
            self.lib.hipEventDestroy(self.arr[i])


def run_decodes(torch, code, dQ, ds, T, steps, warmup, fp16, F, schedule="auto"):
    ws = code.alloc_workspace(F, T, msg_fp16=fp16)
    out = (torch.empty((F, code.n), dtype=torch.uint8, device="cuda"),
           torch.empty(F, dtype=torch.int32, device="cuda"),
           torch.empty(F, dtype=torch.uint8, device="cuda"), None)
    for _ in range(warmup):
        code.decode(dQ, ds, T, msg_fp16=fp16, workspace=ws, out=out, schedule=schedule)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(steps):
        code.decode(dQ, ds, T, msg_fp16=fp16, workspace=ws, out=out, schedule=schedule)
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
    total_ms = evs[0].elapsed_time(evs[steps])
    iters = out[1].cpu().numpy()
    conv = out[2].cpu().numpy()
    return {"total_ms": total_ms, "per_ms": per, "wall_s": wall, "iters": iters, "conv": conv,
            "bits": out[0].cpu().numpy()}


def frame_errors(bits, x):
    """Frames whose decoded word differs from the key anywhere (a frame that
    converged to another word of the same syndrome coset counts as an error)."""
    k = int(np.sum(np.any(bits != x, axis=1)))
    F = int(x.shape[0])
    return {"frame_errors": k, "frames": F, "fer": k / F, "ci95": wilson(k, F)}


def kernel_roofline(torch, code, dQ, ds, T, steps, F, info, fp16=False):
    """Average durations of the check and variable passes from HIP events
    that the launches record at the start and end of every kernel (on the
    decode stream), over `steps` decodes."""
    ev = HipEvents(4 * T)
    ws = code.alloc_workspace(F, T, msg_fp16=fp16)
    out = (torch.empty((F, code.n), dtype=torch.uint8, device="cuda"),
           torch.empty(F, dtype=torch.int32, device="cuda"),
           torch.empty(F, dtype=torch.uint8, device="cuda"), None)
    cn_ms = np.zeros(T)
    vn_ms = np.zeros(T)
    for _ in range(steps):
        code.decode(dQ, ds, T, msg_fp16=fp16, workspace=ws, out=out, timing_events=ev.arr,
                    schedule="launches")
        torch.cuda.synchronize()
        for t in range(1, T + 1):
            cn_ms[t - 1] += ev.elapsed_ms(4 * (t - 1), 4 * (t - 1) + 1)
            vn_ms[t - 1] += ev.elapsed_ms(4 * (t - 1) + 2, 4 * (t - 1) + 3)
    ev.close()
    iters = out[1].cpu().numpy()
    cn_ms /= steps
    vn_ms /= steps
    w = 2 if fp16 else 4
    Z = info["Z"]
    E_state = info["state_edges"]
    E_d1 = info["deg1_cols"] * Z
    NC = info["core_cols"]
    m = info["m"]
    P = info["owner_groups"] * Z      # owner-group partial sums
    E_other = E_state - info["owned_edges"]
    # algorithmic bytes per frame (w-byte messages): the check pass reads and
    # writes each stored message once (writes only at t = 1), reads the
    # degree-1 inputs and the packed syndrome bits, and writes the partial
    # sums; the variable pass reads the messages outside owner blocks, the
    # partial sums and the core channel LLRs, and writes the core totals.
    cn_bytes = np.array([(w if t == 1 else 2 * w) * E_state + 4 * E_d1 + m / 8 + 4 * P
                         for t in range(1, T + 1)])
    vn_bytes = np.full(T, w * E_other + 4 * P + 8 * NC * Z, dtype=np.float64)
    active_cn = np.array([np.sum(iters >= t - 1) for t in range(1, T + 1)])
    active_vn = np.array([np.sum(iters >= t) for t in range(1, T + 1)])
    cn_gbs = float(np.sum(cn_bytes * active_cn) / (np.sum(cn_ms) * 1e-3) / 1e9)
    vn_gbs = float(np.sum(vn_bytes * active_vn) / (np.sum(vn_ms) * 1e-3) / 1e9)
    tot = np.sum(cn_ms) + np.sum(vn_ms)
    return {
        "check_pass": {"avg_ms": float(np.mean(cn_ms)), "achieved_GBs": cn_gbs,
                       "bytes_per_frame": float(cn_bytes[-1]),
                       "bytes_per_launch": float(cn_bytes[-1]) * F,
                       "share": float(np.sum(cn_ms) / tot)},
        "variable_pass": {"avg_ms": float(np.mean(vn_ms)), "achieved_GBs": vn_gbs,
                          "bytes_per_frame": float(vn_bytes[-1]),
                          "bytes_per_launch": float(vn_bytes[-1]) * F,
                          "share": float(np.sum(vn_ms) / tot)},
    }


def roofline_entry(kr, F, where, fp16=False):
    """The roofline object of the dominant kernel (the check pass) from the
    per-kernel events of kernel_roofline: its HBM roofline, and beside it the
    instruction-issue ceiling from the counters; `bound` names the ceiling
    that allows the longer minimum time (HBM bytes at 8 TB/s, or issue slots
    at the VALU issue peak)."""
    dom = max(kr, key=lambda k: kr[k]["share"])
    k = kr[dom]
    hbm_ms = k["bytes_per_launch"] / (HBM_PEAK_GBS * 1e9) * 1e3
    iss = issue_ceiling(f"{dom}_{'fp16' if fp16 else 'fp32'}", F, k["avg_ms"])
    ent = {"bound": "hbm", "kernel": dom, "achieved": round(k["achieved_GBs"], 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(k["achieved_GBs"] / HBM_PEAK_GBS, 4),
           "traffic": None if fp16 else measured_traffic(dom, F),
           "algorithmic_bytes": k["bytes_per_launch"], "avg_ms": k["avg_ms"],
           "hbm_min_ms": hbm_ms, "issue": iss, "working_set": where, "kernels": kr}
    if iss is not None and iss["min_ms"] > hbm_ms:
        # instruction issue allows less than HBM does: report against it
        ent.update({"bound": "alu", "achieved": round(iss["issue_slots"] / (k["avg_ms"] * 1e-3) / 1e9, 1),
                    "peak": VALU_ISSUE_PEAK / 1e9, "unit": "G wave64 issue slots/s",
                    "frac": round(iss["frac"], 4), "hbm_frac": round(k["achieved_GBs"] / HBM_PEAK_GBS, 4)})
    return ent


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads() -> int:
    """Host threads this process may run on (its CPU affinity), else the CPU count."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def end_to_end(torch, code, x, Q, T, steps, F):
    """Decode time including the transfers (Table IV's latency includes them):
    LLRs and syndromes from pinned host memory to the device, the decode, and
    bits, iteration counts and flags back to pinned host memory, one stream."""
    hQ = torch.from_numpy(Q).pin_memory()
    hx = torch.from_numpy(x).pin_memory()
    dQ = torch.empty_like(hQ, device="cuda")
    dx = hx.cuda()
    hs = code.syndrome(dx).cpu().pin_memory()
    ds = torch.empty_like(hs, device="cuda")
    ws = code.alloc_workspace(F, T)
    out = (torch.empty((F, code.n), dtype=torch.uint8, device="cuda"),
           torch.empty(F, dtype=torch.int32, device="cuda"),
           torch.empty(F, dtype=torch.uint8, device="cuda"), None)
    hb = torch.empty((F, code.n), dtype=torch.uint8).pin_memory()
    hi = torch.empty(F, dtype=torch.int32).pin_memory()
    hc = torch.empty(F, dtype=torch.uint8).pin_memory()

    def once():
        dQ.copy_(hQ, non_blocking=True)
        ds.copy_(hs, non_blocking=True)
        code.decode(dQ, ds, T, workspace=ws, out=out)
        hb.copy_(out[0], non_blocking=True)
        hi.copy_(out[1], non_blocking=True)
        hc.copy_(out[2], non_blocking=True)

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        once()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"ms_per_step": ms, "mbit_s": F * code.n / (ms * 1e-3) / 1e6,
            "transfer_bytes": int(hQ.numel() * 4 + hs.numel() + hb.numel() + 5 * F)}


def cpu_baseline(base, Z, n, snr, seed, threads, iters_sample):
    """The FP64 oracle as it stands, on `threads` frames of the same workload x
    `iters_sample` iterations (early stop off), scaled to the metric's 100
    iterations.  Input generation and the syndrome are outside the timing."""
    import oracle
    from paper_1702_07740_amd import synth
    ocode = oracle.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(n, threads, snr, seed=seed)
    s = ocode.syndrome(x)
    t0 = time.perf_counter()
    ocode.decode(Q, s, iters_sample, early_stop=False, threads=threads)
    wall = time.perf_counter() - t0
    mbps = threads * n * iters_sample / (wall * 100.0) / 1e6
    return {"value": mbps, "unit": "Mbit/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": f"{threads} frames x {iters_sample} iterations of n={n}, early stop off, "
                      f"one frame per thread, {wall:.1f} s wall on {threads} threads "
                      f"({wall * threads:.0f} s of CPU work), scaled to 100 iterations"}


def wilson(k, n, z=1.959964):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (float(max(0.0, c - h)), float(min(1.0, c + h)))


def workload_mixed(torch, ldpc, args):
    """64 frames over the 9 codes R in {0.02, 0.05, 0.1} x Z in {2048, 4096, 6667}
    (frame f decodes with code f mod 9), each at its BP threshold + 0.3 dB, max 100
    iterations: one engine run (all codes batched per iteration) against the plain
    FP32 path (one ldpc_decode_batch per code, in sequence)."""
    from paper_1702_07740_amd import serve, synth
    thr = serve.template_thresholds()
    combos = [(R, Z) for R in (0.02, 0.05, 0.1) for Z in (2048, 4096, 6667)]
    counts = [len(range(i, 64, 9)) for i in range(9)]
    groups = []
    for (R, Z), F in zip(combos, counts):
        code = ldpc.Code(synth.template_for_rate(R, Z, seed=1), Z)
        snr = thr[R] + 0.3
        x, Q = synth.biawgn_frames(code.n, F, snr, seed=3000 + Z + int(R * 1000))
        dx = torch.from_numpy(x).cuda()
        groups.append((R, Z, F, snr, code, torch.from_numpy(Q).cuda(), code.syndrome(dx), x))
    torch.cuda.synchronize()
    T = args.max_iters
    total_bits = sum(g[2] * g[4].n for g in groups)

    def plain(fp16=False):
        outs = []
        for R, Z, F, snr, code, Q, s, x in groups:
            outs.append(code.decode(Q, s, T, msg_fp16=fp16))
        return outs

    from paper_1702_07740_amd import autotune
    reqs = [(code, Q, s) for R, Z, F, snr, code, Q, s, x in groups]
    cpt32, tune32 = autotune.tune_engine(reqs, msg_fp16=False, use_cache=False)
    cpt16, tune16 = autotune.tune_engine(reqs, msg_fp16=True, use_cache=False)

    def engine(fp16=False):
        eng = ldpc.Engine(64 << 30, max_slots=16, msg_fp16=fp16,
                          checks_per_thread=cpt16 if fp16 else cpt32)
        tickets = [eng.submit(code, Q, s, T) for R, Z, F, snr, code, Q, s, x in groups]
        res = eng.drain(tickets)
        eng.close()
        return [res[t] for t in tickets]

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out

    reps = max(1, min(args.steps, 5))
    t_plain, o_plain = timed(lambda: plain(False), reps)
    t_eng, o_eng = timed(lambda: engine(False), reps)
    t_eng16, o_eng16 = timed(lambda: engine(True), reps)
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) for a, b in zip(o_plain, o_eng))
    fer = {}
    for name, outs in (("plain_fp32", o_plain), ("engine_fp32", o_eng), ("engine_fp16", o_eng16)):
        errs = sum(int(np.sum(np.any(o[0].cpu().numpy() != g[7], axis=1))) for o, g in zip(outs, groups))
        fer[name] = {"frame_errors": errs, "frames": 64, "fer": errs / 64, "ci95": wilson(errs, 64)}
    return {
        "metric": "raw decoded Mbit/s, 64 mixed frames (R 0.02/0.05/0.1 x Z 2048/4096/6667)",
        "value": round(total_bits / t_eng / 1e6, 3), "unit": "Mbit/s", "n_gpus": 1,
        "steps": reps, "warmup": 1, "ms_per_step": round(t_eng * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "mixed codes in one engine batch, threshold + 0.3 dB, max "
                               f"{T} iterations", "codes": [[R, Z, F, round(snr, 3)] for R, Z, F, snr, *_ in groups]},
        "plain_fp32_mbit_s": round(total_bits / t_plain / 1e6, 3),
        "engine_fp16_mbit_s": round(total_bits / t_eng16 / 1e6, 3),
        "engine_equals_plain_bitwise": bool(same), "fer": fer,
        "autotune": {"fp32": {"checks_per_thread": cpt32, "ms": tune32},
                     "fp16": {"checks_per_thread": cpt16, "ms": tune16}},
    }


def workload_small(torch, ldpc, args):
    """The small template (Z = 64, n = 9,600), 16 frames at -15.4 dB, 100
    iterations.  Launch-bound on the per-iteration schedule, so the default
    schedule here is the frame-resident one (one launch per decode, state in
    LDS).  Also timed: the per-iteration launches, eager and replayed from a
    captured HIP graph, FP16 messages, and the resident schedule at more
    frames."""
    from paper_1702_07740_amd import synth
    Z, F, T = 64, 16, args.max_iters
    base = synth.template_base(144, Z, seed=1)
    code = ldpc.Code(base, Z)
    x, Q = synth.biawgn_frames(code.n, F, args.snr, seed=2026)
    dQ = torch.from_numpy(Q).cuda()
    ds = code.syndrome(torch.from_numpy(x).cuda())
    ws = code.alloc_workspace(F, T)
    out = (torch.empty((F, code.n), dtype=torch.uint8, device="cuda"),
           torch.empty(F, dtype=torch.int32, device="cuda"),
           torch.empty(F, dtype=torch.uint8, device="cuda"), None)

    def timed(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    bits = F * code.n
    auto = code.schedule(F=F)
    auto_ms = timed(lambda: code.decode(dQ, ds, T, workspace=ws, out=out), args.steps)
    avg_iters = float(out[1].float().mean().item())
    res_ms = timed(lambda: code.decode(dQ, ds, T, workspace=ws, out=out, schedule="resident"),
                   args.steps)
    ws16 = code.alloc_workspace(F, T, msg_fp16=True)
    res16_ms = timed(lambda: code.decode(dQ, ds, T, workspace=ws16, out=out, msg_fp16=True,
                                         schedule="resident"), args.steps)
    split_ms = timed(lambda: code.decode(dQ, ds, T, workspace=ws, out=out, schedule="split"),
                     args.steps)
    split16_ms = timed(lambda: code.decode(dQ, ds, T, workspace=ws16, out=out, msg_fp16=True,
                                           schedule="split"), args.steps)
    eager_ms = timed(lambda: code.decode(dQ, ds, T, workspace=ws, out=out, schedule="launches"),
                     args.steps)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        code.decode(dQ, ds, T, workspace=ws, out=out, schedule="launches")
        with torch.cuda.graph(graph, stream=side):
            code.decode(dQ, ds, T, workspace=ws, out=out, schedule="launches")
    torch.cuda.current_stream().wait_stream(side)
    graph_ms = timed(graph.replay, args.steps)
    del graph
    sweep = {}
    for Fs in (32, 64, 256, 1024):
        xs, Qs = synth.biawgn_frames(code.n, Fs, args.snr, seed=2027)
        dQs = torch.from_numpy(Qs).cuda()
        dss = code.syndrome(torch.from_numpy(xs).cuda())
        wss = code.alloc_workspace(Fs, T)
        for sch in ("resident", "launches", "split"):
            if sch == "split" and Fs > 256:
                continue
            ms = timed(lambda: code.decode(dQs, dss, T, workspace=wss, schedule=sch),
                       max(3, args.steps // 4))
            sweep.setdefault(str(Fs), {})[sch] = {"ms": ms, "mbit_s": round(Fs * code.n / ms / 1e3, 3)}
        sweep[str(Fs)]["auto"] = code.schedule(F=Fs)
        del dQs, dss, wss
    return {
        "metric": "raw decoded Mbit/s, small template n=9,600, 16 frames, 100 iters",
        "value": round(bits / auto_ms / 1e3, 3), "unit": "Mbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 3, "ms_per_step": auto_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"R=0.02 template, Z=64 (n=9,600), 16 BIAWGN frames at {args.snr} dB, "
                               f"max {T} iterations, early stop; automatic schedule ({auto})"},
        "resident": {"ms_per_step": res_ms, "mbit_s": round(bits / res_ms / 1e3, 3)},
        "resident_fp16": {"ms_per_step": res16_ms, "mbit_s": round(bits / res16_ms / 1e3, 3)},
        "split": {"ms_per_step": split_ms, "mbit_s": round(bits / split_ms / 1e3, 3)},
        "split_fp16": {"ms_per_step": split16_ms, "mbit_s": round(bits / split16_ms / 1e3, 3)},
        "launches_eager": {"ms_per_step": eager_ms, "mbit_s": round(bits / eager_ms / 1e3, 3)},
        "launches_graph": {"ms_per_step": graph_ms, "mbit_s": round(bits / graph_ms / 1e3, 3)},
        "resident_frames": sweep,
        "avg_iters": avg_iters,
    }


def workload_frontend(torch, ldpc, args):
    """8-D reconciliation: Bob's message and Alice's LLRs on the device (octonion
    products), then FP16-message decoding of the n = 1,000,050 code; 8 frames."""
    from paper_1702_07740_amd import synth
    Z, F, T, d = 6667, args.frames, args.max_iters, 8
    code = ldpc.Code(synth.template_base(144, Z, seed=1), Z)
    sigma2 = synth.sigma2_from_snr_db(args.snr)
    c, X, Zn = synth.reconciliation_inputs(code.n, d, F, args.snr, seed=44)
    dc = torch.from_numpy(c).cuda()
    dX = torch.from_numpy(X.astype(np.float32)).cuda()
    dY = torch.from_numpy((X + Zn).astype(np.float32)).cuda()
    s = code.syndrome(dc)
    M = ldpc.reconciliation_message(dc, dY, d=d)
    ws = code.alloc_workspace(F, T, msg_fp16=True)
    L = torch.empty((F, code.n), dtype=torch.float32, device="cuda")

    def step():
        ldpc.reconciliation_llr(dX, M, code.n, sigma2, d=d, out=L)
        return code.decode(L, s, T, msg_fp16=True, workspace=ws)

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        out = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    errs = int(np.sum(np.any(out[0].cpu().numpy() != c, axis=1)))
    return {
        "metric": "raw decoded Mbit/s, 8-D reconciliation front-end + FP16 decode, n=1,000,050",
        "value": round(F * code.n / (ms * 1e-3) / 1e6, 3), "unit": "Mbit/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"d=8 reconciliation, {F} frames at {args.snr} dB, FP16 messages, "
                               f"max {T} iterations", "n": code.n, "Z": Z, "frames": F},
        "fer": errs / F, "avg_iters": float(out[1].float().mean().item()),
    }


def workload_serving(torch, ldpc, args):
    """Poisson requests of mixed codes through the engine (continuous batching,
    admission by HBM budget) against the plain FP32 one-at-a-time path on the same
    trace."""
    import copy
    from paper_1702_07740_amd import serve
    pools = serve.make_pools(ldpc, torch)
    # capacity probe: a saturating burst through the engine
    burst = serve.poisson_trace(len(pools), 1e6, 64 / 1e6 + 1e-9, seed=1)[:64]
    for r in burst:
        r.arrival = 0.0
    st, _ = serve.run_engine(ldpc, torch, pools, copy.deepcopy(burst), 200 << 30)
    cap = st["requests"] / st["wall_s"]
    lam = args.serve_load * cap
    trace = serve.poisson_trace(len(pools), lam, args.duration, seed=11)
    print(f"[bench] serving: capacity {cap:.1f} req/s, {len(trace)} requests", file=sys.stderr,
          flush=True)
    caps = {}
    for c in [int(float(x)) for x in args.serve_caps.split(",")]:
        st_c, _ = serve.run_engine(ldpc, torch, pools, copy.deepcopy(trace), 200 << 30,
                                   max_step_edges=c)
        caps[str(c)] = st_c
        print(f"[bench] serving: engine, 200 GB budget, step cap {c} edges: {st_c}",
              file=sys.stderr, flush=True)
    eng = caps[str(int(float(args.serve_caps.split(",")[0])))]
    small, _ = serve.run_engine(ldpc, torch, pools, copy.deepcopy(trace), 256 << 20)
    print(f"[bench] serving: engine, 256 MB budget {small}", file=sys.stderr, flush=True)
    one = None
    if not args.no_one_at_a_time:
        one, _ = serve.run_one_at_a_time(ldpc, torch, pools, copy.deepcopy(trace))
        print(f"[bench] serving: one at a time {one}", file=sys.stderr, flush=True)
    return {
        "metric": "serving: raw decoded Mbit/s and p50/p99 latency, Poisson mixed-code requests",
        "value": round(eng["mbit_s"], 3), "unit": "Mbit/s", "n_gpus": 1, "steps": len(trace),
        "warmup": 0, "ms_per_step": eng["mean_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals at {lam:.1f} req/s ({args.serve_load:.0%} of "
                               f"measured capacity {cap:.1f} req/s) for {args.duration} s; R in "
                               "{0.02,0.05,0.1}, Z in {1024,2048,4096,6667}, 1-4 frames, "
                               "threshold + 0.3 dB, max 100 iterations",
                   "budget_bytes": 200 << 30,
                   "max_step_edges": int(float(args.serve_caps.split(",")[0]))},
        "latency_ms": {"p50": eng["p50_ms"], "p99": eng["p99_ms"]},
        "engine": eng, "engine_by_step_cap": caps, "engine_256MB_budget": small,
        "one_at_a_time_fp32": one,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--snr", type=float, default=-15.4)
    ap.add_argument("--max-iters", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-hbm-point", action="store_true")
    ap.add_argument("--no-e2e", action="store_true")
    ap.add_argument("--workload", default="decode",
                    choices=["decode", "mixed", "frontend", "serving", "small"],
                    help="decode: the n=1,000,050 headline; mixed: 64 frames of 9 codes in one "
                         "engine batch; frontend: 8-D reconciliation + FP16 decode; serving: "
                         "Poisson requests through the engine")
    ap.add_argument("--duration", type=float, default=60.0, help="serving run length (s)")
    ap.add_argument("--serve-caps", default="24e6,0",
                    help="serving: engine step caps in edge visits (first = reported; 0 = none)")
    ap.add_argument("--no-one-at-a-time", action="store_true",
                    help="serving: skip the one-request-at-a-time baseline")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="serving arrival rate as a fraction of measured capacity")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 3 times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(frames are independent, so more GPUs would shard frames with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1702_07740_amd import ldpc, synth

    if args.workload != "decode":
        fn = {"mixed": workload_mixed, "frontend": workload_frontend, "small": workload_small,
              "serving": workload_serving}[args.workload]
        print(json.dumps(fn(torch, ldpc, args)), flush=True)
        return

    Z, F, T = 6667, args.frames, args.max_iters
    base = synth.template_base(144, Z, seed=1)
    code = ldpc.Code(base, Z)
    n, m = code.n, code.m
    schedule = code.schedule(F=F)
    print(f"[bench] code n={n} m={m} frames={F} snr={args.snr} T={T} schedule={schedule}",
          file=sys.stderr, flush=True)
    x, Q = synth.biawgn_frames(n, F, args.snr, seed=2026)
    dQ = torch.from_numpy(Q).cuda()
    ds = code.syndrome(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()

    r32 = run_decodes(torch, code, dQ, ds, T, args.steps, args.warmup, False, F)
    print(f"[bench] fp32 done {r32['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    value = F * n * args.steps / (r32["total_ms"] * 1e-3) / 1e6
    fe32 = frame_errors(r32["bits"], x)
    info = code.info
    res = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mbit/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r32["total_ms"] / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "QC multi-edge R=0.02 template, Z=6667 (n=1,000,050), "
                               f"{F} BIAWGN frames at {args.snr} dB, max {T} iterations, early stop",
                   "n": n, "Z": Z, "rate": 0.02, "frames": F, "snr_db": args.snr,
                   "max_iters": T, "early_stop": True, "messages": "fp32", "schedule": schedule},
        "latency_ms": {"p50": float(np.percentile(r32["per_ms"], 50)),
                       "p99": float(np.percentile(r32["per_ms"], 99))},
        "fer": fe32["fer"], "fer_detail": fe32,
        "avg_iters": float(np.mean(r32["iters"])),
        # information throughput K' = K_raw R (1 - FER) (Sec. IV-A)
        "info_mbit_s": round(value * 0.02 * (1.0 - fe32["fer"]), 6),
        "context": {"paper_gtx1080_kraw_mbit_s": PAPER_KRAW_MBPS},
    }
    # whole-path roofline: algorithmic bytes per frame-iteration (every stored
    # message read and written once, all channel LLRs, the syndrome bits)
    b_min = 8 * info["state_edges"] + 4 * n + m / 8
    iters_done = float(np.sum(r32["iters"]))
    res["path_roofline"] = {
        "bytes_per_bit_iteration": b_min / n,
        "achieved_GBs": b_min * iters_done * args.steps / (r32["total_ms"] * 1e-3) / 1e9,
    }
    res["path_roofline"]["frac"] = res["path_roofline"]["achieved_GBs"] / HBM_PEAK_GBS

    if not args.no_fp16:
        r16 = run_decodes(torch, code, dQ, ds, T, args.steps, args.warmup, True, F)
        v16 = F * n * args.steps / (r16["total_ms"] * 1e-3) / 1e6
        fe16 = frame_errors(r16["bits"], x)
        res["fp16"] = {"value": round(v16, 3), "ms_per_step": r16["total_ms"] / args.steps,
                       "p99_ms": float(np.percentile(r16["per_ms"], 99)),
                       "fer": fe16["fer"], "fer_detail": fe16,
                       "avg_iters": float(np.mean(r16["iters"])),
                       "schedule": code.schedule(F=F, msg_fp16=True)}
        print(f"[bench] fp16 done {r16['total_ms']:.1f} ms", file=sys.stderr, flush=True)

    if not args.no_roofline:
        steps_r = max(2, min(args.steps, 5))
        kr = kernel_roofline(torch, code, dQ, ds, T, steps_r, F, info)
        res["roofline"] = roofline_entry(kr, F, "cache-resident: about 131 MB of decode state and "
                                                "inputs for 8 frames, inside the 256 MB Infinity "
                                                "Cache")
        if "fp16" in res:
            kr16 = kernel_roofline(torch, code, dQ, ds, T, steps_r, F, info, fp16=True)
            res["fp16"]["roofline"] = roofline_entry(kr16, F, "cache-resident", fp16=True)
        print("[bench] roofline done", file=sys.stderr, flush=True)

    if not args.no_hbm_point:
        # an HBM-resident point: 32 frames (about 525 MB of decode state and
        # inputs, twice the Infinity Cache), same decode
        F2 = 32
        x2, Q2 = synth.biawgn_frames(n, F2, args.snr, seed=2027)
        dQ2 = torch.from_numpy(Q2).cuda()
        ds2 = code.syndrome(torch.from_numpy(x2).cuda())
        steps2 = max(2, min(args.steps, 5))
        r2 = run_decodes(torch, code, dQ2, ds2, T, steps2, 1, False, F2)
        kr2 = kernel_roofline(torch, code, dQ2, ds2, T, 2, F2, info)
        v2 = F2 * n * steps2 / (r2["total_ms"] * 1e-3) / 1e6
        res["hbm_point"] = {
            "frames": F2, "value": round(v2, 3), "ms_per_step": r2["total_ms"] / steps2,
            "path_roofline_frac": b_min * float(np.sum(r2["iters"])) * steps2
            / (r2["total_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "roofline": roofline_entry(kr2, F2, "HBM-resident: about 525 MB, twice the "
                                                "Infinity Cache")}
        del dQ2, ds2
        print("[bench] hbm point done", file=sys.stderr, flush=True)

    if not args.no_e2e:
        e2e = end_to_end(torch, code, x, Q, T, max(2, min(args.steps, 5)), F)
        res["end_to_end"] = {"mbit_s": round(e2e["mbit_s"], 3), "ms_per_step": e2e["ms_per_step"],
                             "includes": "LLR and syndrome upload from pinned host memory, "
                                         "decode, bits/iterations/flags download"}
        print("[bench] end to end done", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        threads = cpu_threads()
        res["cpu_baseline"] = cpu_baseline(base, Z, n, args.snr, 2026, threads, 8)
        res["cpu_baseline"]["gpu_over_oracle"] = round(value / res["cpu_baseline"]["value"], 1)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)

    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
