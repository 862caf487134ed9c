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


def run_decodes(torch, code, dQ, ds, T, steps, warmup, fp16, F):
    ws = code.alloc_workspace(F, T, msg_fp16=fp16)
    out = (torch.empty((F, code.n), dtype=torch.uint8, device="cuda"),
           torch.empty(F, dtype=torch.int32, device="cuda"),
           torch.empty(F, dtype=torch.uint8, device="cuda"), None)
    for _ in range(warmup):
        code.decode(dQ, ds, T, msg_fp16=fp16, workspace=ws, out=out)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(steps):
        code.decode(dQ, ds, T, msg_fp16=fp16, workspace=ws, out=out)
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
    total_ms = evs[0].elapsed_time(evs[steps])
    iters = out[1].cpu().numpy()
    conv = out[2].cpu().numpy()
    return {"total_ms": total_ms, "per_ms": per, "wall_s": wall, "iters": iters, "conv": conv}


def kernel_roofline(torch, code, dQ, ds, T, steps, F, info):
    """Average durations of the check and variable passes from HIP events
    recorded on the decode stream around every launch, over `steps` decodes."""
    ev = HipEvents(2 * T + 1)
    ws = code.alloc_workspace(F, T)
    out = (torch.empty((F, code.n), dtype=torch.uint8, device="cuda"),
           torch.empty(F, dtype=torch.int32, device="cuda"),
           torch.empty(F, dtype=torch.uint8, device="cuda"), None)
    cn_ms = np.zeros(T)
    vn_ms = np.zeros(T)
    for _ in range(steps):
        code.decode(dQ, ds, T, workspace=ws, out=out, timing_events=ev.arr)
        torch.cuda.synchronize()
        for t in range(1, T + 1):
            cn_ms[t - 1] += ev.elapsed_ms(2 * (t - 1), 2 * (t - 1) + 1)
            vn_ms[t - 1] += ev.elapsed_ms(2 * (t - 1) + 1, 2 * t)
    ev.close()
    iters = out[1].cpu().numpy()
    cn_ms /= steps
    vn_ms /= steps
    Z = info["Z"]
    E_state = info["state_edges"]
    E_d1 = info["deg1_cols"] * Z
    NC = info["core_cols"]
    m = info["m"]
    # algorithmic bytes per frame (FP32 messages): each stored message read once
    # and written once per check pass (written only at t = 1), the degree-1
    # channel LLRs and the packed syndrome bits; the variable pass reads every
    # message once, the core channel LLRs, and writes the core totals.
    cn_bytes = np.array([(4 if t == 1 else 8) * E_state + 4 * E_d1 + m / 8 for t in range(1, T + 1)])
    vn_bytes = np.full(T, 4 * E_state + 8 * NC * Z, dtype=np.float64)
    active_cn = np.array([np.sum(iters >= t - 1) for t in range(1, T + 1)])
    active_vn = np.array([np.sum(iters >= t) for t in range(1, T + 1)])
    cn_gbs = float(np.sum(cn_bytes * active_cn) / (np.sum(cn_ms) * 1e-3) / 1e9)
    vn_gbs = float(np.sum(vn_bytes * active_vn) / (np.sum(vn_ms) * 1e-3) / 1e9)
    return {
        "check_pass": {"avg_ms": float(np.mean(cn_ms)), "achieved_GBs": cn_gbs,
                       "bytes_per_frame": float(cn_bytes[-1]), "share": float(np.sum(cn_ms) / (np.sum(cn_ms) + np.sum(vn_ms)))},
        "variable_pass": {"avg_ms": float(np.mean(vn_ms)), "achieved_GBs": vn_gbs,
                          "bytes_per_frame": float(vn_bytes[-1]), "share": float(np.sum(vn_ms) / (np.sum(cn_ms) + np.sum(vn_ms)))},
    }


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
            "sample": f"{threads} frames x {iters_sample} iterations of n={n}, early stop off, "
                      f"{wall:.1f} s wall on {threads} threads, scaled to 100 iterations"}


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

    Z, F, T = 6667, args.frames, args.max_iters
    base = synth.template_base(144, Z, seed=1)
    code = ldpc.Code(base, Z)
    n, m = code.n, code.m
    print(f"[bench] code n={n} m={m} frames={F} snr={args.snr} T={T}", file=sys.stderr, flush=True)
    x, Q = synth.biawgn_frames(n, F, args.snr, seed=2026)
    dQ = torch.from_numpy(Q).cuda()
    ds = code.syndrome(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()

    r32 = run_decodes(torch, code, dQ, ds, T, args.steps, args.warmup, False, F)
    print(f"[bench] fp32 done {r32['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    value = F * n * args.steps / (r32["total_ms"] * 1e-3) / 1e6
    res = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mbit/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r32["total_ms"] / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "QC multi-edge R=0.02 template, Z=6667 (n=1,000,050), "
                               f"{F} BIAWGN frames at {args.snr} dB, max {T} iterations, early stop",
                   "n": n, "Z": Z, "rate": 0.02, "frames": F, "snr_db": args.snr,
                   "max_iters": T, "early_stop": True, "messages": "fp32"},
        "latency_ms": {"p50": float(np.percentile(r32["per_ms"], 50)),
                       "p99": float(np.percentile(r32["per_ms"], 99))},
        "fer": float(1.0 - np.mean(r32["conv"])),
        "avg_iters": float(np.mean(r32["iters"])),
        "context": {"paper_gtx1080_kraw_mbit_s": PAPER_KRAW_MBPS},
    }
    info = code.info
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
        res["fp16"] = {"value": round(v16, 3), "ms_per_step": r16["total_ms"] / args.steps,
                       "p99_ms": float(np.percentile(r16["per_ms"], 99)),
                       "fer": float(1.0 - np.mean(r16["conv"])),
                       "avg_iters": float(np.mean(r16["iters"]))}
        print(f"[bench] fp16 done {r16['total_ms']:.1f} ms", file=sys.stderr, flush=True)

    if not args.no_roofline:
        kr = kernel_roofline(torch, code, dQ, ds, T, max(2, min(args.steps, 5)), F, info)
        dom = max(kr, key=lambda k: kr[k]["share"])
        res["roofline"] = {"bound": "hbm", "kernel": dom,
                           "achieved": round(kr[dom]["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(kr[dom]["achieved_GBs"] / HBM_PEAK_GBS, 4),
                           "traffic": None, "avg_ms": kr[dom]["avg_ms"], "kernels": kr}
        print("[bench] roofline done", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        threads = max(1, min(16, os.cpu_count() or 1))
        res["cpu_baseline"] = cpu_baseline(base, Z, n, args.snr, 2026, threads, 4)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)

    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
