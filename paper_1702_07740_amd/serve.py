"""Request loop over the multi-request engine: Poisson arrivals of decode
requests of mixed codes, admission by HBM budget, continuous batching, and
latency / throughput accounting; plus the one-request-at-a-time baseline on
the same arrival trace.

Workload (the serving configuration): every request draws a rate from
{0.02, 0.05, 0.1}, a lifting size from {1024, 2048, 4096, 6667} and 1-4
frames; frames are BIAWGN at the code's BP threshold + 0.3 dB; decoding runs
at most 100 iterations with early stop.  Frame inputs are generated on the
host once per (rate, Z) pool and kept on the device, so the loop measures
decoding, not input generation.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass, field

import numpy as np

from paper_1702_07740_amd import synth

RATES = (0.02, 0.05, 0.1)
LIFTS = (1024, 2048, 4096, 6667)
THRESHOLD_MARGIN_DB = 0.3
_THR_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "template_thresholds.json")


def template_thresholds():
    with open(_THR_PATH) as fh:
        t = json.load(fh)
    return {r: t[str(r)]["threshold_db"] for r in RATES}


@dataclass
class Pool:
    """Device-resident frames of one (rate, Z) code: llr [P][n], syndrome [P][m]."""
    rate: float
    Z: int
    code: object
    llr: object
    syn: object
    snr_db: float


@dataclass
class Req:
    arrival: float
    pool: int
    frames: list
    index: int = 0
    max_iters: int = 100
    ticket: int = 0
    done_at: float = field(default=float("nan"))


def pool_frames(rate, Z, n, frames_per_pool=8, seed=5):
    """Host inputs (key bits, channel LLRs) of the (rate, Z) pool: frames at the
    code's BP threshold + THRESHOLD_MARGIN_DB, drawn from a seed of their own."""
    snr = template_thresholds()[rate] + THRESHOLD_MARGIN_DB
    return synth.biawgn_frames(n, frames_per_pool, snr, seed=seed + 1000 * Z + int(rate * 1000))


def make_pools(ldpc, torch, lifts=LIFTS, rates=RATES, frames_per_pool=8, seed=5):
    thr = template_thresholds()
    pools = []
    for rate in rates:
        for Z in lifts:
            base = synth.template_for_rate(rate, Z, seed=1)
            code = ldpc.Code(base, Z)
            snr = thr[rate] + THRESHOLD_MARGIN_DB
            x, Q = pool_frames(rate, Z, code.n, frames_per_pool, seed)
            dQ = torch.from_numpy(Q).cuda()
            syn = code.syndrome(torch.from_numpy(x).cuda())
            pools.append(Pool(rate, Z, code, dQ, syn, snr))
    torch.cuda.synchronize()
    return pools


def poisson_trace(n_pools, rate_per_s, duration_s, frames_per_pool=8, max_frames=4, seed=7):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            return out
        p = int(rng.integers(0, n_pools))
        F = int(rng.integers(1, max_frames + 1))
        first = int(rng.integers(0, frames_per_pool - F + 1))
        out.append(Req(t, p, list(range(first, first + F)), index=len(out)))


def _inputs(pools, r):
    P = pools[r.pool]
    a, b = r.frames[0], r.frames[-1] + 1
    return P.code, P.llr[a:b], P.syn[a:b]


def run_engine(ldpc, torch, pools, trace, budget_bytes, max_slots=64, msg_fp16=False,
               keep_outputs=False, max_step_edges=0):
    """Serve `trace` in real time through the engine.  Returns stats (and outputs).

    max_step_edges caps the work of one engine step (frames x edges of the
    admitted requests), which bounds the step time and so the latency of every
    admitted request; requests beyond it wait in the queue."""
    eng = ldpc.Engine(budget_bytes, max_slots=max_slots, msg_fp16=msg_fp16,
                      max_step_edges=max_step_edges)
    by_ticket, outputs = {}, {}
    pending = list(trace)
    pending.reverse()
    done = 0
    peak_active = 0
    t0 = time.perf_counter()
    while done < len(trace):
        now = time.perf_counter() - t0
        while pending and pending[-1].arrival <= now:
            r = pending.pop()
            code, q, s = _inputs(pools, r)
            r.ticket = eng.submit(code, q, s, r.max_iters)
            by_ticket[r.ticket] = r
        for t in eng.poll():
            r = by_ticket.pop(t)
            r.done_at = time.perf_counter() - t0
            res = eng.result(t)
            if keep_outputs:
                outputs[r.index] = tuple(x.cpu().numpy() for x in res)
            done += 1
        active, queued = eng.step()
        peak_active = max(peak_active, active)
        if active == 0 and queued == 0 and not by_ticket:
            # idle: wait for the next arrival
            if pending:
                wait = pending[-1].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.002))
            else:
                torch.cuda.current_stream().synchronize()
    wall = time.perf_counter() - t0
    eng.close()
    return _stats(pools, trace, wall, peak_active), outputs


def run_one_at_a_time(ldpc, torch, pools, trace, keep_outputs=False):
    """The same trace through plain FP32 ldpc_decode_batch, one request at a time."""
    import sys
    outputs = {}
    t0 = time.perf_counter()
    last = t0
    for i, r in enumerate(trace):
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        if time.perf_counter() - last > 20.0:  # progress, so a long replay is seen to run
            last = time.perf_counter()
            print(f"[serve] one at a time: {i} of {len(trace)} requests", file=sys.stderr,
                  flush=True)
        code, q, s = _inputs(pools, r)
        bits, it, conv, _ = code.decode(q, s, r.max_iters)
        torch.cuda.current_stream().synchronize()
        r.done_at = time.perf_counter() - t0
        if keep_outputs:
            outputs[r.index] = (bits.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy())
    wall = time.perf_counter() - t0
    return _stats(pools, trace, wall, 1), outputs


def _stats(pools, trace, wall, peak_active):
    lat = np.array([r.done_at - r.arrival for r in trace]) * 1e3
    bits = sum(len(r.frames) * pools[r.pool].code.n for r in trace)
    return {
        "requests": len(trace), "wall_s": wall,
        "mbit_s": bits / wall / 1e6,
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_ms": float(np.mean(lat)) if len(lat) else None,
        "peak_in_flight": peak_active,
    }
