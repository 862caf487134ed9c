"""Schedule autotuner for the decoder.

Tunables:
- checks per thread (1, 2 or 4) of the per-iteration check kernel: how many
  checks of a base row one thread handles, i.e. how many wavefronts cover one
  circulant block.  More checks per thread amortise the row's table reads and
  keep more loads in flight per thread; fewer give more workgroups for small Z
  and few frames;
- for a single decode call, also the number of streams of the per-iteration
  launches (one, or the two halves of the frames on two streams: two double
  the launches of an iteration and pay only where each half's iteration
  outlasts the host's launch rate), and the schedule: per-iteration launches,
  the frame-resident kernel (one workgroup per frame, state in LDS) or the
  frame-split kernel (a few co-resident workgroups per frame), where the
  code's state fits.

Results do not depend on the choice (the arithmetic is identical), so the tuner
only measures time: each candidate decodes the actual batch with early stop
off, timed with HIP events, and the fastest wins.  A single decode is timed at
its own iteration count, so that per-call costs (set-up, read-out, the fork and
join of two streams) weigh as they will in use: at 8 iterations one stream
looked faster on the n = 1,000,050 batch of 8 frames, at 100 two streams are.
Choices are cached in a JSON file keyed by the workload's shape, precision and
device name (LDPC_AUTOTUNE_CACHE overrides the path).
"""
from __future__ import annotations

import json
import os
import threading

CANDIDATES = (1, 2, 4)
_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("LDPC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1702_07740_amd",
                                       "autotune.json"))


def _load_cache():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(key, value):
    with _lock:
        cache = _load_cache()
        cache[key] = value
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)


def _key(kind, shapes, fp16):
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return json.dumps({"kind": kind, "shapes": shapes, "fp16": bool(fp16), "device": dev},
                      sort_keys=True)


def _shape(code, F):
    i = code.info
    return [i["mb"], i["nb"], i["Z"], i["blocks"], i["core_cols"], int(F)]


def _time(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def name_of(cfg) -> str:
    """The candidate name of a tune_decode configuration."""
    if cfg["schedule"] == "launches":
        return f"launches/{cfg['checks_per_thread']}/{cfg['streams']}"
    return cfg["schedule"]


def tune_decode(code, llr, syndrome, msg_fp16=False, iters=100, use_cache=True):
    """Best decode configuration for ldpc_decode_batch on this batch.

    Returns (best, ms): best = keyword arguments of Code.decode,
    {"schedule": "launches", "checks_per_thread": 1 | 2 | 4, "streams": 1 | 2}
    or {"schedule": "resident" | "split", "checks_per_thread": 0, "streams": 0};
    ms = the time of each candidate, keyed by name_of: "launches/<cpt>/<streams>",
    "resident" or "split".  iters: the decode's max_iters (part of the cache key).
    """
    from paper_1702_07740_amd import ldpc
    F = llr.shape[0]
    key = _key("decode3", [_shape(code, F), int(iters)], msg_fp16)
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return hit["best"], hit["ms"]
    ws = code.alloc_workspace(F, iters, msg_fp16=msg_fp16)
    cands = {}
    for cpt in CANDIDATES:
        for streams in ((1, 2) if F >= 2 else (1,)):
            cfg = {"schedule": "launches", "checks_per_thread": cpt, "streams": streams}
            cands[name_of(cfg)] = cfg
    for sch in ("resident", "split"):
        try:
            code.schedule(F=F, msg_fp16=msg_fp16, schedule=sch)
            cands[sch] = {"schedule": sch, "checks_per_thread": 0, "streams": 0}
        except ldpc.LdpcError:
            pass  # the frame's state does not fit one workgroup's LDS, or too many frames
    ms = {}
    for name, cfg in cands.items():
        ms[name] = _time(lambda: code.decode(llr, syndrome, iters, early_stop=False,
                                             msg_fp16=msg_fp16, workspace=ws, **cfg))
    best = cands[min(ms, key=ms.get)]
    _store(key, {"best": best, "ms": ms})
    return best, ms


def tune_engine(requests, msg_fp16=False, iters=8, use_cache=True):
    """Best checks_per_thread for an engine batch of (code, llr, syndrome) requests."""
    from paper_1702_07740_amd import ldpc
    key = _key("engine", sorted(_shape(c, q.shape[0]) for c, q, s in requests), msg_fp16)
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return hit["best"], hit["ms"]
    ms = {}
    for cpt in CANDIDATES:
        def run():
            eng = ldpc.Engine(64 << 30, max_slots=min(64, len(requests)), msg_fp16=msg_fp16,
                              early_stop=False, checks_per_thread=cpt)
            tickets = [eng.submit(c, q, s, iters) for c, q, s in requests]
            eng.drain(tickets)
            eng.close()
        ms[cpt] = _time(run, reps=2)
    best = min(ms, key=ms.get)
    _store(key, {"best": best, "ms": ms})
    return best, ms
