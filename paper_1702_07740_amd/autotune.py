"""Schedule autotuner for the decoder.

Tunables:
- checks per thread (1, 2 or 4) of the per-iteration check kernel: how many
  checks of a base row one thread handles, i.e. how many wavefronts cover one
  circulant block.  More checks per thread amortise the row's table reads and
  keep more loads in flight per thread; fewer give more workgroups for small Z
  and few frames;
- for a single decode call, also the schedule: per-iteration launches or the
  frame-resident kernel (one workgroup per frame, state in LDS), where the
  code's state fits.

Results do not depend on the choice (the arithmetic is identical), so the tuner
only measures time: each candidate decodes the actual batch for a few
iterations with early stop off, timed with HIP events, and the fastest wins.
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


def tune_decode(code, llr, syndrome, msg_fp16=False, iters=8, use_cache=True):
    """Best decode configuration for ldpc_decode_batch on this batch.

    Returns (best, ms): best = {"schedule": "launches" | "resident",
    "checks_per_thread": 1 | 2 | 4 (0 for the resident schedule)}, ms = the time
    of each candidate, keyed "launches/<cpt>" or "resident".
    """
    from paper_1702_07740_amd import ldpc
    key = _key("decode2", [_shape(code, llr.shape[0])], msg_fp16)
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return hit["best"], hit["ms"]
    ws = code.alloc_workspace(llr.shape[0], iters, msg_fp16=msg_fp16)
    cands = {f"launches/{cpt}": {"schedule": "launches", "checks_per_thread": cpt}
             for cpt in CANDIDATES}
    try:
        code.schedule(F=llr.shape[0], msg_fp16=msg_fp16, schedule="resident")
        cands["resident"] = {"schedule": "resident", "checks_per_thread": 0}
    except ldpc.LdpcError:
        pass  # the frame's state does not fit one workgroup's LDS
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
