"""Shared parity checks: HIP decoder outputs against the FP64 oracle.

Tolerances (stated once, used by every parity test):
  * posterior LLRs: |L_gpu - L_ref| <= 1e-3 * max(|L_ref|, 1)   (FP32 messages),
    held for every frame up to POSTERIOR_HORIZON iterations.  Near the BP
    threshold the iteration is chaotic: rounding differences between FP32 and
    FP64 grow from ~5e-6 at t = 10 to ~3e-4 at t = 30 and past 1e-3 after ~50
    iterations, so later posteriors of frames that did not converge are
    compared through decisions instead.  This horizon belongs to FP32 BP
    itself, not to the kernels' Phi: an FP32 decoder with Phi correctly
    rounded to FP32 drifts from the oracle just as fast (on the n = 9,600
    template at -14 dB: 5e-6, 4.6e-5, 4.1e-4, 2.4e-3, 5.8e-2 at t = 10, 30,
    50, 70, 100, against 2.1e-5, 8.9e-5, 7.3e-4, 2.9e-3, 5.9e-2 with the
    kernels' Phi).  Exit posteriors of frames converged on both sides at the
    same iteration are gated at every iteration count, by exit_rtol(t)
    (see exit_posterior_check);
  * syndromes and converged flags: bit-exact; converged <=> H x = s, with
    H x recomputed on the CPU by the oracle;
  * hard decisions: bit-exact on frames that converge on both sides;
  * iteration counts: within +-1 on frames that converge on both sides, and
    equal to max_iters on frames that converge on neither side;
  * one-sided convergence: a frame may converge on one side only.  BP near
    the threshold does not settle for many iterations, and an FP32 and an
    FP64 trajectory that agree to 1e-3 for the first ~30 iterations can part
    after that, so a frame that one side finishes shortly before max_iters
    may still be searching on the other.  The allowance is
    one_sided_allowance(F) = max(1, ceil(F / 8)) frames per batch, asserted
    by every caller of check_decode_parity (a larger count means the two
    decoders disagree on more than the last iterations of marginal frames).
  * FP16 message storage (fp16=True): the same checks except iteration
    counts, which are not compared: half-precision storage changes the
    trajectory, so a frame may converge a few iterations earlier or later;
    frame error rates are compared statistically instead.
"""
import math

import numpy as np

LLR_RTOL = 1e-3
POSTERIOR_HORIZON = 30


def exit_rtol(t: int) -> float:
    """Relative bound (on the scale of LLR_RTOL: |err| <= rtol * max(|L|, 1))
    for the exit posteriors of a frame that converged on both sides at
    iteration t.  LLR_RTOL up to POSTERIOR_HORIZON; beyond it the envelope of
    the FP32 drift measured with a correctly rounded Phi, which grows about
    tenfold every 20 iterations, capped at 1 (|err| <= max(|L|, 1): the same
    sign wherever |L| > 1, and no gross error) from t = 90 on.  At t = 99, a
    frame that converged after a long transient differed by 0.21 with the
    correctly rounded Phi and by 0.55 with the kernels."""
    if t <= POSTERIOR_HORIZON:
        return LLR_RTOL
    return min(1.0, LLR_RTOL * 10.0 ** ((t - POSTERIOR_HORIZON) / 20.0))


def one_sided_allowance(F: int) -> int:
    return max(1, math.ceil(F / 8))


def llr_close(L_gpu, L_ref, rtol=LLR_RTOL):
    L_gpu = np.asarray(L_gpu, dtype=np.float64)
    L_ref = np.asarray(L_ref, dtype=np.float64)
    err = np.abs(L_gpu - L_ref)
    bound = rtol * np.maximum(np.abs(L_ref), 1.0)
    bad = err > bound
    return (not bad.any()), float(np.max(err / bound)) if err.size else 0.0, int(bad.sum())


def check_decode_parity(ocode, Q, s, gpu_bits, gpu_iters, gpu_conv, ref, max_iters,
                        allowance=None, fp16=False):
    """ref = oracle.decode(...) on the same inputs.  Returns a summary dict.

    Asserts the converged flag against H x = s recomputed on the CPU, the
    decisions and iteration counts of frames converged on both sides, the
    counts of frames converged on neither, and that at most ``allowance``
    (default one_sided_allowance(F)) frames converge on one side only.
    """
    bits_r, L_r, it_r, conv_r = ref
    F = Q.shape[0]
    gpu_conv = np.asarray(gpu_conv).astype(bool)
    conv_r = np.asarray(conv_r).astype(bool)
    # converged flag <=> H x = s, recomputed on the CPU from the GPU's bits
    syn = ocode.syndrome(gpu_bits)
    for f in range(F):
        assert bool(gpu_conv[f]) == bool(np.array_equal(syn[f], s[f])), f"frame {f}: flag vs H x"
    both = np.logical_and(gpu_conv, conv_r)
    for f in np.nonzero(both)[0]:
        assert np.array_equal(gpu_bits[f], bits_r[f]), f"frame {f}: decisions differ"
        if not fp16:
            assert abs(int(gpu_iters[f]) - int(it_r[f])) <= 1, f"frame {f}: iterations"
    neither = np.logical_and(~gpu_conv, ~conv_r)
    for f in np.nonzero(neither)[0]:
        assert int(gpu_iters[f]) == max_iters and int(it_r[f]) == max_iters
    summ = {"both": int(both.sum()), "gpu_only": int((gpu_conv & ~conv_r).sum()),
            "ref_only": int((~gpu_conv & conv_r).sum()), "neither": int(neither.sum())}
    lim = one_sided_allowance(F) if allowance is None else allowance
    assert summ["gpu_only"] + summ["ref_only"] <= lim, f"one-sided convergence {summ} > {lim}"
    return summ


def exit_posterior_check(L_gpu, ref, gpu_iters, gpu_conv):
    """Exit posteriors of every frame converged on both sides at the same
    iteration, gated at exit_rtol(t).  Returns per-frame (iterations, worst
    and p99 of err / (LLR_RTOL max(|L|, 1))) for the report."""
    bits_r, L_r, it_r, conv_r = ref
    both = np.logical_and(np.asarray(gpu_conv).astype(bool), np.asarray(conv_r).astype(bool))
    rows = []
    for f in np.nonzero(both)[0]:
        if int(gpu_iters[f]) != int(it_r[f]):
            continue
        g = np.asarray(L_gpu[f], dtype=np.float64)
        r = np.asarray(L_r[f], dtype=np.float64)
        rel = np.abs(g - r) / (LLR_RTOL * np.maximum(np.abs(r), 1.0))
        rows.append((int(gpu_iters[f]), float(rel.max()), float(np.percentile(rel, 99))))
        rtol = exit_rtol(int(gpu_iters[f]))
        ok, worst, nbad = llr_close(g, r, rtol)
        assert ok, f"frame {f} (t = {int(gpu_iters[f])}): exit posterior worst {worst:.3g} of {rtol}"
    return rows
