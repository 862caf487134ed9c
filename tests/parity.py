"""Shared parity checks: HIP decoder outputs against the FP64 oracle.

Tolerances (stated once, used by every parity test):
  * posterior LLRs: |L_gpu - L_ref| <= 1e-3 * max(|L_ref|, 1)   (FP32 messages),
    held for every frame up to POSTERIOR_HORIZON iterations.  Near the BP
    threshold the iteration is chaotic: rounding differences between FP32 and
    FP64 grow from ~5e-6 at t = 10 to ~3e-4 at t = 30 and past 1e-3 after ~50
    iterations, so later posteriors are compared through decisions instead;
  * syndromes and converged flags: bit-exact; converged <=> H x = s, with
    H x recomputed on the CPU by the oracle;
  * hard decisions: bit-exact on frames that converge on both sides;
  * iteration counts: within +-1 on frames that converge on both sides, and
    equal to max_iters on frames that converge on neither side.
"""
import numpy as np

LLR_RTOL = 1e-3
POSTERIOR_HORIZON = 30


def llr_close(L_gpu, L_ref, rtol=LLR_RTOL):
    L_gpu = np.asarray(L_gpu, dtype=np.float64)
    L_ref = np.asarray(L_ref, dtype=np.float64)
    err = np.abs(L_gpu - L_ref)
    bound = rtol * np.maximum(np.abs(L_ref), 1.0)
    bad = err > bound
    return (not bad.any()), float(np.max(err / bound)) if err.size else 0.0, int(bad.sum())


def check_decode_parity(ocode, Q, s, gpu_bits, gpu_iters, gpu_conv, ref, max_iters):
    """ref = oracle.decode(...) on the same inputs.  Returns a summary dict."""
    bits_r, L_r, it_r, conv_r = ref
    F = Q.shape[0]
    # converged flag <=> H x = s, recomputed on the CPU from the GPU's bits
    syn = ocode.syndrome(gpu_bits)
    for f in range(F):
        assert bool(gpu_conv[f]) == bool(np.array_equal(syn[f], s[f])), f"frame {f}: flag vs H x"
    both = np.logical_and(gpu_conv.astype(bool), conv_r)
    for f in np.nonzero(both)[0]:
        assert np.array_equal(gpu_bits[f], bits_r[f]), f"frame {f}: decisions differ"
        assert abs(int(gpu_iters[f]) - int(it_r[f])) <= 1, f"frame {f}: iterations"
    neither = np.logical_and(~gpu_conv.astype(bool), ~conv_r)
    for f in np.nonzero(neither)[0]:
        assert int(gpu_iters[f]) == max_iters and int(it_r[f]) == max_iters
    return {"both": int(both.sum()), "gpu_only": int((gpu_conv.astype(bool) & ~conv_r).sum()),
            "ref_only": int((~gpu_conv.astype(bool) & conv_r).sum()), "neither": int(neither.sum())}
