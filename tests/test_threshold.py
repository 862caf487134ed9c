"""Density evolution tool (base-graph BP thresholds on the BIAWGN channel).

Pinned to textbook values: the Shannon limit of the BIAWGN channel at rate
1/2 (0.187 dB) and the BP threshold of the regular (3,6) ensemble
(sigma* = 0.8809, i.e. 1.10 dB in SNR = 1/sigma^2).  The stored template
thresholds are re-checked at +-0.2 dB.
"""
import json
import os

import numpy as np

from paper_1702_07740_amd import synth, threshold


def test_shannon_limits():
    assert abs(threshold.shannon_limit_db(0.5) - 0.187) < 0.005
    # the rate-0.02 limit the paper's efficiency figures refer to
    assert abs(threshold.shannon_limit_db(0.02) - (-15.51)) < 0.01
    # eq. snr(beta): R = 0.02 at beta = 0.99 -> -15.47 dB, the paper's d = 8 point
    assert abs(synth.snr_db_from_beta(0.02, 0.99) - (-15.47)) < 0.01


def test_regular_3_6_threshold():
    base = np.zeros((3, 6), dtype=np.int32)
    assert threshold.de_converges(base, 1.30, n_samples=10000, max_iters=300)
    assert not threshold.de_converges(base, 0.90, n_samples=10000, max_iters=300)


def test_stored_template_thresholds_bracket():
    path = os.path.join(os.path.dirname(threshold.__file__), "template_thresholds.json")
    thr = json.load(open(path))
    t = thr["0.1"]["threshold_db"]
    base = synth.template_for_rate(0.1, 8, seed=1)
    assert threshold.de_converges(base, t + 0.2, n_samples=10000, max_iters=300)
    assert not threshold.de_converges(base, t - 0.2, n_samples=10000, max_iters=300)
    for r in ("0.02", "0.05", "0.1"):
        assert thr[r]["threshold_db"] > thr[r]["shannon_limit_db"]
