"""The frame-resident schedule (one workgroup per frame, state in LDS) and the
frame-split schedule (several co-resident workgroups per frame) against the
FP64 oracle and, bit for bit, against the per-iteration launches.

Every case prints its name, seed and shape before touching the GPU.
"""
import numpy as np
import pytest

from paper_1702_07740_amd import synth
from tests.parity import check_decode_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ldpc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_07740_amd import ldpc as mod
    mod.load()
    return mod


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(g, Q, s, T, **kw):
    bits, it, conv, _ = g.decode(_dev(Q), _dev(s), T, **kw)
    torch.cuda.synchronize()
    return bits.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy()


def _split_offered(g, F, fp16):
    from paper_1702_07740_amd import ldpc as mod
    try:
        return g.schedule(F=F, msg_fp16=fp16, schedule="split") == "split"
    except mod.LdpcError:
        return False


def _same(g, Q, s, T, **kw):
    """Decode on every schedule offered for the batch and require identical
    outputs: launches, resident, and frame-split where the batch allows it."""
    a = _run(g, Q, s, T, schedule="launches", **kw)
    b = _run(g, Q, s, T, schedule="resident", **kw)
    for name, u, v in zip(("bits", "iters", "converged"), a, b):
        assert np.array_equal(u, v), (name, kw)
    if _split_offered(g, Q.shape[0], kw.get("msg_fp16", False)):
        c = _run(g, Q, s, T, schedule="split", **kw)
        for name, u, v in zip(("bits", "iters", "converged"), a, c):
            assert np.array_equal(u, v), ("split", name, kw)
    return b


def _general_base(rng, Z):
    """Columns of degree 0, 1 and >= 2; rows of degree 1, 2, 3, 7 and 16,
    one with two degree-1 blocks (generic widths 8 and 16)."""
    base = np.full((7, 21), -1, dtype=np.int32)
    base[0, :16] = rng.integers(0, Z, 16)
    base[1, 2] = 4 % Z
    base[2, [0, 17]] = [3 % Z, 9 % Z]
    base[3, [1, 3, 5, 7, 9, 11, 18]] = rng.integers(0, Z, 7)
    base[4, [0, 2, 4]] = rng.integers(0, Z, 3)
    base[5, [6, 8, 10]] = rng.integers(0, Z, 3)
    base[6, [1, 12, 19, 20]] = rng.integers(0, Z, 4)   # columns 19, 20: degree 1
    return base


# ------------------------------------------------------ schedule selection
def test_schedule_selection(ldpc):
    small = ldpc.Code(synth.template_base(144, 64, seed=1), 64)
    # many frames of a small code: one workgroup per frame and CU pays off
    assert small.schedule(F=1024) == "resident"
    assert small.schedule(F=1024, msg_fp16=True) == "resident"
    assert small.schedule(F=1024, want_llr=True) == "launches"
    assert small.schedule(F=1024, timing=True) == "launches"
    assert small.schedule(F=1024, schedule="launches") == "launches"
    assert small.schedule(F=1, schedule="resident") == "resident"
    with pytest.raises(ldpc.LdpcError) as e:
        small.schedule(want_llr=True, schedule="resident")
    assert e.value.status == ldpc.LDPC_EUNSUPPORTED
    big = ldpc.Code(synth.template_base(144, 6667, seed=1), 6667)
    assert big.schedule(F=8) == "launches"
    assert big.schedule(F=1024) == "launches"
    with pytest.raises(ldpc.LdpcError) as e:
        big.schedule(schedule="resident")
    assert e.value.status == ldpc.LDPC_EUNSUPPORTED
    with pytest.raises(ldpc.LdpcError) as e:
        small.schedule(schedule=4)
    assert e.value.status == ldpc.LDPC_EINVAL
    # the frame-split schedule: small codes, at most 256 frames
    assert small.schedule(F=16, schedule="split") == "split"
    assert small.schedule(F=256, msg_fp16=True, schedule="split") == "split"
    for kw in (dict(F=257), dict(F=1, want_llr=True), dict(F=1, timing=True)):
        with pytest.raises(ldpc.LdpcError) as e:
            small.schedule(schedule="split", **kw)
        assert e.value.status == ldpc.LDPC_EUNSUPPORTED
    with pytest.raises(ldpc.LdpcError) as e:
        big.schedule(F=1, schedule="split")
    assert e.value.status == ldpc.LDPC_EUNSUPPORTED
    # a forced resident decode of a code whose state does not fit fails at
    # the call, before any launch
    Q = torch.zeros((1, big.n), dtype=torch.float32, device="cuda")
    s = torch.zeros((1, big.m), dtype=torch.uint8, device="cuda")
    with pytest.raises(ldpc.LdpcError):
        big.decode(Q, s, 3, schedule="resident")


# ---------------------------------------------------- oracle parity
@pytest.mark.parametrize("schedule", ["resident", "split"])
@pytest.mark.parametrize("snr,F,seed", [(-15.4, 16, 1), (-14.0, 16, 2), (-13.0, 16, 3)])
def test_resident_parity_small_template(ldpc, oracle_mod, snr, F, seed, schedule):
    """The n = 9600 template (Z = 64), 16 frames, max 100 iterations, early stop."""
    Z, T = 64, 100
    base = synth.template_base(144, Z, seed=1)
    g, o = ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(o.n, F, snr, seed=seed)
    s = o.syndrome(x)
    _say(schedule, "decode", "snr", snr, "F", F, "n", o.n)
    bits, it, conv = _run(g, Q, s, T, schedule=schedule)
    summ = check_decode_parity(o, Q, s, bits, it, conv, o.decode(Q, s, T, threads=8), T)
    print("summary", summ, flush=True)


# -------------------------------------- bit-identical to the launches
@pytest.mark.parametrize("fp16", [False, True])
@pytest.mark.parametrize("snr", [-15.4, -13.5, -12.0])
def test_same_as_launches_small_template(ldpc, oracle_mod, snr, fp16):
    Z, F = 64, 16
    base = synth.template_base(144, Z, seed=1)
    g, o = ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(o.n, F, snr, seed=int(-snr * 10))
    s = o.syndrome(x)
    _say("resident = launches", snr, "fp16", fp16)
    bits, it, conv = _same(g, Q, s, 100, msg_fp16=fp16)
    if snr > -13.0:
        assert conv.sum() >= F // 2  # early stop exercised


@pytest.mark.parametrize("T", [0, 1, 2, 7])
def test_same_as_launches_short_runs(ldpc, oracle_mod, T):
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g, o = ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(o.n, 4, -11.0, seed=70 + T)
    s = o.syndrome(x)
    Q[1] = synth.noiseless_llr(x[1], 2.0)   # stops at iteration 0
    _say("resident short", T)
    _same(g, Q, s, T)
    _same(g, Q, s, T, early_stop=False)
    bits, it, conv = _same(g, Q, s, T, check_from_iter=2)
    assert it[1] == min(2, T) and conv[1] == 1
    if T == 0:
        b_r, _, it_r, c_r = o.decode(Q, s, 0)
        assert np.array_equal(bits, b_r) and np.array_equal(conv.astype(bool), c_r)


@pytest.mark.parametrize("Z", [1, 3, 63, 65, 100, 128, 200, 256])
def test_same_as_launches_ragged_lifting(ldpc, oracle_mod, Z):
    base = synth.template_base(24, Z, seed=2)
    g, o = ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(o.n, 5, -4.0, seed=Z)
    s = o.syndrome(x)
    _say("resident ragged Z", Z, "n", o.n)
    bits, it, conv = _same(g, Q, s, 60)
    _same(g, Q, s, 60, msg_fp16=True)
    check_decode_parity(o, Q, s, bits, it, conv, o.decode(Q, s, 60), 60)


@pytest.mark.parametrize("Z", [5, 37, 64])
def test_same_as_launches_general_code(ldpc, oracle_mod, Z):
    rng = np.random.default_rng(90 + Z)
    base = _general_base(rng, Z)
    g, o = ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)
    assert g.info["deg0_cols"] >= 1 and g.info["max_row_degree"] == 16
    x, Q = synth.biawgn_frames(o.n, 4, 0.0, seed=Z)
    s = o.syndrome(x)
    _say("resident general code", base.shape, Z)
    for T in (1, 4, 40):
        bits, it, conv = _same(g, Q, s, T)
        _same(g, Q, s, T, msg_fp16=True)
    check_decode_parity(o, Q, s, bits, it, conv, o.decode(Q, s, 40), 40)


def test_batch_independent(ldpc, oracle_mod):
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g, o = ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(o.n, 6, -13.5, seed=61)
    s = o.syndrome(x)
    _say("resident batch independence")
    for sch in ("resident", "split"):
        full = _run(g, Q, s, 80, schedule=sch)
        for f in (0, 3, 5):
            alone = _run(g, Q[f:f + 1], s[f:f + 1], 80, schedule=sch)
            for u, v in zip(alone, full):
                assert np.array_equal(u[0], v[f])


def test_many_frames(ldpc, oracle_mod):
    """More frames than compute units: several workgroups per CU over time."""
    Z, F = 64, 600
    base = synth.template_base(144, Z, seed=1)
    g, o = ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(o.n, F, -13.5, seed=600)
    s = o.syndrome(x)
    _say("resident many frames", F)
    _same(g, Q, s, 50)


def test_autotuner_picks_the_fastest_schedule(ldpc, oracle_mod, tmp_path, monkeypatch):
    """The autotuner times every (schedule, checks per thread, streams)
    candidate on the actual batch and returns the fastest; its choice decodes
    identically."""
    from paper_1702_07740_amd import autotune
    monkeypatch.setenv("LDPC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    Z, F = 64, 128
    base = synth.template_base(144, Z, seed=1)
    g, o = ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(o.n, F, -13.5, seed=128)
    s = o.syndrome(x)
    dQ, ds = _dev(Q), _dev(s)
    _say("autotune schedule", Z, F)
    best, ms = autotune.tune_decode(g, dQ, ds)
    assert set(ms) == {f"launches/{c}/{n}" for c in (1, 2, 4) for n in (1, 2)} | {"resident",
                                                                                    "split"}
    assert ms[autotune.name_of(best)] == min(ms.values())
    again, _ = autotune.tune_decode(g, dQ, ds)  # from the cache
    assert again == best
    ref = _run(g, Q, s, 50, schedule="launches")
    got = _run(g, Q, s, 50, **best)
    for u, v in zip(ref, got):
        assert np.array_equal(u, v)


def test_lds_budget_boundary(ldpc, oracle_mod):
    """At Z = 128 the R = 0.02 template's FP32 state (306 blocks x 128 x 4 B =
    157 KB of messages alone) exceeds one workgroup's LDS, while its FP16
    state fits: the resident schedule is refused for FP32 and runs, bit-exact
    against the launches, for FP16 messages."""
    Z, F = 128, 8
    base = synth.template_base(144, Z, seed=1)
    g, o = ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)
    assert g.schedule(F=1024) == "launches"
    with pytest.raises(ldpc.LdpcError) as e:
        g.schedule(F=1, schedule="resident")
    assert e.value.status == ldpc.LDPC_EUNSUPPORTED
    assert g.schedule(F=1, msg_fp16=True, schedule="resident") == "resident"
    x, Q = synth.biawgn_frames(o.n, F, -13.8, seed=128)
    s = o.syndrome(x)
    _say("LDS budget boundary", Z, F)
    _same(g, Q, s, 100, msg_fp16=True)
