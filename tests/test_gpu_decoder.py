"""Parity of the HIP decoder (through the C ABI) against the FP64 oracle.

Every case prints its name, seed and shape before touching the GPU.
"""
import numpy as np
import pytest

from paper_1702_07740_amd import synth
from tests.parity import LLR_RTOL, check_decode_parity, exit_posterior_check, llr_close
from tests.qc_dense import random_tree_base

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


def _gpu_decode(gcode, Q, s, T, **kw):
    bits, it, conv, L = gcode.decode(_dev(Q), _dev(s), T, **kw)
    torch.cuda.synchronize()
    return (bits.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy(),
            None if L is None else L.cpu().numpy())


def _codes(ldpc, oracle_mod, base, Z):
    return ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)


# ------------------------------------------------------------ syndromes
@pytest.mark.parametrize("kind,Z", [("template", 64), ("template", 67), ("template", 1),
                                    ("random", 13), ("random", 300), ("template", 6667)])
def test_syndrome_bit_exact(ldpc, oracle_mod, kind, Z):
    rng = np.random.default_rng(Z)
    if kind == "template":
        base = synth.template_base(144, Z, seed=5)
    else:
        base = rng.integers(-1, Z, size=(7, 11)).astype(np.int32)
        base[:, 3] = -1            # a degree-0 column
        base[:, 4] = -1
        base[2, 4] = 5 % Z         # a degree-1 column
        base[np.all(base < 0, axis=1), 0] = 0
    _say("syndrome", kind, "Z", Z, "base", base.shape)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    x = rng.integers(0, 2, size=(3, o.n)).astype(np.uint8)
    got = g.syndrome(_dev(x)).cpu().numpy()
    assert np.array_equal(got, o.syndrome(x))


# ------------------------------------------------- per-iteration posteriors
@pytest.mark.parametrize("snr", [-15.4, -13.0])
@pytest.mark.parametrize("T", [1, 2, 5, 10, 20, 30])
def test_posterior_llr_per_iteration(ldpc, oracle_mod, snr, T):
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    x, Q = synth.biawgn_frames(o.n, 4, snr, seed=40 + T)
    s = o.syndrome(x)
    _say("posterior", "snr", snr, "T", T, "n", o.n)
    bits, it, conv, L = _gpu_decode(g, Q, s, T, early_stop=False, want_llr=True)
    b_r, L_r, it_r, c_r = o.decode(Q, s, T, early_stop=False)
    ok, worst, nbad = llr_close(L, L_r)
    assert ok, f"worst error/bound {worst:.3g}, {nbad} entries over"
    assert np.all(it == T) and np.all(it_r == T)
    margin = 2 * LLR_RTOL * np.maximum(np.abs(L_r), 1.0)
    sure = np.abs(L_r) > margin
    assert np.array_equal(bits[sure], b_r[sure])
    # decisions follow the posterior sign, except within rounding of a tie
    # (degree-1 decisions are taken in the Phi domain, see the decoder notes)
    tie = np.abs(L) <= 1e-5 * np.maximum(np.abs(Q), 1.0)
    assert np.all((bits == (L < 0)) | tie)


# --------------------------------------------------- early-stop decoding
@pytest.mark.parametrize("snr,F,seed", [(-15.4, 16, 1), (-14.0, 16, 2), (-13.0, 16, 3),
                                        (-12.0, 8, 4)])
def test_decode_parity_small_template(ldpc, oracle_mod, snr, F, seed):
    """The n = 9600 template (Z = 64), 16 frames, max 100 iterations, early stop."""
    Z, T = 64, 100
    base = synth.template_base(144, Z, seed=1)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    x, Q = synth.biawgn_frames(o.n, F, snr, seed=seed)
    s = o.syndrome(x)
    _say("decode", "snr", snr, "F", F, "n", o.n)
    bits, it, conv, L = _gpu_decode(g, Q, s, T, want_llr=True)
    ref = o.decode(Q, s, T, threads=8)
    summ = check_decode_parity(o, Q, s, bits, it, conv, ref, T)
    print("summary", summ, flush=True)
    # exit posteriors of every frame that stops at the same iteration on both
    # sides, at every iteration count (the bound widens past the horizon)
    rows = exit_posterior_check(L, ref, it, conv)
    print("exit posteriors (t, worst, p99 err / 1e-3 bound)", rows, flush=True)


def test_noiseless_frames_stop_at_zero(ldpc, oracle_mod):
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    x = synth.random_bits(o.n, 5, seed=9)
    s = o.syndrome(x)
    Q = synth.noiseless_llr(x, 4.0)
    _say("noiseless", "n", o.n)
    bits, it, conv, L = _gpu_decode(g, Q, s, 30, want_llr=True)
    assert np.all(it == 0) and np.all(conv == 1)
    assert np.array_equal(bits, x)
    assert np.array_equal(L, Q)


@pytest.mark.parametrize("which", ["core", "deg1"])
def test_one_weak_wrong_bit(ldpc, oracle_mod, which):
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    x = synth.random_bits(o.n, 1, seed=12)
    s = o.syndrome(x)
    Q = synth.noiseless_llr(x, 5.0)
    v = 2 * Z + 3 if which == "core" else 40 * Z + 5
    Q[0, v] = -0.1 * (1 - 2.0 * x[0, v])
    _say("weak bit", which)
    bits, it, conv, _ = _gpu_decode(g, Q, s, 50)
    assert it[0] == 1 and conv[0] == 1 and np.array_equal(bits[0], x[0])


def test_tree_forest_matches_oracle(ldpc, oracle_mod):
    """A Z-lift of a cycle-free base graph is a forest: BP is exact MAP there."""
    rng = np.random.default_rng(77)
    Z = 64
    base = random_tree_base(rng, 14, 5, Z)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    Q = (rng.uniform(0.2, 2.5, size=(2, o.n)) * rng.choice([-1.0, 1.0], size=(2, o.n))).astype(np.float32)
    s = o.syndrome(rng.integers(0, 2, size=(2, o.n)).astype(np.uint8))
    _say("tree forest", base.shape)
    T = 25
    bits, it, conv, L = _gpu_decode(g, Q, s, T, early_stop=False, want_llr=True)
    _, L_r, _, _ = o.decode(Q, s, T, early_stop=False)
    ok, worst, _ = llr_close(L, L_r)
    assert ok, worst


def test_coset_equivariance_bitwise(ldpc, oracle_mod):
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    rng = np.random.default_rng(5)
    x, Q = synth.biawgn_frames(o.n, 4, -13.0, seed=51)
    s = o.syndrome(x)
    a = rng.integers(0, 2, size=x.shape).astype(np.uint8)
    Q2 = np.where(a == 1, -Q, Q).astype(np.float32)
    s2 = s ^ o.syndrome(a)
    _say("coset")
    b1, i1, c1, L1 = _gpu_decode(g, Q, s, 60, want_llr=True)
    b2, i2, c2, L2 = _gpu_decode(g, Q2, s2, 60, want_llr=True)
    assert np.array_equal(b1 ^ a, b2)
    assert np.array_equal(i1, i2) and np.array_equal(c1, c2)
    assert np.array_equal(np.where(a == 1, -L1, L1), L2)


def test_deterministic_and_batch_independent(ldpc, oracle_mod):
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g = ldpc.Code(base, Z)
    o = oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(o.n, 6, -13.5, seed=61)
    s = o.syndrome(x)
    _say("determinism")
    r1 = _gpu_decode(g, Q, s, 80, want_llr=True)
    r2 = _gpu_decode(g, Q, s, 80, want_llr=True)
    for u, v in zip(r1, r2):
        assert np.array_equal(u, v)
    for f in (0, 3, 5):
        alone = _gpu_decode(g, Q[f:f + 1], s[f:f + 1], 80, want_llr=True)
        for u, v in zip(alone, r1):
            assert np.array_equal(u[0], v[f])


# ------------------------------------------------------------ edge cases
def test_zero_iterations(ldpc, oracle_mod):
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    x, Q = synth.biawgn_frames(o.n, 3, -10.0, seed=3)
    s = o.syndrome(x)
    Q[1] = synth.noiseless_llr(x[1], 2.0)
    _say("T=0")
    bits, it, conv, L = _gpu_decode(g, Q, s, 0, want_llr=True)
    b_r, L_r, it_r, c_r = o.decode(Q, s, 0)
    assert np.array_equal(bits, b_r) and np.all(it == 0)
    assert np.array_equal(conv.astype(bool), c_r) and conv[1] == 1
    assert np.array_equal(L, Q)


def test_check_from_and_no_early_stop(ldpc, oracle_mod):
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    x = synth.random_bits(o.n, 2, seed=13)
    s = o.syndrome(x)
    Q = synth.noiseless_llr(x, 3.0)
    _say("check_from")
    _, it, conv, _ = _gpu_decode(g, Q, s, 20, check_from_iter=4)
    assert np.all(it == 4) and np.all(conv == 1)
    _, it, conv, _ = _gpu_decode(g, Q, s, 7, early_stop=False)
    assert np.all(it == 7) and np.all(conv == 1)


@pytest.mark.parametrize("Z", [1, 3, 63, 65, 257, 1000])
def test_ragged_lifting_sizes(ldpc, oracle_mod, Z):
    base = synth.template_base(24, Z, seed=2)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    x, Q = synth.biawgn_frames(o.n, 3, -4.0, seed=Z)
    s = o.syndrome(x)
    _say("ragged Z", Z, "n", o.n)
    for T in (3,):
        bits, it, conv, L = _gpu_decode(g, Q, s, T, early_stop=False, want_llr=True)
        _, L_r, _, _ = o.decode(Q, s, T, early_stop=False)
        ok, worst, _ = llr_close(L, L_r)
        assert ok, worst
    bits, it, conv, L = _gpu_decode(g, Q, s, 50)
    check_decode_parity(o, Q, s, bits, it, conv, o.decode(Q, s, 50), 50)


def test_general_code_with_degree_0_and_degree_1_rows(ldpc, oracle_mod):
    """Columns of degree 0, 1 and >= 2; check rows of degree 1, 2, 7 and 16."""
    rng = np.random.default_rng(8)
    Z = 37
    mb, nb = 6, 20
    base = np.full((mb, nb), -1, dtype=np.int32)
    base[0, :16] = rng.integers(0, Z, 16)          # degree-16 row
    base[1, 2] = 4                                 # degree-1 row
    base[2, [0, 17]] = [3, 9]                      # degree-2 row, column 17 has degree 1
    base[3, [1, 3, 5, 7, 9, 11, 18]] = rng.integers(0, Z, 7)
    base[4, [0, 2, 4]] = rng.integers(0, Z, 3)
    base[5, [6, 8, 10]] = rng.integers(0, Z, 3)
    # columns 16 and 19 stay empty (degree 0)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    info = g.info
    assert info["deg0_cols"] == 2 and info["max_row_degree"] == 16
    x, Q = synth.biawgn_frames(o.n, 4, 0.0, seed=8)
    s = o.syndrome(x)
    _say("general code", base.shape, Z)
    for T in (1, 4):
        bits, it, conv, L = _gpu_decode(g, Q, s, T, early_stop=False, want_llr=True)
        _, L_r, _, _ = o.decode(Q, s, T, early_stop=False)
        ok, worst, _ = llr_close(L, L_r)
        assert ok, worst
    bits, it, conv, L = _gpu_decode(g, Q, s, 40)
    check_decode_parity(o, Q, s, bits, it, conv, o.decode(Q, s, 40), 40)


def test_invalid_arguments(ldpc):
    Z = 16
    base = synth.template_base(24, Z, seed=2)
    g = ldpc.Code(base, Z)
    lib = ldpc.load()
    Q = torch.zeros((2, g.n), dtype=torch.float32, device="cuda")
    s = torch.zeros((2, g.m), dtype=torch.uint8, device="cuda")
    bits = torch.empty((2, g.n), dtype=torch.uint8, device="cuda")
    it = torch.empty(2, dtype=torch.int32, device="cuda")
    cv = torch.empty(2, dtype=torch.uint8, device="cuda")
    ws = g.alloc_workspace(2, 10)
    o = ldpc.make_opts()
    import ctypes

    def call(F, T, wsp, wsn, q=Q.data_ptr()):
        return lib.ldpc_decode_batch(g.handle, F, q, s.data_ptr(), T, bits.data_ptr(),
                                     it.data_ptr(), cv.data_ptr(), ctypes.byref(o), wsp, wsn, None)

    _say("invalid args")
    assert call(0, 10, ws.data_ptr(), ws.numel()) == ldpc.LDPC_EINVAL
    assert call(2, -1, ws.data_ptr(), ws.numel()) == ldpc.LDPC_EINVAL
    assert call(2, 10, ws.data_ptr(), ws.numel(), q=None) == ldpc.LDPC_EINVAL
    assert call(2, 10, ws.data_ptr(), ws.numel() - 1) == ldpc.LDPC_EWORKSPACE
    assert call(2, 10, None, ws.numel()) == ldpc.LDPC_EWORKSPACE
    assert call(2, 10, ws.data_ptr(), ws.numel()) == ldpc.LDPC_OK
    torch.cuda.synchronize()
    assert np.all(it.cpu().numpy() <= 10)
    for bad in (-1, 3):
        with pytest.raises(ldpc.LdpcError) as err:
            g.decode(Q, s, 10, streams=bad)
        assert err.value.status == ldpc.LDPC_EINVAL
    for bad in (-1, 2):
        with pytest.raises(ldpc.LdpcError) as err:
            g.decode(Q, s, 10, graphs=bad)
        assert err.value.status == ldpc.LDPC_EINVAL
    with pytest.raises(ldpc.LdpcError):
        ldpc.Code(np.array([[0, Z]], dtype=np.int32), Z)
    with pytest.raises(ldpc.LdpcError):
        ldpc.Code(np.zeros((1, 17), dtype=np.int32), Z)   # row degree 17 > 16


class _HipEvents:
    """Caller-created hipEvent_t handles through the HIP runtime torch loaded."""

    def __init__(self, count):
        import ctypes
        self.ct = ctypes
        self.lib = ctypes.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.arr = (ctypes.c_void_p * count)()
        for i in range(count):
            ev = ctypes.c_void_p()
            assert self.lib.hipEventCreate(ctypes.byref(ev)) == 0
            self.arr[i] = ev

    def ms(self, i, j):
        out = self.ct.c_float()
        assert self.lib.hipEventElapsedTime(self.ct.byref(out), self.arr[i], self.arr[j]) == 0
        return out.value

    def close(self):
        for e in self.arr:
            self.lib.hipEventDestroy(e)


def test_timing_events(ldpc, oracle_mod):
    """Per-kernel events change no result, bracket each kernel in order, and
    too short an event array is rejected."""
    Z = 64
    base = synth.template_base(144, Z, seed=1)
    g = ldpc.Code(base, Z)
    x, Q = synth.biawgn_frames(g.n, 4, -15.4, seed=21)
    s = oracle_mod.OracleCode(base, Z).syndrome(x)
    T = 6
    _say("timing events", T)
    ref = _gpu_decode(g, Q, s, T, early_stop=False)
    ev = _HipEvents(4 * T)
    got = _gpu_decode(g, Q, s, T, early_stop=False, timing_events=ev.arr)
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b)
    for t in range(T):
        cn, vn = ev.ms(4 * t, 4 * t + 1), ev.ms(4 * t + 2, 4 * t + 3)
        assert cn > 0 and vn > 0
        assert ev.ms(4 * t + 1, 4 * t + 2) >= 0
        if t:
            assert ev.ms(4 * t - 1, 4 * t) >= 0
    with pytest.raises(ldpc.LdpcError):
        g.decode(_dev(Q), _dev(s), T, timing_events=(ev.ct.c_void_p * (4 * T - 1))())
    torch.cuda.synchronize()
    ev.close()


@pytest.mark.parametrize("Z,F", [(64, 5), (1000, 3)])
def test_two_streams_match_one(ldpc, oracle_mod, Z, F):
    """streams=2 runs the frames in two halves on two streams (here 3 + 2 and
    2 + 1 frames); streams=1, and any call with per-pass events, runs them on
    one.  Bits, iteration counts, flags and posteriors agree exactly, FP32 and
    FP16."""
    base = synth.template_base(144, Z, seed=1)
    g = ldpc.Code(base, Z)
    x, Q = synth.biawgn_frames(g.n, F, -13.5, seed=50 + F)
    s = oracle_mod.OracleCode(base, Z).syndrome(x)
    T = 30
    _say("two streams vs one", Z, F)
    for fp16 in (False, True):
        two = _gpu_decode(g, Q, s, T, msg_fp16=fp16, want_llr=True, schedule="launches",
                          streams=2)
        one = _gpu_decode(g, Q, s, T, msg_fp16=fp16, want_llr=True, schedule="launches",
                          streams=1)
        ev = _HipEvents(4 * T)
        timed = _gpu_decode(g, Q, s, T, msg_fp16=fp16, want_llr=True, schedule="launches",
                            timing_events=ev.arr, streams=2)
        ev.close()
        for name, a, b, c in zip(("bits", "iters", "converged", "llr"), two, one, timed):
            assert np.array_equal(a, b), (name, fp16)
            assert np.array_equal(a, c), (name, fp16)


@pytest.mark.parametrize("streams", [1, 2])
def test_repeated_decodes_replay_the_library_graph(ldpc, oracle_mod, streams):
    """A decode repeated with the same sizes, options and pointers is captured
    by the library at its second call and replayed from the third.  Every call
    matches a decode that launches its kernels one by one (graphs=1) on the
    same inputs, also after the inputs behind the same pointers change, FP32
    and FP16.  Graphs serve one-stream decodes; with streams=2 every call
    launches directly, and must match all the same."""
    Z, F, T = 64, 6, 30
    base = synth.template_base(144, Z, seed=1)
    g = ldpc.Code(base, Z)
    o = oracle_mod.OracleCode(base, Z)
    batches = []
    for seed in (71, 72, 73):
        x, Q = synth.biawgn_frames(g.n, F, -13.5, seed=seed)
        batches.append((Q, o.syndrome(x)))
    _say("library graph replay", Z, F, T, streams)
    for fp16 in (False, True):
        dQ, ds = _dev(batches[0][0]), _dev(batches[0][1])
        ws = g.alloc_workspace(F, T, msg_fp16=fp16)
        out = (torch.empty((F, g.n), dtype=torch.uint8, device="cuda"),
               torch.empty(F, dtype=torch.int32, device="cuda"),
               torch.empty(F, dtype=torch.uint8, device="cuda"), None)
        for call, b in enumerate((0, 0, 1, 2, 0)):
            dQ.copy_(_dev(batches[b][0]))
            ds.copy_(_dev(batches[b][1]))
            g.decode(dQ, ds, T, msg_fp16=fp16, workspace=ws, out=out, streams=streams)
            torch.cuda.synchronize()
            got = [t.cpu().numpy() for t in out[:3]]
            ref = _gpu_decode(g, batches[b][0], batches[b][1], T, msg_fp16=fp16, streams=streams,
                              graphs=1)
            for name, u, v in zip(("bits", "iters", "converged"), got, ref[:3]):
                assert np.array_equal(u, v), (name, fp16, call)


def test_library_graphs_evict_and_alternate(ldpc, oracle_mod):
    """The code handle keeps 4 graphs, least recently used replaced.  Five
    calls of different workspaces in turn keep evicting each other (no key
    reaches its second call while cached); then two alternating calls are
    both captured and replayed.  Every output matches direct launches."""
    Z, F, T = 64, 3, 20
    base = synth.template_base(144, Z, seed=1)
    g = ldpc.Code(base, Z)
    o = oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(g.n, F, -13.5, seed=81)
    s = o.syndrome(x)
    dQ, ds = _dev(Q), _dev(s)
    ref = _gpu_decode(g, Q, s, T, graphs=1)
    wss = [g.alloc_workspace(F, T) for _ in range(5)]
    outs = [(torch.empty((F, g.n), dtype=torch.uint8, device="cuda"),
             torch.empty(F, dtype=torch.int32, device="cuda"),
             torch.empty(F, dtype=torch.uint8, device="cuda"), None) for _ in range(5)]
    _say("library graph eviction", Z, F, T)
    order = [0, 1, 2, 3, 4] * 3 + [0, 1] * 4
    for call, k in enumerate(order):
        for t in outs[k][:3]:
            t.fill_(7)
        g.decode(dQ, ds, T, workspace=wss[k], out=outs[k])
        torch.cuda.synchronize()
        for name, u, v in zip(("bits", "iters", "converged"), outs[k][:3], ref[:3]):
            assert np.array_equal(u.cpu().numpy(), v), (name, call, k)


@pytest.mark.parametrize("schedule", ["launches", "resident"])
def test_decode_replays_from_a_captured_graph(ldpc, oracle_mod, schedule):
    """A whole decode (caller-owned workspace and outputs) captured by stream
    capture replays bit-identically, several times, with eager work between
    the replays (the graph holds kernels only: no memset or copy nodes)."""
    Z, F, T = 64, 16, 40
    base = synth.template_base(144, Z, seed=1)
    g = ldpc.Code(base, Z)
    o = oracle_mod.OracleCode(base, Z)
    x, Q = synth.biawgn_frames(g.n, F, -14.0, seed=31)
    s = o.syndrome(x)
    dQ, ds = _dev(Q), _dev(s)
    ws = g.alloc_workspace(F, T)
    out = (torch.empty((F, g.n), dtype=torch.uint8, device="cuda"),
           torch.empty(F, dtype=torch.int32, device="cuda"),
           torch.empty(F, dtype=torch.uint8, device="cuda"), None)
    _say("graph capture", Z, F, T, schedule)
    g.decode(dQ, ds, T, workspace=ws, out=out, schedule=schedule)
    torch.cuda.synchronize()
    ref = [t.cpu().clone() for t in out[:3]]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        g.decode(dQ, ds, T, workspace=ws, out=out, schedule=schedule)
        with torch.cuda.graph(graph, stream=side):
            g.decode(dQ, ds, T, workspace=ws, out=out, schedule=schedule)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in out[:3]:
            t.fill_(7)
        junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a, b in zip(ref, out[:3]):
            assert torch.equal(a, b.cpu()), f"replay {rep}"
    del graph


# ------------------------------------------- full size (n = 1,000,050)
@pytest.fixture(scope="module")
def full_code(ldpc, oracle_mod):
    Z = 6667
    base = synth.template_base(144, Z, seed=1)
    return ldpc.Code(base, Z), oracle_mod.OracleCode(base, Z)


def test_full_size_posterior_after_two_iterations(full_code):
    g, o = full_code
    x, Q = synth.biawgn_frames(o.n, 2, -15.4, seed=1)
    s = o.syndrome(x)
    _say("full size posterior", o.n)
    bits, it, conv, L = _gpu_decode(g, Q, s, 2, early_stop=False, want_llr=True)
    _, L_r, _, _ = o.decode(Q[:1], s[:1], 2, early_stop=False)
    ok, worst, _ = llr_close(L[0], L_r[0])
    assert ok, worst


def test_full_size_bench_configuration_properties(full_code):
    """The benchmark's decode (8 frames, SNR -15.4 dB, 100 iterations, early stop):
    every frame's flag equals H x = s recomputed on the CPU, and counts are in range."""
    g, o = full_code
    F, T = 8, 100
    x, Q = synth.biawgn_frames(o.n, F, -15.4, seed=1)
    s = o.syndrome(x)
    _say("full size bench config", F, T)
    bits, it, conv, _ = _gpu_decode(g, Q, s, T)
    syn = o.syndrome(bits)
    for f in range(F):
        assert bool(conv[f]) == np.array_equal(syn[f], s[f])
        assert 0 <= it[f] <= T
        assert conv[f] or it[f] == T


def test_full_size_converged_frames_match_oracle(full_code):
    g, o = full_code
    F, T = 2, 100
    x, Q = synth.biawgn_frames(o.n, F, -13.8, seed=2)
    s = o.syndrome(x)
    _say("full size converged parity", F, T)
    bits, it, conv, _ = _gpu_decode(g, Q, s, T)
    ref = o.decode(Q, s, T, threads=2)
    summ = check_decode_parity(o, Q, s, bits, it, conv, ref, T)
    print("summary", summ, it, ref[2], flush=True)
    assert summ["both"] >= 1


def test_full_size_posteriors_at_10_20_30_iterations(full_code):
    """n = 1,000,050, one frame at -15.4 dB, early stop off: posteriors of
    every variable within the 1e-3 bound at t = 10, 20 and 30."""
    from concurrent.futures import ThreadPoolExecutor
    g, o = full_code
    x, Q = synth.biawgn_frames(o.n, 1, -15.4, seed=7)
    s = o.syndrome(x)
    Ts = (10, 20, 30)
    _say("full size posteriors", Ts)
    with ThreadPoolExecutor(max_workers=3) as ex:
        refs = list(ex.map(lambda T: o.decode(Q, s, T, early_stop=False)[1], Ts))
    for T, L_r in zip(Ts, refs):
        _, it, _, L = _gpu_decode(g, Q, s, T, early_stop=False, want_llr=True)
        ok, worst, nbad = llr_close(L, L_r)
        print("T", T, "worst err/bound", worst, flush=True)
        assert ok and np.all(it == T), (T, worst, nbad)


def test_full_size_converged_frames_at_threshold_plus_0_3_db(full_code):
    """8 frames of n = 1,000,050 at the template's BP threshold + 0.3 dB
    (-14.5 dB): the full parity contract, and most frames converge."""
    g, o = full_code
    F, T = 8, 100
    x, Q = synth.biawgn_frames(o.n, F, -14.5, seed=3)
    s = o.syndrome(x)
    _say("full size threshold + 0.3 dB", F, T)
    bits, it, conv, _ = _gpu_decode(g, Q, s, T)
    ref = o.decode(Q, s, T, threads=8)
    summ = check_decode_parity(o, Q, s, bits, it, conv, ref, T)
    print("summary", summ, it, ref[2], flush=True)
    assert summ["both"] >= F // 2


@pytest.mark.parametrize("D", [2, 3, 6, 16])
def test_single_check_update_accuracy_over_the_phi_range(ldpc, oracle_mod, D):
    """One iteration of one base row of degree D (every column has degree 1,
    so L_v = Q_v + m_cv): the message m_cv for input magnitudes spanning
    1e-9 .. 40, i.e. both clamps and every branch of the Phi evaluation."""
    rng = np.random.default_rng(1000 + D)
    Z = 4096
    base = rng.integers(0, Z, size=(1, D)).astype(np.int32)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    mag = np.exp(rng.uniform(np.log(1e-9), np.log(40.0), size=(2, o.n)))
    Q = (mag * rng.choice([-1.0, 1.0], size=(2, o.n))).astype(np.float32)
    s = rng.integers(0, 2, size=(2, o.m)).astype(np.uint8)
    _say("single check accuracy", D)
    _, _, _, L = _gpu_decode(g, Q, s, 1, early_stop=False, want_llr=True)
    _, L_r, _, _ = o.decode(Q, s, 1, early_stop=False)
    m_r = L_r - Q.astype(np.float64)
    err = np.abs(L.astype(np.float64) - L_r)
    bound = 1e-5 * np.maximum(np.abs(L_r), np.abs(m_r)) + 1e-30
    assert np.all(err <= bound), float(np.max(err / bound))


def test_tdomain_check_update_accuracy_over_the_phi_range(ldpc, oracle_mod):
    """One iteration of two checks of degree 3, each with two stored inputs
    (columns 0 and 1, of degree 2) and one degree-1 input: the class whose
    update runs in the t-domain.  Input magnitudes span 1e-9 .. 40, i.e. both
    clamps; the messages are held to 1e-5 of max(|L|, 1) (the t-domain keeps
    absolute, not relative, accuracy for tiny messages)."""
    rng = np.random.default_rng(33)
    Z = 4096
    base = np.full((2, 4), -1, dtype=np.int32)
    base[0, [0, 1, 2]] = [rng.integers(0, Z), rng.integers(0, Z), 0]
    base[1, [0, 1, 3]] = [rng.integers(0, Z), rng.integers(0, Z), 0]
    g, o = _codes(ldpc, oracle_mod, base, Z)
    mag = np.exp(rng.uniform(np.log(1e-9), np.log(40.0), size=(2, o.n)))
    Q = (mag * rng.choice([-1.0, 1.0], size=(2, o.n))).astype(np.float32)
    s = rng.integers(0, 2, size=(2, o.m)).astype(np.uint8)
    _say("t-domain check accuracy")
    for T in (1, 2):
        bits, _, _, L = _gpu_decode(g, Q, s, T, early_stop=False, want_llr=True)
        b_r, L_r, _, _ = o.decode(Q, s, T, early_stop=False)
        err = np.abs(L.astype(np.float64) - L_r)
        bound = 1e-5 * np.maximum(np.abs(L_r), 1.0)
        ratio = err / bound
        for f, v in zip(*np.unravel_index(np.argsort(ratio, axis=None)[-5:], ratio.shape)):
            print("T", T, "frame", f, "var", v, "column", v // Z, "Q", Q[f, v], "L", L[f, v],
                  "oracle", L_r[f, v], "err/bound", ratio[f, v], flush=True)
        assert np.all(err <= bound), (T, float(np.max(ratio)))
        sure = np.abs(L_r) > 1e-5 * np.maximum(np.abs(Q), 1.0)
        assert np.array_equal(bits[sure], b_r[sure])


def test_rows_with_several_degree_1_blocks(ldpc, oracle_mod):
    """Checks joined to two degree-1 variables, and a check joined only to
    degree-1 variables, take the generic row path."""
    rng = np.random.default_rng(9)
    Z = 45
    base = np.full((4, 10), -1, dtype=np.int32)
    base[0, [0, 1, 2]] = rng.integers(0, Z, 3)
    base[1, [0, 1, 2, 3]] = rng.integers(0, Z, 4)      # column 3 has degree 1
    base[2, [0, 4, 5]] = rng.integers(0, Z, 3)         # columns 4, 5 have degree 1
    base[3, [6, 7]] = rng.integers(0, Z, 2)            # only degree-1 columns
    g, o = _codes(ldpc, oracle_mod, base, Z)
    x, Q = synth.biawgn_frames(o.n, 3, 1.0, seed=19)
    s = o.syndrome(x)
    _say("several degree-1 blocks per row")
    for T in (1, 3, 8):
        bits, it, conv, L = _gpu_decode(g, Q, s, T, early_stop=False, want_llr=True)
        _, L_r, _, _ = o.decode(Q, s, T, early_stop=False)
        ok, worst, _ = llr_close(L, L_r)
        assert ok, worst
    bits, it, conv, L = _gpu_decode(g, Q, s, 30)
    check_decode_parity(o, Q, s, bits, it, conv, o.decode(Q, s, 30), 30)


@pytest.mark.parametrize("Z", [64, 1000, 2048])
def test_schedule_does_not_change_results(ldpc, oracle_mod, Z):
    """Checks per thread (1, 2, 4) change no output bit, in FP32 and in FP16.

    Without posterior output every check pass runs at the requested checks
    per thread, so the multi-tile update paths of 1 and 2 checks per thread
    are the ones compared here (posterior output always runs 4).  The FP16
    runs meet the oracle: exact flags, bit-exact decisions and iterations
    within +-1 on frames converged on both sides."""
    base = synth.template_base(144, Z, seed=1)
    g, o = _codes(ldpc, oracle_mod, base, Z)
    F, T = 4, 40
    x, Q = synth.biawgn_frames(o.n, F, -13.5, seed=Z)
    s = o.syndrome(x)
    _say("schedules", Z)
    ref = o.decode(Q, s, T, threads=4)
    for fp16 in (False, True):
        base_run = _gpu_decode(g, Q, s, T, checks_per_thread=4, msg_fp16=fp16)
        summ = check_decode_parity(o, Q, s, *base_run[:3], ref, T, fp16=fp16)
        print("fp16" if fp16 else "fp32", "summary", summ, flush=True)
        assert summ["both"] >= 1
        for cpt in (1, 2):
            r = _gpu_decode(g, Q, s, T, checks_per_thread=cpt, msg_fp16=fp16)
            for u, v in zip(r[:3], base_run[:3]):
                assert np.array_equal(u, v), (cpt, fp16)
    # posteriors (these launches run 4 checks per thread whatever is asked)
    r_llr = _gpu_decode(g, Q, s, T, want_llr=True, checks_per_thread=1)
    for u, v in zip(r_llr[:3], _gpu_decode(g, Q, s, T, checks_per_thread=4)[:3]):
        assert np.array_equal(u, v)
    with pytest.raises(ldpc.LdpcError):
        g.decode(_dev(Q), _dev(s), 5, checks_per_thread=3)


@pytest.mark.parametrize("rate,Z", [(0.02, 64), (0.05, 100), (0.1, 7)])
def test_owner_groups_of_the_templates(ldpc, oracle_mod, rate, Z):
    """Every type-2 row (two core blocks, one degree-1 block) owns one core
    block, the 6 core columns own equally many rows, and each column's owned
    rows form groups of at most 12; codes without such rows have none.  The
    relabelling these groups rest on leaves the syndrome of a word unchanged:
    the library's H x equals the oracle's for random words."""
    base = synth.template_for_rate(rate, Z, seed=1)
    g = ldpc.Code(base, Z)
    n_type2 = synth.N_DEG1_FOR_RATE[rate]
    per_col = n_type2 // synth.N_CORE
    assert g.info["owned_edges"] == n_type2 * Z
    assert g.info["owner_groups"] == synth.N_CORE * -(-per_col // 12)
    o = oracle_mod.OracleCode(base, Z)
    x = np.random.default_rng(7).integers(0, 2, size=(3, g.n), dtype=np.uint8)
    s = g.syndrome(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(s, o.syndrome(x))
    # a code with no type-2 rows: every block non-zero, every column of degree 3
    dense = np.random.default_rng(3).integers(0, Z, size=(3, 6)).astype(np.int32)
    info = ldpc.Code(dense, Z).info
    assert info["owner_groups"] == 0 and info["owned_edges"] == 0
