"""The d-dimensional reconciliation front-end (Sec. II-C.3) against the octonion oracle,
and front-end + decoder end to end."""
import numpy as np
import pytest

from oracle import octonion as oc
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


@pytest.mark.parametrize("d", [1, 2, 4, 8])
@pytest.mark.parametrize("n", [1001, 4096])
def test_message_and_llr_match_oracle(ldpc, d, n):
    F, snr = 3, -15.4
    sigma2 = synth.sigma2_from_snr_db(snr)
    c, X, Z = synth.reconciliation_inputs(n, d, F, snr, seed=d + n)
    X32 = X.astype(np.float32)
    Y32 = (X + Z).astype(np.float32)
    _say("front-end", d, n)
    M_gpu = ldpc.reconciliation_message(_dev(c), _dev(Y32), d=d).cpu().numpy()
    M_ref = oc.bob_message(c, Y32.astype(np.float64), d=d)
    # each output coordinate is a signed sum of d products of +-1 and y
    scale = np.repeat(np.sum(np.abs(oc.tuples(Y32.astype(np.float64), d)), axis=-1), d, axis=-1)
    assert np.all(np.abs(M_gpu - M_ref) <= 1e-6 * scale + 1e-30)
    # Alice: LLRs from the oracle's message (rounded to float32) and X
    M32 = M_ref.astype(np.float32)
    L_gpu = ldpc.reconciliation_llr(_dev(X32), _dev(M32), n, sigma2, d=d).cpu().numpy()
    L_ref = oc.alice_llr(M32.astype(np.float64), X32.astype(np.float64), sigma2, n, d=d)
    tup_scale = (np.sqrt(oc.norm2(oc.tuples(M32.astype(np.float64), d)) *
                         oc.norm2(oc.tuples(X32.astype(np.float64), d))) * 2.0 / (d * sigma2))
    bound = 1e-5 * np.repeat(tup_scale, d, axis=-1)[:, :n] + 1e-30
    assert np.all(np.abs(L_gpu - L_ref) <= bound)
    # noiseless: the signs of the LLRs are the key bits
    M0 = ldpc.reconciliation_message(_dev(c), _dev(X32), d=d)
    L0 = ldpc.reconciliation_llr(_dev(X32), M0, n, sigma2, d=d).cpu().numpy()
    assert np.array_equal((L0 < 0).astype(np.uint8), c)


def test_rejects_bad_dimension(ldpc):
    x = torch.zeros((1, 24), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        ldpc.reconciliation_llr(x, x, 30, 1.0, d=8)     # frames must hold 8 * ceil(30 / 8) = 32
    lib = ldpc.load()
    out = torch.empty((1, 24), dtype=torch.float32, device="cuda")
    assert lib.ldpc_reconciliation_llr(3, 1, 24, x.data_ptr(), x.data_ptr(), 1.0,
                                       out.data_ptr(), None) == ldpc.LDPC_EINVAL
    assert lib.ldpc_reconciliation_llr(8, 1, 24, x.data_ptr(), x.data_ptr(), 0.0,
                                       out.data_ptr(), None) == ldpc.LDPC_EINVAL


@pytest.mark.parametrize("fp16", [False, True])
def test_front_end_then_decode(ldpc, oracle_mod, fp16):
    """8-D reconciliation of the n = 9600 template at -13 dB: the GPU chain
    (message, LLRs, decode) against the oracle chain on the same samples."""
    Z, F, T, d, snr = 64, 8, 100, 8, -13.0
    base = synth.template_base(144, Z, seed=1)
    g = ldpc.Code(base, Z)
    o = oracle_mod.OracleCode(base, Z)
    sigma2 = synth.sigma2_from_snr_db(snr)
    c, X, Zn = synth.reconciliation_inputs(o.n, d, F, snr, seed=11)
    X32 = X.astype(np.float32)
    Y32 = (X + Zn).astype(np.float32)
    s = o.syndrome(c)
    _say("front-end + decode", "fp16" if fp16 else "fp32")
    M = ldpc.reconciliation_message(_dev(c), _dev(Y32), d=d)
    L = ldpc.reconciliation_llr(_dev(X32), M, o.n, sigma2, d=d)
    bits, it, conv, _ = g.decode(L, _dev(s), T, msg_fp16=fp16)
    torch.cuda.synchronize()
    bits, it, conv = bits.cpu().numpy(), it.cpu().numpy(), conv.cpu().numpy()
    Q_ref = oc.alice_llr(oc.bob_message(c, Y32.astype(np.float64), d), X32.astype(np.float64),
                         sigma2, o.n, d)
    ref = o.decode(Q_ref, s, T, threads=8)
    if fp16:
        syn = o.syndrome(bits)
        assert all(bool(conv[f]) == np.array_equal(syn[f], s[f]) for f in range(F))
    else:
        summ = check_decode_parity(o, Q_ref, s, bits, it, conv, ref, T)
        print("summary", summ, flush=True)
    assert conv.sum() >= F // 2
    for f in np.nonzero(conv)[0]:
        assert np.array_equal(bits[f], c[f])   # reconciled: Alice holds Bob's key
