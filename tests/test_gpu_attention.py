"""GPU parity of the attention cross terms (Eq. 2, section 3.1): Pi_MatMul with the server's
uniform share as the plaintext operand, at N = 8192 with three primes and t = 2^41, through
the C ABI.  Per-head shapes of a BERT-base layer at seq 128 (head dimension 64): the two
score cross terms (128 x 64 x 128) and the two value cross terms (128 x 128 x 64 and
64 x 128 x 128).  Every buffer of sampled output ciphertexts bit-exact against the oracle, and
the shares of every product add up to X0 W1 mod 2^l.
"""
import numpy as np
import pytest
import torch

from paper_2305_18396_amd import pimm, workloads

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU-only machines
    pytest.skip("no HIP device", allow_module_level=True)

ELL = 41
_ctx = {}


def log(msg):
    print(f"[gpu-attention] {msg}", flush=True)


def context():
    if "c" not in _ctx:
        _ctx["c"] = pimm.Context(8192, 3, ELL, 14, rerandomize=True)
    return _ctx["c"]


def centred(u):
    v = u.astype(np.int64)
    return np.where(u >= np.uint64(1 << (ELL - 1)), v - (1 << ELL), v).astype(np.int64)


@pytest.mark.parametrize("shape", [(128, 64, 128), (128, 128, 64), (64, 128, 128)])
def test_cross_term_full_head(orc, shape):
    n, r, m = shape
    log(f"cross term n,r,m={shape}")
    ctx = context()
    rng = np.random.default_rng(sum(shape) + 7)
    X0 = rng.integers(0, 1 << ELL, (n, r), dtype=np.uint64)
    W1 = rng.integers(0, 1 << ELL, (r, m), dtype=np.uint64)
    Wc = centred(W1)
    plan = pimm.Plan(ctx, n, r, m)
    tag = 70 + n + r
    cseed, sseed = workloads.seed("client", tag), workloads.seed("server", tag)
    sk, pk = pimm.keygen(ctx, cseed)
    ct = pimm.encrypt(plan, sk, cseed, tag, pimm.encode_input(plan, pimm.to_device_u64(X0)))
    w = pimm.Weights(plan, pimm.to_device_u64(Wc))
    c1, c0s, y1 = pimm.matmul_share(plan, w, pk, sseed, tag, ct)
    y0 = pimm.decrypt(plan, sk, c1, c0s)
    pimm.sync()
    Y = (pimm.to_host_u64(y0) + pimm.to_host_u64(y1)) & np.uint64((1 << ELL) - 1)
    Xo, Wo = X0.astype(object), W1.astype(object)
    want = np.array(Xo.dot(Wo) % (1 << ELL), dtype=np.uint64)
    assert np.array_equal(Y, want)
    # Sampled output ciphertexts against the oracle.
    pyp = orc.Params(8192, 3, ELL, 14, rerandomize=True)
    oplan = orc.Plan(n, r, m, plan.mb, plan.rb, plan.nb, 8192)
    outs = np.unique(np.array([0, plan.O // 2, plan.O - 1], dtype=np.uint32))
    ref = orc.pi_matmul(pyp, oplan, X0, Wc, cseed, sseed, op_id=tag, outs=outs)
    assert np.array_equal(pimm.to_host_u64(c1)[outs], ref["c1"])
    assert np.array_equal(pimm.to_host_u64(c0s)[outs], ref["c0s"])


def test_weights_update_changes_operand(orc):
    """A weight cache re-encoded in place with the next share: the product follows the new
    operand, and the bounds are checked on the stated wmax."""
    ctx = context()
    n, r, m = 128, 64, 128
    rng = np.random.default_rng(90)
    X0 = rng.integers(0, 1 << ELL, (n, r), dtype=np.uint64)
    Wa = rng.integers(0, 1 << ELL, (r, m), dtype=np.uint64)
    Wb = rng.integers(0, 1 << ELL, (r, m), dtype=np.uint64)
    plan = pimm.Plan(ctx, n, r, m)
    cseed, sseed = workloads.seed("client", 90), workloads.seed("server", 90)
    sk, pk = pimm.keygen(ctx, cseed)
    ct = pimm.encrypt(plan, sk, cseed, 1, pimm.encode_input(plan, pimm.to_device_u64(X0)))
    w = pimm.Weights(plan, pimm.to_device_u64(centred(Wa)))
    w.update(pimm.to_device_u64(centred(Wb)), 1 << (ELL - 1))
    c1, c0s, y1 = pimm.matmul_share(plan, w, pk, sseed, 1, ct)
    y0 = pimm.decrypt(plan, sk, c1, c0s)
    pimm.sync()
    Y = (pimm.to_host_u64(y0) + pimm.to_host_u64(y1)) & np.uint64((1 << ELL) - 1)
    assert np.array_equal(Y, np.array(X0.astype(object).dot(Wb.astype(object)) % (1 << ELL),
                                      dtype=np.uint64))
    with pytest.raises(pimm.PimmError) as e:
        w.update(pimm.to_device_u64(centred(Wb)), 1 << 49)
    assert e.value.code == -1
    small = pimm.Context(4096, 2, 37, 12)
    p2 = pimm.Plan(small, n, r, m)
    w2 = pimm.Weights(p2, torch.zeros((r, m), dtype=torch.int64, device=small.device))
    with pytest.raises(pimm.PimmError) as e:
        w2.update(torch.zeros((r, m), dtype=torch.int64, device=small.device), 1 << 36)
    assert e.value.code == -4


def test_cross_terms_over_streams_match_stream_order():
    """Independent cross terms issued over several streams give the same shares as in stream
    order (each product has its own buffers and workspace; the key material is shared)."""
    ctx = context()
    rng = np.random.default_rng(95)
    cseed, sseed = workloads.seed("client", 95), workloads.seed("server", 95)
    sk, pk = pimm.keygen(ctx, cseed)
    half = 1 << (ELL - 1)
    items = []
    for t, (n, r, m) in enumerate([(128, 64, 128), (128, 64, 128), (128, 128, 64), (64, 128, 128)]):
        plan = pimm.Plan(ctx, n, r, m)
        X = pimm.to_device_u64(rng.integers(0, 1 << ELL, (n, r), dtype=np.uint64))
        W = torch.from_numpy(rng.integers(-half, half, (r, m), dtype=np.int64)).to(ctx.device)
        items.append(dict(plan=plan, X=X, W=W, w=pimm.Weights(plan, W), ws=plan.workspace(), op=t))

    def run(streams):
        out = []
        for it in items:
            q = streams[it["op"] % len(streams)] if streams else None
            if q is not None:
                q.wait_stream(torch.cuda.current_stream())
            p = it["plan"]
            with torch.cuda.stream(q) if q is not None else torch.cuda.stream(torch.cuda.current_stream()):
                ct = pimm.encrypt(p, sk, cseed, it["op"], pimm.encode_input(p, it["X"]), ws=it["ws"])
                it["w"].update(it["W"], half)
                c1, c0s, y1 = pimm.matmul_share(p, it["w"], pk, sseed, it["op"], ct, ws=it["ws"])
                y0 = pimm.decrypt(p, sk, c1, c0s, ws=it["ws"])
            out.append((y0, y1))
        torch.cuda.synchronize()
        return [(pimm.to_host_u64(a), pimm.to_host_u64(b)) for a, b in out]

    serial = run(None)
    parallel = run([torch.cuda.Stream() for _ in range(3)])
    for (a0, a1), (b0, b1) in zip(serial, parallel):
        assert np.array_equal(a0, b0) and np.array_equal(a1, b1)
