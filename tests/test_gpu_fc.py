"""GPU parity of the FC completion (section 3.1, the linear layers): pimm_fc_complete
adds x1 W + b to the server's share, bit-exact against the oracle, through the C ABI.

Cases: ragged shapes that span several 64 x 64 output tiles and inner splits, a 1 x 1 x 1
product, entries of x1 above 2^l, no bias, the BERT-base QKV product at full size, an
N = 8192 / l = 41 shape, the whole layer on the GPU (Pi_MatMul on x0, decryption, the
completion) against x W + b, and the exactness guard (PIMM_E_ARG for too large weights).
"""
import numpy as np
import pytest
import torch

from paper_2305_18396_amd import pimm, workloads

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU-only machines
    pytest.skip("no HIP device", allow_module_level=True)


def log(msg):
    print(f"[gpu-fc] {msg}", flush=True)


_ctx_cache = {}


def context(N, L, ell, f, rr=True):
    key = (N, L, ell, f, rr)
    if key not in _ctx_cache:
        _ctx_cache[key] = pimm.Context(N, L, ell, f, rerandomize=rr)
    return _ctx_cache[key]


def run_fc(orc, N, L, ell, f, shape, seed, with_bias=True, wrange=3000):
    n, r, m = shape
    log(f"fc N={N} L={L} l={ell} n,r,m={n},{r},{m} bias={with_bias}")
    ctx = context(N, L, ell, f)
    plan = pimm.Plan(ctx, n, r, m)
    rng = np.random.default_rng(seed)
    W = rng.integers(-wrange, wrange, (r, m)).astype(np.int64)
    X1 = rng.integers(0, 1 << 63, (n, r), dtype=np.uint64)
    b = rng.integers(-(1 << 40), 1 << 40, m).astype(np.int64) if with_bias else None
    Y1 = rng.integers(0, 1 << ell, (n, m), dtype=np.uint64)
    w = pimm.Weights(plan, pimm.to_device_u64(W))
    share = pimm.to_device_u64(Y1)
    bias = None if b is None else torch.from_numpy(b).to(ctx.device)
    pimm.fc_complete(plan, w, pimm.to_device_u64(X1), bias, share)
    pimm.sync()
    want = orc.fc_complete(orc.Params(N, L, ell, f), X1, W, b, Y1)
    return pimm.to_host_u64(share), want


@pytest.mark.parametrize("shape", [(37, 100, 70), (1, 1, 1), (130, 257, 65), (64, 64, 64)])
def test_fc_complete_bitexact(orc, shape):
    got, want = run_fc(orc, 4096, 2, 37, 12, shape, seed=sum(shape))
    assert np.array_equal(got, want)


def test_fc_complete_no_bias(orc):
    got, want = run_fc(orc, 4096, 2, 37, 12, (33, 90, 47), seed=5, with_bias=False)
    assert np.array_equal(got, want)


def test_fc_complete_n8192_l41(orc):
    got, want = run_fc(orc, 8192, 3, 41, 14, (70, 520, 300), seed=41)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("shape", [(128, 768, 2304), (128, 3072, 768)])
def test_fc_complete_full_size_bert_base(orc, shape):
    """The QKV and FFN2 products of the BERT-base layer at seq 128, every entry (FFN2's inner
    dimension is split into pieces of two granules per workgroup)."""
    got, want = run_fc(orc, 4096, 2, 37, 12, shape, seed=shape[1], wrange=600)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("rerand", [True, False])
def test_fc_layer_on_gpu(orc, rerand):
    """x = x0 + x1: Pi_MatMul on x0 (encrypt, fused server step, decrypt), then the server's
    completion; the shares add up to x W + b mod 2^l."""
    N, L, ell, f = 4096, 2, 37, 12
    ctx = context(N, L, ell, f, rerand)
    rng = np.random.default_rng(77)
    n, r, m = 40, 200, 90
    log(f"fc layer rr={rerand} n,r,m={n},{r},{m}")
    X = rng.integers(0, 1 << ell, (n, r), dtype=np.uint64)
    X1 = rng.integers(0, 1 << ell, (n, r), dtype=np.uint64)
    X0 = (X - X1) & np.uint64((1 << ell) - 1)
    W = rng.integers(-2000, 2000, (r, m)).astype(np.int64)
    b = rng.integers(-(1 << 30), 1 << 30, m).astype(np.int64)
    plan = pimm.Plan(ctx, n, r, m)
    cseed, sseed = workloads.seed("client", 31), workloads.seed("server", 31)
    sk, pk = pimm.keygen(ctx, cseed)
    ct = pimm.encrypt(plan, sk, cseed, 5, pimm.encode_input(plan, pimm.to_device_u64(X0)))
    w = pimm.Weights(plan, pimm.to_device_u64(W))
    c1, c0s, y1 = pimm.matmul_share(plan, w, pk, sseed, 5, ct)
    y0 = pimm.decrypt(plan, sk, c1, c0s)
    pimm.fc_complete(plan, w, pimm.to_device_u64(X1), torch.from_numpy(b).to(ctx.device), y1)
    pimm.sync()
    Y = (pimm.to_host_u64(y0) + pimm.to_host_u64(y1)) & np.uint64((1 << ell) - 1)
    want = orc.fc_complete(orc.Params(N, L, ell, f), X, W, b, np.zeros((n, m), np.uint64))
    assert np.array_equal(Y, want)


def test_fc_complete_rejects_inexact_weights():
    """At l = 41 the limb split is 21 bits; r * max|W| * (2^21 - 1) >= 2^53 must be refused
    (the reply's noise bound at N = 8192 with three primes still accepts these weights)."""
    ctx = context(8192, 3, 41, 14)
    n, r, m = 4, 8, 8
    plan = pimm.Plan(ctx, n, r, m)
    W = np.zeros((r, m), np.int64)
    W[3, 5] = 1 << 30
    w = pimm.Weights(plan, pimm.to_device_u64(W))
    share = torch.zeros((n, m), dtype=torch.int64, device=ctx.device)
    x1 = torch.zeros((n, r), dtype=torch.int64, device=ctx.device)
    with pytest.raises(pimm.PimmError) as e:
        pimm.fc_complete(plan, w, x1, None, share)
    assert e.value.code == -1
