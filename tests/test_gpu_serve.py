"""GPU: the continuous-batching server (pimm_serve_*).

A short trace of requests with different prompt lengths runs through a small
layer stack twice: all together (requests admitted while others run, sharing
batched launches) and each alone.  Every request's checksum over its share
pairs must be the same in the mix and alone, and its checksum over the share
sums must equal the one recomputed on the host from X W (X regenerated with the
oracle's ChaCha20 sampler from the documented stream).  A budget that holds
only two requests at a time must still drain the whole trace.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2305_18396_amd import pimm, workloads

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

M64 = (1 << 64) - 1


def mix64(z):
    z = (z + 0x9e3779b97f4a7c15) & M64
    z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & M64
    z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & M64
    return z ^ (z >> 31)


@pytest.fixture(scope="module")
def stack():
    ctx = pimm.Context(4096, 2, 37, 12)
    rng = np.random.default_rng(21)
    shapes = [(768, 256), (256, 768)]
    layers, D = 2, 32
    Ws, weights = [], []
    for _ in range(layers):
        for r, m in shapes:
            W = workloads.weights(rng, r, m, 12)
            plan = pimm.Plan(ctx, 1, r, m, d_fix=D)
            Ws.append(W)
            weights.append(pimm.Weights(plan, pimm.to_device_u64(W)))
    reqs = [(i, s, 0.002 * i, workloads.seed("client", 500 + i), workloads.seed("server", 500 + i))
            for i, s in enumerate([32, 97, 300, 45, 180, 64])]
    return ctx, shapes, layers, D, Ws, weights, reqs


@pytest.mark.parametrize("schedule,tile,min_batch", [
    (pimm.PHASED, (8, 1), 2), (pimm.PERSISTENT, (8, 1), 2), (pimm.PHASED, (8, 4), 2),
    (pimm.PERSISTENT, (4, 2), 2), (pimm.PHASED, (4, 8), 0)])
def test_mix_equals_solo_and_xw(stack, orc, schedule, tile, min_batch):
    """min_batch 2: every step with two or more requests takes the batched pass; 0: the
    server's default (eight)."""
    ctx, shapes, layers, D, Ws, weights, reqs = stack
    srv = pimm.Server(ctx, layers, shapes, weights, D, 4 << 30, 8, schedule=schedule,
                      mac_rows=tile[0], mac_cols=tile[1], min_batch=min_batch)
    mix = srv.run(reqs)
    for rq, res in zip(reqs, mix):
        assert res["steps"] == layers * len(shapes)
        assert res["admit_s"] >= res["arrival_s"] - 1e-9 and res["done_s"] >= res["admit_s"]
        solo = srv.run([rq])[0]
        assert solo["pair_checksum"] == res["pair_checksum"], rq[0]
        assert solo["sum_checksum"] == res["sum_checksum"], rq[0]
    # The share sums are X W for every product of one request.
    rid, seq, _, cs, _ = reqs[1]
    tot = 0
    for k in range(layers * len(shapes)):
        r, m = shapes[k % len(shapes)]
        X = np.zeros(seq * r, np.uint64)
        key = np.frombuffer(cs, np.uint8).copy()
        orc.lib().orc_sample_poly(3, key.ctypes.data_as(ctypes.c_void_p), 10, 0, k, rid, seq * r, 0,
                                  37, None, X.ctypes.data_as(ctypes.c_void_p))
        Y = (X.reshape(seq, r) @ Ws[k].astype(np.uint64)) & np.uint64((1 << 37) - 1)
        for i, v in enumerate(Y.reshape(-1).tolist()):
            tot = (tot + mix64(v ^ mix64((k << 40) ^ i))) & M64
    assert tot == mix[1]["sum_checksum"]


def test_small_budget_drains(stack):
    ctx, shapes, layers, D, Ws, weights, reqs = stack
    srv = pimm.Server(ctx, layers, shapes, weights, D, 1 << 30, 8)
    fp = max(srv.footprint(s) for _, s, *_ in reqs)
    budget = 2 * fp + (64 << 20)
    small = pimm.Server(ctx, layers, shapes, weights, D, budget, 8)
    res = small.run(reqs)
    full = srv.run(reqs)
    for a, b in zip(res, full):
        assert a["pair_checksum"] == b["pair_checksum"]
    # With room for about two requests, later arrivals wait for admission.
    assert max(r["admit_s"] - r["arrival_s"] for r in res) > 0


def mix64_np(z):
    """The checksum's SplitMix64 finaliser over uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, np.uint64) + np.uint64(0x9e3779b97f4a7c15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xbf58476d1ce4e5b9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94d049bb133111eb)
    return z ^ (z >> np.uint64(31))


def oracle_pair_checksum(orc, pyp, D, shapes, Ws, rid, seq, cs, ss):
    """The request's pair checksum recomputed from the oracle's own Pi_MatMul of every product
    of its stack: X drawn from the documented stream (tag 10, op id = product step, object =
    request id), the block plan of area D at the request's length, op id = product step."""
    keys = orc.keygen(pyp, cs)
    key = np.frombuffer(cs, np.uint8).copy()
    tot = 0
    for k, W in enumerate(Ws):
        r, m = shapes[k % len(shapes)]
        X = np.zeros(seq * r, np.uint64)
        orc.lib().orc_sample_poly(3, key.ctypes.data_as(ctypes.c_void_p), 10, 0, k, rid, seq * r,
                                  0, pyp.ell, None, X.ctypes.data_as(ctypes.c_void_p))
        plan = orc.plan_fix(pyp.N, D, seq, r, m)
        ref = orc.pi_matmul(pyp, plan, X.reshape(seq, r), W, cs, ss, op_id=k, keys=keys)
        Y0, Y1 = ref["Y0"].reshape(-1), ref["Y1"].reshape(-1)
        salt = (np.uint64(k) << np.uint64(40)) ^ np.arange(Y0.size, dtype=np.uint64)
        tot = (tot + int(mix64_np(Y0 ^ mix64_np(Y1 ^ salt)).sum(dtype=np.uint64))) & M64
    return tot


@pytest.mark.parametrize("D,ops", [(128, (0, 1, 2, 3)), (32, (1,))])
def test_served_shares_equal_the_oracle(orc, D, ops):
    """A request served in a mix of three, on BERT-base-shaped products (QKV 768x2304, attn-out
    768x768, FFN 768x3072 and 3072x768; N = 4096, two primes, t = 2^37) with weight caches of
    block area D: its checksum over the (client, server) share pairs of every product equals
    the one recomputed from the oracle's Pi_MatMul of the same products (same seeds, op ids and
    block plans).  Block area 128 runs the whole layer; block area 32 (the serving benchmark's
    default) the attention-output product, which keeps the oracle's share of the test short."""
    ctx = pimm.Context(4096, 2, 37, 12)
    shapes = [(r, m) for _, r, m in (workloads.BERT_BASE_SHAPES[o] for o in ops)]
    rng = np.random.default_rng(23 + D)
    Ws, weights = [], []
    for r, m in shapes:
        W = workloads.weights(rng, r, m, 12)
        Ws.append(W)
        weights.append(pimm.Weights(pimm.Plan(ctx, 1, r, m, d_fix=D), pimm.to_device_u64(W)))
    reqs = [(700 + i, s, 0.001 * i, workloads.seed("client", 700 + i),
             workloads.seed("server", 700 + i)) for i, s in enumerate([32, 77, 45])]
    srv = pimm.Server(ctx, 1, shapes, weights, D, 8 << 30, 8, schedule=pimm.PHASED,
                      mac_rows=8, mac_cols=4, min_batch=2)
    res = srv.run(reqs)
    pyp = orc.Params(4096, 2, 37, 12)
    for i in (0, 2):
        rid, seq, _, cs, ss = reqs[i]
        assert res[i]["steps"] == len(shapes)
        want = oracle_pair_checksum(orc, pyp, D, shapes, Ws, rid, seq, cs, ss)
        assert res[i]["pair_checksum"] == want, (D, rid, seq)
