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


@pytest.mark.parametrize("schedule,tile", [(pimm.PHASED, (8, 1)), (pimm.PERSISTENT, (8, 1)),
                                           (pimm.PHASED, (8, 4)), (pimm.PERSISTENT, (4, 2))])
def test_mix_equals_solo_and_xw(stack, orc, schedule, tile):
    ctx, shapes, layers, D, Ws, weights, reqs = stack
    srv = pimm.Server(ctx, layers, shapes, weights, D, 4 << 30, 8, schedule=schedule,
                      mac_rows=tile[0], mac_cols=tile[1])
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
