"""GPU: many products of uneven length and shape in one pass (pimm_batch_*).

Every item's accumulator must be byte-identical to the same product run alone
through pimm_matmul, under the phased and the persistent schedule and every
tile width; sampled items are also checked against the oracle.  A stream
capture of the batch is replayed as a hipGraph several times, with eager work
in between, and every replay must equal the eager result.
"""
import numpy as np
import pytest
import torch

from paper_2305_18396_amd import pimm, workloads

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def log(msg):
    print(f"[gpu-batch] {msg}", flush=True)


@pytest.fixture(scope="module")
def batch_setup():
    """A batch of the uneven workload's kind: BERT-base shapes, lengths spread over
    [16, 512], fixed block area 32 so one weight cache per shape serves every length."""
    ctx = pimm.Context(4096, 2, 37, 12)
    ws_, items = workloads.batched_uneven(count=10, lo=16, hi=512)
    cseed = workloads.seed("client", 300)
    sk, pk = pimm.keygen(ctx, cseed)
    caches = {}
    rows = []
    for k, it in enumerate(items):
        r, m, W = ws_[it.shape_index]
        plan = pimm.Plan(ctx, it.seq, r, m, d_fix=32)
        key = (r, m)
        if key not in caches:
            caches[key] = pimm.Weights(plan, pimm.to_device_u64(W))
        pt = pimm.encode_input(plan, pimm.to_device_u64(it.X))
        ct = pimm.encrypt(plan, sk, cseed, k, pt)
        solo = pimm.matmul(plan, caches[key], ct)
        acc = torch.zeros_like(solo)
        rows.append((plan, caches[key], ct, acc, solo, it, W))
        log(f"item {k}: seq {it.seq} {r}x{m} plan ({plan.mb},{plan.rb},{plan.nb}) "
            f"I={plan.I} O={plan.O}")
    torch.cuda.synchronize()
    batch = pimm.Batch([(p, w, ct, acc) for p, w, ct, acc, *_ in rows])
    return ctx, batch, rows, sk, pk, cseed


@pytest.mark.parametrize("schedule,rows_per_thread,cols,xcd", [
    (pimm.PHASED, 8, 1, True), (pimm.PHASED, 4, 1, False), (pimm.PHASED, 16, 1, True),
    (pimm.PHASED, 4, 2, True), (pimm.PHASED, 8, 2, True), (pimm.PHASED, 2, 4, True),
    (pimm.PHASED, 4, 4, False), (pimm.PHASED, 8, 4, True), (pimm.PHASED, 16, 2, True),
    (pimm.PHASED, 4, 8, True), (pimm.PHASED, 2, 8, False),
    (pimm.PERSISTENT, 8, 1, True), (pimm.PERSISTENT, 16, 1, False), (pimm.PERSISTENT, 4, 2, True),
    (pimm.PERSISTENT, 4, 4, True), (pimm.PERSISTENT, 2, 4, False), (pimm.PERSISTENT, 8, 4, True)])
def test_batch_equals_solo(batch_setup, schedule, rows_per_thread, cols, xcd):
    ctx, batch, rows, *_ = batch_setup
    log(f"schedule {schedule} tile {rows_per_thread}x{cols} xcd {xcd}")
    for r in rows:
        r[3].zero_()
    batch.set_schedule(schedule, rows_per_thread, cols, xcd, 0)
    batch.run()
    batch.status()
    torch.cuda.synchronize()
    for k, r in enumerate(rows):
        assert torch.equal(r[3], r[4]), f"item {k} differs from its solo run"


def test_batch_persistent_small_grid(batch_setup):
    """A persistent grid far smaller than the device still drains every unit."""
    ctx, batch, rows, *_ = batch_setup
    for r in rows:
        r[3].zero_()
    batch.set_schedule(pimm.PERSISTENT, 4, 2, True, 7)
    batch.run()
    batch.status()
    for k, r in enumerate(rows):
        assert torch.equal(r[3], r[4]), k


def test_batch_item_against_oracle(batch_setup, orc):
    ctx, batch, rows, sk, pk, cseed = batch_setup
    batch.set_schedule(pimm.PHASED, 4, 4, True, 0)
    for r in rows:
        r[3].zero_()
    batch.run()
    torch.cuda.synchronize()
    pyp = orc.Params(4096, 2, 37, 12)
    s_ref, _ = orc.keygen(pyp, cseed)
    for k in (0, len(rows) - 1):
        plan, w, ct, acc, solo, it, W = rows[k]
        oplan = orc.Plan(plan.n, plan.r, plan.m, plan.mb, plan.rb, plan.nb, 4096)
        ct_ref = orc.encrypt(pyp, s_ref, cseed, k, orc.encode_input(oplan, it.X))
        assert np.array_equal(pimm.to_host_u64(ct), ct_ref)
        outs = sorted({0, plan.O - 1})
        want = orc.matmul(pyp, oplan, orc.encode_weights(oplan, W), ct_ref, outs)
        assert np.array_equal(pimm.to_host_u64(acc[outs]), want), k


@pytest.mark.parametrize("schedule", [pimm.PHASED, pimm.PERSISTENT])
def test_batch_graph_replay(batch_setup, schedule):
    """Capture the batch into a hipGraph; replay it three times with eager work and
    synchronisations in between; every replay equals the eager result."""
    ctx, batch, rows, *_ = batch_setup
    batch.set_schedule(schedule, 4, 2, True, 0)
    ws = batch.workspace()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        batch.run(ws=ws, stream=s)
    for rep in range(3):
        for r in rows:
            r[3].fill_(-1)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        batch.status(ws=ws)
        for k, r in enumerate(rows):
            assert torch.equal(r[3], r[4]), f"replay {rep} item {k}"
