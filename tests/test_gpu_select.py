"""GPU: protocol-level plan selection (pimm_plan_select, section 3.1.1's open block split).

The call times the server's step for each candidate block area on this device and picks the
one minimising server time + wire time for the stated link speed.  Checked: the wire bytes it
reports are the plan rule's, every time is positive, the choice is the argmin of the reported
figures, a slow link picks the fewest wire bytes and an unbounded one the shortest server step;
and the protocol at the chosen plan still gives shares that add up to X W.
"""
import numpy as np
import pytest
import torch

from paper_2305_18396_amd import pimm, workloads

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def test_plan_select_picks_the_argmin():
    n, r, m = 128, 768, 768
    ctx = pimm.Context(4096, 2, 37, 12, rerandomize=True)
    rng = np.random.default_rng(31)
    W = workloads.weights(rng, r, m, 12)
    Wd = pimm.to_device_u64(W)
    cands = [0, 64, 256]
    prm = pimm.make_params(4096, 2, 37, 12)
    want_wire = []
    for d in cands:
        f = pimm.plan_rule(prm, n, r, m, d_fix=d)
        want_wire.append(f.ct_bytes + f.c1_bytes + f.c0s_bytes)
    for link in (1e3, 1e11, 1e18):
        best, ms, wire = pimm.plan_select(ctx, n, r, m, Wd, link, cands, reps=2)
        print(f"[select] link {link:.0e} bit/s: d={best} ms={ms} wire={wire}", flush=True)
        assert wire == want_wire
        assert all(t > 0 for t in ms)
        totals = [t + w * 8 / link * 1e3 for t, w in zip(ms, wire)]
        assert best == cands[int(np.argmin(totals))]
        if link == 1e3:
            assert best == cands[int(np.argmin(wire))]
        if link == 1e18:
            assert best == cands[int(np.argmin(ms))]
    # The chosen plan runs the protocol to the right shares.
    plan = pimm.Plan(ctx, n, r, m, d_fix=best)
    cs, ss = workloads.seed("client", 41), workloads.seed("server", 41)
    X = workloads.share(rng, n, r, 37)
    party = pimm.Party(ctx, plan, Wd, cs)
    y0, y1 = party.run(pimm.to_device_u64(X), ss, op_id=3)
    Y = (pimm.to_host_u64(y0) + pimm.to_host_u64(y1)) & np.uint64((1 << 37) - 1)
    assert np.array_equal(Y, (X @ W.astype(np.uint64)) & np.uint64((1 << 37) - 1))


def test_plan_select_rejects_bad_arguments():
    ctx = pimm.Context(4096, 2, 37, 12, rerandomize=True)
    W = torch.ones((64, 64), dtype=torch.int64, device="cuda")
    with pytest.raises(pimm.PimmError, match="PIMM_E_ARG"):
        pimm.plan_select(ctx, 16, 64, 64, W, 0.0, [0])
    with pytest.raises(pimm.PimmError, match="PIMM_E_ARG"):
        pimm.plan_select(ctx, 16, 64, 64, W, 1e9, [])
