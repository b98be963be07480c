"""GPU: pimm_matmul_share_noalloc (the fused server step on the library's static
scratch, for callers that cannot allocate) gives the bytes of pimm_matmul_share
with a caller workspace, through the C ABI, on two calls in a row: a
BERT-base-shaped product at sequence 128 (about 105 MiB of scratch), then a
smaller one, so the second call runs on scratch the first one left behind.  A
plan whose scratch exceeds the static size is refused before any work."""
import numpy as np
import pytest
import torch

from paper_2305_18396_amd import pimm, workloads

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def log(msg):
    print(f"[no-alloc] {msg}", flush=True)


def outputs(plan):
    f, c = plan.info, plan.ctx
    return (torch.full((f.O, c.L, c.N), -1, dtype=torch.int64, device="cuda"),
            torch.full((f.O, c.L, f.mb * f.nb), -1, dtype=torch.int64, device="cuda"),
            torch.full((f.n, f.m), -1, dtype=torch.int64, device="cuda"))


def run_pair(ctx, sk, pk, X, W, tag):
    n, r = X.shape
    m = W.shape[1]
    plan = pimm.Plan(ctx, n, r, m)
    cs, ss = workloads.seed("client", 900), workloads.seed("server", tag)
    log(f"product {n}x{r}x{m} plan ({plan.mb},{plan.rb},{plan.nb}) I={plan.I} O={plan.O}")
    ct = pimm.encrypt(plan, sk, cs, tag, pimm.encode_input(plan, pimm.to_device_u64(X)))
    w = pimm.Weights(plan, pimm.to_device_u64(W))
    want = pimm.matmul_share(plan, w, pk, ss, tag, ct)
    got = pimm.matmul_share_noalloc(plan, w, pk, ss, tag, ct, *outputs(plan))
    torch.cuda.synchronize()
    for a, b, name in zip(want, got, ("c1", "c0s", "server share")):
        assert torch.equal(a, b), name
    y0 = pimm.decrypt(plan, sk, got[0], got[1])
    Y = (pimm.to_host_u64(y0) + pimm.to_host_u64(got[2])) & np.uint64((1 << 37) - 1)
    XW = (X @ W.astype(np.uint64)) & np.uint64((1 << 37) - 1)
    assert np.array_equal(Y, XW)


def test_noalloc_equals_workspace_call():
    ctx = pimm.Context(4096, 2, 37, 12, rerandomize=True)
    sk, pk = pimm.keygen(ctx, workloads.seed("client", 900))
    qkv = workloads.bert_base_layer(128)[0]  # 128 x 768 x 2304, the largest scratch
    run_pair(ctx, sk, pk, qkv.X, qkv.W, 901)
    small = workloads.single_matmul()  # 16 x 64 x 64
    run_pair(ctx, sk, pk, small.X, small.W, 902)


def test_noalloc_refuses_plans_beyond_its_scratch():
    ctx = pimm.Context(4096, 2, 37, 12, rerandomize=True)
    sk, pk = pimm.keygen(ctx, workloads.seed("client", 903))
    plan = pimm.Plan(ctx, 512, 768, 2304)  # about 210 MiB of scratch
    w = pimm.Weights(plan, torch.ones((768, 2304), dtype=torch.int64, device="cuda"))
    ct = torch.zeros((plan.I, 2, 2, 4096), dtype=torch.int64, device="cuda")
    with pytest.raises(pimm.PimmError, match="PIMM_E_WORKSPACE"):
        pimm.matmul_share_noalloc(plan, w, pk, workloads.seed("server", 903), 0, ct,
                                  *outputs(plan))
