"""GPU parity of the seed-compressed upload (a wire-format variant of Algorithm 1 step 2),
through the C ABI: pimm_encrypt_seeded and pimm_ct_expand bit-exact against the oracle, the
server's rebuilt ciphertexts equal to the client's, and the whole protocol on the GPU with
only c0 and the public seed uploaded.
"""
import numpy as np
import pytest
import torch

from paper_2305_18396_amd import pimm, workloads

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU-only machines
    pytest.skip("no HIP device", allow_module_level=True)


def log(msg):
    print(f"[gpu-seeded] {msg}", flush=True)


@pytest.mark.parametrize("N,L,ell,f", [(4096, 2, 37, 12), (8192, 3, 41, 14)])
def test_encrypt_seeded_and_expand_bitexact(orc, N, L, ell, f):
    log(f"seeded encrypt/expand N={N} L={L}")
    ctx = pimm.Context(N, L, ell, f)
    rng = np.random.default_rng(N + L)
    n, r, m = 40, 300, 50
    plan = pimm.Plan(ctx, n, r, m)
    X = rng.integers(0, 1 << ell, (n, r), dtype=np.uint64)
    cseed, aseed = workloads.seed("client", 40), workloads.seed("public", 40)
    sk, _ = pimm.keygen(ctx, cseed)
    pt = pimm.encode_input(plan, pimm.to_device_u64(X))
    ct = pimm.encrypt_seeded(plan, sk, cseed, aseed, 9, pt)
    c0 = ct[:, 0].contiguous()
    ex = pimm.ct_expand(plan, aseed, 9, c0)
    pimm.sync()
    pyp = orc.Params(N, L, ell, f)
    s_ref, _ = orc.keygen(pyp, cseed)
    want = orc.encrypt_seeded(pyp, s_ref, cseed, aseed, 9, pimm.to_host_u64(pt))
    assert np.array_equal(pimm.to_host_u64(ct), want)
    assert np.array_equal(pimm.to_host_u64(ex), want)
    assert np.array_equal(pimm.to_host_u64(ex),
                          orc.expand_ct(pyp, aseed, 9, np.ascontiguousarray(want[:, 0])))


def test_seeded_equals_plain_with_same_seed():
    ctx = pimm.Context(4096, 2, 37, 12)
    rng = np.random.default_rng(2)
    plan = pimm.Plan(ctx, 16, 64, 64)
    cseed = workloads.seed("client", 41)
    sk, _ = pimm.keygen(ctx, cseed)
    pt = pimm.encode_input(plan, pimm.to_device_u64(rng.integers(0, 1 << 37, (16, 64), dtype=np.uint64)))
    a = pimm.encrypt_seeded(plan, sk, cseed, cseed, 3, pt)
    b = pimm.encrypt(plan, sk, cseed, 3, pt)
    pimm.sync()
    assert torch.equal(a, b)


def test_protocol_with_seeded_upload_on_gpu():
    """Client: encrypt_seeded, upload c0 and the public seed.  Server: expand, fused product
    with mask and reply.  Client: decrypt.  Shares add up to X W mod 2^l."""
    ell = 37
    ctx = pimm.Context(4096, 2, ell, 12)
    rng = np.random.default_rng(42)
    n, r, m = 50, 256, 120
    X = rng.integers(0, 1 << ell, (n, r), dtype=np.uint64)
    W = rng.integers(-2000, 2000, (r, m)).astype(np.int64)
    plan = pimm.Plan(ctx, n, r, m)
    cseed, sseed, aseed = (workloads.seed(k, 42) for k in ("client", "server", "public"))
    sk, pk = pimm.keygen(ctx, cseed)
    ct = pimm.encrypt_seeded(plan, sk, cseed, aseed, 6, pimm.encode_input(plan, pimm.to_device_u64(X)))
    upload = ct[:, 0].contiguous()
    del ct
    ct_srv = pimm.ct_expand(plan, aseed, 6, upload)
    w = pimm.Weights(plan, pimm.to_device_u64(W))
    c1, c0s, y1 = pimm.matmul_share(plan, w, pk, sseed, 6, ct_srv)
    y0 = pimm.decrypt(plan, sk, c1, c0s)
    pimm.sync()
    Y = (pimm.to_host_u64(y0) + pimm.to_host_u64(y1)) & np.uint64((1 << ell) - 1)
    want = (X @ W.astype(np.uint64)) & np.uint64((1 << ell) - 1)
    assert np.array_equal(Y, want)
