"""GPU parity of grouped plans (G products of one shape as one set of launches) against the
oracle's grouped run.

- small groups, every buffer bit-exact (encodings, ciphertexts, accumulators before and after
  re-randomisation, reply, both shares) under each of the grouped product's tiles, through the
  two-call and the fused server path, and with the reply switched to fewer primes;
- one phase of the attention cross terms at full size: 24 products of 128x64x128 at N = 8192
  with three primes, the plaintext operand a uniform share; every product's shares add up to
  X_p W_p, and three products' replies and shares are bit-exact against the oracle;
- refusals: the FC completion, batches and the matrix-core schedule do not take grouped plans.
"""
import zlib

import numpy as np
import pytest
import torch

from paper_2305_18396_amd import pimm, workloads

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU-only machines
    pytest.skip("no HIP device", allow_module_level=True)


def log(msg):
    print(f"[gpu-grouped] {msg}", flush=True)


def u64(t):
    return pimm.to_host_u64(t)


_ctx = {}


def context(N, L, ell, f, rr=True):
    key = (N, L, ell, f, rr)
    if key not in _ctx:
        _ctx[key] = pimm.Context(N, L, ell, f, rerandomize=rr)
    return _ctx[key]


def xw_mod(X, W, ell):
    Xu = np.asarray(X, dtype=np.uint64)
    Wu = np.asarray(W, dtype=np.int64).astype(np.uint64)
    return (Xu @ Wu) & np.uint64((1 << ell) - 1)


CASES = {
    "g3_n4096": dict(N=4096, L=2, ell=37, f=12, rr=True, shape=(16, 64, 48), plan={}, G=3),
    "g4_n8192": dict(N=8192, L=3, ell=41, f=14, rr=True, shape=(40, 32, 40), plan={}, G=4),
    "g2_ragged_norr": dict(N=4096, L=2, ell=37, f=12, rr=False, shape=(19, 70, 45),
                           plan=dict(mb=3, rb=5, nb=7), G=2),
    "g5_fix64": dict(N=4096, L=2, ell=37, f=12, rr=True, shape=(33, 100, 70), plan=dict(d_fix=64),
                     G=5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_grouped_bitexact(orc, name):
    c = CASES[name]
    n, r, m = c["shape"]
    N, L, ell, f, G = c["N"], c["L"], c["ell"], c["f"], c["G"]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    Xs = [workloads.share(rng, n, r, ell) for _ in range(G)]
    Ws = [workloads.weights(rng, r, m, f) for _ in range(G)]
    tag = 300 + list(CASES).index(name)
    ctx = context(N, L, ell, f, c["rr"])
    plan = pimm.Plan(ctx, n, r, m, groups=G, **c["plan"])
    assert plan.groups == G and plan.I == G * plan.R * plan.K and plan.O == G * plan.M * plan.K
    log(f"case {name}: plan=({plan.mb},{plan.rb},{plan.nb}) G={G} I={plan.I} O={plan.O}")
    cseed, sseed = workloads.seed("client", tag), workloads.seed("server", tag)
    pyp = orc.Params(N, L, ell, f, rerandomize=c["rr"])
    oplan = orc.Plan(n, r, m, plan.mb, plan.rb, plan.nb, N)
    ref = orc.pi_matmul_grouped(pyp, oplan, Xs, Ws, cseed, sseed, op_id=tag)
    sk, pk = pimm.keygen(ctx, cseed)
    pt = pimm.encode_input(plan, pimm.to_device_u64(np.stack(Xs)))
    ct = pimm.encrypt(plan, sk, cseed, tag, pt)
    ct_in = pimm.encrypt_input(plan, sk, cseed, tag, pimm.to_device_u64(np.stack(Xs)))
    w = pimm.Weights(plan, pimm.to_device_u64(np.stack(Ws).astype(np.int64)))
    pimm.sync()
    assert np.array_equal(u64(pt), ref["pt"])
    assert np.array_equal(u64(ct), ref["ct"])
    assert np.array_equal(u64(ct_in), ref["ct"]), "encrypt_input"
    for tile in ((4, 1, 1), (8, 1, 1), (16, 1, 1)):
        plan.set_tuning(*tile)
        acc = pimm.matmul(plan, w, ct)
        pimm.sync()
        assert np.array_equal(u64(acc), ref["acc"]), tile
        c1, c0s, y1 = pimm.mask_share(plan, pk, sseed, tag, acc)
        pimm.sync()
        assert np.array_equal(u64(acc), ref["acc_rr"]), tile
        assert np.array_equal(u64(c1), ref["c1"]) and np.array_equal(u64(c0s), ref["c0s"]), tile
        assert np.array_equal(u64(y1), ref["Y1"]), tile
        d1, d0s, z1 = pimm.matmul_share(plan, w, pk, sseed, tag, ct)
        y0 = pimm.decrypt(plan, sk, d1, d0s)
        pimm.sync()
        assert torch.equal(d1, c1) and torch.equal(d0s, c0s) and torch.equal(z1, y1), tile
        assert np.array_equal(u64(y0), ref["Y0"]), tile
    Y0, Y1 = u64(y0), u64(y1)
    for k in range(G):
        assert np.array_equal((Y0[k] + Y1[k]) & np.uint64(pyp.t - 1), xw_mod(Xs[k], Ws[k], ell)), k
    if L >= 2:
        c1s, c0ss = pimm.mod_switch(plan, w, d1, d0s)
        y0s = pimm.decrypt_switched(plan, sk, c1s, c0ss)
        pimm.sync()
        assert np.array_equal(u64(c1s), orc.mod_switch(pyp, ref["c1"]))
        assert np.array_equal(u64(y0s), ref["Y0"])


def test_grouped_attention_phase_full_size(orc):
    """24 cross terms of 128x64x128 (12 heads x Q0 K1^T and K0 Q1^T) at N = 8192, three primes,
    t = 2^41; the plaintext operand a uniform share in [-2^40, 2^40)."""
    N, L, ell, f, G = 8192, 3, 41, 14, 24
    n, r, m = 128, 64, 128
    ctx = context(N, L, ell, f)
    rng = np.random.default_rng(20230529)
    half = 1 << (ell - 1)
    Xs = [rng.integers(0, 1 << ell, (n, r), dtype=np.uint64) for _ in range(G)]
    Ws = [rng.integers(-half, half, (r, m), dtype=np.int64) for _ in range(G)]
    plan = pimm.Plan(ctx, n, r, m, groups=G)
    log(f"attention phase: plan=({plan.mb},{plan.rb},{plan.nb}) I={plan.I} O={plan.O}")
    tag = 310
    cseed, sseed = workloads.seed("client", tag), workloads.seed("server", tag)
    sk, pk = pimm.keygen(ctx, cseed)
    ct = pimm.encrypt(plan, sk, cseed, tag, pimm.encode_input(plan, pimm.to_device_u64(np.stack(Xs))))
    w = pimm.Weights(plan, torch.from_numpy(np.stack(Ws)).cuda())
    acc = torch.empty((plan.O, 2, L, N), dtype=torch.int64, device="cuda")
    plan.autotune(w, ct, acc, reps=1)
    c1, c0s, y1 = pimm.matmul_share(plan, w, pk, sseed, tag, ct)
    y0 = pimm.decrypt(plan, sk, c1, c0s)
    pimm.sync()
    Y0, Y1 = u64(y0), u64(y1)
    for k in range(G):
        assert np.array_equal((Y0[k] + Y1[k]) & np.uint64((1 << ell) - 1), xw_mod(Xs[k], Ws[k], ell)), k
    # Three products against the oracle: their ciphertexts, reply and shares.
    pyp = orc.Params(N, L, ell, f)
    oplan = orc.Plan(n, r, m, plan.mb, plan.rb, plan.nb, N)
    s_ref, pk_ref = orc.keygen(pyp, cseed)
    I1, O1 = oplan.I, oplan.O
    pt_ref = np.concatenate([orc.encode_input(oplan, X) for X in Xs])
    ct_host = u64(ct)
    assert np.array_equal(ct_host, orc.encrypt(pyp, s_ref, cseed, tag, pt_ref))
    for k in (0, 11, 23):
        local = np.arange(O1, dtype=np.uint32)
        glob = local + np.uint32(k * O1)
        acc_k = orc.matmul(pyp, oplan, orc.encode_weights(oplan, Ws[k]), ct_host[k * I1:(k + 1) * I1],
                           local)
        acc_k = orc.rerandomize(pyp, pk_ref, sseed, tag, acc_k, glob)
        c1_k, c0s_k, sm_k = orc.mask_extract(pyp, oplan, sseed, tag, acc_k, glob)
        assert np.array_equal(u64(c1[k * O1:(k + 1) * O1]), c1_k), k
        assert np.array_equal(u64(c0s[k * O1:(k + 1) * O1]), c0s_k), k
        assert np.array_equal(Y1[k], orc.place_shares(oplan, sm_k, local)), k
        assert np.array_equal(Y0[k], orc.decrypt(pyp, oplan, s_ref, c1_k, c0s_k, local)), k


def test_grouped_refusals():
    ctx = context(4096, 2, 37, 12)
    plan = pimm.Plan(ctx, 16, 64, 48, groups=3)
    rng = np.random.default_rng(1)
    W = pimm.to_device_u64(np.stack([workloads.weights(rng, 64, 48, 12) for _ in range(3)]))
    w = pimm.Weights(plan, W)
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        plan.set_tuning(8, 2, 1)
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        plan.set_tuning(0, 0, 0)
    x1 = torch.zeros((16, 64), dtype=torch.int64, device="cuda")
    share = torch.zeros((16, 48), dtype=torch.int64, device="cuda")
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        pimm.fc_complete(plan, w, x1, None, share)
    ct = torch.zeros((plan.I, 2, 2, 4096), dtype=torch.int64, device="cuda")
    acc = torch.zeros((plan.O, 2, 2, 4096), dtype=torch.int64, device="cuda")
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        pimm.Batch([(plan, w, ct, acc)])
    single = pimm.Plan(ctx, 16, 64, 48)
    with pytest.raises(pimm.PimmError, match="PIMM_E_ARG"):
        pimm.matmul(single, w, ct[:single.I].contiguous())  # weights of a grouped plan
    with pytest.raises(pimm.PimmError, match="PIMM_E_ARG"):
        pimm.Plan(ctx, 16, 64, 48, groups=0)
    pimm.sync()
