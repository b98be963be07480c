"""GPU parity of modulus switching of the reply (pimm_mod_switch, pimm_decrypt_switched) against
the oracle's mod_switch and its decryption with the first L - 1 primes.

- uniform residues with planted edge values (the dropped residue at 0, (q-1)/2, (q+1)/2, q-1;
  the kept ones at 0 and q-1), bit-exact for two, three and four primes;
- the whole protocol on small shapes: the switched reply bit-exact and the client's share equal
  to the oracle's and to the unswitched share;
- every product of the BERT-base layer and two of the BERT-large stack at full size, in the
  fused server call the benchmark times: sampled output ciphertexts bit-exact, the whole share
  equal to the unswitched decryption, the shares adding up to X W;
- refusals: one prime, weights whose bound breaks the switched noise rule, overlapping buffers.
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
    print(f"[gpu-switch] {msg}", flush=True)


def u64(t):
    return pimm.to_host_u64(t)


_ctx_cache = {}


def context(N, L, ell, f, rr=True):
    key = (N, L, ell, f, rr)
    if key not in _ctx_cache:
        _ctx_cache[key] = pimm.Context(N, L, ell, f, rerandomize=rr)
    return _ctx_cache[key]


def xw_mod(X, W, ell, rows=None, cols=None):
    Xu = np.asarray(X, dtype=np.uint64)
    Wu = np.asarray(W, dtype=np.int64).astype(np.uint64)
    if rows is None:
        return (Xu @ Wu) & np.uint64((1 << ell) - 1)
    return (Xu[rows] * Wu[:, cols].T).sum(axis=1, dtype=np.uint64) & np.uint64((1 << ell) - 1)


def planted_residues(rng, q, O, count):
    """[O][L][count] uniform residues, with the edge values of the switch planted at the start."""
    L = len(q)
    x = np.stack([rng.integers(0, qq, size=(O, count), dtype=np.uint64) for qq in q], axis=1)
    qd = q[-1]
    edges_d = [0, 1, (qd - 1) // 2, (qd + 1) // 2, qd - 1]
    edges_k = [0, 1, None]  # None: q_l - 1
    k = 0
    for ed in edges_d:
        for ek in edges_k:
            if k >= count:
                break
            x[0, L - 1, k] = ed
            for l in range(L - 1):
                x[0, l, k] = q[l] - 1 if ek is None else ek
            k += 1
    return x


@pytest.mark.parametrize("N,L,ell,f", [(4096, 2, 37, 12), (8192, 3, 41, 14), (4096, 4, 41, 14)])
def test_switch_uniform_residues_bitexact(orc, N, L, ell, f):
    ctx = context(N, L, ell, f)
    n, r, m = 20, 40, 30
    plan = pimm.Plan(ctx, n, r, m)
    rng = np.random.default_rng(N * 10 + L)
    W = workloads.weights(rng, r, m, f)
    w = pimm.Weights(plan, pimm.to_device_u64(W.astype(np.int64)))
    q = [int(v) for v in ctx.primes()]
    per = plan.mb * plan.nb
    log(f"uniform residues N={N} L={L} O={plan.O} per={per}")
    c1 = planted_residues(rng, q, plan.O, N)
    c0s = planted_residues(rng, q, plan.O, per)
    c1s, c0ss = pimm.mod_switch(plan, w, pimm.to_device_u64(c1), pimm.to_device_u64(c0s))
    pimm.sync()
    pyp = orc.Params(N, L, ell, f)
    assert np.array_equal(u64(c1s), orc.mod_switch(pyp, c1))
    assert np.array_equal(u64(c0ss), orc.mod_switch(pyp, c0s))


CASES = {
    "single": dict(N=4096, L=2, ell=37, f=12, rr=True, shape=(16, 64, 64), plan={}),
    "single_norr": dict(N=4096, L=2, ell=37, f=12, rr=False, shape=(16, 64, 64), plan={}),
    "ragged_explicit": dict(N=4096, L=2, ell=37, f=12, rr=True, shape=(19, 70, 45),
                            plan=dict(mb=3, rb=5, nb=7)),
    "fix256": dict(N=4096, L=2, ell=37, f=12, rr=True, shape=(40, 300, 200), plan=dict(d_fix=256)),
    "n8192_l3": dict(N=8192, L=3, ell=41, f=14, rr=True, shape=(33, 100, 70), plan={}),
    "n8192_l3_mfma": dict(N=8192, L=3, ell=41, f=14, rr=True, shape=(96, 64, 330),
                          plan=dict(mb=4, rb=2, nb=8), tuning=(0, 0, 0)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_switched_protocol_bitexact(orc, name):
    c = CASES[name]
    n, r, m = c["shape"]
    N, L, ell, f = c["N"], c["L"], c["ell"], c["f"]
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 7)
    X = workloads.share(rng, n, r, ell)
    W = workloads.weights(rng, r, m, f)
    tag = 200 + list(CASES).index(name)
    ctx = context(N, L, ell, f, c["rr"])
    plan = pimm.Plan(ctx, n, r, m, **c["plan"])
    log(f"case {name}: plan=({plan.mb},{plan.rb},{plan.nb}) O={plan.O}")
    cseed, sseed = workloads.seed("client", tag), workloads.seed("server", tag)
    sk, pk = pimm.keygen(ctx, cseed)
    ct = pimm.encrypt(plan, sk, cseed, tag, pimm.encode_input(plan, pimm.to_device_u64(X)))
    w = pimm.Weights(plan, pimm.to_device_u64(W.astype(np.int64)))
    if "tuning" in c:
        plan.set_tuning(*c["tuning"])
    c1, c0s, y1 = pimm.matmul_share(plan, w, pk, sseed, tag, ct)
    c1s, c0ss = pimm.mod_switch(plan, w, c1, c0s)
    y0s = pimm.decrypt_switched(plan, sk, c1s, c0ss)
    y0 = pimm.decrypt(plan, sk, c1, c0s)
    pimm.sync()
    pyp = orc.Params(N, L, ell, f, rerandomize=c["rr"])
    oplan = orc.Plan(n, r, m, plan.mb, plan.rb, plan.nb, N)
    ref = orc.pi_matmul(pyp, oplan, X, W, cseed, sseed, op_id=tag)
    assert orc.switch_ok(pyp, oplan, int(np.abs(W).max()))
    c1s_ref = orc.mod_switch(pyp, ref["c1"])
    c0ss_ref = orc.mod_switch(pyp, ref["c0s"])
    assert np.array_equal(u64(c1s), c1s_ref)
    assert np.array_equal(u64(c0ss), c0ss_ref)
    y0s_ref = orc.decrypt(orc.switched_params(pyp), oplan, ref["s"], c1s_ref, c0ss_ref, ref["outs"])
    Y0s = u64(y0s)
    assert np.array_equal(Y0s, y0s_ref)
    assert np.array_equal(Y0s, u64(y0))
    assert np.array_equal((Y0s + u64(y1)) & np.uint64((1 << ell) - 1), xw_mod(X, W, ell))


def check_switch_full_size(orc, ctx, pyp, wl, plan_kw, tag):
    """One full-size product through the fused server call under the autotuned schedule, then the
    switch: sampled output ciphertexts bit-exact against the oracle, the whole switched share
    equal to the unswitched one, the shares adding up to X W (all entries, or 4000 sampled)."""
    n, r, m = wl.shape
    plan = pimm.Plan(ctx, n, r, m, **plan_kw)
    oplan = orc.Plan(n, r, m, plan.mb, plan.rb, plan.nb, ctx.N)
    cseed, sseed = workloads.seed("client", tag), workloads.seed("server", tag)
    log(f"full-size {wl.name}: plan=({plan.mb},{plan.rb},{plan.nb}) I={plan.I} O={plan.O}")
    sk, pk = pimm.keygen(ctx, cseed)
    ct = pimm.encrypt(plan, sk, cseed, tag, pimm.encode_input(plan, pimm.to_device_u64(wl.X)))
    w = pimm.Weights(plan, pimm.to_device_u64(wl.W))
    scratch = torch.empty((plan.O, 2, ctx.L, ctx.N), dtype=torch.int64, device="cuda")
    plan.autotune(w, ct, scratch, reps=1)
    del scratch
    log(f"  schedule {plan.tuning()}")
    c1, c0s, y1 = pimm.matmul_share(plan, w, pk, sseed, tag, ct)
    c1s, c0ss = pimm.mod_switch(plan, w, c1, c0s)
    y0s = pimm.decrypt_switched(plan, sk, c1s, c0ss)
    y0 = pimm.decrypt(plan, sk, c1, c0s)
    pimm.sync()
    outs = sorted({0, plan.O // 2, plan.O - 1})
    s_ref, pk_ref = orc.keygen(pyp, cseed)
    ct_ref = orc.encrypt(pyp, s_ref, cseed, tag, orc.encode_input(oplan, wl.X))
    acc_ref = orc.matmul(pyp, oplan, orc.encode_weights(oplan, wl.W), ct_ref, outs)
    acc_rr = orc.rerandomize(pyp, pk_ref, sseed, tag, acc_ref, outs)
    c1_ref, c0s_ref, _ = orc.mask_extract(pyp, oplan, sseed, tag, acc_rr, outs)
    c1s_ref, c0ss_ref = orc.mod_switch(pyp, c1_ref), orc.mod_switch(pyp, c0s_ref)
    assert np.array_equal(u64(c1s[outs]), c1s_ref)
    assert np.array_equal(u64(c0ss[outs]), c0ss_ref)
    y0s_ref = orc.decrypt(orc.switched_params(pyp), oplan, s_ref, c1s_ref, c0ss_ref, outs)
    sel = orc.place_shares(oplan, np.ones((len(outs), plan.mb * plan.nb), np.uint64), outs) == 1
    Y0s = u64(y0s)
    assert np.array_equal(Y0s[sel], y0s_ref[sel])
    assert np.array_equal(Y0s, u64(y0))
    Ysum = (Y0s + u64(y1)) & np.uint64((1 << wl.ell) - 1)
    if n * r * m <= 400_000_000:
        assert np.array_equal(Ysum, xw_mod(wl.X, wl.W, wl.ell))
    else:
        rng = np.random.default_rng(tag)
        rows, cols = rng.integers(0, n, 4000), rng.integers(0, m, 4000)
        assert np.array_equal(Ysum[rows, cols], xw_mod(wl.X, wl.W, wl.ell, rows, cols))
    # The switched reply's bytes: (L - 1) / L of the reply's.
    L = ctx.L
    assert c1s.numel() * 8 * L == plan.info.c1_bytes * (L - 1)
    assert c0ss.numel() * 8 * L == plan.info.c0s_bytes * (L - 1)


def test_full_size_bert_base_layer_switched(orc):
    ctx = context(4096, 2, 37, 12)
    pyp = orc.Params(4096, 2, 37, 12)
    for i, wl in enumerate(workloads.bert_base_layer(128)):
        check_switch_full_size(orc, ctx, pyp, wl, {}, 230 + i)


@pytest.mark.parametrize("op", [0, 2])
def test_full_size_bert_large_op_switched(orc, op):
    ctx = context(8192, 3, 41, 14)
    pyp = orc.Params(8192, 3, 41, 14)
    wl = workloads.bert_large_layer(512)[op]
    check_switch_full_size(orc, ctx, pyp, wl, dict(d_fix=1024), 240 + op)


def test_switch_refusals():
    one = context(4096, 1, 20, 8)
    plan1 = pimm.Plan(one, 8, 24, 16)
    w1 = pimm.Weights(plan1, pimm.to_device_u64(np.ones((24, 16), np.int64)))
    z = torch.zeros((plan1.O, 1, 4096), dtype=torch.int64, device="cuda")
    zs = torch.zeros((plan1.O, 1, plan1.mb * plan1.nb), dtype=torch.int64, device="cuda")
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        pimm.mod_switch(plan1, w1, z, zs, c1_out=z.clone(), c0s_out=zs.clone())
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        sk1, _ = pimm.keygen(one, workloads.seed("client", 1))
        pimm.decrypt_switched(plan1, sk1, z, zs)
    # Two primes, t = 2^37, the BERT-base QKV plan: weights under the reply's noise rule but over
    # the switched one (their bound is stated through pimm_weights_update).
    ctx = context(4096, 2, 37, 12)
    plan = pimm.Plan(ctx, 128, 768, 768)
    info, prm = plan.info, pimm.make_params(4096, 2, 37, 12)
    wmax = 1_000_000
    assert pimm.noise_ok(prm, info, wmax) and not pimm.switch_ok(prm, info, wmax)
    W = np.ones((768, 768), np.int64)
    w = pimm.Weights(plan, pimm.to_device_u64(W))
    c1 = torch.zeros((plan.O, 2, 4096), dtype=torch.int64, device="cuda")
    c0s = torch.zeros((plan.O, 2, plan.mb * plan.nb), dtype=torch.int64, device="cuda")
    pimm.mod_switch(plan, w, c1, c0s)  # small weights: accepted
    w.update(pimm.to_device_u64(W), wmax)
    with pytest.raises(pimm.PimmError, match="PIMM_E_NOISE"):
        pimm.mod_switch(plan, w, c1, c0s)
    w.update(pimm.to_device_u64(W), 1)
    # Outputs that overlap the inputs.
    with pytest.raises(pimm.PimmError, match="PIMM_E_ARG"):
        pimm.mod_switch(plan, w, c1, c0s, c1_out=c1.view(-1)[: plan.O * 4096].view(plan.O, 1, 4096))
    pimm.sync()
