"""GPU parity: libpimm (HIP, gfx950) against the CPU oracle, through the C ABI.

All arithmetic is integer, so the bar is bit-exact equality of every buffer that
crosses the ABI (public key, plaintexts, ciphertexts, accumulators, the sparse
reply, both shares), plus the user-level contract Y0 + Y1 = X W (mod 2^l)
against a plain integer matrix product.  Small cases span several blocks with
ragged edges; the full-size cases run every BERT-shaped product of the
benchmarks at its real shape and block plan, under the product schedule the
library's autotuner picks on those buffers (as the benchmarks run them) and
under fixed tiles, through the two-call and the fused server path, and compare
sampled ciphertexts and the decrypted shares with the oracle.
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
    print(f"[gpu-parity] {msg}", flush=True)


def u64(t):
    return pimm.to_host_u64(t)


def xw_mod(X, W, ell):
    Xu = np.asarray(X, dtype=np.uint64)
    Wu = np.asarray(W, dtype=np.int64).astype(np.uint64)
    return (Xu @ Wu) & np.uint64((1 << ell) - 1)


def xw_sampled(X, W, ell, rows, cols):
    Xu = np.asarray(X, dtype=np.uint64)[rows]
    Wu = np.asarray(W, dtype=np.int64).astype(np.uint64)[:, cols].T
    return (Xu * Wu).sum(axis=1, dtype=np.uint64) & np.uint64((1 << ell) - 1)


_ctx_cache = {}


def context(N, L, ell, f, rr):
    key = (N, L, ell, f, rr)
    if key not in _ctx_cache:
        _ctx_cache[key] = pimm.Context(N, L, ell, f, rerandomize=rr)
    return _ctx_cache[key]


def test_context_tables(orc):
    log("context tables")
    for N, L in [(4096, 2), (8192, 3)]:
        ctx = context(N, L, 37, 12, True)
        assert ctx.primes() == orc.find_primes(N, L)
        assert ctx.cdt() == orc.cdt_table()


@pytest.mark.parametrize("kind,tag,prime", [(0, 4, 0), (0, 4, 1), (1, 1, 0), (2, 5, 0), (3, 9, 0)])
def test_samplers_bitexact(orc, kind, tag, prime):
    import ctypes
    log(f"sampler kind={kind} tag={tag} prime={prime}")
    ctx = context(4096, 2, 37, 12, True)
    seed = workloads.seed("client", 77)
    got = u64(pimm.sample_poly(ctx, kind, seed, tag, prime, 1234, 56))
    pyp = orc.Params(4096, 2, 37, 12)
    k = np.frombuffer(seed, np.uint8).copy()
    want = np.zeros(4096, np.uint64 if kind in (0, 3) else np.int64)
    cdt = pyp.cdt_arr
    orc.lib().orc_sample_poly(kind, k.ctypes.data_as(ctypes.c_void_p), tag, prime, 1234, 56, 4096,
                              pyp.q[prime], 37, cdt.ctypes.data_as(ctypes.c_void_p),
                              want.ctypes.data_as(ctypes.c_void_p))
    assert np.array_equal(got, want.view(np.uint64))


def test_uniform_fallback_bitexact(orc):
    """A stream whose draw j the rejection rule refuses (tests/golden/uniform_fallback.json, found
    with the oracle's sampler): the GPU sampler takes the fallback stream there, as the oracle."""
    import ctypes
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "uniform_fallback.json")))
    log(f"uniform fallback at N={g['N']} prime {g['prime']} obj {g['obj']} draw {g['j']}")
    ctx = context(g["N"], g["L"], 41, 14, True)
    assert int(ctx.primes()[g["prime"]]) == g["q"]
    seed = workloads.seed("client", g["request"])
    got = u64(pimm.sample_poly(ctx, 0, seed, g["tag"], g["prime"], g["op"], g["obj"]))
    pyp = orc.Params(g["N"], g["L"], 41, 14)
    k = np.frombuffer(seed, np.uint8).copy()
    want = np.zeros(g["N"], np.uint64)
    orc.lib().orc_sample_poly(0, k.ctypes.data_as(ctypes.c_void_p), g["tag"], g["prime"], g["op"],
                              g["obj"], g["N"], g["q"], 41, pyp.cdt_arr.ctypes.data_as(ctypes.c_void_p),
                              want.ctypes.data_as(ctypes.c_void_p))
    assert int(want[g["j"]]) != g["first_draw_low50"]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("N,L", [(4096, 2), (8192, 3)])
def test_poly_mul_bitexact(orc, N, L):
    import ctypes
    log(f"poly_mul N={N} L={L}")
    ctx = context(N, L, 37, 12, True)
    q = ctx.primes()
    rng = np.random.default_rng(N + L)
    count = 3
    a = np.stack([np.stack([rng.integers(0, ql, N, dtype=np.uint64) for ql in q])
                  for _ in range(count)])
    b = np.stack([np.stack([rng.integers(0, ql, N, dtype=np.uint64) for ql in q])
                  for _ in range(count)])
    b[0, 0] = 0
    b[0, 0, 1] = 1  # x * a: a negacyclic shift
    c, _ = pimm.poly_mul(ctx, pimm.to_device_u64(a), pimm.to_device_u64(b))
    got = u64(c)
    pyp = orc.Params(N, L, 37, 12)
    for i in range(count):
        for l in range(L):
            want = np.zeros(N, np.uint64)
            ai, bi = np.ascontiguousarray(a[i, l]), np.ascontiguousarray(b[i, l])
            orc.lib().orc_negacyclic_mul(ai.ctypes.data_as(ctypes.c_void_p),
                                         bi.ctypes.data_as(ctypes.c_void_p),
                                         want.ctypes.data_as(ctypes.c_void_p), N, pyp.q[l],
                                         pyp.psi[l])
            assert np.array_equal(got[i, l], want), (i, l)
    shifted = np.concatenate([[(q[0] - a[0, 0, -1]) % q[0]], a[0, 0, :-1]]).astype(np.uint64)
    assert np.array_equal(got[0, 0], shifted)


def run_both(orc, N, L, ell, f, rr, X, W, plan_kw, tag, tuning=None):
    """Run the protocol on the GPU and in the oracle; return both sets of buffers."""
    ctx = context(N, L, ell, f, rr)
    n, r = X.shape
    m = W.shape[1]
    plan = pimm.Plan(ctx, n, r, m, **plan_kw)
    if tuning is not None:
        plan.set_tuning(*tuning)
    pyp = orc.Params(N, L, ell, f, rerandomize=rr)
    oplan = orc.Plan(n, r, m, plan.mb, plan.rb, plan.nb, N)
    cseed, sseed = workloads.seed("client", tag), workloads.seed("server", tag)
    log(f"case {tag}: N={N} L={L} l={ell} rr={rr} n,r,m={n},{r},{m} "
        f"plan=({plan.mb},{plan.rb},{plan.nb})")
    sk, pk = pimm.keygen(ctx, cseed)
    Xd, Wd = pimm.to_device_u64(X), pimm.to_device_u64(W.astype(np.int64))
    pt = pimm.encode_input(plan, Xd)
    ct = pimm.encrypt(plan, sk, cseed, tag, pt)
    ct_in = pimm.encrypt_input(plan, sk, cseed, tag, Xd)  # steps 1 and 2 in one pass
    w = pimm.Weights(plan, Wd)
    acc = pimm.matmul(plan, w, ct)
    acc0 = u64(acc).copy()
    c1, c0s, y1 = pimm.mask_share(plan, pk, sseed, tag, acc)
    y0 = pimm.decrypt(plan, sk, c1, c0s)
    pimm.sync()
    gpu = dict(pk=None if pk is None else u64(pk), pt=u64(pt), ct=u64(ct), ct_in=u64(ct_in), acc=acc0,
               acc_rr=u64(acc), c1=u64(c1), c0s=u64(c0s), Y1=u64(y1), Y0=u64(y0))
    ref = orc.pi_matmul(pyp, oplan, X, W, cseed, sseed, op_id=tag)
    return gpu, ref, pyp


CASES = {
    "single": dict(N=4096, L=2, ell=37, f=12, rr=True, shape=(16, 64, 64), plan={}),
    "single_norr": dict(N=4096, L=2, ell=37, f=12, rr=False, shape=(16, 64, 64), plan={}),
    "ragged_explicit": dict(N=4096, L=2, ell=37, f=12, rr=True, shape=(19, 70, 45),
                            plan=dict(mb=3, rb=5, nb=7)),
    "fix256": dict(N=4096, L=2, ell=37, f=12, rr=True, shape=(40, 300, 200),
                   plan=dict(d_fix=256)),
    "n8192_l3": dict(N=8192, L=3, ell=41, f=14, rr=True, shape=(33, 100, 70), plan={}),
    "n4096_l1": dict(N=4096, L=1, ell=20, f=8, rr=True, shape=(8, 24, 16), plan={}),
    "scalar": dict(N=4096, L=2, ell=37, f=12, rr=True, shape=(1, 1, 1), plan={}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_protocol_bitexact(orc, name):
    c = CASES[name]
    n, r, m = c["shape"]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    X = workloads.share(rng, n, r, c["ell"])
    W = workloads.weights(rng, r, m, c["f"])
    tag = 10 + list(CASES).index(name)
    gpu, ref, pyp = run_both(orc, c["N"], c["L"], c["ell"], c["f"], c["rr"], X, W, c["plan"], tag)
    if c["rr"]:
        assert np.array_equal(gpu["pk"], ref["pk"]), "public key"
    for k in ("pt", "ct", "acc", "acc_rr", "c1", "c0s", "Y1", "Y0"):
        want = ref[k].view(np.uint64) if ref[k].dtype != np.uint64 else ref[k]
        assert np.array_equal(gpu[k], want), k
    # pimm_encrypt_input (encoding inside the encryption) gives the oracle's ciphertexts too
    assert np.array_equal(gpu["ct_in"], ref["ct"].view(np.uint64)), "ct of encrypt_input"
    Y = (gpu["Y0"] + gpu["Y1"]) & np.uint64(pyp.t - 1)
    assert np.array_equal(Y, xw_mod(X, W, c["ell"]))


@pytest.mark.parametrize("case", ["zeroW", "zeroX", "identity", "maxX"])
def test_protocol_special_inputs(orc, case):
    n, r, m = 9, 32, 32
    rng = np.random.default_rng(5)
    X = workloads.share(rng, n, r, 37)
    W = workloads.weights(rng, r, m, 12)
    if case == "zeroW":
        W[:] = 0
    elif case == "zeroX":
        X[:] = 0
    elif case == "identity":
        W = np.eye(r, m, dtype=np.int64)
    else:
        X[:] = (1 << 37) - 1
    gpu, ref, pyp = run_both(orc, 4096, 2, 37, 12, True, X, W, {}, 40)
    for k in ("ct", "acc_rr", "c1", "c0s", "Y1", "Y0"):
        assert np.array_equal(gpu[k], ref[k].view(np.uint64)), k
    Y = (gpu["Y0"] + gpu["Y1"]) & np.uint64(pyp.t - 1)
    assert np.array_equal(Y, xw_mod(X, W, 37))


def test_deterministic_and_stream_independent():
    log("determinism")
    ctx = context(4096, 2, 37, 12, True)
    wl = workloads.single_matmul()
    plan = pimm.Plan(ctx, *wl.shape)
    party = pimm.Party(ctx, plan, pimm.to_device_u64(wl.W), workloads.seed("client", 3))
    Xd = pimm.to_device_u64(wl.X)
    a0, a1 = party.run(Xd, workloads.seed("server", 3), op_id=9)
    # Calls in flight must not share a workspace: finish the first run before the
    # same plan's workspace is used from another stream.
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b0, b1 = party.run(Xd, workloads.seed("server", 3), op_id=9, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(a0, b0) and torch.equal(a1, b1)
    c0, _ = party.run(Xd, workloads.seed("server", 3), op_id=10)
    assert not torch.equal(a0, c0)


def test_error_paths():
    log("error paths")
    ctx = context(4096, 2, 37, 12, True)
    plan = pimm.Plan(ctx, 16, 64, 64)
    with pytest.raises(pimm.PimmError, match="PIMM_E_NOISE"):
        pimm.Weights(plan, torch.full((64, 64), 1 << 40, dtype=torch.int64, device="cuda"))
    w = pimm.Weights(plan, torch.ones((64, 64), dtype=torch.int64, device="cuda"))
    ct = torch.zeros((plan.I, 2, 2, 4096), dtype=torch.int64, device="cuda")
    tiny = torch.empty(8, dtype=torch.int64, device="cuda")
    with pytest.raises(pimm.PimmError, match="PIMM_E_WORKSPACE"):
        pimm.matmul(plan, w, ct, ws=tiny)
    other = pimm.Plan(ctx, 16, 64, 64, d_fix=64)
    with pytest.raises(pimm.PimmError, match="PIMM_E_ARG"):
        pimm.matmul(other, w, ct)
    with pytest.raises(pimm.PimmError, match="PIMM_E_ARG"):
        pimm.mask_share(plan, None, workloads.seed("server", 0), 0,
                        torch.zeros((plan.O, 2, 2, 4096), dtype=torch.int64, device="cuda"))


def check_layer_op(orc, ctx, pyp, wl, plan_kw, tag, tunings=(None,), nsample_out=2):
    """One full-size product: the contract on every entry (or a sample) and bit-exact
    ciphertexts / accumulators / reply for sampled output ciphertexts, under each product
    schedule in `tunings` ("auto": the library's autotuner on these buffers, as the benchmark
    runs it; a (rows, cols, waves) tuple; None: the plan's default), through both the two-call
    server path and the fused call the benchmark times."""
    n, r, m = wl.shape
    plan = pimm.Plan(ctx, n, r, m, **plan_kw)
    oplan = orc.Plan(n, r, m, plan.mb, plan.rb, plan.nb, ctx.N)
    cseed, sseed = workloads.seed("client", tag), workloads.seed("server", tag)
    log(f"full-size {wl.name}: plan=({plan.mb},{plan.rb},{plan.nb}) I={plan.I} O={plan.O}")
    sk, pk = pimm.keygen(ctx, cseed)
    s_ref, pk_ref = orc.keygen(pyp, cseed)
    assert np.array_equal(u64(pk), pk_ref)
    Xd = pimm.to_device_u64(wl.X)
    pt = pimm.encode_input(plan, Xd)
    ct = pimm.encrypt(plan, sk, cseed, tag, pt)
    w = pimm.Weights(plan, pimm.to_device_u64(wl.W))
    pimm.sync()
    outs = sorted({0, plan.O // 2, plan.O - 1})[:nsample_out + 1]
    # The oracle's side, once per product: encoding, encryption, the sampled accumulators,
    # re-randomisation, reply and decryption.
    pt_ref = orc.encode_input(oplan, wl.X)
    assert np.array_equal(u64(pt), pt_ref)
    ct_ref = orc.encrypt(pyp, s_ref, cseed, tag, pt_ref)
    assert np.array_equal(u64(ct), ct_ref)
    ptA = orc.encode_weights(oplan, wl.W)
    acc_ref = orc.matmul(pyp, oplan, ptA, ct_ref, outs)
    acc_rr = orc.rerandomize(pyp, pk_ref, sseed, tag, acc_ref, outs)
    c1_ref, c0s_ref, sm_ref = orc.mask_extract(pyp, oplan, sseed, tag, acc_rr, outs)
    y0_ref = orc.decrypt(pyp, oplan, s_ref, c1_ref, c0s_ref, outs)
    sel = orc.place_shares(oplan, np.ones((len(outs), plan.mb * plan.nb), np.uint64), outs) == 1
    t = np.uint64((1 << wl.ell) - 1)
    if n * r * m <= 400_000_000:
        want_sum, pick = xw_mod(wl.X, wl.W, wl.ell), (slice(None), slice(None))
    else:
        rng = np.random.default_rng(tag)
        rows = rng.integers(0, n, 4000)
        cols = rng.integers(0, m, 4000)
        want_sum, pick = xw_sampled(wl.X, wl.W, wl.ell, rows, cols), (rows, cols)
    for tuning in tunings:
        if tuning == "auto":
            scratch = torch.empty((plan.O, 2, ctx.L, ctx.N), dtype=torch.int64, device="cuda")
            plan.autotune(w, ct, scratch, reps=1)
            del scratch
        elif tuning is not None:
            plan.set_tuning(*tuning)
        log(f"  schedule {tuning} -> {plan.tuning()}")
        acc = pimm.matmul(plan, w, ct)
        pimm.sync()
        assert np.array_equal(u64(acc[outs]), acc_ref), plan.tuning()
        c1, c0s, y1 = pimm.mask_share(plan, pk, sseed, tag, acc)
        del acc
        y0 = pimm.decrypt(plan, sk, c1, c0s)
        pimm.sync()
        Y0, Y1 = u64(y0), u64(y1)
        assert np.array_equal(((Y0 + Y1) & t)[pick], want_sum)
        assert np.array_equal(u64(c1[outs]), c1_ref)
        assert np.array_equal(u64(c0s[outs]), c0s_ref)
        assert np.array_equal(Y1, orc.place_shares(oplan, sm_ref, outs, out=Y1.copy()))
        assert np.array_equal(Y0[sel], y0_ref[sel])
        # The fused server call (what the benchmark times) under the same schedule.
        d1, d0s, z1 = pimm.matmul_share(plan, w, pk, sseed, tag, ct)
        pimm.sync()
        assert np.array_equal(u64(d1[outs]), c1_ref), plan.tuning()
        assert np.array_equal(u64(d0s[outs]), c0s_ref), plan.tuning()
        assert torch.equal(d1, c1) and torch.equal(d0s, c0s) and torch.equal(z1, y1)
        del c1, c0s, y1, d1, d0s, z1


@pytest.mark.parametrize("layer_d,tunings", [(0, ("auto", (16, 1, 1), None)), (64, ("auto",)),
                                             (128, ("auto",))])
def test_full_size_bert_base_layer(orc, layer_d, tunings):
    """One BERT-base-shaped layer at sequence 128 (the benchmark's workload): the fewest-wire plan
    under the autotuned schedule the benchmark runs, 16x1 and the plan default; block areas 64
    and 128 (the plans of the block-area sweep) under the autotuned schedule."""
    ctx = context(4096, 2, 37, 12, True)
    pyp = orc.Params(4096, 2, 37, 12)
    for i, wl in enumerate(workloads.bert_base_layer(128)):
        check_layer_op(orc, ctx, pyp, wl, dict(d_fix=layer_d), 100 + i + layer_d, tunings)


@pytest.mark.parametrize("op", range(4))
def test_full_size_bert_large_op(orc, op):
    """Every BERT-large-shaped product of the stack (QKV 1024x3072, attn-out 1024x1024, FFN
    1024x4096 and 4096x1024 at seq 512) with N = 8192, three primes, t = 2^41, blocks of area
    1024: under the autotuned schedule the stack benchmark runs, the column-blocked tiles
    4x8 and 8x4 and the matrix-core product (int8 digit products)."""
    ctx = context(8192, 3, 41, 14, True)
    pyp = orc.Params(8192, 3, 41, 14)
    wl = workloads.bert_large_layer(512)[op]
    check_layer_op(orc, ctx, pyp, wl, dict(d_fix=1024), 200 + op,
                   ("auto", (4, 8, 1), (8, 4, 1), MATRIX_CORES))


# Schedule (0, 0, 0): the slot-wise products on the matrix cores (exact int8 digit products).
MATRIX_CORES = (0, 0, 0)


@pytest.mark.parametrize("name,N,L,ell,f,shape,plan_kw", [
    ("mx_ragged", 4096, 2, 37, 12, (200, 100, 70), dict(d_fix=256)),
    ("mx_r64", 4096, 2, 37, 12, (520, 512, 40), dict(mb=8, rb=8, nb=64)),
    ("mx_n8192", 8192, 3, 41, 14, (300, 96, 200), dict(d_fix=512)),
    ("mx_m80", 4096, 2, 37, 12, (96, 64, 330), dict(mb=4, rb=2, nb=8))])
def test_matrix_core_product_bitexact(orc, name, N, L, ell, f, shape, plan_kw):
    """The matrix-core product (schedule (0, 0, 0)) gives the oracle's accumulators and reply,
    through pimm_matmul and the fused call, with ragged row, column and inner tiles (M, K and R
    not multiples of 16, 8 and 64; more than four row tiles)."""
    n, r, m = shape
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    X = workloads.share(rng, n, r, ell)
    W = workloads.weights(rng, r, m, f)
    ctx = context(N, L, ell, f, True)
    plan = pimm.Plan(ctx, n, r, m, **plan_kw)
    assert plan.R <= 64 and plan.K >= 8, (plan.R, plan.K)
    log(f"matrix cores {name}: plan=({plan.mb},{plan.rb},{plan.nb}) M={plan.M} R={plan.R} "
        f"K={plan.K}")
    gpu, ref, pyp = run_both(orc, N, L, ell, f, True, X, W, plan_kw, 300 + len(name),
                             tuning=MATRIX_CORES)
    for k in ("ct", "acc", "acc_rr", "c1", "c0s", "Y1", "Y0"):
        assert np.array_equal(gpu[k], ref[k].view(np.uint64)), k
    Y = (gpu["Y0"] + gpu["Y1"]) & np.uint64(pyp.t - 1)
    assert np.array_equal(Y, xw_mod(X, W, ell))
    # The fused call under the same schedule gives the same reply.
    cs, ss = workloads.seed("client", 300 + len(name)), workloads.seed("server", 300 + len(name))
    sk, pk = pimm.keygen(ctx, cs)
    ct = pimm.to_device_u64(gpu["ct"])
    w = pimm.Weights(plan, pimm.to_device_u64(W))
    plan.set_tuning(*MATRIX_CORES)
    d1, d0s, z1 = pimm.matmul_share(plan, w, pk, ss, 300 + len(name), ct)
    assert np.array_equal(u64(d1), gpu["c1"]) and np.array_equal(u64(d0s), gpu["c0s"])
    assert np.array_equal(u64(z1), gpu["Y1"])


def test_matrix_core_product_refusals():
    """Plans the matrix-core product does not serve (more than 64 inner blocks, fewer than 8
    column blocks) are refused by pimm_plan_set_tuning; weights made for such a plan have no
    digit form, so a matrix-core call on them is refused too."""
    ctx = context(4096, 2, 37, 12, True)
    wide = pimm.Plan(ctx, 128, 3072, 64, mb=4, rb=2, nb=8)  # R = 1536
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        wide.set_tuning(*MATRIX_CORES)
    narrow = pimm.Plan(ctx, 16, 64, 64)  # K = 1
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        narrow.set_tuning(*MATRIX_CORES)
    small = pimm.Plan(ctx, 4, 32, 64, d_fix=64)  # K = 1 at creation: no digit form
    w = pimm.Weights(small, torch.ones((32, 64), dtype=torch.int64, device="cuda"))
    long = pimm.Plan(ctx, 600, 32, 64, d_fix=64)  # K = 10: eligible, but w has no digits
    long.set_tuning(*MATRIX_CORES)
    ct = torch.zeros((long.I, 2, 2, 4096), dtype=torch.int64, device="cuda")
    with pytest.raises(pimm.PimmError, match="PIMM_E_UNSUPPORTED"):
        pimm.matmul(long, w, ct)


TUNINGS = [(g, kb, wv) for g, kb in [(4, 1), (8, 1), (16, 1), (4, 2), (8, 2), (16, 2), (2, 4),
                                    (4, 4), (8, 4), (2, 8), (4, 8)]
           for wv in (1, 2, 4)]


@pytest.mark.parametrize("name,shape,plan_kw", [
    ("ragged_k3", (19, 70, 45), dict(mb=3, rb=5, nb=7)),
    ("fix256_k3", (40, 300, 200), dict(d_fix=256)),
    ("fix512_k13", (100, 64, 48), dict(d_fix=512)),
    ("comm_k1", (16, 64, 64), {})])
def test_product_schedules_bitexact(orc, name, shape, plan_kw):
    """Every product schedule (rows x column blocks per thread, grid size) gives the
    oracle's accumulators, also with ragged row and column tiles."""
    n, r, m = shape
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    X = workloads.share(rng, n, r, 37)
    W = workloads.weights(rng, r, m, 12)
    ctx = context(4096, 2, 37, 12, True)
    plan = pimm.Plan(ctx, n, r, m, **plan_kw)
    pyp = orc.Params(4096, 2, 37, 12)
    oplan = orc.Plan(n, r, m, plan.mb, plan.rb, plan.nb, 4096)
    cs = workloads.seed("client", 70)
    log(f"schedules {name}: plan=({plan.mb},{plan.rb},{plan.nb}) M={plan.M} R={plan.R} K={plan.K}")
    sk, _ = pimm.keygen(ctx, cs)
    ct = pimm.encrypt(plan, sk, cs, 3, pimm.encode_input(plan, pimm.to_device_u64(X)))
    w = pimm.Weights(plan, pimm.to_device_u64(W))
    s_ref, _ = orc.keygen(pyp, cs)
    ct_ref = orc.encrypt(pyp, s_ref, cs, 3, orc.encode_input(oplan, X))
    assert np.array_equal(u64(ct), ct_ref)
    want = orc.matmul(pyp, oplan, orc.encode_weights(oplan, W), ct_ref, list(range(plan.O)))
    for g, kb, wv in TUNINGS:
        plan.set_tuning(g, kb, wv)
        acc = pimm.matmul(plan, w, ct)
        assert np.array_equal(u64(acc), want), (g, kb, wv)


def test_product_schedules_full_size_bert_large():
    """At the BERT-large FFN2 product (K = 64 column blocks) the column-blocked
    schedules give the bytes of the one-column schedule (which the full-size oracle
    check covers)."""
    ctx = context(8192, 3, 41, 14, True)
    wl = workloads.bert_large_layer(512)[3]
    n, r, m = wl.shape
    plan = pimm.Plan(ctx, n, r, m, d_fix=1024)
    cs = workloads.seed("client", 71)
    sk, _ = pimm.keygen(ctx, cs)
    ct = pimm.encrypt(plan, sk, cs, 1, pimm.encode_input(plan, pimm.to_device_u64(wl.X)))
    w = pimm.Weights(plan, pimm.to_device_u64(wl.W))
    plan.set_tuning(8, 1, 1)
    ref = pimm.matmul(plan, w, ct)
    for g, kb, wv in [(4, 4, 1), (2, 4, 2), (8, 2, 4), (8, 4, 1), (16, 2, 2)]:
        log(f"full-size schedule {g}x{kb} waves {wv}")
        plan.set_tuning(g, kb, wv)
        assert torch.equal(pimm.matmul(plan, w, ct), ref), (g, kb, wv)


@pytest.mark.parametrize("name", ["single", "single_norr", "ragged_explicit", "n8192_l3", "fix256",
                                  "scalar", "n4096_l1"])
def test_fused_server_step_equals_two_calls(orc, name):
    """pimm_matmul_share gives the bytes of pimm_matmul followed by pimm_mask_share."""
    c = CASES[name]
    n, r, m = c["shape"]
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 1)
    X = workloads.share(rng, n, r, c["ell"])
    W = workloads.weights(rng, r, m, c["f"])
    ctx = context(c["N"], c["L"], c["ell"], c["f"], c["rr"])
    plan = pimm.Plan(ctx, n, r, m, **c["plan"])
    log(f"fused {name}")
    cs, ss = workloads.seed("client", 60), workloads.seed("server", 60)
    sk, pk = pimm.keygen(ctx, cs)
    ct = pimm.encrypt(plan, sk, cs, 5, pimm.encode_input(plan, pimm.to_device_u64(X)))
    w = pimm.Weights(plan, pimm.to_device_u64(W))
    c1, c0s, y1 = pimm.mask_share(plan, pk, ss, 5, pimm.matmul(plan, w, ct))
    # Poison the shared workspace: the fused call must write every scratch word
    # before it reads it.
    plan.workspace().fill_(-1)
    d1, d0s, z1 = pimm.matmul_share(plan, w, pk, ss, 5, ct)
    for a, b in [(c1, d1), (c0s, d0s), (y1, z1)]:
        assert torch.equal(a, b)
    Y = (u64(pimm.decrypt(plan, sk, d1, d0s)) + u64(z1)) & np.uint64((1 << c["ell"]) - 1)
    assert np.array_equal(Y, xw_mod(X, W, c["ell"]))


def test_fused_full_size_layer():
    """The benchmark's step (fused server call) at the BERT-base shapes: shares add up to X W,
    and the bytes equal the two-call path."""
    ctx = context(4096, 2, 37, 12, True)
    cs, ss = workloads.seed("client", 61), workloads.seed("server", 61)
    sk, pk = pimm.keygen(ctx, cs)
    for i, wl in enumerate(workloads.bert_base_layer(128)):
        n, r, m = wl.shape
        plan = pimm.Plan(ctx, n, r, m)
        log(f"fused full-size {wl.name}")
        ct = pimm.encrypt(plan, sk, cs, i, pimm.encode_input(plan, pimm.to_device_u64(wl.X)))
        w = pimm.Weights(plan, pimm.to_device_u64(wl.W))
        d1, d0s, z1 = pimm.matmul_share(plan, w, pk, ss, i, ct)
        y0 = pimm.decrypt(plan, sk, d1, d0s)
        Y = (u64(y0) + u64(z1)) & np.uint64((1 << 37) - 1)
        assert np.array_equal(Y, xw_mod(wl.X, wl.W, 37))
        c1, c0s, y1 = pimm.mask_share(plan, pk, ss, i, pimm.matmul(plan, w, ct))
        assert torch.equal(c1, d1) and torch.equal(c0s, d0s) and torch.equal(y1, z1)
