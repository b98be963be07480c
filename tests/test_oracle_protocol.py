"""Pins of the oracle's encodings and protocol steps.

- the hand-worked example of Algorithm 1 (tests/golden) for the encodings;
- the plaintext identity pi_C^{-1}(pi_A(A) * pi_B(B)) = AB mod t by Python
  schoolbook multiplication, with mrn = N and with ragged blocks;
- Dec(Enc(m)) = m, Enc(0) -> 0, the exact fresh noise within the Gaussian's cut;
- Dec(a * Enc(b)) = a * b mod (X^N + 1, t) by Python schoolbook;
- the user-level contract Y0 + Y1 = X W (mod 2^l) against a plain numpy integer
  matrix product, for the small-config shapes, special cases (W = I, W = 0,
  X = 0, n = m = r = 1), several plans, with and without re-randomisation;
- the sparse reply (section 3.1.3): decrypting from the kept c0 coefficients
  gives what decrypting the whole masked ciphertext gives;
- the measured noise stays under the analytic bound.
"""
import json
import os

import numpy as np
import pytest

from paper_2305_18396_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def py_negacyclic_int(a, b):
    n = len(a)
    c = [0] * n
    for i in range(n):
        if a[i] == 0:
            continue
        for j in range(n):
            if i + j < n:
                c[i + j] += a[i] * b[j]
            else:
                c[i + j - n] -= a[i] * b[j]
    return c


def xw_mod(X, W, ell):
    """Plain integer product X W mod 2^ell (uint64 wrap-around is exact mod 2^ell)."""
    Xu = np.asarray(X, dtype=np.uint64)
    Wu = np.asarray(W, dtype=np.int64).astype(np.uint64)
    return (Xu @ Wu) & np.uint64((1 << ell) - 1)


def test_alg1_worked_example(orc):
    g = json.load(open(os.path.join(GOLDEN, "alg1_worked_example.json")))
    A, B = np.array(g["A"]), np.array(g["B"])
    W, X = A.T.copy(), B.T.copy()  # the server holds A = W^T, the client B = X^T
    plan = orc.Plan(n=2, r=2, m=2, mb=2, rb=2, nb=2, N=8)
    pa = orc.encode_weights(plan, W)[0].tolist()
    pb = orc.encode_input(plan, X)[0].tolist()
    assert pa == g["a_poly"] and pb == g["b_poly"]
    for ij, e in g["exp_a"].items():
        if ij != "comment":
            assert pa[e] == A[int(ij[0]), int(ij[1])]
    for jk, e in g["exp_b"].items():
        if jk != "comment":
            assert pb[e] == B[int(jk[0]), int(jk[1])]
    c = py_negacyclic_int(pa, pb)
    for ik, pos in g["pos_c"].items():
        if ik != "comment":
            i, k = int(ik[0]), int(ik[1])
            assert plan.pos(i, k) == pos and c[pos] == g["AB"][i][k]


@pytest.mark.parametrize("shape", [(2, 2, 2, 8), (4, 4, 4, 64), (3, 5, 2, 32), (1, 1, 1, 2),
                                   (8, 4, 2, 64), (2, 16, 2, 64)])
def test_encoding_identity_single_block(orc, shape):
    """m r n <= N: decoding the integer product gives AB exactly (also at mrn = N)."""
    m, r, n, N = shape
    rng = np.random.default_rng(sum(shape))
    W = rng.integers(-50, 50, (r, m))
    X = rng.integers(0, 1000, (n, r))
    plan = orc.Plan(n=n, r=r, m=m, mb=m, rb=r, nb=n, N=N)
    c = py_negacyclic_int(orc.encode_weights(plan, W)[0].tolist(),
                          orc.encode_input(plan, X)[0].tolist())
    Y = X @ W
    for k in range(n):
        for i in range(m):
            assert c[plan.pos(i, k)] == Y[k, i]


def test_encoding_identity_blocked_ragged(orc):
    """Blocks with padding: sum over inner blocks of the block products decodes to XW."""
    rng = np.random.default_rng(3)
    n, r, m, N = 5, 7, 6, 32
    W = rng.integers(-9, 9, (r, m))
    X = rng.integers(0, 99, (n, r))
    plan = orc.Plan(n=n, r=r, m=m, mb=4, rb=2, nb=3, N=N)  # 24 <= 32, ragged everywhere
    pa, pb = orc.encode_weights(plan, W), orc.encode_input(plan, X)
    Y = X @ W
    got = np.full((n, m), -10**9)
    for ib in range(plan.M):
        for kb in range(plan.K):
            acc = [0] * N
            for jb in range(plan.R):
                p = py_negacyclic_int(pa[ib * plan.R + jb].tolist(), pb[jb * plan.K + kb].tolist())
                acc = [u + v for u, v in zip(acc, p)]
            for k in range(plan.nb):
                for i in range(plan.mb):
                    row, col = kb * plan.nb + k, ib * plan.mb + i
                    if row < n and col < m:
                        got[row, col] = acc[plan.pos(i, k)]
    assert np.array_equal(got, Y)


@pytest.fixture(scope="module")
def small_params(orc):
    return orc.Params(64, 2, 20, 8)


def test_encrypt_decrypt_roundtrip(orc, small_params):
    p = small_params
    s, _ = orc.keygen(p, workloads.seed("client", 1), with_pk=False)
    rng = np.random.default_rng(0)
    pt = rng.integers(0, p.t, (3, p.N), dtype=np.uint64)
    ct = orc.encrypt(p, s, workloads.seed("client", 1), 7, pt)
    assert np.array_equal(orc.decrypt_full(p, s, ct, query=True), pt)
    assert ct.max() < max(p.q)
    for l, q in enumerate(p.q):
        assert ct[:, :, l].max() < q
    zero = orc.encrypt(p, s, workloads.seed("client", 1), 8, np.zeros((2, p.N), np.uint64))
    assert not np.any(orc.decrypt_full(p, s, zero, query=True))
    # Fresh noise is exactly the Gaussian error: |e| <= 19.
    assert 0 < orc.noise_of(p, s, ct, pt, query=True) <= 19
    assert np.all(np.isin(s, [-1, 0, 1]))


def test_encrypt_is_deterministic_in_seed_and_op(orc, small_params):
    p = small_params
    s, _ = orc.keygen(p, workloads.seed("client", 2), with_pk=False)
    pt = np.ones((1, p.N), np.uint64)
    a = orc.encrypt(p, s, workloads.seed("client", 2), 1, pt)
    b = orc.encrypt(p, s, workloads.seed("client", 2), 1, pt)
    c = orc.encrypt(p, s, workloads.seed("client", 2), 2, pt)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_ctpt_product_decrypts_to_plain_product(orc, small_params):
    """Dec(a * Enc(b)) = a * b in Z_t[X]/(X^N + 1)."""
    p = small_params
    s, _ = orc.keygen(p, workloads.seed("client", 3), with_pk=False)
    rng = np.random.default_rng(5)
    b = rng.integers(0, p.t, p.N)
    a = np.zeros(p.N, np.int64)
    a[:6] = rng.integers(-100, 100, 6)  # a small plaintext like pi_A(W)
    ct = orc.encrypt(p, s, workloads.seed("client", 3), 0, b[None].astype(np.uint64))
    plan = orc.Plan(n=1, r=1, m=1, mb=1, rb=1, nb=1, N=p.N)  # one block, R = K = 1
    acc = orc.matmul(p, plan, a[None], ct, [0])
    want = [v % p.t for v in py_negacyclic_int(a.tolist(), b.tolist())]
    assert orc.decrypt_full(p, s, acc)[0].tolist() == want


def run_protocol(orc, p, plan, X, W, tag=0):
    res = orc.pi_matmul(p, plan, X, W, workloads.seed("client", tag),
                        workloads.seed("server", tag), op_id=tag)
    return res


@pytest.mark.parametrize("rerand", [True, False])
def test_protocol_config_small_matrix(orc, rerand):
    """The small single-matrix workload (X 16x64 share in Z_{2^37}, W 64x64 with 12 fractional
    bits, N = 4096, two primes), communication-optimal plan (16, 16, 16)."""
    wl = workloads.single_matmul()
    p = orc.Params(4096, 2, 37, 12, rerandomize=rerand)
    plan = orc.plan_comm(4096, *wl.shape)
    assert (plan.mb, plan.rb, plan.nb) == (16, 16, 16)
    res = run_protocol(orc, p, plan, wl.X, wl.W, tag=1)
    Y = (res["Y0"] + res["Y1"]) & np.uint64(p.t - 1)
    assert np.array_equal(Y, xw_mod(wl.X, wl.W, 37))
    # Shares are not the product itself (the mask is not zero).
    assert not np.array_equal(res["Y0"], Y)


@pytest.mark.parametrize("case", ["identity", "zeroW", "zeroX", "scalar", "negative", "maxval"])
def test_protocol_special_cases(orc, case):
    p = orc.Params(256, 2, 30, 8)
    rng = np.random.default_rng(11)
    n, r, m = 6, 8, 8
    X = rng.integers(0, p.t, (n, r), dtype=np.uint64)
    W = rng.integers(-200, 200, (r, m))
    if case == "identity":
        W = np.eye(r, m, dtype=np.int64)
    elif case == "zeroW":
        W = np.zeros((r, m), np.int64)
    elif case == "zeroX":
        X = np.zeros((n, r), np.uint64)
    elif case == "scalar":
        n = r = m = 1
        X, W = X[:1, :1], np.array([[-3]])
    elif case == "negative":
        W = -np.abs(W) - 1
    elif case == "maxval":
        X = np.full((n, r), p.t - 1, np.uint64)
        W = np.full((r, m), -255, np.int64)
    plan = orc.plan_comm(p.N, n, r, m)
    res = run_protocol(orc, p, plan, X, W, tag=2)
    Y = (res["Y0"] + res["Y1"]) & np.uint64(p.t - 1)
    want = xw_mod(X, W, p.ell)
    assert np.array_equal(Y, want)
    if case == "identity":
        assert np.array_equal(Y, X[:, :m] & np.uint64(p.t - 1))


@pytest.mark.parametrize("plan_kind", ["comm", "fix16", "fix64", "explicit"])
def test_protocol_plans_ragged(orc, plan_kind):
    p = orc.Params(256, 2, 33, 10)
    rng = np.random.default_rng(13)
    n, r, m = 19, 23, 13
    X = rng.integers(0, p.t, (n, r), dtype=np.uint64)
    W = rng.integers(-400, 400, (r, m))
    if plan_kind == "comm":
        plan = orc.plan_comm(p.N, n, r, m)
    elif plan_kind == "fix16":
        plan = orc.plan_fix(p.N, 16, n, r, m)
    elif plan_kind == "fix64":
        plan = orc.plan_fix(p.N, 64, n, r, m)
    else:
        plan = orc.Plan(n=n, r=r, m=m, mb=3, rb=5, nb=7, N=p.N)
    res = run_protocol(orc, p, plan, X, W, tag=3)
    Y = (res["Y0"] + res["Y1"]) & np.uint64(p.t - 1)
    assert np.array_equal(Y, xw_mod(X, W, p.ell))


def test_sparse_reply_equals_full_decryption(orc):
    """Section 3.1.3: coefficient m_i of m = s c1 + c0 needs only (c0)_i; decrypting the whole
    masked ciphertext at the decoded positions gives the client's share."""
    p = orc.Params(128, 2, 30, 8)
    rng = np.random.default_rng(17)
    n, r, m = 4, 8, 4
    X = rng.integers(0, p.t, (n, r), dtype=np.uint64)
    W = rng.integers(-100, 100, (r, m))
    plan = orc.plan_comm(p.N, n, r, m)
    res = run_protocol(orc, p, plan, X, W, tag=4)
    key = workloads.seed("server", 4)
    for o, y in enumerate(res["outs"]):
        full = res["acc_rr"][o:o + 1].copy()
        mask = np.zeros(p.N, np.uint64)
        import ctypes
        k = np.frombuffer(key, np.uint8).copy()
        orc.lib().orc_sample_poly(3, k.ctypes.data_as(ctypes.c_void_p), orc.TAG_MASK, 0, 4,
                                  int(y), p.N, 0, p.ell, None,
                                  mask.ctypes.data_as(ctypes.c_void_p))
        for l, q in enumerate(p.q):
            d = np.array([(p.delta_l[l] * int(v)) % q for v in mask], np.uint64)
            full[0, 0, l] = (full[0, 0, l] + (q - d)) % np.uint64(q)
        dec = orc.decrypt_full(p, res["s"], full)[0]
        vals = np.array([[dec[plan.pos(i, k)] for i in range(plan.mb)] for k in range(plan.nb)])
        sparse = orc.crt_round(p, orc.decrypt_residues(p, plan, res["s"], res["c1"][o:o + 1],
                                                        res["c0s"][o:o + 1]))[0]
        assert np.array_equal(vals.reshape(-1), sparse)


def test_noise_under_bound(orc):
    """The exact noise of every decoded coefficient of the reply stays under the analytic bound,
    and the bound is within the decryption budget for the BERT-base shapes."""
    p = orc.Params(4096, 2, 37, 12)
    wl = workloads.single_matmul()
    plan = orc.plan_comm(4096, *wl.shape)
    res = run_protocol(orc, p, plan, wl.X, wl.W, tag=5)
    x = orc.decrypt_residues(p, plan, res["s"], res["c1"], res["c0s"])
    Q = p.Q
    coef = [(Q // q) * pow(Q // q, -1, q) for q in p.q]
    vals = orc.crt_round(p, x)
    worst = 0
    for o in range(x.shape[0]):
        for j in range(x.shape[1]):
            v = sum(int(x[o, j, l]) * coef[l] for l in range(p.L)) % Q
            d = (v - p.Delta * int(vals[o, j])) % Q
            d = d - Q if d > Q // 2 else d
            worst = max(worst, abs(d))
    wmax = int(np.abs(wl.W).max())
    assert worst <= orc.noise_bound(p, plan, wmax)
    assert orc.noise_ok(p, plan, wmax)
    for (r, m) in [(768, 2304), (768, 768), (768, 3072), (3072, 768)]:
        pl = orc.plan_comm(4096, 128, r, m)
        assert orc.noise_ok(p, pl, 600)
    # A plaintext lifted uncentred (|w| ~ t) would break the budget: the bound says so.
    assert not orc.noise_ok(p, orc.plan_comm(4096, 128, 3072, 768), p.t // 2)


def _negacyclic_np(a, b):
    """Integer a * b mod (X^N + 1) by full convolution and the wrap X^N = -1 (small entries)."""
    n = len(a)
    c = np.convolve(np.asarray(a, np.int64), np.asarray(b, np.int64))
    out = c[:n].copy()
    out[:n - 1] -= c[n:]
    return out


def _sample(orc, kind, seed, tag, op, obj, p):
    import ctypes
    k = np.frombuffer(seed, np.uint8).copy()
    out = np.zeros(p.N, np.int64)
    orc.lib().orc_sample_poly(kind, k.ctypes.data_as(ctypes.c_void_p), tag, 0, op, obj, p.N, 0, 0,
                              p.cdt_arr.ctypes.data_as(ctypes.c_void_p),
                              out.ctypes.data_as(ctypes.c_void_p))
    return out


@pytest.mark.parametrize("N", [256, 4096])
def test_rerandomisation_adds_an_encryption_of_zero_with_its_exact_noise(orc, N):
    """The re-randomisation adds (u pk0 + e1, u pk1 + e2) with pk = (-a' s + e', a').  Under s
    this decrypts to u e' + e1 + e2 s exactly (the a' s terms cancel), so the decryption of the
    re-randomised reply minus that of the plain product must be that integer polynomial,
    recomputed here by schoolbook from the pinned samplers' u, e', e1, e2 and s.  A flipped
    sign of either product, a swapped component or a wrong stream changes it."""
    p = orc.Params(N, 2, 30, 8)
    rng = np.random.default_rng(29)
    n, r, m = 4, 8, 4
    X = rng.integers(0, p.t, (n, r), dtype=np.uint64)
    W = rng.integers(-100, 100, (r, m))
    plan = orc.plan_comm(p.N, n, r, m)
    res = run_protocol(orc, p, plan, X, W, tag=6)
    cseed, sseed = workloads.seed("client", 6), workloads.seed("server", 6)
    s = _sample(orc, 1, cseed, orc.TAG_SK, 0, 0, p)
    assert np.array_equal(s, res["s"])
    e_pk = _sample(orc, 2, cseed, 3, 0, 0, p)  # pk error e' (tag 3)
    Q = p.Q
    coef = [(Q // q) * pow(Q // q, -1, q) for q in p.q]

    def phase(ct):
        """[c0 + c1 s]_q of every coefficient, centred, as Python integers."""
        x = np.zeros((1, p.N, p.L), np.uint64)
        import ctypes
        orc.lib().orc_decrypt_full_residues(
            p.N, p.L, p.q_arr.ctypes.data_as(ctypes.c_void_p),
            p.psi_arr.ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p), 1,
            np.ascontiguousarray(ct).ctypes.data_as(ctypes.c_void_p), 0,
            x.ctypes.data_as(ctypes.c_void_p))
        out = []
        for j in range(p.N):
            v = sum(int(x[0, j, l]) * coef[l] for l in range(p.L)) % Q
            out.append(v - Q if v > Q // 2 else v)
        return out

    for o, y in enumerate(res["outs"][:2]):
        u = _sample(orc, 1, sseed, 6, 6, int(y), p)
        e1 = _sample(orc, 2, sseed, 7, 6, int(y), p)
        e2 = _sample(orc, 2, sseed, 8, 6, int(y), p)
        want = _negacyclic_np(u, e_pk) + e1 + _negacyclic_np(e2, s)
        got = [a - b for a, b in zip(phase(res["acc_rr"][o:o + 1]), phase(res["acc"][o:o + 1]))]
        got = [((g + Q // 2) % Q) - Q // 2 for g in got]
        assert got == want.tolist()
        assert np.abs(want).max() > 0
