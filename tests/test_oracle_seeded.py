"""Pins of the oracle's seed-compressed upload (a wire-format variant of Algorithm 1 step 2):
c1 = a comes from a public seed, so the client sends c0 and the seed.

- with a_seed = seed the seeded encryption is the plain encryption (pinned elsewhere);
- c1 is the uniform stream of a_seed (tag 4), independent of the secret seed;
- the server's expansion of c0 rebuilds the client's ciphertext byte for byte;
- Dec(expand(c0)) = m for the pinned decryption, and the protocol with the seeded upload
  still gives shares of X W.
"""
import numpy as np
import pytest

from paper_2305_18396_amd import workloads


@pytest.fixture(scope="module")
def params(orc):
    return orc.Params(4096, 2, 37, 12)


def test_seeded_equals_plain_with_same_seed(orc, params):
    rng = np.random.default_rng(3)
    s, _ = orc.keygen(params, workloads.seed("client", 3))
    pt = rng.integers(0, params.t, (3, params.N), dtype=np.uint64)
    seed = workloads.seed("client", 4)
    assert np.array_equal(orc.encrypt_seeded(params, s, seed, seed, 7, pt),
                          orc.encrypt(params, s, seed, 7, pt))


def test_c1_is_public_stream(orc, params):
    rng = np.random.default_rng(5)
    s, _ = orc.keygen(params, workloads.seed("client", 5))
    pt = rng.integers(0, params.t, (2, params.N), dtype=np.uint64)
    a_seed = workloads.seed("public", 5)
    ct1 = orc.encrypt_seeded(params, s, workloads.seed("client", 6), a_seed, 2, pt)
    ct2 = orc.encrypt_seeded(params, s, workloads.seed("client", 7), a_seed, 2, pt)
    assert np.array_equal(ct1[:, 1], ct2[:, 1])
    assert not np.array_equal(ct1[:, 0], ct2[:, 0])
    # c1 is exactly what a plain encryption under a_seed puts there.
    ct3 = orc.encrypt(params, s, a_seed, 2, pt)
    assert np.array_equal(ct1[:, 1], ct3[:, 1])


def test_expand_rebuilds_and_decrypts(orc, params):
    rng = np.random.default_rng(8)
    s, _ = orc.keygen(params, workloads.seed("client", 8))
    pt = rng.integers(0, params.t, (3, params.N), dtype=np.uint64)
    a_seed = workloads.seed("public", 8)
    ct = orc.encrypt_seeded(params, s, workloads.seed("client", 9), a_seed, 11, pt)
    ex = orc.expand_ct(params, a_seed, 11, np.ascontiguousarray(ct[:, 0]))
    assert np.array_equal(ex, ct)
    assert np.array_equal(orc.decrypt_full(params, s, ex, query=True), pt)


def test_protocol_with_seeded_upload(orc):
    p = orc.Params(4096, 2, 37, 12)
    rng = np.random.default_rng(12)
    n, r, m = 9, 40, 30
    X = rng.integers(0, p.t, (n, r), dtype=np.uint64)
    W = rng.integers(-1500, 1500, (r, m))
    plan = orc.plan_comm(p.N, n, r, m)
    cseed, sseed, aseed = (workloads.seed(k, 12) for k in ("client", "server", "public"))
    s, pk = orc.keygen(p, cseed)
    ct = orc.encrypt_seeded(p, s, cseed, aseed, 1, orc.encode_input(plan, X))
    ct = orc.expand_ct(p, aseed, 1, np.ascontiguousarray(ct[:, 0]))
    outs = np.arange(plan.O, dtype=np.uint32)
    acc = orc.rerandomize(p, pk, sseed, 1, orc.matmul(p, plan, orc.encode_weights(plan, W), ct, outs),
                          outs)
    c1, c0s, sm = orc.mask_extract(p, plan, sseed, 1, acc, outs)
    Y = (orc.decrypt(p, plan, s, c1, c0s, outs) + orc.place_shares(plan, sm, outs)) & np.uint64(p.t - 1)
    Xu, Wu = X.astype(np.uint64), W.astype(np.int64).astype(np.uint64)
    assert np.array_equal(Y, (Xu @ Wu) & np.uint64(p.t - 1))
