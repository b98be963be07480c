"""Pins of the oracle's grouped run (G products of one shape as one protocol call; the
attention cross terms of Eq. 2 are such groups: 24 independent products per phase).

- one product as a group of one is the plain protocol, buffer for buffer;
- every product of a group: the two shares add up to X_p W_p (mod 2^l) against a numpy integer
  matrix product, with re-randomisation on and off;
- the products of a group draw from distinct streams: equal inputs give different ciphertexts
  and different masks, and each product's ciphertexts decrypt to its own encoding.
"""
import numpy as np
import pytest

from paper_2305_18396_amd import workloads


def xw_mod(X, W, ell):
    Xu = np.asarray(X, dtype=np.uint64)
    Wu = np.asarray(W, dtype=np.int64).astype(np.uint64)
    return (Xu @ Wu) & np.uint64((1 << ell) - 1)


def test_group_of_one_is_the_plain_protocol(orc):
    p = orc.Params(4096, 2, 37, 12)
    rng = np.random.default_rng(31)
    X = workloads.share(rng, 16, 64, 37)
    W = workloads.weights(rng, 64, 64, 12)
    plan = orc.plan_comm(4096, 16, 64, 64)
    cs, ss = workloads.seed("client", 31), workloads.seed("server", 31)
    a = orc.pi_matmul(p, plan, X, W, cs, ss, op_id=5)
    g = orc.pi_matmul_grouped(p, plan, [X], [W], cs, ss, op_id=5)
    for k in ("pt", "ct", "acc", "acc_rr", "c1", "c0s", "smask"):
        assert np.array_equal(a[k], g[k]), k
    assert np.array_equal(a["Y0"], g["Y0"][0]) and np.array_equal(a["Y1"], g["Y1"][0])


@pytest.mark.parametrize("rr", [True, False])
@pytest.mark.parametrize("N,L,ell,f,shape,G", [
    (4096, 2, 37, 12, (16, 64, 48), 3),
    (8192, 3, 41, 14, (40, 32, 40), 4),
])
def test_every_product_of_a_group(orc, rr, N, L, ell, f, shape, G):
    n, r, m = shape
    p = orc.Params(N, L, ell, f, rerandomize=rr)
    rng = np.random.default_rng(N + G)
    Xs = [workloads.share(rng, n, r, ell) for _ in range(G)]
    Ws = [workloads.weights(rng, r, m, f) for _ in range(G)]
    plan = orc.plan_comm(N, n, r, m)
    g = orc.pi_matmul_grouped(p, plan, Xs, Ws, workloads.seed("client", 32),
                              workloads.seed("server", 32), op_id=9)
    assert g["ct"].shape[0] == G * plan.I and g["c1"].shape[0] == G * plan.O
    for k in range(G):
        Y = (g["Y0"][k] + g["Y1"][k]) & np.uint64(p.t - 1)
        assert np.array_equal(Y, xw_mod(Xs[k], Ws[k], ell)), k


def test_products_of_a_group_use_distinct_streams(orc):
    p = orc.Params(4096, 2, 37, 12)
    rng = np.random.default_rng(33)
    X = workloads.share(rng, 8, 32, 37)
    W = workloads.weights(rng, 32, 32, 12)
    plan = orc.plan_comm(4096, 8, 32, 32)
    g = orc.pi_matmul_grouped(p, plan, [X, X], [W, W], workloads.seed("client", 33),
                              workloads.seed("server", 33), op_id=2)
    I, O = plan.I, plan.O
    assert not np.array_equal(g["ct"][:I], g["ct"][I:])
    assert not np.array_equal(g["smask"][:O], g["smask"][O:])
    dec = orc.decrypt_full(p, g["s"], g["ct"], query=True)
    assert np.array_equal(dec, np.asarray(g["pt"], np.uint64) % np.uint64(p.t))
    assert np.array_equal(g["Y0"][0] + g["Y1"][0] & np.uint64(p.t - 1),
                          g["Y0"][1] + g["Y1"][1] & np.uint64(p.t - 1))
