"""Pins of the oracle's completion of a fully connected layer (section 3.1, the linear
layers): the server adds X1 W + b to its share of X0 W.

- brute force with Python integers on small shapes, with values at the edges of Z_{2^l}
  (X1 near 2^l, negative W and b, entries of X1 above 2^l that must be reduced);
- closed forms: W = I gives Y1 + X1 + b, X1 = 0 gives Y1 + b, no bias gives Y1 + X1 W;
- the whole layer: Pi_MatMul on X0 followed by the completion gives shares of X W + b,
  against a Python-integer matrix product.
"""
import numpy as np
import pytest

from paper_2305_18396_amd import workloads


def brute(X1, W, b, Y1, ell):
    n, r = len(X1), len(X1[0])
    m = len(W[0])
    out = []
    for i in range(n):
        row = []
        for j in range(m):
            acc = int(Y1[i][j])
            for k in range(r):
                acc += (int(X1[i][k]) % (1 << ell)) * int(W[k][j])
            if b is not None:
                acc += int(b[j])
            row.append(acc % (1 << ell))
        out.append(row)
    return np.array(out, dtype=np.uint64)


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 4), (7, 2, 6), (4, 9, 3)])
@pytest.mark.parametrize("ell", [30, 37, 41])
def test_fc_complete_brute_force(orc, shape, ell):
    n, r, m = shape
    p = orc.Params(256, 2, ell, 8)
    rng = np.random.default_rng(100 + n * 31 + r * 7 + m + ell)
    X1 = rng.integers(0, 1 << ell, (n, r), dtype=np.uint64)
    X1[0, 0] = (1 << ell) - 1
    W = rng.integers(-5000, 5000, (r, m))
    W[-1, -1] = -(1 << 20)
    b = rng.integers(-(1 << 30), 1 << 30, m)
    Y1 = rng.integers(0, 1 << ell, (n, m), dtype=np.uint64)
    got = orc.fc_complete(p, X1, W, b, Y1)
    assert np.array_equal(got, brute(X1.tolist(), W.tolist(), b.tolist(), Y1.tolist(), ell))


def test_fc_complete_reduces_x1(orc):
    p = orc.Params(256, 2, 20, 8)
    X1 = np.array([[(1 << 20) + 5, (3 << 20) + 1]], dtype=np.uint64)
    W = np.array([[2], [-1]])
    got = orc.fc_complete(p, X1, W, None, np.zeros((1, 1), np.uint64))
    assert int(got[0, 0]) == (5 * 2 - 1) % (1 << 20)


@pytest.mark.parametrize("case", ["identity", "zeroX1", "nobias"])
def test_fc_complete_closed_forms(orc, case):
    p = orc.Params(256, 2, 37, 12)
    rng = np.random.default_rng(7)
    n, r, m = 5, 6, 6
    mask = np.uint64(p.t - 1)
    X1 = rng.integers(0, p.t, (n, r), dtype=np.uint64)
    W = rng.integers(-300, 300, (r, m))
    b = rng.integers(-(1 << 24), 1 << 24, m)
    Y1 = rng.integers(0, p.t, (n, m), dtype=np.uint64)
    bu = b.astype(np.int64).astype(np.uint64)
    if case == "identity":
        W = np.eye(r, m, dtype=np.int64)
        want = (Y1 + X1 + bu[None, :]) & mask
    elif case == "zeroX1":
        X1 = np.zeros_like(X1)
        want = (Y1 + bu[None, :]) & mask
    else:
        b = None
        want = brute(X1.tolist(), W.tolist(), None, Y1.tolist(), p.ell)
    assert np.array_equal(orc.fc_complete(p, X1, W, b, Y1), want)


@pytest.mark.parametrize("rerand", [True, False])
def test_fc_layer_shares_sum_to_xw_plus_b(orc, rerand):
    """Pi_MatMul on the client's share X0, then the server's completion: the two final shares
    add up to X W + b mod 2^l (Python integers)."""
    p = orc.Params(4096, 2, 37, 12, rerandomize=rerand)
    rng = np.random.default_rng(21)
    n, r, m = 6, 20, 9
    X = rng.integers(0, p.t, (n, r), dtype=np.uint64)
    X1 = rng.integers(0, p.t, (n, r), dtype=np.uint64)
    X0 = (X - X1) & np.uint64(p.t - 1)
    W = rng.integers(-2000, 2000, (r, m))
    b = rng.integers(-(1 << 30), 1 << 30, m)
    plan = orc.plan_comm(p.N, n, r, m)
    res = orc.pi_matmul(p, plan, X0, W, workloads.seed("client", 9), workloads.seed("server", 9),
                        op_id=4)
    Y1 = orc.fc_complete(p, X1, W, b, res["Y1"])
    Y = (res["Y0"] + Y1) & np.uint64(p.t - 1)
    want = brute(X.tolist(), W.tolist(), b.tolist(), np.zeros((n, m), np.uint64).tolist(), p.ell)
    assert np.array_equal(Y, want)
