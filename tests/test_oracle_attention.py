"""Pins of the attention cross terms (Eq. 2, section 3.1): Q K^T on shares Q = Q0 + Q1,
K = K0 + K1 splits into two local products and two cross terms, each a Pi_MatMul whose
plaintext operand is the server's *uniform* share instead of small weights.

- the noise bound refuses such an operand at the two-prime parameters of the BERT-base layer
  and accepts it at N = 8192 with three primes (q about 2^150), which the cross terms use;
- one cross term through the protocol gives shares of X0 W1 mod 2^l (plain integer product);
- the four parts together give shares of Q K^T mod 2^l, and the same for A V.
"""
import numpy as np
import pytest

from paper_2305_18396_amd import workloads

ELL = 41


def centred(u, ell):
    """A share in Z_{2^l} as the signed integer in [-2^(l-1), 2^(l-1)) the server encodes."""
    u = np.asarray(u, dtype=np.uint64).astype(object)
    half = 1 << (ell - 1)
    return np.array([[int(v) - (1 << ell) if int(v) >= half else int(v) for v in row] for row in u],
                    dtype=np.int64)


def prod_mod(A, B, ell):
    A = np.asarray(A, dtype=object)
    B = np.asarray(B, dtype=object)
    return np.array((A.dot(B)) % (1 << ell), dtype=np.uint64)


def cross(orc, p, X0, W1, tag):
    """Pi_MatMul with the client's share X0 encrypted and the server's share W1 as plaintext."""
    n, r = X0.shape
    m = W1.shape[1]
    plan = orc.plan_comm(p.N, n, r, m)
    res = orc.pi_matmul(p, plan, X0, centred(W1, p.ell), workloads.seed("client", tag),
                        workloads.seed("server", tag), op_id=tag)
    return res["Y0"], res["Y1"]


def test_noise_needs_three_primes(orc):
    wmax = 1 << (ELL - 1)
    small = orc.Params(4096, 2, 37, 12)
    assert not orc.noise_ok(small, orc.plan_comm(4096, 128, 64, 128), 1 << 36)
    big = orc.Params(8192, 3, ELL, 14)
    for shape in [(128, 64, 128), (128, 128, 64), (64, 128, 128)]:
        assert orc.noise_ok(big, orc.plan_comm(8192, *shape), wmax)


def test_cross_term_shares(orc):
    p = orc.Params(8192, 3, ELL, 14)
    rng = np.random.default_rng(61)
    X0 = rng.integers(0, p.t, (6, 16), dtype=np.uint64)
    W1 = rng.integers(0, p.t, (16, 10), dtype=np.uint64)
    W1[0, 0], W1[1, 1] = p.t - 1, 1 << (ELL - 1)
    Y0, Y1 = cross(orc, p, X0, W1, 61)
    assert np.array_equal((Y0 + Y1) & np.uint64(p.t - 1), prod_mod(X0, W1, ELL))


def test_attention_scores_and_values_on_shares(orc):
    """QK^T = Q0 K0^T + Q1 K1^T (local) + Q0 K1^T + (K0 Q1^T)^T (cross terms, the client's
    share encrypted each time); A V likewise.  Shapes per head scaled down: seq 6, head dim 8."""
    p = orc.Params(8192, 3, ELL, 14)
    mask = np.uint64(p.t - 1)
    rng = np.random.default_rng(62)
    n, d = 6, 8
    Q, K, V = (rng.integers(0, p.t, (n, d), dtype=np.uint64) for _ in range(3))
    Q1, K1, V1 = (rng.integers(0, p.t, (n, d), dtype=np.uint64) for _ in range(3))
    Q0, K0, V0 = (Q - Q1) & mask, (K - K1) & mask, (V - V1) & mask
    a0, a1 = cross(orc, p, Q0, np.ascontiguousarray(K1.T), 63)            # Q0 K1^T
    b0, b1 = cross(orc, p, K0, np.ascontiguousarray(Q1.T), 64)            # K0 Q1^T
    client = (prod_mod(Q0, K0.T, ELL) + a0 + b0.T) & mask
    server = (prod_mod(Q1, K1.T, ELL) + a1 + b1.T) & mask
    assert np.array_equal((client + server) & mask, prod_mod(Q, K.T, ELL))
    # A V with A shared (n x n) and V shared (n x d).
    A = rng.integers(0, p.t, (n, n), dtype=np.uint64)
    A1 = rng.integers(0, p.t, (n, n), dtype=np.uint64)
    A0 = (A - A1) & mask
    c0, c1 = cross(orc, p, A0, V1, 65)                                     # A0 V1
    e0, e1 = cross(orc, p, np.ascontiguousarray(V0.T), np.ascontiguousarray(A1.T), 66)  # V0^T A1^T
    client = (prod_mod(A0, V0, ELL) + c0 + e0.T) & mask
    server = (prod_mod(A1, V1, ELL) + c1 + e1.T) & mask
    assert np.array_equal((client + server) & mask, prod_mod(A, V, ELL))
