"""Pins of the oracle's parameters, NTT and negacyclic products.

Primes against sympy's primality test and the stated rule (largest primes
below 2^50 with q = 1 mod 2N); psi against its defining property; the NTT
against the direct evaluation a(psi^(2k+1)) it stands for and its inverse; the
negacyclic product against schoolbook multiplication in Z[X]/(X^N + 1) written
in pure Python (tiny N) and in C (N = 4096).
"""
import ctypes
import random

import numpy as np
import pytest


def _vp(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@pytest.mark.parametrize("N,L", [(4096, 2), (8192, 3), (64, 2), (16, 1)])
def test_primes_rule(orc, N, L):
    sympy = pytest.importorskip("sympy")
    qs = orc.find_primes(N, L)
    assert len(qs) == L and qs == sorted(qs, reverse=True) and len(set(qs)) == L
    for q in qs:
        assert sympy.isprime(q) and q % (2 * N) == 1 and q < 2**50
    # "largest": no other prime = 1 mod 2N lies between qs[-1] and 2^50.
    k_hi = (2**50 - 2) // (2 * N)
    k_lo = (qs[-1] - 1) // (2 * N)
    others = [k * 2 * N + 1 for k in range(k_lo, k_hi + 1)
              if sympy.isprime(k * 2 * N + 1)]
    assert sorted(others, reverse=True) == qs


def test_params_configs(orc):
    p = orc.Params(4096, 2, 37, 12)
    assert p.Q == p.q[0] * p.q[1] and p.Delta == p.Q // 2**37
    for q, psi in zip(p.q, p.psi):
        assert pow(psi, 4096, q) == q - 1 and pow(psi, 8192, q) == 1
    p3 = orc.Params(8192, 3, 41, 14)
    assert p3.q[:2] == p.q  # both primes are also 1 mod 16384
    for q, psi in zip(p3.q, p3.psi):
        assert pow(psi, 8192, q) == q - 1


def py_negacyclic(a, b, q):
    """Schoolbook product in Z_q[X]/(X^N + 1), pure Python."""
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                c[i + j] += a[i] * b[j]
            else:
                c[i + j - n] -= a[i] * b[j]
    return [x % q for x in c]


@pytest.mark.parametrize("N", [2, 4, 16, 64])
def test_negacyclic_mul_vs_python_schoolbook(orc, N):
    q = orc.find_primes(N, 1)[0]
    psi = orc.find_psi(q, N)
    rng = random.Random(N)
    for _ in range(5):
        a = [rng.randrange(q) for _ in range(N)]
        b = [rng.randrange(q) for _ in range(N)]
        A, B = np.array(a, np.uint64), np.array(b, np.uint64)
        C = np.zeros(N, np.uint64)
        orc.lib().orc_negacyclic_mul(_vp(A), _vp(B), _vp(C), N, q, psi)
        assert C.tolist() == py_negacyclic(a, b, q)
        C2 = np.zeros(N, np.uint64)
        orc.lib().orc_negacyclic_mul_schoolbook(_vp(A), _vp(B), _vp(C2), N, q)
        assert C2.tolist() == C.tolist()


def test_negacyclic_mul_vs_schoolbook_4096(orc):
    p = orc.Params(4096, 2, 37, 12)
    rng = np.random.default_rng(4)
    for q, psi in zip(p.q, p.psi):
        a = rng.integers(0, q, 4096, dtype=np.uint64)
        b = rng.integers(0, q, 4096, dtype=np.uint64)
        c1, c2 = np.zeros(4096, np.uint64), np.zeros(4096, np.uint64)
        orc.lib().orc_negacyclic_mul(_vp(a), _vp(b), _vp(c1), 4096, q, psi)
        orc.lib().orc_negacyclic_mul_schoolbook(_vp(a), _vp(b), _vp(c2), 4096, q)
        assert np.array_equal(c1, c2)


@pytest.mark.parametrize("N", [8, 32])
def test_ntt_is_evaluation_at_odd_powers(orc, N):
    """A_k = a(psi^(2k+1)) by Horner, and the inverse returns a."""
    q = orc.find_primes(N, 1)[0]
    psi = orc.find_psi(q, N)
    rng = random.Random(7)
    a = [rng.randrange(q) for _ in range(N)]
    A = np.zeros(N, np.uint64)
    av = np.array(a, np.uint64)
    orc.lib().orc_ntt_negacyclic(_vp(av), _vp(A), N, q, psi)
    for k in range(N):
        x = pow(psi, 2 * k + 1, q)
        v = 0
        for coef in reversed(a):
            v = (v * x + coef) % q
        assert int(A[k]) == v
    back = np.zeros(N, np.uint64)
    orc.lib().orc_intt_negacyclic(_vp(A), _vp(back), N, q, psi)
    assert back.tolist() == a


def test_ntt_roundtrip_and_monomial_wrap(orc):
    p = orc.Params(4096, 2, 37, 12)
    q, psi = p.q[0], p.psi[0]
    rng = np.random.default_rng(9)
    a = rng.integers(0, q, 4096, dtype=np.uint64)
    A, back = np.zeros_like(a), np.zeros_like(a)
    orc.lib().orc_ntt_negacyclic(_vp(a), _vp(A), 4096, q, psi)
    orc.lib().orc_intt_negacyclic(_vp(A), _vp(back), 4096, q, psi)
    assert np.array_equal(a, back)
    # X^(N-1) * X = X^N = -1 in the negacyclic ring.
    x1 = np.zeros(4096, np.uint64)
    x1[1] = 1
    xn1 = np.zeros(4096, np.uint64)
    xn1[4095] = 1
    c = np.zeros(4096, np.uint64)
    orc.lib().orc_negacyclic_mul(_vp(x1), _vp(xn1), _vp(c), 4096, q, psi)
    want = np.zeros(4096, np.uint64)
    want[0] = q - 1
    assert np.array_equal(c, want)
