"""Pins of the evaluation form in which a query ciphertext's uniform part travels.

The slot order is a definition (slot z holds the polynomial's value at psi^(2k+1) for the k the
oracle's slot_index gives); what the protocol relies on is checked here against independent
computations:
- slot_index is a permutation of 0 .. N-1;
- the slots of a polynomial are exactly its values at the N odd powers of psi (brute-force
  evaluation), and coefficients -> slots -> coefficients is the identity;
- the slot form is a ring isomorphism: the slots of a negacyclic product (schoolbook) are the
  slot-wise products, and the slots of a sum are the slot-wise sums;
- a fresh encryption, whose c1 is the draws taken as slots, decrypts to its plaintext and its
  c1 is exactly the uniform draws of its stream; its c0, read as slots, is exactly
  Delta pt + e - a s with e the Gaussian draws of its stream and a s a schoolbook product.
"""
import ctypes

import numpy as np
import pytest

from paper_2305_18396_amd import workloads



def small_params(orc, N):
    # A prime q = 1 mod 2N below 2^20 and a primitive 2N-th root, found by brute force here.
    q = 2 * N + 1
    while True:
        if all(q % d for d in range(2, int(q ** 0.5) + 1)):
            break
        q += 2 * N
    for g in range(2, q):
        psi = pow(g, (q - 1) // (2 * N), q)
        if pow(psi, N, q) == q - 1:
            return q, psi


def slots(orc, a, N, q, psi):
    src = np.ascontiguousarray(np.asarray(a, np.uint64))
    out = np.zeros(N, np.uint64)
    orc.lib().orc_coef_to_slots(src.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                                N, q, psi)
    return out


def coefs(orc, S, N, q, psi):
    src = np.ascontiguousarray(np.asarray(S, np.uint64))
    out = np.zeros(N, np.uint64)
    orc.lib().orc_slots_to_coef(src.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                                N, q, psi)
    return out


@pytest.mark.parametrize("N", [16, 64, 4096])
def test_slot_index_is_a_permutation(orc, N):
    k = orc.slot_index(N)
    assert sorted(k.tolist()) == list(range(N))


@pytest.mark.parametrize("N", [16, 32, 64])
def test_slots_are_the_values_at_the_odd_powers(orc, N):
    q, psi = small_params(orc, N)
    rng = np.random.default_rng(N)
    a = rng.integers(0, q, N)
    S = slots(orc, a, N, q, psi)
    k = orc.slot_index(N)
    for z in range(N):
        x = pow(psi, 2 * int(k[z]) + 1, q)
        assert int(S[z]) == sum(int(a[j]) * pow(x, j, q) for j in range(N)) % q
    # every odd power appears once: the slots are the whole evaluation form
    assert sorted(set(int(v) for v in k)) == list(range(N))
    assert np.array_equal(coefs(orc, S, N, q, psi), a.astype(np.uint64))


@pytest.mark.parametrize("N", [32, 256])
def test_slot_form_is_a_ring_isomorphism(orc, N):
    q, psi = small_params(orc, N)
    rng = np.random.default_rng(7 * N)
    a, b = rng.integers(0, q, N), rng.integers(0, q, N)
    # schoolbook negacyclic product and sum
    c = [0] * N
    for i in range(N):
        for j in range(N):
            if i + j < N:
                c[i + j] = (c[i + j] + int(a[i]) * int(b[j])) % q
            else:
                c[i + j - N] = (c[i + j - N] - int(a[i]) * int(b[j])) % q
    Sa, Sb = slots(orc, a, N, q, psi), slots(orc, b, N, q, psi)
    assert [int(v) for v in slots(orc, c, N, q, psi)] == [int(x) * int(y) % q for x, y in zip(Sa, Sb)]
    assert [int(v) for v in slots(orc, (a + b) % q, N, q, psi)] == [(int(x) + int(y)) % q
                                                                  for x, y in zip(Sa, Sb)]


def test_fresh_encryption_in_evaluation_form(orc):
    p = orc.Params(4096, 2, 37, 12)
    seed = workloads.seed("client", 41)
    s, _ = orc.keygen(p, seed)
    rng = np.random.default_rng(41)
    pt = rng.integers(0, p.t, (2, p.N), dtype=np.uint64)
    ct = orc.encrypt(p, s, seed, 3, pt)
    assert np.array_equal(orc.decrypt_full(p, s, ct, query=True), pt)
    # c1 is the stream's uniform draws themselves (no transform applied)
    key = np.frombuffer(seed, np.uint8).copy()
    for x in range(2):
        for l in range(p.L):
            a = np.zeros(p.N, np.uint64)
            orc.lib().orc_sample_poly(0, key.ctypes.data_as(ctypes.c_void_p), orc.TAG_ENC_A, l, 3, x, p.N,
                                      int(p.q[l]), 0, None, a.ctypes.data_as(ctypes.c_void_p))
            assert np.array_equal(ct[x, 1, l], a)
    # read as coefficients instead, the same ciphertext does not decrypt to the plaintext
    assert not np.array_equal(orc.decrypt_full(p, s, ct, query=False), pt)
    # and the coefficient form of c1 is what the slots describe
    c1c = orc.slots_to_coef(p, ct[:, 1])
    assert np.array_equal(orc.coef_to_slots(p, c1c), ct[:, 1])
    # c0 travels as slots too: its coefficients are Delta pt + e - a s, with e the stream's
    # Gaussian draws and a s by schoolbook (no transform on this side)
    c0c = orc.slots_to_coef(p, ct[:, 0])
    assert not np.array_equal(c0c, ct[:, 0])
    cdt = np.ascontiguousarray(p.cdt_arr)
    for x in range(2):
        e = np.zeros(p.N, np.int64)
        orc.lib().orc_sample_poly(2, key.ctypes.data_as(ctypes.c_void_p), orc.TAG_ENC_E, 0, 3, x, p.N, 0, 0,
                                  cdt.ctypes.data_as(ctypes.c_void_p), e.ctypes.data_as(ctypes.c_void_p))
        for l in range(p.L):
            q = int(p.q[l])
            sl = np.array([int(v) % q for v in s], np.uint64)
            a = np.ascontiguousarray(c1c[x, l])
            prod = np.zeros(p.N, np.uint64)
            orc.lib().orc_negacyclic_mul_schoolbook(a.ctypes.data_as(ctypes.c_void_p),
                                                    sl.ctypes.data_as(ctypes.c_void_p),
                                                    prod.ctypes.data_as(ctypes.c_void_p), p.N, q)
            delta = (p.Q // p.t) % q
            want = [(delta * int(pt[x, j]) + int(e[j]) - int(prod[j])) % q for j in range(p.N)]
            assert [int(v) for v in c0c[x, l]] == want
