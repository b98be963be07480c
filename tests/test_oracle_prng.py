"""Pins of the oracle's randomness against things other than itself.

ChaCha20 (RFC 8439 section 2.3) is checked against the OpenSSL command-line
cipher, which takes a 16-byte IV = 32-bit LE block counter || 96-bit nonce and
XORs the keystream into its input (all-zero input gives the keystream).  The
stream layout (draw j = keystream bytes [8j, 8j+8)) is checked against the same
keystream.  Samplers are checked against distributions fixed
independently: the cumulative table against a 50-digit mpmath recomputation,
and sample statistics against the exact probabilities.
"""
import ctypes
import shutil
import subprocess

import numpy as np
import pytest

needs_openssl = pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI absent")


def openssl_keystream(key: bytes, counter: int, nonce: bytes, nbytes: int) -> bytes:
    iv = counter.to_bytes(4, "little") + nonce
    out = subprocess.run(
        ["openssl", "enc", "-chacha20", "-K", key.hex(), "-iv", iv.hex()],
        input=bytes(nbytes), capture_output=True, check=True)
    return out.stdout


def nonce_bytes(tag, prime, op, obj):
    w = [tag | (prime << 8), op, obj]
    return b"".join(x.to_bytes(4, "little") for x in w)


@needs_openssl
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_chacha_block_matches_openssl(orc, seed):
    rng = np.random.default_rng(100 + seed)
    key = rng.integers(0, 256, 32, dtype=np.uint8)
    nonce = rng.integers(0, 2**32, 3, dtype=np.uint64).astype(np.uint32)
    counter = int(rng.integers(0, 2**31))
    out = np.zeros(16, dtype=np.uint32)
    orc.lib().orc_chacha20_block(key.ctypes.data_as(ctypes.c_void_p), counter,
                                 nonce.ctypes.data_as(ctypes.c_void_p),
                                 out.ctypes.data_as(ctypes.c_void_p))
    ks = openssl_keystream(bytes(key), counter, nonce.tobytes(), 64)
    assert out.astype("<u4").tobytes() == ks


@needs_openssl
def test_draw_layout_is_the_keystream(orc):
    key = bytes(range(7, 39))
    tag, prime, op, obj = 4, 2, 0xDEADBEEF, 12345
    ks = openssl_keystream(key, 0, nonce_bytes(tag, prime, op, obj), 16 * 40)
    k = np.frombuffer(key, dtype=np.uint8).copy()
    kp = k.ctypes.data_as(ctypes.c_void_p)
    for j in [0, 1, 7, 8, 9, 31, 79]:
        want = int.from_bytes(ks[8 * j:8 * j + 8], "little")
        assert orc.lib().orc_draw64(kp, tag, prime, op, obj, j) == want


@needs_openssl
def test_samplers_read_the_keystream(orc):
    """Each sampler's value for draw j, recomputed from the OpenSSL keystream bytes."""
    key = bytes(range(100, 132))
    k = np.frombuffer(key, dtype=np.uint8).copy()
    n = 64
    q = 1125899906826241
    cdt = np.asarray(orc.cdt_table(), dtype=np.uint64)

    def sample(kind, tag, prime, op, obj, ell=37, q_=q):
        out = np.zeros(n, dtype=np.uint64 if kind in (0, 3) else np.int64)
        orc.lib().orc_sample_poly(kind, k.ctypes.data_as(ctypes.c_void_p), tag, prime, op, obj, n,
                                  q_, ell, cdt.ctypes.data_as(ctypes.c_void_p),
                                  out.ctypes.data_as(ctypes.c_void_p))
        return out

    # Uniform mod q: the low 50 bits of draw j if below q, else the low 50 bits of draw j of
    # the fallback stream (bit 31 of the tag word set) mod q.  A q just above 2^49 rejects
    # about half the draws, so both streams are read; the parameter rule's q takes the first.
    m50 = (1 << 50) - 1
    ks = openssl_keystream(key, 0, nonce_bytes(4, 1, 5, 6), 8 * n)
    fb = openssl_keystream(key, 0, nonce_bytes(4 | (1 << 31), 1, 5, 6), 8 * n)
    for qq in (q, (1 << 49) + 9):
        want, rejected = [], 0
        for j in range(n):
            x = int.from_bytes(ks[8 * j:8 * j + 8], "little") & m50
            if x >= qq:
                rejected += 1
                x = (int.from_bytes(fb[8 * j:8 * j + 8], "little") & m50) % qq
            want.append(x)
        assert sample(0, 4, 1, 5, 6, q_=qq).tolist() == want
        assert (rejected == 0) if qq == q else (10 < rejected < 54)

    ks = openssl_keystream(key, 0, nonce_bytes(9, 0, 5, 6), 8 * n)
    d = [int.from_bytes(ks[8 * j:8 * j + 8], "little") for j in range(n)]
    assert sample(3, 9, 0, 5, 6, ell=37).tolist() == [v % (1 << 37) for v in d]

    ks = openssl_keystream(key, 0, nonce_bytes(1, 0, 5, 6), 8 * n)
    d = [int.from_bytes(ks[8 * j:8 * j + 8], "little") for j in range(n)]
    assert sample(1, 1, 0, 5, 6).tolist() == [v % 3 - 1 for v in d]


def test_uniform_fallback_fixture(orc):
    """The stored stream position (tests/golden/uniform_fallback.json, written by its script from
    the oracle's sampler) has a rejected first draw: the sampler returns the fallback stream's draw
    there, read back through the 64-bit draw function, and the first draw everywhere else."""
    import json
    import os

    from paper_2305_18396_amd import workloads

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "uniform_fallback.json")))
    p = orc.Params(g["N"], g["L"], 41, 14)
    q = int(p.q[g["prime"]])
    assert q == g["q"]
    key = np.frombuffer(workloads.seed("client", g["request"]), np.uint8).copy()
    kp = key.ctypes.data_as(ctypes.c_void_p)
    out = np.zeros(g["N"], np.uint64)
    orc.lib().orc_sample_poly(0, kp, g["tag"], g["prime"], g["op"], g["obj"], g["N"], q, 41,
                              p.cdt_arr.ctypes.data_as(ctypes.c_void_p),
                              out.ctypes.data_as(ctypes.c_void_p))
    m50 = (1 << 50) - 1
    first = [orc.lib().orc_draw64(kp, g["tag"], g["prime"], g["op"], g["obj"], j) & m50
             for j in range(g["N"])]
    j = g["j"]
    assert first[j] == g["first_draw_low50"] and first[j] >= q
    fb = orc.lib().orc_draw64(kp, g["tag"] | (1 << 31), g["prime"], g["op"], g["obj"], j) & m50
    assert int(out[j]) == fb % q != first[j]
    assert [int(v) for i, v in enumerate(out) if i != j] == [v for i, v in enumerate(first) if i != j]


def _cdt_mpmath():
    """T[k] = floor(2^63 P(|e| <= k)), k = 0..18, for width 3.2 cut at |e| <= 19 (50 digits)."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    s2 = 2 * mpmath.mpf("3.2") ** 2
    rho = [mpmath.e ** (-(mpmath.mpf(x) ** 2) / s2) for x in range(20)]
    total = rho[0] + 2 * mpmath.fsum(rho[1:])
    want, acc = [], rho[0]
    for k in range(19):
        want.append(int(mpmath.floor(acc / total * mpmath.mpf(2) ** 63)))
        acc += 2 * rho[k + 1]
    return want


@needs_openssl
def test_gaussian_sampler_reads_the_keystream(orc):
    """The error sampler's exact draw -> value rule, recomputed from the OpenSSL keystream and
    an mpmath table: with d the 64-bit draw j and u = d mod 2^63 (its low 63 bits),
    |e_j| = #{k : u >= T[k]} and e_j < 0 exactly when bit 63 of d is set.  A flipped sign, a
    shifted 63-bit field or a table read off by one entry each change some of the 4096 values.
    (Whether u = T[k] counts is unobservable on random draws: it has probability 19 / 2^63.)"""
    key = bytes(range(60, 92))
    k = np.frombuffer(key, dtype=np.uint8).copy()
    n = 4096
    T = _cdt_mpmath()
    cdt = np.asarray(T, dtype=np.uint64)
    got = np.zeros(n, dtype=np.int64)
    orc.lib().orc_sample_poly(2, k.ctypes.data_as(ctypes.c_void_p), 5, 0, 7, 3, n, 0, 0,
                              cdt.ctypes.data_as(ctypes.c_void_p),
                              got.ctypes.data_as(ctypes.c_void_p))
    ks = openssl_keystream(key, 0, nonce_bytes(5, 0, 7, 3), 8 * n)
    want = []
    for j in range(n):
        d = int.from_bytes(ks[8 * j:8 * j + 8], "little")
        u = d & ((1 << 63) - 1)
        mag = sum(1 for t in T if u >= t)
        want.append(-mag if d >> 63 else mag)
    assert got.tolist() == want
    # The draws exercise both signs and magnitudes across the table.
    assert min(want) <= -6 and max(want) >= 6


def test_cdt_table_against_mpmath(orc):
    """T[k] = floor(2^63 P(|e| <= k)) for the Gaussian of width 3.2 cut at |e| <= 19,
    recomputed with mpmath at 50 digits (the oracle uses Python's decimal module)."""
    want = _cdt_mpmath()
    assert orc.cdt_table() == want
    assert all(a < b for a, b in zip(want, want[1:]))  # strictly increasing
    assert want[-1] < 2**63


def _poly(orc, kind, tag, n, obj=0, q=0, ell=0):
    key = np.frombuffer(bytes(range(32)), dtype=np.uint8).copy()
    cdt = np.asarray(orc.cdt_table(), dtype=np.uint64)
    out = np.zeros(n, dtype=np.uint64 if kind in (0, 3) else np.int64)
    orc.lib().orc_sample_poly(kind, key.ctypes.data_as(ctypes.c_void_p), tag, 0, 0, obj, n, q, ell,
                              cdt.ctypes.data_as(ctypes.c_void_p),
                              out.ctypes.data_as(ctypes.c_void_p))
    return out


def test_gaussian_statistics(orc):
    """200k draws: mean ~ 0, variance ~ sigma^2 = 10.24, support within the cut, and a chi^2
    test against the exact discrete-Gaussian probabilities."""
    e = _poly(orc, 2, 5, 200_000)
    assert np.abs(e).max() <= 19
    assert abs(e.mean()) < 0.03
    assert abs(e.var() - 10.24) < 0.15
    rho = np.exp(-np.arange(-19, 20) ** 2 / (2 * 3.2 ** 2))
    p = rho / rho.sum()
    counts = np.bincount(e + 19, minlength=39)
    expect = p * len(e)
    keep = expect > 20
    chi2 = (((counts - expect) ** 2) / expect)[keep].sum()
    assert chi2 < 2.5 * keep.sum()  # far inside the tail for ~25 degrees of freedom


def test_ternary_and_mask_and_uniform_statistics(orc):
    t = _poly(orc, 1, 1, 60_000)
    c = np.bincount(t + 1, minlength=3)
    assert set(np.unique(t).tolist()) == {-1, 0, 1}
    assert np.all(np.abs(c - 20_000) < 600)
    m = _poly(orc, 3, 9, 60_000, ell=37)
    assert m.max() < 2**37
    bits = np.array([(m >> np.uint64(b)) & np.uint64(1) for b in range(37)], dtype=np.float64)
    assert np.all(np.abs(bits.mean(axis=1) - 0.5) < 0.012)
    q = 1125899906826241
    u = _poly(orc, 0, 4, 60_000, q=q)
    assert u.max() < q
    hist = np.bincount((u.astype(np.float64) / q * 16).astype(np.int64), minlength=16)
    assert np.all(np.abs(hist - 3750) < 300)


def test_streams_are_separated(orc):
    """Different objects and tags give different streams."""
    a = _poly(orc, 3, 9, 256, obj=0, ell=40)
    b = _poly(orc, 3, 9, 256, obj=1, ell=40)
    c = _poly(orc, 3, 5, 256, obj=0, ell=40)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
