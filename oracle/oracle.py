"""Plain CPU oracle for Pi_MatMul (Algorithm 1, section 3.1.1) over RNS-BFV
(section 2.2) of Liu & Liu, arXiv 2305.18396.

TEST INFRASTRUCTURE ONLY.  This module and the C library beside it are the
parity authority for the HIP library.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it.  It shares no code
with the GPU path and imports nothing from the package.

The slow, direct parts (ChaCha20 streams, negacyclic products, the protocol
steps one ciphertext at a time) live in ``pimm_oracle.c``; this file holds the
parameter rule, the block plan, the encodings of Algorithm 1 step 1, and the
decryption's CRT and rounding in exact Python integers.

Readings where the paper is silent (all listed with their reasons in the
design notes): primes are the L largest primes below 2^50 congruent to 1 mod
2N; encryption is symmetric; the plaintext A is lifted centred; the reply is
re-randomised by a public-key encryption of zero when requested; the mask is
subtracted as Delta * s; the decrypt rounding is round-half-up (ties cannot
occur since t = 2^l and q is odd).  Modulus switching of the reply (an
optional wire format, not in the paper) rounds c q'/q to the nearest integer,
q' the product of the first L - 1 primes.

Parity unpinned: the block-plan rules (plan_comm, plan_fix) and the stream
layout's choices (tag numbers, which nonce word holds what).  They are spec
decisions the paper leaves open; only the protocol invariants (the shares add
up to X W for any plan, the keystream is RFC 8439's) tie them to the paper.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from decimal import Decimal, getcontext

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpimm_oracle.so")

# Stream tags (the same meaning as in pimm_oracle.c).
TAG_SK, TAG_PK_A, TAG_PK_E, TAG_ENC_A, TAG_ENC_E = 1, 2, 3, 4, 5
TAG_RR_U, TAG_RR_E1, TAG_RR_E2, TAG_MASK = 6, 7, 8, 9

SIGMA = 3.2
CDT_LEN = 19
PRIME_BITS = 50

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the C part of the oracle with gcc (OpenMP, -O2)."""
    import subprocess

    src = os.path.join(_HERE, "pimm_oracle.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    """The loaded oracle C library (built on first use if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
        u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        _lib.orc_chacha20_block.argtypes = [vp, u32, vp, vp]
        _lib.orc_draw64.argtypes = [vp, u32, u32, u32, u32, u64]
        _lib.orc_draw64.restype = u64
        _lib.orc_sample_poly.argtypes = [ctypes.c_int, vp, u32, u32, u32, u32, u64, u64,
                                         ctypes.c_uint, vp, vp]
        _lib.orc_ntt_negacyclic.argtypes = [vp, vp, u64, u64, u64]
        _lib.orc_intt_negacyclic.argtypes = [vp, vp, u64, u64, u64]
        _lib.orc_negacyclic_mul.argtypes = [vp, vp, vp, u64, u64, u64]
        _lib.orc_negacyclic_mul_schoolbook.argtypes = [vp, vp, vp, u64, u64]
        _lib.orc_keygen.argtypes = [u64, u64, vp, vp, vp, vp, vp, vp]
        _lib.orc_encrypt.argtypes = [u64, u64, vp, vp, vp, vp, vp, u32, vp, vp, u64, vp]
        _lib.orc_encrypt_seeded.argtypes = [u64, u64, vp, vp, vp, vp, vp, vp, u32, vp, vp, u64, vp]
        _lib.orc_ctpt_matmul.argtypes = [u64, u64, vp, vp, u64, u64, vp, vp, vp, u64, vp]
        _lib.orc_rerandomize.argtypes = [u64, u64, vp, vp, vp, vp, u32, vp, vp, u64, vp]
        _lib.orc_mask_extract.argtypes = [u64, u64, vp, vp, ctypes.c_uint, vp, u32, u64, u64, u64,
                                          vp, u64, vp, vp, vp, vp]
        _lib.orc_decrypt_residues.argtypes = [u64, u64, vp, vp, vp, u64, u64, u64, u64, vp, vp, vp]
        _lib.orc_decrypt_full_residues.argtypes = [u64, u64, vp, vp, vp, u64, vp, ctypes.c_int, vp]
        _lib.orc_slot_index.argtypes = [u64, u64]
        _lib.orc_slot_index.restype = u64
        _lib.orc_slots_to_coef.argtypes = [vp, vp, u64, u64, u64]
        _lib.orc_coef_to_slots.argtypes = [vp, vp, u64, u64, u64]
        _lib.orc_max_threads.restype = ctypes.c_int
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)


def _key(seed: bytes) -> np.ndarray:
    assert len(seed) == 32
    return np.frombuffer(bytes(seed), dtype=np.uint8).copy()


def max_threads() -> int:
    return int(lib().orc_max_threads())


# ---------------------------------------------------------------------------
# Parameters (section 2.2: BFV with N a power of two, t = 2^l, RNS modulus q)
# ---------------------------------------------------------------------------

def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin; the first 12 prime bases decide every n < 3.3e24."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def find_primes(N: int, L: int, bits: int = PRIME_BITS) -> list[int]:
    """The L largest primes q < 2^bits with q = 1 (mod 2N), in descending order."""
    out = []
    k = ((1 << bits) - 2) // (2 * N)
    while len(out) < L:
        cand = k * 2 * N + 1
        if cand < (1 << bits) and is_prime(cand):
            out.append(cand)
        k -= 1
    return out


def find_psi(q: int, N: int) -> int:
    """A primitive 2N-th root of unity mod q: g^((q-1)/2N) for the first g giving psi^N = -1.
    Nothing in NTT form crosses the protocol's wire, so any such root is valid."""
    e = (q - 1) // (2 * N)
    for g in range(2, 1 << 16):
        psi = pow(g, e, q)
        if pow(psi, N, q) == q - 1:
            return psi
    raise ValueError("no primitive root found")


def cdt_table(sigma: float = SIGMA, length: int = CDT_LEN) -> list[int]:
    """T[k] = floor(2^63 * F(k)) for k < length, F(k) = P(|e| <= k) for the discrete Gaussian
    rho(x) = exp(-x^2 / (2 sigma^2)) restricted to |x| <= length.  60-digit decimal arithmetic."""
    getcontext().prec = 60
    s2 = 2 * Decimal(str(sigma)) ** 2
    rho = [(-(Decimal(x) ** 2) / s2).exp() for x in range(length + 1)]
    total = rho[0] + 2 * sum(rho[1:])
    out, acc = [], rho[0]
    for k in range(length):
        out.append(int((acc / total) * (Decimal(2) ** 63)))  # int() truncates = floor (positive)
        acc += 2 * rho[k + 1]
    return out


@dataclass
class Params:
    """RNS-BFV parameters: ring degree N, L primes of 50 bits, t = 2^ell, f fractional bits."""
    N: int
    L: int
    ell: int
    frac_bits: int
    rerandomize: bool = True
    q: list = field(default_factory=list)
    psi: list = field(default_factory=list)
    cdt: list = field(default_factory=list)

    def __post_init__(self):
        assert self.N & (self.N - 1) == 0 and self.N >= 2
        if not self.q:
            self.q = find_primes(self.N, self.L)
        if not self.psi:
            self.psi = [find_psi(q, self.N) for q in self.q]
        if not self.cdt:
            self.cdt = cdt_table()
        self.t = 1 << self.ell
        self.Q = math.prod(self.q)
        self.Delta = self.Q // self.t
        self.delta_l = [self.Delta % q for q in self.q]

    # ctypes views
    @property
    def q_arr(self):
        return _u64(self.q)

    @property
    def psi_arr(self):
        return _u64(self.psi)

    @property
    def cdt_arr(self):
        return _u64(self.cdt)

    @property
    def delta_arr(self):
        return _u64(self.delta_l)


# ---------------------------------------------------------------------------
# Block plan (section 3.1.1: larger matrices are split into blocks; the rule is
# not given, so the rules below are the design's reading)
# ---------------------------------------------------------------------------

def _ceil(a, b):
    return -(-a // b)


def _next_pow2(x):
    return 1 << max(0, (x - 1).bit_length())


@dataclass
class Plan:
    """A = W^T (m x r, server), B = X^T (r x n, client); blocks of (mb, rb, nb), mb*rb*nb <= N."""
    n: int
    r: int
    m: int
    mb: int
    rb: int
    nb: int
    N: int

    def __post_init__(self):
        assert self.mb * self.rb * self.nb <= self.N
        self.M = _ceil(self.m, self.mb)
        self.R = _ceil(self.r, self.rb)
        self.K = _ceil(self.n, self.nb)
        self.I = self.R * self.K
        self.O = self.M * self.K
        self.Wb = self.M * self.R
        self.P = self.M * self.R * self.K

    def pos(self, i, k):
        """Decoded coefficient of output (i, k) inside a block: k*mb*rb + i*rb + rb - 1."""
        return k * self.mb * self.rb + i * self.rb + self.rb - 1


def plan_comm(N: int, n: int, r: int, m: int) -> Plan:
    """Fewest ciphertexts on the wire: minimise (ceil(r/rb) + ceil(m/mb)) * ceil(n/nb) over
    powers of two mb <= nextpow2(m), rb <= nextpow2(r), mb*rb <= N, with nb = min(n, N/(mb rb)).
    Ties go to larger nb, then larger mb."""
    best = None
    mb = 1
    while mb <= min(_next_pow2(m), N):
        rb = 1
        while rb <= _next_pow2(r) and mb * rb <= N:
            nb = min(n, N // (mb * rb))
            cost = (_ceil(r, rb) + _ceil(m, mb)) * _ceil(n, nb)
            key = (cost, -nb, -mb)
            if best is None or key < best[0]:
                best = (key, (mb, rb, nb))
            rb *= 2
        mb *= 2
    mb, rb, nb = best[1]
    return Plan(n, r, m, mb, rb, nb, N)


def plan_fix(N: int, D: int, n: int, r: int, m: int) -> Plan:
    """Fixed block area mb*rb = D (a power of two <= N): split to minimise ceil(r/rb) + ceil(m/mb),
    ties to larger mb; nb = min(n, N/D)."""
    best = None
    mb = 1
    while mb <= D:
        rb = D // mb
        cost = _ceil(r, rb) + _ceil(m, mb)
        key = (cost, -mb)
        if best is None or key < best[0]:
            best = (key, (mb, rb))
        mb *= 2
    mb, rb = best[1]
    return Plan(n, r, m, mb, rb, min(n, N // D), N)


# ---------------------------------------------------------------------------
# Encodings (Algorithm 1, step 1)
# ---------------------------------------------------------------------------

def encode_input(plan: Plan, X: np.ndarray) -> np.ndarray:
    """pi_B per block: pt[jb*K + kb][k*mb*rb + j] = X[kb*nb + k][jb*rb + j] (B = X^T);
    coefficients outside the matrix are 0.  X: [n][r] values < 2^ell."""
    X = np.asarray(X, dtype=np.uint64)
    assert X.shape == (plan.n, plan.r)
    pt = np.zeros((plan.I, plan.N), dtype=np.uint64)
    # Every (row, col) of X lands in exactly one block and one coefficient.
    row, col = np.meshgrid(np.arange(plan.n), np.arange(plan.r), indexing="ij")
    kb, k = np.divmod(row, plan.nb)
    jb, j = np.divmod(col, plan.rb)
    pt[jb * plan.K + kb, k * plan.mb * plan.rb + j] = X[row, col]
    return pt


def encode_weights(plan: Plan, W: np.ndarray) -> np.ndarray:
    """pi_A per block: ptA[ib*R + jb][i*rb + rb - 1 - j] = W[jb*rb + j][ib*mb + i] (A = W^T),
    signed; other coefficients 0.  W: [r][m] signed fixed-point integers."""
    W = np.asarray(W, dtype=np.int64)
    assert W.shape == (plan.r, plan.m)
    pa = np.zeros((plan.Wb, plan.N), dtype=np.int64)
    row, col = np.meshgrid(np.arange(plan.r), np.arange(plan.m), indexing="ij")
    jb, j = np.divmod(row, plan.rb)
    ib, i = np.divmod(col, plan.mb)
    pa[ib * plan.R + jb, i * plan.rb + plan.rb - 1 - j] = W[row, col]
    return pa


# ---------------------------------------------------------------------------
# Protocol steps
# ---------------------------------------------------------------------------

def keygen(params: Params, seed: bytes, with_pk: bool | None = None):
    """Client key generation: ternary s; pk = ([-a's + e']_q, a') when re-randomisation is on."""
    with_pk = params.rerandomize if with_pk is None else with_pk
    N, L = params.N, params.L
    s = np.zeros(N, dtype=np.int64)
    pk = np.zeros((2, L, N), dtype=np.uint64) if with_pk else None
    lib().orc_keygen(N, L, _p(params.q_arr), _p(params.psi_arr), _p(_key(seed)),
                     _p(params.cdt_arr), _p(s), _p(pk) if pk is not None else None)
    return s, pk


def encrypt(params: Params, s: np.ndarray, seed: bytes, op_id: int, pt: np.ndarray) -> np.ndarray:
    """Algorithm 1 step 2: symmetric encryption of each plaintext row.  -> [count][2][L][N]
    in evaluation form (slot_index): c1's slots are the uniform draws of a, c0's are those of
    [Delta pt + e - a s]."""
    pt = _u64(pt)
    count = pt.shape[0]
    ct = np.zeros((count, 2, params.L, params.N), dtype=np.uint64)
    lib().orc_encrypt(params.N, params.L, _p(params.q_arr), _p(params.psi_arr),
                      _p(params.delta_arr), _p(np.ascontiguousarray(s, dtype=np.int64)),
                      _p(_key(seed)), op_id, _p(params.cdt_arr), _p(pt), count, _p(ct))
    return ct


def encrypt_seeded(params: Params, s: np.ndarray, seed: bytes, a_seed: bytes, op_id: int,
                   pt: np.ndarray) -> np.ndarray:
    """Seed-compressed upload (a wire-format variant of Algorithm 1 step 2): the symmetric
    encryption with c1 = a drawn from the public seed a_seed and e from the secret seed, so the
    client sends c0 and a_seed.  -> [count][2][L][N]; with a_seed = seed it equals encrypt()."""
    pt = _u64(pt)
    count = pt.shape[0]
    ct = np.zeros((count, 2, params.L, params.N), dtype=np.uint64)
    lib().orc_encrypt_seeded(params.N, params.L, _p(params.q_arr), _p(params.psi_arr),
                             _p(params.delta_arr), _p(np.ascontiguousarray(s, dtype=np.int64)),
                             _p(_key(seed)), _p(_key(a_seed)), op_id, _p(params.cdt_arr), _p(pt),
                             count, _p(ct))
    return ct


def expand_ct(params: Params, a_seed: bytes, op_id: int, c0: np.ndarray) -> np.ndarray:
    """The server's side of the seed-compressed upload: ct[x][0] = c0[x] and
    ct[x][1][l] = a_l regenerated from a_seed (stream tag 4, prime l, op_id, object x)."""
    c0 = _u64(c0)
    count = c0.shape[0]
    ct = np.zeros((count, 2, params.L, params.N), dtype=np.uint64)
    ct[:, 0] = c0
    key = _key(a_seed)
    for x in range(count):
        for l in range(params.L):
            a = np.zeros(params.N, dtype=np.uint64)
            lib().orc_sample_poly(0, _p(key), TAG_ENC_A, l, op_id, x, params.N, int(params.q_arr[l]),
                                  0, _p(params.cdt_arr), _p(a))
            ct[x, 1, l] = a
    return ct

def matmul(params: Params, plan: Plan, ptA: np.ndarray, ct: np.ndarray, outs=None) -> np.ndarray:
    """Algorithm 1 step 3 ([[c]] = a * [[b]]) summed over the inner blocks, for the requested
    output ciphertexts (all by default).  -> [len(outs)][2][L][N] in coefficient form."""
    outs = np.arange(plan.O, dtype=np.uint32) if outs is None else np.asarray(outs, np.uint32)
    acc = np.zeros((len(outs), 2, params.L, params.N), dtype=np.uint64)
    lib().orc_ctpt_matmul(params.N, params.L, _p(params.q_arr), _p(params.psi_arr), plan.R,
                          plan.K, _p(np.ascontiguousarray(ptA, dtype=np.int64)), _p(_u64(ct)),
                          _p(outs), len(outs), _p(acc))
    return acc


def rerandomize(params: Params, pk: np.ndarray, seed: bytes, op_id: int, acc: np.ndarray,
                outs) -> np.ndarray:
    """acc + Enc_pk(0) per output ciphertext (in place on a copy)."""
    acc = _u64(acc).copy()
    outs = np.asarray(outs, np.uint32)
    lib().orc_rerandomize(params.N, params.L, _p(params.q_arr), _p(params.psi_arr), _p(_u64(pk)),
                          _p(_key(seed)), op_id, _p(params.cdt_arr), _p(outs), len(outs), _p(acc))
    return acc


def mask_extract(params: Params, plan: Plan, seed: bytes, op_id: int, acc: np.ndarray, outs):
    """Algorithm 1 step 3 ([[c]] - s) and the sparse reply of section 3.1.3.
    -> (c1 [o][L][N], c0s [o][L][mb*nb], smask [o][mb*nb])."""
    outs = np.asarray(outs, np.uint32)
    no = len(outs)
    c1 = np.zeros((no, params.L, params.N), dtype=np.uint64)
    c0s = np.zeros((no, params.L, plan.mb * plan.nb), dtype=np.uint64)
    sm = np.zeros((no, plan.mb * plan.nb), dtype=np.uint64)
    lib().orc_mask_extract(params.N, params.L, _p(params.q_arr), _p(params.delta_arr), params.ell,
                           _p(_key(seed)), op_id, plan.mb, plan.rb, plan.nb, _p(outs), no,
                           _p(_u64(acc)), _p(c1), _p(c0s), _p(sm))
    return c1, c0s, sm


def crt_round(params: Params, x: np.ndarray) -> np.ndarray:
    """BFV decryption rounding: x = CRT(residues) in [0, q), v = floor((t*x + floor(q/2)) / q)
    mod t, in exact Python integers.  x: [..., L] residues -> [...] uint64."""
    x = np.asarray(x, dtype=np.uint64)
    shape = x.shape[:-1]
    flat = x.reshape(-1, params.L)
    Q, t = params.Q, params.t
    coef = []
    for q in params.q:
        Ml = Q // q
        coef.append(Ml * pow(Ml, -1, q))
    out = np.zeros(flat.shape[0], dtype=np.uint64)
    half = Q // 2
    for idx in range(flat.shape[0]):
        v = sum(int(flat[idx, l]) * coef[l] for l in range(params.L)) % Q
        out[idx] = ((t * v + half) // Q) % t
    return out.reshape(shape)


def decrypt_residues(params: Params, plan: Plan, s: np.ndarray, c1: np.ndarray,
                     c0s: np.ndarray) -> np.ndarray:
    """Residues of m = c0 + c1*s at the decoded positions.  -> [o][mb*nb][L]."""
    no = c1.shape[0]
    x = np.zeros((no, plan.mb * plan.nb, params.L), dtype=np.uint64)
    lib().orc_decrypt_residues(params.N, params.L, _p(params.q_arr), _p(params.psi_arr),
                               _p(np.ascontiguousarray(s, dtype=np.int64)), plan.mb, plan.rb,
                               plan.nb, no, _p(_u64(c1)), _p(_u64(c0s)), _p(x))
    return x


def decrypt_full(params: Params, s: np.ndarray, ct: np.ndarray, query: bool = False) -> np.ndarray:
    """Decrypt every coefficient of whole ciphertexts [count][2][L][N] -> [count][N] in Z_t.
    query: in evaluation form (a query ciphertext from encrypt); else coefficient form (a
    product's output)."""
    ct = _u64(ct)
    count = ct.shape[0]
    x = np.zeros((count, params.N, params.L), dtype=np.uint64)
    lib().orc_decrypt_full_residues(params.N, params.L, _p(params.q_arr), _p(params.psi_arr),
                                    _p(np.ascontiguousarray(s, dtype=np.int64)), count, _p(ct),
                                    1 if query else 0, _p(x))
    return crt_round(params, x)


def slot_index(N: int) -> np.ndarray:
    """k[z]: slot z of the evaluation form holds the value at psi^(2k+1)."""
    return np.array([lib().orc_slot_index(z, N) for z in range(N)], dtype=np.uint64)


def slots_to_coef(params: Params, S: np.ndarray) -> np.ndarray:
    """Coefficients [..][L][N] of polynomials given by their slots [..][L][N]."""
    S = _u64(S)
    out = np.zeros_like(S)
    flat_s, flat_o = S.reshape(-1, params.L, params.N), out.reshape(-1, params.L, params.N)
    for i in range(flat_s.shape[0]):
        for l in range(params.L):
            src = np.ascontiguousarray(flat_s[i, l])
            dst = np.zeros(params.N, np.uint64)
            lib().orc_slots_to_coef(_p(src), _p(dst), params.N, int(params.q[l]), int(params.psi[l]))
            flat_o[i, l] = dst
    return out


def coef_to_slots(params: Params, a: np.ndarray) -> np.ndarray:
    """Slots [..][L][N] of polynomials given by their coefficients [..][L][N]."""
    a = _u64(a)
    out = np.zeros_like(a)
    flat_a, flat_o = a.reshape(-1, params.L, params.N), out.reshape(-1, params.L, params.N)
    for i in range(flat_a.shape[0]):
        for l in range(params.L):
            src = np.ascontiguousarray(flat_a[i, l])
            dst = np.zeros(params.N, np.uint64)
            lib().orc_coef_to_slots(_p(src), _p(dst), params.N, int(params.q[l]), int(params.psi[l]))
            flat_o[i, l] = dst
    return out


def noise_of(params: Params, s: np.ndarray, ct: np.ndarray, expected: np.ndarray,
             query: bool = False) -> int:
    """Exact decryption noise max |[c0 + c1 s]_q - Delta*m| over the coefficients of ct,
    with m the expected plaintext [count][N] (centred representative mod q); query as for
    decrypt_full."""
    ct = _u64(ct)
    count = ct.shape[0]
    x = np.zeros((count, params.N, params.L), dtype=np.uint64)
    lib().orc_decrypt_full_residues(params.N, params.L, _p(params.q_arr), _p(params.psi_arr),
                                    _p(np.ascontiguousarray(s, dtype=np.int64)), count, _p(ct),
                                    1 if query else 0, _p(x))
    Q = params.Q
    coef = [(Q // q) * pow(Q // q, -1, q) for q in params.q]
    worst = 0
    for o in range(count):
        for j in range(params.N):
            v = sum(int(x[o, j, l]) * coef[l] for l in range(params.L)) % Q
            d = (v - params.Delta * int(expected[o][j])) % Q
            if d > Q // 2:
                d -= Q
            worst = max(worst, abs(d))
    return worst


def place_shares(plan: Plan, vals: np.ndarray, outs, out: np.ndarray | None = None) -> np.ndarray:
    """pi_C^{-1} (Algorithm 1 step 4) per block: entry (k*mb + i) of output ciphertext
    y = ib*K + kb goes to Y[kb*nb + k][ib*mb + i]; padded rows/columns are dropped."""
    Y = np.zeros((plan.n, plan.m), dtype=np.uint64) if out is None else out
    for o, y in enumerate(np.asarray(outs).tolist()):
        ib, kb = divmod(int(y), plan.K)
        for k in range(plan.nb):
            row = kb * plan.nb + k
            if row >= plan.n:
                break
            for i in range(plan.mb):
                col = ib * plan.mb + i
                if col >= plan.m:
                    break
                Y[row, col] = vals[o, k * plan.mb + i]
    return Y


def decrypt(params: Params, plan: Plan, s: np.ndarray, c1: np.ndarray, c0s: np.ndarray,
            outs=None) -> np.ndarray:
    """Client decryption and decoding (Algorithm 1 step 4): the client's share [n][m]."""
    outs = np.arange(plan.O) if outs is None else outs
    v = crt_round(params, decrypt_residues(params, plan, s, c1, c0s))
    return place_shares(plan, v, outs)


def noise_bound(params: Params, plan: Plan, wmax: int) -> int:
    """Worst-case decryption noise |E| at a decoded coefficient of the reply, as an exact integer.
    With e_max = 19 (the Gaussian's tail cut) and D = mb*rb nonzero plaintext coefficients:
      R*D*wmax*e_max        the products a * e of every inner block,
      (q mod t)*(r*wmax+1)  Delta*t = q - (q mod t), so each multiple of t carried by the
                            integer product a*b (at most r*wmax of them) and the mask's
                            wrap past t leave (q mod t) behind,
      2*N*e_max + e_max     u*e' + e1 + e2*s of the re-randomisation (when it is on)."""
    emax = CDT_LEN
    D = plan.mb * plan.rb
    qt = params.Q % params.t
    b = plan.R * D * wmax * emax + qt * (plan.r * wmax + 1)
    if params.rerandomize:
        b += 2 * params.N * emax + emax
    return b


def noise_ok(params: Params, plan: Plan, wmax: int) -> bool:
    """Decryption rounds to the right value when t*|E - m*(q mod t)/t| < q/2 for every m < t,
    which 2*t*(E + (q mod t)) < q guarantees."""
    E = noise_bound(params, plan, wmax)
    return 2 * params.t * (E + params.Q % params.t) < params.Q


def pi_matmul(params: Params, plan: Plan, X: np.ndarray, W: np.ndarray, client_seed: bytes,
              server_seed: bytes, op_id: int = 0, outs=None, keys=None):
    """The whole protocol for one matrix product Y = X W (Algorithm 1 with A = W^T, B = X^T).
    Returns a dict with every intermediate.  outs restricts the server work and the decryption
    to a subset of output ciphertexts (for spot checks at full size)."""
    s, pk = keys if keys is not None else keygen(params, client_seed)
    pt = encode_input(plan, X)
    ptA = encode_weights(plan, W)
    ct = encrypt(params, s, client_seed, op_id, pt)
    outs = np.arange(plan.O, dtype=np.uint32) if outs is None else np.asarray(outs, np.uint32)
    acc = matmul(params, plan, ptA, ct, outs)
    if params.rerandomize:
        acc_rr = rerandomize(params, pk, server_seed, op_id, acc, outs)
    else:
        acc_rr = acc
    c1, c0s, sm = mask_extract(params, plan, server_seed, op_id, acc_rr, outs)
    Y0 = decrypt(params, plan, s, c1, c0s, outs)
    Y1 = place_shares(plan, sm, outs)
    return dict(s=s, pk=pk, pt=pt, ptA=ptA, ct=ct, acc=acc, acc_rr=acc_rr, c1=c1, c0s=c0s,
                smask=sm, Y0=Y0, Y1=Y1, outs=outs)


def pi_matmul_grouped(params: Params, plan: Plan, Xs, Ws, client_seed: bytes, server_seed: bytes,
                      op_id: int = 0, keys=None):
    """G products of one shape (one plan), Y_p = X_p W_p, run as one protocol call: the G
    inputs are encrypted together, input ciphertext x of product p being ciphertext p*I + x of
    the group, and output ciphertext y of product p being p*O + y of the group (the objects of
    the re-randomisation and mask streams).  Each product follows Algorithm 1 on its own
    blocks; only the stream objects tie them together.
    -> dict with the group's ct, acc, acc_rr, c1, c0s (stacked, product-major) and the shares
    Y0, Y1 [G][n][m]."""
    G = len(Xs)
    s, pk = keys if keys is not None else keygen(params, client_seed)
    pt = np.concatenate([encode_input(plan, X) for X in Xs])
    ct = encrypt(params, s, client_seed, op_id, pt)
    local = np.arange(plan.O, dtype=np.uint32)
    acc = np.concatenate([matmul(params, plan, encode_weights(plan, W), ct[p * plan.I:(p + 1) * plan.I],
                                 local) for p, W in enumerate(Ws)])
    group = np.arange(G * plan.O, dtype=np.uint32)
    acc_rr = rerandomize(params, pk, server_seed, op_id, acc, group) if params.rerandomize else acc
    c1, c0s, sm = mask_extract(params, plan, server_seed, op_id, acc_rr, group)
    v = crt_round(params, decrypt_residues(params, plan, s, c1, c0s))
    Y0 = np.stack([place_shares(plan, v[p * plan.O:(p + 1) * plan.O], local) for p in range(G)])
    Y1 = np.stack([place_shares(plan, sm[p * plan.O:(p + 1) * plan.O], local) for p in range(G)])
    return dict(s=s, pk=pk, pt=pt, ct=ct, acc=acc, acc_rr=acc_rr, c1=c1, c0s=c0s, smask=sm,
                Y0=Y0, Y1=Y1)


def fc_complete(params: Params, X1: np.ndarray, W: np.ndarray, bias, Y1: np.ndarray) -> np.ndarray:
    """Server side of a fully connected layer y = x W + b on additive shares (section 3.1, the
    linear layers).  The input x is shared as X0 (client) + X1 (server) mod 2^l; Pi_MatMul on
    X0 leaves the server with Y1, where Y0 + Y1 = X0 W.  The server holds X1, W and b, so it
    adds its local product and the bias:
        Y1' = Y1 + X1 W + b  (mod 2^l),   Y0 + Y1' = X W + b.
    b is at the scale of the product (2f fractional bits).  uint64 wrap-around arithmetic is
    exact mod 2^l; X1 is read mod 2^l."""
    mask = np.uint64(params.t - 1)
    Xu = np.asarray(X1, dtype=np.uint64) & mask
    Wu = np.asarray(W, dtype=np.int64).astype(np.uint64)
    out = np.asarray(Y1, dtype=np.uint64) + Xu @ Wu
    if bias is not None:
        out = out + np.asarray(bias, dtype=np.int64).astype(np.uint64)[None, :]
    return out & mask


# ---------------------------------------------------------------------------
# Modulus switching of the reply (a wire-format variant of the sparse reply of
# section 3.1.3: fewer residues per coefficient on the wire; not in the paper)
# ---------------------------------------------------------------------------

def switched_params(params: Params) -> Params:
    """Parameters of the reply after modulus switching: the first L - 1 primes,
    q' = q_0 ... q_{L-2} (the last prime is dropped)."""
    assert params.L >= 2
    return Params(params.N, params.L - 1, params.ell, params.frac_bits, params.rerandomize,
                  q=list(params.q[:-1]), psi=list(params.psi[:-1]), cdt=list(params.cdt))


def mod_switch(params: Params, x: np.ndarray) -> np.ndarray:
    """Modulus switching from q to q' = q / q_{L-1}, coefficient by coefficient, by its
    definition: each coefficient c in [0, q) (reconstructed from its L residues by the CRT,
    in exact integers) becomes round(c q' / q) = round(c / q_{L-1}) mod q' (never a tie:
    q_{L-1} is odd).  x: [..., L, count] residues -> [..., L-1, count] residues mod the
    first L-1 primes."""
    x = np.asarray(x, dtype=np.uint64)
    L = params.L
    assert x.shape[-2] == L
    Q = params.Q
    qd = params.q[-1]
    qs = Q // qd
    coef = [(Q // q) * pow(Q // q, -1, q) for q in params.q]
    lead = x.shape[:-2]
    count = x.shape[-1]
    flat = x.reshape(-1, L, count)
    out = np.zeros((flat.shape[0], L - 1, count), dtype=np.uint64)
    for o in range(flat.shape[0]):
        for j in range(count):
            c = sum(int(flat[o, l, j]) * coef[l] for l in range(L)) % Q
            cp = ((2 * c + qd) // (2 * qd)) % qs  # nearest integer to c / q_{L-1}
            for l in range(L - 1):
                out[o, l, j] = cp % params.q[l]
    return out.reshape(*lead, L - 1, count)


def noise_bound_switched(params: Params, plan: Plan, wmax: int) -> int:
    """Worst-case decryption noise of a switched reply coefficient: the reply's noise scaled
    by q'/q (rounded up) plus the rounding of c0 and of the N terms of c1 s (each |e| <= 1/2,
    |s_j| <= 1), i.e. ceil(E q'/q) + (N + 1) / 2 rounded up."""
    E = noise_bound(params, plan, wmax)
    qs = params.Q // params.q[-1]
    return -(-E * qs // params.Q) + (params.N + 2) // 2


def switch_ok(params: Params, plan: Plan, wmax: int) -> bool:
    """A switched reply decrypts to the same share when 2 t (E' + 1) < q' (the message's
    scale q' Delta / q differs from q'/t by less than one unit per t)."""
    qs = params.Q // params.q[-1]
    return 2 * params.t * (noise_bound_switched(params, plan, wmax) + 1) < qs
