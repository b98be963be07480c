/*
 * pimm_oracle.c -- plain CPU oracle for the private matrix-multiplication
 * protocol Pi_MatMul (Algorithm 1, section 3.1.1 of Liu & Liu, "LLMs Can
 * Understand Encrypted Prompt: Towards Privacy-Computing Friendly
 * Transformers", arXiv 2305.18396) over RNS-BFV (section 2.2).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the parity authority for the
 * HIP library.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header, table or constant
 * generator with the GPU path.
 *
 * Everything here is deliberately slow and direct:
 *   - modular products go through unsigned __int128 and '%';
 *   - the negacyclic product a*b mod (X^N+1, q) is a textbook one: twist by
 *     psi^j, iterative radix-2 cyclic NTT with omega = psi^2 (bit-reversal
 *     permutation first), pointwise product, inverse, untwist (the paper's
 *     footnote in section 3.1.3 says polynomial products go through NTT and
 *     elementwise multiplication); a schoolbook version sits beside it so
 *     tests can check one against the other;
 *   - every protocol step follows its definition, one ciphertext at a time.
 *
 * Randomness follows one counter-based generator, the ChaCha20 block
 * function of RFC 8439 section 2.3, implemented here from the RFC text:
 *   key     = the party's 32-byte seed,
 *   nonce   = (tag | prime_index << 8, op_id, object_index) as LE words,
 *   counter = block number, starting at 0.
 * The 64-bit draw number j is keystream bytes [8j, 8j+8) read little-endian.
 * A uniform residue that the first draw cannot give (rejection) comes from the
 * stream's fallback stream, whose tag word has bit 31 set.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* Stream tags (which random object a stream feeds). */
enum {
    TAG_SK = 1,    /* secret key s, ternary */
    TAG_PK_A = 2,  /* public key uniform part a', per prime */
    TAG_PK_E = 3,  /* public key error e' */
    TAG_ENC_A = 4, /* encryption uniform part a, per prime */
    TAG_ENC_E = 5, /* encryption error e */
    TAG_RR_U = 6,  /* re-randomisation ternary u */
    TAG_RR_E1 = 7, /* re-randomisation error on component 0 */
    TAG_RR_E2 = 8, /* re-randomisation error on component 1 */
    TAG_MASK = 9   /* server mask polynomial over Z_t */
};

#define CDT_LEN 19

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* ChaCha20 block function (RFC 8439, section 2.3)                     */
/* ------------------------------------------------------------------ */

static uint32_t rotl32(uint32_t v, int c) { return (v << c) | (v >> (32 - c)); }

static void quarter_round(uint32_t *x, int a, int b, int c, int d)
{
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 16);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 12);
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 8);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 7);
}

void orc_chacha20_block(const uint8_t key[32], uint32_t counter, const uint32_t nonce[3],
                        uint32_t out[16])
{
    uint32_t init[16], x[16];
    init[0] = 0x61707865u; /* "expa" */
    init[1] = 0x3320646eu; /* "nd 3" */
    init[2] = 0x79622d32u; /* "2-by" */
    init[3] = 0x6b206574u; /* "te k" */
    for (int i = 0; i < 8; ++i)
        init[4 + i] = (uint32_t)key[4 * i] | ((uint32_t)key[4 * i + 1] << 8) |
                      ((uint32_t)key[4 * i + 2] << 16) | ((uint32_t)key[4 * i + 3] << 24);
    init[12] = counter;
    init[13] = nonce[0];
    init[14] = nonce[1];
    init[15] = nonce[2];
    memcpy(x, init, sizeof x);
    for (int r = 0; r < 10; ++r) {
        /* column round */
        quarter_round(x, 0, 4, 8, 12);
        quarter_round(x, 1, 5, 9, 13);
        quarter_round(x, 2, 6, 10, 14);
        quarter_round(x, 3, 7, 11, 15);
        /* diagonal round */
        quarter_round(x, 0, 5, 10, 15);
        quarter_round(x, 1, 6, 11, 12);
        quarter_round(x, 2, 7, 8, 13);
        quarter_round(x, 3, 4, 9, 14);
    }
    for (int i = 0; i < 16; ++i) out[i] = x[i] + init[i];
}

static void stream_nonce(uint32_t tag, uint32_t prime, uint32_t op, uint32_t obj, uint32_t n[3])
{
    n[0] = tag | (prime << 8);
    n[1] = op;
    n[2] = obj;
}

/* 64-bit draw number j of stream (tag, prime, op, obj). */
uint64_t orc_draw64(const uint8_t key[32], uint32_t tag, uint32_t prime, uint32_t op, uint32_t obj,
                    uint64_t j)
{
    uint32_t n[3], b[16];
    stream_nonce(tag, prime, op, obj, n);
    orc_chacha20_block(key, (uint32_t)(j / 8), n, b);
    int w = (int)(2 * (j % 8));
    return (uint64_t)b[w] | ((uint64_t)b[w + 1] << 32);
}

/* ------------------------------------------------------------------ */
/* Samplers                                                            */
/* ------------------------------------------------------------------ */

/* The fallback stream of (tag, prime, op, obj): bit 31 of the tag word set. */
#define FALLBACK_TAG 0x80000000u

/* Uniform residue mod q (q < 2^50) by rejection: x = the low 50 bits of draw j,
 * kept when x < q; otherwise x' = the low 50 bits of draw j of the fallback
 * stream, reduced mod q.  For the primes of the parameter rule (within 2^21 of
 * 2^50) a draw is rejected with probability below 2^-29, and the residue is
 * uniform up to a statistical distance below 2^-58. */
static uint64_t sample_uniform(const uint8_t key[32], uint32_t tag, uint32_t prime, uint32_t op,
                               uint32_t obj, uint64_t j, uint64_t q)
{
    const uint64_t m50 = (1ull << 50) - 1;
    uint64_t x = orc_draw64(key, tag, prime, op, obj, j) & m50;
    if (x < q) return x;
    x = orc_draw64(key, tag | FALLBACK_TAG, prime, op, obj, j) & m50;
    return x % q;
}

/* Ternary value in {-1, 0, 1}: (64-bit draw mod 3) - 1. */
static int64_t sample_ternary(const uint8_t key[32], uint32_t tag, uint32_t op, uint32_t obj,
                              uint64_t j)
{
    return (int64_t)(orc_draw64(key, tag, 0, op, obj, j) % 3u) - 1;
}

/* Element of Z_{2^ell}: the low ell bits of the 64-bit draw. */
static uint64_t sample_mask(const uint8_t key[32], uint32_t tag, uint32_t op, uint32_t obj,
                            uint64_t j, unsigned ell)
{
    uint64_t v = orc_draw64(key, tag, 0, op, obj, j);
    return ell >= 64 ? v : (v & ((1ull << ell) - 1));
}

/* Discrete Gaussian by cumulative table: with u the low 63 bits of the draw,
 * |e| is the number of table entries T[k] with u >= T[k]; bit 63 is the sign. */
static int64_t sample_gauss(const uint8_t key[32], uint32_t tag, uint32_t op, uint32_t obj,
                            uint64_t j, const uint64_t *cdt)
{
    uint64_t v = orc_draw64(key, tag, 0, op, obj, j);
    uint64_t u = v & 0x7fffffffffffffffull;
    int64_t mag = 0;
    for (int k = 0; k < CDT_LEN; ++k)
        if (u >= cdt[k]) mag += 1;
    return (v >> 63) ? -mag : mag;
}

/* Sample a whole polynomial of n coefficients; kind: 0 uniform mod q,
 * 1 ternary, 2 gaussian, 3 mask mod 2^ell.  Signed kinds write int64. */
void orc_sample_poly(int kind, const uint8_t key[32], uint32_t tag, uint32_t prime, uint32_t op,
                     uint32_t obj, uint64_t n, uint64_t q, unsigned ell, const uint64_t *cdt,
                     void *out)
{
    for (uint64_t j = 0; j < n; ++j) {
        switch (kind) {
        case 0: ((uint64_t *)out)[j] = sample_uniform(key, tag, prime, op, obj, j, q); break;
        case 1: ((int64_t *)out)[j] = sample_ternary(key, tag, op, obj, j); break;
        case 2: ((int64_t *)out)[j] = sample_gauss(key, tag, op, obj, j, cdt); break;
        default: ((uint64_t *)out)[j] = sample_mask(key, tag, op, obj, j, ell); break;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Modular arithmetic                                                  */
/* ------------------------------------------------------------------ */

static uint64_t mulm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static uint64_t addm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static uint64_t subm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - b) % q); }

static uint64_t powm(uint64_t a, uint64_t e, uint64_t q)
{
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulm(r, a, q);
        a = mulm(a, a, q);
        e >>= 1;
    }
    return r;
}

/* Inverse mod a prime q by Fermat's little theorem. */
static uint64_t invm(uint64_t a, uint64_t q) { return powm(a, q - 2, q); }

/* Signed integer -> residue mod q (negative x maps to q - |x|). */
static uint64_t lift(int64_t x, uint64_t q)
{
    if (x >= 0) return (uint64_t)x % q;
    uint64_t m = (uint64_t)(-(x + 1)) + 1; /* |x| without overflow */
    m %= q;
    return m == 0 ? 0 : q - m;
}

/* ------------------------------------------------------------------ */
/* Textbook NTT and negacyclic products                                */
/* ------------------------------------------------------------------ */

/* In-place cyclic NTT of length n (a power of two): A_k = sum_j a_j omega^(jk).
 * Iterative radix-2 Cooley-Tukey: bit-reversal permutation, then log2(n)
 * butterfly levels of doubling length. */
static void ntt_cyclic(uint64_t *a, uint64_t n, uint64_t omega, uint64_t q)
{
    for (uint64_t i = 1, j = 0; i < n; ++i) {
        uint64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            uint64_t t = a[i];
            a[i] = a[j];
            a[j] = t;
        }
    }
    for (uint64_t len = 2; len <= n; len <<= 1) {
        uint64_t wlen = powm(omega, n / len, q);
        for (uint64_t i = 0; i < n; i += len) {
            uint64_t w = 1;
            for (uint64_t j = 0; j < len / 2; ++j) {
                uint64_t u = a[i + j];
                uint64_t v = mulm(a[i + j + len / 2], w, q);
                a[i + j] = addm(u, v, q);
                a[i + j + len / 2] = subm(u, v, q);
                w = mulm(w, wlen, q);
            }
        }
    }
}

/* Negacyclic NTT: A_k = a(psi^(2k+1)) = sum_j (a_j psi^j) omega^(jk), omega = psi^2.
 * psi must be a primitive 2n-th root of unity mod q. */
void orc_ntt_negacyclic(const uint64_t *a, uint64_t *A, uint64_t n, uint64_t q, uint64_t psi)
{
    uint64_t pw = 1;
    for (uint64_t j = 0; j < n; ++j) {
        A[j] = mulm(a[j] % q, pw, q);
        pw = mulm(pw, psi, q);
    }
    ntt_cyclic(A, n, mulm(psi, psi, q), q);
}

/* Inverse of orc_ntt_negacyclic. */
void orc_intt_negacyclic(const uint64_t *A, uint64_t *a, uint64_t n, uint64_t q, uint64_t psi)
{
    uint64_t psi_inv = invm(psi, q);
    uint64_t n_inv = invm(n % q, q);
    memcpy(a, A, n * sizeof(uint64_t));
    ntt_cyclic(a, n, mulm(psi_inv, psi_inv, q), q);
    uint64_t pw = n_inv;
    for (uint64_t j = 0; j < n; ++j) {
        a[j] = mulm(a[j], pw, q);
        pw = mulm(pw, psi_inv, q);
    }
}

/* c = a * b mod (X^n + 1, q) through the negacyclic NTT.  c may alias a or b. */
void orc_negacyclic_mul(const uint64_t *a, const uint64_t *b, uint64_t *c, uint64_t n, uint64_t q,
                        uint64_t psi)
{
    uint64_t *A = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint64_t *B = (uint64_t *)malloc(n * sizeof(uint64_t));
    orc_ntt_negacyclic(a, A, n, q, psi);
    orc_ntt_negacyclic(b, B, n, q, psi);
    for (uint64_t k = 0; k < n; ++k) A[k] = mulm(A[k], B[k], q);
    orc_intt_negacyclic(A, c, n, q, psi);
    free(A);
    free(B);
}

/* Evaluation form of a query ciphertext (how both of its components travel): slot z
 * of an n-coefficient polynomial holds its value at psi^(2k+1) with
 * k = brv(16 (z mod n/16) + floor(z / (n/16))), brv reversing log2(n) bits.
 * (n >= 16, a power of two.) */
uint64_t orc_slot_index(uint64_t z, uint64_t n)
{
    uint64_t m = n / 16, e = 16 * (z % m) + z / m, k = 0;
    for (uint64_t b = 1; b < n; b <<= 1) {
        k = (k << 1) | (e & 1);
        e >>= 1;
    }
    return k;
}

/* Coefficients of the polynomial whose slots are S (evaluation form -> coefficients). */
void orc_slots_to_coef(const uint64_t *S, uint64_t *a, uint64_t n, uint64_t q, uint64_t psi)
{
    uint64_t *A = (uint64_t *)malloc(n * sizeof(uint64_t));
    for (uint64_t z = 0; z < n; ++z) A[orc_slot_index(z, n)] = S[z] % q;
    orc_intt_negacyclic(A, a, n, q, psi);
    free(A);
}

/* Slots of the polynomial a (coefficients -> evaluation form). */
void orc_coef_to_slots(const uint64_t *a, uint64_t *S, uint64_t n, uint64_t q, uint64_t psi)
{
    uint64_t *A = (uint64_t *)malloc(n * sizeof(uint64_t));
    orc_ntt_negacyclic(a, A, n, q, psi);
    for (uint64_t z = 0; z < n; ++z) S[z] = A[orc_slot_index(z, n)];
    free(A);
}


/* c = a * b mod (X^n + 1, q) by the schoolbook definition:
 * c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+n} a_i b_j. */
void orc_negacyclic_mul_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *c, uint64_t n,
                                   uint64_t q)
{
    uint64_t *r = (uint64_t *)calloc(n, sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i)
        for (uint64_t j = 0; j < n; ++j) {
            uint64_t p = mulm(a[i] % q, b[j] % q, q);
            uint64_t k = i + j;
            if (k < n)
                r[k] = addm(r[k], p, q);
            else
                r[k - n] = subm(r[k - n], p, q);
        }
    memcpy(c, r, n * sizeof(uint64_t));
    free(r);
}

/* ------------------------------------------------------------------ */
/* Protocol steps                                                      */
/* ------------------------------------------------------------------ */

/* Key generation (client).  s_j ternary from stream (SK, 0, 0, 0).  If pk is
 * not NULL, also pk = ([-a'*s + e']_q, a') with a' uniform per prime from
 * (PK_A, l, 0, 0) and e' Gaussian from (PK_E, 0, 0, 0).  pk layout [2][L][n]. */
void orc_keygen(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                const uint8_t key[32], const uint64_t *cdt, int64_t *s, uint64_t *pk)
{
    orc_sample_poly(1, key, TAG_SK, 0, 0, 0, n, 0, 0, cdt, s);
    if (!pk) return;
    int64_t *e = (int64_t *)malloc(n * sizeof(int64_t));
    uint64_t *sl = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint64_t *as = (uint64_t *)malloc(n * sizeof(uint64_t));
    orc_sample_poly(2, key, TAG_PK_E, 0, 0, 0, n, 0, 0, cdt, e);
    for (uint64_t l = 0; l < L; ++l) {
        uint64_t *pk0 = pk + (0 * L + l) * n;
        uint64_t *pk1 = pk + (1 * L + l) * n;
        orc_sample_poly(0, key, TAG_PK_A, (uint32_t)l, 0, 0, n, q[l], 0, cdt, pk1);
        for (uint64_t j = 0; j < n; ++j) sl[j] = lift(s[j], q[l]);
        orc_negacyclic_mul(pk1, sl, as, n, q[l], psi[l]);
        for (uint64_t j = 0; j < n; ++j) pk0[j] = addm(subm(0, as[j], q[l]), lift(e[j], q[l]), q[l]);
    }
    free(e);
    free(sl);
    free(as);
}

/* Symmetric BFV encryption (Algorithm 1, step 2: the client encrypts b).
 * For ciphertext x (0 <= x < count), with e Gaussian from (ENC_E, 0, op, x) and
 * the n uniform draws of (ENC_A, l, op, x) taken as the slots of a_l (its
 * evaluation form, orc_slot_index; a uniform set of evaluations is a uniform
 * polynomial):
 *     c1_l = the slots of a_l,   c0_l = the slots of [Delta_l * pt + e - a_l * s]_{q_l}.
 * The whole ciphertext travels in evaluation form (the slot form is a ring
 * isomorphism, so it is the same ciphertext): the server's product is slot-wise.
 * pt: [count][n] plaintext coefficients in [0, t); ct: [count][2][L][n]. */
void orc_encrypt(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                 const uint64_t *delta_l, const int64_t *s, const uint8_t key[32], uint32_t op,
                 const uint64_t *cdt, const uint64_t *pt, uint64_t count, uint64_t *ct)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t xi = 0; xi < (int64_t)count; ++xi) {
        uint64_t x = (uint64_t)xi;
        int64_t *e = (int64_t *)malloc(n * sizeof(int64_t));
        uint64_t *sl = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *as = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *ac = (uint64_t *)malloc(n * sizeof(uint64_t));
        orc_sample_poly(2, key, TAG_ENC_E, 0, op, (uint32_t)x, n, 0, 0, cdt, e);
        for (uint64_t l = 0; l < L; ++l) {
            uint64_t *c0 = ct + ((x * 2 + 0) * L + l) * n;
            uint64_t *c1 = ct + ((x * 2 + 1) * L + l) * n;
            /* a is drawn in evaluation form (the uniform draws are its slots) and
             * travels that way; c0 is computed from coefficients, then sent as slots. */
            orc_sample_poly(0, key, TAG_ENC_A, (uint32_t)l, op, (uint32_t)x, n, q[l], 0, cdt, c1);
            orc_slots_to_coef(c1, ac, n, q[l], psi[l]);
            for (uint64_t j = 0; j < n; ++j) sl[j] = lift(s[j], q[l]);
            orc_negacyclic_mul(ac, sl, as, n, q[l], psi[l]);
            for (uint64_t j = 0; j < n; ++j) {
                uint64_t m = mulm(delta_l[l], pt[x * n + j] % q[l], q[l]);
                ac[j] = subm(addm(m, lift(e[j], q[l]), q[l]), as[j], q[l]);
            }
            orc_coef_to_slots(ac, c0, n, q[l], psi[l]);
        }
        free(e);
        free(sl);
        free(as);
        free(ac);
    }
}

/* Seed-compressed upload, a wire-format variant of Algorithm 1 step 2: the
 * same symmetric encryption with a_l drawn from a public key (a_key, tag 4)
 * and e from the secret key (e_key, tag 5), so that c1 can be regenerated by
 * the server from a_key.  With a_key = e_key this is orc_encrypt. */
void orc_encrypt_seeded(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                        const uint64_t *delta_l, const int64_t *s, const uint8_t e_key[32],
                        const uint8_t a_key[32], uint32_t op, const uint64_t *cdt,
                        const uint64_t *pt, uint64_t count, uint64_t *ct)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t xi = 0; xi < (int64_t)count; ++xi) {
        uint64_t x = (uint64_t)xi;
        int64_t *e = (int64_t *)malloc(n * sizeof(int64_t));
        uint64_t *sl = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *as = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *ac = (uint64_t *)malloc(n * sizeof(uint64_t));
        orc_sample_poly(2, e_key, TAG_ENC_E, 0, op, (uint32_t)x, n, 0, 0, cdt, e);
        for (uint64_t l = 0; l < L; ++l) {
            uint64_t *c0 = ct + ((x * 2 + 0) * L + l) * n;
            uint64_t *c1 = ct + ((x * 2 + 1) * L + l) * n;
            orc_sample_poly(0, a_key, TAG_ENC_A, (uint32_t)l, op, (uint32_t)x, n, q[l], 0, cdt, c1);
            orc_slots_to_coef(c1, ac, n, q[l], psi[l]);
            for (uint64_t j = 0; j < n; ++j) sl[j] = lift(s[j], q[l]);
            orc_negacyclic_mul(ac, sl, as, n, q[l], psi[l]);
            for (uint64_t j = 0; j < n; ++j) {
                uint64_t m = mulm(delta_l[l], pt[x * n + j] % q[l], q[l]);
                ac[j] = subm(addm(m, lift(e[j], q[l]), q[l]), as[j], q[l]);
            }
            orc_coef_to_slots(ac, c0, n, q[l], psi[l]);
        }
        free(e);
        free(sl);
        free(as);
        free(ac);
    }
}

/* Ciphertext-plaintext product with accumulation over the inner blocks
 * (Algorithm 1, step 3, [[c]] = a * [[b]], summed over the blocks the inner
 * dimension was split into).  For each requested output ciphertext
 * y = ib*K + kb, component c and prime l:
 *     acc = sum_{jb < R} lift(ptA[ib*R + jb]) * ct[jb*K + kb][c][l]   (mod q_l)
 * ptA: [M*R][n] signed plaintext coefficients (lifted to q_l - |w| if negative);
 * ct: [R*K][2][L][n] query ciphertexts (in evaluation form, taken back to
 * coefficients first); outs: the nouts output indices y to compute;
 * acc: [nouts][2][L][n] in coefficient form. */
void orc_ctpt_matmul(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi, uint64_t R,
                     uint64_t K, const int64_t *ptA, const uint64_t *ct, const uint32_t *outs,
                     uint64_t nouts, uint64_t *acc)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t w = 0; w < (int64_t)(nouts * 2 * L); ++w) {
        uint64_t o = (uint64_t)w / (2 * L);
        uint64_t c = ((uint64_t)w / L) % 2;
        uint64_t l = (uint64_t)w % L;
        uint64_t y = outs[o];
        uint64_t ib = y / K, kb = y % K;
        uint64_t *dst = acc + ((o * 2 + c) * L + l) * n;
        uint64_t *a = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *prod = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *cc = (uint64_t *)malloc(n * sizeof(uint64_t));
        memset(dst, 0, n * sizeof(uint64_t));
        for (uint64_t jb = 0; jb < R; ++jb) {
            const int64_t *pa = ptA + (ib * R + jb) * n;
            const uint64_t *src = ct + (((jb * K + kb) * 2 + c) * L + l) * n;
            orc_slots_to_coef(src, cc, n, q[l], psi[l]);  /* queries travel as slots */
            src = cc;
            for (uint64_t j = 0; j < n; ++j) a[j] = lift(pa[j], q[l]);
            orc_negacyclic_mul(a, src, prod, n, q[l], psi[l]);
            for (uint64_t j = 0; j < n; ++j) dst[j] = addm(dst[j], prod[j], q[l]);
        }
        free(a);
        free(prod);
        free(cc);
    }
}

/* Re-randomisation of an output ciphertext by a fresh public-key encryption
 * of zero: acc0 += u*pk0 + e1, acc1 += u*pk1 + e2 (mod q_l), with u ternary
 * from (RR_U, 0, op, y), e1 from (RR_E1, 0, op, y), e2 from (RR_E2, 0, op, y).
 * acc: [nouts][2][L][n] in place; pk: [2][L][n]. */
void orc_rerandomize(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                     const uint64_t *pk, const uint8_t key[32], uint32_t op, const uint64_t *cdt,
                     const uint32_t *outs, uint64_t nouts, uint64_t *acc)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t oi = 0; oi < (int64_t)nouts; ++oi) {
        uint64_t o = (uint64_t)oi;
        uint32_t y = outs[o];
        int64_t *u = (int64_t *)malloc(n * sizeof(int64_t));
        int64_t *e1 = (int64_t *)malloc(n * sizeof(int64_t));
        int64_t *e2 = (int64_t *)malloc(n * sizeof(int64_t));
        uint64_t *ul = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *prod = (uint64_t *)malloc(n * sizeof(uint64_t));
        orc_sample_poly(1, key, TAG_RR_U, 0, op, y, n, 0, 0, cdt, u);
        orc_sample_poly(2, key, TAG_RR_E1, 0, op, y, n, 0, 0, cdt, e1);
        orc_sample_poly(2, key, TAG_RR_E2, 0, op, y, n, 0, 0, cdt, e2);
        for (uint64_t l = 0; l < L; ++l) {
            for (uint64_t j = 0; j < n; ++j) ul[j] = lift(u[j], q[l]);
            for (uint64_t c = 0; c < 2; ++c) {
                uint64_t *dst = acc + ((o * 2 + c) * L + l) * n;
                const int64_t *e = c == 0 ? e1 : e2;
                orc_negacyclic_mul(ul, pk + (c * L + l) * n, prod, n, q[l], psi[l]);
                for (uint64_t j = 0; j < n; ++j)
                    dst[j] = addm(addm(dst[j], prod[j], q[l]), lift(e[j], q[l]), q[l]);
            }
        }
        free(u);
        free(e1);
        free(e2);
        free(ul);
        free(prod);
    }
}

/* Mask and extract (Algorithm 1, step 3, [[c]] - s, and the sparse reply of
 * section 3.1.3).  The server's random polynomial s_y over Z_{2^ell} comes
 * from stream (MASK, 0, op, y), one 64-bit draw per coefficient index.  Only
 * the decoded coefficients pos(i,k) = k*mb*rb + i*rb + rb - 1 are kept:
 *     c1  [nouts][L][n]        = acc1 (all coefficients),
 *     c0s [nouts][L][mb*nb]    at k*mb + i  = [acc0[pos] - Delta_l * s_y[pos]]_{q_l},
 *     smask [nouts][mb*nb]     at k*mb + i  = s_y[pos]   (the server's share). */
void orc_mask_extract(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *delta_l,
                      unsigned ell, const uint8_t key[32], uint32_t op, uint64_t mb, uint64_t rb,
                      uint64_t nb, const uint32_t *outs, uint64_t nouts, const uint64_t *acc,
                      uint64_t *c1, uint64_t *c0s, uint64_t *smask)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t oi = 0; oi < (int64_t)nouts; ++oi) {
        uint64_t o = (uint64_t)oi;
        uint32_t y = outs[o];
        for (uint64_t l = 0; l < L; ++l)
            memcpy(c1 + (o * L + l) * n, acc + ((o * 2 + 1) * L + l) * n, n * sizeof(uint64_t));
        for (uint64_t k = 0; k < nb; ++k)
            for (uint64_t i = 0; i < mb; ++i) {
                uint64_t pos = k * mb * rb + i * rb + rb - 1;
                uint64_t s = sample_mask(key, TAG_MASK, op, y, pos, ell);
                smask[o * mb * nb + k * mb + i] = s;
                for (uint64_t l = 0; l < L; ++l) {
                    uint64_t a0 = acc[((o * 2 + 0) * L + l) * n + pos];
                    c0s[(o * L + l) * mb * nb + k * mb + i] =
                        subm(a0, mulm(delta_l[l], s % q[l], q[l]), q[l]);
                }
            }
    }
}

/* Client side of decryption at the decoded positions (section 3.1.3: the
 * coefficient m_i of m = s*c1 + c0 needs (c0)_i and all of c1):
 *     x[o][k*mb + i][l] = [c0s[o][l][k*mb + i] + (c1[o][l] * s)[pos(i,k)]]_{q_l}.
 * The CRT and the BFV rounding are done by the caller. */
void orc_decrypt_residues(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                          const int64_t *s, uint64_t mb, uint64_t rb, uint64_t nb, uint64_t nouts,
                          const uint64_t *c1, const uint64_t *c0s, uint64_t *x)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t w = 0; w < (int64_t)(nouts * L); ++w) {
        uint64_t o = (uint64_t)w / L, l = (uint64_t)w % L;
        uint64_t *sl = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *prod = (uint64_t *)malloc(n * sizeof(uint64_t));
        for (uint64_t j = 0; j < n; ++j) sl[j] = lift(s[j], q[l]);
        orc_negacyclic_mul(c1 + (o * L + l) * n, sl, prod, n, q[l], psi[l]);
        for (uint64_t k = 0; k < nb; ++k)
            for (uint64_t i = 0; i < mb; ++i) {
                uint64_t pos = k * mb * rb + i * rb + rb - 1;
                uint64_t idx = k * mb + i;
                x[(o * mb * nb + idx) * L + l] =
                    addm(c0s[(o * L + l) * mb * nb + idx], prod[pos], q[l]);
            }
        free(sl);
        free(prod);
    }
}

/* Full decryption residues of whole ciphertexts (every coefficient):
 * x[o][j][l] = [c0 + c1*s]_{q_l}; ct: [count][2][L][n], in evaluation form (a
 * query ciphertext) when slots, else in coefficient form (a product's output).
 * Used by tests of encryption and of the ciphertext-plaintext product. */
void orc_decrypt_full_residues(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                               const int64_t *s, uint64_t count, const uint64_t *ct, int slots,
                               uint64_t *x)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t w = 0; w < (int64_t)(count * L); ++w) {
        uint64_t o = (uint64_t)w / L, l = (uint64_t)w % L;
        uint64_t *sl = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *prod = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *c0 = (uint64_t *)malloc(n * sizeof(uint64_t));
        uint64_t *c1 = (uint64_t *)malloc(n * sizeof(uint64_t));
        const uint64_t *in0 = ct + ((o * 2 + 0) * L + l) * n, *in1 = ct + ((o * 2 + 1) * L + l) * n;
        if (slots) {
            orc_slots_to_coef(in0, c0, n, q[l], psi[l]);
            orc_slots_to_coef(in1, c1, n, q[l], psi[l]);
        } else {
            memcpy(c0, in0, n * sizeof(uint64_t));
            memcpy(c1, in1, n * sizeof(uint64_t));
        }
        for (uint64_t j = 0; j < n; ++j) sl[j] = lift(s[j], q[l]);
        orc_negacyclic_mul(c1, sl, prod, n, q[l], psi[l]);
        for (uint64_t j = 0; j < n; ++j) x[(o * n + j) * L + l] = addm(c0[j], prod[j], q[l]);
        free(sl);
        free(prod);
        free(c0);
        free(c1);
    }
}
