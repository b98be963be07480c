/* The oracle's C functions under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Built with the oracle source into one executable (tests/test_sanitizers.py) and
 * run on small sizes: every sampler, the negacyclic transform and its inverse,
 * the product against the schoolbook one, key generation, encryption, the
 * ciphertext-plaintext product, re-randomisation, mask and extraction, and both
 * decryptions.  A sanitizer report or a failed check ends the run with a nonzero
 * status; the last line is "ok <checks>" otherwise.  The cumulative table here is
 * a monotone stand-in computed in long double: the run checks memory and
 * arithmetic safety, not the sampler's distribution (which the other oracle
 * tests pin). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_chacha20_block(const uint8_t key[32], uint32_t counter, const uint32_t nonce[3],
                        uint32_t out[16]);
uint64_t orc_draw64(const uint8_t key[32], uint32_t tag, uint32_t prime, uint32_t op, uint32_t obj,
                    uint64_t j);
void orc_sample_poly(int kind, const uint8_t key[32], uint32_t tag, uint32_t prime, uint32_t op,
                     uint32_t obj, uint64_t n, uint64_t q, unsigned ell, const uint64_t *cdt,
                     void *out);
void orc_ntt_negacyclic(const uint64_t *a, uint64_t *A, uint64_t n, uint64_t q, uint64_t psi);
void orc_intt_negacyclic(const uint64_t *A, uint64_t *a, uint64_t n, uint64_t q, uint64_t psi);
void orc_negacyclic_mul(const uint64_t *a, const uint64_t *b, uint64_t *c, uint64_t n, uint64_t q,
                        uint64_t psi);
void orc_negacyclic_mul_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *c, uint64_t n,
                                   uint64_t q);
void orc_keygen(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                const uint8_t key[32], const uint64_t *cdt, int64_t *s, uint64_t *pk);
void orc_encrypt(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                 const uint64_t *delta_l, const int64_t *s, const uint8_t key[32], uint32_t op,
                 const uint64_t *cdt, const uint64_t *pt, uint64_t count, uint64_t *ct);
void orc_ctpt_matmul(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi, uint64_t R,
                     uint64_t K, const int64_t *ptA, const uint64_t *ct, const uint32_t *outs,
                     uint64_t nouts, uint64_t *acc);
void orc_rerandomize(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                     const uint64_t *pk, const uint8_t key[32], uint32_t op, const uint64_t *cdt,
                     const uint32_t *outs, uint64_t nouts, uint64_t *acc);
void orc_mask_extract(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *delta_l,
                      unsigned ell, const uint8_t key[32], uint32_t op, uint64_t mb, uint64_t rb,
                      uint64_t nb, const uint32_t *outs, uint64_t nouts, const uint64_t *acc,
                      uint64_t *c1, uint64_t *c0s, uint64_t *smask);
void orc_decrypt_residues(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                          const int64_t *s, uint64_t mb, uint64_t rb, uint64_t nb, uint64_t nouts,
                          const uint64_t *c1, const uint64_t *c0s, uint64_t *x);
void orc_decrypt_full_residues(uint64_t n, uint64_t L, const uint64_t *q, const uint64_t *psi,
                               const int64_t *s, uint64_t count, const uint64_t *ct, int c1_slots,
                               uint64_t *x);
uint64_t orc_slot_index(uint64_t z, uint64_t n);
void orc_slots_to_coef(const uint64_t *S, uint64_t *a, uint64_t n, uint64_t q, uint64_t psi);
void orc_coef_to_slots(const uint64_t *a, uint64_t *S, uint64_t n, uint64_t q, uint64_t psi);

static int checks = 0;

#define CHECK(cond)                                                        \
    do {                                                                   \
        ++checks;                                                          \
        if (!(cond)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            exit(1);                                                       \
        }                                                                  \
    } while (0)

static uint64_t powm(uint64_t a, uint64_t e, uint64_t q)
{
    unsigned __int128 r = 1, b = a % q;
    for (; e; e >>= 1) {
        if (e & 1) r = r * b % q;
        b = b * b % q;
    }
    return (uint64_t)r;
}

/* A primitive 2n-th root of unity mod q (q = 1 mod 2n): psi^n = -1. */
static uint64_t find_psi(uint64_t q, uint64_t n)
{
    for (uint64_t g = 2; g < q; ++g) {
        uint64_t p = powm(g, (q - 1) / (2 * n), q);
        if (powm(p, n, q) == q - 1) return p;
    }
    return 0;
}

int main(void)
{
    enum { N = 32, L = 2, R = 2, K = 3, M = 2, MB = 2, RB = 4, NB = 4 };
    const uint64_t q[L] = {193, 257};  /* both = 1 mod 64 */
    uint64_t psi[L];
    for (int l = 0; l < L; ++l) {
        psi[l] = find_psi(q[l], N);
        CHECK(psi[l] != 0);
    }
    uint64_t cdt[19];
    long double acc = 0.0L, total = 0.0L;
    for (int x = -19; x <= 19; ++x) total += expl(-(long double)(x * x) / (2.0L * 3.2L * 3.2L));
    for (int k = 0; k < 19; ++k) {
        acc += expl(-(long double)(k * k) / (2.0L * 3.2L * 3.2L)) * (k ? 2.0L : 1.0L);
        cdt[k] = (uint64_t)(acc / total * 9223372036854775808.0L);
    }
    uint8_t key[32];
    for (int i = 0; i < 32; ++i) key[i] = (uint8_t)(i * 7 + 1);

    /* Keystream and draws. */
    uint32_t nonce[3] = {1, 2, 3}, blk[16], blk2[16];
    orc_chacha20_block(key, 5, nonce, blk);
    orc_chacha20_block(key, 5, nonce, blk2);
    CHECK(memcmp(blk, blk2, sizeof blk) == 0);
    CHECK(orc_draw64(key, 4, 1, 2, 3, 17) == orc_draw64(key, 4, 1, 2, 3, 17));

    /* Every sampler. */
    uint64_t u[N];
    int64_t v[N];
    orc_sample_poly(0, key, 4, 0, 9, 1, N, q[0], 0, cdt, u);
    for (int j = 0; j < N; ++j) CHECK(u[j] < q[0]);
    orc_sample_poly(1, key, 1, 0, 9, 1, N, 0, 0, cdt, v);
    for (int j = 0; j < N; ++j) CHECK(v[j] >= -1 && v[j] <= 1);
    orc_sample_poly(2, key, 5, 0, 9, 1, N, 0, 0, cdt, v);
    for (int j = 0; j < N; ++j) CHECK(v[j] >= -19 && v[j] <= 19);
    orc_sample_poly(3, key, 9, 0, 9, 1, N, 0, 20, cdt, u);
    for (int j = 0; j < N; ++j) CHECK(u[j] < (1u << 20));

    /* Transform round trip and the product against the schoolbook one. */
    uint64_t a[N], b[N], A[N], back[N], c1[N], c2[N];
    for (int j = 0; j < N; ++j) {
        a[j] = (uint64_t)(j * 31 + 7) % q[0];
        b[j] = (uint64_t)(j * j + 3) % q[0];
    }
    orc_ntt_negacyclic(a, A, N, q[0], psi[0]);
    orc_intt_negacyclic(A, back, N, q[0], psi[0]);
    CHECK(memcmp(a, back, sizeof a) == 0);
    orc_negacyclic_mul(a, b, c1, N, q[0], psi[0]);
    orc_negacyclic_mul_schoolbook(a, b, c2, N, q[0]);
    CHECK(memcmp(c1, c2, sizeof c1) == 0);

    /* Protocol steps on a small plan: keys, encryption of R*K plaintexts, the
     * product of M*R weight blocks, re-randomisation, mask, both decryptions. */
    int64_t s[N];
    uint64_t *pk = calloc(2 * L * N, sizeof(uint64_t));
    orc_keygen(N, L, q, psi, key, cdt, s, pk);
    const uint64_t delta[L] = {7, 11};
    uint64_t *pt = calloc((size_t)R * K * N, sizeof(uint64_t));
    for (int i = 0; i < R * K * N; ++i) pt[i] = (uint64_t)(i % 5);
    uint64_t *ct = calloc((size_t)R * K * 2 * L * N, sizeof(uint64_t));
    orc_encrypt(N, L, q, psi, delta, s, key, 3, cdt, pt, R * K, ct);
    for (int i = 0; i < R * K * 2 * L * N; ++i) CHECK(ct[i] < q[(i / N) % L]);
    int64_t *ptA = calloc((size_t)M * R * N, sizeof(int64_t));
    for (int i = 0; i < M * R * N; ++i) ptA[i] = (i % 7) - 3;
    uint32_t outs[M * K];
    for (int y = 0; y < M * K; ++y) outs[y] = (uint32_t)y;
    uint64_t *accb = calloc((size_t)M * K * 2 * L * N, sizeof(uint64_t));
    orc_ctpt_matmul(N, L, q, psi, R, K, ptA, ct, outs, M * K, accb);
    orc_rerandomize(N, L, q, psi, pk, key, 4, cdt, outs, M * K, accb);
    uint64_t *rc1 = calloc((size_t)M * K * L * N, sizeof(uint64_t));
    uint64_t *rc0 = calloc((size_t)M * K * L * MB * NB, sizeof(uint64_t));
    uint64_t *sm = calloc((size_t)M * K * MB * NB, sizeof(uint64_t));
    orc_mask_extract(N, L, q, delta, 6, key, 5, MB, RB, NB, outs, M * K, accb, rc1, rc0, sm);
    uint64_t *xr = calloc((size_t)M * K * MB * NB * L, sizeof(uint64_t));
    orc_decrypt_residues(N, L, q, psi, s, MB, RB, NB, M * K, rc1, rc0, xr);
    for (int i = 0; i < M * K * MB * NB * L; ++i) CHECK(xr[i] < q[i % L]);
    uint64_t *xf = calloc((size_t)R * K * N * L, sizeof(uint64_t));
    orc_decrypt_full_residues(N, L, q, psi, s, R * K, ct, 1, xf);
    /* Evaluation form: the slot map is a permutation and the two directions invert each other. */
    {
        uint64_t seen[N], back2[N], S[N];
        memset(seen, 0, sizeof seen);
        for (uint64_t z = 0; z < N; ++z) {
            uint64_t k = orc_slot_index(z, N);
            CHECK(k < N && !seen[k]);
            seen[k] = 1;
        }
        orc_coef_to_slots(a, S, N, q[0], psi[0]);
        orc_slots_to_coef(S, back2, N, q[0], psi[0]);
        CHECK(memcmp(a, back2, sizeof back2) == 0);
    }
    free(pk);
    free(pt);
    free(ct);
    free(ptA);
    free(accb);
    free(rc1);
    free(rc0);
    free(sm);
    free(xr);
    free(xf);
    printf("ok %d\n", checks);
    return 0;
}
