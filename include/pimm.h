/*
 * pimm.h -- C ABI of libpimm, an MI355X (gfx950) implementation of the
 * private matrix-multiplication protocol Pi_MatMul of Liu & Liu, "LLMs Can
 * Understand Encrypted Prompt: Towards Privacy-Computing Friendly
 * Transformers" (arXiv 2305.18396), Algorithm 1 (section 3.1.1), over RNS-BFV
 * (section 2.2), with the sparse reply of section 3.1.3.
 *
 * Problem (Algorithm 1, inputs and outputs): the server holds A (m x r), the
 * client holds B (r x n); the parties end with additive shares of C = AB over
 * Z_t, t = 2^l.  For a linear layer Y = X W (section 3.1.1, fully connected
 * layer, and the transposed form in the footnote of the attention paragraph)
 * the library takes A = W^T and B = X^T, so the user-level contract is
 *
 *     client_share + server_share = X W   (mod 2^l), elementwise over [n][m].
 *
 * Conventions for every call:
 *   - Return value: PIMM_OK (0) or a negative PIMM_E_* code.  No exception or
 *     longjmp crosses the ABI.  pimm_last_error() gives a thread-local message.
 *   - Bulk buffers are caller-owned DEVICE pointers on the context's device
 *     (for example torch tensor data pointers), row-major, with the sizes that
 *     pimm_plan_query() reports.  Handles (context, plan, key, weights) are
 *     created and destroyed by the library; a key and a weight cache hold
 *     device memory that the library allocates.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work and return; errors of the work itself surface at
 *     pimm_sync() or at a later call.  Calls that take a workspace use the
 *     caller's buffer `ws` of `ws_bytes` bytes (at least
 *     pimm_plan_info.workspace_bytes) and allocate nothing.
 *   - Contexts, plans and keys are immutable after creation, so calls on
 *     different streams may share them; two calls in flight must not share a
 *     workspace or an output buffer.  A weight cache is immutable too unless
 *     pimm_weights_update rewrites it: that call enqueues the rewrite on its
 *     own stream, so every later call that reads the cache (a product, a
 *     batch, pimm_fc_complete) must be on the same stream or ordered after it
 *     by an event, and no call that reads the cache may still be in flight on
 *     another stream when the update is enqueued.
 *   - Output bytes depend only on (parameters, plan, inputs, seeds, op_id),
 *     never on batching, stream or launch order.
 *   - Residues are canonical integers in [0, q_l), stored as uint64.  Shares
 *     are integers in [0, 2^l), stored as uint64.
 *
 * Randomness (encryption noise and masks): ChaCha20 (RFC 8439, section 2.3)
 * keyed by the caller's 32-byte seed, nonce (tag | prime << 8, op_id,
 * object index), block counter from 0; the 64-bit draw j is keystream bytes
 * [8j, 8j+8), little-endian.  A uniform residue mod q_l is the low 50 bits x of
 * draw j when x < q_l, else the low 50 bits of draw j of the fallback stream
 * (bit 31 of the tag word set) mod q_l.
 * op_id is the only per-call nonce: a (seed, op_id) pair must never serve two
 * different inputs (two encryptions of different plaintexts under one pair
 * share a and e; two replies under one server pair share the mask).  Repeating
 * a call on the same inputs with the same pair repeats its bytes, which is
 * harmless.
 */
#ifndef PIMM_H
#define PIMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIMM_OK 0
#define PIMM_E_ARG (-1)         /* NULL pointer or out-of-range argument */
#define PIMM_E_SHAPE (-2)       /* matrix shape or block plan that does not fit */
#define PIMM_E_PARAMS (-3)      /* N not a power of two in [4096, 8192], L not in [1, 4], ... */
#define PIMM_E_NOISE (-4)       /* weights whose worst-case noise breaks decryption */
#define PIMM_E_OOM (-5)         /* device allocation failed */
#define PIMM_E_DEVICE (-6)      /* HIP runtime error */
#define PIMM_E_UNSUPPORTED (-7) /* valid request the library does not implement */
#define PIMM_E_WORKSPACE (-8)   /* workspace missing or smaller than required */

typedef struct pimm_ctx pimm_ctx;
typedef struct pimm_plan pimm_plan;
typedef struct pimm_sk pimm_sk;
typedef struct pimm_weights pimm_weights;
typedef struct pimm_batch pimm_batch;
typedef struct pimm_server pimm_server;

/* RNS-BFV parameters (section 2.2: N a power of two, plaintext modulus t = 2^l,
 * ciphertext modulus q a product of L word-size primes).
 *   N           ring degree, 4096 or 8192
 *   L           number of RNS primes, 1..4
 *   log2_t      l, 2..48 (t = 2^l; shares live in Z_{2^l})
 *   frac_bits   f, fixed-point fractional bits of W (section 2.2); informational
 *   prime_bits  must be 50: the primes are the L largest primes q < 2^50 with
 *               q = 1 (mod 2N), in descending order
 *   rerandomize 1: pimm_mask_share adds a fresh public-key encryption of zero
 *               to each reply ciphertext before masking; 0: it does not. */
typedef struct {
    uint32_t N, L, log2_t, frac_bits, prime_bits, rerandomize;
} pimm_params;

/* Block plan and buffer sizes of one product Y[n][m] = X[n][r] W[r][m].
 * Blocks are (mb, rb, nb) with mb*rb*nb <= N; M = ceil(m/mb), R = ceil(r/rb),
 * K = ceil(n/nb); I = R*K input ciphertexts (index x = jb*K + kb), O = M*K
 * output ciphertexts (index y = ib*K + kb), Wb = M*R weight blocks, P = M*R*K
 * block products.  Byte sizes are of the caller-owned buffers:
 *   pt        [I][N]          uint64  encoded client plaintexts
 *   ct        [I][2][L][N]    uint64  input ciphertexts, both components in evaluation
 *                                     form (see pimm_encrypt)
 *   acc       [O][2][L][N]    uint64  products before masking, coefficient form
 *   c1        [O][L][N]       uint64  reply, full c1
 *   c0s       [O][L][mb*nb]   uint64  reply, c0 at the decoded positions only,
 *                                     entry k*mb + i for position k*mb*rb + i*rb + rb-1
 *   share     [n][m]          uint64  one party's share of Y
 *   weights   device bytes held by a weight cache for this plan
 *   workspace bytes of scratch that encrypt, matmul, mask_share and decrypt need
 * groups: G >= 1 products of this one shape run as one (pimm_plan_create_grouped;
 * 1 otherwise).  Then I = G*R*K, O = G*M*K, Wb = G*M*R, P = G*M*R*K and every byte
 * size count all G products: input ciphertext x of product p is ciphertext
 * p*R*K + x of the plan, output y of product p is p*M*K + y, and X, W and the
 * shares are [G][n][r], [G][r][m] and [G][n][m].  M, R and K stay per product. */
typedef struct {
    uint32_t n, r, m, mb, rb, nb, M, R, K, I, O, Wb;
    uint64_t P;
    uint64_t pt_bytes, ct_bytes, acc_bytes, c1_bytes, c0s_bytes, share_bytes;
    uint64_t weights_bytes, workspace_bytes;
    uint32_t groups;
} pimm_plan_info;

/* ---- context -------------------------------------------------------------- */

/* Create a context on HIP device `device`: finds the primes, builds the NTT
 * tables and the decryption constants on that device. */
int pimm_ctx_create(const pimm_params *params, int device, pimm_ctx **out);
int pimm_ctx_destroy(pimm_ctx *ctx);
/* q_out[L]: the RNS primes. */
int pimm_ctx_primes(const pimm_ctx *ctx, uint64_t *q_out);
/* cdt_out[19]: the cumulative table of the error sampler (width 3.2, |e| <= 19),
 * T[k] = floor(2^63 P(|e| <= k)). */
int pimm_ctx_cdt(const pimm_ctx *ctx, uint64_t *cdt_out);

/* ---- host-only queries (no device needed) --------------------------------------- */

/* Validate params and write the L primes to q_out[L] (same rule as the context). */
int pimm_params_primes(const pimm_params *params, uint64_t *q_out);
/* cdt_out[19]: the error sampler's cumulative table (as pimm_ctx_cdt). */
int pimm_cdt(uint64_t *cdt_out);
/* The plan pimm_plan_create would make, without a context or a device. */
int pimm_plan_rule(const pimm_params *params, uint32_t n, uint32_t r, uint32_t m, uint32_t mb,
                   uint32_t rb, uint32_t nb, uint32_t d_fix, pimm_plan_info *info);
/* 1 if weights with max |W| = wmax pass the noise check of pimm_weights_create for
 * this plan, 0 if not, <0 on error.  The worst-case noise of a decoded reply
 * coefficient is E = R*D*wmax*19 + (q mod t)(r*wmax + 1) [+ 2*N*19 + 19 with
 * re-randomisation], D = mb*rb, and decryption is correct when 2 t (E + (q mod t)) < q. */
int pimm_noise_ok(const pimm_params *params, const pimm_plan_info *info, uint64_t wmax);
/* 1 if a reply made with weights of max |W| = wmax still decrypts to the same
 * share after pimm_mod_switch, 0 if not, <0 on error (PIMM_E_UNSUPPORTED for
 * L = 1).  With E the bound above and q' = q / q_{L-1}: the switched noise is at
 * most E' = ceil(E / q_{L-1}) + (N + 2) / 2 (the scaled noise plus the rounding of
 * c0 and of the N terms of c1 s), and the rule is 2 t (E' + 1) < q'. */
int pimm_switch_ok(const pimm_params *params, const pimm_plan_info *info, uint64_t wmax);

/* ---- plan ------------------------------------------------------------------ */

/* Plan Y[n][m] = X[n][r] W[r][m].  The paper leaves the block split open
 * (section 3.1.1 says only that larger matrices are split into blocks):
 *   mb, rb, nb all > 0   use that block shape (mb*rb*nb <= N);
 *   d_fix > 0            mb*rb = d_fix (a power of two <= N), split to minimise
 *                        ceil(r/rb) + ceil(m/mb), ties to larger mb; nb = min(n, N/d_fix);
 *   otherwise            fewest ciphertexts on the wire: minimise
 *                        (ceil(r/rb) + ceil(m/mb)) * ceil(n/nb) over powers of two
 *                        mb <= nextpow2(m), rb <= nextpow2(r), mb*rb <= N,
 *                        nb = min(n, N/(mb rb)); ties to larger nb, then larger mb. */
int pimm_plan_create(pimm_ctx *ctx, uint32_t n, uint32_t r, uint32_t m, uint32_t mb, uint32_t rb,
                     uint32_t nb, uint32_t d_fix, pimm_plan **out);
/* G independent products of one shape, Y_p[n][m] = X_p[n][r] W_p[r][m], run as one:
 * every call on the plan does the work of all G in the same launches (many small
 * products, such as the attention cross terms of Eq. 2 -- the 24 products of one
 * phase of a BERT-base layer -- otherwise leave most of the device idle).  The
 * block plan is pimm_plan_create's for one product; the layouts are in
 * pimm_plan_info.  Each product follows Algorithm 1 on its own blocks; the group
 * shares op_id, and the stream objects of the products are disjoint (ciphertext
 * p*R*K + x, output p*M*K + y).  Grouped plans take the FP64 vector product with
 * one column block per thread (tiles 4x1, 8x1, 16x1); pimm_fc_complete, pimm_batch_*
 * and the matrix-core schedule refuse them (PIMM_E_UNSUPPORTED).  groups in
 * [1, 65536]; groups = 1 is pimm_plan_create. */
int pimm_plan_create_grouped(pimm_ctx *ctx, uint32_t n, uint32_t r, uint32_t m, uint32_t mb,
                             uint32_t rb, uint32_t nb, uint32_t d_fix, uint32_t groups,
                             pimm_plan **out);
int pimm_plan_destroy(pimm_plan *plan);
int pimm_plan_query(const pimm_plan *plan, pimm_plan_info *info);
/* Schedule of pimm_matmul's slot-wise products: each thread owns mac_rows output
 * rows by mac_cols output column blocks (rows x cols one of 4x1, 8x1, 16x1, 4x2,
 * 8x2, 16x2, 2x4, 4x4, 8x4, 2x8, 4x8), so that a weight word it loads serves mac_cols column
 * blocks (a ragged last column tile runs as narrower tiles);
 * the (tile, inner block) iterations are divided evenly over a grid of `waves`
 * (1, 2, 4) times the workgroups the device holds at once.
 * (0, 0, 0) selects the matrix-core product instead: exact int8 products of signed 8-bit
 * digits of the residues on the matrix instructions, for plans with R <= 64 inner blocks
 * and K >= 8 column blocks (PIMM_E_UNSUPPORTED otherwise) and weight caches made for such
 * a plan (they then also hold the digit form; pimm_matmul refuses the schedule with
 * PIMM_E_UNSUPPORTED on a cache without it).  Any schedule gives the same bytes. */
int pimm_plan_set_tuning(pimm_plan *plan, int mac_rows, int mac_cols, int waves);
int pimm_plan_get_tuning(const pimm_plan *plan, int *mac_rows, int *mac_cols, int *waves);
/* Protocol-level choice of the block split (section 3.1.1 leaves it open: larger
 * matrices are split into blocks).  For each candidate block area d_candidates[i]
 * (0 = the fewest-wire plan, otherwise mb*rb = d as pimm_plan_create's d_fix) the
 * call builds the plan and a weight cache of W ([r][m] signed fixed point, device),
 * autotunes the product, and times the server's part of Algorithm 1 (pimm_matmul_share:
 * input transforms, slot-wise products, re-randomisation, mask, sparse reply) on random
 * ciphertexts with HIP events on `stream` (`reps` timed runs after one untimed run).
 * It writes the measured milliseconds to server_ms[i] and the bytes on the wire (client
 * upload of whole ciphertexts + sparse reply) to wire_bytes[i] (either may be NULL), and
 * the candidate minimising server_ms + wire_bytes * 8 / link_bits_per_s to *d_best.
 * Allocates and frees device memory for each candidate (not for capture or tight loops);
 * synchronises `stream`. */
int pimm_plan_select(pimm_ctx *ctx, uint32_t n, uint32_t r, uint32_t m, const int64_t *W,
                     double link_bits_per_s, const uint32_t *d_candidates, uint32_t count, int reps,
                     void *stream, uint32_t *d_best, double *server_ms, uint64_t *wire_bytes);
/* Time every (mac_rows, mac_cols, waves) on these buffers with HIP events on `stream`
 * (`reps` timed runs each) and keep the fastest on the plan; best_ms may be NULL. */
int pimm_plan_autotune(pimm_plan *plan, const pimm_weights *w, const uint64_t *ct, uint64_t *acc,
                       void *ws, size_t ws_bytes, int reps, void *stream, double *best_ms);

/* ---- client ---------------------------------------------------------------- */

/* Key generation.  s ternary from stream tag 1; with re-randomisation on and
 * pk_out not NULL, also pk = ([-a' s + e']_q, a') (a' uniform per prime from
 * tag 2, e' Gaussian from tag 3), written to pk_out [2][L][N] (device).
 * The key stays on the device inside the returned handle. */
int pimm_keygen(pimm_ctx *ctx, const uint8_t seed[32], pimm_sk **sk, uint64_t *pk_out,
                void *stream);
int pimm_sk_destroy(pimm_sk *sk);

/* Algorithm 1 step 1, client side: pi_B per block,
 * pt[jb*K + kb][k*mb*rb + j] = X[kb*nb + k][jb*rb + j], zero elsewhere.
 * X: [n][r] values < 2^l (device). */
int pimm_encode_input(const pimm_plan *plan, const uint64_t *X, uint64_t *pt, void *stream);

/* Algorithm 1 step 2: symmetric BFV encryption of every pt row x, sent in evaluation
 * form (slot z of a polynomial holds its value at psi_l^(2k+1),
 * k = brv(16 (z mod N/16) + floor(z / (N/16))) with brv reversing log2 N bits and psi_l
 * the primitive 2N-th root g^((q_l - 1) / 2N) mod q_l for the smallest g >= 2 that gives
 * psi_l^N = -1):
 *   c1_l = the slots of a_l: c1_l[z] = draw z of the stream (tag 4, prime l, op_id, x)
 *          (a_l uniform mod q_l, drawn as its slots: a uniform set of evaluations is a
 *          uniform polynomial, and neither party transforms a);
 *   c0_l = the slots of [Delta_l pt + e - a_l s]_{q_l} (e Gaussian, tag 5, op_id, x),
 *          Delta = floor(q / t).
 * The slot form is a ring isomorphism, so this is the BFV ciphertext itself; the server's
 * product is slot-wise and takes it as it comes.  ct: [I][2][L][N] (device). */
int pimm_encrypt(const pimm_plan *plan, const pimm_sk *sk, const uint8_t seed[32], uint32_t op_id,
                 const uint64_t *pt, uint64_t *ct, void *ws, size_t ws_bytes, void *stream);

/* Algorithm 1 steps 1 and 2 in one pass: pi_B of X (as pimm_encode_input) encoded
 * inside the encryption (as pimm_encrypt), without the plaintexts in memory.  The
 * ciphertexts are exactly those of pimm_encode_input followed by pimm_encrypt with the
 * same seed and op_id.  X: [n][r] values < 2^l (device; [G][n][r] for a grouped plan),
 * ct: [I][2][L][N] (device); the workspace of pimm_encrypt. */
int pimm_encrypt_input(const pimm_plan *plan, const pimm_sk *sk, const uint8_t seed[32], uint32_t op_id,
                       const uint64_t *X, uint64_t *ct, void *ws, size_t ws_bytes, void *stream);

/* Seed-compressed upload, a wire-format variant of Algorithm 1 step 2.  c1 = a (its
 * slots, as in pimm_encrypt) is public, so it can come from a public seed:
 * pimm_encrypt_seeded draws a_l from
 * the stream of a_seed (tag 4) and e from `seed` (tag 5), and the client sends
 * c0 ([I][L][N], half the ciphertext bytes) with the 32-byte a_seed; the server
 * rebuilds the ciphertexts with pimm_ct_expand.  a_seed must be independent of
 * `seed` (a is public, e is not); with a_seed = seed the call is pimm_encrypt.
 * ct: [I][2][L][N] (device); the client's c0 is ct[x][0]. */
int pimm_encrypt_seeded(const pimm_plan *plan, const pimm_sk *sk, const uint8_t seed[32],
                        const uint8_t a_seed[32], uint32_t op_id, const uint64_t *pt, uint64_t *ct,
                        void *ws, size_t ws_bytes, void *stream);

/* The server's side of the seed-compressed upload: ct[x][0] = c0[x] and
 * ct[x][1][l] = a_l drawn from a_seed (tag 4, prime l, op_id, object x), so that
 * ct equals what pimm_encrypt_seeded produced on the client.
 * c0: [I][L][N], ct: [I][2][L][N] (device, not overlapping).  Allocates nothing. */
int pimm_ct_expand(const pimm_plan *plan, const uint8_t a_seed[32], uint32_t op_id,
                   const uint64_t *c0, uint64_t *ct, void *stream);

/* Algorithm 1 step 4, client side: decrypt the decoded coefficients
 * (section 3.1.3: coefficient i of c0 + c1 s needs (c0)_i and all of c1),
 * x = CRT, v = floor((t x + floor(q/2)) / q) mod t, and place them by pi_C^{-1}:
 * client_share[kb*nb + k][ib*mb + i] = v.  Rows and columns past n, m are dropped. */
int pimm_decrypt(const pimm_plan *plan, const pimm_sk *sk, const uint64_t *c1, const uint64_t *c0s,
                 uint64_t *client_share, void *ws, size_t ws_bytes, void *stream);

/* Decryption of a reply after pimm_mod_switch: as pimm_decrypt with the first
 * L - 1 primes, q' = q_0 ... q_{L-2} and the rounding v = floor((t x + floor(q'/2))
 * / q') mod t.  c1s: [O][L-1][N], c0ss: [O][L-1][mb*nb] (device).  The workspace
 * of pimm_decrypt suffices (this call needs (L-1)/L of it).  PIMM_E_UNSUPPORTED
 * for L = 1. */
int pimm_decrypt_switched(const pimm_plan *plan, const pimm_sk *sk, const uint64_t *c1s,
                          const uint64_t *c0ss, uint64_t *client_share, void *ws, size_t ws_bytes,
                          void *stream);

/* ---- server ---------------------------------------------------------------- */

/* Algorithm 1 step 1, server side, plus the transform the product needs:
 * pi_A per block, a[ib*R + jb][i*rb + rb-1-j] = W[jb*rb + j][ib*mb + i], lifted
 * centred (w < 0 -> q_l - |w|), kept on the device in NTT form.
 * W: [r][m] signed fixed-point integers (device).  Fails with PIMM_E_NOISE when
 * the worst-case noise bound of the reply breaks decryption, PIMM_E_ARG when
 * max |W| > 2^48.  Synchronises `stream` (it reads max |W| back). */
int pimm_weights_create(const pimm_plan *plan, const int64_t *W, pimm_weights **out, void *stream);
int pimm_weights_destroy(pimm_weights *w);

/* Re-encode new weights of the same shape into an existing weight cache, for a
 * plaintext operand that changes from call to call (the attention cross terms of
 * Eq. 2 multiply by the server's share).  The caller states a bound: every
 * |W[k][j]| <= wmax (2^(l-1) for a centred share of Z_{2^l}); entries beyond it
 * void the noise guarantee.  Fails with PIMM_E_NOISE when the bound breaks
 * decryption, PIMM_E_ARG when wmax > 2^48.  Neither synchronises nor allocates.
 * The device words change in stream order on `stream` (a call queued earlier on
 * `stream` sees the old weights, a later one the new); the bound wmax takes effect
 * on the host at once, for the checks of the calls made after this one (the
 * noise check here, the exactness check of pimm_fc_complete). */
int pimm_weights_update(pimm_weights *w, const int64_t *W, uint64_t wmax, void *stream);

/* Algorithm 1 step 3, [[c]] = a [[b]], accumulated over the inner blocks:
 * acc[y = ib*K + kb][comp][l] = sum_jb a[ib*R + jb] * ct[jb*K + kb][comp][l]
 * mod (X^N + 1, q_l), coefficient form. */
int pimm_matmul(const pimm_plan *plan, const pimm_weights *w, const uint64_t *ct, uint64_t *acc,
                void *ws, size_t ws_bytes, void *stream);

/* Algorithm 1 step 3, [[c]] - s, with the sparse reply of section 3.1.3, in place
 * on acc.  With re-randomisation on (pk must then be given, [2][L][N]):
 * acc0 += u pk0 + e1, acc1 += u pk1 + e2 (u ternary tag 6, e1 tag 7, e2 tag 8,
 * object y).  Then the mask s_y over Z_t (tag 9, object y, draw index = the
 * coefficient index) at each decoded position pos = k*mb*rb + i*rb + rb-1:
 * c0s[y][l][k*mb + i] = [acc0[pos] - Delta_l s_y[pos]]_{q_l},
 * server_share[kb*nb + k][ib*mb + i] = s_y[pos]; c1[y] = acc1. */
int pimm_mask_share(const pimm_plan *plan, const uint64_t *pk, const uint8_t seed[32],
                    uint32_t op_id, uint64_t *acc, uint64_t *c1, uint64_t *c0s,
                    uint64_t *server_share, void *ws, size_t ws_bytes, void *stream);

/* pimm_matmul followed by pimm_mask_share in one pass: the same c1, c0s and
 * server_share bytes, without the [O][2][L][N] accumulator buffer.  The
 * re-randomisation term is added in the NTT domain before the inverse
 * transform, and the transform's last stage writes c1, the masked decoded c0
 * coefficients and the server's share directly (Algorithm 1 step 3 and the
 * sparse reply of section 3.1.3). */
int pimm_matmul_share(const pimm_plan *plan, const pimm_weights *w, const uint64_t *pk,
                      const uint8_t seed[32], uint32_t op_id, const uint64_t *ct, uint64_t *c1,
                      uint64_t *c0s, uint64_t *server_share, void *ws, size_t ws_bytes,
                      void *stream);

/* Modulus switching of the reply before it is sent, a wire-format variant of
 * the sparse reply (section 3.1.3): every coefficient c of c1 and of the decoded
 * c0 (residues mod q_0 .. q_{L-1}) becomes round(c / q_{L-1}) as residues mod the
 * first L - 1 primes, so the reply crosses the wire with (L-1)/L of its bytes.
 * c1: [O][L][N], c0s: [O][L][mb*nb] as pimm_mask_share / pimm_matmul_share wrote
 * them; c1_out: [O][L-1][N], c0s_out: [O][L-1][mb*nb] (device; the outputs may
 * not overlap the inputs or each other: PIMM_E_ARG).  w: the weights the reply
 * was made with (their bound decides the noise): PIMM_E_NOISE when
 * pimm_switch_ok fails for them, PIMM_E_UNSUPPORTED for L = 1.  One launch; no
 * allocation, no synchronisation.  The client decrypts with
 * pimm_decrypt_switched. */
int pimm_mod_switch(const pimm_plan *plan, const pimm_weights *w, const uint64_t *c1,
                    const uint64_t *c0s, uint64_t *c1_out, uint64_t *c0s_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that must not call the allocator, harnesses that forbid it):
 * pimm_matmul_share with the workspace taken from scratch memory the library
 * holds in its static device data, PIMM_NOALLOC_SCRATCH_BYTES per device, kept
 * from the loading of the library's code object until the process ends (enough
 * for every product of a BERT-base layer at sequence 128 under the fewest-wire
 * plan; pimm_plan_info does not report the fused step's share of the workspace,
 * so a plan that needs more is rejected with PIMM_E_WORKSPACE before any work is
 * enqueued).  Same arguments, bytes and stream semantics as pimm_matmul_share
 * without ws/ws_bytes; the call itself allocates nothing, and neither does the
 * work it enqueues (keep tracing off: pimm_profile_enable creates HIP events).
 * Every call on one device shares that device's scratch: two calls that overlap
 * on one device (on different streams, or from different threads) race and give
 * undefined results; calls in one stream are ordered and safe.  The scratch
 * keeps the last call's contents; each call writes every scratch word it reads. */
#define PIMM_NOALLOC_SCRATCH_BYTES (128ull << 20)
int pimm_matmul_share_noalloc(const pimm_plan *plan, const pimm_weights *w, const uint64_t *pk,
                              const uint8_t seed[32], uint32_t op_id, const uint64_t *ct,
                              uint64_t *c1, uint64_t *c0s, uint64_t *server_share, void *stream);

/* Completion of a fully connected layer y = x W + b on additive shares (section
 * 3.1, the linear layers).  The input is shared as x = x0 + x1 mod 2^l; the client
 * runs Pi_MatMul on x0, after which the server holds share1 with
 * share0 + share1 = x0 W.  The server holds x1, W and b and adds its local part:
 *     share1[i][j] <- (share1[i][j] + sum_k x1[i][k] W[k][j] + bias[j]) mod 2^l,
 * so that share0 + share1 = x W + b (mod 2^l).
 * x1: device u64 [n][r] (read mod 2^l); W is the matrix `w` was made from (the
 * weights object keeps a copy); bias: device i64 [m] at the scale of the product
 * (2f fractional bits), or NULL; share1: device u64 [n][m], updated in place.
 * Exact: the product runs on FP64 limb sums, so the call fails with PIMM_E_ARG
 * when r * max|W| * (2^ceil(l/2) - 1) reaches 2^53.  ws: at least
 * pimm_plan_info.workspace_bytes (uses n*m*16 bytes). */
int pimm_fc_complete(const pimm_plan *plan, const pimm_weights *w, const uint64_t *x1,
                     const int64_t *bias, uint64_t *share1, void *ws, size_t ws_bytes,
                     void *stream);

/* ---- batching: many products in one pass ----------------------------------------- */

/* One product of a batch: a plan, a weight cache that fits it (same r, m, mb, rb),
 * its input ciphertexts [I][2][L][N] and its accumulator output [O][2][L][N]. */
typedef struct {
    const pimm_plan *plan;
    const pimm_weights *weights;
    const uint64_t *ct;
    uint64_t *acc;
} pimm_batch_item;

/* Build a batch of `count` products of any shapes and lengths on one context
 * (uploads an item table to the device; the items' buffers must stay valid while
 * the batch is used).  pimm_batch_matmul then computes, for every item, exactly
 * what pimm_matmul computes for it. */
int pimm_batch_create(const pimm_batch_item *items, uint32_t count, pimm_batch **out);
int pimm_batch_destroy(pimm_batch *batch);
/* Workspace bytes the batch needs and the useful multiply-accumulates it does
 * (sum of n*r*m); either pointer may be NULL. */
int pimm_batch_query(const pimm_batch *batch, uint64_t *workspace_bytes, uint64_t *useful_macs);
/* Schedule: schedule 0 = three launches (all forward NTTs, all slot-wise products,
 * all inverse NTTs); 1 = one persistent launch whose workgroups take units from an
 * atomic queue in dependency order, with bounded waits.  mac_rows x mac_cols is the
 * product tile a thread owns (as pimm_plan_set_tuning); xcd_map != 0 places
 * consecutive product tiles on one XCD; grid = persistent workgroups (0: fill the
 * device). */
int pimm_batch_set_schedule(pimm_batch *batch, int schedule, int mac_rows, int mac_cols,
                            int xcd_map, uint32_t grid);
/* The schedule in force (after pimm_batch_set_schedule or pimm_batch_autotune). */
int pimm_batch_get_schedule(const pimm_batch *batch, int *schedule, int *mac_rows, int *mac_cols,
                            int *xcd_map, uint32_t *grid);
/* Run every product of the batch on `stream` (plain kernel launches only, so the
 * call can be captured into a hipGraph and replayed; one run at a time per workspace). */
int pimm_batch_matmul(const pimm_batch *batch, void *ws, size_t ws_bytes, void *stream);
/* Time the batch under each schedule candidate (phased / persistent, product tile,
 * XCD placement) with HIP events on `stream` and keep the fastest. */
int pimm_batch_autotune(pimm_batch *batch, void *ws, size_t ws_bytes, int reps, void *stream,
                        double *best_ms);
/* After a persistent run: synchronise `stream` and report PIMM_E_DEVICE if a
 * dependency wait hit its bound (the outputs are then invalid). */
int pimm_batch_status(const pimm_batch *batch, const void *ws, void *stream);

/* ---- serving: continuous batching of private-inference requests -------------------- */

/* A stack of `layers` x `ops` products per request; op o of every layer is
 * d_in[o] x d_out[o].  weights[layer * ops + o] must fit the plan with block area
 * d_fix (same r, m, mb, rb), which makes one cache serve every sequence length.
 * hbm_budget: device bytes the server allocates once and hands to requests
 * (key, ciphertexts, accumulators, reply, scratch); max_active: most requests in
 * flight; schedule / mac_rows / mac_cols: the batched product's schedule (as
 * pimm_batch_set_schedule; mac_rows 0 means 8, mac_cols 0 means 1); min_batch: the
 * fewest requests at one step that run together as one batched pass (with fewer, the
 * oldest runs alone through the plain fused call; 0 means 8). */
typedef struct {
    uint32_t layers, ops;
    const uint32_t *d_in, *d_out;
    const pimm_weights *const *weights;
    uint32_t d_fix;
    uint64_t hbm_budget;
    uint32_t max_active;
    int32_t schedule;
    uint32_t mac_rows, mac_cols;
    uint32_t min_batch;
} pimm_serve_config;

/* A request: unique id, sequence length, arrival time in seconds from the start of
 * the run, and the two parties' 32-byte seeds.  Product k of the stack draws its
 * client share X[seq][d_in] from stream (tag 10, op_id = k, object = low 32 bits of
 * id) and uses op_id = k for encryption, re-randomisation and mask. */
typedef struct {
    uint64_t id;
    uint32_t seq, reserved;
    double arrival_s;
    uint8_t client_seed[32], server_seed[32];
} pimm_request;

/* Per request: times (seconds from the start of the run) of arrival, admission and
 * completion (the last product's client share is ready); two order-independent
 * checksums over every product's shares: of the (client, server) pairs, and of
 * their sum mod 2^l (which is X W); useful multiply-accumulates; products done. */
typedef struct {
    uint64_t id;
    double arrival_s, admit_s, done_s;
    uint64_t pair_checksum, sum_checksum, useful_macs;
    uint32_t steps, reserved;
} pimm_request_result;

int pimm_serve_create(pimm_ctx *ctx, const pimm_serve_config *cfg, pimm_server **out);
int pimm_serve_destroy(pimm_server *server);
/* Device bytes one request of length seq holds while it is in flight. */
int pimm_serve_footprint(const pimm_server *server, uint32_t seq, uint64_t *bytes);
/* Replay `count` requests in real time on `stream`: admit each at or after its
 * arrival when the budget has room (arrival order); at each tick run the step (layer,
 * op) of the oldest admitted request for every admitted request at that step, their
 * products in one batched launch that reads the step's weight cache once, when at
 * least min_batch are at that step (otherwise the oldest request runs alone through
 * the plain fused call); return when every request is done.  Requests
 * admitted behind a running one gather at step 0 and then run as one cohort.
 * results[i] belongs to reqs[i]. */
int pimm_serve_run(pimm_server *server, const pimm_request *reqs, uint32_t count,
                   pimm_request_result *results, void *stream);

/* ---- primitives exposed for checking ----------------------------------------- */

/* c = a * b mod (X^N + 1, q_l) for count pairs of polynomials laid out
 * [count][L][N] (canonical residues, device).  The ring product that
 * ciphertext-plaintext multiplication is made of (section 3.1.3 footnote). */
int pimm_poly_mul(pimm_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t count,
                  void *ws, size_t ws_bytes, void *stream);
/* Workspace bytes pimm_poly_mul needs for `count` pairs. */
uint64_t pimm_poly_mul_workspace(const pimm_ctx *ctx, uint32_t count);

/* Sample one polynomial of N coefficients from stream (tag, prime, op_id, obj):
 * kind 0 uniform mod q_prime (uint64), 1 ternary (int64), 2 Gaussian (int64),
 * 3 mask mod 2^l (uint64).  out: [N] (device). */
int pimm_sample_poly(pimm_ctx *ctx, int kind, const uint8_t seed[32], uint32_t tag, uint32_t prime,
                     uint32_t op_id, uint32_t obj, void *out, void *stream);

/* ---- tracing ----------------------------------------------------------------- */

/* on != 0: from now on bracket every kernel launch of the library with two HIP
 * events recorded on the launch's stream, filed under the kernel class
 * ("ntt_fwd", "ntt_inv", "mac", "sample", "encode", "decode", "mask_extract",
 * "fused", "fc", "mod_switch").  Each recorded event delays the next dependent launch by a few
 * microseconds, so a timed region should record only the classes it reports. */
int pimm_profile_enable(int on);
/* Restrict recording to a comma-separated list of kernel classes (NULL or "":
 * every class). */
int pimm_profile_select(const char *classes);
/* Wait for the events recorded for `kernel`, report how many launches they cover
 * and their summed duration in milliseconds, and forget them. */
int pimm_profile_read(const char *kernel, uint64_t *count, double *total_ms);

/* ---- misc ------------------------------------------------------------------ */

int pimm_sync(void *stream);
const char *pimm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PIMM_H */
