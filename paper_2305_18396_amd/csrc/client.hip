// client.hip -- the client's side of Pi_MatMul (Algorithm 1 steps 1, 2 and 4).
#include <string.h>

#include "common.h"
#include "ntt.h"

namespace pimm {


// ---- encode (Algorithm 1 step 1, pi_B) -------------------------------------------

// One thread per plaintext coefficient; every coefficient is written (zeros included).
__global__ void k_encode_input(const uint64_t *X, uint64_t *pt, pimm_plan_info f, int logn)
{
    const size_t N = (size_t)1 << logn;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)f.I * N) return;
    const uint32_t xg = (uint32_t)(gid >> logn);
    const uint32_t jcoef = (uint32_t)(gid & (N - 1));
    // Input x of product g of a grouped plan reads X[g].
    const uint32_t I1 = f.R * f.K, g = xg / I1, x = xg - g * I1;
    X += (size_t)g * f.n * f.r;
    const uint32_t jb = x / f.K, kb = x % f.K;
    const uint32_t D = f.mb * f.rb;
    uint64_t v = 0;
    const uint32_t k = jcoef / D, j = jcoef % D;
    if (k < f.nb && j < f.rb) {
        const uint32_t row = kb * f.nb + k, col = jb * f.rb + j;
        if (row < f.n && col < f.r) v = X[(size_t)row * f.r + col];
    }
    pt[gid] = v;
}

// ---- encrypt (Algorithm 1 step 2) -----------------------------------------------

// Delta_l pt + e for polynomial x*L + l: the coefficients whose forward transform is the
// message part of c0's slots.  Delta_l balanced (|.| <= q_l/2) times pt < t, plus |e| <= 19:
// within 0.6 q_l.  Delta_l travels by value inside the functor (kernel arguments are the only
// host data a kernel may read).
struct LoadEncMsg {
    const uint64_t *pt;  // [I][N], values < t
    const int8_t *e;     // [I][N]
    double delta[kMaxL];
    int logn;
    __device__ double operator()(const PolyIx &pi, int j, double p, double pinv) const
    {
        const size_t at = ((size_t)pi.x << logn) + j;
        return mulmod(delta[pi.l], f64_of(pt[at]), p, pinv) + (double)e[at];
    }
};

// Delta_l pi_B(X) + e for polynomial x*L + l: the encoding of Algorithm 1 step 1 done in the
// encryption's loader, coefficient by coefficient (the values k_encode_input writes): input
// x = (g R + jb) K + kb of product g holds X_g[kb nb + k][jb rb + j] at coefficient k D + j
// (k < nb, j < rb, D = mb rb), zero elsewhere.
struct LoadEncX {
    const uint64_t *X;  // [G][n][r], values < 2^l
    const int8_t *e;    // [I][N]
    double delta[kMaxL];
    FastDiv D, I1, K;   // mb rb, R K, K
    uint32_t rb, nb, n, r;
    int logn;
    __device__ double operator()(const PolyIx &pi, int j, double p, double pinv) const
    {
        // The input's block of X (the same for every element of the workgroup): rows kb nb ..,
        // columns jb rb .., kmax x jmax of them inside X.
        const uint32_t xg = (uint32_t)pi.x, g = I1.div(xg), x = xg - g * I1.d;
        const uint32_t jb = K.div(x), kb = x - jb * K.d;
        const uint32_t kmax = min(nb, n - kb * nb), jmax = min(rb, r - jb * rb);
        const uint64_t *Xb = X + ((size_t)g * n + kb * nb) * r + jb * rb;
        const uint32_t k = D.div((uint32_t)j), jj = (uint32_t)j - k * D.d;
        // Every element reads (X[0] where it holds no input) and selects: a load under a
        // branch would wait for its data before the next element's load is issued.
        const bool in = k < kmax && jj < jmax;
        const uint64_t xv = in ? Xb[(size_t)k * r + jj] : X[0];
        return mulmod(delta[pi.l], f64_of(in ? xv : 0), p, pinv) + (double)e[((size_t)pi.x << logn) + j];
    }
};

// c0's slots [Delta_l pt + e]^ - a^ s^ (mod q_l): the transform's output (balanced) minus a^ s^
// (a^ the ciphertext's c1 slot, canonical; s^ the key's slot, balanced; the product within
// 0.7 q_l), one reduction to the canonical residue.  a^ is read ahead of the transform's last
// pass (Pre: the c0 stores could alias it); the key's doubles cannot alias the stores, so
// their reads are free to move ahead of them.
struct StoreEncC0 {
    uint64_t *ct;      // [I][2][L][N]
    const double *sh;  // [L][N]
    int logn, L;
    struct Pre {
        uint64_t a;
    };
    __device__ Pre pre(const PolyIx &pi, int z) const
    {
        const size_t x = (size_t)pi.x, l = (size_t)pi.l;
        return Pre{ct[(((x * 2 + 1) * L + l) << logn) + z]};
    }
    __device__ void operator()(const PolyIx &pi, int z, double v, double p, double pinv,
                               const Pre &pr) const
    {
        const size_t x = (size_t)pi.x, l = (size_t)pi.l;
        const double as = mulmod(f64_of(pr.a), sh[(l << logn) + z], p, pinv);
        ct[(((x * 2) * L + l) << logn) + z] = to_canonical(v - as, p, pinv);
    }
};

// ---- decrypt (Algorithm 1 step 4, section 3.1.3) ---------------------------------

// (c1 s) of polynomial `poly` (output ciphertext poly / L, prime poly % L) from
// its coefficient form in LDS, at the decoded positions
// pos = k*mb*rb + i*rb + rb-1 -> cs[poly][k*mb + i].
struct DecodedOut {
    uint64_t *cs;
    FastDiv mb;
    uint32_t rb, nb;
    __device__ bool sparse(const PolyIx &) const { return true; }
    template <int LOGN, int T>
    __device__ void run(const PolyIx &pi, const double *lds, const DevParams &dp) const
    {
        const int l = pi.l;
        const double p = dp.p[l], pinv = dp.pinv[l];
        const uint32_t per = mb.d * nb;
        uint64_t *dst = cs + (size_t)pi.poly * per;
        for (uint32_t idx = threadIdx.x; idx < per; idx += blockDim.x) {
            const uint32_t k = mb.div(idx), i = idx - k * mb.d;
            const uint32_t j = (k * mb.d + i) * rb + rb - 1;
            dst[idx] = to_canonical(lds[lds_idx((int)j)], p, pinv);
        }
    }
};

// (c1 s) at the decoded positions of reply polynomial y*L + l, by one workgroup: the forward
// transform of c1 leaves each thread's slots in LDS, where the inverse's first pass (the mirror
// of the forward's last: the same sets on the same threads) reads them back times s^ without a
// barrier; that pass is pruned to the registers the decoded positions depend on (G > 1), the
// other passes follow, and the epilogue reads the decoded positions.  The same values as the
// forward transform to memory followed by k_ntt_inv_lds with LoadSlotsMul, without c1^ leaving
// the compute unit.
template <int LOGN, int G>
__global__ __launch_bounds__(ntt_threads<LOGN>()) void k_decrypt_cs(const uint64_t *c1, const double *sh,
                                                                      DecodedOut epi, DevParams dp)
{
    constexpr int T = ntt_threads<LOGN>();
    using NP = NttPasses<LOGN, T>;
    using P = typename NP::PFirst;
    static_assert(P::PER_THREAD == 1 && P::E == 16 && P::STRIDE == 1, "one set of 16 adjacent slots per thread");
    __shared__ double lds[NP::LDS];
    const int poly = ntt_poly();
    const PolyIx pi = poly_ix(poly, dp.L);
    ntt_fwd_block<LOGN, T>(LoadU64{c1, LOGN}, StoreKeepLds{}, dp, poly, lds);
    const int l = pi.l;
    const double p = dp.p[l], pinv = dp.pinv[l];
    const double *tw = dp.tw_inv + ((size_t)l << LOGN);
    const double *sl = sh + ((size_t)l << LOGN);
    const int S = (int)threadIdx.x;
    const int b0 = lds_idx(P::elem(S, 0));
    double x[P::E];
#pragma unroll
    for (int c = 0; c < P::E; ++c) x[c] = mulmod(lds[b0 + P::lds_off(c)], sl[c * P::NSETS + S], p, pinv);
    if constexpr (G > 1)
        P::template inv_pruned<G>(x, S, tw, p, pinv);
    else
        P::inv(x, S, tw, p, pinv);
#pragma unroll
    for (int c = G - 1; c < P::E; c += G) lds[b0 + P::lds_off(c)] = reduce(x[c], p, pinv);
    // Every wave is past the forward's passes that read the LDS twiddle table.
    __syncthreads();
    load_tw_table<LOGN, T>(tw, lds);
    __syncthreads();
    ntt_inv_rest<LOGN, T, G>(StoreLds{lds}, dp, pi, lds);
    __syncthreads();
    epi.template run<LOGN, T>(pi, lds, dp);
}

template <int LOGN>
static void launch_decrypt_cs(int g, const uint64_t *c1, const double *sh, const DecodedOut &epi, int npoly,
                              const DevParams &dp, hipStream_t s)
{
    if (g == 16)
        hipLaunchKernelGGL((k_decrypt_cs<LOGN, 16>), dim3(npoly), dim3(ntt_threads<LOGN>()), 0, s, c1, sh, epi, dp);
    else if (g == 4)
        hipLaunchKernelGGL((k_decrypt_cs<LOGN, 4>), dim3(npoly), dim3(ntt_threads<LOGN>()), 0, s, c1, sh, epi, dp);
    else
        hipLaunchKernelGGL((k_decrypt_cs<LOGN, 1>), dim3(npoly), dim3(ntt_threads<LOGN>()), 0, s, c1, sh, epi, dp);
}

// Multi-limb helpers (little-endian uint64 limbs, W limbs).
constexpr int W = kMaxL + 1;

__device__ __forceinline__ void limbs_mul_add(uint64_t *x, uint64_t m, uint64_t a)
{
    unsigned __int128 carry = a;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        unsigned __int128 v = (unsigned __int128)x[i] * m + carry;
        x[i] = (uint64_t)v;
        carry = v >> 64;
    }
}

// x -= y; returns the final borrow (1 if the true result is negative).
__device__ __forceinline__ int limbs_sub(uint64_t *x, const uint64_t *y)
{
    uint64_t borrow = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const uint64_t yi = y[i] + borrow;
        const uint64_t nb = (yi < borrow) || (x[i] < yi);
        x[i] -= yi;
        borrow = nb;
    }
    return (int)borrow;
}

__device__ __forceinline__ void limbs_add(uint64_t *x, const uint64_t *y)
{
    uint64_t carry = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const uint64_t s = x[i] + carry;
        const uint64_t c1 = s < carry;
        x[i] = s + y[i];
        carry = c1 + (x[i] < y[i]);
    }
}

// BFV decryption of one coefficient from its residues: x = CRT(res) in [0, q)
// (mixed-radix / Garner form, so no reduction mod q is needed), then
// v = floor((t x + floor(q/2)) / q) mod t.  The quotient is estimated in double
// precision (error below 1/8 for t <= 2^48) and corrected exactly with limbs.
__device__ uint64_t crt_round(const uint64_t *res, const DevParams &dp)
{
    uint64_t v[kMaxL];
    for (int l = 0; l < dp.L; ++l) {
        const double p = dp.p[l], pinv = dp.pinv[l];
        const uint64_t q = dp.q[l];
        uint64_t t = res[l];
        // v[i] < q_i < 2^50 < 2 q_l: the FP64 product takes it unreduced.
        for (int i = 0; i < l; ++i)
            t = sub_mod(t, mul_mod(v[i], (uint64_t)dp.garner_c[l][i], p, pinv), q);
        v[l] = mul_mod(t, (uint64_t)dp.garner_inv[l], p, pinv);
    }
    uint64_t X[W] = {0, 0, 0, 0, 0};
    for (int l = dp.L - 1; l >= 0; --l) {
        if (l == dp.L - 1)
            X[0] = v[l];
        else
            limbs_mul_add(X, dp.q[l], v[l]);
    }
    // num = X * 2^ell + floor(q/2)
    uint64_t num[W];
    const int s = dp.ell;
#pragma unroll
    for (int i = W - 1; i >= 0; --i) num[i] = (X[i] << s) | (i > 0 ? X[i - 1] >> (64 - s) : 0);
    limbs_add(num, dp.halfQ);
    double nd = 0.0;
#pragma unroll
    for (int i = W - 1; i >= 0; --i) nd = nd * 18446744073709551616.0 + (double)num[i];
    uint64_t est = (uint64_t)__builtin_floor(nd / dp.Qd);
    if (est > 0) est -= 1;  // start below the quotient, then step up exactly
    uint64_t prod[W];
#pragma unroll
    for (int i = 0; i < W; ++i) prod[i] = dp.Q[i];
    {
        unsigned __int128 carry = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            unsigned __int128 t = (unsigned __int128)prod[i] * est + carry;
            prod[i] = (uint64_t)t;
            carry = t >> 64;
        }
    }
    // rem = num - est*q >= 0; while rem >= q: rem -= q, est += 1 (at most three steps).
    limbs_sub(num, prod);
    for (int it = 0; it < 4; ++it) {
        uint64_t tmp[W];
#pragma unroll
        for (int i = 0; i < W; ++i) tmp[i] = num[i];
        if (limbs_sub(tmp, dp.Q)) break;
#pragma unroll
        for (int i = 0; i < W; ++i) num[i] = tmp[i];
        est += 1;
    }
    return est & ((1ull << dp.ell) - 1);
}

// One thread per decoded coefficient of each output ciphertext.
__global__ void k_decode(const uint64_t *c0s, const uint64_t *cs, uint64_t *share, pimm_plan_info f,
                         DevParams dp)
{
    const uint32_t per = f.mb * f.nb;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)f.O * per) return;
    const uint32_t o = (uint32_t)(gid / per), idx = (uint32_t)(gid % per);
    const uint32_t k = idx / f.mb, i = idx % f.mb;
    const OutPos op = out_pos(o, f);
    const uint32_t row = op.kb * f.nb + k, col = op.ib * f.mb + i;
    if (row >= f.n || col >= f.m) return;
    uint64_t res[kMaxL];
    for (int l = 0; l < dp.L; ++l) {
        const size_t at = ((size_t)o * dp.L + l) * per + idx;
        res[l] = add_mod(c0s[at], cs[at], dp.q[l]);
    }
    share[(size_t)op.g * f.n * f.m + (size_t)row * f.m + col] = crt_round(res, dp);
}

// Decryption of a reply under the moduli of `c` (the context's, or the first L - 1
// primes after modulus switching): c1 to NTT form, times s^, back to coefficients
// at the decoded positions only, then c0 + c1 s, CRT and rounding per coefficient.
// Workspace: c1^ [O][L][N] doubles, then c1 s at the decoded positions [O][L][mb*nb].
int decrypt_reply(const Ctx &c, const pimm_plan_info &f, const pimm_sk *sk, const uint64_t *c1,
                  const uint64_t *c0s, uint64_t *client_share, void *ws, size_t ws_bytes,
                  hipStream_t s, const char *who)
{
    const size_t L = c.dp.L;
    const size_t per = (size_t)f.mb * f.nb;
    const size_t need = (size_t)f.O * L * per * 8;
    if (!ws || ws_bytes < need) return set_error(PIMM_E_WORKSPACE, "%s: workspace too small", who);
    const int lg = c.dp.logN;
    uint64_t *cs = (uint64_t *)ws;
    int rc;
    {
        const DecodedOut epi{cs, FastDiv::make(f.mb), f.rb, f.nb};
        ProfScope prof("ntt_inv", s);
        if (lg == 12)
            launch_decrypt_cs<12>(prune_factor(f.rb), c1, sk->d_s_hat, epi, (int)(f.O * L), c.dp, s);
        else
            launch_decrypt_cs<13>(prune_factor(f.rb), c1, sk->d_s_hat, epi, (int)(f.O * L), c.dp, s);
        rc = check_hip(hipGetLastError(), "decrypt launch");
    }
    if (!rc) {
        const size_t total = (size_t)f.O * per;
        const int threads = 256;
        ProfScope prof("decode", s);
        hipLaunchKernelGGL(k_decode, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads),
                           0, s, c0s, cs, client_share, f, c.dp);
        rc = check_hip(hipGetLastError(), "decode launch");
    }
    return rc;
}

}  // namespace pimm

using namespace pimm;

extern "C" {

int pimm_encode_input(const pimm_plan *plan, const uint64_t *X, uint64_t *pt, void *stream)
{
    if (!plan || !X || !pt) return set_error(PIMM_E_ARG, "pimm_encode_input: NULL argument");
    const pimm_plan_info &f = plan->info;
    const size_t total = (size_t)f.I << plan->ctx->dp.logN;
    const int threads = 256;
    ProfScope prof("encode", (hipStream_t)stream);
    hipLaunchKernelGGL(k_encode_input, dim3((unsigned)((total + threads - 1) / threads)),
                       dim3(threads), 0, (hipStream_t)stream, X, pt, f, plan->ctx->dp.logN);
    return check_hip(hipGetLastError(), "encode_input launch");
}

// Workspace: a^ [I][L][N] doubles, then e [I][N] (one byte each, in an int64-sized region).
// Symmetric encryption with e drawn from `seed` and a from `a_seed` (the same
// seed for pimm_encrypt).
// The encryption of the plaintexts pt, or (X set) of pi_B(X) encoded on the fly.
static int encrypt_with(const pimm_plan *plan, const pimm_sk *sk, const uint8_t seed[32],
                        const uint8_t a_seed[32], uint32_t op_id, const uint64_t *pt, const uint64_t *X,
                        uint64_t *ct, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !sk || !seed || !a_seed || !(pt || X) || !ct)
        return set_error(PIMM_E_ARG, "pimm_encrypt: NULL argument");
    const Ctx &c = *plan->ctx;
    if (sk->ctx != plan->ctx) return set_error(PIMM_E_ARG, "pimm_encrypt: key of another context");
    const pimm_plan_info &f = plan->info;
    const size_t N = c.params.N, L = c.params.L;
    const size_t need = (size_t)f.I * N * 8 * (L + 1);
    if (!ws || ws_bytes < need) return set_error(PIMM_E_WORKSPACE, "pimm_encrypt: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int lg = c.dp.logN;
    double *ah = (double *)ws;
    int8_t *e = (int8_t *)(ah + (size_t)f.I * L * N);
    const Key key = make_key(seed);
    // c1 = a (uniform per prime, written straight into the ciphertexts) and e: one launch
    // when both come from the same seed, else one per seed.
    const SampleJob ja{0, kTagEncA, 0, (int)f.I, 0, (int)L, ct + L * N, 2 * L * N, N, 0};
    const SampleJob je{kSampleGauss8, kTagEncE, 0, (int)f.I, 0, 1, e, N, 0, 0};
    int rc;
    if (memcmp(seed, a_seed, 32) == 0) {
        SampleJobs js{};
        js.n = 2;
        js.job[0] = ja;
        js.job[1] = je;
        rc = launch_samples(c, key, op_id, js, s);
    } else {
        SampleJobs js{};
        js.n = 1;
        js.job[0] = ja;
        rc = launch_samples(c, make_key(a_seed), op_id, js, s);
        js.job[0] = je;
        if (!rc) rc = launch_samples(c, key, op_id, js, s);
    }
    // The ciphertext travels in evaluation form: a is drawn as its slots (c1 as it is), and
    // c0's slots are the forward transform of Delta pt + e minus a^ s^.
    if (!rc) {
        double delta[kMaxL] = {0.0, 0.0, 0.0, 0.0};
        for (size_t l = 0; l < L; ++l) {
            const uint64_t d = c.dp.delta[l], q = c.q[l];
            delta[l] = d > q / 2 ? -(double)(q - d) : (double)d;
        }
        const StoreEncC0 st{ct, sk->d_s_hat, lg, (int)L};
        if (X) {
            LoadEncX ld{X, e, {0.0, 0.0, 0.0, 0.0}, FastDiv::make(f.mb * f.rb), FastDiv::make(f.R * f.K),
                        FastDiv::make(f.K), f.rb, f.nb, f.n, f.r, lg};
            memcpy(ld.delta, delta, sizeof(delta));
            rc = launch_fwd(c, ld, st, (int)(f.I * L), s);
        } else {
            LoadEncMsg ld{pt, e, {0.0, 0.0, 0.0, 0.0}, lg};
            memcpy(ld.delta, delta, sizeof(delta));
            rc = launch_fwd(c, ld, st, (int)(f.I * L), s);
        }
    }
    return rc;
}

int pimm_encrypt(const pimm_plan *plan, const pimm_sk *sk, const uint8_t seed[32], uint32_t op_id,
                 const uint64_t *pt, uint64_t *ct, void *ws, size_t ws_bytes, void *stream)
{
    return encrypt_with(plan, sk, seed, seed, op_id, pt, nullptr, ct, ws, ws_bytes, stream);
}

int pimm_encrypt_input(const pimm_plan *plan, const pimm_sk *sk, const uint8_t seed[32], uint32_t op_id,
                       const uint64_t *X, uint64_t *ct, void *ws, size_t ws_bytes, void *stream)
{
    if (!X) return set_error(PIMM_E_ARG, "pimm_encrypt_input: NULL argument");
    return encrypt_with(plan, sk, seed, seed, op_id, nullptr, X, ct, ws, ws_bytes, stream);
}

int pimm_encrypt_seeded(const pimm_plan *plan, const pimm_sk *sk, const uint8_t seed[32],
                        const uint8_t a_seed[32], uint32_t op_id, const uint64_t *pt, uint64_t *ct,
                        void *ws, size_t ws_bytes, void *stream)
{
    if (!pt) return set_error(PIMM_E_ARG, "pimm_encrypt_seeded: NULL argument");
    return encrypt_with(plan, sk, seed, a_seed, op_id, pt, nullptr, ct, ws, ws_bytes, stream);
}

// Workspace: cs [O][L][mb*nb] uint64 (the residues of c1 s at the decoded positions).
int pimm_decrypt(const pimm_plan *plan, const pimm_sk *sk, const uint64_t *c1, const uint64_t *c0s,
                 uint64_t *client_share, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !sk || !c1 || !c0s || !client_share)
        return set_error(PIMM_E_ARG, "pimm_decrypt: NULL argument");
    if (sk->ctx != plan->ctx) return set_error(PIMM_E_ARG, "pimm_decrypt: key of another context");
    return decrypt_reply(*plan->ctx, plan->info, sk, c1, c0s, client_share, ws, ws_bytes,
                         (hipStream_t)stream, "pimm_decrypt");
}

}  // extern "C"
