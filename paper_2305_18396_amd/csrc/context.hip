// context.hip -- parameters, plans, keys, sampling and the ring-product primitive.
//
// Parameters follow section 2.2 (BFV with RNS: N a power of two, t = 2^l,
// q a product of word-size primes).  The paper fixes only N = 8192 and
// q ~ 180 bits for its runs; the library takes N, L and l from the caller and
// uses the L largest primes below 2^50 that are 1 mod 2N (so negacyclic NTTs
// of length N exist and every residue is an exact double).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "common.h"
#include "mfma.h"
#include "ntt.h"

extern "C" int pimm_host_cdt(int len, uint64_t *out);

namespace pimm {

static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return PIMM_OK;
    if (e == hipErrorOutOfMemory) return set_error(PIMM_E_OOM, "%s: %s", what, hipGetErrorString(e));
    return set_error(PIMM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

Key make_key(const uint8_t seed[32])
{
    Key k;
    for (int i = 0; i < 8; ++i)
        k.w[i] = (uint32_t)seed[4 * i] | ((uint32_t)seed[4 * i + 1] << 8) |
                 ((uint32_t)seed[4 * i + 2] << 16) | ((uint32_t)seed[4 * i + 3] << 24);
    return k;
}

// ---- host integer arithmetic -------------------------------------------------

using u128 = unsigned __int128;

static uint64_t h_mul(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

static uint64_t h_pow(uint64_t a, uint64_t e, uint64_t q)
{
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = h_mul(r, a, q);
        a = h_mul(a, a, q);
        e >>= 1;
    }
    return r;
}

static uint64_t h_inv(uint64_t a, uint64_t q) { return h_pow(a, q - 2, q); }

// Miller-Rabin with the first twelve prime bases: deterministic below 3.3e24.
static bool h_is_prime(uint64_t n)
{
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t b : bases)
        if (n % b == 0) return n == b;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++s;
    }
    for (uint64_t a : bases) {
        uint64_t x = h_pow(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < s; ++i) {
            x = h_mul(x, x, n);
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

static uint32_t bitrev(uint32_t x, int bits)
{
    uint32_t r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

// Residue v in [0, q) as the balanced double in (-q/2, q/2].
static double balanced(uint64_t v, uint64_t q)
{
    return v > q / 2 ? -(double)(q - v) : (double)v;
}

// Little-endian multi-limb helpers for q = prod q_l (at most 4 x 50 bits).
static void limbs_mul_small(uint64_t *x, int n, uint64_t m)
{
    u128 carry = 0;
    for (int i = 0; i < n; ++i) {
        u128 v = (u128)x[i] * m + carry;
        x[i] = (uint64_t)v;
        carry = v >> 64;
    }
}

static uint64_t limbs_mod_small(const uint64_t *x, int n, uint64_t q)
{
    uint64_t r = 0;
    for (int i = n - 1; i >= 0; --i) r = (uint64_t)((((u128)r << 64) | x[i]) % q);
    return r;
}

static void limbs_shr(const uint64_t *x, uint64_t *y, int n, int s)
{
    for (int i = 0; i < n; ++i) {
        int w = i + s / 64, b = s % 64;
        uint64_t lo = w < n ? x[w] >> b : 0;
        uint64_t hi = (b && w + 1 < n) ? x[w + 1] << (64 - b) : 0;
        y[i] = lo | hi;
    }
}

// q = q_0 ... q_{L-1} as limbs, floor(q/2), Delta = floor(q / 2^l) mod q_i and q as a
// double, for the first L primes of q[].
static void fill_modulus(DevParams &d, const uint64_t *q, int L, int log2_t)
{
    uint64_t Q[kMaxL + 1] = {1, 0, 0, 0, 0};
    for (int l = 0; l < L; ++l) limbs_mul_small(Q, kMaxL + 1, q[l]);
    memcpy(d.Q, Q, sizeof Q);
    limbs_shr(Q, d.halfQ, kMaxL + 1, 1);
    uint64_t Delta[kMaxL + 1];
    limbs_shr(Q, Delta, kMaxL + 1, log2_t);
    for (int l = 0; l < kMaxL; ++l) d.delta[l] = l < L ? limbs_mod_small(Delta, kMaxL + 1, q[l]) : 0;
    long double qd = 0.0L;
    for (int i = kMaxL; i >= 0; --i) qd = qd * 18446744073709551616.0L + (long double)Q[i];
    d.Qd = (double)qd;
}

// ---- context -----------------------------------------------------------------

static int build_context(const pimm_params &prm, int device, Ctx *c, bool upload)
{
    if (prm.N < (1u << kMinLogN) || prm.N > (1u << kMaxLogN) || (prm.N & (prm.N - 1)))
        return set_error(PIMM_E_PARAMS, "N = %u must be a power of two in [%d, %d]", prm.N,
                         1 << kMinLogN, 1 << kMaxLogN);
    if (prm.L < 1 || prm.L > (uint32_t)kMaxL)
        return set_error(PIMM_E_PARAMS, "L = %u must be in [1, %d]", prm.L, kMaxL);
    if (prm.log2_t < 2 || prm.log2_t > 48)
        return set_error(PIMM_E_PARAMS, "log2_t = %u must be in [2, 48]", prm.log2_t);
    if (prm.prime_bits != 50)
        return set_error(PIMM_E_PARAMS, "prime_bits = %u: only 50-bit primes are supported",
                         prm.prime_bits);
    c->params = prm;
    c->device = device;
    const int N = (int)prm.N, L = (int)prm.L;
    int logN = 0;
    while ((1 << logN) < N) ++logN;

    // Primes: the L largest q < 2^50 with q = 1 mod 2N, descending.
    uint64_t k = ((1ull << 50) - 2) / (2ull * N);
    for (int l = 0; l < L; --k) {
        uint64_t cand = k * 2ull * N + 1;
        if (cand < (1ull << 50) && h_is_prime(cand)) c->q[l++] = cand;
    }
    // psi: g^((q-1)/2N) for the first g with psi^N = -1 (then psi has order exactly 2N).
    for (int l = 0; l < L; ++l) {
        const uint64_t q = c->q[l];
        c->psi[l] = 0;
        for (uint64_t g = 2; g < 1000; ++g) {
            uint64_t ps = h_pow(g, (q - 1) / (2ull * N), q);
            if (h_pow(ps, N, q) == q - 1) {
                c->psi[l] = ps;
                break;
            }
        }
        if (!c->psi[l]) return set_error(PIMM_E_PARAMS, "no 2N-th root of unity mod q_%d", l);
    }

    DevParams &d = c->dp;
    memset(&d, 0, sizeof d);
    d.N = N;
    d.logN = logN;
    d.L = L;
    d.ell = (int)prm.log2_t;
    for (int l = 0; l < L; ++l) {
        d.q[l] = c->q[l];
        d.p[l] = (double)c->q[l];
        d.pinv[l] = 1.0 / (double)c->q[l];
        d.n_inv[l] = balanced(h_inv((uint64_t)N, c->q[l]), c->q[l]);
    }
    fill_modulus(d, c->q, L, (int)prm.log2_t);
    // Garner constants for the mixed-radix CRT.
    for (int l = 0; l < L; ++l) {
        uint64_t prod = 1 % c->q[l];
        for (int i = 0; i < l; ++i) {
            d.garner_c[l][i] = (double)prod;
            prod = h_mul(prod, c->q[i] % c->q[l], c->q[l]);
        }
        d.garner_inv[l] = (double)h_inv(prod, c->q[l]);
    }
    if (pimm_host_cdt(kCdtLen, d.cdt) != 0) return set_error(PIMM_E_PARAMS, "CDT table failed");

    if (!upload) return PIMM_OK;
    // Twiddles: forward psi^bitrev(k), inverse psi^-bitrev(k), balanced doubles.
    std::vector<double> tw(2ull * L * N);
    for (int l = 0; l < L; ++l) {
        const uint64_t q = c->q[l], pinvv = h_inv(c->psi[l], q);
        for (int i = 0; i < N; ++i) {
            uint32_t e = bitrev((uint32_t)i, logN);
            tw[(size_t)l * N + i] = balanced(h_pow(c->psi[l], e, q), q);
            tw[((size_t)L + l) * N + i] = balanced(h_pow(pinvv, e, q), q);
        }
    }
    int rc = check_hip(hipSetDevice(device), "hipSetDevice");
    if (rc) return rc;
    rc = check_hip(hipMalloc((void **)&c->d_tw, tw.size() * sizeof(double)), "hipMalloc twiddles");
    if (rc) return rc;
    rc = check_hip(hipMemcpy(c->d_tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice),
                   "copy twiddles");
    if (rc) return rc;
    d.tw_fwd = c->d_tw;
    d.tw_inv = c->d_tw + (size_t)L * N;
    return PIMM_OK;
}

// ---- plans -------------------------------------------------------------------

static uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

uint64_t fused_workspace_bytes(const Ctx &c, const pimm_plan_info &f)
{
    const uint64_t N = c.params.N, L = c.params.L;
    return (((uint64_t)f.I + f.O) * 2 * L * N + 2 * L * N + (uint64_t)f.O * L * N +
            (uint64_t)f.O * 3 * N) * 8;
}

static void fill_info(const Ctx &c, pimm_plan_info &f)
{
    const uint64_t N = c.params.N, L = c.params.L;
    if (f.groups < 1) f.groups = 1;
    const uint32_t G = f.groups;
    f.M = (uint32_t)ceil_div(f.m, f.mb);
    f.R = (uint32_t)ceil_div(f.r, f.rb);
    f.K = (uint32_t)ceil_div(f.n, f.nb);
    f.I = G * f.R * f.K;
    f.O = G * f.M * f.K;
    f.Wb = G * f.M * f.R;
    f.P = (uint64_t)G * f.M * f.R * f.K;
    f.pt_bytes = (uint64_t)f.I * N * 8;
    f.ct_bytes = (uint64_t)f.I * 2 * L * N * 8;
    f.acc_bytes = (uint64_t)f.O * 2 * L * N * 8;
    f.c1_bytes = (uint64_t)f.O * L * N * 8;
    f.c0s_bytes = (uint64_t)f.O * L * f.mb * f.nb * 8;
    f.share_bytes = (uint64_t)G * f.n * f.m * 8;
    f.weights_bytes = (uint64_t)f.Wb * L * N * 8;
    if (mfma_eligible(f)) f.weights_bytes += digit_cache_bytes(c, f);  // digit form (mfma.h)
    // Scratch of each call (see the call's implementation for the layout).
    const uint64_t enc = (uint64_t)f.I * N * 8 * (L + 1);
    const uint64_t mm = ((uint64_t)f.I + f.O) * 2 * L * N * 8;
    const uint64_t msk = 2 * L * N * 8 + (uint64_t)f.O * L * N * 8 + (uint64_t)f.O * 3 * N * 8;
    const uint64_t dec = (uint64_t)f.O * L * f.mb * f.nb * 8;
    uint64_t ws = enc;
    const uint64_t fused = fused_workspace_bytes(c, f);
    if (fused > ws) ws = fused;
    if (mm > ws) ws = mm;
    if (msk > ws) ws = msk;
    if (dec > ws) ws = dec;
    if (G == 1) {
        uint32_t fc_kc = 0, fc_pieces = 0;
        fc_cut(f.n, f.r, f.m, &fc_kc, &fc_pieces);
        const uint64_t fc = (uint64_t)fc_pieces * f.n * f.m * 2 * 8;  // the FC completion's partial sums
        if (fc > ws) ws = fc;
    }
    f.workspace_bytes = ws;
}

int plan_rule(const Ctx &c, uint32_t n, uint32_t r, uint32_t m, uint32_t mb, uint32_t rb,
              uint32_t nb, uint32_t d_fix, pimm_plan_info &f)
{
    const uint64_t N = c.params.N;
    memset(&f, 0, sizeof f);
    f.n = n;
    f.r = r;
    f.m = m;
    if (mb && rb && nb) {
        if ((uint64_t)mb * rb * nb > N)
            return set_error(PIMM_E_SHAPE, "block %u x %u x %u exceeds N = %llu", mb, rb, nb,
                             (unsigned long long)N);
        f.mb = mb;
        f.rb = rb;
        f.nb = nb;
    } else if (d_fix) {
        if ((d_fix & (d_fix - 1)) || d_fix > N)
            return set_error(PIMM_E_SHAPE, "d_fix = %u must be a power of two <= N", d_fix);
        uint64_t best_cost = ~0ull, bm = 1;
        for (uint64_t tm = 1; tm <= d_fix; tm *= 2) {
            uint64_t cost = ceil_div(r, d_fix / tm) + ceil_div(m, tm);
            if (cost < best_cost || (cost == best_cost && tm > bm)) {
                best_cost = cost;
                bm = tm;
            }
        }
        f.mb = (uint32_t)bm;
        f.rb = (uint32_t)(d_fix / bm);
        f.nb = (uint32_t)(n < N / d_fix ? n : N / d_fix);
    } else {
        uint64_t best_cost = ~0ull, bnb = 0, bmb = 0, brb = 0;
        for (uint64_t tm = 1; tm <= next_pow2(m) && tm <= N; tm *= 2)
            for (uint64_t tr = 1; tr <= next_pow2(r) && tm * tr <= N; tr *= 2) {
                uint64_t tn = N / (tm * tr);
                if (tn > n) tn = n;
                uint64_t cost = (ceil_div(r, tr) + ceil_div(m, tm)) * ceil_div(n, tn);
                bool better = cost < best_cost || (cost == best_cost && tn > bnb) ||
                              (cost == best_cost && tn == bnb && tm > bmb);
                if (better) {
                    best_cost = cost;
                    bnb = tn;
                    bmb = tm;
                    brb = tr;
                }
            }
        f.mb = (uint32_t)bmb;
        f.rb = (uint32_t)brb;
        f.nb = (uint32_t)bnb;
    }
    fill_info(c, f);
    if ((uint64_t)f.Wb * c.params.L >= (1ull << 31) || (uint64_t)f.I * 2 * c.params.L >= (1ull << 31))
        return set_error(PIMM_E_SHAPE, "plan has too many blocks for one launch");
    return PIMM_OK;
}

// Worst-case decryption noise of a reply coefficient (exact, 128-bit):
//   R*D*wmax*19           products a * e of every inner block (|e| <= 19),
//   (q mod t)(r*wmax + 1) Delta*t = q - (q mod t): each multiple of t carried by
//                         the integer product a*b and the mask's wrap past t,
//   2*N*19 + 19           u*e' + e1 + e2*s of the re-randomisation (if on).
static unsigned __int128 noise_bound(const Ctx &c, const pimm_plan_info &f, uint64_t wmax)
{
    using u128 = unsigned __int128;
    const uint64_t t = 1ull << c.params.log2_t;
    const uint64_t qt = c.dp.Q[0] & (t - 1);
    const u128 D = (u128)f.mb * f.rb;
    u128 E = (u128)f.R * D * wmax * kCdtLen + (u128)qt * ((u128)f.r * wmax + 1);
    if (c.params.rerandomize) E += (u128)2 * c.params.N * kCdtLen + kCdtLen;
    return E;
}

// lhs < Q for lhs < 2^128 and Q as kMaxL + 1 limbs.
static bool u128_below(unsigned __int128 lhs, const uint64_t *Q)
{
    const uint64_t l[kMaxL + 1] = {(uint64_t)lhs, (uint64_t)(lhs >> 64), 0, 0, 0};
    for (int i = kMaxL; i >= 0; --i)
        if (l[i] != Q[i]) return l[i] < Q[i];
    return false;
}

// Decryption rounds correctly when 2 t (E + (q mod t)) < q.
bool noise_ok(const Ctx &c, const pimm_plan_info &f, uint64_t wmax)
{
    using u128 = unsigned __int128;
    const uint64_t t = 1ull << c.params.log2_t;
    const uint64_t qt = c.dp.Q[0] & (t - 1);
    // lhs = 2 t (E + qt) as limbs; compare with q.
    const u128 a = noise_bound(c, f, wmax) + qt;
    uint64_t lhs[kMaxL + 1] = {0, 0, 0, 0, 0};
    const int sh = (int)c.params.log2_t + 1;  // 3 .. 49
    // a < 2^110, so a << sh < 2^160 spans three limbs.
    const u128 lo = a << sh;
    lhs[0] = (uint64_t)lo;
    lhs[1] = (uint64_t)(lo >> 64);
    lhs[2] = (uint64_t)(a >> (128 - sh));
    for (int i = kMaxL; i >= 0; --i) {
        if (lhs[i] != c.dp.Q[i]) return lhs[i] < c.dp.Q[i];
    }
    return false;
}

// Modulus switching of the reply to q' = q / q_{L-1}.  Each coefficient c becomes
// round(c / q_{L-1}); in c0 + c1 s the noise becomes E q'/q = E / q_{L-1} plus the
// rounding of c0 and of the N products of c1 with the ternary key (each rounding at
// most 1/2), so E' = ceil(E / q_{L-1}) + (N + 2) / 2.  The message's scale becomes
// Delta q'/q, which is q'/t less (q mod t) q'/(q t) < 1, so decryption mod q' still
// rounds to the reply's value when 2 t (E' + 1) < q'.
bool switch_ok(const Ctx &c, const pimm_plan_info &f, uint64_t wmax)
{
    using u128 = unsigned __int128;
    const int L = c.params.L;
    if (L < 2) return false;
    const uint64_t qd = c.q[L - 1];
    const u128 E = noise_bound(c, f, wmax);
    const u128 Es = (E + qd - 1) / qd + (c.params.N + 2) / 2;  // < 2^61
    const u128 lhs = (u128)2 * (1ull << c.params.log2_t) * (Es + 1);  // < 2^104
    uint64_t Qs[kMaxL + 1] = {1, 0, 0, 0, 0};
    for (int l = 0; l < L - 1; ++l) limbs_mul_small(Qs, kMaxL + 1, c.q[l]);
    return u128_below(lhs, Qs);
}

// The reply's parameters after the switch: the first L - 1 primes with their
// transform and CRT tables as they are (the tables are per prime and the Garner
// constants of prime l depend only on the primes before it), and q', floor(q'/2),
// Delta' = floor(q' / t) and q' as a double.  qd_inv[l] = q_{L-1}^{-1} mod q_l,
// balanced, for l < L - 1.
void switched_params(const Ctx &c, DevParams &d, double *qd_inv)
{
    const int L = c.params.L;
    d = c.dp;
    d.L = L - 1;
    fill_modulus(d, c.q, L - 1, (int)c.params.log2_t);
    for (int l = 0; l < kMaxL; ++l)
        qd_inv[l] = l < L - 1 ? balanced(h_inv(c.q[L - 1] % c.q[l], c.q[l]), c.q[l]) : 0.0;
}

// ---- sampling kernels --------------------------------------------------------

// One thread per ChaCha20 block of stream (tag, prime, op, obj0 + o):
// KIND 0 writes eight uniform residues mod q_prime (uint64), 1 eight ternary
// values (int64), 2 eight Gaussian values (int64), 3 eight Z_{2^l} values (uint64).
template <int KIND>
__device__ __forceinline__ void sample_block(const Key &key, uint32_t op, const SampleJob &jb,
                                             uint32_t gid, const DevParams &dp, const uint64_t *cdt32)
{
    constexpr int per = 8;
    // gid = (o * nprime + li) * (N / 8) + b; the host keeps every job below 2^31 threads.
    const int lognb = dp.logN - 3;
    const uint32_t rest = gid >> lognb;
    if (rest >= (uint32_t)jb.nprime * (uint32_t)jb.nobj) return;
    const uint32_t b = gid & ((1u << lognb) - 1u);
    const uint32_t o = jb.pdiv.div(rest);
    const uint32_t li = rest - o * (uint32_t)jb.nprime;
    const int l = jb.prime0 + (int)li;
    uint32_t w[16];
    chacha_block(key, (uint32_t)b, nonce0(jb.tag, KIND == 0 ? (uint32_t)l : 0u), op,
                 jb.obj0 + (uint32_t)o, w);
    const size_t base = (size_t)o * jb.obj_stride + (size_t)li * jb.prime_stride + (size_t)b * per;
    if (KIND == 0) {
        // Uniform mod q_l: the low 50 bits of the draw when below q_l; the rare
        // rejected draws (probability below 2^-29) take the same draw of the
        // fallback stream, whose residue below 2^50 < 2 q_l is reduced by one
        // subtraction.
        const uint64_t m50 = (1ull << 50) - 1, q = dp.q[l];
        uint64_t *dst = (uint64_t *)jb.out + base;
        uint32_t rejected = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint64_t x = word64(w, i) & m50;
            dst[i] = x;
            rejected |= (x >= q ? 1u : 0u) << i;
        }
        if (rejected) {
            chacha_block(key, (uint32_t)b, nonce0(jb.tag, (uint32_t)l) | kFallbackTag, op,
                         jb.obj0 + (uint32_t)o, w);
            for (int i = 0; i < 8; ++i) {
                if (!((rejected >> i) & 1u)) continue;
                const uint64_t x = word64(w, i) & m50;
                dst[i] = x >= q ? x - q : x;
            }
        }
    } else if (KIND == 1) {
        int64_t *dst = (int64_t *)jb.out + base;
#pragma unroll
        for (int i = 0; i < 8; ++i) dst[i] = ternary_of(word64(w, i));
    } else if (KIND == 2) {
        int64_t *dst = (int64_t *)jb.out + base;
#pragma unroll
        for (int i = 0; i < 8; ++i) dst[i] = gauss_of_lds(word64(w, i), cdt32);
    } else if (KIND == kSampleTernary8 || KIND == kSampleGauss8) {
        // The same values as kinds 1 and 2 (|value| <= 19), one byte each.
        uint64_t packed = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t v = KIND == kSampleTernary8 ? ternary_of(word64(w, i))
                                                      : gauss_of_lds(word64(w, i), cdt32);
            packed |= (uint64_t)(uint8_t)(int8_t)v << (8 * i);
        }
        *(uint64_t *)((int8_t *)jb.out + base) = packed;
    } else {
        uint64_t *dst = (uint64_t *)jb.out + base;
#pragma unroll
        for (int i = 0; i < 8; ++i) dst[i] = mask_of(word64(w, i), dp.ell);
    }
}

// Up to kMaxSampleJobs independent sampling jobs of one party and operation in
// one launch: workgroups [first_k, first_k + blocks_k) serve job k.
__global__ __launch_bounds__(256) void k_sample(Key key, uint32_t op, SampleJobs js, DevParams dp)
{
    // The Gaussian table in LDS for gauss_of_lds (every workgroup, whatever its job's kind:
    // the barrier must be reached by all of its threads).
    __shared__ uint64_t cdt32[kCdtPad];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kCdtPad; ++k) cdt32[k] = k < kCdtLen ? dp.cdt[k] : ~0ull;
    }
    __syncthreads();
    uint32_t b = blockIdx.x;
    int k = 0;
    while (k + 1 < js.n && b >= js.job[k].blocks) {
        b -= js.job[k].blocks;
        ++k;
    }
    const SampleJob &jb = js.job[k];
    const uint32_t gid = b * blockDim.x + threadIdx.x;
    switch (jb.kind) {
    case 0: sample_block<0>(key, op, jb, gid, dp, cdt32); break;
    case 1: sample_block<1>(key, op, jb, gid, dp, cdt32); break;
    case 2: sample_block<2>(key, op, jb, gid, dp, cdt32); break;
    case kSampleTernary8: sample_block<kSampleTernary8>(key, op, jb, gid, dp, cdt32); break;
    case kSampleGauss8: sample_block<kSampleGauss8>(key, op, jb, gid, dp, cdt32); break;
    default: sample_block<3>(key, op, jb, gid, dp, cdt32); break;
    }
}

int launch_samples(const Ctx &c, const Key &key, uint32_t op, SampleJobs js, hipStream_t s)
{
    if (js.n < 1 || js.n > kMaxSampleJobs) return set_error(PIMM_E_ARG, "launch_samples: %d jobs", js.n);
    const int threads = 256;
    unsigned grid = 0;
    for (int k = 0; k < js.n; ++k) {
        SampleJob &jb = js.job[k];
        const int per = 8;
        const long total = jb.nobj > 0 ? (long)(c.dp.N / per) * jb.nprime * jb.nobj : 0;
        if (total >= (1l << 31) || jb.nprime < 1)
            return set_error(PIMM_E_SHAPE, "launch_samples: job %d has %ld blocks of draws", k, total);
        jb.blocks = (uint32_t)((total + threads - 1) / threads);
        jb.pdiv = FastDiv::make((uint32_t)jb.nprime);
        grid += jb.blocks;
    }
    if (!grid) return PIMM_OK;
    ProfScope prof("sample", s);
    hipLaunchKernelGGL(k_sample, dim3(grid), dim3(threads), 0, s, key, op, js, c.dp);
    return check_hip(hipGetLastError(), "sample launch");
}

int launch_sample(const Ctx &c, int kind, const Key &key, uint32_t tag, uint32_t op, uint32_t obj0,
                  int nobj, int prime0, int nprime, void *out, size_t obj_stride,
                  size_t prime_stride, hipStream_t s)
{
    SampleJobs js{};
    js.n = 1;
    js.job[0] = SampleJob{kind, tag, obj0, nobj, prime0, nprime, out, obj_stride, prime_stride, 0};
    return launch_samples(c, key, op, js, s);
}

// pk0[l][j] = [e'_j - (a' s)_j]_{q_l}: storer of the inverse NTT of a'^ s^.
struct StorePk0 {
    const int64_t *e;
    uint64_t *pk0;  // [L][N]
    int logn;
    // The error word, read ahead of the transform's last pass.
    using Pre = int64_t;
    __device__ Pre pre(const PolyIx &, int j) const { return e[j]; }
    __device__ void operator()(const PolyIx &pi, int j, double v, double p, double pinv, Pre ej) const
    {
        const uint64_t q = (uint64_t)p;
        const uint64_t as = to_canonical(v, p, pinv);
        pk0[((size_t)pi.poly << logn) + j] = sub_mod(lift_small(ej, q), as, q);
    }
};

// Key generation into caller buffers: s (ternary, stream SK), s^ = NTT(s), and
// when pk is given and re-randomisation is on, pk = ([-a' s + e']_q, a').
// tmp: L*N doubles and e: N int64 of scratch.
int keygen_into(const Ctx &c, const Key &key, int64_t *s, double *s_hat, uint64_t *pk, double *tmp,
                int64_t *e, hipStream_t st)
{
    const int N = (int)c.params.N, L = (int)c.params.L, lg = c.dp.logN;
    int rc = launch_sample(c, 1, key, kTagSK, 0, 0, 1, 0, 1, s, 0, 0, st);
    if (!rc) rc = launch_fwd(c, LoadI64Shared{s, lg}, StoreSlots{s_hat, lg}, L, st);
    if (rc || !pk || !c.params.rerandomize) return rc;
    uint64_t *pk1 = pk + (size_t)L * N;
    rc = launch_sample(c, 0, key, kTagPkA, 0, 0, 1, 0, L, pk1, 0, (size_t)N, st);
    if (!rc) rc = launch_sample(c, 2, key, kTagPkE, 0, 0, 1, 0, 1, e, 0, 0, st);
    if (!rc) rc = launch_fwd(c, LoadU64{pk1, lg}, StoreSlots{tmp, lg}, L, st);
    if (!rc)
        rc = launch_inv(c, LoadSlotsMul{tmp, s_hat, lg, 1}, StorePk0{e, pk, lg}, L, st);
    return rc;
}

}  // namespace pimm

using namespace pimm;

// ---- C ABI -------------------------------------------------------------------

extern "C" {

const char *pimm_last_error(void) { return g_err; }

int pimm_sync(void *stream)
{
    return check_hip(hipStreamSynchronize((hipStream_t)stream), "stream synchronize");
}

int pimm_ctx_create(const pimm_params *params, int device, pimm_ctx **out)
{
    if (!params || !out) return set_error(PIMM_E_ARG, "pimm_ctx_create: NULL argument");
    pimm_ctx *c = new pimm_ctx();
    int rc = build_context(*params, device, c, true);
    // The device address of the static scratch of pimm_matmul_share_noalloc, taken
    // once per device while the device is current (build_context made it current).
    if (!rc) rc = bind_noalloc_scratch(device);
    if (rc) {
        if (c->d_tw) (void)hipFree(c->d_tw);
        delete c;
        return rc;
    }
    *out = c;
    return PIMM_OK;
}

int pimm_ctx_destroy(pimm_ctx *ctx)
{
    if (!ctx) return PIMM_OK;
    if (ctx->d_tw) (void)hipFree(ctx->d_tw);
    delete ctx;
    return PIMM_OK;
}

int pimm_ctx_primes(const pimm_ctx *ctx, uint64_t *q_out)
{
    if (!ctx || !q_out) return set_error(PIMM_E_ARG, "pimm_ctx_primes: NULL argument");
    for (uint32_t l = 0; l < ctx->params.L; ++l) q_out[l] = ctx->q[l];
    return PIMM_OK;
}

int pimm_ctx_cdt(const pimm_ctx *ctx, uint64_t *cdt_out)
{
    if (!ctx || !cdt_out) return set_error(PIMM_E_ARG, "pimm_ctx_cdt: NULL argument");
    memcpy(cdt_out, ctx->dp.cdt, sizeof ctx->dp.cdt);
    return PIMM_OK;
}

int pimm_params_primes(const pimm_params *params, uint64_t *q_out)
{
    if (!params || !q_out) return set_error(PIMM_E_ARG, "pimm_params_primes: NULL argument");
    Ctx c;
    int rc = build_context(*params, 0, &c, false);
    if (rc) return rc;
    for (uint32_t l = 0; l < params->L; ++l) q_out[l] = c.q[l];
    return PIMM_OK;
}

int pimm_cdt(uint64_t *cdt_out)
{
    if (!cdt_out) return set_error(PIMM_E_ARG, "pimm_cdt: NULL argument");
    if (pimm_host_cdt(kCdtLen, cdt_out) != 0) return set_error(PIMM_E_PARAMS, "CDT table failed");
    return PIMM_OK;
}

int pimm_plan_rule(const pimm_params *params, uint32_t n, uint32_t r, uint32_t m, uint32_t mb,
                   uint32_t rb, uint32_t nb, uint32_t d_fix, pimm_plan_info *info)
{
    if (!params || !info) return set_error(PIMM_E_ARG, "pimm_plan_rule: NULL argument");
    if (!n || !r || !m) return set_error(PIMM_E_SHAPE, "empty matrix %u x %u x %u", n, r, m);
    Ctx c;
    int rc = build_context(*params, 0, &c, false);
    if (rc) return rc;
    return plan_rule(c, n, r, m, mb, rb, nb, d_fix, *info);
}

int pimm_noise_ok(const pimm_params *params, const pimm_plan_info *info, uint64_t wmax)
{
    if (!params || !info) return set_error(PIMM_E_ARG, "pimm_noise_ok: NULL argument");
    Ctx c;
    int rc = build_context(*params, 0, &c, false);
    if (rc) return rc;
    return noise_ok(c, *info, wmax) ? 1 : 0;
}

int pimm_switch_ok(const pimm_params *params, const pimm_plan_info *info, uint64_t wmax)
{
    if (!params || !info) return set_error(PIMM_E_ARG, "pimm_switch_ok: NULL argument");
    Ctx c;
    int rc = build_context(*params, 0, &c, false);
    if (rc) return rc;
    if (c.params.L < 2)
        return set_error(PIMM_E_UNSUPPORTED, "pimm_switch_ok: one prime cannot be dropped");
    return switch_ok(c, *info, wmax) ? 1 : 0;
}

int pimm_plan_create(pimm_ctx *ctx, uint32_t n, uint32_t r, uint32_t m, uint32_t mb, uint32_t rb,
                     uint32_t nb, uint32_t d_fix, pimm_plan **out)
{
    if (!ctx || !out) return set_error(PIMM_E_ARG, "pimm_plan_create: NULL argument");
    if (!n || !r || !m) return set_error(PIMM_E_SHAPE, "empty matrix %u x %u x %u", n, r, m);
    pimm_plan_info f;
    int rc = plan_rule(*ctx, n, r, m, mb, rb, nb, d_fix, f);
    if (rc) return rc;
    pimm_plan *p = new pimm_plan();
    p->ctx = ctx;
    p->info = f;
    *out = p;
    return PIMM_OK;
}

int pimm_plan_create_grouped(pimm_ctx *ctx, uint32_t n, uint32_t r, uint32_t m, uint32_t mb,
                             uint32_t rb, uint32_t nb, uint32_t d_fix, uint32_t groups,
                             pimm_plan **out)
{
    if (!ctx || !out) return set_error(PIMM_E_ARG, "pimm_plan_create_grouped: NULL argument");
    if (groups < 1 || groups > 65536)
        return set_error(PIMM_E_ARG, "pimm_plan_create_grouped: groups = %u not in [1, 65536]", groups);
    if (!n || !r || !m) return set_error(PIMM_E_SHAPE, "empty matrix %u x %u x %u", n, r, m);
    pimm_plan_info f;
    int rc = plan_rule(*ctx, n, r, m, mb, rb, nb, d_fix, f);
    if (rc) return rc;
    f.groups = groups;
    fill_info(*ctx, f);
    const uint64_t L = ctx->params.L;
    if ((uint64_t)groups * f.M * f.R * L >= (1ull << 31) ||
        (uint64_t)groups * f.R * f.K * 2 * L >= (1ull << 31) ||
        (uint64_t)groups * f.M * f.K * 2 * L >= (1ull << 31))
        return set_error(PIMM_E_SHAPE, "grouped plan has too many blocks for one launch");
    pimm_plan *p = new pimm_plan();
    p->ctx = ctx;
    p->info = f;
    *out = p;
    return PIMM_OK;
}

int pimm_plan_destroy(pimm_plan *plan)
{
    delete plan;
    return PIMM_OK;
}

int pimm_plan_query(const pimm_plan *plan, pimm_plan_info *info)
{
    if (!plan || !info) return set_error(PIMM_E_ARG, "pimm_plan_query: NULL argument");
    *info = plan->info;
    return PIMM_OK;
}

int pimm_sample_poly(pimm_ctx *ctx, int kind, const uint8_t seed[32], uint32_t tag, uint32_t prime,
                     uint32_t op_id, uint32_t obj, void *out, void *stream)
{
    if (!ctx || !seed || !out) return set_error(PIMM_E_ARG, "pimm_sample_poly: NULL argument");
    if (kind < 0 || kind > 3) return set_error(PIMM_E_ARG, "kind %d not in 0..3", kind);
    if (kind == 0 && prime >= ctx->params.L)
        return set_error(PIMM_E_ARG, "prime %u >= L", prime);
    if (kind != 0 && prime != 0) return set_error(PIMM_E_ARG, "only uniform draws are per prime");
    return launch_sample(*ctx, kind, make_key(seed), tag, op_id, obj, 1, (int)prime, 1, out, 0, 0,
                         (hipStream_t)stream);
}

int pimm_keygen(pimm_ctx *ctx, const uint8_t seed[32], pimm_sk **sk_out, uint64_t *pk_out,
                void *stream)
{
    if (!ctx || !seed || !sk_out) return set_error(PIMM_E_ARG, "pimm_keygen: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const int N = (int)ctx->params.N, L = (int)ctx->params.L;
    int rc = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
    if (rc) return rc;
    pimm_sk *sk = new pimm_sk();
    sk->ctx = ctx;
    double *tmp = nullptr;
    int64_t *e = nullptr;
    rc = check_hip(hipMalloc((void **)&sk->d_s, (size_t)N * 8), "hipMalloc sk");
    if (!rc) rc = check_hip(hipMalloc((void **)&sk->d_s_hat, (size_t)L * N * 8), "hipMalloc sk");
    if (!rc) rc = check_hip(hipMalloc((void **)&tmp, (size_t)L * N * 8), "hipMalloc keygen");
    if (!rc) rc = check_hip(hipMalloc((void **)&e, (size_t)N * 8), "hipMalloc keygen");
    if (!rc) rc = keygen_into(*ctx, make_key(seed), sk->d_s, sk->d_s_hat, pk_out, tmp, e, s);
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "keygen synchronize");
    if (tmp) (void)hipFree(tmp);
    if (e) (void)hipFree(e);
    if (rc) {
        pimm_sk_destroy(sk);
        return rc;
    }
    *sk_out = sk;
    return PIMM_OK;
}

int pimm_sk_destroy(pimm_sk *sk)
{
    if (!sk) return PIMM_OK;
    if (sk->d_s) (void)hipFree(sk->d_s);
    if (sk->d_s_hat) (void)hipFree(sk->d_s_hat);
    delete sk;
    return PIMM_OK;
}

uint64_t pimm_poly_mul_workspace(const pimm_ctx *ctx, uint32_t count)
{
    if (!ctx) return 0;
    return 2ull * count * ctx->params.L * ctx->params.N * 8;
}

int pimm_poly_mul(pimm_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t count,
                  void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx || !a || !b || !c) return set_error(PIMM_E_ARG, "pimm_poly_mul: NULL argument");
    if (ws_bytes < pimm_poly_mul_workspace(ctx, count) || (!ws && count))
        return set_error(PIMM_E_WORKSPACE, "pimm_poly_mul: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int np = (int)(count * ctx->params.L);
    const int lg = ctx->dp.logN;
    double *ah = (double *)ws, *bh = ah + ((size_t)np << lg);
    int rc = launch_fwd(*ctx, LoadU64{a, lg}, StoreSlots{ah, lg}, np, s);
    if (!rc) rc = launch_fwd(*ctx, LoadU64{b, lg}, StoreSlots{bh, lg}, np, s);
    if (!rc) rc = launch_inv(*ctx, LoadSlotsMul{ah, bh, lg, 0}, StoreU64{c, lg}, np, s);
    return rc;
}

}  // extern "C"
