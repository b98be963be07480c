// common.h -- internal types and device arithmetic of libpimm (gfx950).
//
// Residue arithmetic on the hot path runs on the FP64 vector unit, which on
// CDNA4 issues one FMA per lane per clock while 32-bit integer multiplies run
// at a quarter of that.  All primes are below 2^50, so residues and their
// small multiples are exact doubles, and a product a*b (< 2^103) splits
// exactly into h + l with h = RN(a*b) and l = fma(a, b, -h) (the
// error-free product of Dekker / Ogita-Rump-Oishi).  The reduction estimates
// the quotient k = rint(h / p) from a double reciprocal and forms
// (h - k p) + l with one more fma; both steps are exact because the true
// value is an integer far below 2^53 (the floating-point modular product of
// van der Hoeven, Lecerf and Quintin, "Modular SIMD arithmetic in
// Mathemagix", 2014).  Values are kept "balanced": any double of magnitude
// below a few p stands for its residue; canonical [0, q) integers appear only
// where data crosses the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pimm.h"

namespace pimm {

constexpr int kMaxL = 4;
constexpr int kCdtLen = 19;
constexpr int kMinLogN = 12;
constexpr int kMaxLogN = 13;

// Stream tags: which random object a ChaCha20 stream feeds.
enum Tag : uint32_t {
    kTagSK = 1,
    kTagPkA = 2,
    kTagPkE = 3,
    kTagEncA = 4,
    kTagEncE = 5,
    kTagRrU = 6,
    kTagRrE1 = 7,
    kTagRrE2 = 8,
    kTagMask = 9,
};

// Everything a kernel needs to know about the parameters, passed by value.
struct DevParams {
    int N, logN, L, ell;
    double p[kMaxL], pinv[kMaxL];
    uint64_t q[kMaxL];
    uint64_t delta[kMaxL];           // floor(q / t) mod q_l
    double n_inv[kMaxL];             // N^-1 mod q_l, balanced
    double garner_inv[kMaxL];        // (q_0 ... q_{l-1})^-1 mod q_l
    double garner_c[kMaxL][kMaxL];   // (q_0 ... q_{i-1}) mod q_l for i < l
    uint64_t Q[kMaxL + 1];           // q, little-endian 64-bit limbs
    uint64_t halfQ[kMaxL + 1];       // floor(q / 2)
    double Qd;                       // q rounded to a double
    uint64_t cdt[kCdtLen];
    const double *tw_fwd;            // [L][N] psi^bitrev(k), balanced
    const double *tw_inv;            // [L][N] psi^-bitrev(k), balanced
};

// Polynomial `poly` of a [..][L][N] buffer: its prime l = poly % L and x = poly / L
// (the ciphertext, or ciphertext and component, it belongs to).
struct PolyIx {
    int poly, l, x;
};

__device__ __forceinline__ PolyIx poly_ix(int poly, int L)
{
    const int x = poly / L;
    return PolyIx{poly, poly - x * L, x};
}

// Output ciphertext y of a plan (of a grouped plan too): y = (g*M + ib)*K + kb for
// product g, block row ib and block column kb; its share entries go to share + g*n*m.
struct OutPos {
    uint32_t g, ib, kb;
};
__host__ __device__ __forceinline__ OutPos out_pos(uint32_t y, const pimm_plan_info &f)
{
    const uint32_t rowblk = y / f.K;
    return OutPos{rowblk / f.M, rowblk % f.M, y - rowblk * f.K};
}

// 32-byte ChaCha20 key as little-endian words.
struct Key {
    uint32_t w[8];
};

// ---------------------------------------------------------------------------
// FP64 residue arithmetic
// ---------------------------------------------------------------------------

// a*b - k*p for the k nearest a*b/p: exact; for |a| <= B p, |b| <= p/2 the result
// lies within (0.5 + 0.1875 B) p of zero.
__device__ __forceinline__ double mulmod(double a, double b, double p, double pinv)
{
    const double h = a * b;
    const double l = __builtin_fma(a, b, -h);
    const double k = __builtin_rint(h * pinv);
    const double r = __builtin_fma(-k, p, h);
    return r + l;
}

// x - k*p for the k nearest x/p: |result| <= p/2 (+ a few units) for |x| < 2^52.
__device__ __forceinline__ double reduce(double x, double p, double pinv)
{
    return __builtin_fma(-__builtin_rint(x * pinv), p, x);
}

// Exact conversions between integers in [0, 2^52) and doubles through the bit
// pattern: 2^52 + v has exponent 52 and mantissa v, so setting the exponent bits
// of v (or adding 2^52 to the double) and removing 2^52 again converts with one
// floating-point and one integer operation.
__device__ __forceinline__ double f64_of(uint64_t v)
{
    return __longlong_as_double((long long)(v | 0x4330000000000000ull)) - 4503599627370496.0;
}
__device__ __forceinline__ uint64_t u64_of(double x)
{
    return (uint64_t)__double_as_longlong(x + 4503599627370496.0) - 0x4330000000000000ull;
}

// Balanced double (|x| < 2^52) -> canonical residue in [0, p): the reduction
// leaves |x| <= p/2 plus a few units, so one correction of the sign suffices.
__device__ __forceinline__ uint64_t to_canonical(double x, double p, double pinv)
{
    x = reduce(x, p, pinv);
    if (x < 0.0) x += p;
    return u64_of(x);
}

// Canonical residues: exact add/sub for values < 2^63.
__device__ __forceinline__ uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q)
{
    uint64_t s = a + b;
    return s >= q ? s - q : s;
}
__device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q)
{
    return a >= b ? a - b : a + q - b;
}
// Signed integer of magnitude below q -> canonical residue (the callers pass
// noise and ternary values, |x| <= 19).
__device__ __forceinline__ uint64_t lift_small(int64_t x, uint64_t q)
{
    return x >= 0 ? (uint64_t)x : q - (uint64_t)(-x);
}
// Canonical product through the FP64 path (a, b < 2^52).
__device__ __forceinline__ uint64_t mul_mod(uint64_t a, uint64_t b, double p, double pinv)
{
    return to_canonical(mulmod(f64_of(a), f64_of(b), p, pinv), p, pinv);
}

// n / d for n * d < 2^32 by one multiply-high: M = ceil(2^32 / d).  d = 1 (whose M would not
// fit in 32 bits) takes M = 0 and adds n through the mask `one`, so there is no branch: a branch
// in an unrolled loop of loads would make each load wait for the previous one's data.
struct FastDiv {
    uint32_t d, M, one;
    static FastDiv make(uint32_t d)
    {
        return FastDiv{d, d == 1 ? 0u : (uint32_t)(((1ull << 32) + d - 1) / d), d == 1 ? 0xffffffffu : 0u};
    }
    __device__ __forceinline__ uint32_t div(uint32_t n) const { return __umulhi(n, M) + (n & one); }
    __device__ __forceinline__ uint32_t mod(uint32_t n) const { return n - div(n) * d; }
};

// ---------------------------------------------------------------------------
// ChaCha20 block function (RFC 8439 section 2.3) and the samplers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t rotl(uint32_t v, int c) { return (v << c) | (v >> (32 - c)); }

#define PIMM_QR(a, b, c, d)                  \
    a += b; d ^= a; d = rotl(d, 16);         \
    c += d; b ^= c; b = rotl(b, 12);         \
    a += b; d ^= a; d = rotl(d, 8);          \
    c += d; b ^= c; b = rotl(b, 7);

__device__ __forceinline__ void chacha_block(const Key &k, uint32_t counter, uint32_t n0, uint32_t n1,
                                             uint32_t n2, uint32_t out[16])
{
    const uint32_t s0 = 0x61707865u, s1 = 0x3320646eu, s2 = 0x79622d32u, s3 = 0x6b206574u;
    uint32_t x0 = s0, x1 = s1, x2 = s2, x3 = s3;
    uint32_t x4 = k.w[0], x5 = k.w[1], x6 = k.w[2], x7 = k.w[3];
    uint32_t x8 = k.w[4], x9 = k.w[5], x10 = k.w[6], x11 = k.w[7];
    uint32_t x12 = counter, x13 = n0, x14 = n1, x15 = n2;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        PIMM_QR(x0, x4, x8, x12)
        PIMM_QR(x1, x5, x9, x13)
        PIMM_QR(x2, x6, x10, x14)
        PIMM_QR(x3, x7, x11, x15)
        PIMM_QR(x0, x5, x10, x15)
        PIMM_QR(x1, x6, x11, x12)
        PIMM_QR(x2, x7, x8, x13)
        PIMM_QR(x3, x4, x9, x14)
    }
    out[0] = x0 + s0; out[1] = x1 + s1; out[2] = x2 + s2; out[3] = x3 + s3;
    out[4] = x4 + k.w[0]; out[5] = x5 + k.w[1]; out[6] = x6 + k.w[2]; out[7] = x7 + k.w[3];
    out[8] = x8 + k.w[4]; out[9] = x9 + k.w[5]; out[10] = x10 + k.w[6]; out[11] = x11 + k.w[7];
    out[12] = x12 + counter; out[13] = x13 + n0; out[14] = x14 + n1; out[15] = x15 + n2;
}
#undef PIMM_QR

// Nonce word 0 of a stream.
__device__ __forceinline__ uint32_t nonce0(uint32_t tag, uint32_t prime) { return tag | (prime << 8); }
// Bit of the first nonce word that selects a stream's fallback stream (the draws
// that replace rejected uniform residues).
constexpr uint32_t kFallbackTag = 0x80000000u;

__device__ __forceinline__ int64_t ternary_of(uint64_t v) { return (int64_t)(v % 3u) - 1; }

__device__ __forceinline__ int64_t gauss_of(uint64_t v, const uint64_t *cdt)
{
    const uint64_t u = v & 0x7fffffffffffffffull;
    int64_t mag = 0;
#pragma unroll
    for (int k = 0; k < kCdtLen; ++k) mag += (u >= cdt[k]) ? 1 : 0;
    return (v >> 63) ? -mag : mag;
}

// The same value with the table in LDS, padded to 32 entries with all-ones words (above any
// 63-bit u): the count of entries <= u by a five-step binary search (the table ascends)
// instead of 19 compares.
constexpr int kCdtPad = 32;
static_assert(kCdtLen <= kCdtPad, "CDT table padding");
__device__ __forceinline__ int64_t gauss_of_lds(uint64_t v, const uint64_t *cdt32)
{
    const uint64_t u = v & 0x7fffffffffffffffull;
    int pos = 0;
#pragma unroll
    for (int step = kCdtPad / 2; step >= 1; step >>= 1) pos += (cdt32[pos + step - 1] <= u) ? step : 0;
    const int64_t mag = pos;
    return (v >> 63) ? -mag : mag;
}

__device__ __forceinline__ uint64_t mask_of(uint64_t v, int ell)
{
    return ell >= 64 ? v : (v & ((1ull << ell) - 1));
}

__device__ __forceinline__ uint64_t word64(const uint32_t b[16], int i)
{
    return (uint64_t)b[2 * i] | ((uint64_t)b[2 * i + 1] << 32);
}

// Workgroups of a launch are dispatched round-robin over the 8 XCDs (each with
// its own L2).  xcd_local maps workgroup b to a logical index such that the
// workgroups one XCD receives get one contiguous range of logical indices, so
// neighbouring work items (which share input slices) share an L2.
__device__ __forceinline__ uint32_t xcd_local(uint32_t b, uint32_t nblocks)
{
    const uint32_t xcd = b % 8, k = b / 8;
    const uint32_t per = nblocks / 8, rem = nblocks % 8;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
}

// ---------------------------------------------------------------------------
// Host-side objects
// ---------------------------------------------------------------------------

struct Ctx {
    pimm_params params;
    int device;
    DevParams dp;             // with device table pointers
    double *d_tw = nullptr;   // [2][L][N] device: forward then inverse twiddles
    uint64_t q[kMaxL];
    uint64_t psi[kMaxL];
};

struct Plan {
    Ctx *ctx = nullptr;
    pimm_plan_info info;
    // Product schedule: mac_rows = 0 selects the matrix-core product (mfma.hip);
    // otherwise the FP64 vector product with this tile.
    int mac_rows = 8;  // output rows per product thread
    int mac_cols = 1;  // output column blocks per product thread
    int waves = 1;     // product grid = waves x the workgroups the device holds at once
};

struct SecretKey {
    Ctx *ctx;
    int64_t *d_s = nullptr;   // [N] ternary coefficients
    double *d_s_hat = nullptr; // [L][N] NTT of s, balanced
};

struct Weights {
    Ctx *ctx = nullptr;
    pimm_plan_info info;        // of the plan it was made for (r, m, mb, rb, M, R, Wb matter)
    double *d_w_hat = nullptr;  // [L][N/256][M][R][256] NTT slots, balanced
    double *d_w_plain = nullptr;  // [r][m] the weights as doubles (the FC completion's product)
    void *d_w_dig = nullptr;      // digit form for the matrix-core product (mfma.h), or null
    int64_t wmax = 0;
};

// Error reporting (thread-local message).
int set_error(int code, const char *fmt, ...);
int check_hip(hipError_t e, const char *what);
Key make_key(const uint8_t seed[32]);
bool noise_ok(const Ctx &c, const pimm_plan_info &f, uint64_t wmax);
// Modulus switching of the reply (the last prime dropped): whether the switched
// reply still decrypts to the reply's value, and the parameters of the first L - 1
// primes with q_{L-1}^{-1} mod q_l (balanced) for l < L - 1.
bool switch_ok(const Ctx &c, const pimm_plan_info &f, uint64_t wmax);
void switched_params(const Ctx &c, DevParams &d, double *qd_inv);
// Decryption of a reply under the moduli of c (client.hip).
int decrypt_reply(const Ctx &c, const pimm_plan_info &f, const pimm_sk *sk, const uint64_t *c1,
                  const uint64_t *c0s, uint64_t *client_share, void *ws, size_t ws_bytes,
                  hipStream_t s, const char *who);
bool weights_fit(const Weights *w, const Plan *plan);
// PIMM_OK when the matrix-core product can run this plan on these weights.
int mfma_ready(const Plan *plan, const Weights *w, const char *who);
// FC completion (fc.hip): the weights as doubles, and whether the limb sums of
// X1 W stay exact for this shape, share width and weight bound.
int weights_plain(const int64_t *W, double *Wd, size_t n, hipStream_t s);
bool fc_exact(const pimm_plan_info &f, int ell, uint64_t wmax);

// The FC completion's cut of the inner dimension: whole granules of 64 inner rows
// per workgroup, as many pieces as keep about two workgroups per compute unit
// over the 64 x 64 output tiles.  Each piece writes its own partial sums (two
// limbs), so the workspace holds pieces * n * m * 2 doubles.
inline void fc_cut(uint32_t n, uint32_t r, uint32_t m, uint32_t *kc, uint32_t *pieces)
{
    const uint64_t tiles = (uint64_t)((m + 63) / 64) * ((n + 63) / 64);
    const uint64_t granules = (r + 63) / 64;
    uint64_t per = tiles * granules / 512;
    if (per < 1) per = 1;
    if (per > granules) per = granules;
    *kc = (uint32_t)(per * 64);
    *pieces = (uint32_t)((r + *kc - 1) / *kc);
}
uint64_t fused_workspace_bytes(const Ctx &c, const pimm_plan_info &f);
// Takes the device address of pimm_matmul_share_noalloc's static scratch on
// `device` (current at the call), once per device (noalloc.hip).
int bind_noalloc_scratch(int device);
int plan_rule(const Ctx &c, uint32_t n, uint32_t r, uint32_t m, uint32_t mb, uint32_t rb, uint32_t nb,
              uint32_t d_fix, pimm_plan_info &f);

// Brackets one kernel launch with HIP events when profiling is on.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();

  private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    bool active_ = false;
};

// Sampler kinds: 0 uniform mod q_l (uint64), 1 ternary (int64), 2 Gaussian (int64),
// 3 mask mod 2^l (uint64); the library's own scratch also takes ternary and Gaussian
// values as one signed byte each (|value| <= 19), which every kernel that reads them
// widens again.
constexpr int kSampleTernary8 = 4;
constexpr int kSampleGauss8 = 5;

// One sampling job (see k_sample): `nobj` objects x `nprime` primes of draws
// from stream (tag, prime, op, obj0 + o), written at out + o * obj_stride +
// prime_index * prime_stride.
constexpr int kMaxSampleJobs = 3;
struct SampleJob {
    int kind;
    uint32_t tag, obj0;
    int nobj, prime0, nprime;
    void *out;
    size_t obj_stride, prime_stride;
    uint32_t blocks;  // workgroups of this job (set by launch_samples)
    FastDiv pdiv;     // division by nprime (set by launch_samples)
};
struct SampleJobs {
    SampleJob job[kMaxSampleJobs];
    int n;
};
int launch_samples(const Ctx &c, const Key &key, uint32_t op, SampleJobs js, hipStream_t s);
int launch_sample(const Ctx &c, int kind, const Key &key, uint32_t tag, uint32_t op, uint32_t obj0,
                  int nobj, int prime0, int nprime, void *out, size_t obj_stride,
                  size_t prime_stride, hipStream_t s);

// Launch helpers implemented in the kernel translation units.
// Slot-wise products of one plan into zeroed-then-accumulated acc^ (mac.hip).
// The fused server step after the product (server.hip), on a workspace laid out as
// pimm_matmul_share's; pk may be NULL without re-randomisation.
// mx_layout: acc^ is in the matrix-core product's layout (acc_run_index)
// instead of [O][2][L][N].
int fused_tail(const pimm_plan *plan, const uint64_t *pk, const Key &key, uint32_t op_id,
               double *ws, uint64_t *c1, uint64_t *c0s, uint64_t *server_share, bool mx_layout,
               hipStream_t s);
// The product of one plan (acc^ zeroed first unless `zeroed` says the caller did).
int launch_mac(const Ctx &c, const pimm_plan_info &f, int G, int KB, int waves, const double *Wt,
               const double *Ct, double *Ah, bool zeroed, hipStream_t s);

}  // namespace pimm

// The C handle types are the internal objects.
struct pimm_ctx : pimm::Ctx {};
struct pimm_plan : pimm::Plan {};
struct pimm_sk : pimm::SecretKey {};
struct pimm_weights : pimm::Weights {};
