// server.hip -- the server's side of Pi_MatMul (Algorithm 1 steps 1 and 3 and
// the sparse reply of section 3.1.3).
//
// The product [[c]] = a [[b]] of step 3, accumulated over the inner blocks, is
// for every NTT slot z and prime l a small modular matrix product
//     acc^[ib, kb](z) = sum_jb  W^[ib, jb](z) * c^[jb, kb](z),
// done for both ciphertext components.  The weight transforms W^ are computed
// once per weight matrix and kept in HBM (the weights are static), so the
// per-call work is: forward NTT of the I input ciphertexts, the slot-wise
// products (which stream W^ once: 8 bytes per two modular MACs when each
// weight block meets one input column block), and the inverse NTT of the O
// accumulators.
#include <string.h>

#include "common.h"
#include "mac.h"
#include "ntt.h"

namespace pimm {

int launch_sample(const Ctx &c, int kind, const Key &key, uint32_t tag, uint32_t op, uint32_t obj0,
                  int nobj, int prime0, int nprime, void *out, size_t obj_stride,
                  size_t prime_stride, hipStream_t s);

// ---- weights (Algorithm 1 step 1, pi_A) ---------------------------------------------

// Coefficient j of block w = ib*R + jb of pi_A(W^T), read straight from W [r][m]:
// j = i*rb + rb - 1 - jj holds W[jb*rb + jj][ib*mb + i]; j >= mb*rb is zero.
struct LoadWeights {
    const int64_t *W;
    uint32_t r, m, mb, rb, R;
    int L;
    __device__ double operator()(int poly, int, int j, double, double) const
    {
        const uint32_t uj = (uint32_t)j;
        if (uj >= mb * rb) return 0.0;
        const uint32_t w = (uint32_t)(poly / L);
        const uint32_t ib = w / R, jb = w % R;
        const uint32_t i = uj / rb, jj = rb - 1 - uj % rb;
        const uint32_t row = jb * rb + jj, col = ib * mb + i;
        if (row >= r || col >= m) return 0.0;
        return (double)W[(size_t)row * m + col];
    }
};

__global__ void k_absmax(const int64_t *W, size_t n, unsigned long long *out)
{
    unsigned long long best = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int64_t v = W[i];
        const unsigned long long a = v < 0 ? (unsigned long long)(-(v + 1)) + 1 : (unsigned long long)v;
        best = a > best ? a : best;
    }
    atomicMax(out, best);
}

// ---- the slot-wise products (step 3) -----------------------------------------

// Grid: x = (N / 256) slot chunks times L primes, y = ceil(M / G) row tiles,
// z = K column blocks times S splits of the inner dimension.  Split s covers
// inner blocks [s R / S, (s+1) R / S) and writes partial accumulators at
// Ah + s * O * 2 * L * N.
template <int G>
__global__ __launch_bounds__(256) void k_mac(const double *__restrict__ Wh,
                                             const double *__restrict__ Ch, double *__restrict__ Ah,
                                             int M, int R, int K, int S, DevParams dp)
{
    const int chunks = dp.N >> 8;
    const int l = blockIdx.x / chunks;
    const int z = ((blockIdx.x % chunks) << 8) + threadIdx.x;
    const int kb = (int)blockIdx.z % K, sp = (int)blockIdx.z / K;
    const int jb0 = (int)((int64_t)R * sp / S), jb1 = (int)((int64_t)R * (sp + 1) / S);
    const size_t part = (size_t)M * K * 2 * dp.L * dp.N;
    mac_tile<G>(Wh, Ch, Ah + sp * part, M, R, K, dp, l, z, (int)blockIdx.y * G, kb, jb0, jb1);
}

int launch_mac(const Ctx &c, const pimm_plan_info &f, int G, int S, const double *Wh,
               const double *Ch, double *Ah, hipStream_t s)
{
    const unsigned gx = (unsigned)((c.params.N >> 8) * c.params.L);
    const unsigned gz = (unsigned)(f.K * S);
    ProfScope prof("mac", s);
    switch (G) {
    case 4:
        hipLaunchKernelGGL(k_mac<4>, dim3(gx, (f.M + 3) / 4, gz), dim3(256), 0, s, Wh, Ch, Ah,
                           (int)f.M, (int)f.R, (int)f.K, S, c.dp);
        break;
    case 16:
        hipLaunchKernelGGL(k_mac<16>, dim3(gx, (f.M + 15) / 16, gz), dim3(256), 0, s, Wh, Ch, Ah,
                           (int)f.M, (int)f.R, (int)f.K, S, c.dp);
        break;
    default:
        hipLaunchKernelGGL(k_mac<8>, dim3(gx, (f.M + 7) / 8, gz), dim3(256), 0, s, Wh, Ch, Ah,
                           (int)f.M, (int)f.R, (int)f.K, S, c.dp);
        break;
    }
    return check_hip(hipGetLastError(), "mac launch");
}

// Sum of S partial accumulators [S][O*2*L][N] of one polynomial.
struct LoadSlotsSum {
    const double *a;
    size_t part;  // doubles between partials
    int logn, S;
    __device__ double operator()(int poly, int, int z, double p, double pinv) const
    {
        const double *q = a + ((size_t)poly << logn) + z;
        double v = q[0];
        for (int k = 1; k < S; ++k) v += q[k * part];
        return reduce(v, p, pinv);
    }
};

// ---- re-randomisation, mask and extraction --------------------------------------

// Pointwise u^[o][l] * pk^[comp][l] for polynomials [O][2][L].
struct LoadRerand {
    const double *uh;   // [O][L][N]
    const double *pkh;  // [2][L][N]
    int logn, L;
    __device__ double operator()(int poly, int l, int z, double p, double pinv) const
    {
        const size_t o = (size_t)(poly / (2 * L));
        const size_t comp = (size_t)((poly / L) % 2);
        return mulmod(uh[((o * L + l) << logn) + z], pkh[((comp * L + l) << logn) + z], p, pinv);
    }
};

// acc[o][comp][l][j] += (u pk_comp)_j + e_comp[j]  (mod q_l); e: [O][2][N].
struct StoreAddErr {
    uint64_t *acc;
    const int64_t *e;
    int logn, L;
    __device__ void operator()(int poly, int l, int j, double v, double p, double pinv) const
    {
        const uint64_t q = (uint64_t)p;
        const size_t at = ((size_t)poly << logn) + j;
        const uint64_t up = to_canonical(v, p, pinv);
        const uint64_t ee = lift_signed(e[((size_t)(poly / L) << logn) + j], q);
        acc[at] = add_mod(add_mod(acc[at], up, q), ee, q);
    }
};

// One thread per decoded coefficient of each output ciphertext y:
// s = mask draw number pos of stream (MASK, 0, op, y);
// c0s[y][l][k*mb + i] = [acc0[pos] - Delta_l s]_{q_l}; server share = s.
__global__ void k_mask_extract(Key key, uint32_t op, const uint64_t *acc, uint64_t *c0s,
                               uint64_t *share, pimm_plan_info f, DevParams dp)
{
    const uint32_t per = f.mb * f.nb;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)f.O * per) return;
    const uint32_t y = (uint32_t)(gid / per), idx = (uint32_t)(gid % per);
    const uint32_t k = idx / f.mb, i = idx % f.mb;
    const uint32_t pos = k * f.mb * f.rb + i * f.rb + f.rb - 1;
    uint32_t w[16];
    chacha_block(key, pos / 8, nonce0(kTagMask, 0), op, y, w);
    const uint64_t sm = mask_of(word64(w, (int)(pos % 8)), dp.ell);
    const size_t N = (size_t)dp.N, L = (size_t)dp.L;
    for (int l = 0; l < dp.L; ++l) {
        const uint64_t q = dp.q[l];
        const uint64_t a0 = acc[(((size_t)y * 2 + 0) * L + l) * N + pos];
        c0s[((size_t)y * L + l) * per + idx] = sub_mod(a0, mul_mod(dp.delta[l], sm, dp.p[l], dp.pinv[l]), q);
    }
    const uint32_t ib = y / f.K, kb = y % f.K;
    const uint32_t row = kb * f.nb + k, col = ib * f.mb + i;
    if (row < f.n && col < f.m) share[(size_t)row * f.m + col] = sm;
}

}  // namespace pimm

using namespace pimm;

namespace pimm {
// A weight cache holds pi_A blocks in NTT form; it serves every plan with the
// same context, matrix shape (r, m) and block split (mb, rb), whatever n and nb.
bool weights_fit(const Weights *w, const Plan *plan)
{
    const pimm_plan_info &a = w->info, &b = plan->info;
    return w->ctx == plan->ctx && a.r == b.r && a.m == b.m && a.mb == b.mb && a.rb == b.rb;
}
}  // namespace pimm

extern "C" {

int pimm_weights_create(const pimm_plan *plan, const int64_t *W, pimm_weights **out, void *stream)
{
    if (!plan || !W || !out) return set_error(PIMM_E_ARG, "pimm_weights_create: NULL argument");
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    hipStream_t s = (hipStream_t)stream;
    int rc = check_hip(hipSetDevice(c.device), "hipSetDevice");
    if (rc) return rc;
    unsigned long long *d_max = nullptr, h_max = 0;
    rc = check_hip(hipMalloc((void **)&d_max, sizeof *d_max), "hipMalloc absmax");
    if (rc) return rc;
    rc = check_hip(hipMemsetAsync(d_max, 0, sizeof *d_max, s), "memset absmax");
    if (!rc) {
        hipLaunchKernelGGL(k_absmax, dim3(1024), dim3(256), 0, s, W, (size_t)f.r * f.m, d_max);
        rc = check_hip(hipGetLastError(), "absmax launch");
    }
    if (!rc) rc = check_hip(hipMemcpyAsync(&h_max, d_max, sizeof h_max, hipMemcpyDeviceToHost, s),
                            "copy absmax");
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "absmax synchronize");
    (void)hipFree(d_max);
    if (rc) return rc;
    if (!noise_ok(c, f, h_max))
        return set_error(PIMM_E_NOISE,
                         "max |W| = %llu: worst-case noise of the reply breaks decryption for "
                         "these parameters and this plan",
                         h_max);
    pimm_weights *w = new pimm_weights();
    w->ctx = plan->ctx;
    w->info = plan->info;
    w->wmax = (int64_t)h_max;
    rc = check_hip(hipMalloc((void **)&w->d_w_hat, f.weights_bytes), "hipMalloc weights");
    if (!rc)
        rc = launch_fwd(c, LoadWeights{W, f.r, f.m, f.mb, f.rb, f.R, (int)c.params.L},
                        StoreSlots{w->d_w_hat, c.dp.logN}, (int)(f.Wb * c.params.L), s);
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "weights synchronize");
    if (rc) {
        pimm_weights_destroy(w);
        return rc;
    }
    *out = w;
    return PIMM_OK;
}

int pimm_weights_destroy(pimm_weights *w)
{
    if (!w) return PIMM_OK;
    if (w->d_w_hat) (void)hipFree(w->d_w_hat);
    delete w;
    return PIMM_OK;
}

// Workspace: c^ [I][2][L][N] doubles, then acc^ [O][2][L][N] doubles.
int pimm_matmul(const pimm_plan *plan, const pimm_weights *w, const uint64_t *ct, uint64_t *acc,
                void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !w || !ct || !acc) return set_error(PIMM_E_ARG, "pimm_matmul: NULL argument");
    if (!weights_fit(w, plan))
        return set_error(PIMM_E_ARG, "pimm_matmul: weights were made for another shape or block split");
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    const size_t N = c.params.N, L = c.params.L;
    const size_t need = ((size_t)f.I + (size_t)plan->splits * f.O) * 2 * L * N * 8;
    if (!ws || ws_bytes < need) return set_error(PIMM_E_WORKSPACE, "pimm_matmul: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int lg = c.dp.logN;
    double *ch = (double *)ws;
    double *ah = ch + (size_t)f.I * 2 * L * N;
    const int G = plan->mac_rows, S = plan->splits;
    int rc = launch_fwd(c, LoadU64{ct, lg}, StoreSlots{ch, lg}, (int)(f.I * 2 * L), s);
    if (!rc) rc = launch_mac(c, f, G, S, w->d_w_hat, ch, ah, s);
    if (!rc) {
        if (S == 1)
            rc = launch_inv(c, LoadSlots{ah, lg}, StoreU64{acc, lg}, (int)(f.O * 2 * L), s);
        else
            rc = launch_inv(c, LoadSlotsSum{ah, (size_t)f.O * 2 * L * N, lg, S}, StoreU64{acc, lg},
                            (int)(f.O * 2 * L), s);
    }
    return rc;
}

// Workspace (re-randomisation on): pk^ [2][L][N] doubles, u^ [O][L][N] doubles,
// u [O][N] int64, e [O][2][N] int64.
int pimm_mask_share(const pimm_plan *plan, const uint64_t *pk, const uint8_t seed[32],
                    uint32_t op_id, uint64_t *acc, uint64_t *c1, uint64_t *c0s,
                    uint64_t *server_share, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !seed || !acc || !c1 || !c0s || !server_share)
        return set_error(PIMM_E_ARG, "pimm_mask_share: NULL argument");
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    const size_t N = c.params.N, L = c.params.L;
    hipStream_t s = (hipStream_t)stream;
    const int lg = c.dp.logN;
    const Key key = make_key(seed);
    int rc = PIMM_OK;
    if (c.params.rerandomize) {
        if (!pk) return set_error(PIMM_E_ARG, "pimm_mask_share: re-randomisation needs pk");
        const size_t need = 2 * L * N * 8 + (size_t)f.O * L * N * 8 + (size_t)f.O * 3 * N * 8;
        if (!ws || ws_bytes < need)
            return set_error(PIMM_E_WORKSPACE, "pimm_mask_share: workspace too small");
        double *pkh = (double *)ws;
        double *uh = pkh + 2 * L * N;
        int64_t *u = (int64_t *)(uh + (size_t)f.O * L * N);
        int64_t *e = u + (size_t)f.O * N;
        rc = launch_fwd(c, LoadU64{pk, lg}, StoreSlots{pkh, lg}, (int)(2 * L), s);
        if (!rc) rc = launch_sample(c, 1, key, kTagRrU, op_id, 0, (int)f.O, 0, 1, u, N, 0, s);
        if (!rc) rc = launch_sample(c, 2, key, kTagRrE1, op_id, 0, (int)f.O, 0, 1, e, 2 * N, 0, s);
        if (!rc) rc = launch_sample(c, 2, key, kTagRrE2, op_id, 0, (int)f.O, 0, 1, e + N, 2 * N, 0, s);
        if (!rc)
            rc = launch_fwd(c, LoadI64Shared{u, lg, (int)L}, StoreSlots{uh, lg}, (int)(f.O * L), s);
        if (!rc)
            rc = launch_inv(c, LoadRerand{uh, pkh, lg, (int)L}, StoreAddErr{acc, e, lg, (int)L},
                            (int)(f.O * 2 * L), s);
    }
    if (!rc) {
        const size_t total = (size_t)f.O * f.mb * f.nb;
        const int threads = 256;
        ProfScope prof("mask_extract", s);
        hipLaunchKernelGGL(k_mask_extract, dim3((unsigned)((total + threads - 1) / threads)),
                           dim3(threads), 0, s, key, op_id, acc, c0s, server_share, f, c.dp);
        rc = check_hip(hipGetLastError(), "mask_extract launch");
    }
    if (!rc)
        rc = check_hip(hipMemcpy2DAsync(c1, L * N * 8, acc + L * N, 2 * L * N * 8, L * N * 8, f.O,
                                        hipMemcpyDeviceToDevice, s),
                       "copy c1");
    return rc;
}

}  // extern "C"
