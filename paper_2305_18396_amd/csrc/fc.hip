// fc.hip -- the server's completion of a fully connected layer on additive shares
// (section 3.1, the linear layers): after Pi_MatMul on the client's share X0 the
// server holds Y1 with Y0 + Y1 = X0 W mod 2^l; it adds its own share's product
// and the bias, Y1 <- Y1 + X1 W + b (mod 2^l), so that Y0 + Y1 = X W + b.
//
// X1 W is an integer product mod 2^l.  It runs on the FP64 matrix cores, exactly: each
// entry of X1 (read mod 2^l) is split as xh 2^S + xl with S = ceil(l / 2), the
// weights are small signed integers, and both limb products are summed in
// doubles.  Every partial sum is an integer of magnitude at most
// r (2^S - 1) max|W|, which the call checks to be below 2^53, so the sums are
// exact in any order (each piece of the inner dimension writes its own partial
// sums, which the epilogue adds).
// The epilogue turns the two sums into integers and finishes mod 2^l.
#include "common.h"

namespace pimm {

namespace {

constexpr int kFcT = 64;   // output tile: 64 rows of X1 by 64 columns of W
constexpr int kFcK = 16;   // inner step held in LDS

// part[z][0][i][j] = sum_k xl[i][k] W[k][j] and part[z][1][i][j] = sum_k xh[i][k] W[k][j]
// over piece z of the inner dimension, on the FP64 matrix cores.  v_mfma_f64_16x16x4f64 takes, from lane
// l of a wave, A[l % 16][l / 16] and B[l / 16][l % 16] of a 16x4 by 4x16 product and keeps
// D[l / 16 + 4 t][l % 16] in value t of the lane's four accumulators.  Wave w of the
// workgroup owns the 32 x 32 quarter (w / 2, w % 2) of the 64 x 64 tile: two row blocks by
// two column blocks of 16, for both limbs.  The products of integers and their sums stay
// exact (all below 2^53), so the matrix cores' rounding never acts.
typedef double fc_v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_fc_gemm(const uint64_t *__restrict__ X1,
                                                 const double *__restrict__ Wd,
                                                 double *__restrict__ acc, int n, int r, int m,
                                                 int kc, int S, uint64_t xmask)
{
    __shared__ double xl[kFcK][kFcT], xh[kFcK][kFcT], wt[kFcK][kFcT];
    const int lane = (int)threadIdx.x % 64, wave = (int)threadIdx.x / 64;
    const int j0 = (int)blockIdx.x * kFcT, i0 = (int)blockIdx.y * kFcT;
    const int k0 = (int)blockIdx.z * kc;
    const int k1 = k0 + kc < r ? k0 + kc : r;
    const int rbase = (wave / 2) * 32, cbase = (wave % 2) * 32;
    const int li = lane % 16, lk = lane / 16;
    const uint64_t lmask = ((uint64_t)1 << S) - 1;
    fc_v4d dl[2][2], dh[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) dl[a][b] = dh[a][b] = fc_v4d{0.0, 0.0, 0.0, 0.0};

    for (int kk = k0; kk < k1; kk += kFcK) {
        for (int e = (int)threadIdx.x; e < kFcT * kFcK; e += 256) {
            const int i = e / kFcK, k = e % kFcK;
            const int gi = i0 + i, gk = kk + k;
            const uint64_t v = (gi < n && gk < k1) ? X1[(size_t)gi * r + gk] & xmask : 0;
            xl[k][i] = (double)(v & lmask);
            xh[k][i] = (double)(v >> S);
        }
        for (int e = (int)threadIdx.x; e < kFcK * kFcT; e += 256) {
            const int k = e / kFcT, j = e % kFcT;
            const int gk = kk + k, gj = j0 + j;
            wt[k][j] = (gk < k1 && gj < m) ? Wd[(size_t)gk * m + gj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s4 = 0; s4 < kFcK; s4 += 4) {
            const int k = s4 + lk;
            double al[2], ah[2], bw[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                al[a] = xl[k][rbase + 16 * a + li];
                ah[a] = xh[k][rbase + 16 * a + li];
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) bw[b] = wt[k][cbase + 16 * b + li];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    dl[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(al[a], bw[b], dl[a][b], 0, 0, 0);
                    dh[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ah[a], bw[b], dh[a][b], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    const size_t plane = (size_t)n * m;
    double *part = acc + (size_t)blockIdx.z * 2 * plane;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = i0 + rbase + 16 * a + lk + 4 * t, j = j0 + cbase + 16 * b + li;
                if (i < n && j < m) {
                    part[(size_t)i * m + j] = dl[a][b][t];
                    part[plane + (size_t)i * m + j] = dh[a][b][t];
                }
            }
}

// share[i][j] <- (share[i][j] + lo + hi 2^S + b[j]) mod 2^l, in uint64 wrap-around
// arithmetic (exact mod 2^l); lo and hi are the exact integer sums of the pieces.
__global__ void k_fc_finish(const double *__restrict__ acc, int pieces,
                            const int64_t *__restrict__ bias, uint64_t *__restrict__ share, int n,
                            int m, int S, uint64_t tmask)
{
    const size_t plane = (size_t)n * m;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < plane;
         idx += (size_t)gridDim.x * blockDim.x) {
        double sl = 0.0, sh = 0.0;
        for (int z = 0; z < pieces; ++z) {
            sl += acc[(size_t)z * 2 * plane + idx];
            sh += acc[(size_t)z * 2 * plane + plane + idx];
        }
        const uint64_t lo = (uint64_t)(int64_t)sl;
        const uint64_t hi = (uint64_t)(int64_t)sh;
        uint64_t v = share[idx] + lo + (hi << S);
        if (bias) v += (uint64_t)bias[idx % (size_t)m];
        share[idx] = v & tmask;
    }
}

__global__ void k_w_to_f64(const int64_t *__restrict__ W, double *__restrict__ Wd, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        Wd[i] = (double)W[i];
}

}  // namespace

int weights_plain(const int64_t *W, double *Wd, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_w_to_f64, dim3(1024), dim3(256), 0, s, W, Wd, n);
    return check_hip(hipGetLastError(), "weights copy launch");
}

// Bit split of X1's entries: S = ceil(l / 2).
static int fc_split(int ell) { return (ell + 1) / 2; }

bool fc_exact(const pimm_plan_info &f, int ell, uint64_t wmax)
{
    using u128 = unsigned __int128;
    const int S = fc_split(ell);
    const u128 bound = (u128)f.r * ((((u128)1) << S) - 1) * wmax;
    return bound < ((u128)1 << 53);
}

}  // namespace pimm

using namespace pimm;

extern "C" {

int pimm_fc_complete(const pimm_plan *plan, const pimm_weights *w, const uint64_t *x1,
                     const int64_t *bias, uint64_t *share1, void *ws, size_t ws_bytes,
                     void *stream)
{
    if (!plan || !w || !x1 || !share1) return set_error(PIMM_E_ARG, "pimm_fc_complete: NULL argument");
    if (!weights_fit(w, plan))
        return set_error(PIMM_E_ARG, "pimm_fc_complete: weights were made for another shape or block split");
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    if (f.groups > 1 || !w->d_w_plain)
        return set_error(PIMM_E_UNSUPPORTED, "pimm_fc_complete: grouped plans are not supported");
    const int ell = (int)c.params.log2_t;
    if (!fc_exact(f, ell, (uint64_t)w->wmax))
        return set_error(PIMM_E_ARG,
                         "pimm_fc_complete: r * max|W| * 2^%d reaches 2^53 (max|W| = %lld): the "
                         "limb sums would not be exact",
                         fc_split(ell), (long long)w->wmax);
    uint32_t kc = 0, pieces = 0;
    fc_cut(f.n, f.r, f.m, &kc, &pieces);
    if ((f.n + kFcT - 1) / kFcT > 65535 || pieces > 65535)
        return set_error(PIMM_E_SHAPE, "pimm_fc_complete: n = %u or r = %u too large for one launch",
                         f.n, f.r);
    const size_t need = (size_t)pieces * f.n * f.m * 2 * 8;
    if (!ws || ws_bytes < need) return set_error(PIMM_E_WORKSPACE, "pimm_fc_complete: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    int rc = check_hip(hipSetDevice(c.device), "hipSetDevice");
    if (rc) return rc;
    double *acc = (double *)ws;
    const int S = fc_split(ell);
    const uint64_t tmask = ell >= 64 ? ~0ull : (((uint64_t)1 << ell) - 1);
    ProfScope prof("fc", s);
    const dim3 grid((f.m + kFcT - 1) / kFcT, (f.n + kFcT - 1) / kFcT, pieces);
    hipLaunchKernelGGL(k_fc_gemm, grid, dim3(256), 0, s, x1, (const double *)w->d_w_plain, acc,
                       (int)f.n, (int)f.r, (int)f.m, (int)kc, S, tmask);
    hipLaunchKernelGGL(k_fc_finish, dim3(1024), dim3(256), 0, s, (const double *)acc, (int)pieces,
                       bias, share1, (int)f.n, (int)f.m, S, tmask);
    return check_hip(hipGetLastError(), "fc launch");
}

}  // extern "C"
