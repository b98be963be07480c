// switch.hip -- modulus switching of the reply, a wire-format variant of the
// sparse reply (section 3.1.3).
//
// The reply's noise is tiny next to q (a few dozen bits against 100 or 150), so
// the server can drop the last RNS prime before sending: every coefficient c of
// c1 and of the decoded part of c0 becomes round(c / q_{L-1}) mod q', q' the
// product of the first L - 1 primes, and each crosses the wire with L - 1
// residues instead of L.  The client decrypts with the first L - 1 primes.  In
// residues: with r the centred residue of c mod q_{L-1}, c - r is a multiple of
// q_{L-1} and (c - r) / q_{L-1} is the rounded quotient, so its residue mod q_l
// is (c_l - r) q_{L-1}^{-1} mod q_l, one exact FP64 modular product per prime.
#include "common.h"

namespace pimm {

struct SwitchArgs {
    const uint64_t *c1, *c0s;  // [O][L][N], [O][L][per]
    uint64_t *c1_out, *c0s_out;  // [O][L-1][N], [O][L-1][per]
    uint32_t O, per;
    double qd_inv[kMaxL];  // q_{L-1}^{-1} mod q_l, balanced
};

// One thread per coefficient of c1 (first O*N threads) and of the decoded c0
// (next O*per): reads its L residues, writes L - 1.  Consecutive threads take
// consecutive coefficients, so every load and store of a wave is one run.
__global__ __launch_bounds__(256) void k_mod_switch(SwitchArgs a, DevParams dp)
{
    const size_t n1 = (size_t)a.O << dp.logN;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n1 + (size_t)a.O * a.per) return;
    const int L = dp.L;
    const uint64_t *x;
    uint64_t *y;
    size_t cnt;
    if (gid < n1) {
        const size_t o = gid >> dp.logN, j = gid & (((size_t)1 << dp.logN) - 1);
        cnt = (size_t)1 << dp.logN;
        x = a.c1 + o * L * cnt + j;
        y = a.c1_out + o * (L - 1) * cnt + j;
    } else {
        const size_t g = gid - n1, o = g / a.per, j = g % a.per;
        cnt = a.per;
        x = a.c0s + o * L * cnt + j;
        y = a.c0s_out + o * (L - 1) * cnt + j;
    }
    const uint64_t qd = dp.q[L - 1];
    const uint64_t rd = x[(size_t)(L - 1) * cnt];
    const double r = rd > qd / 2 ? -(double)(qd - rd) : (double)rd;  // |r| < q_{L-1}/2
    for (int l = 0; l < L - 1; ++l) {
        // |c_l - r| < 1.5 * 2^50: exact as a double, and within the mulmod's range.
        const double v = mulmod(f64_of(x[(size_t)l * cnt]) - r, a.qd_inv[l], dp.p[l], dp.pinv[l]);
        y[(size_t)l * cnt] = to_canonical(v, dp.p[l], dp.pinv[l]);
    }
}

static bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bbytes && y < x + abytes;
}

}  // namespace pimm

using namespace pimm;

extern "C" {

int pimm_mod_switch(const pimm_plan *plan, const pimm_weights *w, const uint64_t *c1,
                    const uint64_t *c0s, uint64_t *c1_out, uint64_t *c0s_out, void *stream)
{
    if (!plan || !w || !c1 || !c0s || !c1_out || !c0s_out)
        return set_error(PIMM_E_ARG, "pimm_mod_switch: NULL argument");
    const Ctx &c = *plan->ctx;
    if (c.params.L < 2)
        return set_error(PIMM_E_UNSUPPORTED, "pimm_mod_switch: one prime cannot be dropped");
    if (!weights_fit(w, plan)) return set_error(PIMM_E_ARG, "pimm_mod_switch: weights of another plan");
    const pimm_plan_info &f = plan->info;
    if (!switch_ok(c, f, (uint64_t)w->wmax))
        return set_error(PIMM_E_NOISE,
                         "pimm_mod_switch: the switched reply's noise bound breaks decryption "
                         "(max |W| = %lld)",
                         (long long)w->wmax);
    const size_t L = c.params.L, N = c.params.N, per = (size_t)f.mb * f.nb;
    const size_t in1 = (size_t)f.O * L * N * 8, in0 = (size_t)f.O * L * per * 8;
    const size_t out1 = (size_t)f.O * (L - 1) * N * 8, out0 = (size_t)f.O * (L - 1) * per * 8;
    if (overlaps(c1_out, out1, c1, in1) || overlaps(c1_out, out1, c0s, in0) ||
        overlaps(c0s_out, out0, c1, in1) || overlaps(c0s_out, out0, c0s, in0) ||
        overlaps(c1_out, out1, c0s_out, out0))
        return set_error(PIMM_E_ARG, "pimm_mod_switch: output buffers overlap");
    SwitchArgs a;
    a.c1 = c1;
    a.c0s = c0s;
    a.c1_out = c1_out;
    a.c0s_out = c0s_out;
    a.O = f.O;
    a.per = (uint32_t)per;
    DevParams sw;  // the kernel runs on the L primes; it takes the inverses from here
    switched_params(c, sw, a.qd_inv);
    const size_t total = (size_t)f.O * (N + per);
    const int threads = 256;
    hipStream_t s = (hipStream_t)stream;
    ProfScope prof("mod_switch", s);
    hipLaunchKernelGGL(k_mod_switch, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0,
                       s, a, c.dp);
    return check_hip(hipGetLastError(), "mod_switch launch");
}

int pimm_decrypt_switched(const pimm_plan *plan, const pimm_sk *sk, const uint64_t *c1s,
                          const uint64_t *c0ss, uint64_t *client_share, void *ws, size_t ws_bytes,
                          void *stream)
{
    if (!plan || !sk || !c1s || !c0ss || !client_share)
        return set_error(PIMM_E_ARG, "pimm_decrypt_switched: NULL argument");
    if (sk->ctx != plan->ctx)
        return set_error(PIMM_E_ARG, "pimm_decrypt_switched: key of another context");
    const Ctx &c = *plan->ctx;
    if (c.params.L < 2)
        return set_error(PIMM_E_UNSUPPORTED, "pimm_decrypt_switched: one prime cannot be dropped");
    Ctx sw = c;
    double qd_inv[kMaxL];
    switched_params(c, sw.dp, qd_inv);
    sw.params.L = c.params.L - 1;
    return decrypt_reply(sw, plan->info, sk, c1s, c0ss, client_share, ws, ws_bytes,
                         (hipStream_t)stream, "pimm_decrypt_switched");
}

}  // extern "C"
