// The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Linked against a build of every library source whose host pass carries the
// sanitizers (tests/test_sanitizers.py), and run on a machine with or without a
// GPU: the host-only queries (parameter rule, primes, cumulative table, block
// plans, noise and switching rules) over many shapes, checked against their own
// invariants, every entry point's NULL-argument refusal, and context creation on a
// device index that does not exist.  Nothing here launches a kernel.  A sanitizer
// report or a failed check ends the run with a nonzero status; the last line is
// "ok <checks>" otherwise.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>

#include "pimm.h"

static int checks = 0;

#define CHECK(cond)                                                                 \
    do {                                                                            \
        ++checks;                                                                   \
        if (!(cond)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond, \
                         pimm_last_error());                                        \
            std::exit(1);                                                           \
        }                                                                           \
    } while (0)

static uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

static void check_plan(const pimm_params &p, uint32_t n, uint32_t r, uint32_t m, uint32_t d_fix)
{
    pimm_plan_info f;
    std::memset(&f, 0xab, sizeof f);
    const int rc = pimm_plan_rule(&p, n, r, m, 0, 0, 0, d_fix, &f);
    if (rc != PIMM_OK) {
        CHECK(rc == PIMM_E_SHAPE);
        return;
    }
    CHECK(f.n == n && f.r == r && f.m == m);
    CHECK((uint64_t)f.mb * f.rb * f.nb <= p.N);
    CHECK(f.M == ceil_div(m, f.mb) && f.R == ceil_div(r, f.rb) && f.K == ceil_div(n, f.nb));
    CHECK(f.I == f.R * f.K && f.O == f.M * f.K && f.Wb == f.M * f.R);
    CHECK(f.P == (uint64_t)f.M * f.R * f.K);
    CHECK(f.ct_bytes == (uint64_t)f.I * 2 * p.L * p.N * 8);
    CHECK(f.c1_bytes == (uint64_t)f.O * p.L * p.N * 8);
    CHECK(f.c0s_bytes == (uint64_t)f.O * p.L * f.mb * f.nb * 8);
    CHECK(f.share_bytes == (uint64_t)n * m * 8);
    if (d_fix) CHECK(f.mb * f.rb == d_fix || f.mb * f.rb <= d_fix);
    // The noise rules are monotone in the weight bound, and switching is stricter.
    const int a = pimm_noise_ok(&p, &f, 1), b = pimm_noise_ok(&p, &f, 1ull << 40);
    CHECK(a >= 0 && b >= 0 && (b <= a));
    if (p.L >= 2) {
        const int s1 = pimm_switch_ok(&p, &f, 1), s2 = pimm_switch_ok(&p, &f, 1ull << 40);
        CHECK(s1 >= 0 && s2 >= 0 && s2 <= s1 && s1 <= a);
    } else {
        CHECK(pimm_switch_ok(&p, &f, 1) == PIMM_E_UNSUPPORTED);
    }
}

int main()
{
    // Parameters: valid ones give descending primes = 1 mod 2N below 2^50; invalid ones
    // are refused.
    const uint32_t Ns[2] = {4096, 8192};
    for (uint32_t N : Ns)
        for (uint32_t L = 1; L <= 4; ++L) {
            pimm_params p{N, L, 37, 12, 50, 1};
            uint64_t q[4] = {0, 0, 0, 0};
            CHECK(pimm_params_primes(&p, q) == PIMM_OK);
            for (uint32_t l = 0; l < L; ++l) {
                CHECK(q[l] < (1ull << 50) && q[l] % (2ull * N) == 1);
                if (l) CHECK(q[l] < q[l - 1]);
            }
        }
    const pimm_params bad[] = {{1000, 2, 37, 12, 50, 1}, {2048, 2, 37, 12, 50, 1},
                               {4096, 0, 37, 12, 50, 1}, {4096, 5, 37, 12, 50, 1},
                               {4096, 2, 1, 12, 50, 1},  {4096, 2, 49, 12, 50, 1},
                               {4096, 2, 37, 12, 40, 1}};
    for (const pimm_params &p : bad) {
        uint64_t q[8];
        CHECK(pimm_params_primes(&p, q) == PIMM_E_PARAMS);
        CHECK(std::strlen(pimm_last_error()) > 0);
    }
    uint64_t cdt[19];
    CHECK(pimm_cdt(cdt) == PIMM_OK);
    for (int k = 1; k < 19; ++k) CHECK(cdt[k] > cdt[k - 1]);
    CHECK(cdt[18] < (1ull << 63));

    // Block plans over many shapes, both ring degrees, with and without a fixed area.
    const uint32_t dims[] = {1, 2, 3, 7, 16, 64, 100, 128, 300, 512, 768, 1024, 3072, 4096};
    const uint32_t areas[] = {0, 16, 64, 256, 1024, 4096};
    for (uint32_t N : Ns)
        for (uint32_t L = 1; L <= 3; ++L) {
            pimm_params p{N, L, L == 1 ? 20u : 37u, 12, 50, 1};
            for (uint32_t n : dims)
                for (uint32_t r : dims)
                    for (uint32_t m : {1u, 64u, 768u, 3072u})
                        for (uint32_t d : areas) check_plan(p, n, r, m, d);
        }
    pimm_plan_info f;
    pimm_params p{4096, 2, 37, 12, 50, 1};
    CHECK(pimm_plan_rule(&p, 0, 4, 4, 0, 0, 0, 0, &f) == PIMM_E_SHAPE);
    CHECK(pimm_plan_rule(&p, 5, 6, 7, 2, 3, 4, 0, &f) == PIMM_OK && f.M == 4 && f.R == 2 && f.K == 2);
    CHECK(pimm_plan_rule(&p, 5, 6, 7, 64, 64, 64, 0, &f) == PIMM_E_SHAPE);
    CHECK(pimm_plan_rule(nullptr, 5, 6, 7, 0, 0, 0, 0, &f) == PIMM_E_ARG);
    CHECK(pimm_noise_ok(nullptr, &f, 1) == PIMM_E_ARG);
    CHECK(pimm_switch_ok(&p, nullptr, 1) == PIMM_E_ARG);

    // NULL arguments: every entry point refuses them before touching a device.
    uint8_t seed[32] = {0};
    uint64_t word = 0;
    CHECK(pimm_ctx_create(nullptr, 0, nullptr) == PIMM_E_ARG);
    CHECK(pimm_ctx_primes(nullptr, &word) == PIMM_E_ARG);
    CHECK(pimm_ctx_cdt(nullptr, cdt) == PIMM_E_ARG);
    CHECK(pimm_plan_create(nullptr, 1, 1, 1, 0, 0, 0, 0, nullptr) == PIMM_E_ARG);
    CHECK(pimm_plan_query(nullptr, &f) == PIMM_E_ARG);
    CHECK(pimm_plan_set_tuning(nullptr, 8, 1, 1) == PIMM_E_ARG);
    CHECK(pimm_keygen(nullptr, seed, nullptr, nullptr, nullptr) == PIMM_E_ARG);
    CHECK(pimm_encode_input(nullptr, nullptr, nullptr, nullptr) == PIMM_E_ARG);
    CHECK(pimm_encrypt(nullptr, nullptr, seed, 0, nullptr, nullptr, nullptr, 0, nullptr) == PIMM_E_ARG);
    CHECK(pimm_encrypt_seeded(nullptr, nullptr, seed, seed, 0, nullptr, nullptr, nullptr, 0, nullptr) ==
          PIMM_E_ARG);
    CHECK(pimm_ct_expand(nullptr, seed, 0, nullptr, nullptr, nullptr) == PIMM_E_ARG);
    CHECK(pimm_decrypt(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == PIMM_E_ARG);
    CHECK(pimm_decrypt_switched(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
          PIMM_E_ARG);
    CHECK(pimm_weights_create(nullptr, nullptr, nullptr, nullptr) == PIMM_E_ARG);
    CHECK(pimm_weights_update(nullptr, nullptr, 1, nullptr) == PIMM_E_ARG);
    CHECK(pimm_matmul(nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == PIMM_E_ARG);
    CHECK(pimm_mask_share(nullptr, nullptr, seed, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                          nullptr) == PIMM_E_ARG);
    CHECK(pimm_matmul_share(nullptr, nullptr, nullptr, seed, 0, nullptr, nullptr, nullptr, nullptr,
                            nullptr, 0, nullptr) == PIMM_E_ARG);
    CHECK(pimm_matmul_share_noalloc(nullptr, nullptr, nullptr, seed, 0, nullptr, nullptr, nullptr,
                                    nullptr, nullptr) == PIMM_E_ARG);
    CHECK(pimm_mod_switch(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == PIMM_E_ARG);
    CHECK(pimm_fc_complete(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == PIMM_E_ARG);
    CHECK(pimm_batch_create(nullptr, 0, nullptr) == PIMM_E_ARG);
    CHECK(pimm_serve_create(nullptr, nullptr, nullptr) == PIMM_E_ARG);
    CHECK(pimm_poly_mul(nullptr, nullptr, nullptr, nullptr, 1, nullptr, 0, nullptr) == PIMM_E_ARG);
    CHECK(pimm_sample_poly(nullptr, 0, seed, 4, 0, 0, 0, nullptr, nullptr) == PIMM_E_ARG);
    CHECK(pimm_plan_select(nullptr, 1, 1, 1, nullptr, 1e9, nullptr, 0, 1, nullptr, nullptr, nullptr,
                           nullptr) == PIMM_E_ARG);
    CHECK(pimm_profile_read(nullptr, nullptr, nullptr) < 0);

    // A device index that does not exist: refused with a device error, nothing leaked into
    // the handle.
    pimm_ctx *ctx = reinterpret_cast<pimm_ctx *>(&word);
    const int rc = pimm_ctx_create(&p, 1 << 20, &ctx);
    CHECK(rc == PIMM_E_DEVICE || rc == PIMM_E_ARG);
    CHECK(std::strlen(pimm_last_error()) > 0);

    std::printf("ok %d\n", checks);
    return 0;
}
