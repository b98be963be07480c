// cdt.cpp -- cumulative table of the encryption-error sampler, in quad precision.
//
// The error distribution is the discrete Gaussian of width sigma = 3.2 cut at
// |e| <= 19: rho(x) = exp(-x^2 / (2 sigma^2)) = exp(-25 x^2 / 512), which is
// exact as a rational exponent because 2 sigma^2 = 512/25.  The table entry
// T[k] = floor(2^63 P(|e| <= k)), k = 0 .. 18; a sample takes u = 63 random
// bits and sets |e| = #{k : u >= T[k]}.  Computed once per context with
// 113-bit floats; the floor is exact unless 2^63 P(|e| <= k) lies within
// about 2^-45 of an integer, which it does not for this width.
#include <quadmath.h>
#include <stdint.h>

extern "C" __attribute__((visibility("hidden"))) int pimm_host_cdt(int len, uint64_t *out)
{
    if (len <= 0 || len > 64) return -1;
    __float128 rho[65];
    for (int x = 0; x <= len; ++x) rho[x] = expq(-((__float128)(25 * x * x)) / 512);
    __float128 total = rho[0];
    for (int x = 1; x <= len; ++x) total += 2 * rho[x];
    __float128 acc = rho[0];
    const __float128 two63 = ldexpq((__float128)1, 63);
    for (int k = 0; k < len; ++k) {
        __float128 v = floorq(acc / total * two63);
        out[k] = (uint64_t)v;
        acc += 2 * rho[k + 1];
    }
    return 0;
}
