/* pimm_probe.h -- device ceilings for the rooflines of libpimm's kernels.
 *
 * These calls are measurement tools, not part of the private-inference
 * protocol: they time small synthetic kernels on one device and return the
 * sustained rate of one resource, so that the product kernels can be compared
 * with what the device itself delivers next to its published peak (8 TB/s of
 * HBM3E, 78.6 TFLOP/s of FP64 vector arithmetic on MI355X).
 *
 * The residue arithmetic of libpimm runs on the FP64 vector unit (an exact
 * two-product and a rounded quotient per modular product); the integer probes
 * time the 64-bit Barrett and Shoup products the same work could use instead.
 *
 * Each call allocates its buffers on `device`, runs one untimed launch, then
 * `reps` timed launches on a stream of its own, frees everything and writes
 * the rate to *rate.  Errors: PIMM_E_ARG for a bad kind, size or pointer,
 * PIMM_E_OOM if the buffers do not fit, PIMM_E_DEVICE for a HIP failure.
 */
#ifndef PIMM_PROBE_H
#define PIMM_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pimm_probe_kind {
    /* Streaming read of `size` bytes (16-byte non-temporal loads, each wave over one
     * contiguous span); rate in bytes/s. */
    PIMM_PROBE_READ = 0,
    /* Copy of `size` bytes into a second buffer; rate counts read + write bytes/s. */
    PIMM_PROBE_COPY = 1,
    /* Independent FP64 fma chains, `size` fmas per lane; rate in flop/s (2 per fma). */
    PIMM_PROBE_FMA64 = 2,
    /* FP64 modular products of the library (50-bit prime), `size` per lane; rate in products/s. */
    PIMM_PROBE_MODMUL_F64 = 3,
    /* uint64 Barrett modular products, `size` per lane; rate in products/s. */
    PIMM_PROBE_MODMUL_BARRETT = 4,
    /* uint64 Shoup products by a fixed multiplier, `size` per lane; rate in products/s. */
    PIMM_PROBE_MODMUL_SHOUP = 5,
    /* As PIMM_PROBE_READ with 8-byte loads (the product's load width); bytes/s. */
    PIMM_PROBE_READ8 = 6,
};

/* Run probe `kind` on `device`.  For the three memory probes `size` is the
 * buffer size in bytes (a multiple of 16, at least 16 MiB); the rate is the
 * best over a few grid sizes.  For the arithmetic probes `size` is the chain
 * length per lane (at least 1024).  `reps` >= 1. */
int pimm_probe(int device, int kind, uint64_t size, int reps, double *rate);

#ifdef __cplusplus
}
#endif

#endif /* PIMM_PROBE_H */
