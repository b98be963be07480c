// mfma.hip -- the slot-wise products of Algorithm 1 step 3 on the matrix cores.
//
// For NTT slot z and prime l the product summed over the inner blocks,
//     acc^[ib, col](z) = sum_jb W^[ib, jb](z) c^[jb, col](z)   (mod q_l),
// is a small matrix product per slot; col runs over the K column blocks and the
// two ciphertext components (col = 2 kb + comp).  When many column blocks share
// each weight block it is bound by arithmetic, not by the weight stream, and
// the exact int8 matrix instructions of CDNA4 do it much faster than the FP64
// vector unit:
//
//   * every residue x (a balanced weight, |x| < 2^49, or a canonical input below
//     2^50) is split into seven signed 8-bit digits, x = sum_{a<7} d_a 256^a,
//     d_a in [-128, 127];
//   * sum_jb W c = sum_{d<13} 256^d T_d with T_d = sum_{a+b=d} sum_jb dW_a dc_b,
//     each T_d an exact int32 (|T_d| <= 7 * 64 * 2^14 < 2^23): the 49 digit pairs
//     are int8 matrix products (v_mfma_i32_16x16x64_i8, the inner dimension = the
//     inner blocks, at most 64, zero-padded) accumulated into 13 int32 tiles;
//   * the epilogue pairs the T_d in int32, forms three exact doubles below 2^48
//     and reduces g0 + g1 2^32 + g2 2^64 mod q_l (combine() below).
// Every step is exact, so the result is the residue the FP64 vector product
// gives; after the reduction that every consumer applies it is the same double.
//
// Digits without integer conversions: for an integer-valued double |x| < 2^51 the
// bits of x + 1.5 * 2^52 are 0x4338000000000000 + x.  Adding B - 0x4338000000000000
// with B = sum_{a<7} 128 * 256^a gives w = x + B in [0, 2^56); its bytes u_a satisfy
// x = sum_a (u_a - 128) 256^a, and u_a XOR 0x80 is the two's-complement byte of
// d_a = u_a - 128.
//
// Operand layout of the instruction (checked on the device): lane t holds row
// t % 16 of A and column t % 16 of B, with inner indices 16 (t / 16) + e in byte e
// of its 16 bytes; the 16 x 16 int32 result has row 4 (t / 16) + v, column t % 16
// in element v of lane t.
//
// Layouts:
//   digit weight cache  [L][N][7][Mt][64 lanes][16 B]   (A fragments, Mt = ceil(M/16))
//   c0, c1 (u64)        the query ciphertexts [I][2][L][N] (in evaluation form: read in
//                                                        place, 64 bytes per polynomial and
//                                                        tile)
//   acc^ (f64)          [L][N/8][O][2][8]               (read by the output transform; a
//                                                        tile's 8 slots are one run, so its
//                                                        stores cover whole 64-byte runs)
#include "common.h"
#include "mfma.h"

namespace pimm {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

constexpr uint64_t kDigitBias = 0x0080808080808080ull;    // B = sum_{a<7} 128 * 256^a
constexpr uint64_t kMagicBits = 0x4338000000000000ull;    // bits of 1.5 * 2^52
constexpr double kMagic = 6755399441055744.0;             // 1.5 * 2^52

// Seven digit bytes (two's complement) of an integer-valued double |x| < 2^51, byte a = d_a.
__device__ __forceinline__ uint64_t digits7(double x)
{
    const uint64_t bits = (uint64_t)__double_as_longlong(x + kMagic);
    return (bits + (kDigitBias - kMagicBits)) ^ kDigitBias;
}

__device__ __forceinline__ uint32_t byte_of(uint64_t w, int a) { return (uint32_t)(w >> (8 * a)) & 0xffu; }

// The dword {byte a of w0, byte a of w1, byte a of w2, byte a of w3} with three byte
// permutes (v_perm_b32 picks bytes of {src0 : src1}, src1 in bytes 0..3; selector 0x0c
// gives zero).
__device__ __forceinline__ uint32_t gather_byte(uint64_t w0, uint64_t w1, uint64_t w2, uint64_t w3,
                                                int a)
{
    const int sh = a < 4 ? 0 : 32, bb = a & 3;
    const uint32_t sel = 0x0c0c0000u | ((uint32_t)(4 + bb) << 8) | (uint32_t)bb;
    const uint32_t t01 = __builtin_amdgcn_perm((uint32_t)(w1 >> sh), (uint32_t)(w0 >> sh), sel);
    const uint32_t t23 = __builtin_amdgcn_perm((uint32_t)(w3 >> sh), (uint32_t)(w2 >> sh), sel);
    return __builtin_amdgcn_perm(t23, t01, 0x05040100u);
}

// ---- the digit weight cache -----------------------------------------------------

// One 64-lane group per (prime l, slot z, row tile it): lane t builds the A fragments
// of rows it*16 + t%16 and inner blocks 16(t/16) .. +15 for the seven digits, from the
// FP64 cache [L][N/256][M][R][256].  Entries past M or R are zero.
__global__ __launch_bounds__(256) void k_w_digits(const double *__restrict__ Wt, v4i *__restrict__ Wd,
                                                  int M, int R, int Mt, int logn, int L)
{
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t groups = ((size_t)L << logn) * Mt;
    if (gid >= groups * 64) return;
    const int lane = (int)(gid & 63);
    const size_t grp = gid >> 6;
    const int it = (int)(grp % Mt);
    const size_t lz = grp / Mt;  // l * N + z
    const int z = (int)(lz & (((size_t)1 << logn) - 1));
    const int l = (int)(lz >> logn);
    const int ib = it * 16 + (lane & 15), jb0 = 16 * (lane >> 4);
    const size_t chunks = (size_t)1 << (logn - 8);
    uint64_t w[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int jb = jb0 + e;
        w[e] = 0;
        if (ib < M && jb < R)
            w[e] = digits7(Wt[((((size_t)l * chunks + (z >> 8)) * M + ib) * R + jb) * 256 + (z & 255)]);
    }
    v4i *dst = Wd + (lz * 7 * Mt + it) * 64 + lane;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
        v4i f;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            f[k] = (int)(byte_of(w[4 * k], a) | (byte_of(w[4 * k + 1], a) << 8) |
                         (byte_of(w[4 * k + 2], a) << 16) | (byte_of(w[4 * k + 3], a) << 24));
        dst[(size_t)a * Mt * 64] = f;
    }
}

// ---- the product ----------------------------------------------------------------

struct MfmaArgs {
    const v4i *Wd;
    const uint64_t *ct;  // the query ciphertexts [I][2][L][N], in evaluation form
    double *Ah;
    int M, R, K, I, O, Mt, CT, RG, NC, logn, L;
    double c64[kMaxL];  // 2^64 mod q_l, balanced
};

// The residue sum_d 256^d T_d (mod p) of result element v, exactly:
//   P_k = T_2k + 2^8 T_2k+1 in int32 (|P_k| < 7 * 2^28 + 2^23 < 2^31);
//   g0 = P0 + 2^16 P1, g1 = P2 + 2^16 P3, g2 = P4 + 2^16 P5 + 2^32 T12 (exact doubles,
//   |g| < 2^48, since |T12| <= 64 * 8: the top digit of a balanced weight, |x| <= p/2 < 2^49,
//   is in [-2, 2] and that of an input, a canonical residue below 2^50, in [-2, 4]);
//   value = g0 + g1 2^32 + g2 2^64: the first product is a power of two, so its quotient
//   k = rint(g1 2^32 / p) leaves fma(-k, p, g1 2^32) exact; the second is a floating-point
//   modular product by 2^64 mod p; one reduction ends in [-p/2, p/2].
__device__ __forceinline__ double combine(const v4i *T, int v, double p, double pinv, double pinv32,
                                          double c64)
{
    const int P0 = T[1][v] * 256 + T[0][v], P1 = T[3][v] * 256 + T[2][v];
    const int P2 = T[5][v] * 256 + T[4][v], P3 = T[7][v] * 256 + T[6][v];
    const int P4 = T[9][v] * 256 + T[8][v], P5 = T[11][v] * 256 + T[10][v];
    const double g0 = __builtin_fma((double)P1, 65536.0, (double)P0);
    const double g1 = __builtin_fma((double)P3, 65536.0, (double)P2);
    const double g2 = __builtin_fma((double)T[12][v], 4294967296.0,
                                    __builtin_fma((double)P5, 65536.0, (double)P4));
    const double k1 = __builtin_rint(g1 * pinv32);
    const double r1 = __builtin_fma(-k1, p, g1 * 4294967296.0);
    return reduce(g0 + r1 + mulmod(g2, c64, p, pinv), p, pinv);
}

constexpr int kMfmaSlots = 8;    // slots per workgroup (half a 16-slot chunk)
constexpr int kMfmaParts = 16 / kMfmaSlots;  // workgroups per 16-slot chunk
constexpr int kMfmaThreads = 256;  // 4 waves, one 16-row tile each
constexpr int kSlotLds = 512;      // v4i per slot region (8 KiB)
constexpr int kMfmaPerCu = 16 / kMfmaSlots;  // workgroups per compute unit (128 KiB of LDS)

// Workgroup: prime l, slots zc*16 + h*8 .. +7, column tile ct (16 columns), row tiles
// rg*4 .. rg*4+3 (one per wave).  LDS holds one 8 KiB region per slot: first the slot's
// B fragments ([digit][column][4 x 16 B], the 16-byte groups of column j rotated by
// (j / 4) % 4 so that the 16 lanes of a group hit distinct banks), then, once every wave
// has issued its products for the slot, the slot's results ([wave][row v][lane] doubles),
// which the wave finally writes out with lanes remapped so that each row's 16 columns x
// 8 slots go out as one contiguous 1 KiB run of the accumulator runs (acc_run_index).
// The inputs come as 64-byte pieces: whole runs of c0^ and 8 consecutive slots of each
// c1 polynomial, read in place from the ciphertexts (each a different polynomial, so the
// piece size sets how well those reads use DRAM: with 4 slots per workgroup (32 KiB, four
// per CU) the product was 9% slower).  64 KiB of LDS: two workgroups share a compute unit.
// Logical index (from xcd_local, so that the halves and the column tiles of a chunk run
// side by side on one XCD and share its L2)
//     lb = (((l * NC + zc) * RG + rg) * CT + ct) * 2 + h.
__global__ __launch_bounds__(kMfmaThreads, kMfmaPerCu) void k_mac_mfma(MfmaArgs g, DevParams dp)
{
    __shared__ v4i lds[kMfmaSlots * kSlotLds];
    uint32_t lb = xcd_local(blockIdx.x, gridDim.x);
    const int h = (int)(lb % kMfmaParts);
    lb /= kMfmaParts;
    const int ct = (int)(lb % g.CT);
    lb /= g.CT;
    const int rg = (int)(lb % g.RG);
    lb /= g.RG;
    const int zc = (int)(lb % g.NC);
    const int l = (int)(lb / g.NC);
    const int tid = (int)threadIdx.x;
    const int zt = zc * 16 + h * kMfmaSlots;  // the tile's first slot

    // Inputs: thread (q, j) takes inner blocks 4q .. 4q+3 of column j for the workgroup's slots.  All
    // loads are issued before any is used (absent blocks read a valid line and are zeroed
    // afterwards), so their latencies overlap.  The first half of the slots is split into
    // digits and its products start while the second half's loads are still arriving; the
    // second half goes to LDS before slot kMfmaSlots / 2.
    // Column (kb, c) reads component c of the query ciphertexts in place (canonical residues
    // in slot order).
    const int jq = tid & 15, qq = tid >> 4;
    const int colq = ct * 16 + jq, kbq = colq >> 1, compq = colq & 1;
    u64x2 v[4][kMfmaSlots / 2];
    bool ok[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int jb = 4 * qq + r;
        ok[r] = jb < g.R && kbq < g.K;
        const size_t x = (size_t)jb * g.K + kbq;
        const uint64_t *src = !ok[r] ? g.ct : g.ct + ((((x * 2 + compq) * g.L + l) << g.logn) + zt);
#pragma unroll
        for (int s2 = 0; s2 < kMfmaSlots / 2; ++s2) v[r][s2] = ((const u64x2 *)src)[s2];
    }
    uint32_t *ld32 = (uint32_t *)lds;
    const int grpq = (qq >> 2) ^ ((jq >> 2) & 3);
    auto to_lds = [&](int s) {
        uint64_t w[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint64_t b = (s & 1) ? v[r][s >> 1].y : v[r][s >> 1].x;
            w[r] = ok[r] ? digits7(f64_of(b)) : 0;
        }
#pragma unroll
        for (int b = 0; b < 7; ++b)
            ld32[s * kSlotLds * 4 + (b * 16 + jq) * 16 + grpq * 4 + (qq & 3)] =
                gather_byte(w[0], w[1], w[2], w[3], b);
    };
#pragma unroll
    for (int s = 0; s < kMfmaSlots / 2; ++s) to_lds(s);
    __syncthreads();

    const int wv = tid >> 6, lane = tid & 63;
    const int it = rg * 4 + wv;
    const bool active = it < g.Mt;  // whole waves; idle waves still meet every barrier
    const int jl = lane & 15, gq = lane >> 4;
    const double p = dp.p[l], pinv = dp.pinv[l];
    const double pinv32 = 4294967296.0 * pinv, c64 = g.c64[l];
    const size_t fstride = (size_t)g.Mt * 64;  // v4i between the digits of one slot
    const size_t sstride = 7 * fstride;        // v4i between consecutive slots
    const int bgrp = gq ^ ((jl >> 2) & 3);
    const size_t z0 = (size_t)zc * 16 + h * kMfmaSlots;
    // Weight fragment x of slot s + 1 is requested as soon as the 7 products that use
    // fragment x of slot s are issued, so its latency hides behind the rest of the slot.
    // Plain (cached) loads: the workgroups of the other column tiles of the chunk read the
    // same fragments from the XCD's L2.
    const v4i *wbase = g.Wd + ((((size_t)l << g.logn) + z0) * 7 * g.Mt + (active ? it : 0)) * 64 + lane;
    v4i A[7];
    if (active) {
#pragma unroll
        for (int d = 0; d < 7; ++d) A[d] = wbase[d * fstride];
    }
#pragma unroll
    for (int s = 0; s < kMfmaSlots; ++s) {
        if (s == kMfmaSlots / 2) {
            // Second half of the slots: their regions are untouched by the first half's results.
#pragma unroll
            for (int s1 = kMfmaSlots / 2; s1 < kMfmaSlots; ++s1) to_lds(s1);
            __syncthreads();
        }
        v4i T[13];
        if (active) {
            v4i B[7];
#pragma unroll
            for (int d = 0; d < 7; ++d) B[d] = lds[s * kSlotLds + (d * 16 + jl) * 4 + bgrp];
#pragma unroll
            for (int d = 0; d < 13; ++d) T[d] = v4i{0, 0, 0, 0};
#pragma unroll
            for (int x = 0; x < 7; ++x) {
#pragma unroll
                for (int y = 0; y < 7; ++y)
                    T[x + y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[x], B[y], T[x + y], 0, 0, 0);
                if (s + 1 < kMfmaSlots) A[x] = wbase[(s + 1) * sstride + x * fstride];
            }
        }
        __syncthreads();  // every wave has read slot s's fragments: its region takes results
        if (active) {
            double *st = (double *)(lds + s * kSlotLds) + (size_t)wv * 4 * 64 + lane;
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) st[vv * 64] = combine(T, vv, p, pinv, pinv32, c64);
        }
    }
    if (!active) return;
    // Lane k of a store instruction writes 2 slots (16 bytes) of one (row, column): the 8 S
    // lanes of a row cover its 16 columns x S slots as one contiguous run, and an
    // instruction covers 8 / S rows.
    constexpr int LPR = 8 * kMfmaSlots, RPI = 64 / LPR, HALF = kMfmaSlots / 2;
    static_assert(kAccRun % kMfmaSlots == 0 && 16 % kAccRun == 0 && 64 % LPR == 0, "output runs");
    const int kk = lane % LPR, sp = kk % HALF, cl = kk / HALF;
    const int colg = ct * 16 + cl, kb = colg >> 1, comp = colg & 1;
    const double *res = (const double *)lds + (size_t)wv * 4 * 64 + cl;
    // Run of the tile's slots and their offset in it.
    const size_t zr = ((size_t)l * g.NC + zc) * (16 / kAccRun) + (h * kMfmaSlots) / kAccRun;
    const int zoff = (h * kMfmaSlots) % kAccRun;
#pragma unroll
    for (int i = 0; i < 16 / RPI; ++i) {
        const int row = RPI * i + lane / LPR;  // = 4 gq + vv of the results
        const int ib = it * 16 + row;
        if (ib >= g.M || kb >= g.K) continue;
        const double *src = res + (row >> 2) * 16 + (row & 3) * 64;
        double2 *dst = (double2 *)(g.Ah +
            ((zr * g.O + (size_t)ib * g.K + kb) * 2 + comp) * kAccRun + zoff + 2 * sp);
        *dst = double2{src[(2 * sp) * kSlotLds * 2], src[(2 * sp + 1) * kSlotLds * 2]};
    }
}

// ---- host side ------------------------------------------------------------------

static double balanced_pow2(uint64_t q, int e)
{
    unsigned __int128 r = 1;
    for (int i = 0; i < e; ++i) r = (r * 2) % q;
    const uint64_t v = (uint64_t)r;
    return v > q / 2 ? -(double)(q - v) : (double)v;
}

bool mfma_eligible(const pimm_plan_info &f) { return f.R <= 64 && f.K >= 8 && f.groups <= 1; }

uint64_t digit_cache_bytes(const Ctx &c, const pimm_plan_info &f)
{
    const uint64_t Mt = (f.M + 15) / 16;
    return (uint64_t)c.params.L * c.params.N * 7 * Mt * 1024;
}

int build_weight_digits(const Ctx &c, const pimm_plan_info &f, const double *Wt, void *Wd,
                        hipStream_t s)
{
    const int Mt = (int)((f.M + 15) / 16);
    const size_t threads = (size_t)c.params.L * c.params.N * Mt * 64;
    hipLaunchKernelGGL(k_w_digits, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, Wt,
                       (v4i *)Wd, (int)f.M, (int)f.R, Mt, c.dp.logN, (int)c.params.L);
    return check_hip(hipGetLastError(), "weight digits launch");
}

int launch_mac_mfma(const Ctx &c, const pimm_plan_info &f, const void *Wd, const uint64_t *ct, double *Ah,
                    hipStream_t s)
{
    if (!mfma_eligible(f))
        return set_error(PIMM_E_UNSUPPORTED,
                         "matrix-core product needs at most 64 inner blocks and 8 column blocks "
                         "(plan has R = %u, K = %u)", f.R, f.K);
    MfmaArgs g{};
    g.Wd = (const v4i *)Wd;
    g.ct = ct;
    g.L = (int)c.params.L;
    g.Ah = Ah;
    g.M = (int)f.M;
    g.R = (int)f.R;
    g.K = (int)f.K;
    g.I = (int)f.I;
    g.O = (int)f.O;
    g.Mt = (int)((f.M + 15) / 16);
    g.CT = (int)((2 * f.K + 15) / 16);
    g.RG = (g.Mt + 3) / 4;
    g.NC = (int)(c.params.N / 16);
    g.logn = c.dp.logN;
    for (uint32_t l = 0; l < c.params.L; ++l) g.c64[l] = balanced_pow2(c.q[l], 64);
    const uint64_t blocks = (uint64_t)c.params.L * g.NC * g.RG * g.CT * kMfmaParts;
    if (blocks > 0x7fffffffull) return set_error(PIMM_E_SHAPE, "matrix-core product grid too large");
    ProfScope prof("mac", s);
    hipLaunchKernelGGL(k_mac_mfma, dim3((unsigned)blocks), dim3(kMfmaThreads), 0, s, g, c.dp);
    return check_hip(hipGetLastError(), "matrix-core product launch");
}

}  // namespace pimm
