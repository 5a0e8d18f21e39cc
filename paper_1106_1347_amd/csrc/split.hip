// FP64 product from exact low-precision digit products ("split" method).
//
// Not a method of the paper; it reuses WinogradScaled's infinity-norm
// scaling (Section 2.3.2) and computes the same result as the CPU model of
// the oracle, bit for bit:
//   1. lambda from NormInf(A), NormInf(B) (optional); A' = 2^l A, B' = 2^-l B.
//   2. e_i = E(max_k |A'_ik|) + 1 per row of A', f_j likewise per column of
//      B' (E = frexp exponent), so every scaled entry lies in [-1/2, 1/2].
//   3. s signed digits of beta bits per entry by repeated round-to-nearest:
//      d_t = rint(2^beta r_{t-1}), r_t = 2^beta r_{t-1} - d_t, |d_t| <= 2^(beta-1).
//   4. For g = 2..s+1: G_g = sum_{t+u=g} D_A^(t) D_B^(u), an exact integer
//      matrix formed on the matrix cores (digits are exact in bf16/fp16/int8;
//      products and partial sums stay below the accumulator's exact range
//      and are flushed to FP64 before they could exceed it, each group at
//      the interval its own number of pairs allows).
//   5. The groups, from the finest scale (g = s+1) down, are merged into
//      runs of L consecutive groups; a run with finest group f holds the
//      exact integer T = sum_{g in run} G_g 2^(beta (f - g)) (L is the
//      largest of 3, 2, 1 whose worst-case run sums stay within 2^53, so T
//      is exact in FP64).  c = 0; run by run from the finest,
//      c = c + 2^(-beta f) T (one rounding per run); C_ij = 2^(e_i + f_j) c.
//
// Digit types: BF16 (default beta = 8, at most 9: |d| <= 256 has 8
// significant bits), FP16 (default and at most 9), both with FP32
// accumulation on the 16x16x32 MFMA; INT8 (default 7: |d| <= 64 fits a
// signed byte; INT32 accumulation, 16x16x64 MFMA).  INT8 with beta = 8
// takes byte digits instead of step 3 (see cut): e_i one larger, the
// scaled entry rounded once to 8 s bits and written in base 256 with
// digits in [-128, 127]; steps 4 and 5 are unchanged.
//
// Layouts (workspace): K is padded to a multiple of 64 entries and cut into
// blocks of 64 bytes (64 int8 or 32 bf16/fp16 digits: one MFMA step of
// every digit type).  Digits of A are stored as SA[kb][t][i][64 bytes] and
// digits of B transposed as SB[kb][u][j][64 bytes] (kb = K block, t/u =
// digit), so the 16 rows x 64 bytes one MFMA operand block needs are one
// contiguous KiB; rows are padded with zeros to the tile sizes, so the
// GEMM's loads need no bounds checks.
#include <string.h>

#include <type_traits>

#include "batch.h"
#include "launch.h"
#include "reduce.h"
#include "split.h"

namespace mmm {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int KT = 64;  // K padding (entries)
constexpr int KB = 64;  // bytes of K per MFMA step and per digit block

enum DType { DT_BF16 = 0, DT_FP16 = 1, DT_INT8 = 2 };

template <int DT>
struct Digit;
template <>
struct Digit<DT_BF16> {
    static constexpr int esize = 2, mfma_k = 32;
    static constexpr double budget = 16777216.0;  // 2^24: exact FP32 integers
};
template <>
struct Digit<DT_FP16> {
    static constexpr int esize = 2, mfma_k = 32;
    static constexpr double budget = 16777216.0;
};
template <>
struct Digit<DT_INT8> {
    static constexpr int esize = 1, mfma_k = 64;
    static constexpr double budget = 2147483647.0;  // int32
};

// Workgroup tile: nw waves side by side along N, each owning wbm blocks of
// 16 rows and one block of 16 columns, so BM = 16 wbm and BN = 16 nw; minw
// waves per SIMD; `stages` K blocks in flight (LDS stages of A, register
// sets of B).  Sized so that the group accumulators (s per output), when
// flushing the 2 s FP64 registers per output, and the B digit fragments
// fit the register share of minw waves without spills.
#ifndef MMM_SPLIT_WBM
#define MMM_SPLIT_WBM 4
#endif
#ifndef MMM_SPLIT_MINW
#define MMM_SPLIT_MINW 2
#endif
#ifndef MMM_SPLIT_NW
#define MMM_SPLIT_NW 4
#endif
#ifndef MMM_SPLIT_STAGES
#define MMM_SPLIT_STAGES 2
#endif
#ifndef MMM_SPLIT_SCHED
#define MMM_SPLIT_SCHED 6  // scheduling hints for digit counts from this value up (0: never)
#endif
// the 64 x 64 LDS kernel for 16-bit digits with flushing (4 or 5 digits)
#ifndef MMM_SPLIT_LDS2
#define MMM_SPLIT_LDS2 1
#endif
#ifndef MMM_SPLIT_LDS2_STAGES
#define MMM_SPLIT_LDS2_STAGES 2
#endif
#ifndef MMM_SPLIT_LDS2_WM
#define MMM_SPLIT_LDS2_WM 2  // waves along the rows (32 rows each)
#endif
#ifndef MMM_SPLIT_LDS2_WN
#define MMM_SPLIT_LDS2_WN 2  // waves along the columns (32 columns each)
#endif
// the flushing tile for 4..6 digits
#ifndef MMM_SPLIT_FWBM
#define MMM_SPLIT_FWBM 2
#endif
#ifndef MMM_SPLIT_FMINW
#define MMM_SPLIT_FMINW 2
#endif
#ifndef MMM_SPLIT_FSTAGES
#define MMM_SPLIT_FSTAGES 2
#endif
struct TileCfg {
    int wbm, minw, nw, stages;
    constexpr int bm() const { return 16 * wbm; }
    constexpr int bn() const { return 16 * nw; }
    constexpr int threads() const { return 64 * nw; }
};
__host__ __device__ constexpr TileCfg tile_cfg(int dt, int s, bool flush)
{
    return (void)dt, !flush ? (s <= 7 ? TileCfg{MMM_SPLIT_WBM, MMM_SPLIT_MINW, MMM_SPLIT_NW, MMM_SPLIT_STAGES}
                                      : TileCfg{2, 2, 4, 2})
                            : (s <= 3 ? TileCfg{4, 2, 4, 2}
                                      : (s <= 6 ? TileCfg{MMM_SPLIT_FWBM, MMM_SPLIT_FMINW, 4, MMM_SPLIT_FSTAGES}
                                                : TileCfg{2, 1, 4, 2}));
}
// The persistent batch kernel keeps the job-table walk live as well, so it
// takes smaller register footprints: 4 waves and two stages without
// flushing, one wave per SIMD where the flushing tile is at the two-wave
// limit.  Its tiles divide the single-product ones, so one workspace
// layout serves both.
// Variant 1 ("narrow") halves the tile's rows for products whose row count
// would leave most of a wide tile empty; the halved accumulator set lets a
// one-wave-per-SIMD tile run two waves per SIMD.
__host__ __device__ constexpr TileCfg narrow_cfg(TileCfg t)
{
    return t.wbm > 1 ? TileCfg{t.wbm / 2, t.minw < 2 ? 2 : t.minw, t.nw, t.stages} : t;
}
__host__ __device__ constexpr TileCfg grouped_tile_cfg(int dt, int s, bool flush, int variant = 0, int ppa = 8)
{
    // ppa < s: accumulators per pair subgroup (no flushing), up to s(s+1)/2
    // per output, so the tile keeps two row blocks per wave
    return variant == 1 ? narrow_cfg(grouped_tile_cfg(dt, s, flush, 0, ppa))
                        : (!flush ? (ppa < s ? TileCfg{2, 2, 4, 2} : (s <= 7 ? TileCfg{4, 2, 4, 2} : TileCfg{2, 2, 4, 2}))
                                  : (s >= 4 ? TileCfg{2, 1, 4, 2} : tile_cfg(dt, s, flush)));
}

// digit width: the configured one, else the type's default
__host__ inline int beta_of(int dt, int bits) { return bits ? bits : (dt == DT_BF16 ? 8 : (dt == DT_FP16 ? 9 : 7)); }

// e = E(mx) + 1 (0 for an all-zero vector)
__device__ inline int vec_exponent(double mx)
{
    if (!(mx > 0.0)) return 0;
    int e;
    frexp(mx, &e);
    return e + 1;
}

template <int DT>
__device__ inline void store_digits(char* dst, const double* d)
{
    // 8 digits -> 8 elements (16 bytes for 2-byte types, 8 bytes for int8)
    if (DT == DT_INT8) {
        unsigned int lo = 0, hi = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) lo |= ((unsigned int)(unsigned char)(signed char)(int)d[q]) << (8 * q);
#pragma unroll
        for (int q = 0; q < 4; ++q) hi |= ((unsigned int)(unsigned char)(signed char)(int)d[4 + q]) << (8 * q);
        *reinterpret_cast<uint2*>(dst) = make_uint2(lo, hi);
    } else {
        unsigned short h[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (DT == DT_BF16) {
                const float f = (float)d[q];  // |d| <= 2^8: 8 significant bits, so the top 16 bits are exact
                h[q] = (unsigned short)(__float_as_uint(f) >> 16);
            } else {
                const _Float16 x = (_Float16)(float)d[q];  // |d| <= 2^8: exact in fp16 (11 bits)
                h[q] = *reinterpret_cast<const unsigned short*>(&x);
            }
        }
        uint4 v;
        v.x = h[0] | ((unsigned int)h[1] << 16);
        v.y = h[2] | ((unsigned int)h[3] << 16);
        v.z = h[4] | ((unsigned int)h[5] << 16);
        v.w = h[6] | ((unsigned int)h[7] << 16);
        *reinterpret_cast<uint4*>(dst) = v;
    }
}

// Byte digits of 8 bits (int8, beta = 8) do not fit the nearest-digit rule
// (|d| <= 128 needs 257 values): the scaled entry r (|r| < 1/4, from one
// more exponent step) is rounded once to 8 s fractional bits, X =
// rint(r 2^(8 s)), and X is written in base 256 with digits in
// [-128, 127], least significant first: d = ((X + 128) mod 256) - 128,
// X = (X - d) / 256.
__host__ __device__ constexpr bool byte_digits(int dt, int beta) { return dt == DT_INT8 && beta == 8; }

// Digits of 8 consecutive entries along k of one row of A (or one column
// of B).  x[q] are the unscaled entries (0 outside the matrix).
template <int DT>
__device__ inline void cut(const double* x, double sc, int e, int s, int beta, char* out, i64 slice_stride)
{
    const double up = (double)(1 << beta);
    double r[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = ldexp(x[q] * sc, -e);
    if (DT == DT_INT8 && beta == 8) {
        // X (an exact integer in binary64) is cut 24 bits at a time: X =
        // 2^24 hi + lo with 0 <= lo < 2^24 (exact floor and difference), the
        // next three digits come from lo in 32-bit integers, and what is left
        // of lo after them (the carry, 0 or 1) joins hi.  Same digits as the
        // whole-integer rule, in 32-bit arithmetic.
        double X[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) X[q] = rint(ldexp(r[q], 8 * s));
        for (int t = s - 1; t >= 0;) {
            double hi[8];
            int lo[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                hi[q] = floor(X[q] * 0x1p-24);
                lo[q] = (int)(X[q] - hi[q] * 0x1p24);
            }
            for (int n = 0; n < 3 && t >= 0; ++n, --t) {
                unsigned int w0 = 0, w1 = 0;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int v = ((lo[q] + 128) & 255) - 128;
                    lo[q] = (lo[q] - v) >> 8;
                    if (q < 4) w0 |= (unsigned int)(v & 255) << (8 * q);
                    else w1 |= (unsigned int)(v & 255) << (8 * (q - 4));
                }
                *reinterpret_cast<uint2*>(out + t * slice_stride) = make_uint2(w0, w1);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) X[q] = hi[q] + (double)lo[q];
        }
        return;
    }
    for (int t = 0; t < s; ++t) {
        double d[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double y = r[q] * up;
            d[q] = rint(y);
            r[q] = y - d[q];
        }
        store_digits<DT>(out + t * slice_stride, d);
    }
}

// A: one thread per (row i < Np, 8-entry chunk of the padded K); the
// threads of one 64-byte digit block are adjacent, then rows, then blocks,
// so the digit stores of a wave are contiguous.
template <int DT>
// rmax_raw: rmax holds max_k |A_ik| before the 2^lambda scaling (exact to
// scale afterwards: x -> fl(2^lambda x) is monotone, so it commutes with max).
__device__ __forceinline__ void split_a_body(const double* __restrict__ A, i64 N, i64 P, i64 Np, i64 Kp,
                                             const double* __restrict__ rmax, const int* lam, int s, int beta,
                                             char* __restrict__ SA, int* __restrict__ ea, i64 block, i64 nblocks,
                                             bool rmax_raw = false)
{
    constexpr int ES = Digit<DT>::esize;
    constexpr int TB = KB / (8 * ES);  // threads per 64-byte block
    const i64 total = Np * (Kp / 8);
    const double sc = lam ? ldexp(1.0, *lam) : 1.0;
    for (i64 c = block * 256 + threadIdx.x; c < total; c += nblocks * 256) {
        const int q = (int)(c % TB);
        const i64 rest = c / TB, i = rest % Np, kb = rest / Np;
        const i64 k0 = kb * (KB / ES) + q * 8;
        const int e = i < N ? vec_exponent(rmax_raw ? rmax[i] * sc : rmax[i]) + byte_digits(DT, beta) : 0;
        double x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = (i < N && k0 + r < P) ? A[i * P + k0 + r] : 0.0;
        char* out = SA + (kb * s * Np + i) * KB + q * 8 * ES;
        cut<DT>(x, sc, e, s, beta, out, Np * KB);
        if (k0 == 0) ea[i] = e;
    }
}

// B (P x M, row-major) to SB[kb][u][j][64 bytes]: a 64 (k) x kBJ (j) tile
// goes through LDS so both the loads (along j) and the stores (64-byte
// blocks of neighbouring columns) are contiguous.  kBJ = 32 keeps the tile
// at 17 KiB of LDS, so the workgroups that share the launch (A's, which
// need none) are not limited to four per CU by it.
template <int DT>
__device__ __forceinline__ void split_b_body(const double* __restrict__ B, i64 P, i64 M, i64 Mp, i64 Kp,
                                             const double* __restrict__ cmax, const int* lam, int s, int beta,
                                             char* __restrict__ SB, int* __restrict__ fb, i64 block,
                                             double (*T)[kBJ + 1], bool cmax_raw = false)
{
    constexpr int ES = Digit<DT>::esize;
    constexpr int TB = KB / (8 * ES);  // threads per 64-byte block
    const i64 tiles_j = Mp / kBJ;
    const i64 kt = block / tiles_j;
    const i64 j0 = (block - kt * tiles_j) * kBJ, k0 = kt * 64;
    const int tid = threadIdx.x;
    const double sc = lam ? ldexp(1.0, -*lam) : 1.0;
#pragma unroll
    for (int q = 0; q < 64 * kBJ / 256; ++q) {
        const int e = q * 256 + tid, kr = e / kBJ, jc = e % kBJ;
        const i64 k = k0 + kr, j = j0 + jc;
        T[kr][jc] = (k < P && j < M) ? B[k * M + j] : 0.0;
    }
    __syncthreads();
    // 256 chunks of 8 entries (kBJ columns x 64 k), one per thread
    {
        const int c = tid;
        const int q = c % TB, jc = (c / TB) % kBJ, blk = c / (TB * kBJ);
        const int kk = blk * (KB / ES) + q * 8;
        const i64 j = j0 + jc;
        const int e = j < M ? vec_exponent(cmax_raw ? cmax[j] * sc : cmax[j]) + byte_digits(DT, beta) : 0;
        double x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = T[kk + r][jc];
        const i64 kb = kt * ES + blk;
        char* out = SB + (kb * s * Mp + j) * KB + q * 8 * ES;
        cut<DT>(x, sc, e, s, beta, out, Mp * KB);
        if (kt == 0 && kk == 0) fb[j] = e;
    }
}

// One launch for both operands' digits: workgroups below nblk_a stride over
// A's (row, 8-entry chunk) pairs, the rest take one 64 x kBJ tile of B each.
template <int DT>
__global__ __launch_bounds__(256) void split_ab_kernel(const double* __restrict__ A, i64 N, i64 P, i64 Np, i64 Kp,
                                                       const double* __restrict__ rmax, const int* lam, int s,
                                                       int beta, char* __restrict__ SA, int* __restrict__ ea, i64 nblk_a,
                                                       const double* __restrict__ B, i64 M, i64 Mp,
                                                       const double* __restrict__ cmax, char* __restrict__ SB,
                                                       int* __restrict__ fb)
{
    __shared__ double T[64][kBJ + 1];
    const i64 b = blockIdx.x;
    if (b < nblk_a) split_a_body<DT>(A, N, P, Np, Kp, rmax, lam, s, beta, SA, ea, b, nblk_a, true);
    else split_b_body<DT>(B, P, M, Mp, Kp, cmax, lam, s, beta, SB, fb, b - nblk_a, T, true);
}

// ---- the digit-product GEMM -------------------------------------------------

template <int DT>
struct Mfma;
template <>
struct Mfma<DT_BF16> {
    typedef v4f acc_t;
    __device__ static acc_t run(u32x4 a, u32x4 b, acc_t c)
    {
        v8bf x, y;
        __builtin_memcpy(&x, &a, 16);
        __builtin_memcpy(&y, &b, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
    }
};
template <>
struct Mfma<DT_FP16> {
    typedef v4f acc_t;
    __device__ static acc_t run(u32x4 a, u32x4 b, acc_t c)
    {
        v8h x, y;
        __builtin_memcpy(&x, &a, 16);
        __builtin_memcpy(&y, &b, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
    }
};
template <>
struct Mfma<DT_INT8> {
    typedef v4i acc_t;
    __device__ static acc_t run(u32x4 a, u32x4 b, acc_t c)
    {
        v4i x, y;
        __builtin_memcpy(&x, &a, 16);
        __builtin_memcpy(&y, &b, 16);
        return __builtin_amdgcn_mfma_i32_16x16x64_i8(x, y, c, 0, 0, 0);
    }
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

// Slot of 16-byte chunk c of row r (r < 16) in a 16-row x 64-byte LDS
// block.  Row r starts at byte 64 r; XOR-ing the chunk with a function of
// r spreads the 16 rows of one chunk column over all banks, so the MFMA
// operand reads (lane: row l % 16, chunk l / 16) are free of conflicts.
__device__ __forceinline__ int swz(int r, int c) { return c ^ (((r >> 1) ^ (r >> 2)) & 3); }

// Issue order of one K block's digit pairs for the instruction scheduler:
// the A fragments of digits 0 and 1 first, then after the S - t MFMAs of
// each (t, i) the read of fragment (t + 2, i), so every LDS read is two
// digit levels ahead of its first use.
template <int S, int WBM, int T = 0, int I = 0>
__device__ __forceinline__ void sched_digit_pairs()
{
    if constexpr (T == 0 && I == 0) __builtin_amdgcn_sched_group_barrier(0x100, S >= 2 ? 2 * WBM : WBM, 0);
    if constexpr (T < S) {
        __builtin_amdgcn_sched_group_barrier(0x008, S - T, 0);
        if constexpr (T + 2 < S) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        if constexpr (I + 1 < WBM) sched_digit_pairs<S, WBM, T, I + 1>();
        else sched_digit_pairs<S, WBM, T + 1, 0>();
    }
}

// Workgroup of NW waves side by side along N; wave w owns columns
// n0 + 16 w .. n0 + 16 w + 15 and all BM rows (WBM blocks of 16).  Per K
// block of 64 bytes:
//   A: the S digit planes of the BM rows (S x BM x 64 bytes, contiguous
//      KiBs in the workspace) are loaded straight into LDS (16 bytes per
//      lane, lane l of a wave instruction landing at base + 16 l, rows
//      swizzled by swz), NST stages, no staging registers;
//   B: each wave loads its own S fragments (16 columns x 64 bytes per
//      digit: one KiB) into registers, NST sets;
// the loads of block kb + NST - 1 are issued while block kb computes;
// then every wave runs the s(s+1)/2 kept digit pairs, pair (t, u)
// accumulating into group t + u.  Both MFMAs used take lane l's operand
// as row (A) / column (B) l % 16 and bytes 16 (l / 16) .. 16 (l / 16) + 15
// of the K block; result element r of lane l is D[4 (l / 16) + r][l % 16].
// Accumulators without flushing for products whose K is too long for a
// whole group in one accumulator but short enough for PPA pairs: group g's
// g + 1 pairs are spread over ceil((g + 1) / PPA) accumulators (pair (t, u)
// in the (t / PPA)-th), each holding at most PPA pairs' products of the
// whole K.  PPA >= S is one accumulator per group.
constexpr int subs_of(int g, int ppa) { return (g + ppa) / ppa; }
constexpr int acc_base(int g, int ppa) { return g == 0 ? 0 : acc_base(g - 1, ppa) + subs_of(g - 1, ppa); }

template <int DT, int S, bool FLUSH, int WBM, int NW, int NST, int PPA = S>
__device__ __forceinline__ void split_tile(const char* __restrict__ SA, const char* __restrict__ SB,
                                           const int* __restrict__ ea, const int* __restrict__ fb,
                                           double* __restrict__ C, i64 N, i64 M, i64 Np, i64 Mp, i64 Kp, i64 tm,
                                           i64 tn, int beta, int unit, int runlen, char* lds)
{
    typedef Digit<DT> D;
    typedef typename Mfma<DT>::acc_t acc_t;
    constexpr TileCfg TC{WBM, 1, NW, NST};
    constexpr int BM = TC.bm(), BN = TC.bn();
    constexpr int G = S;                  // groups g = 2 .. S+1 -> index g-2
    constexpr int NBLK = S * WBM;         // KiB blocks of A per K block
    constexpr int STAGE = NBLK * 1024;
    const i64 m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const i64 steps = Kp * D::esize / KB;
    const i64 plane_a = Np * KB, plane_b = Mp * KB;  // bytes of one digit plane of one K block

    static_assert(!FLUSH || PPA >= S, "flushing keeps one accumulator per group");
    constexpr int NACC = acc_base(G, PPA);
    acc_t acc[NACC][WBM];
    double acc64[FLUSH ? G : 1][FLUSH ? WBM : 1][4];
#pragma unroll
    for (int g = 0; g < NACC; ++g)
#pragma unroll
        for (int i = 0; i < WBM; ++i) acc[g][i] = (acc_t){0, 0, 0, 0};
    if (FLUSH)
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int i = 0; i < WBM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[g][i][r] = 0.0;

    // per-lane byte offsets (32 bits) from wave-uniform bases: the loads
    // take a scalar base plus a vector offset, so no 64-bit per-lane
    // addresses are kept live.  A: row lane / 4 of a KiB block, swizzled chunk.
    const int dr = lane >> 2;
    const unsigned offa = (unsigned)(dr * KB + swz(dr, lane & 3) * 16);
    const unsigned offb = (unsigned)((wave * 16 + li) * KB + lq * 16);
    const char* sa0 = SA + m0 * KB;  // row m0 of digit plane 0 of K block 0
    const char* sb0 = SB + n0 * KB;
    const int rd = li * KB + swz(li, lq) * 16;  // this lane's fragment within a KiB block

    auto issue_a = [&](i64 kb, int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < (NBLK + NW - 1) / NW; ++q) {
            const int blk = q * NW + wave;  // block = (digit t, 16-row block) written by this wave instruction
            if (NBLK % NW == 0 || blk < NBLK) {
                const int t = blk / WBM, rb = blk % WBM;
                const char* base = sa0 + (kb * S + t) * plane_a + rb * 16 * KB;
                __builtin_amdgcn_global_load_lds((gbl_ptr_t)(base + offa), (lds_ptr_t)(lds + buf * STAGE + blk * 1024),
                                                 16, 0, 0);
            }
        }
    };
    // B fragments of NST K blocks: the one in use and the NST - 1 in flight
    u32x4 bring[NST][S];
    auto load_b = [&](i64 kb, u32x4(&b)[S]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < S; ++u) b[u] = *reinterpret_cast<const u32x4*>(sb0 + (kb * S + u) * plane_b + offb);
    };
    // memory instructions this wave issues per K block (fewest over the
    // waves), so that waiting for "at most n blocks' worth outstanding"
    // is never too lax
    constexpr int PER_BLOCK = NBLK / NW + S;

    // Group g (pairs with t + u = g, index from 0) holds g + 1 digit pairs;
    // `unit` is the number of steps one pair's products can be summed
    // within the accumulator's exact range, so group g may run
    // unit / (g + 1) steps between flushes: (g + 1) (unit / (g + 1)) <= unit
    // pairs' worth of products, each of its partial sums within the range.
    int left[FLUSH ? G : 1];
#pragma unroll
    for (int g = 0; g < (FLUSH ? G : 1); ++g) left[g] = unit / (g + 1);
#pragma unroll
    for (int q = 0; q < NST - 1; ++q)
        if (q < steps) {
            issue_a(q, q);
            load_b(q, bring[q]);
        }
    // K block kb uses stage and B slot kb % NST; the loop is unrolled NST
    // times so both are compile-time constants.
    auto step = [&](auto slot, i64 kb) __attribute__((always_inline)) {
        constexpr int J = decltype(slot)::value;
        // this block's A has landed in LDS (own loads; the later blocks'
        // loads may still be in flight) and B in registers; after the
        // barrier every wave's A has landed and every wave is done with the
        // stage the loads issued next overwrite
        const i64 ahead = (steps - 1 - kb) < (NST - 2) ? (steps - 1 - kb) : (NST - 2);
        if (NST >= 4 && ahead >= 2) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * PER_BLOCK) : "memory");
        else if (NST >= 3 && ahead >= 1) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(PER_BLOCK) : "memory");
        else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (kb + NST - 1 < steps) {
            issue_a(kb + NST - 1, (J + NST - 1) % NST);
            load_b(kb + NST - 1, bring[(J + NST - 1) % NST]);
        }
        const char* la = lds + J * STAGE + rd;
#pragma unroll
        for (int t = 0; t < S; ++t)
#pragma unroll
            for (int i = 0; i < WBM; ++i) {
                const u32x4 a = *reinterpret_cast<const u32x4*>(la + (t * WBM + i) * 1024);
#pragma unroll
                for (int u = 0; u + t < S; ++u) {
                    const int k = acc_base(t + u, PPA) + t / PPA;
                    acc[k][i] = Mfma<DT>::run(a, bring[J][u], acc[k][i]);
                }
            }
        if (MMM_SPLIT_SCHED > 0 && S >= MMM_SPLIT_SCHED) sched_digit_pairs<S, WBM>();
        if (FLUSH) {
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (--left[g] == 0) {
                    left[g] = unit / (g + 1);
#pragma unroll
                    for (int i = 0; i < WBM; ++i) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc64[g][i][r] += (double)acc[g][i][r];
                        acc[g][i] = (acc_t){0, 0, 0, 0};
                    }
                }
        }
    };
    for (i64 kb = 0; kb < steps; kb += NST) {
        step(std::integral_constant<int, 0>(), kb);
        if (kb + 1 < steps) step(std::integral_constant<int, 1>(), kb + 1);
        if (NST >= 3 && kb + 2 < steps) step(std::integral_constant<int, (NST >= 3 ? 2 : 0)>(), kb + 2);
        if (NST >= 4 && kb + 3 < steps) step(std::integral_constant<int, (NST >= 4 ? 3 : 0)>(), kb + 3);
    }

    // runs of `runlen` groups from the finest (index G - 1, scale 2^(-beta (G + 1)))
    // down: T = sum G_g 2^(beta pos), pos = the group's distance from its
    // run's finest group, exact; each run added to c with one rounding; then
    // the scale 2^(e_i + f_j)
    const i64 gn = n0 + wave * 16 + li;
#pragma unroll
    for (int i = 0; i < WBM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const i64 gm = m0 + i * 16 + 4 * lq + r;
            double c = 0.0, T = 0.0;
            int pos = 0;
#pragma unroll
            for (int g = G - 1; g >= 0; --g) {
                double Gg = FLUSH ? acc64[g][i][r] + (double)acc[g][i][r] : (double)acc[acc_base(g, PPA)][i][r];
                // the other accumulators of the group (exact integers: exact sums)
#pragma unroll
                for (int k = 1; k < subs_of(g, PPA); ++k) Gg = Gg + (double)acc[acc_base(g, PPA) + k][i][r];
                T = pos == 0 ? Gg : T + Gg * ldexp(1.0, beta * pos);
                if (pos == runlen - 1 || g == 0) {
                    c = c + ldexp(T, -beta * (g + pos + 2));
                    pos = 0;
                } else {
                    ++pos;
                }
            }
            if (gm < N && gn < M) C[gm * M + gn] = ldexp(c, ea[gm] + fb[gn]);
        }
}

// ---- 16-bit digits with flushing: both operands in LDS, 2 x 2 blocks per wave --
//
// With the recombination in runs of three groups, an output needs one FP32
// accumulator per group but only two FP64 run accumulators (instead of one
// per group), which leaves room for each wave to own 2 x 2 blocks of
// 16 x 16 outputs.  A workgroup of 4 waves (2 x 2) then owns a 64 x 64 tile
// and reads 20 KiB of digits per K block (S = 5) for 60 products per wave,
// against 30 KiB for 30 products of the 32 x 64 tile: a third fewer bytes
// per product.  Both operands' digit planes go global -> LDS by
// global_load_lds (1 KiB blocks of 16 rows or columns x 64 bytes, the
// chunks swizzled as in split_tile), two stages; each wave then reads all
// its 4 S fragments of the K block and runs the products group by group,
// finest group last.
//
// Flushes follow a static schedule instead of per-group counters: the K loop
// is unrolled over periods of 8 steps and group g (g + 1 pairs) restarts
// every iv_g steps, iv_g the largest power of two not above
// min(8, unit / (g + 1)) (unit: steps one pair may accumulate exactly), so
// its partial sums stay in FP32's exact range.  Restarting means its old
// FP32 value goes into its run's FP64 accumulator (weighted by
// 2^(beta pos), exact) and its first product of the step takes a zero
// accumulator; with the groups run in ascending order, the flush of a
// finer group can issue while the matrix cores work on the coarser ones.
// Where a flush happens cannot change the exact sums, so every schedule
// within the range gives the same bits.
template <int BETA>
struct FlushSched {
    static constexpr int unit = 1 << (21 - 2 * BETA);  // 2^24 / 2^(2 beta - 2) / 32
    static constexpr int period = 8;
    static constexpr int iv(int g)
    {
        const int q = unit / (g + 1);
        int p = 1;
        while (p * 2 <= q && p * 2 <= period) p *= 2;
        return p;
    }
    // groups starting a window at step j of a period (bit g)
    static constexpr unsigned starts(int j, int S)
    {
        unsigned m = 0;
        for (int g = 0; g < S; ++g)
            if (j % iv(g) == 0) m |= 1u << g;
        return m;
    }
};

constexpr int popcount_c(unsigned m) { return m ? (int)(m & 1u) + popcount_c(m >> 1) : 0; }

// Digit level 0 of a step in the LDS kernel: 4 S products, and 32 flush operations
// (16 conversions, 16 fused adds) per group starting a window; interleave
// them so that the flushes issue in the shadow of the products.
template <int NM, int NV, int K = 0>
__device__ __forceinline__ void sched_level0_k()
{
    if constexpr (K < NM) {
        constexpr int nv = NV / NM + (K < NV % NM ? 1 : 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if constexpr (nv > 0) __builtin_amdgcn_sched_group_barrier(0x002, nv, 0);
        sched_level0_k<NM, NV, K + 1>();
    }
}
template <int S, int NFLUSH>
__device__ __forceinline__ void sched_level0()
{
    sched_level0_k<4 * S, 32 * NFLUSH>();
}

template <int DT, int S, int BETA, int NST, int WM, int WN>
__device__ __forceinline__ void split_tile_lds2(const char* __restrict__ SA, const char* __restrict__ SB,
                                                const int* __restrict__ ea, const int* __restrict__ fb,
                                                double* __restrict__ C, i64 N, i64 M, i64 Np, i64 Mp, i64 Kp, i64 tm,
                                                i64 tn, char* lds)
{
    typedef typename Mfma<DT>::acc_t acc_t;
    typedef FlushSched<BETA> F;
    constexpr int BM = 32 * WM, BN = 32 * WN, NW = WM * WN;
    constexpr int RBA = BM / 16, RBB = BN / 16;  // 16-row / 16-column blocks per digit
    constexpr int ABLK = S * RBA, NBLK = ABLK + S * RBB;  // KiB blocks per stage: A's, then B's
    constexpr int STAGE = NBLK * 1024;
    constexpr int R = (S + 2) / 3;  // runs of three groups, from the finest
    static_assert(RBA <= NW && RBB <= NW, "one block of each digit per wave at most");
    const i64 m0 = tm * BM, n0 = tn * BN;
    // the wave index is uniform across the wave: said so, the compiler keeps
    // the per-wave bases in scalar registers (loads: scalar base + 32-bit lane offset)
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WM, wn = wave / WM;  // this wave: rows 32 wm .., columns 32 wn ..
    const int li = lane & 15, lq = lane >> 4;
    const i64 steps = Kp * 2 / KB;
    const i64 plane_a = Np * KB, plane_b = Mp * KB;

    acc_t acc[S][2][2];
    double run64[R][2][2][4];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) run64[q][i][j][r] = 0.0;

    // the loads of a stage: for every digit, wave w brings A's 16-row block w
    // (w < BM / 16) and B's 16-column block w (w < BN / 16); lane l lands at
    // byte 16 l of the block, taking the source chunk the swizzle puts there
    const int dr = lane >> 2;
    const unsigned offs = (unsigned)(dr * KB + swz(dr, lane & 3) * 16);
    const char* sa0 = SA + (m0 + wave * 16) * KB;
    const char* sb0 = SB + (n0 + wave * 16) * KB;
    const int rd = li * KB + swz(li, lq) * 16;  // this lane's fragment within a KiB block
    auto issue = [&](i64 kb, int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < S; ++q) {
            if (RBA == NW || wave < RBA)
                __builtin_amdgcn_global_load_lds((gbl_ptr_t)(sa0 + (kb * S + q) * plane_a + offs),
                                                 (lds_ptr_t)(lds + buf * STAGE + (q * RBA + wave) * 1024), 16, 0, 0);
            if (RBB == NW || wave < RBB)
                __builtin_amdgcn_global_load_lds((gbl_ptr_t)(sb0 + (kb * S + q) * plane_b + offs),
                                                 (lds_ptr_t)(lds + buf * STAGE + (ABLK + q * RBB + wave) * 1024), 16, 0, 0);
        }
    };

    // one K block: J = stage; the groups in START begin a new exact-range
    // window at this step: the FP32 value of their previous window goes into
    // their run's FP64 accumulator (weighted by 2^(beta pos), exact) and
    // their first product here takes a zero accumulator.  Products run level
    // by level, level t taking digit t of A against every digit u of B with
    // t + u < S; level 0 gives group u its first product at position u, so
    // the flush of group u can issue while the matrix cores work on groups
    // 0 .. u - 1.
    // K block kb lives in stage kb % NST; the loads of the next NST - 2
    // blocks may still be in flight while it is used
    auto step = [&](auto Sc, i64 kb) __attribute__((always_inline)) {
        constexpr unsigned START = decltype(Sc)::value;
        // this block's loads (own) have landed; after the barrier everyone's
        // have, and everyone is done with the stage the next loads overwrite
        // (block kb - 1's).  The next NST - 2 blocks' loads may stay in flight.
        const i64 ahead = steps - 1 - kb;
        if (NST >= 4 && ahead >= 2) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(4 * S) : "memory");
        else if (NST >= 3 && ahead >= 1) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * S) : "memory");
        else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        const int J = (int)(kb % NST);
        if (kb + NST - 1 < steps) issue(kb + NST - 1, J == 0 ? NST - 1 : J - 1);
        const char* la = lds + J * STAGE + rd;
        u32x4 bf[S][2];
#pragma unroll
        for (int u = 0; u < S; ++u)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                bf[u][j] = *reinterpret_cast<const u32x4*>(la + (ABLK + u * RBB + wn * 2 + j) * 1024);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            u32x4 af[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = *reinterpret_cast<const u32x4*>(la + (t * RBA + wm * 2 + i) * 1024);
#pragma unroll
            for (int u = 0; u + t < S; ++u) {
                const int g = t + u;
                const bool restart = t == 0 && ((START >> g) & 1u);
                if (restart) {
                    const int q = (S - 1 - g) / 3;
                    const double w = (double)(1ull << (BETA * ((S - 1 - g) % 3)));
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                run64[q][i][j][r] = fma((double)acc[g][i][j][r], w, run64[q][i][j][r]);
                                // computed here, not sunk to the end of the tile with
                                // the FP32 values kept alive (spilled) until then
                                asm volatile("" : "+v"(run64[q][i][j][r]));
                            }
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[g][i][j] = Mfma<DT>::run(af[i], bf[u][j], restart ? (acc_t){0, 0, 0, 0} : acc[g][i][j]);
            }
            // level 0: each product of group u issues between the flush
            // operations of the groups after it (cvt + fma per value)
            if (t == 0) sched_level0<S, popcount_c(START)>();
            // keep the levels in order (LDS reads may move up a level): the
            // scheduler would otherwise gather the zero-accumulator products
            // at the end and lengthen the fragments' lifetimes past the
            // register budget
            __builtin_amdgcn_sched_barrier(0x100);
        }
    };

    // a window of group g starts at step j of a period when j is a multiple
    // of iv_g: every group starts one at the first step of each period (the
    // first of the tile adds the zero accumulators to the runs)
    constexpr unsigned ALL = (1u << S) - 1;
#pragma unroll
    for (int g = 0; g < S; ++g)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[g][i][j] = (acc_t){0, 0, 0, 0};
#define MMM_LDS2_STEP(j) step(std::integral_constant<unsigned, F::starts(j, S)>(), kb + (j))
    i64 kb = 0;
#pragma unroll
    for (int q = 0; q < NST - 1; ++q)
        if (q < steps) issue(q, q);
    for (; kb + F::period <= steps; kb += F::period) {
        MMM_LDS2_STEP(0);
        MMM_LDS2_STEP(1);
        MMM_LDS2_STEP(2);
        MMM_LDS2_STEP(3);
        MMM_LDS2_STEP(4);
        MMM_LDS2_STEP(5);
        MMM_LDS2_STEP(6);
        MMM_LDS2_STEP(7);
    }
#undef MMM_LDS2_STEP
    // the last steps are windows of one step each
    for (; kb < steps; ++kb) step(std::integral_constant<unsigned, ALL>(), kb);

    // close the last windows, then runs from the finest: c = c + 2^(-beta (f + 2)) T
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const i64 gn = n0 + wn * 32 + j * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
#pragma unroll
                for (int g = 0; g < S; ++g)
                    run64[(S - 1 - g) / 3][i][j][r] = fma((double)acc[g][i][j][r],
                                                          (double)(1ull << (BETA * ((S - 1 - g) % 3))),
                                                          run64[(S - 1 - g) / 3][i][j][r]);
                double c = 0.0;
#pragma unroll
                for (int q = 0; q < R; ++q) c = c + ldexp(run64[q][i][j][r], -BETA * (S - 1 - 3 * q + 2));
                const i64 gm = m0 + wm * 32 + i * 16 + 4 * lq + r;
                if (gm < N && gn < M) C[gm * M + gn] = ldexp(c, ea[gm] + fb[gn]);
            }
        }
}

// Tile order of the single-product GEMMs.  Workgroups are dealt round robin
// to the 8 XCDs; each XCD gets a contiguous range of tiles and walks it in
// groups of 256 rows (256 / bm tile rows), column by column inside a group.
// The resident tiles of an XCD then share the digit blocks of their rows and
// columns in its L2, and the digit rows that all XCDs use at one time (8
// groups of 256 rows) stay within the memory-side cache while every column
// passes by: at 8192^3 with 64-row tiles, 256-row groups fetch a third
// fewer bytes from beyond L2 than 512-row groups (counted) and run 5-8%
// faster.
__device__ inline void tile_order(i64 b, i64 tiles_m, i64 tiles_n, int bm, i64& tm, i64& tn)
{
    const i64 total = tiles_m * tiles_n;
    if (total % 8 == 0) b = (b % 8) * (total / 8) + b / 8;
    const i64 G = bm >= 256 ? 1 : 256 / bm;
    const i64 grp = b / (G * tiles_n), first = grp * G;
    const i64 gs = (tiles_m - first) < G ? (tiles_m - first) : G;
    const i64 w = b - grp * G * tiles_n;
    tm = first + w % gs;
    tn = w / gs;
}

constexpr int kLds2BM = 32 * MMM_SPLIT_LDS2_WM, kLds2BN = 32 * MMM_SPLIT_LDS2_WN;
constexpr int kLds2Threads = 64 * MMM_SPLIT_LDS2_WM * MMM_SPLIT_LDS2_WN;

template <int DT, int S, int BETA>
__global__ __launch_bounds__(kLds2Threads, 2) void split_gemm_lds2_kernel(const char* __restrict__ SA, const char* __restrict__ SB,
                                                              const int* __restrict__ ea, const int* __restrict__ fb,
                                                              double* __restrict__ C, i64 N, i64 M, i64 Np, i64 Mp,
                                                              i64 Kp, i64 tiles_m, i64 tiles_n)
{
    extern __shared__ __align__(16) char lds[];
    i64 tm, tn;
    tile_order(blockIdx.x, tiles_m, tiles_n, kLds2BM, tm, tn);
    split_tile_lds2<DT, S, BETA, MMM_SPLIT_LDS2_STAGES, MMM_SPLIT_LDS2_WM, MMM_SPLIT_LDS2_WN>(
        SA, SB, ea, fb, C, N, M, Np, Mp, Kp, tm, tn, lds);
}

template <int DT, int S, bool FLUSH>
__global__ __launch_bounds__(tile_cfg(DT, S, FLUSH).threads(), tile_cfg(DT, S, FLUSH).minw) void split_gemm_kernel(const char* __restrict__ SA, const char* __restrict__ SB,
                                                         const int* __restrict__ ea, const int* __restrict__ fb,
                                                         double* __restrict__ C, i64 N, i64 M, i64 Np, i64 Mp,
                                                         i64 Kp, i64 tiles_m, i64 tiles_n, int beta, int unit,
                                                         int runlen)
{
    extern __shared__ __align__(16) char lds[];
    i64 tm, tn;
    tile_order(blockIdx.x, tiles_m, tiles_n, tile_cfg(DT, S, FLUSH).bm(), tm, tn);
    split_tile<DT, S, FLUSH, tile_cfg(DT, S, FLUSH).wbm, tile_cfg(DT, S, FLUSH).nw, tile_cfg(DT, S, FLUSH).stages>(SA, SB, ea, fb, C, N, M, Np, Mp, Kp, tm, tn,
                                                          beta, unit, runlen, lds);
}

// Persistent grid over the tiles of a group of split jobs (same digit type,
// count and tile variant): tile t is job p's (t - prefix[p])-th tile,
// row-major over ceil(N / BM) x (Mp / BN) tiles.
template <int DT, int S, bool FLUSH, int V, int PPA>
__global__ __launch_bounds__(grouped_tile_cfg(DT, S, FLUSH, V, PPA).threads(), grouped_tile_cfg(DT, S, FLUSH, V, PPA).minw) void split_gemm_grouped_kernel(const SplitJob* __restrict__ jobs,
                                                                 const i64* __restrict__ prefix, int njobs,
                                                                 int beta, int unit, TileSchedule sch)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ int slot;
    constexpr TileCfg TC = grouped_tile_cfg(DT, S, FLUSH, V, PPA);
    for (;;) {
        const int q = claim_tile(sch, &slot);
        if (q >= sch.total) break;
        const i64 t = sch.list[q];
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const SplitJob& j = jobs[lo];
        const i64 local = t - prefix[lo];
        const i64 tiles_n = j.Mp / TC.bn();
        split_tile<DT, S, FLUSH, TC.wbm, TC.nw, TC.stages, PPA>(j.SA, j.SB, j.ea, j.fb, j.C, j.N, j.M, j.Np, j.Mp, j.Kp, local / tiles_n,
                                 local % tiles_n, beta, unit, j.runlen, lds);
        __syncthreads();
    }
    release_tiles(sch);
}

// ---- batched preprocessing: blockIdx.y selects the job -----------------------

// One pass over a row-major rows x len matrix (a single product's A or B),
// 16 rows per workgroup streamed through LDS in chunks of 256 columns:
//   NORMS:  each of 16 lanes folds its row's NormInf sum (Section 1.4) in
//           order from 0.0; the largest goes to *norm by an atomic max;
//   ROWMAX: 16 threads per row take the max |x| of 16 columns each and
//           fold them by shuffles (to rmax, unscaled);
//   COLMAX: each thread takes one column's max |x| over the workgroup's
//           rows, stored to cpart[workgroup][column] (colmax_kernel folds
//           the workgroups).
// Only the sums are bound to an order; the maxima use every thread.
// *norm is cleared beforehand.
template <bool NORMS, bool ROWMAX, bool COLMAX>
__device__ __forceinline__ void stats_body(const double* __restrict__ X, i64 rows, i64 len,
                                           double* __restrict__ norm, double* __restrict__ rmax,
                                           double* __restrict__ cpart, i64 block, double (*T)[RV][RL + 1])
{
    static_assert(RL == 256, "one column of the chunk per thread");
    const int tid = threadIdx.x;
    const i64 v0 = block * RV;
    const i64 nchunks = (len + RL - 1) / RL;
    double r[RPER];
    auto load = [&](i64 c) {
#pragma unroll
        for (int q = 0; q < RPER; ++q) {
            const int e = q * 256 + tid, v = e / RL, x = e % RL;
            const i64 gv = v0 + v, gx = c * RL + x;
            r[q] = (gv < rows && gx < len) ? X[gv * len + gx] : 0.0;
        }
    };
    // |x| at the store, so the loads of the next chunk stay in flight while
    // this one is folded
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < RPER; ++q) {
            const int e = q * 256 + tid;
            T[buf][e / RL][e % RL] = fabs(r[q]);
        }
    };
    double acc = 0.0, mx = 0.0;
    if (nchunks > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (i64 c = 0; c < nchunks; ++c) {
        const int cur = (int)(c & 1);
        if (c + 1 < nchunks) load(c + 1);
        if (NORMS && tid < RV) {
            const i64 rem = len - c * RL;
            const int cnt = rem < RL ? (int)rem : RL;
            const double* row = T[cur][tid];
            if (cnt == RL) acc = fold_chunk<RED_ABS_SUM>(row, acc);  // entries already |x|
            else
                for (int x = 0; x < cnt; ++x) acc = acc + row[x];
        }
        if (ROWMAX) {
            // entries past the end were stored as 0.0, below every |x|
            const double* row = T[cur][tid / 16];
            double m = 0.0;
#pragma unroll
            for (int x = 0; x < RL / 16; ++x) m = max_s13(m, row[x * 16 + tid % 16]);
            mx = max_s13(mx, m);
        }
        if (COLMAX) {
            double m = 0.0;
#pragma unroll
            for (int v = 0; v < RV; ++v) m = max_s13(m, T[cur][v][tid]);
            const i64 gx = c * RL + tid;
            if (gx < len) cpart[block * len + gx] = m;
        }
        if (c + 1 < nchunks) store(cur ^ 1);
        __syncthreads();
    }
    if (NORMS && tid < RV && v0 + tid < rows)
        atomicMax(reinterpret_cast<unsigned long long*>(norm), (unsigned long long)__double_as_longlong(acc));
    if (ROWMAX) {
        // the 16 partial maxima of a row sit in 16 neighbouring lanes
        unsigned long long u = (unsigned long long)__double_as_longlong(mx);
        for (int o = 1; o < 16; o *= 2) {
            const unsigned long long w = __shfl_xor(u, o);
            u = w > u ? w : u;
        }
        if (tid % 16 == 0 && v0 + tid / 16 < rows) rmax[v0 + tid / 16] = __longlong_as_double((long long)u);
    }
}

// One launch for both operands: workgroups below nblk_a take 16 rows of A
// (its norm and row maxima), the rest 16 rows of B (its norm and per-
// workgroup column maxima), so the two passes share the machine.
template <bool NORMS>
__global__ __launch_bounds__(256) void stats_pair_kernel(const double* __restrict__ A, i64 N, i64 P,
                                                         double* __restrict__ nA, double* __restrict__ rmax,
                                                         i64 nblk_a, const double* __restrict__ B, i64 M,
                                                         double* __restrict__ nB, double* __restrict__ cpart)
{
    __shared__ double T[2][RV][RL + 1];
    const i64 b = blockIdx.x;
    if (b < nblk_a) stats_body<NORMS, true, false>(A, N, P, nA, rmax, nullptr, b, T);
    else stats_body<NORMS, false, true>(B, P, M, nB, nullptr, cpart, b - nblk_a, T);
}

// cmax[j] = max over the nparts rows of cpart (nparts x M) of column j:
// 32 columns per workgroup, 8 threads per column striding the parts, then
// folded through LDS.
__global__ __launch_bounds__(256) void colmax_kernel(const double* __restrict__ cpart, i64 nparts, i64 M,
                                                     double* __restrict__ cmax)
{
    __shared__ double T[8][32];
    const int tid = threadIdx.x, cc = tid % 32, ps = tid / 32;
    const i64 j = (i64)blockIdx.x * 32 + cc;
    double m = 0.0;
    if (j < M)
        for (i64 p = ps; p < nparts; p += 8) m = max_s13(m, cpart[p * M + j]);
    T[ps][cc] = m;
    __syncthreads();
    if (ps == 0 && j < M) {
#pragma unroll
        for (int q = 1; q < 8; ++q) m = max_s13(m, T[q][cc]);
        cmax[j] = m;
    }
}

// Clears the atomic-max targets of every job (one workgroup per job): the
// two norms and the column maxima of B.
__global__ __launch_bounds__(256) void jobs_zero_stats_kernel(const SplitJob* __restrict__ jobs)
{
    const SplitJob& j = jobs[blockIdx.x];
    if (threadIdx.x == 0) {
        *j.nA = 0.0;
        *j.nB = 0.0;
    }
    for (i64 c = threadIdx.x; c < j.M; c += 256) j.cmax[c] = 0.0;
}

// Largest of non-negative doubles by their bit patterns (which order them
// as numbers), over the lanes of a wave.
__device__ inline unsigned long long wave_max_bits(unsigned long long u, int from)
{
    for (int o = from; o < 64; o *= 2) {
        const unsigned long long v = __shfl_xor(u, o);
        u = v > u ? v : u;
    }
    return u;
}

// One pass over a strip of 64 rows of A or B (one wave, one row per lane):
//   - NormInf (Section 1.4): each lane sums |x| along its row in order from
//     0.0, as the sequential definition does; the largest row sum of the
//     wave goes to the job's norm by an atomic max (NORMS only);
//   - A: max_k |A_ik| of each row to rmax (before any 2^lambda scaling);
//   - B: max_k |B_kj| of each column over the strip's rows, folded into
//     cmax by an atomic max (cleared beforehand).
// Rows are staged through LDS 16 columns at a time so the loads are
// contiguous 128-byte runs; the next 16 columns are in flight meanwhile.
template <bool NORMS>
__global__ __launch_bounds__(64) void jobs_stats_kernel(const SplitJob* __restrict__ jobs,
                                                        const JobBlock* __restrict__ strips)
{
    __shared__ double T[kStatRows][17];
    const JobBlock st = strips[blockIdx.x];
    const SplitJob& j = jobs[st.job];
    const int lane = threadIdx.x;
    const bool side_b = st.side != 0;
    const double* X = side_b ? j.B : j.A;
    const i64 rows = side_b ? j.P : j.N, len = side_b ? j.M : j.P, r0 = st.index;
    double sum = 0.0, mx = 0.0, r[16];
    // the next 16 columns are loaded while this block of them is folded
    auto load = [&](i64 c0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int rr = q * 4 + lane / 16, cc = lane % 16;
            const i64 gr = r0 + rr, gc = c0 + cc;
            r[q] = (gr < rows && gc < len) ? X[gr * len + gc] : 0.0;
        }
    };
    load(0);
    for (i64 c0 = 0; c0 < len; c0 += 16) {
#pragma unroll
        for (int q = 0; q < 16; ++q) T[q * 4 + lane / 16][lane % 16] = fabs(r[q]);
        __syncthreads();
        if (c0 + 16 < len) load(c0 + 16);
        const int cnt = len - c0 < 16 ? (int)(len - c0) : 16;
        for (int x = 0; x < cnt; ++x) {
            const double v = T[lane][x];
            if (NORMS) sum = sum + v;
            mx = max_s13(mx, v);
        }
        if (side_b) {
            const int cc = lane % 16, g = lane / 16;
            double m = 0.0;
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) m = max_s13(m, T[g * 16 + rr][cc]);
            const unsigned long long u = wave_max_bits((unsigned long long)__double_as_longlong(m), 16);
            if (lane < 16 && c0 + lane < len) atomicMax(reinterpret_cast<unsigned long long*>(&j.cmax[c0 + lane]), u);
        }
        __syncthreads();
    }
    const bool live = r0 + lane < rows;
    if (!side_b && live) j.rmax[r0 + lane] = mx;
    if (NORMS) {
        const unsigned long long u = wave_max_bits(live ? (unsigned long long)__double_as_longlong(sum) : 0ull, 1);
        if (lane == 0) atomicMax(reinterpret_cast<unsigned long long*>(side_b ? j.nB : j.nA), u);
    }
}

__global__ void jobs_lambda_kernel(const SplitJob* jobs, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const double a = *jobs[i].nA, b = *jobs[i].nB;
        int res = 0;
        if (a > 0.0 && b > 0.0 && !isinf(a) && !isinf(b)) {
            int eA, eB;
            const double fa = frexp(a, &eA);
            const double fb = frexp(b, &eB);
            const long long d = (long long)eB - (long long)eA;
            const long long x = fb >= fa ? d + 1 : d;
            res = (int)(x >= 0 ? x / 2 : -((-x + 1) / 2));
        }
        *jobs[i].lam = res;
    }
}

// Digits of every job of a group in one launch: workgroups below na take
// an entry of the A table (a range of one job's (row, 8-entry chunk)
// pairs), the rest an entry of the B table (one 64 x kBJ tile of a job's B).
template <int DT>
__global__ __launch_bounds__(256) void jobs_split_ab_kernel(const SplitJob* __restrict__ jobs,
                                                            const JobBlock* __restrict__ ablocks, i64 na,
                                                            const JobBlock* __restrict__ bblocks, int beta,
                                                            bool scaled)
{
    __shared__ double T[64][kBJ + 1];
    const i64 w = blockIdx.x;
    if (w < na) {
        const JobBlock b = ablocks[w];
        const SplitJob& j = jobs[b.job];
        split_a_body<DT>(j.A, j.N, j.P, j.Np, j.Kp, j.rmax, scaled ? j.lam : nullptr, j.s, beta, j.SA, j.ea, b.index,
                         split_a_blocks(j), true);
    } else {
        const JobBlock b = bblocks[w - na];
        const SplitJob& j = jobs[b.job];
        split_b_body<DT>(j.B, j.P, j.M, j.Mp, j.Kp, j.cmax, scaled ? j.lam : nullptr, j.s, beta, j.SB, j.fb, b.index,
                         T, true);
    }
}

struct SplitLayout {
    int dt = 0, s = 0, beta = 0, unit = 0, runlen = 1;
    bool flush = false;
    i64 Np = 0, Mp = 0, Kp = 0;
    size_t nA = 0, nB = 0, lam = 0, rmax = 0, cmax = 0, ea = 0, fb = 0, SA = 0, SB = 0, bytes = 0;
};

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// the LDS stages of the A digit planes (S x BM rows x 64 bytes each)
size_t split_lds_bytes(const TileCfg& tc, int s) { return (size_t)tc.stages * s * tc.bm() * KB; }

// Exact-accumulation budget: digit products are at most 2^(2 beta - 2) in
// magnitude, so one digit pair's products may be summed over
// budget / 2^(2 beta - 2) entries of K, i.e. this many MFMA k-steps, before
// a partial sum could leave the accumulator's exact range (FP32: 2^24;
// INT32: 2^31 - 1).  A group of p pairs gets unit / p steps; the fullest
// group holds s pairs, so a digit count needs unit / s >= 1.
// Run length of the recombination (step 5): the largest of 3, 2, 1 for
// which every run of consecutive groups, from the finest, keeps its
// worst-case exact sum within 2^53.  Group g (0-based) holds g + 1 digit
// pairs, each product at most 2^(2 beta - 2), summed over P entries; inside
// a run group g is weighted by 2^(beta (f - g)), f the run's finest group.
int split_run_length(int s, int beta, i64 P)
{
    for (int L = 3; L >= 2; --L) {
        bool ok = true;
        for (int f = s - 1; f >= 0 && ok; f -= L) {
            unsigned __int128 worst = 0;
            for (int g = f; g > f - L && g >= 0; --g)
                worst += ((unsigned __int128)(g + 1) * (unsigned __int128)P) << (2 * beta - 2 + beta * (f - g));
            ok = worst <= ((unsigned __int128)1 << 53);
        }
        if (ok) return L;
    }
    return 1;
}

int flush_unit(int dt, int beta)
{
    const double prod = ldexp(1.0, 2 * beta - 2);
    const double budget = dt == DT_INT8   ? Digit<DT_INT8>::budget
                          : dt == DT_FP16 ? Digit<DT_FP16>::budget
                                          : Digit<DT_BF16>::budget;
    const int mk = dt == DT_INT8   ? Digit<DT_INT8>::mfma_k
                   : dt == DT_FP16 ? Digit<DT_FP16>::mfma_k
                                   : Digit<DT_BF16>::mfma_k;
    const double steps = budget / prod / mk;
    return steps >= 1e9 ? 1000000000 : (int)steps;
}

bool split_layout(i64 N, i64 P, i64 M, const mmm_config& c, SplitLayout& L)
{
    L.dt = c.split_type;
    L.s = c.split_slices;
    L.beta = beta_of(L.dt, c.split_bits);
    L.unit = flush_unit(L.dt, L.beta);
    if (L.unit / L.s < 1) return false;
    const int es = L.dt == DT_INT8 ? 1 : 2;
    const int mk = L.dt == DT_INT8 ? Digit<DT_INT8>::mfma_k : Digit<DT_BF16>::mfma_k;
    L.Kp = cdiv(P, KT) * KT;
    L.flush = L.unit / L.s < L.Kp / mk;
    L.runlen = split_run_length(L.s, L.beta, P);
    const TileCfg tc = tile_cfg(L.dt, L.s, L.flush);
    // 16-bit digits with flushing may run the LDS kernel: pad for both tiles
    // (all tile sides are powers of two)
    const int pm = L.dt != DT_INT8 && L.flush && tc.bm() < kLds2BM ? kLds2BM : tc.bm();
    const int pn = L.dt != DT_INT8 && L.flush && tc.bn() < kLds2BN ? kLds2BN : tc.bn();
    L.Np = cdiv(N, pm) * pm;
    L.Mp = cdiv(M, pn) * pn;
    const double sa = (double)L.Np * L.Kp * L.s * es, sb = (double)L.Mp * L.Kp * L.s * es;
    if (sa + sb > 4.0e18) return false;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = al(off + bytes);
        return at;
    };
    L.nA = take(8);
    L.nB = take(8);
    L.lam = take(4);
    L.rmax = take(8 * (size_t)N);
    L.cmax = take(8 * (size_t)M);
    L.ea = take(4 * (size_t)L.Np);
    L.fb = take(4 * (size_t)L.Mp);
    L.SA = take((size_t)sa);
    L.SB = take((size_t)sb);
    L.bytes = off;
    return true;
}

template <int DT, int S, int BETA>
hipError_t launch_split_lds2(const SplitLayout& L, char* ws, double* C, i64 N, i64 M, hipStream_t st)
{
    const i64 tiles_m = L.Np / kLds2BM, tiles_n = L.Mp / kLds2BN;
    const i64 blocks = tiles_m * tiles_n;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const size_t lds = (size_t)MMM_SPLIT_LDS2_STAGES * S * (kLds2BM + kLds2BN) * KB;
    auto kern = split_gemm_lds2_kernel<DT, S, BETA>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kLds2Threads), lds, st, (const char*)(ws + L.SA),
                       (const char*)(ws + L.SB), (const int*)(ws + L.ea), (const int*)(ws + L.fb), C, N, M, L.Np, L.Mp,
                       L.Kp, tiles_m, tiles_n);
    return hipGetLastError();
}

template <int DT, int S, bool FLUSH>
hipError_t launch_split_gemm(const SplitLayout& L, char* ws, double* C, i64 N, i64 M, hipStream_t st)
{
    constexpr TileCfg TC = tile_cfg(DT, S, FLUSH);
    const i64 tiles_m = L.Np / TC.bm(), tiles_n = L.Mp / TC.bn();
    const i64 blocks = tiles_m * tiles_n;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const size_t lds = split_lds_bytes(TC, S);
    auto kern = split_gemm_kernel<DT, S, FLUSH>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(TC.threads()), lds, st, (const char*)(ws + L.SA),
                       (const char*)(ws + L.SB), (const int*)(ws + L.ea), (const int*)(ws + L.fb), C, N, M, L.Np, L.Mp,
                       L.Kp, tiles_m, tiles_n, L.beta, L.unit, L.runlen);
    return hipGetLastError();
}

template <int DT, int S>
hipError_t dispatch_flush(const SplitLayout& L, char* ws, double* C, i64 N, i64 M, hipStream_t st)
{
    if (L.unit / S < 1) return hipErrorNotSupported;
    if (!L.flush) return launch_split_gemm<DT, S, false>(L, ws, C, N, M, st);
#if MMM_SPLIT_LDS2
    // 16-bit digits, 4 or 5 of them, recombined in runs of three: the 64 x 64 LDS kernel
    if constexpr (DT != DT_INT8 && (S == 4 || S == 5)) {
        if (L.runlen == 3 && L.beta == 9) return launch_split_lds2<DT, S, 9>(L, ws, C, N, M, st);
        if (L.runlen == 3 && L.beta == 8) return launch_split_lds2<DT, S, 8>(L, ws, C, N, M, st);
    }
#endif
    return launch_split_gemm<DT, S, true>(L, ws, C, N, M, st);
}

template <int DT>
hipError_t dispatch_s(const SplitLayout& L, char* ws, double* C, i64 N, i64 M, hipStream_t st)
{
    switch (L.s) {
    case 1: return dispatch_flush<DT, 1>(L, ws, C, N, M, st);
    case 2: return dispatch_flush<DT, 2>(L, ws, C, N, M, st);
    case 3: return dispatch_flush<DT, 3>(L, ws, C, N, M, st);
    case 4: return dispatch_flush<DT, 4>(L, ws, C, N, M, st);
    case 5: return dispatch_flush<DT, 5>(L, ws, C, N, M, st);
    case 6: return dispatch_flush<DT, 6>(L, ws, C, N, M, st);
    case 7: return dispatch_flush<DT, 7>(L, ws, C, N, M, st);
    case 8: return dispatch_flush<DT, 8>(L, ws, C, N, M, st);
    default: return hipErrorNotSupported;
    }
}

template <int DT>
hipError_t run_split_dt(const double* A, const double* B, double* C, i64 N, i64 P, i64 M, const SplitLayout& L,
                        bool scale, char* ws, hipStream_t st)
{
    hipError_t e;
    int* lam = scale ? (int*)(ws + L.lam) : nullptr;
    double* nA = (double*)(ws + L.nA);
    double* nB = (double*)(ws + L.nB);
    double* rmax = (double*)(ws + L.rmax);
    double* cmax = (double*)(ws + L.cmax);
    // one pass per operand, both in one launch: A's norm and row maxima, B's
    // norm and column maxima (the maxima before the 2^lambda scaling, which
    // the digit pass applies when it forms the exponents).  B's
    // per-workgroup column maxima (cdiv(P, 16) x M doubles, at most half of
    // B's digit planes) are staged in the digit-plane region, which the
    // digit pass overwrites only afterwards.
    const i64 nparts = cdiv(P, RV);
    double* cpart = (double*)(ws + L.SB);
    if (scale && (e = launch_fill_zero(nA, 1, st)) != hipSuccess) return e;
    if (scale && (e = launch_fill_zero(nB, 1, st)) != hipSuccess) return e;
    const i64 nblk_a = cdiv(N, RV);
    if (nblk_a + nparts > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    if (scale)
        hipLaunchKernelGGL(stats_pair_kernel<true>, dim3((unsigned)(nblk_a + nparts)), dim3(256), 0, st, A, N, P, nA,
                           rmax, nblk_a, B, M, nB, cpart);
    else
        hipLaunchKernelGGL(stats_pair_kernel<false>, dim3((unsigned)(nblk_a + nparts)), dim3(256), 0, st, A, N, P,
                           nullptr, rmax, nblk_a, B, M, nullptr, cpart);
    hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)cdiv(M, 32)), dim3(256), 0, st, cpart, nparts, M, cmax);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (scale && (e = launch_lambda(nA, nB, lam, st)) != hipSuccess) return e;
    {
        i64 blk_a = cdiv(L.Np * (L.Kp / 8), 256);
        if (blk_a > 256 * 64) blk_a = 256 * 64;
        const i64 blk_b = (L.Kp / 64) * (L.Mp / kBJ);
        if (blk_a + blk_b > 0x7fffffffLL) return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL((split_ab_kernel<DT>), dim3((unsigned)(blk_a + blk_b)), dim3(256), 0, st, A, N, P, L.Np,
                           L.Kp, rmax, lam, L.s, L.beta, ws + L.SA, (int*)(ws + L.ea), blk_a, B, M, L.Mp, cmax,
                           ws + L.SB,
                           (int*)(ws + L.fb));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    timer_begin(st);
    e = dispatch_s<DT>(L, ws, C, N, M, st);
    timer_end(st);
    return e;
}

template <int DT, int S, bool FLUSH, int V, int PPA>
hipError_t launch_grouped_gemm(const SplitJob* jobs, const i64* prefix, int n, int beta, int unit, int grid,
                               TileSchedule sch, hipStream_t st)
{
    constexpr TileCfg TC = grouped_tile_cfg(DT, S, FLUSH, V, PPA);
    const size_t lds = split_lds_bytes(TC, S);
    auto kern = split_gemm_grouped_kernel<DT, S, FLUSH, V, PPA>;
    if (!jobs) return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(TC.threads()), lds, st, jobs, prefix, n, beta, unit, sch);
    return hipGetLastError();
}

template <int DT, int S, bool FLUSH, int PPA>
hipError_t grouped_variant(const SplitGroup& g, const SplitJob* jobs, const i64* prefix, int n, int grid,
                           TileSchedule sch, hipStream_t st)
{
    if (g.variant == 1) return launch_grouped_gemm<DT, S, FLUSH, 1, PPA>(jobs, prefix, n, g.beta, g.unit, grid, sch, st);
    return launch_grouped_gemm<DT, S, FLUSH, 0, PPA>(jobs, prefix, n, g.beta, g.unit, grid, sch, st);
}

template <int DT, int S>
hipError_t grouped_flush(const SplitGroup& g, const SplitJob* jobs, const i64* prefix, int n, int grid,
                         TileSchedule sch, hipStream_t st)
{
    if (g.flush) return grouped_variant<DT, S, true, S>(g, jobs, prefix, n, grid, sch, st);
    // pair-subgroup accumulators: 16-bit digits only (int8 never needs them)
    if constexpr (DT != DT_INT8 && S > 2) {
        if (g.ppa == 2) return grouped_variant<DT, S, false, 2>(g, jobs, prefix, n, grid, sch, st);
        if (g.ppa == 1) return grouped_variant<DT, S, false, 1>(g, jobs, prefix, n, grid, sch, st);
    }
    return grouped_variant<DT, S, false, S>(g, jobs, prefix, n, grid, sch, st);
}

template <int DT>
hipError_t grouped_s(const SplitGroup& g, const SplitJob* jobs, const i64* prefix, int n, int grid, TileSchedule sch,
                     hipStream_t st)
{
    switch (g.s) {
    case 1: return grouped_flush<DT, 1>(g, jobs, prefix, n, grid, sch, st);
    case 2: return grouped_flush<DT, 2>(g, jobs, prefix, n, grid, sch, st);
    case 3: return grouped_flush<DT, 3>(g, jobs, prefix, n, grid, sch, st);
    case 4: return grouped_flush<DT, 4>(g, jobs, prefix, n, grid, sch, st);
    case 5: return grouped_flush<DT, 5>(g, jobs, prefix, n, grid, sch, st);
    case 6: return grouped_flush<DT, 6>(g, jobs, prefix, n, grid, sch, st);
    case 7: return grouped_flush<DT, 7>(g, jobs, prefix, n, grid, sch, st);
    case 8: return grouped_flush<DT, 8>(g, jobs, prefix, n, grid, sch, st);
    default: return hipErrorNotSupported;
    }
}

template <int DT>
hipError_t launch_split_prep_dt(const SplitJob* jobs, int n, const SplitTables& tab, bool scale, int beta,
                                hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipError_t e;
    const dim3 blk(256);
    hipLaunchKernelGGL(jobs_zero_stats_kernel, dim3((unsigned)n), blk, 0, st, jobs);
    if (tab.nstrips > 0) {
        if (scale)
            hipLaunchKernelGGL(jobs_stats_kernel<true>, dim3((unsigned)tab.nstrips), dim3(64), 0, st, jobs, tab.strips);
        else
            hipLaunchKernelGGL(jobs_stats_kernel<false>, dim3((unsigned)tab.nstrips), dim3(64), 0, st, jobs, tab.strips);
    }
    if (scale) hipLaunchKernelGGL(jobs_lambda_kernel, dim3((unsigned)cdiv(n, 256)), blk, 0, st, jobs, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const i64 nab = (i64)tab.nablocks + tab.nbblocks;
    if (nab > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    if (nab > 0)
        hipLaunchKernelGGL(jobs_split_ab_kernel<DT>, dim3((unsigned)nab), blk, 0, st, jobs,
                           tab.ablocks, (i64)tab.nablocks, tab.bblocks, beta, scale);
    return hipGetLastError();
}

}  // namespace

size_t split_workspace_bytes(i64 N, i64 P, i64 M, const mmm_config& c)
{
    SplitLayout L;
    if (!split_layout(N, P, M, c, L)) return (size_t)-1;
    return L.bytes;
}

hipError_t run_split(const double* A, const double* B, double* C, i64 N, i64 P, i64 M, const mmm_config& c,
                     char* ws, hipStream_t s)
{
    SplitLayout L;
    if (!split_layout(N, P, M, c, L)) return hipErrorNotSupported;
    const bool scale = c.split_scale_lambda != 0;
    switch (c.split_type) {
    case DT_BF16: return run_split_dt<DT_BF16>(A, B, C, N, P, M, L, scale, ws, s);
    case DT_FP16: return run_split_dt<DT_FP16>(A, B, C, N, P, M, L, scale, ws, s);
    case DT_INT8: return run_split_dt<DT_INT8>(A, B, C, N, P, M, L, scale, ws, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace mmm

namespace mmm {

size_t split_job_bytes(i64 N, i64 P, i64 M, int dt, int s, int bits, int variant, SplitGroup& grp, i64& Np,
                       i64& Mp, i64& Kp)
{
    mmm_config c = mmm_config_default();
    c.split_type = dt;
    c.split_slices = s;
    c.split_bits = bits;
    SplitLayout L;
    if (!split_layout(N, P, M, c, L)) return (size_t)-1;
    // K too long for a whole group per accumulator but short enough for two
    // pairs (or one) of 16-bit digits: pair-subgroup accumulators instead of
    // flushing (the tiles of a batch have short K)
    grp.ppa = s;
    grp.flush = L.flush;
    if (L.flush && dt != DT_INT8 && s > 2) {
        const i64 steps = L.Kp / Digit<DT_BF16>::mfma_k;
        if (2 * steps <= L.unit) grp.ppa = 2, grp.flush = false;
        else if (steps <= L.unit) grp.ppa = 1, grp.flush = false;
    }
    const TileCfg tc = grouped_tile_cfg(dt, s, grp.flush, variant, grp.ppa);
    grp.dt = dt;
    grp.s = s;
    grp.beta = L.beta;
    grp.unit = L.unit;
    grp.variant = variant;
    grp.bm = tc.bm();
    grp.bn = tc.bn();
    grp.per_cu = tc.minw * 4 / tc.nw > 0 ? tc.minw * 4 / tc.nw : 1;
    Np = L.Np;
    Mp = L.Mp;
    Kp = L.Kp;
    return L.bytes;
}

void split_job_bind(SplitJob& j, char* base, int dt, int s, int bits)
{
    j.s = s;
    mmm_config c = mmm_config_default();
    c.split_type = dt;
    c.split_slices = s;
    c.split_bits = bits;
    SplitLayout L;
    split_layout(j.N, j.P, j.M, c, L);
    j.runlen = L.runlen;
    j.Np = L.Np;
    j.Mp = L.Mp;
    j.Kp = L.Kp;
    j.nA = (double*)(base + L.nA);
    j.nB = (double*)(base + L.nB);
    j.lam = (int*)(base + L.lam);
    j.rmax = (double*)(base + L.rmax);
    j.cmax = (double*)(base + L.cmax);
    j.ea = (int*)(base + L.ea);
    j.fb = (int*)(base + L.fb);
    j.SA = base + L.SA;
    j.SB = base + L.SB;
}

hipError_t split_grouped_prepare(const SplitGroup& g)
{
    // a null job table only sets the kernel's dynamic LDS limit
    switch (g.dt) {
    case DT_BF16: return grouped_s<DT_BF16>(g, nullptr, nullptr, 0, 0, TileSchedule{nullptr, nullptr, 0}, nullptr);
    case DT_FP16: return grouped_s<DT_FP16>(g, nullptr, nullptr, 0, 0, TileSchedule{nullptr, nullptr, 0}, nullptr);
    case DT_INT8: return grouped_s<DT_INT8>(g, nullptr, nullptr, 0, 0, TileSchedule{nullptr, nullptr, 0}, nullptr);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_split_prep(int dt, int beta, const SplitJob* jobs, int n, const SplitTables& tab, bool scale_lambda,
                             hipStream_t s)
{
    switch (dt) {
    case DT_BF16: return launch_split_prep_dt<DT_BF16>(jobs, n, tab, scale_lambda, beta, s);
    case DT_FP16: return launch_split_prep_dt<DT_FP16>(jobs, n, tab, scale_lambda, beta, s);
    case DT_INT8: return launch_split_prep_dt<DT_INT8>(jobs, n, tab, scale_lambda, beta, s);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_split_group_gemm(const SplitGroup& grp, const SplitJob* jobs, int n, const i64* prefix,
                                   i64 total_tiles, TileSchedule sched, int grid, hipStream_t s)
{
    if (n <= 0 || total_tiles <= 0) return hipSuccess;
    switch (grp.dt) {
    case DT_BF16: return grouped_s<DT_BF16>(grp, jobs, prefix, n, grid, sched, s);
    case DT_FP16: return grouped_s<DT_FP16>(grp, jobs, prefix, n, grid, sched, s);
    case DT_INT8: return grouped_s<DT_INT8>(grp, jobs, prefix, n, grid, sched, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace mmm
