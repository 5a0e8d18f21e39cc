// Inner-product methods of Section 2 on the FP64 vector ALUs of gfx950:
// NaivStandard (2.1.1), NaivOnArray (2.1.2), NaivKahan (2.1.3),
// NaivLoopUnrollingTwo/Three/Four (2.2) and the main loop of
// WinogradOriginal (2.3.1, also used by WinogradScaled 2.3.2); beyond the
// paper, compensated dot products (Ogita, Rump and Oishi's Dot2).
//
// Every output entry is owned by one lane, which runs the paper's recurrence
// over k (or over the index pairs) in ascending order.  The file is built
// with -ffp-contract=off, so each product and each sum is rounded on its own
// exactly as the recurrence is written; with the same order this makes the
// results equal bit for bit to a sequential binary64 evaluation.  Only the
// optional fused variant of the naive method calls fma() explicitly.
//
// Tiling: 256 threads (16 x 16) per workgroup own a BM x BN tile of C
// (128 x 64 for the naive and Winograd loops, 64 x 64 for Kahan, whose state
// is two doubles per entry), each thread a TM x TN register block (rows
// ty*TM + i, columns h*BN/2 + tx*TN/2 + j).  K advances in steps of 16 (32
// for Kahan, 24 for groups of three) through LDS.  Two ways to fill LDS:
//   - direct loads (every tile inside the matrices, K a whole number of
//     steps, 16-byte aligned operands with even leading dimensions): each
//     step's A and B tiles go global -> LDS by global_load_lds_dwordx4 (no
//     staging registers) into two stages, the next step's loads in flight
//     while the current one computes.  The A tile keeps the global row-major
//     order with its 16-byte chunks XOR-swizzled per row, so one ds_read_b128
//     returns (A_ik, A_i,k+1) and the rows the 4 thread rows of a wave read
//     fall in distinct banks; the B tile is row-major.
//   - register staging (everything else): each step's tiles are loaded into
//     registers, stored to LDS (A k-major), then used; edge tiles check
//     bounds.
// Within a step each operation of the recurrence is issued for a whole row
// (Winograd) or the whole register block (naive, Kahan) before the next one,
// so the FP64 pipeline sees independent chains; the per-entry order of
// operations, and hence every rounding, is unchanged.
#include <type_traits>

#include "common.h"
#include "launch.h"

// Tile shapes (BM, BN, TM, TN), K steps and occupancy; overridable at build
// time.  Defaults measured on MI355X at 4096^3 (two waves per SIMD).
#ifndef MMM_VALU_NAIVE_TILE
#define MMM_VALU_NAIVE_TILE 128, 64, 8, 4
#endif
#ifndef MMM_VALU_KAHAN_TILE
#define MMM_VALU_KAHAN_TILE 64, 64, 4, 4
#endif
#ifndef MMM_VALU_WINO_TILE
#define MMM_VALU_WINO_TILE 128, 64, 8, 4
#endif
// NaivStandard on the direct-load path: no staging registers, room for an
// 8 x 8 block per thread
#ifndef MMM_VALU_WINO_DMA_TILE
#define MMM_VALU_WINO_DMA_TILE 128, 128, 8, 8
#endif
#ifndef MMM_VALU_NAIVE_DMA_TILE
#define MMM_VALU_NAIVE_DMA_TILE 128, 128, 8, 8
#endif
#ifndef MMM_VALU_MINWAVES
#define MMM_VALU_MINWAVES 2
#endif
#ifndef MMM_VALU_BK
#define MMM_VALU_BK 16
#endif
#ifndef MMM_VALU_KAHAN_BK
#define MMM_VALU_KAHAN_BK 32
#endif
#ifndef MMM_VALU_DMA
#define MMM_VALU_DMA 1
#endif
// waves per SIMD of the direct-load kernels (Kahan: its 64 KiB of LDS per
// workgroup allow two)
#ifndef MMM_VALU_DMA_MINWAVES
#define MMM_VALU_DMA_MINWAVES 2
#endif

namespace mmm {

namespace {

constexpr int NT = 256;

enum Op {
    OP_NAIVE = 0,
    OP_NAIVE_FMA = 1,
    OP_KAHAN = 2,
    OP_WINOGRAD = 3,
    OP_UNROLL2 = 4,  // NaivLoopUnrollingTwo / Three / Four
    OP_UNROLL3 = 5,
    OP_UNROLL4 = 6,
    OP_ON_ARRAY = 7,  // NaivOnArray
    OP_DOT2 = 8       // compensated dot products (TwoProduct + TwoSum), beyond the paper
};
__host__ __device__ constexpr int unroll_q(int op) { return op == OP_UNROLL2 ? 2 : (op == OP_UNROLL3 ? 3 : (op == OP_UNROLL4 ? 4 : 0)); }

__device__ inline i64 xcd_remap(i64 b, i64 total)
{
    // Workgroups are dealt round robin to the 8 XCDs; give each XCD a
    // contiguous range of tiles so that neighbouring tiles share its L2.
    if (total % 8 != 0) return b;
    return (b % 8) * (total / 8) + b / 8;
}

// Tile (tm, tn) of problem `prob` for flattened block b, grouped 8 tile
// rows at a time inside a problem.
__device__ inline void tile_of(i64 b, i64 tiles_m, i64 tiles_n, i64& prob, i64& tm, i64& tn)
{
    const i64 per = tiles_m * tiles_n;
    prob = b / per;
    const i64 r = b - prob * per;
    const i64 G = 8;
    const i64 group = r / (G * tiles_n);
    const i64 first = group * G;
    const i64 gs = (tiles_m - first) < G ? (tiles_m - first) : G;
    const i64 w = r - group * G * tiles_n;
    tm = first + w % gs;
    tn = w / gs;
}

// ---- the arithmetic of one k, one Winograd pair or one unrolled group ------
// for a TM x TN register block.  Each operation is issued for the whole
// block (row for Winograd) before the next; per entry the recurrence and its
// roundings are the paper's.

template <int OP, int TM, int TN>
__device__ __forceinline__ void arith_k(const double (&a)[TM], const double (&b)[TN], double (&acc)[TM][TN],
                                        double (&cmp)[TM][TN])
{
    if constexpr (OP == OP_KAHAN) {
        // Kahan's compensated summation in its classic published form
        // (Higham, Algorithm 4.2): the product x is rounded on its own, the
        // corrected term y = x - c is added, c = (t - sum) - y recovers the
        // rounding error of that addition.  cmp holds c.
        double x[TM][TN], y[TM][TN], t[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) x[i][j] = a[i] * b[j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) y[i][j] = x[i][j] - cmp[i][j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) t[i][j] = acc[i][j] + y[i][j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                cmp[i][j] = (t[i][j] - acc[i][j]) - y[i][j];
                acc[i][j] = t[i][j];
            }
    } else if constexpr (OP == OP_DOT2) {
        // Ogita-Rump-Oishi Dot2: x + y = a b exactly (TwoProduct), s + e =
        // p + x exactly (TwoSum), p = s, q = q + (e + y); the entry is p + q
        double x[TM][TN], s[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) x[i][j] = a[i] * b[j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) s[i][j] = acc[i][j] + x[i][j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const double y = fma(a[i], b[j], -x[i][j]);
                const double z = s[i][j] - acc[i][j];
                const double e = (acc[i][j] - (s[i][j] - z)) + (x[i][j] - z);
                acc[i][j] = s[i][j];
                cmp[i][j] = cmp[i][j] + (e + y);
            }
    } else if constexpr (OP == OP_NAIVE_FMA) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    } else if constexpr (OP == OP_NAIVE) {  // aux = aux + a * b, a row of the block at a time
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            double x[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) x[j] = a[i] * b[j];
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = acc[i][j] + x[j];
        }
    } else {  // NaivOnArray: the same recurrence, the whole block at a time
        double x[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) x[i][j] = a[i] * b[j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = acc[i][j] + x[i][j];
    }
}

// Winograd pair (k, k+1): (A_{i,k} + B_{k+1,j}) (A_{i,k+1} + B_{k,j})
template <int TM, int TN>
__device__ __forceinline__ void arith_pair(const double (&a0)[TM], const double (&a1)[TM], const double (&b0)[TN],
                                           const double (&b1)[TN], double (&acc)[TM][TN])
{
    // half a row of 8 at a time: 8 independent sums per stage, with half the
    // temporaries live (room for the 8 x 8 block's loop without spills)
    constexpr int H = TN > 4 ? TN / 2 : TN;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j0 = 0; j0 < TN; j0 += H) {
            double u[H], v[H], w[H];
#pragma unroll
            for (int j = 0; j < H; ++j) u[j] = a0[i] + b1[j0 + j];
#pragma unroll
            for (int j = 0; j < H; ++j) v[j] = a1[i] + b0[j0 + j];
#pragma unroll
            for (int j = 0; j < H; ++j) w[j] = u[j] * v[j];
#pragma unroll
            for (int j = 0; j < H; ++j) acc[i][j0 + j] = acc[i][j0 + j] + w[j];
        }
}

// a group of Q consecutive k: (p_1 + p_2 (+ p_3 (+ p_4))) left to right,
// then added to the running sum
template <int Q, int TM, int TN>
__device__ __forceinline__ void arith_group(const double (&a)[Q][TM], const double (&b)[Q][TN],
                                            double (&acc)[TM][TN])
{
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        double grp[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) grp[j] = a[0][i] * b[0][j];
#pragma unroll
        for (int r = 1; r < Q; ++r)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const double x = a[r][i] * b[r][j];
                grp[j] = grp[j] + x;
            }
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = acc[i][j] + grp[j];
    }
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

template <int BM, int BN, int TM, int TN, int OP>
struct ValuTile {
    // K per LDS step; a multiple of the group length of the unrolled sums
    static constexpr int BK =
        OP == OP_KAHAN ? MMM_VALU_KAHAN_BK : (OP == OP_UNROLL3 ? 24 : MMM_VALU_BK);
    static constexpr int Q = unroll_q(OP);
    static_assert((BM / TM) * (BN / TN) == NT, "256 threads");
    static_assert(BM / TM == 16 && BN / TN == 16, "16 x 16 thread grid");
    static_assert((BM * BK) % NT == 0 && (BK * BN) % NT == 0, "every thread moves whole elements of a step");
    static constexpr int LA = BM * BK / NT;  // A elements each thread moves per step (register staging)
    static constexpr int LB = BK * BN / NT;
    static constexpr int TH = TN / 2;        // columns per half
    static constexpr int KSTEP = (OP == OP_WINOGRAD) ? 2 : (Q ? Q : 1);
    // the grouped part of the k range (the rest is added in the epilogue)
    __host__ __device__ static i64 kmax_of(i64 P) { return (OP == OP_WINOGRAD) ? 2 * (P / 2) : (Q ? Q * (P / Q) : P); }

    // direct loads: 16-byte chunks per A row, KiB blocks of A and B per step
    static constexpr int CH = BK / 2;
    static constexpr int NA = BM * BK / 128, NB = BK * BN / 128;
    static constexpr bool DMA_OK = TN % 4 == 0 && (CH & (CH - 1)) == 0 && NA % 4 == 0 && NB % 4 == 0 && Q != 3;

    struct SmemReg {
        double As[BK][BM + 2];
        double Bs[BK][BN + 2];
    };
    struct SmemDma {
        double A[2][BM * BK];  // row-major, chunk c of row r in slot c ^ swz(r)
        double B[2][BK * BN];  // row-major
    };

    __device__ __forceinline__ static int swz(int r) { return (r / TM) & (CH - 1); }
    // Slot of 16-byte chunk c in a B row (direct loads).  At 4 columns per
    // thread and half, the 16 threads of a row read every other chunk, 32
    // bytes apart; flipping the low bit of the chunks in odd blocks of 16
    // puts those reads on all 16 bank groups.
    __device__ __forceinline__ static int bslot(int c) { return TH % 4 == 0 ? c ^ ((c >> 4) & 1) : c; }

    // NaivOnArray: the running sum lives in the entries of C; every K step
    // reads them and writes them back (the first step starts from the zeroed
    // entries)
    template <bool CHECK>
    __device__ __forceinline__ static void c_io(const Gemm& g, i64 m0, i64 n0, bool store, double (&acc)[TM][TN])
    {
        if constexpr (OP == OP_ON_ARRAY) {
            const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const i64 gm = m0 + ty * TM + i;
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int j = 0; j < TH; ++j) {
                        const i64 gn = n0 + h * (BN / 2) + tx * TH + j;
                        if (CHECK && (gm >= g.N || gn >= g.M)) continue;
                        if (store) g.C[gm * g.ldc + gn] = acc[i][h * TH + j];
                        else acc[i][h * TH + j] = g.C[gm * g.ldc + gn];
                    }
            }
        }
    }

    // Register staging.  CHECK: bounds-check every load (edge tiles);
    // otherwise only the last K step is checked.
    template <bool CHECK>
    __device__ __forceinline__ static void mainloop_reg(const Gemm& g, i64 m0, i64 n0, i64 kmax, SmemReg& sm,
                                                        double (&acc)[TM][TN], double (&cmp)[TM][TN])
    {
        const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
        const i64 ntiles = (kmax + BK - 1) / BK;
        double ra[LA], rb[LB];
        auto gload = [&](i64 t, bool check) __attribute__((always_inline)) {
            const i64 k0 = t * BK;
#pragma unroll
            for (int q = 0; q < LA; ++q) {
                const int e = q * NT + tid, r = e / BK, k = e % BK;
                const i64 gm = m0 + r, gk = k0 + k;
                if (check) ra[q] = (gm < g.N && gk < kmax) ? g.A[gm * g.lda + gk] : 0.0;
                else ra[q] = g.A[gm * g.lda + gk];
            }
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                const int e = q * NT + tid, k = e / BN, n = e % BN;
                const i64 gk = k0 + k, gn = n0 + n;
                if (check) rb[q] = (gk < kmax && gn < g.M) ? g.B[gk * g.ldb + gn] : 0.0;
                else rb[q] = g.B[gk * g.ldb + gn];
            }
        };
        auto lstore = [&]() __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < LA; ++q) {
                const int e = q * NT + tid;
                sm.As[e % BK][e / BK] = ra[q];
            }
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                const int e = q * NT + tid;
                sm.Bs[e / BN][e % BN] = rb[q];
            }
        };
        auto frag_a = [&](int k, double(&a)[TM]) __attribute__((always_inline)) {
            if constexpr (TM % 2 == 0) {
#pragma unroll
                for (int i = 0; i < TM; i += 2) {
                    const double2 v = *reinterpret_cast<const double2*>(&sm.As[k][ty * TM + i]);
                    a[i] = v.x;
                    a[i + 1] = v.y;
                }
            } else {
                // one row per lane (the 16 x 32 latency tile): no pairs to read
#pragma unroll
                for (int i = 0; i < TM; ++i) a[i] = sm.As[k][ty * TM + i];
            }
        };
        auto frag_b = [&](int k, double(&b)[TN]) __attribute__((always_inline)) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (TH % 2 == 0) {
#pragma unroll
                    for (int j = 0; j < TH; j += 2) {
                        const double2 v = *reinterpret_cast<const double2*>(&sm.Bs[k][h * (BN / 2) + tx * TH + j]);
                        b[h * TH + j] = v.x;
                        b[h * TH + j + 1] = v.y;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < TH; ++j) b[h * TH + j] = sm.Bs[k][h * (BN / 2) + tx * TH + j];
                }
            }
        };
        auto step = [&](int k) __attribute__((always_inline)) {
            if constexpr (OP == OP_WINOGRAD) {
                double a0[TM], a1[TM], b0[TN], b1[TN];
                frag_a(k, a0);
                frag_a(k + 1, a1);
                frag_b(k, b0);
                frag_b(k + 1, b1);
                arith_pair<TM, TN>(a0, a1, b0, b1, acc);
            } else if constexpr (Q != 0) {
                double a[Q][TM], b[Q][TN];
#pragma unroll
                for (int r = 0; r < Q; ++r) {
                    frag_a(k + r, a[r]);
                    frag_b(k + r, b[r]);
                }
                arith_group<Q, TM, TN>(a, b, acc);
            } else {
                double a[TM], b[TN];
                frag_a(k, a);
                frag_b(k, b);
                arith_k<OP, TM, TN>(a, b, acc, cmp);
            }
        };
        auto compute = [&](i64 t) __attribute__((always_inline)) {
            const i64 rem = kmax - t * BK;
            if (rem >= BK) {
#pragma unroll
                for (int k = 0; k < BK; k += KSTEP) step(k);
            } else {
                const int kc = (int)rem;
                for (int k = 0; k < kc; k += KSTEP) step(k);
            }
        };
        if (OP == OP_ON_ARRAY) c_io<CHECK>(g, m0, n0, true, acc);  // C = 0
        for (i64 t = 0; t < ntiles; ++t) {
            gload(t, CHECK || (t + 1) * BK > kmax);
            __syncthreads();  // the previous step's reads of the buffer are done
            lstore();
            __syncthreads();
            c_io<CHECK>(g, m0, n0, false, acc);
            compute(t);
            c_io<CHECK>(g, m0, n0, true, acc);
        }
    }

    // Direct loads (host has checked: tile inside the matrices, kmax a
    // multiple of BK, aligned operands with even leading dimensions).
    template <bool PART>
    __device__ __forceinline__ static void mainloop_dma(const Gemm& g, i64 m0, i64 n0, i64 kmax, SmemDma& sm,
                                                        double (&acc)[TM][TN], double (&cmp)[TM][TN])
    {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, tx = tid % 16, ty = tid / 16;
        // PART: a partial last step, whose loads read zero-padded operands
        // (host-checked); otherwise kmax is a whole number of steps
        const i64 nt = PART ? (kmax + BK - 1) / BK : kmax / BK;
        // lane l of a wave instruction writes LDS bytes 16 l .. 16 l + 15 of
        // its KiB block; it fetches the global chunk that belongs there.
        // Per-lane element offsets from the tile's corner are 32-bit (host-
        // checked), the corner itself wave-uniform, so no 64-bit per-lane
        // addresses stay live across the loop.
        unsigned offa[NA / 4], offb[NB / 4];
#pragma unroll
        for (int q = 0; q < NA / 4; ++q) {
            const int p = (q * 4 + wave) * 64 + lane;
            const int r = p / CH, c = (p % CH) ^ swz(r);
            offa[q] = (unsigned)(r * g.lda + 2 * c);
        }
#pragma unroll
        for (int q = 0; q < NB / 4; ++q) {
            const int p = (q * 4 + wave) * 64 + lane;
            const int r = p / (BN / 2), c = bslot(p % (BN / 2));
            offb[q] = (unsigned)(r * g.ldb + 2 * c);
        }
        const double* a_corner = g.A + m0 * g.lda;
        const double* b_corner = g.B + n0;
        auto issue = [&](i64 t, int buf) __attribute__((always_inline)) {
            const i64 k0 = t * BK;
            const double* a0 = a_corner + k0;
            const double* b0 = b_corner + k0 * g.ldb;
#pragma unroll
            for (int q = 0; q < NA / 4; ++q)
                __builtin_amdgcn_global_load_lds((gbl_ptr_t)(a0 + offa[q]), (lds_ptr_t)&sm.A[buf][(q * 4 + wave) * 128],
                                                 16, 0, 0);
#pragma unroll
            for (int q = 0; q < NB / 4; ++q)
                __builtin_amdgcn_global_load_lds((gbl_ptr_t)(b0 + offb[q]), (lds_ptr_t)&sm.B[buf][(q * 4 + wave) * 128],
                                                 16, 0, 0);
        };
        // operands of k = 2 kp and 2 kp + 1
        auto frag_pair = [&](int buf, int kp, double(&a0)[TM], double(&a1)[TM], double(&b0)[TN],
                             double(&b1)[TN]) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int r = ty * TM + i;
                const double2 v = *reinterpret_cast<const double2*>(&sm.A[buf][r * BK + 2 * (kp ^ swz(r))]);
                a0[i] = v.x;
                a1[i] = v.y;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int j = 0; j < TH; j += 2) {
                    const int col = 2 * bslot((h * (BN / 2) + tx * TH + j) / 2);
                    const double2 v0 = *reinterpret_cast<const double2*>(&sm.B[buf][(2 * kp) * BN + col]);
                    const double2 v1 = *reinterpret_cast<const double2*>(&sm.B[buf][(2 * kp + 1) * BN + col]);
                    b0[h * TH + j] = v0.x;
                    b0[h * TH + j + 1] = v0.y;
                    b1[h * TH + j] = v1.x;
                    b1[h * TH + j + 1] = v1.y;
                }
        };
        auto compute = [&](int buf) __attribute__((always_inline)) {
            if constexpr (Q == 4) {
#pragma unroll
                for (int kp = 0; kp < BK / 2; kp += 2) {
                    double a[4][TM], b[4][TN];
                    frag_pair(buf, kp, a[0], a[1], b[0], b[1]);
                    frag_pair(buf, kp + 1, a[2], a[3], b[2], b[3]);
                    arith_group<4, TM, TN>(a, b, acc);
                }
            } else {
#pragma unroll
                for (int kp = 0; kp < BK / 2; ++kp) {
                    double a[2][TM], b[2][TN];
                    frag_pair(buf, kp, a[0], a[1], b[0], b[1]);
                    if constexpr (OP == OP_WINOGRAD) {
                        arith_pair<TM, TN>(a[0], a[1], b[0], b[1], acc);
                    } else if constexpr (Q == 2) {
                        arith_group<2, TM, TN>(a, b, acc);
                    } else {
                        arith_k<OP, TM, TN>(a[0], b[0], acc, cmp);
                        arith_k<OP, TM, TN>(a[1], b[1], acc, cmp);
                    }
                }
            }
        };
        // the last step when K is not a whole number of steps: kc < BK
        // entries (a multiple of the group length; Winograd: even)
        auto compute_part = [&](int buf, int kc) __attribute__((always_inline)) {
            if constexpr (Q == 4) {
                for (int kp = 0; kp < kc / 2; kp += 2) {
                    double a[4][TM], b[4][TN];
                    frag_pair(buf, kp, a[0], a[1], b[0], b[1]);
                    frag_pair(buf, kp + 1, a[2], a[3], b[2], b[3]);
                    arith_group<4, TM, TN>(a, b, acc);
                }
            } else {
                for (int kp = 0; kp < kc / 2; ++kp) {
                    double a[2][TM], b[2][TN];
                    frag_pair(buf, kp, a[0], a[1], b[0], b[1]);
                    if constexpr (OP == OP_WINOGRAD) {
                        arith_pair<TM, TN>(a[0], a[1], b[0], b[1], acc);
                    } else if constexpr (Q == 2) {
                        arith_group<2, TM, TN>(a, b, acc);
                    } else {
                        arith_k<OP, TM, TN>(a[0], b[0], acc, cmp);
                        arith_k<OP, TM, TN>(a[1], b[1], acc, cmp);
                    }
                }
                if constexpr (OP != OP_WINOGRAD && Q == 0) {
                    if (kc & 1) {
                        double a[2][TM], b[2][TN];
                        frag_pair(buf, kc / 2, a[0], a[1], b[0], b[1]);
                        arith_k<OP, TM, TN>(a[0], b[0], acc, cmp);
                    }
                }
            }
        };
        if (OP == OP_ON_ARRAY) c_io<false>(g, m0, n0, true, acc);  // C = 0
        // whole steps first (the same loop as without a partial step), then
        // the partial one
        const i64 nfull = kmax / BK;
        if (nt > 0) issue(0, 0);
        for (i64 t = 0; t < nfull; ++t) {
            const int cur = (int)(t & 1);
            // own loads of this step have landed; after the barrier every
            // wave's have, and every wave is done with the other stage
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (t + 1 < nt) issue(t + 1, cur ^ 1);
            c_io<false>(g, m0, n0, false, acc);
            compute(cur);
            c_io<false>(g, m0, n0, true, acc);
        }
        if constexpr (PART) {
            if (nfull < nt) {
                const int cur = (int)(nfull & 1);
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                c_io<false>(g, m0, n0, false, acc);
                compute_part(cur, (int)(kmax - nfull * BK));
                c_io<false>(g, m0, n0, true, acc);
            }
        }
    }

    // MODE 0: register staging; 1: direct loads, whole K steps; 2: direct
    // loads with a partial last step
    template <int MODE>
    __device__ __forceinline__ static void run(const Gemm& g, i64 tm, i64 tn, const double* __restrict__ yv,
                                               const double* __restrict__ zv,
                                               typename std::conditional<MODE != 0, SmemDma, SmemReg>::type& sm)
    {
        const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
        const i64 m0 = tm * BM, n0 = tn * BN;
        const i64 kmax = kmax_of(g.P);
        double acc[TM][TN], cmp[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                acc[i][j] = 0.0;
                cmp[i][j] = 0.0;
            }
        if constexpr (MODE != 0) {
            mainloop_dma<MODE == 2>(g, m0, n0, kmax, sm, acc, cmp);
        } else {
            if (m0 + BM <= g.N && n0 + BN <= g.M) mainloop_reg<false>(g, m0, n0, kmax, sm, acc, cmp);
            else mainloop_reg<true>(g, m0, n0, kmax, sm, acc, cmp);
        }

        const bool odd = (OP == OP_WINOGRAD) && (g.P % 2 == 1);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const i64 gm = m0 + ty * TM + i;
            if (gm >= g.N) continue;
            double yi = 0.0, alast = 0.0;
            if (OP == OP_WINOGRAD) {
                yi = yv[gm];
                if (odd) alast = g.A[gm * g.lda + (g.P - 1)];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int j = 0; j < TH; ++j) {
                    const i64 gn = n0 + h * (BN / 2) + tx * TH + j;
                    if (gn >= g.M) continue;
                    double c = acc[i][h * TH + j];
                    if (OP == OP_DOT2) c = c + cmp[i][h * TH + j];
                    if (Q) {
                        // leftover P mod Q products, one at a time, k ascending
                        for (i64 k = kmax; k < g.P; ++k) {
                            const double x = g.A[gm * g.lda + k] * g.B[k * g.ldb + gn];
                            c = c + x;
                        }
                    }
                    if (OP == OP_WINOGRAD) {
                        c = (c - yi) - zv[gn];
                        if (odd) {
                            const double tail = alast * g.B[(g.P - 1) * g.ldb + gn];
                            c = c + tail;
                        }
                    }
                    g.C[gm * g.ldc + gn] = c;
                }
        }
    }
};

template <int BM, int BN, int TM, int TN, int OP, int MODE, class Src>
__global__ __launch_bounds__(NT, (MODE != 0 && OP != OP_KAHAN && OP != OP_DOT2) ? MMM_VALU_DMA_MINWAVES
                                                                                : MMM_VALU_MINWAVES) void
valu_gemm_kernel(Src src, i64 tiles_m, i64 tiles_n, i64 total, const double* __restrict__ yv,
                 const double* __restrict__ zv)
{
    typedef ValuTile<BM, BN, TM, TN, OP> T;
    __shared__ __align__(16) typename std::conditional<MODE != 0, typename T::SmemDma, typename T::SmemReg>::type sm;
    i64 prob, tm, tn;
    tile_of(xcd_remap(blockIdx.x, total), tiles_m, tiles_n, prob, tm, tn);
    T::template run<MODE>(src.get(prob), tm, tn, yv, zv, sm);
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Direct loads need every tile inside the matrices and 16-byte aligned rows
// of A and B; the grouped K range a whole number of steps (mode 1) or
// operands readable up to the next whole step (mode 2, zero-padded copies).
// Returns the mode, 0 when the problem takes register staging.
template <class T>
int direct_mode(const SingleSrc& src, i64 bm, i64 bn)
{
    const Gemm& g = src.g;
    const i64 kmax = T::kmax_of(g.P);
    const i64 kcap = g.kcap > g.P ? g.kcap : g.P;
    if (!(MMM_VALU_DMA && T::DMA_OK && g.N % bm == 0 && g.M % bn == 0 && kmax > 0 && g.lda % 2 == 0 &&
          g.ldb % 2 == 0 && aligned16(g.A) && aligned16(g.B)))
        return 0;
    // the loads' per-lane element offsets are 32-bit
    if ((double)bm * g.lda + T::BK * (double)g.ldb + bn >= 4294967296.0) return 0;
    if (kmax % T::BK == 0) return 1;
    return kcap >= (kmax + T::BK - 1) / T::BK * T::BK ? 2 : 0;
}

template <int BM, int BN, int TM, int TN, int OP, int MODE, class Src>
hipError_t launch_valu_mode(const Src& src, i64 tiles_m, i64 tiles_n, i64 total, const double* yv, const double* zv,
                            hipStream_t s)
{
    hipLaunchKernelGGL((valu_gemm_kernel<BM, BN, TM, TN, OP, MODE, Src>), dim3((unsigned)total), dim3(NT), 0, s,
                       src, tiles_m, tiles_n, total, yv, zv);
    return hipGetLastError();
}

template <int BM, int BN, int TM, int TN, int OP, class Src>
hipError_t launch_valu(const Src& src, i64 N, i64 M, const double* yv, const double* zv,
                       hipStream_t s)
{
    typedef ValuTile<BM, BN, TM, TN, OP> T;
    const i64 tiles_m = cdiv(N, BM), tiles_n = cdiv(M, BN);
    const i64 total = tiles_m * tiles_n * src.count();
    if (total == 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    // Strassen leaves never take direct loads (their operands are views)
    if constexpr (T::DMA_OK && std::is_same<Src, SingleSrc>::value) {
        const int mode = direct_mode<T>(src, BM, BN);
        if (mode == 1) return launch_valu_mode<BM, BN, TM, TN, OP, 1>(src, tiles_m, tiles_n, total, yv, zv, s);
        if (mode == 2) return launch_valu_mode<BM, BN, TM, TN, OP, 2>(src, tiles_m, tiles_n, total, yv, zv, s);
    }
    return launch_valu_mode<BM, BN, TM, TN, OP, 0>(src, tiles_m, tiles_n, total, yv, zv, s);
}

// Launch the whole-step direct-load kernel of this tile shape when the
// problem qualifies; false otherwise (nothing launched, and no other
// kernel of this shape is instantiated).
template <int BM, int BN, int TM, int TN, int OP, class Src>
bool try_launch_direct(const Src& src, i64 N, i64 M, const double* yv, const double* zv,
                       hipStream_t s, hipError_t& err)
{
    typedef ValuTile<BM, BN, TM, TN, OP> T;
    if constexpr (!T::DMA_OK || !std::is_same<Src, SingleSrc>::value) {
        return false;
    } else {
        if (direct_mode<T>(src, BM, BN) != 1) return false;
        const i64 tiles_m = cdiv(N, BM), tiles_n = cdiv(M, BN);
        const i64 total = tiles_m * tiles_n * src.count();
        if (total == 0 || total > 0x7fffffffLL) return false;
        err = launch_valu_mode<BM, BN, TM, TN, OP, 1>(src, tiles_m, tiles_n, total, yv, zv, s);
        return true;
    }
}

template <int BM, int BN, int TM, int TN>
struct Shape {
    static constexpr int bm = BM, bn = BN, tm = TM, tn = TN;
};
typedef Shape<MMM_VALU_NAIVE_TILE> NaiveShape;
typedef Shape<MMM_VALU_KAHAN_TILE> KahanShape;
typedef Shape<MMM_VALU_WINO_TILE> WinoShape;

// Tile of the inner-product methods for problems past the small case.
// Kahan keeps two doubles per entry, the longer groups and the on-array
// round trips more operands in flight: 64 x 64 tiles for those.
template <int OP>
struct ShapeOf {
    static constexpr bool small =
        OP == OP_KAHAN || OP == OP_UNROLL3 || OP == OP_UNROLL4 || OP == OP_ON_ARRAY || OP == OP_DOT2;
    typedef typename std::conditional<
        OP == OP_WINOGRAD, WinoShape,
        typename std::conditional<OP == OP_KAHAN || OP == OP_DOT2, KahanShape,
                                  typename std::conditional<small, Shape<64, 64, 4, 4>, NaiveShape>::type>::type>::type
        type;
};

// A product whose tiles would not give every CU a workgroup (fewer than
// kFillTiles of the method's own shape) is bound by latency, not by
// throughput: it takes the 32 x 32 tile (2 x 2 entries per lane) when that
// still gives half the CUs a workgroup, else the 16 x 32 one (1 x 2).  The
// tile shape only decides which lane computes an entry, never the order of
// its operations, so every shape gives the same bits.
constexpr i64 kFillTiles = 256;

template <int OP, class Src>
bool launch_latency_tile(const Src& src, i64 N, i64 M, const double* yv, const double* zv, hipStream_t s,
                         hipError_t& err)
{
    typedef typename ShapeOf<OP>::type S;
    const i64 cnt = src.count();
    if (cdiv(N, S::bm) * cdiv(M, S::bn) * cnt >= kFillTiles) return false;
    // NaivLoopUnrollingThree's K step of 24 does not split into whole loads
    // of a 16-row tile's 256 threads: it keeps the 32 x 32 tile
    if constexpr (OP == OP_UNROLL3) {
        err = launch_valu<32, 32, 2, 2, OP>(src, N, M, yv, zv, s);
    } else {
        if (cdiv(N, 32) * cdiv(M, 32) * cnt >= kFillTiles / 2) err = launch_valu<32, 32, 2, 2, OP>(src, N, M, yv, zv, s);
        else err = launch_valu<16, 32, 1, 2, OP>(src, N, M, yv, zv, s);
    }
    return true;
}

// Small problems (every dimension <= 48, e.g. the m x m leaves of the
// paper's Strassen embedding) use 32 x 32 tiles.
template <int OP, class Src>
hipError_t launch_naive_like(const Src& src, i64 N, i64 M, hipStream_t s)
{
    if (N <= 48 && M <= 48) return launch_valu<32, 32, 2, 2, OP>(src, N, M, nullptr, nullptr, s);
    hipError_t lerr = hipSuccess;
    if (launch_latency_tile<OP>(src, N, M, nullptr, nullptr, s, lerr)) return lerr;
    if constexpr (OP == OP_NAIVE || OP == OP_NAIVE_FMA) {
        typedef Shape<MMM_VALU_NAIVE_DMA_TILE> D;
        hipError_t err = hipSuccess;
        if (try_launch_direct<D::bm, D::bn, D::tm, D::tn, OP>(src, N, M, nullptr, nullptr, s, err))
            return err;
    }
    typedef typename ShapeOf<OP>::type S;
    return launch_valu<S::bm, S::bn, S::tm, S::tn, OP>(src, N, M, nullptr, nullptr, s);
}

// Copies for the tile the launcher takes at this shape (the 128 x 64 naive
// tile's conditions also admit the 128 x 128 one when M allows it: both take
// whole steps over the zero-padded K).
template <int OP>
ValuPad pad_plan_op(i64 N, i64 P, i64 M, bool zero_k)
{
    typedef typename ShapeOf<OP>::type S;
    typedef ValuTile<S::bm, S::bn, S::tm, S::tn, OP> T;
    ValuPad p{0, false, false};
    if (!MMM_VALU_DMA || !T::DMA_OK || (N <= 48 && M <= 48) || N % S::bm != 0 || M % S::bn != 0) return p;
    if ((double)N * (double)P * (double)M < kPadMinWork) return p;
    const i64 kmax = T::kmax_of(P);
    if (kmax <= 0 || (P % 2 == 0 && kmax % T::BK == 0)) return p;  // direct loads as it is
    const i64 kw = cdiv(kmax, T::BK) * T::BK;                      // K the last step loads
    if (zero_k) {
        p.kp = cdiv(P, T::BK) * T::BK;
        p.copy_b = p.kp > P;
        p.zero_k = true;
    } else {
        p.kp = kw > P + (P & 1) ? kw : P + (P & 1);
        p.copy_b = kw > P;
    }
    return p;
}

}  // namespace

ValuPad valu_pad_plan(ValuKind kind, i64 N, i64 P, i64 M)
{
    switch (kind) {
    case VK_NAIVE: return pad_plan_op<OP_NAIVE>(N, P, M, true);
    case VK_NAIVE_FMA: return pad_plan_op<OP_NAIVE_FMA>(N, P, M, true);
    case VK_KAHAN: return pad_plan_op<OP_KAHAN>(N, P, M, false);
    case VK_WINOGRAD: return pad_plan_op<OP_WINOGRAD>(N, P, M, false);
    case VK_ON_ARRAY: return pad_plan_op<OP_ON_ARRAY>(N, P, M, false);
    case VK_UNROLL2: return pad_plan_op<OP_UNROLL2>(N, P, M, false);
    case VK_UNROLL3: return pad_plan_op<OP_UNROLL3>(N, P, M, false);
    case VK_UNROLL4: return pad_plan_op<OP_UNROLL4>(N, P, M, false);
    case VK_DOT2: return pad_plan_op<OP_DOT2>(N, P, M, false);
    }
    return ValuPad{0, false, false};
}

hipError_t launch_naive(const Gemm& g, bool fused, hipStream_t s)
{
    SingleSrc src{g};
    return fused ? launch_naive_like<OP_NAIVE_FMA>(src, g.N, g.M, s) : launch_naive_like<OP_NAIVE>(src, g.N, g.M, s);
}

hipError_t launch_naive_strassen_leaves(const StrassenLeafSrc& src, hipStream_t s)
{
    const int d = src.T.depth;
    return launch_naive_like<OP_NAIVE>(src, src.T.n[d], src.T.m[d], s);
}

hipError_t launch_naive_variant(const Gemm& g, int variant, hipStream_t s)
{
    SingleSrc src{g};
    switch (variant) {
    case 0: return launch_naive_like<OP_ON_ARRAY>(src, g.N, g.M, s);
    case 2: return launch_naive_like<OP_UNROLL2>(src, g.N, g.M, s);
    case 3: return launch_naive_like<OP_UNROLL3>(src, g.N, g.M, s);
    case 4: return launch_naive_like<OP_UNROLL4>(src, g.N, g.M, s);
    case 5: return launch_naive_like<OP_DOT2>(src, g.N, g.M, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_kahan(const Gemm& g, hipStream_t s)
{
    SingleSrc src{g};
    return launch_naive_like<OP_KAHAN>(src, g.N, g.M, s);
}

hipError_t launch_winograd_main(const Gemm& g, const double* y, const double* z, hipStream_t s)
{
    SingleSrc src{g};
    typedef typename ShapeOf<OP_WINOGRAD>::type S;
    typedef Shape<MMM_VALU_WINO_DMA_TILE> D;
    hipError_t err = hipSuccess;
    if (launch_latency_tile<OP_WINOGRAD>(src, g.N, g.M, y, z, s, err)) return err;
    if (try_launch_direct<D::bm, D::bn, D::tm, D::tn, OP_WINOGRAD>(src, g.N, g.M, y, z, s, err))
        return err;
    return launch_valu<S::bm, S::bn, S::tm, S::tn, OP_WINOGRAD>(src, g.N, g.M, y, z, s);
}

}  // namespace mmm
