// Inner-product methods of Section 2 on the FP64 vector ALUs of gfx950:
// NaivStandard (2.1.1), NaivKahan (2.1.3) and the main loop of
// WinogradOriginal (2.3.1, also used by WinogradScaled 2.3.2).
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
// is two doubles per entry), each thread a TM x TN register block (rows ty*TM + i, columns h*BN/2 +
// tx*TN/2 + j).  K advances in steps of 16 (32 for Kahan) through LDS tiles:
// the A tile is stored k-major so a thread reads its TM rows as one
// contiguous run, the B tile row-major.  With PREFETCH the global loads of
// step t+1 are issued before the arithmetic of step t and held in registers;
// without it each step's tile is loaded and stored before the arithmetic
// (fewer registers, more resident waves to hide the latency).  Within a step
// each operation of the recurrence is issued for a whole row (Winograd) or
// the whole register block (naive, Kahan) before the next one, so the FP64
// pipeline sees independent chains; the per-entry order of operations, and
// hence every rounding, is unchanged.  Tiles that lie inside the matrices
// take a path without bounds checks.
#include <type_traits>

#include "common.h"
#include "launch.h"

// Tile shapes (BM, BN, TM, TN), staging and occupancy hints; overridable at
// build time.  Defaults (measured on MI355X at 4096^3): two waves per SIMD
// without register prefetch beat one wave per SIMD with it by 10-20%.
#ifndef MMM_VALU_NAIVE_TILE
#define MMM_VALU_NAIVE_TILE 128, 64, 8, 4
#endif
#ifndef MMM_VALU_KAHAN_TILE
#define MMM_VALU_KAHAN_TILE 64, 64, 4, 4
#endif
#ifndef MMM_VALU_WINO_TILE
#define MMM_VALU_WINO_TILE 128, 64, 8, 4
#endif
#ifndef MMM_VALU_PREFETCH
#define MMM_VALU_PREFETCH 0
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
// evaluate each operation of a step for a whole row / block of entries
// before the next (independent chains for the FP64 pipeline)
#ifndef MMM_VALU_ILP
#define MMM_VALU_ILP 1
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
    OP_ON_ARRAY = 7  // NaivOnArray
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

template <int BM, int BN, int TM, int TN, int OP, bool SCALED>
struct ValuTile {
    // K per LDS step; a multiple of the group length of the unrolled sums
    static constexpr int BK = OP == OP_KAHAN ? MMM_VALU_KAHAN_BK : (OP == OP_UNROLL3 ? 24 : MMM_VALU_BK);
    static constexpr int Q = unroll_q(OP);
    static_assert((BM / TM) * (BN / TN) == NT, "256 threads");
    static_assert(BM / TM == 16 && BN / TN == 16, "16 x 16 thread grid");
    static constexpr int LA = BM * BK / NT;  // A elements each thread moves per step
    static constexpr int LB = BK * BN / NT;
    static constexpr int TH = TN / 2;        // columns per half
    static constexpr int KSTEP = (OP == OP_WINOGRAD) ? 2 : (Q ? Q : 1);

    static constexpr int NBUF = MMM_VALU_PREFETCH ? 2 : 1;
    struct Smem {
        double As[NBUF][BK][BM + 2];
        double Bs[NBUF][BK][BN + 2];
    };

    // Accumulate the whole K range into acc (and cmp for Kahan).  CHECK:
    // bounds-check every load (edge tiles); otherwise only the last K step
    // is checked.
    template <bool CHECK>
    __device__ __forceinline__ static void mainloop(const Gemm& g, i64 m0, i64 n0, i64 kmax, double sa, double sb,
                                                    Smem& sm, double (&acc)[TM][TN], double (&cmp)[TM][TN])
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
                double v;
                if (check) v = (gm < g.N && gk < kmax) ? g.A[gm * g.lda + gk] : 0.0;
                else v = g.A[gm * g.lda + gk];
                ra[q] = SCALED ? v * sa : v;
            }
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                const int e = q * NT + tid, k = e / BN, n = e % BN;
                const i64 gk = k0 + k, gn = n0 + n;
                double v;
                if (check) v = (gk < kmax && gn < g.M) ? g.B[gk * g.ldb + gn] : 0.0;
                else v = g.B[gk * g.ldb + gn];
                rb[q] = SCALED ? v * sb : v;
            }
        };
        auto lstore = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < LA; ++q) {
                const int e = q * NT + tid;
                sm.As[buf][e % BK][e / BK] = ra[q];
            }
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                const int e = q * NT + tid;
                sm.Bs[buf][e / BN][e % BN] = rb[q];
            }
        };
        auto frag_a = [&](int buf, int k, double* a) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < TM; i += 2) {
                const double2 v = *reinterpret_cast<const double2*>(&sm.As[buf][k][ty * TM + i]);
                a[i] = v.x;
                a[i + 1] = v.y;
            }
        };
        auto frag_b = [&](int buf, int k, double* b) __attribute__((always_inline)) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (TH % 2 == 0) {
#pragma unroll
                    for (int j = 0; j < TH; j += 2) {
                        const double2 v =
                            *reinterpret_cast<const double2*>(&sm.Bs[buf][k][h * (BN / 2) + tx * TH + j]);
                        b[h * TH + j] = v.x;
                        b[h * TH + j + 1] = v.y;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < TH; ++j) b[h * TH + j] = sm.Bs[buf][k][h * (BN / 2) + tx * TH + j];
                }
            }
        };
        auto step = [&](int buf, int k) __attribute__((always_inline)) {
            if (OP == OP_WINOGRAD) {
                // pair (k, k+1): (A_{i,k} + B_{k+1,j}) (A_{i,k+1} + B_{k,j})
                double a0[TM], a1[TM], b0[TN], b1[TN];
                frag_a(buf, k, a0);
                frag_a(buf, k + 1, a1);
                frag_b(buf, k, b0);
                frag_b(buf, k + 1, b1);
                if (MMM_VALU_ILP) {
                    // one row of the register block at a time, each
                    // operation for all its columns before the next
#pragma unroll
                    for (int i = 0; i < TM; ++i) {
                        double u[TN], v[TN], w[TN];
#pragma unroll
                        for (int j = 0; j < TN; ++j) u[j] = a0[i] + b1[j];
#pragma unroll
                        for (int j = 0; j < TN; ++j) v[j] = a1[i] + b0[j];
#pragma unroll
                        for (int j = 0; j < TN; ++j) w[j] = u[j] * v[j];
#pragma unroll
                        for (int j = 0; j < TN; ++j) acc[i][j] = acc[i][j] + w[j];
                    }
                    return;
                }
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        const double u = a0[i] + b1[j];
                        const double v = a1[i] + b0[j];
                        const double w = u * v;
                        acc[i][j] = acc[i][j] + w;
                    }
            } else if (Q) {
                // a group of Q consecutive k: (p_1 + p_2 (+ p_3 (+ p_4))) summed
                // left to right, then added to the running sum
                double a[Q ? Q : 1][TM], b[Q ? Q : 1][TN];
#pragma unroll
                for (int r = 0; r < Q; ++r) {
                    frag_a(buf, k + r, a[r]);
                    frag_b(buf, k + r, b[r]);
                }
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
            } else {
                double a[TM], b[TN];
                frag_a(buf, k, a);
                frag_b(buf, k, b);
                if (MMM_VALU_ILP && OP == OP_KAHAN) {
                    // each operation of the recurrence for all entries of
                    // the register block before the next
                    double x[TM][TN], e[TM][TN], t[TM][TN];
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) x[i][j] = a[i] * b[j];
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) e[i][j] = cmp[i][j] + x[i][j];
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) t[i][j] = acc[i][j] + e[i][j];
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) {
                            cmp[i][j] = (acc[i][j] - t[i][j]) + e[i][j];
                            acc[i][j] = t[i][j];
                        }
                    return;
                }
                if (MMM_VALU_ILP && (OP == OP_NAIVE || OP == OP_ON_ARRAY)) {
                    // all products of the step first, then the sums
                    double x[TM][TN];
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) x[i][j] = a[i] * b[j];
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) acc[i][j] = acc[i][j] + x[i][j];
                    return;
                }
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        if (OP == OP_NAIVE || OP == OP_ON_ARRAY) {
                            const double x = a[i] * b[j];
                            acc[i][j] = acc[i][j] + x;
                        } else if (OP == OP_NAIVE_FMA) {
                            acc[i][j] = fma(a[i], b[j], acc[i][j]);
                        } else {
                            // Kahan as printed: err = err + x; t = sum + err;
                            // err = (sum - t) + err; sum = t.
                            const double x = a[i] * b[j];
                            const double e = cmp[i][j] + x;
                            const double t = acc[i][j] + e;
                            cmp[i][j] = (acc[i][j] - t) + e;
                            acc[i][j] = t;
                        }
                    }
            }
        };
        auto compute = [&](int buf, i64 t) __attribute__((always_inline)) {
            const i64 rem = kmax - t * BK;
            if (rem >= BK) {
#pragma unroll
                for (int k = 0; k < BK; k += KSTEP) step(buf, k);
            } else {
                const int kc = (int)rem;
                for (int k = 0; k < kc; k += KSTEP) step(buf, k);
            }
        };
        auto need_check = [&](i64 t) __attribute__((always_inline)) { return CHECK || (t + 1) * BK > kmax; };
        // NaivOnArray: the running sum lives in the entries of C; every K
        // step reads them and writes them back (the first step starts from
        // the zeroed entries)
        auto c_io = [&](bool store) __attribute__((always_inline)) {
            if (OP != OP_ON_ARRAY) return;
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
        };
        if (OP == OP_ON_ARRAY) c_io(true);  // C = 0

        if (MMM_VALU_PREFETCH) {
            if (ntiles > 0) {
                gload(0, need_check(0));
                lstore(0);
            }
            __syncthreads();
            for (i64 t = 0; t < ntiles; ++t) {
                const int cur = (int)(t & 1);
                if (t + 1 < ntiles) gload(t + 1, need_check(t + 1));
                c_io(false);
                compute(cur, t);
                c_io(true);
                if (t + 1 < ntiles) lstore(cur ^ 1);
                __syncthreads();
            }
        } else {
            for (i64 t = 0; t < ntiles; ++t) {
                gload(t, need_check(t));
                __syncthreads();  // the previous step's reads of the buffer are done
                lstore(0);
                __syncthreads();
                c_io(false);
                compute(0, t);
                c_io(true);
            }
        }
    }

    __device__ __forceinline__ static void run(const Gemm& g, i64 tm, i64 tn, const double* __restrict__ yv,
                                               const double* __restrict__ zv, const int* lam, Smem& sm)
    {
        const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
        const i64 m0 = tm * BM, n0 = tn * BN;
        // the grouped part of the k range; the rest is added in the epilogue
        const i64 kmax = (OP == OP_WINOGRAD) ? 2 * (g.P / 2) : (Q ? Q * (g.P / Q) : g.P);
        double sa = 1.0, sb = 1.0;
        if (SCALED) {
            const int l = *lam;
            sa = ldexp(1.0, l);
            sb = ldexp(1.0, -l);
        }
        double acc[TM][TN], cmp[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                acc[i][j] = 0.0;
                cmp[i][j] = 0.0;
            }
        if (m0 + BM <= g.N && n0 + BN <= g.M) mainloop<false>(g, m0, n0, kmax, sa, sb, sm, acc, cmp);
        else mainloop<true>(g, m0, n0, kmax, sa, sb, sm, acc, cmp);

        const bool odd = (OP == OP_WINOGRAD) && (g.P % 2 == 1);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const i64 gm = m0 + ty * TM + i;
            if (gm >= g.N) continue;
            double yi = 0.0, alast = 0.0;
            if (OP == OP_WINOGRAD) {
                yi = yv[gm];
                if (odd) alast = SCALED ? g.A[gm * g.lda + (g.P - 1)] * sa : g.A[gm * g.lda + (g.P - 1)];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int j = 0; j < TH; ++j) {
                    const i64 gn = n0 + h * (BN / 2) + tx * TH + j;
                    if (gn >= g.M) continue;
                    double c = acc[i][h * TH + j];
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
                            const double bl =
                                SCALED ? g.B[(g.P - 1) * g.ldb + gn] * sb : g.B[(g.P - 1) * g.ldb + gn];
                            const double tail = alast * bl;
                            c = c + tail;
                        }
                    }
                    g.C[gm * g.ldc + gn] = c;
                }
        }
    }
};

template <int BM, int BN, int TM, int TN, int OP, bool SCALED, class Src>
__global__ __launch_bounds__(NT, MMM_VALU_MINWAVES) void valu_gemm_kernel(Src src, i64 tiles_m, i64 tiles_n,
                                                                          i64 total, const double* __restrict__ yv,
                                                                          const double* __restrict__ zv,
                                                                          const int* lam)
{
    typedef ValuTile<BM, BN, TM, TN, OP, SCALED> T;
    __shared__ __align__(16) typename T::Smem sm;
    i64 prob, tm, tn;
    tile_of(xcd_remap(blockIdx.x, total), tiles_m, tiles_n, prob, tm, tn);
    T::run(src.get(prob), tm, tn, yv, zv, lam, sm);
}

template <int BM, int BN, int TM, int TN, int OP, bool SCALED, class Src>
hipError_t launch_valu(const Src& src, i64 N, i64 M, const double* yv, const double* zv, const int* lam,
                       hipStream_t s)
{
    const i64 tiles_m = cdiv(N, BM), tiles_n = cdiv(M, BN);
    const i64 total = tiles_m * tiles_n * src.count();
    if (total == 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((valu_gemm_kernel<BM, BN, TM, TN, OP, SCALED, Src>), dim3((unsigned)total), dim3(NT), 0, s,
                       src, tiles_m, tiles_n, total, yv, zv, lam);
    return hipGetLastError();
}

template <int BM, int BN, int TM, int TN>
struct Shape {
    static constexpr int bm = BM, bn = BN, tm = TM, tn = TN;
};
typedef Shape<MMM_VALU_NAIVE_TILE> NaiveShape;
typedef Shape<MMM_VALU_KAHAN_TILE> KahanShape;
typedef Shape<MMM_VALU_WINO_TILE> WinoShape;

// Small problems (every dimension <= 48, e.g. the m x m leaves of the
// paper's Strassen embedding) use 32 x 32 tiles.
template <int OP, class Src>
hipError_t launch_naive_like(const Src& src, i64 N, i64 M, hipStream_t s)
{
    if (N <= 48 && M <= 48) return launch_valu<32, 32, 2, 2, OP, false>(src, N, M, nullptr, nullptr, nullptr, s);
    // Kahan keeps two doubles per entry, the longer groups and the on-array
    // round trips more operands in flight: 64 x 64 tiles for those
    constexpr bool small = OP == OP_KAHAN || OP == OP_UNROLL3 || OP == OP_UNROLL4 || OP == OP_ON_ARRAY;
    typedef typename std::conditional<OP == OP_KAHAN, KahanShape,
                                      typename std::conditional<small, Shape<64, 64, 4, 4>, NaiveShape>::type>::type S;
    return launch_valu<S::bm, S::bn, S::tm, S::tn, OP, false>(src, N, M, nullptr, nullptr, nullptr, s);
}

}  // namespace

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
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_kahan(const Gemm& g, hipStream_t s)
{
    SingleSrc src{g};
    return launch_naive_like<OP_KAHAN>(src, g.N, g.M, s);
}

hipError_t launch_winograd_main(const Gemm& g, const double* y, const double* z, const int* lam, hipStream_t s)
{
    SingleSrc src{g};
    typedef WinoShape S;
    if (lam) return launch_valu<S::bm, S::bn, S::tm, S::tn, OP_WINOGRAD, true>(src, g.N, g.M, y, z, lam, s);
    return launch_valu<S::bm, S::bn, S::tm, S::tn, OP_WINOGRAD, false>(src, g.N, g.M, y, z, nullptr, s);
}

}  // namespace mmm
