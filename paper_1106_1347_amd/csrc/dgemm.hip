// C = A B in FP64 on the matrix cores of gfx950 (v_mfma_f64_16x16x4_f64).
//
// The definition of Section 2.1 evaluated with the hardware's fused FP64
// multiply-accumulate; rounding order differs from the sequential sum, so
// results agree with it to a normwise tolerance (and exactly on integer
// data).  Also the leaf product of the Strassen recursion and the FP64 half
// of batches.
//
// Tiling: a 256-thread workgroup (4 waves, 2 x 2) owns a BM x BN tile of C;
// each wave owns WMB x WNB MFMA blocks of 16 x 16 (accumulators of 4
// doubles).  Tile shapes: 128 x 128 (4 x 4 blocks per wave), 64 x 64
// (2 x 2) and 128 x 64 (4 x 2).  K advances 16 at a time through LDS:
// A tile row-major [BM][16+2], B tile [16][BN+2] (padding breaks LDS bank
// aliasing); two workgroups per CU overlap one's loads with the other's
// MFMAs.  Tiles inside the matrices load without bounds checks.  Single products remap workgroups
// so each XCD works on a contiguous, 8-row-grouped range of tiles; batches
// run a persistent grid that deals the tiles of every problem round robin.
//
// MFMA operand layout (16x16x4, one double per lane for A and B): lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element r of
// lane l is D[l / 16 + 4 r][l % 16].
#include "batch.h"
#include "common.h"
#include "launch.h"

// Occupancy hint, register staging of the next K step and K step length;
// overridable at build time.  Defaults (measured on MI355X): two waves per
// SIMD, each K step loaded right before use, beat one wave per SIMD with a
// register-staged prefetch (53.7 vs 48.6 TFLOP/s at 8192^3).
#ifndef MMM_DGEMM_MINWAVES
#define MMM_DGEMM_MINWAVES 2
#endif
#ifndef MMM_DGEMM_PREFETCH
#define MMM_DGEMM_PREFETCH 0
#endif
#ifndef MMM_DGEMM_BK
#define MMM_DGEMM_BK 16
#endif
#ifndef MMM_DGEMM_DMA
#define MMM_DGEMM_DMA 1
#endif

namespace mmm {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BK = MMM_DGEMM_BK, NT = 256;

template <int WMB, int WNB>
struct DTile {
    static constexpr int BM = 32 * WMB, BN = 32 * WNB;
    static constexpr int LA = BM * BK / NT, LB = BK * BN / NT;
    static constexpr int NBUF = MMM_DGEMM_PREFETCH ? 2 : 1;
    struct Smem {
        double As[NBUF][BM][BK + 2];
        double Bs[NBUF][BK][BN + 2];
    };

    template <bool CHECK>
    __device__ __forceinline__ static void mainloop(const Gemm& g, i64 m0, i64 n0, Smem& sm, v4d (&acc)[WMB][WNB])
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm = wave >> 1, wn = wave & 1;
        const int li = lane & 15, lk = lane >> 4;
        const i64 ntiles = (g.P + BK - 1) / BK;
        double ra[LA], rb[LB];
        auto gload = [&](i64 t, bool check) __attribute__((always_inline)) {
            const i64 k0 = t * BK;
#pragma unroll
            for (int q = 0; q < LA; ++q) {
                const int e = q * NT + tid, r = e / BK, k = e % BK;
                const i64 gm = m0 + r, gk = k0 + k;
                if (check) ra[q] = (gm < g.N && gk < g.P) ? g.A[gm * g.lda + gk] : 0.0;
                else ra[q] = g.A[gm * g.lda + gk];
            }
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                const int e = q * NT + tid, k = e / BN, n = e % BN;
                const i64 gk = k0 + k, gn = n0 + n;
                if (check) rb[q] = (gk < g.P && gn < g.M) ? g.B[gk * g.ldb + gn] : 0.0;
                else rb[q] = g.B[gk * g.ldb + gn];
            }
        };
        auto lstore = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < LA; ++q) {
                const int e = q * NT + tid;
                sm.As[buf][e / BK][e % BK] = ra[q];
            }
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                const int e = q * NT + tid;
                sm.Bs[buf][e / BN][e % BN] = rb[q];
            }
        };
        auto compute = [&](int cur) __attribute__((always_inline)) {
#pragma unroll
            for (int ks = 0; ks < BK / 4; ++ks) {
                double a[WMB], b[WNB];
#pragma unroll
                for (int i = 0; i < WMB; ++i) a[i] = sm.As[cur][wm * WMB * 16 + i * 16 + li][ks * 4 + lk];
#pragma unroll
                for (int j = 0; j < WNB; ++j) b[j] = sm.Bs[cur][ks * 4 + lk][wn * WNB * 16 + j * 16 + li];
#pragma unroll
                for (int i = 0; i < WMB; ++i)
#pragma unroll
                    for (int j = 0; j < WNB; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        };
        auto need_check = [&](i64 t) __attribute__((always_inline)) { return CHECK || (t + 1) * BK > g.P; };
        if (MMM_DGEMM_PREFETCH) {
            if (ntiles > 0) {
                gload(0, need_check(0));
                lstore(0);
            }
            __syncthreads();
            for (i64 t = 0; t < ntiles; ++t) {
                const int cur = (int)(t & 1);
                if (t + 1 < ntiles) gload(t + 1, need_check(t + 1));
                compute(cur);
                if (t + 1 < ntiles) lstore(cur ^ 1);
                __syncthreads();
            }
        } else {
            for (i64 t = 0; t < ntiles; ++t) {
                gload(t, need_check(t));
                __syncthreads();  // the previous step's reads of the buffer are done
                lstore(0);
                __syncthreads();
                compute(0);
            }
            __syncthreads();
        }
    }

    __device__ __forceinline__ static void run(const Gemm& g, i64 tm, i64 tn, Smem& sm)
    {
        const i64 m0 = tm * BM, n0 = tn * BN;
        v4d acc[WMB][WNB];
#pragma unroll
        for (int i = 0; i < WMB; ++i)
#pragma unroll
            for (int j = 0; j < WNB; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
        if (m0 + BM <= g.N && n0 + BN <= g.M) mainloop<false>(g, m0, n0, sm, acc);
        else mainloop<true>(g, m0, n0, sm, acc);
        store(g, m0, n0, acc);
    }

    __device__ __forceinline__ static void store(const Gemm& g, i64 m0, i64 n0, v4d (&acc)[WMB][WNB])
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm = wave >> 1, wn = wave & 1;
        const int li = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int i = 0; i < WMB; ++i)
#pragma unroll
            for (int j = 0; j < WNB; ++j) {
                const i64 gn = n0 + wn * WNB * 16 + j * 16 + li;
                if (gn >= g.M) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const i64 gm = m0 + wm * WMB * 16 + i * 16 + lk + 4 * r;
                    if (gm < g.N) {
                        double* c = g.C + gm * g.ldc + gn;
                        *c = g.accumulate ? *c + acc[i][j][r] : acc[i][j][r];
                    }
                }
            }
    }
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

// 128 x 128 tiles whose operands are loaded straight from global memory into
// LDS (16 bytes per lane, lane l of a wave instruction landing at
// base + 16 l), two K steps of 16 in flight: no staging registers, so the
// next step's loads overlap the current step's MFMAs.  The layouts are XOR
// swizzled:
//   A tile (128 rows x 16 k, 8 chunks of 2 doubles per row): chunk c of row r
//     sits in slot c ^ ((r >> 1) & 7) of that row; the 8-byte fragment reads
//     (16 rows of one k) still meet a two-way bank conflict (counted), which
//     costs less than the alternative measured: 16-byte reads of chunk pairs
//     with slot c ^ (r & 7), conflict-free but 8% slower overall (82% against
//     88% MFMA-busy cycles at 8192^3);
//   B tile (16 k-rows x 128 columns, 64 chunks per row): chunk c of row k sits
//     in slot c ^ (8 (k & 1)); its fragment reads are conflict-free.
// Used for tiles inside the matrices with 16-byte aligned rows (even leading
// dimensions, aligned bases) and P a multiple of 16.
struct DmaTile {
    static constexpr int BM = 128, BN = 128, KS = 16;
    struct Smem {
        double A[2][BM * KS];
        double B[2][KS * BN];
    };

    __device__ __forceinline__ static void issue(const Gemm& g, i64 m0, i64 n0, i64 t, int buf, Smem& sm)
    {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const i64 k0 = t * KS;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int blk = q * 4 + wave;  // 1 KiB block of the tile written by this wave instruction
            const int p = blk * 64 + lane;
            const int r = p >> 3, c = (p & 7) ^ ((r >> 1) & 7);
            const double* src = g.A + (m0 + r) * g.lda + k0 + 2 * c;
            __builtin_amdgcn_global_load_lds((gbl_ptr_t)src, (lds_ptr_t)&sm.A[buf][blk * 128], 16, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int blk = q * 4 + wave;
            const int p = blk * 64 + lane;
            const int kr = p >> 6, c = (p & 63) ^ (8 * (kr & 1));
            const double* src = g.B + (k0 + kr) * g.ldb + n0 + 2 * c;
            __builtin_amdgcn_global_load_lds((gbl_ptr_t)src, (lds_ptr_t)&sm.B[buf][blk * 128], 16, 0, 0);
        }
    }

    __device__ __forceinline__ static double lds_a(const Smem& sm, int buf, int r, int k)
    {
        return sm.A[buf][r * KS + ((((k >> 1) ^ ((r >> 1) & 7))) << 1) + (k & 1)];
    }
    __device__ __forceinline__ static double lds_b(const Smem& sm, int buf, int k, int n)
    {
        return sm.B[buf][k * BN + ((((n >> 1) ^ (8 * (k & 1)))) << 1) + (n & 1)];
    }

    __device__ __forceinline__ static void mainloop(const Gemm& g, i64 m0, i64 n0, Smem& sm, v4d (&acc)[4][4])
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm = wave >> 1, wn = wave & 1;
        const int li = lane & 15, lk = lane >> 4;
        const i64 nt = g.P / KS;
        if (nt > 0) issue(g, m0, n0, 0, 0, sm);
        for (i64 t = 0; t < nt; ++t) {
            const int cur = (int)(t & 1);
            // this step's tile has landed in LDS (own loads), and every wave
            // is done with the buffer the next step overwrites
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (t + 1 < nt) issue(g, m0, n0, t + 1, cur ^ 1, sm);
#pragma unroll
            for (int ks = 0; ks < KS / 4; ++ks) {
                double a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = lds_a(sm, cur, wm * 64 + i * 16 + li, ks * 4 + lk);
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = lds_b(sm, cur, ks * 4 + lk, wn * 64 + j * 16 + li);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
};

__device__ inline i64 xcd_remap(i64 b, i64 total)
{
    if (total % 8 != 0) return b;
    return (b % 8) * (total / 8) + b / 8;
}

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

template <int WMB, int WNB, class Src>
__global__ __launch_bounds__(NT, MMM_DGEMM_MINWAVES) void dgemm_mfma_kernel(Src src, i64 tiles_m, i64 tiles_n, i64 total)
{
    typedef DTile<WMB, WNB> T;
    __shared__ __align__(16) typename T::Smem sm;
    i64 prob, tm, tn;
    tile_of(xcd_remap(blockIdx.x, total), tiles_m, tiles_n, prob, tm, tn);
    T::run(src.get(prob), tm, tn, sm);
}

// Every tile of every problem through the direct-load path (the host has
// checked that all of them qualify).
template <class Src>
__global__ __launch_bounds__(NT, MMM_DGEMM_MINWAVES) void dgemm_dma_kernel(Src src, i64 tiles_m, i64 tiles_n, i64 total)
{
    __shared__ __align__(16) DmaTile::Smem sm;
    i64 prob, tm, tn;
    tile_of(xcd_remap(blockIdx.x, total), tiles_m, tiles_n, prob, tm, tn);
    const Gemm g = src.get(prob);
    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
    DmaTile::mainloop(g, tm * 128, tn * 128, sm, acc);
    DTile<4, 4>::store(g, tm * 128, tn * 128, acc);
}

// Persistent grid over the tiles of many problems: tile t belongs to the
// problem p with prefix[p] <= t < prefix[p+1] and is its (t - prefix[p])-th
// tile in row-major tile order.  Workgroups claim tiles from the schedule.
template <int WMB, int WNB>
__global__ __launch_bounds__(NT, MMM_DGEMM_MINWAVES) void dgemm_grouped_kernel(const Gemm* __restrict__ probs,
                                                           const i64* __restrict__ prefix, int nprob,
                                                           TileSchedule sch)
{
    typedef DTile<WMB, WNB> T;
    __shared__ __align__(16) typename T::Smem sm;
    __shared__ int slot;
    for (;;) {
        const int q = claim_tile(sch, &slot);
        if (q >= sch.total) break;
        const i64 t = sch.list[q];
        int lo = 0, hi = nprob - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const Gemm g = probs[lo];
        const i64 local = t - prefix[lo];
        const i64 tiles_n = (g.M + T::BN - 1) / T::BN;
        T::run(g, local / tiles_n, local % tiles_n, sm);
        __syncthreads();
    }
    release_tiles(sch);
}

template <int WMB, int WNB, class Src>
hipError_t launch_dgemm_src(const Src& src, i64 N, i64 M, hipStream_t s)
{
    typedef DTile<WMB, WNB> T;
    const i64 tiles_m = cdiv(N, T::BM), tiles_n = cdiv(M, T::BN);
    const i64 total = tiles_m * tiles_n * src.count();
    if (total == 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((dgemm_mfma_kernel<WMB, WNB, Src>), dim3((unsigned)total), dim3(NT), 0, s, src, tiles_m, tiles_n,
                       total);
    return hipGetLastError();
}

template <class Src>
hipError_t launch_dgemm_dma(const Src& src, i64 N, i64 M, hipStream_t s)
{
    const i64 tiles_m = N / 128, tiles_n = M / 128;
    const i64 total = tiles_m * tiles_n * src.count();
    if (total == 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((dgemm_dma_kernel<Src>), dim3((unsigned)total), dim3(NT), 0, s, src, tiles_m, tiles_n, total);
    return hipGetLastError();
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

template <class Src>
hipError_t launch_dgemm_auto(const Src& src, i64 N, i64 M, hipStream_t s)
{
    // 128 x 128 tiles when they alone fill the 256 CUs, 64 x 64 when those
    // still give half the CUs a workgroup, else 32 x 32 (a small product is
    // bound by latency; every output takes the same MFMAs in the same order
    // whatever the tile, so the bits do not change)
    const i64 big = cdiv(N, 128) * cdiv(M, 128) * src.count();
    if (big >= 256) return launch_dgemm_src<4, 4>(src, N, M, s);
    if (cdiv(N, 64) * cdiv(M, 64) * src.count() >= 128) return launch_dgemm_src<2, 2>(src, N, M, s);
    return launch_dgemm_src<1, 1>(src, N, M, s);
}

}  // namespace

// P not a multiple of 16 keeps a large product off the direct-load kernel;
// zero-padding K to the next multiple adds exact zeros to every sum.
ValuPad dgemm_pad_plan(i64 N, i64 P, i64 M)
{
    ValuPad p{0, false, false};
    if (!MMM_DGEMM_DMA || N % 128 != 0 || M % 128 != 0 || (N / 128) * (M / 128) < 256 || P % 16 == 0) return p;
    if ((double)N * (double)P * (double)M < kPadMinWork) return p;
    p.kp = cdiv(P, 16) * 16;
    p.copy_b = true;
    p.zero_k = true;
    return p;
}

hipError_t launch_dgemm(const Gemm& g, hipStream_t s)
{
    SingleSrc src{g};
    if (MMM_DGEMM_DMA && g.N % 128 == 0 && g.M % 128 == 0 && g.P % 16 == 0 && g.lda % 2 == 0 && g.ldb % 2 == 0 &&
        aligned16(g.A) && aligned16(g.B) && (g.N / 128) * (g.M / 128) >= 256)
        return launch_dgemm_dma(src, g.N, g.M, s);
    return launch_dgemm_auto(src, g.N, g.M, s);
}

hipError_t launch_dgemm_strassen_leaves(const StrassenLeafSrc& src, hipStream_t s)
{
    const StrassenTree& T = src.T;
    const int d = T.depth;
    // every leaf operand is the root, a quadrant view or a dense slot: all
    // leading dimensions and offsets stay even when these are (views of a
    // misaligned root are copied to their slots by the sum passes)
    bool ok = MMM_DGEMM_DMA && T.n[d] % 128 == 0 && T.m[d] % 128 == 0 && T.p[d] % 16 == 0 &&
              (T.copy_leaf_views_a || (T.lda % 2 == 0 && aligned16(T.A))) &&
              (T.copy_leaf_views_b || (T.ldb % 2 == 0 && aligned16(T.B)));
    for (int e = 1; e <= d && ok; ++e)
        ok = T.p[e] % 2 == 0 && T.m[e] % 2 == 0 && aligned16(T.WA[e]) && aligned16(T.WB[e]);
    if (ok) return launch_dgemm_dma(src, T.n[d], T.m[d], s);
    return launch_dgemm_auto(src, T.n[d], T.m[d], s);
}

int dgemm_tile_bm(int tile) { return tile == DGEMM_TILE_64x64 ? 64 : 128; }
int dgemm_tile_bn(int tile) { return tile == DGEMM_TILE_128x128 ? 128 : 64; }

// Workgroups of the persistent grouped kernel that fit on one CU at once (its
// register and LDS footprint for that tile shape), so the grid can fill the
// chip: smaller tiles leave room for more resident workgroups, whose loads
// then overlap.  With `share`, only as many as leave each SIMD at least
// kShareVgprs of its 512 registers per lane for the kernels of another graph
// branch: a grid that takes the whole register file keeps every other
// kernel's waves off the chip while it runs (a workgroup of NT = 256 threads
// puts one wave on each of the CU's four SIMDs).
constexpr int kShareVgprs = 64;

template <class K>
int grouped_per_cu(K kern, bool share)
{
    int n = 0;
    hipFuncAttributes fa;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, NT, 0) != hipSuccess || n < 1 ||
        hipFuncGetAttributes(&fa, (const void*)kern) != hipSuccess) {
        (void)hipGetLastError();
        return 2;
    }
    const int vgprs = (fa.numRegs + 7) / 8 * 8;  // allocated in granules of 8
    while (share && n > 1 && vgprs > 0 && 512 - n * vgprs < kShareVgprs) --n;
    return n;
}

int dgemm_grouped_per_cu(int tile, bool share)
{
    if (tile == DGEMM_TILE_128x128) return grouped_per_cu(dgemm_grouped_kernel<4, 4>, share);
    if (tile == DGEMM_TILE_64x64) return grouped_per_cu(dgemm_grouped_kernel<2, 2>, share);
    return grouped_per_cu(dgemm_grouped_kernel<4, 2>, share);
}

hipError_t launch_dgemm_grouped(int tile, const Gemm* probs, const i64* prefix, int nprob, i64 total, int grid,
                                TileSchedule sch, hipStream_t s)
{
    if (total == 0 || nprob == 0) return hipSuccess;
    if (tile == DGEMM_TILE_128x128)
        hipLaunchKernelGGL((dgemm_grouped_kernel<4, 4>), dim3(grid), dim3(NT), 0, s, probs, prefix, nprob, sch);
    else if (tile == DGEMM_TILE_64x64)
        hipLaunchKernelGGL((dgemm_grouped_kernel<2, 2>), dim3(grid), dim3(NT), 0, s, probs, prefix, nprob, sch);
    else
        hipLaunchKernelGGL((dgemm_grouped_kernel<4, 2>), dim3(grid), dim3(NT), 0, s, probs, prefix, nprob, sch);
    return hipGetLastError();
}

}  // namespace mmm
