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
// (2 x 2) and 128 x 64 (4 x 2).  K advances 16 at a time through
// double-buffered LDS: A tile row-major [BM][16+2], B tile [16][BN+2]
// (padding breaks LDS bank aliasing).  The next K step's global loads are
// issued before the current step's MFMAs.  Single products remap workgroups
// so each XCD works on a contiguous, 8-row-grouped range of tiles; batches
// run a persistent grid that deals the tiles of every problem round robin.
//
// MFMA operand layout (16x16x4, one double per lane for A and B): lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element r of
// lane l is D[l / 16 + 4 r][l % 16].
#include "batch.h"
#include "common.h"
#include "launch.h"

namespace mmm {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BK = 16, NT = 256;

template <int WMB, int WNB>
struct DTile {
    static constexpr int BM = 32 * WMB, BN = 32 * WNB;
    static constexpr int LA = BM * BK / NT, LB = BK * BN / NT;
    struct Smem {
        double As[2][BM][BK + 2];
        double Bs[2][BK][BN + 2];
    };

    __device__ __forceinline__ static void run(const Gemm& g, i64 tm, i64 tn, Smem& sm)
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm = wave >> 1, wn = wave & 1;
        const int li = lane & 15, lk = lane >> 4;
        const i64 m0 = tm * BM, n0 = tn * BN;
        const i64 ntiles = (g.P + BK - 1) / BK;

        v4d acc[WMB][WNB];
#pragma unroll
        for (int i = 0; i < WMB; ++i)
#pragma unroll
            for (int j = 0; j < WNB; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

        double ra[LA], rb[LB];
        auto gload = [&](i64 t) __attribute__((always_inline)) {
            const i64 k0 = t * BK;
#pragma unroll
            for (int q = 0; q < LA; ++q) {
                const int e = q * NT + tid, r = e / BK, k = e % BK;
                const i64 gm = m0 + r, gk = k0 + k;
                ra[q] = (gm < g.N && gk < g.P) ? g.A[gm * g.lda + gk] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                const int e = q * NT + tid, k = e / BN, n = e % BN;
                const i64 gk = k0 + k, gn = n0 + n;
                rb[q] = (gk < g.P && gn < g.M) ? g.B[gk * g.ldb + gn] : 0.0;
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

        if (ntiles > 0) {
            gload(0);
            lstore(0);
        }
        __syncthreads();
        for (i64 t = 0; t < ntiles; ++t) {
            const int cur = (int)(t & 1);
            if (t + 1 < ntiles) gload(t + 1);
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
            if (t + 1 < ntiles) lstore(cur ^ 1);
            __syncthreads();
        }

#pragma unroll
        for (int i = 0; i < WMB; ++i)
#pragma unroll
            for (int j = 0; j < WNB; ++j) {
                const i64 gn = n0 + wn * WNB * 16 + j * 16 + li;
                if (gn >= g.M) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const i64 gm = m0 + wm * WMB * 16 + i * 16 + lk + 4 * r;
                    if (gm < g.N) g.C[gm * g.ldc + gn] = acc[i][j][r];
                }
            }
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
__global__ __launch_bounds__(NT) void dgemm_mfma_kernel(Src src, i64 tiles_m, i64 tiles_n, i64 total)
{
    typedef DTile<WMB, WNB> T;
    __shared__ __align__(16) typename T::Smem sm;
    i64 prob, tm, tn;
    tile_of(xcd_remap(blockIdx.x, total), tiles_m, tiles_n, prob, tm, tn);
    T::run(src.get(prob), tm, tn, sm);
}

// Persistent grid over the tiles of many problems: tile t belongs to the
// problem p with prefix[p] <= t < prefix[p+1] and is its (t - prefix[p])-th
// tile in row-major tile order.  Workgroup b takes tiles b, b + grid, ...
template <int WMB, int WNB>
__global__ __launch_bounds__(NT) void dgemm_grouped_kernel(const Gemm* __restrict__ probs,
                                                           const i64* __restrict__ prefix, int nprob, i64 total)
{
    typedef DTile<WMB, WNB> T;
    __shared__ __align__(16) typename T::Smem sm;
    for (i64 t = blockIdx.x; t < total; t += gridDim.x) {
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
hipError_t launch_dgemm_auto(const Src& src, i64 N, i64 M, hipStream_t s)
{
    // 128 x 128 tiles when they alone fill the 256 CUs, 64 x 64 otherwise
    const i64 big = cdiv(N, 128) * cdiv(M, 128) * src.count();
    if (big >= 256) return launch_dgemm_src<4, 4>(src, N, M, s);
    return launch_dgemm_src<2, 2>(src, N, M, s);
}

}  // namespace

hipError_t launch_dgemm(const Gemm& g, hipStream_t s)
{
    SingleSrc src{g};
    return launch_dgemm_auto(src, g.N, g.M, s);
}

hipError_t launch_dgemm_strassen_leaves(const StrassenLeafSrc& src, hipStream_t s)
{
    const int d = src.T.depth;
    return launch_dgemm_auto(src, src.T.n[d], src.T.m[d], s);
}

int dgemm_tile_bm(int tile) { return tile == DGEMM_TILE_64x64 ? 64 : 128; }
int dgemm_tile_bn(int tile) { return tile == DGEMM_TILE_128x128 ? 128 : 64; }

hipError_t launch_dgemm_grouped(int tile, const Gemm* probs, const i64* prefix, int nprob, i64 total, int grid,
                                hipStream_t s)
{
    if (total == 0 || nprob == 0) return hipSuccess;
    if (tile == DGEMM_TILE_128x128)
        hipLaunchKernelGGL((dgemm_grouped_kernel<4, 4>), dim3(grid), dim3(NT), 0, s, probs, prefix, nprob, total);
    else if (tile == DGEMM_TILE_64x64)
        hipLaunchKernelGGL((dgemm_grouped_kernel<2, 2>), dim3(grid), dim3(NT), 0, s, probs, prefix, nprob, total);
    else
        hipLaunchKernelGGL((dgemm_grouped_kernel<4, 2>), dim3(grid), dim3(NT), 0, s, probs, prefix, nprob, total);
    return hipGetLastError();
}

}  // namespace mmm
