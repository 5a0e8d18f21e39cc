// Auxiliary routines of Section 1 (Plus, Minus, MultiplyWithScalar,
// NormInf), the sequential vector reductions of WinogradOriginal's
// precompute (y_i, z_k) and WinogradScaled's norms, and the copies of the
// direct-load paths (zero-padded operands, WinogradScaled's scaled
// operands).  All are bound by HBM bandwidth.
//
// Built with -ffp-contract=off: every sum and product is rounded on its
// own, and each reduction runs over its vector in ascending order, so the
// results equal a sequential binary64 evaluation bit for bit.
#include <algorithm>

#include "common.h"
#include "launch.h"
#include "reduce.h"

namespace mmm {

namespace {

template <int OP>
__device__ inline double ew(double a, double b, double alpha)
{
    if (OP == EW_PLUS) return a + b;
    if (OP == EW_MINUS) return a - b;
    return alpha * a;
}

typedef double dbl2 __attribute__((ext_vector_type(2)));

// Plus / Minus / MultiplyWithScalar.  Aligned operands: each thread takes 4
// pairs of doubles 256 pairs apart, issues the four 16-byte loads of each
// operand before any arithmetic, and loads and stores non-temporally (every
// byte is touched once): 6.4 TB/s on 8192^2 Plus against 4.6 TB/s for a
// grid-stride loop of single pairs.  Otherwise 8-byte accesses.
template <int OP, bool VEC>
__global__ __launch_bounds__(256) void ew_kernel(const double* A, const double* B, double alpha, double* C, i64 n)
{
    if (VEC) {
        const i64 n2 = n / 2;
        const dbl2* A2 = reinterpret_cast<const dbl2*>(A);
        const dbl2* B2 = reinterpret_cast<const dbl2*>(B);
        dbl2* C2 = reinterpret_cast<dbl2*>(C);
        for (i64 i0 = (i64)blockIdx.x * 1024 + threadIdx.x; i0 < n2; i0 += (i64)gridDim.x * 1024) {
            dbl2 a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const i64 i = i0 + u * 256;
                if (i < n2) {
                    a[u] = __builtin_nontemporal_load(A2 + i);
                    if (OP != EW_SCALE) b[u] = __builtin_nontemporal_load(B2 + i);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const i64 i = i0 + u * 256;
                if (i < n2) {
                    dbl2 c;
                    c.x = ew<OP>(a[u].x, OP != EW_SCALE ? b[u].x : 0.0, alpha);
                    c.y = ew<OP>(a[u].y, OP != EW_SCALE ? b[u].y : 0.0, alpha);
                    __builtin_nontemporal_store(c, C2 + i);
                }
            }
        }
        if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0)
            C[n - 1] = ew<OP>(A[n - 1], OP != EW_SCALE ? B[n - 1] : 0.0, alpha);
    } else {
        for (i64 i = (i64)blockIdx.x * 256 + threadIdx.x; i < n; i += (i64)gridDim.x * 256)
            C[i] = ew<OP>(A[i], OP != EW_SCALE ? B[i] : 0.0, alpha);
    }
}

// workgroups covering `work` items at `per` items per thread, at most 2^31 - 1
// (the kernels loop when capped)
unsigned grid_for(i64 work, i64 per)
{
    const i64 b = cdiv(work, 256 * per);
    return (unsigned)(b < 1 ? 1 : (b > 0x7fffffffLL ? 0x7fffffffLL : b));
}

template <int OP>
hipError_t launch_ew(const double* A, const double* B, double alpha, double* C, i64 n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const bool vec = ((uintptr_t)A % 16 == 0) && ((uintptr_t)C % 16 == 0) && (OP == EW_SCALE || (uintptr_t)B % 16 == 0);
    if (vec)
        hipLaunchKernelGGL((ew_kernel<OP, true>), dim3(grid_for(n / 2, 4)), dim3(256), 0, s, A, B, alpha, C, n);
    else
        hipLaunchKernelGGL((ew_kernel<OP, false>), dim3(grid_for(n, 4)), dim3(256), 0, s, A, B, alpha, C, n);
    return hipGetLastError();
}

template <int OP, bool COLS, bool FOLD_MAX>
__global__ __launch_bounds__(256) void vecred_kernel(const double* __restrict__ X, i64 ld, i64 nvec, i64 len,
                                                     double* __restrict__ out)
{
    __shared__ double T[2][RV][RL + 1];
    vecred_body<OP, COLS, FOLD_MAX>(X, ld, nvec, len, out, blockIdx.x, T);
}

__device__ inline long long floor_half(long long x) { return x >= 0 ? x / 2 : -((-x + 1) / 2); }

// Section 2.3.2: largest integer lambda with 1/2 <= 2^(2 lambda) nA/nB <= 2.
// Write nA = a 2^eA, nB = b 2^eB (a, b in [1/2, 1)), d = eB - eA and
// x = 2 lambda - d; the condition is 1/2 <= (a/b) 2^x <= 2.  For b > a it
// holds for x in {0, 1}, for b < a for x in {-1, 0}, for a = b for
// x in {-1, 0, 1}; the largest lambda is floor((d+1)/2) when b >= a and
// floor(d/2) otherwise.
__device__ inline int winograd_lambda(double a, double b)
{
    int res = 0;
    if (a > 0.0 && b > 0.0 && !isinf(a) && !isinf(b)) {
        int eA, eB;
        const double fa = frexp(a, &eA);
        const double fb = frexp(b, &eB);
        const long long d = (long long)eB - (long long)eA;
        res = (int)(fb >= fa ? floor_half(d + 1) : floor_half(d));
    }
    return res;
}

__global__ void lambda_kernel(const double* nA, const double* nB, int* lam) { *lam = winograd_lambda(*nA, *nB); }

// Row-block copies: workgroup b takes row b / chunks, columns
// 1024 (b % chunks) .. + 1023, 4 entries per thread, loads first; the grid
// loops when rows x chunks exceeds it.
__global__ __launch_bounds__(256) void pad_kernel(const double* src, i64 lds, i64 r, i64 c, double* dst, i64 ldd,
                                                   i64 R, i64 C)
{
    const i64 chunks = (C + 1023) / 1024;
    for (i64 vb = blockIdx.x; vb < R * chunks; vb += gridDim.x) {
        const i64 i = vb / chunks, j0 = (vb - i * chunks) * 1024 + threadIdx.x;
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const i64 j = j0 + u * 256;
            v[u] = (i < r && j < c) ? src[i * lds + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (j0 + u * 256 < C) dst[i * ldd + j0 + u * 256] = v[u];
    }
}

// dst = 2^(sign * lambda) src for a rows x cols block (Section 2.3.2's
// scaled operands), laid out as pad_kernel.  The factor is a power of two,
// so every entry is the exact product (the same value whichever kernel
// applies it).  dst may equal src.
__global__ __launch_bounds__(256) void scale_kernel(const double* src, i64 lds, i64 rows, i64 cols, double* dst,
                                                     i64 ldd, const int* lam, int sign)
{
    const double sc = ldexp(1.0, sign * *lam);
    const i64 chunks = (cols + 1023) / 1024;
    for (i64 vb = blockIdx.x; vb < rows * chunks; vb += gridDim.x) {
        const i64 i = vb / chunks, j0 = (vb - i * chunks) * 1024 + threadIdx.x;
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const i64 j = j0 + u * 256;
            v[u] = j < cols ? src[i * lds + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (j0 + u * 256 < cols) dst[i * ldd + j0 + u * 256] = v[u] * sc;
    }
}

// Both of WinogradScaled's operands in one launch: workgroups below blk_a
// write 2^lambda A, the rest 2^-lambda B, each workgroup taking lambda from
// the two norms itself (the rule above), so no separate lambda launch is
// needed.  Same layout and exact products as scale_kernel.
__device__ __forceinline__ void scale_rows(const double* src, i64 lds, i64 rows, i64 cols, double* dst, i64 ldd,
                                           double sc, i64 first, i64 stride)
{
    const i64 chunks = (cols + 1023) / 1024;
    for (i64 vb = first; vb < rows * chunks; vb += stride) {
        const i64 i = vb / chunks, j0 = (vb - i * chunks) * 1024 + threadIdx.x;
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const i64 j = j0 + u * 256;
            v[u] = j < cols ? src[i * lds + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (j0 + u * 256 < cols) dst[i * ldd + j0 + u * 256] = v[u] * sc;
    }
}

__global__ __launch_bounds__(256) void scale_pair_kernel(const double* srcA, i64 ldsA, i64 rowsA, i64 colsA,
                                                          double* dstA, i64 lddA, i64 blk_a, const double* srcB,
                                                          i64 ldsB, i64 rowsB, i64 colsB, double* dstB, i64 lddB,
                                                          const double* nA, const double* nB)
{
    const int lam = winograd_lambda(*nA, *nB);
    const i64 b = blockIdx.x;
    if (b < blk_a) scale_rows(srcA, ldsA, rowsA, colsA, dstA, lddA, ldexp(1.0, lam), b, blk_a);
    else scale_rows(srcB, ldsB, rowsB, colsB, dstB, lddB, ldexp(1.0, -lam), b - blk_a, (i64)gridDim.x - blk_a);
}

__global__ __launch_bounds__(256) void zero_kernel(double* dst, i64 n)
{
    for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < n; e += (i64)gridDim.x * 256) dst[e] = 0.0;
}

// Two independent reductions in one launch (workgroups below nblk1 take the
// first, the rest the second), so each fills the CUs the other leaves idle.
template <int OP, bool COLS1, bool COLS2, bool FOLD_MAX>
__global__ __launch_bounds__(256) void vecred_pair_kernel(const double* __restrict__ X1, i64 ld1, i64 nvec1,
                                                          i64 len1, double* __restrict__ out1, i64 nblk1,
                                                          const double* __restrict__ X2, i64 ld2, i64 nvec2,
                                                          i64 len2, double* __restrict__ out2)
{
    __shared__ double T[2][RV][RL + 1];
    const i64 b = blockIdx.x;
    if (b < nblk1) vecred_body<OP, COLS1, FOLD_MAX>(X1, ld1, nvec1, len1, out1, b, T);
    else vecred_body<OP, COLS2, FOLD_MAX>(X2, ld2, nvec2, len2, out2, b - nblk1, T);
}

template <int OP, bool COLS1, bool COLS2, bool FOLD_MAX>
hipError_t launch_pair(const double* X1, i64 ld1, i64 nvec1, i64 len1, double* out1, const double* X2, i64 ld2,
                       i64 nvec2, i64 len2, double* out2, hipStream_t s)
{
    const i64 nb1 = cdiv(nvec1, RV), nb2 = cdiv(nvec2, RV);
    if (nb1 + nb2 == 0) return hipSuccess;
    if (nb1 + nb2 > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((vecred_pair_kernel<OP, COLS1, COLS2, FOLD_MAX>), dim3((unsigned)(nb1 + nb2)), dim3(256), 0, s,
                       X1, ld1, nvec1, len1, out1, nb1, X2, ld2, nvec2, len2, out2);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_elementwise(EwOp op, const double* A, const double* B, double alpha, double* C, i64 n,
                              hipStream_t s)
{
    if (op == EW_PLUS) return launch_ew<EW_PLUS>(A, B, alpha, C, n, s);
    if (op == EW_MINUS) return launch_ew<EW_MINUS>(A, B, alpha, C, n, s);
    return launch_ew<EW_SCALE>(A, B, alpha, C, n, s);
}

hipError_t launch_norm_inf(const double* X, i64 rows, i64 cols, double* out, hipStream_t s)
{
    hipError_t e = launch_fill_zero(out, 1, s);
    if (e != hipSuccess || rows <= 0) return e;
    hipLaunchKernelGGL((vecred_kernel<RED_ABS_SUM, false, true>), dim3((unsigned)cdiv(rows, RV)), dim3(256), 0, s, X,
                       cols, rows, cols, out);
    return hipGetLastError();
}

hipError_t launch_norm_inf_pair(const double* A, i64 N, i64 P, double* nA, const double* B, i64 M, double* nB,
                                hipStream_t s)
{
    hipError_t e = launch_fill_zero(nA, 1, s);
    if (e == hipSuccess) e = launch_fill_zero(nB, 1, s);
    if (e != hipSuccess) return e;
    return launch_pair<RED_ABS_SUM, false, false, true>(A, P, N, P, nA, B, M, P, M, nB, s);
}

hipError_t launch_winograd_yz(const double* A, i64 lda, i64 N, i64 P, double* y, const double* B, i64 ldb, i64 M,
                              double* z, hipStream_t s)
{
    return launch_pair<RED_PAIR_SUM, false, true, false>(A, lda, N, P, y, B, ldb, M, P, z, s);
}

hipError_t launch_lambda(const double* nA, const double* nB, int* lam, hipStream_t s)
{
    hipLaunchKernelGGL(lambda_kernel, dim3(1), dim3(1), 0, s, nA, nB, lam);
    return hipGetLastError();
}

hipError_t launch_pad_copy(const double* src, i64 lds, i64 r, i64 c, double* dst, i64 ldd, i64 R, i64 C,
                           hipStream_t s)
{
    if (R <= 0 || C <= 0) return hipSuccess;
    hipLaunchKernelGGL(pad_kernel, dim3(grid_for(R * cdiv(C, 1024) * 256, 1)), dim3(256), 0, s, src, lds, r, c, dst, ldd,
                       R, C);
    return hipGetLastError();
}

hipError_t launch_scale_pow2(const double* src, i64 lds, i64 rows, i64 cols, double* dst, i64 ldd, const int* lam,
                             int sign, hipStream_t s)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(rows * cdiv(cols, 1024) * 256, 1)), dim3(256), 0, s, src, lds, rows,
                       cols, dst, ldd, lam, sign);
    return hipGetLastError();
}

hipError_t launch_scale_pow2_pair(const double* srcA, i64 ldsA, i64 rowsA, i64 colsA, double* dstA, i64 lddA,
                                  const double* srcB, i64 ldsB, i64 rowsB, i64 colsB, double* dstB, i64 lddB,
                                  const double* nA, const double* nB, hipStream_t s)
{
    // each half at most 2^30 workgroups (they loop beyond), so the sum fits the grid
    const i64 ba = rowsA > 0 && colsA > 0 ? std::min<i64>(grid_for(rowsA * cdiv(colsA, 1024) * 256, 1), 1 << 30) : 0;
    const i64 bb = rowsB > 0 && colsB > 0 ? std::min<i64>(grid_for(rowsB * cdiv(colsB, 1024) * 256, 1), 1 << 30) : 0;
    if (ba + bb == 0) return hipSuccess;
    hipLaunchKernelGGL(scale_pair_kernel, dim3((unsigned)(ba + bb)), dim3(256), 0, s, srcA, ldsA, rowsA, colsA, dstA,
                       lddA, ba, srcB, ldsB, rowsB, colsB, dstB, lddB, nA, nB);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* dst, i64 n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    i64 blocks = cdiv(n, 256 * 4);
    if (blocks > 256 * 16) blocks = 256 * 16;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, n);
    return hipGetLastError();
}

}  // namespace mmm
