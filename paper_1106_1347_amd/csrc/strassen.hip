// Block additions of Strassen's algorithm (Section 2.4), breadth first.
//
// Level e of the recursion holds 7^e nodes.  For every node of level e-1
// the pre-kernel forms, in one pass over the four quadrants of its
// operands, the operand sums its seven children need (StrassenNaiv: five on
// each side; StrassenWinograd: four on each side, A1, A2, B1, B2 included),
// writing them to the children's slots; the remaining children take a
// quadrant unchanged (see view_quadrant_a / view_quadrant_b).  After the 7^L
// leaf products, the post-kernel of level e folds the seven child products
// of each node of level e-1 into that node's four result quadrants.
//
// Each entry is one chain of additions evaluated left to right as printed
// (built with -ffp-contract=off), so every intermediate equals the
// sequential evaluation bit for bit.  The kernels are bound by HBM (or
// Infinity Cache) bandwidth: per entry of a quadrant the StrassenWinograd
// pre-kernel moves 4 reads + 4 writes per operand side, the post-kernel 7
// reads + 4 writes.
#include "common.h"
#include "launch.h"

namespace mmm {

namespace {

constexpr int EPT = 4;  // entries per thread

template <int VARIANT, bool IS_B>
__global__ __launch_bounds__(256) void strassen_pre_kernel(StrassenTree T, int level, i64 bpp)
{
    const i64 parent = blockIdx.x / bpp;
    const i64 chunk = blockIdx.x - parent * bpp;
    const View par = strassen_operand(T, level - 1, parent, IS_B);
    const i64 rows = IS_B ? T.p[level] : T.n[level];
    const i64 cols = IS_B ? T.m[level] : T.p[level];
    const i64 sz = rows * cols;
    double* W = (IS_B ? T.WB[level] : T.WA[level]) + parent * 7 * sz;
    const i64 base = chunk * 256 * EPT + threadIdx.x;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const i64 e = base + u * 256;
        if (e >= sz) break;
        const i64 r = e / cols, c = e - r * cols;
        const double* q = par.p + r * par.ld + c;
        const double x11 = q[0];
        const double x12 = q[cols];
        const double x21 = q[rows * par.ld];
        const double x22 = q[rows * par.ld + cols];
        if (VARIANT == 0) {
            if (!IS_B) {
                W[0 * sz + e] = x11 + x22;  // H1 = (A11 + A22)(..)
                W[1 * sz + e] = x21 + x22;  // H2 = (A21 + A22) B11
                W[4 * sz + e] = x11 + x12;  // H5 = (A11 + A12) B22
                W[5 * sz + e] = x21 - x11;  // H6 = (A21 - A11)(..)
                W[6 * sz + e] = x12 - x22;  // H7 = (A12 - A22)(..)
            } else {
                W[0 * sz + e] = x11 + x22;  // H1 = (..)(B11 + B22)
                W[2 * sz + e] = x12 - x22;  // H3 = A11 (B12 - B22)
                W[3 * sz + e] = x21 - x11;  // H4 = A22 (B21 - B11)
                W[5 * sz + e] = x11 + x12;  // H6 = (..)(B11 + B12)
                W[6 * sz + e] = x21 + x22;  // H7 = (..)(B21 + B22)
            }
        } else {
            if (!IS_B) {
                const double a1 = x11 - x21;  // A1 = A11 - A21
                const double a2 = x22 - a1;   // A2 = A22 - A1
                W[2 * sz + e] = a2;           // H3 = A2 B2
                W[3 * sz + e] = x21 + x22;    // H4 = (A21 + A22)(..)
                W[4 * sz + e] = a1;           // H5 = A1 B1
                W[5 * sz + e] = x12 - a2;     // H6 = (A12 - A2) B22
            } else {
                const double b1 = x22 - x12;  // B1 = B22 - B12
                const double b2 = b1 + x11;   // B2 = B1 + B11
                W[2 * sz + e] = b2;           // H3 = A2 B2
                W[3 * sz + e] = x12 - x11;    // H4 = (..)(B12 - B11)
                W[4 * sz + e] = b1;           // H5 = A1 B1
                W[6 * sz + e] = x21 - b2;     // H7 = A22 (B21 - B2)
            }
        }
    }
}

template <int VARIANT>
__global__ __launch_bounds__(256) void strassen_post_kernel(StrassenTree T, int level, i64 bpp, double* C, i64 ldc)
{
    const i64 parent = blockIdx.x / bpp;
    const i64 chunk = blockIdx.x - parent * bpp;
    const i64 rows = T.n[level], cols = T.m[level];
    const i64 sz = rows * cols;
    const double* H = T.H[level] + parent * 7 * sz;
    double* out;
    i64 ld;
    if (level - 1 >= 1) {
        out = T.H[level - 1] + parent * T.n[level - 1] * T.m[level - 1];
        ld = T.m[level - 1];
    } else {
        out = C;
        ld = ldc;
    }
    const i64 base = chunk * 256 * EPT + threadIdx.x;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const i64 e = base + u * 256;
        if (e >= sz) break;
        const i64 r = e / cols, c = e - r * cols;
        const double h1 = H[0 * sz + e], h2 = H[1 * sz + e], h3 = H[2 * sz + e], h4 = H[3 * sz + e];
        const double h5 = H[4 * sz + e], h6 = H[5 * sz + e], h7 = H[6 * sz + e];
        double c11, c12, c21, c22;
        if (VARIANT == 0) {
            c11 = ((h1 + h4) - h5) + h7;
            c12 = h3 + h5;
            c21 = h2 + h4;
            c22 = ((h1 + h3) - h2) + h6;
        } else {
            const double h8 = h1 + h3;
            const double h9 = h8 + h4;
            c11 = h1 + h2;
            c12 = h9 + h6;
            c21 = (h8 + h5) + h7;
            c22 = h9 + h5;
        }
        double* o = out + r * ld + c;
        o[0] = c11;
        o[cols] = c12;
        o[rows * ld] = c21;
        o[rows * ld + cols] = c22;
    }
}

i64 pow7(int e)
{
    i64 r = 1;
    for (int i = 0; i < e; ++i) r *= 7;
    return r;
}

}  // namespace

hipError_t launch_strassen_pre(const StrassenTree& T, int level, hipStream_t s)
{
    const i64 parents = pow7(level - 1);
    for (int side = 0; side < 2; ++side) {
        const i64 sz = side ? T.p[level] * T.m[level] : T.n[level] * T.p[level];
        const i64 bpp = cdiv(sz, 256 * EPT);
        const i64 blocks = parents * bpp;
        if (blocks == 0) continue;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
        if (T.variant == 0) {
            if (side)
                hipLaunchKernelGGL((strassen_pre_kernel<0, true>), dim3((unsigned)blocks), dim3(256), 0, s, T, level, bpp);
            else
                hipLaunchKernelGGL((strassen_pre_kernel<0, false>), dim3((unsigned)blocks), dim3(256), 0, s, T, level, bpp);
        } else {
            if (side)
                hipLaunchKernelGGL((strassen_pre_kernel<1, true>), dim3((unsigned)blocks), dim3(256), 0, s, T, level, bpp);
            else
                hipLaunchKernelGGL((strassen_pre_kernel<1, false>), dim3((unsigned)blocks), dim3(256), 0, s, T, level, bpp);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_strassen_post(const StrassenTree& T, int level, double* C, i64 ldc, hipStream_t s)
{
    const i64 parents = pow7(level - 1);
    const i64 sz = T.n[level] * T.m[level];
    const i64 bpp = cdiv(sz, 256 * EPT);
    const i64 blocks = parents * bpp;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    if (T.variant == 0)
        hipLaunchKernelGGL((strassen_post_kernel<0>), dim3((unsigned)blocks), dim3(256), 0, s, T, level, bpp, C, ldc);
    else
        hipLaunchKernelGGL((strassen_post_kernel<1>), dim3((unsigned)blocks), dim3(256), 0, s, T, level, bpp, C, ldc);
    return hipGetLastError();
}

}  // namespace mmm
