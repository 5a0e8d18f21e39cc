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
        // leaves whose operand would be a misaligned view of the root get a copy
        if (level == T.depth && (IS_B ? T.copy_leaf_views_b : T.copy_leaf_views_a)) {
            const double xq[4] = {x11, x12, x21, x22};
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                const int quad = IS_B ? view_quadrant_b(VARIANT, c) : view_quadrant_a(VARIANT, c);
                if (quad >= 0) W[c * sz + e] = xq[quad];
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

// Operand of child c (0..6, i.e. H_{c+1}) from the four quadrant entries
// of its parent's operand, exactly as the single-level kernel forms it (a
// view child returns its quadrant entry).
template <int VARIANT, bool IS_B>
__device__ __forceinline__ double child_value(int c, double x11, double x12, double x21, double x22)
{
    if (VARIANT == 0) {
        if (!IS_B) {
            switch (c) {
            case 0: return x11 + x22;
            case 1: return x21 + x22;
            case 2: return x11;
            case 3: return x22;
            case 4: return x11 + x12;
            case 5: return x21 - x11;
            default: return x12 - x22;
            }
        }
        switch (c) {
        case 0: return x11 + x22;
        case 1: return x11;
        case 2: return x12 - x22;
        case 3: return x21 - x11;
        case 4: return x22;
        case 5: return x11 + x12;
        default: return x21 + x22;
        }
    }
    if (!IS_B) {
        const double a1 = x11 - x21;
        const double a2 = x22 - a1;
        switch (c) {
        case 0: return x11;
        case 1: return x12;
        case 2: return a2;
        case 3: return x21 + x22;
        case 4: return a1;
        case 5: return x12 - a2;
        default: return x22;
        }
    }
    const double b1 = x22 - x12;
    const double b2 = b1 + x11;
    switch (c) {
    case 0: return x11;
    case 1: return x21;
    case 2: return b2;
    case 3: return x12 - x11;
    case 4: return b1;
    case 5: return x22;
    default: return x21 - b2;
    }
}

// The four result quadrants of a node from its seven child products, as
// the single-level post-kernel forms them.
template <int VARIANT>
__device__ __forceinline__ void fold_products(const double (&h)[7], double& c11, double& c12, double& c21,
                                              double& c22)
{
    if (VARIANT == 0) {
        c11 = ((h[0] + h[3]) - h[4]) + h[6];
        c12 = h[2] + h[4];
        c21 = h[1] + h[3];
        c22 = ((h[0] + h[2]) - h[1]) + h[5];
    } else {
        const double h8 = h[0] + h[2];
        const double h9 = h8 + h[3];
        c11 = h[0] + h[1];
        c12 = h9 + h[5];
        c21 = (h8 + h[4]) + h[6];
        c22 = h9 + h[4];
    }
}

// W adjacent entries of a row (W = 1, or 2 when rows, strides and bases are
// even and 16-byte aligned): one load or store per W entries
template <int W>
struct Vec;
template <>
struct Vec<1> {
    typedef double T;
    __device__ static T ld(const double* p) { return *p; }
    __device__ static void st(double* p, T v) { *p = v; }
    __device__ static double get(const T& v, int) { return v; }
    __device__ static void set(T& v, int, double x) { v = x; }
};
template <>
struct Vec<2> {
    typedef double2 T;
    __device__ static T ld(const double* p) { return *reinterpret_cast<const double2*>(p); }
    __device__ static void st(double* p, T v) { *reinterpret_cast<double2*>(p) = v; }
    __device__ static double get(const T& v, int k) { return k ? v.y : v.x; }
    __device__ static void set(T& v, int k, double x) { (k ? v.y : v.x) = x; }
};

// Levels f and f + 1 in one pass: for every node of level f - 1, each
// thread reads the 16 entries of the node's operand that one position of a
// level-(f+1) block touches (W adjacent positions at a time), forms the
// 7 x 4 level-f operand entries in registers (level f is never written)
// and writes the level-(f+1) operands that are not views of the node's own
// operand.
template <int VARIANT, bool IS_B, int W>
__device__ __forceinline__ void strassen_pre2_body(const StrassenTree& T, int f, i64 bpp, i64 block)
{
    typedef Vec<W> V;
    const i64 parent = block / bpp;
    const i64 chunk = block - parent * bpp;
    const View par = strassen_operand(T, f - 1, parent, IS_B);
    const i64 rows = IS_B ? T.p[f + 1] : T.n[f + 1];
    const i64 cols = IS_B ? T.m[f + 1] : T.p[f + 1];
    const i64 sz = rows * cols;
    double* W_ = (IS_B ? T.WB[f + 1] : T.WA[f + 1]) + parent * 49 * sz;
    const i64 base = chunk * 256 * EPT + threadIdx.x;
    // leaves whose operand would be a misaligned view of the root get a copy
    const bool copy_views = f + 1 == T.depth && (IS_B ? T.copy_leaf_views_b : T.copy_leaf_views_a);
#pragma unroll 1
    for (int u = 0; u < EPT; ++u) {
        const i64 e = (base + u * 256) * W;
        if (e >= sz) break;
        const i64 r = e / cols, c = e - r * cols;
        const double* q = par.p + r * par.ld + c;
        typename V::T x[4][4];  // x[i][j]: block (i, j) of the 4 x 4 grid of level-(f+1) blocks
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) x[i][j] = V::ld(q + i * rows * par.ld + j * cols);
#pragma unroll
        for (int c1 = 0; c1 < 7; ++c1) {
            typename V::T y[2][2];  // level-f operand of child c1, its quadrant (qi, qj)
#pragma unroll
            for (int qi = 0; qi < 2; ++qi)
#pragma unroll
                for (int qj = 0; qj < 2; ++qj)
#pragma unroll
                    for (int k = 0; k < W; ++k)
                        V::set(y[qi][qj], k,
                               child_value<VARIANT, IS_B>(c1, V::get(x[qi][qj], k), V::get(x[qi][2 + qj], k),
                                                          V::get(x[2 + qi][qj], k), V::get(x[2 + qi][2 + qj], k)));
            const bool v1 = (IS_B ? view_quadrant_b(VARIANT, c1) : view_quadrant_a(VARIANT, c1)) >= 0;
#pragma unroll
            for (int c2 = 0; c2 < 7; ++c2) {
                const bool v2 = (IS_B ? view_quadrant_b(VARIANT, c2) : view_quadrant_a(VARIANT, c2)) >= 0;
                if (v1 && v2 && !copy_views) continue;  // a view of the node's own operand
                typename V::T o;
#pragma unroll
                for (int k = 0; k < W; ++k)
                    V::set(o, k, child_value<VARIANT, IS_B>(c2, V::get(y[0][0], k), V::get(y[0][1], k),
                                                            V::get(y[1][0], k), V::get(y[1][1], k)));
                V::st(W_ + (c1 * 7 + c2) * sz + e, o);
            }
        }
    }
}

// Both operands' fused pre-passes in one launch: workgroups below blocks_a
// take A's nodes, the rest B's, so the second operand's workgroups fill the
// CUs the first leaves idle at its tail.
template <int VARIANT, int W>
__global__ __launch_bounds__(256) void strassen_pre2_kernel(StrassenTree T, int f, i64 bpp_a, i64 blocks_a, i64 bpp_b)
{
    const i64 b = blockIdx.x;
    if (b < blocks_a) strassen_pre2_body<VARIANT, false, W>(T, f, bpp_a, b);
    else strassen_pre2_body<VARIANT, true, W>(T, f, bpp_b, b - blocks_a);
}

// Levels f + 1 and f folded in one pass: for every node of level f - 1,
// each thread reads its 49 grandchild products at one position (W adjacent
// positions at a time), forms the 7 x 4 level-f product entries in
// registers (level f is never written) and writes the 16 entries of the
// node's product that position feeds.
template <int VARIANT, int W>
__global__ __launch_bounds__(256) void strassen_post2_kernel(StrassenTree T, int f, i64 bpp, double* C, i64 ldc)
{
    typedef Vec<W> V;
    const i64 parent = blockIdx.x / bpp;
    const i64 chunk = blockIdx.x - parent * bpp;
    const i64 rows = T.n[f + 1], cols = T.m[f + 1];
    const i64 sz = rows * cols;
    const double* H = T.H[f + 1] + parent * 49 * sz;
    double* out;
    i64 ld;
    if (f - 1 >= 1) {
        out = T.H[f - 1] + parent * T.n[f - 1] * T.m[f - 1];
        ld = T.m[f - 1];
    } else {
        out = C;
        ld = ldc;
    }
    const i64 base = chunk * 256 * EPT + threadIdx.x;
#pragma unroll 1
    for (int u = 0; u < EPT; ++u) {
        const i64 e = (base + u * 256) * W;
        if (e >= sz) break;
        const i64 r = e / cols, c = e - r * cols;
        double z[7][2][2][W];  // level-f product of child c1, its quadrant (qi, qj), position k
#pragma unroll
        for (int c1 = 0; c1 < 7; ++c1) {
            typename V::T hv[7];
#pragma unroll
            for (int c2 = 0; c2 < 7; ++c2) hv[c2] = V::ld(H + (c1 * 7 + c2) * sz + e);
#pragma unroll
            for (int k = 0; k < W; ++k) {
                double h[7];
#pragma unroll
                for (int c2 = 0; c2 < 7; ++c2) h[c2] = V::get(hv[c2], k);
                fold_products<VARIANT>(h, z[c1][0][0][k], z[c1][0][1][k], z[c1][1][0][k], z[c1][1][1][k]);
            }
        }
        double* o = out + r * ld + c;
#pragma unroll
        for (int qi = 0; qi < 2; ++qi)
#pragma unroll
            for (int qj = 0; qj < 2; ++qj) {
                typename V::T c11, c12, c21, c22;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    double h[7];
#pragma unroll
                    for (int c1 = 0; c1 < 7; ++c1) h[c1] = z[c1][qi][qj][k];
                    double v11, v12, v21, v22;
                    fold_products<VARIANT>(h, v11, v12, v21, v22);
                    V::set(c11, k, v11);
                    V::set(c12, k, v12);
                    V::set(c21, k, v21);
                    V::set(c22, k, v22);
                }
                V::st(o + qi * rows * ld + qj * cols, c11);
                V::st(o + qi * rows * ld + (2 + qj) * cols, c12);
                V::st(o + (2 + qi) * rows * ld + qj * cols, c21);
                V::st(o + (2 + qi) * rows * ld + (2 + qj) * cols, c22);
            }
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

namespace mmm {

// Two entries per position when every row length, stride and base the
// fused passes touch at levels up to f + 1 is even and 16-byte aligned.
bool strassen_pairs_ok(const StrassenTree& T, int f, const double* C, i64 ldc)
{
    auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    if (!al(T.A) || !al(T.B) || (T.lda & 1) || (T.ldb & 1)) return false;
    if (C && (!al(C) || (ldc & 1))) return false;
    for (int e = 1; e <= f + 1 && e <= T.depth; ++e)
        if ((T.n[e] | T.p[e] | T.m[e]) & 1) return false;
    return true;
}

hipError_t launch_strassen_pre2(const StrassenTree& T, int f, hipStream_t s)
{
    const i64 parents = pow7(f - 1);
    const bool pairs = strassen_pairs_ok(T, f, nullptr, 0);
    const i64 sz_a = T.n[f + 1] * T.p[f + 1], sz_b = T.p[f + 1] * T.m[f + 1];
    const i64 bpp_a = cdiv(pairs ? sz_a / 2 : sz_a, 256 * EPT), bpp_b = cdiv(pairs ? sz_b / 2 : sz_b, 256 * EPT);
    const i64 blocks_a = parents * bpp_a, blocks = blocks_a + parents * bpp_b;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 g((unsigned)blocks), b(256);
#define MMM_PRE2(V, W) hipLaunchKernelGGL((strassen_pre2_kernel<V, W>), g, b, 0, s, T, f, bpp_a, blocks_a, bpp_b)
    if (pairs) {
        if (T.variant == 0) MMM_PRE2(0, 2);
        else MMM_PRE2(1, 2);
    } else {
        if (T.variant == 0) MMM_PRE2(0, 1);
        else MMM_PRE2(1, 1);
    }
#undef MMM_PRE2
    return hipGetLastError();
}

hipError_t launch_strassen_post2(const StrassenTree& T, int f, double* C, i64 ldc, hipStream_t s)
{
    const i64 parents = pow7(f - 1);
    const i64 sz = T.n[f + 1] * T.m[f + 1];
    const bool pairs = strassen_pairs_ok(T, f, f - 1 >= 1 ? nullptr : C, ldc);
    const i64 bpp = cdiv(pairs ? sz / 2 : sz, 256 * EPT);
    const i64 blocks = parents * bpp;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 g((unsigned)blocks), b(256);
    if (pairs) {
        if (T.variant == 0) hipLaunchKernelGGL((strassen_post2_kernel<0, 2>), g, b, 0, s, T, f, bpp, C, ldc);
        else hipLaunchKernelGGL((strassen_post2_kernel<1, 2>), g, b, 0, s, T, f, bpp, C, ldc);
    } else {
        if (T.variant == 0) hipLaunchKernelGGL((strassen_post2_kernel<0, 1>), g, b, 0, s, T, f, bpp, C, ldc);
        else hipLaunchKernelGGL((strassen_post2_kernel<1, 1>), g, b, 0, s, T, f, bpp, C, ldc);
    }
    return hipGetLastError();
}

}  // namespace mmm
