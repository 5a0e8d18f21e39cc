// Internal declarations shared by the gfx950 kernels of libmmm.
//
// Everything here is device-side plumbing: problem descriptors with leading
// dimensions, the resolver that locates the operands of a Strassen node by
// walking its base-7 path, and launch helpers.  The arithmetic of each
// method lives in the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mmm.h"

namespace mmm {

typedef int64_t i64;

// One product C = A B with leading dimensions (row-major views).
struct Gemm {
    const double* A;
    i64 lda;
    const double* B;
    i64 ldb;
    double* C;
    i64 ldc;
    i64 N, P, M;
    // columns of A (and rows of B) that may be read, >= P: larger when the
    // operands are zero-padded copies, which lets the direct-load kernels
    // load a whole last K step (0 means P)
    i64 kcap;
    // DGEMM kernels only: 1 = C <- C + A B (the product added to C with one
    // rounding per entry) instead of C <- A B
    int accumulate;
};

// A single product: every workgroup works on the same problem.
struct SingleSrc {
    Gemm g;
    __host__ __device__ i64 count() const { return 1; }
    __device__ Gemm get(i64) const { return g; }
};

constexpr int kMaxDepth = 12;

// The Strassen recursion laid out breadth first.  Level d (1..depth) has
// 7^d nodes; node q at level d is child c = q % 7 of node q / 7 at level
// d-1.  Child c of a node computes the product H_{c+1} of the paper's list
// for that variant.  Operands of a child are either a quadrant of the
// parent's operand (a view, no copy) or a sum materialised by the level's
// pre-kernel in slot (q) of WA[d] / WB[d], each slot dense with leading
// dimension p[d] (A side) or m[d] (B side).  Products of level d live in
// H[d], node q at H[d] + q * n[d] * m[d], dense.
struct StrassenTree {
    int variant;  // 0 StrassenNaiv, 1 StrassenWinograd
    int depth;
    int fused;    // level whose sums and products are never written (0 = none): formed in registers by the
                  // two-level kernels of levels fused and fused + 1
    const double* A;
    i64 lda;
    const double* B;
    i64 ldb;
    // leaf operands that are quadrant views of the root are instead written
    // to their level slots (A side, B side): set when the root's rows are
    // not 16-byte aligned, so the leaf product can still load them directly
    bool copy_leaf_views_a, copy_leaf_views_b;
    i64 n[kMaxDepth + 1], p[kMaxDepth + 1], m[kMaxDepth + 1];
    double* WA[kMaxDepth + 1];
    double* WB[kMaxDepth + 1];
    double* H[kMaxDepth + 1];
};

// Which children take a quadrant of the parent's operand unchanged, and
// which quadrant (0 = X11, 1 = X12, 2 = X21, 3 = X22); -1 = materialised.
//   StrassenNaiv:     H3 = A11 (..), H4 = A22 (..); H2 = (..) B11, H5 = (..) B22
//   StrassenWinograd: H1 = A11 B11, H2 = A12 B21, H6 = (..) B22, H7 = A22 (..)
__host__ __device__ inline int view_quadrant_a(int variant, int c)
{
    if (variant == 0) return c == 2 ? 0 : (c == 3 ? 3 : -1);
    return c == 0 ? 0 : (c == 1 ? 1 : (c == 6 ? 3 : -1));
}
__host__ __device__ inline int view_quadrant_b(int variant, int c)
{
    if (variant == 0) return c == 1 ? 0 : (c == 4 ? 3 : -1);
    return c == 0 ? 0 : (c == 1 ? 2 : (c == 5 ? 3 : -1));
}

struct View {
    const double* p;
    i64 ld;
};

// Operand of node q at level d (A side when is_b is false).  A child takes
// a view of its parent's operand only when that operand exists in memory;
// below the fused level (whose sums live only in registers) every child is
// materialised.  Never called for the fused level itself.
__device__ inline View strassen_operand(const StrassenTree& T, int d, i64 q, bool is_b)
{
    View v{is_b ? T.B : T.A, is_b ? T.ldb : T.lda};
    // digits of q, most significant first
    i64 pw = 1;
    for (int e = 1; e < d; ++e) pw *= 7;
    i64 prefix = 0;
    bool virt = false;  // the operand so far exists only in registers
    for (int e = 1; e <= d; ++e) {
        const int c = (int)((q / pw) % 7);
        pw /= 7;
        const int quad = is_b ? view_quadrant_b(T.variant, c) : view_quadrant_a(T.variant, c);
        const i64 rows = is_b ? T.p[e] : T.n[e];
        const i64 cols = is_b ? T.m[e] : T.p[e];
        const bool copied = e == T.depth && (is_b ? T.copy_leaf_views_b : T.copy_leaf_views_a);
        if (quad >= 0 && !virt && !copied) {
            v.p += (quad >> 1) * rows * v.ld + (quad & 1) * cols;
        } else if (e == T.fused) {
            virt = true;
        } else {
            v.p = (is_b ? T.WB[e] : T.WA[e]) + (prefix * 7 + c) * rows * cols;
            v.ld = cols;
            virt = false;
        }
        prefix = prefix * 7 + c;
    }
    return v;
}

// The 7^depth leaf products of a Strassen tree as a batch.
struct StrassenLeafSrc {
    StrassenTree T;
    i64 leaves;
    __host__ __device__ i64 count() const { return leaves; }
    __device__ Gemm get(i64 q) const
    {
        const int d = T.depth;
        View a = strassen_operand(T, d, q, false);
        View b = strassen_operand(T, d, q, true);
        Gemm g{};  // every field set: no kcap, no accumulation
        g.A = a.p;
        g.lda = a.ld;
        g.B = b.p;
        g.ldb = b.ld;
        g.C = T.H[d] + q * T.n[d] * T.m[d];
        g.ldc = T.m[d];
        g.N = T.n[d];
        g.P = T.p[d];
        g.M = T.m[d];
        return g;
    }
};

// Blocks of a 2-D tiling of every problem of a batch of equal shapes,
// flattened into blockIdx.x (grid y and z are limited to 65535).
__device__ inline void flat_tile(i64 tiles_m, i64 tiles_n, i64& prob, i64& tm, i64& tn)
{
    const i64 b = blockIdx.x;
    const i64 per = tiles_m * tiles_n;
    prob = b / per;
    const i64 r = b - prob * per;
    tm = r / tiles_n;
    tn = r - tm * tiles_n;
}

inline i64 cdiv(i64 a, i64 b) { return (a + b - 1) / b; }

// Record a message for mmm_last_error (thread local) and return `st`.
mmm_status set_error(mmm_status st, const char* fmt, ...);
// MMM_OK when every field of the config is valid (message set otherwise).
mmm_status check_config(const mmm_config& c);

// Kernel timer (mmm_timer_start / mmm_timer_stop): while it is on for the
// calling thread, the launch of each call's dominant kernel is bracketed by
// a pair of HIP events recorded on the stream it runs on.
void timer_begin(hipStream_t s);
void timer_end(hipStream_t s);

}  // namespace mmm
