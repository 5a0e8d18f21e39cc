// Host-side launchers of the gfx950 kernels (internal to libmmm).
#pragma once

#include "common.h"

namespace mmm {

// Zero-padded operand copies for a large product whose tiles fit N and M
// but whose P keeps it off the direct-load kernels (rows of A not 16-byte
// aligned, or K not a whole number of steps): A' is N x kp (leading
// dimension kp, zero beyond column P), B' is kp x M (zero beyond row P) when
// copy_b.  zero_k: the product runs over all kp columns, which only adds
// exact zeros to naive sums; otherwise it stops at P and kp bounds the
// columns a last partial step may load (Gemm::kcap).  kp == 0: no copies.
struct ValuPad {
    i64 kp;
    bool copy_b;
    bool zero_k;
};
// Problems below this many multiply-adds (N P M) are not worth the copies.
constexpr double kPadMinWork = 4294967296.0;
enum ValuKind {
    VK_NAIVE = 0,
    VK_NAIVE_FMA,
    VK_KAHAN,
    VK_WINOGRAD,
    VK_ON_ARRAY,
    VK_UNROLL2,
    VK_UNROLL3,
    VK_UNROLL4,
    VK_DOT2,
};

// valu_gemm.hip
// The copies a product of this kind and shape takes (shape only: pointers
// are unknown when the workspace is sized).
ValuPad valu_pad_plan(ValuKind kind, i64 N, i64 P, i64 M);
hipError_t launch_naive(const Gemm& g, bool fused, hipStream_t s);
hipError_t launch_naive_strassen_leaves(const StrassenLeafSrc& src, hipStream_t s);
hipError_t launch_kahan(const Gemm& g, hipStream_t s);
// NaivOnArray (variant 0), NaivLoopUnrollingTwo/Three/Four (variant 2/3/4) or
// compensated dot products (variant 5)
hipError_t launch_naive_variant(const Gemm& g, int variant, hipStream_t s);
// WinogradOriginal's main loop and odd-P tail on operands g (WinogradScaled
// passes its materialised 2^lambda A, 2^-lambda B): C = pairs - y - z (+ tail).
hipError_t launch_winograd_main(const Gemm& g, const double* y, const double* z, hipStream_t s);

// dgemm.hip
ValuPad dgemm_pad_plan(i64 N, i64 P, i64 M);
hipError_t launch_dgemm(const Gemm& g, hipStream_t s);
hipError_t launch_dgemm_strassen_leaves(const StrassenLeafSrc& src, hipStream_t s);

// aux.hip
enum EwOp { EW_PLUS = 0, EW_MINUS = 1, EW_SCALE = 2 };
hipError_t launch_elementwise(EwOp op, const double* A, const double* B, double alpha, double* C, i64 n,
                              hipStream_t s);

// Sequential reductions of the rows or columns of a row-major matrix:
//   RED_ABS_SUM   out[v] = sum_q |x_q|            (q ascending, from 0.0)
//   RED_PAIR_SUM  out[v] = sum_p x_{2p} x_{2p+1}  (p ascending, from 0.0)
enum RedOp { RED_ABS_SUM = 0, RED_PAIR_SUM = 1 };
// Section 1.4: *out = max_i sum_j |X_ij| (row sums sequential in j).
hipError_t launch_norm_inf(const double* X, i64 rows, i64 cols, double* out, hipStream_t s);
// Both NormInfs of an A (N x P) and B (P x M) in one launch.
hipError_t launch_norm_inf_pair(const double* A, i64 N, i64 P, double* nA, const double* B, i64 M, double* nB,
                                hipStream_t s);
// Winograd's y (pair sums along the rows of A, N x P, leading dim lda) and z
// (pair sums down the columns of B, P x M, leading dim ldb) in one launch.
hipError_t launch_winograd_yz(const double* A, i64 lda, i64 N, i64 P, double* y, const double* B, i64 ldb, i64 M,
                              double* z, hipStream_t s);
hipError_t launch_lambda(const double* nA, const double* nB, int* lam, hipStream_t s);
// Copy an r x c block (leading dims lds/ldd) into the top-left of an
// R x C destination whose remaining entries are set to zero.
hipError_t launch_pad_copy(const double* src, i64 lds, i64 r, i64 c, double* dst, i64 ldd, i64 R, i64 C,
                           hipStream_t s);
hipError_t launch_fill_zero(double* dst, i64 n, hipStream_t s);
// dst = 2^(sign * *lam) src, rows x cols (leading dims lds / ldd; lam on
// the device); dst may equal src.
hipError_t launch_scale_pow2(const double* src, i64 lds, i64 rows, i64 cols, double* dst, i64 ldd, const int* lam,
                             int sign, hipStream_t s);
// Both scaled operands of WinogradScaled in one launch (2^lambda A and
// 2^-lambda B, lambda from the device norms nA, nB by Section 2.3.2's rule).
hipError_t launch_scale_pow2_pair(const double* srcA, i64 ldsA, i64 rowsA, i64 colsA, double* dstA, i64 lddA,
                                  const double* srcB, i64 ldsB, i64 rowsB, i64 colsB, double* dstB, i64 lddB,
                                  const double* nA, const double* nB, hipStream_t s);

// strassen.hip
hipError_t launch_strassen_pre(const StrassenTree& T, int level, hipStream_t s);
hipError_t launch_strassen_post(const StrassenTree& T, int level, double* C, i64 ldc, hipStream_t s);
// Levels f and f + 1 of the recursion in one pass each way (level f is never
// written): operand sums of levels f and f + 1 from the operands of level
// f - 1, and the products of level f - 1 from those of level f + 1.
hipError_t launch_strassen_pre2(const StrassenTree& T, int f, hipStream_t s);
hipError_t launch_strassen_post2(const StrassenTree& T, int f, double* C, i64 ldc, hipStream_t s);

}  // namespace mmm
