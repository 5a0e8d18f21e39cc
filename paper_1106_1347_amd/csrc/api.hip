// C ABI of libmmm (declared in include/mmm.h): argument validation,
// workspace planning and dispatch of the methods to the gfx950 kernels.
// Nothing here computes matrix entries; every entry is produced by a
// kernel.  No call allocates device memory except mmm_batch_create.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "common.h"
#include "launch.h"
#include "split.h"

using namespace mmm;

#include <vector>

namespace {
thread_local char g_err[512] = "";

// Event pairs of the kernel timer: `used` in recording order, `spare` kept
// for reuse after a stop.
struct KernelTimer {
    bool on = false;
    bool failed = false;
    std::vector<hipEvent_t> used, spare;
    ~KernelTimer()
    {
        for (hipEvent_t e : used) (void)hipEventDestroy(e);
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
    }
    void record(hipStream_t s)
    {
        hipEvent_t e = nullptr;
        if (!spare.empty()) {
            e = spare.back();
            spare.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            failed = true;
            return;
        }
        if (hipEventRecord(e, s) != hipSuccess) failed = true;
        used.push_back(e);
    }
};
thread_local KernelTimer g_timer;
}  // namespace

namespace mmm {
void timer_begin(hipStream_t s)
{
    if (g_timer.on) g_timer.record(s);
}
void timer_end(hipStream_t s)
{
    if (g_timer.on) g_timer.record(s);
}
}  // namespace mmm

namespace mmm {

mmm_status set_error(mmm_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

}  // namespace mmm

namespace {

#define fail mmm::set_error

mmm_status from_hip(hipError_t e, const char* what)
{
    if (e == hipSuccess) return MMM_OK;
    return fail(MMM_ELAUNCH, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool overlap(const void* a, size_t abytes, const void* b, size_t bbytes)
{
    if (!a || !b || abytes == 0 || bbytes == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

}  // namespace

mmm_status mmm::check_config(const mmm_config& c)
{
    for (int i = 0; i < 8; ++i)
        if (c.reserved[i] != 0) return fail(MMM_EINVAL, "config: reserved fields must be zero");
    if (c.strassen_levels < 0 || c.strassen_levels > kMaxDepth)
        return fail(MMM_EINVAL, "config: strassen_levels %d outside 0..%d", c.strassen_levels, kMaxDepth);
    if (c.pad_mode != MMM_PAD_PAPER && c.pad_mode != MMM_PAD_LEVELS) return fail(MMM_EINVAL, "config: bad pad_mode");
    if (c.strassen_leaf != MMM_LEAF_DGEMM && c.strassen_leaf != MMM_LEAF_NAIVE)
        return fail(MMM_EINVAL, "config: bad strassen_leaf");
    if (c.split_slices < 1 || c.split_slices > kMaxSlices)
        return fail(MMM_EINVAL, "config: split_slices %d outside 1..%d", c.split_slices, kMaxSlices);
    if (c.split_type != MMM_SLICE_BF16 && c.split_type != MMM_SLICE_FP16 && c.split_type != MMM_SLICE_INT8)
        return fail(MMM_EINVAL, "config: bad split_type");
    if (c.split_scale_lambda != 0 && c.split_scale_lambda != 1) return fail(MMM_EINVAL, "config: bad split_scale_lambda");
    if (c.split_bits != 0 && (c.split_bits < 2 || c.split_bits > (c.split_type == MMM_SLICE_INT8 ? 8 : 9)))
        return fail(MMM_EINVAL, "config: split_bits %d outside 2..%d for this digit type", c.split_bits,
                    c.split_type == MMM_SLICE_INT8 ? 7 : 9);
    if (c.naive_fma != 0 && c.naive_fma != 1) return fail(MMM_EINVAL, "config: bad naive_fma");
    return MMM_OK;
}

namespace {

mmm_status check_cfg(const mmm_config& c) { return mmm::check_config(c); }

// ---- Strassen planning (Section 2.4) ---------------------------------------

struct StrassenPlan {
    int depth = 0;
    bool direct_naive = false;  // paper rule gave k = 0: one naive product
    bool direct_dgemm = false;  // peeling left no core: one DGEMM product
    bool pad = false;
    // peeling (LEVELS mode, DGEMM leaf): the recursion runs on the leading
    // Np x Pp x Mp core of the caller's operands, whose sizes are the largest
    // multiples of its granularity; the leftover columns of A (rows of B),
    // rows of A and columns of B are DGEMM products added or written
    // afterwards
    bool peel = false;
    bool naive_leaf = false;
    i64 Np = 0, Pp = 0, Mp = 0;
    i64 n[kMaxDepth + 1], p[kMaxDepth + 1], m[kMaxDepth + 1];
    size_t off_A = 0, off_B = 0, off_C = 0;
    size_t off_WA[kMaxDepth + 1], off_WB[kMaxDepth + 1], off_H[kMaxDepth + 1];
    size_t bytes = 0;
};

i64 pow7(int e)
{
    i64 r = 1;
    for (int i = 0; i < e; ++i) r *= 7;
    return r;
}

// Returns false when the plan would not fit in 64-bit sizes.
bool plan_strassen(i64 N, i64 P, i64 M, const mmm_config& c, StrassenPlan& pl)
{
    if (c.pad_mode == MMM_PAD_PAPER) {
        // X = max{N,P,M}, k = floor(log2 X) - 4 (at least 0), m = floor(X 2^-k) + 1, Y = m 2^k
        i64 X = N > P ? N : P;
        X = X > M ? X : M;
        int lg = -1;
        for (i64 t = X; t > 0; t >>= 1) ++lg;
        int k = lg - 4;
        if (k < 0) k = 0;
        if (k == 0) {
            pl.direct_naive = true;
            return true;
        }
        if (k > kMaxDepth) return false;
        const i64 mm = (X >> k) + 1;
        pl.depth = k;
        pl.Np = pl.Pp = pl.Mp = mm << k;
        pl.naive_leaf = true;
    } else {
        pl.depth = c.strassen_levels;
        const i64 q = (i64)1 << pl.depth;
        pl.naive_leaf = c.strassen_leaf == MMM_LEAF_NAIVE;
        // the DGEMM leaf takes its direct-load path when the leaf depth is a
        // multiple of 16, so its core P is a multiple of 16 2^L (for P of at
        // least 64 2^L); the naive leaf pads every side to a multiple of 2^L
        // (zero rows and columns), the block split that defines its rounding
        const i64 qp = (!pl.naive_leaf && P >= 64 * q) ? 16 * q : q;
        if (!pl.naive_leaf) {
            // peel instead of padding: the core is what the block split divides
            pl.Np = N / q * q;
            pl.Pp = P / qp * qp;
            pl.Mp = M / q * q;
            if (pl.Np == 0 || pl.Pp == 0 || pl.Mp == 0) {
                pl.direct_dgemm = true;
                return true;
            }
            pl.peel = pl.Np != N || pl.Pp != P || pl.Mp != M;
        } else {
            pl.Np = cdiv(N, q) * q;
            pl.Pp = cdiv(P, qp) * qp;
            pl.Mp = cdiv(M, q) * q;
        }
    }
    pl.pad = pl.Np != N || pl.Pp != P || pl.Mp != M;
    if (pl.peel) pl.pad = false;
    size_t off = 0;
    auto take = [&](double elems) -> size_t {
        const size_t at = off;
        off = align_up(off + (size_t)elems * sizeof(double));
        return at;
    };
    // guard against absurd sizes before doing integer arithmetic
    double total = 0;
    for (int d = 0; d <= pl.depth; ++d) {
        pl.n[d] = pl.Np >> d;
        pl.p[d] = pl.Pp >> d;
        pl.m[d] = pl.Mp >> d;
        if (d > 0)
            total += (double)pow7(d) * ((double)pl.n[d] * pl.p[d] + (double)pl.p[d] * pl.m[d] + (double)pl.n[d] * pl.m[d]);
    }
    total += (double)pl.Np * pl.Pp + (double)pl.Pp * pl.Mp + (double)pl.Np * pl.Mp;
    if (total * 8.0 > 9.0e18) return false;
    if (pl.pad) {
        pl.off_A = take((double)pl.Np * pl.Pp);
        pl.off_B = take((double)pl.Pp * pl.Mp);
        pl.off_C = take((double)pl.Np * pl.Mp);
    }
    // the deepest two levels run fused (run_strassen): level depth - 1's
    // sums and products live only in registers and get no buffers
    const int fused = pl.depth >= 2 ? pl.depth - 1 : 0;
    for (int d = 1; d <= pl.depth; ++d) {
        if (d == fused) {
            pl.off_WA[d] = pl.off_WB[d] = pl.off_H[d] = 0;
            continue;
        }
        const double nodes = (double)pow7(d);
        pl.off_WA[d] = take(nodes * pl.n[d] * pl.p[d]);
        pl.off_WB[d] = take(nodes * pl.p[d] * pl.m[d]);
        pl.off_H[d] = take(nodes * pl.n[d] * pl.m[d]);
    }
    pl.bytes = off;
    return true;
}

mmm_status run_strassen(int variant, const double* A, const double* B, double* C, i64 N, i64 P, i64 M,
                        const StrassenPlan& pl, char* ws, hipStream_t s)
{
    hipError_t e;
    if (pl.direct_naive) return from_hip(launch_naive(Gemm{A, P, B, M, C, M, N, P, M}, false, s), "naive");
    if (pl.direct_dgemm) return from_hip(launch_dgemm(Gemm{A, P, B, M, C, M, N, P, M}, s), "dgemm");
    StrassenTree T;
    memset(&T, 0, sizeof(T));
    T.variant = variant;
    T.depth = pl.depth;
    // the deepest two levels run as one pass each way (level depth - 1 is
    // never written)
    T.fused = pl.depth >= 2 ? pl.depth - 1 : 0;
    double* Croot = C;
    i64 ldc = M;
    if (pl.pad) {
        double* Ap = (double*)(ws + pl.off_A);
        double* Bp = (double*)(ws + pl.off_B);
        if ((e = launch_pad_copy(A, P, N, P, Ap, pl.Pp, pl.Np, pl.Pp, s)) != hipSuccess) return from_hip(e, "pad A");
        if ((e = launch_pad_copy(B, M, P, M, Bp, pl.Mp, pl.Pp, pl.Mp, s)) != hipSuccess) return from_hip(e, "pad B");
        T.A = Ap;
        T.lda = pl.Pp;
        T.B = Bp;
        T.ldb = pl.Mp;
        Croot = (double*)(ws + pl.off_C);
        ldc = pl.Mp;
    } else {
        // the caller's operands (or, when peeling, their leading core): leaf
        // operands that stay views of them need 16-byte aligned rows for the
        // direct-load leaf product, else the sum passes copy them
        T.A = A;
        T.lda = P;
        T.B = B;
        T.ldb = M;
        T.copy_leaf_views_a = !pl.naive_leaf && (((uintptr_t)A & 15) || (P & 1));
        T.copy_leaf_views_b = !pl.naive_leaf && (((uintptr_t)B & 15) || (M & 1));
    }
    for (int d = 0; d <= pl.depth; ++d) {
        T.n[d] = pl.n[d];
        T.p[d] = pl.p[d];
        T.m[d] = pl.m[d];
        if (d > 0 && d != T.fused) {
            T.WA[d] = (double*)(ws + pl.off_WA[d]);
            T.WB[d] = (double*)(ws + pl.off_WB[d]);
            T.H[d] = (double*)(ws + pl.off_H[d]);
        }
    }
    T.H[0] = Croot;  // the depth-0 "leaf" is the whole product
    for (int d = 1; d <= pl.depth; ++d) {
        if (d == T.fused) {
            if ((e = launch_strassen_pre2(T, d, s)) != hipSuccess) return from_hip(e, "strassen pre");
            ++d;
        } else if ((e = launch_strassen_pre(T, d, s)) != hipSuccess) {
            return from_hip(e, "strassen pre");
        }
    }
    StrassenLeafSrc leaves{T, pow7(pl.depth)};
    timer_begin(s);
    e = pl.naive_leaf ? launch_naive_strassen_leaves(leaves, s) : launch_dgemm_strassen_leaves(leaves, s);
    timer_end(s);
    if (e != hipSuccess) return from_hip(e, "strassen leaves");
    for (int d = pl.depth; d >= 1; --d) {
        if (T.fused && d == T.fused + 1) {
            if ((e = launch_strassen_post2(T, T.fused, Croot, ldc, s)) != hipSuccess) return from_hip(e, "strassen post");
            --d;
        } else if ((e = launch_strassen_post(T, d, Croot, ldc, s)) != hipSuccess) {
            return from_hip(e, "strassen post");
        }
    }
    if (pl.pad && (e = launch_pad_copy(Croot, ldc, N, M, C, M, N, M, s)) != hipSuccess) return from_hip(e, "extract C");
    if (pl.peel) {
        // C = A B over the peeled parts, with Nc, Pc, Mc the core sizes:
        //   C[:Nc, :Mc] += A[:Nc, Pc:] B[Pc:, :Mc]   (the leftover inner terms)
        //   C[:Nc, Mc:]  = A[:Nc, :] B[:, Mc:]       (the leftover columns)
        //   C[Nc:, :]    = A[Nc:, :] B               (the leftover rows)
        const i64 Nc = pl.Np, Pc = pl.Pp, Mc = pl.Mp;
        if (Pc < P) {
            Gemm g{A + Pc, P, B + Pc * M, M, C, M, Nc, P - Pc, Mc};
            g.accumulate = 1;
            if ((e = launch_dgemm(g, s)) != hipSuccess) return from_hip(e, "peeled inner terms");
        }
        if (Mc < M && (e = launch_dgemm(Gemm{A, P, B + Mc, M, C + Mc, M, Nc, P, M - Mc}, s)) != hipSuccess)
            return from_hip(e, "peeled columns");
        if (Nc < N && (e = launch_dgemm(Gemm{A + Nc * P, P, B, M, C + Nc * M, M, N - Nc, P, M}, s)) != hipSuccess)
            return from_hip(e, "peeled rows");
    }
    return MMM_OK;
}

// ---- Winograd (Section 2.3) workspace ---------------------------------------

struct WinoLayout {
    size_t y = 0, z = 0, nA = 0, nB = 0, bytes = 0;
};

WinoLayout wino_layout(i64 N, i64 M, bool scaled)
{
    WinoLayout w;
    size_t off = 0;
    w.y = off;
    off = align_up(off + sizeof(double) * (size_t)(N > 0 ? N : 1));
    w.z = off;
    off = align_up(off + sizeof(double) * (size_t)(M > 0 ? M : 1));
    if (scaled) {
        w.nA = off;
        off = align_up(off + sizeof(double));
        w.nB = off;
        off = align_up(off + sizeof(double));
    }
    w.bytes = off;
    return w;
}

// g may point at zero-padded copies of A and B (then g.A != A, g.B != B).
// WinogradScaled materialises 2^lambda A and 2^-lambda B, as the paper does:
// in place in those copies, else at sws (N x P, then P x M); y, z and the
// main loop then run on the scaled operands.
mmm_status run_winograd(const double* A, const double* B, const Gemm& g, bool scaled, char* ws, char* sws,
                        hipStream_t s)
{
    const i64 N = g.N, P = g.P, M = g.M;
    const WinoLayout w = wino_layout(N, M, scaled);
    double* y = (double*)(ws + w.y);
    double* z = (double*)(ws + w.z);
    Gemm gs = g;
    hipError_t e;
    if (scaled) {
        double* nA = (double*)(ws + w.nA);
        double* nB = (double*)(ws + w.nB);
        if ((e = launch_norm_inf_pair(A, N, P, nA, B, M, nB, s)) != hipSuccess) return from_hip(e, "norms");
        double* As = g.A != A ? (double*)g.A : (double*)sws;
        if (g.A == A) {
            gs.A = As;
            gs.lda = P;
            sws += align_up(sizeof(double) * (size_t)N * (size_t)P);
        }
        double* Bs = g.B != B ? (double*)g.B : (double*)sws;
        if (g.B == B) {
            gs.B = Bs;
            gs.ldb = M;
        }
        // 2^lambda A and 2^-lambda B in one launch, lambda taken from the norms there
        if ((e = launch_scale_pow2_pair(g.A, g.lda, N, P, As, gs.lda, g.B, g.ldb, P, M, Bs, gs.ldb, nA, nB, s)) !=
            hipSuccess)
            return from_hip(e, "scale");
    }
    // y_i over the rows of (scaled) A, z_k over the columns of (scaled) B
    if ((e = launch_winograd_yz(gs.A, gs.lda, N, P, y, gs.B, gs.ldb, M, z, s)) != hipSuccess) return from_hip(e, "y, z");
    timer_begin(s);
    e = launch_winograd_main(gs, y, z, s);
    timer_end(s);
    return from_hip(e, "winograd");
}

// The single-kernel methods bracket their one product kernel.
void timer_begin_if(mmm_method m, hipStream_t s)
{
    switch (m) {
    case MMM_NAIVE:
    case MMM_KAHAN:
    case MMM_NAIVE_ON_ARRAY:
    case MMM_NAIVE_UNROLL2:
    case MMM_NAIVE_UNROLL3:
    case MMM_NAIVE_UNROLL4:
    case MMM_DOT2:
    case MMM_DGEMM: timer_begin(s); break;
    default: break;
    }
}

// Bytes of WinogradScaled's scaled operands beyond the padded copies.
size_t scaled_bytes(const ValuPad& p, i64 N, i64 P, i64 M)
{
    if (8.0 * ((double)N * P + (double)P * M) > 9.0e18) return (size_t)-1;
    return (p.kp ? 0 : align_up(sizeof(double) * (size_t)N * (size_t)P)) +
           (p.copy_b ? 0 : align_up(sizeof(double) * (size_t)P * (size_t)M));
}

// ---- zero-padded operand copies (direct loads at a ragged P) ----------------

ValuPad pad_plan(mmm_method method, i64 N, i64 P, i64 M, const mmm_config& c)
{
    switch (method) {
    case MMM_NAIVE: return valu_pad_plan(c.naive_fma ? VK_NAIVE_FMA : VK_NAIVE, N, P, M);
    case MMM_KAHAN: return valu_pad_plan(VK_KAHAN, N, P, M);
    case MMM_NAIVE_ON_ARRAY: return valu_pad_plan(VK_ON_ARRAY, N, P, M);
    case MMM_NAIVE_UNROLL2: return valu_pad_plan(VK_UNROLL2, N, P, M);
    case MMM_NAIVE_UNROLL3: return valu_pad_plan(VK_UNROLL3, N, P, M);
    case MMM_NAIVE_UNROLL4: return valu_pad_plan(VK_UNROLL4, N, P, M);
    case MMM_DOT2: return valu_pad_plan(VK_DOT2, N, P, M);
    case MMM_DGEMM: return dgemm_pad_plan(N, P, M);
    case MMM_WINOGRAD: return valu_pad_plan(VK_WINOGRAD, N, P, M);
    case MMM_WINOGRAD_SCALED: return valu_pad_plan(VK_WINOGRAD, N, P, M);  // the main loop runs unscaled
    default: return ValuPad{0, false, false};
    }
}

size_t pad_a_bytes(const ValuPad& p, i64 N) { return align_up(sizeof(double) * (size_t)N * (size_t)p.kp); }

// (size_t)-1 when the copies could not be addressed
size_t pad_bytes(const ValuPad& p, i64 N, i64 M)
{
    if (!p.kp) return 0;
    if (8.0 * (double)p.kp * ((double)N + (double)M) > 9.0e18) return (size_t)-1;
    return pad_a_bytes(p, N) + (p.copy_b ? align_up(sizeof(double) * (size_t)p.kp * (size_t)M) : 0);
}

// Writes the copies to ws and points g at them.
hipError_t apply_pad(const ValuPad& p, Gemm& g, char* ws, hipStream_t s)
{
    if (!p.kp) return hipSuccess;
    double* Ap = (double*)ws;
    hipError_t e = launch_pad_copy(g.A, g.lda, g.N, g.P, Ap, p.kp, g.N, p.kp, s);
    if (e != hipSuccess) return e;
    if (p.copy_b) {
        double* Bp = (double*)(ws + pad_a_bytes(p, g.N));
        if ((e = launch_pad_copy(g.B, g.ldb, g.P, g.M, Bp, g.M, p.kp, g.M, s)) != hipSuccess) return e;
        g.B = Bp;
        g.ldb = g.M;
    }
    g.A = Ap;
    g.lda = p.kp;
    if (p.zero_k) g.P = p.kp;
    else g.kcap = p.kp;
    return hipSuccess;
}

}  // namespace

extern "C" {

mmm_config mmm_config_default(void)
{
    mmm_config c;
    memset(&c, 0, sizeof(c));
    c.strassen_levels = 2;
    c.pad_mode = MMM_PAD_LEVELS;
    c.strassen_leaf = MMM_LEAF_DGEMM;
    c.split_slices = 6;
    c.split_type = MMM_SLICE_BF16;
    c.split_scale_lambda = 1;
    c.naive_fma = 0;
    return c;
}

size_t mmm_workspace_bytes(mmm_method method, int64_t N, int64_t P, int64_t M, const mmm_config* cfgp)
{
    const mmm_config c = cfgp ? *cfgp : mmm_config_default();
    if (N < 0 || P < 0 || M < 0 || check_cfg(c) != MMM_OK) return (size_t)-1;
    if (N == 0 || M == 0 || P == 0) return 0;
    switch (method) {
    case MMM_NAIVE:
    case MMM_KAHAN:
    case MMM_DGEMM:
    case MMM_NAIVE_ON_ARRAY:
    case MMM_NAIVE_UNROLL2:
    case MMM_NAIVE_UNROLL3:
    case MMM_NAIVE_UNROLL4:
    case MMM_DOT2:
        return pad_bytes(pad_plan(method, N, P, M, c), N, M);
    case MMM_WINOGRAD:
    case MMM_WINOGRAD_SCALED: {
        const ValuPad pl = pad_plan(method, N, P, M, c);
        const size_t pb = pad_bytes(pl, N, M);
        const size_t sb = method == MMM_WINOGRAD_SCALED ? scaled_bytes(pl, N, P, M) : 0;
        if (pb == (size_t)-1 || sb == (size_t)-1) return (size_t)-1;
        return wino_layout(N, M, method == MMM_WINOGRAD_SCALED).bytes + pb + sb;
    }
    case MMM_STRASSEN_NAIVE:
    case MMM_STRASSEN_WINOGRAD: {
        StrassenPlan pl;
        if (!plan_strassen(N, P, M, c, pl)) return (size_t)-1;
        return pl.bytes;
    }
    case MMM_SPLIT:
        return split_workspace_bytes(N, P, M, c);
    default:
        return (size_t)-1;
    }
}

mmm_status mmm_multiply(const double* A, const double* B, double* C, int64_t N, int64_t P, int64_t M,
                        mmm_method method, const mmm_config* cfgp, void* workspace, size_t workspace_bytes,
                        void* stream)
{
    const mmm_config c = cfgp ? *cfgp : mmm_config_default();
    mmm_status st = check_cfg(c);
    if (st != MMM_OK) return st;
    if (N < 0 || P < 0 || M < 0) return fail(MMM_EINVAL, "negative size (%lld, %lld, %lld)", (long long)N, (long long)P, (long long)M);
    if ((int)method < 0 || (int)method >= MMM_METHOD_COUNT) return fail(MMM_EINVAL, "unknown method %d", (int)method);
    if (N == 0 || M == 0) return MMM_OK;
    if (!C) return fail(MMM_EINVAL, "C is null");
    if (P > 0 && (!A || !B)) return fail(MMM_EINVAL, "A or B is null");
    const size_t cb = sizeof(double) * (size_t)N * (size_t)M;
    if (overlap(C, cb, A, sizeof(double) * (size_t)N * (size_t)P) || overlap(C, cb, B, sizeof(double) * (size_t)P * (size_t)M))
        return fail(MMM_EALIAS, "C overlaps A or B");
    hipStream_t s = (hipStream_t)stream;
    if (P == 0) return from_hip(launch_fill_zero(C, N * M, s), "zero C");

    const size_t need = mmm_workspace_bytes(method, N, P, M, &c);
    if (need == (size_t)-1) return fail(MMM_EINVAL, "problem too large for the chosen plan");
    if (need > 0) {
        if (!workspace) return fail(MMM_EWORKSPACE, "workspace of %zu bytes required", need);
        if (workspace_bytes < need) return fail(MMM_EWORKSPACE, "workspace %zu < %zu bytes", workspace_bytes, need);
        if ((uintptr_t)workspace % kAlign) return fail(MMM_EWORKSPACE, "workspace must be %zu-byte aligned", kAlign);
        if (overlap(workspace, need, C, cb) || overlap(workspace, need, A, sizeof(double) * (size_t)N * (size_t)P) ||
            overlap(workspace, need, B, sizeof(double) * (size_t)P * (size_t)M))
            return fail(MMM_EALIAS, "workspace overlaps an operand");
    }
    char* ws = (char*)workspace;
    Gemm g{A, P, B, M, C, M, N, P, M};
    // the Winograd vectors sit before the copies, WinogradScaled's scaled
    // operands after them
    const size_t pad_at = method == MMM_WINOGRAD || method == MMM_WINOGRAD_SCALED
                              ? wino_layout(N, M, method == MMM_WINOGRAD_SCALED).bytes
                              : 0;
    const ValuPad plan = pad_plan(method, N, P, M, c);
    hipError_t pe = apply_pad(plan, g, ws + pad_at, s);
    if (pe != hipSuccess) return from_hip(pe, "pad operands");
    char* sws = ws ? ws + pad_at + pad_bytes(plan, N, M) : nullptr;
    // the single-kernel methods: the product kernel is the dominant one
    hipError_t ke = hipSuccess;
    const char* kname = nullptr;
    timer_begin_if(method, s);
    switch (method) {
    case MMM_NAIVE: ke = launch_naive(g, c.naive_fma != 0, s), kname = "naive"; break;
    case MMM_KAHAN: ke = launch_kahan(g, s), kname = "kahan"; break;
    case MMM_NAIVE_ON_ARRAY: ke = launch_naive_variant(g, 0, s), kname = "naive on array"; break;
    case MMM_NAIVE_UNROLL2:
    case MMM_NAIVE_UNROLL3:
    case MMM_NAIVE_UNROLL4:
        ke = launch_naive_variant(g, 2 + (int)(method - MMM_NAIVE_UNROLL2), s), kname = "naive unrolled";
        break;
    case MMM_DOT2: ke = launch_naive_variant(g, 5, s), kname = "dot2"; break;
    case MMM_DGEMM: ke = launch_dgemm(g, s), kname = "dgemm"; break;
    default: break;
    }
    if (kname) {
        timer_end(s);
        return from_hip(ke, kname);
    }
    switch (method) {
    case MMM_WINOGRAD:
        return run_winograd(A, B, g, false, ws, sws, s);
    case MMM_WINOGRAD_SCALED:
        return run_winograd(A, B, g, true, ws, sws, s);
    case MMM_STRASSEN_NAIVE:
    case MMM_STRASSEN_WINOGRAD: {
        StrassenPlan pl;
        if (!plan_strassen(N, P, M, c, pl)) return fail(MMM_EINVAL, "strassen plan too large");
        return run_strassen(method == MMM_STRASSEN_NAIVE ? 0 : 1, A, B, C, N, P, M, pl, ws, s);
    }
    case MMM_SPLIT: {
        hipError_t e = run_split(A, B, C, N, P, M, c, ws, s);
        if (e == hipErrorNotSupported) return fail(MMM_EUNSUPPORTED, "split configuration not supported");
        return from_hip(e, "split");
    }
    default:
        return fail(MMM_EINVAL, "unknown method");
    }
}

static mmm_status ew_call(EwOp op, const double* A, const double* B, double alpha, double* C, int64_t rows,
                          int64_t cols, void* stream)
{
    if (rows < 0 || cols < 0) return fail(MMM_EINVAL, "negative size");
    const i64 n = rows * cols;
    if (n == 0) return MMM_OK;
    if (!A || !C || (op != EW_SCALE && !B)) return fail(MMM_EINVAL, "null pointer");
    const size_t nb = sizeof(double) * (size_t)n;
    if ((C != A && overlap(C, nb, A, nb)) || (op != EW_SCALE && C != B && overlap(C, nb, B, nb)))
        return fail(MMM_EALIAS, "C partially overlaps an operand");
    return from_hip(launch_elementwise(op, A, B, alpha, C, n, (hipStream_t)stream), "elementwise");
}

mmm_status mmm_plus(const double* A, const double* B, double* C, int64_t rows, int64_t cols, void* stream)
{
    return ew_call(EW_PLUS, A, B, 0.0, C, rows, cols, stream);
}

mmm_status mmm_minus(const double* A, const double* B, double* C, int64_t rows, int64_t cols, void* stream)
{
    return ew_call(EW_MINUS, A, B, 0.0, C, rows, cols, stream);
}

mmm_status mmm_multiply_with_scalar(double alpha, const double* A, double* C, int64_t rows, int64_t cols, void* stream)
{
    return ew_call(EW_SCALE, A, nullptr, alpha, C, rows, cols, stream);
}

mmm_status mmm_norm_inf(const double* A, int64_t rows, int64_t cols, double* out, void* stream)
{
    if (rows < 0 || cols < 0) return fail(MMM_EINVAL, "negative size");
    if (!out) return fail(MMM_EINVAL, "out is null");
    if (rows * cols > 0 && !A) return fail(MMM_EINVAL, "A is null");
    return from_hip(launch_norm_inf(A, rows, cols, out, (hipStream_t)stream), "norm_inf");
}

mmm_status mmm_winograd_lambda(const double* normA, const double* normB, int32_t* lambda_out, void* stream)
{
    if (!normA || !normB || !lambda_out) return fail(MMM_EINVAL, "null pointer");
    return from_hip(launch_lambda(normA, normB, (int*)lambda_out, (hipStream_t)stream), "lambda");
}

mmm_status mmm_timer_start(void)
{
    for (hipEvent_t e : g_timer.used) g_timer.spare.push_back(e);
    g_timer.used.clear();
    g_timer.failed = false;
    g_timer.on = true;
    return MMM_OK;
}

mmm_status mmm_timer_stop(double* total_ms, int64_t* launches)
{
    if (!total_ms || !launches) return fail(MMM_EINVAL, "null pointer");
    g_timer.on = false;
    *total_ms = 0.0;
    *launches = 0;
    if (g_timer.failed) return fail(MMM_ELAUNCH, "timer: an event could not be created or recorded");
    const size_t n = g_timer.used.size() / 2 * 2;
    for (size_t i = 0; i < n; i += 2) {
        hipError_t e = hipEventSynchronize(g_timer.used[i + 1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, g_timer.used[i], g_timer.used[i + 1]);
        if (e != hipSuccess) return from_hip(e, "timer");
        *total_ms += ms;
        ++*launches;
    }
    return MMM_OK;
}

const char* mmm_status_string(mmm_status s)
{
    switch (s) {
    case MMM_OK: return "ok";
    case MMM_EINVAL: return "invalid argument";
    case MMM_EALIAS: return "output overlaps an input";
    case MMM_EWORKSPACE: return "workspace too small or misaligned";
    case MMM_EUNSUPPORTED: return "unsupported";
    case MMM_ELAUNCH: return "kernel launch failed";
    case MMM_ENOMEM: return "out of memory";
    default: return "unknown status";
    }
}

const char* mmm_last_error(void) { return g_err; }

int32_t mmm_version(void) { return 100; }

}  // extern "C"
