/*
 * mmm.h -- C ABI of the MI355X (gfx950) library for dense FP64 matrix
 * multiplication by the methods of Hedtke, "Methods of Matrix
 * Multiplication", arXiv:1106.1347, version 1.
 *
 * Problem statement (Introduction of the paper): A is an N x P matrix and B
 * a P x M matrix with entries of type double; every call computes C = AB
 * (N x M).  Matrices are row-major and contiguous (entry (i, j) of an r x c
 * matrix at offset i*c + j); there is no leading-dimension argument.
 *
 * Memory: every matrix and vector pointer is a DEVICE pointer owned by the
 * caller, valid on the current HIP device.  The library never allocates
 * device memory inside mmm_multiply or the auxiliary calls; methods that
 * need scratch space take a caller-allocated workspace whose size
 * mmm_workspace_bytes reports.  Batch plans (mmm_batch_*) own the device
 * memory for their descriptor tables; mmm_batch_destroy frees it.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the legacy
 * default stream).  Calls are asynchronous: they validate arguments on the
 * host, enqueue kernels on `stream` and return.  No call synchronises the
 * device.
 *
 * Errors: every call returns an mmm_status.  Argument errors are detected on
 * the host before anything is enqueued, so a failed call has no effect on
 * device memory.  MMM_ELAUNCH reports a HIP launch error.  The library never
 * aborts, exits or throws across this interface.  mmm_last_error returns a
 * thread-local message describing the last failure on the calling thread.
 *
 * Zero sizes: N = 0 or M = 0 writes nothing; P = 0 writes C = 0 (the empty
 * sum).  Negative sizes are MMM_EINVAL.
 */
#ifndef MMM_H
#define MMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MMM_OK = 0,
    MMM_EINVAL = 1,      /* bad size, null pointer with nonzero size, bad method or config */
    MMM_EALIAS = 2,      /* C overlaps A or B in mmm_multiply */
    MMM_EWORKSPACE = 3,  /* workspace smaller than mmm_workspace_bytes, or misaligned */
    MMM_EUNSUPPORTED = 4,/* valid request that is not implemented (e.g. a digit count without exact accumulation) */
    MMM_ELAUNCH = 5,     /* HIP reported an error when enqueuing */
    MMM_ENOMEM = 6       /* batch plan could not allocate its tables */
} mmm_status;

/* The methods.  Comments name the section of the paper each one follows. */
typedef enum {
    MMM_NAIVE = 0,             /* 2.1.1 NaivStandard: sum_k a_ik b_kj, k ascending, register accumulator */
    MMM_KAHAN = 1,             /* 2.1.3 NaivKahan: the same sum with Kahan's compensation */
    MMM_WINOGRAD = 2,          /* 2.3.1 WinogradOriginal: pair products minus y_i, z_k, odd-P tail */
    MMM_WINOGRAD_SCALED = 3,   /* 2.3.2 WinogradScaled: WinogradOriginal on (2^l A, 2^-l B),
                                  both materialised in the workspace */
    MMM_STRASSEN_NAIVE = 4,    /* 2.4.1 StrassenNaiv: 7 products, 18 additions per level */
    MMM_STRASSEN_WINOGRAD = 5, /* 2.4.2 StrassenWinograd: 7 products, 15 additions per level */
    MMM_DGEMM = 6,             /* the definition of 2.1 evaluated on FP64 matrix cores */
    MMM_SPLIT = 7,             /* FP64 product from exact low-precision digit products */
    MMM_NAIVE_ON_ARRAY = 8,    /* 2.1.2 NaivOnArray: the naive sum kept in the entry of C itself */
    MMM_NAIVE_UNROLL2 = 9,     /* 2.2.1 NaivLoopUnrollingTwo: products summed in pairs, pair sums accumulated */
    MMM_NAIVE_UNROLL3 = 10,    /* 2.2.2 NaivLoopUnrollingThree: in groups of three */
    MMM_NAIVE_UNROLL4 = 11,    /* 2.2.3 NaivLoopUnrollingFour: in groups of four */
    MMM_DOT2 = 12,             /* beyond the paper: 2.1.3's compensation extended to the products (TwoProduct by
                                  FMA + TwoSum, Ogita-Rump-Oishi Dot2), about twice the working precision */
    MMM_METHOD_COUNT = 13
} mmm_method;

/* Strassen embedding.  PAPER: the square Y x Y zero embedding of Section
 * 2.4.1 (X = max{N,P,M}, k = floor(log2 X) - 4, m = floor(X 2^-k) + 1,
 * Y = m 2^k, k clamped at 0), k levels, naive m x m leaf.  LEVELS:
 * `strassen_levels` levels, each dimension padded to a multiple of
 * 2^levels (with the DGEMM leaf and P >= 64 2^levels, P to a multiple of
 * 16 2^levels, so that the leaf depth suits the matrix cores' K step). */
typedef enum { MMM_PAD_PAPER = 0, MMM_PAD_LEVELS = 1 } mmm_pad_mode;

/* Leaf product of the Strassen recursion (the algorithm alpha_{m,0}). */
typedef enum { MMM_LEAF_DGEMM = 0, MMM_LEAF_NAIVE = 1 } mmm_leaf;

/* Digit type of the split product. */
typedef enum { MMM_SLICE_BF16 = 0, MMM_SLICE_FP16 = 1, MMM_SLICE_INT8 = 2 } mmm_slice_type;

typedef struct {
    int32_t strassen_levels;    /* LEVELS mode recursion depth, 0..12 (default 2) */
    int32_t pad_mode;           /* mmm_pad_mode (default MMM_PAD_LEVELS) */
    int32_t strassen_leaf;      /* mmm_leaf; PAPER mode always uses the naive leaf (default DGEMM) */
    int32_t split_slices;       /* number of digits s per operand, 1..8 (default 6) */
    int32_t split_type;         /* mmm_slice_type (default BF16) */
    int32_t split_scale_lambda; /* 1: apply WinogradScaled's 2^(+-lambda) before slicing (default 1) */
    int32_t naive_fma;          /* NAIVE only. 0: product and sum rounded separately as in the
                                   paper (default); 1: fused multiply-add */
    int32_t split_bits;         /* digit width beta of the split product: 0 = the digit type's default
                                   (bf16 8, fp16 9, int8 7); bf16 and fp16 2..9, int8 2..8 (a digit of
                                   beta bits is at most 2^(beta-1) in magnitude, which the type holds
                                   exactly; int8 with 8 bits takes byte digits in [-128, 127]: each
                                   scaled entry, one exponent step smaller, rounded once to 8 s bits
                                   and written in base 256; with every allowed width and digit count,
                                   the fullest digit-pair group stays in the accumulator's exact range
                                   for at least one matrix-core step) */
    int32_t reserved[8];        /* must be zero */
} mmm_config;

/* Default configuration (values above). */
mmm_config mmm_config_default(void);

/* Bytes of workspace mmm_multiply needs for this method, shape and config
 * (0 for methods that need none).  Returns (size_t)-1 for invalid
 * arguments.  The inner-product methods (NAIVE ... DOT2) and DGEMM need none
 * except for large products (N P M >= 2^32) whose N and M are multiples of
 * the kernel tile but whose P gives A rows that are not 16-byte aligned or a
 * K range that is not a whole number of kernel steps (P = 4097, say): those
 * run on zero-padded copies of A (N x kp) and, when K is ragged, B (kp x M),
 * kp = P rounded up to at most the next multiple of 32.  The result is the
 * same as without the copies (bit for bit for the methods defined by a
 * summation order).  WinogradScaled also holds 2^l A and 2^-l B (in the
 * padded copies where those exist, else N x P and P x M doubles). */
size_t mmm_workspace_bytes(mmm_method method, int64_t N, int64_t P, int64_t M, const mmm_config* cfg);

/* C = A B by `method`.  A: N x P, B: P x M, C: N x M, device, row-major.
 * C must not overlap A or B (MMM_EALIAS).  `cfg` may be NULL (defaults).
 * `workspace` is a device buffer of at least mmm_workspace_bytes(...)
 * bytes, 256-byte aligned, or NULL when that size is 0; its contents on
 * entry are ignored and on exit undefined.  Concurrent calls must not share
 * a workspace.  Asynchronous on `stream`. */
mmm_status mmm_multiply(const double* A, const double* B, double* C, int64_t N, int64_t P, int64_t M,
                        mmm_method method, const mmm_config* cfg, void* workspace, size_t workspace_bytes,
                        void* stream);

/* Section 1.1 (Plus): C = A + B, rows x cols, one rounding per entry.  C
 * may equal A or B (in place); partial overlap is MMM_EALIAS. */
mmm_status mmm_plus(const double* A, const double* B, double* C, int64_t rows, int64_t cols, void* stream);

/* Section 1.2 (Minus): C = A - B, as mmm_plus. */
mmm_status mmm_minus(const double* A, const double* B, double* C, int64_t rows, int64_t cols, void* stream);

/* Section 1.5 (MultiplyWithScalar): C = alpha A.  C may equal A. */
mmm_status mmm_multiply_with_scalar(double alpha, const double* A, double* C, int64_t rows, int64_t cols,
                                    void* stream);

/* Section 1.4 (NormInf): *out = max_i sum_j |A_ij|, each row summed with j
 * ascending from 0.0, written to the device double `out` (0 for an empty
 * matrix). */
mmm_status mmm_norm_inf(const double* A, int64_t rows, int64_t cols, double* out, void* stream);

/* Section 2.3.2: the scaling exponent lambda of WinogradScaled from two
 * device norms, written to the device int `lambda_out`: the largest
 * integer with 1/2 <= 2^(2 lambda) normA / normB <= 2 (0 when a norm is
 * zero, infinite or NaN). */
mmm_status mmm_winograd_lambda(const double* normA, const double* normB, int32_t* lambda_out, void* stream);

/* ---- Products without any allocation ---------------------------------- */

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, hosts that forbid allocation on the hot
 * path): mmm_multiply with its workspace taken from a library-owned device
 * array of MMM_NOALLOC_SCRATCH_BYTES bytes instead of a caller buffer.
 * Each device the library runs on holds its own array from the first call
 * there until the process ends; the call itself allocates and frees
 * nothing.  Arguments, layout, asynchrony and results are those of
 * mmm_multiply (bitwise the same C).  A product whose mmm_workspace_bytes
 * exceeds the array is refused with MMM_EWORKSPACE before anything is
 * enqueued.  The array keeps whatever the last call left in it (every
 * method clears what it needs cleared); calls on one device that overlap
 * in time share it and race, so the caller serialises them (one stream, or
 * events between streams). */
#define MMM_NOALLOC_SCRATCH_BYTES (64u << 20)
mmm_status mmm_multiply_noalloc(const double* A, const double* B, double* C, int64_t N, int64_t P, int64_t M,
                                mmm_method method, const mmm_config* cfg, void* stream);
/* Size of that array in bytes (MMM_NOALLOC_SCRATCH_BYTES). */
size_t mmm_noalloc_scratch_bytes(void);

/* ---- Batches: many independent products in one launch sequence ------- */

typedef struct {
    const double* A; /* device, N x P */
    const double* B; /* device, P x M */
    double* C;       /* device, N x M; must not overlap any other problem's C, A or B */
    int64_t N, P, M;
    int32_t method;  /* MMM_DGEMM or MMM_SPLIT */
    int32_t slices;  /* split digits (MMM_SPLIT), 0 = the config's default */
    int32_t tile;    /* tile shape: 0 = library's choice; DGEMM 1 = 128x128, 2 = 64x64, 3 = 128x64;
                        SPLIT 1 = the wide tile, 2 = the narrow tile (half its rows) */
    int32_t reserved;/* must be zero */
} mmm_problem;

typedef struct mmm_batch mmm_batch;

/* Build a plan for `count` (1..65535) problems: validates them, chooses
 * tile shapes, allocates device tables and workspace (owned by the plan),
 * uploads the descriptors and records the launch sequence into a HIP graph
 * (FP64 and split halves on parallel branches).  Synchronous with respect
 * to `stream`.  Pointers inside the problems are captured; the caller must
 * keep the matrices alive while the plan is launched.  Each product is
 * computed exactly as a single mmm_multiply call with the same method and
 * config would compute it (bitwise), whatever else is in the batch. */
mmm_status mmm_batch_create(const mmm_problem* problems, int32_t count, const mmm_config* cfg, void* stream,
                            mmm_batch** plan_out);

/* Enqueue every product of the plan on `stream` (a fixed, short sequence of
 * persistent kernels; no host synchronisation, capturable in a HIP graph).
 * Launches of one plan must not overlap on the device (they share the
 * plan's workspace and tile counters): keep them on one stream, or order
 * them with events. */
mmm_status mmm_batch_launch(mmm_batch* plan, void* stream);

/* Free the plan's device memory (synchronises the plan's last stream). */
mmm_status mmm_batch_destroy(mmm_batch* plan);

/* ---- Diagnostics ------------------------------------------------------ */

/* Kernel timer, per calling thread.  After mmm_timer_start, every
 * mmm_multiply on this thread records a pair of HIP events on its stream
 * immediately before and after the launch of its dominant kernel (the
 * product kernel of NAIVE ... DOT2 and DGEMM, WinogradOriginal's main loop,
 * the Strassen leaf launch, the split product's digit GEMM); no other work
 * is added to the stream.  mmm_timer_stop ends the recording, waits for the
 * recorded events and returns the summed elapsed time in milliseconds and
 * the number of bracketed launches.  Not for use under graph capture. */
mmm_status mmm_timer_start(void);
mmm_status mmm_timer_stop(double* total_ms, int64_t* launches);

const char* mmm_status_string(mmm_status s);
const char* mmm_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t mmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MMM_H */
