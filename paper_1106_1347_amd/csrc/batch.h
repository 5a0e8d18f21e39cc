// Batches of independent products (internal to libmmm).
#pragma once

#include "common.h"

namespace mmm {

// DGEMM tile shapes a batch problem may request (mmm_problem.tile).
enum DgemmTile { DGEMM_TILE_AUTO = 0, DGEMM_TILE_128x128 = 1, DGEMM_TILE_64x64 = 2, DGEMM_TILE_128x64 = 3 };

int dgemm_tile_bm(int tile);
int dgemm_tile_bn(int tile);
int dgemm_grouped_per_cu(int tile, bool share);
// Tiles of a persistent grouped kernel: the global tile indices list[0 ..
// total - 1], longest first (sorted on the host).  Workgroups claim the
// next position from ctr[0] by an atomic add until the list runs out, then
// count themselves out on ctr[1]; the last one out puts both back to zero
// for the next launch (the plan zeroes them once).  A workgroup that starts
// late, with the chip busy on another branch of the batch, claims fewer
// tiles instead of finishing last.  Launches sharing one counter pair must
// not overlap.
struct TileSchedule {
    const int* list;
    int* ctr;
    int total;
};

// Position of the calling workgroup's next tile (the same for every thread;
// `slot` is a __shared__ int of the kernel).  The caller keeps a barrier
// between its use of one position and the next claim.
__device__ inline int claim_tile(const TileSchedule& sch, int* slot)
{
    if (threadIdx.x == 0) *slot = atomicAdd(sch.ctr, 1);
    __syncthreads();
    return *slot;
}

// Called once by every workgroup after its last (failed) claim.
__device__ inline void release_tiles(const TileSchedule& sch)
{
    if (threadIdx.x == 0 && atomicAdd(sch.ctr + 1, 1) == (int)gridDim.x - 1) {
        atomicExch(sch.ctr, 0);
        atomicExch(sch.ctr + 1, 0);
    }
}

// Persistent grid of `grid` workgroups over the `total` tiles of `nprob`
// problems (device tables: probs[nprob], prefix[nprob + 1]).
hipError_t launch_dgemm_grouped(int tile, const Gemm* probs, const i64* prefix, int nprob, i64 total, int grid,
                                TileSchedule sch, hipStream_t s);

// One split problem of a batch: operands, output and its workspace slices.
struct SplitJob {
    const double* A;
    const double* B;
    double* C;
    i64 N, P, M;
    i64 Np, Mp, Kp;
    double* nA;   // norms (device scalars)
    double* nB;
    int* lam;
    double* rmax; // N
    double* cmax; // M
    int* ea;      // Np
    int* fb;      // Mp
    char* SA;
    char* SB;
    int runlen;   // recombination run length (depends on P)
    int s;        // digits per operand
};

// Split tile variants a batch problem may request (mmm_problem.tile).
enum SplitTile { SPLIT_TILE_AUTO = 0, SPLIT_TILE_WIDE = 1, SPLIT_TILE_NARROW = 2 };

// Split jobs of one digit count, accumulation scheme and tile shape (the
// digit type and width are the batch config's).
struct SplitGroup {
    int dt, s;
    int beta;     // digit width
    int unit;     // MFMA steps one digit pair may accumulate exactly
    int variant;  // 0: the wide tile, 1: the narrow one (half the rows)
    bool flush;
    int ppa;      // without flushing: digit pairs per accumulator (s: one accumulator per group)
    int bm, bn;
    int per_cu;  // workgroups of the group's kernel resident per CU
};

// One workgroup's share of a split group's preprocessing, from tables
// built with the plan (so no workgroup is launched without work):
//   statistics: 64 rows of job `job`'s A (side 0) or B (side 1) from row
//               `index`;
//   digits of A: the `index`-th 256 groups of 8 entries of the job's A;
//   digits of B: the `index`-th 64 x 64 tile of the job's B.
struct JobBlock {
    int job;
    int side;
    i64 index;
};
constexpr int kStatRows = 64;
struct SplitTables {
    const JobBlock* strips;
    int nstrips;
    const JobBlock* ablocks;
    int nablocks;
    const JobBlock* bblocks;
    int nbblocks;
};
// Workgroups of the digit passes for one job (host and device agree).
__host__ __device__ inline i64 split_a_blocks(const SplitJob& j) { return (j.Np * (j.Kp / 8) + 255) / 256; }
constexpr int kBJ = 32;  // columns of B per digit-pass workgroup (64 k each)
__host__ __device__ inline i64 split_b_blocks(const SplitJob& j) { return (j.Kp / 64) * (j.Mp / kBJ); }

// Workspace bytes for one split job; fills the job's Np/Mp/Kp and returns
// (size_t)-1 when unsupported.  Offsets of the job's buffers inside its
// workspace are assigned by split_job_bind.
size_t split_job_bytes(i64 N, i64 P, i64 M, int dt, int s, int bits, int variant, SplitGroup& grp, i64& Np,
                       i64& Mp, i64& Kp);
void split_job_bind(SplitJob& j, char* base, int dt, int s, int bits);
// Host-side set-up of a group's kernels (dynamic LDS size); call once
// before recording launches into a graph.
hipError_t split_grouped_prepare(const SplitGroup& grp);
// Enqueue the preprocessing of `n` split jobs of any group (device table
// `jobs`, work tables `tab` over it): norms and maxima, lambda, digits.
hipError_t launch_split_prep(int dt, int beta, const SplitJob* jobs, int n, const SplitTables& tab, bool scale_lambda,
                             hipStream_t s);
// Enqueue the digit GEMM of one group's `n` jobs (device table `jobs`, tile
// prefix `prefix`, schedule `sched`) on a persistent grid of `grid` workgroups.
hipError_t launch_split_group_gemm(const SplitGroup& grp, const SplitJob* jobs, int n, const i64* prefix,
                                   i64 total_tiles, TileSchedule sched, int grid, hipStream_t s);

}  // namespace mmm
