// Sequential vector reductions of the auxiliary kernels; the split
// product's statistics pass uses the same layout (device code, internal to
// libmmm).
#pragma once

#include "common.h"
#include "launch.h"

namespace mmm {

__device__ inline double max_s13(double x, double y) { return x >= y ? x : y; }  // Section 1.3

// Sequential reduction of 16 vectors per workgroup.  The workgroup streams
// each vector in chunks of 256 entries through double-buffered LDS with
// coalesced loads (rows: 2 KiB runs; columns: 128-byte runs of 16
// neighbouring columns); 16 lanes then fold their vector's chunk in order.
constexpr int RV = 16, RL = 256, RPER = RV * RL / 256;

template <int OP, bool COLS, bool FOLD_MAX>
__device__ __forceinline__ void vecred_body(const double* __restrict__ X, i64 ld, i64 nvec, i64 len,
                                            double* __restrict__ out, i64 block, double (*T)[RV][RL + 1])
{
    const int tid = threadIdx.x;
    const i64 v0 = block * RV;
    const i64 lim = (OP == RED_PAIR_SUM) ? 2 * (len / 2) : len;
    const i64 nchunks = (lim + RL - 1) / RL;
    double r[RPER];
    auto load = [&](i64 c) {
#pragma unroll
        for (int q = 0; q < RPER; ++q) {
            const int e = q * 256 + tid;
            const int v = COLS ? (e % RV) : (e / RL);
            const int x = COLS ? (e / RV) : (e % RL);
            const i64 gv = v0 + v, gx = c * RL + x;
            double val = 0.0;
            if (gv < nvec && gx < lim) val = COLS ? X[gx * ld + gv] : X[gv * ld + gx];
            r[q] = val;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < RPER; ++q) {
            const int e = q * 256 + tid;
            const int v = COLS ? (e % RV) : (e / RL);
            const int x = COLS ? (e / RV) : (e % RL);
            T[buf][v][x] = r[q];
        }
    };
    double acc = 0.0;
    if (nchunks > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (i64 c = 0; c < nchunks; ++c) {
        const int cur = (int)(c & 1);
        if (c + 1 < nchunks) load(c + 1);
        if (tid < RV) {
            const i64 rem = lim - c * RL;
            const int cnt = rem < RL ? (int)rem : RL;
            const double* row = T[cur][tid];
            if (OP == RED_ABS_SUM) {
                for (int x = 0; x < cnt; ++x) acc = acc + fabs(row[x]);
            } else if (OP == RED_PAIR_SUM) {
                for (int x = 0; x < cnt; x += 2) {
                    const double a = row[x];
                    const double b = row[x + 1];
                    const double p = a * b;
                    acc = acc + p;
                }
            }
        }
        if (c + 1 < nchunks) store(cur ^ 1);
        __syncthreads();
    }
    if (tid < RV && v0 + tid < nvec) {
        if (FOLD_MAX) {
            // max over vectors of non-negative values: the order of binary64
            // bit patterns of non-negative numbers is their numeric order
            atomicMax(reinterpret_cast<unsigned long long*>(out), (unsigned long long)__double_as_longlong(acc));
        } else {
            out[v0 + tid] = acc;
        }
    }
}

}  // namespace mmm
