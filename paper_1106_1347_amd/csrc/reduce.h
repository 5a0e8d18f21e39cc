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

// Folds one full chunk of RL entries of a vector (in LDS) into acc in
// order.  The LDS reads run one group of 16 entries ahead of the adds, so
// the dependent chain of adds does not wait on LDS latency per group; the
// empty asm statements keep the compiler from hoisting later groups' reads
// (which would hold the whole chunk in registers).
template <int OP>
__device__ __forceinline__ double fold_group(const double (&v)[16], double acc)
{
    if (OP == RED_ABS_SUM) {
#pragma unroll
        for (int e = 0; e < 16; ++e) acc = acc + fabs(v[e]);
    } else {
#pragma unroll
        for (int e = 0; e < 16; e += 2) {
            const double p = v[e] * v[e + 1];
            acc = acc + p;
        }
    }
    return acc;
}

template <int OP>
__device__ __forceinline__ double fold_chunk(const double* row, double acc)
{
    constexpr int G = 16;
    static_assert(RL % (2 * G) == 0, "chunk must hold an even number of groups");
    double va[G], vb[G];
#pragma unroll
    for (int e = 0; e < G; ++e) va[e] = row[e];
#pragma unroll 1
    for (int g = 0; g < RL; g += 2 * G) {
#pragma unroll
        for (int e = 0; e < G; ++e) vb[e] = row[g + G + e];
        asm volatile("" ::: "memory");
        acc = fold_group<OP>(va, acc);
        if (g + 2 * G < RL) {
#pragma unroll
            for (int e = 0; e < G; ++e) va[e] = row[g + 2 * G + e];
        }
        asm volatile("" ::: "memory");
        acc = fold_group<OP>(vb, acc);
    }
    return acc;
}

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
            if (cnt == RL) {
                acc = fold_chunk<OP>(row, acc);
            } else if (OP == RED_ABS_SUM) {
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
