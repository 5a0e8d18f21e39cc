// Batches of independent products (mmm_batch_*): one plan, one HIP graph.
//
// The plan groups the FP64 problems by DGEMM tile shape and the split
// problems by (digit type, digit count, flush scheme, tile variant,
// accumulator scheme); every group runs as one persistent kernel over a
// grid sized to the chip, whose workgroups claim the group's tiles longest
// first from a counter (so one that starts late, behind another branch's
// work, takes fewer tiles).  All split jobs share one preprocessing chain:
// one pass over every 64-row strip of every problem's A and B for the norms
// and row/column maxima (a strip table built here), lambda, and one digit
// pass over tables of row chunks and column tiles.  The FP64 groups run on
// one branch of one HIP graph, dispatched first; the split preprocessing
// runs on another beside them and then forks into a few branches for the
// split groups.  A tile's arithmetic does not depend on the tile shape or
// on which workgroup runs it, so every result equals the single-call result
// bit for bit.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "batch.h"
#include "common.h"
#include "split.h"

using namespace mmm;

struct mmm_batch {
    void* dmem = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;
};

namespace {

#define bfail mmm::set_error

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

#ifndef MMM_BATCH_SPLIT_BRANCHES
#define MMM_BATCH_SPLIT_BRANCHES 2
#endif
// graph branches the split groups spread over (beside the FP64 branch)
constexpr size_t kSplitBranches = MMM_BATCH_SPLIT_BRANCHES;

struct DGroup {
    int tile;
    std::vector<Gemm> probs;
    std::vector<i64> prefix;
    std::vector<int> slist;
    int grid = 0;
    size_t off_probs = 0, off_prefix = 0, off_ctr = 0, off_slist = 0;
};

struct SGroup {
    SplitGroup g;
    std::vector<SplitJob> jobs;
    std::vector<size_t> ws_off;
    std::vector<i64> prefix;
    std::vector<int> slist;
    int grid = 0;
    int first = 0;  // index of the group's first job in the plan's job table
    size_t off_prefix = 0, off_ctr = 0, off_slist = 0;
};

struct Interval {
    uintptr_t lo, hi;
    bool out;
    int idx;
};

// Claim order of a group's tiles: longest first by estimated cost (stable,
// so the tiles of one problem stay together within a cost), each claimed
// by whichever workgroup is free next.
void longest_first(const std::vector<i64>& cost, std::vector<int>& list)
{
    list.resize(cost.size());
    for (size_t t = 0; t < list.size(); ++t) list[t] = (int)t;
    std::stable_sort(list.begin(), list.end(), [&](int a, int b) { return cost[a] > cost[b]; });
}

int pick_tile(const mmm_problem& p)
{
    if (p.tile != DGEMM_TILE_AUTO) return p.tile;
    return (p.N >= 256 && p.M >= 256) ? DGEMM_TILE_128x128 : DGEMM_TILE_64x64;
}

}  // namespace

extern "C" {

mmm_status mmm_batch_create(const mmm_problem* problems, int32_t count, const mmm_config* cfgp, void* stream,
                            mmm_batch** plan_out)
{
    if (!plan_out) return bfail(MMM_EINVAL, "plan_out is null");
    *plan_out = nullptr;
    if (!problems || count < 1 || count > 65535) return bfail(MMM_EINVAL, "count must be 1..65535");
    const mmm_config c = cfgp ? *cfgp : mmm_config_default();
    if (check_config(c) != MMM_OK) return MMM_EINVAL;

    // validation and aliasing
    std::vector<Interval> iv;
    for (int i = 0; i < count; ++i) {
        const mmm_problem& p = problems[i];
        if (p.N < 0 || p.P < 0 || p.M < 0) return bfail(MMM_EINVAL, "problem %d: negative size", i);
        if (p.method != MMM_DGEMM && p.method != MMM_SPLIT)
            return bfail(MMM_EINVAL, "problem %d: batches take MMM_DGEMM or MMM_SPLIT", i);
        if (p.slices < 0 || p.slices > kMaxSlices) return bfail(MMM_EINVAL, "problem %d: slices outside 0..8", i);
        if (p.tile < 0 || p.tile > (p.method == MMM_SPLIT ? 2 : 3) || p.reserved != 0)
            return bfail(MMM_EINVAL, "problem %d: bad tile", i);
        if (p.N > 0 && p.M > 0 && !p.C) return bfail(MMM_EINVAL, "problem %d: C is null", i);
        if (p.N > 0 && p.M > 0 && p.P > 0 && (!p.A || !p.B)) return bfail(MMM_EINVAL, "problem %d: A or B is null", i);
        if (p.N > 0 && p.M > 0) iv.push_back({(uintptr_t)p.C, (uintptr_t)p.C + 8 * (size_t)(p.N * p.M), true, i});
        if (p.N > 0 && p.P > 0) iv.push_back({(uintptr_t)p.A, (uintptr_t)p.A + 8 * (size_t)(p.N * p.P), false, i});
        if (p.P > 0 && p.M > 0) iv.push_back({(uintptr_t)p.B, (uintptr_t)p.B + 8 * (size_t)(p.P * p.M), false, i});
    }
    std::sort(iv.begin(), iv.end(), [](const Interval& a, const Interval& b) { return a.lo < b.lo; });
    // sweep: any output interval overlapping anything else is an alias
    {
        uintptr_t reach_any = 0, reach_out = 0;
        for (size_t k = 0; k < iv.size(); ++k) {
            const Interval& x = iv[k];
            if (x.lo < reach_out || (x.out && x.lo < reach_any))
                return bfail(MMM_EALIAS, "problem %d: an output overlaps another operand", x.idx);
            reach_any = std::max(reach_any, x.hi);
            if (x.out) reach_out = std::max(reach_out, x.hi);
        }
    }

    // grouping
    std::map<int, DGroup> dg;
    std::map<std::tuple<int, int, bool, int, int>, SGroup> sg;
    size_t split_ws = 0;
    for (int i = 0; i < count; ++i) {
        const mmm_problem& p = problems[i];
        if (p.N == 0 || p.M == 0) continue;
        if (p.method == MMM_DGEMM || p.P == 0) {
            const int tile = pick_tile(p);
            DGroup& g = dg[tile];
            g.tile = tile;
            g.probs.push_back(Gemm{p.A, p.P, p.B, p.M, p.C, p.M, p.N, p.P, p.M});
        } else {
            const int s = p.slices ? p.slices : c.split_slices;
            SplitGroup grp;
            i64 Np, Mp, Kp;
            const int variant = p.tile == SPLIT_TILE_NARROW ? 1 : 0;
            const size_t bytes = split_job_bytes(p.N, p.P, p.M, c.split_type, s, c.split_bits, variant, grp, Np, Mp, Kp);
            if (bytes == (size_t)-1) return bfail(MMM_EUNSUPPORTED, "problem %d: split configuration", i);
            SGroup& g = sg[std::make_tuple(grp.dt, grp.s, grp.flush, grp.variant, grp.ppa)];
            g.g = grp;
            SplitJob j;
            memset(&j, 0, sizeof(j));
            j.A = p.A;
            j.B = p.B;
            j.C = p.C;
            j.N = p.N;
            j.P = p.P;
            j.M = p.M;
            j.Np = Np;  // padded sizes, needed for the work tables (split_job_bind sets the same)
            j.Mp = Mp;
            j.Kp = Kp;
            g.jobs.push_back(j);
            g.ws_off.push_back(split_ws);
            split_ws = al256(split_ws + bytes);
        }
    }

    // persistent grids: every CU, as many workgroups as fit
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(MMM_ELAUNCH, "batch: cannot query the device");
    }

    // device memory layout: tables first, then the split workspaces
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = al256(off + bytes);
        return at;
    };
    for (auto& kv : dg) {
        DGroup& g = kv.second;
        const int bm = dgemm_tile_bm(g.tile), bn = dgemm_tile_bn(g.tile);
        g.prefix.assign(g.probs.size() + 1, 0);
        std::vector<i64> cost;  // K steps of 16 plus the fixed cost of a tile
        for (size_t k = 0; k < g.probs.size(); ++k) {
            const i64 nt = cdiv(g.probs[k].N, bm) * cdiv(g.probs[k].M, bn);
            g.prefix[k + 1] = g.prefix[k] + nt;
            cost.insert(cost.end(), (size_t)nt, cdiv(g.probs[k].P, 16) + 4);
        }
        if (g.prefix.back() > 0x7fffffff) return bfail(MMM_EUNSUPPORTED, "batch: too many DGEMM tiles in one plan");
        // beside split jobs, leave registers for the split branch's kernels
        g.grid = (int)std::min<i64>(g.prefix.back(), (i64)cus * dgemm_grouped_per_cu(g.tile, !sg.empty()));
        longest_first(cost, g.slist);
        g.off_probs = take(sizeof(Gemm) * g.probs.size());
        g.off_prefix = take(sizeof(i64) * g.prefix.size());
        g.off_ctr = take(2 * sizeof(int));
        g.off_slist = take(sizeof(int) * (g.slist.size() ? g.slist.size() : 1));
    }
    // every split job of every group in one table (group by group), with
    // one set of preprocessing work tables over it: statistics strips of 64
    // rows of every job's A and B, then the digit passes' workgroups
    std::vector<JobBlock> strips, ablocks, bblocks;
    int njobs = 0;
    for (auto& kv : sg) {
        SGroup& g = kv.second;
        g.first = njobs;
        for (size_t k = 0; k < g.jobs.size(); ++k) {
            const SplitJob& j = g.jobs[k];
            const int id = njobs + (int)k;
            for (i64 r = 0; r < j.N; r += kStatRows) strips.push_back(JobBlock{id, 0, r});
            for (i64 r = 0; r < j.P; r += kStatRows) strips.push_back(JobBlock{id, 1, r});
            for (i64 b = 0, nb = split_a_blocks(j); b < nb; ++b) ablocks.push_back(JobBlock{id, 0, b});
            for (i64 b = 0, nb = split_b_blocks(j); b < nb; ++b) bblocks.push_back(JobBlock{id, 1, b});
        }
        njobs += (int)g.jobs.size();
    }
    if (strips.size() > 0x7fffffffu || ablocks.size() > 0x7fffffffu || bblocks.size() > 0x7fffffffu)
        return bfail(MMM_EUNSUPPORTED, "batch: split problems too large for one plan");
    const size_t off_jobs = take(sizeof(SplitJob) * (size_t)njobs);
    const size_t off_strips = take(sizeof(JobBlock) * strips.size());
    const size_t off_ablocks = take(sizeof(JobBlock) * ablocks.size());
    const size_t off_bblocks = take(sizeof(JobBlock) * bblocks.size());
    for (auto& kv : sg) {
        SGroup& g = kv.second;
        g.prefix.assign(g.jobs.size() + 1, 0);
        g.off_prefix = take(sizeof(i64) * g.prefix.size());
        std::vector<i64> cost;  // K blocks of 64 plus the fixed cost of a tile
        for (size_t k = 0; k < g.jobs.size(); ++k) {
            // row tiles over N only: the padded rows of the digit layout
            // beyond them are zeros that no tile needs
            const i64 nt = cdiv(g.jobs[k].N, g.g.bm) * (g.jobs[k].Mp / g.g.bn);
            g.prefix[k + 1] = g.prefix[k] + nt;
            cost.insert(cost.end(), (size_t)nt, g.jobs[k].Kp / 64 + 2);
        }
        if (g.prefix.back() > 0x7fffffff) return bfail(MMM_EUNSUPPORTED, "batch: too many split tiles in one plan");
        g.grid = (int)std::min<i64>(g.prefix.back(), (i64)cus * g.g.per_cu);
        longest_first(cost, g.slist);
        g.off_ctr = take(2 * sizeof(int));
        g.off_slist = take(sizeof(int) * (g.slist.size() ? g.slist.size() : 1));
    }
    const size_t off_ws = off;
    const size_t total = off + split_ws + 256;

    mmm_batch* plan = new mmm_batch();
    hipStream_t s = (hipStream_t)stream;
    if (hipMalloc(&plan->dmem, total) != hipSuccess) {
        delete plan;
        (void)hipGetLastError();
        return bfail(MMM_ENOMEM, "batch: cannot allocate %zu bytes", total);
    }
    char* base = (char*)plan->dmem;
    for (auto& kv : sg) {
        SGroup& g = kv.second;
        for (size_t k = 0; k < g.jobs.size(); ++k) split_job_bind(g.jobs[k], base + off_ws + g.ws_off[k], g.g.dt, g.g.s, c.split_bits);
    }
    // upload tables
    std::vector<char> host(off_ws > 0 ? off_ws : 1, 0);
    for (auto& kv : dg) {
        memcpy(host.data() + kv.second.off_probs, kv.second.probs.data(), sizeof(Gemm) * kv.second.probs.size());
        memcpy(host.data() + kv.second.off_prefix, kv.second.prefix.data(), sizeof(i64) * kv.second.prefix.size());
        memcpy(host.data() + kv.second.off_slist, kv.second.slist.data(), sizeof(int) * kv.second.slist.size());
    }
    memcpy(host.data() + off_strips, strips.data(), sizeof(JobBlock) * strips.size());
    memcpy(host.data() + off_ablocks, ablocks.data(), sizeof(JobBlock) * ablocks.size());
    memcpy(host.data() + off_bblocks, bblocks.data(), sizeof(JobBlock) * bblocks.size());
    for (auto& kv : sg) {
        memcpy(host.data() + off_jobs + sizeof(SplitJob) * (size_t)kv.second.first, kv.second.jobs.data(),
               sizeof(SplitJob) * kv.second.jobs.size());
        memcpy(host.data() + kv.second.off_prefix, kv.second.prefix.data(), sizeof(i64) * kv.second.prefix.size());
        memcpy(host.data() + kv.second.off_slist, kv.second.slist.data(), sizeof(int) * kv.second.slist.size());
    }
    // (the tile counters stay zero: the host image is zero-filled)
    hipError_t e = hipSuccess;
    if (off_ws > 0) e = hipMemcpyAsync(base, host.data(), off_ws, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);

    for (auto& kv : sg)
        if (e == hipSuccess) e = split_grouped_prepare(kv.second.g);

    // record the launch sequence.  The FP64 groups come first, on the
    // capture stream: their persistent grids are dispatched at once and
    // keep the matrix cores busy while the split branch's memory-bound
    // preprocessing runs beside them.  After that shared preprocessing the
    // split groups (largest first, each to the branch with the fewest tiles
    // so far) run on at most kSplitBranches branches, so that every branch
    // of the graph keeps a hardware queue of its own: a branch that shares
    // one waits behind the other's persistent kernel.
    std::vector<SGroup*> order;
    for (auto& kv : sg) order.push_back(&kv.second);
    std::stable_sort(order.begin(), order.end(),
                     [](const SGroup* a, const SGroup* b) { return a->prefix.back() > b->prefix.back(); });
    const size_t nlanes = std::min<size_t>(order.size(), kSplitBranches);
    std::vector<std::vector<SGroup*>> lanes(nlanes);
    {
        std::vector<i64> load(nlanes, 0);
        for (SGroup* g : order) {
            const size_t b = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
            lanes[b].push_back(g);
            load[b] += g->prefix.back();
        }
    }
    const size_t nbr = nlanes > 0 ? nlanes - 1 : 0;  // split branches beside `side`
    hipStream_t cap = nullptr, side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, prepped = nullptr;
    std::vector<hipStream_t> br(nbr, nullptr);
    std::vector<hipEvent_t> brj(nbr, nullptr);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&prepped, hipEventDisableTiming);
    for (size_t i = 0; i < nbr && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&brj[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipEventRecord(fork, cap);
        for (auto& kv : dg) {
            if (le != hipSuccess) break;
            DGroup& g = kv.second;
            const TileSchedule sch{(const int*)(base + g.off_slist), (int*)(base + g.off_ctr), (int)g.slist.size()};
            le = launch_dgemm_grouped(g.tile, (const Gemm*)(base + g.off_probs), (const i64*)(base + g.off_prefix),
                                      (int)g.probs.size(), g.prefix.back(), g.grid, sch, cap);
        }
        if (le == hipSuccess) le = hipStreamWaitEvent(side, fork, 0);
        const SplitJob* jobs = (const SplitJob*)(base + off_jobs);
        if (le == hipSuccess && njobs > 0) {
            const SplitTables tab{(const JobBlock*)(base + off_strips), (int)strips.size(),
                                  (const JobBlock*)(base + off_ablocks), (int)ablocks.size(),
                                  (const JobBlock*)(base + off_bblocks), (int)bblocks.size()};
            const SplitGroup& g0 = sg.begin()->second.g;
            le = launch_split_prep(g0.dt, g0.beta, jobs, njobs, tab, c.split_scale_lambda != 0, side);
        }
        if (le == hipSuccess && nbr > 0) le = hipEventRecord(prepped, side);
        for (size_t b = 0; b < nlanes && le == hipSuccess; ++b) {
            hipStream_t gs = b == 0 ? side : br[b - 1];
            if (b > 0) le = hipStreamWaitEvent(gs, prepped, 0);
            for (SGroup* gp : lanes[b]) {
                if (le != hipSuccess) break;
                SGroup& g = *gp;
                const TileSchedule sch{(const int*)(base + g.off_slist), (int*)(base + g.off_ctr),
                                       (int)g.slist.size()};
                le = launch_split_group_gemm(g.g, jobs + g.first, (int)g.jobs.size(), (const i64*)(base + g.off_prefix),
                                             g.prefix.back(), sch, g.grid, gs);
            }
            if (le == hipSuccess && b > 0) le = hipEventRecord(brj[b - 1], gs);
        }
        if (le == hipSuccess) le = hipEventRecord(join, side);
        if (le == hipSuccess) le = hipStreamWaitEvent(cap, join, 0);
        for (size_t i = 0; i < nbr && le == hipSuccess; ++i) le = hipStreamWaitEvent(cap, brj[i], 0);
        e = hipStreamEndCapture(cap, &plan->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (prepped) (void)hipEventDestroy(prepped);
    for (size_t i = 0; i < nbr; ++i) {
        if (brj[i]) (void)hipEventDestroy(brj[i]);
        if (br[i]) (void)hipStreamDestroy(br[i]);
    }
    if (side) (void)hipStreamDestroy(side);
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        const mmm_status st = bfail(MMM_ELAUNCH, "batch create: %s", hipGetErrorString(e));
        (void)hipGetLastError();
        mmm_batch_destroy(plan);
        return st;
    }
    *plan_out = plan;
    return MMM_OK;
}

mmm_status mmm_batch_launch(mmm_batch* plan, void* stream)
{
    if (!plan || !plan->exec) return bfail(MMM_EINVAL, "plan is null");
    const hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess) return bfail(MMM_ELAUNCH, "graph launch: %s", hipGetErrorString(e));
    plan->last = (hipStream_t)stream;
    return MMM_OK;
}

mmm_status mmm_batch_destroy(mmm_batch* plan)
{
    if (!plan) return MMM_OK;
    if (plan->exec) (void)hipStreamSynchronize(plan->last);
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->dmem) (void)hipFree(plan->dmem);
    delete plan;
    return MMM_OK;
}

}  // extern "C"
