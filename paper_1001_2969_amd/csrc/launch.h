// Kernel launches that a batched step can record and replay.
//
// Every launch of the library goes through launch() (a kernel written as a
// body over a virtual block index, which a batch can run for many discharges
// in one launch) or RZ_LAUNCH (any other kernel, which a batch replays as
// is).  Outside a recorded step both simply launch on the given stream.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstring>
#include <functional>
#include <tuple>
#include <vector>

namespace rz {

// Block index and grid size as the body sees them: the hardware values for a
// single launch, the job-local ones inside a batched launch.
struct Blk {
    int x, y, nx, ny;
};

// One discharge's share of a batched launch: its arguments and its blocks
// [first, first + nx * ny) of the launch.
template <typename A> struct Job {
    A a;
    int first, nx, ny, pad;
};

template <typename A, void (*Body)(const Blk &, const A &), int MT>
__global__ __launch_bounds__(MT) void k_one(A a)
{
    Body(Blk{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y}, a);
}

// The job table is read-only for the whole launch (__restrict__): the body's
// argument fields are loaded once and kept, as kernel arguments would be.
template <typename A, void (*Body)(const Blk &, const A &), int MT>
__global__ __launch_bounds__(MT) void k_many(const Job<A> *__restrict__ jobs, int nj)
{
    // the job holding this block: the last one starting at or before it
    int lo = 0, hi = nj - 1;
    const int bx = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].first <= bx) lo = mid;
        else hi = mid - 1;
    }
    const Job<A> &J = jobs[lo];
    const int l = bx - J.first;
    Body(Blk{l % J.nx, l / J.nx, J.nx, J.ny}, J.a);
}

// One launch of a recorded step.
struct LaunchRec {
    const void *key = nullptr;  // the kernel instance
    unsigned gx = 1, gy = 1, threads = 1;
    size_t lds = 0;
    // batchable launches: argument bytes, the layout of Job<A>, and the
    // launcher of k_many
    std::vector<unsigned char> args;
    size_t job_size = 0, job_align = 0, first_off = 0;
    hipError_t (*many)(const void *jobs, int nj, int blocks, unsigned threads, size_t lds,
                       hipStream_t st) = nullptr;
    // other launches: the launch itself, on a given stream
    std::function<void(hipStream_t)> raw;
};

struct Recorder {
    std::vector<LaunchRec> recs;
};

// Set (per host thread) while a batched step records a discharge's step.
extern thread_local Recorder *g_recorder;

template <typename A, void (*Body)(const Blk &, const A &), int MT>
hipError_t launch_many(const void *jobs, int nj, int blocks, unsigned threads, size_t lds,
                       hipStream_t st)
{
    hipLaunchKernelGGL((k_many<A, Body, MT>), dim3(blocks), dim3(threads), lds, st,
                       (const Job<A> *)jobs, nj);
    return hipGetLastError();
}

template <typename A, void (*Body)(const Blk &, const A &), int MT>
hipError_t launch(dim3 grid, dim3 block, size_t lds, hipStream_t st, const A &a)
{
    if (Recorder *r = g_recorder) {
        LaunchRec L;
        L.key = (const void *)&k_many<A, Body, MT>;
        L.gx = grid.x;
        L.gy = grid.y;
        L.threads = block.x;
        L.lds = lds;
        L.args.resize(sizeof(A));
        std::memcpy(L.args.data(), &a, sizeof(A));
        L.job_size = sizeof(Job<A>);
        L.job_align = alignof(Job<A>);
        L.first_off = offsetof(Job<A>, first);
        L.many = &launch_many<A, Body, MT>;
        r->recs.push_back(std::move(L));
        return hipSuccess;
    }
    hipLaunchKernelGGL((k_one<A, Body, MT>), grid, block, lds, st, a);
    return hipPeekAtLastError();  // left set for a caller's hipGetLastError
}

// launch() with HIP events attached to the kernel's own dispatch (ev0 at
// its start, ev1 at its end; hipExtLaunchKernel), so that the elapsed time
// between them is the kernel's run time without the dispatch around it.
// Without events, or while a batched step records, the same as launch().
template <typename A, void (*Body)(const Blk &, const A &), int MT>
hipError_t launch_ev(dim3 grid, dim3 block, size_t lds, hipStream_t st, const A &a,
                     hipEvent_t ev0, hipEvent_t ev1)
{
    if (g_recorder || !ev0 || !ev1) return launch<A, Body, MT>(grid, block, lds, st, a);
    hipExtLaunchKernelGGL((k_one<A, Body, MT>), grid, block, (std::uint32_t)lds, st, ev0, ev1, 0,
                          a);
    return hipPeekAtLastError();
}

template <typename F>
void launch_raw(const void *key, dim3 grid, dim3 block, size_t lds, hipStream_t st, F f)
{
    if (Recorder *r = g_recorder) {
        LaunchRec L;
        L.key = key;
        L.gx = grid.x;
        L.gy = grid.y;
        L.threads = block.x;
        L.lds = lds;
        L.raw = f;
        r->recs.push_back(std::move(L));
        return;
    }
    f(st);  // the caller reads the launch status with hipGetLastError
}

}  // namespace rz

// The launch shape and the kernel arguments are evaluated when the launch is
// made (or recorded), never later.
#define RZ_LAUNCH(kernel, grid, block, lds, st, ...)                                            \
    ::rz::launch_raw((const void *)&(kernel), grid, block, lds, st,                             \
                     [g_ = dim3(grid), b_ = dim3(block), l_ = (size_t)(lds),                    \
                      t_ = std::make_tuple(__VA_ARGS__)](hipStream_t s_) {                       \
                         std::apply(                                                            \
                             [&](const auto &...x_) {                                           \
                                 hipLaunchKernelGGL(kernel, g_, b_, l_, s_, x_...);             \
                             },                                                                 \
                             t_);                                                               \
                     })
