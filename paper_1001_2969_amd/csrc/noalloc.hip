// Deposit of Sec. 2.4 into a caller's grid without any allocation
// (rzpic_deposit_noalloc): for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).  The fixed-point
// accumulators live in a file-scope device array, one copy per device,
// located once per device with hipGetSymbolAddress.
#include "rzpic.h"

#include "device.h"

#include <cmath>
#include <mutex>

namespace rz {

// Accumulators of the allocation-free deposit: one 64-bit fixed-point word per
// node, at most kNoAllocNodes nodes (8 MiB per device, held until the process
// ends).  Host code never passes the array's name to a kernel: it is a
// host-side stand-in there; the device address comes from hipGetSymbolAddress.
constexpr int kNoAllocNodes = 1 << 20;
static __device__ __align__(256) unsigned long long scratch[kNoAllocNodes];

constexpr int kMaxDevices = 64;
static unsigned long long *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Zero the first nn accumulators (a fill kernel, not a memset: the call may be
// captured into a graph).
__global__ void k_noalloc_zero(unsigned long long *acc, int nn)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x)
        acc[g] = 0;
}

// N_ij += w S_z S_r for the particles [0, n): the weights and the
// fixed-point contribution of every other deposit of the library, added by
// global atomics (integer sums: the order of arrival does not matter).
template <typename T>
__global__ void k_noalloc_deposit(Mesh m, const T *r, const T *z, const T *w, int64_t n,
                                  unsigned long long *acc, double inv_quantum, int32_t *status)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const W4<T> q = weights<T>(m, r[p], z[p]);
        deposit4_at<T>(acc, q.g, m.nr, q, (double)w[p], inv_quantum, status);
    }
}

// Counts in physical particles: N = accumulator * quantum (as rzpic_grid_copy
// returns them).  A negative accumulator (fixed-point overflow) is flagged.
__global__ void k_noalloc_convert(const unsigned long long *acc, int nn, double quantum,
                                  double *out, int32_t *status)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x) {
        const long long a = (long long)acc[g];
        if (a < 0) atomicOr(status, kStNumeric);
        out[g] = (double)a * quantum;
    }
}

}  // namespace rz

using namespace rz;

rzpic_status rz_fail(rzpic_status s, const char *msg);

extern "C" rzpic_status rzpic_deposit_noalloc(const rzpic_deposit_args *a, void *stream)
{
    if (!a) return rz_fail(RZPIC_EINVAL, "deposit_noalloc: null argument");
    if (a->nr < 3 || a->nz < 2 || !(a->R > 0) || !(a->L > 0))
        return rz_fail(RZPIC_EINVAL, "deposit_noalloc: need nr >= 3, nz >= 2, R > 0, L > 0");
    if ((int64_t)a->nr * a->nz > kNoAllocNodes)
        return rz_fail(RZPIC_EINVAL,
                       "deposit_noalloc: nr * nz exceeds its 1048576-node accumulator array");
    if (a->precision != RZPIC_FP64 && a->precision != RZPIC_MIXED)
        return rz_fail(RZPIC_EINVAL, "deposit_noalloc: precision must be RZPIC_FP64 or RZPIC_MIXED");
    if (a->weighting != RZPIC_W_ZR2 && a->weighting != RZPIC_W_ZR)
        return rz_fail(RZPIC_EINVAL, "deposit_noalloc: unknown weighting");
    const int bits = a->fixed_point_bits ? a->fixed_point_bits
                                         : (a->precision == RZPIC_MIXED ? 26 : 46);
    if (bits < 0 || bits > (a->precision == RZPIC_MIXED ? 30 : 52) || !(a->w_ref > 0))
        return rz_fail(RZPIC_EINVAL, "deposit_noalloc: fixed_point_bits out of range or w_ref <= 0");
    if (a->n < 0 || a->n > ((int64_t)1 << 29) - kChunk)
        return rz_fail(RZPIC_EINVAL, "deposit_noalloc: particle count out of range");
    if (a->n > 0 && (!a->r || !a->z || !a->w))
        return rz_fail(RZPIC_EINVAL, "deposit_noalloc: null particle array");
    if (!a->out || !a->status) return rz_fail(RZPIC_EINVAL, "deposit_noalloc: null output");

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return rz_fail(RZPIC_EHIP, "deposit_noalloc: no current device");
    unsigned long long *acc;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
                return rz_fail(RZPIC_EHIP, "deposit_noalloc: hipGetSymbolAddress failed");
            g_scratch_ptr[dev] = (unsigned long long *)ptr;
        }
        acc = g_scratch_ptr[dev];
    }

    const hipStream_t st = (hipStream_t)stream;
    const int nn = a->nr * a->nz;
    Mesh m{};
    m.nr = a->nr;
    m.nz = a->nz;
    m.nn = nn;
    m.weighting = a->weighting;
    m.R = a->R;
    m.L = a->L;
    m.hr = a->R / (double)(a->nr - 1);
    m.hz = a->L / (double)(a->nz - 1);
    m.inv_hr = 1.0 / m.hr;
    m.inv_hz = 1.0 / m.hz;
    const double quantum = a->w_ref * std::ldexp(1.0, -bits);
    const int threads = 256;
    const int gblocks = (nn + threads - 1) / threads < 2048 ? (nn + threads - 1) / threads : 2048;
    hipLaunchKernelGGL(k_noalloc_zero, dim3(gblocks), dim3(threads), 0, st, acc, nn);
    if (hipGetLastError() != hipSuccess) return rz_fail(RZPIC_EHIP, "deposit_noalloc: launch failed");
    if (a->n > 0) {
        const int64_t want = (a->n + threads - 1) / threads;
        const int pblocks = (int)(want < 8192 ? want : 8192);
        if (a->precision == RZPIC_MIXED)
            hipLaunchKernelGGL(k_noalloc_deposit<float>, dim3(pblocks), dim3(threads), 0, st, m,
                               (const float *)a->r, (const float *)a->z, (const float *)a->w,
                               a->n, acc, 1.0 / quantum, a->status);
        else
            hipLaunchKernelGGL(k_noalloc_deposit<double>, dim3(pblocks), dim3(threads), 0, st, m,
                               (const double *)a->r, (const double *)a->z,
                               (const double *)a->w, a->n, acc, 1.0 / quantum, a->status);
        if (hipGetLastError() != hipSuccess)
            return rz_fail(RZPIC_EHIP, "deposit_noalloc: launch failed");
    }
    hipLaunchKernelGGL(k_noalloc_convert, dim3(gblocks), dim3(threads), 0, st,
                       (const unsigned long long *)acc, nn, quantum, a->out, a->status);
    if (hipGetLastError() != hipSuccess) return rz_fail(RZPIC_EHIP, "deposit_noalloc: launch failed");
    return RZPIC_OK;
}
