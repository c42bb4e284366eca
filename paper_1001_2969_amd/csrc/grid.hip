// Node-grid kernels: densities, charge and susceptibility from the deposit,
// E = -grad phi, and fixed-point <-> double conversion of the deposit.
#include "device.h"

namespace rz {

// Every node of the deposit (finalize_node).
__global__ void k_finalize(GridArgs g)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.nn; k += gridDim.x * blockDim.x)
        finalize_node(g, k);
}

hipError_t launch_finalize(const GridArgs &g, hipStream_t st)
{
    int threads = 256, blocks = (g.nn + threads - 1) / threads;
    RZ_LAUNCH(k_finalize, dim3(blocks), dim3(threads), 0, st, g);
    return hipGetLastError();
}

// E = -grad phi: centred differences inside, one-sided on z = 0, z = L and
// r = R, E_r = 0 on the axis.  Also the interleaved (E_r, E_z) copy that the
// particle gather reads (in the particles' precision).
template <typename T>
struct k_efield_A {
    int nr;
    int nz;
    double hr;
    double hz;
    const double *phi;
    double *er;
    double *ez;
    typename Vec2<T>::type *E2;
    unsigned long long *zero0;  // cleared on every node when set
    unsigned long long *zero1;
    unsigned long long *clear;  // cleared by block 0: nclear counters
    int nclear;
};

template <typename T>
__device__ __forceinline__ void k_efield_body(const Blk &kb_, const k_efield_A<T> &A_)
{
    auto nr = A_.nr;
    auto nz = A_.nz;
    auto hr = A_.hr;
    auto hz = A_.hz;
    auto phi = A_.phi;
    auto er = A_.er;
    auto ez = A_.ez;
    auto E2 = A_.E2;

    const int nn = nr * nz;
    if (kb_.x == 0)
        for (int t = threadIdx.x; t < A_.nclear; t += blockDim.x) A_.clear[t] = 0;
    for (int g = kb_.x * blockDim.x + threadIdx.x; g < nn; g += kb_.nx * blockDim.x) {
        int i = g / nr, j = g - i * nr;
        double vz, vr;
        if (i == 0) vz = -(phi[g + nr] - phi[g]) / hz;
        else if (i == nz - 1) vz = -(phi[g] - phi[g - nr]) / hz;
        else vz = -(phi[g + nr] - phi[g - nr]) / (2.0 * hz);
        if (j == 0) vr = 0.0;
        else if (j == nr - 1) vr = -(phi[g] - phi[g - 1]) / hr;
        else vr = -(phi[g + 1] - phi[g - 1]) / (2.0 * hr);
        er[g] = vr;
        ez[g] = vz;
        typename Vec2<T>::type e;
        e.x = (T)vr;
        e.y = (T)vz;
        E2[g] = e;
        if (A_.zero0) A_.zero0[g] = 0;
        if (A_.zero1) A_.zero1[g] = 0;
    }
}


template <typename T>
hipError_t launch_efield(int nr, int nz, double hr, double hz, const double *phi, double *er,
                         double *ez, typename Vec2<T>::type *E2, hipStream_t st,
                         unsigned long long *zero0, unsigned long long *zero1,
                         unsigned long long *clear, int nclear)
{
    int nn = nr * nz, threads = 256, blocks = (nn + threads - 1) / threads;
    (void)launch<k_efield_A<T>, k_efield_body<T>, 256>(dim3(blocks), dim3(threads), 0, st, k_efield_A<T>{nr, nz, hr, hz, phi, er, ez, E2, zero0, zero1, clear, nclear});
    return hipGetLastError();
}

// Interleaved gather copy of caller-written E_r, E_z.
template <typename T>
__global__ void k_pack_e2(int nn, const double *er, const double *ez, typename Vec2<T>::type *E2)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x) {
        typename Vec2<T>::type e;
        e.x = (T)er[g];
        e.y = (T)ez[g];
        E2[g] = e;
    }
}

template <typename T>
hipError_t launch_pack_e2(int nn, const double *er, const double *ez, typename Vec2<T>::type *E2,
                          hipStream_t st)
{
    int threads = 256, blocks = (nn + threads - 1) / threads;
    RZ_LAUNCH((k_pack_e2<T>), dim3(blocks), dim3(threads), 0, st, nn, er, ez, E2);
    return hipGetLastError();
}

__global__ void k_acc_convert(int nn, unsigned long long *acc, double *dev, double quantum,
                              int to_acc)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x) {
        if (to_acc) acc[g] = (unsigned long long)__double2ll_rn(dev[g] / quantum);
        else dev[g] = (double)(long long)acc[g] * quantum;
    }
}

hipError_t launch_acc_convert(int nn, unsigned long long *acc, double *dev, double quantum,
                              int to_acc, hipStream_t st)
{
    int threads = 256, blocks = (nn + threads - 1) / threads;
    RZ_LAUNCH(k_acc_convert, dim3(blocks), dim3(threads), 0, st, nn, acc, dev, quantum,
                       to_acc);
    return hipGetLastError();
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t st)
{
    int threads = 256;
    int64_t b = (n + threads - 1) / threads;
    int blocks = (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
    RZ_LAUNCH(k_fill_u64, dim3(blocks), dim3(threads), 0, st, p, n);
    return hipGetLastError();
}

template hipError_t launch_pack_e2<double>(int, const double *, const double *, double2 *,
                                           hipStream_t);
template hipError_t launch_pack_e2<float>(int, const double *, const double *, float2 *,
                                          hipStream_t);
template hipError_t launch_efield<double>(int, int, double, double, const double *, double *,
                                          double *, double2 *, hipStream_t, unsigned long long *,
                                          unsigned long long *, unsigned long long *, int);
template hipError_t launch_efield<float>(int, int, double, double, const double *, double *,
                                         double *, float2 *, hipStream_t, unsigned long long *,
                                         unsigned long long *, unsigned long long *, int);

}  // namespace rz
