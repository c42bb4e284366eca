// z-semi-coarsening multigrid of Sec. 2.5 (Algorithm 1, V(0,1)): finite-volume
// 5-point operator, full-weighting restriction along z, exact coarsest line
// solve, and on the way up the prolonged correction followed by one zebra
// sweep of exact r-line solves (parallel cyclic reduction in LDS, one block
// per line).
#include "device.h"

namespace rz {

template <typename T> __device__ __forceinline__ T face(T a, T b, int rule)
{
    return rule == 1 ? (a > b ? a : b) : (T)0.5 * (a + b);
}

// Coefficients at unknown (i, j): face fluxes of the control volume divided
// by its volume (axis: no inner face, outer face pi hr hz, volume pi hr^2 hz/4).
template <typename T> struct Coef {
    T a, b, c, d, e;
};

template <typename T>
__device__ __forceinline__ Coef<T> coef(const T *eps, int nr, int i, int j, T inv_hz2, T inv_hr2,
                                        int rule)
{
    const T *ec = eps + (size_t)i * nr;
    Coef<T> k;
    k.a = face<T>(ec[j - nr], ec[j], rule) * inv_hz2;
    k.c = face<T>(ec[j], ec[j + nr], rule) * inv_hz2;
    if (j == 0) {
        k.d = (T)0;
        k.e = (T)4 * face<T>(ec[0], ec[1], rule) * inv_hr2;
    } else {
        T jj = (T)j;
        k.d = face<T>(ec[j - 1], ec[j], rule) * ((jj - (T)0.5) / jj) * inv_hr2;
        k.e = face<T>(ec[j], ec[j + 1], rule) * ((jj + (T)0.5) / jj) * inv_hr2;
    }
    k.b = k.a + k.c + k.d + k.e;
    return k;
}

__global__ void k_set_bc(double *phi, int nr, int nz, double V)
{
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nr + nz; t += gridDim.x * blockDim.x) {
        if (t < nr) {
            phi[t] = t < nr - 1 ? V : 0.0;
            phi[(size_t)(nz - 1) * nr + t] = 0.0;
        } else {
            phi[(size_t)(t - nr) * nr + nr - 1] = 0.0;
        }
    }
}

hipError_t mg_set_bc(double *phi, int nr, int nz, double V, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_bc, dim3(1), dim3(256), 0, st, phi, nr, nz, V);
    return hipGetLastError();
}

__device__ __forceinline__ void atomic_max_abs(unsigned long long *norm, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMax(norm, (unsigned long long)__double_as_longlong(fabs(v)));
}

// res = f - A u on the interior unknowns of the finest level (0 elsewhere),
// optionally its max-norm.  zero_interior: u taken as its boundary values only.
__global__ void k_resid(const double *u, const double *f, const double *eps, int nr, int nz,
                        double inv_hz2, double inv_hr2, int rule, double *res,
                        unsigned long long *norm, int zero_interior)
{
    const int nn = nr * nz;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x) {
        int i = g / nr, j = g - i * nr;
        if (i == 0 || i == nz - 1 || j == nr - 1) {
            if (res) res[g] = 0.0;
            continue;
        }
        Coef<double> k = coef<double>(eps, nr, i, j, inv_hz2, inv_hr2, rule);
        auto U = [&](int gg) {
            int ii = gg / nr, jj = gg - ii * nr;
            bool bnd = ii == 0 || ii == nz - 1 || jj == nr - 1;
            return (zero_interior && !bnd) ? 0.0 : u[gg];
        };
        double Au = k.b * U(g) - k.a * U(g - nr) - k.c * U(g + nr) - k.e * U(g + 1);
        if (j > 0) Au -= k.d * U(g - 1);
        double r = f[g] - Au;
        if (res) res[g] = r;
        if (norm) atomic_max_abs(norm, r);
    }
}

hipError_t mg_resid_norm(const MgLevels &m, const double *u, const double *f, int zero_interior,
                         unsigned long long *norm, hipStream_t st)
{
    const int L = m.L, nr = m.nr, nz = m.nzl[L];
    const double hz = m.hzl[L];
    int nn = nr * nz, threads = 256, blocks = (nn + threads - 1) / threads;
    hipLaunchKernelGGL(k_resid, dim3(blocks), dim3(threads), 0, st, u, f, m.eps64[L], nr, nz,
                       1.0 / (hz * hz), 1.0 / (m.hr * m.hr), m.chi_face, (double *)nullptr, norm,
                       zero_interior);
    return hipGetLastError();
}

// Restriction of the fine residual down every level, f^{l-1} = FW_z(f^l)
// (u^l = 0 on the coarse levels, so their residual is f^l itself).  Columns
// are independent: each block stages `cpb` columns of all rows in LDS.
template <typename T>
__global__ void k_restrict_down(const double *res, MgLevels m, int mixed, int cpb)
{
    extern __shared__ double sbuf[];
    const int L = m.L, nr = m.nr, nz = m.nzl[L];
    double *cur = sbuf, *nxt = sbuf + (size_t)cpb * nz;
    const int j0 = blockIdx.x * cpb;
    for (int t = threadIdx.x; t < cpb * nz; t += blockDim.x) {
        int cj = t / nz, i = t - cj * nz, j = j0 + cj;
        double v = (j < nr - 1) ? res[(size_t)i * nr + j] : 0.0;
        cur[t] = v;
        if (mixed && j < nr - 1 && i > 0 && i < nz - 1) m.f32[L][(size_t)i * nr + j] = (float)v;
    }
    __syncthreads();
    int nzf = nz;
    for (int l = L - 1; l >= 1; --l) {
        const int nzc = m.nzl[l];
        T *fo = mixed ? (T *)m.f32[l] : (T *)m.f64[l];
        for (int t = threadIdx.x; t < cpb * nzc; t += blockDim.x) {
            int cj = t / nzc, I = t - cj * nzc, j = j0 + cj;
            double v = 0.0;
            if (I > 0 && I < nzc - 1) {
                const double *col = cur + (size_t)cj * nzf;
                v = 0.25 * col[2 * I - 1] + 0.5 * col[2 * I] + 0.25 * col[2 * I + 1];
                if (mixed) v = (double)(float)v;  // coarse right-hand sides in FP32
            }
            nxt[(size_t)cj * nzc + I] = v;
            if (j < nr - 1 && I > 0 && I < nzc - 1) fo[(size_t)I * nr + j] = (T)v;
        }
        __syncthreads();
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
        nzf = nzc;
    }
}

// epsilon on every level: full weighting along z, electrode rows injected.
__global__ void k_restrict_eps(MgLevels m, int mixed, int cpb)
{
    extern __shared__ double sbuf[];
    const int L = m.L, nr = m.nr, nz = m.nzl[L];
    double *cur = sbuf, *nxt = sbuf + (size_t)cpb * nz;
    const int j0 = blockIdx.x * cpb;
    for (int t = threadIdx.x; t < cpb * nz; t += blockDim.x) {
        int cj = t / nz, i = t - cj * nz, j = j0 + cj;
        cur[t] = j < nr ? m.eps64[L][(size_t)i * nr + j] : 1.0;
    }
    __syncthreads();
    int nzf = nz;
    for (int l = L - 1; l >= 1; --l) {
        const int nzc = m.nzl[l];
        for (int t = threadIdx.x; t < cpb * nzc; t += blockDim.x) {
            int cj = t / nzc, I = t - cj * nzc, j = j0 + cj;
            const double *col = cur + (size_t)cj * nzf;
            double v;
            if (I == 0) v = col[0];
            else if (I == nzc - 1) v = col[nzf - 1];
            else v = 0.25 * col[2 * I - 1] + 0.5 * col[2 * I] + 0.25 * col[2 * I + 1];
            nxt[(size_t)cj * nzc + I] = v;
            if (j < nr) {
                m.eps64[l][(size_t)I * nr + j] = v;
                if (mixed) m.eps32[l][(size_t)I * nr + j] = (float)v;
            }
        }
        __syncthreads();
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
        nzf = nzc;
    }
}

static int cols_per_block(int nz) { return nz >= 256 ? 1 : 256 / (nz - 1 > 0 ? nz - 1 : 1); }

hipError_t mg_restrict_eps(const MgLevels &m, int mixed, hipStream_t st)
{
    const int nz = m.nzl[m.L];
    int cpb = cols_per_block(nz);
    if (cpb < 1) cpb = 1;
    int blocks = (m.nr + cpb - 1) / cpb;
    size_t lds = 2 * (size_t)cpb * nz * sizeof(double);
    if (m.L > 1)
        hipLaunchKernelGGL(k_restrict_eps, dim3(blocks), dim3(256), lds, st, m, mixed, cpb);
    return hipGetLastError();
}

template <typename T> struct LineArgs {
    int nr, nzl, rule, parity, zero_old;
    T inv_hz2, inv_hr2;
    const T *eps;
    T *u;
    const T *f;
    const T *uc;  // coarse correction injected into the even neighbours, or null
};

// One zebra half-sweep on a level: block b solves line i (odd rows 2b+1 or
// even rows 2b+2) exactly for j = 0..nr-2,
//   -d x_{j-1} + b x_j - e x_{j+1} = f + a u_{i-1} + c u_{i+1} (+ e u_wall),
// by parallel cyclic reduction in LDS.
template <typename T> __global__ __launch_bounds__(1024) void k_line(LineArgs<T> p)
{
    extern __shared__ unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    const int nr = p.nr, n = nr - 1, nzl = p.nzl;
    const int i = p.parity ? 2 * blockIdx.x + 1 : 2 * blockIdx.x + 2;
    T *A = sm, *Bd = sm + n, *C = sm + 2 * n, *Rr = sm + 3 * n;
    T *A2 = sm + 4 * n, *B2 = sm + 5 * n, *C2 = sm + 6 * n, *R2 = sm + 7 * n;
    auto nb = [&](int row, int j) -> T {
        bool bnd = row == 0 || row == nzl - 1;
        T v = p.zero_old ? (T)0 : p.u[(size_t)row * nr + j];
        if (!bnd && p.uc) v += p.uc[(size_t)(row >> 1) * nr + j];
        return v;
    };
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        Coef<T> k = coef<T>(p.eps, nr, i, j, p.inv_hz2, p.inv_hr2, p.rule);
        T g = p.f[(size_t)i * nr + j] + k.a * nb(i - 1, j) + k.c * nb(i + 1, j);
        T e = k.e;
        if (j == n - 1) {
            g += e * (p.zero_old ? (T)0 : p.u[(size_t)i * nr + nr - 1]);
            e = (T)0;
        }
        A[j] = -k.d;
        Bd[j] = k.b;
        C[j] = -e;
        Rr[j] = g;
    }
    __syncthreads();
    for (int s = 1; s < n; s <<= 1) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            T a = A[j], b = Bd[j], c = C[j], r = Rr[j], a2 = (T)0, c2 = (T)0;
            if (j >= s) {
                T k1 = a / Bd[j - s];
                a2 = -A[j - s] * k1;
                b -= C[j - s] * k1;
                r -= Rr[j - s] * k1;
            }
            if (j + s < n) {
                T k2 = c / Bd[j + s];
                c2 = -C[j + s] * k2;
                b -= A[j + s] * k2;
                r -= Rr[j + s] * k2;
            }
            A2[j] = a2;
            B2[j] = b;
            C2[j] = c2;
            R2[j] = r;
        }
        __syncthreads();
        T *t;
        t = A; A = A2; A2 = t;
        t = Bd; Bd = B2; B2 = t;
        t = C; C = C2; C2 = t;
        t = Rr; Rr = R2; R2 = t;
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x) p.u[(size_t)i * nr + j] = Rr[j] / Bd[j];
}

template <typename T>
static hipError_t line(const MgLevels &m, int l, int parity, int zero_old, T *u, const T *f,
                       const T *eps, const T *uc, hipStream_t st)
{
    LineArgs<T> p;
    p.nr = m.nr;
    p.nzl = m.nzl[l];
    p.rule = m.chi_face;
    p.parity = parity;
    p.zero_old = zero_old;
    const double hz = m.hzl[l];
    p.inv_hz2 = (T)(1.0 / (hz * hz));
    p.inv_hr2 = (T)(1.0 / (m.hr * m.hr));
    p.eps = eps;
    p.u = u;
    p.f = f;
    p.uc = uc;
    const int rows = parity ? (p.nzl - 1) / 2 : (p.nzl - 3) / 2;
    if (rows <= 0) return hipSuccess;
    const int n = m.nr - 1;
    int threads = ((n + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    size_t lds = 8 * (size_t)n * sizeof(T);
    hipLaunchKernelGGL((k_line<T>), dim3(rows), dim3(threads), lds, st, p);
    return hipGetLastError();
}

__global__ void k_add_corr(double *phi, const float *u, int nr, int nz)
{
    const int nn = nr * nz;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x) {
        int i = g / nr, j = g - i * nr;
        if (i > 0 && i < nz - 1 && j < nr - 1) phi[g] += (double)u[g];
    }
}

// One V(0,1) cycle on phi.  FP64: every level in double with phi itself on
// the finest level.  Mixed: the finest residual in double, the correction
// cycle in float on every level, phi += correction in double.
hipError_t mg_vcycle(const MgLevels &m, int mixed, double *phi, const double *f,
                     unsigned long long *norm, hipStream_t st)
{
    const int L = m.L, nr = m.nr, nz = m.nzl[L];
    const double hz = m.hzl[L];
    const int nn = nr * nz;
    hipError_t e;
    if (!mixed && L == 1) return line<double>(m, 1, 1, 0, phi, f, m.eps64[1], nullptr, st);
    {
        int threads = 256, blocks = (nn + threads - 1) / threads;
        hipLaunchKernelGGL(k_resid, dim3(blocks), dim3(threads), 0, st, (const double *)phi, f,
                           (const double *)m.eps64[L], nr, nz, 1.0 / (hz * hz),
                           1.0 / (m.hr * m.hr), m.chi_face, m.res, norm, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        int cpb = cols_per_block(nz);
        int blocks = (nr - 1 + cpb - 1) / cpb;
        size_t lds = 2 * (size_t)cpb * nz * sizeof(double);
        if (mixed)
            hipLaunchKernelGGL((k_restrict_down<float>), dim3(blocks), dim3(256), lds, st,
                               (const double *)m.res, m, mixed, cpb);
        else
            hipLaunchKernelGGL((k_restrict_down<double>), dim3(blocks), dim3(256), lds, st,
                               (const double *)m.res, m, mixed, cpb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (mixed) {
        if ((e = line<float>(m, 1, 1, 1, m.u32[1], m.f32[1], m.eps32[1], nullptr, st))) return e;
        for (int l = 2; l <= L; ++l) {
            if ((e = line<float>(m, l, 1, 1, m.u32[l], m.f32[l], m.eps32[l], m.u32[l - 1], st)))
                return e;
            if ((e = line<float>(m, l, 0, 0, m.u32[l], m.f32[l], m.eps32[l], nullptr, st)))
                return e;
        }
        int threads = 256, blocks = (nn + threads - 1) / threads;
        hipLaunchKernelGGL(k_add_corr, dim3(blocks), dim3(threads), 0, st, phi,
                           (const float *)m.u32[L], nr, nz);
        return hipGetLastError();
    }
    if ((e = line<double>(m, 1, 1, 1, m.u64[1], m.f64[1], m.eps64[1], nullptr, st))) return e;
    for (int l = 2; l <= L; ++l) {
        const bool fine = l == L;
        double *u = fine ? phi : m.u64[l];
        const double *ff = fine ? f : m.f64[l];
        if ((e = line<double>(m, l, 1, fine ? 0 : 1, u, ff, m.eps64[l], m.u64[l - 1], st)))
            return e;
        if ((e = line<double>(m, l, 0, 0, u, ff, m.eps64[l], nullptr, st))) return e;
    }
    return hipSuccess;
}

}  // namespace rz
