// z-semi-coarsening multigrid of Sec. 2.5 (Algorithm 1, V(0,1)): finite-volume
// 5-point operator, full-weighting restriction along z, exact coarsest line
// solve, and on the way up the prolonged correction followed by one zebra
// sweep of exact r-line solves (parallel cyclic reduction in LDS, one block
// per line).
#include <cstring>

#include "device.h"
#include "lists.h"

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
    RZ_LAUNCH(k_set_bc, dim3(1), dim3(256), 0, st, phi, nr, nz, V);
    return hipGetLastError();
}

__device__ __forceinline__ void atomic_max_abs(unsigned long long *norm, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMax(norm, (unsigned long long)__double_as_longlong(fabs(v)));
}

// Max-norm of f - A u over the interior unknowns of the finest level.
// zero_interior: u taken as its boundary values only.
__global__ void k_resid(const double *u, const double *f, const double *eps, int nr, int nz,
                        double inv_hz2, double inv_hr2, int rule, unsigned long long *norm,
                        int zero_interior)
{
    const int nn = nr * nz;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x) {
        int i = g / nr, j = g - i * nr;
        if (i == 0 || i == nz - 1 || j == nr - 1) continue;
        Coef<double> k = coef<double>(eps, nr, i, j, inv_hz2, inv_hr2, rule);
        auto U = [&](int gg) {
            int ii = gg / nr, jj = gg - ii * nr;
            bool bnd = ii == 0 || ii == nz - 1 || jj == nr - 1;
            return (zero_interior && !bnd) ? 0.0 : u[gg];
        };
        double Au = k.b * U(g) - k.a * U(g - nr) - k.c * U(g + nr) - k.e * U(g + 1);
        if (j > 0) Au -= k.d * U(g - 1);
        atomic_max_abs(norm, f[g] - Au);
    }
}

hipError_t mg_resid_norm(const MgLevels &m, const double *u, const double *f, int zero_interior,
                         unsigned long long *norm, hipStream_t st)
{
    const int L = m.L, nr = m.nr, nz = m.nzl[L];
    const double hz = m.hzl[L];
    int nn = nr * nz, threads = 256, blocks = (nn + threads - 1) / threads;
    RZ_LAUNCH(k_resid, dim3(blocks), dim3(threads), 0, st, u, f, m.eps64[L], nr, nz,
                       1.0 / (hz * hz), 1.0 / (m.hr * m.hr), m.chi_face, norm, zero_interior);
    return hipGetLastError();
}

// epsilon on every level: full weighting along z, electrode rows injected.
__global__ void k_restrict_eps(MgLevels m, int mixed, int cpb)
{
    extern __shared__ double sbuf[];
    const int L = m.L, nr = m.nr, nz = m.nzl[L];
    double *cur = sbuf, *nxt = sbuf + (size_t)cpb * nz;
    const int j0 = blockIdx.x * cpb;
    for (int t = threadIdx.x; t < cpb * nz; t += blockDim.x) {
        int i = t / cpb, cj = t - i * cpb, j = j0 + cj;
        cur[cj * nz + i] = j < nr ? m.eps64[L][(size_t)i * nr + j] : 1.0;
    }
    __syncthreads();
    int nzf = nz;
    for (int l = L - 1; l >= 1; --l) {
        const int nzc = m.nzl[l];
        for (int t = threadIdx.x; t < cpb * nzc; t += blockDim.x) {
            int I = t / cpb, cj = t - I * cpb, j = j0 + cj;
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

// Columns per block of the column-parallel grid launches (finalize, way
// down, table preparation): about 64 nodes a block, so that a small mesh
// still spreads over many compute units (128 blocks at 129x65).
static int cols_per_block(int nz) { return nz >= 64 ? 1 : 64 / (nz - 1 > 0 ? nz - 1 : 1); }

hipError_t mg_restrict_eps(const MgLevels &m, int mixed, hipStream_t st)
{
    const int nz = m.nzl[m.L];
    int cpb = cols_per_block(nz);
    if (cpb < 1) cpb = 1;
    int blocks = (m.nr + cpb - 1) / cpb;
    size_t lds = 2 * (size_t)cpb * nz * sizeof(double);
    if (m.L > 1)
        RZ_LAUNCH(k_restrict_eps, dim3(blocks), dim3(256), lds, st, m, mixed, cpb);
    return hipGetLastError();
}

// The step's grid preparation in one launch, a block per group of cpb
// columns: the deposit finalized on every node of its columns
// (finalize_node), epsilon restricted down every level as k_restrict_eps
// does, the Dirichlet values of phi0 and phi1 (V on z = 0 for r < R, 0 on
// z = L and r = R) and, by block 0, `nclear` counters cleared.
struct k_finalize_mg_A {
    GridArgs g;
    MgLevels m;
    int mixed;
    int cpb;
    double *phi0;
    double *phi1;
    double V;
    unsigned long long *clear;
    int nclear;
};

__device__ __forceinline__ void k_finalize_mg_body(const Blk &kb_, const k_finalize_mg_A &A_)
{
    const auto &g = A_.g;
    const auto &m = A_.m;
    auto mixed = A_.mixed;
    auto cpb = A_.cpb;
    auto phi0 = A_.phi0;
    auto phi1 = A_.phi1;
    auto V = A_.V;
    auto clear = A_.clear;
    auto nclear = A_.nclear;

    extern __shared__ double sbuf[];
    const int L = m.L, nr = m.nr, nz = m.nzl[L];
    double *cur = sbuf, *nxt = sbuf + (size_t)cpb * nz;
    const int j0 = kb_.x * cpb;
    if (kb_.x == 0)
        for (int t = threadIdx.x; t < nclear; t += blockDim.x) clear[t] = 0;
    // consecutive threads take consecutive columns of a row (contiguous
    // loads and stores); LDS holds the block's columns one after another
    for (int t = threadIdx.x; t < cpb * nz; t += blockDim.x) {
        const int i = t / cpb, cj = t - i * cpb, j = j0 + cj;
        double e = 1.0;
        if (j < nr) {
            const int k = i * nr + j;
            e = finalize_node(g, k);
            if (i == 0 || i == nz - 1 || j == nr - 1) {
                const double b = (i == 0 && j < nr - 1) ? V : 0.0;
                phi0[k] = b;
                if (phi1) phi1[k] = b;
            }
        }
        cur[cj * nz + i] = e;
    }
    __syncthreads();
    int nzf = nz;
    for (int l = L - 1; l >= 1; --l) {
        const int nzc = m.nzl[l];
        for (int t = threadIdx.x; t < cpb * nzc; t += blockDim.x) {
            int I = t / cpb, cj = t - I * cpb, j = j0 + cj;
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


hipError_t mg_finalize(const GridArgs &g, const MgLevels &m, int mixed, double *phi0, double *phi1,
                       double V, unsigned long long *clear, int nclear, hipStream_t st)
{
    const int nz = m.nzl[m.L];
    int cpb = cols_per_block(nz);
    if (cpb < 1) cpb = 1;
    const int blocks = (m.nr + cpb - 1) / cpb;
    const size_t lds = 2 * (size_t)cpb * nz * sizeof(double);
    (void)launch<k_finalize_mg_A, k_finalize_mg_body, 256>(dim3(blocks), dim3(256), lds, st, k_finalize_mg_A{g, m, mixed, cpb, phi0, phi1, V, clear, nclear});
    return hipGetLastError();
}

template <typename T> struct LineArgs {
    int nr, nzl, rule, parity, zero_old;
    T inv_hz2, inv_hr2;
    const T *eps;
    T *u;
    const T *f;
    const T *uc;  // coarse correction injected into the even neighbours, or null
    double *add_to;  // if set, each solved value is also added here (phi += correction)
};

// One zebra half-sweep on a level: block b solves line i (odd rows 2b+1 or
// even rows 2b+2) exactly for j = 0..nr-2,
//   -d x_{j-1} + b x_j - e x_{j+1} = f + a u_{i-1} + c u_{i+1} (+ e u_wall),
// by parallel cyclic reduction in LDS.
template <typename T>
struct k_line_A {
    LineArgs<T> p;
};

template <typename T>
__device__ __forceinline__ void k_line_body(const Blk &kb_, const k_line_A<T> &A_)
{
    const auto &p = A_.p;

    extern __shared__ unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    const int nr = p.nr, n = nr - 1, nzl = p.nzl;
    const int i = p.parity ? 2 * kb_.x + 1 : 2 * kb_.x + 2;
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
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const T x = Rr[j] / Bd[j];
        p.u[(size_t)i * nr + j] = x;
        if (p.add_to) p.add_to[(size_t)i * nr + j] += (double)x;
    }
}


// The same half-sweep for lines too long for k_line's LDS (8 (nr-1) values):
// the partition method.  Thread t owns Q consecutive unknowns (a segment,
// padded past nr-2 with decoupled identity rows) and eliminates inside it in
// registers: a forward sweep leaves every row coupled only to the last
// unknown of the previous segment, y_{t-1}, and to its successor; a backward
// sweep expresses the segment's first unknown through y_{t-1} and its own last
// unknown y_t.  The T last unknowns then satisfy a tridiagonal system, solved
// by cyclic reduction in LDS, and each thread substitutes back.  The line
// matrices are strictly diagonally dominant, so no pivoting is needed.
template <typename T, int EPT>
__device__ __forceinline__ void pcr(T *A, T *Bd, T *C, T *Rr, int n, int ne);

// LDS slot of element e of a staged chunk: one pad slot after every Q
// elements, so that a thread's segment read (stride Q + 1) spreads over the
// banks while the coalesced staging writes stay contiguous.
template <int Q> __device__ __forceinline__ int part_slot(int e) { return e + e / Q; }

// Staging passes of k_line_part: a pass stages the rows of NT / P segments
// (Q NT / P rows of four values) in LDS; P keeps a pass at 80 KB or less (72
// KB for Q = 8, 80 KB for Q = 4, in either precision), so that two FP32
// blocks share a compute unit's 160 KB of LDS.
template <typename T, int Q> constexpr int part_passes()
{
    return Q * (int)sizeof(T) / 16 > 1 ? Q * (int)sizeof(T) / 16 : 1;
}

template <typename T, int Q> constexpr size_t part_lds()
{
    constexpr int P = part_passes<T, Q>();
    constexpr size_t ch = (size_t)Q * kLongThreads / P;
    constexpr size_t stage = 4 * (ch + ch / Q);
    constexpr size_t red = 7 * (size_t)kLongThreads;
    return (stage > red ? stage : red) * sizeof(T);
}

// two FP32 partition-solver blocks per compute unit (k_line_part_f32)
static_assert(2 * part_lds<float, 2>() <= 160 * 1024, "FP32 Q=2 staging exceeds half the LDS");
static_assert(2 * part_lds<float, 4>() <= 160 * 1024, "FP32 Q=4 staging exceeds half the LDS");
static_assert(2 * part_lds<float, 8>() <= 160 * 1024, "FP32 Q=8 staging exceeds half the LDS");
static_assert(part_lds<double, 8>() <= 160 * 1024 && part_lds<double, 4>() <= 160 * 1024,
              "FP64 staging exceeds the LDS");

template <typename T, int Q>
__device__ __forceinline__ void line_part_body(const LineArgs<T> &p)
{
    extern __shared__ unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    constexpr int NT = kLongThreads;
    constexpr int P = part_passes<T, Q>();
    constexpr int TPP = NT / P;          // segments staged per pass
    constexpr int CH = TPP * Q;          // rows staged per pass
    constexpr int CHP = CH + CH / Q;     // with the pad slots
    constexpr int RPT = CH / NT;         // rows each thread stages per pass
    static_assert(RPT * NT == CH && TPP * P == NT, "staging shape");
    T *SA = sm, *SB = sm + CHP, *SC = sm + 2 * CHP, *SR = sm + 3 * CHP;
    const int nr = p.nr, n = nr - 1, nzl = p.nzl;
    const int i = p.parity ? 2 * blockIdx.x + 1 : 2 * blockIdx.x + 2;
    const int t = threadIdx.x, mine = t / TPP, tl = t - mine * TPP;
    auto nb = [&](int row, int j) -> T {
        bool bnd = row == 0 || row == nzl - 1;
        T v = p.zero_old ? (T)0 : p.u[(size_t)row * nr + j];
        if (!bnd && p.uc) v += p.uc[(size_t)(row >> 1) * nr + j];
        return v;
    };
    // rows of the segment: a x_{j-1} + b x_j + c x_{j+1} = r.  Each pass
    // forms its rows with coalesced loads (thread t: rows k NT + t of the
    // chunk) into LDS; the threads whose segments lie in the chunk then read
    // them back and eliminate.
    T ap[Q], bp[Q], c[Q], rp[Q];
    for (int ps = 0; ps < P; ++ps) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int e = k * NT + t, j = ps * CH + e;
            T a = (T)0, b = (T)1, cc = (T)0, r = (T)0;
            if (j < n) {
                Coef<T> kf = coef<T>(p.eps, nr, i, j, p.inv_hz2, p.inv_hr2, p.rule);
                T g = p.f[(size_t)i * nr + j] + kf.a * nb(i - 1, j) + kf.c * nb(i + 1, j);
                T ee = kf.e;
                if (j == n - 1) {
                    g += ee * (p.zero_old ? (T)0 : p.u[(size_t)i * nr + nr - 1]);
                    ee = (T)0;
                }
                a = j == 0 ? (T)0 : -kf.d;
                b = kf.b;
                cc = -ee;
                r = g;
            }
            const int x = part_slot<Q>(e);
            SA[x] = a;
            SB[x] = b;
            SC[x] = cc;
            SR[x] = r;
        }
        __syncthreads();
        if (mine == ps) {
            // forward elimination inside the segment; ap couples to y_{t-1}
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int x = tl * (Q + 1) + q;
                const T a = SA[x], b = SB[x], r = SR[x];
                if (q == 0) {
                    ap[0] = a;
                    bp[0] = b;
                    rp[0] = r;
                } else {
                    const T mq = a / bp[q - 1];
                    ap[q] = -mq * ap[q - 1];
                    bp[q] = b - mq * c[q - 1];
                    rp[q] = r - mq * rp[q - 1];
                }
                c[q] = SC[x];
            }
        }
        __syncthreads();
    }
    T *RA = sm, *RB = sm + NT, *RC = sm + 2 * NT, *RR = sm + 3 * NT;
    T *X0 = sm + 4 * NT, *X1 = sm + 5 * NT, *X2 = sm + 6 * NT;
    // first unknown of the segment = al y_{t-1} + be y_t + ga
    T al = (T)0, be = (T)1, ga = (T)0;
#pragma unroll
    for (int q = Q - 2; q >= 0; --q) {
        const T ib = (T)1 / bp[q];
        const T nal = -(ap[q] + c[q] * al) * ib;
        const T nbe = -c[q] * be * ib;
        const T nga = (rp[q] - c[q] * ga) * ib;
        al = nal;
        be = nbe;
        ga = nga;
    }
    X0[t] = al;
    X1[t] = be;
    X2[t] = ga;
    __syncthreads();
    // reduced row of y_t: the segment's last row with its successor (the next
    // segment's first unknown) expressed through y_t and y_{t+1}
    {
        const T cl = c[Q - 1];
        const T nal = t + 1 < NT ? X0[t + 1] : (T)0, nbe = t + 1 < NT ? X1[t + 1] : (T)0;
        const T nga = t + 1 < NT ? X2[t + 1] : (T)0;
        RA[t] = ap[Q - 1];
        RB[t] = bp[Q - 1] + cl * nal;
        RC[t] = cl * nbe;
        RR[t] = rp[Q - 1] - cl * nga;
    }
    __syncthreads();
    pcr<T, 1>(RA, RB, RC, RR, NT, NT);
    const T yt = RR[t] / RB[t];
    const T yp = t > 0 ? RR[t - 1] / RB[t - 1] : (T)0;
    // back substitution into rp (rp[q] becomes the unknown t Q + q)
    rp[Q - 1] = yt;
#pragma unroll
    for (int q = Q - 2; q >= 0; --q) rp[q] = (rp[q] - ap[q] * yp - c[q] * rp[q + 1]) / bp[q];
    __syncthreads();
    // the solution leaves through LDS, pass by pass, in coalesced stores
    for (int ps = 0; ps < P; ++ps) {
        if (mine == ps) {
#pragma unroll
            for (int q = 0; q < Q; ++q) SA[tl * (Q + 1) + q] = rp[q];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int e = k * NT + t, j = ps * CH + e;
            if (j < n) {
                const T x = SA[part_slot<Q>(e)];
                p.u[(size_t)i * nr + j] = x;
                if (p.add_to) p.add_to[(size_t)i * nr + j] += (double)x;
            }
        }
        __syncthreads();
    }
}

// The block holds 16 wavefronts for the whole solve, mostly waiting at its
// barriers, so a second block on the compute unit hides that latency.  The
// FP32 form fits two blocks (at most 64 VGPRs, which costs the 8-unknown
// segments a few spilled registers, and <= 80 KB of LDS); the FP64 form,
// with 8 doubles per thread in each of four arrays, fits one.
template <typename T, int Q>
__global__ __launch_bounds__(kLongThreads) void k_line_part(LineArgs<T> p)
{
    line_part_body<T, Q>(p);
}

template <int Q>
__global__ __launch_bounds__(kLongThreads, 8) void k_line_part_f32(LineArgs<float> p)
{
    line_part_body<float, Q>(p);
}

template <typename T>
static hipError_t line(const MgLevels &m, int l, int parity, int zero_old, T *u, const T *f,
                       const T *eps, const T *uc, hipStream_t st, double *add_to = nullptr)
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
    p.add_to = add_to;
    const int rows = parity ? (p.nzl - 1) / 2 : (p.nzl - 3) / 2;
    if (rows <= 0) return hipSuccess;
    const int n = m.nr - 1;
    size_t lds = 8 * (size_t)n * sizeof(T);
    if (m.long_lines != 2 && lds <= m.lds_budget && n <= 1024 * 4) {
        int threads = ((n + 63) / 64) * 64;
        if (threads > 1024) threads = 1024;
        (void)launch<k_line_A<T>, k_line_body<T>, 1024>(dim3(rows), dim3(threads), lds, st, k_line_A<T>{p});
        return hipGetLastError();
    }
    // long lines: segments of Q unknowns per thread
    const int q = (n + kLongThreads - 1) / kLongThreads;
    if constexpr (sizeof(T) == sizeof(float)) {
        if (q <= 2)
            RZ_LAUNCH((k_line_part_f32<2>), dim3(rows), dim3(kLongThreads), (part_lds<T, 2>()), st, p);
        else if (q <= 4)
            RZ_LAUNCH((k_line_part_f32<4>), dim3(rows), dim3(kLongThreads), (part_lds<T, 4>()), st, p);
        else if (q <= 8)
            RZ_LAUNCH((k_line_part_f32<8>), dim3(rows), dim3(kLongThreads), (part_lds<T, 8>()), st, p);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    } else {
        if (q <= 2)
            RZ_LAUNCH((k_line_part<T, 2>), dim3(rows), dim3(kLongThreads), (part_lds<T, 2>()), st, p);
        else if (q <= 4)
            RZ_LAUNCH((k_line_part<T, 4>), dim3(rows), dim3(kLongThreads), (part_lds<T, 4>()), st, p);
        else if (q <= 8)
            RZ_LAUNCH((k_line_part<T, 8>), dim3(rows), dim3(kLongThreads), (part_lds<T, 8>()), st, p);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
}

struct k_add_corr_A {
    double *phi;
    const float *u;
    int nr;
    int nz;
};

__device__ __forceinline__ void k_add_corr_body(const Blk &kb_, const k_add_corr_A &A_)
{
    auto phi = A_.phi;
    auto u = A_.u;
    auto nr = A_.nr;
    auto nz = A_.nz;

    const int nn = nr * nz;
    for (int g = kb_.x * blockDim.x + threadIdx.x; g < nn; g += kb_.nx * blockDim.x) {
        int i = g / nr, j = g - i * nr;
        if (i > 0 && i < nz - 1 && j < nr - 1) phi[g] += (double)u[g];
    }
}


// Down-leg of the V(0,1) cycle: the block takes `cpb` unknown columns of the
// finest level, forms the residual f - A u there (u, eps staged in LDS with a
// one-column halo) and restricts it along z down every level,
// f^{l-1} = FW_z(f^l) (the coarse u^l are zero, so their residual is f^l).
// Mixed: the finest residual is also stored in FP32 as the right-hand side of
// the correction.
template <typename T>
__device__ __forceinline__ void down_body(const double *u, const double *f, const MgLevels &m,
                                          int mixed, int cpb, int blk)
{
    extern __shared__ double sbuf[];
    const int L = m.L, nr = m.nr, nz = m.nzl[L];
    const int w = cpb + 2;  // staged columns j0-1 .. j0+cpb
    double *us = sbuf, *es = sbuf + (size_t)w * nz;
    double *cur = es + (size_t)w * nz, *nxt = cur + (size_t)cpb * nz;
    const int j0 = blk * cpb;
    // the right-hand side of this thread's first residual node, loaded with
    // the staged columns rather than after their barrier (one round trip to
    // memory less)
    double f_first = 0.0;
    if ((int)threadIdx.x < cpb * nz) {
        const int i = threadIdx.x / cpb, j = j0 + (int)threadIdx.x - i * cpb;
        if (j < nr - 1 && i > 0 && i < nz - 1) f_first = f[(size_t)i * nr + j];
    }
    // consecutive threads take consecutive columns of a row (the loads of a
    // row are contiguous); LDS holds the block's columns one after another
    for (int t = threadIdx.x; t < w * nz; t += blockDim.x) {
        int i = t / w, cj = t - i * w, j = j0 - 1 + cj;
        bool in = j >= 0 && j < nr;
        us[cj * nz + i] = in ? u[(size_t)i * nr + j] : 0.0;
        es[cj * nz + i] = in ? m.eps64[L][(size_t)i * nr + j] : 1.0;
    }
    __syncthreads();
    const double hz = m.hzl[L];
    const double iz2 = 1.0 / (hz * hz), ir2 = 1.0 / (m.hr * m.hr);
    for (int t = threadIdx.x; t < cpb * nz; t += blockDim.x) {
        int i = t / cpb, cj = t - i * cpb, j = j0 + cj;
        double r = 0.0;
        if (j < nr - 1 && i > 0 && i < nz - 1) {
            const int k = (cj + 1) * nz + i;  // staged index of (i, j)
            auto E = [&](int di, int dj) { return es[k + dj * nz + di]; };
            auto U = [&](int di, int dj) { return us[k + dj * nz + di]; };
            double a = face<double>(E(-1, 0), E(0, 0), m.chi_face) * iz2;
            double c = face<double>(E(0, 0), E(1, 0), m.chi_face) * iz2;
            double d, e;
            if (j == 0) {
                d = 0.0;
                e = 4.0 * face<double>(E(0, 0), E(0, 1), m.chi_face) * ir2;
            } else {
                double jj = (double)j;
                d = face<double>(E(0, -1), E(0, 0), m.chi_face) * ((jj - 0.5) / jj) * ir2;
                e = face<double>(E(0, 0), E(0, 1), m.chi_face) * ((jj + 0.5) / jj) * ir2;
            }
            double b = a + c + d + e;
            double Au = b * U(0, 0) - a * U(-1, 0) - c * U(1, 0) - e * U(0, 1);
            if (j > 0) Au -= d * U(0, -1);
            r = (t == (int)threadIdx.x ? f_first : f[(size_t)i * nr + j]) - Au;
            if (mixed) m.f32[L][(size_t)i * nr + j] = (float)r;
        }
        cur[cj * nz + i] = r;
    }
    __syncthreads();
    int nzf = nz;
    for (int l = L - 1; l >= 1; --l) {
        const int nzc = m.nzl[l];
        T *fo = mixed ? (T *)m.f32[l] : (T *)m.f64[l];
        for (int t = threadIdx.x; t < cpb * nzc; t += blockDim.x) {
            int I = t / cpb, cj = t - I * cpb, j = j0 + cj;
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

template <typename T>
struct k_down_A {
    const double *u;
    const double *f;
    MgLevels m;
    int mixed;
    int cpb;
};

template <typename T>
__device__ __forceinline__ void k_down_body(const Blk &kb_, const k_down_A<T> &A_)
{
    auto u = A_.u;
    auto f = A_.f;
    const auto &m = A_.m;
    auto mixed = A_.mixed;
    auto cpb = A_.cpb;

    down_body<T>(u, f, m, mixed, cpb, kb_.x);
}


// The same down leg row by row, for large meshes (coalesced along r; the
// column form above reads a z-column per block).  The first launch takes the
// cells (I, j) of level L-1: it forms the finest residual on rows 2I-1, 2I,
// 2I+1 and restricts it, f^{L-1}_I = FW_z(r), so the finest residual never
// goes to memory; the mixed form also stores it in FP32 on rows 2I-1 and 2I
// (and the last interior row) as the correction's right-hand side.  The odd
// row between two blocks' row ranges is formed by both, identically.
// Then one launch per coarser level, f^{l-1} = FW_z(f^l), with the
// arithmetic of down_body.
__device__ __forceinline__ double resid_node(const double *u, const double *f, const double *ep,
                                             int64_t g, int nr, int j, double iz2, double ir2,
                                             int rule)
{
    auto E = [&](int di, int dj) { return ep[g + (int64_t)di * nr + dj]; };
    auto U = [&](int di, int dj) { return u[g + (int64_t)di * nr + dj]; };
    double a = face<double>(E(-1, 0), E(0, 0), rule) * iz2;
    double c = face<double>(E(0, 0), E(1, 0), rule) * iz2;
    double d, e;
    if (j == 0) {
        d = 0.0;
        e = 4.0 * face<double>(E(0, 0), E(0, 1), rule) * ir2;
    } else {
        double jj = (double)j;
        d = face<double>(E(0, -1), E(0, 0), rule) * ((jj - 0.5) / jj) * ir2;
        e = face<double>(E(0, 0), E(0, 1), rule) * ((jj + 0.5) / jj) * ir2;
    }
    double b = a + c + d + e;
    double Au = b * U(0, 0) - a * U(-1, 0) - c * U(1, 0) - e * U(0, 1);
    if (j > 0) Au -= d * U(0, -1);
    return f[g] - Au;
}

// Coarse rows of k_resid_restrict_rows per block: a thread walks them in
// order, carrying the residual of row 2I+1 over as the next row's 2I'-1.
constexpr int kResidRows = 8;

template <typename T>
__global__ void k_resid_restrict_rows(const double *u, const double *f, MgLevels m, T *dst,
                                      int mixed)
{
    const int L = m.L, nr = m.nr, nzc = m.nzl[L - 1];
    const double *ep = m.eps64[L];
    const double hz = m.hzl[L];
    const double iz2 = 1.0 / (hz * hz), ir2 = 1.0 / (m.hr * m.hr);
    float *f32 = mixed ? (float *)m.f32[L] : nullptr;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int I0 = 1 + blockIdx.y * kResidRows;
    const int I1 = I0 + kResidRows < nzc - 1 ? I0 + kResidRows : nzc - 1;
    if (j >= nr - 1) return;  // no barrier follows
    double r1 = resid_node(u, f, ep, (int64_t)(2 * I0 - 1) * nr + j, nr, j, iz2, ir2, m.chi_face);
    for (int I = I0; I < I1; ++I) {
        const int64_t g = (int64_t)(2 * I - 1) * nr + j;
        const double r2 = resid_node(u, f, ep, g + nr, nr, j, iz2, ir2, m.chi_face);
        const double r3 = resid_node(u, f, ep, g + 2 * nr, nr, j, iz2, ir2, m.chi_face);
        double v = 0.25 * r1 + 0.5 * r2 + 0.25 * r3;
        if (mixed) {
            v = (double)(float)v;  // coarse right-hand sides in FP32
            f32[g] = (float)r1;
            f32[g + nr] = (float)r2;
            if (I == nzc - 2) f32[g + 2 * nr] = (float)r3;
        }
        dst[(int64_t)I * nr + j] = (T)v;
        r1 = r3;
    }
}

// f^{l-1} from the level above (src: the finest residual, or f^l as stored).
template <typename S, typename T>
__global__ void k_restrict_rows(const S *src, T *dst, int nr, int nzc, int mixed)
{
    const int64_t ncell = (int64_t)(nzc - 2) * (nr - 1);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int I = 1 + (int)(t / (nr - 1)), j = (int)(t % (nr - 1));
        const int64_t r0 = (int64_t)(2 * I - 1) * nr + j;
        double v = 0.25 * (double)src[r0] + 0.5 * (double)src[r0 + nr] +
                   0.25 * (double)src[r0 + 2 * nr];
        if (mixed) v = (double)(float)v;  // coarse right-hand sides in FP32
        dst[(int64_t)I * nr + j] = (T)v;
    }
}

static int grid_blocks(int64_t n, int threads)
{
    const int64_t b = (n + threads - 1) / threads;
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

static hipError_t down_rows(const MgLevels &m, int mixed, const double *phi, const double *f,
                            hipStream_t st)
{
    const int L = m.L, nr = m.nr;
    const int threads = 256;
    for (int l = L - 1; l >= 1; --l) {
        const int nzc = m.nzl[l];
        const int blocks = grid_blocks((int64_t)(nzc - 2) * (nr - 1), threads);
        if (l == L - 1) {
            const dim3 g2((nr - 1 + threads - 1) / threads, (nzc - 2 + kResidRows - 1) / kResidRows);
            if (mixed)
                RZ_LAUNCH((k_resid_restrict_rows<float>), g2, dim3(threads), 0, st, phi, f, m,
                          m.f32[l], mixed);
            else
                RZ_LAUNCH((k_resid_restrict_rows<double>), g2, dim3(threads), 0, st, phi, f, m,
                          m.f64[l], mixed);
        } else if (mixed) {
            RZ_LAUNCH((k_restrict_rows<float, float>), dim3(blocks), dim3(threads), 0, st,
                      (const float *)m.f32[l + 1], m.f32[l], nr, nzc, mixed);
        } else {
            RZ_LAUNCH((k_restrict_rows<double, double>), dim3(blocks), dim3(threads), 0, st,
                      (const double *)m.f64[l + 1], m.f64[l], nr, nzc, mixed);
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Parallel cyclic reduction of `ne` tridiagonal equations held in LDS
// (A x_{j-1} + B x_j + C x_{j+1} = R), grouped in systems of n consecutive
// equations.  Each thread keeps its equations' new coefficients in registers
// between the two barriers of a step.  On return R/B is the solution.
template <typename T, int EPT>
__device__ __forceinline__ void pcr(T *A, T *Bd, T *C, T *Rr, int n, int ne)
{
    for (int s = 1; s < n; s <<= 1) {
        T na[EPT], nb[EPT], ncc[EPT], nr[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = threadIdx.x + q * blockDim.x;
            if (e >= ne) continue;
            const int j = e % n;
            T a = A[e], b = Bd[e], c = C[e], r = Rr[e], a2 = (T)0, c2 = (T)0;
            if (j >= s) {
                T k1 = a / Bd[e - s];
                a2 = -A[e - s] * k1;
                b -= C[e - s] * k1;
                r -= Rr[e - s] * k1;
            }
            if (j + s < n) {
                T k2 = c / Bd[e + s];
                c2 = -C[e + s] * k2;
                b -= A[e + s] * k2;
                r -= Rr[e + s] * k2;
            }
            na[q] = a2;
            nb[q] = b;
            ncc[q] = c2;
            nr[q] = r;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = threadIdx.x + q * blockDim.x;
            if (e >= ne) continue;
            A[e] = na[q];
            Bd[e] = nb[q];
            C[e] = ncc[q];
            Rr[e] = nr[q];
        }
        __syncthreads();
    }
}

// The coarse levels 1..K in one block, entirely in LDS: the exact solve of the
// single line of level 1, then for l = 2..K the prolonged correction (injected
// into the even lines the odd lines read) and one zebra sweep.  The coarse u^l
// start from zero; u^K is written out for the next level's prolongation.
template <typename T, int EPT>
struct k_bottom_A {
    MgLevels m;
    int mixed;
};

template <typename T, int EPT>
__device__ __forceinline__ void k_bottom_body(const Blk &kb_, const k_bottom_A<T, EPT> &A_)
{
    const auto &m = A_.m;
    auto mixed = A_.mixed;

    extern __shared__ unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    const int K = m.K, nr = m.nr, n = nr - 1;
    // level l occupies [eps | f | u] rows of nzl[l] x nr from lev(l)
    auto lev = [&](int l) {
        size_t o = 0;
        for (int q = 1; q < l; ++q) o += 3 * (size_t)m.nzl[q] * nr;
        return sm + o;
    };
    T *A = lev(K + 1);
    const int emax = ((m.nzl[K] - 1) / 2) * n;
    T *Bd = A + emax, *C = Bd + emax, *Rr = C + emax;
    for (int l = 1; l <= K; ++l) {
        const size_t sz = (size_t)m.nzl[l] * nr;
        T *le = lev(l);
        const T *ge = mixed ? (const T *)m.eps32[l] : (const T *)m.eps64[l];
        const T *gf = mixed ? (const T *)m.f32[l] : (const T *)m.f64[l];
        for (size_t t = threadIdx.x; t < sz; t += blockDim.x) {
            le[t] = ge[t];
            le[sz + t] = gf[t];
            le[2 * sz + t] = (T)0;
        }
    }
    __syncthreads();
    const T ir2 = (T)(1.0 / (m.hr * m.hr));
    for (int l = 1; l <= K; ++l) {
        const int nzl = m.nzl[l];
        const T iz2 = (T)(1.0 / (m.hzl[l] * m.hzl[l]));
        const size_t sz = (size_t)nzl * nr;
        const T *le = lev(l), *lf = le + sz;
        T *u = lev(l) + 2 * sz;
        const T *uc = l > 1 ? lev(l - 1) + 2 * (size_t)m.nzl[l - 1] * nr : nullptr;
        for (int parity = 1; parity >= 0; --parity) {
            const int lines = parity ? (nzl - 1) / 2 : (nzl - 3) / 2;
            if (lines <= 0) continue;
            const int ne = lines * n;
            for (int e = threadIdx.x; e < ne; e += blockDim.x) {
                const int t = e / n, j = e - t * n;
                const int i = parity ? 2 * t + 1 : 2 * t + 2;
                Coef<T> k = coef<T>(le, nr, i, j, iz2, ir2, m.chi_face);
                auto nb = [&](int row) -> T {
                    if (row == 0 || row == nzl - 1) return (T)0;
                    T v = u[(size_t)row * nr + j];
                    if (parity && uc) v += uc[(size_t)(row >> 1) * nr + j];
                    return v;
                };
                A[e] = j == 0 ? (T)0 : -k.d;
                Bd[e] = k.b;
                C[e] = j == n - 1 ? (T)0 : -k.e;
                Rr[e] = lf[(size_t)i * nr + j] + k.a * nb(i - 1) + k.c * nb(i + 1);
            }
            __syncthreads();
            pcr<T, EPT>(A, Bd, C, Rr, n, ne);
            for (int e = threadIdx.x; e < ne; e += blockDim.x) {
                const int t = e / n, j = e - t * n;
                const int i = parity ? 2 * t + 1 : 2 * t + 2;
                u[(size_t)i * nr + j] = Rr[e] / Bd[e];
            }
            __syncthreads();
        }
    }
    T *gu = mixed ? (T *)m.u32[K] : (T *)m.u64[K];
    const size_t szK = (size_t)m.nzl[K] * nr;
    const T *uK = lev(K) + 2 * szK;
    for (size_t t = threadIdx.x; t < szK; t += blockDim.x) gu[t] = uK[t];
}


template <typename T> struct LevelArgs {
    int nr, nzl, rule, zero_old;
    T iz2, ir2;
    const T *eps, *f;
    const T *u_in;   // old values (finest FP64 level), else null
    const T *uc;     // coarse correction injected into the even neighbours
    T *u_out;        // new values of the level, or null
    double *add_to;  // mixed finest level: phi += correction of the owned lines
};

// One zebra sweep of a level in one launch.  Block b owns even line i = 2b+2:
// it solves the odd lines i-1 and i+1 (neighbours: even lines with their old
// value plus the injected coarse correction) -- the odd lines next to two even
// lines are solved, identically, by both blocks -- then line i from them.
// Odd line i-1 is owned by block i, and the last odd line by the last block.
template <typename T, int EPT>
struct k_level_A {
    LevelArgs<T> p;
};

template <typename T, int EPT>
__device__ __forceinline__ void k_level_body(const Blk &kb_, const k_level_A<T, EPT> &A_)
{
    const auto &p = A_.p;

    extern __shared__ unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    const int nr = p.nr, n = nr - 1, nzl = p.nzl;
    const int i = 2 * kb_.x + 2;
    const bool last = i + 1 == nzl - 2;
    T *A = sm, *Bd = A + 2 * n, *C = Bd + 2 * n, *Rr = C + 2 * n;
    auto old = [&](int row, int j) -> T {
        return p.zero_old ? (T)0 : p.u_in[(size_t)row * nr + j];
    };
    auto nb = [&](int row, int j) -> T {
        T v = old(row, j);
        if (row != 0 && row != nzl - 1 && p.uc) v += p.uc[(size_t)(row >> 1) * nr + j];
        return v;
    };
    // odd lines i-1 (t = 0) and i+1 (t = 1)
    for (int e = threadIdx.x; e < 2 * n; e += blockDim.x) {
        const int t = e / n, j = e - t * n;
        const int io = i - 1 + 2 * t;
        Coef<T> k = coef<T>(p.eps, nr, io, j, p.iz2, p.ir2, p.rule);
        T g = p.f[(size_t)io * nr + j] + k.a * nb(io - 1, j) + k.c * nb(io + 1, j);
        T ce = k.e;
        if (j == n - 1) {
            g += ce * old(io, nr - 1);
            ce = (T)0;
        }
        A[e] = j == 0 ? (T)0 : -k.d;
        Bd[e] = k.b;
        C[e] = -ce;
        Rr[e] = g;
    }
    __syncthreads();
    pcr<T, EPT>(A, Bd, C, Rr, n, 2 * n);
    // solutions of the odd lines stay in Rr (as x = R/B), then the even line
    for (int e = threadIdx.x; e < 2 * n; e += blockDim.x) {
        const int t = e / n, j = e - t * n;
        const int io = i - 1 + 2 * t;
        const T x = Rr[e] / Bd[e];
        Rr[e] = x;
        if (p.u_out) p.u_out[(size_t)io * nr + j] = x;
        if (p.add_to && (t == 0 || last)) p.add_to[(size_t)io * nr + j] += (double)x;
    }
    __syncthreads();
    T *A2 = Rr + 2 * n, *B2 = A2 + n, *C2 = B2 + n, *R2 = C2 + n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        Coef<T> k = coef<T>(p.eps, nr, i, j, p.iz2, p.ir2, p.rule);
        T g = p.f[(size_t)i * nr + j] + k.a * Rr[j] + k.c * Rr[n + j];
        T ce = k.e;
        if (j == n - 1) {
            g += ce * old(i, nr - 1);
            ce = (T)0;
        }
        A2[j] = j == 0 ? (T)0 : -k.d;
        B2[j] = k.b;
        C2[j] = -ce;
        R2[j] = g;
    }
    __syncthreads();
    pcr<T, EPT>(A2, B2, C2, R2, n, n);
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const T x = R2[j] / B2[j];
        if (p.u_out) p.u_out[(size_t)i * nr + j] = x;
        if (p.add_to) p.add_to[(size_t)i * nr + j] += (double)x;
    }
}


template <typename T>
static hipError_t level_sweep(const MgLevels &m, int l, int zero_old, const T *u_in,
                              const T *uc, T *u_out, const T *f, const T *eps, double *add_to,
                              hipStream_t st)
{
    LevelArgs<T> p;
    p.nr = m.nr;
    p.nzl = m.nzl[l];
    p.rule = m.chi_face;
    p.zero_old = zero_old;
    p.iz2 = (T)(1.0 / (m.hzl[l] * m.hzl[l]));
    p.ir2 = (T)(1.0 / (m.hr * m.hr));
    p.eps = eps;
    p.f = f;
    p.u_in = u_in;
    p.uc = uc;
    p.u_out = u_out;
    p.add_to = add_to;
    const int blocks = (p.nzl - 3) / 2;
    if (blocks <= 0) return hipSuccess;
    const int n = m.nr - 1;
    int threads = ((2 * n + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    const int ept = (2 * n + threads - 1) / threads;  // 2 n <= 4096 here: at most 4
    size_t lds = 12 * (size_t)n * sizeof(T);
    if (ept <= 1)
        (void)launch<k_level_A<T, 1>, k_level_body<T, 1>, 1024>(dim3(blocks), dim3(threads), lds, st, k_level_A<T, 1>{p});
    else if (ept <= 2)
        (void)launch<k_level_A<T, 2>, k_level_body<T, 2>, 1024>(dim3(blocks), dim3(threads), lds, st, k_level_A<T, 2>{p});
    else
        (void)launch<k_level_A<T, 4>, k_level_body<T, 4>, 1024>(dim3(blocks), dim3(threads), lds, st, k_level_A<T, 4>{p});
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Single-block path.
//
// Line tables.  Every interior line (level l, row i) is the tridiagonal system
// -d x_{j-1} + b x_j - e x_{j+1} = g of its r-line; the matrix does not change
// during a solve, so the multipliers of the parallel cyclic reduction are
// formed once here and a sweep only carries right-hand sides.  The table of
// one line holds rows of n = nr - 1 values:
//   a | c | b after the last step | k1, k2 of step 0 | k1, k2 of step 1 | ...
// with k1 = A_j / B_{j-s} (0 for j < s) and k2 = C_j / B_{j+s} (0 for
// j + s >= n), s = 2^step, exactly the products the reduction forms.
template <typename T> __device__ __forceinline__ void factor_body(const MgLevels &m, int mixed, int blk)
{
    if (blk >= m.line_off[m.L + 1]) {
        // the FP64 operator of the finest level, row by row: a, b, c, d, e
        const int L = m.L, nr = m.nr, n = nr - 1, nn = m.nzl[L] * nr;
        const int i = blk - m.line_off[L + 1] + 1;
        const double iz2 = 1.0 / (m.hzl[L] * m.hzl[L]), ir2 = 1.0 / (m.hr * m.hr);
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            Coef<double> k = coef<double>(m.eps64[L], nr, i, j, iz2, ir2, m.chi_face);
            const size_t g = (size_t)i * nr + j;
            m.cf64[g] = k.a;
            m.cf64[nn + g] = k.b;
            m.cf64[2 * (size_t)nn + g] = k.c;
            m.cf64[3 * (size_t)nn + g] = k.d;
            m.cf64[4 * (size_t)nn + g] = k.e;
        }
        return;
    }
    extern __shared__ unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    const int line = blk;
    int l = 1;
    while (line >= m.line_off[l + 1]) ++l;
    const int i = line - m.line_off[l] + 1;
    const int nr = m.nr, n = nr - 1, tn = m.tab_row;
    T *tab = (T *)m.tab + (size_t)line * m.tab_stride;
    const T *eps = mixed ? (const T *)m.eps32[l] : (const T *)m.eps64[l];
    const T iz2 = (T)(1.0 / (m.hzl[l] * m.hzl[l])), ir2 = (T)(1.0 / (m.hr * m.hr));
    T *A = sm, *Bd = A + n, *C = Bd + n;
    const int j = threadIdx.x;  // blockDim.x >= n
    if (j < n) {
        Coef<T> k = coef<T>(eps, nr, i, j, iz2, ir2, m.chi_face);
        tab[2 * j] = k.a;
        tab[2 * j + 1] = k.c;
        A[j] = j == 0 ? (T)0 : -k.d;
        Bd[j] = k.b;
        C[j] = j == n - 1 ? (T)0 : -k.e;
    }
    __syncthreads();
    int q = 0;
    for (int s = 1; s < n; s <<= 1, ++q) {
        T a2 = (T)0, b = (T)0, c2 = (T)0;
        if (j < n) {
            T a = A[j], c = C[j], k1 = (T)0, k2 = (T)0;
            b = Bd[j];
            if (j >= s) {
                k1 = a / Bd[j - s];
                a2 = -A[j - s] * k1;
                b -= C[j - s] * k1;
            }
            if (j + s < n) {
                k2 = c / Bd[j + s];
                c2 = -C[j + s] * k2;
                b -= A[j + s] * k2;
            }
            tab[(size_t)(3 + 2 * q) * tn + 2 * j] = k1;
            tab[(size_t)(3 + 2 * q) * tn + 2 * j + 1] = k2;
        }
        __syncthreads();
        if (j < n) {
            A[j] = a2;
            Bd[j] = b;
            C[j] = c2;
        }
        __syncthreads();
    }
    if (j < n) tab[2 * tn + j] = Bd[j];
    // the padding of every row (read by vector loads of whole lane groups):
    // zero coefficients and multipliers and b_final 1, so that it stays
    // finite and inert
    if (j >= n && j < tn) {
        tab[2 * tn + j] = (T)1;
        for (int p = 0; p <= m.S; ++p) {
            const size_t base = p == 0 ? 0 : (size_t)(1 + 2 * p) * tn;
            tab[base + 2 * j] = (T)0;
            tab[base + 2 * j + 1] = (T)0;
        }
    }
}

template <typename T>
struct k_factor_A {
    MgLevels m;
    int mixed;
};

template <typename T>
__device__ __forceinline__ void k_factor_body(const Blk &kb_, const k_factor_A<T> &A_)
{
    const auto &m = A_.m;
    auto mixed = A_.mixed;

    factor_body<T>(m, mixed, kb_.x);
}


// Split path, first launch of a solve: the line tables of every level
// (blocks [0, nfb)) and, beside them, the first cycle's finest residual
// restricted to every level (the remaining blocks, cpb columns each).
template <typename T>
struct k_prep_A {
    const double *u;
    const double *f;
    MgLevels m;
    int mixed;
    int cpb;
    int nfb;
};

template <typename T>
__device__ __forceinline__ void k_prep_body(const Blk &kb_, const k_prep_A<T> &A_)
{
    auto u = A_.u;
    auto f = A_.f;
    const auto &m = A_.m;
    auto mixed = A_.mixed;
    auto cpb = A_.cpb;
    auto nfb = A_.nfb;

    if ((int)kb_.x < nfb) factor_body<T>(m, mixed, kb_.x);
    else down_body<T>(u, f, m, mixed, cpb, kb_.x - nfb);
}


static size_t down_lds(int nz, int cpb)
{
    return (2 * (size_t)(cpb + 2) + 2 * (size_t)cpb) * nz * sizeof(double);
}

hipError_t mg_prep(const MgLevels &m, int mixed, const double *phi, const double *f,
                   hipStream_t st)
{
    const int nz = m.nzl[m.L], n = m.nr - 1;
    const int cpb = cols_per_block(nz);
    const int nfb = m.line_off[m.L + 1], nd = (n + cpb - 1) / cpb;
    size_t lds = down_lds(nz, cpb);
    const size_t lf = 3 * (size_t)n * (mixed ? sizeof(float) : sizeof(double));
    if (lf > lds) lds = lf;
    if (mixed)
        (void)launch<k_prep_A<float>, k_prep_body<float>, 256>(dim3(nfb + nd), dim3(256), lds, st, k_prep_A<float>{phi, f, m, mixed, cpb, nfb});
    else
        (void)launch<k_prep_A<double>, k_prep_body<double>, 256>(dim3(nfb + nd), dim3(256), lds, st, k_prep_A<double>{phi, f, m, mixed, cpb, nfb});
    return hipGetLastError();
}

// Step pipelining: the list maintenance of one step runs beside the grid
// preparation of the next, in two launches of kSuper threads instead of
// four.  The grid blocks come first (the longer chains), then the list
// blocks, (superchunk, job) flattened superchunk-fastest.  The bodies loop
// over blockDim.x, so they run unchanged at this width.
struct k_fin_scan_A {
    k_finalize_mg_A f;
    ScanJobs j;
    int nf, nsc;
};

__device__ __forceinline__ void k_fin_scan_body(const Blk &kb_, const k_fin_scan_A &A_)
{
    if (kb_.x < A_.nf) {
        k_finalize_mg_body(Blk{kb_.x, 0, A_.nf, 1}, A_.f);
        return;
    }
    const int b = kb_.x - A_.nf;
    scan_body(Blk{b % A_.nsc, b / A_.nsc, A_.nsc, 3}, A_.j);
}

template <typename T> struct k_prep_dl_A {
    k_prep_A<T> p;
    ScanJobs j;
    int np, nsc;
};

template <typename T>
__device__ __forceinline__ void k_prep_dl_body(const Blk &kb_, const k_prep_dl_A<T> &A_)
{
    if (kb_.x < A_.np) {
        k_prep_body<T>(Blk{kb_.x, 0, A_.np, 1}, A_.p);
        return;
    }
    const int b = kb_.x - A_.np;
    dead_list_body(Blk{b % A_.nsc, b / A_.nsc, A_.nsc, 2}, A_.j);
}

static int superchunks(int64_t max_chunks)
{
    const int64_t nsc = (max_chunks + kSuper - 1) / kSuper;
    return nsc < 1 ? 1 : (int)nsc;
}

hipError_t mg_finalize_scan(const GridArgs &g, const MgLevels &m, int mixed, double *phi0,
                            double *phi1, double V, const ScanJobs &j, int64_t max_chunks,
                            hipStream_t st)
{
    const int nz = m.nzl[m.L];
    int cpb = cols_per_block(nz);
    if (cpb < 1) cpb = 1;
    const int nf = (m.nr + cpb - 1) / cpb, nsc = superchunks(max_chunks);
    const size_t lds = 2 * (size_t)cpb * nz * sizeof(double);
    static_assert(sizeof(k_fin_scan_A) <= 4096, "kernel arguments");
    (void)launch<k_fin_scan_A, k_fin_scan_body, kSuper>(
        dim3(nf + 3 * nsc), dim3(kSuper), lds, st,
        k_fin_scan_A{k_finalize_mg_A{g, m, mixed, cpb, phi0, phi1, V, nullptr, 0}, j, nf, nsc});
    return hipGetLastError();
}

hipError_t mg_prep_dead_list(const MgLevels &m, int mixed, const double *phi, const double *f,
                             const ScanJobs &j, int64_t max_chunks, hipStream_t st)
{
    const int nz = m.nzl[m.L], n = m.nr - 1;
    const int cpb = cols_per_block(nz);
    const int nfb = m.line_off[m.L + 1], nd = (n + cpb - 1) / cpb, nsc = superchunks(max_chunks);
    size_t lds = down_lds(nz, cpb);
    const size_t lf = 3 * (size_t)n * (mixed ? sizeof(float) : sizeof(double));
    if (lf > lds) lds = lf;
    const dim3 grid(nfb + nd + 2 * nsc);
    if (mixed) {
        static_assert(sizeof(k_prep_dl_A<float>) <= 4096, "kernel arguments");
        (void)launch<k_prep_dl_A<float>, k_prep_dl_body<float>, kSuper>(
            grid, dim3(kSuper), lds, st,
            k_prep_dl_A<float>{k_prep_A<float>{phi, f, m, mixed, cpb, nfb}, j, nfb + nd, nsc});
    } else {
        static_assert(sizeof(k_prep_dl_A<double>) <= 4096, "kernel arguments");
        (void)launch<k_prep_dl_A<double>, k_prep_dl_body<double>, kSuper>(
            grid, dim3(kSuper), lds, st,
            k_prep_dl_A<double>{k_prep_A<double>{phi, f, m, mixed, cpb, nfb}, j, nfb + nd, nsc});
    }
    return hipGetLastError();
}

hipError_t mg_factor(const MgLevels &m, int mixed, hipStream_t st)
{
    // one block per line of every level, then one per interior row of the
    // finest level for its FP64 operator
    const int blocks = m.line_off[m.L + 1] + (m.nzl[m.L] - 2), n = m.nr - 1;
    const int threads = ((n + 63) / 64) * 64;  // n <= 256 on this path
    if (mixed)
        (void)launch<k_factor_A<float>, k_factor_body<float>, 256>(dim3(blocks), dim3(threads), 3 * n * sizeof(float), st, k_factor_A<float>{m, mixed});
    else
        (void)launch<k_factor_A<double>, k_factor_body<double>, 256>(dim3(blocks), dim3(threads), 3 * n * sizeof(double), st, k_factor_A<double>{m, mixed});
    return hipGetLastError();
}

// V(0,1) cycles in one block of 16 wavefronts.  Level l keeps [u | f] rows in
// LDS (FP64: levels below the finest; the finest level is phi and the global
// right-hand side).  Down: the finest residual in FP64 (to a global scratch),
// restricted along z level by level.  Up: one wavefront per r-line, Q
// unknowns per lane (j = q*64 + lane); the reduction steps exchange
// right-hand sides across lanes with shuffles, so a line needs no block
// barrier, and the block synchronises once per half-sweep.
// One r-line per wavefront: Q unknowns per lane (j = q*64 + lane).  The
// line's table (coefficients a, c of the neighbouring lines, the final
// diagonal and the reduction multipliers of every step) is loaded with
// clamped indices, so that no load sits behind a lane-dependent branch.
template <typename T, int Q, int SMAX> struct LineTab {
    T ta[Q], tc[Q], bf[Q], k1[SMAX][Q], k2[SMAX][Q];
};

// Layout of a line table (factor_body), tn = tab_row elements per row: the
// coefficients a, c of unknown j at 2j and 2j + 1 (a pair row of 2 tn
// elements), b_final at 2 tn + j, then for reduction step st the
// multipliers k1, k2 at (3 + 2 st) tn + 2j and + 1.  Values used together
// sit side by side, so that one load brings both.
__device__ __forceinline__ size_t tab_pair_row(int p)  // p = 0: (a, c); p = 1 + st: (k1, k2)
{
    return p == 0 ? 0 : (size_t)(1 + 2 * p);
}

// The pair (x, y) of unknown j of pair row p at the 32-bit byte offset
// 2 j sizeof(T): the row base is the same for the whole wavefront (scalar
// registers), the offset one register that every row shares (j < n <= 8192).
template <typename T>
__device__ __forceinline__ void tab_pair_at(const T *tb, int p, int tn, uint32_t off2, T &x, T &y)
{
    typedef T V __attribute__((ext_vector_type(2)));
    const V v = *(const V *)((const char *)(tb + tab_pair_row(p) * (size_t)tn) + off2);
    x = v[0];
    y = v[1];
}

// The loads alone (clamped indices), then the masking of unknowns past the
// line's end and of reduction steps past S: a prefetched table is masked only
// when it is used, so nothing waits for its loads before then.
template <typename T, int Q, int SMAX>
__device__ __forceinline__ void line_tab_fetch(const T *tb, int n, int tn, int S, int lane,
                                               LineTab<T, Q, SMAX> &t)
{
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = q * 64 + lane;
        const int jj = j < n ? j : n - 1;
        const uint32_t off = (uint32_t)jj * (uint32_t)sizeof(T);
        tab_pair_at(tb, 0, tn, 2 * off, t.ta[q], t.tc[q]);
        t.bf[q] = *(const T *)((const char *)(tb + 2 * (size_t)tn) + off);
#pragma unroll
        for (int st = 0; st < SMAX; ++st) {
            const int sc = st < S ? st : S - 1;
            tab_pair_at(tb, 1 + sc, tn, 2 * off, t.k1[st][q], t.k2[st][q]);
        }
    }
}

template <typename T, int Q, int SMAX>
__device__ __forceinline__ void line_tab_mask(int n, int S, int lane, LineTab<T, Q, SMAX> &t)
{
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const bool ok = q * 64 + lane < n;
        t.bf[q] = ok ? t.bf[q] : (T)1;
#pragma unroll
        for (int st = 0; st < SMAX; ++st) {
            const bool have = ok && st < S;
            t.k1[st][q] = have ? t.k1[st][q] : (T)0;
            t.k2[st][q] = have ? t.k2[st][q] : (T)0;
        }
    }
}

template <typename T, int Q, int SMAX>
__device__ __forceinline__ void line_tab_load(const T *tb, int n, int tn, int S, int lane,
                                              LineTab<T, Q, SMAX> &t)
{
    line_tab_fetch<T, Q, SMAX>(tb, n, tn, S, lane, t);
    line_tab_mask<T, Q, SMAX>(n, S, lane, t);
}

// The reduction steps on the right-hand sides R (zero for j >= n), then the
// solution x = R / b_final in R.  Neighbours at distance s come through lane
// shuffles (s < 64) or other registers of the same lane (s >= 64).
template <typename T, int Q, int SMAX>
__device__ __forceinline__ void line_pcr(T (&R)[Q], const LineTab<T, Q, SMAX> &t, int S, int lane)
{
#pragma unroll
    for (int st = 0; st < SMAX; ++st) {
        if (st >= S) break;
        const int s = 1 << st;
        T nR[Q];
        if (s < 64) {
            T dn[Q], up[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                dn[q] = __shfl(R[q], (lane - s) & 63, 64);
                up[q] = __shfl(R[q], (lane + s) & 63, 64);
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const T left = lane >= s ? dn[q] : (q > 0 ? dn[q > 0 ? q - 1 : 0] : (T)0);
                const T right = lane + s < 64 ? up[q] : (q + 1 < Q ? up[q + 1 < Q ? q + 1 : q] : (T)0);
                nR[q] = R[q] - left * t.k1[st][q] - right * t.k2[st][q];
            }
        } else {
            const int kq = s >> 6;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const T left = q >= kq ? R[q >= kq ? q - kq : 0] : (T)0;
                const T right = q + kq < Q ? R[q + kq < Q ? q + kq : q] : (T)0;
                nR[q] = R[q] - left * t.k1[st][q] - right * t.k2[st][q];
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) R[q] = nR[q];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) R[q] = R[q] / t.bf[q];
}

template <typename T, int Q>
struct k_solve_A {
    MgLevels m;
    int mixed;
    double *phi;
    const double *f;
    double V;
    int cycles;
    int coarse;
};

template <typename T, int Q>
__device__ __forceinline__ void k_solve_body(const Blk &kb_, const k_solve_A<T, Q> &A_)
{
    const auto &m = A_.m;
    auto mixed = A_.mixed;
    auto phi = A_.phi;
    auto f = A_.f;
    auto V = A_.V;
    auto cycles = A_.cycles;
    auto coarse = A_.coarse;

    constexpr int SMAX = Q == 1 ? 6 : Q == 2 ? 7 : 8;
    constexpr int RU = 4;  // residuals per thread computed before any is stored
    extern __shared__ unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    const int L = m.L, nr = m.nr, n = nr - 1, nz = m.nzl[L], S = m.S;
    // wave index through readfirstlane: the compiler then knows it is uniform
    // across the wavefront, and the level tables it indexes (line offsets,
    // level sizes) come through scalar loads
    const int lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    auto lev = [&](int l) {  // u of level l; its f follows at + nzl * nr
        size_t o = 0;
        for (int q = 1; q < l; ++q) o += 2 * (size_t)m.nzl[q] * nr;
        return sm + o;
    };
    // ---- up: exact coarsest line, then prolongation + zebra sweep per level
    auto up = [&](int top) {
    for (int l = 1; l <= top; ++l) {
        const int nzl = m.nzl[l];
        const bool fine = l == L, direct = fine && !mixed;
        // LDS rows of this level (not used when direct) and of the level below
        T *ul = lev(direct ? 1 : l);
        const T *fl = ul + (size_t)(direct ? 0 : nzl) * nr;
        const T *uc = lev(l > 1 ? l - 1 : 1);
        for (int parity = 1; parity >= 0; --parity) {
            const int lines = parity ? (nzl - 1) / 2 : (nzl - 3) / 2;
            for (int t = wave; t < lines; t += nwaves) {
                const int i = parity ? 2 * t + 1 : 2 * t + 2;
                const T *tb = (const T *)m.tab + (size_t)(m.line_off[l] + i - 1) * m.tab_stride;
                LineTab<T, Q, SMAX> tab;
                line_tab_load<T, Q, SMAX>(tb, n, m.tab_row, S, lane, tab);
                T R[Q];
                double ph[Q];  // phi of the line (mixed finest level: phi += x)
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int j = q * 64 + lane;
                    const bool ok = j < n;
                    const int jj = ok ? j : n - 1;
                    // neighbour rows: coarse correction injected into the even
                    // rows i-1, i+1 (their index halves), or the level's own rows
                    const T cl = uc[(size_t)((i - 1) >> 1) * nr + jj];
                    const T ch = uc[(size_t)((i + 1) >> 1) * nr + jj];
                    const bool inj = parity && l > 1;
                    const T cl_ = (inj && i - 1 > 0) ? cl : (T)0;
                    const T ch_ = (inj && i + 1 < nzl - 1) ? ch : (T)0;
                    T lo, hi, g;
                    ph[q] = 0.0;
                    if (direct) {
                        const double vlo = phi[(size_t)(i - 1) * nr + jj];
                        const double vhi = phi[(size_t)(i + 1) * nr + jj];
                        lo = (T)(vlo + (double)cl_);
                        hi = (T)(vhi + (double)ch_);
                        g = (T)f[(size_t)i * nr + jj];
                    } else {
                        const T ol = ul[(size_t)(i - 1) * nr + jj], oh = ul[(size_t)(i + 1) * nr + jj];
                        lo = parity ? cl_ : ol;
                        hi = parity ? ch_ : oh;
                        g = fl[(size_t)i * nr + jj];
                        if (fine) ph[q] = phi[(size_t)i * nr + jj];
                    }
                    R[q] = ok ? g + tab.ta[q] * lo + tab.tc[q] * hi : (T)0;
                }
                line_pcr<T, Q, SMAX>(R, tab, S, lane);
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int j = q * 64 + lane;
                    if (j >= n) continue;
                    const T x = R[q];
                    const size_t at = (size_t)i * nr + j;
                    if (direct) {
                        phi[at] = (double)x;
                    } else {
                        ul[at] = x;
                        if (fine) phi[at] = ph[q] + (double)x;
                    }
                }
            }
            __syncthreads();
        }
    }
    };
    if (coarse) {
        // levels 1..L-1 only: their right-hand sides come from a multi-block
        // residual and restriction launch, the correction u^{L-1} goes back to
        // global memory for the finest level's launch
        // The levels' global arrays are one block laid out like this LDS
        // image (u then f of each level), so the copy is one flat loop; each
        // thread issues a batch of loads (up to 24) before any store, so the
        // copy costs one global round trip.  The u rows it brings along are
        // written by the sweeps before they are read.
        {
            constexpr int U = 24;
            size_t total = 0;
            for (int l = 1; l <= L - 1; ++l) total += 2 * (size_t)m.nzl[l] * nr;
            const T *src = (const T *)m.coarse_uf;
            for (size_t t0 = threadIdx.x; t0 < total; t0 += (size_t)U * blockDim.x) {
                T v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const size_t t = t0 + (size_t)u * blockDim.x;
                    v[u] = src[t < total ? t : total - 1];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const size_t t = t0 + (size_t)u * blockDim.x;
                    if (t < total) sm[t] = v[u];
                }
            }
        }
        __syncthreads();
        up(L - 1);
        const size_t szc = (size_t)m.nzl[L - 1] * nr;
        const T *uc = lev(L - 1);
        T *gu = mixed ? (T *)m.u32[L - 1] : (T *)m.u64[L - 1];
        for (size_t t = threadIdx.x; t < szc; t += blockDim.x) gu[t] = uc[t];
        return;
    }
    for (int t = threadIdx.x; t < nr + nz; t += blockDim.x) {
        if (t < nr) {
            phi[t] = t < nr - 1 ? V : 0.0;
            phi[(size_t)(nz - 1) * nr + t] = 0.0;
        } else {
            phi[(size_t)(t - nr) * nr + nr - 1] = 0.0;
        }
    }
    __syncthreads();
    for (int cyc = 0; cyc < cycles; ++cyc) {
        // ---- down.  Memory accesses carry no lane-dependent branch (indices
        // are clamped instead), so the loads of four unknowns per thread are in
        // flight together.
        if (mixed || L > 1) {
            T *fL = lev(mixed ? L : 1) + (size_t)(mixed ? nz : 0) * nr;  // used when mixed
            const int nn = nz * nr, NI = (nz - 2) * n;
            // all residuals of a chunk first (loads only), then their stores:
            // a store before a load would make every later load wait for it.
            // Unknown g = (i-1) n + j walks with the block stride, (i, j)
            // carried along without a division.
            const double *ca = m.cf64, *cb = ca + nn, *cc = cb + nn, *cd = cc + nn, *ce = cd + nn;
            const int si = (int)blockDim.x / n, sj = (int)blockDim.x - si * n;
            int i0 = 1 + (int)threadIdx.x / n, j0 = (int)threadIdx.x - (i0 - 1) * n;
            for (int g0 = threadIdx.x; g0 < NI; g0 += RU * blockDim.x) {
                double r[RU];
                int ii = i0, jj = j0;
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    // clamp past the end to the last unknown (loads stay in bounds)
                    const bool in = g0 + u * (int)blockDim.x < NI;
                    const int i = in ? ii : nz - 2, j = in ? jj : n - 1;
                    const int o = i * nr + j, w = j > 0 ? o - 1 : o;
                    const double Au = cb[o] * phi[o] - ca[o] * phi[o - nr] - cc[o] * phi[o + nr] -
                                      ce[o] * phi[o + 1] - cd[o] * phi[w];  // d = 0 on the axis
                    r[u] = f[o] - Au;
                    ii += si;
                    jj += sj;
                    if (jj >= n) {
                        jj -= n;
                        ++ii;
                    }
                }
                ii = i0;
                jj = j0;
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    if (g0 + u * (int)blockDim.x < NI) {
                        const size_t k = (size_t)ii * nr + jj;
                        if (L > 1) m.res[k] = r[u];
                        if (mixed) fL[k] = (T)r[u];
                    }
                    ii += si;
                    jj += sj;
                    if (jj >= n) {
                        jj -= n;
                        ++ii;
                    }
                }
                i0 = ii;
                j0 = jj;
            }
            __syncthreads();
            if (L > 1) {
                const int nzc = m.nzl[L - 1], NC = (nzc - 2) * n;
                T *fc = lev(L - 1) + (size_t)nzc * nr;
                for (int g0 = threadIdx.x; g0 < NC; g0 += 4 * blockDim.x) {
                    double v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int g = min(g0 + u * (int)blockDim.x, NC - 1);
                        const int I = 1 + g / n, j = g - (I - 1) * n;
                        const double *col = m.res + j;
                        v[u] = 0.25 * col[(size_t)(2 * I - 1) * nr] + 0.5 * col[(size_t)(2 * I) * nr] +
                               0.25 * col[(size_t)(2 * I + 1) * nr];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int g = g0 + u * (int)blockDim.x;
                        if (g < NC) {
                            const int I = 1 + g / n, j = g - (I - 1) * n;
                            fc[(size_t)I * nr + j] = (T)v[u];
                        }
                    }
                }
                __syncthreads();
                for (int l = L - 2; l >= 1; --l) {
                    const int nzl = m.nzl[l], nzf = m.nzl[l + 1];
                    T *fo = lev(l) + (size_t)nzl * nr;
                    const T *fi = lev(l + 1) + (size_t)nzf * nr;
                    for (int g = threadIdx.x; g < (nzl - 2) * n; g += blockDim.x) {
                        const int I = 1 + g / n, j = g - (I - 1) * n;
                        const T *col = fi + j;
                        double v = 0.25 * (double)col[(size_t)(2 * I - 1) * nr] +
                                   0.5 * (double)col[(size_t)(2 * I) * nr] +
                                   0.25 * (double)col[(size_t)(2 * I + 1) * nr];
                        fo[(size_t)I * nr + j] = (T)v;
                    }
                    __syncthreads();
                }
            }
        }
        up(L);
    }
}


static hipError_t solve_block(const MgLevels &m, int mixed, double *phi, const double *f, double V,
                              int cycles, int coarse, hipStream_t st)
{
    const int n = m.nr - 1;
    const size_t lds = m.solve_lds;
    if (mixed) {
        if (n <= 64)
            (void)launch<k_solve_A<float, 1>, k_solve_body<float, 1>, 1024>(dim3(1), dim3(1024), lds, st, k_solve_A<float, 1>{m, mixed, phi, f, V, cycles, coarse});
        else if (n <= 128)
            (void)launch<k_solve_A<float, 2>, k_solve_body<float, 2>, 1024>(dim3(1), dim3(1024), lds, st, k_solve_A<float, 2>{m, mixed, phi, f, V, cycles, coarse});
        else
            (void)launch<k_solve_A<float, 4>, k_solve_body<float, 4>, 1024>(dim3(1), dim3(1024), lds, st, k_solve_A<float, 4>{m, mixed, phi, f, V, cycles, coarse});
    } else {
        if (n <= 64)
            (void)launch<k_solve_A<double, 1>, k_solve_body<double, 1>, 1024>(dim3(1), dim3(1024), lds, st, k_solve_A<double, 1>{m, mixed, phi, f, V, cycles, coarse});
        else
            (void)launch<k_solve_A<double, 2>, k_solve_body<double, 2>, 1024>(dim3(1), dim3(1024), lds, st, k_solve_A<double, 2>{m, mixed, phi, f, V, cycles, coarse});
    }
    return hipGetLastError();
}

// Finest level of the split cycle, one block of two wavefronts per even line
// i = 2b+2.  Wavefronts 0 and 1 solve the odd lines i-1 and i+1 (line i+1 is
// solved again, identically, by block b+1), then wavefront 0 solves line i
// from them.  Block b owns lines i-1 and i, the last block also line nz-2.
// FP64: phi_in (old values, plus the injected coarse correction on the even
// rows) to phi_out.  Mixed: the correction from zero with the FP32 residual as
// right-hand side, added to phi in place (phi_in == phi_out).
template <typename T, int Q>
struct k_fine_A {
    MgLevels m;
    int mixed;
    const double *phi_in;
    double *phi_out;
    const double *f;
};

template <typename T, int Q>
__device__ __forceinline__ void k_fine_body(const Blk &kb_, const k_fine_A<T, Q> &A_)
{
    const auto &m = A_.m;
    auto mixed = A_.mixed;
    auto phi_in = A_.phi_in;
    auto phi_out = A_.phi_out;
    auto f = A_.f;

    constexpr int SMAX = Q == 1 ? 6 : Q == 2 ? 7 : 8;
    __shared__ T xs[2][Q * 64];
    const int L = m.L, nr = m.nr, n = nr - 1, nz = m.nzl[L], S = m.S;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int i = 2 * kb_.x + 2;
    const bool last = i + 1 == nz - 2;
    const T *uc = mixed ? (const T *)m.u32[L - 1] : (const T *)m.u64[L - 1];
    const T *fr = (const T *)m.f32[L];  // mixed: FP32 residual
    const T *tab0 = (const T *)m.tab + (size_t)(m.line_off[L] - 1) * m.tab_stride;
    // wavefront 0 also fetches the even line's table, phi and right-hand side
    // while it reduces its odd line, so that the even line starts right after
    // the barrier
    LineTab<T, Q, SMAX> te;
    double ph2[Q];
    T g2[Q];
    {
        const int io = i - 1 + 2 * w;
        LineTab<T, Q, SMAX> tb;
        line_tab_load<T, Q, SMAX>(tab0 + (size_t)io * m.tab_stride, n, m.tab_row, S, lane, tb);
        T R[Q];
        double ph[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j = q * 64 + lane;
            const bool ok = j < n;
            const int jj = ok ? j : n - 1;
            const T cl = uc[(size_t)((io - 1) >> 1) * nr + jj];
            const T ch = uc[(size_t)((io + 1) >> 1) * nr + jj];
            const T cl_ = io - 1 > 0 ? cl : (T)0;
            const T ch_ = io + 1 < nz - 1 ? ch : (T)0;
            const double pl = phi_in[(size_t)(io - 1) * nr + jj];
            const double phh = phi_in[(size_t)(io + 1) * nr + jj];
            ph[q] = phi_in[(size_t)io * nr + jj];
            T lo, hi, g;
            if (mixed) {
                lo = cl_;
                hi = ch_;
                g = fr[(size_t)io * nr + jj];
            } else {
                lo = (T)(pl + (double)cl_);
                hi = (T)(phh + (double)ch_);
                g = (T)f[(size_t)io * nr + jj];
            }
            R[q] = ok ? g + tb.ta[q] * lo + tb.tc[q] * hi : (T)0;
        }
        if (w == 0) {
            line_tab_fetch<T, Q, SMAX>(tab0 + (size_t)i * m.tab_stride, n, m.tab_row, S, lane, te);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int j = q * 64 + lane;
                const int jj = j < n ? j : n - 1;
                ph2[q] = phi_in[(size_t)i * nr + jj];
                g2[q] = mixed ? fr[(size_t)i * nr + jj] : (T)f[(size_t)i * nr + jj];
            }
        }
        line_pcr<T, Q, SMAX>(R, tb, S, lane);
        const bool own = w == 0 || last;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j = q * 64 + lane;
            if (j >= n) continue;
            xs[w][j] = R[q];
            if (own) phi_out[(size_t)io * nr + j] = mixed ? ph[q] + (double)R[q] : (double)R[q];
        }
    }
    __syncthreads();
    if (w == 0) {
        line_tab_mask<T, Q, SMAX>(n, S, lane, te);
        T R[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j = q * 64 + lane;
            const bool ok = j < n;
            const int jj = ok ? j : n - 1;
            R[q] = ok ? g2[q] + te.ta[q] * xs[0][jj] + te.tc[q] * xs[1][jj] : (T)0;
        }
        line_pcr<T, Q, SMAX>(R, te, S, lane);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j = q * 64 + lane;
            if (j >= n) continue;
            phi_out[(size_t)i * nr + j] = mixed ? ph2[q] + (double)R[q] : (double)R[q];
        }
    }
}


template <typename T>
static hipError_t fine_sweep(const MgLevels &m, int mixed, const double *phi_in, double *phi_out,
                             const double *f, hipStream_t st)
{
    const int n = m.nr - 1, blocks = (m.nzl[m.L] - 3) / 2;
    if (blocks <= 0) return hipSuccess;
    if (n <= 64)
        (void)launch<k_fine_A<T, 1>, k_fine_body<T, 1>, 128>(dim3(blocks), dim3(128), 0, st, k_fine_A<T, 1>{m, mixed, phi_in, phi_out, f});
    else if (n <= 128)
        (void)launch<k_fine_A<T, 2>, k_fine_body<T, 2>, 128>(dim3(blocks), dim3(128), 0, st, k_fine_A<T, 2>{m, mixed, phi_in, phi_out, f});
    else
        (void)launch<k_fine_A<T, 4>, k_fine_body<T, 4>, 128>(dim3(blocks), dim3(128), 0, st, k_fine_A<T, 4>{m, mixed, phi_in, phi_out, f});
    return hipGetLastError();
}

// Up leg of the split cycle in one launch (Algorithm 1's way up: exact
// coarsest line, then per level the injected correction and one zebra sweep).
// Block b owns the finest level's even line i = 2b+2 and odd line i-1 (the
// last block also i+1), as in k_fine.  Before its finest lines it solves,
// level by level from the coarsest, every coarser line they depend on: an
// odd line of level l needs rows (r-1)/2 and (r+1)/2 of level l-1, an even
// line the odd lines beside it.  Those lines form a window of at most five
// consecutive lines per level (three odd, two even), so each block repeats a
// few lines of every coarse level that its neighbours also solve, with the
// same tables and arithmetic and therefore the same values.  The coarse
// levels then cost 31 compute units a few line tables each, instead of one
// compute unit all of them, and the cycle needs no separate coarse launch.
// A line's inputs (table, right-hand side, phi) are fetched three phases
// before it is solved (FP64 and four unknowns per lane: two): data that other
// compute units wrote takes longer to arrive than two phases last.
constexpr int kUpWin = 5;         // lines of one level's window
constexpr int kUpThreads = 192;   // three wavefronts: a phase has at most three lines

template <typename T, int Q> struct k_up_A {
    MgLevels m;
    int mixed;
    const double *phi_in;
    double *phi_out;
    const double *f;
};

template <typename T, int Q, int SMAX> struct UpIn {
    LineTab<T, Q, SMAX> tab;
    T g[Q];                // right-hand side
    double pl[Q], ph[Q];   // finest level, FP64: phi_in of rows r-1 and r+1
    double pc[Q];          // finest level, mixed: phi of row r
};

static size_t up_lds(const MgLevels &m, int mixed)
{
    return (size_t)(m.L + 1) * kUpWin * m.nr * (mixed ? sizeof(float) : sizeof(double));
}

// A 64-bit address the whole wavefront shares, kept in scalar registers (so
// that a load adds a 32-bit lane offset to it, with no per-lane address
// arithmetic).
template <typename P> __device__ __forceinline__ P *uniform_ptr(P *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P *)(((uint64_t)hi << 32) | lo);
}

template <typename T> __device__ __forceinline__ T ld_off(const T *base, uint32_t off)
{
    typedef const __attribute__((address_space(1))) char gchar;
    typedef const __attribute__((address_space(1))) T gT;
    return *(gT *)((gchar *)base + off);
}

// Q consecutive elements at a 32-bit byte offset from a wavefront-uniform
// base, in one load (base + off aligned to Q elements).
template <typename T, int Q>
__device__ __forceinline__ void ld_vec(const T *base, uint32_t off, T (&dst)[Q])
{
    if constexpr (Q == 1) {
        dst[0] = ld_off(base, off);
    } else {
        typedef T V __attribute__((ext_vector_type(Q)));
        typedef const __attribute__((address_space(1))) char gchar;
        typedef const __attribute__((address_space(1))) V gV;
        const V v = *(gV *)((gchar *)base + off);
#pragma unroll
        for (int q = 0; q < Q; ++q) dst[q] = v[q];
    }
}

// Q consecutive elements at a byte offset from a wavefront-uniform base that
// is aligned to one element only (rows of nr elements), in one load.
template <typename T, int Q>
__device__ __forceinline__ void ld_vec_u(const T *base, uint32_t off, T (&dst)[Q])
{
    typedef T V __attribute__((ext_vector_type(Q), aligned(sizeof(T))));
    typedef const __attribute__((address_space(1))) char gchar;
    typedef const __attribute__((address_space(1))) V gV;
    const V v = *(gV *)((gchar *)base + off);
#pragma unroll
    for (int q = 0; q < Q; ++q) dst[q] = v[q];
}

// line_pcr for lanes that hold Q consecutive unknowns (j = Q lane + q): the
// same reduction steps, term for term, with the neighbours at distance
// s < Q in the lane itself or the next lane, and those at s >= Q a lane
// shuffle of s / Q away.
template <typename T, int Q, int SMAX>
__device__ __forceinline__ void line_pcr_adj(T (&R)[Q], const LineTab<T, Q, SMAX> &t, int S,
                                             int lane)
{
#pragma unroll
    for (int st = 0; st < SMAX; ++st) {
        if (st >= S) break;
        const int s = 1 << st;
        T nR[Q];
        if (s < Q) {
            T fl[Q], fr[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                // lane - 1 holds unknown j - s for q < s, lane + 1 unknown j + s for q >= Q - s
                fl[q] = q < s ? __shfl(R[q < s ? q - s + Q : 0], (lane - 1) & 63, 64) : (T)0;
                fr[q] = q >= Q - s ? __shfl(R[q >= Q - s ? q + s - Q : 0], (lane + 1) & 63, 64) : (T)0;
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const T left = q >= s ? R[q >= s ? q - s : 0] : (lane >= 1 ? fl[q] : (T)0);
                const T right = q + s < Q ? R[q + s < Q ? q + s : 0] : (lane < 63 ? fr[q] : (T)0);
                nR[q] = R[q] - left * t.k1[st][q] - right * t.k2[st][q];
            }
        } else {
            const int d = s / Q;
            T dn[Q], up[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                dn[q] = __shfl(R[q], (lane - d) & 63, 64);
                up[q] = __shfl(R[q], (lane + d) & 63, 64);
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const T left = lane >= d ? dn[q] : (T)0;
                const T right = lane + d < 64 ? up[q] : (T)0;
                nR[q] = R[q] - left * t.k1[st][q] - right * t.k2[st][q];
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) R[q] = nR[q];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) R[q] = R[q] / t.bf[q];
}

// The levels of a mesh with nz = 2^L + 1 rows have nz_l = 2^l + 1 rows; the
// line tables of level l start at line 2^l - l - 1 (levels 1..l-1 hold
// nz_q - 2 interior lines each), and the coarse block (u then f of each level)
// holds level l's u at row 2 (2^l + l - 3) and its f nz_l rows later.
__device__ __forceinline__ int up_nzl(int l) { return (1 << l) + 1; }
__device__ __forceinline__ int up_line_off(int l) { return (1 << l) - l - 1; }
__device__ __forceinline__ size_t up_f_row(int l) { return 2 * (size_t)((1 << l) + l - 3) + up_nzl(l); }

template <typename T, int Q>
__device__ __forceinline__ void k_up_body(const Blk &kb_, const k_up_A<T, Q> &A_)
{
    const MgLevels &m = A_.m;
    constexpr bool mixed = sizeof(T) == 4;  // FP32 tables are the mixed form's
    const double *phi_in = A_.phi_in;
    double *phi_out = A_.phi_out;
    const double *f = A_.f;
    constexpr int SMAX = Q == 1 ? 6 : Q == 2 ? 7 : 8;
    extern __shared__ unsigned char smem_raw[];
    T *win = (T *)smem_raw;  // [level][kUpWin][nr]: the window's solutions
    const int L = m.L, nr = m.nr, n = nr - 1, nz = up_nzl(L), S = m.S;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nph = 2 * L - 1;
    if (wave >= kUpThreads / 64) {
        // the spare wavefronts of a wider launch (k_up_app_body): the phases'
        // barriers only
        for (int ph = 0; ph < nph; ++ph) __syncthreads();
        return;
    }
    const int i = 2 * kb_.x + 2;
    const bool last = i + 1 == nz - 2;
    // The window of level l, k = L - l levels below the finest: the rows its
    // level above reads are [p, q] with p = max(floor(i / 2^k) - 1, 0) and
    // q = floor((i + 2^k - 1) / 2^k) + 1, its lines [p, q] widened to odd ends
    // and kept inside the interior (the closed form of narrowing [i-1, i+1]
    // level by level: each odd line reads the rows (r-1)/2, (r+1)/2 below it).
    auto wlo = [&](int l) {
        const int k = L - l, p = (i >> k) - 1 > 0 ? (i >> k) - 1 : 0;
        const int a = (p - 1) | 1;
        return a > 1 ? a : 1;
    };
    auto whi = [&](int l) {
        const int k = L - l, b = (((i + (1 << k) - 1) >> k) + 1) | 1;
        return b < (1 << l) - 1 ? b : (1 << l) - 1;
    };
    auto W = [&](int l, int r) {  // row r of level l in the window (clamped into it)
        int k = r - wlo(l);
        k = k < 0 ? 0 : k >= kUpWin ? kUpWin - 1 : k;
        return win + ((size_t)l * kUpWin + k) * nr;
    };
    auto cnt_of = [&](int l, int par) {
        const int d = whi(l) - wlo(l);
        return par ? d / 2 + 1 : d / 2;
    };
    // Level l's odd lines, then its even lines, level by level from l = 1:
    // step k = 0 .. 2L-1 is level k/2 + 1, odd lines (even k) or even lines.
    // Level 1 has no even line, so the phases are the steps but that one
    // (phase ph is step ph + (ph > 0)).  A phase has at most three lines and
    // the block three wavefronts, so wavefront w solves line w of each phase
    // that has one.
    const T *coarse = (const T *)m.coarse_uf;
    const T *fr = mixed ? (const T *)m.f32[L] : nullptr;  // mixed: FP32 residual
    const T *tab = (const T *)m.tab;
    const size_t tstride = m.tab_stride;
    // The inputs of this wavefront's line of phase ph: its table rows
    // (pairs a, c | b_final | pairs k1, k2 of each step, see factor_body),
    // right-hand side and phi.  A lane holds the Q consecutive unknowns
    // j = Q lane + q, so that a pair row comes in one load of 2Q elements
    // and b_final in one of Q (the rows are padded to whole groups; a lane
    // past the row's end takes its last group), and with Q = 2 the
    // right-hand side and phi one load per row: 11 loads per phase of the
    // mixed form, and the wavefront's loads of three phases ahead fit the
    // 63 it can have in flight (five buffers, four ahead, measured slower:
    // the extra registers cost more than the deeper overlap gains).  Every
    // wavefront fetches in every phase (a wavefront without a line there,
    // or a phase past the last, takes another line of the block), so that
    // the loads in flight are the same on every path.  The byte offsets of
    // the lane's group in each row, from the start of a line's table, are
    // the same for every line: computed once, they leave a load one scalar
    // base per line and no address arithmetic per row.
    const int tn = m.tab_row;
    const int e0 = Q * lane + Q <= tn ? Q * lane : tn - Q;
    const uint32_t ot = (uint32_t)e0 * (uint32_t)sizeof(T);
    const uint32_t rowb = (uint32_t)tn * (uint32_t)sizeof(T);
    const uint32_t o_bf = 2 * rowb + ot;
    uint32_t o_pair[SMAX + 1];
    o_pair[0] = 2 * ot;
    // scalar bases of the right-hand side and phi rows: a row is a 32-bit
    // byte offset added to the lane's
    const T *coarse_b = uniform_ptr(coarse), *fr_b = uniform_ptr(fr), *tab_b = uniform_ptr(tab);
    const uint32_t tstride_b = (uint32_t)(tstride * sizeof(T));
    const double *phi_b = uniform_ptr(phi_in), *f_b = uniform_ptr(f);
#pragma unroll
    for (int st = 0; st < SMAX; ++st) {
        const int sc = st < S ? st : S - 1;
        o_pair[1 + st] = (uint32_t)tab_pair_row(1 + sc) * rowb + 2 * ot;
    }
    auto fetch = [&](int ph, UpIn<T, Q, SMAX> &in) {
        const int k = ph + (ph > 0);
        int l = k / 2 + 1, par = !(k & 1), t = wave;
        if (ph >= nph) {
            l = 1;
            par = 1;
            t = 0;
        } else {
            const int c = cnt_of(l, par);
            if (t >= c) {
                if (c > 0) {
                    t = c - 1;
                } else {
                    par = 1;  // level 1 has no even line
                    t = 0;
                }
            }
        }
        const int r = (par ? wlo(l) : wlo(l) + 1) + 2 * t;
        const bool fine = l == L;
        // the line's table: a 32-bit byte offset from the tables' scalar base
        const T *tb = (const T *)((const char *)tab_b +
                                  (uint32_t)(up_line_off(l) + r - 1) * tstride_b);
        const T *fl = coarse + (up_f_row(l) + r) * nr;
        T pr[2 * Q];
        ld_vec<T, 2 * Q>(tb, o_pair[0], pr);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            in.tab.ta[q] = pr[2 * q];
            in.tab.tc[q] = pr[2 * q + 1];
        }
        ld_vec<T, Q>(tb, o_bf, in.tab.bf);
#pragma unroll
        for (int st = 0; st < SMAX; ++st) {
            ld_vec<T, 2 * Q>(tb, o_pair[1 + st], pr);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                in.tab.k1[st][q] = pr[2 * q];
                in.tab.k2[st][q] = pr[2 * q + 1];
            }
        }
        if constexpr (Q == 2) {
            // one load of the lane's two unknowns per row: the pair starts at
            // j = 2 lane and ends at most at column n, the row's last; lanes
            // past the line's end (masked where used) take the row's last pair
            const int g0 = 2 * lane + 1 <= n ? 2 * lane : n - 1;
            const uint32_t og = (uint32_t)g0 * (uint32_t)sizeof(T);
            const uint32_t od = (uint32_t)g0 * (uint32_t)sizeof(double);
            double z[2];
            in.pl[0] = in.pl[1] = in.ph[0] = in.ph[1] = in.pc[0] = in.pc[1] = 0.0;
            const uint32_t row = (uint32_t)r * (uint32_t)nr;
            if (!fine) {
                const uint32_t cr = (uint32_t)(up_f_row(l) + r) * (uint32_t)nr;
                ld_vec_u<T, 2>(coarse_b, og + cr * (uint32_t)sizeof(T), in.g);
            } else if (mixed) {
                ld_vec_u<T, 2>(fr_b, og + row * (uint32_t)sizeof(T), in.g);
                ld_vec_u<double, 2>(phi_b, od + row * 8u, in.pc);
            } else {
                ld_vec_u<double, 2>(f_b, od + row * 8u, z);
                in.g[0] = (T)z[0];
                in.g[1] = (T)z[1];
                ld_vec_u<double, 2>(phi_b, od + (row - (uint32_t)nr) * 8u, in.pl);
                ld_vec_u<double, 2>(phi_b, od + (row + (uint32_t)nr) * 8u, in.ph);
            }
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int j = Q * lane + q;
                const int jj = j < n ? j : n - 1;
                const uint32_t og = (uint32_t)jj * (uint32_t)sizeof(T);
                const uint32_t od = (uint32_t)jj * (uint32_t)sizeof(double);
                in.pl[q] = in.ph[q] = in.pc[q] = 0.0;
                if (!fine) {
                    in.g[q] = ld_off(uniform_ptr(fl), og);
                } else if (mixed) {
                    in.g[q] = ld_off(uniform_ptr(fr + (size_t)r * nr), og);
                    in.pc[q] = ld_off(uniform_ptr(phi_in + (size_t)r * nr), od);
                } else {
                    in.g[q] = (T)ld_off(uniform_ptr(f + (size_t)r * nr), od);
                    in.pl[q] = ld_off(uniform_ptr(phi_in + (size_t)(r - 1) * nr), od);
                    in.ph[q] = ld_off(uniform_ptr(phi_in + (size_t)(r + 1) * nr), od);
                }
            }
        }
    };
    // The line of phase ph, if this wavefront has one, then the barrier.
    // The table needs no masking: reduction steps past S are not run, and the
    // unknowns past the line's end (holding the padding or the row's last
    // group, all finite) meet only multipliers that are zero in the table of
    // every unknown.
    auto run = [&](int ph, const UpIn<T, Q, SMAX> &in) {
        const int k = ph + (ph > 0);
        const int l = k / 2 + 1, par = !(k & 1), nzl = up_nzl(l);
        const bool fine = l == L;
        if (wave < cnt_of(l, par)) {
            const int r = (par ? wlo(l) : wlo(l) + 1) + 2 * wave;
            const int lb = par ? (l > 1 ? l - 1 : 1) : l;
            const T *ulo = W(lb, par ? (r - 1) >> 1 : r - 1);
            const T *uhi = W(lb, par ? (r + 1) >> 1 : r + 1);
            const bool inj = par && l > 1;
            T R[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int j = Q * lane + q;
                const bool ok = j < n;
                const int jj = ok ? j : n - 1;
                const T a = ulo[jj], b = uhi[jj];
                T lo, hi;
                if (par) {
                    // odd line: the coarse correction injected into the even
                    // rows r-1, r+1 (zero on the electrodes)
                    const T cl = inj && r - 1 > 0 ? a : (T)0;
                    const T ch = inj && r + 1 < nzl - 1 ? b : (T)0;
                    if (fine && !mixed) {
                        lo = (T)(in.pl[q] + (double)cl);
                        hi = (T)(in.ph[q] + (double)ch);
                    } else {
                        lo = cl;
                        hi = ch;
                    }
                } else {
                    lo = a;
                    hi = b;
                }
                R[q] = ok ? in.g[q] + in.tab.ta[q] * lo + in.tab.tc[q] * hi : (T)0;
            }
            line_pcr_adj<T, Q, SMAX>(R, in.tab, S, lane);
            T *ur = W(l, r);
            const bool own = fine && (r == i - 1 || r == i || (last && r == i + 1));
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int j = Q * lane + q;
                if (j >= n) continue;
                ur[j] = R[q];
                if (own)
                    phi_out[(size_t)r * nr + j] = mixed ? in.pc[q] + (double)R[q] : (double)R[q];
            }
        }
        __syncthreads();
    };
    // Buffers in fixed roles: phase ph reads buffer ph mod 4 while the
    // inputs of phases ph + 1 .. ph + 3 are on their way (a phase is shorter
    // than a load from memory written by other compute units); where four
    // buffers would not fit the registers (FP64, or four unknowns per lane),
    // three, two phases ahead.
    UpIn<T, Q, SMAX> b0, b1, b2;
    fetch(0, b0);
    fetch(1, b1);
    if constexpr (Q * sizeof(T) <= 8) {
        UpIn<T, Q, SMAX> b3;
        fetch(2, b2);
        for (int ph = 0; ph < nph; ph += 4) {
            fetch(ph + 3, b3);
            run(ph, b0);
            if (ph + 1 >= nph) break;
            fetch(ph + 4, b0);
            run(ph + 1, b1);
            if (ph + 2 >= nph) break;
            fetch(ph + 5, b1);
            run(ph + 2, b2);
            if (ph + 3 >= nph) break;
            fetch(ph + 6, b2);
            run(ph + 3, b3);
        }
    } else {
        for (int ph = 0; ph < nph; ph += 3) {
            fetch(ph + 2, b2);
            run(ph, b0);
            if (ph + 1 >= nph) break;
            fetch(ph + 3, b0);
            run(ph + 1, b1);
            if (ph + 2 >= nph) break;
            fetch(ph + 4, b1);
            run(ph + 2, b2);
        }
    }
}

// The way up beside the appending of a pending list tail (step
// pipelining), at kSuper threads: the way-up blocks first (their spare
// wavefronts take the barriers only), then the appending's.  Only where the
// way up's registers fit two wavefronts of the block per SIMD.
template <typename T, int Q> struct k_up_app_A {
    k_up_A<T, Q> u;
    AppendJob<T> a;
    int nu, nsc;
};

template <typename T, int Q>
__device__ __forceinline__ void k_up_app_body(const Blk &kb_, const k_up_app_A<T, Q> &A_)
{
    if (kb_.x < A_.nu) {
        k_up_body<T, Q>(Blk{kb_.x, 0, A_.nu, 1}, A_.u);
        return;
    }
    const int b = kb_.x - A_.nu;
    append_body<T>(Blk{b % A_.nsc, b / A_.nsc, A_.nsc, 2}, A_.a);
}

template <typename T, int Q>
static hipError_t up_app(const k_up_A<T, Q> &u, int blocks, size_t lds, ListTail &t,
                         hipStream_t st)
{
    static_assert(sizeof(k_up_app_A<T, Q>) <= 4096, "kernel arguments");
    k_up_app_A<T, Q> a{u, {}, blocks, t.nsc};
    std::memcpy(&a.a, t.app, sizeof a.a);
    (void)launch<k_up_app_A<T, Q>, k_up_app_body<T, Q>, kSuper>(
        dim3(blocks + 2 * t.nsc), dim3(kSuper), lds, st, a);
    t.stage = 0;
    return hipGetLastError();
}

template <typename T>
static hipError_t up_sweep(const MgLevels &m, int mixed, const double *phi_in, double *phi_out,
                           const double *f, hipStream_t st, ListTail *tail = nullptr)
{
    const int n = m.nr - 1, blocks = (m.nzl[m.L] - 3) / 2;
    if (blocks <= 0) return hipSuccess;
    if ((mixed != 0) != (sizeof(T) == 4)) return hipErrorInvalidValue;  // k_up_body's form
    const size_t lds = up_lds(m, mixed);
    if (tail && tail->stage == 1 && (tail->fp32 != 0) == (mixed != 0)) {
        if (n <= 64) return up_app<T, 1>(k_up_A<T, 1>{m, mixed, phi_in, phi_out, f}, blocks, lds,
                                         *tail, st);
        if constexpr (sizeof(T) == 4)
            if (n <= 128)
                return up_app<T, 2>(k_up_A<T, 2>{m, mixed, phi_in, phi_out, f}, blocks, lds,
                                    *tail, st);
    }
    if (n <= 64)
        (void)launch<k_up_A<T, 1>, k_up_body<T, 1>, kUpThreads>(dim3(blocks), dim3(kUpThreads), lds, st, k_up_A<T, 1>{m, mixed, phi_in, phi_out, f});
    else if (n <= 128)
        (void)launch<k_up_A<T, 2>, k_up_body<T, 2>, kUpThreads>(dim3(blocks), dim3(kUpThreads), lds, st, k_up_A<T, 2>{m, mixed, phi_in, phi_out, f});
    else if constexpr (sizeof(T) == 4)  // the FP64 split cycle takes lines of up to 128 unknowns
        (void)launch<k_up_A<T, 4>, k_up_body<T, 4>, kUpThreads>(dim3(blocks), dim3(kUpThreads), lds, st, k_up_A<T, 4>{m, mixed, phi_in, phi_out, f});
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t mg_solve_block(const MgLevels &m, int mixed, double *phi, const double *f, double V,
                          int cycles, hipStream_t st)
{
    return solve_block(m, mixed, phi, f, V, cycles, 0, st);
}

void mg_plan(MgLevels &m, int mixed, size_t lds_budget, int path)
{
    const size_t es = mixed ? sizeof(float) : sizeof(double);
    const int n = m.nr - 1;
    m.lds_budget = lds_budget;
    // the level kernel holds three lines of four arrays (12 n values) in LDS
    // and reduces 2 n values with at most four per thread
    // 2: the long-line path forced, every line by the partition method
    m.long_lines = path == 3 ? 2 : 12 * (size_t)n * es > lds_budget || 2 * n > 4 * 1024;
    // single-block path
    int S = 0;
    while ((1 << S) < n) ++S;
    m.S = S;
    int off = 0;
    for (int l = 1; l <= m.L; ++l) {
        m.line_off[l] = off;
        off += m.nzl[l] - 2;
    }
    m.line_off[m.L + 1] = off;
    m.tab_row = (n + 7) & ~7;  // pair rows of 8-aligned groups: aligned vector loads
    m.tab_stride = (size_t)(3 + 2 * S) * m.tab_row;
    size_t lds = 0;
    for (int l = 1; l <= (mixed ? m.L : m.L - 1); ++l) lds += 2 * (size_t)m.nzl[l] * m.nr * es;
    m.solve_lds = lds;
    const bool fits = n <= (mixed ? 256 : 128) && lds <= lds_budget && !m.long_lines;
    // the one-launch way up computes level sizes and table offsets in closed
    // form (nz_l = 2^l + 1, first line 2^l - l - 1)
    bool closed = true;
    for (int l = 1; l <= m.L; ++l)
        closed = closed && m.nzl[l] == (1 << l) + 1 && m.line_off[l] == (1 << l) - l - 1;
    m.split = fits && path == 0 && m.L > 1 && up_lds(m, mixed) <= lds_budget && closed;
    m.one_block = fits && (path == 1 || (path == 0 && m.L == 1));
    // multi-launch path: levels of the bottom kernel
    m.K = 0;
    m.bottom_lds = 0;
    size_t lev = 0;
    for (int K = 1; K <= m.L - 1; ++K) {
        lev += 3 * (size_t)m.nzl[K] * m.nr * es;
        const size_t emax = (size_t)((m.nzl[K] - 1) / 2) * n;
        const size_t bytes = lev + 4 * emax * es;
        if (bytes > lds_budget || emax > 4 * 1024) break;
        m.K = K;
        m.bottom_lds = bytes;
    }
}

template <typename T>
static hipError_t bottom(const MgLevels &m, int mixed, hipStream_t st)
{
    const int n = m.nr - 1;
    const int emax = ((m.nzl[m.K] - 1) / 2) * n;
    const int ept = (emax + 1023) / 1024;
    if (ept <= 1)
        (void)launch<k_bottom_A<T, 1>, k_bottom_body<T, 1>, 1024>(dim3(1), dim3(1024), m.bottom_lds, st, k_bottom_A<T, 1>{m, mixed});
    else if (ept <= 2)
        (void)launch<k_bottom_A<T, 2>, k_bottom_body<T, 2>, 1024>(dim3(1), dim3(1024), m.bottom_lds, st, k_bottom_A<T, 2>{m, mixed});
    else
        (void)launch<k_bottom_A<T, 4>, k_bottom_body<T, 4>, 1024>(dim3(1), dim3(1024), m.bottom_lds, st, k_bottom_A<T, 4>{m, mixed});
    return hipGetLastError();
}

// One V(0,1) cycle on phi.  FP64: every level in double, the finest level on
// phi itself.  Mixed: the finest residual in double, the correction cycle in
// float on every level, phi += correction in double.
// The way down beside the next stage of a pending list tail (step
// pipelining), at kSuper threads: the way-down blocks first, then the hole
// filling's (fill_blocks per species) or the appending's blocks.  down_body
// and the list bodies loop over the block's threads.
constexpr int kTailFillBlocks = 128;

template <typename T> struct k_down_fill_A {
    k_down_A<T> d;
    Fill2Args<T> f;
    int nd;
};

template <typename T>
__device__ __forceinline__ void k_down_fill_body(const Blk &kb_, const k_down_fill_A<T> &A_)
{
    if (kb_.x < A_.nd) {
        k_down_body<T>(Blk{kb_.x, 0, A_.nd, 1}, A_.d);
        return;
    }
    const int b = kb_.x - A_.nd;
    fill2_body<T>(Blk{b % kTailFillBlocks, b / kTailFillBlocks, kTailFillBlocks, 2}, A_.f);
}

template <typename T> struct k_down_app_A {
    k_down_A<T> d;
    AppendJob<T> a;
    int nd, nsc;
};

template <typename T>
__device__ __forceinline__ void k_down_app_body(const Blk &kb_, const k_down_app_A<T> &A_)
{
    if (kb_.x < A_.nd) {
        k_down_body<T>(Blk{kb_.x, 0, A_.nd, 1}, A_.d);
        return;
    }
    const int b = kb_.x - A_.nd;
    append_body<T>(Blk{b % A_.nsc, b / A_.nsc, A_.nsc, 2}, A_.a);
}

template <typename T>
static hipError_t down_tail(const MgLevels &m, int mixed, const double *phi, const double *f,
                            int cpb, ListTail &t, hipStream_t st)
{
    const int nr = m.nr, nz = m.nzl[m.L], nd = (nr - 1 + cpb - 1) / cpb;
    const k_down_A<T> d{phi, f, m, mixed, cpb};
    if (t.stage == 2) {
        static_assert(sizeof(k_down_fill_A<T>) <= 4096, "kernel arguments");
        k_down_fill_A<T> a{d, {}, nd};
        std::memcpy(&a.f, t.fill, sizeof a.f);
        (void)launch<k_down_fill_A<T>, k_down_fill_body<T>, kSuper>(
            dim3(nd + 2 * kTailFillBlocks), dim3(kSuper), down_lds(nz, cpb), st, a);
        t.stage = 1;
    } else {
        static_assert(sizeof(k_down_app_A<T>) <= 4096, "kernel arguments");
        k_down_app_A<T> a{d, {}, nd, t.nsc};
        std::memcpy(&a.a, t.app, sizeof a.a);
        (void)launch<k_down_app_A<T>, k_down_app_body<T>, kSuper>(
            dim3(nd + 2 * t.nsc), dim3(kSuper), down_lds(nz, cpb), st, a);
        t.stage = 0;
    }
    return hipGetLastError();
}

static hipError_t down(const MgLevels &m, int mixed, const double *phi, const double *f,
                       hipStream_t st, ListTail *tail = nullptr)
{
    if (m.long_lines) return down_rows(m, mixed, phi, f, st);
    const int nr = m.nr, nz = m.nzl[m.L];
    const int cpb = cols_per_block(nz);
    if (tail && tail->stage > 0 && (tail->fp32 != 0) == (mixed != 0)) {
        if (mixed) return down_tail<float>(m, mixed, phi, f, cpb, *tail, st);
        return down_tail<double>(m, mixed, phi, f, cpb, *tail, st);
    }
    if (mixed)
        (void)launch<k_down_A<float>, k_down_body<float>, 256>(dim3((nr - 1 + cpb - 1) / cpb), dim3(256), down_lds(nz, cpb), st, k_down_A<float>{phi, f, m, mixed, cpb});
    else
        (void)launch<k_down_A<double>, k_down_body<double>, 256>(dim3((nr - 1 + cpb - 1) / cpb), dim3(256), down_lds(nz, cpb), st, k_down_A<double>{phi, f, m, mixed, cpb});
    return hipGetLastError();
}

hipError_t mg_vcycle(const MgLevels &m, int mixed, double *&phi, double *&phi_alt,
                     const double *f, int skip_down, hipStream_t st, ListTail *tail)
{
    const int L = m.L, nr = m.nr, nz = m.nzl[L];
    hipError_t e;
    if (L == 1) {
        // a single interior line: the cycle is its exact solve
        if (!mixed) return line<double>(m, 1, 1, 0, phi, f, m.eps64[1], nullptr, st);
        int cpb = cols_per_block(nz);
        size_t lds = (2 * (size_t)(cpb + 2) + 2 * (size_t)cpb) * nz * sizeof(double);
        (void)launch<k_down_A<float>, k_down_body<float>, 256>(dim3((nr - 1 + cpb - 1) / cpb), dim3(256), lds, st, k_down_A<float>{(const double *)phi, f, m, mixed, cpb});
        if ((e = line<float>(m, 1, 1, 1, m.u32[1], m.f32[1], m.eps32[1], nullptr, st))) return e;
        const int nn = nr * nz, threads = 256, blocks = (nn + threads - 1) / threads;
        (void)launch<k_add_corr_A, k_add_corr_body, 256>(dim3(blocks), dim3(threads), 0, st, k_add_corr_A{phi, (const float *)m.u32[1], nr, nz});
        return hipGetLastError();
    }
    // the residual of the finest level restricted to every level (unless the
    // solve's first launch has done it for this cycle)
    if (!skip_down &&
        (e = down(m, mixed, phi, f, st, m.split ? tail : nullptr)) != hipSuccess)
        return e;
    if (m.split) {
        // the way up in one launch: each block of the finest level's sweep
        // with the coarse lines it depends on (up_sweep); or (split_coarse)
        // the coarse levels in one workgroup, then the finest level's sweep
        if (!m.split_coarse) {
            if (mixed) return up_sweep<float>(m, mixed, phi, phi, f, st, tail);
            e = up_sweep<double>(m, mixed, phi, phi_alt, f, st, tail);
            double *t = phi;
            phi = phi_alt;
            phi_alt = t;
            return e;
        }
        if ((e = solve_block(m, mixed, phi, f, 0.0, 1, 1, st)) != hipSuccess) return e;
        if (mixed) return fine_sweep<float>(m, mixed, phi, phi, f, st);
        e = fine_sweep<double>(m, mixed, phi, phi_alt, f, st);
        double *t = phi;
        phi = phi_alt;
        phi_alt = t;
        return e;
    }
    if (m.long_lines) {
        // r-lines longer than the level kernel's LDS: every level as two
        // half-sweeps of line solves (odd lines with the injected coarse
        // correction, then even lines), in place
        for (int l = 1; l <= L; ++l) {
            const bool fine = l == L;
            if (mixed) {
                float *u = m.u32[l];
                const float *uc = l > 1 ? m.u32[l - 1] : nullptr;
                // finest level: phi += correction as each line is solved (the
                // odd lines are final once their half-sweep is done)
                double *add = fine ? phi : nullptr;
                if ((e = line<float>(m, l, 1, 1, u, m.f32[l], m.eps32[l], uc, st, add))) return e;
                if ((e = line<float>(m, l, 0, 0, u, m.f32[l], m.eps32[l], nullptr, st, add))) return e;
            } else {
                double *u = fine ? phi : m.u64[l];
                const double *fl = fine ? f : m.f64[l];
                const double *uc = l > 1 ? m.u64[l - 1] : nullptr;
                if ((e = line<double>(m, l, 1, fine ? 0 : 1, u, fl, m.eps64[l], uc, st))) return e;
                if ((e = line<double>(m, l, 0, 0, u, fl, m.eps64[l], nullptr, st))) return e;
            }
        }
        return hipSuccess;
    }
    int done = m.K;
    if (m.K >= 1) {
        e = mixed ? bottom<float>(m, mixed, st) : bottom<double>(m, mixed, st);
        if (e != hipSuccess) return e;
    } else {
        e = mixed ? line<float>(m, 1, 1, 1, m.u32[1], m.f32[1], m.eps32[1], nullptr, st)
                  : line<double>(m, 1, 1, 1, m.u64[1], m.f64[1], m.eps64[1], nullptr, st);
        if (e != hipSuccess) return e;
        done = 1;
    }
    for (int l = done + 1; l <= L; ++l) {
        const bool fine = l == L;
        if (mixed) {
            e = level_sweep<float>(m, l, 1, nullptr, m.u32[l - 1], fine ? nullptr : m.u32[l],
                                   m.f32[l], m.eps32[l], fine ? phi : nullptr, st);
        } else if (fine) {
            e = level_sweep<double>(m, l, 0, phi, m.u64[l - 1], phi_alt, f, m.eps64[l], nullptr,
                                    st);
            double *t = phi;
            phi = phi_alt;
            phi_alt = t;
        } else {
            e = level_sweep<double>(m, l, 1, nullptr, m.u64[l - 1], m.u64[l], m.f64[l],
                                    m.eps64[l], nullptr, st);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rz
