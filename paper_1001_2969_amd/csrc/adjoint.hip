// Adjoint of a window of N collision-free merged steps: the reverse-mode
// gradient of a smooth ion-flux objective with respect to the z = 0
// electrode voltage (its dc and rf amplitudes) and the weights of the
// particles at the start of the window.
//
// Forward: the ordinary merged step (Sec. 2.1), with the particle state, the
// deposit accumulators and phi kept every K steps.  Reverse, segment by
// segment from the last: restore the segment's checkpoint, recompute its
// steps keeping each step's entry state, chi and the solved phi, then walk
// them backwards:
//   - one pass per species over the step's entry particles recomputes the
//     final push and the first push with rotation (Sec. 2.3), adds the
//     deposit adjoint at the new position (Sec. 2.4 weights) and the
//     objective term, and carries the adjoint back through both pushes and
//     the field gather, scattering dJ/dE onto the nodes;
//   - dJ/dphi = -grad^T dJ/dE; the field equation's adjoint is a solve with
//     the same operator (Sec. 2.5: the finite-volume operator times the
//     control volumes is symmetric), done by the same multigrid; from it the
//     adjoints of the charge density, of chi through the face
//     permittivities, and of the electrode voltage;
//   - those give the adjoint of the deposited counts N_ij of each species,
//     which the pass of the previous step reads.
// Particle adjoints are indexed by identity (no collisions and no weight
// split: identities are neither created nor reused), so the compaction and
// any tile sort of the forward steps need no bookkeeping.
//
// The objective is J = sum over steps and live ions of
//   (q_i dt / delta) w (-v_z) exp(-z / delta),
// the ion current toward the powered electrode, weighted to the layer of
// thickness delta in front of it, summed over the window.
#include "ctx.h"
#include "device.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

using namespace rz;

namespace rz {
namespace {

// Adjoint state of one species, indexed by particle identity: per identity
// 8 doubles (64 bytes, one aligned segment) holding the adjoint of the entry
// state r, z, v_r, v_theta, v_z, a_r, a_z and dJ/dw accumulated over the
// window.  Identity order is not particle order once particles are sorted;
// one contiguous record per identity keeps each access a single segment.
struct AdjLam {
    double *rec;  // [cap][8]
    int64_t cap;  // identities are < cap
};
constexpr int kLamW = 7;  // index of dJ/dw in a record

__device__ __forceinline__ double block_sum(double v, double *sh)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) t += sh[w];
    return t;  // in thread 0
}

// d s_r1 / d r of the radial weights at radius r in radial cell j.
__device__ __forceinline__ double dsr_dr(const Mesh &m, double r, int j)
{
    if (m.weighting == 1) return m.inv_hr;
    return 2.0 * (r * m.inv_hr) * m.inv_hr / (double)(2 * j + 1);
}

// Copy of a species' live particles and its count (checkpoints, tape, restore).
__global__ void k_adj_copy(Parts<double> src, const Counts *scnt, Parts<double> dst, Counts *dcnt)
{
    const int64_t n = scnt->n;
    if (blockIdx.x == 0 && threadIdx.x == 0) *dcnt = *scnt;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        dst.r[i] = src.r[i];
        dst.z[i] = src.z[i];
        dst.vr[i] = src.vr[i];
        dst.vt[i] = src.vt[i];
        dst.vz[i] = src.vz[i];
        dst.ar[i] = src.ar[i];
        dst.az[i] = src.az[i];
        dst.w[i] = src.w[i];
        dst.id[i] = src.id[i];
    }
}

// Objective of one step: per-block partial sums over the live ions.
__global__ __launch_bounds__(256) void k_adj_objective(Parts<double> p, const Counts *cnt, double cJ,
                                                       double inv_delta, double *partial)
{
    __shared__ double sh[4];
    const int64_t n = cnt->n;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        acc += cJ * p.w[i] * (-p.vz[i]) * exp(-p.z[i] * inv_delta);
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// *J += the partial sums, in block order.
__global__ __launch_bounds__(256) void k_adj_sum(const double *partial, int nb, double *J)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partial[b];
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) *J += t;
}

struct AdjPassArgs {
    Parts<double> p;  // entry state of the step
    const Counts *cnt;
    Mesh m;
    double dt, k1, k2, qm;
    const double2 *E2;   // E of the step's solve
    const double *nbar;  // adjoint of this species' deposited counts at the exit positions, or null
    double *ebar_r, *ebar_z;
    AdjLam lam;
    int objective;  // species carries the objective
    double cJ, inv_delta;
    unsigned long long *err;
    // LDS window of dJ/dE (particles sorted by tile): the tile of the block's
    // first particle plus kAdjHalo cells; 0 = every contribution to global atomics
    int win, tile_z, tile_r;
};

constexpr int kAdjHalo = 4;

// LDS bytes of the dJ/dE window of a tile_z x tile_r tile.
__host__ __device__ constexpr size_t adj_window_bytes(int tile_z, int tile_r)
{
    return 2 * sizeof(double) * (size_t)(tile_z + 2 * kAdjHalo + 1) *
           (size_t)(tile_r + 2 * kAdjHalo + 1);
}

// Reverse of one step of one species (see the file comment).  The forward
// arithmetic is that of the fused pass: gather, final push with the axis
// rule, absorption, first push with rotation, absorption.  Each block takes
// a contiguous range of the particles.
__global__ __launch_bounds__(256) void k_adj_particles(AdjPassArgs a)
{
    extern __shared__ double lwin[];
    const int64_t n = a.cnt->n;
    const Mesh &m = a.m;
    const double dt = a.dt, half = 0.5;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = b0 + per < n ? b0 + per : n;
    // window nodes [wi0, wi0 + wni) x [wj0, wj0 + wnj); none when wni = 0
    int wi0 = 0, wj0 = 0, wni = 0, wnj = 0;
    if (a.win && b0 < b1) {
        const W4<double> q0 = weights<double>(m, a.p.r[b0], a.p.z[b0]);
        const int ti = q0.i / a.tile_z, tj = q0.j / a.tile_r;
        const int ci0 = ti * a.tile_z - kAdjHalo > 0 ? ti * a.tile_z - kAdjHalo : 0;
        const int cj0 = tj * a.tile_r - kAdjHalo > 0 ? tj * a.tile_r - kAdjHalo : 0;
        int ci1 = (ti + 1) * a.tile_z + kAdjHalo, cj1 = (tj + 1) * a.tile_r + kAdjHalo;
        ci1 = ci1 < m.nz - 1 ? ci1 : m.nz - 1;  // cells [ci0, ci1), nodes [ci0, ci1]
        cj1 = cj1 < m.nr - 1 ? cj1 : m.nr - 1;
        wi0 = ci0;
        wj0 = cj0;
        wni = ci1 - ci0 + 1;
        wnj = cj1 - cj0 + 1;
    }
    const int wn = wni * wnj;
    double *lr_win = lwin, *lz_win = lwin + wn;
    for (int g = threadIdx.x; g < 2 * wn; g += blockDim.x) lwin[g] = 0.0;
    if (a.win) __syncthreads();
    const unsigned wci = wni > 1 ? (unsigned)(wni - 1) : 0u, wcj = wnj > 1 ? (unsigned)(wnj - 1) : 0u;

    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        const uint64_t id = a.p.id[i];
        if (id >= (uint64_t)a.lam.cap) {
            atomicOr(a.err, 1ull);
            continue;
        }
        double2 *rec = (double2 *)(a.lam.rec + 8 * id);
        const double r0 = a.p.r[i], z0 = a.p.z[i], vr0 = a.p.vr[i], vt0 = a.p.vt[i];
        const double vz0 = a.p.vz[i], ar0 = a.p.ar[i], az0 = a.p.az[i], w = a.p.w[i];
        const double2 l01 = rec[0], l23 = rec[1], l45 = rec[2], l67 = rec[3];
        // gather
        const W4<double> q = weights<double>(m, r0, z0);
        const double2 e00 = a.E2[q.g], e01 = a.E2[q.g + 1], e10 = a.E2[q.g + m.nr],
                      e11 = a.E2[q.g + m.nr + 1];
        const double w00 = q.sz0 * q.sr0, w01 = q.sz0 * q.sr1, w10 = q.sz1 * q.sr0,
                     w11 = q.sz1 * q.sr1;
        const double Er = w00 * e00.x + w01 * e01.x + w10 * e10.x + w11 * e11.x;
        const double Ez = w00 * e00.y + w01 * e01.y + w10 * e10.y + w11 * e11.y;
        // final push, axis rule
        double r1 = r0 + a.k1 * Er;
        const double z1 = z0 + a.k1 * Ez;
        double vr1 = vr0 + a.k2 * Er;
        const double vz1 = vz0 + a.k2 * Ez;
        double ar1 = half * (a.qm * Er + ar0);
        const double az1 = half * (a.qm * Ez + az0);
        double sr = 1.0, sv = 1.0, sa = 1.0;  // derivatives of the axis rule
        if (r1 < 0.0) {
            r1 = -r1;
            sr = -1.0;
            sv = vr1 < 0.0 ? -1.0 : 1.0;
            sa = ar1 < 0.0 ? -1.0 : 1.0;
            vr1 = fabs(vr1);
            ar1 = fabs(ar1);
        }
        bool dead = z1 <= 0.0 || z1 >= m.L || r1 >= m.R;
        // first push and rotation (a_theta = 0)
        const double vx = vr1 + half * ar1 * dt;
        const double vy = vt0;
        const double x = r1 + vx * dt;
        const double y = vy * dt;
        const double vz2 = vz1 + half * az1 * dt;
        const double z2 = z1 + vz2 * dt;
        const double rn = sqrt(x * x + y * y);
        double c = 1.0, sn = 0.0;
        if (rn > 0.0) {
            c = x / rn;
            sn = y / rn;
        }
        const double r2 = rn;
        dead = dead || z2 <= 0.0 || z2 >= m.L || r2 >= m.R;
        if (dead) {  // nothing after this step depends on the particle
            rec[0] = make_double2(0.0, 0.0);
            rec[1] = make_double2(0.0, 0.0);
            rec[2] = make_double2(0.0, 0.0);
            rec[3] = make_double2(0.0, l67.y);
            continue;
        }
        // adjoint of the exit state: later steps, this step's deposit, the objective
        double lr = l01.x, lz = l01.y, lvr = l23.x, lvt = l23.y;
        double lvz = l45.x, lar = l45.y, laz = l67.x;
        double wb = l67.y;
        if (a.nbar) {
            const W4<double> q2 = weights<double>(m, r2, z2);
            const double n00 = a.nbar[q2.g], n01 = a.nbar[q2.g + 1], n10 = a.nbar[q2.g + m.nr],
                         n11 = a.nbar[q2.g + m.nr + 1];
            wb += q2.sz0 * q2.sr0 * n00 + q2.sz0 * q2.sr1 * n01 + q2.sz1 * q2.sr0 * n10 +
                  q2.sz1 * q2.sr1 * n11;
            const double ds = dsr_dr(m, r2, q2.j);
            lr += w * ds * ((q2.sz0 * n01 + q2.sz1 * n11) - (q2.sz0 * n00 + q2.sz1 * n10));
            lz += w * m.inv_hz * ((q2.sr0 * n10 + q2.sr1 * n11) - (q2.sr0 * n00 + q2.sr1 * n01));
        }
        if (a.objective) {
            const double e = exp(-z2 * a.inv_delta);
            wb += a.cJ * (-vz2) * e;
            lvz += -a.cJ * w * e;
            lz += a.cJ * w * vz2 * e * a.inv_delta;
        }
        // reverse of the rotation onto r = |(x, y)|
        double xb, yb;
        if (rn > 0.0) {
            const double cb = lvr * vx + lvt * vy + lar * ar1;
            const double sb = lvr * vy - lvt * vx;
            const double tau = (cb * sn - sb * c) / rn;
            xb = lr * c + sn * tau;
            yb = lr * sn - c * tau;
        } else {
            xb = lr;
            yb = 0.0;
        }
        // reverse of the first push
        const double vxb = lvr * c - lvt * sn + xb * dt;
        const double vyb = lvr * sn + lvt * c + yb * dt;
        const double ar1b = lar * c + vxb * half * dt;
        const double vz2b = lvz + lz * dt;
        const double az1b = laz + vz2b * half * dt;
        // reverse of the axis rule and of the final push
        const double r1pb = sr * xb, vr1pb = sv * vxb, ar1pb = sa * ar1b;
        const double Erb = a.k1 * r1pb + a.k2 * vr1pb + half * a.qm * ar1pb;
        const double Ezb = a.k1 * lz + a.k2 * vz2b + half * a.qm * az1b;
        // reverse of the gather: position terms, then dJ/dE onto the nodes
        const double ds0 = dsr_dr(m, r0, q.j);
        const double dEr_dr = ds0 * ((q.sz0 * e01.x + q.sz1 * e11.x) - (q.sz0 * e00.x + q.sz1 * e10.x));
        const double dEz_dr = ds0 * ((q.sz0 * e01.y + q.sz1 * e11.y) - (q.sz0 * e00.y + q.sz1 * e10.y));
        const double dEr_dz = m.inv_hz * ((q.sr0 * e10.x + q.sr1 * e11.x) - (q.sr0 * e00.x + q.sr1 * e01.x));
        const double dEz_dz = m.inv_hz * ((q.sr0 * e10.y + q.sr1 * e11.y) - (q.sr0 * e00.y + q.sr1 * e01.y));
        rec[0] = make_double2(r1pb + Erb * dEr_dr + Ezb * dEz_dr, lz + Erb * dEr_dz + Ezb * dEz_dz);
        rec[1] = make_double2(vr1pb, vyb);
        rec[2] = make_double2(vz2b, half * ar1pb);
        rec[3] = make_double2(half * az1b, wb);
        const int li = q.i - wi0, lj = q.j - wj0;
        if ((unsigned)li < wci && (unsigned)lj < wcj) {
            const int l = li * wnj + lj;
            atomicAdd(lr_win + l, w00 * Erb);
            atomicAdd(lr_win + l + 1, w01 * Erb);
            atomicAdd(lr_win + l + wnj, w10 * Erb);
            atomicAdd(lr_win + l + wnj + 1, w11 * Erb);
            atomicAdd(lz_win + l, w00 * Ezb);
            atomicAdd(lz_win + l + 1, w01 * Ezb);
            atomicAdd(lz_win + l + wnj, w10 * Ezb);
            atomicAdd(lz_win + l + wnj + 1, w11 * Ezb);
        } else {
            unsafeAtomicAdd(a.ebar_r + q.g, w00 * Erb);
            unsafeAtomicAdd(a.ebar_r + q.g + 1, w01 * Erb);
            unsafeAtomicAdd(a.ebar_r + q.g + m.nr, w10 * Erb);
            unsafeAtomicAdd(a.ebar_r + q.g + m.nr + 1, w11 * Erb);
            unsafeAtomicAdd(a.ebar_z + q.g, w00 * Ezb);
            unsafeAtomicAdd(a.ebar_z + q.g + 1, w01 * Ezb);
            unsafeAtomicAdd(a.ebar_z + q.g + m.nr, w10 * Ezb);
            unsafeAtomicAdd(a.ebar_z + q.g + m.nr + 1, w11 * Ezb);
        }
    }
    if (!a.win) return;
    __syncthreads();
    for (int g = threadIdx.x; g < wn; g += blockDim.x) {
        const int k = (wi0 + g / wnj) * m.nr + wj0 + g % wnj;
        const double vr = lr_win[g], vz = lz_win[g];
        if (vr != 0.0) unsafeAtomicAdd(a.ebar_r + k, vr);
        if (vz != 0.0) unsafeAtomicAdd(a.ebar_z + k, vz);
    }
}

// dJ/dw of the deposit at the window's first positions.
__global__ __launch_bounds__(256) void k_adj_wdep(Parts<double> p, const Counts *cnt, Mesh m,
                                                  const double *nbar, AdjLam lam,
                                                  unsigned long long *err)
{
    const int64_t n = cnt->n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t id = p.id[i];
        if (id >= (uint64_t)lam.cap) {
            atomicOr(err, 1ull);
            continue;
        }
        const W4<double> q = weights<double>(m, p.r[i], p.z[i]);
        lam.rec[8 * id + kLamW] += q.sz0 * q.sr0 * nbar[q.g] + q.sz0 * q.sr1 * nbar[q.g + 1] +
                        q.sz1 * q.sr0 * nbar[q.g + m.nr] + q.sz1 * q.sr1 * nbar[q.g + m.nr + 1];
    }
}

// dJ/dpsi on the nodes for a relative perturbation psi of the window's
// initial density, w_p -> w_p (1 + sum_k S_k(x_p) psi_k) for both species:
// sum_p (dJ/dw_p) w_p S_k(x_p).
__global__ __launch_bounds__(256) void k_adj_density(Parts<double> p, const Counts *cnt, Mesh m,
                                                     AdjLam lam, double *gpsi)
{
    const int64_t n = cnt->n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t id = p.id[i];
        if (id >= (uint64_t)lam.cap) continue;  // reported by the reverse pass
        const double g = lam.rec[8 * id + kLamW] * p.w[i];
        if (g == 0.0) continue;
        const W4<double> q = weights<double>(m, p.r[i], p.z[i]);
        unsafeAtomicAdd(gpsi + q.g, q.sz0 * q.sr0 * g);
        unsafeAtomicAdd(gpsi + q.g + 1, q.sz0 * q.sr1 * g);
        unsafeAtomicAdd(gpsi + q.g + m.nr, q.sz1 * q.sr0 * g);
        unsafeAtomicAdd(gpsi + q.g + m.nr + 1, q.sz1 * q.sr1 * g);
    }
}

// dJ/dw by identity out of the records.
__global__ void k_adj_wbar_out(AdjLam lam, double *out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < lam.cap;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = lam.rec[8 * i + kLamW];
}

// Control-volume weight of column j relative to pi hr^2 hz (the factor that
// makes the operator symmetric): 2j off the axis, 1/4 on it.
__device__ __forceinline__ double omega(int j) { return j == 0 ? 0.25 : 2.0 * (double)j; }

__device__ __forceinline__ bool unknown(int i, int j, int nr, int nz)
{
    return i >= 1 && i <= nz - 2 && j <= nr - 2;
}

struct GridAdjArgs {
    int nr, nz;
    double hr, hz, dt;
    const double *ebar_r, *ebar_z;
    double *phibar;       // dJ/dphi on every node
    double *f, *eps;      // the adjoint solve's right-hand side and permittivity
    const double *chi;    // chi of the step
    const double *phi;    // phi of the step's solve
    const double *mu;     // adjoint solve's solution (zero on the Dirichlet nodes)
    const double *vol;    // weighting volumes
    double q0, m0, q1, m1;
    double *nbar0, *nbar1;
};

// dJ/dphi = -(grad)^T dJ/dE with the differences of the E kernel (centred
// inside, one-sided on z = 0, z = L and r = R, E_r = 0 on the axis); the
// adjoint solve's right-hand side dJ/dphi / omega on the unknowns; eps = 1 + chi.
__global__ void k_adj_phibar(GridAdjArgs g)
{
    const int nr = g.nr, nz = g.nz, nn = nr * nz;
    const double ihz = 1.0 / g.hz, ihr = 1.0 / g.hr;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nn; k += gridDim.x * blockDim.x) {
        const int i = k / nr, j = k - i * nr;
        double pb = 0.0;
        if (i == 0) pb += g.ebar_z[k] * ihz;
        if (i == nz - 1) pb -= g.ebar_z[k] * ihz;
        if (i >= 1) pb -= g.ebar_z[k - nr] * (i - 1 == 0 ? ihz : 0.5 * ihz);
        if (i + 1 <= nz - 1) pb += g.ebar_z[k + nr] * (i + 1 == nz - 1 ? ihz : 0.5 * ihz);
        if (j == nr - 1) pb -= g.ebar_r[k] * ihr;
        if (j - 1 >= 1) pb -= g.ebar_r[k - 1] * 0.5 * ihr;
        if (j + 1 <= nr - 1) pb += g.ebar_r[k + 1] * (j + 1 == nr - 1 ? ihr : 0.5 * ihr);
        g.phibar[k] = pb;
        g.f[k] = unknown(i, j, nr, nz) ? pb / omega(j) : 0.0;
        g.eps[k] = 1.0 + g.chi[k];
    }
}

// From the adjoint solution mu: dJ/df = omega mu on the unknowns, dJ/dchi
// through the averaged face permittivities (each face (P, Q) of the operator
// contributes -1/2 G_PQ (mu_P - mu_Q)(phi_P - phi_Q) to both ends, G_PQ the
// symmetric face coefficient), and the adjoint of each species' counts,
// N_s -> n_s = N_s / V -> rho, chi.
__global__ void k_adj_nbar(GridAdjArgs g)
{
    const int nr = g.nr, nz = g.nz, nn = nr * nz;
    const double ihz2 = 1.0 / (g.hz * g.hz), ihr2 = 1.0 / (g.hr * g.hr);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nn; k += gridDim.x * blockDim.x) {
        const int i = k / nr, j = k - i * nr;
        const double m0 = g.mu[k], p0 = g.phi[k], om = omega(j);
        double cb = 0.0;
        if (i > 0) cb -= 0.5 * om * ihz2 * (m0 - g.mu[k - nr]) * (p0 - g.phi[k - nr]);
        if (i < nz - 1) cb -= 0.5 * om * ihz2 * (m0 - g.mu[k + nr]) * (p0 - g.phi[k + nr]);
        if (j > 0) cb -= 0.5 * (double)(2 * j - 1) * ihr2 * (m0 - g.mu[k - 1]) * (p0 - g.phi[k - 1]);
        if (j < nr - 1)
            cb -= 0.5 * (double)(2 * j + 1) * ihr2 * (m0 - g.mu[k + 1]) * (p0 - g.phi[k + 1]);
        const double fb = unknown(i, j, nr, nz) ? om * m0 : 0.0;
        const double dt2 = g.dt * g.dt, iv = 1.0 / g.vol[k];
        g.nbar0[k] = (g.q0 * fb / kEps0 + cb * g.q0 * g.q0 * dt2 / (2.0 * g.m0 * kEps0)) * iv;
        g.nbar1[k] = (g.q1 * fb / kEps0 + cb * g.q1 * g.q1 * dt2 / (2.0 * g.m1 * kEps0)) * iv;
    }
}

// dJ/dV of the step's electrode value: the direct dependence of E on the
// z = 0 nodes plus their coupling into the first row of unknowns; added to
// dJ/dV_dc and, times sin(2 pi f t), to dJ/dV_rf.  One block.
__global__ __launch_bounds__(256) void k_adj_vbar(GridAdjArgs g, double sinv, double *gv)
{
    __shared__ double sh[4];
    const int nr = g.nr;
    const double ihz2 = 1.0 / (g.hz * g.hz);
    double acc = 0.0;
    for (int j = threadIdx.x; j < nr - 1; j += blockDim.x) {
        const double face = 0.5 * ((1.0 + g.chi[j]) + (1.0 + g.chi[nr + j]));
        acc += g.phibar[j] + omega(j) * g.mu[nr + j] * face * ihz2;
    }
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        gv[0] += t;
        gv[1] += t * sinv;
    }
}

}  // namespace
}  // namespace rz

// ===========================================================================

struct rzpic_adjoint {
    rzpic_ctx *c = nullptr;
    rzpic_adjoint_config cfg{};
    int nck = 0;  // checkpoints: window start of each segment, and the window end
    int K = 0;
    double delta = 0.0, tol = 0.0;
    int max_cycles = 0;
    std::vector<void *> allocs;
    // particle copies: [slot][species]
    std::vector<Parts<double>> ck[2], tape[2];
    Counts *ck_cnt = nullptr, *tape_cnt = nullptr;  // [slot][2]
    unsigned long long *ck_acc = nullptr;           // [slot][2][nn]
    double *ck_phi = nullptr;                       // [slot][2][nn] (phi, phi_alt)
    double *seg_chi = nullptr, *seg_phi = nullptr;  // [K][nn]
    double *er = nullptr, *ez = nullptr, *E2 = nullptr;
    double *ebar = nullptr;  // [2][nn]
    double *phibar = nullptr, *mu = nullptr, *mu_alt = nullptr, *nbar = nullptr;  // nbar [2][nn]
    double *lam[2] = {nullptr, nullptr};  // [cap_s][8]
    double *partial = nullptr, *J = nullptr, *gv = nullptr;
    unsigned long long *err = nullptr;
    int64_t step0 = -1;
    bool have_forward = false;
};

// Defined in runtime.hip.
rzpic_status rz_fail(rzpic_status s, const char *msg);
Mesh rz_mesh(const rzpic_ctx *c);
rzpic_status rz_settle(rzpic_ctx *c);
SpeciesK rz_species(const rzpic_ctx *c, int s);
rzpic_status rz_cycles(rzpic_ctx *c, double V, double *&u, double *&u_alt, double tol,
                       int max_cycles, int *cycles, double *relres);

namespace {

constexpr int kObjBlocks = 1024;

rzpic_status failf(rzpic_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return rz_fail(st, buf);
}

#define AHIP(expr)                                                                            \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return failf(RZPIC_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                         __FILE__, __LINE__);                                                 \
    } while (0)

#define ATRY(expr)                      \
    do {                                \
        rzpic_status s_ = (expr);       \
        if (s_ != RZPIC_OK) return s_;  \
    } while (0)

template <typename T> rzpic_status aalloc(rzpic_adjoint *a, T **p, size_t count)
{
    void *q = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 256;
    if (hipMalloc(&q, bytes) != hipSuccess)
        return failf(RZPIC_ENOMEM, "adjoint: hipMalloc(%zu) failed", bytes);
    if (hipMemset(q, 0, bytes) != hipSuccess) {
        (void)hipFree(q);
        return failf(RZPIC_EHIP, "adjoint: hipMemset failed");
    }
    a->allocs.push_back(q);
    *p = (T *)q;
    return RZPIC_OK;
}

rzpic_status alloc_parts(rzpic_adjoint *a, Parts<double> &p, int64_t cap)
{
    double *f[8];
    for (auto &x : f) ATRY(aalloc(a, &x, (size_t)cap));
    p.r = f[0];
    p.z = f[1];
    p.vr = f[2];
    p.vt = f[3];
    p.vz = f[4];
    p.ar = f[5];
    p.az = f[6];
    p.w = f[7];
    ATRY(aalloc(a, &p.id, (size_t)cap));
    return RZPIC_OK;
}

Parts<double> ctx_parts(const rzpic_ctx *c, int s)
{
    const rzpic_species_view &v = c->sp[s].v;
    Parts<double> p{};
    p.r = (double *)v.r;
    p.z = (double *)v.z;
    p.vr = (double *)v.vr;
    p.vt = (double *)v.vt;
    p.vz = (double *)v.vz;
    p.ar = (double *)v.ar;
    p.az = (double *)v.az;
    p.w = (double *)v.w;
    p.id = v.id;
    return p;
}

AdjLam lam_of(const rzpic_adjoint *a, int s) { return AdjLam{a->lam[s], a->cfg.id_capacity[s]}; }

// Blocks of the reverse particle pass: contiguous ranges of about 4096
// particles of the capacity each.
int pass_blocks(int64_t cap)
{
    int64_t b = (cap + 4095) / 4096;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

int copy_blocks(int64_t cap)
{
    int64_t b = (cap + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

// Window state of the context <-> checkpoint `slot` (particles, counts, the
// deposit accumulators and both phi buffers).
rzpic_status checkpoint(rzpic_adjoint *a, int slot, bool save)
{
    rzpic_ctx *c = a->c;
    const size_t nn = (size_t)c->nn;
    for (int s = 0; s < 2; ++s) {
        Parts<double> cp = ctx_parts(c, s), kp = a->ck[s][slot];
        Counts *kc = a->ck_cnt + 2 * slot + s;
        const int nb = copy_blocks(c->sp[s].cap);
        if (save) hipLaunchKernelGGL(k_adj_copy, dim3(nb), dim3(256), 0, c->st, cp, c->cnt + s, kp, kc);
        else hipLaunchKernelGGL(k_adj_copy, dim3(nb), dim3(256), 0, c->st, kp, kc, cp, c->cnt + s);
        AHIP(hipGetLastError());
        unsigned long long *ka = a->ck_acc + (2 * (size_t)slot + s) * nn;
        if (save) AHIP(hipMemcpyAsync(ka, c->acc[s], nn * 8, hipMemcpyDeviceToDevice, c->st));
        else AHIP(hipMemcpyAsync(c->acc[s], ka, nn * 8, hipMemcpyDeviceToDevice, c->st));
    }
    double *kp = a->ck_phi + 2 * (size_t)slot * nn;
    if (save) {
        AHIP(hipMemcpyAsync(kp, c->phi, nn * 8, hipMemcpyDeviceToDevice, c->st));
        AHIP(hipMemcpyAsync(kp + nn, c->phi_alt, nn * 8, hipMemcpyDeviceToDevice, c->st));
    } else {
        AHIP(hipMemcpyAsync(c->phi, kp, nn * 8, hipMemcpyDeviceToDevice, c->st));
        AHIP(hipMemcpyAsync(c->phi_alt, kp + nn, nn * 8, hipMemcpyDeviceToDevice, c->st));
    }
    return RZPIC_OK;
}

rzpic_status objective(rzpic_adjoint *a)
{
    rzpic_ctx *c = a->c;
    const double cJ = c->sp[1].v.q * c->c.dt / a->delta;
    hipLaunchKernelGGL(k_adj_objective, dim3(kObjBlocks), dim3(256), 0, c->st, ctx_parts(c, 1),
                       (const Counts *)(c->cnt + 1), cJ, 1.0 / a->delta, a->partial);
    hipLaunchKernelGGL(k_adj_sum, dim3(1), dim3(256), 0, c->st, (const double *)a->partial,
                       kObjBlocks, a->J);
    AHIP(hipGetLastError());
    return RZPIC_OK;
}

rzpic_status check_ctx(const rzpic_ctx *c)
{
    if (c->mixed) return rz_fail(RZPIC_EINVAL, "adjoint: the context must be FP64");
    for (int s = 0; s < 2; ++s) {
        if (!c->sp[s].bound) return rz_fail(RZPIC_ESTATE, "adjoint: both species must be bound");
        if (c->sp[s].v.mc_model != RZPIC_MC_NONE)
            return rz_fail(RZPIC_EINVAL,
                           "adjoint: the window is collision-free (species mc_model must be "
                           "RZPIC_MC_NONE)");
    }
    if (c->c.resize_every != 0)
        return rz_fail(RZPIC_EINVAL, "adjoint: weight splitting must be off (resize_every = 0)");
    if (c->c.mg_fixed_cycles > 0)
        return rz_fail(RZPIC_EINVAL,
                       "adjoint: the field solves must be converged (mg_fixed_cycles = 0)");
    if (c->c.chi_face != RZPIC_FACE_AVG)
        return rz_fail(RZPIC_EINVAL, "adjoint: needs the averaged face permittivity");
    if (c->c.damping != RZPIC_DAMP_D1)
        return rz_fail(RZPIC_EINVAL, "adjoint: the window differentiates the D1 push");
    if (c->c.circuit_C > 0.0)
        return rz_fail(RZPIC_EINVAL, "adjoint: the electrode must be driven directly (circuit_C = 0)");
    if (c->c.ion_subcycle > 1)
        return rz_fail(RZPIC_EINVAL, "adjoint: ions must move every step (ion_subcycle <= 1)");
    if (c->c.push_form != RZPIC_PUSH_LOCAL)
        return rz_fail(RZPIC_EINVAL, "adjoint: needs the local-frame push (push_form = LOCAL)");
    if (c->children_pending[0] || c->children_pending[1])
        return rz_fail(RZPIC_ESTATE, "adjoint: new particles are staged");
    return RZPIC_OK;
}

}  // namespace

// ===========================================================================

extern "C" {

rzpic_status rzpic_adjoint_create(rzpic_ctx *c, const rzpic_adjoint_config *cfg,
                                  rzpic_adjoint **out)
{
    if (!c || !cfg || !out) return rz_fail(RZPIC_EINVAL, "adjoint: null argument");
    *out = nullptr;
    ATRY(check_ctx(c));
    ATRY(rz_settle(c));  // a pipelined step's pending list maintenance
    if (cfg->n_steps < 1) return rz_fail(RZPIC_EINVAL, "adjoint: n_steps must be >= 1");
    if (cfg->checkpoint_every < 0)
        return rz_fail(RZPIC_EINVAL, "adjoint: checkpoint_every must be >= 0");
    for (int s = 0; s < 2; ++s)
        if (cfg->id_capacity[s] < 1 || cfg->id_capacity[s] > ((int64_t)1 << 40))
            return rz_fail(RZPIC_EINVAL, "adjoint: id_capacity out of range");
    if (!(cfg->delta >= 0.0) || !(cfg->tol >= 0.0) || cfg->max_cycles < 0)
        return rz_fail(RZPIC_EINVAL, "adjoint: delta, tol and max_cycles must be >= 0");
    rzpic_adjoint *a = new rzpic_adjoint();
    a->c = c;
    a->cfg = *cfg;
    a->K = cfg->checkpoint_every > 0 ? cfg->checkpoint_every : 10;
    if (a->K > cfg->n_steps) a->K = cfg->n_steps;
    a->nck = (cfg->n_steps + a->K - 1) / a->K + 1;
    a->delta = cfg->delta > 0.0 ? cfg->delta : 2.0 * c->hz;
    a->tol = cfg->tol > 0.0 ? cfg->tol : c->c.mg_tol;
    a->max_cycles = cfg->max_cycles > 0 ? cfg->max_cycles : c->c.mg_max_cycles;
    auto bail = [&](rzpic_status st) {
        for (void *p : a->allocs) (void)hipFree(p);
        delete a;
        return st;
    };
    const size_t nn = (size_t)c->nn;
    rzpic_status st = RZPIC_OK;
    for (int s = 0; s < 2 && st == RZPIC_OK; ++s) {
        a->ck[s].resize(a->nck);
        a->tape[s].resize(a->K);
        for (auto &p : a->ck[s])
            if (st == RZPIC_OK) st = alloc_parts(a, p, c->sp[s].cap);
        for (auto &p : a->tape[s])
            if (st == RZPIC_OK) st = alloc_parts(a, p, c->sp[s].cap);
        if (st == RZPIC_OK) st = aalloc(a, &a->lam[s], 8 * (size_t)cfg->id_capacity[s]);
    }
    if (st == RZPIC_OK) st = aalloc(a, &a->ck_cnt, 2 * (size_t)a->nck);
    if (st == RZPIC_OK) st = aalloc(a, &a->tape_cnt, 2 * (size_t)a->K);
    if (st == RZPIC_OK) st = aalloc(a, &a->ck_acc, 2 * (size_t)a->nck * nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->ck_phi, 2 * (size_t)a->nck * nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->seg_chi, (size_t)a->K * nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->seg_phi, (size_t)a->K * nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->er, nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->ez, nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->E2, 2 * nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->ebar, 2 * nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->phibar, nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->mu, nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->mu_alt, nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->nbar, 2 * nn);
    if (st == RZPIC_OK) st = aalloc(a, &a->partial, kObjBlocks);
    if (st == RZPIC_OK) st = aalloc(a, &a->J, 1);
    if (st == RZPIC_OK) st = aalloc(a, &a->gv, 2);
    if (st == RZPIC_OK) st = aalloc(a, &a->err, 1);
    if (st != RZPIC_OK) return bail(st);
    *out = a;
    return RZPIC_OK;
}

rzpic_status rzpic_adjoint_destroy(rzpic_adjoint *a)
{
    if (!a) return RZPIC_OK;
    (void)hipStreamSynchronize(a->c->st);
    for (void *p : a->allocs) (void)hipFree(p);
    delete a;
    return RZPIC_OK;
}

rzpic_status rzpic_adjoint_forward(rzpic_adjoint *a, int64_t step0, double *J_out)
{
    if (!a || !J_out) return rz_fail(RZPIC_EINVAL, "adjoint: null argument");
    rzpic_ctx *c = a->c;
    ATRY(check_ctx(c));
    ATRY(rz_settle(c));  // a pipelined step's pending list maintenance
    const int N = a->cfg.n_steps;
    if (step0 < 0 || step0 + N > 0xFFFFFFFFLL)
        return rz_fail(RZPIC_EINVAL, "adjoint: step range out of bounds");
    a->have_forward = false;
    AHIP(launch_fill_u64((unsigned long long *)a->J, 1, c->st));
    for (int k = 0; k < N; ++k) {
        if (k % a->K == 0) ATRY(checkpoint(a, k / a->K, true));
        ATRY(rzpic_step(c, step0 + k));
        ATRY(objective(a));
    }
    ATRY(checkpoint(a, a->nck - 1, true));
    AHIP(hipMemcpyAsync(J_out, a->J, sizeof(double), hipMemcpyDeviceToHost, c->st));
    AHIP(hipStreamSynchronize(c->st));
    ATRY(rzpic_sync(c));
    a->step0 = step0;
    a->have_forward = true;
    return RZPIC_OK;
}

rzpic_status rzpic_adjoint_backward(rzpic_adjoint *a, double grad_V[2], double *grad_w0,
                                    double *grad_w1, double *grad_density)
{
    if (!a || !grad_V) return rz_fail(RZPIC_EINVAL, "adjoint: null argument");
    if (!a->have_forward)
        return rz_fail(RZPIC_ESTATE, "adjoint: backward needs a completed forward window");
    rzpic_ctx *c = a->c;
    ATRY(check_ctx(c));
    ATRY(rz_settle(c));  // a pipelined step's pending list maintenance
    hipStream_t st = c->st;
    const int N = a->cfg.n_steps, K = a->K, nr = c->c.nr, nz = c->c.nz;
    const size_t nn = (size_t)c->nn;
    const Mesh m = rz_mesh(c);
    const SpeciesK sk[2] = {rz_species(c, 0), rz_species(c, 1)};
    for (int s = 0; s < 2; ++s)
        AHIP(launch_fill_u64((unsigned long long *)a->lam[s], 8 * a->cfg.id_capacity[s], st));
    AHIP(launch_fill_u64((unsigned long long *)a->gv, 2, st));
    AHIP(launch_fill_u64(a->err, 1, st));
    AHIP(launch_fill_u64((unsigned long long *)a->nbar, 2 * nn, st));
    AHIP(launch_fill_u64((unsigned long long *)a->mu, nn, st));
    AHIP(launch_fill_u64((unsigned long long *)a->mu_alt, nn, st));
    bool have_nbar = false;  // the last step's exit deposit feeds no solve of the window
    // dJ/dE in LDS windows when the particles are kept sorted by tile
    const size_t wlds = adj_window_bytes(c->c.tile_z, c->c.tile_r);
    const bool win = c->c.sort_every > 0 && wlds <= 64 * 1024;

    GridAdjArgs g{};
    g.nr = nr;
    g.nz = nz;
    g.hr = c->hr;
    g.hz = c->hz;
    g.dt = c->c.dt;
    g.ebar_r = a->ebar;
    g.ebar_z = a->ebar + nn;
    g.phibar = a->phibar;
    g.f = c->f;
    g.eps = c->eps;
    g.vol = c->vol;
    g.q0 = c->sp[0].v.q;
    g.m0 = c->sp[0].v.m;
    g.q1 = c->sp[1].v.q;
    g.m1 = c->sp[1].v.m;
    g.nbar0 = a->nbar;
    g.nbar1 = a->nbar + nn;
    const int gthreads = 256, gblocks = (int)((nn + gthreads - 1) / gthreads);

    const int nseg = a->nck - 1;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int k0 = seg * K, k1 = (k0 + K < N) ? k0 + K : N;
        // recompute the segment, keeping each step's entry state, chi and phi
        ATRY(checkpoint(a, seg, false));
        for (int k = k0; k < k1; ++k) {
            const int slot = k - k0;
            for (int s = 0; s < 2; ++s) {
                hipLaunchKernelGGL(k_adj_copy, dim3(copy_blocks(c->sp[s].cap)), dim3(256), 0, st,
                                   ctx_parts(c, s), (const Counts *)(c->cnt + s),
                                   a->tape[s][slot], a->tape_cnt + 2 * slot + s);
                AHIP(hipGetLastError());
            }
            ATRY(rzpic_step(c, a->step0 + k));
            AHIP(hipMemcpyAsync(a->seg_chi + slot * nn, c->chi, nn * 8, hipMemcpyDeviceToDevice, st));
            AHIP(hipMemcpyAsync(a->seg_phi + slot * nn, c->phi, nn * 8, hipMemcpyDeviceToDevice, st));
        }
        // reverse
        for (int k = k1 - 1; k >= k0; --k) {
            const int slot = k - k0;
            const double *phi = a->seg_phi + slot * nn, *chi = a->seg_chi + slot * nn;
            AHIP(launch_efield<double>(nr, nz, c->hr, c->hz, phi, a->er, a->ez, (double2 *)a->E2,
                                       st));
            AHIP(launch_fill_u64((unsigned long long *)a->ebar, 2 * nn, st));
            for (int s = 0; s < 2; ++s) {
                AdjPassArgs p{};
                p.p = a->tape[s][slot];
                p.cnt = a->tape_cnt + 2 * slot + s;
                p.m = m;
                p.dt = c->c.dt;
                p.k1 = sk[s].k1;
                p.k2 = sk[s].k2;
                p.qm = sk[s].qm;
                p.E2 = (const double2 *)a->E2;
                p.nbar = have_nbar ? a->nbar + s * nn : nullptr;
                p.ebar_r = a->ebar;
                p.ebar_z = a->ebar + nn;
                p.lam = lam_of(a, s);
                p.objective = s == 1;
                p.cJ = c->sp[1].v.q * c->c.dt / a->delta;
                p.inv_delta = 1.0 / a->delta;
                p.err = a->err;
                p.win = win ? 1 : 0;
                p.tile_z = c->c.tile_z;
                p.tile_r = c->c.tile_r;
                hipLaunchKernelGGL(k_adj_particles, dim3(pass_blocks(c->sp[s].cap)), dim3(256),
                                   win ? wlds : 0, st, p);
                AHIP(hipGetLastError());
            }
            g.chi = chi;
            g.phi = phi;
            hipLaunchKernelGGL(k_adj_phibar, dim3(gblocks), dim3(gthreads), 0, st, g);
            AHIP(hipGetLastError());
            AHIP(mg_restrict_eps(c->mg, 0, st));
            AHIP(mg_set_bc(a->mu, nr, nz, 0.0, st));
            AHIP(mg_set_bc(a->mu_alt, nr, nz, 0.0, st));
            int cyc = 0;
            double rr = 0.0;
            ATRY(rz_cycles(c, 0.0, a->mu, a->mu_alt, a->tol, a->max_cycles, &cyc, &rr));
            g.mu = a->mu;
            hipLaunchKernelGGL(k_adj_nbar, dim3(gblocks), dim3(gthreads), 0, st, g);
            const double t = (double)(a->step0 + k + 1) * c->c.dt;
            const double sinv = std::sin(kTwoPi * c->c.f_rf * t);
            hipLaunchKernelGGL(k_adj_vbar, dim3(1), dim3(256), 0, st, g, sinv, a->gv);
            AHIP(hipGetLastError());
            have_nbar = true;
            if (k == 0)
                for (int s = 0; s < 2; ++s) {
                    hipLaunchKernelGGL(k_adj_wdep, dim3(copy_blocks(c->sp[s].cap)), dim3(256), 0,
                                       st, a->tape[s][0], (const Counts *)a->tape_cnt + s, m,
                                       (const double *)(a->nbar + s * nn), lam_of(a, s), a->err);
                    AHIP(hipGetLastError());
                }
        }
    }
    if (grad_density) {
        AHIP(launch_fill_u64((unsigned long long *)grad_density, nn, st));
        for (int s = 0; s < 2; ++s) {
            hipLaunchKernelGGL(k_adj_density, dim3(copy_blocks(c->sp[s].cap)), dim3(256), 0, st,
                               a->ck[s][0], (const Counts *)a->ck_cnt + s, m, lam_of(a, s),
                               grad_density);
            AHIP(hipGetLastError());
        }
    }
    // the context returns to the end of the window
    ATRY(checkpoint(a, a->nck - 1, false));
    double *gw[2] = {grad_w0, grad_w1};
    for (int s = 0; s < 2; ++s)
        if (gw[s]) {
            hipLaunchKernelGGL(k_adj_wbar_out, dim3(copy_blocks(a->cfg.id_capacity[s])), dim3(256),
                               0, st, lam_of(a, s), gw[s]);
            AHIP(hipGetLastError());
        }
    unsigned long long herr = 0;
    AHIP(hipMemcpyAsync(grad_V, a->gv, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    AHIP(hipMemcpyAsync(&herr, a->err, sizeof herr, hipMemcpyDeviceToHost, st));
    AHIP(hipStreamSynchronize(st));
    if (herr) return rz_fail(RZPIC_EINVAL, "adjoint: a particle identity is >= id_capacity");
    return rzpic_sync(c);
}

}  // extern "C"
