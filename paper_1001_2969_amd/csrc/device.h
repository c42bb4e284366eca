// Device helpers: counter-based random numbers, particle/grid weights, the
// particle push steps and the collision outcomes, shared by the kernels.
#pragma once

#include "internal.h"

namespace rz {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): per round the words
// (c0, c2) are multiplied by the published 32-bit multipliers; the high halves
// are xored with the other two words and the key, which is bumped by the
// published Weyl constants between rounds.

struct U4 {
    uint32_t x, y, z, w;
};

// a ^ b ^ k in one instruction (the three-input bitwise operation of gfx950,
// truth table 0x96), k a wavefront-uniform key word in a scalar register.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// Each round's two products as full 64-bit products (one multiply-add
// instruction each).  The key enters opaque, so that its round values are
// formed by scalar adds at every use instead of being kept (and spilled)
// across the caller's loop.  The key must be uniform over the wavefront.
__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = U4{xor3_key((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
               xor3_key((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Two uniforms in (0,1) from draw block `blk` of (seed, species, id, step):
// counter (id lo, id hi, step, species<<16 | blk), key = seed; each pair of
// words gives a 52-bit integer u and U = (u + 1/2) 2^-52, exact in FP64.
// The two 52-bit integers u of that draw, before the conversion.
__device__ __forceinline__ void draw_u52(uint64_t seed, int s, uint64_t id, uint32_t step,
                                        uint32_t blk, uint64_t &ua, uint64_t &ub)
{
    U4 c{(uint32_t)id, (uint32_t)(id >> 32), step, ((uint32_t)s << 16) | (blk & 0xFFFFu)};
    U4 x = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    ua = ((uint64_t)x.x << 20) | (uint64_t)(x.y >> 12);
    ub = ((uint64_t)x.z << 20) | (uint64_t)(x.w >> 12);
}

__device__ __forceinline__ double u52_unit(uint64_t u) { return ((double)u + 0.5) * 0x1p-52; }

__device__ __forceinline__ void uniform2(uint64_t seed, int s, uint64_t id, uint32_t step,
                                         uint32_t blk, double &a, double &b)
{
    uint64_t ua, ub;
    draw_u52(seed, s, id, step, blk, ua, ub);
    a = u52_unit(ua);
    b = u52_unit(ub);
}

// The null-collision candidate test U0 < P_null decided on the integer u of
// U0 = (u + 1/2) 2^-52: u + 1/2 < P_null 2^52 (both sides exact in FP64)
// holds exactly for u < ceil(P_null 2^52 - 1/2), the threshold the host
// computes once (SpeciesK::cand_u52).  Same decision, no conversion.
__device__ __forceinline__ bool is_candidate(uint64_t ua, uint64_t cand_u52) { return ua < cand_u52; }

__device__ __forceinline__ void normal2(double ua, double ub, double &n1, double &n2)
{
    double rad = sqrt(-2.0 * log(ua));
    double sn, cs;
    sincos(kTwoPi * ub, &sn, &cs);
    n1 = rad * cs;
    n2 = rad * sn;
}

// ---------------------------------------------------------------------------
// Bilinear weights of Sec. 2.4 in (z, r^2) or (z, r).

template <typename T> struct W4 {
    int g;       // index of node (i, j)
    int i, j;    // cell
    T sz0, sz1, sr0, sr1;
};

// 1 / (2j + 1), correctly rounded in double (then rounded to T): computed in
// registers rather than looked up, which would put a dependent memory round
// trip in front of every weighting.
template <typename T> __device__ __forceinline__ T inv2j1(int j)
{
    return (T)(1.0 / (double)(2 * j + 1));
}
// FP32 particles: the hardware reciprocal (within 1 ulp of FP32), one
// instruction instead of an FP64 division; every FP32 kernel weights alike.
template <> __device__ __forceinline__ float inv2j1<float>(int j)
{
    return __builtin_amdgcn_rcpf((float)(2 * j + 1));
}

template <typename T> __device__ __forceinline__ W4<T> weights(const Mesh &m, T r, T z)
{
    W4<T> q;
    const T ihz = (T)m.inv_hz, ihr = (T)m.inv_hr;
    T xz = z * ihz, xr = r * ihr;
    int i = (int)xz, j = (int)xr;
    i = i < 0 ? 0 : (i > m.nz - 2 ? m.nz - 2 : i);
    j = j < 0 ? 0 : (j > m.nr - 2 ? m.nr - 2 : j);
    q.g = i * m.nr + j;
    q.i = i;
    q.j = j;
    T zi = (T)i * (T)m.hz, zi1 = (T)(i + 1) * (T)m.hz;
    q.sz0 = (zi1 - z) * ihz;
    q.sz1 = (z - zi) * ihz;
    if (m.weighting == 1) {
        T rj = (T)j * (T)m.hr, rj1 = (T)(j + 1) * (T)m.hr;
        q.sr0 = (rj1 - r) * ihr;
        q.sr1 = (r - rj) * ihr;
    } else {
        // (r_{j+1}^2 - r^2) / (r_{j+1}^2 - r_j^2) with r = x hr: ((j+1)^2 - x^2) / (2j+1)
        T x2 = xr * xr;
        T inv = inv2j1<T>(j);
        q.sr0 = ((T)((j + 1) * (j + 1)) - x2) * inv;
        q.sr1 = (x2 - (T)(j * j)) * inv;
    }
    return q;
}

// ---------------------------------------------------------------------------
// Cross sections (Sec. 2.6): linear interpolation, 1/E law above the table.
// Evaluated with contraction off so that it rounds exactly like the host
// reference arithmetic on identical inputs (decisions depend on it).

__device__ __forceinline__ double xsec_at(const Xsec &x, int k, double eps)
{
#pragma clang fp contract(off)
    const double *sg = x.sigma + (size_t)k * x.ne;
    if (eps >= x.emax) return sg[x.ne - 1] * (x.emax / eps);
    double xx = eps / x.de;
    int j = (int)xx;
    if (j > x.ne - 2) j = x.ne - 2;
    double t = xx - (double)j;
    return sg[j] + t * (sg[j + 1] - sg[j]);
}

// Process chosen by a candidate with uniform u1: the first k with
// u1 * nu_max < sum_{k' <= k} n_gas sigma_k'(eps) g, or -1 (null collision).
__device__ __forceinline__ int choose_process(const Xsec &x, double n_gas, double thr_nu, double eps,
                                           double g)
{
#pragma clang fp contract(off)
    double cum = 0.0;
    for (int k = 0; k < x.nproc; ++k) {
        cum += n_gas * xsec_at(x, k, eps) * g;
        if (thr_nu < cum) return k;
    }
    return -1;
}

// Whether an electron candidate makes a real collision (some process k with
// thr_nu < sum_{k' <= k} n_gas sigma_k'(eps) g, i.e. thr_nu below the total,
// the cumulative sums being non-decreasing): the decision of choose_process,
// bit for bit.  A cheap estimate of the total decides all but a band around
// it: eps/de by a multiplication with 1/de (a few ulp of x, so sigma within
// ~1e-12 of its largest table value) and g by the FP32 square root (within
// 3e-7); outside a band of 1e-6 of the estimate plus Xsec::band_abs (the
// bound of the table error) the exact total lies on the same side.  Inside
// the band the exact evaluation decides.
__device__ __forceinline__ bool electron_real(const Xsec &x, double n_gas, double thr_nu,
                                              double eps, double v2)
{
#pragma clang fp contract(off)
    if (eps < x.emax) {
        const double g = (double)__builtin_amdgcn_sqrtf((float)v2);
        const double xx = eps * x.inv_de;
        int j = (int)xx;
        if (j > x.ne - 2) j = x.ne - 2;
        const double t = xx - (double)j;
        double sT = 0.0;
        for (int k = 0; k < x.nproc; ++k) {
            const double *sg = x.sigma + (size_t)k * x.ne;
            sT += sg[j] + t * (sg[j + 1] - sg[j]);
        }
        const double est = n_gas * sT * g;
        const double band = 1e-6 * est + x.band_abs;
        if (thr_nu < est - band) return true;
        if (thr_nu > est + band) return false;
    }
    return choose_process(x, n_gas, thr_nu, eps, sqrt(v2)) >= 0;
}

__device__ __forceinline__ double energy_ev(double v0, double v1, double v2, double ekin)
{
#pragma clang fp contract(off)
    double v2s = v0 * v0 + v1 * v1 + v2 * v2;
    return v2s * ekin;
}

__device__ __forceinline__ double sumsq3(double a, double b, double c)
{
#pragma clang fp contract(off)
    return a * a + b * b + c * c;
}

// ---------------------------------------------------------------------------
// Collision outcomes (Sec. 2.6) in a precision O of their own.  The decisions
// (candidate, process, the threshold test, and for ions the Maxwellian target
// the relative energy is formed with) are always made in FP64, bit for bit as
// the reference arithmetic; the outcome (scattering angles, the shared energy
// of an ionization, new-particle velocities) is formed in O: FP64 in the FP64
// form, FP32 with the hardware transcendental instructions in the mixed form,
// whose particles hold FP32 velocities anyway.
template <typename O> struct OMath;
template <> struct OMath<double> {
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    // (1 + e)^R
    static __device__ __forceinline__ double pow1p(double e, double R) { return pow(1.0 + e, R); }
    // sine and cosine of 2 pi u
    static __device__ __forceinline__ void sincos_turns(double u, double &s, double &c)
    {
        sincos(kTwoPi * u, &s, &c);
    }
    static __device__ __forceinline__ double log_(double x) { return log(x); }
    static __device__ __forceinline__ double tan_(double x) { return tan(x); }
    static __device__ __forceinline__ double atan_(double x) { return atan(x); }
};
template <> struct OMath<float> {
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float pow1p(float e, float R)
    {
        return __builtin_amdgcn_exp2f(R * __builtin_amdgcn_logf(1.0f + e));
    }
    // the hardware sine and cosine take their argument in turns
    static __device__ __forceinline__ void sincos_turns(float u, float &s, float &c)
    {
        s = __builtin_amdgcn_sinf(u);
        c = __builtin_amdgcn_cosf(u);
    }
    static __device__ __forceinline__ float log_(float x)
    {
        return __builtin_amdgcn_logf(x) * 0.69314718055994531f;
    }
    static __device__ __forceinline__ float tan_(float x) { return tanf(x); }
    static __device__ __forceinline__ float atan_(float x) { return atanf(x); }
};

// Turn unit vector u by polar angle chi (cosine cx) and azimuth 2 pi t about
// itself; azimuth measured from p = (a x u)/|a x u|, a = z (or x if u is within
// ~8 degrees of z), q = u x p.
template <typename O>
__device__ __forceinline__ void turn(O &u0, O &u1, O &u2, O cx, O t)
{
    using M = OMath<O>;
    O px, py, pz;
    if (fabs(u2) < (O)0.99) {
        px = -u1;
        py = u0;
        pz = (O)0;
    } else {
        px = (O)0;
        py = -u2;
        pz = u1;
    }
    O pn = M::sqrt_(px * px + py * py + pz * pz);
    px /= pn;
    py /= pn;
    pz /= pn;
    O qx = u1 * pz - u2 * py;
    O qy = u2 * px - u0 * pz;
    O qz = u0 * py - u1 * px;
    O sx = M::sqrt_(fmax((O)0, (O)1 - cx * cx));
    O sp, cp;
    M::sincos_turns(t, sp, cp);
    O n0 = cx * u0 + sx * (cp * px + sp * qx);
    O n1 = cx * u1 + sx * (cp * py + sp * qy);
    O n2 = cx * u2 + sx * (cp * pz + sp * qz);
    u0 = n0;
    u1 = n1;
    u2 = n2;
}

// Vahedi & Surendra (1995) electron scattering angle, eps in eV.
template <typename O> __device__ __forceinline__ O cos_chi_e(O eps, O R)
{
    if (!(eps > (O)0)) return (O)1 - (O)2 * R;
    O c = ((O)2 + eps - (O)2 * OMath<O>::pow1p(eps, R)) / eps;
    return fmin((O)1, fmax((O)-1, c));
}

// Two standard normals from a uniform pair (Box-Muller) in precision O.
template <typename O> __device__ __forceinline__ void normal2o(O ua, O ub, O &n1, O &n2)
{
    using M = OMath<O>;
    O rad = M::sqrt_((O)-2 * M::log_(ua));
    O sn, cs;
    M::sincos_turns(ub, sn, cs);
    n1 = rad * cs;
    n2 = rad * sn;
}

struct Child {
    double vr, vt, vz;
};

// Outcome of a null-collision candidate (Sec. 2.6; the candidate test itself,
// U0 < P_null with block 0 of the draws, is made by the caller, which passes
// U1 = ub).  Returns the event code (1 null, 2+k process k).  v[] is updated in place; an
// ionization fills the ejected electron and the new ion velocities and sets
// *iz.  Draw blocks: 0 = (candidate, process); electrons: 1 = (chi, phi),
// 2 = (ejected energy, chi_ej), 3 = (phi_ej, -), 4-5 = ion normals;
// ions: 1-2 = target normals, 3 = (cos chi, phi) in the centre of mass.
// O: precision of the outcome (see OMath).
template <typename O>
__device__ __forceinline__ int collide_candidate(const SpeciesK &sp, const Phys &ph, uint64_t id,
                                              uint32_t step, double ub, double &v0, double &v1,
                                              double &v2, int &iz, Child &ce, Child &ci)
{
    using M = OMath<O>;
    iz = 0;
    double thr_nu;
    {
#pragma clang fp contract(off)
        thr_nu = ub * sp.nu_max;
    }
    if (sp.mc_model == 1) {
        double eps = energy_ev(v0, v1, v2, sp.ekin);
        double vm = sqrt(sumsq3(v0, v1, v2));
        int k = choose_process(sp.xs, ph.n_gas, thr_nu, eps, vm);
        if (k < 0) return 1;
        double ex;
        {
#pragma clang fp contract(off)
            ex = eps - sp.xs.thr[k];
        }
        const int kind = sp.xs.kind[k];
        if (kind != 0 && ex < 0.0) return 1;
        O u0 = (O)0, u1 = (O)0, u2 = (O)1;
        if (vm > 0.0) {
            u0 = (O)(v0 / vm);
            u1 = (O)(v1 / vm);
            u2 = (O)(v2 / vm);
        }
        double ra, rb;
        uniform2(ph.seed, sp.s, id, step, 1, ra, rb);
        const O m = (O)sp.m, qe = (O)kE;
        if (kind == 0) {
            const O e = (O)eps;
            O cx = cos_chi_e<O>(e, (O)ra);
            O eps1 = e * ((O)1 - ((O)2 * m / (O)ph.m_gas) * ((O)1 - cx));
            turn<O>(u0, u1, u2, cx, (O)rb);
            O s1 = M::sqrt_((O)2 * eps1 * qe / m);
            v0 = (double)(s1 * u0);
            v1 = (double)(s1 * u1);
            v2 = (double)(s1 * u2);
            return 2 + k;
        }
        const O eo = (O)ex;
        if (kind == 1) {
            O cx = cos_chi_e<O>(eo, (O)ra);
            turn<O>(u0, u1, u2, cx, (O)rb);
            O s1 = M::sqrt_((O)2 * eo * qe / m);
            v0 = (double)(s1 * u0);
            v1 = (double)(s1 * u1);
            v2 = (double)(s1 * u2);
            return 2 + k;
        }
        double rc, rd, re, rf;
        uniform2(ph.seed, sp.s, id, step, 2, rc, rd);
        uniform2(ph.seed, sp.s, id, step, 3, re, rf);
        const O B = (O)sp.xs.ejB;
        O eej = B * M::tan_((O)rc * M::atan_(eo / ((O)2 * B)));
        O esc = eo - eej;
        O s0 = u0, s1_ = u1, s2 = u2;
        turn<O>(s0, s1_, s2, cos_chi_e<O>(esc, (O)ra), (O)rb);
        O e0 = u0, e1 = u1, e2 = u2;
        turn<O>(e0, e1, e2, cos_chi_e<O>(eej, (O)rd), (O)re);
        O vs = M::sqrt_((O)2 * esc * qe / m);
        O ve = M::sqrt_((O)2 * eej * qe / m);
        v0 = (double)(vs * s0);
        v1 = (double)(vs * s1_);
        v2 = (double)(vs * s2);
        ce.vr = (double)(ve * e0);
        ce.vt = (double)(ve * e1);
        ce.vz = (double)(ve * e2);
        double g1a, g1b, g2a, g2b;
        O n1, n2, n3, n4;
        uniform2(ph.seed, sp.s, id, step, 4, g1a, g1b);
        uniform2(ph.seed, sp.s, id, step, 5, g2a, g2b);
        normal2o<O>((O)g1a, (O)g1b, n1, n2);
        normal2o<O>((O)g2a, (O)g2b, n3, n4);
        const O vth = (O)ph.vth_gas;
        ci.vr = (double)(vth * n1);
        ci.vt = (double)(vth * n2);
        ci.vz = (double)(vth * n3);
        iz = 1;
        return 2 + k;
    }
    if (sp.mc_model == 2) {
        // the target's velocity decides the relative energy: FP64 always
        double g1a, g1b, g2a, g2b, n1, n2, n3, n4;
        uniform2(ph.seed, sp.s, id, step, 1, g1a, g1b);
        uniform2(ph.seed, sp.s, id, step, 2, g2a, g2b);
        normal2(g1a, g1b, n1, n2);
        normal2(g2a, g2b, n3, n4);
        double t0 = ph.vth_gas * n1, t1 = ph.vth_gas * n2, t2 = ph.vth_gas * n3;
        double g0, gg1, gg2;
        {
#pragma clang fp contract(off)
            g0 = v0 - t0;
            gg1 = v1 - t1;
            gg2 = v2 - t2;
        }
        double g2s = sumsq3(g0, gg1, gg2);
        double eps;
        {
#pragma clang fp contract(off)
            eps = g2s * sp.ekin;
        }
        double gm = sqrt(g2s);
        int k = choose_process(sp.xs, ph.n_gas, thr_nu, eps, gm);
        if (k < 0) return 1;
        double ra, rb;
        uniform2(ph.seed, sp.s, id, step, 3, ra, rb);
        const O cx = (O)1 - (O)2 * (O)ra;
        const O sx = M::sqrt_(fmax((O)0, (O)1 - cx * cx));
        O sp_, cp_;
        M::sincos_turns((O)rb, sp_, cp_);
        const O Mg = (O)ph.m_gas, mi = (O)sp.m;
        const O fcm = Mg / (mi + Mg), gmo = (O)gm;
        const O d0 = sx * cp_, d1 = sx * sp_, d2 = cx;
        v0 = (double)((mi * (O)v0 + Mg * (O)t0) / (mi + Mg) + fcm * gmo * d0);
        v1 = (double)((mi * (O)v1 + Mg * (O)t1) / (mi + Mg) + fcm * gmo * d1);
        v2 = (double)((mi * (O)v2 + Mg * (O)t2) / (mi + Mg) + fcm * gmo * d2);
        return 2 + k;
    }
    return 0;
}

// Node k of the deposit: n_s = N_s / V, rho = sum q n, chi = sum q^2 n dt_s^2 /
// (2 m eps0) (the implicit susceptibility of Sec. 2.1 in SI, dt_s the
// species' time step; the ion term only when the ions move in the coming
// step), eps = 1 + chi, f = rho / eps0; returns eps.  A negative accumulator means the fixed-point
// range overflowed.
__device__ __forceinline__ double finalize_node(const GridArgs &g, int k)
{
    long long a0 = (long long)g.acc0[k], a1 = (long long)g.acc1[k];
    if (a0 < 0 || a1 < 0) atomicOr(g.status, kStNumeric);
    double n0 = ((double)a0 * g.quantum0) / g.vol[k];
    double n1 = ((double)a1 * g.quantum1) / g.vol[k];
    g.dens0[k] = n0;
    g.dens1[k] = n1;
    double rho = 0.0, chi = 0.0;
    rho += g.q0 * n0;
    if (g.friedman) {
        // Friedman damping: the implicit coefficient theta/2 instead of 1/2
        double x = g.q0 * g.q0 * n0 * g.dt * g.dt / (2.0 * g.m0 * kEps0);
        x *= g.theta;
        chi += x;
    } else {
        chi += g.q0 * g.q0 * n0 * g.dt * g.dt / (2.0 * g.m0 * kEps0);
    }
    rho += g.q1 * n1;
    if (g.ion_chi) {
        if (g.friedman) {
            double x = g.q1 * g.q1 * n1 * g.dt1 * g.dt1 / (2.0 * g.m1 * kEps0);
            x *= g.theta;
            chi += x;
        } else {
            chi += g.q1 * g.q1 * n1 * g.dt1 * g.dt1 / (2.0 * g.m1 * kEps0);
        }
    }
    g.rho[k] = rho;
    g.chi[k] = chi;
    const double eps = 1.0 + chi;
    g.eps[k] = eps;
    if (g.eps32) g.eps32[k] = (float)eps;
    g.f[k] = rho / kEps0;
    if (g.zero_acc) {
        g.acc0w[k] = 0;
        if (!g.keep1) g.acc1w[k] = 0;
    }
    return eps;
}

// ---------------------------------------------------------------------------
// Wavefront scans (a chunk of particles is one 64-lane wavefront).

__device__ __forceinline__ int lane_rank(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Rank of this lane among the lanes with f set (lane order), and their number.
__device__ __forceinline__ int wave_rank(bool f, int &total)
{
    unsigned long long m = __ballot(f);
    total = __popcll(m);
    return lane_rank(m);
}

// Exclusive prefix over the wavefront of a non-negative int, and the total.
__device__ __forceinline__ int wave_excl_sum(int v, int &total)
{
    const int lane = threadIdx.x & 63;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

// Exclusive prefix of a non-negative int over the block, and its total.
__device__ __forceinline__ int block_excl_sum(int v, int &total, int *sh)
{
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
    int wt;
    int x = wave_excl_sum(v, wt);
    if (lane == 0) sh[wv] = wt;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        int c = sh[w];
        before += w < wv ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return before + x;
}

// Round-to-nearest-even of |x| < 2^51 to an integer, exactly: adding 1.5*2^52
// leaves the integer in the low mantissa bits.
__device__ __forceinline__ long long round_fixed(double x)
{
    const double magic = 6755399441055744.0;
    double y = x + magic;
    return (long long)(__double_as_longlong(y) - __double_as_longlong(magic));
}

// ---------------------------------------------------------------------------
// Deposit of one particle (Sec. 2.4): N_ij += w S_z S_r, accumulated in fixed
// point (quantum = w_ref 2^-bits) so that the sum does not depend on order.
// Contributions must stay below 2^51 quanta (a weight below 2^(51-bits)
// w_ref); a larger one is flagged and the step reports RZPIC_ENUMERIC.
// The four nodes of the cell sit at acc[g], acc[g + 1], acc[g + stride] and
// acc[g + stride + 1] (stride nr for a whole grid, the row length of a window).
template <typename T>
__device__ __forceinline__ void deposit4_at(unsigned long long *acc, int g, int stride,
                                            const W4<T> &q, double w, double inv_quantum,
                                            int32_t *status)
{
    const double ws = w * inv_quantum;
    if (!(fabs(ws) < 0x1p51)) atomicOr(status, kStNumeric);
    const double a = (double)q.sz0 * (double)q.sr0, b = (double)q.sz0 * (double)q.sr1;
    const double c = (double)q.sz1 * (double)q.sr0, d = (double)q.sz1 * (double)q.sr1;
    __hip_atomic_fetch_add(acc + g, (unsigned long long)round_fixed(ws * a), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(acc + g + 1, (unsigned long long)round_fixed(ws * b),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(acc + g + stride, (unsigned long long)round_fixed(ws * c),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(acc + g + stride + 1, (unsigned long long)round_fixed(ws * d),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// FP32 particles: each contribution is formed in FP32 and rounded to a
// 32-bit integer number of quanta (below 1.5 2^30: with the mixed form's
// default quantum w_ref 2^-26, weights up to 24 w_ref; a larger one is
// flagged), then added to the same 64-bit accumulators.  The sum stays
// exact and order-free; the contribution carries the FP32 rounding of the
// particle state it comes from.
template <>
__device__ __forceinline__ void deposit4_at<float>(unsigned long long *acc, int g, int stride,
                                                   const W4<float> &q, double w,
                                                   double inv_quantum, int32_t *status)
{
    const float ws = (float)w * (float)inv_quantum;
    if (!(fabsf(ws) < 0x1.8p30f)) atomicOr(status, kStNumeric);
    const float a = q.sz0 * q.sr0, b = q.sz0 * q.sr1;
    const float c = q.sz1 * q.sr0, d = q.sz1 * q.sr1;
    const long long qa = (int)__builtin_rintf(ws * a), qb = (int)__builtin_rintf(ws * b);
    const long long qc = (int)__builtin_rintf(ws * c), qd = (int)__builtin_rintf(ws * d);
    __hip_atomic_fetch_add(acc + g, (unsigned long long)qa, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(acc + g + 1, (unsigned long long)qb, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(acc + g + stride, (unsigned long long)qc, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(acc + g + stride + 1, (unsigned long long)qd, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// FP32 particles into a 32-bit copy of the whole grid (a block's LDS copy):
// the same int32 contributions as above, added to 32-bit accumulators.  Each
// add returns the value it replaced, so an add that wraps past 2^32 (or, for
// a negative contribution, below 0) is known exactly, and the 2^32 quanta it
// carries go to the 64-bit accumulator of the same node in gacc.  The sum,
// lo + carries 2^32, is the integer the 64-bit accumulators would hold.
__device__ __forceinline__ void lds32_add(uint32_t *lo, unsigned long long *gacc, int g, int v)
{
    const uint32_t old =
        __hip_atomic_fetch_add(lo + g, (uint32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const uint32_t now = old + (uint32_t)v;
    if (v >= 0 ? now < old : now > old)
        atomicAdd(gacc + g, v >= 0 ? 0x100000000ull : 0xFFFFFFFF00000000ull);
}

__device__ __forceinline__ void deposit4_lds32(uint32_t *lo, unsigned long long *gacc, int g,
                                               int stride, const W4<float> &q, double w,
                                               double inv_quantum, int32_t *status)
{
    const float ws = (float)w * (float)inv_quantum;
    if (!(fabsf(ws) < 0x1.8p30f)) atomicOr(status, kStNumeric);
    const float a = q.sz0 * q.sr0, b = q.sz0 * q.sr1;
    const float c = q.sz1 * q.sr0, d = q.sz1 * q.sr1;
    const int qa = (int)__builtin_rintf(ws * a), qb = (int)__builtin_rintf(ws * b);
    const int qc = (int)__builtin_rintf(ws * c), qd = (int)__builtin_rintf(ws * d);
    lds32_add(lo, gacc, g, qa);
    lds32_add(lo, gacc, g + 1, qb);
    lds32_add(lo, gacc, g + stride, qc);
    lds32_add(lo, gacc, g + stride + 1, qd);
}

}  // namespace rz
