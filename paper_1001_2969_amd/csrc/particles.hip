// Particle kernels: the fused pass of the D1 cycle (gather, final push,
// Monte Carlo, first push, deposit), initialisation and the pass over staged
// new particles.
#include "device.h"
#include <type_traits>

namespace rz {

template <typename T>
__device__ __forceinline__ void deposit4(unsigned long long *acc, const Mesh &m, const W4<T> &q,
                                         double w, double inv_quantum, int32_t *status)
{
    deposit4_at<T>(acc, q.g, m.nr, q, w, inv_quantum, status);
}

__device__ __forceinline__ void tally_add(unsigned long long *t, int b, double w, double inv_q)
{
    atomicAdd(t + b, (unsigned long long)round_fixed(w * inv_q));
}

template <typename T> struct PState {
    T r, z, vr, vt, vz, ar, az, w;
    T at;  // a_theta, global X-Y-Z push only
};

// Absorption at the electrodes (z <= 0, z >= L) and the wall (r >= R).
template <typename T> __device__ __forceinline__ int boundary_of(const PState<T> &s, const Phys &ph)
{
    if (s.z <= (T)0) return 0;
    if (s.z >= (T)ph.L) return 1;
    if (s.r >= (T)ph.R) return 2;
    return -1;
}

// First push in the local X-Y frame plus rotation (Sec. 2.3).  Local form:
// a_theta = 0.  Global X-Y-Z form (xyz): a_theta kicks v_theta and the damped
// acceleration turns with the frame (the Cartesian push seen from the
// particle's meridian plane).
// kn: the factor of the stored acceleration, 1/2 for D1 (abar_{n-1}/2), 1
// for Friedman damping (the stored known part B of abar_n).
template <typename T>
__device__ __forceinline__ void first_push(PState<T> &s, T dt, bool xyz, T kn)
{
    // no contraction: every kernel instance that inlines the push rounds alike
#pragma clang fp contract(off)
    const T half = (T)0.5;
    T vx = s.vr + kn * s.ar * dt;
    T vy = xyz ? s.vt + half * s.at * dt : s.vt;
    T x = s.r + vx * dt;
    T y = vy * dt;
    T vz = s.vz + kn * s.az * dt;
    T z = s.z + vz * dt;
    T rn = sqrt(x * x + y * y);
    T c = (T)1, sn = (T)0;
    if (rn > (T)0) {
        if constexpr (std::is_same<T, float>::value) {
            // FP32 particles: one hardware reciprocal for both cosines (the
            // radius keeps the correctly rounded square root; only the
            // velocities and a_r see the extra ulp)
            const float inv = __builtin_amdgcn_rcpf(rn);
            c = x * inv;
            sn = y * inv;
        } else {
            c = x / rn;
            sn = y / rn;
        }
    }
    s.r = rn;
    s.z = z;
    s.vr = vx * c + vy * sn;
    s.vt = -vx * sn + vy * c;
    s.vz = vz;
    if (xyz) {
        const T ar = s.ar, at = s.at;
        s.ar = ar * c + at * sn;
        s.at = -ar * sn + at * c;
    } else {
        s.ar = s.ar * c;
    }
}

// Gather of E at (r, z) with the deposit weights (any position: the cell is
// clamped to the mesh).
template <typename T>
__device__ __forceinline__ void gather_E(const Mesh &m, const typename Vec2<T>::type *E2, T r, T z,
                                         T &Er, T &Ez)
{
    W4<T> q = weights<T>(m, r, z);
    auto e00 = E2[q.g], e01 = E2[q.g + 1], e10 = E2[q.g + m.nr], e11 = E2[q.g + m.nr + 1];
    T w00 = q.sz0 * q.sr0, w01 = q.sz0 * q.sr1, w10 = q.sz1 * q.sr0, w11 = q.sz1 * q.sr1;
    Er = w00 * e00.x + w01 * e01.x + w10 * e10.x + w11 * e11.x;
    Ez = w00 * e00.y + w01 * e01.y + w10 * e10.y + w11 * e11.y;
}

// Final push with the gathered field, the damped-acceleration update and the
// axis rule (Sec. 2.1, 2.3).
// Global X-Y-Z form (xyz): E has no theta component at the particle, so a_theta
// is damped by the same average, and a particle pushed through the axis goes
// on at the other side (the local frame turns by pi) instead of the axis rule.
// Friedman damping (fr, fc = theta/2, local push): abar_n = fc a + B, and
// the particle keeps the next step's known part
// B' = (1 - fc) ((1 - fc) a + fc abar_n) in (ar, az), with the same axis rule.
template <typename T>
__device__ __forceinline__ void final_push(PState<T> &s, T Er, T Ez, T k1, T k2, T qm, bool xyz,
                                           bool fr = false, T fc = (T)0)
{
#pragma clang fp contract(off)
    T r = s.r + k1 * Er;
    T z = s.z + k1 * Ez;
    T vr = s.vr + k2 * Er;
    T vz = s.vz + k2 * Ez;
    if (fr) {
        const T c1 = (T)1 - fc, aEr = qm * Er, aEz = qm * Ez;
        const T abr = fc * aEr + s.ar, abz = fc * aEz + s.az;
        T br = c1 * (c1 * aEr + fc * abr);
        const T bz = c1 * (c1 * aEz + fc * abz);
        if (r < (T)0) {
            r = -r;
            vr = fabs(vr);
            br = fabs(br);
        }
        s.r = r;
        s.z = z;
        s.vr = vr;
        s.vz = vz;
        s.ar = br;
        s.az = bz;
        return;
    }
    T ar = (T)0.5 * (qm * Er + s.ar);
    T az = (T)0.5 * (qm * Ez + s.az);
    if (xyz) {
        T at = (T)0.5 * s.at, vt = s.vt;
        if (r < (T)0) {
            r = -r;
            vr = -vr;
            vt = -vt;
            ar = -ar;
            at = -at;
        }
        s.vt = vt;
        s.at = at;
    } else if (r < (T)0) {
        r = -r;
        vr = fabs(vr);
        ar = fabs(ar);
    }
    s.r = r;
    s.z = z;
    s.vr = vr;
    s.vz = vz;
    s.ar = ar;
    s.az = az;
}

// Element i of a particle array through a 32-bit byte offset.  Capacities
// stay below 2^29 (rzpic_bind_species), so i * sizeof(T) fits in 32 bits:
// the access takes the array base in scalar registers plus one offset that
// every array of the record shares, with no 64-bit address arithmetic.
template <typename T> __device__ __forceinline__ T &el(T *base, int64_t i)
{
    return *(T *)((char *)base + (uint32_t)((uint32_t)i * (uint32_t)sizeof(T)));
}

template <typename T> __device__ __forceinline__ PState<T> load(const Parts<T> &p, int64_t i)
{
    return PState<T>{el(p.r, i), el(p.z, i), el(p.vr, i), el(p.vt, i), el(p.vz, i),
                     el(p.ar, i), el(p.az, i), el(p.w, i), p.at ? el(p.at, i) : (T)0};
}

// load() with the a_theta array's presence fixed at compile time: no load
// behind a branch, so the compiler's memory-counter waits stay exact across a
// loop that keeps loads in flight from one iteration to the next.
template <typename T, bool X> __device__ __forceinline__ PState<T> load_x(const Parts<T> &p, int64_t i)
{
    return PState<T>{el(p.r, i), el(p.z, i), el(p.vr, i), el(p.vt, i), el(p.vz, i),
                     el(p.ar, i), el(p.az, i), el(p.w, i), X ? el(p.at, i) : (T)0};
}

template <typename T>
__device__ __forceinline__ void store(const Parts<T> &p, int64_t i, const PState<T> &s, bool w)
{
    el(p.r, i) = s.r;
    el(p.z, i) = s.z;
    el(p.vr, i) = s.vr;
    el(p.vt, i) = s.vt;
    el(p.vz, i) = s.vz;
    el(p.ar, i) = s.ar;
    el(p.az, i) = s.az;
    if (p.at) el(p.at, i) = s.at;
    if (w) el(p.w, i) = s.w;
}

// One pass over the particles of a species.  Each wavefront processes chunks
// of 64 consecutive particles (no block barrier in the loop); MODE selects the
// steps (M_* bits).  With M_MC a particle that draws U0 < P_null is a
// candidate: it keeps its final-pushed state, joins the candidate list and
// skips the rest of the pass (the collision kernel takes over).  The merged
// form records each chunk's dead particles as a lane mask.
//
// Deposit targets: by default global atomics on the grid of the species
// (chunks grid-strided over the wavefronts).  M_LDS: the block deposits into
// its own LDS copy of the whole grid, written out once at the end to its
// slice.  M_TILE: the block takes a contiguous range of particles (planned at
// the last tile sort, so they sit in one or two tiles) and deposits into an
// LDS window of those tiles plus a drift margin; a particle outside the
// window, and the chunks beyond the planned ranges, go to global atomics.  The
// window is added to the grid once at the end.
//
// The body takes the block's index lb among the gb blocks of its species, so
// that one launch can run the passes of both species side by side.
template <typename T, int MODE>
__device__ __forceinline__ void pass_body(const PassArgs<T> &a, int lb, int gb)
{
    extern __shared__ unsigned long long lds_acc[];
    __shared__ unsigned long long sh_cand;
    __shared__ int sh_bucket;

    const Mesh &m = a.mesh;
    const int64_t n = a.cnt->n;
    const int64_t nch = (n + kChunk - 1) / kChunk;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int64_t wave = ((int64_t)lb * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gb * blockDim.x) >> 6;
    const T dt = (T)a.sp.dt;
    const T k1 = (T)a.sp.k1, k2 = (T)a.sp.k2, qm = (T)a.sp.qm;
    const bool xyz = a.p.at != nullptr;  // global X-Y-Z push (a_theta kept)
    constexpr bool kLds = (MODE & M_LDS) != 0;
    constexpr bool kTile = (MODE & M_TILE) != 0;
    constexpr bool kDep = (MODE & M_DEP) != 0;
    constexpr bool kMc = (MODE & M_MC) != 0;
    // FP32 particles deposit into a 32-bit LDS grid (deposit4_lds32)
    constexpr bool kNarrow = kLds && std::is_same<T, float>::value;
    uint32_t *const lds32 = (uint32_t *)lds_acc;
    const bool mc_on = kMc && a.sp.mc_model != 0;
    unsigned long long *dep = a.acc;

    if (kMc && a.crec && lb == 0 && threadIdx.x == 0) a.crec->n_parent = n;
    if (kMc && threadIdx.x == 0) {
        sh_cand = 0;
        sh_bucket = 0;
    }
    if (a.psteps && lb == 0 && threadIdx.x == 0) atomicAdd(a.psteps, (unsigned long long)n);
    if (kLds) {
        if (kNarrow)
            for (int g = threadIdx.x; g < m.nn; g += blockDim.x) lds32[g] = 0;
        else
            for (int g = threadIdx.x; g < m.nn; g += blockDim.x) lds_acc[g] = 0;
        dep = lds_acc;
    }
    // tiled form: planned chunks per block and this block's window
    int64_t q = 0;
    int4 win = make_int4(0, 0, 0, 0);
    if (kTile) {
        if (a.tile_pb && a.tile_nb == gb) {
            q = tiled_q(*a.tile_pb);
            win = a.tile_win[lb];
        }
        if (win.z < 2 || win.w < 2 || win.z * win.w > kWinNodes) win = make_int4(0, 0, 0, 0);
        for (int g = threadIdx.x; g < win.z * win.w; g += blockDim.x) lds_acc[g] = 0;
    }
    // cells inside the window: 0 <= i - i0 < ci, 0 <= j - j0 < cj (none if empty)
    const unsigned ci = win.z > 1 ? (unsigned)(win.z - 1) : 0u;
    const unsigned cj = win.w > 1 ? (unsigned)(win.w - 1) : 0u;
    if (kLds || kTile || kMc) __syncthreads();

    // candidates of this block go to its own bucket of the candidate list
    const int64_t bchunks =
        kTile ? q + tiled_q2(nch, gb, q) : ((nch + nwaves - 1) / nwaves) * wpb;
    int32_t *bucket = a.ch.cand + (int64_t)lb * bchunks * kChunk;

    // The rest of the cycle of chunk c from its loaded state s, identity pid
    // and gathered field (Er, Ez).
    auto chunk = [&](int64_t c, PState<T> s, uint64_t pid, T Er, T Ez, auto &&after_mc) {
        const int64_t pi = c * kChunk + lane;
        const bool valid = pi < n;
        bool live = valid;
        if ((MODE & M_MARK) && valid) live = s.w >= (T)0;
        bool died = false, moved = false;
        if ((MODE & M_FINAL) && live) {
            final_push<T>(s, Er, Ez, k1, k2, qm, xyz, a.phys.friedman != 0, (T)a.phys.fc);
            moved = true;
            int b = boundary_of(s, a.phys);
            if (b >= 0) {
                tally_add(a.tally, b, (double)s.w, a.sp.inv_quantum);
                live = false;
                died = true;
            }
        }
        // Null-collision candidate test; for electrons (target at rest) the
        // process choice is cheap and a null event is settled here, so only
        // real collisions (and every ion candidate) go to the bucket.
        bool cand = false;
        if (kMc) {
            int code = 0;
            bool tested = false;
            if (live && mc_on) {
                uint64_t ua, ub;
                draw_u52(a.phys.seed, a.sp.s, pid, a.step, 0, ua, ub);
                if (is_candidate(ua, a.sp.cand_u52)) {
                    tested = true;
                    cand = true;
                    if (a.sp.mc_model == 1) {
                        double thr_nu, eps;
                        const double vv = sumsq3((double)s.vr, (double)s.vt, (double)s.vz);
                        {
#pragma clang fp contract(off)
                            thr_nu = u52_unit(ub) * a.sp.nu_max;
                            eps = vv * a.sp.ekin;  // energy_ev, term for term
                        }
                        if (!electron_real(a.sp.xs, a.phys.n_gas, thr_nu, eps, vv)) {
                            cand = false;
                            code = 1;
                        }
                    }
                }
            }
            if (valid && a.ev) a.ev[pi] = (uint8_t)code;
            int ntested;
            wave_rank(tested, ntested);
            if (lane == 0 && ntested) atomicAdd(&sh_cand, (unsigned long long)ntested);
            int tot;
            int r = wave_rank(cand, tot);
            int base = 0;
            if (tot > 0) {
                if (lane == 0) base = atomicAdd(&sh_bucket, tot);
                base = __shfl(base, 0, 64);
            }
            if (cand) bucket[base + r] = (int32_t)pi;
            if (lane == 0) {
                a.ch.ev[c] = 0;
                a.ch.se[c] = 0;
                a.ch.si[c] = 0;
            }
        }
        after_mc();
        if ((MODE & M_FIRST) && live && !cand) {
            first_push<T>(s, dt, xyz, a.phys.friedman ? (T)1 : (T)0.5);
            moved = true;
            int b = boundary_of(s, a.phys);
            if (b >= 0) {
                tally_add(a.tally, b, (double)s.w, a.sp.inv_quantum);
                live = false;
                died = true;
            }
        }
        if (kDep && live && !cand) {
            const W4<T> w4 = weights<T>(m, s.r, s.z);
            if (kTile) {
                const int li = w4.i - win.x, lj = w4.j - win.y;
                if ((unsigned)li < ci && (unsigned)lj < cj)
                    deposit4_at<T>(lds_acc, li * win.w + lj, win.w, w4, (double)s.w,
                                   a.sp.inv_quantum, a.status);
                else
                    deposit4<T>(a.acc, m, w4, (double)s.w, a.sp.inv_quantum, a.status);
            } else if constexpr (kNarrow) {
                deposit4_lds32(lds32, a.acc, w4.g, m.nr, w4, (double)s.w, a.sp.inv_quantum,
                               a.status);
            } else {
                deposit4<T>(dep, m, w4, (double)s.w, a.sp.inv_quantum, a.status);
            }
        }
        if (valid) {
            if ((MODE & M_MARK) && died) el(a.p.w, pi) = (T)-1;
            else if (live && moved) store(a.p, pi, s, false);
        }
        if (MODE & M_LISTS) {
            unsigned long long dm = __ballot(died);
            if (lane == 0) a.ch.dead[c] = dm;
        }
    };

    // kUnroll chunks per iteration, c, c + step, ... (those below end): the
    // loads and field gathers of all of them are in flight together before
    // any is pushed.  Loads are unconditional (an index past n reads particle
    // 0 and is discarded), so no branch separates them.  Two chunks pay off
    // where the memory system has the most requests to hide (the tiled and
    // global forms, at full occupancy); the whole-grid LDS form, whose
    // resident wavefronts its LDS limits, measured best with one.
    constexpr int kUnroll = kLds ? 1 : 2;
    auto group = [&](int64_t c, int64_t step, int64_t end) {
        int64_t cc[kUnroll];
        PState<T> s[kUnroll];
        uint64_t pid[kUnroll];
        T Er[kUnroll], Ez[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            cc[u] = c + u * step < end ? c + u * step : -1;
            const int64_t pi = cc[u] * kChunk + lane;
            const int64_t pl = cc[u] >= 0 && pi < n ? pi : 0;
            s[u] = load(a.p, pl);
            pid[u] = kMc ? el(a.p.id, pl) : 0;
            Er[u] = Ez[u] = (T)0;
        }
        if (MODE & M_FINAL) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                gather_E<T>(m, a.E2, s[u].r, s[u].z, Er[u], Ez[u]);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (cc[u] >= 0) chunk(cc[u], s[u], pid[u], Er[u], Ez[u], [] {});
    };
    if (kTile) {
        // the planned range, then this block's share of the chunks beyond
        const int wib = threadIdx.x >> 6;
        const int64_t c0 = (int64_t)lb * q;
        const int64_t c1 = c0 + q < nch ? c0 + q : nch;
        for (int64_t c = c0 + wib; c < c1; c += kUnroll * wpb) group(c, wpb, c1);
        const int64_t q2 = tiled_q2(nch, gb, q);
        const int64_t d0 = (int64_t)gb * q + (int64_t)lb * q2;
        const int64_t d1 = d0 + q2 < nch ? d0 + q2 : nch;
        for (int64_t c = d0 + wib; c < d1; c += kUnroll * wpb) group(c, wpb, d1);
    } else if (kLds) {
        // Software pipeline: the next chunk's particle loads are issued after
        // this chunk's Monte Carlo test (whose cross-section loads would
        // otherwise wait for them) and fly during its first push, deposit and
        // stores.  The loads are unconditional (past the end they read
        // particle 0, unused) and the a_theta choice is a compile-time
        // branch: a load behind a branch would make the compiler wait for
        // every load in flight.
        auto pipeline = [&](auto xyz_c) {
            constexpr bool X = decltype(xyz_c)::value;
            auto fetch = [&](int64_t cc, PState<T> &st, uint64_t &id) {
                const int64_t pi = cc * kChunk + lane;
                const int64_t pl = cc < nch && pi < n ? pi : 0;
                st = load_x<T, X>(a.p, pl);
                id = kMc ? el(a.p.id, pl) : 0;
            };
            PState<T> sn;
            uint64_t pn;
            fetch(wave, sn, pn);
            for (int64_t c = wave; c < nch; c += nwaves) {
                const PState<T> s = sn;
                const uint64_t pid = pn;
                T Er = (T)0, Ez = (T)0;
                if (MODE & M_FINAL) gather_E<T>(m, a.E2, s.r, s.z, Er, Ez);
                chunk(c, s, pid, Er, Ez, [&] {
                    // after this chunk's loads in issue order
                    __builtin_amdgcn_sched_barrier(0);
                    fetch(c + nwaves, sn, pn);
                    __builtin_amdgcn_sched_barrier(0);
                });
            }
        };
        if (xyz)
            pipeline(std::true_type{});
        else
            pipeline(std::false_type{});
    } else {
        for (int64_t c = wave; c < nch; c += kUnroll * nwaves) group(c, nwaves, nch);
    }
    if (kMc) {
        __syncthreads();
        if (threadIdx.x == 0) {
            if (lb < a.nbuckets) a.ch.ncand[lb] = sh_bucket;
            if (sh_cand) atomicAdd(a.mcstat, sh_cand);
        }
    }
    if (kLds) {
        __syncthreads();
        if (kNarrow) {
            uint32_t *out = (uint32_t *)a.slices + (size_t)lb * slice_stride(m.nn, 1);
            for (int g = threadIdx.x; g < m.nn; g += blockDim.x) out[g] = lds32[g];
        } else {
            unsigned long long *out = (unsigned long long *)a.slices + (size_t)lb * m.nn;
            for (int g = threadIdx.x; g < m.nn; g += blockDim.x) out[g] = lds_acc[g];
        }
    }
    if (kTile) {
        __syncthreads();
        for (int g = threadIdx.x; g < win.z * win.w; g += blockDim.x) {
            const unsigned long long v = lds_acc[g];
            if (v) {
                const int i = g / win.w, j = g - i * win.w;
                atomicAdd(a.acc + (size_t)(win.x + i) * m.nr + win.y + j, v);
            }
        }
    }
}

template <typename T, int MODE> __global__ __launch_bounds__(1024) void k_pass(PassArgs<T> a)
{
    pass_body<T, MODE>(a, blockIdx.x, gridDim.x);
}

// The arguments of the first (second = false) or second species of a
// two-species launch, whose argument block holds the second species'
// arguments right after the first's.  They are read at a block-uniform byte
// offset that an opaque scalar move hides from the compiler, so that one
// copy of a body serves both species and holds one set of arguments in
// scalar registers.  Written as two inlined calls (one per species), the
// second copy has its arguments loaded ahead and spilled to vector lanes,
// and re-reads them with v_readlane in its loop; as one call on a selected
// reference the compiler selects between both sets, with the same result.
// The collision kernel takes its arguments this way (1.2 us faster in the
// mixed form, 2.6 us in FP64; its VGPRs 133 -> 98 in the mixed form).
template <typename T>
__device__ __forceinline__ const PassArgs<T> &species_args(const PassArgs<T> &first, bool second)
{
    uint32_t off = second ? (uint32_t)sizeof(PassArgs<T>) : 0u;
    asm volatile("s_mov_b32 %0, %1" : "=s"(off) : "s"(off));
    return *(const PassArgs<T> *)((const char *)&first + off);
}

// Both species in one launch: blocks [0, b0) take species 0, the rest species 1.
template <typename T> struct Pass2Args {
    PassArgs<T> a0, a1;
    int b0;
};

template <typename T, int MODE> __device__ __forceinline__ void pass2_body(const Blk &k, const Pass2Args<T> &a)
{
    // one inlined copy per species: measured a little faster than one copy
    // on species_args (below), although the second copy here re-reads
    // spilled scalar registers with v_readlane in its loop
    if (k.x < a.b0) pass_body<T, MODE>(a.a0, k.x, a.b0);
    else pass_body<T, MODE>(a.a1, k.x - a.b0, k.nx - a.b0);
}

// Collision kernel over the candidate list (any order: every result below is
// keyed by the particle index, combined with order-free integer atomics).
// Applies the outcome (Sec. 2.6), records events and new particles in the
// chunk masks and the staging slot of the parent, and with M_FIRST finishes
// the cycle of the candidate and its new particles (first push, absorption,
// deposit).
template <typename T, int MODE>
__device__ __forceinline__ void collide_body(const PassArgs<T> &a, int lb, int gb)
{
    extern __shared__ unsigned long long lds_acc[];
    __shared__ unsigned long long sh_stat[1 + kMaxProc];
    const Mesh &m = a.mesh;
    constexpr bool kLds = (MODE & M_LDS) != 0;
    constexpr bool kFirst = (MODE & M_FIRST) != 0;
    const T dt = (T)a.sp.dt;
    const bool xyz = a.p.at != nullptr;  // global X-Y-Z push (a_theta kept)
    unsigned long long *dep = a.acc;
    if (threadIdx.x < 1 + kMaxProc) sh_stat[threadIdx.x] = 0;
    if (kLds) {
        for (int g = threadIdx.x; g < m.nn; g += blockDim.x) lds_acc[g] = 0;
        dep = lds_acc;
    }
    __syncthreads();
    // buckets of the pass blocks; R wavefronts share a bucket (segments of 64)
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)lb * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gb * blockDim.x) >> 6;
    const int64_t nch = (a.cnt->n + kChunk - 1) / kChunk;
    const int64_t NB = a.nbuckets;
    const int64_t pass_waves = NB * a.bucket_waves;
    int64_t bchunks;
    if (a.tiled) {
        const int64_t q = a.tile_pb && a.tile_nb == NB ? tiled_q(*a.tile_pb) : 0;
        bchunks = q + tiled_q2(nch, (int)NB, q);
    } else {
        bchunks = ((nch + pass_waves - 1) / pass_waves) * a.bucket_waves;
    }
    const int64_t bsize = bchunks * kChunk;
    const int64_t R = nwaves >= NB ? nwaves / NB : 1;
    for (int64_t t = wave; t < NB * R; t += nwaves) {
      const int64_t b = t % NB, seg = t / NB;
      const int nb = a.ch.ncand[b];
      for (int64_t j = seg * kChunk + lane; j < nb; j += R * kChunk) {
        const int64_t pi = a.ch.cand[b * bsize + j];
        const int64_t c = pi >> 6;
        const unsigned long long bit = 1ull << (pi & 63);
        PState<T> s = load(a.p, pi);
        const uint64_t id = a.p.id[pi];
        double ua, ub;
        uniform2(a.phys.seed, a.sp.s, id, a.step, 0, ua, ub);
        double v0 = s.vr, v1 = s.vt, v2 = s.vz;
        int iz = 0;
        Child che{}, chi{};
        int ev = collide_candidate<T>(a.sp, a.phys, id, a.step, ub, v0, v1, v2, iz, che, chi);
        if (ev >= 2) {
            s.vr = (T)v0;
            s.vt = (T)v1;
            s.vz = (T)v2;
            atomicAdd(&sh_stat[1 + ev - 2], 1ull);
        }
        if (a.ev) a.ev[pi] = (uint8_t)ev;
        PState<T> ne{}, ni{};
        bool ne_live = false, ni_live = false;
        if (iz) {
            // new electron and ion at the parent's position with its weight;
            // the ion's damped acceleration scaled by the charge-to-mass ratios
            ne = PState<T>{s.r, s.z, (T)che.vr, (T)che.vt, (T)che.vz, s.ar, s.az, s.w, s.at};
            ni = PState<T>{s.r,
                           s.z,
                           (T)chi.vr,
                           (T)chi.vt,
                           (T)chi.vz,
                           (T)((double)s.ar * a.phys.ion_acc_ratio),
                           (T)((double)s.az * a.phys.ion_acc_ratio),
                           s.w,
                           (T)((double)s.at * a.phys.ion_acc_ratio)};
            ne_live = ni_live = true;
        }
        bool live = true;
        if (kFirst) {
            first_push<T>(s, dt, xyz, a.phys.friedman ? (T)1 : (T)0.5);
            int b = boundary_of(s, a.phys);
            if (b >= 0) {
                tally_add(a.tally, b, (double)s.w, a.sp.inv_quantum);
                live = false;
                atomicOr(a.ch.dead + c, bit);
            }
            if (iz) {
                first_push<T>(ne, dt, xyz, a.phys.friedman ? (T)1 : (T)0.5);
                b = boundary_of(ne, a.phys);
                if (b >= 0) {
                    tally_add(a.tally, b, (double)ne.w, a.sp.inv_quantum);
                    ne_live = false;
                }
                first_push<T>(ni, (T)a.phys.ion_dt, xyz, a.phys.friedman ? (T)1 : (T)0.5);
                b = boundary_of(ni, a.phys);
                if (b >= 0) {
                    tally_add(a.tally_ion, b, (double)ni.w, a.phys.ion_inv_quantum);
                    ni_live = false;
                }
            }
            if (live)
                deposit4<T>(dep, m, weights<T>(m, s.r, s.z), (double)s.w, a.sp.inv_quantum,
                            a.status);
            if (ne_live)
                deposit4<T>(dep, m, weights<T>(m, ne.r, ne.z), (double)ne.w, a.sp.inv_quantum,
                            a.status);
            if (ni_live)
                deposit4<T>(a.acc_ion, m, weights<T>(m, ni.r, ni.z), (double)ni.w,
                            a.phys.ion_inv_quantum, a.status);
        }
        if (live) store(a.p, pi, s, false);
        if (iz) {
            PState<T> e = ne, i = ni;
            if (!ne_live) e.w = (T)-1;
            if (!ni_live) i.w = (T)-1;
            store(a.ce, pi, e, true);
            store(a.ci, pi, i, true);
            atomicOr(a.ch.ev + c, bit);
            if (ne_live) atomicOr(a.ch.se + c, bit);
            if (ni_live) atomicOr(a.ch.si + c, bit);
        }
      }
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x < 1 + kMaxProc && sh_stat[threadIdx.x])
        atomicAdd(a.mcstat + threadIdx.x, sh_stat[threadIdx.x]);
    if (kLds) {
        unsigned long long *out = (unsigned long long *)a.slices + (size_t)lb * m.nn;
        for (int g = threadIdx.x; g < m.nn; g += blockDim.x) out[g] = lds_acc[g];
    }
}

template <typename T, int MODE> __global__ __launch_bounds__(256) void k_collide(PassArgs<T> a)
{
    collide_body<T, MODE>(a, blockIdx.x, gridDim.x);
}

// Collisions of both species in one launch: blocks [0, c0) species 0,
// [c0, c0 + c1) species 1.
template <typename T> struct Collide2Args {
    PassArgs<T> a0, a1;
    int c0, c1;
};

template <typename T, int MODE> __device__ __forceinline__ void collide2_body(const Blk &k, const Collide2Args<T> &a)
{
    static_assert(offsetof(Collide2Args<T>, a1) == sizeof(PassArgs<T>), "a1 must follow a0");
    const bool ion = k.x >= a.c0;
    collide_body<T, MODE>(species_args(a.a0, ion), ion ? k.x - a.c0 : k.x, ion ? a.c1 : a.c0);
}

// The sum of the pass's LDS slices into the deposit grids: block
// (s, y, x) of 2 x by x bx adds slices y, y + by, ... of species s at nodes
// [256x, 256x + 256) and adds the sum atomically.  A body of its own rather
// than blocks of the collision kernel, whose large register allocation
// would leave them at one wavefront per SIMD; a batched step runs it for
// many discharges in one launch.
__device__ __forceinline__ void slice_sum_body(const Blk &k, const SliceSum &r)
{
    if (r.narrow) {
        // 32-bit slices: block x of species s takes nodes [32 x', 32 x' + 32)
        // (x' = x mod bx) as 8 groups of four; its 256 threads are 8 groups
        // x 32 parts, part p summing slices p, p + 32, ... of its group with
        // 16-byte loads (slices padded to whole groups, slice_stride), up to
        // twelve in flight; the parts are added in LDS and each node gets one
        // atomic.
        constexpr int G = kSliceSumGroups, P = 256 / G, U = 12;
        __shared__ unsigned long long part[P][G][4];
        const int s = k.x / r.bx, x = k.x % r.bx;
        const int grp = threadIdx.x % G, p = threadIdx.x / G;
        const int g4 = x * G + grp, g = 4 * g4;
        const int nb = r.nb[s];
        unsigned long long s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        if (g < r.nn) {
            const size_t stride = slice_stride(r.nn, 1) / 4;
            const uint4 *sl = (const uint4 *)r.slices[s] + g4;
            for (int q = p; q < nb; q += U * P) {
                uint4 v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int qq = q + P * u;
                    v[u] = sl[(size_t)(qq < nb ? qq : nb - 1) * stride];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (q + P * u >= nb) break;
                    s0 += v[u].x;
                    s1 += v[u].y;
                    s2 += v[u].z;
                    s3 += v[u].w;
                }
            }
        }
        part[p][grp][0] = s0;
        part[p][grp][1] = s1;
        part[p][grp][2] = s2;
        part[p][grp][3] = s3;
        __syncthreads();
        if (threadIdx.x < 4 * G) {
            const int gg = threadIdx.x >> 2, c = threadIdx.x & 3, node = 4 * (x * G + gg) + c;
            unsigned long long t = 0;
#pragma unroll
            for (int q = 0; q < P; ++q) t += part[q][gg][c];
            if (node < r.nn) atomicAdd(r.acc[s] + node, t);
        }
        return;
    }
    const int per = r.bx * r.by;
    const int s = k.x / per, x = k.x % r.bx, y = (k.x % per) / r.bx;
    const int g = x * blockDim.x + threadIdx.x;
    if (g >= r.nn) return;
    const unsigned long long *sl = (const unsigned long long *)r.slices[s];
    unsigned long long sum = 0;
    for (int q = y; q < r.nb[s]; q += r.by) sum += sl[(size_t)q * r.nn + g];
    atomicAdd(r.acc[s] + g, sum);
}

hipError_t launch_slice_sum(const SliceSum &r, hipStream_t st)
{
    const int blocks = r.narrow ? 2 * r.bx : 2 * r.bx * r.by;
    return launch<SliceSum, slice_sum_body, 256>(dim3(blocks), dim3(256), 0, st, r);
}

// Staged new particles of species cs (unmerged form): first push or deposit
// of the children recorded in the electron chunk masks (slot = parent index).
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_staged(PassArgs<T> a, int cs)
{
    const Mesh &m = a.mesh;
    const T dt = (T)a.sp.dt;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nch = (a.crec->n_parent + kChunk - 1) / kChunk;
    unsigned long long *alive = cs == 0 ? a.ch.se : a.ch.si;
    for (int64_t c = wave; c < nch; c += nwaves) {
        const unsigned long long bit = 1ull << lane;
        if (!(alive[c] & bit)) continue;
        int64_t slot = c * kChunk + lane;
        PState<T> s = load(a.p, slot);
        if (MODE & M_FIRST) {
            first_push<T>(s, dt, a.p.at != nullptr, a.phys.friedman ? (T)1 : (T)0.5);
            int b = boundary_of(s, a.phys);
            if (b >= 0) {
                tally_add(a.tally, b, (double)s.w, a.sp.inv_quantum);
                a.p.w[slot] = (T)-1;
                atomicAnd(alive + c, ~bit);
                continue;
            }
            store(a.p, slot, s, false);
        }
        if (MODE & M_DEP)
            deposit4<T>(a.acc, m, weights<T>(m, s.r, s.z), (double)s.w, a.sp.inv_quantum,
                        a.status);
    }
}

// Sec. 2.3 initialisation (C-ABI rzpic_init_particles).
template <typename T>
__global__ void k_init(Parts<T> p, int64_t n, double wcoef, double vth, uint64_t id0, int s,
                       Phys ph)
{
    const uint32_t kInit = 0xFFFFFFFFu;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t id = id0 + (uint64_t)i;
        double u0, u1, a0, a1, b0, b1, n1, n2, n3, n4;
        uniform2(ph.seed, s, id, kInit, 0, u0, u1);
        uniform2(ph.seed, s, id, kInit, 1, a0, a1);
        uniform2(ph.seed, s, id, kInit, 2, b0, b1);
        normal2(a0, a1, n1, n2);
        normal2(b0, b1, n3, n4);
        double r = u0 * ph.R;
        p.r[i] = (T)r;
        p.z[i] = (T)(u1 * ph.L);
        p.vr[i] = (T)(vth * n1);
        p.vt[i] = (T)(vth * n2);
        p.vz[i] = (T)(vth * n3);
        p.ar[i] = (T)0;
        p.az[i] = (T)0;
        if (p.at) p.at[i] = (T)0;
        p.w[i] = (T)(wcoef * r);
        p.id[i] = id;
    }
}

template <typename T>
hipError_t launch_pass(int mode, const PassArgs<T> &a, int blocks, int threads, size_t lds,
                       hipStream_t st)
{
#define RZ_CASE(M)                                                                     \
    case M:                                                                            \
        RZ_LAUNCH((k_pass<T, M>), dim3(blocks), dim3(threads), lds, st, a); \
        break;
    switch (mode) {
        RZ_CASE(M_FINAL | M_MC | M_FIRST | M_DEP | M_LISTS)
        RZ_CASE(M_FINAL | M_MC | M_FIRST | M_DEP | M_LISTS | M_LDS)
        RZ_CASE(M_FIRST | M_DEP | M_LISTS)
        RZ_CASE(M_FIRST | M_DEP | M_LISTS | M_LDS)
        RZ_CASE(M_DEP)
        RZ_CASE(M_DEP | M_LDS)
        RZ_CASE(M_DEP | M_MARK)
        RZ_CASE(M_DEP | M_MARK | M_LDS)
        RZ_CASE(M_DEP | M_TILE)
        RZ_CASE(M_DEP | M_MARK | M_TILE)
        RZ_CASE(M_FIRST | M_DEP | M_LISTS | M_TILE)
        RZ_CASE(M_FINAL | M_MARK)
        RZ_CASE(M_FIRST | M_MARK)
        RZ_CASE(M_MC | M_MARK)
    default:
        return hipErrorInvalidValue;
    }
#undef RZ_CASE
    return hipGetLastError();
}

template <typename T>
hipError_t launch_collide(int mode, const PassArgs<T> &a, int blocks, int threads, size_t lds,
                          hipStream_t st)
{
    if (mode == (M_FIRST | M_LDS))
        RZ_LAUNCH((k_collide<T, M_FIRST | M_LDS>), dim3(blocks), dim3(threads), lds, st, a);
    else if (mode == M_FIRST)
        RZ_LAUNCH((k_collide<T, M_FIRST>), dim3(blocks), dim3(threads), 0, st, a);
    else if (mode == 0)
        RZ_LAUNCH((k_collide<T, 0>), dim3(blocks), dim3(threads), 0, st, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_staged(int mode, const PassArgs<T> &a, int cs, hipStream_t st)
{
    const int blocks = 1024, threads = 256;
    if (mode == M_FIRST)
        RZ_LAUNCH((k_staged<T, M_FIRST>), dim3(blocks), dim3(threads), 0, st, a, cs);
    else if (mode == M_DEP)
        RZ_LAUNCH((k_staged<T, M_DEP>), dim3(blocks), dim3(threads), 0, st, a, cs);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init(Parts<T> p, int64_t n, double n0, double T_eV, uint64_t id0, int s,
                       const Phys &phys, double m, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    double wcoef = kTwoPi * n0 * phys.R * phys.L / (double)n;
    double vth = sqrt(T_eV * kE / m);
    int threads = 256;
    int64_t blocks64 = (n + threads - 1) / threads;
    int blocks = (int)(blocks64 < 65536 ? blocks64 : 65536);
    RZ_LAUNCH((k_init<T>), dim3(blocks), dim3(threads), 0, st, p, n, wcoef, vth, id0, s,
                       phys);
    return hipGetLastError();
}

// Fused merged pass of both species (blocks [0, b0) species 0, [b0, b0+b1)
// species 1), then their collision kernels in one launch (c0 + c1 blocks).
template <typename T>
hipError_t launch_pass2(int mode, const PassArgs<T> &a0, const PassArgs<T> &a1, int b0, int b1,
                        int threads, size_t lds, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    constexpr int kBase = M_FINAL | M_MC | M_FIRST | M_DEP | M_LISTS;
    const Pass2Args<T> a{a0, a1, b0};
    const dim3 grid(b0 + b1), block(threads);
    if (mode == (kBase | M_LDS))
        return launch_ev<Pass2Args<T>, pass2_body<T, kBase | M_LDS>, 1024>(grid, block, lds, st, a,
                                                                           ev0, ev1);
    if (mode == (kBase | M_TILE))
        return launch_ev<Pass2Args<T>, pass2_body<T, kBase | M_TILE>, 1024>(grid, block, lds, st,
                                                                            a, ev0, ev1);
    if (mode == kBase)
        return launch_ev<Pass2Args<T>, pass2_body<T, kBase>, 1024>(grid, block, 0, st, a, ev0, ev1);
    return hipErrorInvalidValue;
}

template <typename T> int pass2_tiled_blocks_per_cu(int threads)
{
    constexpr int kMode = M_FINAL | M_MC | M_FIRST | M_DEP | M_LISTS | M_TILE;
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, k_one<Pass2Args<T>, pass2_body<T, kMode>, 1024>, threads,
        (size_t)kWinNodes * sizeof(unsigned long long));
    return e == hipSuccess && nb > 0 ? nb : 1;
}

template <typename T>
hipError_t launch_collide2(const PassArgs<T> &a0, const PassArgs<T> &a1, int c0, int c1,
                           int threads, hipStream_t st)
{
    return launch<Collide2Args<T>, collide2_body<T, M_FIRST>, 256>(
        dim3(c0 + c1), dim3(threads), 0, st, Collide2Args<T>{a0, a1, c0, c1});
}

// The collisions and the slice sum in one launch: blocks [0, c0 + c1) run the
// collision body, the rest the slice sum (independent work: the collided
// particles' deposits and the slices' sums are integer atomics on the same
// grids).  The slice sum's HBM reads then overlap the collisions' chains of
// dependent loads.  FP32 particles only: there the collision body holds 98
// VGPRs, so the slice-sum blocks keep five wavefronts per SIMD (in FP64 it
// holds 245, one wavefront per SIMD, and the two launch apart).
struct CollideSumArgsF {
    Collide2Args<float> c;
    SliceSum r;
};

__device__ __forceinline__ void collide_sum_body(const Blk &k, const CollideSumArgsF &a)
{
    const int nc = a.c.c0 + a.c.c1;
    if (k.x < nc) collide2_body<float, M_FIRST>(Blk{k.x, 0, nc, 1}, a.c);
    else slice_sum_body(Blk{k.x - nc, 0, k.nx - nc, 1}, a.r);
}

hipError_t launch_collide_sum(const PassArgs<float> &a0, const PassArgs<float> &a1, int c0,
                              int c1, const SliceSum &r, hipStream_t st)
{
    const int ns = r.narrow ? 2 * r.bx : 2 * r.bx * r.by;
    return launch<CollideSumArgsF, collide_sum_body, 256>(
        dim3(c0 + c1 + ns), dim3(256), 0, st,
        CollideSumArgsF{Collide2Args<float>{a0, a1, c0, c1}, r});
}

template <typename T> int pass2_lds_blocks_per_cu(int threads, size_t lds)
{
    constexpr int kMode = M_FINAL | M_MC | M_FIRST | M_DEP | M_LISTS | M_LDS;
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, k_one<Pass2Args<T>, pass2_body<T, kMode>, 1024>, threads, lds);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

template int pass2_tiled_blocks_per_cu<double>(int);
template int pass2_tiled_blocks_per_cu<float>(int);
template int pass2_lds_blocks_per_cu<double>(int, size_t);
template int pass2_lds_blocks_per_cu<float>(int, size_t);
template hipError_t launch_pass2<double>(int, const PassArgs<double> &, const PassArgs<double> &,
                                         int, int, int, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_pass2<float>(int, const PassArgs<float> &, const PassArgs<float> &, int,
                                        int, int, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_collide2<double>(const PassArgs<double> &, const PassArgs<double> &,
                                            int, int, int, hipStream_t);
template hipError_t launch_collide2<float>(const PassArgs<float> &, const PassArgs<float> &, int,
                                           int, int, hipStream_t);
template hipError_t launch_pass<double>(int, const PassArgs<double> &, int, int, size_t,
                                        hipStream_t);
template hipError_t launch_pass<float>(int, const PassArgs<float> &, int, int, size_t, hipStream_t);
template hipError_t launch_collide<double>(int, const PassArgs<double> &, int, int, size_t,
                                           hipStream_t);
template hipError_t launch_collide<float>(int, const PassArgs<float> &, int, int, size_t,
                                          hipStream_t);
template hipError_t launch_staged<double>(int, const PassArgs<double> &, int, hipStream_t);
template hipError_t launch_staged<float>(int, const PassArgs<float> &, int, hipStream_t);
template hipError_t launch_init<double>(Parts<double>, int64_t, double, double, uint64_t, int,
                                        const Phys &, double, hipStream_t);
template hipError_t launch_init<float>(Parts<float>, int64_t, double, double, uint64_t, int,
                                       const Phys &, double, hipStream_t);

}  // namespace rz
