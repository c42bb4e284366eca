// Host runtime of the C ABI declared in include/rzpic.h: context and
// configuration checks, device allocations, and the launch sequences of the
// cycle of Sec. 2.1 on the caller's stream.
#include "rzpic.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"
#include "internal.h"

using namespace rz;

namespace {

thread_local std::string g_err;

rzpic_status fail(rzpic_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(RZPIC_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                \
    } while (0)

void free_sort(SpeciesState &ss)
{
    for (void *&p : ss.sort_buf)
        if (p) {
            (void)hipFree(p);
            p = nullptr;
        }
    for (void *p : {(void *)ss.sort_off, (void *)ss.sort_part, (void *)ss.tile_pb,
                    (void *)ss.tile_win})
        if (p) (void)hipFree(p);
    ss.sort_off = ss.sort_part = ss.tile_pb = nullptr;
    ss.tile_win = nullptr;
    ss.sort_seg = ss.sort_nseg = 0;
    ss.tile_nb = 0;
}

}  // namespace


namespace {

template <typename T> rzpic_status dalloc(rzpic_ctx *c, T **p, size_t count)
{
    void *q = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(RZPIC_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    e = hipMemset(q, 0, bytes);
    if (e != hipSuccess) return fail(RZPIC_EHIP, "hipMemset failed: %s", hipGetErrorString(e));
    c->allocs.push_back(q);
    *p = (T *)q;
    return RZPIC_OK;
}

#define TRY(expr)                            \
    do {                                     \
        rzpic_status s_ = (expr);            \
        if (s_ != RZPIC_OK) return s_;       \
    } while (0)

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Ions subcycled every K >= 2 steps take K dt; everything else dt.
int ion_K(const rzpic_ctx *c) { return c->c.ion_subcycle > 1 ? c->c.ion_subcycle : 1; }

double dt_of(const rzpic_ctx *c, int s) { return s == 1 ? ion_K(c) * c->c.dt : c->c.dt; }

Mesh mesh_of(const rzpic_ctx *c)
{
    Mesh m;
    m.nr = c->c.nr;
    m.nz = c->c.nz;
    m.nn = c->nn;
    m.weighting = c->c.weighting;
    m.R = c->c.R;
    m.L = c->c.L;
    m.hr = c->hr;
    m.hz = c->hz;
    m.inv_hr = 1.0 / c->hr;
    m.inv_hz = 1.0 / c->hz;
    return m;
}

Phys phys_of(const rzpic_ctx *c)
{
    Phys p;
    p.dt = c->c.dt;
    p.n_gas = c->c.n_gas;
    p.T_gas = c->c.T_gas;
    p.m_gas = c->c.m_gas;
    p.vth_gas = c->c.m_gas > 0 ? std::sqrt(kKb * c->c.T_gas / c->c.m_gas) : 0.0;
    p.R = c->c.R;
    p.L = c->c.L;
    p.seed = c->c.seed;
    const rzpic_species_view &e = c->sp[0].v, &i = c->sp[1].v;
    p.ion_acc_ratio = (c->sp[0].bound && c->sp[1].bound) ? (i.q * e.m) / (e.q * i.m) : 0.0;
    p.ion_inv_quantum = 1.0 / c->quantum[1];
    p.ion_dt = dt_of(c, 1);
    p.friedman = c->c.damping == RZPIC_DAMP_FRIEDMAN ? 1 : 0;
    p.fc = 0.5 * c->c.theta;
    return p;
}

double pair_mass(const rzpic_ctx *c, int s)
{
    const rzpic_species_view &v = c->sp[s].v;
    if (v.mc_model == RZPIC_MC_ION) return v.m * c->c.m_gas / (v.m + c->c.m_gas);
    return v.m;
}

SpeciesK species_of(const rzpic_ctx *c, int s)
{
    SpeciesK k{};
    const SpeciesState &ss = c->sp[s];
    const rzpic_species_view &v = ss.v;
    k.s = s;
    k.mc_model = ss.has_xsec ? v.mc_model : RZPIC_MC_NONE;
    k.q = v.q;
    k.m = v.m;
    k.qm = v.q / v.m;
    k.dt = dt_of(c, s);
    // implicit coefficient: 1/2 (D1), theta/2 (Friedman damping)
    const double cf = c->c.damping == RZPIC_DAMP_FRIEDMAN ? 0.5 * c->c.theta : 0.5;
    k.k1 = cf * k.qm * k.dt * k.dt;
    k.k2 = cf * k.qm * k.dt;
    k.inv_quantum = 1.0 / c->quantum[s];
    k.p_null = ss.p_null;
    k.nu_max = ss.nu_max;
    // U0 = (u + 1/2) 2^-52 < P_null exactly when u < ceil(P_null 2^52 - 1/2):
    // the scaling by 2^52 and the subtraction are exact in FP64
    const double P = std::ldexp(ss.p_null, 52);
    k.cand_u52 = P > 0.5 ? (uint64_t)std::ceil(P - 0.5) : 0;
    k.mu = ss.bound ? pair_mass(c, s) : 1.0;
    k.ekin = 0.5 * k.mu / kE;
    k.xs = ss.xs;
    return k;
}

template <typename T> Parts<T> parts_of(const rzpic_species_view &v)
{
    Parts<T> p;
    p.r = (T *)v.r;
    p.z = (T *)v.z;
    p.vr = (T *)v.vr;
    p.vt = (T *)v.vt;
    p.vz = (T *)v.vz;
    p.ar = (T *)v.ar;
    p.az = (T *)v.az;
    p.w = (T *)v.w;
    p.id = v.id;
    p.at = (T *)v.at;  // null unless the global X-Y-Z push (bind_species)
    return p;
}

template <typename T> Parts<T> stage_of(const rzpic_ctx *c, int cs)
{
    Parts<T> p{};
    void *const *a = c->sp[0].stage[cs];
    p.r = (T *)a[0];
    p.z = (T *)a[1];
    p.vr = (T *)a[2];
    p.vt = (T *)a[3];
    p.vz = (T *)a[4];
    p.ar = (T *)a[5];
    p.az = (T *)a[6];
    p.w = (T *)a[7];
    p.id = nullptr;
    p.at = (T *)a[8];
    return p;
}

template <typename T> PassArgs<T> pass_args(rzpic_ctx *c, int s, uint32_t step)
{
    PassArgs<T> a{};
    a.p = parts_of<T>(c->sp[s].v);
    if (s == 0 && c->sp[0].stage[0][0]) {
        a.ce = stage_of<T>(c, 0);
        a.ci = stage_of<T>(c, 1);
    }
    a.cnt = c->cnt + s;
    a.ch = c->sp[s].ch;
    a.mesh = mesh_of(c);
    a.phys = phys_of(c);
    a.sp = species_of(c, s);
    a.E2 = (const typename Vec2<T>::type *)c->E2;
    a.acc = c->acc[s];
    a.acc_ion = c->acc[1];
    a.slices = c->slices;
    a.tally = c->tally + 3 * s;
    a.tally_ion = c->tally + 3;
    a.mcstat = c->mcstat + (1 + kMaxProc) * s;
    a.ev = c->sp[s].v.mc_event;
    a.crec = s == 0 ? c->crec : nullptr;
    a.status = c->status;
    a.step = step;
    a.tile_pb = c->sp[s].tile_pb;
    a.tile_win = c->sp[s].tile_win;
    a.tile_nb = c->sp[s].tile_nb;
    return a;
}

// Pass blocks of species s, at most `most`: about one per parts_per_block
// (8192 unless tuned) particles of capacity, since every block of a deposit
// form pays a fixed cost (zeroing and writing out its LDS grid or window)
// that only pays off over enough particles.
// Bytes of one node of a block's LDS deposit grid (and of its slice): FP32
// particles accumulate in 32 bits with carries to the global grid.
template <typename T> constexpr size_t lds_elem() { return sizeof(T) == 4 ? 4 : 8; }

int pass_blocks(const rzpic_ctx *c, int s, int most)
{
    const int64_t ppb = c->parts_per_block;
    const int64_t want = (c->sp[s].cap + ppb - 1) / ppb;
    if (most < 1) most = 1;
    return (int)(want < 1 ? 1 : (want < most ? want : most));
}

// Blocks of the whole-grid LDS pass that fit on the device at once with
// `threads` per block (LDS, wavefronts and registers), at most the slices
// allocated: the merged pass runs one round of blocks.
int lds_resident_of(const rzpic_ctx *c, int threads)
{
    const size_t lds = (size_t)c->nn * (c->mixed ? sizeof(uint32_t) : sizeof(unsigned long long));
    int per_cu = (int)(c->lds_cu / (lds + 1024));
    const int wave_cap = 2048 / threads;
    const int occ = c->mixed ? pass2_lds_blocks_per_cu<float>(threads, lds)
                             : pass2_lds_blocks_per_cu<double>(threads, lds);
    if (per_cu > wave_cap) per_cu = wave_cap;
    if (per_cu > occ) per_cu = occ;
    if (per_cu < 1) per_cu = 1;
    const int b = c->cus * per_cu;
    return b < c->slice_blocks ? b : c->slice_blocks;
}

// Blocks of the tiled pass of species s: at most the blocks the merged pass
// keeps resident at once, shared by the two species (one round, no tail).
// The window plan of the sort is made for this count.
int tiled_blocks(const rzpic_ctx *c, int s)
{
    return pass_blocks(c, s, c->cus * c->tile_per_cu / 2);
}

rzpic_status need_species(rzpic_ctx *c, int s)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    if (s < 0 || s > 1) return fail(RZPIC_EINVAL, "species %d out of range (0 or 1)", s);
    if (!c->sp[s].bound) return fail(RZPIC_ESTATE, "species %d is not bound", s);
    return RZPIC_OK;
}

rzpic_status need_both(rzpic_ctx *c)
{
    TRY(need_species(c, 0));
    TRY(need_species(c, 1));
    return RZPIC_OK;
}

// Results of rzpic_solve_dev on the device: the cycles run and the relative
// residual, either given (tolerance mode, known on the host) or formed from
// the norms the fixed-cycle solve left in norm[0] (residual) and norm[1]
// (scale), as the host does.
__global__ void k_solve_out(int32_t *cycles, double *relres, int k, double rr,
                            const unsigned long long *norm)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (cycles) *cycles = k;
    if (relres) {
        if (norm) {
            const double rn = __longlong_as_double((long long)norm[0]);
            const double sc = __longlong_as_double((long long)norm[1]);
            rr = sc > 0 ? rn / sc : rn;
        }
        *relres = rr;
    }
}

__global__ void k_set_count(Counts *cnt, int64_t n, uint64_t next_id)
{
    cnt->n = n;
    cnt->next_id = next_id;
}

__global__ void k_prep_solve(int nn, const double *rho, const double *chi, double *eps,
                             float *eps32, double *f)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x) {
        double e = 1.0 + chi[g];
        eps[g] = e;
        if (eps32) eps32[g] = (float)e;
        f[g] = rho[g] / kEps0;
    }
}

void mark(rzpic_ctx *c, int k);

// Particle pass of species s in `mode` (LDS variant chosen here).
template <typename T> rzpic_status run_pass(rzpic_ctx *c, int s, int mode, uint32_t step)
{
    PassArgs<T> a = pass_args<T>(c, s, step);
    int blocks, threads = c->pass_threads;
    size_t lds = 0;
    if ((mode & M_DEP) && c->lds_form) {
        mode |= M_LDS;
        lds = (size_t)c->nn * lds_elem<T>();
        blocks = pass_blocks(c, s, c->slice_blocks);
    } else if ((mode & M_DEP) && !(mode & M_MC)) {
        mode |= M_TILE;
        lds = (size_t)kWinNodes * sizeof(unsigned long long);
        blocks = tiled_blocks(c, s);
        a.tiled = 1;
    } else {
        int64_t need = (c->sp[s].cap + threads - 1) / threads;
        blocks = c->cus * (2048 / threads);
        if (need < blocks) blocks = (int)(need > 0 ? need : 1);
    }
    const bool mc = (mode & M_MC) && a.sp.mc_model != RZPIC_MC_NONE;
    if (mode & M_MC) HIPCHK(launch_fill_u64(a.mcstat, 1 + kMaxProc, c->st));
    a.nbuckets = blocks;
    a.bucket_waves = threads / 64;
    if (blocks * (threads / 64) > kMaxWaves)
        return fail(RZPIC_EINVAL, "pass of %d wavefronts exceeds %d", blocks * threads / 64, kMaxWaves);
    HIPCHK(launch_pass<T>(mode, a, blocks, threads, lds, c->st));
    if (mode & M_LDS)
        HIPCHK(launch_reduce_slices(c->acc[s], c->slices, lds_elem<T>() == 4, blocks, c->nn, c->st));
    if (mc) {
        // candidates: outcome, and in the merged form their first push and deposit
        const bool merged = (mode & M_FIRST) != 0;
        int cmode = merged ? M_FIRST : 0;
        const double expect = c->sp[s].p_null * (double)c->sp[s].cap;
        int cblocks = c->cus * 2, cthreads = 256;
        size_t clds = 0;
        if (merged && c->lds_form && expect > 65536.0 &&
            (size_t)c->nn * sizeof(unsigned long long) + 1024 <= c->lds_block) {
            // few blocks: each flushes a whole grid copy
            cmode |= M_LDS;
            clds = (size_t)c->nn * sizeof(unsigned long long);
            cblocks = c->cus / 2 > 0 ? c->cus / 2 : 1;
            if (const char *e = std::getenv("RZPIC_COLLIDE_BLOCKS")) {
                int b = std::atoi(e);
                if (b > 0) cblocks = b;
            }
            if (cblocks > c->slice_blocks) cblocks = c->slice_blocks;
        } else if (expect < 4096.0) {
            cblocks = c->cus / 4 > 0 ? c->cus / 4 : 1;
        }
        HIPCHK(launch_collide<T>(cmode, a, cblocks, cthreads, clds, c->st));
        if (cmode & M_LDS)
            HIPCHK(launch_reduce_slices(c->acc[s], c->slices, 0, cblocks, c->nn, c->st));
    }
    return RZPIC_OK;
}

// The merged step's particle work for both species in two launches: the
// fused pass of both species side by side (each block privatises the grid of
// its species in LDS), then the collision kernels of both species with the
// sum of the LDS slices into the two deposit grids beside them.  ions =
// false (subcycled ions in a step where they do not move): no ion blocks in
// either launch, every LDS slice to the electrons.
template <typename T> rzpic_status run_pass_both(rzpic_ctx *c, uint32_t step, bool ions = true)
{
    PassArgs<T> a[2] = {pass_args<T>(c, 0, step), pass_args<T>(c, 1, step)};
    const int threads = c->pass_threads;
    int mode = M_FINAL | M_MC | M_FIRST | M_DEP | M_LISTS;
    int b[2];
    size_t lds = 0;
    if (c->lds_form) {
        mode |= M_LDS;
        lds = (size_t)c->nn * lds_elem<T>();
        const int most = c->lds_resident;
        b[0] = pass_blocks(c, 0, most / 2);
        b[1] = pass_blocks(c, 1, most - most / 2);
        if (!ions) {  // the electrons take the ions' blocks too
            b[0] = b[0] + b[1] < most ? b[0] + b[1] : most;
            b[1] = 0;
        }
    } else {
        // grid larger than LDS: contiguous block ranges with LDS windows of
        // the tiles planned at the last sort (global atomics without a plan)
        mode |= M_TILE;
        lds = (size_t)kWinNodes * sizeof(unsigned long long);
        for (int s = 0; s < 2; ++s) b[s] = tiled_blocks(c, s);
        if (!ions) b[1] = 0;
    }
    for (int s = 0; s < 2; ++s) {
        a[s].psteps = c->psteps + s;
        a[s].nbuckets = b[s];
        a[s].bucket_waves = threads / 64;
        a[s].tiled = (mode & M_TILE) ? 1 : 0;
    }
    a[1].slices = (char *)c->slices + (size_t)b[0] * slice_stride(c->nn, lds_elem<T>() == 4) * lds_elem<T>();
    if ((b[0] + b[1]) * (threads / 64) > kMaxWaves)
        return fail(RZPIC_EINVAL, "pass of %d wavefronts exceeds %d", (b[0] + b[1]) * threads / 64,
                    kMaxWaves);
    // step timing: the pass's events on its own dispatch (its run time alone)
    hipEvent_t e4 = nullptr, e5 = nullptr;
    if (c->timing && c->ev_used < rzpic_ctx::kPool) {
        e4 = c->evpool[(size_t)c->ev_used * rzpic_ctx::kEvPerStep + 4];
        e5 = c->evpool[(size_t)c->ev_used * rzpic_ctx::kEvPerStep + 5];
    }
    HIPCHK(launch_pass2<T>(mode, a[0], a[1], b[0], b[1], threads, lds, c->st, e4, e5));
    // collision kernels: four wavefronts per bucket with many candidates
    // (each lane then takes about one: the chain of dependent loads per
    // candidate is the kernel's time), one per bucket otherwise (ion
    // candidates are rare), deposits by global atomics
    const int cthreads = 256, wpb = cthreads / 64;
    int cb[2];
    for (int s = 0; s < 2; ++s) {
        const double expect = c->sp[s].p_null * (double)c->sp[s].cap;
        // at least three wavefronts per CU when there are many candidates, so
        // that fewer, larger pass blocks (more threads each) do not thin
        // out the collisions' waves
        const int many = 4 * b[s] > 3 * c->cus ? 4 * b[s] : 3 * c->cus;
        const int want = expect > 16.0 * b[s] ? many : b[s];
        cb[s] = (want + wpb - 1) / wpb;
        if (a[s].sp.mc_model == RZPIC_MC_NONE) cb[s] = 1;
    }
    if (!ions) cb[1] = 0;  // no ion candidates were collected
    SliceSum r{};
    if (mode & M_LDS) {
        for (int s = 0; s < 2; ++s) {
            r.acc[s] = c->acc[s];
            r.slices[s] = a[s].slices;
            r.nb[s] = b[s];
        }
        r.nn = c->nn;
        r.narrow = lds_elem<T>() == 4;
        // 32-bit slices: 4 kSliceSumGroups nodes per block (slice_sum_body);
        // 64-bit: 256 nodes per block, the slices split over by blocks
        const int per_block = r.narrow ? 4 * kSliceSumGroups : cthreads;
        r.bx = (c->nn + per_block - 1) / per_block;
        const int nb = b[0] > b[1] ? b[0] : b[1];
        r.by = r.narrow ? 1 : nb < 32 ? nb : 32;
    }
    // the collisions and (whole-grid LDS form) the slice sum: in one launch
    // for FP32 particles (launch_collide_sum); in FP64 the slice sum runs in
    // a kernel of its own, since in one launch its blocks would run at the
    // collision kernel's register allocation (one wavefront per SIMD).  All
    // are bodies a batched step runs for many discharges at once.
    if constexpr (sizeof(T) == 4) {
        if (mode & M_LDS) HIPCHK(launch_collide_sum(a[0], a[1], cb[0], cb[1], r, c->st));
        else HIPCHK(launch_collide2<T>(a[0], a[1], cb[0], cb[1], cthreads, c->st));
    } else {
        HIPCHK(launch_collide2<T>(a[0], a[1], cb[0], cb[1], cthreads, c->st));
        if (mode & M_LDS) HIPCHK(launch_slice_sum(r, c->st));
    }
    mark(c, 6);
    return RZPIC_OK;
}

template <typename T> rzpic_status run_staged(rzpic_ctx *c, int cs, int mode)
{
    // children of species cs staged by the electron pass
    PassArgs<T> a = pass_args<T>(c, cs, 0);
    a.p = stage_of<T>(c, cs);
    a.ch = c->sp[0].ch;
    a.crec = c->crec;
    a.acc = c->acc[cs];
    a.tally = c->tally + 3 * cs;
    a.sp = species_of(c, cs);
    HIPCHK(launch_staged<T>(mode, a, cs, c->st));
    return RZPIC_OK;
}

// The next step's grid preparation run by a step's list maintenance (step
// pipelining): mg_finalize's arguments (no clearing) and the solve's
// electrode voltage.
struct NextGrid {
    GridArgs g;
    double V;
    bool defer;  // keep the hole filling and appending for the next step's way down
};

// List maintenance of the species in `which` (bit s): superchunk totals,
// sorted dead lists, hole filling, appending of staged children.  With
// `next`, the superchunk totals and the dead lists run beside the next
// step's grid preparation (mg_finalize_scan, mg_prep_dead_list).
template <typename T>
rzpic_status run_fixup(rzpic_ctx *c, int which, const NextGrid *next = nullptr)
{
    ScanJobs j{};
    j.children = (c->children_pending[0] || c->children_pending[1]) && !c->children_scanned;
    j.ech = c->sp[0].ch;
    j.ecnt = c->cnt;
    j.icnt = c->cnt + 1;
    j.crec = c->crec;
    j.status = c->status;
    int64_t max_chunks = 1;
    for (int s = 0; s < 2; ++s) {
        j.dead[s] = (which >> s) & 1;
        j.kids[s] = j.dead[s] && c->children_pending[s];
        j.ch[s] = c->sp[s].ch;
        j.cnt[s] = c->cnt + s;
        j.fix[s] = c->fix + s;
        j.cap[s] = c->sp[s].cap;
        int64_t nch = (c->sp[s].cap + kChunk - 1) / kChunk;
        if (c->sp[s].bound && nch > max_chunks) max_chunks = nch;
    }
    if (next)
        HIPCHK(mg_finalize_scan(next->g, c->mg, c->mixed, c->phi, c->phi_alt, next->V, j,
                                max_chunks, c->st));
    else
        HIPCHK(launch_scan(j, max_chunks, c->st));
    if (j.children) c->children_scanned = true;
    if (next)
        HIPCHK(mg_prep_dead_list(c->mg, c->mixed, c->phi, c->f, j, max_chunks, c->st));
    else
        HIPCHK(launch_dead_list(j, max_chunks, c->st));
    Parts<T> none{};
    if (next && next->defer && j.dead[0] && j.dead[1]) {
        // step pipelining: kept for the next step's way-down launches
        list_tail_keep<T>(c->tail, parts_of<T>(c->sp[0].v), parts_of<T>(c->sp[1].v),
                          c->sp[0].ch, c->sp[1].ch, c->fix, c->fix + 1, j,
                          c->sp[0].bound ? parts_of<T>(c->sp[0].v) : none,
                          c->sp[1].bound ? parts_of<T>(c->sp[1].v) : none, stage_of<T>(c, 0),
                          stage_of<T>(c, 1), c->cnt, c->cnt + 1, max_chunks);
    } else {
        if (j.dead[0] && j.dead[1]) {
            HIPCHK(launch_fill2<T>(parts_of<T>(c->sp[0].v), parts_of<T>(c->sp[1].v),
                                   c->sp[0].ch, c->sp[1].ch, c->fix, c->fix + 1, c->st));
        } else {
            for (int s = 0; s < 2; ++s)
                if (j.dead[s])
                    HIPCHK(launch_fill<T>(parts_of<T>(c->sp[s].v), c->sp[s].ch, c->fix + s,
                                          c->st));
        }
        HIPCHK(launch_append<T>(j, c->sp[0].bound ? parts_of<T>(c->sp[0].v) : none,
                                c->sp[1].bound ? parts_of<T>(c->sp[1].v) : none,
                                stage_of<T>(c, 0), stage_of<T>(c, 1), c->cnt, c->cnt + 1,
                                max_chunks, c->st));
    }
    for (int s = 0; s < 2; ++s)
        if (j.kids[s]) c->children_pending[s] = false;
    if (!c->children_pending[0] && !c->children_pending[1]) c->children_scanned = false;
    return RZPIC_OK;
}

// V(0,1) cycles on u with right-hand side f (level tables prepared, the
// Dirichlet values of u and u_alt set): `fixed` > 0 cycles without a test,
// else cycles until ||f - A u||_inf <= tol ||f_bc||_inf (at most
// max_cycles).  Tolerance mode runs the cycles in batches with one
// synchronisation per batch: u is kept before each cycle of the batch and
// the residual norm before the batch and after each cycle is recorded, so
// the solve ends exactly at the first cycle that meets the tolerance (u
// restored from its snapshot), as a test after every cycle would.  The
// first batch takes the cycles the last solve of the same buffer (hint)
// needed, later ones 2, 4, 8, ...  Meshes without snapshots test after
// every cycle.  *k receives the cycles run; with want_res (always in
// tolerance mode) *relres the final relative residual.  The V-cycle may
// exchange u and u_alt.
rzpic_status run_cycles(rzpic_ctx *c, double V, double *&u, double *&u_alt, const double *f,
                        int fixed, double tol, int max_cycles, bool want_res, int *k_out,
                        double *relres, int *hint = nullptr)
{
    const bool ob = c->mg.one_block != 0;
    bool down_done = false;  // the first cycle's restriction came with the tables
    const bool ready = c->prep_ready;  // tables and restriction made by the previous step
    c->prep_ready = false;
    if (c->mg.split) {
        if (!ready) HIPCHK(mg_prep(c->mg, c->mixed, u, f, c->st));
        down_done = true;
    } else if (ob) {
        HIPCHK(mg_factor(c->mg, c->mixed, c->st));
    }
    auto cycles_run = [&](int kk) -> hipError_t {
        if (ob) return mg_solve_block(c->mg, c->mixed, u, f, V, kk, c->st);
        for (int q = 0; q < kk; ++q) {
            hipError_t e = mg_vcycle(c->mg, c->mixed, u, u_alt, f, down_done ? 1 : 0, c->st,
                                     &c->tail);
            down_done = false;
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    auto as_double = [](unsigned long long v) {
        double d;
        std::memcpy(&d, &v, 8);
        return d;
    };
    auto resid = [&](double &rn, double &sc) -> rzpic_status {
        HIPCHK(launch_fill_u64(c->norm, 2, c->st));
        HIPCHK(mg_resid_norm(c->mg, u, f, 1, c->norm + 1, c->st));
        HIPCHK(mg_resid_norm(c->mg, u, f, 0, c->norm, c->st));
        HIPCHK(hipMemcpyAsync(c->normk_host, c->norm, 2 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        rn = as_double(c->normk_host[0]);
        sc = as_double(c->normk_host[1]);
        return RZPIC_OK;
    };
    int k = 0;
    rzpic_status st = RZPIC_OK;
    if (fixed > 0) {
        HIPCHK(cycles_run(fixed));
        k = fixed;
        *k_out = k;
        if (want_res) {
            double rn, sc;
            TRY(resid(rn, sc));
            *relres = sc > 0 ? rn / sc : rn;
        }
        return st;
    }
    const size_t nb = (size_t)c->nn * sizeof(double);
    HIPCHK(launch_fill_u64(c->norm, 2, c->st));
    HIPCHK(mg_resid_norm(c->mg, u, f, 1, c->norm + 1, c->st));
    int batch = hint && *hint > 0 ? *hint : 1, next = 2;
    double rr = 0.0;
    for (;;) {
        int B = c->ring_slots > 0 ? batch : 0;
        if (B > c->ring_slots) B = c->ring_slots;
        if (B > max_cycles - k) B = max_cycles - k;
        if (B < 0) B = 0;
        HIPCHK(launch_fill_u64(c->normk, B + 1, c->st));
        HIPCHK(mg_resid_norm(c->mg, u, f, 0, c->normk, c->st));
        for (int q = 0; q < B; ++q) {
            HIPCHK(hipMemcpyAsync(c->ring + (size_t)q * c->nn, u, nb, hipMemcpyDeviceToDevice,
                                  c->st));
            HIPCHK(cycles_run(1));
            HIPCHK(mg_resid_norm(c->mg, u, f, 0, c->normk + q + 1, c->st));
        }
        HIPCHK(hipMemcpyAsync(c->normk_host, c->normk, (B + 1) * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(c->normk_host + B + 1, c->norm + 1, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        const double sc = as_double(c->normk_host[B + 1]);
        int q = 0;
        while (q <= B && !(as_double(c->normk_host[q]) <= tol * sc)) ++q;
        if (q <= B) {
            // converged after k + q cycles: the later cycles of the batch undone
            if (q < B)
                HIPCHK(hipMemcpyAsync(u, c->ring + (size_t)q * c->nn, nb, hipMemcpyDeviceToDevice,
                                      c->st));
            k += q;
            rr = sc > 0 ? as_double(c->normk_host[q]) / sc : as_double(c->normk_host[q]);
            break;
        }
        k += B;
        if (k >= max_cycles) {
            const double rn = as_double(c->normk_host[B]);
            rr = sc > 0 ? rn / sc : rn;
            st = fail(RZPIC_ENOTCONV, "multigrid: relative residual %.3e after %d cycles", rr, k);
            break;
        }
        if (B == 0) {  // no snapshots: one cycle, then the test again
            HIPCHK(cycles_run(1));
            ++k;
        }
        // a solve that needs more than its hint: batches of 2, 4, 8, ...
        batch = next;
        next = next * 2 < c->ring_slots ? next * 2 : c->ring_slots;
    }
    if (hint) *hint = k > 0 ? k : 1;
    *k_out = k;
    *relres = rr;
    return st;
}

// prepared: the step's grid launch (mg_finalize) has formed eps and f,
// restricted eps and set the Dirichlet values of both phi buffers.
rzpic_status solve_impl(rzpic_ctx *c, double t, bool prepared, int32_t *cycles, double *relres)
{
    const int nr = c->c.nr, nz = c->c.nz;
    const double V = c->c.V_dc + c->c.V_rf * std::sin(kTwoPi * c->c.f_rf * t);
    if (!prepared) {
        int threads = 256, blocks = (c->nn + threads - 1) / threads;
        RZ_LAUNCH(k_prep_solve, dim3(blocks), dim3(threads), 0, c->st, c->nn,
                           (const double *)c->rho, (const double *)c->chi, c->eps,
                           c->mixed ? c->mg.eps32[c->L] : nullptr, c->f);
        HIPCHK(hipGetLastError());
        HIPCHK(mg_restrict_eps(c->mg, c->mixed, c->st));
        if (c->c.circuit_C > 0.0) {
            HIPCHK(mg_set_bc(c->phiP, nr, nz, 0.0, c->st));
            HIPCHK(mg_set_bc(c->phiP_alt, nr, nz, 0.0, c->st));
        } else {
            HIPCHK(mg_set_bc(c->phi, nr, nz, V, c->st));
            HIPCHK(mg_set_bc(c->phi_alt, nr, nz, V, c->st));
        }
    }
    int k = 0;
    double rr = c->last_relres;
    if (c->c.circuit_C > 0.0) {
        // external circuit: the charge solution (electrode at 0 V) and the
        // unit Laplace solution (electrode at 1 V) with the same operator,
        // then the circuit update and phi = phi_P + V phi_L
        HIPCHK(mg_set_bc(c->phiL, nr, nz, 1.0, c->st));
        HIPCHK(mg_set_bc(c->phiL_alt, nr, nz, 1.0, c->st));
        int k2 = 0;
        double rr2 = rr;
        rzpic_status s1 = run_cycles(c, 0.0, c->phiP, c->phiP_alt, c->f, c->c.mg_fixed_cycles,
                                     c->c.mg_tol, c->c.mg_max_cycles, cycles || relres, &k, &rr,
                                     &c->cyc_hint[1]);
        if (s1 != RZPIC_OK && s1 != RZPIC_ENOTCONV) return s1;
        rzpic_status s2 = run_cycles(c, 1.0, c->phiL, c->phiL_alt, c->fzero,
                                     c->c.mg_fixed_cycles, c->c.mg_tol, c->c.mg_max_cycles,
                                     cycles || relres, &k2, &rr2, &c->cyc_hint[2]);
        if (s2 != RZPIC_OK && s2 != RZPIC_ENOTCONV) return s2;
        CircuitArgs a{};
        a.nr = nr;
        a.rule = c->c.chi_face;
        a.hr = c->hr;
        a.hz = c->hz;
        a.C = c->c.circuit_C;
        a.Vs = V;
        a.eps = c->eps;
        a.rho = c->rho;
        a.vol = c->vol;
        a.phiP = c->phiP;
        a.phiL = c->phiL;
        a.tally = c->tally;
        for (int s = 0; s < 2; ++s) {
            a.q[s] = c->sp[s].bound ? c->sp[s].v.q : 0.0;
            a.quantum[s] = c->quantum[s];
        }
        a.st = c->circ;
        HIPCHK(launch_circuit(a, c->st));
        HIPCHK(launch_combine(c->nn, c->phiP, c->phiL, c->circ, c->phi, c->st));
        c->last_cycles = k > k2 ? k : k2;
        c->last_relres = rr > rr2 ? rr : rr2;
        if (cycles) *cycles = c->last_cycles;
        if (relres) *relres = c->last_relres;
        return s1 != RZPIC_OK ? s1 : s2;
    }
    rzpic_status st = run_cycles(c, V, c->phi, c->phi_alt, c->f, c->c.mg_fixed_cycles,
                                 c->c.mg_tol, c->c.mg_max_cycles, cycles || relres, &k, &rr,
                                 &c->cyc_hint[0]);
    c->last_cycles = k;
    c->last_relres = rr;
    if (cycles) *cycles = k;
    if (relres) *relres = c->last_relres;
    return st;
}

// prepared: the grid of this step was finalized by the previous step's
// list maintenance (step pipelining), which leaves the deposit grids and the
// Monte Carlo counters as they were: they are cleared here instead, before
// the pass (the ion grid only if the ions move in this step).
rzpic_status efield_impl(rzpic_ctx *c, bool prepared = false, bool ions = true)
{
    unsigned long long *z0 = prepared ? c->acc[0] : nullptr;
    unsigned long long *z1 = prepared && ions ? c->acc[1] : nullptr;
    unsigned long long *cl = prepared ? c->mcstat : nullptr;
    const int ncl = prepared ? 2 * (1 + kMaxProc) : 0;
    if (c->mixed)
        HIPCHK(launch_efield<float>(c->c.nr, c->c.nz, c->hr, c->hz, c->phi, c->er, c->ez,
                                    (float2 *)c->E2, c->st, z0, z1, cl, ncl));
    else
        HIPCHK(launch_efield<double>(c->c.nr, c->c.nz, c->hr, c->hz, c->phi, c->er, c->ez,
                                     (double2 *)c->E2, c->st, z0, z1, cl, ncl));
    return RZPIC_OK;
}

// ions: the ions move in the coming step (their chi term on, their deposit
// rebuilt by it); otherwise their deposit is kept and they add charge only.
GridArgs grid_args(rzpic_ctx *c, int zero_acc, bool ions = true)
{
    GridArgs g{};
    g.nr = c->c.nr;
    g.nz = c->c.nz;
    g.nn = c->nn;
    g.hr = c->hr;
    g.hz = c->hz;
    g.dt = c->c.dt;
    g.acc0 = c->acc[0];
    g.acc1 = c->acc[1];
    g.quantum0 = c->quantum[0];
    g.quantum1 = c->quantum[1];
    g.q0 = c->sp[0].v.q;
    g.q1 = c->sp[1].v.q;
    g.m0 = c->sp[0].bound ? c->sp[0].v.m : 1.0;
    g.m1 = c->sp[1].bound ? c->sp[1].v.m : 1.0;
    g.vol = c->vol;
    g.dens0 = c->dens[0];
    g.dens1 = c->dens[1];
    g.rho = c->rho;
    g.chi = c->chi;
    g.eps = c->eps;
    g.f = c->f;
    g.eps32 = c->mixed ? c->mg.eps32[c->L] : nullptr;
    g.zero_acc = zero_acc;
    g.acc0w = c->acc[0];
    g.acc1w = c->acc[1];
    g.status = c->status;
    g.dt1 = dt_of(c, 1);
    g.friedman = c->c.damping == RZPIC_DAMP_FRIEDMAN ? 1 : 0;
    g.theta = c->c.theta;
    g.ion_chi = ions ? 1 : 0;
    g.keep1 = ions ? 0 : 1;
    return g;
}

rzpic_status finalize_impl(rzpic_ctx *c, int zero_acc)
{
    HIPCHK(launch_finalize(grid_args(c, zero_acc), c->st));
    return RZPIC_OK;
}

template <typename T> rzpic_status deposit_impl(rzpic_ctx *c)
{
    for (int s = 0; s < 2; ++s) HIPCHK(launch_fill_u64(c->acc[s], c->nn, c->st));
    for (int s = 0; s < 2; ++s) TRY(run_pass<T>(c, s, M_DEP | M_MARK, 0));
    for (int s = 0; s < 2; ++s)
        if (c->children_pending[s]) TRY(run_staged<T>(c, s, M_DEP));
    return RZPIC_OK;
}

// Resize of species s in step `step` (the key of the zero-order draws).  The
// zero-order form marks the particles it removes (w = -1); the caller
// compacts (zero_order_compact).
template <typename T> rzpic_status resize_impl(rzpic_ctx *c, int s, int64_t step)
{
    ResizeKey k{};
    k.zero_order = c->c.resize_mode == RZPIC_RESIZE_ZERO_ORDER;
    k.s = s;
    k.seed = c->c.seed;
    k.step = (uint32_t)step;
    HIPCHK(launch_resize<T>(parts_of<T>(c->sp[s].v), c->cnt + s, c->sp[s].ch, c->clrec + s, k,
                            c->c.resize_wcoef, 0.5 * c->hr, c->sp[s].cap, c->status, c->st));
    return RZPIC_OK;
}

// Compaction after a zero-order resize of the species in `which` (bit s).
template <typename T> rzpic_status zero_order_compact(rzpic_ctx *c, int which)
{
    if (c->c.resize_mode != RZPIC_RESIZE_ZERO_ORDER) return RZPIC_OK;
    for (int s = 0; s < 2; ++s)
        if ((which >> s) & 1)
            HIPCHK(launch_dead_scan<T>(parts_of<T>(c->sp[s].v), c->cnt + s, c->sp[s].ch, c->st));
    return run_fixup<T>(c, which);
}

// Scratch of the tile sort of species s (sized by its capacity).
rzpic_status sort_alloc(rzpic_ctx *c, int s)
{
    SpeciesState &ss = c->sp[s];
    if (ss.sort_off) return RZPIC_OK;
    const size_t cap = (size_t)ss.cap + kChunk;
    const size_t es = c->mixed ? sizeof(float) : sizeof(double);
    // Segments (one wavefront each walks its segment serially): at most 8192
    // of them, which keeps every CU busy, and at most 2^22 (tile, segment)
    // counts for the scan; at least 256 particles.
    int64_t seg = 256;
    while (((int64_t)cap + seg - 1) / seg > 8192 ||
           ((int64_t)cap + seg - 1) / seg * c->nt > ((int64_t)1 << 22))
        seg *= 2;
    ss.sort_seg = seg;
    ss.sort_nseg = ((int64_t)cap + seg - 1) / seg;
    const size_t M = (size_t)ss.sort_nseg * c->nt + 1;
    auto get = [&](void **p, size_t bytes) -> rzpic_status {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            *p = nullptr;
            free_sort(ss);
            return fail(RZPIC_ENOMEM, "hipMalloc(%zu) for the tile sort failed", bytes);
        }
        return RZPIC_OK;
    };
    for (int f = 0; f < 8; ++f) TRY(get(&ss.sort_buf[f], cap * es));
    TRY(get(&ss.sort_buf[8], cap * sizeof(uint64_t)));
    if (ss.v.at) TRY(get(&ss.sort_buf[9], cap * es));
    TRY(get((void **)&ss.sort_off, M * sizeof(int64_t)));
    TRY(get((void **)&ss.sort_part, 4096 * sizeof(int64_t)));
    TRY(get((void **)&ss.tile_pb, sizeof(int64_t)));
    TRY(get((void **)&ss.tile_win, (size_t)kMaxWaves * sizeof(int4)));
    HIPCHK(launch_fill_u64((unsigned long long *)ss.tile_pb, 1, c->st));
    return RZPIC_OK;
}

// Stable counting sort of species s by tile, then the window plan of its
// tiled pass.  Positions are unchanged, so the deposit grids stay valid.
template <typename T> rzpic_status sort_impl(rzpic_ctx *c, int s)
{
    if (c->nt > kMaxTiles)
        return fail(RZPIC_EINVAL, "%d tiles exceed %d: enlarge tile_z / tile_r", c->nt, kMaxTiles);
    TRY(sort_alloc(c, s));
    SpeciesState &ss = c->sp[s];
    SortArgs<T> a{};
    a.p = parts_of<T>(ss.v);
    Parts<T> t{};
    T **tf[8] = {&t.r, &t.z, &t.vr, &t.vt, &t.vz, &t.ar, &t.az, &t.w};
    for (int f = 0; f < 8; ++f) *tf[f] = (T *)ss.sort_buf[f];
    t.id = (uint64_t *)ss.sort_buf[8];
    t.at = (T *)ss.sort_buf[9];
    a.tmp = t;
    a.cnt = c->cnt + s;
    a.hr = c->hr;
    a.hz = c->hz;
    a.nr = c->c.nr;
    a.nz = c->c.nz;
    a.tile_z = c->c.tile_z;
    a.tile_r = c->c.tile_r;
    a.ntr = c->ntr;
    a.nt = c->nt;
    a.kbits = c->kbits;
    a.seg = ss.sort_seg;
    a.nseg = ss.sort_nseg;
    a.off = ss.sort_off;
    a.part = ss.sort_part;
    a.tile_pb = ss.tile_pb;
    a.tile_win = ss.tile_win;
    a.nb = tiled_blocks(c, s);
    HIPCHK(launch_sort<T>(a, c->st));
    ss.tile_nb = a.nb;
    return RZPIC_OK;
}

// Timing marks of one step: 0 start, 1 after finalize, 2 after solve,
// 3 after E, 4/5 around the fused pass kernel, 6 after the collision kernels
// and the slice reduction, 7 after list maintenance, 8 after a weight split
// (if any), 9 end (after a tile sort, if any).
rzpic_status flush_timing(rzpic_ctx *c);

void mark(rzpic_ctx *c, int k)
{
    if (!c->timing || c->ev_used >= rzpic_ctx::kPool) return;
    (void)hipEventRecord(c->evpool[(size_t)c->ev_used * rzpic_ctx::kEvPerStep + k], c->st);
}

rzpic_status flush_timing(rzpic_ctx *c)
{
    if (c->ev_used == 0) return RZPIC_OK;
    const int E = rzpic_ctx::kEvPerStep;
    HIPCHK(hipEventSynchronize(c->evpool[(size_t)(c->ev_used - 1) * E + E - 1]));
    auto el = [&](hipEvent_t a, hipEvent_t b) {
        float t = 0.f;
        (void)hipEventElapsedTime(&t, a, b);
        return (double)t;
    };
    for (int st = 0; st < c->ev_used; ++st) {
        hipEvent_t *e = &c->evpool[(size_t)st * E];
        c->acc_ms[0] += el(e[0], e[9]);
        c->acc_ms[1] += el(e[1], e[2]);
        c->acc_ms[2] += el(e[4], e[5]);
        c->acc_ms[3] += el(e[5], e[6]);
        c->acc_ms[4] += el(e[0], e[1]) + el(e[2], e[4]);
        c->acc_ms[5] += el(e[6], e[7]);
        c->acc_ms[6] += el(e[7], e[8]);
        c->acc_ms[7] += el(e[8], e[9]);
    }
    c->acc_steps += c->ev_used;
    c->ev_used = 0;
    return RZPIC_OK;
}

// Whether step pipelining can prepare the grid of the step after a step
// that makes no weight split: the split solve path (mg_prep), one operator
// per step (no circuit) and a fixed number of cycles.
static bool can_prepare(const rzpic_ctx *c)
{
    return c->mg.split && c->c.circuit_C <= 0.0 && c->c.mg_fixed_cycles > 0;
}

// pipe: step pipelining (a directly launched step with rzpic_set_step_pipeline
// on); this step then skips its grid preparation when the previous step made
// it, and makes the next step's when it can.
template <typename T> rzpic_status step_impl(rzpic_ctx *c, int64_t n, bool pipe = false)
{
    TRY(need_both(c));
    if (c->children_pending[0] || c->children_pending[1])
        return fail(RZPIC_ESTATE, "new particles are staged: call rzpic_compact first");
    if (c->timing && c->ev_used >= rzpic_ctx::kPool) TRY(flush_timing(c));
    const bool pre = pipe && c->prepared == n;
    c->prepared = -1;
    if (!pre) HIPCHK(list_tail_flush(c->tail, c->st));
    mark(c, 0);
    // subcycled ions move only in every K-th step
    const bool ions = n % ion_K(c) == ion_K(c) - 1;
    if (!pre) {
        // finalize, eps restriction, Dirichlet values of both phi buffers and
        // the Monte Carlo counters cleared, in one launch
        const double t = (double)(n + 1) * c->c.dt;
        const double V = c->c.V_dc + c->c.V_rf * std::sin(kTwoPi * c->c.f_rf * t);
        const bool circ = c->c.circuit_C > 0.0;  // then phi_P takes the electrode at 0 V
        HIPCHK(mg_finalize(grid_args(c, 1, ions), c->mg, c->mixed, circ ? c->phiP : c->phi,
                           circ ? c->phiP_alt : c->phi_alt, circ ? 0.0 : V, c->mcstat,
                           2 * (1 + kMaxProc), c->st));
    }
    mark(c, 1);
    c->prep_ready = pre;
    const rzpic_status ss = solve_impl(c, (double)(n + 1) * c->c.dt, true, nullptr, nullptr);
    c->prep_ready = false;
    TRY(ss);
    // what of the previous step's list maintenance the way-down launches did
    // not take (fewer than three cycles) runs before the pass reads the lists
    HIPCHK(list_tail_flush(c->tail, c->st));
    c->acc_cycles += c->last_cycles;
    mark(c, 2);
    TRY(efield_impl(c, pre, ions));
    mark(c, 3);
    TRY(run_pass_both<T>(c, (uint32_t)n, ions));
    if (!ions)  // the ions keep state and deposit; their compaction only appends children
        HIPCHK(launch_fill_u64(c->sp[1].ch.dead, c->sp[1].nchunks_max, c->st));
    c->children_pending[0] = c->children_pending[1] = c->sp[0].v.mc_model == RZPIC_MC_ELECTRON;
    c->children_scanned = false;
    // Weight split, then the deposit from scratch; a tile sort due at this
    // step runs in between (the fixed-point deposit does not depend on the
    // particle order, and the sorted order gives the deposit its windows).
    const bool resize = c->c.resize_every > 0 && n % c->c.resize_every == c->c.resize_every - 1;
    const bool sort = c->c.sort_every > 0 && n % c->c.sort_every == c->c.sort_every - 1;
    // step pipelining: the deposit is final once the collisions have run
    // (no weight split follows), so the next step's grid preparation runs
    // in the list maintenance's launches; it leaves the deposit grids and
    // the counters to the next step's E launch
    const bool prep_next = pipe && !resize && can_prepare(c) && n + 1 <= 0xFFFFFFFELL;
    NextGrid next{};
    // the hole filling and appending go with the next step's way down,
    // unless a tile sort of this step reads the compacted particles
    next.defer = !sort;
    if (prep_next) {
        const int64_t m = n + 1;
        const double t = (double)(m + 1) * c->c.dt;
        next.V = c->c.V_dc + c->c.V_rf * std::sin(kTwoPi * c->c.f_rf * t);
        next.g = grid_args(c, 0, m % ion_K(c) == ion_K(c) - 1);
    }
    TRY(run_fixup<T>(c, 3, prep_next ? &next : nullptr));
    mark(c, 7);
    if (resize) {
        for (int s = 0; s < 2; ++s) TRY(resize_impl<T>(c, s, n));
        TRY(zero_order_compact<T>(c, 3));
    }
    mark(c, 8);
    if (sort)
        for (int s = 0; s < 2; ++s) TRY(sort_impl<T>(c, s));
    if (resize) {
        for (int s = 0; s < 2; ++s) HIPCHK(launch_fill_u64(c->acc[s], c->nn, c->st));
        for (int s = 0; s < 2; ++s) TRY(run_pass<T>(c, s, M_DEP, 0));
    }
    mark(c, 9);
    if (c->timing) c->ev_used++;
    if (prep_next) c->prepared = n + 1;
    return RZPIC_OK;
}

}  // namespace

// ===========================================================================
// Helpers of the batched step (batch.hip).

rzpic_status rz_fail(rzpic_status s, const char *msg) { return fail(s, "%s", msg); }

hipStream_t rz_stream(const rzpic_ctx *c) { return c->st; }

// What a pipelined step left of its list maintenance, launched on the
// context's stream (batches and gradient windows read the particles).
rzpic_status rz_settle(rzpic_ctx *c)
{
    HIPCHK(list_tail_flush(c->tail, c->st));
    return RZPIC_OK;
}

// Whether a context can join a batch: its step must launch kernels only (no
// synchronisation, no timing events) and both species must be bound.
int rz_batchable(const rzpic_ctx *c, std::string &why)
{
    if (!c->sp[0].bound || !c->sp[1].bound) {
        why = "both species must be bound";
        return 0;
    }
    if (c->c.mg_fixed_cycles <= 0) {
        why = "the multigrid must run a fixed number of cycles (mg_fixed_cycles > 0)";
        return 0;
    }
    if (c->timing) {
        why = "step timing must be off";
        return 0;
    }
    if (c->children_pending[0] || c->children_pending[1]) {
        why = "new particles are staged: call rzpic_compact first";
        return 0;
    }
    return 1;
}

// ===========================================================================
// Helpers of the adjoint window (adjoint.hip).

Mesh rz_mesh(const rzpic_ctx *c) { return mesh_of(c); }

SpeciesK rz_species(const rzpic_ctx *c, int s) { return species_of(c, s); }

// Tolerance-mode cycles on u (u_alt its partner buffer) for the system the
// caller prepared in the context (eps restricted, f, Dirichlet values).
rzpic_status rz_cycles(rzpic_ctx *c, double V, double *&u, double *&u_alt, double tol,
                       int max_cycles, int *cycles, double *relres)
{
    return run_cycles(c, V, u, u_alt, c->f, 0, tol, max_cycles, true, cycles, relres,
                      &c->cyc_hint[3]);
}

// ===========================================================================
// C ABI

// Calls that change what the next step's grid preparation reads (particles,
// deposits, potentials, voltages, solver settings) drop a preparation made by
// step pipelining; the next step then prepares its grid itself.
static rzpic_status unprepare(rzpic_ctx *c)
{
    c->prepared = -1;
    HIPCHK(list_tail_flush(c->tail, c->st));
    return RZPIC_OK;
}

// Calls that read the particles or their counts first launch what a
// pipelined step left of its list maintenance.
static rzpic_status settle(rzpic_ctx *c)
{
    HIPCHK(list_tail_flush(c->tail, c->st));
    return RZPIC_OK;
}

extern "C" {

const char *rzpic_last_error(void) { return g_err.c_str(); }

void rzpic_constants(double out[6])
{
    out[0] = kE;
    out[1] = kMe;
    out[2] = kAmu;
    out[3] = kEps0;
    out[4] = kKb;
    out[5] = kTwoPi;
}

rzpic_status rzpic_create(const rzpic_config *cfg, void *stream, rzpic_ctx **out)
{
    if (!cfg || !out) return fail(RZPIC_EINVAL, "null argument");
    *out = nullptr;
    const rzpic_config &k = *cfg;
    if (k.nr < 3 || k.nr - 1 > kMaxLine)
        return fail(RZPIC_EINVAL, "nr = %d: need 3 <= nr <= %d", k.nr, kMaxLine + 1);
    if (k.nz < 3 || !is_pow2(k.nz - 1))
        return fail(RZPIC_EINVAL, "nz = %d: nz-1 must be a power of two >= 2", k.nz);
    if (!(k.R > 0) || !(k.L > 0) || !(k.dt > 0))
        return fail(RZPIC_EINVAL, "R, L and dt must be positive");
    if (k.precision != RZPIC_FP64 && k.precision != RZPIC_MIXED)
        return fail(RZPIC_EINVAL, "precision must be RZPIC_FP64 or RZPIC_MIXED");
    if (k.weighting != RZPIC_W_ZR2 && k.weighting != RZPIC_W_ZR)
        return fail(RZPIC_EINVAL, "unknown weighting %d", k.weighting);
    if (k.chi_face != RZPIC_FACE_AVG && k.chi_face != RZPIC_FACE_MAX)
        return fail(RZPIC_EINVAL, "unknown chi_face %d", k.chi_face);
    if (k.mg_fixed_cycles < 0 || (k.mg_fixed_cycles == 0 && (k.mg_max_cycles < 1 || !(k.mg_tol > 0))))
        return fail(RZPIC_EINVAL, "need mg_fixed_cycles > 0, or mg_max_cycles >= 1 and mg_tol > 0");
    if (k.fixed_point_bits < 0 || k.fixed_point_bits > 52)
        return fail(RZPIC_EINVAL, "fixed_point_bits = %d out of [0, 52]", k.fixed_point_bits);
    if (k.precision == RZPIC_MIXED && k.fixed_point_bits > 30)
        return fail(RZPIC_EINVAL,
                    "fixed_point_bits = %d: the mixed form forms 32-bit contributions (at most 30)",
                    k.fixed_point_bits);
    if (k.resize_every < 0 || (k.resize_every > 0 && !(k.resize_wcoef > 0)))
        return fail(RZPIC_EINVAL, "resize_every > 0 needs resize_wcoef > 0");
    if (k.sort_every < 0 || k.tile_z < 0 || k.tile_r < 0)
        return fail(RZPIC_EINVAL, "sort_every, tile_z and tile_r must be >= 0");
    if (!(k.circuit_C >= 0.0) || !std::isfinite(k.circuit_C))
        return fail(RZPIC_EINVAL, "circuit_C must be finite and >= 0");
    if (k.ion_subcycle < 0) return fail(RZPIC_EINVAL, "ion_subcycle must be >= 0");
    if (k.push_form != RZPIC_PUSH_LOCAL && k.push_form != RZPIC_PUSH_XYZ)
        return fail(RZPIC_EINVAL, "unknown push_form %d", k.push_form);
    if (k.resize_mode != RZPIC_RESIZE_SPLIT && k.resize_mode != RZPIC_RESIZE_ZERO_ORDER)
        return fail(RZPIC_EINVAL, "unknown resize_mode %d", k.resize_mode);
    if (k.damping != RZPIC_DAMP_D1 && k.damping != RZPIC_DAMP_FRIEDMAN)
        return fail(RZPIC_EINVAL, "unknown damping %d", k.damping);
    if (k.damping == RZPIC_DAMP_FRIEDMAN && k.push_form != RZPIC_PUSH_LOCAL)
        return fail(RZPIC_EINVAL, "Friedman damping takes the local push (push_form 0)");
    if (k.damping == RZPIC_DAMP_FRIEDMAN && !(k.theta >= 0.0 && k.theta <= 1.0))
        return fail(RZPIC_EINVAL, "Friedman damping: theta = %g outside [0, 1]", k.theta);

    rzpic_ctx *c = new rzpic_ctx();
    c->c = k;
    if (c->c.fixed_point_bits == 0) c->c.fixed_point_bits = k.precision == RZPIC_MIXED ? 26 : 46;
    c->st = (hipStream_t)stream;
    c->mixed = k.precision == RZPIC_MIXED;
    c->hr = k.R / (double)(k.nr - 1);
    c->hz = k.L / (double)(k.nz - 1);
    c->nn = k.nr * k.nz;
    if (c->c.tile_z == 0) c->c.tile_z = 16;
    if (c->c.tile_r == 0) c->c.tile_r = 32;
    c->ntr = (k.nr - 2) / c->c.tile_r + 1;
    c->nt = ((k.nz - 2) / c->c.tile_z + 1) * c->ntr;
    while ((1 << c->kbits) < c->nt) ++c->kbits;
    if (k.sort_every > 0 && c->nt > kMaxTiles) {
        const int nt = c->nt;
        delete c;
        return fail(RZPIC_EINVAL, "%d tiles exceed %d: enlarge tile_z / tile_r", nt, kMaxTiles);
    }
    int L = 0;
    while ((1 << L) < k.nz - 1) ++L;
    c->L = L;
    auto bail = [&](rzpic_status s) {
        std::string keep = g_err;
        rzpic_destroy(c);
        g_err = keep;
        return s;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(RZPIC_EHIP, "no HIP device"));
    int v = 0;
    (void)hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, c->device);
    c->cus = v > 0 ? v : 1;
    (void)hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
    c->lds_block = (size_t)v;
    (void)hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device);
    c->lds_cu = v > 0 ? (size_t)v : c->lds_block;
    // the multigrid's down leg holds a whole z-column (8 values per node) in LDS
    if ((size_t)64 * k.nz > c->lds_block)
        return bail(fail(RZPIC_EINVAL, "nz = %d: a z-column of the multigrid does not fit in "
                                       "one workgroup's LDS (%zu bytes)",
                         k.nz, c->lds_block));
    if (const char *e = std::getenv("RZPIC_PASS_THREADS")) {
        int t = std::atoi(e);
        if (t == 256 || t == 512 || t == 1024) c->pass_threads = t;
    }
    const size_t nn = (size_t)c->nn;
    rzpic_status s;
#define A(p, n)                                  \
    if ((s = dalloc(c, &(p), (n))) != RZPIC_OK) \
        return bail(s);
    A(c->phi, nn) A(c->phi_alt, nn) A(c->rho, nn) A(c->chi, nn) A(c->er, nn) A(c->ez, nn) A(c->dens[0], nn)
    A(c->dens[1], nn) A(c->vol, nn) A(c->f, nn) A(c->eps, nn)
    {
        double2 *e2;
        A(e2, nn) c->E2 = e2;
    }
    A(c->acc[0], nn) A(c->acc[1], nn)
    A(c->cnt, 2) A(c->fix, 2) A(c->crec, 1) A(c->clrec, 2) A(c->tally, 6)
    A(c->mcstat, 2 * (1 + kMaxProc)) A(c->norm, 2) A(c->status, 1) A(c->psteps, 2)
    A(c->normk, rzpic_ctx::kRingMax + 1)
    {
        // snapshots of the finest level for batched tolerance-mode cycles,
        // within 64 MiB
        const size_t per = nn * sizeof(double);
        size_t cap = per > 0 ? ((size_t)64 << 20) / per : 0;
        const int slots = (int)(cap < (size_t)rzpic_ctx::kRingMax ? cap : rzpic_ctx::kRingMax);
        if (slots > 0) A(c->ring, (size_t)slots * nn)
        c->ring_slots = slots;
        void *h = nullptr;
        if (hipHostMalloc(&h, (rzpic_ctx::kRingMax + 2) * sizeof(unsigned long long)) !=
            hipSuccess)
            return bail(fail(RZPIC_ENOMEM, "hipHostMalloc of the residual buffer failed"));
        c->normk_host = (unsigned long long *)h;
    }
    if (k.circuit_C > 0.0) {
        A(c->phiP, nn) A(c->phiP_alt, nn) A(c->phiL, nn) A(c->phiL_alt, nn) A(c->fzero, nn)
        A(c->circ, 1)
    }
    // LDS privatisation of the whole deposit grid when it fits.
    // (32-bit elements for FP32 particles, see deposit4_lds32)
    const size_t lds_need = nn * (c->mixed ? sizeof(uint32_t) : sizeof(unsigned long long)) + 1024;
    if (lds_need <= c->lds_block && !std::getenv("RZPIC_NO_LDS")) {
        // blocks per CU: as many as LDS allows up to the 32-wave limit
        int per_cu = (int)(c->lds_cu / lds_need);
        int wave_cap = 2048 / c->pass_threads;
        const int occ = c->mixed ? pass2_lds_blocks_per_cu<float>(c->pass_threads, lds_need - 1024)
                                 : pass2_lds_blocks_per_cu<double>(c->pass_threads, lds_need - 1024);
        if (per_cu < 1) per_cu = 1;
        if (per_cu > wave_cap) per_cu = wave_cap;
        if (per_cu > occ) per_cu = occ;
        c->slice_blocks = c->cus * per_cu;
        if (const char *e = std::getenv("RZPIC_SLICE_BLOCKS")) {
            int b = std::atoi(e);
            if (b > 0 && b <= 65536) c->slice_blocks = b;
        }
        A(c->slices, (size_t)c->slice_blocks * nn)
        c->lds_ok = c->lds_form = true;
        c->lds_resident = c->slice_blocks;
    } else {
        c->tile_per_cu = c->mixed ? pass2_tiled_blocks_per_cu<float>(c->pass_threads)
                                  : pass2_tiled_blocks_per_cu<double>(c->pass_threads);
    }
    // multigrid levels
    MgLevels &m = c->mg;
    m.L = L;
    m.nr = k.nr;
    m.chi_face = k.chi_face;
    m.hr = c->hr;
    // u and f of the coarse levels 1..L-1 in one block, level by level (the
    // layout the single-workgroup coarse solve holds in LDS)
    size_t coarse_elems = 0;
    for (int l = 1; l < L; ++l) coarse_elems += 2 * (((size_t)1 << l) + 1) * (size_t)k.nr;
    float *cuf32 = nullptr;
    double *cuf64 = nullptr;
    if (c->mixed) {
        A(cuf32, coarse_elems) m.coarse_uf = cuf32;
    } else {
        A(cuf64, coarse_elems) m.coarse_uf = cuf64;
    }
    for (int l = 1; l <= L; ++l) {
        m.nzl[l] = (1 << l) + 1;
        m.hzl[l] = c->hz * (double)(1 << (L - l));
        size_t sz = (size_t)m.nzl[l] * k.nr;
        if (l == L) {
            m.eps64[l] = c->eps;
        } else {
            A(m.eps64[l], sz)
        }
        if (c->mixed) {
            A(m.eps32[l], sz)
            if (l == L) {
                A(m.u32[l], sz) A(m.f32[l], sz)
            } else {
                m.u32[l] = cuf32;
                m.f32[l] = cuf32 + sz;
                cuf32 += 2 * sz;
            }
        } else if (l < L) {
            m.u64[l] = cuf64;
            m.f64[l] = cuf64 + sz;
            cuf64 += 2 * sz;
        }
    }
    {
        // cycle path: the split form unless RZPIC_MG_PATH names another
        // ("block", "multi" or "long"; for tests and measurements)
        int path = 0;
        if (const char *e = std::getenv("RZPIC_MG_PATH")) {
            if (!std::strcmp(e, "block")) path = 1;
            else if (!std::strcmp(e, "multi")) path = 2;
            else if (!std::strcmp(e, "long")) path = 3;
        }
        // the split cycle's way up: one launch (default) or the coarse
        // levels in one workgroup and then the finest level's sweep
        // (RZPIC_MG_UP=coarse; the same values, for tests and measurements)
        const char *ue = std::getenv("RZPIC_MG_UP");
        m.split_coarse = ue && !std::strcmp(ue, "coarse") ? 1 : 0;
        mg_plan(m, c->mixed, c->lds_block, path);
    }
    if (m.one_block || m.split) {
        const size_t tab = (size_t)m.line_off[L + 1] * m.tab_stride;
        if (c->mixed) {
            float *t;
            A(t, tab) m.tab = t;
        } else {
            double *t;
            A(t, tab) m.tab = t;
        }
        A(m.res, nn)
        A(m.cf64, 5 * nn)
    }
#undef A
    // weighting volumes (Sec. 2.4, radial neighbours clamped to the axis and
    // the wall, half axial cells on the electrodes)
    std::vector<double> vol(nn);
    const double PI = 3.141592653589793;
    for (int i = 0; i < k.nz; ++i) {
        double zf = (i == 0 || i == k.nz - 1) ? 0.5 * c->hz : c->hz;
        for (int j = 0; j < k.nr; ++j) {
            int jp = j + 1 < k.nr ? j + 1 : k.nr - 1, jm = j > 0 ? j - 1 : 0;
            double rj = j * c->hr, rp = jp * c->hr, rm = jm * c->hr, rf;
            if (k.weighting == RZPIC_W_ZR) rf = (PI / 3.0) * (rp * (rj + rp) - rm * (rj + rm));
            else rf = 0.5 * PI * (rp * rp - rm * rm);
            vol[(size_t)i * k.nr + j] = rf * zf;
        }
    }
    if (hipMemcpy(c->vol, vol.data(), nn * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(RZPIC_EHIP, "table upload failed"));
    *out = c;
    return RZPIC_OK;
}

rzpic_status rzpic_destroy(rzpic_ctx *c)
{
    if (!c) return RZPIC_OK;
    // the caller's particle arrays end compacted: what a pipelined step kept
    // of its list maintenance runs first
    (void)list_tail_flush(c->tail, c->st);
    if (c->st) (void)hipStreamSynchronize(c->st);
    else (void)hipDeviceSynchronize();
    for (void *p : c->allocs) (void)hipFree(p);
    for (int s = 0; s < 2; ++s) {
        for (int a = 0; a < 2; ++a)
            for (int f = 0; f < 9; ++f)
                if (c->sp[s].stage[a][f]) (void)hipFree(c->sp[s].stage[a][f]);
        if (c->sp[s].sigma.p) (void)hipFree(c->sp[s].sigma.p);
        free_sort(c->sp[s]);
    }
    for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
    for (hipGraphExec_t &g : c->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    if (c->normk_host) (void)hipHostFree(c->normk_host);
    delete c;
    return RZPIC_OK;
}

rzpic_status rzpic_set_stream(rzpic_ctx *c, void *stream)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    if (c->tail.stage) {
        // the new stream does not wait for the old one: what a pipelined
        // step left runs and ends before the switch
        HIPCHK(list_tail_flush(c->tail, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
    }
    TRY(unprepare(c));
    c->st = (hipStream_t)stream;
    return RZPIC_OK;
}

rzpic_status rzpic_bind_species(rzpic_ctx *c, int32_t s, const rzpic_species_view *v)
{
    if (!c || !v) return fail(RZPIC_EINVAL, "null argument");
    TRY(unprepare(c));
    if (s < 0 || s > 1) return fail(RZPIC_EINVAL, "species %d out of range", s);
    if (!v->r || !v->z || !v->vr || !v->vt || !v->vz || !v->ar || !v->az || !v->w || !v->id)
        return fail(RZPIC_EINVAL, "species %d: null particle array", s);
    // particle kernels address the arrays by 32-bit byte offsets (8-byte ids)
    if (v->capacity < 1 || v->capacity > ((int64_t)1 << 29) - kChunk)
        return fail(RZPIC_EINVAL, "species %d: capacity %lld out of range", s, (long long)v->capacity);
    if (!(v->m > 0) || !(v->w_ref > 0))
        return fail(RZPIC_EINVAL, "species %d: need m > 0 and w_ref > 0", s);
    if (v->mc_model < RZPIC_MC_NONE || v->mc_model > RZPIC_MC_ION)
        return fail(RZPIC_EINVAL, "species %d: unknown mc_model", s);
    if (v->mc_model == RZPIC_MC_ELECTRON && s != 0)
        return fail(RZPIC_EINVAL, "the electron collision model is species 0");
    if (c->c.push_form == RZPIC_PUSH_XYZ && !v->at)
        return fail(RZPIC_EINVAL, "species %d: the global X-Y-Z push needs the a_theta array", s);
    HIPCHK(c->st ? hipStreamSynchronize(c->st) : hipDeviceSynchronize());
    SpeciesState &ss = c->sp[s];
    for (int a = 0; a < 2; ++a)
        for (int f = 0; f < 9; ++f)
            if (ss.stage[a][f]) {
                (void)hipFree(ss.stage[a][f]);
                ss.stage[a][f] = nullptr;
            }
    free_sort(ss);
    ss.v = *v;
    if (c->c.push_form != RZPIC_PUSH_XYZ) ss.v.at = nullptr;  // the local form keeps no a_theta
    ss.cap = v->capacity;
    ss.bound = true;
    c->quantum[s] = v->w_ref * std::ldexp(1.0, -c->c.fixed_point_bits);
    const int64_t nch = (v->capacity + kChunk - 1) / kChunk + 1;
    ss.nchunks_max = nch;
    const size_t cap = (size_t)v->capacity + kChunk;  // slots of the last chunk
    rzpic_status st;
#define A(p, n)                                   \
    if ((st = dalloc(c, &(p), (n))) != RZPIC_OK) \
        return st;
    const int64_t nsc = nch / kSuper + 2;
    A(ss.ch.dead, nch) A(ss.ch.ev, nch) A(ss.ch.se, nch) A(ss.ch.si, nch)
    A(ss.ch.clone_cnt, nch) A(ss.ch.clone_off, nch)
    A(ss.ch.sc_dead, nsc) A(ss.ch.sc_ev, nsc) A(ss.ch.sc_se, nsc) A(ss.ch.sc_si, nsc)
    A(ss.ch.dead_glob, cap) A(ss.ch.pcount, cap) A(ss.ch.cand, cap + (size_t)kChunk * (kMaxWaves + 1)) A(ss.ch.ncand, kMaxWaves)
#undef A
    if (s == 0 && v->mc_model == RZPIC_MC_ELECTRON) {
        size_t es = c->mixed ? sizeof(float) : sizeof(double);
        const int nf = c->c.push_form == RZPIC_PUSH_XYZ ? 9 : 8;
        for (int a = 0; a < 2; ++a)
            for (int f = 0; f < nf; ++f) HIPCHK(hipMalloc(&ss.stage[a][f], cap * es));
    }
    if (c->c.sort_every > 0) TRY(sort_alloc(c, s));
    RZ_LAUNCH(k_set_count, dim3(1), dim3(1), 0, c->st, c->cnt + s, (int64_t)0, (uint64_t)0);
    HIPCHK(hipGetLastError());
    return RZPIC_OK;
}

rzpic_status rzpic_set_count(rzpic_ctx *c, int32_t s, int64_t n, uint64_t next_id)
{
    TRY(need_species(c, s));
    TRY(unprepare(c));
    if (n < 0 || n > c->sp[s].cap)
        return fail(RZPIC_EINVAL, "count %lld outside [0, capacity %lld]", (long long)n,
                    (long long)c->sp[s].cap);
    RZ_LAUNCH(k_set_count, dim3(1), dim3(1), 0, c->st, c->cnt + s, n, next_id);
    HIPCHK(hipGetLastError());
    return RZPIC_OK;
}

rzpic_status rzpic_get_count(rzpic_ctx *c, int32_t s, int64_t *n, uint64_t *next_id)
{
    TRY(need_species(c, s));
    TRY(settle(c));
    Counts h;
    HIPCHK(hipMemcpyAsync(&h, c->cnt + s, sizeof h, hipMemcpyDeviceToHost, c->st));
    // synchronises, then returns (and clears) a pending device-side failure;
    // the counts are valid either way
    rzpic_status st = rzpic_sync(c);
    if (n) *n = h.n;
    if (next_id) *next_id = h.next_id;
    return st;
}

rzpic_status rzpic_set_xsec(rzpic_ctx *c, int32_t s, int32_t nproc, const int32_t *kind,
                            const double *thr_eV, double de, int32_t ne, const double *sigma,
                            double ej_B)
{
    TRY(need_species(c, s));
    TRY(unprepare(c));
    if (nproc < 1 || nproc > kMaxProc || ne < 2 || !(de > 0) || !kind || !thr_eV || !sigma)
        return fail(RZPIC_EINVAL, "cross sections: need 1 <= nproc <= %d, ne >= 2, de > 0", kMaxProc);
    for (int k = 0; k < nproc; ++k)
        if (kind[k] < RZPIC_P_ELASTIC || kind[k] > RZPIC_P_IONIZATION)
            return fail(RZPIC_EINVAL, "cross sections: unknown process kind %d", kind[k]);
    for (int k = 0; k < nproc; ++k)
        if (kind[k] == RZPIC_P_IONIZATION && (s != 0 || !c->sp[1].bound))
            return fail(RZPIC_EINVAL, "ionization needs electrons as species 0 and ions bound as species 1");
    SpeciesState &ss = c->sp[s];
    HIPCHK(c->st ? hipStreamSynchronize(c->st) : hipDeviceSynchronize());
    if (ss.sigma.p) {
        (void)hipFree(ss.sigma.p);
        ss.sigma.p = nullptr;
    }
    size_t bytes = (size_t)nproc * ne * sizeof(double);
    HIPCHK(hipMalloc(&ss.sigma.p, bytes));
    HIPCHK(hipMemcpy(ss.sigma.p, sigma, bytes, hipMemcpyHostToDevice));
    Xsec &x = ss.xs;
    x.sigma = (const double *)ss.sigma.p;
    x.nproc = nproc;
    x.ne = ne;
    x.de = de;
    x.emax = (double)(ne - 1) * de;
    x.inv_de = 1.0 / de;
    x.ejB = ej_B;
    // electron_real's estimate takes eps/de as eps * (1/de): within 3.3e-16 x
    // of the quotient, so each interpolated sigma_k moves by at most
    // 6.6e-12 of its largest table value (its slope per unit x is bounded by
    // that value, and x < ne); times n_gas and the pair speed at the table's
    // end, with a factor 3 to spare.
    {
        double ssum = 0.0;
        for (int k = 0; k < nproc; ++k) {
            double smax = 0.0;
            for (int j = 0; j < ne; ++j)
                smax = std::fmax(smax, std::fabs(sigma[(size_t)k * ne + j]));
            ssum += smax;
        }
        const double gmax = std::sqrt(2.0 * x.emax * kE / pair_mass(c, s));
        x.band_abs = 2e-11 * std::fabs(c->c.n_gas) * gmax * ssum;
    }
    for (int k = 0; k < nproc; ++k) {
        x.kind[k] = kind[k];
        x.thr[k] = thr_eV[k];
    }
    // nu_max: on [eps_j, eps_j+1] the interpolated sigma_T is at most its
    // larger end value and the pair speed at most g(eps_j+1); above the table
    // sigma_T g decreases, so these interval bounds bound every energy.
    const double mu = pair_mass(c, s);
    double numax = 0.0;
    for (int j = 0; j + 1 < ne; ++j) {
        double s0 = 0.0, s1 = 0.0;
        for (int k = 0; k < nproc; ++k) {
            s0 += sigma[(size_t)k * ne + j];
            s1 += sigma[(size_t)k * ne + j + 1];
        }
        double smax = s0 > s1 ? s0 : s1;
        double e1 = (double)(j + 1) * de;
        double g = std::sqrt(2.0 * e1 * kE / mu);
        double nu = c->c.n_gas * smax * g;
        if (nu > numax) numax = nu;
    }
    ss.nu_max = numax;
    ss.p_null = -std::expm1(-numax * dt_of(c, s));
    ss.has_xsec = true;
    return RZPIC_OK;
}

rzpic_status rzpic_get_mc_consts(rzpic_ctx *c, int32_t s, double *nu_max, double *p_null)
{
    TRY(need_species(c, s));
    if (nu_max) *nu_max = c->sp[s].nu_max;
    if (p_null) *p_null = c->sp[s].p_null;
    return RZPIC_OK;
}

rzpic_status rzpic_init_particles(rzpic_ctx *c, int32_t s, int64_t n, double n0, double T_eV,
                                  uint64_t id0)
{
    TRY(need_species(c, s));
    TRY(unprepare(c));
    if (n < 0 || n > c->sp[s].cap) return fail(RZPIC_EINVAL, "n = %lld exceeds capacity", (long long)n);
    if (!(T_eV >= 0) || !(n0 >= 0)) return fail(RZPIC_EINVAL, "need n0 >= 0 and T_eV >= 0");
    Phys ph = phys_of(c);
    if (c->mixed)
        HIPCHK(launch_init<float>(parts_of<float>(c->sp[s].v), n, n0, T_eV, id0, s, ph, c->sp[s].v.m, c->st));
    else
        HIPCHK(launch_init<double>(parts_of<double>(c->sp[s].v), n, n0, T_eV, id0, s, ph, c->sp[s].v.m, c->st));
    RZ_LAUNCH(k_set_count, dim3(1), dim3(1), 0, c->st, c->cnt + s, n, id0 + (uint64_t)n);
    HIPCHK(hipGetLastError());
    return RZPIC_OK;
}

rzpic_status rzpic_push_first(rzpic_ctx *c, int32_t s)
{
    TRY(need_species(c, s));
    TRY(unprepare(c));
    if (c->mixed) {
        TRY(run_pass<float>(c, s, M_FIRST | M_MARK, 0));
        if (c->children_pending[s]) TRY(run_staged<float>(c, s, M_FIRST));
    } else {
        TRY(run_pass<double>(c, s, M_FIRST | M_MARK, 0));
        if (c->children_pending[s]) TRY(run_staged<double>(c, s, M_FIRST));
    }
    return RZPIC_OK;
}

rzpic_status rzpic_push_final(rzpic_ctx *c, int32_t s)
{
    TRY(need_species(c, s));
    TRY(unprepare(c));
    if (c->mixed) TRY(run_pass<float>(c, s, M_FINAL | M_MARK, 0));
    else TRY(run_pass<double>(c, s, M_FINAL | M_MARK, 0));
    return RZPIC_OK;
}

rzpic_status rzpic_collide(rzpic_ctx *c, int32_t s, int64_t step)
{
    TRY(need_species(c, s));
    TRY(unprepare(c));
    if (!c->sp[s].has_xsec) return RZPIC_OK;
    if (s == 0 && (c->children_pending[0] || c->children_pending[1]))
        return fail(RZPIC_ESTATE, "new particles already staged: call rzpic_compact first");
    if (c->mixed) TRY(run_pass<float>(c, s, M_MC | M_MARK, (uint32_t)step));
    else TRY(run_pass<double>(c, s, M_MC | M_MARK, (uint32_t)step));
    if (s == 0 && c->sp[0].v.mc_model == RZPIC_MC_ELECTRON) {
        c->children_pending[0] = c->children_pending[1] = true;
        c->children_scanned = false;
    }
    return RZPIC_OK;
}

rzpic_status rzpic_deposit(rzpic_ctx *c)
{
    TRY(need_both(c));
    TRY(unprepare(c));
    if (c->mixed) TRY(deposit_impl<float>(c));
    else TRY(deposit_impl<double>(c));
    TRY(finalize_impl(c, 0));
    return RZPIC_OK;
}

rzpic_status rzpic_solve(rzpic_ctx *c, double t, int32_t *cycles, double *relres)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(unprepare(c));
    return solve_impl(c, t, false, cycles, relres);
}

rzpic_status rzpic_solve_dev(rzpic_ctx *c, double t, int32_t *cycles_dev, double *relres_dev)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(unprepare(c));
    const bool fixed = c->c.mg_fixed_cycles > 0;
    int32_t k = 0;
    double rr = 0.0;
    // fixed cycles: nothing asked on the host, so nothing synchronises
    TRY(solve_impl(c, t, false, fixed ? nullptr : &k, fixed ? nullptr : &rr));
    if (!cycles_dev && !relres_dev) return RZPIC_OK;
    const unsigned long long *norm = nullptr;
    if (fixed) {
        k = c->c.mg_fixed_cycles;
        if (relres_dev) {
            if (c->c.circuit_C > 0.0)
                return fail(RZPIC_EINVAL, "solve_dev: the residual of a circuit solve is per "
                                          "solution; ask rzpic_solve");
            HIPCHK(launch_fill_u64(c->norm, 2, c->st));
            HIPCHK(mg_resid_norm(c->mg, c->phi, c->f, 1, c->norm + 1, c->st));
            HIPCHK(mg_resid_norm(c->mg, c->phi, c->f, 0, c->norm, c->st));
            norm = c->norm;
        }
    }
    RZ_LAUNCH(k_solve_out, dim3(1), dim3(64), 0, c->st, cycles_dev, relres_dev, (int)k, rr, norm);
    HIPCHK(hipGetLastError());
    return RZPIC_OK;
}

rzpic_status rzpic_grid_view(rzpic_ctx *c, rzpic_grid *out)
{
    if (!c || !out) return fail(RZPIC_EINVAL, "null argument");
    out->nr = c->c.nr;
    out->nz = c->c.nz;
    out->phi = c->phi;
    out->rho = c->rho;
    out->chi = c->chi;
    out->er = c->er;
    out->ez = c->ez;
    out->dens[0] = c->dens[0];
    out->dens[1] = c->dens[1];
    out->vol = c->vol;
    out->phi_p = c->phiP;
    out->phi_l = c->phiL;
    return RZPIC_OK;
}

rzpic_status rzpic_set_grid_source(rzpic_ctx *c, const double *rho, const double *chi)
{
    if (!c || !rho || !chi) return fail(RZPIC_EINVAL, "null argument");
    TRY(unprepare(c));
    const size_t bytes = (size_t)c->nn * sizeof(double);
    HIPCHK(hipMemcpyAsync(c->rho, rho, bytes, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->chi, chi, bytes, hipMemcpyDeviceToDevice, c->st));
    return RZPIC_OK;
}

rzpic_status rzpic_set_mg(rzpic_ctx *c, double tol, int32_t max_cycles, int32_t fixed_cycles)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(unprepare(c));
    if (fixed_cycles < 0 || (fixed_cycles == 0 && (max_cycles < 1 || !(tol > 0))))
        return fail(RZPIC_EINVAL, "need fixed_cycles > 0, or max_cycles >= 1 and tol > 0");
    c->c.mg_tol = tol;
    c->c.mg_max_cycles = max_cycles;
    c->c.mg_fixed_cycles = fixed_cycles;
    return RZPIC_OK;
}

rzpic_status rzpic_set_voltage(rzpic_ctx *c, double V_dc, double V_rf, double f_rf)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(unprepare(c));
    if (!std::isfinite(V_dc) || !std::isfinite(V_rf) || !std::isfinite(f_rf))
        return fail(RZPIC_EINVAL, "voltage parameters must be finite");
    c->c.V_dc = V_dc;
    c->c.V_rf = V_rf;
    c->c.f_rf = f_rf;
    return RZPIC_OK;
}

rzpic_status rzpic_set_circuit(rzpic_ctx *c, double V, double Q, double Qc)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(unprepare(c));
    if (!c->circ) return fail(RZPIC_EINVAL, "the context has no external circuit (circuit_C = 0)");
    if (!std::isfinite(V) || !std::isfinite(Q) || !std::isfinite(Qc))
        return fail(RZPIC_EINVAL, "circuit state must be finite");
    HIPCHK(launch_circuit_set(c->circ, V, Q, Qc, c->st));
    return RZPIC_OK;
}

rzpic_status rzpic_get_circuit(rzpic_ctx *c, double out[6])
{
    if (!c || !out) return fail(RZPIC_EINVAL, "null argument");
    if (!c->circ) return fail(RZPIC_EINVAL, "the context has no external circuit (circuit_C = 0)");
    CircuitState h{};
    HIPCHK(hipMemcpyAsync(&h, c->circ, sizeof h, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    out[0] = h.V;
    out[1] = h.Q;
    out[2] = h.Qc;
    out[3] = h.Qconv;
    out[4] = h.Qp;
    out[5] = h.Ql;
    return RZPIC_OK;
}

rzpic_status rzpic_efield(rzpic_ctx *c)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    return efield_impl(c);
}

rzpic_status rzpic_compact(rzpic_ctx *c, int32_t s)
{
    TRY(need_species(c, s));
    TRY(unprepare(c));
    if (s == 1 && c->children_pending[1] && !c->sp[0].bound)
        return fail(RZPIC_ESTATE, "species 0 must stay bound while new ions are staged");
    if (c->mixed) {
        HIPCHK(launch_dead_scan<float>(parts_of<float>(c->sp[s].v), c->cnt + s, c->sp[s].ch, c->st));
        TRY(run_fixup<float>(c, 1 << s));
    } else {
        HIPCHK(launch_dead_scan<double>(parts_of<double>(c->sp[s].v), c->cnt + s, c->sp[s].ch, c->st));
        TRY(run_fixup<double>(c, 1 << s));
    }
    return RZPIC_OK;
}

rzpic_status rzpic_resize(rzpic_ctx *c, int32_t s)
{
    TRY(need_species(c, s));
    TRY(unprepare(c));
    if (!(c->c.resize_wcoef > 0)) return fail(RZPIC_EINVAL, "resize_wcoef must be positive");
    if (c->children_pending[s]) return fail(RZPIC_ESTATE, "call rzpic_compact before rzpic_resize");
    if (c->mixed) {
        TRY(resize_impl<float>(c, s, 0));
        TRY(zero_order_compact<float>(c, 1 << s));
    } else {
        TRY(resize_impl<double>(c, s, 0));
        TRY(zero_order_compact<double>(c, 1 << s));
    }
    return RZPIC_OK;
}

rzpic_status rzpic_sort(rzpic_ctx *c, int32_t s)
{
    TRY(need_species(c, s));
    TRY(unprepare(c));
    if (c->children_pending[s]) return fail(RZPIC_ESTATE, "call rzpic_compact before rzpic_sort");
    if (c->mixed) TRY(sort_impl<float>(c, s));
    else TRY(sort_impl<double>(c, s));
    return RZPIC_OK;
}

rzpic_status rzpic_prologue(rzpic_ctx *c)
{
    TRY(need_both(c));
    TRY(unprepare(c));
    if (c->children_pending[0] || c->children_pending[1])
        return fail(RZPIC_ESTATE, "new particles are staged: call rzpic_compact first");
    for (int s = 0; s < 2; ++s) HIPCHK(launch_fill_u64(c->acc[s], c->nn, c->st));
    const int mode = M_FIRST | M_DEP | M_LISTS;
    if (c->mixed) {
        for (int s = 0; s < 2; ++s) TRY(run_pass<float>(c, s, mode, 0));
        TRY(run_fixup<float>(c, 3));
    } else {
        for (int s = 0; s < 2; ++s) TRY(run_pass<double>(c, s, mode, 0));
        TRY(run_fixup<double>(c, 3));
    }
    return RZPIC_OK;
}

// Launch configuration of the fused pass: threads per block, particles of
// capacity per block, and the deposit form (the whole grid privatised in
// each block's LDS, or the LDS windows of the tiles planned at the last
// sort).  The results do not depend on it (integer deposit, identities from
// event ranks, compaction by index), only the speed.
static rzpic_status set_pass_config(rzpic_ctx *c, int threads, int64_t ppb, bool lds)
{
    c->pass_threads = threads;
    c->parts_per_block = ppb;
    c->lds_form = lds && c->lds_ok;
    if (c->lds_form)
        c->lds_resident = lds_resident_of(c, threads);
    else
        c->tile_per_cu = c->mixed ? pass2_tiled_blocks_per_cu<float>(threads)
                                  : pass2_tiled_blocks_per_cu<double>(threads);
    // the tile plan is made for the tiled pass's block count: plan again
    for (int s = 0; s < 2; ++s)
        if (c->sp[s].tile_pb) {
            if (c->mixed) TRY(sort_impl<float>(c, s));
            else TRY(sort_impl<double>(c, s));
        }
    return RZPIC_OK;
}

static rzpic_status set_shape(rzpic_ctx *c, int threads, int64_t ppb)
{
    return set_pass_config(c, threads, ppb, c->lds_form);
}

// Whether a configuration fits the pass's bucket layout (at most kMaxWaves
// wavefronts) and, for the whole-grid form, the LDS.
static bool config_fits(const rzpic_ctx *c, int threads, int64_t ppb, bool lds)
{
    if (lds && !c->lds_ok) return false;
    rzpic_ctx t = *c;  // copy of the scalars pass_blocks / tiled_blocks read
    t.pass_threads = threads;
    t.parts_per_block = ppb;
    if (!lds)
        t.tile_per_cu = c->mixed ? pass2_tiled_blocks_per_cu<float>(threads)
                                 : pass2_tiled_blocks_per_cu<double>(threads);
    int b0, b1;
    if (lds) {
        const int most = lds_resident_of(c, threads);
        b0 = pass_blocks(&t, 0, most / 2);
        b1 = pass_blocks(&t, 1, most - most / 2);
    } else {
        b0 = tiled_blocks(&t, 0);
        b1 = tiled_blocks(&t, 1);
    }
    return (int64_t)(b0 + b1) * (threads / 64) <= kMaxWaves;
}

static bool shape_fits(const rzpic_ctx *c, int threads, int64_t ppb)
{
    return config_fits(c, threads, ppb, c->lds_form);
}

// Tile shape of the sort (cells in z and r).  The sort's scratch is sized by
// the tile count: it is freed here (after the stream has drained) and
// allocated again by the next sort; a species that has a plan is sorted
// again at once, by the new tiles.
static rzpic_status set_tiles(rzpic_ctx *c, int tz, int tr)
{
    if (tz < 1 || tr < 1) return fail(RZPIC_EINVAL, "tile_z and tile_r must be >= 1");
    const int ntr = (c->c.nr - 2) / tr + 1;
    const int nt = ((c->c.nz - 2) / tz + 1) * ntr;
    if (nt > kMaxTiles)
        return fail(RZPIC_EINVAL, "%d tiles exceed %d: enlarge tile_z / tile_r", nt, kMaxTiles);
    if (tz == c->c.tile_z && tr == c->c.tile_r) return RZPIC_OK;
    const bool planned[2] = {c->sp[0].tile_pb != nullptr, c->sp[1].tile_pb != nullptr};
    if (c->sp[0].sort_off || c->sp[1].sort_off) HIPCHK(hipStreamSynchronize(c->st));
    for (int s = 0; s < 2; ++s) free_sort(c->sp[s]);
    c->c.tile_z = tz;
    c->c.tile_r = tr;
    c->ntr = ntr;
    c->nt = nt;
    c->kbits = 0;
    while ((1 << c->kbits) < c->nt) ++c->kbits;
    for (int s = 0; s < 2; ++s)
        if (planned[s]) {
            if (c->mixed) TRY(sort_impl<float>(c, s));
            else TRY(sort_impl<double>(c, s));
        }
    return RZPIC_OK;
}

// ===========================================================================
// Helpers of the batch autotuner (batch.hip).

// What the tuner groups contexts by: {nr, nz, FP32 particles, the whole
// grid fits LDS, tile-sorted steps}.
void rz_tune_key(const rzpic_ctx *c, int32_t out[5])
{
    out[0] = c->c.nr;
    out[1] = c->c.nz;
    out[2] = c->mixed;
    out[3] = c->lds_ok ? 1 : 0;
    out[4] = c->c.sort_every > 0 ? 1 : 0;
}

int rz_config_fits(const rzpic_ctx *c, int threads, int64_t ppb, int lds)
{
    return config_fits(c, threads, ppb, lds != 0) ? 1 : 0;
}

rzpic_status rz_set_config(rzpic_ctx *c, int threads, int64_t ppb, int lds, int tz, int tr)
{
    HIPCHK(list_tail_flush(c->tail, c->st));  // the tiles may re-sort the particles
    TRY(set_tiles(c, tz, tr));
    return set_pass_config(c, threads, ppb, lds != 0);
}

void rz_get_config(const rzpic_ctx *c, int32_t out[5])
{
    out[0] = c->pass_threads;
    out[1] = (int32_t)c->parts_per_block;
    out[2] = c->lds_form ? RZPIC_FORM_LDS : RZPIC_FORM_TILED;
    out[3] = c->c.tile_z;
    out[4] = c->c.tile_r;
}

// One step captured from the stream and replayed as a graph.  The step's
// launches are recorded by stream capture (their arguments evaluated now, as
// in a direct step), and the executable graph of the step's variant is
// updated with them in place (hipGraphExecUpdate: same kernels, new
// arguments), or instantiated when the variant is new or the update is
// refused.  Replaying a graph saves the GPU about a microsecond of dispatch
// per kernel against launching the same kernels one by one.
static rzpic_status step_graph(rzpic_ctx *c, int64_t n)
{
    const bool ions = n % ion_K(c) == ion_K(c) - 1;
    const bool resize = c->c.resize_every > 0 && n % c->c.resize_every == c->c.resize_every - 1;
    const bool sort = c->c.sort_every > 0 && n % c->c.sort_every == c->c.sort_every - 1;
    hipGraphExec_t &ex = c->gexec[(ions ? 1 : 0) | (resize ? 2 : 0) | (sort ? 4 : 0)];
    HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    const rzpic_status s = c->mixed ? step_impl<float>(c, n) : step_impl<double>(c, n);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(c->st, &g);
    if (s != RZPIC_OK || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (s != RZPIC_OK) return s;
        return fail(RZPIC_EHIP, "step capture: %s", hipGetErrorString(ce));
    }
    if (ex) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult r = hipGraphExecUpdateSuccess;
        if (hipGraphExecUpdate(ex, g, &bad, &r) != hipSuccess || r != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(ex);
            ex = nullptr;
        }
    }
    hipError_t e = hipSuccess;
    if (!ex) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        ex = nullptr;
        return fail(RZPIC_EHIP, "step graph instantiation: %s", hipGetErrorString(e));
    }
    HIPCHK(hipGraphLaunch(ex, c->st));
    return RZPIC_OK;
}

rzpic_status rzpic_step(rzpic_ctx *c, int64_t step)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    if (step < 0 || step > 0xFFFFFFFELL) return fail(RZPIC_EINVAL, "step out of range");
    // graph replay unless a batch records this step, timing events are on or
    // the solve runs to a tolerance (it synchronises)
    if (c->step_graph && !g_recorder && !c->timing && c->c.mg_fixed_cycles > 0) {
        TRY(settle(c));  // outside the capture
        return step_graph(c, step);
    }
    const bool pipe = c->pipeline && !g_recorder;
    return c->mixed ? step_impl<float>(c, step, pipe) : step_impl<double>(c, step, pipe);
}

rzpic_status rzpic_set_step_pipeline(rzpic_ctx *c, int32_t on)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    c->pipeline = on != 0;
    c->prepared = -1;
    return RZPIC_OK;
}

rzpic_status rzpic_set_step_graph(rzpic_ctx *c, int32_t on)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(unprepare(c));
    if (on) {
        if (!c->st)
            return fail(RZPIC_EINVAL, "graph replay needs a stream other than the null stream");
        if (c->c.mg_fixed_cycles <= 0)
            return fail(RZPIC_EINVAL, "graph replay needs a fixed number of V-cycles "
                                      "(mg_fixed_cycles > 0): a tolerance-mode solve synchronises");
    }
    c->step_graph = on != 0;
    return RZPIC_OK;
}

rzpic_status rzpic_autotune(rzpic_ctx *c, int32_t steps, int64_t step0, double *table,
                            int32_t best[2], int64_t *next_step)
{
    if (!c || !best || !next_step) return fail(RZPIC_EINVAL, "null argument");
    TRY(settle(c));
    if (steps < 1) return fail(RZPIC_EINVAL, "steps must be >= 1");
    TRY(need_both(c));
    if (c->timing) return fail(RZPIC_EINVAL, "autotune needs step timing off");
    static const int kThreads[4] = {256, 512, 768, 1024};
    static const int64_t kPpb[4] = {2048, 4096, 8192, 16384};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int64_t n = step0;
    double best_ms = -1.0;
    double times[16];
    int bt = c->pass_threads;
    int64_t bp = c->parts_per_block;
    rzpic_status st = RZPIC_OK;
    for (int ti = 0; ti < 4 && st == RZPIC_OK; ++ti)
        for (int pi = 0; pi < 4 && st == RZPIC_OK; ++pi) {
            double ms = -1.0;
            if (shape_fits(c, kThreads[ti], kPpb[pi])) {
                st = set_shape(c, kThreads[ti], kPpb[pi]);
                if (st == RZPIC_OK) st = rzpic_step(c, n++);  // warm-up
                if (st == RZPIC_OK && hipEventRecord(e0, c->st) != hipSuccess)
                    st = fail(RZPIC_EHIP, "hipEventRecord failed");
                for (int k = 0; k < steps && st == RZPIC_OK; ++k) st = rzpic_step(c, n++);
                float f = 0.0f;
                if (st == RZPIC_OK && (hipEventRecord(e1, c->st) != hipSuccess ||
                                       hipEventSynchronize(e1) != hipSuccess ||
                                       hipEventElapsedTime(&f, e0, e1) != hipSuccess))
                    st = fail(RZPIC_EHIP, "event timing failed");
                if (st == RZPIC_OK) {
                    ms = f / steps;
                    if (best_ms < 0.0 || ms < best_ms) best_ms = ms;
                }
            }
            times[4 * ti + pi] = ms;
            if (table) {
                table[3 * (4 * ti + pi) + 0] = kThreads[ti];
                table[3 * (4 * ti + pi) + 1] = (double)kPpb[pi];
                table[3 * (4 * ti + pi) + 2] = ms;
            }
        }
    // the first shape (table order) within 2 % of the fastest: near-ties do
    // not flip the choice from run to run
    for (int k = 0; k < 16 && best_ms > 0.0; ++k)
        if (times[k] > 0.0 && times[k] <= 1.02 * best_ms) {
            bt = kThreads[k / 4];
            bp = kPpb[k % 4];
            break;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RZPIC_OK) return st;
    TRY(set_shape(c, bt, bp));
    best[0] = bt;
    best[1] = (int32_t)bp;
    *next_step = n;
    return rzpic_sync(c);
}

rzpic_status rzpic_set_pass_shape(rzpic_ctx *c, int32_t threads, int32_t parts_per_block)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(settle(c));  // a new shape may re-sort the particles
    if ((threads != 256 && threads != 512 && threads != 768 && threads != 1024) ||
        parts_per_block < 64)
        return fail(RZPIC_EINVAL,
                    "threads must be 256, 512, 768 or 1024 and parts_per_block >= 64");
    if (c->sp[0].bound && c->sp[1].bound && !shape_fits(c, threads, parts_per_block))
        return fail(RZPIC_EINVAL, "the shape exceeds the pass's wavefront limit");
    return set_shape(c, threads, parts_per_block);
}

rzpic_status rzpic_set_pass_form(rzpic_ctx *c, int32_t form)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(settle(c));  // a new form may re-sort the particles
    if (form != RZPIC_FORM_AUTO && form != RZPIC_FORM_LDS && form != RZPIC_FORM_TILED)
        return fail(RZPIC_EINVAL, "form must be RZPIC_FORM_AUTO, RZPIC_FORM_LDS or RZPIC_FORM_TILED");
    if (form == RZPIC_FORM_LDS && !c->lds_ok)
        return fail(RZPIC_EINVAL, "the deposit grid does not fit one workgroup's LDS");
    const bool lds = form != RZPIC_FORM_TILED && c->lds_ok;
    if (c->sp[0].bound && c->sp[1].bound &&
        !config_fits(c, c->pass_threads, c->parts_per_block, lds))
        return fail(RZPIC_EINVAL, "the pass shape exceeds the wavefront limit in that form");
    return set_pass_config(c, c->pass_threads, c->parts_per_block, lds);
}

rzpic_status rzpic_set_tiles(rzpic_ctx *c, int32_t tile_z, int32_t tile_r)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(settle(c));  // new tiles re-sort the particles
    return set_tiles(c, tile_z, tile_r);
}

rzpic_status rzpic_get_pass_config(rzpic_ctx *c, int32_t out[5])
{
    if (!c || !out) return fail(RZPIC_EINVAL, "null argument");
    rz_get_config(c, out);
    return RZPIC_OK;
}

rzpic_status rzpic_grid_copy(rzpic_ctx *c, int32_t which, double *dev, int32_t to_ctx)
{
    if (!c || !dev) return fail(RZPIC_EINVAL, "null argument");
    if (to_ctx) TRY(unprepare(c));
    else TRY(settle(c));
    double *src = nullptr;
    switch (which) {
    case RZPIC_G_PHI: src = c->phi; break;
    case RZPIC_G_RHO: src = c->rho; break;
    case RZPIC_G_CHI: src = c->chi; break;
    case RZPIC_G_ER: src = c->er; break;
    case RZPIC_G_EZ: src = c->ez; break;
    case RZPIC_G_DENS0: src = c->dens[0]; break;
    case RZPIC_G_DENS1: src = c->dens[1]; break;
    case RZPIC_G_VOL: src = c->vol; break;
    case RZPIC_G_PHI_P:
    case RZPIC_G_PHI_L:
        if (!c->circ) return fail(RZPIC_EINVAL, "grid %d needs the external circuit", which);
        if (to_ctx) return fail(RZPIC_EINVAL, "grid %d is read-only", which);
        src = which == RZPIC_G_PHI_P ? c->phiP : c->phiL;
        break;
    case RZPIC_G_N0:
    case RZPIC_G_N1: {
        int s = which - RZPIC_G_N0;
        HIPCHK(launch_acc_convert(c->nn, c->acc[s], dev, c->quantum[s], to_ctx ? 1 : 0, c->st));
        return RZPIC_OK;
    }
    default: return fail(RZPIC_EINVAL, "unknown grid %d", which);
    }
    size_t bytes = (size_t)c->nn * sizeof(double);
    if (to_ctx) {
        if (which == RZPIC_G_VOL || which == RZPIC_G_DENS0 || which == RZPIC_G_DENS1)
            return fail(RZPIC_EINVAL, "grid %d is read-only", which);
        HIPCHK(hipMemcpyAsync(src, dev, bytes, hipMemcpyDeviceToDevice, c->st));
        if (which == RZPIC_G_ER || which == RZPIC_G_EZ) {
            // the gather reads the interleaved copy: repack it
            if (c->mixed)
                HIPCHK(launch_pack_e2<float>(c->nn, c->er, c->ez, (float2 *)c->E2, c->st));
            else
                HIPCHK(launch_pack_e2<double>(c->nn, c->er, c->ez, (double2 *)c->E2, c->st));
        }
    } else {
        HIPCHK(hipMemcpyAsync(dev, src, bytes, hipMemcpyDeviceToDevice, c->st));
    }
    return RZPIC_OK;
}

rzpic_status rzpic_sync(rzpic_ctx *c)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    TRY(settle(c));
    int32_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, c->status, sizeof h, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (h) {
        int32_t zero = 0;
        HIPCHK(hipMemcpy(c->status, &zero, sizeof zero, hipMemcpyHostToDevice));
        if (h & kStCapacity) return fail(RZPIC_ECAPACITY, "particle capacity exceeded");
        return fail(RZPIC_ENUMERIC, "fixed-point deposit overflow or non-finite value");
    }
    return RZPIC_OK;
}

rzpic_status rzpic_get_diag(rzpic_ctx *c, rzpic_diag *out)
{
    if (!c || !out) return fail(RZPIC_EINVAL, "null argument");
    TRY(settle(c));
    std::memset(out, 0, sizeof *out);
    Counts cn[2];
    unsigned long long tal[6], ms[2 * (1 + kMaxProc)];
    int32_t stw = 0;
    HIPCHK(hipMemcpyAsync(cn, c->cnt, sizeof cn, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(tal, c->tally, sizeof tal, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(ms, c->mcstat, sizeof ms, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(&stw, c->status, sizeof stw, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    for (int s = 0; s < 2; ++s) {
        out->count[s] = cn[s].n;
        out->next_id[s] = cn[s].next_id;
        for (int b = 0; b < 3; ++b)
            out->absorbed[s][b] = (double)(long long)tal[3 * s + b] * c->quantum[s];
        out->candidates[s] = (int64_t)ms[(1 + kMaxProc) * s];
        for (int k = 0; k < kMaxProc; ++k) out->events[s][k] = (int64_t)ms[(1 + kMaxProc) * s + 1 + k];
    }
    unsigned long long ps[2];
    HIPCHK(hipMemcpy(ps, c->psteps, sizeof ps, hipMemcpyDeviceToHost));
    out->particle_steps[0] = ps[0];
    out->particle_steps[1] = ps[1];
    out->last_cycles = c->last_cycles;
    out->last_relres = c->last_relres;
    out->status = stw & kStCapacity ? RZPIC_ECAPACITY : (stw ? RZPIC_ENUMERIC : RZPIC_OK);
    return (rzpic_status)out->status;
}

rzpic_status rzpic_set_timing(rzpic_ctx *c, int32_t enable)
{
    if (!c) return fail(RZPIC_EINVAL, "null context");
    if (enable && c->evpool.empty()) {
        c->evpool.resize((size_t)rzpic_ctx::kPool * rzpic_ctx::kEvPerStep);
        for (auto &e : c->evpool) HIPCHK(hipEventCreate(&e));
    }
    if (!enable) TRY(flush_timing(c));
    c->timing = enable != 0;
    return RZPIC_OK;
}

rzpic_status rzpic_get_timing(rzpic_ctx *c, double out[12])
{
    if (!c || !out) return fail(RZPIC_EINVAL, "null argument");
    TRY(flush_timing(c));
    unsigned long long ps[2];
    HIPCHK(hipMemcpyAsync(ps, c->psteps, sizeof ps, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    const double k = c->acc_steps > 0 ? (double)c->acc_steps : 1.0;
    out[0] = c->acc_steps;
    out[1] = c->acc_ms[0] / k;
    out[2] = c->acc_ms[1] / k;
    out[3] = c->acc_cycles / k;
    out[4] = c->acc_ms[2] / k;
    out[5] = c->acc_ms[3] / k;
    out[6] = c->acc_ms[4] / k;
    out[7] = c->acc_ms[5] / k;
    out[8] = ((double)ps[0] - c->acc_n[0]) / k;
    out[9] = ((double)ps[1] - c->acc_n[1]) / k;
    out[10] = c->acc_ms[6] / k;
    out[11] = c->acc_ms[7] / k;
    c->acc_n[0] = (double)ps[0];
    c->acc_n[1] = (double)ps[1];
    for (double &v : c->acc_ms) v = 0.0;
    c->acc_cycles = 0;
    c->acc_steps = 0;
    return RZPIC_OK;
}

}  // extern "C"
