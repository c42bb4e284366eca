// Internal definitions shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.h"

namespace rz {

// Physical constants (CODATA 2018, SI).
constexpr double kE = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kKb = 1.380649e-23;
constexpr double kTwoPi = 6.283185307179586;

constexpr int kMaxProc = 4;
constexpr int kMaxLevels = 16;
constexpr int kChunk = 64;       // particles per chunk: one wavefront
constexpr int kMaxWaves = 16384; // wavefronts of a particle pass (bounds the bucket padding)
constexpr int kLongThreads = 1024;            // threads of a long-line solve
constexpr int kMaxLine = 8 * kLongThreads;    // longest r-line (nr - 1 unknowns) the smoother takes
constexpr int kMaxTiles = 2048;  // tiles of the particle sort
constexpr int kWinNodes = 4096;  // LDS deposit window of a tiled pass block (nodes)
constexpr int kWinHalo = 8;      // cells of drift margin around a block's tiles

// Device status bits (sticky).
enum : int32_t {
    kStCapacity = 1,
    kStNumeric = 2,
};

// Pass mode bits of the particle kernel.
enum : int {
    M_FINAL = 1,   // gather + final push + axis rule + absorption
    M_MC = 2,      // null-collision Monte Carlo, children staged
    M_FIRST = 4,   // first push + rotation + absorption
    M_DEP = 8,     // deposit at the (new) position
    M_MARK = 16,   // unmerged form: dead particles carry w = -1, skipped on input
    M_LISTS = 32,  // merged form: per-chunk dead lists built in the pass
    M_LDS = 64,    // deposit into an LDS copy of the whole grid, flushed to a slice
    M_TILE = 128,  // blocks take contiguous particle ranges and deposit into an
                   // LDS window of the tiles their (sorted) particles occupy
};
// The fused pass only tests for Monte Carlo candidates (M_MC): a candidate
// keeps its final-pushed state and goes to the candidate list, where the
// collision kernel applies the outcome and, in the merged form, its first
// push and deposit.

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename T> struct Parts {
    T *r, *z, *vr, *vt, *vz, *ar, *az, *w;
    uint64_t *id;
    T *at;  // a_theta of the global X-Y-Z push; null in the local form
};

struct Mesh {
    int nr, nz, nn, weighting;
    double R, L, hr, hz, inv_hr, inv_hz;
};

struct Xsec {
    const double *sigma;   // [nproc][ne]
    int nproc, ne;
    double de, emax;
    double inv_de;         // 1 / de (the estimate of electron_real)
    double band_abs;       // absolute part of electron_real's undecided band
    int kind[kMaxProc];
    double thr[kMaxProc];
    double ejB;
};

struct SpeciesK {
    int s, mc_model;
    double q, m, qm;
    double k1, k2;          // c q/m dt^2, c q/m dt: c = 1/2 (D1), theta/2 (Friedman)
    double dt;              // time step of the species (K dt for subcycled ions)
    double inv_quantum;     // 2^bits / w_ref
    double p_null, nu_max;
    uint64_t cand_u52;      // candidate iff the 52-bit u of U0 is below this
    double ekin;            // 0.5 * (pair mass) / e : eV per (m/s)^2
    double mu;              // pair mass
    Xsec xs;
};

struct Phys {
    double dt, n_gas, T_gas, m_gas, vth_gas;
    double R, L;
    uint64_t seed;
    double ion_acc_ratio;   // q_i m_e / (q_e m_i) for new ions
    double ion_inv_quantum; // fixed-point scale of the ion deposit
    double ion_dt;          // time step of the ions (first push of new ions)
    int friedman;           // Friedman's adjustable damping instead of D1
    double fc;              // Friedman: theta / 2, the implicit coefficient
};

struct Counts {      // per species, device resident
    int64_t n;       // live particles in the array
    uint64_t next_id;
};

struct FixRec {       // per species, written by the dead-list scan
    int64_t n_old, dead, keep, pad;
};

struct ChildRec {     // new particles staged by the electron pass
    int64_t n_parent;                // electron count when they were staged
    int64_t ev_total;                // ionization events
    int64_t surv_total[2];           // survivors per child species
    uint64_t next_id_old[2];         // identities before this batch
};

struct CloneRec {     // weight split of one species
    int64_t n_old, total, ok, pad;
    uint64_t next_id_old;
};

constexpr int kSuper = 512;      // chunks per superchunk (two-level offsets)

struct Chunks {       // per parent species; chunk = 64 consecutive particles (lane = bit)
    unsigned long long *dead;   // absorbed particles
    unsigned long long *ev;     // ionization events (electron chunks)
    unsigned long long *se, *si;// new electron / new ion still alive
    int32_t *sc_dead, *sc_ev, *sc_se, *sc_si;  // set bits per superchunk
    int64_t *clone_off;
    int32_t *clone_cnt;         // per chunk (resize)
    int64_t *dead_glob;         // sorted global dead list
    int32_t *pcount;            // per particle clone count (resize)
    int32_t *cand;              // Monte Carlo candidates: per-wavefront buckets
    int32_t *ncand;             // candidates per bucket
};

template <typename T> struct PassArgs {
    Parts<T> p;              // particles of species s
    Parts<T> ce, ci;         // staging of new electrons / ions (electron pass)
    const Counts *cnt;
    Chunks ch;
    Mesh mesh;
    Phys phys;
    SpeciesK sp;
    const typename Vec2<T>::type *E2;
    unsigned long long *acc;      // deposit of species s (global)
    unsigned long long *acc_ion;  // deposit of new ions (global)
    void *slices;                 // per-block LDS flush [gridDim][nn]: 32-bit elements
                                  //    for FP32 particles, 64-bit for FP64
    unsigned long long *tally;    // [3] absorbed weight of species s, fixed point
    unsigned long long *tally_ion;
    unsigned long long *mcstat;   // [1 + kMaxProc] candidates, events per process
    uint8_t *ev;                  // optional per-particle event codes
    ChildRec *crec;               // electron pass records n_parent here
    unsigned long long *psteps;   // if set: += particles entering the pass
    int nbuckets;                 // blocks of the pass (= candidate buckets)
    int bucket_waves;             // wavefronts per pass block
    int32_t *status;
    uint32_t step;
    // M_TILE: block ranges and deposit windows planned at the last sort
    // (per_block = 0 or a plan made for another block count: no windows)
    int tiled;                    // the pass ran with M_TILE (bucket layout)
    int tile_nb;                  // pass blocks the plan was made for
    const int64_t *tile_pb;       // particles per block, multiple of kChunk
    const int4 *tile_win;         // [tile_nb] window {i0, j0, ni, nj} in nodes
};

// Candidate bucket of each pass block: chunks it may process.  Grid-stride
// form: ceil(nch / waves) per wavefront; tiled form: its planned range plus
// its share of the chunks beyond the planned ones.
__host__ __device__ inline int64_t tiled_q(int64_t pb) { return pb / kChunk; }
__host__ __device__ inline int64_t tiled_q2(int64_t nch, int nb, int64_t q)
{
    const int64_t rem = nch - (int64_t)nb * q;
    return rem > 0 ? (rem + nb - 1) / nb : 0;
}

// Elements between consecutive slices: whole groups of four for 32-bit
// elements (16-byte loads in the slice sum), nn for 64-bit ones.
__host__ __device__ inline size_t slice_stride(int nn, int narrow)
{
    return narrow ? ((size_t)nn + 3) & ~(size_t)3 : (size_t)nn;
}

// Sum of per-block LDS deposit slices into the deposit grids of both
// species (launch_slice_sum).  64-bit slices: block b of the 2 * bx * by
// blocks takes species b / (bx by), nodes of column block b % bx (256 per
// block) and every by-th slice.  32-bit slices (narrow): block b of the
// 2 * bx blocks takes species b / bx and 4 kSliceSumGroups nodes, all slices.
constexpr int kSliceSumGroups = 8;

struct SliceSum {
    unsigned long long *acc[2];
    const void *slices[2];
    int nb[2];
    int nn, bx, by;
    int narrow;  // 32-bit slice elements (FP32 particles)
};

// Host-side launchers (defined in the .hip files).
template <typename T>
hipError_t launch_pass(int mode, const PassArgs<T> &a, int blocks, int threads, size_t lds,
                       hipStream_t st);
// ev0, ev1 (optional): events attached to the kernel's own start and end.
template <typename T>
hipError_t launch_pass2(int mode, const PassArgs<T> &a0, const PassArgs<T> &a1, int b0, int b1,
                        int threads, size_t lds, hipStream_t st, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
// Resident blocks per CU of the tiled merged pass (register and LDS limits).
template <typename T> int pass2_tiled_blocks_per_cu(int threads);
// Resident blocks per CU of the merged pass with a whole-grid LDS copy of
// `lds` bytes (register and LDS limits).
template <typename T> int pass2_lds_blocks_per_cu(int threads, size_t lds);
template <typename T>
hipError_t launch_collide2(const PassArgs<T> &a0, const PassArgs<T> &a1, int c0, int c1,
                           int threads, hipStream_t st);
template <typename T>
hipError_t launch_collide(int mode, const PassArgs<T> &a, int blocks, int threads, size_t lds,
                          hipStream_t st);
template <typename T>
hipError_t launch_staged(int mode, const PassArgs<T> &a, int cs, hipStream_t st);
template <typename T>
hipError_t launch_init(Parts<T> p, int64_t n, double n0, double T_eV, uint64_t id0, int s,
                       const Phys &phys, double m, hipStream_t st);

// fixup.hip: deterministic removal of absorbed particles and appending of new
// ones (identities in parent order, independent of the launch shape).
struct ScanJobs {
    // children staged by the electron pass (electron chunks)
    int children;
    Chunks ech;
    const Counts *ecnt, *icnt;
    ChildRec *crec;
    int kids[2];   // append the staged children of species 0 / 1
    // dead lists of species 0 and 1
    int dead[2];
    Chunks ch[2];
    const Counts *cnt[2];
    FixRec *fix[2];
    int64_t cap[2];
    int32_t *status;
};
// Superchunk totals of the masks (children and/or dead particles).
hipError_t launch_scan(const ScanJobs &j, int64_t max_chunks, hipStream_t st);
// Sorted global dead lists and the kept counts, both species in one launch.
hipError_t launch_dead_list(const ScanJobs &j, int64_t max_chunks, hipStream_t st);
template <typename T>
hipError_t launch_dead_scan(Parts<T> p, const Counts *cnt, Chunks ch, hipStream_t st);
template <typename T>
hipError_t launch_fill(Parts<T> p, Chunks ch, const FixRec *fix, hipStream_t st);
template <typename T>
hipError_t launch_fill2(Parts<T> p0, Parts<T> p1, Chunks ch0, Chunks ch1, const FixRec *fix0,
                        const FixRec *fix1, hipStream_t st);
// Append the staged children after the kept particles of each species (slot
// = parent index, identities in parent order) and commit the counts.
template <typename T>
hipError_t launch_append(const ScanJobs &j, Parts<T> dst0, Parts<T> dst1, Parts<T> stage0,
                         Parts<T> stage1, Counts *cnt0, Counts *cnt1, int64_t max_chunks,
                         hipStream_t st);
// The hole filling and appending of a step's list maintenance kept for
// later launches (step pipelining): they run beside the next step's way-down
// launches (mg_vcycle), or on their own (list_tail_flush).  stage: 2 both
// pending, 1 the appending, 0 nothing.  The launch arguments are kept as
// bytes (Fill2Args<T>, AppendJob<T> of the particles' type).
constexpr int kTailFillBytes = 512, kTailAppBytes = 1536;
struct ListTail {
    int stage = 0;
    int fp32 = 0;
    int nsc = 1;  // superchunks of the appending
    alignas(16) unsigned char fill[kTailFillBytes];
    alignas(16) unsigned char app[kTailAppBytes];
};
template <typename T>
void list_tail_keep(ListTail &t, Parts<T> p0, Parts<T> p1, Chunks ch0, Chunks ch1,
                    const FixRec *fix0, const FixRec *fix1, const ScanJobs &j, Parts<T> dst0,
                    Parts<T> dst1, Parts<T> stage0, Parts<T> stage1, Counts *cnt0, Counts *cnt1,
                    int64_t max_chunks);
// Launches what is pending, on its own (stage becomes 0).
hipError_t list_tail_flush(ListTail &t, hipStream_t st);
// Mode of the periodic resize: the weight-conserving split, or zero-order
// particle-based resizing with draws keyed by (seed, s, id, step).
struct ResizeKey {
    int zero_order, s;
    uint64_t seed;
    uint32_t step;
};
template <typename T>
hipError_t launch_resize(Parts<T> p, Counts *cnt, Chunks ch, CloneRec *rec, const ResizeKey &k,
                         double wcoef, double half_hr, int64_t cap, int32_t *status,
                         hipStream_t st);
// The slice sum of a merged step on its own (blockDim 256; r.bx * 256 >= nn).
hipError_t launch_slice_sum(const SliceSum &r, hipStream_t st);
// FP32 particles: the collisions of both species and the slice sum in one launch.
hipError_t launch_collide_sum(const PassArgs<float> &a0, const PassArgs<float> &a1, int c0,
                              int c1, const SliceSum &r, hipStream_t st);
hipError_t launch_reduce_slices(unsigned long long *acc, const void *slices, int narrow, int nb,
                                int nn, hipStream_t st);

// sort.hip: stable counting sort of a species by tile of the cell of each
// particle, and the window plan of the tiled pass.
template <typename T> struct SortArgs {
    Parts<T> p, tmp;         // particles; staging of the sorted copy
    const Counts *cnt;
    double hr, hz;           // the key divides positions by the spacings
    int nr, nz, tile_z, tile_r, ntr, nt, kbits;
    int64_t seg, nseg;       // particles per segment (one wavefront), segments
    int64_t *off;            // [nt * nseg + 1]: counts, then exclusive offsets
    int64_t *part;           // scan partial sums
    int64_t *tile_pb;        // plan: particles per pass block
    int4 *tile_win;          // plan: [nb] deposit windows
    int nb;                  // pass blocks of the plan
};
template <typename T> hipError_t launch_sort(const SortArgs<T> &a, hipStream_t st);

// grid.hip
struct GridArgs {
    int nr, nz, nn;
    double hr, hz, dt;
    const unsigned long long *acc0, *acc1;
    double quantum0, quantum1;
    double q0, q1, m0, m1;
    const double *vol;
    double *dens0, *dens1, *rho, *chi, *eps, *f;
    float *eps32;
    int zero_acc;
    unsigned long long *acc0w, *acc1w;
    int32_t *status;
    double dt1;   // ion time step in chi
    int friedman; // Friedman damping: each chi term scaled by theta
    double theta;
    int ion_chi;  // the ions move in the coming step: their chi term is on
    int keep1;    // keep the ion deposit (subcycled ions that do not move)
};
hipError_t launch_finalize(const GridArgs &g, hipStream_t st);
template <typename T>
hipError_t launch_efield(int nr, int nz, double hr, double hz, const double *phi, double *er,
                         double *ez, typename Vec2<T>::type *E2, hipStream_t st,
                         unsigned long long *zero0 = nullptr, unsigned long long *zero1 = nullptr,
                         unsigned long long *clear = nullptr, int nclear = 0);
template <typename T>
hipError_t launch_pack_e2(int nn, const double *er, const double *ez, typename Vec2<T>::type *E2,
                          hipStream_t st);
hipError_t launch_acc_convert(int nn, unsigned long long *acc, double *dev, double quantum,
                              int to_acc, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t st);

// mg.hip
struct MgLevels {
    int L, nr;
    int nzl[kMaxLevels + 1];
    double hzl[kMaxLevels + 1];
    double *eps64[kMaxLevels + 1];
    float *eps32[kMaxLevels + 1];
    double *u64[kMaxLevels + 1], *f64[kMaxLevels + 1];
    float *u32[kMaxLevels + 1], *f32[kMaxLevels + 1];
    int chi_face;
    double hr;
    int K;                 // coarse levels 1..K solved by the single-block bottom kernel
    size_t bottom_lds;     // its LDS bytes
    // Single-block cycles: every level's right-hand side and correction held
    // in LDS (FP64: the finest level is phi itself, in global memory), the
    // line matrices factored beforehand into per-line tables.
    int one_block;         // 1: every cycle in one single-workgroup launch
    int split;             // 1: per cycle a residual/restriction launch, then the way
                           //    up: each finest-level block with the coarse lines
                           //    it depends on (or, split_coarse, the coarse levels
                           //    in one workgroup and then the finest level's sweep)
    int split_coarse;      // 1: the split cycle's two-launch way up
    int S;                 // reduction steps of an r-line (ceil(log2(nr - 1)))
    int line_off[kMaxLevels + 2];  // first table line of each level; line_off[L+1] = total
    int tab_row;           // elements per row of a line table: nr - 1 rounded up to a
                           //    multiple of 8 (the padding: zero coefficients and
                           //    multipliers, b_final 1)
    size_t tab_stride;     // elements per line table: (3 + 2 S) tab_row
    void *tab;             // line tables, float (mixed) or double
    void *coarse_uf;       // levels 1..L-1: u then f of each level in one block
                           //    (float when mixed), the coarse solve's LDS image
    double *res;           // finest-level residual scratch
    double *cf64;          // FP64 operator of the finest level: a, b, c, d, e arrays [nz][nr]
    size_t solve_lds;      // LDS bytes of the single-block kernel
    size_t lds_budget;     // LDS bytes of one workgroup
    int long_lines;        // r-lines solved by the partition method, two half-sweeps per level
};
hipError_t mg_restrict_eps(const MgLevels &m, int mixed, hipStream_t st);
// The merged step's grid preparation in one launch: finalize every node,
// restrict epsilon down the levels, set the Dirichlet values of phi0 (and of
// phi1 if non-null) for the electrode voltage V, clear `nclear` counters.
hipError_t mg_finalize(const GridArgs &g, const MgLevels &m, int mixed, double *phi0, double *phi1,
                       double V, unsigned long long *clear, int nclear, hipStream_t st);
hipError_t mg_resid_norm(const MgLevels &m, const double *u, const double *f, int zero_interior,
                         unsigned long long *norm, hipStream_t st);
hipError_t mg_set_bc(double *phi, int nr, int nz, double V, hipStream_t st);
// Plans both cycle paths for `lds_budget` bytes of LDS per block: the
// single-block path when every level fits (one_block, S, line_off,
// tab_stride, solve_lds; the caller allocates tab with line_off[L+1] *
// tab_stride elements and res), and the levels of the bottom kernel of the
// multi-launch path (K, bottom_lds).
// path: 0 split where it fits (single block for one-line meshes), 1 single
// block where it fits, 2 multi-launch, 3 long-line half-sweeps.
void mg_plan(MgLevels &m, int mixed, size_t lds_budget, int path);
// Single-block path: factor every line matrix of every level (once per solve,
// after mg_restrict_eps), then run `cycles` V(0,1) cycles on phi in one
// launch, the Dirichlet values of phi set first.
hipError_t mg_factor(const MgLevels &m, int mixed, hipStream_t st);
hipError_t mg_solve_block(const MgLevels &m, int mixed, double *phi, const double *f, double V,
                          int cycles, hipStream_t st);
// One V(0,1) cycle of the multi-launch path.  FP64: the finest level
// alternates between phi and phi_alt (both carry the boundary values); the
// pointers are swapped.  With a pending list tail (step pipelining), its
// next stage runs in the way-down launch of the split path, beside it.
hipError_t mg_vcycle(const MgLevels &m, int mixed, double *&phi, double *&phi_alt,
                     const double *f, int skip_down, hipStream_t st, ListTail *tail = nullptr);
// Split path, first launch of a solve (after the Dirichlet values are set):
// the line tables and the first cycle's residual restriction; that cycle then
// runs mg_vcycle with skip_down = 1.
hipError_t mg_prep(const MgLevels &m, int mixed, const double *phi, const double *f,
                   hipStream_t st);
// Step pipelining: the superchunk totals of the list maintenance (as
// launch_scan) beside mg_finalize without its counter clearing (nothing is
// cleared: the deposit grids keep their values), then the dead lists (as
// launch_dead_list) beside mg_prep; the split path only.
hipError_t mg_finalize_scan(const GridArgs &g, const MgLevels &m, int mixed, double *phi0,
                            double *phi1, double V, const ScanJobs &j, int64_t max_chunks,
                            hipStream_t st);
hipError_t mg_prep_dead_list(const MgLevels &m, int mixed, const double *phi, const double *f,
                             const ScanJobs &j, int64_t max_chunks, hipStream_t st);

}  // namespace rz
