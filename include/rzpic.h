/*
 * rzpic.h -- C ABI of the MI355X (gfx950) library for the hot path of the
 * implicit electrostatic r-z PIC/MC model of Wang, Jiang & Wang (arXiv
 * 1001.2969): the direct-implicit particle cycle (Sec. 2.1, 2.3), weighting
 * with radius-dependent volumes (Sec. 2.4), weight splitting (Sec. 2.2),
 * null-collision Monte Carlo (Sec. 2.6) and the z-semi-coarsening multigrid
 * field solve of div((1+chi) grad phi) = -rho/eps0 (Sec. 2.5, Algorithm 1).
 *
 * Conventions
 *   - Every entry point returns an rzpic_status; no exception crosses the ABI.
 *     On failure rzpic_last_error() returns a message (thread-local).
 *   - "device" pointers are HIP device allocations on the context's device;
 *     "host" pointers are ordinary host memory.  The library never frees a
 *     pointer it did not allocate.
 *   - Work is enqueued asynchronously on the context's stream unless a call
 *     says it synchronises.  Device-side failures (capacity overflow,
 *     fixed-point overflow, non-finite values) set a sticky status word that
 *     the next synchronising call returns.
 *   - Mesh: nr nodes in r (r_j = j*hr, hr = R/(nr-1)), nz nodes in z
 *     (z_i = i*hz, hz = L/(nz-1)), nz-1 a power of two.  Grids are row-major
 *     [nz][nr] (r contiguous), double precision, index i*nr + j.
 *   - Species 0 are electrons, species 1 positive ions.  Particle records are
 *     structures of arrays {r, z, v_r, v_theta, v_z, a_r, a_z, w, id}
 *     (Sec. 2.3 record plus the weight of Sec. 2.2 and a 64-bit identity).
 *     Positions in m, velocities in m/s, damped accelerations in m/s^2,
 *     weights in physical particles.  Real arrays are double in RZPIC_FP64
 *     and float in RZPIC_MIXED.
 */
#ifndef RZPIC_H
#define RZPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rzpic_status {
    RZPIC_OK = 0,
    RZPIC_EINVAL = 1,     /* bad argument or configuration                  */
    RZPIC_ENOMEM = 2,     /* device allocation failed                       */
    RZPIC_EHIP = 3,       /* a HIP runtime call failed                      */
    RZPIC_ECAPACITY = 4,  /* particle capacity exceeded (children dropped)  */
    RZPIC_ENOTCONV = 5,   /* multigrid did not reach the tolerance          */
    RZPIC_ENUMERIC = 6,   /* fixed-point overflow or non-finite value       */
    RZPIC_ESTATE = 7      /* call out of order (e.g. species not bound)     */
} rzpic_status;

enum { RZPIC_FP64 = 0, RZPIC_MIXED = 1 };          /* precision            */
enum { RZPIC_W_ZR2 = 0, RZPIC_W_ZR = 1 };          /* weighting, Sec. 2.4  */
enum { RZPIC_FACE_AVG = 0, RZPIC_FACE_MAX = 1 };   /* half-point chi, Sec. 2.5 */
enum { RZPIC_MC_NONE = 0, RZPIC_MC_ELECTRON = 1, RZPIC_MC_ION = 2 };
/* Particle push (Sec. 2.3): the local X-Y push with rotation, a_theta dropped
 * (default), or the global X-Y-Z push (Cartesian particles in the 2-D field),
 * carried in the particle's local frame: a_theta is kept (species view `at`),
 * turned with the frame at every first push and damped by the final push
 * (E has no theta component at the particle), and a particle the final push
 * carries through the axis goes on at the other side (frame turned by pi)
 * instead of the axis rule. */
enum { RZPIC_PUSH_LOCAL = 0, RZPIC_PUSH_XYZ = 1 };
/* Periodic resize (Sec. 2.2): the weight-conserving split (default), or
 * zero-order particle-based resizing: a particle of weight w whose weight at
 * its radius should be w_r = resize_wcoef * max(r, hr/2) is kept as
 * floor(w/w_r) copies plus one more with probability frac(w/w_r) (first
 * uniform of draw block 6 of (seed, s, id, step)), each of weight w_r; none
 * removes it; duplicates copy its record, take new identities in parent
 * order and are appended, then the array is compacted (rzpic_resize alone
 * keys its draws by step 0). */
enum { RZPIC_RESIZE_SPLIT = 0, RZPIC_RESIZE_ZERO_ORDER = 1 };
/* Time-averaged acceleration of the implicit push.  RZPIC_DAMP_D1: the D1
 * scheme of Sec. 2.1, abar_n = (a_{n+1} + abar_{n-1}) / 2.
 * RZPIC_DAMP_FRIEDMAN: the adjustable damping of A. Friedman, J. Comput.
 * Phys. 90 (1990) 292 (cited in the discussion of Sec. 4), read as
 *   abar_n = (theta/2) a_{n+1}
 *          + (1 - theta/2) [(1 - theta/2) a_n + (theta/2) abar_{n-1}]
 * with 0 <= theta <= 1: leapfrog at theta = 0, more damping of the fast
 * oscillations as theta grows.  The implicit coefficient of a_{n+1} (and so
 * chi) is theta/2 instead of 1/2, and the species views' ar, az hold the
 * known part B = abar_n - (theta/2) a_{n+1} of the next step instead of
 * abar (zero at initialisation, as abar).  Local push only; the gradient
 * window (rzpic_adjoint_*) takes D1. */
enum { RZPIC_DAMP_D1 = 0, RZPIC_DAMP_FRIEDMAN = 1 };
enum { RZPIC_P_ELASTIC = 0, RZPIC_P_EXCITATION = 1, RZPIC_P_IONIZATION = 2 };
/* Grid selectors of rzpic_grid_copy.  N0/N1 are the deposited physical
 * particle counts N_ij of Sec. 2.4 (kept internally in fixed point). */
enum {
    RZPIC_G_PHI = 0, RZPIC_G_RHO = 1, RZPIC_G_CHI = 2, RZPIC_G_ER = 3, RZPIC_G_EZ = 4,
    RZPIC_G_N0 = 5, RZPIC_G_N1 = 6, RZPIC_G_DENS0 = 7, RZPIC_G_DENS1 = 8, RZPIC_G_VOL = 9,
    RZPIC_G_PHI_P = 10, RZPIC_G_PHI_L = 11  /* external circuit: charge and unit Laplace solutions */
};
/* Per-particle Monte Carlo event codes written to rzpic_species_view.mc_event:
 * 0 not a candidate, 1 null collision, 2+k real collision of process k. */
enum { RZPIC_EV_NONE = 0, RZPIC_EV_NULL = 1, RZPIC_EV_PROC0 = 2 };

typedef struct rzpic_config {
    int32_t nr, nz;           /* nodes; nr >= 3, nz-1 = 2^k, k >= 1          */
    double R, L, dt;          /* radius, electrode gap (m), time step (s)    */
    int32_t precision;        /* RZPIC_FP64 or RZPIC_MIXED                    */
    int32_t weighting;        /* RZPIC_W_ZR2 (default) or RZPIC_W_ZR          */
    int32_t chi_face;         /* RZPIC_FACE_AVG or RZPIC_FACE_MAX             */
    int32_t fixed_point_bits; /* deposit quantum = w_ref * 2^-bits (0 -> 46 in
                               * RZPIC_FP64, 26 in RZPIC_MIXED): one
                               * contribution must stay below 2^51 quanta in
                               * FP64 (weights below 2^(51-bits) w_ref) and
                               * below 1.5 2^30 in MIXED, which forms each
                               * contribution in FP32 as a 32-bit integer
                               * (weights below 1.5 2^(30-bits) w_ref; at most
                               * 30 bits there, else EINVAL); a node's total
                               * must stay below 2^63.  46 bits keep the
                               * rounding of the FP64 deposit near 1e-14 of a
                               * node's count */
    double V_dc, V_rf, f_rf;  /* z=0 electrode: V_dc + V_rf sin(2 pi f_rf t) */
    uint64_t seed;            /* Philox key of every random draw             */
    double mg_tol;            /* relative L-inf residual target (Sec. 2.5)   */
    int32_t mg_max_cycles;    /* cap on V(0,1) cycles per solve              */
    int32_t mg_fixed_cycles;  /* > 0: exactly this many cycles, no test      */
    int32_t resize_every;     /* weight split period in steps, 0 = never     */
    int32_t sort_every;       /* tile sort period in steps (rzpic_sort of both
                               * species at the end of every sort_every-th
                               * step), 0 = never                            */
    double resize_wcoef;      /* split weight w_r(r) = resize_wcoef*max(r,hr/2) */
    double n_gas, T_gas, m_gas; /* neutral density (m^-3), temperature (K), mass (kg) */
    int32_t tile_z, tile_r;   /* cells per sort tile in z and r (0 -> 16, 32);
                               * at most 2048 tiles                          */
    double circuit_C;         /* > 0: a blocking capacitor of this capacitance
                               * (F) between the source V_dc + V_rf sin(2 pi
                               * f_rf t) and the z=0 electrode, whose potential
                               * then follows the circuit (Sec. 2.5, see
                               * rzpic_set_circuit); 0: driven directly      */
    int32_t ion_subcycle;     /* K >= 2: the ions (species 1) move only in every
                               * K-th step (steps K-1, 2K-1, ...) with time step
                               * K dt (pushes, P_null, chi), the subcycling of
                               * Sec. 2.7; in the other steps their deposit is
                               * kept and they add charge but no chi, and ions
                               * born from ionizations are first-pushed with
                               * K dt.  0 or 1: every step.  rzpic_step only:
                               * the single operations act as in a step where
                               * the ions move. */
    int32_t push_form;        /* RZPIC_PUSH_LOCAL (0) or RZPIC_PUSH_XYZ        */
    int32_t resize_mode;      /* RZPIC_RESIZE_SPLIT (0) or RZPIC_RESIZE_ZERO_ORDER */
    int32_t damping;          /* RZPIC_DAMP_D1 (0) or RZPIC_DAMP_FRIEDMAN       */
    double theta;             /* RZPIC_DAMP_FRIEDMAN: damping parameter in [0, 1] */
} rzpic_config;

typedef struct rzpic_species_view {
    /* device arrays of `capacity` elements (double in FP64, float in MIXED) */
    void *r, *z, *vr, *vt, *vz, *ar, *az, *w;
    uint64_t *id;             /* device, unique particle identities          */
    uint8_t *mc_event;        /* optional device array (capacity bytes) of MC
                                 event codes of the last collision pass, or NULL */
    int64_t capacity;         /* elements of every array above              */
    double q, m;              /* charge (C) and mass (kg)                    */
    double w_ref;             /* reference weight of the fixed-point deposit */
    int32_t mc_model;         /* RZPIC_MC_*                                  */
    int32_t reserved0;
    void *at;                 /* RZPIC_PUSH_XYZ: device array of `capacity`
                               * a_theta values (moved with the particles);
                               * ignored by the local push                   */
} rzpic_species_view;

typedef struct rzpic_diag {
    int64_t count[2];          /* live particles per species                */
    uint64_t next_id[2];       /* next identity to assign per species       */
    double absorbed[2][3];     /* cumulative weight absorbed at z=0, z=L, r=R */
    int64_t candidates[2];     /* MC candidates of the last collision pass  */
    int64_t events[2][4];      /* real collisions per process, last pass    */
    int32_t last_cycles;       /* V-cycles of the last solve                */
    int32_t status;            /* sticky device status (rzpic_status)       */
    double last_relres;        /* ||f - A phi||_inf / ||f_bc||_inf, last solve (tol mode) */
    uint64_t particle_steps[2];/* cumulative live particles entering rzpic_step passes */
} rzpic_diag;

typedef struct rzpic_ctx rzpic_ctx;

/* Create a context on the current HIP device.  `stream` is a hipStream_t (NULL
 * = default stream).  Allocates every internal grid and multigrid level;
 * particle work buffers are allocated by rzpic_bind_species.  Validates the
 * configuration (EINVAL with a message). */
rzpic_status rzpic_create(const rzpic_config *cfg, void *stream, rzpic_ctx **out);
/* Free a context and everything it allocated (synchronises its stream). */
rzpic_status rzpic_destroy(rzpic_ctx *ctx);
/* Change the stream later work is enqueued on. */
rzpic_status rzpic_set_stream(rzpic_ctx *ctx, void *stream);

/* Attach caller-owned particle arrays of species s (0 or 1), of capacity
 * 1 .. 2^29 - 64 (EINVAL beyond).  The arrays must outlive the binding.  Allocates per-species scratch sized by `capacity`
 * (chunk tables, new-particle staging).  The particle count becomes 0. */
rzpic_status rzpic_bind_species(rzpic_ctx *ctx, int32_t s, const rzpic_species_view *v);
/* Set the live count n (<= capacity) and the next identity of species s
 * (asynchronous host-to-device write). */
rzpic_status rzpic_set_count(rzpic_ctx *ctx, int32_t s, int64_t n, uint64_t next_id);
/* Read the live count and next identity.  Synchronises the stream, and like
 * rzpic_sync returns (and clears) a pending device-side failure such as
 * RZPIC_ECAPACITY; the counts are written either way. */
rzpic_status rzpic_get_count(rzpic_ctx *ctx, int32_t s, int64_t *n, uint64_t *next_id);

/* Cross sections of species s (Sec. 2.6) on the uniform energy grid
 * eps_k = k*de eV, k < ne: host arrays kind[nproc] (RZPIC_P_*), thr_eV[nproc]
 * and sigma[nproc][ne] (m^2, linearly interpolated, 1/E above the table).
 * ej_B is the ejected-electron energy constant (eV) of ionization.  Computes
 * the null-collision frequency nu_max (a rigorous bound of n_gas*sigma_T*g
 * over all energies) and P_null = 1 - exp(-nu_max dt) on the host. */
rzpic_status rzpic_set_xsec(rzpic_ctx *ctx, int32_t s, int32_t nproc, const int32_t *kind,
                            const double *thr_eV, double de, int32_t ne, const double *sigma,
                            double ej_B);
rzpic_status rzpic_get_mc_consts(rzpic_ctx *ctx, int32_t s, double *nu_max, double *p_null);

/* Sec. 2.3 initialisation of n particles of species s: r = U R, z = U L,
 * w = 2 pi n0 R L r / n (uniform density n0), Maxwellian velocities at T_eV,
 * zero damped accelerations, identities id0 .. id0+n-1 (Philox draws keyed by
 * (seed, s, id, step 0xFFFFFFFF)).  Sets the count to n. */
rzpic_status rzpic_init_particles(rzpic_ctx *ctx, int32_t s, int64_t n, double n0,
                                  double T_eV, uint64_t id0);

/* --- the cycle of Sec. 2.1, one operation per call --------------------- */
/* First push in the local X-Y frame and rotation onto the new radius
 * (Sec. 2.3); absorbed particles are marked and tallied. */
rzpic_status rzpic_push_first(rzpic_ctx *ctx, int32_t s);
/* Deposit N_ij of both species from scratch (Sec. 2.4), then n = N/V,
 * rho = sum q n and chi = sum q^2 n dt^2 / (2 m eps0) (Sec. 2.1). */
rzpic_status rzpic_deposit(rzpic_ctx *ctx);
/* Multigrid solve (Sec. 2.5) of the implicit field equation with phi = V(t)
 * on z = 0, 0 on z = L and r = R, warm-started from the current phi.
 * Fixed-cycle mode runs config.mg_fixed_cycles V(0,1) cycles without a
 * test; otherwise cycles until the relative residual <= mg_tol, tested after
 * every cycle.  That mode synchronises once per batch of cycles, not once per
 * cycle: the solution is kept before each cycle of a batch, so the solve
 * still stops at the first cycle that meets the tolerance (the first batch
 * takes the cycles the previous solve needed; meshes above 8M nodes test
 * after every cycle).  cycles / relres (host, may be NULL) receive the
 * cycles run and the final relative residual (requesting them synchronises).
 * ENOTCONV if the tolerance is not met. */
rzpic_status rzpic_solve(rzpic_ctx *ctx, double t, int32_t *cycles, double *relres);
/* The same solve with its results left on the device: cycles_dev (device
 * int32) and relres_dev (device double), each may be NULL, are written on
 * the stream.  Fixed-cycle mode never synchronises (relres_dev costs two
 * residual kernels; EINVAL with an external circuit, whose two solutions
 * have a residual each); tolerance mode synchronises as rzpic_solve. */
rzpic_status rzpic_solve_dev(rzpic_ctx *ctx, double t, int32_t *cycles_dev, double *relres_dev);
/* Change the multigrid cycling of later solves (same meaning as the config
 * fields mg_tol, mg_max_cycles, mg_fixed_cycles). */
rzpic_status rzpic_set_mg(rzpic_ctx *ctx, double tol, int32_t max_cycles, int32_t fixed_cycles);
/* E = -grad phi on the nodes. */
rzpic_status rzpic_efield(rzpic_ctx *ctx);
/* Gather of E at the first-pushed position, final push, damped-acceleration
 * update, axis rule and absorption (Sec. 2.1, 2.3). */
rzpic_status rzpic_push_final(rzpic_ctx *ctx, int32_t s);
/* Null-collision Monte Carlo of species s at step `step` (Sec. 2.6).  New
 * particles wait in staging until rzpic_compact; rzpic_push_first and
 * rzpic_deposit include them. */
rzpic_status rzpic_collide(rzpic_ctx *ctx, int32_t s, int64_t step);
/* Remove absorbed particles (holes below n-D filled in order by the live
 * particles of [n-D, n)) and append the staged new particles of species s. */
rzpic_status rzpic_compact(rzpic_ctx *ctx, int32_t s);
/* Weight split of Sec. 2.2 (clones appended in parent order). */
rzpic_status rzpic_resize(rzpic_ctx *ctx, int32_t s);
/* Stable sort of the particles of species s by tile (Sec. 2.7 orders
 * particles by cell for the weighting): key = tile of the cell
 * (floor(z/hz), floor(r/hr)), clamped to the mesh, tiles of tile_z x tile_r
 * cells numbered r fastest; particles of one tile keep their order.  Moves
 * every particle array (mc_event is not reordered).  When the deposit grid
 * does not fit in LDS, later particle passes give each block a contiguous
 * range of the sorted array and deposit into an LDS window of its tiles; the
 * results do not depend on it.  ESTATE while new particles are staged.
 * Allocates the sort's scratch on first use unless config.sort_every > 0
 * (then rzpic_bind_species does). */
rzpic_status rzpic_sort(rzpic_ctx *ctx, int32_t s);
/* After initialisation: first push, deposit and compaction of both species. */
rzpic_status rzpic_prologue(rzpic_ctx *ctx);
/* One merged step n (Sec. 2.1): finalize rho/chi, solve at t = (n+1) dt,
 * E, one fused particle pass per species (gather, final push, MC, first
 * push, deposit), compaction, the periodic weight split (with the deposit
 * redone) and the periodic tile sort.  Equal, bit for bit, to the
 * composition of the single operations above. */
rzpic_status rzpic_step(rzpic_ctx *ctx, int64_t step);

/* Graph replay of rzpic_step (off by default): each step's launches are
 * captured from the context's stream and replayed as one HIP graph, the
 * executable graph of the step's variant (ions moving or not, weight split,
 * tile sort) updated in place with the step's arguments.  The results are
 * those of the direct step, bit for bit; the GPU saves about a microsecond
 * of dispatch per kernel.  Steps run directly while step timing is on,
 * while a batch records them, or when the solve runs to a tolerance.
 * EINVAL when enabling on the null stream or with mg_fixed_cycles = 0.
 * The executable graphs are freed by rzpic_destroy. */
rzpic_status rzpic_set_step_graph(rzpic_ctx *ctx, int32_t on);

/* Step pipelining of rzpic_step (off by default): a directly launched step
 * n that makes no weight split also prepares the grid of step n + 1 (the
 * finalize of its deposit, the epsilon levels, the Dirichlet values for the
 * voltage at t = (n+2) dt, the line tables and the first restriction of the
 * solve), in the launches of its own list maintenance; step n + 1, if it
 * comes next, skips that preparation and clears the deposit grids and the
 * Monte Carlo counters in its E launch.  Unless a tile sort follows in step
 * n, its hole filling and appending are kept and run in step n + 1's
 * way-down and way-up launches.  Particles, potentials and counters after
 * every step are those of unpipelined steps, bit for bit; between steps,
 * rho, chi, eps, the densities and the electrode rows of phi are already
 * those of the next step.  Every call that reads or changes particles,
 * counts or grids (rzpic_get_count, rzpic_sync, rzpic_get_diag,
 * rzpic_grid_copy, and every operation) first launches the kept filling and
 * appending on the context's stream, so the particle arrays are final once
 * such a call has been made: a caller reading the bound arrays directly
 * calls rzpic_sync first.  Applies only to the split solve path with a
 * fixed number of cycles and no external circuit; graph-replayed and
 * batched steps prepare their own grid.  Every call that changes particles,
 * deposits, potentials, voltages or solver settings drops the preparation;
 * writes through a grid view (rzpic_grid_view) between steps do not, so a
 * caller that writes phi there turns pipelining off first. */
rzpic_status rzpic_set_step_pipeline(rzpic_ctx *ctx, int32_t on);

/* Launch shape of the fused particle pass: threads per block (256, 512, 768
 * or 1024) and particles of capacity per block (default 512 threads, 8192).
 * Results do not depend on it (integer deposit, identities from event
 * ranks, compaction by index), only the speed.  A tile-sorted context is
 * sorted again so that its tile plan fits the new block count.  EINVAL for
 * a shape beyond the pass's wavefront limit. */
rzpic_status rzpic_set_pass_shape(rzpic_ctx *ctx, int32_t threads, int32_t parts_per_block);
/* Autotuner of that shape: for each of threads {256, 512, 768, 1024} x
 * particles per block {2048, 4096, 8192, 16384} that fits, one warm-up and
 * `steps` timed rzpic_step calls (HIP events on the context's stream),
 * starting at step `step0`; keeps the first shape in that order within 2 %
 * of the fastest (near-ties do not flip between runs).  table (host, may be NULL)
 * receives 16 rows {threads, parts_per_block, ms per step or -1 if skipped};
 * best = {threads, parts_per_block}; *next_step the next step index.  The
 * simulation advances by the steps run.  Synchronises. */
rzpic_status rzpic_autotune(rzpic_ctx *ctx, int32_t steps, int64_t step0, double *table,
                            int32_t best[2], int64_t *next_step);

/* Deposit form of the fused pass (speed only: the deposit of Sec. 2.4 is
 * the same integer sum in every form).  RZPIC_FORM_AUTO: each block
 * privatises the whole grid in LDS when it fits (the default);
 * RZPIC_FORM_LDS: that form, EINVAL when the grid does not fit one
 * workgroup's LDS; RZPIC_FORM_TILED: each block deposits into an LDS window
 * of the tiles planned at the last tile sort (rzpic_sort, or the periodic
 * sort of rzpic_step), by global atomics without a plan.  A context with a
 * plan is sorted again for the block count of the new form.  EINVAL when
 * the current pass shape exceeds the wavefront limit in that form. */
enum { RZPIC_FORM_AUTO = 0, RZPIC_FORM_LDS = 1, RZPIC_FORM_TILED = 2 };
rzpic_status rzpic_set_pass_form(rzpic_ctx *ctx, int32_t form);
/* Tile shape of the particle sort: tile_z x tile_r cells (both >= 1, at
 * most 2048 tiles, EINVAL otherwise).  Speed only; the particle order after
 * a sort follows the tiles.  Synchronises the stream when sort scratch
 * exists (it is sized by the tile count and allocated again); a species
 * that has a plan is sorted again at once by the new tiles. */
rzpic_status rzpic_set_tiles(rzpic_ctx *ctx, int32_t tile_z, int32_t tile_r);
/* The pass configuration in use: out = {threads, parts_per_block, form
 * (RZPIC_FORM_LDS or RZPIC_FORM_TILED), tile_z, tile_r} (host array). */
rzpic_status rzpic_get_pass_config(rzpic_ctx *ctx, int32_t out[5]);

/* Device pointers of the context's own grids ([nz][nr] doubles, row-major),
 * for reading and writing them in place with no copy.  Owned by the context
 * (valid until rzpic_destroy), except that FP64 solves move phi between two
 * buffers: phi (and phi_p, phi_l) is valid until the next rzpic_solve,
 * rzpic_solve_dev or rzpic_step.  rho and chi written here are the sources
 * of the next rzpic_solve (rzpic_step forms them from the deposit).  er and
 * ez are the nodal field of the last rzpic_efield (the particle gather reads
 * its own packed copy: write them through rzpic_grid_copy).  phi_p, phi_l:
 * the external circuit's charge and unit Laplace solutions, NULL without a
 * circuit.  dens: the particle densities n_s = N_s / V of the last finalize,
 * vol the weighting volumes V_ij (Sec. 2.4). */
typedef struct rzpic_grid {
    int32_t nr, nz;
    double *phi, *rho, *chi, *er, *ez;
    double *dens[2];
    double *vol;
    double *phi_p, *phi_l;
} rzpic_grid;
rzpic_status rzpic_grid_view(rzpic_ctx *ctx, rzpic_grid *out);
/* Source of a solver-only use (rzpic_solve without particles): copies
 * rho (C/m^3) and chi (device arrays of nz*nr doubles, caller-owned, read
 * before the call returns on the stream) into the context's grids.
 * Asynchronous. */
rzpic_status rzpic_set_grid_source(rzpic_ctx *ctx, const double *rho, const double *chi);

/* Copy grid `which` (RZPIC_G_*) between the context and a caller device
 * buffer of nz*nr doubles: to_ctx = 0 reads from the context, 1 writes into
 * it (PHI, RHO, CHI, ER, EZ, N0, N1 writable).  Asynchronous. */
rzpic_status rzpic_grid_copy(rzpic_ctx *ctx, int32_t which, double *dev, int32_t to_ctx);
/* Diagnostics (synchronises; returns the sticky device status). */
rzpic_status rzpic_get_diag(rzpic_ctx *ctx, rzpic_diag *out);
/* Synchronise the stream and return (and clear) the sticky device status. */
rzpic_status rzpic_sync(rzpic_ctx *ctx);
/* Message of the last failure on this thread. */
const char *rzpic_last_error(void);
/* Physical constants used inside the library: e, m_e, amu, eps0, k_B, 2 pi. */
void rzpic_constants(double out[6]);
/* Device-time accounting of rzpic_step with HIP events on the context's
 * stream (off by default; each event costs the stream a few microseconds).
 * rzpic_get_timing synchronises and returns, averaged over the steps recorded
 * since the previous call (then resets):
 *   out[0] steps recorded            out[1] whole step (ms)
 *   out[2] field solve (ms)          out[3] V-cycles per solve
 *   out[4] fused particle pass of both species, the kernel alone (ms)
 *   out[5] collision kernels of both species + deposit slice sum (ms)
 *   out[6] finalize + E field (ms)   out[7] list maintenance (ms)
 *   out[8] electrons, out[9] ions entering the pass (per step)
 *   out[10] weight split (ms, 0 on other steps)
 *   out[11] tile sort and the deposit redone after a weight split (ms) */
rzpic_status rzpic_set_timing(rzpic_ctx *ctx, int32_t enable);
rzpic_status rzpic_get_timing(rzpic_ctx *ctx, double out[12]);

/* --- batched steps of independent discharges ---------------------------- */
/* Many independent discharges (contexts of any mesh, particle count and
 * precision) stepped together.  Each rzpic_batch_step performs rzpic_step on
 * every context, equal to it bit for bit, but groups the discharges whose
 * launch sequences are identical (same mesh, precision and options) and runs
 * each group position by position: kernels written for it cover the whole
 * group in one launch (a device job table gives each discharge its arguments
 * and blocks), the others are launched per discharge; the groups run on up to
 * four streams of their own.  Requirements, checked at create and at every
 * step (EINVAL): both species bound, mg_fixed_cycles > 0 (no solve
 * synchronises), step timing off, no staged new particles.  A step that fails
 * while recording leaves the contexts recorded before it advanced on the
 * host: destroy them.  The batch orders itself after the contexts' streams
 * and the streams after the batch; the contexts must not be stepped
 * elsewhere meanwhile.  ctxs is a host array of n handles (copied).  The
 * batch allocates a device job table and two pinned staging buffers, grown
 * as needed. */
typedef struct rzpic_batch rzpic_batch;
rzpic_status rzpic_batch_create(rzpic_ctx *const *ctxs, int32_t n, void *stream,
                                rzpic_batch **out);
rzpic_status rzpic_batch_step(rzpic_batch *batch, int64_t step);
/* Replay steps from a captured HIP graph (off by default): a step whose
 * launches are all batched is captured (job-table upload, fork, launches,
 * join) the first time its layout occurs for each of the two staging
 * buffers, and later such steps relaunch that graph after writing their job
 * tables; other steps (tile sort, weight split) launch directly.  Needs a
 * non-null batch stream (EINVAL). */
rzpic_status rzpic_batch_set_graph(rzpic_batch *batch, int32_t on);
/* out[0] groups, out[1] launches and out[2] of them batched, last step. */
rzpic_status rzpic_batch_stats(rzpic_batch *batch, int32_t out[3]);
/* Autotuner of the pass configuration of a batch (Sec. 2.7's regime of
 * many particles on small grids, where the per-block fixed costs of the
 * deposit decide the speed): the contexts are grouped by mesh and
 * precision, and for each group, stepped as a batch of its own, one warm-up
 * and `steps` timed steps (HIP events on the batch stream) are run for its
 * current configuration, then for each launch shape (threads {256, 512,
 * 1024} x particles per block {2048, 4096, 8192, 16384}) in each deposit
 * form the group can run (RZPIC_FORM_LDS where the grid fits LDS,
 * RZPIC_FORM_TILED where the contexts sort, sort_every > 0), then, where
 * they sort, for tile shapes {8x16, 8x32, 16x16, 16x32, 16x64, 32x32,
 * 32x64} (z x r cells, at most 2048 tiles) with the fastest tiled shape.  Each group
 * keeps the first configuration, in that order, within 2 % of its fastest.
 * Groups whose search took fewer steps are stepped on to the same step, so
 * every context ends at *next_step.  table (host, may be NULL): up to
 * max_rows rows of 8 doubles {group, threads, parts_per_block, form, tile_z,
 * tile_r, ms per step, chosen 0/1}; *rows (may be NULL) the rows the search
 * made.  The simulation advances; results do not depend on the
 * configuration (particle order after a sort follows the tiles).
 * Synchronises. */
rzpic_status rzpic_batch_autotune(rzpic_batch *batch, int32_t steps, int64_t step0,
                                  double *table, int32_t max_rows, int32_t *rows,
                                  int64_t *next_step);
rzpic_status rzpic_batch_destroy(rzpic_batch *batch);

/* Change the z = 0 electrode voltage V_dc + V_rf sin(2 pi f_rf t) of later
 * solves (config fields of the same names; finite values, else EINVAL). */
rzpic_status rzpic_set_voltage(rzpic_ctx *ctx, double V_dc, double V_rf, double f_rf);

/* --- external circuit (config.circuit_C > 0) ----------------------------- */
/* Sec. 2.5, the superposition of Vahedi: each solve computes phi_P (the
 * charge with the electrode at 0 V) and phi_L (no charge, electrode at 1 V)
 * with the same operator and cycling (two solves, warm-started from their
 * previous solutions), the electrode charges Q_P of phi_P and Q_L of phi_L
 * (Gauss's law on the electrode nodes' half cells: the displacement
 * eps0 (1+chi) E through their upper faces and the side face towards the
 * wall node, less the deposited charge of row 0), the charge Q_conv that
 * reached the electrode since the previous solve (z = 0 tallies), then
 *   V = (Q - Q_c + Q_conv + C V_s(t) - Q_P) / (Q_L + C),
 *   Q <- Q_P + V Q_L,  Q_c <- C (V_s(t) - V),  phi = phi_P + V phi_L.
 * The state starts at V = Q = Q_c = 0; rzpic_set_circuit sets it
 * (asynchronous), rzpic_get_circuit reads {V, Q, Q_c, Q_conv, Q_P, Q_L} of
 * the last solve (synchronises).  EINVAL without a circuit. */
rzpic_status rzpic_set_circuit(rzpic_ctx *ctx, double V, double Q, double Qc);
rzpic_status rzpic_get_circuit(rzpic_ctx *ctx, double out[6]);

/* --- adjoint of a collision-free window ---------------------------------- */
/* Reverse-mode gradient, over a window of N merged steps (Sec. 2.1) without
 * collisions or weight splits, of the smooth ion-flux objective
 *   J = sum_{n < N} sum_{live ions p after step n} (q_i dt / delta) w_p (-v_z,p) exp(-z_p / delta),
 * with respect to the electrode voltage parameters V_dc and V_rf and to the
 * weights the particles have when the window starts.  The gradient is that of
 * the exactly solved field equation: the context must run converged solves
 * (mg_fixed_cycles = 0; the adjoint solves use the same multigrid to `tol`),
 * FP64, averaged face permittivities (chi_face = RZPIC_FACE_AVG),
 * resize_every = 0, and both species bound with mc_model = RZPIC_MC_NONE.
 * Particles absorbed in the window contribute up to their absorption; the
 * set of absorbed particles is held fixed (the objective is not
 * differentiable where a particle meets a wall).  Memory: ceil(N/K) + 1
 * checkpoints and K per-step copies of both species' arrays (sized by their
 * capacities), 8 doubles per identity of each species, and grids. */
typedef struct rzpic_adjoint_config {
    int32_t n_steps;          /* N >= 1                                        */
    int32_t checkpoint_every; /* K: state kept every K steps (0 -> 10)         */
    int64_t id_capacity[2];   /* identities of species s lie in [0, id_capacity[s]) */
    double delta;             /* objective layer thickness, m (0 -> 2 hz)      */
    double tol;               /* adjoint solves' relative residual (0 -> mg_tol) */
    int32_t max_cycles;       /* cap on their V-cycles (0 -> mg_max_cycles)    */
    int32_t reserved;
} rzpic_adjoint_config;
typedef struct rzpic_adjoint rzpic_adjoint;
/* Allocate the window's workspace for `ctx` (which must outlive it). */
rzpic_status rzpic_adjoint_create(rzpic_ctx *ctx, const rzpic_adjoint_config *cfg,
                                  rzpic_adjoint **out);
/* Run steps step0 .. step0+N-1 on the context (as rzpic_step), keeping the
 * checkpoints; *J (host) receives the objective.  Synchronises. */
rzpic_status rzpic_adjoint_forward(rzpic_adjoint *adj, int64_t step0, double *J);
/* Gradient of the last forward window: grad_V (host) = {dJ/dV_dc, dJ/dV_rf};
 * grad_w0 / grad_w1 (device, id_capacity[s] doubles, may be NULL) receive
 * dJ/dw by particle identity (0 for identities not present); grad_density
 * (device, nz*nr doubles, may be NULL) the gradient with respect to a
 * relative perturbation psi of the initial density field on the nodes, the
 * weights of both species at the window start becoming
 * w_p (1 + sum_k S_k(x_p) psi_k) with the Sec. 2.4 weights S_k at the
 * particle's position: sum_p (dJ/dw_p) w_p S_k(x_p).  Recomputes the
 * window segment by segment and leaves the context in its state at the end
 * of the window.  EINVAL if a particle identity is >= id_capacity.
 * Synchronises. */
rzpic_status rzpic_adjoint_backward(rzpic_adjoint *adj, double grad_V[2], double *grad_w0,
                                    double *grad_w1, double *grad_density);
rzpic_status rzpic_adjoint_destroy(rzpic_adjoint *adj);

/* --- deposit without allocation ------------------------------------------ */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * deposit N_ij of Sec. 2.4 of one species' particles into the caller's grid,
 * with the fixed-point arithmetic of rzpic_deposit: the counts equal, bit for
 * bit, the N0/N1 grid rzpic_grid_copy returns after rzpic_deposit of the same
 * particles and quantum.  Nothing is allocated: the accumulators are a fixed
 * device array of 2^20 nodes inside the library (8 MiB on each device it
 * runs on, kept until the process ends); nr * nz above 2^20 is EINVAL.  Every
 * call on a device shares that array, so calls that overlap on one device
 * (other streams, other host threads) race; calls on one stream are ordered.
 * Asynchronous on `stream` (a hipStream_t, NULL = default stream); the
 * current device is the one used. */
typedef struct rzpic_deposit_args {
    int32_t nr, nz;           /* mesh nodes, nr >= 3, nz >= 2                 */
    double R, L;              /* radius and electrode gap (m)                 */
    int32_t precision;        /* RZPIC_FP64: r, z, w are double; RZPIC_MIXED:
                               * float, contributions formed in FP32 as the
                               * mixed form does                              */
    int32_t weighting;        /* RZPIC_W_ZR2 or RZPIC_W_ZR                    */
    int32_t fixed_point_bits; /* quantum = w_ref 2^-bits (0 -> 46 in FP64, 26 in
                               * MIXED; at most 52 / 30)                      */
    int32_t reserved;
    double w_ref;             /* reference weight of the quantum (> 0)        */
    const void *r, *z, *w;    /* device arrays of the n particles, inside the
                               * mesh (positions in m, weights)               */
    int64_t n;                /* particle count, 0 .. 2^29 - 64               */
    double *out;              /* device, nz*nr doubles [nz][nr]: N_ij in
                               * physical particles                           */
    int32_t *status;          /* device int32: 2 (the fixed-point overflow bit)
                               * is ORed in on overflow; the caller clears it */
} rzpic_deposit_args;
rzpic_status rzpic_deposit_noalloc(const rzpic_deposit_args *a, void *stream);

#ifdef __cplusplus
}
#endif
#endif
