/*
 * rzo.h -- plain FP64 CPU oracle of the implicit r-z PIC/MC hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the package smoke check and the CPU-baseline leg of the benchmark may load
 * it; the product path never calls into it.  It shares no source, header,
 * table or constant with the GPU library.
 *
 * Method: Wang, Jiang & Wang, "Implicit and electrostatic particle-in-cell /
 * Monte Carlo model in two-dimensional and axisymmetric geometry I" (arXiv
 * 1001.2969).  Section numbers below refer to that paper.
 *
 * Conventions
 *   mesh      nr nodes in r (r_j = j*hr, hr = R/(nr-1)) and nz nodes in z
 *             (z_i = i*hz, hz = L/(nz-1)); nz-1 must be a power of two >= 2.
 *   grids     row-major [nz][nr] doubles, index i*nr + j.
 *   species   0 = electrons, 1 = positive ions (the paper's argon case).
 *   units     SI; energies handed to the cross-section tables are in eV.
 * Every function returns 0 on success and a negative value on bad input.
 */
#ifndef RZO_H
#define RZO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rzo rzo;

/* Weighting schemes of Sec. 2.4. */
enum { RZO_W_ZR2 = 0, RZO_W_ZR = 1 };
/* Half-point susceptibility rules of Sec. 2.5. */
enum { RZO_FACE_AVG = 0, RZO_FACE_MAX = 1 };
/* Monte Carlo target models of Sec. 2.6. */
enum { RZO_MC_NONE = 0, RZO_MC_ELECTRON = 1, RZO_MC_ION = 2 };
/* Collision process kinds. */
enum { RZO_P_ELASTIC = 0, RZO_P_EXCITATION = 1, RZO_P_IONIZATION = 2 };
/* Grid selectors for rzo_get_grid / rzo_set_grid. */
enum {
    RZO_G_PHI = 0, RZO_G_RHO = 1, RZO_G_CHI = 2, RZO_G_ER = 3, RZO_G_EZ = 4,
    RZO_G_N0 = 5, RZO_G_N1 = 6,      /* deposited physical-particle counts N_ij */
    RZO_G_DENS0 = 7, RZO_G_DENS1 = 8,/* number densities n_ij = N_ij / V_ij   */
    RZO_G_VOL = 9,                   /* weighting volumes V_ij                 */
    RZO_G_PHI_P = 10, RZO_G_PHI_L = 11 /* external circuit: the two superposed solutions */
};
/* Per-particle Monte Carlo event codes (rzo_get_events). */
enum { RZO_EV_NONE = 0, RZO_EV_NULL = 1, RZO_EV_PROC0 = 2 };

typedef struct {
    int32_t nr, nz;
    double R, L, dt;
    int32_t weighting;       /* RZO_W_*                                     */
    int32_t chi_face;        /* RZO_FACE_*                                  */
    double V_dc, V_rf, f_rf; /* electrode z=0 potential V_dc+V_rf sin(2 pi f t) */
    uint64_t seed;           /* Philox key                                  */
    double mg_tol;           /* relative L-inf residual target              */
    int32_t mg_max_cycles;   /* cap on V-cycles per solve                   */
    int32_t mg_fixed_cycles; /* >0: exactly this many cycles, no test       */
    int32_t resize_every;    /* weight split period in steps (0 = never)    */
    int32_t sort_every;      /* tile sort period in steps (0 = never)       */
    double resize_wcoef;     /* w_r(r) = resize_wcoef * max(r, hr/2)        */
    double n_gas, T_gas, m_gas; /* background neutral density, K, kg        */
    int32_t tile_z, tile_r;  /* tile of the sort key, in cells              */
    double circuit_C;        /* >0: blocking capacitor (F) between the source
                              * V_dc+V_rf sin(2 pi f t) and the z=0 electrode  */
    int32_t ion_subcycle;    /* K >= 2: ions (species 1) move every K-th step
                              * with dt_i = K dt; 0 or 1: every step         */
    int32_t push_form;       /* RZO_PUSH_LOCAL (Sec. 2.3 local X-Y push, a_theta
                              * dropped) or RZO_PUSH_XYZ (the global X-Y-Z push) */
    int32_t resize_mode;     /* RZO_RESIZE_SPLIT (weight-conserving split) or
                              * RZO_RESIZE_ZERO_ORDER (particle-based, Sec. 2.2) */
    int32_t damping;         /* RZO_DAMP_D1 (Sec. 2.1) or RZO_DAMP_FRIEDMAN       */
    double theta;            /* RZO_DAMP_FRIEDMAN: damping parameter in [0, 1]  */
} rzo_config;
enum { RZO_PUSH_LOCAL = 0, RZO_PUSH_XYZ = 1 };
/* Time-averaged acceleration of the implicit push.  D1 (Sec. 2.1):
 * abar_n = (a_{n+1} + abar_{n-1}) / 2.  FRIEDMAN, the adjustable damping of
 * A. Friedman, J. Comput. Phys. 90 (1990) 292, as read here:
 *   abar_n = (theta/2) a_{n+1}
 *          + (1 - theta/2) [(1 - theta/2) a_n + (theta/2) abar_{n-1}],
 * leapfrog for theta = 0, the implicit coefficient of a_{n+1} (and with it
 * chi) theta/2 instead of 1/2.  The particle then carries the known part
 * B = abar_n - (theta/2) a_{n+1} in place of abar (ar, az), a_n being the
 * acceleration of the final push that ends step n-1.  Local push only. */
enum { RZO_DAMP_D1 = 0, RZO_DAMP_FRIEDMAN = 1 };
enum { RZO_RESIZE_SPLIT = 0, RZO_RESIZE_ZERO_ORDER = 1 };

rzo *rzo_create(const rzo_config *cfg);
void rzo_destroy(rzo *o);

/* Physical constants used by the oracle: e, m_e, amu, eps0, k_B, 2*pi. */
void rzo_constants(double out[6]);

/* Species setup: charge, mass, Monte Carlo model (RZO_MC_*). */
int rzo_set_species(rzo *o, int s, double q, double m, int mc_model);
/* Replace the particle list of species s (copies the arrays). */
int rzo_set_particles(rzo *o, int s, int64_t n, const double *r, const double *z,
                      const double *vr, const double *vt, const double *vz,
                      const double *ar, const double *az, const double *w,
                      const uint64_t *id, uint64_t next_id);
int64_t rzo_count(const rzo *o, int s);
uint64_t rzo_next_id(const rzo *o, int s);
/* Azimuthal damped acceleration a_theta (kept by RZO_PUSH_XYZ only; zero after
 * rzo_set_particles): set / read the first n entries. */
int rzo_set_at(rzo *o, int s, int64_t n, const double *at);
int rzo_get_at(const rzo *o, int s, double *at);
int rzo_get_particles(const rzo *o, int s, double *r, double *z, double *vr,
                      double *vt, double *vz, double *ar, double *az, double *w,
                      uint64_t *id);
/* Per-particle MC event codes of the last collision pass (length count at
 * that pass, in the array order the pass saw). */
int rzo_get_events(const rzo *o, int s, uint8_t *ev, int64_t n);

/* Cross sections on a uniform energy grid eps_k = k*de (eV), k < ne; sigma is
 * [nproc][ne] in m^2; thr in eV; ej_B is the Opal ejected-energy constant. */
int rzo_set_xsec(rzo *o, int s, int nproc, const int32_t *kind, const double *thr,
                 double de, int32_t ne, const double *sigma, double ej_B);
int rzo_mc_consts(const rzo *o, int s, double *nu_max, double *p_null);

/* Sec. 2.3 initialisation: n particles, r and z uniform, w proportional to r,
 * Maxwellian velocities at T_eV, zero accelerations, ids id0.. */
int rzo_init_particles(rzo *o, int s, int64_t n, double n0, double T_eV, uint64_t id0);

/* Individual operations (Sec. 2.1 cycle). */
int rzo_push_first(rzo *o, int s);          /* first push + rotation + absorb   */
int rzo_deposit(rzo *o);                    /* N_ij from scratch, then n, rho, chi */
int rzo_solve(rzo *o, double t, int32_t *cycles, double *relres);
int rzo_efield(rzo *o);
int rzo_push_final(rzo *o, int s);          /* gather + final push + axis + absorb */
int rzo_collide(rzo *o, int s, int64_t step);
int rzo_compact(rzo *o, int s);
int rzo_resize(rzo *o, int s);
/* The resize of step `step` (the zero-order draws are keyed by it;
 * rzo_resize uses step 0). */
int rzo_resize_step(rzo *o, int s, int64_t step);
/* Stable counting sort of species s by the tile (tile_z x tile_r cells) of
 * each particle's cell; returns the number of tiles. */
int rzo_sort(rzo *o, int s);
/* Tile key of a position (the key rzo_sort orders by). */
int32_t rzo_tile_key(const rzo *o, double r, double z);
/* Whole step n (finalize, solve at t=(n+1)dt, E, particles, compact, resize).
 * merged!=0: one pass per species; merged==0: one pass per operation. */
int rzo_step(rzo *o, int64_t n, int merged);
/* Prologue after init: first push, deposit, compact (Sec. 2.1 with a=0). */
int rzo_prologue(rzo *o);

/* Grid access. */
int rzo_get_grid(const rzo *o, int which, double *out);
int rzo_set_grid(rzo *o, int which, const double *in);
/* Absorbed physical-particle weight of species s at z=0, z=L, r=R. */
int rzo_absorbed(const rzo *o, int s, double out[3]);
/* External circuit state (circuit_C > 0): set {V, Q, Q_c}; read
 * {V, Q, Q_c, Q_conv, Q_P, Q_L} of the last solve. */
int rzo_set_circuit(rzo *o, double V, double Q, double Qc);
int rzo_circuit(const rzo *o, double out[6]);

/* Pieces exposed for pinning. */
/* y = A u on the finest level (interior nodes; boundary entries of y = 0). */
int rzo_apply_op(const rzo *o, const double *u, double *y);
/* Tridiagonal solve  -d_j x_{j-1} + b_j x_j - e_j x_{j+1} = g_j. */
int rzo_thomas(int32_t n, const double *d, const double *b, const double *e,
               const double *g, double *x);
/* Philox4x32-10 block. */
void rzo_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* The two uniforms of draw block `blk` for (species, id, step). */
void rzo_uniform_pair(uint64_t seed, int s, uint64_t id, uint32_t step, uint32_t blk,
                      double out[2]);
/* Cross section of process k of species s at energy eps (eV). */
double rzo_xsec(const rzo *o, int s, int k, double eps);

#ifdef __cplusplus
}
#endif
#endif
