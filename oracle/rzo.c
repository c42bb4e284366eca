/*
 * rzo.c -- plain FP64 CPU oracle of the implicit r-z PIC/MC hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the GPU library.  Every routine follows the paper (Wang, Jiang &
 * Wang, arXiv 1001.2969) step by step in straight loops; the places where the
 * paper is silent carry the reading used, stated in the comment.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared rzo.c -lm
 * (-ffp-contract=off keeps every product and sum rounded separately, so the
 * order of operations written here is the order evaluated.)
 */
#include "rzo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 values, SI. */
#define Q_E 1.602176634e-19
#define M_EL 9.1093837015e-31
#define AMU 1.66053906660e-27
#define EPS0 8.8541878128e-12
#define K_B 1.380649e-23
#define TWO_PI 6.283185307179586
#define PI_ 3.141592653589793

#define MAXLEV 24
#define MAXPROC 4

typedef struct {
    double q, m;
    int mc_model;
    int64_t n;      /* particles in the array proper                        */
    int64_t npend;  /* children created this step, stored at [n, n+npend)  */
    int64_t cap;
    double *r, *z, *vr, *vt, *vz, *ar, *az, *w;
    double *at;     /* a_theta of the global X-Y-Z push (zero otherwise)    */
    uint64_t *id;
    unsigned char *dead;
    uint8_t *ev;
    int64_t nev;
    uint64_t next_id;
    int nproc;
    int kind[MAXPROC];
    double thr[MAXPROC];
    double de;
    int ne;
    double *sigma;
    double ejB;
    double nu_max, p_null;
    double absorbed[3];
} species;

struct rzo {
    rzo_config c;
    double hr, hz;
    int nn;
    int L;                       /* multigrid levels 1..L, level L is the mesh */
    int nzl[MAXLEV + 1];
    double hzl[MAXLEV + 1];
    double *eps_l[MAXLEV + 1];   /* epsilon = 1 + chi on each level           */
    double *u_l[MAXLEV + 1];     /* level L uses phi                          */
    double *f_l[MAXLEV + 1];     /* level L right-hand side rho/eps0          */
    double *res;                 /* residual scratch (finest size)            */
    double *phi, *rho, *chi, *er, *ez, *vol;
    double *N[2], *dens[2];
    double *ld, *lb, *le, *lg, *lx, *lcp, *lgp; /* line-solve scratch          */
    species sp[2];
    /* external circuit: the charge solution with the electrode at 0 V, the
     * Laplace solution with it at 1 V, a zero right-hand side, and the state */
    double *phiP, *phiL, *zero;
    double cV, cQ, cQc, cQconv, cQp, cQl;
    double absorbed_prev[2];     /* weight absorbed at z=0 by the last solve   */
};

void rzo_constants(double out[6])
{
    out[0] = Q_E;
    out[1] = M_EL;
    out[2] = AMU;
    out[3] = EPS0;
    out[4] = K_B;
    out[5] = TWO_PI;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the */
/* published multipliers, the key bumped by the published Weyl constants.   */

void rzo_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Counter layout: (id lo, id hi, step, species<<16 | block); key = seed.
 * Each 32-bit pair becomes a 52-bit integer u and U = (u + 1/2) 2^-52, which
 * lies strictly inside (0,1) and is computed exactly in FP64. */
void rzo_uniform_pair(uint64_t seed, int s, uint64_t id, uint32_t step, uint32_t blk,
                      double out[2])
{
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step,
                       ((uint32_t)s << 16) | (blk & 0xFFFFu)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    rzo_philox(ctr, key, x);
    uint64_t ua = ((uint64_t)x[0] << 20) | (uint64_t)(x[1] >> 12);
    uint64_t ub = ((uint64_t)x[2] << 20) | (uint64_t)(x[3] >> 12);
    out[0] = ((double)ua + 0.5) * 0x1p-52;
    out[1] = ((double)ub + 0.5) * 0x1p-52;
}

/* Box-Muller: two standard normals from one uniform pair. */
static void normal_pair(const double u[2], double out[2])
{
    double rad = sqrt(-2.0 * log(u[0]));
    out[0] = rad * cos(TWO_PI * u[1]);
    out[1] = rad * sin(TWO_PI * u[1]);
}

/* ------------------------------------------------------------------------ */
/* Setup                                                                    */

static int ispow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

/* Time step of a species: ions take K dt when they are subcycled every K
 * steps (Sec. 2.7, the subcycling of Vahedi et al.), electrons dt. */
static int ion_K(const rzo *o) { return o->c.ion_subcycle > 1 ? o->c.ion_subcycle : 1; }

static double dt_of(const rzo *o, const species *sp)
{
    return sp == &o->sp[1] ? (double)ion_K(o) * o->c.dt : o->c.dt;
}

/* Whether the ions move in step n: every K-th step, n = K-1, 2K-1, ... */
static int ion_step(const rzo *o, int64_t n) { return n % ion_K(o) == ion_K(o) - 1; }


rzo *rzo_create(const rzo_config *cfg)
{
    if (!cfg || cfg->nr < 3 || cfg->nz < 3 || !ispow2(cfg->nz - 1) || !(cfg->R > 0) ||
        !(cfg->L > 0) || !(cfg->dt > 0))
        return NULL;
    if (cfg->sort_every < 0 || (cfg->sort_every > 0 && (cfg->tile_z < 1 || cfg->tile_r < 1)))
        return NULL;
    if (!(cfg->circuit_C >= 0.0)) return NULL;
    if (cfg->damping != RZO_DAMP_D1 && cfg->damping != RZO_DAMP_FRIEDMAN) return NULL;
    if (cfg->damping == RZO_DAMP_FRIEDMAN &&
        (cfg->push_form != RZO_PUSH_LOCAL || !(cfg->theta >= 0.0 && cfg->theta <= 1.0)))
        return NULL;
    rzo *o = (rzo *)calloc(1, sizeof(rzo));
    if (!o) return NULL;
    o->c = *cfg;
    o->hr = cfg->R / (double)(cfg->nr - 1);
    o->hz = cfg->L / (double)(cfg->nz - 1);
    o->nn = cfg->nr * cfg->nz;
    int L = 0;
    while ((1 << L) < cfg->nz - 1) ++L;
    o->L = L;
    for (int l = 1; l <= L; ++l) {
        o->nzl[l] = (1 << l) + 1;
        o->hzl[l] = o->hz * (double)(1 << (L - l));
        size_t sz = (size_t)o->nzl[l] * cfg->nr;
        o->eps_l[l] = (double *)calloc(sz, sizeof(double));
        o->f_l[l] = (double *)calloc(sz, sizeof(double));
        if (l < L) o->u_l[l] = (double *)calloc(sz, sizeof(double));
    }
    size_t nn = (size_t)o->nn;
    o->res = (double *)calloc(nn, sizeof(double));
    o->phi = (double *)calloc(nn, sizeof(double));
    o->u_l[L] = o->phi; /* the finest level iterates on phi itself */
    o->rho = (double *)calloc(nn, sizeof(double));
    o->chi = (double *)calloc(nn, sizeof(double));
    o->er = (double *)calloc(nn, sizeof(double));
    o->ez = (double *)calloc(nn, sizeof(double));
    o->vol = (double *)calloc(nn, sizeof(double));
    for (int s = 0; s < 2; ++s) {
        o->N[s] = (double *)calloc(nn, sizeof(double));
        o->dens[s] = (double *)calloc(nn, sizeof(double));
    }
    size_t nr = (size_t)cfg->nr;
    o->ld = (double *)calloc(nr, sizeof(double));
    o->lb = (double *)calloc(nr, sizeof(double));
    o->le = (double *)calloc(nr, sizeof(double));
    o->lg = (double *)calloc(nr, sizeof(double));
    o->lx = (double *)calloc(nr, sizeof(double));
    o->lcp = (double *)calloc(nr, sizeof(double));
    o->lgp = (double *)calloc(nr, sizeof(double));
    if (cfg->circuit_C > 0.0) {
        o->phiP = (double *)calloc(nn, sizeof(double));
        o->phiL = (double *)calloc(nn, sizeof(double));
        o->zero = (double *)calloc(nn, sizeof(double));
    }

    /* Weighting volumes of Sec. 2.4.  Radial factor: the paper's V_j with the
     * outer neighbour clamped to the wall node at j = nr-1 (only the inner
     * half-cell exists there) and the inner one clamped to the axis at j = 0,
     * which reproduces its V_0.  Axial factor: hz inside, hz/2 on the two
     * electrode rows (only one half-cell lies inside the gap). */
    for (int i = 0; i < cfg->nz; ++i) {
        double zf = (i == 0 || i == cfg->nz - 1) ? 0.5 * o->hz : o->hz;
        for (int j = 0; j < cfg->nr; ++j) {
            int jp = j + 1 < cfg->nr ? j + 1 : cfg->nr - 1;
            int jm = j - 1 >= 0 ? j - 1 : 0;
            double rj = (double)j * o->hr, rp = (double)jp * o->hr, rm = (double)jm * o->hr;
            double rf;
            if (cfg->weighting == RZO_W_ZR)
                rf = (PI_ / 3.0) * (rp * (rj + rp) - rm * (rj + rm));
            else
                rf = 0.5 * PI_ * (rp * rp - rm * rm);
            o->vol[(size_t)i * cfg->nr + j] = rf * zf;
        }
    }
    return o;
}

static void free_species(species *sp)
{
    free(sp->r); free(sp->z); free(sp->vr); free(sp->vt); free(sp->vz);
    free(sp->ar); free(sp->az); free(sp->w); free(sp->id); free(sp->dead); free(sp->at);
    free(sp->ev); free(sp->sigma);
}

void rzo_destroy(rzo *o)
{
    if (!o) return;
    for (int l = 1; l <= o->L; ++l) {
        free(o->eps_l[l]); free(o->f_l[l]);
        if (l < o->L) free(o->u_l[l]);
    }
    free(o->res); free(o->phi); free(o->rho); free(o->chi); free(o->er); free(o->ez);
    free(o->vol);
    for (int s = 0; s < 2; ++s) { free(o->N[s]); free(o->dens[s]); free_species(&o->sp[s]); }
    free(o->ld); free(o->lb); free(o->le); free(o->lg); free(o->lx); free(o->lcp);
    free(o->lgp);
    free(o->phiP); free(o->phiL); free(o->zero);
    free(o);
}

/* memcpy/memset of particle arrays that may be empty (and then unallocated):
 * a zero-length call with a null pointer is undefined in C, so skip it. */
static void copy_bytes(void *dst, const void *src, size_t n)
{
    if (n) memcpy(dst, src, n);
}

static void zero_bytes(void *dst, size_t n)
{
    if (n) memset(dst, 0, n);
}

static int grow(species *sp, int64_t need)
{
    if (need <= sp->cap) return 0;
    int64_t cap = sp->cap > 0 ? sp->cap : 1024;
    while (cap < need) cap *= 2;
#define RE(p, T)                                                    \
    do {                                                            \
        void *q_ = realloc((p), (size_t)cap * sizeof(T));           \
        if (!q_) return -1;                                         \
        (p) = (T *)q_;                                              \
    } while (0)
    RE(sp->r, double); RE(sp->z, double); RE(sp->vr, double); RE(sp->vt, double);
    RE(sp->vz, double); RE(sp->ar, double); RE(sp->az, double); RE(sp->w, double);
    RE(sp->at, double);
    RE(sp->id, uint64_t); RE(sp->dead, unsigned char);
#undef RE
    sp->cap = cap;
    return 0;
}

int rzo_set_species(rzo *o, int s, double q, double m, int mc_model)
{
    if (!o || s < 0 || s > 1 || !(m > 0)) return -1;
    o->sp[s].q = q;
    o->sp[s].m = m;
    o->sp[s].mc_model = mc_model;
    return 0;
}

int rzo_set_particles(rzo *o, int s, int64_t n, const double *r, const double *z,
                      const double *vr, const double *vt, const double *vz,
                      const double *ar, const double *az, const double *w,
                      const uint64_t *id, uint64_t next_id)
{
    if (!o || s < 0 || s > 1 || n < 0) return -1;
    species *sp = &o->sp[s];
    if (grow(sp, n) != 0) return -2;
    size_t b = (size_t)n * sizeof(double);
    copy_bytes(sp->r, r, b); copy_bytes(sp->z, z, b); copy_bytes(sp->vr, vr, b);
    copy_bytes(sp->vt, vt, b); copy_bytes(sp->vz, vz, b); copy_bytes(sp->ar, ar, b);
    copy_bytes(sp->az, az, b); copy_bytes(sp->w, w, b);
    zero_bytes(sp->at, b);
    copy_bytes(sp->id, id, (size_t)n * sizeof(uint64_t));
    zero_bytes(sp->dead, (size_t)n);
    sp->n = n;
    sp->npend = 0;
    sp->next_id = next_id;
    return 0;
}

int rzo_set_at(rzo *o, int s, int64_t n, const double *at)
{
    if (!o || s < 0 || s > 1 || n < 0 || n > o->sp[s].n) return -1;
    copy_bytes(o->sp[s].at, at, (size_t)n * sizeof(double));
    return 0;
}

int rzo_get_at(const rzo *o, int s, double *at)
{
    if (!o || s < 0 || s > 1) return -1;
    copy_bytes(at, o->sp[s].at, (size_t)o->sp[s].n * sizeof(double));
    return 0;
}

int64_t rzo_count(const rzo *o, int s) { return o->sp[s].n + o->sp[s].npend; }
uint64_t rzo_next_id(const rzo *o, int s) { return o->sp[s].next_id; }

int rzo_get_particles(const rzo *o, int s, double *r, double *z, double *vr,
                      double *vt, double *vz, double *ar, double *az, double *w,
                      uint64_t *id)
{
    const species *sp = &o->sp[s];
    size_t n = (size_t)(sp->n + sp->npend);
    size_t b = n * sizeof(double);
    copy_bytes(r, sp->r, b); copy_bytes(z, sp->z, b); copy_bytes(vr, sp->vr, b);
    copy_bytes(vt, sp->vt, b); copy_bytes(vz, sp->vz, b); copy_bytes(ar, sp->ar, b);
    copy_bytes(az, sp->az, b); copy_bytes(w, sp->w, b);
    copy_bytes(id, sp->id, n * sizeof(uint64_t));
    return 0;
}

int rzo_get_events(const rzo *o, int s, uint8_t *ev, int64_t n)
{
    const species *sp = &o->sp[s];
    if (n > sp->nev) return -1;
    copy_bytes(ev, sp->ev, (size_t)n);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cross sections (Sec. 2.6): linear interpolation on the tabulated grid and  */
/* the 1/E law above the last tabulated energy.                              */

static double xsec(const species *sp, int k, double eps)
{
    const double *sg = sp->sigma + (size_t)k * (size_t)sp->ne;
    double emax = (double)(sp->ne - 1) * sp->de;
    if (eps >= emax) return sg[sp->ne - 1] * (emax / eps);
    double x = eps / sp->de;
    int j = (int)x;
    if (j > sp->ne - 2) j = sp->ne - 2;
    double t = x - (double)j;
    return sg[j] + t * (sg[j + 1] - sg[j]);
}

double rzo_xsec(const rzo *o, int s, int k, double eps) { return xsec(&o->sp[s], k, eps); }

/* Reduced mass of the collision pair: the target is at rest for electrons,
 * a Maxwellian neutral for ions (Sec. 2.6). */
static double pair_mass(const rzo *o, const species *sp)
{
    if (sp->mc_model == RZO_MC_ION) return sp->m * o->c.m_gas / (sp->m + o->c.m_gas);
    return sp->m;
}

int rzo_set_xsec(rzo *o, int s, int nproc, const int32_t *kind, const double *thr,
                 double de, int32_t ne, const double *sigma, double ej_B)
{
    if (!o || s < 0 || s > 1 || nproc < 1 || nproc > MAXPROC || ne < 2 || !(de > 0))
        return -1;
    species *sp = &o->sp[s];
    free(sp->sigma);
    sp->sigma = (double *)malloc((size_t)nproc * (size_t)ne * sizeof(double));
    if (!sp->sigma) return -2;
    memcpy(sp->sigma, sigma, (size_t)nproc * (size_t)ne * sizeof(double));
    sp->nproc = nproc;
    for (int k = 0; k < nproc; ++k) {
        sp->kind[k] = kind[k];
        sp->thr[k] = thr[k];
    }
    sp->de = de;
    sp->ne = ne;
    sp->ejB = ej_B;
    /* Null-collision frequency: an upper bound of n_g sigma_T(eps) g(eps) over
     * every energy.  On [eps_j, eps_j+1] the interpolated sigma_T is at most the
     * larger end value and the pair speed g at most g(eps_j+1); above the table
     * sigma_T g falls as eps^-1/2, so the last interval bounds the tail. */
    double mu = pair_mass(o, sp);
    double numax = 0.0;
    for (int j = 0; j + 1 < ne; ++j) {
        double s0 = 0.0, s1 = 0.0;
        for (int k = 0; k < nproc; ++k) {
            s0 += sigma[(size_t)k * ne + j];
            s1 += sigma[(size_t)k * ne + j + 1];
        }
        double smax = s0 > s1 ? s0 : s1;
        double e1 = (double)(j + 1) * de;
        double g = sqrt(2.0 * e1 * Q_E / mu);
        double nu = o->c.n_gas * smax * g;
        if (nu > numax) numax = nu;
    }
    sp->nu_max = numax;
    sp->p_null = -expm1(-numax * dt_of(o, sp));
    return 0;
}

int rzo_mc_consts(const rzo *o, int s, double *nu_max, double *p_null)
{
    *nu_max = o->sp[s].nu_max;
    *p_null = o->sp[s].p_null;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Particle <-> grid weights (Sec. 2.4).                                     */

typedef struct {
    int i, j;
    double sz0, sz1, sr0, sr1;
} wts;

static wts weights(const rzo *o, double r, double z)
{
    wts q;
    int nr = o->c.nr, nz = o->c.nz;
    int i = (int)(z / o->hz);
    int j = (int)(r / o->hr);
    if (i < 0) i = 0;
    if (i > nz - 2) i = nz - 2;
    if (j < 0) j = 0;
    if (j > nr - 2) j = nr - 2;
    double zi = (double)i * o->hz, zi1 = (double)(i + 1) * o->hz;
    double rj = (double)j * o->hr, rj1 = (double)(j + 1) * o->hr;
    q.i = i;
    q.j = j;
    q.sz0 = (zi1 - z) / o->hz;
    q.sz1 = (z - zi) / o->hz;
    if (o->c.weighting == RZO_W_ZR) {
        q.sr0 = (rj1 - r) / o->hr;
        q.sr1 = (r - rj) / o->hr;
    } else {
        double den = rj1 * rj1 - rj * rj;
        q.sr0 = (rj1 * rj1 - r * r) / den;
        q.sr1 = (r * r - rj * rj) / den;
    }
    return q;
}

static void deposit_one(rzo *o, int s, int64_t p)
{
    species *sp = &o->sp[s];
    wts q = weights(o, sp->r[p], sp->z[p]);
    double w = sp->w[p];
    size_t nr = (size_t)o->c.nr;
    size_t g = (size_t)q.i * nr + (size_t)q.j;
    double *N = o->N[s];
    N[g] += w * q.sz0 * q.sr0;
    N[g + 1] += w * q.sz0 * q.sr1;
    N[g + nr] += w * q.sz1 * q.sr0;
    N[g + nr + 1] += w * q.sz1 * q.sr1;
}

static void gather(const rzo *o, double r, double z, double *Er, double *Ez)
{
    wts q = weights(o, r, z);
    size_t nr = (size_t)o->c.nr;
    size_t g = (size_t)q.i * nr + (size_t)q.j;
    *Er = q.sz0 * q.sr0 * o->er[g] + q.sz0 * q.sr1 * o->er[g + 1] +
          q.sz1 * q.sr0 * o->er[g + nr] + q.sz1 * q.sr1 * o->er[g + nr + 1];
    *Ez = q.sz0 * q.sr0 * o->ez[g] + q.sz0 * q.sr1 * o->ez[g + 1] +
          q.sz1 * q.sr0 * o->ez[g + nr] + q.sz1 * q.sr1 * o->ez[g + nr + 1];
}

static void deposit_all(rzo *o)
{
    for (int s = 0; s < 2; ++s) {
        memset(o->N[s], 0, (size_t)o->nn * sizeof(double));
        species *sp = &o->sp[s];
        for (int64_t p = 0; p < sp->n + sp->npend; ++p)
            if (!sp->dead[p]) deposit_one(o, s, p);
    }
}

/* n = N/V, rho = sum q n, chi = sum q^2 n dt_s^2 / (2 m eps0): the
 * susceptibility of Sec. 2.1 written in SI units (one half of (omega_p dt_s)^2
 * per species, dt_s its time step).  `ions` = 0: the ions do not move in the
 * coming step, so they add charge but no susceptibility. */
static void finalize_ions(rzo *o, int ions)
{
    for (int g = 0; g < o->nn; ++g) {
        double rho = 0.0, chi = 0.0;
        for (int s = 0; s < 2; ++s) {
            double n = o->N[s][g] / o->vol[g];
            o->dens[s][g] = n;
            double q = o->sp[s].q, m = o->sp[s].m;
            double dt = dt_of(o, &o->sp[s]);
            rho += q * n;
            if (s == 0 || ions) {
                double x = q * q * n * dt * dt / (2.0 * m * EPS0);
                /* Friedman: implicit coefficient theta/2 instead of 1/2 */
                if (o->c.damping == RZO_DAMP_FRIEDMAN) x *= o->c.theta;
                chi += x;
            }
        }
        o->rho[g] = rho;
        o->chi[g] = chi;
    }
}

static void finalize(rzo *o) { finalize_ions(o, 1); }

int rzo_deposit(rzo *o)
{
    deposit_all(o);
    finalize(o);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Particle pushes (Sec. 2.1 D1 scheme, Sec. 2.3 local X-Y coordinates).    */

/* Absorption at the electrodes z<=0, z>=L and the wall r>=R (Sec. 2.3); the
 * removed weight is added to that boundary's tally.  Returns 1 if absorbed. */
static int absorb(rzo *o, species *sp, int64_t p)
{
    int b = -1;
    if (sp->z[p] <= 0.0) b = 0;
    else if (sp->z[p] >= o->c.L) b = 1;
    else if (sp->r[p] >= o->c.R) b = 2;
    if (b < 0) return 0;
    sp->dead[p] = 1;
    /* the OpenMP timing build (rzo_omp.c) pushes particles in parallel */
#ifdef _OPENMP
#pragma omp atomic
#endif
    sp->absorbed[b] += sp->w[p];
    return 1;
}

/* First push in the particle's local X-Y frame (X along r, Y along theta),
 * followed by the rotation onto the new radial direction.  a_theta is not
 * stored (the damping of a_theta is not accumulated), so v_y' = v_theta and
 * the rotated a_theta is dropped. */
static int first_push_one(rzo *o, species *sp, int64_t p)
{
    double dt = dt_of(o, sp);
    const int xyz = o->c.push_form == RZO_PUSH_XYZ;
    /* the known part of abar_n: abar_{n-1}/2 (D1), B (Friedman) */
    const double kn = o->c.damping == RZO_DAMP_FRIEDMAN ? 1.0 : 0.5;
    double vx = sp->vr[p] + kn * sp->ar[p] * dt;
    double vy = xyz ? sp->vt[p] + 0.5 * sp->at[p] * dt : sp->vt[p];
    double x = sp->r[p] + vx * dt;
    double y = vy * dt;
    double vz = sp->vz[p] + kn * sp->az[p] * dt;
    double z = sp->z[p] + vz * dt;
    double rn = sqrt(x * x + y * y);
    double c = 1.0, s = 0.0;
    if (rn > 0.0) {
        c = x / rn;
        s = y / rn;
    }
    sp->r[p] = rn;
    sp->z[p] = z;
    sp->vr[p] = vx * c + vy * s;
    sp->vt[p] = -vx * s + vy * c;
    sp->vz[p] = vz;
    if (xyz) {
        double ar = sp->ar[p], at = sp->at[p];
        sp->ar[p] = ar * c + at * s;
        sp->at[p] = -ar * s + at * c;
    } else {
        sp->ar[p] = sp->ar[p] * c;
    }
    return absorb(o, sp, p);
}

/* Final push in X-Y coordinates for i = r, z with E gathered at the first-
 * pushed position, the damped acceleration update, then the axis rule
 * (radial position, velocity and acceleration made positive) and absorption. */
static int final_push_one(rzo *o, species *sp, int64_t p)
{
    double dt = dt_of(o, sp);
    double qm = sp->q / sp->m;
    double Er, Ez;
    gather(o, sp->r[p], sp->z[p], &Er, &Ez);
    double aEr = qm * Er, aEz = qm * Ez;
    if (o->c.damping == RZO_DAMP_FRIEDMAN) {
        /* x += (theta/2) a dt^2, v += (theta/2) a dt; abar_n = (theta/2) a
         * + B; the next step's known part
         * B' = (1 - theta/2) ((1 - theta/2) a + (theta/2) abar_n) */
        const double c = 0.5 * o->c.theta, c1 = 1.0 - c;
        double r = sp->r[p] + c * aEr * dt * dt;
        double z = sp->z[p] + c * aEz * dt * dt;
        double vr = sp->vr[p] + c * aEr * dt;
        double vz = sp->vz[p] + c * aEz * dt;
        const double abr = c * aEr + sp->ar[p], abz = c * aEz + sp->az[p];
        double br = c1 * (c1 * aEr + c * abr);
        double bz = c1 * (c1 * aEz + c * abz);
        if (r < 0.0) { /* the axis rule of the D1 push */
            r = -r;
            vr = fabs(vr);
            br = fabs(br);
        }
        sp->r[p] = r;
        sp->z[p] = z;
        sp->vr[p] = vr;
        sp->vz[p] = vz;
        sp->ar[p] = br;
        sp->az[p] = bz;
        return absorb(o, sp, p);
    }
    double r = sp->r[p] + 0.5 * aEr * dt * dt;
    double z = sp->z[p] + 0.5 * aEz * dt * dt;
    double vr = sp->vr[p] + 0.5 * aEr * dt;
    double vz = sp->vz[p] + 0.5 * aEz * dt;
    double ar = 0.5 * (aEr + sp->ar[p]);
    double az = 0.5 * (aEz + sp->az[p]);
    if (o->c.push_form == RZO_PUSH_XYZ) {
        /* Cartesian final push: E has no theta component at the particle, so
         * a_theta is damped by the same average; a particle pushed through
         * the axis continues on the other side (the local frame turns by pi) */
        double at = 0.5 * sp->at[p];
        double vt = sp->vt[p];
        if (r < 0.0) {
            r = -r;
            vr = -vr;
            vt = -vt;
            ar = -ar;
            at = -at;
        }
        sp->vt[p] = vt;
        sp->at[p] = at;
    } else if (r < 0.0) {
        r = -r;
        vr = fabs(vr);
        ar = fabs(ar);
    }
    sp->r[p] = r;
    sp->z[p] = z;
    sp->vr[p] = vr;
    sp->vz[p] = vz;
    sp->ar[p] = ar;
    sp->az[p] = az;
    return absorb(o, sp, p);
}

int rzo_push_first(rzo *o, int s)
{
    species *sp = &o->sp[s];
    for (int64_t p = 0; p < sp->n + sp->npend; ++p)
        if (!sp->dead[p]) first_push_one(o, sp, p);
    return 0;
}

int rzo_push_final(rzo *o, int s)
{
    species *sp = &o->sp[s];
    for (int64_t p = 0; p < sp->n; ++p)
        if (!sp->dead[p]) final_push_one(o, sp, p);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Monte Carlo collisions (Sec. 2.6).                                       */

/* Turn the unit vector u by polar angle chi (cosine cx) and azimuth phi
 * about itself.  The azimuth is measured from p = (axis x u)/|axis x u| with
 * axis = z unless u is within ~8 degrees of z, then axis = x; q = u x p. */
static void turn(double u[3], double cx, double phi)
{
    double px, py, pz;
    if (fabs(u[2]) < 0.99) {
        px = -u[1];
        py = u[0];
        pz = 0.0;
    } else {
        px = 0.0;
        py = -u[2];
        pz = u[1];
    }
    double pn = sqrt(px * px + py * py + pz * pz);
    px /= pn;
    py /= pn;
    pz /= pn;
    double qx = u[1] * pz - u[2] * py;
    double qy = u[2] * px - u[0] * pz;
    double qz = u[0] * py - u[1] * px;
    double sx = sqrt(fmax(0.0, 1.0 - cx * cx));
    double cp = cos(phi), sp = sin(phi);
    double nx = cx * u[0] + sx * (cp * px + sp * qx);
    double ny = cx * u[1] + sx * (cp * py + sp * qy);
    double nz = cx * u[2] + sx * (cp * pz + sp * qz);
    u[0] = nx;
    u[1] = ny;
    u[2] = nz;
}

/* Electron scattering angle of Vahedi & Surendra (1995):
 * cos chi = (2 + eps - 2 (1+eps)^R) / eps, eps in eV. */
static double cos_chi_e(double eps, double R)
{
    if (!(eps > 0.0)) return 1.0 - 2.0 * R;
    double c = (2.0 + eps - 2.0 * pow(1.0 + eps, R)) / eps;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    return c;
}

static int64_t append(species *sp, double r, double z, double vr, double vt, double vz,
                      double ar, double az, double w, double at)
{
    int64_t k = sp->n + sp->npend;
    if (grow(sp, k + 1) != 0) return -1;
    sp->r[k] = r; sp->z[k] = z; sp->vr[k] = vr; sp->vt[k] = vt; sp->vz[k] = vz;
    sp->ar[k] = ar; sp->az[k] = az; sp->w[k] = w; sp->at[k] = at;
    sp->id[k] = sp->next_id++;
    sp->dead[k] = 0;
    sp->npend++;
    return k;
}

/* One particle's null-collision test and, when a real process is chosen, its
 * outcome.  Uniform pairs: block 0 = (candidate, process); electrons: block 1
 * = (chi, phi) of the scattered electron, block 2 = (ejected energy, chi of
 * the ejected electron), block 3 = (phi of the ejected electron, unused),
 * blocks 4-5 = normals of the new ion; ions: blocks 1-2 = target normals,
 * block 3 = (cos chi, phi) in the centre-of-mass frame. */
static uint8_t collide_one(rzo *o, int s, int64_t p, uint32_t step)
{
    species *sp = &o->sp[s];
    uint64_t seed = o->c.seed;
    uint64_t pid = sp->id[p];
    double u[2];
    rzo_uniform_pair(seed, s, pid, step, 0, u);
    if (!(u[0] < sp->p_null)) return RZO_EV_NONE;
    double thr_nu = u[1] * sp->nu_max;
    double v[3] = {sp->vr[p], sp->vt[p], sp->vz[p]};

    if (sp->mc_model == RZO_MC_ELECTRON) {
        double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        double eps = v2 * (0.5 * sp->m / Q_E);
        double vm = sqrt(v2);
        double cum = 0.0;
        int k = -1;
        for (int kk = 0; kk < sp->nproc; ++kk) {
            cum += o->c.n_gas * xsec(sp, kk, eps) * vm;
            if (thr_nu < cum) {
                k = kk;
                break;
            }
        }
        if (k < 0) return RZO_EV_NULL;
        double un[3];
        if (vm > 0.0) {
            un[0] = v[0] / vm;
            un[1] = v[1] / vm;
            un[2] = v[2] / vm;
        } else {
            un[0] = 0.0;
            un[1] = 0.0;
            un[2] = 1.0;
        }
        double ua[2];
        rzo_uniform_pair(seed, s, pid, step, 1, ua);
        int kind = sp->kind[k];
        if (kind == RZO_P_ELASTIC) {
            double cx = cos_chi_e(eps, ua[0]);
            double eps1 = eps * (1.0 - (2.0 * sp->m / o->c.m_gas) * (1.0 - cx));
            turn(un, cx, TWO_PI * ua[1]);
            double sp1 = sqrt(2.0 * eps1 * Q_E / sp->m);
            sp->vr[p] = sp1 * un[0];
            sp->vt[p] = sp1 * un[1];
            sp->vz[p] = sp1 * un[2];
            return (uint8_t)(RZO_EV_PROC0 + k);
        }
        double ex = eps - sp->thr[k];
        /* The interpolated table can be non-zero just below a threshold; such
         * a draw leaves the electron unchanged (treated as a null event). */
        if (ex < 0.0) return RZO_EV_NULL;
        if (kind == RZO_P_EXCITATION) {
            double cx = cos_chi_e(ex, ua[0]);
            turn(un, cx, TWO_PI * ua[1]);
            double sp1 = sqrt(2.0 * ex * Q_E / sp->m);
            sp->vr[p] = sp1 * un[0];
            sp->vt[p] = sp1 * un[1];
            sp->vz[p] = sp1 * un[2];
            return (uint8_t)(RZO_EV_PROC0 + k);
        }
        /* Ionization: the energy left above threshold is shared by the
         * ejected electron, B tan(R atan(ex / 2B)) (Opal et al.), and the
         * scattered one; each is turned by the angle law at its own energy. */
        double ub[2], uc[2], un1[2], un2[2];
        rzo_uniform_pair(seed, s, pid, step, 2, ub);
        rzo_uniform_pair(seed, s, pid, step, 3, uc);
        double B = sp->ejB;
        double eej = B * tan(ub[0] * atan(ex / (2.0 * B)));
        double esc = ex - eej;
        double us[3] = {un[0], un[1], un[2]};
        double ue[3] = {un[0], un[1], un[2]};
        turn(us, cos_chi_e(esc, ua[0]), TWO_PI * ua[1]);
        turn(ue, cos_chi_e(eej, ub[1]), TWO_PI * uc[0]);
        double vs = sqrt(2.0 * esc * Q_E / sp->m);
        double ve = sqrt(2.0 * eej * Q_E / sp->m);
        sp->vr[p] = vs * us[0];
        sp->vt[p] = vs * us[1];
        sp->vz[p] = vs * us[2];
        /* New electron and ion at the parent's position with the parent's
         * weight; the ion's damped acceleration is the parent's scaled by the
         * charge-to-mass ratios (Sec. 2.6), the electron's is the parent's. */
        species *ion = &o->sp[1];
        append(sp, sp->r[p], sp->z[p], ve * ue[0], ve * ue[1], ve * ue[2], sp->ar[p],
               sp->az[p], sp->w[p], sp->at[p]);
        rzo_uniform_pair(seed, s, pid, step, 4, un1);
        rzo_uniform_pair(seed, s, pid, step, 5, un2);
        double g1[2], g2[2];
        normal_pair(un1, g1);
        normal_pair(un2, g2);
        double vth = sqrt(K_B * o->c.T_gas / o->c.m_gas);
        double ratio = (ion->q * sp->m) / (sp->q * ion->m);
        append(ion, sp->r[p], sp->z[p], vth * g1[0], vth * g1[1], vth * g2[0],
               sp->ar[p] * ratio, sp->az[p] * ratio, sp->w[p], sp->at[p] * ratio);
        return (uint8_t)(RZO_EV_PROC0 + k);
    }

    if (sp->mc_model == RZO_MC_ION) {
        double u1[2], u2[2], g1[2], g2[2];
        rzo_uniform_pair(seed, s, pid, step, 1, u1);
        rzo_uniform_pair(seed, s, pid, step, 2, u2);
        normal_pair(u1, g1);
        normal_pair(u2, g2);
        double vth = sqrt(K_B * o->c.T_gas / o->c.m_gas);
        double vg[3] = {vth * g1[0], vth * g1[1], vth * g2[0]};
        double g[3] = {v[0] - vg[0], v[1] - vg[1], v[2] - vg[2]};
        double g2s = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        double mu = pair_mass(o, sp);
        double eps = g2s * (0.5 * mu / Q_E);
        double gm = sqrt(g2s);
        double cum = 0.0;
        int k = -1;
        for (int kk = 0; kk < sp->nproc; ++kk) {
            cum += o->c.n_gas * xsec(sp, kk, eps) * gm;
            if (thr_nu < cum) {
                k = kk;
                break;
            }
        }
        if (k < 0) return RZO_EV_NULL;
        /* Isotropic scattering in the centre-of-mass frame (elastic). */
        double ua[2];
        rzo_uniform_pair(seed, s, pid, step, 3, ua);
        double cx = 1.0 - 2.0 * ua[0];
        double sx = sqrt(fmax(0.0, 1.0 - cx * cx));
        double ph = TWO_PI * ua[1];
        double M = o->c.m_gas, m = sp->m;
        double fcm = M / (m + M);
        for (int d = 0; d < 3; ++d) {
            double vcm = (m * v[d] + M * vg[d]) / (m + M);
            double gd = d == 0 ? sx * cos(ph) : (d == 1 ? sx * sin(ph) : cx);
            v[d] = vcm + fcm * gm * gd;
        }
        sp->vr[p] = v[0];
        sp->vt[p] = v[1];
        sp->vz[p] = v[2];
        return (uint8_t)(RZO_EV_PROC0 + k);
    }
    return RZO_EV_NONE;
}

static int ensure_ev(species *sp)
{
    if (sp->nev < sp->n || !sp->ev) {
        free(sp->ev);
        sp->ev = (uint8_t *)calloc((size_t)(sp->n > 0 ? sp->n : 1), 1);
        if (!sp->ev) return -1;
    }
    sp->nev = sp->n;
    zero_bytes(sp->ev, (size_t)sp->n);
    return 0;
}

int rzo_collide(rzo *o, int s, int64_t step)
{
    species *sp = &o->sp[s];
    if (sp->mc_model == RZO_MC_NONE || sp->nproc == 0) return 0;
    if (ensure_ev(sp) != 0) return -2;
    int64_t n = sp->n;
    for (int64_t p = 0; p < n; ++p)
        if (!sp->dead[p]) sp->ev[p] = collide_one(o, s, p, (uint32_t)step);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* List maintenance.                                                         */

static void move_particle(species *sp, int64_t dst, int64_t src)
{
    sp->r[dst] = sp->r[src]; sp->z[dst] = sp->z[src]; sp->vr[dst] = sp->vr[src];
    sp->vt[dst] = sp->vt[src]; sp->vz[dst] = sp->vz[src]; sp->ar[dst] = sp->ar[src];
    sp->az[dst] = sp->az[src]; sp->w[dst] = sp->w[src]; sp->id[dst] = sp->id[src];
    sp->at[dst] = sp->at[src];
    sp->dead[dst] = sp->dead[src];
}

/* Removal of absorbed particles: with D dead among the n array particles, the
 * holes below n-D are filled, in increasing order, by the live particles of
 * [n-D, n) in increasing order; then the surviving children of this step are
 * appended in creation order. */
int rzo_compact(rzo *o, int s)
{
    species *sp = &o->sp[s];
    int64_t n = sp->n, D = 0;
    for (int64_t p = 0; p < n; ++p) D += sp->dead[p];
    int64_t keep = n - D;
    int64_t src = keep;
    for (int64_t h = 0; h < keep; ++h) {
        if (!sp->dead[h]) continue;
        while (sp->dead[src]) ++src;
        move_particle(sp, h, src);
        ++src;
    }
    int64_t dst = keep;
    for (int64_t c = n; c < n + sp->npend; ++c) {
        if (sp->dead[c]) continue;
        move_particle(sp, dst, c);
        ++dst;
    }
    sp->n = dst;
    sp->npend = 0;
    zero_bytes(sp->dead, (size_t)sp->n);
    return 0;
}

/* Weight split of Sec. 2.2: a particle heavier than w_r(r) is split into
 * N = floor(w/w_r) clones of weight w_r, the parent keeping w - N w_r; when
 * that remainder is not positive (w an exact multiple) one clone fewer is made
 * and the parent keeps w_r.  Clones copy the full phase-space record, take new
 * ids in parent order and are appended after the array. */
static int resize_split(rzo *o, int s)
{
    species *sp = &o->sp[s];
    double half = 0.5 * o->hr;
    int64_t n = sp->n;
    for (int64_t p = 0; p < n; ++p) {
        double rr = sp->r[p] > half ? sp->r[p] : half;
        double wr = o->c.resize_wcoef * rr;
        double w = sp->w[p];
        if (!(w > wr)) continue;
        double k = floor(w / wr);
        double rem = w - k * wr;
        int64_t nc = rem > 0.0 ? (int64_t)k : (int64_t)k - 1;
        if (nc <= 0) continue;
        sp->w[p] = w - (double)nc * wr;
        for (int64_t c = 0; c < nc; ++c)
            if (append(sp, sp->r[p], sp->z[p], sp->vr[p], sp->vt[p], sp->vz[p], sp->ar[p],
                       sp->az[p], wr, sp->at[p]) < 0)
                return -2;
    }
    sp->n += sp->npend;
    sp->npend = 0;
    return 0;
}

/* Zero-order particle-based resizing (Sec. 2.2, after Bird): the weight a
 * particle should have at its present radius is w_r(r); with ratio
 * q = w / w_r it is kept as N = floor(q) copies plus one more with
 * probability q - floor(q) (first uniform of draw block 6 of (seed, s, id,
 * step)), each of weight w_r, so the charge is conserved on average.  N = 0
 * removes it; the N - 1 duplicates copy its phase space, take new ids in
 * parent order and are appended; then the array is compacted. */
static int resize_zero_order(rzo *o, int s, int64_t step)
{
    species *sp = &o->sp[s];
    double half = 0.5 * o->hr;
    int64_t n = sp->n;
    for (int64_t p = 0; p < n; ++p) {
        double rr = sp->r[p] > half ? sp->r[p] : half;
        double wr = o->c.resize_wcoef * rr;
        double q = sp->w[p] / wr;
        double k = floor(q);
        double u[2];
        rzo_uniform_pair(o->c.seed, s, sp->id[p], (uint32_t)step, 6, u);
        int64_t N = (int64_t)k + (u[0] < q - k ? 1 : 0);
        if (N == 0) {
            sp->dead[p] = 1;
            continue;
        }
        sp->w[p] = wr;
        for (int64_t c = 1; c < N; ++c)
            if (append(sp, sp->r[p], sp->z[p], sp->vr[p], sp->vt[p], sp->vz[p], sp->ar[p],
                       sp->az[p], wr, sp->at[p]) < 0)
                return -2;
    }
    sp->n += sp->npend;
    sp->npend = 0;
    return rzo_compact(o, s);
}

int rzo_resize_step(rzo *o, int s, int64_t step)
{
    if (o->c.resize_mode == RZO_RESIZE_ZERO_ORDER) return resize_zero_order(o, s, step);
    return resize_split(o, s);
}

int rzo_resize(rzo *o, int s) { return rzo_resize_step(o, s, 0); }

/* Tile key of a position: the cell (i, j) = (floor(z / hz), floor(r / hr)),
 * clamped to the mesh, and its tile of tile_z x tile_r cells, numbered with
 * r fastest.  (The paper sorts particles by cell to speed up weighting and
 * finds no gain on its CPUs, Sec. 2.7; here the key only has to be the same
 * on both implementations.) */
static int ntiles_r(const rzo *o) { return (o->c.nr - 2) / o->c.tile_r + 1; }
static int ntiles_z(const rzo *o) { return (o->c.nz - 2) / o->c.tile_z + 1; }

int32_t rzo_tile_key(const rzo *o, double r, double z)
{
    int i = (int)floor(z / o->hz), j = (int)floor(r / o->hr);
    if (i < 0) i = 0;
    if (i > o->c.nz - 2) i = o->c.nz - 2;
    if (j < 0) j = 0;
    if (j > o->c.nr - 2) j = o->c.nr - 2;
    return (int32_t)((i / o->c.tile_z) * ntiles_r(o) + j / o->c.tile_r);
}

/* Stable counting sort of the particle array by tile key: particles of a
 * lower tile first, the array order kept among those of one tile. */
int rzo_sort(rzo *o, int s)
{
    species *sp = &o->sp[s];
    if (o->c.tile_z < 1 || o->c.tile_r < 1) return -1;
    const int nt = ntiles_z(o) * ntiles_r(o);
    const int64_t n = sp->n;
    int64_t *start = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
    int32_t *key = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    double *tmp = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    uint64_t *tid = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
    int64_t *dst = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!start || !key || !tmp || !tid || !dst) {
        free(start); free(key); free(tmp); free(tid); free(dst);
        return -2;
    }
    for (int64_t p = 0; p < n; ++p) {
        key[p] = rzo_tile_key(o, sp->r[p], sp->z[p]);
        start[key[p] + 1]++;
    }
    for (int t = 0; t < nt; ++t) start[t + 1] += start[t];
    for (int64_t p = 0; p < n; ++p) dst[p] = start[key[p]]++;
    double *f[9] = {sp->r, sp->z, sp->vr, sp->vt, sp->vz, sp->ar, sp->az, sp->w, sp->at};
    for (int k = 0; k < 9; ++k) {
        for (int64_t p = 0; p < n; ++p) tmp[dst[p]] = f[k][p];
        copy_bytes(f[k], tmp, (size_t)n * sizeof(double));
    }
    for (int64_t p = 0; p < n; ++p) tid[dst[p]] = sp->id[p];
    copy_bytes(sp->id, tid, (size_t)n * sizeof(uint64_t));
    free(start); free(key); free(tmp); free(tid); free(dst);
    return nt;
}

/* ------------------------------------------------------------------------ */
/* Field solver (Sec. 2.5).                                                  */

static double face(const rzo *o, double a, double b)
{
    if (o->c.chi_face == RZO_FACE_MAX) return a > b ? a : b;
    return 0.5 * (a + b);
}

/* Finite-volume coefficients at unknown (i, j) of a level with axial spacing
 * hz: the flux through each control-volume face divided by the volume.
 * r-faces sit at r_j +- hr/2 with area 2 pi r hz, z-faces have area 2 pi r_j hr
 * (pi hr^2/4 on the axis), the volume is 2 pi r_j hr hz (pi hr^2 hz / 4 on the
 * axis, which has no inner face).  b = a + c + d + e. */
static void coef(const rzo *o, const double *eps, double hz, int i, int j, double *a,
                 double *b, double *c, double *d, double *e)
{
    int nr = o->c.nr;
    double hr = o->hr;
    const double *ec = eps + (size_t)i * nr;
    double hz2 = hz * hz, hr2 = hr * hr;
    *a = face(o, ec[j - nr], ec[j]) / hz2;
    *c = face(o, ec[j], ec[j + nr]) / hz2;
    if (j == 0) {
        *d = 0.0;
        *e = 4.0 * face(o, ec[0], ec[1]) / hr2;
    } else {
        double jj = (double)j;
        *d = face(o, ec[j - 1], ec[j]) * (jj - 0.5) / (jj * hr2);
        *e = face(o, ec[j], ec[j + 1]) * (jj + 0.5) / (jj * hr2);
    }
    *b = *a + *c + *d + *e;
}

/* res = f - A u on the interior rows of level l; zero on boundary nodes. */
static void residual(rzo *o, int l, const double *u, const double *f, double *res)
{
    int nr = o->c.nr, nzl = o->nzl[l];
    memset(res, 0, (size_t)nzl * nr * sizeof(double));
    for (int i = 1; i < nzl - 1; ++i)
        for (int j = 0; j < nr - 1; ++j) {
            double a, b, c, d, e;
            coef(o, o->eps_l[l], o->hzl[l], i, j, &a, &b, &c, &d, &e);
            size_t g = (size_t)i * nr + j;
            double Au = b * u[g] - a * u[g - nr] - c * u[g + nr] - e * u[g + 1];
            if (j > 0) Au -= d * u[g - 1];
            res[g] = f[g] - Au;
        }
}

static double maxabs_interior(const rzo *o, int l, const double *x)
{
    int nr = o->c.nr, nzl = o->nzl[l];
    double m = 0.0;
    for (int i = 1; i < nzl - 1; ++i)
        for (int j = 0; j < nr - 1; ++j) {
            double v = fabs(x[(size_t)i * nr + j]);
            if (v > m) m = v;
        }
    return m;
}

/* Full weighting [1/4 1/2 1/4] along z from level l to level l-1. */
static void restrict_fw(const rzo *o, int l, const double *fine, double *coarse)
{
    int nr = o->c.nr, nzc = o->nzl[l - 1];
    memset(coarse, 0, (size_t)nzc * nr * sizeof(double));
    for (int I = 1; I < nzc - 1; ++I)
        for (int j = 0; j < nr - 1; ++j)
            coarse[(size_t)I * nr + j] = 0.25 * fine[(size_t)(2 * I - 1) * nr + j] +
                                         0.5 * fine[(size_t)(2 * I) * nr + j] +
                                         0.25 * fine[(size_t)(2 * I + 1) * nr + j];
}

/* u^l += P u^{l-1}: linear interpolation along z (coincident lines copied,
 * in-between lines the mean of the two coarse neighbours). */
static void prolong_add(const rzo *o, int l, const double *uc, double *u)
{
    int nr = o->c.nr, nzl = o->nzl[l];
    for (int i = 1; i < nzl - 1; ++i)
        for (int j = 0; j < nr - 1; ++j) {
            double add;
            if (i % 2 == 0)
                add = uc[(size_t)(i / 2) * nr + j];
            else
                add = 0.5 * (uc[(size_t)(i / 2) * nr + j] + uc[(size_t)(i / 2 + 1) * nr + j]);
            u[(size_t)i * nr + j] += add;
        }
}

int rzo_thomas(int32_t n, const double *d, const double *b, const double *e,
               const double *g, double *x)
{
    if (n < 1) return -1;
    double *cp = (double *)malloc((size_t)n * sizeof(double));
    double *gp = (double *)malloc((size_t)n * sizeof(double));
    if (!cp || !gp) {
        free(cp);
        free(gp);
        return -2;
    }
    cp[0] = e[0] / b[0];
    gp[0] = g[0] / b[0];
    for (int j = 1; j < n; ++j) {
        double den = b[j] - d[j] * cp[j - 1];
        cp[j] = e[j] / den;
        gp[j] = (g[j] + d[j] * gp[j - 1]) / den;
    }
    x[n - 1] = gp[n - 1];
    for (int j = n - 2; j >= 0; --j) x[j] = gp[j] + cp[j] * x[j + 1];
    free(cp);
    free(gp);
    return 0;
}

/* Exact solve of line i of level l for j = 0..nr-2 with the neighbouring lines
 * i-1, i+1 and the wall value u_{i,nr-1} taken from u as it stands. */
static void line_solve(rzo *o, int l, double *u, const double *f, int i)
{
    int nr = o->c.nr, n = nr - 1;
    for (int j = 0; j < n; ++j) {
        double a, b, c, d, e;
        coef(o, o->eps_l[l], o->hzl[l], i, j, &a, &b, &c, &d, &e);
        size_t g = (size_t)i * nr + j;
        double rhs = f[g] + a * u[g - nr] + c * u[g + nr];
        if (j == n - 1) {
            rhs += e * u[g + 1];
            e = 0.0;
        }
        o->ld[j] = d;
        o->lb[j] = b;
        o->le[j] = e;
        o->lg[j] = rhs;
    }
    rzo_thomas(n, o->ld, o->lb, o->le, o->lg, o->lx);
    for (int j = 0; j < n; ++j) u[(size_t)i * nr + j] = o->lx[j];
}

/* Zebra line relaxation: every odd line, then every even line. */
static void line_smooth(rzo *o, int l, double *u, const double *f)
{
    int nzl = o->nzl[l];
    for (int i = 1; i < nzl - 1; i += 2) line_solve(o, l, u, f, i);
    for (int i = 2; i < nzl - 1; i += 2) line_solve(o, l, u, f, i);
}

/* Algorithm 1, the V(0,1) cycle: residual restricted down with u^l = 0 on every
 * coarse level, exact solve of the single line of level 1, then on the way up
 * the prolonged correction is added and one line smoothing is applied. */
static void vcycle(rzo *o)
{
    int L = o->L, nr = o->c.nr;
    double *uL = o->u_l[L], *fL = o->f_l[L];
    if (L == 1) {
        line_smooth(o, 1, uL, fL);
        return;
    }
    residual(o, L, uL, fL, o->res);
    restrict_fw(o, L, o->res, o->f_l[L - 1]);
    for (int l = L - 1; l >= 2; --l) {
        memset(o->u_l[l], 0, (size_t)o->nzl[l] * nr * sizeof(double));
        residual(o, l, o->u_l[l], o->f_l[l], o->res); /* = f^l since u^l = 0 */
        restrict_fw(o, l, o->res, o->f_l[l - 1]);
    }
    memset(o->u_l[1], 0, (size_t)o->nzl[1] * nr * sizeof(double));
    line_solve(o, 1, o->u_l[1], o->f_l[1], 1);
    for (int l = 2; l <= L; ++l) {
        prolong_add(o, l, o->u_l[l - 1], o->u_l[l]);
        line_smooth(o, l, o->u_l[l], o->f_l[l]);
    }
}

/* Coarse-level epsilon: full weighting along z, electrode rows injected. */
static void build_levels(rzo *o)
{
    int nr = o->c.nr, L = o->L;
    double *eL = o->eps_l[L];
    for (int g = 0; g < o->nn; ++g) eL[g] = 1.0 + o->chi[g];
    for (int l = L; l >= 2; --l) {
        const double *ef = o->eps_l[l];
        double *ec = o->eps_l[l - 1];
        int nzc = o->nzl[l - 1];
        for (int j = 0; j < nr; ++j) {
            ec[j] = ef[j];
            ec[(size_t)(nzc - 1) * nr + j] = ef[(size_t)(o->nzl[l] - 1) * nr + j];
        }
        for (int I = 1; I < nzc - 1; ++I)
            for (int j = 0; j < nr; ++j)
                ec[(size_t)I * nr + j] = 0.25 * ef[(size_t)(2 * I - 1) * nr + j] +
                                         0.5 * ef[(size_t)(2 * I) * nr + j] +
                                         0.25 * ef[(size_t)(2 * I + 1) * nr + j];
    }
}

/* Dirichlet data of u: V on the powered electrode z = 0 (r < R), 0 V on the
 * grounded electrode z = L and on the wall r = R including both corners. */
static void set_bc(rzo *o, double *u, double V)
{
    int nr = o->c.nr, nz = o->c.nz;
    for (int j = 0; j < nr; ++j) {
        u[j] = j < nr - 1 ? V : 0.0;
        u[(size_t)(nz - 1) * nr + j] = 0.0;
    }
    for (int i = 0; i < nz; ++i) u[(size_t)i * nr + nr - 1] = 0.0;
}

/* Algorithm 1 on u (warm start: its interior) for the right-hand side fr and
 * the electrode value V, with the levels' epsilon already built: cycles until
 * the relative residual test of Sec. 2.5 holds, or the fixed count. */
static int solve_on(rzo *o, double *u, const double *fr, double V, int32_t *cycles,
                    double *relres)
{
    int L = o->L, nr = o->c.nr, nz = o->c.nz;
    double *f = o->f_l[L];
    if (f != fr) memcpy(f, fr, (size_t)o->nn * sizeof(double));
    set_bc(o, u, V);
    double *keep = o->u_l[L];
    o->u_l[L] = u;
    /* Scale of the relative residual: the residual of the boundary data with
     * a zero interior, i.e. the right-hand side of the interior system. */
    double *ubc = (double *)calloc((size_t)o->nn, sizeof(double));
    for (int j = 0; j < nr; ++j) {
        ubc[j] = u[j];
        ubc[(size_t)(nz - 1) * nr + j] = u[(size_t)(nz - 1) * nr + j];
    }
    residual(o, L, ubc, f, o->res);
    double scale = maxabs_interior(o, L, o->res);
    free(ubc);
    int k = 0;
    int status = 0;
    for (;;) {
        if (o->c.mg_fixed_cycles > 0) {
            if (k >= o->c.mg_fixed_cycles) break;
        } else {
            residual(o, L, u, f, o->res);
            double rn = maxabs_interior(o, L, o->res);
            if (rn <= o->c.mg_tol * scale) break;
            if (k >= o->c.mg_max_cycles) {
                status = 1;
                break;
            }
        }
        vcycle(o);
        ++k;
    }
    residual(o, L, u, f, o->res);
    double rn = maxabs_interior(o, L, o->res);
    o->u_l[L] = keep;
    if (cycles) *cycles = k;
    if (relres) *relres = scale > 0.0 ? rn / scale : rn;
    return status;
}

/* Charge on the z = 0 electrode (r < R) of the potential u with the charge
 * density rho (NULL: none), by Gauss's law on the union of the electrode
 * nodes' half cells (0 <= z <= hz/2): the displacement eps0 (1+chi) E flowing
 * out through their upper faces (area 2 pi r_j hr, pi hr^2/4 on the axis, at
 * distance hz from row 1) and through the side face of the last one towards
 * the wall node (area pi r_{nr-3/2} hz at distance hr), less the charge the
 * deposit assigns to the half cells, rho V on row 0. */
static double electrode_charge(const rzo *o, const double *u, const double *rho)
{
    int nr = o->c.nr;
    double hr = o->hr, hz = o->hz;
    const double *eps = o->eps_l[o->L];
    double q = 0.0;
    for (int j = 0; j < nr - 1; ++j) {
        double area = j == 0 ? PI_ * 0.25 * hr * hr : 2.0 * PI_ * (double)j * hr * hr;
        q += EPS0 * face(o, eps[j], eps[nr + j]) * area * (u[j] - u[nr + j]) / hz;
        if (rho) q -= rho[j] * o->vol[j];
    }
    int jw = nr - 2;
    double rface = ((double)jw + 0.5) * hr;
    q += EPS0 * face(o, eps[jw], eps[jw + 1]) * PI_ * rface * hz / hr * (u[jw] - u[jw + 1]);
    return q;
}

/* External circuit (Sec. 2.5, the superposition of Vahedi): phi_P solves the
 * field equation with the charge and the electrode at 0 V, phi_L the same
 * operator without charge and the electrode at 1 V; the electrode charge of
 * phi = phi_P + V phi_L is Q_P + V Q_L.  The blocking-capacitor equation
 *   Q^t = Q^{t-1} + C (V_s^t - V^t) - Q_c^{t-1} + Q_conv^t,  Q_c^t = C (V_s^t - V^t),
 * with Q_conv the charge absorbed at the electrode since the previous solve
 * (this step's first push and the previous step's final push), gives V^t. */
static int circuit_solve(rzo *o, double Vs, const double *f, int32_t *cycles, double *relres)
{
    int32_t c1 = 0, c2 = 0;
    double r1 = 0.0, r2 = 0.0;
    int st = solve_on(o, o->phiP, f, 0.0, &c1, &r1);
    int st2 = solve_on(o, o->phiL, o->zero, 1.0, &c2, &r2);
    double C = o->c.circuit_C;
    double Qp = electrode_charge(o, o->phiP, o->rho);
    double Ql = electrode_charge(o, o->phiL, NULL);
    double Qconv = 0.0;
    for (int s = 0; s < 2; ++s) {
        Qconv += o->sp[s].q * (o->sp[s].absorbed[0] - o->absorbed_prev[s]);
        o->absorbed_prev[s] = o->sp[s].absorbed[0];
    }
    double V = (o->cQ - o->cQc + Qconv + C * Vs - Qp) / (Ql + C);
    o->cV = V;
    o->cQ = Qp + V * Ql;
    o->cQc = C * (Vs - V);
    o->cQconv = Qconv;
    o->cQp = Qp;
    o->cQl = Ql;
    for (int g = 0; g < o->nn; ++g) o->phi[g] = o->phiP[g] + V * o->phiL[g];
    if (cycles) *cycles = c1 > c2 ? c1 : c2;
    if (relres) *relres = r1 > r2 ? r1 : r2;
    return st ? st : st2;
}

int rzo_set_circuit(rzo *o, double V, double Q, double Qc)
{
    if (!o || !(o->c.circuit_C > 0.0)) return -1;
    o->cV = V;
    o->cQ = Q;
    o->cQc = Qc;
    return 0;
}

int rzo_circuit(const rzo *o, double out[6])
{
    out[0] = o->cV;
    out[1] = o->cQ;
    out[2] = o->cQc;
    out[3] = o->cQconv;
    out[4] = o->cQp;
    out[5] = o->cQl;
    return o->c.circuit_C > 0.0 ? 0 : -1;
}

int rzo_solve(rzo *o, double t, int32_t *cycles, double *relres)
{
    int L = o->L;
    double V = o->c.V_dc + o->c.V_rf * sin(TWO_PI * o->c.f_rf * t);
    double *f = o->f_l[L];
    for (int g = 0; g < o->nn; ++g) f[g] = o->rho[g] / EPS0;
    build_levels(o);
    if (o->c.circuit_C > 0.0) return circuit_solve(o, V, f, cycles, relres);
    return solve_on(o, o->phi, f, V, cycles, relres);
}

/* E = -grad phi: centred differences inside, one-sided on the electrodes and
 * the wall, E_r = 0 on the axis. */
int rzo_efield(rzo *o)
{
    int nr = o->c.nr, nz = o->c.nz;
    const double *u = o->phi;
    for (int i = 0; i < nz; ++i)
        for (int j = 0; j < nr; ++j) {
            size_t g = (size_t)i * nr + j;
            double ez, er;
            if (i == 0)
                ez = -(u[g + nr] - u[g]) / o->hz;
            else if (i == nz - 1)
                ez = -(u[g] - u[g - nr]) / o->hz;
            else
                ez = -(u[g + nr] - u[g - nr]) / (2.0 * o->hz);
            if (j == 0)
                er = 0.0;
            else if (j == nr - 1)
                er = -(u[g] - u[g - 1]) / o->hr;
            else
                er = -(u[g + 1] - u[g - 1]) / (2.0 * o->hr);
            o->ez[g] = ez;
            o->er[g] = er;
        }
    return 0;
}

int rzo_apply_op(const rzo *o, const double *u, double *y)
{
    rzo *m = (rzo *)o;
    int L = o->L, nr = o->c.nr;
    double *zero = (double *)calloc((size_t)o->nn, sizeof(double));
    build_levels(m);
    residual(m, L, u, zero, y);
    for (int g = 0; g < o->nn; ++g) y[g] = -y[g];
    (void)nr;
    free(zero);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Initialisation, step, grid access.                                        */

int rzo_init_particles(rzo *o, int s, int64_t n, double n0, double T_eV, uint64_t id0)
{
    species *sp = &o->sp[s];
    if (n < 0 || grow(sp, n) != 0) return -1;
    double wcoef = TWO_PI * n0 * o->c.R * o->c.L / (double)n;
    double vth = sqrt(T_eV * Q_E / sp->m);
    const uint32_t INIT = 0xFFFFFFFFu;
    for (int64_t p = 0; p < n; ++p) {
        uint64_t id = id0 + (uint64_t)p;
        double u0[2], u1[2], u2[2], g1[2], g2[2];
        rzo_uniform_pair(o->c.seed, s, id, INIT, 0, u0);
        rzo_uniform_pair(o->c.seed, s, id, INIT, 1, u1);
        rzo_uniform_pair(o->c.seed, s, id, INIT, 2, u2);
        normal_pair(u1, g1);
        normal_pair(u2, g2);
        double r = u0[0] * o->c.R;
        sp->r[p] = r;
        sp->z[p] = u0[1] * o->c.L;
        sp->vr[p] = vth * g1[0];
        sp->vt[p] = vth * g1[1];
        sp->vz[p] = vth * g2[0];
        sp->ar[p] = 0.0;
        sp->az[p] = 0.0;
        sp->at[p] = 0.0;
        sp->w[p] = wcoef * r;
        sp->id[p] = id;
        sp->dead[p] = 0;
    }
    sp->n = n;
    sp->npend = 0;
    sp->next_id = id0 + (uint64_t)n;
    return 0;
}

int rzo_prologue(rzo *o)
{
    for (int s = 0; s < 2; ++s) rzo_push_first(o, s);
    deposit_all(o);
    for (int s = 0; s < 2; ++s) rzo_compact(o, s);
    return 0;
}

int rzo_step(rzo *o, int64_t n, int merged)
{
    /* subcycled ions (Sec. 2.7): they move only in every K-th step; in the
     * others their deposit is kept and they add no susceptibility */
    const int ions = ion_step(o, n);
    finalize_ions(o, ions);
    int32_t cyc;
    double rr;
    int st = rzo_solve(o, (double)(n + 1) * o->c.dt, &cyc, &rr);
    rzo_efield(o);
    uint32_t step = (uint32_t)n;
    if (merged) {
        for (int s = 0; s < 2; ++s)
            if (s == 0 || ions) memset(o->N[s], 0, (size_t)o->nn * sizeof(double));
        for (int s = 0; s < 2; ++s) {
            if (s == 1 && !ions) continue;
            species *sp = &o->sp[s];
            int do_mc = sp->mc_model != RZO_MC_NONE && sp->nproc > 0;
            if (do_mc && ensure_ev(sp) != 0) return -2;
            int64_t np = sp->n;
            for (int64_t p = 0; p < np; ++p) {
                if (final_push_one(o, sp, p)) continue;
                if (do_mc) sp->ev[p] = collide_one(o, s, p, step);
                if (first_push_one(o, sp, p)) continue;
                deposit_one(o, s, p);
            }
        }
        for (int s = 0; s < 2; ++s) {
            species *sp = &o->sp[s];
            for (int64_t c = sp->n; c < sp->n + sp->npend; ++c) {
                if (first_push_one(o, sp, c)) continue;
                deposit_one(o, s, c);
            }
        }
    } else {
        for (int s = 0; s < 2; ++s)
            if (s == 0 || ions) rzo_push_final(o, s);
        for (int s = 0; s < 2; ++s)
            if (s == 0 || ions) rzo_collide(o, s, n);
        for (int s = 0; s < 2; ++s) {
            if (s == 0 || ions) {
                rzo_push_first(o, s);
            } else {
                species *sp = &o->sp[s]; /* children of this step's ionizations */
                for (int64_t c = sp->n; c < sp->n + sp->npend; ++c) first_push_one(o, sp, c);
            }
        }
        deposit_all(o);
    }
    for (int s = 0; s < 2; ++s) rzo_compact(o, s);
    if (o->c.resize_every > 0 && n % o->c.resize_every == o->c.resize_every - 1) {
        for (int s = 0; s < 2; ++s)
            if (rzo_resize_step(o, s, n) != 0) return -2;
        deposit_all(o);
    }
    if (o->c.sort_every > 0 && n % o->c.sort_every == o->c.sort_every - 1)
        for (int s = 0; s < 2; ++s)
            if (rzo_sort(o, s) < 0) return -2;
    return st;
}

static double *grid_ptr(const rzo *o, int which)
{
    switch (which) {
    case RZO_G_PHI: return o->phi;
    case RZO_G_RHO: return o->rho;
    case RZO_G_CHI: return o->chi;
    case RZO_G_ER: return o->er;
    case RZO_G_EZ: return o->ez;
    case RZO_G_N0: return o->N[0];
    case RZO_G_N1: return o->N[1];
    case RZO_G_DENS0: return o->dens[0];
    case RZO_G_DENS1: return o->dens[1];
    case RZO_G_VOL: return o->vol;
    case RZO_G_PHI_P: return o->phiP;
    case RZO_G_PHI_L: return o->phiL;
    default: return NULL;
    }
}

int rzo_get_grid(const rzo *o, int which, double *out)
{
    double *p = grid_ptr(o, which);
    if (!p) return -1;
    memcpy(out, p, (size_t)o->nn * sizeof(double));
    return 0;
}

int rzo_set_grid(rzo *o, int which, const double *in)
{
    double *p = grid_ptr(o, which);
    if (!p || which == RZO_G_VOL || which == RZO_G_PHI_P || which == RZO_G_PHI_L) return -1;
    memcpy(p, in, (size_t)o->nn * sizeof(double));
    return 0;
}

int rzo_absorbed(const rzo *o, int s, double out[3])
{
    for (int b = 0; b < 3; ++b) out[b] = o->sp[s].absorbed[b];
    return 0;
}
