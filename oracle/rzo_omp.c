/*
 * rzo_omp.c -- OpenMP timing build of the FP64 CPU oracle (test
 * infrastructure only: the CPU baseline of the benchmark and its test).
 *
 * It includes the oracle's source unchanged and adds one entry point,
 * rzo_omp_step, which runs a merged step (rzo_step with merged != 0) with the
 * particle loops spread over threads.  Every particle still goes through the
 * oracle's own functions in the order of the step (final push, collision,
 * first push, deposit); only the loops are reordered, as in the unmerged
 * step of Sec. 2.1 (the oracle's merged and unmerged steps agree):
 *   1. final push of every particle (parallel);
 *   2. the candidate draw U0 of every live particle (parallel), then the
 *      collision outcome of the candidates in array order (serial: new
 *      particles take their identities in parent order);
 *   3. first push and deposit (parallel, one deposit buffer per thread,
 *      summed in thread order), then the new particles (serial).
 * The deposit sums in another order than the serial oracle, so results agree
 * with it to rounding (1e-12 relative is tested), not bit for bit.  The
 * particle phase and the field solve are timed separately.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared rzo_omp.c -lm
 */
#include "rzo.c"

#include <omp.h>

static double *omp_buf;      /* nthreads * nn deposit buffers */
static size_t omp_buf_len;

void rzo_omp_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

int rzo_omp_threads(void) { return omp_get_max_threads(); }

static int omp_deposit_buffers(const rzo *o, int nt)
{
    size_t need = (size_t)nt * (size_t)o->nn;
    if (need > omp_buf_len) {
        free(omp_buf);
        omp_buf = (double *)malloc(need * sizeof(double));
        if (!omp_buf) {
            omp_buf_len = 0;
            return -1;
        }
        omp_buf_len = need;
    }
    return 0;
}

/* One merged step n; *t_particles and *t_solve (may be NULL) receive the
 * seconds of the particle phase (pushes, collisions, deposit, list
 * maintenance) and of the field solve (finalize, multigrid, E), *cycles
 * (may be NULL) the V-cycles of the solve. */
int rzo_omp_step(rzo *o, int64_t n, double *t_particles, double *t_solve, int32_t *cycles)
{
    double t0 = omp_get_wtime();
    const int ions = ion_step(o, n);
    finalize_ions(o, ions);
    int32_t cyc;
    double rr;
    int st = rzo_solve(o, (double)(n + 1) * o->c.dt, &cyc, &rr);
    rzo_efield(o);
    double t1 = omp_get_wtime();
    const uint32_t step = (uint32_t)n;
    const int nt = omp_get_max_threads();
    if (omp_deposit_buffers(o, nt) != 0) return -2;
    const int nn = o->nn;
    const size_t nr = (size_t)o->c.nr;
    for (int s = 0; s < 2; ++s) {
        if (s == 1 && !ions) continue;
        species *sp = &o->sp[s];
        const int64_t np = sp->n;
        const int do_mc = sp->mc_model != RZO_MC_NONE && sp->nproc > 0;
        if (do_mc && ensure_ev(sp) != 0) return -2;
        /* 1. final push */
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < np; ++p) final_push_one(o, sp, p);
        /* 2. candidates in parallel (the same draw collide_one makes first),
         * outcomes in array order */
        if (do_mc) {
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < np; ++p) {
                sp->ev[p] = 0;
                if (sp->dead[p]) continue;
                double u[2];
                rzo_uniform_pair(o->c.seed, s, sp->id[p], step, 0, u);
                if (u[0] < sp->p_null) sp->ev[p] = 0xFF;
            }
            for (int64_t p = 0; p < np; ++p)
                if (sp->ev[p] == 0xFF) sp->ev[p] = collide_one(o, s, p, step);
        }
        /* 3. first push and deposit, one buffer per thread */
#pragma omp parallel
        {
            double *N = omp_buf + (size_t)omp_get_thread_num() * (size_t)nn;
            memset(N, 0, (size_t)nn * sizeof(double));
#pragma omp for schedule(static)
            for (int64_t p = 0; p < np; ++p) {
                if (sp->dead[p] || first_push_one(o, sp, p)) continue;
                wts q = weights(o, sp->r[p], sp->z[p]);
                const double w = sp->w[p];
                const size_t g = (size_t)q.i * nr + (size_t)q.j;
                N[g] += w * q.sz0 * q.sr0;
                N[g + 1] += w * q.sz0 * q.sr1;
                N[g + nr] += w * q.sz1 * q.sr0;
                N[g + nr + 1] += w * q.sz1 * q.sr1;
            }
        }
        double *Ns = o->N[s];
        memset(Ns, 0, (size_t)nn * sizeof(double));
        for (int t = 0; t < nt; ++t) {
            const double *N = omp_buf + (size_t)t * (size_t)nn;
            for (int g = 0; g < nn; ++g) Ns[g] += N[g];
        }
    }
    /* the new particles of this step, after both species */
    for (int s = 0; s < 2; ++s) {
        species *sp = &o->sp[s];
        for (int64_t c = sp->n; c < sp->n + sp->npend; ++c) {
            if (first_push_one(o, sp, c)) continue;
            deposit_one(o, s, c);
        }
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
    double t2 = omp_get_wtime();
    if (t_solve) *t_solve = t1 - t0;
    if (t_particles) *t_particles = t2 - t1;
    if (cycles) *cycles = cyc;
    return st;
}
