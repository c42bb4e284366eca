// Deterministic list maintenance after a particle pass: per-chunk counts are
// scanned in chunk order, absorbed particles leave holes that are filled in
// increasing order by the live particles of the tail, and new particles are
// appended in parent order with consecutive identities.  The resulting array
// does not depend on the launch shape or on the order atomics land in.
#include "device.h"

namespace rz {

// Exclusive scan of in[0..n) into out[] by one block; returns the total.
__device__ int64_t block_scan_tiles(const int32_t *in, int64_t *out, int64_t n, int *sh)
{
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += blockDim.x) {
        int64_t i = base + threadIdx.x;
        int v = i < n ? in[i] : 0;
        int tot;
        int ex = block_excl_sum(v, tot, sh);
        if (i < n) out[i] = carry + ex;
        carry += tot;
    }
    return carry;
}

__global__ __launch_bounds__(1024) void k_scan(ScanJobs j)
{
    __shared__ int sh[64];
    const int B = j.chunk;
    if (blockIdx.x == 0) {
        if (!j.children) return;
        const int64_t nch = (j.crec->n_parent + B - 1) / B;
        int64_t ev = block_scan_tiles(j.ech.ev_cnt, j.ech.ev_off, nch, sh);
        int64_t se = block_scan_tiles(j.ech.surv_e, j.ech.surv_e_off, nch, sh);
        int64_t si = block_scan_tiles(j.ech.surv_i, j.ech.surv_i_off, nch, sh);
        if (threadIdx.x == 0) {
            j.crec->ev_total = ev;
            j.crec->surv_total[0] = se;
            j.crec->surv_total[1] = si;
            j.crec->next_id_old[0] = j.ecnt->next_id;
            j.crec->next_id_old[1] = j.icnt->next_id;
        }
        return;
    }
    const int s = blockIdx.x - 1;
    if (!j.dead[s]) return;
    const int64_t n = j.cnt[s]->n;
    const int64_t nch = (n + B - 1) / B;
    int64_t d = block_scan_tiles(j.ch[s].dead_cnt, j.ch[s].dead_off, nch, sh);
    if (threadIdx.x == 0) {
        j.fix[s]->n_old = n;
        j.fix[s]->dead = d;
        j.fix[s]->keep = n - d;
    }
}

hipError_t launch_scan(const ScanJobs &j, hipStream_t st)
{
    hipLaunchKernelGGL(k_scan, dim3(3), dim3(1024), 0, st, j);
    return hipGetLastError();
}

// Unmerged form: per-chunk lists of the particles marked dead (w < 0).
template <typename T>
__global__ __launch_bounds__(256) void k_dead_scan(const T *w, const Counts *cnt, Chunks ch)
{
    __shared__ int sh[64];
    const int B = blockDim.x;
    const int64_t n = cnt->n;
    const int64_t nch = (n + B - 1) / B;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        int64_t i = c * B + threadIdx.x;
        bool f[4] = {i < n && w[i] < (T)0, false, false, false};
        int rank[4], tot[4];
        block_rank4(f, rank, tot, sh);
        if (f[0]) ch.dead_list[c * B + rank[0]] = threadIdx.x;
        if (threadIdx.x == 0) ch.dead_cnt[c] = tot[0];
    }
}

template <typename T>
hipError_t launch_dead_scan(Parts<T> p, const Counts *cnt, Chunks ch, int chunk, hipStream_t st)
{
    hipLaunchKernelGGL((k_dead_scan<T>), dim3(1024), dim3(chunk), 0, st, p.w, cnt, ch);
    return hipGetLastError();
}

__global__ void k_dead_list(Chunks ch, const FixRec *fix, int B)
{
    const int64_t nch = (fix->n_old + B - 1) / B;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        int cnt = ch.dead_cnt[c];
        int64_t off = ch.dead_off[c];
        for (int k = threadIdx.x; k < cnt; k += blockDim.x)
            ch.dead_glob[off + k] = c * B + ch.dead_list[c * B + k];
    }
}

hipError_t launch_dead_list(Chunks ch, const Counts *cnt, const FixRec *fix, int chunk,
                            hipStream_t st)
{
    (void)cnt;
    hipLaunchKernelGGL(k_dead_list, dim3(1024), dim3(256), 0, st, ch, fix, chunk);
    return hipGetLastError();
}

// Hole m (the m-th dead index below keep) receives the m-th live particle of
// [keep, n).  With T_k the dead indices >= keep (sorted), that particle is
// keep + m + k for the smallest k whose T_k lies beyond it.
template <typename T> __global__ void k_fill(Parts<T> p, const int64_t *dead, const FixRec *fix)
{
    const int64_t D = fix->dead, keep = fix->keep;
    if (D == 0) return;
    int64_t lo = 0, hi = D;  // H = number of dead indices < keep
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (dead[mid] < keep) lo = mid + 1;
        else hi = mid;
    }
    const int64_t H = lo;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < H;
         m += (int64_t)gridDim.x * blockDim.x) {
        int64_t a = 0, b = D - H;
        while (a < b) {
            int64_t k = (a + b) >> 1;
            if (dead[H + k] - keep - k > m) b = k;
            else a = k + 1;
        }
        const int64_t src = keep + m + a, dst = dead[m];
        p.r[dst] = p.r[src];
        p.z[dst] = p.z[src];
        p.vr[dst] = p.vr[src];
        p.vt[dst] = p.vt[src];
        p.vz[dst] = p.vz[src];
        p.ar[dst] = p.ar[src];
        p.az[dst] = p.az[src];
        p.w[dst] = p.w[src];
        p.id[dst] = p.id[src];
    }
}

template <typename T>
hipError_t launch_fill(Parts<T> p, Chunks ch, const FixRec *fix, hipStream_t st)
{
    hipLaunchKernelGGL((k_fill<T>), dim3(256), dim3(256), 0, st, p, ch.dead_glob, fix);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(1024) void k_append(Parts<T> dst, Parts<T> stage, int cs, Chunks ech,
                                                 int children, const ChildRec *crec,
                                                 const FixRec *fix, Counts *cnt, int64_t cap,
                                                 int32_t *status)
{
    __shared__ int sh[64];
    const int B = blockDim.x;
    const int64_t keep = fix->keep;
    if (children) {
        const int32_t *surv = cs == 0 ? ech.surv_e : ech.surv_i;
        const int64_t *surv_off = cs == 0 ? ech.surv_e_off : ech.surv_i_off;
        (void)surv;
        const uint64_t id0 = crec->next_id_old[cs];
        const int64_t nch = (crec->n_parent + B - 1) / B;
        for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
            const int ne = ech.ev_cnt[c];
            if (ne == 0) continue;  // uniform over the block
            const int k = threadIdx.x;
            const int64_t slot = c * B + k;
            bool alive = k < ne && stage.w[slot] >= (T)0;
            int tot;
            int rank = block_excl_sum(alive ? 1 : 0, tot, sh);
            int64_t to = keep + surv_off[c] + rank;
            if (alive && to < cap) {
                dst.r[to] = stage.r[slot];
                dst.z[to] = stage.z[slot];
                dst.vr[to] = stage.vr[slot];
                dst.vt[to] = stage.vt[slot];
                dst.vz[to] = stage.vz[slot];
                dst.ar[to] = stage.ar[slot];
                dst.az[to] = stage.az[slot];
                dst.w[to] = stage.w[slot];
                dst.id[to] = id0 + (uint64_t)(ech.ev_off[c] + k);
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t n_new = keep;
        if (children) {
            int64_t surv = crec->surv_total[cs];
            int64_t room = cap - keep;
            if (surv > room) {
                atomicOr(status, kStCapacity);
                surv = room;
            }
            n_new += surv;
            cnt->next_id = crec->next_id_old[cs] + (uint64_t)crec->ev_total;
        }
        cnt->n = n_new;
    }
}

template <typename T>
hipError_t launch_append(Parts<T> dst, Parts<T> stage, int cs, Chunks ech, int children,
                         const ChildRec *crec, const FixRec *fix, Counts *cnt, int64_t cap,
                         int chunk, int32_t *status, hipStream_t st)
{
    hipLaunchKernelGGL((k_append<T>), dim3(children ? 1024 : 1), dim3(chunk), 0, st, dst, stage, cs,
                       ech, children, crec, fix, cnt, cap, status);
    return hipGetLastError();
}

// Weight split (Sec. 2.2): clone count of each particle.  Contraction is off
// so that the count of an exact multiple is decided exactly as written.
__device__ __forceinline__ int clones_of(double w, double r, double wcoef, double half_hr,
                                         double &wr)
{
#pragma clang fp contract(off)
    double rr = r > half_hr ? r : half_hr;
    wr = wcoef * rr;
    if (!(w > wr)) return 0;
    double k = floor(w / wr);
    double rem = w - k * wr;
    long long nc = rem > 0.0 ? (long long)k : (long long)k - 1;
    return nc > 0 ? (int)nc : 0;
}

__device__ __forceinline__ double split_rest(double w, int nc, double wr)
{
#pragma clang fp contract(off)
    return w - (double)nc * wr;
}

template <typename T>
__global__ __launch_bounds__(256) void k_resize_count(Parts<T> p, const Counts *cnt, Chunks ch,
                                                      double wcoef, double half_hr)
{
    __shared__ int sh[64];
    const int B = blockDim.x;
    const int64_t n = cnt->n;
    const int64_t nch = (n + B - 1) / B;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        int64_t i = c * B + threadIdx.x;
        int nc = 0;
        if (i < n) {
            double wr;
            nc = clones_of((double)p.w[i], (double)p.r[i], wcoef, half_hr, wr);
            ch.pcount[i] = nc;
        }
        int tot;
        block_excl_sum(nc, tot, sh);
        if (threadIdx.x == 0) ch.clone_cnt[c] = tot;
    }
}

__global__ __launch_bounds__(1024) void k_resize_scan(const Counts *cnt, Chunks ch, CloneRec *rec,
                                                      int B, int64_t cap)
{
    __shared__ int sh[64];
    const int64_t n = cnt->n;
    const int64_t nch = (n + B - 1) / B;
    int64_t tot = block_scan_tiles(ch.clone_cnt, ch.clone_off, nch, sh);
    if (threadIdx.x == 0) {
        rec->n_old = n;
        rec->total = tot;
        rec->ok = n + tot <= cap;
        rec->next_id_old = cnt->next_id;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_resize_scatter(Parts<T> p, Counts *cnt, Chunks ch,
                                                        const CloneRec *rec, double wcoef,
                                                        double half_hr, int32_t *status)
{
    __shared__ int sh[64];
    const int B = blockDim.x;
    const int64_t n = rec->n_old;
    if (!rec->ok) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, kStCapacity);
        return;
    }
    const int64_t nch = (n + B - 1) / B;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        int64_t i = c * B + threadIdx.x;
        int nc = i < n ? ch.pcount[i] : 0;
        int tot;
        int ex = block_excl_sum(nc, tot, sh);
        if (nc > 0) {
            double wr;
            double w = (double)p.w[i];
            clones_of(w, (double)p.r[i], wcoef, half_hr, wr);
            const T r = p.r[i], z = p.z[i], vr = p.vr[i], vt = p.vt[i], vz = p.vz[i];
            const T ar = p.ar[i], az = p.az[i];
            p.w[i] = (T)split_rest(w, nc, wr);
            int64_t base = n + ch.clone_off[c] + ex;
            for (int k = 0; k < nc; ++k) {
                int64_t d = base + k;
                p.r[d] = r;
                p.z[d] = z;
                p.vr[d] = vr;
                p.vt[d] = vt;
                p.vz[d] = vz;
                p.ar[d] = ar;
                p.az[d] = az;
                p.w[d] = (T)wr;
                p.id[d] = rec->next_id_old + (uint64_t)(ch.clone_off[c] + ex + k);
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cnt->n = n + rec->total;
        cnt->next_id = rec->next_id_old + (uint64_t)rec->total;
    }
}

template <typename T>
hipError_t launch_resize(Parts<T> p, Counts *cnt, Chunks ch, CloneRec *rec, int chunk,
                         double wcoef, double half_hr, int64_t cap, int32_t *status,
                         hipStream_t st)
{
    hipLaunchKernelGGL((k_resize_count<T>), dim3(1024), dim3(chunk), 0, st, p, cnt, ch, wcoef,
                       half_hr);
    hipLaunchKernelGGL(k_resize_scan, dim3(1), dim3(1024), 0, st, cnt, ch, rec, chunk, cap);
    hipLaunchKernelGGL((k_resize_scatter<T>), dim3(1024), dim3(chunk), 0, st, p, cnt, ch, rec,
                       wcoef, half_hr, status);
    return hipGetLastError();
}

// acc[g] += sum over blocks of the per-block LDS copies.
__global__ void k_reduce_slices(unsigned long long *acc, const unsigned long long *slices, int nb,
                                int nn)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += gridDim.x * blockDim.x) {
        unsigned long long s = 0;
        for (int b = 0; b < nb; ++b) s += slices[(size_t)b * nn + g];
        acc[g] += s;
    }
}

hipError_t launch_reduce_slices(unsigned long long *acc, const unsigned long long *slices, int nb,
                                int nn, hipStream_t st)
{
    int threads = 256;
    int blocks = (nn + threads - 1) / threads;
    hipLaunchKernelGGL(k_reduce_slices, dim3(blocks), dim3(threads), 0, st, acc, slices, nb, nn);
    return hipGetLastError();
}

template hipError_t launch_dead_scan<double>(Parts<double>, const Counts *, Chunks, int,
                                             hipStream_t);
template hipError_t launch_dead_scan<float>(Parts<float>, const Counts *, Chunks, int, hipStream_t);
template hipError_t launch_fill<double>(Parts<double>, Chunks, const FixRec *, hipStream_t);
template hipError_t launch_fill<float>(Parts<float>, Chunks, const FixRec *, hipStream_t);
template hipError_t launch_append<double>(Parts<double>, Parts<double>, int, Chunks, int,
                                          const ChildRec *, const FixRec *, Counts *, int64_t,
                                          int, int32_t *, hipStream_t);
template hipError_t launch_append<float>(Parts<float>, Parts<float>, int, Chunks, int,
                                         const ChildRec *, const FixRec *, Counts *, int64_t, int,
                                         int32_t *, hipStream_t);
template hipError_t launch_resize<double>(Parts<double>, Counts *, Chunks, CloneRec *, int, double,
                                          double, int64_t, int32_t *, hipStream_t);
template hipError_t launch_resize<float>(Parts<float>, Counts *, Chunks, CloneRec *, int, double,
                                         double, int64_t, int32_t *, hipStream_t);

}  // namespace rz
