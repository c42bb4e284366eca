// Deterministic list maintenance after a particle pass: per-chunk counts are
// scanned in chunk order, absorbed particles leave holes that are filled in
// increasing order by the live particles of the tail, and new particles are
// appended in parent order with consecutive identities.  The resulting array
// does not depend on the launch shape or on the order atomics land in.
#include "device.h"

namespace rz {

__device__ __forceinline__ int count_of(const int32_t *in, int64_t i) { return in[i]; }
__device__ __forceinline__ int count_of(const unsigned long long *in, int64_t i)
{
    return __popcll(in[i]);
}

// Exclusive scan of the counts of in[0..n) (ints, or the set bits of lane
// masks) into out[] by one block of 1024 threads, 8 consecutive items per
// thread per tile; returns the total.
template <typename C>
__device__ int64_t block_scan_tiles(const C *in, int64_t *out, int64_t n, int *sh)
{
    constexpr int kItems = 8;
    int64_t carry = 0;
    const int64_t tile = (int64_t)blockDim.x * kItems;
    for (int64_t base = 0; base < n; base += tile) {
        const int64_t i0 = base + (int64_t)threadIdx.x * kItems;
        int v[kItems];
        int sum = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            v[k] = i0 + k < n ? count_of(in, i0 + k) : 0;
            sum += v[k];
        }
        int tot;
        int ex = block_excl_sum(sum, tot, sh);
        int64_t run = carry + ex;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (i0 + k < n) out[i0 + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    return carry;
}

__global__ __launch_bounds__(1024) void k_scan(ScanJobs j)
{
    __shared__ int sh[64];
    if (blockIdx.x == 0) {
        if (!j.children) return;
        const int64_t nch = (j.crec->n_parent + kChunk - 1) / kChunk;
        int64_t ev = block_scan_tiles(j.ech.ev, j.ech.ev_off, nch, sh);
        int64_t se = block_scan_tiles(j.ech.se, j.ech.se_off, nch, sh);
        int64_t si = block_scan_tiles(j.ech.si, j.ech.si_off, nch, sh);
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
    const int64_t nch = (n + kChunk - 1) / kChunk;
    int64_t d = block_scan_tiles(j.ch[s].dead, j.ch[s].dead_off, nch, sh);
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
template <typename T> __global__ __launch_bounds__(256) void k_dead_scan(const T *w, const Counts *cnt, Chunks ch)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t n = cnt->n;
    const int64_t nch = (n + kChunk - 1) / kChunk;
    for (int64_t c = wave; c < nch; c += nwaves) {
        int64_t i = c * kChunk + lane;
        unsigned long long dm = __ballot(i < n && w[i] < (T)0);
        if (lane == 0) ch.dead[c] = dm;
    }
}

template <typename T>
hipError_t launch_dead_scan(Parts<T> p, const Counts *cnt, Chunks ch, hipStream_t st)
{
    hipLaunchKernelGGL((k_dead_scan<T>), dim3(1024), dim3(256), 0, st, p.w, cnt, ch);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_dead_list(Chunks ch, const FixRec *fix)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nch = (fix->n_old + kChunk - 1) / kChunk;
    if (fix->dead == 0) return;
    const unsigned long long below = (1ull << lane) - 1;
    for (int64_t c = wave; c < nch; c += nwaves) {
        unsigned long long dm = ch.dead[c];
        if ((dm >> lane) & 1)
            ch.dead_glob[ch.dead_off[c] + __popcll(dm & below)] = c * kChunk + lane;
    }
}

hipError_t launch_dead_list(Chunks ch, const FixRec *fix, hipStream_t st)
{
    hipLaunchKernelGGL(k_dead_list, dim3(1024), dim3(256), 0, st, ch, fix);
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
__global__ __launch_bounds__(256) void k_append(Parts<T> dst, Parts<T> stage, int cs, Chunks ech,
                                                int children, const ChildRec *crec,
                                                const FixRec *fix, Counts *cnt, int64_t cap,
                                                int32_t *status)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t keep = fix->keep;
    if (children) {
        const int64_t *surv_off = cs == 0 ? ech.se_off : ech.si_off;
        const unsigned long long *alive = cs == 0 ? ech.se : ech.si;
        const uint64_t id0 = crec->next_id_old[cs];
        const int64_t nch = (crec->n_parent + kChunk - 1) / kChunk;
        const unsigned long long below = (1ull << lane) - 1;
        for (int64_t c = wave; c < nch; c += nwaves) {
            const unsigned long long am = alive[c];
            if (!((am >> lane) & 1)) continue;
            const int64_t slot = c * kChunk + lane;
            const int64_t to = keep + surv_off[c] + __popcll(am & below);
            if (to < cap) {
                dst.r[to] = stage.r[slot];
                dst.z[to] = stage.z[slot];
                dst.vr[to] = stage.vr[slot];
                dst.vt[to] = stage.vt[slot];
                dst.vz[to] = stage.vz[slot];
                dst.ar[to] = stage.ar[slot];
                dst.az[to] = stage.az[slot];
                dst.w[to] = stage.w[slot];
                dst.id[to] = id0 + (uint64_t)(ech.ev_off[c] + __popcll(ech.ev[c] & below));
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
                         int32_t *status, hipStream_t st)
{
    hipLaunchKernelGGL((k_append<T>), dim3(children ? 1024 : 1), dim3(256), 0, st, dst, stage, cs,
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
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t n = cnt->n;
    const int64_t nch = (n + kChunk - 1) / kChunk;
    for (int64_t c = wave; c < nch; c += nwaves) {
        int64_t i = c * kChunk + lane;
        int nc = 0;
        if (i < n) {
            double wr;
            nc = clones_of((double)p.w[i], (double)p.r[i], wcoef, half_hr, wr);
            ch.pcount[i] = nc;
        }
        int tot;
        wave_excl_sum(nc, tot);
        if (lane == 0) ch.clone_cnt[c] = tot;
    }
}

__global__ __launch_bounds__(1024) void k_resize_scan(const Counts *cnt, Chunks ch, CloneRec *rec,
                                                      int64_t cap)
{
    __shared__ int sh[64];
    const int64_t n = cnt->n;
    const int64_t nch = (n + kChunk - 1) / kChunk;
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
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t n = rec->n_old;
    if (!rec->ok) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, kStCapacity);
        return;
    }
    const int64_t nch = (n + kChunk - 1) / kChunk;
    for (int64_t c = wave; c < nch; c += nwaves) {
        int64_t i = c * kChunk + lane;
        int nc = i < n ? ch.pcount[i] : 0;
        int tot;
        int ex = wave_excl_sum(nc, tot);
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
hipError_t launch_resize(Parts<T> p, Counts *cnt, Chunks ch, CloneRec *rec, double wcoef,
                         double half_hr, int64_t cap, int32_t *status, hipStream_t st)
{
    hipLaunchKernelGGL((k_resize_count<T>), dim3(1024), dim3(256), 0, st, p, cnt, ch, wcoef,
                       half_hr);
    hipLaunchKernelGGL(k_resize_scan, dim3(1), dim3(1024), 0, st, cnt, ch, rec, cap);
    hipLaunchKernelGGL((k_resize_scatter<T>), dim3(1024), dim3(256), 0, st, p, cnt, ch, rec,
                       wcoef, half_hr, status);
    return hipGetLastError();
}

// acc[g] += sum over blocks of the per-block LDS copies: block (x, y) sums
// slices y, y + gridDim.y, ... of nodes [256x, 256x + 256) and adds the
// (integer) partial sum atomically.
__global__ __launch_bounds__(256) void k_reduce_slices(unsigned long long *acc,
                                                       const unsigned long long *slices, int nb,
                                                       int nn)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nn) return;
    unsigned long long s = 0;
    for (int b = blockIdx.y; b < nb; b += gridDim.y) s += slices[(size_t)b * nn + g];
    atomicAdd(acc + g, s);
}

hipError_t launch_reduce_slices(unsigned long long *acc, const unsigned long long *slices, int nb,
                                int nn, hipStream_t st)
{
    int threads = 256;
    int bx = (nn + threads - 1) / threads;
    int by = nb < 32 ? nb : 32;
    hipLaunchKernelGGL(k_reduce_slices, dim3(bx, by), dim3(threads), 0, st, acc, slices, nb, nn);
    return hipGetLastError();
}

template hipError_t launch_dead_scan<double>(Parts<double>, const Counts *, Chunks, hipStream_t);
template hipError_t launch_dead_scan<float>(Parts<float>, const Counts *, Chunks, hipStream_t);
template hipError_t launch_fill<double>(Parts<double>, Chunks, const FixRec *, hipStream_t);
template hipError_t launch_fill<float>(Parts<float>, Chunks, const FixRec *, hipStream_t);
template hipError_t launch_append<double>(Parts<double>, Parts<double>, int, Chunks, int,
                                          const ChildRec *, const FixRec *, Counts *, int64_t,
                                          int32_t *, hipStream_t);
template hipError_t launch_append<float>(Parts<float>, Parts<float>, int, Chunks, int,
                                         const ChildRec *, const FixRec *, Counts *, int64_t,
                                         int32_t *, hipStream_t);
template hipError_t launch_resize<double>(Parts<double>, Counts *, Chunks, CloneRec *, double,
                                          double, int64_t, int32_t *, hipStream_t);
template hipError_t launch_resize<float>(Parts<float>, Counts *, Chunks, CloneRec *, double,
                                         double, int64_t, int32_t *, hipStream_t);

}  // namespace rz
