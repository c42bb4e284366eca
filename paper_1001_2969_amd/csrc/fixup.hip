// Deterministic list maintenance after a particle pass: per-chunk counts are
// scanned in chunk order, absorbed particles leave holes that are filled in
// increasing order by the live particles of the tail, and new particles are
// appended in parent order with consecutive identities.  The resulting array
// does not depend on the launch shape or on the order atomics land in.
#include <cstring>

#include "device.h"
#include "lists.h"

namespace rz {

// Exclusive scan of in[0..n) into out[] by one block of 1024 threads, 8
// consecutive items per thread per tile; returns the total (weight split).
__device__ int64_t block_scan_tiles(const int32_t *in, int64_t *out, int64_t n, int *sh)
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
            v[k] = i0 + k < n ? in[i0 + k] : 0;
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

hipError_t launch_scan(const ScanJobs &j, int64_t max_chunks, hipStream_t st)
{
    int64_t nsc = (max_chunks + kSuper - 1) / kSuper;
    if (nsc < 1) nsc = 1;
    return launch<ScanJobs, scan_body, kSuper>(dim3((unsigned)nsc, 3), dim3(kSuper), 0, st, j);
}

hipError_t launch_dead_list(const ScanJobs &j, int64_t max_chunks, hipStream_t st)
{
    int64_t nsc = (max_chunks + kSuper - 1) / kSuper;
    if (nsc < 1) nsc = 1;
    return launch<ScanJobs, dead_list_body, kSuper>(dim3((unsigned)nsc, 2), dim3(kSuper), 0, st, j);
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
    RZ_LAUNCH((k_dead_scan<T>), dim3(1024), dim3(256), 0, st, p.w, cnt, ch);
    return hipGetLastError();
}

template <typename T> __global__ void k_fill(Parts<T> p, const int64_t *dead, const FixRec *fix)
{
    fill_body<T>(Blk{(int)blockIdx.x, 0, (int)gridDim.x, 1}, p, dead, fix);
}

template <typename T>
hipError_t launch_fill(Parts<T> p, Chunks ch, const FixRec *fix, hipStream_t st)
{
    RZ_LAUNCH((k_fill<T>), dim3(256), dim3(256), 0, st, p, ch.dead_glob, fix);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill2(Parts<T> p0, Parts<T> p1, Chunks ch0, Chunks ch1, const FixRec *fix0,
                        const FixRec *fix1, hipStream_t st)
{
    Fill2Args<T> a;
    a.p[0] = p0;
    a.p[1] = p1;
    a.dead[0] = ch0.dead_glob;
    a.dead[1] = ch1.dead_glob;
    a.fix[0] = fix0;
    a.fix[1] = fix1;
    return launch<Fill2Args<T>, fill2_body<T>, 256>(dim3(256, 2), dim3(256), 0, st, a);
}

template <typename T>
hipError_t launch_append(const ScanJobs &j, Parts<T> dst0, Parts<T> dst1, Parts<T> stage0,
                         Parts<T> stage1, Counts *cnt0, Counts *cnt1, int64_t max_chunks,
                         hipStream_t st)
{
    AppendArgs<T> g;
    g.dst[0] = dst0;
    g.dst[1] = dst1;
    g.stage[0] = stage0;
    g.stage[1] = stage1;
    g.cnt[0] = cnt0;
    g.cnt[1] = cnt1;
    int64_t nsc = (max_chunks + kSuper - 1) / kSuper;
    if (nsc < 1) nsc = 1;
    return launch<AppendJob<T>, append_body<T>, kSuper>(dim3((unsigned)nsc, 2), dim3(kSuper), 0, st,
                                                        AppendJob<T>{j, g});
}

template <typename T>
void list_tail_keep(ListTail &t, Parts<T> p0, Parts<T> p1, Chunks ch0, Chunks ch1,
                    const FixRec *fix0, const FixRec *fix1, const ScanJobs &j, Parts<T> dst0,
                    Parts<T> dst1, Parts<T> stage0, Parts<T> stage1, Counts *cnt0, Counts *cnt1,
                    int64_t max_chunks)
{
    static_assert(sizeof(Fill2Args<T>) <= kTailFillBytes, "fill arguments");
    static_assert(sizeof(AppendJob<T>) <= kTailAppBytes, "append arguments");
    Fill2Args<T> f;
    f.p[0] = p0;
    f.p[1] = p1;
    f.dead[0] = ch0.dead_glob;
    f.dead[1] = ch1.dead_glob;
    f.fix[0] = fix0;
    f.fix[1] = fix1;
    AppendJob<T> a{};
    a.j = j;
    a.g.dst[0] = dst0;
    a.g.dst[1] = dst1;
    a.g.stage[0] = stage0;
    a.g.stage[1] = stage1;
    a.g.cnt[0] = cnt0;
    a.g.cnt[1] = cnt1;
    std::memcpy(t.fill, &f, sizeof f);
    std::memcpy(t.app, &a, sizeof a);
    const int64_t nsc = (max_chunks + kSuper - 1) / kSuper;
    t.nsc = nsc < 1 ? 1 : (int)nsc;
    t.fp32 = sizeof(T) == 4;
    t.stage = 2;
}

template <typename T> static hipError_t tail_flush(ListTail &t, hipStream_t st)
{
    if (t.stage == 2) {
        Fill2Args<T> f;
        std::memcpy(&f, t.fill, sizeof f);
        (void)launch<Fill2Args<T>, fill2_body<T>, 256>(dim3(256, 2), dim3(256), 0, st, f);
        t.stage = 1;
    }
    if (t.stage == 1) {
        AppendJob<T> a;
        std::memcpy(&a, t.app, sizeof a);
        (void)launch<AppendJob<T>, append_body<T>, kSuper>(dim3((unsigned)t.nsc, 2), dim3(kSuper),
                                                            0, st, a);
        t.stage = 0;
    }
    return hipGetLastError();
}

hipError_t list_tail_flush(ListTail &t, hipStream_t st)
{
    if (t.stage == 0) return hipSuccess;
    return t.fp32 ? tail_flush<float>(t, st) : tail_flush<double>(t, st);
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

// Zero-order particle-based resizing (Sec. 2.2): copies kept of a particle of
// weight w at radius r, floor(q) plus one with probability q - floor(q),
// q = w / w_r (first uniform of draw block 6); each copy weighs w_r.
__device__ __forceinline__ int copies_of(double w, double r, double wcoef, double half_hr,
                                         const ResizeKey &k, uint64_t id, double &wr)
{
#pragma clang fp contract(off)
    double rr = r > half_hr ? r : half_hr;
    wr = wcoef * rr;
    double q = w / wr;
    double fl = floor(q);
    double ua, ub;
    uniform2(k.seed, k.s, id, k.step, 6, ua, ub);
    return (int)fl + (ua < q - fl ? 1 : 0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_resize_count(Parts<T> p, const Counts *cnt, Chunks ch,
                                                      ResizeKey key, double wcoef, double half_hr)
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
            if (key.zero_order) {
                const int N = copies_of((double)p.w[i], (double)p.r[i], wcoef, half_hr, key,
                                        p.id[i], wr);
                nc = N > 1 ? N - 1 : 0;
            } else {
                nc = clones_of((double)p.w[i], (double)p.r[i], wcoef, half_hr, wr);
            }
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
                                                        const CloneRec *rec, ResizeKey key,
                                                        double wcoef, double half_hr,
                                                        int32_t *status)
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
        if (i < n && (nc > 0 || key.zero_order)) {
            double wr;
            double w = (double)p.w[i];
            T wpar;
            if (key.zero_order) {  // none kept: marked for the compaction that follows
                const int N = copies_of(w, (double)p.r[i], wcoef, half_hr, key, p.id[i], wr);
                wpar = N == 0 ? (T)-1 : (T)wr;
            } else {
                clones_of(w, (double)p.r[i], wcoef, half_hr, wr);
                wpar = (T)split_rest(w, nc, wr);
            }
            const T r = p.r[i], z = p.z[i], vr = p.vr[i], vt = p.vt[i], vz = p.vz[i];
            const T ar = p.ar[i], az = p.az[i], at = p.at ? p.at[i] : (T)0;
            p.w[i] = wpar;
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
                if (p.at) p.at[d] = at;
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
hipError_t launch_resize(Parts<T> p, Counts *cnt, Chunks ch, CloneRec *rec, const ResizeKey &k,
                         double wcoef, double half_hr, int64_t cap, int32_t *status,
                         hipStream_t st)
{
    RZ_LAUNCH((k_resize_count<T>), dim3(1024), dim3(256), 0, st, p, cnt, ch, k, wcoef,
                       half_hr);
    RZ_LAUNCH(k_resize_scan, dim3(1), dim3(1024), 0, st, cnt, ch, rec, cap);
    RZ_LAUNCH((k_resize_scatter<T>), dim3(1024), dim3(256), 0, st, p, cnt, ch, rec, k,
                       wcoef, half_hr, status);
    return hipGetLastError();
}

// acc[g] += sum over blocks of the per-block LDS copies: block (x, y) sums
// slices y, y + gridDim.y, ... of nodes [256x, 256x + 256) and adds the
// (integer) partial sum atomically.  narrow: 32-bit slice elements.
__global__ __launch_bounds__(256) void k_reduce_slices(unsigned long long *acc, const void *slices,
                                                       int narrow, int nb, int nn)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nn) return;
    unsigned long long s = 0;
    if (narrow) {
        const uint32_t *sl = (const uint32_t *)slices;
        const size_t stride = slice_stride(nn, 1);
        for (int b = blockIdx.y; b < nb; b += gridDim.y) s += sl[(size_t)b * stride + g];
    } else {
        const unsigned long long *sl = (const unsigned long long *)slices;
        for (int b = blockIdx.y; b < nb; b += gridDim.y) s += sl[(size_t)b * nn + g];
    }
    atomicAdd(acc + g, s);
}

hipError_t launch_reduce_slices(unsigned long long *acc, const void *slices, int narrow, int nb,
                                int nn, hipStream_t st)
{
    int threads = 256;
    int bx = (nn + threads - 1) / threads;
    int by = nb < 32 ? nb : 32;
    RZ_LAUNCH(k_reduce_slices, dim3(bx, by), dim3(threads), 0, st, acc, slices, narrow, nb, nn);
    return hipGetLastError();
}

template hipError_t launch_dead_scan<double>(Parts<double>, const Counts *, Chunks, hipStream_t);
template hipError_t launch_dead_scan<float>(Parts<float>, const Counts *, Chunks, hipStream_t);
template void list_tail_keep<double>(ListTail &, Parts<double>, Parts<double>, Chunks, Chunks,
                                    const FixRec *, const FixRec *, const ScanJobs &,
                                    Parts<double>, Parts<double>, Parts<double>, Parts<double>,
                                    Counts *, Counts *, int64_t);
template void list_tail_keep<float>(ListTail &, Parts<float>, Parts<float>, Chunks, Chunks,
                                   const FixRec *, const FixRec *, const ScanJobs &, Parts<float>,
                                   Parts<float>, Parts<float>, Parts<float>, Counts *, Counts *,
                                   int64_t);
template hipError_t launch_fill<double>(Parts<double>, Chunks, const FixRec *, hipStream_t);
template hipError_t launch_fill<float>(Parts<float>, Chunks, const FixRec *, hipStream_t);
template hipError_t launch_fill2<double>(Parts<double>, Parts<double>, Chunks, Chunks,
                                         const FixRec *, const FixRec *, hipStream_t);
template hipError_t launch_fill2<float>(Parts<float>, Parts<float>, Chunks, Chunks, const FixRec *,
                                        const FixRec *, hipStream_t);
template hipError_t launch_append<double>(const ScanJobs &, Parts<double>, Parts<double>,
                                          Parts<double>, Parts<double>, Counts *, Counts *, int64_t,
                                          hipStream_t);
template hipError_t launch_append<float>(const ScanJobs &, Parts<float>, Parts<float>,
                                         Parts<float>, Parts<float>, Counts *, Counts *, int64_t,
                                         hipStream_t);
template hipError_t launch_resize<double>(Parts<double>, Counts *, Chunks, CloneRec *,
                                          const ResizeKey &, double, double, int64_t, int32_t *,
                                          hipStream_t);
template hipError_t launch_resize<float>(Parts<float>, Counts *, Chunks, CloneRec *,
                                         const ResizeKey &, double, double, int64_t, int32_t *,
                                         hipStream_t);

}  // namespace rz
