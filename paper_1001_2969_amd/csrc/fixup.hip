// Deterministic list maintenance after a particle pass: per-chunk counts are
// scanned in chunk order, absorbed particles leave holes that are filled in
// increasing order by the live particles of the tail, and new particles are
// appended in parent order with consecutive identities.  The resulting array
// does not depend on the launch shape or on the order atomics land in.
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

// Hole m (the m-th dead index below keep) receives the m-th live particle of
// [keep, n).  With T_k the dead indices >= keep (sorted), that particle is
// keep + m + k for the smallest k whose T_k lies beyond it.
template <typename T>
__device__ __forceinline__ void fill_body(const Blk &kb, const Parts<T> &p, const int64_t *dead,
                                          const FixRec *fix)
{
    const int64_t D = fix->dead, keep = fix->keep;
    if (D == 0) return;
    const int64_t H = wave_lower_bound(dead, D, keep);  // dead indices < keep
    for (int64_t m = kb.x * (int64_t)blockDim.x + threadIdx.x; m < H;
         m += (int64_t)kb.nx * blockDim.x) {
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
        if (p.at) p.at[dst] = p.at[src];
    }
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

// Both species in one launch (the block row selects the species).
template <typename T> struct Fill2Args {
    Parts<T> p[2];
    const int64_t *dead[2];
    const FixRec *fix[2];
};

template <typename T> __device__ __forceinline__ void fill2_body(const Blk &k, const Fill2Args<T> &a)
{
    fill_body<T>(k, a.p[k.y], a.dead[k.y], a.fix[k.y]);
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

// Append of the staged children of species blockIdx.y after its kept
// particles: the survivor and event offsets of each electron chunk come from
// the superchunk prefix and an in-block scan; slot = parent index, identity =
// next identity + event rank.  Block (0, cs) commits the count and identity.
template <typename T> struct AppendArgs {
    Parts<T> dst[2], stage[2];
    Counts *cnt[2];
};

template <typename T> struct AppendJob {
    ScanJobs j;
    AppendArgs<T> g;
};

template <typename T> __device__ __forceinline__ void append_body(const Blk &kb, const AppendJob<T> &aj)
{
    __shared__ int sh[64];
    __shared__ int64_t sh64[16];
    const ScanJobs &j = aj.j;
    const AppendArgs<T> &g = aj.g;
    const int cs = kb.y;
    if (!j.dead[cs]) return;
    const int64_t sc = kb.x;
    const int64_t keep = j.fix[cs]->keep;
    const int64_t cap = j.cap[cs];
    const bool kids = j.kids[cs] != 0;
    int64_t nch = 0, nsc = 0;
    const int32_t *sc_alive = cs == 0 ? j.ech.sc_se : j.ech.sc_si;
    if (kids) {
        nch = (j.crec->n_parent + kChunk - 1) / kChunk;
        nsc = (nch + kSuper - 1) / kSuper;
    }
    // this chunk's masks, loaded before the prefix sums (whose barriers
    // would otherwise hold them back)
    const unsigned long long *alive = cs == 0 ? j.ech.se : j.ech.si;
    const int64_t c = sc * kSuper + threadIdx.x;
    const bool inc = kids && sc < nsc && c < nch;
    const unsigned long long am = inc ? alive[c] : 0ull;
    const unsigned long long em = inc ? j.ech.ev[c] : 0ull;
    if (sc == 0) {
        int64_t surv = 0, evs = 0;
        if (kids) prefix2_of(sc_alive, j.ech.sc_ev, nsc, sh64, surv, evs);
        if (threadIdx.x == 0) {
            const int64_t room = cap - keep;
            if (surv > room) {
                atomicOr(j.status, kStCapacity);
                surv = room;
            }
            g.cnt[cs]->n = keep + surv;
            if (kids) g.cnt[cs]->next_id = j.crec->next_id_old[cs] + (uint64_t)evs;
        }
    }
    if (!kids || sc >= nsc) return;
    int64_t sbase, ebase;
    prefix2_of(sc_alive, j.ech.sc_ev, sc, sh64, sbase, ebase);
    // both in-block scans in one: survivors in the low 16 bits (at most
    // 512 x 64 in a superchunk), events above (whose superchunk total, from
    // the scan, must stay below 2^15 for the packed int; else two scans)
    int tot;
    int64_t soff, eoff;
    if (j.ech.sc_ev[sc] < 32768) {
        const int both = block_excl_sum(__popcll(am) | (__popcll(em) << 16), tot, sh);
        soff = sbase + (both & 0xFFFF);
        eoff = ebase + (both >> 16);
    } else {
        soff = sbase + block_excl_sum(__popcll(am), tot, sh);
        eoff = ebase + block_excl_sum(__popcll(em), tot, sh);
    }
    const uint64_t id0 = j.crec->next_id_old[cs];
    const Parts<T> &dst = g.dst[cs], &stage = g.stage[cs];
    unsigned long long m = am;
    int64_t k = 0;
    while (m) {
        const int lane = __ffsll((long long)m) - 1;
        m &= m - 1;
        const int64_t slot = c * kChunk + lane;
        const int64_t to = keep + soff + k++;
        if (to >= cap) continue;
        dst.r[to] = stage.r[slot];
        dst.z[to] = stage.z[slot];
        dst.vr[to] = stage.vr[slot];
        dst.vt[to] = stage.vt[slot];
        dst.vz[to] = stage.vz[slot];
        dst.ar[to] = stage.ar[slot];
        dst.az[to] = stage.az[slot];
        dst.w[to] = stage.w[slot];
        if (dst.at) dst.at[to] = stage.at[slot];
        dst.id[to] = id0 + (uint64_t)(eoff + __popcll(em & ((1ull << lane) - 1)));
    }
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
