// Device bodies of the list maintenance shared by its own launches
// (fixup.hip) and by the launches that run them beside the multigrid's
// (mg.hip, step pipelining): block sums, the superchunk scan, the dead
// lists, the hole filling and the appending of new particles.
#pragma once

#include "device.h"

namespace rz {

// Sum over the block of one value per thread (all threads must call).
__device__ __forceinline__ int64_t block_sum64(int64_t v, int64_t *sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    int64_t t = 0;
    for (int w = 0; w < nw; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// Sum of sc[0..upto) by the whole block.
__device__ __forceinline__ int64_t prefix_of(const int32_t *sc, int64_t upto, int64_t *sh)
{
    int64_t v = 0;
    for (int64_t k = threadIdx.x; k < upto; k += blockDim.x) v += sc[k];
    return block_sum64(v, sh);
}

// Sums of a[0..upto) and b[0..upto) by the whole block in one reduction:
// the two (non-negative, each total below 2^32) packed in one 64-bit word.
__device__ __forceinline__ void prefix2_of(const int32_t *a, const int32_t *b, int64_t upto,
                                           int64_t *sh, int64_t &sa, int64_t &sb)
{
    uint64_t v = 0;
    for (int64_t k = threadIdx.x; k < upto; k += blockDim.x)
        v += (uint64_t)(uint32_t)a[k] | ((uint64_t)(uint32_t)b[k] << 32);
    const uint64_t t = (uint64_t)block_sum64((int64_t)v, sh);
    sa = (int64_t)(t & 0xFFFFFFFFull);
    sb = (int64_t)(t >> 32);
}

// Entries of the sorted a[0..D) below x, found by the whole wavefront: each
// round probes 64 evenly spaced entries of the remaining range at once, so
// that a range of D entries takes about log64(D) dependent loads instead of
// log2(D).  Every lane returns the same count.
__device__ __forceinline__ int64_t wave_lower_bound(const int64_t *a, int64_t D, int64_t x)
{
    const int lane = threadIdx.x & 63;
    int64_t lo = 0, hi = D;  // the count lies in [lo, hi]
    while (lo < hi) {
        const int64_t len = hi - lo;
        if (len <= 64) {
            const bool t = lane < len && a[lo + lane] < x;
            return lo + __popcll(__ballot(t));
        }
        const int64_t pk = lo + ((int64_t)(lane + 1) * len) / 64 - 1;  // pk(63) = hi - 1
        const int cnt = __popcll(__ballot(a[pk] < x));
        const int64_t pl = lo + ((int64_t)cnt * len) / 64 - 1;        // the last probe below x
        const int64_t ph = lo + ((int64_t)(cnt + 1) * len) / 64 - 1;  // the first at or above
        if (cnt > 0) lo = pl + 1;
        if (cnt < 64) hi = ph;
    }
    return lo;
}

// Superchunk totals: block (sc, 0) sums the children masks of its 512
// electron chunks, blocks (sc, 1 + s) the dead masks of species s.
__device__ __forceinline__ void scan_body(const Blk &k, const ScanJobs &j)
{
    __shared__ int sh[64];
    const int job = k.y;
    const int64_t sc = k.x;
    const int64_t c = sc * kSuper + threadIdx.x;
    int tot;
    if (job == 0) {
        if (!j.children) return;
        if (sc == 0 && threadIdx.x == 0) {
            j.crec->next_id_old[0] = j.ecnt->next_id;
            j.crec->next_id_old[1] = j.icnt->next_id;
        }
        const int64_t nch = (j.crec->n_parent + kChunk - 1) / kChunk;
        if (sc * kSuper >= nch) return;
        const bool in = c < nch;
        block_excl_sum(in ? __popcll(j.ech.ev[c]) : 0, tot, sh);
        if (threadIdx.x == 0) j.ech.sc_ev[sc] = tot;
        block_excl_sum(in ? __popcll(j.ech.se[c]) : 0, tot, sh);
        if (threadIdx.x == 0) j.ech.sc_se[sc] = tot;
        block_excl_sum(in ? __popcll(j.ech.si[c]) : 0, tot, sh);
        if (threadIdx.x == 0) j.ech.sc_si[sc] = tot;
        return;
    }
    const int s = job - 1;
    if (!j.dead[s]) return;
    const int64_t nch = (j.cnt[s]->n + kChunk - 1) / kChunk;
    if (sc * kSuper >= nch && sc > 0) return;
    block_excl_sum(c < nch ? __popcll(j.ch[s].dead[c]) : 0, tot, sh);
    if (threadIdx.x == 0) j.ch[s].sc_dead[sc] = tot;
}

// Sorted dead list of species blockIdx.y: superchunk prefix + the in-block
// scan of the chunk counts give each chunk's offset; its set lanes follow in
// increasing order.  Block (0, s) records n, the dead total and the kept count.
__device__ __forceinline__ void dead_list_body(const Blk &k, const ScanJobs &j)
{
    __shared__ int sh[64];
    __shared__ int64_t sh64[16];
    const int s = k.y;
    if (!j.dead[s]) return;
    const int64_t sc = k.x;
    const int64_t n = j.cnt[s]->n;
    const int64_t nch = (n + kChunk - 1) / kChunk;
    const int64_t nsc = (nch + kSuper - 1) / kSuper;
    const Chunks &ch = j.ch[s];
    if (sc == 0) {
        int64_t D = prefix_of(ch.sc_dead, nsc, sh64);
        if (threadIdx.x == 0) {
            j.fix[s]->n_old = n;
            j.fix[s]->dead = D;
            j.fix[s]->keep = n - D;
        }
    }
    if (sc >= nsc) return;
    const int64_t c = sc * kSuper + threadIdx.x;
    unsigned long long m = c < nch ? ch.dead[c] : 0ull;
    const int64_t base = prefix_of(ch.sc_dead, sc, sh64);
    int tot;
    int64_t off = base + block_excl_sum(__popcll(m), tot, sh);
    while (m) {
        int lane = __ffsll((long long)m) - 1;
        ch.dead_glob[off++] = c * kChunk + lane;
        m &= m - 1;
    }
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


}  // namespace rz
