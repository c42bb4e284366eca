// Device bodies of the list maintenance shared by its own launches
// (fixup.hip) and by the launches that run them beside the next step's grid
// preparation (mg.hip): block sums, the superchunk scan and the dead lists.
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

}  // namespace rz
