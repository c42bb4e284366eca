// Stable counting sort of a species' particles by spatial tile, and the plan
// of the tiled particle pass built from it.
//
// The key of a particle is the tile of its cell (floor(z / hz), floor(r / hr)),
// clamped to the mesh, with tiles of tile_z x tile_r cells numbered r fastest.
// (The paper orders particles by cell to speed up the weighting, Sec. 2.7.)
// Within a tile the array order is kept, so the result is the unique stable
// order and the identities of later new particles, which follow the array
// order, do not depend on the launch shape.
//
// Work split: a segment of `seg` consecutive particles is one wavefront.
//   count   per segment and tile, key-major: off[k * nseg + g]
//   scan    exclusive prefix over off (three launches)
//   scatter each wavefront walks its segment 64 particles at a time; lanes
//           with equal keys are matched by ballots over the key bits, ranked
//           by lane, and written to off[k] + rank of the sorted copy
//   copy    the sorted copy back into the caller's arrays
//   plan    the particle range of each pass block and its deposit window
#include "device.h"

namespace rz {

namespace {

constexpr int kSortThreads = 256;  // four segments per block
constexpr int kScanThreads = 256, kScanPer = 16, kScanBlock = kScanThreads * kScanPer;

template <typename T>
__device__ __forceinline__ int tile_of(const SortArgs<T> &a, T r, T z)
{
    double fi = floor((double)z / a.hz), fj = floor((double)r / a.hr);
    const double imax = (double)(a.nz - 2), jmax = (double)(a.nr - 2);
    fi = fi >= 0.0 ? (fi <= imax ? fi : imax) : 0.0;
    fj = fj >= 0.0 ? (fj <= jmax ? fj : jmax) : 0.0;
    const int i = (int)fi, j = (int)fj;
    return (i / a.tile_z) * a.ntr + j / a.tile_r;
}

// Lanes of the wavefront that are valid and carry the same key as this lane.
__device__ __forceinline__ unsigned long long key_match(int key, bool valid, int kbits)
{
    unsigned long long m = __ballot(valid);
    for (int b = 0; b < kbits; ++b) {
        const bool bit = (key >> b) & 1;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

template <typename T> __global__ __launch_bounds__(kSortThreads) void k_sort_count(SortArgs<T> a)
{
    extern __shared__ int32_t sh_cnt[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * (kSortThreads / 64) + w;
    int32_t *cnt = sh_cnt + w * a.nt;
    for (int k = lane; k < a.nt; k += 64) cnt[k] = 0;
    __syncthreads();
    if (g < a.nseg) {
        const int64_t n = a.cnt->n;
        const int64_t p0 = g * a.seg;
        const int64_t p1 = p0 + a.seg < n ? p0 + a.seg : n;
        for (int64_t q = p0; q < p1; q += 64) {
            const int64_t p = q + lane;
            const bool valid = p < p1;
            const int key = valid ? tile_of(a, a.p.r[p], a.p.z[p]) : 0;
            const unsigned long long m = key_match(key, valid, a.kbits);
            if (valid && lane_rank(m) == 0) cnt[key] += __popcll(m);
        }
        for (int k = lane; k < a.nt; k += 64) a.off[(int64_t)k * a.nseg + g] = cnt[k];
    }
}

// Exclusive prefix of v over the block (kScanThreads threads) and the total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t &total)
{
    __shared__ int64_t sh_w[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) sh_w[w] = x;
    __syncthreads();
    int64_t before = 0;
    total = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) {
        if (k < w) before += sh_w[k];
        total += sh_w[k];
    }
    __syncthreads();
    return before + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sum(const int64_t *x, int64_t M,
                                                            int64_t *part)
{
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    int64_t v = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = b0 + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < M) v += x[i];
    }
    int64_t tot;
    block_excl_scan(v, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Exclusive prefix of part[0, nb), nb <= kScanBlock, in one block.
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int64_t *part, int nb)
{
    int64_t v[kScanPer];
    int64_t s = 0;
    const int base = threadIdx.x * kScanPer;
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < nb ? part[base + k] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t run = block_excl_scan(s, tot);
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < nb) part[base + k] = run;
        run += v[k];
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int64_t *x, int64_t M,
                                                              const int64_t *part)
{
    // each thread takes kScanPer consecutive elements of the block's range
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    int64_t v[kScanPer];
    int64_t s = 0;
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < M ? x[base + k] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t run = block_excl_scan(s, tot) + part[blockIdx.x];
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < M) x[base + k] = run;
        run += v[k];
    }
}

template <typename T>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(SortArgs<T> a)
{
    extern __shared__ int64_t sh_next[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * (kSortThreads / 64) + w;
    int64_t *next = sh_next + w * a.nt;
    if (g < a.nseg)
        for (int k = lane; k < a.nt; k += 64) next[k] = a.off[(int64_t)k * a.nseg + g];
    __syncthreads();
    if (g >= a.nseg) return;
    const int64_t n = a.cnt->n;
    const int64_t p0 = g * a.seg;
    const int64_t p1 = p0 + a.seg < n ? p0 + a.seg : n;
    for (int64_t q = p0; q < p1; q += 64) {
        const int64_t p = q + lane;
        const bool valid = p < p1;
        T r = 0, z = 0;
        if (valid) {
            r = a.p.r[p];
            z = a.p.z[p];
        }
        const int key = valid ? tile_of(a, r, z) : 0;
        const unsigned long long m = key_match(key, valid, a.kbits);
        const int rank = lane_rank(m);
        int64_t base = 0;
        if (valid) base = next[key];
        // one lane per key advances the key's next slot (read above first)
        if (valid && rank == 0) next[key] = base + __popcll(m);
        if (valid) {
            const int64_t d = base + rank;
            a.tmp.r[d] = r;
            a.tmp.z[d] = z;
            a.tmp.vr[d] = a.p.vr[p];
            a.tmp.vt[d] = a.p.vt[p];
            a.tmp.vz[d] = a.p.vz[p];
            a.tmp.ar[d] = a.p.ar[p];
            a.tmp.az[d] = a.p.az[p];
            a.tmp.w[d] = a.p.w[p];
            a.tmp.id[d] = a.p.id[p];
            if (a.p.at) a.tmp.at[d] = a.p.at[p];
        }
    }
}

template <typename T> __global__ void k_sort_copy(SortArgs<T> a)
{
    const int64_t n = a.cnt->n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        a.p.r[i] = a.tmp.r[i];
        a.p.z[i] = a.tmp.z[i];
        a.p.vr[i] = a.tmp.vr[i];
        a.p.vt[i] = a.tmp.vt[i];
        a.p.vz[i] = a.tmp.vz[i];
        a.p.ar[i] = a.tmp.ar[i];
        a.p.az[i] = a.tmp.az[i];
        a.p.w[i] = a.tmp.w[i];
        a.p.id[i] = a.tmp.id[i];
        if (a.p.at) a.p.at[i] = a.tmp.at[i];
    }
}

// Plan of the tiled pass: nb blocks take ranges of P particles (P a multiple
// of kChunk, nb * P >= n).  A block's window covers the tiles of its range in
// the row of tiles holding most of it, widened by a drift margin of up to
// kWinHalo cells and clipped to the mesh; within kWinNodes nodes.
template <typename T> __global__ void k_tile_plan(SortArgs<T> a)
{
    const int64_t n = a.cnt->n;
    const int nb = a.nb;
    int64_t P = (n + nb - 1) / nb;
    P = (P + kChunk - 1) / kChunk * kChunk;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.tile_pb = P;
    const int lb = blockIdx.x * blockDim.x + threadIdx.x;
    if (lb >= nb) return;
    int4 win = make_int4(0, 0, 0, 0);
    const int64_t lo = (int64_t)lb * P;
    const int64_t hi = lo + P < n ? lo + P : n;
    if (lo < hi) {
        // first particle of tile k (tile k occupies [start(k), start(k + 1)))
        auto start = [&](int k) -> int64_t { return k >= a.nt ? n : a.off[(int64_t)k * a.nseg]; };
        auto tile_at = [&](int64_t p) {  // the last tile starting at or before p
            int l = 0, h = a.nt - 1;
            while (l < h) {
                const int mid = (l + h + 1) / 2;
                if (start(mid) <= p) l = mid;
                else h = mid - 1;
            }
            return l;
        };
        const int t0 = tile_at(lo), t1 = tile_at(hi - 1);
        int row = t0 / a.ntr;
        int64_t most = -1;
        for (int rz = t0 / a.ntr; rz <= t1 / a.ntr; ++rz) {
            int64_t b0 = start(rz * a.ntr), b1 = start((rz + 1) * a.ntr);
            b0 = b0 > lo ? b0 : lo;
            b1 = b1 < hi ? b1 : hi;
            if (b1 - b0 > most) {
                most = b1 - b0;
                row = rz;
            }
        }
        const int ta = t0 > row * a.ntr ? t0 : row * a.ntr;
        const int tb = t1 < row * a.ntr + a.ntr - 1 ? t1 : row * a.ntr + a.ntr - 1;
        // cells [cz0, cz1) x [cr0, cr1) of those tiles
        const int cz0 = row * a.tile_z;
        const int cz1 = (row + 1) * a.tile_z < a.nz - 1 ? (row + 1) * a.tile_z : a.nz - 1;
        const int cr0 = (ta % a.ntr) * a.tile_r;
        const int cr1 = (tb % a.ntr + 1) * a.tile_r < a.nr - 1 ? (tb % a.ntr + 1) * a.tile_r
                                                                : a.nr - 1;
        for (int h = kWinHalo;; h >>= 1) {
            const int z0 = cz0 - h > 0 ? cz0 - h : 0;
            const int z1 = cz1 + h < a.nz - 1 ? cz1 + h : a.nz - 1;
            const int r0 = cr0 - h > 0 ? cr0 - h : 0;
            const int r1 = cr1 + h < a.nr - 1 ? cr1 + h : a.nr - 1;
            const int ni = z1 - z0 + 1, nj = r1 - r0 + 1;  // nodes
            if (ni * nj <= kWinNodes) {
                win = make_int4(z0, r0, ni, nj);
                break;
            }
            if (h == 0) {
                // tiles larger than a window: the middle columns of the range
                const int njm = kWinNodes / ni;
                if (njm >= 2) {
                    int s0 = (r0 + r1) / 2 - (njm - 1) / 2;
                    s0 = s0 < a.nr - njm ? s0 : a.nr - njm;
                    s0 = s0 > 0 ? s0 : 0;
                    win = make_int4(z0, s0, ni, njm);
                }
                break;
            }
        }
    }
    a.tile_win[lb] = win;
}

}  // namespace

template <typename T> hipError_t launch_sort(const SortArgs<T> &a, hipStream_t st)
{
    if (a.nt < 1 || a.nt > kMaxTiles || a.nb < 1 || a.nb > kMaxWaves) return hipErrorInvalidValue;
    const int64_t M = (int64_t)a.nt * a.nseg;
    const int64_t nbk = (M + kScanBlock - 1) / kScanBlock;
    if (nbk > kScanBlock || nbk > 4096) return hipErrorInvalidValue;
    const int blocks = (int)((a.nseg + kSortThreads / 64 - 1) / (kSortThreads / 64));
    RZ_LAUNCH(k_sort_count<T>, dim3(blocks), dim3(kSortThreads),
                       (size_t)(kSortThreads / 64) * a.nt * sizeof(int32_t), st, a);
    RZ_LAUNCH(k_scan_sum, dim3((unsigned)nbk), dim3(kScanThreads), 0, st, a.off, M,
                       a.part);
    RZ_LAUNCH(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, a.part, (int)nbk);
    RZ_LAUNCH(k_scan_apply, dim3((unsigned)nbk), dim3(kScanThreads), 0, st, a.off, M,
                       a.part);
    RZ_LAUNCH(k_sort_scatter<T>, dim3(blocks), dim3(kSortThreads),
                       (size_t)(kSortThreads / 64) * a.nt * sizeof(int64_t), st, a);
    const int64_t span = a.nseg * a.seg;
    const int cblocks = (int)((span + 255) / 256 < 8192 ? (span + 255) / 256 : 8192);
    RZ_LAUNCH(k_sort_copy<T>, dim3(cblocks), dim3(256), 0, st, a);
    RZ_LAUNCH(k_tile_plan<T>, dim3((a.nb + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

template hipError_t launch_sort<double>(const SortArgs<double> &, hipStream_t);
template hipError_t launch_sort<float>(const SortArgs<float> &, hipStream_t);

}  // namespace rz
