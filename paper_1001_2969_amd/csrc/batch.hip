// Batched steps of independent discharges.
//
// A batched step records the launches of every discharge's merged step
// (rzpic_step in record mode: the host-side bookkeeping runs, no kernel is
// launched), groups the discharges whose launch sequences are identical
// (same kernels and block shapes: the same mesh, precision and options), and
// replays each group position by position on a stream of its own.  At a
// position whose kernel is written as a body over a virtual block index, one
// launch covers the whole group: a job table gives each discharge its
// arguments and its range of blocks.  Other kernels are launched once per
// discharge.  Every block runs exactly what it runs in the discharge's own
// step, so a batched step equals the separate steps bit for bit.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

#include "rzpic.h"

#include <hip/hip_runtime.h>

#include "internal.h"

namespace rz {
thread_local Recorder *g_recorder = nullptr;
}

using namespace rz;

// Defined in runtime.hip (C ABI helpers shared with the batch).
extern "C" rzpic_status rzpic_step(rzpic_ctx *ctx, int64_t step);
rzpic_status rz_fail(rzpic_status s, const char *msg);
hipStream_t rz_stream(const rzpic_ctx *c);
rzpic_status rz_settle(rzpic_ctx *c);
int rz_batchable(const rzpic_ctx *c, std::string &why);
extern "C" {
void rz_tune_key(const rzpic_ctx *c, int32_t out[5]);
int rz_config_fits(const rzpic_ctx *c, int threads, int64_t ppb, int lds);
rzpic_status rz_set_config(rzpic_ctx *c, int threads, int64_t ppb, int lds, int tz, int tr);
void rz_get_config(const rzpic_ctx *c, int32_t out[5]);
}

namespace {

constexpr int kStreams = 4;  // the device's hardware queues

struct Staging {
    void *host = nullptr;  // pinned
    size_t cap = 0;
    hipEvent_t done = nullptr;  // the upload that last read it
    bool used = false;
    // captured step reading this buffer, and the layout it was captured for
    hipGraphExec_t exec = nullptr;
    std::vector<size_t> layout;
};

}  // namespace

struct rzpic_batch {
    std::vector<rzpic_ctx *> ctx;
    hipStream_t st = nullptr;
    hipStream_t streams[kStreams] = {};
    hipEvent_t fork = nullptr, join[kStreams] = {}, ctx_ev = nullptr;
    Staging stage[2];
    int which = 0;
    void *dev = nullptr;
    size_t dev_cap = 0;
    std::vector<Recorder> rec;
    int nstreams = kStreams;  // streams the groups are spread over
    bool graph = false;       // replay captured steps
    int32_t classes = 0, launches = 0, batched = 0;
};

namespace {

rzpic_status hipfail(hipError_t e, const char *what)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return rz_fail(RZPIC_EHIP, buf);
}

#define BCHK(expr, what)                         \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hipfail(e_, what); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

extern "C" {

rzpic_status rzpic_batch_create(rzpic_ctx *const *ctxs, int32_t n, void *stream, rzpic_batch **out)
{
    if (!ctxs || !out || n < 1) return rz_fail(RZPIC_EINVAL, "batch: need contexts and n >= 1");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return rz_fail(RZPIC_EINVAL, "batch: null context");
        std::string why;
        if (!rz_batchable(ctxs[i], why)) {
            char buf[256];
            std::snprintf(buf, sizeof buf, "batch: context %d: %s", i, why.c_str());
            return rz_fail(RZPIC_EINVAL, buf);
        }
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return rz_fail(RZPIC_EINVAL, "batch: a context appears twice");
    }
    rzpic_batch *b = new rzpic_batch();
    b->ctx.assign(ctxs, ctxs + n);
    b->st = (hipStream_t)stream;
    b->rec.resize(n);
    if (const char *e = std::getenv("RZPIC_BATCH_STREAMS")) {
        const int k = std::atoi(e);
        if (k >= 1 && k <= kStreams) b->nstreams = k;
    }
    auto bail = [&](rzpic_status s) {
        rzpic_batch_destroy(b);
        return s;
    };
    hipError_t e = hipSuccess;
    for (int k = 0; k < kStreams && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&b->streams[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ctx_ev, hipEventDisableTiming);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&b->stage[k].done, hipEventDisableTiming);
    if (e != hipSuccess) return bail(hipfail(e, "batch: stream/event creation"));
    *out = b;
    return RZPIC_OK;
}

rzpic_status rzpic_batch_destroy(rzpic_batch *b)
{
    if (!b) return RZPIC_OK;
    if (b->st) (void)hipStreamSynchronize(b->st);
    for (int k = 0; k < kStreams; ++k) {
        if (b->streams[k]) {
            (void)hipStreamSynchronize(b->streams[k]);
            (void)hipStreamDestroy(b->streams[k]);
        }
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->ctx_ev) (void)hipEventDestroy(b->ctx_ev);
    for (auto &s : b->stage) {
        if (s.exec) (void)hipGraphExecDestroy(s.exec);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.host) (void)hipHostFree(s.host);
    }
    if (b->dev) (void)hipFree(b->dev);
    delete b;
    return RZPIC_OK;
}

rzpic_status rzpic_batch_step(rzpic_batch *b, int64_t step)
{
    if (!b) return rz_fail(RZPIC_EINVAL, "null batch");
    const int n = (int)b->ctx.size();
    for (int i = 0; i < n; ++i) {
        std::string why;
        if (!rz_batchable(b->ctx[i], why)) {
            char buf[256];
            std::snprintf(buf, sizeof buf, "batch: context %d: %s", i, why.c_str());
            return rz_fail(RZPIC_EINVAL, buf);
        }
        // a pipelined step's pending list maintenance precedes the batch
        // (which orders itself after the contexts' streams)
        rzpic_status ss = rz_settle(b->ctx[i]);
        if (ss != RZPIC_OK) return ss;
    }
    // record every discharge's step (host bookkeeping only)
    for (int i = 0; i < n; ++i) {
        b->rec[i].recs.clear();
        g_recorder = &b->rec[i];
        const rzpic_status s = rzpic_step(b->ctx[i], step);
        g_recorder = nullptr;
        if (s != RZPIC_OK) return s;
    }
    // groups of identical launch sequences, in order of first appearance
    std::vector<std::vector<int>> groups;
    {
        std::map<std::vector<std::pair<const void *, unsigned>>, int> sig_group;
        for (int i = 0; i < n; ++i) {
            std::vector<std::pair<const void *, unsigned>> sig;
            sig.reserve(b->rec[i].recs.size());
            for (const LaunchRec &L : b->rec[i].recs) sig.emplace_back(L.key, L.threads);
            auto it = sig_group.find(sig);
            if (it == sig_group.end()) {
                sig_group.emplace(std::move(sig), (int)groups.size());
                groups.push_back({i});
            } else {
                groups[it->second].push_back(i);
            }
        }
    }
    // job tables of the batched positions: layout, then contents
    struct Table {
        size_t off;
        int blocks;
    };
    std::vector<std::vector<Table>> tables(groups.size());
    size_t total = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        const int i0 = groups[g][0];
        const size_t npos = b->rec[i0].recs.size();
        tables[g].assign(npos, Table{0, 0});
        for (size_t p = 0; p < npos; ++p) {
            const LaunchRec &L = b->rec[i0].recs[p];
            if (!L.many) continue;
            total = align_up(total, 256);
            tables[g][p].off = total;
            total += L.job_size * groups[g].size();
        }
    }
    Staging &S = b->stage[b->which];
    if (total > 0) {
        if (S.used) BCHK(hipEventSynchronize(S.done), "batch: staging reuse");
        if (total > S.cap) {
            if (S.exec) BCHK(hipGraphExecDestroy(S.exec), "batch: graph free");
            S.exec = nullptr;
            if (S.host) BCHK(hipHostFree(S.host), "batch: staging free");
            S.host = nullptr;
            S.cap = 0;
            BCHK(hipHostMalloc(&S.host, total * 2), "batch: staging allocation");
            S.cap = total * 2;
        }
        if (total > b->dev_cap) {
            // earlier steps may still read the old table
            BCHK(hipStreamSynchronize(b->st), "batch: table reallocation");
            for (auto &t : b->stage) {
                if (t.exec) BCHK(hipGraphExecDestroy(t.exec), "batch: graph free");
                t.exec = nullptr;
            }
            if (b->dev) BCHK(hipFree(b->dev), "batch: table free");
            b->dev = nullptr;
            b->dev_cap = 0;
            BCHK(hipMalloc(&b->dev, total * 2), "batch: table allocation");
            b->dev_cap = total * 2;
        }
        unsigned char *h = (unsigned char *)S.host;
        for (size_t g = 0; g < groups.size(); ++g) {
            const int i0 = groups[g][0];
            for (size_t p = 0; p < tables[g].size(); ++p) {
                const LaunchRec &L0 = b->rec[i0].recs[p];
                if (!L0.many) continue;
                int first = 0;
                for (size_t k = 0; k < groups[g].size(); ++k) {
                    const LaunchRec &L = b->rec[groups[g][k]].recs[p];
                    unsigned char *job = h + tables[g][p].off + k * L0.job_size;
                    std::memset(job, 0, L0.job_size);
                    std::memcpy(job, L.args.data(), L.args.size());
                    const int nx = (int)L.gx, ny = (int)L.gy;
                    int *f = (int *)(job + L0.first_off);
                    f[0] = first;
                    f[1] = nx;
                    f[2] = ny;
                    first += nx * ny;
                }
                tables[g][p].blocks = first;
            }
        }
    }
    // order after the contexts' own streams, upload, fork
    {
        std::vector<hipStream_t> seen;
        for (rzpic_ctx *c : b->ctx) {
            hipStream_t cs = rz_stream(c);
            if (cs == b->st || std::find(seen.begin(), seen.end(), cs) != seen.end()) continue;
            seen.push_back(cs);
            BCHK(hipEventRecord(b->ctx_ev, cs), "batch: event");
            BCHK(hipStreamWaitEvent(b->st, b->ctx_ev, 0), "batch: wait");
        }
    }
    // the step's device work: upload, fork, every group's launches, join
    int launches = 0, batched = 0;
    const int nst = (int)std::min<size_t>(groups.size(), (size_t)b->nstreams);
    auto enqueue = [&]() -> rzpic_status {
        launches = batched = 0;
        if (total > 0)
            BCHK(hipMemcpyAsync(b->dev, S.host, total, hipMemcpyHostToDevice, b->st),
                 "batch: upload");
        BCHK(hipEventRecord(b->fork, b->st), "batch: event");
        for (int k = 0; k < nst; ++k)
            BCHK(hipStreamWaitEvent(b->streams[k], b->fork, 0), "batch: wait");
        for (size_t g = 0; g < groups.size(); ++g) {
            hipStream_t gs = b->streams[g % b->nstreams];
            const std::vector<int> &mem = groups[g];
            const Recorder &R0 = b->rec[mem[0]];
            for (size_t p = 0; p < R0.recs.size(); ++p) {
                const LaunchRec &L0 = R0.recs[p];
                if (L0.many) {
                    size_t lds = 0;
                    for (int i : mem) lds = std::max(lds, b->rec[i].recs[p].lds);
                    BCHK(L0.many((const unsigned char *)b->dev + tables[g][p].off, (int)mem.size(),
                                 tables[g][p].blocks, L0.threads, lds, gs),
                         "batch: launch");
                    ++launches;
                    ++batched;
                } else {
                    for (int i : mem) {
                        b->rec[i].recs[p].raw(gs);
                        BCHK(hipGetLastError(), "batch: launch");
                        ++launches;
                    }
                }
            }
        }
        for (int k = 0; k < nst; ++k) {
            BCHK(hipEventRecord(b->join[k], b->streams[k]), "batch: event");
            BCHK(hipStreamWaitEvent(b->st, b->join[k], 0), "batch: wait");
        }
        return RZPIC_OK;
    };
    // A step whose launches are all batched can be replayed from a capture:
    // only the job tables (uploaded from the staging buffer) change between
    // such steps, as long as the groups, kernels, shapes and table layout do.
    bool all_batched = true;
    std::vector<size_t> layout;
    for (size_t g = 0; g < groups.size(); ++g) {
        layout.push_back(groups[g].size());
        for (int i : groups[g]) layout.push_back((size_t)i);
        const Recorder &R0 = b->rec[groups[g][0]];
        for (size_t p = 0; p < R0.recs.size(); ++p) {
            const LaunchRec &L0 = R0.recs[p];
            all_batched = all_batched && L0.many != nullptr;
            size_t lds = 0;
            for (int i : groups[g]) lds = std::max(lds, b->rec[i].recs[p].lds);
            layout.insert(layout.end(), {(size_t)L0.key, L0.threads, lds, tables[g][p].off,
                                         (size_t)tables[g][p].blocks});
        }
    }
    layout.push_back(total);
    int nl = 0, nb = 0;  // launches of the step, batched ones
    for (size_t g = 0; g < groups.size(); ++g)
        for (const LaunchRec &L0 : b->rec[groups[g][0]].recs) {
            nl += L0.many ? 1 : (int)groups[g].size();
            nb += L0.many ? 1 : 0;
        }
    if (b->graph && all_batched && b->st) {
        if (!S.exec || S.layout != layout) {
            if (S.exec) BCHK(hipGraphExecDestroy(S.exec), "batch: graph free");
            S.exec = nullptr;
            hipGraph_t gr = nullptr;
            BCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal), "batch: capture");
            const rzpic_status es = enqueue();
            const hipError_t ce = hipStreamEndCapture(b->st, &gr);
            if (es != RZPIC_OK) {
                if (gr) (void)hipGraphDestroy(gr);
                return es;
            }
            if (ce != hipSuccess) return hipfail(ce, "batch: capture");
            const hipError_t ie = hipGraphInstantiate(&S.exec, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (ie != hipSuccess) {
                S.exec = nullptr;
                return hipfail(ie, "batch: graph instantiation");
            }
            S.layout = layout;
        }
        BCHK(hipGraphLaunch(S.exec, b->st), "batch: graph launch");
    } else {
        const rzpic_status es = enqueue();
        if (es != RZPIC_OK) return es;
    }
    if (total > 0) {
        BCHK(hipEventRecord(S.done, b->st), "batch: event");
        S.used = true;
        b->which ^= 1;
    }
    // the contexts' streams continue after the batch
    BCHK(hipEventRecord(b->ctx_ev, b->st), "batch: event");
    {
        std::vector<hipStream_t> seen;
        for (rzpic_ctx *c : b->ctx) {
            hipStream_t cs = rz_stream(c);
            if (cs == b->st || std::find(seen.begin(), seen.end(), cs) != seen.end()) continue;
            seen.push_back(cs);
            BCHK(hipStreamWaitEvent(cs, b->ctx_ev, 0), "batch: wait");
        }
    }
    b->classes = (int32_t)groups.size();
    b->launches = nl;
    b->batched = nb;
    (void)launches;
    (void)batched;
    return RZPIC_OK;
}

rzpic_status rzpic_batch_set_graph(rzpic_batch *b, int32_t on)
{
    if (!b) return rz_fail(RZPIC_EINVAL, "null batch");
    if (on && !b->st)
        return rz_fail(RZPIC_EINVAL, "batch: graph replay needs a stream other than the null stream");
    b->graph = on != 0;
    return RZPIC_OK;
}

// Autotuner of the pass configuration per group of like discharges (same
// mesh and precision): the launch shape, the deposit form and the tile
// shape are tried on the group's discharges stepped as a batch of their
// own, timed with HIP events on the batch stream.
rzpic_status rzpic_batch_autotune(rzpic_batch *b, int32_t steps, int64_t step0, double *table,
                                  int32_t max_rows, int32_t *rows, int64_t *next_step)
{
    if (!b || !next_step) return rz_fail(RZPIC_EINVAL, "null argument");
    if (steps < 1) return rz_fail(RZPIC_EINVAL, "steps must be >= 1");
    if (table && max_rows < 0) return rz_fail(RZPIC_EINVAL, "max_rows must be >= 0");
    const int n = (int)b->ctx.size();
    std::map<std::vector<int32_t>, std::vector<int>> by_key;
    std::vector<std::vector<int32_t>> key_order;
    for (int i = 0; i < n; ++i) {
        std::vector<int32_t> k(5);
        rz_tune_key(b->ctx[i], k.data());
        auto it = by_key.find(k);
        if (it == by_key.end()) {
            by_key.emplace(k, std::vector<int>{i});
            key_order.push_back(k);
        } else {
            it->second.push_back(i);
        }
    }
    struct Cfg {
        int threads;
        int64_t ppb;
        int lds, tz, tr;
    };
    static const int kThreads[3] = {256, 512, 1024};
    static const int64_t kPpb[4] = {2048, 4096, 8192, 16384};
    static const int kTiles[7][2] = {{8, 16}, {8, 32}, {16, 16}, {16, 32}, {16, 64}, {32, 32}, {32, 64}};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BCHK(hipEventCreate(&e0), "autotune: event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return rz_fail(RZPIC_EHIP, "autotune: event");
    }
    // earlier batched steps drain before configurations change
    {
        const hipError_t se = b->st ? hipStreamSynchronize(b->st) : hipDeviceSynchronize();
        if (se != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return hipfail(se, "autotune: sync");
        }
    }
    int nrow = 0;
    std::vector<int64_t> at(key_order.size(), step0);  // next step of each group
    rzpic_status st = RZPIC_OK;
    for (size_t g = 0; g < key_order.size() && st == RZPIC_OK; ++g) {
        const std::vector<int32_t> &key = key_order[g];
        std::vector<rzpic_ctx *> mem;
        for (int i : by_key[key]) mem.push_back(b->ctx[i]);
        rzpic_batch *sb = nullptr;
        st = rzpic_batch_create(mem.data(), (int32_t)mem.size(), b->st, &sb);
        if (st != RZPIC_OK) break;
        sb->graph = b->graph && b->st;
        sb->nstreams = 1;
        int32_t cur[5];
        rz_get_config(mem[0], cur);
        std::vector<Cfg> tried;
        std::vector<double> ms;
        auto fits = [&](const Cfg &c) {
            for (rzpic_ctx *x : mem)
                if (!rz_config_fits(x, c.threads, c.ppb, c.lds)) return false;
            return true;
        };
        auto timed = [&](const Cfg &c) -> rzpic_status {
            for (rzpic_ctx *x : mem) {
                const rzpic_status s = rz_set_config(x, c.threads, c.ppb, c.lds, c.tz, c.tr);
                if (s != RZPIC_OK) return s;
            }
            rzpic_status s = rzpic_batch_step(sb, at[g]++);  // warm-up (and capture)
            if (s != RZPIC_OK) return s;
            BCHK(hipEventRecord(e0, b->st), "autotune: event");
            for (int k = 0; k < steps; ++k)
                if ((s = rzpic_batch_step(sb, at[g]++)) != RZPIC_OK) return s;
            BCHK(hipEventRecord(e1, b->st), "autotune: event");
            BCHK(hipEventSynchronize(e1), "autotune: sync");
            float f = 0.0f;
            BCHK(hipEventElapsedTime(&f, e0, e1), "autotune: timing");
            tried.push_back(c);
            ms.push_back((double)f / steps);
            return RZPIC_OK;
        };
        // the configuration in use first: near-ties keep it
        const Cfg start{cur[0], (int64_t)cur[1], cur[2] == RZPIC_FORM_LDS ? 1 : 0, cur[3], cur[4]};
        st = timed(start);
        // launch shapes in each form the group can run (the tiled form only
        // where the steps sort, so that it has a plan)
        for (int lds = 1; lds >= 0 && st == RZPIC_OK; --lds) {
            if (lds ? !key[3] : !key[4]) continue;
            for (int ti = 0; ti < 3 && st == RZPIC_OK; ++ti)
                for (int pi = 0; pi < 4 && st == RZPIC_OK; ++pi) {
                    const Cfg c{kThreads[ti], kPpb[pi], lds, start.tz, start.tr};
                    const bool same = c.threads == start.threads && c.ppb == start.ppb &&
                                      c.lds == start.lds;
                    if (!same && fits(c)) st = timed(c);
                }
        }
        // tile shapes around the best configuration of the tiled form
        auto best_of = [&](int form) {  // first within 2 % of the fastest
            double lo = -1.0;
            for (size_t k = 0; k < ms.size(); ++k)
                if (form < 0 || tried[k].lds == form) lo = lo < 0.0 || ms[k] < lo ? ms[k] : lo;
            for (size_t k = 0; k < ms.size(); ++k)
                if ((form < 0 || tried[k].lds == form) && ms[k] <= 1.02 * lo) return (int)k;
            return -1;
        };
        if (st == RZPIC_OK && key[4]) {
            const int bt = best_of(0);
            if (bt >= 0)
                for (int k = 0; k < 7 && st == RZPIC_OK; ++k) {
                    Cfg c = tried[bt];
                    c.tz = kTiles[k][0];
                    c.tr = kTiles[k][1];
                    const int ntr = (key[0] - 2) / c.tr + 1;
                    if (((key[1] - 2) / c.tz + 1) * ntr > 2048) continue;
                    if (c.tz == tried[bt].tz && c.tr == tried[bt].tr) continue;
                    st = timed(c);
                }
        }
        const int win = st == RZPIC_OK ? best_of(-1) : -1;
        if (win >= 0) {
            const Cfg &c = tried[win];
            for (rzpic_ctx *x : mem)
                if (st == RZPIC_OK) st = rz_set_config(x, c.threads, c.ppb, c.lds, c.tz, c.tr);
        }
        for (size_t k = 0; k < tried.size() && table; ++k, ++nrow) {
            if (nrow >= max_rows) continue;
            double *r = table + (size_t)8 * nrow;
            r[0] = (double)g;
            r[1] = tried[k].threads;
            r[2] = (double)tried[k].ppb;
            r[3] = tried[k].lds ? RZPIC_FORM_LDS : RZPIC_FORM_TILED;
            r[4] = tried[k].tz;
            r[5] = tried[k].tr;
            r[6] = ms[k];
            r[7] = (int)k == win ? 1.0 : 0.0;
        }
        if (!table) nrow += (int)tried.size();
        // the group's own streams drain before its batch goes
        const hipError_t se = b->st ? hipStreamSynchronize(b->st) : hipDeviceSynchronize();
        rzpic_batch_destroy(sb);
        if (st == RZPIC_OK && se != hipSuccess) st = hipfail(se, "autotune: sync");
    }
    // every discharge at the same next step: the groups behind catch up
    int64_t last = step0;
    for (int64_t a : at) last = a > last ? a : last;
    for (size_t g = 0; g < key_order.size() && st == RZPIC_OK; ++g) {
        if (at[g] == last) continue;
        std::vector<rzpic_ctx *> mem;
        for (int i : by_key[key_order[g]]) mem.push_back(b->ctx[i]);
        rzpic_batch *sb = nullptr;
        st = rzpic_batch_create(mem.data(), (int32_t)mem.size(), b->st, &sb);
        while (st == RZPIC_OK && at[g] < last) st = rzpic_batch_step(sb, at[g]++);
        if (sb) {
            if (b->st) (void)hipStreamSynchronize(b->st);
            rzpic_batch_destroy(sb);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RZPIC_OK) return st;
    if (rows) *rows = nrow;
    *next_step = last;
    return RZPIC_OK;
}

rzpic_status rzpic_batch_stats(rzpic_batch *b, int32_t out[3])
{
    if (!b || !out) return rz_fail(RZPIC_EINVAL, "null argument");
    out[0] = b->classes;
    out[1] = b->launches;
    out[2] = b->batched;
    return RZPIC_OK;
}

}  // extern "C"
