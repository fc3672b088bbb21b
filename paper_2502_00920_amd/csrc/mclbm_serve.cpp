// Continuous-batching server of the mclbm C ABI: many simulations of different
// sizes, materials, loads and step counts advanced together on one GPU.
//
// A round advances every active simulation by up to K steps.  The batch is
// split into four groups, two per material, balanced by lattice nodes.  For
// each step and group the host writes a table of the group's simulations
// (their step arguments: buffers by step parity, wall values at their own step
// index, work items), uploads the round's tables with one copy, and replays on
// each of four streams a graph of the group's K launches of the batched step
// kernel: the kernel reads its table from device memory, one work item per
// wave, so a graph serves every round whose items fit its grid; a round with
// more items captures the group's graph again on a grid at least twice as
// large.  A step of a group lasts about as long as one work item (a march over
// a chunk of at most 16 rows), whatever its size; the groups' steps are
// independent and run side by
// side on the hardware queues, so that one group's tail overlaps another's
// work.  Between rounds the host collects the simulations that have finished (their displacement is copied to the caller's buffer) and
// admits waiting requests in arrival order while a slot is free and their
// arena fits in the caller's device pool (first fit).  Requests that arrive
// while others are on the GPU join at the next round and share its launches.
// After each round a scan of every active simulation's displacement flags the
// ones that hold values that are not finite or have passed their growth limit;
// they end at the next turn as unstable instead of running out their steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "mclbm.h"
#include "mclbm_internal.hpp"

#define MCLBM_EXPORT extern "C" __attribute__((visibility("default")))

using namespace mclbm;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

#define SV_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) return set_error(MCLBM_EHIP, hipGetErrorString(e_));    \
    } while (0)

// first fit over the arena part of the pool, free blocks merged on release
struct Heap {
    std::map<size_t, size_t> free_;  // offset -> bytes
    void init(size_t off, size_t bytes) {
        free_.clear();
        if (bytes) free_[off] = bytes;
    }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, roff = it->first + bytes;
            free_.erase(it);
            if (rest) free_[roff] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Request {
    mclbm_params p;
    mclbm_side_spec side[4];
    std::vector<double> table[4];  // TABLE programs, copied at submission
    std::vector<double> u0;  // empty: zero
    int64_t nsteps = 0;
    double* u_out = nullptr;
    int state = MCLBM_REQ_WAITING;
    int status = MCLBM_OK;
    size_t off = 0, bytes = 0;
    mclbm_sim* sim = nullptr;
    int64_t done_steps = 0;
    int64_t round_steps = 0;
    int slot = -1;  // its entry in the round's failure scan
};

}  // namespace

constexpr int kGroups = 4;  // groups 0, 1: St. Venant-Kirchhoff; 2, 3: neo-Hooke

struct mclbm_server {
    mclbm_server_config cfg;
    int prec = 0;
    char* pool = nullptr;
    size_t pool_bytes = 0;
    hipStream_t stream = nullptr;
    size_t step_bytes = 0, table_bytes = 0;
    size_t scan_off = 0, flags_off = 0, reserved_bytes = 0;  // in the reserved head of the pool
    uint32_t* host_flags = nullptr;                             // pinned: the round's scan flags
    Heap heap;
    char* host_table = nullptr;  // pinned staging of one round's tables
    int64_t next_id = 1;
    std::deque<int64_t> waiting;
    std::vector<int64_t> active;
    std::unordered_map<int64_t, Request> reqs;
    hipStream_t gstream[kGroups] = {};
    hipGraphExec_t graph[kGroups] = {};
    int graph_march[kGroups] = {}, graph_wall[kGroups] = {};  // grids of each captured graph
    hipEvent_t fork = nullptr, join[kGroups] = {};
    hipEvent_t round_done = nullptr;
    bool in_flight = false;
    int64_t ndone = 0;
};

namespace {

int check_config(const mclbm_server_config* c) {
    if (!c) return set_error(MCLBM_EINVAL, "config is NULL");
    if (c->precision != MCLBM_F64 && c->precision != MCLBM_F32 && c->precision != MCLBM_F16 &&
        c->precision != MCLBM_BF16)
        return set_error(MCLBM_EINVAL, "unknown storage precision");
    if (c->steps_per_round < 1 || c->steps_per_round > 1024)
        return set_error(MCLBM_EINVAL, "steps_per_round must be in 1..1024");
    if (c->max_active < 1 || c->max_active > 1024) return set_error(MCLBM_EINVAL, "max_active must be in 1..1024");
    return MCLBM_OK;
}

// table of step k, group g
size_t table_off(const mclbm_server* sv, int k, int g) { return ((size_t)k * kGroups + g) * sv->step_bytes; }

// the reserved head of the pool: the step tables of a round, the failure-scan
// table and its flags (uploaded together, the flags as zeros)
void layout_reserved(const mclbm_server_config* c, size_t* tables, size_t* scan_off, size_t* flags_off,
                     size_t* total) {
    *tables = (size_t)c->steps_per_round * kGroups * batch_step_bytes(c->max_active);
    *scan_off = *tables;
    *flags_off = *scan_off + align_up((size_t)c->max_active * sizeof(ScanEntry));
    *total = *flags_off + align_up((size_t)c->max_active * sizeof(uint32_t));
}

void release(mclbm_server* sv, Request& r) {
    if (r.sim) {
        mclbm_destroy(r.sim);
        r.sim = nullptr;
    }
    if (r.bytes) sv->heap.release(r.off, r.bytes);
    r.bytes = 0;
    r.u0.clear();
    r.u0.shrink_to_fit();
}

// copy the result out, check it, free the arena
int finish(mclbm_server* sv, Request& r) {
    int rc = mclbm_read(r.sim, MCLBM_FIELD_U, r.u_out, 0);
    if (rc == MCLBM_OK) {
        mclbm_diag_out d;
        const int dr = mclbm_diag(r.sim, &d);
        r.status = dr == MCLBM_EUNSTABLE ? MCLBM_EUNSTABLE : (dr == MCLBM_OK ? MCLBM_OK : dr);
    } else {
        r.status = rc;
    }
    release(sv, r);
    r.state = MCLBM_REQ_DONE;
    sv->ndone++;
    return MCLBM_OK;
}

// create, set up and initialise r's simulation in its arena (asynchronous on the stream)
int start(mclbm_server* sv, Request& r) {
    int rc = mclbm_create(&r.p, sv->pool + r.off, r.bytes, sv->stream, &r.sim);
    for (int i = 0; rc == MCLBM_OK && i < 4; i++) rc = mclbm_set_side(r.sim, i, &r.side[i]);
    if (rc == MCLBM_OK) rc = mclbm_init(r.sim, r.u0.empty() ? nullptr : r.u0.data(), nullptr, 0);
    return rc;
}

// the K steps of group gi as one graph, on its stream, on grids of the given blocks
int capture(mclbm_server* sv, int gi, int march_blocks, int wall_blocks) {
    hipStream_t st = sv->gstream[gi];
    SV_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int k = 0; k < sv->cfg.steps_per_round && err == hipSuccess; k++)
        err = launch_batch_step(sv->prec, gi < 2 ? MAT_SVK : MAT_NH,
                                reinterpret_cast<const BatchStep*>(sv->pool + table_off(sv, k, gi)), march_blocks,
                                wall_blocks, st);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (err == hipSuccess) err = ec;
    if (err == hipSuccess) err = hipGraphInstantiate(&sv->graph[gi], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (err != hipSuccess) return set_error(MCLBM_EHIP, hipGetErrorString(err));
    sv->graph_march[gi] = march_blocks;
    sv->graph_wall[gi] = wall_blocks;
    return MCLBM_OK;
}

}  // namespace

MCLBM_EXPORT int mclbm_server_plan(const mclbm_server_config* cfg, size_t* reserved_bytes) {
    if (int rc = check_config(cfg)) return rc;
    size_t tables, scan, flags, total;
    layout_reserved(cfg, &tables, &scan, &flags, &total);
    if (reserved_bytes) *reserved_bytes = total;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_server_create(const mclbm_server_config* cfg, void* pool, size_t pool_bytes, void* stream,
                                     mclbm_server** out) {
    if (int rc = check_config(cfg)) return rc;
    if (!out) return set_error(MCLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!pool || reinterpret_cast<uintptr_t>(pool) % kAlign)
        return set_error(MCLBM_EINVAL, "pool must be a 256-byte aligned device pointer");
    mclbm_server* sv = new (std::nothrow) mclbm_server;
    if (!sv) return set_error(MCLBM_EINVAL, "out of host memory");
    sv->cfg = *cfg;
    sv->prec = cfg->precision == MCLBM_F64   ? PREC_F64
               : cfg->precision == MCLBM_F32 ? PREC_F32
               : cfg->precision == MCLBM_F16 ? PREC_F16
                                             : PREC_BF16;
    sv->pool = static_cast<char*>(pool);
    sv->pool_bytes = pool_bytes;
    sv->stream = static_cast<hipStream_t>(stream);
    sv->step_bytes = batch_step_bytes(cfg->max_active);
    layout_reserved(cfg, &sv->table_bytes, &sv->scan_off, &sv->flags_off, &sv->reserved_bytes);
    if (pool_bytes < sv->reserved_bytes) {
        delete sv;
        return set_error(MCLBM_ETOOSMALL, "pool smaller than mclbm_server_plan's reserved bytes");
    }
    sv->heap.init(sv->reserved_bytes, pool_bytes - sv->reserved_bytes);
    bool ok = hipHostMalloc(reinterpret_cast<void**>(&sv->host_table), sv->reserved_bytes, hipHostMallocDefault) ==
                  hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&sv->host_flags), (size_t)cfg->max_active * sizeof(uint32_t),
                            hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&sv->round_done, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&sv->fork, hipEventDisableTiming) == hipSuccess;
    for (int g = 0; ok && g < kGroups; g++)  // default priority
        ok = hipStreamCreateWithFlags(&sv->gstream[g], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&sv->join[g], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        mclbm_server_destroy(sv);
        return set_error(MCLBM_EHIP, "pinned staging, stream or event creation failed");
    }
    std::memset(sv->host_table, 0, sv->reserved_bytes);
    std::memset(sv->host_flags, 0, (size_t)cfg->max_active * sizeof(uint32_t));
    *out = sv;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_server_submit(mclbm_server* sv, const mclbm_params* p, const mclbm_side_spec* sides,
                                     const double* u0, int64_t nsteps, double* u_out, int64_t* id_out) {
    if (!sv || !p || !sides || !u_out || !id_out) return set_error(MCLBM_EINVAL, "NULL argument");
    size_t bytes = 0;
    if (int rc = mclbm_plan(p, &bytes, nullptr, nullptr)) return rc;
    if (p->precision != sv->cfg.precision)
        return set_error(MCLBM_EINVAL, "request precision differs from the server's");
    if (p->material != MCLBM_SVK && p->material != MCLBM_NEOHOOKE)
        return set_error(MCLBM_EINVAL, "the server runs St. Venant-Kirchhoff and neo-Hooke materials");
    if (p->boundary_order == 2 || p->time_levels == 1)
        return set_error(MCLBM_EINVAL, "the server runs the fused step: first-order boundary differences and "
                                       "the current time level only");
    if (nsteps < 1) return set_error(MCLBM_EINVAL, "nsteps must be >= 1");
    bytes = align_up(bytes);
    if (bytes > sv->pool_bytes - sv->reserved_bytes)
        return set_error(MCLBM_ETOOSMALL, "the request's arena exceeds the server's pool");
    for (int i = 0; i < 4; i++)  // validate the side programs now rather than at admission
        if (int rc = check_side_program(&sides[i])) return rc;
    const int64_t id = sv->next_id++;
    Request& r = sv->reqs[id];
    r.p = *p;
    std::memcpy(r.side, sides, sizeof r.side);
    for (int i = 0; i < 4; i++)
        if (sides[i].kind == MCLBM_LOAD_TABLE) {
            r.table[i].assign(sides[i].table, sides[i].table + sides[i].table_len);
            r.side[i].table = r.table[i].data();
        }
    if (u0) r.u0.assign(u0, u0 + 2 * (size_t)p->nx * p->ny);
    r.nsteps = nsteps;
    r.u_out = u_out;
    r.bytes = bytes;
    sv->waiting.push_back(id);
    *id_out = id;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_server_progress(mclbm_server* sv, int64_t* done_ids, int32_t cap, int32_t* ndone) {
    if (!sv || !ndone || (cap > 0 && !done_ids)) return set_error(MCLBM_EINVAL, "NULL argument");
    *ndone = 0;
    // 1. the round in flight: account its steps, collect the finished simulations
    if (sv->in_flight) {
        SV_HIP(hipEventSynchronize(sv->round_done));
        sv->in_flight = false;
        std::vector<int64_t> still;
        for (int64_t id : sv->active) {
            Request& r = sv->reqs[id];
            advance(r.sim, r.round_steps);
            r.done_steps += r.round_steps;
            r.round_steps = 0;
            // runs on unless it has all its steps or its displacement is no longer finite
            const bool failed = r.slot >= 0 && sv->host_flags[r.slot] != 0;
            r.slot = -1;
            if (r.done_steps < r.nsteps && !failed) {
                still.push_back(id);
                continue;
            }
            if (int rc = finish(sv, r)) return rc;
            if (*ndone < cap) done_ids[(*ndone)++] = id;
        }
        sv->active.swap(still);
    }
    // 2. admission in arrival order: a free slot and room in the pool
    while (!sv->waiting.empty() && (int)sv->active.size() < sv->cfg.max_active) {
        const int64_t id = sv->waiting.front();
        Request& r = sv->reqs[id];
        if (!sv->heap.alloc(r.bytes, &r.off)) break;
        sv->waiting.pop_front();
        if (int rc = start(sv, r)) {
            r.status = rc;
            release(sv, r);
            r.state = MCLBM_REQ_DONE;
            sv->ndone++;
            if (*ndone < cap) done_ids[(*ndone)++] = id;
            continue;
        }
        r.state = MCLBM_REQ_ACTIVE;
        sv->active.push_back(id);
    }
    if (sv->active.empty()) return MCLBM_OK;
    // 3. the round's tables: step k of every simulation with steps left, by material
    const int K = sv->cfg.steps_per_round;
    for (int k = 0; k < K; k++)
        for (int g = 0; g < kGroups; g++) {
            BatchStep* st = reinterpret_cast<BatchStep*>(sv->host_table + table_off(sv, k, g));
            st->nsims = 0;
            st->nitems = 0;
            st->nsegs = 0;
        }
    // groups: largest lattices first, each to the lighter of its material's two
    std::vector<int64_t> order(sv->active);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        const Request& ra = sv->reqs[a];
        const Request& rb = sv->reqs[b];
        return (int64_t)ra.p.nx * ra.p.ny > (int64_t)rb.p.nx * rb.p.ny;
    });
    int64_t load[kGroups] = {0, 0, 0, 0};
    for (int64_t id : order) {
        Request& r = sv->reqs[id];
        r.round_steps = std::min<int64_t>(K, r.nsteps - r.done_steps);
        const int g0 = r.p.material == MCLBM_SVK ? 0 : 2;
        const int gi = load[g0] <= load[g0 + 1] ? g0 : g0 + 1;
        load[gi] += (int64_t)r.p.nx * r.p.ny;
        for (int k = 0; k < r.round_steps; k++) {
            BatchStep* st = reinterpret_cast<BatchStep*>(sv->host_table + table_off(sv, k, gi));
            BatchEntry& e = st->e[st->nsims++];
            batch_entry(r.sim, k, &e);
            e.item0 = st->nitems;
            st->nitems += e.nstrip * e.nchunk;
            e.seg0 = st->nsegs;
            st->nsegs += wall_segs(e.a.g).total;
        }
    }
    // the failure scan of every simulation's displacement after the round; its
    // flags go up as zeros with the tables
    ScanEntry* scan = reinterpret_cast<ScanEntry*>(sv->host_table + sv->scan_off);
    int nscan = 0;
    for (int64_t id : sv->active) {
        Request& r = sv->reqs[id];
        r.slot = nscan;
        scan_entry(r.sim, r.round_steps, nscan, &scan[nscan]);
        nscan++;
    }
    std::memset(sv->host_table + sv->flags_off, 0, (size_t)nscan * sizeof(uint32_t));
    // 4. one upload, then the four groups' graphs side by side
    SV_HIP(hipMemcpyAsync(sv->pool, sv->host_table, sv->reserved_bytes, hipMemcpyHostToDevice, sv->stream));
    // a group's graph serves every round whose tables fit its grids (a wave per
    // work item, a block per wall segment); a larger round captures it again,
    // with grids twice as large or more
    for (int g = 0; g < kGroups; g++) {
        int mb = 0, wb = 0;
        for (int k = 0; k < K; k++) {
            const BatchStep* t = reinterpret_cast<const BatchStep*>(sv->host_table + table_off(sv, k, g));
            mb = std::max(mb, batch_grid((t->nitems + 3) / 4));
            wb = std::max(wb, batch_grid(t->nsegs));
        }
        if (sv->graph[g] && sv->graph_march[g] >= mb && sv->graph_wall[g] >= wb) continue;
        if (sv->graph[g]) {
            SV_HIP(hipGraphExecDestroy(sv->graph[g]));
            sv->graph[g] = nullptr;
        }
        if (int rc = capture(sv, g, std::max(mb, sv->graph_march[g]), std::max(wb, sv->graph_wall[g]))) return rc;
    }
    SV_HIP(hipEventRecord(sv->fork, sv->stream));
    for (int g = 0; g < kGroups; g++) {
        SV_HIP(hipStreamWaitEvent(sv->gstream[g], sv->fork, 0));
        SV_HIP(hipGraphLaunch(sv->graph[g], sv->gstream[g]));
        SV_HIP(hipEventRecord(sv->join[g], sv->gstream[g]));
        SV_HIP(hipStreamWaitEvent(sv->stream, sv->join[g], 0));
    }
    uint32_t* dflags = reinterpret_cast<uint32_t*>(sv->pool + sv->flags_off);
    SV_HIP(launch_nanscan(reinterpret_cast<const ScanEntry*>(sv->pool + sv->scan_off), nscan, dflags, sv->stream));
    SV_HIP(hipMemcpyAsync(sv->host_flags, dflags, (size_t)nscan * sizeof(uint32_t), hipMemcpyDeviceToHost,
                          sv->stream));
    SV_HIP(hipEventRecord(sv->round_done, sv->stream));
    sv->in_flight = true;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_server_result(mclbm_server* sv, int64_t id, int32_t* state, int32_t* status) {
    if (!sv || !state || !status) return set_error(MCLBM_EINVAL, "NULL argument");
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return set_error(MCLBM_EINVAL, "unknown request id");
    *state = it->second.state;
    *status = it->second.status;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_server_steps(mclbm_server* sv, int64_t id, int64_t* steps) {
    if (!sv || !steps) return set_error(MCLBM_EINVAL, "NULL argument");
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return set_error(MCLBM_EINVAL, "unknown request id");
    *steps = it->second.done_steps;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_server_counts(mclbm_server* sv, int64_t* waiting, int64_t* active, int64_t* done) {
    if (!sv) return set_error(MCLBM_EINVAL, "NULL server");
    if (waiting) *waiting = (int64_t)sv->waiting.size();
    if (active) *active = (int64_t)sv->active.size();
    if (done) *done = sv->ndone;
    return MCLBM_OK;
}

MCLBM_EXPORT int mclbm_server_destroy(mclbm_server* sv) {
    if (!sv) return MCLBM_OK;
    if (sv->in_flight) (void)hipEventSynchronize(sv->round_done);
    for (auto& kv : sv->reqs) release(sv, kv.second);
    for (int g = 0; g < kGroups; g++) {
        if (sv->graph[g]) (void)hipGraphExecDestroy(sv->graph[g]);
        if (sv->join[g]) (void)hipEventDestroy(sv->join[g]);
        if (sv->gstream[g]) (void)hipStreamDestroy(sv->gstream[g]);
    }
    if (sv->fork) (void)hipEventDestroy(sv->fork);
    if (sv->round_done) (void)hipEventDestroy(sv->round_done);
    if (sv->host_table) (void)hipHostFree(sv->host_table);
    if (sv->host_flags) (void)hipHostFree(sv->host_flags);
    delete sv;
    return MCLBM_OK;
}
