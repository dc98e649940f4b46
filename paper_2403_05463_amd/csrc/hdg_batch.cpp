// Batches of independent meshes advanced together (continuous batching): each
// member keeps its own state, RK register, time step and parameters resident
// in device memory, and every RK stage of the whole batch is one persistent
// launch per (kernel kind, order) over the union of the members' tiles.  The
// kernels compute each element exactly as for a mesh on its own, so a member's
// result does not depend on what else is in the batch.
#include <cmath>
#include <cstring>

#include "hdg_host.h"

using hdg::Epi;
using hdg::LaunchCfg;
using hdg::Member;
using hdg::StageArgs;
using hdg::Tile;
using hdg::TilePlan;

struct hdg_batch {
    struct Slot {
        hdg_mesh *mesh = nullptr;
        double *q = nullptr, *dq = nullptr;
        double dt = 0.0;
        bool stale = false;                    // freed since the plans were last built
    };
    hdg_ctx *ctx = nullptr;
    std::vector<Slot> slots;
    Member *members = nullptr;                 // device table, one record per slot
    std::vector<TilePlan> plans[2];
    LaunchCfg cfg[2][2][hdg::kMaxN + 1];
    bool dirty = true;                         // plans out of date with the slots
    int64_t version = 0;                       // bumped on every membership change
    int64_t last_call_version = -1;            // membership of the previous stepping call
    // Completion of this batch's launches.  Every call that launches waits
    // for the previous call's event first when it runs on another stream, so
    // the calls form one chain and `done`, recorded behind the last call,
    // completes only after every launch the batch has made.  Tile lists, the
    // member table and the captured graph are rewritten or freed only once
    // the work that reads them is ordered before (same stream) or has
    // completed (host wait on `done`).
    hipEvent_t done = nullptr;
    bool done_recorded = false;
    hipStream_t last_stream = nullptr;
    // captured RK steps
    bool graphs = true;
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t g_version = -1;
    int g_prec = -1;
};

namespace {

hdg_status fail(hdg_status s, const std::string &msg) { return hdg::set_error(s, msg); }

// Wait until every launch this batch has made has completed.
void wait_idle(hdg_batch *b)
{
    if (b->done_recorded) (void)hipEventSynchronize(b->done);
}

// Order stream s after the batch's previous call (on whatever stream it ran).
hdg_status join_chain(hdg_batch *b, hipStream_t s)
{
    if (!b->done) HDG_HIP(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
    if (b->done_recorded && b->last_stream != s) HDG_HIP(hipStreamWaitEvent(s, b->done, 0));
    return HDG_OK;
}

hdg_status mark_done(hdg_batch *b, hipStream_t s)
{
    HDG_HIP(hipEventRecord(b->done, s));
    b->done_recorded = true;
    b->last_stream = s;
    return HDG_OK;
}

void free_plans(hdg_batch *b)
{
    wait_idle(b);
    for (auto &v : b->plans) {
        for (auto &pl : v) {
            if (pl.tiles) (void)hipFree(pl.tiles);
            if (pl.elems) (void)hipFree(pl.elems);
        }
        v.clear();
    }
}

void drop_graph(hdg_batch *b)
{
    // the executable may still be running its last replay
    if (b->gexec) {
        wait_idle(b);
        (void)hipGraphExecDestroy(b->gexec);
    }
    b->gexec = nullptr;
    b->g_version = -1;
    b->g_prec = -1;
}

const TilePlan *find_plan(const hdg_batch *b, int kind, int N, int B)
{
    for (const auto &pl : b->plans[kind])
        if (pl.N == N && pl.B == B && pl.ntiles > 0) return &pl;
    return nullptr;
}

// Device buffer of at least `need` items for a tile list, grown by doubling:
// the old buffer is freed only after the batch's launches have completed.
template <class T>
hdg_status ensure_capacity(hdg_batch *b, T *&buf, int64_t &cap, int64_t need)
{
    if (need <= cap) return HDG_OK;
    int64_t n = cap > 0 ? cap : 64;
    while (n < need) n *= 2;
    if (buf) {
        wait_idle(b);
        (void)hipFree(buf);
        buf = nullptr;
        cap = 0;
    }
    HDG_HIP(hipMalloc((void **)&buf, (size_t)n * sizeof(T)));
    cap = n;
    return HDG_OK;
}

// Tile lists over every member, for every (kind, order, workgroup size).
// A plan keeps its device buffers across membership changes (they only grow);
// the new lists are copied in on stream s, behind the batch's earlier
// launches (the chain on s), so no host wait is needed unless a buffer grows.
hdg_status rebuild_plans(hdg_batch *b, hipStream_t s)
{
    for (auto &v : b->plans)
        for (auto &pl : v) pl.ntiles = 0;
    for (int kind = 0; kind < 2; ++kind)
        for (int N = 2; N <= hdg::kMaxN; ++N)
            for (int B : hdg::kBlocks) {
                if (!hdg::shape_supported(N, B)) continue;
                std::vector<Tile> tiles;
                std::vector<int32_t> elems;
                for (size_t s = 0; s < b->slots.size(); ++s) {
                    const hdg_mesh *m = b->slots[s].mesh;
                    if (!m || (!m->mixed && m->N != N)) continue;
                    // a member of several orders gives this plan its order-N elements
                    const std::vector<int> &Ne = m->Ne;
                    std::vector<int> cls(m->ne);
                    for (int64_t e = 0; e < m->ne; ++e)
                        cls[e] = Ne[e] != N ? -1
                                 : kind == hdg::kTileViscous ? (m->flag[e] ? 1 : -1) : m->flag[e];
                    hdg::cut_tiles(m->order, Ne, cls, (int)s, B, kind, tiles, elems);
                }
                if (tiles.empty()) continue;
                TilePlan *pl = nullptr;
                for (auto &q : b->plans[kind])
                    if (q.N == N && q.B == B) pl = &q;
                if (!pl) {
                    b->plans[kind].emplace_back();
                    pl = &b->plans[kind].back();
                    pl->N = N;
                    pl->B = B;
                }
                hdg_status st = ensure_capacity(b, pl->tiles, pl->tiles_cap, (int64_t)tiles.size());
                if (st == HDG_OK) st = ensure_capacity(b, pl->elems, pl->elems_cap, (int64_t)elems.size());
                if (st != HDG_OK) return st;
                pl->ntiles = (int32_t)tiles.size();
                pl->chunk = (pl->ntiles + hdg::kXcd - 1) / hdg::kXcd;
                // host copies kept with the plan: the source of an asynchronous copy stays valid
                pl->h_tiles.swap(tiles);
                pl->h_elems.swap(elems);
                HDG_HIP(hipMemcpyAsync(pl->tiles, pl->h_tiles.data(), pl->h_tiles.size() * sizeof(Tile),
                                       hipMemcpyHostToDevice, s));
                HDG_HIP(hipMemcpyAsync(pl->elems, pl->h_elems.data(), pl->h_elems.size() * sizeof(int32_t),
                                       hipMemcpyHostToDevice, s));
            }
    b->dirty = false;
    for (auto &sl : b->slots) sl.stale = false;
    return HDG_OK;
}

// One fused RK stage of every member: viscous kernels of each order, then
// residual kernels.  Stage input is each member's qB if parity, else qA.
hdg_status batch_stage(hdg_batch *b, bool f32, double A, double B, int stage, int parity, hipStream_t s)
{
    for (int kind = 0; kind < 2; ++kind) {
        // members of several orders: their mortar kernels (BR1 lift before the
        // viscous kernels, numerical fluxes before the residual kernels), one
        // launch per member and pair of orders, reading the stage's input state
        for (size_t slot = 0; slot < b->slots.size(); ++slot) {
            const hdg_mesh *m = b->slots[slot].mesh;
            if (!m || m->mort_h.empty()) continue;
            for (int Nh = 3; Nh <= hdg::kMaxN; ++Nh)
                for (int Nl = 2; Nl < Nh; ++Nl) {
                    const int key = hdg::pair_key(Nl, Nh);
                    StageArgs a{};
                    a.mem = b->members + slot;
                    a.I64 = b->ctx->I64;
                    a.I32 = b->ctx->I32;
                    a.W64 = b->ctx->W64;
                    a.W32 = b->ctx->W32;
                    a.parity = parity;
                    a.mlist = m->mlist + m->mlist_off[kind][key];
                    a.mcount = (int32_t)(m->mlist_off[kind][key + 1] - m->mlist_off[kind][key]);
                    if (a.mcount == 0) continue;
                    (void)hipGetLastError();
                    const hipError_t e = hdg::launch_mortar(kind == 0, Nl, Nh, f32, a, s);
                    if (e != hipSuccess)
                        return fail(HDG_EHIP, std::string("batch mortar launch: ") + hipGetErrorString(e));
                }
        }
        for (int N = 2; N <= hdg::kMaxN; ++N) {
            const LaunchCfg &cf = b->cfg[kind][f32][N];
            const TilePlan *pl = find_plan(b, kind, N, cf.B);
            if (!pl) continue;
            StageArgs a{};
            a.mem = b->members;
            a.tiles = pl->tiles;
            a.elems = pl->elems;
            a.ntiles = pl->ntiles;
            a.chunk = pl->chunk;
            a.D64 = b->ctx->D64;
            a.D32 = b->ctx->D32;
            a.rkA = A;
            a.rkB = B;
            a.first_stage = stage == 0 ? 1 : 0;
            a.store_dq = stage == 2 ? 0 : 1;
            a.parity = parity;
            const int grid = hdg::launch_grid(*pl, kind, Epi::RkStage, f32, cf.persistent, b->ctx->n_cu);
            (void)hipGetLastError();
            hipError_t e = kind == hdg::kTileViscous ? hdg::launch_viscous(N, pl->B, f32, cf.persistent, a, grid, s)
                                                     : hdg::launch_residual(N, pl->B, Epi::RkStage, f32, cf.persistent, a, grid, s);
            if (e != hipSuccess) return fail(HDG_EHIP, std::string("batch kernel launch: ") + hipGetErrorString(e));
        }
    }
    return HDG_OK;
}

const double kA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
const double kB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

// nsteps RK steps from parity 0; returns the final parity (nsteps odd -> 1).
hdg_status batch_steps(hdg_batch *b, int32_t nsteps, bool f32, hipStream_t s)
{
    int parity = 0;
    for (int32_t step = 0; step < nsteps; ++step)
        for (int st = 0; st < 3; ++st) {
            hdg_status r = batch_stage(b, f32, kA[st], kB[st], st, parity, s);
            if (r != HDG_OK) return r;
            parity ^= 1;
        }
    return HDG_OK;
}

hdg_status check_batch(hdg_batch *b)
{
    if (!b) return fail(HDG_EINVAL, "NULL batch");
    HDG_HIP(hipSetDevice(b->ctx->device));
    return HDG_OK;
}

}  // namespace

extern "C" {

hdg_status hdg_batch_create(hdg_ctx *ctx, int32_t max_members, hdg_batch **out)
{
    if (!ctx || !out || max_members < 1) return fail(HDG_EINVAL, "batch_create: need a context and max_members >= 1");
    *out = nullptr;
    HDG_HIP(hipSetDevice(ctx->device));
    auto *b = new hdg_batch();
    b->ctx = ctx;
    b->slots.resize(max_members);
    for (auto &kc : b->cfg)
        for (auto &pc : kc)
            for (int N = 2; N <= hdg::kMaxN; ++N) pc[N] = hdg::default_cfg(N);
    hipError_t e = hipMalloc((void **)&b->members, sizeof(Member) * max_members);
    if (e != hipSuccess) {
        delete b;
        return fail(HDG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    e = hipMemset(b->members, 0, sizeof(Member) * max_members);
    if (e != hipSuccess) {
        (void)hipFree(b->members);
        delete b;
        return fail(HDG_EHIP, std::string("hipMemset: ") + hipGetErrorString(e));
    }
    hdg::ctx_retain(ctx);
    *out = b;
    return HDG_OK;
}

void hdg_batch_destroy(hdg_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    wait_idle(b);
    drop_graph(b);
    free_plans(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->done) (void)hipEventDestroy(b->done);
    (void)hipFree(b->members);
    hdg_ctx *ctx = b->ctx;
    delete b;
    hdg::ctx_release(ctx);
}

hdg_status hdg_batch_add(hdg_batch *b, hdg_mesh *m, double *q, double *dq, double dt, int32_t *slot)
{
    hdg_status st = check_batch(b);
    if (st != HDG_OK) return st;
    if (!m || !q || !dq || q == dq) return fail(HDG_EINVAL, "batch_add: need a mesh and distinct q, dq");
    if (m->ctx->device != b->ctx->device) return fail(HDG_EINVAL, "batch_add: mesh is on another device");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HDG_EINVAL, "batch_add: need dt > 0");
    // a free slot, preferably one no plan has referred to since the last
    // rebuild; launches in flight may read any slot of the member table, so
    // the record is written once the batch's launches have completed
    int32_t free_slot = -1;
    for (size_t s = 0; s < b->slots.size(); ++s) {
        if (b->slots[s].mesh == m) return fail(HDG_EINVAL, "batch_add: mesh is already a member");
        if (!b->slots[s].mesh && !b->slots[s].stale && free_slot < 0) free_slot = (int32_t)s;
    }
    if (free_slot < 0)
        for (size_t s = 0; s < b->slots.size() && free_slot < 0; ++s)
            if (!b->slots[s].mesh) free_slot = (int32_t)s;
    if (free_slot < 0) return fail(HDG_ENOMEM, "batch_add: no free slot");
    Member mb = m->host_member;
    mb.qA = q;
    mb.qB = m->qpp;
    mb.dq = dq;
    mb.dt = dt;
    wait_idle(b);
    HDG_HIP(hipMemcpy(b->members + free_slot, &mb, sizeof(Member), hipMemcpyHostToDevice));
    b->slots[free_slot] = hdg_batch::Slot{m, q, dq, dt, false};
    b->dirty = true;
    ++b->version;
    if (slot) *slot = free_slot;
    return HDG_OK;
}

hdg_status hdg_batch_remove(hdg_batch *b, int32_t slot)
{
    hdg_status st = check_batch(b);
    if (st != HDG_OK) return st;
    if (slot < 0 || slot >= (int32_t)b->slots.size() || !b->slots[slot].mesh)
        return fail(HDG_EINVAL, "batch_remove: no member in this slot");
    b->slots[slot] = hdg_batch::Slot{};
    b->slots[slot].stale = true;
    b->dirty = true;
    ++b->version;
    return HDG_OK;
}

hdg_status hdg_batch_info(const hdg_batch *b, int32_t *n_members, int64_t *n_elements, int64_t *n_nodes)
{
    if (!b) return fail(HDG_EINVAL, "NULL batch");
    int32_t nm = 0;
    int64_t ne = 0, nn = 0;
    for (const auto &s : b->slots)
        if (s.mesh) {
            ++nm;
            ne += s.mesh->ne;
            nn += s.mesh->nodes;
        }
    if (n_members) *n_members = nm;
    if (n_elements) *n_elements = ne;
    if (n_nodes) *n_nodes = nn;
    return HDG_OK;
}

hdg_status hdg_batch_rk3_steps(hdg_batch *b, int32_t nsteps, hdg_prec prec, void *stream)
{
    hdg_status st = check_batch(b);
    if (st != HDG_OK) return st;
    if (nsteps < 0) return fail(HDG_EINVAL, "batch_rk3_steps: nsteps >= 0");
    if (prec != HDG_F64 && prec != HDG_F32) return fail(HDG_EINVAL, "prec must be HDG_F64 or HDG_F32");
    hipStream_t s = (hipStream_t)stream;
    const bool f32 = prec == HDG_F32;
    st = join_chain(b, s);
    if (st != HDG_OK) return st;
    // membership as in the previous call: a captured graph pays off; right
    // after a change (a member joined or left) the steps run eagerly, so that
    // a stream of joins and leaves costs no capture and no host wait
    const bool stable = b->version == b->last_call_version;
    b->last_call_version = b->version;
    if (b->dirty) {
        drop_graph(b);
        st = rebuild_plans(b, s);
        if (st != HDG_OK) return st;
    }
    int32_t eager = nsteps;
    if (b->graphs && stable && nsteps >= 2) {
        if (!b->gexec || b->g_version != b->version || b->g_prec != (int)prec) {
            drop_graph(b);
            if (!b->cap) HDG_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
            for (int kind = 0; kind < 2; ++kind)
                for (int N = 2; N <= hdg::kMaxN; ++N) {
                    const LaunchCfg &cf = b->cfg[kind][f32][N];
                    if (const TilePlan *pl = find_plan(b, kind, N, cf.B))
                        (void)hdg::launch_grid(*pl, kind, Epi::RkStage, f32, cf.persistent, b->ctx->n_cu);
                }
            (void)hipGetLastError();
            std::lock_guard<std::mutex> device_lock(hdg::device_mutex());
            HDG_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
            hdg_status r = batch_steps(b, 2, f32, b->cap);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->cap, &g);
            if (r != HDG_OK) {
                if (g) (void)hipGraphDestroy(g);
                return r;
            }
            if (e != hipSuccess) return fail(HDG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                b->gexec = nullptr;
                return fail(HDG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            b->g_version = b->version;
            b->g_prec = (int)prec;
        }
        for (int32_t k = 0; k < nsteps / 2; ++k) {
            const hipError_t e = hipGraphLaunch(b->gexec, s);
            if (e != hipSuccess) {
                (void)mark_done(b, s);
                return fail(HDG_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
            }
        }
        eager = nsteps % 2;
    }
    st = batch_steps(b, eager, f32, s);
    if (st == HDG_OK && eager % 2) {
        // odd number of stages in total: the states sit in the ping-pong buffers
        for (const auto &sl : b->slots)
            if (sl.mesh && st == HDG_OK) {
                const hipError_t e = hipMemcpyAsync(sl.q, sl.mesh->qpp, (size_t)sl.mesh->nodes * 4 * sizeof(double),
                                                    hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) st = fail(HDG_EHIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
            }
    }
    // recorded whatever happened above, so that later waits cover every launch made
    const hdg_status md = mark_done(b, s);
    return st != HDG_OK ? st : md;
}

hdg_status hdg_batch_set_graphs(hdg_batch *b, int32_t enable)
{
    hdg_status st = check_batch(b);
    if (st != HDG_OK) return st;
    drop_graph(b);
    b->graphs = enable != 0;
    return HDG_OK;
}

hdg_status hdg_batch_autotune(hdg_batch *b, int32_t reps, void *stream)
{
    hdg_status st = check_batch(b);
    if (st != HDG_OK) return st;
    if (reps < 1) return fail(HDG_EINVAL, "batch_autotune: reps >= 1");
    hipStream_t s = (hipStream_t)stream;
    st = join_chain(b, s);
    if (st != HDG_OK) return st;
    drop_graph(b);
    if (b->dirty) {
        st = rebuild_plans(b, s);
        if (st != HDG_OK) return st;
    }
    hipEvent_t e0, e1;
    HDG_HIP(hipEventCreate(&e0));
    HDG_HIP(hipEventCreate(&e1));
    // a fused stage from each member's qA into its ping-pong buffer; it
    // writes each member's RK register, which holds nothing between steps
    for (int pi = 0; pi < 2 && st == HDG_OK; ++pi)
        for (int kind = 0; kind < 2 && st == HDG_OK; ++kind)
            for (int N = 2; N <= hdg::kMaxN && st == HDG_OK; ++N) {
                LaunchCfg best;
                best.us = -1.0;
                for (int B : hdg::kBlocks) {
                    const TilePlan *pl = find_plan(b, kind, N, B);
                    if (!pl) continue;
                    for (int pers = 1; pers >= 0 && st == HDG_OK; --pers) {
                        StageArgs a{};
                        a.mem = b->members;
                        a.tiles = pl->tiles;
                        a.elems = pl->elems;
                        a.ntiles = pl->ntiles;
                        a.chunk = pl->chunk;
                        a.D64 = b->ctx->D64;
                        a.D32 = b->ctx->D32;
                        a.rkA = 0.0;
                        a.rkB = 0.5;
                        a.first_stage = 1;
                        a.store_dq = 1;
                        a.parity = 0;
                        const int grid = hdg::launch_grid(*pl, kind, Epi::RkStage, pi == 1, pers != 0, b->ctx->n_cu);
                        auto once = [&]() -> hdg_status {
                            (void)hipGetLastError();
                            hipError_t e = kind == hdg::kTileViscous
                                               ? hdg::launch_viscous(N, B, pi == 1, pers != 0, a, grid, s)
                                               : hdg::launch_residual(N, B, Epi::RkStage, pi == 1, pers != 0, a, grid,
                                                                      s);
                            return e == hipSuccess ? HDG_OK : fail(HDG_EHIP, std::string("autotune launch: ") +
                                                                                 hipGetErrorString(e));
                        };
                        st = once();
                        if (st != HDG_OK) break;
                        if (hipEventRecord(e0, s) != hipSuccess) { st = fail(HDG_EHIP, "hipEventRecord"); break; }
                        for (int r = 0; r < reps && st == HDG_OK; ++r) st = once();
                        float ms = 0.0f;
                        if (st != HDG_OK || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                            if (st == HDG_OK) st = fail(HDG_EHIP, "autotune event timing");
                            break;
                        }
                        LaunchCfg cf;
                        cf.B = B;
                        cf.persistent = pers != 0;
                        cf.us = 1e3 * ms / reps;
                        if (best.us < 0.0 || cf.us < best.us) best = cf;
                    }
                }
                if (st == HDG_OK && best.us >= 0.0) b->cfg[kind][pi][N] = best;
            }
    const hdg_status md = mark_done(b, s);
    b->last_call_version = b->version;         // the next call at this membership may capture
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st != HDG_OK ? st : md;
}

hdg_status hdg_batch_get_launch(const hdg_batch *b, int32_t kernel_class, hdg_prec prec, int32_t N,
                                hdg_launch_cfg *out)
{
    if (!b || !out || kernel_class < 0 || kernel_class > HDG_KERNEL_RESIDUAL || (prec != HDG_F64 && prec != HDG_F32) ||
        N < 2 || N > hdg::kMaxN)
        return fail(HDG_EINVAL, "batch_get_launch: bad argument");
    const LaunchCfg &c = b->cfg[kernel_class][prec == HDG_F32][N];
    out->block = c.B;
    out->persistent = c.persistent ? 1 : 0;
    out->us_per_launch = c.us;
    return HDG_OK;
}

}  // extern "C"
