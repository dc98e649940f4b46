// Host-side state shared by the C ABI translation units: contexts, meshes,
// tile plans and launch configurations.
#pragma once

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "hdg_internal.h"

// The context's tables are shared by every mesh and batch made from it: it
// is reference counted (hdg_init and each successful create take a count,
// hdg_finalize and each destroy return one), so that the handles may be
// released in any order.
struct hdg_ctx {
    std::atomic<int> refs{1};
    int device = 0;
    int n_cu = 0;
    double *D64 = nullptr;     // derivative matrices for N = 2..8, packed at d_offset(N)
    float *D32 = nullptr;
    double *I64 = nullptr;     // interpolation matrices between orders, at i_offset(Nl, Nh)
    float *I32 = nullptr;
    double *W64 = nullptr;     // GLL weights, at w_offset(N)
    float *W32 = nullptr;
    double *scratch = nullptr; // this device's reduction scratch (kReduceScratchBlocks x 13 doubles)
};

namespace hdg {

inline void ctx_retain(hdg_ctx *c) { c->refs.fetch_add(1, std::memory_order_relaxed); }

// Returns one count; the last one frees the tables and the context.
inline void ctx_release(hdg_ctx *c)
{
    if (c->refs.fetch_sub(1, std::memory_order_acq_rel) != 1) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    void *ps[] = {c->D64, c->D32, c->I64, c->I32, c->W64, c->W32};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete c;
}

// Tile list of one kernel kind, one order N and one workgroup size, on the device.
struct TilePlan {
    int N = 0, B = 0;
    int32_t ntiles = 0, chunk = 0;
    Tile *tiles = nullptr;
    int32_t *elems = nullptr;
    int64_t *emo = nullptr;          // metric block of each entry of elems (meshes whose translates share one)
    int64_t *eoe = nullptr;          // first node of each entry's element (meshes of mixed order)
    // batches: device capacity (items) and the host copy of the last upload
    int64_t tiles_cap = 0, elems_cap = 0;
    std::vector<Tile> h_tiles;
    std::vector<int32_t> h_elems;
};

// Launch configuration of one (kernel kind, precision, order): workgroup size
// and grid (persistent: resident workgroups only, or one workgroup per tile).
struct LaunchCfg {
    int B = 512;
    bool persistent = true;
    double us = 0.0;           // measured mean launch time when tuned, else 0
};

// Split the elements (visited in `order`) into tiles of equal (N, class), each
// of at most tile_ept(N, B, kind) elements; tiles are ordered by the position
// of their first element, so the tile list keeps the spatial order.  Classes
// are 0 and 1 (-1: left out); a tile's class is stored as its flag.
inline void cut_tiles(const std::vector<int32_t> &order, const std::vector<int> &Ne, const std::vector<int> &cls,
               int member, int B, int kind, std::vector<Tile> &tiles, std::vector<int32_t> &elems)
{
    struct Chunk { size_t pos; int cls; std::vector<int32_t> e; };
    std::vector<Chunk> done;
    std::vector<Chunk> open(2 * (hdg::kMaxN + 1));
    std::vector<bool> has(open.size(), false);
    for (size_t r = 0; r < order.size(); ++r) {
        const int32_t e = order[r];
        if (cls[e] < 0) continue;
        const int key = cls[e] * (hdg::kMaxN + 1) + Ne[e];
        const int ept = hdg::tile_ept(Ne[e], B, kind);
        if (!has[key]) {
            open[key] = Chunk{r, cls[e], {}};
            has[key] = true;
        }
        open[key].e.push_back(e);
        if ((int)open[key].e.size() == ept) {
            done.push_back(std::move(open[key]));
            has[key] = false;
        }
    }
    for (size_t k = 0; k < open.size(); ++k)
        if (has[k]) done.push_back(std::move(open[k]));
    std::sort(done.begin(), done.end(), [](const Chunk &a, const Chunk &b) { return a.pos < b.pos; });
    for (auto &c : done) {
        tiles.push_back(Tile{member, c.cls, (int32_t)c.e.size(), (int32_t)elems.size()});
        elems.insert(elems.end(), c.e.begin(), c.e.end());
    }
}


// Workgroup sizes with kernels; 384 lanes (six waves) serve order 7, whose
// 343 nodes would leave a third of a 512-lane workgroup idle.
constexpr int kBlocks[4] = {128, 256, 384, 512};

// Untuned launch configuration of order N: the smallest workgroup that fits
// an element, one workgroup per tile.
inline LaunchCfg default_cfg(int N)
{
    LaunchCfg c;
    for (int B : kBlocks)
        if (tile_ept(N, B, kTileViscous) > 0 && tile_ept(N, B, kTileResidual) > 0) {
            c.B = B;
            break;
        }
    c.persistent = false;
    return c;
}
constexpr int kMaxEvents = 65536;

// Held while a HIP graph is captured and while a mesh allocates, uploads or
// frees device memory: those calls, made from another thread during a
// capture, invalidate it.
std::mutex &device_mutex();

// Set the thread's last-error message and return s.
hdg_status set_error(hdg_status s, const std::string &msg);

// Grid of a launch over plan pl: every tile, or (persistent) only as many
// workgroups as stay resident on n_cu CUs; a multiple of kXcd.
int launch_grid(const TilePlan &pl, int kind, Epi epi, bool f32, bool persistent, int n_cu);

}  // namespace hdg

#define HDG_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return hdg::set_error(HDG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define HDG_TRY(call)                                                                      \
    do {                                                                                   \
        const hdg_status st_ = (call);                                                     \
        if (st_ != HDG_OK) return st_;                                                     \
    } while (0)

namespace hdg {

// Side streams (default priority) and events for the independent launches of
// one phase of a stage; made once, outside any capture.
struct SideStreams {
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};

    hdg_status create()
    {
        if (fork) return HDG_OK;
        for (int i = 0; i < kSide; ++i) {
            HDG_HIP(hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking));
            HDG_HIP(hipEventCreateWithFlags(&join[i], hipEventDisableTiming));
        }
        HDG_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        return HDG_OK;
    }
    void destroy()
    {
        for (int i = 0; i < kSide; ++i) {
            if (side[i]) (void)hipStreamDestroy(side[i]);
            if (join[i]) (void)hipEventDestroy(join[i]);
            side[i] = nullptr;
            join[i] = nullptr;
        }
        if (fork) (void)hipEventDestroy(fork);
        fork = nullptr;
    }
};

// Launches of one phase of a stage that do not depend on each other (the
// mortar pairs, the orders): the first runs on the launch stream, later ones
// round-robin on side streams that first wait for the launch stream's work
// before the phase; end() joins them back.  Under capture the fork and join
// become graph edges, so the graph's branches may run concurrently.  With
// `par` false everything runs on the launch stream.
class Phase {
public:
    Phase(SideStreams &ss, hipStream_t s, bool par) : ss_(ss), s_(s), par_(par && ss.fork) {}
    hdg_status begin()
    {
        n_ = 0;
        if (par_) HDG_HIP(hipEventRecord(ss_.fork, s_));
        return HDG_OK;
    }
    // stream for the next launch
    hdg_status next(hipStream_t &st)
    {
        const int k = n_++;
        if (!par_ || k == 0) {
            st = s_;
            return HDG_OK;
        }
        const int i = (k - 1) % SideStreams::kSide;
        if (!used_[i]) {
            HDG_HIP(hipStreamWaitEvent(ss_.side[i], ss_.fork, 0));
            used_[i] = true;
        }
        st = ss_.side[i];
        return HDG_OK;
    }
    hdg_status end()
    {
        for (int i = 0; i < SideStreams::kSide; ++i)
            if (used_[i]) {
                HDG_HIP(hipEventRecord(ss_.join[i], ss_.side[i]));
                HDG_HIP(hipStreamWaitEvent(s_, ss_.join[i], 0));
                used_[i] = false;
            }
        return HDG_OK;
    }

private:
    SideStreams &ss_;
    hipStream_t s_;
    bool par_;
    int n_ = 0;
    bool used_[SideStreams::kSide] = {};
};

}  // namespace hdg

struct hdg_mesh {
    hdg_ctx *ctx = nullptr;
    int64_t ne = 0;
    int P = 0, N = 0, N2 = 0, N3 = 0;
    int64_t nfaces = 0;
    hdg_params prm{};
    double inv_wend = 0.0;
    std::vector<uint8_t> flag;
    std::vector<double> x;                 // node coordinates, host
    std::vector<int32_t> order;            // processing order
    int32_t n_visc = 0;
    // device buffers
    double *metric = nullptr, *fgeo = nullptr, *fvt = nullptr, *wvis = nullptr, *qpp = nullptr, *mass = nullptr;
    double *delta = nullptr, *partials = nullptr, *final13 = nullptr;
    // FP32 copies (one rounding of the FP64 set-up) read by the HDG_F32 kernels
    float *metric32 = nullptr, *fgeo32 = nullptr;
    hdg::FaceRef *conn = nullptr;
    std::vector<hdg::FaceRef> conn_h;              // host copy (neighbour-flag bits refreshed with the flags)
    std::vector<int64_t> moff_h;                   // host copy of moff (meshes with shared metric blocks)
    std::vector<int64_t> eoff_h;                   // host copy of eoff (meshes of mixed order)
    uint8_t *flag_d = nullptr;
    int64_t *moff = nullptr;                       // first node of each element's metric block (translates
                                                   // share one), or NULL: blocks in element order
    int64_t metric_blocks = 0;                     // distinct metric blocks
    int64_t *eoff = nullptr, *foff = nullptr;     // element / face offsets (meshes of mixed order)
    int8_t *Ne_d = nullptr;                        // per-element N (meshes of mixed order)
    bool mixed = false;                            // elements of more than one order
    std::vector<int> Ne;                           // per-element N
    int64_t nodes = 0;                             // total nodes
    // mortars (faces between orders)
    std::vector<hdg::MortarRef> mort_h;
    hdg::MortarRef *mort = nullptr;
    double *mslab = nullptr, *mgeo = nullptr;
    float *mgeo32 = nullptr;
    hdg::MortarRef *mlist = nullptr;               // mortar records, with the sides' current flags: lift
                                                   // lists, then flux lists, by (Nl, Nh)
    int64_t mlist_off[2][hdg::kPairKeys + 1] = {}; // [kind][pair_key] start in mlist (kind 0 lift, 1 flux)
    hdg::Member *member = nullptr;              // the mesh's member record (device)
    hdg::Member host_member{};
    // tile plans per kernel kind, for every (order, workgroup size) pair;
    // on a one-order mesh with flagged elements, the residual tiles of Euler
    // elements none of whose neighbours is flagged sit apart: they read nothing
    // the viscous kernel writes, so they run alongside it
    std::vector<hdg::TilePlan> plans[2];
    std::vector<hdg::TilePlan> plans_indep;
    hipStream_t indep_stream = nullptr;            // their stream (made at creation)
    hipEvent_t indep_fork = nullptr, indep_join = nullptr;
    // clustering, made on first use: feature tile plans over every element
    // (one per order) and the mixture's device state and scratch
    std::vector<hdg::TilePlan> feat_plans;
    hdg::GmmState *gmm = nullptr;
    double *gmm_partials = nullptr;
    uint8_t *gmm_flags = nullptr;
    int gmm_nblocks = 0;
    hdg::LaunchCfg cfg[2][2][hdg::kMaxN + 1];   // [kind][precision][N]
    int nblocks_reduce = 0;
    int64_t bytes = 0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;            // pairs (start, stop)
    std::vector<int> ev_kind;
    size_t ev_used = 0;
    // RK steps captured as a HIP graph (two steps, so the ping-pong state
    // ends where it started), replayed on the caller's stream
    bool graphs = true;
    hipStream_t cap = nullptr;             // private stream used only for capture
    hipEvent_t g_done = nullptr;           // recorded behind the last replay of gexec
    hdg::SideStreams ss;                   // for the independent launches of a stage's phases
    hipGraphExec_t gexec = nullptr;
    const double *g_q = nullptr;
    const double *g_dq = nullptr;
    double g_dt = 0.0;
    int g_prec = -1;
};
