// C ABI of the hybrid NS-LES / Euler DGSEM residual library (declared in
// include/hdg.h): mesh ingest and validation, device buffers, the launch
// sequence of one residual / one RK stage, reductions and kernel timing.
#include <algorithm>
#include <thread>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hdg_host.h"

using hdg::Epi;
using hdg::FaceRef;
using hdg::kBlocks;
using hdg::kMaxEvents;
using hdg::LaunchCfg;
using hdg::Member;
using hdg::StageArgs;
using hdg::Tile;
using hdg::TilePlan;

namespace {
thread_local std::string g_err;
}  // namespace

namespace hdg {

std::mutex &device_mutex()
{
    static std::mutex mu;
    return mu;
}

hdg_status set_error(hdg_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

int launch_grid(const TilePlan &pl, int kind, Epi epi, bool f32, bool persistent, int n_cu)
{
    int64_t g = pl.ntiles;
    if (persistent) {
        const int per_cu = resident_blocks_per_cu(kind, pl.N, pl.B, epi, f32);
        g = std::min<int64_t>(g, (int64_t)per_cu * n_cu);
    }
    g = (g + kXcd - 1) / kXcd * kXcd;
    return (int)std::max<int64_t>(g, kXcd);
}

}  // namespace hdg

namespace {

hdg_status fail(hdg_status s, const std::string &msg) { return hdg::set_error(s, msg); }

// fn(e) for every element on up to 16 host threads (elements interleaved);
// fn writes only what belongs to its element.
template <class F>
void parallel_elements(int64_t ne, F fn)
{
    const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
    const int nt = (int)std::min<int64_t>(std::min<int64_t>(16, hw), ne / 256 + 1);
    if (nt <= 1) {
        for (int64_t e = 0; e < ne; ++e) fn(e);
        return;
    }
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            for (int64_t e = t; e < ne; e += nt) fn(e);
        });
    for (auto &th : pool) th.join();
}

int face_node(int N, int f, int a, int b)
{
    const int s = (f & 1) ? N - 1 : 0, d = f / 2;
    return d == 0 ? s + N * (a + N * b) : d == 1 ? a + N * (s + N * b) : a + N * (b + N * s);
}

void orient_map(int o, int M, int a, int b, int &a2, int &b2)
{
    const int s = (o & 1) ? b : a, t = (o & 1) ? a : b;
    a2 = (o & 2) ? M - s : s;
    b2 = (o & 4) ? M - t : t;
}

}  // namespace



namespace {

template <class T>
hdg_status dev_alloc(hdg_mesh *m, T **p, size_t count)
{
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) return fail(HDG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    m->bytes += (int64_t)(count * sizeof(T));
    return HDG_OK;
}

void free_device(hdg_mesh *m)
{
    void *ptrs[] = {m->moff, m->metric, m->fgeo, m->fvt, m->wvis, m->qpp, m->mass, m->delta, m->partials,
                    m->final13, m->conn, m->flag_d, m->metric32, m->fgeo32, m->eoff, m->foff, m->member,
                    m->Ne_d, m->mort, m->mslab, m->mgeo, m->mgeo32, m->mlist, m->gmm, m->gmm_partials,
                    m->gmm_flags};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &pl : m->feat_plans) {
        if (pl.tiles) (void)hipFree(pl.tiles);
        if (pl.elems) (void)hipFree(pl.elems);
        if (pl.emo) (void)hipFree(pl.emo);
        if (pl.eoe) (void)hipFree(pl.eoe);
    }
    m->feat_plans.clear();
    for (auto &v : m->plans) {
        for (auto &pl : v) {
            if (pl.tiles) (void)hipFree(pl.tiles);
            if (pl.elems) (void)hipFree(pl.elems);
            if (pl.emo) (void)hipFree(pl.emo);
            if (pl.eoe) (void)hipFree(pl.eoe);
        }
        v.clear();
    }
    for (auto &pl : m->plans_indep) {
        if (pl.tiles) (void)hipFree(pl.tiles);
        if (pl.elems) (void)hipFree(pl.elems);
        if (pl.emo) (void)hipFree(pl.emo);
        if (pl.eoe) (void)hipFree(pl.eoe);
    }
    m->plans_indep.clear();
    if (m->indep_stream) (void)hipStreamDestroy(m->indep_stream);
    if (m->indep_fork) (void)hipEventDestroy(m->indep_fork);
    if (m->indep_join) (void)hipEventDestroy(m->indep_join);
    m->indep_stream = nullptr;
    m->indep_fork = m->indep_join = nullptr;
    for (hipEvent_t e : m->ev) (void)hipEventDestroy(e);
    m->ev.clear();
    if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
    if (m->cap) (void)hipStreamDestroy(m->cap);
    if (m->g_done) (void)hipEventDestroy(m->g_done);
    m->gexec = nullptr;
    m->cap = nullptr;
    m->g_done = nullptr;
    m->ss.destroy();
}

hdg_status check_params(const hdg_params *p)
{
    if (!p) return fail(HDG_EINVAL, "params is NULL");
    if (!(p->c0sq > 0.0) || !(p->nu >= 0.0) || !(p->C_les >= 0.0))
        return fail(HDG_EINVAL, "params: need c0sq > 0, nu >= 0, C_les >= 0");
    if (p->les_model < 0 || p->les_model > 2) return fail(HDG_EINVAL, "params: les_model must be 0, 1 or 2");
    if (p->mixed_face != 0 && p->mixed_face != 1) return fail(HDG_EINVAL, "params: mixed_face must be 0 or 1");
    if (p->riemann != HDG_ROE && p->riemann != HDG_RUSANOV)
        return fail(HDG_EINVAL, "params: riemann must be HDG_ROE or HDG_RUSANOV");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(p->q_inf[k])) return fail(HDG_EINVAL, "params: q_inf not finite");
    return HDG_OK;
}


const TilePlan *find_plan(const hdg_mesh *m, int kind, int N, int B)
{
    for (const auto &pl : m->plans[kind])
        if (pl.N == N && pl.B == B) return &pl;
    return nullptr;
}

// Drop the captured RK graph (its launches bake in plans, shapes and buffers).
void drop_graph(hdg_mesh *m)
{
    // the executable may still run (its branches on several streams): wait
    // for its last replay before destroying it
    if (m->gexec && m->g_done) (void)hipEventSynchronize(m->g_done);
    if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
    m->gexec = nullptr;
    m->g_prec = -1;
}

// Flags and the tile plans of every (order, workgroup size) the mesh uses.
hdg_status upload_plans(hdg_mesh *m)
{
    drop_graph(m);
    m->n_visc = 0;
    for (int64_t e = 0; e < m->ne; ++e) m->n_visc += m->flag[e];
    HDG_HIP(hipMemcpy(m->flag_d, m->flag.data(), m->ne, hipMemcpyHostToDevice));
    if (!m->conn_h.empty()) {
        for (FaceRef &r : m->conn_h) {
            r.code &= ~hdg::kNbrViscBit;
            if (r.nbr >= 0 && m->flag[r.nbr]) r.code |= hdg::kNbrViscBit;
        }
        HDG_HIP(hipMemcpy(m->conn, m->conn_h.data(), m->conn_h.size() * sizeof(FaceRef), hipMemcpyHostToDevice));
    }
    const std::vector<int> &Ne = m->Ne;
    std::vector<int> cls(m->ne);
    for (auto *v : {&m->plans[0], &m->plans[1], &m->plans_indep}) {
        for (auto &pl : *v) {
            if (pl.tiles) (void)hipFree(pl.tiles);
            if (pl.elems) (void)hipFree(pl.elems);
            if (pl.emo) (void)hipFree(pl.emo);
            if (pl.eoe) (void)hipFree(pl.eoe);
        }
        v->clear();
    }
    // Euler elements whose face neighbours are all Euler (one-order meshes
    // with flagged elements): their residual reads no viscous trace
    std::vector<uint8_t> indep(m->ne, 0);
    if (!m->mixed && m->n_visc > 0 && m->n_visc < m->ne)
        for (int64_t e = 0; e < m->ne; ++e) {
            bool ok = !m->flag[e];
            for (int f = 0; f < 6 && ok; ++f) {
                const int32_t nb = m->conn_h[e * 6 + f].nbr;
                ok = nb < 0 || !m->flag[nb];
            }
            indep[e] = ok ? 1 : 0;
        }
    // a handful of independent elements (a scattered mask: almost every Euler
    // element has a flagged neighbour) is not worth a launch and a fork of
    // its own
    int64_t n_indep = 0;
    for (int64_t e = 0; e < m->ne; ++e) n_indep += indep[e];
    if (16 * n_indep < m->ne) std::fill(indep.begin(), indep.end(), (uint8_t)0);
    for (int kind = 0; kind < 3; ++kind) {
        std::vector<hdg::TilePlan> &dst = kind == 2 ? m->plans_indep : m->plans[kind];
        for (int64_t e = 0; e < m->ne; ++e)
            cls[e] = kind == hdg::kTileViscous ? (m->flag[e] ? 1 : -1)
                     : kind == 1           ? (indep[e] ? -1 : m->flag[e])
                                           : (indep[e] ? 0 : -1);
        const int tkind = kind == hdg::kTileViscous ? hdg::kTileViscous : hdg::kTileResidual;
        for (int N = 2; N <= hdg::kMaxN; ++N) {
            std::vector<int> cn(m->ne);
            bool any = false;
            for (int64_t e = 0; e < m->ne; ++e) {
                cn[e] = Ne[e] == N ? cls[e] : -1;
                any = any || cn[e] >= 0;
            }
            if (!any) continue;
            for (int B : kBlocks) {
                if (!hdg::shape_supported(N, B)) continue;
                std::vector<Tile> tiles;
                std::vector<int32_t> elems;
                hdg::cut_tiles(m->order, Ne, cn, 0, B, tkind, tiles, elems);
                TilePlan pl;
                pl.N = N;
                pl.B = B;
                pl.ntiles = (int32_t)tiles.size();
                pl.chunk = (pl.ntiles + hdg::kXcd - 1) / hdg::kXcd;
                HDG_HIP(hipMalloc((void **)&pl.tiles, tiles.size() * sizeof(Tile)));
                HDG_HIP(hipMalloc((void **)&pl.elems, elems.size() * sizeof(int32_t)));
                HDG_HIP(hipMemcpy(pl.tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice));
                HDG_HIP(hipMemcpy(pl.elems, elems.data(), elems.size() * sizeof(int32_t), hipMemcpyHostToDevice));
                if (!m->moff_h.empty()) {
                    // the metric block of each entry next to its element id: the
                    // kernels' metric loads then wait for one load fewer
                    std::vector<int64_t> emo(elems.size());
                    for (size_t k = 0; k < elems.size(); ++k) emo[k] = m->moff_h[elems[k]];
                    HDG_HIP(hipMalloc((void **)&pl.emo, emo.size() * sizeof(int64_t)));
                    HDG_HIP(hipMemcpy(pl.emo, emo.data(), emo.size() * sizeof(int64_t), hipMemcpyHostToDevice));
                }
                if (m->mixed) {
                    // likewise each entry's first node, instead of a lookup in eoff
                    std::vector<int64_t> eoe(elems.size());
                    for (size_t k = 0; k < elems.size(); ++k) eoe[k] = m->eoff_h[elems[k]];
                    HDG_HIP(hipMalloc((void **)&pl.eoe, eoe.size() * sizeof(int64_t)));
                    HDG_HIP(hipMemcpy(pl.eoe, eoe.data(), eoe.size() * sizeof(int64_t), hipMemcpyHostToDevice));
                }
                dst.push_back(pl);
            }
        }
    }
    // mortar lists by (Nl, Nh): lift (a flagged side), flux (all); copies of
    // the records in list order, so that a mortar kernel loads its record
    // without first loading an id, with the sides' flags in `flags`
    if (!m->mort_h.empty()) {
        std::vector<hdg::MortarRef> lists;
        for (int kind = 0; kind < 2; ++kind)
            for (int key = 0; key <= hdg::kPairKeys; ++key) {
                m->mlist_off[kind][key] = (int64_t)lists.size();
                if (key == hdg::kPairKeys) continue;
                for (size_t k = 0; k < m->mort_h.size(); ++k) {
                    const hdg::MortarRef &r = m->mort_h[k];
                    if (hdg::pair_key(r.Nl, r.Nh) != key) continue;
                    if (kind == 0 && !m->flag[r.eh] && !m->flag[r.el]) continue;
                    hdg::MortarRef c = r;
                    c.flags = (m->flag[r.eh] ? 1 : 0) | (m->flag[r.el] ? 2 : 0);
                    lists.push_back(c);
                }
            }
        HDG_HIP(hipMemcpy(m->mlist, lists.data(), lists.size() * sizeof(hdg::MortarRef), hipMemcpyHostToDevice));
    }
    return HDG_OK;
}

void fill_member_params(Member &mb, const hdg_params &p)
{
    mb.c0sq = p.c0sq;
    mb.nu = p.nu;
    mb.C_les = p.C_les;
    mb.les_model = p.les_model;
    mb.mixed_face = p.mixed_face;
    mb.riemann = p.riemann;
    for (int k = 0; k < 4; ++k) mb.qinf[k] = p.q_inf[k];
}

hdg_status upload_member(hdg_mesh *m)
{
    fill_member_params(m->host_member, m->prm);
    HDG_HIP(hipMemcpy(m->member, &m->host_member, sizeof(Member), hipMemcpyHostToDevice));
    return HDG_OK;
}

int grid_for(const hdg_mesh *m, const TilePlan &pl, int kind, Epi epi, bool f32, bool persistent)
{
    return hdg::launch_grid(pl, kind, epi, f32, persistent, m->ctx->n_cu);
}

// Launch, with the kernel timer's events recorded by the dispatch itself
// (start and end of the kernel) while timing is on.
template <class F>
hdg_status timed(hdg_mesh *m, int kind, F launch)
{
    const bool rec = m->timing && m->ev_used + 2 <= m->ev.size();
    hdg::LaunchEvents ev;
    if (rec) {
        ev.start = m->ev[m->ev_used];
        ev.stop = m->ev[m->ev_used + 1];
    }
    (void)hipGetLastError();   // the launch check below must see this launch's status only
    hipError_t e = launch(ev);
    if (e != hipSuccess) return fail(HDG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    if (rec) {
        m->ev_kind[m->ev_used / 2] = kind;
        m->ev_used += 2;
    }
    return HDG_OK;
}

StageArgs stage_args(const hdg_mesh *m, const TilePlan &pl)
{
    StageArgs a{};
    a.mem = m->member;
    a.tiles = pl.tiles;
    a.elems = pl.elems;
    a.emo = pl.emo;
    a.eoe = pl.eoe;
    a.ntiles = pl.ntiles;
    a.chunk = pl.chunk;
    a.D64 = m->ctx->D64;
    a.D32 = m->ctx->D32;
    a.I64 = m->ctx->I64;
    a.I32 = m->ctx->I32;
    a.W64 = m->ctx->W64;
    a.W32 = m->ctx->W32;
    return a;
}

// One launch of kernel `kind` over the order-N tiles with configuration cf.
hdg_status launch_one(hdg_mesh *m, int kind, int N, const LaunchCfg &cf, const double *q, void *out, double *dq,
                      Epi epi, bool f32, double A, double B, double dt, int stage, hipStream_t s, bool time_it,
                      bool indep = false)
{
    const TilePlan *pl = nullptr;
    if (indep) {
        for (const auto &p : m->plans_indep)
            if (p.N == N && p.B == cf.B) pl = &p;
    } else {
        pl = find_plan(m, kind, N, cf.B);
    }
    if (!pl) return HDG_OK;
    StageArgs a = stage_args(m, *pl);
    a.q_in = q;
    a.q_out = epi == Epi::RkStage ? (double *)out : nullptr;
    a.r = epi == Epi::Residual ? out : nullptr;
    a.dq = dq;
    a.dt = dt;
    a.rkA = A;
    a.rkB = B;
    a.first_stage = stage == 0 ? 1 : 0;
    a.store_dq = stage == 2 ? 0 : 1;
    const int grid = grid_for(m, *pl, kind, epi, f32, cf.persistent);
    auto go = [&](const hdg::LaunchEvents &ev) {
        return kind == hdg::kTileViscous ? hdg::launch_viscous(N, pl->B, f32, cf.persistent, a, grid, s, ev)
                                         : hdg::launch_residual(N, pl->B, epi, f32, cf.persistent, a, grid, s, ev);
    };
    if (time_it) return timed(m, kind == hdg::kTileViscous ? HDG_KERNEL_VISCOUS : HDG_KERNEL_RESIDUAL, go);
    (void)hipGetLastError();
    hipError_t e = go(hdg::LaunchEvents{});
    if (e != hipSuccess) return fail(HDG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return HDG_OK;
}

// One residual evaluation (EPI Residual) or one fused RK stage (EPI RkStage):
// per kind (viscous, then residual) the mortar kernels of every pair of
// orders, then the element kernels of every order; launches within each of
// these four phases are independent.
hdg_status run_stage(hdg_mesh *m, const double *q, void *out, double *dq, Epi epi, bool f32, double A,
                     double B, double dt, int stage, hipStream_t s)
{
    const int pi = f32 ? 1 : 0;
    hdg::Phase ph(m->ss, s, !m->timing);
    // residual tiles that read nothing the viscous kernel writes run on their
    // own stream alongside the viscous kernel and the other residual tiles
    // (a parallel branch of a captured graph); serial while kernel timing is on
    const bool split = !m->plans_indep.empty();
    hipStream_t is = split && !m->timing ? m->indep_stream : s;
    if (split) {
        if (is != s) {
            HDG_HIP(hipEventRecord(m->indep_fork, s));
            HDG_HIP(hipStreamWaitEvent(is, m->indep_fork, 0));
        }
        for (int N = 2; N <= hdg::kMaxN; ++N)
            HDG_TRY(launch_one(m, 1, N, m->cfg[1][pi][N], q, out, dq, epi, f32, A, B, dt, stage, is, true, true));
        if (is != s) HDG_HIP(hipEventRecord(m->indep_join, is));
    }
    for (int kind = 0; kind < 2; ++kind) {
        // mortars: BR1 lift terms (kind 0) before the viscous kernels, numerical
        // fluxes (kind 1) after them and before the residual kernels
        if (!m->mort_h.empty()) {
            HDG_TRY(ph.begin());
            for (int Nh = 3; Nh <= hdg::kMaxN; ++Nh)
                for (int Nl = 2; Nl < Nh; ++Nl) {
                    const int key = hdg::pair_key(Nl, Nh);
                    StageArgs a{};
                    a.mem = m->member;
                    a.I64 = m->ctx->I64;
                    a.I32 = m->ctx->I32;
                    a.W64 = m->ctx->W64;
                    a.W32 = m->ctx->W32;
                    a.q_in = q;
                    a.mlist = m->mlist + m->mlist_off[kind][key];
                    a.mcount = (int32_t)(m->mlist_off[kind][key + 1] - m->mlist_off[kind][key]);
                    if (a.mcount == 0) continue;
                    hipStream_t ls;
                    HDG_TRY(ph.next(ls));
                    HDG_TRY(timed(m, HDG_KERNEL_MORTAR, [&](const hdg::LaunchEvents &ev) {
                        return hdg::launch_mortar(kind == 0, Nl, Nh, f32, a, ls, ev);
                    }));
                }
            HDG_TRY(ph.end());
        }
        HDG_TRY(ph.begin());
        for (int N = 2; N <= hdg::kMaxN; ++N) {
            if (!find_plan(m, kind, N, m->cfg[kind][pi][N].B)) continue;
            hipStream_t ls;
            HDG_TRY(ph.next(ls));
            HDG_TRY(launch_one(m, kind, N, m->cfg[kind][pi][N], q, out, dq, epi, f32, A, B, dt, stage, ls, true));
        }
        HDG_TRY(ph.end());
    }
    if (is != s) HDG_HIP(hipStreamWaitEvent(s, m->indep_join, 0));
    return HDG_OK;
}

// Sizes, pointers, uniform order, symmetric connectivity with mutually inverse
// orientation codes.
hdg_status validate_desc(const hdg_mesh_desc *d, int &P)
{
    if (d->n_elem <= 0 || !d->P || !d->xyz_geom || !d->flag || !d->nbr || !d->nbr_face || !d->orient)
        return fail(HDG_EINVAL, "mesh description: empty mesh or NULL array");
    if (d->geom_order < 1 || d->geom_order > 12) return fail(HDG_EINVAL, "geom_order must be 1..12");
    P = d->P[0];
    const int64_t ne = d->n_elem;
    for (int64_t e = 0; e < ne; ++e)
        if (d->P[e] < 1 || d->P[e] > hdg::kMaxN - 1) return fail(HDG_EUNSUPPORTED, "polynomial order must be 1..7");
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f) {
            const int32_t e2 = d->nbr[e * 6 + f];
            if (e2 < 0) {
                if (e2 != HDG_WALL && e2 != HDG_FARFIELD)
                    return fail(HDG_EMESH, "element " + std::to_string(e) + ": bad boundary code");
                continue;
            }
            const int f2 = d->nbr_face[e * 6 + f];
            if (e2 >= ne || f2 < 0 || f2 > 5 || d->nbr[(int64_t)e2 * 6 + f2] != e || d->nbr_face[(int64_t)e2 * 6 + f2] != f)
                return fail(HDG_EMESH, "element " + std::to_string(e) + " face " + std::to_string(f) +
                                           ": asymmetric connectivity");
            if (d->P[e2] != d->P[e] && std::min(d->P[e], d->P[e2]) < std::max(2, d->geom_order))
                return fail(HDG_EUNSUPPORTED, "element " + std::to_string(e) + " face " + std::to_string(f) +
                                                  ": a face between orders needs a lower order >= 2 and >= geom_order");
            if (d->P[e2] != d->P[e] &&
                !hdg::mortar_pair_supported(std::min(d->P[e], d->P[e2]) + 1, std::max(d->P[e], d->P[e2]) + 1))
                return fail(HDG_EUNSUPPORTED, "element " + std::to_string(e) + " face " + std::to_string(f) +
                                                  ": no mortar kernel for this pair of orders");
            const int o = d->orient[e * 6 + f], o2 = d->orient[(int64_t)e2 * 6 + f2];
            if (o < 0 || o > 7 || o2 < 0 || o2 > 7)
                return fail(HDG_EMESH, "element " + std::to_string(e) + ": orientation code out of range");
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    int a2, b2, a3, b3;
                    orient_map(o, 1, a, b, a2, b2);
                    orient_map(o2, 1, a2, b2, a3, b3);
                    if (a3 != a || b3 != b)
                        return fail(HDG_EMESH, "element " + std::to_string(e) + " face " + std::to_string(f) +
                                                   ": orientation codes are not inverse");
                }
        }
    return HDG_OK;
}

}  // namespace

extern "C" {

const char *hdg_last_error(void) { return g_err.c_str(); }

hdg_status hdg_init(hdg_ctx **ctx, int32_t device)
{
    if (!ctx) return fail(HDG_EINVAL, "ctx is NULL");
    int n = 0;
    HDG_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(HDG_EINVAL, "no such device " + std::to_string(device));
    HDG_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    HDG_HIP(hipGetDeviceProperties(&prop, device));
    double *scr = nullptr;
    const hipError_t es = hdg::scratch_address(device, &scr);
    if (es != hipSuccess) return fail(HDG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(es));
    auto *c = new hdg_ctx();
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    c->scratch = scr;
    // derivative matrices of every supported order, FP64 and one FP32 rounding
    std::vector<double> d64(hdg::kDTableSize);
    for (int N = 2; N <= hdg::kMaxN; ++N) {
        std::vector<double> xi, w, D;
        hdg::gll_rule(N - 1, xi, w, D);
        std::copy(D.begin(), D.end(), d64.begin() + hdg::d_offset(N));
    }
    std::vector<float> d32(d64.begin(), d64.end());
    // interpolation between the GLL nodes of two orders, and GLL weights
    std::vector<double> i64(hdg::kITableSize, 0.0), w64(hdg::kWTableSize, 0.0);
    for (int Nh = 3; Nh <= hdg::kMaxN; ++Nh)
        for (int Nl = 2; Nl < Nh; ++Nl) {
            std::vector<double> I;
            hdg::gll_interp(Nl - 1, Nh - 1, I);
            std::copy(I.begin(), I.end(), i64.begin() + hdg::i_offset(Nl, Nh));
        }
    for (int N = 2; N <= hdg::kMaxN; ++N) {
        std::vector<double> xi, w, D;
        hdg::gll_rule(N - 1, xi, w, D);
        std::copy(w.begin(), w.end(), w64.begin() + hdg::w_offset(N));
    }
    std::vector<float> i32(i64.begin(), i64.end()), w32(w64.begin(), w64.end());
    hipError_t e1 = hipMalloc((void **)&c->D64, d64.size() * 8);
    hipError_t e2 = hipMalloc((void **)&c->D32, d32.size() * 4);
    hipError_t e3 = hipMalloc((void **)&c->I64, i64.size() * 8);
    hipError_t e4 = hipMalloc((void **)&c->I32, i32.size() * 4);
    hipError_t e5 = hipMalloc((void **)&c->W64, w64.size() * 8);
    hipError_t e6 = hipMalloc((void **)&c->W32, w32.size() * 4);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess || e5 != hipSuccess ||
        e6 != hipSuccess) {
        void *ps[] = {c->D64, c->D32, c->I64, c->I32, c->W64, c->W32};
        for (void *p : ps)
            if (p) (void)hipFree(p);
        delete c;
        return fail(HDG_ENOMEM, "hipMalloc of the operator tables failed");
    }
    HDG_HIP(hipMemcpy(c->D64, d64.data(), d64.size() * 8, hipMemcpyHostToDevice));
    HDG_HIP(hipMemcpy(c->D32, d32.data(), d32.size() * 4, hipMemcpyHostToDevice));
    HDG_HIP(hipMemcpy(c->I64, i64.data(), i64.size() * 8, hipMemcpyHostToDevice));
    HDG_HIP(hipMemcpy(c->I32, i32.data(), i32.size() * 4, hipMemcpyHostToDevice));
    HDG_HIP(hipMemcpy(c->W64, w64.data(), w64.size() * 8, hipMemcpyHostToDevice));
    HDG_HIP(hipMemcpy(c->W32, w32.data(), w32.size() * 4, hipMemcpyHostToDevice));
    *ctx = c;
    return HDG_OK;
}

void hdg_finalize(hdg_ctx *ctx)
{
    if (ctx) hdg::ctx_release(ctx);
}

hdg_status hdg_mesh_create(hdg_ctx *ctx, const hdg_mesh_desc *d, const hdg_params *params, hdg_mesh **out)
{
    if (!ctx || !d || !out) return fail(HDG_EINVAL, "NULL argument");
    *out = nullptr;
    int P = 0;
    hdg_status st = validate_desc(d, P);
    if (st != HDG_OK) return st;
    st = check_params(params);
    if (st != HDG_OK) return st;
    const int64_t ne = d->n_elem;
    HDG_HIP(hipSetDevice(ctx->device));

    // translates share one metric block: group them first, so that set-up
    // computes each block once
    hdg::BoundaryOrders bo;
    hdg::boundary_orders(*d, bo);
    std::vector<int32_t> rep;
    const int64_t nblocks = hdg::metric_groups(*d, rep, &bo);
    const bool share = nblocks < ne;
    hdg::HostGeometry g;
    std::string msg;
    if (!hdg::build_geometry(*d, g, msg, share ? &rep : nullptr, &bo)) return fail(HDG_EMESH, msg);

    auto *m = new hdg_mesh();
    m->metric_blocks = nblocks;
    m->ctx = ctx;
    m->ne = ne;
    m->Ne = g.Ne;
    m->nodes = g.nodes;
    m->mixed = false;
    for (int64_t e = 0; e < ne; ++e) m->mixed = m->mixed || g.Ne[e] != g.Ne[0];
    m->P = m->mixed ? 0 : P;
    m->N = m->mixed ? 0 : P + 1;
    m->N2 = m->N * m->N;
    m->N3 = m->N2 * m->N;
    m->prm = *params;
    m->inv_wend = m->mixed ? 0.0 : 1.0 / g.w[0];
    for (auto &kc : m->cfg)
        for (auto &pc : kc)
            for (int n = 2; n <= hdg::kMaxN; ++n) pc[n] = hdg::default_cfg(n);
    m->flag.assign(d->flag, d->flag + ne);
    for (auto &f : m->flag) f = f ? 1 : 0;
    const std::vector<int> &Ne = g.Ne;
    const std::vector<int64_t> &off = g.off;
    auto Ja_at = [&](int64_t e, int i, int c, int n) {
        const int N = Ne[e];
        return g.Ja[9 * g.moff[e] + (int64_t)(i * 3 + c) * N * N * N + n];
    };

    // Faces.  A conforming face (both sides of one order) is canonical with
    // the lower element id as owner (lower local face on a tie); a face
    // between orders is a mortar named by its higher-order side.
    auto mortar_face = [&](int64_t e, int f) {
        const int32_t e2 = d->nbr[e * 6 + f];
        return e2 >= 0 && Ne[e2] != Ne[e];
    };
    std::vector<int32_t> fid(ne * 6, -1);
    auto is_owner = [&](int64_t e, int f) {
        const int32_t e2 = d->nbr[e * 6 + f];
        if (e2 < 0) return true;
        const int f2 = d->nbr_face[e * 6 + f];
        return e < e2 || (e == e2 && f < f2);
    };
    int64_t nf = 0, nfn = 0, nm = 0, slab = 0, geo = 0;
    std::vector<int64_t> foff;
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f) {
            if (mortar_face(e, f)) {
                const int64_t e2 = d->nbr[e * 6 + f];
                if (Ne[e] < Ne[e2]) continue;      // named from the higher side
                hdg::MortarRef r{};
                r.eh = (int32_t)e;
                r.fh = f;
                r.el = (int32_t)e2;
                r.fl = d->nbr_face[e * 6 + f];
                r.Nh = Ne[e];
                r.Nl = Ne[e2];
                r.code_h = d->orient[e * 6 + f] & 7;
                r.slab = slab;
                r.geo = geo;
                r.oh = off[e];
                r.ol = off[e2];
                slab += hdg::mslab_size(r.Nh, r.Nl);
                geo += (int64_t)r.Nh * r.Nh;
                fid[e * 6 + f] = (int32_t)nm;
                fid[e2 * 6 + r.fl] = (int32_t)nm;
                m->mort_h.push_back(r);
                ++nm;
            } else if (is_owner(e, f)) {
                fid[e * 6 + f] = (int32_t)nf++;
                foff.push_back(nfn);
                nfn += (int64_t)Ne[e] * Ne[e];
            }
        }
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f)
            if (!mortar_face(e, f) && !is_owner(e, f))
                fid[e * 6 + f] = fid[(int64_t)d->nbr[e * 6 + f] * 6 + d->nbr_face[e * 6 + f]];
    m->nfaces = nf;
    if (slab > INT32_MAX) {
        delete m;    // nothing on the device yet
        return fail(HDG_EUNSUPPORTED, "mortar slabs need fewer than 2^31 values");
    }
    std::vector<double> fgeo(std::max<int64_t>(nfn, 1) * 4), mgeo(std::max<int64_t>(geo, 1) * 4);
    std::vector<FaceRef> conn(ne * 6);
    auto put_normal = [&](double *o, int64_t e, int f, int n) {
        const int i = f / 2;
        const double sg = (f & 1) ? 1.0 : -1.0;
        double v[3];
        for (int c = 0; c < 3; ++c) v[c] = sg * Ja_at(e, i, c, n);
        const double sc = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        o[0] = v[0] / sc;
        o[1] = v[1] / sc;
        o[2] = v[2] / sc;
        o[3] = sc;
    };
    // records and face geometry, element by element (each owned face and each
    // mortar is written by one element only)
    parallel_elements(ne, [&](int64_t e) {
        for (int f = 0; f < 6; ++f) {
            FaceRef &r = conn[e * 6 + f];
            r.face = fid[e * 6 + f];
            r.nbr = d->nbr[e * 6 + f];
            r.nbr_off = 0;
            const int N = Ne[e];
            if (mortar_face(e, f)) {
                const bool hi = Ne[e] > Ne[r.nbr];
                // the other side's order and the slab travel in the record, so
                // that the element kernels need not load the mortar's
                r.code = hdg::kMortarBit | (hi ? hdg::kOwnerBit : 0) | Ne[r.nbr];
                r.nbr_off = (int32_t)m->mort_h[r.face].slab;
                if (hi) {
                    const hdg::MortarRef &mr = m->mort_h[r.face];
                    for (int b = 0; b < N; ++b)
                        for (int a = 0; a < N; ++a)
                            put_normal(&mgeo[(mr.geo + a + N * b) * 4], e, f, face_node(N, f, a, b));
                }
                continue;
            }
            const bool own = is_owner(e, f);
            r.code = (r.nbr >= 0 ? (d->orient[e * 6 + f] & 7) | ((d->nbr_face[e * 6 + f] & 7) << 3) : 0) |
                     (own ? hdg::kOwnerBit : 0);
            if (!own) continue;
            for (int b = 0; b < N; ++b)
                for (int a = 0; a < N; ++a)
                    put_normal(&fgeo[(foff[r.face] + a + N * b) * 4], e, f, face_node(N, f, a, b));
        }
    });
    // meshes of mixed order: a conforming face's record carries its first
    // face node and the neighbour's first node, so that the kernels' trace,
    // geometry and neighbour loads wait for no table lookup
    if (m->mixed) {
        if (g.nodes > INT32_MAX || nfn > INT32_MAX) {
            delete m;    // nothing on the device yet
            return fail(HDG_EUNSUPPORTED, "a mesh of mixed order needs fewer than 2^31 nodes and face nodes");
        }
        for (FaceRef &r : conn)
            if (!(r.code & hdg::kMortarBit)) {
                r.face = (int32_t)foff[r.face];
                if (r.nbr >= 0) r.nbr_off = (int32_t)off[r.nbr];
            }
    }
    // metric blocks: one per group of translates, [block][10][N^3]; moff[e] is
    // the first node of the block element e reads
    std::vector<int64_t> moff;
    int64_t mnodes = g.nodes;
    if (share) {
        moff.assign(ne, -1);
        mnodes = 0;
        for (int64_t e = 0; e < ne; ++e)
            if (rep[e] == e) {
                moff[e] = mnodes;
                mnodes += (int64_t)Ne[e] * Ne[e] * Ne[e];
            }
        for (int64_t e = 0; e < ne; ++e) moff[e] = moff[rep[e]];
    }
    std::vector<double> metric(mnodes * 10), mass(g.nodes);
    parallel_elements(ne, [&](int64_t e) {
        const int N = Ne[e], N3 = N * N * N;
        const std::vector<double> &w = g.ws[N];
        const bool first = !share || rep[e] == e;
        const int64_t mo = share ? moff[e] : off[e];
        for (int n = 0; n < N3; ++n) {
            const double J = g.J[g.moff[e] + n];
            if (first) {
                metric[10 * mo + n] = 1.0 / J;
                for (int k = 0; k < 9; ++k)
                    metric[10 * mo + (int64_t)(1 + k) * N3 + n] = g.Ja[9 * g.moff[e] + (int64_t)k * N3 + n];
            }
            const int a = n % N, b = (n / N) % N, c = n / (N * N);
            mass[off[e] + n] = w[a] * w[b] * w[c] * J;
        }
    });
    m->x = std::move(g.x);
    // the processing order keeps each group of translates together
    m->order = hdg::locality_order(*d, share ? &rep : nullptr);
    m->nblocks_reduce = (int)std::min<int64_t>(1024, (g.nodes + 255) / 256);
    m->nblocks_reduce = (int)std::min<int64_t>(m->nblocks_reduce, ne);

    std::lock_guard<std::mutex> device_lock(hdg::device_mutex());
    hdg_status s2 = HDG_OK;
    auto chk = [&](hdg_status s) { if (s2 == HDG_OK) s2 = s; };
    chk(dev_alloc(m, &m->metric, metric.size()));
    chk(dev_alloc(m, &m->mass, mass.size()));
    chk(dev_alloc(m, &m->fgeo, fgeo.size()));
    chk(dev_alloc(m, &m->fvt, (size_t)std::max<int64_t>(nfn, 1) * 6));
    chk(dev_alloc(m, &m->wvis, (size_t)g.nodes * 3));
    chk(dev_alloc(m, &m->qpp, (size_t)g.nodes * 4));
    chk(dev_alloc(m, &m->delta, (size_t)ne));
    chk(dev_alloc(m, &m->metric32, metric.size()));
    chk(dev_alloc(m, &m->fgeo32, fgeo.size()));
    chk(dev_alloc(m, &m->partials, (size_t)m->nblocks_reduce * 13));
    chk(dev_alloc(m, &m->final13, 13));
    chk(dev_alloc(m, &m->conn, conn.size()));
    if (share) chk(dev_alloc(m, &m->moff, (size_t)ne));
    chk(dev_alloc(m, &m->flag_d, (size_t)ne));
    chk(dev_alloc(m, &m->member, 1));
    if (m->mixed) {
        chk(dev_alloc(m, &m->eoff, (size_t)ne));
        chk(dev_alloc(m, &m->foff, foff.size()));
        chk(dev_alloc(m, &m->Ne_d, (size_t)ne));
    }
    if (nm > 0) {
        chk(dev_alloc(m, &m->mort, (size_t)nm));
        chk(dev_alloc(m, &m->mslab, (size_t)slab));       // FP64 slabs; FP32 ones use the first half
        chk(dev_alloc(m, &m->mgeo, mgeo.size()));
        chk(dev_alloc(m, &m->mgeo32, mgeo.size()));
        chk(dev_alloc(m, &m->mlist, (size_t)2 * nm));
    }
    if (s2 != HDG_OK) {
        free_device(m);
        delete m;
        return s2;
    }
    auto up = [&](void *dst, const void *src, size_t n) -> hdg_status {
        HDG_HIP(hipMemcpy(dst, src, n, hipMemcpyHostToDevice));
        return HDG_OK;
    };
    chk(up(m->metric, metric.data(), metric.size() * 8));
    chk(up(m->mass, mass.data(), mass.size() * 8));
    chk(up(m->fgeo, fgeo.data(), fgeo.size() * 8));
    chk(up(m->delta, g.delta.data(), g.delta.size() * 8));
    {
        std::vector<float> m32(metric.begin(), metric.end()), f32(fgeo.begin(), fgeo.end());
        chk(up(m->metric32, m32.data(), m32.size() * 4));
        chk(up(m->fgeo32, f32.data(), f32.size() * 4));
    }
    chk(up(m->conn, conn.data(), conn.size() * sizeof(FaceRef)));
    if (share) chk(up(m->moff, moff.data(), moff.size() * sizeof(int64_t)));
    if (share) m->moff_h = moff;
    if (m->mixed) m->eoff_h = off;
    m->conn_h = conn;
    if (m->mixed) {
        std::vector<int8_t> n8(Ne.begin(), Ne.end());
        chk(up(m->eoff, off.data(), off.size() * 8));
        chk(up(m->foff, foff.data(), foff.size() * 8));
        chk(up(m->Ne_d, n8.data(), n8.size()));
    }
    if (nm > 0) {
        std::vector<float> g32(mgeo.begin(), mgeo.end());
        chk(up(m->mort, m->mort_h.data(), m->mort_h.size() * sizeof(hdg::MortarRef)));
        chk(up(m->mgeo, mgeo.data(), mgeo.size() * 8));
        chk(up(m->mgeo32, g32.data(), g32.size() * 4));
    }
    {
        Member &mb = m->host_member;
        mb = Member{};
        mb.qA = nullptr;
        mb.qB = m->qpp;
        mb.metric[0] = m->metric;
        mb.metric[1] = m->metric32;
        mb.fgeo[0] = m->fgeo;
        mb.fgeo[1] = m->fgeo32;
        mb.fvt = m->fvt;
        mb.wvis = m->wvis;
        mb.conn = m->conn;
        mb.flag = m->flag_d;
        mb.delta = m->delta;
        mb.moff = m->moff;
        // one order: offsets are e N^3 and face N^2, no tables
        mb.eoff = m->mixed ? m->eoff : nullptr;
        mb.foff = m->mixed ? m->foff : nullptr;
        mb.mort = m->mort;
        mb.mslab = m->mslab;
        mb.mgeo[0] = m->mgeo;
        mb.mgeo[1] = m->mgeo32;
    }
    if (s2 == HDG_OK) s2 = upload_member(m);
    if (s2 == HDG_OK) s2 = upload_plans(m);
    // side streams for the concurrent phases, which only a mesh of several
    // orders has launches for; made here, never under a caller's capture, and
    // under the library mutex taken above for the uploads
    if (s2 == HDG_OK && m->mixed) s2 = m->ss.create();
    // the stream of the residual tiles that run alongside the viscous kernel
    if (s2 == HDG_OK && !m->mixed) {
        hipError_t e1 = hipStreamCreateWithFlags(&m->indep_stream, hipStreamNonBlocking);
        hipError_t e2 = hipEventCreateWithFlags(&m->indep_fork, hipEventDisableTiming);
        hipError_t e3 = hipEventCreateWithFlags(&m->indep_join, hipEventDisableTiming);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
            s2 = fail(HDG_EHIP, "stream or event creation for the independent residual tiles failed");
    }
    if (s2 != HDG_OK) {
        free_device(m);
        delete m;
        return s2;
    }
    hdg::ctx_retain(ctx);
    *out = m;
    return HDG_OK;
}

void hdg_mesh_destroy(hdg_mesh *m)
{
    if (!m) return;
    std::lock_guard<std::mutex> device_lock(hdg::device_mutex());
    (void)hipSetDevice(m->ctx->device);
    (void)hipDeviceSynchronize();
    free_device(m);
    hdg_ctx *ctx = m->ctx;
    delete m;
    hdg::ctx_release(ctx);
}

hdg_status hdg_mesh_set_flags(hdg_mesh *m, const uint8_t *flag_host)
{
    if (!m || !flag_host) return fail(HDG_EINVAL, "NULL argument");
    HDG_HIP(hipSetDevice(m->ctx->device));
    HDG_HIP(hipDeviceSynchronize());
    for (int64_t e = 0; e < m->ne; ++e) m->flag[e] = flag_host[e] ? 1 : 0;
    return upload_plans(m);
}

hdg_status hdg_mesh_set_params(hdg_mesh *m, const hdg_params *params)
{
    if (!m) return fail(HDG_EINVAL, "NULL mesh");
    hdg_status st = check_params(params);
    if (st != HDG_OK) return st;
    HDG_HIP(hipSetDevice(m->ctx->device));
    HDG_HIP(hipDeviceSynchronize());        // launches in flight read the member record
    m->prm = *params;
    drop_graph(m);
    return upload_member(m);
}

hdg_status hdg_mesh_info(const hdg_mesh *m, int64_t *n_nodes, int64_t *state_len, int64_t *device_bytes,
                         int32_t *n_viscous)
{
    if (!m) return fail(HDG_EINVAL, "NULL mesh");
    if (n_nodes) *n_nodes = m->nodes;
    if (state_len) *state_len = 4 * m->nodes;
    if (device_bytes) *device_bytes = m->bytes;
    if (n_viscous) *n_viscous = m->n_visc;
    return HDG_OK;
}

hdg_status hdg_mesh_metric_blocks(const hdg_mesh *m, int64_t *blocks)
{
    if (!m || !blocks) return fail(HDG_EINVAL, "NULL argument");
    *blocks = m->metric_blocks;
    return HDG_OK;
}

hdg_status hdg_mesh_node_coords(const hdg_mesh *m, double *xyz)
{
    if (!m || !xyz) return fail(HDG_EINVAL, "NULL argument");
    std::memcpy(xyz, m->x.data(), m->x.size() * sizeof(double));
    return HDG_OK;
}

hdg_status hdg_mesh_geometry(const hdg_mesh_desc *d, double *xyz, double *J, double *Ja, double *xi, double *w,
                             double *D)
{
    if (!d) return fail(HDG_EINVAL, "NULL description");
    int P = 0;
    hdg_status st = validate_desc(d, P);
    if (st != HDG_OK) return st;
    hdg::HostGeometry g;
    std::string msg;
    if (!hdg::build_geometry(*d, g, msg)) return fail(HDG_EMESH, msg);
    for (int64_t e = 0; e < d->n_elem; ++e)
        if (g.Ne[e] != g.Ne[0] && (xi || w || D))
            return fail(HDG_EUNSUPPORTED, "geometry: xi, w and D are per order; pass NULL for a mesh of mixed order");
    if (xyz) std::memcpy(xyz, g.x.data(), g.x.size() * sizeof(double));
    if (J) std::memcpy(J, g.J.data(), g.J.size() * sizeof(double));
    if (Ja) std::memcpy(Ja, g.Ja.data(), g.Ja.size() * sizeof(double));
    if (xi) std::memcpy(xi, g.xi.data(), g.xi.size() * sizeof(double));
    if (w) std::memcpy(w, g.w.data(), g.w.size() * sizeof(double));
    if (D) std::memcpy(D, g.D.data(), g.D.size() * sizeof(double));
    return HDG_OK;
}

hdg_status hdg_residual(hdg_mesh *m, const void *q, void *r, hdg_prec prec, void *stream)
{
    if (!m || !q || !r) return fail(HDG_EINVAL, "NULL argument");
    if (q == r) return fail(HDG_EINVAL, "residual must not alias the state");
    if (prec != HDG_F64 && prec != HDG_F32) return fail(HDG_EINVAL, "prec must be HDG_F64 or HDG_F32");
    HDG_HIP(hipSetDevice(m->ctx->device));
    return run_stage(m, (const double *)q, r, nullptr, Epi::Residual, prec == HDG_F32, 0.0, 0.0, 0.0, 1,
                     (hipStream_t)stream);
}

hdg_status hdg_rk3_steps(hdg_mesh *m, double *q, double *dq, double dt, int32_t nsteps, hdg_prec prec,
                         void *stream)
{
    static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    static const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    if (!m || !q || !dq) return fail(HDG_EINVAL, "NULL argument");
    if (q == dq) return fail(HDG_EINVAL, "dq must not alias q");
    if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0) return fail(HDG_EINVAL, "need dt > 0 and nsteps >= 0");
    if (prec != HDG_F64 && prec != HDG_F32) return fail(HDG_EINVAL, "prec must be HDG_F64 or HDG_F32");
    HDG_HIP(hipSetDevice(m->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const bool f32 = prec == HDG_F32;
    auto one_step = [&](double *&cur, double *&nxt, hipStream_t st_) -> hdg_status {
        for (int st = 0; st < 3; ++st) {
            hdg_status r = run_stage(m, cur, nxt, dq, Epi::RkStage, f32, A[st], B[st], dt, st, st_);
            if (r != HDG_OK) return r;
            std::swap(cur, nxt);
        }
        return HDG_OK;
    };
    int32_t eager = nsteps;
    if (m->graphs && !m->timing && nsteps >= 2) {
        // two RK steps (six stages) per replay: q -> qpp -> q ... ends in q
        if (!m->gexec || m->g_q != q || m->g_dq != dq || m->g_dt != dt || m->g_prec != (int)prec) {
            drop_graph(m);
            if (!m->cap) HDG_HIP(hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking));
            if (!m->g_done) HDG_HIP(hipEventCreateWithFlags(&m->g_done, hipEventDisableTiming));
            // occupancy queries happen before capture, not inside it
            for (int kind = 0; kind < 2; ++kind)
                for (int N = 2; N <= hdg::kMaxN; ++N) {
                    const LaunchCfg &cf = m->cfg[kind][f32][N];
                    if (const TilePlan *pl = find_plan(m, kind, N, cf.B))
                        (void)grid_for(m, *pl, kind, Epi::RkStage, f32, cf.persistent);
                }
            (void)hipGetLastError();
            std::lock_guard<std::mutex> device_lock(hdg::device_mutex());
            HDG_HIP(hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal));
            double *cur = q, *nxt = m->qpp;
            hdg_status r = one_step(cur, nxt, m->cap);
            if (r == HDG_OK) r = one_step(cur, nxt, m->cap);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(m->cap, &g);
            if (r != HDG_OK) {
                if (g) (void)hipGraphDestroy(g);
                return r;
            }
            if (e != hipSuccess) return fail(HDG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&m->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                m->gexec = nullptr;
                return fail(HDG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            m->g_q = q;
            m->g_dq = dq;
            m->g_dt = dt;
            m->g_prec = (int)prec;
        }
        for (int32_t k = 0; k < nsteps / 2; ++k) HDG_HIP(hipGraphLaunch(m->gexec, s));
        HDG_HIP(hipEventRecord(m->g_done, s));
        eager = nsteps % 2;
    }
    double *cur = q, *nxt = m->qpp;
    for (int32_t step = 0; step < eager; ++step) {
        hdg_status r = one_step(cur, nxt, s);
        if (r != HDG_OK) return r;
    }
    if (cur != q) HDG_HIP(hipMemcpyAsync(q, cur, (size_t)m->nodes * 4 * 8, hipMemcpyDeviceToDevice, s));
    return HDG_OK;
}

hdg_status hdg_mesh_set_graphs(hdg_mesh *m, int32_t enable)
{
    if (!m) return fail(HDG_EINVAL, "NULL mesh");
    HDG_HIP(hipSetDevice(m->ctx->device));
    drop_graph(m);
    m->graphs = enable != 0;
    return HDG_OK;
}

hdg_status hdg_reduce(hdg_mesh *m, const double *r, double out_sum[4], double out_l2[4], double out_max[4],
                      void *stream)
{
    if (!m || !r) return fail(HDG_EINVAL, "NULL argument");
    HDG_HIP(hipSetDevice(m->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = m->mixed ? hdg::launch_reduce_mixed(r, m->mass, m->eoff, m->Ne_d, m->ne, m->partials,
                                                       m->nblocks_reduce, m->final13, s)
                            : hdg::launch_reduce(m->N, r, m->mass, m->ne, m->partials, m->nblocks_reduce, m->final13, s);
    if (e != hipSuccess) return fail(HDG_EHIP, std::string("reduce launch: ") + hipGetErrorString(e));
    double h[13];
    HDG_HIP(hipMemcpyAsync(h, m->final13, sizeof h, hipMemcpyDeviceToHost, s));
    HDG_HIP(hipStreamSynchronize(s));
    for (int f = 0; f < 4; ++f) {
        if (out_sum) out_sum[f] = h[f];
        if (out_l2) out_l2[f] = std::sqrt(h[4 + f]);
        if (out_max) out_max[f] = h[8 + f];
    }
    if (h[12] != 0.0) return fail(HDG_ENONFINITE, "non-finite value in reduced array");
    return HDG_OK;
}

hdg_status hdg_max_wave_speed(hdg_mesh *m, const double *q, double *out, void *stream)
{
    if (!m || !q || !out) return fail(HDG_EINVAL, "max_wave_speed: NULL argument");
    HDG_HIP(hipSetDevice(m->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // the reduction's partial and result buffers (one call at a time per mesh,
    // as for hdg_reduce)
    hipError_t e = hdg::launch_wave_speed(q, m->mixed ? m->eoff : nullptr, m->mixed ? m->Ne_d : nullptr, m->N, m->ne,
                                          m->prm.c0sq, m->partials, m->nblocks_reduce, m->final13, s);
    if (e != hipSuccess) return fail(HDG_EHIP, std::string("wave speed launch: ") + hipGetErrorString(e));
    double h[2];
    HDG_HIP(hipMemcpyAsync(h, m->final13, sizeof h, hipMemcpyDeviceToHost, s));
    HDG_HIP(hipStreamSynchronize(s));
    *out = h[0];
    if (h[1] != 0.0) return fail(HDG_ENONFINITE, "non-finite velocity in the state");
    return HDG_OK;
}

hdg_status hdg_reduce_noalloc(hdg_mesh *m, const double *r, double *out, void *stream)
{
    if (!m || !r || !out) return fail(HDG_EINVAL, "reduce_noalloc: NULL argument");
    if (!m->ctx->scratch) return fail(HDG_EHIP, "reduce_noalloc: no scratch address on this device");
    if (m->nblocks_reduce > hdg::kReduceScratchBlocks)
        return fail(HDG_EUNSUPPORTED, "reduce_noalloc: the mesh needs " + std::to_string(m->nblocks_reduce) +
                                          " partial sums per value, the scratch holds " +
                                          std::to_string(hdg::kReduceScratchBlocks));
    HDG_HIP(hipSetDevice(m->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // the same kernels and workgroup count as hdg_reduce, with the partials in
    // the device's scratch array and the 13 results in the caller's buffer
    hipError_t e = m->mixed ? hdg::launch_reduce_mixed(r, m->mass, m->eoff, m->Ne_d, m->ne, m->ctx->scratch,
                                                       m->nblocks_reduce, out, s)
                            : hdg::launch_reduce(m->N, r, m->mass, m->ne, m->ctx->scratch, m->nblocks_reduce, out, s);
    if (e != hipSuccess) return fail(HDG_EHIP, std::string("reduce launch: ") + hipGetErrorString(e));
    return HDG_OK;
}

hdg_status hdg_timing_enable(hdg_mesh *m, int32_t enable)
{
    if (!m) return fail(HDG_EINVAL, "NULL mesh");
    HDG_HIP(hipSetDevice(m->ctx->device));
    if (enable && m->ev.empty()) {
        m->ev.resize(kMaxEvents);
        m->ev_kind.assign(kMaxEvents / 2, -1);
        for (auto &e : m->ev) HDG_HIP(hipEventCreate(&e));
    }
    m->timing = enable != 0;
    m->ev_used = 0;
    return HDG_OK;
}

hdg_status hdg_timing_read(hdg_mesh *m, int32_t kind, double *total_ms, int64_t *launches)
{
    if (!m || kind < 0 || kind >= HDG_KERNEL_COUNT) return fail(HDG_EINVAL, "bad argument");
    HDG_HIP(hipSetDevice(m->ctx->device));
    double tot = 0.0;
    int64_t cnt = 0;
    if (m->ev_used > 0) HDG_HIP(hipEventSynchronize(m->ev[m->ev_used - 1]));
    for (size_t p = 0; p < m->ev_used / 2; ++p) {
        if (m->ev_kind[p] != kind) continue;
        float ms = 0.0f;
        HDG_HIP(hipEventElapsedTime(&ms, m->ev[2 * p], m->ev[2 * p + 1]));
        tot += ms;
        ++cnt;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    return HDG_OK;
}

hdg_status hdg_timing_samples(hdg_mesh *m, int32_t kind, float *us, int64_t capacity, int64_t *count)
{
    if (!m || !count || kind < 0 || kind >= HDG_KERNEL_COUNT || capacity < 0 || (capacity > 0 && !us))
        return fail(HDG_EINVAL, "timing_samples: bad argument");
    HDG_HIP(hipSetDevice(m->ctx->device));
    if (m->ev_used > 0) HDG_HIP(hipEventSynchronize(m->ev[m->ev_used - 1]));
    int64_t cnt = 0;
    for (size_t p = 0; p < m->ev_used / 2; ++p) {
        if (m->ev_kind[p] != kind) continue;
        if (cnt < capacity) {
            float ms = 0.0f;
            HDG_HIP(hipEventElapsedTime(&ms, m->ev[2 * p], m->ev[2 * p + 1]));
            us[cnt] = ms * 1000.0f;
        }
        ++cnt;
    }
    *count = cnt;
    return HDG_OK;
}

hdg_status hdg_mesh_autotune(hdg_mesh *m, const double *q, int32_t reps, void *stream)
{
    if (!m || !q || reps < 1) return fail(HDG_EINVAL, "autotune: need a mesh, a state and reps >= 1");
    HDG_HIP(hipSetDevice(m->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const size_t nq = (size_t)m->nodes * 4;     // every order: the RK register of the whole mesh
    double *dq = nullptr;
    HDG_HIP(hipMalloc((void **)&dq, nq * sizeof(double)));
    hipEvent_t e0, e1;
    hdg_status st = HDG_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = fail(HDG_EHIP, "hipEventCreate");
    if (st == HDG_OK && hipMemsetAsync(dq, 0, nq * sizeof(double), s) != hipSuccess) st = fail(HDG_EHIP, "hipMemsetAsync");
    const bool was_timing = m->timing;
    m->timing = false;
    drop_graph(m);
    // a whole RK stage as the RK driver runs it (every launch, with the
    // concurrent branches), so that each choice is timed in the company it
    // keeps; the next state goes to the internal ping-pong buffer, which a
    // later step overwrites.  Residual kernels first, then viscous ones.
    for (int pi = 0; pi < 2 && st == HDG_OK; ++pi)
        for (int kind : {1, 0}) {
            if (st != HDG_OK) break;
            for (int N = 2; N <= hdg::kMaxN && st == HDG_OK; ++N) {
                LaunchCfg best;
                best.us = -1.0;
                for (int B : kBlocks) {
                    if (!find_plan(m, kind, N, B)) continue;
                    for (int pers = 1; pers >= 0 && st == HDG_OK; --pers) {
                        LaunchCfg cf;
                        cf.B = B;
                        cf.persistent = pers != 0;
                        m->cfg[kind][pi][N] = cf;
                        auto once = [&] {
                            return run_stage(m, q, m->qpp, dq, Epi::RkStage, pi == 1, -0.5, 0.5, 1e-9, 1, s);
                        };
                        st = once();
                        // the least of three timings of reps stages back to back:
                        // other work on the device only ever adds time
                        cf.us = -1.0;
                        for (int trial = 0; trial < 3 && st == HDG_OK; ++trial) {
                            if (hipEventRecord(e0, s) != hipSuccess) { st = fail(HDG_EHIP, "hipEventRecord"); break; }
                            for (int r = 0; r < reps && st == HDG_OK; ++r) st = once();
                            if (st != HDG_OK) break;
                            float ms = 0.0f;
                            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                                st = fail(HDG_EHIP, "autotune event timing");
                                break;
                            }
                            const double us = 1e3 * ms / reps;
                            if (cf.us < 0.0 || us < cf.us) cf.us = us;
                        }
                        if (st != HDG_OK) break;
                        if (best.us < 0.0 || cf.us < best.us) best = cf;
                    }
                }
                if (best.us >= 0.0) m->cfg[kind][pi][N] = best;
            }
        }
    m->timing = was_timing;
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(dq);
    return st;
}

hdg_status hdg_mesh_get_launch(const hdg_mesh *m, int32_t kernel_class, hdg_prec prec, int32_t N, hdg_launch_cfg *out)
{
    if (!m || !out || kernel_class < 0 || kernel_class > HDG_KERNEL_RESIDUAL || (prec != HDG_F64 && prec != HDG_F32) ||
        N < 2 || N > hdg::kMaxN)
        return fail(HDG_EINVAL, "get_launch: bad argument");
    const LaunchCfg &c = m->cfg[kernel_class][prec == HDG_F32][N];
    out->block = c.B;
    out->persistent = c.persistent ? 1 : 0;
    out->us_per_launch = c.us;
    return HDG_OK;
}

hdg_status hdg_mesh_set_launch(hdg_mesh *m, int32_t kernel_class, hdg_prec prec, int32_t N, const hdg_launch_cfg *cfg)
{
    if (!m || !cfg || kernel_class < 0 || kernel_class > HDG_KERNEL_RESIDUAL || (prec != HDG_F64 && prec != HDG_F32) ||
        N < 2 || N > hdg::kMaxN)
        return fail(HDG_EINVAL, "set_launch: bad argument");
    if (!hdg::shape_supported(N, cfg->block)) return fail(HDG_EUNSUPPORTED, "set_launch: no kernel for this order and block");
    drop_graph(m);
    LaunchCfg &c = m->cfg[kernel_class][prec == HDG_F32][N];
    c.B = cfg->block;
    c.persistent = cfg->persistent != 0;
    c.us = 0.0;
    return HDG_OK;
}

hdg_status hdg_stream_copy(hdg_ctx *ctx, void *dst, const void *src, int64_t nbytes, void *stream)
{
    if (!ctx || !dst || !src || nbytes < 0 || (nbytes % 16) != 0 || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16))
        return fail(HDG_EINVAL, "copy: need 16-byte aligned pointers and a multiple of 16 bytes");
    HDG_HIP(hipSetDevice(ctx->device));
    hipError_t e = hdg::launch_copy(dst, src, nbytes, (hipStream_t)stream);
    if (e != hipSuccess) return fail(HDG_EHIP, std::string("copy launch: ") + hipGetErrorString(e));
    return HDG_OK;
}

}  // extern "C"
