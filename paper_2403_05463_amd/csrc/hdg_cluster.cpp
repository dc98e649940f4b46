// Clustering of the flow into a viscous/rotational and an inviscid region
// (Sec. 2.1): node features from the BR1 gradient, a two-component Gaussian
// mixture fitted by EM on the device, element means of the memberships and
// the element regions that become the equation flags.
#include <cmath>
#include <cstring>

#include "hdg_host.h"

using hdg::GmmState;
using hdg::StageArgs;
using hdg::Tile;
using hdg::TilePlan;

namespace {

hdg_status fail(hdg_status s, const std::string &msg) { return hdg::set_error(s, msg); }

constexpr int kTolChunk = 8;   // EM iterations between convergence checks when a tolerance is set

// Tile plans over every element, one per order present, for the feature
// kernels; they do not depend on the flags, so they are made once.
hdg_status feature_plans(hdg_mesh *m)
{
    if (!m->feat_plans.empty()) return HDG_OK;
    std::lock_guard<std::mutex> device_lock(hdg::device_mutex());
    for (int N = 2; N <= hdg::kMaxN; ++N) {
        std::vector<int> cls(m->ne);
        bool any = false;
        for (int64_t e = 0; e < m->ne; ++e) {
            cls[e] = m->Ne[e] == N ? 0 : -1;
            any = any || cls[e] == 0;
        }
        if (!any) continue;
        TilePlan pl;
        pl.N = N;
        pl.B = hdg::feature_block(N);
        std::vector<Tile> tiles;
        std::vector<int32_t> elems;
        hdg::cut_tiles(m->order, m->Ne, cls, 0, pl.B, hdg::kTileViscous, tiles, elems);
        pl.ntiles = (int32_t)tiles.size();
        pl.chunk = (pl.ntiles + hdg::kXcd - 1) / hdg::kXcd;
        HDG_HIP(hipMalloc((void **)&pl.tiles, tiles.size() * sizeof(Tile)));
        HDG_HIP(hipMalloc((void **)&pl.elems, elems.size() * sizeof(int32_t)));
        m->feat_plans.push_back(pl);
        HDG_HIP(hipMemcpy(pl.tiles, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice));
        HDG_HIP(hipMemcpy(pl.elems, elems.data(), elems.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    return HDG_OK;
}

StageArgs base_args(const hdg_mesh *m, const double *q)
{
    StageArgs a{};
    a.mem = m->member;
    a.D64 = m->ctx->D64;
    a.D32 = m->ctx->D32;
    a.I64 = m->ctx->I64;
    a.I32 = m->ctx->I32;
    a.W64 = m->ctx->W64;
    a.W32 = m->ctx->W32;
    a.q_in = q;
    return a;
}

hdg_status gmm_scratch(hdg_mesh *m)
{
    if (m->gmm) return HDG_OK;
    std::lock_guard<std::mutex> device_lock(hdg::device_mutex());
    const int64_t want = (m->nodes + 255) / 256;
    m->gmm_nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(hdg::kMaxGmmBlocks, want));
    HDG_HIP(hipMalloc((void **)&m->gmm_partials, (size_t)m->gmm_nblocks * hdg::kGmmStats * sizeof(double)));
    HDG_HIP(hipMalloc((void **)&m->gmm_flags, (size_t)m->ne));
    HDG_HIP(hipMalloc((void **)&m->gmm, sizeof(GmmState)));
    m->bytes += (int64_t)((size_t)m->gmm_nblocks * hdg::kGmmStats * sizeof(double) + m->ne + sizeof(GmmState));
    return HDG_OK;
}

}  // namespace

extern "C" {

hdg_status hdg_cluster_features(hdg_mesh *m, const double *q, double *features, void *stream)
{
    if (!m || !q || !features) return fail(HDG_EINVAL, "cluster_features: NULL argument");
    HDG_HIP(hipSetDevice(m->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    hdg_status st = feature_plans(m);
    if (st != HDG_OK) return st;
    // BR1 lift of every mortar (the flux lists hold them all)
    if (!m->mort_h.empty())
        for (int Nh = 3; Nh <= hdg::kMaxN; ++Nh)
            for (int Nl = 2; Nl < Nh; ++Nl) {
                const int key = hdg::pair_key(Nl, Nh);
                StageArgs a = base_args(m, q);
                a.mlist = m->mlist + m->mlist_off[1][key];
                a.mcount = (int32_t)(m->mlist_off[1][key + 1] - m->mlist_off[1][key]);
                if (a.mcount == 0) continue;
                (void)hipGetLastError();
                HDG_HIP(hdg::launch_mortar(true, Nl, Nh, false, a, s));
            }
    for (const TilePlan &pl : m->feat_plans) {
        StageArgs a = base_args(m, q);
        a.tiles = pl.tiles;
        a.elems = pl.elems;
        a.ntiles = pl.ntiles;
        a.chunk = pl.chunk;
        a.r = features;
        a.nodes = m->nodes;
        const int grid = hdg::launch_grid(pl, hdg::kTileViscous, hdg::Epi::Residual, false, false, m->ctx->n_cu);
        (void)hipGetLastError();
        HDG_HIP(hdg::launch_features(pl.N, a, grid, s));
    }
    return HDG_OK;
}

hdg_status hdg_cluster_fit(hdg_mesh *m, const double *features, const hdg_gmm_opts *opts, hdg_gmm_result *res,
                           double *p_visc, double *elem_pv, uint8_t *flags, void *stream)
{
    if (!m || !features || !opts || !res || !flags) return fail(HDG_EINVAL, "cluster_fit: NULL argument");
    if (opts->iterations < 0 || opts->iterations > 100000 || !(opts->reg_covar >= 0.0) ||
        !std::isfinite(opts->reg_covar) || !(opts->tol >= 0.0) || !std::isfinite(opts->tol))
        return fail(HDG_EINVAL, "cluster_fit: need 0 <= iterations <= 100000, finite reg_covar >= 0 and tol >= 0");
    HDG_HIP(hipSetDevice(m->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    hdg_status st = gmm_scratch(m);
    if (st != HDG_OK) return st;
    const int64_t n = m->nodes;
    (void)hipGetLastError();
    for (int mode = 0; mode < 3; ++mode)
        HDG_HIP(hdg::launch_gmm_pass(mode, features, n, m->gmm, m->gmm_partials, m->gmm_nblocks, opts->reg_covar,
                                     opts->tol, s));
    // with a tolerance, iterations go in chunks and the device's convergence
    // flag is read between them, so a converged fit launches no more passes
    const int chunk = opts->tol > 0.0 ? kTolChunk : std::max(opts->iterations, 1);
    for (int it = 0; it < opts->iterations;) {
        const int end = std::min(opts->iterations, it + chunk);
        for (; it < end; ++it)
            HDG_HIP(hdg::launch_gmm_pass(3, features, n, m->gmm, m->gmm_partials, m->gmm_nblocks, opts->reg_covar,
                                         opts->tol, s));
        if (opts->tol > 0.0 && it < opts->iterations) {
            GmmState g;
            HDG_HIP(hipMemcpyAsync(&g, m->gmm, sizeof(GmmState), hipMemcpyDeviceToHost, s));
            HDG_HIP(hipStreamSynchronize(s));
            if (g.converged || g.degenerate) break;
        }
    }
    HDG_HIP(hdg::launch_gmm_assign(features, n, m->gmm, m->mixed ? m->eoff : nullptr, m->mixed ? m->Ne_d : nullptr,
                                   m->mixed ? 0 : m->N3, m->ne, p_visc, elem_pv, m->gmm_flags, s));
    GmmState g;
    HDG_HIP(hipMemcpyAsync(&g, m->gmm, sizeof(GmmState), hipMemcpyDeviceToHost, s));
    HDG_HIP(hipMemcpyAsync(flags, m->gmm_flags, (size_t)m->ne, hipMemcpyDeviceToHost, s));
    HDG_HIP(hipStreamSynchronize(s));

    std::memset(res, 0, sizeof(*res));
    for (int f = 0; f < 3; ++f) {
        res->feat_mean[f] = g.fm[f];
        res->feat_std[f] = g.fs[f];
    }
    res->degenerate = g.degenerate;
    if (g.degenerate) {
        res->weight[0] = 1.0;
        for (int k = 0; k < 2; ++k)
            for (int d = 0; d < 3; ++d) res->cov[k][d][d] = 1.0;
        res->log_likelihood = NAN;
    } else {
        const int vis = g.mu[0][2] > g.mu[1][2] ? 0 : 1;
        const int order[2] = {1 - vis, vis};
        static const int pk[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
        for (int j = 0; j < 2; ++j) {
            const int k = order[j];
            res->weight[j] = g.w[k];
            for (int a = 0; a < 3; ++a) {
                res->mean[j][a] = g.mu[k][a];
                for (int b = 0; b < 3; ++b) res->cov[j][a][b] = g.cov[k][pk[a][b]];
            }
        }
        res->log_likelihood = g.ll;
    }
    res->iterations = g.degenerate ? 0 : g.iter;
    res->converged = g.converged;
    int64_t nv = 0;
    for (int64_t e = 0; e < m->ne; ++e) nv += flags[e] != 0;
    res->n_viscous = nv;
    return HDG_OK;
}

}  // extern "C"
