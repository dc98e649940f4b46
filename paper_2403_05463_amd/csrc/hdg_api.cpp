// C ABI of the hybrid NS-LES / Euler DGSEM residual library (declared in
// include/hdg.h): mesh ingest and validation, device buffers, the launch
// sequence of one residual / one RK stage, reductions and kernel timing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hdg_internal.h"

using hdg::ElemArgs;
using hdg::Epi;
using hdg::FaceRef;

namespace {

thread_local std::string g_err;

hdg_status fail(hdg_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HDG_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(HDG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

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

constexpr int kMaxEvents = 65536;

}  // namespace

struct hdg_ctx {
    int device;
};

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
    double *delta = nullptr, *Dmat = nullptr, *partials = nullptr, *final13 = nullptr;
    // FP32 copies (one rounding of the FP64 set-up) read by the HDG_F32 kernels
    float *metric32 = nullptr, *fgeo32 = nullptr, *Dmat32 = nullptr;
    FaceRef *conn = nullptr;
    uint8_t *flag_d = nullptr;
    int32_t *list_visc = nullptr, *list_all = nullptr;
    int nblocks_reduce = 0;
    int64_t bytes = 0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;            // pairs (start, stop)
    std::vector<int> ev_kind;
    size_t ev_used = 0;
};

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
    void *ptrs[] = {m->metric, m->fgeo, m->fvt, m->wvis, m->qpp, m->mass, m->delta, m->Dmat, m->partials,
                    m->final13, m->conn, m->flag_d, m->list_visc, m->list_all, m->metric32, m->fgeo32,
                    m->Dmat32};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (hipEvent_t e : m->ev) (void)hipEventDestroy(e);
    m->ev.clear();
}

hdg_status check_params(const hdg_params *p)
{
    if (!p) return fail(HDG_EINVAL, "params is NULL");
    if (!(p->c0sq > 0.0) || !(p->nu >= 0.0) || !(p->C_les >= 0.0))
        return fail(HDG_EINVAL, "params: need c0sq > 0, nu >= 0, C_les >= 0");
    if (p->les_model < 0 || p->les_model > 2) return fail(HDG_EINVAL, "params: les_model must be 0, 1 or 2");
    if (p->mixed_face != 0 && p->mixed_face != 1) return fail(HDG_EINVAL, "params: mixed_face must be 0 or 1");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(p->q_inf[k])) return fail(HDG_EINVAL, "params: q_inf not finite");
    return HDG_OK;
}

// Flagged-element list in the processing order, and the flags.
hdg_status upload_lists(hdg_mesh *m)
{
    std::vector<int32_t> v;
    for (int32_t e : m->order)
        if (m->flag[e]) v.push_back(e);
    m->n_visc = (int32_t)v.size();
    if (!v.empty()) HDG_HIP(hipMemcpy(m->list_visc, v.data(), v.size() * 4, hipMemcpyHostToDevice));
    HDG_HIP(hipMemcpy(m->flag_d, m->flag.data(), m->ne, hipMemcpyHostToDevice));
    return HDG_OK;
}

ElemArgs base_args(const hdg_mesh *m, bool f32)
{
    ElemArgs a{};
    a.metric = f32 ? (const void *)m->metric32 : (const void *)m->metric;
    a.fgeo = f32 ? (const void *)m->fgeo32 : (const void *)m->fgeo;
    a.conn = m->conn;
    a.flag = m->flag_d;
    a.fvt = m->fvt;
    a.wvis = m->wvis;
    a.delta = m->delta;
    a.Dmat = f32 ? (const void *)m->Dmat32 : (const void *)m->Dmat;
    a.c0sq = m->prm.c0sq;
    a.nu = m->prm.nu;
    a.C_les = m->prm.C_les;
    a.les_model = m->prm.les_model;
    a.mixed_face = m->prm.mixed_face;
    for (int k = 0; k < 4; ++k) a.qinf[k] = m->prm.q_inf[k];
    a.inv_wend = m->inv_wend;
    return a;
}

void set_list(ElemArgs &a, const int32_t *list, int32_t count)
{
    a.list = list;
    a.count = count;
    a.per_xcd = (count + hdg::kXcd - 1) / hdg::kXcd;
}

// Launch with optional event bracketing for the kernel timer.
template <class F>
hdg_status timed(hdg_mesh *m, int kind, hipStream_t s, F launch)
{
    const bool rec = m->timing && m->ev_used + 2 <= m->ev.size();
    if (rec) HDG_HIP(hipEventRecord(m->ev[m->ev_used], s));
    hipError_t e = launch();
    if (e != hipSuccess) return fail(HDG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    if (rec) {
        HDG_HIP(hipEventRecord(m->ev[m->ev_used + 1], s));
        m->ev_kind[m->ev_used / 2] = kind;
        m->ev_used += 2;
    }
    return HDG_OK;
}

// One residual evaluation (EPI Residual) or one fused RK stage (EPI RkStage).
hdg_status run_stage(hdg_mesh *m, const double *q, void *out, double *dq, Epi epi, bool f32, double A,
                     double B, double dt, bool first, hipStream_t s)
{
    ElemArgs a = base_args(m, f32);
    a.q = q;
    a.out = out;
    a.dq = dq;
    a.rkA = A;
    a.rkB = B;
    a.dt = dt;
    a.first_stage = first ? 1 : 0;
    ElemArgs av = a;
    set_list(av, m->list_visc, m->n_visc);
    hdg_status st = timed(m, HDG_KERNEL_VISCOUS, s, [&] { return hdg::launch_viscous(m->N, f32, av, s); });
    if (st != HDG_OK) return st;
    ElemArgs ar = a;
    set_list(ar, m->list_all, (int32_t)m->ne);
    return timed(m, HDG_KERNEL_RESIDUAL, s, [&] { return hdg::launch_residual(m->N, epi, f32, ar, s); });
}

// Sizes, pointers, uniform order, symmetric connectivity with mutually inverse
// orientation codes.
hdg_status validate_desc(const hdg_mesh_desc *d, int &P)
{
    if (d->n_elem <= 0 || !d->P || !d->xyz_geom || !d->flag || !d->nbr || !d->nbr_face || !d->orient)
        return fail(HDG_EINVAL, "mesh description: empty mesh or NULL array");
    if (d->geom_order < 1 || d->geom_order > 12) return fail(HDG_EINVAL, "geom_order must be 1..12");
    P = d->P[0];
    if (P < 1 || P > hdg::kMaxN - 1) return fail(HDG_EUNSUPPORTED, "polynomial order must be 1..7");
    const int64_t ne = d->n_elem;
    for (int64_t e = 0; e < ne; ++e)
        if (d->P[e] != P) return fail(HDG_EUNSUPPORTED, "non-uniform polynomial order");
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
    *ctx = new hdg_ctx{device};
    return HDG_OK;
}

void hdg_finalize(hdg_ctx *ctx) { delete ctx; }

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

    hdg::HostGeometry g;
    std::string msg;
    if (!hdg::build_geometry(*d, P, g, msg)) return fail(HDG_EMESH, msg);

    auto *m = new hdg_mesh();
    m->ctx = ctx;
    m->ne = ne;
    m->P = P;
    m->N = P + 1;
    m->N2 = m->N * m->N;
    m->N3 = m->N2 * m->N;
    m->prm = *params;
    m->inv_wend = 1.0 / g.w[0];
    m->flag.assign(d->flag, d->flag + ne);
    for (auto &f : m->flag) f = f ? 1 : 0;
    const int N = m->N, N2 = m->N2, N3 = m->N3;

    // canonical faces: the owner is the lower element id (lower local face on a tie)
    std::vector<int32_t> fid(ne * 6, -1);
    auto is_owner = [&](int64_t e, int f) {
        const int32_t e2 = d->nbr[e * 6 + f];
        if (e2 < 0) return true;
        const int f2 = d->nbr_face[e * 6 + f];
        return e < e2 || (e == e2 && f < f2);
    };
    int64_t nf = 0;
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f)
            if (is_owner(e, f)) fid[e * 6 + f] = (int32_t)nf++;
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f)
            if (!is_owner(e, f)) fid[e * 6 + f] = fid[(int64_t)d->nbr[e * 6 + f] * 6 + d->nbr_face[e * 6 + f]];
    m->nfaces = nf;
    std::vector<double> fgeo(nf * N2 * 4);
    std::vector<FaceRef> conn(ne * 6);
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f) {
            const bool own = is_owner(e, f);
            FaceRef &r = conn[e * 6 + f];
            r.face = fid[e * 6 + f];
            r.nbr = d->nbr[e * 6 + f];
            r.code = (r.nbr >= 0 ? (d->orient[e * 6 + f] & 7) | ((d->nbr_face[e * 6 + f] & 7) << 3) : 0) |
                     (own ? hdg::kOwnerBit : 0);
            r.pad = 0;
            if (!own) continue;
            const int i = f / 2;
            const double sg = (f & 1) ? 1.0 : -1.0;
            for (int b = 0; b < N; ++b)
                for (int a = 0; a < N; ++a) {
                    const int n = face_node(N, f, a, b);
                    double v[3];
                    for (int c = 0; c < 3; ++c) v[c] = sg * g.Ja[((e * 3 + i) * 3 + c) * N3 + n];
                    const double s = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                    double *o = &fgeo[((size_t)r.face * N2 + a + N * b) * 4];
                    o[0] = v[0] / s;
                    o[1] = v[1] / s;
                    o[2] = v[2] / s;
                    o[3] = s;
                }
        }
    std::vector<double> metric(ne * 10 * N3), mass(ne * N3);
    for (int64_t e = 0; e < ne; ++e)
        for (int n = 0; n < N3; ++n) {
            const double J = g.J[e * N3 + n];
            metric[(e * 10) * N3 + n] = 1.0 / J;
            for (int k = 0; k < 9; ++k) metric[(e * 10 + 1 + k) * N3 + n] = g.Ja[(e * 9 + k) * N3 + n];
            const int a = n % N, b = (n / N) % N, c = n / N2;
            mass[e * N3 + n] = g.w[a] * g.w[b] * g.w[c] * J;
        }
    m->x = std::move(g.x);
    m->order = hdg::locality_order(*d);
    m->nblocks_reduce = (int)std::min<int64_t>(1024, (ne * N3 + 255) / 256);

    hdg_status s2 = HDG_OK;
    auto chk = [&](hdg_status s) { if (s2 == HDG_OK) s2 = s; };
    chk(dev_alloc(m, &m->metric, metric.size()));
    chk(dev_alloc(m, &m->mass, mass.size()));
    chk(dev_alloc(m, &m->fgeo, fgeo.size()));
    chk(dev_alloc(m, &m->fvt, (size_t)nf * 2 * N2 * 3));
    chk(dev_alloc(m, &m->wvis, (size_t)ne * 3 * N3));
    chk(dev_alloc(m, &m->qpp, (size_t)ne * 4 * N3));
    chk(dev_alloc(m, &m->delta, (size_t)ne));
    chk(dev_alloc(m, &m->Dmat, (size_t)N2));
    chk(dev_alloc(m, &m->metric32, metric.size()));
    chk(dev_alloc(m, &m->fgeo32, fgeo.size()));
    chk(dev_alloc(m, &m->Dmat32, (size_t)N2));
    chk(dev_alloc(m, &m->partials, (size_t)m->nblocks_reduce * 13));
    chk(dev_alloc(m, &m->final13, 13));
    chk(dev_alloc(m, &m->conn, conn.size()));
    chk(dev_alloc(m, &m->flag_d, (size_t)ne));
    chk(dev_alloc(m, &m->list_visc, (size_t)ne));
    chk(dev_alloc(m, &m->list_all, (size_t)ne));
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
    chk(up(m->Dmat, g.D.data(), g.D.size() * 8));
    {
        std::vector<float> m32(metric.begin(), metric.end()), f32(fgeo.begin(), fgeo.end()),
            d32(g.D.begin(), g.D.end());
        chk(up(m->metric32, m32.data(), m32.size() * 4));
        chk(up(m->fgeo32, f32.data(), f32.size() * 4));
        chk(up(m->Dmat32, d32.data(), d32.size() * 4));
    }
    chk(up(m->conn, conn.data(), conn.size() * sizeof(FaceRef)));
    chk(up(m->list_all, m->order.data(), m->order.size() * sizeof(int32_t)));
    if (s2 == HDG_OK) s2 = upload_lists(m);
    if (s2 != HDG_OK) {
        free_device(m);
        delete m;
        return s2;
    }
    *out = m;
    return HDG_OK;
}

void hdg_mesh_destroy(hdg_mesh *m)
{
    if (!m) return;
    (void)hipSetDevice(m->ctx->device);
    (void)hipDeviceSynchronize();
    free_device(m);
    delete m;
}

hdg_status hdg_mesh_set_flags(hdg_mesh *m, const uint8_t *flag_host)
{
    if (!m || !flag_host) return fail(HDG_EINVAL, "NULL argument");
    HDG_HIP(hipSetDevice(m->ctx->device));
    HDG_HIP(hipDeviceSynchronize());
    for (int64_t e = 0; e < m->ne; ++e) m->flag[e] = flag_host[e] ? 1 : 0;
    return upload_lists(m);
}

hdg_status hdg_mesh_set_params(hdg_mesh *m, const hdg_params *params)
{
    if (!m) return fail(HDG_EINVAL, "NULL mesh");
    hdg_status st = check_params(params);
    if (st != HDG_OK) return st;
    m->prm = *params;
    return HDG_OK;
}

hdg_status hdg_mesh_info(const hdg_mesh *m, int64_t *n_nodes, int64_t *state_len, int64_t *device_bytes,
                         int32_t *n_viscous)
{
    if (!m) return fail(HDG_EINVAL, "NULL mesh");
    if (n_nodes) *n_nodes = m->ne * m->N3;
    if (state_len) *state_len = 4 * m->ne * m->N3;
    if (device_bytes) *device_bytes = m->bytes;
    if (n_viscous) *n_viscous = m->n_visc;
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
    if (!hdg::build_geometry(*d, P, g, msg)) return fail(HDG_EMESH, msg);
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
    return run_stage(m, (const double *)q, r, nullptr, Epi::Residual, prec == HDG_F32, 0.0, 0.0, 0.0, false,
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
    double *cur = q, *nxt = m->qpp;
    for (int32_t step = 0; step < nsteps; ++step)
        for (int st = 0; st < 3; ++st) {
            hdg_status r = run_stage(m, cur, nxt, dq, Epi::RkStage, prec == HDG_F32, A[st], B[st], dt, st == 0, s);
            if (r != HDG_OK) return r;
            std::swap(cur, nxt);
        }
    if (cur != q) HDG_HIP(hipMemcpyAsync(q, cur, (size_t)m->ne * 4 * m->N3 * 8, hipMemcpyDeviceToDevice, s));
    return HDG_OK;
}

hdg_status hdg_reduce(hdg_mesh *m, const double *r, double out_sum[4], double out_l2[4], double out_max[4],
                      void *stream)
{
    if (!m || !r) return fail(HDG_EINVAL, "NULL argument");
    HDG_HIP(hipSetDevice(m->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hdg::launch_reduce(m->N, r, m->mass, m->ne, m->partials, m->nblocks_reduce, m->final13, s);
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
