// Internal declarations shared by the host set-up, the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hdg.h"

namespace hdg {

constexpr int kMaxN = 8;          // P <= 7
constexpr int kXcd = 8;           // MI355X: 8 accelerator complex dies, each with its own L2

// One record per (element, local face), consumed by the kernels.
struct FaceRef {
    int32_t face;     // conforming face: where its nodes start in the face geometry and viscous
                      // traces (one-order meshes: the canonical face id f, nodes from f N^2; meshes
                      // of mixed order: that first face node itself); mortar face: the mortar id
    int32_t nbr;      // neighbour element, or HDG_WALL / HDG_FARFIELD
    int32_t code;     // bits 0-2 orientation, bits 3-5 neighbour's local face, bit 6 owner
    int32_t nbr_off;  // meshes of mixed order, conforming face: the neighbour's first node; mortar
                      // face: the first value of the mortar's slab; else 0
};

constexpr int kOwnerBit = 1 << 6;   // conforming face: this side owns it; mortar: this is the higher side
constexpr int kMortarBit = 1 << 7;  // face between elements of different order: `face` is the mortar id,
                                    // `nbr_off` the first value of its slab, bits 0-3 of the code the
                                    // other side's order N
constexpr int kNbrViscBit = 1 << 8; // the neighbour is flagged (kept current with the flags), so a face
                                    // task issues its viscous-trace loads without first loading the flag

// A face between elements of different order, coupled through a mortar of
// the higher order in the higher side's face frame.  Its slab (values of the
// compute type) holds, at each side's own face nodes: viscous traces [3][N^2]
// (h, l), surface terms [4][N^2] (h, l), the higher side's mortar velocity
// u* - u_r [3][Nh^2] (its s n is the element's own) and the lower side's
// projected BR1 lift terms [9][Nl^2].
struct MortarRef {
    int32_t eh, fh, el, fl;  // higher / lower order element and local face
    int32_t Nh, Nl;          // nodes per direction on each side
    int32_t code_h;          // orientation code of the higher side (its face coords -> the lower side's)
    int32_t flags;           // list copies (mortar kernels): bit 0 higher side flagged, bit 1 lower side
    int64_t slab;            // first value of the slab
    int64_t geo;             // first mortar node in the mortar geometry [node][4]: n (higher side outward), s
    int64_t oh, ol;          // first node of each side's element (its state starts at 4 o)
};

__host__ __device__ constexpr int64_t mslab_tr(int Nh, int Nl, bool hi) { return hi ? 0 : 3 * Nh * Nh; }
__host__ __device__ constexpr int64_t mslab_surf(int Nh, int Nl, bool hi)
{
    return 3 * (Nh * Nh + Nl * Nl) + (hi ? 0 : 4 * Nh * Nh);
}
__host__ __device__ constexpr int64_t mslab_lift(int Nh, int Nl, bool hi)
{
    return 7 * (Nh * Nh + Nl * Nl) + (hi ? 0 : 3 * Nh * Nh);
}
__host__ __device__ constexpr int64_t mslab_size(int Nh, int Nl) { return 10 * Nh * Nh + 16 * Nl * Nl; }

// Mortar lists are kept per (Nl, Nh) pair, at key Nh (kMaxN + 1) + Nl.
constexpr int kPairKeys = (kMaxN + 1) * (kMaxN + 1);
__host__ __device__ constexpr int pair_key(int Nl, int Nh) { return Nh * (kMaxN + 1) + Nl; }

// Work is cut into tiles: up to tile_ept() elements of one polynomial order
// and one equation class, all from one member mesh, processed together by one
// workgroup of B lanes (element s of the tile owns lanes [s N^3, (s+1) N^3)).
struct Tile {
    int32_t member;         // index into the member table
    int32_t flag;           // equation flag shared by the tile's elements (residual and viscous tiles);
                            // the order is the kernel's, one plan per order
    int32_t count;          // elements in this tile (1 .. tile_ept)
    int32_t first;          // first entry in the element array
};

enum TileKind : int { kTileViscous = 0, kTileResidual = 1 };

// LDS budget of one workgroup of B lanes (eight 128-lane, four 256-lane,
// three 384-lane or two 512-lane workgroups share a 160 KB CU).
constexpr int tile_lds_budget(int B)
{
    return B <= 128 ? 20 * 1024 : B <= 256 ? 40 * 1024 : B <= 384 ? 52 * 1024 : 78 * 1024;
}

// Lanes per element: N^3 packed for N <= 3 (several elements share a wave),
// whole 64-lane waves from N = 4 on, so that the element is uniform per wave.
constexpr int tile_lanes(int N)
{
    const int n3 = N * N * N;
    return n3 < 64 ? n3 : (n3 + 63) / 64 * 64;
}

// Elements per tile for order N, workgroup size B and kernel kind, sized for
// FP64 LDS (the same tiles serve both precisions); 0 if an element needs more
// than B lanes.
constexpr int tile_ept(int N, int B, int kind)
{
    const int n3 = N * N * N, n2 = N * N;
    // FP64 LDS arrays plus the element id and six face records staged per tile
    const int per = (12 * n3 + (kind == kTileViscous ? 18 : 24) * n2) * 8 + 4 + 6 * 16;
    const int by_lanes = B / tile_lanes(N);
    const int by_lds = (tile_lds_budget(B) - n2 * 8) / per;
    return by_lanes < by_lds ? by_lanes : by_lds;
}

// Per-mesh data of the element kernels (device resident, one record per
// member mesh of a launch).  Element e's state starts at 4 eoff[e], its
// metric terms at 10 eoff[e], its viscous part at 3 eoff[e]; face f's
// geometry at 4 foff[f] and viscous traces at 6 foff[f].  Metric terms, face
// geometry and viscous scratch exist in FP64 and FP32; the kernel reads the
// copy of its compute type.
struct Member {
    double *qA, *qB;        // RK ping-pong states (qA is the caller's)
    double *dq;             // RK register
    const void *metric[2];  // [e][10][N^3]: 1/J, then Ja^i_d; [0] FP64, [1] FP32
    const void *fgeo[2];    // [face][N^2][4]: owner's unit outward normal, surface scale
    void *fvt;              // [face][2 sides][3][N^2]: viscous flux . (s n), side 0 = owner
    void *wvis;             // [e][3][N^3]: viscous part of the reference divergence
    const FaceRef *conn;    // [e][6]
    const uint8_t *flag;    // [e]
    const double *delta;    // [e] LES filter width
    const int64_t *moff;    // [e] first node of the metric block e reads (translates share one), or
                            // NULL: e's own, at its first node
    const int64_t *eoff;    // [e] first node of the element; NULL: e N^3 (one order)
    const int64_t *foff;    // [face] first face node of the face; NULL: face N^2.  Set on a mesh of
                            // mixed order, whose face records then hold these offsets themselves
    const MortarRef *mort;  // [mortar] faces between orders (NULL if none)
    void *mslab;            // mortar slabs (compute type)
    const void *mgeo[2];    // mortar geometry [node][4], FP64 and FP32
    double c0sq, nu, C_les, dt;
    double qinf[4];
    int32_t les_model, mixed_face;
    int32_t riemann;        // HDG_ROE or HDG_RUSANOV
    int32_t pad;
};

// Arguments of one persistent launch over a tile list.  With q_in set, the
// launch has a single member and reads/writes the given buffers (and dt);
// otherwise each member's ping-pong pair is selected by `parity`.
struct StageArgs {
    const Member *mem;
    const Tile *tiles;
    const int32_t *elems;   // member-local element ids, grouped by tile
    const int64_t *emo;     // per entry of elems: first node of the element's metric block (shared by its
                            // translates), or NULL: the member's own offsets
    const int64_t *eoe;     // per entry of elems: the element's first node (meshes of mixed order), or
                            // NULL: the member's offsets
    int32_t ntiles;
    int32_t chunk;          // tiles per XCD chunk; the grid is a multiple of kXcd
    const double *D64;      // derivative matrices for N = 2..8, packed at d_offset(N)
    const float *D32;
    const double *I64;      // interpolation matrices Nl -> Nh nodes, packed at i_offset(Nl, Nh)
    const float *I32;
    const double *W64;      // GLL weights of N nodes at w_offset(N)
    const float *W32;
    const MortarRef *mlist; // mortar kernels: records of this launch's mortars, in list order
    int32_t mcount;
    const double *q_in;     // single-member mode
    double *q_out;
    double *dq;
    void *r;                // residual output (compute type)
    double dt;
    double rkA, rkB;        // fused RK stage: dq = A dq + dt R; q_next = q + B dq
    int32_t first_stage;    // A = 0: dq is not read
    int32_t store_dq;       // 0: dq is not written (the step's last stage: the next stage, the first of
                            // a step, does not read it)
    int32_t parity;         // member mode: stage input is qB if set, else qA
    int64_t nodes;          // node features: stride of the [3][nodes] output at r
};

// Two-component Gaussian mixture over standardised node features (device
// resident, rewritten by each update so that EM iterations need no host).
// Component k: weight w, mean mu, covariance cov (packed xx, xy, xz, yy, yz,
// zz), the inverse Li of its lower Cholesky factor (packed 00, 10, 11, 20,
// 21, 22) and cst = 3/2 log(2 pi) + log det L.
struct GmmState {
    double fm[3], fs[3], fsi[3];   // feature means, scales (s_Q, s_Q^3/2, s_Q) and their inverses
    double w[2], logw[2];
    double mu[2][3];
    double cov[2][6];
    double Li[2][6];
    double cst[2];
    double ll;                     // mean log-likelihood of the last E-step
    int32_t degenerate;            // no node above the mean Q_Omega: no second region
    int32_t iter;                  // E-steps taken
    int32_t converged;             // the last change of ll was below the tolerance: later passes skip
    int32_t pad;
};
constexpr int kGmmStats = 21;      // per component: sum r, sum r d (3), sum r d d^T (6); + sum log-likelihood
constexpr int kMaxGmmBlocks = 1024; // workgroups of a mixture pass (partial sums per value); measured against 512 and 2048

// Offset of the N x N derivative matrix in the packed table (N = 2..8).
__host__ __device__ constexpr int d_offset(int N) { return (N - 1) * N * (2 * N - 1) / 6 - 1; }
constexpr int kDTableSize = d_offset(kMaxN + 1);
// Offset of the Nh x Nl interpolation matrix (2 <= Nl < Nh <= 8) and of the N weights.
__host__ __device__ constexpr int i_offset(int Nl, int Nh) { return (Nh * kMaxN + Nl) * kMaxN * kMaxN; }
constexpr int kITableSize = (kMaxN + 1) * kMaxN * kMaxN * kMaxN;
__host__ __device__ constexpr int w_offset(int N) { return N * kMaxN; }
constexpr int kWTableSize = (kMaxN + 1) * kMaxN;

enum class Epi : int { Residual = 0, RkStage = 1 };

// Kernel launchers (hdg_kernels.hip): one kernel per (kind, order N,
// workgroup size B, persistence) over a tile list of order-N tiles; grid of
// `grid` workgroups, a multiple of kXcd (non-persistent: kXcd * chunk or
// more).  Return hipSuccess or the launch error.
// With ev.start set, the dispatch itself records ev.start and ev.stop when
// the kernel starts and ends (the kernel timer: the span is the kernel's own
// duration, without the queue's gaps around it).
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
hipError_t launch_viscous(int N, int B, bool f32, bool persistent, const StageArgs &a, int grid, hipStream_t s,
                          const LaunchEvents &ev = {});
hipError_t launch_residual(int N, int B, Epi epi, bool f32, bool persistent, const StageArgs &a, int grid,
                           hipStream_t s, const LaunchEvents &ev = {});
// Mortar kernels of the pair (Nl, Nh) over the records a.mlist[0 .. a.mcount): the lift
// kernel (before the viscous kernels) forms the BR1 lift terms, the flux
// kernel (after them) the surface terms.  Only supported pairs launch.
bool mortar_pair_supported(int Nl, int Nh);
hipError_t launch_mortar(bool lift, int Nl, int Nh, bool f32, const StageArgs &a, hipStream_t s,
                         const LaunchEvents &ev = {});
// Reductions of a mesh of mixed order: element after element, eoff / Ne per element.
hipError_t launch_reduce_mixed(const double *r, const double *mass, const int64_t *eoff, const int8_t *Ne,
                               int64_t n_elem, double *partials, int nblocks, double *final13, hipStream_t s);
// Node features of every element (BR1 gradient invariants) over the order-N
// tiles of plan `a` (viscous-kind tiles, workgroup size feature_block(N)).
int feature_block(int N);
hipError_t launch_features(int N, const StageArgs &a, int grid, hipStream_t s);
// Gaussian mixture passes over n nodes of features X[3][n]: mode 0 feature
// sums, 1 squared deviations, 2 initial split, 3 E-step with statistics;
// each pass is followed by its update of *st (reg: covariance ridge; tol:
// an E-step pass whose log-likelihood changed by less ends the fit).
hipError_t launch_gmm_pass(int mode, const double *X, int64_t n, GmmState *st, double *partials, int nblocks,
                           double reg, double tol, hipStream_t s);
// Memberships p_v per node (optional), element means (optional) and element
// regions from the fitted mixture; element e has N3 nodes from e N3, or
// Ne[e]^3 from eoff[e] when eoff is set.
hipError_t launch_gmm_assign(const double *X, int64_t n, const GmmState *st, const int64_t *eoff, const int8_t *Ne,
                             int N3, int64_t ne, double *p_visc, double *elem_pv, uint8_t *flags, hipStream_t s);
// Resident workgroups per CU of a kernel configuration (occupancy query).
int resident_blocks_per_cu(int kind, int N, int B, Epi epi, bool f32);
// Whether kernels are instantiated for order N with workgroup size B.
bool shape_supported(int N, int B);
// Largest wave speed |u| + sqrt(|u|^2 + c0^2) over a state and a non-finite
// flag into final2[2] (nblocks partial pairs; element ranges as the reduction).
// eoff / Ne per element on a mesh of mixed order, else NULL and order N.
hipError_t launch_wave_speed(const double *q, const int64_t *eoff, const int8_t *Ne, int N, int64_t n_elem,
                             double c0sq, double *partials, int nblocks, double *final2, hipStream_t s);
hipError_t launch_reduce(int N, const double *r, const double *mass, int64_t n_elem,
                         double *partials, int nblocks, double *final13, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, int64_t nbytes, hipStream_t s);

// The allocation-free reduction keeps its partial sums in a device array of
// fixed size (kReduceScratchBlocks workgroups x 13 values) in hdg_kernels.hip.
// scratch_address gives its address on `device`, which must be current; the
// first call per device looks it up, later calls return the kept address.
constexpr int kReduceScratchBlocks = 1024;
constexpr int kMaxDevices = 64;
hipError_t scratch_address(int device, double **ptr);

// Host-side mesh geometry (hdg_setup.cpp), element after element: element e
// has Ne[e] nodes per direction and starts at node off[e].
struct HostGeometry {
    int N = 0, N3 = 0;                     // order of element 0 (all, on a one-order mesh)
    std::vector<int> Ne;
    std::vector<int64_t> off;
    int64_t nodes = 0;
    std::vector<double> xi, w, D;          // GLL rule and derivative matrix of element 0's order
    std::vector<double> xis[kMaxN + 1], ws[kMaxN + 1], Ds[kMaxN + 1];   // every order in use
    std::vector<double> x;                 // [e][3][Ne^3]
    std::vector<int64_t> moff;             // [e] first node of e's values in J and Ja: off[e], or with
                                           // translates sharing, the group's one slot
    std::vector<double> J;                 // [slot][Ne^3]
    std::vector<double> Ja;                // [slot][3][3][Ne^3]
    std::vector<double> delta;             // [e]
};

void gll_rule(int P, std::vector<double> &xi, std::vector<double> &w, std::vector<double> &D);
// Lagrange interpolation from the GLL nodes of order Plo to those of order
// Phi, I[i][k] = l_k(xi_i), evaluated in extended precision.
void gll_interp(int Plo, int Phi, std::vector<double> &I);
// Interpolate geometry to the GLL nodes of each element's order and build
// curl-form metric terms.  Returns false (with msg) on a non-positive Jacobian.
// With rep (metric_groups), an element other than its group's first copies
// that one's J, Ja and filter width instead of computing them; its node
// coordinates are its own.
// Metric terms where orders meet.  The curl-form product field
// V_k = x_l dx_m/dxi_k is restricted on the element boundary before its curl
// is taken, so that both sides of every face carry one polynomial s n:
//  - edge rule: on an edge around which the orders differ, the component
//    along the edge becomes its interpolant at the GLL points of degree
//    P_E - 1, P_E the lowest order around the edge;
//  - face rule: on a face between orders P_lo < P_hi, both sides give each
//    tangential component its interpolant of degree P_lo - 1 along its own
//    direction and P_lo across it (edge values along it from the edge rule).
// The face normal then has degree <= P_lo - 1 per face direction on both
// sides, which the mortar's exact integration against the lower side's basis
// reproduces (free stream); the discrete metric identities hold for any nodal
// V.  face[e][6] is P_lo on a face between orders, edge[e][12] is P_E on an
// edge where orders differ (edge k runs along xi^(k/4); bit 0 / bit 1 of k
// is the end of the lower / higher other direction), 0 elsewhere.
struct BoundaryOrders {
    std::vector<int8_t> face, edge;
    bool any = false;       // some face or edge is restricted
};
void boundary_orders(const hdg_mesh_desc &d, BoundaryOrders &b);
bool build_geometry(const hdg_mesh_desc &d, HostGeometry &g, std::string &msg,
                    const std::vector<int32_t> *rep = nullptr, const BoundaryOrders *bo = nullptr);
// Spatially local processing order of the elements (recursive bisection of
// centroids).  With rep (metric-sharing groups: rep[e] is the element whose
// metric block e reads), the groups are ordered by the bisection of their
// mean centroids and each group's elements follow one another, so that the
// block is read from HBM once and then from the cache.
std::vector<int32_t> locality_order(const hdg_mesh_desc &d, const std::vector<int32_t> *rep = nullptr);
// Elements that are translates of one another (same order, same restricted
// faces and edges, control points relative to the first one equal to 1e-12
// of the element's size) share one metric block: rep[e] is the first such
// element.  Returns the number of distinct blocks.
int64_t metric_groups(const hdg_mesh_desc &d, std::vector<int32_t> &rep, const BoundaryOrders *bo = nullptr);

}  // namespace hdg
