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
    int32_t face;   // canonical face id: index into face geometry and viscous traces
    int32_t nbr;    // neighbour element, or HDG_WALL / HDG_FARFIELD
    int32_t code;   // bits 0-2 orientation, bits 3-5 neighbour's local face, bit 6 owner
    int32_t pad;
};

constexpr int kOwnerBit = 1 << 6;

// Arguments of every element kernel (plain pointers, all device memory).
// The state, the RK register and the RK stage are always FP64; metric terms,
// face geometry, derivative matrix, viscous scratch and a residual output
// are in the kernel's compute type (double, or float for HDG_F32).
struct ElemArgs {
    const double *q;        // state in, [e][4][N^3]
    void *out;              // residual [e][4][N^3] (compute type), or the next RK state (double)
    double *dq;             // RK register (fused stage only)
    const void *metric;     // [e][10][N^3]: 1/J, then Ja^i_d for i = 0..2, d = 0..2
    const void *fgeo;       // [face][N^2][4]: unit normal (outward for the owner), surface scale s
    const FaceRef *conn;    // [e][6]
    const uint8_t *flag;    // [e]
    void *fvt;              // [face][2 sides][3][N^2]: viscous flux . (s n), side 0 = owner
    void *wvis;             // [e][3][N^3]: viscous part of the reference divergence (flagged elements)
    const int32_t *list;    // elements handled by this launch
    const double *delta;    // [e] LES filter width
    const void *Dmat;       // [N][N] derivative matrix, D[i][j] = l_j'(xi_i)
    int32_t count;          // entries in list
    int32_t per_xcd;        // list entries per XCD (grid = kXcd * per_xcd)
    double c0sq, nu, C_les;
    int32_t les_model, mixed_face;
    double qinf[4];
    double inv_wend;        // 1 / w_0 (end-point quadrature weight)
    double rkA, rkB, dt;    // fused RK stage: dq = A dq + dt R; q_next = q + B dq
    int32_t first_stage;    // A = 0: dq is not read
};

enum class Epi : int { Residual = 0, RkStage = 1 };

// Kernel launchers (hdg_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_viscous(int N, bool f32, const ElemArgs &a, hipStream_t s);
hipError_t launch_residual(int N, Epi epi, bool f32, const ElemArgs &a, hipStream_t s);
hipError_t launch_reduce(int N, const double *r, const double *mass, int64_t n_elem,
                         double *partials, int nblocks, double *final13, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, int64_t nbytes, hipStream_t s);

// Host-side mesh geometry (hdg_setup.cpp).
struct HostGeometry {
    int N = 0, N3 = 0;
    std::vector<double> xi, w, D;          // GLL rule and derivative matrix
    std::vector<double> x;                 // [e][3][N3]
    std::vector<double> J;                 // [e][N3]
    std::vector<double> Ja;                // [e][3][3][N3]
    std::vector<double> delta;             // [e]
};

void gll_rule(int P, std::vector<double> &xi, std::vector<double> &w, std::vector<double> &D);
// Interpolate geometry to the GLL nodes and build curl-form metric terms.
// Returns false (with msg) on a non-positive Jacobian.
bool build_geometry(const hdg_mesh_desc &d, int P, HostGeometry &g, std::string &msg);
// Spatially local processing order of the elements (recursive bisection of centroids).
std::vector<int32_t> locality_order(const hdg_mesh_desc &d);

}  // namespace hdg
