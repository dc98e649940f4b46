/*
 * FP64 CPU oracle for the hybrid NS-LES / Euler DGSEM residual.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and hdg_oracle.c are used by the
 * test suite, by the smoke check and by the benchmark's CPU-baseline leg.
 * The product path never includes, links or calls it, and it shares no code
 * with the HIP library.
 *
 * Data conventions (the interface format, shared with the library only as a
 * documented layout):
 *   - state / residual: element after element, [4][N_e^3] each, N_e = P_e + 1,
 *     fields (p, u, v, w), node a + N b + N^2 c;
 *   - geometry: [e][3][(Pg+1)^3] control points at equispaced reference
 *     positions -1 + 2k/Pg;
 *   - connectivity: nbr[e][6] (element, -1 wall, -2 far field), nbr_face[e][6],
 *     orient[e][6] (bit0 swap, bit1 flip first, bit2 flip second face axis);
 *   - flag[e] = 1: Navier-Stokes + LES element, 0: Euler element.
 */
#ifndef HDG_ORACLE_H
#define HDG_ORACLE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double c0sq;       /* artificial sound speed squared */
    double nu;         /* kinematic viscosity on viscous elements */
    int les_model;     /* 0 none, 1 Smagorinsky, 2 Vreman */
    double C_les;      /* Cs (Smagorinsky) or Cv (Vreman) */
    int mixed_face;    /* 0: viscous flux averaged with a zero Euler side; 1: zero on mixed faces */
    double q_inf[4];   /* far-field state */
    int riemann;       /* numerical flux: 0 Roe (Sec. 2.3), 1 Rusanov */
} orc_params;

typedef struct orc_mesh orc_mesh;

/* Gauss-Lobatto-Legendre rule of order P: nodes xi[P+1], weights w[P+1],
 * derivative matrix D[(P+1)*(P+1)], D[i*(P+1)+j] = l_j'(xi_i). */
void orc_lgl(int P, double *xi, double *w, double *D);

/* Returns NULL on invalid input; orc_last_error() says why. */
orc_mesh *orc_mesh_new(int n_elem, int P, int Pg, const double *xyz_geom,
                       const int *nbr, const signed char *nbr_face,
                       const signed char *orient, const unsigned char *flag);
/* Per-element orders P[e]; faces between different orders are coupled through
 * a mortar (see hdg_oracle.c) and need a lower order >= 2 and >= Pg. */
orc_mesh *orc_mesh_new_mixed(int n_elem, const int *P, int Pg, const double *xyz_geom,
                             const int *nbr, const signed char *nbr_face,
                             const signed char *orient, const unsigned char *flag);
size_t orc_mesh_nodes(const orc_mesh *m);
void orc_mesh_free(orc_mesh *m);
const char *orc_last_error(void);
void orc_set_flags(orc_mesh *m, const unsigned char *flag);

void orc_node_coords(const orc_mesh *m, double *xyz);          /* [e][3][N_e^3] */
void orc_metrics(const orc_mesh *m, double *J, double *Ja);    /* [e][N_e^3], [e][3][3][N_e^3] */
double orc_filter_width(const orc_mesh *m, int e);

/* Building blocks exposed for the pins. */
void orc_roe_flux(double c0sq, const double *qL, const double *qR, const double *n, double *F);
void orc_rusanov_flux(double c0sq, const double *qL, const double *qR, const double *n, double *F);
double orc_les_nut(int model, double C, double delta, const double *G); /* G[r*3+d] = du_r/dx_d */

/* BR1 gradient on every viscous element (others left untouched): G[e][3][3][N_e^3]. */
void orc_gradient(const orc_mesh *m, const orc_params *p, const double *q, double *G);
/* Residual R = dq/dt. */
void orc_residual(const orc_mesh *m, const orc_params *p, const double *q, double *R);
/* nsteps of the 3-stage low-storage RK, q updated in place. */
void orc_rk3_steps(const orc_mesh *m, const orc_params *p, double *q, double dt, int nsteps);
/* The same RK driver applied to dy/dt = lambda * y (complex lambda), for the pins. */
void orc_rk3_linear(double lam_re, double lam_im, double dt, int nsteps, double *y_re, double *y_im);
/* The same RK driver applied to dy/dt = -y^2. */
double orc_rk3_riccati(double y0, double dt, int nsteps);

void orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
