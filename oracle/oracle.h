/*
 * Reference oracle for the compressible-gas Material Point Method of
 * Baioni, Benacchio, Capone, de Falco, "Portable, massively parallel
 * implementation of a Material Point Method for compressible flows"
 * (arXiv 2404.17057).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, sequential FP64
 * transcription of the paper's time loop (Sec. 3, steps (i)-(xiv), and
 * Algorithm 1 "Time loop sketch").  It exists to check the GPU library
 * against.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no
 * source, header or helper with the GPU library.
 *
 * Every quantity is double precision.  Particles are processed in ascending
 * id order, one at a time; the grid is a dense node array.
 */
#ifndef MPM_ORACLE_H
#define MPM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define ORC_OK             0
#define ORC_E_ARG         -1
#define ORC_E_NONPHYSICAL -4   /* J = 1 + dt*div(v) <= 0, or a non-finite value */
#define ORC_E_STATE       -7   /* stepping a handle that already failed */

/* Basis functions: Q1 = bilinear / trilinear finite elements (Sec. 2.2);
 * B2 = quadratic B-splines (the higher-order basis the conclusions name). */
#define ORC_Q1 1
#define ORC_B2 2

/* Domain faces (Sec. 4.1, cylinder boundary conditions). */
#define ORC_FACE_WALL    0   /* slip: normal momentum and force set to zero   */
#define ORC_FACE_INFLOW  1   /* prescribed inflow velocity                     */
#define ORC_FACE_OUTFLOW 2   /* free; particles crossing it are recycled       */

/* Artificial viscosity (Sec. 2.1, eq. muart). */
#define ORC_AV_PAPER 0   /* q = c0 (rho h D)^2 - c1 h sqrt(gamma p/rho) D, as printed */
#define ORC_AV_BOOK  1   /* q = c0 rho (h D)^2 - c1 rho h c D, dimensionally consistent */

typedef struct {
    int32_t dim;               /* 2 or 3 */
    int32_t n[3];              /* cells per axis (n[2] ignored in 2D) */
    double lo[3], hi[3];       /* domain box; the cell size must be equal on all axes */
    int32_t shape;             /* ORC_Q1 or ORC_B2 */
    int32_t av_form;           /* ORC_AV_PAPER or ORC_AV_BOOK */
    double gamma, c0, c1, cfl;
    int32_t face[3][2];        /* per axis, low and high face type */
    double inflow_rho, inflow_p, inflow_u[3];
    double recycle_mass;       /* mass given to a particle recycled at the inflow */
    uint64_t seed;             /* key of the recycling hash */
    double t_end;              /* > 0: runs stop exactly at t_end */
} orc_problem;

typedef struct orc_state orc_state;

/* Create a state.  Particle arrays are copied.  x, v: dim arrays of np;
 * gradv: dim*dim arrays of np (row-major a*dim+b = d v_a / d x_b), may be
 * NULL for zero.  id must be a permutation of 0..np-1.  cell_mask (may be
 * NULL) has one byte per cell, x fastest; node_normal (may be NULL if
 * cell_mask is NULL) has dim arrays over the node grid, x fastest. */
int orc_create(const orc_problem *pb, int64_t np,
               const double *const *x, const double *const *v,
               const double *mass, const double *rho, const double *eint,
               const double *const *gradv, const uint32_t *id,
               const uint8_t *cell_mask, const double *const *node_normal,
               orc_state **out);
void orc_destroy(orc_state *s);

/* Advance n_steps steps; n_steps <= 0 runs until t_end. */
int orc_step(orc_state *s, int64_t n_steps);

/* Set the next time step explicitly (used to drive both implementations
 * with the same dt).  Returns ORC_E_ARG if dt <= 0. */
int orc_set_dt(orc_state *s, double dt);

/* Run the loops on n OpenMP threads (default 1).  With n > 1 the two P2G
 * scatters add per-thread partial node sums in thread order, so results
 * differ from one thread by FP64 rounding only.  ORC_E_ARG if n < 1, or
 * n > 1 in a build without OpenMP. */
int orc_set_threads(orc_state *s, int n);

/* FP32 state: on != 0 rounds the particle fields (X, V, M, rho, E, G) to
 * FP32 now and after every step; the arithmetic stays FP64.  Test support:
 * the effect of FP32 storage alone on a long run. */
int orc_set_fp32_state(orc_state *s, int on);

/* Read-out of the grid-projected density: mass[i] = sum_k M_k phi_i(X_k)
 * and vol[i] = sum_k (M_k / rho_k) phi_i(X_k) at the current positions (two
 * arrays over the node grid, x fastest); the projected density is
 * mass / vol where vol > 0. */
int orc_projected(orc_state *s, double *mass, double *vol);

/* Particle fields in id order, one double array of np per component. */
#define ORC_F_X    0   /* dim components */
#define ORC_F_V    1   /* dim */
#define ORC_F_M    2
#define ORC_F_RHO  3
#define ORC_F_E    4
#define ORC_F_P    5   /* pressure (derived) */
#define ORC_F_Q    6   /* artificial pressure used in the next step (derived) */
#define ORC_F_G    7   /* dim*dim */
#define ORC_F_VOL  8   /* M / rho */
#define ORC_F_VBAR 9   /* dim: the G2P velocity of the last step */
int orc_get_particles(const orc_state *s, int field, double *out);

/* Grid snapshot of the last step, node grid x fastest, component-major.
 * Nodes per axis: n+1 for Q1 (cell vertices), n+2 for B2 (one per
 * B-spline of the clamped knot vector). */
#define ORC_G_M     0  /* nodal mass */
#define ORC_G_P     1  /* dim: momentum as mapped (before boundary conditions) */
#define ORC_G_F     2  /* dim: internal force as mapped (before boundary conditions) */
#define ORC_G_PUPD  3  /* dim: momentum after boundary conditions and the update */
#define ORC_G_P2    4  /* dim: re-mapped momentum after boundary conditions */
#define ORC_G_FBC   5  /* dim: force after boundary conditions */
int orc_get_grid(const orc_state *s, int which, double *out);
int orc_grid_shape(const orc_state *s, int32_t nodes[3]);

/* t, dt of the next step, dt of the last step, steps done, and six FP64
 * sums: total mass, momentum (3), internal energy sum M e, kinetic energy
 * sum M |v|^2 / 2.  wall_escapes counts particles clamped back inside. */
int orc_status(const orc_state *s, double *t, double *dt_next, double *dt_last,
               int64_t *step, double conserved[6], int64_t *wall_escapes);

/* Building blocks, exported so that tests can pin them in isolation. */

/* One-dimensional basis at reduced coordinate s = (x - lo)/h: writes the
 * first node index (in physical node numbering, Q1 clamped to the last cell
 * n-1), and the width (2 or 3) values and derivatives (per unit s). */
int orc_basis_1d(int shape, int n, double s, int32_t *first, double *w, double *dw);

/* Artificial viscosity q(rho, p, D) for cell size h (Sec. 2.1, eq. muart). */
double orc_artificial_viscosity(int av_form, double c0, double c1, double gamma,
                                double h, double rho, double p, double divv);

/* One obstacle projection of a nodal vector (eqs. normali1, normali2). */
void orc_obstacle_project(int dim, const double *n, double *u);

/* Velocity gradient G[a][b] = sum_i u_i[a] d_b phi_i at a point, for a
 * nodal field given as dim arrays over the node grid of problem pb. */
int orc_nodal_gradient(const orc_problem *pb, const double *const *u,
                       const double *point, double *G);

/* The recycling hash: splitmix64 finaliser applied to the given word. */
uint64_t orc_splitmix64(uint64_t z);

#ifdef __cplusplus
}
#endif
#endif
