/*
 * Reference oracle: the paper's MPM time loop in plain sequential FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written from Sec. 2.2 (basis,
 * lumped mass, P2G / G2P / P2GD / G2PD operators, obstacle projection, CFL),
 * Sec. 3 (steps (i)-(xiv) of the time loop) and Algorithm 1 of the paper.
 * Where the paper is silent or ambiguous the reading taken is stated at the
 * point of use.  No blocking, fusion or reordering: every operator is a
 * separate loop over particles (in id order) or over nodes.
 *
 * Threads (orc_set_threads; default 1, the reference order): the loops over
 * particles and over nodes are independent per iteration and may run on
 * several OpenMP threads.  The only sums across particles are the two P2G
 * scatters; with more than one thread each thread scatters a contiguous
 * block of ids into its own node arrays, and those are added in thread
 * order, so the result differs from one thread by FP64 rounding only.  Used
 * to time the CPU baseline on all host cores and to shorten long runs.
 *
 * FP32 state (orc_set_fp32_state; off by default): the particle state is
 * rounded to FP32 at the call and after every step, the arithmetic staying
 * FP64.  It measures what storing the state in FP32 alone does to a long
 * run, the floor an FP32-state implementation is compared against.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct orc_state {
    orc_problem pb;
    double h;
    int nn[3];             /* nodes per axis */
    int64_t nnodes;
    int64_t np;
    /* particles, id order */
    double *x[3], *v[3], *M, *rho, *E, *G[9], *vbar[3];
    /* nodes */
    uint8_t *obst;         /* 1 = corner of an obstacle cell */
    double *nrm[3];
    double *m, *p[3], *f[3], *pbc[3], *fbc[3], *pu[3], *p2[3];
    /* scratch: per-particle accelerations; nodal velocity fields u/m */
    double *acc[3], *vn[3], *an[3], *v2n[3];
    double t, dt, dt_last;
    int64_t step;
    int64_t wall_escapes;
    int failed;
    int nthreads;          /* OpenMP threads of the loops (1: sequential)   */
    int fp32_state;        /* round the particle state to FP32 after a step  */
    double *priv;          /* nthreads * (1 + 2 dim) node arrays (P2G sums) */
};

/* ---------------------------------------------------------------- basis -- */

/* Knot t_i of the open (clamped) uniform knot vector of quadratic B-splines
 * on n cells, in cell units: 0,0,0,1,2,...,n-1,n,n,n (i = 0..n+4). */
static double knot(int n, int i) {
    int k = i - 2;
    if (k < 0) k = 0;
    if (k > n) k = n;
    return (double)k;
}

/* Cox-de Boor recursion: B_{j,p}(s) for the degree-p B-spline j on the
 * clamped knot vector, with s known to lie in knot span `span`
 * (t_span <= s < t_{span+1}).  Terms with a zero-length knot interval are 0. */
static double cox_de_boor(int n, int j, int p, int span, double s) {
    if (p == 0) return j == span ? 1.0 : 0.0;
    double r = 0.0;
    double d1 = knot(n, j + p) - knot(n, j);
    double d2 = knot(n, j + p + 1) - knot(n, j + 1);
    if (d1 > 0.0) r += (s - knot(n, j)) / d1 * cox_de_boor(n, j, p - 1, span, s);
    if (d2 > 0.0) r += (knot(n, j + p + 1) - s) / d2 * cox_de_boor(n, j + 1, p - 1, span, s);
    return r;
}

/* Derivative of a degree-2 B-spline:
 * 2 [B_{j,1}/(t_{j+2}-t_j) - B_{j+1,1}/(t_{j+3}-t_{j+1})]. */
static double cox_de_boor_deriv2(int n, int j, int span, double s) {
    double r = 0.0;
    double d1 = knot(n, j + 2) - knot(n, j);
    double d2 = knot(n, j + 3) - knot(n, j + 1);
    if (d1 > 0.0) r += 2.0 * cox_de_boor(n, j, 1, span, s) / d1;
    if (d2 > 0.0) r -= 2.0 * cox_de_boor(n, j + 1, 1, span, s) / d2;
    return r;
}

int orc_basis_1d(int shape, int n, double s, int32_t *first, double *w, double *dw) {
    if (shape == ORC_Q1) {
        /* Q1 element of cell c (Sec. 2.2): nodes c and c+1, phi_c = 1 - t,
         * phi_{c+1} = t with t = s - c.  A point on a cell face belongs to
         * the upper cell; the last face belongs to the last cell. */
        int c = (int)floor(s);
        if (c < 0) c = 0;
        if (c > n - 1) c = n - 1;
        double t = s - c;
        *first = c;
        w[0] = 1.0 - t;  dw[0] = -1.0;
        w[1] = t;        dw[1] = 1.0;
        return 2;
    }
    if (shape == ORC_B2) {
        /* B2: quadratic B-splines on the clamped knot vector whose knots are
         * the cell faces, n+2 functions per axis.  On cell c (knot span c+2)
         * the non-zero functions are B_c, B_{c+1}, B_{c+2}.  On a domain face
         * only the first (last) function is non-zero, where it equals 1. */
        if (n < 2) return 0;
        int c = (int)floor(s);
        if (c < 0) c = 0;
        if (c > n - 1) c = n - 1;
        *first = c;
        for (int j = 0; j < 3; ++j) {
            w[j] = cox_de_boor(n, c + j, 2, c + 2, s);
            dw[j] = cox_de_boor_deriv2(n, c + j, c + 2, s);
        }
        return 3;
    }
    return 0;
}

/* All stencil nodes of one point: flat node indices, weights and gradients
 * (gradient in physical units, i.e. divided by h).  Returns the count. */
typedef struct {
    int count;
    int64_t node[27];
    double w[27];
    double dw[27][3];
} stencil;

static void point_stencil(const orc_problem *pb, double h, const int nn[3],
                          const double *pt, stencil *st) {
    int dim = pb->dim;
    int32_t first[3] = {0, 0, 0};
    double w1[3][3], d1[3][3];
    int width = 0;
    for (int a = 0; a < dim; ++a) {
        double s = (pt[a] - pb->lo[a]) / h;
        width = orc_basis_1d(pb->shape, pb->n[a], s, &first[a], w1[a], d1[a]);
    }
    int wz = dim == 3 ? width : 1;
    st->count = 0;
    for (int k = 0; k < wz; ++k)
        for (int j = 0; j < width; ++j)
            for (int i = 0; i < width; ++i) {
                int idx[3] = {i, j, k};
                int64_t flat = 0, stride = 1;
                double w = 1.0;
                for (int a = 0; a < dim; ++a) {
                    flat += (int64_t)(first[a] + idx[a]) * stride;
                    stride *= nn[a];
                    w *= w1[a][idx[a]];
                }
                double grad[3] = {0, 0, 0};
                for (int a = 0; a < dim; ++a) {
                    double gcomp = d1[a][idx[a]] / h;
                    for (int b = 0; b < dim; ++b)
                        if (b != a) gcomp *= w1[b][idx[b]];
                    grad[a] = gcomp;
                }
                int c = st->count++;
                st->node[c] = flat;
                st->w[c] = w;
                for (int a = 0; a < 3; ++a) st->dw[c][a] = grad[a];
            }
}

/* G2P of a nodal vector field at one point: out[a] = sum_i phi_i u_a(i)
 * (eq. g2p_gen). */
static void stencil_interp(const stencil *st, int dim, double *const *u, double *out) {
    for (int a = 0; a < dim; ++a) out[a] = 0.0;
    for (int c = 0; c < st->count; ++c)
        for (int a = 0; a < dim; ++a) out[a] += st->w[c] * u[a][st->node[c]];
}

/* G2PD of a nodal vector field at one point: G[a][b] = sum_i u_a(i) d_b phi_i
 * (eq. g2pd_gen), row-major a*dim+b. */
static void stencil_gradient(const stencil *st, int dim, double *const *u, double *G) {
    for (int c = 0; c < dim * dim; ++c) G[c] = 0.0;
    for (int c = 0; c < st->count; ++c)
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b)
                G[a * dim + b] += u[a][st->node[c]] * st->dw[c][b];
}

/* ------------------------------------------------------ constitutive laws -- */

static double eos_pressure(double gamma, double rho, double e) {
    return (gamma - 1.0) * rho * e;                  /* perfect gas (Sec. 2.1) */
}

/* Sound speed sqrt(gamma p / rho); a negative pressure gives 0. */
static double sound_speed(double gamma, double rho, double p) {
    double c2 = gamma * p / rho;
    return c2 > 0.0 ? sqrt(c2) : 0.0;
}

double orc_artificial_viscosity(int av_form, double c0, double c1, double gamma,
                                double h, double rho, double p, double divv) {
    /* Only active in compression, div v < 0 (Sec. 2.1, eq. muart). */
    if (!(divv < 0.0)) return 0.0;
    double c = sound_speed(gamma, rho, p);
    if (av_form == ORC_AV_BOOK)
        return c0 * rho * (h * divv) * (h * divv) - c1 * rho * h * c * divv;
    double r = rho * h * divv;
    return c0 * r * r - c1 * h * c * divv;
}

void orc_obstacle_project(int dim, const double *n, double *u) {
    /* u' = u - ((u.n - |u.n|)/2) n : removes only the component pointing
     * into the obstacle (n points out of it) (eqs. normali1, normali2). */
    double un = 0.0;
    for (int a = 0; a < dim; ++a) un += u[a] * n[a];
    double k = 0.5 * (un - fabs(un));
    for (int a = 0; a < dim; ++a) u[a] -= k * n[a];
}

uint64_t orc_splitmix64(uint64_t z) {
    /* One output of Steele-Lea-Flood's SplitMix64 whose state is z before the
     * call: add the golden-ratio increment, then the variant-13 finaliser. */
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------- helpers -- */

/* Node index along axis a of a flat node index (x fastest). */
static int node_index(const orc_state *s, int64_t flat, int a) {
    int64_t r = flat;
    for (int b = 0; b < a; ++b) r /= s->nn[b];
    return (int)(r % s->nn[a]);
}

/* Boundary conditions on one nodal vector (Sec. 3 steps (iii) and (vii),
 * the obstacle treatment of Sec. 2.2 and the wind-tunnel conditions of
 * Sec. 4.1).  Order: obstacle projection, wall faces, inflow faces.
 * is_force: inflow sets the force to zero instead of m * u_in. */
static void apply_bc_node(const orc_state *s, int64_t i, double *u, int is_force) {
    const orc_problem *pb = &s->pb;
    int dim = pb->dim;
    if (s->obst[i]) {
        double n[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) n[a] = s->nrm[a][i];
        orc_obstacle_project(dim, n, u);
    }
    /* The boundary nodes of a face are the first / last node along its axis:
     * the only ones whose basis function is non-zero on the face. */
    for (int a = 0; a < dim; ++a) {
        int ia = node_index(s, i, a);
        if ((ia == 0 && pb->face[a][0] == ORC_FACE_WALL) ||
            (ia == s->nn[a] - 1 && pb->face[a][1] == ORC_FACE_WALL))
            u[a] = 0.0;
    }
    for (int a = 0; a < dim; ++a) {
        int ia = node_index(s, i, a);
        if ((ia == 0 && pb->face[a][0] == ORC_FACE_INFLOW) ||
            (ia == s->nn[a] - 1 && pb->face[a][1] == ORC_FACE_INFLOW)) {
            for (int b = 0; b < dim; ++b)
                u[b] = is_force ? 0.0 : s->m[i] * pb->inflow_u[b];
        }
    }
}

/* Per-particle artificial pressure with the lagged divergence tr G. */
static double particle_q(const orc_state *s, int64_t k, double P) {
    const orc_problem *pb = &s->pb;
    double D = 0.0;
    for (int a = 0; a < pb->dim; ++a) D += s->G[a * pb->dim + a][k];
    return orc_artificial_viscosity(pb->av_form, pb->c0, pb->c1, pb->gamma, s->h,
                                    s->rho[k], P, D);
}

static double compute_dt(const orc_state *s, double vmax, double cmax) {
    double dt = s->pb.cfl * s->h / (vmax + cmax);
    if (s->pb.t_end > 0.0) {
        double rest = s->pb.t_end - s->t;
        if (rest < dt) dt = rest;
        if (dt < 0.0) dt = 0.0;
    }
    return dt;
}

/* ------------------------------------------------------------- lifecycle -- */

int orc_grid_shape(const orc_state *s, int32_t nodes[3]) {
    for (int a = 0; a < 3; ++a) nodes[a] = s->nn[a];
    return ORC_OK;
}

void orc_destroy(orc_state *s) {
    if (!s) return;
    for (int a = 0; a < 3; ++a) {
        free(s->x[a]); free(s->v[a]); free(s->vbar[a]); free(s->acc[a]);
        free(s->nrm[a]); free(s->p[a]); free(s->f[a]); free(s->pbc[a]);
        free(s->fbc[a]); free(s->pu[a]); free(s->p2[a]);
        free(s->vn[a]); free(s->an[a]); free(s->v2n[a]);
    }
    for (int c = 0; c < 9; ++c) free(s->G[c]);
    free(s->M); free(s->rho); free(s->E); free(s->obst); free(s->m);
    free(s->priv);
    free(s);
}

static int check_problem(const orc_problem *pb, double *h_out) {
    if (pb->dim != 2 && pb->dim != 3) return ORC_E_ARG;
    if (pb->shape != ORC_Q1 && pb->shape != ORC_B2) return ORC_E_ARG;
    if (pb->av_form != ORC_AV_PAPER && pb->av_form != ORC_AV_BOOK) return ORC_E_ARG;
    if (!(pb->gamma > 1.0) || !(pb->cfl > 0.0)) return ORC_E_ARG;
    double h = 0.0;
    for (int a = 0; a < pb->dim; ++a) {
        if (pb->n[a] < 2 || !(pb->hi[a] > pb->lo[a])) return ORC_E_ARG;
        double ha = (pb->hi[a] - pb->lo[a]) / pb->n[a];
        if (a == 0) h = ha;
        else if (fabs(ha - h) > 1e-9 * h) return ORC_E_ARG;   /* equal cells only */
        for (int side = 0; side < 2; ++side)
            if (pb->face[a][side] < ORC_FACE_WALL || pb->face[a][side] > ORC_FACE_OUTFLOW)
                return ORC_E_ARG;
    }
    *h_out = h;
    return ORC_OK;
}

int orc_create(const orc_problem *pb, int64_t np,
               const double *const *x, const double *const *v,
               const double *mass, const double *rho, const double *eint,
               const double *const *gradv, const uint32_t *id,
               const uint8_t *cell_mask, const double *const *node_normal,
               orc_state **out) {
    double h;
    if (!pb || !out || np < 0 || !x || !v || !mass || !rho || !eint || !id)
        return ORC_E_ARG;
    if (check_problem(pb, &h) != ORC_OK) return ORC_E_ARG;
    if (cell_mask && !node_normal) return ORC_E_ARG;
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    if (!s) return ORC_E_ARG;
    s->pb = *pb;
    s->h = h;
    int dim = pb->dim;
    s->nnodes = 1;
    for (int a = 0; a < 3; ++a) {
        s->nn[a] = a < dim ? pb->n[a] + (pb->shape == ORC_B2 ? 2 : 1) : 1;
        s->nnodes *= s->nn[a];
    }
    s->np = np;
    s->nthreads = 1;
    size_t pbytes = (size_t)(np > 0 ? np : 1) * sizeof(double);
    size_t nbytes = (size_t)s->nnodes * sizeof(double);
    for (int a = 0; a < 3; ++a) {
        s->x[a] = calloc(1, pbytes); s->v[a] = calloc(1, pbytes);
        s->vbar[a] = calloc(1, pbytes); s->acc[a] = calloc(1, pbytes);
        s->nrm[a] = calloc(1, nbytes); s->p[a] = calloc(1, nbytes);
        s->f[a] = calloc(1, nbytes); s->pbc[a] = calloc(1, nbytes);
        s->fbc[a] = calloc(1, nbytes); s->pu[a] = calloc(1, nbytes);
        s->p2[a] = calloc(1, nbytes);
        s->vn[a] = calloc(1, nbytes); s->an[a] = calloc(1, nbytes);
        s->v2n[a] = calloc(1, nbytes);
    }
    for (int c = 0; c < 9; ++c) s->G[c] = calloc(1, pbytes);
    s->M = calloc(1, pbytes); s->rho = calloc(1, pbytes); s->E = calloc(1, pbytes);
    s->obst = calloc(1, (size_t)s->nnodes); s->m = calloc(1, nbytes);
    if (!s->M || !s->rho || !s->E || !s->obst || !s->m) { orc_destroy(s); return ORC_E_ARG; }

    /* Particles are stored in id order. */
    uint8_t *seen = calloc(1, (size_t)(np > 0 ? np : 1));
    for (int64_t k = 0; k < np; ++k) {
        uint32_t q = id[k];
        if ((int64_t)q >= np || seen[q]) { free(seen); orc_destroy(s); return ORC_E_ARG; }
        seen[q] = 1;
        for (int a = 0; a < dim; ++a) {
            s->x[a][q] = x[a][k];
            s->v[a][q] = v[a][k];
            if (!(x[a][k] >= pb->lo[a] && x[a][k] < pb->hi[a])) {
                free(seen); orc_destroy(s); return ORC_E_ARG;
            }
        }
        s->M[q] = mass[k]; s->rho[q] = rho[k]; s->E[q] = eint[k];
        if (!(mass[k] > 0.0) || !(rho[k] > 0.0)) { free(seen); orc_destroy(s); return ORC_E_ARG; }
        for (int c = 0; c < dim * dim; ++c) s->G[c][q] = gradv ? gradv[c][k] : 0.0;
    }
    free(seen);

    /* Obstacle nodes: nodes whose position lies in the closure of a masked
     * cell (reading of the obstacle-cell marking of Sec. 2.2).  Q1 nodes are
     * the cell vertices, so these are the corners of the masked cells; B2
     * nodes sit at the Greville points 0, 1/2, 3/2, ..., n-1/2, n (cell
     * units), so node j lies in cell min(max(j-1, 0), n-1). */
    if (cell_mask) {
        for (int64_t i = 0; i < s->nnodes; ++i) {
            int is_obst = 0;
            if (pb->shape == ORC_B2) {
                int64_t cflat = 0, stride = 1;
                for (int a = 0; a < dim; ++a) {
                    int j = node_index(s, i, a) - 1;
                    if (j < 0) j = 0;
                    if (j > pb->n[a] - 1) j = pb->n[a] - 1;
                    cflat += j * stride;
                    stride *= pb->n[a];
                }
                is_obst = cell_mask[cflat] != 0;
            } else {
                /* any of the up to 2^dim cells sharing this vertex */
                int corners = 1 << dim;
                for (int q = 0; q < corners && !is_obst; ++q) {
                    int64_t cflat = 0, stride = 1;
                    int ok = 1;
                    for (int a = 0; a < dim; ++a) {
                        int j = node_index(s, i, a) - ((q >> a) & 1);
                        if (j < 0 || j > pb->n[a] - 1) { ok = 0; break; }
                        cflat += j * stride;
                        stride *= pb->n[a];
                    }
                    if (ok && cell_mask[cflat]) is_obst = 1;
                }
            }
            if (is_obst) {
                s->obst[i] = 1;
                for (int a = 0; a < dim; ++a) s->nrm[a][i] = node_normal[a][i];
            }
        }
    }

    /* First time step from the initial state (Sec. 2.2, CFL; Sec. 3 (xiii)). */
    double vmax = 0.0, cmax = 0.0;
    for (int64_t k = 0; k < np; ++k) {
        double vv = 0.0;
        for (int a = 0; a < dim; ++a) vv += s->v[a][k] * s->v[a][k];
        vv = sqrt(vv);
        double c = sound_speed(pb->gamma, s->rho[k], eos_pressure(pb->gamma, s->rho[k], s->E[k]));
        if (vv > vmax) vmax = vv;
        if (c > cmax) cmax = c;
    }
    s->t = 0.0;
    s->dt = (vmax + cmax > 0.0) ? compute_dt(s, vmax, cmax) : 0.0;
    s->dt_last = 0.0;
    *out = s;
    return ORC_OK;
}

int orc_set_dt(orc_state *s, double dt) {
    if (!s || !(dt > 0.0)) return ORC_E_ARG;
    s->dt = dt;
    return ORC_OK;
}

int orc_set_threads(orc_state *s, int n) {
    if (!s || n < 1) return ORC_E_ARG;
#ifndef _OPENMP
    if (n > 1) return ORC_E_ARG;
#endif
    free(s->priv);
    s->priv = NULL;
    if (n > 1) {
        s->priv = (double *)malloc((size_t)n * (1 + 2 * s->pb.dim) * s->nnodes * sizeof(double));
        if (!s->priv) { s->nthreads = 1; return ORC_E_ARG; }
    }
    s->nthreads = n;
    return ORC_OK;
}

/* Round every stored particle field (X, V, M, rho, E, G) to FP32. */
static void round_state_fp32(orc_state *s) {
    const int dim = s->pb.dim;
    const int nt = s->nthreads;
    (void)nt;
#pragma omp parallel for num_threads(nt) if (nt > 1)
    for (int64_t k = 0; k < s->np; ++k) {
        for (int a = 0; a < dim; ++a) {
            s->x[a][k] = (double)(float)s->x[a][k];
            s->v[a][k] = (double)(float)s->v[a][k];
        }
        s->M[k] = (double)(float)s->M[k];
        s->rho[k] = (double)(float)s->rho[k];
        s->E[k] = (double)(float)s->E[k];
        for (int i = 0; i < dim * dim; ++i) s->G[i][k] = (double)(float)s->G[i][k];
    }
}

int orc_set_fp32_state(orc_state *s, int on) {
    if (!s) return ORC_E_ARG;
    s->fp32_state = on != 0;
    if (s->fp32_state) round_state_fp32(s);
    return ORC_OK;
}

/* ------------------------------------------------------------- one step -- */

/* Nodal value u/m, zero where the node carries no mass (reading: nodes with
 * m <= 0 do not contribute to G2P and G2PD). */
static double ratio(double u, double m) { return m > 0.0 ? u / m : 0.0; }

/* The P2G sums of particles k0 .. k1-1, in id order, added into out:
 * which = 0: mass, momentum and internal force (step (ii)), out = m, p[3],
 * f[3]; which = 1: the updated momentum M V' (step (vi)), out = p2[3];
 * which = 2: mass and volume M / rho at the current positions (the
 * grid-projected density read-out, not a step), out = m, vol. */
static void scatter_range(const orc_state *s, int which, int64_t k0, int64_t k1, double *const *out) {
    const orc_problem *pb = &s->pb;
    const int dim = pb->dim;
    const double gam = pb->gamma;
    stencil st;
    for (int64_t k = k0; k < k1; ++k) {
        double pt[3] = {s->x[0][k], s->x[1][k], dim == 3 ? s->x[2][k] : 0.0};
        point_stencil(pb, s->h, s->nn, pt, &st);
        if (which == 1) {
            for (int c = 0; c < st.count; ++c)
                for (int a = 0; a < dim; ++a)
                    out[a][st.node[c]] += s->M[k] * s->v[a][k] * st.w[c];
            continue;
        }
        if (which == 2) {
            for (int c = 0; c < st.count; ++c) {
                out[0][st.node[c]] += s->M[k] * st.w[c];
                out[1][st.node[c]] += s->M[k] / s->rho[k] * st.w[c];
            }
            continue;
        }
        double P = eos_pressure(gam, s->rho[k], s->E[k]);
        double Q = particle_q(s, k, P);
        double vol = s->M[k] / s->rho[k];
        for (int c = 0; c < st.count; ++c) {
            int64_t i = st.node[c];
            out[0][i] += s->M[k] * st.w[c];
            for (int a = 0; a < dim; ++a) {
                out[1 + a][i] += s->M[k] * s->v[a][k] * st.w[c];
                out[1 + dim + a][i] += (P + Q) * vol * st.dw[c][a];
            }
        }
    }
}

/* One P2G over all particles into out (the arrays of scatter_range,
 * zeroed by the caller): with one thread in id order; with several,
 * per-thread node arrays over contiguous id blocks, then added in thread
 * order. */
static void scatter(orc_state *s, int which, double *const *out) {
    const int dim = s->pb.dim;
    const int nq = which == 0 ? 1 + 2 * dim : (which == 1 ? dim : 2);
    const int64_t NN = s->nnodes;
    if (s->nthreads <= 1) {
        scatter_range(s, which, 0, s->np, out);
        return;
    }
#pragma omp parallel num_threads(s->nthreads)
    {
#ifdef _OPENMP
        const int t = omp_get_thread_num(), nt = omp_get_num_threads();
#else
        const int t = 0, nt = 1;
#endif
        double *mine[7];
        for (int q = 0; q < nq; ++q) {
            mine[q] = s->priv + ((size_t)t * nq + q) * NN;
            memset(mine[q], 0, (size_t)NN * sizeof(double));
        }
        scatter_range(s, which, s->np * t / nt, s->np * (t + 1) / nt, mine);
#pragma omp barrier
#pragma omp for
        for (int64_t i = 0; i < NN; ++i)
            for (int q = 0; q < nq; ++q) {
                double sum = 0.0;
                for (int u = 0; u < nt; ++u) sum += s->priv[((size_t)u * nq + q) * NN + i];
                out[q][i] = sum;
            }
    }
}

static int one_step(orc_state *s) {
    const orc_problem *pb = &s->pb;
    const int dim = pb->dim;
    const double dt = s->dt;
    const double gam = pb->gamma;
    const int64_t NN = s->nnodes;
    const int nt = s->nthreads;

    /* (i) Grid reset: all accumulators start from zero. */
    memset(s->m, 0, (size_t)NN * sizeof(double));
    for (int a = 0; a < 3; ++a) {
        memset(s->p[a], 0, (size_t)NN * sizeof(double));
        memset(s->f[a], 0, (size_t)NN * sizeof(double));
        memset(s->p2[a], 0, (size_t)NN * sizeof(double));
    }

    /* (ii) P2G of mass and momentum, P2GD of the internal force
     * f_i = sum_k (P_k + Q_k) (M_k / rho_k) grad phi_i (eq. mxa=f). */
    {
        double *out[7] = {s->m};
        for (int a = 0; a < dim; ++a) { out[1 + a] = s->p[a]; out[1 + dim + a] = s->f[a]; }
        scatter(s, 0, out);
    }

    /* (iii) Boundary conditions on momentum and force. */
#pragma omp parallel for num_threads(nt) if (nt > 1)
    for (int64_t i = 0; i < NN; ++i) {
        double u[3] = {0, 0, 0}, fv[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) { u[a] = s->p[a][i]; fv[a] = s->f[a][i]; }
        apply_bc_node(s, i, u, 0);
        apply_bc_node(s, i, fv, 1);
        for (int a = 0; a < dim; ++a) { s->pbc[a][i] = u[a]; s->fbc[a][i] = fv[a]; }
    }

    /* (iv) Momentum update on the grid: (mv)' = mv + dt f. */
    for (int a = 0; a < dim; ++a)
        for (int64_t i = 0; i < NN; ++i) s->pu[a][i] = s->pbc[a][i] + dt * s->fbc[a][i];

    /* (v) G2P of (mv)'/m into Vbar and of f/m into A (callables theta of
     * Sec. 3); then V' = V + dt A. */
    for (int a = 0; a < dim; ++a)
        for (int64_t i = 0; i < NN; ++i) {
            s->vn[a][i] = ratio(s->pu[a][i], s->m[i]);
            s->an[a][i] = ratio(s->fbc[a][i], s->m[i]);
        }
#pragma omp parallel for num_threads(nt) if (nt > 1)
    for (int64_t k = 0; k < s->np; ++k) {
        stencil st;
        double pt[3] = {s->x[0][k], s->x[1][k], dim == 3 ? s->x[2][k] : 0.0};
        point_stencil(pb, s->h, s->nn, pt, &st);
        double vb[3] = {0, 0, 0}, A[3] = {0, 0, 0};
        stencil_interp(&st, dim, s->vn, vb);
        stencil_interp(&st, dim, s->an, A);
        for (int a = 0; a < dim; ++a) {
            s->vbar[a][k] = vb[a];
            s->acc[a][k] = A[a];
        }
    }
    for (int64_t k = 0; k < s->np; ++k)
        for (int a = 0; a < dim; ++a) s->v[a][k] += dt * s->acc[a][k];

    /* (vi) P2G of the updated momentum M V'. */
    scatter(s, 1, s->p2);

    /* (vii) Boundary conditions on the re-mapped momentum. */
#pragma omp parallel for num_threads(nt) if (nt > 1)
    for (int64_t i = 0; i < NN; ++i) {
        double u[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) u[a] = s->p2[a][i];
        apply_bc_node(s, i, u, 0);
        for (int a = 0; a < dim; ++a) s->p2[a][i] = u[a];
    }

    /* (viii) G2PD of (mv)/m: velocity gradient; energy, density update.
     * P and Q are those of the state at the start of the step, the same
     * values used in the force of (ii). */
    for (int a = 0; a < dim; ++a)
        for (int64_t i = 0; i < NN; ++i) s->v2n[a][i] = ratio(s->p2[a][i], s->m[i]);
    int bad = 0;
#pragma omp parallel for num_threads(nt) if (nt > 1) reduction(| : bad)
    for (int64_t k = 0; k < s->np; ++k) {
        stencil st;
        double pt[3] = {s->x[0][k], s->x[1][k], dim == 3 ? s->x[2][k] : 0.0};
        point_stencil(pb, s->h, s->nn, pt, &st);
        double G[9] = {0};
        stencil_gradient(&st, dim, s->v2n, G);
        double D = 0.0;
        for (int a = 0; a < dim; ++a) D += G[a * dim + a];
        double P = eos_pressure(gam, s->rho[k], s->E[k]);
        double Q = particle_q(s, k, P);
        double J = 1.0 + dt * D;
        if (!(J > 0.0)) bad = 1;
        s->E[k] = s->E[k] - dt * (P + Q) * D / s->rho[k];
        s->rho[k] = s->rho[k] / J;
        for (int c = 0; c < dim * dim; ++c) s->G[c][k] = G[c];
    }

    /* (ix) Postponed move with the G2P velocity: X' = X + dt Vbar.
     * Outflow (Sec. 4.1: a particle leaving through an outflow face is
     * regenerated in a random cell at the inflow boundary, with the inflow
     * state): the particle re-enters at the x_lo inflow face, as far past
     * it as it went past the face it left (through x_hi: shifted back by the
     * domain length), its transverse coordinates drawn from a counter hash
     * of (seed, step, id). */
    int64_t escapes = 0;
#pragma omp parallel for num_threads(nt) if (nt > 1) reduction(+ : escapes)
    for (int64_t k = 0; k < s->np; ++k) {
        for (int a = 0; a < dim; ++a) s->x[a][k] += dt * s->vbar[a][k];
        int recycled = 0;
        /* the outflow face it crossed, if any (x_hi first, then lo/hi of y, z) */
        int out_axis = -1;
        double past = 0.0;
        if (pb->face[0][1] == ORC_FACE_OUTFLOW && s->x[0][k] >= pb->hi[0]) out_axis = 0;
        for (int a = 1; a < dim && out_axis < 0; ++a) {
            if (pb->face[a][0] == ORC_FACE_OUTFLOW && s->x[a][k] < pb->lo[a]) {
                out_axis = a; past = pb->lo[a] - s->x[a][k];
            } else if (pb->face[a][1] == ORC_FACE_OUTFLOW && s->x[a][k] >= pb->hi[a]) {
                out_axis = a; past = s->x[a][k] - pb->hi[a];
            }
        }
        if (out_axis >= 0) {
            if (out_axis == 0) s->x[0][k] -= (pb->hi[0] - pb->lo[0]);
            else s->x[0][k] = pb->lo[0] + past;
            for (int a = 1; a < dim; ++a) {
                uint64_t word = pb->seed ^ ((uint64_t)s->step << 32) ^ (uint64_t)k ^
                                ((uint64_t)(a - 1) << 56);
                double u = (double)(orc_splitmix64(word) >> 11) * 0x1.0p-53;
                s->x[a][k] = pb->lo[a] + (pb->hi[a] - pb->lo[a]) * u;
            }
            for (int a = 0; a < dim; ++a) s->v[a][k] = pb->inflow_u[a];
            s->rho[k] = pb->inflow_rho;
            s->E[k] = pb->inflow_p / ((gam - 1.0) * pb->inflow_rho);
            s->M[k] = pb->recycle_mass;
            for (int c = 0; c < dim * dim; ++c) s->G[c][k] = 0.0;
            recycled = 1;
        }
        if (!recycled) {
            /* Any other exit is prevented by the CFL bound; clamp the
             * particle back inside and count the event once. */
            int escaped = 0;
            for (int a = 0; a < dim; ++a) {
                double L = pb->hi[a] - pb->lo[a];
                if (s->x[a][k] < pb->lo[a]) { s->x[a][k] = pb->lo[a]; escaped = 1; }
                else if (s->x[a][k] >= pb->hi[a]) { s->x[a][k] = pb->hi[a] - 1e-9 * L; escaped = 1; }
            }
            escapes += escaped;
        }
    }
    s->wall_escapes += escapes;

    /* (xiii)-(xiv) CFL from |V'|, |Vbar| and the updated sound speed; advance t. */
    double vmax = 0.0, cmax = 0.0;
#pragma omp parallel for num_threads(nt) if (nt > 1) reduction(max : vmax, cmax) reduction(| : bad)
    for (int64_t k = 0; k < s->np; ++k) {
        double a1 = 0.0, a2 = 0.0;
        for (int a = 0; a < dim; ++a) {
            a1 += s->v[a][k] * s->v[a][k];
            a2 += s->vbar[a][k] * s->vbar[a][k];
        }
        a1 = sqrt(a1); a2 = sqrt(a2);
        if (a1 > vmax) vmax = a1;
        if (a2 > vmax) vmax = a2;
        double c = sound_speed(gam, s->rho[k], eos_pressure(gam, s->rho[k], s->E[k]));
        if (c > cmax) cmax = c;
        if (!isfinite(s->E[k]) || !isfinite(s->rho[k])) bad = 1;
    }
    s->t += dt;
    s->dt_last = dt;
    s->step += 1;
    s->dt = (vmax + cmax > 0.0) ? compute_dt(s, vmax, cmax) : 0.0;
    if (bad) { s->failed = 1; return ORC_E_NONPHYSICAL; }
    return ORC_OK;
}

int orc_step(orc_state *s, int64_t n_steps) {
    if (!s) return ORC_E_ARG;
    if (s->failed) return ORC_E_STATE;
    if (n_steps <= 0) {
        if (!(s->pb.t_end > 0.0)) return ORC_E_ARG;
        while (s->t < s->pb.t_end && s->dt > 0.0) {
            int rc = one_step(s);
            if (rc) return rc;
            if (s->fp32_state) round_state_fp32(s);
        }
        return ORC_OK;
    }
    for (int64_t n = 0; n < n_steps; ++n) {
        if (s->pb.t_end > 0.0 && !(s->t < s->pb.t_end)) break;
        if (!(s->dt > 0.0)) break;
        int rc = one_step(s);
        if (rc) return rc;
        if (s->fp32_state) round_state_fp32(s);
    }
    return ORC_OK;
}

/* --------------------------------------------------------------- output -- */

int orc_get_particles(const orc_state *s, int field, double *out) {
    if (!s || !out) return ORC_E_ARG;
    const int dim = s->pb.dim;
    const int64_t np = s->np;
    const double gam = s->pb.gamma;
    switch (field) {
    case ORC_F_X: for (int a = 0; a < dim; ++a) memcpy(out + a * np, s->x[a], np * sizeof(double)); break;
    case ORC_F_V: for (int a = 0; a < dim; ++a) memcpy(out + a * np, s->v[a], np * sizeof(double)); break;
    case ORC_F_VBAR: for (int a = 0; a < dim; ++a) memcpy(out + a * np, s->vbar[a], np * sizeof(double)); break;
    case ORC_F_M: memcpy(out, s->M, np * sizeof(double)); break;
    case ORC_F_RHO: memcpy(out, s->rho, np * sizeof(double)); break;
    case ORC_F_E: memcpy(out, s->E, np * sizeof(double)); break;
    case ORC_F_P: for (int64_t k = 0; k < np; ++k) out[k] = eos_pressure(gam, s->rho[k], s->E[k]); break;
    case ORC_F_Q:
        for (int64_t k = 0; k < np; ++k) out[k] = particle_q(s, k, eos_pressure(gam, s->rho[k], s->E[k]));
        break;
    case ORC_F_G: for (int c = 0; c < dim * dim; ++c) memcpy(out + c * np, s->G[c], np * sizeof(double)); break;
    case ORC_F_VOL: for (int64_t k = 0; k < np; ++k) out[k] = s->M[k] / s->rho[k]; break;
    default: return ORC_E_ARG;
    }
    return ORC_OK;
}

int orc_get_grid(const orc_state *s, int which, double *out) {
    if (!s || !out) return ORC_E_ARG;
    const int dim = s->pb.dim;
    const int64_t NN = s->nnodes;
    double *const *src = NULL;
    switch (which) {
    case ORC_G_M: memcpy(out, s->m, NN * sizeof(double)); return ORC_OK;
    case ORC_G_P: src = s->p; break;
    case ORC_G_F: src = s->f; break;
    case ORC_G_PUPD: src = s->pu; break;
    case ORC_G_P2: src = s->p2; break;
    case ORC_G_FBC: src = s->fbc; break;
    default: return ORC_E_ARG;
    }
    for (int a = 0; a < dim; ++a) memcpy(out + a * NN, src[a], NN * sizeof(double));
    return ORC_OK;
}

int orc_projected(orc_state *s, double *mass, double *vol) {
    /* P2G of the particle masses and volumes M / rho at the current
     * positions: the grid-projected density is mass / vol where vol > 0
     * (an Eulerian read-out of the particle density; eq. p2g_gen with the
     * mass and the volume as particle fields). */
    if (!s || !mass || !vol) return ORC_E_ARG;
    memset(mass, 0, (size_t)s->nnodes * sizeof(double));
    memset(vol, 0, (size_t)s->nnodes * sizeof(double));
    double *out[2] = {mass, vol};
    scatter(s, 2, out);
    return ORC_OK;
}

int orc_status(const orc_state *s, double *t, double *dt_next, double *dt_last,
               int64_t *step, double conserved[6], int64_t *wall_escapes) {
    if (!s) return ORC_E_ARG;
    const int dim = s->pb.dim;
    if (t) *t = s->t;
    if (dt_next) *dt_next = s->dt;
    if (dt_last) *dt_last = s->dt_last;
    if (step) *step = s->step;
    if (wall_escapes) *wall_escapes = s->wall_escapes;
    if (conserved) {
        for (int c = 0; c < 6; ++c) conserved[c] = 0.0;
        for (int64_t k = 0; k < s->np; ++k) {
            double v2 = 0.0;
            conserved[0] += s->M[k];
            for (int a = 0; a < dim; ++a) {
                conserved[1 + a] += s->M[k] * s->v[a][k];
                v2 += s->v[a][k] * s->v[a][k];
            }
            conserved[4] += s->M[k] * s->E[k];
            conserved[5] += 0.5 * s->M[k] * v2;
        }
    }
    return s->failed ? ORC_E_NONPHYSICAL : ORC_OK;
}

int orc_nodal_gradient(const orc_problem *pb, const double *const *u,
                       const double *point, double *G) {
    double h;
    if (!pb || !u || !point || !G) return ORC_E_ARG;
    if (check_problem(pb, &h) != ORC_OK) return ORC_E_ARG;
    int nn[3];
    for (int a = 0; a < 3; ++a) nn[a] = a < pb->dim ? pb->n[a] + (pb->shape == ORC_B2 ? 2 : 1) : 1;
    stencil st;
    point_stencil(pb, h, nn, point, &st);
    stencil_gradient(&st, pb->dim, (double *const *)u, G);
    return ORC_OK;
}
