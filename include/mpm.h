/*
 * mpm.h -- C ABI of the MI355X (gfx950) implementation of the per-step hot
 * path of the compressible-gas Material Point Method of Baioni, Benacchio,
 * Capone, de Falco, "Portable, massively parallel implementation of a
 * Material Point Method for compressible flows" (arXiv 2404.17057).
 *
 * One time step (Sec. 3, step 3, sub-steps (i)-(xiv); Algorithm 1 "Time loop
 * sketch"):
 *   P2G of mass and momentum, P2GD of the internal force ((ii); eqs.
 *     p2g_gen, p2gd_gen, mxa=f)
 *   obstacle, wall and inflow conditions on momentum and force ((iii); eqs.
 *     normali1, normali2; wind-tunnel conditions of Sec. 4.1)
 *   grid momentum update ((iv))
 *   G2P of velocity and acceleration, FLIP velocity update ((v); eq. g2p_gen)
 *   P2G of the updated momentum and its boundary conditions ((vi)-(vii))
 *   G2PD velocity gradient, energy, density and pressure update ((viii);
 *     eq. g2pd_gen; ideal-gas state equation and artificial viscosity, eq. muart)
 *   postponed move with the G2P velocity ((ix)), outflow recycling (Sec. 4.1)
 *   particle-to-cell map ((x)) and re-ordering ((xii), optional in the
 *     paper, here a cell sort every step)
 *   CFL time step from particle velocities and sound speed ((xiii)-(xiv);
 *     Sec. 2.2, eq. CFL)
 * Sub-step (i), the grid reset, is the zero start of every P2G sum; (xi),
 * intermediate output, is mpm_read_fields between runs.
 *
 * Conventions
 *   - Every call returns an int status (MPM_OK or a negative MPM_E_* code);
 *     no exception crosses the ABI; out-parameters are untouched on error.
 *   - Device memory: the caller owns one device workspace of at least
 *     mpm_footprint() bytes per problem and keeps it alive until
 *     mpm_destroy().  The library allocates no device memory on the stepping
 *     path beyond what the HIP runtime takes to instantiate the captured
 *     step graphs; mpm_read_grid allocates a temporary buffer
 *     (mpm_read_grid_noalloc does not).
 *   - Streams: `hip_stream` is a hipStream_t passed as void* (NULL = the
 *     default stream).  All work is enqueued on it; mpm_step and
 *     mpm_step_batch return without waiting.
 *   - The handle is owned by the library and is not thread-safe.
 *   - Errors detected on the device (J = 1 + dt div v <= 0, non-finite
 *     state, fixed-point overflow) are sticky: the problem stops advancing
 *     and the next mpm_status / mpm_read_fields returns the code; after that
 *     mpm_step returns MPM_E_STATE.
 *   - A particle that a step would move out through a wall (which the CFL
 *     bound excludes) is put back inside, on the wall or just below the
 *     high face, and counted in mpm_counters()[1]; it is not an error.
 */
#ifndef MPM_H
#define MPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    MPM_OK = 0,
    MPM_E_ARG = -1,          /* invalid argument or descriptor                 */
    MPM_E_WORKSPACE = -2,    /* workspace missing, misaligned or too small     */
    MPM_E_HIP = -3,          /* a HIP runtime call failed                      */
    MPM_E_NONPHYSICAL = -4,  /* J <= 0 or a non-finite value on the device     */
    MPM_E_OVERFLOW = -5,     /* fixed-point accumulator out of range           */
    MPM_E_UNSUPPORTED = -6,  /* valid request this build does not implement    */
    MPM_E_STATE = -7,        /* operation not allowed in the handle's state    */
    MPM_E_SCRATCH = -8       /* request larger than the fixed scratch buffer   */
};

/* Basis functions (Sec. 2.2: Q1 bilinear/trilinear elements; quadratic
 * B-splines on the clamped knot vector of the cell faces, the higher-order
 * basis named in Sec. 5). */
enum { MPM_Q1 = 1, MPM_B2 = 2 };

/* Arithmetic of the particle state and of the P2G accumulation. */
enum {
    MPM_FP64 = 0,          /* FP64 state, FP64 atomic accumulation              */
    MPM_FP32_ACC_F64 = 1,  /* FP32 state, FP64 atomic accumulation              */
    MPM_FP32_ACC_F32 = 2,  /* FP32 state, FP32 atomic accumulation              */
    MPM_FP32_FIX64 = 3,    /* FP32 state, 64-bit fixed-point integer accumulation:
                              sums are order-independent and bit-reproducible   */
    MPM_FP64_COLOR = 4     /* FP64 state; each P2G by grid colouring (Sec. 5:
                              cells coloured so that cells of one colour have
                              disjoint stencils, 3^dim colours for B2), one
                              pass per colour with plain adds and no atomics,
                              every cell's particles summed in id order:
                              bit-reproducible without fixed point.  B2 only
                              (Q1: MPM_E_UNSUPPORTED)                          */
};

/* Domain face types (Sec. 4.1, eq. bc).  WALL: the normal momentum and force
 * of the face's nodes are set to 0.  INFLOW: momentum m u_in, force 0.
 * OUTFLOW: no condition; a particle leaving through it is regenerated at the
 * inflow boundary with the inflow state (Sec. 4.1): through x_hi it is
 * shifted back by the domain length, through a y or z face it re-enters at
 * x_lo as far past it as it went past the face it left; its transverse
 * coordinates come from a hash of (seed, step, id).  An OUTFLOW face needs
 * x_lo to be INFLOW and cannot be x_lo (else MPM_E_UNSUPPORTED). */
enum { MPM_FACE_WALL = 0, MPM_FACE_INFLOW = 1, MPM_FACE_OUTFLOW = 2 };

/* Artificial viscosity (Sec. 2.1, eq. muart): as printed,
 * q = c0 (rho h D)^2 - c1 h sqrt(gamma p / rho) D, or the textbook form
 * q = c0 rho (h D)^2 - c1 rho h c D; both only where D = div v < 0. */
enum { MPM_AV_PAPER = 0, MPM_AV_BOOK = 1 };

typedef struct {
    int32_t dim;            /* 2 or 3                                              */
    int32_t n[3];           /* cells per axis (>= 2; n[2] ignored in 2D); at most
                               2^31 cells once each axis is padded to whole tiles
                               (16x16 in 2D, 8x8x4 in 3D) and 2^31 - 1 nodes, else
                               MPM_E_UNSUPPORTED                                  */
    double lo[3], hi[3];    /* domain box; cells must be square/cubic (equal h)     */
    int32_t shape;          /* MPM_Q1 or MPM_B2                                     */
    int32_t precision;      /* MPM_FP64 ... MPM_FP32_FIX64                          */
    int32_t av_form;        /* MPM_AV_PAPER or MPM_AV_BOOK                          */
    double gamma, c0, c1;   /* ideal gas ratio; artificial viscosity constants      */
    double cfl;             /* dt = cfl * h / (max|v| + max c)                      */
    int32_t face[3][2];     /* per axis: [low face, high face] type                 */
    double inflow_rho, inflow_p, inflow_u[3]; /* state imposed at INFLOW faces and
                                                 given to recycled particles; with
                                                 an INFLOW or OUTFLOW face rho > 0,
                                                 p >= 0, all finite, else MPM_E_ARG */
    double recycle_mass;    /* mass of a recycled particle (> 0 with an OUTFLOW
                               face, else MPM_E_ARG)                              */
    int64_t n_particles;    /* at most 2^30 - 4 (FP32 state) or 2^29 - 2 (FP64):
                               each particle array stays below 4 GiB, else
                               MPM_E_UNSUPPORTED                                  */
    uint64_t seed;          /* key of the recycling hash                            */
    double t_end;           /* > 0: the last step is shortened to land on t_end     */
    double rho_ref, u_ref;  /* fixed-point references; 0 = derived from the initial
                               state (max density; 4 max(|v| + c))                  */
    double t0;              /* restart: time of the given state (>= 0; 0 = fresh) */
    int64_t step0;          /* restart: steps already taken (>= 0); keys the
                               recycling hash, so a resumed run recycles as the
                               uninterrupted one                                  */
    double dt0;             /* restart: the next time step (mpm_status dt_next);
                               <= 0 derives it from the given state. With the
                               particle fields read back after a run (G and id
                               included), the same rho_ref / u_ref and these
                               three values, MPM_FP32_FIX64 resumes bit for bit;
                               invalid values give MPM_E_ARG                      */
} mpm_desc;

/* Host particle arrays, all of length n_particles, read only during
 * mpm_init.  x, v: dim arrays; gradv: dim*dim arrays, row-major
 * gradv[a*dim+b] = d v_a / d x_b, or all NULL for zero; id: a permutation of
 * 0..n_particles-1 (results are returned in id order). */
typedef struct {
    const double *x[3];
    const double *v[3];
    const double *mass;
    const double *rho;
    const double *eint;     /* specific internal energy                             */
    const double *gradv[9];
    const uint32_t *id;
} mpm_particles_host;

/* Obstacle (Sec. 2.2, eqs. normali1/normali2, sdf), host arrays read only
 * during mpm_init; pass NULL for none.  cell_mask: one byte per cell, x
 * fastest (non-zero = obstacle cell).  node_normal: dim arrays over the
 * node grid (mpm_grid_shape), x fastest, unit normals pointing out of the
 * obstacle.  Obstacle nodes are the nodes whose position lies in a masked
 * cell (Q1: cell vertices; B2: Greville points 0, 1/2, 3/2, ..., n-1/2, n). */
typedef struct {
    const uint8_t *cell_mask;
    const double *node_normal[3];
} mpm_obstacle_host;

typedef struct mpm_handle mpm_handle;

/* Device bytes one problem needs in its workspace (particle state of two
 * step parities, grid accumulators, sort tables; Sec. 3 step 2 keeps all of
 * it on the device for the whole run).  Errors: MPM_E_ARG. */
int mpm_footprint(const mpm_desc *desc, size_t *device_bytes);

/* Sec. 3 step 2 (the method's object is constructed once and its grid and
 * particle data copied to the device once; the inputs are generated
 * separately, step 1): build a problem in the caller's workspace (device
 * pointer, 256-byte aligned, >= mpm_footprint bytes).  Copies the particles
 * to the device (one host-to-device transfer, converted to the state
 * precision), sets up the static node flags and obstacle normals (the
 * boundary markers and unit normals of step 1 and Sec. 2.2, eq. sdf), the
 * fixed-point quanta, the first cell sort and the first time step (eq. CFL
 * from |V| and the sound speed of the initial state).  Synchronises
 * `hip_stream` before returning.  The host arrays are only read.
 * Errors: MPM_E_ARG (descriptor, ids not a permutation, particle outside
 * the box, non-positive mass or density), MPM_E_WORKSPACE, MPM_E_HIP. */
int mpm_init(const mpm_desc *desc, const mpm_particles_host *particles,
             const mpm_obstacle_host *obstacle, void *dev_workspace,
             size_t workspace_bytes, void *hip_stream, mpm_handle **out);

/* Sec. 3 step 3, the time advancing loop (sub-steps (i)-(xiv) above;
 * Algorithm 1): enqueue n_steps time steps (asynchronous).  Steps after
 * t_end (t_end > 0) or after a device error are skipped on the device.
 * n_steps <= 0 runs to t_end (requires t_end > 0; synchronises once per 64
 * steps to check).  The first call on a handle captures its step graphs
 * (16, 8, 4, 2 and 1 steps; host work of a few milliseconds, before
 * anything is enqueued); every call replays them.  Errors: MPM_E_ARG,
 * MPM_E_STATE (a device error was already reported), MPM_E_HIP. */
int mpm_step(mpm_handle *h, int64_t n_steps, void *hip_stream);

/* The loop of mpm_step for several independent problems at once (the
 * serving form; the paper runs one problem): every sweep of a step is one
 * launch whose workgroups cover the tiles of all problems.  Problems must
 * share dim, shape and precision (else MPM_E_UNSUPPORTED).  n_steps[i]
 * steps for problem i (>= 0); problems that finish early idle.  Up to 64
 * problems per call.  The steps are replays of captured graphs (16, 8, 4, 2
 * and 1 steps): the library keeps, per device, the graphs of the last batch
 * composition (the set of problems), and a call with another composition
 * captures its graphs again (a few milliseconds of host work, before
 * anything is enqueued).  Asynchronous; calls from several host threads are
 * serialised.  Errors: MPM_E_ARG (also a negative step count),
 * MPM_E_UNSUPPORTED, MPM_E_STATE, MPM_E_HIP. */
int mpm_step_batch(mpm_handle *const *hs, int32_t n, const int64_t *n_steps,
                   void *hip_stream);

/* Sec. 3 step 3 (xi) and step 4 (device-to-host copy of the particle
 * state, at intermediate moments and at the end): particle fields, returned
 * as double in id order.  Bit i of field_mask selects field i below;
 * host_out[j] receives the j-th selected field, a caller-owned buffer of
 * n_particles * ncomp doubles, component-major.  Synchronises the stream.
 * Errors: MPM_E_ARG (mask bit beyond MPM_F_ID, a NULL buffer), MPM_E_HIP;
 * otherwise the sticky device error, if any, after copying. */
enum {
    MPM_F_X = 0,    /* dim components                                */
    MPM_F_V = 1,    /* dim                                           */
    MPM_F_M = 2,
    MPM_F_RHO = 3,
    MPM_F_E = 4,    /* specific internal energy                      */
    MPM_F_P = 5,    /* pressure (gamma-1) rho e                      */
    MPM_F_Q = 6,    /* artificial pressure of the next step          */
    MPM_F_G = 7,    /* velocity gradient, dim*dim, row-major (see    */
                    /* below)                                        */
    MPM_F_VOL = 8,  /* M / rho                                       */
    MPM_F_ID = 9
};
/* A step keeps only tr G per particle (the artificial viscosity reads
 * nothing else); the whole G is written by the last step of each run
 * (mpm_step / mpm_step_batch call, or the step reaching t_end).  MPM_F_G
 * returns MPM_E_STATE, without copying, if the last run stopped early
 * without an error (a zero time step: every velocity and sound speed 0). */
int mpm_read_fields(mpm_handle *h, uint32_t field_mask, double *const *host_out,
                    void *hip_stream);

/* Grid snapshot of the last completed step as double, node grid x fastest,
 * component-major (dim comps for MPM_G_P .. MPM_G_FBC, one otherwise):
 * raw P2G mass / momentum / force (Sec. 3 (ii)), momentum after the
 * conditions and the update ((iii)-(iv)), force after the conditions,
 * re-mapped momentum after the conditions ((vi)-(vii)), and the node flags.
 * 2D grids hold each node's finished sum in the state precision (the value
 * the gather sweeps use); 3D grids hold the accumulator words (exact in the
 * fixed-point mode).
 * MPM_G_MPROJ and MPM_G_VOLPROJ are not part of a step: the P2G (eq.
 * p2g_gen) of the particle masses and of the volumes M / rho at the current
 * positions, computed when asked with FP64 atomics; their ratio where the
 * volume is positive is the grid-projected density, an Eulerian read-out
 * of the particle density.  Allocates a temporary device buffer.
 * Synchronises the stream.  Errors: MPM_E_ARG, MPM_E_HIP. */
enum { MPM_G_M = 0, MPM_G_P = 1, MPM_G_F = 2, MPM_G_PUPD = 3, MPM_G_P2 = 4,
       MPM_G_FBC = 5, MPM_G_FLAGS = 6, MPM_G_MPROJ = 7, MPM_G_VOLPROJ = 8 };
int mpm_read_grid(mpm_handle *h, int32_t which, double *host_out, void *hip_stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid it): mpm_read_grid with the
 * same arguments and output, staged through a fixed device buffer of the
 * library (32 MiB per GPU, held until the process ends) instead of a
 * temporary allocation; it calls no allocating routine.  A snapshot larger
 * than the buffer (ncomp * nodes * 8 bytes > 32 MiB, e.g. a 2D grid of
 * more than 2^21 nodes for a vector field) returns MPM_E_SCRATCH.  Every
 * call on a GPU uses that GPU's one buffer: calls that overlap on one GPU
 * (different host threads, or streams not ordered with each other) race
 * and must not be made.  Synchronises the stream.  Errors: MPM_E_ARG,
 * MPM_E_SCRATCH, MPM_E_HIP. */
int mpm_read_grid_noalloc(mpm_handle *h, int32_t which, double *host_out, void *hip_stream);

/* Sec. 3 (xiii)-(xiv) (the time step and the time it advances to) and the
 * checks of a run: time, next and last time step, completed steps and FP64
 * sums over the particles: mass, momentum (3), internal energy sum M e,
 * kinetic energy sum M |v|^2 / 2, as of the last completed step (with
 * `conserved`, one small kernel on the stream reduces them from that step's
 * per-tile sums).  Synchronises the stream.  Any pointer may be NULL.
 * Returns the sticky device error (MPM_E_NONPHYSICAL / MPM_E_OVERFLOW),
 * else MPM_OK. */
int mpm_status(mpm_handle *h, double *t, double *dt_next, double *dt_last,
               int64_t *step, double conserved[6], void *hip_stream);

/* Diagnostic counters: [0] particles whose cell changed between sort and
 * use (handled on a slow path), [1] particles clamped back through a wall,
 * [2] particles recycled at the outflow, [3] reserved (0).  Synchronises. */
int mpm_counters(mpm_handle *h, uint64_t counters[4], void *hip_stream);

/* Per-sweep timing: runs n_steps steps eagerly with a HIP event after each
 * of the MPM_NUM_SWEEPS sweeps of a step and writes the average milliseconds
 * per sweep, in this order: [0] P2G; [1] 2D frame-node reduction (the sums
 * of the frame nodes each tile shares with its neighbours; no kernel in 3D,
 * where those nodes take atomics); [2] G2P + velocity update + P2G of the
 * updated momentum + sort histogram; [3] tile bases of the new order;
 * [4] cell offsets of the new order (2D: with the frame-node reduction of
 * the momentum P2G); [5] G2PD + particle update + move + scatter; [6] time
 * step.  The steps are real steps of the problem, enqueued in batches of
 * 32 steps.  Each slot's time includes the event's own cost (the barrier
 * of an event record); a slot with no kernel (slot [3] when every problem
 * has at most 4096 tiles) measures that cost alone.  Synchronises the
 * stream. */
#define MPM_NUM_SWEEPS 7
int mpm_profile_step(mpm_handle *h, int64_t n_steps, double ms_per_sweep[MPM_NUM_SWEEPS], void *hip_stream);

/* Nodes per axis (n+1 for Q1, n+2 for B2; 1 for unused axes). */
int mpm_grid_shape(const mpm_handle *h, int32_t nodes[3]);

/* Release the handle (host memory only; the workspace stays the caller's). */
int mpm_destroy(mpm_handle *h);

/* Static description of a status code. */
const char *mpm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
