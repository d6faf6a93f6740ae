// Internal layout shared by the host orchestration and the gfx950 kernels.
//
// One problem lives in one caller-owned device workspace.  Its descriptor
// (ProbDev) sits at the start of the workspace; the sweeps read it at the
// start of every workgroup, and the finalize kernel writes the per-step state
// (t, dt, parity, active, error bits), so that a captured graph of several
// steps replays without host involvement.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

// -------------------------------------------------------------- precision --
enum Prec { P_FP64 = 0, P_F32_A64 = 1, P_F32_A32 = 2, P_F32_FIX = 3, P_FP64_COL = 4 };

// real: particle state and node arithmetic; acc: global grid accumulators;
// lacc: per-lane and LDS partial sums.  In the fixed-point precision every
// contribution is rounded to a whole number of quanta before it is added, so
// the partial sums are integers held exactly in FP64 (|sum| < 2^53) and the
// global accumulators are int64.  colour: the P2G sums go through passes of
// a grid colouring with plain adds (FP64 state; no atomics).
template <int PREC> struct PrecT;
template <> struct PrecT<P_FP64>    { using real = double; using acc = double;    using lacc = double; static constexpr bool fixed = false; static constexpr bool colour = false; };
template <> struct PrecT<P_F32_A64> { using real = float;  using acc = double;    using lacc = double; static constexpr bool fixed = false; static constexpr bool colour = false; };
template <> struct PrecT<P_F32_A32> { using real = float;  using acc = float;     using lacc = float;  static constexpr bool fixed = false; static constexpr bool colour = false; };
template <> struct PrecT<P_F32_FIX> { using real = float;  using acc = long long; using lacc = double; static constexpr bool fixed = true;  static constexpr bool colour = false; };
template <> struct PrecT<P_FP64_COL> { using real = double; using acc = double;   using lacc = double; static constexpr bool fixed = false; static constexpr bool colour = true; };

// ------------------------------------------------------------- constants --
enum Shape { S_Q1 = 1, S_B2 = 2 };
enum Face { F_WALL = 0, F_INFLOW = 1, F_OUTFLOW = 2 };

// Node flag bits (static, set at init from the faces and the obstacle mask).
enum : uint8_t { NF_WALL_X = 1, NF_WALL_Y = 2, NF_WALL_Z = 4, NF_INFLOW = 8, NF_OBST = 16 };

// Sticky error bits.
// (A particle clamped back through a wall is counted, DG_WALL, not an error.)
enum : uint32_t { ERR_NONPHYS = 1u, ERR_NONFINITE = 2u, ERR_OVERFLOW = 4u, ERR_INTERNAL = 16u };

// Diagnostic counters (u64).
enum { DG_MISMATCH = 0, DG_WALL = 1, DG_RECYCLE = 2 };   // diag[3] is reserved (0)


// Per-tile partial results of the update sweep (doubles, stored q-major):
// squared max speed, squared max sound speed, mass, momentum (3), M e, M v^2/2.
enum { PT_N = 8 };

// Particle fields stored per parity (arrays of `real`).
// Particle fields.  PF_D holds tr G, the only part of the velocity gradient
// the step itself reads (artificial viscosity); the full G (PF_G, row-major)
// is written by the last step of each run.
enum { PF_X = 0, PF_V = 3, PF_M = 6, PF_RHO = 7, PF_E = 8, PF_G = 9, PF_D = 18, PF_N = 19 };

// Whether a problem of dimension dim stores field f (X and V keep their
// first dim components, G its first dim^2).
__host__ __device__ constexpr bool field_used(int dim, int f) {
    return f < PF_V ? f - PF_X < dim : f < PF_M ? f - PF_V < dim : (f >= PF_G && f < PF_D) ? f - PF_G < dim * dim : true;
}
// Position of field f among the stored fields of one parity (f = PF_N: how
// many there are).  The workspace keeps the stored fields of a parity
// consecutive, one stride apart, in this order.
__host__ __device__ constexpr int field_slot(int dim, int f) {
    int s = 0;
    for (int g = 0; g < f; ++g) s += field_used(dim, g) ? 1 : 0;
    return s;
}

// Tile sizes (cells) per dimension: one lane per cell, 256 lanes per group.
template <int DIM> struct Tile;
template <> struct Tile<2> { static constexpr int X = 16, Y = 16, Z = 1, CELLS = 256; };
template <> struct Tile<3> { static constexpr int X = 8, Y = 8, Z = 4, CELLS = 256; };

constexpr int kBlock = 256;          // threads per workgroup in every sweep
constexpr int kScanItems = 16;       // cells per thread in the scan
constexpr int kScanChunk = kBlock * kScanItems;
constexpr int kMaxBatch = 64;        // problems per batched launch
constexpr int kSweeps = 7;           // sweeps per step: p2g, frame reduce (2D), g2p, tile scan, cell scan,
                                     // update, finalize

struct ProbDev {
    // ---- static geometry and parameters (written once at init)
    int dim, shape, prec, av_form;
    int n[3];             // cells per axis (1 for unused axes)
    int nn[3];            // nodes per axis
    int ntile[3];         // tiles per axis
    int ntiles;           // product of ntile
    int nchunks;          // scan chunks
    long long ncells_pad; // ntiles * cells per tile (size of the key space)
    long long nnodes;
    long long np;
    double lo[3], hi[3], h, inv_h;
    double gamma, c0, c1, cfl;
    int face[3][2];
    double inflow_rho, inflow_p, inflow_e, inflow_u[3], recycle_mass;
    unsigned long long seed;
    double t_end;
    double q_m, q_p, inv_q_m, inv_q_p;   // fixed-point quanta (powers of two)
    int has_obstacle, pad0;

    // ---- device pointers into the workspace
    void *part[2][PF_N];      // particle fields, per parity (real*)
    uint32_t *pid[2];         // particle ids, per parity
    uint32_t *key, *rank;     // new cell key and rank within the cell (from S2); a rank
                              // with the top bit clear is relative to the tile's base
    uint32_t *basetab;        // per tile: first rank of its particles in each footprint cell
    uint32_t *count;          // per-cell histogram of the new keys
    uint32_t *offs[2];        // exclusive prefix of counts, per parity (+1 entry)
    uint32_t *blocksum;       // scan chunk sums (initial sort only)
    uint32_t *ttot;           // per tile: particles of the next order in the tile
    uint32_t *tbase;          // exclusive prefix of ttot (ntiles + 1)
    void *gA[2];              // per step parity: m, p[d], I[d]: (1 + 2 dim) * nnodes acc words
    void *gB[2];              // per step parity: p2[d]: dim * nnodes acc words
    void *haloA, *haloB;      // 2D: per tile, the frame-node partial sums of S1 (NQ per node)
                              // and of the P2G of S2 (dim per node), q-major; null in 3D
    double *partials;         // PT_N * ntiles, q-major
    uint8_t *nflag;
    void *nrm;                // dim * nnodes real, or null

    // ---- per-step state (device-updated)
    double t, dt, dt_last;
    long long step, steps_left;
    int active, parity;
    uint32_t err, pad1;
    long long g_step;     // step count at which PF_G was last written whole

    unsigned long long diag[4];
    double cons[6];
};

// Work table of one batched launch: problem i owns workgroups
// [start[i], start[i+1]).  Passed by value (kernel argument segment).
struct WorkTab {
    ProbDev *prob[kMaxBatch];
    int start[kMaxBatch + 1];
    int n;
    int max_tiles;            // largest tile count of the problems
};

// Up to this many tiles per problem, the cell-offset scan computes each
// tile's base itself (the sum of the earlier tiles' totals) and the tile
// scan is not launched.
constexpr int kFuseTiles = 4096;

}  // namespace mpm
