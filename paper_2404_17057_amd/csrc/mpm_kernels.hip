// gfx950 kernels of the MPM step.
//
// Every sweep is a batched launch: workgroup b belongs to problem
// find_prob(wt, b) and covers one tile of cells (or one chunk of the key
// space).  Particles are kept sorted by the tile-major key of their cell, so
// the particles of a tile are one contiguous range.
//
// Per step (all problems of a batch together), seven sweeps:
//   k_p2g          S1: P2G mass, momentum, impulse dt*f (Sec. 3 (ii)); also
//                  clears the cell histogram of its tile (and, in 3D, the
//                  frame nodes of the other grid buffer for the next step)
//   k_frame_reduce 2D: the frame nodes shared by neighbouring tiles, summed
//                  from the tiles' halo records into the grid
//   k_g2p          S2: conditions + update on the tile load, G2P, FLIP
//                  velocity update, new cell and rank, P2G of M V'
//                  (Sec. 3 (iii)-(vi)); per-tile totals of the new order
//   k_tilescan     one workgroup per problem: tile bases of the new order
//                  (only for problems of more than kFuseTiles tiles)
//   k_cellscan     per tile: offsets of the new order (tile base + cell
//                  prefix); 2D: the frame nodes of the P2G of S2
//   k_update       S3: conditions on p2 on the tile load, G2PD, energy /
//                  density update, move, recycling, scatter into the new
//                  sorted order; per-tile CFL maxima and FP64 sums
//                  (Sec. 3 (vii)-(x), (xii))
//   k_finalize     one workgroup per problem: next dt, t, parity ((xiii)-(xiv))
// Grid accumulators and particle arrays are double-buffered by step parity.
// (An in-kernel "last workgroup" hand-off would need an agent-scope release
// per workgroup, which on this GPU writes back the whole L2 of an XCD.)
//
// P2G (S1, S2): one lane per cell.  The lane walks the particles of its
// cell and sums their contributions to the cell's stencil nodes in
// registers (a particle-level pre-reduction: lanes of one instruction touch
// distinct nodes), then adds the sums into an LDS tile of the footprint
// nodes.  The nodes only this tile reaches are stored into the grid; the
// frame shared with neighbouring tiles goes through per-tile halo records
// (2D) or global atomics (3D).  In the fixed-point precision every
// contribution is rounded to an int64 quantum before any addition, so all
// sums are exact and independent of order.
#include "mpm_device.hpp"

namespace mpm {

template <typename R> struct R3 { R v[3]; };

__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total);

// Tile coordinates of tile t and this lane's cell.
template <int DIM>
__device__ __forceinline__ void tile_cell(const ProbDev *P, int t, int c0[3], int lc[3]) {
    constexpr int TX = Tile<DIM>::X, TY = Tile<DIM>::Y, TZ = Tile<DIM>::Z;
    const int tx = t % P->ntile[0];
    const int ty = (t / P->ntile[0]) % P->ntile[1];
    const int tz = DIM == 3 ? t / (P->ntile[0] * P->ntile[1]) : 0;
    c0[0] = tx * TX; c0[1] = ty * TY; c0[2] = tz * TZ;
    const int l = threadIdx.x;
    lc[0] = l % TX; lc[1] = (l / TX) % TY; lc[2] = DIM == 3 ? l / (TX * TY) : 0;
}

// A tile none of whose cells is the first or last of an axis: the B2
// stencils of its particles take only the uniform pieces (bit for bit the
// values the general form gives there).  A particle whose cell lies outside
// the tile is summed by the general code of each sweep.
template <int DIM, int SHAPE>
__device__ __forceinline__ bool tile_interior(const View &V, const int c0[3]) {
    if constexpr (SHAPE != S_B2) return false;
    constexpr int T[3] = {Tile<DIM>::X, Tile<DIM>::Y, Tile<DIM>::Z};
    bool in = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) in = in && c0[a] >= 1 && c0[a] + T[a] <= V.n[a] - 1;
    return in;
}

// Footprint flush of an LDS partial-sum tile, one value per thread and
// pass (q-major).  Nodes that only this tile's cells reach (local index
// W-1 .. T-1 on every axis) are stored into the grid.  The frame shared with
// neighbouring tiles goes, in 2D, into this tile's halo record (plain
// stores; the readers sum the records of the tiles holding a node), and in
// 3D is added to the grid with one atomic per non-zero value (the frame was
// cleared the step before).
template <int DIM> constexpr bool kHalo = DIM == 2;

// Consecutive tiles per XCD in the tile order of the sweeps (xcd_tile).
// Groups of four keep neighbouring tiles' shared cache lines in one L2
// (cylinder: S2 −10 %, S3 −5 %; 256^3 blast in int64 fixed point: S1 −4 %,
// S2 −1 %, where groups of two or eight gain less).  The other 3D
// precision modes keep the round-robin order in S1 and S2, whose frame nodes
// go through global atomics: FP64 atomics of neighbouring tiles on one XCD
// contend (FP64 S1 +60 %).
template <int DIM, int PREC> constexpr int kXcdGroup = DIM == 2 || PREC == P_F32_FIX ? 4 : 1;
constexpr int kXcdGroupS3 = 4;

// MASS0: value q = 0 is a mass (quantum q_m; the others are momenta, q_p).
template <int DIM, int SHAPE, int PREC, int NQ, bool MASS0>
__device__ __forceinline__ void flush_tile(const ProbDev *P, int t, const int c0[3],
                                           const typename PrecT<PREC>::lacc *tile,
                                           void *g, void *halo, uint32_t &flags) {
    using G = Geo<DIM, SHAPE>;
    using L = typename PrecT<PREC>::lacc;
    using A = typename PrecT<PREC>::acc;
    using GW = typename GridW<DIM, PREC>::type;
    const long long NN = P->nnodes;
    GLOBAL_AS GW *gg = gmem((GW *)g);
    for (int i = threadIdx.x; i < NQ * G::TN; i += kBlock) {
        const int q = i / G::TN, li = i - q * G::TN;
        const int ix = li % G::NX, iy = (li / G::NX) % G::NY, iz = li / (G::NX * G::NY);
        const int gx = c0[0] + ix, gy = c0[1] + iy, gz = c0[2] + iz;
        if (gx >= P->nn[0] || gy >= P->nn[1] || gz >= P->nn[2]) continue;
        const bool own = ix >= G::W - 1 && ix < G::TX && iy >= G::W - 1 && iy < G::TY &&
                         (DIM == 2 || (iz >= G::W - 1 && iz < G::TZ));
        const L val = tile[i];
        if (own) {
            const A a = lacc_to_acc<PREC>(val, flags);
            if constexpr (DIM == 2)
                gg[q * NN + node_index(P, gx, gy, gz)] = from_acc<PREC>(a, MASS0 && q == 0 ? P->q_m : P->q_p, flags);
            else
                gg[q * NN + node_index(P, gx, gy, gz)] = a;
        } else if constexpr (kHalo<DIM>) {
            GLOBAL_AS A *h = gmem((A *)halo);
            h[((long long)q * P->ntiles + t) * Frame2<SHAPE>::NFR + frame_slot<SHAPE>(ix, iy)] =
                lacc_to_acc<PREC>(val, flags);
        } else if (val != (L)0) {
            glb_add(&gg[q * NN + node_index(P, gx, gy, gz)], lacc_to_acc<PREC>(val, flags));
        }
    }
}

// Weight j of an axis by selects (a rolled loop then indexes no array).
template <int W, typename R> __device__ __forceinline__ R pick(const R w[3], int j) {
    return W == 3 ? (j == 0 ? w[0] : (j == 1 ? w[1] : w[2])) : (j == 0 ? w[0] : w[1]);
}

// -------------------------------------------------------------------- S1 --
// Per-particle factors of S1: x-axis products of the separable stencil sums
// for mass, momentum and impulse (all in quanta in the fixed-point mode).
template <int DIM, int SHAPE, typename R> struct S1Factors {
    static constexpr int W = Geo<DIM, SHAPE>::W;
    R mx[W], fx[W], gx[W], px[3][W];
};

// The S1 inputs of one particle.
template <typename R> struct S1In {
    R M, rho, e, v[3], D;    // D = tr G of the previous step
};

template <int DIM, typename R>
__device__ __forceinline__ S1In<R> s1_load_global(const ProbDev *P, int par, uint32_t k) {
    S1In<R> in;
    in.M = gmem((const R *)P->part[par][PF_M])[k];
    in.rho = gmem((const R *)P->part[par][PF_RHO])[k];
    in.e = gmem((const R *)P->part[par][PF_E])[k];
    in.v[0] = in.v[1] = in.v[2] = 0;
    in.D = gmem((const R *)P->part[par][PF_D])[k];
#pragma unroll
    for (int a = 0; a < DIM; ++a) in.v[a] = gmem((const R *)P->part[par][PF_V + a])[k];
    return in;
}

// The per-particle scalars of S1, s[0..4] = M, dt (P+Q) (M/rho) / h and
// M v[0..2] in quanta (the 1/h turns d/ds into d/dx); all zero when `use`
// is false (the particle is summed elsewhere).
template <int DIM, int PREC, class PP>
__device__ __forceinline__ void s1_scalars(const PP *P, const S1In<typename PrecT<PREC>::real> &in,
                                           typename PrecT<PREC>::real s[5], bool use) {
    using R = typename PrecT<PREC>::real;
    const R gam = (R)P->gamma, h = (R)P->h;
    const R M = in.M, rho = in.rho, e = in.e, D = in.D;
    const R p = eos_p(gam, rho, e);
    const R q = art_visc(P->av_form, (R)P->c0, (R)P->c1, gam, h, rho, p, D);
    const R sm = PrecT<PREC>::fixed ? (R)P->inv_q_m : (R)1;
    const R sp = PrecT<PREC>::fixed ? (R)P->inv_q_p : (R)1;
    s[0] = use ? M * sm : (R)0;
    s[1] = use ? (R)P->dt * (p + q) * (M * recip(rho)) * (R)P->inv_h * sp : (R)0;
    s[2] = s[3] = s[4] = (R)0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) s[2 + a] = use ? M * in.v[a] * sp : (R)0;
}

// x-axis products of the S1 scalars.
template <int DIM, int SHAPE, typename R>
__device__ __forceinline__ void s1_products(const R s[5], const Stencil<DIM, SHAPE, R> &st,
                                            S1Factors<DIM, SHAPE, R> &f) {
    constexpr int W = Geo<DIM, SHAPE>::W;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        f.mx[j] = s[0] * st.w[0][j];
        f.fx[j] = s[1] * st.dw[0][j];
        f.gx[j] = s[1] * st.w[0][j];
#pragma unroll
        for (int a = 0; a < DIM; ++a) f.px[a][j] = s[2 + a] * st.w[0][j];
    }
}

template <int DIM, int SHAPE, int PREC, class PP>
__device__ __forceinline__ void s1_factors(const PP *P, const S1In<typename PrecT<PREC>::real> &in,
                                           const Stencil<DIM, SHAPE, typename PrecT<PREC>::real> &st,
                                           S1Factors<DIM, SHAPE, typename PrecT<PREC>::real> &f, bool use = true) {
    using R = typename PrecT<PREC>::real;
    constexpr int W = Geo<DIM, SHAPE>::W;
    const R gam = (R)P->gamma, h = (R)P->h;
    const R M = in.M, rho = in.rho, e = in.e, D = in.D;
    const R *v = in.v;
    const R p = eos_p(gam, rho, e);
    const R q = art_visc(P->av_form, (R)P->c0, (R)P->c1, gam, h, rho, p, D);
    const R sm = PrecT<PREC>::fixed ? (R)P->inv_q_m : (R)1;
    const R sp = PrecT<PREC>::fixed ? (R)P->inv_q_p : (R)1;
    // M, M v and the impulse dt (P+Q) (M/rho) / h (the 1/h turns d/ds into d/dx);
    // all zero when `use` is false (the particle is summed elsewhere)
    const R Ms = use ? M * sm : (R)0;
    const R Fs = use ? (R)P->dt * (p + q) * (M * recip(rho)) * (R)P->inv_h * sp : (R)0;
    R MVs[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) MVs[a] = use ? M * v[a] * sp : (R)0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        f.mx[j] = Ms * st.w[0][j];
        f.fx[j] = Fs * st.dw[0][j];
        f.gx[j] = Fs * st.w[0][j];
#pragma unroll
        for (int a = 0; a < DIM; ++a) f.px[a][j] = MVs[a] * st.w[0][j];
    }
}

// 3D FP32 S1: the first kS1CacheJ particles of every cell keep their scalars
// in LDS (40 KiB); slot (j, lane) of field i is fcache[(i * J + j) * 256 +
// lane], so the lanes of one access touch consecutive words
template <int DIM, typename R> constexpr uint32_t kS1CacheJ = DIM == 3 && sizeof(R) == 4 ? 8 : 0;

template <int DIM, int SHAPE, int PREC>
__global__ __launch_bounds__(kBlock) void k_p2g(WorkTab wt) {
    using G = Geo<DIM, SHAPE>;
    using R = typename PrecT<PREC>::real;
    using L = typename PrecT<PREC>::lacc;
    using A = typename PrecT<PREC>::acc;
    constexpr int NQ = 1 + 2 * DIM;
    constexpr int W = G::W;
    // Particle fields read per particle: X[DIM], V[DIM], M, rho, e, tr G
    constexpr int NPF = 2 * DIM + 4;
    __shared__ L tile[NQ * G::TN];

    const int pi = find_prob(wt, blockIdx.x);
    const ProbDev *P = wt.prob[pi];
    if (!P->active) return;
    const int t = xcd_tile<kXcdGroup<DIM, PREC>>(blockIdx.x - wt.start[pi], P->ntiles);
    // Field pointers of the staged particle arrays, read before any store
    // of the kernel so that they stay uniform (scalar) loads.
    const GLOBAL_AS R *src[NPF];
    {
        const int par0 = P->parity;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            src[a] = gmem((const R *)P->part[par0][PF_X + a]);
            src[DIM + a] = gmem((const R *)P->part[par0][PF_V + a]);
        }
        src[2 * DIM] = gmem((const R *)P->part[par0][PF_M]);
        src[2 * DIM + 1] = gmem((const R *)P->part[par0][PF_RHO]);
        src[2 * DIM + 2] = gmem((const R *)P->part[par0][PF_E]);
        src[2 * DIM + 3] = gmem((const R *)P->part[par0][PF_D]);
    }
    const View V = make_view(P);

    for (int i = threadIdx.x; i < NQ * G::TN; i += kBlock) tile[i] = (L)0;
    __syncthreads();

    int c0[3], lc0[3];
    tile_cell<DIM>(P, t, c0, lc0);
    const bool interior = tile_interior<DIM, SHAPE>(V, c0);
    const bool valid = c0[0] + lc0[0] < P->n[0] && c0[1] + lc0[1] < P->n[1] &&
                       (DIM == 2 || c0[2] + lc0[2] < P->n[2]);
    const int par = P->parity;
    const GLOBAL_AS uint32_t *off = gmem((const uint32_t *)P->offs[par]);
    const uint32_t key = (uint32_t)t * G::CELLS + threadIdx.x;
    const uint32_t beg = valid ? off[key] : 0, end = valid ? off[key + 1] : 0;
    const int *lc = lc0;
    const int cell[3] = {c0[0] + lc[0], c0[1] + lc[1], c0[2] + lc[2]};
    uint32_t flags = 0;
    uint32_t mismatch = 0;

    // Next order: clear this tile's cell histogram and tile total (read by
    // nothing in this sweep, filled by S2).  3D, next step's grid: clear the
    // frame nodes of the other buffer, which the flush adds to atomically
    // (the owned nodes are overwritten by stores; in 2D the frame sums go
    // through the halo records instead).  Each frame node is cleared once,
    // by its designated tile: per axis the tile whose cells start at or below
    // the node and end above it, min(g / T, ntile - 1), which holds the node
    // in its footprint.
    gmem(P->count)[key] = 0;
    if (threadIdx.x == 0) gmem(P->ttot)[t] = 0;
    if constexpr (!kHalo<DIM>) {
        GLOBAL_AS A *gAn = gmem((A *)P->gA[par ^ 1]);
        GLOBAL_AS A *gBn = gmem((A *)P->gB[par ^ 1]);
        const long long NN = P->nnodes;
        const int tx = c0[0] / G::TX, ty = c0[1] / G::TY, tz = c0[2] / G::TZ;
        for (int li = threadIdx.x; li < G::TN; li += kBlock) {
            const int ix = li % G::NX, iy = (li / G::NX) % G::NY, iz = li / (G::NX * G::NY);
            const bool own = ix >= G::W - 1 && ix < G::TX && iy >= G::W - 1 && iy < G::TY &&
                             (DIM == 2 || (iz >= G::W - 1 && iz < G::TZ));
            const int gx = c0[0] + ix, gy = c0[1] + iy, gz = c0[2] + iz;
            if (own || gx >= P->nn[0] || gy >= P->nn[1] || gz >= P->nn[2]) continue;
            if (min(gx / G::TX, P->ntile[0] - 1) != tx || min(gy / G::TY, P->ntile[1] - 1) != ty ||
                min(gz / G::TZ, P->ntile[2] - 1) != tz)
                continue;
            const long long node = node_index(P, gx, gy, gz);
#pragma unroll
            for (int q = 0; q < NQ; ++q) gAn[q * NN + node] = (A)0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) gBn[a * NN + node] = (A)0;
        }
    }

    // 3D FP32: the per-particle scalars of each cell's first FJ particles,
    // computed by the first z-slab pass and read by the other two
    constexpr uint32_t FJ = kS1CacheJ<DIM, R>;
    __shared__ R fcache[FJ > 0 ? 5 * FJ * kBlock : 1];
    // Each lane walks the particles of its cell; the fields of the next
    // particle are loaded while the current one is summed (the index is
    // clamped, so the last iteration reloads its own particle).
    // The particle loop, compiled once for interior tiles (uniform B2
    // pieces only) and once for tiles at a domain face.
    auto sweep = [&](auto edge_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
#pragma unroll 1
        for (int pass = 0; pass < G::PASSES; ++pass) {
            L acc[G::WP][NQ];
#pragma unroll
            for (int s = 0; s < G::WP; ++s)
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc[s][q] = acc_zero<PREC>();

            // a particle whose scalars the first pass cached loads only X again
            auto need = [&](int f, uint32_t kk) { return !(pass > 0 && f >= DIM && kk - beg < FJ); };
            R cur[NPF];
#pragma unroll
            for (int f = 0; f < NPF; ++f) cur[f] = end > beg && need(f, beg) ? ldk(src[f], beg) : (R)0;
#pragma unroll 1
            for (uint32_t k = beg; k < end; ++k) {
                R nxt[NPF];
                const uint32_t kn = min(k + 1, end - 1);
#pragma unroll
                for (int f = 0; f < NPF; ++f) nxt[f] = need(f, kn) ? ldk(src[f], kn) : (R)0;
                R x[3] = {0, 0, 0};
                S1In<R> in;
                in.v[0] = in.v[1] = in.v[2] = 0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    x[a] = cur[a];
                    in.v[a] = cur[DIM + a];
                }
                in.D = cur[2 * DIM + 3];
                in.M = cur[2 * DIM];
                in.rho = cur[2 * DIM + 1];
                in.e = cur[2 * DIM + 2];
                Stencil<DIM, SHAPE, R> st;
                make_stencil<DIM, SHAPE, R, EDGE>(&V, x, st);
                // A particle whose cell changed between sort and use adds zeros
                // here (no divergence in the register sums) and is summed by the
                // deferred loop below (rare).
                const bool own = st.c[0] == cell[0] && st.c[1] == cell[1] && (DIM == 2 || st.c[2] == cell[2]);
                if (pass == 0) mismatch += own ? 0u : 1u;
                // the particle's scalars: computed, or in 3D cached by the first
                // pass for the other two
                R sc[5];
                const uint32_t kj = k - beg;
                if (pass > 0 && kj < FJ) {
#pragma unroll
                    for (int i = 0; i < 5; ++i) sc[i] = fcache[(i * FJ + kj) * kBlock + threadIdx.x];
                } else {
                    s1_scalars<DIM, PREC>(&V, in, sc, own);
                    if (kj < FJ)
#pragma unroll
                        for (int i = 0; i < 5; ++i) fcache[(i * FJ + kj) * kBlock + threadIdx.x] = sc[i];
                }
                S1Factors<DIM, SHAPE, R> f;
                s1_products<DIM, SHAPE, R>(sc, st, f);
                const R wz = DIM == 3 ? pick<W, R>(st.w[2], pass) : (R)1;
                const R dwz = DIM == 3 ? pick<W, R>(st.dw[2], pass) : (R)0;
#pragma unroll
                for (int jy = 0; jy < W; ++jy) {
                    const auto wyz = weight<PREC>(DIM == 3 ? st.w[1][jy] * wz : st.w[1][jy]);
                    const auto dyz = weight<PREC>(DIM == 3 ? st.dw[1][jy] * wz : st.dw[1][jy]);
                    const auto ydz = weight<PREC>(st.w[1][jy] * dwz);
#pragma unroll
                    for (int jx = 0; jx < W; ++jx) {
                        L *ac = acc[jy * W + jx];
                        ac[0] = accum<PREC>(ac[0], f.mx[jx], wyz);
#pragma unroll
                        for (int a = 0; a < DIM; ++a) ac[1 + a] = accum<PREC>(ac[1 + a], f.px[a][jx], wyz);
                        ac[1 + DIM] = accum<PREC>(ac[1 + DIM], f.fx[jx], wyz);
                        ac[2 + DIM] = accum<PREC>(ac[2 + DIM], f.gx[jx], dyz);
                        if constexpr (DIM == 3) ac[3 + DIM] = accum<PREC>(ac[3 + DIM], f.gx[jx], ydz);
                    }
                }
#pragma unroll
                for (int f = 0; f < NPF; ++f) cur[f] = nxt[f];
            }
            if (end > beg) {
                const int lz = DIM == 3 ? lc[2] + pass : 0;
#pragma unroll
                for (int jy = 0; jy < W; ++jy)
#pragma unroll
                    for (int jx = 0; jx < W; ++jx) {
                        const int li = (lz * G::NY + (lc[1] + jy)) * G::NX + (lc[0] + jx);
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            // zeros are added too: a test per value costs more
                            // than the LDS atomic it saves (2D S1 52.3 -> 49.9
                            // us, 3D S1 6.59 -> 6.45 ms)
                            lds_add(&tile[q * G::TN + li], unbias<PREC>(acc[jy * W + jx][q]));
                        }
                    }
            }
        }
    };
    if (interior) sweep(std::false_type{});
    else sweep(std::true_type{});
    if (mismatch) {
        // Particles whose cell changed between sort and use: their
        // contributions go one by one into the LDS tile (their cell must
        // still lie in this tile).
#pragma unroll 1
        for (uint32_t k = beg; k < end; ++k) {
            R x[3] = {0, 0, 0};
            for (int a = 0; a < DIM; ++a) x[a] = gmem((const R *)P->part[par][PF_X + a])[k];
            Stencil<DIM, SHAPE, R> st;
            make_stencil<DIM, SHAPE, R>(P, x, st);
            if (st.c[0] == cell[0] && st.c[1] == cell[1] && (DIM == 2 || st.c[2] == cell[2])) continue;
            const int l0[3] = {st.c[0] - c0[0], st.c[1] - c0[1], DIM == 3 ? st.c[2] - c0[2] : 0};
            if (l0[0] < 0 || l0[0] >= G::TX || l0[1] < 0 || l0[1] >= G::TY ||
                (DIM == 3 && (l0[2] < 0 || l0[2] >= G::TZ))) {
                flags |= ERR_INTERNAL;
                continue;
            }
            S1Factors<DIM, SHAPE, R> f;
            s1_factors<DIM, SHAPE, PREC>(&V, s1_load_global<DIM, R>(P, par, k), st, f);
#pragma unroll 1
            for (int jz = 0; jz < (DIM == 3 ? W : 1); ++jz)
#pragma unroll 1
                for (int jy = 0; jy < W; ++jy) {
                    const R wz = DIM == 3 ? pick<W, R>(st.w[2], jz) : (R)1;
                    const R wy = pick<W, R>(st.w[1], jy), dy = pick<W, R>(st.dw[1], jy);
                    const R wyz = wy * wz, dyz = dy * wz;
                    const R ydz = DIM == 3 ? wy * pick<W, R>(st.dw[2], jz) : (R)0;
                    for (int jx = 0; jx < W; ++jx) {
                        const int li = ((l0[2] + jz) * G::NY + (l0[1] + jy)) * G::NX + (l0[0] + jx);
                        lds_add(&tile[li], term_exact<PREC>(f.mx[jx], wyz));
                        for (int a = 0; a < DIM; ++a) lds_add(&tile[(1 + a) * G::TN + li], term_exact<PREC>(f.px[a][jx], wyz));
                        lds_add(&tile[(1 + DIM) * G::TN + li], term_exact<PREC>(f.fx[jx], wyz));
                        lds_add(&tile[(2 + DIM) * G::TN + li], term_exact<PREC>(f.gx[jx], dyz));
                        if (DIM == 3) lds_add(&tile[(3 + DIM) * G::TN + li], term_exact<PREC>(f.gx[jx], ydz));
                    }
                }
        }
    }
    __syncthreads();
    flush_tile<DIM, SHAPE, PREC, NQ, true>(P, t, c0, tile, P->gA[par], P->haloA, flags);
    if (flags & (ERR_OVERFLOW | ERR_INTERNAL)) atomicOr((uint32_t *)&P->err, flags & (ERR_OVERFLOW | ERR_INTERNAL));
    if (mismatch) atomicAdd((unsigned long long *)&P->diag[DG_MISMATCH], (unsigned long long)mismatch);
}

// Per-node stride of the staged footprint: vstar and dvel (S2), plus v2 (S3).
// Floats per staged node.  S2's 2 DIM fields take one pad float: an odd
// stride spreads the lane-per-cell G2P reads over the LDS banks (3D S2 6.38
// -> 6.24 ms; 2D unchanged).  S3's 3 DIM is odd in 3D.
template <int DIM, bool WITH_B> constexpr int stage_stride() { return WITH_B ? 3 * DIM : 2 * DIM + 1; }

// Stage the tile footprint of nodes, interleaved per node:
// lds[li * NF + f]: f < DIM vstar, DIM <= f < 2 DIM dvel, 2 DIM <= f v2 (S3).
template <int DIM, int SHAPE, int PREC, bool WITH_B>
__device__ __forceinline__ void stage_tile(const ProbDev *P, const int c0[3],
                                           typename PrecT<PREC>::real *lds, uint32_t &flags) {
    using G = Geo<DIM, SHAPE>;
    using R = typename PrecT<PREC>::real;
    constexpr int NF = stage_stride<DIM, WITH_B>();
#pragma unroll 1
    for (int li = threadIdx.x; li < G::TN; li += kBlock) {
        const int ix = li % G::NX, iy = (li / G::NX) % G::NY, iz = li / (G::NX * G::NY);
        const int gx = c0[0] + ix, gy = c0[1] + iy, gz = c0[2] + iz;
        R vs[3] = {0, 0, 0}, dv[3] = {0, 0, 0}, v2[3] = {0, 0, 0};
        if (gx < P->nn[0] && gy < P->nn[1] && gz < P->nn[2]) {
            const long long node = node_index(P, gx, gy, gz);
            stage_A<DIM, PREC>(P, node, vs, dv, flags);
            if constexpr (WITH_B) stage_B<DIM, PREC>(P, node, v2, flags);
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            lds[li * NF + a] = vs[a];
            lds[li * NF + DIM + a] = dv[a];
            if constexpr (WITH_B) lds[li * NF + 2 * DIM + a] = v2[a];
        }
    }
}

// Staged value f of node (l0 + j) of the footprint.
template <int DIM, int SHAPE, typename R, int NF>
__device__ __forceinline__ const R *node_ptr(const R *lds, const int l0[3], int jx, int jy, int jz) {
    using G = Geo<DIM, SHAPE>;
    return lds + (((l0[2] + jz) * G::NY + (l0[1] + jy)) * G::NX + (l0[0] + jx)) * NF;
}

// G2P of one staged vector field (fields OFF..OFF+DIM-1 of the node) at one
// particle, summed row by row: out = sum_z,y w_z w_y (sum_x w_x f).  S2 and
// S3 both call this (vstar and dvel), so the same particle gets the same
// bits in both sweeps.  ROLLED keeps the z loop of 3D rolled (fewer live
// registers; the same operations in the same order).
template <int DIM, int SHAPE, typename R, int NF, int OFF, bool ROLLED = false>
__device__ __forceinline__ void g2p_field(const R *lds, const Stencil<DIM, SHAPE, R> &st, const int l0[3], R out[3]) {
    constexpr int W = Geo<DIM, SHAPE>::W;
    constexpr int kZUnroll = ROLLED ? 1 : 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = 0;
#pragma unroll kZUnroll
    for (int jz = 0; jz < (DIM == 3 ? W : 1); ++jz)
#pragma unroll
        for (int jy = 0; jy < W; ++jy) {
            R row[3] = {0, 0, 0};
#pragma unroll
            for (int jx = 0; jx < W; ++jx) {
                const R *nd = node_ptr<DIM, SHAPE, R, NF>(lds, l0, jx, jy, jz);
#pragma unroll
                for (int a = 0; a < DIM; ++a) row[a] += st.w[0][jx] * nd[OFF + a];
            }
            const R wyz = DIM == 3 ? st.w[1][jy] * pick<W, R>(st.w[2], jz) : st.w[1][jy];
#pragma unroll
            for (int a = 0; a < DIM; ++a) out[a] += wyz * row[a];
        }
}

// The same G2P sums computed from the global grid, for a particle whose
// stencil leaves the staged footprint: node values from the same staging
// functions, summed in the same order.  vbar and dv are the G2P of vstar and
// dvel; with WITH_G, Gm is the G2PD of v2.  Used only by the deferred loops.
template <int DIM, int SHAPE, int PREC, bool WITH_G>
__device__ __forceinline__ void g2p_global(const ProbDev *P, const Stencil<DIM, SHAPE, typename PrecT<PREC>::real> &st,
                                           typename PrecT<PREC>::real vbar[3], typename PrecT<PREC>::real dv[3],
                                           typename PrecT<PREC>::real Gm[9], uint32_t &flags) {
    using R = typename PrecT<PREC>::real;
    constexpr int W = Geo<DIM, SHAPE>::W;
    const R inv_h = (R)P->inv_h;
    for (int a = 0; a < 3; ++a) { vbar[a] = 0; dv[a] = 0; }
    for (int c = 0; c < 9; ++c) Gm[c] = 0;
#pragma unroll 1
    for (int jz = 0; jz < (DIM == 3 ? W : 1); ++jz)
#pragma unroll 1
        for (int jy = 0; jy < W; ++jy) {
            R row[3] = {0, 0, 0}, rowd[3] = {0, 0, 0}, row2[3] = {0, 0, 0}, sx[3] = {0, 0, 0};
            for (int jx = 0; jx < W; ++jx) {
                const long long node = node_index(P, st.c[0] + jx, st.c[1] + jy, DIM == 3 ? st.c[2] + jz : 0);
                R vs[3], d[3], v2[3] = {0, 0, 0};
                stage_A<DIM, PREC>(P, node, vs, d, flags);
                if constexpr (WITH_G) stage_B<DIM, PREC>(P, node, v2, flags);
                for (int a = 0; a < DIM; ++a) {
                    row[a] += st.w[0][jx] * vs[a];
                    rowd[a] += st.w[0][jx] * d[a];
                    if constexpr (WITH_G) {
                        row2[a] += st.w[0][jx] * v2[a];
                        sx[a] += st.dw[0][jx] * v2[a];
                    }
                }
            }
            const R wyz = DIM == 3 ? st.w[1][jy] * st.w[2][jz] : st.w[1][jy];
            const R dyz = DIM == 3 ? st.dw[1][jy] * st.w[2][jz] : st.dw[1][jy];
            const R ydz = DIM == 3 ? st.w[1][jy] * st.dw[2][jz] : (R)0;
            for (int a = 0; a < DIM; ++a) {
                vbar[a] += wyz * row[a];
                dv[a] += wyz * rowd[a];
                if constexpr (WITH_G) {
                    Gm[a * DIM + 0] += wyz * sx[a];
                    Gm[a * DIM + 1] += dyz * row2[a];
                    if (DIM == 3) Gm[a * DIM + 2] += ydz * row2[a];
                }
            }
        }
    for (int c = 0; c < DIM * DIM; ++c) Gm[c] *= inv_h;
}

// Local index of a cell in the tile's destination footprint (cells c0-1 ..
// c0+T per axis), or -1 when the cell lies outside it.
template <int DIM>
__device__ __forceinline__ int dest_local(const int c0[3], const int cn[3]) {
    constexpr int TX = Tile<DIM>::X, TY = Tile<DIM>::Y, TZ = Tile<DIM>::Z;
    const int lx = cn[0] - c0[0] + 1, ly = cn[1] - c0[1] + 1, lz = DIM == 3 ? cn[2] - c0[2] + 1 : 0;
    if (lx < 0 || lx >= TX + 2 || ly < 0 || ly >= TY + 2 || (DIM == 3 && (lz < 0 || lz >= TZ + 2))) return -1;
    return (lz * (TY + 2) + ly) * (TX + 2) + lx;
}
template <int DIM> struct DestFoot {
    static constexpr int N = (Tile<DIM>::X + 2) * (Tile<DIM>::Y + 2) * (DIM == 3 ? Tile<DIM>::Z + 2 : 1);
};

// Rank word of a particle in the next order.  Bit 31 set: bits 0-30 are the
// rank in the cell's global count.  Clear: bits 21-30 are the destination
// cell's index in the tile's destination footprint, bits 0-20 the rank among
// this tile's particles of that cell.
constexpr uint32_t kRankGlobal = 0x80000000u;
constexpr int kRankShift = 21;
constexpr uint32_t kRankMask = (1u << kRankShift) - 1u;
static_assert(DestFoot<3>::N <= 1024 && DestFoot<2>::N <= 1024, "footprint index must fit 10 bits");

// -------------------------------------------------------------------- S2 --
// New position of a particle -> its new cell key, and its rank within the
// cell: from the tile's LDS histogram when the cell lies in the tile's
// destination footprint (made global by one atomic per cell at the end),
// else straight from the global histogram (flagged).
template <int DIM, typename R, class PP>
__device__ __forceinline__ void s2_key_rank(const PP *P, GLOBAL_AS uint32_t *count, GLOBAL_AS uint32_t *ttot, const R x[3],
                                            const R vbar[3], R dt, IdAt id, const int c0[3], uint32_t *hist,
                                            uint32_t &nk, uint32_t &rank, uint32_t &flags) {
    R xn[3] = {x[0], x[1], x[2]};
    advect<DIM, R>(P, xn, vbar, dt, id);
    int cn[3];
    cell_of<DIM, R>(P, xn, cn);
    nk = cell_key<DIM>(P, cn);
    const int dl = dest_local<DIM>(c0, cn);
    if (dl >= 0) {
        const uint32_t r = atomicAdd(&hist[dl], 1u);
        if (r > kRankMask) flags |= ERR_INTERNAL;
        rank = ((uint32_t)dl << kRankShift) | (r & kRankMask);
    } else {
        rank = __hip_atomic_fetch_add(&count[nk], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) | kRankGlobal;
        __hip_atomic_fetch_add(&ttot[nk / Tile<DIM>::CELLS], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

constexpr uint32_t kRankBuf = 2048;   // S2: rank words staged in LDS per tile
// 3D FP32 S2: V' of each cell's first 8 particles kept in LDS (24 KiB) by
// the first z-slab pass for the other two (with an FP64 state the larger
// tile leaves it slower); slot (j, lane) of component a is
// vcache[(a * J + j) * 256 + lane]
template <int DIM, typename R> constexpr uint32_t kVCacheJ = DIM == 3 && sizeof(R) == 4 ? 8 : 0;

template <int DIM, int SHAPE, int PREC>
__global__ __launch_bounds__(kBlock) void k_g2p(WorkTab wt) {
    using G = Geo<DIM, SHAPE>;
    using R = typename PrecT<PREC>::real;
    using L = typename PrecT<PREC>::lacc;
    constexpr int W = G::W;
    constexpr int NF = stage_stride<DIM, false>();
    constexpr int ND = DestFoot<DIM>::N;
    // the colouring precision does its P2G of M V' in colour passes after
    // this sweep; here only the G2P of the move, the new cell and the rank
    constexpr bool kP2G = !PrecT<PREC>::colour;
    // Particle fields read per particle: X[DIM], V[DIM], M (the id only for a
    // particle recycled at the outflow)
    constexpr int NPF = 2 * DIM + 1;
    __shared__ R stage[NF * G::TN];
    __shared__ L tile[DIM * G::TN];
    __shared__ uint32_t hist[ND];

    const int pi = find_prob(wt, blockIdx.x);
    const ProbDev *P = wt.prob[pi];
    if (!P->active) return;
    const int t = xcd_tile<kXcdGroup<DIM, PREC>>(blockIdx.x - wt.start[pi], P->ntiles);
    // Field pointers, read before any store of the kernel (uniform loads)
    const GLOBAL_AS R *src[NPF];
    const GLOBAL_AS uint32_t *idg;
    {
        const int par0 = P->parity;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            src[a] = gmem((const R *)P->part[par0][PF_X + a]);
            src[DIM + a] = gmem((const R *)P->part[par0][PF_V + a]);
        }
        src[2 * DIM] = gmem((const R *)P->part[par0][PF_M]);
        idg = gmem((const uint32_t *)P->pid[par0]);
    }
    const View V = make_view(P);
    GLOBAL_AS uint32_t *const cnt_g = gmem(P->count), *const ttot_g = gmem(P->ttot);
    int c0[3], lc0[3];
    tile_cell<DIM>(P, t, c0, lc0);
    const bool interior = tile_interior<DIM, SHAPE>(V, c0);
    uint32_t flags = 0;

    for (int i = threadIdx.x; i < DIM * G::TN; i += kBlock) tile[i] = (L)0;
    for (int i = threadIdx.x; i < ND; i += kBlock) hist[i] = 0;
    stage_tile<DIM, SHAPE, PREC, false>(P, c0, stage, flags);
    __syncthreads();

    const bool valid = c0[0] + lc0[0] < P->n[0] && c0[1] + lc0[1] < P->n[1] &&
                       (DIM == 2 || c0[2] + lc0[2] < P->n[2]);
    const int par = P->parity;
    const GLOBAL_AS uint32_t *off = gmem((const uint32_t *)P->offs[par]);
    const uint32_t key = (uint32_t)t * G::CELLS + threadIdx.x;
    const uint32_t beg = valid ? off[key] : 0, end = valid ? off[key + 1] : 0;
    const int *lc = lc0;
    const int cell[3] = {c0[0] + lc[0], c0[1] + lc[1], c0[2] + lc[2]};
    const GLOBAL_AS R *Mp = gmem((const R *)P->part[par][PF_M]);
    const GLOBAL_AS uint32_t *ids = gmem((const uint32_t *)P->pid[par]);
    const R dt = (R)V.dt;
    const R sp = PrecT<PREC>::fixed ? (R)V.inv_q_p : (R)1;
    uint32_t mismatch = 0;

    // Rank words of the tile's particle range [tb, tb + kRankBuf) are
    // collected in LDS and stored contiguously at the end (a lane per cell
    // would store them 64 cells apart); the rest of a denser tile directly.
    GLOBAL_AS uint32_t *rankg = gmem(P->rank);
    const uint32_t tb = off[(uint32_t)t * G::CELLS];
    const uint32_t tn = off[(uint32_t)(t + 1) * G::CELLS] - tb;
    __shared__ uint32_t rbuf[kRankBuf];
    constexpr uint32_t VJ = kVCacheJ<DIM, R>;
    __shared__ R vcache[VJ > 0 ? DIM * VJ * kBlock : 1];
    auto put_rank = [&](uint32_t k, uint32_t rk) {
        if (k - tb < kRankBuf) rbuf[k - tb] = rk;
        else stk(rankg, k, rk);
    };
    // Each lane walks the particles of its cell, loading the next
    // particle's fields while the current one is processed.
    // (compiled once for interior tiles, uniform B2 pieces only, and once
    // for tiles at a domain face)
    auto sweep = [&](auto edge_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
#pragma unroll 1
        for (int pass = 0; pass < (kP2G ? G::PASSES : 1); ++pass) {
            L acc[G::WP][DIM];
#pragma unroll
            for (int s = 0; s < G::WP; ++s)
#pragma unroll
                for (int a = 0; a < DIM; ++a) acc[s][a] = acc_zero<PREC>();

            // V of a particle whose V' the first pass cached is not loaded again
            auto need = [&](int f, uint32_t kk) {
                return !(pass > 0 && f >= DIM && f < 2 * DIM && kk - beg < VJ);
            };
            R cur[NPF];
#pragma unroll
            for (int f = 0; f < NPF; ++f) cur[f] = end > beg && need(f, beg) ? ldk(src[f], beg) : (R)0;
#pragma unroll 1
            for (uint32_t k = beg; k < end; ++k) {
                R nxt[NPF];
                const uint32_t kn = min(k + 1, end - 1);
#pragma unroll
                for (int f = 0; f < NPF; ++f) nxt[f] = need(f, kn) ? ldk(src[f], kn) : (R)0;
                R x[3] = {0, 0, 0}, v[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    x[a] = cur[a];
                    v[a] = cur[DIM + a];
                }
                Stencil<DIM, SHAPE, R> st;
                make_stencil<DIM, SHAPE, R, EDGE>(&V, x, st);
                // A particle whose cell changed between sort and use adds zeros
                // here and is handled by the deferred loop below (rare).
                const bool own = st.c[0] == cell[0] && st.c[1] == cell[1] && (DIM == 2 || st.c[2] == cell[2]);
                if (pass == 0) mismatch += own ? 0u : 1u;
                // G2P of the velocity increment, row by row: V' = V + dv.  V'
                // is not stored (the update sweep recomputes it from the same
                // staged values, same bits).  In 3D the first pass keeps it in
                // LDS for the other two.
                const uint32_t kj = k - beg;
                if (!kP2G) {
                    // V' is not needed here
                } else if (pass > 0 && kj < VJ) {
#pragma unroll
                    for (int a = 0; a < DIM; ++a) v[a] = vcache[(a * VJ + kj) * kBlock + threadIdx.x];
                } else {
                    R dv[3];
                    g2p_field<DIM, SHAPE, R, NF, DIM>(stage, st, lc, dv);
#pragma unroll
                    for (int a = 0; a < DIM; ++a) v[a] = v[a] + dv[a];
                    if (kj < VJ)
#pragma unroll
                        for (int a = 0; a < DIM; ++a) vcache[(a * VJ + kj) * kBlock + threadIdx.x] = v[a];
                }
                if (pass == 0 && own) {
                    // G2P of vstar: the move, the new cell key and the rank
                    R vbar[3];
                    g2p_field<DIM, SHAPE, R, NF, 0>(stage, st, lc, vbar);
                    uint32_t nk, rk;
                    s2_key_rank<DIM, R>(&V, cnt_g, ttot_g, x, vbar, dt, IdAt{idg, k}, c0, hist, nk, rk, flags);
                    put_rank(k, rk);
                }
                if constexpr (kP2G) {
                const R Ms = own ? cur[2 * DIM] * sp : (R)0;
                R px[3][W];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const R mv = own ? Ms * v[a] : (R)0;
#pragma unroll
                    for (int j = 0; j < W; ++j) px[a][j] = mv * st.w[0][j];
                }
                const R wz = DIM == 3 ? pick<W, R>(st.w[2], pass) : (R)1;
#pragma unroll
                for (int jy = 0; jy < W; ++jy) {
                    const auto wyz = weight<PREC>(DIM == 3 ? st.w[1][jy] * wz : st.w[1][jy]);
#pragma unroll
                    for (int jx = 0; jx < W; ++jx)
#pragma unroll
                        for (int a = 0; a < DIM; ++a) acc[jy * W + jx][a] = accum<PREC>(acc[jy * W + jx][a], px[a][jx], wyz);
                }
                }
#pragma unroll
                for (int f = 0; f < NPF; ++f) cur[f] = nxt[f];
            }
            if (kP2G && end > beg) {
                const int lz = DIM == 3 ? lc[2] + pass : 0;
#pragma unroll
                for (int jy = 0; jy < W; ++jy)
#pragma unroll
                    for (int jx = 0; jx < W; ++jx) {
                        const int li = (lz * G::NY + (lc[1] + jy)) * G::NX + (lc[0] + jx);
#pragma unroll
                        for (int a = 0; a < DIM; ++a) {
                            lds_add(&tile[a * G::TN + li], unbias<PREC>(acc[jy * W + jx][a]));
                        }
                    }
            }
        }
    };
    if (interior) sweep(std::false_type{});
    else sweep(std::true_type{});
    if (mismatch) {
        // Particles whose cell changed between sort and use: G2P from the
        // global grid, P2G into the LDS tile (their cell must still lie in
        // this tile).
#pragma unroll 1
        for (uint32_t k = beg; k < end; ++k) {
            R x[3] = {0, 0, 0}, v[3] = {0, 0, 0};
            for (int a = 0; a < DIM; ++a) {
                x[a] = gmem((const R *)P->part[par][PF_X + a])[k];
                v[a] = gmem((const R *)P->part[par][PF_V + a])[k];
            }
            Stencil<DIM, SHAPE, R> st;
            make_stencil<DIM, SHAPE, R>(&V, x, st);
            if (st.c[0] == cell[0] && st.c[1] == cell[1] && (DIM == 2 || st.c[2] == cell[2])) continue;
            const int l0[3] = {st.c[0] - c0[0], st.c[1] - c0[1], DIM == 3 ? st.c[2] - c0[2] : 0};
            if (l0[0] < 0 || l0[0] >= G::TX || l0[1] < 0 || l0[1] >= G::TY ||
                (DIM == 3 && (l0[2] < 0 || l0[2] >= G::TZ))) {
                flags |= ERR_INTERNAL;
                continue;
            }
            R vbar[3], dv[3], Gd[9];
            g2p_global<DIM, SHAPE, PREC, false>(P, st, vbar, dv, Gd, flags);
            for (int a = 0; a < DIM; ++a) v[a] = v[a] + dv[a];
            uint32_t nk, rk;
            s2_key_rank<DIM, R>(&V, cnt_g, ttot_g, x, vbar, dt, IdAt{ids, k}, c0, hist, nk, rk, flags);
            put_rank(k, rk);
            const R Ms = Mp[k] * sp;
            if (!kP2G) continue;
#pragma unroll 1
            for (int jz = 0; jz < (DIM == 3 ? W : 1); ++jz)
#pragma unroll 1
                for (int jy = 0; jy < W; ++jy)
                    for (int jx = 0; jx < W; ++jx) {
                        const R wy = pick<W, R>(st.w[1], jy);
                        const R wyz = DIM == 3 ? wy * pick<W, R>(st.w[2], jz) : wy;
                        const int li = ((l0[2] + jz) * G::NY + (l0[1] + jy)) * G::NX + (l0[0] + jx);
                        for (int a = 0; a < DIM; ++a)
                            lds_add(&tile[a * G::TN + li], term_exact<PREC>((Ms * v[a]) * st.w[0][jx], wyz));
                    }
        }
    }
    __shared__ uint32_t ttl[27];
    if (threadIdx.x < 27) ttl[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < min(tn, kRankBuf); i += kBlock) stk(rankg, tb + i, rbuf[i]);
    if constexpr (kP2G) flush_tile<DIM, SHAPE, PREC, DIM, false>(P, t, c0, tile, P->gB[par], P->haloB, flags);
    // One global histogram atomic per destination cell of this tile: the
    // tile's particles of that cell get the ranks base .. base + hist - 1.
    // Tile totals are gathered per destination tile (the tile and its
    // neighbours) before going global.
    GLOBAL_AS uint32_t *bt = gmem(P->basetab) + (long long)t * ND;
    const int ttx = c0[0] / G::TX, tty = c0[1] / G::TY, ttz = c0[2] / G::TZ;
    for (int i = threadIdx.x; i < ND; i += kBlock) {
        const uint32_t cnt = hist[i];
        if (!cnt) continue;
        const int lx = i % (G::TX + 2), ly = (i / (G::TX + 2)) % (G::TY + 2), lz = i / ((G::TX + 2) * (G::TY + 2));
        const int cn[3] = {c0[0] + lx - 1, c0[1] + ly - 1, DIM == 3 ? c0[2] + lz - 1 : 0};
        bt[i] = __hip_atomic_fetch_add(&cnt_g[cell_key<DIM>(P, cn)], cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int dx = (cn[0] >= c0[0] + G::TX) - (cn[0] < c0[0]);
        const int dy = (cn[1] >= c0[1] + G::TY) - (cn[1] < c0[1]);
        const int dz = DIM == 3 ? (cn[2] >= c0[2] + G::TZ) - (cn[2] < c0[2]) : 0;
        atomicAdd(&ttl[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)], cnt);
    }
    __syncthreads();
    if (threadIdx.x < 27 && ttl[threadIdx.x]) {
        const int i = threadIdx.x;
        const int dx = i % 3 - 1, dy = (i / 3) % 3 - 1, dz = i / 9 - 1;
        const long long tile = ((long long)(ttz + dz) * P->ntile[1] + (tty + dy)) * P->ntile[0] + (ttx + dx);
        __hip_atomic_fetch_add(&ttot_g[tile], ttl[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (flags & (ERR_OVERFLOW | ERR_INTERNAL)) atomicOr((uint32_t *)&P->err, flags & (ERR_OVERFLOW | ERR_INTERNAL));
    if (mismatch) atomicAdd((unsigned long long *)&P->diag[DG_MISMATCH], (unsigned long long)mismatch);
}

// ------------------------------------------------------ colouring P2G --
// The P2G of the colouring precision (grid colouring, Sec. 5): a cell's B2
// stencil spans W = 3 nodes per axis, so cells whose coordinates agree modulo
// 3 have disjoint stencils.  One launch per colour; one thread per cell of
// that colour sums its cell's particles, in increasing particle id (a
// canonical order, whatever order the sort left), into registers and adds
// the sums into the grid with plain loads and stores: no other thread of the
// launch touches those nodes, and the launches of one P2G run in colour
// order.  Sums are therefore bit-reproducible without fixed point.

// Zeroes this step's grids (the colour passes add into them) and, like S1,
// the cell histogram and tile totals of the next order.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_zero_grid(WorkTab wt) {
    const int pi = find_prob(wt, blockIdx.x);
    ProbDev *P = wt.prob[pi];
    if (!P->active) return;
    const int t = blockIdx.x - wt.start[pi];
    const int par = P->parity;
    gmem(P->count)[(uint32_t)t * Tile<DIM>::CELLS + threadIdx.x] = 0;
    if (threadIdx.x == 0) gmem(P->ttot)[t] = 0;
    const long long na = (long long)(1 + 2 * DIM) * P->nnodes, nb = (long long)DIM * P->nnodes;
    const long long per = (na + nb + P->ntiles - 1) / P->ntiles;
    GLOBAL_AS double *ga = gmem((double *)P->gA[par]);
    GLOBAL_AS double *gb = gmem((double *)P->gB[par]);
    const long long i1 = min((long long)(t + 1) * per, na + nb);
    for (long long i = (long long)t * per + threadIdx.x; i < i1; i += kBlock) {
        if (i < na) ga[i] = 0.0;
        else gb[i - na] = 0.0;
    }
}

// One colour pass.  WHICH = 0: m, p and dt f of S1 into gA; WHICH = 1: the
// P2G of M V' into gB, V' = V + dt A from the conditioned grid of S1 (the
// same values and order as the gather sweeps).
template <int DIM, int SHAPE, int PREC, int WHICH>
__global__ __launch_bounds__(kBlock) void k_p2g_colour(WorkTab wt, int colour) {
    using G = Geo<DIM, SHAPE>;
    using R = typename PrecT<PREC>::real;
    constexpr int W = G::W;
    constexpr int NQ = WHICH == 0 ? 1 + 2 * DIM : DIM;
    const int pi = find_prob(wt, blockIdx.x);
    const ProbDev *P = wt.prob[pi];
    if (!P->active) return;
    const int col[3] = {colour % W, (colour / W) % W, DIM == 3 ? colour / (W * W) : 0};
    int m[3] = {1, 1, 1};
#pragma unroll
    for (int a = 0; a < DIM; ++a) m[a] = P->n[a] > col[a] ? (P->n[a] - col[a] + W - 1) / W : 0;
    const long long g = (long long)(blockIdx.x - wt.start[pi]) * kBlock + threadIdx.x;
    if (g >= (long long)m[0] * m[1] * m[2]) return;
    const int cell[3] = {col[0] + W * (int)(g % m[0]), col[1] + W * (int)((g / m[0]) % m[1]),
                         DIM == 3 ? col[2] + W * (int)(g / ((long long)m[0] * m[1])) : 0};
    const View V = make_view(P);
    const int par = P->parity;
    const GLOBAL_AS uint32_t *off = gmem((const uint32_t *)P->offs[par]);
    const uint32_t key = cell_key<DIM>(P, cell);
    const uint32_t beg = off[key], end = off[key + 1];
    if (end == beg) return;
    const GLOBAL_AS uint32_t *ids = gmem((const uint32_t *)P->pid[par]);
    GLOBAL_AS double *grid = gmem((double *)(WHICH == 0 ? P->gA[par] : P->gB[par]));
    const long long NN = P->nnodes;
    uint32_t flags = 0;
    // The order by id: for a cell of at most KMAX particles the ids are held
    // in registers and ranked there; a fuller cell is scanned in global
    // memory for each next id.
    constexpr int KMAX = 16;
    const uint32_t n = end - beg;
    uint32_t idr[KMAX], rk[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) idr[j] = (uint32_t)j < n ? ids[beg + j] : 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        uint32_t r = 0;
#pragma unroll
        for (int i = 0; i < KMAX; ++i) r += idr[i] < idr[j] ? 1u : 0u;
        rk[j] = r;
    }
    // 2D, the P2G of M V': the cell's W x W conditioned nodes, staged once
    // (dt f / m), summed as the gather sweeps sum them
    R dvn[DIM == 2 && WHICH == 1 ? G::WP : 1][DIM];
    if constexpr (DIM == 2 && WHICH == 1) {
#pragma unroll
        for (int jy = 0; jy < W; ++jy)
#pragma unroll
            for (int jx = 0; jx < W; ++jx) {
                R vs[3], dv[3];
                stage_A<DIM, PREC>(P, node_index(P, cell[0] + jx, cell[1] + jy, 0), vs, dv, flags);
#pragma unroll
                for (int a = 0; a < DIM; ++a) dvn[jy * W + jx][a] = dv[a];
            }
    }
#pragma unroll 1
    for (int pass = 0; pass < G::PASSES; ++pass) {
        double acc[G::WP][NQ];
#pragma unroll
        for (int s = 0; s < G::WP; ++s)
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[s][q] = 0.0;
        uint32_t prev = 0;
#pragma unroll 1
        for (uint32_t r = 0; r < n; ++r) {
            uint32_t k = beg;
            if (n <= (uint32_t)KMAX) {
#pragma unroll
                for (int j = 0; j < KMAX; ++j) k += rk[j] == r ? (uint32_t)j : 0u;
            } else {
                uint32_t best = 0xFFFFFFFFu;
                for (uint32_t j = beg; j < end; ++j) {
                    const uint32_t id = ids[j];
                    if ((r == 0 || id > prev) && id <= best) { best = id; k = j; }
                }
                prev = best;
            }
            R x[3] = {0, 0, 0};
#pragma unroll
            for (int a = 0; a < DIM; ++a) x[a] = gmem((const R *)P->part[par][PF_X + a])[k];
            Stencil<DIM, SHAPE, R> st;
            make_stencil<DIM, SHAPE, R>(&V, x, st);
            if (st.c[0] != cell[0] || st.c[1] != cell[1] || (DIM == 3 && st.c[2] != cell[2])) {
                // a particle outside the cell it was sorted into would add to
                // another thread's nodes: refused (the sort and the stencil
                // compute the cell by the same expression, so never seen)
                flags |= ERR_INTERNAL;
                continue;
            }
            const R wz = DIM == 3 ? pick<W, R>(st.w[2], pass) : (R)1;
            if constexpr (WHICH == 0) {
                S1Factors<DIM, SHAPE, R> f;
                s1_factors<DIM, SHAPE, PREC>(&V, s1_load_global<DIM, R>(P, par, k), st, f);
                const R dwz = DIM == 3 ? pick<W, R>(st.dw[2], pass) : (R)0;
#pragma unroll
                for (int jy = 0; jy < W; ++jy) {
                    const R wyz = DIM == 3 ? st.w[1][jy] * wz : st.w[1][jy];
                    const R dyz = DIM == 3 ? st.dw[1][jy] * wz : st.dw[1][jy];
                    const R ydz = st.w[1][jy] * dwz;
#pragma unroll
                    for (int jx = 0; jx < W; ++jx) {
                        double *ac = acc[jy * W + jx];
                        ac[0] += f.mx[jx] * wyz;
#pragma unroll
                        for (int a = 0; a < DIM; ++a) ac[1 + a] += f.px[a][jx] * wyz;
                        ac[1 + DIM] += f.fx[jx] * wyz;
                        ac[2 + DIM] += f.gx[jx] * dyz;
                        if constexpr (DIM == 3) ac[3 + DIM] += f.gx[jx] * ydz;
                    }
                }
            } else {
                R dv[3] = {0, 0, 0}, v[3] = {0, 0, 0};
                if constexpr (DIM == 2) {
                    // the G2P of dt f / m row by row, as g2p_field
#pragma unroll
                    for (int jy = 0; jy < W; ++jy) {
                        R row[3] = {0, 0, 0};
#pragma unroll
                        for (int jx = 0; jx < W; ++jx)
#pragma unroll
                            for (int a = 0; a < DIM; ++a) row[a] += st.w[0][jx] * dvn[jy * W + jx][a];
                        const R wyz = st.w[1][jy];
#pragma unroll
                        for (int a = 0; a < DIM; ++a) dv[a] += wyz * row[a];
                    }
                } else {
                    R vbar[3], Gd[9];
                    g2p_global<DIM, SHAPE, PREC, false>(P, st, vbar, dv, Gd, flags);
                }
                const R M = gmem((const R *)P->part[par][PF_M])[k];
#pragma unroll
                for (int a = 0; a < DIM; ++a) v[a] = gmem((const R *)P->part[par][PF_V + a])[k] + dv[a];
#pragma unroll
                for (int jy = 0; jy < W; ++jy) {
                    const R wyz = DIM == 3 ? st.w[1][jy] * wz : st.w[1][jy];
#pragma unroll
                    for (int jx = 0; jx < W; ++jx)
#pragma unroll
                        for (int a = 0; a < DIM; ++a) acc[jy * W + jx][a] += ((M * v[a]) * st.w[0][jx]) * wyz;
                }
            }
        }
#pragma unroll
        for (int jy = 0; jy < W; ++jy)
#pragma unroll
            for (int jx = 0; jx < W; ++jx) {
                const long long node = node_index(P, cell[0] + jx, cell[1] + jy, DIM == 3 ? cell[2] + pass : 0);
#pragma unroll
                for (int q = 0; q < NQ; ++q) grid[q * NN + node] += acc[jy * W + jx][q];
            }
    }
    if (flags & ERR_INTERNAL) atomicOr((uint32_t *)&P->err, ERR_INTERNAL);
}

// Wave-level reductions over the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Block reduction of the PT_N partials (entries 0-1 max, the rest sums);
// the result is valid in thread 0.  red: PT_N * (blockDim / 64) doubles.
__device__ __forceinline__ void block_reduce_partials(double part[PT_N], double *red) {
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < PT_N; ++q) part[q] = q < 2 ? wave_max(part[q]) : wave_sum(part[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < PT_N; ++q) red[q * nw + w] = part[q];
    __syncthreads();
    if (w == 0) {
        // the wave totals, reduced across the lanes of wave 0 (maxima are
        // >= 0, so 0 is the identity of both operations here)
#pragma unroll
        for (int q = 0; q < PT_N; ++q) {
            const double r = lane < nw ? red[q * nw + lane] : 0.0;
            part[q] = q < 2 ? wave_max(r) : wave_sum(r);
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ scan --
// Exclusive prefix of the cell histogram into offs[parity ^ 1].
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
    // Inclusive scans within the four waves, then the wave totals in LDS.
    constexpr int NW = kBlock / 64;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint32_t t = sh[i];
        base += i < w ? t : 0u;
        tot += t;
    }
    total = tot;
    __syncthreads();
    return base + incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_a(WorkTab wt) {
    __shared__ uint32_t sh[kBlock];
    const int pi = find_prob(wt, blockIdx.x);
    ProbDev *P = wt.prob[pi];
    if (!P->active) return;
    const int ch = blockIdx.x - wt.start[pi];
    const long long base = (long long)ch * kScanChunk + (long long)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const long long c = base + i;
        if (c < P->ncells_pad) s += P->count[c];
    }
    uint32_t total;
    block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0) P->blocksum[ch] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_b(WorkTab wt) {
    __shared__ uint32_t sh[kBlock];
    const int pi = find_prob(wt, blockIdx.x);
    ProbDev *P = wt.prob[pi];
    if (!P->active) return;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < P->nchunks; b0 += kBlock) {
        const int i = b0 + threadIdx.x;
        const uint32_t v = i < P->nchunks ? P->blocksum[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, sh, total);
        if (i < P->nchunks) P->blocksum[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_c(WorkTab wt) {
    __shared__ uint32_t sh[kBlock];
    const int pi = find_prob(wt, blockIdx.x);
    ProbDev *P = wt.prob[pi];
    if (!P->active) return;
    const int ch = blockIdx.x - wt.start[pi];
    uint32_t *out = P->offs[P->parity ^ 1];
    const long long base = (long long)ch * kScanChunk + (long long)threadIdx.x * kScanItems;
    uint32_t vals[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const long long c = base + i;
        vals[i] = c < P->ncells_pad ? P->count[c] : 0u;
        s += vals[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sh, total) + P->blocksum[ch];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const long long c = base + i;
        if (c < P->ncells_pad) out[c] = run;
        run += vals[i];
    }
    if (ch == P->nchunks - 1 && threadIdx.x == 0) out[P->ncells_pad] = (uint32_t)P->np;
}

// One workgroup per problem: exclusive prefix of the per-tile totals of the
// next order (each thread scans a run of consecutive tiles; wave scans of
// the run totals, then one scan of the wave totals).
__global__ __launch_bounds__(1024) void k_tilescan(WorkTab wt) {
    __shared__ uint32_t wtot[16];
    ProbDev *P = wt.prob[blockIdx.x];
    if (!P->active) return;
    const int n = P->ntiles;
    const int per = (n + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    uint32_t run = 0;
    for (int i = 0; i < per; ++i)
        if (b0 + i < n) run += P->ttot[b0 + i];
    const uint32_t incl = wave_incl_scan(run);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    uint32_t wbase = 0;
    for (int i = 0; i < w; ++i) wbase += wtot[i];
    uint32_t ex = wbase + incl - run;
    for (int i = 0; i < per; ++i)
        if (b0 + i < n) {
            P->tbase[b0 + i] = ex;
            ex += P->ttot[b0 + i];
        }
    if (threadIdx.x == 1023) P->tbase[n] = wbase + incl;
}

// The frame nodes that tile t reduces (it is the first tile holding them on
// both axes): the sum of the halo records of the tiles holding each node,
// stored into the grid in the state precision (MASS0: value 0 is a mass).
template <int SHAPE, int PREC, int NQ, bool MASS0>
__device__ __forceinline__ void reduce_frame(ProbDev *P, int t, GLOBAL_AS typename PrecT<PREC>::real *grid,
                                             const GLOBAL_AS typename PrecT<PREC>::acc *halo) {
    using A = typename PrecT<PREC>::acc;
    using F = Frame2<SHAPE>;
    const int tx = t % P->ntile[0], ty = t / P->ntile[0];
    for (int sl = threadIdx.x; sl < F::NFR; sl += blockDim.x) {
        int lx, ly;
        frame_pos<SHAPE>(sl, lx, ly);
        const int gx = tx * F::T + lx, gy = ty * F::T + ly;
        if (gx >= P->nn[0] || gy >= P->nn[1]) continue;
        if (min(gx / F::T, P->ntile[0] - 1) != tx || min(gy / F::T, P->ntile[1] - 1) != ty) continue;
        const long long node = node_index(P, gx, gy, 0);
        A raw[NQ];
        gather_frame<SHAPE, NQ, A>(P, halo, gx, gy, raw);
        uint32_t flags = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            grid[q * P->nnodes + node] = from_acc<PREC>(raw[q], MASS0 && q == 0 ? P->q_m : P->q_p, flags);
        if (flags) atomicOr((uint32_t *)&P->err, flags);
    }
}

// Per tile: offsets of the next order, tile base + prefix of the tile's
// cell counts (written into offs[parity ^ 1]).  The tile base comes from the
// tile scan, or, when every problem of the launch has at most kFuseTiles
// tiles, is summed here from the earlier tiles' totals.  2D: also the p2
// frame nodes this tile reduces, summed from the halo records of S2 into
// the grid for the update sweep and the read-back.
template <int DIM, int SHAPE, int PREC>
__global__ __launch_bounds__(kBlock) void k_cellscan(WorkTab wt) {
    __shared__ uint32_t sh[kBlock];
    const int pi = find_prob(wt, blockIdx.x);
    ProbDev *P = wt.prob[pi];
    if (!P->active) return;
    const int t = xcd_tile<kXcdGroup<DIM, PREC>>(blockIdx.x - wt.start[pi], P->ntiles);
    uint32_t *out = P->offs[P->parity ^ 1];
    const uint32_t c = (uint32_t)t * kBlock + threadIdx.x;
    const bool fused = wt.max_tiles <= kFuseTiles;
    __shared__ uint32_t wsum[kBlock / 64];
    if (fused) {
        // this thread's share of the earlier tiles' totals, summed per wave;
        // the scan's barrier below publishes the wave sums
        const GLOBAL_AS uint32_t *tt = gmem((const uint32_t *)P->ttot);
        uint32_t run = 0;
        for (int i = threadIdx.x; i < t; i += kBlock) run += tt[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) run += __shfl_xor(run, o, 64);
        if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = run;
    }
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(P->count[c], sh, total);
    uint32_t base;
    if (fused) {
        base = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) base += wsum[w];
    } else {
        base = P->tbase[t];
    }
    out[c] = base + ex;
    if (t == P->ntiles - 1 && threadIdx.x == 0) out[P->ncells_pad] = base + total;
    if constexpr (kHalo<DIM> && !PrecT<PREC>::colour) {
        using R = typename PrecT<PREC>::real;
        using A = typename PrecT<PREC>::acc;
        reduce_frame<SHAPE, PREC, DIM, false>(P, t, gmem((R *)P->gB[P->parity]), gmem((const A *)P->haloB));
    }
}

// 2D, right after S1: the frame nodes of the grid, summed from the halo
// records of S1 by their reducer tiles (one thread per frame position).
template <int DIM, int SHAPE, int PREC>
__global__ __launch_bounds__(kBlock) void k_frame_reduce(WorkTab wt) {
    if constexpr (kHalo<DIM>) {
        using R = typename PrecT<PREC>::real;
        using A = typename PrecT<PREC>::acc;
        const int pi = find_prob(wt, blockIdx.x);
        ProbDev *P = wt.prob[pi];
        if (!P->active) return;
        const int t = xcd_tile<kXcdGroup<DIM, PREC>>(blockIdx.x - wt.start[pi], P->ntiles);
        reduce_frame<SHAPE, PREC, 1 + 2 * DIM, true>(P, t, gmem((R *)P->gA[P->parity]), gmem((const A *)P->haloA));
    }
}

// -------------------------------------------------------------- finalize --
// Next time step from the per-tile maxima of the step just done (Sec. 2.2,
// CFL; Sec. 3 (xiii)-(xiv)) and the time.  Thread 0 of one
// workgroup per problem holds the reduced partials.
// Time-stepping state of a problem, read in one batch of loads.
struct StepState {
    double dt, t, cfl, h, t_end;
    long long step, steps_left;
    int parity;
    uint32_t err;
};

__device__ __forceinline__ StepState read_step_state(const ProbDev *P) {
    StepState s;
    s.dt = P->dt;
    s.t = P->t;
    s.cfl = P->cfl;
    s.h = P->h;
    s.t_end = P->t_end;
    s.step = P->step;
    s.steps_left = P->steps_left;
    s.parity = P->parity;
    s.err = P->err;
    return s;
}

// The next time step from the CFL maxima part[0..1]; with `sums`, also the
// conserved sums part[2..7].
__device__ void finalize_problem(ProbDev *P, StepState s, bool advance, const double part[PT_N], bool sums) {
    const double vmax = sqrt(part[0]);
    const double cmax = sqrt(part[1]);
    if (advance) {
        // the update sweep wrote the whole G if this step ends the run
        if (s.steps_left <= 1 || (s.t_end > 0.0 && !(s.t + s.dt < s.t_end))) P->g_step = s.step + 1;
        P->dt_last = s.dt;
        s.t = s.t + s.dt;
        P->t = s.t;
        P->step = s.step + 1;
        s.steps_left -= 1;
        P->steps_left = s.steps_left;
        P->parity = s.parity ^ 1;
    }
    double dtn = (vmax + cmax > 0.0) ? s.cfl * s.h / (vmax + cmax) : 0.0;
    if (s.t_end > 0.0) {
        const double rest = s.t_end - s.t;
        if (rest < dtn) dtn = rest;
        if (dtn < 0.0) dtn = 0.0;
    }
    P->dt = dtn;
    if (sums)
        for (int c = 0; c < 6; ++c) P->cons[c] = part[2 + c];
    P->active = (s.steps_left > 0 && s.err == 0 && dtn > 0.0 &&
                 (s.t_end <= 0.0 || s.t < s.t_end)) ? 1 : 0;
}

// Reduction of the per-tile partials q0 .. q1-1 of one problem by one
// workgroup (the others stay 0).
template <int Q0 = 0, int Q1 = PT_N>
__device__ __forceinline__ void reduce_tile_partials(const GLOBAL_AS double *partials, int ntiles, double part[PT_N],
                                                     double *red) {
#pragma unroll
    for (int q = 0; q < PT_N; ++q) part[q] = 0.0;
#pragma unroll 2
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
#pragma unroll
        for (int q = Q0; q < Q1; ++q) {
            const double v = partials[(long long)q * ntiles + t];
            part[q] = q < 2 ? fmax(part[q], v) : part[q] + v;
        }
    block_reduce_partials(part, red);
}

constexpr int kWideBlock = 1024;

__global__ __launch_bounds__(kWideBlock) void k_finalize(WorkTab wt) {
    __shared__ double red[PT_N * (kWideBlock / 64)];
    ProbDev *P = wt.prob[blockIdx.x];
    // every descriptor read in one batch, before the first store
    const int active = P->active, ntiles = P->ntiles;
    const GLOBAL_AS double *partials = gmem((const double *)P->partials);
    const StepState st = read_step_state(P);
    if (!active) return;
    // only the CFL maxima: the conserved sums are reduced when they are read
    double part[PT_N];
    reduce_tile_partials<0, 2>(partials, ntiles, part, red);
    if (threadIdx.x == 0) finalize_problem(P, st, true, part, false);
}

// The FP64 conserved sums of the last step (or of the initial state), from
// the per-tile partials it left; launched when the sums are read.
__global__ __launch_bounds__(kWideBlock) void k_conserved(ProbDev *P) {
    __shared__ double red[PT_N * (kWideBlock / 64)];
    double part[PT_N];
    reduce_tile_partials<2, PT_N>(gmem((const double *)P->partials), P->ntiles, part, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 6; ++c) P->cons[c] = part[2 + c];
}

// -------------------------------------------------------------------- S3 --
// Running per-tile results of S3.
struct S3Sums {
    double vmax2, cmax2, M, MV[3], ME, MK;
    unsigned long long mis, rec, wall;
};

// The S3 inputs of one particle, all read at its index in the current order.
template <typename R> struct S3In {
    R x[3], v[3], M, rho, e, Dprev;
    uint32_t id, rk;
};

// Particle fields of S3, source (this step's parity) and destination (the
// next): stored field f of a parity lies field_slot(DIM, f) strides of fs
// bytes past its first stored field f0.  Twenty-odd field pointers held
// across the particle loop spill from the scalar registers and are reloaded
// for every particle; a base and a stride are four registers, and the
// addresses are formed at each load and store instead (empty asm below).
template <int DIM, typename R> struct S3Src {
    const GLOBAL_AS char *f0;
    long long fs;
    const GLOBAL_AS uint32_t *id, *rank;
};

template <int DIM, typename R> struct S3Dst {
    GLOBAL_AS char *f0;
    long long fs;
    GLOBAL_AS uint32_t *id;
    const GLOBAL_AS uint32_t *noff;
    bool full_g;              // the last step of the run: write the whole G too
};

// Stored field F of a parity (first field f0, stride fs bytes).
template <int DIM, int F, typename R, typename C>
__device__ __forceinline__ auto field_ptr(C *f0, long long fs) {
    using T = typename std::conditional<std::is_const<C>::value, const R, R>::type;
    return (GLOBAL_AS T *)(f0 + field_slot(DIM, F) * fs);
}

template <int DIM, typename R>
__device__ __forceinline__ S3In<R> s3_load(const S3Src<DIM, R> &sp, uint32_t k) {
    // base and stride pass through an empty asm: the compiler cannot hoist
    // the field addresses out of the loop (where they would spill)
    const GLOBAL_AS char *f0 = sp.f0;
    long long fs = sp.fs;
    asm volatile("" : "+s"(f0), "+s"(fs));
    S3In<R> in;
#pragma unroll
    for (int a = 0; a < 3; ++a) { in.x[a] = 0; in.v[a] = 0; }
    in.Dprev = ldk(field_ptr<DIM, PF_D, R>(f0, fs), k);
    in.x[0] = ldk(field_ptr<DIM, PF_X + 0, R>(f0, fs), k);
    in.x[1] = ldk(field_ptr<DIM, PF_X + 1, R>(f0, fs), k);
    in.v[0] = ldk(field_ptr<DIM, PF_V + 0, R>(f0, fs), k);
    in.v[1] = ldk(field_ptr<DIM, PF_V + 1, R>(f0, fs), k);
    if constexpr (DIM == 3) {
        in.x[2] = ldk(field_ptr<DIM, PF_X + 2, R>(f0, fs), k);
        in.v[2] = ldk(field_ptr<DIM, PF_V + 2, R>(f0, fs), k);
    }
    in.M = ldk(field_ptr<DIM, PF_M, R>(f0, fs), k);
    in.rho = ldk(field_ptr<DIM, PF_RHO, R>(f0, fs), k);
    in.e = ldk(field_ptr<DIM, PF_E, R>(f0, fs), k);
    in.id = ldk(sp.id, k);
    in.rk = ldk(sp.rank, k);
    return in;
}

// The whole particle update of S3 for one particle whose old stencil is st:
// G2PD / G2P (from the staged footprint, or from the global grid when
// GLOBAL), energy and density update, move, recycling, scatter into the
// next sorted order, CFL maxima and FP64 sums.
template <int DIM, int SHAPE, int PREC, bool GLOBAL>
__device__ __forceinline__ void s3_particle(const ProbDev *P, const View *V, const S3Dst<DIM, typename PrecT<PREC>::real> &dst,
                                            const S3In<typename PrecT<PREC>::real> &in,
                                            const Stencil<DIM, SHAPE, typename PrecT<PREC>::real> &st,
                                            const int l0[3],
                                            const typename PrecT<PREC>::real *stage, const uint32_t *sfoot,
                                            S3Sums &sums, uint32_t &flags) {
    using G = Geo<DIM, SHAPE>;
    using R = typename PrecT<PREC>::real;
    constexpr int W = G::W;
    const R dt = (R)V->dt;
    const R gam = (R)V->gamma, h = (R)V->h, inv_h = (R)V->inv_h;

    R x[3] = {in.x[0], in.x[1], in.x[2]}, v[3] = {in.v[0], in.v[1], in.v[2]};
    R M = in.M;
    const R rho = in.rho, e = in.e, Dprev = in.Dprev;
    const uint32_t id = in.id, rk = in.rk;

    R Gm[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) Gm[c] = 0;
    R vbar[3] = {0, 0, 0};
    R dv[3] = {0, 0, 0};
    if constexpr (!GLOBAL) {
        constexpr int NF = stage_stride<DIM, true>();
        // G2PD of v2, summed row by row (z loop rolled: fewer live registers)
#pragma unroll 1
        for (int jz = 0; jz < (DIM == 3 ? W : 1); ++jz)
#pragma unroll
            for (int jy = 0; jy < W; ++jy) {
                R row2[3] = {0, 0, 0}, sx[3] = {0, 0, 0};
#pragma unroll
                for (int jx = 0; jx < W; ++jx) {
                    const R *nd = node_ptr<DIM, SHAPE, R, NF>(stage, l0, jx, jy, jz);
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        row2[a] += st.w[0][jx] * nd[2 * DIM + a];
                        sx[a] += st.dw[0][jx] * nd[2 * DIM + a];
                    }
                }
                const R wz = DIM == 3 ? pick<W, R>(st.w[2], jz) : (R)1;
                const R wyz = DIM == 3 ? st.w[1][jy] * wz : st.w[1][jy];
                const R dyz = DIM == 3 ? st.dw[1][jy] * wz : st.dw[1][jy];
                const R ydz = DIM == 3 ? st.w[1][jy] * pick<W, R>(st.dw[2], jz) : (R)0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    Gm[a * DIM + 0] += wyz * sx[a];
                    Gm[a * DIM + 1] += dyz * row2[a];
                    if (DIM == 3) Gm[a * DIM + 2] += ydz * row2[a];
                }
            }
#pragma unroll
        for (int c = 0; c < DIM * DIM; ++c) Gm[c] *= inv_h;
        g2p_field<DIM, SHAPE, R, NF, 0, true>(stage, st, l0, vbar);
        g2p_field<DIM, SHAPE, R, NF, DIM, true>(stage, st, l0, dv);
    } else {
        g2p_global<DIM, SHAPE, PREC, true>(P, st, vbar, dv, Gm, flags);
    }
    // FLIP velocity update V' = V + dt A, the same bits as in the G2P sweep
#pragma unroll
    for (int a = 0; a < DIM; ++a) v[a] = v[a] + dv[a];

    R D = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) D += Gm[a * DIM + a];
    const R p = eos_p(gam, rho, e);
    const R q = art_visc(V->av_form, (R)V->c0, (R)V->c1, gam, h, rho, p, Dprev);
    const R J = (R)1 + dt * D;
    if (!(J > (R)0)) flags |= ERR_NONPHYS;
    // Internal energy in FP64 registers: e' = e - dt (P+Q) D / rho.  1/rho:
    // from an FP32 state, the hardware reciprocal and one Newton step in
    // FP64 (relative error ~1e-14); from an FP64 state, a division.
    double irho;
    if constexpr (sizeof(R) == 4) {
        const double r0 = (double)recip(rho);
        irho = r0 * fma(-(double)rho, r0, 2.0);
    } else {
        irho = 1.0 / (double)rho;
    }
    const double en = (double)e - V->dt * ((double)p + (double)q) * (double)D * irho;
    R rhon = rho * recip(J);
    R En = (R)en;

    const int mv = advect<DIM, R>(V, x, vbar, dt, IdVal{id});
    if (mv == 1) {
        ++sums.rec;
#pragma unroll
        for (int a = 0; a < DIM; ++a) v[a] = (R)V->inflow_u[a];
        rhon = (R)V->inflow_rho;
        En = (R)V->inflow_e;
        M = (R)V->recycle_mass;
#pragma unroll
        for (int c = 0; c < 9; ++c) Gm[c] = 0;
    } else if (mv == 2) {
        ++sums.wall;
    }
    if (!isfinite((double)En) || !isfinite((double)rhon)) flags |= ERR_NONFINITE;

    // Slot in the next sorted order: the cell's offset plus the rank (the
    // offset plus this tile's base in the cell is staged per footprint cell).
    const uint32_t np = (uint32_t)V->np;
    uint32_t slot;
    if (rk & kRankGlobal) {
        int cn[3];
        cell_of<DIM, R>(V, x, cn);
        slot = dst.noff[cell_key<DIM>(V, cn)] + (rk & ~kRankGlobal);
    } else {
        const uint32_t dl = min((rk >> kRankShift) & 1023u, (uint32_t)DestFoot<DIM>::N - 1u);
        slot = sfoot[dl] + (rk & kRankMask);
    }
    if (slot >= np) {
        flags |= ERR_INTERNAL;
        return;
    }
    GLOBAL_AS char *f0 = dst.f0;
    long long fs = dst.fs;
    asm volatile("" : "+s"(f0), "+s"(fs));
    stk(field_ptr<DIM, PF_X + 0, R>(f0, fs), slot, x[0]);
    stk(field_ptr<DIM, PF_X + 1, R>(f0, fs), slot, x[1]);
    stk(field_ptr<DIM, PF_V + 0, R>(f0, fs), slot, v[0]);
    stk(field_ptr<DIM, PF_V + 1, R>(f0, fs), slot, v[1]);
    if constexpr (DIM == 3) {
        stk(field_ptr<DIM, PF_X + 2, R>(f0, fs), slot, x[2]);
        stk(field_ptr<DIM, PF_V + 2, R>(f0, fs), slot, v[2]);
    }
    stk(field_ptr<DIM, PF_M, R>(f0, fs), slot, M);
    stk(field_ptr<DIM, PF_RHO, R>(f0, fs), slot, rhon);
    stk(field_ptr<DIM, PF_E, R>(f0, fs), slot, En);
    // tr G of the stored gradient (zero for a recycled particle): the sum
    // the next step would form from the stored diagonal, the same bits
    stk(field_ptr<DIM, PF_D, R>(f0, fs), slot, mv == 1 ? (R)0 : D);
    if (dst.full_g) {
        stk(field_ptr<DIM, PF_G + 0, R>(f0, fs), slot, Gm[0]);
        stk(field_ptr<DIM, PF_G + 1, R>(f0, fs), slot, Gm[1]);
        stk(field_ptr<DIM, PF_G + 2, R>(f0, fs), slot, Gm[2]);
        stk(field_ptr<DIM, PF_G + 3, R>(f0, fs), slot, Gm[3]);
        if constexpr (DIM == 3) {
            stk(field_ptr<DIM, PF_G + 4, R>(f0, fs), slot, Gm[4]);
            stk(field_ptr<DIM, PF_G + 5, R>(f0, fs), slot, Gm[5]);
            stk(field_ptr<DIM, PF_G + 6, R>(f0, fs), slot, Gm[6]);
            stk(field_ptr<DIM, PF_G + 7, R>(f0, fs), slot, Gm[7]);
            stk(field_ptr<DIM, PF_G + 8, R>(f0, fs), slot, Gm[8]);
        }
    }
    stk(dst.id, slot, id);

    // CFL maxima (squared) and FP64 sums of the new state
    double v2 = 0, vb2 = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        v2 += (double)v[a] * (double)v[a];
        vb2 += (double)vbar[a] * (double)vbar[a];
        sums.MV[a] += (double)M * (double)v[a];
    }
    sums.vmax2 = fmax(sums.vmax2, fmax(v2, vb2));
    const R pn = eos_p(gam, rhon, En);
    sums.cmax2 = fmax(sums.cmax2, (double)(gam * pn * recip(rhon)));
    sums.M += (double)M;
    sums.ME += (double)M * (double)En;
    sums.MK += 0.5 * (double)M * v2;
}

// Workgroups per CU S3 is compiled for: 2D fixed point keeps four (at most
// 128 registers per lane).
template <int DIM, int PREC> constexpr int kUpdateBlocks = DIM == 2 && PREC == P_F32_FIX ? 4 : 1;

template <int DIM, int SHAPE, int PREC>
__global__ __launch_bounds__(kBlock, (kUpdateBlocks<DIM, PREC>)) void k_update(WorkTab wt) {
    using G = Geo<DIM, SHAPE>;
    using R = typename PrecT<PREC>::real;
    constexpr int NF = stage_stride<DIM, true>();
    constexpr int ND = DestFoot<DIM>::N;
    __shared__ R stage[NF * G::TN];
    __shared__ uint32_t sfoot[ND];
    __shared__ double red[PT_N * (kBlock / 64)];

    const int pi = find_prob(wt, blockIdx.x);
    ProbDev *P = wt.prob[pi];
    if (!P->active) return;
    const int t = xcd_tile<kXcdGroupS3>(blockIdx.x - wt.start[pi], P->ntiles);
    // Field pointers, read before any store of the kernel (uniform loads)
    S3Src<DIM, R> src;
    S3Dst<DIM, R> dst;
    {
        const int par0 = P->parity, np1 = par0 ^ 1;
        // stride between stored fields (X has at least two components)
        const long long fs = (const char *)P->part[par0][PF_X + 1] - (const char *)P->part[par0][PF_X];
        src.f0 = gmem((const char *)P->part[par0][PF_X]);
        src.fs = fs;
        src.id = gmem((const uint32_t *)P->pid[par0]);
        src.rank = gmem((const uint32_t *)P->rank);
        dst.f0 = gmem((char *)P->part[np1][PF_X]);
        dst.fs = fs;
        // the run ends with this step when it is its last counted step or
        // reaches t_end (the same test the time-step kernel makes)
        const double t_end = P->t_end;
        dst.full_g = P->steps_left <= 1 || (t_end > 0.0 && !(P->t + P->dt < t_end));
        dst.id = gmem((uint32_t *)P->pid[np1]);
        dst.noff = gmem((const uint32_t *)P->offs[np1]);
    }
    const View V = make_view(P);
    int c0[3], lc[3];
    tile_cell<DIM>(P, t, c0, lc);
    const bool interior = tile_interior<DIM, SHAPE>(V, c0);
    uint32_t flags = 0;
    stage_tile<DIM, SHAPE, PREC, true>(P, c0, stage, flags);
    // Per destination footprint cell: its offset in the next order plus
    // this tile's base among the cell's particles (only cells that receive
    // particles from this tile are read).
    {
        const GLOBAL_AS uint32_t *bt = gmem((const uint32_t *)P->basetab) + (long long)t * ND;
        const GLOBAL_AS uint32_t *noff = gmem((const uint32_t *)P->offs[P->parity ^ 1]);
        for (int i = threadIdx.x; i < ND; i += kBlock) {
            const int lx = i % (G::TX + 2), ly = (i / (G::TX + 2)) % (G::TY + 2), lz = i / ((G::TX + 2) * (G::TY + 2));
            const int cn[3] = {c0[0] + lx - 1, c0[1] + ly - 1, DIM == 3 ? c0[2] + lz - 1 : 0};
            const bool in_dom = cn[0] >= 0 && cn[0] < P->n[0] && cn[1] >= 0 && cn[1] < P->n[1] &&
                                (DIM == 2 || (cn[2] >= 0 && cn[2] < P->n[2]));
            sfoot[i] = in_dom ? noff[cell_key<DIM>(P, cn)] + bt[i] : 0u;
        }
    }
    __syncthreads();

    const int par = P->parity;
    const GLOBAL_AS uint32_t *off = gmem((const uint32_t *)P->offs[par]);
    const uint32_t pbeg = off[(uint32_t)t * G::CELLS], pend = off[(uint32_t)(t + 1) * G::CELLS];
    S3Sums sums = {0, 0, 0, {0, 0, 0}, 0, 0, 0, 0, 0};

    // (compiled once for interior tiles, uniform B2 pieces only, and once
    // for tiles at a domain face)
    auto sweep = [&](auto edge_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
        // 3D: the lane's next particle is loaded while this one is updated
        // (the index clamped to the tile's last particle).  2D S3, held at
        // 128 registers, would spill the extra inputs.
        constexpr bool AHEAD = DIM == 3;
        uint32_t k = pbeg + threadIdx.x;
        S3In<R> nxt{};
        if (AHEAD && pbeg < pend) nxt = s3_load<DIM, R>(src, min(k, pend - 1));
#pragma unroll 1
        for (; k < pend; k += kBlock) {
            S3In<R> in;                                      // every input in one round trip
            if constexpr (AHEAD) {
                in = nxt;
                nxt = s3_load<DIM, R>(src, min(k + kBlock, pend - 1));
            } else {
                in = s3_load<DIM, R>(src, k);
            }
            Stencil<DIM, SHAPE, R> st;
            make_stencil<DIM, SHAPE, R, EDGE>(&V, in.x, st);
            const int l0[3] = {st.c[0] - c0[0], st.c[1] - c0[1], DIM == 3 ? st.c[2] - c0[2] : 0};
            const bool inside = l0[0] >= 0 && l0[0] < G::TX && l0[1] >= 0 && l0[1] < G::TY &&
                                (DIM == 2 || (l0[2] >= 0 && l0[2] < G::TZ));
            if (!inside) { ++sums.mis; continue; }       // handled below (rare)
            s3_particle<DIM, SHAPE, PREC, false>(P, &V, dst, in, st, l0, stage, sfoot, sums, flags);
        }
    };
    if (interior) sweep(std::false_type{});
    else sweep(std::true_type{});
    if (sums.mis) {
#pragma unroll 1
        for (uint32_t k = pbeg + threadIdx.x; k < pend; k += kBlock) {
            const S3In<R> in = s3_load<DIM, R>(src, k);
            Stencil<DIM, SHAPE, R> st;
            make_stencil<DIM, SHAPE, R>(&V, in.x, st);
            const int l0[3] = {st.c[0] - c0[0], st.c[1] - c0[1], DIM == 3 ? st.c[2] - c0[2] : 0};
            const bool inside = l0[0] >= 0 && l0[0] < G::TX && l0[1] >= 0 && l0[1] < G::TY &&
                                (DIM == 2 || (l0[2] >= 0 && l0[2] < G::TZ));
            if (inside) continue;
            s3_particle<DIM, SHAPE, PREC, true>(P, &V, dst, in, st, l0, stage, sfoot, sums, flags);
        }
    }

    // Per-tile partials (one plain store each): squared CFL maxima and the
    // FP64 sums; the finalize kernel reduces them.
    double part[PT_N] = {sums.vmax2, sums.cmax2, sums.M, sums.MV[0], sums.MV[1], sums.MV[2], sums.ME, sums.MK};
    block_reduce_partials(part, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < PT_N; ++q) gmem(P->partials)[(long long)q * P->ntiles + t] = part[q];
    const uint32_t errs = flags & (ERR_NONPHYS | ERR_NONFINITE | ERR_OVERFLOW | ERR_INTERNAL);
    if (errs) atomicOr((uint32_t *)&P->err, errs);
    if (sums.mis) atomicAdd((unsigned long long *)&P->diag[DG_MISMATCH], sums.mis);
    if (sums.rec) atomicAdd((unsigned long long *)&P->diag[DG_RECYCLE], sums.rec);
    if (sums.wall) atomicAdd((unsigned long long *)&P->diag[DG_WALL], sums.wall);
}

// Arm problems for a run of steps: steps_left and the active flag.
struct ArmArgs { long long n[kMaxBatch]; };
__global__ void k_arm(WorkTab wt, ArmArgs aa) {
    const int i = threadIdx.x;
    if (i >= wt.n) return;
    ProbDev *P = wt.prob[i];
    P->steps_left = aa.n[i];
    P->active = (aa.n[i] > 0 && P->err == 0 && P->dt > 0.0 &&
                 (P->t_end <= 0.0 || P->t < P->t_end)) ? 1 : 0;
}

// ------------------------------------------------------------------ init --
// Key and rank of every particle of the unsorted input (held in parity 1).
template <int DIM, typename R>
__global__ __launch_bounds__(kBlock) void k_init_keys(ProbDev *P) {
    const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (k >= P->np) return;
    R x[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) x[a] = gmem((const R *)P->part[1][PF_X + a])[k];
    int c[3];
    cell_of<DIM, R>(P, x, c);
    const uint32_t nk = cell_key<DIM>(P, c);
    gmem(P->key)[k] = nk;
    P->rank[k] = atomicAdd(&P->count[nk], 1u);
}

// Scatter parity 1 -> parity 0 in key order.
template <int DIM, typename R>
__global__ __launch_bounds__(kBlock) void k_init_permute(ProbDev *P) {
    const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (k >= P->np) return;
    const uint32_t slot = P->offs[0][P->key[k]] + P->rank[k];
    if (slot >= (uint32_t)P->np) { atomicOr((uint32_t *)&P->err, ERR_INTERNAL); return; }
    for (int f = 0; f < PF_N; ++f) {
        if (!P->part[1][f] || f == PF_D) continue;
        gmem((R *)P->part[0][f])[slot] = gmem((const R *)P->part[1][f])[k];
    }
    // tr G, summed as the step sums it
    R D = 0;
    for (int a = 0; a < DIM; ++a) D += gmem((const R *)P->part[1][PF_G + a * DIM + a])[k];
    gmem((R *)P->part[0][PF_D])[slot] = D;
    P->pid[0][slot] = P->pid[1][k];
}

// Initial maxima and sums of the sorted state (parity 0).
template <int DIM, int SHAPE, typename R>
__global__ __launch_bounds__(kBlock) void k_init_stats(ProbDev *P) {
    using G = Geo<DIM, SHAPE>;
    __shared__ double red[PT_N * (kBlock / 64)];
    const int t = blockIdx.x;
    const uint32_t pbeg = P->offs[0][(uint32_t)t * G::CELLS], pend = P->offs[0][(uint32_t)(t + 1) * G::CELLS];
    double vmax = 0, cmax = 0, s[6] = {0, 0, 0, 0, 0, 0};
    const R gam = (R)P->gamma;
    for (uint32_t k = pbeg + threadIdx.x; k < pend; k += kBlock) {
        double v2 = 0;
        const R M = gmem((const R *)P->part[0][PF_M])[k];
        for (int a = 0; a < DIM; ++a) {
            const R va = gmem((const R *)P->part[0][PF_V + a])[k];
            v2 += (double)va * (double)va;
            s[1 + a] += (double)M * (double)va;
        }
        const R rho = gmem((const R *)P->part[0][PF_RHO])[k];
        const R e = gmem((const R *)P->part[0][PF_E])[k];
        vmax = fmax(vmax, sqrt(v2));
        cmax = fmax(cmax, (double)sound(gam, rho, eos_p(gam, rho, e)));
        s[0] += (double)M;
        s[4] += (double)M * (double)e;
        s[5] += 0.5 * (double)M * v2;
    }
    double part[PT_N] = {vmax * vmax, cmax * cmax, s[0], s[1], s[2], s[3], s[4], s[5]};
    block_reduce_partials(part, red);
    if (threadIdx.x == 0)
        for (int q = 0; q < PT_N; ++q) P->partials[(long long)q * P->ntiles + t] = part[q];
}

__global__ __launch_bounds__(kWideBlock) void k_init_finalize(ProbDev *P) {
    __shared__ double red[PT_N * (kWideBlock / 64)];
    double part[PT_N];
    reduce_tile_partials(gmem((const double *)P->partials), P->ntiles, part, red);
    if (threadIdx.x != 0) return;
    finalize_problem(P, read_step_state(P), false, part, true);
    P->active = 0;
    P->parity = 0;
}

// ------------------------------------------------------------ diagnostics --
// Grid snapshot as double (raw accumulators or after the conditions).
template <int DIM, int PREC>
__global__ __launch_bounds__(kBlock) void k_grid_diag(ProbDev *P, int which, double *out) {
    using R = typename PrecT<PREC>::real;
    using GW = typename GridW<DIM, PREC>::type;
    const long long node = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long NN = P->nnodes;
    if (node >= NN) return;
    const GW *gA = (const GW *)P->gA[P->parity ^ 1];
    const GW *gB = (const GW *)P->gB[P->parity ^ 1];
    // 2D grids hold scaled values already
    const bool scaled = PrecT<PREC>::fixed && DIM == 3;
    const double qm = scaled ? P->q_m : 1.0, qp = scaled ? P->q_p : 1.0;
    const double dtl = P->dt_last > 0 ? P->dt_last : 1.0;
    const uint8_t fl = P->nflag[node];
    const double m = (double)gA[node] * qm;
    double u[3] = {0, 0, 0};
    switch (which) {
    case 0: out[node] = m; return;
    case 6: out[node] = (double)fl; return;
    case 1: for (int a = 0; a < DIM; ++a) out[a * NN + node] = (double)gA[(1 + a) * NN + node] * qp; return;
    case 2: for (int a = 0; a < DIM; ++a) out[a * NN + node] = (double)gA[(1 + DIM + a) * NN + node] * qp / dtl; return;
    default: break;
    }
    // conditions applied in the state precision, as in the sweeps
    uint32_t flags = 0;
    R mr = grid_val<DIM, PREC>(gA[node], P->q_m, flags);
    R p[3] = {0, 0, 0}, I[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) {
        if (which == 4) p[a] = grid_val<DIM, PREC>(gB[a * NN + node], P->q_p, flags);
        else p[a] = grid_val<DIM, PREC>(gA[(1 + a) * NN + node], P->q_p, flags);
        I[a] = grid_val<DIM, PREC>(gA[(1 + DIM + a) * NN + node], P->q_p, flags);
    }
    if (fl) { node_bc<DIM, R>(P, fl, node, mr, p, false); node_bc<DIM, R>(P, fl, node, mr, I, true); }
    for (int a = 0; a < DIM; ++a) {
        if (which == 3) u[a] = (double)(p[a] + I[a]);
        else if (which == 4) u[a] = (double)p[a];
        else u[a] = (double)I[a] / dtl;
        out[a * NN + node] = u[a];
    }
}

// Read-out of the grid-projected density (not part of a step): P2G of the
// particle masses (which 0) or volumes M / rho (which 1) at the current
// positions, FP64 atomics into a zeroed node array.
__global__ __launch_bounds__(kBlock) void k_fill(double *out, long long n, double v) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = v;
}

template <int DIM, int SHAPE, int PREC>
__global__ __launch_bounds__(kBlock) void k_project(const ProbDev *P, int which, double *out) {
    using G = Geo<DIM, SHAPE>;
    using R = typename PrecT<PREC>::real;
    const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (k >= P->np) return;
    const int par = P->parity;
    R x[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) x[a] = ((const R *)P->part[par][PF_X + a])[k];
    const R M = ((const R *)P->part[par][PF_M])[k];
    const R rho = ((const R *)P->part[par][PF_RHO])[k];
    const double f = which == 0 ? (double)M : (double)M / (double)rho;
    Stencil<DIM, SHAPE, R> st;
    make_stencil<DIM, SHAPE, R>(P, x, st);
    for (int jz = 0; jz < (DIM == 3 ? G::W : 1); ++jz)
        for (int jy = 0; jy < G::W; ++jy)
            for (int jx = 0; jx < G::W; ++jx) {
                double w = (double)st.w[0][jx] * (double)st.w[1][jy];
                if (DIM == 3) w *= (double)st.w[2][jz];
                atomicAdd(&out[node_index(P, st.c[0] + jx, st.c[1] + jy, DIM == 3 ? st.c[2] + jz : 0)], f * w);
            }
}

// ------------------------------------------------------------- launchers --
// One sweep of the step (part 0..5 in launch order).
template <int DIM, int SHAPE, int PREC>
void launch_part_t(int part, const WorkTab &tiles, const WorkTab &single, hipStream_t s) {
    const dim3 grid(tiles.start[tiles.n]);
    // colouring precision: colour passes of at most one thread per cell, over
    // the tile grid of workgroups (more than the cells of one colour need)
    constexpr int kColours = Geo<DIM, SHAPE>::W * Geo<DIM, SHAPE>::W * (DIM == 3 ? Geo<DIM, SHAPE>::W : 1);
    switch (part) {
    case 0:
        if constexpr (PrecT<PREC>::colour) {
            hipLaunchKernelGGL((k_zero_grid<DIM>), grid, dim3(kBlock), 0, s, tiles);
            for (int c = 0; c < kColours; ++c)
                hipLaunchKernelGGL((k_p2g_colour<DIM, SHAPE, PREC, 0>), grid, dim3(kBlock), 0, s, tiles, c);
        } else {
            hipLaunchKernelGGL((k_p2g<DIM, SHAPE, PREC>), grid, dim3(kBlock), 0, s, tiles);
        }
        break;
    case 1:
        if (kHalo<DIM> && !PrecT<PREC>::colour)
            hipLaunchKernelGGL((k_frame_reduce<DIM, SHAPE, PREC>), grid, dim3(Frame2<SHAPE>::NFR), 0, s, tiles);
        break;
    case 2:
        hipLaunchKernelGGL((k_g2p<DIM, SHAPE, PREC>), grid, dim3(kBlock), 0, s, tiles);
        if constexpr (PrecT<PREC>::colour)
            for (int c = 0; c < kColours; ++c)
                hipLaunchKernelGGL((k_p2g_colour<DIM, SHAPE, PREC, 1>), grid, dim3(kBlock), 0, s, tiles, c);
        break;
    case 3:
        if (tiles.max_tiles > kFuseTiles) hipLaunchKernelGGL(k_tilescan, dim3(single.n), dim3(1024), 0, s, single);
        break;
    case 4: hipLaunchKernelGGL((k_cellscan<DIM, SHAPE, PREC>), grid, dim3(kBlock), 0, s, tiles); break;
    case 5: hipLaunchKernelGGL((k_update<DIM, SHAPE, PREC>), grid, dim3(kBlock), 0, s, tiles); break;
    default: hipLaunchKernelGGL(k_finalize, dim3(single.n), dim3(kWideBlock), 0, s, single); break;
    }
}

template <int DIM, int SHAPE, int PREC>
void launch_step_t(const WorkTab &tiles, const WorkTab &single, hipStream_t s) {
    for (int part = 0; part < kSweeps; ++part) launch_part_t<DIM, SHAPE, PREC>(part, tiles, single, s);
}

template <int DIM, int SHAPE, int PREC>
void launch_init_t(ProbDev *dP, const ProbDev &h, hipStream_t s) {
    using R = typename PrecT<PREC>::real;
    WorkTab one{};
    one.prob[0] = dP; one.start[0] = 0; one.start[1] = 1; one.n = 1;
    const unsigned nb = (unsigned)((h.np + kBlock - 1) / kBlock);
    if (nb) hipLaunchKernelGGL((k_init_keys<DIM, R>), dim3(nb), dim3(kBlock), 0, s, dP);
    WorkTab ch{};
    ch.prob[0] = dP; ch.start[0] = 0; ch.start[1] = h.nchunks; ch.n = 1;
    // the scan writes offs[parity ^ 1] = offs[0] while parity is 1 and active is 1
    hipLaunchKernelGGL(k_scan_a, dim3(h.nchunks), dim3(kBlock), 0, s, ch);
    hipLaunchKernelGGL(k_scan_b, dim3(1), dim3(kBlock), 0, s, one);
    hipLaunchKernelGGL(k_scan_c, dim3(h.nchunks), dim3(kBlock), 0, s, ch);
    if (nb) hipLaunchKernelGGL((k_init_permute<DIM, R>), dim3(nb), dim3(kBlock), 0, s, dP);
    hipLaunchKernelGGL((k_init_stats<DIM, SHAPE, R>), dim3(h.ntiles), dim3(kBlock), 0, s, dP);
    hipLaunchKernelGGL(k_init_finalize, dim3(1), dim3(kWideBlock), 0, s, dP);
}

template <int DIM, int SHAPE, int PREC>
void launch_grid_diag_t(ProbDev *dP, const ProbDev &h, int which, double *out, hipStream_t s) {
    const unsigned nb = (unsigned)((h.nnodes + kBlock - 1) / kBlock);
    if (which < 7) {
        hipLaunchKernelGGL((k_grid_diag<DIM, PREC>), dim3(nb), dim3(kBlock), 0, s, dP, which, out);
        return;
    }
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(kBlock), 0, s, out, h.nnodes, 0.0);
    const unsigned npb = (unsigned)((h.np + kBlock - 1) / kBlock);
    if (npb) hipLaunchKernelGGL((k_project<DIM, SHAPE, PREC>), dim3(npb), dim3(kBlock), 0, s, dP, which - 7, out);
}

// Runtime dispatch over the instantiated variants.
#define MPM_DISPATCH(DIMV, SHAPEV, PRECV, CALL)                                   \
    do {                                                                          \
        if ((DIMV) == 2 && (SHAPEV) == S_B2) {                                    \
            switch (PRECV) {                                                      \
            case P_FP64: CALL(2, S_B2, P_FP64); break;                            \
            case P_F32_A64: CALL(2, S_B2, P_F32_A64); break;                      \
            case P_F32_A32: CALL(2, S_B2, P_F32_A32); break;                      \
            case P_FP64_COL: CALL(2, S_B2, P_FP64_COL); break;                  \
            default: CALL(2, S_B2, P_F32_FIX); break;                             \
            }                                                                     \
        } else if ((DIMV) == 3 && (SHAPEV) == S_B2) {                             \
            switch (PRECV) {                                                      \
            case P_FP64: CALL(3, S_B2, P_FP64); break;                            \
            case P_F32_A64: CALL(3, S_B2, P_F32_A64); break;                      \
            case P_F32_A32: CALL(3, S_B2, P_F32_A32); break;                      \
            case P_FP64_COL: CALL(3, S_B2, P_FP64_COL); break;                  \
            default: CALL(3, S_B2, P_F32_FIX); break;                             \
            }                                                                     \
        } else if ((DIMV) == 2) {                                                 \
            switch (PRECV) {                                                      \
            case P_FP64: CALL(2, S_Q1, P_FP64); break;                            \
            default: CALL(2, S_Q1, P_F32_FIX); break;                             \
            }                                                                     \
        } else {                                                                  \
            switch (PRECV) {                                                      \
            case P_FP64: CALL(3, S_Q1, P_FP64); break;                            \
            default: CALL(3, S_Q1, P_F32_FIX); break;                             \
            }                                                                     \
        }                                                                         \
    } while (0)

void launch_step(int dim, int shape, int prec, const WorkTab &tiles, const WorkTab &single, hipStream_t s) {
#define CALL_STEP(D, S, Pr) launch_step_t<D, S, Pr>(tiles, single, s)
    MPM_DISPATCH(dim, shape, prec, CALL_STEP);
#undef CALL_STEP
}

void launch_part(int dim, int shape, int prec, int part, const WorkTab &tiles, const WorkTab &single,
                 hipStream_t s) {
#define CALL_PART(D, S, Pr) launch_part_t<D, S, Pr>(part, tiles, single, s)
    MPM_DISPATCH(dim, shape, prec, CALL_PART);
#undef CALL_PART
}

void launch_init(int dim, int shape, int prec, ProbDev *dP, const ProbDev &h, hipStream_t s) {
#define CALL_INIT(D, S, Pr) launch_init_t<D, S, Pr>(dP, h, s)
    MPM_DISPATCH(dim, shape, prec, CALL_INIT);
#undef CALL_INIT
}

void launch_grid_diag(int dim, int shape, int prec, ProbDev *dP, const ProbDev &h, int which,
                      double *out, hipStream_t s) {
#define CALL_DIAG(D, S, Pr) launch_grid_diag_t<D, S, Pr>(dP, h, which, out, s)
    MPM_DISPATCH(dim, shape, prec, CALL_DIAG);
#undef CALL_DIAG
}

void launch_conserved(ProbDev *dP, hipStream_t s) {
    hipLaunchKernelGGL(k_conserved, dim3(1), dim3(kWideBlock), 0, s, dP);
}

void launch_arm(const WorkTab &single, const long long *n, hipStream_t s) {
    ArmArgs aa{};
    for (int i = 0; i < single.n; ++i) aa.n[i] = n[i];
    hipLaunchKernelGGL(k_arm, dim3(1), dim3(kMaxBatch), 0, s, single, aa);
}

}  // namespace mpm
