// Device-side building blocks of the MPM step for gfx950.
#pragma once

#include <type_traits>

#include "mpm_common.hpp"

namespace mpm {

// Pointers read from the problem descriptor are generic; re-typing them to
// the global address space lets the compiler use global (not flat) memory
// instructions, which do not share the LDS wait counter.
#define GLOBAL_AS __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GLOBAL_AS T *gmem(T *p) { return (GLOBAL_AS T *)p; }
template <typename T> __device__ __forceinline__ const GLOBAL_AS T *gmem(const T *p) { return (const GLOBAL_AS T *)p; }

template <int DIM, int SHAPE> struct Geo {
    static constexpr int W = SHAPE == S_B2 ? 3 : 2;          // nodes per axis in a stencil
    static constexpr int TX = Tile<DIM>::X, TY = Tile<DIM>::Y, TZ = Tile<DIM>::Z;
    static constexpr int NX = TX + W - 1, NY = TY + W - 1;   // tile footprint in nodes
    static constexpr int NZ = DIM == 3 ? TZ + W - 1 : 1;
    static constexpr int TN = NX * NY * NZ;
    static constexpr int WP = W * W;                          // stencil nodes per z-slab
    static constexpr int PASSES = DIM == 3 ? W : 1;           // z-slabs of the stencil
    static constexpr int CELLS = Tile<DIM>::CELLS;
};

// ------------------------------------------------------------------ basis --
// One axis of the basis at reduced coordinate s = (x - lo)/h.  Returns the
// cell c (first stencil node); w/dw are the values and d/ds derivatives of
// the W non-zero functions.
//
// Q1 (Sec. 2.2): phi_c = 1 - u, phi_{c+1} = u, u = s - c.
// B2: quadratic B-splines on the clamped knot vector of the cell faces
// (0,0,0,1,...,n-1,n,n,n).  In an interior cell the three functions are the
// uniform pieces (1-u)^2/2, 1/2 + u(1-u), u^2/2.  The knot multiplicity
// changes the pieces in the first cell, (1-u)^2, u(2 - 3u/2), u^2/2, and
// symmetrically in the last cell, so that only the first (last) function is
// non-zero on the domain face.  EDGE = false: the caller knows the cell is
// neither the first nor the last (an interior tile), and only the uniform
// pieces are evaluated.
template <int SHAPE, typename R, bool EDGE = true>
__device__ __forceinline__ int basis1(R s, int n, R w[3], R dw[3]) {
    int c = (int)floor(s);
    c = c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
    const R u = s - (R)c;
    const R v = (R)1 - u;
    if constexpr (SHAPE == S_Q1) {
        w[0] = v;  dw[0] = (R)-1;
        w[1] = u;  dw[1] = (R)1;
    } else if constexpr (!EDGE) {
        w[0] = (R)0.5 * v * v;   dw[0] = -v;
        w[1] = (R)0.5 + u * v;   dw[1] = (R)1 - (R)2 * u;
        w[2] = (R)0.5 * u * u;   dw[2] = u;
    } else {
        // interior pieces, then the first / last cell by selection (no branches)
        const bool first = c == 0, last = c == n - 1;
        const R hv2 = (R)0.5 * v * v, hu2 = (R)0.5 * u * u;
        w[0] = first ? v * v : hv2;
        dw[0] = first ? (R)-2 * v : -v;
        w[1] = first ? u * ((R)2 - (R)1.5 * u) : (last ? v * ((R)2 - (R)1.5 * v) : (R)0.5 + u * v);
        dw[1] = first ? (R)2 - (R)3 * u : (last ? (R)1 - (R)3 * u : (R)1 - (R)2 * u);
        w[2] = last ? u * u : hu2;
        dw[2] = last ? (R)2 * u : u;
    }
    return c;
}

// Loop-invariant parameters of a problem, read from the descriptor at kernel
// entry, before the kernel's first store, so that the reads are uniform
// (scalar) loads and the values stay in registers through loops that store
// to global memory.  Field names match the descriptor's: the helpers below
// take either.
struct View {
    int n[3], nn[3], ntile[3];
    int face[3][2];
    int av_form;
    long long nnodes, np, step;
    unsigned long long seed;
    double lo[3], hi[3], h, inv_h, dt, gamma, c0, c1;
    double q_m, q_p, inv_q_m, inv_q_p;
    double inflow_rho, inflow_e, inflow_u[3], recycle_mass;
};

__device__ __forceinline__ View make_view(const ProbDev *P) {
    View v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v.n[a] = P->n[a];
        v.nn[a] = P->nn[a];
        v.ntile[a] = P->ntile[a];
        v.face[a][0] = P->face[a][0];
        v.face[a][1] = P->face[a][1];
        v.lo[a] = P->lo[a];
        v.hi[a] = P->hi[a];
        v.inflow_u[a] = P->inflow_u[a];
    }
    v.av_form = P->av_form;
    v.nnodes = P->nnodes;
    v.np = P->np;
    v.step = P->step;
    v.seed = P->seed;
    v.h = P->h;
    v.inv_h = P->inv_h;
    v.dt = P->dt;
    v.gamma = P->gamma;
    v.c0 = P->c0;
    v.c1 = P->c1;
    v.q_m = P->q_m;
    v.q_p = P->q_p;
    v.inv_q_m = P->inv_q_m;
    v.inv_q_p = P->inv_q_p;
    v.inflow_rho = P->inflow_rho;
    v.inflow_e = P->inflow_e;
    v.recycle_mass = P->recycle_mass;
    return v;
}

// Particle stencil: per-axis cells, weights and derivatives.
template <int DIM, int SHAPE, typename R> struct Stencil {
    int c[3];
    R w[3][3], dw[3][3];
};

template <int DIM, int SHAPE, typename R, bool EDGE = true, class PP>
__device__ __forceinline__ void make_stencil(const PP *P, const R x[3], Stencil<DIM, SHAPE, R> &st) {
    const R inv_h = (R)P->inv_h;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const R s = (x[a] - (R)P->lo[a]) * inv_h;
        st.c[a] = basis1<SHAPE, R, EDGE>(s, P->n[a], st.w[a], st.dw[a]);
    }
    if constexpr (DIM == 2) st.c[2] = 0;
}

// ---------------------------------------------------------- constitutive --
// 1/x for x > 0: in FP32 the hardware reciprocal (within 1 ulp; the state
// is FP32, so a correctly rounded quotient buys nothing), in FP64 a
// division.
template <typename R> __device__ __forceinline__ R recip(R x) {
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(x);
    else return (R)1 / x;
}

template <typename R> __device__ __forceinline__ R eos_p(R gamma, R rho, R e) {
    return (gamma - (R)1) * rho * e;                 // perfect gas (Sec. 2.1)
}
// Sound speed sqrt(max(gamma P / rho, 0)): in FP32 the hardware square
// root (within 1 ulp; it feeds only the artificial viscosity, whose FP32
// inputs carry that much already), in FP64 the correctly rounded one.
template <typename R> __device__ __forceinline__ R sound(R gamma, R rho, R p) {
    const R c2 = gamma * p * recip(rho);
    if constexpr (sizeof(R) == 4) return c2 > (R)0 ? __builtin_amdgcn_sqrtf(c2) : (R)0;
    else return c2 > (R)0 ? sqrt(c2) : (R)0;
}
// Artificial pressure (Sec. 2.1, eq. muart), only for div v < 0.
template <typename R>
__device__ __forceinline__ R art_visc(int form, R c0, R c1, R gamma, R h, R rho, R p, R D) {
    if (!(D < (R)0)) return (R)0;
    const R c = sound(gamma, rho, p);
    if (form == 1) return c0 * rho * (h * D) * (h * D) - c1 * rho * h * c * D;
    const R r = rho * h * D;
    return c0 * r * r - c1 * h * c * D;
}

// -------------------------------------------------------- fixed point --
// Contributions are scaled to quanta and, in the fixed-point precision,
// rounded to whole quanta before any addition, so every partial sum is an
// integer and exact in FP64.
//
// A contribution is the product a*b of two FP32 factors (e.g. M w_x and
// w_y).  A per-lane partial sum holds B + S, with S the integer sum in quanta
// and B = 1.5 * 2^52, and a contribution is added by one FP64 FMA,
// fma(a, b', B + S), where b' is b in FP64 with the lowest bit of its
// significand set (fix_weight).  Why that is exact and order-free:
//   a = A 2^alpha with A < 2^24 an integer (FP32), b' = Bo 2^beta with Bo an
//   odd 53-bit integer, so the lowest set bit of a b' = A Bo 2^(alpha+beta)
//   is 2^(alpha+beta+tz(A)) <= |a b'| / 2^52, below 1/2 while |a b'| < 2^51.
//   a b' is then never an odd multiple of 1/2, B + S + a b' (in [2^52, 2^53),
//   where the doubles are exactly the integers) is never halfway between two
//   of them, and round-to-nearest yields B + S + round(a b') for every
//   integer S.
// b' exceeds |b| by at most one FP64 ulp (2^-52 relative), less than the
// spacing of the exact FP32 products, so round(a b') is round(a b) with
// exact halves rounded away from zero: symmetric under a -> -a, as the
// mirror symmetries of a problem need.  (Without the odd bit one FMA would
// round an exact half by the parity of S, i.e. by the order of the
// additions.)  |S| stays below 2^51.
constexpr double kFixBias = 6755399441055744.0;     // 1.5 * 2^52

__device__ __forceinline__ double fix_weight(float b) {
    return __longlong_as_double(__double_as_longlong((double)b) | 1LL);
}

// Start value of a partial sum, and the sum it holds.
template <int PREC> __device__ __forceinline__ typename PrecT<PREC>::lacc acc_zero() {
    return PrecT<PREC>::fixed ? (typename PrecT<PREC>::lacc)kFixBias : (typename PrecT<PREC>::lacc)0;
}
template <int PREC>
__device__ __forceinline__ typename PrecT<PREC>::lacc unbias(typename PrecT<PREC>::lacc s) {
    if constexpr (PrecT<PREC>::fixed) return s - kFixBias;
    else return s;
}

// Weight factor of the contributions (fixed point: b' above).
template <int PREC> struct WeightT {
    using type = typename std::conditional<PrecT<PREC>::fixed, double, typename PrecT<PREC>::real>::type;
};
template <int PREC>
__device__ __forceinline__ typename WeightT<PREC>::type weight(typename PrecT<PREC>::real b) {
    if constexpr (PrecT<PREC>::fixed) return fix_weight(b);
    else return b;
}

// Partial sum s plus the contribution a*b (b from weight()).
template <int PREC>
__device__ __forceinline__ typename PrecT<PREC>::lacc accum(typename PrecT<PREC>::lacc s, typename PrecT<PREC>::real a,
                                                            typename WeightT<PREC>::type b) {
    if constexpr (PrecT<PREC>::fixed) return fma((double)a, b, s);
    else return s + (typename PrecT<PREC>::lacc)(a * b);
}

// One contribution on its own: the same integer as the accumulated form.
template <int PREC>
__device__ __forceinline__ typename PrecT<PREC>::lacc term_exact(typename PrecT<PREC>::real a,
                                                                 typename PrecT<PREC>::real b) {
    if constexpr (PrecT<PREC>::fixed) return fma((double)a, fix_weight(b), kFixBias) - kFixBias;
    else return (typename PrecT<PREC>::lacc)(a * b);
}

// Partial sum -> global accumulator word.  Fixed point: the integer-valued
// double becomes an int64; beyond 2^50 quanta the overflow bit is raised
// (node sums stay near 2^32 quanta per cell mass).
template <int PREC>
__device__ __forceinline__ typename PrecT<PREC>::acc lacc_to_acc(typename PrecT<PREC>::lacc v, uint32_t &flags) {
    if constexpr (PrecT<PREC>::fixed) {
        if (!(fabs(v) < 1125899906842624.0)) { flags |= ERR_OVERFLOW; return 0; }
        // v is an integer with |v| < 2^50: v + 1.5 * 2^52 is exact and lies in
        // [2^52, 2^53), where the bit pattern of a double grows by one per unit
        return __double_as_longlong(v + kFixBias) - __double_as_longlong(kFixBias);
    } else {
        return (typename PrecT<PREC>::acc)v;
    }
}

// int64 -> double, exact for |a| < 2^53 (two 32-bit conversions).
__device__ __forceinline__ double i64_to_f64(long long a) {
    const int hi = (int)(a >> 32);
    const unsigned lo = (unsigned)(a & 0xffffffffLL);
    return fma((double)hi, 4294967296.0, (double)lo);
}

template <int PREC>
__device__ __forceinline__ typename PrecT<PREC>::real from_acc(typename PrecT<PREC>::acc a, double q, uint32_t &flags) {
    using R = typename PrecT<PREC>::real;
    if constexpr (PrecT<PREC>::fixed) {
        const long long lim = 1LL << 50;
        if (a >= lim || a <= -lim) flags |= ERR_OVERFLOW;
        return (R)(i64_to_f64(a) * q);                       // q is a power of two
    } else {
        (void)q;
        return (R)a;
    }
}

// Word type of the grid buffers.  A 2D node's sum is finished by exactly one
// writer (the owning tile's flush, or the reduction of the frame), which
// stores it scaled to the state precision, the value every reader uses.
// 3D frame nodes take global atomics, so 3D grids hold accumulator words.
template <int DIM, int PREC> struct GridW {
    using type = typename std::conditional<DIM == 2, typename PrecT<PREC>::real, typename PrecT<PREC>::acc>::type;
};

// Value of a grid word in the state precision (q: its quantum).
template <int DIM, int PREC>
__device__ __forceinline__ typename PrecT<PREC>::real grid_val(typename GridW<DIM, PREC>::type w, double q,
                                                              uint32_t &flags) {
    if constexpr (DIM == 2) {
        (void)q; (void)flags;
        return w;
    } else {
        return from_acc<PREC>(w, q, flags);
    }
}

// -------------------------------------------------------------- atomics --
__device__ __forceinline__ void lds_add(long long *p, long long v) {
    atomicAdd((unsigned long long *)p, (unsigned long long)v);
}
__device__ __forceinline__ void lds_add(double *p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void lds_add(float *p, float v) { atomicAdd(p, v); }

__device__ __forceinline__ void glb_add(long long *p, long long v) {
    atomicAdd((unsigned long long *)p, (unsigned long long)v);
}
__device__ __forceinline__ void glb_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void glb_add(float *p, float v) { unsafeAtomicAdd(p, v); }
// The same on global-address-space pointers (global, not flat, atomics).
__device__ __forceinline__ void glb_add(GLOBAL_AS long long *p, long long v) {
    __hip_atomic_fetch_add((GLOBAL_AS unsigned long long *)p, (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void glb_add(GLOBAL_AS double *p, double v) { unsafeAtomicAdd((double *)p, v); }
__device__ __forceinline__ void glb_add(GLOBAL_AS float *p, float v) { unsafeAtomicAdd((float *)p, v); }

// ------------------------------------------------------------ boundary --
// Conditions on one nodal vector (Sec. 3 steps (iii), (vii)): obstacle
// projection u -= ((u.n - |u.n|)/2) n (eqs. normali1/2), then the normal
// component at wall faces, then the inflow state (momentum m u_in, force 0).
template <int DIM, typename R>
__device__ __forceinline__ void node_bc(const ProbDev *P, uint8_t fl, long long node, R m, R u[3], bool is_force) {
    if (fl & NF_OBST) {
        const GLOBAL_AS R *nrm = gmem((const R *)P->nrm);
        R n[3] = {0, 0, 0};
        R un = 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) { n[a] = nrm[a * P->nnodes + node]; un += u[a] * n[a]; }
        const R k = (R)0.5 * (un - fabs(un));
#pragma unroll
        for (int a = 0; a < DIM; ++a) u[a] -= k * n[a];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        if (fl & (NF_WALL_X << a)) u[a] = (R)0;
    if (fl & NF_INFLOW) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) u[a] = is_force ? (R)0 : m * (R)P->inflow_u[a];
    }
}

// ------------------------------------------------------ recycling hash --
// SplitMix64 output for state z (Steele, Lea, Flood 2014): golden-ratio
// increment, then the finaliser.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Postponed move X' = X + dt Vbar (Sec. 3 step (ix)).  A particle crossing an
// OUTFLOW high-x face re-enters at x - L_x with its transverse coordinates
// drawn from splitmix64(seed ^ step<<32 ^ id ^ (a-1)<<56) (reading of the
// random inflow cell of Sec. 4.1); any other exit is clamped and counted.
// Returns 1 when the particle was recycled, 2 when clamped, 0 otherwise.
// `id` gives the particle id (a value, or a load made only for a recycled
// particle).
struct IdVal {
    uint32_t v;
    __device__ uint32_t operator()() const { return v; }
};
struct IdAt {
    const GLOBAL_AS uint32_t *p;
    uint32_t k;
    __device__ uint32_t operator()() const { return p[k]; }
};
template <int DIM, typename R, class PP, class ID>
__device__ __forceinline__ int advect(const PP *P, R x[3], const R vbar[3], R dt, const ID &id) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) x[a] = x[a] + dt * vbar[a];
    // Outflow: through x_hi the particle is shifted back by the domain
    // length; through a y / z outflow face it re-enters at the x_lo inflow
    // face as far past it as it went past the face it left.  The transverse
    // coordinates come from the recycling hash.
    int out_axis = -1;
    R past = 0;
    if (P->face[0][1] == F_OUTFLOW && x[0] >= (R)P->hi[0]) out_axis = 0;
#pragma unroll
    for (int a = 1; a < DIM; ++a) {
        if (out_axis >= 0) break;
        if (P->face[a][0] == F_OUTFLOW && x[a] < (R)P->lo[a]) {
            out_axis = a;
            past = (R)P->lo[a] - x[a];
        } else if (P->face[a][1] == F_OUTFLOW && x[a] >= (R)P->hi[a]) {
            out_axis = a;
            past = x[a] - (R)P->hi[a];
        }
    }
    if (out_axis >= 0) {
        x[0] = out_axis == 0 ? x[0] - (R)(P->hi[0] - P->lo[0]) : (R)P->lo[0] + past;
#pragma unroll
        for (int a = 1; a < DIM; ++a) {
            const unsigned long long word = P->seed ^ ((unsigned long long)P->step << 32) ^
                                            (unsigned long long)id() ^ ((unsigned long long)(a - 1) << 56);
            const double u = (double)(splitmix64(word) >> 11) * 0x1.0p-53;
            x[a] = (R)(P->lo[a] + (P->hi[a] - P->lo[a]) * u);
        }
        return 1;
    }
    int clamped = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const R lo = (R)P->lo[a], hi = (R)P->hi[a];
        if (x[a] < lo) { x[a] = lo; clamped = 2; }
        else if (x[a] >= hi) {
            R in = (R)(P->hi[a] - 1e-9 * (P->hi[a] - P->lo[a]));
            if (in >= hi) in = nextafter(hi, lo);
            x[a] = in;
            clamped = 2;
        }
    }
    return clamped;
}

// Tile-major cell key of a cell triple.
template <int DIM, class PP>
__device__ __forceinline__ uint32_t cell_key(const PP *P, const int c[3]) {
    constexpr int TX = Tile<DIM>::X, TY = Tile<DIM>::Y, TZ = Tile<DIM>::Z;
    const int tx = c[0] / TX, ty = c[1] / TY, tz = DIM == 3 ? c[2] / TZ : 0;
    const int lx = c[0] - tx * TX, ly = c[1] - ty * TY, lz = DIM == 3 ? c[2] - tz * TZ : 0;
    const long long tile = ((long long)tz * P->ntile[1] + ty) * P->ntile[0] + tx;
    return (uint32_t)(tile * Tile<DIM>::CELLS + (lz * TY + ly) * TX + lx);
}

// Cell triple of a position (the first stencil node of the basis).
template <int DIM, typename R, class PP>
__device__ __forceinline__ void cell_of(const PP *P, const R x[3], int c[3]) {
    const R inv_h = (R)P->inv_h;
    c[2] = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const R s = (x[a] - (R)P->lo[a]) * inv_h;
        int ca = (int)floor(s);
        c[a] = ca < 0 ? 0 : (ca > P->n[a] - 1 ? P->n[a] - 1 : ca);
    }
}

// ----------------------------------------------------------- node staging --
// Nodal values the gather sweeps need, computed from the integer / float
// accumulators with the boundary conditions applied:
//   vstar = (p + I)/m  with p, I after the conditions (I = dt f, the impulse)
//   dvel  = I/m        (the velocity increment dt f/m)
//   v2    = p2/m       with p2 after the momentum conditions
// Nodes without mass give 0.
template <int DIM, int PREC>
__device__ __forceinline__ void stage_A(const ProbDev *P, long long node,
                                        typename PrecT<PREC>::real vstar[3],
                                        typename PrecT<PREC>::real dvel[3], uint32_t &flags) {
    using R = typename PrecT<PREC>::real;
    using GW = typename GridW<DIM, PREC>::type;
    const GLOBAL_AS GW *g = gmem((const GW *)P->gA[P->parity]);
    const long long NN = P->nnodes;
    GW raw[1 + 2 * DIM];
#pragma unroll
    for (int q = 0; q < 1 + 2 * DIM; ++q) raw[q] = g[q * NN + node];
    const R m = grid_val<DIM, PREC>(raw[0], P->q_m, flags);
    R p[3] = {0, 0, 0}, I[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        p[a] = grid_val<DIM, PREC>(raw[1 + a], P->q_p, flags);
        I[a] = grid_val<DIM, PREC>(raw[1 + DIM + a], P->q_p, flags);
    }
    const uint8_t fl = gmem((const uint8_t *)P->nflag)[node];
    if (fl) {
        node_bc<DIM, R>(P, fl, node, m, p, false);
        node_bc<DIM, R>(P, fl, node, m, I, true);
    }
    const R inv_m = m > (R)0 ? recip(m) : (R)0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        vstar[a] = (p[a] + I[a]) * inv_m;
        dvel[a] = I[a] * inv_m;
    }
}

template <int DIM, int PREC>
__device__ __forceinline__ void stage_B(const ProbDev *P, long long node,
                                        typename PrecT<PREC>::real v2[3], uint32_t &flags) {
    using R = typename PrecT<PREC>::real;
    using GW = typename GridW<DIM, PREC>::type;
    const GLOBAL_AS GW *gA = gmem((const GW *)P->gA[P->parity]);
    const GLOBAL_AS GW *gB = gmem((const GW *)P->gB[P->parity]);
    const long long NN = P->nnodes;
    const R m = grid_val<DIM, PREC>(gA[node], P->q_m, flags);
    R p[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) p[a] = grid_val<DIM, PREC>(gB[a * NN + node], P->q_p, flags);
    const uint8_t fl = gmem((const uint8_t *)P->nflag)[node];
    if (fl) node_bc<DIM, R>(P, fl, node, m, p, false);
    const R inv_m = m > (R)0 ? recip(m) : (R)0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) v2[a] = p[a] * inv_m;
}

template <class PP>
__device__ __forceinline__ long long node_index(const PP *P, int ix, int iy, int iz) {
    return (long long)ix + (long long)P->nn[0] * ((long long)iy + (long long)P->nn[1] * iz);
}

// ---------------------------------------------------------- frame halos --
// 2D: the footprint of a tile (NX x NX nodes, NX = T + W - 1) holds the
// nodes that only its own cells reach (local index W-1 .. T-1 on both axes,
// "owned") and a frame shared with the neighbouring tiles.  The P2G sweeps
// store the owned sums into the grid and the frame sums into the tile's
// halo record instead of adding them atomically; a frame node's value is the
// sum over the 1-4 tiles whose footprint holds it, always in the same order.
template <int SHAPE> struct Frame2 {
    static constexpr int T = Tile<2>::X;                 // tiles are square in 2D
    static constexpr int E = SHAPE == S_B2 ? 2 : 1;      // W - 1
    static constexpr int NX = T + E;
    static constexpr int NFR = 4 * E * T;                // frame nodes per tile
};
static_assert(Tile<2>::X == Tile<2>::Y, "square 2D tiles");

// Slot of frame position (lx, ly) in a tile's halo record.
template <int SHAPE> __device__ __forceinline__ int frame_slot(int lx, int ly) {
    using F = Frame2<SHAPE>;
    if (ly < F::E) return ly * F::NX + lx;
    if (ly >= F::T) return F::E * F::NX + (ly - F::T) * F::NX + lx;
    return 2 * F::E * F::NX + (ly - F::E) * 2 * F::E + (lx < F::E ? lx : lx - F::T + F::E);
}

// Frame position of halo slot sl (the inverse of frame_slot).
template <int SHAPE> __device__ __forceinline__ void frame_pos(int sl, int &lx, int &ly) {
    using F = Frame2<SHAPE>;
    if (sl < 2 * F::E * F::NX) {
        const int r = sl / F::NX;
        ly = r < F::E ? r : r - F::E + F::T;
        lx = sl % F::NX;
        return;
    }
    sl -= 2 * F::E * F::NX;
    ly = F::E + sl / (2 * F::E);
    const int c = sl % (2 * F::E);
    lx = c < F::E ? c : c - F::E + F::T;
}

// Tiles along one axis whose footprint holds node g, with g's local index
// in each.  The first is the node's reducer tile.
template <int SHAPE> __device__ __forceinline__ int frame_contrib(int g, int ntile, int t[2], int l[2]) {
    using F = Frame2<SHAPE>;
    int t1 = g / F::T;
    if (t1 > ntile - 1) t1 = ntile - 1;
    t[0] = t1;
    l[0] = g - t1 * F::T;
    t[1] = t1;
    l[1] = l[0];
    if (l[0] < F::E && t1 > 0) {
        t[1] = t1 - 1;
        l[1] = l[0] + F::T;
        return 2;
    }
    return 1;
}

// Accumulators q < NQ of frame node (gx, gy): the sum of the halo entries
// of the tiles holding it.  All candidate entries are loaded at once (a
// missing second tile re-reads the first entry, which for a frame node is
// always a frame position, and is masked out), then summed in a fixed
// order.
template <int SHAPE, int NQ, typename A>
__device__ __forceinline__ void gather_frame(const ProbDev *P, const GLOBAL_AS A *halo, int gx, int gy, A out[NQ]) {
    using F = Frame2<SHAPE>;
    int tx[2], lx[2], ty[2], ly[2];
    const int cx = frame_contrib<SHAPE>(gx, P->ntile[0], tx, lx);
    const int cy = frame_contrib<SHAPE>(gy, P->ntile[1], ty, ly);
    const long long ntl = P->ntiles;
    long long base[4];
    bool use[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int i = c >> 1, j = c & 1;
        use[c] = i < cx && j < cy;
        const int ii = use[c] ? i : 0, jj = use[c] ? j : 0;
        base[c] = ((long long)ty[jj] * P->ntile[0] + tx[ii]) * F::NFR + frame_slot<SHAPE>(lx[ii], ly[jj]);
    }
    A v[4][NQ];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[c][q] = halo[(long long)q * ntl * F::NFR + base[c]];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        A sum = (A)0;
#pragma unroll
        for (int c = 0; c < 4; ++c) sum += use[c] ? v[c][q] : (A)0;
        out[q] = sum;
    }
}

// Tile of local workgroup j (of n) when groups of G consecutive tiles go to
// one XCD: workgroups are dealt to the 8 XCDs round-robin (j % 8), so tile
// t = (k / G) * 8G + (j % 8) * G + k % G with k = j / 8 keeps G neighbouring
// tiles (and, when 8G divides the tile row, the tiles above and below) on
// the XCD whose L2 holds their shared cache lines.  A bijection on
// [0, n): the tail beyond the last full 8G block keeps j.
template <int G>
__device__ __forceinline__ int xcd_tile(int j, int n) {
    constexpr int M = 8 * G;
    if (G <= 1 || j >= (n / M) * M) return j;
    const int k = j >> 3, x = j & 7;
    return (k / G) * M + x * G + (k % G);
}

// Element k of a particle array addressed with a 32-bit byte offset (the
// particle count is limited so that every array stays below 4 GiB): the
// access then takes the array base from scalar registers plus one vector
// offset, instead of a 64-bit address computed per access.
template <typename T>
__device__ __forceinline__ T ldk(const GLOBAL_AS T *base, uint32_t k) {
    return *(const GLOBAL_AS T *)((const GLOBAL_AS char *)base + k * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stk(GLOBAL_AS T *base, uint32_t k, T v) {
    *(GLOBAL_AS T *)((GLOBAL_AS char *)base + k * (uint32_t)sizeof(T)) = v;
}

// Problem owning workgroup b of a batched launch.
__device__ __forceinline__ int find_prob(const WorkTab &wt, int b) {
    int lo = 0, hi = wt.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wt.start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace mpm
