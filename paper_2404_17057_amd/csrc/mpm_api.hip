// Host side of the C ABI declared in include/mpm.h: descriptor checks,
// workspace layout, initial upload and cell sort, stepping (eager launches or
// replays of a captured hipGraph of several steps), batching and read-back.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_common.hpp"

namespace mpm {
void launch_step(int dim, int shape, int prec, const WorkTab &tiles, const WorkTab &single, hipStream_t s);
void launch_init(int dim, int shape, int prec, ProbDev *dP, const ProbDev &h, hipStream_t s);
void launch_grid_diag(int dim, int shape, int prec, ProbDev *dP, const ProbDev &h, int which,
                      double *out, hipStream_t s);
void launch_arm(const WorkTab &single, const long long *n, hipStream_t s);
void launch_conserved(ProbDev *dP, hipStream_t s);
void launch_part(int dim, int shape, int prec, int part, const WorkTab &tiles, const WorkTab &single,
                 hipStream_t s);
}  // namespace mpm

using namespace mpm;

namespace {

constexpr int kGraphSteps = 16;      // steps per replay of the largest captured graph
// Captured graphs of a handle: 16, 8, 4, 2 and 1 steps, so that any step
// count is a run of graph replays (the binary digits of the remainder).
constexpr int kGraphLevels = 5;
constexpr int graph_steps(int level) { return kGraphSteps >> level; }
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Fixed device scratch of mpm_read_grid_noalloc: the staging buffer of one
// grid snapshot.  Every GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` only names the symbol; its device
// address, per device, comes from hipGetSymbolAddress (scratch_address).
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices];

// Device address of the current device's `scratch`, resolved once per device.
int scratch_address(double **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MPM_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MPM_E_HIP;
        g_scratch[dev] = (double *)p;
    }
    *out = g_scratch[dev];
    return MPM_OK;
}

struct Layout {
    int dim, shape, prec;
    int nn[3], ntile[3], ntiles, nchunks;
    long long ncells_pad, nnodes, np;
    size_t real_sz, acc_sz;
    // byte offsets
    size_t off_prob, off_part[2][PF_N], off_pid[2], off_key, off_rank, off_basetab;
    size_t off_gA[2], off_gB[2], off_haloA, off_haloB, off_count, off_ttot, off_tbase, off_zero_end, off_offs[2], off_blocksum,
        off_nflag, off_nrm, off_partials, total;
    int has_obstacle;
};

int check_desc(const mpm_desc *d, double *h_out) {
    if (!d) return MPM_E_ARG;
    if (d->dim != 2 && d->dim != 3) return MPM_E_ARG;
    if (d->shape != MPM_Q1 && d->shape != MPM_B2) return MPM_E_ARG;
    if (d->precision < MPM_FP64 || d->precision > MPM_FP64_COLOR) return MPM_E_ARG;
    if (d->av_form != MPM_AV_PAPER && d->av_form != MPM_AV_BOOK) return MPM_E_ARG;
    if (!(d->gamma > 1.0) || !(d->cfl > 0.0) || d->n_particles < 0) return MPM_E_ARG;
    // particle arrays are addressed with 32-bit byte offsets: each must stay
    // below 4 GiB
    const long long real_sz = (d->precision == MPM_FP64 || d->precision == MPM_FP64_COLOR) ? 8 : 4;
    if (d->n_particles * real_sz > 0xFFFFFFF0LL) return MPM_E_UNSUPPORTED;
    if (d->shape == MPM_Q1 && d->precision != MPM_FP64 && d->precision != MPM_FP32_FIX64)
        return MPM_E_UNSUPPORTED;   // (the colouring is built for B2's 3^dim colours)
    double h = 0;
    for (int a = 0; a < d->dim; ++a) {
        if (d->n[a] < 2 || !(d->hi[a] > d->lo[a])) return MPM_E_ARG;
        const double ha = (d->hi[a] - d->lo[a]) / d->n[a];
        if (a == 0) h = ha;
        else if (fabs(ha - h) > 1e-9 * h) return MPM_E_ARG;
        for (int s = 0; s < 2; ++s)
            if (d->face[a][s] < MPM_FACE_WALL || d->face[a][s] > MPM_FACE_OUTFLOW) return MPM_E_ARG;
    }
    // particles leaving through an outflow face re-enter at the x_lo face,
    // which must then be the inflow face (and cannot itself be an outflow)
    for (int a = 0; a < d->dim; ++a)
        for (int s = 0; s < 2; ++s)
            if (d->face[a][s] == MPM_FACE_OUTFLOW &&
                ((a == 0 && s == 0) || d->face[0][0] != MPM_FACE_INFLOW))
                return MPM_E_UNSUPPORTED;
    // an INFLOW face imposes, and recycling through an OUTFLOW face
    // regenerates particles with, the inflow state: it must be physical
    bool inflow = false, outflow = false;
    for (int a = 0; a < d->dim; ++a)
        for (int s = 0; s < 2; ++s) {
            inflow |= d->face[a][s] == MPM_FACE_INFLOW;
            outflow |= d->face[a][s] == MPM_FACE_OUTFLOW;
        }
    if (inflow || outflow) {
        if (!(d->inflow_rho > 0) || !isfinite(d->inflow_rho) || !(d->inflow_p >= 0) || !isfinite(d->inflow_p))
            return MPM_E_ARG;
        for (int a = 0; a < d->dim; ++a)
            if (!isfinite(d->inflow_u[a])) return MPM_E_ARG;
    }
    if (outflow && (!(d->recycle_mass > 0) || !isfinite(d->recycle_mass))) return MPM_E_ARG;
    // restart state
    if (!(d->t0 >= 0) || !isfinite(d->t0) || d->step0 < 0 || !isfinite(d->dt0)) return MPM_E_ARG;
    // cell keys and tile-major cell indices are 32-bit, node indices are
    // int: at most 2^31 padded cells and 2^31 - 1 nodes
    {
        const int T[3] = {d->dim == 2 ? Tile<2>::X : Tile<3>::X, d->dim == 2 ? Tile<2>::Y : Tile<3>::Y,
                          d->dim == 2 ? Tile<2>::Z : Tile<3>::Z};
        const int extra = d->shape == MPM_B2 ? 2 : 1;
        double cells_pad = 1.0, nodes = 1.0;
        for (int a = 0; a < d->dim; ++a) {
            cells_pad *= (double)((d->n[a] + (long long)T[a] - 1) / T[a]) * T[a];
            nodes *= (double)d->n[a] + extra;
        }
        if (cells_pad > 2147483648.0 || nodes > 2147483647.0) return MPM_E_UNSUPPORTED;
    }
    *h_out = h;
    return MPM_OK;
}

Layout make_layout(const mpm_desc *d) {
    Layout L{};
    L.dim = d->dim;
    L.shape = d->shape;
    L.prec = d->precision;
    L.np = d->n_particles;
    const int extra = d->shape == MPM_B2 ? 2 : 1;
    const int T[3] = {d->dim == 2 ? Tile<2>::X : Tile<3>::X, d->dim == 2 ? Tile<2>::Y : Tile<3>::Y,
                      d->dim == 2 ? Tile<2>::Z : Tile<3>::Z};
    L.nnodes = 1;
    L.ntiles = 1;
    for (int a = 0; a < 3; ++a) {
        const int n = a < d->dim ? d->n[a] : 1;
        L.nn[a] = a < d->dim ? n + extra : 1;
        L.ntile[a] = a < d->dim ? (n + T[a] - 1) / T[a] : 1;
        L.nnodes *= L.nn[a];
        L.ntiles *= L.ntile[a];
    }
    L.ncells_pad = (long long)L.ntiles * 256;
    L.nchunks = (int)((L.ncells_pad + kScanChunk - 1) / kScanChunk);
    L.real_sz = (d->precision == MPM_FP64 || d->precision == MPM_FP64_COLOR) ? 8 : 4;
    L.acc_sz = d->precision == MPM_FP32_ACC_F32 ? 4 : 8;
    size_t o = 0;
    L.off_prob = o; o = align_up(o + sizeof(ProbDev));
    // The stored fields of one parity are consecutive arrays one stride
    // apart, field f at field_slot(dim, f) strides past the first: the update
    // sweep addresses them that way.
    const size_t fstride = align_up((size_t)L.np * L.real_sz);
    for (int p = 0; p < 2; ++p) {
        for (int f = 0; f < PF_N; ++f)
            L.off_part[p][f] = field_used(d->dim, f) ? o + (size_t)field_slot(d->dim, f) * fstride : (size_t)-1;
        o += (size_t)field_slot(d->dim, PF_N) * fstride;
        L.off_pid[p] = o; o = align_up(o + (size_t)L.np * 4);
    }
    L.off_key = o; o = align_up(o + (size_t)L.np * 4);
    L.off_rank = o; o = align_up(o + (size_t)L.np * 4);
    {
        // per tile: one u32 per cell of its destination footprint (tile + 1 cell)
        const size_t nd = d->dim == 2 ? (size_t)(Tile<2>::X + 2) * (Tile<2>::Y + 2)
                                      : (size_t)(Tile<3>::X + 2) * (Tile<3>::Y + 2) * (Tile<3>::Z + 2);
        L.off_basetab = o; o = align_up(o + (size_t)L.ntiles * nd * 4);
    }
    for (int p = 0; p < 2; ++p) {
        L.off_gA[p] = o; o = align_up(o + (size_t)(1 + 2 * d->dim) * L.nnodes * L.acc_sz);
        L.off_gB[p] = o; o = align_up(o + (size_t)d->dim * L.nnodes * L.acc_sz);
    }
    L.off_haloA = L.off_haloB = (size_t)-1;
    if (d->dim == 2) {
        // per tile, the frame nodes of its footprint (4 (W-1) T of them)
        const size_t nfr = (size_t)4 * (d->shape == MPM_B2 ? 2 : 1) * Tile<2>::X;
        L.off_haloA = o; o = align_up(o + (size_t)(1 + 2 * d->dim) * L.ntiles * nfr * L.acc_sz);
        L.off_haloB = o; o = align_up(o + (size_t)d->dim * L.ntiles * nfr * L.acc_sz);
    }
    L.off_count = o; o = align_up(o + (size_t)L.ncells_pad * 4);
    L.off_ttot = o; o = align_up(o + (size_t)L.ntiles * 4);
    L.off_zero_end = o;
    L.off_tbase = o; o = align_up(o + (size_t)(L.ntiles + 1) * 4);
    for (int p = 0; p < 2; ++p) { L.off_offs[p] = o; o = align_up(o + (size_t)(L.ncells_pad + 1) * 4); }
    L.off_blocksum = o; o = align_up(o + (size_t)L.nchunks * 4);
    L.off_nflag = o; o = align_up(o + (size_t)L.nnodes);
    L.off_nrm = o; o = align_up(o + (size_t)d->dim * L.nnodes * L.real_sz);
    L.off_partials = o; o = align_up(o + (size_t)L.ntiles * PT_N * 8);
    L.total = o;
    return L;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? MPM_OK : MPM_E_HIP; }

}  // namespace

struct mpm_handle {
    Layout L;
    ProbDev host;          // static part, host mirror
    ProbDev *dev;          // device descriptor (workspace start)
    char *ws;
    int reported_err;
    double *scratch;       // this device's copy of `scratch` (mpm_read_grid_noalloc)
    // graphs of single-problem stepping, captured by the first mpm_step
    hipGraphExec_t gexec[kGraphLevels];
    hipStream_t cap;
};

namespace {

void make_tables(mpm_handle *const *hs, int n, WorkTab &tiles, WorkTab &single) {
    tiles = WorkTab{}; single = WorkTab{};
    int bt = 0;
    for (int i = 0; i < n; ++i) {
        ProbDev *p = hs[i]->dev;
        tiles.prob[i] = single.prob[i] = p;
        tiles.start[i] = bt; bt += hs[i]->host.ntiles;
        single.start[i] = i;
    }
    tiles.start[n] = bt; single.start[n] = n;
    tiles.n = single.n = n;
    int mt = 0;
    for (int i = 0; i < n; ++i) mt = std::max(mt, hs[i]->host.ntiles);
    tiles.max_tiles = single.max_tiles = mt;
}


// Capture `steps` steps of the work tables into *exec: the executable graph
// is updated in place when it exists (same topology, new kernel arguments),
// else instantiated.
int capture_steps(int dim, int shape, int prec, const WorkTab &tiles, const WorkTab &single, int steps,
                  hipStream_t cap, hipGraphExec_t *exec) {
    hipGraph_t g;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPM_E_HIP;
    for (int k = 0; k < steps; ++k) launch_step(dim, shape, prec, tiles, single, cap);
    if (hipStreamEndCapture(cap, &g) != hipSuccess) return MPM_E_HIP;
    int st = MPM_OK;
    if (*exec) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(*exec, g, &bad, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(*exec);
            *exec = nullptr;
        }
    }
    if (!*exec && hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess) {
        *exec = nullptr;
        st = MPM_E_HIP;
    }
    (void)hipGraphDestroy(g);
    return st;
}

// Graphs of batched stepping, per device: the step graphs (16, 8, 4, 2, 1
// steps) of the last batch composition seen at each level.  A composition
// is the kernel variant and the work tables (the problems' descriptors and
// tile counts): everything a captured launch bakes in, as the kernels read
// the rest from the descriptors at run time.
struct BatchKey {
    int dim, shape, prec, pad;
    WorkTab tiles;
};
struct BatchGraphs {
    BatchKey key[kGraphLevels];
    bool valid[kGraphLevels];
    hipGraphExec_t exec[kGraphLevels];
    hipStream_t cap;
};
std::mutex g_batch_mu;
BatchGraphs g_batch[kMaxDevices];

int read_dynamic(mpm_handle *h, ProbDev *out, hipStream_t s) {
    if (hipStreamSynchronize(s) != hipSuccess) return MPM_E_HIP;
    if (hipMemcpy(out, h->dev, sizeof(ProbDev), hipMemcpyDeviceToHost) != hipSuccess) return MPM_E_HIP;
    return MPM_OK;
}

int err_code(uint32_t err) {
    if (err & ERR_INTERNAL) return MPM_E_STATE;
    if (err & ERR_OVERFLOW) return MPM_E_OVERFLOW;
    if (err & (ERR_NONPHYS | ERR_NONFINITE)) return MPM_E_NONPHYSICAL;
    return MPM_OK;
}

}  // namespace

extern "C" {

const char *mpm_strerror(int code) {
    switch (code) {
    case MPM_OK: return "ok";
    case MPM_E_ARG: return "invalid argument";
    case MPM_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case MPM_E_HIP: return "HIP runtime error";
    case MPM_E_NONPHYSICAL: return "non-physical state (J <= 0 or non-finite value)";
    case MPM_E_OVERFLOW: return "fixed-point accumulator overflow";
    case MPM_E_UNSUPPORTED: return "unsupported configuration";
    case MPM_E_STATE: return "handle is in an error state";
    case MPM_E_SCRATCH: return "request larger than the fixed device scratch buffer (32 MiB)";
    default: return "unknown status";
    }
}

int mpm_footprint(const mpm_desc *desc, size_t *device_bytes) {
    double h;
    int rc = check_desc(desc, &h);
    if (rc) return rc;
    if (!device_bytes) return MPM_E_ARG;
    *device_bytes = make_layout(desc).total;
    return MPM_OK;
}

int mpm_init(const mpm_desc *d, const mpm_particles_host *pp, const mpm_obstacle_host *obs,
             void *dev_workspace, size_t workspace_bytes, void *hip_stream, mpm_handle **out) {
    double h;
    int rc = check_desc(d, &h);
    if (rc) return rc;
    if (!pp || !out) return MPM_E_ARG;
    const int dim = d->dim;
    const long long np = d->n_particles;
    if (np > 0) {
        for (int a = 0; a < dim; ++a)
            if (!pp->x[a] || !pp->v[a]) return MPM_E_ARG;
        if (!pp->mass || !pp->rho || !pp->eint || !pp->id) return MPM_E_ARG;
    }
    if (obs && obs->cell_mask)
        for (int a = 0; a < dim; ++a)
            if (!obs->node_normal[a]) return MPM_E_ARG;
    const Layout L = make_layout(d);
    if (!dev_workspace || ((uintptr_t)dev_workspace % kAlign) != 0 || workspace_bytes < L.total)
        return MPM_E_WORKSPACE;
    hipStream_t s = (hipStream_t)hip_stream;

    // ---- host-side checks of the particle set
    std::vector<uint8_t> seen((size_t)np, 0);
    double rho_max = 0, u_max = 0;
    for (long long k = 0; k < np; ++k) {
        const uint32_t q = pp->id[k];
        if ((long long)q >= np || seen[q]) return MPM_E_ARG;
        seen[q] = 1;
        double v2 = 0;
        for (int a = 0; a < dim; ++a) {
            const double x = pp->x[a][k];
            if (!(x >= d->lo[a] && x < d->hi[a])) return MPM_E_ARG;
            v2 += pp->v[a][k] * pp->v[a][k];
        }
        if (!isfinite(v2)) return MPM_E_ARG;
        if (!(pp->mass[k] > 0) || !(pp->rho[k] > 0) || !isfinite(pp->eint[k])) return MPM_E_ARG;
        rho_max = std::max(rho_max, pp->rho[k]);
        const double pr = (d->gamma - 1.0) * pp->rho[k] * pp->eint[k];
        const double c2 = d->gamma * pr / pp->rho[k];
        u_max = std::max(u_max, sqrt(v2) + (c2 > 0 ? sqrt(c2) : 0.0));
    }

    mpm_handle *H = (mpm_handle *)calloc(1, sizeof(mpm_handle));
    if (!H) return MPM_E_ARG;
    if (scratch_address(&H->scratch) != MPM_OK) { free(H); return MPM_E_HIP; }
    H->L = L;
    H->ws = (char *)dev_workspace;
    H->dev = (ProbDev *)(H->ws + L.off_prob);
    ProbDev &P = H->host;
    memset(&P, 0, sizeof(P));
    P.dim = dim; P.shape = d->shape; P.prec = d->precision; P.av_form = d->av_form;
    for (int a = 0; a < 3; ++a) {
        P.n[a] = a < dim ? d->n[a] : 1;
        P.nn[a] = L.nn[a];
        P.ntile[a] = L.ntile[a];
        P.lo[a] = a < dim ? d->lo[a] : 0.0;
        P.hi[a] = a < dim ? d->hi[a] : 1.0;
        P.face[a][0] = a < dim ? d->face[a][0] : MPM_FACE_WALL;
        P.face[a][1] = a < dim ? d->face[a][1] : MPM_FACE_WALL;
        P.inflow_u[a] = a < dim ? d->inflow_u[a] : 0.0;
    }
    P.ntiles = L.ntiles; P.nchunks = L.nchunks; P.ncells_pad = L.ncells_pad;
    P.nnodes = L.nnodes; P.np = np;
    P.h = h; P.inv_h = 1.0 / h;
    P.gamma = d->gamma; P.c0 = d->c0; P.c1 = d->c1; P.cfl = d->cfl;
    P.inflow_rho = d->inflow_rho; P.inflow_p = d->inflow_p;
    P.inflow_e = d->inflow_rho > 0 ? d->inflow_p / ((d->gamma - 1.0) * d->inflow_rho) : 0.0;
    P.recycle_mass = d->recycle_mass;
    P.seed = d->seed;
    P.t_end = d->t_end;
    // a resumed run continues the clock and the step count (the step keys the
    // recycling hash); the given G is the whole gradient of that step
    P.t = d->t0;
    P.step = d->step0;
    P.g_step = d->step0;
    // Fixed-point quanta: powers of two so that scaling is exact.  Mass:
    // 2^-32 of the mass of a cell at the reference density; momentum and
    // impulse: that times the power of two above the reference speed.
    {
        const double rho_ref = d->rho_ref > 0 ? d->rho_ref : (rho_max > 0 ? rho_max : 1.0);
        double u_ref = d->u_ref > 0 ? d->u_ref : 4.0 * u_max;
        if (!(u_ref > 0)) u_ref = 1.0;
        const double cellm = rho_ref * pow(h, dim);
        P.q_m = ldexp(1.0, (int)floor(log2(cellm)) - 32);
        P.q_p = P.q_m * ldexp(1.0, (int)ceil(log2(u_ref)));
        P.inv_q_m = 1.0 / P.q_m;
        P.inv_q_p = 1.0 / P.q_p;
    }
    P.has_obstacle = (obs && obs->cell_mask) ? 1 : 0;
    for (int p = 0; p < 2; ++p) {
        for (int f = 0; f < PF_N; ++f)
            P.part[p][f] = L.off_part[p][f] == (size_t)-1 ? nullptr : (void *)(H->ws + L.off_part[p][f]);
        P.pid[p] = (uint32_t *)(H->ws + L.off_pid[p]);
        P.offs[p] = (uint32_t *)(H->ws + L.off_offs[p]);
    }
    P.key = (uint32_t *)(H->ws + L.off_key);
    P.rank = (uint32_t *)(H->ws + L.off_rank);
    P.basetab = (uint32_t *)(H->ws + L.off_basetab);
    P.count = (uint32_t *)(H->ws + L.off_count);
    P.blocksum = (uint32_t *)(H->ws + L.off_blocksum);
    for (int p = 0; p < 2; ++p) {
        P.gA[p] = H->ws + L.off_gA[p];
        P.gB[p] = H->ws + L.off_gB[p];
    }
    P.ttot = (uint32_t *)(H->ws + L.off_ttot);
    P.tbase = (uint32_t *)(H->ws + L.off_tbase);
    P.nflag = (uint8_t *)(H->ws + L.off_nflag);
    P.nrm = H->ws + L.off_nrm;
    P.partials = (double *)(H->ws + L.off_partials);
    P.haloA = L.off_haloA == (size_t)-1 ? nullptr : (void *)(H->ws + L.off_haloA);
    P.haloB = L.off_haloB == (size_t)-1 ? nullptr : (void *)(H->ws + L.off_haloB);
    P.parity = 1;      // the unsorted input goes to parity 1, the sort writes parity 0
    P.active = 1;

    int st = MPM_OK;
    // ---- particle upload (converted to the state precision) into parity 1
    {
        std::vector<char> buf((size_t)std::max<long long>(np, 1) * 8);
        auto put = [&](int f, const double *src, int axis) -> int {
            if (!P.part[1][f]) return MPM_OK;
            if (L.real_sz == 8) {
                if (src) memcpy(buf.data(), src, (size_t)np * 8);
                else memset(buf.data(), 0, (size_t)np * 8);
            } else {
                float *dst = (float *)buf.data();
                for (long long k = 0; k < np; ++k) dst[k] = src ? (float)src[k] : 0.0f;
                if (axis >= 0) {
                    // a position just below hi can round up to hi in float
                    const float hi = (float)d->hi[axis], lo = (float)d->lo[axis];
                    for (long long k = 0; k < np; ++k) {
                        if (dst[k] >= hi) dst[k] = nextafterf(hi, lo);
                        if (dst[k] < lo) dst[k] = lo;
                    }
                }
            }
            return hip_ok(hipMemcpy(P.part[1][f], buf.data(), (size_t)np * L.real_sz, hipMemcpyHostToDevice));
        };
        for (int a = 0; a < dim && !st; ++a) st = put(PF_X + a, pp->x[a], a);
        for (int a = 0; a < dim && !st; ++a) st = put(PF_V + a, pp->v[a], -1);
        if (!st) st = put(PF_M, pp->mass, -1);
        if (!st) st = put(PF_RHO, pp->rho, -1);
        if (!st) st = put(PF_E, pp->eint, -1);
        for (int c = 0; c < dim * dim && !st; ++c) st = put(PF_G + c, pp->gradv[c], -1);
        if (!st && np > 0)
            st = hip_ok(hipMemcpy(P.pid[1], pp->id, (size_t)np * 4, hipMemcpyHostToDevice));
    }
    // ---- node flags and obstacle normals (static boundary description)
    if (!st) {
        std::vector<uint8_t> flag((size_t)L.nnodes, 0);
        std::vector<char> nrm((size_t)dim * L.nnodes * L.real_sz, 0);
        for (long long i = 0; i < L.nnodes; ++i) {
            long long r = i;
            int idx[3];
            for (int a = 0; a < 3; ++a) { idx[a] = (int)(r % L.nn[a]); r /= L.nn[a]; }
            uint8_t f = 0;
            for (int a = 0; a < dim; ++a) {
                const bool lo = idx[a] == 0, hi = idx[a] == L.nn[a] - 1;
                if ((lo && d->face[a][0] == MPM_FACE_WALL) || (hi && d->face[a][1] == MPM_FACE_WALL))
                    f |= (uint8_t)(NF_WALL_X << a);
                if ((lo && d->face[a][0] == MPM_FACE_INFLOW) || (hi && d->face[a][1] == MPM_FACE_INFLOW))
                    f |= NF_INFLOW;
            }
            if (P.has_obstacle) {
                bool ob = false;
                if (d->shape == MPM_B2) {
                    // node j sits at a Greville point inside cell clamp(j-1)
                    long long cflat = 0, stride = 1;
                    for (int a = 0; a < dim; ++a) {
                        int c = idx[a] - 1;
                        c = c < 0 ? 0 : (c > d->n[a] - 1 ? d->n[a] - 1 : c);
                        cflat += c * stride;
                        stride *= d->n[a];
                    }
                    ob = obs->cell_mask[cflat] != 0;
                } else {
                    for (int q = 0; q < (1 << dim) && !ob; ++q) {
                        long long cflat = 0, stride = 1;
                        bool ok = true;
                        for (int a = 0; a < dim; ++a) {
                            const int c = idx[a] - ((q >> a) & 1);
                            if (c < 0 || c > d->n[a] - 1) { ok = false; break; }
                            cflat += c * stride;
                            stride *= d->n[a];
                        }
                        if (ok && obs->cell_mask[cflat]) ob = true;
                    }
                }
                if (ob) {
                    f |= NF_OBST;
                    for (int a = 0; a < dim; ++a) {
                        const double nv = obs->node_normal[a][i];
                        if (L.real_sz == 8) ((double *)nrm.data())[a * L.nnodes + i] = nv;
                        else ((float *)nrm.data())[a * L.nnodes + i] = (float)nv;
                    }
                }
            }
            flag[(size_t)i] = f;
        }
        st = hip_ok(hipMemcpy(P.nflag, flag.data(), (size_t)L.nnodes, hipMemcpyHostToDevice));
        if (!st) st = hip_ok(hipMemcpy(P.nrm, nrm.data(), nrm.size(), hipMemcpyHostToDevice));
    }
    // both grid buffers, the histogram and the tile totals start at zero
    if (!st) st = hip_ok(hipMemsetAsync(H->ws + L.off_gA[0], 0, L.off_zero_end - L.off_gA[0], s));
    if (!st) st = hip_ok(hipMemcpyAsync(H->dev, &P, sizeof(ProbDev), hipMemcpyHostToDevice, s));
    if (!st) {
        launch_init(dim, d->shape, d->precision, H->dev, P, s);
        st = hip_ok(hipGetLastError());
    }
    // a resumed run takes the next time step it was given instead of the one
    // derived from the state (the init reduction sees |V| only, not the
    // moved-with velocity of the step that produced the state)
    if (!st && d->dt0 > 0)
        st = hip_ok(hipMemcpyAsync(&H->dev->dt, &d->dt0, sizeof(double), hipMemcpyHostToDevice, s));
    if (!st) st = hip_ok(hipStreamSynchronize(s));
    if (st) { free(H); return st; }
    *out = H;
    return MPM_OK;
}

int mpm_step_batch(mpm_handle *const *hs, int32_t n, const int64_t *n_steps, void *hip_stream) {
    if (!hs || n <= 0 || n > kMaxBatch || !n_steps) return MPM_E_ARG;
    long long maxn = 0;
    for (int i = 0; i < n; ++i) {
        if (!hs[i] || n_steps[i] < 0) return MPM_E_ARG;
        if (hs[i]->reported_err) return MPM_E_STATE;
        if (hs[i]->L.dim != hs[0]->L.dim || hs[i]->L.shape != hs[0]->L.shape ||
            hs[i]->L.prec != hs[0]->L.prec)
            return MPM_E_UNSUPPORTED;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return MPM_E_ARG;
        maxn = std::max<long long>(maxn, n_steps[i]);
    }
    hipStream_t s = (hipStream_t)hip_stream;
    BatchKey key{};
    key.dim = hs[0]->L.dim;
    key.shape = hs[0]->L.shape;
    key.prec = hs[0]->L.prec;
    WorkTab single;
    make_tables(hs, n, key.tiles, single);
    std::vector<long long> nn(n);
    for (int i = 0; i < n; ++i) nn[i] = n_steps[i];
    launch_arm(single, nn.data(), s);
    if (maxn == 0) return hip_ok(hipGetLastError());
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MPM_E_HIP;
    std::lock_guard<std::mutex> lock(g_batch_mu);
    BatchGraphs &B = g_batch[dev];
    if (!B.cap && hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking) != hipSuccess) return MPM_E_HIP;
    // Replays of the step graphs of this composition (16 steps, then the
    // binary digits of the remainder), captured when the composition differs
    // from the last one seen at that level.
    auto level = [&](int lv) -> int {
        if (!B.valid[lv] || memcmp(&B.key[lv], &key, sizeof(BatchKey)) != 0) {
            B.valid[lv] = false;
            const int st = capture_steps(key.dim, key.shape, key.prec, key.tiles, single, graph_steps(lv),
                                         B.cap, &B.exec[lv]);
            if (st) return st;
            B.key[lv] = key;
            B.valid[lv] = true;
        }
        return hip_ok(hipGraphLaunch(B.exec[lv], s));
    };
    long long left = maxn;
    for (; left >= kGraphSteps; left -= kGraphSteps)
        if (int st = level(0)) return st;
    for (int lv = 1; lv < kGraphLevels; ++lv)
        if (left & graph_steps(lv))
            if (int st = level(lv)) return st;
    return MPM_OK;
}

int mpm_step(mpm_handle *h, int64_t n_steps, void *hip_stream) {
    if (!h) return MPM_E_ARG;
    if (h->reported_err) return MPM_E_STATE;
    hipStream_t s = (hipStream_t)hip_stream;
    mpm_handle *one[1] = {h};
    WorkTab tiles, single;
    make_tables(one, 1, tiles, single);
    const bool to_end = n_steps <= 0;
    if (to_end && !(h->host.t_end > 0)) return MPM_E_ARG;
    // The first call captures the step graphs (16, 8, 4, 2 and 1 steps);
    // every later call, of any step count, is graph replays only.  The
    // kernels read the per-step state from the device descriptor, so the
    // graphs are reusable.
    if (!h->gexec[0]) {
        if (!h->cap && hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) return MPM_E_HIP;
        for (int lv = 0; lv < kGraphLevels; ++lv) {
            const int st = capture_steps(h->L.dim, h->L.shape, h->L.prec, tiles, single, graph_steps(lv), h->cap,
                                         &h->gexec[lv]);
            if (st) {
                for (int j = 0; j < kGraphLevels; ++j)
                    if (h->gexec[j]) { (void)hipGraphExecDestroy(h->gexec[j]); h->gexec[j] = nullptr; }
                return st;
            }
        }
    }
    const long long armed = to_end ? (1LL << 60) : n_steps;
    launch_arm(single, &armed, s);
    if (to_end) {
        for (;;) {
            for (int r = 0; r < 4; ++r)
                if (hipGraphLaunch(h->gexec[0], s) != hipSuccess) return MPM_E_HIP;
            ProbDev cur;
            if (read_dynamic(h, &cur, s)) return MPM_E_HIP;
            if (!cur.active) break;
        }
        return MPM_OK;
    }
    long long left = n_steps;
    for (; left >= kGraphSteps; left -= kGraphSteps)
        if (hipGraphLaunch(h->gexec[0], s) != hipSuccess) return MPM_E_HIP;
    for (int lv = 1; lv < kGraphLevels; ++lv)
        if (left & graph_steps(lv))
            if (hipGraphLaunch(h->gexec[lv], s) != hipSuccess) return MPM_E_HIP;
    return MPM_OK;
}

int mpm_status(mpm_handle *h, double *t, double *dt_next, double *dt_last, int64_t *step,
               double conserved[6], void *hip_stream) {
    if (!h) return MPM_E_ARG;
    if (conserved) launch_conserved(h->dev, (hipStream_t)hip_stream);
    ProbDev cur;
    if (read_dynamic(h, &cur, (hipStream_t)hip_stream)) return MPM_E_HIP;
    if (t) *t = cur.t;
    if (dt_next) *dt_next = cur.dt;
    if (dt_last) *dt_last = cur.dt_last;
    if (step) *step = cur.step;
    if (conserved) for (int c = 0; c < 6; ++c) conserved[c] = cur.cons[c];
    const int e = err_code(cur.err);
    if (e) h->reported_err = 1;
    return e;
}

int mpm_counters(mpm_handle *h, uint64_t counters[4], void *hip_stream) {
    if (!h || !counters) return MPM_E_ARG;
    ProbDev cur;
    if (read_dynamic(h, &cur, (hipStream_t)hip_stream)) return MPM_E_HIP;
    for (int c = 0; c < 4; ++c) counters[c] = cur.diag[c];
    return MPM_OK;
}

int mpm_read_fields(mpm_handle *h, uint32_t field_mask, double *const *host_out, void *hip_stream) {
    if (!h || (field_mask && !host_out) || (field_mask >> 10)) return MPM_E_ARG;
    ProbDev cur;
    if (read_dynamic(h, &cur, (hipStream_t)hip_stream)) return MPM_E_HIP;
    const Layout &L = h->L;
    const long long np = L.np;
    const int dim = L.dim, par = cur.parity;
    std::vector<uint32_t> ids((size_t)std::max<long long>(np, 1));
    if (np && hipMemcpy(ids.data(), h->host.pid[par], (size_t)np * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return MPM_E_HIP;
    std::vector<char> raw((size_t)std::max<long long>(np, 1) * 8);
    auto fetch = [&](int f, std::vector<double> &dst) -> int {
        dst.assign((size_t)np, 0.0);
        if (!np) return MPM_OK;
        if (hipMemcpy(raw.data(), h->host.part[par][f], (size_t)np * L.real_sz, hipMemcpyDeviceToHost) != hipSuccess)
            return MPM_E_HIP;
        for (long long k = 0; k < np; ++k)
            dst[ids[k]] = L.real_sz == 8 ? ((double *)raw.data())[k] : (double)((float *)raw.data())[k];
        return MPM_OK;
    };
    std::vector<double> a, b, c2;
    int j = 0;
    for (int f = 0; f < 10; ++f) {
        if (!(field_mask & (1u << f))) continue;
        double *o = host_out[j++];
        if (!o) return MPM_E_ARG;
        switch (f) {
        case MPM_F_X: case MPM_F_V:
            for (int ax = 0; ax < dim; ++ax) {
                if (fetch((f == MPM_F_X ? PF_X : PF_V) + ax, a)) return MPM_E_HIP;
                memcpy(o + ax * np, a.data(), (size_t)np * 8);
            }
            break;
        case MPM_F_M: if (fetch(PF_M, a)) return MPM_E_HIP; memcpy(o, a.data(), (size_t)np * 8); break;
        case MPM_F_RHO: if (fetch(PF_RHO, a)) return MPM_E_HIP; memcpy(o, a.data(), (size_t)np * 8); break;
        case MPM_F_E: if (fetch(PF_E, a)) return MPM_E_HIP; memcpy(o, a.data(), (size_t)np * 8); break;
        case MPM_F_P:
            if (fetch(PF_RHO, a) || fetch(PF_E, b)) return MPM_E_HIP;
            for (long long k = 0; k < np; ++k) o[k] = (h->host.gamma - 1.0) * a[k] * b[k];
            break;
        case MPM_F_Q: {
            if (fetch(PF_RHO, a) || fetch(PF_E, b)) return MPM_E_HIP;
            std::vector<double> D;
            if (fetch(PF_D, D)) return MPM_E_HIP;
            const double g = h->host.gamma, hh = h->host.h;
            for (long long k = 0; k < np; ++k) {
                double q = 0;
                if (D[k] < 0) {
                    const double p = (g - 1.0) * a[k] * b[k];
                    const double cc = g * p / a[k] > 0 ? sqrt(g * p / a[k]) : 0.0;
                    if (h->host.av_form == MPM_AV_BOOK)
                        q = h->host.c0 * a[k] * (hh * D[k]) * (hh * D[k]) - h->host.c1 * a[k] * hh * cc * D[k];
                    else
                        q = h->host.c0 * (a[k] * hh * D[k]) * (a[k] * hh * D[k]) - h->host.c1 * hh * cc * D[k];
                }
                o[k] = q;
            }
            break;
        }
        case MPM_F_G:
            // the full gradient is written by the last step of each run
            if (cur.g_step != cur.step && !err_code(cur.err)) return MPM_E_STATE;
            for (int cc = 0; cc < dim * dim; ++cc) {
                if (fetch(PF_G + cc, a)) return MPM_E_HIP;
                memcpy(o + cc * np, a.data(), (size_t)np * 8);
            }
            break;
        case MPM_F_VOL:
            if (fetch(PF_M, a) || fetch(PF_RHO, b)) return MPM_E_HIP;
            for (long long k = 0; k < np; ++k) o[k] = a[k] / b[k];
            break;
        case MPM_F_ID:
            for (long long k = 0; k < np; ++k) o[ids[k]] = (double)ids[k];
            break;
        }
    }
    const int e = err_code(cur.err);
    if (e) h->reported_err = 1;
    return e;
}

int mpm_read_grid(mpm_handle *h, int32_t which, double *host_out, void *hip_stream) {
    if (!h || !host_out || which < MPM_G_M || which > MPM_G_VOLPROJ) return MPM_E_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    const int ncomp = (which == MPM_G_M || which >= MPM_G_FLAGS) ? 1 : h->L.dim;
    const size_t bytes = (size_t)ncomp * h->L.nnodes * 8;
    double *tmp = nullptr;
    if (hipMalloc(&tmp, bytes) != hipSuccess) return MPM_E_HIP;
    launch_grid_diag(h->L.dim, h->L.shape, h->L.prec, h->dev, h->host, which, tmp, s);
    int st = hip_ok(hipGetLastError());
    if (!st) st = hip_ok(hipStreamSynchronize(s));
    if (!st) st = hip_ok(hipMemcpy(host_out, tmp, bytes, hipMemcpyDeviceToHost));
    (void)hipFree(tmp);
    return st;
}

int mpm_read_grid_noalloc(mpm_handle *h, int32_t which, double *host_out, void *hip_stream) {
    if (!h || !host_out || which < MPM_G_M || which > MPM_G_VOLPROJ) return MPM_E_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    const int ncomp = (which == MPM_G_M || which >= MPM_G_FLAGS) ? 1 : h->L.dim;
    const size_t bytes = (size_t)ncomp * h->L.nnodes * 8;
    if (bytes > kScratchBytes) return MPM_E_SCRATCH;
    if (!h->scratch) return MPM_E_STATE;
    // the kernel writes every element of the snapshot: nothing of the last
    // call's contents is read
    launch_grid_diag(h->L.dim, h->L.shape, h->L.prec, h->dev, h->host, which, h->scratch, s);
    int st = hip_ok(hipGetLastError());
    if (!st) st = hip_ok(hipMemcpyAsync(host_out, h->scratch, bytes, hipMemcpyDeviceToHost, s));
    if (!st) st = hip_ok(hipStreamSynchronize(s));
    return st;
}

int mpm_profile_step(mpm_handle *h, int64_t n_steps, double ms_per_sweep[MPM_NUM_SWEEPS], void *hip_stream) {
    if (!h || n_steps <= 0 || !ms_per_sweep) return MPM_E_ARG;
    if (h->reported_err) return MPM_E_STATE;
    hipStream_t s = (hipStream_t)hip_stream;
    mpm_handle *one[1] = {h};
    WorkTab tiles, single;
    make_tables(one, 1, tiles, single);
    const long long armed = n_steps;
    launch_arm(single, &armed, s);
    // Steps are enqueued in batches (events for every sweep of up to kBatch
    // steps), so the device does not wait for the host between steps.
    constexpr int kBatch = 32;
    hipEvent_t ev[kBatch][kSweeps + 1];
    int made = 0, st = MPM_OK;
    for (int b = 0; b < kBatch && !st; ++b)
        for (int i = 0; i <= kSweeps && !st; ++i) {
            st = hip_ok(hipEventCreate(&ev[b][i]));
            if (!st) ++made;
        }
    double acc[kSweeps] = {0};
    for (long long k0 = 0; k0 < n_steps && !st; k0 += kBatch) {
        const int nb = (int)std::min<long long>(kBatch, n_steps - k0);
        for (int b = 0; b < nb && !st; ++b) {
            st = hip_ok(hipEventRecord(ev[b][0], s));
            for (int part = 0; part < kSweeps && !st; ++part) {
                launch_part(h->L.dim, h->L.shape, h->L.prec, part, tiles, single, s);
                st = hip_ok(hipEventRecord(ev[b][part + 1], s));
            }
        }
        if (!st) st = hip_ok(hipEventSynchronize(ev[nb - 1][kSweeps]));
        for (int b = 0; b < nb && !st; ++b)
            for (int part = 0; part < kSweeps && !st; ++part) {
                float ms = 0;
                st = hip_ok(hipEventElapsedTime(&ms, ev[b][part], ev[b][part + 1]));
                acc[part] += ms;
            }
    }
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i / (kSweeps + 1)][i % (kSweeps + 1)]);
    if (st) return st;
    for (int part = 0; part < kSweeps; ++part) ms_per_sweep[part] = acc[part] / (double)n_steps;
    return MPM_OK;
}

int mpm_grid_shape(const mpm_handle *h, int32_t nodes[3]) {
    if (!h || !nodes) return MPM_E_ARG;
    for (int a = 0; a < 3; ++a) nodes[a] = h->L.nn[a];
    return MPM_OK;
}

int mpm_destroy(mpm_handle *h) {
    if (!h) return MPM_E_ARG;
    for (int lv = 0; lv < kGraphLevels; ++lv)
        if (h->gexec[lv]) (void)hipGraphExecDestroy(h->gexec[lv]);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    free(h);
    return MPM_OK;
}

}  // extern "C"
