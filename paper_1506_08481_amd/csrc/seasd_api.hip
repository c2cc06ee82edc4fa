// seasd_api.hip - the C ABI declared in include/seasd.h: handle, configuration,
// workspace, the mobility product and the GMRES far-field solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/seasd.h"
#include "seasd_internal.h"
#include "seasd_learn.h"
#include "seasd_math.h"

using namespace seasd;


struct seasd_handle_s {
    int device = 0;
    seasd_config cfg{};
    bool have_cfg = false;
    // product workspace
    DevBuf bin_of, counts, start, fill, perm, amax, err, sp, sfrac, sa, sx, ybuf, rgrid, spec, twiddle;
    DevBuf rgrid2, spec2;   // hybrid size approach: the k-space Laplacian fields
    DevBuf ncount, nstats, list, total, wrec, scan_tmp;
    int cap = 64;             // neighbour-list slots per sphere, grown on demand
    int pair_group = 1;       // lanes per sphere of the pair sum chosen for the held geometry
    int static_pair_group = 1;   // the same choice for the allocation-free product
    int64_t geom_n = -1;      // spheres in the geometry currently held in the workspace
    int twiddle_M = 0;
    // solver workspace
    DevBuf w, z, u, r, bred, hdev, partial, blocks, inv, coef, singular, one_pos, one_rad, one_x, one_y;
    DeviceGmres gm;
    // near-field / far-field solve: 6N vectors, diagonal-block inverses of
    // R + lambda I, the near-field GMRES
    DevBuf mv6, mw6, mp6, mu6, mt6, rinv, mbad;
    DevBuf ic_rows, ic_lrp, ic_lcol, ic_lval, ic_urp, ic_ucol, ic_uval, ic_linv;   // incomplete factor
    DeviceGmres gm_near;
    // block-diagonal fit cache: (a_min, a_max, grid, P, m, xi, rc_factor, eta, precision, cell A[9])
    double pc_key[18] = {0};
    bool pc_valid = false;
    double pc_amax = 0.0;
    // learned preconditioner
    seasd_net net = nullptr;       // attached (not owned)
    seasd_net own_net = nullptr;   // loaded by seasd_precond_load
    DevBuf inv2, bad, lx0, lg, lb, lax, lres;
    PhaseTimer timer;
    hipStream_t last_stream = nullptr;
    // list statistics read back after each neighbour-list build: pinned host
    // words and the event that marks their copy
    unsigned long long* ns_host = nullptr;
    hipEvent_t ev_stats = nullptr;
    // second stream of a product: the neighbour list and the pair sum run on
    // it beside the window records, spreading and transforms (fork after the
    // binning, join before the gather)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // SEASD_MIXED: set while a solve's Arnoldi step runs its product
    bool step_fp32 = false;
};

static int hip_ok(hipError_t e) { return e == hipSuccess ? 0 : SEASD_E_HIP; }

// A restart cycle of a SEASD_MIXED solve ends once its residual estimate has
// fallen by this factor: the FP32 product's relative error (below 1e-6 at the
// configurations the autotuner picks) times the preconditioned system's
// condition number bounds what one cycle can gain on the FP64 residual.
constexpr double kMixedCycleRtol = 1e-5;

// The same operator with the mobility products it queues in FP32 (for the
// Arnoldi steps of a SEASD_MIXED solve); every other step stays as it is.
template <typename Op>
static std::function<int(const double*, double*)> fp32_steps(seasd_handle h, Op& op) {
    return [h, &op](const double* in, double* out) -> int {
        h->step_fp32 = true;
        const int e = op(in, out);
        h->step_fp32 = false;
        return e;
    };
}

extern "C" const char* seasd_error_string(int32_t code) {
    switch (code) {
        case SEASD_OK: return "success";
        case SEASD_E_INVALID_ARG: return "invalid argument";
        case SEASD_E_NONFINITE: return "non-finite position, radius or moment";
        case SEASD_E_OVERLAP: return "overlapping spheres (r < a_i + a_j)";
        case SEASD_E_CUTOFF: return "window or cut-off does not fit the cell";
        case SEASD_E_SINGULAR: return "singular preconditioner block";
        case SEASD_E_HIP: return "HIP runtime error";
        case SEASD_E_NOMEM: return "device allocation failed";
        case SEASD_E_UNSUPPORTED: return "unsupported request (cell shape, unequal grids or size approach)";
        case SEASD_E_SCRATCH: return "request exceeds the static workspace of the allocation-free product";
        case SEASD_E_FORMAT: return "weights file missing, mismatched or failing its checksum";
        case SEASD_W_NOT_CONVERGED: return "solve did not reach the tolerance";
        case SEASD_W_PRECOND_FALLBACK: return "learned preconditioner rejected, block-diagonal used";
        default: return "unknown code";
    }
}

extern "C" int seasd_default_config(seasd_config* c) {
    if (!c) return SEASD_E_INVALID_ARG;
    std::memset(c, 0, sizeof(*c));
    c->grid[0] = c->grid[1] = c->grid[2] = 64;
    c->P = 16;
    c->size_approach = SEASD_SIZE_REAL;
    c->m = 0.0;
    c->xi = 0.5;
    c->rc_factor = 4.0;
    c->eta = 1.0;
    c->precision = SEASD_FP64;
    c->parts = SEASD_PARTS_ALL;
    c->compressible = 1;
    c->checks = 1;
    c->tol = 1e-6;
    c->max_iter = 1000;
    c->restart = 50;
    c->precond = SEASD_PRECOND_BLOCKDIAG;
    return SEASD_OK;
}

// Workspace of the allocation-free product (seasd_mobility_apply_static):
// one array per GPU, held until the process ends. Host code never uses the
// array's name as an address: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) when a handle is created
// there, and kept here.
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[SEASD_STATIC_SCRATCH_BYTES];
static void* g_scratch_ptr[kMaxDevices] = {nullptr};
static std::mutex g_scratch_mu;

static int static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return SEASD_E_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return SEASD_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return SEASD_E_HIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    hipSetDevice(prev);
    if (e != hipSuccess || !p) return SEASD_E_HIP;
    g_scratch_ptr[device] = p;
    return SEASD_OK;
}

extern "C" int seasd_create(seasd_handle* out, int32_t device) {
    if (!out) return SEASD_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SEASD_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return SEASD_E_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SEASD_E_HIP;
    if (int rc = static_scratch_setup(device)) return rc;
    auto* h = new seasd_handle_s();
    h->device = device;
    seasd_default_config(&h->cfg);
    h->have_cfg = true;
    *out = h;
    return SEASD_OK;
}

extern "C" int seasd_destroy(seasd_handle h) {
    if (!h) return SEASD_OK;
    hipSetDevice(h->device);
    DevBuf* bufs[] = {&h->bin_of, &h->counts, &h->start, &h->fill, &h->perm, &h->amax, &h->err,
                      &h->sp, &h->sfrac, &h->sa, &h->sx, &h->ybuf, &h->rgrid, &h->spec, &h->rgrid2, &h->spec2, &h->twiddle,
                      &h->ncount, &h->nstats, &h->list, &h->total, &h->wrec, &h->scan_tmp,
                      &h->w, &h->z, &h->u, &h->r, &h->bred, &h->hdev, &h->partial, &h->blocks,
                      &h->inv, &h->coef, &h->singular, &h->one_pos, &h->one_rad, &h->one_x, &h->one_y,
                      &h->inv2, &h->bad, &h->lx0, &h->lg, &h->lb, &h->lax, &h->lres,
                      &h->mv6, &h->mw6, &h->mp6, &h->mu6, &h->mt6, &h->rinv, &h->mbad, &h->ic_rows,
                      &h->ic_lrp, &h->ic_lcol, &h->ic_lval, &h->ic_urp, &h->ic_ucol, &h->ic_uval, &h->ic_linv};
    for (DevBuf* b : bufs) b->release();
    if (h->ns_host) hipHostFree(h->ns_host);
    if (h->ev_stats) hipEventDestroy(h->ev_stats);
    if (h->side) hipStreamDestroy(h->side);
    if (h->ev_fork) hipEventDestroy(h->ev_fork);
    if (h->ev_join) hipEventDestroy(h->ev_join);
    if (h->own_net) seasd_net_destroy(h->own_net);
    h->timer.destroy();
    h->gm.release();
    h->gm_near.release();
    delete h;
    return SEASD_OK;
}

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

extern "C" int seasd_set_config(seasd_handle h, const seasd_config* c) {
    if (!h || !c) return SEASD_E_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        if (!pow2(c->grid[d]) || c->grid[d] < 8 || c->grid[d] > 256) return SEASD_E_INVALID_ARG;
    if (c->P < 4 || c->P > 32 || c->P > c->grid[0]) return SEASD_E_INVALID_ARG;
    if (!(std::isfinite(c->m)) || !(c->xi > 0.0) || !std::isfinite(c->xi)) return SEASD_E_INVALID_ARG;
    if (!(c->rc_factor > 1.0) || !std::isfinite(c->rc_factor)) return SEASD_E_INVALID_ARG;
    if (!(c->eta > 0.0) || !std::isfinite(c->eta)) return SEASD_E_INVALID_ARG;
    if (c->precision != SEASD_FP64 && c->precision != SEASD_FP32 && c->precision != SEASD_MIXED)
        return SEASD_E_INVALID_ARG;
    if (c->parts < 0 || c->parts > SEASD_PARTS_ALL) return SEASD_E_INVALID_ARG;
    if (c->restart < 1 || c->restart > 200 || c->max_iter < 1) return SEASD_E_INVALID_ARG;
    if (!(c->tol > 0.0)) return SEASD_E_INVALID_ARG;
    if (c->precond != SEASD_PRECOND_NONE && c->precond != SEASD_PRECOND_BLOCKDIAG &&
        c->precond != SEASD_PRECOND_LEARNED_GUESS)
        return SEASD_E_INVALID_ARG;
    if (c->size_approach < 0 || c->size_approach > 2) return SEASD_E_INVALID_ARG;
    // valid requests this build does not carry out: unequal grids and the
    // wave-space size approach
    if (c->grid[1] != c->grid[0] || c->grid[2] != c->grid[0]) return SEASD_E_UNSUPPORTED;
    if (c->size_approach == SEASD_SIZE_WAVE) return SEASD_E_UNSUPPORTED;
    h->cfg = *c;
    h->have_cfg = true;
    return SEASD_OK;
}

// Lattice vectors (host box[9] = a1, a2, a3) into a Cell. Accepted shapes:
// a1 = (a1x, 0, 0), a2 = (a2x, a2y, 0), a3 = (0, 0, a3z), positive diagonal,
// |a2x| <= a1x; off-pattern entries below 1e-12 of the largest length count as
// zero.
static int parse_cell(const double* box, Cell* cell) {
    if (!box) return SEASD_E_INVALID_ARG;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(box[i])) return SEASD_E_INVALID_ARG;
    const double a1x = box[0], a2x = box[3], a2y = box[4], a3z = box[8];
    if (!(a1x > 0.0) || !(a2y > 0.0) || !(a3z > 0.0)) return SEASD_E_INVALID_ARG;
    const double scale = std::max(std::max(a1x, a2y), std::max(a3z, std::fabs(a2x)));
    const double tol = 1e-12 * scale;
    const int zero_idx[5] = {1, 2, 5, 6, 7};   // a1y, a1z, a2z, a3x, a3y
    for (int k : zero_idx)
        if (std::fabs(box[k]) > tol) return SEASD_E_UNSUPPORTED;
    if (std::fabs(a2x) > a1x * (1.0 + 1e-12)) return SEASD_E_UNSUPPORTED;
    Cell c{};
    // A row-major, columns a1 a2 a3
    c.a[0] = a1x;
    c.a[1] = a2x;
    c.a[4] = a2y;
    c.a[8] = a3z;
    c.ainv[0] = 1.0 / a1x;
    c.ainv[1] = -a2x / (a1x * a2y);
    c.ainv[4] = 1.0 / a2y;
    c.ainv[8] = 1.0 / a3z;
    for (int d = 0; d < 3; ++d) {
        const double* row = c.ainv + 3 * d;
        c.height[d] = 1.0 / std::sqrt(row[0] * row[0] + row[1] * row[1] + row[2] * row[2]);
    }
    c.volume = a1x * a2y * a3z;
    *cell = c;
    return SEASD_OK;
}

static double min_height(const Cell& c) { return std::min(c.height[0], std::min(c.height[1], c.height[2])); }

// product workspace for n spheres on the configured grid (bins are the 8^3
// spreading tiles)
static int ensure_product_ws(seasd_handle h, int64_t n, hipStream_t st) {
    const int M = h->cfg.grid[0];
    const int nb = M / 8;
    const size_t nbins = (size_t)nb * nb * nb;
    const size_t R = h->cfg.precision == SEASD_FP32 ? 4 : 8;
    int rc = 0;
    rc |= h->bin_of.ensure(sizeof(int) * n);
    rc |= h->counts.ensure(sizeof(int) * nbins);
    rc |= h->start.ensure(sizeof(int) * (nbins + 1));
    rc |= h->fill.ensure(sizeof(int) * nbins);
    rc |= h->perm.ensure(sizeof(int) * n);
    rc |= h->amax.ensure(sizeof(unsigned long long));
    rc |= h->err.ensure(sizeof(int));
    rc |= h->sp.ensure(sizeof(double) * 3 * n);
    rc |= h->sfrac.ensure(sizeof(double) * 3 * n);
    rc |= h->sa.ensure(sizeof(double) * n);
    rc |= h->sx.ensure(sizeof(double) * 12 * n);
    rc |= h->ybuf.ensure(sizeof(double) * 12 * n);
    rc |= h->ncount.ensure(sizeof(int) * n);
    rc |= h->nstats.ensure(2 * sizeof(unsigned long long));
    rc |= h->scan_tmp.ensure(sizeof(int) * (((size_t)std::max<int64_t>(n, (int64_t)nbins) + 2047) / 2048 + 2));
    rc |= h->wrec.ensure(R * rec_stride(h->cfg.P) * n);   // padded window records
    if (h->cfg.parts & SEASD_PARTS_WAVE) {
        rc |= h->rgrid.ensure(R * 4 * (size_t)M * M * M);
        rc |= h->spec.ensure(R * 4 * (size_t)M * M * M);
        if (h->cfg.size_approach == SEASD_SIZE_HYBRID) {   // the k-space Laplacian fields
            rc |= h->rgrid2.ensure(R * 4 * (size_t)M * M * M);
            rc |= h->spec2.ensure(R * 4 * (size_t)M * M * M);
        }
    } else {
        rc |= h->rgrid.ensure(R * 4);
    }
    rc |= h->twiddle.ensure(sizeof(double) * 2 * M);
    if (rc) return SEASD_E_NOMEM;
    if (h->twiddle_M != M) {
        if (launch_twiddles(M, h->twiddle.as<double>(), st)) return SEASD_E_HIP;
        h->twiddle_M = M;
    }
    return SEASD_OK;
}

static void fill_args(seasd_handle h, ApplyArgs& A, int64_t n, const double* pos, const double* radius,
                      const Cell& cell, const double* x, double* y, bool checks, int compressible) {
    const seasd_config& c = h->cfg;
    A = ApplyArgs{};
    A.n = n;
    A.pos = pos;
    A.radius = radius;
    A.x = x;
    A.y = y;
    A.cell = cell;
    const int M = c.grid[0];
    A.M = M;
    A.P = c.P;
    A.nb = M / 8;
    for (int d = 0; d < 3; ++d) A.reach_per_len[d] = A.nb / cell.height[d];
    A.xi = c.xi;
    A.rc_factor = c.rc_factor;
    A.inv_eta = 1.0 / c.eta;
    // window on the fractional grid (Sec. 3.1, eqs. shape and theta-param)
    const double m = c.m > 0.0 ? c.m : std::sqrt(kPi * c.P);
    const double beta = 2.0 * m * m / ((double)c.P * c.P);
    const double* ai = cell.ainv;
    // J = M A^-1, Q = J^T J, g = beta J^T u
    const double J00 = M * ai[0], J01 = M * ai[1], J11 = M * ai[4], J22 = M * ai[8];
    const double Qxx = J00 * J00, Qxy = J00 * J01, Qyy = J01 * J01 + J11 * J11, Qzz = J22 * J22;
    WinGeom& w = A.win;
    w.beta = beta;
    w.Gxx = beta * J00;
    w.Gyx = beta * J01;
    w.Gyy = beta * J11;
    w.Gzz = beta * J22;
    w.Qxx = beta * (Qxx - Qzz);
    w.Qxy = beta * Qxy;
    w.Qyy = beta * (Qyy - Qzz);
    w.bq = beta * (Qxx + Qyy + Qzz);
    w.bz = beta * Qzz;
    const double qtol = 1e-12 * beta * Qzz;
    w.sheared = std::fabs(w.Qxx) > qtol || std::fabs(w.Qxy) > qtol || std::fabs(w.Qyy) > qtol;
    w.cwv = std::pow(beta / kPi, 1.5);
    w.cw = w.cwv * (double)M * M * M / cell.volume;
    A.kdeconv = 2.0 * kPi * kPi / (beta * (double)M * M);
    A.parts = c.parts;
    A.compressible = compressible;
    A.checks = checks ? 1 : 0;
    // SEASD_MIXED: FP32 only for the Arnoldi steps of a far-field solve (the
    // FP64 workspace holds the FP32 grids and records as well)
    A.fp32 = c.precision == SEASD_FP32 || (c.precision == SEASD_MIXED && h->step_fp32);
    A.bin_of = h->bin_of.as<int>();
    A.counts = h->counts.as<int>();
    A.start = h->start.as<int>();
    A.fill = h->fill.as<int>();
    A.perm = h->perm.as<int>();
    A.scan_tmp = h->scan_tmp.as<int>();
    A.ncount = h->ncount.as<int>();
    A.nstats = h->nstats.as<unsigned long long>();
    A.pair_group = h->pair_group;
    A.cap = h->cap;
    A.list = h->list.as<int2>();
    A.amax_bits = h->amax.as<unsigned long long>();
    A.err = h->err.as<int>();
    A.sp = h->sp.as<double>();
    A.st = h->sfrac.as<double>();
    A.sa = h->sa.as<double>();
    A.sx = h->sx.as<double>();
    A.ybuf = h->ybuf.as<double>();
    A.wrec = h->wrec.p;
    A.rgrid = h->rgrid.p;
    A.spec = h->spec.p;
    A.hybrid = c.size_approach == SEASD_SIZE_HYBRID && (c.parts & SEASD_PARTS_WAVE);
    A.rgrid2 = A.hybrid ? h->rgrid2.p : nullptr;
    A.spec2 = A.hybrid ? h->spec2.p : nullptr;
    A.twiddle = h->twiddle.as<double>();
}

// The product's second stream (created once per handle), forked from st.
static int fork_side(seasd_handle h, hipStream_t st) {
    // each object is created once; one that failed is tried again on the next call
    if (!h->ev_fork && hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess) {
        h->ev_fork = nullptr;
        return SEASD_E_HIP;
    }
    if (!h->ev_join && hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
        h->ev_join = nullptr;
        return SEASD_E_HIP;
    }
    // default priority (as every stream here); ordered against st by events only
    if (!h->side && hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
        h->side = nullptr;
        return SEASD_E_HIP;
    }
    if (hipEventRecord(h->ev_fork, st) != hipSuccess || hipStreamWaitEvent(h->side, h->ev_fork, 0) != hipSuccess)
        return SEASD_E_HIP;
    return SEASD_OK;
}

static int join_side(seasd_handle h, hipStream_t st) {
    h->timer.end(h->side);
    if (hipEventRecord(h->ev_join, h->side) != hipSuccess || hipStreamWaitEvent(st, h->ev_join, 0) != hipSuccess)
        return SEASD_E_HIP;
    return SEASD_OK;
}

// Queue one product. With reuse_geometry the binning and neighbour list of the
// previous call (same spheres) are kept and only the moments are re-binned;
// then the pair sum runs on the handle's second stream beside the wave-space
// part and the gather waits for both (N = 1e4 bidisperse solve at 128^3: 0.146
// -> 0.138 s). A product that builds its geometry runs every phase on st: the
// list and the pair sum beside spreading gained 1.3 % but share spreading's
// CUs, so its time no longer measures the kernel alone.
// Building a geometry waits once for the list statistics (one 16-byte copy
// into pinned memory) to confirm the list fit its slots and to choose the pair
// sum's lanes per sphere for the next products; the pair sum and the wave part
// are queued before that wait. Everything else is queued without
// synchronisation.
static int queue_apply(seasd_handle h, int64_t n, const double* pos, const double* radius, const Cell& L,
                       const double* x, double* y, hipStream_t st, bool checks, bool reuse_geometry = false,
                       int compressible = -1) {
    if (compressible < 0) compressible = h->cfg.compressible;
    int rc = ensure_product_ws(h, n, st);
    if (rc) return rc;
    ApplyArgs A;
    fill_args(h, A, n, pos, radius, L, x, y, checks, compressible);
    if (checks && hipMemsetAsync(A.err, 0, sizeof(int), st) != hipSuccess) return SEASD_E_HIP;
    h->timer.start_product();
    if (reuse_geometry && h->geom_n == n) {
        if (launch_moments(A, st)) return SEASD_E_HIP;
        if ((rc = fork_side(h, st))) return rc;
        if (launch_pair(A, h->side, &h->timer) || launch_wave(A, st, &h->timer)) return SEASD_E_HIP;
        if ((rc = join_side(h, st))) return rc;
        if (launch_gather(A, st, &h->timer)) return SEASD_E_HIP;
    } else {
        h->geom_n = -1;
        if (launch_geometry(A, st, &h->timer)) return SEASD_E_HIP;
        if (!h->ns_host) {
            if (hipHostMalloc((void**)&h->ns_host, 2 * sizeof(unsigned long long)) != hipSuccess) {
                h->ns_host = nullptr;
                return SEASD_E_NOMEM;
            }
            if (hipEventCreateWithFlags(&h->ev_stats, hipEventDisableTiming) != hipSuccess) return SEASD_E_HIP;
        }
        bool queued = false;
        for (int attempt = 0; attempt < 3; ++attempt) {
            if (h->list.ensure(sizeof(int2) * (size_t)h->cap * n)) return SEASD_E_NOMEM;
            A.list = h->list.as<int2>();
            A.cap = h->cap;
            if (attempt > 0 && hipMemsetAsync(A.nstats, 0, 2 * sizeof(unsigned long long), st) != hipSuccess)
                return SEASD_E_HIP;
            if (launch_pairlist(A, st)) return SEASD_E_HIP;
            if (!(A.parts & kPartsReal)) break;
            if (hipMemcpyAsync(h->ns_host, A.nstats, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipEventRecord(h->ev_stats, st) != hipSuccess)
                return SEASD_E_HIP;
            // The pair sum (lanes per sphere as chosen for the previous
            // geometry: the choice changes the speed, not the result) and the
            // wave part are queued before waiting for the statistics, so the
            // GPU keeps working meanwhile; a list that overflowed its slots is
            // built again and the pair sum repeated before the gather.
            if (launch_pair(A, st, &h->timer)) return SEASD_E_HIP;
            if (!queued) {
                if (launch_wave(A, st, &h->timer)) return SEASD_E_HIP;
                queued = true;
            }
            if (hipEventSynchronize(h->ev_stats) != hipSuccess) return SEASD_E_HIP;
            const unsigned long long mxl = h->ns_host[0], sum = h->ns_host[1];
            // lists much longer than the average (spheres of very different
            // sizes): one thread per sphere would leave most lanes waiting for
            // the longest list of their wavefront
            h->pair_group = ((double)mxl > kPairImbalance * (double)sum / (double)n) ? 64 : 1;
            A.pair_group = h->pair_group;
            const int mx = (int)mxl;
            if (mx <= h->cap) break;
            h->cap = mx + mx / 4 + 8;     // rare: grow and list again
        }
        h->geom_n = n;
        if (!queued) {
            if (launch_pair(A, st, &h->timer) || launch_wave(A, st, &h->timer)) return SEASD_E_HIP;
        }
        if (launch_gather(A, st, &h->timer)) return SEASD_E_HIP;
    }
    h->last_stream = st;
    return SEASD_OK;
}

static int read_err(seasd_handle h, hipStream_t st) {
    int e = 0;
    if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
    if (hipMemcpy(&e, h->err.p, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SEASD_E_HIP;
    if (e & kErrNonfinite) return SEASD_E_NONFINITE;
    if (e & kErrOverlap) return SEASD_E_OVERLAP;
    if (e & kErrCutoff) return SEASD_E_CUTOFF;
    return SEASD_OK;
}

extern "C" int seasd_mobility_apply(seasd_handle h, int64_t n, const double* pos, const double* radius,
                                    const double* box, const double* x, double* y, void* stream) {
    if (!h || n < 1 || n > (int64_t)1 << 28 || !pos || !radius || !x || !y) return SEASD_E_INVALID_ARG;
    if (x == y) return SEASD_E_INVALID_ARG;
    Cell L;
    int rc = parse_cell(box, &L);
    if (rc) return rc;
    if (hipSetDevice(h->device) != hipSuccess) return SEASD_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    rc = queue_apply(h, n, pos, radius, L, x, y, st, h->cfg.checks != 0);
    if (rc) return rc;
    if (h->cfg.checks) return read_err(h, st);
    return SEASD_OK;
}

// Bump allocation of 256-byte aligned pieces from the static workspace.
struct ScratchCarve {
    char* base;
    size_t off, cap;
    bool ok = true;
    template <typename T>
    T* take(size_t count) {
        const size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
        if (off + bytes > cap) {
            ok = false;
            return nullptr;
        }
        T* p = reinterpret_cast<T*>(base + off);
        off += bytes;
        return p;
    }
};

extern "C" int seasd_mobility_apply_static(seasd_handle h, int64_t n, const double* pos, const double* radius,
                                           const double* box, const double* x, double* y, void* stream) {
    if (!h || n < 1 || n > (int64_t)1 << 28 || !pos || !radius || !x || !y) return SEASD_E_INVALID_ARG;
    if (x == y) return SEASD_E_INVALID_ARG;
    Cell L;
    int rc = parse_cell(box, &L);
    if (rc) return rc;
    if (h->device < 0 || h->device >= kMaxDevices || !g_scratch_ptr[h->device]) return SEASD_E_HIP;
    if (hipSetDevice(h->device) != hipSuccess) return SEASD_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    const seasd_config& c = h->cfg;
    const int M = c.grid[0];
    const int nb = M / 8;
    const size_t nbins = (size_t)nb * nb * nb;
    const size_t R = c.precision == SEASD_FP32 ? 4 : 8;
    const bool wave = (c.parts & SEASD_PARTS_WAVE) != 0;
    const bool hyb = wave && c.size_approach == SEASD_SIZE_HYBRID;
    const size_t g = wave ? R * 4 * (size_t)M * M * M : R * 4;

    // every piece of the product workspace, in the order ensure_product_ws lists them
    ScratchCarve cv{static_cast<char*>(g_scratch_ptr[h->device]), 0, (size_t)SEASD_STATIC_SCRATCH_BYTES};
    ApplyArgs A;
    fill_args(h, A, n, pos, radius, L, x, y, c.checks != 0, c.compressible);
    A.bin_of = cv.take<int>(n);
    A.counts = cv.take<int>(nbins);
    A.start = cv.take<int>(nbins + 1);
    A.fill = cv.take<int>(nbins);
    A.perm = cv.take<int>(n);
    A.amax_bits = cv.take<unsigned long long>(1);
    A.err = cv.take<int>(1);
    A.sp = cv.take<double>(3 * n);
    A.st = cv.take<double>(3 * n);
    A.sa = cv.take<double>(n);
    A.sx = cv.take<double>(12 * n);
    A.ybuf = cv.take<double>(12 * n);
    A.ncount = cv.take<int>(n);
    A.nstats = cv.take<unsigned long long>(2);
    A.scan_tmp = cv.take<int>((std::max<size_t>((size_t)n, nbins) + 2047) / 2048 + 2);
    A.wrec = cv.take<char>(R * rec_stride(c.P) * n);
    A.rgrid = cv.take<char>(g);
    A.spec = wave ? cv.take<char>(g) : nullptr;
    A.rgrid2 = hyb ? cv.take<char>(g) : nullptr;
    A.spec2 = hyb ? cv.take<char>(g) : nullptr;
    double* tw = cv.take<double>(2 * (size_t)M);
    A.twiddle = tw;
    if (!cv.ok) return SEASD_E_SCRATCH;
    // the neighbour list takes the rest
    const size_t room = (cv.cap - cv.off) / (sizeof(int2) * (size_t)n);
    A.cap = (int)std::min<size_t>(room, 4096);
    if (A.cap < 1) return SEASD_E_SCRATCH;
    A.list = cv.take<int2>((size_t)A.cap * n);
    if (!cv.ok) return SEASD_E_SCRATCH;
    A.pair_group = h->static_pair_group;

    PhaseTimer off;
    if (launch_twiddles(M, tw, st)) return SEASD_E_HIP;
    if (launch_clear_ints(1, A.err, st)) return SEASD_E_HIP;
    if (launch_geometry(A, st, &off)) return SEASD_E_HIP;
    if (launch_pairlist(A, st)) return SEASD_E_HIP;
    unsigned long long ns[2] = {0, 0};
    const bool real = (A.parts & kPartsReal) != 0;
    if (real && hipMemcpyAsync(ns, A.nstats, sizeof(ns), hipMemcpyDeviceToHost, st) != hipSuccess) return SEASD_E_HIP;
    if (launch_pair(A, st, &off) || launch_wave(A, st, &off)) return SEASD_E_HIP;
    if (real) {
        if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
        if (ns[0] > (unsigned long long)A.cap) return SEASD_E_SCRATCH;
        // lanes per sphere of the pair sum for the next call (speed only)
        h->static_pair_group = ((double)ns[0] > kPairImbalance * (double)ns[1] / (double)n) ? 64 : 1;
    }
    if (launch_gather(A, st, &off)) return SEASD_E_HIP;
    if (c.checks) {
        int e = 0;
        if (hipMemcpyAsync(&e, A.err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SEASD_E_HIP;
        if (e & kErrNonfinite) return SEASD_E_NONFINITE;
        if (e & kErrOverlap) return SEASD_E_OVERLAP;
        if (e & kErrCutoff) return SEASD_E_CUTOFF;
    }
    return SEASD_OK;
}

extern "C" int seasd_profile_enable(seasd_handle h, int32_t enable) {
    if (!h) return SEASD_E_INVALID_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return SEASD_E_HIP;
    h->timer.enabled = enable != 0;
    h->timer.products = 0;
    return SEASD_OK;
}

extern "C" int seasd_profile_read(seasd_handle h, double* ms, int32_t count) {
    if (!h || !ms || count < 0) return SEASD_E_INVALID_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return SEASD_E_HIP;
    if (h->timer.products > 0 && hipStreamSynchronize(h->last_stream) != hipSuccess) return SEASD_E_HIP;
    std::vector<double> out(kNumPhases + 1, 0.0);
    const int np = h->timer.products;
    constexpr int S = PhaseTimer::kSlots;
    for (int p = 0; p < np; ++p) {
        const int u = h->timer.used[p];
        for (int k = 0; k < u; ++k) {
            const int ph = h->timer.order[p * S + k];
            if (ph < 0) continue;
            // the phase runs until the next mark on its own stream
            int k2 = k + 1;
            while (k2 < u && h->timer.on[p * S + k2] != h->timer.on[p * S + k]) ++k2;
            if (k2 >= u) continue;
            float t = 0.f;
            if (hipEventElapsedTime(&t, h->timer.ev[p * S + k], h->timer.ev[p * S + k2]) != hipSuccess)
                return SEASD_E_HIP;
            out[ph] += t;
        }
    }
    for (int k = 0; k < kNumPhases; ++k) out[k] = np ? out[k] / np : 0.0;
    out[kNumPhases] = np;
    for (int k = 0; k < count && k <= kNumPhases; ++k) ms[k] = out[k];
    h->timer.products = 0;
    return kNumPhases;
}

// ---------------------------------------------------------------------------
// far-field solve

// Single-sphere blocks M_ii(a) = self(a) + Q(a^2), Q quadratic in a^2: sample
// the product on one sphere alone in the cell at three radii (12 unit inputs
// each), remove the single-sphere self terms, fit the quadratic exactly.
static int build_preconditioner(seasd_handle h, int64_t n, const double* radius, const Cell& L, hipStream_t st) {
    int rc = 0;
    rc |= h->coef.ensure(sizeof(double) * 3 * 144);
    rc |= h->blocks.ensure(sizeof(double) * 144 * n);
    rc |= h->inv.ensure(sizeof(double) * 144 * n);
    rc |= h->singular.ensure(sizeof(int));
    rc |= h->one_pos.ensure(sizeof(double) * 3);
    rc |= h->one_rad.ensure(sizeof(double));
    rc |= h->one_x.ensure(sizeof(double) * 12);
    rc |= h->one_y.ensure(sizeof(double) * 12);
    if (rc) return SEASD_E_NOMEM;
    // radius range (host reduction; setup cost only)
    std::vector<double> rad(n);
    if (hipMemcpy(rad.data(), radius, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) return SEASD_E_HIP;
    double amin = rad[0], amax = rad[0];
    for (double a : rad) {
        if (!(a > 0.0) || !std::isfinite(a)) return SEASD_E_NONFINITE;
        amin = std::fmin(amin, a);
        amax = std::fmax(amax, a);
    }
    h->pc_amax = amax;
    const seasd_config& cf = h->cfg;
    const double key[18] = {amin, amax, (double)cf.grid[0], (double)cf.P, cf.m, cf.xi, cf.rc_factor, cf.eta,
                            (double)cf.precision, L.a[0], L.a[1], L.a[2], L.a[3], L.a[4], L.a[5], L.a[6], L.a[7],
                            L.a[8]};
    const bool cached = h->pc_valid && std::memcmp(key, h->pc_key, sizeof(key)) == 0;
    if (!cached) {
        h->pc_valid = false;
        double samp[3] = {amin, 0.5 * (amin + amax), amax};
        if (amax - amin < 1e-3 * amax) {
            samp[0] = amin;
            samp[1] = 1.25 * amin;
            samp[2] = 1.5 * amin;
        }
        const double zero3[3] = {0.0, 0.0, 0.0};
        if (hipMemcpy(h->one_pos.p, zero3, sizeof(zero3), hipMemcpyHostToDevice) != hipSuccess) return SEASD_E_HIP;
        double Q[3][144];
        const double eta = h->cfg.eta;
        for (int s = 0; s < 3; ++s) {
            if (hipMemcpy(h->one_rad.p, &samp[s], sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return SEASD_E_HIP;
            for (int b = 0; b < 12; ++b) {
                double e[12] = {0};
                e[b] = 1.0;
                if (hipMemcpyAsync(h->one_x.p, e, sizeof(e), hipMemcpyHostToDevice, st) != hipSuccess) return SEASD_E_HIP;
                rc = queue_apply(h, 1, h->one_pos.as<double>(), h->one_rad.as<double>(), L, h->one_x.as<double>(),
                                 h->one_y.as<double>(), st, false);
                if (rc) return rc;
                double col[12];
                if (hipMemcpyAsync(col, h->one_y.p, sizeof(col), hipMemcpyDeviceToHost, st) != hipSuccess) return SEASD_E_HIP;
                if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
                for (int r = 0; r < 12; ++r) Q[s][12 * r + b] = col[r];
            }
            const double a = samp[s], a3 = a * a * a;
            for (int c = 0; c < 3; ++c) Q[s][13 * c] -= 1.0 / (6.0 * kPi * eta * a);
            for (int c = 3; c < 6; ++c) Q[s][13 * c] -= 1.0 / (8.0 * kPi * eta * a3);
            for (int c = 6; c < 11; ++c) Q[s][13 * c] -= 3.0 / (20.0 * kPi * eta * a3);
            Q[s][13 * 11] -= 3.0 / (16.0 * kPi * eta * a3);
        }
        // Q(A) = C0 + C1 A + C2 A^2 through the three samples (Lagrange form)
        double A[3] = {samp[0] * samp[0], samp[1] * samp[1], samp[2] * samp[2]};
        std::vector<double> coef(3 * 144, 0.0);
        for (int s = 0; s < 3; ++s) {
            const int p = (s + 1) % 3, q = (s + 2) % 3;
            const double den = (A[s] - A[p]) * (A[s] - A[q]);
            const double l0 = A[p] * A[q] / den, l1 = -(A[p] + A[q]) / den, l2 = 1.0 / den;
            for (int e = 0; e < 144; ++e) {
                coef[e] += l0 * Q[s][e];
                coef[144 + e] += l1 * Q[s][e];
                coef[288 + e] += l2 * Q[s][e];
            }
        }
        if (hipMemcpy(h->coef.p, coef.data(), sizeof(double) * 3 * 144, hipMemcpyHostToDevice) != hipSuccess)
            return SEASD_E_HIP;
        std::memcpy(h->pc_key, key, sizeof(key));
        h->pc_valid = true;
    }
    if (launch_build_blocks(n, radius, h->coef.as<double>(), h->cfg.xi, h->cfg.eta, h->blocks.as<double>(), st))
        return SEASD_E_HIP;
    if (hipMemsetAsync(h->singular.p, 0, sizeof(int), st) != hipSuccess) return SEASD_E_HIP;
    if (launch_block_invert(n, h->blocks.as<double>(), h->inv.as<double>(), h->singular.as<int>(), st))
        return SEASD_E_HIP;
    int sing = 0;
    if (hipMemcpyAsync(&sing, h->singular.p, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return SEASD_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
    return sing ? SEASD_E_SINGULAR : SEASD_OK;
}

static int dot_host(seasd_handle h, int64_t len, int k, const double* V, int64_t ld, const double* w,
                    double* out_host, hipStream_t st) {
    if (launch_dots(len, k, V, ld, w, h->partial.as<double>(), h->hdev.as<double>(), st)) return SEASD_E_HIP;
    if (hipMemcpyAsync(out_host, h->hdev.p, sizeof(double) * k, hipMemcpyDeviceToHost, st) != hipSuccess)
        return SEASD_E_HIP;
    return hip_ok(hipStreamSynchronize(st));
}

// Binning of the given configuration into the product workspace (no
// neighbour list: the next product rebuilds its geometry). x: any valid
// [n][12] array (gathered along, unused).
static int prepare_geometry(seasd_handle h, int64_t n, const double* pos, const double* radius, const Cell& L,
                            const double* x, hipStream_t st, ApplyArgs& A) {
    int rc = ensure_product_ws(h, n, st);
    if (rc) return rc;
    fill_args(h, A, n, pos, radius, L, x, nullptr, h->cfg.checks != 0, 0);
    if (hipMemsetAsync(A.err, 0, sizeof(int), st) != hipSuccess) return SEASD_E_HIP;
    PhaseTimer off;
    h->geom_n = -1;
    if (launch_geometry(A, st, &off)) return SEASD_E_HIP;
    if (h->cfg.checks) return read_err(h, st);
    return SEASD_OK;
}

// Learned part of a solve or a training step: graph and forward pass of the
// attached network on the binned configuration in A.
static int learned_forward(seasd_handle h, seasd_net net, const Cell& L, const ApplyArgs& A, hipStream_t st) {
    if (net_device(net) != h->device) return SEASD_E_INVALID_ARG;
    if (!(min_height(L) > 4.0 * kEdgeCut * h->pc_amax)) return SEASD_E_CUTOFF;   // edges reach below half the cell
    if (hipMemsetAsync(A.err, 0, sizeof(int), st) != hipSuccess) return SEASD_E_HIP;
    int rc = net_build_graph(net, A, st);
    if (rc) return rc;
    if ((rc = read_err(h, st))) return rc;   // a missing reverse edge reads as a cut-off failure
    return net_forward(net, st);
}

// Rescaled blocks into h->inv2 and the initial guess x0 for b; *fallback = 1
// when the network output is rejected.
static int learned_setup(seasd_handle h, int64_t n, const double* pos, const double* radius, const Cell& L,
                         const double* b, double* x0, bool geometry_current, hipStream_t st, int* fallback) {
    ApplyArgs A;
    int rc;
    if (geometry_current) {
        fill_args(h, A, n, pos, radius, L, b, nullptr, false, 0);
    } else if ((rc = prepare_geometry(h, n, pos, radius, L, b, st, A))) {
        return rc;
    }
    if ((rc = learned_forward(h, h->net, L, A, st))) return rc;
    if (h->inv2.ensure(sizeof(double) * 144 * n) || h->bad.ensure(sizeof(int))) return SEASD_E_NOMEM;
    if (hipMemsetAsync(h->bad.p, 0, sizeof(int), st) != hipSuccess) return SEASD_E_HIP;
    if ((rc = net_learned_blocks(h->net, h->inv.as<double>(), h->perm.as<int>(), h->inv2.as<double>(),
                                 h->bad.as<int>(), st)))
        return rc;
    if ((rc = net_x0(h->net, h->inv.as<double>(), h->perm.as<int>(), 1, b, nullptr, x0, st))) return rc;
    if ((rc = check_finite(12 * n, x0, h->bad.as<int>(), st))) return rc;
    int bad = 0;
    if (hipMemcpyAsync(&bad, h->bad.p, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return SEASD_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
    *fallback = bad ? 1 : 0;
    return SEASD_OK;
}

extern "C" int seasd_solve_farfield(seasd_handle h, int64_t n, const double* pos, const double* radius,
                                    const double* box, const double* b, double* x, seasd_solve_stats* stats,
                                    void* stream) {
    if (!h || n < 1 || n > (int64_t)1 << 28 || !pos || !radius || !b || !x) return SEASD_E_INVALID_ARG;
    Cell L;
    int rc = parse_cell(box, &L);
    if (rc) return rc;
    if (hipSetDevice(h->device) != hipSuccess) return SEASD_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    const seasd_config c = h->cfg;
    const int64_t len = 12 * n;
    seasd_solve_stats S{};
    rc = 0;
    rc |= h->w.ensure(sizeof(double) * len);
    rc |= h->z.ensure(sizeof(double) * len);
    rc |= h->u.ensure(sizeof(double) * len);
    rc |= h->r.ensure(sizeof(double) * len);
    rc |= h->bred.ensure(sizeof(double) * len);
    rc |= h->hdev.ensure(sizeof(double) * 256);
    rc |= h->partial.ensure(sizeof(double) * 256 * 256);
    if (rc) return SEASD_E_NOMEM;
    if ((rc = h->gm.ensure(len, c.restart, c.max_iter))) return rc == -7 ? SEASD_E_NOMEM : SEASD_E_HIP;
    double* w = h->w.as<double>();
    double* z = h->z.as<double>();
    double* u = h->u.as<double>();
    double* bred = h->bred.as<double>();
    const bool pc = c.precond != SEASD_PRECOND_NONE;
    const bool learned = c.precond == SEASD_PRECOND_LEARNED_GUESS;
    if (learned && !h->net) return SEASD_E_INVALID_ARG;
    if (pc) {  // before the geometry: its single-sphere products use the shared workspace
        rc = build_preconditioner(h, n, radius, L, st);
        if (rc) return rc;
    }
    auto t1 = std::chrono::steady_clock::now();
    S.setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    bool have_geometry = false;
    bool first = true;
    int err_rc = SEASD_OK;
    // product with the incompressible components only (trace input and output zeroed)
    auto apply11 = [&](const double* in, double* out) -> int {
        const bool chk = first && c.checks && !c.compressible;
        first = false;
        int e = queue_apply(h, n, pos, radius, L, in, out, st, chk, have_geometry, 0);
        if (e) return e;
        have_geometry = true;
        if (chk && (e = read_err(h, st))) {
            err_rc = e;
            return e;
        }
        return SEASD_OK;
    };
    const double* pc_blocks = h->inv.as<double>();
    auto precond = [&](const double* in, double* out) -> int {
        if (!pc) return hip_ok(hipMemcpyAsync(out, in, sizeof(double) * len, hipMemcpyDeviceToDevice, st));
        return launch_block_apply(n, pc_blocks, in, out, st) ? SEASD_E_HIP : SEASD_OK;
    };
    // One-way pressure-moment coupling (Sec. 2.3 and 4.1): only the part of
    // each pressure moment fixed by its own trace equation, s_self = b_trace /
    // M_self, drives source flows in the solve; the interaction part follows
    // from the pressure Faxen law once F, T, S are known.
    int extra_matvecs = 0;
    if (c.compressible) {
        if (launch_trace_op(n, 0, radius, c.eta, b, nullptr, z, st)) return SEASD_E_HIP;
        rc = queue_apply(h, n, pos, radius, L, z, w, st, c.checks != 0, false, 1);
        if (rc) return rc;
        ++extra_matvecs;
        if (c.checks && (rc = read_err(h, st))) return rc;
        if (launch_trace_op(n, 1, radius, c.eta, b, w, bred, st)) return SEASD_E_HIP;
    } else {
        if (hipMemsetAsync(w, 0, sizeof(double) * len, st) != hipSuccess) return SEASD_E_HIP;
        if (launch_trace_op(n, 1, radius, c.eta, b, w, bred, st)) return SEASD_E_HIP;
    }
    // x holds the caller's guess for F, T, S; its trace entries are ignored
    if (launch_trace_op(n, 1, radius, c.eta, x, nullptr, z, st) ||
        hipMemcpyAsync(x, z, sizeof(double) * len, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return SEASD_E_HIP;
    // learned preconditioner: the network's initial guess (its outputs also
    // pass the finiteness and range checks of the rescaled blocks)
    int fallback = 0, guess = 0;
    if (learned) {
        auto tl = std::chrono::steady_clock::now();
        rc = learned_setup(h, n, pos, radius, L, bred, x, c.compressible != 0, st, &fallback);
        if (rc) return rc;
        if (fallback) {
            if (hipMemsetAsync(x, 0, sizeof(double) * len, st) != hipSuccess) return SEASD_E_HIP;
        } else {
            guess = 1;
            // the true residual judges the guess: scale it by the alpha that
            // minimises |b' - alpha A x0|, dropping it when alpha <= 0
            if ((rc = apply11(x, u))) return rc;
            ++extra_matvecs;
            double ba = 0.0, aa = 0.0;
            if ((rc = dot_host(h, len, 1, bred, len, u, &ba, st))) return rc;
            if ((rc = dot_host(h, len, 1, u, len, u, &aa, st))) return rc;
            const double alpha = (aa > 0.0 && ba > 0.0) ? ba / aa : 0.0;
            if (alpha == 0.0) guess = 0;
            if (launch_axpby(len, alpha, x, 0.0, z, st) ||
                hipMemcpyAsync(x, z, sizeof(double) * len, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return SEASD_E_HIP;
            S.guess_scale = alpha;
        }
        if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
        S.learned_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tl).count();
    }
    GmresResult G;
    // SEASD_MIXED: the FP32 product inside the cycles, the FP64 one for every
    // restart's true residual
    const std::function<int(const double*, double*)> apply_step = fp32_steps(h, apply11);
    const bool mixed = c.precision == SEASD_MIXED;
    rc = h->gm.solve(apply11, precond, bred, x, c.tol, c.max_iter, st, &G, mixed ? &apply_step : nullptr,
                     mixed ? kMixedCycleRtol : 0.0);
    if (rc) return err_rc ? err_rc : (rc == -6 ? SEASD_E_HIP : rc);
    // pressure moments from the pressure Faxen law: s = M_self^-1 (b_trace - p-coupling(F, S))
    if (launch_trace_op(n, 1, radius, c.eta, x, nullptr, z, st)) return SEASD_E_HIP;   // z = (F, T, S, 0)
    if (c.compressible) {
        rc = queue_apply(h, n, pos, radius, L, z, w, st, false, have_geometry, 1);
        if (rc) return rc;
        ++extra_matvecs;
        if (launch_trace_op(n, 1, radius, c.eta, z, nullptr, x, st)) return SEASD_E_HIP;
        if (launch_trace_op(n, 2, radius, c.eta, b, w, x, st)) return SEASD_E_HIP;
    } else if (hipMemcpyAsync(x, z, sizeof(double) * len, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        return SEASD_E_HIP;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
    S.iterations = G.iterations;
    S.restarts = G.restarts;
    S.matvecs = G.matvecs + extra_matvecs;
    S.true_residual = G.true_residual;
    S.initial_residual = G.initial_residual;
    S.converged = G.converged;
    S.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    S.precond_used = learned && !fallback ? c.precond : c.precond == SEASD_PRECOND_NONE ? 0 : 1;
    S.guess_used = guess;
    if (stats) *stats = S;
    if (!S.converged) return SEASD_W_NOT_CONVERGED;
    return fallback ? SEASD_W_PRECOND_FALLBACK : SEASD_OK;
}

// ---------------------------------------------------------------------------
// far-field Brownian forces: x = M^(-1/2) psi by the initial value problem of
// Sec. 4.3 (eqs. ivp-1, ivp-forward, ivp-backward)

extern "C" int seasd_solve_mixed(seasd_handle h, int64_t n, const double* pos, const double* radius,
                                 const double* box, const seasd_bsr6* rnf, double lambda, const double* fp,
                                 const double* einf, double* f, double* s, double* u, seasd_solve_stats* stats,
                                 void* stream) {
    if (!h || n < 1 || n > (int64_t)1 << 26 || !pos || !radius || !rnf || !fp || !einf || !f || !s || !u)
        return SEASD_E_INVALID_ARG;
    if (!rnf->rowptr || !rnf->col || !rnf->val || rnf->nnzb < 0 || rnf->nnzb > ((int64_t)1 << 31) - 1)
        return SEASD_E_INVALID_ARG;
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return SEASD_E_INVALID_ARG;
    Cell L;
    int rc = parse_cell(box, &L);
    if (rc) return rc;
    if (hipSetDevice(h->device) != hipSuccess) return SEASD_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    const seasd_config c = h->cfg;
    const int64_t len = 12 * n, len6 = 6 * n;
    rc = 0;
    rc |= h->w.ensure(sizeof(double) * len);
    rc |= h->z.ensure(sizeof(double) * len);
    rc |= h->u.ensure(sizeof(double) * len);
    rc |= h->bred.ensure(sizeof(double) * len);
    rc |= h->inv2.ensure(sizeof(double) * 144 * n);
    rc |= h->singular.ensure(sizeof(int));
    rc |= h->mv6.ensure(sizeof(double) * len6);
    rc |= h->mw6.ensure(sizeof(double) * len6);
    rc |= h->mp6.ensure(sizeof(double) * len6);
    rc |= h->mu6.ensure(sizeof(double) * len6);
    rc |= h->mt6.ensure(sizeof(double) * len6);
    rc |= h->rinv.ensure(sizeof(double) * 36 * n);
    rc |= h->mbad.ensure(sizeof(int));
    if (rc) return SEASD_E_NOMEM;
    if ((rc = h->gm.ensure(len, c.restart, c.max_iter))) return rc == -7 ? SEASD_E_NOMEM : SEASD_E_HIP;
    const int near_iter = std::max(100, (int)(6 * n));
    if ((rc = h->gm_near.ensure(len6, std::min(c.restart, 60), near_iter))) return rc == -7 ? SEASD_E_NOMEM : SEASD_E_HIP;
    seasd_solve_stats S{};
    // preconditioner blocks (Sec. 4.2): M_ii with the sphere's own images, the
    // inverses of the diagonal blocks of R + lambda I, and their combination
    if ((rc = build_preconditioner(h, n, radius, L, st))) return rc;
    if (launch_clear_ints(1, h->mbad.as<int>(), st) ||
        launch_bsr6_diag_inv(n, rnf->rowptr, rnf->col, rnf->val, lambda, h->rinv.as<double>(), h->mbad.as<int>(), st) ||
        launch_mixed_blocks(n, h->blocks.as<double>(), h->rinv.as<double>(), lambda, h->inv2.as<double>(), st) ||
        launch_clear_ints(1, h->singular.as<int>(), st) ||
        launch_block_invert(n, h->inv2.as<double>(), h->inv2.as<double>(), h->singular.as<int>(), st))
        return SEASD_E_HIP;
    {
        int bad = 0, sing = 0;
        if (hipMemcpyAsync(&bad, h->mbad.p, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&sing, h->singular.p, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SEASD_E_HIP;
        if (bad || sing) return SEASD_E_SINGULAR;
    }
    // near-field preconditioner: incomplete block Cholesky factor of Rt in a
    // multicolour order, factorised on the host, applied on the device
    BlockIC0Host ic;
    {
        std::vector<int32_t> rp_h(n + 1), col_h(rnf->nnzb);
        std::vector<double> val_h(36 * (size_t)rnf->nnzb);
        if (hipMemcpy(rp_h.data(), rnf->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost) != hipSuccess)
            return SEASD_E_HIP;
        if (rp_h[0] != 0 || rp_h[n] != rnf->nnzb) return SEASD_E_INVALID_ARG;
        for (int64_t i = 0; i < n; ++i)
            if (rp_h[i + 1] < rp_h[i]) return SEASD_E_INVALID_ARG;
        if (rnf->nnzb > 0 &&
            (hipMemcpy(col_h.data(), rnf->col, sizeof(int32_t) * rnf->nnzb, hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(val_h.data(), rnf->val, sizeof(double) * 36 * rnf->nnzb, hipMemcpyDeviceToHost) != hipSuccess))
            return SEASD_E_HIP;
        for (int32_t j : col_h)
            if (j < 0 || j >= n) return SEASD_E_INVALID_ARG;
        if (build_block_ic0(n, rp_h, col_h, val_h, lambda, &ic)) return SEASD_E_SINGULAR;
        auto up = [&](DevBuf& d, const void* src, size_t bytes) -> int {
            if (d.ensure(std::max<size_t>(bytes, 8))) return SEASD_E_NOMEM;
            if (bytes && hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return SEASD_E_HIP;
            return SEASD_OK;
        };
        int e = 0;
        if ((e = up(h->ic_rows, ic.rows.data(), sizeof(int32_t) * ic.rows.size())) ||
            (e = up(h->ic_lrp, ic.lrp.data(), sizeof(int32_t) * ic.lrp.size())) ||
            (e = up(h->ic_lcol, ic.lcol.data(), sizeof(int32_t) * ic.lcol.size())) ||
            (e = up(h->ic_lval, ic.lval.data(), sizeof(double) * ic.lval.size())) ||
            (e = up(h->ic_urp, ic.urp.data(), sizeof(int32_t) * ic.urp.size())) ||
            (e = up(h->ic_ucol, ic.ucol.data(), sizeof(int32_t) * ic.ucol.size())) ||
            (e = up(h->ic_uval, ic.uval.data(), sizeof(double) * ic.uval.size())) ||
            (e = up(h->ic_linv, ic.linv.data(), sizeof(double) * ic.linv.size())))
            return e;
        if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;   // host vectors leave scope
    }
    S.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    double* v6 = h->mv6.as<double>();
    double* w6 = h->mw6.as<double>();
    double* p6 = h->mp6.as<double>();
    double* u6 = h->mu6.as<double>();
    double* z12 = h->z.as<double>();
    double* rhs = h->bred.as<double>();
    double* y12 = h->u.as<double>();
    const double near_tol = std::max(0.1 * c.tol, 1e-14);
    bool near_ok = true;
    // out = (L L^T)^-1 in with the incomplete factor: forward solve colour by
    // colour into mt6, backward solve in reverse colour order into out
    double* t6 = h->mt6.as<double>();
    auto ic_apply = [&](const double* in, double* out) -> int {
        const int32_t* rows = h->ic_rows.as<int32_t>();
        for (int c = 0; c < ic.ncolours; ++c) {
            const int a = ic.colour_start[c], cnt = ic.colour_start[c + 1] - a;
            if (launch_ic_solve_colour(cnt, rows + a, h->ic_lrp.as<int32_t>(), h->ic_lcol.as<int32_t>(),
                                       h->ic_lval.as<double>(), h->ic_linv.as<double>(), 0, in, t6, st))
                return SEASD_E_HIP;
        }
        for (int c = ic.ncolours - 1; c >= 0; --c) {
            const int a = ic.colour_start[c], cnt = ic.colour_start[c + 1] - a;
            if (launch_ic_solve_colour(cnt, rows + a, h->ic_urp.as<int32_t>(), h->ic_ucol.as<int32_t>(),
                                       h->ic_uval.as<double>(), h->ic_linv.as<double>(), 1, t6, out, st))
                return SEASD_E_HIP;
        }
        return SEASD_OK;
    };
    // w = (R + lambda I)^-1 v on 6N vectors (GMRES with the incomplete factor as preconditioner)
    auto near_solve = [&](const double* v, double* w) -> int {
        auto op = [&](const double* in, double* out) -> int {
            return launch_bsr6_spmv(n, rnf->rowptr, rnf->col, rnf->val, lambda, in, out, st) ? SEASD_E_HIP : SEASD_OK;
        };
        int e0 = ic_apply(v, w);   // start from the preconditioner's approximation
        if (e0) return e0;
        GmresResult G;
        int e = h->gm_near.solve(op, ic_apply, v, w, near_tol, near_iter, st, &G);
        if (e) return e == -6 ? SEASD_E_HIP : e;
        S.inner_iterations += G.iterations;
        if (!G.converged) near_ok = false;
        return SEASD_OK;
    };
    bool have_geometry = false;
    bool first = true;
    int err_rc = SEASD_OK;
    // out = M in on the 11 incompressible components (trace in and out zero)
    auto apply11 = [&](const double* in, double* out) -> int {
        const bool chk = first && c.checks;
        first = false;
        int e = queue_apply(h, n, pos, radius, L, in, out, st, chk, have_geometry, 0);
        if (e) return e;
        have_geometry = true;
        if (chk && (e = read_err(h, st))) {
            err_rc = e;
            return e;
        }
        return SEASD_OK;
    };
    // Mt y = D y + M (y - lambda D y), D y = [Rt^-1 y_F; 0]
    auto applyMt = [&](const double* in, double* out) -> int {
        int e;
        if (launch_ft_ops(n, 0, 0.0, in, nullptr, v6, st)) return SEASD_E_HIP;
        if ((e = near_solve(v6, w6))) return e;
        if (launch_ft_ops(n, 1, -lambda, in, w6, z12, st)) return SEASD_E_HIP;
        if ((e = apply11(z12, out))) return e;
        return launch_ft_ops(n, 1, 1.0, out, w6, out, st) ? SEASD_E_HIP : SEASD_OK;
    };
    auto precond = [&](const double* in, double* out) -> int {
        return launch_block_apply(n, h->inv2.as<double>(), in, out, st) ? SEASD_E_HIP : SEASD_OK;
    };
    // right-hand side (eq. HI-solve): (lambda M - I) D [Fp; 0] + [0; E]
    int extra = 0;
    if (hipMemcpyAsync(p6, fp, sizeof(double) * len6, hipMemcpyDeviceToDevice, st) != hipSuccess) return SEASD_E_HIP;
    if ((rc = near_solve(p6, w6))) return err_rc ? err_rc : rc;
    if (hipMemsetAsync(z12, 0, sizeof(double) * len, st) != hipSuccess ||
        launch_ft_ops(n, 1, lambda, z12, w6, z12, st))
        return SEASD_E_HIP;
    if ((rc = apply11(z12, rhs))) return err_rc ? err_rc : rc;
    ++extra;
    if (launch_ft_ops(n, 1, -1.0, rhs, w6, rhs, st) || launch_ft_ops(n, 2, 0.0, nullptr, einf, rhs, st))
        return SEASD_E_HIP;
    // y = 0 start
    if (hipMemsetAsync(y12, 0, sizeof(double) * len, st) != hipSuccess) return SEASD_E_HIP;
    GmresResult G;
    const std::function<int(const double*, double*)> step32 = fp32_steps(h, applyMt);
    const bool mixed = c.precision == SEASD_MIXED;
    rc = h->gm.solve(applyMt, precond, rhs, y12, c.tol, c.max_iter, st, &G, mixed ? &step32 : nullptr,
                     mixed ? kMixedCycleRtol : 0.0);
    if (rc) return err_rc ? err_rc : (rc == -6 ? SEASD_E_HIP : rc);
    // U = Rt^-1 (y_F + Fp), F = y_F - lambda U, S = y_S
    if (launch_ft_ops(n, 0, 0.0, y12, fp, v6, st)) return SEASD_E_HIP;
    if ((rc = near_solve(v6, u6))) return rc;
    if (launch_mixed_out(n, y12, u6, lambda, f, s, st) ||
        hipMemcpyAsync(u, u6, sizeof(double) * len6, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return SEASD_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
    S.iterations = G.iterations;
    S.restarts = G.restarts;
    S.matvecs = G.matvecs + extra;
    S.converged = G.converged && near_ok;
    S.true_residual = G.true_residual;
    S.initial_residual = G.initial_residual;
    S.precond_used = SEASD_PRECOND_BLOCKDIAG;
    S.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = S;
    return S.converged ? SEASD_OK : SEASD_W_NOT_CONVERGED;
}

extern "C" int seasd_brownian_farfield(seasd_handle h, int64_t n, const double* pos, const double* radius,
                                       const double* box, const double* psi, double* x, double dtau,
                                       seasd_brownian_stats* stats, void* stream) {
    if (!h || n < 1 || n > (int64_t)1 << 28 || !pos || !radius || !psi || !x || psi == x) return SEASD_E_INVALID_ARG;
    if (!(dtau > 0.0) || !(dtau <= 1.0)) return SEASD_E_INVALID_ARG;
    Cell L;
    int rc = parse_cell(box, &L);
    if (rc) return rc;
    if (hipSetDevice(h->device) != hipSuccess) return SEASD_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    const seasd_config c = h->cfg;
    const int64_t len = 12 * n;
    rc = 0;
    rc |= h->w.ensure(sizeof(double) * len);
    rc |= h->z.ensure(sizeof(double) * len);
    rc |= h->u.ensure(sizeof(double) * len);
    rc |= h->r.ensure(sizeof(double) * len);
    rc |= h->bred.ensure(sizeof(double) * len);
    rc |= h->inv2.ensure(sizeof(double) * 144 * n);
    rc |= h->singular.ensure(sizeof(int));
    if (rc) return SEASD_E_NOMEM;
    if ((rc = h->gm.ensure(len, c.restart, c.max_iter))) return rc == -7 ? SEASD_E_NOMEM : SEASD_E_HIP;
    // the mobility's own blocks M_ii (self and images), for the shifted preconditioners
    if ((rc = build_preconditioner(h, n, radius, L, st))) return rc;
    // dimensionless operator A = s M (s = 6 pi eta a_min): eigenvalues of order one
    double amin = 0.0;
    {
        std::vector<double> rad(n);
        if (hipMemcpy(rad.data(), radius, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) return SEASD_E_HIP;
        amin = *std::min_element(rad.begin(), rad.end());
    }
    const double s = 6.0 * kPi * c.eta * amin;
    double* xv = h->u.as<double>();    // the IVP state
    double* rhs = h->bred.as<double>();
    double* tmp = h->w.as<double>();
    double* sol = h->r.as<double>();
    bool have_geometry = false;
    bool first = true;
    // y = s M11 in (incompressible block, trace zeroed)
    auto applyA = [&](const double* in, double* out) -> int {
        const bool chk = first && c.checks;
        first = false;
        int e = queue_apply(h, n, pos, radius, L, in, out, st, chk, have_geometry, 0);
        if (e) return e;
        have_geometry = true;
        if (chk && (e = read_err(h, st))) return e;
        return launch_axpby(len, 0.0, in, s, out, st) ? SEASD_E_HIP : SEASD_OK;
    };
    seasd_brownian_stats B{};
    B.scale = s;
    // solve (alpha I + beta A) y = b with the shifted block-diagonal preconditioner
    auto shifted_solve = [&](double alpha, double beta, const double* b, double* y) -> int {
        int e = 0;
        if (launch_shift_blocks(n, h->blocks.as<double>(), alpha, beta * s, h->inv2.as<double>(), st)) return SEASD_E_HIP;
        if (hipMemsetAsync(h->singular.p, 0, sizeof(int), st) != hipSuccess) return SEASD_E_HIP;
        if (launch_block_invert(n, h->inv2.as<double>(), h->inv2.as<double>(), h->singular.as<int>(), st))
            return SEASD_E_HIP;
        auto op = [&](const double* in, double* out) -> int {
            int q = applyA(in, out);
            if (q) return q;
            return launch_axpby(len, alpha, in, beta, out, st) ? SEASD_E_HIP : SEASD_OK;
        };
        auto pcond = [&](const double* in, double* out) -> int {
            return launch_block_apply(n, h->inv2.as<double>(), in, out, st) ? SEASD_E_HIP : SEASD_OK;
        };
        // start from the right-hand side scaled by the operator's diagonal size
        if (hipMemcpyAsync(y, b, sizeof(double) * len, hipMemcpyDeviceToDevice, st) != hipSuccess) return SEASD_E_HIP;
        GmresResult G;
        const std::function<int(const double*, double*)> step32 = fp32_steps(h, op);
        const bool mixed = c.precision == SEASD_MIXED;
        e = h->gm.solve(op, pcond, b, y, c.tol, c.max_iter, st, &G, mixed ? &step32 : nullptr,
                        mixed ? kMixedCycleRtol : 0.0);
        if (e) return e == -6 ? SEASD_E_HIP : e;
        B.iterations += G.iterations;
        B.matvecs += G.matvecs;
        B.solves += 1;
        B.max_residual = std::max(B.max_residual, G.true_residual);
        if (!G.converged) B.converged = 0;
        return SEASD_OK;
    };
    B.converged = 1;
    // x(0) = psi on the 11 incompressible components
    if (launch_trace_op(n, 1, radius, c.eta, psi, nullptr, xv, st)) return SEASD_E_HIP;
    const int K = std::max(1, (int)std::lround(1.0 / dtau));
    const double dt = 1.0 / K;
    for (int i = 0; i < K; ++i) {
        const double ta = i * dt, tb = (i + 1) * dt;
        // forward half step: x' = x - (dt/4) [ta I + (1 - ta) A]^-1 (A - I) x
        if ((rc = applyA(xv, tmp))) return rc;
        ++B.matvecs;
        if (launch_axpby(len, -1.0, xv, 1.0, tmp, st)) return SEASD_E_HIP;   // (A - I) x
        if ((rc = shifted_solve(ta, 1.0 - ta, tmp, sol))) return rc;
        if (launch_axpby(len, -0.25 * dt, sol, 1.0, xv, st)) return SEASD_E_HIP;
        // backward half step: [(tb - dt/4) I + (1 - tb + dt/4) A] x_new = [tb I + (1 - tb) A] x'
        if ((rc = applyA(xv, tmp))) return rc;
        ++B.matvecs;
        if (launch_axpby(len, tb, xv, 1.0 - tb, tmp, st)) return SEASD_E_HIP;
        if (hipMemcpyAsync(sol, xv, sizeof(double) * len, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return SEASD_E_HIP;
        if ((rc = shifted_solve(tb - 0.25 * dt, 1.0 - tb + 0.25 * dt, tmp, sol))) return rc;
        if (hipMemcpyAsync(xv, sol, sizeof(double) * len, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return SEASD_E_HIP;
    }
    // M^(-1/2) psi = sqrt(s) A^(-1/2) psi
    if (launch_axpby(len, std::sqrt(s), xv, 0.0, x, st)) return SEASD_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
    B.steps = K;
    B.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = B;
    return B.converged ? SEASD_OK : SEASD_W_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// learned preconditioner: attach, load, loss / gradient and training steps

extern "C" int seasd_precond_attach(seasd_handle h, seasd_net net) {
    if (!h) return SEASD_E_INVALID_ARG;
    h->net = net;
    return SEASD_OK;
}

extern "C" int seasd_precond_load(seasd_handle h, const char* path) {
    if (!h || !path) return SEASD_E_INVALID_ARG;
    seasd_net net = nullptr;
    int rc = seasd_net_create(&net, h->device, 0);
    if (rc) return rc;
    if ((rc = seasd_net_load(net, path))) {
        seasd_net_destroy(net);
        return rc;
    }
    if (h->own_net) {
        if (h->net == h->own_net) h->net = nullptr;
        seasd_net_destroy(h->own_net);
    }
    h->own_net = net;
    h->net = net;
    return SEASD_OK;
}

// Network guess for nrhs right-hand sides and, when asked, the training loss
// (mean relative residual ||b' - A x0||^2 / ||b'||^2 with the method's own
// product), its gradient and an Adam step. The gradient with respect to x0 is
// -2 A (b' - A x0) / (nrhs ||b'||^2) (A symmetric), so each right-hand side
// costs two products.
static int net_step(seasd_handle h, seasd_net net, int64_t n, const double* pos, const double* radius,
                    const double* box, int32_t nrhs, const double* b, double* x0, double* loss, float* grad,
                    bool adam, float lr, void* stream) {
    if (!h || !net || n < 1 || n > (int64_t)1 << 26 || !pos || !radius || !b || nrhs < 1 || nrhs > 4096)
        return SEASD_E_INVALID_ARG;
    Cell L;
    int rc = parse_cell(box, &L);
    if (rc) return rc;
    if (hipSetDevice(h->device) != hipSuccess) return SEASD_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = build_preconditioner(h, n, radius, L, st))) return rc;
    ApplyArgs A;
    if ((rc = prepare_geometry(h, n, pos, radius, L, b, st, A))) return rc;
    if ((rc = learned_forward(h, net, L, A, st))) return rc;
    const int64_t len = 12 * n;
    rc = 0;
    rc |= h->lx0.ensure(sizeof(double) * len * nrhs);
    rc |= h->lg.ensure(sizeof(double) * len * nrhs);
    rc |= h->lb.ensure(sizeof(double) * len);
    rc |= h->lax.ensure(sizeof(double) * len);
    rc |= h->lres.ensure(sizeof(double) * len);
    rc |= h->hdev.ensure(sizeof(double) * 256);
    rc |= h->partial.ensure(sizeof(double) * 256 * 256);
    if (rc) return SEASD_E_NOMEM;
    double* X0 = h->lx0.as<double>();
    double* G = h->lg.as<double>();
    double* bq = h->lb.as<double>();
    double* ax = h->lax.as<double>();
    double* res = h->lres.as<double>();
    const double* inv = h->inv.as<double>();
    if ((rc = net_x0(net, inv, h->perm.as<int>(), nrhs, b, nullptr, X0, st))) return rc;
    if (x0 && hipMemcpyAsync(x0, X0, sizeof(double) * len * nrhs, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return SEASD_E_HIP;
    if (loss || grad || adam) {
        double total = 0.0;
        bool geometry = false;
        for (int q = 0; q < nrhs; ++q) {
            // b' (trace dropped), r = b' - A x0, g = -2 A r / (nrhs |b'|^2)
            if (launch_trace_op(n, 1, radius, h->cfg.eta, b + q * len, nullptr, bq, st)) return SEASD_E_HIP;
            if ((rc = queue_apply(h, n, pos, radius, L, X0 + q * len, ax, st, false, geometry, 0))) return rc;
            geometry = true;
            if (launch_axpby(len, 1.0, bq, 0.0, res, st) || launch_axpby(len, -1.0, ax, 1.0, res, st))
                return SEASD_E_HIP;
            double rr = 0.0, bb = 0.0;
            if ((rc = dot_host(h, len, 1, res, len, res, &rr, st))) return rc;
            if ((rc = dot_host(h, len, 1, bq, len, bq, &bb, st))) return rc;
            if (!(bb > 0.0)) return SEASD_E_INVALID_ARG;
            total += rr / bb / nrhs;
            if (grad || adam) {
                if ((rc = queue_apply(h, n, pos, radius, L, res, ax, st, false, true, 0))) return rc;
                if (launch_axpby(len, -2.0 / (nrhs * bb), ax, 0.0, G + q * len, st)) return SEASD_E_HIP;
            }
        }
        if (loss) *loss = total;
        if (grad || adam) {
            if ((rc = net_x0(net, inv, h->perm.as<int>(), nrhs, b, G, nullptr, st))) return rc;
            if ((rc = net_backward(net, st))) return rc;
            if (grad && (rc = net_grads_to_host(net, grad, seasd_net_param_count(), st))) return rc;
            if (adam && (rc = net_adam(net, lr, st))) return rc;
        }
    }
    return hip_ok(hipStreamSynchronize(st));
}

extern "C" int seasd_net_loss_grad(seasd_handle h, seasd_net net, int64_t n, const double* pos, const double* radius,
                                   const double* box, int32_t nrhs, const double* b, double* x0, double* loss,
                                   float* grad, void* stream) {
    return net_step(h, net, n, pos, radius, box, nrhs, b, x0, loss, grad, false, 0.f, stream);
}

extern "C" int seasd_net_train_step(seasd_handle h, seasd_net net, int64_t n, const double* pos,
                                    const double* radius, const double* box, int32_t nrhs, const double* b, float lr,
                                    double* loss, void* stream) {
    if (!(lr > 0.f) || !std::isfinite(lr)) return SEASD_E_INVALID_ARG;
    return net_step(h, net, n, pos, radius, box, nrhs, b, nullptr, loss, nullptr, true, lr, stream);
}

// ---------------------------------------------------------------------------
// autotuner and batched products

extern "C" int seasd_autotune(int64_t n, const double* box, double a_min, double a_max, double target,
                              int32_t precision, seasd_config* cfg) {
    if (!cfg || n < 1 || !(a_min > 0.0) || !(a_max >= a_min) || !(target > 0.0)) return SEASD_E_INVALID_ARG;
    Cell cell;
    int rc = parse_cell(box, &cell);
    if (rc) return rc;
    const double L = min_height(cell);   // the finest grid spacing sets the window rules
    seasd_default_config(cfg);
    cfg->precision = precision;
    cfg->checks = 0;
    // grid: xi follows the spacing (below), so a finer grid shortens the
    // real-space cut-off and the pair sum shrinks as h^3 while the FFTs grow
    // as M^3 log M; the Faxen terms of the window lose accuracy once h falls
    // below about 0.2 a_max (measured FP32 errors against converged FP64
    // products at h/a_max = 0.85, 0.42, 0.27, 0.21, 0.17, 0.14: 1.2e-7,
    // 2.1e-7, 4.1e-7, 5.9e-7, 1.9e-6, 3.8e-6). For 1e-6 targets take the
    // finest grid with h >= 0.21 a_max; tighter targets keep h near 0.4 a_max.
    int M = 32;
    if (target >= 1e-6) {
        while (M < 256 && L / (2 * M) >= 0.21 * a_max) M *= 2;
    } else {
        while (M < 256 && L / M > 0.42 * a_max) M *= 2;
    }
    const double h = L / M;
    // Measured at h/a = 0.39-0.40 against the converged oracle (FP64 window
    // error; FP32 adds ~5e-7): (xi a, rc_factor, P, m/sqrt(pi P)) =
    //   (0.8, 3.0, 16, 0.85) -> 4.6e-7,  (0.7, 3.5, 16, 0.95) -> 6.6e-8,
    //   (0.7, 3.5, 14, 0.95) -> 4.6e-7,  (0.6, 3.5, 12, 0.95) -> 3.7e-6.
    // xi scales as 1/h (fixed k-space tail); xi r_c is held for the smallest
    // pair (r_c = rc_factor * 2 a_min), as in the scans with a = 1.
    double xi_h, rcx, mf;
    int P;
    if (target >= 1e-5) { xi_h = 0.6 * 0.397; rcx = 0.6 * 3.5; P = 12; mf = 0.95; }
    else if (target >= 1e-6 || precision == SEASD_FP32) { xi_h = 0.8 * 0.397; rcx = 0.8 * 3.0; P = 16; mf = 0.85; }
    else { xi_h = 0.7 * 0.397; rcx = 0.7 * 3.5; P = 16; mf = 0.95; }
    cfg->grid[0] = cfg->grid[1] = cfg->grid[2] = M;
    cfg->xi = xi_h / h;
    cfg->rc_factor = std::max(1.5, rcx / (cfg->xi * a_min));
    cfg->P = std::min(P, M);
    cfg->m = mf * std::sqrt(kPi * cfg->P);
    return SEASD_OK;
}

struct seasd_batch_s {
    int device = 0;
    int nsys = 0;
    std::vector<int64_t> off;
    std::vector<Cell> cells;
    std::vector<seasd_handle> sub;
    std::vector<seasd_config> cfg;
    DevBuf pos, rad, xin, yout;
    MultiPlan* plan = nullptr;
    hipStream_t streams[2] = {};
    hipEvent_t fork = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" int seasd_batch_destroy(seasd_batch b) {
    if (!b) return SEASD_OK;
    hipSetDevice(b->device);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->join) hipEventDestroy(b->join);
    if (b->fork) hipEventDestroy(b->fork);
    multi_plan_free(b->plan);
    for (auto& st : b->streams)
        if (st) hipStreamDestroy(st);
    for (auto h : b->sub) seasd_destroy(h);
    b->pos.release();
    b->rad.release();
    b->xin.release();
    b->yout.release();
    delete b;
    return SEASD_OK;
}

extern "C" int seasd_batch_create(seasd_handle h, int32_t nsys, const int64_t* offsets, const double* pos,
                                  const double* radius, const double* boxes, const seasd_config* per_sys,
                                  double target, seasd_batch* out, void* stream) {
    if (!h || !out || nsys < 1 || !offsets || !pos || !radius || !boxes) return SEASD_E_INVALID_ARG;
    *out = nullptr;
    if (offsets[0] != 0) return SEASD_E_INVALID_ARG;
    for (int k = 0; k < nsys; ++k)
        if (offsets[k + 1] <= offsets[k]) return SEASD_E_INVALID_ARG;
    if (!per_sys && !(target > 0.0)) return SEASD_E_INVALID_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return SEASD_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    auto* b = new seasd_batch_s();
    b->device = h->device;
    b->nsys = nsys;
    b->off.assign(offsets, offsets + nsys + 1);
    const int64_t N = offsets[nsys];
    int rc = 0;
    auto fail = [&](int code) {
        seasd_batch_destroy(b);
        return code;
    };
    for (int k = 0; k < nsys; ++k) {
        Cell ck;
        if ((rc = parse_cell(boxes + 9 * k, &ck))) return fail(rc);
        b->cells.push_back(ck);
    }
    if (b->pos.ensure(sizeof(double) * 3 * N) || b->rad.ensure(sizeof(double) * N) ||
        b->xin.ensure(sizeof(double) * 12 * N) || b->yout.ensure(sizeof(double) * 12 * N))
        return fail(SEASD_E_NOMEM);
    if (hipMemcpyAsync(b->pos.p, pos, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->rad.p, radius, sizeof(double) * N, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemsetAsync(b->xin.p, 0, sizeof(double) * 12 * N, st) != hipSuccess)
        return fail(SEASD_E_HIP);
    std::vector<double> rad(N);
    if (hipMemcpyAsync(rad.data(), radius, sizeof(double) * N, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(SEASD_E_HIP);
    // per-suspension handles, configurations and geometries
    for (int k = 0; k < nsys; ++k) {
        const int64_t n = offsets[k + 1] - offsets[k];
        seasd_config c;
        if (per_sys) {
            c = per_sys[k];
        } else {
            // the real-space tail is held for pairs of 10th-percentile
            // spheres; the grid spacing follows the 99th-percentile radius:
            // the global error is carried by the bulk of the spheres, and the
            // few largest do not need the finer-than-needed grid a_max would
            // set (measured on members of the many-suspension workload: one
            // grid step finer is faster and stays below 1e-6 against the oracle)
            std::vector<double> rk(rad.begin() + offsets[k], rad.begin() + offsets[k + 1]);
            std::sort(rk.begin(), rk.end());
            const double asmall = rk[(size_t)(0.1 * (rk.size() - 1))];
            const double amax = rk[(size_t)(0.99 * (rk.size() - 1))];
            if ((rc = seasd_autotune(n, boxes + 9 * k, asmall, amax, target, h->cfg.precision, &c))) return fail(rc);
            c.eta = h->cfg.eta;
            c.compressible = h->cfg.compressible;
        }
        c.checks = 0;
        seasd_handle sh = nullptr;
        if ((rc = seasd_create(&sh, h->device))) return fail(rc);
        b->sub.push_back(sh);
        if ((rc = seasd_set_config(sh, &c))) return fail(rc);
        b->cfg.push_back(c);
        const int64_t o = offsets[k];
        rc = queue_apply(sh, n, b->pos.as<double>() + 3 * o, b->rad.as<double>() + o, b->cells[k],
                         b->xin.as<double>() + 12 * o, b->yout.as<double>() + 12 * o, st, false);
        if (rc) return fail(rc);
    }
    if (hipStreamSynchronize(st) != hipSuccess) return fail(SEASD_E_HIP);
    // one launch per phase and kernel variant for all suspensions
    std::vector<ApplyArgs> args(nsys);
    for (int k = 0; k < nsys; ++k) {
        const int64_t n = offsets[k + 1] - offsets[k], o = offsets[k];
        fill_args(b->sub[k], args[k], n, b->pos.as<double>() + 3 * o, b->rad.as<double>() + o, b->cells[k],
                  b->xin.as<double>() + 12 * o, b->yout.as<double>() + 12 * o, false, b->cfg[k].compressible);
    }
    if ((rc = multi_plan_build(args.data(), nsys, &b->plan, st)))
        return fail(rc == -8 ? SEASD_E_UNSUPPORTED : (rc == -7 ? SEASD_E_NOMEM : SEASD_E_HIP));
    // capture: the binned moments, then the pair sums on a second stream
    // beside the wave-space chain, joined before the gather
    for (auto& s2 : b->streams)
        if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) return fail(SEASD_E_HIP);
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess)
        return fail(SEASD_E_HIP);
    hipStream_t cap = b->streams[0], side = b->streams[1];
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return fail(SEASD_E_HIP);
    bool ok = multi_queue_moments(b->plan, cap) == 0 && hipEventRecord(b->fork, cap) == hipSuccess &&
              hipStreamWaitEvent(side, b->fork, 0) == hipSuccess && multi_queue_pair(b->plan, side) == 0 &&
              hipEventRecord(b->join, side) == hipSuccess && multi_queue_wave(b->plan, cap) == 0 &&
              hipStreamWaitEvent(cap, b->join, 0) == hipSuccess && multi_queue_gather(b->plan, cap) == 0;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cap, &g);
    if (!ok || ec != hipSuccess || !g) {
        if (g) hipGraphDestroy(g);
        return fail(SEASD_E_HIP);
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) return fail(SEASD_E_HIP);
    *out = b;
    return SEASD_OK;
}

extern "C" int seasd_batch_apply(seasd_batch b, const double* x, double* y, void* stream) {
    if (!b || !x || !y || x == y) return SEASD_E_INVALID_ARG;
    if (hipSetDevice(b->device) != hipSuccess) return SEASD_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = b->off[b->nsys];
    if (hipMemcpyAsync(b->xin.p, x, sizeof(double) * 12 * N, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return SEASD_E_HIP;
    if (hipGraphLaunch(b->exec, st) != hipSuccess) return SEASD_E_HIP;
    if (hipMemcpyAsync(y, b->yout.p, sizeof(double) * 12 * N, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return SEASD_E_HIP;
    return SEASD_OK;
}

extern "C" int seasd_batch_configs(seasd_batch b, seasd_config* out) {
    if (!b || !out) return SEASD_E_INVALID_ARG;
    for (int k = 0; k < b->nsys; ++k) out[k] = b->cfg[k];
    return SEASD_OK;
}

extern "C" int seasd_mobility_apply_batched(seasd_handle h, int32_t nsys, const int64_t* offsets,
                                            const double* pos, const double* radius, const double* boxes,
                                            const seasd_config* per_sys, const double* x, double* y,
                                            void* stream) {
    seasd_batch b = nullptr;
    int rc = seasd_batch_create(h, nsys, offsets, pos, radius, boxes, per_sys, 1e-6, &b, stream);
    if (rc) return rc;
    rc = seasd_batch_apply(b, x, y, stream);
    if (rc == SEASD_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = SEASD_E_HIP;
    seasd_batch_destroy(b);
    return rc;
}
