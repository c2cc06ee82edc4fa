// seasd_internal.h - shared declarations between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

namespace seasd {

constexpr int kPartsReal = 1, kPartsWave = 2, kPartsSelf = 4;
// a wavefront per sphere in the pair sum once the longest neighbour list
// exceeds this multiple of the mean (measured: N = 5e4 spheres of radii 1 and
// 2 at r_c = 6 (a_i + a_j), ratio about 5: 3.8 -> 0.76 ms; N = 1e5 equal
// spheres at r_c = 3 (a_i + a_j), ratio about 1.3: one thread per sphere is
// 1.35x faster)
constexpr double kPairImbalance = 2.0;

// window records: a header of kRecHead reals, then the 1-D window factors
// x[P], y[P], z[P]; the length is rounded up to 4 reals so that staged records
// keep 16-byte alignment
constexpr int kRecHead = 24;
__host__ __device__ inline int rec_stride(int P) { return (kRecHead + 3 * P + 3) & ~3; }
constexpr int kErrNonfinite = 1, kErrOverlap = 2, kErrCutoff = 4;

enum Phase {
    kPhaseBin = 0,
    kPhasePair,
    kPhaseWindow,
    kPhaseSpread,
    kPhaseFftXFwd,
    kPhaseFftYFwd,
    kPhaseFftZ,
    kPhaseFftYInv,
    kPhaseFftXInv,
    kPhaseGather,
    kNumPhases
};

// When enabled, records one HIP event at the start of each phase (and one at
// the end of each stream's part) of every product on the stream that runs the
// phase, without synchronising.
// Event sets are kept per product until read, so a run of back-to-back
// products can be timed phase by phase.
struct PhaseTimer {
    // a product marks each phase's start on the stream that runs it and ends
    // each stream's sequence with an end marker; a phase lasts until the next
    // mark on its own stream (a product may use two streams)
    static constexpr int kSlots = kNumPhases + 6;
    bool enabled = false;
    std::vector<hipEvent_t> ev;     // kSlots per recorded product
    std::vector<int> order;         // phase of each slot (-1: end marker)
    std::vector<hipStream_t> on;    // stream of each slot
    std::vector<int> used;          // slots used per product
    int products = 0;
    void start_product() {
        if (!enabled) return;
        ++products;
        if ((int)used.size() < products) {
            used.push_back(0);
            for (int k = 0; k < kSlots; ++k) {
                hipEvent_t e;
                hipEventCreate(&e);
                ev.push_back(e);
                order.push_back(-1);
                on.push_back(nullptr);
            }
        }
        used[products - 1] = 0;
    }
    void mark(int phase, hipStream_t st) {
        if (!enabled || products == 0) return;
        int& u = used[products - 1];
        if (u >= kSlots) return;
        const int slot = (products - 1) * kSlots + u;
        order[slot] = phase;
        on[slot] = st;
        hipEventRecord(ev[slot], st);
        ++u;
    }
    void begin(int phase, hipStream_t st) { mark(phase, st); }
    void end(hipStream_t st) { mark(-1, st); }
    void destroy() {
        for (auto e : ev) hipEventDestroy(e);
        ev.clear();
        order.clear();
        on.clear();
        used.clear();
        products = 0;
    }
};

// device buffer that only grows
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int ensure(size_t need) {   // 0, or -7 (SEASD_E_NOMEM) when the allocation fails
        if (need <= bytes) return 0;
        if (p) {
            hipDeviceSynchronize();  // queued work may still read the old buffer
            hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, need) != hipSuccess) {
            p = nullptr;
            return -7;
        }
        bytes = need;
        return 0;
    }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

// Periodic cell with lattice vectors a1, a2, a3 as the columns of A (Sec. 2.2).
// Supported shapes: a1 = (a1x, 0, 0), a2 = (a2x, a2y, 0), a3 = (0, 0, a3z)
// with positive diagonal and |a2x| <= a1x: cubes, rectangular boxes and boxes
// sheared in the x-y plane (a2 = (gamma L, L, 0), the simple-shear cell of
// Sec. 3.2, eq. non-ortho-shape). Fractional coordinates t = A^-1 r.
struct Cell {
    double a[9];        // A row-major: a[3 i + j] = component i of lattice vector j
    double ainv[9];     // A^-1 row-major
    double height[3];   // cell thickness across the faces spanned by the other two vectors
    double volume;
};

__host__ __device__ inline void cell_frac(const Cell& c, double x, double y, double z, double* t) {
    t[0] = c.ainv[0] * x + c.ainv[1] * y + c.ainv[2] * z;
    t[1] = c.ainv[3] * x + c.ainv[4] * y + c.ainv[5] * z;
    t[2] = c.ainv[6] * x + c.ainv[7] * y + c.ainv[8] * z;
}
__host__ __device__ inline void cell_cart(const Cell& c, double t0, double t1, double t2, double* r) {
    r[0] = c.a[0] * t0 + c.a[1] * t1 + c.a[2] * t2;
    r[1] = c.a[3] * t0 + c.a[4] * t1 + c.a[5] * t2;
    r[2] = c.a[6] * t0 + c.a[7] * t1 + c.a[8] * t2;
}

// Window geometry on an M^3 grid in fractional coordinates (Sec. 3.1-3.2).
// The window is h = C exp(-beta |u|^2) with u the offset from the centre in
// grid units (eqs. shape, theta-param: beta = 2 m^2 / P^2, so that h falls
// to exp(-m^2/2) at |u| = P/2), C = (beta/pi)^(3/2) M^3 / V. Its Cartesian
// gradient is grad h = -2 g h with g = beta J^T u, J = M A^-1; for the
// supported cells g = (Gxx u_x, Gyx u_x + Gyy u_y, Gzz u_z). The Faxen
// operators (1 + a^2 lap/6) and grad (1 + a^2 lap/10) of eq. grid-space (with
// lap = grad_t^T B^T B grad_t / (4 pi^2), eq. non-ortho-shape) act on h as
//   (1 + a^2 lap/6) h = h (c0 + c1 |g|^2),
//   grad (1 + a^2 lap/10) h = -h [g (e0 + d1 |g|^2) - (4/5) a^2 Qt (g_x, g_y, 0)],
// c0 = 1 - a^2 bq/3, c1 = 2 a^2/3, e0 = 2 - 2 a^2 bq/5 - 4 a^2 bz/5, d1 = 4 a^2/5,
// with bq = beta tr(J^T J), bz = beta (J^T J)_zz and Qt = beta ((J^T J)_xy - (J^T J)_zz I)
// (zero for a cube or a box with equal spacings in x and y).
struct WinGeom {
    double beta;              // Gaussian exponent in grid units
    double Gxx, Gyx, Gyy, Gzz;
    double Qxx, Qxy, Qyy;     // Qt (x-y block)
    double bq, bz;
    double cw;                // C, the spreading weight
    double cwv;               // C V / M^3 = (beta/pi)^(3/2), the gather weight
    bool sheared;             // Qt != 0
};

struct ApplyArgs {
    int64_t n;
    const double* pos;
    const double* radius;
    const double* x;
    double* y;
    Cell cell;
    double reach_per_len[3];  // bins per unit length across each pair of faces (nb / height)
    double xi, rc_factor, inv_eta;
    WinGeom win;
    double kdeconv;           // deconvolution exp(kdeconv |q|^2), q the integer wave vector
    int M, P, nb, parts, compressible, checks, fp32;
    // workspace
    int* bin_of;
    int* counts;
    int* start;
    int* fill;
    int* perm;
    int* scan_tmp;   // block sums of the device scans
    int* ncount;     // [n] neighbours per binned sphere
    unsigned long long* nstats;   // [0] largest entry of ncount, [1] their sum
    int pair_group;  // lanes per sphere of the pair sum from kWaveSpheres spheres on (1 or 64)
    int cap;         // list slots per sphere
    int2* list;      // [n][cap] neighbour entries (j, packed image shift)
    unsigned long long* amax_bits;
    int* err;
    double* sp;      // [n][3] binned centres, Cartesian, wrapped into the cell
    double* st;      // [n][3] binned centres, fractional coordinates in [0, 1)
    double* sa;
    double* sx;
    double* ybuf;
    void* wrec;      // [n][rec_stride(P)] R window records
    void* rgrid;
    void* spec;
    int hybrid;      // hybrid size approach: Faxen Laplacians of the read-out in k space
    void* rgrid2;    // hybrid: [z][y][x] of R4 (Lvx, Lvy, Lvz, 0), Lv = (lap/6) v
    void* spec2;     // hybrid: half spectrum of the same four fields
    const double* twiddle;
};

int launch_twiddles(int M, double* tw, hipStream_t st);
int launch_clear_ints(int n, int* p, hipStream_t st);
int launch_geometry(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);
int launch_pairlist(const ApplyArgs& a, hipStream_t st);
int launch_moments(const ApplyArgs& a, hipStream_t st);
int launch_wave(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);
int launch_pair(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);
int launch_gather(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);

// Batched launches over many suspensions (seasd_kernels.hip): each phase is
// one launch per kernel variant for the whole batch, every workgroup taking a
// (suspension, block) item. Build returns 0, -8 (mixed precisions, the hybrid
// size approach or a partial product: not batched), -7 or -6.
struct MultiPlan;
int multi_plan_build(const ApplyArgs* args, int nsys, MultiPlan** out, hipStream_t st);
void multi_plan_free(MultiPlan* p);
int multi_queue_moments(const MultiPlan* p, hipStream_t st);   // binned copies of the moments
int multi_queue_pair(const MultiPlan* p, hipStream_t st);      // pair sums into ybuf
int multi_queue_wave(const MultiPlan* p, hipStream_t st);      // window records, spreading, FFT chain
int multi_queue_gather(const MultiPlan* p, hipStream_t st);    // gather, y = ybuf + wave part

// GMRES / preconditioner helpers (seasd_solver.hip)
int launch_block_apply(int64_t n, const double* blocks, const double* v, double* z, hipStream_t st);
int launch_block_invert(int64_t n, const double* a, double* inv, int* singular, hipStream_t st);
int launch_shift_blocks(int64_t n, const double* blocks, double alpha, double beta, double* out, hipStream_t st);
int launch_dots(int64_t len, int k, const double* V, int64_t ld, const double* w, double* partial,
                double* out, hipStream_t st);
int launch_gemv_sub(int64_t len, int k, const double* V, int64_t ld, const double* h, double* w,
                    hipStream_t st);
int launch_axpby(int64_t len, double a, const double* x, double b, double* y, hipStream_t st);
int launch_trace_op(int64_t n, int mode, const double* radius, double eta, const double* b, const double* in,
                    double* out, hipStream_t st);
int launch_build_blocks(int64_t n, const double* radius, const double* coef, double xi, double eta,
                        double* blocks, hipStream_t st);
// near-field / far-field solve (seasd_solver.hip)
// incomplete block Cholesky factor of R + lambda I, multicolour order (host side)
struct BlockIC0Host {
    int ncolours = 0;
    double shift = 0.0;                   // relative diagonal scaling that avoided a breakdown
    std::vector<int32_t> colour_start;    // [ncolours + 1] into rows
    std::vector<int32_t> rows;            // block rows grouped by colour
    std::vector<int32_t> lrp, lcol;       // forward rows: L_ik, k before i
    std::vector<double> lval;
    std::vector<int32_t> urp, ucol;       // backward rows: L_ji^T, j after i
    std::vector<double> uval;
    std::vector<double> linv;             // [n][6][6] inverses of the diagonal factors
};
int build_block_ic0(int64_t n, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col,
                    const std::vector<double>& val, double lambda, BlockIC0Host* out);
int launch_ic_solve_colour(int nrows, const int32_t* rows, const int32_t* rp, const int32_t* cl, const double* blk,
                           const double* linv, int dir, const double* v, double* x, hipStream_t st);
int launch_bsr6_spmv(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val, double lambda,
                     const double* x, double* y, hipStream_t st);
int launch_bsr6_diag_inv(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val, double lambda,
                         double* out, int* bad, hipStream_t st);
int launch_block6_apply(int64_t n, const double* B, const double* v, double* z, hipStream_t st);
int launch_mixed_blocks(int64_t n, const double* M, const double* Rinv, double lambda, double* out, hipStream_t st);
int launch_ft_ops(int64_t n, int mode, double alpha, const double* y12, const double* v6, double* out,
                  hipStream_t st);
int launch_mixed_out(int64_t n, const double* y12, const double* u6, double lambda, double* f6, double* s5,
                     hipStream_t st);

// Restarted right-preconditioned GMRES with the Arnoldi process on the device
// (seasd_gmres.hip). apply_A(in, out) and apply_P(in, out) queue out = A in
// and out = P in on the solve's stream; vectors have len entries.
struct GmresResult {
    int iterations = 0, restarts = 0, matvecs = 0, converged = 0;
    double true_residual = 0.0, initial_residual = 0.0;
};

struct DeviceGmres {
    int64_t len = 0;
    int m = 0, chunk = 0, nblk = 0, dper = 1, ndc = 0;
    DevBuf V, w, z, u, r, small, partial, counters;
    double* resid_host = nullptr;   // pinned, fine-grained: per-step residual estimates
    double* resid_hdev = nullptr;   // its device-side address
    int resid_host_n = 0;
    std::vector<hipEvent_t> events;
    bool counters_clear = false;
    int ensure(int64_t len, int m, int max_steps);   // 0, -7 (no memory) or -6 (HIP)
    void release();
    double norm(const double* v, hipStream_t st, int* rc);   // synchronises
    // x in: initial guess, out: solution; stops when |b - A x| <= tol |b| (true
    // residual at each restart) or after max_iter Arnoldi steps. With
    // apply_step the Arnoldi steps use that operator instead of apply_A (a
    // cheaper approximation: the restart cycles become iterative refinement)
    // and a cycle also ends once its residual estimate is below cycle_rtol
    // times the residual it started from.
    int solve(const std::function<int(const double*, double*)>& apply_A,
              const std::function<int(const double*, double*)>& apply_P, const double* b, double* x, double tol,
              int max_iter, hipStream_t st, GmresResult* res,
              const std::function<int(const double*, double*)>* apply_step = nullptr, double cycle_rtol = 0.0);
};

// neighbour graph of the learned preconditioner (seasd_kernels.hip): edges
// s -> j between binned spheres with |r| < cut (a_s + a_j). Count pass: deg
// and rowptr (n + 1 entries, exclusive scan); fill pass: edge arrays, reverse
// edge index, edge and node features (16 floats each).
int launch_edge_count(const ApplyArgs& a, double cut, int* deg, int* rowptr, hipStream_t st);
int launch_edge_fill(const ApplyArgs& a, double cut, const int* rowptr, int* esrc, int* edst, int* erev,
                     float4* geo, float* fe, float* fn, hipStream_t st);

}  // namespace seasd
