// seasd_internal.h - shared declarations between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
// the end) of every product on the launching stream, without synchronising.
// Event sets are kept per product until read, so a run of back-to-back
// products can be timed phase by phase.
struct PhaseTimer {
    static constexpr int kSlots = kNumPhases + 1;
    bool enabled = false;
    std::vector<hipEvent_t> ev;     // kSlots per recorded product
    std::vector<int> order;         // phase of each slot (-1: end marker)
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
        hipEventRecord(ev[slot], st);
        ++u;
    }
    void begin(int phase, hipStream_t st) { mark(phase, st); }
    void end(hipStream_t st) { mark(-1, st); }
    void destroy() {
        for (auto e : ev) hipEventDestroy(e);
        ev.clear();
        order.clear();
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

struct ApplyArgs {
    int64_t n;
    const double* pos;
    const double* radius;
    const double* x;
    double* y;
    double L, binw, xi, rc_factor, inv_eta;
    double h, alpha, tau, cw;
    int M, P, nb, tile, parts, compressible, checks, fp32;
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
    double* sp;
    double* sa;
    double* sx;
    double* ybuf;
    void* wrec;      // [n][rec_stride(P)] R window records
    void* rgrid;
    void* spec;
    const double* twiddle;
};

int launch_geometry(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);
int launch_pairlist(const ApplyArgs& a, hipStream_t st);
int launch_moments(const ApplyArgs& a, hipStream_t st);
int launch_compute(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);
int launch_wave(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);
int launch_pair(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);
int launch_gather(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);

// GMRES / preconditioner helpers (seasd_solver.hip)
int launch_block_apply(int64_t n, const double* blocks, const double* v, double* z, hipStream_t st);
int launch_block_invert(int64_t n, const double* a, double* inv, int* singular, hipStream_t st);
int launch_dots(int64_t len, int k, const double* V, int64_t ld, const double* w, double* partial,
                double* out, hipStream_t st);
int launch_gemv_sub(int64_t len, int k, const double* V, int64_t ld, const double* h, double* w,
                    hipStream_t st);
int launch_axpby(int64_t len, double a, const double* x, double b, double* y, hipStream_t st);
int launch_trace_op(int64_t n, int mode, const double* radius, double eta, const double* b, const double* in,
                    double* out, hipStream_t st);
int launch_build_blocks(int64_t n, const double* radius, const double* coef, double xi, double eta,
                        double* blocks, hipStream_t st);

// neighbour graph of the learned preconditioner (seasd_kernels.hip): edges
// s -> j between binned spheres with |r| < cut (a_s + a_j). Count pass: deg
// and rowptr (n + 1 entries, exclusive scan); fill pass: edge arrays, reverse
// edge index, edge and node features (16 floats each).
int launch_edge_count(const ApplyArgs& a, double cut, int* deg, int* rowptr, hipStream_t st);
int launch_edge_fill(const ApplyArgs& a, double cut, const int* rowptr, int* esrc, int* edst, int* erev,
                     float4* geo, float* fe, float* fn, hipStream_t st);

}  // namespace seasd
