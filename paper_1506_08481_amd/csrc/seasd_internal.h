// seasd_internal.h - shared declarations between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace seasd {

constexpr int kPartsReal = 1, kPartsWave = 2, kPartsSelf = 4;
constexpr int kErrNonfinite = 1, kErrOverlap = 2, kErrCutoff = 4;

enum Phase {
    kPhaseBin = 0,
    kPhasePair,
    kPhaseSpread,
    kPhaseFftXFwd,
    kPhaseFftYFwd,
    kPhaseFftZ,
    kPhaseFftYInv,
    kPhaseFftXInv,
    kPhaseGather,
    kNumPhases
};

// Records one HIP event at the start of each phase on the launching stream
// when enabled; the duration of a phase is the time to the next event.
struct PhaseTimer {
    bool enabled = false;
    hipEvent_t ev[kNumPhases + 1] = {};
    int order[kNumPhases + 1];
    int count = 0;
    bool created = false;
    void reset() { count = 0; }
    void begin(int phase, hipStream_t st) {
        if (!enabled) return;
        if (count <= kNumPhases) {
            order[count] = phase;
            hipEventRecord(ev[count], st);
            ++count;
        }
    }
    void end(hipStream_t st) {
        if (!enabled) return;
        if (count <= kNumPhases) {
            order[count] = -1;
            hipEventRecord(ev[count], st);
            ++count;
        }
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
    int M, P, nb, parts, compressible, checks, fp32;
    // workspace
    int* bin_of;
    int* counts;
    int* start;
    int* fill;
    int* perm;
    unsigned long long* amax_bits;
    int* err;
    double* sp;
    double* sa;
    double* sx;
    double* ybuf;
    void* rgrid;
    void* spec;
    const double* twiddle;
};

int launch_apply(const ApplyArgs& a, hipStream_t st, PhaseTimer* tm);

// GMRES / preconditioner helpers (seasd_solver.hip)
int launch_block_apply(int64_t n, const double* blocks, const double* v, double* z, hipStream_t st);
int launch_block_invert(int64_t n, const double* a, double* inv, int* singular, hipStream_t st);
int launch_dots(int64_t len, int k, const double* V, int64_t ld, const double* w, double* partial,
                double* out, hipStream_t st);
int launch_gemv_sub(int64_t len, int k, const double* V, int64_t ld, const double* h, double* w,
                    hipStream_t st);
int launch_axpby(int64_t len, double a, const double* x, double b, double* y, hipStream_t st);
int launch_build_blocks(int64_t n, const double* radius, const double* coef, double xi, double eta,
                        double* blocks, hipStream_t st);

}  // namespace seasd
