// seasd_gmres.hip - restarted, right-preconditioned GMRES in FP64 with the
// Arnoldi process on the device (the far-field solve of Sec. 4.1-4.2 and the
// shifted solves of the Brownian initial value problem, Sec. 4.3).
//
// Per Arnoldi step j (basis V_0..V_j, new vector w = A P V_j), classical
// Gram-Schmidt twice in four passes over w, each reading the basis once:
//   k_gs_dots2d + k_gs_reduce   h1 = V^T w (workgroups over entries x groups
//                               of 4 vectors, then one wavefront per vector)
//   k_gs_sub                    w -= V h1 (one thread per entry)
//   k_gs_dots2d + k_gs_reduce   h2 = V^T w
//   k_gs_finish + k_gs_givens   w -= V h2, |w|; H[:, j] = h1 + h2,
//                               H[j+1, j] = |w|, the Givens rotations of the
//                               least-squares problem, the residual estimate
//                               |g_(j+1)| and 1/|w|
//   k_gs_scale                  V_(j+1) = w / |w|
// The step needs no host round trip; the host reads one scalar per step, one
// step behind, while the next step is already queued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "seasd_internal.h"

namespace seasd {

constexpr int kGsThreads = 256;
constexpr int kGsChunkMax = 2048;   // vector entries per workgroup of the norm

__device__ inline double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kGsThreads / 64; ++k) t += red[k];
    return t;
}

// true in every thread of the last workgroup of the (1- or 2-D) grid to
// arrive, which then resets the counter
__device__ inline bool last_block(unsigned* counter) {
    __shared__ bool last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(counter, 1u);
        last = prev == gridDim.x * gridDim.y - 1;
        if (last) *counter = 0u;
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

__device__ inline double wave_sum(double s) {
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// Partial sums of V^T w over a two-dimensional grid: workgroup (c, g) takes
// entries c * per * 256 .. (per per thread) and basis vectors 4 g .. 4 g + 3,
// so a step has enough workgroups in flight to stream the basis at memory
// speed however few vectors it holds. k_gs_reduce sums the partials: a
// kernel boundary rather than a last-workgroup reduction, whose per-workgroup
// fence and atomic cost more than a launch at this many workgroups.
constexpr int kDotGroup = 4;   // basis vectors per workgroup

__global__ __launch_bounds__(kGsThreads) void k_gs_dots2d(int64_t len, int per, int k, const double* __restrict__ V,
                                                          int64_t ld, const double* __restrict__ w,
                                                          double* __restrict__ partial) {
    __shared__ double red[kDotGroup][kGsThreads / 64];
    const int nc = gridDim.x;
    const int c = blockIdx.x, q0 = blockIdx.y * kDotGroup;
    const int64_t i0 = (int64_t)c * per * kGsThreads;
    double s[kDotGroup] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int e = 0; e < per; ++e) {
        const int64_t i = i0 + e * kGsThreads + threadIdx.x;
        if (i < len) {
            const double wi = w[i];
#pragma unroll
            for (int u = 0; u < kDotGroup; ++u)
                if (q0 + u < k) s[u] += V[(q0 + u) * ld + i] * wi;
        }
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < kDotGroup; ++u) {
        const double t = wave_sum(s[u]);
        if (lane == 0) red[u][wv] = t;
    }
    __syncthreads();
    if (threadIdx.x < kDotGroup && q0 + (int)threadIdx.x < k) {
        double t = 0.0;
        for (int q = 0; q < kGsThreads / 64; ++q) t += red[threadIdx.x][q];
        partial[(size_t)(q0 + threadIdx.x) * nc + c] = t;
    }
}

// out[q] = sum over the nc partial sums of basis vector q: one wavefront per q
__global__ __launch_bounds__(kGsThreads) void k_gs_reduce(int nc, int k, const double* __restrict__ partial,
                                                          double* __restrict__ out) {
    const int q = blockIdx.x * (kGsThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (q >= k) return;
    double t = 0.0;
    for (int b = lane; b < nc; b += 64) t += partial[(size_t)q * nc + b];
    t = wave_sum(t);
    if (lane == 0) out[q] = t;
}

// w -= V h, one thread per entry
__global__ __launch_bounds__(256) void k_gs_sub(int64_t len, int k, const double* __restrict__ V, int64_t ld,
                                               const double* __restrict__ h, double* __restrict__ w) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
#pragma unroll 8
    for (int q = 0; q < k; ++q) s += h[q] * V[q * ld + i];
    w[i] -= s;
}

// Device state of one restart cycle: H[(m + 1) x m] row-major (stride m),
// cs, sn [m], g [m + 1], then the scalars below.
struct GsState {
    double* H;
    double* cs;
    double* sn;
    double* g;
    double* h1;
    double* h2;
    double* inv_hn;   // 1 / |w| (0 on breakdown)
    double* resid;    // [max steps] |g_(j+1)| per step, for the host
};

// w -= V h2 and the partial sums of |w|^2, one per workgroup
__global__ __launch_bounds__(kGsThreads) void k_gs_finish(int64_t len, int chunk, int k, const double* __restrict__ V,
                                                          int64_t ld, const double* __restrict__ h2,
                                                          double* __restrict__ w, double* __restrict__ pnorm) {
    __shared__ double red[kGsThreads / 64];
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int n = (int)std::min<int64_t>(chunk, len - i0);
    double s2 = 0.0;
    for (int i = threadIdx.x; i < n; i += kGsThreads) {
        double s = 0.0;
#pragma unroll 8
        for (int q = 0; q < k; ++q) s += h2[q] * V[q * ld + i0 + i];
        const double v = w[i0 + i] - s;
        w[i0 + i] = v;
        s2 += v * v;
    }
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) pnorm[blockIdx.x] = s2;
}

// |w| from the nc partial sums; H[:, j] = h1 + h2, H[j+1, j] = |w|; the
// Givens rotations of the least-squares problem; the residual estimate
// |g_(j+1)| (written to host memory) and 1/|w|. One wavefront: the column
// and the rotations are staged in LDS so that the sequential sweep over the
// earlier rotations waits on no global load.
constexpr int kMaxRestart = 200;

__global__ __launch_bounds__(64) void k_gs_givens(int nc, int j, int m, const double* __restrict__ pnorm, GsState S,
                                                  double* __restrict__ resid_host) {
    __shared__ double col[kMaxRestart + 2], cs[kMaxRestart + 2], sn[kMaxRestart + 2];
    const int lane = threadIdx.x;
    double nrm2 = 0.0;
    for (int b = lane; b < nc; b += 64) nrm2 += pnorm[b];
    nrm2 = wave_sum(nrm2);
    for (int q = lane; q <= j; q += 64) {
        col[q] = S.h1[q] + S.h2[q];
        cs[q] = S.cs[q];
        sn[q] = S.sn[q];
    }
    __syncthreads();
    if (lane == 0) {
        const double hn = sqrt(nrm2);
        // the earlier rotations applied down column j
        double a = col[0];
        for (int q = 0; q < j; ++q) {
            const double b = col[q + 1];
            col[q] = cs[q] * a + sn[q] * b;
            a = -sn[q] * a + cs[q] * b;
        }
        const double den = hypot(a, hn);
        const double c = den > 0.0 ? a / den : 1.0, s = den > 0.0 ? hn / den : 0.0;
        S.cs[j] = c;
        S.sn[j] = s;
        col[j] = den;
        col[j + 1] = 0.0;
        const double gj = S.g[j];
        S.g[j + 1] = -s * gj;
        S.g[j] = c * gj;
        *S.inv_hn = hn > 0.0 ? 1.0 / hn : 0.0;
        // the host stops on a zero |w| (the Krylov space is invariant): report 0
        resid_host[j] = hn > 0.0 ? fabs(s * gj) : 0.0;
    }
    __syncthreads();
    for (int q = lane; q <= j + 1; q += 64) S.H[q * m + j] = col[q];
}

__global__ void k_gs_scale(int64_t len, const double* __restrict__ w, const double* __restrict__ inv,
                           double* __restrict__ v) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < len) v[i] = w[i] * (*inv);
}

// g = (beta, 0, ..., 0), V_0 = r / beta
__global__ void k_gs_start(int64_t len, int m, double beta, const double* __restrict__ r, double* __restrict__ v0,
                           double* __restrict__ g) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i <= m) g[i] = (i == 0) ? beta : 0.0;
    if (i < len) v0[i] = r[i] / beta;
}

// y = H^-1 g (upper triangular, j columns), then u = V y
__global__ void k_gs_backsolve(int j, int m, const double* __restrict__ H, const double* __restrict__ g,
                               double* __restrict__ y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int q = j - 1; q >= 0; --q) {
        double s = g[q];
        for (int c = q + 1; c < j; ++c) s -= H[q * m + c] * y[c];
        y[q] = H[q * m + q] != 0.0 ? s / H[q * m + q] : 0.0;
    }
}

__global__ void k_gs_combine(int64_t len, int j, const double* __restrict__ V, int64_t ld,
                             const double* __restrict__ y, double* __restrict__ u) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int q = 0; q < j; ++q) s += y[q] * V[q * ld + i];
    u[i] = s;
}

// |v|^2 into out (one workgroup per chunk, reduced by the last)
__global__ __launch_bounds__(kGsThreads) void k_norm2(int64_t len, int chunk, const double* __restrict__ v,
                                                      double* __restrict__ partial, unsigned* counter,
                                                      double* __restrict__ out) {
    __shared__ double red[kGsThreads / 64];
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int n = (int)std::min<int64_t>(chunk, len - i0);
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kGsThreads) s += v[i0 + i] * v[i0 + i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
    if (!last_block(counter)) return;
    if (threadIdx.x >= 64) return;
    double t = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += 64) t += partial[b];
    t = wave_sum(t);
    if (threadIdx.x == 0) *out = t;
}

// ---------------------------------------------------------------------------
// host driver

static inline unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int DeviceGmres::ensure(int64_t len_, int m_, int max_steps) {
    if (m_ < 1 || m_ > kMaxRestart) return -6;   // seasd_set_config holds restart to [1, 200]
    len = len_;
    m = m_;
    // at least 1024 entries per workgroup (several loads in flight per lane,
    // and few partial sums for the last workgroup to reduce), about 128
    // workgroups for long vectors
    chunk = (int)std::min<int64_t>(kGsChunkMax, std::max<int64_t>(1024, (len + 127) / 128));
    nblk = (int)((len + chunk - 1) / chunk);
    // the two-dimensional dot products: 1, 2 or 4 entries per thread, at most
    // about 2048 workgroups along the vector
    dper = len <= 2048 * kGsThreads ? 1 : len <= 4096 * kGsThreads ? 2 : 4;
    ndc = (int)((len + (int64_t)dper * kGsThreads - 1) / ((int64_t)dper * kGsThreads));
    int rc = 0;
    rc |= V.ensure(sizeof(double) * len * (m + 1));
    rc |= w.ensure(sizeof(double) * len);
    rc |= z.ensure(sizeof(double) * len);
    rc |= u.ensure(sizeof(double) * len);
    rc |= r.ensure(sizeof(double) * len);
    rc |= small.ensure(sizeof(double) * ((size_t)(m + 1) * m + 5 * (m + 2) + 8));
    rc |= partial.ensure(sizeof(double) * (size_t)(m + 2) * std::max(nblk, ndc));
    rc |= counters.ensure(sizeof(unsigned) * 4);
    if (rc) return -7;
    if (!counters_clear) {
        if (hipMemset(counters.p, 0, sizeof(unsigned) * 4) != hipSuccess) return -6;
        counters_clear = true;
    }
    if ((int)resid_host_n < m + 1) {
        if (resid_host) hipHostFree(resid_host);
        resid_host = nullptr;
        // fine-grained pinned memory: k_gs_givens writes each step's
        // residual estimate straight to the host
        if (hipHostMalloc((void**)&resid_host, sizeof(double) * (m + 1), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess)
            return -7;
        if (hipHostGetDevicePointer((void**)&resid_hdev, resid_host, 0) != hipSuccess) return -6;
        resid_host_n = m + 1;
    }
    while ((int)events.size() < m + 1) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return -6;
        events.push_back(e);
    }
    (void)max_steps;
    return 0;
}

void DeviceGmres::release() {
    DevBuf* bufs[] = {&V, &w, &z, &u, &r, &small, &partial, &counters};
    for (DevBuf* b : bufs) b->release();
    if (resid_host) hipHostFree(resid_host);
    resid_host = nullptr;
    resid_hdev = nullptr;
    resid_host_n = 0;
    for (auto e : events) hipEventDestroy(e);
    events.clear();
    counters_clear = false;
}

double DeviceGmres::norm(const double* v, hipStream_t st, int* rc) {
    double* out = small.as<double>() + (size_t)(m + 1) * m + 5 * (m + 2) + 2;
    hipLaunchKernelGGL(k_norm2, dim3(nblk), dim3(kGsThreads), 0, st, len, chunk, v, partial.as<double>(),
                       counters.as<unsigned>() + 3, out);
    double h = 0.0;
    if (hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        *rc = -6;
        return 0.0;
    }
    return std::sqrt(h);
}

int DeviceGmres::solve(const std::function<int(const double*, double*)>& apply_A,
                       const std::function<int(const double*, double*)>& apply_P, const double* b, double* x,
                       double tol, int max_iter, hipStream_t st, GmresResult* res,
                       const std::function<int(const double*, double*)>* apply_step, double cycle_rtol) {
    GmresResult R{};
    int rc = 0;
    const double bnorm = norm(b, st, &rc);
    if (rc) return rc;
    if (bnorm == 0.0) {
        if (hipMemsetAsync(x, 0, sizeof(double) * len, st) != hipSuccess) return -6;
        R.converged = 1;
        if (res) *res = R;
        return hipStreamSynchronize(st) == hipSuccess ? 0 : -6;
    }
    double* sm = small.as<double>();
    GsState S;
    S.H = sm;
    S.cs = sm + (size_t)(m + 1) * m;
    S.sn = S.cs + (m + 2);
    S.g = S.sn + (m + 2);
    S.h1 = S.g + (m + 2);
    S.h2 = S.h1 + (m + 2);
    S.inv_hn = S.h2 + (m + 2);   // the norm scratch of norm() sits one slot further on
    double* yv = S.cs;           // the back substitution reuses cs (free once a cycle ends)
    double* Vp = V.as<double>();
    double* wp = w.as<double>();
    double* zp = z.as<double>();
    double* up = u.as<double>();
    double* rp = r.as<double>();
    double* part = partial.as<double>();
    const unsigned gl = blocks_of(len, 256);
    int total = 0;
    double relres = 0.0;
    for (;;) {
        // true residual r = b - A x
        if ((rc = apply_A(x, rp))) return rc;
        ++R.matvecs;
        if (launch_axpby(len, 1.0, b, -1.0, rp, st)) return -6;
        const double beta = norm(rp, st, &rc);
        if (rc) return rc;
        relres = beta / bnorm;
        if (R.restarts == 0) R.initial_residual = relres;
        if (relres <= tol || total >= max_iter) break;
        hipLaunchKernelGGL(k_gs_start, dim3(blocks_of(std::max<int64_t>(len, m + 1), 256)), dim3(256), 0, st, len, m,
                           beta, rp, Vp, S.g);
        int jend = 0;
        bool stop = false;
        int queued = 0;   // steps queued in this cycle
        auto check = [&](int q) -> int {   // wait for step q's residual estimate
            if (hipEventSynchronize(events[q]) != hipSuccess) return -6;
            const double e = resid_host[q];
            jend = q + 1;
            if (e / bnorm <= 0.5 * tol || e <= cycle_rtol * beta || e == 0.0 || !std::isfinite(e)) stop = true;
            return 0;
        };
        for (int j = 0; j < m && total + j < max_iter && !stop; ++j) {
            if ((rc = apply_P(Vp + (size_t)j * len, zp))) return rc;
            if ((rc = apply_step ? (*apply_step)(zp, wp) : apply_A(zp, wp))) return rc;
            ++R.matvecs;
            // classical Gram-Schmidt applied twice: h1 = V^T w, w -= V h1,
            // h2 = V^T w, w -= V h2, then |w| and the Givens update
            const int k = j + 1;
            const dim3 g2d((unsigned)ndc, (unsigned)((k + kDotGroup - 1) / kDotGroup));
            const unsigned gr = (unsigned)((k + kGsThreads / 64 - 1) / (kGsThreads / 64));
            double* pnorm = part + (size_t)(m + 1) * ndc;
            hipLaunchKernelGGL(k_gs_dots2d, g2d, dim3(kGsThreads), 0, st, len, dper, k, Vp, (int64_t)len, wp, part);
            hipLaunchKernelGGL(k_gs_reduce, dim3(gr), dim3(kGsThreads), 0, st, ndc, k, part, S.h1);
            hipLaunchKernelGGL(k_gs_sub, dim3(gl), dim3(256), 0, st, len, k, Vp, (int64_t)len, S.h1, wp);
            hipLaunchKernelGGL(k_gs_dots2d, g2d, dim3(kGsThreads), 0, st, len, dper, k, Vp, (int64_t)len, wp, part);
            hipLaunchKernelGGL(k_gs_reduce, dim3(gr), dim3(kGsThreads), 0, st, ndc, k, part, S.h2);
            hipLaunchKernelGGL(k_gs_finish, dim3(ndc), dim3(kGsThreads), 0, st, len, dper * kGsThreads, k, Vp,
                               (int64_t)len, S.h2, wp, pnorm);
            hipLaunchKernelGGL(k_gs_givens, dim3(1), dim3(64), 0, st, ndc, j, m, pnorm, S, resid_hdev);
            hipLaunchKernelGGL(k_gs_scale, dim3(gl), dim3(256), 0, st, len, wp, S.inv_hn, Vp + (size_t)(j + 1) * len);
            // the event's release makes the kernel's write to host memory visible
            if (hipEventRecord(events[j], st) != hipSuccess) return -6;
            queued = j + 1;
            // one step behind: step j - 1 has long finished when step j's work is queued
            if (j >= 1 && (rc = check(j - 1))) return rc;
        }
        if (!stop && queued > 0 && (rc = check(queued - 1))) return rc;
        if (hipGetLastError() != hipSuccess) return -6;
        total += jend;
        R.iterations = total;
        // x += P (V y) with the steps that count
        hipLaunchKernelGGL(k_gs_backsolve, dim3(1), dim3(64), 0, st, jend, m, S.H, S.g, yv);
        hipLaunchKernelGGL(k_gs_combine, dim3(gl), dim3(256), 0, st, len, jend, Vp, (int64_t)len, yv, up);
        if ((rc = apply_P(up, zp))) return rc;
        if (launch_axpby(len, 1.0, zp, 1.0, x, st)) return -6;
        ++R.restarts;
    }
    R.true_residual = relres;
    R.converged = relres <= tol ? 1 : 0;
    R.iterations = total;
    if (res) *res = R;
    return hipStreamSynchronize(st) == hipSuccess ? 0 : -6;
}

}  // namespace seasd
