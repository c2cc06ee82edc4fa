// seasd_solver.hip - device kernels of the far-field solve (Sec. 4.1-4.2):
// reductions and vector updates for GMRES in FP64, and the block-diagonal
// preconditioner (per-sphere 12x12 blocks, built and inverted in FP64).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "seasd_internal.h"

namespace seasd {

constexpr int kDotBlocks = 256;
constexpr int kDotThreads = 256;
constexpr int kMaxDots = 256;

// partial[k][block] = sum over this block's elements of V[k][i] w[i]
__global__ __launch_bounds__(kDotThreads) void k_dots_partial(int64_t len, int k, const double* __restrict__ V,
                                                              int64_t ld, const double* __restrict__ w,
                                                              double* __restrict__ partial) {
    __shared__ double red[kDotThreads / 64];
    const int64_t chunk = (len + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * chunk, i1 = (i0 + chunk < len) ? i0 + chunk : len;
    for (int q = 0; q < k; ++q) {
        const double* v = V + q * ld;
        double s = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) s += v[i] * w[i];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int j = 0; j < kDotThreads / 64; ++j) t += red[j];
            partial[(size_t)q * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

__global__ void k_dots_final(int k, int nparts, const double* __restrict__ partial, double* __restrict__ out) {
    const int q = blockIdx.x;
    if (q >= k) return;
    __shared__ double red[64];
    double s = 0.0;
    for (int j = threadIdx.x; j < nparts; j += 64) s += partial[(size_t)q * nparts + j];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int j = 0; j < 64; ++j) t += red[j];
        out[q] = t;
    }
}

// w[i] -= sum_q h[q] V[q][i]
__global__ void k_gemv_sub(int64_t len, int k, const double* __restrict__ V, int64_t ld,
                           const double* __restrict__ h, double* __restrict__ w) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += h[q] * V[q * ld + i];
    w[i] -= s;
}

__global__ void k_axpby(int64_t len, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= len) return;
    y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];  // b = 0: y may be uninitialised
}

// z_i = B_i v_i with B_i a 12x12 block per sphere (row-major)
__global__ void k_block_apply(int64_t n, const double* __restrict__ B, const double* __restrict__ v,
                              double* __restrict__ z) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i = t / 12;
    const int r = (int)(t % 12);
    if (i >= n) return;
    const double* b = B + 144 * i + 12 * r;
    const double* x = v + 12 * i;
    double s = 0.0;
    for (int c = 0; c < 12; ++c) s += b[c] * x[c];
    z[12 * i + r] = s;
}

// block_i = single-sphere mobility(a_i) + C0 + C1 a_i^2 + C2 a_i^4, where the
// C's carry the sphere's interaction with its own periodic images and the
// wave-space self correction (a polynomial of degree two in a^2).
__global__ void k_build_blocks(int64_t n, const double* __restrict__ radius, const double* __restrict__ coef,
                               double eta, double* __restrict__ blocks) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = radius[i], A = a * a;
    const double pi = 3.14159265358979323846;
    double* b = blocks + 144 * i;
    for (int e = 0; e < 144; ++e) b[e] = coef[e] + A * coef[144 + e] + A * A * coef[288 + e];
    for (int c = 0; c < 3; ++c) b[13 * c] += 1.0 / (6.0 * pi * eta * a);
    for (int c = 3; c < 6; ++c) b[13 * c] += 1.0 / (8.0 * pi * eta * a * A);
    for (int c = 6; c < 11; ++c) b[13 * c] += 3.0 / (20.0 * pi * eta * a * A);
    b[13 * 11] += 3.0 / (16.0 * pi * eta * a * A);
    // the far-field solve runs on the 11 incompressible components: the trace
    // row and column are replaced by the identity
    for (int c = 0; c < 12; ++c) b[12 * 11 + c] = b[12 * c + 11] = 0.0;
    b[13 * 11] = 1.0;
}

// Pressure-moment steps of the one-way compressible solve (Sec. 2.3, 4.1):
//   mode 0: out = (0,...,0, s_self) with s_self = (16/3) pi eta a^3 b_trace
//   mode 1: out = (b - in) on the 11 incompressible components (in = NULL: b), 0 on the trace
//   mode 2: out_trace = (16/3) pi eta a^3 (b_trace - in_trace)
__global__ void k_trace_op(int64_t n, int mode, const double* __restrict__ radius, double eta,
                           const double* __restrict__ b, const double* __restrict__ in, double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = radius[i];
    const double d = 16.0 / 3.0 * 3.14159265358979323846 * eta * a * a * a;
    const double* bi = b + 12 * i;
    double* o = out + 12 * i;
    if (mode == 0) {
        for (int c = 0; c < 11; ++c) o[c] = 0.0;
        o[11] = d * bi[11];
    } else if (mode == 1) {
        for (int c = 0; c < 11; ++c) o[c] = in ? bi[c] - in[12 * i + c] : bi[c];
        o[11] = 0.0;
    } else {
        o[11] = d * (bi[11] - in[12 * i + 11]);
    }
}

// out_i = alpha I + beta B_i on the 11 incompressible components (identity on
// the trace row and column): the blocks of the shifted operators of the
// Brownian initial value problem
__global__ void k_shift_blocks(int64_t n, const double* __restrict__ B, double alpha, double beta,
                               double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int r = 0; r < 12; ++r)
        for (int c = 0; c < 12; ++c) {
            double v = (r < 11 && c < 11) ? beta * B[144 * i + 12 * r + c] : 0.0;
            if (r == c) v += (r < 11) ? alpha : 1.0;
            out[144 * i + 12 * r + c] = v;
        }
}

// inverse of each 12x12 block by Gauss-Jordan elimination with partial pivoting
__global__ void k_block_invert(int64_t n, const double* __restrict__ in, double* __restrict__ out,
                               int* __restrict__ singular) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a[12][12], x[12][12];
    for (int r = 0; r < 12; ++r)
        for (int c = 0; c < 12; ++c) {
            a[r][c] = in[144 * i + 12 * r + c];
            x[r][c] = (r == c) ? 1.0 : 0.0;
        }
    double scale = 0.0;
    for (int r = 0; r < 12; ++r) scale = fmax(scale, fabs(a[r][r]));
    for (int c = 0; c < 12; ++c) {
        int piv = c;
        for (int r = c + 1; r < 12; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (!(fabs(a[piv][c]) > 1e-14 * scale)) {
            atomicOr(singular, 1);
            return;
        }
        if (piv != c)
            for (int k = 0; k < 12; ++k) {
                double t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t;
                t = x[c][k]; x[c][k] = x[piv][k]; x[piv][k] = t;
            }
        const double inv = 1.0 / a[c][c];
        for (int k = 0; k < 12; ++k) {
            a[c][k] *= inv;
            x[c][k] *= inv;
        }
        for (int r = 0; r < 12; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            if (f == 0.0) continue;
            for (int k = 0; k < 12; ++k) {
                a[r][k] -= f * a[c][k];
                x[r][k] -= f * x[c][k];
            }
        }
    }
    for (int r = 0; r < 12; ++r)
        for (int c = 0; c < 12; ++c) out[144 * i + 12 * r + c] = x[r][c];
}

static inline unsigned grid1(int64_t work, int t) { return (unsigned)((work + t - 1) / t); }

int launch_dots(int64_t len, int k, const double* V, int64_t ld, const double* w, double* partial,
                double* out, hipStream_t st) {
    if (k <= 0) return 0;
    if (k > kMaxDots) return -1;
    hipLaunchKernelGGL(k_dots_partial, dim3(kDotBlocks), dim3(kDotThreads), 0, st, len, k, V, ld, w, partial);
    hipLaunchKernelGGL(k_dots_final, dim3(k), dim3(64), 0, st, k, kDotBlocks, partial, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gemv_sub(int64_t len, int k, const double* V, int64_t ld, const double* h, double* w,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_gemv_sub, dim3(grid1(len, 256)), dim3(256), 0, st, len, k, V, ld, h, w);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_axpby(int64_t len, double a, const double* x, double b, double* y, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, dim3(grid1(len, 256)), dim3(256), 0, st, len, a, x, b, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_block_apply(int64_t n, const double* blocks, const double* v, double* z, hipStream_t st) {
    hipLaunchKernelGGL(k_block_apply, dim3(grid1(12 * n, 256)), dim3(256), 0, st, n, blocks, v, z);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_build_blocks(int64_t n, const double* radius, const double* coef, double /*xi*/, double eta,
                        double* blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_build_blocks, dim3(grid1(n, 128)), dim3(128), 0, st, n, radius, coef, eta, blocks);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_trace_op(int64_t n, int mode, const double* radius, double eta, const double* b, const double* in,
                    double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_trace_op, dim3(grid1(n, 256)), dim3(256), 0, st, n, mode, radius, eta, b, in, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_shift_blocks(int64_t n, const double* blocks, double alpha, double beta, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_shift_blocks, dim3(grid1(n, 128)), dim3(128), 0, st, n, blocks, alpha, beta, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_block_invert(int64_t n, const double* a, double* inv, int* singular, hipStream_t st) {
    hipLaunchKernelGGL(k_block_invert, dim3(grid1(n, 64)), dim3(64), 0, st, n, a, inv, singular);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace seasd
