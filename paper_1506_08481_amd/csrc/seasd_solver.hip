// seasd_solver.hip - device kernels of the far-field solve (Sec. 4.1-4.2):
// reductions and vector updates for GMRES in FP64, and the block-diagonal
// preconditioner (per-sphere 12x12 blocks, built and inverted in FP64).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

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

namespace seasd {

// ---------------------------------------------------------------------------
// near-field / far-field solve (Sec. 4.1): the near-field resistance R as a
// block-sparse matrix of 6x6 blocks (force and torque against velocity and
// spin), block rows rowptr / col, blocks row-major

// y = (R + lambda I) x on 6N vectors; thread (i, r) computes row r of block row i
__global__ void k_bsr6_spmv(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, double lambda, const double* __restrict__ x,
                            double* __restrict__ y) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i = t / 6;
    const int r = (int)(t % 6);
    if (i >= n) return;
    double s = lambda * x[6 * i + r];
    for (int b = rowptr[i]; b < rowptr[i + 1]; ++b) {
        const double* v = val + 36 * (size_t)b + 6 * r;
        const double* xj = x + 6 * (size_t)col[b];
        for (int c = 0; c < 6; ++c) s += v[c] * xj[c];
    }
    y[6 * i + r] = s;
}

// inverse of each diagonal block of R + lambda I (Gauss-Jordan, partial
// pivoting); bad |= 1 for a missing diagonal block, 2 for a singular one
__global__ void k_bsr6_diag_inv(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                const double* __restrict__ val, double lambda, double* __restrict__ out,
                                int* __restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int bd = -1;
    for (int b = rowptr[i]; b < rowptr[i + 1]; ++b)
        if (col[b] == (int32_t)i) bd = b;
    double a[6][6], x[6][6];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            a[r][c] = (bd >= 0 ? val[36 * (size_t)bd + 6 * r + c] : 0.0) + (r == c ? lambda : 0.0);
            x[r][c] = (r == c) ? 1.0 : 0.0;
        }
    if (bd < 0 && lambda == 0.0) {
        atomicOr(bad, 1);
        return;
    }
    double scale = 0.0;
    for (int r = 0; r < 6; ++r) scale = fmax(scale, fabs(a[r][r]));
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        for (int r = c + 1; r < 6; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (!(fabs(a[piv][c]) > 1e-14 * scale)) {
            atomicOr(bad, 2);
            return;
        }
        if (piv != c)
            for (int k = 0; k < 6; ++k) {
                double t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t;
                t = x[c][k]; x[c][k] = x[piv][k]; x[piv][k] = t;
            }
        const double inv = 1.0 / a[c][c];
        for (int k = 0; k < 6; ++k) {
            a[c][k] *= inv;
            x[c][k] *= inv;
        }
        for (int r = 0; r < 6; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            if (f == 0.0) continue;
            for (int k = 0; k < 6; ++k) {
                a[r][k] -= f * a[c][k];
                x[r][k] -= f * x[c][k];
            }
        }
    }
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) out[36 * i + 6 * r + c] = x[r][c];
}

// z_i = B_i v_i with B_i a 6x6 block per sphere
__global__ void k_block6_apply(int64_t n, const double* __restrict__ B, const double* __restrict__ v,
                               double* __restrict__ z) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i = t / 6;
    const int r = (int)(t % 6);
    if (i >= n) return;
    const double* b = B + 36 * i + 6 * r;
    const double* x = v + 6 * i;
    double s = 0.0;
    for (int c = 0; c < 6; ++c) s += b[c] * x[c];
    z[6 * i + r] = s;
}

// per-sphere block of the shifted operator of eq. fM-comp with the
// block-diagonal approximations of Sec. 4.2 (eq. rfu-approx):
//   out = (I - lambda M_ii) D_i + M_ii,  D_i = diag(Rt_ii^-1, 0),
// on the 11 incompressible components (identity on the trace row and column)
__global__ void k_mixed_blocks(int64_t n, const double* __restrict__ M, const double* __restrict__ Rinv,
                               double lambda, double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* m = M + 144 * i;
    const double* ri = Rinv + 36 * i;
    double* o = out + 144 * i;
    for (int r = 0; r < 12; ++r)
        for (int c = 0; c < 12; ++c) {
            double v = 0.0;
            if (r < 11 && c < 11) {
                v = m[12 * r + c];
                if (c < 6) {   // ((I - lambda M) D)[r][c] = D[r][c] - lambda sum_k M[r][k] D[k][c]
                    double md = 0.0;
                    for (int k = 0; k < 6; ++k) md += m[12 * r + k] * ri[6 * k + c];
                    v += (r < 6 ? ri[6 * r + c] : 0.0) - lambda * md;
                }
            } else if (r == c) {
                v = 1.0;
            }
            o[12 * r + c] = v;
        }
}

// 6N <-> 12N vector steps of the mixed solve (force-torque entries are
// components 0..5 of each sphere's 12, the stresslet 6..10, the trace 11):
//   mode 0: out6 = y12[ft] (+ add6 when given)
//   mode 1: out12 = y12 + alpha [w6; 0]        (out12 may be y12)
//   mode 2: out12[6..10] += e5
__global__ void k_ft_ops(int64_t n, int mode, double alpha, const double* __restrict__ y12,
                         const double* __restrict__ v6, double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mode == 0) {
        for (int c = 0; c < 6; ++c) out[6 * i + c] = y12[12 * i + c] + (v6 ? v6[6 * i + c] : 0.0);
    } else if (mode == 1) {
        for (int c = 0; c < 12; ++c) out[12 * i + c] = y12[12 * i + c] + (c < 6 ? alpha * v6[6 * i + c] : 0.0);
    } else {
        for (int c = 0; c < 5; ++c) out[12 * i + 6 + c] += v6[5 * i + c];
    }
}

// outputs of the mixed solve: F = y_F - lambda U, S = y_S
__global__ void k_mixed_out(int64_t n, const double* __restrict__ y12, const double* __restrict__ u6, double lambda,
                            double* __restrict__ f6, double* __restrict__ s5) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < 6; ++c) f6[6 * i + c] = y12[12 * i + c] - lambda * u6[6 * i + c];
    for (int c = 0; c < 5; ++c) s5[5 * i + c] = y12[12 * i + 6 + c];
}

int launch_bsr6_spmv(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val, double lambda,
                     const double* x, double* y, hipStream_t st) {
    hipLaunchKernelGGL(k_bsr6_spmv, dim3(grid1(6 * n, 256)), dim3(256), 0, st, n, rowptr, col, val, lambda, x, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_bsr6_diag_inv(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val, double lambda,
                         double* out, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_bsr6_diag_inv, dim3(grid1(n, 64)), dim3(64), 0, st, n, rowptr, col, val, lambda, out, bad);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_block6_apply(int64_t n, const double* B, const double* v, double* z, hipStream_t st) {
    hipLaunchKernelGGL(k_block6_apply, dim3(grid1(6 * n, 256)), dim3(256), 0, st, n, B, v, z);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mixed_blocks(int64_t n, const double* M, const double* Rinv, double lambda, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_mixed_blocks, dim3(grid1(n, 64)), dim3(64), 0, st, n, M, Rinv, lambda, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_ft_ops(int64_t n, int mode, double alpha, const double* y12, const double* v6, double* out,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_ft_ops, dim3(grid1(n, 256)), dim3(256), 0, st, n, mode, alpha, y12, v6, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mixed_out(int64_t n, const double* y12, const double* u6, double lambda, double* f6, double* s5,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_mixed_out, dim3(grid1(n, 256)), dim3(256), 0, st, n, y12, u6, lambda, f6, s5);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace seasd

namespace seasd {

// ---------------------------------------------------------------------------
// Incomplete block Cholesky factor (zero fill-in) of the near-field matrix
// Rt = R + lambda I with a multicolour ordering: a greedy colouring of the
// block graph puts no two coupled spheres in one colour, so the triangular
// solves of the preconditioner run colour by colour, every block row of a
// colour in parallel. Factor rows are kept under their original sphere index.
//   L x = v:    x_i = Linv_ii (v_i - sum_{k before i} L_ik x_k), colours in order
//   L^T z = y:  z_i = Linv_ii^T (y_i - sum_{j after i} L_ji^T z_j), colours reversed

// one colour of the forward (dir = 0) or backward (dir = 1) block triangular solve;
// thread (row of this colour, component r)
__global__ void k_ic_solve_colour(int nrows, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                                  const int32_t* __restrict__ cl, const double* __restrict__ blk,
                                  const double* __restrict__ linv, int dir, const double* __restrict__ v,
                                  double* __restrict__ x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = t / 6;
    if (q >= nrows) return;
    const int i = rows[q];
    // residual of the 6 entries of row i (each thread forms all 6: they feed the 6x6 solve)
    double res[6];
    for (int c = 0; c < 6; ++c) res[c] = v[6 * (size_t)i + c];
    for (int b = rp[i]; b < rp[i + 1]; ++b) {
        const double* B = blk + 36 * (size_t)b;   // forward: L_ik; backward: L_ji^T (stored transposed)
        const double* xk = x + 6 * (size_t)cl[b];
        for (int r = 0; r < 6; ++r) {
            double s = 0.0;
            for (int c = 0; c < 6; ++c) s += B[6 * r + c] * xk[c];
            res[r] -= s;
        }
    }
    const int r = t % 6;
    const double* Li = linv + 36 * (size_t)i;
    double s = 0.0;
    if (dir == 0)
        for (int c = 0; c < 6; ++c) s += Li[6 * r + c] * res[c];
    else
        for (int c = 0; c < 6; ++c) s += Li[6 * c + r] * res[c];
    x[6 * (size_t)i + r] = s;   // rows of one colour do not couple: x of other rows is final; v != x
}

int launch_ic_solve_colour(int nrows, const int32_t* rows, const int32_t* rp, const int32_t* cl, const double* blk,
                           const double* linv, int dir, const double* v, double* x, hipStream_t st) {
    if (nrows <= 0) return 0;
    hipLaunchKernelGGL(k_ic_solve_colour, dim3(grid1(6 * (int64_t)nrows, 192)), dim3(192), 0, st, nrows, rows, rp,
                       cl, blk, linv, dir, v, x);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---- host factorisation --------------------------------------------------

static bool chol6(const double* A, double* Lo) {   // A = Lo Lo^T, Lo lower triangular
    for (int k = 0; k < 36; ++k) Lo[k] = 0.0;
    for (int j = 0; j < 6; ++j) {
        double d = A[6 * j + j];
        for (int k = 0; k < j; ++k) d -= Lo[6 * j + k] * Lo[6 * j + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        const double ljj = std::sqrt(d);
        Lo[6 * j + j] = ljj;
        for (int i = j + 1; i < 6; ++i) {
            double s = A[6 * i + j];
            for (int k = 0; k < j; ++k) s -= Lo[6 * i + k] * Lo[6 * j + k];
            Lo[6 * i + j] = s / ljj;
        }
    }
    return true;
}

static void inv_lower6(const double* Lo, double* Li) {   // Li = Lo^-1 (lower triangular)
    for (int k = 0; k < 36; ++k) Li[k] = 0.0;
    for (int c = 0; c < 6; ++c) {
        Li[6 * c + c] = 1.0 / Lo[6 * c + c];
        for (int r = c + 1; r < 6; ++r) {
            double s = 0.0;
            for (int k = c; k < r; ++k) s += Lo[6 * r + k] * Li[6 * k + c];
            Li[6 * r + c] = -s / Lo[6 * r + r];
        }
    }
}

int build_block_ic0(int64_t n, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col,
                    const std::vector<double>& val, double lambda, BlockIC0Host* out) {
    // symmetric block graph without the diagonal
    std::vector<std::vector<int32_t>> nb(n);
    for (int64_t i = 0; i < n; ++i)
        for (int b = rowptr[i]; b < rowptr[i + 1]; ++b) {
            const int32_t j = col[b];
            if (j == i) continue;
            nb[i].push_back(j);
            nb[j].push_back((int32_t)i);
        }
    for (auto& v : nb) {
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    // greedy colouring in index order
    std::vector<int32_t> colour(n, -1);
    int ncol = 0;
    {
        std::vector<int> mark;
        for (int64_t i = 0; i < n; ++i) {
            mark.assign(ncol + 1, 0);
            for (int32_t j : nb[i])
                if (colour[j] >= 0) mark[colour[j]] = 1;
            int c = 0;
            while (c < ncol && mark[c]) ++c;
            colour[i] = c;
            ncol = std::max(ncol, c + 1);
        }
    }
    // factor order: by colour, then index
    std::vector<int64_t> ord(n);
    out->colour_start.assign(ncol + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++out->colour_start[colour[i] + 1];
    for (int c = 0; c < ncol; ++c) out->colour_start[c + 1] += out->colour_start[c];
    out->rows.assign(n, 0);
    {
        std::vector<int> fillc(out->colour_start.begin(), out->colour_start.end() - 1);
        for (int64_t i = 0; i < n; ++i) out->rows[fillc[colour[i]]++] = (int32_t)i;
    }
    for (int64_t p = 0; p < n; ++p) ord[out->rows[p]] = p;
    // block A_ij of Rt (sum of stored blocks, both triangles as given)
    auto block = [&](int64_t i, int32_t j, double* B) {
        for (int k = 0; k < 36; ++k) B[k] = 0.0;
        for (int b = rowptr[i]; b < rowptr[i + 1]; ++b)
            if (col[b] == j)
                for (int k = 0; k < 36; ++k) B[k] += val[36 * (size_t)b + k];
        if (j == i)
            for (int d = 0; d < 6; ++d) B[7 * d] += lambda;
    };
    // L_ik for k before i, looked up by (i, k)
    std::vector<std::vector<std::pair<int32_t, int32_t>>> lidx(n);   // (k, slot), sorted by k
    std::vector<double> Lblk;
    std::vector<double> Ldiag(36 * (size_t)n), Linv(36 * (size_t)n);
    double shift = 0.0;
    for (int attempt = 0; attempt < 12; ++attempt) {
        bool ok = true;
        Lblk.clear();
        for (auto& v : lidx) v.clear();
        for (int64_t p = 0; p < n && ok; ++p) {
            const int64_t i = out->rows[p];
            // neighbours before i in the order, in order
            std::vector<int32_t> before;
            for (int32_t k : nb[i])
                if (ord[k] < p) before.push_back(k);
            std::sort(before.begin(), before.end(), [&](int32_t a, int32_t b) { return ord[a] < ord[b]; });
            double D[36];
            block(i, (int32_t)i, D);
            if (shift > 0.0)
                for (int d = 0; d < 6; ++d) D[7 * d] *= 1.0 + shift;
            for (int32_t k : before) {
                double S[36];
                block(i, k, S);
                // S -= sum over m before k coupled to both of L_im L_km^T
                for (const auto& ek : lidx[k]) {
                    const int32_t m = ek.first;
                    auto it = std::lower_bound(lidx[i].begin(), lidx[i].end(), std::make_pair(m, (int32_t)-1));
                    if (it == lidx[i].end() || it->first != m) continue;
                    const double* Lim = Lblk.data() + 36 * (size_t)it->second;
                    const double* Lkm = Lblk.data() + 36 * (size_t)ek.second;
                    for (int r = 0; r < 6; ++r)
                        for (int c = 0; c < 6; ++c) {
                            double s = 0.0;
                            for (int q = 0; q < 6; ++q) s += Lim[6 * r + q] * Lkm[6 * c + q];
                            S[6 * r + c] -= s;
                        }
                }
                // L_ik = S L_kk^-T
                const double* Lik_inv = Linv.data() + 36 * (size_t)k;
                const int32_t slot = (int32_t)(Lblk.size() / 36);
                Lblk.resize(Lblk.size() + 36);
                double* Lik = Lblk.data() + 36 * (size_t)slot;
                for (int r = 0; r < 6; ++r)
                    for (int c = 0; c < 6; ++c) {
                        double s = 0.0;
                        for (int q = 0; q < 6; ++q) s += S[6 * r + q] * Lik_inv[6 * c + q];
                        Lik[6 * r + c] = s;
                    }
                auto pos = std::lower_bound(lidx[i].begin(), lidx[i].end(), std::make_pair(k, (int32_t)-1));
                lidx[i].insert(pos, std::make_pair(k, slot));
                for (int r = 0; r < 6; ++r)
                    for (int c = 0; c < 6; ++c) {
                        double s = 0.0;
                        for (int q = 0; q < 6; ++q) s += Lik[6 * r + q] * Lik[6 * c + q];
                        D[6 * r + c] -= s;
                    }
            }
            if (!chol6(D, Ldiag.data() + 36 * i)) {
                ok = false;
                break;
            }
            inv_lower6(Ldiag.data() + 36 * i, Linv.data() + 36 * i);
        }
        if (ok) {
            out->shift = shift;
            // forward rows: L_ik (k before i); backward rows: L_ki^T for k after i
            out->lrp.assign(n + 1, 0);
            out->urp.assign(n + 1, 0);
            std::vector<std::vector<std::pair<int32_t, int32_t>>> after(n);   // (i, slot of L_ik) per k
            for (int64_t i = 0; i < n; ++i)
                for (const auto& e : lidx[i]) after[e.first].push_back(std::make_pair((int32_t)i, e.second));
            out->lcol.clear();
            out->lval.clear();
            out->ucol.clear();
            out->uval.clear();
            for (int64_t i = 0; i < n; ++i) {
                for (const auto& e : lidx[i]) {
                    out->lcol.push_back(e.first);
                    out->lval.insert(out->lval.end(), Lblk.begin() + 36 * (size_t)e.second,
                                     Lblk.begin() + 36 * (size_t)e.second + 36);
                }
                out->lrp[i + 1] = (int32_t)out->lcol.size();
                for (const auto& e : after[i]) {
                    out->ucol.push_back(e.first);
                    const double* Lki = Lblk.data() + 36 * (size_t)e.second;   // L_{e.first, i}
                    for (int r = 0; r < 6; ++r)
                        for (int c = 0; c < 6; ++c) out->uval.push_back(Lki[6 * c + r]);
                }
                out->urp[i + 1] = (int32_t)out->ucol.size();
            }
            out->linv = Linv;
            out->ncolours = ncol;
            return 0;
        }
        // breakdown: scale the diagonal blocks up (the threshold of Sec. 4.1) and start again
        shift = (shift == 0.0) ? 1e-3 : shift * 10.0;
    }
    return -1;
}

}  // namespace seasd
