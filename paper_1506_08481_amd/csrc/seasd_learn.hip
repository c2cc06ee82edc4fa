// seasd_learn.hip - the learned far-field preconditioner: a two-layer
// message-passing network on the neighbour graph that rescales each sphere's
// block-diagonal preconditioner block (Sec. 4.2) and predicts a GMRES
// initial guess. Dense layers run on the matrix cores (BF16 operands, FP32
// accumulation, v_mfma_f32_16x16x16_bf16); graph gathers and segment sums
// are plain kernels with fixed summation order; the initial guess, its loss
// and the rescaled blocks are FP64. Training (loss gradient by hand-written
// backward kernels, Adam) runs here too.
//
// Network (H = 64; edges s -> j with |r| < 2 (a_s + a_j)):
//   h = relu(x W_in + b_in)
//   twice: [U|V] = h W_uv; a_sj = relu(U_s + V_j + e_sj W_e + b_a);
//          m_sj = relu(a_sj W_m + b_m); g_s = sum_j m_sj / 16;
//          h <- h + relu([h|g] W_h + b_h)
//   o_s = h W_o + b_o (log-scalings of the F, T, S groups)
//   c_sj = m_sj W_c + b_c (coefficients of 15 covariant pair structures)
//   blocks: S_s B_s S_s with S = diag(exp(o/2)) per group, B_s the inverse
//           block of the block-diagonal preconditioner
//   x0_s = S B S b_s + sum_j sigma_s * Q(c_sj, u_sj) (sigma_j * b_j),
//          sigma = sqrt(diag B)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/seasd.h"
#include "seasd_internal.h"
#include "seasd_learn.h"
#include "seasd_math.h"

namespace seasd {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (short)(u >> 16);
}

// ---------------------------------------------------------------------------
// dense layer Y = [X1 | X2] W (+ bias, epilogue) on the matrix cores.
// Wt: BF16 [NOUT][K] (W transposed), staged in LDS once per workgroup. Each
// wavefront computes 16-row tiles: lane l loads X[row0 + l%16][k + 4 (l/16) ..]
// (A operand) and Wt[n + l%16][k + 4 (l/16) ..] (B operand) and holds
// Y[row0 + 4 (l/16) + v][n + l%16], v = 0..3, of the result.

enum { kEpiNone = 0, kEpiRelu = 1, kEpiEdge = 2, kEpiResid = 3, kEpiAdd = 4 };

template <int K1, int K2, int NOUT, int EPI>
__global__ __launch_bounds__(256) void k_dense(int64_t R, const float* __restrict__ X1, const float* __restrict__ X2,
                                               const short* __restrict__ Wt, const float* __restrict__ bias,
                                               float* __restrict__ Y, float* __restrict__ Y2,
                                               const float* __restrict__ base, const int* __restrict__ esrc,
                                               const int* __restrict__ edst) {
    constexpr int K = K1 + K2;
    constexpr int NB = NOUT / 16;
    static_assert(K % 16 == 0 && NOUT % 16 == 0, "tile multiples");
    __shared__ short w[NOUT * K];
    for (int i = threadIdx.x; i < NOUT * K; i += 256) w[i] = Wt[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t ntiles = (R + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < ntiles; t += (int64_t)gridDim.x * 4) {
        const int64_t row0 = t * 16;
        f32x4 acc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int64_t ra = row0 + lr;
        const bool va = ra < R;
#pragma unroll
        for (int kk = 0; kk < K / 16; ++kk) {
            const int k = kk * 16 + lk * 4;
            float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
            if (va) {
                if (K2 == 0 || k < K1)
                    xv = *reinterpret_cast<const float4*>(X1 + ra * K1 + k);
                else
                    xv = *reinterpret_cast<const float4*>(X2 + ra * K2 + (k - K1));
            }
            bf16x4 a;
            a[0] = to_bf16(xv.x);
            a[1] = to_bf16(xv.y);
            a[2] = to_bf16(xv.z);
            a[3] = to_bf16(xv.w);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const short* wp = w + (nb * 16 + lr) * K + k;
                bf16x4 b;
                b[0] = wp[0];
                b[1] = wp[1];
                b[2] = wp[2];
                b[3] = wp[3];
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int col = nb * 16 + lr;
            const float bv = bias ? bias[col] : 0.f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + 4 * lk + v;
                if (row >= R) continue;
                float val = acc[nb][v] + bv;
                const int64_t o = row * NOUT + col;
                if (EPI == kEpiNone) {
                    Y[o] = val;
                } else if (EPI == kEpiRelu) {
                    Y[o] = fmaxf(val, 0.f);
                } else if (EPI == kEpiEdge) {
                    val += base[(int64_t)esrc[row] * 128 + col] + base[(int64_t)edst[row] * 128 + 64 + col];
                    Y[o] = fmaxf(val, 0.f);
                } else if (EPI == kEpiResid) {
                    const float r = fmaxf(val, 0.f);
                    Y2[o] = r;
                    Y[o] = base[o] + r;
                } else {
                    Y[o] = base[o] + val;
                }
            }
        }
    }
}

// weight gradient dW = [X1 | X2]^T dZ over a chunk of rows per workgroup:
// partial[blockIdx.x][K][NOUT]. A operand: X^T (lane l loads
// X[r + 4 (l/16) + v][k + l%16]); B operand: dZ (lane l loads
// dZ[r + 4 (l/16) + v][n + l%16]).
template <int K1, int K2, int NOUT>
__global__ __launch_bounds__(256) void k_wgrad(int64_t R, int64_t chunk, const float* __restrict__ X1,
                                               const float* __restrict__ X2, const float* __restrict__ dZ,
                                               float* __restrict__ partial) {
    constexpr int K = K1 + K2, TK = K / 16, TN = NOUT / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = (r0 + chunk < R) ? r0 + chunk : R;
    float* out = partial + (size_t)blockIdx.x * K * NOUT;
    for (int t = wave; t < TK * TN; t += 4) {
        const int tk = t / TN, tn = t % TN;
        const int kc = tk * 16 + lr, nc = tn * 16 + lr;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int64_t rb = r0; rb < r1; rb += 16) {
            bf16x4 a, b;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = rb + 4 * lk + v;
                float xv = 0.f, zv = 0.f;
                if (row < r1) {
                    xv = (K2 == 0 || kc < K1) ? X1[row * K1 + kc] : X2[row * K2 + (kc - K1)];
                    zv = dZ[row * NOUT + nc];
                }
                a[v] = to_bf16(xv);
                b[v] = to_bf16(zv);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(size_t)(tk * 16 + 4 * lk + v) * NOUT + tn * 16 + lr] = acc[v];
    }
}

// column sums of dZ (bias gradients) over the same row chunks, FP32
template <int NOUT>
__global__ __launch_bounds__(256) void k_colsum(int64_t R, int64_t chunk, const float* __restrict__ dZ,
                                                float* __restrict__ partial) {
    __shared__ float red[256];
    const int c = threadIdx.x % NOUT, part = threadIdx.x / NOUT;
    constexpr int NP = 256 / NOUT;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = (r0 + chunk < R) ? r0 + chunk : R;
    float s = 0.f;
    for (int64_t r = r0 + part; r < r1; r += NP) s += dZ[r * NOUT + c];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < NOUT) {
        float t = 0.f;
        for (int p = 0; p < NP; ++p) t += red[p * NOUT + threadIdx.x];
        partial[(size_t)blockIdx.x * NOUT + threadIdx.x] = t;
    }
}

__global__ void k_reduce_parts(int nparts, int64_t size, const float* __restrict__ partial, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= size) return;
    float s = 0.f;
    for (int p = 0; p < nparts; ++p) s += partial[(size_t)p * size + i];
    out[i] = s;
}

// g_s = scale * sum over row s of M[e]   (64 columns)
__global__ __launch_bounds__(256) void k_segsum(int n, const int* __restrict__ rowptr, const float* __restrict__ M,
                                                float scale, float* __restrict__ g, int ldg) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = (int)(t >> 6), c = (int)(t & 63);
    if (s >= n) return;
    float acc = 0.f;
    for (int e = rowptr[s]; e < rowptr[s + 1]; ++e) acc += M[(int64_t)e * 64 + c];
    g[(int64_t)s * ldg + c] = scale * acc;
}

// dUV[s] = [sum_{e in row s} dA[e] | sum_{e in row s} dA[rev e]]
__global__ __launch_bounds__(256) void k_segsum_uv(int n, const int* __restrict__ rowptr, const int* __restrict__ erev,
                                                   const float* __restrict__ dA, float* __restrict__ duv) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = (int)(t >> 6), c = (int)(t & 63);
    if (s >= n) return;
    float u = 0.f, v = 0.f;
    for (int e = rowptr[s]; e < rowptr[s + 1]; ++e) {
        u += dA[(int64_t)e * 64 + c];
        v += dA[(int64_t)erev[e] * 64 + c];
    }
    duv[(int64_t)s * 128 + c] = u;
    duv[(int64_t)s * 128 + 64 + c] = v;
}

// dZm[e] = (scale * dHG[src e][64 + c] + extra[e]) * (Mo[e] > 0)
__global__ void k_msg_back(int64_t E, const int* __restrict__ esrc, const float* __restrict__ dhg, float scale,
                           const float* __restrict__ extra, const float* __restrict__ Mo, float* __restrict__ dz) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * 64) return;
    const int64_t e = t >> 6;
    const int c = (int)(t & 63);
    float v = scale * dhg[(int64_t)esrc[e] * 128 + 64 + c];
    if (extra) v += extra[t];
    dz[t] = Mo[t] > 0.f ? v : 0.f;
}

// out = d * (y > 0) (ldd, ldo: row strides; 64 columns)
__global__ void k_relu_back(int64_t R, const float* __restrict__ d, int ldd, const float* __restrict__ y,
                            float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= R * 64) return;
    const int64_t r = t >> 6;
    const int c = (int)(t & 63);
    out[t] = y[t] > 0.f ? d[r * ldd + c] : 0.f;
}

// dh_out = dh + dhg[:, 0:64]
__global__ void k_add_half(int64_t R, const float* __restrict__ dh, const float* __restrict__ dhg,
                           float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= R * 64) return;
    out[t] = dh[t] + dhg[(t >> 6) * 128 + (t & 63)];
}

// ---------------------------------------------------------------------------
// the 15 covariant structures T_k(u) between (F, T, S) and (U, Omega, E)

__device__ inline void sym_outer(const double* a, const double* b, double* X) {   // sym(a b^T)
    X[0] = a[0] * b[0];
    X[1] = a[1] * b[1];
    X[2] = a[2] * b[2];
    X[3] = 0.5 * (a[0] * b[1] + a[1] * b[0]);
    X[4] = 0.5 * (a[0] * b[2] + a[2] * b[0]);
    X[5] = 0.5 * (a[1] * b[2] + a[2] * b[1]);
}
__device__ inline void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline void symv(const double* S, const double* v, double* o) {   // S (xx yy zz xy xz yz) v
    o[0] = S[0] * v[0] + S[3] * v[1] + S[4] * v[2];
    o[1] = S[3] * v[0] + S[1] * v[1] + S[5] * v[2];
    o[2] = S[4] * v[0] + S[5] * v[1] + S[2] * v[2];
}
__device__ inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// out += sum_k c[k] T_k(u) w
__device__ inline void struct_apply(const float* c, const double* u, const double* w, double* out) {
    const double* wF = w;
    const double* wT = w + 3;
    double S[6], Su[3], q[5], uu[6], t3[3], X[6], e[5];
    s5_to_sym(w + 6, S);
    symv(S, u, Su);
    const double uSu = dot3(u, Su), uF = dot3(u, wF), uT = dot3(u, wT);
    sym_outer(u, u, uu);
    sym_to_e5(uu, q);
    double uxT[3], uxF[3], uxSu[3];
    cross3(u, wT, uxT);
    cross3(u, wF, uxF);
    cross3(u, Su, uxSu);
    for (int a = 0; a < 3; ++a) {
        out[a] += c[0] * wF[a] + c[1] * u[a] * uF + c[2] * uxT[a] + c[6] * Su[a] + c[7] * u[a] * uSu;
        out[3 + a] += c[3] * uxF[a] + c[4] * wT[a] + c[5] * u[a] * uT + c[10] * uxSu[a];
    }
    // E rows: c8 (Y_k u).wF + c11 (Y_k u).(wT x u) + c13 (Y_k u).(S u) = <Y_k, sym(u p^T)>
    cross3(wT, u, t3);
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = c[8] * wF[a] + c[11] * t3[a] + c[13] * Su[a];
    sym_outer(u, p, X);
    sym_to_e5(X, e);
    const double qs = c[9] * uF + c[14] * uSu;
    for (int k = 0; k < 5; ++k) out[6 + k] += e[k] + qs * q[k] + c[12] * w[6 + k];
}

// dc[k] += t . T_k(u) w
__device__ inline void struct_grad(const double* u, const double* w, const double* t, double* dc) {
    const double* wF = w;
    const double* wT = w + 3;
    const double* tF = t;
    const double* tT = t + 3;
    double S[6], St[6], Su[3], uu[6], q[5], tmp[3];
    s5_to_sym(w + 6, S);
    s5_to_sym(t + 6, St);   // <t_E, e5(sym(a b^T))> = a^T St b
    symv(S, u, Su);
    const double uSu = dot3(u, Su), uF = dot3(u, wF), uT = dot3(u, wT);
    const double tFu = dot3(tF, u), tTu = dot3(tT, u);
    sym_outer(u, u, uu);
    sym_to_e5(uu, q);
    double tq = 0.0, tw = 0.0;
    for (int k = 0; k < 5; ++k) {
        tq += t[6 + k] * q[k];
        tw += t[6 + k] * w[6 + k];
    }
    double Stu[3];
    symv(St, u, Stu);   // St u; then u^T St b = Stu . b
    dc[0] += dot3(tF, wF);
    dc[1] += tFu * uF;
    cross3(u, wT, tmp);
    dc[2] += dot3(tF, tmp);
    cross3(u, wF, tmp);
    dc[3] += dot3(tT, tmp);
    dc[4] += dot3(tT, wT);
    dc[5] += tTu * uT;
    dc[6] += dot3(tF, Su);
    dc[7] += tFu * uSu;
    dc[8] += dot3(Stu, wF);
    dc[9] += tq * uF;
    cross3(u, Su, tmp);
    dc[10] += dot3(tT, tmp);
    cross3(wT, u, tmp);
    dc[11] += dot3(Stu, tmp);
    dc[12] += tw;
    dc[13] += dot3(Stu, Su);
    dc[14] += tq * uSu;
}

__device__ inline int group_of(int c) { return c < 3 ? 0 : (c < 6 ? 1 : 2); }

// Initial guess for every binned sphere s (gin == NULL), or the gradients of
// sum(gin * x0) with respect to o and c (gin != NULL); b, gin, x0:
// [nrhs][n][12] in caller order.
__global__ __launch_bounds__(64) void k_x0_net(int n, int nrhs, const int* __restrict__ perm,
                                               const int* __restrict__ rowptr, const int* __restrict__ edst,
                                               const float4* __restrict__ geo, const double* __restrict__ inv,
                                               const float* __restrict__ o, const float* __restrict__ c,
                                               const double* __restrict__ b, const double* __restrict__ gin,
                                               double* __restrict__ x0, float* __restrict__ dO,
                                               float* __restrict__ dC) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    const double* B = inv + 144 * (size_t)i;
    double sig[11], sc[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        sig[k] = sqrt(B[13 * k]);
        sc[k] = exp(0.5 * (double)o[16 * (size_t)s + group_of(k)]);
    }
    const int e0 = rowptr[s], e1 = rowptr[s + 1];
    double dOF = 0.0, dOT = 0.0, dOS = 0.0;
    const size_t nn = (size_t)n * 12;
    for (int q = 0; q < nrhs; ++q) {
        const double* bi = b + q * nn + 12 * (size_t)i;
        double sb[11], Bsb[11];
#pragma unroll
        for (int k = 0; k < 11; ++k) sb[k] = sc[k] * bi[k];
#pragma unroll
        for (int r = 0; r < 11; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 11; ++k) acc += B[12 * r + k] * sb[k];
            Bsb[r] = acc;
        }
        if (!gin) {
            double y[11];
#pragma unroll
            for (int k = 0; k < 11; ++k) y[k] = 0.0;
            for (int e = e0; e < e1; ++e) {
                const int j = perm[edst[e]];
                const double* Bj = inv + 144 * (size_t)j;
                const double* bj = b + q * nn + 12 * (size_t)j;
                double wj[11];
#pragma unroll
                for (int k = 0; k < 11; ++k) wj[k] = sqrt(Bj[13 * k]) * bj[k];
                const float4 g4 = geo[e];
                const double u[3] = {g4.x, g4.y, g4.z};
                struct_apply(c + 16 * (size_t)e, u, wj, y);
            }
            double* xo = x0 + q * nn + 12 * (size_t)i;
#pragma unroll
            for (int k = 0; k < 11; ++k) xo[k] = sc[k] * Bsb[k] + sig[k] * y[k];
            xo[11] = 0.0;
            continue;
        }
        const double* gi = gin + q * nn + 12 * (size_t)i;
        // dL/ds_k = g_k (B S b)_k + b_k (B^T S g)_k ; dL/do = sum over the group of s_k/2 dL/ds_k
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            double btg = 0.0;
#pragma unroll
            for (int r = 0; r < 11; ++r) btg += B[12 * r + k] * sc[r] * gi[r];
            const double v = 0.5 * sc[k] * (gi[k] * Bsb[k] + bi[k] * btg);
            if (k < 3)
                dOF += v;
            else if (k < 6)
                dOT += v;
            else
                dOS += v;
        }
        double t[11];
#pragma unroll
        for (int k = 0; k < 11; ++k) t[k] = sig[k] * gi[k];
        for (int e = e0; e < e1; ++e) {
            const int j = perm[edst[e]];
            const double* Bj = inv + 144 * (size_t)j;
            const double* bj = b + q * nn + 12 * (size_t)j;
            double wj[11], d15[15];
#pragma unroll
            for (int k = 0; k < 11; ++k) wj[k] = sqrt(Bj[13 * k]) * bj[k];
#pragma unroll
            for (int k = 0; k < 15; ++k) d15[k] = 0.0;
            const float4 g4 = geo[e];
            const double u[3] = {g4.x, g4.y, g4.z};
            struct_grad(u, wj, t, d15);
            float* dce = dC + 16 * (size_t)e;
#pragma unroll
            for (int k = 0; k < 15; ++k) dce[k] = (q == 0 ? 0.f : dce[k]) + (float)d15[k];
            dce[15] = 0.f;
        }
    }
    if (gin) {
        float* d = dO + 16 * (size_t)s;
        d[0] = (float)dOF;
        d[1] = (float)dOT;
        d[2] = (float)dOS;
        for (int k = 3; k < 16; ++k) d[k] = 0.f;
    }
}

// out_i = S_i B_i S_i (12x12, trace row and column kept); bad |= 1 when an
// output is not finite or a scaling is beyond e^{+-8}
__global__ void k_learned_blocks(int n, const int* __restrict__ perm, const double* __restrict__ inv,
                                 const float* __restrict__ o, double* __restrict__ out, int* __restrict__ bad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    double sc[12];
    bool ok = true;
    for (int k = 0; k < 12; ++k) {
        const double ov = k < 11 ? (double)o[16 * (size_t)s + group_of(k)] : 0.0;
        ok = ok && isfinite(ov) && fabs(ov) < 16.0;
        sc[k] = exp(0.5 * ov);
    }
    const double* B = inv + 144 * (size_t)i;
    double* D = out + 144 * (size_t)i;
    for (int r = 0; r < 12; ++r)
        for (int k = 0; k < 12; ++k) {
            const double v = sc[r] * B[12 * r + k] * sc[k];
            ok = ok && isfinite(v);
            D[12 * r + k] = v;
        }
    if (!ok) atomicOr(bad, 1);
}

__global__ void k_nonfinite(int64_t len, const double* __restrict__ x, int* __restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len && !isfinite(x[t])) atomicOr(bad, 1);
}

// squared 2-norm of the gradient (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_sqnorm(int64_t P, const float* __restrict__ g, float* __restrict__ out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < P; i += 256) s += g[i] * g[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Adam on the FP32 master copy with the gradient clipped to 2-norm <= clip
// (a non-finite gradient skips the step), then the BF16 copies W and W^T of
// every weight
__global__ void k_adam(int64_t P, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, const float* __restrict__ sqnorm, float clip, float lr, float b1,
                       float b2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float nrm = sqrtf(*sqnorm);
    if (!isfinite(nrm)) return;
    const float gi = g[i] * (nrm > clip ? clip / nrm : 1.f);
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / bc1) / (sqrtf(v / bc2) + eps);
}

__global__ void k_pack_bf16(int nw, const int64_t* __restrict__ table, const float* __restrict__ p,
                            short* __restrict__ wn, short* __restrict__ wt) {
    const int w = blockIdx.y;
    if (w >= nw) return;
    const int64_t off = table[3 * w], K = table[3 * w + 1], N = table[3 * w + 2];
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < K * N;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = idx / N, c = idx % N;
        const short v = to_bf16(p[off + idx]);
        wn[off + idx] = v;
        wt[off + c * K + k] = v;
    }
}

}  // namespace seasd

// ===========================================================================
// host side

using namespace seasd;

namespace {

constexpr int kH = 64;
constexpr float kClip = 1.0f;   // gradient 2-norm bound of an Adam step

struct Layout {
    int64_t W_in, b_in, W_uv[2], W_e[2], b_a[2], W_m[2], b_m[2], W_h[2], b_h[2], W_o, b_o, W_c, b_c, total;
    std::vector<int64_t> weights;   // (offset, fan_in, fan_out) triples
};

Layout make_layout() {
    Layout L{};
    int64_t off = 0;
    auto take = [&](int64_t size) {
        const int64_t o = off;
        off += size;
        return o;
    };
    auto weight = [&](int64_t K, int64_t N) {
        const int64_t o = take(K * N);
        L.weights.insert(L.weights.end(), {o, K, N});
        return o;
    };
    L.W_in = weight(16, kH);
    L.b_in = take(kH);
    for (int l = 0; l < 2; ++l) {
        L.W_uv[l] = weight(kH, 2 * kH);
        L.W_e[l] = weight(16, kH);
        L.b_a[l] = take(kH);
        L.W_m[l] = weight(kH, kH);
        L.b_m[l] = take(kH);
        L.W_h[l] = weight(2 * kH, kH);
        L.b_h[l] = take(kH);
    }
    L.W_o = weight(kH, 16);
    L.b_o = take(16);
    L.W_c = weight(kH, 16);
    L.b_c = take(16);
    L.total = off;
    return L;
}

inline unsigned grid1(int64_t work, int t) { return (unsigned)((work + t - 1) / t); }

uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t fnv1a(const void* data, size_t bytes, uint64_t h = 1469598103934665603ull) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < bytes; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

struct seasd_net_s {
    int device = 0;
    Layout lay;
    int64_t step = 0;
    bool bf_dirty = true;
    DevBuf params, grads, mom1, mom2, wn, wt, table;
    // graph of the current configuration
    int64_t n = 0, E = 0;
    DevBuf deg, rowptr, esrc, edst, erev, geo, fe, fn;
    // activations
    DevBuf h0, uv[2], a[2], m[2], g[2], r[2], hl[2], o, c;
    // backward workspace
    DevBuf dO, dC, dh, dh2, dhg, duv, dzn, dze, dze2, partial, bad, gnorm;
};

namespace seasd {

int64_t net_param_count(seasd_net net) { return net->lay.total; }

static int net_pack(seasd_net net, hipStream_t st) {
    if (!net->bf_dirty) return 0;
    const int nw = (int)(net->lay.weights.size() / 3);
    hipLaunchKernelGGL(k_pack_bf16, dim3(16, nw), dim3(256), 0, st, nw, net->table.as<int64_t>(),
                       net->params.as<float>(), net->wn.as<short>(), net->wt.as<short>());
    net->bf_dirty = false;
    return hipGetLastError() == hipSuccess ? 0 : SEASD_E_HIP;
}

int net_build_graph(seasd_net net, const ApplyArgs& A, hipStream_t st) {
    const int64_t n = A.n;
    int rc = 0;
    rc |= net->deg.ensure(sizeof(int) * n);
    rc |= net->rowptr.ensure(sizeof(int) * (n + 1));
    if (rc) return SEASD_E_NOMEM;
    if (launch_edge_count(A, kEdgeCut, net->deg.as<int>(), net->rowptr.as<int>(), st)) return SEASD_E_HIP;
    int E = 0;
    if (hipMemcpyAsync(&E, net->rowptr.as<int>() + n, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
        return SEASD_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SEASD_E_HIP;
    const size_t Ec = (size_t)(E > 0 ? E : 1);
    rc |= net->esrc.ensure(sizeof(int) * Ec);
    rc |= net->edst.ensure(sizeof(int) * Ec);
    rc |= net->erev.ensure(sizeof(int) * Ec);
    rc |= net->geo.ensure(sizeof(float4) * Ec);
    rc |= net->fe.ensure(sizeof(float) * 16 * Ec);
    rc |= net->fn.ensure(sizeof(float) * 16 * n);
    if (rc) return SEASD_E_NOMEM;
    if (launch_edge_fill(A, kEdgeCut, net->rowptr.as<int>(), net->esrc.as<int>(), net->edst.as<int>(),
                         net->erev.as<int>(), net->geo.as<float4>(), net->fe.as<float>(), net->fn.as<float>(), st))
        return SEASD_E_HIP;
    net->n = n;
    net->E = E;
    // activations
    const size_t nn = (size_t)n, ee = Ec;
    rc |= net->h0.ensure(sizeof(float) * kH * nn);
    for (int l = 0; l < 2; ++l) {
        rc |= net->uv[l].ensure(sizeof(float) * 2 * kH * nn);
        rc |= net->a[l].ensure(sizeof(float) * kH * ee);
        rc |= net->m[l].ensure(sizeof(float) * kH * ee);
        rc |= net->g[l].ensure(sizeof(float) * kH * nn);
        rc |= net->r[l].ensure(sizeof(float) * kH * nn);
        rc |= net->hl[l].ensure(sizeof(float) * kH * nn);
    }
    rc |= net->o.ensure(sizeof(float) * 16 * nn);
    rc |= net->c.ensure(sizeof(float) * 16 * ee);
    return rc ? SEASD_E_NOMEM : 0;
}

template <int K1, int K2, int NOUT, int EPI>
static void dense(int64_t R, const float* X1, const float* X2, const short* Wt, const float* bias, float* Y,
                  float* Y2, const float* base, const int* esrc, const int* edst, hipStream_t st) {
    if (R <= 0) return;
    const int64_t tiles = (R + 15) / 16;
    const unsigned blocks = (unsigned)std::min<int64_t>((tiles + 3) / 4, 4096);
    hipLaunchKernelGGL((k_dense<K1, K2, NOUT, EPI>), dim3(blocks), dim3(256), 0, st, R, X1, X2, Wt, bias, Y, Y2,
                       base, esrc, edst);
}

int net_forward(seasd_net net, hipStream_t st) {
    int rc = net_pack(net, st);
    if (rc) return rc;
    const Layout& L = net->lay;
    const float* P = net->params.as<float>();
    const short* WT = net->wt.as<short>();
    const int64_t n = net->n, E = net->E;
    dense<16, 0, 64, kEpiRelu>(n, net->fn.as<float>(), nullptr, WT + L.W_in, P + L.b_in, net->h0.as<float>(), nullptr,
                               nullptr, nullptr, nullptr, st);
    const float* h = net->h0.as<float>();
    for (int l = 0; l < 2; ++l) {
        dense<64, 0, 128, kEpiNone>(n, h, nullptr, WT + L.W_uv[l], nullptr, net->uv[l].as<float>(), nullptr, nullptr,
                                    nullptr, nullptr, st);
        dense<16, 0, 64, kEpiEdge>(E, net->fe.as<float>(), nullptr, WT + L.W_e[l], P + L.b_a[l], net->a[l].as<float>(),
                                   nullptr, net->uv[l].as<float>(), net->esrc.as<int>(), net->edst.as<int>(), st);
        dense<64, 0, 64, kEpiRelu>(E, net->a[l].as<float>(), nullptr, WT + L.W_m[l], P + L.b_m[l],
                                   net->m[l].as<float>(), nullptr, nullptr, nullptr, nullptr, st);
        hipLaunchKernelGGL(k_segsum, dim3(grid1(n * 64, 256)), dim3(256), 0, st, (int)n, net->rowptr.as<int>(),
                           net->m[l].as<float>(), kAgg, net->g[l].as<float>(), 64);
        dense<64, 64, 64, kEpiResid>(n, h, net->g[l].as<float>(), WT + L.W_h[l], P + L.b_h[l], net->hl[l].as<float>(),
                                     net->r[l].as<float>(), h, nullptr, nullptr, st);
        h = net->hl[l].as<float>();
    }
    dense<64, 0, 16, kEpiNone>(n, h, nullptr, WT + L.W_o, P + L.b_o, net->o.as<float>(), nullptr, nullptr, nullptr,
                               nullptr, st);
    dense<64, 0, 16, kEpiNone>(E, net->m[1].as<float>(), nullptr, WT + L.W_c, P + L.b_c, net->c.as<float>(), nullptr,
                               nullptr, nullptr, nullptr, st);
    return hipGetLastError() == hipSuccess ? 0 : SEASD_E_HIP;
}

int net_x0(seasd_net net, const double* inv, const int* perm, int nrhs, const double* b, const double* gin,
           double* x0, hipStream_t st) {
    const int64_t n = net->n, E = net->E;
    if (gin) {
        int rc = 0;
        rc |= net->dO.ensure(sizeof(float) * 16 * n);
        rc |= net->dC.ensure(sizeof(float) * 16 * (E > 0 ? E : 1));
        if (rc) return SEASD_E_NOMEM;
    }
    hipLaunchKernelGGL(k_x0_net, dim3(grid1(n, 64)), dim3(64), 0, st, (int)n, nrhs, perm, net->rowptr.as<int>(),
                       net->edst.as<int>(), net->geo.as<float4>(), inv, net->o.as<float>(), net->c.as<float>(), b, gin,
                       x0, net->dO.as<float>(), net->dC.as<float>());
    return hipGetLastError() == hipSuccess ? 0 : SEASD_E_HIP;
}

// grads[off..] = dW of one dense layer (and of its bias when boff >= 0)
template <int K1, int K2, int NOUT>
static int wgrad(seasd_net net, int64_t R, const float* X1, const float* X2, const float* dZ, int64_t woff,
                 int64_t boff, hipStream_t st) {
    float* G = net->grads.as<float>();
    constexpr int K = K1 + K2;
    if (R <= 0) {
        if (hipMemsetAsync(G + woff, 0, sizeof(float) * K * NOUT, st) != hipSuccess) return SEASD_E_HIP;
        if (boff >= 0 && hipMemsetAsync(G + boff, 0, sizeof(float) * NOUT, st) != hipSuccess) return SEASD_E_HIP;
        return 0;
    }
    int64_t chunk = ((R + 239) / 240 + 15) / 16 * 16;
    if (chunk < 256) chunk = 256;
    const int nparts = (int)((R + chunk - 1) / chunk);
    float* part = net->partial.as<float>();
    hipLaunchKernelGGL((k_wgrad<K1, K2, NOUT>), dim3(nparts), dim3(256), 0, st, R, chunk, X1, X2, dZ, part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(grid1(K * NOUT, 256)), dim3(256), 0, st, nparts, (int64_t)K * NOUT, part,
                       G + woff);
    if (boff >= 0) {
        hipLaunchKernelGGL((k_colsum<NOUT>), dim3(nparts), dim3(256), 0, st, R, chunk, dZ, part);
        hipLaunchKernelGGL(k_reduce_parts, dim3(grid1(NOUT, 64)), dim3(64), 0, st, nparts, (int64_t)NOUT, part,
                           G + boff);
    }
    return hipGetLastError() == hipSuccess ? 0 : SEASD_E_HIP;
}

int net_backward(seasd_net net, hipStream_t st) {
    const Layout& L = net->lay;
    const short* WN = net->wn.as<short>();
    const int64_t n = net->n, E = net->E, Ec = E > 0 ? E : 1;
    int rc = 0;
    rc |= net->dh.ensure(sizeof(float) * kH * n);
    rc |= net->dh2.ensure(sizeof(float) * kH * n);
    rc |= net->dhg.ensure(sizeof(float) * 2 * kH * n);
    rc |= net->duv.ensure(sizeof(float) * 2 * kH * n);
    rc |= net->dzn.ensure(sizeof(float) * kH * n);
    rc |= net->dze.ensure(sizeof(float) * kH * Ec);
    rc |= net->dze2.ensure(sizeof(float) * kH * Ec);
    rc |= net->partial.ensure(sizeof(float) * 240 * 128 * 64);
    if (rc) return SEASD_E_NOMEM;
    float* dh = net->dh.as<float>();
    float* dh2 = net->dh2.as<float>();
    float* dhg = net->dhg.as<float>();
    float* duv = net->duv.as<float>();
    float* dzn = net->dzn.as<float>();
    float* dze = net->dze.as<float>();
    float* dze2 = net->dze2.as<float>();
    const float* dO = net->dO.as<float>();
    const float* dC = net->dC.as<float>();
    // heads: dm_extra (edge rows) in dze2, dh in dh
    if ((rc = wgrad<64, 0, 16>(net, E, net->m[1].as<float>(), nullptr, dC, L.W_c, L.b_c, st))) return rc;
    dense<16, 0, 64, kEpiNone>(E, dC, nullptr, WN + L.W_c, nullptr, dze2, nullptr, nullptr, nullptr, nullptr, st);
    if ((rc = wgrad<64, 0, 16>(net, n, net->hl[1].as<float>(), nullptr, dO, L.W_o, L.b_o, st))) return rc;
    dense<16, 0, 64, kEpiNone>(n, dO, nullptr, WN + L.W_o, nullptr, dh, nullptr, nullptr, nullptr, nullptr, st);
    for (int l = 1; l >= 0; --l) {
        const float* hin = l == 0 ? net->h0.as<float>() : net->hl[0].as<float>();
        // update layer: dz = dh * (r > 0); d[h|g] = dz W_h^T
        hipLaunchKernelGGL(k_relu_back, dim3(grid1(n * 64, 256)), dim3(256), 0, st, n, dh, 64, net->r[l].as<float>(),
                           dzn);
        if ((rc = wgrad<64, 64, 64>(net, n, hin, net->g[l].as<float>(), dzn, L.W_h[l], L.b_h[l], st))) return rc;
        dense<64, 0, 128, kEpiNone>(n, dzn, nullptr, WN + L.W_h[l], nullptr, dhg, nullptr, nullptr, nullptr, nullptr,
                                    st);
        hipLaunchKernelGGL(k_add_half, dim3(grid1(n * 64, 256)), dim3(256), 0, st, n, dh, dhg, dh2);   // dh_in part
        // message: dz_m = (dg[src]/16 + extra) * (m > 0); da = dz_m W_m^T
        if (E > 0) {
            hipLaunchKernelGGL(k_msg_back, dim3(grid1(E * 64, 256)), dim3(256), 0, st, E, net->esrc.as<int>(), dhg,
                               kAgg, l == 1 ? dze2 : nullptr, net->m[l].as<float>(), dze);
        }
        if ((rc = wgrad<64, 0, 64>(net, E, net->a[l].as<float>(), nullptr, dze, L.W_m[l], L.b_m[l], st))) return rc;
        dense<64, 0, 64, kEpiNone>(E, dze, nullptr, WN + L.W_m[l], nullptr, dze2, nullptr, nullptr, nullptr, nullptr,
                                   st);
        // edge pre-activation: dz_a = da * (a > 0)
        if (E > 0)
            hipLaunchKernelGGL(k_relu_back, dim3(grid1(E * 64, 256)), dim3(256), 0, st, E, dze2, 64,
                               net->a[l].as<float>(), dze);
        if ((rc = wgrad<16, 0, 64>(net, E, net->fe.as<float>(), nullptr, dze, L.W_e[l], L.b_a[l], st))) return rc;
        hipLaunchKernelGGL(k_segsum_uv, dim3(grid1(n * 64, 256)), dim3(256), 0, st, (int)n, net->rowptr.as<int>(),
                           net->erev.as<int>(), dze, duv);
        if ((rc = wgrad<64, 0, 128>(net, n, hin, nullptr, duv, L.W_uv[l], -1, st))) return rc;
        // dh_in = dh2 + dUV W_uv^T
        dense<128, 0, 64, kEpiAdd>(n, duv, nullptr, WN + L.W_uv[l], nullptr, dh, nullptr, dh2, nullptr, nullptr, st);
    }
    hipLaunchKernelGGL(k_relu_back, dim3(grid1(n * 64, 256)), dim3(256), 0, st, n, dh, 64, net->h0.as<float>(), dzn);
    if ((rc = wgrad<16, 0, 64>(net, n, net->fn.as<float>(), nullptr, dzn, L.W_in, L.b_in, st))) return rc;
    return hipGetLastError() == hipSuccess ? 0 : SEASD_E_HIP;
}

int net_adam(seasd_net net, float lr, hipStream_t st) {
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.f - std::pow(b1, (float)net->step), bc2 = 1.f - std::pow(b2, (float)net->step);
    if (net->gnorm.ensure(sizeof(float))) return SEASD_E_NOMEM;
    hipLaunchKernelGGL(k_sqnorm, dim3(1), dim3(256), 0, st, net->lay.total, net->grads.as<float>(),
                       net->gnorm.as<float>());
    hipLaunchKernelGGL(k_adam, dim3(grid1(net->lay.total, 256)), dim3(256), 0, st, net->lay.total,
                       net->params.as<float>(), net->grads.as<float>(), net->mom1.as<float>(), net->mom2.as<float>(),
                       net->gnorm.as<float>(), kClip, lr, b1, b2, 1e-8f, bc1, bc2);
    net->bf_dirty = true;
    return hipGetLastError() == hipSuccess ? net_pack(net, st) : SEASD_E_HIP;
}

int net_learned_blocks(seasd_net net, const double* inv, const int* perm, double* out, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_learned_blocks, dim3(grid1(net->n, 128)), dim3(128), 0, st, (int)net->n, perm, inv,
                       net->o.as<float>(), out, bad);
    return hipGetLastError() == hipSuccess ? 0 : SEASD_E_HIP;
}

int check_finite(int64_t len, const double* x, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_nonfinite, dim3(grid1(len, 256)), dim3(256), 0, st, len, x, bad);
    return hipGetLastError() == hipSuccess ? 0 : SEASD_E_HIP;
}

int net_device(seasd_net net) { return net->device; }
int64_t net_edges(seasd_net net) { return net->E; }

int net_grads_to_host(seasd_net net, float* host, int64_t count, hipStream_t st) {
    if (count != net->lay.total) return SEASD_E_INVALID_ARG;
    if (hipMemcpyAsync(host, net->grads.p, sizeof(float) * count, hipMemcpyDeviceToHost, st) != hipSuccess)
        return SEASD_E_HIP;
    return hipStreamSynchronize(st) == hipSuccess ? 0 : SEASD_E_HIP;
}

}  // namespace seasd

// ---------------------------------------------------------------------------
// C ABI: network object, parameters, files

extern "C" int seasd_net_create(seasd_net* out, int32_t device, uint64_t seed) {
    if (!out) return SEASD_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SEASD_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return SEASD_E_HIP;
    auto* net = new seasd_net_s();
    net->device = device;
    net->lay = make_layout();
    const int64_t P = net->lay.total;
    int rc = 0;
    rc |= net->params.ensure(sizeof(float) * P);
    rc |= net->grads.ensure(sizeof(float) * P);
    rc |= net->mom1.ensure(sizeof(float) * P);
    rc |= net->mom2.ensure(sizeof(float) * P);
    rc |= net->wn.ensure(sizeof(short) * P);
    rc |= net->wt.ensure(sizeof(short) * P);
    rc |= net->table.ensure(sizeof(int64_t) * net->lay.weights.size());
    rc |= net->bad.ensure(sizeof(int));
    if (rc) {
        seasd_net_destroy(net);
        return SEASD_E_NOMEM;
    }
    // uniform(-sqrt(6/fan_in), +) weights from splitmix64 (fan_in counting the
    // used inputs: 4 node and 5 edge features), zero biases, heads x 0.01
    std::vector<float> p(P, 0.f);
    uint64_t state = seed;
    const Layout& L = net->lay;
    for (size_t w = 0; w < L.weights.size(); w += 3) {
        const int64_t off = L.weights[w], K = L.weights[w + 1], N = L.weights[w + 2];
        const bool node_in = off == L.W_in, edge_in = off == L.W_e[0] || off == L.W_e[1];
        const int64_t used = node_in ? 4 : (edge_in ? 5 : K);
        const double lim = std::sqrt(6.0 / used) * ((off == L.W_o || off == L.W_c) ? 0.01 : 1.0);
        for (int64_t k = 0; k < K; ++k)
            for (int64_t c = 0; c < N; ++c) {
                const double u = (splitmix64(state) >> 11) * (1.0 / 9007199254740992.0);
                p[off + k * N + c] = k < used ? (float)((2.0 * u - 1.0) * lim) : 0.f;
            }
    }
    std::vector<float> zero(P, 0.f);
    if (hipMemcpy(net->params.p, p.data(), sizeof(float) * P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->mom1.p, zero.data(), sizeof(float) * P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->mom2.p, zero.data(), sizeof(float) * P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->table.p, L.weights.data(), sizeof(int64_t) * L.weights.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
        seasd_net_destroy(net);
        return SEASD_E_HIP;
    }
    if (net_pack(net, nullptr) || hipDeviceSynchronize() != hipSuccess) {
        seasd_net_destroy(net);
        return SEASD_E_HIP;
    }
    *out = net;
    return SEASD_OK;
}

extern "C" int seasd_net_destroy(seasd_net net) {
    if (!net) return SEASD_OK;
    hipSetDevice(net->device);
    DevBuf* bufs[] = {&net->params, &net->grads, &net->mom1, &net->mom2, &net->wn, &net->wt, &net->table,
                      &net->deg, &net->rowptr, &net->esrc, &net->edst, &net->erev, &net->geo, &net->fe, &net->fn,
                      &net->h0, &net->uv[0], &net->uv[1], &net->a[0], &net->a[1], &net->m[0], &net->m[1],
                      &net->g[0], &net->g[1], &net->r[0], &net->r[1], &net->hl[0], &net->hl[1], &net->o, &net->c,
                      &net->dO, &net->dC, &net->dh, &net->dh2, &net->dhg, &net->duv, &net->dzn, &net->dze,
                      &net->dze2, &net->partial, &net->bad, &net->gnorm};
    for (DevBuf* b : bufs) b->release();
    delete net;
    return SEASD_OK;
}

extern "C" int64_t seasd_net_param_count(void) { return make_layout().total; }

extern "C" int seasd_net_get_params(seasd_net net, float* host, int64_t count) {
    if (!net || !host || count != net->lay.total) return SEASD_E_INVALID_ARG;
    if (hipSetDevice(net->device) != hipSuccess) return SEASD_E_HIP;
    if (hipDeviceSynchronize() != hipSuccess) return SEASD_E_HIP;
    return hipMemcpy(host, net->params.p, sizeof(float) * count, hipMemcpyDeviceToHost) == hipSuccess ? SEASD_OK
                                                                                                        : SEASD_E_HIP;
}

extern "C" int seasd_net_set_params(seasd_net net, const float* host, int64_t count) {
    if (!net || !host || count != net->lay.total) return SEASD_E_INVALID_ARG;
    if (hipSetDevice(net->device) != hipSuccess) return SEASD_E_HIP;
    if (hipDeviceSynchronize() != hipSuccess) return SEASD_E_HIP;
    if (hipMemcpy(net->params.p, host, sizeof(float) * count, hipMemcpyHostToDevice) != hipSuccess) return SEASD_E_HIP;
    net->bf_dirty = true;
    if (net_pack(net, nullptr) || hipDeviceSynchronize() != hipSuccess) return SEASD_E_HIP;
    return SEASD_OK;
}

// file: "SEASDNET" | u32 version | u32 reserved | i64 count | i64 step |
// f32 params[count] | f32 adam m[count] | f32 adam v[count] | u64 FNV-1a of
// everything before it
static constexpr uint32_t kNetVersion = 1;

extern "C" int seasd_net_save(seasd_net net, const char* path) {
    if (!net || !path) return SEASD_E_INVALID_ARG;
    if (hipSetDevice(net->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return SEASD_E_HIP;
    const int64_t P = net->lay.total;
    std::vector<unsigned char> buf(8 + 4 + 4 + 8 + 8 + 3 * 4 * (size_t)P);
    unsigned char* q = buf.data();
    std::memcpy(q, "SEASDNET", 8);
    std::memcpy(q + 8, &kNetVersion, 4);
    std::memset(q + 12, 0, 4);
    std::memcpy(q + 16, &P, 8);
    std::memcpy(q + 24, &net->step, 8);
    float* f = reinterpret_cast<float*>(q + 32);
    if (hipMemcpy(f, net->params.p, 4 * P, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(f + P, net->mom1.p, 4 * P, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(f + 2 * P, net->mom2.p, 4 * P, hipMemcpyDeviceToHost) != hipSuccess)
        return SEASD_E_HIP;
    const uint64_t sum = fnv1a(buf.data(), buf.size());
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return SEASD_E_FORMAT;
    const bool ok = std::fwrite(buf.data(), 1, buf.size(), fp) == buf.size() && std::fwrite(&sum, 8, 1, fp) == 1;
    return (std::fclose(fp) == 0 && ok) ? SEASD_OK : SEASD_E_FORMAT;
}

extern "C" int seasd_net_load(seasd_net net, const char* path) {
    if (!net || !path) return SEASD_E_INVALID_ARG;
    const int64_t P = net->lay.total;
    const size_t bytes = 32 + 3 * 4 * (size_t)P;
    std::vector<unsigned char> buf(bytes);
    uint64_t sum = 0;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return SEASD_E_FORMAT;
    const bool got = std::fread(buf.data(), 1, bytes, fp) == bytes && std::fread(&sum, 8, 1, fp) == 1;
    unsigned char extra;
    const bool at_end = std::fread(&extra, 1, 1, fp) == 0;
    std::fclose(fp);
    if (!got || !at_end) return SEASD_E_FORMAT;
    uint32_t ver = 0;
    int64_t cnt = 0, step = 0;
    std::memcpy(&ver, buf.data() + 8, 4);
    std::memcpy(&cnt, buf.data() + 16, 8);
    std::memcpy(&step, buf.data() + 24, 8);
    if (std::memcmp(buf.data(), "SEASDNET", 8) != 0 || ver != kNetVersion || cnt != P) return SEASD_E_FORMAT;
    if (fnv1a(buf.data(), bytes) != sum) return SEASD_E_FORMAT;
    if (hipSetDevice(net->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return SEASD_E_HIP;
    const float* f = reinterpret_cast<const float*>(buf.data() + 32);
    if (hipMemcpy(net->params.p, f, 4 * P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->mom1.p, f + P, 4 * P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->mom2.p, f + 2 * P, 4 * P, hipMemcpyHostToDevice) != hipSuccess)
        return SEASD_E_HIP;
    net->step = step;
    net->bf_dirty = true;
    if (net_pack(net, nullptr) || hipDeviceSynchronize() != hipSuccess) return SEASD_E_HIP;
    return SEASD_OK;
}
