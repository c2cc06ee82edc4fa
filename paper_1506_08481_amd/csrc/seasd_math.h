// seasd_math.h - scalar physics of the mobility product, shared by the
// kernels: the real-space pair coupling, the self terms and the basis maps.
//
// Real-space pair coupling (Sec. 2.1-2.3 and 3.3). For r = r_i - r_j the
// velocity field of sphere j's moments, read through sphere i's Faxen laws,
// is a set of differential operators acting on two screened radial kernels:
//   chi(r) = r erfc(xi r) - exp(-xi^2 r^2)/(xi sqrt(pi))  (the bracket of
//            eq. oseen-ewald-rs; J_R = (I lap - grad grad) chi),
//   phi(r) = erfc(xi r)/(4 pi r)                         (eq. source-split).
// Derivatives of a radial f are expressed through its hierarchy
// f_n = ((1/r) d/dr)^n f: grad f = r f_1, grad grad f = I f_1 + r r f_2, ...;
// and the Laplacian maps hierarchies as (lap f)_n = (2n+3) f_(n+1) + r^2 f_(n+2).
// For erfc(xi r)/r the hierarchy is (-1)^n B_n with the upward recurrence
// B_n = [(2n-1) B_(n-1) + (2 xi^2)^n exp(-xi^2 r^2)/(xi sqrt(pi))] / r^2, so
// chi_n = (-1)^(n-1) B_(n-1) and phi_n = (-1)^n B_n / (4 pi).
// The Faxen factors (1 + a^2 lap/6) on force/velocity and (1 + a^2 lap/10) on
// stresslet/strain (eqs. faxen-f, faxen-s, mul-expand) become polynomials in
// these Laplacian hierarchies; every block below is written as a contraction
// of the moments with r, the identity and those scalar functions.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace seasd {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;
constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kSqrt3 = 1.73205080756887729353;
constexpr double kSqrt6 = 2.44948974278317809820;

template <typename R>
__host__ __device__ inline R erfc_(R v);
template <>
__host__ __device__ inline double erfc_<double>(double v) { return erfc(v); }
template <>
__host__ __device__ inline float erfc_<float>(float v) { return erfcf(v); }

template <typename R>
__host__ __device__ inline R exp_(R v);
template <>
__host__ __device__ inline double exp_<double>(double v) { return exp(v); }
template <>
__host__ __device__ inline float exp_<float>(float v) { return expf(v); }

// Traceless-symmetric coordinates (orthonormal basis) -> tensor (6 unique:
// xx, yy, zz, xy, xz, yz).
template <typename R>
__host__ __device__ inline void s5_to_sym(const R* s, R* S) {
    const R i2 = R(1.0 / kSqrt2), i6 = R(1.0 / kSqrt6);
    S[0] = s[0] * i2 - s[1] * i6;
    S[1] = -s[0] * i2 - s[1] * i6;
    S[2] = R(2) * s[1] * i6;
    S[3] = s[2] * i2;
    S[4] = s[3] * i2;
    S[5] = s[4] * i2;
}

// Symmetric tensor (xx, yy, zz, xy, xz, yz) -> its five traceless coordinates.
template <typename R>
__host__ __device__ inline void sym_to_e5(const R* X, R* e) {
    const R i2 = R(1.0 / kSqrt2), i6 = R(1.0 / kSqrt6), s2 = R(kSqrt2);
    e[0] = (X[0] - X[1]) * i2;
    e[1] = (R(2) * X[2] - X[0] - X[1]) * i6;
    e[2] = s2 * X[3];
    e[3] = s2 * X[4];
    e[4] = s2 * X[5];
}

// Single-sphere mobility minus the continuum wave-space self term, per
// component group (eq. uf-self for U; the spin, strain and trace rows follow
// from the same integral of the i=j wave-space symbol).
template <typename R>
__host__ __device__ inline void self_diag(R a, R xi, R eta, R* d4) {
    const R p32 = R(kPi * kSqrtPi);
    const R a2 = a * a, x2 = xi * xi;
    d4[0] = R(1) / (R(6 * kPi) * eta * a) -
            xi * (R(9) - R(10) * a2 * x2 + R(7) * a2 * a2 * x2 * x2) / (R(18) * p32 * eta);
    d4[1] = R(1) / (R(8 * kPi) * eta * a * a2) - R(5) * xi * x2 / (R(12) * p32 * eta);
    d4[2] = R(3) / (R(20 * kPi) * eta * a * a2) -
            xi * x2 * (R(25) - R(42) * a2 * x2 + R(27) * a2 * a2 * x2 * x2) / (R(50) * p32 * eta);
    d4[3] = R(3) / (R(16 * kPi) * eta * a * a2);
}

// Accumulate into y (12 values) the real-space coupling of target i with
// source moments xj (12 values: F3, T3, S5, s6) at displacement d = r_i - r_j.
template <typename R>
__host__ __device__ inline void pair_coupling(R dx, R dy, R dz, R ai, R aj, R xi, R inv_eta,
                                              const R* xj, R* y) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R r = sqrt(r2);
    const R ir2 = R(1) / r2;
    // B_0 .. B_7
    R B[8];
    B[0] = erfc_<R>(xi * r) / r;
    const R g = exp_<R>(-xi * xi * r2) / (xi * R(kSqrtPi));
    R tx = R(2) * xi * xi, txn = tx;
    for (int n = 1; n < 8; ++n) {
        B[n] = (R(2 * n - 1) * B[n - 1] + txn * g) * ir2;
        txn *= tx;
    }
    // chi_1..chi_8 (index 0 unused)
    R c[9];
    for (int n = 1; n <= 8; ++n) c[n] = (n & 1) ? B[n - 1] : -B[n - 1];
    // (lap chi)_n, n = 1..6 and (lap^2 chi)_n, n = 1..4
    R L1[7], L2[5];
    for (int n = 1; n <= 6; ++n) L1[n] = R(2 * n + 3) * c[n + 1] + r2 * c[n + 2];
    for (int n = 1; n <= 4; ++n) L2[n] = R(2 * n + 3) * L1[n + 1] + r2 * L1[n + 2];
    // phi_1..phi_4 and (lap phi)_1..2
    const R i4p = R(1.0 / (4 * kPi));
    R ph[5];
    for (int n = 1; n <= 4; ++n) ph[n] = ((n & 1) ? -B[n] : B[n]) * i4p;
    R LP[3];
    for (int n = 1; n <= 2; ++n) LP[n] = R(2 * n + 3) * ph[n + 1] + r2 * ph[n + 2];

    const R Ai = ai * ai, Aj = aj * aj;
    const R i6 = R(1) / R(6), i10 = R(1) / R(10);
    // composite (1 + al lap)(1 + be lap) chi at index n
    auto comp = [&](R al, R be, int n) { return c[n] + (al + be) * L1[n] + al * be * L2[n]; };

    const R F0 = xj[0], F1 = xj[1], F2 = xj[2];
    const R T0 = xj[3], T1 = xj[4], T2 = xj[5];
    R S[6];
    s5_to_sym(xj + 6, S);
    const R s6 = xj[11];
    const R Srx = S[0] * dx + S[3] * dy + S[4] * dz;
    const R Sry = S[3] * dx + S[1] * dy + S[5] * dz;
    const R Srz = S[4] * dx + S[5] * dy + S[2] * dz;
    const R rSr = dx * Srx + dy * Sry + dz * Srz;
    const R rF = dx * F0 + dy * F1 + dz * F2;
    const R rT = dx * T0 + dy * T1 + dz * T2;
    const R c8 = inv_eta * R(1.0 / (8 * kPi));
    const R c16 = inv_eta * R(1.0 / (16 * kPi));
    const R c32 = inv_eta * R(1.0 / (32 * kPi));
    const R cq = inv_eta * R(kSqrt3 / 4);

    // ---- velocity row
    R u0, u1, u2;
    {   // U <- F: (1/8pi eta)[(2 psi_1 + r^2 psi_2) F - psi_2 r (r.F)]
        const R p1 = comp(Ai * i6, Aj * i6, 1), p2 = comp(Ai * i6, Aj * i6, 2);
        const R a = c8 * (R(2) * p1 + r2 * p2), b = -c8 * p2 * rF;
        u0 = a * F0 + b * dx;
        u1 = a * F1 + b * dy;
        u2 = a * F2 + b * dz;
    }
    {   // U <- T: (1/16pi eta) g_1 (r x T), g = (1 + Ai lap/6) lap chi
        const R g1 = c16 * (L1[1] + Ai * i6 * L2[1]);
        u0 += g1 * (dy * T2 - dz * T1);
        u1 += g1 * (dz * T0 - dx * T2);
        u2 += g1 * (dx * T1 - dy * T0);
    }
    {   // U <- S: -(1/8pi eta)[(3 psi_2 + r^2 psi_3) S r - psi_3 r (r.S.r)]
        const R p2 = comp(Ai * i6, Aj * i10, 2), p3 = comp(Ai * i6, Aj * i10, 3);
        const R a = -c8 * (R(3) * p2 + r2 * p3), b = c8 * p3 * rSr;
        u0 += a * Srx + b * dx;
        u1 += a * Sry + b * dy;
        u2 += a * Srz + b * dz;
    }
    {   // U <- s6: source flow, -(sqrt3/4 eta) psi_1 r s6, psi = (1 + Ai lap/6) phi
        const R q = -cq * (ph[1] + Ai * i6 * LP[1]) * s6;
        u0 += q * dx;
        u1 += q * dy;
        u2 += q * dz;
    }
    // ---- spin row
    R w0, w1, w2;
    {   // W <- F: (1/16pi eta) (lap psi)_1 (r x F), psi = (1 + Aj lap/6) chi
        const R g1 = c16 * (L1[1] + Aj * i6 * L2[1]);
        w0 = g1 * (dy * F2 - dz * F1);
        w1 = g1 * (dz * F0 - dx * F2);
        w2 = g1 * (dx * F1 - dy * F0);
    }
    {   // W <- T: (1/32pi eta)[g_2 r (r.T) - (2 g_1 + r^2 g_2) T], g = lap chi
        const R a = -c32 * (R(2) * L1[1] + r2 * L1[2]), b = c32 * L1[2] * rT;
        w0 += a * T0 + b * dx;
        w1 += a * T1 + b * dy;
        w2 += a * T2 + b * dz;
    }
    {   // W <- S: -(1/16pi eta) g_2 (r x S r), g = lap (1 + Aj lap/10) chi
        const R g2 = -c16 * (L1[2] + Aj * i10 * L2[2]);
        w0 += g2 * (dy * Srz - dz * Sry);
        w1 += g2 * (dz * Srx - dx * Srz);
        w2 += g2 * (dx * Sry - dy * Srx);
    }
    // ---- strain row, accumulated as a symmetric tensor X (xx,yy,zz,xy,xz,yz)
    R X[6];
    {   // E <- F: (1/8pi eta)[(3 psi_2 + r^2 psi_3) sym(F r) - psi_3 (r.F) r r]
        const R p2 = comp(Ai * i10, Aj * i6, 2), p3 = comp(Ai * i10, Aj * i6, 3);
        const R a = c8 * (R(3) * p2 + r2 * p3), b = -c8 * p3 * rF;
        X[0] = a * F0 * dx + b * dx * dx;
        X[1] = a * F1 * dy + b * dy * dy;
        X[2] = a * F2 * dz + b * dz * dz;
        X[3] = a * R(0.5) * (F0 * dy + F1 * dx) + b * dx * dy;
        X[4] = a * R(0.5) * (F0 * dz + F2 * dx) + b * dx * dz;
        X[5] = a * R(0.5) * (F1 * dz + F2 * dy) + b * dy * dz;
    }
    {   // E <- T: (1/16pi eta) g_2 sym(r (r x T)), g = (1 + Ai lap/10) lap chi
        const R g2 = c16 * (L1[2] + Ai * i10 * L2[2]);
        const R v0 = dy * T2 - dz * T1, v1 = dz * T0 - dx * T2, v2 = dx * T1 - dy * T0;
        X[0] += g2 * dx * v0;
        X[1] += g2 * dy * v1;
        X[2] += g2 * dz * v2;
        X[3] += g2 * R(0.5) * (dx * v1 + dy * v0);
        X[4] += g2 * R(0.5) * (dx * v2 + dz * v0);
        X[5] += g2 * R(0.5) * (dy * v2 + dz * v1);
    }
    {   // E <- S: -(1/8pi eta)[(3 psi_2 + r^2 psi_3) S + (3 psi_3 + r^2 psi_4) sym(r S r)
        //                      - psi_4 (r.S.r) r r], psi = (1 + Ai lap/10)(1 + Aj lap/10) chi
        const R al = Ai * i10, be = Aj * i10;
        const R p2 = comp(al, be, 2), p3 = comp(al, be, 3), p4 = comp(al, be, 4);
        const R a = -c8 * (R(3) * p2 + r2 * p3);
        const R b = -c8 * (R(3) * p3 + r2 * p4);
        const R cc = c8 * p4 * rSr;
        X[0] += a * S[0] + b * dx * Srx + cc * dx * dx;
        X[1] += a * S[1] + b * dy * Sry + cc * dy * dy;
        X[2] += a * S[2] + b * dz * Srz + cc * dz * dz;
        X[3] += a * S[3] + b * R(0.5) * (dx * Sry + dy * Srx) + cc * dx * dy;
        X[4] += a * S[4] + b * R(0.5) * (dx * Srz + dz * Srx) + cc * dx * dz;
        X[5] += a * S[5] + b * R(0.5) * (dy * Srz + dz * Sry) + cc * dy * dz;
    }
    {   // E <- s6: -(sqrt3/4 eta) psi_2 s6 r r, psi = (1 + Ai lap/10) phi
        const R q = -cq * (ph[2] + Ai * i10 * LP[2]) * s6;
        X[0] += q * dx * dx;
        X[1] += q * dy * dy;
        X[2] += q * dz * dz;
        X[3] += q * dx * dy;
        X[4] += q * dx * dz;
        X[5] += q * dy * dz;
    }
    // ---- trace row: pressure Faxen law, -(sqrt3/4 eta) p'(r_i)
    const R e6 = cq * rF * (ph[1] + Aj * i6 * LP[1]) - cq * rSr * (ph[2] + Aj * i10 * LP[2]);

    R e[5];
    sym_to_e5(X, e);
    y[0] += u0;
    y[1] += u1;
    y[2] += u2;
    y[3] += w0;
    y[4] += w1;
    y[5] += w2;
    y[6] += e[0];
    y[7] += e[1];
    y[8] += e[2];
    y[9] += e[3];
    y[10] += e[4];
    y[11] += e6;
}

}  // namespace seasd
