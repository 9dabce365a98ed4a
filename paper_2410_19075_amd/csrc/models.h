// Per-element model arithmetic shared by the ring and lattice kernels: the
// stage value, the coupling map and the local right-hand side.
#pragma once

#include "nd_dev.h"

namespace nd {


// ------------------------------------------------------------------ models
// sin and cos of one double: Cody-Waite reduction by pi/2 (two-part constant,
// each part subtracted with one fused multiply-add), then the Taylor series of
// sin and cos on [-pi/4, pi/4] up to degrees 15 and 16 (truncation below 5e-17)
// evaluated by Horner in r^2, and the quadrant swap.  The reduced argument
// carries the rounding of the first subtraction (up to half an ulp of r, about
// 5.5e-17 near pi/4) and the neglected third part of pi/2 (grows with |x|);
// measured against glibc over 1.6e7 arguments up to 3e13 the largest absolute
// error was 1.1e-16.  Inf and NaN give NaN.
__device__ __forceinline__ void sincos_cw(double x, double* sp, double* cp) {
    const double q = rint(x * 0.63661977236758134308);          // x / (pi/2), nearest
    const double r1 = fma(-q, 1.5707963267948966192, x);        // pi/2 rounded to double
    const double r = fma(-q, 6.123233995736766036e-17, r1);     // pi/2 minus that
    const double r2 = r * r;
    double ps = -1.0 / 1307674368000.0;                          // -1/15!
    ps = fma(ps, r2, 1.0 / 6227020800.0);
    ps = fma(ps, r2, -1.0 / 39916800.0);
    ps = fma(ps, r2, 1.0 / 362880.0);
    ps = fma(ps, r2, -1.0 / 5040.0);
    ps = fma(ps, r2, 1.0 / 120.0);
    ps = fma(ps, r2, -1.0 / 6.0);
    const double sn = fma(r * r2, ps, r);
    double pc = 1.0 / 20922789888000.0;                          // 1/16!
    pc = fma(pc, r2, -1.0 / 87178291200.0);
    pc = fma(pc, r2, 1.0 / 479001600.0);
    pc = fma(pc, r2, -1.0 / 3628800.0);
    pc = fma(pc, r2, 1.0 / 40320.0);
    pc = fma(pc, r2, -1.0 / 720.0);
    pc = fma(pc, r2, 1.0 / 24.0);
    pc = fma(pc, r2, -0.5);
    const double cs = fma(r2, pc, 1.0);
    const int k = (int)(q - 4.0 * floor(q * 0.25));  // quadrant q mod 4, exact for any integer q  // two's complement: also right for negative q
    const double s0 = (k & 1) ? cs : sn, c0 = (k & 1) ? sn : cs;
    *sp = (k & 2) ? -s0 : s0;
    *cp = ((k + 1) & 2) ? -c0 : c0;
}

template <int MODEL, class KT>
struct RingModel;

// Kuramoto-Sakaguchi, Eq. (3) with m = 0, eps = 1:
//   k_i = omega + mu/(2P) sum_j sin(z_j - z_i - alpha)
//       = omega + mu/(2P) [cos(z_i + alpha) S_i - sin(z_i + alpha) C_i]
// with (C_i, S_i) the window sums of (cos z_j, sin z_j).
// p = {omega, mu/(2P), cos alpha, sin alpha}
template <class KT>
struct RingModel<ND_KURAMOTO, KT> {
    static constexpr int V = 1;
    __device__ static __forceinline__ double2 map(const double* z) {
        double s, c;
        if constexpr (sizeof(KT) == 8) {
            sincos_cw(z[0], &s, &c);
        } else {
            // bulk float: reduce to revolutions in double, then the hardware
            // sin/cos (their argument is in revolutions)
            double r = z[0] * 0.15915494309189535;  // 1 / (2 pi)
            r -= rint(r);
            float rf = (float)r;
            s = (double)__builtin_amdgcn_sinf(rf);
            c = (double)__builtin_amdgcn_cosf(rf);
        }
        return make_double2(c, s);
    }
    __device__ static __forceinline__ void rhs(const NetDesc& d, const double* z, double2 xo, double2 W,
                                               double* k) {
        (void)z;
        if constexpr (sizeof(KT) == 8) {
            const double ca = xo.x * d.p[2] - xo.y * d.p[3];
            const double sa = xo.y * d.p[2] + xo.x * d.p[3];
            k[0] = d.p[0] + d.p[1] * (ca * W.y - sa * W.x);
        } else {
            const float cf = (float)xo.x, sf = (float)xo.y;
            const float ca = cf * (float)d.p[2] - sf * (float)d.p[3];
            const float sa = sf * (float)d.p[2] + cf * (float)d.p[3];
            k[0] = d.p[0] + d.p[1] * ((double)ca * W.y - (double)sa * W.x);
        }
    }
};

// Kuramoto-Sakaguchi with inertia, Eq. (3) with m != 0, as a first-order
// system in (phi, psi = dphi/dt); the coupling is the Kuramoto one on phi:
//   dphi = psi,  dpsi = (omega - eps psi + mu/L [cos(phi+alpha) S - sin(phi+alpha) C]) / m
// p = {omega, mu/L, cos alpha, sin alpha, eps, 1/m}
template <class KT>
struct RingModel<ND_KURAMOTO_INERTIA, KT> {
    static constexpr int V = 2;
    __device__ static __forceinline__ double2 map(const double* z) { return RingModel<ND_KURAMOTO, KT>::map(z); }
    __device__ static __forceinline__ void rhs(const NetDesc& d, const double* z, double2 xo, double2 W,
                                               double* k) {
        double force[1];
        RingModel<ND_KURAMOTO, KT>::rhs(d, z, xo, W, force);  // omega + coupling, as first-order Kuramoto
        k[0] = z[1];
        if constexpr (sizeof(KT) == 8) {
            k[1] = fma(-d.p[4], z[1], force[0]) * d.p[5];
        } else {
            k[1] = (double)(((float)force[0] - (float)d.p[4] * (float)z[1]) * (float)d.p[5]);
        }
    }
};

// FitzHugh-Nagumo, Eq. (2) (tau = 0, D = 0, I_app = 0) with the rotational
// coupling B(phi) on (u_j - u_i, v_j - v_i), kappa = sigma / 2P:
//   eps du = u - u^3/3 - v + kappa ( cos phi Du + sin phi Dv)
//       dv = u + a         + kappa (-sin phi Du + cos phi Dv)
// Du = sum_j u_j - 2P u_i, Dv likewise (double, before any rounding to float).
// The divisions by 3 and eps are multiplications by the rounded reciprocals
// (a last-bit difference from the division; no division sequence per element).
// p = {eps, a, kappa, cos phi, sin phi, 2P, 1/eps}
template <class KT>
struct RingModel<ND_FHN, KT> {
    static constexpr int V = 2;
    __device__ static __forceinline__ double2 map(const double* z) { return make_double2(z[0], z[1]); }
    __device__ static __forceinline__ void rhs(const NetDesc& d, const double* z, double2 xo, double2 W,
                                               double* k) {
        (void)xo;
        const double u = z[0], v = z[1];
        const double Du = W.x - d.p[5] * u;
        const double Dv = W.y - d.p[5] * v;
        if constexpr (sizeof(KT) == 8) {
            const double cu = d.p[2] * (d.p[3] * Du + d.p[4] * Dv);
            const double cv = d.p[2] * (d.p[3] * Dv - d.p[4] * Du);
            k[0] = (u - u * u * u * (1.0 / 3.0) - v + cu) * d.p[6];
            k[1] = u + d.p[1] + cv;
        } else {
            const float uf = (float)u, vf = (float)v, duf = (float)Du, dvf = (float)Dv;
            const float kap = (float)d.p[2], cph = (float)d.p[3], sph = (float)d.p[4];
            const float cu = kap * (cph * duf + sph * dvf);
            const float cv = kap * (cph * dvf - sph * duf);
            k[0] = (double)((uf - uf * uf * uf * (1.0f / 3.0f) - vf + cu) * (float)d.p[6]);
            k[1] = (double)(uf + (float)d.p[1] + cv);
        }
    }
};

template <class KT>
__device__ __forceinline__ double kq(double k) {
    return (double)(KT)k;  // the value that is stored (and that every reader sees)
}

// Stage value z_v(idx) = y + c dt k_prev (stage 1: y).  Written once here so the
// producer of the tile sums and every reader of the window ends agree bitwise.
template <int V, class KT, class YP, class KP>
__device__ __forceinline__ void stage_z(YP y, KP kp, double cdt, int64_t n, int64_t idx, double* z) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const double yy = y[v * n + idx];
        z[v] = kp ? fma(cdt, (double)kp[v * n + idx], yy) : yy;
    }
}

}  // namespace nd
