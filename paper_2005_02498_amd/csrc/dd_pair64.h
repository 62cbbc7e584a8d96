// Per-pair device functions: contribution sigma^i(x) b_j of one source
// segment i to the stress at a target Gauss point x, already contracted with
// the target's Burgers vector (the Peach-Koehler force is linear in sigma,
// so partial sums of sigma b_j can be accumulated instead of 6 stresses).
//
// Closed form (lengths in units of the core width a, stress in units of mu):
// with R0 = x - x1, y = R0.t, rho = R0 - y t, d2 = rho.rho + 1, the endpoint
// coordinates u1 = -y and u2 = L - y, Ra_k = sqrt(d2 + u_k^2) and the line
// integrals I_{n,k} = int u^k Ra^-n du over [u1, u2] of the non-singular
// isotropic kernel, the field of the straight segment regroups as
//   sigma = S(t, w) + S(rho, z) + kd 1,    S(p, r) = p (x) r + r (x) p,
//   w  = -k1 g0 (rho x b) + (k2 I31 - k1 g1) c + q k2 (1.5 I52 t - 3 I51 rho)
//   z  = -k2 I30 c + 1.5 q k2 I50 rho
//   kd = q k2 (I30 + 3 I50)
// with c = b x t, q = c.rho, g0 = 2 I30 + 3 I50, g1 = 2 I31 + 3 I51,
// k1 = 1/(8 pi), k2 = 1/(4 pi (1 - nu)); then
//   sigma b_j = t (w.b_j) + w (t.b_j) + rho (z.b_j) + z (rho.b_j) + kd b_j.
#pragma once

#include <hip/hip_runtime.h>

namespace dd {

// 1/sqrt(x) and 1/x in FP64 for x >= 1 (every argument here is at least the
// squared core width, 1 in scaled units): the hardware estimate refined by one
// third-order step, Householder's iteration y <- y (1 + e/2 + 3 e^2/8) with
// e = 1 - x y^2 for the inverse square root, and r <- r (1 + e + e^2) with
// e = 1 - x r for the reciprocal.  Each step cubes the estimate's relative
// error.
__device__ __forceinline__ double rsqrt64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ double rcp64(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
}

// FP64: endpoint differences taken directly,
//   I30 = (s2 - s1)/d2, I31 = r1 - r2, I50 = ((3 s2 - s2^3) - (3 s1 - s1^3))/(3 d2^2),
//   I51 = (r1^3 - r2^3)/3, I52 = (s2^3 - s1^3)/(3 d2), with r = 1/Ra, s = u r.
// r at an endpoint depends only on the distance to that node, so when the
// source starts at the node where the previous source (same target point)
// ended, its r1 is the previous r2: `chained` (uniform across the wave) skips
// that inverse square root; `rprev` carries r2 to the next call.
__device__ __forceinline__ void pair_sigma_b_f64c(
    double x0, double x1, double x2, double bj0, double bj1, double bj2,
    double p0, double p1, double p2, double t0, double t1, double t2, double L,
    double b0, double b1, double b2, double c0, double c1, double c2,
    double k1, double k2, bool chained, double &rprev, double &o0, double &o1, double &o2)
{
    const double R0 = x0 - p0, R1 = x1 - p1, R2 = x2 - p2;
    const double y = R0 * t0 + R1 * t1 + R2 * t2;
    const double h0 = R0 - y * t0, h1 = R1 - y * t1, h2 = R2 - y * t2;   // rho
    const double d2 = h0 * h0 + h1 * h1 + h2 * h2 + 1.0;
    const double u2 = L - y;
    double r1;
    if (chained) r1 = rprev;
    else r1 = rsqrt64(d2 + y * y);
    const double r2 = rsqrt64(d2 + u2 * u2);
    rprev = r2;
    const double id2 = rcp64(d2);
    const double s1 = -y * r1, s2 = u2 * r2;
    const double s1c = s1 * s1 * s1, s2c = s2 * s2 * s2;
    const double I30 = (s2 - s1) * id2;
    const double I31 = r1 - r2;
    const double I50 = ((3.0 * s2 - s2c) - (3.0 * s1 - s1c)) * (id2 * id2) * (1.0 / 3.0);
    const double I51 = (r1 * r1 * r1 - r2 * r2 * r2) * (1.0 / 3.0);
    const double I52 = (s2c - s1c) * id2 * (1.0 / 3.0);
    const double g0 = 2.0 * I30 + 3.0 * I50;
    const double g1 = 2.0 * I31 + 3.0 * I51;
    const double q = c0 * h0 + c1 * h1 + c2 * h2;
    const double rb0 = h1 * b2 - h2 * b1, rb1 = h2 * b0 - h0 * b2, rb2 = h0 * b1 - h1 * b0;
    const double A = -k1 * g0, Cc = k2 * I31 - k1 * g1, qk = q * k2;
    const double Tt = 1.5 * qk * I52, Tr = -3.0 * qk * I51;
    const double Zc = -k2 * I30, Zr = 1.5 * qk * I50;
    const double kd = qk * (I30 + 3.0 * I50);
    // sigma b_j = t (w.b_j) + w (t.b_j) + rho (z.b_j) + z (rho.b_j) + kd b_j, with w and z
    // expanded: coefficients of the five vectors rho x b, c, t, rho and b_j
    const double tb = t0 * bj0 + t1 * bj1 + t2 * bj2;
    const double hb = h0 * bj0 + h1 * bj1 + h2 * bj2;
    const double cb = c0 * bj0 + c1 * bj1 + c2 * bj2;
    const double rbb = rb0 * bj0 + rb1 * bj1 + rb2 * bj2;
    const double wb = A * rbb + Cc * cb + Tt * tb + Tr * hb;
    const double zb = Zc * cb + Zr * hb;
    const double Pr = A * tb, Pc = Cc * tb + Zc * hb, Pt = wb + Tt * tb, Ph = Tr * tb + zb + Zr * hb;
    o0 = Pr * rb0 + Pc * c0 + Pt * t0 + Ph * h0 + kd * bj0;
    o1 = Pr * rb1 + Pc * c1 + Pt * t1 + Ph * h1 + kd * bj1;
    o2 = Pr * rb2 + Pc * c2 + Pt * t2 + Ph * h2 + kd * bj2;
}

// Unchained form (isolated pairs, e.g. the near-field branch of the mixed path).
__device__ __forceinline__ void pair_sigma_b_f64(
    double x0, double x1, double x2, double bj0, double bj1, double bj2,
    double p0, double p1, double p2, double t0, double t1, double t2, double L,
    double b0, double b1, double b2, double c0, double c1, double c2,
    double k1, double k2, double &o0, double &o1, double &o2)
{
    double r = 0.0;
    pair_sigma_b_f64c(x0, x1, x2, bj0, bj1, bj2, p0, p1, p2, t0, t1, t2, L, b0, b1, b2, c0, c1,
                      c2, k1, k2, false, r, o0, o1, o2);
}

}  // namespace dd
