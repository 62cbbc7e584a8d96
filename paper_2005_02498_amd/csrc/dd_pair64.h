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
//
// The device form divides by k2 (the caller scales the sum once): with
// kr = k1/k2 = (1 - nu)/2 and k2 - 2 k1 = nu k2 the coefficients become
//   w/k2  = -kr g0 (rho x b) + (nu I31 - kr D51) c + q (P/2 t - D51 rho)
//   z/k2  = -I30 c + q E50/2 rho,       kd/k2 = q (I30 + E50)
// in terms of D51 = 3 I51 = r1^3 - r2^3, P = 3 I52 and E50 = 3 I50, with
// r = 1/Ra and s = u r at the two endpoints:
//   I30 = (s2 - s1)/d2,  P = (s2^3 - s1^3)/d2 = I30 (s1^2 + s1 s2 + s2^2),
//   E50 = (3 I30 - P)/d2,
//   I31 = r1 - r2,       g0 = 2 I30 + E50.
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

// Adds sigma^i b_j / k2 of source (p, t, L, b, c) at target point x to
// (a0, a1, a2) + ak b_j: the kd b_j term is returned as its scalar kd, added
// to ak, since b_j is the same for every source of a target point (the caller
// adds ak b_j once).  r1 and r1c = r1^3 belong to the source's first node and
// are supplied by the caller; r2 and r2c are returned, so that a source
// starting where this one ends (same target point) reuses them as its r1,
// r1c.  kr = (1 - nu)/2.
__device__ __forceinline__ void pair_acc_f64(
    double x0, double x1, double x2, double bj0, double bj1, double bj2,
    double p0, double p1, double p2, double t0, double t1, double t2, double L,
    double b0, double b1, double b2, double c0, double c1, double c2,
    double kr, double nu, double r1, double r1c, double &r2, double &r2c,
    double &a0, double &a1, double &a2, double &ak)
{
    const double R0 = x0 - p0, R1 = x1 - p1, R2 = x2 - p2;
    const double y = fma(R2, t2, fma(R1, t1, R0 * t0));
    const double h0 = fma(-y, t0, R0), h1 = fma(-y, t1, R1), h2 = fma(-y, t2, R2);   // rho
    const double d2 = fma(h2, h2, fma(h1, h1, fma(h0, h0, 1.0)));
    const double u2 = L - y;
    r2 = rsqrt64(fma(u2, u2, d2));
    r2c = r2 * r2 * r2;
    const double id2 = rcp64(d2);
    const double s1 = -y * r1, s2 = u2 * r2;
    const double D1 = s2 - s1;
    const double I30 = D1 * id2;
    const double P = I30 * fma(s1, s1 + s2, s2 * s2);   // s2^3 - s1^3 = D1 (s1^2 + s1 s2 + s2^2)
    const double E50 = fma(3.0, I30, -P) * id2;
    const double I31 = r1 - r2;
    const double D51 = r1c - r2c;
    const double g0 = fma(2.0, I30, E50);
    const double q = fma(c2, h2, fma(c1, h1, c0 * h0));
    const double A = -kr * g0;
    const double Cc = fma(nu, I31, -kr * D51);
    ak = fma(q, I30 + E50, ak);   // kd
    const double rb0 = fma(h1, b2, -h2 * b1), rb1 = fma(h2, b0, -h0 * b2), rb2 = fma(h0, b1, -h1 * b0);
    // sigma b_j = t (w.b_j) + w (t.b_j) + rho (z.b_j) + z (rho.b_j) + kd b_j, with w and z
    // expanded: coefficients of the four vectors rho x b, c, t, rho (q P/2 and -q D51 are
    // the t and rho coefficients of w/k2, q E50/2 the rho coefficient of z/k2)
    const double tb = fma(t2, bj2, fma(t1, bj1, t0 * bj0));
    const double hb = fma(h2, bj2, fma(h1, bj1, h0 * bj0));
    const double cb = fma(c2, bj2, fma(c1, bj1, c0 * bj0));
    const double rbb = fma(rb2, bj2, fma(rb1, bj1, rb0 * bj0));
    const double Pt = fma(q, fma(P, tb, -D51 * hb), fma(Cc, cb, A * rbb));
    const double Ph = fma(q, fma(E50, hb, -D51 * tb), -I30 * cb);
    const double Pc = fma(Cc, tb, -I30 * hb);
    const double Pr = A * tb;
    a0 = fma(Ph, h0, fma(Pt, t0, fma(Pc, c0, fma(Pr, rb0, a0))));
    a1 = fma(Ph, h1, fma(Pt, t1, fma(Pc, c1, fma(Pr, rb1, a1))));
    a2 = fma(Ph, h2, fma(Pt, t2, fma(Pc, c2, fma(Pr, rb2, a2))));
}

// One isolated pair (the near-field branch of the mixed path): adds
// sigma^i b_j / k2 of the source whose FP64 record is d (x1, t, L, b, c in
// entries 0..12) to (a0, a1, a2).
__device__ __forceinline__ void pair_acc_isolated_f64(double x0, double x1, double x2, double bj0,
                                                      double bj1, double bj2, const double *d,
                                                      double kr, double nu, double &a0, double &a1,
                                                      double &a2)
{
    const double R0 = x0 - d[0], R1 = x1 - d[1], R2 = x2 - d[2];
    const double r1 = rsqrt64(fma(R2, R2, fma(R1, R1, fma(R0, R0, 1.0))));
    double r2, r2c, ak = 0.0;
    pair_acc_f64(x0, x1, x2, bj0, bj1, bj2, d[0], d[1], d[2], d[3], d[4], d[5], d[6], d[7], d[8],
                 d[9], d[10], d[11], d[12], kr, nu, r1, r1 * r1 * r1, r2, r2c, a0, a1, a2, ak);
    a0 = fma(ak, bj0, a0);
    a1 = fma(ak, bj1, a1);
    a2 = fma(ak, bj2, a2);
}

}  // namespace dd
