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
    const double w0 = A * rb0 + Cc * c0 + Tt * t0 + Tr * h0;
    const double w1 = A * rb1 + Cc * c1 + Tt * t1 + Tr * h1;
    const double w2 = A * rb2 + Cc * c2 + Tt * t2 + Tr * h2;
    const double Zc = -k2 * I30, Zr = 1.5 * qk * I50;
    const double z0 = Zc * c0 + Zr * h0, z1 = Zc * c1 + Zr * h1, z2 = Zc * c2 + Zr * h2;
    const double kd = qk * (I30 + 3.0 * I50);
    const double wb = w0 * bj0 + w1 * bj1 + w2 * bj2;
    const double tb = t0 * bj0 + t1 * bj1 + t2 * bj2;
    const double zb = z0 * bj0 + z1 * bj1 + z2 * bj2;
    const double hb = h0 * bj0 + h1 * bj1 + h2 * bj2;
    o0 = t0 * wb + w0 * tb + h0 * zb + z0 * hb + kd * bj0;
    o1 = t1 * wb + w1 * tb + h1 * zb + z1 * hb + kd * bj1;
    o2 = t2 * wb + w2 * tb + h2 * zb + z2 * hb + kd * bj2;
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

// FP32, far pairs.  y and rho are formed in FP64 by the caller and rounded
// once.  The endpoint differences are rearranged so that no two nearly equal
// numbers are subtracted when the target lies far away or on the extension
// of the segment:
//   I31 = L (u1 + u2) r1 r2 / (Ra1 + Ra2)
//   I30 = L (u1 + u2) r1 r2 / (u2 Ra1 + u1 Ra2)          if u1 u2 > 0
//       = (s2 - s1) / d2                                 otherwise
//   1 - s1 s2 = r1 r2 P,  P = d2 (d2 + u1^2 + u2^2) / (Ra1 Ra2 + u1 u2)  if u1 u2 > 0
//                         P = Ra1 Ra2 - u1 u2                            otherwise
//   I50 = I30 (d2 (r1^2 + r2^2) + r1 r2 P) / (3 d2)
//   I51 = I31 (r1^2 + r1 r2 + r2^2) / 3
//   I52 = I30 (s1^2 + s1 s2 + s2^2) / 3
// (from s2^3 - s1^3 = (s2 - s1)(s1^2 + s1 s2 + s2^2), 1 - s^2 = d2 r^2 and
// u2^2 Ra1^2 - u1^2 Ra2^2 = d2 (u2^2 - u1^2)).
__device__ __forceinline__ void pair_sigma_b_f32(
    float y, float h0, float h1, float h2, float bj0, float bj1, float bj2,
    float t0, float t1, float t2, float L, float b0, float b1, float b2,
    float c0, float c1, float c2, float k1, float k2, float &o0, float &o1, float &o2)
{
    const float d2 = h0 * h0 + h1 * h1 + h2 * h2 + 1.0f;
    const float u1 = -y, u2 = L - y;
    const float Ra1s = d2 + u1 * u1, Ra2s = d2 + u2 * u2;
    const float r1 = __builtin_amdgcn_rsqf(Ra1s), r2 = __builtin_amdgcn_rsqf(Ra2s);
    const float Ra1 = Ra1s * r1, Ra2 = Ra2s * r2;
    const float s1 = u1 * r1, s2 = u2 * r2;
    const float rr = r1 * r2;
    const float Lus = L * (L - 2.0f * y) * rr;
    const bool same = u1 * u2 > 0.0f;
    const float id2 = __builtin_amdgcn_rcpf(d2);
    const float I30 = same ? Lus * __builtin_amdgcn_rcpf(u2 * Ra1 + u1 * Ra2) : (s2 - s1) * id2;
    const float P = same ? d2 * (d2 + u1 * u1 + u2 * u2) * __builtin_amdgcn_rcpf(Ra1 * Ra2 + u1 * u2)
                         : Ra1 * Ra2 - u1 * u2;
    const float I31 = Lus * __builtin_amdgcn_rcpf(Ra1 + Ra2);
    const float I50 = I30 * (d2 * (r1 * r1 + r2 * r2) + rr * P) * id2 * (1.0f / 3.0f);
    const float I51 = I31 * (r1 * r1 + rr + r2 * r2) * (1.0f / 3.0f);
    const float I52 = I30 * (s1 * s1 + s1 * s2 + s2 * s2) * (1.0f / 3.0f);
    const float g0 = 2.0f * I30 + 3.0f * I50;
    const float g1 = 2.0f * I31 + 3.0f * I51;
    const float q = c0 * h0 + c1 * h1 + c2 * h2;
    const float rb0 = h1 * b2 - h2 * b1, rb1 = h2 * b0 - h0 * b2, rb2 = h0 * b1 - h1 * b0;
    const float A = -k1 * g0, Cc = k2 * I31 - k1 * g1, qk = q * k2;
    const float Tt = 1.5f * qk * I52, Tr = -3.0f * qk * I51;
    const float w0 = A * rb0 + Cc * c0 + Tt * t0 + Tr * h0;
    const float w1 = A * rb1 + Cc * c1 + Tt * t1 + Tr * h1;
    const float w2 = A * rb2 + Cc * c2 + Tt * t2 + Tr * h2;
    const float Zc = -k2 * I30, Zr = 1.5f * qk * I50;
    const float z0 = Zc * c0 + Zr * h0, z1 = Zc * c1 + Zr * h1, z2 = Zc * c2 + Zr * h2;
    const float kd = qk * (I30 + 3.0f * I50);
    const float wb = w0 * bj0 + w1 * bj1 + w2 * bj2;
    const float tb = t0 * bj0 + t1 * bj1 + t2 * bj2;
    const float zb = z0 * bj0 + z1 * bj1 + z2 * bj2;
    const float hb = h0 * bj0 + h1 * bj1 + h2 * bj2;
    o0 = t0 * wb + w0 * tb + h0 * zb + z0 * hb + kd * bj0;
    o1 = t1 * wb + w1 * tb + h1 * zb + z1 * hb + kd * bj1;
    o2 = t2 * wb + w2 * tb + h2 * zb + z2 * hb + kd * bj2;
}


// FP32, well-separated pairs (target at least GAUSS_BAND source lengths from
// the source midpoint): 2-point Gauss-Legendre quadrature of the integrand
// along the source instead of the closed form.  With R = rho + v t at the
// source points (v = y - s_g, s_g = L (1/2 -+ 1/(2 sqrt 3)), weight L/2),
// R x b = rho x b - v c and q = c.R = c.rho, the integrand contracted with b_j,
//   K b_j = al [ (R x b)(t.b_j) + t ((R x b).b_j) ] + be b_j
//         + ga [ R (c.b_j) + c (R.b_j) ] + de R (R.b_j),
//   al = -k1 (2/Ra^3 + 3/Ra^5), be = k2 q (1/Ra^3 + 3/Ra^5),
//   ga = -k2/Ra^3, de = 3 k2 q / Ra^5,   Ra^2 = d2 + v^2,
// is summed over the two points as coefficients of the five vectors
// rho x b, c, t, b_j, rho.  Quadrature error below 2e-7 relative at that
// separation.
constexpr float GAUSS_BAND = 30.0f;

__device__ __forceinline__ void pair_sigma_b_f32_gauss2(
    float y, float h0, float h1, float h2, float bj0, float bj1, float bj2,
    float t0, float t1, float t2, float L, float b0, float b1, float b2,
    float c0, float c1, float c2, float k1, float k2, float &o0, float &o1, float &o2)
{
    const float d2 = h0 * h0 + h1 * h1 + h2 * h2 + 1.0f;
    const float rb0 = h1 * b2 - h2 * b1, rb1 = h2 * b0 - h0 * b2, rb2 = h0 * b1 - h1 * b0;
    const float tb = t0 * bj0 + t1 * bj1 + t2 * bj2;
    const float cb = c0 * bj0 + c1 * bj1 + c2 * bj2;
    const float hb = h0 * bj0 + h1 * bj1 + h2 * bj2;
    const float rbb = rb0 * bj0 + rb1 * bj1 + rb2 * bj2;
    const float q = c0 * h0 + c1 * h1 + c2 * h2;
    const float W = 0.5f * L;
    const float cA = -W * k1, cB = W * k2 * q, cG = -W * k2, cD = 3.0f * cB;
    const float hoff = 0.28867513459481288225f * L;   // L / (2 sqrt 3)
    const float vm = y - 0.5f * L;
    float P1 = 0.f, Pc = 0.f, Pt = 0.f, Pb = 0.f, Ph = 0.f;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const float v = g ? vm - hoff : vm + hoff;
        const float ir = __builtin_amdgcn_rsqf(d2 + v * v);
        const float ir2 = ir * ir, ir3 = ir * ir2, ir5 = ir3 * ir2;
        const float s1 = ir3 + 3.0f * ir5;
        const float al = cA * (s1 + ir3), be = cB * s1, ga = cG * ir3, de = cD * ir5;
        const float Rbj = hb + v * tb;
        const float Rbb = rbb - v * cb;
        const float p1 = al * tb;
        const float Dg = ga * cb + de * Rbj;
        P1 += p1;
        Pc += ga * Rbj - p1 * v;
        Pt += al * Rbb + Dg * v;
        Pb += be;
        Ph += Dg;
    }
    o0 = P1 * rb0 + Pc * c0 + Pt * t0 + Pb * bj0 + Ph * h0;
    o1 = P1 * rb1 + Pc * c1 + Pt * t1 + Pb * bj1 + Ph * h1;
    o2 = P1 * rb2 + Pc * c2 + Pt * t2 + Pb * bj2 + Ph * h2;
}

}  // namespace dd
