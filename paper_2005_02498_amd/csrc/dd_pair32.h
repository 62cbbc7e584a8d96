// FP32 per-pair device functions of the mixed-precision path (same
// regrouped closed form as dd_pair64.h, in FP32 with the endpoint
// differences rearranged, and a 2-point source quadrature).
#pragma once

#include <hip/hip_runtime.h>

namespace dd {

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
    const float Zc = -k2 * I30, Zr = 1.5f * qk * I50;
    const float kd = qk * (I30 + 3.0f * I50);
    // sigma b_j = t (w.b_j) + w (t.b_j) + rho (z.b_j) + z (rho.b_j) + kd b_j, with w and z
    // expanded: coefficients of the five vectors rho x b, c, t, rho and b_j
    const float tb = t0 * bj0 + t1 * bj1 + t2 * bj2;
    const float hb = h0 * bj0 + h1 * bj1 + h2 * bj2;
    const float cb = c0 * bj0 + c1 * bj1 + c2 * bj2;
    const float rbb = rb0 * bj0 + rb1 * bj1 + rb2 * bj2;
    const float wb = A * rbb + Cc * cb + Tt * tb + Tr * hb;
    const float zb = Zc * cb + Zr * hb;
    const float Pr = A * tb, Pc = Cc * tb + Zc * hb, Pt = wb + Tt * tb, Ph = Tr * tb + zb + Zr * hb;
    o0 = Pr * rb0 + Pc * c0 + Pt * t0 + Ph * h0 + kd * bj0;
    o1 = Pr * rb1 + Pc * c1 + Pt * t1 + Ph * h1 + kd * bj1;
    o2 = Pr * rb2 + Pc * c2 + Pt * t2 + Ph * h2 + kd * bj2;
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
