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
// along the source instead of the closed form.  Source points xm -+ hoff t
// (hoff = L / (2 sqrt 3), weight W = L/2 each); with e = x - xm, ym = e.t,
// rho = e - ym t, the axial coordinates of the target relative to the two
// points are v = ym +- hoff and Ra^2 = |e|^2 + 1 + hoff^2 +- 2 hoff ym.  With
// R = rho + v t, R x b = rho x b - v c and q = c.rho, the integrand
// contracted with b_j (divided by k2, kr = k1/k2 = (1 - nu)/2) is
//   K b_j = al [ (R x b)(t.b_j) + t ((R x b).b_j) ] + be b_j
//         + ga [ R (c.b_j) + c (R.b_j) ] + de R (R.b_j),
//   al = -kr (2/Ra^3 + 3/Ra^5), be = q (1/Ra^3 + 3/Ra^5),
//   ga = -1/Ra^3, de = 3 q / Ra^5.
// Summed over the two points it depends on them only through
//   S3 = sum W/Ra^3, S5 = sum W/Ra^5, S3v = sum W v/Ra^3, S5v = sum W v/Ra^5,
//   S5vv = sum W v^2/Ra^5,
// and collects as coefficients of rho x b, c, t, b_j and rho:
//   rho x b : (t.b_j) Sal                       Sal = -kr (2 S3 + 3 S5)
//   c       : (rho.b_j) Sga + (t.b_j) Sgv       Sga = -S3, Sgv = -nu S3v + 3 kr S5v
//   t       : ((rho x b).b_j) Sal + (c.b_j) Sgv + 3 q ((rho.b_j) S5v + (t.b_j) S5vv)
//   b_j     : q (S3 + 3 S5)
//   rho     : (c.b_j) Sga + 3 q ((rho.b_j) S5 + (t.b_j) S5v)
// The quadrature error is below 2e-7 relative at that separation.
constexpr float GAUSS_BAND = 30.0f;

// e = target - source midpoint; s = the source's FP32 record (see REC32A);
// adds K b_j / k2 to (f0, f1, f2).
__device__ __forceinline__ void quad2_acc_f32(float e0, float e1, float e2, float ee, const float *s,
                                              float bj0, float bj1, float bj2, float kr, float nu,
                                              float &f0, float &f1, float &f2)
{
    const float t0 = s[6], t1 = s[7], t2 = s[8], hoff = s[10], W = s[18];
    const float b0 = s[11], b1 = s[12], b2 = s[13], c0 = s[14], c1 = s[15], c2 = s[16];
    const float ym = fmaf(e2, t2, fmaf(e1, t1, e0 * t0));
    const float h0 = fmaf(-ym, t0, e0), h1 = fmaf(-ym, t1, e1), h2 = fmaf(-ym, t2, e2);
    const float base = ee + s[19], tw = s[20] * ym;
    const float vA = ym + hoff, vB = ym - hoff;
    const float iA = __builtin_amdgcn_rsqf(base + tw), iB = __builtin_amdgcn_rsqf(base - tw);
    const float iA2 = iA * iA, iB2 = iB * iB;
    const float iA3 = iA2 * iA, iB3 = iB2 * iB;
    const float iA5 = iA3 * iA2, iB5 = iB3 * iB2;
    const float pA = iA5 * vA, pB = iB5 * vB;
    const float S3 = W * (iA3 + iB3), S5 = W * (iA5 + iB5);
    const float S3v = W * fmaf(iA3, vA, iB3 * vB), S5v = W * (pA + pB);
    const float S5vv = W * fmaf(pA, vA, pB * vB);
    const float rb0 = fmaf(h1, b2, -h2 * b1), rb1 = fmaf(h2, b0, -h0 * b2), rb2 = fmaf(h0, b1, -h1 * b0);
    const float tb = fmaf(t2, bj2, fmaf(t1, bj1, t0 * bj0));
    const float hb = fmaf(h2, bj2, fmaf(h1, bj1, h0 * bj0));
    const float cb = fmaf(c2, bj2, fmaf(c1, bj1, c0 * bj0));
    const float rbb = fmaf(rb2, bj2, fmaf(rb1, bj1, rb0 * bj0));
    const float q = fmaf(c2, h2, fmaf(c1, h1, c0 * h0));
    const float q3 = 3.0f * q;
    const float Sal = -kr * fmaf(2.0f, S3, 3.0f * S5);
    const float Sgv = fmaf(-nu, S3v, 3.0f * kr * S5v);
    const float Cr = tb * Sal;
    const float Cc = fmaf(tb, Sgv, -hb * S3);
    const float Ct = fmaf(rbb, Sal, fmaf(cb, Sgv, q3 * fmaf(hb, S5v, tb * S5vv)));
    const float Cb = q * fmaf(3.0f, S5, S3);
    const float Ch = fmaf(-cb, S3, q3 * fmaf(hb, S5, tb * S5v));
    f0 = fmaf(Cb, bj0, fmaf(Ch, h0, fmaf(Ct, t0, fmaf(Cc, c0, fmaf(Cr, rb0, f0)))));
    f1 = fmaf(Cb, bj1, fmaf(Ch, h1, fmaf(Ct, t1, fmaf(Cc, c1, fmaf(Cr, rb1, f1)))));
    f2 = fmaf(Cb, bj2, fmaf(Ch, h2, fmaf(Ct, t2, fmaf(Cc, c2, fmaf(Cr, rb2, f2)))));
}

}  // namespace dd
