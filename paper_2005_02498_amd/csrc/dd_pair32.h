// FP32 per-pair device functions of the mixed-precision path (the regrouped
// closed form of dd_pair64.h in FP32 with the endpoint differences
// rearranged, and a 2-point source quadrature).
#pragma once

#include <hip/hip_runtime.h>

#include "dd_common.h"

namespace dd {

// Pairs whose target lies nearly on the source's axis, ym^2 > K^2 (rho^2 + 1)
// with ym the axial offset from the source midpoint and rho the perpendicular
// part (units of a), K = 16, leave the FP32 branches for the FP64 closed
// form.  Outside that cone both FP32 branches stay within about 3e-6 of the
// pair's own contribution (a CPU emulation of these routines on screw and
// mixed sources at 20 to 5e4 a); inside it the FP32 rho of a screw source can
// be off by more than its own size.
constexpr float COLLINEAR_K2 = 256.0f;

// FP32, far pairs: adds sigma^i b_j / k2 (the regrouped closed form of
// dd_pair64.h, kr = (1 - nu)/2) to (f0, f1, f2) + fk b_j (the b_j term's
// scalar goes to fk; the caller adds fk b_j once).  y, rho and hh = |rho|^2 are
// formed by the caller in FP32 from the offset to the source midpoint, so rho
// carries an absolute error of order |y - L/2| 6e-8; the caller keeps nearly
// collinear pairs (COLLINEAR_K2) away from this routine, and for the others
// that error is small against rho and against the field.  The endpoint
// differences are rearranged so that no two nearly equal numbers are
// subtracted when the target lies far away or on the extension of the segment
// (u1 = -y, u2 = L - y, r = 1/Ra, s = u r):
//   I31 = L (u1 + u2) r1 r2 / (Ra1 + Ra2)
//   I30 = L (u1 + u2) r1 r2 / (u2 Ra1 + u1 Ra2)          if u1 u2 > 0
//       = (s2 - s1) / d2                                 otherwise
//   1 - s1 s2 = r1 r2 P,  P = d2 (d2 + u1^2 + u2^2) / (Ra1 Ra2 + u1 u2)  if u1 u2 > 0
//                         P = Ra1 Ra2 - u1 u2                            otherwise
//   E50 = 3 I50 = I30 (d2 (r1^2 + r2^2) + r1 r2 P) / d2
//   D51 = 3 I51 = I31 (r1^2 + r1 r2 + r2^2)
//   P3  = 3 I52 = I30 (s1^2 + s1 s2 + s2^2)
// (from s2^3 - s1^3 = (s2 - s1)(s1^2 + s1 s2 + s2^2), 1 - s^2 = d2 r^2 and
// u2^2 Ra1^2 - u1^2 Ra2^2 = d2 (u2^2 - u1^2)).  The four reciprocals come in
// pairs from two: 1/X and 1/Y as Y/(X Y) and X/(X Y).  b and c come scaled by
// a factor 1/iw (the source record's quadrature weight): the field is linear
// in them, and iw enters through q, A, Cc and I30 where they meet a scaled
// quantity.
__device__ __forceinline__ void pair_acc_f32(
    float y, float h0, float h1, float h2, float hh, float bj0, float bj1, float bj2,
    float t0, float t1, float t2, float L, float b0, float b1, float b2,
    float c0, float c1, float c2, float iw, float kr, float nu, float &f0, float &f1, float &f2, float &fk)
{
    const float d2 = hh + 1.0f;
    const float u2 = L - y;
    const float Ra1s = fmaf(y, y, d2), Ra2s = fmaf(u2, u2, d2);
    const float r1 = __builtin_amdgcn_rsqf(Ra1s), r2 = __builtin_amdgcn_rsqf(Ra2s);
    const float Ra1 = Ra1s * r1, Ra2 = Ra2s * r2;
    const float s1 = -y * r1, s2 = u2 * r2;
    const float rr = r1 * r2;
    const float Lus = L * fmaf(-2.0f, y, L) * rr;
    const bool same = y * u2 < 0.0f;                    // u1 u2 > 0
    const float Aq = fmaf(u2, Ra1, -y * Ra2);           // u2 Ra1 + u1 Ra2 (> 0 when same)
    const float Bq = fmaf(Ra1, Ra2, -y * u2);           // Ra1 Ra2 + u1 u2 (>= d2 when same)
    const float Cs = Ra1 + Ra2;
    const float iAB = __builtin_amdgcn_rcpf(Aq * Bq), iCD = __builtin_amdgcn_rcpf(Cs * d2);
    const float id2 = Cs * iCD;
    const float I30 = same ? Lus * (Bq * iAB) : (s2 - s1) * id2;
    const float Pm = same ? d2 * (Ra1s + u2 * u2) * (Aq * iAB) : fmaf(y, u2, Ra1 * Ra2);
    const float I31 = Lus * (d2 * iCD);
    const float r12 = fmaf(r1, r1, r2 * r2);
    const float E50 = I30 * fmaf(d2, r12, rr * Pm) * id2;
    const float D51 = I31 * (r12 + rr);
    const float P3 = I30 * fmaf(s1, s1 + s2, s2 * s2);
    const float g0 = fmaf(2.0f, I30, E50);
    const float q = iw * fmaf(c2, h2, fmaf(c1, h1, c0 * h0));
    const float A = -kr * g0 * iw;                      // meets rho x b (scaled)
    const float Cc = fmaf(nu, I31, -kr * D51) * iw;     // meets c (scaled)
    const float I30s = I30 * iw;                        // where it meets c
    fk = fmaf(q, I30 + E50, fk);   // kd
    const float rb0 = fmaf(h1, b2, -h2 * b1), rb1 = fmaf(h2, b0, -h0 * b2), rb2 = fmaf(h0, b1, -h1 * b0);
    // sigma b_j / k2 as coefficients of the five vectors rho x b, c, t, rho and b_j
    const float tb = fmaf(t2, bj2, fmaf(t1, bj1, t0 * bj0));
    const float hb = fmaf(h2, bj2, fmaf(h1, bj1, h0 * bj0));
    const float cb = fmaf(c2, bj2, fmaf(c1, bj1, c0 * bj0));
    const float rbb = fmaf(rb2, bj2, fmaf(rb1, bj1, rb0 * bj0));
    const float Pt = fmaf(q, fmaf(P3, tb, -D51 * hb), fmaf(Cc, cb, A * rbb));
    const float Ph = fmaf(q, fmaf(E50, hb, -D51 * tb), -I30s * cb);
    const float Pc = fmaf(Cc, tb, -I30s * hb);
    const float Pr = A * tb;
    f0 = fmaf(Ph, h0, fmaf(Pt, t0, fmaf(Pc, c0, fmaf(Pr, rb0, f0))));
    f1 = fmaf(Ph, h1, fmaf(Pt, t1, fmaf(Pc, c1, fmaf(Pr, rb1, f1))));
    f2 = fmaf(Ph, h2, fmaf(Pt, t2, fmaf(Pc, c2, fmaf(Pr, rb2, f2))));
}


// FP32, well-separated pairs: Gauss-Legendre quadrature of the integrand
// along the source instead of the closed form, used when the target lies far
// enough from the source midpoint (30 source lengths for 2 points, 6 for 3:
// the rule's error is then below 2e-7 relative).  Source points xm + sg t with
// weights wg; with e = x - xm, ym = e.t, rho = e - ym t, the axial coordinate
// of the target relative to a point is v = ym - sg and Ra^2 = |e|^2 + 1 +
// sg^2 - 2 sg ym.  With R = rho + v t, R x b = rho x b - v c and q = c.rho,
// the integrand contracted with b_j (divided by k2, kr = k1/k2 = (1 - nu)/2)
// is
//   K b_j = al [ (R x b)(t.b_j) + t ((R x b).b_j) ] + be b_j
//         + ga [ R (c.b_j) + c (R.b_j) ] + de R (R.b_j),
//   al = -kr (2/Ra^3 + 3/Ra^5), be = q (1/Ra^3 + 3/Ra^5),
//   ga = -1/Ra^3, de = 3 q / Ra^5.
// Summed over the points it depends on them only through
//   S3 = sum w/Ra^3, S5 = sum w/Ra^5, S3v = sum w v/Ra^3, S5v = sum w v/Ra^5,
//   S5vv = sum w v^2/Ra^5,
// with w the weights relative to Wo: Wo itself is carried by b and c,
// and collects as coefficients of rho x b, c, t, b_j and rho:
//   rho x b : (t.b_j) Sal                       Sal = -kr (2 S3 + 3 S5)
//   c       : (rho.b_j) Sga + (t.b_j) Sgv       Sga = -S3, Sgv = -nu S3v + 3 kr S5v
//   t       : ((rho x b).b_j) Sal + (c.b_j) Sgv + 3 q ((rho.b_j) S5v + (t.b_j) S5vv)
//   b_j     : q (S3 + 3 S5)
//   rho     : (c.b_j) Sga + 3 q ((rho.b_j) S5 + (t.b_j) S5v)

// The moments are collected as the coefficients of the five vectors (that of
// b_j added to fk); shared by the 2- and 3-point rules.  three = 3, passed in
// a vector register by the caller: an FP32 instruction with a literal or
// scalar-register operand issues at half the rate of one whose operands are
// all vector registers.
__device__ __forceinline__ void quad_moments_acc_f32(float e0, float e1, float e2, float ym, const float *s,
                                                     float S3, float S5, float S3v, float S5v, float S5vv,
                                                     float bj0, float bj1, float bj2, float kr, float nu, float three,
                                                     float &f0, float &f1, float &f2, float &fk)
{
    const float t0 = s[R32_T], t1 = s[R32_T + 1], t2 = s[R32_T + 2];
    const float b0 = s[R32_B], b1 = s[R32_B + 1], b2 = s[R32_B + 2];
    const float c0 = s[R32_C], c1 = s[R32_C + 1], c2 = s[R32_C + 2];
    const float h0 = fmaf(-ym, t0, e0), h1 = fmaf(-ym, t1, e1), h2 = fmaf(-ym, t2, e2);
    const float rb0 = fmaf(h1, b2, -h2 * b1), rb1 = fmaf(h2, b0, -h0 * b2), rb2 = fmaf(h0, b1, -h1 * b0);
    const float tb = fmaf(t2, bj2, fmaf(t1, bj1, t0 * bj0));
    const float hb = fmaf(h2, bj2, fmaf(h1, bj1, h0 * bj0));
    const float cb = fmaf(c2, bj2, fmaf(c1, bj1, c0 * bj0));
    const float rbb = fmaf(rb2, bj2, fmaf(rb1, bj1, rb0 * bj0));
    const float q = fmaf(c2, h2, fmaf(c1, h1, c0 * h0));
    const float q3 = three * q;
    const float Sal = -kr * fmaf(2.0f, S3, three * S5);
    const float Sgv = fmaf(-nu, S3v, three * kr * S5v);
    const float Cr = tb * Sal;
    const float Cc = fmaf(tb, Sgv, -hb * S3);
    const float Ct = fmaf(rbb, Sal, fmaf(cb, Sgv, q3 * fmaf(hb, S5v, tb * S5vv)));
    fk = fmaf(q, fmaf(three, S5, S3), fk);
    const float Ch = fmaf(-cb, S3, q3 * fmaf(hb, S5, tb * S5v));
    f0 = fmaf(Ch, h0, fmaf(Ct, t0, fmaf(Cc, c0, fmaf(Cr, rb0, f0))));
    f1 = fmaf(Ch, h1, fmaf(Ct, t1, fmaf(Cc, c1, fmaf(Cr, rb1, f1))));
    f2 = fmaf(Ch, h2, fmaf(Ct, t2, fmaf(Cc, c2, fmaf(Cr, rb2, f2))));
}

// e = target - source midpoint, ee = |e|^2, ym = e.t; s = the source's FP32 record (see
// REC32A), whose b and c carry the weight Wo; adds K b_j / k2 to (f0, f1, f2)
// + fk b_j.  2-point rule: points at v = ym -+ hq, weight Wo each (in b, c).
__device__ __forceinline__ void quad2_acc_f32(float e0, float e1, float e2, float ee, float ym, const float *s,
                                              float bj0, float bj1, float bj2, float kr, float nu, float three,
                                              float &f0, float &f1, float &f2, float &fk)
{
    const float hq = s[R32_HQ];
    const float base = ee + s[R32_RA0], tw = s[R32_TW] * ym;
    const float vA = ym + hq, vB = ym - hq;
    const float iA = __builtin_amdgcn_rsqf(base + tw), iB = __builtin_amdgcn_rsqf(base - tw);
    const float iA2 = iA * iA, iB2 = iB * iB;
    const float iA3 = iA2 * iA, iB3 = iB2 * iB;
    const float iA5 = iA3 * iA2, iB5 = iB3 * iB2;
    const float pA = iA5 * vA, pB = iB5 * vB;
    const float S3 = iA3 + iB3, S5 = iA5 + iB5;
    const float S3v = fmaf(iA3, vA, iB3 * vB), S5v = pA + pB;
    const float S5vv = fmaf(pA, vA, pB * vB);
    quad_moments_acc_f32(e0, e1, e2, ym, s, S3, S5, S3v, S5v, S5vv, bj0, bj1, bj2, kr, nu, three, f0, f1, f2, fk);
}

// 3-point rule: points at v = ym -+ hq with weight Wo (in b, c) and at v = ym
// with weight Wc, relative weight Wc/Wo = 8/5 (Gauss-Legendre, hq = (L/2)
// sqrt(3/5), Wo = 5L/18, Wc = 8L/18).
// Its error is below 2e-7 relative beyond 6 source lengths from the midpoint.
__device__ __forceinline__ void quad3_acc_f32(float e0, float e1, float e2, float ee, float ym, const float *s,
                                              float bj0, float bj1, float bj2, float kr, float nu, float three,
                                              float &f0, float &f1, float &f2, float &fk)
{
    const float hq = s[R32_HQ], Wc = s[R32_WC];
    const float base = ee + s[R32_RA0], tw = s[R32_TW] * ym;
    const float vA = ym + hq, vB = ym - hq;
    const float iA = __builtin_amdgcn_rsqf(base + tw), iB = __builtin_amdgcn_rsqf(base - tw);
    const float iC = __builtin_amdgcn_rsqf(ee + 1.0f);
    const float iA2 = iA * iA, iB2 = iB * iB, iC2 = iC * iC;
    const float iA3 = iA2 * iA, iB3 = iB2 * iB, iC3 = iC2 * iC;
    const float iA5 = iA3 * iA2, iB5 = iB3 * iB2, iC5 = iC3 * iC2;
    const float pA = iA5 * vA, pB = iB5 * vB, pC = iC5 * ym;
    const float S3 = fmaf(Wc, iC3, iA3 + iB3), S5 = fmaf(Wc, iC5, iA5 + iB5);
    const float S3v = fmaf(Wc, iC3 * ym, fmaf(iA3, vA, iB3 * vB));
    const float S5v = fmaf(Wc, pC, pA + pB);
    const float S5vv = fmaf(Wc, pC * ym, fmaf(pA, vA, pB * vB));
    quad_moments_acc_f32(e0, e1, e2, ym, s, S3, S5, S3v, S5v, S5vv, bj0, bj1, bj2, kr, nu, three, f0, f1, f2, fk);
}

}  // namespace dd
