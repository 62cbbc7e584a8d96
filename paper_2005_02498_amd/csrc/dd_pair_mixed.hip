// a2, mixed FP32/FP64 path: the all-pairs kernel k_pair_mixed and its launcher.
#include "dd_common.h"
#include "dd_pair32.h"
#include "dd_pair64.h"

namespace dd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Mixed precision.  As in the FP64 kernel, every lane of a wavefront works on
// the same source at the same time.  FP64 records are read with scalar loads.
// QN = the source-quadrature points of the variant (0: none, 2 or 3).  With
// QN > 0 the FP32 records are staged through LDS TILE sources at a time (the
// quadrature's FP32 instructions issue faster with every operand in a vector
// register) and each source is first located in FP32 relative to its midpoint
// (positions split into FP32 high and low parts, so the offset carries no
// rounding of the absolute coordinates): when, for every target point of the
// wavefront, the midpoint lies outside the source's band (max(30 L, cutoff +
// L/2) for 2 points, max(6 L, cutoff + L/2) for 3), the source is evaluated by
// FP32 quadrature.  With QN = 0 the FP32 records are read with scalar loads.
// Other pairs get their axial and perpendicular parts in FP32 from the same
// midpoint offset: those closer than the cutoff (minimum distance from the
// Gauss point to the closed source segment), and nearly collinear ones (the
// target within an angle of about 1/16 of the source's axis, seen from its
// midpoint), are evaluated in FP64 from the FP64 record, the rest by the
// cancellation-free FP32 closed form.  Nearly collinear pairs never take the
// quadrature either: in FP32 their perpendicular part rho carries an absolute
// error of order |ym| 6e-8, which is large against rho itself there, and for a
// screw source (b along t) the field on its axis consists of terms linear in
// rho alone.  FP32 contributions are summed in FP32 over TILE sources
// at a time, then added to FP64 sums; all sums are in units of k2 and scaled
// once at the end.
template <int QN>
__global__ __launch_bounds__(TILE) void k_pair_mixed(const Item *__restrict__ items,
                                                     const Tile *__restrict__ tiles,
                                                     const double *__restrict__ rec,
                                                     const double *__restrict__ ra,
                                                     const float *__restrict__ rf, int64_t ns,
                                                     GaussRule g, double kr, double nu, double k2,
                                                     float cut, double *__restrict__ partial,
                                                     unsigned long long *near_count)
{
    __shared__ f32x4 shr[QN ? TILE : 1][REC32A / 4];   // FP32 records of one stage of sources
    __shared__ unsigned n_near_block, n_quad_block;
    const Item it = items[blockIdx.x];
    const Tile tl = tiles[it.tile];
    const int lane = threadIdx.x;
    const bool valid = lane < tl.n_points;
    const int64_t p = tl.point_begin + (valid ? lane : 0);
    const int Q = g.n;
    const int64_t j = p / Q;
    const int q = (int)(p - j * Q);
    double sq = g.s[0];
    for (int k = 1; k < DD_MAX_GAUSS; ++k)
        if (k == q) sq = g.s[k];
    const double L = rec[6 * ns + j];
    const double xq0 = rec[0 * ns + j] + sq * L * rec[3 * ns + j];
    const double xq1 = rec[1 * ns + j] + sq * L * rec[4 * ns + j];
    const double xq2 = rec[2 * ns + j] + sq * L * rec[5 * ns + j];
    const float xh0 = (float)xq0, xh1 = (float)xq1, xh2 = (float)xq2;
    const float xl0 = (float)(xq0 - (double)xh0), xl1 = (float)(xq1 - (double)xh1),
                xl2 = (float)(xq2 - (double)xh2);
    const double bj0 = rec[7 * ns + j], bj1 = rec[8 * ns + j], bj2 = rec[9 * ns + j];
    const float fb0 = (float)bj0, fb1 = (float)bj1, fb2 = (float)bj2;
    const float fkr = (float)kr, fnu = (float)nu, cut2 = cut * cut;
    // constants of the FP32 arithmetic in vector registers (the empty asm keeps
    // them there): an FP32 instruction with a literal operand issues at half rate
    // kap = K^2 / (1 + K^2): the collinear test ym^2 (1 + K^2) <= K^2 (ee + 1)
    // as ym^2 <= kap (ee + 1), one instruction fewer
    float three = 3.0f, ck2 = COLLINEAR_K2, kap = COLLINEAR_K2 / (1.0f + COLLINEAR_K2);
    asm volatile("" : "+v"(three), "+v"(ck2), "+v"(kap));
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    unsigned n_near = 0, n_quad_src = 0;
    if (lane == 0) {
        n_near_block = 0;
        n_quad_block = 0;
    }
    __syncthreads();   // the counters are cleared before any wavefront adds to them

    for (int64_t base = it.src_begin; base < it.src_end; base += TILE) {
        const int n = (int)min(it.src_end - base, (int64_t)TILE);
        // the target's own segment as a source index of this stage (-1: not in it)
        const int self = j >= base && j < base + n ? (int)(j - base) : -1;
        float f0 = 0.f, f1 = 0.f, f2 = 0.f, fk = 0.f;
        if (QN) {
            __syncthreads();
            if (lane < n) {
                const f32x4 *g4 = reinterpret_cast<const f32x4 *>(rf + (base + lane) * REC32A);
#pragma unroll
                for (int f = 0; f < REC32A / 4; ++f) shr[lane][f] = g4[f];
            }
            __syncthreads();
        }
        const float *s = rf + base * REC32A;
        for (int k = 0; k < n; ++k, s += REC32A) {
            float r[REC32A];
            if (QN) {
                // from LDS (broadcast reads): the FP32 quadrature then runs on
                // vector-register operands, which issue faster than FP32
                // instructions with a scalar operand; the fields only the
                // other pairs use are read below, for those
#pragma unroll
                for (int f = 0; f < R32_QUAD_VECS; ++f) {
                    const f32x4 v = shr[k][f];
                    r[4 * f] = v[0];
                    r[4 * f + 1] = v[1];
                    r[4 * f + 2] = v[2];
                    r[4 * f + 3] = v[3];
                }
            } else {
                // straight from memory into scalar registers (two loads, one wait)
                const f32x16 va = *reinterpret_cast<const f32x16 *>(s);
                const f32x8 vb = *reinterpret_cast<const f32x8 *>(s + 16);
#pragma unroll
                for (int f = 0; f < 16; ++f) r[f] = va[f];
#pragma unroll
                for (int f = 0; f < 8; ++f) r[16 + f] = vb[f];
            }
            // offset from the source midpoint, from the split FP32 positions:
            // accurate to the rounding of its own size
            const float e0 = (xh0 - r[R32_XH]) + (xl0 - r[R32_XL]);
            const float e1 = (xh1 - r[R32_XH + 1]) + (xl1 - r[R32_XL + 1]);
            const float e2 = (xh2 - r[R32_XH + 2]) + (xl2 - r[R32_XL + 2]);
            // axial coordinate from the midpoint
            const float ym = fmaf(e2, r[R32_T + 2], fmaf(e1, r[R32_T + 1], e0 * r[R32_T]));
            const float ym2 = ym * ym;
            if (QN) {
                const float ee = fmaf(e2, e2, fmaf(e1, e1, e0 * e0));
                // outside the band and not nearly collinear (ym^2 > K^2 (rho^2 + 1)
                // with rho^2 = ee - ym^2, see COLLINEAR_K2)
                // every active lane passes both tests: the two comparison masks
                // against exec, in scalar registers (a ballot of their
                // conjunction would select and re-compare per lane)
                const uint64_t quad = __builtin_amdgcn_ballot_w64(ee >= r[R32_BAND]) &
                                      __builtin_amdgcn_ballot_w64(ym2 <= fmaf(kap, ee, kap));
                if (quad == __builtin_amdgcn_read_exec()) {
                    ++n_quad_src;
                    if (QN == 2)
                        quad2_acc_f32(e0, e1, e2, ee, ym, r, fb0, fb1, fb2, fkr, fnu, three, f0, f1, f2, fk);
                    else
                        quad3_acc_f32(e0, e1, e2, ee, ym, r, fb0, fb1, fb2, fkr, fnu, three, f0, f1, f2, fk);
                    continue;
                }
            }
            if (QN) {
#pragma unroll
                for (int f = R32_QUAD_VECS; f < REC32A / 4; ++f) {
                    const f32x4 v = shr[k][f];
                    r[4 * f] = v[0];
                    r[4 * f + 1] = v[1];
                    r[4 * f + 2] = v[2];
                    r[4 * f + 3] = v[3];
                }
            }
            // axial coordinate from the first node and perpendicular part
            const float Ls = r[R32_L];
            const float y = fmaf(0.5f, Ls, ym);
            const float h0 = fmaf(-ym, r[R32_T], e0), h1 = fmaf(-ym, r[R32_T + 1], e1), h2 = fmaf(-ym, r[R32_T + 2], e2);
            const float hh = fmaf(h2, h2, fmaf(h1, h1, h0 * h0));
            const float ya = y - __builtin_amdgcn_fmed3f(y, 0.f, Ls);   // y clamped to [0, L]: one instruction
            // FP64: near pairs, and nearly collinear ones (rho carries an absolute
            // error of order |ym| eps32 in FP32)
            if (hh + ya * ya < cut2 || ym2 > fmaf(ck2, hh, ck2)) {
                // k through an empty asm: the comparison stays in this branch
                // instead of becoming a per-lane counter stepped every source
                int ks = k;
                asm volatile("" : "+s"(ks));
                if (ks != self) {
                    n_near += valid ? 1u : 0u;
                    pair_acc_isolated_f64(xq0, xq1, xq2, bj0, bj1, bj2, ra + (base + k) * RECA, kr, nu, a0, a1, a2);
                }
            } else {
                // the record's b and c carry the quadrature weight (1 without a quadrature)
                pair_acc_f32(y, h0, h1, h2, hh, fb0, fb1, fb2, r[R32_T], r[R32_T + 1], r[R32_T + 2], Ls, r[R32_B],
                             r[R32_B + 1], r[R32_B + 2], r[R32_C], r[R32_C + 1], r[R32_C + 2], QN ? r[R32_IW] : 1.0f,
                             fkr, fnu, f0, f1, f2, fk);
            }
        }
        a0 += (double)fmaf(fk, fb0, f0);   // the b_j terms of the stage at once
        a1 += (double)fmaf(fk, fb1, f1);
        a2 += (double)fmaf(fk, fb2, f2);
    }
    if (valid) {
        double *o = partial + it.slot * 3 * TILE;
        o[lane] = k2 * a0;
        o[TILE + lane] = k2 * a1;
        o[2 * TILE + lane] = k2 * a2;
    }
    const unsigned n_quad = valid ? n_quad_src : 0u;
    if (n_near) atomicAdd(&n_near_block, n_near);
    if (n_quad) atomicAdd(&n_quad_block, n_quad);
    __syncthreads();
    if (lane == 0 && n_near_block) atomicAdd(near_count, (unsigned long long)n_near_block);
    if (lane == 0 && n_quad_block) atomicAdd(near_count + 1, (unsigned long long)n_quad_block);
}

void launch_pair_mixed(const Item *items, const Tile *tiles, const double *rec, const float *rec32, int64_t ns,
                       const GaussRule &g, double k1, double k2, float cut, double *partial,
                       unsigned long long *counters, int64_t n_items, int variant, hipStream_t st)
{
    const double kr = k1 / k2, nu = 1.0 - 2.0 * kr;
    const double *ra = rec + (int64_t)REC64 * ns;
    const int qn = quad_points(variant);
    if (qn == 2)
        hipLaunchKernelGGL(k_pair_mixed<2>, dim3((unsigned)n_items), dim3(TILE), 0, st, items, tiles, rec, ra,
                           rec32, ns, g, kr, nu, k2, cut, partial, counters);
    else if (qn == 3)
        hipLaunchKernelGGL(k_pair_mixed<3>, dim3((unsigned)n_items), dim3(TILE), 0, st, items, tiles, rec, ra,
                           rec32, ns, g, kr, nu, k2, cut, partial, counters);
    else
        hipLaunchKernelGGL(k_pair_mixed<0>, dim3((unsigned)n_items), dim3(TILE), 0, st, items, tiles, rec, ra,
                           rec32, ns, g, kr, nu, k2, cut, partial, counters);
}

}  // namespace dd
