// a2, mixed FP32/FP64 path: the all-pairs kernel k_pair_mixed and its launcher.
#include "dd_common.h"
#include "dd_pair32.h"
#include "dd_pair64.h"

namespace dd {

// Mixed precision.  Each pair is first located in FP32 from FP32 positions:
// when, for every target point of the wavefront, the source midpoint lies at
// least max(30 L, cutoff + L/2) away, the source is evaluated by FP32 2-point
// quadrature (the
// integrand is evaluated directly, so FP32 position rounding costs at most
// ~1e-6 relative there).  Other pairs get their offset, axial and
// perpendicular parts in FP64: those closer than the cutoff (minimum distance
// from the Gauss point to the closed source segment) are evaluated in FP64,
// the rest by the cancellation-free FP32 closed form.  FP32 contributions
// are accumulated in FP32 over one LDS stage, then added to FP64 sums.
template <bool FP32_FIRST>
__global__ __launch_bounds__(TILE) void k_pair_mixed(const Item *__restrict__ items,
                                                     const Tile *__restrict__ tiles,
                                                     const double *__restrict__ rec,
                                                     const float *__restrict__ rec32,
                                                     int64_t ns, GaussRule g, double k1,
                                                     double k2, float cut,
                                                     double *__restrict__ partial,
                                                     unsigned long long *near_count)
{
    __shared__ double shx[6][TILE];    // x1, t (FP64)
    __shared__ float shf[10][TILE];    // t, L, b, c (FP32)
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
    const float xf0 = (float)xq0, xf1 = (float)xq1, xf2 = (float)xq2;
    const double bj0 = rec[7 * ns + j], bj1 = rec[8 * ns + j], bj2 = rec[9 * ns + j];
    const float fb0 = (float)bj0, fb1 = (float)bj1, fb2 = (float)bj2;
    const float fk1 = (float)k1, fk2 = (float)k2, cut2 = cut * cut;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    unsigned n_near = 0, n_quad = 0;
    if (lane == 0) {
        n_near_block = 0;
        n_quad_block = 0;
    }

    for (int64_t base = it.src_begin; base < it.src_end; base += TILE) {
        const int n = (int)min<int64_t>(TILE, it.src_end - base);
        __syncthreads();
        if (lane < n) {
            const int64_t sidx = base + lane;
#pragma unroll
            for (int k = 0; k < 6; ++k) shx[k][lane] = rec[k * ns + sidx];
#pragma unroll
            for (int k = 0; k < 10; ++k) shf[k][lane] = rec32[k * ns + sidx];
        }
        __syncthreads();
        float f0 = 0.f, f1 = 0.f, f2 = 0.f;
        for (int m = 0; m < n; ++m) {
            const int64_t i = base + m;
            const float t0 = shf[0][m], t1 = shf[1][m], t2 = shf[2][m], Ls = shf[3][m];
            const float GB = fmaxf(GAUSS_BAND * Ls, cut + 0.5f * Ls);
            const double T0 = shx[3][m], T1 = shx[4][m], T2 = shx[5][m];
            float y, h0, h1, h2, hh, c0, c1, c2;
            bool quad;
            if (FP32_FIRST) {
                // FP32 location from FP32 positions: enough for the quadrature
                // branch (no cancellation there, ~1e-6 relative at worst)
                const float e0 = xf0 - (float)shx[0][m], e1 = xf1 - (float)shx[1][m], e2 = xf2 - (float)shx[2][m];
                y = e0 * t0 + e1 * t1 + e2 * t2;
                h0 = e0 - y * t0; h1 = e1 - y * t1; h2 = e2 - y * t2;
                hh = h0 * h0 + h1 * h1 + h2 * h2;
                const float ym = y - 0.5f * Ls;
                quad = __all(hh + ym * ym >= GB * GB);
            }
            if (!FP32_FIRST || !quad) {
                // offset, axial and perpendicular parts in FP64, rounded once
                const double R0 = xq0 - shx[0][m], R1 = xq1 - shx[1][m], R2 = xq2 - shx[2][m];
                const double yd = R0 * T0 + R1 * T1 + R2 * T2;
                y = (float)yd;
                h0 = (float)(R0 - yd * T0); h1 = (float)(R1 - yd * T1); h2 = (float)(R2 - yd * T2);
                hh = h0 * h0 + h1 * h1 + h2 * h2;
                if (!FP32_FIRST) {
                    const float ym = y - 0.5f * Ls;
                    quad = __all(hh + ym * ym >= GB * GB);
                }
            }
            if (quad) {
                n_quad += valid ? 1u : 0u;
                pair_sigma_b_f32_gauss2(y, h0, h1, h2, fb0, fb1, fb2, t0, t1, t2, Ls, shf[4][m], shf[5][m],
                                        shf[6][m], shf[7][m], shf[8][m], shf[9][m], fk1, fk2, c0, c1, c2);
                f0 += c0;
                f1 += c1;
                f2 += c2;
                continue;
            }
            const float ya = y - fminf(fmaxf(y, 0.f), Ls);
            if (hh + ya * ya < cut2) {
                if (i != j) {
                    n_near += valid ? 1u : 0u;
                    double d0, d1, d2;
                    pair_sigma_b_f64(xq0, xq1, xq2, bj0, bj1, bj2, shx[0][m], shx[1][m], shx[2][m],
                                     T0, T1, T2, rec[6 * ns + i], rec[7 * ns + i], rec[8 * ns + i],
                                     rec[9 * ns + i], rec[10 * ns + i], rec[11 * ns + i],
                                     rec[12 * ns + i], k1, k2, d0, d1, d2);
                    a0 += d0;
                    a1 += d1;
                    a2 += d2;
                }
            } else {
                pair_sigma_b_f32(y, h0, h1, h2, fb0, fb1, fb2, t0, t1, t2, Ls, shf[4][m], shf[5][m],
                                 shf[6][m], shf[7][m], shf[8][m], shf[9][m], fk1, fk2, c0, c1, c2);
                f0 += c0;
                f1 += c1;
                f2 += c2;
            }
        }
        a0 += (double)f0;
        a1 += (double)f1;
        a2 += (double)f2;
    }
    if (valid) {
        double *o = partial + it.slot * 3 * TILE;
        o[lane] = a0;
        o[TILE + lane] = a1;
        o[2 * TILE + lane] = a2;
    }
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
    if (variant)
        hipLaunchKernelGGL(k_pair_mixed<true>, dim3((unsigned)n_items), dim3(TILE), 0, st, items, tiles, rec, rec32,
                           ns, g, k1, k2, cut, partial, counters);
    else
        hipLaunchKernelGGL(k_pair_mixed<false>, dim3((unsigned)n_items), dim3(TILE), 0, st, items, tiles, rec, rec32,
                           ns, g, k1, k2, cut, partial, counters);
}

}  // namespace dd
