// a2, FP64 path: the all-pairs kernel k_pair64 and its launcher.
#include "dd_common.h"
#include "dd_pair64.h"

namespace dd {

// ------------------------------------------ a2: the all-pairs FP64 kernel --
// One workgroup = one work item: up to TILE target Gauss points (one per
// lane) against a contiguous source range.  Every lane of a wavefront works on
// the same source at the same time, so the source records are read with
// scalar loads into scalar registers (no LDS staging, no barriers) and enter
// the arithmetic as uniform operands.  Each lane accumulates sigma b_j / k2
// (3 values) over the range; the item's sums, scaled by k2, go to their own
// slot, reduced in a fixed order later.
//
// Sources come in runs that share nodes (loops stored in order): the inverse
// distance to a run's first node is computed once, then each source reuses
// the previous source's far-end value.  Only the part of the range that holds
// the tile's own segments tests for the excluded self pair.
template <bool SELF>
__device__ __forceinline__ void pair64_range(const double *__restrict__ ra, int64_t b, int64_t e,
                                             int64_t j, double xq0, double xq1, double xq2, double bj0,
                                             double bj1, double bj2, double kr, double nu, double &a0,
                                             double &a1, double &a2, double &ak)
{
    for (int64_t m = b; m < e;) {
        const double *c = ra + m * RECA;
        // uniform run length (>= 1), counted in 32 bits so that the loop
        // control stays on the scalar unit
        const int n = (int)min(e - m, (int64_t)__double_as_longlong(c[13]));
        const double R0 = xq0 - c[0], R1 = xq1 - c[1], R2 = xq2 - c[2];
        double r1 = rsqrt64(fma(R2, R2, fma(R1, R1, fma(R0, R0, 1.0))));
        double r1c = r1 * r1 * r1;
        int k = 0;
        if (!SELF) {
            // two sources per iteration: the second takes the first's far-end
            // values and leaves its own where the first's near-end values were,
            // so no register copy is made per source
            for (; k + 2 <= n; k += 2, c += 2 * RECA) {
                double r2, r2c;
                pair_acc_f64(xq0, xq1, xq2, bj0, bj1, bj2, c[0], c[1], c[2], c[3], c[4], c[5], c[6],
                             c[7], c[8], c[9], c[10], c[11], c[12], kr, nu, r1, r1c, r2, r2c, a0, a1,
                             a2, ak);
                const double *d = c + RECA;
                pair_acc_f64(xq0, xq1, xq2, bj0, bj1, bj2, d[0], d[1], d[2], d[3], d[4], d[5], d[6],
                             d[7], d[8], d[9], d[10], d[11], d[12], kr, nu, r2, r2c, r1, r1c, a0, a1,
                             a2, ak);
            }
        }
        for (; k < n; ++k, c += RECA) {
            double r2, r2c;
            if (SELF) {
                double n0 = a0, n1 = a1, n2 = a2, nk = ak;
                pair_acc_f64(xq0, xq1, xq2, bj0, bj1, bj2, c[0], c[1], c[2], c[3], c[4], c[5], c[6],
                             c[7], c[8], c[9], c[10], c[11], c[12], kr, nu, r1, r1c, r2, r2c, n0, n1,
                             n2, nk);
                const bool self = m + k == j;
                a0 = self ? a0 : n0;
                a1 = self ? a1 : n1;
                a2 = self ? a2 : n2;
                ak = self ? ak : nk;
            } else {
                pair_acc_f64(xq0, xq1, xq2, bj0, bj1, bj2, c[0], c[1], c[2], c[3], c[4], c[5], c[6],
                             c[7], c[8], c[9], c[10], c[11], c[12], kr, nu, r1, r1c, r2, r2c, a0, a1,
                             a2, ak);
            }
            r1 = r2;
            r1c = r2c;
        }
        m += n;
    }
}

__global__ __launch_bounds__(TILE) void k_pair64(const Item *__restrict__ items,
                                                 const Tile *__restrict__ tiles,
                                                 const double *__restrict__ rec,
                                                 const double *__restrict__ ra, int64_t ns,
                                                 GaussRule g, double kr, double nu, double k2,
                                                 double *__restrict__ partial)
{
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
    const double bj0 = rec[7 * ns + j], bj1 = rec[8 * ns + j], bj2 = rec[9 * ns + j];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, ak = 0.0;

    // the tile's own segments [jlo, jhi] split the range in three parts
    const int64_t jlo = tl.point_begin / Q, jhi = (tl.point_begin + tl.n_points - 1) / Q;
    const int64_t b = it.src_begin, e = it.src_end;
    const int64_t s0 = min(max(b, jlo), e), s1 = min(max(b, jhi + 1), e);
    pair64_range<false>(ra, b, s0, j, xq0, xq1, xq2, bj0, bj1, bj2, kr, nu, a0, a1, a2, ak);
    pair64_range<true>(ra, s0, s1, j, xq0, xq1, xq2, bj0, bj1, bj2, kr, nu, a0, a1, a2, ak);
    pair64_range<false>(ra, s1, e, j, xq0, xq1, xq2, bj0, bj1, bj2, kr, nu, a0, a1, a2, ak);
    a0 = fma(ak, bj0, a0);   // the b_j terms of every source at once
    a1 = fma(ak, bj1, a1);
    a2 = fma(ak, bj2, a2);
    if (valid) {
        double *o = partial + it.slot * 3 * TILE;
        o[lane] = k2 * a0;
        o[TILE + lane] = k2 * a1;
        o[2 * TILE + lane] = k2 * a2;
    }
}

void launch_pair64(const Item *items, const Tile *tiles, const double *rec, int64_t ns, const GaussRule &g,
                   double k1, double k2, double *partial, int64_t n_items, hipStream_t st)
{
    const double kr = k1 / k2, nu = 1.0 - 2.0 * kr;
    hipLaunchKernelGGL(k_pair64, dim3((unsigned)n_items), dim3(TILE), 0, st, items, tiles, rec,
                       rec + (int64_t)REC64 * ns, ns, g, kr, nu, k2, partial);
}

}  // namespace dd
