// a2, FP64 path: the all-pairs kernel k_pair64 and its launcher.
#include "dd_common.h"
#include "dd_pair64.h"

namespace dd {

// ------------------------------------------ a2: the all-pairs FP64 kernel --
// One workgroup = one work item: up to TILE target Gauss points (one per
// lane) against a contiguous source range, staged through LDS TILE sources at
// a time.  Each lane accumulates sigma b_j (3 values) over the range; the
// item's partial sums go to their own slot, reduced in a fixed order later.
// Only LDS stages that overlap the tile's own segments test for the excluded
// self pair.
template <bool SELF>
__device__ __forceinline__ void pair64_stage(double (*sh)[TILE], int n, int64_t base, int64_t j,
                                             double xq0, double xq1, double xq2, double bj0,
                                             double bj1, double bj2, double k1, double k2,
                                             double &a0, double &a1, double &a2)
{
    // runs of sources sharing consecutive nodes: one fresh inverse distance
    // per run, then each source reuses the previous source's far endpoint
    for (int m = 0; m < n;) {
        const int run = min(__builtin_amdgcn_readfirstlane((int)sh[13][m]), n - m);
        const double R0 = xq0 - sh[0][m], R1 = xq1 - sh[1][m], R2 = xq2 - sh[2][m];
        double rprev = rsqrt64(R0 * R0 + R1 * R1 + R2 * R2 + 1.0);
        for (int e = m + run; m < e; ++m) {
            double c0, c1, c2;
            pair_sigma_b_f64c(xq0, xq1, xq2, bj0, bj1, bj2, sh[0][m], sh[1][m], sh[2][m], sh[3][m],
                              sh[4][m], sh[5][m], sh[6][m], sh[7][m], sh[8][m], sh[9][m], sh[10][m],
                              sh[11][m], sh[12][m], k1, k2, true, rprev, c0, c1, c2);
            if (SELF) {
                const bool self = (base + m) == j;
                a0 += self ? 0.0 : c0;
                a1 += self ? 0.0 : c1;
                a2 += self ? 0.0 : c2;
            } else {
                a0 += c0;
                a1 += c1;
                a2 += c2;
            }
        }
    }
}

__global__ __launch_bounds__(TILE) void k_pair64(const Item *__restrict__ items,
                                                 const Tile *__restrict__ tiles,
                                                 const double *__restrict__ rec, int64_t ns,
                                                 GaussRule g, double k1, double k2,
                                                 double *__restrict__ partial)
{
    __shared__ double sh[14][TILE];
    const Item it = items[blockIdx.x];
    const Tile tl = tiles[it.tile];
    const int lane = threadIdx.x;
    const bool valid = lane < tl.n_points;
    const int64_t p = tl.point_begin + (valid ? lane : 0);
    const int Q = g.n;
    const int64_t j = p / Q;
    const int q = (int)(p - j * Q);
    const int64_t jlo = tl.point_begin / Q, jhi = (tl.point_begin + tl.n_points - 1) / Q;
    double sq = g.s[0];
    for (int k = 1; k < DD_MAX_GAUSS; ++k)
        if (k == q) sq = g.s[k];
    const double L = rec[6 * ns + j];
    const double xq0 = rec[0 * ns + j] + sq * L * rec[3 * ns + j];
    const double xq1 = rec[1 * ns + j] + sq * L * rec[4 * ns + j];
    const double xq2 = rec[2 * ns + j] + sq * L * rec[5 * ns + j];
    const double bj0 = rec[7 * ns + j], bj1 = rec[8 * ns + j], bj2 = rec[9 * ns + j];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;

    for (int64_t base = it.src_begin; base < it.src_end; base += TILE) {
        const int n = (int)min<int64_t>(TILE, it.src_end - base);
        __syncthreads();
        if (lane < n) {
#pragma unroll
            for (int k = 0; k < 14; ++k) sh[k][lane] = rec[k * ns + base + lane];
        }
        __syncthreads();
        if (base <= jhi && base + n > jlo)
            pair64_stage<true>(sh, n, base, j, xq0, xq1, xq2, bj0, bj1, bj2, k1, k2, a0, a1, a2);
        else
            pair64_stage<false>(sh, n, base, j, xq0, xq1, xq2, bj0, bj1, bj2, k1, k2, a0, a1, a2);
    }
    if (valid) {
        double *o = partial + it.slot * 3 * TILE;
        o[lane] = a0;
        o[TILE + lane] = a1;
        o[2 * TILE + lane] = a2;
    }
}

void launch_pair64(const Item *items, const Tile *tiles, const double *rec, int64_t ns, const GaussRule &g,
                   double k1, double k2, double *partial, int64_t n_items, hipStream_t st)
{
    hipLaunchKernelGGL(k_pair64, dim3((unsigned)n_items), dim3(TILE), 0, st, items, tiles, rec, ns, g, k1, k2,
                       partial);
}

}  // namespace dd
