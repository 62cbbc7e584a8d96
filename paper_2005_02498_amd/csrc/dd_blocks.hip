// Block coupling of the DD boxes to the continuum mesh (Sec. "DD-MFDM
// coupling"): block averages of a Gauss-point field, the L2 projection of a
// blockwise-constant field onto the continuous trilinear space of the block
// mesh with its two-level isoparametric interpolation to the Gauss points
// (subsection "Obtaining L^p, V at Gauss point of element"), and the
// non-negative-dissipation fix (Eq. Lp_gauss, Eq. V_gauss).
//
// Geometry: n x n square blocks of side B, thickness h, one brick through the
// thickness; each block holds m x m x 1 trilinear elements with 2 x 2 x 2
// Gauss points.  Numbering as in dd.h.
//
// The projection.  With one brick through the thickness and a field that
// does not depend on z, the consistent mass matrix of the block mesh is
// M_z (x) M_y (x) M_x (1D linear-element mass matrices, M = (L/6) tridiag(1,
// [2, 4, ..., 4, 2], 1)) and the load vector is (h/2)(1, 1) (x) b_xy, where
// b_xy at a corner node is B^2/4 times the sum of the values of the blocks
// around it.  Since M_z (1, 1) = (h/2)(1, 1), the solution does not depend on
// z and its in-plane part solves (M_y (x) M_x) A = b_xy, that is
//   A = (6/B)^2 (K^-1 (x) K^-1) b_xy,   K = tridiag(1, [2, 4, ..., 4, 2], 1):
// one tridiagonal solve along x for every row of nodes, then one along y for
// every column.  K is strictly diagonally dominant, so elimination without
// pivoting (the Thomas algorithm) is stable; its factors depend only on n and
// are computed on the host when n changes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dd_common.h"

namespace dd {

namespace {

constexpr int MAX_COMP = 16;
constexpr double ISO_GP = 0.57735026918962576451;   // 1/sqrt(3)

struct BlockGeom {
    int64_t n, m, ne;   // blocks per side, elements per block side, elements per domain side
    double B, h;
    int c;              // components
};

// Mean of the block's m^2 * 8 Gauss-point values (equal Gauss weights on the
// uniform affine mesh), one workgroup per block.  The block's values lie in m
// contiguous runs (one per row of elements) of m * 8 * c doubles; thread t
// reads entries q = t, t + S, t + 2S, ... of every run, S = c * floor(256 / c),
// so it always holds component t % c (reads are coalesced).  For each q the
// runs are read eight at a time into eight partial sums (run ly into sum
// ly % 8, the last m % 8 runs into sum 0), so that eight loads are in flight;
// the eight sums are added in order, then the per-thread sums per component
// in thread order.
__global__ __launch_bounds__(256) void k_block_average(BlockGeom G, const double *__restrict__ f,
                                                       double *__restrict__ out)
{
    __shared__ double sh[256];
    const int64_t r = blockIdx.x;
    const int64_t bx = r % G.n, by = r / G.n;
    const int t = threadIdx.x;
    const int S = G.c * (256 / G.c);
    double acc = 0.0;
    if (t < S) {
        const int m = (int)G.m, run = (int)(G.m * 8 * G.c);
        const int64_t rs = G.ne * 8 * G.c;   // doubles from one run (element row) to the next
        const double *src = f + (by * G.m * G.ne + bx * G.m) * 8 * G.c;
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int q = t; q < run; q += S) {
            int ly = 0;
            for (; ly + 8 <= m; ly += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] += src[(int64_t)(ly + u) * rs + q];
            }
            for (; ly < m; ++ly) a[0] += src[(int64_t)ly * rs + q];
        }
        acc = ((((((a[0] + a[1]) + a[2]) + a[3]) + a[4]) + a[5]) + a[6]) + a[7];
    }
    sh[t] = acc;
    __syncthreads();
    if (t < G.c) {
        double s = 0.0;
        for (int u = t; u < S; u += G.c) s += sh[u];
        out[r * G.c + t] = s / (double)(G.m * G.m * 8);
    }
}

// Load vector of the in-plane system at node (i, j): B^2/4 times the sum of the
// values of the (up to four) blocks that have it as a corner.
__global__ void k_block_rhs(BlockGeom G, const double *__restrict__ fb, double *__restrict__ A)
{
    const int64_t N = G.n + 1;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * N * G.c) return;
    const int k = (int)(t % G.c);
    const int64_t node = t / G.c, i = node % N, j = node / N;
    double s = 0.0;
    for (int dy = -1; dy <= 0; ++dy)
        for (int dx = -1; dx <= 0; ++dx) {
            const int64_t bx = i + dx, by = j + dy;
            if (bx >= 0 && bx < G.n && by >= 0 && by < G.n) s += fb[(by * G.n + bx) * G.c + k];
        }
    A[t] = 0.25 * G.B * G.B * s;
}

// Solve K y = scale * d along one line of nodes for every line: line l,
// entry q at [base(l) + q * stride] of the arrays.  The forward sweep reads
// d from `io` and leaves its results in `tmp`; the backward sweep writes y
// back to `io`.  Reading and writing different arrays lets each sweep keep
// several loads in flight.  rden[q] = 1/den_q holds the Thomas factors of K
// (den_0 = 2, den_q = diag_q - 1/den_{q-1}); with unit off-diagonals it is
// also the back-substitution factor.
__global__ void k_block_tridiag(int64_t lines, int64_t N, int64_t c, int64_t along_y, const double *__restrict__ rden,
                                double scale, double *__restrict__ io, double *__restrict__ tmp)
{
    const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (l >= lines) return;
    const int64_t k = l % c, line = l / c;
    // along x: line = row j, entries (j, i); along y: line = column i, entries (j, i)
    const int64_t base = along_y ? line * c + k : line * N * c + k;
    const int64_t stride = along_y ? N * c : c;
    double prev = 0.0;
#pragma unroll 8
    for (int64_t q = 0; q < N; ++q) {
        prev = (scale * io[base + q * stride] - prev) * rden[q];
        tmp[base + q * stride] = prev;
    }
    double next = 0.0;
#pragma unroll 8
    for (int64_t q = N - 1; q >= 0; --q) {
        next = tmp[base + q * stride] - rden[q] * next;
        io[base + q * stride] = next;
    }
}

// Two-level interpolation: the element's corner nodes from the block's
// shape functions at their block-isoparametric coordinates, then the Gauss
// point from the element's shape functions.  Restricted to an element (an
// axis-aligned sub-box of its block) the block's trilinear field is itself
// trilinear, so the element's interpolation reproduces it: the two levels
// compose to the block's shape functions at the Gauss point's block
// coordinates, which is what is evaluated here (4 weights instead of 16).
// The block field does not depend on z, so the z factors drop out.  One
// thread per Gauss point of an element row (blockIdx.y): its four weights
// once, then its CT components (CT = 0: G.c of them) into LDS, from where
// the workgroup writes its 256 points' values as one contiguous run.  im =
// 1/m, formed once on the host.
template <int CT>
__global__ __launch_bounds__(256) void k_block_interp(BlockGeom G, const double *__restrict__ A,
                                                      double *__restrict__ out, double im)
{
    __shared__ double sh[256 * (CT ? CT : MAX_COMP)];
    const int C = CT ? CT : G.c;
    const int N = (int)G.n + 1, m = (int)G.m;
    const int row_gp = (int)G.ne * 8;
    const int p0 = blockIdx.x * 256, p = p0 + (int)threadIdx.x;
    const int ey = blockIdx.y, by = ey / m;
    if (p < row_gp) {
        const int ex = p >> 3, g = p & 7;
        const int bx = ex / m;
        const double xg = (2 * (g & 1) - 1) * ISO_GP, yg = (2 * ((g >> 1) & 1) - 1) * ISO_GP;
        // the Gauss point in its block's isoparametric coordinates
        const double xb = -1.0 + ((double)(2 * (ex - bx * m) + 1) + xg) * im;
        const double yb = -1.0 + ((double)(2 * (ey - by * m) + 1) + yg) * im;
        const double f00 = (1.0 - xb) * (1.0 - yb), f10 = (1.0 + xb) * (1.0 - yb);
        const double f01 = (1.0 - xb) * (1.0 + yb), f11 = (1.0 + xb) * (1.0 + yb);
        // block-mesh nodes: (n + 1)^2 c values can pass 2^31, so these indices are 64-bit
        const int64_t q0 = ((int64_t)by * N + bx) * C, q1 = q0 + (int64_t)N * C;
#pragma unroll
        for (int k = 0; k < C; ++k)
            sh[threadIdx.x * C + k] =
                0.25 * (f00 * A[q0 + k] + f10 * A[q0 + C + k] + f01 * A[q1 + k] + f11 * A[q1 + C + k]);
    }
    __syncthreads();
    const int nv = min(256, row_gp - p0) * C;
    double *o = out + ((int64_t)ey * row_gp + p0) * C;
    for (int i = threadIdx.x; i < nv; i += 256) o[i] = sh[i];
}

// Eq. Lp_gauss: if d = T : Lp < 0, Lp <- Lp - d T / |T|^2.  Eq. V_gauss: with
// w = X T alpha, (X T alpha)_i = eps_ijk (T alpha)_jk, if beta = V . w < 0,
// V <- V - beta w / |w|^2.  Zero T (or w) leaves the field as it is.
__global__ void k_dissipation_fix(int64_t n, const double *__restrict__ T, const double *__restrict__ alpha,
                                  double *__restrict__ Lp, double *__restrict__ V)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n) return;
    double t[9];
    for (int k = 0; k < 9; ++k) t[k] = T[9 * g + k];
    if (Lp) {
        double l[9], d = 0.0, t2 = 0.0;
        for (int k = 0; k < 9; ++k) {
            l[k] = Lp[9 * g + k];
            d += t[k] * l[k];
            t2 += t[k] * t[k];
        }
        if (d < 0.0 && t2 > 0.0) {
            const double f = d / t2;
            for (int k = 0; k < 9; ++k) Lp[9 * g + k] = l[k] - f * t[k];
        }
    }
    if (V) {
        double a[9], P[9];
        for (int k = 0; k < 9; ++k) a[k] = alpha[9 * g + k];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) P[3 * i + j] = t[3 * i] * a[j] + t[3 * i + 1] * a[3 + j] + t[3 * i + 2] * a[6 + j];
        const double w0 = P[5] - P[7], w1 = P[6] - P[2], w2 = P[1] - P[3];
        const double v0 = V[3 * g], v1 = V[3 * g + 1], v2 = V[3 * g + 2];
        const double beta = v0 * w0 + v1 * w1 + v2 * w2, w2n = w0 * w0 + w1 * w1 + w2 * w2;
        if (beta < 0.0 && w2n > 0.0) {
            const double f = beta / w2n;
            V[3 * g] = v0 - f * w0;
            V[3 * g + 1] = v1 - f * w1;
            V[3 * g + 2] = v2 - f * w2;
        }
    }
}

int check_mesh(const dd_block_mesh *mesh, int c, BlockGeom &G)
{
    if (!mesh) return set_error(DD_EINVAL, "null mesh");
    if (mesh->n < 1 || mesh->m < 1) return set_error(DD_EINVAL, "n and m must be >= 1");
    if (!(mesh->B > 0.0) || !std::isfinite(mesh->B) || !(mesh->h > 0.0) || !std::isfinite(mesh->h))
        return set_error(DD_EINVAL, "block size and thickness must be finite and > 0");
    if (c < 1 || c > MAX_COMP) return set_error(DD_EINVAL, "components must be 1..%d", MAX_COMP);
    if ((int64_t)mesh->n * mesh->m > 65535) return set_error(DD_EINVAL, "n * m must be at most 65535");
    if ((int64_t)mesh->n * mesh->n > INT32_MAX) return set_error(DD_EINVAL, "n must be at most 46340");
    G.n = mesh->n;
    G.m = mesh->m;
    G.ne = G.n * G.m;
    G.B = mesh->B;
    G.h = mesh->h;
    G.c = c;
    return DD_OK;
}

}  // namespace

}  // namespace dd

using namespace dd;

extern "C" int dd_block_average(const dd_block_mesh *mesh, int c, const double *f_gp, double *f_block, void *stream)
{
    ::dd::Range range_("dd_block_average");
    clear_error();
    BlockGeom G;
    int rc;
    if ((rc = check_mesh(mesh, c, G))) return rc;
    if (!f_gp || !f_block) return set_error(DD_EINVAL, "null field");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_block_average, dim3((unsigned)(G.n * G.n)), dim3(256), 0, st, G, f_gp, f_block);
    DD_HIP(hipGetLastError());
    if (validation_on()) DD_HIP(hipStreamSynchronize(st));
    return DD_OK;
}

extern "C" int dd_block_to_gauss(const dd_block_mesh *mesh, int c, const double *f_block, double *f_gp,
                                 void *stream)
{
    ::dd::Range range_("dd_block_to_gauss");
    clear_error();
    BlockGeom G;
    int rc;
    if ((rc = check_mesh(mesh, c, G))) return rc;
    if (!f_gp || !f_block) return set_error(DD_EINVAL, "null field");
    hipStream_t st = (hipStream_t)stream;
    Workspace *ws;
    if ((rc = workspace(&ws))) return rc;
    const int64_t N = G.n + 1;
    void *p;
    if ((rc = ensure(ws, WS_BLOCK_A, sizeof(double) * 2 * N * N * c, &p))) return rc;
    double *A = (double *)p, *tmp = A + N * N * c;
    // Thomas factors of K = tridiag(1, [2, 4, ..., 4, 2], 1), size N: 1/den_q,
    // uploaded again only when n changes
    if ((rc = ensure(ws, WS_BLOCK_FAC, sizeof(double) * N, &p))) return rc;
    double *rden = (double *)p;
    if (ws->block_fac_n != N) {
        std::vector<double> fac(N);
        double den = 2.0;
        for (int64_t q = 0; q < N; ++q) {
            const double diag = (q == 0 || q == N - 1) ? 2.0 : 4.0;
            den = q == 0 ? diag : diag - 1.0 / den;
            fac[q] = 1.0 / den;
        }
        DD_HIP(hipMemcpyAsync(rden, fac.data(), sizeof(double) * N, hipMemcpyHostToDevice, st));
        DD_HIP(hipStreamSynchronize(st));   // fac is pageable and short-lived
        ws->block_fac_n = N;
    }
    const int64_t nodes = N * N * c;
    hipLaunchKernelGGL(k_block_rhs, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, st, G, f_block, A);
    const int64_t lines = N * c;
    const double scale = 6.0 / G.B;
    hipLaunchKernelGGL(k_block_tridiag, dim3((unsigned)((lines + 255) / 256)), dim3(256), 0, st, lines, N,
                       (int64_t)c, (int64_t)0, (const double *)rden, scale, A, tmp);
    hipLaunchKernelGGL(k_block_tridiag, dim3((unsigned)((lines + 255) / 256)), dim3(256), 0, st, lines, N,
                       (int64_t)c, (int64_t)1, (const double *)rden, scale, A, tmp);
    const dim3 grid((unsigned)((G.ne * 8 + 255) / 256), (unsigned)G.ne);
    const double im = 1.0 / (double)G.m;
    if (c == 9)
        hipLaunchKernelGGL(k_block_interp<9>, grid, dim3(256), 0, st, G, (const double *)A, f_gp, im);
    else if (c == 3)
        hipLaunchKernelGGL(k_block_interp<3>, grid, dim3(256), 0, st, G, (const double *)A, f_gp, im);
    else
        hipLaunchKernelGGL(k_block_interp<0>, grid, dim3(256), 0, st, G, (const double *)A, f_gp, im);
    DD_HIP(hipGetLastError());
    if (validation_on()) DD_HIP(hipStreamSynchronize(st));
    return DD_OK;
}

extern "C" int dd_dissipation_fix(int64_t n_gp, const double *T, const double *alpha, double *Lp, double *V,
                                  void *stream)
{
    ::dd::Range range_("dd_dissipation_fix");
    clear_error();
    if (n_gp < 0) return set_error(DD_EINVAL, "n_gp must be >= 0");
    if (n_gp == 0) return DD_OK;
    if (!T) return set_error(DD_EINVAL, "null stress");
    if (V && !alpha) return set_error(DD_EINVAL, "V needs alpha");
    if (n_gp > (int64_t)INT32_MAX * 256) return set_error(DD_EINVAL, "too many Gauss points");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_dissipation_fix, dim3((unsigned)((n_gp + 255) / 256)), dim3(256), 0, st, n_gp, T, alpha,
                       Lp, V);
    DD_HIP(hipGetLastError());
    if (validation_on()) DD_HIP(hipStreamSynchronize(st));
    return DD_OK;
}
