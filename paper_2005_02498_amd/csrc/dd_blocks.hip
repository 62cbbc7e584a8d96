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
// are computed once on the host.
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
// uniform affine mesh), one workgroup per block, fixed-order tree reduction.
__global__ __launch_bounds__(256) void k_block_average(BlockGeom G, const double *__restrict__ f,
                                                       double *__restrict__ out)
{
    __shared__ double sh[256][MAX_COMP + 1];
    const int64_t r = blockIdx.x;
    const int64_t bx = r % G.n, by = r / G.n;
    const int64_t per = G.m * G.m * 8;
    double acc[MAX_COMP];
    for (int k = 0; k < MAX_COMP; ++k) acc[k] = 0.0;
    for (int64_t q = threadIdx.x; q < per; q += 256) {
        const int64_t el = q >> 3, g = q & 7;
        const int64_t ex = bx * G.m + el % G.m, ey = by * G.m + el / G.m;
        const double *src = f + ((ey * G.ne + ex) * 8 + g) * G.c;
        for (int k = 0; k < G.c; ++k) acc[k] += src[k];
    }
    for (int k = 0; k < G.c; ++k) sh[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < G.c; ++k) sh[threadIdx.x][k] += sh[threadIdx.x + s][k];
        __syncthreads();
    }
    if ((int)threadIdx.x < G.c) out[r * G.c + threadIdx.x] = sh[0][threadIdx.x] / (double)per;
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

// In-place solve K y = scale * d along one line of nodes for every line:
// line l, entry q at A[base(l) + q * stride].  den[q] and cp[q] are the
// Thomas factors of K (den_0 = 2, cp_q = 1/den_q, den_q = diag_q - cp_{q-1}).
__global__ void k_block_tridiag(int64_t lines, int64_t N, int64_t c, int64_t along_y, const double *__restrict__ den,
                                const double *__restrict__ cp, double scale, double *__restrict__ A)
{
    const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (l >= lines) return;
    const int64_t k = l % c, line = l / c;
    // along x: line = row j, entries (j, i); along y: line = column i, entries (j, i)
    const int64_t base = along_y ? line * c + k : line * N * c + k;
    const int64_t stride = along_y ? N * c : c;
    double prev = 0.0;
    for (int64_t q = 0; q < N; ++q) {
        const double d = scale * A[base + q * stride];
        prev = (d - prev) / den[q];
        A[base + q * stride] = prev;
    }
    double next = 0.0;
    for (int64_t q = N - 1; q >= 0; --q) {
        const double y = A[base + q * stride] - (q + 1 < N ? cp[q] * next : 0.0);
        A[base + q * stride] = y;
        next = y;
    }
}

// Two-level interpolation: the element's corner nodes from the block's
// shape functions at their block-isoparametric coordinates, then the Gauss
// point from the element's shape functions.  The block field does not depend
// on z, so the z factors of both levels sum to one and drop out.
__global__ void k_block_interp(BlockGeom G, const double *__restrict__ A, double *__restrict__ out)
{
    const int64_t N = G.n + 1;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= G.ne * G.ne * 8) return;
    const int64_t e = p >> 3;
    const int g = (int)(p & 7);
    const int64_t ex = e % G.ne, ey = e / G.ne;
    const int64_t bx = ex / G.m, by = ey / G.m;
    const double xg = (2 * (g & 1) - 1) * ISO_GP, yg = (2 * ((g >> 1) & 1) - 1) * ISO_GP;
    double val[MAX_COMP];
    for (int k = 0; k < G.c; ++k) val[k] = 0.0;
    for (int ky = 0; ky < 2; ++ky)
        for (int kx = 0; kx < 2; ++kx) {
            // element corner (kx, ky) in block coordinates
            const double xb = -1.0 + 2.0 * (double)(ex - bx * G.m + kx) / (double)G.m;
            const double yb = -1.0 + 2.0 * (double)(ey - by * G.m + ky) / (double)G.m;
            const double we = 0.25 * (1.0 + (2 * kx - 1) * xg) * (1.0 + (2 * ky - 1) * yg);
            for (int qy = 0; qy < 2; ++qy)
                for (int qx = 0; qx < 2; ++qx) {
                    const double wb = 0.25 * (1.0 + (2 * qx - 1) * xb) * (1.0 + (2 * qy - 1) * yb);
                    const double *a = A + ((by + qy) * N + bx + qx) * G.c;
                    for (int k = 0; k < G.c; ++k) val[k] += we * wb * a[k];
                }
        }
    for (int k = 0; k < G.c; ++k) out[p * G.c + k] = val[k];
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
    if ((int64_t)mesh->n * mesh->m > 65536) return set_error(DD_EINVAL, "n * m must be at most 65536");
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
    if ((rc = ensure(ws, WS_BLOCK_A, sizeof(double) * N * N * c, &p))) return rc;
    double *A = (double *)p;
    // Thomas factors of K = tridiag(1, [2, 4, ..., 4, 2], 1), size N
    std::vector<double> fac(2 * N);
    double *den = fac.data(), *cp = fac.data() + N;
    for (int64_t q = 0; q < N; ++q) {
        const double diag = (q == 0 || q == N - 1) ? 2.0 : 4.0;
        den[q] = q == 0 ? diag : diag - cp[q - 1];
        cp[q] = 1.0 / den[q];
    }
    if ((rc = ensure(ws, WS_BLOCK_FAC, sizeof(double) * 2 * N, &p))) return rc;
    double *dfac = (double *)p;
    DD_HIP(hipMemcpyAsync(dfac, fac.data(), sizeof(double) * 2 * N, hipMemcpyHostToDevice, st));
    DD_HIP(hipStreamSynchronize(st));   // fac is pageable and short-lived
    const int64_t nodes = N * N * c;
    hipLaunchKernelGGL(k_block_rhs, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, st, G, f_block, A);
    const int64_t lines = N * c;
    const double scale = 6.0 / G.B;
    hipLaunchKernelGGL(k_block_tridiag, dim3((unsigned)((lines + 255) / 256)), dim3(256), 0, st, lines, N,
                       (int64_t)c, (int64_t)0, (const double *)dfac, (const double *)(dfac + N), scale, A);
    hipLaunchKernelGGL(k_block_tridiag, dim3((unsigned)((lines + 255) / 256)), dim3(256), 0, st, lines, N,
                       (int64_t)c, (int64_t)1, (const double *)dfac, (const double *)(dfac + N), scale, A);
    const int64_t gps = G.ne * G.ne * 8;
    hipLaunchKernelGGL(k_block_interp, dim3((unsigned)((gps + 255) / 256)), dim3(256), 0, st, G,
                       (const double *)A, f_gp);
    DD_HIP(hipGetLastError());
    if (validation_on()) DD_HIP(hipStreamSynchronize(st));
    return DD_OK;
}

extern "C" int dd_dissipation_fix(int64_t n_gp, const double *T, const double *alpha, double *Lp, double *V,
                                  void *stream)
{
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
