// The exact band: for target/source pairs whose midpoints are close, the
// Peach-Koehler force of the source integrated exactly along the target
// (against the two linear shape functions) instead of by the Q-point rule.
//
// The all-pairs kernels are left as they are; for each near pair this file
// computes the difference (exact integral - Q-point rule) and the epilogue
// adds it to the target's end forces.  Steps, all on the device so that the
// force evaluation stays capturable in a graph:
//   k_near_groups   per 64 consecutive segments: the keys (x1 + x2, |x2 - x1|^2,
//                   physical units) and a bounding sphere of the group;
//   k_near_list     one wavefront per 64 targets: source groups whose sphere
//                   can hold a near pair are scanned and every target keeps
//                   its near sources in increasing index order (at most
//                   NEAR_CAP), with per-wavefront totals;
//   k_scan          prefix of the per-wavefront totals;
//   k_near_compact  one flat array of (target, source) pairs;
//   k_near_exact    one thread per pair: the exact integral on panels graded
//                   towards the integrand's complex singularities, minus the
//                   Q-point rule, as two end-force vectors.
//
// Near rule (the same arithmetic, in the same order, as the oracle's, with
// contraction of products into fused multiply-adds turned off so that the
// decision is bitwise the same): with S = x1 + x2 and D = x2 - x1,
//   near(i, j)  <=>  |S_i - S_j|^2 < c2 (|D_i|^2 + |D_j|^2),   c2 = 2 eta^2,
// i.e. midpoints closer than eta sqrt((L_i^2 + L_j^2) / 2).
//
// The exact integral: along the target x(u) = x1 + u L t, u in [0, 1], the
// field of a straight source is analytic except near three complex points
// (lengths in units of a, where R_a vanishes): the projections of the two
// source endpoints, at u_k +- i sqrt(e_k^2 + 1)/L with e_k their distance
// from the target line, and the closest approach of the two lines, at
// u_c +- i sqrt(e^2 + 1)/(L sin theta), where the squared distance to the
// source line plus the core term vanishes.  Panels are grown left to right
// and halved until every such point lies outside the panel's Bernstein
// ellipse of parameter 5; each panel takes 12-point Gauss-Legendre (error
// ~5^-24 times the integrand's size on the ellipse: within 1e-14 of the
// pair's integral on loop-like geometries, at about 40 evaluations a pair).
#include <hip/hip_runtime.h>

#include "dd_common.h"
#include "dd_pair64.h"
#include "dd_scan.h"

namespace dd {

namespace {

constexpr double ELLIPSE_IA2 = 1.0 / (2.6 * 2.6);   // 1/A^2, A = (5 + 1/5)/2
constexpr double ELLIPSE_IB2 = 1.0 / (2.4 * 2.4);   // 1/B^2, B = (5 - 1/5)/2
constexpr int PANEL_POINTS = 12;
constexpr int MAX_PANELS = 256;

__device__ __forceinline__ int64_t inst_of(const NearArgs &A, int64_t s)
{
    return A.seg_inst ? A.seg_inst[s] : 0;
}

// x1 + x2 and |x2 - x1|^2 of segment s in the caller's units, written out
// without contraction (the near decision must match the oracle's bit for bit).
__device__ __forceinline__ void near_key(const double *xa, const double *xb, double *k)
{
#pragma clang fp contract(off)
    const double d0 = xb[0] - xa[0], d1 = xb[1] - xa[1], d2 = xb[2] - xa[2];
    k[0] = xa[0] + xb[0];
    k[1] = xa[1] + xb[1];
    k[2] = xa[2] + xb[2];
    k[3] = d0 * d0 + d1 * d1 + d2 * d2;
}

__device__ __forceinline__ bool near_test(const double *ki, const double *kj, double c2)
{
#pragma clang fp contract(off)
    const double e0 = ki[0] - kj[0], e1 = ki[1] - kj[1], e2 = ki[2] - kj[2];
    const double dd = e0 * e0 + e1 * e1 + e2 * e2;
    return dd < c2 * (ki[3] + kj[3]);
}

template <class T>
__device__ __forceinline__ T wave_max(T v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const T u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_min(T v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const T u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    return v;
}

// One wavefront per group of 64 consecutive segments (the last one may be
// partial): keys, and a sphere (centre C = key of the group's first segment,
// radius R = max |S_i - C| + sqrt(c2 |D_i|^2)) holding, for every segment of
// the group, every point closer than the band allows.
__global__ __launch_bounds__(256) void k_near_groups(NearArgs A)
{
    const int lane = threadIdx.x & 63;
    const int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t s = g * 64 + lane;
    if (g * 64 >= A.ns) return;   // whole wavefront
    const bool live = s < A.ns;
    double k[4] = {0, 0, 0, 0};
    if (live) {
        const int64_t inst = inst_of(A, s);
        const int64_t n0 = A.node_off ? A.node_off[inst] : 0;
        const int64_t nn = A.node_off ? A.node_off[inst + 1] - n0 : A.nn;
        int64_t i1 = A.seg_nodes[s], i2 = A.seg_nodes[A.ns + s];
        // out-of-range indices are reported by the segment preparation; stay in bounds here
        if (i1 < 0 || i1 >= nn || i2 < 0 || i2 >= nn) i1 = i2 = 0;
        const double xa[3] = {A.x[n0 + i1], A.x[A.nn + n0 + i1], A.x[2 * A.nn + n0 + i1]};
        const double xb[3] = {A.x[n0 + i2], A.x[A.nn + n0 + i2], A.x[2 * A.nn + n0 + i2]};
        near_key(xa, xb, k);
        double *o = A.key + 4 * s;
        o[0] = k[0]; o[1] = k[1]; o[2] = k[2]; o[3] = k[3];
    }
    const double c0 = __shfl(k[0], 0, 64), c1 = __shfl(k[1], 0, 64), c2 = __shfl(k[2], 0, 64);
    double r = 0.0;
    if (live) {
        const double e0 = k[0] - c0, e1 = k[1] - c1, e2 = k[2] - c2;
        r = sqrt(e0 * e0 + e1 * e1 + e2 * e2) + sqrt(A.c2 * k[3]);
    }
    r = wave_max(r);
    if (lane == 0) {
        double *o = A.grp + 4 * g;
        o[0] = c0; o[1] = c1; o[2] = c2;
        o[3] = r * (1.0 + 1e-9);   // rounding margin: the sphere test only pre-selects
    }
}

// One wavefront per group of 64 targets (lane = target).
__global__ __launch_bounds__(256) void k_near_list(NearArgs A)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t j = w * 64 + lane;
    if (w * 64 >= A.ns) return;   // whole wavefront
    const bool live = j < A.ns;
    int64_t sb = 0, se = 0;
    double kj[4] = {0, 0, 0, 0};
    if (live) {
        const int64_t inst = inst_of(A, j);
        sb = A.seg_off ? A.seg_off[inst] : 0;
        se = A.seg_off ? A.seg_off[inst + 1] : A.ns;
        for (int c = 0; c < 4; ++c) kj[c] = A.key[4 * j + c];
    }
    // source groups of every instance this wavefront's targets belong to
    const int64_t g_lo = wave_min(live ? sb / 64 : INT64_MAX);
    const int64_t g_hi = wave_max(live ? (se - 1) / 64 : (int64_t)-1);
    const double *gt = A.grp + 4 * w;
    const double tc0 = gt[0], tc1 = gt[1], tc2 = gt[2], tr = gt[3];
    int32_t cnt = 0;
    int32_t *out = A.list + j * NEAR_CAP;
    for (int64_t g0 = g_lo; g0 <= g_hi; g0 += 64) {
        const int64_t g = g0 + lane;
        bool hit = false;
        if (g <= g_hi) {
            const double *gs = A.grp + 4 * g;
            const double e0 = gs[0] - tc0, e1 = gs[1] - tc1, e2 = gs[2] - tc2;
            const double rr = (gs[3] + tr) * (1.0 + 1e-9);
            hit = e0 * e0 + e1 * e1 + e2 * e2 < rr * rr;
        }
        uint64_t mask = __ballot(hit);
        while (mask) {
            const int b = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            const int64_t i0 = (g0 + b) * 64, i1 = i0 + 64 < A.ns ? i0 + 64 : A.ns;
            for (int64_t i = i0; i < i1; ++i) {
                const double *ki = A.key + 4 * i;
                if (live && i >= sb && i < se && i != j && near_test(ki, kj, A.c2)) {
                    if (cnt < NEAR_CAP) out[cnt] = (int32_t)i;
                    ++cnt;
                }
            }
        }
    }
    if (cnt > NEAR_CAP) atomicOr(A.flags, FLAG_NEAR_FULL);
    int32_t c = cnt < NEAR_CAP ? cnt : NEAR_CAP;
    // exclusive prefix of the clamped counts within the wavefront
    int32_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (live) {
        A.cnt[j] = c;
        A.loc[j] = incl - c;
    }
    if (lane == 63) A.wtot[w] = incl;
}

// One thread per target: its pairs at woff[wave] + loc[j] in the flat arrays.
__global__ void k_near_compact(NearArgs A)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= A.ns) return;
    const int64_t base = (int64_t)A.woff[j >> 6] + A.loc[j];
    const int c = A.cnt[j];
    A.ptr[j] = (int32_t)base;
    for (int k = 0; k < c; ++k) {
        const int64_t p = base + k;
        if (p >= A.pair_cap) {
            atomicOr(A.flags, FLAG_NEAR_FULL);
            break;
        }
        A.pair_t[p] = (int32_t)j;
        A.pair_s[p] = A.list[j * NEAR_CAP + k];
    }
}

struct Focus {
    double p[3], d[3];   // real part and distance from the real axis, in target units u
};

__device__ __forceinline__ bool panel_ok(double lo, double hi, const Focus &F)
{
    const double ih = 2.0 / (hi - lo), c = 0.5 * (lo + hi);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double X = (F.p[k] - c) * ih, Y = F.d[k] * ih;
        if (X * X * ELLIPSE_IA2 + Y * Y * ELLIPSE_IB2 < 1.0) return false;
    }
    return true;
}

// One thread per near pair (grid-stride).  corr[p] = L_j k2 ((E - G) x t_j)
// for the two ends, E the exact and G the Q-point weighted integrals of
// sigma^i b_j / k2, in the units of the epilogue's end forces.
__global__ __launch_bounds__(256) void k_near_exact(NearArgs A)
{
    const int64_t ns = A.ns;
    const int64_t P0 = A.woff[A.n_waves];
    const int64_t P = P0 < A.pair_cap ? P0 : A.pair_cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const double *rec = A.rec;
    const double *ra = rec + (int64_t)REC64 * ns;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += stride) {
        const int64_t j = A.pair_t[p], i = A.pair_s[p];
        const double X0 = rec[0 * ns + j], X1 = rec[1 * ns + j], X2 = rec[2 * ns + j];
        const double t0 = rec[3 * ns + j], t1 = rec[4 * ns + j], t2 = rec[5 * ns + j];
        const double L = rec[6 * ns + j];
        const double b0 = rec[7 * ns + j], b1 = rec[8 * ns + j], b2 = rec[9 * ns + j];
        const double *d = ra + i * RECA;
        const double iL = 1.0 / L;
        // the three singular points, in units of the target parameter u
        Focus F;
        const double st0 = d[3], st1 = d[4], st2 = d[5], Ls = d[6];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const double w0 = d[0] + e * Ls * st0 - X0, w1 = d[1] + e * Ls * st1 - X1,
                         w2 = d[2] + e * Ls * st2 - X2;
            const double y = w0 * t0 + w1 * t1 + w2 * t2;
            const double h0 = w0 - y * t0, h1 = w1 - y * t1, h2 = w2 - y * t2;
            F.p[e] = y * iL;
            F.d[e] = sqrt(h0 * h0 + h1 * h1 + h2 * h2 + 1.0) * iL;
        }
        {
            // closest approach of the lines X + alpha t and P1 + beta ts
            const double n0 = t1 * st2 - t2 * st1, n1 = t2 * st0 - t0 * st2, n2 = t0 * st1 - t1 * st0;
            const double s2 = n0 * n0 + n1 * n1 + n2 * n2;   // sin^2 theta
            if (s2 > 1e-20) {
                const double w0 = X0 - d[0], w1 = X1 - d[1], w2 = X2 - d[2];
                const double ct = t0 * st0 + t1 * st1 + t2 * st2;
                const double dt = t0 * w0 + t1 * w1 + t2 * w2, ds = st0 * w0 + st1 * w1 + st2 * w2;
                const double alpha = (ct * ds - dt) / s2;
                const double e = (w0 * n0 + w1 * n1 + w2 * n2);
                F.p[2] = alpha * iL;
                F.d[2] = sqrt((e * e / s2 + 1.0) / s2) * iL;
            } else {
                F.p[2] = 0.0;
                F.d[2] = 1e300;   // parallel lines: the distance to the source line is constant
            }
        }
        double a10 = 0, a11 = 0, a12 = 0, a20 = 0, a21 = 0, a22 = 0;
        double lo = 0.0, wd = 1.0;
        int panels = 0;
        while (lo < 1.0) {
            double hi = fmin(lo + wd, 1.0);
            while (hi - lo > 1e-7 && !panel_ok(lo, hi, F)) hi = lo + 0.5 * (hi - lo);
            const double h = hi - lo;
            for (int k = 0; k < PANEL_POINTS; ++k) {
                const double u = lo + h * A.gp.s[k];
                const double wk = h * A.gp.w[k];
                const double uL = u * L;
                double g0 = 0, g1 = 0, g2 = 0;
                pair_acc_isolated_f64(X0 + uL * t0, X1 + uL * t1, X2 + uL * t2, b0, b1, b2, d, A.kr, A.nu, g0,
                                      g1, g2);
                const double w1 = wk * (1.0 - u), w2 = wk * u;
                a10 += w1 * g0; a11 += w1 * g1; a12 += w1 * g2;
                a20 += w2 * g0; a21 += w2 * g1; a22 += w2 * g2;
            }
            wd = 2.0 * h;
            lo = hi;
            if (++panels >= MAX_PANELS) {
                atomicOr(A.flags, FLAG_NEAR_PANELS);
                break;
            }
        }
        // minus the Q-point rule the all-pairs kernel applied to this pair
        for (int q = 0; q < A.g.n; ++q) {
            const double u = A.g.s[q], uL = u * L;
            double g0 = 0, g1 = 0, g2 = 0;
            pair_acc_isolated_f64(X0 + uL * t0, X1 + uL * t1, X2 + uL * t2, b0, b1, b2, d, A.kr, A.nu, g0, g1,
                                  g2);
            const double w1 = A.g.w[q] * (1.0 - u), w2 = A.g.w[q] * u;
            a10 -= w1 * g0; a11 -= w1 * g1; a12 -= w1 * g2;
            a20 -= w2 * g0; a21 -= w2 * g1; a22 -= w2 * g2;
        }
        const double sc = L * A.k2;
        double *o = A.corr + 6 * p;
        o[0] = sc * (a11 * t2 - a12 * t1);
        o[1] = sc * (a12 * t0 - a10 * t2);
        o[2] = sc * (a10 * t1 - a11 * t0);
        o[3] = sc * (a21 * t2 - a22 * t1);
        o[4] = sc * (a22 * t0 - a20 * t2);
        o[5] = sc * (a20 * t1 - a21 * t0);
    }
}

}  // namespace

void launch_near(const NearArgs &A, hipStream_t st)
{
    if (A.ns <= 0) return;
    const int64_t waves = (A.ns + 63) / 64;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    hipLaunchKernelGGL(k_near_groups, dim3(blocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_near_list, dim3(blocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, (const int32_t *)A.wtot, waves, A.woff);
    hipLaunchKernelGGL(k_near_compact, dim3((unsigned)((A.ns + 255) / 256)), dim3(256), 0, st, A);
    const int64_t cap_blocks = (A.pair_cap + 255) / 256;
    const unsigned eb = (unsigned)(cap_blocks < 4096 ? (cap_blocks > 0 ? cap_blocks : 1) : 4096);
    hipLaunchKernelGGL(k_near_exact, dim3(eb), dim3(256), 0, st, A);
}

}  // namespace dd
