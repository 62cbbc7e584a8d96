// The exact band: for target/source pairs whose midpoints are close, the
// Peach-Koehler force of the source integrated exactly along the target
// (against the two linear shape functions) instead of by the Q-point rule.
//
// The all-pairs kernels are left as they are; for each near pair this file
// computes the difference (exact integral - Q-point rule) and the epilogue
// adds it to the target's end forces.  Steps, all on the device so that the
// force evaluation stays capturable in a graph:
//   k_near_keys     per segment its key (x1 + x2, |x2 - x1|^2, physical
//                   units), per NEAR_GROUP consecutive segments a bounding
//                   sphere;
//   k_near_list<0>  one thread per target and source split: source groups
//                   whose sphere can hold a near pair are scanned and every
//                   target counts its near sources per split;
//   k_near_count    per-target totals over the splits, their prefix within
//                   the wavefront and per-wavefront totals;
//   k_scan          prefix of the per-wavefront totals: every target's first
//                   slot in one flat array of (target, source) pairs, and the
//                   total, from which the caller sizes that array;
//   k_near_list<1>  the same search again, each split writing its sources in
//                   increasing index order straight into the target's slots
//                   (pairs past the array's capacity are dropped and flagged);
//   k_near_exact    four lanes per pair: the exact integral on panels graded
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
constexpr int NEAR_CHUNK = 128;   // source groups (spheres and keys) staged in LDS at a time

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

// One thread per segment: its key; the NEAR_GROUP lanes of a group (the last
// one may be partial) then form the group's sphere (centre C = key of its
// first segment, radius R = max |S_i - C| + sqrt(c2 |D_i|^2)), which holds
// S_j of every segment j that can be near one of them, since near(i, j)
// implies |S_i - S_j| < sqrt(c2 |D_i|^2) + sqrt(c2 |D_j|^2).  The sphere is
// stored in FP32 with R widened by 4e-6 (|C|_1 + R), more than the rounding
// of the FP32 test below can take away.
__global__ __launch_bounds__(256) void k_near_keys(NearArgs A)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, first = lane & ~(NEAR_GROUP - 1);
    if (s - (lane - first) >= A.ns) return;   // whole group past the end
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
    const double c0 = __shfl(k[0], first, 64), c1 = __shfl(k[1], first, 64), c2 = __shfl(k[2], first, 64);
    double r = 0.0;
    if (live) {
        const double e0 = k[0] - c0, e1 = k[1] - c1, e2 = k[2] - c2;
        r = sqrt(e0 * e0 + e1 * e1 + e2 * e2) + sqrt(A.c2 * k[3]);
    }
    for (int o = 1; o < NEAR_GROUP; o <<= 1) r = fmax(r, __shfl_xor(r, o, 64));
    if (lane == first) {
        r += 4e-6 * (fabs(c0) + fabs(c1) + fabs(c2) + r);
        A.sph[s / NEAR_GROUP] = make_float4((float)c0, (float)c1, (float)c2, (float)r);
    }
}

// One workgroup per 256 targets (lane = target) and source split
// (blockIdx.y): the source groups of every instance the workgroup's targets
// belong to are cut into A.splits contiguous ranges, so that a large volume
// spreads over many workgroups.  Their spheres and keys are staged in LDS
// NEAR_CHUNK groups at a time; each target tests its own key against each
// sphere in FP32 (widened as above by 4e-6 of its magnitudes) and, for the
// groups some lane of the wavefront hits, the FP64 near rule decides source
// by source.  FILL = 0 counts each split's near sources (scnt); FILL = 1
// repeats the same search and writes them, in increasing source order, to
// the target's slots of the flat pair arrays: slot woff[wave] + loc[j] plus
// the counts of the splits before this one.  Split 0 also records the
// target's first slot (ptr).
template <int FILL>
__global__ __launch_bounds__(256) void k_near_list(NearArgs A)
{
    __shared__ float4 sh[NEAR_CHUNK];
    __shared__ double shk[4 * NEAR_GROUP * NEAR_CHUNK];
    __shared__ long long sh_lo[4], sh_hi[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int split = blockIdx.y, S = A.splits;
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + tid;
    const bool live = j < A.ns;
    int64_t sb = 0, se = 0;
    double kj[4] = {0, 0, 0, 0};
    float fj0 = 3e38f, fj1 = 3e38f, fj2 = 3e38f, rj = 0.f;
    if (live) {
        const int64_t inst = inst_of(A, j);
        sb = A.seg_off ? A.seg_off[inst] : 0;
        se = A.seg_off ? A.seg_off[inst + 1] : A.ns;
        for (int c = 0; c < 4; ++c) kj[c] = A.key[4 * j + c];
        fj0 = (float)kj[0];
        fj1 = (float)kj[1];
        fj2 = (float)kj[2];
        const double r = sqrt(A.c2 * kj[3]);
        rj = (float)(r + 4e-6 * (fabs(kj[0]) + fabs(kj[1]) + fabs(kj[2]) + r));
    }
    // first slot of this split's sources (fill pass)
    int64_t slot = 0;
    if (FILL && live) {
        slot = A.woff[j >> 6] + A.loc[j];
        if (split == 0) A.ptr[j] = slot;
        for (int s2 = 0; s2 < split; ++s2) slot += A.scnt[j * S + s2];
    }
    // source groups of every instance this workgroup's targets belong to
    const long long glo = wave_min(live ? (long long)(sb / NEAR_GROUP) : (long long)INT64_MAX);
    const long long ghi = wave_max(live ? (long long)((se - 1) / NEAR_GROUP) : -1LL);
    if (lane == 0) {
        sh_lo[wv] = glo;
        sh_hi[wv] = ghi;
    }
    __syncthreads();
    long long g_lo = sh_lo[0], g_hi = sh_hi[0];
    for (int k = 1; k < 4; ++k) {
        g_lo = sh_lo[k] < g_lo ? sh_lo[k] : g_lo;
        g_hi = sh_hi[k] > g_hi ? sh_hi[k] : g_hi;
    }
    // this split's part of [g_lo, g_hi]
    const long long per = (g_hi - g_lo + S) / S;
    const long long s_lo = g_lo + split * per;
    const long long s_hi = s_lo + per - 1 < g_hi ? s_lo + per - 1 : g_hi;
    int32_t cnt = 0;
    bool full = false;
    for (long long gc = s_lo; gc <= s_hi; gc += NEAR_CHUNK) {
        __syncthreads();   // the previous chunk is no longer read
        const int n_here = (int)(s_hi - gc + 1 < NEAR_CHUNK ? s_hi - gc + 1 : NEAR_CHUNK);
        if (tid < NEAR_CHUNK) {
            const long long g = gc + tid;
            sh[tid] = tid < n_here ? A.sph[g] : make_float4(3e38f, 3e38f, 3e38f, 0.f);
        }
        // the keys of the chunk's sources, coalesced
        const int64_t kbase = 4 * gc * NEAR_GROUP, kend = 4 * A.ns;
        for (int q = tid; q < 4 * NEAR_GROUP * NEAR_CHUNK; q += 256)
            shk[q] = kbase + q < kend ? A.key[kbase + q] : 0.0;
        __syncthreads();
        // four spheres per round (independent tests); entries past n_here hold
        // a sentinel that no target hits
        for (int k = 0; k < n_here; k += 4) {
            bool hit[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 c = sh[k + u];
                const float e0 = fj0 - c.x, e1 = fj1 - c.y, e2 = fj2 - c.z, rr = c.w + rj;
                hit[u] = live && e0 * e0 + e1 * e1 + e2 * e2 < rr * rr;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (__ballot(hit[u]) == 0) continue;
                const int64_t i0 = (gc + k + u) * NEAR_GROUP;
                const double *kg = shk + 4 * NEAR_GROUP * (k + u);
#pragma unroll
                for (int q = 0; q < NEAR_GROUP; ++q) {
                    const int64_t i = i0 + q;
                    if (hit[u] && i < A.ns && i >= sb && i < se && i != j && near_test(kg + 4 * q, kj, A.c2)) {
                        if (FILL) {
                            const int64_t p = slot + cnt;
                            if (p < A.pair_cap) {
                                A.pair_t[p] = (int32_t)j;
                                A.pair_s[p] = (int32_t)i;
                            } else {
                                full = true;
                            }
                        }
                        ++cnt;
                    }
                }
            }
        }
    }
    if (!FILL && live) A.scnt[j * S + split] = cnt;
    if (full) atomicOr(A.flags, FLAG_NEAR_FULL);
}

// One thread per target: the near count over all splits, its exclusive
// prefix within the wavefront, and per-wavefront totals for the scan.
__global__ __launch_bounds__(256) void k_near_count(NearArgs A)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t c = 0;
    if (j < A.ns)
        for (int s = 0; s < A.splits; ++s) c += A.scnt[j * A.splits + s];
    int64_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (j < A.ns) {
        A.cnt[j] = (int32_t)c;
        A.loc[j] = incl - c;
    }
    const int64_t w = j >> 6;
    if (lane == 63 && w < A.n_waves) A.wtot[w] = incl;
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

// Four lanes per near pair (grid-stride over pairs).  The lanes of a pair
// build the same panels; lane r takes points r, r + 4 and r + 8 of each
// 12-point panel and the Q-point nodes q = r (mod 4); the four partial sums
// are combined by a fixed butterfly, so results are reproducible.
// corr[p] = L_j k2 ((E - G) x t_j) for the two ends, E the exact and G the
// Q-point weighted integrals of sigma^i b_j / k2, in the units of the
// epilogue's end forces.
constexpr int LANES_PER_PAIR = 4;

__global__ __launch_bounds__(256) void k_near_exact(NearArgs A)
{
    const int64_t ns = A.ns;
    const int64_t P0 = A.woff[A.n_waves];
    const int64_t P = P0 < A.pair_cap ? P0 : A.pair_cap;
    const int r = threadIdx.x % LANES_PER_PAIR;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / LANES_PER_PAIR;
    const double *rec = A.rec;
    const double *ra = rec + (int64_t)REC64 * ns;
    // every lane of a wavefront runs the same number of rounds (shuffles below)
    const int64_t first = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / LANES_PER_PAIR;
    const int64_t wave_first = first - (threadIdx.x & 63) / LANES_PER_PAIR;
    for (int64_t pw = wave_first; pw < P; pw += stride) {
        const int64_t p = pw + (first - wave_first);
        const bool live = p < P;
        double a10 = 0, a11 = 0, a12 = 0, a20 = 0, a21 = 0, a22 = 0;
        double t0 = 0, t1 = 0, t2 = 0, L = 0;
        if (live) {
            const int64_t j = A.pair_t[p], i = A.pair_s[p];
            const double X0 = rec[0 * ns + j], X1 = rec[1 * ns + j], X2 = rec[2 * ns + j];
            t0 = rec[3 * ns + j]; t1 = rec[4 * ns + j]; t2 = rec[5 * ns + j];
            L = rec[6 * ns + j];
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
            double lo = 0.0, wd = 1.0;
            int panels = 0;
            while (lo < 1.0) {
                double hi = fmin(lo + wd, 1.0);
                while (hi - lo > 1e-7 && !panel_ok(lo, hi, F)) hi = lo + 0.5 * (hi - lo);
                const double h = hi - lo;
#pragma unroll
                for (int k = r; k < PANEL_POINTS; k += LANES_PER_PAIR) {
                    const double u = lo + h * A.gp.s[k];
                    const double wk = h * A.gp.w[k];
                    const double uL = u * L;
                    double g0 = 0, g1 = 0, g2 = 0;
                    pair_acc_isolated_f64(X0 + uL * t0, X1 + uL * t1, X2 + uL * t2, b0, b1, b2, d, A.kr, A.nu,
                                          g0, g1, g2);
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
            for (int q = r; q < A.g.n; q += LANES_PER_PAIR) {
                const double u = A.g.s[q], uL = u * L;
                double g0 = 0, g1 = 0, g2 = 0;
                pair_acc_isolated_f64(X0 + uL * t0, X1 + uL * t1, X2 + uL * t2, b0, b1, b2, d, A.kr, A.nu, g0,
                                      g1, g2);
                const double w1 = A.g.w[q] * (1.0 - u), w2 = A.g.w[q] * u;
                a10 -= w1 * g0; a11 -= w1 * g1; a12 -= w1 * g2;
                a20 -= w2 * g0; a21 -= w2 * g1; a22 -= w2 * g2;
            }
        }
        // butterfly over the pair's four lanes (every lane of the wavefront takes part)
#pragma unroll
        for (int o = 1; o < LANES_PER_PAIR; o <<= 1) {
            a10 += __shfl_xor(a10, o, 64); a11 += __shfl_xor(a11, o, 64); a12 += __shfl_xor(a12, o, 64);
            a20 += __shfl_xor(a20, o, 64); a21 += __shfl_xor(a21, o, 64); a22 += __shfl_xor(a22, o, 64);
        }
        if (live && r == 0) {
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
}

}  // namespace

void launch_near_count(const NearArgs &A, hipStream_t st)
{
    if (A.ns <= 0) return;
    const unsigned tb = (unsigned)((A.ns + 255) / 256);
    hipLaunchKernelGGL(k_near_keys, dim3(tb), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_near_list<0>, dim3(tb, (unsigned)A.splits), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_near_count, dim3(tb), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, (const int64_t *)A.wtot, A.n_waves, A.woff);
}

void launch_near_fill(const NearArgs &A, hipStream_t st)
{
    if (A.ns <= 0) return;
    const unsigned tb = (unsigned)((A.ns + 255) / 256);
    hipLaunchKernelGGL(k_near_list<1>, dim3(tb, (unsigned)A.splits), dim3(256), 0, st, A);
    const int64_t cap_blocks = (A.pair_cap * LANES_PER_PAIR + 255) / 256;
    const unsigned eb = (unsigned)(cap_blocks < 8192 ? (cap_blocks > 0 ? cap_blocks : 1) : 8192);
    hipLaunchKernelGGL(k_near_exact, dim3(eb), dim3(256), 0, st, A);
}

}  // namespace dd
