// Pair-force path of libdd.so: segment preparation, the all-pairs kernels,
// the per-segment quadrature epilogue, node gathers, glide + Euler, slip
// rates, and the public entry points dd_nodal_forces / dd_glide_step /
// dd_burst_batch.
//
// Units inside the kernels: lengths are divided by the core width a and
// stresses by mu, so the non-singular closed form is evaluated with a = 1 and
// mu = 1; forces are multiplied back by mu a^2.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "dd_common.h"
#include "dd_pair64.h"
#include "dd_scan.h"

namespace dd {

// ---------------------------------------------------------------- helpers --
__global__ void k_fill_u32(unsigned *p, int64_t n, unsigned v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_check_finite(const double *p, int64_t n, unsigned *flags)
{
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(p[i]);
    if (bad) atomicOr(flags, FLAG_NONFINITE);
}

static inline unsigned grid_for(int64_t n, int block = 256, int64_t cap = 4096)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Instance lookup helpers: node_off / seg_off / seg_inst may be null for a
// single volume (instance 0 owns everything).
struct Layout {
    const int64_t *node_off;   // device [n_inst+1] or null
    const int64_t *seg_off;    // device [n_inst+1] or null
    const int32_t *seg_inst;   // device [n_segs] or null
    const int64_t *tile_begin; // device [n_inst+1] or null
    int64_t nn, ns;            // totals
};

__device__ __forceinline__ int seg_instance(const Layout &L, int64_t s)
{
    return L.seg_inst ? L.seg_inst[s] : 0;
}
__device__ __forceinline__ int64_t node_begin(const Layout &L, int inst)
{
    return L.node_off ? L.node_off[inst] : 0;
}
__device__ __forceinline__ int64_t node_count(const Layout &L, int inst)
{
    return L.node_off ? L.node_off[inst + 1] - L.node_off[inst] : L.nn;
}
__device__ __forceinline__ int64_t seg_begin(const Layout &L, int inst)
{
    return L.seg_off ? L.seg_off[inst] : 0;
}

// Global node ids of segment s (instance-local indices clamped into range on
// the device, flagged when they were not).
__device__ __forceinline__ bool seg_ends(const Layout &L, const int32_t *seg_nodes, int64_t s,
                                         int64_t &g1, int64_t &g2)
{
    int inst = seg_instance(L, s);
    int64_t n0 = node_begin(L, inst), nn = node_count(L, inst);
    int64_t i1 = seg_nodes[s], i2 = seg_nodes[L.ns + s];
    bool ok = nn > 0 && i1 >= 0 && i1 < nn && i2 >= 0 && i2 < nn;
    if (!ok) {
        i1 = 0;
        i2 = 0;
        if (nn <= 0) n0 = 0;   // only reachable when nn_total > 0 is checked on host
    }
    g1 = n0 + i1;
    g2 = n0 + i2;
    return ok;
}

// -------------------------------------------------------- a1: preparation --
struct PrepArgs {
    Layout L;
    const double *x;
    const int32_t *seg_nodes;
    const double *burgers;
    const double *normal;
    double inv_a;
    double *rec64;        // [REC64][ns], then [ns][RECA]
    float *rec32;         // [ns][REC32A] or null
    float cut;            // near-field cutoff in units of a (FP32 record)
    int quadn;            // source-quadrature points of the mixed kernel variant (0, 2, 3)
    int32_t *sys;         // [ns] slip system or -1, or null
    unsigned *flags;
};

constexpr int PREP_BLOCK = 256;   // threads per workgroup of k_seg_prep

// FP64 record of segment s with nodes g1 -> g2, in units of a: x1, the unit
// tangent t, the length L, b and c = b x t (r[0..12]).  Returns L.
__device__ __forceinline__ double seg_record(const double *x, int64_t nn, int64_t g1, int64_t g2,
                                             const double *burgers, int64_t ns, int64_t s, double inv_a, double *r)
{
    double d[3];
    for (int k = 0; k < 3; ++k) {
        r[k] = x[k * nn + g1] * inv_a;
        d[k] = x[k * nn + g2] * inv_a - r[k];
        r[7 + k] = burgers[k * ns + s] * inv_a;
    }
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double iL = 1.0 / L;
    for (int k = 0; k < 3; ++k) r[3 + k] = d[k] * iL;
    r[6] = L;
    r[10] = r[8] * r[5] - r[9] * r[4];
    r[11] = r[9] * r[3] - r[7] * r[5];
    r[12] = r[7] * r[4] - r[8] * r[3];
    return L;
}

// Slip system of a segment (FCC table): the system whose plane normal and
// slip direction match its normal and Burgers vector up to sign, or -1.
__device__ __forceinline__ int seg_system(const double *b, const double *nv)
{
    int found = -1;
    const double bl = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    for (int al = 0; al < 12 && found < 0; ++al) {
        double n[3], m[3];
        fcc(al, n, m);
        const double cn = fabs(n[0] * nv[0] + n[1] * nv[1] + n[2] * nv[2]);
        const double cb = fabs(m[0] * b[0] + m[1] * b[1] + m[2] * b[2]);
        if (cn > 1.0 - 1e-6 && bl > 0.0 && cb > (1.0 - 1e-6) * bl) found = al;
    }
    return found;
}

__global__ __launch_bounds__(PREP_BLOCK) void k_seg_prep(PrepArgs A)
{
    __shared__ int64_t sh_g1[PREP_BLOCK], sh_g2[PREP_BLOCK];
    __shared__ int sh_inst[PREP_BLOCK];
    __shared__ unsigned char sh_chain[PREP_BLOCK];
    const int tid = threadIdx.x;
    const int64_t s = blockIdx.x * (int64_t)PREP_BLOCK + tid;
    const int64_t ns = A.L.ns, nn = A.L.nn;
    const bool live = s < ns;
    unsigned fl = 0;
    int64_t g1 = -1, g2 = -1;
    int inst = -1;
    if (live) {
        if (!seg_ends(A.L, A.seg_nodes, s, g1, g2)) fl |= FLAG_BAD_INDEX;
        inst = seg_instance(A.L, s);
    }
    sh_g1[tid] = g1;
    sh_g2[tid] = g2;
    sh_inst[tid] = inst;
    __syncthreads();
    // does the next segment of this workgroup start at the node where this one ends?
    sh_chain[tid] = live && tid + 1 < PREP_BLOCK && sh_inst[tid + 1] == inst && sh_g1[tid + 1] == g2;
    __syncthreads();
    if (!live) return;
    double rr[13];
    const double L = seg_record(A.x, nn, g1, g2, A.burgers, ns, s, A.inv_a, rr);
    if (!(L > 0.0) || !isfinite(L)) fl |= FLAG_ZERO_LENGTH;
    const double x1[3] = {rr[0], rr[1], rr[2]}, t[3] = {rr[3], rr[4], rr[5]};
    const double b[3] = {rr[7], rr[8], rr[9]}, c[3] = {rr[10], rr[11], rr[12]};
    double nv[3] = {A.normal[s], A.normal[ns + s], A.normal[2 * ns + s]};
    double nl = nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2];
    if (!(fabs(nl - 1.0) <= 2e-6)) fl |= FLAG_BAD_NORMAL;
    double *r = A.rec64;
    r[0 * ns + s] = x1[0]; r[1 * ns + s] = x1[1]; r[2 * ns + s] = x1[2];
    r[3 * ns + s] = t[0];  r[4 * ns + s] = t[1];  r[5 * ns + s] = t[2];
    r[6 * ns + s] = L;
    r[7 * ns + s] = b[0];  r[8 * ns + s] = b[1];  r[9 * ns + s] = b[2];
    r[10 * ns + s] = c[0]; r[11 * ns + s] = c[1]; r[12 * ns + s] = c[2];
    // length of the run of segments starting here in which each next segment
    // starts at the node where the one before it ends (loops stored in order),
    // within this workgroup's segments: the all-pairs kernel computes the
    // inverse distance to a shared node once per run
    int run = 1;
    while (tid + run < PREP_BLOCK && sh_chain[tid + run - 1]) ++run;
    r[13 * ns + s] = (double)run;
    {
        double *ra = r + (int64_t)REC64 * ns + s * RECA;
        ra[0] = x1[0]; ra[1] = x1[1]; ra[2] = x1[2];
        ra[3] = t[0];  ra[4] = t[1];  ra[5] = t[2];
        ra[6] = L;
        ra[7] = b[0];  ra[8] = b[1];  ra[9] = b[2];
        ra[10] = c[0]; ra[11] = c[1]; ra[12] = c[2];
        ra[13] = __longlong_as_double((long long)run);
        ra[14] = 0.0;  ra[15] = 0.0;
    }
    if (A.rec32) {
        float *q = A.rec32 + s * REC32A;
        // source quadrature of the variant: Gauss-Legendre points on the source
        double hq = 0.0, wo = 1.0, wc = 0.0, band = 0.0;
        if (A.quadn == 2) {
            hq = L * 0.28867513459481288225;            // L / (2 sqrt 3)
            wo = 0.5 * L;
            band = fmax(30.0 * L, (double)A.cut + 0.5 * L);
        } else if (A.quadn == 3) {
            hq = L * 0.38729833462074168852;            // (L / 2) sqrt(3/5)
            wo = L * (5.0 / 18.0);
            wc = L * (8.0 / 18.0);
            band = fmax(6.0 * L, (double)A.cut + 0.5 * L);
        }
        for (int k = 0; k < 3; ++k) {
            const double xm = x1[k] + 0.5 * L * t[k];
            q[R32_XH + k] = (float)xm;
            q[R32_XL + k] = (float)(xm - (double)q[k]);
            q[R32_T + k] = (float)t[k];
            q[R32_B + k] = (float)(wo * b[k]);
            q[R32_C + k] = (float)(wo * c[k]);
        }
        q[R32_L] = (float)L;
        q[R32_HQ] = (float)hq;
        q[R32_BAND] = (float)(band * band);
        q[R32_IW] = (float)(1.0 / wo);
        q[R32_RA0] = (float)(1.0 + hq * hq);
        q[R32_TW] = (float)(2.0 * hq);
        q[R32_WC] = (float)(wc / wo);
        q[22] = 0.f; q[23] = 0.f;
    }
    if (A.sys) A.sys[s] = seg_system(b, nv);
    if (fl) atomicOr(A.flags, fl);
}

// ------------------------------------------- node -> (segment, end) lists --
__global__ void k_csr_count(Layout L, const int32_t *seg_nodes, int32_t *cnt)
{
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= L.ns) return;
    int64_t g1, g2;
    if (!seg_ends(L, seg_nodes, s, g1, g2)) return;   // bad segment: attached to nothing
    atomicAdd(&cnt[g1], 1);
    atomicAdd(&cnt[g2], 1);
}


__global__ void k_csr_fill(Layout L, const int32_t *seg_nodes, const int32_t *ptr,
                           int32_t *cursor, int32_t *list)
{
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= L.ns) return;
    int64_t g[2];
    if (!seg_ends(L, seg_nodes, s, g[0], g[1])) return;
    for (int e = 0; e < 2; ++e) {
        // counts down from the node's count: slots ptr .. ptr + count - 1
        const int32_t k = atomicSub(&cursor[g[e]], 1) - 1;
        list[ptr[g[e]] + k] = (int32_t)(2 * s + e);
    }
}

// Sort each node's list by (segment, end) so that every later gather sums in
// a fixed order (results do not depend on the atomics above).
__global__ void k_csr_sort(const int32_t *ptr, int64_t nn, int32_t *list)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nn) return;
    int32_t b = ptr[n], e = ptr[n + 1];
    for (int32_t i = b + 1; i < e; ++i) {
        int32_t v = list[i], k = i - 1;
        while (k >= b && list[k] > v) {
            list[k + 1] = list[k];
            --k;
        }
        list[k + 1] = v;
    }
}

// ------------------------------ a3 + a4: Peach-Koehler and the quadrature --
struct Sig6 { double v[6]; };

__global__ void k_segment_ends(Layout L, const Tile *__restrict__ tiles,
                               const double *__restrict__ partial,
                               const double *__restrict__ rec, GaussRule g,
                               const double *__restrict__ sig_dev, Sig6 sig_val,
                               double inv_mu, double fscale, double *__restrict__ segF,
                               const int64_t *__restrict__ near_ptr, const int32_t *__restrict__ near_cnt,
                               const double *__restrict__ near_corr, int64_t pair_cap)
{
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t ns = L.ns;
    if (j >= ns) return;
    const int inst = seg_instance(L, j);
    const int Q = g.n;
    const int64_t lp0 = (j - seg_begin(L, inst)) * Q;
    const int64_t tb = L.tile_begin ? L.tile_begin[inst] : 0;
    double S[6];
    for (int k = 0; k < 6; ++k) S[k] = (sig_dev ? sig_dev[6 * inst + k] : sig_val.v[k]) * inv_mu;
    const double t0 = rec[3 * ns + j], t1 = rec[4 * ns + j], t2 = rec[5 * ns + j];
    const double Ls = rec[6 * ns + j];
    const double b0 = rec[7 * ns + j], b1 = rec[8 * ns + j], b2 = rec[9 * ns + j];
    // applied part: sigma_app b (Voigt xx yy zz yz xz xy)
    const double ab0 = S[0] * b0 + S[5] * b1 + S[4] * b2;
    const double ab1 = S[5] * b0 + S[1] * b1 + S[3] * b2;
    const double ab2 = S[4] * b0 + S[3] * b1 + S[2] * b2;
    double F1[3] = {0, 0, 0}, F2[3] = {0, 0, 0};
    // an instance left out of the work plan (idle in this pass) has no tiles
    const bool has_tiles = !L.tile_begin || L.tile_begin[inst + 1] > tb;
    for (int q = 0; q < Q; ++q) {
        const int64_t lp = lp0 + q;
        const Tile T = has_tiles ? tiles[tb + lp / TILE] : Tile{0, 0, 0, 0};
        const int lane = (int)(lp % TILE);
        double s0 = 0, s1 = 0, s2 = 0;
        for (int c = 0; c < T.n_chunks; ++c) {
            const double *o = partial + (T.slot_begin + c) * 3 * TILE;
            s0 += o[lane];
            s1 += o[TILE + lane];
            s2 += o[2 * TILE + lane];
        }
        s0 += ab0;
        s1 += ab1;
        s2 += ab2;
        // f = (sigma b) x t
        const double f0 = s1 * t2 - s2 * t1;
        const double f1 = s2 * t0 - s0 * t2;
        const double f2 = s0 * t1 - s1 * t0;
        const double w1 = Ls * g.w[q] * (1.0 - g.s[q]), w2 = Ls * g.w[q] * g.s[q];
        F1[0] += w1 * f0; F1[1] += w1 * f1; F1[2] += w1 * f2;
        F2[0] += w2 * f0; F2[1] += w2 * f1; F2[2] += w2 * f2;
    }
    // exact band: (exact - Q-point) for this target's near sources, in source order
    if (near_ptr) {
        const int64_t p0 = near_ptr[j];
        const int nc = near_cnt[j];
        for (int k = 0; k < nc && p0 + k < pair_cap; ++k) {
            const double *o = near_corr + 6 * (p0 + k);
            F1[0] += o[0]; F1[1] += o[1]; F1[2] += o[2];
            F2[0] += o[3]; F2[1] += o[4]; F2[2] += o[5];
        }
    }
    for (int k = 0; k < 3; ++k) {
        segF[k * ns + j] = F1[k] * fscale;
        segF[(3 + k) * ns + j] = F2[k] * fscale;
    }
}

// F_n = sum over the node's (segment, end) list in sorted order.
__global__ void k_node_gather(const int32_t *__restrict__ ptr, const int32_t *__restrict__ list,
                              int64_t nn, int64_t ns, const double *__restrict__ segF,
                              double *__restrict__ F)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nn) return;
    double f0 = 0, f1 = 0, f2 = 0;
    for (int32_t k = ptr[n]; k < ptr[n + 1]; ++k) {
        const int32_t e = list[k];
        const int64_t s = e >> 1;
        const int end = e & 1;
        f0 += segF[(3 * end + 0) * ns + s];
        f1 += segF[(3 * end + 1) * ns + s];
        f2 += segF[(3 * end + 2) * ns + s];
    }
    F[n] = f0;
    F[nn + n] = f1;
    F[2 * nn + n] = f2;
}

// ---------------------------------------------- a5 + a6: glide and Euler --
// Collects the distinct slip-plane normals (up to sign) of a node's
// segments: the first three in nrm, their number in cnt.
__device__ __forceinline__ void add_normal(double ns0, double ns1, double ns2, double (&nrm)[3][3], int &cnt)
{
    bool dup = false;
    for (int c = 0; c < 3; ++c)
        if (c < cnt && fabs(nrm[c][0] * ns0 + nrm[c][1] * ns1 + nrm[c][2] * ns2) > 1.0 - 1e-12) dup = true;
    if (!dup) {
        if (cnt < 3) {
            nrm[cnt][0] = ns0; nrm[cnt][1] = ns1; nrm[cnt][2] = ns2;
        }
        ++cnt;
    }
}

// Glide velocity v = P F / (B ell) of a free node with cnt distinct normals:
// one normal -> its component removed; two -> projected on their
// intersection line (cnt >= 3 and fixed nodes are handled by the caller).
__device__ __forceinline__ void glide_velocity(double F0, double F1, double F2, double ell, double invB,
                                               const double (&nrm)[3][3], int cnt, double &v0, double &v1,
                                               double &v2)
{
    const double sc = invB / ell;
    v0 = F0 * sc;
    v1 = F1 * sc;
    v2 = F2 * sc;
    if (cnt == 1) {
        const double vn = v0 * nrm[0][0] + v1 * nrm[0][1] + v2 * nrm[0][2];
        v0 -= vn * nrm[0][0];
        v1 -= vn * nrm[0][1];
        v2 -= vn * nrm[0][2];
    } else {
        double l0 = nrm[0][1] * nrm[1][2] - nrm[0][2] * nrm[1][1];
        double l1 = nrm[0][2] * nrm[1][0] - nrm[0][0] * nrm[1][2];
        double l2 = nrm[0][0] * nrm[1][1] - nrm[0][1] * nrm[1][0];
        const double il = 1.0 / sqrt(l0 * l0 + l1 * l1 + l2 * l2);
        l0 *= il; l1 *= il; l2 *= il;
        const double vl = v0 * l0 + v1 * l1 + v2 * l2;
        v0 = vl * l0; v1 = vl * l1; v2 = vl * l2;
    }
}

// Per node: ell = 1/2 sum L_s over attached segments, v = P F / (B ell), with
// P from the distinct slip-plane normals among them.  FROM_REC: lengths from
// the segment records (x unchanged since they were made), so the node can be
// advanced in the same pass; otherwise lengths come from x and the Euler
// update is a separate kernel.
template <bool FROM_REC>
__global__ void k_glide(Layout L, const int32_t *__restrict__ ptr, const int32_t *__restrict__ list,
                        const int32_t *__restrict__ seg_nodes, const double *__restrict__ normal,
                        const double *__restrict__ rec, double a, double *x,
                        const double *__restrict__ F, const uint8_t *__restrict__ pinned,
                        const uint8_t *__restrict__ held, const uint8_t *__restrict__ active, double invB,
                        double dt, double *__restrict__ vel)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nn = L.nn, ns = L.ns;
    if (n >= nn) return;
    // nodes of an idle instance (active[instance] == 0) do not move
    const bool idle = active && ptr[n + 1] > ptr[n] && !active[seg_instance(L, list[ptr[n]] >> 1)];
    double ell = 0.0;
    double nrm[3][3];
    int cnt = 0;
    for (int32_t k = ptr[n]; k < ptr[n + 1]; ++k) {
        const int64_t s = list[k] >> 1;
        double Ls;
        if (FROM_REC) {
            Ls = rec[6 * ns + s] * a;
        } else {
            int64_t g1, g2;
            seg_ends(L, seg_nodes, s, g1, g2);
            double d0 = x[g2] - x[g1], d1 = x[nn + g2] - x[nn + g1], d2 = x[2 * nn + g2] - x[2 * nn + g1];
            Ls = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        }
        ell += 0.5 * Ls;
        add_normal(normal[s], normal[ns + s], normal[2 * ns + s], nrm, cnt);
    }
    double v0 = 0, v1 = 0, v2 = 0;
    const bool fixed = idle || (pinned && pinned[n]) || (held && held[n]) || !(ell > 0.0) || cnt == 0 || cnt >= 3;
    if (!fixed) glide_velocity(F[n], F[nn + n], F[2 * nn + n], ell, invB, nrm, cnt, v0, v1, v2);
    if (vel) {
        vel[n] = v0;
        vel[nn + n] = v1;
        vel[2 * nn + n] = v2;
    }
    if (FROM_REC) {
        x[n] += v0 * dt;
        x[nn + n] += v1 * dt;
        x[2 * nn + n] += v2 * dt;
    }
}

// ----------------------------------- junctions and thermal activation --
// Squared distance from p to the segment a -> b, written out without fused
// multiply-adds (the capture decision must match the oracle's bit for bit).
__device__ __forceinline__ double point_segment_d2(const double *p, const double *a, const double *b)
{
#pragma clang fp contract(off)
    const double d0 = b[0] - a[0], d1 = b[1] - a[1], d2 = b[2] - a[2];
    const double w0 = p[0] - a[0], w1 = p[1] - a[1], w2 = p[2] - a[2];
    const double dd = d0 * d0 + d1 * d1 + d2 * d2;
    double t = (w0 * d0 + w1 * d1 + w2 * d2) / dd;
    t = fmin(fmax(t, 0.0), 1.0);
    const double e0 = p[0] - (a[0] + t * d0);
    const double e1 = p[1] - (a[1] + t * d1);
    const double e2 = p[2] - (a[2] + t * d2);
    return e0 * e0 + e1 * e1 + e2 * e2;
}

__device__ __forceinline__ double release_time(double t, double f, double a)
{
#pragma clang fp contract(off)
    return t + f * a;
}

struct JunctionArgs {
    double rc2, rf2, a;      // capture radius^2, (2 capture radius)^2, maximum breaking time
    double tk;               // this step's offset k dt from the call's start time
    const double *t0;        // the call's start time (device, written before the step graph runs)
    double rc;               // capture radius
    int32_t K;
    const double *fractions;
    int32_t *junction, *ignore, *count;
    double *release;
    // sessile segments in index order: position in the list of segment s
    // (valid where s is sessile; pos[seg_off[i]] .. pos[seg_off[i + 1]] are
    // instance i's), their indices, end points (their nodes never move) and
    // bounding spheres of each (midpoint, half length) and of JUNC_GROUP
    // consecutive entries
    const int32_t *pos, *ses_idx;
    const double *ses_x, *ses_ssp, *ses_sph, *ses_sup;
};
constexpr int JUNC_GROUP = 8;
constexpr int JUNC_SUPER = 8;   // groups per second-level sphere (64 list entries)

// Bounding spheres of the compact sessile list (centre, radius each): per
// entry, per JUNC_GROUP entries and per JUNC_SUPER groups.
struct JunctionSpheres {
    const double *ssp, *sph, *sup;
};

// Sessile segments (both nodes pinned): flags for the scan.
__global__ void k_ses_flag(Layout L, const int32_t *__restrict__ seg_nodes, const uint8_t *__restrict__ pinned,
                           int32_t *__restrict__ flag)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= L.ns) return;
    int64_t g1, g2;
    seg_ends(L, seg_nodes, s, g1, g2);
    flag[s] = pinned && pinned[g1] && pinned[g2] ? 1 : 0;
}

// The compact list of sessile segments and their end points.
__global__ void k_ses_compact(Layout L, const int32_t *__restrict__ seg_nodes, const double *__restrict__ x,
                              const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                              int32_t *__restrict__ idx, double *__restrict__ sx, double *__restrict__ ssp)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= L.ns || !flag[s]) return;
    int64_t g1, g2;
    seg_ends(L, seg_nodes, s, g1, g2);
    const int64_t q = pos[s], nn = L.nn;
    idx[q] = (int32_t)s;
    double *o = sx + 6 * q;
    o[0] = x[g1]; o[1] = x[nn + g1]; o[2] = x[2 * nn + g1];
    o[3] = x[g2]; o[4] = x[nn + g2]; o[5] = x[2 * nn + g2];
    // the segment's own sphere: a point closer than r to it is closer than
    // L/2 + r to its midpoint
    const double d0 = o[3] - o[0], d1 = o[4] - o[1], d2 = o[5] - o[2];
    double *m = ssp + 4 * q;
    m[0] = 0.5 * (o[0] + o[3]); m[1] = 0.5 * (o[1] + o[4]); m[2] = 0.5 * (o[2] + o[5]);
    m[3] = 0.5 * sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

// Bounding sphere of JUNC_GROUP consecutive entries of the list: centre = the
// first segment's midpoint, radius = max |m_i - C| + L_i / 2, so that a point
// closer than r to any of them is closer than R + r to C.
__global__ void k_ses_spheres(int64_t ns, const int32_t *__restrict__ pos, const double *__restrict__ sx,
                              double *__restrict__ sph)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n_ses = pos[ns];
    const int64_t q0 = g * JUNC_GROUP;
    if (q0 >= n_ses) return;
    const int64_t q1 = q0 + JUNC_GROUP < n_ses ? q0 + JUNC_GROUP : n_ses;
    const double *f = sx + 6 * q0;
    const double c0 = 0.5 * (f[0] + f[3]), c1 = 0.5 * (f[1] + f[4]), c2 = 0.5 * (f[2] + f[5]);
    double r = 0.0;
    for (int64_t q = q0; q < q1; ++q) {
        const double *e = sx + 6 * q;
        const double m0 = 0.5 * (e[0] + e[3]) - c0, m1 = 0.5 * (e[1] + e[4]) - c1, m2 = 0.5 * (e[2] + e[5]) - c2;
        const double d0 = e[3] - e[0], d1 = e[4] - e[1], d2 = e[5] - e[2];
        r = fmax(r, sqrt(m0 * m0 + m1 * m1 + m2 * m2) + 0.5 * sqrt(d0 * d0 + d1 * d1 + d2 * d2));
    }
    double *o = sph + 4 * g;
    o[0] = c0; o[1] = c1; o[2] = c2; o[3] = r;
}

// Bounding sphere of JUNC_SUPER consecutive group spheres (centre = the
// first one's), so that the searches skip 64 list entries with one test.
__global__ void k_ses_super(int64_t ns, const int32_t *__restrict__ pos, const double *__restrict__ sph,
                            double *__restrict__ sup)
{
    const int64_t G = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n_grp = (pos[ns] + JUNC_GROUP - 1) / JUNC_GROUP;
    const int64_t g0 = G * JUNC_SUPER;
    if (g0 >= n_grp) return;
    const int64_t g1 = g0 + JUNC_SUPER < n_grp ? g0 + JUNC_SUPER : n_grp;
    const double *f = sph + 4 * g0;
    const double c0 = f[0], c1 = f[1], c2 = f[2];
    double r = 0.0;
    for (int64_t g = g0; g < g1; ++g) {
        const double *e = sph + 4 * g;
        const double m0 = e[0] - c0, m1 = e[1] - c1, m2 = e[2] - c2;
        r = fmax(r, sqrt(m0 * m0 + m1 * m1 + m2 * m2) + e[3]);
    }
    double *o = sup + 4 * G;
    o[0] = c0; o[1] = c1; o[2] = c2; o[3] = r;
}

// Search of the sessile list entries [q_lo, q_hi) in index order for the
// first one that test(q) accepts, skipping second-level and group spheres
// (centre c, radius r) with |m - c| >= r + reach (m: the searcher's centre).
// Returns the entry or -1.  When every active lane of the wavefront searches
// the same range, the bounds are taken wave-uniform, so that the sphere
// loads are the same address across the wavefront (scalar loads, one per
// wavefront instead of one per lane).
template <class Test>
__device__ __forceinline__ int64_t sessile_search(const JunctionSpheres &S, int64_t q_lo, int64_t q_hi,
                                                  const double m[3], double reach, Test &&test)
{
    // sphere j of 8 consecutive ones starting at base (indices clamped to
    // last, so that every load stays inside the list) tested at once: the
    // loads are issued together, one wait for all eight
    auto hits8 = [&](const double *sp, int64_t base, int64_t first, int64_t last) -> unsigned {
        double c[8][4];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t i = base + j < last ? base + j : last;
#pragma unroll
            for (int d = 0; d < 4; ++d) c[j][d] = sp[4 * i + d];
        }
        unsigned mask = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double e0 = m[0] - c[j][0], e1 = m[1] - c[j][1], e2 = m[2] - c[j][2];
            const double rr = (c[j][3] + reach) * (1.0 + 1e-9);
            if (base + j >= first && base + j <= last && e0 * e0 + e1 * e1 + e2 * e2 < rr * rr) mask |= 1u << j;
        }
        return mask;
    };
    auto run = [&](const int64_t qa0, const int64_t qb0) -> int64_t {
        if (qa0 >= qb0) return -1;
        const int64_t g_lo = qa0 / JUNC_GROUP, g_hi = (qb0 + JUNC_GROUP - 1) / JUNC_GROUP;
        const int64_t G_lo = g_lo / JUNC_SUPER, G_hi = (g_hi + JUNC_SUPER - 1) / JUNC_SUPER;
        for (int64_t G0 = G_lo; G0 < G_hi; G0 += 8) {
            for (unsigned mG = hits8(S.sup, G0, G_lo, G_hi - 1); mG; mG &= mG - 1) {
                const int64_t G = G0 + __builtin_ctz(mG);
                for (unsigned mg = hits8(S.sph, G * JUNC_SUPER, g_lo, g_hi - 1); mg; mg &= mg - 1) {
                    const int64_t g = G * JUNC_SUPER + __builtin_ctz(mg);
                    const int64_t qa = g * JUNC_GROUP > qa0 ? g * JUNC_GROUP : qa0;
                    const int64_t qb = (g + 1) * JUNC_GROUP < qb0 ? (g + 1) * JUNC_GROUP : qb0;
                    for (unsigned mq = hits8(S.ssp, g * JUNC_GROUP, qa, qb - 1); mq; mq &= mq - 1) {
                        const int64_t q = g * JUNC_GROUP + __builtin_ctz(mq);
                        if (test(q)) return q;
                    }
                }
            }
        }
        return -1;
    };
    const int32_t lo0 = __builtin_amdgcn_readfirstlane((int32_t)q_lo);
    const int32_t hi0 = __builtin_amdgcn_readfirstlane((int32_t)q_hi);
    if (__builtin_amdgcn_ballot_w64(q_lo == lo0 && q_hi == hi0) == __builtin_amdgcn_read_exec())
        return run(lo0, hi0);
    return run(q_lo, q_hi);
}

// Junction checks at the start of a step (Sec. "Thermal activation", Eq. tb),
// one thread per node: a held node is released once t reaches its release
// time; a free mobile node forgets the segment it last broke from beyond
// 2 r_c, then is captured by the first sessile segment of its instance (both
// nodes pinned), in index order and other than that one, closer than r_c,
// with release = t + f a, f = fractions[n][count mod K].  held[n] = 1 for the
// nodes the glide step must keep fixed.  The sessile segments come from the
// compact list; groups, and then segments, whose bounding sphere is out of
// reach are skipped before the exact distance (a division) is formed, which
// leaves the index order of the tests unchanged.
__global__ __launch_bounds__(256) void k_junctions(Layout L, const int32_t *__restrict__ seg_nodes, const double *__restrict__ x,
                            const uint8_t *__restrict__ pinned, JunctionArgs J, int n_inst,
                            const uint8_t *__restrict__ active, const int64_t *__restrict__ fast_steps, double dt,
                            int k, uint8_t *__restrict__ held)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nn = L.nn;
    if (n >= nn) return;
    if (!pinned || pinned[n]) {
        held[n] = 0;
        return;
    }
    // the node's instance: last i with node_off[i] <= n
    int lo = 0, hi = n_inst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L.node_off[mid] <= n) lo = mid; else hi = mid;
    }
    // an instance left out of this pass keeps its state (and does not move)
    if (active && !active[lo]) {
        held[n] = 0;
        return;
    }
    // time: the instance's fast clock (steps taken so far times dt), or the call's
    const double t = fast_steps ? (double)(fast_steps[lo] + k) * dt : *J.t0 + J.tk;
    const int32_t js = J.junction[n];
    if (js >= 0) {
        if (t >= J.release[n]) {
            J.ignore[n] = js;
            J.junction[n] = -1;
            held[n] = 0;
        } else {
            held[n] = 1;
        }
        return;
    }
    const int64_t sb = L.seg_off[lo], se = L.seg_off[lo + 1];
    const double p[3] = {x[n], x[nn + n], x[2 * nn + n]};
    int64_t ig = J.ignore[n];
    if (ig >= sb && ig < se) {
        int64_t g1, g2;
        seg_ends(L, seg_nodes, ig, g1, g2);
        const double a[3] = {x[g1], x[nn + g1], x[2 * nn + g1]}, b[3] = {x[g2], x[nn + g2], x[2 * nn + g2]};
        if (point_segment_d2(p, a, b) > J.rf2) {
            ig = -1;
            J.ignore[n] = -1;
        }
    } else {
        ig = -1;
    }
    // the instance's sessile segments, in index order, sphere by sphere
    const JunctionSpheres S{J.ses_ssp, J.ses_sph, J.ses_sup};
    const int64_t qf = sessile_search(S, J.pos[sb], J.pos[se], p, J.rc, [&](const int64_t q) {
        if (J.ses_idx[q] == ig) return false;
        const double *e = J.ses_x + 6 * q;
        return point_segment_d2(p, e, e + 3) < J.rc2;
    });
    if (qf >= 0) {
        const int32_t cn = J.count[n];
        const int32_t kf = ((cn % J.K) + J.K) % J.K;
        J.junction[n] = J.ses_idx[qf];
        J.release[n] = release_time(t, J.fractions[n * J.K + kf], J.a);
        J.count[n] = cn + 1;
        held[n] = 1;
        return;
    }
    held[n] = 0;
}

// Junction arguments from the caller's parameters, and the compact list of
// sessile segments (flags, scan, compaction, spheres) for positions x; held
// receives the per-node hold mask each step.
int junction_prepare(Workspace *ws, const Layout &L, const int32_t *seg_nodes, const double *x,
                     const uint8_t *pinned, const dd_junctions *jn, JunctionArgs &J, uint8_t **held,
                     hipStream_t st)
{
    const int64_t nn = L.nn, ns = L.ns;
    void *p;
    int rc;
    if ((rc = ensure(ws, WS_HELD, std::max<int64_t>(nn, 1), &p))) return rc;
    *held = (uint8_t *)p;
    J = JunctionArgs{};
    J.rc2 = jn->capture_radius * jn->capture_radius;
    J.rf2 = (2.0 * jn->capture_radius) * (2.0 * jn->capture_radius);
    J.a = jn->max_break_time;
    J.K = jn->n_fractions;
    J.fractions = jn->fractions;
    J.junction = jn->junction;
    J.ignore = jn->ignore;
    J.count = jn->count;
    J.release = jn->release;
    J.rc = jn->capture_radius;
    if ((rc = ensure(ws, WS_SES, sizeof(int32_t) * (3 * ns + 1 + scan_scratch_len(ns)), &p))) return rc;
    int32_t *flag = (int32_t *)p, *pos = flag + ns, *idx = pos + ns + 1, *scan_tmp = idx + ns;
    const int64_t n_grp = (ns + JUNC_GROUP - 1) / JUNC_GROUP, n_sup = (n_grp + JUNC_SUPER - 1) / JUNC_SUPER;
    if ((rc = ensure(ws, WS_SES_X, sizeof(double) * (10 * ns + 4 * n_grp + 4 * n_sup + 8), &p))) return rc;
    double *sx = (double *)p, *ssp = sx + 6 * ns, *sph = ssp + 4 * ns, *sup = sph + 4 * n_grp + 4;
    const unsigned gs = grid_for(ns, 256, INT32_MAX);
    hipLaunchKernelGGL(k_ses_flag, dim3(gs), dim3(256), 0, st, L, seg_nodes, pinned, flag);
    launch_scan<int32_t>(flag, ns, pos, scan_tmp, st);
    hipLaunchKernelGGL(k_ses_compact, dim3(gs), dim3(256), 0, st, L, seg_nodes, x, (const int32_t *)flag,
                       (const int32_t *)pos, idx, sx, ssp);
    hipLaunchKernelGGL(k_ses_spheres, dim3(grid_for(n_grp, 256, INT32_MAX)), dim3(256), 0, st, ns,
                       (const int32_t *)pos, (const double *)sx, sph);
    hipLaunchKernelGGL(k_ses_super, dim3(grid_for(n_sup, 256, INT32_MAX)), dim3(256), 0, st, ns,
                       (const int32_t *)pos, (const double *)sph, sup);
    J.pos = pos;
    J.ses_idx = idx;
    J.ses_x = sx;
    J.ses_ssp = ssp;
    J.ses_sph = sph;
    J.ses_sup = sup;
    return DD_OK;
}

// ---------------------------------------------------------- junction nodes --
// Junction nodes (Sec. "Thermal activation", Eq. tb): a mobile segment that
// comes closer than the capture radius to a sessile segment of its instance
// is split at its point of closest approach by a pinned node taken from the
// instance's node slots, with the out-half in a segment slot; the node is
// removed when its junction breaks (the rules and the slot layout are those
// of dd_junction_nodes in dd.h).  Decisions and the junction point are formed
// in FP64 without fused multiply-adds, in the same order of operations as the
// oracle, so that both take the same decisions.

// Closest approach of the segments p -> p2 and q -> q2: the squared distance,
// and in u the parameter of the closest point on the first.  The unclamped
// parameter on the first line is (b f - c e) / (a e - b^2) (a = d1.d1,
// b = d1.d2, c = d1.r, e = d2.d2, f = d2.r, r = p - q), clamped to [0, 1];
// the second parameter v = (b u + f) / e follows, and when v leaves [0, 1]
// it is clamped and u recomputed for that end of the second segment.
__device__ __forceinline__ double seg_seg_closest(const double *p, const double *p2, const double *q,
                                                  const double *q2, double &u_out)
{
#pragma clang fp contract(off)
    const double d10 = p2[0] - p[0], d11 = p2[1] - p[1], d12 = p2[2] - p[2];
    const double d20 = q2[0] - q[0], d21 = q2[1] - q[1], d22 = q2[2] - q[2];
    const double r0 = p[0] - q[0], r1 = p[1] - q[1], r2 = p[2] - q[2];
    const double a = d10 * d10 + d11 * d11 + d12 * d12;
    const double e = d20 * d20 + d21 * d21 + d22 * d22;
    const double f = d20 * r0 + d21 * r1 + d22 * r2;
    const double c = d10 * r0 + d11 * r1 + d12 * r2;
    const double b = d10 * d20 + d11 * d21 + d12 * d22;
    const double den = a * e - b * b;
    double u = den > 0.0 ? fmin(fmax((b * f - c * e) / den, 0.0), 1.0) : 0.0;
    double v = (b * u + f) / e;
    if (v < 0.0) {
        v = 0.0;
        u = fmin(fmax(-c / a, 0.0), 1.0);
    } else if (v > 1.0) {
        v = 1.0;
        u = fmin(fmax((b - c) / a, 0.0), 1.0);
    }
    const double w0 = (p[0] + u * d10) - (q[0] + v * d20);
    const double w1 = (p[1] + u * d11) - (q[1] + v * d21);
    const double w2 = (p[2] + u * d12) - (q[2] + v * d22);
    u_out = u;
    return w0 * w0 + w1 * w1 + w2 * w2;
}

struct JNodeArgs {
    double rc, rc2, rf2, a, lmin;      // capture radius, its square, (2 r_c)^2, max breaking time, l_min
    double tk;                         // this step's offset k dt from the call's start time
    const double *t0;                  // the call's start time (device, written before the step graph runs)
    const int64_t *fast;               // or per instance the fast steps taken so far (PTA), null: t0 + tk
    double fdt;                        //   the fast step dt
    int fk;                            //   and this step's index in the run
    int32_t K, Kf;                     // slots per instance, fractions per instance
    const double *fractions;           // [n_inst][Kf]
    double *release;                   // [nn]
    int32_t *ses;                      // [nn] batch index of the sessile segment, -1: free slot
    int32_t *ignore;                   // [ns] 1 while the segment keeps the point of its last junction
    double *point;                     // [3][ns] that point
    int32_t *count, *missed;           // [n_inst]
    const int32_t *flag;               // [ns] sessile
    const int32_t *pos, *ses_idx;      // the compact sessile list (as for JunctionArgs)
    const double *ses_x, *ses_ssp, *ses_sph, *ses_sup;
    int32_t *cand;                     // [ns] sessile candidate of a segment, -1: none
    double *cand_u;                    // [ns] its parameter on the segment
};

// Time of a topology step of instance inst: its fast clock, (fast steps
// taken so far + this step's index) dt, when the caller keeps one (the PTA
// driver), else the call's start time plus k dt (both as the oracle forms
// them).
__device__ __forceinline__ double jn_time(const JNodeArgs &J, int inst)
{
    return J.fast ? (double)(J.fast[inst] + J.fk) * J.fdt : *J.t0 + J.tk;
}

// Sessile segments for junction nodes: an instance's own segment (not a
// segment slot) between two of its own nodes (not node slots or dummies),
// both pinned.
__global__ void k_jn_ses_flag(Layout L, const int32_t *__restrict__ seg_nodes, const uint8_t *__restrict__ pinned,
                              int32_t K, int32_t *__restrict__ flag)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= L.ns) return;
    const int inst = seg_instance(L, s);
    const int64_t sl = s - L.seg_off[inst], n_s = L.seg_off[inst + 1] - L.seg_off[inst];
    const int64_t n_n = node_count(L, inst);
    int64_t g1, g2;
    const bool ok = seg_ends(L, seg_nodes, s, g1, g2);
    const int64_t a = seg_nodes[s], b = seg_nodes[L.ns + s];
    flag[s] = ok && sl < n_s - K && a < n_n - K - 2 && b < n_n - K - 2 && pinned[g1] && pinned[g2] ? 1 : 0;
}

// Releases (one workgroup per instance): node slots in index order whose
// junction has broken at time t are removed; the node's in-segment takes the
// end node of its out-segment, which becomes a free segment slot (D1 -> D2,
// Burgers vector 0); the merged segment keeps the junction point.
__global__ __launch_bounds__(256) void k_jn_release(Layout L, int32_t *__restrict__ seg_nodes,
                                                    const double *__restrict__ x, double *__restrict__ burgers,
                                                    double *__restrict__ normal, JNodeArgs J,
                                                    const uint8_t *__restrict__ active, uint32_t *__restrict__ flags)
{
    const int inst = blockIdx.x, tid = threadIdx.x;
    if (active && !active[inst]) return;
    const int64_t n0 = L.node_off[inst], n_n = L.node_off[inst + 1] - n0;
    const int64_t s0 = L.seg_off[inst], n_s = L.seg_off[inst + 1] - s0, ns = L.ns;
    if (n_n < J.K + 2 || n_s < J.K) return;
    const int32_t d1 = (int32_t)(n_n - 2), d2 = (int32_t)(n_n - 1);
    const double t = jn_time(J, inst);
    __shared__ int64_t s_in, s_out;
    for (int64_t jl = n_n - J.K - 2; jl < n_n - 2; ++jl) {
        const int64_t j = n0 + jl;
        if (!(J.ses[j] >= 0 && t >= J.release[j])) continue;   // the same for every thread
        if (tid == 0) {
            s_in = -1;
            s_out = -1;
        }
        __syncthreads();
        for (int64_t q = tid; q < n_s; q += blockDim.x) {
            if (seg_nodes[ns + s0 + q] == jl) s_in = q;
            if (seg_nodes[s0 + q] == jl) s_out = q;
        }
        __syncthreads();
        if (tid == 0) {
            if (s_in >= 0 && s_out >= 0) {
                const int64_t a = s0 + s_in, b = s0 + s_out;
                seg_nodes[ns + a] = seg_nodes[ns + b];
                seg_nodes[b] = d1;
                seg_nodes[ns + b] = d2;
                for (int c = 0; c < 3; ++c) {
                    burgers[c * ns + b] = 0.0;
                    normal[c * ns + b] = c == 2 ? 1.0 : 0.0;
                }
                J.ignore[a] = 1;   // the merged segment keeps the junction point
                for (int c = 0; c < 3; ++c) J.point[c * ns + a] = x[c * L.nn + j];
                J.ignore[b] = 0;
            } else {
                atomicOr(flags, FLAG_BAD_INDEX);   // inconsistent slot state: the node is dropped
            }
            J.ses[j] = -1;
        }
        __syncthreads();
    }
}

// Candidates (one thread per segment): a mobile segment (not sessile, not a
// free slot) that keeps the point of its last junction forgets it once
// farther than 2 r_c from it and is no candidate before; then it takes the
// first sessile segment of its instance in index order closer than r_c.
// Groups and segments whose bounding spheres are out of reach
// (|m_s - m_k| >= h_s + h_k + r_c) are skipped, which leaves the order of the
// exact tests unchanged.
__global__ __launch_bounds__(256) void k_jn_candidates(Layout L, const int32_t *__restrict__ seg_nodes, const double *__restrict__ x,
                                JNodeArgs J, const uint8_t *__restrict__ active)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= L.ns) return;
    J.cand[s] = -1;
    const int inst = seg_instance(L, s);
    if (active && !active[inst]) return;
    const int64_t n_n = node_count(L, inst), nn = L.nn;
    int64_t g1, g2;
    if (!seg_ends(L, seg_nodes, s, g1, g2) || J.flag[s]) return;
    if (seg_nodes[s] == n_n - 2 && seg_nodes[L.ns + s] == n_n - 1) return;   // a free segment slot
    const double p[3] = {x[g1], x[nn + g1], x[2 * nn + g1]}, p2[3] = {x[g2], x[nn + g2], x[2 * nn + g2]};
    const int64_t sb = L.seg_off[inst], se = L.seg_off[inst + 1];
    if (J.ignore[s]) {
        const double pt[3] = {J.point[s], J.point[L.ns + s], J.point[2 * L.ns + s]};
        if (point_segment_d2(pt, p, p2) > J.rf2)
            J.ignore[s] = 0;
        else
            return;
    }
    const double m[3] = {0.5 * (p[0] + p2[0]), 0.5 * (p[1] + p2[1]), 0.5 * (p[2] + p2[2])};
    const double t0 = p2[0] - p[0], t1 = p2[1] - p[1], t2 = p2[2] - p[2];
    const double hs = 0.5 * sqrt(t0 * t0 + t1 * t1 + t2 * t2);
    const JunctionSpheres S{J.ses_ssp, J.ses_sph, J.ses_sup};
    double u = 0.0;
    const int64_t qf = sessile_search(S, J.pos[sb], J.pos[se], m, hs + J.rc, [&](const int64_t q) {
        const double *e = J.ses_x + 6 * q;
        return seg_seg_closest(p, p2, e, e + 3, u) < J.rc2;
    });
    if (qf >= 0) {
        J.cand[s] = J.ses_idx[qf];
        J.cand_u[s] = u;
    }
}

// Captures (one workgroup per instance), in segment index order: a candidate
// segment a -> b longer than 2 l_min gets a junction node j in the lowest
// free node slot at the clamped parameter u in [l_min / L, 1 - l_min / L],
// becomes a -> j, and the lowest free segment slot becomes j -> b with its
// Burgers vector and normal; both halves keep the junction point; the node
// is released at t + f a, f = fractions[instance][count mod Kf].  Without a
// free slot the capture is counted in missed.
__global__ __launch_bounds__(256) void k_jn_capture(Layout L, int32_t *__restrict__ seg_nodes, double *__restrict__ x,
                                                    double *__restrict__ burgers, double *__restrict__ normal,
                                                    JNodeArgs J, const uint8_t *__restrict__ active)
{
#pragma clang fp contract(off)
    const int inst = blockIdx.x, tid = threadIdx.x;
    if (active && !active[inst]) return;
    const int64_t n0 = L.node_off[inst], n_n = L.node_off[inst + 1] - n0;
    const int64_t s0 = L.seg_off[inst], n_s = L.seg_off[inst + 1] - s0, ns = L.ns, nn = L.nn;
    if (n_n < J.K + 2 || n_s < J.K) return;
    const int32_t d1 = (int32_t)(n_n - 2), d2 = (int32_t)(n_n - 1);
    __shared__ uint8_t has[256];
    for (int64_t base = 0; base < n_s; base += blockDim.x) {
        const int64_t q = base + tid;
        const bool c = q < n_s && J.cand[s0 + q] >= 0;
        has[tid] = c ? 1 : 0;
        if (__syncthreads_count(c) && tid == 0) {
            for (int i = 0; i < (int)blockDim.x && base + i < n_s; ++i) {
                if (!has[i]) continue;
                const int64_t s = s0 + base + i;
                const int32_t k = J.cand[s];
                const int64_t a = seg_nodes[s], b = seg_nodes[ns + s];
                if (a < 0 || a >= n_n || b < 0 || b >= n_n) continue;
                const int64_t ga = n0 + a, gb = n0 + b;
                const double e0 = x[gb] - x[ga], e1 = x[nn + gb] - x[nn + ga], e2 = x[2 * nn + gb] - x[2 * nn + ga];
                const double Ls = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
                if (!(Ls > 2.0 * J.lmin)) continue;
                const double u = fmin(fmax(J.cand_u[s], J.lmin / Ls), 1.0 - J.lmin / Ls);
                int64_t jl = -1, s2l = -1;
                for (int64_t r = n_n - J.K - 2; r < n_n - 2 && jl < 0; ++r)
                    if (J.ses[n0 + r] < 0) jl = r;
                for (int64_t r = n_s - J.K; r < n_s && s2l < 0; ++r)
                    if (seg_nodes[s0 + r] == d1 && seg_nodes[ns + s0 + r] == d2) s2l = r;
                if (jl < 0 || s2l < 0) {
                    J.missed[inst] += 1;
                    continue;
                }
                const int64_t j = n0 + jl, s2 = s0 + s2l;
                x[j] = x[ga] + u * e0;
                x[nn + j] = x[nn + ga] + u * e1;
                x[2 * nn + j] = x[2 * nn + ga] + u * e2;
                seg_nodes[ns + s] = (int32_t)jl;
                seg_nodes[s2] = (int32_t)jl;
                seg_nodes[ns + s2] = (int32_t)b;
                for (int cc = 0; cc < 3; ++cc) {
                    burgers[cc * ns + s2] = burgers[cc * ns + s];
                    normal[cc * ns + s2] = normal[cc * ns + s];
                }
                J.ignore[s] = 1;
                J.ignore[s2] = 1;
                for (int cc = 0; cc < 3; ++cc) J.point[cc * ns + s] = J.point[cc * ns + s2] = x[cc * nn + j];
                const int32_t cn = J.count[inst];
                const int32_t kf = ((cn % J.Kf) + J.Kf) % J.Kf;
                J.release[j] = release_time(jn_time(J, inst), J.fractions[(int64_t)inst * J.Kf + kf], J.a);
                J.ses[j] = k;
                J.count[inst] = cn + 1;
            }
        }
        __syncthreads();
    }
}

// Junction-node arguments from the caller's parameters, and the compact list
// of sessile segments (they never change: their nodes are pinned).
int jnode_prepare(Workspace *ws, const Layout &L, const int32_t *seg_nodes, const double *x, const uint8_t *pinned,
                  const dd_junction_nodes *jn, JNodeArgs &J, hipStream_t st)
{
    const int64_t ns = L.ns;
    void *p;
    int rc;
    J = JNodeArgs{};
    J.rc = jn->capture_radius;
    J.rc2 = jn->capture_radius * jn->capture_radius;
    J.rf2 = (2.0 * jn->capture_radius) * (2.0 * jn->capture_radius);
    J.a = jn->max_break_time;
    J.lmin = jn->min_length;
    J.K = jn->n_slots;
    J.Kf = jn->n_fractions;
    J.fractions = jn->fractions;
    J.release = jn->release;
    J.ses = jn->ses;
    J.ignore = jn->ignore;
    J.point = jn->point;
    J.count = jn->count;
    J.missed = jn->missed;
    if ((rc = ensure(ws, WS_SES, sizeof(int32_t) * (3 * ns + 1 + scan_scratch_len(ns)), &p))) return rc;
    int32_t *flag = (int32_t *)p, *pos = flag + ns, *idx = pos + ns + 1, *scan_tmp = idx + ns;
    const int64_t n_grp = (ns + JUNC_GROUP - 1) / JUNC_GROUP, n_sup = (n_grp + JUNC_SUPER - 1) / JUNC_SUPER;
    if ((rc = ensure(ws, WS_SES_X, sizeof(double) * (10 * ns + 4 * n_grp + 4 * n_sup + 8), &p))) return rc;
    double *sx = (double *)p, *ssp = sx + 6 * ns, *sph = ssp + 4 * ns, *sup = sph + 4 * n_grp + 4;
    if ((rc = ensure(ws, WS_JN_CAND, (sizeof(int32_t) + sizeof(double)) * std::max<int64_t>(ns, 1), &p))) return rc;
    J.cand_u = (double *)p;
    J.cand = (int32_t *)(J.cand_u + std::max<int64_t>(ns, 1));
    const unsigned gs = grid_for(ns, 256, INT32_MAX);
    hipLaunchKernelGGL(k_jn_ses_flag, dim3(gs), dim3(256), 0, st, L, seg_nodes, pinned, J.K, flag);
    launch_scan<int32_t>(flag, ns, pos, scan_tmp, st);
    hipLaunchKernelGGL(k_ses_compact, dim3(gs), dim3(256), 0, st, L, seg_nodes, x, (const int32_t *)flag,
                       (const int32_t *)pos, idx, sx, ssp);
    hipLaunchKernelGGL(k_ses_spheres, dim3(grid_for(n_grp, 256, INT32_MAX)), dim3(256), 0, st, ns,
                       (const int32_t *)pos, (const double *)sx, sph);
    hipLaunchKernelGGL(k_ses_super, dim3(grid_for(n_sup, 256, INT32_MAX)), dim3(256), 0, st, ns,
                       (const int32_t *)pos, (const double *)sph, sup);
    J.flag = flag;
    J.pos = pos;
    J.ses_idx = idx;
    J.ses_x = sx;
    J.ses_ssp = ssp;
    J.ses_sph = sph;
    J.ses_sup = sup;
    return DD_OK;
}

__global__ void k_euler(int64_t nn, double *x, const double *__restrict__ vel, double dt)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 3 * nn) return;
    x[i] += vel[i] * dt;
}

// ---------------------------------------------- a7: slip-rate accumulation --
// One workgroup per instance; per-lane sums reduced in a fixed tree order.
// mode 0: gdot_alpha(k) from velocities, added to out[inst][12]; mode 1:
// features (resolved shear, mobile and sessile densities) written to
// out[inst][36]; mode 2: gdot_alpha(k) and the line density of the segments
// that belong to a slip system, added to out[inst][13].
// Slip-rate contribution of a segment with unit tangent t, Burgers vector b
// (units of a) and length Ls on its system (n, m): (b.m) Ls ((t x vbar).n) / V,
// vbar the mean velocity of its nodes g1, g2.
__device__ __forceinline__ double seg_rate(const double *t, const double *b, double Ls, const double *vel,
                                           int64_t nn, int64_t g1, int64_t g2, const double *n, const double *m,
                                           double a, double invV)
{
    const double vb0 = 0.5 * (vel[g1] + vel[g2]);
    const double vb1 = 0.5 * (vel[nn + g1] + vel[nn + g2]);
    const double vb2 = 0.5 * (vel[2 * nn + g1] + vel[2 * nn + g2]);
    const double c0 = t[1] * vb2 - t[2] * vb1, c1 = t[2] * vb0 - t[0] * vb2, c2 = t[0] * vb1 - t[1] * vb0;
    const double bm = (b[0] * m[0] + b[1] * m[1] + b[2] * m[2]) * a;
    return bm * Ls * (c0 * n[0] + c1 * n[1] + c2 * n[2]) * invV;
}

__global__ __launch_bounds__(256) void k_instance_sums(Layout L, int mode,
                                                       const int32_t *__restrict__ seg_nodes,
                                                       const double *__restrict__ rec,
                                                       const int32_t *__restrict__ sys,
                                                       const double *__restrict__ vel,
                                                       const uint8_t *__restrict__ pinned,
                                                       const double *__restrict__ volume,
                                                       const double *__restrict__ sig_dev,
                                                       double a, double *__restrict__ out)
{
    __shared__ double red[24][256];
    const int inst = blockIdx.x;
    const int64_t s0 = L.seg_off ? L.seg_off[inst] : 0;
    const int64_t s1 = L.seg_off ? L.seg_off[inst + 1] : L.ns;
    const int64_t nn = L.nn, ns = L.ns;
    const double invV = 1.0 / volume[inst];
    double acc[24];
    for (int k = 0; k < 24; ++k) acc[k] = 0.0;
    for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const int al = sys[s];
        if (al < 0) continue;
        double n[3], m[3];
        fcc(al, n, m);
        const double Ls = rec[6 * ns + s] * a;
        if (mode == 2) acc[12] += Ls * invV;
        if (mode == 0 || mode == 2) {
            int64_t g1, g2;
            seg_ends(L, seg_nodes, s, g1, g2);
            const double t[3] = {rec[3 * ns + s], rec[4 * ns + s], rec[5 * ns + s]};
            const double b[3] = {rec[7 * ns + s], rec[8 * ns + s], rec[9 * ns + s]};
            const double val = seg_rate(t, b, Ls, vel, nn, g1, g2, n, m, a, invV);
            for (int k = 0; k < 12; ++k)
                if (k == al) acc[k] += val;
        } else {
            int64_t g1, g2;
            seg_ends(L, seg_nodes, s, g1, g2);
            const bool ses = pinned && pinned[g1] && pinned[g2];
            for (int k = 0; k < 12; ++k)
                if (k == al) {
                    if (ses) acc[12 + k] += Ls * invV;
                    else acc[k] += Ls * invV;
                }
        }
    }
    const int nv = mode == 0 ? 12 : (mode == 2 ? 13 : 24);
    for (int k = 0; k < nv; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < nv; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (mode == 0) {
            for (int k = 0; k < 12; ++k) out[12 * inst + k] += red[k][0];
        } else if (mode == 2) {
            for (int k = 0; k < 13; ++k) out[13 * inst + k] += red[k][0];
        } else {
            double S[3][3];
            const double *sv = sig_dev + 6 * inst;
            S[0][0] = sv[0]; S[1][1] = sv[1]; S[2][2] = sv[2];
            S[1][2] = S[2][1] = sv[3];
            S[0][2] = S[2][0] = sv[4];
            S[0][1] = S[1][0] = sv[5];
            for (int al = 0; al < 12; ++al) {
                double n[3], m[3];
                fcc(al, n, m);
                double tau = 0.0;
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) tau += m[r] * S[r][c] * n[c];
                out[36 * inst + al] = tau;
                out[36 * inst + 12 + al] = red[al][0];
                out[36 * inst + 24 + al] = red[12 + al][0];
            }
        }
    }
}

__global__ void k_scale_rates(double *acc, int64_t n, double inv_steps)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) acc[i] *= inv_steps;
}

// ------------------------------------------------ persistent small bursts --
// Every step of a batch of small bursts (FP64, no junctions, no exact band)
// in one launch: G_i co-resident workgroups per instance i (a cooperative
// launch) that meet at one barrier per step.  Each workgroup rebuilds its
// instance's segment records in LDS from the positions of the step; it owns
// a contiguous range of the instance's nodes and evaluates, for every
// segment incident to them (a segment whose nodes lie in two ranges is
// evaluated by both owners), the stress at its Gauss points from every other
// segment, summed over fixed chunks of PB_CHUNK sources in chunk order, then
// the end forces, the nodal forces in node-list order and the glide step of
// its nodes.  No sum depends on G_i, so the results do not depend on how the
// instances are split.  Positions and velocities alternate between two
// buffers from step to step.  The slip-rate sums of a step are formed after
// the next barrier (every velocity is then written; the step's records are
// still in LDS), per workgroup over the segments that start at its nodes, in
// index order, and summed over the workgroups in order at the end.
constexpr int PB_THREADS = 512;
constexpr int PB_MAX_SEGS = 512;    // segments and nodes per instance
constexpr int PB_CHUNK = 8;         // sources per partial sum
constexpr int PB_ITEMS = 1024;      // (target point, chunk) partial sums held at once
constexpr int PB_NODES_PER_WG = 2;  // nodes per workgroup aimed at
constexpr int PB_MAX_G = 128;       // workgroups per instance at most
constexpr uint64_t PB_WAIT_TICKS = 200000000ull;   // longest barrier wait: 2 s of the 100 MHz wall clock

struct PBArgs {
    Layout L;
    const int32_t *seg_nodes;
    const double *burgers, *normal;
    const uint8_t *pinned;
    const double *sigma_app;   // [n_inst][6]
    const double *volume;      // [n_inst]
    const int32_t *csr_ptr, *csr_list;
    const int32_t *wg;         // [4][n_wg]: instance, rank in it, the instance's G, its first workgroup
    int n_wg;
    double *xa, *xb;           // positions: the caller's array and the second buffer [3][nn]
    double *vel;               // [2][3][nn]
    double *wpart;             // [n_wg][12]
    unsigned *arrive;          // [n_wg][16] barrier arrival words (one per 64 bytes), zero at launch
    unsigned *flags;
    double *rate_out;          // [n_inst][12], added to
    GaussRule g;
    double kr, nu, k2, inv_a, a, inv_mu, fscale, invB, dt;
    int n_steps;
};

// Barrier of the G workgroups of one instance (workgroups first ..
// first + G - 1), the step-th since the launch: each workgroup publishes step
// in its own arrival word (one per 64-byte line, after a release fence) and
// waits, one thread per workgroup, until every word of the instance holds at
// least step; then one acquire fence for the workgroup.  A wait longer than
// PB_WAIT_TICKS raises FLAG_BARRIER and returns false (the caller then
// leaves the kernel, and so, after their own wait, do the other workgroups).
__device__ __forceinline__ bool pb_barrier(unsigned *arrive, int wg, int first, int G, unsigned step,
                                           unsigned *flags)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_store(arrive + 16 * wg, step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    if ((int)threadIdx.x < G) {
        const unsigned *f = arrive + 16 * (first + (int)threadIdx.x);
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < step) {
            if (wall_clock64() - t0 > PB_WAIT_TICKS) {
                atomicOr(flags, FLAG_BARRIER);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    ok = __syncthreads_and(ok);
    if (threadIdx.x == 0) __threadfence();
    __syncthreads();
    return ok != 0;
}

__global__ __launch_bounds__(PB_THREADS) void k_burst_persistent(PBArgs A)
{
    __shared__ double s_rec[PB_MAX_SEGS][16];   // x1, t, L, b, c (units of a)
    __shared__ double s_part[PB_ITEMS][3];
    __shared__ double s_segF[PB_MAX_SEGS][6];   // end forces of the listed segments
    __shared__ double s_wacc[12];
    __shared__ int32_t s_list[PB_MAX_SEGS];     // the workgroup's segments (instance-local), index order
    __shared__ int16_t s_loc[PB_MAX_SEGS];      // segment -> list position, -1: not listed
    __shared__ int8_t s_sys[PB_MAX_SEGS];
    __shared__ uint8_t s_own[PB_MAX_SEGS];      // listed segment starts at an owned node
    __shared__ int s_nl;
    const int tid = threadIdx.x, wg = blockIdx.x;
    const int inst = A.wg[wg], w = A.wg[A.n_wg + wg], G = A.wg[2 * A.n_wg + wg], first = A.wg[3 * A.n_wg + wg];
    const Layout &L = A.L;
    const int64_t nn = L.nn, ns = L.ns;
    const int64_t n0 = L.node_off[inst], nn_i = L.node_off[inst + 1] - n0;
    const int64_t s0 = L.seg_off[inst], ns_i = L.seg_off[inst + 1] - s0;
    const int64_t o_lo = n0 + nn_i * w / G, o_hi = n0 + nn_i * (w + 1) / G;   // owned nodes
    const double invV = 1.0 / A.volume[inst];
    unsigned step_no = 0;   // barriers passed

    // the list of segments incident to owned nodes, their slip systems
    if (tid == 0) {
        int nl = 0;
        for (int64_t sl = 0; sl < ns_i; ++sl) {
            int64_t g1, g2;
            seg_ends(L, A.seg_nodes, s0 + sl, g1, g2);
            const bool own1 = g1 >= o_lo && g1 < o_hi, own2 = g2 >= o_lo && g2 < o_hi;
            s_loc[sl] = -1;
            if (own1 || own2) {
                s_loc[sl] = (int16_t)nl;
                s_list[nl] = (int32_t)sl;
                s_own[nl] = own1;
                ++nl;
            }
        }
        s_nl = nl;
        for (int k = 0; k < 12; ++k) s_wacc[k] = 0.0;
    }
    for (int64_t sl = tid; sl < ns_i; sl += PB_THREADS) {
        const int64_t sg = s0 + sl;
        int64_t g1, g2;
        unsigned fl = seg_ends(L, A.seg_nodes, sg, g1, g2) ? 0u : FLAG_BAD_INDEX;
        const double b[3] = {A.burgers[sg], A.burgers[ns + sg], A.burgers[2 * ns + sg]};
        const double nv[3] = {A.normal[sg], A.normal[ns + sg], A.normal[2 * ns + sg]};
        if (!(fabs(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2] - 1.0) <= 2e-6)) fl |= FLAG_BAD_NORMAL;
        s_sys[sl] = (int8_t)seg_system(b, nv);
        if (fl) atomicOr(A.flags, fl);
    }
    __syncthreads();
    const int nl = s_nl;
    const int Q = A.g.n;
    const int nch = (int)((ns_i + PB_CHUNK - 1) / PB_CHUNK);
    const int per_batch = nch > 0 ? (PB_ITEMS / (Q * nch) > 0 ? PB_ITEMS / (Q * nch) : 1) : 1;
    double S6[6];
    for (int k = 0; k < 6; ++k) S6[k] = A.sigma_app[6 * inst + k] * A.inv_mu;

    for (int k = 0; k <= A.n_steps; ++k) {
        const double *xc = (k & 1) ? A.xb : A.xa;   // positions at the start of step k
        if (k > 0) {
            if (!pb_barrier(A.arrive, wg, first, G, ++step_no, A.flags)) return;
            // slip-rate sums of step k - 1 (its records are still in LDS)
            const double *vk = A.vel + (int64_t)((k - 1) & 1) * 3 * nn;
            for (int l = tid; l < nl; l += PB_THREADS) {
                s_part[l][0] = 0.0;
                const int sl = s_list[l], al = s_sys[sl];
                if (!s_own[l] || al < 0) continue;
                int64_t g1, g2;
                seg_ends(L, A.seg_nodes, s0 + sl, g1, g2);
                double n[3], m[3];
                fcc(al, n, m);
                const double *r = s_rec[sl];
                s_part[l][0] = seg_rate(r + 3, r + 7, r[6] * A.a, vk, nn, g1, g2, n, m, A.a, invV);
            }
            __syncthreads();
            if (tid == 0)
                for (int l = 0; l < nl; ++l) {
                    const int al = s_sys[s_list[l]];
                    if (s_own[l] && al >= 0) s_wacc[al] += s_part[l][0];
                }
            __syncthreads();
        }
        if (k == A.n_steps) break;
        // records of step k
        for (int64_t sl = tid; sl < ns_i; sl += PB_THREADS) {
            int64_t g1, g2;
            seg_ends(L, A.seg_nodes, s0 + sl, g1, g2);
            const double Ls = seg_record(xc, nn, g1, g2, A.burgers, ns, s0 + sl, A.inv_a, s_rec[sl]);
            if (!(Ls > 0.0) || !isfinite(Ls)) atomicOr(A.flags, FLAG_ZERO_LENGTH);
        }
        __syncthreads();
        // Gauss-point stresses of the listed segments, in batches of whole segments
        for (int l0 = 0; l0 < nl; l0 += per_batch) {
            const int l1 = l0 + per_batch < nl ? l0 + per_batch : nl;
            const int items = (l1 - l0) * Q * nch;
            for (int it = tid; it < items; it += PB_THREADS) {
                const int c = it % nch, tq = it / nch;
                const int sj = s_list[l0 + tq / Q], q = tq % Q;
                const double *rj = s_rec[sj];
                double sq = A.g.s[0];
                for (int i = 1; i < DD_MAX_GAUSS; ++i)
                    if (i == q) sq = A.g.s[i];
                const double xq0 = rj[0] + sq * rj[6] * rj[3];
                const double xq1 = rj[1] + sq * rj[6] * rj[4];
                const double xq2 = rj[2] + sq * rj[6] * rj[5];
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, ak = 0.0;
                const int c1 = (c + 1) * PB_CHUNK < ns_i ? (c + 1) * PB_CHUNK : (int)ns_i;
                for (int src = c * PB_CHUNK; src < c1; ++src) {
                    if (src == sj) continue;
                    const double *d = s_rec[src];
                    const double R0 = xq0 - d[0], R1 = xq1 - d[1], R2 = xq2 - d[2];
                    const double r1 = rsqrt64(fma(R2, R2, fma(R1, R1, fma(R0, R0, 1.0))));
                    double r2, r2c;
                    pair_acc_f64(xq0, xq1, xq2, rj[7], rj[8], rj[9], d[0], d[1], d[2], d[3], d[4], d[5], d[6],
                                 d[7], d[8], d[9], d[10], d[11], d[12], A.kr, A.nu, r1, r1 * r1 * r1, r2, r2c, a0,
                                 a1, a2, ak);
                }
                s_part[it][0] = A.k2 * fma(ak, rj[7], a0);
                s_part[it][1] = A.k2 * fma(ak, rj[8], a1);
                s_part[it][2] = A.k2 * fma(ak, rj[9], a2);
            }
            __syncthreads();
            // end forces: per listed segment, Gauss points in order, chunks in order
            for (int l = l0 + tid; l < l1; l += PB_THREADS) {
                const double *rj = s_rec[s_list[l]];
                const double t0 = rj[3], t1 = rj[4], t2 = rj[5], Ls = rj[6];
                const double b0 = rj[7], b1 = rj[8], b2 = rj[9];
                const double ab0 = S6[0] * b0 + S6[5] * b1 + S6[4] * b2;
                const double ab1 = S6[5] * b0 + S6[1] * b1 + S6[3] * b2;
                const double ab2 = S6[4] * b0 + S6[3] * b1 + S6[2] * b2;
                double F1[3] = {0, 0, 0}, F2[3] = {0, 0, 0};
                for (int q = 0; q < Q; ++q) {
                    const int base = ((l - l0) * Q + q) * nch;
                    double sa = 0, sb = 0, sc = 0;
                    for (int c = 0; c < nch; ++c) {
                        sa += s_part[base + c][0];
                        sb += s_part[base + c][1];
                        sc += s_part[base + c][2];
                    }
                    sa += ab0;
                    sb += ab1;
                    sc += ab2;
                    const double f0 = sb * t2 - sc * t1, f1 = sc * t0 - sa * t2, f2 = sa * t1 - sb * t0;
                    const double w1 = Ls * A.g.w[q] * (1.0 - A.g.s[q]), w2 = Ls * A.g.w[q] * A.g.s[q];
                    F1[0] += w1 * f0; F1[1] += w1 * f1; F1[2] += w1 * f2;
                    F2[0] += w2 * f0; F2[1] += w2 * f1; F2[2] += w2 * f2;
                }
                for (int c = 0; c < 3; ++c) {
                    s_segF[l][c] = F1[c] * A.fscale;
                    s_segF[l][3 + c] = F2[c] * A.fscale;
                }
            }
            __syncthreads();
        }
        // owned nodes: nodal force in node-list order, glide step into the other buffers
        double *xn = (k & 1) ? A.xa : A.xb;
        double *vn = A.vel + (int64_t)(k & 1) * 3 * nn;
        for (int64_t n = o_lo + tid; n < o_hi; n += PB_THREADS) {
            double F0 = 0, F1 = 0, F2 = 0, ell = 0.0, nrm[3][3];
            int cnt = 0;
            for (int32_t e = A.csr_ptr[n]; e < A.csr_ptr[n + 1]; ++e) {
                const int32_t v = A.csr_list[e];
                const int64_t sg = v >> 1;
                const int end = v & 1, l = s_loc[sg - s0];
                F0 += s_segF[l][3 * end];
                F1 += s_segF[l][3 * end + 1];
                F2 += s_segF[l][3 * end + 2];
                ell += 0.5 * (s_rec[sg - s0][6] * A.a);
                add_normal(A.normal[sg], A.normal[ns + sg], A.normal[2 * ns + sg], nrm, cnt);
            }
            double v0 = 0, v1 = 0, v2 = 0;
            const bool fixed = (A.pinned && A.pinned[n]) || !(ell > 0.0) || cnt == 0 || cnt >= 3;
            if (!fixed) glide_velocity(F0, F1, F2, ell, A.invB, nrm, cnt, v0, v1, v2);
            vn[n] = v0;
            vn[nn + n] = v1;
            vn[2 * nn + n] = v2;
            xn[n] = xc[n] + v0 * A.dt;
            xn[nn + n] = xc[nn + n] + v1 * A.dt;
            xn[2 * nn + n] = xc[2 * nn + n] + v2 * A.dt;
        }
    }
    // an odd number of steps leaves the positions in the second buffer: owned
    // nodes back to the caller's array (every read of it ended at the last barrier)
    if (A.n_steps & 1)
        for (int64_t n = o_lo + tid; n < o_hi; n += PB_THREADS)
            for (int c = 0; c < 3; ++c) A.xa[c * nn + n] = A.xb[c * nn + n];
    if (tid < 12) A.wpart[12 * (int64_t)wg + tid] = s_wacc[tid];
    if (!pb_barrier(A.arrive, wg, first, G, ++step_no, A.flags)) return;
    if (w == 0 && tid < 12) {
        double sum = 0.0;
        for (int v = 0; v < G; ++v) sum += A.wpart[12 * (int64_t)(first + v) + tid];
        A.rate_out[12 * (int64_t)inst + tid] += sum;
    }
}

// =================================================================== host ==
namespace {

int check_material(const dd_material *m, bool need_B)
{
    if (!m) return set_error(DD_EINVAL, "material is null");
    if (!(m->mu > 0.0) || !std::isfinite(m->mu)) return set_error(DD_EINVAL, "mu must be > 0");
    if (!(m->nu > -1.0 && m->nu < 0.5)) return set_error(DD_EINVAL, "nu must lie in (-1, 0.5)");
    if (!(m->a > 0.0) || !std::isfinite(m->a)) return set_error(DD_EINVAL, "core width a must be > 0");
    if (need_B && (!(m->B > 0.0) || !std::isfinite(m->B))) return set_error(DD_EINVAL, "drag B must be > 0");
    return DD_OK;
}

}  // namespace

// The flags word is sticky: kernels OR into it and only a report clears it,
// so a condition raised by a call made with validation off is reported by the
// next call that validates (or by dd_check).
int read_flags(Workspace *ws, hipStream_t st)
{
    DD_HIP(hipMemcpyAsync(ws->flags_host, ws->flags_dev, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    const unsigned f = *ws->flags_host;
    if (!f) return DD_OK;
    *ws->flags_host = 0u;
    DD_HIP(hipMemcpyAsync(ws->flags_dev, ws->flags_host, sizeof(unsigned), hipMemcpyHostToDevice, st));
    DD_HIP(hipStreamSynchronize(st));
    const char *w = " (this call or an earlier one made with validation off)";
    if (f & FLAG_BAD_INDEX)
        return set_error(DD_EINVAL, "a segment references a node index outside its instance%s", w);
    if (f & FLAG_ZERO_LENGTH) return set_error(DD_EINVAL, "zero-length (or non-finite) segment%s", w);
    if (f & FLAG_BAD_NORMAL) return set_error(DD_EINVAL, "slip-plane normal is not of unit length%s", w);
    if (f & FLAG_NONFINITE) return set_error(DD_ENONFINITE, "non-finite value in an output%s", w);
    if (f & FLAG_NEAR_FULL)
        return set_error(DD_ECAPACITY, "exact band: the near pairs of a captured step outgrew the pair store "
                         "sized at the start of the burst%s", w);
    if (f & FLAG_NEAR_PANELS) return set_error(DD_EINVAL, "exact band: a pair integral did not converge%s", w);
    if (f & FLAG_BARRIER)
        return set_error(DD_EHIP, "persistent burst: a workgroup waited too long at a step barrier%s", w);
    return DD_OK;
}

namespace {

template <class T>
int upload(Workspace *ws, Slot s, const std::vector<T> &v, T **dev, hipStream_t st)
{
    void *p;
    int rc = ensure(ws, s, v.size() * sizeof(T), &p);
    if (rc) return rc;
    if (!v.empty()) {
        DD_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        DD_HIP(hipStreamSynchronize(st));   // v is pageable and short-lived
    }
    *dev = (T *)p;
    return DD_OK;
}

// Device state of one force evaluation set-up.
struct ForceCtx {
    Layout L{};
    double *rec64 = nullptr;
    float *rec32 = nullptr;
    int32_t *sys = nullptr;
    double *partial = nullptr;
    double *segF = nullptr;
    int32_t *csr_ptr = nullptr, *csr_list = nullptr, *csr_cnt = nullptr;
    int32_t *scan_tmp = nullptr;   // scratch of the node-list scan (after csr_cnt)
    Tile *tiles = nullptr;
    Item *items = nullptr;
    int64_t n_items = 0;
    GaussRule g{};
    double k1 = 0, k2 = 0, inv_a = 0, inv_mu = 0, fscale = 0, a = 0;
    int precision = DD_FP64;
    int variant = 0;   // mixed kernel: 0 = FP32 quadrature band test first, 1 = no quadrature
    float cut = 0.f;
    bool near_on = false;   // exact band in use (positions, topology and layout are set per launch)
    NearArgs near{};        // pair store (pair_t, pair_s, corr, pair_cap) sized by size_near_pairs
};

// Cache of the last uploaded plan (the tables depend only on sizes).
struct PlanKey {
    std::vector<int64_t> seg_off;
    std::vector<uint8_t> active;   // empty: every instance
    int Q = 0;
    int64_t chunk_len = -1;
    bool operator==(const PlanKey &o) const
    {
        return Q == o.Q && chunk_len == o.chunk_len && seg_off == o.seg_off && active == o.active;
    }
};
PlanKey g_plan_key;   // guarded by the single-caller-per-device rule
int g_plan_dev = -1;
int64_t g_plan_items = 0;
int64_t g_plan_chunk = 0;
int g_last_variant = 0;

int setup(Workspace *ws, hipStream_t st, const std::vector<int64_t> &seg_off_h, int64_t nn,
          const int32_t *seg_nodes, const dd_material *m, int n_gauss, int precision,
          double near_cut, double eta, int64_t chunk_len, bool need_sys, ForceCtx &C,
          const std::vector<uint8_t> *active = nullptr)
{
    const int64_t ns = seg_off_h.back();
    const int n_inst = (int)seg_off_h.size() - 1;
    C.g = gauss_rule(n_gauss);
    C.k1 = 1.0 / (8.0 * M_PI);
    C.k2 = 1.0 / (4.0 * M_PI * (1.0 - m->nu));
    C.a = m->a;
    C.inv_a = 1.0 / m->a;
    C.inv_mu = 1.0 / m->mu;
    C.fscale = m->mu * m->a * m->a;
    C.precision = precision;
    C.cut = (float)near_cut;
    C.L.nn = nn;
    C.L.ns = ns;
    void *p;
    int rc;
    if ((rc = ensure(ws, WS_SEG64, rec64_bytes(ns), &p))) return rc;
    C.rec64 = (double *)p;
    if (precision == DD_MIXED) {
        if ((rc = ensure(ws, WS_SEG32, sizeof(float) * REC32A * std::max<int64_t>(ns, 1), &p))) return rc;
        C.rec32 = (float *)p;
    }
    if (need_sys) {
        if ((rc = ensure(ws, WS_MISC, sizeof(int32_t) * std::max<int64_t>(ns, 1), &p))) return rc;
        C.sys = (int32_t *)p;
    }
    if ((rc = ensure(ws, WS_SEGF, sizeof(double) * 6 * std::max<int64_t>(ns, 1), &p))) return rc;
    C.segF = (double *)p;
    if ((rc = ensure(ws, WS_CSR_PTR, sizeof(int32_t) * (nn + 1), &p))) return rc;
    C.csr_ptr = (int32_t *)p;
    if ((rc = ensure(ws, WS_CSR_LIST, sizeof(int32_t) * std::max<int64_t>(2 * ns, 1), &p))) return rc;
    C.csr_list = (int32_t *)p;
    if ((rc = ensure(ws, WS_CSR_CNT, sizeof(int32_t) * (std::max<int64_t>(nn, 1) + scan_scratch_len(nn)), &p)))
        return rc;
    C.csr_cnt = (int32_t *)p;
    C.scan_tmp = C.csr_cnt + std::max<int64_t>(nn, 1);

    // plan tables (cached by size)
    PlanKey key;
    key.seg_off = seg_off_h;
    key.Q = n_gauss;
    key.chunk_len = chunk_len;
    if (active) key.active = *active;
    if (!(key == g_plan_key) || g_plan_dev != ws->device || !ws->ptr[WS_TILES]) {
        Plan P;
        make_plan(seg_off_h, n_gauss, chunk_len, P, active);
        Tile *dt;
        Item *di;
        int64_t *dtb;
        if ((rc = upload(ws, WS_TILES, P.tiles, &dt, st))) return rc;
        if ((rc = upload(ws, WS_ITEMS, P.items, &di, st))) return rc;
        std::vector<int64_t> offs;   // [tile_begin (n_inst+1)]
        offs = P.tile_begin;
        if ((rc = upload(ws, WS_OFFS, offs, &dtb, st))) return rc;
        g_plan_key = key;
        g_plan_dev = ws->device;
        g_plan_items = (int64_t)P.items.size();
        g_plan_chunk = P.chunk_len;
    }
    C.tiles = (Tile *)ws->ptr[WS_TILES];
    C.items = (Item *)ws->ptr[WS_ITEMS];
    C.L.tile_begin = n_inst > 1 || active ? (const int64_t *)ws->ptr[WS_OFFS] : nullptr;
    C.n_items = g_plan_items;
    if ((rc = ensure(ws, WS_PARTIAL, sizeof(double) * 3 * TILE * std::max<int64_t>(C.n_items, 1), &p)))
        return rc;
    C.partial = (double *)p;
    (void)seg_nodes;
    const double c2 = 2.0 * eta * eta;
    C.near_on = c2 > 0.0 && ns > 0;
    if (C.near_on) {
        if (ns > (int64_t)INT32_MAX)
            return set_error(DD_EINVAL, "the exact band supports at most %d segments", INT32_MAX);
        NearArgs &N = C.near;
        N = NearArgs{};
        N.ns = ns;
        N.nn = nn;
        N.n_waves = (ns + 63) / 64;
        N.c2 = c2;
        N.kr = C.k1 / C.k2;
        N.nu = m->nu;
        N.k2 = C.k2;
        N.g = C.g;
        N.gp = gauss_rule(12);
        N.rec = C.rec64;
        N.flags = ws->flags_dev;
        if ((rc = ensure(ws, WS_NEAR_KEY, sizeof(double) * 4 * ns, &p))) return rc;
        N.key = (double *)p;
        if ((rc = ensure(ws, WS_NEAR_SPH, sizeof(float4) * ((ns + NEAR_GROUP - 1) / NEAR_GROUP), &p))) return rc;
        N.sph = (float4 *)p;
        // split the source range of an instance over several workgroups when
        // the targets alone give fewer than ~4096 wavefronts: at least 64
        // source groups per split, at most 32 splits
        int64_t max_inst = 0;
        for (size_t i = 0; i + 1 < seg_off_h.size(); ++i) max_inst = std::max(max_inst, seg_off_h[i + 1] - seg_off_h[i]);
        const int64_t groups = (max_inst + NEAR_GROUP - 1) / NEAR_GROUP;
        const int64_t want = std::min<int64_t>((groups + 63) / 64, (262144 + ns - 1) / ns);
        N.splits = (int)std::min<int64_t>(32, std::max<int64_t>(1, want));
        // counts: scnt [ns][splits] and cnt [ns] (int32), then loc and ptr [ns] (int64)
        if ((rc = ensure(ws, WS_NEAR_IDX, sizeof(int32_t) * (1 + N.splits) * ns + 2 * sizeof(int64_t) * ns + 16, &p)))
            return rc;
        N.cnt = (int32_t *)p;
        N.scnt = N.cnt + ns;
        N.loc = (int64_t *)(((uintptr_t)(N.scnt + (int64_t)N.splits * ns) + 15) & ~(uintptr_t)15);
        N.ptr = N.loc + ns;
        if ((rc = ensure(ws, WS_NEAR_WAVE, sizeof(int64_t) * (2 * N.n_waves + 1), &p))) return rc;
        N.wtot = (int64_t *)p;
        N.woff = N.wtot + N.n_waves;
        // the pair store as it stands (grown by size_near_pairs)
        N.pair_cap = (int64_t)std::min(ws->cap[WS_NEAR_PAIR] / (2 * sizeof(int32_t)),
                                       ws->cap[WS_NEAR_CORR] / (6 * sizeof(double)));
        N.pair_t = (int32_t *)ws->ptr[WS_NEAR_PAIR];
        N.pair_s = N.pair_t + N.pair_cap;
        N.corr = (double *)ws->ptr[WS_NEAR_CORR];
    }
    return DD_OK;
}

// Makes the near-pair store hold at least `need` pairs (synchronises the
// device when it grows) and points C.near at it.
int grow_near_pairs(ForceCtx &C, Workspace *ws, int64_t need)
{
    NearArgs &N = C.near;
    if (need <= N.pair_cap && N.pair_t) return DD_OK;
    const int64_t cap = std::max<int64_t>(need, 1024);
    void *p;
    int rc;
    if ((rc = ensure(ws, WS_NEAR_PAIR, sizeof(int32_t) * 2 * cap, &p))) return rc;
    N.pair_t = (int32_t *)p;
    N.pair_s = N.pair_t + cap;
    if ((rc = ensure(ws, WS_NEAR_CORR, sizeof(double) * 6 * cap, &p))) return rc;
    N.corr = (double *)p;
    N.pair_cap = cap;
    return DD_OK;
}

// Counts the near pairs at positions x (the count pass and its scan), reads
// the total back (synchronising the stream) and grows the pair store to
// `factor` times it plus `extra` per segment.
int size_near_pairs(ForceCtx &C, Workspace *ws, const double *x, const int32_t *seg_nodes, double factor,
                    int64_t extra, hipStream_t st)
{
    NearArgs N = C.near;
    N.x = x;
    N.seg_nodes = seg_nodes;
    N.seg_inst = C.L.seg_inst;
    N.seg_off = C.L.seg_off;
    N.node_off = C.L.node_off;
    launch_near_count(N, st);
    int64_t *host = (int64_t *)((char *)ws->flags_host + 64);
    DD_HIP(hipMemcpyAsync(host, N.woff + N.n_waves, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    const int64_t total = *host;
    if (total < 0 || total > (int64_t)INT32_MAX)
        return set_error(DD_ECAPACITY, "exact band: %lld near pairs (at most %d); use a narrower band",
                         (long long)total, INT32_MAX);
    return grow_near_pairs(C, ws, std::min<int64_t>((int64_t)INT32_MAX,
                                                    (int64_t)(factor * (double)total) + extra * C.L.ns));
}

// Topology-only work: CSR of node -> (segment, end).
void launch_csr(const ForceCtx &C, const int32_t *seg_nodes, hipStream_t st)
{
    const int64_t nn = C.L.nn, ns = C.L.ns;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nn)), dim3(256), 0, st, (unsigned *)C.csr_cnt, nn, 0u);
    hipLaunchKernelGGL(k_csr_count, dim3(grid_for(ns, 256, INT32_MAX)), dim3(256), 0, st, C.L, seg_nodes,
                       C.csr_cnt);
    launch_scan<int32_t>(C.csr_cnt, nn, C.csr_ptr, C.scan_tmp, st);
    hipLaunchKernelGGL(k_csr_fill, dim3(grid_for(ns, 256, INT32_MAX)), dim3(256), 0, st, C.L, seg_nodes,
                       C.csr_ptr, C.csr_cnt, C.csr_list);
    hipLaunchKernelGGL(k_csr_sort, dim3(grid_for(nn, 256, INT32_MAX)), dim3(256), 0, st, C.csr_ptr, nn,
                       C.csr_list);
}

// The topology kernels of one step at time t0 + tk, t0 read from the device
// (releases, candidates, captures), and the node -> segment lists they
// change.
void launch_jnode_step(const ForceCtx &C, JNodeArgs J, double tk, int k, int n_inst, int32_t *seg_nodes, double *x,
                       double *burgers, double *normal, uint32_t *flags, const uint8_t *active, hipStream_t st)
{
    J.tk = tk;
    J.fk = k;
    hipLaunchKernelGGL(k_jn_release, dim3(n_inst), dim3(256), 0, st, C.L, seg_nodes, (const double *)x, burgers,
                       normal, J, active, flags);
    hipLaunchKernelGGL(k_jn_candidates, dim3(grid_for(C.L.ns, 256, INT32_MAX)), dim3(256), 0, st, C.L,
                       (const int32_t *)seg_nodes, (const double *)x, J, active);
    hipLaunchKernelGGL(k_jn_capture, dim3(n_inst), dim3(256), 0, st, C.L, seg_nodes, x, burgers, normal, J, active);
    launch_csr(C, seg_nodes, st);
}


// a1..a4 for positions x: segment records, pair kernel, epilogue, gather.
// With the exact band, size_pairs = true counts the near pairs first, reads
// the count back (one synchronisation) and sizes the pair store to fit;
// false (graph capture) uses the store as sized beforehand.
int launch_forces(ForceCtx &C, Workspace *ws, const double *x, const int32_t *seg_nodes,
                  const double *burgers, const double *normal, const double *sig_dev, Sig6 sig_val,
                  double *F, hipStream_t st, bool size_pairs)
{
    const int64_t nn = C.L.nn, ns = C.L.ns;
    if (ns > 0) {
        PrepArgs A;
        A.L = C.L;
        A.x = x;
        A.seg_nodes = seg_nodes;
        A.burgers = burgers;
        A.normal = normal;
        A.inv_a = C.inv_a;
        A.rec64 = C.rec64;
        A.rec32 = C.rec32;
        A.cut = C.cut;
        A.quadn = C.precision == DD_MIXED ? quad_points(C.variant) : 0;
        A.sys = C.sys;
        A.flags = ws->flags_dev;
        hipLaunchKernelGGL(k_seg_prep, dim3(grid_for(ns, PREP_BLOCK, INT32_MAX)), dim3(PREP_BLOCK), 0, st, A);
        // The near-pair work needs only the records and runs on the same
        // stream as the pair kernel (alongside it, on a second stream, it
        // slowed the pair kernel by more than its own duration): the count
        // pass before the pair kernel, the list and the exact integrals after
        // it.  With size_pairs the count is read back behind the pair kernel:
        // the host waits for the count (an event), not for the pair kernel, and
        // sizes the pair store before the list is written.
        NearArgs N = C.near;
        int64_t *count_host = nullptr;
        if (C.near_on) {
            N.x = x;
            N.seg_nodes = seg_nodes;
            N.seg_inst = C.L.seg_inst;
            N.seg_off = C.L.seg_off;
            N.node_off = C.L.node_off;
            launch_near_count(N, st);
            if (size_pairs) {
                if (!ws->near_ev) DD_HIP(hipEventCreateWithFlags(&ws->near_ev, hipEventDisableTiming));
                count_host = (int64_t *)((char *)ws->flags_host + 64);
                DD_HIP(hipMemcpyAsync(count_host, N.woff + N.n_waves, sizeof(int64_t), hipMemcpyDeviceToHost, st));
                DD_HIP(hipEventRecord(ws->near_ev, st));
            }
        }
        if (C.n_items > 0) {
            timing_begin(st, ws->capturing);
            if (C.precision == DD_MIXED)
                launch_pair_mixed(C.items, C.tiles, C.rec64, C.rec32, ns, C.g, C.k1, C.k2, C.cut, C.partial,
                                  ws->near_count, C.n_items, C.variant, st);
            else
                launch_pair64(C.items, C.tiles, C.rec64, ns, C.g, C.k1, C.k2, C.partial, C.n_items, st);
            timing_end(st, ws->capturing);
        }
        if (C.near_on) {
            if (size_pairs) {
                DD_HIP(hipEventSynchronize(ws->near_ev));
                const int64_t total = *count_host;
                if (total < 0 || total > (int64_t)INT32_MAX)
                    return set_error(DD_ECAPACITY, "exact band: %lld near pairs (at most %d); use a narrower band",
                                     (long long)total, INT32_MAX);
                int rc;
                if ((rc = grow_near_pairs(C, ws, total))) return rc;
                N.pair_t = C.near.pair_t;
                N.pair_s = C.near.pair_s;
                N.corr = C.near.corr;
                N.pair_cap = C.near.pair_cap;
            }
            launch_near_fill(N, st);
        }
        hipLaunchKernelGGL(k_segment_ends, dim3(grid_for(ns, 256, INT32_MAX)), dim3(256), 0, st, C.L,
                           C.tiles, C.partial, C.rec64, C.g, sig_dev, sig_val, C.inv_mu, C.fscale,
                           C.segF, C.near_on ? (const int64_t *)C.near.ptr : nullptr,
                           (const int32_t *)C.near.cnt, (const double *)C.near.corr, C.near.pair_cap);
    }
    hipLaunchKernelGGL(k_node_gather, dim3(grid_for(nn, 256, INT32_MAX)), dim3(256), 0, st, C.csr_ptr,
                       C.csr_list, nn, ns, C.segF, F);
    return DD_OK;
}

// ------------------------------------------------------------- autotuner --
// The source-range length of a work item (how many sources one workgroup
// streams through LDS for its 256 target points) sets the number of items,
// the partial-sum traffic and the load balance between uneven instances; the
// mixed kernel also has two orders of locating a pair (FP32 first or FP64
// first) whose relative cost depends on how sparse the volume is.  On
// the first call for a given (GPU architecture, Gauss points, precision,
// instance count, total and largest instance size, in powers of two) the
// candidates below are timed with HIP events on one all-pairs pass over the
// caller's own data, and the fastest is kept for the process (and appended
// to the file named by DD_AUTOTUNE_CACHE, read back at start-up).
std::atomic<int> g_autotune{1};
std::atomic<int> g_burst_mode{0};   // dd_set_burst_mode: 0 automatic, 1 step graphs, 2 persistent, one workgroup each
std::atomic<int64_t> g_forced_choice{-1};   // dd_set_plan: encoded split, or -1

struct TuneKey {
    std::string arch;
    int Q, prec, li, ls, lm;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(arch, Q, prec, li, ls, lm) < std::tie(o.arch, o.Q, o.prec, o.li, o.ls, o.lm);
    }
};
std::map<TuneKey, int64_t> g_tuned;
std::mutex g_tune_mu;
bool g_tune_loaded = false;

int ceil_log2(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

void load_tune_cache()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("DD_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *fp = std::fopen(path, "r");
    if (!fp) return;
    char arch[128];
    int Q, prec, li, ls, lm;
    long long c;
    while (std::fscanf(fp, "%127s %d %d %d %d %d %lld", arch, &Q, &prec, &li, &ls, &lm, &c) == 7)
        g_tuned[TuneKey{arch, Q, prec, li, ls, lm}] = c;
    std::fclose(fp);
}

void save_tune(const TuneKey &k, int64_t c)
{
    const char *path = std::getenv("DD_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *fp = std::fopen(path, "a");
    if (!fp) return;
    std::fprintf(fp, "%s %d %d %d %d %d %lld\n", k.arch.c_str(), k.Q, k.prec, k.li, k.ls, k.lm, (long long)c);
    std::fclose(fp);
}

// Returns MIXED_VARIANTS * (chunk length to use, 0 = the built-in heuristic)
// + the mixed kernel's variant.
int tuned_chunk(Workspace *ws, hipStream_t st, const std::vector<int64_t> &so, int64_t nn,
                const Layout &inst, const int32_t *seg_nodes, const double *x, const double *burgers,
                const double *normal, const dd_material *m, int Q, int prec, double cut, bool need_sys,
                int64_t *out)
{
    *out = 0;
    const int64_t forced = g_forced_choice.load();
    if (forced >= 0) {
        *out = forced;
        return DD_OK;
    }
    if (!g_autotune.load()) return DD_OK;
    const int n_inst = (int)so.size() - 1;
    int64_t ns = so.back(), nmax = 0;
    for (int i = 0; i < n_inst; ++i) nmax = std::max(nmax, so[i + 1] - so[i]);
    if (ns < 2 * TILE) return DD_OK;   // nothing to choose
    double evals = 0.0;
    for (int i = 0; i < n_inst; ++i) evals += (double)(so[i + 1] - so[i]) * (double)(so[i + 1] - so[i]) * Q;
    if (evals > 2e10) return DD_OK;   // one timed pass would cost more than the choice can save
    const int reps = evals > 1e9 ? 1 : 2;
    hipDeviceProp_t prop;
    DD_HIP(hipGetDeviceProperties(&prop, ws->device));
    TuneKey key{prop.gcnArchName, Q, prec, ceil_log2(n_inst), ceil_log2(ns), ceil_log2(nmax)};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache();
    auto itk = g_tuned.find(key);
    if (itk != g_tuned.end()) {
        *out = itk->second;
        return DD_OK;
    }
    Range range_("dd autotune");
    // a choice is encoded as MIXED_VARIANTS * chunk_length + mixed-kernel variant
    std::vector<int64_t> chunks = {0};
    // short ranges spread small batches over more CUs; long ones need fewer partial sums
    for (int64_t c = 64; c < nmax; c *= 2) chunks.push_back(c);
    chunks.push_back(((nmax + TILE - 1) / TILE) * TILE);   // one range per tile
    std::vector<int64_t> cands;
    for (int64_t c : chunks)
        for (int v = 0; v < (prec == DD_MIXED ? MIXED_VARIANTS : 1); ++v)
            cands.push_back(MIXED_VARIANTS * c + v);
    hipEvent_t e0, e1;
    DD_HIP(hipEventCreate(&e0));
    DD_HIP(hipEventCreate(&e1));
    double best = 1e300;
    int64_t best_c = 0;
    int rc = DD_OK;
    for (int64_t cv : cands) {
        const int64_t c = cv / MIXED_VARIANTS;
        ForceCtx C;
        if ((rc = setup(ws, st, so, nn, seg_nodes, m, Q, prec, cut, 0.0, c, need_sys, C))) break;
        C.variant = (int)(cv % MIXED_VARIANTS);
        PrepArgs A{};
        A.L = C.L;
        A.L.seg_inst = inst.seg_inst;
        A.L.node_off = inst.node_off;
        A.L.seg_off = inst.seg_off;
        A.x = x;
        A.seg_nodes = seg_nodes;
        A.burgers = burgers;
        A.normal = normal;
        A.inv_a = C.inv_a;
        A.rec64 = C.rec64;
        A.rec32 = C.rec32;
        A.cut = C.cut;
        A.quadn = C.precision == DD_MIXED ? quad_points(C.variant) : 0;
        A.flags = ws->flags_dev;
        hipLaunchKernelGGL(k_seg_prep, dim3(grid_for(ns, PREP_BLOCK, INT32_MAX)), dim3(PREP_BLOCK), 0, st, A);
        double t_min = 1e300;
        for (int rep = 0; rep < reps; ++rep) {
            (void)hipEventRecord(e0, st);
            if (prec == DD_MIXED)
                launch_pair_mixed(C.items, C.tiles, C.rec64, C.rec32, ns, C.g, C.k1, C.k2, C.cut, C.partial,
                                  ws->near_count, C.n_items, C.variant, st);
            else
                launch_pair64(C.items, C.tiles, C.rec64, ns, C.g, C.k1, C.k2, C.partial, C.n_items, st);
            // the reduction of the partial sums grows with the number of work
            // items, so it is part of the cost being compared
            hipLaunchKernelGGL(k_segment_ends, dim3(grid_for(ns, 256, INT32_MAX)), dim3(256), 0, st, A.L,
                               C.tiles, C.partial, C.rec64, C.g, (const double *)nullptr, Sig6{}, C.inv_mu,
                               C.fscale, C.segF, (const int64_t *)nullptr, (const int32_t *)nullptr,
                               (const double *)nullptr, (int64_t)0);
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) {
                rc = set_error(DD_EHIP, "autotuner timing failed");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t_min = std::min(t_min, (double)ms);
        }
        if (rc) break;
        if (t_min < best) {
            best = t_min;
            best_c = cv;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    g_tuned[key] = best_c;
    save_tune(key, best_c);
    *out = best_c;
    return DD_OK;
}

int common_checks(int64_t n_nodes, int64_t n_segs, int n_gauss, int precision, double near_cut, double eta = 0.0)
{
    if (!(eta >= 0.0) || std::isinf(eta)) return set_error(DD_EINVAL, "exact_eta must be finite and >= 0");
    if (n_nodes < 0 || n_segs < 0) return set_error(DD_EINVAL, "negative node or segment count");
    if (n_nodes >= INT32_MAX || 2 * n_segs >= INT32_MAX)
        return set_error(DD_EINVAL, "more than 2^31 nodes or 2^30 segments");
    if (n_segs > 0 && n_nodes == 0) return set_error(DD_EINVAL, "segments without nodes");
    if (n_gauss < 1 || n_gauss > DD_MAX_GAUSS) return set_error(DD_EINVAL, "n_gauss must be in 1..16");
    if (precision != DD_FP64 && precision != DD_MIXED) return set_error(DD_EINVAL, "unknown precision");
    // at least one core width: a segment's own Gauss points then always take the
    // FP64 branch of the mixed kernel, which skips the self pair
    if (precision == DD_MIXED && !(near_cut >= 1.0)) return set_error(DD_EINVAL, "near_cutoff_a must be >= 1");
    return DD_OK;
}

// ------------------------------------------------------- instance tables --
// Segment -> instance and the device copies of the offsets, uploaded only
// when the offsets differ from the last upload (an upload synchronises).
int instance_tables(Workspace *ws, const std::vector<int64_t> &no, const std::vector<int64_t> &so, Layout &inst,
                    hipStream_t st)
{
    const int n_inst = (int)so.size() - 1;
    const int64_t ns = so.back();
    std::vector<int64_t> key(no);
    key.insert(key.end(), so.begin(), so.end());
    int rc;
    if (key != ws->inst_key || !ws->ptr[WS_SEG_INST] || !ws->ptr[WS_INST_OFFS]) {
        std::vector<int32_t> si((size_t)std::max<int64_t>(ns, 1), 0);
        for (int i = 0; i < n_inst; ++i)
            for (int64_t s = so[i]; s < so[i + 1]; ++s) si[s] = i;
        int32_t *d_si;
        if ((rc = upload(ws, WS_SEG_INST, si, &d_si, st))) return rc;
        int64_t *d_offs;
        if ((rc = upload(ws, WS_INST_OFFS, key, &d_offs, st))) return rc;
        ws->inst_key = key;
    }
    inst.seg_inst = (const int32_t *)ws->ptr[WS_SEG_INST];
    inst.node_off = (const int64_t *)ws->ptr[WS_INST_OFFS];
    inst.seg_off = inst.node_off + (n_inst + 1);
    return DD_OK;
}

// ------------------------------------------------------------ step graphs --
struct KeyBuf {
    std::vector<unsigned char> b;
    template <class T>
    KeyBuf &add(const T &v)
    {
        const unsigned char *p = reinterpret_cast<const unsigned char *>(&v);
        b.insert(b.end(), p, p + sizeof(T));
        return *this;
    }
    template <class T>
    KeyBuf &add_vec(const std::vector<T> &v)
    {
        add(v.size());
        const unsigned char *p = reinterpret_cast<const unsigned char *>(v.data());
        b.insert(b.end(), p, p + v.size() * sizeof(T));
        return *this;
    }
    // every workspace address a captured kernel can be handed
    KeyBuf &add_workspace(const Workspace *ws)
    {
        for (int s = 0; s < WS_NSLOTS; ++s) add(ws->ptr[s]);
        return add(ws->flags_dev);
    }
};

// Launches on st the graph cached under `key`, or records one with
// record(capture_stream), instantiates it, caches it and launches it.  No
// synchronisation unless a cached graph has to be evicted.
template <class F>
int launch_cached_graph(Workspace *ws, const KeyBuf &key, F &&record, hipStream_t st)
{
    for (auto &g : ws->graphs)
        if (g.key == key.b) {
            g.last_use = ++ws->graph_clock;
            DD_HIP(hipGraphLaunch(g.exec, st));
            return DD_OK;
        }
    Range range_("dd graph capture");
    if (!ws->capture_stream) DD_HIP(hipStreamCreateWithFlags(&ws->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = ws->capture_stream;
    DD_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    ws->capturing = true;
    const int rc = record(cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    ws->capturing = false;
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return set_error(DD_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return set_error(DD_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    if (ws->graphs.size() >= GRAPH_CACHE) {
        size_t lru = 0;
        for (size_t k = 1; k < ws->graphs.size(); ++k)
            if (ws->graphs[k].last_use < ws->graphs[lru].last_use) lru = k;
        DD_HIP(hipDeviceSynchronize());   // it may still be running
        (void)hipGraphExecDestroy(ws->graphs[lru].exec);
        ws->graphs.erase(ws->graphs.begin() + (std::ptrdiff_t)lru);
    }
    ws->graphs.push_back(GraphEntry{key.b, exec, ++ws->graph_clock});
    DD_HIP(hipGraphLaunch(exec, st));
    return DD_OK;
}

// Before a captured burst with the exact band: a pair store of twice the
// current near-pair count plus 8 per segment (count pass, one
// synchronisation).  Done whenever validation is on (the call synchronises
// anyway) and, with validation off, only while the store is still empty, so
// that repeated asynchronous calls stay asynchronous; a step whose pairs
// outgrow the store raises FLAG_NEAR_FULL.
int presize_near(ForceCtx &C, Workspace *ws, const double *x, const int32_t *seg_nodes, hipStream_t st)
{
    if (!C.near_on) return DD_OK;
    if (!validation_on() && C.near.pair_t) return DD_OK;
    return size_near_pairs(C, ws, x, seg_nodes, 2.0, 8, st);
}

}  // namespace

// ------------------------------------------------ bursts of an active subset --
int burst_batch_init(BurstBatch &B, hipStream_t st)
{
    int rc;
    const int n_inst = B.n_inst;
    const int64_t nn = B.node_off[n_inst];
    Workspace *ws;
    if ((rc = workspace(&ws))) return rc;
    Layout inst{};
    if ((rc = instance_tables(ws, B.node_off, B.seg_off, inst, st))) return rc;
    return tuned_chunk(ws, st, B.seg_off, nn, inst, B.seg_nodes, B.x, B.burgers, B.normal, &B.mat, B.n_gauss,
                       B.precision, B.near_cut, true, &B.choice);
}

int burst_batch_run(const BurstBatch &B, const std::vector<uint8_t> &active, const double *sigma_dev,
                    int n_steps, double *sums_dev, hipStream_t st)
{
    int rc;
    const int n_inst = B.n_inst;
    const int64_t nn = B.node_off[n_inst], ns = B.seg_off[n_inst];
    if (n_steps <= 0 || ns == 0) return DD_OK;
    bool any = false;
    for (int i = 0; i < n_inst; ++i) any = any || (active[i] && B.seg_off[i + 1] > B.seg_off[i]);
    if (!any) return DD_OK;
    Workspace *ws;
    if ((rc = workspace(&ws))) return rc;
    Layout inst{};
    if ((rc = instance_tables(ws, B.node_off, B.seg_off, inst, st))) return rc;
    ForceCtx C;
    if ((rc = setup(ws, st, B.seg_off, nn, B.seg_nodes, &B.mat, B.n_gauss, B.precision, B.near_cut, B.eta,
                    B.choice / MIXED_VARIANTS, true, C, &active)))
        return rc;
    C.variant = (int)(B.choice % MIXED_VARIANTS);
    g_last_variant = C.variant;
    C.L.seg_inst = inst.seg_inst;
    C.L.node_off = inst.node_off;
    C.L.seg_off = inst.seg_off;
    uint8_t *d_act;
    if ((rc = upload(ws, WS_ACTIVE, active, &d_act, st))) return rc;
    void *p;
    if ((rc = ensure(ws, WS_VEL, sizeof(double) * 3 * std::max<int64_t>(nn, 1), &p))) return rc;
    double *vel = (double *)p;
    if ((rc = ensure(ws, WS_FORCE, sizeof(double) * 3 * std::max<int64_t>(nn, 1), &p))) return rc;
    double *F = (double *)p;
    launch_csr(C, B.seg_nodes, st);
    uint8_t *held = nullptr;
    JunctionArgs J{};
    if (B.jn && (rc = junction_prepare(ws, C.L, B.seg_nodes, B.x, B.pinned, B.jn, J, &held, st))) return rc;
    // (the PTA path times junctions by the per-instance fast clock; t0 is
    // never read there, but points at valid memory all the same)
    if ((rc = ensure(ws, WS_T0, sizeof(double), &p))) return rc;
    J.t0 = (const double *)p;
    // junction nodes, timed by the per-instance fast clock
    JNodeArgs JN{};
    if (B.jnodes) {
        if ((rc = jnode_prepare(ws, C.L, B.seg_nodes, B.x, B.pinned, B.jnodes, JN, st))) return rc;
        JN.t0 = (const double *)p;
        JN.fast = B.fast_steps_dev;
        JN.fdt = B.dt;
    }
    if ((rc = presize_near(C, ws, B.x, B.seg_nodes, st))) return rc;
    DD_HIP(hipGetLastError());
    KeyBuf key;
    key.add('r').add(n_inst).add_vec(B.node_off).add_vec(B.seg_off).add_vec(active).add(B.x).add(B.seg_nodes);
    key.add(B.burgers).add(B.normal).add(B.volume).add(B.pinned).add(B.mat).add(B.n_gauss).add(B.precision);
    key.add(B.near_cut).add(B.eta).add(B.dt).add(B.choice).add(sigma_dev).add(sums_dev).add(n_steps);
    key.add(B.jn != nullptr).add(B.fast_steps_dev).add(C.near.pair_cap).add_workspace(ws);
    if (B.jn) key.add(*B.jn);
    key.add(B.jnodes != nullptr);
    if (B.jnodes) {
        dd_junction_nodes kj = *B.jnodes;
        kj.t0 = 0.0;
        key.add(kj);
    }
    const Sig6 sv{};
    rc = launch_cached_graph(ws, key, [&](hipStream_t cs) -> int {
        for (int k = 0; k < n_steps; ++k) {
            if (B.jnodes)
                launch_jnode_step(C, JN, 0.0, k, n_inst, B.seg_nodes_w, B.x, B.burgers_w, B.normal_w, ws->flags_dev,
                                  (const uint8_t *)d_act, cs);
            if (B.jn)
                hipLaunchKernelGGL(k_junctions, dim3(grid_for(nn, 256, INT32_MAX)), dim3(256), 0, cs, C.L,
                                   B.seg_nodes, (const double *)B.x, B.pinned, J, n_inst, (const uint8_t *)d_act,
                                   B.fast_steps_dev, B.dt, k, held);
            const int r = launch_forces(C, ws, B.x, B.seg_nodes, B.burgers, B.normal, sigma_dev, sv, F, cs, false);
            if (r) return r;
            hipLaunchKernelGGL(k_glide<true>, dim3(grid_for(nn, 256, INT32_MAX)), dim3(256), 0, cs, C.L,
                               C.csr_ptr, C.csr_list, B.seg_nodes, B.normal, C.rec64, C.a, B.x, F, B.pinned,
                               (const uint8_t *)held, (const uint8_t *)d_act, 1.0 / B.mat.B, B.dt, vel);
            hipLaunchKernelGGL(k_instance_sums, dim3(n_inst), dim3(256), 0, cs, C.L, 2, B.seg_nodes, C.rec64,
                               C.sys, vel, B.pinned, B.volume, sigma_dev, C.a, sums_dev);
        }
        return DD_OK;
    }, st);
    if (rc) return rc;
    DD_HIP(hipGetLastError());
    return DD_OK;
}

}  // namespace dd

using namespace dd;

extern "C" int dd_set_autotune(int on) { return dd::g_autotune.exchange(on ? 1 : 0); }

extern "C" int dd_set_burst_mode(int mode)
{
    clear_error();
    if (mode < 0 || mode > 2) return set_error(DD_EINVAL, "burst mode must be 0, 1 or 2");
    return dd::g_burst_mode.exchange(mode);
}

extern "C" int dd_check(void *stream)
{
    clear_error();
    Workspace *ws;
    int rc;
    if ((rc = workspace(&ws))) return rc;
    return read_flags(ws, (hipStream_t)stream);
}

extern "C" int dd_set_plan(int64_t chunk_len, int variant)
{
    dd::clear_error();
    if (chunk_len < 0) {
        dd::g_forced_choice.store(-1);
        return DD_OK;
    }
    if (chunk_len != 0 && chunk_len < MIN_CHUNK_LEN)
        return dd::set_error(DD_EINVAL, "chunk_len must be 0 (heuristic) or at least %d", MIN_CHUNK_LEN);
    if (variant < 0 || variant >= MIXED_VARIANTS) return dd::set_error(DD_EINVAL, "variant must be 0, 1 or 2");
    dd::g_forced_choice.store(MIXED_VARIANTS * chunk_len + variant);
    return DD_OK;
}

extern "C" int dd_last_plan(int64_t *chunk_len, int64_t *n_items, int *variant)
{
    if (chunk_len) *chunk_len = g_plan_chunk;
    if (n_items) *n_items = g_plan_items;
    if (variant) *variant = g_last_variant;
    return DD_OK;
}

extern "C" int dd_nodal_forces(int64_t n_nodes, const double *x, int64_t n_segs,
                               const int32_t *seg_nodes, const double *burgers,
                               const double *normal, const double *sigma_app,
                               const dd_material *m, int n_gauss, int precision,
                               double near_cutoff_a, double exact_eta, double *force_out, void *stream)
{
    ::dd::Range range_("dd_nodal_forces");
    clear_error();
    int rc;
    if ((rc = common_checks(n_nodes, n_segs, n_gauss, precision, near_cutoff_a, exact_eta))) return rc;
    if ((rc = check_material(m, false))) return rc;
    if (!sigma_app) return set_error(DD_EINVAL, "sigma_app is null");
    if (n_nodes > 0 && (!x || !force_out)) return set_error(DD_EINVAL, "null x or force_out");
    if (n_segs > 0 && (!seg_nodes || !burgers || !normal)) return set_error(DD_EINVAL, "null segment array");
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(sigma_app[k])) return set_error(DD_EINVAL, "non-finite sigma_app");
    if (n_nodes == 0) return DD_OK;
    hipStream_t st = (hipStream_t)stream;
    Workspace *ws;
    if ((rc = workspace(&ws))) return rc;
    ForceCtx C;
    std::vector<int64_t> so = {0, n_segs};
    int64_t choice = 0;
    Layout flat{};
    if ((rc = tuned_chunk(ws, st, so, n_nodes, flat, seg_nodes, x, burgers, normal, m, n_gauss, precision,
                          near_cutoff_a, false, &choice)))
        return rc;
    if ((rc = setup(ws, st, so, n_nodes, seg_nodes, m, n_gauss, precision, near_cutoff_a, exact_eta,
                    choice / MIXED_VARIANTS, false, C)))
        return rc;
    C.variant = (int)(choice % MIXED_VARIANTS);
    g_last_variant = C.variant;
    launch_csr(C, seg_nodes, st);
    Sig6 sv;
    for (int k = 0; k < 6; ++k) sv.v[k] = sigma_app[k];
    if ((rc = launch_forces(C, ws, x, seg_nodes, burgers, normal, nullptr, sv, force_out, st, true))) return rc;
    DD_HIP(hipGetLastError());
    if (validation_on()) {
        hipLaunchKernelGGL(k_check_finite, dim3(grid_for(3 * n_nodes)), dim3(256), 0, st, force_out,
                           3 * n_nodes, ws->flags_dev);
        return read_flags(ws, st);
    }
    return DD_OK;
}

extern "C" int dd_glide_step(int64_t n_nodes, double *x, const double *force, int64_t n_segs,
                             const int32_t *seg_nodes, const double *normal, const uint8_t *pinned,
                             const dd_material *m, double dt, double *vel_out, void *stream)
{
    ::dd::Range range_("dd_glide_step");
    clear_error();
    int rc;
    if ((rc = common_checks(n_nodes, n_segs, 1, DD_FP64, 1.0))) return rc;
    if (!m || !(m->B > 0.0) || !std::isfinite(m->B)) return set_error(DD_EINVAL, "drag B must be > 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(DD_EINVAL, "dt must be > 0");
    if (n_nodes > 0 && (!x || !force)) return set_error(DD_EINVAL, "null x or force");
    if (n_segs > 0 && (!seg_nodes || !normal)) return set_error(DD_EINVAL, "null segment array");
    if (n_nodes == 0) return DD_OK;
    hipStream_t st = (hipStream_t)stream;
    Workspace *ws;
    if ((rc = workspace(&ws))) return rc;
    Layout L{};
    L.nn = n_nodes;
    L.ns = n_segs;
    void *p;
    if ((rc = ensure(ws, WS_CSR_PTR, sizeof(int32_t) * (n_nodes + 1), &p))) return rc;
    ForceCtx C;
    C.L = L;
    C.csr_ptr = (int32_t *)p;
    if ((rc = ensure(ws, WS_CSR_LIST, sizeof(int32_t) * std::max<int64_t>(2 * n_segs, 1), &p))) return rc;
    C.csr_list = (int32_t *)p;
    if ((rc = ensure(ws, WS_CSR_CNT, sizeof(int32_t) * (n_nodes + scan_scratch_len(n_nodes)), &p))) return rc;
    C.csr_cnt = (int32_t *)p;
    C.scan_tmp = C.csr_cnt + n_nodes;
    double *vel = vel_out;
    if (!vel) {
        if ((rc = ensure(ws, WS_VEL, sizeof(double) * 3 * n_nodes, &p))) return rc;
        vel = (double *)p;
    }
    launch_csr(C, seg_nodes, st);
    if (validation_on() && n_segs > 0) {
        // index and normal checks (the prep kernel also computes lengths)
        if ((rc = ensure(ws, WS_SEG64, rec64_bytes(n_segs), &p))) return rc;
        PrepArgs A{};
        A.L = L;
        A.x = x;
        A.seg_nodes = seg_nodes;
        A.burgers = normal;   // any [3][n_segs] array: only the checks matter here
        A.normal = normal;
        A.inv_a = 1.0;
        A.rec64 = (double *)p;
        A.flags = ws->flags_dev;
        hipLaunchKernelGGL(k_seg_prep, dim3(grid_for(n_segs, PREP_BLOCK, INT32_MAX)), dim3(PREP_BLOCK), 0, st, A);
    }
    hipLaunchKernelGGL(k_glide<false>, dim3(grid_for(n_nodes, 256, INT32_MAX)), dim3(256), 0, st, L,
                       C.csr_ptr, C.csr_list, seg_nodes, normal, (const double *)nullptr, 1.0, x, force,
                       pinned, (const uint8_t *)nullptr, (const uint8_t *)nullptr, 1.0 / m->B, dt, vel);
    hipLaunchKernelGGL(k_euler, dim3(grid_for(3 * n_nodes, 256, INT32_MAX)), dim3(256), 0, st, n_nodes, x,
                       vel, dt);
    DD_HIP(hipGetLastError());
    if (validation_on()) {
        hipLaunchKernelGGL(k_check_finite, dim3(grid_for(3 * n_nodes)), dim3(256), 0, st, x, 3 * n_nodes,
                           ws->flags_dev);
        return read_flags(ws, st);
    }
    return DD_OK;
}

extern "C" int dd_step(int64_t n_nodes, double *x, int64_t n_segs, const int32_t *seg_nodes,
                       const double *burgers, const double *normal, const uint8_t *pinned,
                       const double *sigma_app, const dd_material *m, int n_gauss, int precision,
                       double near_cutoff_a, double exact_eta, double dt, double *force_out, double *vel_out,
                       void *stream)
{
    ::dd::Range range_("dd_step");
    clear_error();
    int rc;
    if ((rc = common_checks(n_nodes, n_segs, n_gauss, precision, near_cutoff_a, exact_eta))) return rc;
    if ((rc = check_material(m, true))) return rc;
    if (!sigma_app) return set_error(DD_EINVAL, "sigma_app is null");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(DD_EINVAL, "dt must be > 0");
    if (n_nodes > 0 && !x) return set_error(DD_EINVAL, "null x");
    if (n_segs > 0 && (!seg_nodes || !burgers || !normal)) return set_error(DD_EINVAL, "null segment array");
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(sigma_app[k])) return set_error(DD_EINVAL, "non-finite sigma_app");
    if (n_nodes == 0) return DD_OK;
    hipStream_t st = (hipStream_t)stream;
    Workspace *ws;
    if ((rc = workspace(&ws))) return rc;
    ForceCtx C;
    std::vector<int64_t> so = {0, n_segs};
    int64_t choice = 0;
    Layout flat{};
    if ((rc = tuned_chunk(ws, st, so, n_nodes, flat, seg_nodes, x, burgers, normal, m, n_gauss, precision,
                          near_cutoff_a, false, &choice)))
        return rc;
    if ((rc = setup(ws, st, so, n_nodes, seg_nodes, m, n_gauss, precision, near_cutoff_a, exact_eta,
                    choice / MIXED_VARIANTS, false, C)))
        return rc;
    C.variant = (int)(choice % MIXED_VARIANTS);
    g_last_variant = C.variant;
    void *p;
    double *F = force_out, *vel = vel_out;
    if (!F) {
        if ((rc = ensure(ws, WS_FORCE, sizeof(double) * 3 * n_nodes, &p))) return rc;
        F = (double *)p;
    }
    if (!vel) {
        if ((rc = ensure(ws, WS_VEL, sizeof(double) * 3 * n_nodes, &p))) return rc;
        vel = (double *)p;
    }
    launch_csr(C, seg_nodes, st);
    Sig6 sv;
    for (int k = 0; k < 6; ++k) sv.v[k] = sigma_app[k];
    if ((rc = launch_forces(C, ws, x, seg_nodes, burgers, normal, nullptr, sv, F, st, true))) return rc;
    // lengths from the segment records of this force pass: x can move in the same kernel
    hipLaunchKernelGGL(k_glide<true>, dim3(grid_for(n_nodes, 256, INT32_MAX)), dim3(256), 0, st, C.L, C.csr_ptr,
                       C.csr_list, seg_nodes, normal, (const double *)C.rec64, C.a, x, (const double *)F, pinned,
                       (const uint8_t *)nullptr, (const uint8_t *)nullptr, 1.0 / m->B, dt, vel);
    DD_HIP(hipGetLastError());
    if (validation_on()) {
        hipLaunchKernelGGL(k_check_finite, dim3(grid_for(3 * n_nodes)), dim3(256), 0, st, (const double *)F,
                           3 * n_nodes, ws->flags_dev);
        hipLaunchKernelGGL(k_check_finite, dim3(grid_for(3 * n_nodes)), dim3(256), 0, st, (const double *)x,
                           3 * n_nodes, ws->flags_dev);
        return read_flags(ws, st);
    }
    return DD_OK;
}

namespace dd {
namespace {
// The persistent kernel for a batch of small FP64 bursts, when every
// instance fits (at most PB_MAX_SEGS segments and nodes) and all the
// workgroups fit on the device at once; *used = false leaves the call to the
// step graph.  G_i: about PB_NODES_PER_WG nodes per workgroup, at most
// PB_MAX_G; one workgroup per instance in burst mode 2.  The node lists must
// be built.
int launch_persistent(const ForceCtx &C, Workspace *ws, const std::vector<int64_t> &no,
                      const std::vector<int64_t> &so, double *x, const int32_t *seg_nodes, const double *burgers,
                      const double *normal, const uint8_t *pinned, const double *sigma_app, const double *volume,
                      const dd_material *m, int n_steps, double dt, double *rate_avg_out, hipStream_t st,
                      bool *used)
{
    *used = false;
    const int mode = g_burst_mode.load();
    if (mode == 1) return DD_OK;
    const int n_inst = (int)no.size() - 1;
    for (int i = 0; i < n_inst; ++i)
        if (no[i + 1] - no[i] > PB_MAX_SEGS || so[i + 1] - so[i] > PB_MAX_SEGS) return DD_OK;
    int per_cu = 0, cus = 0;
    DD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_burst_persistent, PB_THREADS, 0));
    DD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ws->device));
    const int64_t cap = (int64_t)per_cu * cus;
    if (n_inst > cap) return DD_OK;
    std::vector<int> G(n_inst);
    int64_t total = 0;
    for (int i = 0; i < n_inst; ++i) {
        const int64_t want = (no[i + 1] - no[i] + PB_NODES_PER_WG - 1) / PB_NODES_PER_WG;
        G[i] = mode == 2 ? 1 : (int)std::max<int64_t>(1, std::min<int64_t>(want, PB_MAX_G));
        total += G[i];
    }
    // with fewer workgroups each would carry more nodes, and the step graph is
    // then the faster of the two (measured): only a batch that fits as split
    if (total > cap) return DD_OK;
    const int n_wg = (int)total;
    std::vector<int32_t> tab(4 * (size_t)n_wg);
    for (int i = 0, k = 0; i < n_inst; ++i) {
        const int first = k;
        for (int w = 0; w < G[i]; ++w, ++k) {
            tab[k] = i;
            tab[n_wg + k] = w;
            tab[2 * n_wg + k] = G[i];
            tab[3 * n_wg + k] = first;
        }
    }
    const int64_t nn = no.back();
    void *p;
    int rc;
    if ((rc = ensure(ws, WS_PB, sizeof(double) * (9 * (size_t)std::max<int64_t>(nn, 1) + 12 * (size_t)n_wg), &p)))
        return rc;
    double *xb = (double *)p, *vel2 = xb + 3 * std::max<int64_t>(nn, 1), *wpart = vel2 + 6 * std::max<int64_t>(nn, 1);
    int32_t *wgtab = (int32_t *)ws->ptr[WS_PB_INT];
    if (tab != ws->pb_tab || !wgtab) {   // uploaded (one synchronisation) only when the table changes
        if ((rc = upload(ws, WS_PB_INT, tab, &wgtab, st))) return rc;
        ws->pb_tab = tab;
    }
    // barrier arrival words, zeroed on the stream
    void *pb;
    if ((rc = ensure(ws, WS_PB_BAR, sizeof(unsigned) * 16 * (size_t)n_wg, &pb))) return rc;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(16 * (int64_t)n_wg)), dim3(256), 0, st, (unsigned *)pb,
                       16 * (int64_t)n_wg, 0u);
    PBArgs A{};
    A.L = C.L;
    A.seg_nodes = seg_nodes;
    A.burgers = burgers;
    A.normal = normal;
    A.pinned = pinned;
    A.sigma_app = sigma_app;
    A.volume = volume;
    A.csr_ptr = C.csr_ptr;
    A.csr_list = C.csr_list;
    A.wg = wgtab;
    A.n_wg = n_wg;
    A.xa = x;
    A.xb = xb;
    A.vel = vel2;
    A.wpart = wpart;
    A.arrive = (unsigned *)pb;
    A.flags = ws->flags_dev;
    A.rate_out = rate_avg_out;
    A.g = C.g;
    A.kr = C.k1 / C.k2;
    A.nu = 1.0 - 2.0 * A.kr;
    A.k2 = C.k2;
    A.inv_a = C.inv_a;
    A.a = C.a;
    A.inv_mu = C.inv_mu;
    A.fscale = C.fscale;
    A.invB = 1.0 / m->B;
    A.dt = dt;
    A.n_steps = n_steps;
    void *args[] = {&A};
    const hipError_t e = hipLaunchCooperativeKernel((const void *)k_burst_persistent, dim3((unsigned)n_wg),
                                                    dim3(PB_THREADS), args, 0, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // not launched: the step graph runs instead
        return DD_OK;
    }
    *used = true;
    return DD_OK;
}

int burst_batch_impl(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                     const int32_t *seg_nodes, const double *burgers, const double *normal, const uint8_t *pinned,
                     const double *sigma_app, const double *volume, const dd_material *m, int n_gauss, int precision,
                     double near_cutoff_a, double exact_eta, int n_steps, double dt, const dd_junctions *jn,
                     double *rate_avg_out, double *features_out, void *stream,
                     const dd_junction_nodes *jnodes = nullptr)
{
    int rc;
    if (n_inst < 0) return set_error(DD_EINVAL, "n_inst < 0");
    if (n_inst == 0) return DD_OK;
    if (!node_off || !seg_off) return set_error(DD_EINVAL, "null offsets");
    if (node_off[0] != 0 || seg_off[0] != 0) return set_error(DD_EINVAL, "offsets must start at 0");
    for (int i = 0; i < n_inst; ++i)
        if (node_off[i + 1] < node_off[i] || seg_off[i + 1] < seg_off[i])
            return set_error(DD_EINVAL, "offsets must be non-decreasing");
    for (int i = 0; i < n_inst; ++i)
        if (seg_off[i + 1] > seg_off[i] && node_off[i + 1] == node_off[i])
            return set_error(DD_EINVAL, "instance %d has segments but no nodes", i);
    const int64_t nn = node_off[n_inst], ns = seg_off[n_inst];
    if ((rc = common_checks(nn, ns, n_gauss, precision, near_cutoff_a, exact_eta))) return rc;
    if ((rc = check_material(m, true))) return rc;
    if (n_steps < 0) return set_error(DD_EINVAL, "n_steps < 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(DD_EINVAL, "dt must be > 0");
    if (!sigma_app || !volume || !rate_avg_out) return set_error(DD_EINVAL, "null sigma_app, volume or rate_avg_out");
    if (nn > 0 && !x) return set_error(DD_EINVAL, "null x");
    if (ns > 0 && (!seg_nodes || !burgers || !normal)) return set_error(DD_EINVAL, "null segment array");
    if (jn) {
        if (!(jn->capture_radius >= 0.0) || !std::isfinite(jn->capture_radius) || !(jn->max_break_time >= 0.0) ||
            !std::isfinite(jn->max_break_time) || !std::isfinite(jn->t0))
            return set_error(DD_EINVAL, "junctions: capture radius and breaking time must be finite and >= 0, t0 finite");
        if (jn->n_fractions < 1) return set_error(DD_EINVAL, "junctions: n_fractions must be >= 1");
        if (nn > 0 && (!jn->fractions || !jn->junction || !jn->release || !jn->ignore || !jn->count))
            return set_error(DD_EINVAL, "junctions: null state or fractions array");
    }
    if (jnodes) {
        const dd_junction_nodes *J = jnodes;
        if (!(J->capture_radius >= 0.0) || !std::isfinite(J->capture_radius) || !(J->max_break_time >= 0.0) ||
            !std::isfinite(J->max_break_time) || !std::isfinite(J->t0) || !(J->min_length >= 0.0) ||
            !std::isfinite(J->min_length))
            return set_error(DD_EINVAL, "junction nodes: capture radius, breaking time and min_length must be "
                                        "finite and >= 0, t0 finite");
        if (J->n_slots < 1 || J->n_fractions < 1)
            return set_error(DD_EINVAL, "junction nodes: n_slots and n_fractions must be >= 1");
        if (!J->fractions || !J->release || !J->ses || !J->ignore || !J->point || !J->count || !J->missed)
            return set_error(DD_EINVAL, "junction nodes: null state or fractions array");
        if (exact_eta != 0.0) return set_error(DD_EINVAL, "junction nodes: no exact band (exact_eta must be 0)");
        for (int i = 0; i < n_inst; ++i)
            if (node_off[i + 1] - node_off[i] < (int64_t)J->n_slots + 2 || seg_off[i + 1] - seg_off[i] < J->n_slots)
                return set_error(DD_EINVAL, "junction nodes: instance %d has fewer than n_slots + 2 nodes or n_slots "
                                            "segments", i);
    }
    hipStream_t st = (hipStream_t)stream;
    Workspace *ws;
    if ((rc = workspace(&ws))) return rc;

    std::vector<int64_t> so(seg_off, seg_off + n_inst + 1), no(node_off, node_off + n_inst + 1);
    Layout inst{};
    if ((rc = instance_tables(ws, no, so, inst, st))) return rc;
    ForceCtx C;
    int64_t choice = 0;
    if ((rc = tuned_chunk(ws, st, so, nn, inst, seg_nodes, x, burgers, normal, m, n_gauss, precision,
                          near_cutoff_a, true, &choice)))
        return rc;
    if ((rc = setup(ws, st, so, nn, seg_nodes, m, n_gauss, precision, near_cutoff_a, exact_eta,
                    choice / MIXED_VARIANTS, true, C)))
        return rc;
    C.variant = (int)(choice % MIXED_VARIANTS);
    g_last_variant = C.variant;
    C.L.seg_inst = inst.seg_inst;
    C.L.node_off = inst.node_off;
    C.L.seg_off = inst.seg_off;
    C.L.tile_begin = (const int64_t *)ws->ptr[WS_OFFS];
    void *p;
    if ((rc = ensure(ws, WS_VEL, sizeof(double) * 3 * std::max<int64_t>(nn, 1), &p))) return rc;
    double *vel = (double *)p;
    if ((rc = ensure(ws, WS_FORCE, sizeof(double) * 3 * std::max<int64_t>(nn, 1), &p))) return rc;
    double *F = (double *)p;
    uint8_t *held = nullptr;
    if ((rc = ensure(ws, WS_T0, sizeof(double), &p))) return rc;
    double *t0_dev = (double *)p;
    JunctionArgs J{};
    if (jn && (rc = junction_prepare(ws, C.L, seg_nodes, x, pinned, jn, J, &held, st))) return rc;
    J.t0 = t0_dev;
    JNodeArgs JN{};
    if (jnodes && (rc = jnode_prepare(ws, C.L, seg_nodes, x, pinned, jnodes, JN, st))) return rc;
    JN.t0 = t0_dev;

    launch_csr(C, seg_nodes, st);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(12 * (int64_t)n_inst)), dim3(256), 0, st, rate_avg_out,
                       12 * (int64_t)n_inst, 0.0);
    Sig6 sv{};
    // features of the initial state
    if (features_out && ns > 0) {
        PrepArgs A;
        A.L = C.L;
        A.x = x;
        A.seg_nodes = seg_nodes;
        A.burgers = burgers;
        A.normal = normal;
        A.inv_a = C.inv_a;
        A.rec64 = C.rec64;
        A.rec32 = C.rec32;
        A.cut = C.cut;
        A.quadn = C.precision == DD_MIXED ? quad_points(C.variant) : 0;
        A.sys = C.sys;
        A.flags = ws->flags_dev;
        hipLaunchKernelGGL(k_seg_prep, dim3(grid_for(ns, PREP_BLOCK, INT32_MAX)), dim3(PREP_BLOCK), 0, st, A);
        hipLaunchKernelGGL(k_instance_sums, dim3(n_inst), dim3(256), 0, st, C.L, 1, seg_nodes, C.rec64, C.sys,
                           (const double *)nullptr, pinned, volume, sigma_app, C.a, features_out);
    } else if (features_out) {
        hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(36 * (int64_t)n_inst)), dim3(256), 0, st, features_out,
                           36 * (int64_t)n_inst, 0.0);
    }
    DD_HIP(hipGetLastError());

    // small FP64 bursts: every step in one persistent launch, when it fits
    bool persistent = false;
    if (n_steps > 0 && ns > 0 && !jn && !jnodes && exact_eta == 0.0 && precision == DD_FP64 &&
        (rc = launch_persistent(C, ws, no, so, x, seg_nodes, burgers, normal, pinned, sigma_app, volume, m, n_steps,
                                dt, rate_avg_out, st, &persistent)))
        return rc;
    if (persistent) {
        hipLaunchKernelGGL(k_scale_rates, dim3(grid_for(12 * (int64_t)n_inst, 256, INT32_MAX)), dim3(256), 0,
                           st, rate_avg_out, 12 * (int64_t)n_inst, 1.0 / n_steps);
    } else if (n_steps > 0 && ns > 0) {
        if ((rc = presize_near(C, ws, x, seg_nodes, st))) return rc;
        // the whole step loop as one graph, cached for calls with the same key
        KeyBuf key;
        key.add('b').add(n_inst).add_vec(no).add_vec(so).add(x).add(seg_nodes).add(burgers).add(normal);
        key.add(pinned).add(sigma_app).add(volume).add(*m).add(n_gauss).add(precision).add(near_cutoff_a);
        key.add(exact_eta).add(n_steps).add(dt).add(choice).add(rate_avg_out).add(jn != nullptr);
        key.add(C.near.pair_cap).add_workspace(ws);
        // the start time is not part of the key: the step kernels read it from
        // the device, where it is stored on the caller's stream before the
        // graph is launched, so that consecutive calls share one graph
        if (jn) {
            dd_junctions kj = *jn;
            kj.t0 = 0.0;
            key.add(kj);
        }
        key.add(jnodes != nullptr);
        if (jnodes) {
            dd_junction_nodes kj = *jnodes;
            kj.t0 = 0.0;
            key.add(kj);
        }
        if (jn || jnodes)
            hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, st, t0_dev, (int64_t)1, jn ? jn->t0 : jnodes->t0);
        rc = launch_cached_graph(ws, key, [&](hipStream_t cs) -> int {
            for (int k = 0; k < n_steps; ++k) {
                if (jnodes)   // (the public call passes these arrays as writable)
                    launch_jnode_step(C, JN, k * dt, k, n_inst, const_cast<int32_t *>(seg_nodes), x,
                                      const_cast<double *>(burgers), const_cast<double *>(normal), ws->flags_dev,
                                      nullptr, cs);
                if (jn) {
                    J.tk = k * dt;
                    hipLaunchKernelGGL(k_junctions, dim3(grid_for(nn, 256, INT32_MAX)), dim3(256), 0, cs, C.L,
                                       seg_nodes, (const double *)x, pinned, J, n_inst, (const uint8_t *)nullptr,
                                       (const int64_t *)nullptr, dt, k, held);
                }
                const int r = launch_forces(C, ws, x, seg_nodes, burgers, normal, sigma_app, sv, F, cs, false);
                if (r) return r;
                hipLaunchKernelGGL(k_glide<true>, dim3(grid_for(nn, 256, INT32_MAX)), dim3(256), 0, cs, C.L,
                                   C.csr_ptr, C.csr_list, seg_nodes, normal, C.rec64, C.a, x, F, pinned,
                                   (const uint8_t *)held, (const uint8_t *)nullptr, 1.0 / m->B, dt, vel);
                hipLaunchKernelGGL(k_instance_sums, dim3(n_inst), dim3(256), 0, cs, C.L, 0, seg_nodes, C.rec64,
                                   C.sys, vel, pinned, volume, sigma_app, C.a, rate_avg_out);
            }
            return DD_OK;
        }, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_scale_rates, dim3(grid_for(12 * (int64_t)n_inst, 256, INT32_MAX)), dim3(256), 0,
                           st, rate_avg_out, 12 * (int64_t)n_inst, 1.0 / n_steps);
    }
    DD_HIP(hipGetLastError());
    if (validation_on()) {
        hipLaunchKernelGGL(k_check_finite, dim3(grid_for(12 * (int64_t)n_inst)), dim3(256), 0, st,
                           rate_avg_out, 12 * (int64_t)n_inst, ws->flags_dev);
        if (nn > 0)
            hipLaunchKernelGGL(k_check_finite, dim3(grid_for(3 * nn)), dim3(256), 0, st, x, 3 * nn,
                               ws->flags_dev);
        return read_flags(ws, st);
    }
    return DD_OK;
}
}  // namespace
}  // namespace dd

extern "C" int dd_burst_batch(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                              const int32_t *seg_nodes, const double *burgers, const double *normal,
                              const uint8_t *pinned, const double *sigma_app, const double *volume,
                              const dd_material *m, int n_gauss, int precision, double near_cutoff_a,
                              double exact_eta, int n_steps, double dt, double *rate_avg_out,
                              double *features_out, void *stream)
{
    ::dd::Range range_("dd_burst_batch");
    clear_error();
    return burst_batch_impl(n_inst, node_off, seg_off, x, seg_nodes, burgers, normal, pinned, sigma_app, volume, m,
                            n_gauss, precision, near_cutoff_a, exact_eta, n_steps, dt, nullptr, rate_avg_out,
                            features_out, stream);
}

extern "C" int dd_burst_batch_junctions(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                                        const int32_t *seg_nodes, const double *burgers, const double *normal,
                                        const uint8_t *pinned, const double *sigma_app, const double *volume,
                                        const dd_material *m, int n_gauss, int precision, double near_cutoff_a,
                                        double exact_eta, int n_steps, double dt, const dd_junctions *junctions,
                                        double *rate_avg_out, double *features_out, void *stream)
{
    ::dd::Range range_("dd_burst_batch_junctions");
    clear_error();
    if (!junctions) return set_error(DD_EINVAL, "null junction parameters");
    return burst_batch_impl(n_inst, node_off, seg_off, x, seg_nodes, burgers, normal, pinned, sigma_app, volume, m,
                            n_gauss, precision, near_cutoff_a, exact_eta, n_steps, dt, junctions, rate_avg_out,
                            features_out, stream);
}

extern "C" int dd_burst_batch_junction_nodes(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off,
                                             double *x, int32_t *seg_nodes, double *burgers, double *normal,
                                             const uint8_t *pinned, const double *sigma_app, const double *volume,
                                             const dd_material *m, int n_gauss, int precision, double near_cutoff_a,
                                             int n_steps, double dt, const dd_junction_nodes *junctions,
                                             double *rate_avg_out, double *features_out, void *stream)
{
    ::dd::Range range_("dd_burst_batch_junction_nodes");
    clear_error();
    if (!junctions) return set_error(DD_EINVAL, "null junction-node parameters");
    return burst_batch_impl(n_inst, node_off, seg_off, x, seg_nodes, burgers, normal, pinned, sigma_app, volume, m,
                            n_gauss, precision, near_cutoff_a, 0.0, n_steps, dt, nullptr, rate_avg_out, features_out,
                            stream, junctions);
}

// ======================================================= no-allocation call --
// dd_nodal_forces_noalloc: dd_nodal_forces for callers that cannot allocate
// (code under graph capture, serving loops).  Every buffer the force pass
// needs beyond the caller's arrays comes from `scratch`, a file-scope device
// array of NOALLOC_BYTES that each GPU holds from the library's load until
// the process ends.  Host code never uses the array's name as an address:
// its device address is taken once per device with hipGetSymbolAddress.
namespace dd {
namespace {

constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};   // device address of `scratch` per device

int scratch_address(void **out)
{
    int dev = 0;
    DD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return set_error(DD_EINVAL, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(DD_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DD_OK;
}

// Tiles of TILE consecutive Gauss points of one volume and, per tile, C items
// over consecutive source ranges of chunk_len; item i = tile (i / C), range
// (i % C), partial slot i.
__global__ void k_plan_flat(Tile *tiles, Item *items, int64_t ns, int Q, int64_t chunk_len, int64_t n_tiles,
                            int64_t C)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_tiles * C) return;
    const int64_t t = i / C, c = i - t * C;
    Item it;
    it.tile = (int32_t)t;
    it.pad = 0;
    it.src_begin = c * chunk_len;
    it.src_end = min(ns, it.src_begin + chunk_len);
    it.slot = i;
    items[i] = it;
    if (c == 0) {
        Tile tl;
        tl.point_begin = t * TILE;
        tl.n_points = (int32_t)min((int64_t)TILE, ns * Q - t * TILE);
        tl.n_chunks = (int32_t)C;
        tl.slot_begin = t * C;
        tiles[t] = tl;
    }
}

// Carves the force pass's buffers out of the scratch array; returns the bytes
// needed in *need (whether or not they fit).
struct Carve {
    unsigned char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count)
    {
        T *p = reinterpret_cast<T *>(base + off);
        off += (count * sizeof(T) + 255) & ~size_t(255);
        return p;
    }
};

}  // namespace
}  // namespace dd

extern "C" int dd_nodal_forces_noalloc(int64_t n_nodes, const double *x, int64_t n_segs,
                                       const int32_t *seg_nodes, const double *burgers, const double *normal,
                                       const double *sigma_app, const dd_material *m, int n_gauss,
                                       int precision, double near_cutoff_a, double *force_out, void *stream)
{
    ::dd::Range range_("dd_nodal_forces_noalloc");
    clear_error();
    int rc;
    if ((rc = common_checks(n_nodes, n_segs, n_gauss, precision, near_cutoff_a))) return rc;
    if ((rc = check_material(m, false))) return rc;
    if (!sigma_app) return set_error(DD_EINVAL, "sigma_app is null");
    if (n_nodes > 0 && (!x || !force_out)) return set_error(DD_EINVAL, "null x or force_out");
    if (n_segs > 0 && (!seg_nodes || !burgers || !normal)) return set_error(DD_EINVAL, "null segment array");
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(sigma_app[k])) return set_error(DD_EINVAL, "non-finite sigma_app");
    // the work split: as dd_set_plan fixes it, else the built-in heuristic
    // (the autotuner would allocate and synchronise)
    const int64_t forced = g_forced_choice.load();
    const int64_t n_tiles = (n_segs * n_gauss + TILE - 1) / TILE;
    int64_t chunk_len = forced > 0 ? forced / MIXED_VARIANTS : 0;
    const int variant = forced >= 0 ? (int)(forced % MIXED_VARIANTS) : 0;
    if (chunk_len <= 0) chunk_len = heuristic_chunk(n_tiles, n_segs);
    const int64_t n_chunks = n_segs > 0 ? (n_segs + chunk_len - 1) / chunk_len : 0;
    const int64_t n_items = n_tiles * n_chunks;
    // what the pass needs, in the order it is carved below
    Carve sz{nullptr};
    sz.take<unsigned char>(256);                                   // flags word, mixed-kernel counters
    sz.take<double>((size_t)REC64_TOTAL * (size_t)std::max<int64_t>(n_segs, 1));
    if (precision == DD_MIXED) sz.take<float>((size_t)REC32A * (size_t)std::max<int64_t>(n_segs, 1));
    sz.take<double>(6 * (size_t)std::max<int64_t>(n_segs, 1));    // end forces
    sz.take<int32_t>((size_t)n_nodes + 1);                          // node lists: offsets
    sz.take<int32_t>(2 * (size_t)std::max<int64_t>(n_segs, 1));   //   entries
    sz.take<int32_t>((size_t)(std::max<int64_t>(n_nodes, 1) + scan_scratch_len(n_nodes)));   //   counters, scan
    sz.take<Tile>((size_t)std::max<int64_t>(n_tiles, 1));
    sz.take<Item>((size_t)std::max<int64_t>(n_items, 1));
    sz.take<double>(3 * (size_t)TILE * (size_t)std::max<int64_t>(n_items, 1));   // partial sums
    if (sz.off > NOALLOC_BYTES)
        return set_error(DD_ECAPACITY, "dd_nodal_forces_noalloc: this problem needs %zu bytes of scratch, more "
                         "than the %zu it has (%lld segments, %d Gauss points, %lld work items)", sz.off,
                         NOALLOC_BYTES, (long long)n_segs, n_gauss, (long long)n_items);
    if (n_nodes == 0) return DD_OK;
    void *base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    hipStream_t st = (hipStream_t)stream;
    Carve cv{(unsigned char *)base};
    Workspace ws;   // addresses only: nothing here is allocated
    ws.flags_dev = cv.take<unsigned>(64);
    ws.near_count = (unsigned long long *)(ws.flags_dev + 32);
    ws.capturing = true;   // no event timing (events would be created on first use)
    ForceCtx C;
    C.g = gauss_rule(n_gauss);
    C.k1 = 1.0 / (8.0 * M_PI);
    C.k2 = 1.0 / (4.0 * M_PI * (1.0 - m->nu));
    C.a = m->a;
    C.inv_a = 1.0 / m->a;
    C.inv_mu = 1.0 / m->mu;
    C.fscale = m->mu * m->a * m->a;
    C.precision = precision;
    C.variant = variant;
    C.cut = (float)near_cutoff_a;
    C.L.nn = n_nodes;
    C.L.ns = n_segs;
    C.rec64 = cv.take<double>((size_t)REC64_TOTAL * (size_t)std::max<int64_t>(n_segs, 1));
    if (precision == DD_MIXED) C.rec32 = cv.take<float>((size_t)REC32A * (size_t)std::max<int64_t>(n_segs, 1));
    C.segF = cv.take<double>(6 * (size_t)std::max<int64_t>(n_segs, 1));
    C.csr_ptr = cv.take<int32_t>((size_t)n_nodes + 1);
    C.csr_list = cv.take<int32_t>(2 * (size_t)std::max<int64_t>(n_segs, 1));
    C.csr_cnt = cv.take<int32_t>((size_t)(std::max<int64_t>(n_nodes, 1) + scan_scratch_len(n_nodes)));
    C.scan_tmp = C.csr_cnt + std::max<int64_t>(n_nodes, 1);
    C.tiles = cv.take<Tile>((size_t)std::max<int64_t>(n_tiles, 1));
    C.items = cv.take<Item>((size_t)std::max<int64_t>(n_items, 1));
    C.partial = cv.take<double>(3 * (size_t)TILE * (size_t)std::max<int64_t>(n_items, 1));
    C.n_items = n_items;
    if (n_items > 0)
        hipLaunchKernelGGL(k_plan_flat, dim3(grid_for(n_items, 256, INT32_MAX)), dim3(256), 0, st, C.tiles,
                           C.items, n_segs, n_gauss, chunk_len, n_tiles, n_chunks);
    launch_csr(C, seg_nodes, st);
    Sig6 sv;
    for (int k = 0; k < 6; ++k) sv.v[k] = sigma_app[k];
    if ((rc = launch_forces(C, &ws, x, seg_nodes, burgers, normal, nullptr, sv, force_out, st, false))) return rc;
    DD_HIP(hipGetLastError());
    return DD_OK;
}
