// The Practical Time Averaging (PTA) slow-time step for a batch of
// independent DD volumes (dd_pta_step): host control over the fast runs,
// which advance on the GPU chunk by chunk for the volumes that still need
// them (burst_batch_run).  Per-chunk sums come back to the host (13 doubles
// per volume); positions stay in device memory.
#include <cmath>
#include <type_traits>
#include <vector>

#include "dd_common.h"

namespace dd {
namespace {

__global__ void k_pta_fill(double *p, int64_t n, double v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_pta_flags(const double *__restrict__ p, int64_t n, unsigned *flags)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n && !isfinite(p[i])) atomicOr(flags, FLAG_NONFINITE);
}

// copies the node positions of the instances with mask[i] != 0 from src to dst
__global__ void k_copy_nodes(double *__restrict__ dst, const double *__restrict__ src, int64_t nn,
                             const int64_t *__restrict__ node_off, int n_inst, const uint8_t *__restrict__ mask)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nn) return;
    int lo = 0, hi = n_inst;   // node_off[lo] <= n < node_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (node_off[mid] <= n) lo = mid;
        else hi = mid;
    }
    if (!mask[lo]) return;
    for (int k = 0; k < 3; ++k) dst[k * nn + n] = src[k * nn + n];
}

// copies `comps` arrays of nn per-node values (stride nn) of the instances with
// mask[i] != 0 from src to dst
template <class T>
__global__ void k_copy_masked(T *__restrict__ dst, const T *__restrict__ src, int64_t nn, int comps,
                              const int64_t *__restrict__ node_off, int n_inst, const uint8_t *__restrict__ mask)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nn) return;
    int lo = 0, hi = n_inst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (node_off[mid] <= n) lo = mid;
        else hi = mid;
    }
    if (!mask[lo]) return;
    for (int k = 0; k < comps; ++k) dst[k * nn + n] = src[k * nn + n];
}

// copies per-instance values of the instances with mask[i] != 0
template <class T>
__global__ void k_copy_inst(T *__restrict__ dst, const T *__restrict__ src, int n_inst, const uint8_t *__restrict__ mask)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_inst && mask[i]) dst[i] = src[i];
}

// L^p = sum_alpha gdot_alpha m_alpha (x) n_alpha (row-major 3 x 3)
void lp_from_rates(const double *g, double Lp[9])
{
    for (int k = 0; k < 9; ++k) Lp[k] = 0.0;
    for (int al = 0; al < 12; ++al) {
        double n[3], m[3];
        fcc(al, n, m);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Lp[3 * r + c] += g[al] * m[r] * n[c];
    }
}

double frob(const double *a, int n)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += a[k] * a[k];
    return std::sqrt(s);
}

// running-average state of one fast run per instance
struct Runs {
    std::vector<double> sums;     // [n][13]
    std::vector<int64_t> steps;   // [n]
    std::vector<int> checks;      // [n]
    std::vector<uint8_t> conv;    // [n]
    std::vector<double> prev;     // [n][10]: rho, L^p of the previous check
    explicit Runs(int n) : sums(13 * (size_t)n, 0.0), steps(n, 0), checks(n, 0), conv(n, 0), prev(10 * (size_t)n, 0.0) {}
    void reset(int i)
    {
        for (int k = 0; k < 13; ++k) sums[13 * i + k] = 0.0;
        steps[i] = 0;
        checks[i] = 0;
        conv[i] = 0;
    }
    double rho(int i) const { return steps[i] ? sums[13 * i + 12] / steps[i] : 0.0; }
    void rates(int i, double g[12]) const
    {
        for (int k = 0; k < 12; ++k) g[k] = steps[i] ? sums[13 * i + k] / steps[i] : 0.0;
    }
    void lp(int i, double Lp[9]) const
    {
        double g[12];
        rates(i, g);
        lp_from_rates(g, Lp);
    }
};

struct Driver {
    BurstBatch &B;
    const dd_pta_params &P;
    hipStream_t st;
    Workspace *ws;
    double *sig_dev = nullptr, *sums_dev = nullptr;
    std::vector<double> sums_h;
    // junctions: per instance fast steps taken so far (host copy and device)
    std::vector<int64_t> fast;
    int64_t *fast_dev = nullptr;

    // one chunk of P.chunk_steps for the instances in `act` under `sigma`
    // (host [n][6]); the chunk sums are added to the runs of those instances
    int chunk(const std::vector<uint8_t> &act, const std::vector<double> &sigma, Runs &R)
    {
        const int n = B.n_inst;
        DD_HIP(hipMemcpyAsync(sig_dev, sigma.data(), sizeof(double) * 6 * n, hipMemcpyHostToDevice, st));
        if (fast_dev) DD_HIP(hipMemcpyAsync(fast_dev, fast.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_pta_fill, dim3((unsigned)((13 * (int64_t)n + 255) / 256)), dim3(256), 0, st, sums_dev,
                           13 * (int64_t)n, 0.0);
        int rc = burst_batch_run(B, act, sig_dev, P.chunk_steps, sums_dev, st);
        if (rc) return rc;
        DD_HIP(hipMemcpyAsync(sums_h.data(), sums_dev, sizeof(double) * 13 * n, hipMemcpyDeviceToHost, st));
        DD_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < n; ++i) {
            if (!act[i]) continue;
            for (int k = 0; k < 13; ++k) R.sums[13 * i + k] += sums_h[13 * i + k];
            R.steps[i] += P.chunk_steps;
            R.checks[i] += 1;
            if (fast_dev) fast[i] += P.chunk_steps;
        }
        return DD_OK;
    }

    // fast runs of the instances in `who` until their running averages of rho
    // and L^p converge (from the second check on) or max_chunks checks
    int fast_run(const std::vector<uint8_t> &who, const std::vector<double> &sigma, Runs &R)
    {
        const int n = B.n_inst;
        std::vector<uint8_t> act(who);
        for (;;) {
            bool any = false;
            for (int i = 0; i < n; ++i) any = any || act[i];
            if (!any) return DD_OK;
            int rc = chunk(act, sigma, R);
            if (rc) return rc;
            for (int i = 0; i < n; ++i) {
                if (!act[i]) continue;
                double Lp[9];
                R.lp(i, Lp);
                const double rho = R.rho(i);
                double *pv = &R.prev[10 * i];
                if (R.checks[i] >= 2) {
                    double dL[9];
                    for (int k = 0; k < 9; ++k) dL[k] = Lp[k] - pv[1 + k];
                    if (std::fabs(rho - pv[0]) <= P.tol_rho * std::fabs(rho) &&
                        frob(dL, 9) <= P.tol_lp * frob(Lp, 9)) {
                        R.conv[i] = 1;
                        act[i] = 0;
                    }
                }
                pv[0] = rho;
                for (int k = 0; k < 9; ++k) pv[1 + k] = Lp[k];
                if (R.checks[i] >= P.max_chunks) act[i] = 0;
            }
        }
    }

    int copy_nodes(double *dst, const double *src, const std::vector<uint8_t> &mask)
    {
        const int n = B.n_inst;
        const int64_t nn = B.node_off[n];
        if (nn == 0) return DD_OK;
        uint8_t *d_mask;
        int rc = upload_mask(mask, &d_mask);
        if (rc) return rc;
        hipLaunchKernelGGL(k_copy_nodes, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, dst, src, nn,
                           (const int64_t *)ws->ptr[WS_INST_OFFS], n, (const uint8_t *)d_mask);
        DD_HIP(hipGetLastError());
        return DD_OK;
    }

    // Junction-node state and topology of the masked instances (saved layout:
    // release [nn], burgers, normal, point [3][ns] doubles, then ses [nn],
    // seg_nodes [2][ns], ignore [ns], count, missed [n_inst] int32).
    int node_state(double *buf, const std::vector<uint8_t> &mask, bool to_save)
    {
        const int n = B.n_inst;
        const int64_t nn = B.node_off[n], ns = B.seg_off[n];
        uint8_t *d_mask;
        int rc = upload_mask(mask, &d_mask);
        if (rc) return rc;
        const dd_junction_nodes *J = B.jnodes;
        double *rel = buf, *bur = rel + nn, *nrm = bur + 3 * ns, *pt = nrm + 3 * ns;
        int32_t *ses = (int32_t *)(pt + 3 * ns), *sn = ses + nn, *ig = sn + 2 * ns, *cnt = ig + ns, *mis = cnt + n;
        const int64_t *no = (const int64_t *)ws->ptr[WS_INST_OFFS], *so = no + (n + 1);
        const unsigned gn = (unsigned)((nn + 255) / 256), gs = (unsigned)((ns + 255) / 256);
        const unsigned gi = (unsigned)((n + 255) / 256);
        auto nodes = [&](auto *dst, const auto *src, int comps) {
            if (nn > 0)
                hipLaunchKernelGGL(k_copy_masked<std::remove_cv_t<std::remove_reference_t<decltype(*dst)>>>, dim3(gn),
                                   dim3(256), 0, st, dst, src, nn, comps, no, n, (const uint8_t *)d_mask);
        };
        auto segs = [&](auto *dst, const auto *src, int comps) {
            if (ns > 0)
                hipLaunchKernelGGL(k_copy_masked<std::remove_cv_t<std::remove_reference_t<decltype(*dst)>>>, dim3(gs),
                                   dim3(256), 0, st, dst, src, ns, comps, so, n, (const uint8_t *)d_mask);
        };
        auto insts = [&](int32_t *dst, const int32_t *src) {
            hipLaunchKernelGGL(k_copy_inst<int32_t>, dim3(gi), dim3(256), 0, st, dst, src, n, (const uint8_t *)d_mask);
        };
        if (to_save) {
            nodes(rel, (const double *)J->release, 1);
            nodes(ses, (const int32_t *)J->ses, 1);
            segs(bur, (const double *)B.burgers_w, 3);
            segs(nrm, (const double *)B.normal_w, 3);
            segs(pt, (const double *)J->point, 3);
            segs(sn, (const int32_t *)B.seg_nodes_w, 2);
            segs(ig, (const int32_t *)J->ignore, 1);
            insts(cnt, J->count);
            insts(mis, J->missed);
        } else {
            nodes(J->release, (const double *)rel, 1);
            nodes(J->ses, (const int32_t *)ses, 1);
            segs(B.burgers_w, (const double *)bur, 3);
            segs(B.normal_w, (const double *)nrm, 3);
            segs(J->point, (const double *)pt, 3);
            segs(B.seg_nodes_w, (const int32_t *)sn, 2);
            segs(J->ignore, (const int32_t *)ig, 1);
            insts(J->count, cnt);
            insts(J->missed, mis);
        }
        DD_HIP(hipGetLastError());
        return DD_OK;
    }

    // Junction state of the masked instances: `to_save` copies the caller's
    // state (and fast clocks) into save slot `buf`/`fast_saved`, otherwise back.
    int junction_state(double *buf, std::vector<int64_t> &fast_saved, const std::vector<uint8_t> &mask,
                       bool to_save)
    {
        if (B.jnodes) {
            for (int i = 0; i < B.n_inst; ++i)
                if (mask[i]) {
                    if (to_save) fast_saved[i] = fast[i];
                    else fast[i] = fast_saved[i];
                }
            return node_state(buf, mask, to_save);
        }
        if (!B.jn) return DD_OK;
        const int n = B.n_inst;
        const int64_t nn = B.node_off[n];
        for (int i = 0; i < n; ++i)
            if (mask[i]) {
                if (to_save) fast_saved[i] = fast[i];
                else fast[i] = fast_saved[i];
            }
        if (nn == 0) return DD_OK;
        uint8_t *d_mask;
        int rc = upload_mask(mask, &d_mask);
        if (rc) return rc;
        // saved layout: release [nn] doubles, then junction, ignore, count [nn] int32 each
        double *rel = buf;
        int32_t *ints = (int32_t *)(buf + nn);
        const int64_t *no = (const int64_t *)ws->ptr[WS_INST_OFFS];
        const unsigned g = (unsigned)((nn + 255) / 256);
        const dd_junctions *j = B.jn;
        if (to_save) {
            hipLaunchKernelGGL(k_copy_masked<double>, dim3(g), dim3(256), 0, st, rel, (const double *)j->release, nn, 1,
                               no, n, (const uint8_t *)d_mask);
            hipLaunchKernelGGL(k_copy_masked<int32_t>, dim3(g), dim3(256), 0, st, ints, (const int32_t *)j->junction,
                               nn, 1, no, n, (const uint8_t *)d_mask);
            hipLaunchKernelGGL(k_copy_masked<int32_t>, dim3(g), dim3(256), 0, st, ints + nn, (const int32_t *)j->ignore,
                               nn, 1, no, n, (const uint8_t *)d_mask);
            hipLaunchKernelGGL(k_copy_masked<int32_t>, dim3(g), dim3(256), 0, st, ints + 2 * nn,
                               (const int32_t *)j->count, nn, 1, no, n, (const uint8_t *)d_mask);
        } else {
            hipLaunchKernelGGL(k_copy_masked<double>, dim3(g), dim3(256), 0, st, j->release, (const double *)rel, nn, 1,
                               no, n, (const uint8_t *)d_mask);
            hipLaunchKernelGGL(k_copy_masked<int32_t>, dim3(g), dim3(256), 0, st, j->junction, (const int32_t *)ints,
                               nn, 1, no, n, (const uint8_t *)d_mask);
            hipLaunchKernelGGL(k_copy_masked<int32_t>, dim3(g), dim3(256), 0, st, j->ignore, (const int32_t *)(ints + nn),
                               nn, 1, no, n, (const uint8_t *)d_mask);
            hipLaunchKernelGGL(k_copy_masked<int32_t>, dim3(g), dim3(256), 0, st, j->count,
                               (const int32_t *)(ints + 2 * nn), nn, 1, no, n, (const uint8_t *)d_mask);
        }
        DD_HIP(hipGetLastError());
        return DD_OK;
    }

    int upload_mask(const std::vector<uint8_t> &mask, uint8_t **d)
    {
        void *p;
        int rc = ensure(ws, WS_PTA_MASK, mask.size(), &p);
        if (rc) return rc;
        DD_HIP(hipMemcpyAsync(p, mask.data(), mask.size(), hipMemcpyHostToDevice, st));
        DD_HIP(hipStreamSynchronize(st));
        *d = (uint8_t *)p;
        return DD_OK;
    }
};

}  // namespace
}  // namespace dd

using namespace dd;

namespace dd {
namespace {
int pta_impl(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x, const int32_t *seg_nodes,
             const double *burgers, const double *normal, const uint8_t *pinned, const double *volume,
             const double *stress_rate, const double *t, const dd_pta_params *prm, const dd_material *m, int n_gauss,
             int precision, double near_cutoff_a, double exact_eta, const dd_junctions *jn, int64_t *fast_steps,
             double *out, void *stream, const dd_junction_nodes *jnodes = nullptr)
{
    int rc;
    if (n_inst < 0) return set_error(DD_EINVAL, "n_inst < 0");
    if (n_inst == 0) return DD_OK;
    if (!node_off || !seg_off || !stress_rate || !t || !prm || !m || !out || !volume)
        return set_error(DD_EINVAL, "null argument");
    if (node_off[0] != 0 || seg_off[0] != 0) return set_error(DD_EINVAL, "offsets must start at 0");
    for (int i = 0; i < n_inst; ++i) {
        if (node_off[i + 1] < node_off[i] || seg_off[i + 1] < seg_off[i])
            return set_error(DD_EINVAL, "offsets must be non-decreasing");
        if (seg_off[i + 1] > seg_off[i] && node_off[i + 1] == node_off[i])
            return set_error(DD_EINVAL, "instance %d has segments but no nodes", i);
    }
    const dd_pta_params &P = *prm;
    if (!(P.dt > 0.0) || !std::isfinite(P.dt)) return set_error(DD_EINVAL, "dt must be > 0");
    if (P.chunk_steps < 1 || P.max_chunks < 2) return set_error(DD_EINVAL, "chunk_steps >= 1 and max_chunks >= 2");
    if (!(P.tol_rho >= 0.0) || !(P.tol_lp >= 0.0)) return set_error(DD_EINVAL, "tolerances must be >= 0");
    if (!(P.delta > 0.0) || !std::isfinite(P.delta)) return set_error(DD_EINVAL, "delta must be > 0");
    if (!(P.strain_step > 0.0) || !(P.h_max > 0.0)) return set_error(DD_EINVAL, "strain_step and h_max must be > 0");
    if (P.max_jumps < 0 || std::isnan(P.lpdot_max)) return set_error(DD_EINVAL, "bad jump parameters");
    if (precision != DD_FP64 && precision != DD_MIXED) return set_error(DD_EINVAL, "unknown precision");
    if (n_gauss < 1 || n_gauss > DD_MAX_GAUSS) return set_error(DD_EINVAL, "n_gauss must be in 1..16");
    if (!(m->mu > 0.0) || !(m->nu > -1.0 && m->nu < 0.5) || !(m->a > 0.0) || !(m->B > 0.0))
        return set_error(DD_EINVAL, "bad material");
    for (int i = 0; i < 6 * n_inst; ++i)
        if (!std::isfinite(stress_rate[i])) return set_error(DD_EINVAL, "non-finite stress_rate");
    for (int i = 0; i < n_inst; ++i)
        if (!std::isfinite(t[i])) return set_error(DD_EINVAL, "non-finite t");
    const int64_t nn = node_off[n_inst], ns = seg_off[n_inst];
    if (nn > 0 && !x) return set_error(DD_EINVAL, "null x");
    if (ns > 0 && (!seg_nodes || !burgers || !normal)) return set_error(DD_EINVAL, "null segment array");
    if (nn >= INT32_MAX || 2 * ns >= INT32_MAX) return set_error(DD_EINVAL, "more than 2^31 nodes or 2^30 segments");
    if (precision == DD_MIXED && !(near_cutoff_a >= 1.0)) return set_error(DD_EINVAL, "near_cutoff_a must be >= 1");
    if (!(exact_eta >= 0.0) || std::isinf(exact_eta)) return set_error(DD_EINVAL, "exact_eta must be finite and >= 0");
    if (jn) {
        if (!(jn->capture_radius >= 0.0) || !std::isfinite(jn->capture_radius) || !(jn->max_break_time >= 0.0) ||
            !std::isfinite(jn->max_break_time))
            return set_error(DD_EINVAL, "junctions: capture radius and breaking time must be finite and >= 0");
        if (jn->n_fractions < 1) return set_error(DD_EINVAL, "junctions: n_fractions must be >= 1");
        if (nn > 0 && (!jn->fractions || !jn->junction || !jn->release || !jn->ignore || !jn->count))
            return set_error(DD_EINVAL, "junctions: null state or fractions array");
        if (!fast_steps) return set_error(DD_EINVAL, "junctions: null fast_steps");
        for (int i = 0; i < n_inst; ++i)
            if (fast_steps[i] < 0) return set_error(DD_EINVAL, "junctions: fast_steps must be >= 0");
    }
    if (jnodes) {
        const dd_junction_nodes *J = jnodes;
        if (!(J->capture_radius >= 0.0) || !std::isfinite(J->capture_radius) || !(J->max_break_time >= 0.0) ||
            !std::isfinite(J->max_break_time) || !(J->min_length >= 0.0) || !std::isfinite(J->min_length))
            return set_error(DD_EINVAL, "junction nodes: capture radius, breaking time and min_length must be "
                                        "finite and >= 0");
        if (J->n_slots < 1 || J->n_fractions < 1)
            return set_error(DD_EINVAL, "junction nodes: n_slots and n_fractions must be >= 1");
        if (!J->fractions || !J->release || !J->ses || !J->ignore || !J->point || !J->count || !J->missed)
            return set_error(DD_EINVAL, "junction nodes: null state or fractions array");
        if (exact_eta != 0.0) return set_error(DD_EINVAL, "junction nodes: no exact band (exact_eta must be 0)");
        for (int i = 0; i < n_inst; ++i)
            if (node_off[i + 1] - node_off[i] < (int64_t)J->n_slots + 2 || seg_off[i + 1] - seg_off[i] < J->n_slots)
                return set_error(DD_EINVAL, "junction nodes: instance %d has fewer than n_slots + 2 nodes or n_slots "
                                            "segments", i);
        if (!fast_steps) return set_error(DD_EINVAL, "junction nodes: null fast_steps");
        for (int i = 0; i < n_inst; ++i)
            if (fast_steps[i] < 0) return set_error(DD_EINVAL, "junction nodes: fast_steps must be >= 0");
    }
    hipStream_t st = (hipStream_t)stream;
    Workspace *ws;
    if ((rc = workspace(&ws))) return rc;

    BurstBatch B;
    B.n_inst = n_inst;
    B.node_off.assign(node_off, node_off + n_inst + 1);
    B.seg_off.assign(seg_off, seg_off + n_inst + 1);
    B.x = x;
    B.seg_nodes = seg_nodes;
    B.burgers = burgers;
    B.normal = normal;
    B.volume = volume;
    B.pinned = pinned;
    B.mat = *m;
    B.n_gauss = n_gauss;
    B.precision = precision;
    B.near_cut = near_cutoff_a;
    B.eta = exact_eta;
    B.dt = P.dt;
    if ((rc = burst_batch_init(B, st))) return rc;

    Driver D{B, P, st, ws};
    void *p;
    double *jA = nullptr, *jB = nullptr;
    std::vector<int64_t> fastA(n_inst, 0), fastB(n_inst, 0);
    if (jnodes) {
        if ((rc = ensure(ws, WS_PTA_FAST, sizeof(int64_t) * n_inst, &p))) return rc;
        D.fast_dev = (int64_t *)p;
        D.fast.assign(fast_steps, fast_steps + n_inst);
        B.jnodes = jnodes;
        B.seg_nodes_w = const_cast<int32_t *>(seg_nodes);
        B.burgers_w = const_cast<double *>(burgers);
        B.normal_w = const_cast<double *>(normal);
        B.fast_steps_dev = D.fast_dev;
        const size_t jbytes = sizeof(double) * (size_t)(nn + 9 * ns) + sizeof(int32_t) * (size_t)(nn + 3 * ns + 2 * n_inst);
        if ((rc = ensure(ws, WS_PTA_JA, jbytes, &p))) return rc;
        jA = (double *)p;
        if ((rc = ensure(ws, WS_PTA_JB, jbytes, &p))) return rc;
        jB = (double *)p;
    } else if (jn) {
        if ((rc = ensure(ws, WS_PTA_FAST, sizeof(int64_t) * n_inst, &p))) return rc;
        D.fast_dev = (int64_t *)p;
        D.fast.assign(fast_steps, fast_steps + n_inst);
        B.jn = jn;
        B.fast_steps_dev = D.fast_dev;
        // saved junction state: release (double) and junction, ignore, count (int32) per node
        const size_t jbytes = (sizeof(double) + 3 * sizeof(int32_t)) * (size_t)std::max<int64_t>(nn, 1);
        if ((rc = ensure(ws, WS_PTA_JA, jbytes, &p))) return rc;
        jA = (double *)p;
        if ((rc = ensure(ws, WS_PTA_JB, jbytes, &p))) return rc;
        jB = (double *)p;
    }
    if ((rc = ensure(ws, WS_PTA_SIGMA, sizeof(double) * 6 * n_inst, &p))) return rc;
    D.sig_dev = (double *)p;
    if ((rc = ensure(ws, WS_PTA_SUMS, sizeof(double) * 13 * n_inst, &p))) return rc;
    D.sums_dev = (double *)p;
    D.sums_h.assign(13 * (size_t)n_inst, 0.0);
    if ((rc = ensure(ws, WS_PTA_XA, sizeof(double) * 3 * std::max<int64_t>(nn, 1), &p))) return rc;
    double *xA = (double *)p;
    if ((rc = ensure(ws, WS_PTA_XB, sizeof(double) * 3 * std::max<int64_t>(nn, 1), &p))) return rc;
    double *xB = (double *)p;

    const double delta = P.delta;
    std::vector<double> sigA(6 * (size_t)n_inst), sigB(6 * (size_t)n_inst);
    for (int i = 0; i < n_inst; ++i)
        for (int k = 0; k < 6; ++k) {
            sigA[6 * i + k] = (t[i] - delta) * stress_rate[6 * i + k];
            sigB[6 * i + k] = t[i] * stress_rate[6 * i + k];
        }
    Runs A(n_inst), Bv(n_inst);
    std::vector<int> jumps(n_inst, 0), rerun(n_inst, 0);
    std::vector<uint8_t> todo(n_inst, 0);
    for (int i = 0; i < n_inst; ++i) todo[i] = seg_off[i + 1] > seg_off[i];

    // steps 1-4: paired fast runs, restarted from the end of the t run after a jump
    for (;;) {
        bool any = false;
        for (int i = 0; i < n_inst; ++i) any = any || todo[i];
        if (!any) break;
        for (int i = 0; i < n_inst; ++i)
            if (todo[i]) {
                A.reset(i);
                Bv.reset(i);
            }
        if ((rc = D.fast_run(todo, sigA, A))) return rc;                  // step 1 at l(t - Delta)
        if ((rc = D.copy_nodes(xA, x, todo))) return rc;                   // its end state
        if ((rc = D.junction_state(jA, fastA, todo, true))) return rc;
        if ((rc = D.fast_run(todo, sigB, Bv))) return rc;                 // step 2 at l(t)
        for (int i = 0; i < n_inst; ++i) {
            if (!todo[i]) continue;
            double La[9], Lb[9], d[9];
            A.lp(i, La);
            Bv.lp(i, Lb);
            for (int k = 0; k < 9; ++k) d[k] = (Lb[k] - La[k]) / delta;   // step 3
            if (frob(d, 9) > P.lpdot_max && jumps[i] < P.max_jumps) ++jumps[i];   // step 4: again
            else todo[i] = 0;
        }
    }
    // step 5: continue the t - Delta run from its end state while |R_a| > |R_b|
    std::vector<uint8_t> need(n_inst, 0), any_rerun(n_inst, 0);
    auto update_need = [&]() {
        bool any = false;
        for (int i = 0; i < n_inst; ++i) {
            need[i] = 0;
            if (seg_off[i + 1] == seg_off[i] || rerun[i] >= P.max_chunks) continue;
            double La[9], Lb[9];
            A.lp(i, La);
            Bv.lp(i, Lb);
            need[i] = frob(La, 9) > frob(Lb, 9);
            any = any || need[i];
        }
        return any;
    };
    if (update_need()) {
        any_rerun = need;
        if ((rc = D.copy_nodes(xB, x, any_rerun))) return rc;
        if ((rc = D.copy_nodes(x, xA, any_rerun))) return rc;
        if ((rc = D.junction_state(jB, fastB, any_rerun, true))) return rc;
        if ((rc = D.junction_state(jA, fastA, any_rerun, false))) return rc;
        do {
            if ((rc = D.chunk(need, sigA, A))) return rc;
            for (int i = 0; i < n_inst; ++i) rerun[i] += need[i];
        } while (update_need());
        if ((rc = D.copy_nodes(x, xB, any_rerun))) return rc;   // carry the end of the t run on
        if ((rc = D.junction_state(jB, fastB, any_rerun, false))) return rc;
        DD_HIP(hipStreamSynchronize(st));
    }
    // outputs, step 6
    for (int i = 0; i < n_inst; ++i) {
        double *o = out + (size_t)DD_PTA_OUT * i;
        for (int k = 0; k < DD_PTA_OUT; ++k) o[k] = 0.0;
        double ga[12], gb[12], La[9], Lb[9];
        A.rates(i, ga);
        Bv.rates(i, gb);
        lp_from_rates(ga, La);
        lp_from_rates(gb, Lb);
        o[DD_PTA_RHO_A] = A.rho(i);
        o[DD_PTA_RHO_B] = Bv.rho(i);
        for (int k = 0; k < 12; ++k) {
            o[DD_PTA_G_A + k] = ga[k];
            o[DD_PTA_G_B + k] = gb[k];
        }
        for (int k = 0; k < 9; ++k) {
            o[DD_PTA_LP_A + k] = La[k];
            o[DD_PTA_LP_B + k] = Lb[k];
            o[DD_PTA_LPDOT + k] = (Lb[k] - La[k]) / delta;
        }
        o[DD_PTA_RHODOT] = (Bv.rho(i) - A.rho(i)) / delta;
        const double nlp = frob(Lb, 9);
        o[DD_PTA_H] = nlp > 0.0 ? std::fmin(P.h_max, P.strain_step / nlp) : P.h_max;
        o[DD_PTA_STEPS_A] = (double)A.steps[i];
        o[DD_PTA_STEPS_B] = (double)Bv.steps[i];
        o[DD_PTA_CONV_A] = A.conv[i];
        o[DD_PTA_CONV_B] = Bv.conv[i];
        o[DD_PTA_JUMPS] = jumps[i];
        o[DD_PTA_RERUN] = rerun[i];
    }
    if (validation_on()) {
        if (nn > 0)
            hipLaunchKernelGGL(k_pta_flags, dim3((unsigned)((3 * nn + 255) / 256)), dim3(256), 0, st, x, 3 * nn,
                               ws->flags_dev);
        if ((rc = read_flags(ws, st))) return rc;
    }
    DD_HIP(hipStreamSynchronize(st));
    if (jn || jnodes)
        for (int i = 0; i < n_inst; ++i) fast_steps[i] = D.fast[i];
    return DD_OK;
}
}  // namespace
}  // namespace dd

extern "C" int dd_pta_step(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                           const int32_t *seg_nodes, const double *burgers, const double *normal,
                           const uint8_t *pinned, const double *volume, const double *stress_rate,
                           const double *t, const dd_pta_params *prm, const dd_material *m, int n_gauss,
                           int precision, double near_cutoff_a, double exact_eta, double *out, void *stream)
{
    ::dd::Range range_("dd_pta_step");
    clear_error();
    return pta_impl(n_inst, node_off, seg_off, x, seg_nodes, burgers, normal, pinned, volume, stress_rate, t, prm, m,
                    n_gauss, precision, near_cutoff_a, exact_eta, nullptr, nullptr, out, stream);
}

extern "C" int dd_pta_step_junctions(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                                     const int32_t *seg_nodes, const double *burgers, const double *normal,
                                     const uint8_t *pinned, const double *volume, const double *stress_rate,
                                     const double *t, const dd_pta_params *prm, const dd_material *m, int n_gauss,
                                     int precision, double near_cutoff_a, double exact_eta,
                                     const dd_junctions *junctions, int64_t *fast_steps, double *out, void *stream)
{
    ::dd::Range range_("dd_pta_step_junctions");
    clear_error();
    if (!junctions) return set_error(DD_EINVAL, "null junction parameters");
    return pta_impl(n_inst, node_off, seg_off, x, seg_nodes, burgers, normal, pinned, volume, stress_rate, t, prm, m,
                    n_gauss, precision, near_cutoff_a, exact_eta, junctions, fast_steps, out, stream);
}


extern "C" int dd_pta_step_junction_nodes(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                                          int32_t *seg_nodes, double *burgers, double *normal, const uint8_t *pinned,
                                          const double *volume, const double *stress_rate, const double *t,
                                          const dd_pta_params *prm, const dd_material *m, int n_gauss, int precision,
                                          double near_cutoff_a, const dd_junction_nodes *junctions,
                                          int64_t *fast_steps, double *out, void *stream)
{
    ::dd::Range range_("dd_pta_step_junction_nodes");
    clear_error();
    if (!junctions) return set_error(DD_EINVAL, "null junction-node parameters");
    return pta_impl(n_inst, node_off, seg_off, x, seg_nodes, burgers, normal, pinned, volume, stress_rate, t, prm, m,
                    n_gauss, precision, near_cutoff_a, 0.0, nullptr, fast_steps, out, stream, junctions);
}
