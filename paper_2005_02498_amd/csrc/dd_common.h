// Internal declarations of libdd.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "dd.h"
#include "dd_host.h"

namespace dd {

// ---------------------------------------------------------------- errors --
int set_error(int code, const char *fmt, ...);
void clear_error();
bool validation_on();

// Named roctx range over a host scope (rocprofv3 --marker-trace shows the
// library's calls, graph captures and tuner passes on the timeline; without a
// tool attached each range costs two library calls).
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

#define DD_HIP(call)                                                           \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            return ::dd::set_error(DD_EHIP, "%s failed: %s (%s:%d)", #call,    \
                                   hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

// Flags raised by device-side checks (OR-ed into one word).
enum : unsigned {
    FLAG_BAD_INDEX = 1u,
    FLAG_ZERO_LENGTH = 2u,
    FLAG_BAD_NORMAL = 4u,
    FLAG_NONFINITE = 8u,
    FLAG_NEAR_FULL = 16u,     // a near-pair list or the pair store ran out of room
    FLAG_NEAR_PANELS = 32u,   // an exact-band integral needed more panels than allowed
    FLAG_BARRIER = 64u,       // a persistent burst's barrier wait ran out of polls
};

// -------------------------------------------------------------- workspace --
// Per-device scratch: named slots, grown on demand, freed by dd_shutdown().
enum Slot {
    WS_SEG64 = 0,      // FP64 segment records
    WS_SEG32,          // FP32 segment records (mixed path)
    WS_PARTIAL,        // per work item partial sums
    WS_SEGF,           // per-segment end forces [6][n_segs]
    WS_CSR_PTR,        // node -> incident (segment, end) list: offsets
    WS_CSR_LIST,       //   ... and entries
    WS_CSR_CNT,        //   ... counters
    WS_TILES,          // tile table
    WS_ITEMS,          // work-item table
    WS_SEG_INST,       // segment -> instance
    WS_OFFS,           // device copies of instance offsets
    WS_VEL,            // node velocities
    WS_FORCE,          // node forces (bursts)
    WS_RATE,           // running slip-rate sums
    WS_INST_OFFS,      // instance node and segment offsets
    WS_MISC,
    WS_PROBE,          // output of the vector-peak probe
    WS_ACTIVE,         // per-instance active flags of a partial burst
    WS_PTA_SIGMA,      // PTA driver: applied stress per instance
    WS_PTA_SUMS,       //   per-chunk sums per instance
    WS_PTA_XA,         //   saved positions (end of the t - Delta run)
    WS_PTA_XB,         //   saved positions (end of the t run)
    WS_PTA_MASK,       //   per-instance copy mask
    WS_PTA_FAST,       //   per-instance fast steps (junctions)
    WS_PTA_JA,         //   saved junction state (end of the t - Delta run)
    WS_PTA_JB,         //   saved junction state (end of the t run)
    WS_NEAR_KEY,       // exact band: per-segment keys
    WS_NEAR_SPH,       //   per-group bounding spheres
    WS_NEAR_LIST,      //   per-target near sources
    WS_NEAR_IDX,       //   per-target counts, in-wavefront offsets, first pair
    WS_NEAR_WAVE,      //   per-wavefront totals and their prefix
    WS_NEAR_PAIR,      //   flat (target, source) pairs
    WS_NEAR_CORR,      //   per-pair end-force corrections
    WS_BLOCK_A,        // block coupling: nodal values of the projection
    WS_BLOCK_FAC,      //   tridiagonal factors
    WS_HELD,           // junctions: nodes held in this step
    WS_SES,            //   sessile-segment flags, positions, indices
    WS_SES_X,          //   their end points and bounding spheres
    WS_JN_CAND,        // junction nodes: per-segment candidates and parameters
    WS_T0,             // junction bursts: the call's start time (one double)
    WS_PB,             // persistent bursts: second position buffer, velocities, per-workgroup sums
    WS_PB_INT,         //   workgroup tables
    WS_PB_BAR,         //   barrier arrival words
    WS_NSLOTS
};

// An instantiated step graph and the bytes of everything its kernels'
// arguments were built from (caller pointers and scalars, instance offsets,
// work split, workspace addresses): a call with the same key relaunches it.
struct GraphEntry {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};
constexpr size_t GRAPH_CACHE = 4;   // graphs kept per device (least recently used evicted)

struct Workspace {
    int device = -1;
    void *ptr[WS_NSLOTS] = {};
    size_t cap[WS_NSLOTS] = {};
    unsigned *flags_dev = nullptr;   // one word (sticky: cleared only when reported)
    unsigned *flags_host = nullptr;  // pinned mirror (bytes 64..71: near-pair count read-back)
    hipStream_t capture_stream = nullptr;
    hipEvent_t near_ev = nullptr;    // marks the near-pair count's read-back on the caller's stream
    int64_t block_fac_n = -1;                    // size of the tridiagonal factors in WS_BLOCK_FAC
    unsigned long long *near_count = nullptr;   // device counter (mixed kernel)
    bool capturing = false;
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;
    std::vector<int64_t> inst_key;   // offsets whose instance tables WS_SEG_INST / WS_INST_OFFS hold
    std::vector<int32_t> pb_tab;     // the persistent-burst workgroup table WS_PB_INT holds
};

// Reports (and clears) the flags raised since the last report; synchronises st.
int read_flags(Workspace *ws, hipStream_t st);
// Destroys the cached graphs of ws (synchronising the device first).
void drop_graphs(Workspace *ws);

// Event timing of the all-pairs kernel (dd_timing_enable / dd_timing_read).
bool timing_on();
void timing_begin(hipStream_t st, bool capturing);
void timing_end(hipStream_t st, bool capturing);

// Returns the workspace of the current device (creating it on first use).
int workspace(Workspace **out);
// Makes slot s at least `bytes` large.  Growing synchronises the device first.
int ensure(Workspace *ws, Slot s, size_t bytes, void **out);

// --------------------------------------------------------------- kernels --
// Work decomposition of the pair kernel: a tile is up to TILE consecutive
// target Gauss points of one instance; an item is one tile against one
// contiguous range of that instance's sources.
// FCC slip system alpha = 3 p + d (the order dd.h documents): unit plane
// normal n = P[p] / sqrt(3) and slip direction m = D[p][d] / sqrt(2).  Used by
// the slip-rate kernels (device) and the PTA driver's L^p (host).
__host__ __device__ inline void fcc(int alpha, double n[3], double m[3])
{
    const double r3 = 0.57735026918962576451, r2 = 0.70710678118654752440;
    // plane normals
    const signed char P[4][3] = {{1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {1, 1, -1}};
    // directions, per plane: zero x, zero y, zero z
    const signed char D[4][3][3] = {
        {{0, 1, -1}, {1, 0, -1}, {1, -1, 0}},
        {{0, 1, -1}, {1, 0, 1}, {1, 1, 0}},
        {{0, 1, 1}, {1, 0, -1}, {1, 1, 0}},
        {{0, 1, 1}, {1, 0, 1}, {1, -1, 0}},
    };
    const int p = alpha / 3, d = alpha % 3;
    for (int k = 0; k < 3; ++k) {
        n[k] = P[p][k] * r3;
        m[k] = D[p][d][k] * r2;
    }
}


// FP64 segment records, structure of arrays with stride n_segs:
//  0..2 x1/a, 3..5 t, 6 L/a, 7..9 b/a, 10..12 c = (b/a) x t, 13 length of the
//  run of segments that each start where the one before ends (as a double);
// followed in the same buffer by one RECA-double record per segment (array of
// structures, read with wavefront-uniform scalar loads by the FP64 kernel):
//  0..12 as above, 13 the run length as int64 bits, 14..15 zero.
constexpr int REC64 = 14;
constexpr int RECA = 16;
constexpr int REC64_TOTAL = REC64 + RECA;   // doubles per segment in the buffer
// Bytes of the FP64 record buffer for ns segments.
inline size_t rec64_bytes(int64_t ns)
{
    return sizeof(double) * (size_t)REC64_TOTAL * (size_t)(ns > 1 ? ns : 1);
}
// FP32 segment record of the mixed path, REC32A floats per segment (array of
// structures, read with wavefront-uniform scalar loads or staged in LDS):
// the midpoint xm/a rounded to FP32 and its rounding remainder xm/a - [XH],
// t, and for the source quadrature of the kernel variant in use (points
// xm +- hq t with weight Wo each, plus xm with weight Wc for 3 points) hq,
// Wo b/a, Wo c, the squared band outside which it is used, 1 + hq^2, 2 hq and
// Wc/Wo; then L/a and 1/Wo (read only outside the quadrature) and two zeros.
// Without a quadrature Wo = 1.  The field is linear in b (c = b x t), so a
// rule on the scaled b and c needs no weight; the closed form unscales them
// with 1/Wo.  The quadrature reads the first R32_QUAD_VECS groups of four.
constexpr int R32_XH = 0, R32_XL = 3, R32_T = 6, R32_HQ = 9, R32_B = 10, R32_C = 13, R32_BAND = 16,
              R32_RA0 = 17, R32_TW = 18, R32_WC = 19, R32_L = 20, R32_IW = 21;
constexpr int R32_QUAD_VECS = 5;
constexpr int REC32A = 24;
// Mixed kernel variants: 0 = 2-point source quadrature beyond max(30 L,
// cutoff + L/2), 1 = no quadrature, 2 = 3-point source quadrature beyond
// max(6 L, cutoff + L/2).  A work split is encoded as MIXED_VARIANTS *
// (source-range length) + variant.
constexpr int MIXED_VARIANTS = 3;
inline __host__ __device__ int quad_points(int variant) { return variant == 0 ? 2 : (variant == 2 ? 3 : 0); }


// Exact band (the exact_eta argument of the force calls): near-pair lists and
// the exact target integrals of those pairs, as corrections to the Q-point
// end forces.
constexpr int NEAR_GROUP = 8;  // consecutive segments per bounding sphere of the near search
struct NearArgs {
    int64_t ns = 0, nn = 0, n_waves = 0, pair_cap = 0;
    int splits = 1;                      // source ranges per target (workgroups along y)
    const int32_t *seg_inst = nullptr;   // device [ns] or null (one volume)
    const int64_t *seg_off = nullptr;    // device [n_inst + 1] or null
    const int64_t *node_off = nullptr;   // device [n_inst + 1] or null
    const int32_t *seg_nodes = nullptr;
    const double *x = nullptr;           // positions, caller's units
    const double *rec = nullptr;         // FP64 segment records (lengths in units of a)
    double c2 = 0.0;                     // 2 eta^2
    double kr = 0.0, nu = 0.0, k2 = 0.0;
    GaussRule g{}, gp{};                 // the Q-point rule and the 12-point panel rule
    double *key = nullptr;               // [ns][4]
    float4 *sph = nullptr;               // [ceil(ns / NEAR_GROUP)] sphere centre, radius
    int32_t *scnt = nullptr;             // [ns][splits] near sources per split
    int32_t *cnt = nullptr;              // [ns] near sources per target
    int64_t *loc = nullptr, *ptr = nullptr;                   // [ns] each: in-wavefront prefix, first slot
    int64_t *wtot = nullptr, *woff = nullptr;                 // [n_waves], [n_waves + 1] (woff[n_waves] = total)
    int32_t *pair_t = nullptr, *pair_s = nullptr;             // [pair_cap] each
    double *corr = nullptr;                                   // [pair_cap][6]
    unsigned *flags = nullptr;
};
// Keys, counts and the scan (woff[n_waves] then holds the number of near
// pairs), then, once the pair arrays hold at least that many entries, the
// fill pass and the exact integrals.  Pairs beyond pair_cap are dropped (they
// keep the Q-point rule) and FLAG_NEAR_FULL is raised.
void launch_near_count(const NearArgs &A, hipStream_t st);
void launch_near_fill(const NearArgs &A, hipStream_t st);

// Glide steps of a batch of independent volumes in which only some instances
// advance (the PTA driver's fast runs): burst_batch_init uploads the instance
// tables and picks the work split (autotuner) once; each burst_batch_run
// takes n_steps for the instances with active[i] != 0, each under its own
// applied stress sigma_dev[6 i ..] (device, Voigt, Pa), and adds, per
// instance, the sum over the steps of the 12 resolved slip rates and of the
// line density to sums_dev[13 i ..] (device).  Idle instances keep their
// positions.  The arrays stay owned by the caller.
struct BurstBatch {
    int n_inst = 0;
    std::vector<int64_t> node_off, seg_off;   // host [n_inst + 1]
    double *x = nullptr;
    const int32_t *seg_nodes = nullptr;
    const double *burgers = nullptr, *normal = nullptr, *volume = nullptr;
    const uint8_t *pinned = nullptr;
    dd_material mat{};
    int n_gauss = 2, precision = DD_FP64;
    double near_cut = 20.0, eta = 0.0, dt = 0.0;
    int64_t choice = 0;                       // encoded work split, set by burst_batch_init
    // junctions (null: none): the caller's parameters and state, and per
    // instance the fast steps taken so far (device), whose product with dt is
    // the instance's fast clock
    const dd_junctions *jn = nullptr;
    const int64_t *fast_steps_dev = nullptr;
    // junction nodes (null: none): parameters and state, timed by the same
    // fast clock; captures and releases change the topology in place
    const dd_junction_nodes *jnodes = nullptr;
    int32_t *seg_nodes_w = nullptr;
    double *burgers_w = nullptr, *normal_w = nullptr;
};
int burst_batch_init(BurstBatch &B, hipStream_t st);
int burst_batch_run(const BurstBatch &B, const std::vector<uint8_t> &active, const double *sigma_dev,
                    int n_steps, double *sums_dev, hipStream_t st);

// All-pairs launchers (one workgroup per work item, TILE threads).
void launch_pair64(const Item *items, const Tile *tiles, const double *rec, int64_t ns, const GaussRule &g,
                   double k1, double k2, double *partial, int64_t n_items, hipStream_t st);
void launch_pair_mixed(const Item *items, const Tile *tiles, const double *rec, const float *rec32, int64_t ns,
                       const GaussRule &g, double k1, double k2, float cut, double *partial,
                       unsigned long long *counters, int64_t n_items, int variant, hipStream_t st);

}  // namespace dd
