/*
 * dd.h -- C ABI of libdd.so, the MI355X (gfx950) library for the all-pairs
 * dislocation-segment force path of "Plasticity without phenomenology: a
 * first step" (Chatterjee, Po, Zhang, Acharya, Ghoniem).
 *
 * The paper runs Discrete Dislocation Dynamics (DD) only in short bursts at
 * frozen load (Sec. "Application of PTA for coarse-graining DD simulation",
 * Eq. fast_dd) and averages their output in time (Eq. R_lambda_t).  Inside a
 * burst the time goes to the interaction of every straight segment with every
 * other: the stress of one segment (Sec. "Discrete Dislocation Dynamics": a
 * differential operator on R = x - x' convolved with the dislocation density;
 * here its isotropic, non-singular line-integral form with R_a =
 * sqrt(R.R + a^2), integrated in closed form along the segment) evaluated at
 * Gauss points of every other segment, contracted into Peach-Koehler forces
 * df_k = eps_kjm sigma_ji b_i dl_m, integrated to nodal forces, then the glide
 * velocity of Eq. DD_evol and the node update x(t + dt) = x(t) + w dt.
 *
 * Conventions common to every call
 * --------------------------------
 * Memory.   Array arguments are DEVICE pointers (hipMalloc or a PyTorch-ROCm
 *           tensor's data_ptr) unless marked "host".  The caller owns them;
 *           the library never frees them.  The library keeps a per-device
 *           workspace (grown on demand with hipMalloc, released by
 *           dd_shutdown).  Calls that share a device must not overlap in
 *           time (issue them on one stream, or synchronise between them).
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default
 *           stream).  Work is enqueued on it; outputs are valid once the
 *           stream has been synchronised.  With validation on (the default)
 *           each call also synchronises the stream before returning so that
 *           it can report input errors (see dd_set_validation).
 * Layouts.  Structure of arrays: positions x[3][n_nodes] (all x, then all y,
 *           then all z), burgers[3][n_segs], normal[3][n_segs], forces
 *           [3][n_nodes], float64.  seg_nodes[2][n_segs] int32: segment s
 *           runs from node seg_nodes[s] to node seg_nodes[n_segs + s]; that
 *           order is its line sense t.  pinned[n_nodes] uint8 (non-zero =
 *           immobile node).  sigma_app: Voigt (xx, yy, zz, yz, xz, xy).
 * Units.    Any consistent set: positions, Burgers vectors and the core width
 *           a in one length unit; mu and every stress in one stress unit;
 *           the drag B in stress*time; dt in time.  Forces are returned in
 *           stress*length^2, velocities in length/time.  Internally lengths
 *           are divided by a and stresses by mu, so FP32 work never
 *           underflows whatever the caller's unit.
 * Slip systems.  FCC, 12 systems alpha = 3 p + d: plane normals
 *           p = 0..3: (1,1,1), (-1,1,1), (1,-1,1), (1,1,-1) over sqrt(3); in
 *           plane p the three <110> directions normal to it, d = 0 the one
 *           with zero x component, d = 1 zero y, d = 2 zero z, first non-zero
 *           entry positive, over sqrt(2).
 * Errors.   Every int-returning call returns DD_OK (0) or a negative code and
 *           then dd_last_error() (per thread) says why.  No C++ exception
 *           crosses this interface.  Kernels never read out of bounds, even
 *           on invalid input: bad node indices are clamped on the device and
 *           reported as DD_EINVAL when validation is on.
 */
#ifndef DD_H
#define DD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DD_OK          0
#define DD_EINVAL     (-1)   /* invalid argument or input array contents  */
#define DD_EHIP       (-2)   /* a HIP runtime call failed                 */
#define DD_ENOMEM     (-3)   /* device workspace allocation failed        */
#define DD_ENONFINITE (-4)   /* a NaN or Inf reached an output            */
#define DD_ECAPACITY  (-5)   /* a fixed-size device list ran out of room  */
#define DD_EIO        (-6)   /* a file could not be opened, read or written,
                                or is not a valid file of the expected kind */

#define DD_MAX_GAUSS  16
#define DD_N_SYSTEMS  12
#define DD_N_FEATURES 36

/* Isotropic material: shear modulus mu, Poisson ratio nu, core width a,
 * scalar drag B (Eq. DD_evol with B = B 1).  Valid: mu > 0, -1 < nu < 0.5,
 * a > 0, B > 0 (B is only read by the mobility calls). */
typedef struct { double mu, nu, a, B; } dd_material;

/* DD_FP64: every pair in float64.
 * DD_MIXED: pairs whose minimum distance from the target Gauss point to the
 * source segment is below near_cutoff_a * a, and nearly collinear pairs (the
 * target inside a cone of half-angle about 1/16 around the source's axis,
 * seen from its midpoint: ym^2 > 256 (rho^2 + a^2) for its axial offset ym
 * and perpendicular distance rho), are evaluated in float64; all others in
 * float32 with float32 accumulation over a source tile: the closed form in a
 * cancellation-free arrangement, or, when the target is at least 30 source
 * lengths from the source midpoint, 2-point Gauss-Legendre quadrature of the
 * integrand along the source (error below 2e-7 relative there).  Tile sums,
 * nodal sums and the mobility step stay float64. */
typedef enum { DD_FP64 = 0, DD_MIXED = 1 } dd_precision;

/* Message of the last error on the calling thread ("" if none). */
const char *dd_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int dd_version(void);

/* Turn host-side reporting of input errors and non-finite outputs on (1,
 * default) or off (0).  Off: no synchronisation inside calls; invalid input
 * still cannot make a kernel read out of bounds, but it yields unspecified
 * results instead of an error code.  Returns the previous setting. */
int dd_set_validation(int on);

/* Release the workspace of every device this thread's process used. */
int dd_shutdown(void);

/* Work-item autotuner on (1, default) or off (0: a fixed heuristic).  When
 * on, the first dd_nodal_forces / dd_burst_batch call for a new problem
 * class (GPU architecture, Gauss points, precision, and the instance count,
 * total and largest instance size rounded up to powers of two) times the
 * candidate source-range lengths of a work item (and, for the mixed path,
 * both variants of its kernel) on one all-pairs pass over its own inputs plus
 * the reduction of that pass's partial sums (synchronising the stream), and
 * keeps the fastest for the
 * process; with the environment variable DD_AUTOTUNE_CACHE naming a file,
 * choices are also read from and appended to it.  Results do not depend on
 * the choice beyond the order of floating-point sums.  Returns the previous
 * setting. */
int dd_set_autotune(int on);

/* How dd_burst_batch runs its steps.  0 (default): batches of small FP64
 * bursts (every instance at most 512 segments and 512 nodes; no exact band)
 * run all their steps in one persistent launch, several co-resident
 * workgroups per instance meeting at one barrier per step (about 2 nodes per
 * workgroup, at most 128 per instance), when all of them fit on the device at
 * once; other bursts replay a cached graph of per-step kernels.  1: always the step graph.  2: the persistent launch with one
 * workgroup per instance (a reference point for the split).  The persistent
 * launch's results do not depend on the split; they differ from the step
 * graph's only in the order of floating-point sums.  Returns the previous
 * mode, or DD_EINVAL for a mode other than 0, 1 and 2.  A persistent burst
 * whose workgroups wait too long at a step barrier raises DD_EHIP (reported
 * as the device-side checks are). */
int dd_set_burst_mode(int mode);

/* Report, and clear, the conditions the device-side checks raised since the
 * last report: synchronises `stream` (hipStream_t, may be null) and returns
 * DD_OK, or the error code and message of the first condition in the order
 * DD_EINVAL (bad node index, zero-length segment, normal not of unit
 * length), DD_ENONFINITE, DD_ECAPACITY (exact band: a captured step's near
 * pairs outgrew the pair store, see dd_burst_batch).  Calls made with
 * validation on report them themselves; with validation off they stay
 * pending until this call or the next validating call. */
int dd_check(void *stream);

/* Fix the work split instead of letting the autotuner (or its heuristic)
 * choose it, for reproducible benchmarks and for tests of each kernel
 * variant: chunk_len = source-range length of a work item (0: the built-in
 * heuristic, else at least 16), variant = the mixed kernel's variant (see
 * dd_last_plan).  chunk_len < 0 returns to the automatic choice.  Applies to
 * every later force evaluation in the process.  DD_EINVAL for a chunk_len in
 * 1..15 or a variant other than 0, 1 and 2. */
int dd_set_plan(int64_t chunk_len, int variant);

/* The work split of the most recent force evaluation on this device: the
 * source-range length of a work item, the number of work items, and the
 * mixed kernel's variant.  Variants: 0 = each source is first tested in FP32
 * against a band of max(30 L, cutoff + L/2) around its midpoint, and sources
 * outside it for every target point of a wavefront are evaluated by 2-point
 * Gauss-Legendre quadrature along the source; 1 = no such test, every pair
 * located in FP64 and evaluated by the FP32 closed form or the FP64 near
 * field; 2 = as 0 with 3-point quadrature beyond max(6 L, cutoff + L/2).
 * All three stay within 5e-7 relative of the exact segment field per pair.
 * Any pointer may be null. */
int dd_last_plan(int64_t *chunk_len, int64_t *n_items, int *variant);

/* Measurement hooks (for benchmarks and profilers).  With timing on, every
 * launch of the all-pairs kernel made outside graph capture is bracketed by a
 * HIP event pair recorded on the caller's stream.  dd_timing_read waits for
 * the recorded events and returns, since the last reset: the summed
 * event-to-event time of those launches in milliseconds, the number of
 * launches, and how many (target Gauss point, source segment) evaluations
 * the mixed kernel sent to its FP64 near-field branch and to its FP32
 * source-quadrature branch (both counted whether or not timing is on; the
 * remaining mixed evaluations used the FP32 closed form).  Any output pointer
 * may be null.  reset != 0 clears everything afterwards.  Not for use while
 * another thread calls the library. */
int dd_timing_enable(int on);
int dd_timing_read(double *kernel_ms, int64_t *launches, int64_t *near_evals,
                   int64_t *quad_evals, int reset);

/* Measured vector-ALU peak of the current device, a reference point for the
 * all-pairs kernels' roofline beside the published peaks.  kind selects the
 * fused multiply-add form: 0 = FP64 and 1 = FP32 with one operand the same
 * for every lane (read from a scalar register), 2 = FP64 and 3 = FP32 with
 * every operand per lane (vector registers); FP32 is the unpacked form the
 * library is built with (packed FP32 instructions are disabled).  Runs three
 * warm-up and then `reps` (1..1000) launches of a kernel that keeps 8
 * independent multiply-add chains per lane on 4096 workgroups of 256 lanes,
 * times them with HIP events on `stream` (hipStream_t, may be null), waits,
 * and writes the rate in TFLOP/s (a multiply-add counts 2) to *tflops.
 * Uses a 4 MiB workspace buffer.  DD_EINVAL for a null pointer or a bad
 * kind or reps. */
int dd_vector_peak(int kind, int reps, double *tflops, void *stream);

/* Nodal forces (internal + applied) on every node.
 *  For every segment j and Gauss-Legendre point q of an n_gauss-point rule
 *  on [0, 1] (points s_q, weights w_q):
 *    sigma(x_jq) = sigma_app + sum_{i != j} sigma^i(x_jq)
 *    f_jq = (sigma(x_jq) b_j) x t_j                      (Peach-Koehler)
 *    F[n1(j)] += L_j w_q (1 - s_q) f_jq,  F[n2(j)] += L_j w_q s_q f_jq
 *  where sigma^i is the closed-form non-singular stress of segment i.  A
 *  segment's own field is excluded (it only redistributes force between its
 *  two nodes: its net force vanishes by symmetry).
 * Exact band: the force source i sends to target j's nodes is L_j int_0^1
 *  N(u) (sigma^i(x_j(u)) b_j) x t_j du for the two linear shape functions N
 *  (the Peach-Koehler force of Sec. "Discrete Dislocation Dynamics"
 *  integrated along the target); the rule above takes it with n_gauss
 *  points.  With exact_eta > 0, pairs whose midpoints are closer than
 *  exact_eta sqrt((L_i^2 + L_j^2)/2), i.e. with S = x1 + x2, D = x2 - x1,
 *      |S_i - S_j|^2 < 2 exact_eta^2 (|D_i|^2 + |D_j|^2)
 *  (evaluated in float64 without fused multiply-adds, in this order, on the
 *  caller's positions), take it exactly instead (to ~1e-14 of the pair's
 *  contribution: 12-point Gauss-Legendre on panels graded towards the
 *  integrand's complex singularities).  This removes the quadrature error of
 *  a small n_gauss on adjacent and close segments (several per cent of the
 *  net self-force of an irregular loop at n_gauss = 2); exact_eta = 2 to 4
 *  selects about 4 to 16 near sources per segment in dislocation loops.  The
 *  self pair is never included; the correction is float64 with either
 *  precision.  0 turns the band off.  With the band on, the call counts the
 *  near pairs first and waits once for that count (an event recorded on the
 *  stream after the count pass; the pair kernel is already queued behind it)
 *  to size its pair store, so the call returns only once the count pass has
 *  finished (any number of near sources per segment; at most 2^31 - 1 near
 *  pairs).
 * Arguments: x [3][n_nodes], seg_nodes [2][n_segs], burgers [3][n_segs];
 *  normal [3][n_segs] is validated (unit length) but unused by the force;
 *  sigma_app host [6]; m host; 1 <= n_gauss <= DD_MAX_GAUSS; precision a
 *  dd_precision; near_cutoff_a >= 1 (in units of a, mixed only, checked
 *  only for DD_MIXED; the workload value is 20); exact_eta >= 0 and finite;
 *  force_out [3][n_nodes] (overwritten).
 * Errors: DD_EINVAL for null pointers, counts < 0, bad material, n_gauss out
 *  of range, a bad exact_eta, a node index outside [0, n_nodes), a
 *  zero-length segment or a normal of length differing from 1 by more than
 *  1e-6 (validation on); DD_ENONFINITE if a force is NaN/Inf (validation
 *  on); DD_ECAPACITY for more than 2^31 - 1 near pairs. */
int dd_nodal_forces(int64_t n_nodes, const double *x, int64_t n_segs,
                    const int32_t *seg_nodes, const double *burgers,
                    const double *normal, const double *sigma_app,
                    const dd_material *m, int n_gauss, int precision,
                    double near_cutoff_a, double exact_eta, double *force_out, void *stream);

/* dd_nodal_forces for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, layouts and results as dd_nodal_forces without
 * the exact band (the same numbers bit for bit when both use the same work
 * split: the built-in heuristic, or what dd_set_plan fixes; this call never
 * runs the autotuner).  Every buffer beyond the caller's arrays comes from a
 * fixed device array of 64 MiB that each GPU holds from the library's first
 * use until the process ends, so the call allocates nothing, never
 * synchronises and may be captured in a graph.  Limit: the pass's scratch
 * (about 400 bytes per segment, 6 KiB per work item of 256 Gauss points x one
 * source range, and the node lists) must fit in 64 MiB, e.g. 16,384 segments
 * at 2 or 4 Gauss points; larger problems return DD_ECAPACITY before any
 * device work.  Every call on a GPU uses that GPU's one array: calls that
 * overlap on one device (two streams, two threads) race and give wrong
 * results; calls in one stream are ordered and safe.  Input errors are not
 * reported (as with validation off, results are then unspecified; kernels
 * stay in bounds).
 * Errors: DD_EINVAL as dd_nodal_forces for host-side argument checks;
 *  DD_ECAPACITY as above; DD_EHIP if the array's address cannot be taken. */
int dd_nodal_forces_noalloc(int64_t n_nodes, const double *x, int64_t n_segs,
                            const int32_t *seg_nodes, const double *burgers,
                            const double *normal, const double *sigma_app,
                            const dd_material *m, int n_gauss, int precision,
                            double near_cutoff_a, double *force_out, void *stream);

/* One glide-constrained forward-Euler step (Eq. DD_evol, lumped, scalar B):
 *    ell_n = 1/2 sum_{s attached to n} L_s
 *    v_n   = P_n F_n / (B ell_n),   x_n <- x_n + v_n dt
 *  P_n projects out the component along the slip-plane normal shared by the
 *  node's segments; with two distinct normals (up to sign) v is projected on
 *  the line n1 x n2; with three or more, or when pinned or unattached, v = 0.
 * Arguments: x [3][n_nodes] updated in place; force [3][n_nodes];
 *  seg_nodes, normal as above; pinned [n_nodes] (nullable = none pinned);
 *  m host (B used); dt > 0; vel_out [3][n_nodes] (nullable).
 * Errors: as dd_nodal_forces. */
int dd_glide_step(int64_t n_nodes, double *x, const double *force,
                  int64_t n_segs, const int32_t *seg_nodes,
                  const double *normal, const uint8_t *pinned,
                  const dd_material *m, double dt, double *vel_out,
                  void *stream);

/* One DD time step: dd_nodal_forces at x, then dd_glide_step with those
 * forces (Sec. "Discrete Dislocation Dynamics", Eq. DD_evol), in one call
 * that builds the node-to-segment lists once and takes the segment lengths
 * of the glide step from the force pass, so the Euler update is fused into
 * the glide kernel.  Same results as the two calls up to rounding (lengths
 * are formed in units of a).  Arguments: as the two calls; x [3][n_nodes]
 * updated in place; pinned nullable; m host (mu, nu, a, B); force_out and
 * vel_out [3][n_nodes] nullable (then workspace is used).  Errors: as the two
 * calls. */
int dd_step(int64_t n_nodes, double *x, int64_t n_segs, const int32_t *seg_nodes, const double *burgers,
            const double *normal, const uint8_t *pinned, const double *sigma_app, const dd_material *m,
            int n_gauss, int precision, double near_cutoff_a, double exact_eta, double dt, double *force_out,
            double *vel_out, void *stream);

/* Independent DD bursts at frozen applied stress, all advanced together.
 *  Instance i owns nodes [node_off[i], node_off[i+1]) and segments
 *  [seg_off[i], seg_off[i+1]) of the packed arrays; its seg_nodes are local
 *  to it (0 .. its node count - 1) and instances never interact.  Every step
 *  k = 0 .. n_steps-1 of every instance does: nodal forces of X_k (as
 *  dd_nodal_forces, with that instance's sigma_app), glide velocities v_k,
 *  the per-system slip rate
 *    gdot_alpha(k) = (1/V) sum_{s in alpha} (b_s . m_alpha) L_s
 *                    ((t_s x (v_n1 + v_n2)/2) . n_alpha)
 *  (the segment distortion rate b/A (x) (l x V) times l A, Sec. "Thermal
 *  activation", summed over the volume and resolved on system alpha; s in
 *  alpha when its normal and Burgers direction match the system up to sign),
 *  then X_{k+1} = X_k + v_k dt.  Output: rate_avg_out[i][alpha] =
 *  (1/n_steps) sum_k gdot_alpha(k), the running time average of
 *  Eq. R_lambda_t with equal steps.  x is advanced in place, so a second
 *  call resumes the burst.
 *  features_out (nullable) [n_inst][36]: of the initial state, per system:
 *  [0..11] resolved shear stress m_alpha . sigma_app n_alpha (numerator of
 *  Eq. schmid), [12..23] mobile and [24..35] sessile line length per volume
 *  (a segment is sessile when both its nodes are pinned).
 * Arguments: node_off, seg_off HOST [n_inst+1] int64, non-decreasing, from 0;
 *  x, seg_nodes, burgers, normal, pinned (nullable) packed as above;
 *  sigma_app [n_inst][6] and volume [n_inst] device; m host; n_gauss,
 *  precision, near_cutoff_a, exact_eta as dd_nodal_forces; n_steps >= 0;
 *  dt > 0; rate_avg_out [n_inst][12].
 * Execution: the step loop is captured into a HIP graph, instantiated and
 *  kept (up to 4 per device, least recently used dropped): a later call
 *  with the same arguments (pointers and values), offsets and work split
 *  relaunches it without capture.  With validation off the call is
 *  asynchronous on `stream` (outputs valid after the stream is synchronised)
 *  once the instance tables, work split and graph are cached: the first call
 *  for new offsets uploads tables and may time the work split
 *  (synchronising).  With validation on it synchronises and reports errors.
 *  Exact band: the near-pair store is sized before capture to twice the
 *  near-pair count of the initial positions plus 8 per segment (a count pass
 *  and one synchronisation; with validation off only while the store is
 *  empty); a step whose near pairs outgrow it keeps the n_gauss rule for the
 *  excess pairs and raises DD_ECAPACITY (reported by this call with
 *  validation on, else by dd_check).
 * Errors: as dd_nodal_forces, also for inconsistent offsets. */
int dd_burst_batch(int32_t n_inst, const int64_t *node_off,
                   const int64_t *seg_off, double *x,
                   const int32_t *seg_nodes, const double *burgers,
                   const double *normal, const uint8_t *pinned,
                   const double *sigma_app, const double *volume,
                   const dd_material *m, int n_gauss, int precision,
                   double near_cutoff_a, double exact_eta, int n_steps, double dt,
                   double *rate_avg_out, double *features_out, void *stream);

/* Junctions and their thermally activated breaking (Sec. "Thermal
 * activation", Eq. tb), for dd_burst_batch_junctions.  A mobile node (not
 * pinned) that comes closer than capture_radius to a sessile segment (both
 * its nodes pinned) of its own instance forms a junction: it is held fixed
 * until t_b = f * max_break_time has passed, f = fractions[node][count mod
 * n_fractions] (uniform numbers in [0, 1) supplied by the caller; count = the
 * node's number of junctions so far).  No node is inserted.  The checks run
 * at the start of every step k, at time t0 + k dt: a held node whose release
 * time has come is released (and forms no junction in that step); a free node
 * forgets the segment it last broke from once it is farther than
 * 2 capture_radius from it, then is captured by the first sessile segment in
 * index order, other than that one, closer than capture_radius.  Distances
 * are evaluated in float64 without fused multiply-adds.  State, per node
 * (device arrays [n_nodes], caller-owned, carried from call to call; start
 * with junction = ignore = -1, count = 0): junction = index of the holding
 * segment in the batch's segment arrays or -1, release = its release time,
 * ignore = the segment it last broke from or -1, count.  Units: lengths as
 * the positions, times as dt. */
typedef struct {
    double capture_radius, max_break_time, t0;
    int32_t n_fractions;
    const double *fractions;   /* [n_nodes][n_fractions] */
    int32_t *junction;         /* [n_nodes] */
    double *release;           /* [n_nodes] */
    int32_t *ignore;           /* [n_nodes] */
    int32_t *count;            /* [n_nodes] */
} dd_junctions;

/* dd_burst_batch with junctions (see dd_junctions): the same arguments and
 * outputs; held nodes do not move and contribute no slip rate while held.
 * DD_EINVAL for a null `junctions`, a negative or non-finite radius or
 * breaking time, a non-finite t0, n_fractions < 1 or null arrays. */
int dd_burst_batch_junctions(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                             const int32_t *seg_nodes, const double *burgers, const double *normal,
                             const uint8_t *pinned, const double *sigma_app, const double *volume,
                             const dd_material *m, int n_gauss, int precision, double near_cutoff_a,
                             double exact_eta, int n_steps, double dt, const dd_junctions *junctions,
                             double *rate_avg_out, double *features_out, void *stream);

/* Junction nodes (Sec. "Thermal activation", Eq. tb), for
 * dd_burst_batch_junction_nodes: a mobile dislocation that meets a sessile one
 * is held at their intersection until the junction breaks after
 * t_b = f * max_break_time, and bows around it meanwhile.
 *  - Capture: a mobile segment (not sessile, not a free slot) that comes
 *    closer than capture_radius to a sessile segment of its instance (an
 *    instance's own segment between two of its own pinned nodes) is split at
 *    its point of closest approach (segment-to-segment) by a pinned junction
 *    node: a -> b becomes a -> j and j -> b (same Burgers vector and normal).
 *    The node keeps at least min_length from both ends (parameter clamped to
 *    [min_length / L, 1 - min_length / L]); a segment no longer than
 *    2 min_length forms no junction.
 *  - A segment forms no junction while it is within 2 capture_radius of the
 *    point of its last junction (point-to-segment distance): both halves of
 *    a split keep the junction point (junctions do not nest), and so does
 *    the merged segment after the release.
 *  - Release: at t >= its release time the node is removed: its in-segment
 *    takes the end node of its out-segment, which is freed.
 *  - Order, each step k at time t0 + k dt: releases (node slots in index
 *    order); then captures found on the positions at the start of the step
 *    (per segment the first sessile segment in index order), applied in
 *    segment index order; a capture takes the lowest
 *    free node slot and the lowest free segment slot, and without one it is
 *    not made and counted in missed.  f = fractions[inst][count mod
 *    n_fractions], count = the instance's number of junctions so far.
 *    Distances and the junction point are computed in float64 without fused
 *    multiply-adds.
 *  - Slots: every instance ends its nodes with n_slots node slots and two
 *    dummy nodes D1, D2 (all pinned), and its segments with n_slots segment
 *    slots; a free segment slot is D1 -> D2 with Burgers vector 0 and a unit
 *    normal (it adds no stress, feels no force and belongs to no slip
 *    system).  The caller sets up the free slots; seg_nodes, burgers, normal
 *    and the positions of node slots change in place.
 *  - State (device arrays, caller-owned, carried from call to call; start
 *    with ses = -1, ignore = count = missed = 0): release [n_nodes] (release
 *    time of an active junction node), ses [n_nodes] (batch index of its
 *    sessile segment, -1: the node slot is free), ignore [n_segs] (1 while
 *    the segment keeps the point of its last junction), point [3][n_segs]
 *    (that point), count and missed [n_inst].
 * Units: lengths as the positions, times as dt. */
typedef struct {
    double capture_radius, max_break_time, t0, min_length;
    int32_t n_slots, n_fractions;
    const double *fractions;   /* [n_inst][n_fractions] */
    double *release;           /* [n_nodes] */
    int32_t *ses;              /* [n_nodes] */
    int32_t *ignore;           /* [n_segs] */
    double *point;             /* [3][n_segs] */
    int32_t *count, *missed;   /* [n_inst] */
} dd_junction_nodes;

/* dd_burst_batch with junction nodes (see dd_junction_nodes): the arguments
 * and outputs of dd_burst_batch except exact_eta (no exact band: the
 * topology changes during the call); seg_nodes, burgers and normal are
 * changed in place.  Rates are averaged over the steps; features_out
 * (nullable) describes the state at the start of the call.
 * Errors: DD_EINVAL as dd_burst_batch, and for a null `junctions` or state
 * array, n_slots < 1, n_fractions < 1, a negative or non-finite radius,
 * breaking time or min_length, a non-finite t0, or an instance with fewer
 * than n_slots + 2 nodes or n_slots segments; an inconsistent slot state
 * (a junction node without its two segments) is reported as DD_EINVAL by
 * the call, or by dd_check when validation is off. */
int dd_burst_batch_junction_nodes(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                                  int32_t *seg_nodes, double *burgers, double *normal, const uint8_t *pinned,
                                  const double *sigma_app, const double *volume, const dd_material *m,
                                  int n_gauss, int precision, double near_cutoff_a, int n_steps, double dt,
                                  const dd_junction_nodes *junctions, double *rate_avg_out, double *features_out,
                                  void *stream);

/* One slow-time step of Practical Time Averaging for a batch of independent
 * DD volumes (Sec. "Application of PTA for coarse-graining DD simulation",
 * subsection "Algorithm", steps 1-7).  Volume i is at slow time t[i] under
 * the load l(t) = t * stress_rate[i] (a constant stress-rate tensor).  State
 * functions: the line density rho (segments that belong to a slip system,
 * length over volume) and the plastic distortion rate
 * L^p = sum_alpha gdot_alpha m_alpha (x) n_alpha (gdot as dd_burst_batch;
 * for glide motion this equals (1/V) sum_s b_s (x) (t_s x v_s) L_s).  Their
 * running time averages R (Eq. R_lambda_t, equal fast steps) are advanced in
 * chunks of chunk_steps fast steps and have converged when, from the second
 * check on, |R - R at the previous check| <= tol |R| for rho (tol_rho) and
 * for L^p (tol_lp, Frobenius norm); a fast run stops unconverged after
 * max_chunks checks.
 *  1. from the current microstructure, fast run at l(t - delta) -> R_a;
 *  2. from the end state of 1, fast run at l(t) -> R_b;
 *  3. Lpdot = (R_b^Lp - R_a^Lp) / delta;
 *  4. if |Lpdot| > lpdot_max (a jump), 1-3 again from the end state of 2, at
 *     most max_jumps times;
 *  5. while |R_a^Lp| > |R_b^Lp|, the run of 1 continues from its own end
 *     state one chunk at a time (at most max_chunks more);
 *  6. Lpdot and rhodot = (R_b^rho - R_a^rho) / delta from the final values;
 *     next slow step h = min(h_max, strain_step / |R_b^Lp|).
 * x ends as the end state of step 2 (the microstructure for the next step).
 * All instances advance together on the GPU; only those still running take
 * fast steps.
 * Arguments: node_off, seg_off HOST; x, seg_nodes, burgers, normal, pinned
 *  (nullable) and volume device, as dd_burst_batch; stress_rate HOST
 *  [n_inst][6] Voigt Pa/s; t HOST [n_inst] s; prm, m host; n_gauss,
 *  precision, near_cutoff_a, exact_eta as dd_nodal_forces; out HOST
 *  [n_inst][DD_PTA_OUT] doubles laid out by the DD_PTA_* indices below
 *  (L^p row-major).  Synchronises the stream.
 * Errors: DD_EINVAL for inconsistent offsets or parameters (dt, delta,
 *  strain_step, h_max > 0; chunk_steps >= 1; max_chunks >= 2; tolerances
 *  >= 0; max_jumps >= 0), otherwise as dd_burst_batch. */
typedef struct {
    double dt;            /* fast (DD) time step, s */
    int32_t chunk_steps;  /* fast steps between convergence checks */
    int32_t max_chunks;   /* checks before a fast run stops unconverged */
    double tol_rho;       /* relative tolerance of R^rho (paper: 1e-2) */
    double tol_lp;        /* relative tolerance of R^Lp (paper: 3e-2) */
    double lpdot_max;     /* jump threshold on |Lpdot|, 1/s^2 (paper: 0.05) */
    double delta;         /* slow-time interval, s (paper: 0.1) */
    double strain_step;   /* step control: h |R_b^Lp| <= strain_step (paper: 0.002) */
    double h_max;         /* largest slow step, s */
    int32_t max_jumps;    /* restarts after jumps in one step */
} dd_pta_params;

#define DD_PTA_OUT 64
#define DD_PTA_RHO_A 0    /* R^rho at t - delta */
#define DD_PTA_RHO_B 1    /* R^rho at t */
#define DD_PTA_G_A 2      /* [12] running averages of gdot_alpha at t - delta */
#define DD_PTA_G_B 14     /* [12] ... at t */
#define DD_PTA_LP_A 26    /* [9] R^Lp at t - delta */
#define DD_PTA_LP_B 35    /* [9] R^Lp at t */
#define DD_PTA_LPDOT 44   /* [9] Lpdot */
#define DD_PTA_RHODOT 53  /* rhodot */
#define DD_PTA_H 54       /* next slow step h */
#define DD_PTA_STEPS_A 55 /* fast steps of the t - delta run (step 5 included) */
#define DD_PTA_STEPS_B 56 /* fast steps of the t run */
#define DD_PTA_CONV_A 57  /* 1 if the t - delta run converged */
#define DD_PTA_CONV_B 58  /* 1 if the t run converged */
#define DD_PTA_JUMPS 59   /* restarts taken in step 4 */
#define DD_PTA_RERUN 60   /* chunks added in step 5 */

int dd_pta_step(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                const int32_t *seg_nodes, const double *burgers, const double *normal,
                const uint8_t *pinned, const double *volume, const double *stress_rate,
                const double *t, const dd_pta_params *prm, const dd_material *m, int n_gauss,
                int precision, double near_cutoff_a, double exact_eta, double *out, void *stream);

/* dd_pta_step with junctions (see dd_junctions; Sec. "Thermal activation"):
 * every fast step runs the junction checks first.  The junction state
 * travels with the microstructure: each fast run carries it on from the state
 * it starts from, step 5 continues the t - delta run with the state of that
 * run's own end, and the state at the end of step 2 is what the call leaves
 * in the junction arrays, as for x.  The clock of the checks is the volume's
 * fast clock, fast_steps[i] * dt at the first step, one dt per fast step
 * (junctions->t0 is not used); fast_steps HOST [n_inst] int64, >= 0, in and
 * out: the fast steps the volume had taken, advanced by those of the run
 * carried on.  The other arguments as dd_pta_step.
 * Errors: DD_EINVAL as dd_pta_step, for a null junctions or fast_steps, a
 *  negative fast_steps entry, or junction parameters dd_burst_batch_junctions
 *  rejects. */
int dd_pta_step_junctions(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                          const int32_t *seg_nodes, const double *burgers, const double *normal,
                          const uint8_t *pinned, const double *volume, const double *stress_rate,
                          const double *t, const dd_pta_params *prm, const dd_material *m, int n_gauss,
                          int precision, double near_cutoff_a, double exact_eta, const dd_junctions *junctions,
                          int64_t *fast_steps, double *out, void *stream);

/* dd_pta_step with junction nodes (see dd_junction_nodes; Sec. "Thermal
 * activation"): every fast step runs the releases and captures first, which
 * change x, seg_nodes, burgers and normal in place (every instance carries
 * n_slots node and segment slots as dd_burst_batch_junction_nodes needs).
 * The topology and the junction-node state travel with the microstructure as
 * the positions do: each fast run carries them on from the state it starts
 * from, step 5 continues the t - delta run from that run's own end, and the
 * topology, node state and positions at the end of step 2 are what the call
 * leaves in the caller's arrays.  The clock of a step is the volume's fast
 * clock, (fast_steps[i] + steps taken in this run) * dt (junctions->t0 is not
 * used); fast_steps HOST [n_inst] int64, >= 0, in and out as for
 * dd_pta_step_junctions.  No exact band.  The other arguments as
 * dd_pta_step.
 * Errors: DD_EINVAL as dd_pta_step, for a null junctions or fast_steps, a
 *  negative fast_steps entry, or what dd_burst_batch_junction_nodes rejects. */
int dd_pta_step_junction_nodes(int32_t n_inst, const int64_t *node_off, const int64_t *seg_off, double *x,
                               int32_t *seg_nodes, double *burgers, double *normal, const uint8_t *pinned,
                               const double *volume, const double *stress_rate, const double *t,
                               const dd_pta_params *prm, const dd_material *m, int n_gauss, int precision,
                               double near_cutoff_a, const dd_junction_nodes *junctions, int64_t *fast_steps,
                               double *out, void *stream);

/* Block coupling of the DD boxes to the continuum mesh (Sec. "DD-MFDM
 * coupling").  The domain is n x n square blocks of side B and thickness h,
 * one brick through the thickness (one DD box per block); every block is
 * meshed by m x m x 1 trilinear hexahedra of the continuum calculation, each
 * with 2 x 2 x 2 Gauss points.  Numbering: element e = ey * (n m) + ex
 * (ex, ey in [0, n m)); Gauss point 8 e + 4 gz + 2 gy + gx at isoparametric
 * coordinates ((2 gx - 1), (2 gy - 1), (2 gz - 1)) / sqrt(3); block
 * r = by * n + bx.  Fields: Gauss-point arrays [n_gp][c] and block arrays
 * [n * n][c] of float64 (c components, 1..16: a tensor is 9 components in
 * row-major order ij, a vector 3), device memory owned by the caller.  Valid:
 * n, m >= 1, n m <= 65535, n <= 46340, B, h finite and > 0.  Errors: DD_EINVAL. */
typedef struct { int32_t n, m; double B, h; } dd_block_mesh;

/* Block averages <f>_r = int_{Omega_r} f dv / |Omega_r| of a Gauss-point field
 * (the block stress average of Sec. "DD-MFDM coupling"), by the elements'
 * Gauss rule: on this uniform mesh, the mean of the block's 8 m^2 values. */
int dd_block_average(const dd_block_mesh *mesh, int c, const double *f_gp, double *f_block, void *stream);

/* The blockwise-constant field f_block (e.g. the DD boxes' L^p or V) at every
 * Gauss point, as the paper prescribes (subsection "Obtaining L^p, V at
 * Gauss point of element"): its L2 projection onto the continuous trilinear
 * finite-element space of the block mesh (consistent mass matrix), then the
 * two-level isoparametric interpolation, first to the element's nodes with
 * the block's shape functions, then to the Gauss point with the element's.
 * Uses the device workspace (2 (n + 1)^2 c doubles). */
int dd_block_to_gauss(const dd_block_mesh *mesh, int c, const double *f_block, double *f_gp, void *stream);

/* Non-negative dissipation at n_gp Gauss points (Sec. "Ensuring non-negative
 * dissipation", Eq. Lp_gauss and Eq. V_gauss), in place: where d = T : Lp < 0,
 * Lp <- Lp - d T / |T|^2; where beta = V . (X T alpha) < 0, with
 * (X T alpha)_i = eps_ijk (T alpha)_jk, V <- V - beta (X T alpha) /
 * |X T alpha|^2.  T, alpha, Lp: [n_gp][9] (row-major), V: [n_gp][3].  Lp or V
 * may be null (that part is skipped); alpha may be null when V is.  Where T
 * (or X T alpha) is zero nothing changes. */
int dd_dissipation_fix(int64_t n_gp, const double *T, const double *alpha, double *Lp, double *V, void *stream);

/* ---------------------------------------------------------------------- */
/* Slip-rate surrogate (not in the paper): a 4-member ensemble of MLPs     */
/* 36 -> 256 -> 256 -> 256 -> 12, ReLU hidden layers, that maps the 36     */
/* features above to the 12 burst-averaged slip rates.  bfloat16 weights   */
/* and activations on the matrix cores, float32 accumulation, float32      */
/* master weights and Adam moments.                                        */
/* ---------------------------------------------------------------------- */
#define DD_MLP_IN      36
#define DD_MLP_HIDDEN  256
#define DD_MLP_OUT     12
/* Parameters of one member, flat float32, in this order: W1[256][36],
 * b1[256], W2[256][256], b2[256], W3[256][256], b3[256], W4[12][256], b4[12]
 * (W[out][in]). */
#define DD_MLP_PARAMS  144140

typedef struct dd_mlp dd_mlp;

/* Create an ensemble of n_members (1..8) on the current device with
 * He-uniform weights drawn on the host from `seed` (member k uses seed + k),
 * zero biases, identity input/output scaling.  *out receives the handle. */
int dd_mlp_create(int n_members, uint64_t seed, dd_mlp **out);
int dd_mlp_destroy(dd_mlp *model);

/* Copy one member's parameters in (host float32 [DD_MLP_PARAMS]); resets the
 * Adam state of that member. */
int dd_mlp_set_params(dd_mlp *model, int member, const float *host_params);
/* Copy one member's float32 master parameters out to host memory. */
int dd_mlp_get_params(const dd_mlp *model, int member, float *host_params);

/* Persistence.  dd_mlp_save writes the whole ensemble to `path`: member
 * count, network shape, Adam step count, the scaling of dd_mlp_set_scaling,
 * dd_mlp_set_log_densities and dd_mlp_set_spread_floor, and per member the
 * float32 master parameters and both Adam moments, followed by an FNV-1a
 * checksum.  It writes `path`.tmp first and renames it, so `path` never holds
 * a partial file.  dd_mlp_load reads and checks such a file (magic and
 * version, shape, checksum, no trailing bytes, finite values) before any
 * device call, then creates the ensemble on the current device; *out
 * receives the handle, which the caller releases with dd_mlp_destroy.  A
 * loaded model infers bit for bit as the saved one did, and training resumes
 * where it stopped (same Adam state).  File errors return DD_EIO with the
 * reason in dd_last_error(); *out stays NULL on any error. */
int dd_mlp_save(const dd_mlp *model, const char *path);
int dd_mlp_load(const char *path, dd_mlp **out);
/* Member count and Adam steps taken (host outputs, each nullable). */
int dd_mlp_info(const dd_mlp *model, int *n_members, int64_t *adam_steps);

/* Feature and target standardisation (host arrays): the network sees
 * (feat - in_shift) * in_scale and predicts (rate - out_shift) / out_scale. */
int dd_mlp_set_scaling(dd_mlp *model, const float *in_shift, const float *in_scale,
                       const float *out_shift, const float *out_scale);

/* Density features 12..35 enter the network as log10(rho * dens_scale +
 * dens_floor) (before standardisation) when dens_floor > 0; dens_floor = 0
 * (the default) passes them through unchanged.  Resolved shear stresses
 * (features 0..11) are never transformed. */
int dd_mlp_set_log_densities(dd_mlp *model, float dens_scale, float dens_floor);

/* Floor of the spread denominator in dd_surrogate_rates (default 1e-30):
 * spread = |std|_2 / max(|mean|_2, floor), in rate units.  floor >= 0. */
int dd_mlp_set_spread_floor(dd_mlp *model, float floor);

/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) of
 * every member on the same mini-batch: feat [n][36], target rates [n][12]
 * (device float32, unstandardised); loss_out (device float32
 * [n_members], nullable) receives each member's mean squared error in
 * standardised units before the step.  1 <= n <= 65536. */
int dd_mlp_train_step(dd_mlp *model, int64_t n, const float *feat,
                      const float *target, float lr, float *loss_out,
                      void *stream);

/* Forward and backward pass without the update: grad_out (device float32
 * [n_members][DD_MLP_PARAMS], flat layout of the parameters) receives the
 * gradient of each member's standardised mean squared error on the batch,
 * loss_out (nullable) the losses.  1 <= n <= 65536. */
int dd_mlp_gradients(dd_mlp *model, int64_t n, const float *feat,
                     const float *target, float *grad_out, float *loss_out,
                     void *stream);

/* Ensemble inference: rates [n][12] = member mean (unstandardised), spread
 * [n] = ||population std over members||_2 / max(||mean||_2, 1e-30),
 * needs_dd [n] = spread > spread_tol (DD is the fallback for those points).
 * feat [n][36] device float32; rates, spread, needs_dd device. */
int dd_surrogate_rates(const dd_mlp *model, int64_t n, const float *feat,
                       float *rates, float *spread, uint8_t *needs_dd,
                       float spread_tol, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DD_H */
