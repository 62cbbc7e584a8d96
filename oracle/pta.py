"""Plain-Python oracle of the Practical Time Averaging (PTA) step -- TEST
INFRASTRUCTURE ONLY (imported by tests/ only).

It follows the paper's algorithm for coarse-graining DD in time (Sec.
"Application of PTA for coarse-graining DD simulation", subsection
"Algorithm", steps 1-7) for one DD volume at a time, with every fast step
taken by the FP64 oracle burst routine (``oracle.burst`` one glide step at a
time), and the running time averages of Eq. R_lambda_t with equal fast steps.

State functions (Lambda): the line density rho (total length of the segments
that belong to a slip system, over the volume) and the plastic distortion
rate L^p.  For glide-only motion every segment's contribution b (x) (t x v) L
/ V is parallel to m_alpha (x) n_alpha of its slip system, so
L^p = sum_alpha gdot_alpha m_alpha (x) n_alpha with gdot the 12 resolved slip
rates of the burst routine (pinned in ``tests/test_oracle_pta.py``).

Readings taken where the paper is silent:

* convergence of a running average is checked every ``chunk`` fast steps,
  from the second check on: R has converged when its change since the
  previous check is at most tol * |R| (|.| = absolute value for rho,
  Frobenius norm for L^p), tol_rho for rho and tol_lp for L^p together; a
  run stops unconverged after ``max_chunks`` checks;
* the load is l(t) = t * sigma_rate (a constant stress rate tensor);
* a jump (|Lpdot| > lpdot_max) restarts steps 1-3 from the state at the end
  of step 2, at most ``max_jumps`` times;
* step 5 continues the t - Delta run from its own end state (the state step 2
  started from), chunk by chunk, until |R^Lp_{t-Delta}| <= |R^Lp_t| or
  ``max_chunks`` more checks; the microstructure carried to the next slow
  step is the end state of step 2;
* Lpdot and rhodot are formed after step 5 (the jump test uses the values
  before it); the slow step is h = min(h_max, strain_step / |R^Lp_t|).

With junctions (``Junctions``, the rule of oracle/junctions.py) the junction
state and the fast clock travel with the microstructure: each fast run
carries them on from the state it starts from, the fast clock of a step is
(fast steps taken so far) * dt, and step 5 continues the t - Delta run with
the junction state and clock of its own end, after which the state of the end
of step 2 is carried on, as for the positions.  With junction nodes
(``JunctionNodes``, the rule of oracle/junction_nodes.py) the microstructure
also holds the topology (segment nodes, Burgers vectors, normals, which
captures and releases change): it travels the same way, with the node state
and the fast clock.
"""
from __future__ import annotations

import copy
from dataclasses import dataclass

import numpy as np

from . import burst, fcc_system
from . import junction_nodes as JN
from . import junctions as OJ


@dataclass
class PTAParams:
    dt: float                 # fast (DD) time step, s
    chunk: int = 10           # fast steps between convergence checks
    max_chunks: int = 20      # checks before a run stops unconverged
    tol_rho: float = 1e-2
    tol_lp: float = 3e-2
    lpdot_max: float = 0.05   # 1/s^2
    delta: float = 0.1        # slow-time interval Delta, s
    strain_step: float = 0.002
    h_max: float = 1.0        # s
    max_jumps: int = 2


def lp_from_rates(g):
    """L^p (3x3) from the 12 resolved slip rates: sum_alpha g_alpha m (x) n."""
    L = np.zeros((3, 3))
    for al in range(12):
        n, m = fcc_system(al)
        L += g[al] * np.outer(m, n)
    return L


def converged(prev, now, tol, norm):
    """|now - prev| <= tol |now| (both zero counts as converged)."""
    return norm(now - prev) <= tol * norm(now)


@dataclass
class Junctions:
    r_c: float                 # capture radius, b
    a_max: float               # maximum breaking time a, s
    fractions: np.ndarray      # [nn][K] uniform numbers f of Eq. tb
    state: dict                # per node junction, release, ignore, count
    fast: int = 0              # fast steps taken so far (the fast clock)


@dataclass
class JunctionNodes:
    params: JN.Params          # capture radius, maximum breaking time, l_min, slots (its t0 unused)
    state: dict                # oracle.junction_nodes.new_state
    seg_nodes: np.ndarray      # the topology the node state refers to
    burgers: np.ndarray
    normal: np.ndarray
    fast: int = 0              # fast steps taken so far (the fast clock)


@dataclass
class Run:
    x: np.ndarray        # state at the end of the run
    sums: np.ndarray     # [13]: sum over the steps of gdot (12) and rho
    steps: int
    converged: bool
    jn: Junctions | None = None   # junction state and clock at the end of the run

    @property
    def rho(self):
        return self.sums[12] / self.steps

    @property
    def lp(self):
        return lp_from_rates(self.sums[:12] / self.steps)


def _copy_jn(jn):
    if jn is None:
        return None
    if isinstance(jn, JunctionNodes):
        st = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in jn.state.items()}
        return JunctionNodes(jn.params, st, jn.seg_nodes.copy(), jn.burgers.copy(), jn.normal.copy(), jn.fast)
    return Junctions(jn.r_c, jn.a_max, jn.fractions, {k: v.copy() for k, v in jn.state.items()}, jn.fast)


def _one_step(inst, x, sigma, mat, Q, dt, jn=None):
    """Lambda at state x and the state after one glide step (after the
    junction checks at the fast clock, with the held nodes fixed, when `jn`
    is given; its state and clock advance in place).  With junction nodes the
    releases and captures at the fast clock change x (in place) and the
    topology of `jn` first."""
    s = copy.copy(inst)
    s.x = x
    s.sigma_app = np.asarray(sigma, float)
    if isinstance(jn, JunctionNodes):
        JN.topology_step(x, jn.seg_nodes, jn.burgers, jn.normal, inst.pinned, float(jn.fast) * dt, jn.params,
                         jn.state)
        s.seg_nodes, s.burgers, s.normal = jn.seg_nodes, jn.burgers, jn.normal
        jn.fast += 1
    elif jn is not None:
        held = OJ.update(x, inst.seg_nodes, inst.pinned, float(jn.fast) * dt, jn.r_c, jn.a_max, jn.fractions,
                         jn.state)
        s.pinned = np.maximum(np.asarray(inst.pinned, np.uint8), held)
        jn.fast += 1
    x1, rate, feat = burst(s, mat, Q, 1, dt)
    return x1, rate, float(np.sum(feat[12:]))


def fast_run(inst, x, sigma, mat, Q, P: PTAParams, run: Run | None = None, max_chunks=None, jn=None):
    """Runs chunks of P.chunk steps at fixed load sigma until the running
    averages of rho and L^p converge (or max_chunks checks); continues `run`
    (same state, sums and junction state) when it is given, else starts from
    x and the junction state `jn` (copied)."""
    if run is None:
        run = Run(np.array(x, float), np.zeros(13), 0, False, _copy_jn(jn))
        prev = None
    else:
        run = Run(run.x.copy(), run.sums.copy(), run.steps, False, _copy_jn(run.jn))
        prev = (run.rho, run.lp)
    max_chunks = P.max_chunks if max_chunks is None else max_chunks
    for c in range(max_chunks):
        for _ in range(P.chunk):
            x1, rate, rho = _one_step(inst, run.x, sigma, mat, Q, P.dt, run.jn)
            run.sums[:12] += rate
            run.sums[12] += rho
            run.steps += 1
            run.x = x1
        now = (run.rho, run.lp)
        if prev is not None and converged(prev[0], now[0], P.tol_rho, abs) and \
                converged(prev[1], now[1], P.tol_lp, np.linalg.norm):
            run.converged = True
            return run, c + 1
        prev = now
    return run, max_chunks


def pta_step(inst, t, sigma_rate, mat, Q, P: PTAParams, jn: Junctions | None = None):
    """One slow-time step at time t for one volume (its x is the current
    microstructure; `jn` its junction state and fast clock, if any).  Returns
    a dict with the converged averages, rates, the next step size, counters
    and the microstructure (and junction state) to continue from."""
    sigma_rate = np.asarray(sigma_rate, float)
    x0 = np.array(inst.x, float)
    j0 = jn
    jumps = 0
    while True:
        A, _ = fast_run(inst, x0, (t - P.delta) * sigma_rate, mat, Q, P, jn=j0)      # step 1
        B, _ = fast_run(inst, A.x, t * sigma_rate, mat, Q, P, jn=A.jn)                # step 2
        lpdot = (B.lp - A.lp) / P.delta                                               # step 3
        if np.linalg.norm(lpdot) > P.lpdot_max and jumps < P.max_jumps:               # step 4
            jumps += 1
            x0, j0 = B.x, B.jn
            continue
        break
    rerun_chunks = 0                                                             # step 5
    while np.linalg.norm(A.lp) > np.linalg.norm(B.lp) and rerun_chunks < P.max_chunks:
        A, _ = fast_run(inst, None, (t - P.delta) * sigma_rate, mat, Q, P, run=A, max_chunks=1)
        rerun_chunks += 1
    lpdot = (B.lp - A.lp) / P.delta
    rhodot = (B.rho - A.rho) / P.delta
    nlp = np.linalg.norm(B.lp)                                                   # step 6
    h = min(P.h_max, P.strain_step / nlp) if nlp > 0 else P.h_max
    return {"rho_a": A.rho, "rho_b": B.rho, "g_a": A.sums[:12] / A.steps, "g_b": B.sums[:12] / B.steps,
            "lp_a": A.lp, "lp_b": B.lp, "lpdot": lpdot, "rhodot": rhodot, "h": h,
            "steps_a": A.steps, "steps_b": B.steps, "conv_a": A.converged, "conv_b": B.converged,
            "jumps": jumps, "rerun_chunks": rerun_chunks, "x": B.x, "jn": B.jn}
