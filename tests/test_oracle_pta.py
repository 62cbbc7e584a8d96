"""Pins of the PTA-step oracle (oracle/pta.py) on the CPU: its running
averages, state functions and control rules against independent
computations and hand-worked cases."""
import numpy as np
import pytest

import oracle as O
from oracle import junction_nodes as JN
from oracle import junctions as OJ
from oracle import pta
from paper_2005_02498_amd import workloads as W

Q = 2


def _tiny(seed=1_000_002, loops=2):
    inst = W.subset(W.burst_instance(seed), loops)
    inst.pinned[:] = 0
    return inst


def test_lp_from_rates_equals_direct_segment_sum():
    """L^p = (1/V) sum_s b_s (x) (t_s x vbar_s) L_s, computed directly from the
    oracle's velocities, equals sum_alpha gdot_alpha m_alpha (x) n_alpha built
    from the burst routine's resolved rates: glide keeps t x v along n."""
    inst = _tiny()
    mat = W.material()
    F = O.nodal_forces(inst.x, inst.seg_nodes, inst.burgers, inst.sigma_app, mat["mu"], mat["nu"],
                       mat["a"], Q)
    _, v = O.glide_step(inst.x, F, inst.seg_nodes, inst.normal, inst.pinned, mat["B"], W.DT)
    Lp = np.zeros((3, 3))
    for s in range(inst.n_segs):
        n1, n2 = inst.seg_nodes[:, s]
        d = inst.x[:, n2] - inst.x[:, n1]
        L = np.linalg.norm(d)
        vb = 0.5 * (v[:, n1] + v[:, n2])
        Lp += np.outer(inst.burgers[:, s], np.cross(d / L, vb)) * L / inst.volume
    _, rate, _ = O.burst(inst, mat, Q, 1, W.DT)
    np.testing.assert_allclose(pta.lp_from_rates(rate), Lp, rtol=0, atol=1e-12 * np.abs(Lp).max())
    assert np.abs(Lp).max() > 0


def test_density_is_total_line_length_over_volume():
    inst = _tiny()
    _, _, feat = O.burst(inst, W.material(), Q, 1, W.DT)
    d = inst.x[:, inst.seg_nodes[1]] - inst.x[:, inst.seg_nodes[0]]
    rho = np.linalg.norm(d, axis=0).sum() / inst.volume
    assert abs(feat[12:].sum() - rho) <= 1e-13 * rho


def test_running_average_equals_one_long_burst():
    """Chunked one-step accumulation (never converging) = the burst routine's
    own average over the same steps, and the same final state."""
    inst = _tiny()
    mat = W.material()
    P = pta.PTAParams(dt=W.DT, chunk=4, max_chunks=3, tol_rho=0.0, tol_lp=0.0)
    run, checks = pta.fast_run(inst, inst.x, inst.sigma_app, mat, Q, P)
    assert checks == 3 and run.steps == 12 and not run.converged
    x, rate, _ = O.burst(inst, mat, Q, 12, W.DT)
    np.testing.assert_allclose(run.sums[:12] / run.steps, rate, rtol=1e-12, atol=1e-12 * np.abs(rate).max())
    np.testing.assert_allclose(run.x, x, rtol=0, atol=1e-9)


def test_converged_rule_hand_cases():
    assert pta.converged(1.0, 1.005, 1e-2, abs)
    assert not pta.converged(1.0, 1.02, 1e-2, abs)
    assert pta.converged(0.0, 0.0, 1e-2, abs)
    a = np.eye(3)
    assert pta.converged(a, 1.02 * a, 3e-2, np.linalg.norm)
    assert not pta.converged(a, 1.05 * a, 3e-2, np.linalg.norm)


def test_first_check_never_converges_and_loose_tolerance_stops_at_second():
    inst = _tiny()
    P = pta.PTAParams(dt=W.DT, chunk=3, max_chunks=5, tol_rho=10.0, tol_lp=10.0)
    run, checks = pta.fast_run(inst, inst.x, inst.sigma_app, W.material(), Q, P)
    assert run.converged and checks == 2 and run.steps == 6


def test_pta_step_rules():
    inst = _tiny()
    mat = W.material()
    rate6 = np.array([0, 0, 1e15, 0, 0, 0.0])          # Pa/s: 50 MPa reached at t = 5e-8 s
    base = dict(dt=W.DT, chunk=3, max_chunks=3, delta=1e-8, tol_rho=1e-2, tol_lp=3e-2)
    # no jump allowed to trigger
    r = pta.pta_step(inst, 5e-8, rate6, mat, Q, pta.PTAParams(lpdot_max=np.inf, **base))
    assert r["jumps"] == 0
    nlp = np.linalg.norm(r["lp_b"])
    assert r["h"] == pytest.approx(min(1.0, 0.002 / nlp), rel=1e-15)
    np.testing.assert_allclose(r["lpdot"], (r["lp_b"] - r["lp_a"]) / 1e-8, rtol=1e-15)
    assert np.linalg.norm(r["lp_a"]) <= nlp or r["rerun_chunks"] == 3
    # every check a jump: exactly max_jumps restarts, the state moved on
    r2 = pta.pta_step(inst, 5e-8, rate6, mat, Q, pta.PTAParams(lpdot_max=0.0, max_jumps=2, **base))
    assert r2["jumps"] == 2
    assert r2["steps_a"] >= 6 and r2["steps_b"] >= 6
    assert np.abs(r2["x"] - r["x"]).max() > 0


def _junction_volume():
    inst = W.subset(W.burst_instance(1_000_030), 4)
    inst.pinned[:] = 0
    inst.pinned[64:] = 1                 # loops 3 and 4 are sessile
    ses = [s for s in range(inst.n_segs) if inst.pinned[inst.seg_nodes[0, s]] and inst.pinned[inst.seg_nodes[1, s]]]
    d2 = min(OJ._dist2(inst.x[:, n], inst.x[:, inst.seg_nodes[0, s]], inst.x[:, inst.seg_nodes[1, s]])
             for n in np.nonzero(inst.pinned == 0)[0] for s in ses)
    return inst, 1.5 * float(np.sqrt(d2))


def test_pta_with_zero_capture_radius_is_the_plain_step():
    inst, _ = _junction_volume()
    P = pta.PTAParams(dt=W.DT, delta=1e-8, chunk=2, max_chunks=2, lpdot_max=np.inf)
    rate = np.array([2e14, -1e14, 0, 3e14, 0, 1e14])
    ref = pta.pta_step(inst, 5e-8, rate, W.material(), Q, P)
    jn = pta.Junctions(0.0, 3 * W.DT, np.full((inst.n_nodes, 1), 0.5), OJ.new_state(inst.n_nodes), 7)
    got = pta.pta_step(inst, 5e-8, rate, W.material(), Q, P, jn)
    assert np.array_equal(got["x"], ref["x"]) and np.array_equal(got["lp_b"], ref["lp_b"])
    # the clock carried on is that of the end of the t run (step 5 steps excluded)
    assert got["jn"].fast == 7 + ref["steps_a"] - ref["rerun_chunks"] * P.chunk + ref["steps_b"]
    assert jn.fast == 7 and (jn.state["count"] == 0).all()      # the caller's state is not touched


def test_pta_with_junctions_is_the_step_by_step_junction_burst():
    """No jump and no step 5: the t - Delta run and the t run are, step for
    step, the junction burst routine of oracle/junctions.py at the volume's
    fast clock, one glide step per call; averages, positions and junction
    state agree exactly."""
    inst, r_c = _junction_volume()
    mat = W.material()
    P = pta.PTAParams(dt=W.DT, delta=1e-8, chunk=2, max_chunks=2, lpdot_max=np.inf)
    rate = np.array([2e14, -1e14, 0, 3e14, 0, 1e14])
    fr = np.random.default_rng(5).uniform(0.0, 1.0, (inst.n_nodes, 3))
    f0 = 11
    jn = pta.Junctions(r_c, 3 * W.DT, fr, OJ.new_state(inst.n_nodes), f0)
    got = pta.pta_step(inst, 5e-8, rate, mat, Q, P, jn)
    assert got["rerun_chunks"] == 0 and got["jumps"] == 0
    st = OJ.new_state(inst.n_nodes)
    x = np.array(inst.x, float)
    k = f0
    for sig, n_steps, key in ((5e-8 - 1e-8, got["steps_a"], "g_a"), (5e-8, got["steps_b"], "g_b")):
        acc = np.zeros(12)
        for _ in range(n_steps):
            s = W.Instance(x, inst.seg_nodes, inst.burgers, inst.normal, inst.pinned, sig * rate, inst.volume, {})
            x, r = OJ.burst(s, mat, Q, 1, W.DT, r_c, 3 * W.DT, float(k) * W.DT, fr, st)
            acc += r
            k += 1
        assert np.array_equal(got[key], acc / n_steps)
    assert np.array_equal(got["x"], x)
    for key in ("junction", "release", "ignore", "count"):
        assert np.array_equal(got["jn"].state[key], st[key]), key
    assert got["jn"].fast == k and st["count"].sum() > 0


def _forest(K=4, seed=2):
    inst = W.with_junction_slots(W.junction_forest(seed), K)
    return inst, JN.Params(capture_radius=10.0, max_break_time=3 * W.DT, l_min=2.0, n_slots=K)


def _nodes(inst, Pj, fast=0, seed=5):
    fr = np.random.default_rng(seed).uniform(0.0, 1.0, 3)
    return pta.JunctionNodes(Pj, JN.new_state(inst.n_nodes, inst.n_segs, fr), np.array(inst.seg_nodes),
                             np.array(inst.burgers), np.array(inst.normal), fast)


def test_pta_with_junction_nodes_and_zero_radius_is_the_plain_step():
    """A zero capture radius: the step is the plain PTA step of the slotted
    volume bit for bit (free slot segments add nothing), the topology is
    unchanged, and the fast clock advances by the steps of the carried path."""
    inst, Pj = _forest()
    Pj = JN.Params(0.0, Pj.a, Pj.l_min, Pj.K)
    P = pta.PTAParams(dt=W.DT, delta=1e-8, chunk=2, max_chunks=2, lpdot_max=np.inf)
    rate = np.array([0.0, 0.0, 4e15, 0.0, 0.0, 0.0])
    ref = pta.pta_step(inst, 5e-8, rate, W.material(), Q, P)
    jn = _nodes(inst, Pj, fast=7)
    got = pta.pta_step(inst, 5e-8, rate, W.material(), Q, P, jn)
    assert np.array_equal(got["x"], ref["x"]) and np.array_equal(got["lp_b"], ref["lp_b"])
    assert np.array_equal(got["jn"].seg_nodes, inst.seg_nodes)
    assert got["jn"].fast == 7 + ref["steps_a"] - ref["rerun_chunks"] * P.chunk + ref["steps_b"]
    assert jn.fast == 7 and jn.state["count"] == 0   # the caller's state is not touched


def test_pta_with_junction_nodes_is_the_step_by_step_node_burst():
    """No jump and no step 5: the t - Delta run and the t run are, step for
    step, the junction-node topology step of oracle/junction_nodes.py at the
    volume's fast clock followed by one glide step; averages, positions,
    topology and node state agree exactly, and junctions form."""
    inst, Pj = _forest()
    mat = W.material()
    P = pta.PTAParams(dt=W.DT, delta=1e-8, chunk=2, max_chunks=2, lpdot_max=np.inf)
    rate = np.array([0.0, 0.0, 4e15, 0.0, 0.0, 0.0])
    f0 = 11
    jn = _nodes(inst, Pj, fast=f0)
    got = pta.pta_step(inst, 5e-8, rate, mat, Q, P, jn)
    assert got["rerun_chunks"] == 0 and got["jumps"] == 0
    ref = _nodes(inst, Pj, fast=f0)
    x = np.array(inst.x, float)
    k = f0
    for sig, n_steps, key in ((5e-8 - 1e-8, got["steps_a"], "g_a"), (5e-8, got["steps_b"], "g_b")):
        acc = np.zeros(12)
        for _ in range(n_steps):
            JN.topology_step(x, ref.seg_nodes, ref.burgers, ref.normal, inst.pinned, float(k) * W.DT, Pj, ref.state)
            s = W.Instance(x, ref.seg_nodes, ref.burgers, ref.normal, inst.pinned, sig * rate, inst.volume, {})
            x, r, _ = O.burst(s, mat, Q, 1, W.DT)
            acc += r
            k += 1
        assert np.array_equal(got[key], acc / n_steps)
    assert np.array_equal(got["x"], x)
    for a, b in ((got["jn"].seg_nodes, ref.seg_nodes), (got["jn"].burgers, ref.burgers),
                 (got["jn"].normal, ref.normal)):
        assert np.array_equal(a, b)
    for key in ("release", "ses", "ignore", "point"):
        assert np.array_equal(got["jn"].state[key], ref.state[key]), key
    assert got["jn"].state["count"] == ref.state["count"] > 0
    assert got["jn"].fast == k
