"""The surrogate's gain over DD at equal error, on a small held-out set
(paper_2005_02498_amd/surrogate_study.py; the reduced configuration of
bench.py's live study).  8,192 training bursts (4,096 states x 2
microstructures) of 200 mixed-precision glide steps, 64 held-out states x 8
microstructures.  Errors are relative to each held-out state's mean rates,
with the reference's own noise removed; DD needs n(e) = ceil(E1^2 / e^2)
bursts per state for an error e (E1: one burst against its state's mean)."""
import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_beats_dd_at_equal_error():
    import paper_2005_02498_amd as dd
    from paper_2005_02498_amd import surrogate_study as S

    prev = dd.dd_set_validation(False)
    try:
        st = S.study(4096, 2, 64, 8, 100, learning_curve=False)
    finally:
        dd.dd_set_validation(prev)
    b = st["per_burst_targets"]
    a = b["at_surrogate_error"]
    print(f"E1 {b['error_single_burst']:.3f}, surrogate {b['error_surrogate']:.3f} "
          f"(evaluation half {b['error_surrogate_evaluation_half']:.3f}); DD bursts for that error "
          f"{a['dd_bursts_per_state']}; calibrated fallback {a['fallback_fraction']:.2f}, "
          f"speed-up {a['speedup']:.2f} ({a['speedup_without_fallback']:.3g} without fallback); "
          f"error by spread quartile {[round(e, 3) for e in b['error_by_spread_quartile']]}")
    # the network is more accurate than one DD burst: DD needs at least two
    # bursts per state to match it
    assert b["error_surrogate"] < 0.8 * b["error_single_burst"]
    assert a["dd_bursts_per_state"] >= 2
    # at that error, with the threshold calibrated on the other half of the
    # held-out states, some states keep the surrogate's answer and the cost
    # per state is below DD's
    assert a["fallback_fraction"] < 1.0
    assert a["speedup"] > 1.0
    # the ensemble spread ranks the errors: the highest-spread quartile is
    # worse than the lowest
    q = b["error_by_spread_quartile"]
    assert q[3] > q[0]
