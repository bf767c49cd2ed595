"""Host logic of the cold / seeded / refresh schedule (section 2, paragraph
"Eigenvectors evolution"): decisions from recorded solve diagnostics."""
import pytest

from paper_1007_4400_amd.policy import RestartPolicy


def _info(sin, cost=1000):
    return {"seed_sin_rms": sin, "col_degrees": cost, "outer_iters": 3}


def test_direct_steps_then_seeded():
    p = RestartPolicy(direct_steps=2)
    assert p.next_mode() == "cold"
    p.record("cold", {"col_degrees": 5000})
    assert p.next_mode() == "cold"
    p.record("cold", {"col_degrees": 5000})
    assert p.next_mode() == "seeded"


def test_shrinking_angles_stay_seeded():
    p = RestartPolicy()
    p.record("cold", {})
    for s in (0.1, 0.06, 0.03, 0.015, 0.007):
        assert p.next_mode() == "seeded"
        p.record("seeded", _info(s))
    assert p.next_mode() == "seeded"


def test_flat_angles_refresh():
    p = RestartPolicy(flat_steps=2, flat_ratio=0.95)
    p.record("cold", {})
    for s in (0.1, 0.05):
        p.record("seeded", _info(s))
    assert p.next_mode() == "seeded"
    p.record("seeded", _info(0.049))  # flat once
    assert p.next_mode() == "seeded"
    p.record("seeded", _info(0.0485))  # flat twice: progress has flattened out
    assert p.next_mode() == "cold"
    p.record("cold", {})
    assert p.next_mode() == "seeded"  # a new series starts


def test_large_move_and_cost_growth_refresh():
    p = RestartPolicy(max_sin_rms=0.3)
    p.record("cold", {})
    p.record("seeded", _info(0.5))
    assert p.next_mode() == "cold"
    q = RestartPolicy(max_cost_growth=2.0)
    q.record("cold", {})
    q.record("seeded", _info(0.1, cost=1000))
    q.record("seeded", _info(0.05, cost=2500))
    assert q.next_mode() == "cold"


def test_seeded_step_needs_monitor():
    p = RestartPolicy()
    p.record("cold", {})
    with pytest.raises(ValueError):
        p.record("seeded", {"col_degrees": 10})


def test_settled_angles_are_not_flat():
    """A settled sequence reports angles at rounding level (or exactly zero):
    they do not shrink any more, but that is convergence, not stalled
    progress, so no refresh is forced; a flat series above the floor still is."""
    p = RestartPolicy(flat_steps=2, flat_ratio=0.95)
    p.record("cold", {})
    for s in (1e-4, 0.0, 0.0, 0.0, 0.0):
        p.record("seeded", _info(s))
        assert p.next_mode() == "seeded"
    q = RestartPolicy(flat_steps=2, flat_ratio=0.95, settled_sin_rms=1e-10)
    q.record("cold", {})
    for s in (1e-12, 1.1e-12, 1.2e-12):
        q.record("seeded", _info(s))
    assert q.next_mode() == "seeded"
    r = RestartPolicy(flat_steps=2, flat_ratio=0.95)
    r.record("cold", {})
    for s in (1e-6, 1e-6, 1e-6):
        r.record("seeded", _info(s))
    assert r.next_mode() == "cold"
