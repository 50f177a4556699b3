"""Pins for the weak predictor reference (Section 4.3, Fig. 6 text)."""
import json
import os

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_default_diagram_matches_text():
    fx = json.load(open(os.path.join(GOLDEN, "weak_pvu_sec4_3.json")))
    ns, init, mask, succ, fail = oracle.weak_default_diagram()
    assert ns == 6 and init == fx["initial_state"]
    assert sorted(i for i in range(ns) if mask >> i & 1) == fx["attempt_states"]
    assert sorted(i for i in range(ns) if not mask >> i & 1) == fx["dormant_states"]
    for t in fx["transitions_stated_in_text"]:
        assert oracle.weak_next(t["state"], t["changed"]) == t["next"], t
    for t in fx["reading_not_in_text"]:
        for ch in (False, True):   # dormant states move regardless of outcome
            assert oracle.weak_next(t["state"], ch) == t["next"], t


def test_state3_has_failed_twice_and_sleeps_two_iterations():
    # any path into state 3 from an attempt needs two failures in a row
    s = 0
    s = oracle.weak_next(s, False); assert s == 5
    s = oracle.weak_next(s, False); assert s == 3
    _, _, mask, _, _ = oracle.weak_default_diagram()
    attempts = []
    for _ in range(8):
        attempts.append(bool(mask >> s & 1))
        s = oracle.weak_next(s, False)
    # 3 (sleep), 2 (sleep), 1 (attempt, fails -> 4), 4, 3, 2 sleep, 1 attempt ...
    assert attempts == [False, False, True, False, False, False, True, False]


def test_any_success_returns_to_initial():
    for st in (0, 1, 5):
        assert oracle.weak_next(st, True) == 0


def test_invalid_state():
    assert oracle.weak_next(7, False) == -1
