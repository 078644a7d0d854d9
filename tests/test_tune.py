"""Autotuner search (CPU): a fake runner whose cost depends on the candidate, timed on a
fake clock, so the choice is checked without a GPU."""
from __future__ import annotations

import pytest

from paper_2204_05821_amd import tune


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def search(monkeypatch, cost, knobs, result=lambda cand: ([], [1, 2])):
    clock = FakeClock()
    monkeypatch.setattr(tune.time, "perf_counter", clock)

    class Runner:
        def __init__(self, cand):
            self.cand = cand

        def close(self):
            pass

    def run(r):
        clock.t += cost(r.cand) / 1e3
        return result(r.cand)

    return tune.autotune(Runner, run, key="test", rounds=3, reps=1, knobs=knobs, cache_path=None,
                         sync=lambda: None)


KN = [("key_bits", [0, 32, 64]), ("range_edges", [0, 1024, 2048]), ("scan_items", [8, 16])]


def reverse(knobs):
    return [(name, list(reversed(vals))) for name, vals in reversed(knobs)]


def test_differences_within_the_margin_keep_the_defaults_in_any_order(monkeypatch):
    # every candidate within 0.5% of the defaults: the defaults stay, whatever the order
    cost = lambda c: 100.0 - 0.4 * (c["key_bits"] == 32) - 0.3 * (c["range_edges"] == 1024)
    for kn in (KN, reverse(KN)):
        best, rep = search(monkeypatch, cost, kn)
        assert {k: best[k] for k in ("key_bits", "range_edges", "scan_items")} == \
            {"key_bits": 0, "range_edges": 0, "scan_items": 16}, rep["ms"][:3]


def test_a_clear_winner_is_taken_in_any_order(monkeypatch):
    cost = lambda c: 100.0 - 8.0 * (c["range_edges"] == 1024) - 5.0 * (c["scan_items"] == 8)
    for kn in (KN, reverse(KN)):
        best, _ = search(monkeypatch, cost, kn)
        assert best["range_edges"] == 1024 and best["scan_items"] == 8 and best["key_bits"] == 0


def test_every_value_is_timed_in_every_round(monkeypatch):
    _, rep = search(monkeypatch, lambda c: 10.0, KN)
    assert rep["rounds"] == 3 and all(len(v) >= 3 for v in rep["samples"].values())


def test_a_candidate_that_changes_the_result_is_an_error(monkeypatch):
    with pytest.raises(AssertionError):
        search(monkeypatch, lambda c: 10.0, KN, result=lambda c: ([], [1, 2 + (c["scan_items"] == 8)]))
