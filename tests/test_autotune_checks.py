"""The autotuner's result checks, on the CPU with a stand-in for the library:
a candidate alpha or shape whose pi(x) differs from Table 1 (or from the
first candidate where Table 1 has no entry), or a batch whose values change
with alpha, stops the tuner instead of entering the tuning table."""
import sys
import types

import pytest

from paper_1503_01839_amd import autotune as A


def fake_library(bad_alpha=None, bad_batch_alpha=None):
    m = types.ModuleType("paper_1503_01839_amd")

    def pi_count_ex(x, alpha=0.0, segment_kib=0, wg_size=0):
        exact = {10**7: 664579, 10**8: 5761455}.get(x, 1000 + x % 97)
        return types.SimpleNamespace(pi=exact + (1 if alpha == bad_alpha else 0), ms_total=1.0)

    def pi_count_batch(xs, alpha=0.0):
        return [x % 1009 + (1 if alpha == bad_batch_alpha else 0) for x in xs]

    m.pi_count_ex = pi_count_ex
    m.pi_count_batch = pi_count_batch
    return m


@pytest.fixture
def swap_library(monkeypatch):
    def swap(**kw):
        monkeypatch.setitem(sys.modules, "paper_1503_01839_amd", fake_library(**kw))
    return swap


def quiet(*a, **k):
    pass


def test_consistent_candidates_pass(swap_library):
    swap_library()
    table = A.tune(7.0, 8.0, reps=1, log=quiet)
    assert [row[0] for row in table] == [7.0, 7.5, 8.0]
    A.tune_batch(table, reps=1, log=quiet)


def test_wrong_pi_at_a_power_of_ten_stops_the_tuner(swap_library):
    swap_library(bad_alpha=2)  # 10^7 and 10^8 are Table 1 rows
    with pytest.raises(A.ResultMismatch):
        A.tune(7.0, 7.0, reps=1, log=quiet)


def test_disagreeing_candidates_stop_the_tuner(swap_library):
    swap_library(bad_alpha=3)  # 10^7.5 is in no table: candidates must agree
    with pytest.raises(A.ResultMismatch):
        A.tune(7.5, 7.5, reps=1, log=quiet)


def test_batch_alpha_changing_results_stops_the_tuner(swap_library):
    swap_library(bad_batch_alpha=4)
    table = [(8.0, 4.0, 1.0, (32, 512), 4.0)]
    with pytest.raises(A.ResultMismatch):
        A.tune_batch(table, reps=1, log=quiet)
