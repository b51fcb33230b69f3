"""Host-side checks of the serving loop's admission policy and request stream."""
import numpy as np

from paper_1711_01175_amd.serving import admit_fifo
from workloads.requests import request_stream


def test_admission_respects_slots_budget_and_order():
    waiting = [("a", 4), ("b", 3), ("c", 1), ("d", 2)]
    adm, rej = admit_fifo(waiting, n_active=0, used_bytes=0, slots=8, budget=8)
    assert adm == ["a", "b", "c"] and rej == []          # d would overflow the budget
    adm, rej = admit_fifo(waiting, n_active=6, used_bytes=0, slots=8, budget=100)
    assert adm == ["a", "b"]                               # two free slots
    adm, rej = admit_fifo(waiting, n_active=0, used_bytes=5, slots=8, budget=8)
    assert adm == []                                       # head of line blocks
    adm, rej = admit_fifo([("x", 20), ("y", 2)], 0, 0, 4, 10)
    assert rej == ["x"] and adm == ["y"]                   # larger than the whole budget


def test_request_stream_is_seeded_and_poisson():
    a = request_stream(64, rate=10.0)
    b = request_stream(64, rate=10.0)
    assert [r.n for r in a] == [r.n for r in b]
    assert all(8 <= r.n <= 24 and r.N in (3, 4, 5) for r in a)
    assert all(np.all(np.abs(r.xs) <= 0.9) for r in a)
    gaps = np.diff([r.arrival for r in a])
    assert np.all(gaps >= 0) and abs(gaps.mean() - 0.1) < 0.05
    assert [r.arrival for r in request_stream(8)] == [0.0] * 8


def test_energy_guard_decisions():
    """A request is stopped when its energy is NaN or infinite, or grows by
    more than the limit within one chunk once it is positive; growth from
    zero (the source switching on) and ordinary growth pass."""
    from paper_1711_01175_amd.serving import energy_check
    assert energy_check(0.0, 1e-20, 1e6) is None
    assert energy_check(1e-20, 1e-16, 1e6) is None
    assert energy_check(1.0, 1e6, 1e6) is None
    assert "grew" in energy_check(1.0, 1.0000001e6, 1e6)
    assert energy_check(1.0, float("nan"), 1e6) == "non-finite energy"
    assert energy_check(0.0, float("inf"), 1e6) == "non-finite energy"
    assert energy_check(1.0, 1e30, None) is None
