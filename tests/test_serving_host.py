"""Host-side checks of the serving loop's admission policy and request stream."""
import numpy as np

from paper_1711_01175_amd.serving import admit_backfill
from workloads.requests import request_stream


def test_admission_respects_slots_budget_and_order():
    waiting = [("a", 4), ("b", 3), ("c", 1), ("d", 2)]
    adm, rej = admit_backfill(waiting, n_active=0, used_bytes=0, slots=8, budget=8)
    assert adm == ["a", "b", "c"] and rej == []          # d would overflow the budget
    adm, rej = admit_backfill(waiting, n_active=6, used_bytes=0, slots=8, budget=100)
    assert adm == ["a", "b"]                               # two free slots
    adm, rej = admit_backfill(waiting, n_active=0, used_bytes=5, slots=8, budget=8)
    assert adm == []                                       # nothing running retires: no backfill
    adm, rej = admit_backfill([("x", 20), ("y", 2)], 0, 0, 4, 10)
    assert rej == ["x"] and adm == ["y"]                   # larger than the whole budget


def test_backfilling_never_delays_the_head():
    """budget 10, two running requests of 4 bytes each (5 and 20 steps
    left): a head of 6 fits once the first retires, with nothing to spare, so
    nothing passes it; a head of 5 leaves 1 byte spare at its reservation, so
    only a request of 1 byte that fits now may pass."""
    running = [(5, 4), (20, 4)]
    adm, _ = admit_backfill([("big", 6), ("small", 2), ("tiny", 1)], 2, 8, 8, 10, running)
    assert adm == []
    adm, _ = admit_backfill([("big", 5), ("small", 2), ("tiny", 1)], 2, 8, 8, 10, running)
    assert adm == ["tiny"]
    # a head that needs both retirements: 2 + 4 + 4 = 10 free then, 1 spare
    adm, _ = admit_backfill([("huge", 9), ("small", 2), ("tiny", 1), ("tiny2", 1)], 2, 8, 8, 10, running)
    assert adm == ["tiny"]
    # slots: 3 slots, 2 running; the head's reservation needs the slot freed
    # by the first retirement and the free slot stays spare
    adm, _ = admit_backfill([("big", 5), ("tiny", 1), ("tiny2", 1)], 2, 8, 3, 10, running)
    assert adm == ["tiny"]
    adm, _ = admit_backfill([("big", 5), ("tiny", 1)], 3, 8, 3, 10, running + [(30, 0)])
    assert adm == []                                       # no free slot now
    # requests retiring in the same chunk free their memory together
    adm, _ = admit_backfill([("big", 8), ("tiny", 2)], 2, 8, 8, 10, [(5, 4), (5, 4)])
    assert adm == ["tiny"]


def test_backfilling_in_a_simulated_serving_loop():
    """A small simulation of the serving loop (every running request advances
    one step per tick, 6 slots, 8 bytes): at every tick where the head of the
    queue waits, the requests admitted past it leave its reservation intact
    (replaying the running requests' retirements with them included frees
    the head's memory and slot no later than without them); over the whole
    stream requests start earlier than under strict arrival order, on
    average and at worst, and the stream ends no later."""
    import random
    rng = random.Random(5)
    reqs = [(i, rng.choice([1, 2, 3, 6]), rng.randint(3, 12)) for i in range(40)]   # (id, bytes, steps)
    slots, budget = 6, 8

    def fits_at(running, fp):
        """ticks until fp bytes and a slot are free, if nothing else is admitted"""
        free_b, free_s = budget - sum(r[1] for r in running), slots - len(running)
        for t, grp in enumerate(sorted({r[2] for r in running})):
            if free_b >= fp and free_s >= 1:
                return 0 if t == 0 else prev
            free_b += sum(r[1] for r in running if r[2] == grp)
            free_s += sum(1 for r in running if r[2] == grp)
            prev = grp
        return prev if running else 0

    def simulate(backfill):
        waiting, running, start, t = list(reqs), [], {}, 0
        while waiting or running:
            used = sum(r[1] for r in running)
            rel = [(r[2], r[1]) for r in running] if backfill else []
            adm, _ = admit_backfill([(r[0], r[1]) for r in waiting], len(running), used, slots, budget, rel)
            head = next((w for w in waiting if w[0] not in adm), None)
            passed = [w for w in waiting if w[0] in adm and head is not None and w[0] > head[0]]
            if passed:
                before = fits_at(running, head[1])
                after = fits_at(running + [[w[0], w[1], 10 ** 6] for w in passed], head[1])
                assert after <= before, (t, head, passed)
            for r in [w for w in waiting if w[0] in adm]:
                start[r[0]] = t
                running.append([r[0], r[1], r[2]])
            waiting = [w for w in waiting if w[0] not in adm]
            for r in running:
                r[2] -= 1
            running = [r for r in running if r[2] > 0]
            t += 1
        return start, t

    (fifo, t_fifo), (bf, t_bf) = simulate(False), simulate(True)
    assert sum(bf.values()) < sum(fifo.values())
    assert max(bf.values()) <= max(fifo.values())
    assert t_bf <= t_fifo


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


def test_media_sampled_with_torch_match_numpy():
    """The server samples media through torch's CPU kernels: the same
    formula as the numpy path, equal to within rounding."""
    import torch
    from workloads import media
    x = np.random.default_rng(3).uniform(-1, 1, size=(500, 11, 3))
    kw = dict(phases=(0.1, 0.2, 0.3, 0.4), amps=(1.1, 0.9, 1.2))
    for a, b in zip(media.smooth(x, **kw), media.smooth(torch.from_numpy(x), **kw)):
        assert isinstance(b, torch.Tensor) and b.dtype == torch.float64
        assert np.allclose(a, b.numpy(), rtol=4e-16, atol=0)
