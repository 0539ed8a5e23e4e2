"""Host logic of the serving form (CPU): the bond-dimension bound used for HBM
admission, and the continuous-batching scheduler driven with a stand-in state
class (no device)."""
import itertools

import numpy as np
import pytest

from paper_2303_11409_amd import serving
from workloads import circuits


def brute_caps(L, N, d):
    """Schmidt-rank bound of every cut of an N-photon state with occupations < d,
    by enumerating the strings on each side."""
    caps = []
    for b in range(L + 1):
        left = {}
        for s in itertools.product(range(d), repeat=b):
            left[sum(s)] = left.get(sum(s), 0) + 1
        right = {}
        for s in itertools.product(range(d), repeat=L - b):
            right[sum(s)] = right.get(sum(s), 0) + 1
        caps.append(max(1, sum(min(left.get(N - c, 0), right.get(c, 0)) for c in range(N + 1))))
    return caps


@pytest.mark.parametrize("L,N,d", [(6, 3, 4), (7, 4, 3), (5, 5, 2), (8, 4, 5)])
def test_bond_caps_match_enumeration(L, N, d):
    assert serving.bond_caps(L, N, d, 0) == brute_caps(L, N, d)
    capped = serving.bond_caps(L, N, d, 5)
    assert capped == [min(5, c) for c in brute_caps(L, N, d)]


class FakeState:
    live = 0

    def __init__(self, occ, d, chi_max=0, cutoff=0.0, device=None):
        self.occ = list(occ)
        FakeState.live += 1

    def close(self):
        FakeState.live -= 1

    def norm2(self):
        return 1.0

    def amplitudes(self, p):
        return np.zeros(len(p), dtype=np.complex128)

    def bond_dims(self):
        return [1] * (len(self.occ) + 1)


def test_scheduler_continuous_batching_and_budget(monkeypatch):
    calls = []

    def fake_batch(states, layers):
        calls.append(len(states))
        return [np.zeros(len(s)) for s, _ in layers]

    monkeypatch.setattr(serving, "MPS", FakeState)
    monkeypatch.setattr(serving, "apply_batch", fake_batch)
    cfgs = circuits.config_batch_mix(6, seed=3, l_range=(6, 10), chi_choices=(8, 16))
    reqs = serving.poisson_requests(cfgs, rate=1.0, seed=1, n_patterns=4)
    for i, r in enumerate(reqs):            # arrivals in simulated time units
        r.arrival = [0, 0, 3, 4, 30, 31][i]
    clock = {"t": -1.0}

    def tick():
        clock["t"] += 1.0
        return clock["t"]

    per = [serving.state_bytes(c["L"], sum(c["occupation"]), 4, c["chi_max"]) for c in cfgs]
    budget = max(per) * 2                   # at most about two requests at a time
    rep = serving.Server(budget, clock=tick).run(reqs)
    assert len(rep.completed) == 6 and rep.pending == 0
    assert rep.peak_bytes <= budget
    assert FakeState.live == 0              # every state released
    assert max(calls) >= 2                  # requests overlapped in one batch call
    assert rep.gates == sum(len(c["gates"]) for c in cfgs)
    for r in rep.completed:
        assert r.done_at >= r.admitted_at >= r.arrival
        assert r.result["amplitudes"].shape == (4,)


def test_scheduler_refuses_oversized_request_and_keeps_serving(monkeypatch):
    """A request whose footprint exceeds the whole budget is refused at its
    arrival (error result, no state created) while the others are served."""
    def fake_batch(states, layers):
        return [np.zeros(len(s)) for s, _ in layers]

    monkeypatch.setattr(serving, "MPS", FakeState)
    monkeypatch.setattr(serving, "apply_batch", fake_batch)
    small = circuits.config_batch_mix(3, seed=3, l_range=(6, 8), chi_choices=(8,))
    big = circuits.config_batch_mix(1, seed=5, l_range=(12, 12), chi_choices=(64,))
    cfgs = [small[0], big[0], small[1], small[2]]
    reqs = serving.poisson_requests(cfgs, rate=1.0, seed=1, n_patterns=4)
    for i, r in enumerate(reqs):
        r.arrival = [0, 1, 2, 3][i]
    clock = {"t": -1.0}

    def tick():
        clock["t"] += 1.0
        return clock["t"]

    per = [serving.state_bytes(c["L"], sum(c["occupation"]), 4, c["chi_max"]) for c in cfgs]
    budget = 2 * max(per[0], per[2], per[3])
    assert per[1] > budget
    rep = serving.Server(budget, clock=tick).run(reqs)
    assert [r.rid for r in rep.refused] == [1]
    assert "error" in rep.refused[0].result and rep.refused[0].state is None
    assert sorted(r.rid for r in rep.completed) == [0, 2, 3]
    assert rep.pending == 0 and FakeState.live == 0


def test_scheduler_reports_unfinished_requests_as_censored(monkeypatch):
    """A window that ends while requests wait or run reports them: pending
    counts them, and the censored latencies (arrival to the window's end) join
    the completed ones, so percentiles over all arrivals are not computed over
    the survivors only."""
    def fake_batch(states, layers):
        return [np.zeros(len(s)) for s, _ in layers]

    monkeypatch.setattr(serving, "MPS", FakeState)
    monkeypatch.setattr(serving, "apply_batch", fake_batch)
    cfgs = circuits.config_batch_mix(5, seed=3, l_range=(6, 8), chi_choices=(8,))
    reqs = serving.poisson_requests(cfgs, rate=1.0, seed=1, n_patterns=4)
    for i, r in enumerate(reqs):
        r.arrival = [0, 0, 0, 0, 0][i]
    clock = {"t": -1.0}

    def tick():
        clock["t"] += 1.0
        return clock["t"]

    per = [serving.state_bytes(c["L"], sum(c["occupation"]), 4, c["chi_max"]) for c in cfgs]
    rep = serving.Server(sum(per), max_active=1, clock=tick).run(reqs, until=12.0)
    assert 0 < len(rep.completed) < 5
    assert rep.pending == 5 - len(rep.completed) == len(rep.unfinished)
    cens = rep.censored_latencies()
    assert cens.size == 5
    assert np.all(cens[len(rep.completed):] >= 0.0)
    assert cens.max() >= rep.latencies().max()
    assert FakeState.live == 0


def test_scheduler_lanes(monkeypatch):
    """Two lanes (threads): every request runs in its own lane, all complete, the
    shared budget holds."""
    lanes_seen = {}

    class LaneState(FakeState):
        def __init__(self, occ, d, chi_max=0, cutoff=0.0, device=None):
            super().__init__(occ, d, chi_max, cutoff, device)
            self.device = device

    def fake_batch(states, layers):
        devs = {id(s.device) for s in states}
        assert len(devs) == 1                  # a batch never mixes lanes
        for s in states:
            lanes_seen[len(s.occ)] = s.device
        return [np.zeros(len(s)) for s, _ in layers]

    monkeypatch.setattr(serving, "MPS", LaneState)
    monkeypatch.setattr(serving, "apply_batch", fake_batch)
    cfgs = circuits.config_batch_mix(8, seed=3, l_range=(6, 12), chi_choices=(8, 16))
    reqs = serving.poisson_requests(cfgs, rate=1e6, seed=1, n_patterns=4)
    dev_small, dev_large = object(), object()
    per = [serving.state_bytes(c["L"], sum(c["occupation"]), 4, c["chi_max"]) for c in cfgs]
    srv = serving.Server(3 * max(per), devices=[dev_large, dev_small],
                         lane_of=lambda sp: 0 if sp["L"] >= 10 else 1)
    rep = srv.run(reqs)
    assert len(rep.completed) == 8 and rep.pending == 0 and FakeState.live == 0
    assert rep.peak_bytes <= 3 * max(per)
    for L, dev in lanes_seen.items():
        assert dev is (dev_large if L >= 10 else dev_small)
