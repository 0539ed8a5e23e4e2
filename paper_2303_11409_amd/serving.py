"""Serving form: continuous batching of boson-sampling simulations.

Requests (circuits) arrive over time.  A request is admitted as soon as it has
arrived and its state fits the HBM budget; every admitted request keeps its MPS
resident on the device between layers.  Each iteration of the loop advances
every active request by one brickwork layer, all of them together in one
``mps_apply_batch`` call (the batching form), so requests that arrive while
others run join the next iteration and their work shares the same launches.
Requests may be split into lanes (for instance large circuits apart from small
ones): each lane runs this loop in its own host thread on its own stream, so
an iteration of one lane does not wait for the slowest sector of another and
the lanes' kernels fill the device together.
A request whose last layer is done is retired: its result (norm, summed
discarded weight, sampled amplitudes) is read out, its device memory returns to
the budget and its latency (arrival to result) is recorded.  A request whose
footprint alone exceeds the budget can never be admitted: it is refused (it
gets an error result at once) and the loop goes on with the others.

The per-request device footprint used for admission is the state's allocation
bound: site tensors of cap[s] x cap[s+1] complex128 and Schmidt vectors of
cap[b] doubles, where cap[b] = min(chi_max, sum_c min(#left strings with N - c
photons, #right strings with c photons)) is the largest dimension bond b can
reach (the Fock-space bound of the U(1) charges), plus the two Theta
workspaces of its largest update.
"""
from __future__ import annotations

import functools
import math
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from .binding import MPS, apply_batch


def _strings(sites: int, d: int, n_max: int) -> List[int]:
    """Number of occupation strings of `sites` modes, occupations < d, with n photons."""
    cnt = [1] + [0] * n_max
    for _ in range(sites):
        nxt = [0] * (n_max + 1)
        for n, c in enumerate(cnt):
            if c:
                for k in range(d):
                    if n + k <= n_max:
                        nxt[n + k] += c
        cnt = nxt
    return cnt


@functools.lru_cache(maxsize=None)
def _bond_caps(L: int, N: int, d: int, chi_max: int) -> tuple:
    caps = []
    for b in range(L + 1):
        left, right = _strings(b, d, N), _strings(L - b, d, N)
        tot = sum(min(left[N - c], right[c]) for c in range(N + 1))
        if chi_max > 0:
            tot = min(tot, chi_max)
        caps.append(max(1, tot))
    return tuple(caps)


def bond_caps(L: int, N: int, d: int, chi_max: int) -> List[int]:
    """Largest dimension each bond of an N-photon state on L modes can reach."""
    return list(_bond_caps(int(L), int(N), int(d), int(chi_max)))


def state_bytes(L: int, N: int, d: int, chi_max: int) -> int:
    """Device bytes a request may hold: its state plus its largest update's Theta
    workspaces (the sectors of one update hold at most d * cap_s * cap_{s+2}
    entries, raw and scaled)."""
    caps = bond_caps(L, N, d, chi_max)
    state = sum(16 * caps[s] * caps[s + 1] for s in range(L)) + sum(8 * c for c in caps)
    theta = max(2 * 16 * d * caps[s] * caps[s + 2] for s in range(L - 1)) if L > 1 else 0
    return state + theta


@dataclass
class Request:
    """A simulation request.  spec names the circuit (L, n_photons, d, chi_max
    and whatever build needs); the circuit (occupation, layers, gates, cutoff)
    and the patterns are built when the request is admitted."""
    rid: int
    arrival: float                     # seconds since the start of the run
    spec: dict
    build: Callable[[dict], dict]      # spec -> circuit
    n_patterns: int = 16
    pattern_seed: int = 0
    cfg: Optional[dict] = None
    patterns: Optional[np.ndarray] = None
    bytes: int = 0
    state: Optional[MPS] = None
    next_layer: int = 0
    discarded: float = 0.0
    admitted_at: float = math.nan
    done_at: float = math.nan
    result: Optional[dict] = None
    refused: Optional[str] = None      # why the request was refused admission

    def materialize(self) -> None:
        from workloads import circuits as _c  # circuit and pattern generators (inputs only)
        if self.cfg is None:
            self.cfg = self.build(self.spec)
        if self.patterns is None:
            self.patterns = _c.sample_patterns(self.spec["L"], self.spec["n_photons"], self.spec["d"],
                                               self.n_patterns, self.pattern_seed)


@dataclass
class ServeReport:
    completed: List[Request] = field(default_factory=list)
    refused: List[Request] = field(default_factory=list)
    unfinished: List[Request] = field(default_factory=list)   # arrived, not done when the run ended
    pending: int = 0                   # len(unfinished)
    iterations: int = 0
    gates: int = 0
    seconds: float = 0.0
    peak_active: int = 0
    peak_bytes: int = 0

    def latencies(self) -> np.ndarray:
        """Arrival to result of the completed requests."""
        return np.array([r.done_at - r.arrival for r in self.completed])

    def censored_latencies(self) -> np.ndarray:
        """Every arrived, admissible request: the completed ones' latencies and,
        for a request still waiting or running when the run ended, the time from
        its arrival to the end (a lower bound of its latency).  Percentiles of
        this set are lower bounds of the percentiles over all arrivals."""
        done = [r.done_at - r.arrival for r in self.completed]
        cut = [max(0.0, self.seconds - r.arrival) for r in self.unfinished]
        return np.array(done + cut)


def finish(req: Request) -> dict:
    m = req.state
    return {"norm2": m.norm2(), "discarded": req.discarded, "amplitudes": m.amplitudes(req.patterns),
            "bond_dims": m.bond_dims()}


class Server:
    """Continuous-batching loop over a fixed list of requests with arrival times.

    hbm_budget: bytes of device memory the admitted requests may hold together
    (shared by all lanes).
    max_active: upper bound on simultaneously admitted requests per lane (an
    int for every lane, or one value per lane).
    devices: one TorchDevice per lane (each with its own stream); None means one
    lane on the default device.  Each lane is a host thread that runs the loop
    on its own requests and stream, so the lanes' launches share the device.
    lane_of: request spec -> lane index (default: lane 0).
    clock: returns seconds since the start (monotonic); tests may pass a
    simulated clock.
    state_opts: extra keyword options of every request's MPS (for instance
    sweep_graph=1)."""

    def __init__(self, hbm_budget: int, max_active=1024, device=None,
                 clock: Optional[Callable[[], float]] = None, devices: Optional[Sequence] = None,
                 lane_of: Optional[Callable[[dict], int]] = None, state_opts: Optional[dict] = None):
        self.hbm_budget = int(hbm_budget)
        self.state_opts = dict(state_opts or {})
        self.devices = list(devices) if devices else [device]
        nl = len(self.devices)
        ma = list(max_active) if isinstance(max_active, (list, tuple)) else [max_active] * nl
        if len(ma) != nl:
            raise ValueError("one max_active per lane")
        self.max_active = [int(x) for x in ma]
        self.lane_of = lane_of or (lambda spec: 0)
        self._t0 = None
        self._clock = clock
        self._lock = threading.Lock()

    def now(self) -> float:
        if self._clock is not None:
            return self._clock()
        return time.perf_counter() - self._t0

    def run(self, requests: Sequence[Request], until: Optional[float] = None) -> ServeReport:
        """Serve the requests until all are done or `until` seconds have passed;
        returns the report."""
        self._t0 = time.perf_counter()
        nl = len(self.devices)
        queues: List[List[Request]] = [[] for _ in range(nl)]
        rep = ServeReport()
        for r in sorted(requests, key=lambda r: r.arrival):
            sp = r.spec
            r.bytes = state_bytes(sp["L"], sp["n_photons"], sp["d"], sp["chi_max"])
            lane = int(self.lane_of(sp))
            if not 0 <= lane < nl:
                raise ValueError(f"lane {lane} of request {r.rid} outside 0..{nl - 1}")
            queues[lane].append(r)
        self._used = 0
        self._active_total = 0
        errors: List[BaseException] = []
        pending: List[List[Request]] = [[] for _ in range(nl)]

        def lane_loop(k: int) -> None:
            try:
                pending[k] = self._lane(k, queues[k], rep, until)
            except BaseException as e:          # re-raised by run()
                errors.append(e)

        if nl == 1:
            lane_loop(0)
        else:
            threads = [threading.Thread(target=lane_loop, args=(k,), daemon=True) for k in range(nl)]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
        if errors:
            raise errors[0]
        rep.seconds = self.now()
        rep.unfinished = sorted((r for p in pending for r in p), key=lambda r: r.arrival)
        rep.pending = len(rep.unfinished)
        rep.refused.sort(key=lambda r: r.arrival)
        return rep

    def _lane(self, k: int, queue: List[Request], rep: ServeReport, until: Optional[float]) -> List[Request]:
        active: List[Request] = []
        qi = 0
        try:
            while qi < len(queue) or active:
                t = self.now()
                if until is not None and t >= until:
                    break
                # admit every arrived request of this lane that fits, in arrival order
                while qi < len(queue) and queue[qi].arrival <= t and len(active) < self.max_active[k]:
                    r = queue[qi]
                    if r.bytes > self.hbm_budget:
                        # can never fit: refuse it and serve the others
                        r.refused = f"needs {r.bytes} bytes of device memory, more than the budget"
                        r.result = {"error": r.refused}
                        r.done_at = t
                        with self._lock:
                            rep.refused.append(r)
                        qi += 1
                        continue
                    with self._lock:
                        if self._used + r.bytes > self.hbm_budget:
                            break
                        self._used += r.bytes
                        self._active_total += 1
                        rep.peak_active = max(rep.peak_active, self._active_total)
                        rep.peak_bytes = max(rep.peak_bytes, self._used)
                    r.materialize()
                    c = r.cfg
                    r.state = MPS(c["occupation"], c["d"], chi_max=c["chi_max"], cutoff=c["cutoff"],
                                  device=self.devices[k], **self.state_opts)
                    r.admitted_at = t
                    active.append(r)
                    qi += 1
                if not active:
                    # idle until the next arrival
                    if qi < len(queue):
                        wait = queue[qi].arrival - self.now()
                        if wait > 0 and self._clock is None:
                            time.sleep(min(wait, 0.01))
                    continue
                # one layer of every active request of this lane, together
                layers = []
                ng = 0
                for r in active:
                    lay = r.cfg["layers"][r.next_layer]
                    layers.append(([g.site for g in lay], [g.u for g in lay]))
                    ng += len(lay)
                disc = apply_batch([r.state for r in active], layers)
                still = []
                done = []
                for r, dsc in zip(active, disc):
                    r.discarded += float(np.sum(dsc))
                    r.next_layer += 1
                    if r.next_layer >= len(r.cfg["layers"]):
                        r.result = finish(r)
                        r.done_at = self.now()
                        r.state.close()
                        r.state = None
                        done.append(r)
                    else:
                        still.append(r)
                active = still
                with self._lock:
                    rep.gates += ng
                    rep.iterations += 1
                    for r in done:
                        self._used -= r.bytes
                        self._active_total -= 1
                        rep.completed.append(r)
        finally:
            for r in active:
                if r.state is not None:
                    r.state.close()
                    r.state = None
        end = self.now()
        return active + [r for r in queue[qi:] if r.arrival < end and r.bytes <= self.hbm_budget]


def poisson_requests(specs: Sequence[dict], rate: float, seed: int, build: Optional[Callable] = None,
                     n_patterns: int = 16, pattern_seed0: int = 5000) -> List[Request]:
    """Requests for the given specs with exponential inter-arrival times of mean
    1/rate (numpy.random.default_rng(seed)); request j returns the amplitudes
    of n_patterns uniform patterns drawn with seed pattern_seed0 + j.  A spec
    that is already a circuit (has "layers") needs no build."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j, sp in enumerate(specs):
        t += float(rng.exponential(1.0 / rate))
        if "layers" in sp:
            spec = dict(sp, n_photons=sum(sp["occupation"]))
            fn = lambda s, c=sp: c
        else:
            spec, fn = sp, build
        out.append(Request(rid=j, arrival=t, spec=spec, build=fn, n_patterns=n_patterns,
                           pattern_seed=pattern_seed0 + j))
    return out
