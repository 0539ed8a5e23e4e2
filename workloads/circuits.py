"""Seeded synthetic circuits and occupation patterns for linear-optics boson sampling.

This module is input generation only.  It produces the gate lists (two-mode
2x2 unitaries on adjacent modes) and the occupation patterns that both the
CPU oracle and the GPU library consume.  It holds none of the matrix-product
state arithmetic: no Fock-space gate elements, no contraction, no SVD.

Conventions (readings of the paper, which states no gate convention):

* A circuit is a list of ``Gate(site, u)`` applied in list order.  ``site``
  is the 0-based left mode; the gate acts on modes ``site`` and ``site+1``.
* A 2x2 (or LxL) mode unitary maps creation operators column-wise,
  ``a_j^dagger -> sum_i U[i, j] a_i^dagger``.  The whole circuit's mode
  unitary is ``U = U_G ... U_2 U_1``.
* Brickwork beam splitter ``u(theta, phi) = [[cos t, -e^{-i phi} sin t],
  [e^{i phi} sin t, cos t]]`` with ``theta ~ U[0, pi/2]``, ``phi ~ U[0, 2 pi)``,
  drawn theta-then-phi per gate from ``numpy.random.default_rng(seed)``.
  Layer ``l`` holds gates on ``(j, j+1)`` for ``j = l mod 2, l mod 2 + 2, ...``.
* Haar unitary by Mezzadri's recipe (QR of a complex Gaussian matrix with the
  phases of R's diagonal moved into Q).
* Clements rectangular mesh (Clements et al., Optica 3, 1460 (2016)): nulling
  alternately with column and row operations, then the left factors are
  pushed through the diagonal so every factor sits on the input side.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np


@dataclass(frozen=True)
class Gate:
    site: int            # 0-based left mode; acts on (site, site+1)
    u: np.ndarray        # 2x2 complex128 mode unitary

    def __post_init__(self):
        u = np.asarray(self.u, dtype=np.complex128)
        if u.shape != (2, 2):
            raise ValueError("gate unitary must be 2x2")
        object.__setattr__(self, "u", u)


def beam_splitter(theta: float, phi: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -np.exp(-1j * phi) * s],
                     [np.exp(1j * phi) * s, c]], dtype=np.complex128)


def haar_unitary(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def embed(u2: np.ndarray, site: int, n: int) -> np.ndarray:
    """The n x n mode unitary of a two-mode gate (identity elsewhere)."""
    m = np.eye(n, dtype=np.complex128)
    m[site:site + 2, site:site + 2] = u2
    return m


def circuit_unitary(gates: Sequence[Gate], n: int) -> np.ndarray:
    """U = U_G ... U_1 for the gate list (first gate applied first)."""
    u = np.eye(n, dtype=np.complex128)
    for g in gates:
        u[g.site:g.site + 2, :] = g.u @ u[g.site:g.site + 2, :]
    return u


def _col_null(a: complex, b: complex) -> np.ndarray:
    """2x2 unitary R with (a, b) @ R = (0, rho)."""
    rho = math.hypot(abs(a), abs(b))
    if rho == 0.0:
        return np.eye(2, dtype=np.complex128)
    return np.array([[b, np.conj(a)], [-a, np.conj(b)]], dtype=np.complex128) / rho


def _row_null(a: complex, b: complex) -> np.ndarray:
    """2x2 unitary Lm with Lm @ (a, b)^T = (rho, 0)^T."""
    rho = math.hypot(abs(a), abs(b))
    if rho == 0.0:
        return np.eye(2, dtype=np.complex128)
    return np.array([[np.conj(a), np.conj(b)], [-b, a]], dtype=np.complex128) / rho


def clements_gates(u: np.ndarray) -> Tuple[List[Gate], np.ndarray]:
    """Decompose an n x n unitary into n(n-1)/2 adjacent two-mode unitaries
    in the rectangular (Clements) arrangement, plus an output phase screen.

    Returns ``(gates, phases)`` where ``circuit_unitary(gates) `` times
    ``diag(phases)`` on the output side reconstructs ``u``; the phases that
    differ from 1 are also appended to ``gates`` as diagonal two-mode gates by
    ``clements_circuit``.
    """
    n = u.shape[0]
    v = np.array(u, dtype=np.complex128, copy=True)
    right: List[Tuple[int, np.ndarray]] = []   # v <- v @ R on columns (c, c+1)
    left: List[Tuple[int, np.ndarray]] = []    # v <- Lm @ v on rows (r-1, r)
    for i in range(1, n):
        if i % 2 == 1:
            for j in range(i):
                row, col = n - 1 - j, i - 1 - j
                r = _col_null(v[row, col], v[row, col + 1])
                v[:, col:col + 2] = v[:, col:col + 2] @ r
                right.append((col, r))
        else:
            for j in range(1, i + 1):
                row, col = n + j - i - 1, j - 1
                lm = _row_null(v[row - 1, col], v[row, col])
                v[row - 1:row + 1, :] = lm @ v[row - 1:row + 1, :]
                left.append((row - 1, lm))
    dvec = np.diag(v).copy()
    # u = (L_1^-1 ... L_k^-1) D (R_m^-1 ... R_1^-1); push D leftwards.
    ws: List[Tuple[int, np.ndarray]] = []
    for a, lm in reversed(left):
        w2 = lm.conj().T @ np.diag(dvec[a:a + 2])
        dvec[a] = 1.0
        dvec[a + 1] = 1.0
        ws.append((a, w2))
    # application order: R_1^-1 ... R_m^-1, then W_k ... W_1 (ws is W_k first)
    gates = [Gate(c, r.conj().T) for c, r in right]
    gates += [Gate(a, w2) for a, w2 in ws]
    return gates, dvec


def clements_circuit(u: np.ndarray, phase_tol: float = 1e-15) -> List[Gate]:
    """Full gate list realising ``u``: the mesh, then diagonal two-mode gates
    carrying the output phases that are not 1."""
    n = u.shape[0]
    gates, dvec = clements_gates(u)
    todo = [k for k in range(n) if abs(dvec[k] - 1.0) > phase_tol]
    done = set()
    for k in todo:
        if k in done:
            continue
        s = k if k + 1 < n else k - 1
        g = np.diag([dvec[s], dvec[s + 1]]).astype(np.complex128)
        done.update((s, s + 1))
        gates.append(Gate(s, g))
    return gates


def brickwork(n_modes: int, depth: int, seed: int) -> List[Gate]:
    """Seeded brickwork of beam splitters; layer l acts on (j, j+1), j = l mod 2 (step 2)."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for layer in range(depth):
        for j in range(layer % 2, n_modes - 1, 2):
            theta = rng.uniform(0.0, math.pi / 2)
            phi = rng.uniform(0.0, 2 * math.pi)
            gates.append(Gate(j, beam_splitter(theta, phi)))
    return gates


def brickwork_layers(n_modes: int, depth: int, seed: int) -> List[List[Gate]]:
    """The same gates as ``brickwork`` grouped by layer (gates of one layer act on disjoint pairs)."""
    gates = brickwork(n_modes, depth, seed)
    layers: List[List[Gate]] = []
    k = 0
    for layer in range(depth):
        cnt = len(range(layer % 2, n_modes - 1, 2))
        layers.append(gates[k:k + cnt])
        k += cnt
    return layers


def count_patterns(n_modes: int, n_photons: int, d: int) -> int:
    """Number of occupation strings with the given total and every occupation < d."""
    table = _suffix_counts(n_modes, n_photons, d)
    return table[0][n_photons]


def _suffix_counts(n_modes: int, n_photons: int, d: int):
    # cnt[k][n] = strings over modes k..L-1 with total n, each entry < d
    cnt = [[0] * (n_photons + 1) for _ in range(n_modes + 1)]
    cnt[n_modes][0] = 1
    for k in range(n_modes - 1, -1, -1):
        for n in range(n_photons + 1):
            cnt[k][n] = sum(cnt[k + 1][n - a] for a in range(min(d - 1, n) + 1))
    return cnt


def sample_patterns(n_modes: int, n_photons: int, d: int, count: int, seed: int) -> np.ndarray:
    """``count`` occupation strings drawn uniformly from all strings with the
    given photon number and every occupation < d (exact, by suffix counts)."""
    cnt = _suffix_counts(n_modes, n_photons, d)
    if cnt[0][n_photons] == 0:
        raise ValueError("no admissible pattern")
    rng = np.random.default_rng(seed)
    out = np.zeros((count, n_modes), dtype=np.int32)
    for t in range(count):
        left = n_photons
        for k in range(n_modes):
            weights = [cnt[k + 1][left - a] if a <= left else 0 for a in range(d)]
            total = sum(weights)
            x = int(rng.integers(0, total)) if total < 2 ** 62 else _big_randint(rng, total)
            a = 0
            while x >= weights[a]:
                x -= weights[a]
                a += 1
            out[t, k] = a
            left -= a
    return out


def charge_path_patterns(bond_charges: Sequence[Sequence[int]], d: int, count: int, seed: int) -> np.ndarray:
    """``count`` occupation strings drawn uniformly from the strings whose
    right-charge path c_0 = N, c_{k+1} = c_k - occ_k visits only charges
    present on every bond (so none of them is structurally zero in a state
    with these bond charges); occupations < d."""
    L = len(bond_charges) - 1
    present = [set(int(c) for c in b) for b in bond_charges]
    # paths[k][c] = admissible strings over modes k..L-1 starting at charge c on bond k
    paths: List[dict] = [dict() for _ in range(L + 1)]
    paths[L] = {0: 1} if 0 in present[L] else {}
    for k in range(L - 1, -1, -1):
        for c in present[k]:
            n = sum(paths[k + 1].get(c - a, 0) for a in range(d))
            if n:
                paths[k][c] = n
    n0 = next(iter(present[0]))
    if paths[0].get(n0, 0) == 0:
        raise ValueError("no admissible charge path")
    rng = np.random.default_rng(seed)
    out = np.zeros((count, L), dtype=np.int32)
    for t in range(count):
        c = n0
        for k in range(L):
            weights = [paths[k + 1].get(c - a, 0) for a in range(d)]
            total = sum(weights)
            x = int(rng.integers(0, total)) if total < 2 ** 62 else _big_randint(rng, total)
            a = 0
            while x >= weights[a]:
                x -= weights[a]
                a += 1
            out[t, k] = a
            c -= a
    return out


def _big_randint(rng, total: int) -> int:
    nbits = total.bit_length() + 64
    while True:
        x = 0
        for _ in range((nbits + 62) // 63):
            x = (x << 63) | int(rng.integers(0, 2 ** 63))
        x %= (1 << nbits)
        lim = (1 << nbits) - ((1 << nbits) % total)
        if x < lim:
            return x % total


def all_patterns(n_modes: int, n_photons: int, d: int) -> np.ndarray:
    """Every occupation string with the given total and each occupation < d, lexicographic."""
    out: List[Tuple[int, ...]] = []

    def rec(prefix, k, left):
        if k == n_modes:
            if left == 0:
                out.append(tuple(prefix))
            return
        for a in range(min(d - 1, left) + 1):
            prefix.append(a)
            rec(prefix, k + 1, left - a)
            prefix.pop()

    rec([], 0, n_photons)
    return np.array(out, dtype=np.int32).reshape(len(out), n_modes)


# ---------------------------------------------------------------------------
# The benchmark workloads, as data.  Each returns a plain dict so the oracle
# and the GPU path read identical inputs.

def config_small_exact(seed: int = 1) -> dict:
    """L=8, d=5, |1,1,1,1,0,0,0,0>, Haar 8x8 via a Clements mesh, no truncation."""
    L = 8
    u = haar_unitary(L, seed)
    return dict(name="L8_d5_N4_clements_exact", L=L, d=5, occupation=[1, 1, 1, 1, 0, 0, 0, 0],
                unitary=u, gates=clements_circuit(u), chi_max=0, cutoff=0.0)


def config_brickwork(L: int, n_photons: int, placement: str, d: int, depth: int,
                     chi_max: int, cutoff: float, seed: int, name: str) -> dict:
    occ = [0] * L
    if placement == "first":
        for k in range(n_photons):
            occ[k] = 1
    elif placement == "even":
        for k in range(n_photons):
            occ[2 * k] = 1
    else:
        raise ValueError(placement)
    return dict(name=name, L=L, d=d, occupation=occ, gates=brickwork(L, depth, seed),
                layers=brickwork_layers(L, depth, seed), chi_max=chi_max, cutoff=cutoff)


def config_plain_gpu(seed: int = 2) -> dict:
    """L=32, 16 photons in modes 0-15, d=4, 32 brickwork layers, chi_max=512, cutoff 1e-12."""
    return config_brickwork(32, 16, "first", 4, 32, 512, 1e-12, seed, "L32_N16_d4_chi512")


def config_precision(seed: int = 3, chi_max: int = 2048) -> dict:
    """L=64, 32 photons in even modes, d=4, 64 brickwork layers, chi_max=2048."""
    return config_brickwork(64, 32, "even", 4, 64, chi_max, 1e-12, seed, f"L64_N32_d4_chi{chi_max}")


def config_batch_mix(n_circuits: int = 512, seed: int = 4, l_range=(16, 48),
                     chi_choices=(64, 128, 256, 512), cutoff: float = 1e-12,
                     depth_scale: float = 1.0) -> list:
    """The batching-form mix: circuit i has L ~ U{l_range}, floor(L/2) single
    photons in the first floor(L/2) modes, d = 4, a brickwork of depth
    round(depth_scale * L) with circuit seed 4000 + i, chi_max drawn from
    chi_choices, discarded-weight cutoff 1e-12.  L and chi_max are drawn from
    numpy.random.default_rng(seed) in circuit order (L first)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_circuits):
        L = int(rng.integers(l_range[0], l_range[1] + 1))
        chi = int(chi_choices[int(rng.integers(0, len(chi_choices)))])
        depth = max(1, int(round(depth_scale * L)))
        out.append(config_brickwork(L, L // 2, "first", 4, depth, chi, cutoff, 4000 + i,
                                    f"mix{i}_L{L}_chi{chi}"))
    return out


def serving_mix_specs(n_requests: int, seed: int = 5, large_frac: float = 0.05,
                      l_range=(16, 48), chi_choices=(64, 128, 256, 512), large_chi: int = 1024,
                      large_L: int = 64, depth_scale: float = 1.0) -> list:
    """The serving-form request mix, as light specs (built into circuits by
    config_from_spec): request j is, with probability large_frac, a large
    circuit (large_L modes, large_L/2 photons in the first modes, d = 4, depth
    large_L, chi_max = large_chi), else a circuit of the batching mix's
    distribution (L ~ U{l_range}, floor(L/2) photons in the first modes, depth
    L, chi_max ~ chi_choices); circuit seed 5000 + j, cutoff 1e-12.  The kind,
    L and chi_max are drawn from numpy.random.default_rng(seed) in request
    order."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n_requests):
        if rng.random() < large_frac:
            L, chi = large_L, large_chi
        else:
            L = int(rng.integers(l_range[0], l_range[1] + 1))
            chi = int(chi_choices[int(rng.integers(0, len(chi_choices)))])
        depth = max(1, int(round(depth_scale * L)))
        out.append(dict(L=L, n_photons=L // 2, d=4, depth=depth, chi_max=chi, cutoff=1e-12,
                        seed=5000 + j, name=f"req{j}_L{L}_chi{chi}"))
    return out


def config_from_spec(spec: dict) -> dict:
    """The brickwork circuit a serving spec names."""
    return config_brickwork(spec["L"], spec["n_photons"], "first", spec["d"], spec["depth"],
                            spec["chi_max"], spec["cutoff"], spec["seed"], spec["name"])


def config_serving_mix(n_requests: int, seed: int = 5, **kw) -> list:
    """The serving-form request mix as built circuits (see serving_mix_specs)."""
    return [config_from_spec(s) for s in serving_mix_specs(n_requests, seed, **kw)]


def _fock_counts(sites: int, d: int, n_max: int) -> list:
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


def synthetic_state(L: int, N: int, d: int, chi: int, width: float = 3.0, lam_min: float = 1e-4,
                    seed: int = 30):
    """A random block-sparse U(1) MPS with saturated bonds, the stand-in for a
    chi-saturated layer of the precision workload.  Bond k carries right
    charges c in [max(0, N - k(d-1)), min(N, (L-k)(d-1))] with multiplicities
    proportional to exp(-(c - c0)^2 / (2 width^2)), c0 = N (L - k) / L,
    normalised to min(chi, Fock bound of the bond) and clipped per charge by
    the number of left and right occupation strings; Gamma entries are complex
    Gaussian on the blocks the charge rule allows (c_left - c_right in 0..d-1),
    zero elsewhere; each bond's lambda decays exponentially from 1 to lam_min
    (in a random order).  Returns (bond_charges, gammas, lambdas) as taken by
    MPS.from_vidal; gammas[s] is (dim_s, dim_{s+1}) complex128."""
    rng = np.random.default_rng(seed)
    charges = []
    for k in range(L + 1):
        lo, hi = max(0, N - k * (d - 1)), min(N, (L - k) * (d - 1))
        left, right = _fock_counts(k, d, N), _fock_counts(L - k, d, N)
        cap = {c: min(left[N - c], right[c]) for c in range(lo, hi + 1)}
        cap = {c: v for c, v in cap.items() if v > 0}
        total = min(chi, sum(cap.values()))
        c0 = N * (L - k) / L
        w = {c: math.exp(-(c - c0) ** 2 / (2.0 * width ** 2)) for c in cap}
        ws = sum(w.values())
        cnt = {c: min(cap[c], int(total * w[c] / ws)) for c in cap}
        left_over = total - sum(cnt.values())
        for c in sorted(cap, key=lambda x: -w[x]):
            if left_over <= 0:
                break
            add = min(cap[c] - cnt[c], left_over)
            cnt[c] += add
            left_over -= add
        charges.append({c: v for c, v in cnt.items() if v > 0})
    # drop, until none is left, every charge without an admissible partner on a
    # neighbouring bond (c_left - c_right in 0..d-1), as the charge rule needs
    changed = True
    while changed:
        changed = False
        for k in range(L + 1):
            keep = {}
            for c, v in charges[k].items():
                ok_l = k == 0 or any(c + a in charges[k - 1] for a in range(d))
                ok_r = k == L or any(c - a in charges[k + 1] for a in range(d))
                if ok_l and ok_r:
                    keep[c] = v
                else:
                    changed = True
            charges[k] = keep
    charges = [[c for c in sorted(cnt) for _ in range(cnt[c])] for cnt in charges]
    gammas = []
    for s in range(L):
        cl = np.array(charges[s])[:, None]
        cr = np.array(charges[s + 1])[None, :]
        allowed = (cl - cr >= 0) & (cl - cr <= d - 1)
        g = (rng.standard_normal(allowed.shape) + 1j * rng.standard_normal(allowed.shape)) / math.sqrt(2.0)
        g *= allowed
        gammas.append(g.astype(np.complex128))
    lambdas = []
    for k in range(L + 1):
        n = len(charges[k])
        lam = np.exp(np.linspace(0.0, math.log(lam_min), n)) if n > 1 else np.ones(1)
        lambdas.append(rng.permutation(lam))
    return charges, gammas, lambdas
