"""Seeded inputs for Hamiltonian time evolution (TEBD) with a U(1) charge.

Input generator shared by the tests, the oracle runs and the GPU runs; it holds
none of the MPS update.  The paper names two lattice models whose
Hamiltonians commute with a particle number (Sec. I and Sec. II: [H, N] = 0),
besides linear optics:

* the XXZ spin-1/2 chain,
      H = J sum_i (Sx_i Sx_{i+1} + Sy_i Sy_{i+1} + Delta Sz_i Sz_{i+1}) - hz sum_i Sz_i,
  with occupation n = 1 for spin up (Sz = n - 1/2) and d = 2, so the charge
  is the number of up spins (the magnetisation plus L/2);
  Sx Sx + Sy Sy = (S+ S- + S- S+) / 2;
* the Bose-Hubbard chain,
      H = -J sum_i (b_i^+ b_{i+1} + b_{i+1}^+ b_i) + U/2 sum_i n_i (n_i - 1) - mu sum_i n_i,
  with occupations 0..d-1 per site (the MPS local cutoff d).

Two models with a discrete Abelian charge (Z_n, the particle number mod n;
the paper's general Abelian symmetries, Sec. I) and local dimension d = n:

* the transverse-field Ising chain, H = -J sum_i X_i X_{i+1} - h sum_i Z_i,
  Z = diag(1, -1) on occupations (0, 1): X X changes the occupation count by
  0 or 2, so its parity (Z_2) is conserved;
* the Z_n clock chain in its charge basis, tau = diag(omega^p) (omega =
  exp(2 pi i / n)) and sigma the shift |p> -> |p + 1 mod n>:
  H = -J sum_i (sigma_i sigma_{i+1}^dagger + h.c.) - f sum_i (tau_i + tau_i^dagger),
  which conserves sum_i p_i mod n.

Bond Hamiltonians h_i on sites (i, i+1) carry the bond's coupling plus the
on-site terms shared between the two bonds of each site (half each; an end
site's terms go fully to its only bond), so sum_i h_i = H.  Matrices are
d^2 x d^2 with index p*d + q, p the occupation of the left site.

A Trotter factor is exp(-i t h) (real time) or exp(-t h) (imaginary time),
by scipy.linalg.expm.  A second-order step of length dt is: the even bonds
(0-1, 2-3, ...) for dt/2, the odd bonds (1-2, 3-4, ...) for dt, the even
bonds for dt/2 again; with `merge` the closing half step of one step and the
opening half step of the next are one layer of length dt (exact, since the
even bonds commute among themselves).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np
import scipy.linalg


@dataclass
class DenseGate:
    site: int
    g4: np.ndarray            # d^2 x d^2, row p*d+q (after), column a*d+b (before)


def _lowering(d: int) -> np.ndarray:
    b = np.zeros((d, d))
    for n in range(1, d):
        b[n - 1, n] = np.sqrt(n)
    return b


def xxz_bond(J: float, delta: float, hz: float = 0.0, w_left: float = 0.5, w_right: float = 0.5) -> np.ndarray:
    """h for one bond of the XXZ chain (d = 2); w_left/w_right weight the field
    on the two sites (1/2 inside the chain, 1 at an end)."""
    sp = np.array([[0.0, 0.0], [1.0, 0.0]])        # S+ = |1><0|
    sm = sp.T
    sz = np.diag([-0.5, 0.5])
    one = np.eye(2)
    h = J * (0.5 * (np.kron(sp, sm) + np.kron(sm, sp)) + delta * np.kron(sz, sz))
    h = h - hz * (w_left * np.kron(sz, one) + w_right * np.kron(one, sz))
    return h.astype(np.complex128)


def bose_hubbard_bond(d: int, J: float, U: float, mu: float = 0.0, w_left: float = 0.5,
                      w_right: float = 0.5, mu_right: float = None) -> np.ndarray:
    """h for one bond of the Bose-Hubbard chain with occupations 0..d-1; the
    chemical potential of the right site is mu_right (default mu)."""
    b = _lowering(d)
    bd = b.T
    n = np.diag(np.arange(d, dtype=float))
    one = np.eye(d)
    mr = mu if mu_right is None else mu_right
    onsite_l = 0.5 * U * n @ (n - one) - mu * n
    onsite_r = 0.5 * U * n @ (n - one) - mr * n
    h = -J * (np.kron(bd, b) + np.kron(b, bd))
    h = h + w_left * np.kron(onsite_l, one) + w_right * np.kron(one, onsite_r)
    return h.astype(np.complex128)


def ising_bond(J: float, h: float, w_left: float = 0.5, w_right: float = 0.5) -> np.ndarray:
    """h for one bond of the transverse-field Ising chain (d = 2)."""
    x = np.array([[0.0, 1.0], [1.0, 0.0]])
    z = np.diag([1.0, -1.0])
    one = np.eye(2)
    return (-J * np.kron(x, x) - h * (w_left * np.kron(z, one) + w_right * np.kron(one, z))).astype(np.complex128)


def clock_bond(n: int, J: float, f: float, w_left: float = 0.5, w_right: float = 0.5) -> np.ndarray:
    """h for one bond of the Z_n clock chain in the charge basis (d = n)."""
    w = np.exp(2j * np.pi / n)
    sig = np.zeros((n, n), dtype=np.complex128)
    for p in range(n):
        sig[(p + 1) % n, p] = 1.0
    tau = np.diag(w ** np.arange(n))
    one = np.eye(n)
    hop = np.kron(sig, sig.conj().T)
    field = tau + tau.conj().T
    return -J * (hop + hop.conj().T) - f * (w_left * np.kron(field, one) + w_right * np.kron(one, field))


# Two species of hard-core bosons on one site: p = 2 a + b with a, b in {0, 1}
# the occupations of species up and down; each species' number is a U(1)
# charge of its own (U(1) x U(1)).
TWO_SPECIES_CHARGES = np.array([[p // 2, p % 2] for p in range(4)])


def two_species_bond(J: float, U: float, w_left: float = 0.5, w_right: float = 0.5) -> np.ndarray:
    """h for one bond of the two-species hard-core boson chain (d = 4):
    -J sum_sigma (b+_{i,sigma} b_{i+1,sigma} + h.c.) + U n_up n_down on each site."""
    low = np.array([[0.0, 1.0], [0.0, 0.0]])          # |1> -> |0>
    one2 = np.eye(2)
    b_up, b_dn = np.kron(low, one2), np.kron(one2, low)
    one = np.eye(4)
    h = np.zeros((16, 16))
    for b in (b_up, b_dn):
        h = h - J * (np.kron(b.T, b) + np.kron(b, b.T))
    nn = (b_up.T @ b_up) @ (b_dn.T @ b_dn)
    h = h + U * (w_left * np.kron(nn, one) + w_right * np.kron(one, nn))
    return h.astype(np.complex128)


def trotter_gate(h: np.ndarray, t: float, imaginary: bool = False) -> np.ndarray:
    """exp(-i t h), or exp(-t h) with imaginary."""
    return scipy.linalg.expm((-t if imaginary else -1j * t) * h)


def bond_hamiltonians(model: str, L: int, d: int, **p) -> List[np.ndarray]:
    """h_0 .. h_{L-2} of the chain (end sites' on-site terms on their one bond)."""
    out = []
    for i in range(L - 1):
        wl = 1.0 if i == 0 else 0.5
        wr = 1.0 if i == L - 2 else 0.5
        if model == "xxz":
            if d != 2:
                raise ValueError("the XXZ chain has d = 2")
            out.append(xxz_bond(p.get("J", 1.0), p.get("delta", 1.0), p.get("hz", 0.0), wl, wr))
        elif model == "bose_hubbard":
            # mu_sites: a site-dependent chemical potential (overrides mu)
            ms = p.get("mu_sites")
            ml = ms[i] if ms is not None else p.get("mu", 0.0)
            mr = ms[i + 1] if ms is not None else p.get("mu", 0.0)
            out.append(bose_hubbard_bond(d, p.get("J", 1.0), p.get("U", 1.0), ml, wl, wr, mr))
        elif model == "ising":
            if d != 2:
                raise ValueError("the Ising chain has d = 2")
            out.append(ising_bond(p.get("J", 1.0), p.get("h", 1.0), wl, wr))
        elif model == "clock":
            out.append(clock_bond(d, p.get("J", 1.0), p.get("f", 1.0), wl, wr))
        elif model == "two_species":
            if d != 4:
                raise ValueError("the two-species chain has d = 4")
            out.append(two_species_bond(p.get("J", 1.0), p.get("U", 1.0), wl, wr))
        else:
            raise ValueError(model)
    return out


def hamiltonian_dense(hb: Sequence[np.ndarray], L: int, d: int) -> np.ndarray:
    """H = sum_i h_i on the full d^L space (index sum_s occ_s d^(L-1-s)); small L only."""
    dim = d ** L
    H = np.zeros((dim, dim), dtype=np.complex128)
    for i, h in enumerate(hb):
        H += np.kron(np.kron(np.eye(d ** i), h), np.eye(d ** (L - i - 2)))
    return H


def trotter_layers(hb: Sequence[np.ndarray], dt: float, steps: int, order: int = 2, merge: bool = True,
                   imaginary: bool = False) -> List[List[DenseGate]]:
    """Layers of dense gates for `steps` Trotter steps of length dt."""
    L = len(hb) + 1
    even = list(range(0, L - 1, 2))
    odd = list(range(1, L - 1, 2))

    def layer(bonds, t):
        return [DenseGate(i, trotter_gate(hb[i], t, imaginary)) for i in bonds]

    if order == 1:
        out = []
        for _ in range(steps):
            out += [layer(even, dt), layer(odd, dt)]
        return [l for l in out if l]
    if order != 2:
        raise ValueError("order 1 or 2")
    if steps <= 0:
        return []
    if not merge:
        out = []
        for _ in range(steps):
            out += [layer(even, dt / 2), layer(odd, dt), layer(even, dt / 2)]
        return [l for l in out if l]
    out = [layer(even, dt / 2)]
    for k in range(steps):
        out.append(layer(odd, dt))
        out.append(layer(even, dt if k < steps - 1 else dt / 2))
    return [l for l in out if l]


def neel(L: int) -> List[int]:
    """|up, down, up, ...>: L//2 + L%2 up spins."""
    return [1 - (i % 2) for i in range(L)]


def config_tebd(model: str, L: int, d: int, occupation: Sequence[int], dt: float, steps: int,
                chi_max: int, cutoff: float = 0.0, order: int = 2, imaginary: bool = False, **p) -> dict:
    hb = bond_hamiltonians(model, L, d, **p)
    occ = [int(x) for x in occupation]
    if len(occ) != L or any(o < 0 or o >= d for o in occ):
        raise ValueError("occupation must have L entries in 0..d-1")
    layers = trotter_layers(hb, dt, steps, order=order, imaginary=imaginary)
    modulus = d if model in ("ising", "clock") else 0
    cmap = TWO_SPECIES_CHARGES if model == "two_species" else None
    return {"model": model, "L": L, "d": d, "occupation": occ, "n_photons": sum(occ), "modulus": modulus,
            "charge_map": cmap, "dt": dt,
            "steps": steps, "order": order, "imaginary": imaginary, "params": dict(p),
            "chi_max": chi_max, "cutoff": cutoff, "layers": layers,
            "gates": [g for lay in layers for g in lay]}


def config_xxz(L: int = 64, steps: int = 40, dt: float = 0.05, chi_max: int = 256, delta: float = 1.0,
               J: float = 1.0, hz: float = 0.0, cutoff: float = 0.0) -> dict:
    """Quench of the Neel state under the XXZ chain (Delta = 1: Heisenberg)."""
    return config_tebd("xxz", L, 2, neel(L), dt, steps, chi_max, cutoff, J=J, delta=delta, hz=hz)


def config_bose_hubbard(L: int = 64, d: int = 4, steps: int = 40, dt: float = 0.05, chi_max: int = 256,
                        J: float = 1.0, U: float = 2.0, mu: float = 0.0, cutoff: float = 0.0,
                        filling: int = 1) -> dict:
    """Quench of the Mott product state (filling bosons on every site)."""
    return config_tebd("bose_hubbard", L, d, [filling] * L, dt, steps, chi_max, cutoff, J=J, U=U, mu=mu)


def config_xxz_quench() -> dict:
    """The measured XXZ workload: L = 64, Neel state (32 up spins), J = 1,
    Delta = 0.5, 200 second-order steps of dt = 0.05 (T = 10; 12632 gates in
    401 layers), chi_max = 256 (reached near T = 7), cutoff 1e-12."""
    return config_xxz(L=64, steps=200, dt=0.05, chi_max=256, delta=0.5, cutoff=1e-12)


def config_bose_hubbard_quench() -> dict:
    """The measured Bose-Hubbard workload: L = 64, density wave |2,0,2,0,...>
    (64 bosons), d = 4, J = 1, U = 2, weak disorder mu_i ~ U[-0.5, 0.5]
    (numpy.random.default_rng(7)), 60 second-order steps of dt = 0.05 (T = 3;
    3812 gates in 121 layers), chi_max = 256, cutoff 1e-12."""
    mu = [float(x) for x in np.random.default_rng(7).uniform(-0.5, 0.5, size=64)]
    return config_tebd("bose_hubbard", 64, 4, [2, 0] * 32, 0.05, 60, 256, 1e-12, J=1.0, U=2.0, mu_sites=mu)


def config_ising_quench() -> dict:
    """The measured Z_2 workload: transverse-field Ising chain, L = 64, all
    spins in occupation 0, J = 1, h = 0.5, 200 second-order steps of dt = 0.05
    (T = 10; 12632 gates), chi_max = 256, cutoff 1e-12."""
    return config_tebd("ising", 64, 2, [0] * 64, 0.05, 200, 256, 1e-12, J=1.0, h=0.5)


def config_clock_quench() -> dict:
    """The measured Z_3 workload: Z_3 clock chain, L = 64, all sites in charge
    0, J = 1, f = 0.3, 60 second-order steps of dt = 0.05 (T = 3; 3812 gates),
    chi_max = 256, cutoff 1e-12."""
    return config_tebd("clock", 64, 3, [0] * 64, 0.05, 60, 256, 1e-12, J=1.0, f=0.3)


def zn_patterns(L: int, d: int, charge: int, count: int, seed: int, modulus: int = 0) -> np.ndarray:
    """count uniform occupation strings (occupations < d) whose particle number
    is `charge` mod n, n = modulus or d when 0 (rejection sampling,
    numpy.random.default_rng(seed))."""
    n = modulus or d
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        t = rng.integers(0, d, size=L)
        if int(t.sum()) % n == charge % n:
            out.append(t)
    return np.array(out, dtype=np.int32)


def charge_map_patterns(L: int, charge_map, total, count: int, seed: int) -> np.ndarray:
    """count occupation strings drawn uniformly from the strings of L local
    states whose charges charge_map[p] (tuples) sum to `total`: exact suffix
    counts per partial charge, then a chain of draws
    (numpy.random.default_rng(seed))."""
    cm = [tuple(int(x) for x in row) for row in np.asarray(charge_map).reshape(len(charge_map), -1)]
    total = tuple(int(x) for x in total)
    d = len(cm)
    # ways[k][c] = strings over sites k..L-1 whose charges sum to c
    ways = [dict() for _ in range(L + 1)]
    ways[L] = {tuple(0 for _ in total): 1}
    for k in range(L - 1, -1, -1):
        w = {}
        for c, n in ways[k + 1].items():
            for q in cm:
                c2 = tuple(a + b for a, b in zip(c, q))
                if all(a <= t for a, t in zip(c2, total)):
                    w[c2] = w.get(c2, 0) + n
        ways[k] = w
    if ways[0].get(total, 0) == 0:
        raise ValueError("no string carries that charge")
    rng = np.random.default_rng(seed)
    out = np.zeros((count, L), dtype=np.int32)
    for t in range(count):
        rem = total
        for k in range(L):
            opts = [(p, tuple(a - b for a, b in zip(rem, cm[p]))) for p in range(d)]
            wts = [ways[k + 1].get(r, 0) if all(x >= 0 for x in r) else 0 for _, r in opts]
            x = int(rng.integers(0, sum(wts)))
            p = 0
            while x >= wts[p]:
                x -= wts[p]
                p += 1
            out[t, k] = p
            rem = opts[p][1]
    return out


def random_zn_gate(d: int, seed: int, unitary: bool = True, modulus: int = 0) -> np.ndarray:
    """A random d^2 x d^2 gate that conserves p + q mod n, n = modulus or d when
    0 (a Z_n charge, n >= d): a Haar-random (or complex Gaussian) block for each
    total mod n, over the pairs (p, q) of occupations below d with that total."""
    n = modulus or d
    rng = np.random.default_rng(seed)
    g = np.zeros((d * d, d * d), dtype=np.complex128)
    for tot in range(n):
        idx = [p * d + q for p in range(d) for q in range(d) if (p + q) % n == tot]
        if not idx:
            continue
        k = len(idx)
        z = (rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))) / np.sqrt(2)
        if unitary:
            q, r = np.linalg.qr(z)
            z = q * (np.diag(r) / np.abs(np.diag(r)))
        g[np.ix_(idx, idx)] = z
    return g


def random_charge_conserving(d: int, seed: int, unitary: bool = True) -> np.ndarray:
    """A random d^2 x d^2 gate that conserves p + q: a Haar-random (or, with
    unitary False, complex Gaussian) block for each local charge n."""
    rng = np.random.default_rng(seed)
    g = np.zeros((d * d, d * d), dtype=np.complex128)
    for n in range(2 * d - 1):
        idx = [p * d + (n - p) for p in range(max(0, n - d + 1), min(d - 1, n) + 1)]
        k = len(idx)
        z = (rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))) / np.sqrt(2)
        if unitary:
            q, r = np.linalg.qr(z)
            z = q * (np.diag(r) / np.abs(np.diag(r)))
        g[np.ix_(idx, idx)] = z
    return g
