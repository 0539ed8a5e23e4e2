"""Brute-force Fock-space simulation (small L only).

Test infrastructure (see the package header).

The state is an explicit vector over every occupation string with the given
photon number N and each occupation < d.  A two-mode gate on (s, s+1) maps
each basis string to the strings that differ only on those two modes, with
the elements of ``twomode.element``; occupations >= d are dropped (the local
cutoff P_d G P_d).  No tensor network is involved.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import twomode


class FockState:
    """modulus 0: the basis holds every string with the input's particle number;
    n >= 2: every string whose particle number equals the input's mod n (a
    Z_n charge)."""

    def __init__(self, occupation: Sequence[int], d: int, modulus: int = 0, charge_map=None):
        self.L = len(occupation)
        self.d = d
        self.N = int(sum(occupation))
        self.modulus = int(modulus)
        # charge_map (d x K): K U(1) charges; the basis holds every string with
        # the input's charge vector
        self.cmap = None if charge_map is None else np.asarray(charge_map, dtype=np.int64).reshape(d, -1)
        if max(occupation) >= d:
            raise ValueError("input occupation exceeds the local cutoff")
        self.basis: List[Tuple[int, ...]] = []
        if self.cmap is not None:
            total = self.cmap[list(occupation)].sum(axis=0)
            for t in itertools.product(range(d), repeat=self.L):
                if np.array_equal(self.cmap[list(t)].sum(axis=0), total):
                    self.basis.append(tuple(t))
        elif self.modulus:
            for t in itertools.product(range(d), repeat=self.L):
                if sum(t) % self.modulus == self.N % self.modulus:
                    self.basis.append(tuple(t))
        else:
            self._enumerate([], 0, self.N)
        self.index: Dict[Tuple[int, ...], int] = {t: i for i, t in enumerate(self.basis)}
        self.psi = np.zeros(len(self.basis), dtype=np.complex128)
        self.psi[self.index[tuple(int(x) for x in occupation)]] = 1.0

    def _enumerate(self, prefix, k, left):
        if k == self.L:
            if left == 0:
                self.basis.append(tuple(prefix))
            return
        for a in range(min(self.d - 1, left) + 1):
            prefix.append(a)
            self._enumerate(prefix, k + 1, left - a)
            prefix.pop()

    def apply(self, site: int, u: np.ndarray) -> None:
        s = site
        out = np.zeros_like(self.psi)
        cache: Dict[Tuple[int, int, int, int], complex] = {}
        for i, t in enumerate(self.basis):
            amp = self.psi[i]
            if amp == 0:
                continue
            a, b = t[s], t[s + 1]
            tot = a + b
            for p in range(max(0, tot - (self.d - 1)), min(self.d - 1, tot) + 1):
                q = tot - p
                key = (p, q, a, b)
                if key not in cache:
                    cache[key] = twomode.element(u, p, q, a, b)
                t2 = t[:s] + (p, q) + t[s + 2:]
                out[self.index[t2]] += cache[key] * amp
        self.psi = out

    def apply_dense(self, site: int, g: np.ndarray) -> None:
        """Any two-site gate as a d^2 x d^2 matrix (row p*d+q, column a*d+b).
        Every element is visited: one that moves a basis string out of the
        N-particle sector raises ValueError (the gate breaks the charge)."""
        s, d = site, self.d
        g = np.asarray(g, dtype=np.complex128).reshape(d * d, d * d)
        out = np.zeros_like(self.psi)
        for i, t in enumerate(self.basis):
            amp = self.psi[i]
            if amp == 0:
                continue
            col = t[s] * d + t[s + 1]
            for p in range(d):
                for q in range(d):
                    el = g[p * d + q, col]
                    if el == 0:
                        continue
                    t2 = t[:s] + (p, q) + t[s + 2:]
                    j = self.index.get(t2)
                    if j is None:
                        raise ValueError(f"gate element ({p}{q},{t[s]}{t[s + 1]}) leaves the charge sector")
                    out[j] += el * amp
        self.psi = out

    def amplitude(self, occ: Sequence[int]) -> complex:
        t = tuple(int(x) for x in occ)
        i = self.index.get(t)
        return 0.0 + 0.0j if i is None else complex(self.psi[i])

    def norm2(self) -> float:
        return float(np.vdot(self.psi, self.psi).real)

    def schmidt_ranks(self, bond: int, tol: float = 1e-10) -> Dict[int, int]:
        """Per right-charge c (photons right of the cut), the rank of the block
        of the state matrix psi[(left string), (right string)] with that c."""
        blocks: Dict[int, Dict[Tuple[int, ...], Dict[Tuple[int, ...], complex]]] = {}
        for i, t in enumerate(self.basis):
            if self.cmap is not None:
                c = tuple(int(x) for x in self.cmap[list(t[bond:])].sum(axis=0)) if bond < self.L else \
                    tuple([0] * self.cmap.shape[1])
            else:
                c = sum(t[bond:]) % self.modulus if self.modulus else sum(t[bond:])
            blocks.setdefault(c, {}).setdefault(t[:bond], {})[t[bond:]] = self.psi[i]
        ranks: Dict[int, int] = {}
        smax = 0.0
        svals: Dict[int, np.ndarray] = {}
        for c, rows in blocks.items():
            rkeys = sorted(rows)
            ckeys = sorted({k for r in rows.values() for k in r})
            cidx = {k: j for j, k in enumerate(ckeys)}
            m = np.zeros((len(rkeys), len(ckeys)), dtype=np.complex128)
            for i, rk in enumerate(rkeys):
                for ck, v in rows[rk].items():
                    m[i, cidx[ck]] = v
            sv = np.linalg.svd(m, compute_uv=False)
            svals[c] = sv
            if sv.size:
                smax = max(smax, float(sv[0]))
        for c, sv in svals.items():
            r = int(np.sum(sv > tol * smax))
            if r:
                ranks[c] = r
        return ranks


def run(occupation: Sequence[int], d: int, gates, modulus: int = 0, charge_map=None) -> FockState:
    """Gates with .u (mode unitary) or .g4 (dense two-site matrix)."""
    st = FockState(occupation, d, modulus, charge_map)
    for g in gates:
        if hasattr(g, "g4"):
            st.apply_dense(g.site, g.g4)
        else:
            st.apply(g.site, g.u)
    return st
