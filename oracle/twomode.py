"""Fock-basis matrix elements of a two-mode linear-optics gate.

Test infrastructure (see the package header).

The paper states that the dynamics conserve the charge (Sec. II, [H, N] = 0);
for a beam splitter the conserved charge is the total photon number, so the
two-mode gate is block diagonal in n = p + q.  Its elements follow from the
mode map a^dagger -> u00 a^dagger + u10 b^dagger, b^dagger -> u01 a^dagger
+ u11 b^dagger applied to |m, n> = a^dagger^m b^dagger^n / sqrt(m! n!) |0>:

    <p, q| G |m, n> = sqrt(p! q! / (m! n!))
        * sum_{j + l = p} C(m, j) C(n, l) u00^j u10^(m-j) u01^l u11^(n-l)

With a local cutoff d (occupations 0..d-1, Eq. (E1)'s "dimension d") the gate
the MPS can apply is the projection P_d G P_d: elements with any occupation
>= d are dropped.  That projection is not unitary once n >= d.
"""
from __future__ import annotations

import math

import numpy as np


def element(u: np.ndarray, p: int, q: int, m: int, n: int) -> complex:
    """<p, q| G(u) |m, n> for the two-mode gate of 2x2 mode unitary u."""
    if p + q != m + n or min(p, q, m, n) < 0:
        return 0.0 + 0.0j
    u00, u01, u10, u11 = u[0, 0], u[0, 1], u[1, 0], u[1, 1]
    s = 0.0 + 0.0j
    for j in range(0, min(m, p) + 1):
        l = p - j
        if l < 0 or l > n:
            continue
        s += (math.comb(m, j) * math.comb(n, l)
              * u00 ** j * u10 ** (m - j) * u01 ** l * u11 ** (n - l))
    return s * math.sqrt(math.factorial(p) * math.factorial(q)
                         / (math.factorial(m) * math.factorial(n)))


def block(u: np.ndarray, ntot: int, d: int | None = None) -> np.ndarray:
    """G^(ntot): the gate restricted to total photon number ntot.

    Basis ordered by the first-mode occupation p descending: (p, ntot - p),
    so the one-photon block in the basis (|1,0>, |0,1>) is u itself.
    With a cutoff d only p, ntot - p < d are kept (P_d G P_d).
    """
    ps = [p for p in range(ntot, -1, -1) if d is None or (p < d and ntot - p < d)]
    g = np.zeros((len(ps), len(ps)), dtype=np.complex128)
    for a, p in enumerate(ps):
        for b, m in enumerate(ps):
            g[a, b] = element(u, p, ntot - p, m, ntot - m)
    return g


def dense(u: np.ndarray, d: int) -> np.ndarray:
    """P_d G P_d as a (d*d) x (d*d) matrix, index (p, q) -> p*d + q."""
    g = np.zeros((d * d, d * d), dtype=np.complex128)
    for p in range(d):
        for q in range(d):
            for m in range(d):
                n = p + q - m
                if 0 <= n < d:
                    g[p * d + q, m * d + n] = element(u, p, q, m, n)
    return g
