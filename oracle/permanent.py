"""Permanents and closed-form Fock amplitudes of a linear-optics unitary.

Test infrastructure (see the package header).  Independent of the MPS method:
for an untruncated circuit with local cutoff d > N these values are what the
MPS must reproduce exactly (up to rounding).

Closed form used (standard boson-sampling identity): with creation operators
mapped column-wise, a_j^dagger -> sum_i U[i, j] a_i^dagger, the amplitude of
output pattern m from input pattern n is

    <m| U_hat |n> = Per(U[T, S]) / sqrt(prod_j n_j! * prod_i m_i!)

where S lists column j repeated n_j times and T lists row i repeated m_i times.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def permanent_naive(a: np.ndarray) -> complex:
    """Sum over all permutations (definition).  Only for n <= 7."""
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[0]
    if n == 0:
        return 1.0 + 0.0j
    total = 0.0 + 0.0j
    for perm in itertools.permutations(range(n)):
        p = 1.0 + 0.0j
        for i in range(n):
            p *= a[i, perm[i]]
        total += p
    return total


def permanent_ryser(a: np.ndarray) -> complex:
    """Ryser's inclusion-exclusion formula visited in Gray-code order.

    Per(A) = (-1)^n sum_{S subset [n]} (-1)^{|S|} prod_i sum_{j in S} a_ij.
    """
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[0]
    if n == 0:
        return 1.0 + 0.0j
    row_sums = np.zeros(n, dtype=np.complex128)
    total = 0.0 + 0.0j
    in_set = [False] * n
    size = 0
    for k in range(1, 1 << n):
        # Gray code: flip the lowest set bit position of k
        j = (k & -k).bit_length() - 1
        if in_set[j]:
            row_sums -= a[:, j]
            in_set[j] = False
            size -= 1
        else:
            row_sums += a[:, j]
            in_set[j] = True
            size += 1
        term = np.prod(row_sums)
        total += -term if (size % 2) else term
    return total * (-1) ** n


def fock_amplitude(u: np.ndarray, n_in, m_out) -> complex:
    """<m_out| U_hat |n_in> by the permanent formula; 0 when photon numbers differ."""
    n_in = [int(x) for x in n_in]
    m_out = [int(x) for x in m_out]
    if sum(n_in) != sum(m_out):
        return 0.0 + 0.0j
    cols = [j for j, c in enumerate(n_in) for _ in range(c)]
    rows = [i for i, c in enumerate(m_out) for _ in range(c)]
    sub = np.asarray(u, dtype=np.complex128)[np.ix_(rows, cols)]
    norm = 1.0
    for c in n_in + m_out:
        norm *= math.factorial(c)
    return permanent_ryser(sub) / math.sqrt(norm)
