"""Pins of the oracle for two independent U(1) charges (U(1) x U(1); no GPU).

Two species of hard-core bosons, p = 2 a + b on a site with a, b the up and
down occupations, each species' number conserved.  The oracle audits each
charge with its own operator and reads joint charges on common eigenvectors;
its brute force keeps every string with the input's pair of numbers.  Pins:

* at U = 0 the species do not interact and hard-core bosons with
  nearest-neighbour hopping are free fermions (no Jordan-Wigner string
  between neighbours), so every amplitude is the product of two
  determinants of the gates' single-particle matrices, one per species;
* at U != 0 the Trotter evolution approaches exp(-iHT) in the full 4^L
  space as dt^2, with H built from site operators directly, and the exact
  evolution never leaves the input's pair of numbers;
* the audit's joint charges per bond equal the brute-force Schmidt ranks of
  each (up, down) charge block, also under a bond cap.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import dense_mps, fock
from workloads import hamiltonians as ham

CM = ham.TWO_SPECIES_CHARGES


def exp2(t, ax):
    """exp(-i t ax X)."""
    c, s = math.cos(ax * t), math.sin(ax * t)
    return np.array([[c, -1j * s], [-1j * s, c]])


def schedule(L, dt, steps):
    even, odd = list(range(0, L - 1, 2)), list(range(1, L - 1, 2))
    out = [(even, dt / 2)]
    for k in range(steps):
        out.append((odd, dt))
        out.append((even, dt if k < steps - 1 else dt / 2))
    return [(b, t) for b, t in out if b]


def test_free_species_are_two_determinants():
    L, J, dt, steps = 6, 0.9, 0.3, 3
    occ = [3, 0, 2, 1, 0, 2]                      # up = (1,0,1,0,0,1), down = (1,0,0,1,0,0)
    cfg = ham.config_tebd("two_species", L, 4, occ, dt, steps, chi_max=0, J=J, U=0.0)
    assert cfg["charge_map"] is not None
    U1 = np.eye(L, dtype=np.complex128)
    for bonds, t in schedule(L, dt, steps):
        for s in bonds:
            e = np.eye(L, dtype=np.complex128)
            e[s:s + 2, s:s + 2] = exp2(t, -J)        # one particle on the bond: -J X
            U1 = e @ U1
    up_in = [j for j in range(L) if occ[j] // 2]
    dn_in = [j for j in range(L) if occ[j] % 2]
    st = fock.run(occ, 4, cfg["gates"], charge_map=CM)
    m = dense_mps.DenseMPS(occ, 4, charge_map=CM).run(cfg["gates"])
    pats = np.array(st.basis, dtype=np.int64)
    want = []
    for t in st.basis:
        up = [j for j in range(L) if t[j] // 2]
        dn = [j for j in range(L) if t[j] % 2]
        want.append(np.linalg.det(U1[np.ix_(up, up_in)]) * np.linalg.det(U1[np.ix_(dn, dn_in)]))
    want = np.array(want)
    assert np.max(np.abs(st.psi - want)) < 1e-12
    assert np.max(np.abs(m.amplitudes(pats) - want)) < 1e-12
    for b in range(L + 1):
        assert m.audit_clean(b)
        assert m.bond_charges(b) == st.schmidt_ranks(b), b


def _site_op(op, i, L):
    return np.kron(np.kron(np.eye(4 ** i), op), np.eye(4 ** (L - i - 1)))


def test_interacting_species_trotter_order_and_sector():
    L, J, Uint = 4, 1.0, 1.7
    occ = [3, 1, 0, 2]
    low = np.array([[0.0, 1.0], [0.0, 0.0]])
    b_up, b_dn = np.kron(low, np.eye(2)), np.kron(np.eye(2), low)
    H = np.zeros((4 ** L, 4 ** L), dtype=np.complex128)
    for i in range(L - 1):
        for b in (b_up, b_dn):
            hop = _site_op(b.T, i, L) @ _site_op(b, i + 1, L)
            H -= J * (hop + hop.conj().T)
    nn = (b_up.T @ b_up) @ (b_dn.T @ b_dn)
    H += Uint * sum(_site_op(nn, i, L) for i in range(L))
    hb = ham.bond_hamiltonians("two_species", L, 4, J=J, U=Uint)
    assert np.max(np.abs(ham.hamiltonian_dense(hb, L, 4) - H)) < 1e-13
    T = 0.8
    psi0 = np.zeros(4 ** L, dtype=np.complex128)
    psi0[sum(o * 4 ** (L - 1 - s) for s, o in enumerate(occ))] = 1.0
    exact = scipy.linalg.expm(-1j * T * H) @ psi0
    total = CM[occ].sum(axis=0)
    strings = list(itertools.product(range(4), repeat=L))
    inside = [np.array_equal(CM[list(t)].sum(axis=0), total) for t in strings]
    assert np.max(np.abs(exact[[not x for x in inside]])) < 1e-12
    pats = [t for t, x in zip(strings, inside) if x]
    ex = np.array([exact[sum(o * 4 ** (L - 1 - s) for s, o in enumerate(t))] for t in pats])
    errs = []
    for steps in (4, 8, 16):
        cfg = ham.config_tebd("two_species", L, 4, occ, T / steps, steps, chi_max=0, J=J, U=Uint)
        st = fock.run(occ, 4, cfg["gates"], charge_map=CM)
        errs.append(np.linalg.norm(np.array([st.amplitude(t) for t in pats]) - ex))
    assert errs[0] > 1e-4
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5, errs


def test_joint_audit_under_truncation():
    """With a bond cap and no degenerate cut (smallest margin 3.5e-6), every kept
    subspace stays closed under both charges.  (A reflection-and-swap symmetric
    input such as 3,0,1,2,0,3 ties at the cut, margin 3e-17, and the dense SVD
    may then mix charge sectors: the audit reports it.)"""
    cfg = ham.config_tebd("two_species", 6, 4, [3, 0, 1, 2, 1, 0], 0.2, 5, 6, 1e-12, J=1.0, U=2.0)
    st = fock.run(cfg["occupation"], 4, cfg["gates"], charge_map=CM)
    m = dense_mps.DenseMPS(cfg["occupation"], 4, chi_max=6, cutoff=1e-12, charge_map=CM).run(cfg["gates"])
    assert max(r.discarded for r in m.records) > 1e-8
    assert min(r.margin for r in m.records) > 1e-9
    for b in range(7):
        assert m.audit_clean(b)
        h = m.bond_charges(b)
        assert sum(h.values()) == m.bond_dims()[b]
        assert set(h) <= set(st.schmidt_ranks(b))          # only charges the exact state has
