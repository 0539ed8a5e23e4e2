"""Pins of the oracle for discrete Abelian charges (Z_n, the particle number
mod n; no GPU).

The dense oracle needs no symmetry; what changes for Z_n is its charge audit
(the unitary omega^Q tracked in the Schmidt basis instead of Q) and the brute
force's basis (every string whose particle number is the input's mod n).  Both
are checked against what the physics fixes:

* two Ising sites: the even sector {|00>, |11>} evolves by
  [[-2h, -J], [-J, 2h]] and the odd sector {|01>, |10>} by -J X, each 2 x 2
  exponential written out in closed form;
* whole chains (Ising, Z_2; clock, Z_3): the bond Hamiltonians sum to H built
  from site operators directly, the exact evolution exp(-iHT) in the full d^L
  space never leaves the input's charge sector, and the second-order Trotter
  evolution in the oracle approaches it as dt^2;
* the audit's per-charge bond dimensions equal the brute-force Schmidt ranks
  of each charge block.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import dense_mps, fock
from workloads import hamiltonians as ham


def exp2(t, a0, ax, az):
    """exp(-i t (a0 I + ax X + az Z)) for real coefficients."""
    r = math.hypot(ax, az)
    c, s = math.cos(r * t), (math.sin(r * t) / r if r > 0 else t)
    return np.exp(-1j * t * a0) * np.array([[c - 1j * s * az, -1j * s * ax], [-1j * s * ax, c + 1j * s * az]])


@pytest.mark.parametrize("start", [(0, 0), (0, 1)])
def test_two_ising_sites_closed_form(start):
    J, h, t = 0.8, 0.35, 0.9
    g = ham.trotter_gate(ham.ising_bond(J, h, 1.0, 1.0), t)
    if start == (0, 0):
        # even sector (|00>, |11>): H = [[-2h, -J], [-J, 2h]] = -J X - 2h Z
        v = exp2(t, 0.0, -J, -2 * h) @ np.array([1.0, 0.0])
        ref = {(0, 0): v[0], (1, 1): v[1], (0, 1): 0.0, (1, 0): 0.0}
    else:
        # odd sector (|01>, |10>): H = -J X (the fields cancel)
        v = exp2(t, 0.0, -J, 0.0) @ np.array([1.0, 0.0])
        ref = {(0, 1): v[0], (1, 0): v[1], (0, 0): 0.0, (1, 1): 0.0}
    st = fock.FockState(list(start), 2, modulus=2)
    st.apply_dense(0, g)
    m = dense_mps.DenseMPS(list(start), 2, modulus=2).run([ham.DenseGate(0, g)])
    for pat, want in ref.items():
        assert abs(st.amplitude(pat) - want) < 1e-14
        assert abs(m.amplitude(pat) - want) < 1e-14


def _site_op(op, i, L):
    d = op.shape[0]
    return np.kron(np.kron(np.eye(d ** i), op), np.eye(d ** (L - i - 1)))


def _ising_direct(L, J, h):
    x = np.array([[0.0, 1.0], [1.0, 0.0]])
    z = np.diag([1.0, -1.0])
    H = -J * sum(_site_op(x, i, L) @ _site_op(x, i + 1, L) for i in range(L - 1))
    return H - h * sum(_site_op(z, i, L) for i in range(L))


def _clock_direct(L, n, J, f):
    w = np.exp(2j * np.pi / n)
    sig = np.roll(np.eye(n), 1, axis=0)               # |p> -> |p + 1 mod n>
    tau = np.diag(w ** np.arange(n))
    H = -J * sum(_site_op(sig, i, L) @ _site_op(sig.conj().T, i + 1, L) for i in range(L - 1))
    H = H + H.conj().T
    return H - f * sum(_site_op(tau + tau.conj().T, i, L) for i in range(L))


@pytest.mark.parametrize("model", ["ising", "clock"])
def test_zn_chain_sector_and_trotter_order(model):
    if model == "ising":
        L, d, occ, p = 7, 2, [1, 0, 0, 1, 1, 0, 0], dict(J=1.0, h=0.6)
        Hd = _ising_direct(L, **p)
    else:
        L, d, occ, p = 5, 3, [1, 0, 2, 0, 1], dict(J=1.0, f=0.4)
        Hd = _clock_direct(L, 3, **p)
    n = d
    hb = ham.bond_hamiltonians(model, L, d, **p)
    assert np.max(np.abs(ham.hamiltonian_dense(hb, L, d) - Hd)) < 1e-13
    T = 0.8
    psi0 = np.zeros(d ** L, dtype=np.complex128)
    psi0[sum(o * d ** (L - 1 - s) for s, o in enumerate(occ))] = 1.0
    exact = scipy.linalg.expm(-1j * T * Hd) @ psi0
    strings = list(itertools.product(range(d), repeat=L))
    inside = [sum(t) % n == sum(occ) % n for t in strings]
    # the exact evolution stays in the input's Z_n sector, and leaves it otherwise unconstrained
    assert np.max(np.abs(exact[[not x for x in inside]])) < 1e-12
    pats = [t for t, x in zip(strings, inside) if x]
    ex = np.array([exact[sum(o * d ** (L - 1 - s) for s, o in enumerate(t))] for t in pats])
    assert len({sum(t) for t in pats if abs(ex[pats.index(t)]) > 1e-6}) > 1   # not a U(1) state
    errs = []
    for steps in (4, 8, 16):
        cfg = ham.config_tebd(model, L, d, occ, T / steps, steps, chi_max=0, **p)
        assert cfg["modulus"] == n
        st = fock.run(occ, d, cfg["gates"], modulus=n)
        errs.append(np.linalg.norm(np.array([st.amplitude(t) for t in pats]) - ex))
        if steps == 16:
            m = dense_mps.DenseMPS(occ, d, modulus=n).run(cfg["gates"])
            got = m.amplitudes(np.array(pats))
            assert np.max(np.abs(got - np.array([st.amplitude(t) for t in pats]))) < 1e-12
            for b in range(L + 1):
                assert m.audit_clean(b), b
                assert m.bond_charges(b) == st.schmidt_ranks(b), b
    assert errs[0] > 1e-4
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5, errs


def test_zn_audit_under_truncation():
    """With a bond cap the kept subspace stays closed under the Z_3 charge (the
    audit is clean) and the bookkeeping follows the cut."""
    cfg = ham.config_tebd("clock", 6, 3, [0, 1, 2, 0, 1, 2], 0.2, 6, 6, 1e-12, J=1.0, f=0.5)
    m = dense_mps.DenseMPS(cfg["occupation"], 3, chi_max=6, cutoff=1e-12, modulus=3).run(cfg["gates"])
    assert max(r.discarded for r in m.records) > 1e-8
    for b in range(7):
        assert m.audit_clean(b)
        assert sum(m.bond_charges(b).values()) == m.bond_dims()[b]
        assert set(m.bond_charges(b)) <= {0, 1, 2}


def test_u1_gate_is_a_zn_gate_but_not_conversely():
    """A particle-number-conserving gate also conserves the number mod n; the
    Ising bond changes the number by two and is refused by the U(1) brute
    force."""
    g = ham.trotter_gate(ham.ising_bond(1.0, 0.3), 0.4)
    st = fock.FockState([0, 0, 1], 2, modulus=2)
    st.apply_dense(0, g)
    assert abs(st.amplitude([1, 1, 1])) > 1e-3
    with pytest.raises(ValueError):
        fock.FockState([0, 0, 1], 2).apply_dense(0, g)


@pytest.mark.parametrize("d,n", [(2, 3), (3, 4), (3, 5), (4, 5), (4, 6)])
def test_zn_below_modulus_against_the_full_space(d, n):
    """Z_n with d < n (several local states can no longer share a residue, but
    a charge difference need not be an occupation): random gates that conserve
    (p + q) mod n applied in the full d^L space by Kronecker products.  The
    state stays in the input's class mod n; the brute force and the dense oracle
    reproduce it; the audit is clean and each bond's charges (right-hand
    occupation sums mod n) carry the ranks of the full state's blocks."""
    L = 5
    rng = np.random.default_rng(500 + 10 * d + n)
    occ = [int(x) for x in rng.integers(0, d, size=L)]
    gates = [ham.DenseGate(int(rng.integers(0, L - 1)), ham.random_zn_gate(d, int(rng.integers(1 << 30)), modulus=n))
             for _ in range(14)]
    psi = np.zeros(d ** L, dtype=np.complex128)
    psi[sum(o * d ** (L - 1 - s) for s, o in enumerate(occ))] = 1.0
    for g in gates:
        op = np.kron(np.kron(np.eye(d ** g.site), g.g4), np.eye(d ** (L - g.site - 2)))
        psi = op @ psi
    strings = list(itertools.product(range(d), repeat=L))
    inside = np.array([sum(t) % n == sum(occ) % n for t in strings])
    assert np.max(np.abs(psi[~inside])) < 1e-13
    totals = {sum(t) for t, a in zip(strings, psi) if abs(a) > 1e-6}
    # two sites change their total only when it can wrap past n: 2(d-1) >= n
    assert (len(totals) > 1) == (2 * (d - 1) >= n), totals
    st = fock.run(occ, d, gates, modulus=n)
    ex = np.array([psi[sum(o * d ** (L - 1 - s) for s, o in enumerate(t))] for t in st.basis])
    assert len(st.basis) == int(inside.sum())
    assert np.max(np.abs(st.psi - ex)) < 1e-13
    m = dense_mps.DenseMPS(occ, d, modulus=n).run(gates)
    assert np.max(np.abs(m.amplitudes(np.array(st.basis)) - ex)) < 1e-12
    for b in range(L + 1):
        M = psi.reshape(d ** b, d ** (L - b))
        right = list(itertools.product(range(d), repeat=L - b))
        ranks = {}
        for c in range(n):
            cols = [j for j, t in enumerate(right) if sum(t) % n == c]
            if cols:
                sv = np.linalg.svd(M[:, cols], compute_uv=False)
                r = int(np.sum(sv > 1e-10))
                if r:
                    ranks[c] = r
        assert m.audit_clean(b), b
        assert m.bond_charges(b) == ranks, (b, m.bond_charges(b), ranks)
        assert st.schmidt_ranks(b) == ranks, b
