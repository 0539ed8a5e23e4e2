"""Pins of the oracle's import of a charge-labelled Vidal state (no GPU).

DenseMPS.from_vidal turns per-bond right-charges, Gamma matrices without a
physical index and Schmidt values into the dense MPS, by the Kronecker delta of
Eq. (E2) (Sec. II).  It is checked against the (E2) sum written out over index
paths with explicit loops, against a brute-force Fock vector evolved by the
same gate, and against the product-state constructor.
"""
import collections

import numpy as np
import pytest

from oracle import dense_mps, fock
from workloads import circuits


def e2_amplitude(occ, charges, gammas, lambdas):
    """c_{i_1..i_L} of Eq. (E2) by a sum over every index path (a_1, ..., a_{L-1}):
    prod_s Gamma[s][a_s, a_{s+1}] lambda[s+1][a_{s+1}], each factor kept only when
    c_s(a_s) - c_{s+1}(a_{s+1}) equals the occupation i_s."""
    L = len(gammas)
    total = 0.0 + 0.0j

    def rec(s, a, acc):
        nonlocal total
        if s == L:
            total += acc
            return
        for b in range(len(charges[s + 1])):
            if charges[s][a] - charges[s + 1][b] != occ[s]:
                continue
            g = gammas[s][a, b]
            if g == 0:
                continue
            rec(s + 1, b, acc * g * lambdas[s + 1][b])

    rec(0, 0, 1.0 + 0.0j)
    return total


@pytest.fixture(scope="module")
def small_state():
    # L=6, N=4, d=3: bonds up to 10 indices, several charges per bond
    return circuits.synthetic_state(6, 4, 3, 10, lam_min=0.1, seed=11)


@pytest.mark.parametrize("form", ["hastings", "vidal"])
def test_import_amplitudes_equal_the_e2_sum(small_state, form):
    charges, gammas, lambdas = small_state
    m = dense_mps.DenseMPS.from_vidal(3, 4, charges, gammas, lambdas, form=form)
    pats = circuits.all_patterns(6, 4, 3)
    got = m.amplitudes(pats)
    exp = np.array([e2_amplitude(p, charges, gammas, lambdas) for p in pats.tolist()])
    assert np.count_nonzero(exp) > len(exp) // 2
    assert np.max(np.abs(got - exp)) <= 1e-13 * np.max(np.abs(exp))
    # a wrong photon number has no charge path: exactly zero in the dense form too
    assert m.amplitude([1, 1, 1, 1, 1, 0]) == 0.0


def test_import_labels_are_the_audit_charges(small_state):
    charges, gammas, lambdas = small_state
    m = dense_mps.DenseMPS.from_vidal(3, 4, charges, gammas, lambdas)
    for b, ch in enumerate(charges):
        assert m.bond_charges(b) == dict(sorted(collections.Counter(ch).items()))
        assert m.audit_clean(b)


def test_import_then_gate_equals_brute_force(small_state):
    """An untruncated gate on the imported state gives the Fock vector of the
    (E2) amplitudes with the gate applied by explicit index loops."""
    charges, gammas, lambdas = small_state
    u = circuits.beam_splitter(0.61, 2.3)
    for site in (0, 2, 4):
        m = dense_mps.DenseMPS.from_vidal(3, 4, charges, gammas, lambdas)
        st = fock.FockState([2, 2, 0, 0, 0, 0], 3)
        st.psi = np.array([e2_amplitude(t, charges, gammas, lambdas) for t in st.basis])
        m.apply_gate(site, u)
        st.apply(site, u)
        pats = np.array(st.basis, dtype=np.int32)
        got = m.amplitudes(pats)
        assert np.max(np.abs(got - st.psi)) <= 1e-12 * np.max(np.abs(st.psi)), site
        assert m.audit_clean(site + 1)
        assert abs(m.norm2() - st.norm2()) <= 1e-12 * st.norm2()


def test_import_of_a_product_state_matches_the_constructor():
    occ = [2, 0, 1, 3, 0]
    N = sum(occ)
    charges = [[N - sum(occ[:b])] for b in range(6)]
    gam = [np.ones((1, 1), dtype=np.complex128) for _ in range(5)]
    lam = [np.ones(1) for _ in range(6)]
    a = dense_mps.DenseMPS.from_vidal(4, N, charges, gam, lam, chi_max=6, cutoff=1e-12)
    b = dense_mps.DenseMPS(occ, 4, chi_max=6, cutoff=1e-12)
    gates = circuits.brickwork(5, 4, 9)
    a.run(gates)
    b.run(gates)
    pats = circuits.all_patterns(5, N, 4)
    np.testing.assert_array_equal(a.amplitudes(pats), b.amplitudes(pats))
    assert [r.discarded for r in a.records] == [r.discarded for r in b.records]


def test_import_rejects_charge_violations(small_state):
    charges, gammas, lambdas = small_state
    bad = [g.copy() for g in gammas]
    # an entry whose charge difference is outside 0..d-1
    cl, cr = np.array(charges[2])[:, None], np.array(charges[3])[None, :]
    i, j = np.argwhere((cl - cr < 0) | (cl - cr > 2))[0]
    bad[2][i, j] = 1.0
    with pytest.raises(ValueError):
        dense_mps.DenseMPS.from_vidal(3, 4, charges, bad, lambdas)
    wrong = [list(c) for c in charges]
    wrong[0] = [3]
    with pytest.raises(ValueError):
        dense_mps.DenseMPS.from_vidal(3, 4, wrong, gammas, lambdas)


def test_charge_path_patterns_follow_present_charges(small_state):
    charges, _, _ = small_state
    pats = circuits.charge_path_patterns(charges, 3, 200, 3)
    present = [set(c) for c in charges]
    for p in pats.tolist():
        c = 4
        for k, x in enumerate(p):
            assert 0 <= x < 3
            c -= x
            assert c in present[k + 1]
        assert c == 0
