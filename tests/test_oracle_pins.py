"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each check compares the oracle with something other than itself: a closed
form (permanents, Hong-Ou-Mandel, factorials), a brute-force computation
(Fock state vector, exhaustive sorting), or an invariant (unitarity, norm,
photon-number conservation).  A plausible slip anywhere in the oracle -- a
transposed mode unitary, a missing sqrt(n!) factor, a wrong contraction
index, a dropped gate term -- breaks at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import dense_mps, fock, permanent, twomode
from workloads import circuits


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rand_u2(rng):
    return circuits.haar_unitary(2, int(rng.integers(1 << 30)))


# ---------------------------------------------------------------- permanents
def test_ryser_equals_definition():
    rng = np.random.default_rng(0)
    for n in range(1, 7):
        a = rand_c(rng, n, n)
        assert abs(permanent.permanent_ryser(a) - permanent.permanent_naive(a)) <= 1e-12 * (1 + abs(permanent.permanent_naive(a)))


def test_permanent_closed_forms():
    for n in range(1, 9):
        assert abs(permanent.permanent_ryser(np.eye(n)) - 1.0) < 1e-12
        assert abs(permanent.permanent_ryser(np.ones((n, n))) - math.factorial(n)) < 1e-9 * math.factorial(n)
    a = np.array([[1 + 2j, 3 - 1j], [0.5j, -2.0]])
    assert abs(permanent.permanent_ryser(a) - (a[0, 0] * a[1, 1] + a[0, 1] * a[1, 0])) < 1e-14


# ---------------------------------------------------------- two-mode gate
def test_one_photon_block_is_the_mode_unitary():
    rng = np.random.default_rng(1)
    for _ in range(5):
        u = rand_u2(rng)
        np.testing.assert_allclose(twomode.block(u, 1), u, atol=1e-15)


def test_blocks_unitary_without_cutoff():
    rng = np.random.default_rng(2)
    for _ in range(3):
        u = rand_u2(rng)
        for n in range(0, 7):
            g = twomode.block(u, n)
            np.testing.assert_allclose(g.conj().T @ g, np.eye(n + 1), atol=1e-13)


def test_hong_ou_mandel_zero():
    u = np.array([[1, -1], [1, 1]], dtype=np.complex128) / math.sqrt(2)
    assert abs(twomode.element(u, 1, 1, 1, 1)) < 1e-16
    assert abs(abs(twomode.element(u, 2, 0, 1, 1)) ** 2 - 0.5) < 1e-15


def test_gate_elements_equal_permanent_formula():
    rng = np.random.default_rng(3)
    u = rand_u2(rng)
    for tot in range(0, 6):
        for m in range(tot + 1):
            for p in range(tot + 1):
                ref = permanent.fock_amplitude(u, (m, tot - m), (p, tot - p))
                assert abs(twomode.element(u, p, tot - p, m, tot - m) - ref) < 1e-13


def test_dense_gate_conserves_and_projects():
    rng = np.random.default_rng(4)
    u = rand_u2(rng)
    d = 3
    g = twomode.dense(u, d)
    for p, q, m, n in itertools.product(range(d), repeat=4):
        if p + q != m + n:
            assert g[p * d + q, m * d + n] == 0
        else:
            assert g[p * d + q, m * d + n] == twomode.element(u, p, q, m, n)
    # with the cutoff the n >= d blocks are not unitary (leak)
    blk = twomode.block(u, 3, d)
    assert np.linalg.norm(blk.conj().T @ blk - np.eye(blk.shape[0])) > 1e-3


# ---------------------------------------------------------- input generators
def test_haar_and_clements():
    u = circuits.haar_unitary(8, 1)
    np.testing.assert_allclose(u.conj().T @ u, np.eye(8), atol=1e-14)
    gates, _ = circuits.clements_gates(u)
    assert len(gates) == 28
    full = circuits.clements_circuit(u)
    np.testing.assert_allclose(circuits.circuit_unitary(full, 8), u, atol=1e-13)
    for g in full:
        np.testing.assert_allclose(g.u.conj().T @ g.u, np.eye(2), atol=1e-14)


def test_brickwork_shape():
    layers = circuits.brickwork_layers(32, 32, 2)
    assert sum(len(l) for l in layers) == 496
    for lay in layers:
        sites = [g.site for g in lay]
        assert all(b - a >= 2 for a, b in zip(sites, sites[1:]))


def test_pattern_sampler_uniform():
    L, N, d = 4, 3, 3
    allp = circuits.all_patterns(L, N, d)
    assert len(allp) == circuits.count_patterns(L, N, d)
    smp = circuits.sample_patterns(L, N, d, 6000, seed=7)
    assert np.all(smp.sum(1) == N) and smp.max() < d
    keys = {tuple(p): 0 for p in allp}
    for p in smp:
        keys[tuple(p)] += 1
    counts = np.array(list(keys.values()), dtype=float)
    exp = 6000 / len(allp)
    chi2 = float(np.sum((counts - exp) ** 2 / exp))
    assert chi2 < 3 * len(allp)


# ---------------------------------------------------------- dense MPS oracle
@pytest.fixture(scope="module")
def exact_case():
    cfg = circuits.config_small_exact()
    pats = circuits.all_patterns(8, 4, 5)
    ref = np.array([permanent.fock_amplitude(cfg["unitary"], cfg["occupation"], p) for p in pats])
    return cfg, pats, ref


def test_exact_circuit_matches_permanents(exact_case):
    cfg, pats, ref = exact_case
    assert len(pats) == 330
    assert abs(np.sum(np.abs(ref) ** 2) - 1) < 1e-13
    for form in ("hastings", "vidal"):
        m = dense_mps.DenseMPS(cfg["occupation"], 5, form=form).run(cfg["gates"])
        amp = m.amplitudes(pats)
        assert np.max(np.abs(amp - ref)) < 1e-12
        assert abs(1 - m.norm2()) < 1e-13


def test_fock_brute_force_matches_permanents(exact_case):
    cfg, pats, ref = exact_case
    st = fock.run(cfg["occupation"], 5, cfg["gates"])
    got = np.array([st.amplitude(p) for p in pats])
    assert np.max(np.abs(got - ref)) < 1e-13


def test_conservation_off_sector_amplitudes(exact_case):
    cfg, _, _ = exact_case
    m = dense_mps.DenseMPS(cfg["occupation"], 5).run(cfg["gates"])
    rng = np.random.default_rng(5)
    bad = rng.integers(0, 5, size=(200, 8))
    bad = bad[bad.sum(1) != 4]
    assert np.max(np.abs(m.amplitudes(bad))) < 1e-14


def test_bookkeeping_equals_brute_force_schmidt_ranks(exact_case):
    cfg, _, _ = exact_case
    m = dense_mps.DenseMPS(cfg["occupation"], 5).run(cfg["gates"])
    st = fock.run(cfg["occupation"], 5, cfg["gates"])
    for b in range(1, 8):
        assert m.audit_clean(b)
        assert m.bond_charges(b) == dict(sorted(st.schmidt_ranks(b).items()))
    assert m.bond_charges(0) == {4: 1} and m.bond_charges(8) == {0: 1}


def test_product_state_charges():
    occ = [2, 0, 1, 3, 0, 1]
    m = dense_mps.DenseMPS(occ, 4)
    for b in range(7):
        assert m.bond_charges(b) == {sum(occ[b:]): 1}


@pytest.mark.parametrize("seed", range(6))
def test_cutoff_leak_matches_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    L = int(rng.integers(3, 7))
    d = int(rng.integers(2, 4))
    occ = [int(x) for x in rng.integers(0, d, size=L)]
    if sum(occ) == 0:
        occ[0] = 1
    gates = [circuits.Gate(int(rng.integers(0, L - 1)), rand_u2(rng)) for _ in range(3 * L)]
    st = fock.run(occ, d, gates)
    m = dense_mps.DenseMPS(occ, d).run(gates)
    pats = circuits.all_patterns(L, sum(occ), d)
    got = m.amplitudes(pats)
    ref = np.array([st.amplitude(p) for p in pats])
    assert np.max(np.abs(got - ref)) < 1e-12
    assert abs(m.norm2() - st.norm2()) < 1e-12
    assert st.norm2() <= 1 + 1e-13


def _cut_brute(s, chi_max, cutoff, zero_tol):
    n = len(s)
    tot = sum(x * x for x in s)
    best = None
    for k in range(n + 1):
        tail = sum(x * x for x in s[k:])
        if tail <= cutoff * tot:
            best = k
            break
    kz = sum(1 for x in s if x > zero_tol * s[0])
    k = min(best, kz)
    if chi_max > 0:
        k = min(k, chi_max)
    return max(k, 1)


def test_truncation_rule_brute_force():
    rng = np.random.default_rng(6)
    for _ in range(300):
        n = int(rng.integers(1, 40))
        s = np.sort(np.abs(rng.standard_normal(n)) ** rng.uniform(1, 12))[::-1]
        s[rng.random(n) < 0.1] = 0.0
        s = np.sort(s)[::-1]
        if s[0] == 0:
            s[0] = 1.0
        chi = int(rng.integers(0, 45))
        eps = float(10.0 ** rng.uniform(-14, -1))
        r = dense_mps.truncation(s, chi, eps, 1e-13)
        assert r.kept == _cut_brute(list(s), chi, eps, 1e-13)
        assert abs(r.discarded - float(np.sum(s[r.kept:] ** 2))) <= 1e-15 * r.total


def test_discarded_weight_identity_and_norm_monotone():
    # d > N: gates are unitary, so every norm change is truncation
    cfg = circuits.config_brickwork(10, 3, "first", 4, 10, 6, 1e-12, 11, "t")
    m = dense_mps.DenseMPS(cfg["occupation"], 4, chi_max=6, cutoff=1e-12)
    prev = 1.0
    total_disc = 0.0
    for g in cfg["gates"]:
        rec = m.apply_gate(g.site, g.u)
        total_disc += rec.discarded
        nrm = m.norm2()
        assert nrm <= prev + 1e-13
        prev = nrm
        assert abs(rec.leak) < 1e-13
    assert total_disc > 1e-8              # the cap really truncated
    loss = 1.0 - prev
    assert abs(loss - total_disc) <= 0.05 * total_disc + 1e-13


def test_untruncated_unitary_norm_preserved():
    cfg = circuits.config_brickwork(10, 4, "first", 5, 10, 0, 0.0, 12, "t")
    m = dense_mps.DenseMPS(cfg["occupation"], 5).run(cfg["gates"])
    assert abs(1 - m.norm2()) < 1e-13
    u = circuits.circuit_unitary(cfg["gates"], 10)
    rng = np.random.default_rng(9)
    pats = circuits.sample_patterns(10, 4, 5, 40, 9)
    for p in pats:
        assert abs(m.amplitude(p) - permanent.fock_amplitude(u, cfg["occupation"], p)) < 1e-12
