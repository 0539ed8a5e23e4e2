"""Pins of the oracle's exact sampler (no GPU).

The environment sampler (``sampling.mps_samples``) is compared with the plain
definition (``sampling.brute_force_samples``, marginals summed over a table of
every pattern's probability) whose table comes from a route that shares
nothing with the environments: permanents for an exact circuit, the oracle's
(E1) amplitudes for a truncated state.  The inverse-CDF rule is pinned on the
Hong-Ou-Mandel pair, whose conditionals are known in closed form, and by the
frequencies of many draws.
"""
import numpy as np
import pytest

from oracle import dense_mps, permanent, sampling
from workloads import circuits


def test_exact_circuit_samples_equal_brute_force_and_permanents():
    cfg = circuits.config_small_exact()
    m = dense_mps.DenseMPS(cfg["occupation"], 5).run(cfg["gates"])
    pats = circuits.all_patterns(8, 4, 5)
    table = {tuple(int(x) for x in p): abs(permanent.fock_amplitude(cfg["unitary"], cfg["occupation"], p)) ** 2
             for p in pats}
    u = np.random.default_rng(11).random((200, 8))
    a, pa = sampling.brute_force_samples(table, 8, 5, u)
    b, pb = sampling.mps_samples(m, u)
    assert np.array_equal(a, b)
    assert np.max(np.abs(pa - pb)) < 1e-13
    for pat, p in zip(b, pb):
        assert abs(p - table[tuple(int(x) for x in pat)]) < 1e-13


def test_truncated_state_samples_equal_brute_force():
    cfg = circuits.config_brickwork(9, 4, "first", 3, 8, 5, 1e-12, 13, "t")
    m = dense_mps.DenseMPS(cfg["occupation"], 3, chi_max=5, cutoff=1e-12).run(cfg["gates"])
    assert max(r.discarded for r in m.records) > 1e-6            # truncated and not normalised
    pats = circuits.all_patterns(9, 4, 3)
    amps = m.amplitudes(pats)
    table = {tuple(int(x) for x in p): abs(a) ** 2 for p, a in zip(pats, amps)}
    assert abs(sum(table.values()) - m.norm2()) < 1e-12
    u = np.random.default_rng(12).random((150, 9))
    a, pa = sampling.brute_force_samples(table, 9, 3, u)
    b, pb = sampling.mps_samples(m, u)
    assert np.array_equal(a, b)
    assert np.max(np.abs(pa - pb)) < 1e-12


def test_hong_ou_mandel_inverse_cdf():
    # |1,1> through a 50:50 beam splitter: (2,0) and (0,2) with 1/2 each, never (1,1);
    # the last mode is drawn first: occupation 0 (pattern (2,0)) for u < 1/2, else 2
    m = dense_mps.DenseMPS([1, 1], 3).run([circuits.Gate(0, circuits.beam_splitter(np.pi / 4, 0.0))])
    u = np.array([[0.9, 0.3], [0.9, 0.7], [0.1, 0.49], [0.1, 0.51]])
    pats, prob = sampling.mps_samples(m, u)
    assert pats.tolist() == [[2, 0], [0, 2], [2, 0], [0, 2]]
    assert np.allclose(prob, 0.5, atol=1e-14)


def test_product_state_is_certain():
    m = dense_mps.DenseMPS([0, 2, 1, 0], 3)
    pats, prob = sampling.mps_samples(m, np.random.default_rng(1).random((5, 4)))
    assert (pats == np.array([0, 2, 1, 0])).all()
    assert np.allclose(prob, 1.0, atol=1e-15)


def test_sample_frequencies_follow_the_distribution():
    rng = np.random.default_rng(3)
    gates = [circuits.Gate(int(rng.integers(0, 3)), circuits.haar_unitary(2, int(rng.integers(1 << 30))))
             for _ in range(10)]
    m = dense_mps.DenseMPS([1, 1, 1, 0], 4).run(gates)
    pats = circuits.all_patterns(4, 3, 4)
    amps = m.amplitudes(pats)
    p_exact = np.abs(amps) ** 2 / m.norm2()
    n = 20000
    got, prob = sampling.mps_samples(m, rng.random((n, 4)))
    index = {tuple(int(x) for x in p): k for k, p in enumerate(pats)}
    counts = np.bincount([index[tuple(int(x) for x in g)] for g in got], minlength=len(pats))
    keep = p_exact * n >= 5
    chi2 = float(np.sum((counts[keep] - n * p_exact[keep]) ** 2 / (n * p_exact[keep])))
    dof = int(keep.sum()) - 1
    # 99.9 % quantile of chi-square is below dof + 4.5 sqrt(2 dof) + 10 for these sizes
    assert chi2 < dof + 4.5 * np.sqrt(2 * dof) + 10, (chi2, dof)
    # returned probabilities are those of the patterns
    assert np.max(np.abs(prob - p_exact[[index[tuple(int(x) for x in g)] for g in got]])) < 1e-13
