"""Seeded input generators (CPU): the synthetic saturated state and the
batching and serving mixes.  They hold no arithmetic of the method; these
tests check that the inputs have the structure the method requires."""
import numpy as np

from workloads import circuits


def test_synthetic_state_obeys_the_charge_rule():
    L, N, d, chi = 12, 6, 4, 40
    ch, gam, lam = circuits.synthetic_state(L, N, d, chi, seed=3)
    assert len(ch) == L + 1 and len(gam) == L and len(lam) == L + 1
    assert ch[0] == [N] and ch[L] == [0]                      # Eq. (E4) boundaries
    for k in range(L + 1):
        c = np.array(ch[k])
        assert np.all(np.diff(c) >= 0)                          # sorted
        assert np.all((c >= max(0, N - k * (d - 1))) & (c <= min(N, (L - k) * (d - 1))))
        assert len(c) <= chi and len(lam[k]) == len(c)
        assert np.all(lam[k] > 0) and np.max(lam[k]) <= 1.0
    for s in range(L):
        cl, cr = np.array(ch[s])[:, None], np.array(ch[s + 1])[None, :]
        allowed = (cl - cr >= 0) & (cl - cr <= d - 1)
        assert gam[s].shape == allowed.shape
        assert np.all(gam[s][~allowed] == 0)                    # Eq. (E2): no entry off the charge rule
        assert np.all(np.abs(gam[s][allowed]) > 0)
        # every charge has a partner on both neighbouring bonds
        assert np.all(allowed.any(axis=1)) and np.all(allowed.any(axis=0))


def test_synthetic_state_saturates_the_cap():
    ch, _, _ = circuits.synthetic_state(24, 12, 4, 256, seed=5)
    dims = [len(c) for c in ch]
    assert max(dims) == 256 and dims[12] == 256


def test_mixes_are_seeded_and_shaped():
    a = circuits.config_batch_mix(16, seed=4)
    b = circuits.config_batch_mix(16, seed=4)
    for x, y in zip(a, b):
        assert x["L"] == y["L"] and x["chi_max"] == y["chi_max"]
        assert all(np.array_equal(g.u, h.u) for g, h in zip(x["gates"], y["gates"]))
        assert 16 <= x["L"] <= 48 and x["chi_max"] in (64, 128, 256, 512)
        assert sum(x["occupation"]) == x["L"] // 2 and len(x["layers"]) == x["L"]
    specs = circuits.serving_mix_specs(2000, seed=5)
    large = [s for s in specs if s["L"] == 64]
    assert 0.03 < len(large) / len(specs) < 0.07
    assert all(s["chi_max"] == 1024 and s["depth"] == 64 and s["n_photons"] == 32 for s in large)
    c = circuits.config_from_spec(specs[0])
    assert len(c["layers"]) == specs[0]["depth"] and sum(c["occupation"]) == specs[0]["n_photons"]


def test_zn_input_generators():
    """Z_n patterns lie in the requested charge class and cover it; random Z_n
    gates are unitary and conserve the local charge mod n exactly."""
    from workloads import hamiltonians as ham
    pats = ham.zn_patterns(6, 3, 4, 400, 1)
    assert pats.shape == (400, 6) and pats.min() >= 0 and pats.max() < 3
    assert np.all(pats.sum(axis=1) % 3 == 1)
    assert len({tuple(p) for p in pats.tolist()}) > 150          # 243 strings in the class
    for d in (2, 3, 4):
        g = ham.random_zn_gate(d, 5)
        assert np.max(np.abs(g.conj().T @ g - np.eye(d * d))) < 1e-13
        for r in range(d * d):
            for c in range(d * d):
                if (r // d + r % d - c // d - c % d) % d:
                    assert g[r, c] == 0
    # n above d: the charge classes of p + q mod n (some of them one pair long)
    for d, n in ((2, 3), (3, 4), (3, 5)):
        g = ham.random_zn_gate(d, 6, modulus=n)
        assert np.max(np.abs(g.conj().T @ g - np.eye(d * d))) < 1e-13
        for r in range(d * d):
            for c in range(d * d):
                if (r // d + r % d - c // d - c % d) % n:
                    assert g[r, c] == 0
        # a class holding more than one pair mixes it: not a diagonal gate
        assert np.count_nonzero(np.abs(g) > 1e-12) > d * d
    pats = ham.zn_patterns(5, 3, 2, 300, 2, modulus=5)
    assert pats.max() < 3 and np.all(pats.sum(axis=1) % 5 == 2)


def test_charge_map_patterns_uniform_over_the_sector():
    """Strings drawn for a pair of species numbers carry exactly that pair and
    cover the sector uniformly (chi-square against the exact count)."""
    import collections
    import math

    import scipy.stats
    from workloads import hamiltonians as ham
    cm = ham.TWO_SPECIES_CHARGES
    pats = ham.charge_map_patterns(6, cm, (3, 2), 20000, 2)
    assert all(tuple(cm[list(p)].sum(axis=0)) == (3, 2) for p in pats)
    cnt = collections.Counter(map(tuple, pats.tolist()))
    assert len(cnt) == math.comb(6, 3) * math.comb(6, 2)     # hard-core species on 6 sites
    assert scipy.stats.chisquare(np.array(list(cnt.values()))).pvalue > 1e-3
