"""Two independent U(1) charges (U(1) x U(1)) on the HIP gate path (MI355X):
two species of hard-core bosons, local state p = 2 a + b carrying the pair of
species numbers (a, b), each conserved by the hopping and the on-site
interaction of the Trotter gates (the paper's general Abelian symmetries,
Sec. I).  The GPU keeps the pair as one charge; the oracle never uses it
(dense TEBD, joint charge audit; Fock brute force over the pair's sector).

Tolerances are those of the complex128 path: amplitudes 1e-10 of the largest,
Schmidt values 1e-10 of the bond's largest, bookkeeping (charge pairs and
multiplicities) bit-exact where the oracle's cut margins exceed 1e-9.
"""
import itertools

import numpy as np
import pytest

from oracle import dense_mps, fock, sampling
from workloads import hamiltonians as ham

pytestmark = pytest.mark.gpu

TOL = 1e-10
CM = ham.TWO_SPECIES_CHARGES


@pytest.fixture(scope="module")
def mps_cls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2303_11409_amd import MPS
    return MPS


def close_amps(got, ref, tol=TOL):
    scale = max(float(np.max(np.abs(ref))), 1e-300)
    per = float(np.max(np.abs(got - ref))) / scale
    normwise = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
    assert per <= tol and normwise <= tol, (per, normwise)


def run(MPS, cfg):
    m = MPS(cfg["occupation"], 4, chi_max=cfg["chi_max"], cutoff=cfg["cutoff"], charge_map=CM)
    disc = []
    for lay in cfg["layers"]:
        disc.extend(m.apply_layer_dense([g.site for g in lay], [g.g4 for g in lay]))
    return m, np.array(disc)


def test_two_species_exact_vs_brute_force(mps_cls):
    """No truncation: every amplitude of the input's (up, down) sector against
    the Fock-space brute force, strings of other sectors exactly zero, the
    norm, and every bond's charge pairs against the brute force's Schmidt
    ranks per pair."""
    occ = [3, 0, 2, 1, 0, 2]
    cfg = ham.config_tebd("two_species", 6, 4, occ, 0.3, 3, 0, 0.0, J=0.9, U=1.1)
    m, _ = run(mps_cls, cfg)
    st = fock.run(occ, 4, cfg["gates"], charge_map=CM)
    pats = np.array(st.basis, dtype=np.int32)
    close_amps(m.amplitudes(pats), st.psi)
    total = tuple(CM[occ].sum(axis=0))
    others = np.array([t for t in itertools.product(range(4), repeat=6)
                       if tuple(CM[list(t)].sum(axis=0)) != total][:300], dtype=np.int32)
    assert np.all(m.amplitudes(others) == 0)
    assert abs(m.norm2() - 1.0) <= 1e-12
    for b in range(7):
        assert m.bond_sectors(b) == st.schmidt_ranks(b), b
    m.close()


def test_two_species_truncated_vs_oracle(mps_cls):
    """A 10-site quench with the bond cap binding: per-gate discarded weights,
    Schmidt values, every bond's charge pairs (the oracle's joint audit) and
    amplitudes of uniform strings of the sector against the dense oracle; the
    exact samples as the oracle draws them."""
    occ = [3, 0, 1, 2, 1, 0, 3, 2, 0, 1]
    cfg = ham.config_tebd("two_species", 10, 4, occ, 0.15, 8, 14, 1e-12, J=1.0, U=2.0)
    m, disc = run(mps_cls, cfg)
    ref = dense_mps.DenseMPS(occ, 4, chi_max=14, cutoff=1e-12, charge_map=CM).run(cfg["gates"])
    assert min(r.margin for r in ref.records) > 1e-9
    odisc = np.array([r.discarded for r in ref.records])
    assert odisc.max() > 1e-8                       # the cap does cut
    assert np.max(np.abs(disc - odisc)) <= 1e-12
    for b in range(11):
        assert ref.audit_clean(b), b
        assert m.bond_sectors(b) == ref.bond_charges(b), b
        got = np.sort(m.bond_lambda(b))[::-1]
        assert got.shape == ref.lam[b].shape, b
        assert np.max(np.abs(got - ref.lam[b])) <= TOL * ref.lam[b][0], b
    pats = ham.charge_map_patterns(10, CM, CM[occ].sum(axis=0), 400, 11)
    close_amps(m.amplitudes(pats), ref.amplitudes(pats))
    assert abs(m.norm2() - ref.norm2()) <= TOL
    u = np.random.default_rng(75).random((200, 10))
    sp, sprob = m.sample(u)
    rp, rprob, marg = sampling.mps_samples(ref, u, margins=True)
    clear = marg > 1e-9
    assert clear.sum() > 150
    assert np.array_equal(sp[clear], rp[clear])
    assert np.max(np.abs(sprob - rprob) / rprob) <= 1e-10
    assert all(tuple(CM[list(p)].sum(axis=0)) == tuple(CM[occ].sum(axis=0)) for p in sp)
    m.close()


def test_two_species_rules(mps_cls):
    """A two-component state refuses mode unitaries and a gate that turns one
    species into the other (it keeps a + b but not the pair), before any
    change; a gate that conserves both numbers is accepted."""
    from paper_2303_11409_amd import MPSError
    from workloads import circuits
    m = mps_cls([2, 1, 0, 0], 4, charge_map=CM)
    before = m.amplitudes(np.array([[2, 1, 0, 0]], dtype=np.int32))
    with pytest.raises(MPSError):
        m.apply_layer([0], [circuits.beam_splitter(0.3, 0.1)])
    swap = np.eye(16, dtype=np.complex128)
    # |up on site 0> <-> |down on site 0> with site 1 empty: (1,0) <-> (0,1)
    a, b = 2 * 4 + 0, 1 * 4 + 0
    swap[[a, b]] = swap[[b, a]]
    with pytest.raises(MPSError) as e:
        m.apply_layer_dense([0], [swap])
    assert e.value.status == -2
    assert np.array_equal(m.amplitudes(np.array([[2, 1, 0, 0]], dtype=np.int32)), before)
    ok = ham.config_tebd("two_species", 4, 4, [2, 1, 0, 0], 0.2, 1, 0, 0.0, J=1.0, U=0.5)
    for lay in ok["layers"]:
        m.apply_layer_dense([g.site for g in lay], [g.g4 for g in lay])
    assert abs(m.norm2() - 1.0) <= 1e-12
    m.close()
