"""Pins of the oracle's dense-gate (Hamiltonian TEBD) path (no GPU).

The dense-gate update of the oracle (``DenseMPS.apply_dense``) and its brute
force (``FockState.apply_dense``) are checked against closed forms that the
physics of the two U(1) lattice models fixes, independent of both:

* the XX chain (XXZ with Delta = 0) is free fermions: nearest-neighbour
  hopping S+_i S-_{i+1} equals c_i^+ c_{i+1} (Jordan-Wigner, no string between
  neighbours), so every amplitude is a determinant of the product of the
  gates' 2x2 single-particle matrices;
* one magnon of the XXZ chain with any Delta and field moves by a
  single-particle matrix whose entries follow from the two-site energies;
* the Bose-Hubbard chain at U = 0 is linear optics: amplitudes are
  permanents (with a cutoff d above the particle number);
* two sites of the Bose-Hubbard chain with two bosons: the symmetric and
  antisymmetric sectors evolve by a 2x2 and a 1x1 closed form;
* the second-order Trotter error of a whole chain against exp(-i H T) in
  the full Hilbert space falls by four when the step halves, with H built
  from the spin and boson operators directly rather than from the bond list.
Each 2x2 exponential below is written out as
exp(-i t (a0 + a.sigma)) = e^{-i t a0} (cos(|a| t) - i sin(|a| t) a.sigma / |a|).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import dense_mps, fock, permanent, twomode
from workloads import circuits, hamiltonians as ham


def exp2(t, a0, ax, az):
    """exp(-i t (a0 I + ax X + az Z)) for real coefficients."""
    r = math.hypot(ax, az)
    c, s = math.cos(r * t), (math.sin(r * t) / r if r > 0 else t)
    m = np.array([[c - 1j * s * az, -1j * s * ax], [-1j * s * ax, c + 1j * s * az]])
    return np.exp(-1j * t * a0) * m


def gate_times(layers):
    """(site, time) of every gate: recovered from the Trotter schedule."""
    return [(g.site, t) for lay, t in layers for g in lay]


def schedule(L, dt, steps):
    """The merged second-order schedule: list of (bonds, time)."""
    even, odd = list(range(0, L - 1, 2)), list(range(1, L - 1, 2))
    out = [(even, dt / 2)]
    for k in range(steps):
        out.append((odd, dt))
        out.append((even, dt if k < steps - 1 else dt / 2))
    return [(b, t) for b, t in out if b]


def embed(m2, s, L):
    u = np.eye(L, dtype=np.complex128)
    u[s:s + 2, s:s + 2] = m2
    return u


def oracle_runs(occ, d, layers, pats):
    gates = [g for lay in layers for g in lay]
    st = fock.run(occ, d, gates)
    mp = dense_mps.DenseMPS(occ, d).run(gates)
    return np.array([st.amplitude(p) for p in pats]), mp.amplitudes(pats), st, mp


def test_trotter_schedule_times():
    L, dt, steps = 7, 0.1, 3
    cfg = ham.config_xxz(L=L, steps=steps, dt=dt, chi_max=0, delta=0.0)
    sch = schedule(L, dt, steps)
    assert [sorted(g.site for g in lay) for lay in cfg["layers"]] == [b for b, _ in sch]
    # each layer's gates are exp(-i t h) of their bonds: recover t from one element
    hb = ham.bond_hamiltonians("xxz", L, 2, J=1.0, delta=0.0)
    for lay, (_, t) in zip(cfg["layers"], sch):
        for g in lay:
            assert np.allclose(g.g4, ham.trotter_gate(hb[g.site], t), atol=1e-14)
    # total time per bond = steps * dt
    tot = {}
    for b, t in sch:
        for s in b:
            tot[s] = tot.get(s, 0.0) + t
    assert all(abs(v - steps * dt) < 1e-12 for v in tot.values())


def test_xx_chain_is_free_fermions():
    L, dt, steps, J = 8, 0.35, 3, 1.3
    occ = ham.neel(L)
    cfg = ham.config_tebd("xxz", L, 2, occ, dt, steps, chi_max=0, J=J, delta=0.0, hz=0.0)
    # single-particle matrix of one gate of time t: exp(-i t (J/2) X)
    U = np.eye(L, dtype=np.complex128)
    for b, t in schedule(L, dt, steps):
        for s in b:
            U = embed(exp2(t, 0.0, J / 2, 0.0), s, L) @ U
    n = sum(occ)
    pats = circuits.all_patterns(L, n, 2)
    cols = [j for j in range(L) if occ[j]]
    ref = np.array([np.linalg.det(U[np.ix_([i for i in range(L) if p[i]], cols)]) for p in pats])
    bf, mp, st, dm = oracle_runs(occ, 2, cfg["layers"], pats)
    assert np.max(np.abs(bf - ref)) < 1e-12
    assert np.max(np.abs(mp - ref)) < 1e-12
    # the boson formula is a different answer: the determinant is what is pinned
    perm = np.array([permanent.fock_amplitude(U, occ, p) for p in pats])
    assert np.max(np.abs(perm - ref)) > 1e-2
    assert abs(dm.norm2() - 1.0) < 1e-12


def test_xxz_one_magnon_closed_form():
    L, dt, steps, J, delta, hz = 7, 0.3, 4, 1.1, 0.8, 0.35
    occ = [0, 0, 0, 1, 0, 0, 0]
    cfg = ham.config_tebd("xxz", L, 2, occ, dt, steps, chi_max=0, J=J, delta=delta, hz=hz)
    U = np.eye(L, dtype=np.complex128)
    for b, t in schedule(L, dt, steps):
        for s in b:
            wl = 1.0 if s == 0 else 0.5
            wr = 1.0 if s == L - 2 else 0.5
            # both spins down: J Delta / 4 + hz (wl + wr) / 2; the magnon on the bond:
            # diagonal -J Delta / 4 -+ hz (wl - wr) / 2, hopping J / 2
            e_out = J * delta / 4 + hz * (wl + wr) / 2
            m = np.diag(np.full(L, np.exp(-1j * t * e_out)))
            m[s:s + 2, s:s + 2] = exp2(t, -J * delta / 4, J / 2, -hz * (wl - wr) / 2)
            U = m @ U
    pats = circuits.all_patterns(L, 1, 2)
    ref = np.array([U[list(p).index(1), 3] for p in pats])
    bf, mp, _, _ = oracle_runs(occ, 2, cfg["layers"], pats)
    assert np.max(np.abs(bf - ref)) < 1e-12
    assert np.max(np.abs(mp - ref)) < 1e-12


def test_bose_hubbard_free_limit_is_linear_optics():
    L, dt, steps, J, mu = 5, 0.25, 3, 0.9, 0.4
    occ = [1, 0, 1, 0, 1]
    d = sum(occ) + 1                     # no occupation reaches the cutoff
    cfg = ham.config_tebd("bose_hubbard", L, d, occ, dt, steps, chi_max=0, J=J, U=0.0, mu=mu)
    U = np.eye(L, dtype=np.complex128)
    for b, t in schedule(L, dt, steps):
        for s in b:
            wl = 1.0 if s == 0 else 0.5
            wr = 1.0 if s == L - 2 else 0.5
            # one boson on the bond: -J X hopping, -mu w on each site
            U = embed(exp2(t, -mu * (wl + wr) / 2, -J, -mu * (wl - wr) / 2), s, L) @ U
    pats = circuits.all_patterns(L, sum(occ), d)
    ref = np.array([permanent.fock_amplitude(U, occ, p) for p in pats])
    bf, mp, _, _ = oracle_runs(occ, d, cfg["layers"], pats)
    assert np.max(np.abs(bf - ref)) < 1e-12
    assert np.max(np.abs(mp - ref)) < 1e-12


@pytest.mark.parametrize("start", [(1, 1), (2, 0)])
def test_bose_hubbard_two_sites_two_bosons(start):
    J, U, mu, t = 0.7, 2.3, 0.2, 0.9
    g = ham.trotter_gate(ham.bose_hubbard_bond(3, J, U, mu, 1.0, 1.0), t)
    lay = [[ham.DenseGate(0, g)]]
    # symmetric sector {(|20> + |02>)/sqrt2, |11>}: [[U - 2mu, -2J], [-2J, -2mu]];
    # antisymmetric (|20> - |02>)/sqrt2: U - 2mu
    sym = exp2(t, U / 2 - 2 * mu, -2 * J, U / 2)
    anti = np.exp(-1j * t * (U - 2 * mu))
    if start == (1, 1):
        v = sym @ np.array([0.0, 1.0])
        ref = {(2, 0): v[0] / math.sqrt(2), (1, 1): v[1], (0, 2): v[0] / math.sqrt(2)}
    else:
        v = sym @ np.array([1 / math.sqrt(2), 0.0])
        a = anti / math.sqrt(2)
        ref = {(2, 0): (v[0] + a) / math.sqrt(2), (1, 1): v[1], (0, 2): (v[0] - a) / math.sqrt(2)}
    pats = np.array(list(ref))
    bf, mp, _, _ = oracle_runs(list(start), 3, lay, pats)
    want = np.array([ref[tuple(p)] for p in pats])
    assert np.max(np.abs(bf - want)) < 1e-13
    assert np.max(np.abs(mp - want)) < 1e-13


def _site_op(op, i, L):
    d = op.shape[0]
    return np.kron(np.kron(np.eye(d ** i), op), np.eye(d ** (L - i - 1)))


def _xxz_direct(L, J, delta, hz):
    sx = np.array([[0, 1], [1, 0]]) / 2
    sy = np.array([[0, -1j], [1j, 0]]) / 2
    sz = np.diag([-0.5, 0.5])            # occupation 1 = spin up
    H = sum(J * (_site_op(sx, i, L) @ _site_op(sx, i + 1, L) + _site_op(sy, i, L) @ _site_op(sy, i + 1, L)
                 + delta * _site_op(sz, i, L) @ _site_op(sz, i + 1, L)) for i in range(L - 1))
    return H - hz * sum(_site_op(sz, i, L) for i in range(L))


def _bh_direct(L, d, J, U, mu):
    b = np.diag(np.sqrt(np.arange(1, d)), 1)
    n = np.diag(np.arange(d, dtype=float))
    H = -J * sum(_site_op(b.T, i, L) @ _site_op(b, i + 1, L) + _site_op(b, i, L) @ _site_op(b.T, i + 1, L)
                 for i in range(L - 1))
    return H + sum(_site_op(0.5 * U * n @ (n - np.eye(d)) - mu * n, i, L) for i in range(L))


@pytest.mark.parametrize("model", ["xxz", "bose_hubbard"])
def test_bonds_sum_to_hamiltonian_and_trotter_order(model):
    L = 6
    if model == "xxz":
        d, occ, p = 2, ham.neel(L), dict(J=1.0, delta=1.4, hz=0.3)
        Hd = _xxz_direct(L, **p)
    else:
        d, occ, p = 3, [1, 2, 0, 1, 1, 0], dict(J=1.0, U=1.7, mu=0.25)
        Hd = _bh_direct(L, d, **p)
    hb = ham.bond_hamiltonians(model, L, d, **p)
    assert np.max(np.abs(ham.hamiltonian_dense(hb, L, d) - Hd)) < 1e-13
    T = 0.8
    psi0 = np.zeros(d ** L, dtype=np.complex128)
    psi0[sum(o * d ** (L - 1 - s) for s, o in enumerate(occ))] = 1.0
    import scipy.linalg
    exact = scipy.linalg.expm(-1j * T * Hd) @ psi0
    pats = circuits.all_patterns(L, sum(occ), d)
    idx = [sum(int(o) * d ** (L - 1 - s) for s, o in enumerate(pt)) for pt in pats]
    ex = exact[idx]
    # the whole evolution stays in the N-particle sector of the full space
    assert abs(np.linalg.norm(ex) - 1.0) < 1e-12
    errs = []
    for steps in (4, 8, 16):
        cfg = ham.config_tebd(model, L, d, occ, T / steps, steps, chi_max=0, **p)
        st = fock.run(occ, d, cfg["gates"])
        errs.append(np.linalg.norm(np.array([st.amplitude(pt) for pt in pats]) - ex))
    assert errs[0] > 1e-4
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5, errs


def test_dense_path_equals_mode_unitary_path():
    rng = np.random.default_rng(9)
    L, d = 5, 3
    occ = [2, 0, 1, 1, 0]
    gates = [circuits.Gate(int(rng.integers(0, L - 1)), circuits.haar_unitary(2, int(rng.integers(1 << 30))))
             for _ in range(12)]
    dgates = [ham.DenseGate(g.site, twomode.dense(g.u, d)) for g in gates]
    pats = circuits.all_patterns(L, sum(occ), d)
    a = fock.run(occ, d, gates)
    b = fock.run(occ, d, dgates)
    assert np.max(np.abs(a.psi - b.psi)) < 1e-14
    m1 = dense_mps.DenseMPS(occ, d, chi_max=6).run(gates)
    m2 = dense_mps.DenseMPS(occ, d, chi_max=6).run(dgates)
    assert np.max(np.abs(m1.amplitudes(pats) - m2.amplitudes(pats))) < 1e-13


def test_random_charge_conserving_gate_structure():
    for d in (2, 3, 4):
        g = ham.random_charge_conserving(d, 7)
        assert np.max(np.abs(g.conj().T @ g - np.eye(d * d))) < 1e-13
        for r, c in itertools.product(range(d * d), repeat=2):
            if r // d + r % d != c // d + c % d:
                assert g[r, c] == 0


def test_brute_force_rejects_charge_breaking_gate():
    g = np.eye(4, dtype=np.complex128)
    g[1, 0] = 0.1                         # |00> -> |01>: adds a particle
    st = fock.FockState([0, 0, 1], 2)
    st.apply_dense(1, np.eye(4))
    with pytest.raises(ValueError):
        fock.FockState([0, 0, 1], 2).apply_dense(0, g)


def test_site_dependent_potential_sums_to_hamiltonian():
    """With a chemical potential per site the bond Hamiltonians still sum to
    H = -J sum (b^+ b + h.c.) + U/2 sum n(n-1) - sum_i mu_i n_i."""
    L, d, J, U = 5, 3, 0.8, 1.3
    mu = [0.3, -0.2, 0.45, 0.0, -0.35]
    hb = ham.bond_hamiltonians("bose_hubbard", L, d, J=J, U=U, mu_sites=mu)
    b = np.diag(np.sqrt(np.arange(1, d)), 1)
    n = np.diag(np.arange(d, dtype=float))
    H = -J * sum(_site_op(b.T, i, L) @ _site_op(b, i + 1, L) + _site_op(b, i, L) @ _site_op(b.T, i + 1, L)
                 for i in range(L - 1))
    H = H + sum(_site_op(0.5 * U * n @ (n - np.eye(d)) - mu[i] * n, i, L) for i in range(L))
    assert np.max(np.abs(ham.hamiltonian_dense(hb, L, d) - H)) < 1e-13
