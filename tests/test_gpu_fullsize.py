"""Full-size and fallback paths of the HIP gate path against the oracle (MI355X).

* a synthetic chi=2048 state imported through mps_create (Gamma, lambda) and
  four central gates at chi_max = 2048: the cut over more than 4096 candidate
  values (the select kernel's device-memory sort), Jacobi sectors of about a
  thousand vectors and the amplitude kernel at bond dimension 2048, against
  results the oracle stored (tests/golden, written from oracle/ only);
* the scalar Jacobi finish and the device-memory sort forced on the bench
  circuit's first layers, against the oracle at the complex128 bars;
* the weight removed by the local cutoff, per gate, against the oracle;
* non-convergence and allocation failure leave the state unchanged.

Tolerances are those of the complex128 path: amplitudes per entry and
normwise 1e-10 relative to the largest reference amplitude, Schmidt values
1e-10 of the bond's largest, bookkeeping bit-exact.
"""
import json
import os

import numpy as np
import pytest

from oracle import dense_mps
from workloads import circuits

pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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
    return per


def lambda_by_charge(m, bond):
    """The GPU's Schmidt values of a bond grouped by charge (ascending charge,
    descending value within a charge, as mps_bond_lambda orders them)."""
    lam = m.bond_lambda(bond)
    out, o = {}, 0
    for c, n in sorted(m.bond_sectors(bond).items()):
        out[c] = lam[o:o + n]
        o += n
    return out


def test_chi2048_synthetic_gates_vs_stored_oracle(mps_cls):
    path = os.path.join(GOLDEN, "SYN_L64_chi2048_4gates.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle results for the chi=2048 gates not written yet")
    ref = json.load(open(path))
    L, N, d = ref["L"], ref["N"], ref["d"]
    charges, gammas, lambdas = circuits.synthetic_state(L, N, d, ref["chi"], seed=ref["state_seed"])
    print(f"chi=2048 synthetic state, sites {ref['sites']}", flush=True)
    m = mps_cls.from_vidal(d, N, charges, gammas, lambdas, chi_max=ref["chi_max"], cutoff=ref["cutoff"])
    del gammas
    layer = {g.site: g for g in circuits.brickwork_layers(L, 1, ref["circuit_seed"])[0]}
    sites = ref["sites"]
    # the gates act on disjoint pairs: one layer equals the oracle's gate-by-gate run
    disc = m.apply_layer(sites, [layer[s].u for s in sites])
    st = m.stats()
    assert st["polish_launches"] == 0
    for i, s in enumerate(sites):
        bond = s + 1
        got = lambda_by_charge(m, bond)
        exp = {int(c): np.array(v) for c, v in ref["lambda_by_charge"][str(bond)].items()}
        total = float(np.sum(m.bond_lambda(bond) ** 2)) + disc[i]
        # every cut binds at chi_max with a margin far above the FP64 noise of the values
        assert ref["margin"][i] is not None and ref["margin"][i] > 1e-9
        assert sum(len(v) for v in got.values()) == ref["kept"][i]
        assert abs(disc[i] - ref["discarded"][i]) <= 1e-10 * total, (s, disc[i], ref["discarded"][i])
        assert sorted(got) == sorted(exp), s
        smax = max(float(v[0]) for v in exp.values())
        for c in exp:
            assert got[c].shape == exp[c].shape, (s, c)
            assert np.max(np.abs(got[c] - exp[c])) <= TOL * smax, (s, c)
    for b in range(L + 1):
        assert m.bond_sectors(b) == {int(k): v for k, v in ref["bond_charges"][b].items()}, b
    pats = np.array(ref["patterns"], dtype=np.int32)
    amp = np.array(ref["amp_re"]) + 1j * np.array(ref["amp_im"])
    close_amps(m.amplitudes(pats), amp)
    m.close()


def _prefix(layers=6):
    cfg = circuits.config_plain_gpu()
    return cfg, cfg["layers"][:layers]


@pytest.fixture(scope="module")
def prefix_oracle():
    cfg, layers = _prefix()
    ref = dense_mps.DenseMPS(cfg["occupation"], 4, chi_max=512, cutoff=1e-12)
    for lay in layers:
        ref.run(lay)
    return ref


@pytest.mark.parametrize("variant", ["scalar_finish", "global_sort"])
def test_forced_fallbacks_on_the_32_mode_prefix(mps_cls, prefix_oracle, variant):
    """First six layers of the L=32, N=16, d=4, chi_max=512 circuit with (a)
    only two blocked Jacobi sweeps, so sectors are finished by the scalar
    one-sided sweeps, or (b) the cut's sort forced through device memory."""
    cfg, layers = _prefix()
    kw = {"blocked_sweeps": 2} if variant == "scalar_finish" else {"select_scratch": 1}
    m = mps_cls(cfg["occupation"], 4, chi_max=512, cutoff=1e-12, **kw)
    disc = []
    for lay in layers:
        disc.extend(m.apply_layer([g.site for g in lay], [g.u for g in lay]))
    ref = prefix_oracle
    if variant == "scalar_finish":
        assert m.stats()["polish_launches"] > 0
    assert min(r.margin for r in ref.records) > 1e-9
    odisc = np.array([r.discarded for r in ref.records])
    assert np.max(np.abs(np.array(disc) - odisc)) <= 1e-12
    for b in range(33):
        assert ref.audit_clean(b)
        assert m.bond_sectors(b) == ref.bond_charges(b), b
        got = np.sort(m.bond_lambda(b))[::-1]
        assert got.shape == ref.lam[b].shape
        assert np.max(np.abs(got - ref.lam[b])) <= TOL * ref.lam[b][0], b
    pats = circuits.sample_patterns(32, 16, 4, 256, 102)
    close_amps(m.amplitudes(pats), ref.amplitudes(pats))
    assert abs(m.norm2() - ref.norm2()) <= TOL
    m.close()


def test_leak_per_gate_vs_oracle(mps_cls):
    """The weight each gate loses to the local cutoff (d=3 < N=6: blocks of
    total photon number 3..4 are projected), per gate, against the oracle's
    record; the split form's products carry it within their own error."""
    cfg = circuits.config_brickwork(12, 6, "first", 3, 12, 10, 1e-12, 21, "t")
    ref = dense_mps.DenseMPS(cfg["occupation"], 3, chi_max=10, cutoff=1e-12).run(cfg["gates"])
    m = mps_cls(cfg["occupation"], 3, chi_max=10, cutoff=1e-12)
    got = []
    for g in cfg["gates"]:
        m.apply_gate(g.site, g.u)
        got.extend(m.last_leaks())
    exp = np.array([r.leak for r in ref.records])
    assert np.max(exp) > 1e-3                      # the cutoff does remove weight
    assert np.max(np.abs(np.array(got) - exp)) <= 1e-12
    assert abs(m.stats()["leak_total"] - exp.sum()) <= 1e-11
    m.close()


def test_noconv_leaves_the_state_unchanged(mps_cls):
    """With one Jacobi sweep allowed, the first sector of two vectors cannot be
    confirmed converged: the update fails with MPS_E_NOCONV before it writes
    anything, and the state reads back exactly as before the call."""
    from paper_2303_11409_amd import MPSError
    cfg = circuits.config_brickwork(8, 4, "first", 4, 6, 0, 1e-12, 61, "t")
    m = mps_cls(cfg["occupation"], 4, cutoff=1e-12, max_sweeps=1)
    pats = circuits.sample_patterns(8, 4, 4, 128, 9)
    failed = False
    for lay in cfg["layers"]:
        before_amp = m.amplitudes(pats)
        before_b = [m.bond_sectors(b) for b in range(9)]
        before_l = [m.bond_lambda(b) for b in range(9)]
        try:
            m.apply_layer([g.site for g in lay], [g.u for g in lay])
        except MPSError as e:
            assert e.status == -5
            failed = True
            assert np.array_equal(m.amplitudes(pats), before_amp)
            assert [m.bond_sectors(b) for b in range(9)] == before_b
            for b in range(9):
                assert np.array_equal(m.bond_lambda(b), before_l[b])
            break
    assert failed
    m.close()


def test_nomem_leaves_the_state_unchanged(mps_cls):
    """An allocator that refuses every request above a byte budget: creation
    within the budget works, a larger update fails with MPS_E_NOMEM and the
    state reads back exactly as before."""
    import ctypes as C
    from paper_2303_11409_amd import MPSError, TorchDevice
    from paper_2303_11409_amd import binding

    class Budget(TorchDevice):
        def __init__(self, budget):
            super().__init__()
            self.budget, self.used = budget, 0
            inner_alloc, inner_free = self._alloc_cb, self._free_cb
            sizes = {}

            def alloc(nbytes, ctx):
                if self.used + nbytes > self.budget:
                    return None
                p = inner_alloc(nbytes, ctx)
                if p:
                    sizes[p] = nbytes
                    self.used += nbytes
                return p

            def free(ptr, ctx):
                self.used -= sizes.pop(ptr, 0)
                inner_free(ptr, ctx)

            self._alloc_cb = binding.ALLOC_FN(alloc)
            self._free_cb = binding.FREE_FN(free)

    cfg = circuits.config_brickwork(16, 8, "first", 4, 8, 64, 1e-12, 62, "t")
    dev = Budget(1 << 40)
    m = mps_cls(cfg["occupation"], 4, chi_max=64, cutoff=1e-12, device=dev)
    pats = circuits.sample_patterns(16, 8, 4, 64, 10)
    lay = cfg["layers"][0]
    m.apply_layer([g.site for g in lay], [g.u for g in lay])
    m.amplitudes(pats)
    # from here on no workspace may grow: the bonds (and so the workspaces of
    # the next updates) grow layer by layer, so some update must be refused
    dev.budget = dev.used + 4096
    failed = False
    for lay in cfg["layers"][1:]:
        before = m.amplitudes(pats)
        before_b = [m.bond_sectors(b) for b in range(17)]
        try:
            m.apply_layer([g.site for g in lay], [g.u for g in lay])
        except MPSError as e:
            assert e.status == -3
            failed = True
            assert np.array_equal(m.amplitudes(pats), before)
            assert [m.bond_sectors(b) for b in range(17)] == before_b
            break
    assert failed
    m.close()
