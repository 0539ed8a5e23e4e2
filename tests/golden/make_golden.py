"""Writes the stored oracle results used by the full-size GPU parity test.

Runs ONLY the CPU oracle (oracle/dense_mps.py) on the seeded workload from
workloads/circuits.py or workloads/hamiltonians.py and stores, as JSON text:
  * the amplitudes of 1024 occupation patterns drawn uniformly (seed 102 for
    the 32-mode circuit, 103 for the 64-mode one, 104, 105 and 106 for the
    XXZ, Bose-Hubbard and Ising quenches; for the Ising quench among strings
    of the input's charge mod 2) plus the input pattern,
  * <psi|psi> by full contraction,
  * every bond's right-charge histogram from the oracle's charge audit,
  * every gate's discarded weight and cut margin,
  * the Schmidt values of the central bonds.

A name in PREFIXES stores the first layers of a workload only (every bond's
Schmidt values too): BH_L64_d4_chi256_T3_L53 is the Bose-Hubbard quench up to
its first near-tie at the cut.

A name ending in _gesvd repeats its workload with LAPACK's QR-iteration SVD
(gesvd) in place of divide and conquer (gesdd): a second correct FP64 run of
the same algorithm whose rounding differs, which measures how far two such
runs drift apart over a long truncated evolution.

SYN_L64_chi2048_4gates imports the synthetic chi=2048 state
(circuits.synthetic_state(64, 32, 4, 2048, seed=30)) through the oracle's
Eq. (E2) import and applies the four central gates of the first brickwork
layer of the 64-mode circuit (seed 3), at sites 28, 30, 32 and 34; it stores
each gate's kept count, discarded weight and cut margin, every bond's
charges, the Schmidt values of the touched bonds per charge, and 1024
amplitudes drawn along charge paths present in the input state (seed 107).

Usage:  python tests/golden/make_golden.py L32_N16_d4_chi512
        python tests/golden/make_golden.py L64_N32_d4_chi256
        python tests/golden/make_golden.py XXZ_L64_chi256_T10
        python tests/golden/make_golden.py BH_L64_d4_chi256_T3
        python tests/golden/make_golden.py ISING_L64_chi256_T10
        python tests/golden/make_golden.py ISING_L64_chi256_T10_gesvd
        python tests/golden/make_golden.py BH_L64_d4_chi256_T3_gesvd
        python tests/golden/make_golden.py BH_L64_d4_chi256_T3_L53
        python tests/golden/make_golden.py SYN_L64_chi2048_4gates
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import dense_mps  # noqa: E402
from workloads import circuits, hamiltonians  # noqa: E402

WORKLOADS = {
    "L32_N16_d4_chi512": (lambda: circuits.config_plain_gpu(), 102),
    # the precision-form circuit (64 modes, 32 photons in even modes, 64 layers)
    # at a bond cap the oracle finishes in minutes
    "L64_N32_d4_chi256": (lambda: circuits.config_precision(seed=3, chi_max=256), 103),
    # Hamiltonian time evolution (dense Trotter gates), the measured quenches
    "XXZ_L64_chi256_T10": (hamiltonians.config_xxz_quench, 104),
    "BH_L64_d4_chi256_T3": (hamiltonians.config_bose_hubbard_quench, 105),
    # the Z_2 (transverse-field Ising) quench: charge = occupation count mod 2
    "ISING_L64_chi256_T10": (hamiltonians.config_ising_quench, 106),
}


# prefixes: (workload, layers) -- the part of an evolution that FP64 determines
# (the disordered Bose-Hubbard quench's first stored cut margin below 1e-11 of
# s_0 is at gate 1686, in layer 53; its first 53 layers hold 1670 gates)
PREFIXES = {
    "BH_L64_d4_chi256_T3_L53": ("BH_L64_d4_chi256_T3", 53),
}


SYNTHETIC = {
    # name: (L, N, d, chi, state seed, circuit seed, gate sites, chi_max, cutoff, pattern seed)
    "SYN_L64_chi2048_4gates": (64, 32, 4, 2048, 30, 3, (28, 30, 32, 34), 2048, 1e-12, 107),
}


def lambda_by_charge(m, bond: int) -> dict:
    """Schmidt values of a bond grouped by the charge the audit gives each
    Schmidt vector (the diagonal of Q in the kept basis), descending."""
    q = m.q[bond]
    off = q - np.diag(np.diag(q))
    assert np.max(np.abs(off)) <= 1e-6, "audit matrix not diagonal in the kept basis"
    out: dict = {}
    for lam, qi in zip(m.lam[bond], np.diag(q).real):
        c = m.N - int(round(float(qi)))
        out.setdefault(str(c), []).append(float(lam))
    return {c: sorted(v, reverse=True) for c, v in sorted(out.items(), key=lambda kv: int(kv[0]))}


def main_synthetic(name: str) -> None:
    L, N, d, chi, sseed, cseed, sites, chi_max, cutoff, pseed = SYNTHETIC[name]
    charges, gammas, lambdas = circuits.synthetic_state(L, N, d, chi, seed=sseed)
    pats = circuits.charge_path_patterns(charges, d, 1024, pseed)
    m = dense_mps.DenseMPS.from_vidal(d, N, charges, gammas, lambdas, chi_max=chi_max, cutoff=cutoff)
    del gammas
    layer = {g.site: g for g in circuits.brickwork_layers(L, 1, cseed)[0]}
    t0 = time.time()
    for s in sites:
        rec = m.apply_gate(s, layer[s].u)
        print(f"gate at site {s}: kept {rec.kept}, discarded {rec.discarded:.3e}, "
              f"margin {rec.margin:.3e}, {time.time() - t0:.0f} s", flush=True)
    amp = m.amplitudes(pats)
    out = {
        "workload": name,
        "generator": "tests/golden/make_golden.py (oracle/dense_mps.py only)",
        "L": L, "d": d, "N": N, "chi": chi, "state_seed": sseed, "circuit_seed": cseed,
        "sites": list(sites), "chi_max": chi_max, "cutoff": cutoff, "pattern_seed": pseed,
        "patterns": pats.tolist(),
        "amp_re": amp.real.tolist(), "amp_im": amp.imag.tolist(),
        "kept": [r.kept for r in m.records],
        "discarded": [r.discarded for r in m.records],
        "margin": [r.margin if np.isfinite(r.margin) else None for r in m.records],
        "bond_charges": [{str(k): v for k, v in m.bond_charges(b).items()} for b in range(L + 1)],
        "audit_clean": [m.audit_clean(b) for b in range(L + 1)],
        "lambda_by_charge": {str(s + 1): lambda_by_charge(m, s + 1) for s in sites},
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


def main(name: str) -> None:
    if name in SYNTHETIC:
        main_synthetic(name)
        return
    driver = "gesdd"
    if name.endswith("_gesvd"):
        driver = "gesvd"
    base = name[:-len("_gesvd")] if driver == "gesvd" else name
    nlayers = None
    if base in PREFIXES:
        base, nlayers = PREFIXES[base]
    make, pattern_seed = WORKLOADS[base]
    cfg = make()
    if nlayers is not None:
        cfg["layers"] = cfg["layers"][:nlayers]
        cfg["gates"] = [g for lay in cfg["layers"] for g in lay]
    L, d = cfg["L"], cfg["d"]
    N = sum(cfg["occupation"])
    mod = cfg.get("modulus", 0)
    m = dense_mps.DenseMPS(cfg["occupation"], d, chi_max=cfg["chi_max"], cutoff=cfg["cutoff"], modulus=mod,
                           svd_driver=driver)
    t0 = time.time()
    for li, lay in enumerate(cfg["layers"]):
        m.run(lay)
        print(f"layer {li + 1}/{len(cfg['layers'])} chi {max(m.bond_dims())} "
              f"{time.time() - t0:.0f} s", flush=True)
    if mod:
        pats = hamiltonians.zn_patterns(L, d, N, 1024, pattern_seed)
    else:
        pats = circuits.sample_patterns(L, N, d, 1024, pattern_seed)
    pats = np.vstack([pats, np.array(cfg["occupation"], dtype=np.int32)[None, :]])
    amp = m.amplitudes(pats)
    out = {
        "workload": name,
        "generator": "tests/golden/make_golden.py (oracle/dense_mps.py only)",
        "svd_driver": driver,
        "L": L, "d": d, "N": N, "modulus": mod, "chi_max": cfg["chi_max"], "cutoff": cfg["cutoff"],
        "patterns": pats.tolist(),
        "amp_re": amp.real.tolist(), "amp_im": amp.imag.tolist(),
        "norm2": m.norm2(),
        "bond_charges": [{str(k): v for k, v in m.bond_charges(b).items()} for b in range(L + 1)],
        "audit_clean": [m.audit_clean(b) for b in range(L + 1)],
        "discarded": [r.discarded for r in m.records],
        "margin": [r.margin if np.isfinite(r.margin) else None for r in m.records],
        "lambda_center": {str(b): m.lam[b].tolist() for b in (L // 2 - 1, L // 2, L // 2 + 1)},
        "layers": len(cfg["layers"]),
        "lambda_all": ({str(b): m.lam[b].tolist() for b in range(L + 1)} if nlayers is not None else None),
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "L32_N16_d4_chi512")
