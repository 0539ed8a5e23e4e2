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

Usage:  python tests/golden/make_golden.py L32_N16_d4_chi512
        python tests/golden/make_golden.py L64_N32_d4_chi256
        python tests/golden/make_golden.py XXZ_L64_chi256_T10
        python tests/golden/make_golden.py BH_L64_d4_chi256_T3
        python tests/golden/make_golden.py ISING_L64_chi256_T10
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


def main(name: str) -> None:
    make, pattern_seed = WORKLOADS[name]
    cfg = make()
    L, d = cfg["L"], cfg["d"]
    N = sum(cfg["occupation"])
    mod = cfg.get("modulus", 0)
    m = dense_mps.DenseMPS(cfg["occupation"], d, chi_max=cfg["chi_max"], cutoff=cfg["cutoff"], modulus=mod)
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
        "L": L, "d": d, "N": N, "modulus": mod, "chi_max": cfg["chi_max"], "cutoff": cfg["cutoff"],
        "patterns": pats.tolist(),
        "amp_re": amp.real.tolist(), "amp_im": amp.imag.tolist(),
        "norm2": m.norm2(),
        "bond_charges": [{str(k): v for k, v in m.bond_charges(b).items()} for b in range(L + 1)],
        "audit_clean": [m.audit_clean(b) for b in range(L + 1)],
        "discarded": [r.discarded for r in m.records],
        "margin": [r.margin if np.isfinite(r.margin) else None for r in m.records],
        "lambda_center": {str(b): m.lam[b].tolist() for b in (L // 2 - 1, L // 2, L // 2 + 1)},
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "L32_N16_d4_chi512")
