"""CPU oracle for the U(1)-symmetric MPS gate path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct complex128 reference written
from the paper's statement of the method (Sec. II: the Vidal-form MPS of
Eq. (E1), the right-charge labels and Kronecker deltas of Eqs. (E2)-(E4), and
the two-site update by SVD with a bond-dimension cap chi).  (E1)-(E4) name the
four displayed relations of Sec. II in order: the Vidal-form amplitude, the
U(1) amplitude with Kronecker deltas, the right-charge definition, and the
charge balance with c = N on the left and 0 on the right.  It deliberately
uses NO symmetry: the MPS is dense, the two-site matrix is the full
(chi*d) x (d*chi) matrix and its SVD is LAPACK's.  It shares no code with the
GPU library and imports nothing from it.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it.  The product path never does.

Modules
-------
permanent  -- Ryser and naive permanents; Fock amplitudes of a linear-optics
              unitary (closed form, used as a pin).
twomode    -- Fock-basis matrix elements of a two-mode gate (symmetric power
              of the 2x2 mode unitary), projected to occupations < d.
fock       -- brute-force state vector in the N-photon, occupation<d sector.
dense_mps  -- dense (no-symmetry) MPS TEBD with the same truncation rule as
              the GPU path, amplitudes (E1), full-contraction norm, and an
              independent charge audit of every bond; gates given as mode
              unitaries or as dense two-site matrices (Hamiltonian TEBD); with a
              modulus n the charge is the particle number mod n (Z_n) and the
              audit tracks the unitary omega^Q instead of Q; with a charge map
              (d x K) the state carries K independent U(1) charges, each
              audited by its own operator.
sampling   -- exact chain-rule sampling of output patterns, by brute force
              over a probability table and from the dense MPS's environments.
"""
