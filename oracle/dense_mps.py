"""Dense (no-symmetry) matrix-product-state TEBD in complex128.

Test infrastructure (see the package header).  This is the oracle for the
GPU path: it runs the same algorithm -- the two-site update by SVD of the
paper's Sec. II -- without using the U(1) structure anywhere.

Representation (Sec. II, Eq. (E1)): sites s = 0..L-1 (the paper's 1..M),
bonds b = 0..L with bond b between site b-1 and site b; bonds 0 and L have
dimension 1.  Two storage forms, identical in exact arithmetic:

* ``vidal``:    Gamma[s] of shape (chi_s, d, chi_{s+1}) and lambda[b], the
                amplitude being Gamma[0] lambda[1] Gamma[1] ... Gamma[L-1].
* ``hastings``: B[s] = Gamma[s] lambda[s+1] (column-scaled), so the
                amplitude is the plain product B[0] B[1] ... B[L-1] and the
                update needs no division by lambda.  This is the default and
                the form the GPU path stores.

Two-site update on sites (s, s+1) (TEBD; the paper's "local updates"):

1. theta~ = B[s] B[s+1] contracted over bond s+1, shape (chi_s, d, d, chi_{s+2});
2. apply the projected two-mode gate P_d G P_d on the two physical indices;
3. theta = lambda[s] * theta~ (row scaling), reshaped (chi_s d) x (d chi_{s+2});
4. full SVD theta = U S V^dagger (LAPACK);
5. keep K singular values by the cut rule of ``truncation``;
6. B[s+1] = V^dagger[:K], lambda[s+1] = S[:K], B[s] = theta~ V[:, :K]
   (= lambda[s]^-1 U S in exact arithmetic); no renormalisation.

Charge audit (bookkeeping reference, independent of the block structure):
for every bond the oracle keeps Q[b], the matrix of the photon number of
sites < b in the left Schmidt basis of bond b.  A gate on bond s+1 updates
Q[s+1] = U_K^dagger (Q[s] (x) 1 + 1 (x) diag(0..d-1)) U_K.  Its eigenvalues
are integers when the kept subspace is closed under the charge; the bond's
right-charge labels of Eq. (E3) are N minus those eigenvalues.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.linalg

from . import twomode


@dataclass
class CutResult:
    kept: int
    discarded: float        # sum of squared dropped singular values
    total: float            # sum of all squared singular values
    margin: float           # (s[K-1] - s[K]) / s[0]; inf when nothing dropped


def truncation(s: np.ndarray, chi_max: int, cutoff: float, zero_tol: float) -> CutResult:
    """Global cut over one two-site matrix's singular values (sorted descending).

    K = min(chi_max, K_eps, K_zero) where
      K_eps  = smallest K with sum_{i>=K} s_i^2 <= cutoff * sum_i s_i^2,
      K_zero = number of s_i > zero_tol * s_0  (numerically-zero values dropped),
    chi_max <= 0 meaning no cap.  K is at least 1.  The discarded weight is
    sum_{i>=K} s_i^2.  Sec. II names chi as the maximum bond dimension; the
    weight criterion and the zero floor are readings (the paper is silent).
    """
    s = np.asarray(s, dtype=np.float64)
    n = s.size
    if n == 0 or not (s[0] > 0.0) or not np.all(np.isfinite(s)):
        raise FloatingPointError("two-site matrix vanished or is not finite")
    sq = s * s
    tail = np.zeros(n + 1)
    tail[:n] = np.cumsum(sq[::-1])[::-1]
    total = float(tail[0])
    k_eps = int(np.argmax(tail <= cutoff * total))   # first index meeting the bound
    k_zero = int(np.sum(s > zero_tol * s[0]))
    k = min(k_eps, k_zero)
    if chi_max and chi_max > 0:
        k = min(k, chi_max)
    k = max(k, 1)
    margin = float((s[k - 1] - s[k]) / s[0]) if k < n else math.inf
    return CutResult(kept=k, discarded=float(tail[k]), total=total, margin=margin)


def _svd(m: np.ndarray, driver: str = "gesdd"):
    """LAPACK SVD.  gesdd (divide and conquer) by default, falling back to
    gesvd (QR iteration) if it fails; driver="gesvd" takes QR iteration
    throughout -- a second, independently rounded FP64 SVD of the same matrix."""
    if driver == "gesvd":
        return scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesvd")
    try:
        return scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:
        return scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesvd")


@dataclass
class GateRecord:
    site: int
    kept: int
    discarded: float
    margin: float
    leak: float             # norm of theta lost to the local cutoff (P_d)
    audit_ok: bool


class DenseMPS:
    """Dense MPS of L modes with local dimension d, started in a Fock product state."""

    def __init__(self, occupation: Sequence[int], d: int, chi_max: int = 0,
                 cutoff: float = 0.0, zero_tol: float = 1e-13, form: str = "hastings",
                 modulus: int = 0, charge_map=None, svd_driver: str = "gesdd"):
        occ = [int(x) for x in occupation]
        if any(o < 0 or o >= d for o in occ):
            raise ValueError("occupation outside 0..d-1")
        if form not in ("hastings", "vidal"):
            raise ValueError(form)
        if svd_driver not in ("gesdd", "gesvd"):
            raise ValueError(svd_driver)
        self.svd_driver = svd_driver
        self.L, self.d, self.N = len(occ), d, sum(occ)
        # modulus 0: the charge is the particle number (U(1)); n >= 2: the
        # particle number mod n (Z_n), audited through the unitary omega^Q
        self.modulus = int(modulus)
        # charge_map (d x K integers): K independent U(1) charges, local state p
        # carrying charge_map[p]; each component is audited by its own operator
        self.cmap = None if charge_map is None else np.asarray(charge_map, dtype=np.int64).reshape(d, -1)
        self.chi_max, self.cutoff, self.zero_tol, self.form = chi_max, cutoff, zero_tol, form
        self.t: List[np.ndarray] = []          # B (hastings) or Gamma (vidal)
        for o in occ:
            a = np.zeros((1, d, 1), dtype=np.complex128)
            a[0, o, 0] = 1.0
            self.t.append(a)
        self.lam: List[np.ndarray] = [np.ones(1) for _ in range(self.L + 1)]
        left = np.concatenate([[0], np.cumsum(occ)])
        if self.cmap is not None:
            K = self.cmap.shape[1]
            lk = np.concatenate([np.zeros((1, K), dtype=np.int64), np.cumsum(self.cmap[occ], axis=0)])
            self.total = tuple(int(x) for x in lk[-1])
            self.qk = [[np.array([[float(lk[b, k])]], dtype=np.complex128) for b in range(self.L + 1)]
                       for k in range(K)]
            self.q = self.qk[0]
        elif self.modulus:
            w = np.exp(2j * np.pi / self.modulus)
            self.q: List[np.ndarray] = [np.array([[w ** int(left[b])]], dtype=np.complex128)
                                        for b in range(self.L + 1)]
        else:
            self.q = [np.array([[float(left[b])]], dtype=np.complex128) for b in range(self.L + 1)]
        self.records: List[GateRecord] = []

    @classmethod
    def from_vidal(cls, d: int, n_photons: int, bond_charges: Sequence[Sequence[int]],
                   gammas: Sequence[np.ndarray], lambdas: Sequence[np.ndarray], chi_max: int = 0,
                   cutoff: float = 0.0, zero_tol: float = 1e-13, form: str = "hastings",
                   svd_driver: str = "gesdd") -> "DenseMPS":
        """A U(1) state given in the charge-labelled Vidal form of Eq. (E2):
        bond b's indices carry right-charges bond_charges[b] (Eq. (E3); bond 0
        is {N}, bond L is {0}, Eq. (E4)), gammas[s] is the chi_s x chi_{s+1}
        matrix Gamma[s] with no physical index, and lambdas[b] the bond's
        values.  The Kronecker delta of (E2) puts entry (a, b) of gammas[s] on
        physical index i = c_s(a) - c_{s+1}(b); an entry with i outside
        0..d-1 must be zero (ValueError otherwise).  The dense tensor is
        Gamma[s][a, i, b] = delta(i, c_s(a) - c_{s+1}(b)) gammas[s][a, b],
        stored as B = Gamma lambda[s+1] in the Hastings form.  The charge audit
        starts from the given labels: Q[b] = diag(N - c_b), the photons left of
        the bond."""
        L = len(gammas)
        if len(bond_charges) != L + 1 or len(lambdas) != L + 1:
            raise ValueError("need L+1 bonds of charges and of lambdas")
        ch = [np.asarray(c, dtype=np.int64).reshape(-1) for c in bond_charges]
        if ch[0].tolist() != [n_photons] or ch[L].tolist() != [0]:
            raise ValueError("bond 0 must carry {N} and bond L {0} (Eq. (E4))")
        obj = cls([0] * L, d, chi_max=chi_max, cutoff=cutoff, zero_tol=zero_tol, form=form,
                  svd_driver=svd_driver)
        obj.N = int(n_photons)
        obj.lam = [np.asarray(l, dtype=np.float64).reshape(-1).copy() for l in lambdas]
        obj.t = []
        for s in range(L):
            g = np.asarray(gammas[s], dtype=np.complex128)
            if g.shape != (ch[s].size, ch[s + 1].size) or obj.lam[s + 1].size != ch[s + 1].size:
                raise ValueError(f"site {s}: shapes do not match the bond dimensions")
            phys = ch[s][:, None] - ch[s + 1][None, :]
            if np.any(g[(phys < 0) | (phys >= d)] != 0):
                raise ValueError(f"site {s}: an entry violates the charge rule of Eq. (E2)")
            gam = np.zeros((ch[s].size, d, ch[s + 1].size), dtype=np.complex128)
            for i in range(d):
                gam[:, i, :] = np.where(phys == i, g, 0.0)
            obj.t.append(gam * obj.lam[s + 1][None, None, :] if form == "hastings" else gam)
        obj.q = [np.diag((obj.N - c).astype(np.complex128)) for c in ch]
        return obj

    # ------------------------------------------------------------------ update
    def apply_gate(self, site: int, u: np.ndarray) -> GateRecord:
        """Two-mode linear-optics gate of 2x2 mode unitary u (P_d G P_d)."""
        return self.apply_dense(site, twomode.dense(np.asarray(u, dtype=np.complex128), self.d))

    def apply_dense(self, site: int, g: np.ndarray) -> GateRecord:
        """Any two-site gate as a d^2 x d^2 matrix, row p*d+q, column m*d+n
        (a TEBD step of a Hamiltonian; the charge is not assumed here)."""
        s, d = site, self.d
        if not 0 <= s < self.L - 1:
            raise IndexError("gate site out of range")
        a, b = self.t[s], self.t[s + 1]
        chl, chr_ = a.shape[0], b.shape[2]
        # theta~[x, i, j, z] = sum_y a[x, i, y] b[y, j, z] (a matrix product over
        # the middle bond; in the Vidal form with lambda on the middle and right bonds)
        if self.form == "hastings":
            th = np.tensordot(a, b, axes=([2], [0]))
        else:
            th = np.tensordot(a * self.lam[s + 1][None, None, :], b * self.lam[s + 2][None, None, :],
                              axes=([2], [0]))
        lam_l = self.lam[s]
        g4 = np.asarray(g, dtype=np.complex128).reshape(d, d, d, d)
        before = float(np.sum(np.abs(lam_l[:, None, None, None] * th) ** 2))
        # the gate on the two physical indices: th'[x, p, q, z] = sum_mn g4[p, q, m, n] th[x, m, n, z]
        th = np.ascontiguousarray(np.tensordot(g4, th, axes=([2, 3], [1, 2])).transpose(2, 0, 1, 3))
        theta = lam_l[:, None, None, None] * th
        after = float(np.sum(np.abs(theta) ** 2))
        mat = theta.reshape(chl * d, d * chr_)
        uu, sv, vh = _svd(mat, self.svd_driver)
        cut = truncation(sv, self.chi_max, self.cutoff, self.zero_tol)
        k = cut.kept
        vk = vh[:k]
        if self.form == "hastings":
            self.t[s + 1] = vk.reshape(k, d, chr_)
            self.t[s] = (th.reshape(chl * d, d * chr_) @ vk.conj().T).reshape(chl, d, k)
        else:
            self.t[s] = (uu[:, :k] / np.repeat(self.lam[s], d)[:, None]).reshape(chl, d, k)
            self.t[s + 1] = (vk.reshape(k, d, chr_) / self.lam[s + 2][None, None, :])
        self.lam[s + 1] = sv[:k].copy()
        # charge audit of the new bond s+1
        uk = uu[:, :k]
        if self.cmap is not None:
            for comp, qb in enumerate(self.qk):
                row = np.kron(qb[s], np.eye(d)) + np.kron(np.eye(chl), np.diag(self.cmap[:, comp].astype(float)))
                qb[s + 1] = uk.conj().T @ row @ uk
            qrow = None
        elif self.modulus:
            w = np.exp(2j * np.pi / self.modulus)
            qrow = np.kron(self.q[s], np.diag(w ** np.arange(d)))
        else:
            qrow = np.kron(self.q[s], np.eye(d)) + np.kron(np.eye(chl), np.diag(np.arange(d)))
        if qrow is not None:
            self.q[s + 1] = uk.conj().T @ qrow @ uk
        ok = self.audit_clean(s + 1)
        rec = GateRecord(site=s, kept=k, discarded=cut.discarded, margin=cut.margin,
                         leak=before - after, audit_ok=ok)
        self.records.append(rec)
        return rec

    def run(self, gates) -> "DenseMPS":
        """Gates with .u (mode unitary) or .g4 (dense two-site matrix)."""
        for g in gates:
            if hasattr(g, "g4"):
                self.apply_dense(g.site, g.g4)
            else:
                self.apply_gate(g.site, g.u)
        return self

    # ------------------------------------------------------------- read-outs
    def site_matrices(self) -> List[np.ndarray]:
        """The Hastings tensors B[s] (shape chi_s x d x chi_{s+1}) in either form."""
        if self.form == "hastings":
            return self.t
        return [self.t[s] * self.lam[s + 1][None, None, :] for s in range(self.L)]

    def amplitude(self, occ: Sequence[int]) -> complex:
        """c_{i_1..i_L} by contracting the chain, Eq. (E1).  Occupations >= d are
        outside the local space and give 0; a wrong photon number is still
        contracted (it is zero only up to rounding in this dense form)."""
        occ = [int(x) for x in occ]
        if any(o < 0 or o >= self.d for o in occ):
            return 0.0 + 0.0j
        bs = self.site_matrices()
        v = np.ones((1,), dtype=np.complex128)
        for s, o in enumerate(occ):
            v = v @ bs[s][:, o, :]
        return complex(v[0])

    def amplitudes(self, patterns: np.ndarray) -> np.ndarray:
        """(E1) for many patterns; patterns go through in groups small enough
        that the gathered blocks stay near 256 MiB."""
        pats = np.asarray(patterns, dtype=np.int64)
        bs = self.site_matrices()
        out = np.zeros(pats.shape[0], dtype=np.complex128)
        valid = np.all((pats >= 0) & (pats < self.d), axis=1)
        idx = np.nonzero(valid)[0]
        chi = max(self.bond_dims())
        group = max(1, int((1 << 28) // (16 * chi * chi)))
        for g0 in range(0, idx.size, group):
            sel = idx[g0:g0 + group]
            v = np.ones((sel.size, 1), dtype=np.complex128)
            for s in range(self.L):
                blk = bs[s][:, pats[sel, s], :]          # (chi_s, n, chi_{s+1})
                v = np.einsum("nx,xny->ny", v, blk)
            out[sel] = v[:, 0]
        return out

    def norm2(self) -> float:
        """<psi|psi> by full contraction of the transfer matrices."""
        e = np.ones((1, 1), dtype=np.complex128)
        for bt in self.site_matrices():
            # E'[c, d] = sum_i sum_ab conj(B[a, i, c]) E[a, b] B[b, i, d]
            e = sum(bt[:, i, :].conj().T @ (e @ bt[:, i, :]) for i in range(bt.shape[1]))
        return float(e[0, 0].real)

    def bond_dims(self) -> List[int]:
        return [self.lam[b].size for b in range(self.L + 1)]

    def _left_charges(self, bond: int) -> np.ndarray:
        """Left charges of the Schmidt vectors of a bond as real numbers (integers
        when the audit is clean): eigenvalues of the left particle number, or
        for Z_n the phases of omega^Q times n / (2 pi), taken in [0, n)."""
        if self.modulus:
            ev = np.linalg.eigvals(self.q[bond])
            return np.mod(np.angle(ev) * self.modulus / (2 * np.pi), self.modulus)
        return np.linalg.eigvalsh(self.q[bond])

    def _joint_left_charges(self, bond: int) -> np.ndarray:
        """K components' left charges of a bond's Schmidt vectors (rows): the
        commuting operators are diagonalised together through a generic
        combination, and each one's value read off on the common eigenvectors."""
        ops = [qb[bond] for qb in self.qk]
        weights = [1.0, 0.6180339887498949, 0.41421356237309515, 0.7320508075688772][:len(ops)]
        _, v = np.linalg.eigh(sum(w * o for w, o in zip(weights, ops)))
        return np.stack([np.real(np.einsum("ij,ik,kj->j", v.conj(), o, v)) for o in ops], axis=1)

    def bond_charges(self, bond: int) -> Dict:
        """Right-charge histogram of a bond from the charge audit (Eq. (E3));
        for Z_n the right charge is taken mod n; with a charge map the keys
        are tuples of the K components."""
        if self.cmap is not None:
            hist_t: Dict = {}
            for row in self._joint_left_charges(bond):
                c = tuple(t - int(round(float(x))) for t, x in zip(self.total, row))
                hist_t[c] = hist_t.get(c, 0) + 1
            return dict(sorted(hist_t.items()))
        hist: Dict[int, int] = {}
        for e in self._left_charges(bond):
            c = self.N - int(round(float(e)))
            if self.modulus:
                c %= self.modulus
            hist[c] = hist.get(c, 0) + 1
        return dict(sorted(hist.items()))

    def audit_clean(self, bond: int, tol: float = 1e-6) -> bool:
        if self.cmap is not None:
            ev = self._joint_left_charges(bond)
            return bool(np.all(np.abs(ev - np.round(ev)) <= tol))
        ev = self._left_charges(bond)
        dev = np.abs(ev - np.round(ev))
        if self.modulus:
            dev = np.minimum(dev, np.abs(ev - self.modulus))
        return bool(np.all(dev <= tol))
