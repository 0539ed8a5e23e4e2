"""Exact sampling of output patterns -- TEST INFRASTRUCTURE ONLY.

The paper names boson-sampling circuits as a U(1) workload (Sec. I); their
output is a random occupation pattern i_1..i_L drawn with probability
P(i) = |c_i|^2 / sum_j |c_j|^2, c_i the amplitudes of Eq. (E2).  The paper
gives no sampling procedure; this module and the GPU path both use the chain
rule (perfect sampling from an MPS, as in Ferris and Vidal 2012), taking the
modes from the last to the first:

    P(i_k | i_{k+1..L}) = P(i_k, i_{k+1..L}) / P(i_{k+1..L}),

and the occupation of mode k is the smallest i whose cumulative conditional
probability exceeds u_k, with u_k a caller-supplied uniform variate in [0, 1)
(u[j, k] for sample j).  Two independent implementations:

* ``brute_force_samples``: the plain definition over a table of every
  pattern's probability (marginals by summation); small L only.
* ``mps_samples``: the dense oracle MPS with left environments
  E_k = sum over i_1..i_k of (B^{i_1}..B^{i_k})^dagger (B^{i_1}..B^{i_k})
  (a chi_k x chi_k matrix, no symmetry used); the unnormalised marginal of a
  suffix whose contraction from the right is the vector v is v^dagger E_k v.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np


def _pick(p: np.ndarray, u: float) -> int:
    """Smallest i with u * sum(p) < p[0] + ... + p[i] (last positive if none)."""
    tot = float(np.sum(p))
    acc = 0.0
    for i, x in enumerate(p):
        acc += float(x)
        if u * tot < acc:
            return i
    return int(np.flatnonzero(p > 0)[-1])


def brute_force_samples(table: Dict[Tuple[int, ...], float], L: int, d: int,
                        uniforms: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Chain-rule samples from a table pattern -> unnormalised probability.
    Returns (patterns [count, L], normalised probabilities [count])."""
    total = sum(table.values())
    u = np.asarray(uniforms, dtype=np.float64)
    out = np.zeros((u.shape[0], L), dtype=np.int32)
    prob = np.zeros(u.shape[0])
    for j in range(u.shape[0]):
        suffix: List[int] = []
        for k in range(L - 1, -1, -1):
            p = np.zeros(d)
            for pat, w in table.items():
                if list(pat[k + 1:]) == suffix:
                    p[pat[k]] += w
            i = _pick(p, u[j, k])
            suffix = [i] + suffix
        out[j] = suffix
        prob[j] = table[tuple(suffix)] / total
    return out, prob


def left_environments(mps) -> List[np.ndarray]:
    """E_0 .. E_L of a dense oracle MPS (Hastings form: amplitude B_0 .. B_{L-1})."""
    if mps.form != "hastings":
        raise ValueError("the environments need the Hastings form")
    E = [np.ones((1, 1), dtype=np.complex128)]
    for s in range(mps.L):
        t = mps.t[s]
        e = np.zeros((t.shape[2], t.shape[2]), dtype=np.complex128)
        for i in range(mps.d):
            bi = t[:, i, :]
            e += bi.conj().T @ E[-1] @ bi
        E.append(e)
    return E


def decision_margin(p: np.ndarray, u: float) -> float:
    """Distance of u * sum(p) from the nearest cumulative boundary, over sum(p)."""
    tot = float(np.sum(p))
    return float(np.min(np.abs(u * tot - np.cumsum(p)))) / tot


def mps_samples(mps, uniforms: np.ndarray, margins: bool = False):
    """Chain-rule samples from the dense oracle MPS, modes L-1 down to 0.
    Returns (patterns [count, L], probabilities |c_i|^2 / <psi|psi> [count])
    and, with margins, each sample's smallest decision margin (a draw whose
    margin is at rounding level may go either way in another precision)."""
    E = left_environments(mps)
    u = np.asarray(uniforms, dtype=np.float64)
    L, d = mps.L, mps.d
    out = np.zeros((u.shape[0], L), dtype=np.int32)
    prob = np.ones(u.shape[0])
    marg = np.full(u.shape[0], np.inf)
    for j in range(u.shape[0]):
        v = np.ones(1, dtype=np.complex128)            # contraction of the chosen suffix
        for k in range(L - 1, -1, -1):
            t = mps.t[k]
            ws = [t[:, i, :] @ v for i in range(d)]
            p = np.array([float(np.real(np.vdot(w, E[k] @ w))) for w in ws])
            p = np.maximum(p, 0.0)
            i = _pick(p, u[j, k])
            marg[j] = min(marg[j], decision_margin(p, u[j, k]))
            prob[j] *= p[i] / float(np.sum(p))
            out[j, k] = i
            v = ws[i] / np.sqrt(p[i])
    if margins:
        return out, prob, marg
    return out, prob
