"""Interpolated step-6' probabilities across energies (Sec. V A, "Interpolation"): oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Never called by the HIP library.

The paper computes the step-6' probabilities p_i (Eqs. (75), (76)) at some energies and,
where the probabilities at two nearby energies differ by less than five percent, takes those
at every energy between the two by linear interpolation.  Readings taken here (each one is
listed in the design notes):
  * the difference of two energies is measured row by row, as the L1 distance
    sum_i |p(i|j; E_a) - p(i|j; E_b)| of the two normalised rows of every state j (probes and
    injection rows); an interval [E_a, E_b] between neighbouring nodes may be interpolated
    when the largest of these distances is at most 0.05;
  * an energy inside an interval that may not be interpolated is computed exactly, i.e. it
    becomes a node itself;
  * between nodes E_a < E_b, alpha = (E - E_a) / (E_b - E_a) and every row is
    (1 - alpha) p_a + alpha p_b; the row total c_p = Tr Gamma_p A that scales the estimator
    (Eq. (66)) is interpolated the same way.
A draw from the interpolated row is a draw from a mixture: take the row of E_b with
probability alpha, else the row of E_a, and draw from it.
"""
from __future__ import annotations

import numpy as np

from oracle import dense as D

TOL = 0.05
TWO32 = 4294967296.0


def bracket(nodes, E):
    """(lo, alpha): the interval [nodes[lo], nodes[lo + 1]] holding E and the position of E in
    it; (len - 1, 0) at the last node.  nodes must ascend; E outside them is an error."""
    nodes = np.asarray(nodes, dtype=np.float64)
    if np.any(np.diff(nodes) <= 0.0):
        raise ValueError("nodes must be strictly ascending")
    if not (nodes[0] <= E <= nodes[-1]):
        raise ValueError("energy outside the nodes")
    if E == nodes[-1]:
        return len(nodes) - 1, 0.0
    lo = int(np.searchsorted(nodes, E, side="right")) - 1
    return lo, (E - nodes[lo]) / (nodes[lo + 1] - nodes[lo])


def alpha_fixed32(alpha: float) -> int:
    """The mixture weight as a 32-bit threshold: the row of the upper node is taken when a
    uniform 32-bit word is below it."""
    return min(int(alpha * TWO32), 0xFFFFFFFF)


def normalised_rows(K):
    K = np.asarray(K, dtype=np.float64)
    return K / K.sum(axis=1, keepdims=True)


def row_distances(Ka, Kb):
    """L1 distance between the normalised rows of two kernels, one value per state."""
    return np.abs(normalised_rows(Ka) - normalised_rows(Kb)).sum(axis=1)


def refine(node_E, node_K, fine_E, tol=TOL):
    """The fine energies that must be computed exactly: those strictly inside an interval of
    neighbouring nodes whose rows differ by more than tol (largest row distance)."""
    d = [float(row_distances(node_K[i], node_K[i + 1]).max()) for i in range(len(node_E) - 1)]
    out = []
    for E in fine_E:
        lo, a = bracket(node_E, E)
        if a > 0.0 and d[lo] > tol:
            out.append(E)
    return out, d


def interpolated_kernel_rows(Ka, Kb, alpha):
    """(1 - alpha) p_a + alpha p_b, row by row, and the interpolated row totals."""
    P = (1.0 - alpha) * normalised_rows(Ka) + alpha * normalised_rows(Kb)
    c = (1.0 - alpha) * Ka.sum(axis=1) + alpha * Kb.sum(axis=1)
    return P, c


def interpolated_transmission(Ka, Kb, alpha, inject_lead=0):
    """Exact expectation of the interpolated walk's estimator: c_p times the probability that
    a walker injected at lead p is absorbed at the other lead, for the Markov chain of the
    interpolated rows."""
    P, c = interpolated_kernel_rows(Ka, Kb, alpha)
    n = P.shape[0]
    h_R = D.absorption_probabilities(P)  # rows already sum to one
    row = n - 2 + inject_lead
    p_exit = h_R[row] if inject_lead == 0 else 1.0 - h_R[row]
    return float(c[row] * p_exit)
