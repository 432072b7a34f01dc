"""Orbital ordering by a Fiedler reduction of the band width (H2O section: the molecular
orbitals of the MPS runs are ordered this way before the MPO is built).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Reading (the paper names the method and its source, no formula): the orbitals are the
vertices of a weighted graph with edge weights w_ij = |h_ij| + |(ij|ji)| (i != j), the
magnitudes of the one-body hopping and of the exchange integral between the two orbitals;
the Fiedler vector is the eigenvector of the second smallest eigenvalue of the graph
Laplacian Lap = diag(sum_j w_ij) - w, and the new order sorts the orbitals by its
components (ascending; ties by orbital index).  The vector's overall sign is fixed so that
its first component does not exceed its last.  perm[k] is the old orbital at position k.
"""
from __future__ import annotations

import numpy as np


def coupling(h, eri=None):
    """w_ij = |h_ij| + |(ij|ji)| off the diagonal, 0 on it."""
    w = np.abs(np.asarray(h, dtype=np.float64)).copy()
    if eri is not None:
        w = w + np.abs(np.einsum("ijji->ij", np.asarray(eri, dtype=np.float64)))
    np.fill_diagonal(w, 0.0)
    return w


def laplacian(w):
    return np.diag(w.sum(axis=1)) - w


def fiedler_vector(w):
    """(lambda_2, v_2) of the Laplacian of w, by a dense symmetric eigensolver."""
    lam, V = np.linalg.eigh(laplacian(w))
    return lam[1], V[:, 1]


def fiedler_order(h, eri=None):
    """Permutation (new position -> old orbital)."""
    L = np.asarray(h).shape[0]
    if L <= 2:
        return np.arange(L)
    _, v = fiedler_vector(coupling(h, eri))
    if v[0] > v[-1]:
        v = -v
    return np.argsort(v, kind="stable")


def permute(h, eri, perm):
    """Integrals relabelled to the new order: h'_kl = h_{perm k, perm l}, likewise all four
    indices of (pq|rs)."""
    p = np.asarray(perm)
    return h[np.ix_(p, p)], eri[np.ix_(p, p, p, p)]


def bandwidth(w, tol=0.0):
    """max |i - j| over entries with |w_ij| > tol."""
    i, j = np.nonzero(np.abs(w) > tol)
    return int(np.max(np.abs(i - j))) if len(i) else 0


def weighted_spread(w):
    """sum_ij |w_ij| (i - j)^2: the quadratic band-width measure the ordering relaxes."""
    idx = np.arange(w.shape[0])
    return float(np.sum(np.abs(w) * (idx[:, None] - idx[None, :]) ** 2))
