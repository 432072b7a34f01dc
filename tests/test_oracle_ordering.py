"""Pins of the oracle's Fiedler orbital ordering (H2O section) against closed forms and
graph facts that do not go through its own formula."""
import itertools

import numpy as np
import scipy.sparse.linalg as spla

import synth
from oracle import fci, mps, ordering


def _chain(L, rng):
    """Tridiagonal hopping with random nonzero weights (a path graph)."""
    h = np.diag(np.linspace(-1.0, 1.0, L))
    t = 0.5 + rng.random(L - 1)
    h[np.arange(L - 1), np.arange(1, L)] = -t
    h[np.arange(1, L), np.arange(L - 1)] = -t
    return h


def test_uniform_path_closed_form():
    """Path Laplacian with unit weights: lambda_2 = 2 (1 - cos(pi/L)), Fiedler vector
    proportional to cos(pi (k + 1/2) / L), strictly monotone."""
    for L in (3, 7, 16):
        w = np.zeros((L, L))
        w[np.arange(L - 1), np.arange(1, L)] = w[np.arange(1, L), np.arange(L - 1)] = 1.0
        lam, v = ordering.fiedler_vector(w)
        assert abs(lam - 2 * (1 - np.cos(np.pi / L))) < 1e-12
        ref = np.cos(np.pi * (np.arange(L) + 0.5) / L)
        ref /= np.linalg.norm(ref)
        assert abs(abs(v @ ref) - 1) < 1e-12


def test_shuffled_chain_is_restored():
    """Any relabelling of a chain comes back to bandwidth 1 (the natural order or its
    reverse): the one ordering of a path graph that is tridiagonal."""
    rng = np.random.default_rng(0)
    for L in (4, 9, 24, 60):
        h = _chain(L, rng)
        P = rng.permutation(L)
        hs = h[np.ix_(P, P)]
        perm = ordering.fiedler_order(hs)
        assert sorted(perm) == list(range(L))
        back = P[perm]
        assert list(back) in (list(range(L)), list(range(L))[::-1])
        assert ordering.bandwidth(hs[np.ix_(perm, perm)] - np.diag(np.diag(hs)), 1e-14) == 1


def test_exchange_term_uses_ijji():
    """Orbitals coupled only through exchange integrals (ij|ji) along a chain, with a uniform
    Coulomb (ii|jj) between all pairs: the chain is found, so the weight reads (ij|ji) and
    not (ii|jj) (which alone is a complete graph with a degenerate Fiedler space)."""
    L = 8
    rng = np.random.default_rng(1)
    P = rng.permutation(L)
    eri = np.zeros((L,) * 4)
    for a in range(L):
        for b in range(L):
            eri[a, a, b, b] = 0.7
    for a in range(L - 1):
        x = 0.2 + 0.1 * rng.random()
        for (i, j) in ((a, a + 1), (a + 1, a)):
            eri[i, j, j, i] = eri[j, i, i, j] = x
    h = np.diag(rng.standard_normal(L))
    hs, es = ordering.permute(h, eri, P)
    back = P[ordering.fiedler_order(hs, es)]
    assert list(back) in (list(range(L)), list(range(L))[::-1])


def test_two_clusters_stay_contiguous():
    """Two strongly coupled groups joined by one weak edge: the Fiedler vector separates
    them (spectral bisection), so each group occupies a contiguous block of the order."""
    rng = np.random.default_rng(2)
    L = 10
    A = set(rng.choice(L, 5, replace=False).tolist())
    h = np.zeros((L, L))
    for i, j in itertools.combinations(range(L), 2):
        if (i in A) == (j in A):
            h[i, j] = h[j, i] = 1.0 + rng.random()
    a, b = min(A), min(set(range(L)) - A)
    h[a, b] = h[b, a] = 1e-3
    perm = ordering.fiedler_order(h)
    side = [int(p in A) for p in perm]
    assert side in ([1] * 5 + [0] * 5, [0] * 5 + [1] * 5)


def test_tiny_band_matrices_reach_brute_force_bandwidth():
    """Shuffled band matrices (band b, weights decaying with distance) of L = 7: the Fiedler
    order reaches the minimum bandwidth over all 5040 orderings."""
    rng = np.random.default_rng(4)
    L = 7
    for b in (1, 2, 3):
        w = np.zeros((L, L))
        for i in range(L):
            for j in range(i + 1, min(L, i + b + 1)):
                w[i, j] = w[j, i] = np.exp(-(j - i)) * (0.8 + 0.4 * rng.random())
        P = rng.permutation(L)
        ws = w[np.ix_(P, P)]
        best = min(ordering.bandwidth(ws[np.ix_(p, p)]) for p in map(list, itertools.permutations(range(L))))
        perm = ordering.fiedler_order(ws)
        assert best == b
        assert ordering.bandwidth(ws[np.ix_(perm, perm)]) == best


def test_permutation_leaves_the_spectrum_unchanged():
    """Relabelling the orbitals is a change of basis: the sector spectrum of the Hamiltonian
    of Eq. (hamil) is the same in either order (a relabelling of only some of the four
    indices would change it)."""
    L = 6
    h, eri, _ = synth.integrals(L, seed=11)
    perm = np.random.default_rng(5).permutation(L)
    hp, ep = ordering.permute(h, eri, perm)
    sp = fci.Space.sector(L, 2, 3)
    e1 = np.linalg.eigvalsh(fci.hamiltonian(sp, h, eri).toarray())
    e2 = np.linalg.eigvalsh(fci.hamiltonian(sp, hp, ep).toarray())
    assert np.max(np.abs(e1 - e2)) < 1e-10
    partial = eri[np.ix_(perm, perm, np.arange(L), np.arange(L))]
    e3 = np.linalg.eigvalsh(fci.hamiltonian(sp, hp, partial).toarray())
    assert np.max(np.abs(e1 - e3)) > 1e-3


def test_fiedler_order_lowers_truncation_weight():
    """The point of the ordering: with local integrals scrambled, the ground state truncated
    to a small bond dimension loses less weight in the Fiedler order than in the scrambled
    one (and the order found is the local one of the generator)."""
    L = 8
    Q = (4, 4)
    h, eri, _ = synth.integrals(L, ell=1.0, seed=21)
    P = np.random.default_rng(6).permutation(L)
    hs, es = ordering.permute(h, eri, P)
    perm = ordering.fiedler_order(hs, es)
    assert list(P[perm]) in (list(range(L)), list(range(L))[::-1])
    space = fci.Space.sector(L, *Q)
    disc = []
    for (a, b) in ((hs, es), ordering.permute(hs, es, perm)):
        H = fci.hamiltonian(space, a, b)
        _, v = spla.eigsh(H, k=1, which="SA", tol=1e-12)
        _, d = mps.from_full(space.embed(v[:, 0]), L, Q, Dmax=12)
        disc.append(d)
    assert disc[1] < 0.01 * disc[0]


def test_laplacian_quadratic_form_and_courant_fischer():
    """The identity sum_ij w_ij (x_i - x_j)^2 = 2 x^T Lap x for any x (with x the positions
    this is the spread the ordering relaxes), Lap 1 = 0, and the variational property of the
    Fiedler value: no unit vector orthogonal to 1 has a smaller Rayleigh quotient, and the
    Fiedler vector is such a vector that attains it."""
    rng = np.random.default_rng(23)
    L = 9
    w = np.abs(rng.standard_normal((L, L)))
    w = w + w.T
    np.fill_diagonal(w, 0.0)
    lap = ordering.laplacian(w)
    idx = np.arange(L, dtype=float)
    assert abs(ordering.weighted_spread(w) - 2 * idx @ lap @ idx) < 1e-10 * ordering.weighted_spread(w)
    for _ in range(5):
        x = rng.standard_normal(L)
        direct = sum(w[i, j] * (x[i] - x[j]) ** 2 for i in range(L) for j in range(L))
        assert abs(direct - 2 * x @ lap @ x) < 1e-10 * direct
    assert np.allclose(lap @ np.ones(L), 0.0, atol=1e-12)
    lam2, v = ordering.fiedler_vector(w)
    assert abs(v.sum()) < 1e-10 and abs(v @ v - 1) < 1e-12
    assert abs(v @ lap @ v - lam2) < 1e-12 * lam2
    for _ in range(200):
        x = rng.standard_normal(L)
        x -= x.mean()
        assert x @ lap @ x / (x @ x) >= lam2 * (1 - 1e-12)
