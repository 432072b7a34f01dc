"""Seeded synthetic inputs shared by the CPU oracle tests, the GPU tests and the benchmark.

This module only *draws* inputs: one-/two-electron integrals, dipole matrices, initial
determinants, bond-sector allocations, determinant bond bases and random complex blocks.
It holds none of the method's arithmetic (no Hamiltonian, no contraction, no SVD), so
that the oracle and the HIP path share nothing but these inputs.

Conventions used by every consumer:
  * L spatial orbitals; the local state of orbital p is n = n_up + 2*n_dn in {0,1,2,3}
    (|0>, |up>, |dn>, |up dn>), stored as uint8 "occupation codes".
  * Charges are (n_up, n_dn) pairs counted over the sites left of a bond.
  * Integrals are real; eri[p,q,r,s] = (pq|rs) in chemists' notation with 8-fold symmetry.

The paper's molecular integrals (PySCF / Molpro runs) are not available, so the
integral generator follows the shapes of the paper's systems: a diagonal ladder of
orbital energies, off-diagonal couplings decaying with orbital distance, and a
Coulomb-like diagonal part of the two-electron integrals.
"""
from __future__ import annotations

import math
from itertools import product

import numpy as np

LOCAL_CHARGE = ((0, 0), (1, 0), (0, 1), (1, 1))  # (n_up, n_dn) of local state 0..3


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def integrals(L: int, ell: float = 2.0, seed: int | None = None):
    """Synthetic real integrals (h, eri, e0) for L orbitals.

    h_pq (p != q) = sym(G)_pq * exp(-|p-q|/ell), G ~ N(0,1); h_pp = linspace(-2, 0, L).
    (pq|rs) = sym8(B) * 0.1*exp(-(|p-q|+|r-s|)/ell - |p+q-r-s|/(2 ell)), B ~ N(0,1),
    plus (pp|qq) += 0.5/(1+|p-q|).  Default seed = L.
    """
    rng = _rng(L if seed is None else seed)
    idx = np.arange(L)
    dist = np.abs(idx[:, None] - idx[None, :])
    G = rng.standard_normal((L, L))
    h = 0.5 * (G + G.T) * np.exp(-dist / ell)
    np.fill_diagonal(h, np.linspace(-2.0, 0.0, L))
    B = rng.standard_normal((L, L, L, L))
    S = (B + B.transpose(1, 0, 2, 3) + B.transpose(0, 1, 3, 2) + B.transpose(1, 0, 3, 2)
         + B.transpose(2, 3, 0, 1) + B.transpose(3, 2, 0, 1) + B.transpose(2, 3, 1, 0)
         + B.transpose(3, 2, 1, 0)) / 8.0
    p, q, r, s = np.meshgrid(idx, idx, idx, idx, indexing="ij")
    decay = 0.1 * np.exp(-(np.abs(p - q) + np.abs(r - s)) / ell - np.abs(p + q - r - s) / (2 * ell))
    eri = S * decay
    for a in range(L):
        for b in range(L):
            eri[a, a, b, b] += 0.5 / (1.0 + abs(a - b))
    return np.ascontiguousarray(h), np.ascontiguousarray(eri), 0.0


def dipole_matrix(L: int, ell: float = 2.0, seed: int | None = None):
    """Random symmetric one-body matrix mu_pq = sym(N(0,1)) * exp(-|p-q|/ell). Default seed L+1."""
    rng = _rng(L + 1 if seed is None else seed)
    idx = np.arange(L)
    dist = np.abs(idx[:, None] - idx[None, :])
    G = rng.standard_normal((L, L))
    return np.ascontiguousarray(0.5 * (G + G.T) * np.exp(-dist / ell))


def ionized_determinant(L: int, N0: int, seed: int | None = None):
    """Occupation codes of a random determinant with ceil(N0/2) up and floor(N0/2) down
    electrons, after removing one random occupied up electron (N = N0-1, 2Sz = -1 for
    even N0).  Default seed L+2."""
    rng = _rng(L + 2 if seed is None else seed)
    n_up, n_dn = (N0 + 1) // 2, N0 // 2
    up = rng.choice(L, size=n_up, replace=False)
    dn = rng.choice(L, size=n_dn, replace=False)
    occ = np.zeros(L, dtype=np.uint8)
    occ[up] |= 1
    occ[dn] |= 2
    hole = up[rng.integers(0, n_up)]
    occ[hole] &= 2
    return occ


def determinant(L: int, n_up: int, n_dn: int, seed: int):
    """Random determinant with given spin populations (occupation codes)."""
    rng = _rng(seed)
    occ = np.zeros(L, dtype=np.uint8)
    occ[rng.choice(L, size=n_up, replace=False)] |= 1
    occ[rng.choice(L, size=n_dn, replace=False)] |= 2
    return occ


def occ_charge(occ):
    occ = np.asarray(occ)
    return int(np.sum(occ & 1)), int(np.sum((occ >> 1) & 1))


def _sector_max(L, i, Nu, Nd, q):
    nu, nd = q
    if nu < 0 or nd < 0 or nu > i or nd > i:
        return 0
    ru, rd = Nu - nu, Nd - nd
    if ru < 0 or rd < 0 or ru > L - i or rd > L - i:
        return 0
    left = math.comb(i, nu) * math.comb(i, nd)
    right = math.comb(L - i, ru) * math.comb(L - i, rd)
    return min(left, right)


def sector_allocation(L: int, Nu: int, Nd: int, D: int, sigma: float = 1.0):
    """Bond-sector dimensions for benchmark states.

    Returns a list of L+1 dicts {(n_up, n_dn): dim}.  Dims are D*w_q/sum(w) rounded and
    clamped to the combinatorial maximum, with
    w_q = exp(-[(n_up - Nu*i/L)^2 + (n_dn - Nd*i/L)^2] / (2 sigma^2)).
    """
    bonds = []
    for i in range(L + 1):
        qs = [(a, b) for a in range(0, i + 1) for b in range(0, i + 1) if _sector_max(L, i, Nu, Nd, (a, b)) > 0]
        w = np.array([math.exp(-((a - Nu * i / L) ** 2 + (b - Nd * i / L) ** 2) / (2 * sigma ** 2)) for a, b in qs])
        dims = {}
        tot = w.sum()
        for (a, b), wq in zip(qs, w):
            d = int(round(D * wq / tot))
            d = min(d, _sector_max(L, i, Nu, Nd, (a, b)))
            if d > 0:
                dims[(a, b)] = d
        if not dims:  # always keep the most probable sector
            best = qs[int(np.argmax(w))]
            dims[best] = 1
        bonds.append(dims)
    bonds[0] = {(0, 0): 1}
    bonds[L] = {(Nu, Nd): 1}
    return bonds


def random_complex(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _hamming(a, b):
    return int(np.count_nonzero(np.asarray(a) != np.asarray(b)))


def det_basis_sets(L, Nu, Nd, dims_per_bond, ref_occ, seed, left_upto, right_from):
    """Orthonormal determinant bases for the bonds of a 'determinant-basis' MPS.

    Left bases S_i (i = 0..left_upto) are lists of occupation tuples of sites 0..i-1,
    built forward so that every element of S_{i+1} extends an element of S_i (prefix
    closure).  Right bases T_i (i = right_from..L) are tuples of sites i..L-1 built
    backward with suffix closure.  In each sector, candidates closest (Hamming distance)
    to the reference determinant are preferred, ties broken by the seeded generator, so
    that the bases are densely connected by single and double excitations.

    Returns (S, T) with S[i] = {charge: [tuples]} and T[i] = {left-charge: [tuples]}.
    """
    rng = _rng(seed)
    ref = tuple(int(x) for x in ref_occ)
    S = {0: {(0, 0): [()]}}
    for i in range(left_upto):
        cand = {}
        for q, lst in S[i].items():
            for t in lst:
                for s in range(4):
                    nq = (q[0] + LOCAL_CHARGE[s][0], q[1] + LOCAL_CHARGE[s][1])
                    if _sector_max(L, i + 1, Nu, Nd, nq) == 0:
                        continue
                    cand.setdefault(nq, []).append(t + (s,))
        want = dims_per_bond[i + 1]
        nxt = {}
        for nq in sorted(cand):
            c = cand[nq]
            d = want.get(nq, 0)
            if d == 0:
                continue
            key = [(_hamming(x, ref[: i + 1]), rng.random()) for x in c]
            order = sorted(range(len(c)), key=lambda j: key[j])
            nxt[nq] = [c[j] for j in order[:d]]
        S[i + 1] = nxt
    Q = (Nu, Nd)
    T = {L: {Q: [()]}}
    for i in range(L - 1, right_from - 1, -1):
        cand = {}
        for q, lst in T[i + 1].items():
            for t in lst:
                for s in range(4):
                    nq = (q[0] - LOCAL_CHARGE[s][0], q[1] - LOCAL_CHARGE[s][1])
                    if _sector_max(L, i, Nu, Nd, nq) == 0:
                        continue
                    cand.setdefault(nq, []).append((s,) + t)
        want = dims_per_bond[i]
        nxt = {}
        for nq in sorted(cand):
            c = cand[nq]
            d = want.get(nq, 0)
            if d == 0:
                continue
            key = [(_hamming(x, ref[i:]), rng.random()) for x in c]
            order = sorted(range(len(c)), key=lambda j: key[j])
            nxt[nq] = [c[j] for j in order[:d]]
        T[i] = nxt
    return S, T


def local_states():
    return list(product(range(2), range(2)))


def _panel_layout(left, right):
    """Panel layout of a site tensor given ascending sector lists [(q, dim)] of its bonds:
    returns (offset per left sector, width per left sector, {(s, n): (t, col)})."""
    rindex = {q: (t, d) for t, (q, d) in enumerate(right)}
    offs, widths, blocks = [], [], {}
    off = 0
    for s, (q, d) in enumerate(left):
        w = 0
        for n in range(4):
            nq = (q[0] + LOCAL_CHARGE[n][0], q[1] + LOCAL_CHARGE[n][1])
            if nq in rindex:
                t, dt = rindex[nq]
                blocks[(s, n)] = (t, w)
                w += dt
        offs.append(off)
        widths.append(w)
        off += d * w
    return offs, widths, blocks, off


def det_basis_state(L, Nu, Nd, D, sigma=1.0, seed=0, centre=None):
    """A block-sparse state whose bonds left of `centre` and right of `centre + 2` are
    orthonormal determinant bases (0/1 selection tensors), in the library's panel layout.

    With such a state the two-site effective Hamiltonian at bond (centre, centre+1) is the
    FCI Hamiltonian restricted to the determinants  S[a] (x) n1 (x) n2 (x) T[b].
    Returns (bonds, data, S_c, T_c2) where bonds are ascending [(n_up, n_dn, dim)] lists,
    data the concatenated complex site tensors, S_c / T_c2 dicts charge -> determinant list.
    """
    c = L // 2 - 1 if centre is None else centre
    alloc = sector_allocation(L, Nu, Nd, D, sigma)
    ref = determinant(L, Nu, Nd, seed + 7)
    S, T = det_basis_sets(L, Nu, Nd, alloc, ref, seed, left_upto=c, right_from=c + 2)
    bond_sets = {}
    for i in range(c + 1):
        bond_sets[i] = S[i]
    for i in range(c + 2, L + 1):
        bond_sets[i] = T[i]
    # bond c+1: every charge reachable from both sides, dimension 1 (its tensors are unused)
    left_q = {(q[0] + LOCAL_CHARGE[n][0], q[1] + LOCAL_CHARGE[n][1]) for q in S[c] for n in range(4)}
    right_q = {(q[0] - LOCAL_CHARGE[n][0], q[1] - LOCAL_CHARGE[n][1]) for q in T[c + 2] for n in range(4)}
    mid = sorted(left_q & right_q)
    bonds = []
    for i in range(L + 1):
        if i == c + 1:
            bonds.append([(q[0], q[1], 1) for q in mid])
        else:
            bonds.append([(q[0], q[1], len(bond_sets[i][q])) for q in sorted(bond_sets[i])])
    data = []
    for i in range(L):
        left = [((a, b), d) for a, b, d in bonds[i]]
        right = [((a, b), d) for a, b, d in bonds[i + 1]]
        offs, widths, blocks, size = _panel_layout(left, right)
        A = np.zeros(size, dtype=np.complex128)
        if i < c:  # left selection: S_{i+1}[b] = S_i[a] + (n,)
            index = {}
            for t, (q, d) in enumerate(right):
                for b, det in enumerate(bond_sets[i + 1][q]):
                    index[det] = (t, b)
            for s, (q, d) in enumerate(left):
                for a, det in enumerate(bond_sets[i][q]):
                    for n in range(4):
                        hit = index.get(det + (n,))
                        if hit is None or (s, n) not in blocks:
                            continue
                        t, b = hit
                        _, col = blocks[(s, n)]
                        A[offs[s] + a * widths[s] + col + b] = 1.0
        elif i >= c + 2:  # right selection: T_i[a] = (n,) + T_{i+1}[b]
            index = {}
            for t, (q, d) in enumerate(right):
                for b, det in enumerate(bond_sets[i + 1][q]):
                    index[det] = (t, b)
            for s, (q, d) in enumerate(left):
                for a, det in enumerate(bond_sets[i][q]):
                    n = det[0]
                    hit = index.get(det[1:])
                    if hit is None or (s, n) not in blocks:
                        continue
                    t, b = hit
                    _, col = blocks[(s, n)]
                    A[offs[s] + a * widths[s] + col + b] = 1.0
        data.append(A)
    return bonds, np.concatenate(data), S[c], T[c + 2]


def random_state(L, Nu, Nd, D, sigma=1.0, seed=0):
    """Random block-sparse state with the sector allocation above (complex Gaussian
    blocks, panel layout).  Returns (bonds, data)."""
    alloc = sector_allocation(L, Nu, Nd, D, sigma)
    bonds = [[(q[0], q[1], d) for q, d in sorted(b.items())] for b in alloc]
    rng = _rng(seed)
    data = []
    for i in range(L):
        left = [((a, b), d) for a, b, d in bonds[i]]
        right = [((a, b), d) for a, b, d in bonds[i + 1]]
        size = _panel_layout(left, right)[3]
        data.append(random_complex(rng, size) / np.sqrt(max(1, D)))
    return bonds, np.concatenate(data)


def random_unitary(rng, n):
    """Haar-like random unitary of order n (QR of a complex Gaussian, phases of R removed)."""
    q, r = np.linalg.qr(random_complex(rng, (n, n)))
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def rotate_bases(bonds, data, centre, seed):
    """Rotates the bond bases of a determinant-basis state (det_basis_state) by a random
    unitary per bond sector: bonds 1..centre and centre+2..L-1 (the bonds of the environments
    of the two-site block at (centre, centre+1)).  Site tensor i becomes U_i^H A_i U_{i+1}
    block by block, so the bond bases stay orthonormal, span the same determinants and become
    complex.  Returns the new data (panel layout, same bonds)."""
    rng = _rng(seed)
    L = len(bonds) - 1
    U = []
    for i in range(L + 1):
        rot = 1 <= i <= centre or centre + 2 <= i <= L - 1
        U.append({(a, b): (random_unitary(rng, d) if rot else np.eye(d)) for a, b, d in bonds[i]})
    out, off = [], 0
    for i in range(L):
        left = [((a, b), d) for a, b, d in bonds[i]]
        right = [((a, b), d) for a, b, d in bonds[i + 1]]
        offs, widths, blocks, size = _panel_layout(left, right)
        A = np.array(data[off:off + size], dtype=np.complex128)
        B = A.copy()
        for (s, n), (t, col) in blocks.items():
            ds, dt = left[s][1], right[t][1]
            panel = A[offs[s]:offs[s] + ds * widths[s]].reshape(ds, widths[s])
            blk = U[i][left[s][0]].conj().T @ panel[:, col:col + dt] @ U[i + 1][right[t][0]]
            B[offs[s]:offs[s] + ds * widths[s]].reshape(ds, widths[s])[:, col:col + dt] = blk
        out.append(B)
        off += size
    assert off == len(data)
    return np.concatenate(out)
