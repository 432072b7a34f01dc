"""Full-CI (occupation-number) representation and the electronic Hamiltonian.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Basis (Methods, Eq. (fci)): spin orbitals j = 2p + s (p spatial orbital, s = 0 up,
s = 1 down), ordered 1up, 1dn, 2up, 2dn, ...  A configuration is the bit mask
m = sum_j n_j 2^j and stands for the state  prod_{j ascending} (a_j^+)^{n_j} |vac>,
the lowest spin orbital's creator leftmost.  Hence
    a_j |m>  and  a_j^+ |m>  carry the sign (-1)^{#occupied k < j}.
Vectors are indexed by the "Fock index" x = sum_p n_p 4^(L-1-p), n_p = n_up + 2 n_dn,
i.e. orbital 1 is the most significant base-4 digit (the MPS ordering of Eq. (mps)).

Hamiltonian (Eq. (hamil)) with V_ijkl = (ik|jl) taken from chemists' (pq|rs):
    H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pr|qs) [E_pr E_qs - delta_qr E_ps] + E0,
    E_pq = sum_sigma a^+_{p sigma} a_{q sigma},
which is the normal-ordered two-body sum of Eq. (hamil) rewritten with the
anticommutator {a_r, a^+_q} = delta_qr.  A term-by-term brute-force application of
a^+ a^+ a a (function `apply_term_string`) pins this rewriting on tiny systems.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
import scipy.sparse as sp


def popcount(x):
    return np.bitwise_count(np.asarray(x, dtype=np.uint64)).astype(np.int64)


def fock_index(masks, L):
    masks = np.asarray(masks, dtype=np.int64)
    x = np.zeros_like(masks)
    for p in range(L):
        n = ((masks >> (2 * p)) & 1) + 2 * ((masks >> (2 * p + 1)) & 1)
        x += n * (4 ** (L - 1 - p))
    return x


def mask_from_occ(occ):
    """Occupation codes (n_up + 2 n_dn per orbital) -> spin-orbital bit mask."""
    m = 0
    for p, n in enumerate(occ):
        n = int(n)
        if n & 1:
            m |= 1 << (2 * p)
        if n & 2:
            m |= 1 << (2 * p + 1)
    return m


@lru_cache(maxsize=32)
def sector_basis(L: int, n_up: int, n_dn: int):
    """All masks with the given spin populations, sorted by Fock index.
    Returns (masks, fock) int64 arrays."""
    from itertools import combinations
    ups = [sum(1 << (2 * p) for p in c) for c in combinations(range(L), n_up)]
    dns = [sum(1 << (2 * p + 1) for p in c) for c in combinations(range(L), n_dn)]
    masks = np.array([u | d for u in ups for d in dns], dtype=np.int64)
    fock = fock_index(masks, L)
    order = np.argsort(fock)
    return masks[order], fock[order]


def full_basis(L: int):
    """Every configuration of the Fock space (4^L), in Fock-index order."""
    fock = np.arange(4 ** L, dtype=np.int64)
    masks = np.zeros_like(fock)
    for p in range(L):
        n = (fock // (4 ** (L - 1 - p))) % 4
        masks |= (n & 1) << (2 * p)
        masks |= ((n >> 1) & 1) << (2 * p + 1)
    return masks, fock


class Space:
    """A set of configurations (a spin sector or the whole Fock space)."""

    def __init__(self, L, masks):
        self.L = L
        self.masks = np.asarray(masks, dtype=np.int64)
        self.dim = len(self.masks)
        self.fock = fock_index(self.masks, L)
        self._sorted = np.argsort(self.masks)
        self._smask = self.masks[self._sorted]

    @classmethod
    def sector(cls, L, n_up, n_dn):
        return cls(L, sector_basis(L, n_up, n_dn)[0])

    @classmethod
    def full(cls, L):
        return cls(L, full_basis(L)[0])

    def lookup(self, m):
        pos = np.searchsorted(self._smask, m)
        pos = np.clip(pos, 0, self.dim - 1)
        ok = self._smask[pos] == m
        return self._sorted[pos], ok

    def embed(self, v):
        """Sector vector -> full Fock-space vector (length 4^L)."""
        out = np.zeros(4 ** self.L, dtype=np.complex128)
        out[self.fock] = v
        return out

    def restrict(self, full):
        return np.asarray(full)[self.fock]


def hop_matrix(space: Space, i: int, j: int):
    """Sparse matrix of a_i^+ a_j (spin orbitals) on `space` (which must be closed under it)."""
    m = space.masks
    if i == j:
        d = ((m >> j) & 1).astype(np.float64)
        return sp.diags(d, format="csr")
    occ_j = (m >> j) & 1
    occ_i = (m >> i) & 1
    ok = (occ_j == 1) & (occ_i == 0)
    src = np.nonzero(ok)[0]
    m0 = m[src]
    m1 = m0 ^ (1 << j)
    s1 = popcount(m0 & ((1 << j) - 1))
    s2 = popcount(m1 & ((1 << i) - 1))
    new = m1 | (1 << i)
    dst, found = space.lookup(new)
    if not np.all(found):
        raise ValueError("space not closed under a_i^+ a_j")
    vals = np.where((s1 + s2) % 2 == 0, 1.0, -1.0)
    return sp.csr_matrix((vals, (dst, src)), shape=(space.dim, space.dim))


def annihilator(src: Space, dst: Space, j: int):
    """Sparse matrix of a_j (spin orbital j) from `src` to `dst` (the sector with one electron
    of that spin less), with the sign (-1)^{#occupied k < j} of the module convention."""
    m = src.masks
    occ = ((m >> j) & 1) == 1
    cols = np.nonzero(occ)[0]
    m0 = m[cols]
    rows, found = dst.lookup(m0 ^ (1 << j))
    if not np.all(found):
        raise ValueError("destination space does not hold a_j |src>")
    vals = np.where(popcount(m0 & ((1 << j) - 1)) % 2 == 0, 1.0, -1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dst.dim, src.dim))


def excitation_ops(space: Space):
    """Spin-summed E_pq = sum_s a^+_{2p+s} a_{2q+s} for all p, q."""
    L = space.L
    E = {}
    for p in range(L):
        for q in range(L):
            E[p, q] = hop_matrix(space, 2 * p, 2 * q) + hop_matrix(space, 2 * p + 1, 2 * q + 1)
    return E


def one_body_operator(space: Space, t, E=None):
    """sum_pq t_pq E_pq (spin-conserving one-body operator)."""
    E = excitation_ops(space) if E is None else E
    L = space.L
    out = sp.csr_matrix((space.dim, space.dim))
    for p in range(L):
        for q in range(L):
            if t[p, q] != 0.0:
                out = out + t[p, q] * E[p, q]
    return out.tocsr()


def hamiltonian(space: Space, h, eri, e0=0.0):
    """Sparse FCI Hamiltonian of Eq. (hamil) on `space` (the E_pq form above)."""
    L = space.L
    E = excitation_ops(space)
    H = one_body_operator(space, h, E)
    # two-body: 1/2 sum_pr E_pr F_pr with F_pr = sum_qs (pr|qs) E_qs
    coo = [E[q, s].tocoo() for q in range(L) for s in range(L)]
    rows = np.concatenate([c.row for c in coo])
    cols = np.concatenate([c.col for c in coo])
    data = [c.data for c in coo]
    lens = [len(d) for d in data]
    data = np.concatenate(data)
    for p in range(L):
        for r in range(L):
            w = np.repeat(eri[p, r].reshape(-1), lens)
            F = sp.csr_matrix((w * data, (rows, cols)), shape=(space.dim, space.dim))
            H = H + 0.5 * (E[p, r] @ F)
    # - 1/2 sum_pqs (pq|qs) E_ps
    k = np.einsum("pqqs->ps", eri)
    H = H - 0.5 * one_body_operator(space, k, E)
    H = H + e0 * sp.identity(space.dim, format="csr")
    return H.tocsr()


class HamiltonianOp:
    """Matrix-free H @ v for sectors too large to assemble (L = 10)."""

    def __init__(self, space: Space, h, eri, e0=0.0):
        self.space = space
        self.L = space.L
        self.E = excitation_ops(space)
        self.h, self.eri, self.e0 = h, eri, e0
        self.k = np.einsum("pqqs->ps", eri)
        self.shape = (space.dim, space.dim)
        self.dtype = np.complex128

    def matvec(self, v):
        v = np.asarray(v)
        if v.ndim == 2:  # a block of vectors, column by column
            return np.stack([self.matvec(v[:, j]) for j in range(v.shape[1])], axis=1)
        L = self.L
        w = np.stack([self.E[q, s] @ v for q in range(L) for s in range(L)])  # (L^2, dim)
        u = self.eri.reshape(L * L, L * L) @ w                                  # (L^2, dim)
        out = self.e0 * v
        for p in range(L):
            for r in range(L):
                a = p * L + r
                out = out + self.E[p, r] @ (self.h[p, r] * v - 0.5 * self.k[p, r] * v + 0.5 * u[a])
        return out

    def __matmul__(self, v):
        return self.matvec(v)


# ---------------------------------------------------------------- brute force (pins)
def apply_term_string(mask: int, ops):
    """Apply a product of spin-orbital operators to one configuration.

    ops: list of (j, dagger) in written order (leftmost first); applied right to left.
    Returns (sign, new_mask) or (0, None) when the result vanishes."""
    sign = 1
    m = mask
    for j, dag in reversed(ops):
        occ = (m >> j) & 1
        if dag and occ:
            return 0, None
        if not dag and not occ:
            return 0, None
        if bin(m & ((1 << j) - 1)).count("1") % 2:
            sign = -sign
        m ^= 1 << j
    return sign, m


def hamiltonian_bruteforce(space: Space, h, eri, e0=0.0):
    """Dense H from term-by-term application of Eq. (hamil) (tiny L only)."""
    L = space.L
    H = np.zeros((space.dim, space.dim))
    index = {int(m): k for k, m in enumerate(space.masks)}
    for col, m in enumerate(space.masks):
        m = int(m)
        H[col, col] += e0
        for p in range(L):
            for q in range(L):
                for s in range(2):
                    sg, nm = apply_term_string(m, [(2 * p + s, True), (2 * q + s, False)])
                    if sg:
                        H[index[nm], col] += h[p, q] * sg
        # 1/2 sum V_ijkl c+_{i s} c+_{j t} c_{l t} c_{k s},  V_ijkl = (ik|jl)
        for i in range(L):
            for j in range(L):
                for k in range(L):
                    for l in range(L):
                        v = eri[i, k, j, l]
                        if v == 0.0:
                            continue
                        for s in range(2):
                            for t in range(2):
                                ops = [(2 * i + s, True), (2 * j + t, True), (2 * l + t, False), (2 * k + s, False)]
                                sg, nm = apply_term_string(m, ops)
                                if sg:
                                    H[index[nm], col] += 0.5 * v * sg
    return H


# ---------------------------------------------------------------- observables
def number_ops(space: Space):
    m = space.masks
    nu = sum(((m >> (2 * p)) & 1) for p in range(space.L))
    nd = sum(((m >> (2 * p + 1)) & 1) for p in range(space.L))
    return nu.astype(float), nd.astype(float)


def norm2(v):
    return float(np.real(np.vdot(v, v)))


def one_rdm(space: Space, v, E=None):
    """One-particle reduced density matrix gamma_pq = <v|E_pq|v> / <v|v> with the spin-summed
    E_pq = sum_s a^+_{ps} a_{qs} (the accuracy measure of the H2O section), by its definition:
    one expectation value per (p, q)."""
    E = excitation_ops(space) if E is None else E
    n2 = norm2(v)
    L = space.L
    g = np.zeros((L, L), dtype=np.complex128)
    for p in range(L):
        for q in range(L):
            g[p, q] = np.vdot(v, E[p, q] @ v) / n2
    return g


def expectation(op, v):
    """<v|op|v> / <v|v> (the normalisation of c16: RK4 does not conserve the norm)."""
    return complex(np.vdot(v, op @ v)) / norm2(v)
