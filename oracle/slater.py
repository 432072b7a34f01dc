"""Slater-Condon matrix elements of the Hamiltonian of Eq. (hamil) between determinants.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Written independently of oracle.fci: it uses the antisymmetrised spin-orbital integrals
<pq||rs> = <pq|rs> - <pq|sr>, <pq|rs> = (pr|qs) delta(s_p,s_r) delta(s_q,s_s), and the
three textbook rules (coinciding, singly and doubly differing determinants).  The
phase of a differing pair is the sign picked up when the annihilators and creators are
applied to the ket with the Jordan-Wigner convention of the basis (the lowest spin
orbital's creator leftmost).  Valid at any number of orbitals, which is what lets it
check environments and H_eff at the full benchmark sizes.
"""
from __future__ import annotations

import numpy as np


def _occ_list(mask, K):
    return [j for j in range(K) if (mask >> j) & 1]


def _sign_apply(mask, ops):
    """Sign and result of applying ops (written order, applied right to left)."""
    sign = 1
    m = mask
    for j, dag in reversed(ops):
        occ = (m >> j) & 1
        if dag == bool(occ):
            return 0, None
        if bin(m & ((1 << j) - 1)).count("1") & 1:
            sign = -sign
        m ^= 1 << j
    return sign, m


class SlaterCondon:
    def __init__(self, h, eri, e0=0.0):
        self.h = np.asarray(h, dtype=float)
        self.eri = np.asarray(eri, dtype=float)
        self.e0 = float(e0)
        self.L = self.h.shape[0]
        self.K = 2 * self.L

    def phys(self, p, q, r, s):
        """<pq|rs> over spin orbitals."""
        if (p & 1) != (r & 1) or (q & 1) != (s & 1):
            return 0.0
        return self.eri[p >> 1, r >> 1, q >> 1, s >> 1]

    def anti(self, p, q, r, s):
        return self.phys(p, q, r, s) - self.phys(p, q, s, r)

    def hso(self, p, q):
        if (p & 1) != (q & 1):
            return 0.0
        return self.h[p >> 1, q >> 1]

    def element(self, bra: int, ket: int) -> float:
        """<bra|H|ket> for spin-orbital masks."""
        diff = bra ^ ket
        nd = bin(diff).count("1")
        if nd == 0:
            occ = _occ_list(ket, self.K)
            e = self.e0 + sum(self.hso(m, m) for m in occ)
            e += 0.5 * sum(self.anti(m, n, m, n) for m in occ for n in occ)
            return e
        if nd not in (2, 4):
            return 0.0
        if bin(bra).count("1") != bin(ket).count("1"):
            return 0.0
        holes = [j for j in range(self.K) if (diff >> j) & 1 and (ket >> j) & 1]   # in ket, not bra
        parts = [j for j in range(self.K) if (diff >> j) & 1 and (bra >> j) & 1]   # in bra, not ket
        if nd == 2:
            (m,), (p,) = holes, parts
            sg, res = _sign_apply(ket, [(p, True), (m, False)])
            assert res == bra
            occ = _occ_list(ket, self.K)
            return sg * (self.hso(p, m) + sum(self.anti(p, n, m, n) for n in occ))
        m, n = holes
        p, q = parts
        sg, res = _sign_apply(ket, [(p, True), (q, True), (n, False), (m, False)])
        assert res == bra
        return sg * self.anti(p, q, m, n)


def occ_to_mask(occ):
    m = 0
    for p, n in enumerate(occ):
        n = int(n)
        if n & 1:
            m |= 1 << (2 * p)
        if n & 2:
            m |= 1 << (2 * p + 1)
    return m
