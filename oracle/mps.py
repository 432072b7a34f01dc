"""Dense matrix product states with (N_up, N_dn) bond labels, and the fit-based drivers.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

An MPS (Eq. (mps)) is a list of tensors A_i[a, n, b] of shape (D_i, 4, D_{i+1}) plus, for
every bond, the charge (n_up, n_dn) carried by the sites left of it for each bond index.
The local index n = n_up + 2 n_dn follows the basis of oracle.fci, so contracting the
tensors left to right (site 0 most significant) gives the coefficient vector in Fock
order.

Truncation (Methods, "MPS" paragraph): keep the D largest singular values.  Reading used
for the points the paper leaves open: singular values of all charge sectors are sorted
together (value descending, then sector in lexicographic (n_up, n_dn) order, then index);
at most D are kept and only those above svd_cutoff * sigma_max (default 1e-12, the
numerical rank of an FP64 SVD of the sector sizes used; never fewer than one);
nothing is renormalised.

Variational fit (Methods, Eq. (add_min)): C approximates a target |T> = alpha H|psi> +
sum_j beta_j |phi_j> by two-site sweeps.  With the sites left of the pair in left-
orthonormal and the sites right of it in right-orthonormal form, the residual norm is
minimised by the projection theta = (U_left^H (x) 1 (x) 1 (x) V_right^H)|T>, which this
replica computes directly from the dense target (no operator or environment code).  A
sweep is a left-to-right pass over the bonds (0,1)..(L-2,L-1) followed by a right-to-left
pass back to (0,1); the initial guess is the first operand, right-canonicalised.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

QLOC = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.int64)


@dataclass
class MPS:
    tensors: list
    labels: list  # L+1 arrays of shape (D_i, 2)

    @property
    def L(self):
        return len(self.tensors)

    def copy(self):
        return MPS([t.copy() for t in self.tensors], [q.copy() for q in self.labels])

    def bond_dims(self):
        return [q.shape[0] for q in self.labels]


@dataclass
class FitInfo:
    sweeps: int = 0
    norm2: list = field(default_factory=list)
    discarded: list = field(default_factory=list)
    min_gap: float = 1.0


def from_occ(occ):
    """Product state of one determinant (bond dimension 1)."""
    L = len(occ)
    tensors, labels = [], [np.zeros((1, 2), dtype=np.int64)]
    q = np.zeros(2, dtype=np.int64)
    for p in range(L):
        A = np.zeros((1, 4, 1), dtype=np.complex128)
        A[0, int(occ[p]), 0] = 1.0
        tensors.append(A)
        q = q + QLOC[int(occ[p])]
        labels.append(q.reshape(1, 2).copy())
    return MPS(tensors, labels)


def to_full(mps: MPS):
    v = np.ones((1, 1), dtype=np.complex128)
    for A in mps.tensors:
        Dl, d, Dr = A.shape
        v = (v @ A.reshape(Dl, d * Dr)).reshape(-1, Dr)
    return v[:, 0] if v.shape[1] == 1 else v.sum(axis=1)


def _key(q):
    return (int(q[0]), int(q[1]))


LAST_GAP = [1.0]
GAP_LOG = []  # every truncation gap of fits since the last reset (test diagnostics)


def sector_svd(M, row_q, col_q, Dmax, cutoff):
    """Charge-sector SVD of M with the global truncation rule.

    Returns U (R x k), S (k), Vh (k x C), labels (k x 2), discarded weight.  The relative
    gap at the cut, (sigma_D - sigma_{D+1}) / sigma_D, is stored in LAST_GAP[0]; parity of a
    truncated result with another SVD implementation is only well posed when it is not
    tiny (reading c10 of the design notes)."""
    R, C = M.shape
    sectors = sorted(set(map(_key, row_q)) & set(map(_key, col_q)))
    rk = [_key(q) for q in row_q]
    ck = [_key(q) for q in col_q]
    pieces = []
    cand = []
    for sid, q in enumerate(sectors):
        ri = np.array([i for i in range(R) if rk[i] == q], dtype=np.int64)
        ci = np.array([j for j in range(C) if ck[j] == q], dtype=np.int64)
        u, s, vh = np.linalg.svd(M[np.ix_(ri, ci)], full_matrices=False)
        pieces.append((q, ri, ci, u, s, vh))
        for idx, val in enumerate(s):
            cand.append((-val, sid, idx))
    cand.sort()
    smax = -cand[0][0] if cand else 0.0
    keep = [c for c in cand if -c[0] > cutoff * smax][:Dmax]
    if not keep and cand:
        keep = cand[:1]
    LAST_GAP[0] = 1.0
    if len(keep) < len(cand) and -keep[-1][0] > 0:
        nxt = -cand[len(keep)][0]
        if nxt > cutoff * smax:  # a genuine truncation, not the numerical-rank cut
            LAST_GAP[0] = (-keep[-1][0] - nxt) / -keep[-1][0]
    keep_set = set((c[1], c[2]) for c in keep)
    disc = sum(c[0] ** 2 for c in cand if (c[1], c[2]) not in keep_set)
    cols_u, svals, rows_v, labs = [], [], [], []
    for sid, (q, ri, ci, u, s, vh) in enumerate(pieces):
        for idx in range(len(s)):
            if (sid, idx) in keep_set:
                cu = np.zeros(R, dtype=np.complex128)
                cu[ri] = u[:, idx]
                rv = np.zeros(C, dtype=np.complex128)
                rv[ci] = vh[idx, :]
                cols_u.append(cu)
                rows_v.append(rv)
                svals.append(s[idx])
                labs.append(q)
    U = np.stack(cols_u, axis=1)
    Vh = np.stack(rows_v, axis=0)
    return U, np.array(svals), Vh, np.array(labs, dtype=np.int64).reshape(-1, 2), float(disc)


def _config_charges(nsites):
    """Charges of all configurations of `nsites` sites in Fock order."""
    q = np.zeros((4 ** nsites, 2), dtype=np.int64)
    for k in range(nsites):
        digit = (np.arange(4 ** nsites) // (4 ** (nsites - 1 - k))) % 4
        q += QLOC[digit]
    return q


def from_full(vec, L, Q, Dmax=10 ** 9, cutoff=1e-12):
    """Sequential SVD decomposition of a full-space vector of total charge Q
    (Methods: the decomposition exists by reshaping and successive SVDs)."""
    Q = np.asarray(Q, dtype=np.int64)
    labels = [np.zeros((1, 2), dtype=np.int64)]
    tensors = []
    M = np.asarray(vec, dtype=np.complex128).reshape(4, 4 ** (L - 1))
    Dl = 1
    disc = 0.0
    for i in range(L - 1):
        rq = (labels[i][:, None, :] + QLOC[None, :, :]).reshape(-1, 2)
        cq = Q[None, :] - _config_charges(L - i - 1)
        U, S, Vh, lab, d = sector_svd(M, rq, cq, Dmax, cutoff)
        GAP_LOG.append(LAST_GAP[0])
        disc += d
        k = len(S)
        tensors.append(U.reshape(Dl, 4, k))
        labels.append(lab)
        M = (S[:, None] * Vh)
        if i < L - 2:
            M = M.reshape(k * 4, 4 ** (L - i - 2))
        Dl = k
    tensors.append(M.reshape(Dl, 4, 1))
    labels.append(Q.reshape(1, 2).copy())
    return MPS(tensors, labels), disc


def right_canonicalize(mps: MPS, cutoff=1e-12):
    """Sweep right to left with sector SVDs; sites 1..L-1 become right-orthonormal and
    site 0 holds the norm (no truncation beyond the cutoff)."""
    m = mps.copy()
    for i in range(m.L - 1, 0, -1):
        A = m.tensors[i]
        Dl, _, Dr = A.shape
        M = A.reshape(Dl, 4 * Dr)
        rq = m.labels[i]
        cq = (m.labels[i + 1][None, :, :] - QLOC[:, None, :]).reshape(-1, 2)
        U, S, Vh, lab, _ = sector_svd(M, rq, cq, 10 ** 9, cutoff)
        k = len(S)
        m.tensors[i] = Vh.reshape(k, 4, Dr)
        m.labels[i] = lab
        m.tensors[i - 1] = np.einsum("asb,bk->ask", m.tensors[i - 1], U * S[None, :])
    return m


def _left_basis(m: MPS, i):
    v = np.ones((1, 1), dtype=np.complex128)
    for A in m.tensors[:i]:
        Dl, d, Dr = A.shape
        v = (v @ A.reshape(Dl, d * Dr)).reshape(-1, Dr)
    return v  # (4^i, D_i)


def _right_basis(m: MPS, i):
    v = np.ones((1, 1), dtype=np.complex128)
    for A in reversed(m.tensors[i:]):
        Dl, d, Dr = A.shape
        v = (A.reshape(Dl * d, Dr) @ v).reshape(Dl, -1)
    return v  # (D_i, 4^(L-i))


def fit(target, init: MPS, Dmax, n_sweeps=2, cutoff=1e-12, conv_tol=0.0, first_pass_target=None):
    """Two-site variational fit of a dense target (replica of the local solves).

    first_pass_target: if given, the first left-to-right pass projects this vector instead of
    the target (the initial guess of the orthogonal Krylov fits, reading c8 of the design
    notes: a target orthogonal to the guess has no projection on a product-state guess's
    bases, so the bases are first grown on H phi_k, which contains the guess)."""
    L = init.L
    C = right_canonicalize(init, cutoff)
    info = FitInfo()
    T = np.asarray(target, dtype=np.complex128)
    T0 = T if first_pass_target is None else np.asarray(first_pass_target, dtype=np.complex128)
    prev = None
    for sweep in range(n_sweeps):
        last_norm = 0.0
        for direction, bonds in (("lr", range(0, L - 1)), ("rl", range(L - 2, -1, -1))):
            src = T0 if (sweep == 0 and direction == "lr") else T
            for i in bonds:
                Lb = _left_basis(C, i)
                Rb = _right_basis(C, i + 2)
                Dl, Dr = Lb.shape[1], Rb.shape[0]
                Tm = src.reshape(4 ** i, 16, 4 ** (L - i - 2))
                theta = np.einsum("xa,xsy,by->asb", Lb.conj(), Tm, Rb.conj(), optimize=True)
                M = theta.reshape(Dl * 4, 4 * Dr)
                rq = (C.labels[i][:, None, :] + QLOC[None, :, :]).reshape(-1, 2)
                cq = (C.labels[i + 2][None, :, :] - QLOC[:, None, :]).reshape(-1, 2)
                U, S, Vh, lab, d = sector_svd(M, rq, cq, Dmax, cutoff)
                info.discarded.append(d)
                info.min_gap = min(info.min_gap, LAST_GAP[0])
                GAP_LOG.append(LAST_GAP[0])
                k = len(S)
                if direction == "lr":
                    C.tensors[i] = U.reshape(Dl, 4, k)
                    C.tensors[i + 1] = (S[:, None] * Vh).reshape(k, 4, Dr)
                else:
                    C.tensors[i + 1] = Vh.reshape(k, 4, Dr)
                    C.tensors[i] = (U * S[None, :]).reshape(Dl, 4, k)
                C.labels[i + 1] = lab
                last_norm = float(np.sum(S ** 2))
        info.sweeps = sweep + 1
        info.norm2.append(last_norm)
        if conv_tol > 0 and prev is not None and abs(last_norm - prev) <= conv_tol * max(last_norm, 1e-300):
            break
        prev = last_norm
    return C, info


def overlap(a: MPS, b: MPS):
    return complex(np.vdot(to_full(a), to_full(b)))


def scale(m: MPS, alpha):
    out = m.copy()
    out.tensors[0] = out.tensors[0] * alpha
    return out


class DenseOps:
    """The MPS operations of the 'Operations on MPS' section on dense targets.

    Hfull(v) applies the Hamiltonian to a full Fock-space vector."""

    def __init__(self, Hfull, Dmax, n_sweeps=2, cutoff=1e-12):
        self.H = Hfull
        self.Dmax, self.n_sweeps, self.cutoff = Dmax, n_sweeps, cutoff

    def apply_H(self, alpha, psi: MPS, terms=(), H=None, grow_on_H=False):
        """Fit of alpha H psi + sum_j beta_j phi_j from psi; grow_on_H: the first left-to-right
        pass fits alpha H psi alone (the orthogonal Krylov vectors, reading c8)."""
        H = self.H if H is None else H
        h = alpha * H(to_full(psi))
        t = h
        for beta, phi in terms:
            t = t + beta * to_full(phi)
        return fit(t, psi, self.Dmax, self.n_sweeps, self.cutoff, first_pass_target=h if grow_on_H else None)[0]

    def compress(self, terms):
        t = sum(beta * to_full(phi) for beta, phi in terms)
        return fit(t, terms[0][1], self.Dmax, self.n_sweeps, self.cutoff)[0]

    def expect(self, a: MPS, b: MPS, H=None):
        H = self.H if H is None else H
        return complex(np.vdot(to_full(a), H(to_full(b))))

    # ------------------------------------------------------------ drivers
    def rk4_step(self, psi: MPS, dt, H_stages=None):
        """RK4 with fits: k_s = fit(-i dt H u_s); u_{s+1} = compress(psi + c_s k_s);
        psi' = compress(psi + k1/6 + k2/3 + k3/3 + k4/6)."""
        Hs = H_stages or (self.H, self.H, self.H, self.H)
        a = -1j * dt
        k1 = self.apply_H(a, psi, H=Hs[0])
        u2 = self.compress([(1.0, psi), (0.5, k1)])
        k2 = self.apply_H(a, u2, H=Hs[1])
        u3 = self.compress([(1.0, psi), (0.5, k2)])
        k3 = self.apply_H(a, u3, H=Hs[2])
        u4 = self.compress([(1.0, psi), (1.0, k3)])
        k4 = self.apply_H(a, u4, H=Hs[3])
        return self.compress([(1.0, psi), (1 / 6, k1), (1 / 3, k2), (1 / 3, k3), (1 / 6, k4)])

    def krylov_step(self, psi: MPS, dt, m, orthogonal=True):
        """Krylov step with fitted basis vectors (Eqs. (kry_non)/(kry_orth), (krylov_evo))."""
        from .propagate import krylov_coefficients
        s0 = np.sqrt(overlap(psi, psi).real)
        phis = [scale(psi, 1.0 / s0)]
        Hm = np.zeros((m, m), dtype=np.complex128)
        Nm = np.zeros((m, m), dtype=np.complex128)
        Nm[0, 0] = overlap(phis[0], phis[0])
        for k in range(m - 1):
            for j in range(k + 1):
                Hm[j, k] = self.expect(phis[j], phis[k])
                Hm[k, j] = np.conj(Hm[j, k])
            terms = []
            if orthogonal:
                terms = [(-Hm[j, k] / Nm[j, j], phis[j]) for j in range(k + 1)]
            nxt = self.apply_H(1.0, phis[k], terms, grow_on_H=orthogonal)
            nrm = np.sqrt(overlap(nxt, nxt).real)
            nxt = scale(nxt, 1.0 / nrm)
            phis.append(nxt)
            for j in range(k + 2):
                Nm[j, k + 1] = overlap(phis[j], nxt)
                Nm[k + 1, j] = np.conj(Nm[j, k + 1])
        for j in range(m):
            Hm[j, m - 1] = self.expect(phis[j], phis[m - 1])
            Hm[m - 1, j] = np.conj(Hm[j, m - 1])
        c = krylov_coefficients(Nm, Hm, dt)
        out = self.compress([(s0 * ck, ph) for ck, ph in zip(c, phis)])
        return out, Nm, Hm


def dfci_bonds(L, Q):
    """U(1)xU(1) D_FCI per bond: sum_q min(dim_left(q), dim_right(Q - q))."""
    from math import comb
    out = []
    for i in range(L + 1):
        tot = 0
        for nu in range(i + 1):
            for nd in range(i + 1):
                ru, rd = Q[0] - nu, Q[1] - nd
                if 0 <= ru <= L - i and 0 <= rd <= L - i:
                    tot += min(comb(i, nu) * comb(i, nd), comb(L - i, ru) * comb(L - i, rd))
        out.append(tot)
    return out
