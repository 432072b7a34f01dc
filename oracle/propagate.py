"""Time propagators on dense FCI vectors.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Units: atomic units, hbar = 1 (so the paper's 1.21 as step is dt = 0.05).
  * exact:   psi(t) = exp(-i H t) psi(0)                           Eq. (time_evo_opera)
  * rk4:     k_s = -i dt H u_s, psi' = psi + (k1 + 2 k2 + 2 k3 + k4)/6  Eqs. (k1-k4, rk_add)
             (the factor -i/hbar that the printed stage definitions drop is restored; the
             text states the map equals the 4th-order Taylor expansion of the propagator)
  * krylov:  basis phi^0 = psi, phi^{k+1} from H phi^k, either plainly normalised
             (Eq. (kry_non)) or Gram-Schmidt orthogonalised against every previous vector
             (Eq. (kry_orth)); psi' = sum_k [exp(-i dt N^-1 H)]_{k0} phi^k (Eq. (krylov_evo))
             with N_ij = <phi_i|phi_j> and H_ij = <phi_i|H|phi_j>.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def exact(H, psi, t):
    """exp(-i H t) psi: dense eigh up to dimension 6000, scipy's expm_multiply beyond."""
    if isinstance(H, np.ndarray) or H.shape[0] <= 6000:
        Hd = H if isinstance(H, np.ndarray) else H.toarray()
        w, V = np.linalg.eigh(Hd)
        return V @ (np.exp(-1j * w * t) * (V.conj().T @ psi))
    A = spla.LinearOperator(H.shape, matvec=lambda v: -1j * t * (H @ v), dtype=np.complex128)
    return spla.expm_multiply(A, np.asarray(psi, dtype=np.complex128), traceA=0.0)


def rk4(Hmv, psi, dt, t=0.0):
    """One RK4 step; Hmv(t, v) applies H(t).  Stage times t, t+dt/2, t+dt/2, t+dt."""
    k1 = -1j * dt * Hmv(t, psi)
    k2 = -1j * dt * Hmv(t + dt / 2, psi + k1 / 2)
    k3 = -1j * dt * Hmv(t + dt / 2, psi + k2 / 2)
    k4 = -1j * dt * Hmv(t + dt, psi + k3)
    return psi + (k1 + 2 * k2 + 2 * k3 + k4) / 6


def taylor(Hmv, psi, dt, order=4):
    """sum_{k<=order} (-i dt H)^k psi / k!  (closed form the RK4 map must equal)."""
    out = psi.copy()
    term = psi.copy()
    for k in range(1, order + 1):
        term = -1j * dt * Hmv(term) / k
        out = out + term
    return out


def krylov_coefficients(Nm, Hm, dt):
    """c = [exp(-i dt N^-1 H)]_{:,0} via the generalised Hermitian eigenproblem
    H V = N V Lambda, V^H N V = 1:  exp(-i dt N^-1 H) = V exp(-i dt Lambda) V^H N."""
    Hm = 0.5 * (Hm + Hm.conj().T)
    Nm = 0.5 * (Nm + Nm.conj().T)
    lam, V = sla.eigh(Hm, Nm)
    return V @ (np.exp(-1j * dt * lam) * (V.conj().T @ Nm[:, 0]))


def krylov(Hmv, psi, dt, m, orthogonal=True):
    """One Krylov step on dense vectors.  Returns (psi', N, H, c).

    phi^0 = psi/|psi|; for k < m-1: c_jk = <phi_j|H|phi_k>,
    v = H phi^k - sum_{j<=k} c_jk/<phi_j|phi_j> phi^j   (orthogonal) or  v = H phi^k,
    phi^{k+1} = v/|v|.  N and H are the overlap and Hamiltonian matrices of the basis
    (H filled from its upper triangle by Hermiticity); psi' = |psi| sum_k c_k phi^k."""
    s0 = np.sqrt(np.real(np.vdot(psi, psi)))
    phis = [psi / s0]
    Hm = np.zeros((m, m), dtype=np.complex128)
    Hphi = []
    for k in range(m):
        hk = Hmv(phis[k])
        Hphi.append(hk)
        for j in range(k + 1):
            Hm[j, k] = np.vdot(phis[j], hk)
            Hm[k, j] = np.conj(Hm[j, k])
        if k == m - 1:
            break
        v = hk.copy()
        if orthogonal:
            for j in range(k + 1):
                v = v - Hm[j, k] / np.vdot(phis[j], phis[j]) * phis[j]
        phis.append(v / np.sqrt(np.real(np.vdot(v, v))))
    Nm = np.array([[np.vdot(a, b) for b in phis] for a in phis])
    c = krylov_coefficients(Nm, Hm, dt)
    out = s0 * sum(ck * ph for ck, ph in zip(c, phis))
    return out, Nm, Hm, c


def rk4_norm_eigenstate(E, dt):
    """|R(-i E dt)|^2 with R the degree-4 Taylor polynomial (closed form)."""
    z = -1j * E * dt
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    return abs(R) ** 2
