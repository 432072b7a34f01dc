"""Time propagators on dense FCI vectors.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Units: atomic units, hbar = 1 (so the paper's 1.21 as step is dt = 0.05).
  * exact:   psi(t) = exp(-i H t) psi(0)                           Eq. (time_evo_opera)
  * rk4:     k_s = -i dt H u_s, psi' = psi + (k1 + 2 k2 + 2 k3 + k4)/6  the RK4 stage definitions and Eq. (rk_add)
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


def exact(H, psi, t, method="auto"):
    """exp(-i H t) psi (Eq. (time_evo_opera)).

    method "eigh": spectral decomposition of the dense H; "expm": scipy's expm_multiply
    (truncated Taylor series with scaling, for sectors too large for eigh; H may then be a
    matrix-free operator with H @ v); "auto": eigh up to dimension 6000, expm beyond."""
    dense_ok = isinstance(H, np.ndarray) or hasattr(H, "toarray")
    if method == "auto":
        method = "eigh" if dense_ok and H.shape[0] <= 6000 else "expm"
    if method == "eigh":
        Hd = H if isinstance(H, np.ndarray) else H.toarray()
        w, V = np.linalg.eigh(Hd)
        return V @ (np.exp(-1j * w * t) * (V.conj().T @ psi))
    if method != "expm":
        raise ValueError(f"unknown method {method}")
    # scipy's norm estimate also applies the adjoint, (-i t H)^H = +i t H for Hermitian H
    A = spla.LinearOperator(H.shape, matvec=lambda v: -1j * t * (H @ v), rmatvec=lambda v: 1j * t * (H @ v),
                            dtype=np.complex128)
    return spla.expm_multiply(A, np.asarray(psi, dtype=np.complex128), traceA=0.0)


def free_fermion_one_rdm(h, occ, t):
    """Spin-summed gamma_pq(t) = sum_s <a+_{ps} a_{qs}> for V = 0 and a determinant start.

    With V = 0 each electron moves under the one-body h alone: a_{qs}(t) = sum_r U_qr a_{rs}
    with U = exp(-i h t), so <a+_{ps}(t) a_{qs}(t)> = sum_{rr'} conj(U_pr) U_qr' <a+_{rs} a_{r's}>
    and gamma(t) = conj(U) gamma(0) U^T with gamma(0) = diag(n_p) for the determinant with
    occupation codes occ (n_p = number of electrons in orbital p).  Holds at any L."""
    w, V = np.linalg.eigh(np.asarray(h, dtype=np.float64))
    U = (V * np.exp(-1j * w * t)) @ V.conj().T
    n = np.array([(int(o) & 1) + ((int(o) >> 1) & 1) for o in occ], dtype=np.float64)
    return U.conj() @ np.diag(n) @ U.T


def free_fermion_dipole(h, mu, occ, t):
    """<mu>(t) = sum_pq mu_pq gamma_pq(t) for V = 0 (the closed form of free_fermion_one_rdm)."""
    return float(np.real(np.sum(np.asarray(mu) * free_fermion_one_rdm(h, occ, t))))


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


# ---------------------------------------------------------------- field-driven dynamics
# H(t) = H0 + E(t) M with E(t) = A f(t), f(t) = sin(omega t) exp(-(t - tc)^2 / (2 tau^2)): the
# time-dependent Hamiltonian of the dipole coupling to a laser pulse (Methods: the one-body
# integrals of Eq. (hamil) carry the field).  Observable: D = <psi_N|mu|psi_N> / <psi_N|psi_N>
# after N RK4 steps of the RK4 stage definitions and Eq. (rk_add) with stage times t, t+dt/2, t+dt/2, t+dt.

def pulse_shape(omega, tc, tau):
    """f(t) such that E(t) = A f(t)."""
    return lambda t: np.sin(omega * t) * np.exp(-((t - tc) ** 2) / (2 * tau ** 2))


def rk4_field_forward(H0, M, psi0, f, A, dt, nsteps):
    """All states psi_0 .. psi_N of the RK4 propagation under H0 + A f(t) M."""
    Hmv = lambda t, v: H0 @ v + (A * f(t)) * (M @ v)
    states = [np.asarray(psi0, dtype=np.complex128)]
    for n in range(nsteps):
        states.append(rk4(Hmv, states[-1], dt, t=n * dt))
    return states


def dipole_response(H0, M, mu, psi0, f, A, dt, nsteps):
    """D(A) = <psi_N|mu|psi_N> / <psi_N|psi_N>."""
    psi = rk4_field_forward(H0, M, psi0, f, A, dt, nsteps)[-1]
    return float((psi.conj() @ (mu @ psi)).real / (psi.conj() @ psi).real)


def dipole_response_gradient(H0, M, mu, psi0, f, A, dt, nsteps):
    """dD/dA of the discrete RK4 map, by its adjoint (reverse mode through the stages).

    Each step is linear, psi_{n+1} = P_n psi_n, so dD/dA = sum_n 2 Re <lam_{n+1}| dP_n/dA psi_n>
    with lam_N = (mu - D) psi_N / |psi_N|^2 and lam_n = P_n^H lam_{n+1}.  With stage operators
    A_s = -i dt H(t_s), k_s = A_s u_s (u_1 = psi, u_2 = psi + k1/2, u_3 = psi + k2/2,
    u_4 = psi + k3) and psi' = psi + (k1 + 2 k2 + 2 k3 + k4)/6, the stage adjoints are
    kb4 = lam/6, ub4 = A_4^H kb4, kb3 = lam/3 + ub4, ub3 = A_3^H kb3, kb2 = lam/3 + ub3/2,
    ub2 = A_2^H kb2, kb1 = lam/6 + ub2/2, lam_n = lam + ub2 + ub3 + ub4 + A_1^H kb1, and the
    step contributes sum_s 2 Re <kb_s| (-i dt f(t_s) M) u_s> = 2 dt sum_s f(t_s) Im <kb_s|M|u_s>.
    Returns (D, dD/dA)."""
    states = rk4_field_forward(H0, M, psi0, f, A, dt, nsteps)
    H = lambda t: (lambda v: H0 @ v + (A * f(t)) * (M @ v))
    psiN = states[-1]
    nrm = (psiN.conj() @ psiN).real
    D = (psiN.conj() @ (mu @ psiN)).real / nrm
    lam = (mu @ psiN - D * psiN) / nrm
    grad = 0.0
    for n in range(nsteps - 1, -1, -1):
        t = n * dt
        psi = states[n]
        ts = (t, t + dt / 2, t + dt / 2, t + dt)
        k1 = -1j * dt * H(ts[0])(psi)
        u2 = psi + k1 / 2
        k2 = -1j * dt * H(ts[1])(u2)
        u3 = psi + k2 / 2
        k3 = -1j * dt * H(ts[2])(u3)
        u4 = psi + k3
        adj = lambda s, v: 1j * dt * H(ts[s])(v)  # A_s^H v (H Hermitian)
        kb4 = lam / 6
        ub4 = adj(3, kb4)
        kb3 = lam / 3 + ub4
        ub3 = adj(2, kb3)
        kb2 = lam / 3 + ub3 / 2
        ub2 = adj(1, kb2)
        kb1 = lam / 6 + ub2 / 2
        for s, (kb, u) in enumerate(((kb1, psi), (kb2, u2), (kb3, u3), (kb4, u4))):
            grad += 2 * dt * f(ts[s]) * (kb.conj() @ (M @ u)).imag
        lam = lam + ub2 + ub3 + ub4 + adj(0, kb1)
    return float(D), float(grad)


# ---------------------------------------------------------------- Green's function
# Eq. (green_time): G_ij(tau) = -i sum_s <psi0|c+_{is} e^{iH tau} c_{js}|psi0> / sum_s <psi0|c+_{is} c_{js}|psi0>,
# the ionised state c_{js} psi0 propagated backwards in time and projected on c_{is} psi0.
def green_function(L, h, eri, space, nu, nd, psi0, i, j, taus, step=None):
    """G_ij at the times `taus` from the dense vector psi0 on `space`, the (nu, nd) sector.
    step(H, v, dtau) advances v by dtau backwards in time (default: exact exp(+iH dtau)); the
    taus must then be multiples of one step size, starting at 0."""
    from . import fci
    num = np.zeros(len(taus), complex)
    den = 0.0 + 0.0j
    for s in (0, 1):
        if (nu, nd)[s] == 0:
            continue
        dst = fci.Space.sector(L, nu - (s == 0), nd - (s == 1))
        Hd = fci.hamiltonian(dst, h, eri)
        ci = fci.annihilator(space, dst, 2 * i + s) @ psi0
        v = fci.annihilator(space, dst, 2 * j + s) @ psi0
        den += np.vdot(ci, v)
        prev = 0.0
        for k, t in enumerate(taus):
            if step is None:
                w = exact(Hd, v, -t)
            else:
                if k > 0:
                    v = step(Hd, v, t - prev)
                w = v
            prev = t
            num[k] += np.vdot(ci, w)
    return -1j * num / den
