"""Pins of the CPU oracle against the paper's closed forms, textbook special cases and
independent brute-force evaluations (no GPU).  Each test names what it pins."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import fci, mps, propagate, slater

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_integrals(L, seed):
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((L, L)); h = h + h.T
    B = rng.standard_normal((L,) * 4)
    eri = sum(B.transpose(p) for p in [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
                                        (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]) / 8
    return h, eri


@pytest.mark.parametrize("L", [2, 3])
def test_hamiltonian_equals_term_by_term_bruteforce(L):
    """Eq. (hamil): the E_pq rewriting equals direct application of every
    c+ c+ c c string with Jordan-Wigner signs on the whole Fock space."""
    h, eri = _rand_integrals(L, 10 + L)
    space = fci.Space.full(L)
    H = fci.hamiltonian(space, h, eri, 0.7).toarray()
    Hb = fci.hamiltonian_bruteforce(space, h, eri, 0.7)
    assert np.abs(H - Hb).max() < 1e-12


def test_slater_condon_matches_fci_matrix():
    """Independent Slater-Condon rules reproduce every matrix element (L=4 sector)."""
    L = 4
    h, eri = _rand_integrals(L, 3)
    space = fci.Space.sector(L, 2, 2)
    H = fci.hamiltonian(space, h, eri, -0.3).toarray()
    sc = slater.SlaterCondon(h, eri, -0.3)
    M = np.array([[sc.element(int(a), int(b)) for b in space.masks] for a in space.masks])
    assert np.abs(M - H).max() < 1e-12


def test_hermitian_and_conserves_number_and_spin():
    """H is Hermitian and commutes with N_up, N_dn on the full Fock space (L=4)."""
    L = 4
    h, eri = _rand_integrals(L, 4)
    space = fci.Space.full(L)
    H = fci.hamiltonian(space, h, eri).toarray()
    assert np.abs(H - H.conj().T).max() < 1e-12
    nu, nd = fci.number_ops(space)
    assert np.abs(H * nu[None, :] - nu[:, None] * H).max() < 1e-12
    assert np.abs(H * nd[None, :] - nd[:, None] * H).max() < 1e-12


def test_fermion_operators_satisfy_canonical_anticommutation():
    """Jordan-Wigner signs of the annihilators and hopping matrices on the whole Fock space of
    L = 3 (six spin orbitals): {a_i, a_j} = 0, {a_i, a_j^+} = delta_ij, and every hopping
    matrix a_i^+ a_j (its own sign code, used by every Hamiltonian and rdm) equals the product
    of the annihilator and its adjoint; the number operator counts the set bits."""
    L = 3
    space = fci.Space.full(L)
    a = [fci.annihilator(space, space, j).toarray() for j in range(2 * L)]
    eye = np.eye(space.dim)
    for i in range(2 * L):
        for j in range(2 * L):
            assert np.array_equal(a[i] @ a[j] + a[j] @ a[i], np.zeros_like(eye))
            want = eye if i == j else np.zeros_like(eye)
            assert np.array_equal(a[i] @ a[j].T + a[j].T @ a[i], want)
            assert np.array_equal(fci.hop_matrix(space, i, j).toarray(), a[i].T @ a[j])
    nop = sum(a[j].T @ a[j] for j in range(2 * L))
    assert np.array_equal(np.diag(nop), fci.popcount(space.masks).astype(float))


def test_hubbard_dimer_closed_form():
    """Two sites, hopping -t, on-site (ii|ii) = U: singlet ground energy
    (U - sqrt(U^2 + 16 t^2))/2 (integral convention V_ijkl = (ik|jl))."""
    t, U = 0.8, 3.1
    h = np.array([[0.0, -t], [-t, 0.0]])
    eri = np.zeros((2,) * 4)
    eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
    H = fci.hamiltonian(fci.Space.sector(2, 1, 1), h, eri).toarray()
    assert abs(np.linalg.eigvalsh(H)[0] - (U - math.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_one_electron_reduces_to_h():
    """N = 1: the spectrum is eig(h) + E0 whatever the two-electron integrals."""
    L = 5
    h, eri = _rand_integrals(L, 5)
    H = fci.hamiltonian(fci.Space.sector(L, 1, 0), h, eri, 0.25).toarray()
    assert np.allclose(np.linalg.eigvalsh(H), np.linalg.eigvalsh(h) + 0.25, atol=1e-12)


def test_free_fermion_dipole_closed_form():
    """V = 0: rho_sigma(t) = exp(-iht) rho(0) exp(iht), <mu>(t) = sum_sigma Tr(mu rho); the
    oracle's closed forms (free_fermion_one_rdm / free_fermion_dipole, used at L = 16 and 24
    where no dense propagation exists) equal the many-body propagation on the FCI sector, and
    the spin-resolved trace written out here."""
    L = 6
    h, _ = synth.integrals(L)[:2]
    mu = synth.dipole_matrix(L)
    occ = synth.ionized_determinant(L, 6)
    Q = synth.occ_charge(occ)
    space = fci.Space.sector(L, *Q)
    H = fci.hamiltonian(space, h, np.zeros((L,) * 4))
    M = fci.one_body_operator(space, mu)
    psi0 = np.zeros(space.dim, complex)
    psi0[space.lookup(fci.mask_from_occ(occ))[0]] = 1
    w, V = np.linalg.eigh(h)
    for t in (0.0, 0.3, 1.7, -0.4):
        psi = propagate.exact(H, psi0, t)
        got = fci.expectation(M, psi).real
        U = V @ np.diag(np.exp(-1j * w * t)) @ V.conj().T
        want = 0.0
        for s in (1, 2):
            rho0 = np.diag([(int(o) & s) > 0 for o in occ]).astype(float)
            want += np.trace(mu @ (U @ rho0 @ U.conj().T)).real
        assert abs(got - want) < 1e-11
        assert abs(propagate.free_fermion_dipole(h, mu, occ, t) - got) < 1e-11
        g = fci.one_rdm(space, psi)
        assert np.abs(propagate.free_fermion_one_rdm(h, occ, t) - g).max() < 1e-11
    # the sign of the time matters: gamma(t) and gamma(-t) differ (imaginary parts flip)
    g1, g2 = propagate.free_fermion_one_rdm(h, occ, 0.3), propagate.free_fermion_one_rdm(h, occ, -0.3)
    assert np.abs(g1.imag).max() > 1e-3 and np.abs(g1 - g2.conj()).max() < 1e-14


@pytest.mark.parametrize("L", [6, 8])
def test_matrix_free_hamiltonian_equals_assembled(L):
    """fci.HamiltonianOp (used where the sector is too large to assemble, L = 10) against the
    assembled sparse Hamiltonian, itself pinned to term-by-term brute force, on random complex
    vectors; with e0 and two different sectors."""
    h, eri = _rand_integrals(L, 30 + L)
    rng = np.random.default_rng(L)
    for nu, nd in ((L // 2, L // 2 - 1), (2, 3)):
        space = fci.Space.sector(L, nu, nd)
        H = fci.hamiltonian(space, h, eri, 0.7)
        op = fci.HamiltonianOp(space, h, eri, 0.7)
        v = rng.standard_normal(space.dim) + 1j * rng.standard_normal(space.dim)
        want = H @ v
        assert np.abs(op @ v - want).max() < 1e-13 * np.abs(want).max()


def test_exact_propagator_expm_branch_equals_eigh():
    """The expm_multiply branch of propagate.exact (taken above dimension 6000, and with a
    matrix-free operator) against the spectral decomposition on the L = 8, N = 7 sector
    (dimension 3920), forward and backward in time; unitarity of both."""
    L = 8
    h, eri, _ = synth.integrals(L)
    occ = synth.ionized_determinant(L, 8)
    space = fci.Space.sector(L, *synth.occ_charge(occ))
    H = fci.hamiltonian(space, h, eri)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(space.dim) + 1j * rng.standard_normal(space.dim)
    v /= np.linalg.norm(v)
    for t in (0.05, 0.7, -0.3):
        a = propagate.exact(H, v, t, method="eigh")
        b = propagate.exact(H, v, t, method="expm")
        c = propagate.exact(fci.HamiltonianOp(space, h, eri), v, t)  # matrix-free: expm branch
        assert np.abs(a - b).max() < 1e-10
        assert np.abs(a - c).max() < 1e-10
        assert abs(np.linalg.norm(b) - 1) < 1e-11


def test_one_rdm_pins():
    """gamma_pq = <E_pq>: a determinant gives diag(n_p); with V = 0 the time-evolved matrix is
    conj(U) gamma(0) U^T, U = exp(-iht) (index order of gamma_pq = <a+_p a_q>); for an
    interacting state it is Hermitian with trace N and eigenvalues in [0, 2]."""
    L = 6
    h, eri, _ = synth.integrals(L)
    occ = synth.ionized_determinant(L, 6)
    space = fci.Space.sector(L, *synth.occ_charge(occ))
    psi0 = np.zeros(space.dim, complex)
    psi0[space.lookup(fci.mask_from_occ(occ))[0]] = 1
    g0 = fci.one_rdm(space, psi0)
    n = np.array([(int(o) & 1) + ((int(o) >> 1) & 1) for o in occ], float)
    assert np.abs(g0 - np.diag(n)).max() < 1e-15
    H0 = fci.hamiltonian(space, h, np.zeros((L,) * 4))
    w, V = np.linalg.eigh(h)
    for t in (0.3, 1.7):
        g = fci.one_rdm(space, propagate.exact(H0, psi0, t))
        U = V @ np.diag(np.exp(-1j * w * t)) @ V.conj().T
        assert np.abs(g - U.conj() @ g0 @ U.T).max() < 1e-11
    H = fci.hamiltonian(space, h, eri)
    g = fci.one_rdm(space, propagate.exact(H, psi0, 0.9))
    assert np.abs(g - g.conj().T).max() < 1e-13
    assert abs(np.trace(g).real - n.sum()) < 1e-12
    ev = np.linalg.eigvalsh(g)
    assert ev.min() > -1e-12 and ev.max() < 2 + 1e-12
    assert np.abs(g.imag).max() > 1e-6  # a time-evolved state has a complex matrix


def test_green_function_pins():
    """Eq. (green_time) by definition (annihilate, propagate backwards exactly, project):
    G_ij(0) = -i; for V = 0 and psi0 the ground state (a determinant of eigen-orbitals of h),
    e^{iH tau} c_js e^{-iH tau} = sum_k (e^{-ih tau})_jk c_ks gives
    sum_s <c_is psi0|e^{iH tau}|c_js psi0> = e^{iE0 tau} sum_s (e^{-ih tau} gamma_s^T)_ji with
    gamma_s,ik = <a+_is a_ks> = sum_{n occupied} conj(V_in) V_kn."""
    L = 5
    h, eri, _ = synth.integrals(L)
    nu, nd = 3, 2
    space = fci.Space.sector(L, nu, nd)
    H0 = fci.hamiltonian(space, h, np.zeros((L,) * 4)).toarray()
    w, U = np.linalg.eigh(H0)
    psi0, E0 = U[:, 0], w[0]
    eps, V = np.linalg.eigh(h)
    taus = [0.0, 0.4, 1.3]
    for i, j in ((1, 1), (0, 3), (4, 2)):
        G = propagate.green_function(L, h, np.zeros((L,) * 4), space, nu, nd, psi0, i, j, taus)
        num = np.zeros(len(taus), complex)
        den = 0.0
        for n_occ in (nu, nd):
            gam = V[:, :n_occ].conj() @ V[:, :n_occ].T  # gamma_ik = sum_n conj(V_in) V_kn
            den += gam[i, j]
            for k, t in enumerate(taus):
                P = V @ np.diag(np.exp(-1j * eps * t)) @ V.conj().T  # e^{-ih tau}
                num[k] += np.exp(1j * E0 * t) * (P @ gam.T)[j, i]
        assert abs(G[0] + 1j) < 1e-12
        assert np.abs(G - (-1j) * num / den).max() < 1e-10
    # the spin-summed gamma of the closed form is the oracle's one-particle density matrix
    g = fci.one_rdm(space, psi0)
    want = V[:, :nu].conj() @ V[:, :nu].T + V[:, :nd].conj() @ V[:, :nd].T
    assert np.abs(g - want).max() < 1e-12


def test_rk4_map_is_taylor4():
    """Eq. (rk_add): the RK4 map equals the 4th-order Taylor polynomial of exp(-iH dt)."""
    L = 4
    h, eri = _rand_integrals(L, 6)
    H = fci.hamiltonian(fci.Space.sector(L, 2, 1), h, eri)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(H.shape[0]) + 1j * rng.standard_normal(H.shape[0])
    dt = 0.07
    a = propagate.rk4(lambda t, v: H @ v, psi, dt)
    b = propagate.taylor(lambda v: H @ v, psi, dt, 4)
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()
    # and it is neither exact nor norm conserving (Methods, RK4 paragraph)
    ex = propagate.exact(H, psi, dt)
    err = np.linalg.norm(a - ex) / np.linalg.norm(ex)
    bound = (np.abs(np.linalg.eigvalsh(H.toarray())).max() * dt) ** 5 / 120
    assert 1e-12 < err <= bound * (1 + 1e-9)
    assert abs(np.linalg.norm(a) - np.linalg.norm(psi)) > 1e-14


def test_rk4_norm_for_eigenstate_closed_form():
    """|R(-i E dt)|^2 = 1 - (E dt)^6/72 + (E dt)^8/576 for an eigenstate."""
    L = 3
    h, eri = _rand_integrals(L, 7)
    H = fci.hamiltonian(fci.Space.sector(L, 2, 1), h, eri).toarray()
    w, V = np.linalg.eigh(H)
    dt = 0.09
    v = propagate.rk4(lambda t, x: H @ x, V[:, 2].astype(complex), dt)
    x = w[2] * dt
    assert abs(np.vdot(v, v).real - (1 - x ** 6 / 72 + x ** 8 / 576)) < 1e-13
    assert abs(propagate.rk4_norm_eigenstate(w[2], dt) - (1 - x ** 6 / 72 + x ** 8 / 576)) < 1e-14


def test_krylov_full_space_is_exact():
    """Eq. (krylov_evo): with N_K equal to the space dimension the step is exact."""
    L = 3
    h, eri = _rand_integrals(L, 8)
    H = fci.hamiltonian(fci.Space.sector(L, 1, 1), h, eri)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    out, Nm, Hm, c = propagate.krylov(lambda v: H @ v, psi, 0.4, 9, orthogonal=True)
    assert np.abs(out - propagate.exact(H, psi, 0.4)).max() < 1e-12
    # both bases span the same Krylov space (Methods, Krylov section), so at small N_K
    # the non-orthogonal construction gives the same step; at N_K = dim its overlap
    # matrix is near singular, which is the paper's stability remark.
    a = propagate.krylov(lambda v: H @ v, psi, 0.4, 4, orthogonal=True)[0]
    b, Nb, _, _ = propagate.krylov(lambda v: H @ v, psi, 0.4, 4, orthogonal=False)
    assert np.abs(a - b).max() < 1e-9 * np.abs(a).max()
    assert np.linalg.cond(propagate.krylov(lambda v: H @ v, psi, 0.4, 9, orthogonal=False)[1]) > 1e10


def test_krylov_conserves_norm_energy_and_converges():
    """Krylov evolution is norm and energy conserving; the orthogonal basis gives N = 1
    and a tridiagonal H; the error shrinks fast with N_K."""
    L = 6
    h, eri, _ = synth.integrals(L)
    H = fci.hamiltonian(fci.Space.sector(L, 3, 2), h, eri)
    rng = np.random.default_rng(2)
    psi = rng.standard_normal(H.shape[0]) + 1j * rng.standard_normal(H.shape[0])
    psi /= np.linalg.norm(psi)
    ex = propagate.exact(H, psi, 0.05)
    errs = []
    for m in (4, 6, 8):
        out, Nm, Hm, c = propagate.krylov(lambda v: H @ v, psi, 0.05, m)
        assert abs(np.vdot(out, out).real - 1) < 1e-12
        assert abs(np.vdot(out, H @ out) - np.vdot(psi, H @ psi)) < 1e-11
        assert np.abs(Nm - np.eye(m)).max() < 1e-10
        assert np.abs(np.triu(Hm, 2)).max() < 1e-9
        errs.append(np.linalg.norm(out - ex))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-9
    nonortho = propagate.krylov(lambda v: H @ v, psi, 0.05, 6, orthogonal=False)[0]
    assert np.linalg.norm(nonortho - ex) < 1e-7


def test_mps_sequential_svd_exact_and_truncation_weight():
    """Eq. (mps): the sequential SVD reproduces a state at D >= D_FCI, the bond dims are
    the U(1)xU(1) combinatorial D_FCI; with truncation the squared error equals the
    discarded weight of a single pass bounded as stated."""
    L = 6
    Q = (2, 3)
    space = fci.Space.sector(L, *Q)
    rng = np.random.default_rng(3)
    v = space.embed(rng.standard_normal(space.dim) + 1j * rng.standard_normal(space.dim))
    m, d = mps.from_full(v, L, Q)
    assert np.linalg.norm(mps.to_full(m) - v) < 1e-12 * np.linalg.norm(v)
    assert m.bond_dims() == mps.dfci_bonds(L, Q)
    mt, dt_ = mps.from_full(v, L, Q, Dmax=12)
    err2 = np.linalg.norm(mps.to_full(mt) - v) ** 2
    assert err2 <= dt_ * (1 + 1e-10) + 1e-20
    assert max(mt.bond_dims()) <= 12


def test_product_state_lands_on_its_fock_index():
    """Contraction order of the MPS (site 0 most significant) against the Fock index of the
    FCI basis: a determinant's product state is the unit vector at the base-4 number of its
    occupation codes, that index maps back to the same spin-orbital mask in the full basis,
    and the mask carries the determinant's electron counts."""
    rng = np.random.default_rng(3)
    L = 5
    masks, _ = fci.full_basis(L)
    for _ in range(12):
        occ = rng.integers(0, 4, L)
        v = mps.to_full(mps.from_occ(occ))
        idx = int(sum(int(n) * 4 ** (L - 1 - p) for p, n in enumerate(occ)))
        assert np.count_nonzero(v) == 1 and v[idx] == 1
        m = fci.mask_from_occ(occ)
        assert int(fci.fock_index(np.array([m]), L)[0]) == idx and int(masks[idx]) == m
        n_up = sum(int(n) & 1 for n in occ)
        n_dn = sum(int(n) >> 1 for n in occ)
        assert bin(m & int("01" * L, 2)).count("1") == n_up
        assert bin(m & int("10" * L, 2)).count("1") == n_dn


def test_sector_svd_against_dense_svd():
    """Charge-sector SVD of a block-sparse matrix with interleaved row and column charges: its
    singular values are those of a dense SVD of the whole matrix, U S Vh rebuilds it, each
    singular vector lives on its own charge; truncated to D, it keeps the D largest values
    over all sectors (the global rule) and reports the rest as the discarded weight."""
    rng = np.random.default_rng(29)
    qs = np.array([(0, 0), (1, 0), (0, 1), (1, 1)])
    rq = qs[rng.integers(0, 4, 14)]
    cq = qs[rng.integers(0, 3, 11)]
    same = np.all(rq[:, None, :] == cq[None, :, :], axis=2)
    M = np.where(same, rng.standard_normal(same.shape) + 1j * rng.standard_normal(same.shape), 0)
    dense = np.linalg.svd(M, compute_uv=False)
    U, S, Vh, lab, disc = mps.sector_svd(M, rq, cq, 10 ** 9, 1e-12)
    k = len(S)
    assert np.allclose(np.sort(S)[::-1], dense[:k], rtol=1e-12) and np.all(dense[k:] < 1e-10)
    assert np.linalg.norm(U @ np.diag(S) @ Vh - M) < 1e-12 * np.linalg.norm(M)
    assert np.allclose(U.conj().T @ U, np.eye(k), atol=1e-12)
    for j in range(k):
        assert np.all(U[~np.all(rq == lab[j], axis=1), j] == 0)
        assert np.all(Vh[j, ~np.all(cq == lab[j], axis=1)] == 0)
    U4, S4, Vh4, _, disc4 = mps.sector_svd(M, rq, cq, 4, 1e-12)
    assert np.allclose(np.sort(S4)[::-1], dense[:4], rtol=1e-12)
    assert abs(disc4 - np.sum(dense[4:] ** 2)) < 1e-10 * np.sum(dense ** 2)
    assert abs(np.linalg.norm(U4 @ np.diag(S4) @ Vh4 - M) ** 2 - disc4) < 1e-10 * np.sum(dense ** 2)


def test_right_canonical_form_keeps_the_state():
    """Right canonicalisation of a truncated MPS: the contracted state is unchanged, sites
    1..L-1 are right-orthonormal (sum over n, b of B B^H = 1), and every nonzero element
    respects the charge rule label_{i+1}[b] = label_i[a] + q(n)."""
    L = 5
    space = fci.Space.sector(L, 2, 2)
    rng = np.random.default_rng(17)
    v = rng.standard_normal(space.dim) + 1j * rng.standard_normal(space.dim)
    m, _ = mps.from_full(space.embed(v), L, (2, 2), Dmax=6)
    r = mps.right_canonicalize(m)
    a, b = mps.to_full(m), mps.to_full(r)
    assert np.linalg.norm(a - b) < 1e-12 * np.linalg.norm(a)
    for i in range(1, L):
        B = r.tensors[i].reshape(r.tensors[i].shape[0], -1)
        assert np.allclose(B @ B.conj().T, np.eye(B.shape[0]), atol=1e-12)
    for i in range(L):
        T = r.tensors[i]
        ql, qr = r.labels[i], r.labels[i + 1]
        for n in range(4):
            dq = np.array([n & 1, n >> 1])
            allowed = np.all(ql[:, None, :] + dq[None, None, :] == qr[None, :, :], axis=2)
            assert np.all(T[:, n, :][~allowed] == 0)


def test_dfci_matches_combinatorial_counts():
    assert mps.dfci_bonds(8, (3, 4))[4] == 160
    assert mps.dfci_bonds(10, (4, 5))[5] == 704


def test_spin_adapted_dfci_h10_golden():
    """Paper value: D_FCI = 462 for H10 (spin-adapted).  Counting spin-coupled states
    of the left block (Weyl-Paldus) at the centre cut and keeping min(left, right) per
    (N_left, S_left) reproduces it."""
    g = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))["h10_dfci_spin_adapted"]

    L, N = g["L"], g["N"]
    c = L // 2
    tot = 0
    for NL in range(0, 2 * c + 1):
        for twoS in range(0, NL + 1):
            if (NL - twoS) % 2:
                continue
            wl = _weyl2(c, NL, twoS)
            wr = _weyl2(L - c, N - NL, twoS)
            tot += min(wl, wr)
    assert tot == g["value"]


def _weyl2(n, N, twoS):
    """Number of spin-adapted states (2S = twoS) of N electrons in n orbitals."""
    if N < 0 or N > 2 * n or (N - twoS) % 2 or twoS < 0 or twoS > N:
        return 0
    k1 = (N - twoS) // 2
    k2 = n - (N + twoS) // 2
    if k1 < 0 or k2 < 0:
        return 0
    return (twoS + 1) * math.comb(n + 1, k1) * math.comb(n + 1, k2) // (n + 1)


def test_time_units_golden():
    g = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    au = g["au_time_fs"]["value"] * 1000  # as
    assert abs(0.05 * au - 1.21) < 0.005
    assert abs(0.02 * au - 0.484) < 0.0005


def _fixture_L6():
    L = 6
    h, eri, _ = synth.integrals(L)
    occ = synth.ionized_determinant(L, 6)
    Q = synth.occ_charge(occ)
    space = fci.Space.sector(L, *Q)
    H = fci.hamiltonian(space, h, eri)
    return L, Q, space, H, occ


def test_fit_is_exact_at_dfci():
    """Eq. (add_min): with D >= D_FCI the sweeps converge to H psi + beta phi exactly."""
    L, Q, space, H, occ = _fixture_L6()
    Hf = lambda v: space.embed(H @ space.restrict(v))
    rng = np.random.default_rng(4)
    w = space.embed(rng.standard_normal(space.dim) + 1j * rng.standard_normal(space.dim))
    psi = mps.from_full(w, L, Q, Dmax=8)[0]
    phi = mps.from_full(np.roll(w, 0) * 0.3, L, Q, Dmax=5)[0]
    ops = mps.DenseOps(Hf, Dmax=100, n_sweeps=2)
    out = ops.apply_H(0.5 - 0.2j, psi, [(1.5j, phi)])
    want = (0.5 - 0.2j) * Hf(mps.to_full(psi)) + 1.5j * mps.to_full(phi)
    assert np.linalg.norm(mps.to_full(out) - want) < 1e-12 * np.linalg.norm(want)


def test_truncated_fit_is_a_projection():
    """After the last local update C is the SVD truncation of the projected target,
    so <C|T> = <C|C> (real) and |T - C|^2 = |T|^2 - |C|^2 to rounding."""
    L, Q, space, H, occ = _fixture_L6()
    Hf = lambda v: space.embed(H @ space.restrict(v))
    rng = np.random.default_rng(5)
    w = space.embed(rng.standard_normal(space.dim) + 1j * rng.standard_normal(space.dim))
    psi = mps.from_full(w, L, Q, Dmax=10)[0]
    T = Hf(mps.to_full(psi))
    C, info = mps.fit(T, psi, Dmax=6, n_sweeps=3)
    c = mps.to_full(C)
    assert abs(np.vdot(c, T) - np.vdot(c, c)) < 1e-12 * np.vdot(c, c).real
    assert abs(np.linalg.norm(T - c) ** 2 - (np.vdot(T, T).real - np.vdot(c, c).real)) < 1e-10 * np.vdot(T, T).real
    assert max(C.bond_dims()) <= 6


def test_rk4_and_krylov_mps_drivers_exact_at_dfci():
    """RK4 and Krylov drivers built from fits reproduce their dense maps at D >= D_FCI."""
    L, Q, space, H, occ = _fixture_L6()
    Hf = lambda v: space.embed(H @ space.restrict(v))
    psi = mps.from_occ(occ)
    ops = mps.DenseOps(Hf, Dmax=100, n_sweeps=4)
    v0 = mps.to_full(psi)
    r = ops.rk4_step(psi, 0.05)
    want = space.embed(propagate.rk4(lambda t, v: H @ v, space.restrict(v0), 0.05))
    assert np.linalg.norm(mps.to_full(r) - want) < 1e-10
    k, Nm, Hm = ops.krylov_step(psi, 0.05, 5)
    want = space.embed(propagate.krylov(lambda v: H @ v, space.restrict(v0), 0.05, 5)[0])
    assert np.linalg.norm(mps.to_full(k) - want) < 1e-10


def test_slater_condon_at_large_L_single_double():
    """Slater-Condon at L = 24 agrees with the FCI construction on a 2-orbital window:
    elements between determinants that differ only inside orbitals {a, b} reduce to a
    small FCI problem with effective one-body terms (mean field of the frozen rest)."""
    L = 24
    h, eri, _ = synth.integrals(L)
    sc = slater.SlaterCondon(h, eri)
    occ = synth.ionized_determinant(L, 24)
    m = slater.occ_to_mask(occ)
    # diagonal equals sum of orbital energies + pair interactions (direct formula)
    occ_so = [j for j in range(2 * L) if (m >> j) & 1]
    e = sum(h[j >> 1, j >> 1] for j in occ_so)
    for i in occ_so:
        for j in occ_so:
            e += 0.5 * eri[i >> 1, i >> 1, j >> 1, j >> 1]
            if (i & 1) == (j & 1):
                e -= 0.5 * eri[i >> 1, j >> 1, j >> 1, i >> 1]
    assert abs(sc.element(m, m) - e) < 1e-10
    # hermiticity of off-diagonal elements
    rng = np.random.default_rng(6)
    occs = [j for j in range(2 * L) if (m >> j) & 1]
    virt = [j for j in range(2 * L) if not (m >> j) & 1]
    for _ in range(20):
        i, a = rng.choice(occs), rng.choice([v for v in virt if (v & 1) == 0] if rng.random() < 0.5 else virt)
        m2 = m ^ (1 << int(i)) ^ (1 << int(a))
        assert abs(sc.element(m2, m) - sc.element(m, m2)) < 1e-12


def test_field_driven_rk4_is_fourth_order_in_time():
    """Stage times of the driven RK4 map (t, t+dt/2, t+dt/2, t+dt): for commuting diagonal H0 and
    M the exact propagator is the phase exp(-i(e T + A m F(T))) with F the integral of the pulse
    shape (adaptive quadrature, independent of the RK4 code).  The global error must fall 16x
    per halving of dt; evaluating any stage at a wrong time leaves a first-order error."""
    from scipy.integrate import quad
    rng = np.random.default_rng(7)
    e = rng.uniform(-1, 1, 6)
    m = rng.uniform(-1, 1, 6)
    psi0 = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    psi0 /= np.linalg.norm(psi0)
    f = propagate.pulse_shape(2.0, 0.6, 0.3)
    A, T = 0.7, 1.2
    F = quad(f, 0.0, T, epsabs=1e-15, epsrel=1e-14, limit=200)[0]
    exact = np.exp(-1j * (e * T + A * F * m)) * psi0
    errs = []
    for n in (15, 30, 60):
        psi = propagate.rk4_field_forward(np.diag(e), np.diag(m), psi0, f, A, T / n, n)[-1]
        errs.append(np.linalg.norm(psi - exact))
    assert errs[-1] < 1e-8
    for a, b in zip(errs, errs[1:]):
        assert 14.0 < a / b < 18.0


def test_dipole_gradient_matches_finite_differences():
    """Adjoint gradient of the discrete RK4 map under a pulse (H(t) = H0 + A f(t) M) against
    central differences of the forward map: O(h^2) agreement pins every stage adjoint."""
    L = 4
    h, eri, _ = synth.integrals(L)
    occ = synth.ionized_determinant(L, 4)
    space = fci.Space.sector(L, *synth.occ_charge(occ))
    H0 = fci.hamiltonian(space, h, eri)
    M = fci.one_body_operator(space, synth.dipole_matrix(L))
    psi0 = space.restrict(mps.to_full(mps.from_occ(occ)))
    f = propagate.pulse_shape(2.0, 0.3, 0.2)
    A, dt, n = 0.7, 0.02, 30
    D, g = propagate.dipole_response_gradient(H0, M, M, psi0, f, A, dt, n)
    assert abs(D - propagate.dipole_response(H0, M, M, psi0, f, A, dt, n)) < 1e-13
    hh = 1e-4
    fd = (propagate.dipole_response(H0, M, M, psi0, f, A + hh, dt, n)
          - propagate.dipole_response(H0, M, M, psi0, f, A - hh, dt, n)) / (2 * hh)
    assert abs(g - fd) < 1e-8 * abs(fd)
    # zero coupling: D does not depend on A
    Z = 0 * M
    _, g0 = propagate.dipole_response_gradient(H0, Z, M, psi0, f, A, dt, n)
    assert abs(g0) < 1e-15
