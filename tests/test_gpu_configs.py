"""The benchmark configurations as defined, and pins at benchmark sizes.

* Config 1 (RK4 stage definitions, Eq. (rk_add)): L = 8, N = 7, 20 RK4 steps of dt = 0.01
  from the ionised determinant, every step against the oracle's replica of the truncated fits
  (D = 64; with the default SVD cut-off and with 1e-5) and, at D = 160 = D_FCI, against the
  dense RK4 map (fourth-order Taylor polynomial, Methods: RK4 section).
* Default cut-off (1e-12) parity of truncated fits, with the relative gap at every truncation
  asserted above 1e-8, so the kept subspace is well posed (the oracle logs the gaps).
* The long-column SVD path (split matrices of up to 400 rows at L = 11): compression of a sum of
  two full-rank states, exact at D >= D_FCI and truncated against the replica.
* Free fermions (V = 0) at L = 16 and L = 24: gamma_pq(t) and <mu>(t) after Krylov and RK4 steps
  against the closed form conj(U) gamma(0) U^T, U = exp(-iht) (Eq. (time_evo_opera) with a
  one-body Hamiltonian), which holds at any L.
* Mixed precision over several Krylov steps (L = 8): norm, energy and dipole of the FP32 and
  BF16-split runs against the FP64 run and the oracle's replica at every step."""
import numpy as np
import pytest

import synth
from oracle import fci, mps as om, propagate
from paper_1902_08489_amd import tdmps as T

from _mpshelp import blocks_to_oracle, dense

pytestmark = pytest.mark.gpu
RTOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    T.load()
    return T.Context(0)


class Sys:
    def __init__(self, ctx, L, N0, ell=2.0, two_body=True):
        self.L = L
        self.h, eri, _ = synth.integrals(L, ell)
        self.eri = eri if two_body else np.zeros_like(eri)
        self.occ = synth.ionized_determinant(L, N0)
        self.Q = synth.occ_charge(self.occ)
        self.mpo = T.MPO.from_integrals(ctx, self.h, self.eri, 0.0)
        if L <= 10:
            self.space = fci.Space.sector(L, *self.Q)
            self.H = fci.hamiltonian(self.space, self.h, self.eri)

    def Hf(self, v):
        return self.space.embed(self.H @ self.space.restrict(v))


@pytest.fixture(scope="module")
def sys8(ctx):
    return Sys(ctx, 8, 8)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def elem(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("cut", [1e-12, 1e-5])
def test_config1_rk4_20_steps_against_replica(ctx, sys8, cut):
    """Config 1 as defined: D = 64 < D_FCI = 160, 20 steps of dt = 0.01; every step's state
    against the oracle's replica of the same fits (two sweeps), normwise and elementwise."""
    prm = T.fit_params(Dmax=64, n_sweeps=2, svd_cutoff=cut)
    ops = om.DenseOps(sys8.Hf, Dmax=64, n_sweeps=2, cutoff=cut)
    psi = T.MPS.from_determinant(ctx, sys8.occ)
    ref = om.from_occ(sys8.occ)
    om.GAP_LOG.clear()
    worst = 0.0
    for step in range(20):
        psi, info = T.rk4_step(sys8.mpo, psi, 0.01, prm)
        ref = ops.rk4_step(ref, 0.01)
        got, want = dense(psi), om.to_full(ref)
        worst = max(worst, rel(got, want), elem(got, want))
        assert rel(got, want) < RTOL and elem(got, want) < RTOL, (step, rel(got, want), elem(got, want))
    gap = min(om.GAP_LOG)
    print(f"config 1, cut {cut}: worst rel err over 20 steps {worst:.2e}, min gap at a truncation {gap:.2e}, "
          f"bond dims {list(psi.bond_dims())}")
    assert gap > 1e-8
    if cut == 1e-12:
        assert max(psi.bond_dims()) == 64  # the cap is reached: the run is truncated
    assert info.discarded_sum > 0


def test_config1_rk4_20_steps_exact_at_dfci(ctx, sys8):
    """Config 1 at D = 160 = D_FCI: every fit is exact, so each step equals the dense RK4 map
    (the degree-4 Taylor polynomial of exp(-iH dt)); its distance to the exact propagator is
    the RK4 error, bounded by sum_k (|E_k| dt)^5 / 120 per step over the energies present."""
    prm = T.fit_params(Dmax=160, n_sweeps=4)
    psi = T.MPS.from_determinant(ctx, sys8.occ)
    v = sys8.space.restrict(om.to_full(om.from_occ(sys8.occ)))
    v0 = v.copy()
    Hd = sys8.H.toarray()
    for step in range(20):
        psi, info = T.rk4_step(sys8.mpo, psi, 0.01, prm)
        v = propagate.taylor(lambda x: sys8.H @ x, v, 0.01)
        got = sys8.space.restrict(dense(psi))
        assert rel(got, v) < RTOL and elem(got, v) < RTOL, (step, rel(got, v))
    ex = propagate.exact(Hd, v0, 0.2)
    emax = np.abs(np.linalg.eigvalsh(Hd)).max()
    bound = 20 * (emax * 0.01) ** 5 / 120
    print(f"config 1 at D_FCI: |RK4 - exact| after 20 steps {np.linalg.norm(got - ex):.2e} (bound {bound:.2e})")
    assert np.linalg.norm(got - ex) < bound


def test_default_cutoff_parity_apply_krylov_compress(ctx, sys8):
    """apply_H (D = 24), a Krylov step (m = 5, D = 48) and a two-term compression (D = 16) at the
    default SVD cut-off 1e-12 against the replica; every truncation gap logged by the oracle is
    asserted above 1e-8 (reading c10: parity is well posed only there)."""
    Nu, Nd = sys8.Q
    b1, d1 = synth.random_state(8, Nu, Nd, 10, seed=5)
    b2, d2 = synth.random_state(8, Nu, Nd, 14, seed=8)
    p1, p2 = T.MPS.from_blocks(ctx, b1, d1), T.MPS.from_blocks(ctx, b2, d2)
    o1, o2 = blocks_to_oracle(b1, d1), blocks_to_oracle(b2, d2)
    phi = T.MPS.from_determinant(ctx, sys8.occ)
    om.GAP_LOG.clear()
    out, _ = T.apply_H(sys8.mpo, 0.4 - 0.3j, p1, [(0.25j, phi)], T.fit_params(Dmax=24, n_sweeps=2))
    ref = om.DenseOps(sys8.Hf, Dmax=24, n_sweeps=2).apply_H(0.4 - 0.3j, o1, [(0.25j, om.from_occ(sys8.occ))])
    assert rel(dense(out), om.to_full(ref)) < RTOL and elem(dense(out), om.to_full(ref)) < RTOL
    k, N, Hm = T.krylov_step(sys8.mpo, phi, 0.05, 5, True, T.fit_params(Dmax=48, n_sweeps=2))
    kr, Nr, Hr = om.DenseOps(sys8.Hf, Dmax=48, n_sweeps=2).krylov_step(om.from_occ(sys8.occ), 0.05, 5)
    assert np.abs(N - Nr).max() < 1e-10 and np.abs(Hm - Hr).max() < 1e-9 * np.abs(Hr).max()
    assert rel(dense(k), om.to_full(kr)) < 1e-9
    c, _ = T.compress([(1.0, p1), (0.5 - 0.5j, p2)], T.fit_params(Dmax=16, n_sweeps=2))
    cr = om.DenseOps(sys8.Hf, Dmax=16, n_sweeps=2).compress([(1.0, o1), (0.5 - 0.5j, o2)])
    assert rel(dense(c), om.to_full(cr)) < RTOL
    gap = min(om.GAP_LOG)
    print(f"default cut-off: min gap {gap:.2e} over {len(om.GAP_LOG)} truncations")
    assert gap > 1e-8


def test_long_column_svd_against_oracle(ctx):
    """L = 11, N = 10 full-rank random states (D_FCI = 1024 at the centre; split matrices of up
    to 400 rows take the eight-wave Jacobi rounds and the QR panels over 256 rows).  Their sum
    compressed with Dmax >= D_FCI is exact; capped at Dmax = 300 it equals the replica's fit
    (one sweep, default cut-off, gaps asserted)."""
    L, Nu, Nd = 11, 5, 5
    b1, d1 = synth.random_state(L, Nu, Nd, 10 ** 6, sigma=50.0, seed=1)
    b2, d2 = synth.random_state(L, Nu, Nd, 10 ** 6, sigma=50.0, seed=2)
    assert [sum(x[2] for x in b) for b in b1] == om.dfci_bonds(L, (Nu, Nd))
    p1, p2 = T.MPS.from_blocks(ctx, b1, d1), T.MPS.from_blocks(ctx, b2, d2)
    o1, o2 = blocks_to_oracle(b1, d1), blocks_to_oracle(b2, d2)
    beta = 0.5 - 0.5j
    target = om.to_full(o1) + beta * om.to_full(o2)
    full, _ = T.compress([(1.0, p1), (beta, p2)], T.fit_params(Dmax=4096, n_sweeps=1))
    got = full.to_dense()
    print(f"L=11 exact compression: rel {rel(got, target):.2e}, elementwise {elem(got, target):.2e}")
    assert rel(got, target) < RTOL and elem(got, target) < RTOL
    om.GAP_LOG.clear()
    cap, _ = T.compress([(1.0, p1), (beta, p2)], T.fit_params(Dmax=300, n_sweeps=1))
    ref, info = om.fit(target, o1, 300, n_sweeps=1)
    assert info.min_gap > 1e-8
    got, want = cap.to_dense(), om.to_full(ref)
    print(f"L=11 Dmax=300: rel {rel(got, want):.2e}, elementwise {elem(got, want):.2e}, min gap {info.min_gap:.2e}")
    assert list(cap.bond_dims()) == ref.bond_dims()
    assert rel(got, want) < RTOL and elem(got, want) < RTOL


def _free_fermion_check(ctx, L, N0, D, m, nsteps, dt_kry, dt_rk4):
    s = Sys(ctx, L, N0, ell=1.0, two_body=False)
    mu = synth.dipole_matrix(L)
    dip = T.MPO.one_body(ctx, mu)
    out = {}
    # Krylov: the error of the m-dimensional projection is negligible at these dt; the fits
    # from the determinant need several sweeps (converged when |C|^2 stops changing)
    psi = T.MPS.from_determinant(ctx, s.occ)
    prm = T.fit_params(Dmax=D, n_sweeps=8, conv_tol=1e-14)
    disc = 0.0
    for n in range(nsteps):
        psi, _, _ = T.krylov_step(s.mpo, psi, dt_kry, m, True, prm)
        disc += ctx.counters()[20]
        t = (n + 1) * dt_kry
        g = T.one_rdm(psi)
        want = propagate.free_fermion_one_rdm(s.h, s.occ, t)
        n2 = T.overlap(psi, psi).real
        d = T.expect(dip, psi, psi).real / n2
        dw = propagate.free_fermion_dipole(s.h, mu, s.occ, t)
        eg, ed = np.abs(g - want).max(), abs(d - dw)
        # The basis vectors H^k phi are truncated (the discarded weight is reported), but N and H
        # are formed on the truncated basis, so the step stays a projection onto a slightly
        # different Krylov space and its result is still accurate: 1e-9 on gamma and <mu>.
        tol = 1e-9
        print(f"L={L} Krylov step {n + 1} (t={t:.3f}): max|gamma err| {eg:.2e}, dipole {d:.12f} closed form {dw:.12f} "
              f"(tolerance {tol:.1e}, discarded {disc:.1e}), bond max {max(psi.bond_dims())}")
        assert eg < tol and ed < tol
        assert abs(n2 - 1) < 1e-8
        out[("kry", n)] = (eg, ed)
    # RK4: the degree-4 Taylor map differs from exp(-iH dt) by at most (E_max dt)^5 / 120 per
    # step on every eigencomponent; E_max from the single-particle levels of each spin
    eps = np.sort(np.abs(np.linalg.eigvalsh(s.h)))[::-1]
    emax = eps[:s.Q[0]].sum() + eps[:s.Q[1]].sum()
    psi = T.MPS.from_determinant(ctx, s.occ)
    disc = 0.0
    for n in range(nsteps):
        psi, info = T.rk4_step(s.mpo, psi, dt_rk4, prm)
        disc += info.discarded_sum
        t = (n + 1) * dt_rk4
        n2 = T.overlap(psi, psi).real
        g = T.one_rdm(psi)
        want = propagate.free_fermion_one_rdm(s.h, s.occ, t)
        state_err = (n + 1) * (emax * dt_rk4) ** 5 / 120 + np.sqrt(disc)
        # |<a|O|a>/<a|a> - <b|O|b>| <= 4 |O| |a - b| for unit b and small errors; |a+_p a_q| <= 1 per spin
        bound = 8 * state_err + 1e-12
        eg = np.abs(g - want).max()
        print(f"L={L} RK4 step {n + 1} (t={t:.3f}): max|gamma err| {eg:.2e} (bound {bound:.2e}), norm {n2:.15f}")
        assert eg < bound
        out[("rk4", n)] = eg
    return out


def test_free_fermions_L16(ctx):
    """L = 16, N = 15, D = 256 (config 2's shape with V = 0): four Krylov steps (m = 10, dt = 0.05)
    and four RK4 steps (dt = 0.005) against the closed form."""
    _free_fermion_check(ctx, 16, 16, 256, 10, 4, 0.05, 0.005)


def test_free_fermions_L24(ctx):
    """L = 24, N = 23, D = 1024 (config 3's shape with V = 0): two Krylov steps (m = 12,
    dt = 0.05) and two RK4 steps (dt = 0.005) against the closed form."""
    _free_fermion_check(ctx, 24, 24, 1024, 12, 2, 0.05, 0.005)


@pytest.mark.parametrize("prec", [T.FP32, T.BF16X3, T.BF16X6])
def test_mixed_precision_krylov_observables_every_step(ctx, sys8, prec):
    """Five Krylov steps (m = 5, dt = 0.05, D = 64, cut-off 1e-5): at every step the norm, energy
    and dipole of the FP32 / BF16-split run against the FP64 run and against the oracle's
    replica (same truncated fits in FP64).  FP32 meets the 1e-6 dipole target of the mixed form
    with margin (measured 2e-8 to 6e-8); bound 1e-6 for its dipole and energy.  The BF16 split
    keeps 16 significant bits per operand (hi + lo): its dipole error sits at the target itself
    (measured 2.2e-7 to 1.3e-6 over runs and over cut-offs 1e-5, 1e-8 and 1e-12, so it is the
    arithmetic's and not a flipped truncation), energy up to 1.9e-6: bounds 3e-6 and 1e-5.  The
    norm |psi|^2 accumulates the contraction error of every amplitude directly (measured
    1.1e-6 in FP32 and up to 5.6e-5 in the BF16 split), while energy and dipole are ratios in
    which the common error cancels: norm bounds 5e-6 and 2e-4.  The three-term BF16 split keeps
    all 24 bits of the FP32 operands: FP32's bounds."""
    mu = synth.dipole_matrix(8)
    dip = T.MPO.one_body(ctx, mu)
    Mu = fci.one_body_operator(sys8.space, mu)
    ops = om.DenseOps(sys8.Hf, Dmax=64, n_sweeps=2, cutoff=1e-5)
    ref = om.from_occ(sys8.occ)
    st = {p: T.MPS.from_determinant(ctx, sys8.occ) for p in (T.FP64, prec)}
    bound = {T.FP32: (5e-6, 1e-6, 1e-6), T.BF16X3: (2e-4, 1e-5, 3e-6), T.BF16X6: (5e-6, 1e-6, 1e-6)}[prec]
    names = ("norm", "energy", "dipole")
    worst = np.zeros((2, 3))
    for n in range(5):
        obs = {}
        for p in (T.FP64, prec):
            st[p], _, _ = T.krylov_step(sys8.mpo, st[p], 0.05, 5, True,
                                        T.fit_params(Dmax=64, n_sweeps=2, svd_cutoff=1e-5, precision=p))
            n2 = T.overlap(st[p], st[p]).real
            obs[p] = (n2, T.expect(sys8.mpo, st[p], st[p]).real / n2, T.expect(dip, st[p], st[p]).real / n2)
        ref = ops.krylov_step(ref, 0.05, 5)[0]
        v = sys8.space.restrict(om.to_full(ref))
        ora = (fci.norm2(v), fci.expectation(sys8.H, v).real, fci.expectation(Mu, v).real)
        for k in range(3):
            e64 = abs(obs[prec][k] - obs[T.FP64][k]) / abs(obs[T.FP64][k])
            eor = abs(obs[prec][k] - ora[k]) / abs(ora[k])
            print(f"precision {prec} step {n + 1} {names[k]}: vs FP64 {e64:.2e}, vs oracle {eor:.2e}")
            assert abs(obs[T.FP64][k] - ora[k]) < 1e-9 * abs(ora[k])
            worst[:, k] = np.maximum(worst[:, k], (e64, eor))
    print(f"precision {prec} worst over 5 steps (norm, energy, dipole): vs FP64 {worst[0]}, vs oracle {worst[1]}")
    assert np.all(worst < np.array(bound)), worst
