"""Every output of the two-site effective Hamiltonian against the oracle.

With bond bases that are orthonormal (rotated determinant selections), the local operator of
the fit at bond (c, c+1) is P_bra^H H P_ket, where P maps a two-site tensor theta[a, s1, s2, b]
to the Fock-space vector sum_ab |left_a> |s1 s2> |right_b> (Methods, Eq. (add_min) with the
Hamiltonian of Eq. (hamil)).  The oracle forms P from the dense bond bases of the same states
(its own contraction of the site tensors), applies its FCI Hamiltonian and projects back;
the library applies its MPO environments.  Bra and ket bases are rotated by different random
unitaries per sector, so the environments are complex and bra and ket paths differ.

At L = 10, N = 9 the bases left of the centre bond (sites 4, 5) and right of it are complete,
so theta spans the whole 52,920-dimensional sector; the off-centre bonds use incomplete
(isometric) bases.  Bound: every output element within 1e-12 of the largest output (FP64);
FP32 and the BF16 split within their unit roundoffs times the reduction lengths (below)."""
import numpy as np
import pytest
import torch

import synth
from oracle import fci, mps as om
from paper_1902_08489_amd import tdmps as T

from _mpshelp import blocks_to_oracle, two_site_index

pytestmark = pytest.mark.gpu
# elementwise bounds relative to max |output|: FP64 the stated method tolerance.  FP32 rounds
# every operand and partial sum to 2^-24 = 6e-8; the BF16 split keeps 16 significant bits of
# each operand (hi + lo, 2^-16 = 1.5e-5; the dropped lo*lo term is 2^-32).  The outputs are
# sums of ~1e3..1e4 products with cancellation (the sum of |terms| exceeds |output| by up
# to ~10x), so the bounds are a few times the unit roundoff times that factor: measured at
# L = 10, 2.3e-6 (FP32) and 8.7e-6 (BF16 split).  The three-term BF16 split keeps all 24 bits of the
# FP32 operand and drops products of order 2^-24: FP32's bound.
BOUND = {T.FP64: 1e-12, T.FP32: 1e-5, T.BF16X3: 5e-5, T.BF16X6: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    T.load()
    return T.Context(0)


def _oracle_heff(Hmv, bra, ket, c, theta):
    """P_bra^H H P_ket theta with the oracle's dense bond bases (Eq. (add_min) projection)."""
    L = ket.L
    Lk, Rk = om._left_basis(ket, c), om._right_basis(ket, c + 2)
    Lb, Rb = om._left_basis(bra, c), om._right_basis(bra, c + 2)
    v = np.einsum("xa,asb,by->xsy", Lk, theta, Rk, optimize=True).reshape(-1)
    w = Hmv(v).reshape(4 ** c, 16, 4 ** (L - c - 2))
    return np.einsum("xa,xsy,by->asb", Lb.conj(), w, Rb.conj(), optimize=True)


def _run_case(ctx, L, N0, c, Hmv_factory, precisions=(T.FP64,), seed=3):
    h, eri, _ = synth.integrals(L)
    occ = synth.ionized_determinant(L, N0)
    Nu, Nd = synth.occ_charge(occ)
    space = fci.Space.sector(L, Nu, Nd)
    Hs = Hmv_factory(space, h, eri)

    def Hmv(v):
        # the bases carry the (Nu, Nd) charge: v vanishes outside the sector
        out = np.zeros_like(v)
        out[space.fock] = Hs @ v[space.fock]
        return out

    mpo = T.MPO.from_integrals(ctx, h, eri, 0.0)
    bonds, data, _, _ = synth.det_basis_state(L, Nu, Nd, 10 ** 6, sigma=50.0, seed=seed, centre=c)
    dbra = synth.rotate_bases(bonds, data, c, seed=seed + 100)
    dket = synth.rotate_bases(bonds, data, c, seed=seed + 200)
    bra, ket = T.MPS.from_blocks(ctx, bonds, dbra), T.MPS.from_blocks(ctx, bonds, dket)
    op = T.Heff(mpo, bra, ket, c)
    tot_k, blk_k = op.layout(0)
    tot_b, blk_b = op.layout(1)
    offk, idxk, shape = two_site_index(blk_k, bonds, c)
    offb, idxb, _ = two_site_index(blk_b, bonds, c)
    rng = np.random.default_rng(seed + 7)
    theta = rng.standard_normal(tot_k // 2) + 1j * rng.standard_normal(tot_k // 2)
    tdense = np.zeros(np.prod(shape), complex)
    tdense[idxk] = theta[offk]
    want_dense = _oracle_heff(Hmv, blocks_to_oracle(bonds, dbra), blocks_to_oracle(bonds, dket), c,
                              tdense.reshape(shape)).reshape(-1)
    want = np.zeros(tot_b // 2, complex)
    want[offb] = want_dense[idxb]
    # the layout covers every element the projection can reach
    mask = np.ones(want_dense.size, bool)
    mask[idxb] = False
    assert np.abs(want_dense[mask]).max(initial=0.0) < 1e-13 * np.abs(want).max()
    tin = torch.from_numpy(theta.view(np.float64).copy()).cuda()
    errs = {}
    for p in precisions:
        op.set_precision(p)
        tout = torch.full((tot_b,), float("nan"), dtype=torch.float64, device="cuda")
        op.apply(tin.data_ptr(), tout.data_ptr())
        torch.cuda.synchronize()
        got = tout.cpu().numpy().view(np.complex128)
        err = np.abs(got - want).max() / np.abs(want).max()
        errs[p] = err
        print(f"L={L} bond ({c},{c + 1}) precision {p}: {len(want)} outputs, max |err| / max |out| = {err:.2e}")
        assert np.all(np.isfinite(got))
        assert err < BOUND[p], (p, err)
    return len(want), space.dim, errs


@pytest.mark.parametrize("window", [None, "-1"])
def test_heff_all_outputs_L10_centre_whole_sector(ctx, window, monkeypatch):
    """L = 10, N = 9, bond (4, 5): complete bases on both sides (D_FCI = 256 at cuts 4 and 6),
    so theta is the whole sector; FP64, FP32 and the BF16 split on every output.  With the
    default routing of the operator's pair channels and with the plain rule (shared-block runs
    and the share pass at the centre)."""
    if window is not None:
        monkeypatch.setenv("TDMPS_MPO_ROUTING_WINDOW", window)
    n, dim, _ = _run_case(ctx, 10, 10, 4, fci.HamiltonianOp, precisions=(T.FP64, T.FP32, T.BF16X3, T.BF16X6))
    assert n == dim == 52920


def test_heff_L10_centre_mixed_precisions_fp64_storage(monkeypatch):
    """The mixed precisions with FP64 operand storage (conversion while staging tiles; a
    context created with TDMPS_MIXED_STORAGE=0) give the same bounds on every output, and the
    default FP32 storage halves the T intermediate (plan counter 3: its bytes)."""
    T.load()
    monkeypatch.setenv("TDMPS_MIXED_STORAGE", "0")
    c64 = T.Context(0)
    monkeypatch.delenv("TDMPS_MIXED_STORAGE")
    _run_case(c64, 10, 10, 4, fci.HamiltonianOp, precisions=(T.FP32, T.BF16X3, T.BF16X6))
    t_bytes_64 = c64.counters()[3]
    c32 = T.Context(0)
    _run_case(c32, 10, 10, 4, fci.HamiltonianOp, precisions=(T.FP32,))
    t_bytes_32 = c32.counters()[3]
    print(f"T intermediate: {t_bytes_64:.3e} bytes (FP64 storage), {t_bytes_32:.3e} (FP32 storage)")
    assert t_bytes_32 * 2 == t_bytes_64


@pytest.mark.parametrize("c", [2, 6])
def test_heff_all_outputs_L10_off_centre(ctx, c):
    """L = 10 bonds (2, 3) and (6, 7): both sides of the switch of the operator automaton at the
    chain centre, with one complete and one isometric (selected determinants) bond basis."""
    _run_case(ctx, 10, 10, c, fci.HamiltonianOp)


@pytest.mark.parametrize("c", range(7))
def test_heff_all_outputs_L8_every_bond(ctx, c):
    """L = 8, N = 7: every bond of the chain, all outputs, FP64."""
    _run_case(ctx, 8, 8, c, fci.hamiltonian, seed=11 + c)
