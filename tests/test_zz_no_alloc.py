"""tdmps_heff_apply_noalloc: the two-site effective Hamiltonian product in the library's fixed
device scratch gives the output of tdmps_heff_apply bit for bit (same plan, same kernels, same
fixed summation order), on two calls in a row with the second operator smaller than the first,
and rejects an operator whose intermediates exceed the scratch before doing any device work."""
import numpy as np
import pytest
import torch

import synth
from paper_1902_08489_amd import tdmps as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    T.load()
    return T.Context(0)


def _operator(ctx, L, D, seed, precision=T.FP64):
    h, eri, _ = synth.integrals(L)
    occ = synth.ionized_determinant(L, L)
    Nu, Nd = synth.occ_charge(occ)
    mpo = T.MPO.from_integrals(ctx, h, eri, 0.0)
    b1, d1 = synth.random_state(L, Nu, Nd, D, seed=seed)
    b2, d2 = synth.random_state(L, Nu, Nd, D, seed=seed + 1)
    bra, ket = T.MPS.from_blocks(ctx, b1, d1), T.MPS.from_blocks(ctx, b2, d2)
    op = T.Heff(mpo, bra, ket, L // 2 - 1, precision)
    return op, (mpo, bra, ket)


def _check(op, seed):
    tot_k, _ = op.layout(0)
    tot_b, _ = op.layout(1)
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(tot_k) / np.sqrt(2)
    tin = torch.from_numpy(theta).cuda()
    ref = torch.full((tot_b,), float("nan"), dtype=torch.float64, device="cuda")
    out = torch.full((tot_b,), float("nan"), dtype=torch.float64, device="cuda")
    op.apply(tin.data_ptr(), ref.data_ptr())
    op.apply_noalloc(tin.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    r, o = ref.cpu().numpy(), out.cpu().numpy()
    print(f"no-allocation apply: {tot_b // 2} outputs, max |diff| {np.abs(r - o).max():.1e}")
    assert np.all(np.isfinite(r)) and np.abs(r).max() > 0
    assert np.array_equal(r, o)
    return r


def test_noalloc_matches_apply_twice_second_smaller(ctx):
    big, keep_big = _operator(ctx, 8, 48, seed=1)
    small, keep_small = _operator(ctx, 6, 24, seed=3)
    _check(big, 10)
    _check(small, 11)  # second call, smaller operator: the scratch keeps the first call's contents
    _check(big, 12)    # and back to the larger one
    fp32, keep32 = _operator(ctx, 8, 48, seed=1, precision=T.FP32)
    _check(fp32, 13)


def test_noalloc_rejects_oversize_operator(ctx):
    op, keep = _operator(ctx, 10, 256, seed=5)
    tot_k, _ = op.layout(0)
    tot_b, _ = op.layout(1)
    tin = torch.zeros(tot_k, dtype=torch.float64, device="cuda")
    out = torch.full((tot_b,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(T.TdmpsError) as e:
        op.apply_noalloc(tin.data_ptr(), out.data_ptr())
    assert e.value.code == -1 and "no-allocation scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)  # rejected before any device work
    small, keep_small = _operator(ctx, 6, 24, seed=3)
    _check(small, 14)  # the entry point still works after a rejection
