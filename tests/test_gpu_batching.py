"""Batching: the launch forms of one H_eff*theta (grouped launches, the same launches replayed
from a captured HIP graph, one launch per block product) and every tile shape of the grouped
GEMM, forced or chosen by the autotuner, give the same result bit for bit in FP64: each output
element is accumulated over the same reduction in the same order whatever tile holds it.
The grouped result itself is pinned to Slater-Condon sums in the parity suite (same state
recipe and seeds)."""
import numpy as np
import pytest
import torch

import synth
from paper_1902_08489_amd import tdmps as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    T.load()
    ctx = T.Context(0)  # the library owns a non-default stream (needed for graph capture)
    L, D = 12, 128
    h, eri, _ = synth.integrals(L)
    mpo = T.MPO.from_integrals(ctx, h, eri, 0.0)
    bonds, data, _, _ = synth.det_basis_state(L, 6, 5, D, seed=11)
    st = T.MPS.from_blocks(ctx, bonds, data)
    op = T.Heff(mpo, st, st, L // 2 - 1)
    tot, _ = op.layout(0)
    rng = np.random.default_rng(12)
    theta = rng.standard_normal(tot // 2) + 1j * rng.standard_normal(tot // 2)
    tin = torch.from_numpy(theta.view(np.float64).copy()).cuda()
    ref = torch.empty_like(tin)
    ctx.set_launch_mode(1)
    op.apply(tin.data_ptr(), ref.data_ptr())
    torch.cuda.synchronize()
    return ctx, op, tin, ref.cpu().numpy(), (mpo, st)


def _apply(op, tin):
    out = torch.full_like(tin, float("nan"))
    torch.cuda.synchronize()
    op.apply(tin.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_graph_replay_matches_eager(setup):
    """Every replay of the captured graph equals the eager grouped result; eager work (another
    H_eff apply, torch kernels, synchronisations) runs between the replays, and the output is
    poisoned with NaN before each replay so that a replay that writes nothing fails."""
    ctx, op, tin, ref, _ = setup
    out = torch.empty_like(tin)
    other = torch.empty_like(tin)
    try:
        for rep in range(4):
            ctx.set_launch_mode(2)
            out.fill_(float("nan"))
            torch.cuda.synchronize()
            op.apply(tin.data_ptr(), out.data_ptr())
            got = out.cpu().numpy()
            assert np.array_equal(got, ref), f"replay {rep}"
            ctx.set_launch_mode(1)
            op.apply(tin.data_ptr(), other.data_ptr())  # eager launches of the same plan
            torch.cuda.synchronize()
            assert np.array_equal(other.cpu().numpy(), ref)
            _ = (other * 2.0).sum().item()
    finally:
        ctx.set_launch_mode(1)


def test_per_block_heff_matches_grouped(setup):
    ctx, op, tin, ref, _ = setup
    ctx.set_launch_mode(0)
    try:
        assert np.array_equal(_apply(op, tin), ref)
    finally:
        ctx.set_launch_mode(1)


@pytest.mark.parametrize("cfg", range(T.TILE_CONFIGS))
def test_every_tile_shape_gives_the_same_result(setup, cfg):
    ctx, op, tin, ref, _ = setup
    ctx.set_tile_config(cfg)
    try:
        assert np.array_equal(_apply(op, tin), ref)
    finally:
        ctx.set_tile_config(-1)


def test_autotuned_tiles(setup):
    """The autotuner fills every bucket with a valid shape and a positive measured rate; plans
    built afterwards use it and give the same result."""
    ctx, op, tin, ref, _ = setup
    cfg, tf = ctx.autotune(T.FP64)
    try:
        assert cfg.shape == (8, 8, 3) and cfg.min() >= 0 and cfg.max() < T.TILE_CONFIGS
        assert np.all(np.isfinite(tf)) and tf.min() > 0 and tf.max() < 78.6 * 1.05
        assert np.array_equal(_apply(op, tin), ref)
    finally:
        ctx.clear_tuning()


def test_launch_mode_and_tile_config_errors(setup):
    ctx = setup[0]
    with pytest.raises(T.TdmpsError):
        ctx.set_launch_mode(3)
    with pytest.raises(T.TdmpsError):
        ctx.set_tile_config(T.TILE_CONFIGS)
    with pytest.raises(T.TdmpsError):
        ctx.autotune(7)
