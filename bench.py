"""Benchmark: two-site H_eff*theta throughput at L = 24, D = 1024 (and Krylov steps/s).

Workload (config "Batching" of the benchmark set): L = 24 orbitals, N = 23 (11 up, 12 down),
bond dimension 1024 with the sigma = 1.0 synthetic sector allocation, MPO bond dimension
1226 at the centre.  The state has orthonormal determinant bases on the bonds left and
right of the centre pair, so the environments are exact matrix elements and the centre
H_eff is the FCI Hamiltonian on 1.06e6 product determinants; theta is seeded complex
Gaussian.  A step is one application of H_eff to theta at the centre bond, inputs resident
in HBM.  Throughput is algorithmic TFLOP/s (8 flops per complex multiply-add of the block
products in the order (L theta) -> W -> (. R)), timed with HIP events on the library's
stream.  The line also carries the same apply in the mixed precisions (FP32, BF16 split,
three-term BF16 split) and one m = 12 Krylov step at the same size in FP64 and in a mixed
precision (three-term BF16 split by default) from the same random block state, with the
relative change of norm, energy and dipole.

Other workloads of the benchmark set (each prints its own JSON line; not the default):
  --workload krylov     Krylov time steps (default L = 16, D = 256, m = 10, dt = 0.05), steps/s
                        and the per-step norm, energy and dipole
  --workload precision  one Krylov step per precision (FP64, FP32, BF16 split) from the same
                        state, per-step time and the relative change of norm, energy and
                        dipole against the FP64 run (default L = 30, D = 1024)
  --workload gradient   field-driven RK4 forward + adjoint backward for dD/dA
                        (default L = 16, D = 256, 200 steps of 0.02, checkpoints every 20)
  --workload rdm        one-particle reduced density matrix of a state in one sweep
                        (default L = 16, D = 256)
  --workload green      Green's function G_ii(tau) of Eq. (green_time) on an H10-like chain:
                        Krylov ground state, ionisation, backward Krylov steps (default
                        L = 10, N = 10, D = 30, m = 5, dt = 0.05, i = 4)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|fp32|bf16x3]
       [--krylov 0|1] [--no-cpu-baseline] [--check N] [--workload heff|krylov|precision|gradient]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Dense MFMA peaks (TFLOP/s) in algorithmic flops: the BF16 splits run three (hi + lo) or six
# (hi + mid + lo) bf16 products per real product, so their algorithmic peaks are the bf16 rate
# (2500) over three and over six.
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3, "bf16x6": 2500.0 / 6}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}

# HBM bytes of one centre apply from the hardware-counter runs of this workload
# (profiles/heff_L24_D1024_fp64_counters.md): FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB), the
# factors a 1 GiB device-to-device copy reads on the same counters.  They hold for the plan
# they were taken on (task counts and T bytes below) and this GEMM kernel.
COUNTED_TRAFFIC = {"fp64": {"L": 24, "D": 1024, "tasks": [13322, 516], "T_bytes": 15416401760.0,
                            "bytes": 93.54e9, "read": 76.57e9, "written": 16.97e9, "mfma_busy": 0.623}}


def theta_masks(L, c, blocks, S, Tset):
    """Spin-orbital mask of every element of the centre two-site tensor."""
    from oracle import slater
    masks, where = [], []
    for row in blocks:
        nu, nd, n1, n2, Da, Db = [int(v) for v in row[:6]]
        off = (int(row[6]) | (int(row[7]) << 31)) // 2
        ld = int(row[8])
        q_b = (nu + (n1 & 1) + (n2 & 1), nd + (n1 >> 1) + (n2 >> 1))
        ml = np.array([slater.occ_to_mask(d) for d in S[(nu, nd)]], dtype=np.int64)
        mr = np.array([slater.occ_to_mask((0,) * (c + 2) + tuple(d)) for d in Tset[q_b]], dtype=np.int64)
        mid = slater.occ_to_mask((0,) * c + (n1, n2))
        masks.append((ml[:, None] | mr[None, :] | mid).reshape(-1))
        where.append((off + np.arange(Da)[:, None] * ld + np.arange(Db)[None, :]).reshape(-1))
    return np.concatenate(masks), np.concatenate(where)


def oracle_rows(sc, masks, where, theta, rows):
    """Slater-Condon evaluation of sampled outputs: sum_x' <x|H|x'> theta[x']."""
    out = []
    for x in rows:
        diff = np.bitwise_count((masks ^ masks[x]).astype(np.uint64))
        cand = np.nonzero(diff <= 4)[0]
        terms = np.array([sc.element(int(masks[x]), int(masks[y])) for y in cand])
        vals = terms * theta[where[cand]]
        out.append((np.sum(vals), np.sum(np.abs(vals))))
    return out


def _cpu_worker(job):
    """One host core of the CPU baseline: the oracle's Slater-Condon sums for its share of the
    sampled outputs, for at most `seconds` (a spawned process: numpy and the oracle only)."""
    h, eri, masks, where, theta, rows, seconds = job
    from oracle import slater
    sc = slater.SlaterCondon(h, eri)
    n, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < seconds and n < len(rows):
        oracle_rows(sc, masks, where, theta, rows[n:n + 4])
        n += 4
    return min(n, len(rows)), time.perf_counter() - t1


def cpu_baseline_parallel(h, eri, masks, where, theta, rng, seconds=15.0):
    """The oracle on every host core available to this process (at most 16, the host share of
    one GPU): each core evaluates its own sampled outputs for `seconds`; throughput is the
    outputs done over the wall time, scaled to the whole apply by the output fraction."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    rows = rng.choice(len(masks), size=min(len(masks), 4096 * cores), replace=False)
    jobs = [(h, eri, masks, where, theta, rows[k::cores], seconds) for k in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_cpu_worker, jobs)
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return done, busy, wall, cores


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=list(PREC))
    ap.add_argument("--krylov", type=int, default=1, help="Krylov steps to time (one sweep per fit)")
    ap.add_argument("--mixed", type=int, default=1, help="also time the FP32 and BF16-split H_eff (FP64 runs only)")
    ap.add_argument("--krylov-m", type=int, default=12, help="Krylov dimension (12 in the benchmark definition)")
    ap.add_argument("--krylov-mixed", default="bf16x6", choices=["", "fp32", "bf16x3", "bf16x6"],
                    help="also time the Krylov steps in this precision from the same state ('' skips)")
    ap.add_argument("--check", type=int, default=8, help="sampled outputs checked against Slater-Condon")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--per-block", type=int, default=1, help="also time one launch per block product (baseline)")
    ap.add_argument("--tune", type=int, default=1, help="run the tile-shape autotuner before timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB device to device once before timing (reference for HBM byte counters)")
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--D", type=int, default=None)
    ap.add_argument("--workload", default="heff",
                    choices=["heff", "krylov", "precision", "gradient", "rdm", "green"])
    ap.add_argument("--dt", type=float, default=None)
    ap.add_argument("--sweeps", type=int, default=1, help="fit sweeps per H application (Krylov workloads)")
    ap.add_argument("--conv-tol", type=float, default=0.0, help="fit convergence tolerance on |C|^2 (0: all sweeps)")
    ap.add_argument("--init", default="random", choices=["random", "det"],
                    help="Krylov workloads: random block state at full D, or the ionised determinant")
    ap.add_argument("--observe", type=int, default=0, help="Krylov workloads: record norm, energy, dipole every step")
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3,bf16x6",
                    help="precision workload: the precisions to run (FP64 is the reference)")
    ap.add_argument("--reference", default=None,
                    help="precision workload without fp64: JSON line of an FP64 run of the same workload")
    ap.add_argument("--rk4-steps", type=int, default=200)
    ap.add_argument("--checkpoint", type=int, default=20)
    ap.add_argument("--fd", type=int, default=0, help="gradient workload: also central finite differences")
    ap.add_argument("--backward", type=int, default=1,
                    help="gradient workload: 0 skips the adjoint pass (a finite-difference-only line)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the contraction path is single-device (multi-GPU sharding over MPO "
              "channels is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    def progress(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    import torch
    import synth
    from paper_1902_08489_amd import tdmps as T

    T.load()
    if args.workload != "heff":
        return other_workload(args, progress)
    L, D = args.L or 24, args.D or 1024
    Nu, Nd = (L - 1) // 2, L // 2
    c = L // 2 - 1
    # the library's work runs on this (non-default) stream, and the events are recorded on it
    side = torch.cuda.Stream()
    ctx = T.Context(0, stream=side.cuda_stream)
    h, eri, _ = synth.integrals(L)
    mpo = T.MPO.from_integrals(ctx, h, eri, 0.0)
    bonds, data, S, Tset = synth.det_basis_state(L, Nu, Nd, D, sigma=1.0, seed=L)
    st = T.MPS.from_blocks(ctx, bonds, data)
    progress("state built")
    op = T.Heff(mpo, st, st, c, precision=PREC[args.precision])
    tot, blocks = op.layout(0)
    progress("environments built")
    rng = np.random.Generator(np.random.PCG64(L + 3))
    theta = rng.standard_normal(tot // 2) + 1j * rng.standard_normal(tot // 2)
    tin = torch.from_numpy(theta.view(np.float64).copy()).to("cuda")
    tout = torch.zeros_like(tin)
    torch.cuda.synchronize()

    def timed(n):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(side)
            op.apply(tin.data_ptr(), tout.data_ptr())
            b.record(side)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n * 1e3, [a.elapsed_time(b) for a, b in ev]

    # launch forms and tile rules (untimed probes of a few applies each)
    probe = max(3, min(args.steps, 5))
    ctx.set_launch_mode(1)
    op.apply(tin.data_ptr(), tout.data_ptr())
    grouped_ms, _ = timed(probe)
    ctx.set_launch_mode(2)
    op.apply(tin.data_ptr(), tout.data_ptr())
    graph_ms, _ = timed(probe)
    tune_cfg, t_tune, tuned_ms, tile_rule = None, 0.0, None, "cost model"
    if args.tune:
        t_tune = time.perf_counter()
        tune_cfg, _ = ctx.autotune(PREC[args.precision])
        t_tune = time.perf_counter() - t_tune
        op.apply(tin.data_ptr(), tout.data_ptr())
        tuned_ms, _ = timed(probe)
        tile_rule = "autotuned" if tuned_ms < graph_ms else "cost model"
        progress(f"autotuned in {t_tune:.1f} s")
        if tile_rule != "autotuned":
            ctx.clear_tuning()
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        op.apply(tin.data_ptr(), tout.data_ptr())
    flops = op.flops()
    plan_stats = ctx.counters()
    ms_step, kms = timed(args.steps)
    progress(f"timed {args.steps} applies: {ms_step:.2f} ms each")
    ms_kernel = float(np.mean(kms))
    value = flops / (ms_step * 1e-3) / 1e12
    achieved = flops / (ms_kernel * 1e-3) / 1e12

    out = tout.cpu().numpy().view(np.complex128)
    mixed = None
    if args.mixed and args.precision == "fp64":
        mixed = {}
        for pname in ("fp32", "bf16x3", "bf16x6"):
            op.set_precision(PREC[pname])
            for _ in range(max(1, args.warmup)):
                op.apply(tin.data_ptr(), tout.data_ptr())
            pms, pk = timed(probe)
            rule = "cost model"
            if args.tune:
                # the measured tile table of this precision against its cost model; the faster is kept
                ctx.autotune(PREC[pname])
                op.apply(tin.data_ptr(), tout.data_ptr())
                tms, tk = timed(probe)
                if tms < pms:
                    pms, pk, rule = tms, tk, "autotuned"
                else:
                    ctx.clear_tuning()
                    if tile_rule == "autotuned":
                        ctx.autotune(PREC[args.precision])
                    op.apply(tin.data_ptr(), tout.data_ptr())
                    pms, pk = timed(probe)
            low = tout.cpu().numpy().view(np.complex128)
            mixed[pname] = {"ms_per_apply": pms, "tflops_algorithmic": flops / (pms * 1e-3) / 1e12,
                            "roofline_frac": flops / (float(np.mean(pk)) * 1e-3) / 1e12 / PEAK[pname],
                            "max_abs_err_rel_to_max_fp64": float(np.abs(low - out).max() / np.abs(out).max()),
                            "rel_l2_err_vs_fp64": float(np.linalg.norm(low - out) / np.linalg.norm(out)),
                            "speedup_vs_fp64": ms_step / pms,
                            "operand_storage": "fp64" if os.environ.get("TDMPS_MIXED_STORAGE") == "0" else "fp32",
                            "tile_rule": rule,
                            "T_bytes": ctx.counters()[3]}
            progress(f"{pname}: {pms:.2f} ms per apply")
        op.set_precision(PREC[args.precision])
    # batching baseline: the same H_eff*theta with one kernel launch per block product
    batching = {"graph_ms": graph_ms, "grouped_eager_ms": grouped_ms, "graph_autotuned_ms": tuned_ms,
                "tile_rule_timed": tile_rule, "autotune_seconds": t_tune,
                "autotune_buckets_per_shape": None if tune_cfg is None else
                np.bincount(tune_cfg.ravel(), minlength=T.TILE_CONFIGS).tolist()}
    if args.per_block:
        ctx.set_launch_mode(0)
        op.apply(tin.data_ptr(), tout.data_ptr())
        torch.cuda.synchronize()
        tb = time.perf_counter()
        op.apply(tin.data_ptr(), tout.data_ptr())
        torch.cuda.synchronize()
        per_block_ms = (time.perf_counter() - tb) * 1e3
        ctx.set_launch_mode(2)
        batching.update({"per_block_ms": per_block_ms, "speedup_vs_per_block": per_block_ms / ms_step,
                         "launches_per_block_mode": int(plan_stats[4] + plan_stats[5])})
    check = None
    cpu = None
    if args.check > 0 or not args.no_cpu_baseline:
        from oracle import slater
        sc = slater.SlaterCondon(h, eri)
        masks, where = theta_masks(L, c, blocks, S, Tset)
        if args.check > 0:
            rows = rng.choice(len(masks), size=args.check, replace=False)
            worst = 0.0
            for x, (want, scale) in zip(rows, oracle_rows(sc, masks, where, theta, rows)):
                worst = max(worst, abs(out[where[x]] - want) / scale)
            check = {"sampled_outputs": int(args.check), "max_rel_err": worst,
                     "tol": 1e-12 if args.precision == "fp64" else None}
        if not args.no_cpu_baseline:
            # the oracle as it stands: Slater-Condon sums, one output at a time, ~15 s on every
            # host core of this process (spawned workers, numpy only)
            n, dt, wall, cores = cpu_baseline_parallel(h, eri, masks, where, theta, rng)
            cpu = {"value": flops * (n / len(masks)) / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
                   "sample": f"{n} of {len(masks)} outputs of the same H_eff*theta by Slater-Condon sums on "
                             f"{cores} cores ({dt:.1f} s per core, {wall:.1f} s with process start), scaled by "
                             f"the output fraction"}

    krylov = None
    if args.krylov > 0:
        os.environ["TDMPS_PROGRESS"] = "1"  # the library prints one line per Krylov vector
        bk, dk = synth.random_state(L, Nu, Nd, D, sigma=1.0, seed=L + 5)
        psi = T.MPS.from_blocks(ctx, bk, dk)
        norm0 = np.sqrt(T.overlap(psi, psi).real)  # the step is linear: scaled to unit norm
        psi.scale(1.0 / norm0)
        prm = T.fit_params(Dmax=D, n_sweeps=1, precision=PREC[args.precision])
        c0 = ctx.counters()
        built0, alloc0, alloc_s0 = c0[19], c0[17], c0[18]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.krylov):
            psi, _, _ = T.krylov_step(mpo, psi, 0.05, args.krylov_m, True, prm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        cnt = ctx.counters()
        # Phase clocks are host wall time: without TDMPS_PHASE_TIMING the launches are
        # asynchronous and GPU time lands in whichever phase next waits for the stream, so
        # per-phase rates are reported only when every phase ends with a synchronisation.
        synced = bool(os.environ.get("TDMPS_PHASE_TIMING"))
        executed = cnt[1] + cnt[7] + cnt[8]
        krylov = {"steps_per_s": args.krylov / dt, "s_per_step": dt / args.krylov, "m": args.krylov_m,
                  "sweeps_per_fit": 1,
                  "executed_tflop_last_step": executed / 1e12,
                  "executed_tflops_average": executed / (dt / args.krylov) / 1e12,
                  "phase_seconds_synchronised": synced,
                  "premix_structures_built": int(cnt[19] - built0),
                  "device_allocations": int(cnt[17] - alloc0),
                  "device_allocation_seconds": cnt[18] - alloc_s0,
                  "phase_seconds_last_step": {"heff": cnt[2], "env": cnt[3], "svd": cnt[4], "svd_qr": cnt[15],
                                              "premix": cnt[5], "sandwich_total": cnt[6],
                                              "host_planning_in_heff_env": cnt[16]},
                  "counts_last_step": {"heff": int(cnt[12]), "env_updates": int(cnt[13]), "svd": int(cnt[11]),
                                       "sandwiches": int(cnt[14]), "jacobi_sweeps": int(cnt[9]),
                                       "jacobi_rounds": int(cnt[10])},
                  "tflop_last_step": {"heff_algorithmic": cnt[0] / 1e12, "heff_executed": cnt[1] / 1e12,
                                      "env_executed": cnt[7] / 1e12, "premix_executed": cnt[8] / 1e12}}
        if synced:
            tf = lambda f, t: f / max(t, 1e-9) / 1e12
            krylov["tflops_by_phase"] = {"heff_executed": tf(cnt[1], cnt[2]), "env_executed": tf(cnt[7], cnt[3]),
                                         "premix_executed": tf(cnt[8], cnt[5])}
        if args.krylov_mixed and args.precision == "fp64":
            # the same steps from the same state in a mixed precision; norm, energy and dipole of
            # both results (observable sweeps outside the timed steps)
            psi64 = psi
            psi = T.MPS.from_blocks(ctx, bk, dk)
            psi.scale(1.0 / norm0)
            prm_mixed = T.fit_params(Dmax=D, n_sweeps=1, precision=PREC[args.krylov_mixed])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.krylov):
                psi, _, _ = T.krylov_step(mpo, psi, 0.05, args.krylov_m, True, prm_mixed)
            torch.cuda.synchronize()
            dtm = time.perf_counter() - t1
            progress(f"{args.krylov_mixed} Krylov step: {dtm / args.krylov:.1f} s")
            mu_op = T.MPO.one_body(ctx, synth.dipole_matrix(L))

            def observables(x):
                n2 = T.overlap(x, x).real
                return {"norm2": n2, "energy": T.expect(mpo, x, x).real / n2, "dipole": T.expect(mu_op, x, x).real / n2}

            o64, olow = observables(psi64), observables(psi)
            krylov["mixed"] = {"precision": args.krylov_mixed, "s_per_step": dtm / args.krylov,
                               "speedup_vs_fp64": dt / dtm, "observables_fp64": o64,
                               "rel_err_vs_fp64": {k: abs(olow[k] - o64[k]) / abs(o64[k]) for k in o64}}

    ct = COUNTED_TRAFFIC.get(args.precision)
    traffic = None
    if ct and (L, D) == (ct["L"], ct["D"]) and [int(plan_stats[4]), int(plan_stats[5])] == ct["tasks"] \
            and plan_stats[3] == ct["T_bytes"]:
        traffic = ct["bytes"]
    line = {
        "metric": "H_eff*theta TFLOP/s + Krylov steps/s @L=24 D=1024, mixed vs FP64",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "c128 (f64 MFMA)", "fp32": "c64 (f32 MFMA)", "bf16x3": "bf16 split, f32 accumulate",
                  "bf16x6": "bf16 three-term split, f32 accumulate"}[args.precision],
        "data": "synthetic (seeded integrals and determinant-basis state)",
        "config": {"workload": f"centre two-site H_eff*theta, L={L} N={Nu + Nd} D={D} sigma=1.0, "
                               f"MPO bond dim {int(mpo.bond_dims()[L // 2])}, theta {tot // 2} complex elements in "
                               f"{len(blocks)} blocks",
                   "precision": args.precision, "algorithmic_flops_per_step": flops},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[args.precision], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[args.precision], "traffic": traffic,
                     "traffic_source": None if traffic is None else
                     "rocprofv3 FETCH_SIZE / WRITE_SIZE of this plan, scaled by a 1 GiB copy "
                     "(profiles/heff_L24_D1024_fp64_counters.md); HBM bytes per apply",
                     "kernel": "the grouped block-GEMM launches of one H_eff*theta, replayed as one HIP graph "
                               f"(event-timed on the library stream, {ms_kernel:.2f} ms per step)"},
        "cpu_baseline": cpu,
        "krylov": krylov,
        "batching": batching,
        "mixed_precision": mixed,
        "check": check,
        "plan": {"executed_flops_T_stage": plan_stats[1], "executed_flops_final_stage": plan_stats[2],
                 "T_bytes": plan_stats[3], "tasks": [int(plan_stats[4]), int(plan_stats[5])],
                 "segments": [int(plan_stats[6]), int(plan_stats[7])],
                 "shared_environment_runs": int(plan_stats[8]), "shared_products_bytes": plan_stats[9]},
    }
    print(json.dumps(line), flush=True)


def other_workload(args, progress):
    import torch
    import synth
    from paper_1902_08489_amd import tdmps as T

    side = torch.cuda.Stream()
    ctx = T.Context(0, stream=side.cuda_stream)
    line = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "data": "synthetic (seeded integrals and block-sparse state)"}
    if args.workload == "green":
        L = args.L or 10
        D = args.D or 30
        nu, nd = L // 2, L - L // 2
        dt = args.dt or 0.05
        m = args.krylov_m if args.krylov_m != 12 else 5
        h, eri, _ = synth.integrals(L, 1.0)
        H = T.MPO.from_integrals(ctx, h, eri, 0.0)
        guess = T.MPS.from_determinant(ctx, synth.determinant(L, nu, nd, seed=L))
        t0 = time.perf_counter()
        psi0, E0 = T.krylov_ground(H, guess, 8, 6, T.fit_params(Dmax=max(D, 64), n_sweeps=2))
        t_gs = time.perf_counter() - t0
        progress(f"ground state E0 = {E0:.10f} in {t_gs:.1f} s")
        i = min(4, L - 1)
        prm = T.fit_params(Dmax=D, n_sweeps=1)
        ci = [T.annihilate(psi0, i, s) for s in (0, 1)]
        phi = [T.annihilate(psi0, i, s) for s in (0, 1)]
        den = sum(T.overlap(a, b) for a, b in zip(ci, phi))
        G = [complex(-1j * den / den)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            phi = [T.krylov_step(H, p, -dt, m, True, prm)[0] for p in phi]
            G.append(complex(-1j * sum(T.overlap(a, b) for a, b in zip(ci, phi)) / den))
        dt_step = (time.perf_counter() - t0) / args.steps
        line.update({"metric": f"Green's function steps/s @L={L} D={D} m={m}", "value": 1.0 / dt_step, "unit": "steps/s",
                     "ms_per_step": dt_step * 1e3, "dtype": "fp64",
                     "config": {"workload": f"G_ii(tau), i={i}, of the Krylov ground state, L={L} N={L} D={D} m={m} "
                                            f"dt={dt} (both spins propagated per step)"},
                     "ground_state_energy": E0, "ground_state_seconds": t_gs,
                     "G_imag_last": G[-1].imag, "G_real_last": G[-1].real})
        print(json.dumps(line), flush=True)
        return
    if args.workload == "rdm":
        L = args.L or 16
        D = args.D or 256
        N0 = L
        Nu, Nd = (N0 - 1) // 2, N0 - 1 - (N0 - 1) // 2
        bk, dk = synth.random_state(L, Nu, Nd, D, sigma=1.0, seed=L + 5)
        psi = T.MPS.from_blocks(ctx, bk, dk)
        for _ in range(args.warmup):
            T.one_rdm(psi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g = T.one_rdm(psi)
        dt = (time.perf_counter() - t0) / args.steps
        line.update({"metric": f"1-RDM evaluations/s @L={L} D={D}", "value": 1.0 / dt, "unit": "1/s",
                     "ms_per_step": dt * 1e3, "dtype": "fp64",
                     "config": {"workload": f"gamma_pq of a random block state, L={L} N={N0 - 1} D={D}"},
                     "trace": float(np.trace(g).real), "hermiticity": float(np.abs(g - g.conj().T).max())})
        print(json.dumps(line), flush=True)
        return
    if args.workload in ("krylov", "precision"):
        L = args.L or (16 if args.workload == "krylov" else 30)
        D = args.D or (256 if args.workload == "krylov" else 1024)
        m = args.krylov_m if args.krylov_m != 12 or args.workload == "precision" else 10
        dt = args.dt or 0.05
        N0 = L if args.workload == "krylov" else 28
        ell = 1.0 if args.workload == "krylov" else 2.0
        Nu, Nd = (N0 - 1) // 2, N0 - 1 - (N0 - 1) // 2
        h, eri, _ = synth.integrals(L, ell)
        mu_pq = synth.dipole_matrix(L, ell)
        H = T.MPO.from_integrals(ctx, h, eri, 0.0)
        MU = T.MPO.one_body(ctx, mu_pq)
        if args.init == "det":
            psi0 = T.MPS.from_determinant(ctx, synth.ionized_determinant(L, N0))
            init = "the ionised determinant"
        else:
            bk, dk = synth.random_state(L, Nu, Nd, D, sigma=1.0, seed=L + 5)
            psi0 = T.MPS.from_blocks(ctx, bk, dk)
            psi0.scale(1.0 / np.sqrt(T.overlap(psi0, psi0).real))
            init = "a random block state at full D"
        progress(f"L={L} D={D} state built")

        def observables(psi):
            n2 = T.overlap(psi, psi).real
            return {"norm2": n2, "energy": T.expect(H, psi, psi).real / n2, "dipole": T.expect(MU, psi, psi).real / n2}

        def run(prec, nsteps, warm):
            prm = T.fit_params(Dmax=D, n_sweeps=args.sweeps, conv_tol=args.conv_tol, precision=PREC[prec])
            psi = psi0
            for _ in range(warm):
                psi, _, _ = T.krylov_step(H, psi, dt, m, True, prm)
            traj = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t_obs = 0.0
            for k in range(nsteps):
                psi, _, _ = T.krylov_step(H, psi, dt, m, True, prm)
                if args.observe:
                    # observables are outside the step time (their sweeps are not part of a step)
                    torch.cuda.synchronize()
                    to = time.perf_counter()
                    traj.append({"t": (warm + k + 1) * dt, **observables(psi), "bond_max": int(max(psi.bond_dims()))})
                    t_obs += time.perf_counter() - to
                progress(f"{prec} Krylov step {k + 1} of {nsteps}: {time.perf_counter() - t0:.1f} s")
            torch.cuda.synchronize()
            return (time.perf_counter() - t0 - t_obs) / nsteps, observables(psi), traj

        os.environ["TDMPS_PROGRESS"] = "1"
        sweeps_txt = f"{args.sweeps} sweep(s) per fit" + (f" (stop at |C|^2 change < {args.conv_tol})"
                                                           if args.conv_tol > 0 else "")
        if args.workload == "krylov":
            sps, obs, traj = run(args.precision, args.steps, args.warmup)
            line.update({"metric": f"Krylov steps/s @L={L} D={D} m={m}", "value": 1.0 / sps, "unit": "steps/s",
                         "ms_per_step": sps * 1e3, "dtype": args.precision,
                         "config": {"workload": f"Krylov time step, L={L} N={N0 - 1} D={D} m={m} dt={dt}, "
                                                f"{sweeps_txt}, from {init}",
                                    "precision": args.precision},
                         "observables_after": obs})
            if traj:
                line["trajectory"] = traj
                e = [x["energy"] for x in traj]
                line["energy_drift"] = max(e) - min(e)
        else:
            res = {}
            trajs = {}
            precs = [p for p in args.precisions.split(",") if p]
            if not precs or any(p not in PREC for p in precs):
                raise SystemExit("--precisions: a comma-separated list of fp64, fp32, bf16x3, bf16x6")
            ref_src = "this run"
            if "fp64" not in precs:
                # FP64 reference trajectory of an earlier run of the same workload
                if not args.reference:
                    raise SystemExit("--precisions without fp64 needs --reference (an FP64 line of this workload)")
                with open(args.reference) as f:
                    ref_line = json.loads(f.read().strip().splitlines()[-1])
                res["fp64"] = ref_line["per_precision"]["fp64"]
                trajs["fp64"] = res["fp64"].get("trajectory", [])
                ref_src = f"the FP64 run in {os.path.basename(args.reference)}"
            for prec in precs:
                sps, obs, traj = run(prec, args.steps, 0)
                res[prec] = {"s_per_step": sps, **obs, "trajectory": traj}
                trajs[prec] = traj
            ref = res["fp64"]
            low = [p for p in precs if p != "fp64"]
            for prec in low:
                res[prec]["rel_err_vs_fp64"] = {k: abs(res[prec][k] - ref[k]) / abs(ref[k])
                                                for k in ("norm2", "energy", "dipole")}
                if trajs[prec]:
                    res[prec]["rel_err_vs_fp64_per_step"] = [
                        {k: abs(a[k] - b[k]) / abs(b[k]) for k in ("norm2", "energy", "dipole")}
                        for a, b in zip(trajs[prec], trajs["fp64"])]
                    res[prec]["max_rel_err_vs_fp64_over_steps"] = {
                        k: max(x[k] for x in res[prec]["rel_err_vs_fp64_per_step"]) for k in ("norm2", "energy", "dipole")}
            best = min(low, key=lambda p: res[p]["s_per_step"]) if low else "fp64"
            line.update({"metric": f"Krylov steps/s @L={L} D={D}, mixed vs FP64", "value": 1.0 / res[best]["s_per_step"],
                         "unit": "steps/s", "ms_per_step": res[best]["s_per_step"] * 1e3, "dtype": best,
                         "config": {"workload": f"Krylov time step, L={L} N={N0 - 1} D={D} m={m} dt={dt}, "
                                                f"{sweeps_txt}, from {init}; {args.steps} steps per precision",
                                    "precisions_run": precs, "fp64_reference": ref_src},
                         "speedup_vs_fp64": ref["s_per_step"] / res[best]["s_per_step"], "per_precision": res})
    else:
        L = args.L or 16
        D = args.D or 256
        N0 = L
        Nu, Nd = (N0 - 1) // 2, N0 - 1 - (N0 - 1) // 2
        dt = args.dt or 0.02
        h, eri, _ = synth.integrals(L, 1.0)
        mu_pq = synth.dipole_matrix(L, 1.0)
        H0 = T.MPO.from_integrals(ctx, h, eri, 0.0)
        MU = T.MPO.one_body(ctx, mu_pq)
        psi0 = T.MPS.from_determinant(ctx, synth.ionized_determinant(L, N0))
        prm = T.fit_params(Dmax=D, n_sweeps=args.sweeps, precision=PREC[args.precision])
        pulse = dict(omega=1.0, t_center=2.0, width=0.5)
        os.environ["TDMPS_PROGRESS"] = "1"  # the library prints one line per checkpoint interval
        A = 0.01
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = T.Trajectory(H0, h, mu_pq, MU, psi0, A, pulse["omega"], pulse["t_center"], pulse["width"], dt,
                          args.rk4_steps, args.checkpoint, prm)
        t_fwd = time.perf_counter() - t0
        progress(f"forward {args.rk4_steps} RK4 steps: {t_fwd:.1f} s")
        g, t_bwd = None, 0.0
        if args.backward:
            t0 = time.perf_counter()
            g = tr.backward()
            t_bwd = time.perf_counter() - t0
            progress(f"backward: {t_bwd:.1f} s")
        fd = None
        if args.fd:
            hA = 1e-4
            vp = T.Trajectory(H0, h, mu_pq, MU, psi0, A + hA, pulse["omega"], pulse["t_center"], pulse["width"], dt,
                              args.rk4_steps, args.checkpoint, prm).value
            vm = T.Trajectory(H0, h, mu_pq, MU, psi0, A - hA, pulse["omega"], pulse["t_center"], pulse["width"], dt,
                              args.rk4_steps, args.checkpoint, prm).value
            fd = (vp - vm) / (2 * hA)
            progress(f"finite difference: {fd:.12e}")
        what = "forward+adjoint" if args.backward else "forward"
        line.update({"metric": f"RK4 {what} steps/s @L={L} D={D}", "value": args.rk4_steps / (t_fwd + t_bwd),
                     "unit": "steps/s", "ms_per_step": (t_fwd + t_bwd) / args.rk4_steps * 1e3,
                     "dtype": args.precision,
                     "config": {"workload": f"field-driven RK4, L={L} N={N0 - 1} D={D}, {args.rk4_steps} steps of {dt}, "
                                            f"checkpoints every {args.checkpoint}, E(t) = A sin(t) exp(-(t-2)^2/0.5), "
                                            f"A = {A}, {args.sweeps} sweep(s) per fit"},
                     "forward_s": t_fwd, "backward_s": t_bwd, "dipole": tr.value, "dD_dA": g,
                     "finite_difference": fd,
                     "rel_diff_vs_fd": None if fd is None or g is None else abs(g - fd) / max(abs(fd), 1e-300)})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
