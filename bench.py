"""Throughput of the LOS-dependent P0/P2/P4 estimator on one MI355X.

One step = the whole estimator (catalogue scalars, row sort, LOS-weighted assignment
fused with the x FFT, y FFT with z-power grouping, z FFT fused with the k-hat
contraction and shell binning, finalize) on one synthetic clustered RSD mock that is
already resident in HBM, ending with the FP64 P_l on the host.

Default workload: lognormal RSD mock, P(k) = 2e4 (k/0.1)^-1.5, 512^3 field, L = 2500
Mpc/h at 2000 Mpc/h, nbar = 3e-4 (~4.7e6 galaxies), Kaiser f = 0.75, b = 2, 20x randoms
(~9.4e7), FKP P0 = 1e4, CIC on 512^3, ell = 0, 2, 4, 128 bins of width 2 k_f.

Prints one JSON line (value = mocks per second of the 512^3 workload). The same run then
times the DESI-scale workload (lognormal RSD mock made on the GPU, 3e7 galaxies + 6e8
randoms, L = 4000 Mpc/h, TSC on 1024^3, 22 grids, 256 bins of 2 k_f), the other half of
the metric, reported under "grid_1024" with its own stage times and roofline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the dominant kernel per launch, keyed by (workload, kernel) and reported
# for that workload only, from two rocprofv3 --pmc runs of it (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch), each scaled by what the same
# counter reads for a plain copy of known size (--copy-calibration: FETCH_SIZE reads 0.50
# of the bytes read, WRITE_SIZE 1.00 of the bytes written). Valid only for the kernel
# source it was measured on: the sha256 of the files listed is checked at run time and
# the traffic is reported as null when any of them has changed since.
TRAFFIC_FILES = ["paper_1505_05341_amd/csrc/" + f for f in
                 ("stage_assign.hip", "particle.hpp", "fft_dev.hpp", "plan.hpp", "dft_consts.h", "basis.hpp",
                  "monomial_sums.hpp")]
TRAFFIC = {
    ("clustered_512", "assign_x"): {"sha256": "2e2fc29d24db20123f81de23de0fdbf2b682e02e97bd3e9d8add3a1285b46ccf",
                 "fetch_kib": 879365.0, "write_kib": 7864320.0, "fetch_scale": 2.0, "write_scale": 1.0},
    ("desi_1024", "assign_x"): {"sha256": "2e2fc29d24db20123f81de23de0fdbf2b682e02e97bd3e9d8add3a1285b46ccf",
                 "fetch_kib": 7751049.0, "write_kib": 66893824.0, "fetch_scale": 2.0, "write_scale": 1.0},
}


def source_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    t = TRAFFIC.get((workload, kernel))
    if not t or t["sha256"] is None or t["sha256"] != source_digest(TRAFFIC_FILES):
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size, for scaling the HBM byte counters."""
    import torch
    torch.cuda.set_device(0)
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def plan_bytes(cfg, n_gal, n_ran, slabs=False):
    """Algorithmic HBM bytes of each stage (each input byte read once, each output written
    once). With slabs the x and y transforms alternate and are timed as one stage."""
    N, dn, nbins, ell = cfg["N"], cfg["dn"], cfg["nbins"], cfg["ell_max"]
    K = nbins * dn
    TK = 4 if N >= 2048 else (8 if N >= 1024 else min(16, N // 2))
    Kx = -(-K // TK) * TK
    hstride = 0
    for kt in range(Kx // TK):
        M = math.isqrt(K * K - 1 - (kt * TK) ** 2)
        hstride += N * (2 * M + 1) * TK
    GK = {0: 1, 2: 6, 4: 15}[ell]   # stored x-transformed grids (power of rhat_z below 2)
    ngroups = {0: 1, 2: 4, 4: 9}[ell]
    X = GK * N * N * Kx * 8
    H = ngroups * hstride * 8
    Np = n_gal + n_ran
    out = {
        "scalars": 4 * n_gal + 8 * n_ran,
        "sort": 16 * Np + 16 * Np + 4 * (N * N + 1),
        "assign_x": 16 * Np + 4 * (N * N + 1) + X,
        "fft_y": X + H,
        "fft_z_bin": H,
    }
    if slabs:
        out["assign_x"] += out.pop("fft_y")
    return out


def make_workload(name, grid=2048):
    from paper_1505_05341_amd import catalogs
    if name == "clustered_512":
        gal, ran, cfg = catalogs.clustered_rsd_512()
        desc = ("lognormal RSD mock, 512^3 field, L=2500 Mpc/h at 2000 Mpc/h, nbar=3e-4, f=0.75, b=2, "
                "20x randoms, FKP P0=1e4; CIC 512^3, ell=0,2,4, 128 bins of 2 k_f")
    elif name == "desi_1024":
        gal, ran, cfg = catalogs.desi_scale_1024_device()
        desc = ("lognormal RSD mock made on the GPU, 1024^3 field, L=4000 Mpc/h at 3000 Mpc/h, nbar=4.69e-4, "
                "f=0.75, b=2, 20x randoms, FKP P0=1e4; TSC 1024^3, ell=0,2,4 (22 grids), 256 bins of 2 k_f")
    elif name == "survey":
        gal, ran, cfg = catalogs.survey_shell_device(N=grid)
        desc = ("survey-shaped stand-in for the paper's timing catalogue (Table 1): lognormal RSD mock made on "
                "the GPU (512^3 field), observed from the origin in a 3500 Mpc/h cube and cut to the shell "
                "1200-1800 Mpc/h inside a 48 deg cap (2.1 sr), ~525,000 galaxies + 10x randoms, FKP P0=1e4; "
                "CIC %d^3, ell=0,2,4, %d bins of 2 k_f" % (grid, grid // 4))
    elif name == "tiny_32":
        gal, ran, cfg = catalogs.tiny_plain()
        desc = "2000 uniform galaxies + 20000 randoms, 1000 Mpc/h cube at 1500 Mpc/h; CIC 32^3, ell=0,2,4"
    else:
        raise SystemExit("unknown workload %s" % name)
    return gal, ran, cfg, desc


def cpu_baseline(gal, ran, cfg, workers=16):
    """The FP64 oracle (oracle.estimator.pk_multipoles_lean, the form that fits a host at
    this grid) on a bounded sample of the same workload: its set-up (catalogue scalars,
    lines of sight, the binned half lattice) and the first of the 1, 7 or 22 grids (deposit
    of every particle, library FFT on `workers` threads, shell sums). Per mock = set-up +
    (number of grids) x (time of that grid); the other grids cost the same or more (their
    shell sums carry k-hat products)."""
    from oracle import estimator as est
    c = est.Config(**{k: v for k, v in cfg.items() if k != "x_planes"})
    marks = []
    t0 = time.perf_counter()
    est.pk_multipoles_lean(gal.pos, gal.w, ran.pos, ran.w, c, gal.nbar, ran.nbar, workers=workers,
                           log=lambda msg: marks.append(time.perf_counter()), max_grids=1)
    t_setup, t_grid = marks[0] - t0, marks[1] - marks[0]
    ngrid = len(est.los_monomials(c.ell_max))
    per_mock = t_setup + ngrid * t_grid
    return {"value": 1.0 / per_mock, "unit": "mocks/s", "cores": workers, "kind": "oracle",
            "sample": ("oracle.estimator.pk_multipoles_lean on the same %d particles, set-up (scalars, lines of "
                       "sight, binned half lattice of %d^3) %.1f s + the first of %d grids (FP64 deposit, library "
                       "FFT on %d threads, shell sums) %.1f s; per mock = set-up + %d x grid = %.0f s"
                       % (gal.n + ran.n, c.N, t_setup, ngrid, workers, t_grid, ngrid, per_mock)),
            "measured_s": marks[1] - t0}


def batch_workload(n_mocks, seed=4000):
    """Uneven ensemble: N_gal log-uniform in [2e5, 2e6], randoms 10-20x, L uniform in
    [1000, 2500] Mpc/h centred 0.8 L from the observer, grid 256^3 or 512^3 (nearest to
    L / 4.88), CIC, ell = 0, 2, 4, bins of width 2 k_f. Mocks are made on the GPU."""
    from paper_1505_05341_amd import catalogs
    rng = np.random.default_rng(seed)
    gals, rans, cfgs = [], [], []
    for i in range(n_mocks):
        ng = 10 ** rng.uniform(math.log10(2e5), math.log10(2e6))
        xr = int(rng.integers(10, 21))
        L = float(rng.uniform(1000.0, 2500.0))
        N = 256 if L / 4.88 < 384 else 512
        g, r, box_min = catalogs.lognormal_rsd_device(N_field=256, L=L, center=(0.0, 0.0, 0.8 * L),
                                                      nbar=ng / L ** 3, seed=seed * 1000 + i, ran_factor=xr)
        gals.append(g)
        rans.append(r)
        cfgs.append(catalogs.config_dict(N, box_min, L, assign=2, dn=2))
    return gals, rans, cfgs


def run_batch(args):
    import torch
    import paper_1505_05341_amd as pk
    torch.cuda.set_device(0)
    t = time.perf_counter()
    gals, rans, cfgs = batch_workload(args.mocks)
    torch.cuda.synchronize()
    npart = sum(g.n + r.n for g, r in zip(gals, rans))
    log("generated %d mocks (%d particles) on the GPU in %.1f s" % (len(cfgs), npart, time.perf_counter() - t))
    ws = pk.Workspace()
    res, st = pk.pk_multipoles_batch(gals, rans, cfgs, lanes=args.lanes, workspace=ws)   # warm-up
    assert all(x == 0 for x in st), st
    times = []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, st = pk.pk_multipoles_batch(gals, rans, cfgs, lanes=args.lanes, workspace=ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log("batch pass %d: %.3f s" % (k, times[-1]))
    seq = []
    ws1 = pk.Workspace()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, r, c in zip(gals, rans, cfgs):
        seq.append(pk.pk_multipoles(g, r, c, ws1))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    worst = 0.0
    for a, b in zip(res, seq):
        ok = b["nmodes"] > 0
        raw = np.abs(b["P0"][ok]) + b["noise"][ok]
        for l in (0, 2, 4):
            worst = max(worst, float(np.max(np.abs(a["P%d" % l][ok] - b["P%d" % l][ok]) / raw)))
    best = min(times)
    # host cost per mock of the batch (graph capture, update, launch): the same call on tiny
    # mocks (32^3, 3,000 particles), whose kernels take a few microseconds each
    from paper_1505_05341_amd import catalogs
    tg, tr, tc = catalogs.tiny_plain(n_gal=300, n_ran=3000)
    tg, tr = pk.DeviceCatalog.from_host(tg), pk.DeviceCatalog.from_host(tr)
    ntiny = 256
    pk.pk_multipoles_batch([tg] * ntiny, [tr] * ntiny, [tc] * ntiny, lanes=args.lanes, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pk.pk_multipoles_batch([tg] * ntiny, [tr] * ntiny, [tc] * ntiny, lanes=args.lanes, workspace=ws)
    torch.cuda.synchronize()
    host_ms = 1e3 * (time.perf_counter() - t0) / ntiny
    t0 = time.perf_counter()
    for _ in range(ntiny):
        pk.pk_multipoles(tg, tr, tc, ws1)
    torch.cuda.synchronize()
    single_tiny_ms = 1e3 * (time.perf_counter() - t0) / ntiny
    log("tiny mocks: %.3f ms per mock in a batch, %.3f ms per single call" % (host_ms, single_tiny_ms))
    out = {"metric": "P0/P2/P4 mocks/sec, batched ensemble", "value": len(cfgs) / best, "unit": "mocks/s",
           "n_gpus": 1, "steps": args.steps, "ms_per_batch": best * 1e3, "mocks": len(cfgs),
           "lanes": args.lanes, "sequential_mocks_per_s": len(cfgs) / t_seq,
           "batch_vs_sequential_max_rel_diff": worst, "particles": npart, "dtype": "f32", "data": "synthetic",
           "tiny_mock_ms_per_mock_batched": host_ms, "tiny_mock_ms_per_single_call": single_tiny_ms,
           "config": {"workload": batch_workload.__doc__.split("\n")[0].strip()}}
    print(json.dumps(out), flush=True)


def run_correction(args):
    """Learned coarse-grid correction, end to end: method-generated pairs (each lognormal
    RSD mock measured on the coarse and the fine grid by the estimator itself), training
    on the GPU, held-out error against the fine grid, and the throughput of coarse grid +
    network against the plain fine-grid estimator on the same device-resident mocks."""
    import torch
    import paper_1505_05341_amd as pk
    from paper_1505_05341_amd import catalogs, correction
    torch.cuda.set_device(0)
    geo = dict(L=2500.0, center=(0.0, 0.0, 2000.0), N_coarse=args.coarse, N_fine=args.fine, N_field=args.field,
               nbar_range=(1e-4, 1e-3), ran_factor=10.0)
    ntest = max(4, args.mocks // 8)
    t = time.perf_counter()
    train = correction.make_pairs(args.mocks - ntest, seed0=5000, log=log, **geo)
    test = correction.make_pairs(ntest, seed0=90000, log=log, **geo)
    t_pairs = time.perf_counter() - t
    log("pairs: %d train + %d test mocks in %.1f s" % (args.mocks - ntest, ntest, t_pairs))
    model = correction.Correction(seed=0)
    t = time.perf_counter()
    hist = model.fit(train["X"], train["Y"], train["domain"], epochs=args.epochs, batch=1024, lr=2e-3, log=log)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t
    err = correction.errors_vs_fine(test["meta"], model.predict(test["X"]))
    log("held-out |P - P_fine| / R:", json.dumps(err))
    # throughput on device-resident mocks: coarse + network vs plain fine grid
    mocks = []
    rng = np.random.default_rng(77)
    for i in range(args.timing_mocks):
        nbar = float(10 ** rng.uniform(-4, -3))
        g, r, box_min = catalogs.lognormal_rsd_device(N_field=args.field, L=geo["L"], center=geo["center"], nbar=nbar,
                                                      seed=123000 + i, ran_factor=geo["ran_factor"])
        mocks.append((g, r, box_min, nbar))
    ws = pk.Workspace()
    cc0, cf0 = correction.coarse_fine_configs(mocks[0][2], geo["L"], args.coarse, args.fine)
    for g, r, box_min, nbar in mocks[:1]:   # warm-up of both paths
        model.measure(g, r, box_min, nbar, ws)
        pk.pk_multipoles(g, r, dict(cf0, box_min=box_min), ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for g, r, box_min, nbar in mocks:
        out, how = model.measure(g, r, box_min, nbar, ws)
        assert how == "corrected"
    torch.cuda.synchronize()
    t_cor = (time.perf_counter() - t) / len(mocks)
    t = time.perf_counter()
    for g, r, box_min, nbar in mocks:
        pk.pk_multipoles(g, r, dict(cf0, box_min=box_min), ws)
    torch.cuda.synchronize()
    t_fine = (time.perf_counter() - t) / len(mocks)
    out = {"metric": "learned coarse-grid correction: held-out error vs the fine grid and throughput",
           "coarse_grid": args.coarse, "fine_grid": args.fine, "field_grid": args.field,
           "train_mocks": args.mocks - ntest, "test_mocks": ntest, "train_rows": int(train["X"].shape[0]),
           "epochs": args.epochs, "loss_first_last": [hist[0], hist[-1]],
           "held_out_error_over_raw_power": err,
           "corrected_mocks_per_s": 1.0 / t_cor, "fine_grid_mocks_per_s": 1.0 / t_fine,
           "speedup_vs_fine": t_fine / t_cor, "pair_generation_s": t_pairs, "training_s": t_fit,
           "data": "synthetic lognormal RSD mocks made on the GPU, L=2500 Mpc/h at 2000 Mpc/h, nbar 1e-4..1e-3, "
                   "10x randoms, CIC, ell=0,2,4, bins of 1 k_f up to the coarse Nyquist"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="clustered_512",
                    help="clustered_512 (default), desi_1024, survey (with --grid), tiny_32, batch, correction")
    ap.add_argument("--grid", type=int, default=2048, help="grid of --workload survey (512, 1024 or 2048)")
    ap.add_argument("--x-planes", type=int, default=0,
                    help="planes per slab of the x and y transforms (0 = the library's automatic choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-1024", action="store_true",
                    help="time only the 512^3 workload (by default the DESI-scale 1024^3 TSC workload follows)")
    ap.add_argument("--mocks", type=int, default=256, help="ensemble size for --workload batch")
    ap.add_argument("--lanes", type=int, default=2, help="concurrent lanes for --workload batch")
    ap.add_argument("--coarse", type=int, default=256, help="coarse grid of --workload correction")
    ap.add_argument("--fine", type=int, default=1024, help="fine grid of --workload correction")
    ap.add_argument("--field", type=int, default=512, help="lognormal field grid of --workload correction")
    ap.add_argument("--epochs", type=int, default=80, help="training epochs of --workload correction")
    ap.add_argument("--timing-mocks", type=int, default=8, help="mocks timed by --workload correction")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default column-transform schedules instead of autotuning them first")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "correction":
        run_correction(args)
        return

    import torch
    out = time_workload(args.workload, args, args.grid, with_cpu=not args.no_cpu_baseline)
    if args.workload == "clustered_512" and not args.no_1024:
        # the other half of the metric: the DESI-scale 1024^3 TSC workload in the same run
        torch.cuda.empty_cache()
        second = time_workload("desi_1024", args, args.grid, with_cpu=False)
        second.pop("metric", None)
        for k in ("n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline", "dtype", "data",
                  "cpu_baseline", "h2d_GBps"):
            second.pop(k, None)
        out["grid_1024"] = second
    print(json.dumps(out), flush=True)


def time_workload(name, args, grid, with_cpu):
    """Generates one workload, times args.steps whole-estimator steps after args.warmup
    untimed ones, and returns the JSON record (stage times from HIP events on the launch
    stream, roofline of the dominant kernel)."""
    import torch
    import paper_1505_05341_amd as pk
    from paper_1505_05341_amd import native

    log("generating workload", name)
    t = time.perf_counter()
    gal, ran, cfg, desc = make_workload(name, grid)
    if args.x_planes:
        cfg = dict(cfg, x_planes=args.x_planes)
    log("generated %d galaxies + %d randoms in %.1f s" % (gal.n, ran.n, time.perf_counter() - t))
    torch.cuda.set_device(0)
    torch.cuda.synchronize()
    on_device = isinstance(gal, pk.DeviceCatalog)
    t = time.perf_counter()
    g = gal if on_device else pk.DeviceCatalog.from_host(gal)
    r = ran if on_device else pk.DeviceCatalog.from_host(ran)
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t
    h2d_bytes = 0 if on_device else 20 * (gal.n + ran.n)
    ws = pk.Workspace()
    xs = native.x_planes(cfg, gal.n, ran.n)
    log("workspace %.2f GB, x/y slab of %d planes" % (native.workspace_size(cfg, gal.n, ran.n) / 1e9, xs))

    schedule = native.get_schedule(cfg["N"], cfg["ell_max"])
    if not args.no_autotune:
        t = time.perf_counter()
        schedule = pk.autotune(g, r, cfg, reps=3, workspace=ws)
        log("autotuned column schedules (y, z values per thread): %s in %.2f s" % (schedule, time.perf_counter() - t))
    for i in range(args.warmup):
        pk.pk_multipoles(g, r, cfg, ws)
        log("warmup", i)
    native.set_stage_timing(True)
    stage_sum = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = pk.pk_multipoles(g, r, cfg, ws)
        for k, v in native.stage_times().items():
            stage_sum[k] = stage_sum.get(k, 0.0) + v
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    native.set_stage_timing(False)
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    stage_ms = {k: v / args.steps for k, v in stage_sum.items()}
    log("stage ms", json.dumps({k: round(v, 3) for k, v in stage_ms.items()}))
    slabs = xs < cfg["N"]
    byts = plan_bytes(cfg, gal.n, ran.n, slabs)
    if slabs:   # one stage covers the x and y transforms of every slab
        stage_ms.pop("fft_y", None)
    dom = max((k for k in byts), key=lambda k: stage_ms.get(k, 0.0))
    achieved = byts[dom] / (stage_ms[dom] * 1e-3) / 1e9
    stage_gbs = {k: round(byts[k] / (stage_ms[k] * 1e-3) / 1e9, 1) for k in byts if stage_ms.get(k, 0) > 0}
    log("stage GB/s", json.dumps(stage_gbs))
    value = 1e3 / ms_per_step
    P_check = {"P0_bin1": res["P0"][1], "P2_bin1": res["P2"][1], "P4_bin1": res["P4"][1]}
    del g, r, ws, res
    torch.cuda.empty_cache()

    cpu = None
    if with_cpu and not on_device:
        log("timing the FP64 oracle on a bounded sample")
        cpu = cpu_baseline(gal, ran, cfg)
        log("oracle sample took %.1f s" % cpu.pop("measured_s"))

    out = {
        "metric": "P0/P2/P4 mocks/sec at 512^3 and 1024^3 grid; achieved HBM GB/s vs peak",
        "value": value,
        "unit": "mocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "grid": cfg["N"], "n_gal": gal.n, "n_ran": ran.n,
                   "ell_max": cfg["ell_max"], "assign": "CIC" if cfg["assign"] == 2 else "TSC",
                   "nbins": cfg["nbins"], "dn": cfg["dn"], "x_planes": xs,
                   "fft_schedule": {"y_values_per_thread": schedule[0], "z_values_per_thread": schedule[1]}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None if slabs else measured_traffic(name, dom),
                     "kernel": dom + (" + fft_y (slabs)" if slabs else ""),
                     "kernel_ms": stage_ms[dom], "algorithmic_bytes": byts[dom]},
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "stages_GBps": stage_gbs,
        "h2d_GBps": (h2d_bytes / h2d_s / 1e9) if h2d_bytes else None,
        "cpu_baseline": cpu,
        "P_check": P_check,
    }
    if name == "survey":
        out["metric"] = "P0/P2/P4 mocks/sec, survey-shaped catalogue of the paper's timing table"
        paper_min = {512: 1.2, 1024: 7.5, 2048: 72.5}.get(cfg["N"])
        out["paper_table1"] = None if paper_min is None else {
            "minutes_per_mock": paper_min, "hardware": "16 processors (CPU model not given)",
            "workload": "one BOSS DR11 CMASS NGC mock, ~525,000 galaxies, 10x randoms, L_b = 3500 Mpc/h, CIC"}
    return out


if __name__ == "__main__":
    main()
