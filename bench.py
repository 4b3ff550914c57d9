#!/usr/bin/env python
"""Benchmark of the data-space Hessian build and inversion on one MI355X.

One step = one survey through the whole hot path with inputs resident in HBM:
Green functions by FD with the on-the-fly DFT, Hessian contraction, penalty +
Cholesky, and the multi-source deblur of all sources at all frequencies.

Default workload: layered 1000 x 300 grid (h = 10 m, 40-cell sponge),
200 receivers, nt = 4000 at 0.8 ms, 30 frequencies over 3-15 Hz, 200 sources,
split-BF16 precision form.

Prints one JSON line (see the repository's benchmark contract).
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Hessian build+factor s/survey; multiplier solves/s; % HBM/MFMA roofline"
HBM_PEAK_GBS = 8000.0

# HBM bytes per marching launch measured with rocprofv3 (FETCH_SIZE x 2 +
# WRITE_SIZE x 1 KiB, scales from a 1 GiB copy), keyed by (workload,
# precision, time levels, segment rows, band width, receivers per launch); recorded in
# profiles/survey_layered-1000x300_pmc.md.  Any other shape reports null.
TRAFFIC_SOURCE = ("not measured in this run: the counters of a separate rocprofv3 --pmc collection of "
                  "the same launch shape, profiles/survey_layered-1000x300_pmc.md")
MEASURED_TRAFFIC = {
    ("layered-1000x300-nr200-nt4000-nf30-ns200", "split_bf16", 8, 256, 256, 200): (417482.5 * 2 + 1150948.6) * 1024,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="layered_1000x300",
                    help="layered_1000x300 (default), tiny, batch8 (the eight uneven surveys), serve "
                         "(Poisson request mix over the eight surveys), accuracy (the Hessian "
                         "accuracy test on the 1000 x 300 survey), randomized (one receiver per "
                         "subset, factors reused over iterations, on the 1000 x 300 survey), "
                         "deblur (the multi-source solve alone, by size), compare (both precision "
                         "forms on one workspace) or hbm_probe (streaming rates by access mix)")
    ap.add_argument("--batch-nt", type=int, default=4000, help="time steps of the batch8 surveys")
    ap.add_argument("--deblur-sizes", default="16x16,64x64,128x128,200x200,256x256,300x300,400x400,200x2000",
                    help="deblur: receivers x sources per size (comma separated)")
    ap.add_argument("--staging-gb", type=float, default=32.0,
                    help="batch8: staging budget per survey (sets the receivers stepped together)")
    ap.add_argument("--batch-chunk", type=int, default=512, choices=[256, 512, 1024],
                    help="batch8: time samples per staging window (the spectra are read and written "
                         "once per window: 512 samples with 32 GB per survey measured 4-6 %% faster "
                         "than 256 samples with every receiver at once, or 1024 with fewer)")
    ap.add_argument("--precision", default="split_bf16", choices=["split_bf16", "plain_fp32"])
    ap.add_argument("--weighting", default="long_record", choices=["long_record", "finite_record"],
                    help="Fourier-diagonal weighting: final-spectrum Gram (default) or the finite-record W")
    ap.add_argument("--decim", type=int, default=1,
                    help="finite-record weighting: keep every D-th low-pass filtered sample of the record")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: mean arrivals per second")
    ap.add_argument("--p-build", type=float, default=0.02, help="serve: probability a request is a build")
    ap.add_argument("--duration", type=float, default=120.0, help="serve: seconds of arrivals")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: HBM budget")
    ap.add_argument("--build-slots", type=int, default=2, help="serve: concurrent builds")
    ap.add_argument("--nr-batch", type=int, default=0)
    ap.add_argument("--acc-ns", type=int, default=16, help="accuracy: sources per step")
    ap.add_argument("--cg-iters", type=int, default=60, help="accuracy: cap on the CG baseline's iterations")
    ap.add_argument("--chunk", type=int, default=1024, choices=[256, 512, 1024],
                    help="time samples per DFT staging window")
    ap.add_argument("--windows", type=int, default=2, choices=[1, 2],
                    help="staging windows (2, the default: the DFT of one window runs on a second "
                         "stream beside the stepping of the next, 5-6 %% faster per survey for twice "
                         "the staging memory; 1: one window, DFT after stepping)")
    ap.add_argument("--keep", type=int, nargs=2, default=[0, 0], metavar=("KZ", "KX"),
                    help="contract the leading KZ x KX 2D DCT-II coefficients of the subgrid "
                         "instead of the grid points (0 0: no transform)")
    ap.add_argument("--subsets", type=int, default=100, help="randomized: receiver subsets (receivers kept)")
    ap.add_argument("--reuse", type=int, default=5, help="randomized: iterations per selection")
    ap.add_argument("--iters", type=int, default=20, help="randomized: timed iterations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-receivers", type=int, default=64,
                    help="Green functions in the CPU sample (each over the whole record; all of them "
                         "makes the sample the oracle's whole survey, multipliers compared too)")
    ap.add_argument("--cpu-hessians", type=int, default=3, help="full-size Hessians in the CPU sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (a known-size kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def _errors(a, b, rows=False):
    """Per frequency (axis 0): relative Frobenius error of a against b, the
    largest element-wise difference against b's largest entry, and (rows) the
    same per row of axis 1 against that row's largest entry."""
    fr, el, rw = [], [], []
    for f in range(b.shape[0]):
        d = (a[f] - b[f]).reshape(b.shape[1], -1)
        r = b[f].reshape(b.shape[1], -1)
        fr.append(float(np.linalg.norm(d) / np.linalg.norm(r)))
        el.append(float(np.abs(d).max() / np.abs(r).max()))
        if rows:
            rw.append(float((np.abs(d).max(axis=1) / np.abs(r).max(axis=1)).max()))
    out = {"frob": [float(f"{x:.3e}") for x in fr], "elem": [float(f"{x:.3e}") for x in el]}
    if rows:
        out["row"] = [float(f"{x:.3e}") for x in rw]
    return out


def cpu_baseline(s, n_hess=3, fd_receivers=32, gpu=None):
    """Time the FP64 oracle on a bounded sample of the survey and scale it to one
    survey, stage by stage, each on all the host threads it can use; compare the
    sample's results with the GPU's.

    FD + DFT: the oracle's C recurrence (OpenMP over grid rows, all receivers of
    the sample stepped together) with the DFT taken window by window as BLAS
    matrix products, for ``fd_receivers`` Green functions spread over the line
    and the whole record (nt steps) on the full grid, scaled to nr receivers
    (the cost is linear in them).  Hessian: the FP64 contraction of ``n_hess``
    frequencies (multithreaded BLAS) from seeded spectra, scaled to nf.
    Cholesky and the multi-source solve: all frequencies at full size.  With
    every receiver in the sample the stages are the oracle's whole survey
    (its own Hessians of every frequency, no scaling).

    ``gpu`` (optional): the GPU run's spectra rows of the sampled receivers
    ("G", [nf][k][nsub]), its Hessian ("H"), multipliers ("X"), residuals ("R")
    and mu.  The returned "parity" holds per-frequency errors of the spectra
    and of the sampled receivers' Hessian block against the oracle's, and,
    with every receiver sampled, of all multipliers.
    """
    from oracle import fd, hessian, solve
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        blas_threads = os.cpu_count() or 1
    fd_threads = fd.c_threads()
    v = s.velocity()
    nrs = max(1, min(int(fd_receivers), s.nr))
    idx = sample_receivers(s.nr, nrs)
    full = nrs == s.nr
    t0 = time.perf_counter()
    G = fd.green_dft_windowed(v, s.nb, s.h, s.dt, s.nt, [s.rec_iz[i] for i in idx],
                              [s.rec_ix[i] for i in idx], s.freqs_hz, s.stride)
    t_fd = time.perf_counter() - t0
    if full:
        t0 = time.perf_counter()
        H = hessian.hessian_r1(G)
        t_h = (time.perf_counter() - t0) / s.nf
        n_hess = s.nf
    else:
        # n_hess frequencies' Hessians at full size from seeded spectra
        n_hess = max(1, min(int(n_hess), s.nf))
        rng = np.random.default_rng(0)
        Gs = rng.standard_normal((n_hess, s.nr, s.nsub)) + 1j * rng.standard_normal((n_hess, s.nr, s.nsub))
        t0 = time.perf_counter()
        H1 = hessian.hessian_r1(Gs)[:1]
        t_h = (time.perf_counter() - t0) / n_hess
        del Gs
        H = np.repeat(H1, s.nf, axis=0)
    R = s.residuals().astype(np.complex128)
    mu = gpu["mu"] if gpu is not None else 1e-3 * float(np.real(H[0].trace()))
    t0 = time.perf_counter()
    L = solve.cholesky(solve.penalize(H, mu))
    t_c = time.perf_counter() - t0
    t0 = time.perf_counter()
    Xo = solve.solve(L, R)
    t_s = time.perf_counter() - t0
    fd_survey = t_fd * (s.nr / nrs)
    survey_s = fd_survey + t_h * s.nf + t_c
    what = (f"whole survey: all {s.nr} Green functions x {s.nt} steps" if full else
            f"{nrs} of {s.nr} Green functions (spread over the line) x {s.nt} steps")
    out = {
        "value": survey_s,
        "unit": "s/survey",
        "cores": int(max(fd_threads, blas_threads)),
        "kind": "oracle",
        "sample": (f"FP64 oracle, {what} of FD+DFT on the full grid ({t_fd:.2f} s, C recurrence on "
                   f"{fd_threads} OpenMP threads, DFT by BLAS on {blas_threads} threads), {n_hess} of "
                   f"{s.nf} Hessians at full size ({t_h * n_hess:.2f} s, BLAS on {blas_threads} threads), "
                   f"all {s.nf} Cholesky factorisations ({t_c:.2f} s)"
                   + ("" if full else f"; scaled to {s.nr} Green functions and {s.nf} Hessians")
                   + f". Multi-source solve {t_s:.3f} s ({s.nf * s.ns / t_s:.0f} solves/s)"),
        "stages": {
            "fd_dft": {"s_per_survey": round(fd_survey, 2), "threads": int(fd_threads),
                       "sampled_s": round(t_fd, 3)},
            "hessian": {"s_per_survey": round(t_h * s.nf, 3), "threads": int(blas_threads)},
            "cholesky": {"s_per_survey": round(t_c, 4), "threads": int(blas_threads)},
            "solve": {"s": round(t_s, 4), "threads": int(blas_threads)},
        },
        "solves_per_s": s.nf * s.ns / t_s,
    }
    if gpu is not None:
        Hb = np.stack([G[f] @ G[f].conj().T for f in range(s.nf)])     # the sampled block
        Hg = gpu["H"][:, idx][:, :, idx]
        par = {"scope": (f"all {s.nr} receivers" if full else
                         f"receivers {idx[0]}, {idx[1]}, ..., {idx[-1]} ({nrs} of {s.nr})"),
               "ghat": _errors(gpu["G"], G, rows=True),
               "hhat": _errors(Hg, Hb, rows=True)}
        if full:
            par["x"] = _errors(gpu["X"], Xo, rows=True)
        out["parity"] = par
    return out


def sample_receivers(nr, k):
    """k receiver indices spread evenly over 0..nr-1 (both ends included)."""
    if k >= nr:
        return list(range(nr))
    return sorted({int(round(i * (nr - 1) / max(k - 1, 1))) for i in range(k)})


def run_batch(args):
    """Eight uneven layered surveys: graph-captured builds on per-survey streams,
    one batched factorisation launch, per-survey deblurs of all their sources."""
    import numpy as np
    import torch

    import synth
    from paper_2512_16642_amd import batch, costs

    specs = synth.batch_surveys(nt=args.batch_nt)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    vels = [torch.from_numpy(s.velocity()).to(dev) for s in specs]
    Rs = [torch.from_numpy(s.residuals()).to(dev) for s in specs]
    b = batch.SurveyBatch(specs, precision=args.precision, tune=True,
                          staging_budget_bytes=int(args.staging_gb * (1 << 30)), chunk=args.batch_chunk)
    print(f"# batch8: workspaces {b.workspace_bytes / 1e9:.1f} GB, receivers per batch "
          f"{[sv.nr_batch for sv in b.surveys]}, launch shapes tuned", file=sys.stderr, flush=True)
    b.build(vels, graph=True)
    mu = [1e-3 * l for l in b.lambda_max()]
    for _ in range(args.warmup):
        b.build(vels, graph=True)
        b.factor(mu)
        b.apply(Rs)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    tb = tf = ta = 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(stream)
        b.build(vels, graph=True)
        e[1].record(stream)
        b.factor(mu)            # one launch; waits for its status
        e[2].record(stream)
        b.apply(Rs)
        e[3].record(stream)
        e[3].synchronize()
        tb += e[0].elapsed_time(e[1])
        tf += e[1].elapsed_time(e[2])
        ta += e[2].elapsed_time(e[3])
        print(f"# batch step {k} done", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    K = args.steps
    solves = sum(s.nf * s.ns for s in specs)
    cells = sum(costs.stencil_cell_updates_per_survey(s.nz, s.nx, s.nb, s.nr, s.nt) for s in specs)
    out = {
        "metric": "batched uneven surveys: build+factor s per 8-survey batch; multiplier solves/s",
        "value": round((tb + tf) / K / 1e3, 4),
        "unit": "s/batch",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall / K * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch8-layered-uneven", "precision": args.precision, "nt": args.batch_nt,
                   "surveys": [s.name for s in specs], "staging_gb": args.staging_gb,
                   "chunk": args.batch_chunk, "nr_batch": [sv.nr_batch for sv in b.surveys]},
        "workspace_gb": round(b.workspace_bytes / 1e9, 2),
        "stage_ms": {"build_graph": round(tb / K, 2), "factor_batched": round(tf / K, 3),
                     "apply": round(ta / K, 3)},
        "surveys_per_s": round(len(specs) / ((tb + tf) / K / 1e3), 3),
        "solves_per_s": round(solves / (ta / K / 1e3), 1),
        "gcell_updates_per_s": round(cells / (tb / K / 1e3) / 1e9, 1),
    }
    b.close()
    print(json.dumps(out), flush=True)


def run_compare(args):
    """The chosen (split-BF16) and the plain FP32 form on one and the same
    workspace allocation, built in turn in one process, so that both see the
    same physical placement: survey time and multiplier solves/s of each."""
    import torch

    import synth
    from paper_2512_16642_amd import ehi

    s = synth.WORKLOADS["layered_1000x300"]()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    vel = torch.from_numpy(s.velocity()).to(dev)
    R = torch.from_numpy(s.residuals()).to(dev)
    X = torch.empty_like(R)
    kw = dict(max_ns=s.ns, chunk=args.chunk, windows=args.windows)
    need = max(ehi.workspace_bytes(nz=s.nz, nx=s.nx, nb=s.nb, h=s.h, dt=s.dt, nt=s.nt, stride=s.stride,
                                   rec_iz=s.rec_iz, rec_ix=s.rec_ix, freqs_hz=s.freqs_hz, precision=p,
                                   nr_batch=0, **kw)
               for p in ("split_bf16", "plain_fp32"))
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    res = {}
    mu = None
    for prec in ("split_bf16", "plain_fp32", "split_bf16"):
        sv = ehi.survey_from(s, precision=prec, workspace=ws, **kw)
        sv.build_green(vel)
        sv.build_hessian()
        if mu is None:
            mu = 1e-3 * sv.lambda_max()
        sv.factor(mu)
        sv.apply_multipliers(R, out=X)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        tb = ta = 0.0
        sv.read_profile()
        sv.profile(True)
        for _ in range(args.steps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(st)
            sv.build_green(vel)
            sv.build_hessian()
            sv.factor(mu)
            e[1].record(st)
            sv.apply_multipliers(R, out=X)
            e[2].record(st)
            e[2].synchronize()
            tb += e[0].elapsed_time(e[1])
            ta += e[1].elapsed_time(e[2])
        sv.profile(False)
        prof = sv.read_profile()
        sv.close()
        key = prec if prec not in res else prec + "_again"
        res[key] = {"s_per_survey": round(tb / args.steps / 1e3, 5),
                    "solves_per_s": round(s.nf * s.ns / (ta / args.steps / 1e3), 1),
                    "kernel_ms": {k: round(v[0] / args.steps, 3) for k, v in prof.items()}}
        print(f"# {key}: {res[key]}", file=sys.stderr, flush=True)
    out = {"metric": "chosen vs plain FP32 form on one workspace: s/survey and multiplier solves/s",
           "value": res["split_bf16"]["s_per_survey"], "unit": "s/survey", "n_gpus": 1, "steps": args.steps,
           "warmup": 1, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": s.name, "chunk": args.chunk, "windows": args.windows},
           "forms": res}
    print(json.dumps(out), flush=True)


def run_hbm_probe(args):
    """The HBM rate plain streaming kernels reach for the access mixes of the
    hot kernels (1 GiB per array): the practical ceiling for the stepping
    kernel's mix (two planes read; two planes and the staged samples written)
    and for the DFT's (reads)."""
    import torch

    from paper_2512_16642_amd import ehi

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    nbytes = 1 << 30
    # the stepping kernel's launch per cell: u, w read and written (16 B) and
    # 8 staged samples on the stride-2 subgrid (8 x 4 B x 75,000 / 410,400 =
    # 5.85 B, 1.46 planes of 4 B)
    efrac = 1.462
    bufs = [torch.zeros(nbytes, dtype=torch.uint8, device=dev) for _ in range(4)]
    bufs.append(torch.zeros(int(nbytes * 2), dtype=torch.uint8, device=dev))
    grids = (2048, 4096, 8192, 16384)
    sink = torch.zeros(max(grids) * 256 * 16, dtype=torch.uint8, device=dev)
    mixes = {0: ("copy: 1 read + 1 write", 2.0), 1: ("read", 1.0), 2: ("2 reads + 2 writes", 4.0),
             3: (f"2 reads + {2 + efrac:.3f} writes (the stepping kernel's mix)", 4.0 + efrac),
             4: ("2 reads", 2.0)}
    st = torch.cuda.current_stream()
    res = {}
    for mode, (label, mult) in mixes.items():
        best = 0.0
        per = {}
        for gsz in grids:
            for _ in range(3):
                ehi.hbm_probe(mode, *bufs, e_frac=efrac, grid=gsz, sink=sink)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(20):
                ehi.hbm_probe(mode, *bufs, e_frac=efrac, grid=gsz, sink=sink)
            e1.record(st)
            e1.synchronize()
            tbs = mult * nbytes / (e0.elapsed_time(e1) / 20 / 1e3) / 1e12
            per[gsz] = round(tbs, 3)
            best = max(best, tbs)
        res[label] = {"best_tb_s": round(best, 3), "by_grid": per}
        print(f"# {label}: {per}", file=sys.stderr, flush=True)
    out = {"metric": "HBM rate of plain streaming kernels by access mix", "value": res[mixes[3][0]]["best_tb_s"],
           "unit": "TB/s", "n_gpus": 1, "steps": 20, "warmup": 3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "hbm-probe-1GiB-arrays"}, "mixes": res, "peak_tb_s": HBM_PEAK_GBS / 1e3}
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Serving mix: Poisson arrivals (mean args.rate req/s, rng 2400) of rebuilds
    of the eight uneven surveys (probability args.p_build) and deblurs of
    U{1..256} sources x all frequencies against resident factors, all eight
    surveys resident at the start, HBM budget args.budget_gb."""
    import torch

    import synth
    from paper_2512_16642_amd import serve

    specs = synth.batch_surveys(nt=args.batch_nt)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    eng = serve.EhiEngine(specs, build_slots=args.build_slots, precision=args.precision, tune=True)
    srv = serve.Server(eng, budget_bytes=int(args.budget_gb * 1e9), build_slots=args.build_slots)
    t0 = time.perf_counter()
    srv.preload(range(len(specs)))
    print(f"# serve: {len(specs)} surveys resident in {time.perf_counter() - t0:.1f} s, "
          f"{srv.adm.used / 1e9:.1f} GB of {args.budget_gb:.0f} GB", file=sys.stderr, flush=True)
    # warm the deblur path of every survey (first-launch costs)
    warm = [serve.Request(-1 - k, "deblur", 0.0, k, ns=8, seed=k) for k in range(len(specs))]
    srv.run(warm)
    reqs = serve.poisson_requests(args.duration, args.rate, args.p_build, len(specs), ns_max=256, seed=2400)
    print(f"# serve: {len(reqs)} requests over {args.duration:.0f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    def report(t):
        done = sum(1 for r in reqs if r.status != "pending")
        print(f"# serve t={t:.0f}s: {done}/{len(reqs)} finished, {srv.adm.used / 1e9:.1f} GB held",
              file=sys.stderr, flush=True)

    srv.run(reqs, progress=report)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = serve.latency_stats(reqs)
    solves = sum(specs[r.key].nf * r.ns for r in reqs if r.kind == "deblur" and r.status == "done")
    builds = sum(1 for r in reqs if r.kind == "build" and r.status == "done")
    out = {
        "metric": "serving mix: multiplier solves/s with p50/p99 latency",
        "value": round(solves / wall, 1),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": len(warm),
        "ms_per_step": round(wall / max(1, len(reqs)) * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serve-poisson-batch8", "rate_hz": args.rate, "p_build": args.p_build,
                   "duration_s": args.duration, "budget_gb": args.budget_gb,
                   "build_slots": args.build_slots, "precision": args.precision, "nt": args.batch_nt},
        "latency": st,
        "builds_per_s": round(builds / wall, 3),
        "wall_s": round(wall, 2),
        "hbm_peak_gb": round(srv.adm.peak / 1e9, 1),
        "evictions": srv.evictions,
    }
    srv.close()
    print(json.dumps(out), flush=True)


def run_randomized(args):
    """Randomized receivers with Hessian reuse on the 1000 x 300 survey: every
    selection keeps one receiver drawn from each of ``--subsets`` contiguous
    subsets, is built (Green functions, contraction, lambda_max, factor) once
    and serves ``--reuse`` consecutive iterations; each iteration deblurs all
    sources at all frequencies against the resident factors.  Reports seconds
    per iteration (builds amortised), next to the build and reused-deblur times."""
    import torch

    import synth
    from paper_2512_16642_amd import randomized

    s = synth.layered_1000x300()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    vel = torch.from_numpy(s.velocity()).to(dev)
    R = torch.from_numpy(s.residuals()).to(dev)
    rh = randomized.RandomizedHessian(s, args.subsets, reuse=args.reuse, seed=2024, max_ns=s.ns)
    for it in range(args.reuse):  # warm-up: one selection and its reuses
        rh.deblur(it, vel, R)
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)
    t_build, t_reuse, n_build, n_reuse = 0.0, 0.0, 0, 0
    t0 = time.perf_counter()
    base = args.reuse  # start on a fresh selection
    for it in range(base, base + args.iters):
        b0 = rh.builds
        ta = time.perf_counter()
        _, X = rh.deblur(it, vel, R)
        torch.cuda.synchronize()
        dt = time.perf_counter() - ta
        if rh.builds > b0:
            t_build += dt
            n_build += 1
        else:
            t_reuse += dt
            n_reuse += 1
    wall = time.perf_counter() - t0
    rh.close()
    out = {
        "metric": "randomized receivers with Hessian reuse: s per iteration (selection builds amortised)",
        "value": round(wall / args.iters, 6),
        "unit": "s/iteration",
        "n_gpus": 1,
        "steps": args.iters,
        "warmup": args.reuse,
        "ms_per_step": round(wall / args.iters * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{s.name}-randomized-{args.subsets}of{s.nr}", "subsets": args.subsets,
                   "reuse": args.reuse, "nt": s.nt, "nf": s.nf, "ns": s.ns, "precision": "split_bf16"},
        "build_s": round(t_build / max(n_build, 1), 4),
        "builds": n_build,
        "reused_deblur_ms": round(t_reuse / max(n_reuse, 1) * 1e3, 3),
        "reused_iterations": n_reuse,
        "solves_per_s_reused": round(s.nf * s.ns / (t_reuse / max(n_reuse, 1)), 1) if n_reuse else None,
    }
    print(json.dumps(out), flush=True)


def run_deblur(args):
    """The deblur alone (ehi_apply_multipliers) at a list of sizes: seeded
    Hermitian positive definite Hessians H = A A^H / nr (A complex Gaussian,
    FP64), mu = 1e-3 lambda_max, the 1000 x 300 survey's 30 frequencies, both
    precision forms; every size's right-hand sides deblurred 10 x steps times
    between two events on the survey's stream."""
    import torch

    import synth
    from paper_2512_16642_amd import ehi

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    base = synth.layered_1000x300()
    sizes = [tuple(int(v) for v in x.split("x")) for x in args.deblur_sizes.split(",")]
    reps = 10 * max(1, args.steps)
    rows = []
    for nr, ns in sizes:
        if not (1 <= nr <= 500 and ns >= 1):
            raise SystemExit(f"deblur size {nr}x{ns}: receivers must be in [1, 500]")
        s = base.with_(nt=8, ns=ns, rec_iz=(2,) * nr, rec_ix=tuple(2 + 2 * k for k in range(nr)))
        g = torch.Generator(device="cpu").manual_seed(3100 + nr)
        A = torch.randn((s.nf, nr, nr), dtype=torch.complex128, generator=g)
        H = (A @ A.conj().transpose(1, 2).contiguous() / nr).to(dev)
        R = torch.randn((s.nf, ns, nr), dtype=torch.complex64, generator=g).to(dev)
        row = {"nr": nr, "ns": ns, "nf": s.nf}
        for prec in ("split_bf16", "plain_fp32"):
            sv = ehi.survey_from(s, precision=prec, max_ns=ns)
            sv.load_hessian(H)
            sv.factor(1e-3 * sv.lambda_max())
            X = sv.apply_multipliers(R)
            for _ in range(max(0, args.warmup)):
                sv.apply_multipliers(R, out=X)
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                sv.apply_multipliers(R, out=X)
            e1.record(st)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            row[prec] = {"ms": round(ms, 4), "solves_per_s": round(s.nf * ns / (ms / 1e3), 1)}
            sv.close()
        rows.append(row)
        print(f"# deblur {nr} x {ns}: split {row['split_bf16']['ms']:.4f} ms, "
              f"plain {row['plain_fp32']['ms']:.4f} ms", file=sys.stderr, flush=True)
    head = next((r for r in rows if r["nr"] == 200 and r["ns"] == 200), rows[0])
    out = {"metric": "deblur alone: multiplier solves/s by size", "value": head["split_bf16"]["solves_per_s"],
           "unit": "solves/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"deblur-{head['nr']}x{head['ns']}-nf{head['nf']}"}, "sizes": rows}
    print(json.dumps(out), flush=True)


def run_accuracy(args):
    """The Hessian accuracy test on the 1000 x 300 layered survey: frequencies
    moved to the nearest bins of the 2nt-point transform, factors of the
    smoothed (starting) model built once, then per step, for args.acc_ns
    surface sources: residual spectra, deblur, inverse transform, back-
    propagation S^T, extended forward S and the misfit."""
    import torch

    import synth
    from paper_2512_16642_amd import accuracy, ehi

    base = synth.layered_1000x300()
    s = base.with_(name=base.name + "-bins", freqs_hz=synth.nearest_bins(base.nt, base.dt, base.freqs_hz))
    ns = args.acc_ns
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    v_true = s.velocity()
    v0 = synth.smoothed(v_true, 10)
    sv = ehi.survey_from(s, precision=args.precision, max_ns=ns)
    t0 = time.perf_counter()
    vel0 = torch.from_numpy(v0).to(dev)
    sv.build_green(vel0)
    sv.build_hessian()
    mu = 1e-3 * sv.lambda_max()
    sv.factor(mu)
    torch.cuda.synchronize()
    # the direct method's set-up as timed (Nr PDE solves + contraction + factor)
    e_direct = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    stream0 = torch.cuda.current_stream()
    e_direct[0].record(stream0)
    sv.build_green(vel0)
    sv.build_hessian()
    sv.factor(mu)
    e_direct[1].record(stream0)
    e_direct[1].synchronize()
    direct_setup_ms = e_direct[0].elapsed_time(e_direct[1])
    # observed data from the true model, predicted data from the starting model:
    # Ricker sources (8 Hz) at depth 20 m, spread across x, on the subgrid
    src = torch.zeros((ns, s.nt, s.nzs, s.nxs), dtype=torch.float32, device=dev)
    w = torch.from_numpy(synth.ricker(s.nt, s.dt, 8.0)).to(dev)
    for k in range(ns):
        src[k, :, 1, (k * (s.nxs - 1)) // max(1, ns - 1)] = w
    sv.set_medium(torch.from_numpy(v_true).to(dev))
    d_obs = sv.forward_subgrid(src)
    sv.set_medium(torch.from_numpy(v0).to(dev))
    dd = d_obs - sv.forward_subgrid(src)
    del src
    torch.cuda.synchronize()
    print(f"# accuracy: factors and data ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    db = torch.empty((ns, s.nt, s.nzs, s.nxs), dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        accuracy.accuracy_test(sv, dd, d_obs, db_out=db)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    acc = [0.0] * 4
    t0 = time.perf_counter()
    for k in range(args.steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record(stream)
        dde = accuracy.deblur_time(sv, dd)
        e[1].record(stream)
        sv.backpropagate(dde, out=db)
        e[2].record(stream)
        pred = sv.forward_subgrid(db)
        e[3].record(stream)
        err, rel = ehi.misfit(dd, pred, d_obs)
        e[4].record(stream)
        e[4].synchronize()
        for j in range(4):
            acc[j] += e[j].elapsed_time(e[j + 1])
        print(f"# accuracy step {k} done", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    K = args.steps
    tot = sum(acc) / K
    relerr = rel.cpu().tolist()
    # the Krylov baseline: CG on the time-domain system with two PDE solves per
    # iteration, stopped once every source's fit reaches the direct method's
    # (the paper's rule) or after args.cg_iters iterations
    from paper_2512_16642_amd import krylov
    obs2 = (d_obs.double() ** 2).sum(dim=(1, 2)).cpu()
    e_cg = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e_cg[0].record(stream)
    cgr = krylov.cg(sv, dd, mu, args.cg_iters, target=torch.tensor(relerr, dtype=torch.float64),
                    obs_norm2=obs2)
    e_cg[1].record(stream)
    e_cg[1].synchronize()
    cg_ms = e_cg[0].elapsed_time(e_cg[1])
    cg_its, cg_solves = cgr["iterations"], cgr["pde_solves"]
    cg_rel = cgr["relerr_history"][-1].tolist() if cgr["relerr_history"] else []
    print(f"# accuracy: CG {cgr['iterations']} iterations in {cg_ms / 1e3:.1f} s", file=sys.stderr, flush=True)
    del cgr
    e_gm = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e_gm[0].record(stream)
    gmr = krylov.gmres(sv, dd, mu, args.cg_iters, target=torch.tensor(relerr, dtype=torch.float64),
                       obs_norm2=obs2)
    e_gm[1].record(stream)
    e_gm[1].synchronize()
    gm_ms = e_gm[0].elapsed_time(e_gm[1])
    gm_rel = gmr["relerr_history"][-1].tolist() if gmr["relerr_history"] else []
    print(f"# accuracy: GMRES {gmr['iterations']} iterations in {gm_ms / 1e3:.1f} s", file=sys.stderr, flush=True)
    cells = 2.0 * ns * s.nt * (s.nz + 2 * s.nb) * (s.nx + 2 * s.nb)
    pde_ms = (acc[1] + acc[2]) / K
    out = {
        "metric": "Hessian accuracy test: sources/s (deblur in time + back-propagation + extended forward)",
        "value": round(ns / (tot / 1e3), 3),
        "unit": "sources/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall / K * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": s.name, "sources": ns, "precision": args.precision, "nf_bins": s.nf,
                   "starting_model": "true model box-smoothed over 21 cells"},
        "stage_ms": {"deblur_time": round(acc[0] / K, 3), "backpropagate": round(acc[1] / K, 2),
                     "forward": round(acc[2] / K, 2), "misfit": round(acc[3] / K, 3)},
        "gcell_updates_per_s": round(cells / (pde_ms / 1e3) / 1e9, 1),
        "relerr": {"min": round(min(relerr), 5), "max": round(max(relerr), 5),
                   "mean": round(sum(relerr) / len(relerr), 5)},
        "direct_vs_krylov": {
            "direct": {"pde_solves": s.nr, "setup_s": round(direct_setup_ms / 1e3, 3),
                       "deblur_ms": round(acc[0] / K, 3),
                       "s_for_these_sources": round((direct_setup_ms + acc[0] / K) / 1e3, 3)},
            "cg": {"iterations": cg_its, "pde_solves": cg_solves,
                   "s_for_these_sources": round(cg_ms / 1e3, 3),
                   "reached_direct_fit": bool(cg_rel) and all(c <= d for c, d in zip(cg_rel, relerr)),
                   "relerr_max": round(max(cg_rel), 5) if cg_rel else None},
            "gmres": {"iterations": gmr["iterations"], "pde_solves": gmr["pde_solves"],
                      "s_for_these_sources": round(gm_ms / 1e3, 3),
                      "reached_direct_fit": bool(gm_rel) and all(c <= d for c, d in zip(gm_rel, relerr)),
                      "relerr_max": round(max(gm_rel), 5) if gm_rel else None},
        },
    }
    sv.close()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.workload in ("batch8", "serve", "accuracy", "randomized", "compare", "hbm_probe", "deblur"):
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        {"batch8": run_batch, "serve": run_serve, "accuracy": run_accuracy,
         "randomized": run_randomized, "compare": run_compare, "hbm_probe": run_hbm_probe,
         "deblur": run_deblur}[args.workload](args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU layout is "
              "a design note and is not benchmarked", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2512_16642_amd import costs, ehi

    s = synth.WORKLOADS[args.workload]()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print("# copy calibration: 1 GiB read + 1 GiB written", file=sys.stderr, flush=True)
        del a, b
    vel = torch.from_numpy(s.velocity()).to(dev)
    R = torch.from_numpy(s.residuals()).to(dev)
    X = torch.empty_like(R)
    keep = tuple(args.keep)
    sv = ehi.survey_from(s, precision=args.precision, max_ns=s.ns, nr_batch=args.nr_batch,
                         weighting=args.weighting, chunk=args.chunk, windows=args.windows, keep=keep,
                         decim=args.decim)
    print(f"# workload {s.name} precision {args.precision} workspace {sv.workspace_bytes / 1e9:.2f} GB",
          file=sys.stderr, flush=True)

    # mu = 1e-3 * max_w lambda_max(Hhat(w)) from a first build (not timed)
    sv.build_green(vel)
    sv.build_hessian()
    mu = 1e-3 * sv.lambda_max()
    for _ in range(args.warmup):
        sv.build_green(vel)
        sv.build_hessian()
        sv.factor(mu)
        sv.apply_multipliers(R, out=X)
    torch.cuda.synchronize()
    print(f"# warmup done, mu = {mu:.6e}", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    stage = {"build_green": 0.0, "build_hessian": 0.0, "factor": 0.0, "apply": 0.0}
    sv.read_profile()
    sv.profile(True)
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    for k in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(stream)
        sv.build_green(vel)
        ev[1].record(stream)
        sv.build_hessian()
        ev[2].record(stream)
        sv.factor(mu)
        ev[3].record(stream)
        sv.apply_multipliers(R, out=X)
        ev[4].record(stream)
        ev[4].synchronize()
        for i, key in enumerate(stage):
            stage[key] += ev[i].elapsed_time(ev[i + 1])
        print(f"# step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    sv.profile(False)
    prof = sv.read_profile()
    K = args.steps
    stage_ms = {k: v / K for k, v in stage.items()}
    survey_s = (stage_ms["build_green"] + stage_ms["build_hessian"] + stage_ms["factor"]) / 1e3
    solves_per_s = s.nf * s.ns / (stage_ms["apply"] / 1e3)

    # roofline of the dominant kernel (the marching stencil)
    nrb = args.nr_batch if args.nr_batch > 0 else s.nr
    tblock, seg_rows, band = sv.get_launch()
    step_ms, step_launches = prof["step"]
    cell_updates = costs.stencil_cell_updates_per_survey(s.nz, s.nx, s.nb, s.nr, s.nt)
    bpc = costs.stencil_bytes_per_cell_update(s.nz, s.nx, s.nb, s.stride, nrb, tblock)
    bytes_total = bpc * cell_updates * K
    avg_step_s = step_ms / 1e3 / max(step_launches, 1)
    bytes_launch = bytes_total / max(step_launches, 1)
    achieved = bytes_launch / avg_step_s / 1e9
    roof = {
        "kernel": f"k_march<{tblock}> (stencil, {tblock} time levels per launch, {seg_rows}-row segments, "
                  f"{band}-column bands)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": MEASURED_TRAFFIC.get((s.name, args.precision, tblock, seg_rows, band, nrb)),
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "traffic_source": TRAFFIC_SOURCE,
        "avg_launch_us": round(avg_step_s * 1e6, 2),
        "bytes_per_launch": round(bytes_launch),
        "bytes_per_cell_update": round(bpc, 4),
    }
    if args.windows == 2:
        roof["overlap"] = ("the marching launches run beside the DFT of the previous staging window "
                           "(two windows), which shares HBM: their average is the rate beside it; "
                           "--windows 1 times them alone")
    dft_ms = prof["dft"][0] / K
    dft_bytes = costs.dft_bytes_per_survey(s.nz, s.nx, s.stride, s.nr, s.nt, s.nf, args.chunk)
    dft_flops = costs.dft_flops_per_survey(s.nz, s.nx, s.stride, s.nr, s.nt, s.nf)
    # the finite-record form contracts the running spectra after every step: nt
    # times the final-spectrum contraction
    rep = (s.nt + args.decim - 1) // args.decim if args.weighting == "finite_record" else 1
    herk_flops = costs.herk_flops_per_survey(s.nz, s.nx, s.stride, s.nr, s.nf) * rep
    compressed = keep[0] > 0 and keep[1] > 0
    if compressed:
        # the contraction runs over the kept coefficients instead of the grid points
        herk_flops *= keep[0] * keep[1] / s.nsub
    herk_ms = prof["herk"][0] / K
    # 32 x 32 block pairs in the whole-matrix contraction (final-spectrum form)
    # and in the finite-record contraction, 64 x 64 tile pairs otherwise
    whole = (args.precision == "split_bf16" and args.weighting == "long_record"
             and os.environ.get("EHI_HERK_WHOLE", "1") != "0")
    herk_tile = 32 if (whole or args.weighting == "finite_record") else 64
    out = {
        "metric": METRIC,
        "value": round(survey_s, 6),
        "unit": "s/survey",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(t_wall / K * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": s.name, "precision": args.precision, "weighting": args.weighting,
                   "decim": args.decim,
                   "chunk": args.chunk, "windows": args.windows, "keep": list(keep),
                   "nz": s.nz, "nx": s.nx,
                   "nb": s.nb, "nr": s.nr, "nt": s.nt, "nf": s.nf, "ns": s.ns, "stride": s.stride,
                   "nr_batch": nrb},
        "workspace_gb": round(sv.workspace_bytes / 1e9, 3),
        "solves_per_s": round(solves_per_s, 1),
        "sources_per_s": round(s.ns / (stage_ms["apply"] / 1e3), 2),
        "stage_ms": {k: round(v, 3) for k, v in stage_ms.items()},
        "kernel_ms": {k: round(v[0] / K, 3) for k, v in prof.items()},
        "gcell_updates_per_s": round(cell_updates / (prof["step"][0] / K / 1e3) / 1e9, 2),
        "herk_tflops": round(herk_flops / (herk_ms / 1e3) / 1e12, 2) if herk_ms > 0 else None,
        "herk_mfma_bf16_tflops": (round(costs.herk_bf16_mfma_flops_per_survey(s.nr, s.nsub, s.nf, herk_tile) * rep
                                        / (herk_ms / 1e3) / 1e12, 1)
                                  if herk_ms > 0 and args.precision == "split_bf16" and not compressed
                                  else None),
        "dft_gbs": round(dft_bytes / (dft_ms / 1e3) / 1e9, 1) if dft_ms > 0 else None,
        "dft_tflops": round(dft_flops / (dft_ms / 1e3) / 1e12, 2) if dft_ms > 0 else None,
        "roofline": roof,
    }
    # the Green-function stage as a whole: the stepping's and the DFT's
    # algorithmic bytes over the stage's own time (with two staging windows the
    # two kernels run side by side, so neither one's average duration shows the
    # stage's use of HBM)
    if dft_ms > 0 and stage_ms["build_green"] > 0 and args.weighting == "long_record" and not compressed:
        stage_bytes = bytes_total / K + dft_bytes
        stage_gbs = stage_bytes / (stage_ms["build_green"] / 1e3) / 1e9
        out["roofline_green_stage"] = {"kernels": "k_march + k_dft_bf16x3", "bound": "hbm",
                                       "achieved": round(stage_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(stage_gbs / HBM_PEAK_GBS, 4),
                                       "bytes_per_survey": round(stage_bytes), "stage_ms": round(stage_ms["build_green"], 3)}
    # the two other hot kernels against their own peaks (the contraction on the
    # BF16 matrix cores; the DFT on the FP32 matrix cores, its bytes beside)
    herk_exec = out["herk_mfma_bf16_tflops"]
    if herk_exec is not None:
        # the planning count: three BF16 products (hi.hi, hi.lo, lo.hi) per real
        # product of the useful Hermitian contraction; the executed count
        # (every product the kernel issues, lo.lo and block padding included)
        # beside it
        planned = 3.0 * herk_flops / (herk_ms / 1e3) / 1e12
        kname = ("k_herk_r2 (finite-record, per kept sample)" if args.weighting == "finite_record"
                 else "k_herk_bf16_whole" if whole else "k_herk_bf16")
        out["roofline_herk"] = {"kernel": kname, "bound": "mfma",
                                "achieved": round(planned, 1), "peak": 2500.0, "unit": "TFLOP/s",
                                "frac": round(planned / 2500.0, 4),
                                "count": "3 BF16 products x useful Hermitian flops (8 nr(nr+1)/2 nsub nf)",
                                "executed_tflops": herk_exec, "executed_frac": round(herk_exec / 2500.0, 4)}
    if dft_ms > 0:
        dft_tf = dft_flops / (dft_ms / 1e3) / 1e12
        dft_gbs = dft_bytes / (dft_ms / 1e3) / 1e9
        if os.environ.get("EHI_DFT_FORM") == "0":
            # FP32 matrix cores: 4 flops per sample and frequency at 32 flop/B,
            # bound by the FP32 matrix peak and the HBM together
            out["roofline_dft"] = {"kernel": "k_dft_mfma (FP32 matrix cores)", "bound": "mfma",
                                   "achieved": round(dft_tf, 2), "peak": 157.3, "unit": "TFLOP/s",
                                   "frac": round(dft_tf / 157.3, 4), "hbm_frac": round(dft_gbs / HBM_PEAK_GBS, 4)}
        else:
            # three-part BF16 products (six per product) leave the BF16 matrix
            # cores at a fraction of their peak: the staged samples' bytes bound it
            out["roofline_dft"] = {"kernel": "k_dft_bf16x3 (three-part BF16 on the BF16 matrix cores)",
                                   "bound": "hbm", "achieved": round(dft_gbs, 1), "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(dft_gbs / HBM_PEAK_GBS, 4),
                                   "bytes_per_survey": dft_bytes, "useful_tflops": round(dft_tf, 2),
                                   "bf16_mfma_frac": round(dft_tf * 6 / 2500.0, 4)}
        if args.windows == 2:
            out["roofline_dft"]["overlap"] = ("kernel time on the second stream beside the stepping (two "
                                              "staging windows): all but the last window's DFT hide behind "
                                              "the marching launches, so this rate is not the kernel's alone; "
                                              "--windows 1 times it alone")
    if not args.no_cpu_baseline:
        gpu = None
        if args.weighting == "long_record" and not compressed:
            # the GPU's results the oracle's sample is compared with
            idx = sample_receivers(s.nr, max(1, min(args.cpu_receivers, s.nr)))
            it = torch.tensor(idx, device=dev)
            G = sv.copy_green_dft().reshape(s.nf, s.nr, -1)
            gpu = {"G": G.index_select(1, it).cpu().numpy().astype(np.complex128),
                   "H": sv.copy_hessian().cpu().numpy(),
                   "X": X.cpu().numpy().astype(np.complex128), "mu": mu}
            del G
        print("# timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_hessians, args.cpu_receivers, gpu)
        if "parity" in out["cpu_baseline"]:
            out["parity"] = out["cpu_baseline"].pop("parity")
    sv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
