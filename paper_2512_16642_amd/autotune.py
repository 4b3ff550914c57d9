"""Launch-shape autotuner for the Green-function stepping and the contraction.

The marching kernel's time levels per launch trade HBM traffic against
redundant halo work, and its rows per segment trade redundant halo rows against
the number of workgroups; the best pair depends on the grid and on how many
receivers are stepped together.  ``tune`` times a short build (nt_probe steps)
for each candidate pair on the real grid and receivers and caches the winner in
a JSON file keyed by (padded grid, receivers per batch, arch).  Results never
depend on the launch shape.

``tune_contraction`` does the same for the Hessian contraction: the form
(whole-matrix or tile pairs, split-BF16 final-spectrum surveys) and the number
of grid partitions, timed on random spectra of the survey's sizes (receivers,
subgrid points, frequencies).  The partition count changes only the order of
FP32 partial sums, so results agree to rounding.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

import torch

from . import ehi

TBLOCKS = (4, 8)
SEG_ROWS = (64, 96, 128, 192, 256)


def cache_path() -> str:
    return os.environ.get("EHI_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ehi", "tune.json"))


def _key(spec, nrb: int) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "none"
    return f"{arch}:Z{spec.nz + 2 * spec.nb}:X{spec.nx + 2 * spec.nb}:nrb{nrb}:v3"


def _load() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache: Dict[str, dict]):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(spec, nrb: Optional[int] = None, nt_probe: int = 64, repeats: int = 2) -> dict:
    """Best rows-per-segment for this grid and receiver count (cached)."""
    nrb = spec.nr if not nrb else nrb
    key = _key(spec, nrb)
    cache = _load()
    if key in cache:
        return cache[key]
    probe = spec.with_(nt=nt_probe, rec_iz=spec.rec_iz[:nrb], rec_ix=spec.rec_ix[:nrb])
    vel = torch.from_numpy(probe.velocity()).cuda()
    sv = ehi.survey_from(probe, max_ns=1)
    times = {}
    for tb in TBLOCKS:
        for seg in SEG_ROWS:
            sv.set_launch(tb, seg, 0)
            sv.build_green(vel)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(repeats):
                sv.build_green(vel)
            torch.cuda.synchronize()
            times[(tb, seg)] = (time.perf_counter() - t0) / repeats
    sv.close()
    best = min(times, key=times.get)
    entry = {"tblock": best[0], "seg_rows": best[1], "band": 0,
             "probe_s": {f"{k[0]}x{k[1]}": v for k, v in times.items()}}
    cache[key] = entry
    _store(cache)
    return entry


def apply(sv: "ehi.Survey", spec):
    e = tune(spec, nrb=min(spec.nr, sv_nrb(sv, spec)))
    sv.set_launch(e["tblock"], e["seg_rows"], e.get("band", 0))


def sv_nrb(sv, spec) -> int:
    return getattr(sv, "nr_batch", 0) or spec.nr


HERK_SPLITS = (2, 4, 8, 12, 17, 24, 32, 48, 64)


def _herk_key(spec, precision: str) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "none"
    return f"{arch}:herk:nr{spec.nr}:nsub{spec.nsub}:nf{spec.nf}:{precision}:v3"


def tune_contraction(spec, precision: str = "split_bf16", repeats: int = 3) -> dict:
    """Best (form, partitions) of the final-spectrum contraction for this
    survey's sizes (cached).  form 1 = whole-matrix (4 x 4 tiles of block
    pairs above 224 receivers), 2 = 64 x 64 tile pairs; the plain FP32 form
    has one kernel."""
    key = _herk_key(spec, precision)
    cache = _load()
    if key in cache:
        return cache[key]
    forms = [0] if precision != "split_bf16" else [1, 2]
    kmax = max(1, spec.nsub // 1024)
    # the library's accuracy floor: no partition adds more than 40 stages of 32
    # grid points into its FP32 running sums (fewer partitions are faster by a
    # few per cent and several times less accurate in the multipliers)
    floor = min(64, -(-(-(-spec.nsub // 32)) // 40))
    splits = sorted({s for s in HERK_SPLITS if floor <= s <= kmax} | {max(floor, min(kmax, 64))})
    probe = spec.with_(nt=8)
    g = torch.randn((spec.nf, spec.nr, spec.nzs, spec.nxs), dtype=torch.complex64, device="cuda")
    times = {}
    for form in forms:
        for split in splits:
            sv = ehi.survey_from(probe, precision=precision, max_ns=1, nr_batch=1, herk_split=split,
                                 herk_form=form)
            sv.load_green_dft(g)
            sv.build_hessian()           # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(repeats):
                sv.build_hessian()
            torch.cuda.synchronize()
            times[(form, split)] = (time.perf_counter() - t0) / repeats
            sv.close()
    del g
    best = min(times, key=times.get)
    entry = {"herk_form": best[0], "herk_split": best[1],
             "probe_ms": {f"{k[0]}x{k[1]}": round(v * 1e3, 4) for k, v in times.items()}}
    cache[key] = entry
    _store(cache)
    return entry
