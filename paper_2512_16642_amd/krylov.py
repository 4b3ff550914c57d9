"""The Krylov baseline on the GPU: conjugate gradients on the time-domain
system Q x = dd, Q = S S^T + mu I.

Paper: the iterative alternative to the direct inversion needs two PDE
solves per iteration and per source (Introduction; Hessian accuracy test: CG
stopped once its data fit reaches the direct method's; Table of PDE solves and
CPU times).  Each iteration here is one ``backpropagate`` (S^T p) and one
``forward_subgrid`` (S of that) over all sources of the batch, then the
library's three CG vector kernels.  The fit of the iterate, |dd - S S^T x|^2 =
|r + mu x|^2, comes out of the update kernel, so the paper's stopping rule
costs no extra PDE solve.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import ehi


def _p(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def cg(sv: "ehi.Survey", dd: torch.Tensor, mu: float, maxiter: int,
       target: Optional[torch.Tensor] = None, obs_norm2: Optional[torch.Tensor] = None) -> dict:
    """Batched CG for the records ``dd`` float32 [ns][nr][nt] on survey ``sv``
    (medium loaded).  Stops after ``maxiter`` iterations, or once every record's
    RelErr = fit / obs_norm2 is at or below ``target`` [ns] (both float64 host
    tensors; the check reads ``fit`` back once per iteration).

    Returns x, the iterations run, the PDE solves (2 per iteration per record)
    and the per-iteration RelErr history (when ``obs_norm2`` is given)."""
    L = ehi.lib()
    ns = dd.shape[0]
    ehi._require(dd, torch.float32, (ns, sv.nr, sv.nt), "dd", sv.device)
    n = sv.nr * sv.nt
    x, r, p, Ap = (torch.empty_like(dd) for _ in range(4))
    db = torch.empty((ns, sv.nt, sv.nzs, sv.nxs), dtype=torch.float32, device=sv.device)
    rr, rr_new, pAp, fit = (torch.empty(ns, dtype=torch.float64, device=sv.device) for _ in range(4))
    st = ctypes.c_void_p(0 if sv.stream is None else sv.stream.cuda_stream)
    ehi._check(L.ehi_cg_init(_p(dd), ns, n, _p(x), _p(r), _p(p), _p(rr), st))
    hist = []
    it = 0
    while it < maxiter:
        sv.backpropagate(p, out=db)
        sv.forward_subgrid(db, out=Ap)
        ehi._check(L.ehi_cg_shift_dot(_p(Ap), _p(p), ctypes.c_double(mu), ns, n, _p(pAp), st))
        ehi._check(L.ehi_cg_update(_p(x), _p(r), _p(p), _p(Ap), _p(rr), _p(pAp), ctypes.c_double(mu), ns, n,
                                   _p(rr_new), _p(fit), st))
        ehi._check(L.ehi_cg_direction(_p(p), _p(r), _p(rr_new), _p(rr), ns, n, st))
        rr, rr_new = rr_new, rr
        it += 1
        if obs_norm2 is not None:
            rel = fit.cpu() / obs_norm2
            hist.append(rel)
            if target is not None and bool(torch.all(rel <= target)):
                break
    return {"x": x, "iterations": it, "pde_solves": 2 * it * ns, "relerr_history": hist}
