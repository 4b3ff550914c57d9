"""The Krylov baselines on the GPU: conjugate gradients and GMRES on the
time-domain system Q x = dd, Q = S S^T + mu I.

Paper: the iterative alternative to the direct inversion needs two PDE
solves per iteration and per source (Introduction; Hessian accuracy test: CG
stopped once its data fit reaches the direct method's; Table of PDE solves and
CPU times).  Each iteration here is one ``backpropagate`` (S^T p) and one
``forward_subgrid`` (S of that) over all sources of the batch, then the
library's three CG vector kernels.  The fit of the iterate, |dd - S S^T x|^2 =
|r + mu x|^2, comes out of the update kernel, so the paper's stopping rule
costs no extra PDE solve.

GMRES (one cycle of at most m iterations, no restart) keeps its Arnoldi basis
on the device ([m + 1][ns][nr][nt] float32), orthogonalises each new vector
with two passes of classical Gram-Schmidt (``ehi_mdot`` / ``ehi_combine``,
FP64 sums) and solves the small least-squares problem of the Hessenberg matrix
of every record on the host; the iterate and its misfit dd - S S^T x =
r + mu x are formed in the basis, so its stopping rule also needs no extra PDE
solve.
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


def gmres(sv: "ehi.Survey", dd: torch.Tensor, mu: float, m: int,
          target: Optional[torch.Tensor] = None, obs_norm2: Optional[torch.Tensor] = None) -> dict:
    """Batched GMRES on the records ``dd`` float32 [ns][nr][nt]: at most ``m``
    iterations (one cycle), stopping early once every record's RelErr (fit /
    obs_norm2) is at or below ``target``.  Returns x, the iterations run, the
    PDE solves (2 per iteration per record), the RelErr history (when
    ``obs_norm2`` is given) and the relative residual history."""
    import numpy as np
    L = ehi.lib()
    ns = dd.shape[0]
    ehi._require(dd, torch.float32, (ns, sv.nr, sv.nt), "dd", sv.device)
    n = sv.nr * sv.nt
    vs = ns * n                                     # stride between basis vectors
    dev = sv.device
    st = ctypes.c_void_p(0 if sv.stream is None else sv.stream.cuda_stream)
    V = torch.empty((m + 1, ns, sv.nr, sv.nt), dtype=torch.float32, device=dev)
    w = torch.empty_like(dd)
    t = torch.empty_like(dd)
    db = torch.empty((ns, sv.nt, sv.nzs, sv.nxs), dtype=torch.float32, device=dev)
    hdev = torch.empty((ns, m + 2), dtype=torch.float64, device=dev)
    scratch = torch.empty(ns, dtype=torch.float64, device=dev)

    def mdot(vbase, nvec, vec):
        ehi._check(L.ehi_mdot(_p(vbase), vs, nvec, _p(vec), ns, n, _p(hdev), st))
        return hdev[:, :nvec].cpu().numpy().copy() if nvec == hdev.shape[1] else \
            hdev.view(-1)[:ns * nvec].view(ns, nvec).cpu().numpy().copy()

    def combine(vbase, coef, beta, dst):
        c = torch.from_numpy(np.ascontiguousarray(coef, dtype=np.float64)).to(dev)
        ehi._check(L.ehi_combine(_p(vbase), vs, coef.shape[1], _p(c), ns, n, ctypes.c_double(beta), _p(dst), st))
        return c                                    # keep alive until the stream has used it

    keep = []
    beta = np.sqrt(mdot(dd, 1, dd)[:, 0])
    keep.append(combine(dd, (1.0 / beta)[:, None], 0.0, V[0]))
    H = np.zeros((ns, m + 1, m))
    hist, res = [], []
    y = np.zeros((ns, 0))
    k = 0
    for j in range(m):
        sv.backpropagate(V[j], out=db)
        sv.forward_subgrid(db, out=w)
        ehi._check(L.ehi_cg_shift_dot(_p(w), _p(V[j]), ctypes.c_double(mu), ns, n, _p(scratch), st))
        for _ in range(2):                          # classical Gram-Schmidt, twice
            hh = mdot(V, j + 1, w)
            keep.append(combine(V, -hh, 1.0, w))
            H[:, :j + 1, j] += hh
        hn = np.sqrt(mdot(w, 1, w)[:, 0])
        H[:, j + 1, j] = hn
        keep.append(combine(w, (1.0 / np.where(hn > 0, hn, 1.0))[:, None], 0.0, V[j + 1]))
        k = j + 1
        e1 = np.zeros(k + 1)
        ys, rr = np.zeros((ns, k)), np.zeros(ns)
        for q in range(ns):
            rhs = e1.copy()
            rhs[0] = beta[q]
            ys[q] = np.linalg.lstsq(H[q, :k + 1, :k], rhs, rcond=None)[0]
            rr[q] = np.linalg.norm(rhs - H[q, :k + 1, :k] @ ys[q]) / beta[q]
        y = ys
        res.append(rr)
        if obs_norm2 is not None:
            # r + mu x in the basis: (beta e1 - Hbar y) + mu (y, 0)
            c = -np.einsum("qab,qb->qa", H[:, :k + 1, :k], y)
            c[:, 0] += beta
            c[:, :k] += mu * y
            keep.append(combine(V, c, 0.0, t))
            rel = torch.from_numpy(mdot(t, 1, t)[:, 0]) / obs_norm2
            hist.append(rel)
            if target is not None and bool(torch.all(rel <= target)):
                break
    x = torch.empty_like(dd)
    keep.append(combine(V, y, 0.0, x))
    torch.cuda.synchronize(dev)
    return {"x": x, "iterations": k, "pde_solves": 2 * k * ns, "relerr_history": hist,
            "residual_history": res}

