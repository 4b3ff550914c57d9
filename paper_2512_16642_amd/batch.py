"""Batched uneven surveys: one captured HIP graph for all builds, one batched
factorisation launch, per-survey deblurs.

All arithmetic runs in libehi; this module only orders work: each survey's
Green-function stepping and Hessian contraction are enqueued on a stream of its
own (so small surveys overlap on the device) inside one graph capture
(fork from the capturing stream, join back), and the graph is replayed for every
rebuild.  The factorisation of every frequency of every survey is one launch
(``ehi_factor_batch``).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from . import autotune, ehi


class SurveyBatch:
    def __init__(self, specs: Sequence, precision: str = "split_bf16",
                 staging_budget_bytes: int = 6 << 30, tune: bool = False,
                 device: Optional[torch.device] = None, chunk: int = 256):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.specs = list(specs)
        self.surveys: List[ehi.Survey] = []
        self.streams = [torch.cuda.Stream(self.device) for _ in self.specs]
        for spec, st in zip(self.specs, self.streams):
            nrb = staging_receivers(spec, staging_budget_bytes, chunk)
            # launch shapes are tuned on a short probe before the survey's own
            # workspace is allocated (the probe needs a workspace of its own)
            shape = autotune.tune(spec, nrb=nrb) if tune else None
            herk = autotune.tune_contraction(spec, precision) if tune else {"herk_form": 0, "herk_split": 0}
            sv = ehi.survey_from(spec, precision=precision, nr_batch=nrb, stream=st, chunk=chunk,
                                 herk_form=herk["herk_form"], herk_split=herk["herk_split"])
            if shape is not None:
                sv.set_launch(shape["tblock"], shape["seg_rows"], shape.get("band", 0))
            self.surveys.append(sv)
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self._vels = None

    @property
    def workspace_bytes(self) -> int:
        return sum(sv.workspace_bytes for sv in self.surveys)

    def _enqueue(self, vels, fork_stream):
        ev = torch.cuda.Event()
        ev.record(fork_stream)
        for sv, st, v in zip(self.surveys, self.streams, vels):
            st.wait_event(ev)
            sv.set_stream(st)
            sv.build_green(v)
            sv.build_hessian()
        for st in self.streams:
            fork_stream.wait_stream(st)

    def build(self, vels: Sequence[torch.Tensor], graph: bool = True):
        """Green functions and Hessians of every survey.  With ``graph`` the whole
        sequence is captured once into a HIP graph and replayed afterwards."""
        vels = list(vels)
        if not graph:
            self._enqueue(vels, torch.cuda.current_stream(self.device))
            return
        if self.graph is None or self._vels is None or any(
                a.data_ptr() != b.data_ptr() for a, b in zip(vels, self._vels)):
            torch.cuda.synchronize(self.device)
            g = torch.cuda.CUDAGraph()
            cap = torch.cuda.Stream(self.device)
            with torch.cuda.graph(g, stream=cap):
                self._enqueue(vels, cap)
            self.graph = g
            self._vels = vels
        self.graph.replay()

    def factor(self, mu: Sequence[float]):
        """Penalty and Cholesky of every (survey, frequency): one launch."""
        ehi.factor_batch(self.surveys, mu)

    def lambda_max(self) -> List[float]:
        torch.cuda.synchronize(self.device)
        return [sv.lambda_max() for sv in self.surveys]

    def apply(self, resids: Sequence[torch.Tensor], outs: Optional[Sequence[torch.Tensor]] = None):
        """Deblur every survey's residuals on its own stream; ordered after the
        current stream (where the inputs were produced) and joined back to it."""
        cur = torch.cuda.current_stream(self.device)
        outs = [torch.empty_like(r) for r in resids] if outs is None else list(outs)
        for st in self.streams:
            st.wait_stream(cur)
        for sv, st, r, o in zip(self.surveys, self.streams, resids, outs):
            sv.apply_multipliers(r, out=o, stream=st)
            r.record_stream(st)
            o.record_stream(st)
        for st in self.streams:
            cur.wait_stream(st)
        return outs

    def close(self):
        torch.cuda.synchronize(self.device)
        self.graph = None
        for sv in self.surveys:
            sv.close()


def staging_receivers(spec, budget_bytes: int, chunk: int = 256) -> int:
    """Receivers stepped together so that the DFT staging window fits the budget."""
    nsub = spec.nsub
    nsub_p = (nsub + 255) // 256 * 256
    per = chunk * nsub_p * 4
    return int(max(1, min(spec.nr, budget_bytes // per)))
