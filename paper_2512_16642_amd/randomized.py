"""Randomized receiver selection with Hessian reuse.

Paper: Randomized receiver inversion subsection.  The receiver axis is divided
into subsets and one receiver is drawn at random from each subset at every
iteration; the data-space Hessian is built for the active receivers only, so
its cost falls with the square of their number (Table of computational
complexity; numerical examples: 100 of 273 or 450 receivers).  Reuse: the
factors of one selection serve ``reuse`` consecutive iterations (deblurs)
before the next selection is built, the factors staying resident on the
device in between.

The selection is host logic; building, factoring and deblurring are the
library's calls on a survey whose receivers are the selected ones, so every
result equals that of a survey built directly on those receivers.
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np


def subsets(nr: int, n_subsets: int) -> List[Tuple[int, int]]:
    """Contiguous receiver index ranges [start, stop), as equal as possible
    (the first nr % n_subsets ranges hold one receiver more)."""
    if not 1 <= n_subsets <= nr:
        raise ValueError("need 1 <= n_subsets <= nr")
    base, extra = divmod(nr, n_subsets)
    out, start = [], 0
    for k in range(n_subsets):
        stop = start + base + (1 if k < extra else 0)
        out.append((start, stop))
        start = stop
    return out


def select(nr: int, n_subsets: int, seed: int, draw: int) -> np.ndarray:
    """One receiver index drawn uniformly from each subset, in ascending order;
    draw ``draw`` of the sequence seeded by ``seed`` (numpy PCG64 seeded with
    [seed, draw])."""
    rng = np.random.default_rng([int(seed), int(draw)])
    return np.array([int(rng.integers(a, b)) for a, b in subsets(nr, n_subsets)], dtype=np.int64)


class RandomizedHessian:
    """Selections of ``n_subsets`` receivers out of ``spec``'s, each built once
    and reused for ``reuse`` iterations.

    ``deblur(it, vel, resid)`` takes residuals of all receivers
    ``[nf][ns][nr]`` (device complex64), restricts them to the selection of
    iteration ``it`` and returns ``(indices, multipliers [nf][ns][n_subsets])``.
    A new selection, or a new velocity tensor, triggers a build; otherwise the
    resident factors are reused.
    """

    def __init__(self, spec, n_subsets: int, reuse: int = 1, seed: int = 0,
                 precision: str = "split_bf16", mu_rel: float = 1e-3, max_ns: Optional[int] = None):
        if reuse < 1:
            raise ValueError("reuse must be >= 1")
        self.spec = spec
        self.n_subsets = int(n_subsets)
        self.reuse = int(reuse)
        self.seed = int(seed)
        self.precision = precision
        self.mu_rel = float(mu_rel)
        self.max_ns = max_ns
        self._draw = None
        self._vel = None
        self._sv = None
        self.indices: Optional[np.ndarray] = None
        self.builds = 0

    def selection(self, it: int) -> np.ndarray:
        return select(self.spec.nr, self.n_subsets, self.seed, it // self.reuse)

    def subset_spec(self, indices: np.ndarray):
        s = self.spec
        return s.with_(name=f"{s.name}-sel{len(indices)}",
                       rec_iz=tuple(int(s.rec_iz[k]) for k in indices),
                       rec_ix=tuple(int(s.rec_ix[k]) for k in indices))

    def prepare(self, it: int, vel):
        """Make the factors of iteration ``it``'s selection resident."""
        from . import ehi
        draw = it // self.reuse
        if self._sv is not None and draw == self._draw and vel is self._vel:
            return self._sv
        if self._sv is not None:
            self._sv.close()
            self._sv = None
        idx = self.selection(it)
        sub = self.subset_spec(idx)
        sv = ehi.survey_from(sub, precision=self.precision,
                             max_ns=self.max_ns if self.max_ns is not None else max(1, sub.ns))
        sv.build_green(vel)
        sv.build_hessian()
        sv.factor(self.mu_rel * sv.lambda_max())
        self._sv, self._draw, self._vel, self.indices = sv, draw, vel, idx
        self.builds += 1
        return sv

    def deblur(self, it: int, vel, resid):
        import torch
        sv = self.prepare(it, vel)
        idx = torch.as_tensor(self.indices, device=resid.device)
        r = resid.index_select(2, idx).contiguous()
        return self.indices, sv.apply_multipliers(r)

    def close(self):
        if self._sv is not None:
            self._sv.close()
            self._sv = None
