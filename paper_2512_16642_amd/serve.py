"""Serving loop: survey builds and multiplier deblurs against resident factors.

Requests
  * build  - build (or rebuild) a survey: Green functions, Hessian, lambda_max,
             penalty mu = 1e-3 lambda_max, factorisation.  Admitted when a build
             slot is free and the workspaces of the resident surveys, of the
             builds in flight and of the factors waiting to be retired still fit
             the HBM budget.  When the head of the build queue does not fit,
             resident factors are evicted, least recently used first, until it
             does.  A finished build replaces the survey's previous factors.
             Replaced and evicted factors are retired (workspace released) once
             every deblur issued against them has finished.  A failed build
             releases its workspace and is reported "failed".
  * deblur - X = Qhat^{-1} R for ns sources of a resident survey, all
             frequencies (R seeded per request).  A deblur for a survey that is
             neither resident nor being built is "rejected"; one whose only build
             fails is "rejected" with it.

Continuous batching: at every scheduler tick, all pending deblurs of a resident
survey are concatenated along the source axis and solved by one library call on
the deblur stream, which runs beside the build streams (the device interleaves
their kernels), while new requests keep being admitted as slots and workspace
free up.  The solve treats every source column independently, so a request's
multipliers are bitwise the same alone or inside a merged batch.

The scheduler is device-agnostic: an engine object does the work.  ``EhiEngine``
drives libehi (all arithmetic in its kernels); the unit tests drive the same
scheduler with a host-only engine.  Latency is arrival -> result ready on the
host clock.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    kind: str            # "build" | "deblur"
    arrival: float       # seconds after the start of the run
    key: int             # survey key
    ns: int = 0          # deblur: number of sources
    seed: int = 0        # deblur: residual seed
    t_done: Optional[float] = None
    status: str = "pending"   # pending | done | failed | rejected


class Admission:
    """HBM-budget accounting on the host.  ``take`` never lets ``used`` exceed
    ``budget``; ``peak`` is the largest ``used`` ever reached."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak = 0

    def can_take(self, nbytes: int) -> bool:
        return self.used + nbytes <= self.budget

    def take(self, nbytes: int):
        if not self.can_take(nbytes):
            raise RuntimeError(f"admission over budget: {self.used} + {nbytes} > {self.budget}")
        self.used += nbytes
        self.peak = max(self.peak, self.used)

    def release(self, nbytes: int):
        if nbytes > self.used:
            raise RuntimeError("admission released more than it holds")
        self.used -= nbytes


def poisson_requests(duration_s: float, rate_hz: float, p_build: float, n_keys: int,
                     ns_max: int = 256, seed: int = 2400) -> List[Request]:
    """Poisson arrivals over [0, duration_s).  Each request is a build with
    probability p_build, else a deblur of U{1..ns_max} sources; the survey key
    is uniform over n_keys.  Draw order per request: gap, kind, key, then for a
    deblur ns and the residual seed."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            return out
        if rng.random() < p_build:
            out.append(Request(len(out), "build", t, int(rng.integers(0, n_keys))))
        else:
            key = int(rng.integers(0, n_keys))
            ns = int(rng.integers(1, ns_max + 1))
            out.append(Request(len(out), "deblur", t, key, ns=ns, seed=int(rng.integers(0, 2 ** 31))))


class _Resident:
    __slots__ = ("key", "handle", "nbytes", "inflight", "last_use")

    def __init__(self, key, handle, nbytes, now):
        self.key, self.handle, self.nbytes = key, handle, nbytes
        self.inflight = 0          # deblur batches issued against these factors, not yet finished
        self.last_use = now


class Server:
    """Continuous-batching scheduler over an engine with

    * ``workspace_bytes(key)``              device bytes a survey holds while built/resident
    * ``build(key, slot)``                  blocking build + factor (runs in a worker thread);
                                            returns a handle, raises on failure
    * ``deblur(handle, reqs)``              enqueue one merged solve; returns a ticket
    * ``ready(ticket)``                     has that solve finished
    * ``result(ticket, i)``                 multipliers of ``reqs[i]``
    * ``free(handle)``                      release a survey's device memory
    * ``max_batch_sources``                 cap on the sources merged into one solve
    """

    def __init__(self, engine, budget_bytes: int, build_slots: int = 2,
                 clock: Callable[[], float] = time.perf_counter, keep_results: bool = False,
                 tick_s: float = 2e-4):
        self.eng = engine
        self.adm = Admission(budget_bytes)
        self.slots = build_slots
        self.free_slots = list(range(build_slots))
        self.pool = cf.ThreadPoolExecutor(max_workers=build_slots, thread_name_prefix="ehi-build")
        self.resident: Dict[int, _Resident] = {}
        self.building: Dict[int, tuple] = {}          # rid -> (req, future, nbytes, slot)
        self.retiring: List[_Resident] = []
        self.pending_builds = collections.deque()
        self.pending_deblurs: Dict[int, collections.deque] = collections.defaultdict(collections.deque)
        self.inflight: List[tuple] = []                # (ticket, reqs, resident)
        self.clock = clock
        self.tick_s = tick_s
        self.keep_results = keep_results
        self.results: Dict[int, object] = {}
        self.t0 = clock()
        self.trace: List[tuple] = []                   # (t, used) after every change of ``used``
        self.evictions = 0

    def now(self) -> float:
        return self.clock() - self.t0

    def _take(self, n):
        self.adm.take(n)
        self.trace.append((self.now(), self.adm.used))

    def _release(self, n):
        self.adm.release(n)
        self.trace.append((self.now(), self.adm.used))

    # -- residency --------------------------------------------------------------------
    def preload(self, keys):
        """Build and factor surveys synchronously (initial residency)."""
        for k in keys:
            nbytes = self.eng.workspace_bytes(k)
            self._take(nbytes)
            try:
                h = self.eng.build(k, 0)
            except Exception:
                self._release(nbytes)
                raise
            self._install(k, h, nbytes)

    def _install(self, key, handle, nbytes):
        old = self.resident.get(key)
        self.resident[key] = _Resident(key, handle, nbytes, self.now())
        if old is not None:
            self.retiring.append(old)

    def _evict_for(self, nbytes) -> bool:
        """Retire least recently used resident factors until ``nbytes`` more
        would fit once retirement completes.  False if even evicting every
        resident survey would not make room yet (builds in flight hold it)."""
        pending_free = sum(r.nbytes for r in self.retiring)
        if self.adm.used - pending_free + nbytes <= self.adm.budget:
            return True
        for r in sorted(self.resident.values(), key=lambda r: r.last_use):
            del self.resident[r.key]
            self.retiring.append(r)
            self.evictions += 1
            pending_free += r.nbytes
            if self.adm.used - pending_free + nbytes <= self.adm.budget:
                return True
        return False

    def _retire(self):
        keep = []
        for r in self.retiring:
            if r.inflight == 0:
                self.eng.free(r.handle)
                self._release(r.nbytes)
            else:
                keep.append(r)
        self.retiring = keep

    # -- builds -----------------------------------------------------------------------
    def _admit_builds(self):
        while self.pending_builds and self.free_slots:
            req = self.pending_builds[0]
            nbytes = self.eng.workspace_bytes(req.key)
            if nbytes > self.adm.budget:               # can never fit
                self.pending_builds.popleft()
                self._finish(req, "rejected")
                continue
            if not self.adm.can_take(nbytes):          # wait for memory (FIFO)
                self._evict_for(nbytes)
                self._retire()
                if not self.adm.can_take(nbytes):
                    return
            self.pending_builds.popleft()
            self._take(nbytes)
            slot = self.free_slots.pop()
            fut = self.pool.submit(self.eng.build, req.key, slot)
            self.building[req.rid] = (req, fut, nbytes, slot)

    def _finish_builds(self):
        for rid in [r for r, (_, fut, _, _) in self.building.items() if fut.done()]:
            req, fut, nbytes, slot = self.building.pop(rid)
            self.free_slots.append(slot)
            err = fut.exception()
            if err is not None:
                self._release(nbytes)
                self._finish(req, "failed")
                continue
            self._install(req.key, fut.result(), nbytes)
            self._finish(req, "done")

    def _building_key(self, key) -> bool:
        return any(r.key == key for r in self.pending_builds) or any(
            b[0].key == key for b in self.building.values())

    # -- deblurs ----------------------------------------------------------------------
    def _launch_deblurs(self):
        cap = self.eng.max_batch_sources
        for key, q in self.pending_deblurs.items():
            if not q:
                continue
            res = self.resident.get(key)
            if res is None:
                if not self._building_key(key):
                    while q:
                        self._finish(q.popleft(), "rejected")
                continue
            while q:
                batch, total = [], 0
                while q and total + q[0].ns <= cap:
                    r = q.popleft()
                    batch.append(r)
                    total += r.ns
                if not batch:                          # a single request above the cap
                    self._finish(q.popleft(), "rejected")
                    continue
                ticket = self.eng.deblur(res.handle, batch)
                res.inflight += 1
                res.last_use = self.now()
                self.inflight.append((ticket, batch, res))

    def _finish_deblurs(self):
        keep = []
        for ticket, batch, res in self.inflight:
            if not self.eng.ready(ticket):
                keep.append((ticket, batch, res))
                continue
            for i, r in enumerate(batch):
                if self.keep_results:
                    self.results[r.rid] = self.eng.result(ticket, i)
                self._finish(r, "done")
            res.inflight -= 1
        self.inflight = keep

    def _finish(self, req, status):
        req.status = status
        req.t_done = self.now()

    # -- loop -------------------------------------------------------------------------
    def busy(self) -> bool:
        return bool(self.pending_builds or self.building or self.inflight or self.retiring or any(
            q for q in self.pending_deblurs.values()))

    def step(self):
        self._finish_builds()
        self._finish_deblurs()
        self._retire()
        self._admit_builds()
        self._launch_deblurs()

    def run(self, requests: List[Request], progress: Optional[Callable[[float], None]] = None,
            progress_s: float = 10.0) -> List[Request]:
        """Serve ``requests`` (arrival times relative to the start of this call)
        until all have finished; ``progress(t)`` is called every ``progress_s``."""
        self.t0 = self.clock()
        todo = collections.deque(sorted(requests, key=lambda r: r.arrival))
        next_report = progress_s
        while todo or self.busy():
            if progress is not None and self.now() >= next_report:
                progress(self.now())
                next_report += progress_s
            t = self.now()
            while todo and todo[0].arrival <= t:
                r = todo.popleft()
                if r.kind == "build":
                    self.pending_builds.append(r)
                else:
                    self.pending_deblurs[r.key].append(r)
            self.step()
            time.sleep(self.tick_s)
        return requests

    def close(self):
        self.pool.shutdown(wait=True)
        self._finish_builds()
        while self.inflight:
            self._finish_deblurs()
            time.sleep(self.tick_s)
        for r in list(self.resident.values()) + self.retiring:
            self.eng.free(r.handle)
            self._release(r.nbytes)
        self.resident.clear()
        self.retiring = []


def latency_stats(requests: List[Request]) -> dict:
    """p50/p99 latency (ms) of finished requests per kind and overall, and counts."""
    out = {}
    for kind in ("build", "deblur", "all"):
        lat = [r.t_done - r.arrival for r in requests
               if r.status == "done" and (kind == "all" or r.kind == kind)]
        if lat:
            out[kind] = {"n": len(lat), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                         "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3)}
    for st in ("failed", "rejected"):
        n = sum(1 for r in requests if r.status == st)
        if n:
            out[st] = n
    return out


class EhiEngine:
    """libehi on one GPU.  The deblur stream is created before the build streams
    and every build slot owns one stream, so the deblur stream never shares a
    hardware queue with a build when streams are spread over a few queues.
    Builds run in worker threads; each library call releases the interpreter
    lock, so the scheduler keeps ticking while a build enqueues its launches."""

    def __init__(self, specs, build_slots: int = 2, precision: str = "split_bf16",
                 staging_budget_bytes: int = 6 << 30, max_batch_sources: int = 1024,
                 tune: bool = False, device=None):
        import torch
        from . import autotune, batch, ehi
        import synth
        self._torch, self._ehi, self._synth, self._autotune = torch, ehi, synth, autotune
        self._nrb = batch.staging_receivers
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.specs = list(specs)
        self.precision = precision
        self.staging = staging_budget_bytes
        self.max_batch_sources = max_batch_sources
        self.tune = tune
        self.deblur_stream = torch.cuda.Stream(self.device)
        self.build_streams = [torch.cuda.Stream(self.device) for _ in range(build_slots)]
        self.vels = [torch.from_numpy(s.velocity()).to(self.device) for s in self.specs]
        self._ws = {}
        torch.cuda.synchronize(self.device)

    def workspace_bytes(self, key) -> int:
        if key not in self._ws:
            s = self.specs[key]
            self._ws[key] = self._ehi.workspace_bytes(
                nz=s.nz, nx=s.nx, nb=s.nb, h=s.h, dt=s.dt, nt=s.nt, stride=s.stride,
                rec_iz=s.rec_iz, rec_ix=s.rec_ix, freqs_hz=s.freqs_hz, precision=self.precision,
                max_ns=self.max_batch_sources, nr_batch=self._nrb(s, self.staging)) + 256
        return self._ws[key]

    def build(self, key, slot):
        torch = self._torch
        spec = self.specs[key]
        st = self.build_streams[slot]
        with torch.cuda.device(self.device), torch.cuda.stream(st):
            sv = self._ehi.survey_from(spec, precision=self.precision, max_ns=self.max_batch_sources,
                                       nr_batch=self._nrb(spec, self.staging), stream=st)
            try:
                if self.tune:
                    self._autotune.apply(sv, spec)
                sv.build_green(self.vels[key])
                sv.build_hessian()
                sv.factor(1e-3 * sv.lambda_max())
                st.synchronize()
            except Exception:
                st.synchronize()
                sv.close(sync=False)
                raise
        return sv

    def deblur(self, sv, reqs):
        torch = self._torch
        ds = self.deblur_stream
        with torch.cuda.device(self.device), torch.cuda.stream(ds):
            parts = [self._synth.residuals_device(sv.nf, r.ns, sv.nr, r.seed, self.device) for r in reqs]
            R = parts[0] if len(parts) == 1 else torch.cat(parts, dim=1)
            X = sv.apply_multipliers(R, stream=ds)
            ev = torch.cuda.Event()
            ev.record(ds)
        offs = np.cumsum([0] + [r.ns for r in reqs])
        return (ev, X, offs)

    def ready(self, ticket) -> bool:
        return ticket[0].query()

    def result(self, ticket, i):
        _, X, offs = ticket
        return X[:, offs[i]:offs[i + 1]].clone()

    def alone(self, sv, req):
        """The multipliers of one request solved by itself (same stream)."""
        t = self.deblur(sv, [req])
        t[0].synchronize()
        return self.result(t, 0)

    def free(self, sv):
        # the scheduler frees a survey only after its build stream was synchronised
        # and every deblur event against it has completed: no device-wide wait
        sv.close(sync=False)
