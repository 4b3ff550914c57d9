"""Serving on the GPU: every deblur's multipliers are the same alone and inside
the Poisson mix (merged with other requests, concurrent with rebuilds), and
match the oracle for one sampled request.

Mix: three small surveys (two 101 x 101 tiny variants with 16 and 12
receivers, one ragged 41 x 61), all resident at the start; Poisson arrivals at
40 req/s for 2 s, 15 % rebuilds, deblurs of U{1..64} sources.  Rebuilt factors
are bitwise those they replace (the build is deterministic), so the "alone"
solve against the final factors must reproduce each mixed result exactly.
"""
import numpy as np
import pytest
import torch

import synth

from parity import check  # noqa: E402

pytestmark = pytest.mark.gpu


def _specs():
    t = synth.tiny()
    return [t, t.with_(name="tiny-nr12", rec_iz=t.rec_iz[:12], rec_ix=t.rec_ix[2:14]),
            synth.ragged(nz=41, nx=61, nb=8, nt=200, nr=5, stride=2)]


@pytest.fixture(scope="module")
def served():
    from paper_2512_16642_amd import ehi, serve
    ehi.lib()
    specs = _specs()
    eng = serve.EhiEngine(specs, build_slots=2, max_batch_sources=256)
    srv = serve.Server(eng, budget_bytes=8 << 30, build_slots=2, keep_results=True)
    srv.preload(range(len(specs)))
    reqs = serve.poisson_requests(2.0, 40.0, 0.15, len(specs), ns_max=64, seed=2400)
    srv.run(reqs)
    torch.cuda.synchronize()
    yield specs, eng, srv, reqs
    srv.close()


def test_mix_ran_with_rebuilds_and_merges(served):
    specs, eng, srv, reqs = served
    kinds = {k: sum(1 for r in reqs if r.kind == k) for k in ("build", "deblur")}
    assert kinds["build"] >= 3 and kinds["deblur"] >= 40
    assert all(r.status == "done" for r in reqs), [(r.rid, r.kind, r.status) for r in reqs if r.status != "done"]
    assert srv.adm.peak <= srv.adm.budget
    print("serve mix:", serve_stats(reqs))


def serve_stats(reqs):
    from paper_2512_16642_amd import serve
    return serve.latency_stats(reqs)


def test_each_result_same_alone_and_in_mix(served):
    specs, eng, srv, reqs = served
    n = 0
    for r in reqs:
        if r.kind != "deblur":
            continue
        alone = eng.alone(srv.resident[r.key].handle, r)
        mixed = srv.results[r.rid]
        assert mixed.shape == (specs[r.key].nf, r.ns, specs[r.key].nr)
        assert torch.equal(alone, mixed), r
        n += 1
    assert n >= 40


def test_one_served_request_matches_oracle(served):
    from oracle import fd, hessian, solve
    specs, eng, srv, reqs = served
    r = next(q for q in reqs if q.kind == "deblur" and q.key == 0)
    s = specs[0]
    G = fd.green_dft(s, s.velocity())
    H = hessian.hessian_r1(G)
    mu = 1e-3 * solve.lambda_max(H)
    R = synth.residuals_device(s.nf, r.ns, s.nr, r.seed, "cuda").cpu().numpy().astype(np.complex128)
    Xr = solve.multipliers(H, mu, R)
    X = srv.results[r.rid].cpu().numpy()
    check(X, Xr, 1e-5, 1e-5, 2e-5, "served request vs oracle")


@pytest.fixture(scope="module")
def served_tight():
    # a budget that holds exactly the three resident surveys: every rebuild must
    # evict the least recently used factors (its own old ones included), and
    # deblurs for a survey that is neither resident nor being rebuilt are
    # rejected
    from paper_2512_16642_amd import ehi, serve
    ehi.lib()
    specs = _specs()
    eng = serve.EhiEngine(specs, build_slots=2, max_batch_sources=256)
    budget = sum(eng.workspace_bytes(k) for k in range(len(specs)))
    srv = serve.Server(eng, budget_bytes=budget, build_slots=2, keep_results=True)
    srv.preload(range(len(specs)))
    reqs = serve.poisson_requests(2.0, 40.0, 0.15, len(specs), ns_max=64, seed=2401)
    srv.run(reqs)
    torch.cuda.synchronize()
    yield specs, eng, srv, reqs
    srv.close()


def test_tight_budget_evicts_and_stays_within_it(served_tight):
    specs, eng, srv, reqs = served_tight
    assert srv.evictions > 0
    assert srv.adm.peak <= srv.adm.budget
    assert all(r.status in ("done", "rejected") for r in reqs), [(r.rid, r.kind, r.status) for r in reqs]
    assert all(r.status == "done" for r in reqs if r.kind == "build")
    done = [r for r in reqs if r.kind == "deblur" and r.status == "done"]
    assert len(done) >= 20
    print("tight budget:", srv.evictions, "evictions,",
          sum(1 for r in reqs if r.status == "rejected"), "rejected deblurs")


def test_tight_budget_results_same_as_fresh_factors(served_tight):
    # the build is deterministic, so factors built afresh are bitwise those
    # every served deblur used, whether or not they were evicted since
    specs, eng, srv, reqs = served_tight
    fresh = {}
    try:
        for r in reqs:
            if r.kind != "deblur" or r.status != "done":
                continue
            if r.key not in fresh:
                fresh[r.key] = eng.build(r.key, 0)
            assert torch.equal(eng.alone(fresh[r.key], r), srv.results[r.rid]), r
    finally:
        for sv in fresh.values():
            sv.close()
