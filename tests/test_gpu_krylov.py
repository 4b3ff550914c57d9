"""The Krylov baselines on the GPU (CG and GMRES on Q x = dd with two PDE
solves per iteration) against the oracle's CG and GMRES and the dense
time-domain solve.

Micro survey with every bin of nt = 60 (4 receivers, 24 x 30 grid), two
records in one batch.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fd, hessian, krylov

pytestmark = pytest.mark.gpu


from parity import check, rel  # noqa: E402


@pytest.fixture(scope="module")
def system():
    from paper_2512_16642_amd import ehi
    ehi.lib()
    s = synth.accuracy_micro()
    v = s.velocity()
    op = fd.ForwardOperator(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, s.stride)
    gt = fd.green_samples(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1).reshape(s.nr, s.nt, -1)
    Q0 = hessian.time_domain_matrix(gt, 0.0)
    mu = 1e-2 * float(np.linalg.eigvalsh(Q0)[-1])
    dd = synth.time_residuals(2, s.nr, s.nt, seed=41)
    sv = ehi.survey_from(s, nr_batch=2)
    sv.set_medium(torch.from_numpy(v.astype(np.float32)).cuda())
    yield s, op, Q0, mu, dd, sv
    sv.close()


def test_cg_iterates_match_oracle(system):
    from paper_2512_16642_amd import krylov as gk
    s, op, Q0, mu, dd, sv = system
    out = gk.cg(sv, torch.from_numpy(dd).cuda(), mu, maxiter=6)
    x = out["x"].cpu().numpy()
    assert out["iterations"] == 6 and out["pde_solves"] == 24
    errs = []
    for k in range(2):
        xr, it, _ = krylov.cg(op, dd[k].astype(np.float64), mu, tol=0.0, maxiter=6)
        assert it == 6
        errs.append(rel(x[k], xr))
    print("CG iterate (6 iterations) vs oracle CG", errs)
    assert max(errs) < 1e-6


def test_cg_converges_to_dense_solve_and_fit_identity(system):
    from paper_2512_16642_amd import krylov as gk
    s, op, Q0, mu, dd, sv = system
    obs2 = torch.tensor([float(np.sum(dd[k].astype(np.float64) ** 2)) for k in range(2)], dtype=torch.float64)
    out = gk.cg(sv, torch.from_numpy(dd).cuda(), mu, maxiter=80, obs_norm2=obs2)
    x = out["x"].cpu().numpy()
    hist = torch.stack(out["relerr_history"]).numpy()
    n = Q0.shape[0]
    for k in range(2):
        xs = np.linalg.solve(Q0 + mu * np.eye(n), dd[k].astype(np.float64).reshape(-1)).reshape(s.nr, s.nt)
        e = rel(x[k], xs)
        # the exact solution's misfit is mu x (Hessian accuracy test identity)
        fit_exact = mu * mu * float(np.sum(xs ** 2)) / float(obs2[k])
        print(f"record {k}: CG vs dense solve {e:.2e}; RelErr {hist[-1][k]:.6e} vs mu^2|x|^2/|d|^2 {fit_exact:.6e}")
        assert e < 1e-5
        assert abs(hist[-1][k] - fit_exact) <= 1e-5 * fit_exact
        # the fit the update kernel reports is |dd - S S^T x|^2 of its own iterate
        direct = float(np.sum((dd[k] - op.apply(op.adjoint(x[k].astype(np.float64)))) ** 2)) / float(obs2[k])
        assert abs(hist[-1][k] - direct) <= 1e-3 * direct
    # CG's misfit decreases (up to FP32 noise at the end)
    assert np.all(hist[5] < hist[0])


def test_gmres_iterates_match_oracle(system):
    from paper_2512_16642_amd import krylov as gk
    s, op, Q0, mu, dd, sv = system
    out = gk.gmres(sv, torch.from_numpy(dd).cuda(), mu, m=6)
    x = out["x"].cpu().numpy()
    assert out["iterations"] == 6 and out["pde_solves"] == 24
    errs = []
    for k in range(2):
        xr, it, _, _ = krylov.gmres(op, dd[k].astype(np.float64), mu, m=6, tol=0.0, maxiter=6)
        assert it == 6
        errs.append(rel(x[k], xr))
    print("GMRES iterate (6 iterations) vs oracle GMRES", errs)
    assert max(errs) < 2e-6


def test_gmres_converges_to_dense_solve_and_fit_identity(system):
    from paper_2512_16642_amd import krylov as gk
    s, op, Q0, mu, dd, sv = system
    obs2 = torch.tensor([float(np.sum(dd[k].astype(np.float64) ** 2)) for k in range(2)], dtype=torch.float64)
    out = gk.gmres(sv, torch.from_numpy(dd).cuda(), mu, m=60, obs_norm2=obs2)
    x = out["x"].cpu().numpy()
    hist = torch.stack(out["relerr_history"]).numpy()
    res = np.array(out["residual_history"])
    n = Q0.shape[0]
    for k in range(2):
        xs = np.linalg.solve(Q0 + mu * np.eye(n), dd[k].astype(np.float64).reshape(-1)).reshape(s.nr, s.nt)
        e = rel(x[k], xs)
        fit_exact = mu * mu * float(np.sum(xs ** 2)) / float(obs2[k])
        print(f"record {k}: GMRES vs dense solve {e:.2e}; residual {res[-1][k]:.2e}; "
              f"RelErr {hist[-1][k]:.6e} vs mu^2|x|^2/|d|^2 {fit_exact:.6e}")
        assert e < 1e-5
        assert abs(hist[-1][k] - fit_exact) <= 1e-5 * fit_exact
    # the residual norm of GMRES never increases
    assert np.all(np.diff(res, axis=0) <= 1e-9)
