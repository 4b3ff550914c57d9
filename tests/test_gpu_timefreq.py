"""The steps either side of the deblur and the accuracy test on the GPU,
against the oracle.

Forward modelling S and its transpose on the subgrid sources (ragged grid,
subgrid stride 2, several fields per batch), the residual spectra (ragged
record length), the inverse 2nt-point transform (bins 0 and nt included),
adjointness at two sizes, and the whole accuracy test at full band against the
oracle's run of the same steps.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fd, hessian, solve, timefreq

pytestmark = pytest.mark.gpu


from parity import check, rel  # noqa: E402


@pytest.fixture(scope="module")
def ehi():
    from paper_2512_16642_amd import ehi as mod
    mod.lib()
    return mod


def _ragged():
    return synth.ragged()  # 45 x 77, nt = 157, 5 receivers, stride 2


def _op(s):
    return fd.ForwardOperator(s.velocity(), s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, s.stride)


def _medium_survey(ehi, s, nr_batch=2):
    sv = ehi.survey_from(s, nr_batch=nr_batch)
    sv.set_medium(torch.from_numpy(s.velocity().astype(np.float32)).cuda())
    return sv


def test_forward_subgrid_matches_oracle(ehi):
    s = _ragged()
    f = synth.subgrid_sources(3, s.nt, s.nzs, s.nxs, seed=31)
    sv = _medium_survey(ehi, s)                       # 3 fields in batches of 2
    d = sv.forward_subgrid(torch.from_numpy(f).cuda()).cpu().numpy()
    sv.close()
    op = _op(s)
    ref = np.stack([op.apply(f[k].astype(np.float64)) for k in range(3)])
    check(d, ref, 2e-6, 2e-6, 4e-6, "forward S")


def test_backpropagate_matches_oracle(ehi):
    s = _ragged()
    x = synth.time_residuals(3, s.nr, s.nt, seed=32)
    sv = _medium_survey(ehi, s)
    db = sv.backpropagate(torch.from_numpy(x).cuda()).cpu().numpy()
    sv.close()
    op = _op(s)
    ref = np.stack([op.adjoint(x[k].astype(np.float64)) for k in range(3)])
    check(db.reshape(ref.shape), ref, 2e-6, 2e-6, None, "adjoint S^T")


def test_modelling_needs_a_medium(ehi):
    s = _ragged()
    sv = ehi.survey_from(s)
    with pytest.raises(ehi.EhiError) as e:
        sv.forward_subgrid(torch.zeros((1, s.nt, s.nzs, s.nxs), device="cuda"))
    assert e.value.status == ehi.EHI_ESTATE
    sv.close()


@pytest.mark.parametrize("case", ["tiny", "ragged"])
def test_residual_spectra_match_oracle(ehi, case):
    s = synth.tiny() if case == "tiny" else _ragged()
    dd = synth.time_residuals(5, s.nr, s.nt, seed=33)
    sv = ehi.survey_from(s)
    R = sv.residual_spectra(torch.from_numpy(dd).cuda()).cpu().numpy()
    sv.close()
    ref = timefreq.residual_spectra(dd, s.freqs_hz, s.dt)
    check(R, ref, 3e-7, 3e-7, 6e-7, f"{case} residual spectra")


def test_inverse_transform_matches_oracle(ehi):
    base = _ragged()
    s = base.with_(freqs_hz=synth.transform_bins(base.nt, base.dt, (0, 1, 7, 30, 78, 156, 157)))
    rng = np.random.default_rng(34)
    X = (rng.standard_normal((s.nf, 70, s.nr)) + 1j * rng.standard_normal((s.nf, 70, s.nr))).astype(np.complex64)
    sv = ehi.survey_from(s)
    x = sv.multipliers_to_time(torch.from_numpy(X).cuda()).cpu().numpy()
    sv.close()
    ref = timefreq.to_time(X.astype(np.complex128), s.freqs_hz, s.dt, s.nt)
    check(x, ref, 3e-7, 3e-7, 6e-7, "inverse transform")


def test_inverse_transform_rejects_off_bin_frequencies(ehi):
    s = _ragged()  # 4, 7.5, 11 Hz are not bins for nt = 157, dt = 1 ms
    sv = ehi.survey_from(s)
    with pytest.raises(ehi.EhiError) as e:
        sv.multipliers_to_time(torch.zeros((s.nf, 1, s.nr), dtype=torch.complex64, device="cuda"))
    assert e.value.status == ehi.EHI_EINVAL
    sv.close()


def _adjointness(ehi, s, ns, seed):
    f = torch.from_numpy(synth.subgrid_sources(ns, s.nt, s.nzs, s.nxs, seed)).cuda()
    d = torch.from_numpy(synth.time_residuals(ns, s.nr, s.nt, seed + 1)).cuda()
    sv = _medium_survey(ehi, s, nr_batch=ns)
    Sf = sv.forward_subgrid(f)
    STd = sv.backpropagate(d)
    torch.cuda.synchronize()
    sv.close()
    out = []
    for k in range(ns):
        a = float(torch.dot(Sf[k].double().flatten(), d[k].double().flatten()))
        b = float(torch.dot(f[k].double().flatten(), STd[k].double().flatten()))
        scale = float(Sf[k].double().norm() * d[k].double().norm())
        out.append(abs(a - b) / scale)
    return out


def test_adjointness_tiny(ehi):
    errs = _adjointness(ehi, synth.tiny(), 2, seed=35)
    print("tiny <Sf, d> vs <f, S^T d>", errs)
    assert max(errs) < 1e-6


def test_adjointness_full_size(ehi):
    # the 1000 x 300 layered grid with its 200 receivers, nt = 4000, subgrid stride 2
    errs = _adjointness(ehi, synth.layered_1000x300(), 1, seed=36)
    print("1000x300 <Sf, d> vs <f, S^T d>", errs)
    assert max(errs) < 1e-6


def test_accuracy_test_matches_oracle(ehi):
    s = synth.accuracy_micro()                        # all 61 bins of nt = 60
    v = s.velocity()
    ns = 3
    dd = synth.time_residuals(ns, s.nr, s.nt, seed=37)
    d_obs = dd + synth.time_residuals(ns, s.nr, s.nt, seed=38)
    G = fd.green_dft(s, v)
    H = hessian.hessian_r1(G)
    mu = 1e-2 * solve.lambda_max(H)
    dde_r, db_r, pred_r, err_r, relerr_r = timefreq.accuracy_test(_op(s), H, mu, dd.astype(np.float64),
                                                                  d_obs, s.freqs_hz, s.dt)
    sv = ehi.survey_from(s, nr_batch=2)
    sv.build_green(torch.from_numpy(v.astype(np.float32)).cuda())
    sv.build_hessian()
    sv.factor(mu)
    ddg = torch.from_numpy(dd).cuda()
    X = sv.apply_multipliers(sv.residual_spectra(ddg))
    dde = sv.multipliers_to_time(X)
    db = sv.backpropagate(dde)
    pred = sv.forward_subgrid(db)
    err, relerr = ehi.misfit(ddg, pred, torch.from_numpy(d_obs).cuda())
    out = [t.cpu().numpy() for t in (dde, db, pred, err, relerr)]
    sv.close()
    e = {"dde": rel(out[0], dde_r), "db": rel(out[1].reshape(db_r.shape), db_r),
         "pred": rel(out[2], pred_r), "err": rel(out[3], err_r),
         "relerr": float(np.max(np.abs(out[4] - relerr_r) / relerr_r))}
    print("accuracy test vs oracle:", e, "| RelErr", out[4], "oracle", relerr_r)
    assert e["dde"] < 1e-6 and e["db"] < 5e-6 and e["pred"] < 5e-6
    assert e["err"] < 5e-6 and e["relerr"] < 1e-6
    # element-wise beside the norms (per source)
    check(out[0], dde_r, 1e-6, 1e-6, None, "accuracy test: multipliers in time")
    check(out[1].reshape(db_r.shape), db_r, 5e-6, 5e-6, None, "accuracy test: source extension")
    check(out[2], pred_r, 5e-6, 5e-6, None, "accuracy test: prediction")
    check(out[3], err_r, 5e-6, 5e-6, None, "accuracy test: data error")


@pytest.mark.parametrize("case", ["shared_cell", "four_levels"])
def test_single_level_fallback_matches_oracle(ehi, case):
    # receivers sharing a cell (the receiver map holds one index per cell) or a
    # 4-level launch shape: S and S^T step one level per launch instead
    s = _ragged()
    if case == "shared_cell":
        s = s.with_(rec_iz=s.rec_iz[:4] + (s.rec_iz[1],), rec_ix=s.rec_ix[:4] + (s.rec_ix[1],))
    f = synth.subgrid_sources(2, s.nt, s.nzs, s.nxs, seed=51)
    x = synth.time_residuals(2, s.nr, s.nt, seed=52)
    sv = _medium_survey(ehi, s)
    if case == "four_levels":
        sv.set_launch(4, 0, 0)
    d = sv.forward_subgrid(torch.from_numpy(f).cuda()).cpu().numpy()
    db = sv.backpropagate(torch.from_numpy(x).cuda()).cpu().numpy()
    sv.close()
    op = _op(s)
    ref_f = np.stack([op.apply(f[k].astype(np.float64)) for k in range(2)])
    ref_b = np.stack([op.adjoint(x[k].astype(np.float64)) for k in range(2)])
    check(d, ref_f, 2e-6, 2e-6, 4e-6, f"{case} fallback S")
    check(db.reshape(ref_b.shape), ref_b, 2e-6, 2e-6, None, f"{case} fallback S^T")


def test_march_modelling_independent_of_launch_shape(ehi):
    # the modelling march gives the same bits for every band width and segment
    # height (the segment height of a modelling run is its own choice)
    s = _ragged().with_(nx=700)
    f = torch.from_numpy(synth.subgrid_sources(2, s.nt, s.nzs, s.nxs, seed=53)).cuda()
    x = torch.from_numpy(synth.time_residuals(2, s.nr, s.nt, seed=54)).cuda()
    ref = None
    for band in (256, 384, 448, 512):
        sv = _medium_survey(ehi, s)
        sv.set_launch(8, 0, band)
        out = (sv.forward_subgrid(f).cpu().numpy(), sv.backpropagate(x).cpu().numpy())
        sv.close()
        if ref is None:
            ref = out
        else:
            np.testing.assert_array_equal(out[0], ref[0], err_msg=f"S band {band}")
            np.testing.assert_array_equal(out[1], ref[1], err_msg=f"S^T band {band}")
