"""Batched uneven surveys: graph-captured builds on per-survey streams and the
one-launch factorisation, against the per-survey path and the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import fd, hessian, solve

from parity import check  # noqa: E402

pytestmark = pytest.mark.gpu


def _specs():
    return [synth.tiny().with_(nt=300), synth.ragged(), synth.micro(nz=40, nx=60, nb=6, nt=250, nr=6, stride=2)]


@pytest.fixture(scope="module")
def mods():
    from paper_2512_16642_amd import batch, ehi
    ehi.lib()
    return ehi, batch


def test_graph_batch_matches_eager_and_oracle(mods):
    ehi, batch = mods
    specs = _specs()
    vels = [torch.from_numpy(s.velocity()).cuda() for s in specs]
    # eager, one survey at a time on the current stream
    H_eager = []
    for s, v in zip(specs, vels):
        sv = ehi.survey_from(s)
        sv.build_green(v)
        sv.build_hessian()
        H_eager.append(sv.copy_hessian().cpu().numpy())
        sv.close()
    b = batch.SurveyBatch(specs)
    for rep in range(3):
        b.build(vels, graph=True)
        torch.cuda.synchronize()
        for k, sv in enumerate(b.surveys):
            np.testing.assert_array_equal(sv.copy_hessian().cpu().numpy(), H_eager[k])
        # eager work between replays
        torch.ones(1 << 20, device="cuda").sum().item()
    # one-launch factorisation against per-survey factors
    lam = b.lambda_max()
    mu = [1e-3 * l for l in lam]
    b.factor(mu)
    R = [torch.from_numpy(s.residuals()).cuda() for s in specs]
    X = [x.cpu().numpy() for x in b.apply(R)]
    torch.cuda.synchronize()
    for k, s in enumerate(specs):
        sv = ehi.survey_from(s)
        sv.load_hessian(torch.from_numpy(H_eager[k]).cuda())
        sv.factor(mu[k])
        Xk = sv.apply_multipliers(R[k]).cpu().numpy()
        np.testing.assert_array_equal(Xk, X[k])
        sv.close()
    # oracle end to end for the first survey (same mu)
    s = specs[0]
    Ho = hessian.hessian_r1(fd.green_dft(s, s.velocity()))
    Xo = solve.multipliers(Ho, mu[0], s.residuals().astype(np.complex128))
    check(X[0], Xo, 1e-5, 1e-5, 2e-5, "batch survey 0 multipliers")
    b.close()


def test_factor_batch_reports_failing_survey(mods):
    ehi, batch = mods
    specs = _specs()
    hs = []
    for k, s in enumerate(specs):
        sv = ehi.survey_from(s)
        H = np.zeros((s.nf, s.nr, s.nr), dtype=np.complex128)
        H[:] = np.eye(s.nr)
        if k == 1:
            H[1] = -np.eye(s.nr)
        sv.load_hessian(torch.from_numpy(H).cuda())
        hs.append(sv)
    with pytest.raises(ehi.EhiError) as e:
        ehi.factor_batch(hs, [1e-2] * len(hs))
    assert e.value.status == ehi.EHI_ENOTPD
    assert e.value.bad_survey == 1 and e.value.bad_freq == 1
    # the other surveys are factored and usable
    R = torch.from_numpy(specs[0].residuals()).cuda()
    X = hs[0].apply_multipliers(R).cpu().numpy()
    np.testing.assert_allclose(X, R.cpu().numpy() / (1 + 1e-2), rtol=1e-6, atol=1e-7)
    with pytest.raises(ehi.EhiError):
        hs[1].apply_multipliers(torch.from_numpy(specs[1].residuals()).cuda())
    for sv in hs:
        sv.close()


def test_largest_batch_survey_sampled_against_oracle(mods):
    # the batch's largest survey (1700 x 350 grid, 400 receivers, 40
    # frequencies over 3-20 Hz) on a short record: every stage at its real
    # size, including the whole-matrix contraction's 4 x 4 tiles of block
    # pairs (receivers past 224); six receivers spread over different 32-row
    # blocks and tiles are checked against the oracle's Green functions and the
    # Hessian block among them, and all multipliers against the oracle's solve
    # of the GPU's Hessian
    ehi, _ = mods
    s = synth.batch_survey(1, nt=64)
    v = s.velocity()
    sample = [0, 57, 130, 229, 311, 399]
    sv = ehi.survey_from(s, precision="split_bf16")
    sv.build_green(torch.from_numpy(v).cuda())
    sv.build_hessian()
    G = sv.copy_green_dft().reshape(s.nf, s.nr, -1)
    H = sv.copy_hessian()
    # the deblur of all 400 sources at 40 frequencies from this Hessian,
    # against the oracle's solve of the same Hessian
    Hn = H.cpu().numpy()
    mu = 1e-3 * solve.lambda_max(Hn)
    sv.factor(mu)
    R = s.residuals()
    X = sv.apply_multipliers(torch.from_numpy(R).cuda()).cpu().numpy()
    sv.close()
    Xo = solve.multipliers(Hn, mu, R.astype(np.complex128))
    check(X, Xo, 1e-7, 1.5e-7, 2e-7, "batch survey 1 (400 receivers, 400 sources) multipliers from its Hessian")
    Gs = G[:, sample].cpu().numpy()
    Hs = H[:, sample][:, :, sample].cpu().numpy()
    Go = fd.green_dft(s, v, receivers=sample)
    Ho = np.stack([Go[f] @ Go[f].conj().T for f in range(s.nf)])
    check(Gs, Go, 5e-6, 5e-6, 2e-5, "batch survey 1 (400 receivers) sampled ghat")
    check(Hs, Ho, 1e-5, 1e-5, 2e-5, "batch survey 1 (400 receivers) sampled Hhat block")
