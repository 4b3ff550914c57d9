"""The C-ABI library loads, exports every declared symbol, and validates
descriptors on the host (no GPU needed: no compute is called)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ehi.h")


def _declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(ehi_[a-z_0-9]+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def ehi():
    from paper_2512_16642_amd import ehi as mod
    return mod


def test_header_symbols_exported(ehi):
    L = ehi.lib()
    decl = _declared_symbols()
    assert len(decl) >= 14, decl
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(ehi.SYMBOLS)


def _desc_kw(**over):
    kw = dict(nz=20, nx=30, nb=5, h=10.0, dt=1e-3, nt=50, stride=1, rec_iz=[1, 2], rec_ix=[3, 4],
              freqs_hz=[5.0, 7.0], precision="split_bf16", max_ns=4, nr_batch=0)
    kw.update(over)
    return kw


def test_workspace_bytes_valid(ehi):
    n = ehi.workspace_bytes(**_desc_kw())
    # at least the three wavefield planes and the Green-function spectra
    Zp, Xp = 20 + 10 + 4, 64
    assert n >= 3 * 2 * Zp * Xp * 4 + 2 * 2 * 20 * 30 * 8


@pytest.mark.parametrize("bad", [
    dict(nz=2), dict(nb=-1), dict(h=0.0), dict(dt=-1.0), dict(nt=0), dict(stride=0), dict(stride=9),
    dict(stride=3), dict(nb=513),
    dict(rec_iz=[1, 20]), dict(rec_ix=[-1, 4]), dict(freqs_hz=[]), dict(freqs_hz=[float("nan")]),
    dict(precision=7), dict(max_ns=0), dict(nr_batch=-3), dict(weighting=2),
    dict(weighting="finite_record", precision="plain_fp32"),
    dict(weighting="finite_record", nr_batch=1), dict(chunk=128), dict(chunk=300),
    dict(keep=(3, 0)), dict(keep=(21, 5)), dict(keep=(5, 31)), dict(keep=(-1, 4)),
    dict(keep=(4, 4), weighting="finite_record"),
])
def test_workspace_bytes_rejects(ehi, bad):
    with pytest.raises(ehi.EhiError) as ei:
        ehi.workspace_bytes(**_desc_kw(**bad))
    assert ei.value.status == ehi.EHI_EINVAL
    assert ehi.lib().ehi_last_error().decode()


def test_finite_record_weighting_accepted_with_all_receivers(ehi):
    a = ehi.workspace_bytes(**_desc_kw())
    b = ehi.workspace_bytes(**_desc_kw(weighting="finite_record"))
    c = ehi.workspace_bytes(**_desc_kw(weighting="finite_record", nr_batch=2))
    assert b > a and c == b   # FP64 partial sums of the finite-record contraction


def test_compression_buffers(ehi):
    a = ehi.workspace_bytes(**_desc_kw())
    b = ehi.workspace_bytes(**_desc_kw(keep=(5, 6)))
    c = ehi.workspace_bytes(**_desc_kw(keep=(20, 30)))
    assert a < b < c


def test_longer_staging_window(ehi):
    a = ehi.workspace_bytes(**_desc_kw())
    assert ehi.workspace_bytes(**_desc_kw(chunk=256)) == a
    assert ehi.workspace_bytes(**_desc_kw(chunk=512)) > a
    assert ehi.workspace_bytes(**_desc_kw(chunk=1024)) > ehi.workspace_bytes(**_desc_kw(chunk=512))


def test_workspace_grows_with_sizes(ehi):
    a = ehi.workspace_bytes(**_desc_kw())
    b = ehi.workspace_bytes(**_desc_kw(nt=500))
    c = ehi.workspace_bytes(**_desc_kw(max_ns=400))
    assert b > a and c > a


def test_create_rejects_null_workspace(ehi):
    d, keep = ehi.make_desc(**_desc_kw())
    out = ctypes.c_void_p()
    st = ehi.lib().ehi_create(ctypes.byref(d), None, 0, None, ctypes.byref(out))
    assert st == ehi.EHI_EINVAL and not out.value


def test_create_rejects_small_workspace(ehi):
    d, keep = ehi.make_desc(**_desc_kw())
    out = ctypes.c_void_p()
    # a bogus aligned address: the size check fails before any device access
    st = ehi.lib().ehi_create(ctypes.byref(d), ctypes.c_void_p(1 << 20), 16, None, ctypes.byref(out))
    assert st == ehi.EHI_ENOMEM and not out.value


def test_null_handle_calls_fail_cleanly(ehi):
    L = ehi.lib()
    assert L.ehi_build_hessian(None) == ehi.EHI_EINVAL
    assert L.ehi_factor(None, ctypes.c_double(1.0), None) == ehi.EHI_EINVAL
    assert L.ehi_destroy(None) == ehi.EHI_OK


def test_modelling_calls_validate_on_the_host(ehi):
    L = ehi.lib()
    assert L.ehi_set_medium(None, None) == ehi.EHI_EINVAL
    assert L.ehi_forward_subgrid(None, None, 0, None) == ehi.EHI_EINVAL
    assert L.ehi_backpropagate(None, None, 0, None) == ehi.EHI_EINVAL
    assert L.ehi_residual_spectra(None, None, 0, None, None) == ehi.EHI_EINVAL
    assert L.ehi_multipliers_to_time(None, None, 0, None, None) == ehi.EHI_EINVAL
    # the misfit needs no survey: empty batches succeed, bad sizes and NULLs fail
    assert L.ehi_misfit(None, None, None, 0, 1, None, None, None) == ehi.EHI_OK
    assert L.ehi_misfit(None, None, None, -1, 1, None, None, None) == ehi.EHI_EINVAL
    assert L.ehi_misfit(None, None, None, 1, 0, None, None, None) == ehi.EHI_EINVAL
    assert L.ehi_misfit(None, None, None, 2, 10, None, None, None) == ehi.EHI_EINVAL


def test_two_staging_windows_double_the_staging(ehi):
    one = ehi.workspace_bytes(**_desc_kw(windows=1))
    two = ehi.workspace_bytes(**_desc_kw(windows=2))
    assert two > one
    with pytest.raises(ehi.EhiError):
        ehi.workspace_bytes(**_desc_kw(windows=3))


def test_cg_calls_validate_on_the_host(ehi):
    L = ehi.lib()
    d = ctypes.c_double(1.0)
    assert L.ehi_cg_init(None, 0, 1, None, None, None, None, None) == ehi.EHI_OK
    assert L.ehi_cg_init(None, 1, 1, None, None, None, None, None) == ehi.EHI_EINVAL
    assert L.ehi_cg_shift_dot(None, None, d, -1, 1, None, None) == ehi.EHI_EINVAL
    assert L.ehi_cg_update(None, None, None, None, None, None, d, 1, 0, None, None, None) == ehi.EHI_EINVAL
    assert L.ehi_cg_direction(None, None, None, None, 2, 5, None) == ehi.EHI_EINVAL


def test_block_calls_validate_on_the_host(ehi):
    L = ehi.lib()
    d = ctypes.c_double(1.0)
    assert L.ehi_mdot(None, 10, 0, None, 0, 10, None, None) == ehi.EHI_OK
    assert L.ehi_mdot(None, 10, -1, None, 1, 10, None, None) == ehi.EHI_EINVAL
    assert L.ehi_mdot(None, 10, 2, None, 1, 10, None, None) == ehi.EHI_EINVAL
    assert L.ehi_combine(None, 10, 2000, None, 1, 10, d, None, None) == ehi.EHI_EINVAL
    assert L.ehi_combine(None, 10, 1, None, 1, 0, d, None, None) == ehi.EHI_EINVAL


def test_compressed_workspace_smaller():
    from paper_2512_16642_amd import ehi as mod
    import synth
    s = synth.layered_1000x300()
    kw = dict(nz=s.nz, nx=s.nx, nb=s.nb, h=s.h, dt=s.dt, nt=s.nt, stride=s.stride, rec_iz=s.rec_iz,
              rec_ix=s.rec_ix, freqs_hz=s.freqs_hz, precision="split_bf16", max_ns=s.ns, nr_batch=50,
              chunk=1024)
    plain = mod.workspace_bytes(**kw)
    comp = mod.workspace_bytes(**kw, keep=(38, 125))
    print("workspace (50-receiver batches): uncompressed %.2f GB, compressed %.2f GB" % (plain / 1e9, comp / 1e9))
    assert comp < plain


def test_hbm_probe_argument_checks():
    import ctypes
    from paper_2512_16642_amd import ehi
    L = ehi.lib()
    p = ctypes.c_void_p(1)
    assert L.ehi_hbm_probe(5, p, p, p, p, p, 1024, 0.0, 4, p, None) == ehi.EHI_EINVAL      # mode
    assert L.ehi_hbm_probe(0, p, p, p, p, p, 1000, 0.0, 4, p, None) == ehi.EHI_EINVAL      # bytes % 16
    assert L.ehi_hbm_probe(3, p, p, p, p, p, 1024, 2.5, 4, p, None) == ehi.EHI_EINVAL      # e_frac
    assert L.ehi_hbm_probe(2, p, None, p, p, p, 1024, 0.0, 4, p, None) == ehi.EHI_EINVAL   # b missing
    assert L.ehi_hbm_probe(1, p, p, p, p, p, 1024, 0.0, 0, p, None) == ehi.EHI_EINVAL      # grid
