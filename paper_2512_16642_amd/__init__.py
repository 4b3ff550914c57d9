"""MI355X-native data-space Hessian build and inversion (arXiv 2512.16642).

The compute path is the HIP library ``libehi.so`` (C ABI in include/ehi.h);
``paper_2512_16642_amd.ehi`` is its Python binding.
"""
from .ehi import EhiError, Survey, lib, survey_from, workspace_bytes  # noqa: F401
