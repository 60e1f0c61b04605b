"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, and fails cleanly without a device."""
import ctypes as C
import os
import re

import pytest

import paper_2008_05858_amd as P
from paper_2008_05858_amd import e2e as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "e2e.h")).read()
    return sorted(set(re.findall(r"\b(e2e_[a-z_]+)\s*\(", txt)))


def test_header_declares_expected_api():
    fns = header_functions()
    for need in ["e2e_format_load", "e2e_psf_load", "e2e_render", "e2e_render_batch",
                 "e2e_serve_submit", "e2e_serve_poll"]:
        assert need in fns


def test_library_exports_every_declared_symbol():
    L = C.CDLL(E.LIB_PATH)
    missing = [f for f in header_functions() if not hasattr(L, f)]
    assert not missing, missing
    assert sorted(E.EXPORTS) == header_functions()


def test_version_and_error_string():
    assert "gfx950" in E.e2e_version()
    assert isinstance(E.e2e_last_error(), str)


def test_null_arguments_are_rejected_without_device():
    L = P.lib()
    assert L.e2e_create(None, 0, 0) == E.E2E_EINVAL
    assert L.e2e_format_load(None, None, 0, 0, 0, None) == E.E2E_EINVAL
    assert L.e2e_psf_load(None, None, None) == E.E2E_EINVAL
    assert L.e2e_render(None, None) == E.E2E_EINVAL
    assert L.e2e_render_batch(None, None, 1) == E.E2E_EINVAL
    assert L.e2e_serve_poll(None, 1, 0, None) == E.E2E_EINVAL
    assert L.e2e_noise_poisson(None, None, 0, 1, 0, 0, 0, None) == E.E2E_EINVAL
    assert L.e2e_detector(None, None, None, 0, None, 1, 1, None, 0, None) == E.E2E_EINVAL
    assert L.e2e_extract(None, 1, None, 0, 1.0, None, None, 0, None) == E.E2E_EINVAL
    assert L.e2e_ccf(None, 1, None, None) == E.E2E_EINVAL
    assert L.e2e_autotune(None, None, 1, None) == E.E2E_EINVAL
    assert "NULL" in E.e2e_last_error() or "bad arguments" in E.e2e_last_error()
    L.e2e_destroy(None)


def test_create_reports_missing_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.E2EError) as ei:
        E.e2e_create(0, 0)
    assert ei.value.code in (E.E2E_EDEVICE, E.E2E_EINVAL)
