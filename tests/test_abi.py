"""The C-ABI library loads on a machine without a GPU and exports every entry
point declared in include/roeam.h; argument errors need no device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "roeam.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(roeam_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("roeam_residual", "roeam_step", "roeam_batch_submit", "roeam_batch_poll"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    import paper_1711_09272_amd as P
    L = P.lib()
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing
    assert sorted(P.EXPORTS) == declared_symbols()


def test_null_arguments_are_rejected_without_a_device():
    import paper_1711_09272_amd as P
    L = P.lib()
    assert L.roeam_ctx_destroy(None) == P.EINVAL
    assert L.roeam_grid_destroy(None) == P.EINVAL
    assert L.roeam_residual(None, None, None, None, None, None) == P.EINVAL
    assert L.roeam_step(None, None, None, None, 1, 0.0, 0.0, None) == P.EINVAL
    assert L.roeam_grid_layout(None, None, None, None) == P.EINVAL
    assert L.roeam_grid3d_destroy(None) == P.EINVAL
    assert L.roeam_residual3d(None, None, None, None, None, None) == P.EINVAL
    assert L.roeam_step3d(None, None, None, None, 1, 0.0, 0.0, None) == P.EINVAL
    assert L.roeam_grid3d_layout(None, None, None, None, None) == P.EINVAL
    assert L.roeam_last_error(None) == b"NULL context"
    h = ctypes.c_void_p()
    assert L.roeam_ctx_create(0, None, None) == P.EINVAL
