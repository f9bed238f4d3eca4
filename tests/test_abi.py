"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, and rejects invalid arguments synchronously (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2508_18114_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "lr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lr_[a-z_]+)\s*\(", src)) - {"lr_c64"})


def test_library_exports_every_declared_symbol():
    from paper_2508_18114_amd import lr
    lib = ctypes.CDLL(lr.LIB_PATH)
    decl = _declared_symbols()
    assert decl, "no declarations parsed"
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(lr.EXPORTS)


def test_init_validation_and_workspace():
    from paper_2508_18114_amd import lr
    m = I.readout_model(8, 50, 5)
    h = lr.lr_init(m, 20)
    try:
        nb = lr.lr_workspace_bytes(h)
        # four N x M FP64 complex state arrays at least
        assert nb >= 4 * m.N * 20 * 16
        # unbound context: call order error, nothing enqueued
        assert lr.lr_integrate(h, I.flattop_pulse(0.05, 10.0), 0.0, 1e-3, 10, 1, 0, 0) == lr.LR_ERR_STATE
        assert lr.lr_status(h)[0] == lr.LR_ERR_STATE
    finally:
        lr.lr_destroy(h)
    for bad in (dict(d_q=1), dict(d_r=0), dict(d_f=0)):
        with pytest.raises(lr.LrError) as ei:
            lr.lr_init(m.replace(**bad), 4)
        assert ei.value.code == lr.LR_ERR_ARG
    for M in (0, 33, -1):
        with pytest.raises(lr.LrError):
            lr.lr_init(m, M)
    with pytest.raises(lr.LrError):
        lr.lr_init(I.readout_model(2, 1, 1), 3)          # M > N
    with pytest.raises(lr.LrError):
        lr.lr_init(m.replace(kappa_f=-1.0), 4)
    with pytest.raises(lr.LrError):
        lr.lr_init(m, 4, precision=7)


def test_strerror_is_total():
    from paper_2508_18114_amd import lr
    for code in range(-8, 1):
        assert isinstance(lr.lr_strerror(code), str)
