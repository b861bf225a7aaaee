"""The C ABI library loads and exports every entry point include/sic.h
declares; argument checks that need no GPU return the documented status."""
import ctypes
import os
import re

import pytest

from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import build as hb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        hb.build()
    return B.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sic.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sic_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B._SIGS), set(names) ^ set(B._SIGS)


def test_version_and_status_strings(lib):
    assert B.sic_abi_version() == B.SIC_ABI_VERSION
    assert B.sic_status_str(0) == "ok"
    assert "order" in B.sic_status_str(4)


def _init_status(**kw):
    import numpy as np

    args = dict(L=1.0, n_cells=8, dt=0.1, n_tracers=[4], q=[0.25], closed=[1], x0=np.arange(4) / 4.0,
                v0=np.zeros(4))
    args.update(kw)
    with pytest.raises(B.SicError) as e:
        B.sic_init(**args)
    return e.value.status


def test_invalid_arguments_are_rejected_before_any_device_work(lib):
    import numpy as np

    assert _init_status(n_cells=0) == 1
    assert _init_status(n_cells=B.SIC_MAX_CELLS + 1) == 1
    assert _init_status(L=-1.0) == 1
    assert _init_status(dt=0.0) == 1
    assert _init_status(n_tracers=[1], x0=np.zeros(1), v0=np.zeros(1)) == 1
    assert _init_status(q=[float("nan")]) == 1
    assert _init_status(precision=7) == 1
    assert _init_status(deposit_order=3) == 6
    assert _init_status(l_max=-1.0) == 1
    assert _init_status(l_max=float("nan")) == 1
    assert _init_status(max_tracers=-5) == 1
    h = ctypes.c_void_p()
    assert lib.sic_init(None, None, 0, None, None, None, 0, None, ctypes.byref(h)) == 1
    assert lib.sic_batch_create(0, 1, 8, 0, 0, 0, 0, None, ctypes.byref(h)) == 1
    assert lib.sic_batch_create(100, 1, B.SIC_MAX_CELLS + 1, 0, 0, 0, 0, None, ctypes.byref(h)) == 1
    assert lib.sic_batch_create(100, 1, 8, 0, 3, 0, 0, None, ctypes.byref(h)) == 6
    assert lib.sic_batch_create(100, 1, 8, 0, 0, 4, 0, None, ctypes.byref(h)) == 1  # unknown flag
    n = ctypes.c_int64(0)
    assert lib.sic_refine(None, 1.0, ctypes.byref(n)) == 1
    assert lib.sic_get_layout(None, None, ctypes.byref(n)) == 1
    assert lib.sic_get_charges(None, None, 0) == 1
    assert lib.sic_load_state(None, 0, None, None, None, None, 0) == 1
    assert lib.sic_batch_get_charges(None, 0, None, 0) == 1
    assert lib.sic_batch_get_layout(None, 0, None, ctypes.byref(n)) == 1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(B.SicError):
        B.load()
