"""The C-ABI library builds, loads and exports every entry point of include/bddc.h.

Host-side argument validation is exercised too; nothing here launches GPU work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bddc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:bddc|dpcg|recycle)_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2412_17543_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2412_17543_amd.build import build
        build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("bddc_setup", "dpcg_solve", "recycle_update", "bddc_adjoint_grad", "bddc_destroy",
              "bddc_last_error", "bddc_reset_recycle"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_signatures_cover_header():
    from paper_2412_17543_amd import _lib
    assert set(_declared()) == set(_lib.SIGNATURES)


def test_default_opts(lib):
    from paper_2412_17543_amd import _lib
    o = _lib.Opts()
    lib.bddc_default_opts(ctypes.byref(o))
    assert o.constraints == 3 and o.weights == 1 and o.local_prec == 64
    assert o.recycle_strategy == 4 and o.ritz_freeze_tol == 1e-5 and o.max_it == 1000
    assert o.use_graph == 2 and o.autotune == 1 and o.save_cap == 256 and o.coarse_form == 0
    assert o.adapt_tau == 0.0 and o.adapt_max_per_face == 10
    assert o.adapt2_tau == 0.0 and o.adapt2_max_per_face == 10


def _setup(lib, nx=4, e2s=None, coef=None, **ov):
    from paper_2412_17543_amd import _lib
    e2s = np.zeros(nx ** 3, np.int32) if e2s is None else e2s
    coef = np.ones(nx ** 3) if coef is None else coef
    mesh = _lib.Mesh(nx, nx, nx, 1.0 / nx, None, None)
    part = _lib.Partition(int(e2s.max()) + 1, e2s.ctypes.data, 0, None)
    o = _lib.Opts()
    lib.bddc_default_opts(ctypes.byref(o))
    for k, v in ov.items():
        setattr(o, k, v)
    ctx = ctypes.c_void_p()
    rc = lib.bddc_setup(ctypes.byref(mesh), ctypes.byref(part), coef.ctypes.data, ctypes.byref(o), None,
                        ctypes.byref(ctx))
    return rc, lib.bddc_last_error().decode()


def test_invalid_options_rejected_on_host(lib):
    rc, msg = _setup(lib, local_prec=8)
    assert rc == -1 and "local_prec" in msg
    rc, msg = _setup(lib, recycle_R=1000)
    assert rc == -1
    rc, msg = _setup(lib, recycle_strategy=7)
    assert rc == -1


def test_invalid_partition_rejected_on_host(lib):
    e2s = np.zeros(64, np.int32)
    e2s[3] = -5
    rc, msg = _setup(lib, e2s=e2s)
    assert rc == -1 and "elem_to_sub" in msg
    coef = np.ones(64)
    coef[7] = -1.0
    rc, msg = _setup(lib, e2s=np.zeros(64, np.int32), coef=coef)
    assert rc == -1 and "positive" in msg


def test_null_arguments(lib):
    assert lib.dpcg_solve(None, None, 0, 1e-8, None, None, None) == -1
    assert lib.bddc_apply_schur(None, None, None) == -1
    lib.bddc_destroy(None)


def test_product_path_has_no_cpu_fallback():
    # the package must not import the oracle anywhere
    pkg = os.path.join(ROOT, "paper_2412_17543_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("the oracle", ""), f
