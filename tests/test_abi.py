"""The C-ABI library loads and exports every entry point include/nep.h declares (no GPU calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nep.h")
LIB = os.path.join(ROOT, "paper_2604_24816_amd", "libnep.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nep_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnep.so not built: run __graft_entry__.build()")
    import torch  # noqa: F401  (same HIP runtime as torch)
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_2604_24816_amd import nep
    assert sorted(nep.EXPORTED) == declared_functions()


def test_host_only_calls(lib):
    from paper_2604_24816_amd import inputs as I
    from paper_2604_24816_amd import nep
    lib.nep_status_string.restype = ctypes.c_char_p
    assert lib.nep_status_string(-3) == b"neighbour list capacity exceeded"
    hp = I.FULL_HPARAMS
    n = ctypes.c_int64()
    d = ctypes.c_int32()
    hs = nep._hp_struct(hp)
    assert lib.nep_param_count(ctypes.byref(hs), ctypes.byref(n), ctypes.byref(d)) == 0
    assert n.value == hp.n_params() and d.value == hp.n_desc == 30
    sh = I.SURROGATE_HPARAMS
    ss = nep._hp_struct(sh)
    assert lib.nep_param_count(ctypes.byref(ss), ctypes.byref(n), ctypes.byref(d)) == 0
    assert n.value == sh.n_params() and d.value == 15
    # model creation and workspace sizing are host-only
    m = nep.NEPModel(hp, I.random_model(hp, 0))
    ws = ctypes.c_int64()
    box = np.array([361.5, 361.5, 361.5])
    assert lib.nep_system_workspace_bytes(m.handle, None, ctypes.c_int64(4_000_000),
                                          box.ctypes.data_as(ctypes.c_void_p), 160, 96, ctypes.byref(ws)) == 0
    assert 4e9 < ws.value < 2e10
    bad = np.array([1.0, np.nan])
    with pytest.raises(Exception):
        nep.NEPModel(hp, bad)


@pytest.mark.parametrize("zbl,ok", [((2.0, None, (29.0,)), True), ((2.4, 2.05, (29.0,)), True),
                                    ((7.0, None, (29.0,)), False),    # outer radius beyond rc_radial
                                    ((2.0, 2.0, (29.0,)), False),     # inner radius not below the outer
                                    ((2.0, None, (0.0,)), False)])    # no atomic number
def test_zbl_hparams_validated_on_the_host(lib, zbl, ok):
    from paper_2604_24816_amd import inputs as I
    from paper_2604_24816_amd import nep
    outer, inner, z = zbl
    hp = I.HParams(zbl_outer=outer, zbl_inner_radius=inner, zbl_z=z)
    hs = nep._hp_struct(hp)
    n, d = ctypes.c_int64(), ctypes.c_int32()
    st = lib.nep_param_count(ctypes.byref(hs), ctypes.byref(n), ctypes.byref(d))
    assert (st == 0) == ok
    if ok:
        assert n.value == I.HParams().n_params()   # ZBL adds no parameters


def test_model_file_round_trip(tmp_path):
    from paper_2604_24816_amd import inputs as I
    for hp in (I.FULL_HPARAMS, I.SURROGATE_SHORT_HPARAMS, I.HParams(n_types=2, zbl_outer=2.0, zbl_z=(29.0, 79.0))):
        p = I.random_model(hp, 3)
        f = tmp_path / "m.npz"
        I.save_model(str(f), hp, p)
        hp2, p2 = I.load_model(str(f))
        assert hp2 == hp and np.array_equal(p2, p)
    with pytest.raises(ValueError):
        I.save_model(str(tmp_path / "bad.npz"), I.FULL_HPARAMS, np.zeros(5))
