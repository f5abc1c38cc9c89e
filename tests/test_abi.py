"""Host-side checks of the C ABI that need no GPU: the library loads, exports every entry point
declared in include/amoeba.h, and rejects invalid parameters before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2011_01207_amd import amoeba

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "amoeba.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(amoeba_[a-z_]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    L = amoeba.lib()
    names = declared_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name


def _params(**kw):
    p = amoeba.amoeba_params()
    p.n_atoms = kw.get("n", 648)
    for a in range(3):
        p.box[a] = kw.get("box", 18.63)
        p.grid[a] = kw.get("grid", 24)
    p.cutoff = kw.get("cutoff", 7.0)
    p.buffer = kw.get("buffer", 0.0)
    p.ewald_alpha = kw.get("beta", 0.545)
    p.order = kw.get("order", 5)
    p.precision = kw.get("precision", 0)
    p.max_workspace_bytes = kw.get("cap", 0)
    return p


@pytest.mark.parametrize("kw,frag", [
    ({"n": 0}, "n_atoms"),
    ({"box": -1.0}, "box"),
    ({"cutoff": 9.5}, "half the smallest box edge"),
    ({"cutoff": 7.0, "buffer": 2.5}, "half the smallest box edge"),
    ({"beta": 0.0}, "ewald_alpha"),
    ({"order": 4}, "order 5"),
    ({"grid": 8}, "grid"),
    ({"grid": 4096}, "grid"),
    ({"precision": 7}, "precision"),
    ({"cap": -5}, "max_workspace_bytes"),
])
def test_create_rejects_invalid_parameters(kw, frag):
    L = amoeba.lib()
    h = ctypes.c_void_p()
    p = _params(**kw)
    st = L.amoeba_create(ctypes.byref(p), None, ctypes.byref(h))
    assert st == amoeba.AMOEBA_E_INVALID
    assert frag in L.amoeba_create_error().decode()
    assert not h.value


def test_create_null_arguments():
    L = amoeba.lib()
    h = ctypes.c_void_p()
    assert L.amoeba_create(None, None, ctypes.byref(h)) == amoeba.AMOEBA_E_INVALID
    assert L.amoeba_destroy(None) == amoeba.AMOEBA_OK


def test_calls_on_null_context_are_rejected():
    L = amoeba.lib()
    assert L.amoeba_build_blocklist(None, None) == amoeba.AMOEBA_E_INVALID
    assert L.amoeba_update_blocklist(None, None, None) == amoeba.AMOEBA_E_INVALID
    assert L.amoeba_polarize_configuration(None, None, None, None, None, None, 0, 1e-5, 10, None, None, None, None,
                                           None) == amoeba.AMOEBA_E_INVALID
    assert L.amoeba_dipole_matvec(None, None, None, None) == amoeba.AMOEBA_E_INVALID
    assert L.amoeba_last_error(None) == b"NULL context"


def test_valid_parameters_without_gpu_report_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = amoeba.lib()
    h = ctypes.c_void_p()
    st = L.amoeba_create(ctypes.byref(_params()), None, ctypes.byref(h))
    assert st == amoeba.AMOEBA_E_DEVICE
