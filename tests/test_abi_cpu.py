"""The C ABI: the built library loads and exports every function include/vqe.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(vqe_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["vqe_prepare_reference", "vqe_apply_ansatz", "vqe_expect", "vqe_energy_grad",
                     "vqe_adam_step", "vqe_run", "vqe_ham_from_integrals"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2601_09951_amd import capi
    L = capi.lib()
    assert L._name == capi.LIB_PATH
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(capi.EXPORTED) == declared_functions()


def test_library_is_built_for_gfx950():
    from paper_2601_09951_amd import capi
    data = open(capi.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_strerror_without_device():
    from paper_2601_09951_amd import capi
    L = capi.lib()
    for code in (0, -1, -2, -3, -4, -99):
        assert L.vqe_strerror(code)
    h = ctypes.c_void_p()
    assert L.vqe_ctx_create(-1, ctypes.byref(h)) == 0
    assert L.vqe_ctx_set_loop_mode(h, 1) == 0
    assert L.vqe_ctx_set_loop_mode(h, 5) == capi.VQE_EINVAL
    assert L.vqe_ctx_set_tile(h, 13, 12, 5) == 0
    assert L.vqe_ctx_set_tile(h, 8, 8, 5) == capi.VQE_EINVAL  # k - c < 4
    assert L.vqe_ctx_destroy(h) == 0
