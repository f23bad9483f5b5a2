"""The C-ABI library loads on the CPU host and exports every symbol that
include/quokka.h declares (no compute call: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "quokka.h")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(quokka_\w+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("quokka_hydro_step", "quokka_rad_step", "quokka_batch_step", "quokka_compute_dt",
              "quokka_fill_ghosts", "quokka_ctx_create", "quokka_sync_status"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2110_01792_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(binding.EXPORTED) == set(declared())


def test_null_context_is_rejected_without_a_device():
    from paper_2110_01792_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load()
    assert lib.quokka_hydro_step(None, None, None, 0, None, None, 0.0, None, None) == binding.QK_EINVAL
    assert lib.quokka_sync_status(None, None) == binding.QK_EINVAL
