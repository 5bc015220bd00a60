"""Host-side checks of the C ABI library (no GPU needed): it loads and exports every declared entry point."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bifrost.h")
LIB = os.path.join(ROOT, "paper_2210_02472_amd", "libbifrost_hip.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"BF_API\s+[^;(]*?\b(bf_\w+)\s*\(", txt)))


def test_header_declares_the_pass():
    names = declared()
    for f in ("bf_forces", "bf_force_gradient", "bf_pn1_bh", "bf_dt_min", "bf_fsi_step", "bf_energy",
              "bf_forces_batched", "bf_autotune", "bf_create", "bf_destroy"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (bf_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    extra = sorted(exported - set(declared()))
    assert not extra, f"exported but not declared: {extra}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_covers_the_header():
    from paper_2210_02472_amd import _binding
    lib = _binding.load_library()
    assert lib.bf_version().startswith(b"bifrost-hip")
    src = open(_binding.__file__).read()
    for n in declared():
        assert f'"{n}"' in src or f"lib.{n}" in src, n
    assert lib.bf_status_string(-1) == b"invalid argument"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_arguments_are_rejected_without_a_gpu():
    import ctypes
    from paper_2210_02472_amd import _binding
    lib = _binding.load_library()
    assert lib.bf_create(None, 0, None) == -1
    assert lib.bf_forces(None, None, None, None, 1.0, 0.0, 1, 0.0, None, None, None) == -1
    assert lib.bf_last_error() != b""
    assert lib.bf_destroy(None) == 0
