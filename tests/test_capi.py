"""The C-ABI library loads and exports every entry point its header declares
(no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    with open(os.path.join(ROOT, "include", "grpic.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:grpic_status|const char\*)\s+(grpic_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("grpic_create", "grpic_destroy", "grpic_particles_init", "grpic_fields_init_wald",
              "grpic_push", "grpic_deposit", "grpic_field_advance", "grpic_diagnostics",
              "grpic_last_error", "grpic_get_params"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2511_17701_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    lib = ctypes.CDLL(build.LIB)
    for n in declared():
        assert hasattr(lib, n), n
    from paper_2511_17701_amd import grpic
    assert set(declared()) <= set(grpic.EXPORTS)


def test_argument_errors_reported_without_gpu():
    """Invalid parameters are rejected on the host before any device work."""
    from paper_2511_17701_amd import grpic
    import pytest
    with pytest.raises(grpic.GrpicError, match="n_ghost"):
        grpic.Context(0.9, 1.0, 1.3, 20.0, 32, 32, n_ghost=3)
    with pytest.raises(grpic.GrpicError, match="a"):
        grpic.Context(1.2, 1.0, 1.3, 20.0, 32, 32)
    with pytest.raises(grpic.GrpicError, match="too small"):
        grpic.Context(0.9, 1.0, 1.3, 20.0, 4, 32)
    with pytest.raises(grpic.GrpicError, match="r0"):
        grpic.Context(0.9, 1.0, 1.3, 20.0, 32, 32, r0=1.3)
    with pytest.raises(grpic.GrpicError, match="h0"):
        grpic.Context(0.9, 1.0, 1.3, 20.0, 32, 32, h0=-0.5)
