"""CPU checks of the C ABI: librpi.so loads and exports every function that
include/rpi.h declares (no compute call is made without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_functions_are_exported():
    from paper_2406_16302_amd import native
    lib = native.load_library()
    hdr = open(os.path.join(ROOT, "include", "rpi.h")).read()
    names = sorted(set(re.findall(r"^(?:rpi_status|const char\s*\*)\s*(rpi_\w+)\s*\(", hdr, re.M)))
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert lib.rpi_version().decode().startswith("rpi")


def test_null_arguments_are_rejected_without_device_work():
    from paper_2406_16302_amd import native
    lib = native.load_library()
    assert lib.rpi_build_scene(None, None) == -1
    assert b"null" in lib.rpi_last_error()
    assert lib.rpi_render_residual(None, None, None, None, None, None) == -1
    assert lib.rpi_render_frame(None, None, 1, None, None, None) == -1
