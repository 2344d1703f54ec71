"""The C-ABI library loads and exports every symbol include/rcast.h declares."""
import ctypes
import os
import re

import paper_2509_17390_amd as pkg
from paper_2509_17390_amd import rcast

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def declared_functions():
    """Every rc_* function declared by any header under include/."""
    names = set()
    for f in sorted(os.listdir(INCLUDE)):
        if not f.endswith(".h"):
            continue
        src = open(os.path.join(INCLUDE, f)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(rc_[a-z_0-9]+)\s*\(", src))
    return names


def test_header_and_binding_agree():
    assert declared_functions() == set(rcast.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.rc_version() == 1


def test_struct_layouts_match_header():
    # rc_job: 4 int32, pointer, 2 float, int64 -> 40 bytes on LP64
    assert ctypes.sizeof(rcast.rc_job) == 40
    assert ctypes.sizeof(rcast.rc_build_opts) == 32
    assert rcast.rc_scene_info.scene_lo.offset == 56
    assert ctypes.sizeof(rcast.rc_tuning) == 40      # ten int32 fields
    assert ctypes.sizeof(rcast.rc_gauss_opts) == 32
    assert ctypes.sizeof(rcast.rc_grid) == 48
    assert ctypes.sizeof(rcast.rc_tsdf_opts) == 32
    assert ctypes.sizeof(rcast.rc_fidelity) == 64


def test_error_path_without_device_is_clean():
    import torch
    if torch.cuda.is_available():
        return  # only meaningful where no GPU is visible
    lib = pkg.load()
    h = ctypes.c_void_p()
    st = lib.rc_create(0, 0, ctypes.byref(h))
    assert st == rcast.RC_E_DEVICE or st == rcast.RC_E_INVAL
    assert lib.rc_last_error()
    assert not h.value


def test_c_driver_builds_against_header_and_library():
    """The header is plain C (C11) and the library links from C: the ABI
    driver of the GPU test compiles and links here (it runs on the GPU)."""
    import __graft_entry__
    exe = __graft_entry__.build_abi_driver()
    assert os.path.exists(exe) and os.access(exe, os.X_OK)
