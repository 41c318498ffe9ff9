"""The C-ABI library loads without a GPU and exports every function that
include/*.h declares (no compute calls here)."""
import ctypes
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(mcrt_\w+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["mcrt_create", "mcrt_destroy", "mcrt_set_grid", "mcrt_set_density", "mcrt_iterate",
              "mcrt_final_pass", "mcrt_run", "mcrt_get_temperature", "mcrt_get_sed"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1112_1071_amd import mcrt

    L = mcrt.lib()
    missing = [n for n in sorted(declared_functions()) if not hasattr(L, n)]
    assert not missing, missing


def test_no_device_is_reported_cleanly():
    import torch

    if torch.cuda.is_available():
        return
    from paper_1112_1071_amd import mcrt

    h = ctypes.c_void_p()
    assert mcrt.lib().mcrt_create(ctypes.byref(h), 0) == -4  # MCRT_E_DEVICE
    cfg = mcrt.default_run_cfg()
    assert cfg.n_packets == 100000 and cfg.conv_p == 0.999 and cfg.block_size == 0
