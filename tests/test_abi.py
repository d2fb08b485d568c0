"""The C-ABI library loads without a GPU and exports every symbol that
include/*.h declares; the Python binding binds exactly those names."""
import ctypes
import glob
import os
import re

import pytest

from paper_2312_10070_amd import gsr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(gsr_[a-z_0-9]+)\s*\(", txt, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_entry_points():
    names = header_symbols()
    for core in ("gsr_ctx_create", "gsr_render_fwd", "gsr_render_bwd", "gsr_loss_l1", "gsr_loss_track", "gsr_adam"):
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(gsr.LIB_PATH):
        pytest.skip("libgsr.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(gsr.LIB_PATH)
    missing = [n for n in sorted(header_symbols()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_matches_header():
    assert set(gsr.declared_symbols()) == header_symbols()


def test_host_only_calls():
    if not os.path.exists(gsr.LIB_PATH):
        pytest.skip("libgsr.so not built")
    lib = gsr.load()
    assert lib.gsr_strerror(0) == b"ok"
    assert lib.gsr_strerror(-4).startswith(b"fixed-capacity")
    o = gsr.Opts()
    lib.gsr_default_opts(ctypes.byref(o))
    assert (o.tile_w, o.tile_h) == (16, 16) and abs(o.alpha_min - 1 / 255) < 1e-9 and abs(o.T_min - 1e-4) < 1e-10
    # a NULL context is rejected without touching a device
    assert lib.gsr_set_stream(None, None) == gsr.GSR_EINVAL
    assert lib.gsr_ctx_create(None, 0, None) == gsr.GSR_EINVAL
    # the context-free loss checks its arguments before any device call
    assert lib.gsr_loss_track_noalloc(None, None, None, None, None, None, 4, 0.5, 50.0, None, None, None,
                                      None) == gsr.GSR_EINVAL
    assert b"bad loss arguments" in lib.gsr_last_error(None)
