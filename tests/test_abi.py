"""The C-ABI library loads on a machine without a GPU and exports every
symbol declared in include/nvgs.h (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nvgs.h")
LIB = os.path.join(ROOT, "paper_2511_19202_amd", "libnvgs.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nvgs_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["nvgs_create", "nvgs_destroy", "nvgs_last_error", "nvgs_load_assets", "nvgs_set_instances",
                 "nvgs_query_visibility", "nvgs_render", "nvgs_debug_buffers", "nvgs_reserve",
                 "nvgs_frame_watermarks", "nvgs_set_mlp_shape", "nvgs_autotune", "nvgs_make_labels",
                 "nvgs_train_visibility", "nvgs_mlp_forward", "nvgs_mlp_backward"]:
        assert must in names


def test_library_exports_every_declared_symbol(so):
    missing = [n for n in declared_functions() if not hasattr(so, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    import paper_2511_19202_amd as nvgs
    assert set(declared_functions()) <= set(nvgs.exported_symbols())


def test_struct_layouts_match_the_header():
    """ctypes mirrors of the ABI structs have the sizes the C compiler gives."""
    import subprocess
    import tempfile
    import paper_2511_19202_amd as nvgs
    structs = {"nvgs_create_info": nvgs.CreateInfo, "nvgs_mlp": nvgs.MLP, "nvgs_asset": nvgs.Asset,
               "nvgs_instance": nvgs.Instance, "nvgs_camera": nvgs.Camera, "nvgs_render_opts": nvgs.RenderOpts,
               "nvgs_frame_stats": nvgs.FrameStats, "nvgs_debug_view": nvgs.DebugView,
               "nvgs_train_opts": nvgs.TrainOpts, "nvgs_mlp_shape": nvgs.MlpShape,
               "nvgs_tune_entry": nvgs.TuneEntry, "nvgs_workspace": nvgs.Workspace}
    body = "\n".join(f'printf("%zu\\n", sizeof({k}));' for k in structs)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(f'#include <stdio.h>\n#include "{HEADER}"\nint main(void){{{body}return 0;}}\n')
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-o", exe, c])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    for (name, cls), sz in zip(structs.items(), sizes):
        assert ctypes.sizeof(cls) == sz, name


def test_null_and_invalid_arguments_are_rejected(so):
    so.nvgs_create.restype = ctypes.c_int32
    so.nvgs_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    out = ctypes.c_void_p()
    assert so.nvgs_create(None, ctypes.byref(out)) == 1  # E_INVALID before touching a device
    so.nvgs_load_assets.restype = ctypes.c_int32
    so.nvgs_load_assets.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    assert so.nvgs_load_assets(None, None, 0) == 1
    so.nvgs_sort_pairs.restype = ctypes.c_int32
    so.nvgs_sort_pairs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_int32, ctypes.c_int32]
    assert so.nvgs_sort_pairs(None, None, None, 0, 0, 32) == 1
    so.nvgs_last_error.restype = ctypes.c_char_p
    so.nvgs_last_error.argtypes = [ctypes.c_void_p]
    assert so.nvgs_last_error(None) == b"null context"


def test_allocator_callbacks_return_null_instead_of_raising():
    """A failed torch allocation inside the allocator callback must reach the
    library as NULL (a raising ctypes callback returns an undefined value)."""
    import torch
    import paper_2511_19202_amd as nvgs
    blocks = {}
    alloc, free = nvgs.torch_allocator(torch.device("cpu"), blocks)
    call_alloc = ctypes.cast(alloc, ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p))
    call_free = ctypes.cast(free, ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p))
    p = call_alloc(1024, None)
    assert p and p in blocks
    call_free(p, None)
    assert p not in blocks
    for _ in range(3):  # far beyond any memory: torch raises, the callback returns NULL
        assert call_alloc(1 << 62, None) is None
    call_free(12345, None)  # unknown pointers are ignored
