"""The C-ABI library loads and exports every entry point that include/*.h declares.

CPU-only: no compute call is made, so no GPU is needed.
"""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        for m in re.finditer(r"\b([A-Za-z_]\w*)\s*\(", text):
            name = m.group(1)
            if name.startswith("flip_") and not name.endswith("_t"):
                names.add(name)
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["flip_workspace_bytes", "flip_init", "flip_step", "flip_readback", "flip_stats",
                     "flip_destroy", "flip_status_string", "flip_field_bytes"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2404_01931_amd import flip

    lib = flip.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value
    assert set(flip.EXPORTED) <= set(declared_functions())


def test_status_strings_and_argument_errors_without_gpu():
    from paper_2404_01931_amd import flip

    assert flip.status_string(flip.FLIP_OK) == "ok"
    assert "workspace" in flip.status_string(flip.FLIP_E_WORKSPACE)
    # invalid configurations are rejected before any device work
    cfg, keep = flip.make_config((0, 8, 8), 1 / 8, 1 / 240)
    with pytest.raises(flip.FlipError) as e:
        flip.flip_workspace_bytes(cfg)
    assert e.value.status == flip.FLIP_E_INVALID
    cfg, keep = flip.make_config((8, 8, 8), 1 / 8, -1.0)
    with pytest.raises(flip.FlipError):
        flip.flip_workspace_bytes(cfg)
    cfg, keep = flip.make_config((8, 8, 8), 1 / 8, 1 / 240, flip_ratio=1.5)
    with pytest.raises(flip.FlipError):
        flip.flip_workspace_bytes(cfg)


def test_multigrid_workspace_holds_the_coarse_levels():
    from paper_2404_01931_amd import flip, inputs

    sc = inputs.scene("drop64")
    cfg, keep = flip.scene_config(sc)
    plain = flip.flip_workspace_bytes(cfg)
    cfg, keep = flip.scene_config(sc, flags=flip.FLIP_FLAG_MULTIGRID)
    mg = flip.flip_workspace_bytes(cfg)
    # z = M r and q = A s over the fine tiles (64^3 cells, 4 B each: the FP32
    # solve's direction kernel stores q for the update) plus levels 32^3, 16^3 and 8^3
    # of b and x (4 B each) and n_c (1 B), and per level a list entry (4 B) per
    # restriction block (8 x 4 x 4 cells) and a mark and a list entry per
    # prolongation block (16 x 8 x 8), and the block counts (2 per level, 4 B
    # each, for up to 32 levels); every array is 256-byte aligned
    levels = (32, 16, 8)
    coarse = sum(n ** 3 for n in levels)
    blocks = sum(4 * -(-n // 8) * (-(-n // 4)) ** 2 + 8 * -(-n // 16) * (-(-n // 8)) ** 2 for n in levels)
    need = 2 * 64 ** 3 * 4 + coarse * 9 + blocks + 2 * 32 * 4
    assert mg - plain >= need
    assert mg - plain <= need + (6 * len(levels) + 3) * 256
    # mixed precision: the inner FP32 solves take the same levels (4-byte reals)
    cfg, keep = flip.scene_config(sc, precision=flip.FLIP_MIXED)
    mixed = flip.flip_workspace_bytes(cfg)
    cfg, keep = flip.scene_config(sc, precision=flip.FLIP_MIXED, flags=flip.FLIP_FLAG_MULTIGRID)
    assert flip.flip_workspace_bytes(cfg) - mixed == mg - plain


def test_workspace_size_is_pure_and_grows_with_the_problem():
    from paper_2404_01931_amd import flip, inputs

    sc = inputs.scene("dam32")
    cfg, keep = flip.scene_config(sc, precision=flip.FLIP_FP32)
    a = flip.flip_workspace_bytes(cfg)
    assert a == flip.flip_workspace_bytes(cfg) and a % 256 == 0
    cfg64, keep64 = flip.scene_config(sc, precision=flip.FLIP_FP64)
    assert flip.flip_workspace_bytes(cfg64) > a
    big, keepb = flip.scene_config(inputs.scene("drop64"))
    assert flip.flip_workspace_bytes(big) > a
    # 65,536 particles at 32^3: particle state dominates a lower bound
    assert a > 65536 * 2 * 28


def test_init_rejects_missing_or_short_workspace_without_gpu():
    from paper_2404_01931_amd import flip, inputs

    cfg, keep = flip.scene_config(inputs.scene("dam32"))
    need = flip.flip_workspace_bytes(cfg)
    h = ctypes.c_void_p(0)
    lib = flip.load()
    assert lib.flip_init(ctypes.byref(cfg), None, need, None, ctypes.byref(h)) == flip.FLIP_E_WORKSPACE
    assert lib.flip_init(ctypes.byref(cfg), ctypes.c_void_p(1 << 20), need - 1, None,
                         ctypes.byref(h)) == flip.FLIP_E_WORKSPACE
    assert lib.flip_init(ctypes.byref(cfg), ctypes.c_void_p((1 << 20) + 8), need, None,
                         ctypes.byref(h)) == flip.FLIP_E_WORKSPACE
    assert not h.value


def test_batch_calls_reject_bad_arguments_without_gpu():
    from paper_2404_01931_amd import flip

    lib = flip.load()
    out = ctypes.c_size_t(0)
    # no handles, too many scenes, null handle entries: rejected before any device work
    assert lib.flip_batch_workspace_bytes(None, 0, ctypes.byref(out)) == flip.FLIP_E_INVALID
    arr = (ctypes.c_void_p * 2)()
    assert lib.flip_batch_workspace_bytes(arr, 2, ctypes.byref(out)) == flip.FLIP_E_INVALID
    assert lib.flip_batch_workspace_bytes(arr, flip.FLIP_BATCH_MAX_SCENES + 1,
                                          ctypes.byref(out)) == flip.FLIP_E_INVALID
    b = ctypes.c_void_p(0)
    assert lib.flip_batch_create(arr, 0, 0, None, 0, None, ctypes.byref(b)) == flip.FLIP_E_INVALID
    assert lib.flip_batch_create(arr, 2, 0, None, 0, None, ctypes.byref(b)) == flip.FLIP_E_INVALID
    assert b.value is None
    assert lib.flip_batch_step(None, 1, None) == flip.FLIP_E_INVALID
    lib.flip_batch_destroy(None)


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C layout (size and
    the offset of the last field), checked by compiling the header with gcc."""
    import shutil
    import subprocess

    from paper_2404_01931_amd import flip

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "flip.h"\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu\\n", sizeof(flip_config), sizeof(flip_step_stats), '
                   'offsetof(flip_step_stats, nonfinite), sizeof(flip_region), '
                   'offsetof(flip_config, particle_capacity));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out == [ctypes.sizeof(flip.flip_config), ctypes.sizeof(flip.flip_step_stats),
                   flip.flip_step_stats.nonfinite.offset, ctypes.sizeof(flip.flip_region),
                   flip.flip_config.particle_capacity.offset]
