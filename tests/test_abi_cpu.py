"""CPU checks of the C ABI: the library loads and exports every declared
entry point; argument validation returns before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "g4d.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(g4d_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_surface():
    from paper_2310_10642_amd import g4d
    assert declared_symbols() == sorted(g4d.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_2310_10642_amd import g4d
    if not os.path.exists(g4d.LIB_PATH):
        pytest.skip("libg4d.so not built")
    lib = ctypes.CDLL(g4d.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_header_constants_match_binding():
    from paper_2310_10642_amd import g4d
    text = open(HEADER).read()
    def val(name):
        return int(re.search(rf"\b{name}\s*=\s*(-?\d+)", text).group(1))
    assert val("G4D_EINVAL") == g4d.G4D_EINVAL and val("G4D_ESTATE") == g4d.G4D_ESTATE
    assert val("G4D_GRAD_ACCUMULATE") == g4d.G4D_GRAD_ACCUMULATE
    assert val("G4D_LOSS_L1") == g4d.G4D_LOSS_L1 and val("G4D_LOSS_L2") == g4d.G4D_LOSS_L2
    assert val("G4D_TUNE_STAGE_TIMING") == g4d.G4D_TUNE_STAGE_TIMING
    assert val("G4D_TUNE_ROUND_PAIRS") == g4d.G4D_TUNE_ROUND_PAIRS
    assert val("G4D_TUNE_ROUND_INSTANCES") == g4d.G4D_TUNE_ROUND_INSTANCES
    assert val("G4D_TUNE_SYNC_FREE") == g4d.G4D_TUNE_SYNC_FREE
    assert val("G4D_TUNE_ARENA_INSTANCES") == g4d.G4D_TUNE_ARENA_INSTANCES
    assert val("G4D_TUNE_TILE_ORDER") == g4d.G4D_TUNE_TILE_ORDER
    assert val("G4D_TUNE_AUTOTUNE") == g4d.G4D_TUNE_AUTOTUNE
    assert val("G4D_TUNE_ELLIPSE_CULL") == g4d.G4D_TUNE_ELLIPSE_CULL
    assert val("G4D_TUNE_PERSISTENT_BLOCKS") == g4d.G4D_TUNE_PERSISTENT_BLOCKS
    assert val("G4D_TUNE_LDS_BATCH") == g4d.G4D_TUNE_LDS_BATCH
    assert val("G4D_NUM_STAGES") == len(g4d.STAGES)
    for k, v in g4d.DBG.items():
        assert val("G4D_DBG_" + k.upper()) == v


def test_struct_layouts():
    """The binding's ctypes structs have the sizes and field offsets that a C
    compiler gives the header's structs."""
    import shutil
    import subprocess
    import tempfile
    from paper_2310_10642_amd import g4d
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"g4d_options": g4d.G4DOptions, "g4d_camera": g4d.G4DCamera, "g4d_stats": g4d.G4DStats,
               "g4d_adam_options": g4d.G4DAdamOptions}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "g4d.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['  return 0;', '}']
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        with open(src, "w") as f:
            f.write("\n".join(lines) + "\n")
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            parts = line.split()
            got[tuple(parts[:-1])] = int(parts[-1])
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_validation_before_any_hip_call():
    from paper_2310_10642_amd import g4d
    if not os.path.exists(g4d.LIB_PATH):
        pytest.skip("libg4d.so not built")
    lib = g4d.load_library()
    h = ctypes.c_void_p()
    assert lib.g4d_create(None, None, ctypes.byref(h)) == g4d.G4D_EINVAL
    o = g4d.G4DOptions()
    lib.g4d_default_options(ctypes.byref(o))
    assert (o.sh_degree, o.t_order) == (3, 2) and abs(o.t_cull - 0.05) < 1e-7
    o.sh_degree = 4
    assert lib.g4d_create(ctypes.byref(o), None, ctypes.byref(h)) == g4d.G4D_EINVAL
    o.sh_degree, o.t_period = 3, 0.0
    assert lib.g4d_create(ctypes.byref(o), None, ctypes.byref(h)) == g4d.G4D_EINVAL
    assert lib.g4d_render(None, 1, None, None, None, None, None) == g4d.G4D_EINVAL
    assert lib.g4d_destroy(None) == g4d.G4D_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message before
    touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert p.returncode == 2 and "one GPU only" in p.stderr
