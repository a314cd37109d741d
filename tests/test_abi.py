"""The C-ABI library loads and exports every symbol include/gfcc.h declares (no GPU needed)."""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gfcc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_symbols_exported():
    from paper_1902_06016_amd import gfcc
    declared = _declared()
    assert len(declared) >= 16, declared
    lib = ctypes.CDLL(gfcc.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(gfcc.SYMBOLS) == declared


def test_host_only_entry_points():
    from paper_1902_06016_amd import gfcc
    assert gfcc.dim(10, 20) == 910
    assert gfcc.dim(42, 186) == 160188
    assert gfcc.dim(70, 260) == 627970
    assert gfcc.lib.gfcc_dim(-1, 3) == -1
    # spectral_function computes on the device even for a host G; with no frequency it
    # returns at once
    assert gfcc.spectral_function(np.zeros((0, 2, 2), dtype=np.complex128)).shape == (0,)
    # bad arguments are rejected without touching a device
    assert gfcc.lib.spectral_function(-1, 1, None, 0, None) == gfcc.GFCC_EINVAL
    assert gfcc.lib.gfcc_solve(None, 1, None, 1, None, 0.1, 1e-8, 10, 10, 0, 0, 0, None, None,
                               None, None) == gfcc.GFCC_EINVAL
    assert gfcc.lib.mor_eval(None, 1, None, None, None) == gfcc.GFCC_EINVAL
    assert gfcc.lib.gfcc_destroy(None) == gfcc.GFCC_OK


def test_binding_constants_match_header():
    """Every enum value the header defines has the same value in the Python binding."""
    from paper_1902_06016_amd import gfcc
    text = open(os.path.join(ROOT, "include", "gfcc.h")).read()
    found = dict((k, int(v)) for k, v in re.findall(r"^\s*GFCC_([A-Z0-9_]+) = (\d+)", text, re.M))
    assert {"FP64", "FP32", "FP32_BF16_3BODY", "BF16_PAIRS", "KEEP_FP32", "ESTATE"} <= set(found)
    for name, val in found.items():
        py = getattr(gfcc, name, getattr(gfcc, "GFCC_" + name, None))
        assert py == val, (name, py, val)


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch still leaves one HIP runtime in the process: the
    library binds to the runtime torch's wheel carries instead of loading the system's beside it
    (two runtimes keep separate device state, and contexts fail)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1902_06016_amd import gfcc\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(sorted({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n"
            "print(torch.__file__)\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    paths, torch_file = out.stdout.strip().splitlines()[-2:]
    paths = eval(paths)
    assert len(paths) == 1, paths
    torch_dir = os.path.dirname(os.path.realpath(torch_file))
    assert os.path.realpath(paths[0]).startswith(torch_dir), (paths, torch_dir)
