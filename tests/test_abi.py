"""The C ABI without a GPU: exports, struct layout, and argument checks that
return before any device call."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2311_15088_amd as sph
from paper_2311_15088_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = sph.lib()
    names = declared_functions()
    assert "sph_create" in names and "sph_step" in names and "sph_read" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(sph.EXPORTS) <= set(names)


MIRRORS = [("sph_params", "Params"), ("sph_info", "Info"), ("sph_tuning", "Tuning"),
           ("sph_train_params", "TrainParams"), ("sph_train_report", "TrainReport"),
           ("sph_closure_stats", "ClosureStats")]


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    lines = []
    expect = []
    for cname, pyname in MIRRORS:
        cls = getattr(sph, pyname)
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for f, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {f}));')
            expect.append(getattr(cls, f).offset)
    body = "\n".join(lines)
    src.write_text(f"""#include <stddef.h>
#include <stdio.h>
#include "sph.h"
int main(void) {{
{body}
  return 0;
}}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == expect


def test_closure_constants_match_header():
    text = open(HEADER).read()
    assert f"#define SPH_CLOSURE_PARAMS {sph.CLOSURE_PARAMS}" in text
    assert f"#define SPH_CLOSURE_FEATURES {sph.CLOSURE_FEATURES}" in text
    assert sph.CLOSURE_PARAMS == scenes.mlp_flat(scenes.mlp_init()).size


def _try_create(p, n=4, na=2):
    x = np.full((n, 3), 0.5, np.float32)
    y = np.full((na, 3), 0.5, np.float32)
    with pytest.raises(sph.SphError) as ei:
        sph.Simulation(p, x, x, y, y)
    return ei.value.status


@pytest.mark.parametrize("field,val", [("h", 0.0), ("h", -1.0), ("mass", 0.0), ("rest_density", -5.0),
                                       ("dt", -1e-3), ("r_couple", 0.0), ("kernel_norm", 3), ("v_min", 2.0)])
def test_invalid_parameters_are_rejected(field, val):
    p = scenes.default_params(0.05, 5e-4, (0, 0, 0), (1, 1, 1))
    p[field] = val
    assert _try_create(p) == sph.EINVAL
    assert sph.lib().sph_last_error(None)


def test_inverted_box_is_rejected():
    p = scenes.default_params(0.05, 5e-4, (0, 0, 0), (1, 1, 1))
    p["box_max"] = [1.0, -1.0, 1.0]
    assert _try_create(p) == sph.EINVAL


def test_cell_table_capacity():
    p = scenes.default_params(0.05, 5e-4, (0, 0, 0), (1, 1, 1))
    p["n_buckets"] = 7999  # the grid has 20^3 = 8000 cells
    assert _try_create(p) == sph.ECAPACITY


def test_null_arguments():
    L = sph.lib()
    out = ctypes.c_void_p()
    assert L.sph_create(None, 0, None, None, 0, None, None, None, ctypes.byref(out)) == sph.EINVAL
    assert L.sph_step(None, 1) == sph.EINVAL
    assert L.sph_read(None, 0, None, 0) == sph.EINVAL
    L.sph_destroy(None)
