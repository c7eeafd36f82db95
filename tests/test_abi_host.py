"""CPU-only checks of the C ABI library: it loads, exports every symbol the
header declares, validates leaf structures on the host and evaluates
tracks in FP64 exactly as the oracle does (no GPU calls)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(dv_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("dv_build_scene", "dv_render", "dv_render_backward",
              "dv_serve_submit", "dv_serve_poll", "dv_ctx_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2606_23031_amd import dv
    lib = dv.lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert "gfx950" in dv.version()


def _cube_leaves(level):
    n = 1 << level
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                             indexing="ij"), -1).reshape(-1, 3)
    return np.full(len(g), level, np.uint8), g.T.astype(np.int32).copy()


def _cidx(n, nc=None):
    c = np.arange(8 * n, dtype=np.int32).reshape(8, n)
    return c, (nc if nc is not None else 8 * n)


def test_validation_accepts_valid_octree():
    from paper_2606_23031_amd import dv
    from synth import make_config
    o = make_config(1)["scene"]["octrees"][0]
    st, msg = dv.dv_validate_octree_host(o["level"], o["ijk"], o["corner_idx"],
                                         o["max_level"],
                                         len(o["corner_density"]), 0)
    assert st == 0, msg


@pytest.mark.parametrize("case,expect", [
    ("overlap_parent_child", -4), ("duplicate", -4), ("level_too_deep", -5),
    ("cell_out_of_range", -5), ("corner_out_of_range", -5),
    ("bad_degree", -5), ("bad_max_level", -5)])
def test_validation_rejects(case, expect):
    from paper_2606_23031_amd import dv
    lv, ijk = _cube_leaves(1)
    max_level, deg = 2, 0
    if case == "overlap_parent_child":
        lv = np.concatenate([lv, [2]]).astype(np.uint8)
        ijk = np.concatenate([ijk, [[1], [1], [1]]], 1).astype(np.int32)
    elif case == "duplicate":
        lv = np.concatenate([lv, [1]]).astype(np.uint8)
        ijk = np.concatenate([ijk, [[0], [1], [0]]], 1).astype(np.int32)
    elif case == "level_too_deep":
        lv = lv.copy()
        lv[3] = 3
    elif case == "cell_out_of_range":
        ijk = ijk.copy()
        ijk[2, 5] = 2
    elif case == "bad_degree":
        deg = 4
    elif case == "bad_max_level":
        max_level = 17
    n = lv.shape[0]
    cidx, nc = _cidx(n)
    if case == "corner_out_of_range":
        cidx = cidx.copy()
        cidx[7, 2] = nc
    st, msg = dv.dv_validate_octree_host(lv, ijk, cidx, max_level, nc, deg)
    assert st == expect, (st, msg)
    assert msg


def test_track_pose_matches_oracle():
    from paper_2606_23031_amd import dv
    from oracle import geometry as G
    tr = dict(t=np.array([0.0, 1.0, 4.0]), yaw=np.array([0.1, 0.5, -0.3]),
              trans=np.array([[0, 0, 0.8], [5, 1, 0.8], [20, 3, 0.9]], float))
    for t in (-0.5, 0.0, 0.3, 1.0, 2.7, 4.0, 4.5):
        a1, R1, p1 = dv.dv_track_pose(tr, t)
        a2, R2, p2 = G.pose_at(tr, t)
        assert a1 == a2
        if a1:
            assert np.abs(R1 - R2).max() <= 1e-15
            assert np.abs(p1 - p2).max() <= 1e-14


def test_binding_fails_loudly_without_library(tmp_path):
    # the binding refuses to import when the built library is absent
    import subprocess
    import sys
    code = ("import importlib.util, sys\n"
            "spec = importlib.util.spec_from_file_location('dvtest', sys.argv[1])\n"
            "m = importlib.util.module_from_spec(spec)\n"
            "m.__file__ = sys.argv[1]\n"
            "import os\n"
            "src = open(sys.argv[1]).read().replace('LIB_PATH = os.path.join(HERE, \"libdvox.so\")', 'LIB_PATH = \"/nonexistent/libdvox.so\"')\n"
            "try:\n"
            "    exec(compile(src, 'dv', 'exec'), {'__name__': 'dvtest', '__file__': sys.argv[1]})\n"
            "except ImportError as e:\n"
            "    print('IMPORT_ERROR', e)\n")
    r = subprocess.run([sys.executable, "-c", code,
                        os.path.join(ROOT, "paper_2606_23031_amd", "dv.py")],
                       capture_output=True, text=True)
    assert "IMPORT_ERROR" in r.stdout
