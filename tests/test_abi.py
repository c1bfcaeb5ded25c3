"""CPU checks of the boundary: the HIP library loads and exports every entry point the
public header declares (no GPU call is made), and the GPU build's marching-cubes table
(generated at build time from its rule) equals the oracle's rule, case by case."""
import ctypes
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2412_00291_amd", "libmapcore.so")


def _declared():
    txt = open(os.path.join(ROOT, "include", "mapcore.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(map_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_path():
    names = _declared()
    for n in ("map_create", "map_destroy", "map_integrate_lidar", "map_integrate_labels",
              "map_extract_mesh", "map_query_sdf", "map_sdf_pose_adjoint", "map_stats", "map_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_generated_mc_table_matches_oracle_rule():
    sys.path.insert(0, os.path.join(ROOT, "paper_2412_00291_amd", "csrc"))
    import gen_mc_table
    import oracle
    table = gen_mc_table.build_table()
    for mask in range(256):
        assert [tuple(t) for t in oracle.cube_triangles(mask).tolist()] == list(table[mask]), mask
