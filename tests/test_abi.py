"""CPU-side checks of the C-ABI boundary: the HIP library loads and exports every function declared in
include/lcc.h, and the ctypes structures match the header's layout (no GPU compute)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lcc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lcc_[a-z_]+)\s*\(", src)) - {"lcc_alloc_fn", "lcc_free_fn"})


def test_library_exports_every_declared_symbol():
    from paper_2608_01503_amd import lcc
    lib = lcc.load()
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(lcc.EXPORTED) == names


def test_struct_layouts():
    from paper_2608_01503_amd import lcc
    assert ctypes.sizeof(lcc.lcc_graph) == 64
    assert ctypes.sizeof(lcc.lcc_lambda) == 24
    assert ctypes.sizeof(lcc.lcc_result) == 56
    assert ctypes.sizeof(lcc.lcc_options) == 4 + 4 + 3 * 32 + 8 + 8 + 4 + 4 + 8 + 4 + 4
    assert ctypes.sizeof(lcc.lcc_kernel_stat) == 32 + 8 + 8 + 8
    assert ctypes.sizeof(lcc.lcc_tuning) == 7 * 8 + 4 + 4


def test_host_only_entry_points():
    from paper_2608_01503_amd import lcc
    o = lcc.lcc_default_options()
    assert (o.pass_limit, o.n_phi, o.eps_num, o.eps_den, o.max_levels, o.symmetry) == (6, 2, 1, 10, 64, 0)
    assert (o.phi_num[0], o.phi_den[0], o.phi_until[0], o.phi_num[1], o.phi_den[1], o.phi_until[1]) == (3, 4, 4, 1, 4, 6)
    assert lcc.lcc_workspace_bytes(1000, 10000) > 0
    assert lcc.lcc_status_string(-2) == "graph not symmetric"
    t = lcc.lcc_default_tuning()
    assert lcc.tuning_dict(t) == {"bucket_max": [4, 8, 16, 32, 128, 1024, 8192], "grid_cap": 2048, "hash_shift": 0}
    assert lcc.tuning_dict(lcc.lcc_default_tuning(hash_shift=2))["hash_shift"] == 2
    assert lcc.tuning_dict(lcc.lcc_default_tuning(grid_cap=512))["grid_cap"] == 512
