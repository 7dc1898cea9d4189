"""The C-ABI library loads, exports every entry point its header declares,
and rejects bad configurations without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2207_06649_amd import pmbs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(pmbs_[a-z_]+)\s*\(", src))
    return names


def test_every_declared_symbol_is_exported():
    L = pmbs.lib()
    names = declared_functions()
    assert len(names) >= 14
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_defaults_and_workspace_query():
    cfg = pmbs.default_config()
    assert cfg.solver_iters == 10 and cfg.max_contacts == 128
    assert cfg.dt == pytest.approx(1 / 240)
    n = C.c_size_t(0)
    assert pmbs.lib().pmbs_sim_query_workspace(C.byref(cfg), C.byref(n)) == 0
    # 13 + 8 floats per body, per-env regions, 256-byte aligned
    assert n.value >= 21 * 4 * cfg.max_bodies and n.value % 256 == 0
    cfg2 = pmbs.default_config(pool_slots=100, pool_stride=21)
    n2 = C.c_size_t(0)
    assert pmbs.lib().pmbs_sim_query_workspace(C.byref(cfg2), C.byref(n2)) == 0
    assert n2.value - n.value >= 100 * 21 * 13 * 4


@pytest.mark.parametrize("field,value", [("max_contacts", 100), ("max_envs", 0), ("dt", 0.0),
                                         ("pool_slots", 5)])
def test_bad_config_rejected(field, value):
    cfg = pmbs.default_config(**{field: value})
    n = C.c_size_t(0)
    st = pmbs.lib().pmbs_sim_query_workspace(C.byref(cfg), C.byref(n))
    assert st == -1
    assert pmbs.lib().pmbs_last_error()


def test_create_rejects_small_workspace_without_gpu():
    cfg = pmbs.default_config()
    h = C.c_void_p()
    st = pmbs.lib().pmbs_sim_create(C.byref(cfg), C.c_void_p(256), 16, None, C.byref(h))
    assert st == -2 and not h.value


def test_server_config_and_workspace_size():
    """Server defaults and the workspace size of the node pool (no GPU)."""
    import ctypes as C
    from paper_2207_06649_amd import pmbs
    c = pmbs.server_config(max_requests=4, pool_slots=1000, max_envs=256)
    assert c.max_depth == 5 and c.n_substeps == 120 and c.graph == 1 and c.sim.max_contacts == 256
    n = C.c_size_t(0)
    assert pmbs._server_lib().pmbs_server_query_workspace(C.byref(c), C.byref(n)) == 0
    assert n.value >= 1000 * 31 * 13 * 4
    bad = pmbs.server_config(max_requests=0)
    assert pmbs._server_lib().pmbs_server_query_workspace(C.byref(bad), C.byref(n)) == -1  # invalid argument


def test_counter_record_key_ignores_comments(tmp_path, monkeypatch):
    """The HBM-traffic record is keyed by the kernel sources' code: a comment
    edit keeps the key, a code edit changes it."""
    import shutil
    import bench
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, rel), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    key = bench.kernel_source_hash()
    src = tmp_path / bench.KERNEL_SOURCES[0]
    text = src.read_text()
    src.write_text("// a new comment line\n" + text.replace("// ", "//  ", 3))
    assert bench.kernel_source_hash() == key
    src.write_text(text.replace("constexpr int POLY = 8;", "constexpr int POLY = 9;", 1))
    assert bench.kernel_source_hash() != key
