"""The C-ABI library loads and exports every symbol include/agile.h declares; host-side
validation works without a GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

from paper_2504_19365_amd import agile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "agile.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(agile_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(agile.LIB_PATH):
        pytest.skip("libagile.so not built")
    return agile.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "agile_init" in names and "agile_async_read" in names and "agile_flush" in names
    for n in names:
        assert hasattr(L, n), n
    for n in ("agile_init", "agile_open_store", "agile_async_read", "agile_wait",
              "agile_release", "agile_flush"):
        assert n in names


def test_config_layout_and_defaults(L):
    cfg = agile.default_config()
    assert cfg.struct_size == C.sizeof(agile.Config) == 80
    assert cfg.line_bytes == 4096 and cfg.assoc == 8 and cfg.qp_depth == 64
    assert C.sizeof(agile.Stats) == 15 * 8 and C.sizeof(agile.Tables) == 24


@pytest.mark.parametrize("field,value", [
    ("line_bytes", 6000), ("line_bytes", 2048), ("qp_depth", 32), ("qp_depth", 96),
    ("assoc", 0), ("assoc", 3), ("cache_bytes", 4096 * 2), ("num_qp", 0), ("cache_bytes", 5000),
    ("num_qp", 2000), ("struct_size", 8),
])
def test_init_rejects_bad_config_without_touching_the_gpu(L, field, value):
    cfg = agile.default_config()
    setattr(cfg, field, value)
    h = C.c_void_p()
    assert L.agile_init(C.byref(cfg), C.byref(h)) == agile.EINVAL
    assert not h.value


def test_status_strings(L):
    for s in range(0, -9, -1):
        assert agile.status_string(s).startswith("AGILE_")
    assert L.agile_last_error(None) == b"no context"
