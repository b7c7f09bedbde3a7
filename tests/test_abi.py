"""The C ABI library loads and exports every function include/lbm.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared("lbm.h")
    for n in ("lbm_create", "lbm_destroy", "lbm_set_solid", "lbm_init_drops", "lbm_step", "lbm_measure_angle",
              "lbm_read", "lbm_write", "lbm_last_error"):
        assert n in names


@pytest.mark.parametrize("header", sorted(h for h in os.listdir(os.path.join(ROOT, "include")) if h.endswith(".h")))
def test_library_exports_every_declared_symbol(header):
    from paper_2202_06516_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("liblbm.so not built")
    lib = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in declared(header) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_structs_match_header_sizes():
    # lbm_angle is copied to the caller byte for byte: its size fixes the layout
    from paper_2202_06516_amd import lbm
    assert ctypes.sizeof(lbm.lbm_angle) == 8 + 4 * 4 + 3 * 8 + 3 * 8 + 64 * 8 + 64 * 3 * 8
    assert ctypes.sizeof(lbm.lbm_measure_opts) == 16


def test_config_default_host_only():
    from paper_2202_06516_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("liblbm.so not built")
    cfg = lbm.config_default(lbm.LBM_D2Q9)
    assert cfg.s_e == 1.64 and cfg.s_eps == 1.54 and cfg.s_q == 1.9
    assert abs(cfg.pr_a - 2 / 49) < 1e-16 and abs(cfg.pr_b - 2 / 21) < 1e-16 and cfg.pr_omega == 0.344
    assert cfg.n[2] == 1 and cfg.precision == lbm.LBM_F64


def test_product_path_does_not_import_the_oracle():
    # the library package never reaches into oracle/
    pkg = os.path.join(ROOT, "paper_2202_06516_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "lbm_oracle" not in src, f


def test_bench_refuses_several_gpus():
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]

