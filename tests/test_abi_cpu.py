"""The C-ABI library builds, loads and exports every entry point include/*.h declares (no GPU)."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

from paper_2209_04634_amd import sim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**\s*"
                             r"([a-z][a-z0-9_]*)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sim_create", "sim_push_frame", "sim_push_frames", "sim_drain_events",
                     "sim_drain_keys", "sim_destroy", "sim_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = sim.load()
    out = subprocess.run(["nm", "-D", "--defined-only", sim.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_host_only_entry_points():
    lib = sim.load()
    cfg = sim.SimConfig()
    lib.sim_config_init(ctypes.byref(cfg))
    assert (cfg.method, cfg.transform, cfg.n_interp) == (sim.BASIC, sim.LOG, 10)
    assert cfg.c_pos == pytest.approx(0.2) and cfg.log_eps == pytest.approx(1e-3)
    assert cfg.mask_threshold == -1.0 and cfg.hip_stream is None
    for code in range(0, -9, -1):
        assert lib.sim_strerror(code)
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    assert lib.sim_create(None, ctypes.byref(h)) == sim.E_INVAL
    bad = sim.SimConfig()
    lib.sim_config_init(ctypes.byref(bad))
    bad.width, bad.height = 0, 10
    assert lib.sim_create(ctypes.byref(bad), ctypes.byref(h)) == sim.E_INVAL
    bad.width, bad.height, bad.c_pos = 10, 10, -1.0
    assert lib.sim_create(ctypes.byref(bad), ctypes.byref(h)) == sim.E_INVAL
    bad.c_pos, bad.n_interp = 0.2, 256
    assert lib.sim_create(ctypes.byref(bad), ctypes.byref(h)) == sim.E_INVAL
    bad.n_interp, bad.c_pos = 10, 1e-9     # R + C == R for reachable R
    assert lib.sim_create(ctypes.byref(bad), ctypes.byref(h)) == sim.E_INVAL


def test_product_path_does_not_use_the_oracle():
    """The HIP library and its binding never reference the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2209_04634_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if os.path.isfile(path) and path.endswith((".py", ".hip", ".h", ".cpp")):
            text = open(path).read()
            for needle in ("import oracle", "from oracle", "liboracle", "oracle_", "oracle/"):
                assert needle not in text, (path, needle)
    assert "liboracle" not in open(sim.LIB_PATH, "rb").read().decode("latin1")
