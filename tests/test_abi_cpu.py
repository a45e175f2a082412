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
    # one pixel could fire more than 2^24 events in one interval: 256 * (2 * 255 * 4096 + 3)
    bad.method, bad.transform, bad.n_interp, bad.c_pos, bad.c_neg = sim.DENSE, sim.LINEAR, 255, \
        2.0 ** -12, 2.0 ** -12
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


def test_host_only_entry_points_of_the_wider_rows():
    """New configuration fields, the estimator's parameters and the server's admission are
    validated on the host, before any device call."""
    lib = sim.load()
    cfg = sim.SimConfig()
    lib.sim_config_init(ctypes.byref(cfg))
    assert (cfg.thresh_mode, cfg.flow_source) == (sim.REFERENCE, sim.FLOW_SUPPLIED)
    h = ctypes.c_void_p()
    cfg.width = cfg.height = 16
    for field, value in (("method", 4), ("thresh_mode", 2), ("flow_source", 2)):
        bad = sim.SimConfig.from_buffer_copy(cfg)
        setattr(bad, field, value)
        assert lib.sim_create(ctypes.byref(bad), ctypes.byref(h)) == sim.E_INVAL, field
    for method in (sim.BASIC, sim.DIFFERENCE):          # estimated flow: dense and sparse only
        bad = sim.SimConfig.from_buffer_copy(cfg)
        bad.method, bad.flow_source = method, sim.FLOW_LK
        assert lib.sim_create(ctypes.byref(bad), ctypes.byref(h)) == sim.E_INVAL
    p = sim.SimLkParams()
    lib.sim_lk_params_init(ctypes.byref(p))
    assert (p.levels, p.radius, p.iterations) == (3, 7, 10)
    assert p.eps == pytest.approx(1e-4) and p.min_ratio == pytest.approx(1e-3)
    f = (ctypes.c_uint8 * 64)()
    pts = (ctypes.c_uint32 * 1)()
    fl = (ctypes.c_float * 2)()
    for field, value in (("levels", 5), ("radius", 0), ("radius", 16), ("iterations", 0),
                         ("eps", -1.0)):
        bad = sim.SimLkParams.from_buffer_copy(p)
        setattr(bad, field, value)
        assert lib.sim_lk_flow(f, f, 8, 8, pts, 1, fl, None, ctypes.byref(bad), sim.MEM_HOST,
                               None) == sim.E_INVAL, field
    assert lib.sim_lk_flow(f, f, 0, 8, pts, 1, fl, None, None, sim.MEM_HOST, None) == sim.E_INVAL
    assert lib.sim_lk_flow(f, f, 8, 8, None, 1, fl, None, None, sim.MEM_HOST, None) == sim.E_INVAL
    assert lib.sim_lk_flow(f, f, 8, 8, pts, 0, fl, None, None, sim.MEM_HOST, None) == sim.OK
    # server admission arithmetic and creation are host-side
    out = ctypes.c_uint64()
    small = sim.SimConfig.from_buffer_copy(cfg)
    small.method = sim.SPARSE
    assert lib.srv_footprint(ctypes.byref(small), 4, ctypes.byref(out)) == sim.OK
    sparse_fp = out.value
    small.method = sim.BASIC
    assert lib.srv_footprint(ctypes.byref(small), 4, ctypes.byref(out)) == sim.OK
    assert out.value < sparse_fp and out.value >= 256 * (4 + 2 + 4 + 16 + 32 + 16 + 4)
    srv = ctypes.c_void_p()
    assert lib.srv_create(1 << 30, 0, 4, ctypes.byref(srv)) == sim.E_INVAL
    assert lib.srv_create(1 << 30, 4, 4, ctypes.byref(srv)) == sim.OK
    assert lib.srv_destroy(srv) == sim.OK


def test_noalloc_flow_validates_on_the_host():
    """sim_lk_flow_noalloc refuses bad arguments and requests beyond its fixed scratch before any
    device call."""
    lib = sim.load()
    f = (ctypes.c_uint8 * 64)()
    pts = (ctypes.c_uint32 * 1)()
    fl = (ctypes.c_float * 2)()
    assert lib.sim_lk_flow_noalloc(f, f, 0, 8, pts, 1, fl, None, None, None) == sim.E_INVAL
    assert lib.sim_lk_flow_noalloc(f, f, 8, 8, None, 1, fl, None, None, None) == sim.E_INVAL
    assert lib.sim_lk_flow_noalloc(f, f, 4096, 4096, pts, 1, fl, None, None, None) == \
        sim.E_TOO_BIG
    assert lib.sim_lk_flow_noalloc(f, f, 8, 8, pts, 0, fl, None, None, None) == sim.OK
    assert lib.sim_strerror(sim.E_TOO_BIG) != lib.sim_strerror(-100)


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field offsets (a C program
    built against include/sim.h prints them)."""
    import subprocess
    pairs = [("sim_config", sim.SimConfig), ("sim_lk_params", sim.SimLkParams),
             ("sim_event", sim.SimEvent), ("sim_stats", sim.SimStats),
             ("sim_frames", sim.SimFrames), ("sim_server_stats", sim.ServerStats),
             ("sim_batch_timing", sim.SimBatchTiming)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sim.h"', 'int main(void) {']
    for cname, py in pairs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = {}
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    for ln in out.splitlines():
        c, f, v = ln.split()
        got[(c, f)] = int(v)
    for cname, py in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)
