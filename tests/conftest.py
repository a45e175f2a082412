import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_addoption(parser):
    parser.addoption(
        "--emulated-gpu", action="store_true", default=False,
        help="dry run of the gpu-marked tests on the CPU: the binding loads the CPU emulation of "
             "the HIP sources (tests/cpu_emu) instead of libevsim.so, so each test's logic and "
             "its oracle side execute without a GPU; steps that need torch device memory skip")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "long: a CPU run of a minute or more (sanitizer builds, "
                                       "exhaustive failure sweeps); runs with EMU_LONG=1")
    if config.getoption("--emulated-gpu"):
        sys.path.insert(0, os.path.join(ROOT, "tests", "cpu_emu"))
        import build as emu_build
        from paper_2209_04634_amd import sim
        sim.LIB_PATH = emu_build.build()
        sim._lib = None


def pytest_collection_modifyitems(config, items):
    # the default CPU suite stays a few minutes long; the long runs are opt-in
    if os.environ.get("EMU_LONG") == "1":
        return
    skip = pytest.mark.skip(reason="long CPU run (a minute or more serially); set EMU_LONG=1")
    for item in items:
        if "long" in item.keywords:
            item.add_marker(skip)


def _needs_device(excinfo) -> bool:
    text = str(excinfo.value)
    return any(m in text for m in ("Torch not compiled with CUDA", "No HIP GPUs",
                                   "no NVIDIA driver", "Found no NVIDIA driver",
                                   "CUDA driver initialization failed"))


@pytest.hookimpl(hookwrapper=True)
def pytest_runtest_makereport(item, call):
    outcome = yield
    rep = outcome.get_result()
    if (item.config.getoption("--emulated-gpu") and call.excinfo is not None
            and rep.failed and _needs_device(call.excinfo)):
        rep.outcome = "skipped"
        rep.longrepr = (str(item.fspath), item.location[1] or 0,
                        "emulated dry run: this step needs torch device memory")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle
