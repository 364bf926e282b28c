import importlib.util
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def pytest_sessionstart(session):
    # the package loads libglasso.so at import: build it once if this checkout has none
    lib = os.path.join(ROOT, "paper_2205_10027_amd", "libglasso.so")
    if not os.path.exists(lib):
        spec = importlib.util.spec_from_file_location(
            "_glasso_build", os.path.join(ROOT, "paper_2205_10027_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
