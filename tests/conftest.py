import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def _ensure_built():
    lib = os.path.join(ROOT, "paper_2108_08730_amd", "libhelm27.so")
    if not os.path.exists(lib):
        from paper_2108_08730_amd.build import build
        build()


_ensure_built()
