import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: full-size configuration case")


def _ensure_built():
    lib = os.path.join(ROOT, "paper_1701_05975_amd", "libbcgpu.so")
    if not os.path.exists(lib):
        from paper_1701_05975_amd import build
        build.build()
    olib = os.path.join(ROOT, "oracle", "liboracle.so")
    if not os.path.exists(olib):
        import oracle
        oracle.build()


_ensure_built()
