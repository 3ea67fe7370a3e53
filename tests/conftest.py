import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")


def pytest_sessionstart(session):
    """Sanitizer runs (tests/sanitize.py) point the tests at instrumented
    builds of the library and the oracle through these variables."""
    lib = os.environ.get("T2S2_TEST_LIB")
    if lib:
        import paper_1911_12913_amd as t2s2

        t2s2.LIB_PATH = lib
        t2s2.load_library.__defaults__ = (lib,)
    olib = os.environ.get("T2S2_TEST_ORACLE_LIB")
    if olib:
        import oracle

        oracle._LIB = olib
        oracle._SRC = olib  # same mtime: never rebuilt over the instrumented copy
