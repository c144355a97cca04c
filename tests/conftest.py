import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # tuned schedules of the test session go to a file of its own, not the
    # user's cache (tests of the cache set their own path)
    if "AMGDD_TUNE_CACHE" not in os.environ:
        import tempfile
        os.environ["AMGDD_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="amgdd_tune_"), "schedules.json")
    # optional native backtraces on fatal signals (diagnostics only)
    if os.environ.get("AMGDD_CRASH_TRACE") == "1":
        so = os.path.join(ROOT, "tests", "native", "crash_trace.so")
        if os.path.exists(so):
            import ctypes
            ctypes.CDLL(so).crash_trace_install()
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: larger CPU case")
