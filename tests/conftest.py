import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C ABI)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionfinish(session, exitstatus):
    """Close the library's handles and release its streams and events once the GPU
    tests are done (before the interpreter tears down the HIP runtime)."""
    mod = sys.modules.get("paper_2501_06748_amd")
    torch = sys.modules.get("torch")
    if mod is None or torch is None or not torch.cuda.is_initialized():
        return
    try:
        mod.sbfwi_finalize()
    except Exception as exc:   # reported, never fatal for the session
        print(f"sbfwi_finalize: {exc}", flush=True)
