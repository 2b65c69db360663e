import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    # GPU tests can only run where a GPU is visible; elsewhere they are skipped
    # unless selected explicitly with -m gpu (then they fail loudly instead).
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    markexpr = config.getoption("-m") or ""
    if have_gpu or "gpu" in markexpr.replace("not gpu", ""):
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(autouse=True)
def _close_gpu_contexts(request):
    """Every library context a GPU test opens is closed when the test ends,
    passed or failed (a failed test's traceback would otherwise keep its
    contexts, and their device memory, streams and graphs, alive for the
    rest of the session), and the stream is drained before the next test."""
    if "gpu" not in request.keywords:
        yield
        return
    from paper_2502_09758_amd import maid as M

    opened = []
    inits = {cls: cls.__init__ for cls in (M.Maid, M.MaidBatch)}

    def wrap(cls):
        orig = inits[cls]

        def init(self, *a, **kw):
            orig(self, *a, **kw)
            opened.append(self)
        return init

    for cls in inits:
        cls.__init__ = wrap(cls)
    try:
        yield
    finally:
        for cls, orig in inits.items():
            cls.__init__ = orig
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
        for ctx in opened:
            ctx.close()
        opened.clear()
