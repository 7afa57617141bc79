import os
import sys

# The oracle makes many small LAPACK calls (SVDs of a few hundred columns, QRs
# of thin panels), for which threaded BLAS is slower, not faster. Set before
# NumPy / SciPy load their BLAS libraries (SciPy's own copy reads this too).
for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import pytest  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs the HIP library")
    # BLAS libraries loaded before this file (by a plugin) keep their own
    # thread count; limit those too.
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1, user_api="blas")
    except Exception:
        pass


@pytest.fixture(autouse=True)
def _gpu_context_first(request):
    """GPU tests create torch's device context before the library's first HIP
    call, so torch and the library share one initialised runtime."""
    if request.node.get_closest_marker("gpu") is not None:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
            torch.zeros(1, device="cuda")
    yield
