"""GPU checks of the measurement calls: the matrix-core ceiling loop reports
a rate and a clock in the part's range, and refuses bad arguments."""
import ctypes

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_09481_amd import xeng
    xeng.lib()
    return xeng


def test_mfma_ceiling_in_range(X):
    mac_s, ghz = X.mfma_ceiling(60, 0)
    # 256 CUs x 4 SIMDs x 1024 int8 MAC per cycle at 2.4 GHz = 2.52e15 MAC/s;
    # under the power limit the clock and the rate are lower, never higher
    assert 0.2 * 2.52e15 < mac_s < 1.02 * 2.52e15
    assert 0.5 < ghz < 2.5
    # the rate follows the clock: MACs per shader cycle within the part's
    # 256 x 4 x 1024 = 1048576
    assert mac_s / (ghz * 1e9) < 1.02 * 1048576


def test_mfma_ceiling_argument_errors(X):
    mac, ghz = ctypes.c_double(), ctypes.c_double()
    L = X.lib()
    assert L.xeng_mfma_ceiling(0, 5, ctypes.byref(mac), ctypes.byref(ghz)) == X.XENG_EINVAL
    assert L.xeng_mfma_ceiling(-1, 50, ctypes.byref(mac), ctypes.byref(ghz)) == X.XENG_EINVAL
    assert L.xeng_mfma_ceiling(0, 50, None, ctypes.byref(ghz)) == X.XENG_EINVAL
