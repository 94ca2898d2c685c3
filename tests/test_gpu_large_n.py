"""GPU parity beyond the CHIME-sized channel: every visibility of large
arrays compared with the CPU oracle, bit for bit -- N = 8192 (64 tile rows,
the wide kernel over 1056 windows, a ragged last stage), N = 4112 (a
multiple of 16 but not of the 256-wide window: edge tiles past the last
input) and N = 4000 (not a multiple of 16: the padded path)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_09481_amd import xeng
    xeng.lib()
    return xeng


@pytest.mark.parametrize("n,t", [(8192, 1000), (4112, 777), (4000, 300)])
def test_large_n_matches_oracle(X, n, t):
    print(f"large n={n} t={t}", flush=True)
    x = synth.chime_channel(n, t, seed=6000 + n)
    c = X.Correlator(n, 1)
    try:
        c.correlate(0, torch.from_numpy(x).cuda())
        got = c.dump(0).cpu().numpy()
    finally:
        c.close()
    want = oracle.correlate(x)
    assert got.shape == want.shape == (n * (n + 1) // 2, 2)
    np.testing.assert_array_equal(got.astype(np.int64), want)
