"""The autotuner's persistent cache: a tuned entry is written to the
tune-cache file of the device's architecture (valid JSON), is found by calls
of the same job class (largest N, power-of-two classes of the largest T and
of the job count), and is read back by a fresh process, whose correlation
with it matches the CPU oracle bit for bit."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_09481_amd import xeng
    xeng.lib()
    return xeng


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# the child: a fresh process that reads the cache file at its first device
# use, reports the configuration it found, and saves its correlation
CHILD = r"""
import json, os, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import torch, synth
from paper_2005_09481_amd import xeng
n, t, seed, out = int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]), sys.argv[5]
x = torch.from_numpy(synth.uniform_bytes(n, t, seed=seed)).cuda()
c = xeng.Correlator(n, 1)
tu = xeng.tuning_lookup([(c, 0, x)])
c.correlate(0, x)
np.save(out, c.dump(0).cpu().numpy())
print(json.dumps({"kernel": tu.kernel, "wgs_per_cu": tu.wgs_per_cu, "min_stages": tu.min_stages,
                  "plan_order": tu.plan_order, "source": tu.source}), flush=True)
"""


def test_tuned_entry_persists_and_reloads(X, tmp_path):
    n, t = 512, 2000
    path = X.tune_cache_path(0)
    assert path.startswith(os.environ["XENG_TUNE_DIR"]) and path.endswith(".json")
    x = synth.uniform_bytes(n, t, seed=901)
    c = X.Correlator(n, 1)
    try:
        job = [(c, 0, gpu(x))]
        assert X.tuning_lookup(job).source == X.XENG_TUNE_SETTINGS
        best = X.autotune(job, iters=2)
        print("autotuned", best, flush=True)
        assert best.saved and best.source == X.XENG_TUNE_MEASURED
        assert c.samples_integrated(0) == 0 and not c.dump(0, reset=False).any()

        # the file is JSON and holds the entry for this class
        doc = json.load(open(path))
        assert doc["arch"] == torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        mine = [e for e in doc["entries"] if (e["n"], e["t_class"], e["jobs_class"], e["dma"]) == (n, 10, 0, 1)]
        assert len(mine) == 1
        assert (mine[0]["kernel"], mine[0]["wgs_per_cu"], mine[0]["min_stages"], mine[0]["plan_order"]) == \
            (best.kernel, best.wgs_per_cu, best.min_stages, best.plan_order)

        # same class (T in [1024, 2048)) finds it; another T class does not
        same = X.tuning_lookup([(c, 0, gpu(x[:1500]))])
        assert same.source == X.XENG_TUNE_MEASURED and same.min_stages == best.min_stages
        assert X.tuning_lookup([(c, 0, gpu(synth.uniform_bytes(n, 4096, seed=1)))]).source == X.XENG_TUNE_SETTINGS

        # a fresh process reads the file at its first device use
        out = str(tmp_path / "child.npy")
        env = dict(os.environ)
        r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(n), "1500", "902", out],
                           env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        got = json.loads(r.stdout.strip().splitlines()[-1])
        print("child", got, flush=True)
        assert got == {"kernel": best.kernel, "wgs_per_cu": best.wgs_per_cu, "min_stages": best.min_stages,
                       "plan_order": best.plan_order, "source": X.XENG_TUNE_CACHE_FILE}
        np.testing.assert_array_equal(np.load(out), oracle.correlate(synth.uniform_bytes(n, 1500, seed=902)))
    finally:
        X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)      # drops this process's tuned entries
        c.close()
    assert X.tuning_lookup([(X.Correlator(n, 1), 0, gpu(x))]).source == X.XENG_TUNE_SETTINGS


def test_cache_file_with_bad_lines_is_skipped(X, tmp_path):
    # a file with a foreign architecture, malformed and out-of-range entries:
    # a fresh process ignores all of them and runs with the global settings
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    d = tmp_path / "cache"
    d.mkdir()
    f = d / f"xeng_tune_{arch}.json"
    f.write_text(
        '{"arch": "%s", "format": 1, "entries": [\n'
        '  {"n": 512, "t_class": 10, "jobs_class": 0, "dma": 1, "kernel": 9, "wgs_per_cu": 2, '
        '"min_stages": 4, "plan_order": 1, "us_per_launch": 1.0},\n'
        '  {"n": 512, "t_class": 10, "jobs_class": 0, "dma": 1, "kernel": 0, "wgs_per_cu": 2, '
        '"min_stages": 0, "plan_order": 1, "us_per_launch": 1.0},\n'
        '  {"n": 512, "t_class": 10, "jobs_class": 0, "dma": 1, "kernel": 0,\n'
        ']}\n' % arch)
    env = dict(os.environ, XENG_TUNE_DIR=str(d))
    out = str(tmp_path / "child.npy")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, "512", "1500", "903", out],
                       env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    got = json.loads(r.stdout.strip().splitlines()[-1])
    assert got["source"] == X.XENG_TUNE_SETTINGS
    np.testing.assert_array_equal(np.load(out), oracle.correlate(synth.uniform_bytes(512, 1500, seed=903)))
