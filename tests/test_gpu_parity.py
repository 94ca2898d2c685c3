"""GPU parity: the gfx950 correlator against the CPU oracle, bit for bit.

Integer work, so the bar is exact equality, and every visibility is
compared: small and ragged cases against the oracle run in the test, the
full-size N=2048 channel against the oracle run in the test and its recorded
digest.  Properties that hold at any size (diagonal power, a rank-1 tone's
closed form) are checked beside them."""
import ctypes

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


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(X, x, n=None, re_low=False, reset=True):
    n = x.shape[1] if n is None else n
    c = X.Correlator(n, 1, re_low=re_low)
    c.correlate(0, gpu(x))
    out = c.dump(0, reset=reset).cpu().numpy().astype(np.int64)
    c.close()
    return out


SHAPES = [(1, 1), (1, 100), (2, 33), (3, 7), (5, 64), (31, 31), (64, 4096), (100, 1000),
          (127, 65), (128, 128), (129, 300), (200, 257), (256, 32), (300, 1000), (513, 129)]


@pytest.mark.parametrize("n,t", SHAPES)
def test_mfma_matches_oracle(X, n, t):
    print(f"mfma parity n={n} t={t}", flush=True)
    x = synth.uniform_bytes(n, t, seed=1000 + n + t)
    np.testing.assert_array_equal(run(X, x), oracle.correlate(x))


@pytest.mark.parametrize("n,t", [(1, 5), (7, 33), (64, 4096), (130, 257)])
def test_reference_kernel_matches_oracle(X, n, t):
    x = synth.uniform_bytes(n, t, seed=2000 + n)
    got = X.correlate_reference(gpu(x)).cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(got, oracle.correlate(x))


def test_small_workload_n64_t4096(X):
    x = synth.uniform_bytes(64, 4096, seed=1)
    np.testing.assert_array_equal(run(X, x), oracle.correlate(x))


def test_chime_statistics_n256(X):
    x = synth.chime_channel(256, 2000, seed=2)
    np.testing.assert_array_equal(run(X, x), oracle.correlate(x))


def test_empty_time_axis(X):
    c = X.Correlator(40, 1)
    c.correlate(0, torch.empty((0, 40), dtype=torch.uint8, device="cuda"))
    assert c.samples_integrated(0) == 0
    assert not c.dump(0).any().item()


def test_re_low_order(X):
    x = synth.uniform_bytes(70, 300, seed=3)
    np.testing.assert_array_equal(run(X, x, re_low=True), oracle.correlate(x, re_low=True))


@pytest.mark.parametrize("n,stride,offset", [(100, 101, 0), (100, 128, 1), (61, 67, 3), (128, 130, 2),
                                             (256, 261, 3), (400, 400, 5), (1000, 1001, 1)])
def test_strides_and_misaligned_base(X, n, stride, offset):
    t = 77
    big = synth.uniform_bytes(stride + offset, t, seed=4 + n)
    dev = gpu(big)[:, offset:offset + n]          # row stride = stride + offset
    c = X.Correlator(n, 1)
    c.correlate(0, dev)
    got = c.dump(0).cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(got, oracle.correlate(big[:, offset:offset + n]))


@pytest.mark.parametrize("n", [3, 7, 8, 9, 15, 23, 100, 131, 250])
def test_unaligned_rows_every_base_offset(X, n):
    # rows at every byte offset modulo 8 with a stride that is not a
    # multiple of 8: one 8-byte load per row at any address; the lane whose
    # eight inputs cross input N - 1 reads the eight bytes ending there and
    # shifts (N >= 8), single bytes for N < 8.  T = 70 crosses a stage.
    t, stride = 70, n + 5
    big = synth.uniform_bytes(stride + 8, t, seed=4700 + n)
    for offset in range(8):
        print(f"unaligned rows n={n} offset={offset}", flush=True)
        dev = gpu(big)[:, offset:offset + n]
        c = X.Correlator(n, 1)
        try:
            c.correlate(0, dev)
            got = c.dump(0).cpu().numpy().astype(np.int64)
        finally:
            c.close()
        np.testing.assert_array_equal(got, oracle.correlate(big[:, offset:offset + n]))


def test_accumulates_across_calls(X):
    n = 150
    chunks = [37, 1000, 5, 2048, 1]
    x = synth.uniform_bytes(n, sum(chunks), seed=5)
    c = X.Correlator(n, 2)
    t = 0
    for k in chunks:
        c.correlate(1, gpu(x[t:t + k]))
        t += k
    assert c.samples_integrated(1) == t and c.samples_integrated(0) == 0
    np.testing.assert_array_equal(c.dump(1, reset=False).cpu().numpy(), oracle.correlate(x))
    # keep integrating after a non-resetting dump
    c.correlate(1, gpu(x[:100]))
    ref = oracle.correlate(x) + oracle.correlate(x[:100])
    np.testing.assert_array_equal(c.dump(1).cpu().numpy(), ref)
    assert c.samples_integrated(1) == 0
    assert not c.dump(1).any().item()
    assert not c.dump(0).any().item()


def test_slots_are_independent(X):
    n = 64
    xs = [synth.uniform_bytes(n, 200 + 50 * s, seed=10 + s) for s in range(3)]
    c = X.Correlator(n, 3)
    for s in (2, 0, 1):
        c.correlate(s, gpu(xs[s]))
    for s in range(3):
        np.testing.assert_array_equal(c.dump(s).cpu().numpy(), oracle.correlate(xs[s]))


def test_reset(X):
    x = synth.uniform_bytes(64, 100, seed=20)
    c = X.Correlator(64, 1)
    c.correlate(0, gpu(x))
    c.reset(0)
    assert c.samples_integrated(0) == 0
    c.correlate(0, gpu(x[:10]))
    np.testing.assert_array_equal(c.dump(0).cpu().numpy(), oracle.correlate(x[:10]))


def test_overflow_guard_and_exact_bound(X):
    """All samples -8-8j: every Re term is 128, the largest there is.  At the
    integration bound Re = 128 * 16,777,215 = 2,147,483,520 in every pair;
    one more sample is refused and changes nothing."""
    n = 64
    tmax = X.max_integration()
    chunk = 1 << 20
    zeros = torch.zeros((chunk, n), dtype=torch.uint8, device="cuda")
    c = X.Correlator(n, 1)
    done = 0
    while done < tmax:
        k = min(chunk, tmax - done)
        c.correlate(0, zeros[:k])
        done += k
    assert c.samples_integrated(0) == tmax
    with pytest.raises(X.XengError) as e:
        c.correlate(0, zeros[:1])
    assert e.value.status == X.XENG_EOVERFLOW
    assert c.samples_integrated(0) == tmax
    v = c.dump(0, reset=False).cpu().numpy()
    assert (v[:, 0] == 128 * tmax).all() and (v[:, 0] == 2_147_483_520).all()
    assert (v[:, 1] == 0).all()
    # the refused call changed nothing; after a reset integration resumes
    c.reset(0)
    c.correlate(0, zeros[:1])
    assert (c.dump(0).cpu().numpy()[:, 0] == 128).all()


def test_argument_errors(X):
    c = X.Correlator(32, 2)
    L = X.lib()
    buf = torch.zeros((10, 32), dtype=torch.uint8, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert L.xeng_correlate(c.handle, 2, p, 10, 32, None) == X.XENG_EINVAL     # bad slot
    assert L.xeng_correlate(c.handle, -1, p, 10, 32, None) == X.XENG_EINVAL
    assert L.xeng_correlate(c.handle, 0, p, 10, 31, None) == X.XENG_EINVAL     # stride < N
    assert L.xeng_correlate(c.handle, 0, None, 10, 32, None) == X.XENG_EINVAL  # null samples
    assert L.xeng_correlate(c.handle, 0, p, -1, 32, None) == X.XENG_EINVAL
    assert L.xeng_dump(c.handle, 0, None, 1, None) == X.XENG_EINVAL
    assert c.samples_integrated(0) == 0


def test_dump_to_pinned_host(X):
    x = synth.uniform_bytes(90, 64, seed=21)
    c = X.Correlator(90, 1)
    c.correlate(0, gpu(x))
    host = torch.empty((X.tri(90), 2), dtype=torch.int32, pin_memory=True)
    c.dump(0, out=host)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host.numpy(), oracle.correlate(x))


def kernel_id(X, name):
    """auto: the eight-wave DMA kernel where the job allows it; dma4: its
    four-wave instance; general: the 128 x 128 kernel."""
    return {"auto": X.XENG_KERNEL_AUTO, "general": X.XENG_KERNEL_GENERAL, "dma4": X.XENG_KERNEL_DMA4}[name]


def test_tuning_does_not_change_results(X):
    x = synth.uniform_bytes(512, 2000, seed=22)
    outs = []
    try:
        for wpc, ms, kern in ((2, 4, X.XENG_KERNEL_AUTO), (1, 1, X.XENG_KERNEL_GENERAL),
                              (2, 1, X.XENG_KERNEL_GENERAL), (1, 64, X.XENG_KERNEL_AUTO),
                              (2, 1, X.XENG_KERNEL_AUTO), (2, 4, X.XENG_KERNEL_DMA4),
                              (2, 1, X.XENG_KERNEL_DMA4)):
            X.set_tuning(wpc, ms, kern)
            outs.append(run(X, x))
    finally:
        X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    np.testing.assert_array_equal(outs[0], oracle.correlate(x))


# N a multiple of 16 with aligned arrays takes the DMA kernel; the sample
# counts straddle its 64-sample stages and the pieces' boundaries, and N
# that is not a multiple of its 256-input workgroup tile leaves edge tiles
# (272 and 1904: an odd number of 128-input tiles, so the last workgroup
# tile has no right half).
@pytest.mark.parametrize("n,t", [(256, 1), (256, 63), (256, 64), (256, 65), (512, 1000),
                                 (768, 4097), (1024, 333), (16, 1), (48, 65), (144, 300),
                                 (272, 129), (400, 1000), (1008, 333), (1904, 64), (2000, 200)])
@pytest.mark.parametrize("kernel", ["auto", "general", "dma4"])
def test_both_kernels_match_oracle(X, n, t, kernel):
    print(f"kernel={kernel} n={n} t={t}", flush=True)
    x = synth.uniform_bytes(n, t, seed=3000 + n + t)
    try:
        X.set_tuning(0, 0, kernel_id(X, kernel))
        got = run(X, x)
    finally:
        X.set_tuning(0, 0, X.XENG_KERNEL_AUTO)
    np.testing.assert_array_equal(got, oracle.correlate(x))


@pytest.mark.parametrize("kernel", ["auto", "general", "dma4"])
def test_both_kernels_re_low(X, kernel):
    n, t = 512, 1000
    print(f"re_low kernel={kernel} n={n} t={t}", flush=True)
    x = synth.uniform_bytes(n, t, seed=77)
    try:
        X.set_tuning(0, 0, kernel_id(X, kernel))
        got = run(X, x, re_low=True)
    finally:
        X.set_tuning(0, 0, X.XENG_KERNEL_AUTO)
    np.testing.assert_array_equal(got, oracle.correlate(x, re_low=True))


@pytest.mark.parametrize("kernel", ["auto", "general", "dma4"])
def test_pieces_split_past_register_bound(X, kernel):
    # T beyond 2^16 samples: the DMA kernel's plan cuts every tile into
    # several pieces (atomic flushes); extreme samples maximise the sums
    n, t = 256, 70_000
    print(f"long pieces kernel={kernel} n={n} t={t}", flush=True)
    rng = np.random.default_rng(5)
    x = rng.choice(np.array([0x00, 0x0F, 0xF0, 0xFF, 0x80, 0x08], dtype=np.uint8), size=(t, n))
    try:
        X.set_tuning(1, 1 << 20, kernel_id(X, kernel))
        got = run(X, x)
    finally:
        X.set_tuning(2, 4, X.XENG_KERNEL_AUTO)     # the library's defaults
    np.testing.assert_array_equal(got, oracle.correlate(x))


def test_kernels_mixed_on_one_slot(X):
    # both kernels accumulate into the same layout
    n = 512
    x = synth.uniform_bytes(n, 700, seed=31)
    c = X.Correlator(n, 1)
    try:
        X.set_tuning(0, 0, X.XENG_KERNEL_GENERAL)
        c.correlate(0, gpu(x[:300]))
        X.set_tuning(0, 0, X.XENG_KERNEL_AUTO)
        c.correlate(0, gpu(x[300:]))
    finally:
        X.set_tuning(0, 0, X.XENG_KERNEL_AUTO)
    np.testing.assert_array_equal(c.dump(0).cpu().numpy(), oracle.correlate(x))


# ---------------------------------------------------------------------------
# Full-size workload: N=2048, T=32768, in the launch configuration the
# benchmark times.
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def full_size(X):
    import parity_util as pu
    print("full-size n=2048 t=32768: generating", flush=True)
    x = pu.fc.channel_n2048()
    c = X.Correlator(2048, 1)
    c.correlate(0, gpu(x))
    v = c.dump(0).cpu().numpy().astype(np.int64)
    c.close()
    return x, v


def test_full_size_matches_oracle(X, full_size):
    """Every one of the N(N+1)/2 = 2,098,176 visibilities of the N=2048,
    T=32768 channel, in the launch configuration the benchmark times, equals
    the oracle's (computed here on the host's cores, and its recorded digest)."""
    import parity_util as pu
    x, v = full_size
    print("full-size n=2048 t=32768: oracle", flush=True)
    ref = oracle.correlate(x)
    if not np.array_equal(v, ref):
        raise AssertionError(pu.first_difference(v, ref, 2048))
    pu.assert_matches_oracle_digest("channel_n2048_t32768", v, x)


def test_full_size_diagonal_is_power(X, full_size):
    x, v = full_size
    n = 2048
    re = (x >> 4).astype(np.int64) - 8
    im = (x & 15).astype(np.int64) - 8
    p = (re * re + im * im).sum(axis=0)
    d = np.array([oracle.tri_index(i, i, n) for i in range(n)])
    np.testing.assert_array_equal(v[d, 0], p)
    assert not v[d, 1].any()


def test_full_size_rank1_tone_closed_form(X):
    n, t = 2048, 32768
    x, g_re, g_im = synth.rank1_tone(n, t, seed=9, quarter_turns=1)
    c = X.Correlator(n, 1)
    c.correlate(0, gpu(x))
    v = c.dump(0).cpu().numpy().astype(np.int64)
    iu, ju = np.triu_indices(n)
    # T * g_i * conj(g_j)
    re = t * (g_re[iu] * g_re[ju] + g_im[iu] * g_im[ju])
    im = t * (g_im[iu] * g_re[ju] - g_re[iu] * g_im[ju])
    np.testing.assert_array_equal(v[:, 0], re)
    np.testing.assert_array_equal(v[:, 1], im)


def test_full_size_deterministic(X, full_size):
    x, v = full_size
    c = X.Correlator(2048, 1)
    c.correlate(0, gpu(x))
    np.testing.assert_array_equal(c.dump(0).cpu().numpy(), v)


def test_clock_probe_leaves_results_unchanged(X):
    # the wide kernel's workgroup 0 stamps its start and end; the shader
    # clock derived from the stamps is plausible, and results are unchanged
    x = synth.uniform_bytes(512, 3000, seed=77)
    ref = oracle.correlate(x)
    buf = torch.zeros(8, dtype=torch.int64, device="cuda")
    X.clock_probe(buf)
    try:
        got = run(X, x)
    finally:
        X.clock_probe(None)
    torch.cuda.synchronize()
    c = buf.cpu().numpy()
    print("clock stamps", c[:4].tolist(), "sclk", X.sclk_ghz(buf), flush=True)
    assert c[2] > c[0] > 0 and c[3] > c[1] > 0 and not c[4:].any()
    assert 0.3 < X.sclk_ghz(buf) < 3.5
    np.testing.assert_array_equal(got, ref)
    with pytest.raises(ValueError):
        X.clock_probe(torch.zeros(4, dtype=torch.int32, device="cuda"))


def test_dump_batch_matches_single_dumps_and_oracle(X):
    # several contexts of different N (one with N a multiple of 256, which
    # the DMA kernel integrates) and several slots each; one batched export
    # with resets on some jobs only
    print("dump batch: N in {1, 129, 300, 512}", flush=True)
    cases = [(1, 2, 33), (129, 3, 300), (300, 2, 257), (512, 2, 1024)]
    corrs, data = [], {}
    for n, slots, t in cases:
        c = X.Correlator(n, slots)
        for s in range(slots):
            x = synth.uniform_bytes(n, t + 17 * s, seed=[40, n, s])
            c.correlate(s, gpu(x))
            data[(n, s)] = x
        corrs.append(c)
    jobs, want = [], []
    for c in corrs:
        for s in range(c.n_slots):
            reset = (s + c.n_inputs) % 2 == 0
            jobs.append((c, s, None, reset))
            want.append(oracle.correlate(data[(c.n_inputs, s)]))
    outs = X.dump_batch(jobs)
    for (c, s, _, reset), got, w in zip(jobs, outs, want):
        np.testing.assert_array_equal(got.cpu().numpy().astype(np.int64), w)
        # reset jobs zeroed their slot and counter; the others kept both
        if reset:
            assert c.samples_integrated(s) == 0
            assert not c.dump(s, reset=False).any()
        else:
            assert c.samples_integrated(s) > 0
            np.testing.assert_array_equal(c.dump(s, reset=False).cpu().numpy().astype(np.int64), w)
    # a second batch over a subset, after more data, into caller buffers
    c = corrs[1]
    x = synth.uniform_bytes(129, 64, seed=41)
    c.correlate(0, gpu(x))
    bufs = [torch.full((X.tri(n), 2), -7, dtype=torch.int32, device="cuda") for n in (129, 300)]
    X.dump_batch([(c, 0, bufs[0], True), (corrs[2], 1, bufs[1], True)])
    s0 = oracle.correlate(x) + (0 if (0 + 129) % 2 == 0 else oracle.correlate(data[(129, 0)]))
    np.testing.assert_array_equal(bufs[0].cpu().numpy().astype(np.int64), s0)
    np.testing.assert_array_equal(bufs[1].cpu().numpy().astype(np.int64), oracle.correlate(data[(300, 1)]))
    assert X.dump_batch([]) == []
    for cc in corrs:
        cc.close()


def test_dump_batch_argument_errors(X):
    c = X.Correlator(64, 2)
    d = X.Correlator(128, 1)
    with pytest.raises(X.XengError):
        X.dump_batch([(c, 0), (c, 0)])              # one slot twice
    with pytest.raises(X.XengError):
        X.dump_batch([(c, 2)])                      # no such slot
    with pytest.raises(ValueError):
        X.dump_batch([(c, 0, torch.empty(5, dtype=torch.int32, device="cuda"))])
    L = X.lib()
    arr = (X._DumpJob * 2)()
    out = torch.empty((X.tri(64), 2), dtype=torch.int32, device="cuda")
    arr[0] = X._DumpJob(c.handle, 0, 1, out.data_ptr(), 0, 0)
    arr[1] = X._DumpJob(d.handle, 0, 2, out.data_ptr(), 0, 0)   # reset must be 0 or 1
    assert L.xeng_dump_batch(arr, 2, None) == X.XENG_EINVAL
    arr[1] = X._DumpJob(d.handle, 0, 1, None, 0, 0)             # no output
    assert L.xeng_dump_batch(arr, 2, None) == X.XENG_EINVAL
    arr[1] = X._DumpJob(d.handle, 0, 1, out.data_ptr(), 1, 0)   # reserved must be 0
    assert L.xeng_dump_batch(arr, 2, None) == X.XENG_EINVAL
    c.close()
    d.close()


def test_library_int8_gemm_cross_check(X):
    # an independent GPU path: unpack the samples into int8 matrices with
    # plain tensor ops and form the products with the vendor int8 GEMM
    # (torch._int_mm, int32 accumulation, exact at these sizes):
    #   U = [Re | Im] (N x 2T), W = [-Im | Re];  Re V = U U^T, Im V = U W^T
    # (V_ij = sum x_i conj(x_j): Im = Im_i Re_j - Re_i Im_j)
    n, t = 512, 4096
    print(f"library int8 GEMM cross-check n={n} t={t}", flush=True)
    x = synth.uniform_bytes(n, t, seed=4242)
    xd = gpu(x)
    try:
        hi = (xd >> 4).to(torch.int16) - 8
        lo = (xd & 15).to(torch.int16) - 8
        re, im = hi.to(torch.int8).t(), lo.to(torch.int8).t()          # [n, t]
        u = torch.cat([re, im], dim=1).contiguous()                     # [n, 2t]
        w = torch.cat([-im, re], dim=1).contiguous()
        vr = torch._int_mm(u, u.t().contiguous())
        vi = torch._int_mm(u, w.t().contiguous())
        torch.cuda.synchronize()
    except (RuntimeError, NotImplementedError) as e:
        pytest.skip(f"int8 GEMM not available in this torch build: {e}")
    iu = torch.triu_indices(n, n, device="cuda")
    lib_out = torch.stack([vr[iu[0], iu[1]], vi[iu[0], iu[1]]], dim=1).cpu().numpy().astype(np.int64)
    got = run(X, x)
    np.testing.assert_array_equal(got, lib_out)


# N >= 256 that the DMA kernel cannot read in place (N not a multiple of 16,
# or an odd stride or base) is copied into zero-padded rows first; long
# integrations go in chunks of time rows
@pytest.mark.parametrize("n,t", [(1000, 3000), (2047, 129), (260, 65), (300, 5)])
def test_padded_path_matches_oracle_and_general_kernel(X, n, t):
    print(f"padded path n={n} t={t}", flush=True)
    x = synth.uniform_bytes(n, t, seed=[61, n, t])
    got = run(X, x)
    np.testing.assert_array_equal(got, oracle.correlate(x))
    try:
        X.set_tuning(0, 0, X.XENG_KERNEL_GENERAL)
        gen = run(X, x)
    finally:
        X.set_tuning(0, 0, X.XENG_KERNEL_AUTO)
    np.testing.assert_array_equal(got, gen)


def test_padded_path_accumulates_and_resets(X):
    # two calls into one slot (the second not into a fresh slot), then a
    # reset and a third call
    n = 1000
    xs = [synth.uniform_bytes(n, t, seed=[62, t]) for t in (200, 333, 64)]
    c = X.Correlator(n, 1)
    c.correlate(0, gpu(xs[0]))
    c.correlate(0, gpu(xs[1]))
    assert c.samples_integrated(0) == 533
    got = c.dump(0).cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(got, oracle.correlate(np.concatenate(xs[:2])))
    c.correlate(0, gpu(xs[2]))
    np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64), oracle.correlate(xs[2]))
    c.close()


def test_padded_path_in_chunks(X):
    # the padded path's scratch lowered so that T = 3000 at N = 1000 runs in
    # three chunks of 1472, 1472 and 56 rows (a tail shorter than one
    # 64-sample stage): scratch reused across chunks, the later chunks
    # adding into a slot that already holds the earlier ones, a plan per
    # chunk; then a second call into the same slot
    n, t = 1000, 3000
    print(f"padded path in chunks n={n} t={t}", flush=True)
    xs = [synth.uniform_bytes(n, t, seed=[63, k]) for k in range(2)]
    try:
        X.set_pad_chunk_bytes(1472 * 1008)
        c = X.Correlator(n, 1)
        c.correlate(0, gpu(xs[0]))
        np.testing.assert_array_equal(c.dump(0, reset=False).cpu().numpy().astype(np.int64),
                                      oracle.correlate(xs[0]))
        c.correlate(0, gpu(xs[1]))
        assert c.samples_integrated(0) == 2 * t
        np.testing.assert_array_equal(c.dump(0).cpu().numpy().astype(np.int64),
                                      oracle.correlate(np.concatenate(xs)))
        c.close()
    finally:
        X.set_pad_chunk_bytes(0)


def test_calls_refused_while_capturing(X):
    # only xeng_batch_launch may be captured: the others return
    # XENG_ENOTSUP while their stream captures, queue nothing and leave the
    # counters alone
    n = 64
    L = X.lib()
    c = X.Correlator(n, 2)
    x = gpu(synth.uniform_bytes(n, 100, seed=64))
    c.correlate(0, x)
    torch.cuda.synchronize()
    out = torch.zeros((X.tri(n), 2), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    p = ctypes.c_void_p(x.data_ptr())
    codes = {}
    with torch.cuda.graph(g, stream=s):
        h = ctypes.c_void_p(s.cuda_stream)
        codes["correlate"] = L.xeng_correlate(c.handle, 1, p, 100, n, h)
        codes["dump"] = L.xeng_dump(c.handle, 0, ctypes.c_void_p(out.data_ptr()), 1, h)
        codes["reset"] = L.xeng_reset(c.handle, 0, h)
        arr = (X._Job * 1)()
        arr[0] = X._Job(c.handle, 1, 0, p, 100, n)
        codes["batch"] = L.xeng_correlate_batch(arr, 1, h)
        darr = (X._DumpJob * 1)()
        darr[0] = X._DumpJob(c.handle, 0, 1, out.data_ptr(), 0, 0)
        codes["dump_batch"] = L.xeng_dump_batch(darr, 1, h)
    assert all(v == X.XENG_ENOTSUP for v in codes.values()), codes
    assert c.samples_integrated(0) == 100 and c.samples_integrated(1) == 0
    g.replay()
    torch.cuda.synchronize()
    assert not out.any()
    ref = oracle.correlate(x.cpu().numpy())
    np.testing.assert_array_equal(c.dump(0).cpu().numpy(), ref)
    assert not c.dump(1).any()
    c.close()
