"""GPU tests of the streaming server: real-time frame releases, continuous
batching over channels, admission as slots and device memory free up,
exports every
dump_frames frames.  Each export is compared bit for bit with the oracle on
the frames it covers, and with the same channel served alone."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 256
DUMP = 32          # frames per export (32 x 256 samples): several exports per run


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_09481_amd import xeng
    xeng.lib()
    return xeng


def frames_of(seed, n_frames=48, n=N):
    return synth.stream_frames(n, n_frames, seed=seed)


def expected(frames, first, count=DUMP):
    """Oracle over frames [first, first + count) of a cyclic source."""
    f = frames[[(first + k) % frames.shape[0] for k in range(count)]]
    return oracle.correlate(f.reshape(-1, frames.shape[2]))


def test_exports_match_oracle_and_alone(X):
    srcs = [frames_of(seed=[5, c]) for c in range(4)]
    srv = X.Server(N, dump_frames=DUMP, max_channels=4, launch_period_us=2000.0)
    chans = [srv.admit(torch.from_numpy(f).cuda(), start_s=0.002 * c, total_frames=3 * DUMP)
             for c, f in enumerate(srcs)]
    st = srv.run(0.4)
    print("serve 4 channels", st, flush=True)
    assert st["frames_done"] == 4 * 3 * DUMP and st["frames_dropped"] == 0 and st["dumps"] == 12
    assert st["p99_ms"] > 0
    got = []
    for c, f in zip(chans, srcs):
        info = srv.channel_info(c)
        assert info["state"] == 2 and info["dumps"] == 3 and info["last_dump_first_frame"] == 2 * DUMP
        v = srv.last_dump(c)
        np.testing.assert_array_equal(v.cpu().numpy(), expected(f, 2 * DUMP))
        got.append(v)
    srv.close()
    # channel 0 alone gives the same export
    solo = X.Server(N, dump_frames=DUMP, max_channels=1, launch_period_us=2000.0)
    c0 = solo.admit(torch.from_numpy(srcs[0]).cuda(), total_frames=3 * DUMP)
    solo.run(0.2)
    assert torch.equal(solo.last_dump(c0), got[0])
    solo.close()


def test_staggered_exports(X):
    # XENG_SERVER_STAGGER_EXPORTS: slot s exports at frame counts
    # m * DUMP - s * DUMP / slots; every export still equals the oracle over
    # the frames it covers
    srcs = [frames_of(seed=[8, c]) for c in range(4)]
    srv = X.Server(N, dump_frames=DUMP, max_channels=4, launch_period_us=2000.0, stagger_exports=True)
    chans = [srv.admit(torch.from_numpy(f).cuda(), start_s=0.001 * c, total_frames=3 * DUMP)
             for c, f in enumerate(srcs)]
    st = srv.run(0.4)
    print("staggered exports", st, flush=True)
    assert st["frames_done"] == 4 * 3 * DUMP and st["frames_dropped"] == 0
    firsts = set()
    for c, f in zip(chans, srcs):
        info = srv.channel_info(c)
        phase = info["slot"] * DUMP // 4
        assert info["dumps"] == 3
        # exports after DUMP - phase, 2 DUMP - phase, 3 DUMP - phase frames
        # (the first integration is the short one); the frames past the last
        # export are dropped when the channel finishes
        first = info["last_dump_first_frame"]
        assert first == 2 * DUMP - phase
        np.testing.assert_array_equal(srv.last_dump(c).cpu().numpy(), expected(f, first))
        firsts.add(first)
    assert len(firsts) == 4                      # four different phases
    srv.close()


def test_admission_waits_for_a_free_slot(X):
    # three channels, two slots: the third is admitted when one finishes
    srcs = [frames_of(seed=[6, c]) for c in range(3)]
    srv = X.Server(N, dump_frames=DUMP, max_channels=2, launch_period_us=2000.0)
    chans = [srv.admit(torch.from_numpy(f).cuda(), total_frames=2 * DUMP) for f in srcs]
    assert srv.channel_info(chans[2])["state"] == 0
    st = srv.run(0.4)
    print("admission", st, flush=True)
    assert st["frames_done"] == 3 * 2 * DUMP
    infos = [srv.channel_info(c) for c in chans]
    assert all(i["state"] == 2 and i["dumps"] == 2 for i in infos)
    reused = infos[2]["slot"]
    for c, f, i in zip(chans, srcs, infos):
        if c != chans[2] and i["slot"] == reused:
            with pytest.raises(X.XengError) as e:      # its slot went to channel 2
                srv.last_dump(c)
            assert e.value.status == X.XENG_EBUSY
            continue
        np.testing.assert_array_equal(srv.last_dump(c).cpu().numpy(), expected(f, DUMP))
    srv.close()


def test_host_sourced_frames(X):
    # pinned host frames, gathered into each channel's device ring on
    # release (one gather kernel per pass over every due frame)
    srcs = [frames_of(seed=[7, c], n_frames=40) for c in range(5)]
    srv = X.Server(N, dump_frames=DUMP, max_channels=5, ring_frames=16, launch_period_us=2000.0)
    hosts = [torch.from_numpy(f).pin_memory() for f in srcs]
    chans = [srv.admit(h, start_s=0.0005 * c, total_frames=2 * DUMP) for c, h in enumerate(hosts)]
    st = srv.run(0.3)
    print("host frames", st, flush=True)
    assert st["frames_dropped"] == 0 and st["frames_done"] == 5 * 2 * DUMP
    assert st["frames_gathered"] == 5 * 2 * DUMP
    for c, f in zip(chans, srcs):
        np.testing.assert_array_equal(srv.last_dump(c).cpu().numpy(), expected(f, DUMP))
    srv.close()


def test_host_frames_copied_when_not_gatherable(X):
    # pinned sources at an odd address cannot be gathered with 16-byte
    # loads: they are copied frame by frame on the copy streams (five
    # channels over four streams, so two share one), beside a gathered one
    srcs = [frames_of(seed=[8, c], n_frames=40) for c in range(6)]
    srv = X.Server(N, dump_frames=DUMP, max_channels=6, ring_frames=16, launch_period_us=2000.0)
    hosts = []
    for c, f in enumerate(srcs):
        if c == 5:
            hosts.append(torch.from_numpy(f).pin_memory())
            continue
        raw = torch.empty(f.size + 1, dtype=torch.uint8).pin_memory()
        view = raw[1:].view(f.shape)
        view.copy_(torch.from_numpy(f))
        hosts.append(view)
    chans = [srv.admit(h, start_s=0.0005 * c, total_frames=2 * DUMP) for c, h in enumerate(hosts)]
    st = srv.run(0.3)
    print("copied host frames", st, flush=True)
    assert st["frames_dropped"] == 0 and st["frames_done"] == 6 * 2 * DUMP
    assert st["frames_gathered"] == 2 * DUMP
    for c, f in zip(chans, srcs):
        np.testing.assert_array_equal(srv.last_dump(c).cpu().numpy(), expected(f, DUMP))
    srv.close()


def test_dropped_frames_are_never_integrated(X):
    # a host source whose ring (3 frames) overflows while the server waits
    # out a long launch period: the frames it drops must be passed over, not
    # integrated from the ring's stale contents, and still count towards the
    # export boundaries and the channel's end.  Every frame of the source is
    # the same, so each export is m x V(frame) for the m frames it integrated.
    frame = frames_of(seed=[9, 0], n_frames=1)
    host = torch.from_numpy(frame).pin_memory()
    srv = X.Server(N, dump_frames=16, max_channels=1, ring_frames=3, max_inflight=1,
                   frame_period_us=200.0, launch_period_us=20000.0)
    ch = srv.admit(host, total_frames=32)
    st = srv.run(0.2)
    print("dropping host source", st, flush=True)
    assert st["frames_released"] == 32 and st["frames_dropped"] > 0
    assert st["backlog_frames"] == 0
    assert st["frames_done"] + st["frames_dropped"] == 32
    info = srv.channel_info(ch)
    assert info["state"] == 2 and info["dumps"] == 2 and info["last_dump_first_frame"] == 16
    v1 = oracle.correlate(frame.reshape(-1, N)).astype(np.int64)
    got = srv.last_dump(ch).cpu().numpy().astype(np.int64)
    k = int(np.flatnonzero(v1)[0])
    m = got.flat[k] // v1.flat[k]
    np.testing.assert_array_equal(got, m * v1)
    assert 0 <= m <= 16 and 0 <= st["frames_done"] - m <= 16
    srv.close()


def test_server_argument_checks(X):
    with pytest.raises(X.XengError) as e:
        X.Server(N, dump_frames=0, max_channels=1)
    assert e.value.status == X.XENG_EINVAL
    with pytest.raises(X.XengError) as e:
        X.Server(N, max_channels=0, mem_budget_bytes=1000)          # not one channel fits
    assert e.value.status == X.XENG_ENOMEM
    srv = X.Server(2048, max_channels=0, mem_budget_bytes=3 * (X.slot_bytes(2048) + 2048 * 2049 * 4)
                   + 64 * 256 * 2048)
    assert srv.max_channels == 3                                   # slots the budget holds
    with pytest.raises(ValueError):
        srv.admit(torch.zeros((4, 256, 100), dtype=torch.uint8, device="cuda"))
    srv.close()


def test_full_size_n2048_every_export(X):
    # four device-sourced channels of N = 2048 (each cycling 48 distinct
    # frames), three exports each into an export ring: every export equals
    # the oracle over the frames it covers (recorded digests), and channel
    # 0 served alone gives the same exports as in the mix
    import parity_util as pu
    fc = pu.fc
    n, d = fc.SERVE_N, fc.SERVE_DUMP
    srcs = [fc.serve_source(c) for c in range(fc.SERVE_CHANNELS)]
    print(f"serve n={n}: {fc.SERVE_CHANNELS} channels x {fc.SERVE_EXPORTS} exports", flush=True)

    def serve(channels):
        srv = X.Server(n, dump_frames=d, max_channels=len(channels), launch_period_us=2000.0)
        rings = []
        for k, c in enumerate(channels):
            ch = srv.admit(torch.from_numpy(srcs[c]).cuda(), start_s=0.001 * k,
                           total_frames=fc.SERVE_EXPORTS * d)
            ring = torch.full((fc.SERVE_EXPORTS, X.tri(n), 2), -1, dtype=torch.int32, device="cuda")
            srv.export_ring(ch, ring)
            rings.append((ch, ring))
        st = srv.run(0.5)
        print("serve", channels, st, flush=True)
        assert st["frames_done"] == len(channels) * fc.SERVE_EXPORTS * d and st["frames_dropped"] == 0
        for ch, _ in rings:
            info = srv.channel_info(ch)
            assert info["state"] == 2 and info["dumps"] == fc.SERVE_EXPORTS
        out = [ring.cpu() for _, ring in rings]
        srv.close()
        return out

    mix = serve(list(range(fc.SERVE_CHANNELS)))
    for c, ring in enumerate(mix):
        for m in range(fc.SERVE_EXPORTS):
            pu.assert_matches_oracle_digest(f"serve_n2048_c{c}_e{m}", ring[m].numpy(),
                                            fc.serve_window(srcs[c], m))
    solo = serve([0])
    assert torch.equal(solo[0], mix[0])


def slot_mem(X, n):
    """Device bytes of a server slot: accumulators and export buffer."""
    return X.slot_bytes(n) + n * (n + 1) // 2 * 8


def test_channel_waits_until_freed_memory_admits_it(X):
    # two slots, but a budget of two slots and ONE host ring: the second
    # host source waits for memory (not for a slot), is admitted when the
    # first finishes and leaves its ring, and then runs in the freed slot
    # and ring with nothing newly allocated; every export equals the oracle
    ring_frames = 8
    ring = ring_frames * 256 * N
    srcs = [frames_of(seed=[11, c], n_frames=40) for c in range(2)]
    hosts = [torch.from_numpy(f).pin_memory() for f in srcs]
    srv = X.Server(N, dump_frames=DUMP, max_channels=2, ring_frames=ring_frames, launch_period_us=2000.0,
                   mem_budget_bytes=2 * slot_mem(X, N) + ring)
    assert srv.max_channels == 2
    a = srv.admit(hosts[0], total_frames=2 * DUMP)
    b = srv.admit(hosts[1], total_frames=2 * DUMP)
    rings = [torch.zeros((2, X.tri(N), 2), dtype=torch.int32, device="cuda") for _ in range(2)]
    srv.export_ring(a, rings[0])
    srv.export_ring(b, rings[1])
    st = srv.run(0.4)
    print("admission by memory", st, flush=True)
    ia, ib = srv.channel_info(a), srv.channel_info(b)
    print("channels", ia, ib, flush=True)
    assert st["channels_waiting"] == 0 and st["frames_dropped"] == 0 and st["frames_done"] == 4 * DUMP
    assert st["device_bytes"] == slot_mem(X, N) + ring               # one slot, one ring, both reused
    assert ia["state"] == 2 and ib["state"] == 2 and ib["slot"] == ia["slot"]
    # b waited for a's last frame (released at 2 DUMP - 1 frame periods)
    assert ib["admitted_s"] >= (2 * DUMP - 1) * 655.36e-6 > ia["admitted_s"]
    for r, f in zip(rings, srcs):
        for k in range(2):
            np.testing.assert_array_equal(r[k].cpu().numpy(), expected(f, k * DUMP))
    srv.close()


def test_budget_smaller_than_a_ring_never_admits_a_host_source(X):
    # a budget with room for a slot but not for slot + ring: the device
    # channel runs, the host source waits through the whole run
    dev_src, host_src = frames_of(seed=[12, 0]), frames_of(seed=[12, 1])
    srv = X.Server(N, dump_frames=DUMP, max_channels=2, ring_frames=64, launch_period_us=2000.0,
                   mem_budget_bytes=2 * slot_mem(X, N))
    d = srv.admit(torch.from_numpy(dev_src).cuda(), total_frames=DUMP)
    h = srv.admit(torch.from_numpy(host_src).pin_memory(), total_frames=DUMP)
    st = srv.run(0.1)
    assert st["channels_waiting"] == 1 and st["frames_done"] == DUMP
    assert srv.channel_info(h)["state"] == 0 and srv.channel_info(h)["admitted_s"] < 0
    np.testing.assert_array_equal(srv.last_dump(d).cpu().numpy(), expected(dev_src, 0))
    srv.close()
