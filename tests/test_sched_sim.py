"""The streaming server's scheduling core (csrc/xeng_sched.cpp) on a simulated
device and clock (tests/sched_sim.cpp), on the CPU: exact frame accounting
for every export, ring safety for host sources, drops, staggered export
phases, admission into freed slots and by memory (the server's budget and
the device's free memory at admission time), the in-flight limit and the
statistics.

The core is the same code the HIP server runs; here its Executor is a model
with serial copy and compute queues, so every run is deterministic."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sim_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("sched") / "libsched_sim.so")
    cmd = ["g++", "-std=c++17", "-O1", "-shared", "-fPIC", "-Wall",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2005_09481_amd", "csrc"),
           os.path.join(ROOT, "tests", "sched_sim.cpp"),
           os.path.join(ROOT, "paper_2005_09481_amd", "csrc", "xeng_sched.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    L = ctypes.CDLL(out)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.sim_create.restype = vp
    L.sim_create.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.sim_destroy.argtypes = [vp]
    L.sim_set_free.argtypes = [vp, i64, dbl, i64]
    L.sim_admit.restype = i32
    L.sim_admit.argtypes = [vp, i64, i32, dbl, i64]
    L.sim_run.restype = ctypes.c_int
    L.sim_run.argtypes = [vp, dbl, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    L.sim_log_size.restype = i64
    L.sim_log_size.argtypes = [vp, ctypes.c_int]
    L.sim_log_copy.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64)]
    L.sim_chan.argtypes = [vp, i32, ctypes.POINTER(i64)]
    return L


class Sim:
    def __init__(self, L, dump=16, ring=8, inflight=2, slots=4, stagger=False, frame_us=655.36,
                 launch_us=2000.0, t_idle=20.0, t_copy=50.0, t_launch=100.0, t_frame=5.0, t_export=10.0,
                 slot_bytes=0, ring_bytes=0, budget=0, reserve=0):
        self.L = L
        self.dump, self.ring, self.slots, self.stagger = dump, ring, slots, stagger
        cfg = (ctypes.c_int64 * 10)(256, dump, ring, inflight, slots, int(stagger), slot_bytes, ring_bytes,
                                    budget, reserve)
        per = (ctypes.c_double * 2)(frame_us, launch_us)
        tm = (ctypes.c_double * 5)(t_idle, t_copy, t_launch, t_frame, t_export)
        self.h = L.sim_create(cfg, per, tm)
        self.host = []

    def admit(self, src_frames=64, host=False, start_s=0.0, total=0):
        self.host.append(host)
        return self.L.sim_admit(self.h, src_frames, int(host), start_s, total)

    def set_free(self, before, t_switch, after):
        self.L.sim_set_free(self.h, before, t_switch, after)

    def run(self, seconds):
        ist = (ctypes.c_int64 * 10)()
        dst = (ctypes.c_double * 4)()
        rc = self.L.sim_run(self.h, seconds, ist, dst)
        assert rc == 0
        keys = ["released", "done", "dropped", "launches", "dumps", "backlog", "violations", "resets",
                "waiting", "device_bytes"]
        st = dict(zip(keys, list(ist)))
        st.update(zip(["seconds", "p50_ms", "p99_ms", "max_ms"], list(dst)))
        return st

    def log(self, which):
        n = self.L.sim_log_size(self.h, which)
        buf = (ctypes.c_int64 * max(n, 1))()
        self.L.sim_log_copy(self.h, which, buf)
        return np.array(buf[:n], dtype=np.int64)

    def chan(self, k):
        out = (ctypes.c_int64 * 8)()
        self.L.sim_chan(self.h, k, out)
        return dict(zip(["state", "slot", "released", "done", "dumps", "last_first", "start_ns", "admitted_ns"],
                        list(out)))

    def attaches(self):
        a = self.log(4).reshape(-1, 5)
        return [dict(chan=int(r[0]), slot=int(r[1]), new_slot=bool(r[2]), new_ring=bool(r[3]), t_ns=int(r[4]))
                for r in a]

    def copies(self):
        c = self.log(0).reshape(-1, 2)
        return {k: set(c[c[:, 0] == k, 1].tolist()) for k in range(len(self.host))}

    def integrated(self):
        g = self.log(1).reshape(-1, 3)
        return {k: g[g[:, 1] == k, 2] for k in range(len(self.host))}

    def exports(self):
        e = self.log(2).reshape(-1, 6)
        fr = self.log(3)
        return [dict(chan=int(r[0]), slot=int(r[1]), f0=int(r[2]), f1=int(r[3]),
                     frames=sorted(fr[r[4]:r[4] + r[5]].tolist())) for r in e]

    def close(self):
        self.L.sim_destroy(self.h)


def check_accounting(sim, st):
    """What holds for every run: no violation, each frame integrated at most
    once, every export exactly the integrated frames of its window."""
    assert st["violations"] == 0
    assert st["released"] == st["done"] + st["dropped"] + st["backlog"]
    assert st["backlog"] >= 0
    integ = sim.integrated()
    copies = sim.copies()
    for k, fr in integ.items():
        assert len(fr) == len(set(fr.tolist())), f"channel {k}: a frame integrated twice"
        if sim.host[k]:
            assert set(fr.tolist()) <= copies[k], f"channel {k}: integrated a frame never copied"
    for e in sim.exports():
        done_k = set(integ[e["chan"]].tolist())
        window = set(range(e["f0"], e["f1"]))
        assert set(e["frames"]) == window & done_k, (e["chan"], e["f0"], e["f1"])
    assert sum(len(v) for v in integ.values()) == st["done"]


def test_device_channels_every_frame_once(sim_lib):
    sim = Sim(sim_lib, dump=16, slots=4)
    for c in range(4):
        sim.admit(start_s=0.0001 * c)
    st = sim.run(0.3)
    check_accounting(sim, st)
    assert st["dropped"] == 0 and st["done"] > 0
    for k in range(4):
        ch = sim.chan(k)
        # every released frame integrated (the run waits for queued work)
        assert ch["done"] == ch["released"]
        np.testing.assert_array_equal(np.sort(sim.integrated()[k]), np.arange(ch["done"]))
    ex = sim.exports()
    assert len(ex) == st["dumps"] > 0
    for e in ex:
        # unstaggered: windows [m D, (m + 1) D), complete
        assert e["f1"] % 16 == 0 and e["f0"] == e["f1"] - 16 and len(e["frames"]) == 16
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    sim.close()


def test_staggered_export_phases(sim_lib):
    sim = Sim(sim_lib, dump=16, slots=4, stagger=True)
    for c in range(4):
        sim.admit()
    st = sim.run(0.3)
    check_accounting(sim, st)
    for e in sim.exports():
        phase = e["slot"] * 16 // 4
        assert (e["f1"] + phase) % 16 == 0                 # boundary m D - phase
        assert e["f0"] == max(0, e["f1"] - 16)
        assert len(e["frames"]) == e["f1"] - e["f0"]       # the first window is the short one
    assert {e["slot"] * 4 for e in sim.exports()} == {0, 4, 8, 12}
    sim.close()


def test_host_ring_overflow_drops_are_never_integrated(sim_lib):
    # a 3-frame ring and a launch only every 20 ms: most frames are dropped;
    # the integrated ones are exactly the copied ones, each once, and every
    # export holds its window's copied frames
    sim = Sim(sim_lib, dump=16, ring=3, inflight=1, slots=2, frame_us=200.0, launch_us=20000.0)
    a = sim.admit(src_frames=5, host=True, total=48)
    b = sim.admit(src_frames=7, host=True, total=48, start_s=0.0003)
    st = sim.run(0.5)
    check_accounting(sim, st)
    assert st["dropped"] > 0
    copies = sim.copies()
    for k in (a, b):
        ch = sim.chan(k)
        assert ch["state"] == 2 and ch["released"] == 48 and ch["done"] == 48 and ch["dumps"] == 3
        assert set(sim.integrated()[k].tolist()) == copies[k]
    assert st["dropped"] == 96 - sum(len(v) for v in copies.values())
    assert st["resets"] == 2
    sim.close()


def test_host_ring_without_pressure_drops_nothing(sim_lib):
    sim = Sim(sim_lib, dump=16, ring=16, slots=2, launch_us=1000.0)
    for c in range(2):
        sim.admit(src_frames=5, host=True, total=64, start_s=0.0002 * c)
    st = sim.run(0.2)
    check_accounting(sim, st)
    assert st["dropped"] == 0 and st["done"] == 128 and st["dumps"] == 8
    sim.close()


def test_admission_into_freed_slots(sim_lib):
    # three finite channels, two slots: the third waits, takes the first
    # freed slot, starts its stream then, and its exports hold only its frames
    sim = Sim(sim_lib, dump=8, slots=2)
    c0 = sim.admit(total=16)
    c1 = sim.admit(total=40)
    c2 = sim.admit(total=24)
    assert sim.chan(c2)["state"] == 0 and sim.chan(c2)["slot"] == -1
    st = sim.run(0.3)
    check_accounting(sim, st)
    s0, s2 = sim.chan(c0), sim.chan(c2)
    assert all(sim.chan(k)["state"] == 2 for k in (c0, c1, c2))
    assert s2["slot"] == s0["slot"]                        # the slot c0 freed
    assert s2["start_ns"] > 15 * 655360                    # after c0's last frame (index 15)
    assert [sim.chan(k)["dumps"] for k in (c0, c1, c2)] == [2, 5, 3]
    assert st["resets"] == 3 and st["done"] == 80
    sim.close()


def test_overload_grows_latency_not_errors(sim_lib):
    # integration slower than real time: the backlog and the latency grow,
    # every frame is still accounted for, nothing is integrated twice
    sim = Sim(sim_lib, dump=16, slots=4, t_frame=400.0)
    for c in range(4):
        sim.admit()
    st = sim.run(0.2)
    check_accounting(sim, st)
    fast = Sim(sim_lib, dump=16, slots=4)
    for c in range(4):
        fast.admit()
    st_fast = fast.run(0.2)
    assert st["p99_ms"] > 3 * st_fast["p99_ms"]
    sim.close()
    fast.close()


@pytest.mark.parametrize("inflight", [1, 2, 4])
def test_inflight_limit(sim_lib, inflight):
    # the harness counts a launch issued while max_inflight are unfinished
    sim = Sim(sim_lib, dump=16, slots=3, inflight=inflight, launch_us=0.0, t_launch=3000.0)
    for c in range(3):
        sim.admit()
    st = sim.run(0.1)
    check_accounting(sim, st)
    assert st["launches"] > 3
    sim.close()


def test_host_ring_sustained_overload_interleaves_drops(sim_lib):
    # frames every 100 us into an 8-frame ring, a launch at most every
    # 500 us, integration slower than the frames arrive: copies resume as
    # each launch completes and continue until the next launch is formed, so
    # dropped frames fall between copied ones inside a launch's range; the
    # launch must stop at each gap and pass over it (a launch reading across
    # a gap integrates the ring slot's stale frame, which the harness counts)
    sim = Sim(sim_lib, dump=32, ring=8, inflight=1, slots=1, frame_us=100.0, launch_us=500.0,
              t_launch=50.0, t_frame=80.0, t_copy=20.0)
    sim.admit(src_frames=3, host=True, total=600)
    st = sim.run(0.2)
    check_accounting(sim, st)
    g = sim.integrated()[0]
    copies = sim.copies()[0]
    dropped = set(range(600)) - copies
    # drops strictly inside the span of copied frames, not only at its ends
    assert st["dropped"] == len(dropped) > 0
    assert any(min(copies) < d < max(copies) for d in dropped)
    assert set(g.tolist()) == copies
    assert sim.chan(0)["state"] == 2
    sim.close()


def test_core_under_sanitizers(tmp_path):
    # the scheduling core and the harness built with AddressSanitizer and
    # UndefinedBehaviorSanitizer, every scenario kind run in one process
    exe = str(tmp_path / "sched_sim_asan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2005_09481_amd", "csrc"),
           os.path.join(ROOT, "tests", "sched_sim_main.cpp"), os.path.join(ROOT, "tests", "sched_sim.cpp"),
           os.path.join(ROOT, "paper_2005_09481_amd", "csrc", "xeng_sched.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert r.stdout.count("rc=0") == 4


def test_admission_by_budget_reuses_freed_slot_memory(sim_lib):
    # the budget holds two slots' memory: the third channel waits (a free
    # slot id is there, its memory is not), then takes the slot the first
    # finished channel left, with no new allocation
    sim = Sim(sim_lib, dump=8, slots=4, slot_bytes=1000, budget=2500)
    c0 = sim.admit(total=16)
    c1 = sim.admit(total=40)
    c2 = sim.admit(total=24)
    st = sim.run(0.3)
    check_accounting(sim, st)
    att = {a["chan"]: a for a in sim.attaches()}
    assert att[c0]["new_slot"] and att[c1]["new_slot"] and not att[c2]["new_slot"]
    assert att[c2]["slot"] == att[c0]["slot"]
    assert sim.chan(c2)["admitted_ns"] > 15 * 655360          # after c0's last frame
    assert st["device_bytes"] == 2000 and st["waiting"] == 0
    assert [sim.chan(k)["dumps"] for k in (c0, c1, c2)] == [2, 5, 3]
    sim.close()


def test_admission_waits_for_free_device_memory(sim_lib):
    # the device has too little free memory (less the reserve) until 50 ms
    # into the run: both channels wait, then both are admitted and stream
    sim = Sim(sim_lib, dump=8, slots=4, slot_bytes=1000, reserve=500)
    sim.set_free(1200, 0.05, 10_000)
    a = sim.admit(total=16)
    b = sim.admit(total=16)
    st = sim.run(0.2)
    check_accounting(sim, st)
    for k in (a, b):
        ch = sim.chan(k)
        assert ch["admitted_ns"] >= 50_000_000 and ch["start_ns"] >= 50_000_000
        assert ch["state"] == 2 and ch["done"] == 16 and ch["dumps"] == 2
    sim.close()


def test_admission_stays_waiting_without_memory(sim_lib):
    sim = Sim(sim_lib, dump=8, slots=4, slot_bytes=1000, reserve=500)
    sim.set_free(1200, 10.0, 1200)
    a = sim.admit(total=16)
    st = sim.run(0.05)
    assert st["waiting"] == 1 and st["done"] == 0 and st["device_bytes"] == 0
    assert sim.chan(a)["state"] == 0 and sim.chan(a)["slot"] == -1 and sim.attaches() == []
    sim.close()


def test_host_rings_are_kept_for_the_next_host_channel(sim_lib):
    # budget: two slots and one ring; the second host channel waits for the
    # first's ring (not for a slot), then reuses ring and slot memory
    sim = Sim(sim_lib, dump=8, ring=8, slots=2, slot_bytes=1000, ring_bytes=300, budget=2300)
    a = sim.admit(src_frames=5, host=True, total=16)
    b = sim.admit(src_frames=7, host=True, total=16, start_s=0.0002)
    st = sim.run(0.3)
    check_accounting(sim, st)
    att = {x["chan"]: x for x in sim.attaches()}
    assert att[a]["new_slot"] and att[a]["new_ring"]
    assert not att[b]["new_ring"] and not att[b]["new_slot"]
    assert sim.chan(b)["admitted_ns"] > 15 * 655360
    assert st["device_bytes"] == 1300 and st["dropped"] == 0 and st["done"] == 32
    sim.close()


def test_waiting_channels_are_admitted_in_order(sim_lib):
    # a host channel that needs a ring the budget lacks holds back the
    # device channel behind it (no overtaking), until memory frees up
    sim = Sim(sim_lib, dump=8, ring=8, slots=3, slot_bytes=1000, ring_bytes=300, budget=2300)
    d0 = sim.admit(total=16)
    h1 = sim.admit(src_frames=5, host=True, total=16)      # slot + ring: 2300 with d0's slot
    h2 = sim.admit(src_frames=5, host=True, total=16)      # needs a second ring: waits
    d3 = sim.admit(total=16)                               # would fit (a free slot with memory later)
    st = sim.run(0.4)
    check_accounting(sim, st)
    order = [x["chan"] for x in sim.attaches()]
    assert order == [d0, h1, h2, d3]
    assert sim.chan(h2)["admitted_ns"] <= sim.chan(d3)["admitted_ns"]
    assert all(sim.chan(k)["state"] == 2 for k in (d0, h1, h2, d3))
    sim.close()
