"""Host-only checks of the serving scheduler (fake executor: no GPU work):
FIFO admission by slots and by the arena bytes of a request's whole
footprint (stroke records and server-held outputs), queue capacity,
cancellation, a launch that fails on the device, and that every request
completes exactly once."""

import ctypes as C
import time

import pytest

from paper_2609_08722_amd import _lib as L
from paper_2609_08722_amd import api, synth


def wait_all(srv, tickets, timeout=10.0):
    done, t0 = {}, time.time()
    while len(done) < len(tickets) and time.time() - t0 < timeout:
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        time.sleep(0.001)
    return done


def test_requests_complete_in_fifo_admission_order():
    srv = api.Server(arena_bytes=64 << 20, max_slots=4, fake_device=True,
                     fake_ns_per_pixel_stroke=2e-3)
    pid = srv.register(synth.make_program(500, 8, 0))
    tickets = [srv.submit(pid, "soft" if j % 2 else "hard", 256, 256) for j in range(20)]
    done = wait_all(srv, tickets)
    assert len(done) == 20 and all(r["status"] == L.TBR_OK for r in done.values())
    admits = [done[t]["t_admit"] for t in tickets]
    assert admits == sorted(admits)  # FIFO admission
    for r in done.values():
        assert r["t_submit"] <= r["t_admit"] <= r["t_start"] <= r["t_done"]
        assert r["pixel_strokes"] == 256 * 256 * 500
    st = srv.stats()
    assert st["completed"] == 20 and st["in_flight"] == 0 and st["queued"] == 0
    with pytest.raises(L.TbrError):
        srv.poll(tickets[0])
    srv.close()


def test_admission_limited_by_arena_bytes():
    # arena holds the launch buffers, the program and ~2 requests' records
    n = 4000
    rec = L.load().tbr_serve_request_bytes(n)
    prog_bytes = L.load().tbr_serve_program_bytes(n, 8)
    probe = L.ServeOpts(None, 0, 16, 4096, 8192, 1, 1, 0.0, 0)
    tick = L.load().tbr_serve_tick_bytes(C.byref(probe))
    srv = api.Server(arena_bytes=tick + prog_bytes + 2 * rec + rec // 2, max_slots=16,
                     max_tick_items=8192, streams=1, fake_device=True,
                     fake_ns_per_pixel_stroke=0.1)  # 6.6 ms per request
    pid = srv.register(synth.make_program(n, 8, 1))
    tickets = [srv.submit(pid, "soft", 128, 128) for _ in range(12)]
    peak = 0
    for _ in range(200):
        peak = max(peak, srv.stats()["in_flight"])
        time.sleep(0.0005)
    assert 1 <= peak <= 2  # bounded by arena bytes, not by the 16 slots
    done = wait_all(srv, tickets)
    assert len(done) == 12
    # everything but the program and the launch buffers is released again
    assert srv.stats()["arena_used"] == prog_bytes + tick
    srv.close()


def test_queue_capacity_and_cancel():
    srv = api.Server(arena_bytes=64 << 20, max_slots=1, max_queue=3, streams=1, fake_device=True,
                     fake_ns_per_pixel_stroke=50.0)  # slow: requests stay queued
    pid = srv.register(synth.make_program(1000, 8, 2))
    t0 = srv.submit(pid, "soft", 512, 512)  # admitted and running for ~13 s (modelled)
    time.sleep(0.01)
    queued = [srv.submit(pid, "hard", 64, 64) for _ in range(3)]
    with pytest.raises(L.TbrError) as e:
        srv.submit(pid, "hard", 64, 64)
    assert e.value.status == L.TBR_E_CAPACITY
    assert srv.cancel(queued[1]) == L.TBR_OK
    assert srv.cancel(t0) == L.TBR_PENDING  # already admitted: runs to completion
    r = srv.poll(queued[1])
    assert r["status"] == L.TBR_E_CANCELLED
    assert srv.stats()["cancelled"] == 1
    srv.close()  # destroy with work in flight must not hang


def test_invalid_requests_rejected():
    srv = api.Server(arena_bytes=16 << 20, fake_device=True)
    pid = srv.register(synth.make_program(10, 4, 3))
    for kw in (dict(width=0), dict(height=20000), dict(eps=0.0), dict(tau=-1.0)):
        args = dict(width=64, height=64)
        args.update(kw)
        with pytest.raises(L.TbrError) as e:
            srv.submit(pid, "soft", args.pop("width"), args.pop("height"), **args)
        assert e.value.status == L.TBR_E_INVALID
    with pytest.raises(L.TbrError) as e:
        srv.submit(pid + 100, "soft", 64, 64)
    assert e.value.status == L.TBR_E_NOTFOUND
    with pytest.raises(L.TbrError) as e:  # more tiles than one launch can hold
        srv.submit(pid, "soft", 16384, 16384)
    assert e.value.status == L.TBR_E_NOMEM
    srv.close()


def test_admission_counts_held_outputs_until_release():
    """A request's footprint includes the outputs the server holds for it:
    with room for one 2048^2 request's rgb, the second waits until the first
    is released, not merely until its launch ends."""
    lib = L.load()
    n, W = 300, 2048
    rec = lib.tbr_serve_request_bytes(n)
    out = lib.tbr_serve_output_bytes(W, W, L.TBR_OUT_RGB)
    assert out == W * W * 12
    assert lib.tbr_serve_output_bytes(W, W, L.TBR_OUT_ALL) == W * W * 20
    prog_bytes = lib.tbr_serve_program_bytes(n, 8)
    probe = L.ServeOpts(None, 0, 8, 4096, 1 << 15, 1, 1, 0.0, 0)
    tick = lib.tbr_serve_tick_bytes(C.byref(probe))
    srv = api.Server(arena_bytes=tick + prog_bytes + rec + out + out // 2, max_slots=8,
                     max_tick_items=1 << 15, streams=1, fake_device=True,
                     fake_ns_per_pixel_stroke=1e-4)
    pid = srv.register(synth.make_program(n, 8, 5))
    a = srv.submit(pid, "soft", W, W, arena_outputs=("rgb",))
    b = srv.submit(pid, "soft", W, W, arena_outputs=("rgb",))
    ra = wait_all(srv, [a])[a]
    assert ra["status"] == L.TBR_OK
    time.sleep(0.05)
    st = srv.stats()
    assert st["queued"] == 1 and st["in_flight"] == 0  # b waits for a's held rgb
    assert srv.poll(b) is None
    assert srv.release(a) == L.TBR_OK
    rb = wait_all(srv, [b])[b]
    assert rb["status"] == L.TBR_OK and rb["t_admit"] >= ra["t_done"]
    assert srv.stats()["arena_used"] == tick + prog_bytes + out  # b's rgb is still held
    assert srv.release(b) == L.TBR_OK
    assert srv.stats()["arena_used"] == tick + prog_bytes
    with pytest.raises(L.TbrError) as e:  # a footprint larger than the arena's room
        srv.submit(pid, "hard", W, W, arena_outputs=("rgb", "label", "owner"))
    assert e.value.status == L.TBR_E_NOMEM
    for bad in (dict(arena_outputs=("label",)),):  # a soft request has only rgb
        with pytest.raises(L.TbrError) as e:
            srv.submit(pid, "soft", 64, 64, **bad)
        assert e.value.status == L.TBR_E_INVALID
    srv.close()


def test_failed_launch_reports_a_device_error():
    """Requests of a launch that fails report TBR_E_DEVICE, never TBR_OK,
    and the server accepts no further work."""
    srv = api.Server(arena_bytes=64 << 20, max_slots=2, streams=1, fake_device=True,
                     fake_ns_per_pixel_stroke=1e-3, fake_fail_launch=1)
    pid = srv.register(synth.make_program(200, 8, 6))
    tickets = [srv.submit(pid, "soft", 128, 128) for _ in range(2)]
    t0 = time.time()
    statuses = {}
    while len(statuses) < 2 and time.time() - t0 < 10:
        for t in tickets:
            if t in statuses:
                continue
            try:
                r = srv.poll(t)
                if r is not None:
                    statuses[t] = r["status"]
            except L.TbrError as e:
                statuses[t] = e.status
        time.sleep(0.001)
    assert set(statuses.values()) == {L.TBR_E_DEVICE}
    with pytest.raises(L.TbrError) as e:
        srv.submit(pid, "soft", 64, 64)
    assert e.value.status == L.TBR_E_DEVICE
    assert srv.stats()["completed"] == 0
    srv.close()


def test_large_request_gets_a_launch_of_its_own():
    """Requests of one launch retire together, so a request of at least
    solo_tiles tiles is launched alone: small requests queued before it go
    in one launch, it in the next, and those after it in a third."""
    srv = api.Server(arena_bytes=64 << 20, max_slots=8, streams=1, fake_device=True,
                     fake_ns_per_pixel_stroke=5.0, solo_tiles=1024)
    pid = srv.register(synth.make_program(100, 8, 7))
    first = srv.submit(pid, "soft", 1024, 1024)  # 4096 tiles: the one stream busy for 0.5 s
    time.sleep(0.01)
    small = [srv.submit(pid, "soft", 128, 128) for _ in range(2)]
    big = srv.submit(pid, "hard", 512, 512)      # 1024 tiles
    after = srv.submit(pid, "soft", 64, 64)
    done = wait_all(srv, [first, *small, big, after])
    starts = {t: done[t]["t_start"] for t in done}
    assert starts[small[0]] == starts[small[1]]
    assert starts[first] < starts[small[0]] < starts[big] < starts[after]
    assert srv.stats()["launches"] == 4
    srv.close()
