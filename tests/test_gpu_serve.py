"""GPU checks of the continuous-batching server: every request's result is
bitwise the same whether it runs alone (tbr_render) or packed with others of
different programs, modes and resolutions; a request waits for arena room
for its whole footprint (records and server-held outputs); a short Poisson
replay completes every request."""

import ctypes as C
import time

import numpy as np
import pytest
import torch

from gpu_util import hard_parity, log, require_gpu
from paper_2609_08722_amd import api, serve_driver, synth

pytestmark = pytest.mark.gpu


def test_results_identical_alone_and_in_mix(orc):
    require_gpu()
    rng = np.random.default_rng(7)
    progs = [synth.make_program(int(n), 8, 500 + j) for j, n in enumerate((37, 200, 900, 1500))]
    dps = [api.to_device(p) for p in progs]
    srv = api.Server(arena_bytes=64 << 20, max_slots=8, streams=3)
    pids = [srv.register(p) for p in dps]
    reqs = []
    for q in range(14):
        j = int(rng.integers(0, 4))
        W = int(rng.choice([16, 50, 64, 100, 256]))
        H = int(rng.choice([16, 37, 64, 128]))
        mode = "soft" if q % 2 else "hard"
        rgb = torch.full((H, W, 3), -1.0, device="cuda")
        label = torch.full((H, W), -7, dtype=torch.int32, device="cuda") if mode == "hard" else None
        reqs.append((j, W, H, mode, rgb, label))
    tickets = [srv.submit(pids[j], mode, W, H, rgb=rgb, label=label, tau_c=0.0)
               for j, W, H, mode, rgb, label in reqs]
    pending = set(tickets)
    while pending:
        for t in list(pending):
            if srv.poll(t) is not None:
                pending.discard(t)
    torch.cuda.synchronize()
    stats = srv.stats()
    srv.close()
    log(f"[serve] {len(reqs)} requests in {stats['launches']} launches")
    for (j, W, H, mode, rgb, label) in reqs:
        alone = api.render(dps[j], api.Opts(W, H, tau_c=0.0), mode)
        assert torch.equal(alone["rgb"], rgb), (j, W, H, mode)
        if mode == "hard":
            assert torch.equal(alone["label"], label)
    # and one soft request of the mix against the oracle
    j, W, H, mode, rgb, _ = next(r for r in reqs if r[3] == "soft")
    ref = orc.render(progs[j], W, H, tau_c=0.0, hard=False)["soft"]
    assert np.max(np.abs(rgb.reshape(-1, 3).cpu().numpy() - ref)) <= 1e-4


def test_short_poisson_replay_completes():
    require_gpu()
    mix = synth.ServeMix(rate=200.0, n_programs=16)
    trace = mix.trace(1.5)
    pool = serve_driver.Pool(mix)
    r = serve_driver.run_server(pool, trace, warmup=0.0)
    log(f"[serve] {r}")
    assert r["requests"] == len(trace)
    assert r["p99_ms"] >= r["p50_ms"] > 0


def test_full_size_requests_match_oracle_on_samples(orc):
    """Requests at the serving mix's sizes (up to 2048^2 and 4000 strokes),
    packed by a server configured as the serving benchmark configures it:
    each result is bitwise the standalone render, and 4096 sampled pixels
    per request match the FP64 oracle (soft colours within 1e-4; hard labels
    and owners exactly, outside the 1e-5 boundary band)."""
    require_gpu()
    mix = synth.ServeMix()
    lens = mix.program_lengths()
    picks = [int(np.argmax(lens)), int(np.argmin(lens)), int(np.argsort(lens)[len(lens) // 2])]
    progs = {j: synth.make_program(int(lens[j]), 8, mix.program_seed0 + j) for j in picks}
    dps = {j: api.to_device(p) for j, p in progs.items()}
    arena = sum(api.L.load().tbr_serve_program_bytes(len(p["cx"]), 8) for p in progs.values())
    srv = api.Server(arena_bytes=arena + (96 << 20), max_slots=64, max_queue=1 << 16,
                     max_tick_items=1 << 17, streams=3)
    pids = {j: srv.register(dps[j]) for j in picks}
    reqs = [(picks[0], 2048, "soft"), (picks[0], 2048, "hard"), (picks[1], 256, "soft"),
            (picks[2], 1024, "hard"), (picks[2], 512, "soft"), (picks[1], 2048, "hard")]
    outs = []
    for j, W, mode in reqs:
        rgb = torch.full((W, W, 3), -1.0, device="cuda")
        label = torch.full((W, W), -7, dtype=torch.int32, device="cuda") if mode == "hard" else None
        owner = torch.full((W, W), -7, dtype=torch.int32, device="cuda") if mode == "hard" else None
        outs.append((rgb, label, owner))
    tickets = [srv.submit(pids[j], mode, W, W, rgb=o[0], label=o[1], owner=o[2], tau_c=0.0)
               for (j, W, mode), o in zip(reqs, outs)]
    pending = set(tickets)
    while pending:
        for t in list(pending):
            if srv.poll(t) is not None:
                pending.discard(t)
    torch.cuda.synchronize()
    srv.close()
    for q, ((j, W, mode), (rgb, label, owner)) in enumerate(zip(reqs, outs)):
        alone = api.render(dps[j], api.Opts(W, W, tau_c=0.0), mode)
        assert torch.equal(alone["rgb"], rgb), (j, W, mode)
        pix = synth.sample_pixels(W * W, 4096, 300 + q)
        ipix = torch.from_numpy(pix).cuda()
        ref = orc.render(progs[j], W, W, tau_c=0.0, pixels=pix)
        if mode == "soft":
            err = float(np.abs(rgb.reshape(-1, 3)[ipix].cpu().numpy() - ref["soft"]).max())
            log(f"[serve {W}^2 x {lens[j]} soft] max err {err:.2e}")
            assert err <= 1e-4
        else:
            assert torch.equal(alone["label"], label) and torch.equal(alone["owner"], owner)
            exempt, bad = hard_parity(owner.reshape(-1)[ipix].cpu().numpy(),
                                      label.reshape(-1)[ipix].cpu().numpy(), ref)
            log(f"[serve {W}^2 x {lens[j]} hard] exempt {exempt}, mismatches {bad}")
            assert bad == 0


def test_tick_graph_replays_match_eager_renders():
    """One stream, so every tick replays the same captured graph with new
    parameters: six rounds of requests, each waited for, with eager renders
    and synchronisations in between; every result must equal the eager
    render bitwise."""
    require_gpu()
    rng = np.random.default_rng(11)
    progs = [synth.make_program(int(n), 8, 700 + j) for j, n in enumerate((120, 640, 1500))]
    dps = [api.to_device(p) for p in progs]
    srv = api.Server(arena_bytes=64 << 20, max_slots=4, streams=1)
    pids = [srv.register(p) for p in dps]
    for rnd in range(6):
        reqs = []
        for q in range(int(rng.integers(1, 4))):
            j = int(rng.integers(0, 3))
            W = int(rng.choice([32, 80, 128, 200]))
            mode = "soft" if rng.random() < 0.5 else "hard"
            rgb = torch.full((W, W, 3), -1.0, device="cuda")
            reqs.append((j, W, mode, rgb, srv.submit(pids[j], mode, W, W, rgb=rgb, tau_c=0.0)))
        pending = {t for *_, t in reqs}
        while pending:
            for t in list(pending):
                if srv.poll(t) is not None:
                    pending.discard(t)
        # eager work between replays
        api.render(dps[rnd % 3], api.Opts(48, 48, tau_c=0.0), "soft")
        torch.cuda.synchronize()
        for j, W, mode, rgb, _ in reqs:
            alone = api.render(dps[j], api.Opts(W, W, tau_c=0.0), mode)
            assert torch.equal(alone["rgb"], rgb), (rnd, j, W, mode)
    stats = srv.stats()
    srv.close()
    log(f"[serve] graph replays: {stats['launches']} ticks on one stream")
    assert stats["launches"] >= 6


def test_request_waits_for_arena_room_then_matches_render():
    """The arena holds one 2048^2 request's footprint (stroke records and
    the server-held rgb, label and owner) and not two: the second request
    waits until the first one's outputs are released, then both results
    equal tbr_render bitwise."""
    require_gpu()
    lib = api.L.load()
    mix = synth.ServeMix()
    lens = mix.program_lengths()
    j = int(np.argmax(lens))
    prog = synth.make_program(int(lens[j]), 8, mix.program_seed0 + j)
    dp = api.to_device(prog)
    W, n = 2048, int(lens[j])
    names = ("rgb", "label", "owner")
    foot = lib.tbr_serve_request_bytes(n) + lib.tbr_serve_output_bytes(W, W, api.L.TBR_OUT_ALL)
    opts = api.L.ServeOpts(None, 0, 8, 1 << 16, 1 << 15, 2, 0, 0.0, 0)
    tick = lib.tbr_serve_tick_bytes(C.byref(opts))
    arena = 2 * tick + lib.tbr_serve_program_bytes(n, 8) + foot + foot // 2
    srv = api.Server(arena_bytes=arena, max_slots=8, max_queue=1 << 16, max_tick_items=1 << 15,
                     streams=2)
    pid = srv.register(dp)
    a = srv.submit(pid, "hard", W, W, tau_c=0.0, arena_outputs=names)
    b = srv.submit(pid, "hard", W, W, tau_c=0.0, arena_outputs=names)
    ra = None
    while ra is None:
        ra = srv.poll(a)
    torch.cuda.synchronize()
    got_a = {k: ra[k].clone() for k in names}
    torch.cuda.synchronize()
    time.sleep(0.05)
    st = srv.stats()
    waited = st["queued"] == 1 and srv.poll(b) is None
    assert srv.release(a) == api.L.TBR_OK
    rb = None
    while rb is None:
        rb = srv.poll(b)
    torch.cuda.synchronize()
    got_b = {k: rb[k].clone() for k in names}
    torch.cuda.synchronize()
    assert srv.release(b) == api.L.TBR_OK
    stats = srv.stats()
    srv.close()
    log(f"[serve arena room] footprint {foot / 2**20:.1f} MiB, arena {arena / 2**20:.1f} MiB; "
        f"second request waited: {waited}; admitted {rb['t_admit'] - ra['t_done']:.4f} s "
        f"after the first finished")
    assert waited and rb["t_admit"] >= ra["t_done"]
    assert stats["arena_used"] == 2 * tick + lib.tbr_serve_program_bytes(n, 8)
    alone = api.render(dp, api.Opts(W, W, tau_c=0.0), "hard")
    for got in (got_a, got_b):
        for k in names:
            assert torch.equal(alone[k], got[k]), k
