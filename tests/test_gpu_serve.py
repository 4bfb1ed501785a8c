"""GPU checks of the continuous-batching server: every request's result is
bitwise the same whether it runs alone (tbr_render) or packed with others of
different programs, modes and resolutions; a short Poisson replay completes
every request."""

import numpy as np
import pytest
import torch

from gpu_util import log, require_gpu
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
    pool = serve_driver.Pool(mix, n_buffers=24)
    r = serve_driver.run_server(pool, trace, warmup=0.0)
    log(f"[serve] {r}")
    assert r["requests"] == len(trace)
    assert r["p99_ms"] >= r["p50_ms"] > 0
