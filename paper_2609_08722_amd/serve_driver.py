"""Replay a Poisson trace of render requests through the continuous-batching
server, and through a plain one-request-at-a-time render on the same GPU.

Latency is measured from each request's scheduled arrival time on the
serving clock to the moment its completion is observed, so time a request
spends waiting (for the server or for the plain loop) counts.
"""

from __future__ import annotations

import sys
import time

import numpy as np
import torch

from . import api, synth


class Pool:
    """Device-resident request inputs: seeded programs and output buffers."""

    def __init__(self, mix: synth.ServeMix, n_buffers: int = 48, device="cuda"):
        self.mix = mix
        lens = mix.program_lengths()
        self.programs = [api.to_device(synth.make_program(int(lens[j]), 8,
                                                          mix.program_seed0 + j),
                                       device=device)
                         for j in range(mix.n_programs)]
        self.lengths = lens
        self.free = {}
        self.bufs = {}
        for res in mix.resolutions:
            self.bufs[res] = [torch.empty((res, res, 3), dtype=torch.float32, device=device)
                              for _ in range(n_buffers)]
            self.free[res] = list(range(n_buffers))


def _percentiles(lat):
    if not lat:
        return None, None
    a = np.asarray(lat)
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def run_server(pool: Pool, trace, warmup: float, streams=3, max_slots=64):
    """Serve the trace; returns latency / throughput statistics."""
    arena = sum(api.L.load().tbr_serve_program_bytes(len(p["cx"]), 8) for p in pool.programs)
    srv = api.Server(arena_bytes=arena + (96 << 20), max_slots=max_slots, max_queue=1 << 16,
                     max_tick_items=1 << 17, streams=streams)
    pids = [srv.register(p) for p in pool.programs]
    torch.cuda.synchronize()
    t0 = srv.now() + 0.05
    pending = {}       # ticket -> (request index, resolution, buffer)
    waiting = list(range(len(trace)))
    lat, ps, t_last, done = [], 0, t0, 0
    j = 0
    while j < len(waiting) or pending:
        now = srv.now()
        while j < len(waiting) and trace[waiting[j]].t_arrival + t0 <= now:
            rq = trace[waiting[j]]
            if not pool.free[rq.width]:
                break  # all output buffers of this size are busy: the request waits
            b = pool.free[rq.width].pop()
            t = srv.submit(pids[rq.program], "soft" if rq.soft else "hard", rq.width, rq.width,
                           rgb=pool.bufs[rq.width][b], tau_c=0.0)
            pending[t] = (waiting[j], rq.width, b)
            j += 1
        progressed = False
        for t in list(pending):
            r = srv.poll(t)
            if r is None:
                continue
            progressed = True
            idx, res, b = pending.pop(t)
            pool.free[res].append(b)
            rq = trace[idx]
            if rq.t_arrival >= warmup:
                lat.append(r["t_done"] - (rq.t_arrival + t0))
                ps += r["pixel_strokes"]
                t_last = max(t_last, r["t_done"])
                done += 1
        if not progressed:
            time.sleep(0.0002)
    stats = srv.stats()
    srv.close()
    p50, p99 = _percentiles(lat)
    window = t_last - (t0 + warmup)
    return {"requests": done, "p50_ms": p50 * 1e3, "p99_ms": p99 * 1e3,
            "mean_ms": float(np.mean(lat)) * 1e3,
            "pixel_strokes_per_s": ps / window if window > 0 else None,
            "launches": stats["launches"]}


def run_plain(pool: Pool, trace, warmup: float, deadline: float):
    """One request at a time, in arrival order, one render launch each."""
    stream = torch.cuda.current_stream()
    clock = api.Server.now
    t0 = clock() + 0.05
    lat, ps, t_last, done, dropped = [], 0, t0, 0, 0
    for rq in trace:
        now = clock()
        if now - t0 > deadline:
            dropped += 1
            continue
        if rq.t_arrival + t0 > now:
            time.sleep(rq.t_arrival + t0 - now)
        p = pool.programs[rq.program]
        out = api.render(p, api.Opts(rq.width, rq.width, tau_c=0.0),
                         "soft" if rq.soft else "hard")
        stream.synchronize()
        t_done = clock()
        del out
        if rq.t_arrival >= warmup:
            lat.append(t_done - (rq.t_arrival + t0))
            ps += rq.width * rq.width * len(p["cx"])
            t_last = t_done
            done += 1
    p50, p99 = _percentiles(lat)
    window = t_last - (t0 + warmup)
    return {"requests": done, "dropped_after_deadline": dropped, "p50_ms": p50 * 1e3,
            "p99_ms": p99 * 1e3, "mean_ms": float(np.mean(lat)) * 1e3,
            "pixel_strokes_per_s": ps / window if window > 0 else None}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def serving_benchmark(duration=8.0, warmup=1.0, rate=200.0, plain=True):
    mix = synth.ServeMix(rate=rate)
    trace = mix.trace(duration)
    pool = Pool(mix)
    offered = sum(r.width * r.width * int(pool.lengths[r.program]) for r in trace) / duration
    _log(f"[serve] {len(trace)} requests over {duration:g} s at {rate:g} req/s: server ...")
    out = {"workload": f"Poisson {rate:g} req/s, {duration:g} s ({len(trace)} requests, "
                       f"first {warmup:g} s warm-up), programs of 200-4000 strokes "
                       f"(log-uniform), hard/soft 50/50, 256^2-2048^2",
           "offered_pixel_strokes_per_s": offered,
           "server": run_server(pool, trace, warmup)}
    if plain:
        _log("[serve] one request at a time ...")
        out["plain_one_at_a_time"] = run_plain(pool, trace, warmup, deadline=2.0 * duration)
    return out
