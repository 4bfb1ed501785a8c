"""Replay a Poisson trace of render requests through the continuous-batching
server, and through a plain one-request-at-a-time render on the same GPU.

Latency is measured from each request's scheduled arrival time on the
serving clock to the moment its completion is observed, so time a request
spends waiting (for the server or for the plain loop) counts.
"""

from __future__ import annotations

import ctypes as C
import sys
import time

import numpy as np
import torch

from . import api, synth


class Pool:
    """Device-resident request inputs: the seeded programs of the mix."""

    def __init__(self, mix: synth.ServeMix, device="cuda"):
        self.mix = mix
        lens = mix.program_lengths()
        self.programs = [api.to_device(synth.make_program(int(lens[j]), 8,
                                                          mix.program_seed0 + j),
                                       device=device)
                         for j in range(mix.n_programs)]
        self.lengths = lens


def _percentiles(lat):
    if not lat:
        return None, None
    a = np.asarray(lat)
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def run_server(pool: Pool, trace, warmup: float, streams=3, max_slots=64,
               output_bytes: int = 1 << 30):
    """Serve the trace; returns latency / throughput statistics. The server
    holds every request's rgb output in its arena, so it admits requests by
    their whole footprint (stroke records and output) within output_bytes
    of room beside the programs and launch buffers; each output is given
    back as soon as its request completes."""
    lib = api.L.load()
    progs = sum(lib.tbr_serve_program_bytes(len(p["cx"]), 8) for p in pool.programs)
    probe = api.L.ServeOpts(None, 0, max_slots, 1 << 16, 1 << 17, streams, 0, 0.0, 0)
    ticks = streams * lib.tbr_serve_tick_bytes(C.byref(probe))
    srv = api.Server(arena_bytes=progs + ticks + output_bytes, max_slots=max_slots,
                     max_queue=1 << 16, max_tick_items=1 << 17, streams=streams)
    pids = [srv.register(p) for p in pool.programs]
    torch.cuda.synchronize()
    t0 = srv.now() + 0.05
    pending = {}       # ticket -> request index
    lat, ps, t_last, done = [], 0, t0, 0
    j = 0
    while j < len(trace) or pending:
        now = srv.now()
        while j < len(trace) and trace[j].t_arrival + t0 <= now:
            rq = trace[j]
            t = srv.submit(pids[rq.program], "soft" if rq.soft else "hard", rq.width, rq.width,
                           tau_c=0.0, arena_outputs=("rgb",))
            pending[t] = j
            j += 1
        progressed = False
        for t in list(pending):
            r = srv.poll(t)
            if r is None:
                continue
            progressed = True
            srv.release(t)  # the output is not read here
            idx = pending.pop(t)
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
