"""Simulated light-field cameras feeding the serving loop (pcbz_server_*).

Each camera sends frames at Poisson arrival times.  Frame sizes are drawn
uniformly from 1020 x 1020, 2040 x 2040 and 2040 x 1020 (H x W); even
cameras film beads, odd cameras vessels.  Frames come from pre-rendered
time sequences (one per content, 2040 x 2040, the smaller sizes as top-left
crops) so that rendering stays off the clock; a camera's k-th frame of a
given size is step k of its sequence, so consecutive frames of one camera
and size are consecutive time steps and the temporal candidate applies.

Latency is measured from the scheduled arrival time to the moment the
container is in host memory (server clock = CLOCK_MONOTONIC, like
time.monotonic()).

    python -m paper_2310_09467_amd.cameras --seconds 60 --report serve.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

from . import pcbz, synth

SIZES = ((1020, 1020), (2040, 2040), (2040, 1020))
PITCH, LEVEL = 15, 9
_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_SELECTOR = os.path.join(_HERE, "weights", "selector_lfm.bin")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def arrivals(rate, seconds, seed):
    """Poisson arrival times in [0, seconds) (exponential gaps, numpy PCG64)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            return np.array(out)
        out.append(t)


def schedule(n_cameras, rate, seconds, seed0=100):
    """Merged (time, camera, size index) list in time order; camera c uses seeds
    seed0 + c for its arrivals and sizes."""
    ev = []
    for c in range(n_cameras):
        ts = arrivals(rate, seconds, seed0 + c)
        sizes = np.random.default_rng(10_000 + seed0 + c).integers(0, len(SIZES), len(ts))
        ev += [(float(t), c, int(s)) for t, s in zip(ts, sizes)]
    ev.sort()
    return ev


def render_sequences(steps=8, seed=5):
    """{"beads": [2040x2040 frames], "vessels": [...]}: time sequences."""
    rng = np.random.default_rng(seed)
    _, pos = synth.beads_frame(2040, 2040, 2000, 100.0, seed=seed)
    beads = []
    for k in range(steps):
        f, _ = synth.beads_frame(2040, 2040, 2000, 100.0, seed=seed * 1000 + k, positions=pos)
        beads.append(f)
        pos = pos.copy()
        pos[:, :2] += rng.normal(0.0, 0.05, size=(len(pos), 2))
    scene = synth.VesselScene(seed=seed)
    vessels = [scene.frame(k) for k in range(steps)]
    return {"beads": beads, "vessels": vessels}


def pools(seqs):
    """Pinned host copies: {(content, size index): [frames]}."""
    import torch

    out = {}
    for content, frames in seqs.items():
        for si, (h, w) in enumerate(SIZES):
            lst = []
            for f in frames:
                t = torch.empty((h, w), dtype=torch.int16, pin_memory=True)
                t.copy_(torch.from_numpy(np.ascontiguousarray(f[:h, :w]).view(np.int16)))
                lst.append(t)
            out[(content, si)] = lst
    return out


def content_of(camera):
    return "beads" if camera % 2 == 0 else "vessels"


def run(server, pool, events, temporal=True, on_progress=None, tag0=0):
    """Feeds `events` in real time (tags tag0, tag0 + 1, ...) and collects
    every result.  Returns (results by tag, frame source by tag, t0 on the
    monotonic clock)."""
    counters = {}
    src = {}
    jobs = []
    for tag, (t, cam, si) in enumerate(events, start=tag0):
        key = (cam, si)
        k = counters.get(key, 0)
        counters[key] = k + 1
        frames = pool[(content_of(cam), si)]
        src[tag] = (content_of(cam), si, k % len(frames))
        jobs.append((t, cam, si, frames[k % len(frames)]))
    results = {}
    t0 = time.monotonic() + 0.2
    mask = 0xF if temporal else 0x7
    err = []

    def feed():
        try:
            for tag, (t, cam, si, frame) in enumerate(jobs, start=tag0):
                d = t0 + t - time.monotonic()
                if d > 0:
                    time.sleep(d)
                server.submit(frame, tag, cam, PITCH, LEVEL, mask)
        except Exception as e:  # reported by the caller
            err.append(e)

    th = threading.Thread(target=feed, daemon=True)
    th.start()
    last = time.monotonic()
    while len(results) < len(jobs) and not (err and not th.is_alive()):
        for r in server.poll(256, 50):
            results[r["tag"]] = r
        if on_progress and time.monotonic() - last > 5.0:
            last = time.monotonic()
            on_progress(len(results), len(jobs))
    th.join()
    if err:
        raise err[0]
    return results, src, t0


def summarize(results, events, src, pool, t0):
    lat, raw, comp = [], 0, 0
    done_last = 0.0
    for tag, r in results.items():
        if r["status"] != 0:
            raise RuntimeError(f"frame {tag} failed with status {r['status']}")
        t_arr, cam, si = events[tag]  # tags of the run start at 0
        done = r["submit_ms"] / 1e3 + r["latency_ms"] / 1e3
        lat.append((done - (t0 + t_arr)) * 1e3)
        h, w = SIZES[si]
        raw += 2 * h * w
        comp += len(r["data"])
        done_last = max(done_last, done)
    lat = np.array(lat)
    span = done_last - t0
    return {"frames": len(results), "raw_bytes": raw, "container_bytes": comp, "ratio": raw / comp,
            "wall_s": span, "throughput_mb_s": raw / span / 1e6,
            "offered_mb_s": raw / max(events[-1][0], 1e-9) / 1e6,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())}}


def verify(results, src, pool, seqs, n_check=None, selector=None, min_conf=1.01):
    """Compares served containers with the same frame compressed alone (same
    previous frame and selector).  Served frames repeat (pool entries), so
    each distinct (frame, previous frame) is compressed once and every result
    that shares it is compared; n_check (None: all) limits the results
    compared.  Also returns the size regret of the compared frames against
    judging every band."""
    ctx = pcbz.Context(0)
    tags = sorted(results) if n_check is None else sorted(results)[:n_check]
    alone, exhaustive = {}, {}
    ok, served, exh = 0, 0, 0
    for tag in tags:
        r = results[tag]
        psrc = None if r["prev_tag"] is None else src[r["prev_tag"]]
        key = (src[tag], psrc)
        if key not in alone:
            content, si, k = src[tag]
            h, w = SIZES[si]
            frame = np.ascontiguousarray(seqs[content][k][:h, :w])
            prev = None if psrc is None else np.ascontiguousarray(seqs[psrc[0]][psrc[2]][:h, :w])
            mask = 0xF if prev is not None else 0x7
            ctx.set_selector(selector, min_conf) if selector is not None else ctx.set_selector(None)
            alone[key] = ctx.compress(frame, prev, PITCH, LEVEL, mask)
            ctx.set_selector(None)
            exhaustive[key] = len(ctx.compress(frame, prev, PITCH, LEVEL, mask)) if selector is not None \
                else len(alone[key])
        ok += alone[key] == r["data"]
        served += len(r["data"])
        exh += exhaustive[key]
    ctx.close()
    return {"checked": len(tags), "equal_alone": ok, "distinct": len(alone), "regret": served / max(exh, 1) - 1.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cameras", type=int, default=4)
    ap.add_argument("--rate", type=float, default=50.0, help="frames per second per camera")
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--workers", type=int, default=2)
    ap.add_argument("--selector", default=DEFAULT_SELECTOR, help="selector file, or 'none'")
    ap.add_argument("--min-conf", type=float, default=0.9)
    ap.add_argument("--no-temporal", action="store_true")
    ap.add_argument("--verify", type=int, default=-1,
                    help="results compared with their frame compressed alone (-1: all, 0: none)")
    ap.add_argument("--report", default=None)
    args = ap.parse_args()

    log("rendering sequences")
    seqs = render_sequences()
    pool = pools(seqs)
    events = schedule(args.cameras, args.rate, args.seconds)
    log(f"{len(events)} arrivals over {args.seconds} s")
    ctx = pcbz.Context(0)
    sel = None
    if args.selector and args.selector != "none":
        sel = pcbz.Selector.load_file(ctx, args.selector)
    srv = pcbz.Server(0, int(args.budget_gb * (1 << 30)), args.workers, 0, sel, args.min_conf)
    # warm-up: one frame of each size and content through the server, from
    # cameras that take no part in the run (their state stays separate)
    warm = [(0.0, 1000 + c, s) for c in range(2) for s in range(len(SIZES))]
    run(srv, pool, warm, temporal=False, tag0=1 << 40)
    res, src, t0 = run(srv, pool, events, not args.no_temporal,
                       on_progress=lambda a, b: log(f"  {a}/{b} frames done"))
    rep = summarize(res, events, src, pool, t0)
    rep["server"] = srv.stats()
    rep["server"]["mean_batch"] = rep["server"]["batched_frames"] / max(rep["server"]["batches"], 1)
    srv.close()
    rep["config"] = {"cameras": args.cameras, "rate_per_camera": args.rate, "seconds": args.seconds,
                     "budget_gb": args.budget_gb, "workers": args.workers,
                     "selector": None if sel is None else os.path.basename(args.selector),
                     "min_conf": args.min_conf, "temporal": not args.no_temporal}
    if args.verify:
        rep["verify"] = verify(res, src, pool, seqs, None if args.verify < 0 else args.verify, sel, args.min_conf)
    out = json.dumps(rep, indent=1)
    if args.report:
        with open(args.report, "w") as fh:
            fh.write(out + "\n")
    print(out, flush=True)


if __name__ == "__main__":
    main()
