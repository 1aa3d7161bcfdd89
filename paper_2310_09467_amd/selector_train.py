"""Trains and evaluates the learned arrangement selector on the GPU.

Labels are the arrangement the entropy judgement (paper Sec. 2.1.2, Eq. 1)
picks for each band, computed by the library's own judge kernels; features
come from the library's feature kernel; every forward, backward and AdamW
step runs in the library's matrix-core kernels.  torch only holds device
buffers and does the bookkeeping of the data set (shuffling, gathering
mini-batches, feature statistics).

Data: seeded synthetic bead light fields (the frame model of Sec. 3), coded
at level 9 like the benchmark workload.  Half of the frames are 225 x 225
(15 x 15 lenses, 20 beads, one band), half 2040 x 2040 (136 x 136 lenses,
2000 beads, ten bands); the peak is log-uniform in 20..1000 photons and the
beads' depth slopes lie within 0.1 of a per-frame centre drawn from
[-0.4, 0.4].  Half of the frames have a previous frame (the same beads,
re-exposed, moved by N(0, 0.5^2) lens units in half of those cases), which
enables the temporal candidate (labels are the best of four); the others
have none (best of three) so that the network also sees the prev-less
workload.  Vessel frames (the tube-and-particle model standing in for the
zebrafish data, at 2040 x 2040, 1020 x 1020 and 2040 x 1020) come from twelve
scenes, half of them with the frame one to three steps earlier as previous
frame.  Frames are drawn by worker processes and reduced to features and
labels as they arrive; only the held-out frames are kept.  Held-out bead and
vessel frames use other seeds and another scene.

Evaluation on held-out frames: top-1 agreement with the judgement, and for
each confidence threshold the share of bands still judged and the regret,
the relative growth of the total compressed size against judging every
band.  The threshold picked is the smallest whose regret stays within the
budget (0.5 % by default).

    python -m paper_2310_09467_amd.selector_train --out selector.bin --report report.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import pcbz, synth

H = 2040
PITCH, LEVEL = 15, 9
THRESHOLDS = (0.0, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.98, 0.99, 0.999, 1.01)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


_SCENES = {}


def _scene(seed):
    """Vessel scenes, built once per worker process."""
    if seed not in _SCENES:
        _SCENES.clear()
        _SCENES[seed] = synth.VesselScene(seed=seed)
    return _SCENES[seed]


def draw_frame(job):
    """job = (kind, seed): "small" (225 x 225 beads), "large" (2040 x 2040
    beads) or ("vessel", (scene seed, step)).  Returns (frame, prev or None)."""
    kind, seed = job
    if kind == "vessel":
        sc_seed, step = seed
        rng = np.random.default_rng(sc_seed * 7919 + step)
        shape = synth.SIZE_CLASSES[int(rng.integers(len(synth.SIZE_CLASSES)))]
        sc = _scene(sc_seed)
        frame = sc.frame(step, shape)
        if rng.uniform() < 0.5:
            return frame, None
        return frame, sc.frame(step - int(rng.integers(1, 4)), shape)
    rng = np.random.default_rng(seed)
    h, n = (225, 20) if kind == "small" else (2040, 2000)
    peak = float(np.exp(rng.uniform(np.log(20.0), np.log(1000.0))))
    centre = float(rng.uniform(-0.4, 0.4))
    frame, pos = synth.beads_frame(h, h, n, peak, seed=int(rng.integers(1 << 31)), depth_window=(centre, 0.1))
    if rng.uniform() < 0.5:
        return frame, None
    moved = pos.copy()
    if rng.uniform() < 0.5:
        moved[:, :2] += rng.normal(0.0, 0.5, size=(len(pos), 2))
    prev, _ = synth.beads_frame(h, h, n, peak, seed=int(rng.integers(1 << 31)), positions=moved)
    return frame, prev


def jobs(n_frames, seed0, n_vessel=0, scenes=()):
    """Bead frames alternating small / large, then vessel frames spread over
    the given scene seeds (ordered by scene, so a worker rebuilds few scenes)."""
    out = [("small" if i % 2 == 0 else "large", seed0 + i) for i in range(n_frames)]
    if n_vessel and scenes:
        per = -(-n_vessel // len(scenes))
        for sc in scenes:
            out += [("vessel", (sc, 3 + k)) for k in range(per)]
        out = out[:n_frames + n_vessel]
    return out


class Dataset:
    """Features (device) and judged labels of every band of a set of frames,
    reduced as the worker processes deliver the frames."""

    def __init__(self, ctx, job_list, pool=None, keep_frames=False):
        import torch

        feats, labels, self.frames = [], [], []
        it = pool.imap(draw_frame, job_list, chunksize=2) if pool is not None else map(draw_frame, job_list)
        for i, (frame, prev) in enumerate(it):
            mask = 0xF if prev is not None else 0x7
            feats.append(ctx.features(frame, prev, PITCH, LEVEL, mask))
            labels.append(ctx.judge(frame, prev, PITCH, LEVEL, mask)[0].to(torch.int64))
            if keep_frames:
                self.frames.append((frame, prev, mask))
            if (i + 1) % 100 == 0:
                log(f"  {i + 1}/{len(job_list)} frames")
        self.feat = torch.cat(feats)
        self.label = torch.cat(labels)

    def counts(self):
        return np.bincount(self.label.cpu().numpy(), minlength=4)


def he_params(seed):
    """He-normal weights (fan-in), zero biases, in the library's parameter order."""
    shapes = ((32, 3, 3, 4), (32,), (32, 3, 3, 32), (32,), (32, 3, 3, 32), (32,), (64, 2048), (64,), (4, 64), (4,))
    rng = np.random.default_rng(seed)
    parts = []
    for s in shapes:
        if len(s) == 1:
            parts.append(np.zeros(s))
        else:
            parts.append(rng.normal(0.0, np.sqrt(2.0 / np.prod(s[1:])), size=s))
    theta = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert theta.size == pcbz.selector_num_params()
    return theta


def fit(ctx, data, epochs=30, batch=256, lr=1e-3, weight_decay=1e-4, seed=0):
    """AdamW on class-weighted cross-entropy; returns (selector, loss history)."""
    import torch

    f = data.feat
    mean = f.mean(dim=(0, 1, 2)).cpu().numpy()
    std = f.std(dim=(0, 1, 2)).cpu().numpy() + 1e-3
    norm = np.concatenate([mean, std]).astype(np.float32)
    sel = pcbz.Selector(ctx, he_params(seed), norm)
    cnt = data.counts().astype(np.float64)
    present = cnt > 0
    cw = np.ones(4)
    cw[present] = cnt[present].sum() / (present.sum() * cnt[present])
    cw = np.clip(cw, 0.25, 4.0)
    g = torch.Generator().manual_seed(seed)
    n = f.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(f.device)
        tot = 0.0
        for i in range(0, n, batch):
            idx = perm[i:i + batch]
            tot += sel.train_step(f[idx], data.label[idx], cw, lr, weight_decay) * len(idx)
        hist.append(tot / n)
        if ep % 5 == 0 or ep == epochs - 1:
            log(f"  epoch {ep}: loss {hist[-1]:.4f}")
    return sel, hist, cw


def evaluate(ctx, sel, data, thresholds=THRESHOLDS):
    """Agreement, per-threshold judged share and size regret on `data`."""
    logits = sel.forward(data.feat)
    pred = logits.argmax(dim=1)
    agree = float((pred == data.label).float().mean())
    exhaustive = 0
    for frame, prev, mask in data.frames:
        exhaustive += len(ctx.compress(frame, prev, PITCH, LEVEL, mask))
    rows = []
    try:
        for tau in thresholds:
            ctx.set_selector(sel, tau)
            total, judged, bands = 0, 0, 0
            for frame, prev, mask in data.frames:
                total += len(ctx.compress(frame, prev, PITCH, LEVEL, mask))
                nb, nj = ctx.selector_stats()
                bands += nb
                judged += nj
            rows.append({"min_conf": tau, "judged_frac": judged / max(bands, 1),
                         "regret": total / exhaustive - 1.0, "bytes": total})
    finally:
        ctx.set_selector(None)
    return {"agreement": agree, "exhaustive_bytes": exhaustive, "thresholds": rows}


def pick_threshold(rows, budget):
    ok = [r for r in rows if r["regret"] <= budget]
    return min(ok, key=lambda r: r["min_conf"]) if ok else rows[-1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-frames", type=int, default=4000)
    ap.add_argument("--test-frames", type=int, default=256)
    ap.add_argument("--vessel-frames", type=int, default=1200, help="vessel frames added to the training set")
    ap.add_argument("--test-vessel-frames", type=int, default=96)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--budget", type=float, default=0.005, help="regret budget for the threshold")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=12, help="processes drawing the synthetic frames")
    ap.add_argument("--out", default=None, help="write the trained selector here")
    ap.add_argument("--report", default=None, help="write the evaluation report (JSON) here")
    args = ap.parse_args()

    import multiprocessing as mp

    t0 = time.perf_counter()
    # the workers start before this process touches the GPU
    pool = mp.get_context("spawn").Pool(args.workers) if args.workers > 1 else None
    try:
        ctx = pcbz.Context(0)
        log("held-out sets")
        test_set = Dataset(ctx, jobs(args.test_frames, 20000 + args.seed * 1000000), pool, keep_frames=True)
        test_ves = Dataset(ctx, jobs(0, 0, args.test_vessel_frames, (90 + args.seed,)), pool, keep_frames=True)
        log("training set")
        train_set = Dataset(ctx, jobs(args.train_frames, 10000 + args.seed * 1000000, args.vessel_frames,
                                      tuple(range(60 + 20 * args.seed, 72 + 20 * args.seed))), pool)
    finally:
        if pool is not None:
            pool.close()
            pool.join()
    t1 = time.perf_counter()
    log("labels (train):", train_set.counts().tolist(), "(test):", test_set.counts().tolist())
    sel, hist, cw = fit(ctx, train_set, args.epochs, args.batch, args.lr, seed=args.seed)
    t2 = time.perf_counter()
    log("evaluating")
    ev = evaluate(ctx, sel, test_set)
    ev_v = evaluate(ctx, sel, test_ves)
    train_logits = sel.forward(train_set.feat)
    train_agree = float((train_logits.argmax(dim=1) == train_set.label).float().mean())
    # a threshold must keep both held-out sets within the budget
    worst = [dict(a, regret=max(a["regret"], b["regret"]), judged_frac=max(a["judged_frac"], b["judged_frac"]))
             for a, b in zip(ev["thresholds"], ev_v["thresholds"])]
    pick = pick_threshold(worst, args.budget)
    rep = {
        "train_frames": args.train_frames, "vessel_frames": args.vessel_frames, "test_frames": args.test_frames,
        "test_vessel_frames": args.test_vessel_frames, "test_vessel_bands": int(test_ves.feat.shape[0]),
        "test_vessel_labels": test_ves.counts().tolist(), "test_vessel_agreement": ev_v["agreement"],
        "vessel_thresholds": ev_v["thresholds"],
        "train_bands": int(train_set.feat.shape[0]), "test_bands": int(test_set.feat.shape[0]),
        "train_labels": train_set.counts().tolist(), "test_labels": test_set.counts().tolist(),
        "class_weights": [float(x) for x in cw], "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
        "loss_first": hist[0], "loss_last": hist[-1],
        "train_agreement": train_agree, "test_agreement": ev["agreement"],
        "thresholds": ev["thresholds"], "budget": args.budget, "picked": pick,
        "seconds": {"data": round(t1 - t0, 1), "train": round(t2 - t1, 1)},
    }
    if args.out:
        sel.save(args.out)
    out = json.dumps(rep, indent=1)
    if args.report:
        with open(args.report, "w") as fh:
            fh.write(out + "\n")
    print(out, flush=True)


if __name__ == "__main__":
    main()
