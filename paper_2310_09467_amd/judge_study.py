"""How well the entropy judgement picks the arrangement that really codes
smallest.

The paper chooses, per image, the arrangement with the lowest 2D image
entropy (Sec. 2.1.2, Eq. 1) as a cheap stand-in for coding every candidate,
and lists a better or faster criterion as future work (Sec. 4).  This study
codes every band of every frame once per candidate (forced ids on the GPU),
reads each band's stream length from the container header, and compares the
judged choice with the smallest candidate: agreement, size regret of the
judgement, and how the per-band entropy ranks against the true sizes.

    python -m paper_2310_09467_amd.judge_study --report judge_study.json
"""
from __future__ import annotations

import argparse
import json
import struct
import sys

import numpy as np

from . import pcbz, synth


def band_lengths(blob):
    """Per-band (id, stream bytes) from a PCBZ container header."""
    n_bands = struct.unpack_from("<H", blob, 16)[0]
    out = []
    for b in range(n_bands):
        cid, ln = struct.unpack_from("<BI", blob, 20 + 5 * b)
        out.append((cid, ln))
    return out


def study_frame(ctx, frame, prev, pitch, level, mask):
    """Per band: the judged id, the entropies, and the coded size of each candidate."""
    ids = [c for c in range(4) if (mask >> c) & 1]
    choice, ent, _ = ctx.judge(frame, prev, pitch, level, mask)
    choice = choice.cpu().numpy()
    ent = ent.cpu().numpy()
    nb = len(choice)
    sizes = np.full((nb, 4), -1, np.int64)
    for c in ids:
        blob = ctx.compress(frame, prev, pitch, level, mask, forced=np.full(nb, c, np.uint8))
        for b, (cid, ln) in enumerate(band_lengths(blob)):
            assert cid == c
            sizes[b, c] = ln
    return choice, ent, sizes, ids


def summarize(rows):
    judged = best = 0
    agree = n = 0
    rank_ok = pairs = 0
    for choice, ent, sizes, ids in rows:
        for b in range(len(choice)):
            s = {c: sizes[b, c] for c in ids}
            c_best = min(ids, key=lambda c: (s[c], c))
            judged += s[int(choice[b])]
            best += s[c_best]
            agree += int(choice[b]) == c_best
            n += 1
            for i in ids:
                for j in ids:
                    if i < j and s[i] != s[j]:
                        pairs += 1
                        rank_ok += (ent[b, i] < ent[b, j]) == (s[i] < s[j])
    return {"bands": n, "agreement": agree / max(n, 1), "judge_regret": judged / max(best, 1) - 1.0,
            "judged_bytes": int(judged), "best_bytes": int(best),
            "pairwise_order_agreement": rank_ok / max(pairs, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--vessel-frames", type=int, default=12)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    ctx = pcbz.Context(0)
    sets = {}
    rows = []
    for peak in (20.0, 100.0, 1000.0):
        rows.append(study_frame(ctx, synth.config2_frame(peak), None, 15, 9, 0x7))
    sets["beads_2040_k3"] = summarize(rows)
    print("beads done", file=sys.stderr, flush=True)
    series = synth.vessel_series(args.vessel_frames + 3)
    frames = [f for f, _ in series]
    rows = []
    for i, (f, pi) in enumerate(series):
        if pi is None:
            continue
        rows.append(study_frame(ctx, f, frames[pi], 15, 9, 0xF))
    sets["vessels_k4"] = summarize(rows)
    out = json.dumps(sets, indent=1)
    if args.report:
        with open(args.report, "w") as fh:
            fh.write(out + "\n")
    print(out, flush=True)


if __name__ == "__main__":
    main()
