"""How well the entropy judgement picks the arrangement that really codes
smallest, and how cheaper criteria would do.

The paper chooses, per image, the arrangement with the lowest 2D image
entropy (Sec. 2.1.2, Eq. 1) as a cheap stand-in for coding every candidate,
and lists a better or faster criterion as future work (Sec. 4).  This study
codes every band of every frame once per candidate (forced ids on the GPU),
reads each band's stream length from the container header, and compares the
judged choice with the smallest candidate: agreement, size regret of the
judgement, and how the per-band entropy ranks against the true sizes.  The
same is scored for two cheaper criteria computed from each candidate's band
bytes (read back from a GPU decompression of the forced container):
  order0  the entropy of the bytes themselves (no rotation sort);
  pairs   the entropy of adjacent byte pairs of the bytes as they stand
          (Eq. 1 without the first-byte rotation sort).

    python -m paper_2310_09467_amd.judge_study --report judge_study.json
"""
from __future__ import annotations

import argparse
import json
import struct
import sys

import numpy as np

from . import pcbz, synth
from .pcbz import NCAND


def band_lengths(blob):
    """Per-band (id, stream bytes) from a PCBZ container header."""
    n_bands = struct.unpack_from("<H", blob, 16)[0]
    out = []
    for b in range(n_bands):
        cid, ln = struct.unpack_from("<BI", blob, 20 + 5 * b)
        out.append((cid, ln))
    return out


def _entropy(counts):
    c = counts[counts > 0].astype(np.float64)
    p = c / c.sum()
    return float(-(p * np.log2(p)).sum())


def proxies(x):
    """Cheaper criteria of one band's bytes: order-0 entropy and the entropy
    of adjacent byte pairs without the rotation sort."""
    x = np.asarray(x, np.uint8)
    h0 = _entropy(np.bincount(x, minlength=256))
    q = x[:-1].astype(np.int64) * 256 + x[1:]
    h2 = _entropy(np.bincount(q, minlength=65536)) if q.size else 0.0
    return h0, h2


def study_frame(ctx, frame, prev, pitch, level, mask, with_proxies=False):
    """Per band: the judged id, the entropies, the coded size of each
    candidate, and (with_proxies) the two cheaper criteria of each."""
    ids = [c for c in range(NCAND) if (mask >> c) & 1]
    choice, ent, _ = ctx.judge(frame, prev, pitch, level, mask)
    choice = choice.cpu().numpy()
    ent = ent.cpu().numpy()
    nb = len(choice)
    sizes = np.full((nb, NCAND), -1, np.int64)
    prox = np.full((nb, NCAND, 2), np.nan)
    for c in ids:
        blob = ctx.compress(frame, prev, pitch, level, mask, forced=np.full(nb, c, np.uint8))
        for b, (cid, ln) in enumerate(band_lengths(blob)):
            assert cid == c
            sizes[b, c] = ln
        if with_proxies:
            ctx.decompress(blob, prev=prev)
            n_raw = 2 * frame.size
            raw = ctx.decompress_inspect(4, n_raw)
            off = 0
            for b in range(nb):
                n = _band_bytes(frame.shape, pitch, level, b)
                prox[b, c] = proxies(raw[off:off + n])
                off += n
    return choice, ent, sizes, ids, prox


def _band_bytes(shape, pitch, level, b):
    h, w = shape
    R = max(1, (100000 * level - 19) // (2 * pitch * w))
    ns = h // pitch
    return 2 * min(R, ns - b * R) * pitch * w


def summarize(rows):
    judged = best = 0
    agree = n = 0
    rank_ok = pairs = 0
    px_bytes = [0, 0]
    px_agree = [0, 0]
    have_px = False
    won = {}
    for choice, ent, sizes, ids, prox in rows:
        for b in range(len(choice)):
            s = {c: sizes[b, c] for c in ids}
            c_best = min(ids, key=lambda c: (s[c], c))
            judged += s[int(choice[b])]
            best += s[c_best]
            agree += int(choice[b]) == c_best
            won[int(choice[b])] = won.get(int(choice[b]), 0) + 1
            n += 1
            for i in ids:
                for j in ids:
                    if i < j and s[i] != s[j]:
                        pairs += 1
                        rank_ok += (ent[b, i] < ent[b, j]) == (s[i] < s[j])
            if not np.isnan(prox[b, ids[0], 0]):
                have_px = True
                for k in range(2):
                    c_px = min(ids, key=lambda c: (prox[b, c, k], c))
                    px_bytes[k] += s[c_px]
                    px_agree[k] += c_px == c_best
    out = {"bands": n, "agreement": agree / max(n, 1), "judge_regret": judged / max(best, 1) - 1.0,
           "judged_bytes": int(judged), "best_bytes": int(best),
           "pairwise_order_agreement": rank_ok / max(pairs, 1),
           "judged_ids": {str(k): v for k, v in sorted(won.items())}}
    if have_px:
        for k, name in enumerate(("order0", "pairs")):
            out[f"{name}_agreement"] = px_agree[k] / max(n, 1)
            out[f"{name}_regret"] = px_bytes[k] / max(best, 1) - 1.0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--vessel-frames", type=int, default=12)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    ctx = pcbz.Context(0)
    sets = {}
    rows = []
    for peak in (20.0, 100.0, 1000.0):
        rows.append(study_frame(ctx, synth.config2_frame(peak), None, 15, 9, 0x7, True))
    sets["beads_2040_k3"] = summarize(rows)
    rows = [study_frame(ctx, synth.config2_frame(peak), None, 15, 9, 0xFFF7, True) for peak in (20.0, 1000.0)]
    sets["beads_2040_k15"] = summarize(rows)
    print("beads done", file=sys.stderr, flush=True)
    series = synth.vessel_series(args.vessel_frames + 3)
    frames = [f for f, _ in series]
    rows, rows16 = [], []
    for i, (f, pi) in enumerate(series):
        if pi is None:
            continue
        rows.append(study_frame(ctx, f, frames[pi], 15, 9, 0xF, True))
        if len(rows16) < 3:
            rows16.append(study_frame(ctx, f, frames[pi], 15, 9, 0xFFFF, True))
    sets["vessels_k4"] = summarize(rows)
    sets["vessels_k16"] = summarize(rows16)
    out = json.dumps(sets, indent=1)
    if args.report:
        with open(args.report, "w") as fh:
            fh.write(out + "\n")
    print(out, flush=True)


if __name__ == "__main__":
    main()
