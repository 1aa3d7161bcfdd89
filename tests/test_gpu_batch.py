"""Batched compression: one pass over all bands of many uneven frames, replayed
from a captured graph with an autotuned schedule.  Every frame's container must
equal pcbz_compress of that frame alone and the oracle's (0 bytes tolerance),
on every replay, with eager work in between replays."""
import os
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _batch():
    from paper_2310_09467_amd import synth

    frames, prevs, params = [], [], []
    shapes = [(450, 300), (300, 450), (225, 225), (510, 510), (450, 300), (90, 3345)]
    for i, (h, w) in enumerate(shapes):
        f, pos = synth.beads_frame(h, w, 60, 150.0 + 80 * i, 70 + i)
        p, _ = synth.beads_frame(h, w, 60, 150.0 + 80 * i, 170 + i, positions=pos)
        frames.append(f)
        prevs.append(p if i % 2 == 0 else None)
        params.append((15, 9 if i % 3 else 1, 0xF if i % 2 == 0 else 0x7))
    return frames, prevs, params


def test_graph_replays_equal_single_frames(orc, tmp_path):
    import torch

    from paper_2310_09467_amd import pcbz

    os.environ["PCBZ_TUNE_CACHE"] = str(tmp_path / "tune.jsonl")
    try:
        ctx = pcbz.Context(0)
    finally:
        del os.environ["PCBZ_TUNE_CACHE"]
    ctx.set_graphs(2)  # replay graphs even where an eager call would be faster
    frames, prevs, params = _batch()
    ref = [orc.compress(f, p, pp, lv, m)[0] for f, p, (pp, lv, m) in zip(frames, prevs, params)]
    for rep in range(4):  # first call tunes (eager + captures), later calls replay the graph
        print("replay", rep, flush=True)
        blobs = ctx.compress_batch(frames, prevs, params)
        assert blobs == ref
        # eager work between replays
        assert ctx.compress(frames[2], prevs[2], *params[2]) == ref[2]
        torch.cuda.synchronize()
    assert (tmp_path / "tune.jsonl").exists()
    ctx.close()


def test_forced_choices_in_batch(orc):
    from paper_2310_09467_amd import pcbz

    ctx = pcbz.Context(0)
    ctx.set_graphs(2)  # replay graphs even where an eager call would be faster
    frames, prevs, params = _batch()
    rng = np.random.default_rng(5)
    forced = []
    for f, p, (pp, lv, m) in zip(frames, prevs, params):
        nb = orc.plan(f.shape[0], f.shape[1], pp, lv)[1]
        hi = 4 if p is not None else 3
        forced.append(rng.integers(0, hi, nb).astype(np.uint8))
    for rep in range(2):
        blobs = ctx.compress_batch(frames, prevs, params, forced=forced)
        for f, p, (pp, lv, m), fc, b in zip(frames, prevs, params, forced, blobs):
            assert b == orc.compress(f, p, pp, lv, m, forced_choice=fc)[0]
    ctx.close()


def test_radix_tile_schedules_give_identical_bytes(orc):
    """Eager calls with 8- and 16-element radix tiles agree byte for byte."""
    from paper_2310_09467_amd import pcbz, synth

    f = synth.config2_frame(100.0)
    out = []
    for items in ("8", "16"):
        os.environ["PCBZ_RADIX_ITEMS"] = items
        try:
            ctx = pcbz.Context(0)
        finally:
            del os.environ["PCBZ_RADIX_ITEMS"]
        out.append(ctx.compress(f, None, 15, 9, 7))
        ctx.close()
    assert out[0] == out[1]
    assert out[0] == orc.compress(f, None, 15, 9, 7)[0]


def test_graph_falls_back_when_a_group_is_too_large(orc, tmp_path):
    """A graph learned on noisy frames sorts later rounds group by group; a
    frame of the same shape with groups of 10350 rotations (a 20-byte period)
    cannot be sorted that way and needs more rounds, so the replay flags
    itself and the call is redone eagerly (still exact)."""
    from paper_2310_09467_amd import pcbz, synth

    os.environ["PCBZ_TUNE_CACHE"] = str(tmp_path / "tune.jsonl")
    try:
        ctx = pcbz.Context(0)
    finally:
        del os.environ["PCBZ_TUNE_CACHE"]
    ctx.set_graphs(2)  # replay graphs even where an eager call would be faster
    h, w = 300, 345
    noisy, _ = synth.beads_frame(h, w, 40, 200.0, 11)
    rng = np.random.default_rng(3)
    pat = rng.integers(0, 256, 20, dtype=np.uint8)
    periodic = np.resize(pat, 2 * h * w).view(np.uint16).reshape(h, w).copy()
    nb = orc.plan(h, w, 15, 9)[1]
    raster = [np.zeros(nb, np.uint8)]
    want = {k: orc.compress(f, None, 15, 9, 0x7, forced_choice=raster[0])[0]
            for k, f in (("noisy", noisy), ("periodic", periodic))}
    for rep, name in enumerate(["noisy", "noisy", "periodic", "periodic", "noisy"]):
        print("call", rep, name, flush=True)
        f = noisy if name == "noisy" else periodic
        assert ctx.compress_batch([f], None, [(15, 9, 0x7)], forced=raster) == [want[name]]
    ctx.close()


def test_batch_modes_agree(orc):
    """Eager, autotuned and always-graph batch modes give the same bytes;
    other mode values are refused."""
    from paper_2310_09467_amd import pcbz

    frames, prevs, params = _batch()
    ref = [orc.compress(f, p, pp, lv, m)[0] for f, p, (pp, lv, m) in zip(frames, prevs, params)]
    ctx = pcbz.Context(0)
    for mode in (0, 1, 2, 1):
        ctx.set_graphs(mode)
        for _ in range(2):
            assert ctx.compress_batch(frames, prevs, params) == ref
    with pytest.raises(pcbz.PcbzError):
        ctx.set_graphs(3)
    ctx.close()


def test_tuning_replay_that_fails_leaves_correct_bytes(orc, tmp_path):
    """When a schedule tried by the autotuner does not reproduce the eager
    result (here: a round budget of one doubling round, too few for the data),
    the caller's buffers still end up holding the right containers."""
    from paper_2310_09467_amd import pcbz, synth

    os.environ["PCBZ_TUNE_ROUNDS"] = "1"
    try:
        ctx = pcbz.Context(0)
    finally:
        del os.environ["PCBZ_TUNE_ROUNDS"]
    frames = [synth.config1_frame(3), synth.config1_frame(4)]
    params = [(15, 1, 0x3)] * 2
    ref = [orc.compress(f, None, p, lv, m)[0] for f, (p, lv, m) in zip(frames, params)]
    assert ctx.compress_batch(frames, None, params) == ref  # the tuning call
    assert ctx.last_stats()["bwt_rounds"] > 1  # so a one-round graph cannot reproduce it
    assert ctx.compress_batch(frames, None, params) == ref  # the tuned choice (eager)
    ctx.close()
