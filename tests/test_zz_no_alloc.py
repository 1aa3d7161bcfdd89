"""pcbz_judge_noalloc (the judge on a fixed device workspace) against
pcbz_judge, through the C ABI: choices and fixed-point scores bit-exact,
entropies equal; two calls in a row, the second on a smaller frame (the
workspace keeps the first call's contents); a frame too large for the fixed
workspace is refused with nothing written; no device memory is allocated."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _frames():
    from paper_2310_09467_amd import synth

    big = synth.config2_frame(100.0)  # 2040 x 2040, ten bands at level 9
    big_prev, _ = synth.beads_frame(2040, 2040, 2000, 100.0, 33)
    small, pos = synth.beads_frame(450, 300, 60, 300.0, 71)
    small_prev, _ = synth.beads_frame(450, 300, 60, 300.0, 171, positions=pos)
    return [(big, big_prev, 9, 0xF), (small, small_prev, 1, 0x7), (small, small_prev, 9, 0xF)]


def _same(a, b):
    ca, ea, sa = (t.cpu().numpy() for t in a)
    cb, eb, sb = (t.cpu().numpy() for t in b)
    assert np.array_equal(ca, cb)
    assert np.array_equal(sa, sb)
    assert np.array_equal(np.isnan(ea), np.isnan(eb))
    assert np.array_equal(ea[~np.isnan(ea)], eb[~np.isnan(eb)])


def test_noalloc_judge_equals_judge(orc):
    import torch

    from paper_2310_09467_amd import pcbz

    ctx = pcbz.Context(0)
    for f, pv, level, mask in _frames():
        print("frame", f.shape, "level", level, "mask", hex(mask), flush=True)
        ref = ctx.judge(f, pv, 15, level, mask)
        got = ctx.judge(f, pv, 15, level, mask, noalloc=True)
        torch.cuda.synchronize()
        _same(ref, got)
        # and the oracle's choices on the same frame
        oc, osc, _ = orc.judge(f, pv, 15, level, mask)
        assert np.array_equal(got[0].cpu().numpy(), oc)
        on = [(mask >> i) & 1 == 1 for i in range(16)]
        assert np.array_equal(got[2].cpu().numpy()[:, on], osc[:, on])
    ctx.close()


def test_noalloc_judge_allocates_nothing():
    import torch

    from paper_2310_09467_amd import pcbz

    ctx = pcbz.Context(0)  # a fresh context: its arena is empty
    f, pv, level, mask = _frames()[0]
    fd, pd = pcbz.to_device(f), pcbz.to_device(pv)
    nb, _ = pcbz.plan(2040, 2040, 15, level, mask)
    outs = (torch.empty(nb, dtype=torch.uint8, device="cuda"), torch.empty(nb * 4, dtype=torch.float64, device="cuda"),
            torch.empty(nb * 4, dtype=torch.int64, device="cuda"))
    p = pcbz.Params(2040, 2040, 15, level, mask)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        ctx.judge_into(fd, pd, p, *outs, noalloc=True)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0  # the judge alone allocates ~45 MB of arena
    ctx.close()


def test_noalloc_judge_refuses_frames_above_its_workspace():
    import torch

    from paper_2310_09467_amd import pcbz

    ctx = pcbz.Context(0)
    h, w = 2040, 4080  # two 2040 x 2040 frames' worth: ~90 MB of workspace with four candidates
    f = np.zeros((h, w), np.uint16)
    nb, _ = pcbz.plan(h, w, 15, 9, 0xF)
    choice = torch.full((nb,), 0xAB, dtype=torch.uint8, device="cuda")
    with pytest.raises(pcbz.PcbzError) as ei:
        ctx.judge_into(pcbz.to_device(f), pcbz.to_device(f), pcbz.Params(h, w, 15, 9, 0xF), choice, noalloc=True)
    assert ei.value.code == pcbz.ENOMEM
    torch.cuda.synchronize()
    assert bool((choice == 0xAB).all())
    ctx.close()
