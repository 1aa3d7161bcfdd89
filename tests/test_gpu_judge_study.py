"""GPU check of the judge-fidelity study: per-band lengths read from the
container header add up to the container, the smallest candidate is never
larger than the judged one, and the study's figures are in range."""
import numpy as np
import pytest

from paper_2310_09467_amd import synth

pytestmark = pytest.mark.gpu


def test_judge_study_small():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_09467_amd import judge_study, pcbz

    ctx = pcbz.Context(0)
    frame = synth.config1_frame(1)
    big, _ = synth.beads_frame(450, 300, 40, 300.0, seed=13)
    rows = []
    for f, lv in ((frame, 1), (big, 2)):
        blob = ctx.compress(f, None, 15, lv, 0x7)
        lens = judge_study.band_lengths(blob)
        nb = pcbz.plan(*f.shape, 15, lv, 0x7)[0]
        assert len(lens) == nb
        assert 20 + 5 * nb + sum(ln for _, ln in lens) == len(blob)
        rows.append(judge_study.study_frame(ctx, f, None, 15, lv, 0x7))
    for choice, ent, sizes, ids in rows:
        for b in range(len(choice)):
            assert min(sizes[b, c] for c in ids) <= sizes[b, int(choice[b])]
    s = judge_study.summarize(rows)
    assert 0.0 <= s["agreement"] <= 1.0 and s["judge_regret"] >= 0.0
    assert 0.0 <= s["pairwise_order_agreement"] <= 1.0
