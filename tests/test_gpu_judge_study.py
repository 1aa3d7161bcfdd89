"""GPU check of the judge-fidelity study against the oracle: the judged ids and
entropies equal the oracle's judgement, every per-candidate band size equals
the band length in the oracle's container coded with that candidate forced,
and the study's summary follows from those sizes."""
import numpy as np
import pytest

from paper_2310_09467_amd import synth

pytestmark = pytest.mark.gpu


def test_judge_study_small(orc):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_09467_amd import judge_study, pcbz

    ctx = pcbz.Context(0)
    frame = synth.config1_frame(1)
    big, _ = synth.beads_frame(450, 300, 40, 300.0, seed=13)
    rows = []
    for f, lv, mask in ((frame, 1, 0x7), (big, 2, 0x7), (big, 9, 0xFFF7)):
        row = judge_study.study_frame(ctx, f, None, 15, lv, mask, with_proxies=True)
        choice, ent, sizes, ids, prox = row
        oc, _, oh = orc.judge(f, None, 15, lv, mask)
        np.testing.assert_array_equal(choice, oc)
        for c in ids:
            np.testing.assert_allclose(ent[:, c], oh[:, c], rtol=0, atol=1e-9)
            blob, _ = orc.compress(f, None, 15, lv, mask, forced_choice=np.full(len(oc), c, np.uint8))
            info = orc.peek(blob)
            np.testing.assert_array_equal(sizes[:, c], info["band_len"])
            assert (info["ids"] == c).all()
            # the cheaper criteria from the oracle's arranged bytes of each band
            for b in range(len(oc)):
                x = orc.to_bytes(orc.arrange(f, b, c, None, 15, lv))
                np.testing.assert_allclose(prox[b, c], judge_study.proxies(x), rtol=0, atol=1e-12)
        rows.append(row)
    s = judge_study.summarize(rows)
    # the summary recomputed from the oracle-checked sizes by hand
    n = agree = 0
    judged = best = 0
    for choice, ent, sizes, ids, prox in rows:
        for b in range(len(choice)):
            c_best = min(ids, key=lambda c: (sizes[b, c], c))
            agree += int(choice[b]) == c_best
            judged += sizes[b, int(choice[b])]
            best += sizes[b, c_best]
            n += 1
    assert s["bands"] == n and s["agreement"] == agree / n
    assert s["judge_regret"] == judged / best - 1.0
