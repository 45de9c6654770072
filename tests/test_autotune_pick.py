"""Host logic of the autotuner's choice (no GPU): the fastest candidate,
with ties between the fused and the split row path going to the split path."""
from paper_2408_11472_amd import autotune as at

F, S = at.PATH_FUSED, at.PATH_SPLIT


def test_fastest_wins_when_clearly_faster():
    assert at.pick({(F, 256): 700.0, (F, 64): 900.0, (S, 0): 800.0}) == (F, 256)
    assert at.pick({(F, 256): 820.0, (S, 0): 700.0}) == (S, 0)


def test_tie_within_margin_goes_to_split():
    # 839.9 (split) vs 840.9 (fused): split already fastest
    assert at.pick({(F, 256): 840.9, (S, 0): 839.9}) == (S, 0)
    # fused 1 % faster: within the margin, split kept
    assert at.pick({(F, 256): 825.0, (F, 512): 826.0, (S, 0): 833.0}) == (S, 0)
    # just beyond the margin: fused kept
    t = 800.0
    assert at.pick({(F, 128): t, (S, 0): t * (1 + at.FUSED_MARGIN) * 1.001}) == (F, 128)


def test_without_split_candidate():
    assert at.pick({(F, 128): 2.0, (F, 256): 1.0}) == (F, 256)
