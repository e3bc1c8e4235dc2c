"""Seeded element samples for full-size parity checks (test helpers).

every_tile(E): one element drawn from every run of 16 consecutive elements
(the width of a wave's element tile on the matrix cores) plus the whole first
and last `edge` elements, so that every wave-tile of a launch, its first and
last work-group tiles and a ragged end are all checked."""
import numpy as np


def every_tile(E, seed=0, width=16, edge=512):
    rng = np.random.default_rng(seed)
    starts = np.arange(0, E, width, dtype=np.int64)
    span = np.minimum(width, E - starts)
    picks = starts + (rng.random(starts.size) * span).astype(np.int64)
    ends = np.concatenate([np.arange(min(edge, E)), np.arange(max(0, E - edge), E)])
    return np.unique(np.concatenate([picks, ends]).astype(np.int64))
