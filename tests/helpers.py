"""Shared test helpers: input conversion and comparison against the oracle."""
import numpy as np

import oracle


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def words_np(t):
    """int64 device tensor of sketch words -> uint64 numpy array."""
    return t.cpu().numpy().view(np.uint64)


def sets_rows(S, rows):
    """Sub-view of oracle Sets restricted to the given row indices."""
    rows = np.asarray(rows)
    return oracle.Sets(S.vals, S.start[rows], S.length[rows])


def assert_topk_equal(gi, gs, oi, osc):
    """GPU and oracle top-k lists are identical (indices and FP32 scores)."""
    gi = np.asarray(gi)
    gs = np.asarray(gs)
    bad = np.nonzero((gi != oi).any(1) | (gs.view(np.uint32) != osc.view(np.uint32)).any(1))[0]
    assert len(bad) == 0, "top-k differs for queries %s: gpu %s / %s vs oracle %s / %s" % (
        bad[:5].tolist(), gi[bad[0]][:8].tolist(), gs[bad[0]][:8].tolist(),
        oi[bad[0]][:8].tolist(), osc[bad[0]][:8].tolist())
