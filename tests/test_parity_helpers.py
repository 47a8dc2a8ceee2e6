"""CPU checks of the float parity helper itself: it accepts the oracle's own
rows rounded to float32 and rejects rows whose ids are permuted against
their distances, rows out of (distance, id) order, duplicate ids and a
wrong neighbour."""
import numpy as np
import pytest

import oracle
from parity import assert_float_close


def _case():
    g = np.random.default_rng(11)
    pts = g.random((3000, 3)).astype(np.float32)
    pts[100:140] = pts[7]  # exact ties
    q = np.concatenate([pts[:200], g.random((300, 3)).astype(np.float32)])
    oi, od = oracle.knn_brute(pts, q, 8)
    return pts, q, oi, od


def test_accepts_the_oracle_rounded():
    pts, q, oi, od = _case()
    assert assert_float_close(oi.astype(np.int32), od.astype(np.float32), oi, od, pts, q) == 0


@pytest.mark.parametrize("plant", ["permuted_ids", "order", "duplicate", "wrong_id"])
def test_rejects_planted_mistakes(plant):
    pts, q, oi, od = _case()
    gi, gd = oi.astype(np.int32).copy(), od.astype(np.float32).copy()
    r = 250  # a fresh query: distinct distances
    assert len(set(np.round(od[r], 12))) == 8
    if plant == "permuted_ids":
        gi[r, [1, 2]] = gi[r, [2, 1]]
    elif plant == "order":
        gi[r, [1, 2]] = gi[r, [2, 1]]
        gd[r, [1, 2]] = gd[r, [2, 1]]
    elif plant == "duplicate":
        gi[r, 3] = gi[r, 2]
    else:
        far = int(np.argmax(np.sum((pts.astype(np.float64) - q[r]) ** 2, axis=1)))
        gi[r, 7] = far
    with pytest.raises(AssertionError):
        assert_float_close(gi, gd, oi, od, pts, q)
