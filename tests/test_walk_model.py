"""Host-side model of the activation step's walk (one wave per (query,
subspace)), checked against the oracle's Dynamic Activation (Alg. 3).

On the GPU, lane c holds the row of first-half centre c in centre order, not
in rank order; the second half's centres are sorted (ascending distance, ties
by id) only up to a fixed number of columns; each step takes the smallest
frontier key d1[c] + d2[column], and equal keys go to the smaller d1, then
the smaller centre id.  The claim is that this visits cells in exactly the
order (key, r1, r2) of the ranks, so that it takes the oracle's prefix, and
that a row running out of sorted columns is the only case it has to hand to
the general path.  Distances are drawn as small integers (forced key ties)
or as uniform reals; the walk adds them in float64 like the oracle.
"""
import numpy as np
import pytest

import oracle
from test_oracle_pins import grid_index


def walk(d1, d2, sizes, sk, A, ncol):
    """The GPU walk on the host; None when a row would need a column past ncol."""
    cols = np.lexsort((np.arange(sk), d2))[:ncol]       # second half, rank order
    ptr = np.zeros(sk, np.int64)
    taken, W = [], 0
    for _ in range(sk * sk):
        live = ptr < len(cols)
        if not live.any():
            break
        keys = np.where(live, d1 + d2[cols[np.minimum(ptr, len(cols) - 1)]], np.inf)
        m = keys.min()
        cand = np.nonzero(keys == m)[0]
        if len(cand) > 1:                               # equal keys: smaller d1, then smaller id
            dm = d1[cand].min()
            cand = cand[d1[cand] == dm]
        r = int(cand[0])
        c2 = int(cols[ptr[r]])
        taken.append(r * sk + c2)
        W += int(sizes[r * sk + c2])
        ptr[r] += 1
        if W >= A:
            return taken, W
        if ptr[r] == len(cols) and len(cols) < sk:
            return None                                 # this row's next column is not sorted
    return taken, W


@pytest.mark.parametrize("seed", range(40))
def test_walk_takes_the_oracle_prefix(seed):
    rng = np.random.default_rng(100 + seed)
    sk = int(rng.integers(1, 13))
    sizes = rng.integers(0, 6, size=sk * sk)
    sizes[rng.integers(0, sk * sk)] += 1
    ix = grid_index(sk, sizes.tolist())
    n = int(sizes.sum())
    if seed % 2:
        d1 = rng.integers(0, 4, size=sk).astype(np.float64)
        d2 = rng.integers(0, 4, size=sk).astype(np.float64)
    else:
        d1, d2 = rng.random(sk), rng.random(sk)
    i1 = np.lexsort((np.arange(sk), d1)).astype(np.int32)
    i2 = np.lexsort((np.arange(sk), d2)).astype(np.int32)
    checked = 0
    for A in sorted({1, max(1, n // 4), max(1, n // 2), n}):
        ref_cells, ref_ap = ix.da(0, d1, i1, d2, i2, A, form=0)
        for ncol in (sk, min(sk, 3)):
            got = walk(d1, d2, sizes, sk, A, ncol)
            if got is None:
                assert ncol < sk                        # only a limited column count hands over
                continue
            cells, W = got
            assert sorted(cells) == sorted(ref_cells.tolist())
            assert W == ref_ap
            checked += 1
    assert checked >= 1
