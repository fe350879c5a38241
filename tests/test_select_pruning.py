"""Host-side property test of the rule by which the collision step leaves score
levels out of a tile's id lists, and of the per-tile selection plan.

The candidates of a query are the B points of highest SC-score, ties broken by
lower id (Alg. 4's sort of the scores, with the tie reading of the design
notes).  The GPU counts scores tile by tile (tiles are ranges of consecutive
ids); a block takes the tiles p = g, g + S, g + 2S, ... of a query in order and
lists, per tile, the ids of each non-zero level, except the levels s for which
the block's earlier tiles already hold at least B ids of score >= s.  The
selection then takes, tile by tile in id order, the ids above the threshold T
and its share of the lowest level-T ids, from the lists, with the complete
per-tile histograms.  This test draws random score arrays and checks, with a
plain definition of the candidate set, that every id the selection takes is in
the lists and that the result is that set, for one and several tile groups.
"""
import numpy as np


def candidates_by_definition(scores, B):
    """The B ids of highest score, ties by lower id (ids in ascending order)."""
    order = np.lexsort((np.arange(scores.size), -scores.astype(np.int64)))
    return np.sort(order[:B])


def listed_ids(scores, tile, B, S, ns):
    """Per tile: the set of ids the collision step lists (levels left out as the GPU does)."""
    P = (scores.size + tile - 1) // tile
    lists = [None] * P
    for g in range(S):
        cum = np.zeros(ns + 2, np.int64)          # #{score >= s} over this group's earlier tiles
        for p in range(g, P, S):
            sc = scores[p * tile:(p + 1) * tile]
            s0 = 0
            for s in range(ns, 0, -1):
                if cum[s] >= B:
                    s0 = s
                    break
            ids = np.nonzero(sc > s0)[0] + p * tile
            lists[p] = set(ids.tolist())
            for s in range(1, ns + 1):
                cum[s] += int((sc >= s).sum())
    return lists


def select_from_lists(scores, tile, B, ns, lists):
    """The selection's plan: T from the summed histograms, then tile by tile the
    ids above T and the lowest level-T ids still needed, read from the lists."""
    n = scores.size
    P = (n + tile - 1) // tile
    G = np.array([(scores >= t).sum() for t in range(ns + 2)], np.int64)
    T = max(t for t in range(ns + 1) if G[t] >= B)
    R = B - G[T + 1]
    out, eq_before = [], 0
    for p in range(P):
        sc = scores[p * tile:(p + 1) * tile]
        ids = np.arange(p * tile, p * tile + sc.size)
        gt = ids[sc > T]
        E = int((sc == T).sum())
        take = min(E, max(0, R - eq_before))
        eq_before += E
        if T > 0:
            for i in gt.tolist():
                assert i in lists[p], f"tile {p}: id {i} above T={T} was left out"
            level_t = sorted(i for i in lists[p] if scores[i] == T)
            if take > 0:
                assert len(level_t) == E, f"tile {p}: takes {take} level-{T} ids but lists {len(level_t)} of {E}"
            chosen = sorted(gt.tolist() + level_t[:take])
        else:
            # fewer than B points collide: score-0 ids are those absent from the lists
            nz = sorted(i for i in lists[p] if scores[i] > 0)
            assert nz == gt.tolist()
            zeros = ids[sc == 0].tolist()
            chosen = sorted(gt.tolist() + zeros[:take])
        out.extend(chosen)
    return np.array(out, np.int64)


def test_left_out_levels_are_never_selected():
    rng = np.random.default_rng(7)
    cases = 0
    for trial in range(600):
        ns = int(rng.integers(1, 9))
        n = int(rng.integers(50, 3000))
        tile = int(rng.integers(8, 400))
        P = (n + tile - 1) // tile
        S = int(rng.integers(1, min(P, 4) + 1))
        # skewed scores: mostly 0 and 1, a few high (like activation-driven collisions)
        p_nz = rng.uniform(0.05, 0.9)
        scores = np.where(rng.random(n) < p_nz, rng.geometric(rng.uniform(0.3, 0.9), n), 0)
        scores = np.minimum(scores, ns).astype(np.int64)
        if trial % 2:
            B = int(rng.integers(1, n + 1))
        else:
            # B at a boundary: the count of score >= s over group 0's first tiles, +-1
            s = int(rng.integers(1, ns + 1))
            k = int(rng.integers(1, max(2, (P + S - 1) // S)))
            first = np.concatenate([scores[p * tile:(p + 1) * tile] for p in range(0, P, S)][:k])
            B = int(np.clip((first >= s).sum() + int(rng.integers(-1, 2)), 1, n))
        lists = listed_ids(scores, tile, B, S, ns)
        got = select_from_lists(scores, tile, B, ns, lists)
        ref = candidates_by_definition(scores, B)
        assert np.array_equal(got, ref), f"trial {trial}: n={n} tile={tile} S={S} B={B}"
        cases += 1
    assert cases == 600


def test_tie_level_left_out_after_early_tiles():
    """The SIFT-like situation: almost every colliding point scores 1 and the
    threshold is 1; once the first tiles hold B ids of score >= 1, the later
    tiles list only their few ids of score 2 or more."""
    rng = np.random.default_rng(3)
    n, tile, ns, B = 20000, 1000, 8, 1500
    scores = np.where(rng.random(n) < 0.2, 1, 0)
    hi = rng.choice(n, 300, replace=False)
    scores[hi] = rng.integers(2, 5, hi.size)
    lists = listed_ids(scores, tile, B, 1, ns)
    # tiles after the first ones list no level-1 id
    later = [p for p in range(len(lists)) if p >= 10]
    assert all(all(scores[i] >= 2 for i in lists[p]) for p in later)
    got = select_from_lists(scores, tile, B, ns, lists)
    assert np.array_equal(got, candidates_by_definition(scores, B))
