"""Step models of RLM-sort (recurse-last multiway mergesort, Section 5) and
of multisequence selection (Section 4.1).  TEST INFRASTRUCTURE ONLY (see the
package docstring).

Elements are compared by their ord value; ties are broken by the index of
the sequence holding them and then by their position in it, so every
element is distinct (the tie-breaking of Section 2 and Appendix D).  When the
sequences are consecutive tiles of one input, sorted stably, this order is
(key, input position): the stable order.

Functions
  multi_select   the quickselect-style selection of Section 4.1 (its figure
                 "Multisequence selection algorithm"): random pivot, a binary
                 search in every sequence, recurse on the side that holds
                 rank k.  Returns the element of rank k.
  split_of       positions that cut every sequence after the k smallest
                 elements (what RLM-sort delivers to each part).
  rlm_splits     the r-1 simultaneous selections of one RLM level: part j
                 receives global ranks [floor(j N / r), floor((j+1) N / r)).
  rlm_sort       the whole algorithm of Section 5 on one array: sort tiles
                 ("every PE sorts locally first"), split every group's
                 sequences into r parts of (almost) equal size, deliver each
                 part, merge what a part received into new sorted sequences,
                 recurse on the parts.  Its output must be the plain sort.

Pins (tests/test_oracle_rlm.py): brute force (sort all (key, seq, pos)
triples and count) for multi_select and split_of over many small random and
exhaustive cases, with duplicates; rlm_sort against the textbook mergesort;
planted mistakes in copies of multi_select (pivot compared with <= instead of
<, sequence tie-break reversed, rank off by one) fail those pins.
"""

from __future__ import annotations

import bisect

import numpy as np

from . import rng as orng


def _count_before(seq, i: int, pivot) -> int:
    """Elements of sequence i that precede pivot = (x, q, t) in the total
    order (key, sequence index, position): binary search."""
    x, q, t = pivot
    if i < q:
        return bisect.bisect_right(seq, x)   # equal keys of earlier sequences come first
    if i > q:
        return bisect.bisect_left(seq, x)    # equal keys of later sequences come after
    return t                                  # the pivot's own sequence: positions before t


def multi_select(seqs, k: int, seed: int = 1):
    """Element of global rank k (1-based) among the sorted sequences, as
    (ord value, sequence index, position) (Section 4.1).

    Each round keeps, per sequence i, the window seqs[i][lo_i:hi_i] that may
    still hold the answer.  A pivot is drawn uniformly from the union of the
    windows (one random number over the total window size, located through a
    prefix sum of the window sizes); a binary search in every window finds
    j_i, the number of window elements that precede the pivot.  If at least k
    elements precede it, the answer lies in the left parts; otherwise it lies
    in the right parts, with k reduced by the left parts' total.  A single
    remaining element is the answer.
    """
    p = len(seqs)
    lo = [0] * p
    hi = [len(s) for s in seqs]
    if not 1 <= k <= sum(hi):
        raise ValueError("rank out of range")
    draw = 0
    state = orng.mix64(seed)
    while True:
        sizes = [hi[i] - lo[i] for i in range(p)]
        total = sum(sizes)
        if total == 1:
            i = next(i for i in range(p) if sizes[i])
            return (int(seqs[i][lo[i]]), i, lo[i])
        # pivot: uniform over the union of the windows
        draw += 1
        u = (orng.mix64((state + draw * orng.GAMMA) & orng.M64) * total) >> 64
        q = 0
        while u >= sizes[q]:
            u -= sizes[q]
            q += 1
        t = lo[q] + u
        pivot = (int(seqs[q][t]), q, t)
        # j_i: window elements that precede the pivot
        j = [min(max(_count_before(seqs[i], i, pivot), lo[i]), hi[i]) for i in range(p)]
        left = sum(j[i] - lo[i] for i in range(p))
        if left >= k:
            hi = j
        else:
            k -= left
            lo = j


def split_of(seqs, element):
    """Per sequence, the number of its elements that are at most `element`
    in the total order: cutting there leaves the elements of ranks
    1..rank(element) on the left."""
    x, q, t = element
    return [bisect.bisect_right(s, x) if i < q else (t + 1 if i == q else bisect.bisect_left(s, x))
            for i, s in enumerate(seqs)]


def rank_split(seqs, k: int, seed: int = 1):
    """Cut positions of the k smallest elements (k = 0 and k = total
    included)."""
    if k == 0:
        return [0] * len(seqs)
    if k == sum(len(s) for s in seqs):
        return [len(s) for s in seqs]
    return split_of(seqs, multi_select(seqs, k, seed))


def part_ranks(N: int, r: int):
    """Rank boundaries of r parts of a group of N elements: part j holds
    ranks [floor(j N / r), floor((j+1) N / r)).  Reading: the paper asks for
    parts of n/r elements each; with N not divisible by r the floors spread
    the remainder."""
    return [(j * N) // r for j in range(r + 1)]


def rlm_splits(seqs, r: int, seed: int = 1):
    """The r-1 selections of one level (run side by side in the paper):
    cuts[j][i] for j = 0..r, cuts[0] = 0, cuts[r] = len."""
    N = sum(len(s) for s in seqs)
    return [rank_split(seqs, k, seed + j) for j, k in enumerate(part_ranks(N, r))]


def _merge_pieces(pieces):
    """Stable multiway merge: pieces in sequence order, ties to the lower
    sequence (a heap-free textbook merge of sorted lists, two at a time)."""
    runs = [list(p) for p in pieces if len(p)]
    if not runs:
        return []
    while len(runs) > 1:
        nxt = []
        for a in range(0, len(runs), 2):
            if a + 1 == len(runs):
                nxt.append(runs[a])
                continue
            A, B = runs[a], runs[a + 1]
            out, i, jj = [], 0, 0
            while i < len(A) and jj < len(B):
                if B[jj] < A[i]:
                    out.append(B[jj])
                    jj += 1
                else:
                    out.append(A[i])
                    i += 1
            out.extend(A[i:])
            out.extend(B[jj:])
            nxt.append(out)
        runs = nxt
    return runs[0]


def level_parts(N: int, r: int, tile: int) -> int:
    """Parts a group of N elements is split into: r while the parts stay
    larger than a tile, else just enough parts of at most one tile each (the
    last level).  Reading: the paper fixes r = p/p' per level; here the last
    level takes the count that finishes every part in one merge."""
    return r if N > r * tile else -(-N // tile)


def merge_slices(pieces, tile: int):
    """New sorted sequences of a part: the concatenation of its pieces (in
    sequence order) cut into slices of `tile` elements, each slice merged
    (a PE of the group holding `tile` elements merges what it received)."""
    bounds = np.cumsum([0] + [len(pc) for pc in pieces])
    new = []
    for a in range(0, int(bounds[-1]), tile):
        sl = []
        for i, pc in enumerate(pieces):
            lo = max(a, int(bounds[i]))
            hi = min(a + tile, int(bounds[i + 1]))
            if lo < hi:
                sl.append(pc[lo - int(bounds[i]):hi - int(bounds[i])])
        new.append(_merge_pieces(sl))
    return new


def rlm_sort(ords, tile: int, r: int, seed: int = 1):
    """RLM-sort of one array of ord values (Section 5), small inputs only.

    Every tile of `tile` elements is sorted first (every PE sorts locally).
    A group is a list of sorted sequences.  A group of more than one tile is
    split into level_parts(...) parts of equal size by simultaneous
    selections; part j receives piece j of every sequence and merges them
    into new sequences (merge_slices); the parts are sorted recursively, in
    order, and a group of at most one tile is finished by merging its
    sequences.  Returns the sorted ords.
    """
    def solve(g):
        N = sum(len(s) for s in g)
        if N <= tile:
            return _merge_pieces(g)
        parts = level_parts(N, r, tile)
        cuts = rlm_splits(g, parts, seed)
        res = []
        for j in range(parts):
            pieces = [g[i][cuts[j][i]:cuts[j + 1][i]] for i in range(len(g))]
            res.extend(solve(merge_slices(pieces, tile)))
        return res

    x = [int(v) for v in ords]
    return solve([sorted(x[a:a + tile]) for a in range(0, len(x), tile)])
