"""Step models of one sample-sort level and of the base case.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each function is the plain definition of one step, written so that it can be
checked against the paper by eye.  Keys are handled as their ord values
(non-negative Python ints or uint64 numpy arrays).  Readings of passages the
paper leaves open are stated where they are used.
"""

from __future__ import annotations

import itertools
import math

import numpy as np

from . import rng


# ----------------------------------------------------------------------------
# Base case and sample sorting: all-pairs rank (Section 4.2)
# ----------------------------------------------------------------------------

def all_pairs_rank(ords) -> np.ndarray:
    """Rank of every element by comparing all pairs (Section 4.2).

    The simplest form of the fast work-inefficient sorter compares every pair
    of elements and sums the comparison results per element.  Ties are broken
    by position (Section 2), so
        rank_i = #{j : x_j < x_i} + #{j < i : x_j = x_i}.
    Pins: brute force over permutations, and numpy's stable argsort.
    """
    x = np.asarray(ords, dtype=np.uint64)
    n = x.size
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    less = (x[None, :] < x[:, None]).sum(axis=1)
    eq = (x[None, :] == x[:, None])
    before = np.tril(np.ones((n, n), dtype=bool), k=-1)
    return (less + (eq & before).sum(axis=1)).astype(np.int64)


def sort_by_rank(ords) -> np.ndarray:
    """Place every element at its all-pairs rank."""
    x = np.asarray(ords, dtype=np.uint64)
    out = np.empty_like(x)
    out[all_pairs_rank(x)] = x
    return out


# ----------------------------------------------------------------------------
# Sampling and splitter selection (Section 6)
# ----------------------------------------------------------------------------

def sample(ords, seed: int, level: int, root: int, offset: int, count: int) -> np.ndarray:
    """Random sample with replacement of ``count`` elements (Section 6: a
    sample of size a*b*r).  Positions come from SplitMix64 (``rng``)."""
    x = np.asarray(ords, dtype=np.uint64)
    pos = rng.sample_positions(seed, level, root, offset, x.size, count)
    return x[np.asarray(pos, dtype=np.int64)]


def select_splitters(sorted_sample, a: int, m: int) -> np.ndarray:
    """The m-1 splitters of equidistant rank in the sorted sample (Section 6).

    Reading: with a sample of a*m elements, splitter j (j = 1..m-1) is the
    element of 0-based rank j*a - 1, which leaves exactly a sample elements
    in every bucket.
    """
    s = np.asarray(sorted_sample, dtype=np.uint64)
    if s.size != a * m:
        raise ValueError("sample size must be a*m")
    return s[np.arange(1, m, dtype=np.int64) * a - 1]


def eq_enabled(splitters) -> bool:
    """Equality buckets are switched on for a subproblem when two splitters
    are equal (reading of Appendix D, which adds one comparison per element
    to separate keys equal to a splitter).

    Splitters are sorted, so two equal ones are neighbours.  Pin: brute force
    over every sorted array of up to 6 splitters from a 4-letter alphabet
    ("some two splitters are equal"), which also catches planted mistakes.
    """
    s = np.asarray(splitters, dtype=np.uint64)
    return bool(s.size > 1 and np.any(s[1:] == s[:-1]))


def num_ids(m: int, eq_on: bool) -> int:
    """Number of bucket ids: m regular buckets, plus m-1 equality buckets."""
    return 2 * m - 1 if eq_on else m


def classify(ords, splitters, eq_on: bool) -> np.ndarray:
    """Bucket id of every element (Section 2 "partitioning"; Section 6; App. D).

    Reading of the bucket boundaries: bucket b holds s_b < x <= s_{b+1}, i.e.
    b = #{j : s_j < x}, computed here by a linear scan over the splitters.
    With equality buckets on, an element equal to the splitter just above it
    (x = s_{b+1}, b < m-1) goes to equality bucket 2b+1 and every other one
    to 2b, so ids increase with the key.  Without them the id is b.
    """
    x = np.asarray(ords, dtype=np.uint64)
    s = np.asarray(splitters, dtype=np.uint64)
    b = np.zeros(x.size, dtype=np.int64)
    for sj in s:  # b = sum_j [s_j < x]
        b += (sj < x)
    if not eq_on:
        return b
    m = s.size + 1
    upper = np.where(b < m - 1, s[np.minimum(b, m - 2)], np.uint64(0))
    is_eq = (b < m - 1) & (x == upper)
    return 2 * b + is_eq.astype(np.int64)


def histogram(ids, nb: int) -> np.ndarray:
    """Bucket sizes (Section 6: global bucket sizes by reduction)."""
    h = np.zeros(nb, dtype=np.int64)
    for i in np.asarray(ids, dtype=np.int64):
        h[i] += 1
    return h


def exclusive_scan(v) -> np.ndarray:
    """Exclusive prefix sum (Section 4.3: prefix sum over piece sizes)."""
    out = np.zeros(len(v), dtype=np.int64)
    run = 0
    for i, c in enumerate(v):
        out[i] = run
        run += int(c)
    return out


# ----------------------------------------------------------------------------
# Bucket grouping (Section 6, its lemma, Appendix C)
# ----------------------------------------------------------------------------

def greedy_groups(w, L: int):
    """Scan the bucket sizes and open the next group when the load would
    exceed L (Section 6).  Returns the start index of every group, or None
    when some single bucket exceeds L.

    Reading: the bucket that does not fit opens the next group.
    """
    starts = [0]
    cur = 0
    for j, wj in enumerate(w):
        wj = int(wj)
        if wj > L:
            return None
        if cur + wj <= L:
            cur += wj
        else:
            starts.append(j)
            cur = wj
    return starts


def optimal_load(w, r: int) -> int:
    """Smallest L for which the greedy scan needs at most r groups, by binary
    search on L (Section 6; its lemma proves the result optimal).

    Search range: L* >= max(max w, ceil(W/r)), and L = ceil(W/r) + max w is
    always feasible (every closed group then holds more than W/r).
    """
    W = int(sum(int(v) for v in w))
    mx = max((int(v) for v in w), default=0)
    lo = max(mx, -(-W // r))
    hi = -(-W // r) + mx
    while lo < hi:
        mid = (lo + hi) // 2
        g = greedy_groups(w, mid)
        if g is not None and len(g) <= r:
            hi = mid
        else:
            lo = mid + 1
    return lo


def pack(w, r: int):
    """(L*, group starts): optimal load and the greedy groups under it."""
    L = optimal_load(w, r)
    return L, greedy_groups(w, L)


def pack_bruteforce(w, r: int) -> int:
    """Optimal max group load over every split of the bucket sequence into at
    most r contiguous groups, by enumerating all cut sets.  Pin for the lemma
    of Section 6 (small inputs only)."""
    n = len(w)
    pre = [0]
    for v in w:
        pre.append(pre[-1] + int(v))
    best = None
    for g in range(1, min(r, max(n, 1)) + 1):
        for cuts in itertools.combinations(range(1, n), g - 1):
            b = (0,) + cuts + (n,)
            load = max(pre[b[i + 1]] - pre[b[i]] for i in range(g))
            if best is None or load < best:
                best = load
    return 0 if best is None else best


# ----------------------------------------------------------------------------
# Children of a subproblem and the stable scatter
# ----------------------------------------------------------------------------

REG = 0    # still to be sorted (next level or base case)
FINAL = 1  # an equality bucket: every key equal, already in final order


def children(counts, eq_on: bool, r: int):
    """Split a subproblem's id range into its children, in key order.

    Reading (the paper delivers groups of buckets, Section 6; Appendix D only
    says keys equal to a splitter need no further sorting): with equality
    buckets on, an equality bucket holding at least ceil(N/r) keys is FINAL
    and weighs nothing in the grouping; all other ids keep their size.  The
    ids are grouped by ``pack`` into at most r contiguous groups; each group
    is then cut at its FINAL ids.  Every maximal run of non-FINAL ids with
    keys becomes a REG child, every FINAL id a FINAL child.  Empty pieces are
    dropped.  Returns a list of (first_id, end_id, size, kind).

    Pin: the hand-worked cases of ``tests/golden/children.txt`` (threshold
    met exactly, a final id inside a group, empty pieces after a final id,
    a large regular bucket, equality buckets off, all keys equal), which
    fail for each planted mistake (``>`` for ``>=``, no cut at a final id,
    empty pieces kept, a final id on a regular bucket).
    """
    c = [int(v) for v in counts]
    N = sum(c)
    if N == 0:
        return []
    tfin = -(-N // r)
    final = [eq_on and (i % 2 == 1) and c[i] >= tfin for i in range(len(c))]
    w = [0 if final[i] else c[i] for i in range(len(c))]
    _, starts = pack(w, r)
    ends = starts[1:] + [len(c)]
    out = []
    for gs, ge in zip(starts, ends):
        run_start = gs
        for i in range(gs, ge):
            if final[i]:
                size = sum(c[run_start:i])
                if size:
                    out.append((run_start, i, size, REG))
                out.append((i, i + 1, c[i], FINAL))
                run_start = i + 1
        size = sum(c[run_start:ge])
        if size:
            out.append((run_start, ge, size, REG))
    return out


def child_of_id(kids, nb: int) -> np.ndarray:
    """Index of the child holding each id (-1 for ids without keys)."""
    t = np.full(nb, -1, dtype=np.int64)
    for k, (a, b, _, _) in enumerate(kids):
        t[a:b] = k
    return t


def stable_partition_dest(child_idx, sizes) -> np.ndarray:
    """Destination of every element in the stable counting partition
    (Sections 4.3 and 6: each piece goes to the range its prefix sum labels).

    dst(i) = start(c_i) + #{j < i : c_j = c_i} with start the exclusive prefix
    sum of the child sizes, so each child receives its elements in input
    order.
    """
    start = exclusive_scan(sizes)
    seen = np.zeros(len(sizes), dtype=np.int64)
    dst = np.empty(len(child_idx), dtype=np.int64)
    for i, c in enumerate(np.asarray(child_idx, dtype=np.int64)):
        dst[i] = start[c] + seen[c]
        seen[c] += 1
    return dst


def level_pass(ords, splitters, eq_on: bool, r: int):
    """One level on one subproblem with given splitters: classify, histogram,
    children, stable scatter.  Returns (ids, hist, kids, permuted ords)."""
    x = np.asarray(ords, dtype=np.uint64)
    m = len(splitters) + 1
    ids = classify(x, splitters, eq_on)
    hist = histogram(ids, num_ids(m, eq_on))
    kids = children(hist, eq_on, r)
    cid = child_of_id(kids, len(hist))[ids]
    dst = stable_partition_dest(cid, [k[2] for k in kids])
    out = np.empty_like(x)
    out[dst] = x
    return ids, hist, kids, out


# ----------------------------------------------------------------------------
# Load balance (parity unpinned)
# ----------------------------------------------------------------------------

def imbalance_ok(max_group: int, n: int, r: int, b: int) -> bool:
    """Statistical sanity check from the second lemma of Section 6: with
    overpartitioning b >= 2/eps the largest group stays below (1+eps) n/r with
    high probability.  Parity unpinned (the lemma is probabilistic)."""
    eps = 2.0 / b
    return max_group <= math.ceil((1.0 + eps) * n / r)
