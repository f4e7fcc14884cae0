"""Conflict graph and Cyclades schedule (Section IV-D): the oracle pinned against
library routines, brute force and closed-form special cases, then the library's host
schedule compared with it exactly.  No GPU: celeste_cyclades_batches is host code."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from oracle import schedule as Sch


def random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    adj = [set() for _ in range(n)]
    for s in range(n):
        for t in range(s + 1, n):
            if rng.random() < p:
                adj[s].add(t)
                adj[t].add(s)
    return adj


def to_csr(adj, repeats=False, rng=None):
    ptr, out = [0], []
    for row in adj:
        r = sorted(row)
        if repeats and r:
            r = r + list(rng.choice(r, size=len(r)))   # repeated entries are allowed
            rng.shuffle(r)
        out += r
        ptr.append(len(out))
    return np.array(ptr, np.int32), np.array(out, np.int32)


def rounds_of(bp, bs):
    return [bs[bp[b]:bp[b + 1]].tolist() for b in range(len(bp) - 1)]


# ---------------------------------------------------------------- oracle pins

@pytest.mark.parametrize("n,p,seed", [(1, 0.0, 1), (12, 0.2, 2), (40, 0.05, 3), (40, 0.3, 4), (80, 0.03, 5)])
def test_components_match_scipy(n, p, seed):
    adj = random_graph(n, p, seed)
    rng = np.random.default_rng(seed + 100)
    members = [int(v) for v in rng.permutation(n)[:max(1, n // 2)]]
    comps = Sch.components(adj, members)
    # scipy's connected components of the induced subgraph
    idx = {v: i for i, v in enumerate(members)}
    rows, cols = [], []
    for v in members:
        for w in adj[v]:
            if w in idx:
                rows.append(idx[v])
                cols.append(idx[w])
    g = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(len(members), len(members)))
    k, lab = connected_components(g, directed=False)
    assert len(comps) == k
    for c in comps:
        labs = {lab[idx[v]] for v in c}
        assert len(labs) == 1 and np.sum(lab == labs.pop()) == len(c)
        assert c == sorted(c, key=idx.get)                      # members in sample order
    firsts = [idx[c[0]] for c in comps]
    assert firsts == sorted(firsts)                             # components by first member


def test_special_cases():
    n = 7
    order = [3, 0, 6, 2, 5, 1, 4]
    empty = [set() for _ in range(n)]
    path = [set() for _ in range(n)]
    for s in range(n - 1):
        path[s].add(s + 1)
        path[s + 1].add(s)
    full = [set(range(n)) - {s} for s in range(n)]
    # sample size 1: fully serial, in order, one component per source
    assert Sch.cyclades_rounds(full, order, 1) == ([[v] for v in order], n)
    # no conflicts, one sample: a single round holding the sample in order
    assert Sch.cyclades_rounds(empty, order, n) == ([order], n)
    # path and complete graph, one sample: one component, serial in order
    assert Sch.cyclades_rounds(path, order, n) == ([[v] for v in order], 1)
    assert Sch.cyclades_rounds(full, order, 100) == ([[v] for v in order], 1)
    # two disjoint triangles, interleaved in the order: three rounds of two
    tri = [set() for _ in range(6)]
    for a, b in [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)]:
        tri[a].add(b)
        tri[b].add(a)
    assert Sch.cyclades_rounds(tri, [0, 3, 1, 4, 2, 5], 6) == ([[0, 3], [1, 4], [2, 5]], 2)
    # ragged final sample: samples {0,1,2} and {3}; the path 0-1-2 links all of the first
    path4 = [{1}, {0, 2}, {1, 3}, {2}]
    assert Sch.cyclades_rounds(path4, [0, 1, 2, 3], 3) == ([[0], [1], [2], [3]], 2)
    assert Sch.cyclades_rounds(path4, [0, 2, 1, 3], 2) == ([[0, 2], [1, 3]], 4)


@pytest.mark.parametrize("n,p,B,seed", [(30, 0.1, 7, 11), (50, 0.04, 16, 12), (60, 0.2, 5, 13), (25, 0.0, 4, 14)])
def test_rounds_are_a_valid_serialisation(n, p, B, seed):
    """Invariants that make one epoch equal serial block coordinate ascent in `order`:
    every source once, samples in order, no conflict inside a round, and of two
    conflicting sources of one sample the earlier one in an earlier round."""
    adj = random_graph(n, p, seed)
    order = [int(v) for v in np.random.default_rng(seed).permutation(n)]
    rounds, n_comp = Sch.cyclades_rounds(adj, order, B)
    flat = [v for r in rounds for v in r]
    assert sorted(flat) == list(range(n))
    where = {v: i for i, r in enumerate(rounds) for v in r}
    sample = {v: i // B for i, v in enumerate(order)}
    pos = {v: i for i, v in enumerate(order)}
    for r in rounds:
        assert len({sample[v] for v in r}) == 1
        assert r == sorted(r, key=pos.get)
        for a in r:
            assert not (adj[a] & set(r))
    for a in range(n):
        for b in adj[a]:
            if sample[a] == sample[b] and pos[a] < pos[b]:
                assert where[a] < where[b]
    assert [sample[r[0]] for r in rounds] == sorted(sample[r[0]] for r in rounds)
    assert n_comp >= (n + B - 1) // B


def test_conflict_graph_brute_force_pixels(synth):
    """Adjacency from box intersection equals adjacency from shared pixel sets."""
    f = synth.tiny(S=6, n_bands=2, size=31, side=9, seed=61)
    adj = Sch.conflict_graph(f)
    pix = []
    for s in range(f.n_src):
        cells = set()
        for k in range(f.patch_ptr[s], f.patch_ptr[s + 1]):
            i, r0, c0, h, w = (int(v) for v in f.boxes[k])
            cells |= {(i, r, c) for r in range(r0, r0 + h) for c in range(c0, c0 + w)}
        pix.append(cells)
    for s in range(f.n_src):
        assert adj[s] == {t for t in range(f.n_src) if t != s and pix[s] & pix[t]}
    assert any(adj)   # the case has conflicts


# ---------------------------------------------------------------- library vs oracle

@pytest.mark.parametrize("n,p,B,seed", [(1, 0.0, 1, 21), (2, 1.0, 2, 22), (17, 0.15, 4, 23), (64, 0.05, 64, 24),
                                        (64, 0.05, 10, 25), (200, 0.02, 37, 26), (300, 0.01, 1000, 27),
                                        (90, 0.5, 9, 28)])
def test_library_schedule_equals_oracle(n, p, B, seed):
    from paper_1801_10277_amd import binding as Bd
    adj = random_graph(n, p, seed)
    rng = np.random.default_rng(seed)
    ptr, nbr = to_csr(adj, repeats=(seed % 2 == 0), rng=rng)
    order = rng.permutation(n).astype(np.int32)
    bp, bs, nc = Bd.cyclades_batches(ptr, nbr, order, B)
    rounds, n_comp = Sch.cyclades_rounds(adj, order, B)
    assert rounds_of(bp, bs) == rounds
    assert nc == n_comp


def test_library_schedule_on_field_graph(synth):
    from paper_1801_10277_amd import binding as Bd
    f = synth.region_16src()
    adj = Sch.conflict_graph(f)
    ptr, nbr = to_csr(adj)
    for B, seed in [(4, 1), (8, 2), (f.n_src, 3)]:
        order = np.random.default_rng(seed).permutation(f.n_src).astype(np.int32)
        bp, bs, nc = Bd.cyclades_batches(ptr, nbr, order, B)
        assert (rounds_of(bp, bs), nc) == Sch.cyclades_rounds(adj, order, B)


def test_library_schedule_edge_cases():
    from paper_1801_10277_amd import binding as Bd
    bp, bs, nc = Bd.cyclades_batches(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32), 3)
    assert bp.tolist() == [0] and nc == 0
    ptr = np.array([0, 1, 2, 2], np.int32)
    nbr = np.array([1, 0], np.int32)
    good = np.array([2, 0, 1], np.int32)
    bp, bs, nc = Bd.cyclades_batches(ptr, nbr, good, 3)
    assert rounds_of(bp, bs) == [[2, 0], [1]] and nc == 2
    bad_cases = [
        (ptr, nbr, np.array([0, 0, 1], np.int32), 3),        # not a permutation
        (ptr, nbr, np.array([0, 1, 3], np.int32), 3),        # out of range
        (ptr, nbr, good, 0),                                  # empty samples
        (np.array([0, 2, 1, 2], np.int32), nbr, good, 3),    # decreasing row pointer
        (np.array([1, 1, 2, 2], np.int32), nbr, good, 3),    # row pointer not from 0
        (ptr, np.array([1, 3], np.int32), good, 3),          # neighbour out of range
    ]
    for a, b, o, B in bad_cases:
        with pytest.raises(Bd.CelesteError) as e:
            Bd.cyclades_batches(a, b, o, B)
        assert e.value.code == Bd.CELESTE_EINVAL
