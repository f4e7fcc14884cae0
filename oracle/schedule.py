"""Oracle conflict graph and Cyclades schedule (TEST INFRASTRUCTURE ONLY).

Regier et al. 2018, Section IV-D (task processing): block coordinate ascent over light
sources, with threads coordinated by Cyclades (Pan et al. 2016).  Two sources conflict
when they overlap; conflicting sources are never optimised at the same time.  Each
iteration samples sources at random without replacement, splits the sample into the
connected components of the conflict graph restricted to it, and hands whole
components to threads, so overlapping sampled sources always share a thread.

Readings (the paper leaves them open):
  * "overlap" is read on the patches: s and t conflict when a box of s and a box of t
    lie on the same image and share at least one pixel (those are exactly the pairs
    whose ELBO terms share a pixel term);
  * sampling without replacement is a permutation `order` drawn by the caller, cut into
    consecutive samples of `sample_size` sources, the last one shorter;
  * a thread works through its component in sample order; the step a component's
    r-th member is taken in is called round r.  Components are independent, so
    running round r of every component side by side gives the same result as any
    thread timing, and the same result as serial block coordinate ascent in `order`.
    A round lists its sources in sample order.
Plain Python, quadratic where that is simplest; meant for small and medium inputs.
"""
from collections import deque


def conflict_graph(f):
    """Adjacency sets of the box-overlap graph of field f, by testing every pair of
    boxes: list of sets, one per source."""
    n = int(f.n_src)
    boxes = [[tuple(int(v) for v in f.boxes[k]) for k in range(int(f.patch_ptr[s]), int(f.patch_ptr[s + 1]))]
             for s in range(n)]
    adj = [set() for _ in range(n)]
    for s in range(n):
        for t in range(s + 1, n):
            hit = False
            for (ia, ra, ca, ha, wa) in boxes[s]:
                for (ib, rb, cb, hb, wb) in boxes[t]:
                    rows = min(ra + ha, rb + hb) - max(ra, rb)
                    cols = min(ca + wa, cb + wb) - max(ca, cb)
                    if ia == ib and rows > 0 and cols > 0:
                        hit = True
            if hit:
                adj[s].add(t)
                adj[t].add(s)
    return adj


def components(adj, members):
    """Connected components of the graph restricted to `members` (a list of vertices),
    by breadth-first search; each component lists its vertices in the order of
    `members`, and components come in the order of their first vertex."""
    inside = {v: i for i, v in enumerate(members)}
    seen = set()
    comps = []
    for v in members:
        if v in seen:
            continue
        seen.add(v)
        found = [v]
        queue = deque([v])
        while queue:
            u = queue.popleft()
            for w in adj[u]:
                if w in inside and w not in seen:
                    seen.add(w)
                    found.append(w)
                    queue.append(w)
        comps.append(sorted(found, key=inside.get))
    return comps


def cyclades_rounds(adj, order, sample_size):
    """Cyclades schedule as a list of rounds (lists of sources) and the number of
    components over all samples."""
    rounds = []
    n_comp = 0
    for b0 in range(0, len(order), sample_size):
        sample = [int(v) for v in order[b0:b0 + sample_size]]
        comps = components(adj, sample)
        n_comp += len(comps)
        depth = max(len(c) for c in comps)
        pos = {v: i for i, v in enumerate(sample)}
        for r in range(depth):
            rnd = [c[r] for c in comps if len(c) > r]
            rounds.append(sorted(rnd, key=pos.get))
    return rounds, n_comp


def adjacency_sets(adj_ptr, adj):
    """CSR (row pointers, neighbours) to a list of sets."""
    return [set(int(t) for t in adj[adj_ptr[s]:adj_ptr[s + 1]]) for s in range(len(adj_ptr) - 1)]
