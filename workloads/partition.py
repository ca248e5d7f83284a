"""Non-box partitions of the structured meshes (problem descriptions only).

Two level-1 divisions that box grids cannot produce, and a grouping of
subdomains for the higher levels:

* ``kd_partition``: recursive bisection of the element box, each part cut
  across its longest axis at a seeded position; sibling parts are cut
  independently, so cut planes end on other parts' faces (T-junctions).
* ``grown_partition``: subdomains grown on the element face graph from
  well-spread seed elements, smallest part first, so subdomains have
  staircase faces and neighbours can touch in several separate patches.
* ``grown_groups``: the same growth on the graph of subdomains that share an
  element face, for the level-l divisions of level-(l-1) subdomains (the
  paper divides its pseudo-meshes with a graph partitioner).

Every part is connected.  Seeds come from ``numpy.random.default_rng(seed)``.
"""

from __future__ import annotations

from typing import List, Sequence

import numpy as np


def _elem_index(n_el: Sequence[int]) -> np.ndarray:
    """Element ids of the grid as an array indexed [z, y, x] (or [y, x])."""
    return np.arange(int(np.prod(n_el))).reshape(tuple(n_el)[::-1])


def kd_partition(n_el: Sequence[int], n_parts: int, seed: int, jitter: float = 0.15) -> np.ndarray:
    """Element -> part by recursive bisection.  A part of k subdomains is cut
    across its longest axis (lowest axis on ties) at a fraction
    floor(k/2)/k + U(-jitter, jitter) of its extent (at least one element on
    each side); parts are numbered depth first, the lower side first."""
    rng = np.random.default_rng(seed)
    dim = len(n_el)
    out = np.full(tuple(n_el)[::-1], -1, dtype=np.int32)
    counter = [0]

    def split(lo: List[int], hi: List[int], k: int) -> None:
        if k == 1:
            sl = tuple(slice(lo[d], hi[d]) for d in reversed(range(dim)))
            out[sl] = counter[0]
            counter[0] += 1
            return
        ext = [hi[d] - lo[d] for d in range(dim)]
        ax = int(np.argmax(ext))
        if ext[ax] < 2:
            raise ValueError("part too small to cut")
        k1 = k // 2
        frac = k1 / k + rng.uniform(-jitter, jitter)
        pos = lo[ax] + int(round(frac * ext[ax]))
        pos = min(max(pos, lo[ax] + 1), hi[ax] - 1)
        hi1 = list(hi); hi1[ax] = pos
        lo2 = list(lo); lo2[ax] = pos
        split(list(lo), hi1, k1)
        split(lo2, list(hi), k - k1)

    split([0] * dim, [int(n) for n in n_el], n_parts)
    return out.ravel().astype(np.int32)


def _grid_neighbours(n_el: Sequence[int]) -> List[np.ndarray]:
    """Pairs (a, b) of face-adjacent elements, one array [m, 2] per axis."""
    idx = _elem_index(n_el)
    dim = len(n_el)
    pairs = []
    for d in range(dim):
        ax = dim - 1 - d                     # array axis of grid axis d
        a = np.take(idx, np.arange(idx.shape[ax] - 1), axis=ax).ravel()
        b = np.take(idx, np.arange(1, idx.shape[ax]), axis=ax).ravel()
        pairs.append(np.stack([a, b], axis=1))
    return pairs


def _csr(n: int, edges: np.ndarray):
    """Symmetric adjacency (CSR ptr, adj) of an undirected edge list."""
    e = np.concatenate([edges, edges[:, ::-1]])
    order = np.lexsort((e[:, 1], e[:, 0]))
    e = e[order]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, e[:, 0] + 1, 1)
    return np.cumsum(ptr), e[:, 1].astype(np.int64)


def _bfs_labels(n: int, ptr: np.ndarray, adj: np.ndarray, seeds: np.ndarray):
    """Multi-source breadth-first search: graph distance to the nearest seed
    and the label (seed index) of the nearest one, ties to the lower label."""
    dist = np.full(n, -1, dtype=np.int64)
    lab = np.full(n, -1, dtype=np.int64)
    dist[seeds] = 0
    lab[seeds] = np.arange(len(seeds))
    front = np.asarray(seeds, dtype=np.int64)
    d = 0
    while len(front):
        d += 1
        cnt = ptr[front + 1] - ptr[front]
        src = np.repeat(front, cnt)
        nbr = adj[np.repeat(ptr[front], cnt) + (np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt))]
        keep = dist[nbr] < 0
        nbr, src = nbr[keep], src[keep]
        if not len(nbr):
            break
        order = np.lexsort((lab[src], nbr))
        nbr, src = nbr[order], src[order]
        first = np.ones(len(nbr), dtype=bool)
        first[1:] = nbr[1:] != nbr[:-1]
        nbr, src = nbr[first], src[first]
        dist[nbr] = d
        lab[nbr] = lab[src]
        front = nbr
    return dist, lab


def _grow(n: int, ptr: np.ndarray, adj: np.ndarray, n_parts: int, seed: int) -> np.ndarray:
    """Balanced graph growing: seeds are the first vertex drawn uniformly and
    then, one at a time, a vertex farthest from the seeds so far (lowest index
    on ties); the smallest part (lowest index on ties) then claims the next
    unclaimed vertex of its breadth-first frontier until every vertex is
    claimed.  Each part is connected."""
    import heapq
    from collections import deque
    if n_parts > n:
        raise ValueError("more parts than vertices")
    rng = np.random.default_rng(seed)
    seeds = [int(rng.integers(n))]
    dist, _ = _bfs_labels(n, ptr, adj, np.array(seeds))
    if np.any(dist < 0):
        raise ValueError("graph is not connected")
    for _ in range(n_parts - 1):
        s = int(np.argmax(dist))
        seeds.append(s)
        d2, _ = _bfs_labels(n, ptr, adj, np.array([s]))
        dist = np.minimum(dist, d2)
    lab = np.full(n, -1, dtype=np.int32)
    front = [deque() for _ in range(n_parts)]
    heap = []
    for p, s in enumerate(seeds):
        lab[s] = p
        front[p].extend(adj[ptr[s]:ptr[s + 1]].tolist())
        heapq.heappush(heap, (1, p))
    left = n - n_parts
    while left and heap:
        size, p = heapq.heappop(heap)
        f = front[p]
        while f and lab[f[0]] >= 0:
            f.popleft()
        if not f:
            continue                      # enclosed: this part stops growing
        v = f.popleft()
        lab[v] = p
        left -= 1
        f.extend(adj[ptr[v]:ptr[v + 1]].tolist())
        heapq.heappush(heap, (size + 1, p))
    if left:
        raise ValueError("graph growing left vertices unclaimed")
    return lab


def grown_partition(n_el: Sequence[int], n_parts: int, seed: int) -> np.ndarray:
    """Element -> part: balanced growth on the element face graph."""
    n = int(np.prod(n_el))
    ptr, adj = _csr(n, np.concatenate(_grid_neighbours(n_el)))
    return _grow(n, ptr, adj, n_parts, seed)


def grown_groups(n_el: Sequence[int], elem_to_sub: np.ndarray, n_groups: int, seed: int) -> np.ndarray:
    """Subdomain -> group: balanced growth on the graph of subdomains that
    share an element face."""
    ns = int(elem_to_sub.max()) + 1
    e = np.concatenate(_grid_neighbours(n_el))
    s = elem_to_sub[e]
    s = s[s[:, 0] != s[:, 1]]
    s = np.unique(np.sort(s, axis=1), axis=0)
    ptr, adj = _csr(ns, s)
    return _grow(ns, ptr, adj, n_groups, seed)
