"""Small structured graphs (tuple lists) with closed-form hop distances.

Input construction only: each builder returns (edges int64[m][2], n) and,
where useful, the closed-form distance function used as the expected level.
"""
import itertools

import numpy as np


def as_edges(pairs):
    return np.array(list(pairs), dtype=np.int64).reshape(-1, 2)


def path(n):
    return as_edges((i, i + 1) for i in range(n - 1)), n


def path_dist(n, r):
    return np.abs(np.arange(n) - r)


def star(leaves):
    return as_edges((0, i) for i in range(1, leaves + 1)), leaves + 1


def star_dist(leaves, r):
    n = leaves + 1
    d = np.full(n, 2 if r != 0 else 1, dtype=np.int64)
    d[0] = 0 if r == 0 else 1
    d[r] = 0
    return d


def grid(a, b):
    def vid(i, j):
        return i * b + j
    pairs = []
    for i in range(a):
        for j in range(b):
            if i + 1 < a:
                pairs.append((vid(i, j), vid(i + 1, j)))
            if j + 1 < b:
                pairs.append((vid(i, j), vid(i, j + 1)))
    return as_edges(pairs), a * b


def grid_dist(a, b, r):
    ri, rj = divmod(r, b)
    ii, jj = np.divmod(np.arange(a * b), b)
    return np.abs(ii - ri) + np.abs(jj - rj)


def cycle(n):
    return as_edges((i, (i + 1) % n) for i in range(n)), n


def cycle_dist(n, r):
    d = np.abs(np.arange(n) - r)
    return np.minimum(d, n - d)


def complete(n):
    return as_edges(itertools.combinations(range(n), 2)), n


def complete_dist(n, r):
    d = np.ones(n, dtype=np.int64)
    d[r] = 0
    return d


def binary_tree(depth):
    """Complete binary tree in heap order (children of i: 2i+1, 2i+2)."""
    n = (1 << (depth + 1)) - 1
    return as_edges((i, (i - 1) // 2) for i in range(1, n)), n


def binary_tree_dist(n, r):
    """Tree distance through the lowest common ancestor in heap order."""
    def depth(x):
        return (x + 1).bit_length() - 1
    out = np.empty(n, dtype=np.int64)
    for v in range(n):
        a, b = r, v
        while depth(a) > depth(b):
            a = (a - 1) // 2
        while depth(b) > depth(a):
            b = (b - 1) // 2
        while a != b:
            a, b = (a - 1) // 2, (b - 1) // 2
        out[v] = depth(r) + depth(v) - 2 * depth(a)
    return out


def disjoint_union(*parts):
    """parts: (edges, n) pairs; returns the union with shifted ids and offsets."""
    out, offs, base = [], [], 0
    for e, n in parts:
        out.append(e + base)
        offs.append(base)
        base += n
    return np.concatenate(out).reshape(-1, 2), base, offs


def broom(path_len, leaves):
    """A path 0 .. path_len-1 whose last vertex is the centre of a star; each
    leaf path_len + j also holds a pendant vertex path_len + leaves + j."""
    p, l = path_len, leaves
    pairs = [(i, i + 1) for i in range(p - 1)] + [(p - 1, p + j) for j in range(l)] + \
            [(p + j, p + l + j) for j in range(l)]
    return as_edges(pairs), p + 2 * l


def broom_dist(path_len, leaves):
    """Levels from root 0: i on the path, path_len on a leaf, path_len + 1 on a
    pendant vertex."""
    return np.concatenate([np.arange(path_len), np.full(leaves, path_len),
                           np.full(leaves, path_len + 1)]).astype(np.int32)


def random_graph(rng, n, p):
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].size) < p
    return np.stack([iu[0][keep], iu[1][keep]], axis=1).astype(np.int64), n


def long_path_relabelled(n, seed):
    """A path of n vertices under a random relabelling; returns edges, n, order."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    e = np.stack([perm[:-1], perm[1:]], axis=1).astype(np.int64)
    return e, n, perm
