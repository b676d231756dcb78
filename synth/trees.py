"""Rooted binary trees for synthetic workloads.

Node numbering used throughout the project: tips are 0..N-1, internal nodes
are N..2N-2 and the root is 2N-2.  Branch c is the edge above non-root node c,
so a tree has 2N-2 branches and ``t[c]`` is its length (``t[root]`` is unused
and kept at 0).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Tree:
    n_tips: int
    parent: np.ndarray      # int64 [2N-1]; parent[root] == -1
    children: np.ndarray    # int64 [2N-1, 2]; -1 for tips

    @property
    def n_nodes(self) -> int:
        return 2 * self.n_tips - 1

    @property
    def root(self) -> int:
        return 2 * self.n_tips - 2

    def validate(self) -> None:
        N = self.n_tips
        assert self.parent.shape == (2 * N - 1,) and self.children.shape == (2 * N - 1, 2)
        assert self.parent[self.root] == -1
        for v in range(2 * N - 1):
            if v < N:
                assert (self.children[v] == -1).all()
            else:
                for c in self.children[v]:
                    assert self.parent[c] == v


def _relabel(n_tips: int, kids: dict, root_key) -> Tree:
    """Give tips 0..N-1 (left-to-right) and internal nodes N..2N-2 in post-order (root last)."""
    N = n_tips
    parent = np.full(2 * N - 1, -1, dtype=np.int64)
    children = np.full((2 * N - 1, 2), -1, dtype=np.int64)
    label = {}
    next_tip, next_int = 0, N
    stack = [(root_key, False)]
    while stack:
        key, done = stack.pop()
        ch = kids.get(key)
        if ch is None:
            label[key] = next_tip
            next_tip += 1
        elif done:
            label[key] = next_int
            next_int += 1
            children[label[key]] = [label[ch[0]], label[ch[1]]]
            parent[label[ch[0]]] = label[key]
            parent[label[ch[1]]] = label[key]
        else:
            stack.append((key, True))
            stack.append((ch[1], False))
            stack.append((ch[0], False))
    tree = Tree(N, parent, children)
    tree.validate()
    return tree


def yule_tree(n_tips: int, rng: np.random.Generator) -> Tree:
    """Forward Yule topology: start from a root with two lineages and split a
    uniformly chosen lineage until there are ``n_tips`` lineages."""
    if n_tips < 2:
        raise ValueError("need at least two tips")
    kids = {0: (1, 2)}
    lineages = [1, 2]
    nxt = 3
    while len(lineages) < n_tips:
        i = int(rng.integers(len(lineages)))
        v = lineages[i]
        kids[v] = (nxt, nxt + 1)
        lineages[i] = nxt
        lineages.append(nxt + 1)
        nxt += 2
    return _relabel(n_tips, kids, 0)


def balanced_tree(n_tips: int) -> Tree:
    """Fully balanced topology (n_tips a power of two gives a complete tree)."""
    counter = [1]

    def build(n, kids):
        key = counter[0]
        counter[0] += 1
        if n == 1:
            return key
        left = build(n // 2, kids)
        right = build(n - n // 2, kids)
        kids[key] = (left, right)
        return key

    kids = {}
    root = build(n_tips, kids)
    return _relabel(n_tips, kids, root)


def caterpillar_tree(n_tips: int) -> Tree:
    """Maximally unbalanced (ladder) topology: height N-1."""
    kids = {}
    key = 0
    nxt = 1
    for _ in range(n_tips - 1):
        kids[key] = (nxt, nxt + 1)
        key = nxt + 1
        nxt += 2
    return _relabel(n_tips, kids, 0)


def two_taxon_tree() -> Tree:
    return _relabel(2, {0: (1, 2)}, 0)


def exponential_branches(tree: Tree, mean: float, rng: np.random.Generator) -> np.ndarray:
    """Every branch (both root branches included) iid Exponential with the given mean."""
    t = rng.exponential(mean, size=tree.n_nodes)
    t[tree.root] = 0.0
    return t
