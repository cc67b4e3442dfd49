"""Ring and double-binary-tree topologies (Section II-C, Communication
Channels; Section V-E for the direction of the ring).

Ring: rank ``p`` sends to ``(p + 1) % R`` and receives from ``(p - 1) % R``
(the ReduceScatter description names ``(i+1)%k`` as the destination).  A
set may give its channels other ring orders (``channel_ring``); the step
tables then apply to ring positions instead of rank numbers.

Double binary tree: the paper states only its properties -- no rank is an
inner node of both trees, at most one rank is a leaf in both, and the second
tree mirrors the first for an even rank count or shifts it by one position
for an odd count.  Construction adopted (a reading; the paper gives none):

* Tree A over positions ``0 .. R-1`` (position == rank).  Position 0 is the
  root and has a single child, ``P`` = the largest power of two below ``R``.
  A position ``q >= 1`` whose lowest set bit is ``b`` has parent
  ``(q - b) | 2b``, or ``q - b`` when that value is ``>= R``.
  Its children (only when ``b > 1``) are ``q - b/2`` and the first of
  ``q + b/2, q + b/4, ..., q + 1`` that is ``< R``.
* Tree B: position ``q`` holds rank ``R-1-q`` when ``R`` is even, rank
  ``(q + 1) % R`` when ``R`` is odd.

Child order (first, second) fixes the reduction order at an inner node.
"""
from __future__ import annotations


def ring_next(p: int, nranks: int) -> int:
    return (p + 1) % nranks


def ring_prev(p: int, nranks: int) -> int:
    return (p - 1) % nranks


def channel_ring(nranks: int, channel: int, rings=None) -> list[int]:
    """The ring order of a channel (Section II-C: each channel has its own
    logical ring, set up at initialisation).  ``rings`` is None (every
    channel on the identity ring, rank p sending to p + 1) or a list of ring
    orders, each listing the ranks in ring order; channel c follows
    ``rings[c % len(rings)]`` (a reading: the paper does not say how channels
    map to rings).  Returns the order after checking it is a permutation."""
    if rings is None:
        return list(range(nranks))
    order = [int(r) for r in rings[channel % len(rings)]]
    if sorted(order) != list(range(nranks)):
        raise ValueError("a ring order must be a permutation of the ranks")
    return order


def _lowbit(q: int) -> int:
    return q & -q


def _positions_tree(nranks: int):
    """parent[q], children[q] over positions of tree A."""
    parent = [-1] * nranks
    children: list[list[int]] = [[] for _ in range(nranks)]
    if nranks == 1:
        return parent, children
    top = 1
    while top * 2 < nranks:
        top *= 2
    for q in range(1, nranks):
        b = _lowbit(q)
        up = (q - b) | (2 * b)
        if up >= nranks:
            up = q - b
        parent[q] = up
    # children derived from the stated rule (and cross-checked against parent[])
    children[0] = [top]
    for q in range(1, nranks):
        b = _lowbit(q)
        if b > 1:
            kids = [q - b // 2]
            h = b // 2
            while h >= 1:
                if q + h < nranks:
                    kids.append(q + h)
                    break
                h //= 2
            children[q] = kids
    for q in range(nranks):
        for c in children[q]:
            if parent[c] != q:
                raise AssertionError("tree construction inconsistent")
    return parent, children


def double_binary_tree(nranks: int, ranks_per_node: int = 1):
    """Returns [treeA, treeB]; each is dict(parent=[...], children=[[...]...]) indexed by rank.

    ranks_per_node > 1: chains within a node, the double binary tree across
    nodes (see chain_tree)."""
    if ranks_per_node > 1:
        return chain_tree(nranks, ranks_per_node)
    pparent, pchildren = _positions_tree(nranks)
    trees = []
    for which in (0, 1):
        if which == 0:
            rank_at = list(range(nranks))
        elif nranks % 2 == 0:
            rank_at = [nranks - 1 - q for q in range(nranks)]
        else:
            rank_at = [(q + 1) % nranks for q in range(nranks)]
        parent = [-1] * nranks
        children: list[list[int]] = [[] for _ in range(nranks)]
        for q in range(nranks):
            r = rank_at[q]
            parent[r] = -1 if pparent[q] < 0 else rank_at[pparent[q]]
            children[r] = [rank_at[c] for c in pchildren[q]]
        root = rank_at[0]
        trees.append(dict(parent=parent, children=children, root=root))
    return trees


def tree_depth(tree) -> int:
    parent = tree["parent"]
    best = 0
    for r in range(len(parent)):
        d, x = 0, r
        while parent[x] >= 0:
            x = parent[x]
            d += 1
        best = max(best, d)
    return best


def chain_tree(nranks: int, ranks_per_node: int):
    """Trees that branch only across nodes and form a chain within a node
    (Section V-E, tree AllReduce).  Ranks n*P .. n*P+P-1 form node n
    (P = ranks_per_node, which must divide nranks).  Reading adopted (the
    paper does not say where the inter-node links attach):

    * the nodes form the double binary tree over node indices;
    * within node n the chain runs, for tree A, local 0 <- local 1 <- ... <-
      local P-1 (local 0 is the head) and, for tree B, the reverse (local P-1
      is the head);
    * a node's head sends to its parent node; the parent node takes its first
      node child at its head and its second at the next rank of its chain,
      so no rank has more than two children;
    * at a rank the chain child comes first, then the node child.
    """
    P = ranks_per_node
    if P < 1 or nranks % P:
        raise ValueError("ranks_per_node must divide nranks")
    N = nranks // P
    node_trees = double_binary_tree(N)
    trees = []
    for which in (0, 1):
        nt = node_trees[which]
        order = [[n * P + k for k in (range(P) if which == 0 else range(P - 1, -1, -1))] for n in range(N)]
        parent = [-1] * nranks
        children: list[list[int]] = [[] for _ in range(nranks)]
        for n in range(N):
            for i in range(1, P):
                parent[order[n][i]] = order[n][i - 1]
                children[order[n][i - 1]].append(order[n][i])
        for n in range(N):
            for j, m in enumerate(nt["children"][n]):
                at = order[n][j]
                parent[order[m][0]] = at
                children[at].append(order[m][0])
        trees.append(dict(parent=parent, children=children, root=order[nt["root"]][0]))
    return trees

