"""Pins of the chain-within-node / double-binary-tree-across-nodes topology
(Section V-E, tree AllReduce: branching only across nodes) and of the tree
schedule and fold on it: structural properties that any such tree must have,
the two extreme cases (one rank per node is the plain double binary tree, one
node is a single chain), brute force on integer inputs, and the closed-form
fold against the step simulation."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from oracle import folds
from oracle import simulate as sim
from oracle import topology as topo

SHAPES = [(4, 2), (8, 2), (8, 4), (12, 3), (16, 2), (16, 4), (16, 8), (6, 3)]


def _reaches_root(tree, r):
    seen = set()
    while tree["parent"][r] >= 0:
        assert r not in seen
        seen.add(r)
        r = tree["parent"][r]
    return r == tree["root"]


@pytest.mark.parametrize("R,P", SHAPES)
def test_structure(R, P):
    N = R // P
    node_trees = topo.double_binary_tree(N)
    for t, tree in enumerate(topo.double_binary_tree(R, P)):
        parent, children = tree["parent"], tree["children"]
        assert sum(1 for p in parent if p < 0) == 1
        for r in range(R):
            assert _reaches_root(tree, r)
            assert len(children[r]) <= 2
            for c in children[r]:
                assert parent[c] == r
        # within a node: a chain in local order (tree A) or reversed (tree B)
        for n in range(N):
            local = [n * P + k for k in range(P)]
            if t == 1:
                local = local[::-1]
            for i in range(1, P):
                assert parent[local[i]] == local[i - 1]
            # only the head links to another node
            for i in range(1, P):
                assert parent[local[i]] // P == n
        # across nodes: the heads' links project onto the node-level tree
        for n in range(N):
            head = n * P if t == 0 else n * P + P - 1
            pn = node_trees[t]["parent"][n]
            if pn < 0:
                assert parent[head] < 0
            else:
                assert parent[head] // P == pn
        # a rank's chain child comes before its node child
        for r in range(R):
            kids = children[r]
            if len(kids) == 2:
                assert kids[0] // P == r // P and kids[1] // P != r // P


def test_one_rank_per_node_is_the_plain_double_binary_tree():
    for R in (2, 4, 7, 8, 16):
        a = topo.double_binary_tree(R, 1)
        b = topo.double_binary_tree(R)
        assert a == b


def test_one_node_is_a_single_chain():
    R = 6
    ta, tb = topo.chain_tree(R, R)
    assert ta["root"] == 0 and ta["parent"] == [-1, 0, 1, 2, 3, 4]
    assert tb["root"] == 5 and tb["parent"] == [1, 2, 3, 4, 5, -1]


@pytest.mark.parametrize("R,P", SHAPES)
def test_schedule_equals_definition_on_integers(R, P):
    for n in (1, 17, 1000):
        xs = si.rank_inputs(3, R, "int32", n, lo=-2**20, hi=2**20, extra=R * 100 + P + n)
        want = defs.allreduce(xs, "sum", "int32")
        got = sim.run("allreduce", xs, dtype="int32", nchannels=3, chunk_bytes=64, algo="tree",
                      ranks_per_node=P)
        for g, w in zip(got, want):
            np.testing.assert_array_equal(g, w)


@pytest.mark.parametrize("R,P", [(8, 2), (16, 4), (12, 3)])
@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
def test_fold_equals_schedule(R, P, dtype):
    xs = si.rank_inputs(3, R, dtype, 3001, extra=R + P)
    got = sim.run("allreduce", xs, dtype=dtype, nchannels=4, chunk_bytes=256, algo="tree", ranks_per_node=P)
    want = folds.tree_allreduce(xs, "sum", dtype, 4, ranks_per_node=P)
    for g in got:
        np.testing.assert_array_equal(g.view(np.uint8), want.view(np.uint8))
    # the chain changes the association order: not the plain tree's fold
    plain = folds.tree_allreduce(xs, "sum", dtype, 4)
    assert not np.array_equal(plain.view(np.uint8), want.view(np.uint8))


def test_two_ranks_per_node_worked_case():
    # R = 4, P = 2: nodes {0,1}, {2,3}; node tree A: node 0 root with child 1.
    # Tree A: chain 0 <- 1 and 2 <- 3; node 1's head (2) attaches at node 0's
    # head (0), after its chain child 1.
    ta, tb = topo.chain_tree(4, 2)
    assert ta["parent"] == [-1, 0, 0, 2] and ta["children"][0] == [1, 2] and ta["root"] == 0
    # Tree B: node tree B mirrors (node 1 is the root); chains reversed:
    # 1 <- 0, 3 <- 2; node 0's head (1) attaches at node 1's head (3).
    assert tb["parent"] == [1, 3, 3, -1] and tb["children"][3] == [2, 1] and tb["root"] == 3
