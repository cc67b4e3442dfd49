"""Pins of the oracle's per-channel ring orders (Section II-C: every channel
has its own ring, set up at initialisation).

The main pin is a relabelling: following ring order pi is the identity ring
with rank pi[q] renamed q.  So the schedule simulation on ring pi must equal
the identity-ring simulation -- itself pinned by the paper's step tables and
the brute-force definitions -- run on the relabelled inputs, with its outputs
relabelled back.  The closed-form folds with rings are then checked against
the simulation over several channels and rings, and a wrong ring order (a
plausible slip) must change the bits.
"""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from oracle import folds
from oracle import simulate as sim
from oracle import topology as topo


def _perm(R, seed):
    rng = np.random.default_rng([0x5EED, 77, R, seed])
    return [int(x) for x in rng.permutation(R)]


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


def test_channel_ring_identity_and_checks():
    assert topo.channel_ring(5, 3) == [0, 1, 2, 3, 4]
    assert topo.channel_ring(4, 5, [[0, 1, 2, 3], [3, 1, 0, 2]]) == [3, 1, 0, 2]
    with pytest.raises(ValueError):
        topo.channel_ring(4, 0, [[0, 1, 1, 3]])
    with pytest.raises(ValueError):
        topo.channel_ring(4, 0, [[0, 1, 2]])


@pytest.mark.parametrize("R", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("seed", [1, 2])
def test_ring_order_is_a_relabelling(R, seed):
    pi = _perm(R, seed)
    inv = [pi.index(r) for r in range(R)]
    n = 61 * R
    xs = si.rank_inputs(9, R, "float32", n, extra=seed)  # N(0,1): the association order shows in the bits
    ys = [xs[pi[q]] for q in range(R)]
    kw = dict(dtype="float32", nchannels=1, chunk_bytes=48)
    # AllReduce: every rank holds the same fold
    got = sim.run("allreduce", xs, rings=[pi], **kw)
    want = sim.run("allreduce", ys, **kw)
    for q in range(R):
        assert np.array_equal(_bits(got[pi[q]]), _bits(want[q]))
    # ReduceScatter: rank pi[q] ends with its own block, relabelled as q's
    m = n // R
    blocks = lambda x: [x[j * m:(j + 1) * m] for j in range(R)]  # noqa: E731
    ys_rs = [np.concatenate([blocks(xs[pi[q]])[pi[j]] for j in range(R)]) for q in range(R)]
    got = sim.run("reducescatter", xs, rings=[pi], **kw)
    want = sim.run("reducescatter", ys_rs, **kw)
    for q in range(R):
        assert np.array_equal(_bits(got[pi[q]]), _bits(want[q]))
    # AllGather: blocks are laid out by rank number
    got = sim.run("allgather", xs, rings=[pi], **kw)
    want = sim.run("allgather", ys, **kw)
    for q in range(R):
        g = np.asarray(got[pi[q]]).reshape(R, n)
        w = np.asarray(want[q]).reshape(R, n)
        for j in range(R):
            assert np.array_equal(_bits(g[pi[j]]), _bits(w[j]))
    # Broadcast and Reduce from every root
    for root in range(R):
        got = sim.run("broadcast", xs, root=root, rings=[pi], **kw)
        want = sim.run("broadcast", ys, root=inv[root], **kw)
        for q in range(R):
            assert np.array_equal(_bits(got[pi[q]]), _bits(want[q]))
        got = sim.run("reduce", xs, root=root, rings=[pi], **kw)
        want = sim.run("reduce", ys, root=inv[root], **kw)
        assert np.array_equal(_bits(got[root]), _bits(want[inv[root]]))


@pytest.mark.parametrize("R,C,nr", [(4, 3, 2), (5, 4, 3), (8, 5, 4), (3, 2, 1)])
def test_folds_with_rings_match_the_simulation(R, C, nr):
    rings = [_perm(R, 10 + k) for k in range(nr)]
    n = 97 * R + 5
    xs = si.rank_inputs(9, R, "float32", n, extra=R * 10 + C)
    for chunk_bytes in (32, 160):
        K = chunk_bytes // 4
        got = sim.run("allreduce", xs, dtype="float32", nchannels=C, chunk_bytes=chunk_bytes, rings=rings)
        want = folds.ring_allreduce(xs, "sum", "float32", C, K, rings=rings)
        for r in range(R):
            assert np.array_equal(_bits(got[r]), _bits(want))
        got = sim.run("reduce", xs, root=R - 1, dtype="float32", nchannels=C, chunk_bytes=chunk_bytes, rings=rings)
        assert np.array_equal(_bits(got[R - 1]),
                              _bits(folds.ring_reduce(xs, "sum", "float32", R - 1, nchannels=C, rings=rings)))
    xr = si.rank_inputs(9, R, "float32", 53 * R, extra=R * 10 + C + 1)
    got = sim.run("reducescatter", xr, dtype="float32", nchannels=C, chunk_bytes=64, rings=rings)
    for r in range(R):
        want = folds.ring_reducescatter(xr, "sum", "float32", r, nchannels=C, rings=rings)
        assert np.array_equal(_bits(got[r]), _bits(want))
    # copies and exact sums equal their definitions on any ring
    xi = si.rank_inputs(9, R, "int32", 41 * R, extra=3)
    got = sim.run("allgather", xi, dtype="int32", nchannels=C, chunk_bytes=32, rings=rings)
    want = defs.allgather(xi)
    for r in range(R):
        assert np.array_equal(got[r], want[r])
    got = sim.run("allreduce", xi, dtype="int32", nchannels=C, chunk_bytes=32, rings=rings)
    want = defs.allreduce(xi, "sum", "int32")
    for r in range(R):
        assert np.array_equal(got[r], want[r])
    got = sim.run("broadcast", xi, root=1, dtype="int32", nchannels=C, chunk_bytes=32, rings=rings)
    for r in range(R):
        assert np.array_equal(got[r], xi[1])


def test_pins_catch_a_wrong_ring():
    """The fold on the reversed ring (a plausible slip: walking the ring
    backwards) must differ from the simulation on the ring."""
    R = 6
    ring = _perm(R, 5)
    xs = si.rank_inputs(9, R, "float32", 300, extra=99)
    got = sim.run("allreduce", xs, dtype="float32", nchannels=2, chunk_bytes=64, rings=[ring])[0]
    wrong = folds.ring_allreduce(xs, "sum", "float32", 2, 16, rings=[list(reversed(ring))])
    right = folds.ring_allreduce(xs, "sum", "float32", 2, 16, rings=[ring])
    assert np.array_equal(_bits(got), _bits(right))
    assert not np.array_equal(_bits(got), _bits(wrong))
