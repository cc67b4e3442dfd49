"""Pins of the oracle's point-to-point definitions (Section II-A Send/Recv
and group calls): an independent element loop on tiny inputs, the
transpose property of all-to-all, and planted mistakes that must fail."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs


def _loop_alltoall(xs):
    # element by element from the definition: rank b's element at a*n + i
    # comes from rank a's element at b*n + i
    R = len(xs)
    n = len(xs[0]) // R
    out = [np.empty_like(xs[0]) for _ in range(R)]
    for b in range(R):
        for a in range(R):
            for i in range(n):
                out[b][a * n + i] = xs[a][b * n + i]
    return out


@pytest.mark.parametrize("R,n,dtype", [(2, 1, "int32"), (3, 5, "float32"), (4, 7, "bfloat16"), (8, 3, "int32")])
def test_alltoall_matches_element_loop(R, n, dtype):
    xs = si.rank_inputs(si.WL_P2P, R, dtype, R * n, extra=R * 10 + n)
    got = defs.alltoall(xs)
    want = _loop_alltoall(xs)
    for b in range(R):
        assert np.array_equal(got[b].view(np.uint8), want[b].view(np.uint8))


def test_alltoall_twice_is_identity_and_diagonal_stays():
    R, n = 6, 11
    xs = si.rank_inputs(si.WL_P2P, R, "float32", R * n, extra=1)
    once = defs.alltoall(xs)
    twice = defs.alltoall(once)
    for b in range(R):
        assert np.array_equal(twice[b], xs[b])
        # the block a rank sends to itself does not move
        assert np.array_equal(once[b][b * n:(b + 1) * n], xs[b][b * n:(b + 1) * n])


def test_two_ranks_worked_case():
    xs = [np.array([1, 2, 3, 4], np.int32), np.array([5, 6, 7, 8], np.int32)]
    out = defs.alltoall(xs)
    assert out[0].tolist() == [1, 2, 5, 6]
    assert out[1].tolist() == [3, 4, 7, 8]


def test_planted_index_swap_is_caught():
    # a transposed-roles mistake (rank b takes block a of rank b) must differ
    R, n = 4, 3
    xs = si.rank_inputs(si.WL_P2P, R, "int32", R * n, extra=2)
    wrong = [np.concatenate([xs[b][a * n:(a + 1) * n] for a in range(R)]) for b in range(R)]
    good = defs.alltoall(xs)
    assert any(not np.array_equal(w, g) for w, g in zip(wrong, good))


def test_sendrecv_is_a_bitwise_copy():
    x = si.rank_inputs(si.WL_P2P, 1, "bfloat16", 1001, extra=3)[0]
    y = defs.sendrecv(x)
    assert y is not x and np.array_equal(y.view(np.uint8), x.view(np.uint8))
