"""The parity checker itself (tests/_compare.py), on the CPU: rows built from the oracle's
answer with one planted mistake each must be rejected, and genuine near-ties must be
excused and counted."""
import numpy as np
import pytest

from tests._compare import compare_rows


@pytest.fixture(scope="module")
def case(oracle_lib):
    # integer lattice: many exact ties, so swaps and boundary ties exist
    g = np.arange(5, dtype=np.float32)
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    P = P[np.random.default_rng(0).permutation(P.shape[0])]
    Q = np.array([[2.0, 2.0, 2.0], [0.31, 1.17, 2.63], [2.5, 2.5, 2.5]], np.float32)
    k = 6
    ri, rd, rD = oracle_lib.knn_bruteforce(P, Q, k + 1)
    return P, Q, k, ri, rd, rD


def _rows(case):
    P, Q, k, ri, rd, rD = case
    return ri[:, :k].copy(), rd[:, :k].copy()


def test_exact_rows_pass(case):
    P, Q, k, ri, rd, rD = case
    gi, gd = _rows(case)
    assert compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q) == 0


def test_tied_swap_is_excused(case):
    P, Q, k, ri, rd, rD = case
    gi, gd = _rows(case)
    # query 0 sits on a lattice point: positions 1..6 are the six axis neighbours, all at 1
    assert np.all(rD[0, 1:k] == 1.0)
    gi[0, [1, 2]] = gi[0, [2, 1]]
    with pytest.raises(AssertionError, match="ordered"):
        compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q)   # breaks the (D, rank) order
    # a tie at the set boundary: the oracle's 7th rank (also at distance 1) in place of a
    # tied one keeps the row valid if the row stays ordered by (D, rank)
    gi, gd = _rows(case)
    row = np.sort(np.concatenate([ri[0, 2:k], ri[0, k:k + 1]]))
    gi[0, 1:k] = row
    assert compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q) >= 1


def test_untied_substitute_is_rejected(case):
    P, Q, k, ri, rd, rD = case
    gi, gd = _rows(case)
    # the 2nd query has no ties; put its (k+1)-th rank in place of its k-th, keeping the
    # k-th distance: the returned distance then does not belong to the returned rank
    assert rD[1, k - 1] != rD[1, k]
    gi[1, k - 1] = ri[1, k]
    with pytest.raises(AssertionError):
        compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q)
    # and with its own distance it is not a near-tie of the oracle's k-th
    gd[1, k - 1] = rd[1, k]
    with pytest.raises(AssertionError, match="pos"):
        compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q)


def test_duplicate_rank_is_rejected(case):
    P, Q, k, ri, rd, rD = case
    gi, gd = _rows(case)
    gi[0, 2] = gi[0, 1]
    with pytest.raises(AssertionError, match="twice"):
        compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q)


def test_rank_outside_prefix_or_deleted_is_rejected(case):
    P, Q, k, ri, rd, rD = case
    gi, gd = _rows(case)
    m = int(gi.max())            # the largest returned rank lies outside P_{1:m}
    with pytest.raises(AssertionError, match="prefix"):
        compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q, m=m)
    live = np.ones(P.shape[0], bool)
    live[gi[2, 3]] = False
    with pytest.raises(AssertionError, match="deleted"):
        compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q, live=live)


def test_wrong_distance_and_padding_are_rejected(case):
    P, Q, k, ri, rd, rD = case
    gi, gd = _rows(case)
    gd[2, 4] *= 1.0001
    with pytest.raises(AssertionError, match="rel err"):
        compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q)
    gi, gd = _rows(case)
    gi[1, k - 1] = -1
    gd[1, k - 1] = np.inf
    with pytest.raises(AssertionError, match="padding"):
        compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q)
    gi, gd = _rows(case)
    gd[0, 0] = 1e-30             # query 0 coincides with a point: distance must be exactly 0
    with pytest.raises(AssertionError, match="zero"):
        compare_rows(gi, gd, ri[:, :k], rD[:, :k], P=P, Q=Q)
