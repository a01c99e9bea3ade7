"""The block cores of the sampled full-size checks (tests/blocks.py) agree with the
oracle's full-grid results, on a grid small enough for the full pass (host only)."""
import itertools

import numpy as np
import pytest

import blocks
import oracle
from gpu_util import rand_grid

N = 65


@pytest.fixture(scope="module")
def grids():
    s = oracle.fine_stencil(3, 4, 1.0 / (N - 1))
    u = rand_grid(N, 3, 901)
    f = rand_grid(N, 3, 902) * s[2, 2, 2]
    v = rand_grid((N - 1) // 2 + 1, 3, 903)
    return s, u, f, v


def _starts(B, even):
    # blocks at the grid's sides, across the middle and at ragged positions
    per = blocks.starts(N, B, [0, 7, 30, 33, N - 8, N - 1], even=even)
    return list(itertools.product(per, per, per))[::7]


def test_sweep_and_residual_blocks(grids):
    s, u, f, _ = grids
    om = oracle.jacobi_omega(3)
    full_j = oracle.jacobi(s, om, f, u)
    full_r = oracle.residual(s, f, u)
    B = blocks.SWEEP_B
    for st in _starts(B, False):
        c = blocks.core(st, B, N, blocks.SWEEP_M)
        ref = oracle.jacobi(s, om, blocks.cut(f, st, B), blocks.cut(u, st, B))
        np.testing.assert_allclose(ref[c], blocks.cut(full_j, st, B)[c], rtol=0, atol=1e-12 * np.abs(full_j).max())
        ref = oracle.residual(s, blocks.cut(f, st, B), blocks.cut(u, st, B))
        np.testing.assert_allclose(ref[c], blocks.cut(full_r, st, B)[c], rtol=0, atol=1e-12 * np.abs(full_r).max())


def test_restrict_blocks(grids):
    s, u, f, _ = grids
    full = oracle.restrict(oracle.residual(s, f, u))
    B, CB = blocks.RR_B, blocks.RR_CB
    for st in _starts(B, True):
        c = blocks.core(blocks.coarse(st), CB, (N - 1) // 2 + 1, blocks.RR_M)
        ref = oracle.restrict(oracle.residual(s, blocks.cut(f, st, B), blocks.cut(u, st, B)))
        got = blocks.cut(full, blocks.coarse(st), CB)
        np.testing.assert_allclose(ref[c], got[c], rtol=0, atol=1e-12 * np.abs(full).max())


def test_prolong_blocks(grids):
    _, u, _, v = grids
    full = oracle.prolong_add(v, u.copy())
    B, CB = blocks.PRO_B, blocks.PRO_CB
    for st in _starts(B, True):
        c = blocks.core(st, B, N, blocks.PRO_M)
        ref = oracle.prolong_add(blocks.cut(v, blocks.coarse(st), CB), blocks.cut(u, st, B))
        np.testing.assert_allclose(ref[c], blocks.cut(full, st, B)[c], rtol=0, atol=1e-12 * np.abs(full).max())


def test_points_near_a_block_side_differ(grids):
    """Points next to a block side that is not the grid's boundary do differ from the
    full grid's (their reach leaves the block): the cores leave them out for a reason."""
    s, u, f, v = grids
    om = oracle.jacobi_omega(3)
    full_j = oracle.jacobi(s, om, f, u)
    st = (30, 30, 30)
    ref = oracle.jacobi(s, om, blocks.cut(f, st, 9), blocks.cut(u, st, 9))
    got = blocks.cut(full_j, st, 9)
    assert np.abs(ref[1, 4, 4] - got[1, 4, 4]) > 1e-6
    full_p = oracle.prolong_add(v, u.copy())
    ref = oracle.prolong_add(blocks.cut(v, [15, 15, 15], 9), blocks.cut(u, st, 17).copy())
    got = blocks.cut(full_p, st, 17)
    assert np.abs(ref[1, 8, 8] - got[1, 8, 8]) > 1e-6
