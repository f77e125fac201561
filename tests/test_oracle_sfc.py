"""Pins of the oracle's space-filling-curve keys (Sec. 2.2, Sec. 3).

Nothing here retypes the oracle's loops. Morton is checked against worked
values, a different algorithm (magic-mask bit spreading) and the quadrant
recursion of the Z-order. Hilbert is checked against the properties that
define a Hilbert curve: it is a bijection of every aligned corner cube onto a
prefix of the codes, consecutive codes are grid neighbours, and every aligned
2^j-cube occupies one aligned, contiguous code range.
"""
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sfc_values.txt")


def _golden():
    rows = []
    with open(GOLD) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            t = line.split()
            curve, dim = t[0], int(t[1])
            rows.append((curve, dim, [int(v) for v in t[2:2 + dim]], int(t[2 + dim], 16)))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: f"{r[0]}{r[1]}d-{r[2]}")
def test_golden_values(ora, row):
    curve, dim, p, key = row
    f = ora.morton if curve == "morton" else ora.hilbert
    assert f(dim, p) == key


def test_morton_hand_worked():
    # M(5,3): x=101b, y=011b. Group b holds (y_b, x_b) as bits (2b+1, 2b):
    # b0: x=1,y=1 -> 3; b1: x=0,y=1 -> 8; b2: x=1,y=0 -> 16; total 27.
    assert 3 + 8 + 16 == 27 == 0x1B


def _spread2(v):
    # textbook "part1by1" with magic masks: insert one zero between bits
    v = v.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    for s, m in ((16, 0x0000FFFF0000FFFF), (8, 0x00FF00FF00FF00FF), (4, 0x0F0F0F0F0F0F0F0F),
                 (2, 0x3333333333333333), (1, 0x5555555555555555)):
        v = (v | (v << np.uint64(s))) & np.uint64(m)
    return v


def _spread3(v):
    # textbook "part1by2": insert two zeros between bits of a 21-bit value
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    for s, m in ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF), (8, 0x100F00F00F00F00F),
                 (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249)):
        v = (v | (v << np.uint64(s))) & np.uint64(m)
    return v


@pytest.mark.parametrize("dim", [2, 3])
def test_morton_matches_mask_spreading(ora, dim):
    bits = 31 if dim == 2 else 21
    p = synth.uniform(20000, dim, bits, seed=7)
    keys = ora.encode(p, dim, ora.MORTON)
    if dim == 2:
        ref = _spread2(p[:, 0]) | (_spread2(p[:, 1]) << np.uint64(1))
    else:
        ref = _spread3(p[:, 0]) | (_spread3(p[:, 1]) << np.uint64(1)) | (_spread3(p[:, 2]) << np.uint64(2))
    np.testing.assert_array_equal(keys, ref)


@pytest.mark.parametrize("dim", [2, 3])
def test_morton_quadrant_recursion(ora, dim):
    # Z-order is self-similar: dropping the lowest bit plane of the point
    # drops the lowest D bits of the code.
    bits = 31 if dim == 2 else 21
    p = synth.uniform(5000, dim, bits, seed=8)
    k = ora.encode(p, dim, ora.MORTON)
    k_half = ora.encode(p >> 1, dim, ora.MORTON)
    np.testing.assert_array_equal(k >> np.uint64(dim), k_half)


def _corner_grid(dim, s):
    ax = np.arange(1 << s, dtype=np.uint32)
    g = np.stack(np.meshgrid(*([ax] * dim), indexing="ij"), -1).reshape(-1, dim)
    return g


@pytest.mark.parametrize("dim,s", [(2, 1), (2, 3), (2, 8), (3, 1), (3, 2), (3, 5)])
def test_hilbert_corner_bijection_and_unit_steps(ora, dim, s):
    # The corner cube [0,2^s)^D is a whole sub-curve: it must map onto the
    # code prefix [0, 2^(D s)) one-to-one, and walking the codes in order
    # must move by exactly one grid step each time.
    g = _corner_grid(dim, s)
    k = ora.encode(g, dim, ora.HILBERT)
    order = np.argsort(k)
    np.testing.assert_array_equal(k[order], np.arange(1 << (dim * s), dtype=np.uint64))
    walk = g[order].astype(np.int64)
    steps = np.abs(np.diff(walk, axis=0)).sum(axis=1)
    assert np.all(steps == 1)


@pytest.mark.parametrize("dim,j", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_hilbert_aligned_cubes_are_contiguous(ora, dim, j):
    # Any aligned 2^j-cube anywhere in the domain occupies one aligned block
    # of 2^(D j) consecutive codes, traversed by unit steps.
    bits = 31 if dim == 2 else 21
    corners = synth.uniform(40, dim, bits - j, seed=9).astype(np.uint64) << np.uint64(j)
    local = _corner_grid(dim, j).astype(np.uint64)
    for c in corners:
        cube = (c[None, :] + local).astype(np.uint32)
        k = np.sort(ora.encode(cube, dim, ora.HILBERT))
        size = 1 << (dim * j)
        assert int(k[0]) % size == 0
        np.testing.assert_array_equal(k - k[0], np.arange(size, dtype=np.uint64))
        kk = ora.encode(cube, dim, ora.HILBERT)
        walk = cube[np.argsort(kk)].astype(np.int64)
        assert np.all(np.abs(np.diff(walk, axis=0)).sum(axis=1) == 1)


@pytest.mark.parametrize("dim", [2, 3])
def test_hilbert_prefix_property(ora, dim):
    # coordinates below 2^(W-j) give codes below 2^(D (W-j)) for every j
    W = 32 if dim == 2 else 21
    rng = np.random.default_rng(3)
    for r in range(1, W):
        p = (rng.integers(0, 1 << r, size=(200, dim), dtype=np.uint64)).astype(np.uint32)
        if dim == 2 and r == 32:
            continue
        k = ora.encode(p, dim, ora.HILBERT)
        assert int(k.max()) < (1 << (dim * r))


@pytest.mark.parametrize("dim", [2, 3])
def test_hilbert_is_a_bijection_on_random_points(ora, dim):
    bits = 31 if dim == 2 else 21
    p = np.unique(synth.uniform(50000, dim, bits, seed=11), axis=0)
    k = ora.encode(p, dim, ora.HILBERT)
    assert np.unique(k).size == p.shape[0]


def test_hilbert_endpoints(ora):
    # the curve starts at the origin and, for the full 2D domain, ends at the
    # neighbouring corner on the x axis (code 2^64 - 1)
    assert ora.hilbert(2, [0, 0]) == 0
    assert ora.hilbert(2, [2**32 - 1, 0]) == 2**64 - 1
    assert ora.hilbert(3, [0, 0, 0]) == 0
    assert ora.hilbert(3, [2**21 - 1, 0, 0]) == 2**63 - 1
