"""Pins for the oracle's geometry: hand-worked examples and invariants."""
import numpy as np
import pytest

from conftest import read_golden
from oracle.lattice import Lattice


def test_hand_examples_4444():
    lat = Lattice((4, 4, 4, 4))
    for key, val in read_golden("index_examples_4x4x4x4.txt").items():
        xyzt, want = val.split(":")
        x, y, z, t = (int(v) for v in xyzt.split(","))
        lex, par, eo = (int(v) for v in want.split(","))
        assert lat.lex(x, y, z, t) == lex, key
        assert lat.parity(x, y, z, t) == par, key
        assert lat.eo(x, y, z, t) == eo, key
        assert lat.coords(lex) == (x, y, z, t), key


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 6, 4), (6, 4, 4, 8)])
def test_eo_bijection_and_parity_blocks(dims):
    lat = Lattice(dims)
    e = lat.eo_of_lex()
    assert sorted(e.tolist()) == list(range(lat.N))
    for lex in range(lat.N):
        c = lat.coords(lex)
        assert (e[lex] >= lat.N // 2) == bool(lat.parity(*c))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 6, 4), (6, 4, 4, 8)])
def test_neighbour_invariants(dims):
    lat = Lattice(dims)
    tab = lat.neighbor_table()
    half = lat.N // 2
    idx = np.arange(lat.N)
    for mu in range(4):
        # forward then backward returns to the start
        assert np.array_equal(tab[mu + 4][tab[mu]], idx)
        assert np.array_equal(tab[mu][tab[mu + 4]], idx)
        # every hop flips parity
        assert np.array_equal(tab[mu] >= half, idx < half)
        # L steps in one direction wrap around
        cur = idx.copy()
        for _ in range(dims[mu]):
            cur = tab[mu][cur]
        assert np.array_equal(cur, idx)
        if dims[mu] == 2:  # +mu and -mu reach the same site, still two terms
            assert np.array_equal(tab[mu], tab[mu + 4])


def test_odd_extent_rejected():
    with pytest.raises(ValueError):
        Lattice((3, 4, 4, 4))
    with pytest.raises(ValueError):
        Lattice((4, 4, 4, 0))


def test_neighbour_hand_example():
    lat = Lattice((4, 4, 4, 4))
    tab = lat.neighbor_table()
    # site (3,0,0,0): +x wraps to (0,0,0,0); -t wraps to (3,0,0,3)
    s = lat.eo(3, 0, 0, 0)
    assert tab[0][s] == lat.eo(0, 0, 0, 0) == 0
    assert tab[7][s] == lat.eo(3, 0, 0, 3)
    assert lat.eo(3, 0, 0, 3) == (3 + 192) // 2  # parity (3+3)%2 = 0
