"""Conformer generator (host only): same atoms and bond graph, bond lengths
kept up to the jitter, no close contacts, deterministic streams."""
import numpy as np
import pytest

from paper_2311_01135_amd import molgen


@pytest.mark.parametrize("n_heavy,index", [(3, 0), (9, 1), (11, 2)])
def test_conformers_keep_the_molecule(n_heavy, index):
    z, x = molgen.tree(n_heavy, 5, index)
    jitter = 0.02
    confs = molgen.conformers(z, x, 6, 11, index, jitter=jitter)
    assert len(confs) == 6
    b0 = molgen.bonds(z, x)
    assert len(b0) == len(z) - 1                      # a tree
    d0 = np.array([np.linalg.norm(x[i] - x[j]) for i, j in b0])
    assert np.array_equal(confs[0][1], x) and np.array_equal(confs[0][0], z)
    moved = 0.0
    for zz, xx in confs[1:]:
        assert np.array_equal(zz, z)
        assert molgen.bonds(zz, xx) == b0
        d = np.array([np.linalg.norm(xx[i] - xx[j]) for i, j in b0])
        assert np.abs(d - d0).max() <= 2 * np.sqrt(3) * jitter + 1e-12
        assert molgen._min_dist(xx) >= 0.9
        moved = max(moved, np.abs(xx - x).max())
    if n_heavy >= 4:
        assert moved > 0.5                             # torsions changed the shape


def test_conformers_deterministic():
    z, x = molgen.tree(9, 2, 7)
    a = molgen.conformers(z, x, 4, 3, 7)
    b = molgen.conformers(z, x, 4, 3, 7)
    c = molgen.conformers(z, x, 4, 4, 7)
    for (za, xa), (zb, xb) in zip(a, b):
        assert np.array_equal(xa, xb)
    assert not np.array_equal(a[1][1], c[1][1])
