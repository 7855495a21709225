"""Seeded synthetic molecule generator (inputs only).

This module builds geometries and nothing else: it holds none of the
Kohn-Sham arithmetic, and both the HIP path and the FP64 oracle receive the
arrays it returns.  The paper's workload is GDB11 molecules with 9-11 heavy
atoms from {C, N, O, F} plus hydrogens, as non-equilibrium conformers (paper
section 4, first paragraph).  That dataset is not available, so these
generators produce random saturated trees of the same element set and size.

Recipes
-------
water(seed)
    O at the origin, H at (+-r sin(t/2), 0, r cos(t/2)), r = 0.9572 A,
    t = 104.52 deg; every coordinate is jittered by U(-0.02, 0.02) A.
tree(n_heavy, seed, index)
    Heavy atoms drawn from {C: .70, N: .15, O: .12, F: .03} with valences
    C4 N3 O2 F1.  Atom k > 0 bonds to a uniformly chosen earlier atom with a
    free valence (bond length U(1.40, 1.52) A, direction: the next free
    tetrahedral direction of the parent, tilted by up to 10 deg; the first
    bond of a parent with one neighbour gets angle 109.5 +- 10 deg and a
    uniform dihedral).  Remaining valences are filled with H at 1.09 A in
    the same way.  A draw with a dead end or any pair closer than 0.9 A is
    rejected and redrawn from the same stream.  Every accepted molecule is
    neutral with 8*n_heavy + 2 electrons.
conformers(Z, xyz, n_conf, seed, index)
    Torsion-sampled geometries of one molecule (same atoms and bonds), see
    the function.

Random numbers: SplitMix64(seed * 2**32 + index) seeds xoshiro256**.
"""
from __future__ import annotations

import math
import numpy as np

MASK = (1 << 64) - 1

ELEMENTS = ((6, 0.70), (7, 0.15), (8, 0.12), (9, 0.03))
VALENCE = {6: 4, 7: 3, 8: 2, 9: 1}


def _splitmix64(state: int):
    state = (state + 0x9E3779B97F4A7C15) & MASK
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return state, z ^ (z >> 31)


def _rotl(x: int, k: int) -> int:
    return ((x << k) | (x >> (64 - k))) & MASK


class Xoshiro256ss:
    """xoshiro256** (Blackman & Vigna), seeded through SplitMix64."""

    def __init__(self, seed: int):
        st = seed & MASK
        self.s = []
        for _ in range(4):
            st, z = _splitmix64(st)
            self.s.append(z)

    def next_u64(self) -> int:
        s = self.s
        result = (_rotl((s[1] * 5) & MASK, 7) * 9) & MASK
        t = (s[1] << 17) & MASK
        s[2] ^= s[0]
        s[3] ^= s[1]
        s[1] ^= s[2]
        s[0] ^= s[3]
        s[2] ^= t
        s[3] = _rotl(s[3], 45)
        return result

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        u = (self.next_u64() >> 11) * (1.0 / (1 << 53))
        return lo + (hi - lo) * u

    def randint(self, n: int) -> int:
        return int(self.uniform() * n) % n


def _rng(seed: int, index: int) -> Xoshiro256ss:
    return Xoshiro256ss((seed << 32) + index)


def water(seed: int = 0):
    """Water with seeded +-0.02 A jitter.  Returns (Z int32[3], xyz float64[3,3] in A)."""
    rng = _rng(seed, 0)
    r, th = 0.9572, math.radians(104.52)
    xyz = np.array([[0.0, 0.0, 0.0],
                    [r * math.sin(th / 2), 0.0, r * math.cos(th / 2)],
                    [-r * math.sin(th / 2), 0.0, r * math.cos(th / 2)]])
    for i in range(3):
        for k in range(3):
            xyz[i, k] += rng.uniform(-0.02, 0.02)
    return np.array([8, 1, 1], dtype=np.int32), xyz


def _norm(v):
    """|v| as np.linalg.norm forms it for a vector (sqrt of v . v)."""
    return math.sqrt(v.dot(v))


def _unit(v):
    return v / _norm(v)


def _cross(a, b):
    """a x b of two 3-vectors (the same products and differences as np.cross,
    without its per-call array handling, which dominated the generator)."""
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _perp(u):
    a = np.array([1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    return _unit(_cross(u, a))


def _rotate(v, axis, ang):
    axis = _unit(axis)
    return (v * math.cos(ang) + _cross(axis, v) * math.sin(ang)
            + axis * np.dot(axis, v) * (1 - math.cos(ang)))


def _tilt(rng, d, max_deg=10.0):
    """Rotate unit vector d by U(-max, max) deg about a random axis normal to d."""
    p = _perp(d)
    p = _rotate(p, d, rng.uniform(0.0, 2 * math.pi))
    return _unit(_rotate(d, p, math.radians(rng.uniform(-max_deg, max_deg))))


_TET = math.radians(109.4712206)


def _new_direction(rng, dirs):
    """Next bond direction from an atom whose existing bond directions are dirs."""
    k = len(dirs)
    if k == 0:
        z = rng.uniform(-1.0, 1.0)
        ph = rng.uniform(0.0, 2 * math.pi)
        s = math.sqrt(max(0.0, 1 - z * z))
        return np.array([s * math.cos(ph), s * math.sin(ph), z])
    if k == 1:
        u = dirs[0]
        ang = math.radians(109.5 + rng.uniform(-10.0, 10.0))
        p = _rotate(_perp(u), u, rng.uniform(0.0, 2 * math.pi))
        return _unit(u * math.cos(ang) + p * math.sin(ang))
    if k == 2:
        u1, u2 = dirs
        b = u1 + u2
        b = -_unit(b) if _norm(b) > 1e-8 else _perp(u1)
        nrm = _cross(u1, u2)
        nrm = _unit(nrm) if _norm(nrm) > 1e-8 else _perp(b)
        half = _TET / 2
        sgn = 1.0 if rng.uniform() < 0.5 else -1.0
        return _tilt(rng, _unit(b * math.cos(half) + sgn * nrm * math.sin(half)))
    s = sum(dirs)
    d = -_unit(s) if _norm(s) > 1e-8 else _perp(dirs[0])
    return _tilt(rng, d)


def _min_dist(xyz):
    d = xyz[:, None, :] - xyz[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    r[np.diag_indices(len(xyz))] = np.inf
    return r.min()


def _draw_element(rng):
    u = rng.uniform()
    acc = 0.0
    for z, p in ELEMENTS:
        acc += p
        if u < acc:
            return z
    return ELEMENTS[-1][0]


def tree(n_heavy: int, seed: int, index: int, max_tries: int = 1000):
    """Random saturated tree molecule.  Returns (Z int32[n], xyz float64[n,3] in A)."""
    rng = _rng(seed, index)
    for _ in range(max_tries):
        Z = [_draw_element(rng)]
        pos = [np.zeros(3)]
        dirs = [[]]
        free = [VALENCE[Z[0]]]
        dead = False
        for _k in range(1, n_heavy):
            cand = [i for i in range(len(Z)) if free[i] > 0]
            if not cand:
                dead = True
                break
            z = _draw_element(rng)
            p = cand[rng.randint(len(cand))]
            d = _new_direction(rng, dirs[p])
            L = rng.uniform(1.40, 1.52)
            Z.append(z)
            pos.append(pos[p] + L * d)
            dirs[p].append(d)
            dirs.append([-d])
            free[p] -= 1
            free.append(VALENCE[z] - 1)
        if dead:
            continue
        n_h = 0
        for i in range(n_heavy):
            while free[i] > 0:
                d = _new_direction(rng, dirs[i])
                Z.append(1)
                pos.append(pos[i] + 1.09 * d)
                dirs[i].append(d)
                free[i] -= 1
                n_h += 1
        xyz = np.array(pos)
        if _min_dist(xyz) < 0.9:
            continue
        Zarr = np.array(Z, dtype=np.int32)
        assert int(Zarr.sum()) == 8 * n_heavy + 2
        return Zarr, xyz
    # Large trees rarely come out clash-free as a whole; continue the same
    # stream with placements checked atom by atom (a clashing direction is
    # drawn again; a molecule that cannot be completed is started over).
    for _ in range(max_tries):
        got = _tree_checked(rng, n_heavy)
        if got is not None:
            return got
    raise RuntimeError("tree(): no acceptable molecule after %d draws" % max_tries)


def _place(rng, pos, dirs, p, length, max_local=100):
    """Direction and position of a new bond from atom p keeping every other
    atom at least 0.9 A away, or None."""
    for _ in range(max_local):
        d = _new_direction(rng, dirs[p])
        x = pos[p] + length * d
        if all(_norm(x - q) >= 0.9 for q in pos):
            return d, x
    return None


def _tree_checked(rng, n_heavy):
    Z = [_draw_element(rng)]
    pos = [np.zeros(3)]
    dirs = [[]]
    free = [VALENCE[Z[0]]]
    for _k in range(1, n_heavy):
        cand = [i for i in range(len(Z)) if free[i] > 0]
        if not cand:
            return None
        z = _draw_element(rng)
        p = cand[rng.randint(len(cand))]
        got = _place(rng, pos, dirs, p, rng.uniform(1.40, 1.52))
        if got is None:
            return None
        d, x = got
        Z.append(z)
        pos.append(x)
        dirs[p].append(d)
        dirs.append([-d])
        free[p] -= 1
        free.append(VALENCE[z] - 1)
    for i in range(n_heavy):
        while free[i] > 0:
            got = _place(rng, pos, dirs, i, 1.09)
            if got is None:
                return None
            d, x = got
            Z.append(1)
            pos.append(x)
            dirs[i].append(d)
            free[i] -= 1
    xyz = np.array(pos)
    Zarr = np.array(Z, dtype=np.int32)
    assert int(Zarr.sum()) == 8 * n_heavy + 2 and _min_dist(xyz) >= 0.9
    return Zarr, xyz


def batch(n_mol: int, seed: int, n_heavy=9, start: int = 0):
    """List of (Z, xyz) for molecules start..start+n_mol-1 of a seeded batch.

    n_heavy is an int (all molecules the same size) or a (lo, hi) pair, in
    which case the size of molecule i is drawn uniformly from lo..hi with the
    molecule's own stream (a separate SplitMix64 index space).
    """
    out = []
    for i in range(start, start + n_mol):
        if isinstance(n_heavy, tuple):
            lo, hi = n_heavy
            n = lo + _rng(seed + 0x5151, i).randint(hi - lo + 1)
        else:
            n = n_heavy
        out.append(tree(n, seed, i))
    return out


def batch_without(n_mol: int, seed: int, n_heavy=9, exclude=(9,)):
    """Like batch(), with every molecule that contains an element of exclude
    replaced by the first later tree of its own size that does not (for
    bases that cover fewer elements, e.g. 6-31G here: H, C, N, O)."""
    out = []
    for i in range(n_mol):
        if isinstance(n_heavy, tuple):
            lo, hi = n_heavy
            n = lo + _rng(seed + 0x5151, i).randint(hi - lo + 1)
        else:
            n = n_heavy
        z, x, _ = tree_without(n, seed, i, exclude)
        out.append((z, x))
    return out


def bonds(Z, xyz):
    """Bond list of a generated tree from its distances: heavy-heavy pairs
    within 1.7 A and H-heavy pairs within 1.25 A (the generator places them at
    1.40-1.52 A and 1.09 A; non-bonded pairs are at least 0.9 A apart and
    farther than these cut-offs in practice for these trees)."""
    Z = np.asarray(Z)
    xyz = np.asarray(xyz, dtype=np.float64)
    out = []
    for i in range(len(Z)):
        for j in range(i):
            if Z[i] == 1 and Z[j] == 1:
                continue
            cut = 1.7 if (Z[i] > 1 and Z[j] > 1) else 1.25
            if _norm(xyz[i] - xyz[j]) < cut:
                out.append((j, i))
    return out


def _side(n, bond_list, a, b):
    """Atoms on b's side of bond (a, b) in a tree."""
    adj = [[] for _ in range(n)]
    for i, j in bond_list:
        adj[i].append(j)
        adj[j].append(i)
    seen = {a, b}
    stack = [b]
    out = [b]
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if v not in seen:
                seen.add(v)
                out.append(v)
                stack.append(v)
    return out


def conformers(Z, xyz, n_conf: int, seed: int, index: int = 0, jitter: float = 0.02, max_tries: int = 200):
    """n_conf geometries of one molecule with the same atoms and bond graph:
    conformer 0 is xyz itself; conformer k > 0 turns, one after another, every
    bond between two heavy atoms that both carry further atoms by a torsion
    U(0, 2 pi) (the side of the later atom rotates about the bond axis; a
    torsion that brings any pair closer than 0.9 A or changes the
    distance-derived bond list is redrawn, and after max_tries/10 draws the
    bond keeps its torsion), then moves every coordinate by U(-jitter, jitter)
    A (redrawn under the same two conditions).  Stands in for the several
    non-equilibrium conformers per molecule of the paper's dataset (section
    4); the stream of conformer k is SplitMix64((seed + 0xC0F) * 2**32 +
    index * 65536 + k)."""
    Z = np.asarray(Z, dtype=np.int32)
    xyz0 = np.asarray(xyz, dtype=np.float64)
    n = len(Z)
    bl = bonds(Z, xyz0)
    deg = np.zeros(n, dtype=int)
    for i, j in bl:
        deg[i] += 1
        deg[j] += 1
    rot = [(i, j) for i, j in bl if Z[i] > 1 and Z[j] > 1 and deg[i] > 1 and deg[j] > 1]
    sides = [_side(n, bl, i, j) for i, j in rot]
    out = [(Z.copy(), xyz0.copy())]
    for k in range(1, n_conf):
        rng = _rng(seed + 0xC0F, index * 65536 + k)
        x = xyz0.copy()
        for (i, j), side in zip(rot, sides):
            # a new torsion for this bond, keeping the old one when every
            # try collides with the rest of the molecule
            for _ in range(max_tries // 10):
                ang = rng.uniform(0.0, 2 * math.pi)
                y = x.copy()
                axis = y[j] - y[i]
                for a in side:
                    y[a] = y[j] + _rotate(y[a] - y[j], axis, ang)
                if _min_dist(y) >= 0.9 and bonds(Z, y) == bl:
                    x = y
                    break
        for _ in range(max_tries):
            y = x.copy()
            for a in range(n):
                for c in range(3):
                    y[a, c] += rng.uniform(-jitter, jitter)
            if _min_dist(y) >= 0.9 and bonds(Z, y) == bl:
                out.append((Z.copy(), y))
                break
        else:
            raise RuntimeError("conformers(): no acceptable jitter after %d draws" % max_tries)
    return out


def nbf_sto3g(Z) -> int:
    """Number of STO-3G functions: 1 per H, 5 per C/N/O/F (a count, not arithmetic)."""
    Z = np.asarray(Z)
    return int((Z == 1).sum() + 5 * (Z > 1).sum())


def nbf_631g(Z) -> int:
    """Number of 6-31G functions: 2 per H, 9 per C/N/O (a count, not arithmetic)."""
    Z = np.asarray(Z)
    return int(2 * (Z == 1).sum() + 9 * (Z > 1).sum())


def tree_without(n_heavy: int, seed: int, index: int, exclude=(9,)):
    """First molecule tree(n_heavy, seed, index + k), k = 0, 1, ..., with no
    element in exclude (6-31G here covers H, C, N, O).  Returns (Z, xyz, k)."""
    k = 0
    while True:
        z, x = tree(n_heavy, seed, index + k)
        if not np.isin(z, exclude).any():
            return z, x, k
        k += 1


def pack(mols):
    """Concatenate a list of (Z, xyz) into the flat arrays the C ABI takes."""
    n_atoms = np.array([len(z) for z, _ in mols], dtype=np.int32)
    Z = np.concatenate([z for z, _ in mols]).astype(np.int32)
    xyz = np.concatenate([x for _, x in mols]).astype(np.float64).reshape(-1)
    return n_atoms, Z, np.ascontiguousarray(xyz)
