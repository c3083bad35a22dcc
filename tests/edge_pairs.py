"""Atom pairs placed within a few units in the last place of a cutoff.

Test input construction only.  The cutoff test r < rc (and r < r_list in the
list build) is an exact comparison, so the pair set of a pass is fixed by how
the squared distance of a pair is rounded.  The paper leaves that arithmetic
open; the reading taken here (and in the oracle) forms the separation first,
adds the periodic shift after it, and squares it as (dx dx + dy dy) + dz dz
with every product and sum rounded on its own.

`place` moves one atom of each chosen pair so that this squared distance
sits on a chosen side of rc^2, one step from it, and keeps only placements
that a different rounding would decide the other way: a fused multiply-add
in the sum of squares, or (across a face of the box) the shift added to the
neighbour's coordinate before the difference.  A kernel that decides such a
pair with another arithmetic than the oracle's then disagrees with it on
that pair, which changes the atom's density by the size of rho(rc).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def o3_r2(dx, dy, dz):
    """(dx dx + dy dy) + dz dz, every operation rounded (numpy float64)."""
    dx, dy, dz = np.float64(dx), np.float64(dy), np.float64(dz)
    return (dx * dx + dy * dy) + dz * dz


def fma(a, b, c):
    """a b + c rounded once (exact rational arithmetic, then one rounding)."""
    return float(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def fma_r2(dx, dy, dz):
    """fma(dz, dz, fma(dy, dy, dx dx)): the contracted sum of squares."""
    return fma(dz, dz, fma(dy, dy, float(np.float64(dx) * np.float64(dx))))


def sep_o3(xi, xj, L):
    """x_j - x_i, then the minimum-image shift added (one component)."""
    d = np.float64(xj) - np.float64(xi)
    if d > 0.5 * L:
        d = d - np.float64(L)
    elif d < -0.5 * L:
        d = d + np.float64(L)
    return d


def sep_preshift(xi, xj, L):
    """The neighbour's coordinate moved to its image first, then the difference."""
    d0 = np.float64(xj) - np.float64(xi)
    if d0 > 0.5 * L:
        return (np.float64(xj) - np.float64(L)) - np.float64(xi)
    if d0 < -0.5 * L:
        return (np.float64(xj) + np.float64(L)) - np.float64(xi)
    return d0


def r2_pair(pi, pj, L, how):
    if how == "o3":
        d = [sep_o3(pi[k], pj[k], L) for k in range(3)]
        return float(o3_r2(*d))
    if how == "fma":
        d = [sep_o3(pi[k], pj[k], L) for k in range(3)]
        return fma_r2(*d)
    if how == "preshift_fma":
        d = [sep_preshift(pi[k], pj[k], L) for k in range(3)]
        return fma_r2(*d)
    raise ValueError(how)


def _z_steps(z0, ks):
    """z0 moved k representable steps for each k in ks (one binade: the
    spacing of doubles is constant there); None if the range leaves it."""
    h = np.spacing(np.float64(z0))
    zs = np.float64(z0) + np.asarray(ks, dtype=np.float64) * h
    if np.any(np.spacing(zs) != h) or np.any(zs <= 0.0):
        return None
    return zs


def place(pos, L, i, j, r, inside, cross, rng, tries=200):
    """Move atom j so that the pair (i, j) lies one step inside (inside=True)
    or on (or one step outside) the radius r, along a direction drawn around
    the current separation.  `cross`: the separation must cross the x face
    of the box, else no face at all.  Returns the new position of j or None
    when no discriminating placement was found."""
    r2c = np.float64(r) * np.float64(r)
    pi = pos[i]
    d0 = np.array([sep_o3(pi[k], pos[j][k], L) for k in range(3)])
    other_how = "preshift_fma" if cross else "fma"
    for _ in range(tries):
        u = d0 / np.linalg.norm(d0) + rng.normal(scale=0.02, size=3)
        # a small z component: moving z_j by one step then moves r^2 by about a
        # tenth of a step, so every representable r^2 near rc^2 is reached
        u[2] = (1.0 if rng.random() < 0.5 else -1.0) * rng.uniform(0.003, 0.01)
        u /= np.linalg.norm(u)
        pj = pi + r * u
        pj = pj - L * np.floor(pj / L)          # wrapped into [0, L)
        raw = np.abs(pj - pi)
        if cross and not (raw[0] > 0.5 * L and raw[1] < 0.5 * L and raw[2] < 0.5 * L):
            continue
        if not cross and np.any(raw >= 0.5 * L):
            continue
        # r^2 is monotone in z_j: it grows with z_j when z_j - z_i > 0
        sgn = 1 if sep_o3(pi[2], pj[2], L) > 0 else -1
        ks = np.arange(-3000, 3001)
        zs = _z_steps(pj[2], sgn * ks)
        if zs is None:
            continue
        q = pj.copy()
        r2s = []
        for z in zs[::25]:
            q[2] = z
            r2s.append(r2_pair(pi, q, L, "o3"))
        r2s = np.array(r2s)
        hit = np.nonzero(r2s >= r2c)[0]
        if hit.size == 0 or hit[0] == 0:
            continue
        k0 = (hit[0] - 1) * 25
        for z in zs[k0:k0 + 26]:
            q = pj.copy()
            q[2] = z
            a = r2_pair(pi, q, L, "o3")
            if inside and not (a < r2c and np.nextafter(a, np.inf) >= r2c):
                continue
            if not inside and not (a >= r2c and np.nextafter(a, -np.inf) < r2c):
                continue
            if (r2_pair(pi, q, L, other_how) < r2c) != (a < r2c) and 0.0 <= z < L:
                return q
    return None


def edge_state(pos, L, radii, rng):
    """Positions with one discriminating edge pair per entry of `radii`
    ((r, inside, cross) tuples).  Pairs use distinct atoms; atom i of a
    crossing pair lies near the x = L face, and the partner j is an atom at
    about r from i with a small z offset, moved onto the edge.  Returns
    (pos, pairs) with pairs [(i, j, r, inside, cross)]."""
    pos = np.array(pos, dtype=np.float64)
    n = pos.shape[0]
    used = set()
    pairs = []
    for (r, inside, cross) in radii:
        for _ in range(4000):
            i = int(rng.integers(n))
            if i in used:
                continue
            xi = pos[i]
            if cross and not (L - 0.45 * r < xi[0] < L - 0.05 * r):
                continue
            d = _mi(pos - xi, L)
            dist = np.linalg.norm(d, axis=1)
            ok = (np.abs(dist - r) < 0.7) & (np.abs(d[:, 2]) < 0.8)
            if cross:
                ok &= (xi[0] + d[:, 0] > L)
            else:
                ok &= np.all(np.abs(pos - xi) < 0.5 * L - 0.8, axis=1)
            cand = [int(c) for c in np.nonzero(ok)[0] if int(c) not in used]
            if not cand:
                continue
            j = cand[int(rng.integers(len(cand)))]
            q = place(pos, L, i, j, r, inside, cross, rng)
            if q is None:
                continue
            pos[j] = q
            used.update((i, j))
            pairs.append((i, j, r, inside, cross))
            break
        else:
            raise RuntimeError("no edge pair placed")
    return pos, pairs


def _mi(d, L):
    return d - L * np.round(d / L)
