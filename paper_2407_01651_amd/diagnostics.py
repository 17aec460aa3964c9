"""Morphology diagnostics on macro fields (host side, off the per-step path).

* tip radius of every crystal arm: march along the arm direction R(angle) e_k
  from the seed centre in steps of 0.1 node, interpolate psi bilinearly
  (trilinearly in 3D), take the first crossing from psi > 0 to psi <= 0,
  refined linearly; the tip velocity is the change of that radius over a
  number of steps, in units of W0/tau0 (the paper reports tip velocities in
  these units, Sec. 3.3);
* solid fraction: mean of h(psi) = (psi + 1)/2;
* gas volume sum (1 - phi) and gas centroid;
* per-bubble volume and centroid: connected components of phi < 1/2
  (periodic axes joined), volume = sum (1 - phi) over each component,
  centroid weighted by (1 - phi), circular mean along periodic axes.

Inputs are torch or numpy arrays indexed [z][y][x] (2D: [y][x]).
"""
from __future__ import annotations

import math

import numpy as np


def _np(a):
    try:
        return a.detach().cpu().numpy()
    except AttributeError:
        return np.asarray(a)


def _interp(f, p, periodic):
    """Multilinear interpolation of f (array [.., y, x]) at point p = (x, y[, z])."""
    d = len(p)
    shape = f.shape[::-1]   # (nx, ny[, nz])
    idx0, wts = [], []
    for a in range(d):
        q = p[a]
        if periodic[a]:
            q = q % shape[a]
        else:
            q = min(max(q, 0.0), shape[a] - 1.0)
        i0 = int(math.floor(q))
        t = q - i0
        i1 = i0 + 1
        if periodic[a]:
            i0 %= shape[a]
            i1 %= shape[a]
        else:
            i1 = min(i1, shape[a] - 1)
        idx0.append((i0, i1))
        wts.append(t)
    val = 0.0
    for corner in range(1 << d):
        w = 1.0
        ix = []
        for a in range(d):
            b = (corner >> a) & 1
            w *= wts[a] if b else (1.0 - wts[a])
            ix.append(idx0[a][b])
        val += w * f[tuple(reversed(ix))]
    return val


def tip_radii(psi, seeds, periodic, dim=2, rmax=None, step=0.1):
    """Radius of each arm of each seed: array [nseed, 2*dim] (nan if not found)."""
    f = _np(psi)
    shape = f.shape[::-1]
    rmax = rmax or 0.5 * min(shape[:dim])
    out = np.full((len(seeds), 2 * dim), np.nan)
    for si, s in enumerate(seeds):
        c = np.array([s["x"], s["y"], s.get("z", 0.0)][:dim])
        th = s.get("angle", 0.0)
        axes = []
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = 1.0
            if dim >= 2:
                e2 = e.copy()
                e[0] = math.cos(th) * e2[0] - math.sin(th) * e2[1]
                e[1] = math.sin(th) * e2[0] + math.cos(th) * e2[1]
            axes += [e, -e]
        for k, e in enumerate(axes):
            prev = _interp(f, c, periodic)
            if prev <= 0:
                continue
            r = 0.0
            while r < rmax:
                r2 = r + step
                v = _interp(f, c + r2 * e, periodic)
                if v <= 0:
                    out[si, k] = r + step * prev / (prev - v)
                    break
                prev, r = v, r2
    return out


def solid_fraction(psi):
    return float(((_np(psi) + 1.0) * 0.5).mean())


def gas_stats(phi, periodic):
    """Total gas volume and per-bubble (volume, centroid) list."""
    from scipy import ndimage
    f = _np(phi)
    gas = 1.0 - f
    d = f.ndim
    lab, n = ndimage.label(f < 0.5)
    # join components across periodic faces
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for a in range(d):
        ax = d - 1 - a            # array axis of coordinate a
        if not periodic[a]:
            continue
        first = np.take(lab, 0, axis=ax)
        last = np.take(lab, lab.shape[ax] - 1, axis=ax)
        for u, v in zip(first.ravel(), last.ravel()):
            if u and v:
                ru, rv = find(u), find(v)
                if ru != rv:
                    parent[ru] = rv
    roots = np.array([find(i) for i in range(n + 1)])
    lab = roots[lab]
    out = []
    coords = np.indices(f.shape)
    for r in sorted(set(roots[1:].tolist())):
        m = lab == r
        w = gas[m]
        vol = float(w.sum())
        cen = []
        for a in range(d):
            ax = d - 1 - a
            xs = coords[ax][m].astype(float)
            L = f.shape[ax]
            if periodic[a]:
                ang = 2 * math.pi * xs / L
                z = (w * np.exp(1j * ang)).sum()
                cen.append(float((np.angle(z) % (2 * math.pi)) * L / (2 * math.pi)))
            else:
                cen.append(float((w * xs).sum() / max(vol, 1e-300)))
        out.append(dict(volume=vol, centroid=cen))
    return float(gas.sum()), out
