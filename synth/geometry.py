"""Analytic surfaces sampled uniformly by area (surface point clouds).

The paper builds its graphs from a uniform point cloud on a car surface
(Sec. III.B; Sec. V.C).  The car STL files are not available, so these
generators stand in for them:

* ``sphere``          -- unit sphere, outward normals.
* ``bumpy_ellipsoid`` -- ellipsoid (4, 1.5, 1) with small sinusoidal bumps
                         displaced along the normal.
* ``car_body``        -- extruded rounded box 4.5 x 1.8 x 1.4 with four
                         cylindrical wheels.

Every generator returns ``(pos, normal)`` as float32 arrays ``[n][3]`` of one
i.i.d. stream, so any prefix of the stream is itself a uniform sample and a
subset of every longer prefix (the nested levels of Sec. III.C).
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def sphere(n: int, seed: int):
    """n points uniform on the unit sphere; the normal equals the position."""
    g = _rng(seed)
    p = _unit(g.standard_normal((n, 3)))
    p32 = p.astype(np.float32)
    return p32, p.astype(np.float32)


def _ellipsoid_uniform(n: int, g: np.random.Generator, axes):
    """Area-uniform points on an ellipsoid by rejection from the sphere map.

    A direction u on the unit sphere maps to (a ux, b uy, c uz); the area
    element there is proportional to |(b c ux, a c uy, a b uz)|, whose maximum
    over the sphere is the product of the two largest semi-axes.
    """
    a, b, c = axes
    amax = sorted(axes)[1] * sorted(axes)[2]
    out = []
    have = 0
    while have < n:
        m = max(1024, int((n - have) * 1.6))
        u = _unit(g.standard_normal((m, 3)))
        dens = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
        keep = g.random(m) * amax < dens
        out.append(u[keep])
        have += int(keep.sum())
    u = np.concatenate(out)[:n]
    p = u * np.array(axes)
    n0 = _unit(p / np.array(axes) ** 2)
    return p, n0


def bumpy_ellipsoid(n: int, seed_geom: int, seed_modes: int,
                    axes=(4.0, 1.5, 1.0), amp=0.05, modes=8):
    """Ellipsoid with seeded sinusoidal surface bumps.

    Height field h(p) = amp/modes * sum_m sin(f_m d_m.p + phi_m), with d_m a
    random unit vector, f_m ~ U(1, 6), phi_m ~ U(0, 2 pi).  Points move by
    h(p) along the ellipsoid normal n0; the normal of the bumped surface is
    taken to first order as normalize(n0 - grad h + (n0 . grad h) n0).
    """
    gm = _rng(seed_modes)
    d = _unit(gm.standard_normal((modes, 3)))
    f = gm.uniform(1.0, 6.0, modes)
    phi = gm.uniform(0.0, 2.0 * np.pi, modes)
    p, n0 = _ellipsoid_uniform(n, _rng(seed_geom), axes)
    arg = p @ (d * f[:, None]).T + phi            # [n][modes]
    h = (amp / modes) * np.sin(arg).sum(axis=1)
    grad = (amp / modes) * (np.cos(arg) @ (d * f[:, None]))
    q = p + h[:, None] * n0
    nrm = _unit(n0 - grad + (np.sum(n0 * grad, axis=1))[:, None] * n0)
    return q.astype(np.float32), nrm.astype(np.float32)


# --- car-like body --------------------------------------------------------

_BODY_LEN = 4.5
_BODY_W = 1.8
_BODY_Z0, _BODY_Z1 = 0.2, 1.6
_CORNER = 0.3
_WHEEL_R, _WHEEL_W = 0.35, 0.25
_WHEEL_X = (-1.45, 1.45)
_WHEEL_Y = (-0.775, 0.775)
_WHEEL_Z = 0.35


def _rrect_perimeter(t: np.ndarray):
    """Point and outward normal on the rounded-rectangle cross-section (y, z),
    parametrised by arc length t in [0, P)."""
    hw = _BODY_W / 2 - _CORNER
    zc = (_BODY_Z0 + _BODY_Z1) / 2
    hh = (_BODY_Z1 - _BODY_Z0) / 2 - _CORNER
    r = _CORNER
    segs = [2 * hh, np.pi * r / 2, 2 * hw, np.pi * r / 2, 2 * hh, np.pi * r / 2, 2 * hw, np.pi * r / 2]
    edges = np.concatenate([[0.0], np.cumsum(segs)])
    y = np.empty_like(t)
    z = np.empty_like(t)
    ny = np.empty_like(t)
    nz = np.empty_like(t)
    # straight right side (y = +W/2), going up
    corners = [(hw, hh), (-hw, hh), (-hw, -hh), (hw, -hh)]
    for s in range(8):
        sel = (t >= edges[s]) & (t < edges[s + 1])
        u = t[sel] - edges[s]
        if s % 2 == 0:
            k = s // 2
            if k == 0:
                y[sel], z[sel], ny[sel], nz[sel] = hw + r, -hh + u, 1.0, 0.0
            elif k == 1:
                y[sel], z[sel], ny[sel], nz[sel] = hw - u, hh + r, 0.0, 1.0
            elif k == 2:
                y[sel], z[sel], ny[sel], nz[sel] = -hw - r, hh - u, -1.0, 0.0
            else:
                y[sel], z[sel], ny[sel], nz[sel] = -hw + u, -hh - r, 0.0, -1.0
        else:
            k = s // 2
            cy, cz = corners[k]
            ang = k * np.pi / 2 + u / r
            ny[sel], nz[sel] = np.cos(ang), np.sin(ang)
            y[sel], z[sel] = cy + r * ny[sel], cz + r * nz[sel]
    return y, z + zc, ny, nz, edges[-1]


def _inside_body(p: np.ndarray, tol=1e-9) -> np.ndarray:
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    zc = (_BODY_Z0 + _BODY_Z1) / 2
    hw = _BODY_W / 2 - _CORNER
    hh = (_BODY_Z1 - _BODY_Z0) / 2 - _CORNER
    dy = np.maximum(np.abs(y) - hw, 0.0)
    dz = np.maximum(np.abs(z - zc) - hh, 0.0)
    in_sec = (dy ** 2 + dz ** 2) < (_CORNER - tol) ** 2
    return in_sec & (np.abs(x) < _BODY_LEN / 2 - tol)


def _inside_wheel(p: np.ndarray, tol=1e-9) -> np.ndarray:
    m = np.zeros(len(p), dtype=bool)
    for wx in _WHEEL_X:
        for wy in _WHEEL_Y:
            rr = (p[:, 0] - wx) ** 2 + (p[:, 2] - _WHEEL_Z) ** 2
            m |= (rr < (_WHEEL_R - tol) ** 2) & (np.abs(p[:, 1] - wy) < _WHEEL_W / 2 - tol)
    return m


def _car_batch(m: int, g: np.random.Generator):
    _, _, _, _, per = _rrect_perimeter(np.zeros(0))
    hw = _BODY_W / 2 - _CORNER
    hh = (_BODY_Z1 - _BODY_Z0) / 2 - _CORNER
    cap_area = (2 * hw + 2 * _CORNER) * (2 * hh + 2 * _CORNER) - (4 - np.pi) * _CORNER ** 2
    side = per * _BODY_LEN
    wheel_lat = 2 * np.pi * _WHEEL_R * _WHEEL_W
    wheel_disk = np.pi * _WHEEL_R ** 2
    areas = np.array([side, cap_area, cap_area] + [wheel_lat, wheel_disk, wheel_disk] * 4)
    comp = g.choice(len(areas), size=m, p=areas / areas.sum())
    p = np.zeros((m, 3))
    nr = np.zeros((m, 3))
    # body side wall
    s = comp == 0
    y, z, ny, nz, _ = _rrect_perimeter(g.uniform(0, per, s.sum()))
    p[s] = np.stack([g.uniform(-_BODY_LEN / 2, _BODY_LEN / 2, s.sum()), y, z], 1)
    nr[s] = np.stack([np.zeros_like(y), ny, nz], 1)
    # end caps: rejection inside the rounded rectangle
    for ci, sx in ((1, -1.0), (2, 1.0)):
        s = np.flatnonzero(comp == ci)
        pts = []
        while sum(len(q) for q in pts) < len(s):
            cand = np.stack([g.uniform(-_BODY_W / 2, _BODY_W / 2, 2 * len(s) + 8),
                             g.uniform(_BODY_Z0, _BODY_Z1, 2 * len(s) + 8)], 1)
            zc = (_BODY_Z0 + _BODY_Z1) / 2
            dy = np.maximum(np.abs(cand[:, 0]) - hw, 0.0)
            dz = np.maximum(np.abs(cand[:, 1] - zc) - hh, 0.0)
            pts.append(cand[dy ** 2 + dz ** 2 <= _CORNER ** 2])
        pts = np.concatenate(pts)[: len(s)]
        p[s] = np.stack([np.full(len(s), sx * _BODY_LEN / 2), pts[:, 0], pts[:, 1]], 1)
        nr[s] = np.array([sx, 0.0, 0.0])
    # wheels
    wi = 0
    for wx in _WHEEL_X:
        for wy in _WHEEL_Y:
            base = 3 + 3 * wi
            s = comp == base
            a = g.uniform(0, 2 * np.pi, s.sum())
            p[s] = np.stack([wx + _WHEEL_R * np.cos(a),
                             wy + g.uniform(-_WHEEL_W / 2, _WHEEL_W / 2, s.sum()),
                             _WHEEL_Z + _WHEEL_R * np.sin(a)], 1)
            nr[s] = np.stack([np.cos(a), np.zeros_like(a), np.sin(a)], 1)
            for j, sy in ((1, -1.0), (2, 1.0)):
                s = comp == base + j
                rad = _WHEEL_R * np.sqrt(g.random(s.sum()))
                a = g.uniform(0, 2 * np.pi, s.sum())
                p[s] = np.stack([wx + rad * np.cos(a), np.full(s.sum(), wy + sy * _WHEEL_W / 2),
                                 _WHEEL_Z + rad * np.sin(a)], 1)
                nr[s] = np.array([0.0, sy, 0.0])
            wi += 1
    keep = ~(_inside_body(p) | _inside_wheel(p))
    return p[keep], nr[keep]


def car_body(n: int, seed: int):
    """Area-uniform points on a car-like body: an extruded rounded box
    (length 4.5 along x, width 1.8, height 1.4 with the floor at z = 0.2,
    corner radius 0.3) plus four wheels (radius 0.35, width 0.25, axis along
    y, centred at x = +-1.45, y = +-0.775, z = 0.35).  Points that fall inside
    another solid are dropped, so the stream stays i.i.d. on the union
    surface."""
    g = _rng(seed)
    ps, ns = [], []
    have = 0
    while have < n:
        m = max(4096, int((n - have) * 1.3))
        p, nr = _car_batch(m, g)
        ps.append(p)
        ns.append(nr)
        have += len(p)
    p = np.concatenate(ps)[:n]
    nr = np.concatenate(ns)[:n]
    return p.astype(np.float32), nr.astype(np.float32)
