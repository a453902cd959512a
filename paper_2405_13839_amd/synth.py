"""Seeded synthetic point clouds standing in for the paper's scanned models.

This module only draws inputs: points, area weights, analytic ("truth") normals, part /
component ids and outlier masks. It holds none of the method's arithmetic, and both the
GPU path and the CPU oracle consume exactly the FP32 arrays it returns.

Conventions borrowed from the paper: noise is a percentage of the bounding-box diagonal
(Sec. 6), outliers are uniform in the bounding box (Sec. 6, robustness to outliers), area
weights approximate the surface area each point stands for (Sec. 5.1). Every draw uses
NumPy's PCG64 generator in float64 and is cast to float32 once at the end.

Layout: P, N_true are planar float32 arrays of shape (3, n).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Cloud:
    P: np.ndarray  # (3, n) float32 positions
    area: np.ndarray  # (n,) float32 area weights
    N_true: np.ndarray  # (3, n) float32 analytic outward normals (0 for outliers)
    comp: np.ndarray  # (n,) int32 connected-component id, -1 for outliers
    inlier: np.ndarray  # (n,) bool
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.P.shape[1])


# ----------------------------------------------------------------------------- parts
def _rot(rng):
    """Uniform random rotation (QR of a Gaussian matrix with sign fix)."""
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


class _Part:
    area: float

    def sample(self, rng, m):  # -> (x (m,3), n (m,3))
        raise NotImplementedError

    def inside(self, x):  # strictly inside, x (m,3) -> bool (m,)
        raise NotImplementedError


class _Sphere(_Part):
    def __init__(self, c, R):
        self.c, self.R = np.asarray(c, float), float(R)
        self.area = 4 * math.pi * R * R

    def sample(self, rng, m):
        u = rng.standard_normal((m, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        return self.c + self.R * u, u

    def inside(self, x):
        return np.sum((x - self.c) ** 2, axis=1) < self.R**2


class _Torus(_Part):
    """Tube radius r around a circle of radius R, in a frame (centre c, rotation Rm)."""

    def __init__(self, c, Rm, R, r):
        self.c, self.Rm, self.R, self.r = np.asarray(c, float), np.asarray(Rm, float), float(R), float(r)
        self.area = 4 * math.pi**2 * R * r

    def sample(self, rng, m):
        xs, ns = [], []
        got = 0
        while got < m:
            k = int((m - got) * 1.6) + 16
            th = rng.uniform(0, 2 * math.pi, k)  # tube angle
            ph = rng.uniform(0, 2 * math.pi, k)  # around the axis
            acc = rng.uniform(0, 1, k) < (self.R + self.r * np.cos(th)) / (self.R + self.r)
            th, ph = th[acc], ph[acc]
            nl = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), np.sin(th)], 1)
            xl = np.stack([(self.R + self.r * np.cos(th)) * np.cos(ph),
                           (self.R + self.r * np.cos(th)) * np.sin(ph), self.r * np.sin(th)], 1)
            xs.append(xl)
            ns.append(nl)
            got += xl.shape[0]
        xl = np.concatenate(xs)[:m]
        nl = np.concatenate(ns)[:m]
        return self.c + xl @ self.Rm.T, nl @ self.Rm.T

    def inside(self, x):
        xl = (x - self.c) @ self.Rm
        rho = np.sqrt(xl[:, 0] ** 2 + xl[:, 1] ** 2)
        return (rho - self.R) ** 2 + xl[:, 2] ** 2 < self.r**2


def _ellipsoid_area(a, b, c, nt=400, nph=800):
    th = (np.arange(nt) + 0.5) * math.pi / nt
    ph = (np.arange(nph) + 0.5) * 2 * math.pi / nph
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    st, ct, sp, cp = np.sin(T), np.cos(T), np.sin(Ph), np.cos(Ph)
    # |x_theta x x_phi| for x = (a st cp, b st sp, c ct)
    nx = b * c * st * st * cp
    ny = a * c * st * st * sp
    nz = a * b * st * ct
    return float(np.sum(np.sqrt(nx**2 + ny**2 + nz**2)) * (math.pi / nt) * (2 * math.pi / nph))


class _Ellipsoid(_Part):
    def __init__(self, c, Rm, axes):
        self.c, self.Rm, self.ax = np.asarray(c, float), np.asarray(Rm, float), np.asarray(axes, float)
        self.area = _ellipsoid_area(*self.ax)

    def sample(self, rng, m):
        a, b, c = self.ax
        wmax = max(b * c, a * c, a * b)
        xs, ns = [], []
        got = 0
        while got < m:
            k = int((m - got) * 2.0) + 16
            u = rng.standard_normal((k, 3))
            u /= np.linalg.norm(u, axis=1, keepdims=True)
            # area element of the map u -> (a ux, b uy, c uz) relative to the sphere's
            wgt = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
            acc = rng.uniform(0, 1, k) < wgt / wmax
            u = u[acc]
            xl = u * self.ax
            nl = xl / self.ax**2
            nl /= np.linalg.norm(nl, axis=1, keepdims=True)
            xs.append(xl)
            ns.append(nl)
            got += xl.shape[0]
        xl = np.concatenate(xs)[:m]
        nl = np.concatenate(ns)[:m]
        return self.c + xl @ self.Rm.T, nl @ self.Rm.T

    def inside(self, x):
        xl = (x - self.c) @ self.Rm
        return np.sum((xl / self.ax) ** 2, axis=1) < 1.0


def _sq_f(w, e):
    """Signed power used by superquadrics: sign(w) |w|^e."""
    return np.sign(w) * np.abs(w) ** e


class _Superquadric(_Part):
    """Superellipsoid |x/a|^(2/e2) + |y/b|^(2/e2))^(e2/e1) + |z/c|^(2/e1) = 1."""

    def __init__(self, c, Rm, axes, e1, e2, rng):
        self.c, self.Rm, self.ax = np.asarray(c, float), np.asarray(Rm, float), np.asarray(axes, float)
        self.e1, self.e2 = float(e1), float(e2)
        # area by quadrature of the parametric area element on a fine grid; the cell areas
        # also serve as the sampling table (cells drawn by area, uniform inside a cell)
        self.ne, self.no = 600, 1200
        eta, om, dA = self._grid(self.ne, self.no)
        cell = dA.ravel() * (math.pi / self.ne) * (2 * math.pi / self.no)
        self.area = float(np.sum(cell))
        self.cdf = np.cumsum(cell) / np.sum(cell)

    def _pos(self, eta, om):
        a, b, c = self.ax
        ce, se = np.cos(eta), np.sin(eta)
        co, so = np.cos(om), np.sin(om)
        x = a * _sq_f(ce, self.e1) * _sq_f(co, self.e2)
        y = b * _sq_f(ce, self.e1) * _sq_f(so, self.e2)
        z = c * _sq_f(se, self.e1)
        return np.stack([x, y, z], -1)

    def _normal(self, x):
        a, b, c = self.ax
        e1, e2 = self.e1, self.e2
        ax, ay, az = np.abs(x[..., 0] / a) + 1e-300, np.abs(x[..., 1] / b) + 1e-300, np.abs(x[..., 2] / c) + 1e-300
        g = (ax ** (2 / e2) + ay ** (2 / e2)) ** (e2 / e1 - 1)
        nx = g * (2 / e1) * ax ** (2 / e2 - 1) * np.sign(x[..., 0]) / a
        ny = g * (2 / e1) * ay ** (2 / e2 - 1) * np.sign(x[..., 1]) / b
        nz = (2 / e1) * az ** (2 / e1 - 1) * np.sign(x[..., 2]) / c
        nv = np.stack([nx, ny, nz], -1)
        return nv / np.linalg.norm(nv, axis=-1, keepdims=True)

    def _grid(self, ne, no):
        eta = -math.pi / 2 + (np.arange(ne) + 0.5) * math.pi / ne
        om = -math.pi + (np.arange(no) + 0.5) * 2 * math.pi / no
        E, O = np.meshgrid(eta, om, indexing="ij")
        dA = self._dA(E, O)
        return E, O, dA

    def _dA(self, E, O, h=1e-6):
        xe = (self._pos(E + h, O) - self._pos(E - h, O)) / (2 * h)
        xo = (self._pos(E, O + h) - self._pos(E, O - h)) / (2 * h)
        return np.linalg.norm(np.cross(xe, xo), axis=-1)

    def sample(self, rng, m):
        cells = np.minimum(np.searchsorted(self.cdf, rng.uniform(0, 1, m)), self.cdf.size - 1)
        ie, io = np.divmod(cells, self.no)
        E = -math.pi / 2 + (ie + rng.uniform(0, 1, m)) * math.pi / self.ne
        O = -math.pi + (io + rng.uniform(0, 1, m)) * 2 * math.pi / self.no
        xl = self._pos(E, O)
        nl = self._normal(xl)
        return self.c + xl @ self.Rm.T, nl @ self.Rm.T

    def inside(self, x):
        xl = (x - self.c) @ self.Rm
        a, b, c = self.ax
        v = (np.abs(xl[:, 0] / a) ** (2 / self.e2) + np.abs(xl[:, 1] / b) ** (2 / self.e2)) ** (self.e2 / self.e1)
        return v + np.abs(xl[:, 2] / c) ** (2 / self.e1) < 1.0


class _Box(_Part):
    """Closed box with half-extents h (a thin plate when one extent is small)."""

    def __init__(self, c, Rm, h):
        self.c, self.Rm, self.h = np.asarray(c, float), np.asarray(Rm, float), np.asarray(h, float)
        hx, hy, hz = self.h
        self.faces = np.array([hy * hz, hy * hz, hx * hz, hx * hz, hx * hy, hx * hy]) * 4
        self.area = float(self.faces.sum())

    def sample(self, rng, m):
        f = rng.choice(6, size=m, p=self.faces / self.faces.sum())
        u = rng.uniform(-1, 1, (m, 3)) * self.h
        axis, sgn = f // 2, np.where(f % 2 == 0, 1.0, -1.0)
        u[np.arange(m), axis] = sgn * self.h[axis]
        nl = np.zeros((m, 3))
        nl[np.arange(m), axis] = sgn
        return self.c + u @ self.Rm.T, nl @ self.Rm.T

    def inside(self, x):
        xl = (x - self.c) @ self.Rm
        return np.all(np.abs(xl) < self.h, axis=1)


# ----------------------------------------------------------------------------- union
def _union_cloud(parts, n, noise_frac, outlier_frac, rng, oversample=1.25, meta=None):
    """Uniform-by-area samples of the union of closed parts: samples strictly inside another
    part are dropped, the rest subsampled to the inlier count; noise is Gaussian with
    sigma = noise_frac * (clean bbox diagonal) per coordinate; outliers are uniform in the
    clean bounding box and take the mean inlier area weight."""
    n_out = int(round(n * outlier_frac))
    n_in = n - n_out
    tot_area = sum(p.area for p in parts)
    # draw uniform-by-area samples of every part; when heavy overlap leaves fewer than n_in
    # visible samples, draw again with a larger oversampling factor
    while True:
        xs, ns, pid = [], [], []
        vis_area = 0.0
        overlap = np.eye(len(parts), dtype=bool)
        for k, p in enumerate(parts):
            m = int(math.ceil(oversample * n_in * p.area / tot_area)) + 8
            x, nv = p.sample(rng, m)
            keep = np.ones(m, dtype=bool)
            for j, q in enumerate(parts):
                if j != k:
                    ins = q.inside(x)
                    if ins.any():
                        overlap[k, j] = overlap[j, k] = True
                    keep &= ~ins
            vis_area += p.area * keep.mean()
            xs.append(x[keep])
            ns.append(nv[keep])
            pid.append(np.full(int(keep.sum()), k))
        x = np.concatenate(xs)
        nv = np.concatenate(ns)
        pid = np.concatenate(pid)
        if x.shape[0] >= n_in:
            break
        oversample *= 1.25 * n_in / max(x.shape[0], 1)
    sel = rng.choice(x.shape[0], size=n_in, replace=False)
    x, nv, pid = x[sel], nv[sel], pid[sel]
    # connected components of the overlap graph
    comp_of = np.arange(len(parts))
    for _ in range(len(parts)):
        for a in range(len(parts)):
            for b in range(len(parts)):
                if overlap[a, b]:
                    comp_of[a] = comp_of[b] = min(comp_of[a], comp_of[b])
    _, comp_ids = np.unique(comp_of, return_inverse=True)
    comp = comp_ids[pid]
    lo, hi = x.min(0), x.max(0)
    diag = float(np.linalg.norm(hi - lo))
    sigma = noise_frac * diag
    x = x + rng.standard_normal(x.shape) * sigma
    a_in = vis_area / n_in
    xo = rng.uniform(lo, hi, (n_out, 3))
    P = np.concatenate([x, xo])
    N = np.concatenate([nv, np.zeros((n_out, 3))])
    area = np.full(n, a_in)
    cmp_ = np.concatenate([comp, np.full(n_out, -1)])
    inl = np.concatenate([np.ones(n_in, bool), np.zeros(n_out, bool)])
    perm = rng.permutation(n)
    md = dict(meta or {})
    md.update(dict(n_in=n_in, n_out=n_out, sigma=sigma, bbox_diag=diag, visible_area=vis_area,
                   n_components=int(comp_ids.max()) + 1 if len(parts) else 0))
    return Cloud(P=np.ascontiguousarray(P[perm].T.astype(np.float32)),
                 area=area[perm].astype(np.float32),
                 N_true=np.ascontiguousarray(N[perm].T.astype(np.float32)),
                 comp=cmp_[perm].astype(np.int32), inlier=inl[perm], meta=md)


# --------------------------------------------------------------------------- configs
def sphere(n=2000, noise=0.005, seed=100, R=1.0):
    """Unit sphere: i.i.d. uniform points (normalised Gaussians), Gaussian noise
    sigma = noise * R per coordinate, area weights 4 pi R^2 / n."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    x = R * u + rng.standard_normal((n, 3)) * noise * R
    return Cloud(P=np.ascontiguousarray(x.T.astype(np.float32)),
                 area=np.full(n, 4 * math.pi * R * R / n, dtype=np.float32),
                 N_true=np.ascontiguousarray(u.T.astype(np.float32)),
                 comp=np.zeros(n, np.int32), inlier=np.ones(n, bool),
                 meta=dict(kind="sphere", sigma=noise * R, seed=seed))


def torus_ellipsoids(n=100_000, seed=101, noise_frac=0.0025, outlier_frac=0.05, n_ellipsoids=2):
    """Torus (R=1, r=0.3, axis z, at the origin) united with random ellipsoids: semi-axes
    U[0.2,0.6], uniform random orientation, centre U([-1.3,1.3]^2 x [-0.5,0.5])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [_Torus(np.zeros(3), np.eye(3), 1.0, 0.3)]
    for _ in range(n_ellipsoids):
        ax = rng.uniform(0.2, 0.6, 3)
        c = np.array([rng.uniform(-1.3, 1.3), rng.uniform(-1.3, 1.3), rng.uniform(-0.5, 0.5)])
        parts.append(_Ellipsoid(c, _rot(rng), ax))
    return _union_cloud(parts, n, noise_frac, outlier_frac, rng,
                        meta=dict(kind="torus_ellipsoids", seed=seed))


def superquadrics_plates(n=5_000_000, seed=103, noise_frac=0.001, n_sq=8, n_plates=4):
    """Superquadrics (exponents U[0.2,2], axes U[0.2,0.6]) and thin plates (half-extents
    U[0.2,0.6]^2 x 0.005, i.e. thickness 0.01), random poses with centres in [-1.5,1.5]^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _ in range(n_sq):
        parts.append(_Superquadric(rng.uniform(-1.5, 1.5, 3), _rot(rng), rng.uniform(0.2, 0.6, 3),
                                   rng.uniform(0.2, 2.0), rng.uniform(0.2, 2.0), rng))
    for _ in range(n_plates):
        h = np.array([rng.uniform(0.2, 0.6), rng.uniform(0.2, 0.6), 0.005])
        parts.append(_Box(rng.uniform(-1.5, 1.5, 3), _rot(rng), h))
    return _union_cloud(parts, n, noise_frac, 0.0, rng, oversample=1.4,
                        meta=dict(kind="superquadrics_plates", seed=seed))


def ellipsoids_tori(n=15_000_000, seed=104, noise_frac=0.002, outlier_frac=0.02, n_each=10):
    """Ellipsoids (axes U[0.2,0.6]) and tori (R U[0.3,0.7], r U[0.06,0.2]) with random poses,
    centres in [-2,2]^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _ in range(n_each):
        parts.append(_Ellipsoid(rng.uniform(-2, 2, 3), _rot(rng), rng.uniform(0.2, 0.6, 3)))
    for _ in range(n_each):
        parts.append(_Torus(rng.uniform(-2, 2, 3), _rot(rng), rng.uniform(0.3, 0.7), rng.uniform(0.06, 0.2)))
    return _union_cloud(parts, n, noise_frac, outlier_frac, rng,
                        meta=dict(kind="ellipsoids_tori", seed=seed))


def fibonacci_sphere(n, R=1.0):
    """Deterministic near-uniform sphere points (golden-angle spiral), area 4 pi R^2 / n each;
    used for quadrature-accurate closed-form checks."""
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    ph = math.pi * (1 + 5**0.5) * i
    rr = np.sqrt(1 - z * z)
    u = np.stack([rr * np.cos(ph), rr * np.sin(ph), z])
    return Cloud(P=np.ascontiguousarray((R * u).astype(np.float32)),
                 area=np.full(n, 4 * math.pi * R * R / n, dtype=np.float32),
                 N_true=np.ascontiguousarray(u.astype(np.float32)), comp=np.zeros(n, np.int32),
                 inlier=np.ones(n, bool), meta=dict(kind="fibonacci", R=R))


CONFIGS = {
    1: lambda seed=100: sphere(2000, 0.005, seed),
    2: lambda seed=101: torus_ellipsoids(100_000, seed),
    3: lambda seed=102: torus_ellipsoids(1_000_000, seed),
    4: lambda seed=103: superquadrics_plates(5_000_000, seed),
    5: lambda seed=104: ellipsoids_tori(15_000_000, seed),
}
