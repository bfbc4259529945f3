"""Seeded synthetic inputs: surfaces, reference nodes, near lists, densities.

This module builds the *inputs* of the near-field correction generator and
nothing else.  It holds none of the method's arithmetic (no Koornwinder basis,
no quadrature of the layer-potential kernels, no interpolation matrices); both
the HIP path and the CPU oracle consume what it returns.

Inputs follow the paper's problem statement (Section 5.2, "Precomputation"):
curved triangular patches, each given by samples of its chart at the
interpolation nodes of the reference simplex T0 (Section 2), a set of targets
(here every discretisation node, i.e. on-surface targets), and for every
target the list T_eta(x) of patches whose near-field ball B_{eta R_j}(c_j)
strictly contains it (Section 4, near-field definitions; the strict test is
the one used by the near-list algorithm of Section 5.2).

Readings that the paper leaves open are fixed here and listed in the design doc:
 * interpolation nodes: the paper's Vioreanu-Rokhlin nodes are not printed;
   we use approximate Fekete points (greedy column-pivoted QR on a Chebyshev
   tensor Vandermonde over a lattice strictly inside T0);
 * patch centre c_j: mean of the patch map over a uniform lattice of T0
   (approximates the parametric mean); R_j: max distance from c_j over the
   same lattice including the edges.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
from scipy.spatial import cKDTree

__all__ = [
    "n_nodes", "reference_nodes", "Problem", "sphere_problem", "mixed_problem",
    "star_problem", "config", "CONFIG_NAMES",
]


def n_nodes(d: int) -> int:
    """Number of interpolation nodes for total degree <= d: (d+1)(d+2)/2."""
    return (d + 1) * (d + 2) // 2


# --------------------------------------------------------------------------
# Reference interpolation nodes on T0 = {u >= 0, v >= 0, u + v <= 1}
# --------------------------------------------------------------------------
_NODE_CACHE: dict[int, np.ndarray] = {}


def _cheb(k: int, x: np.ndarray) -> np.ndarray:
    return np.cos(k * np.arccos(np.clip(x, -1.0, 1.0)))


def reference_nodes(d: int) -> np.ndarray:
    """Interior, unisolvent interpolation nodes for polynomials of degree <= d.

    Approximate Fekete points: candidates are the points of a barycentric
    lattice of the triangle shrunk by a margin (all three barycentric
    coordinates >= margin); the first n_d pivots of a column-pivoted QR of the
    transposed Vandermonde of the tensor Chebyshev basis T_a(2u-1) T_b(2v-1),
    a + b <= d, are kept.  The margin is the first Gauss-Legendre abscissa of
    a (d+1)-point rule on [0, 1], which keeps nodes about as close to the
    patch edges as Gauss-type interior nodes of that order are.
    Returns an (n_d, 2) float64 array of (u, v).
    """
    if d in _NODE_CACHE:
        return _NODE_CACHE[d].copy()
    if d < 0 or d > 12:
        raise ValueError("degree out of range")
    nd = n_nodes(d)
    if d == 0:
        out = np.array([[1.0 / 3.0, 1.0 / 3.0]])
        _NODE_CACHE[d] = out
        return out.copy()
    x, _ = np.polynomial.legendre.leggauss(d + 1)
    margin = 0.5 * (x[0] + 1.0)
    M = 24 * (d + 1)
    ii, jj = np.meshgrid(np.arange(M + 1), np.arange(M + 1), indexing="ij")
    keep = ii + jj <= M
    b1 = ii[keep] / M
    b2 = jj[keep] / M
    s = 1.0 - 3.0 * margin
    u = margin + s * b1
    v = margin + s * b2
    cols = []
    for a in range(d + 1):
        for b in range(d + 1 - a):
            cols.append(_cheb(a, 2 * u - 1) * _cheb(b, 2 * v - 1))
    vand = np.stack(cols, axis=0)  # (nd, ncand)
    _, _, piv = scipy.linalg.qr(vand, pivoting=True, mode="economic")
    sel = piv[:nd]
    out = np.stack([u[sel], v[sel]], axis=1)
    _NODE_CACHE[d] = out
    return out.copy()


# --------------------------------------------------------------------------
# Triangulated closed surfaces
# --------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    # outward orientation: (B-A)x(C-A) . centroid > 0
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c)
    f[s < 0] = f[s < 0][:, [0, 2, 1]]
    return v, f


def _subdivide_projected(v, f, levels):
    """Recursive 1->4 midpoint subdivision, projecting new vertices to S^2."""
    verts = [tuple(x) for x in v]
    for _ in range(levels):
        cache = {}
        newf = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                p = (np.array(verts[i]) + np.array(verts[j])) * 0.5
                p /= np.linalg.norm(p)
                cache[key] = len(verts)
                verts.append(tuple(p))
            return cache[key]

        for (a, b, c) in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newf += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        f = np.array(newf, dtype=np.int64)
    return np.array(verts), f


def _geodesic_faces(freq):
    """Frequency-`freq` geodesic subdivision of the icosahedron.

    Returns the flat triangles' corner points (T, 3, 3) on the icosahedron's
    faces (not yet projected) with outward orientation; 20 * freq^2 faces.
    """
    v, f = _icosahedron()
    tris = []
    for (ia, ib, ic) in f:
        A, B, C = v[ia], v[ib], v[ic]

        def P(i, j):
            return A + (i / freq) * (B - A) + (j / freq) * (C - A)

        for i in range(freq):
            for j in range(freq - i):
                tris.append((P(i, j), P(i + 1, j), P(i, j + 1)))
                if i + j < freq - 1:
                    tris.append((P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)))
    return np.array(tris, dtype=np.float64)


# Patch maps T0 -> R^3.  Each map is vectorised: corners (P,3,3) [or extra
# data], uv (L,2) -> points (P,L,3).

def _quad_map(ctrl, uv):
    """6-node quadratic Lagrange map.  ctrl: (P,6,3) = A,B,C,M_AB,M_BC,M_CA."""
    u, v = uv[:, 0], uv[:, 1]
    l0, l1, l2 = 1.0 - u - v, u, v
    N = np.stack([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                  4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0], axis=1)  # (L,6)
    return np.einsum("lk,pkc->plc", N, ctrl)


def _flat(corners, uv):
    A = corners[:, 0, :][:, None, :]
    B = corners[:, 1, :][:, None, :]
    C = corners[:, 2, :][:, None, :]
    return A + uv[None, :, 0:1] * (B - A) + uv[None, :, 1:2] * (C - A)


def _ellipsoid_map(corners, uv, axes):
    p = _flat(corners, uv)
    p = p / np.linalg.norm(p, axis=2, keepdims=True)
    return p * np.asarray(axes)[None, None, :]


def _real_sph_harm(l, m, xyz):
    """Real orthonormal spherical harmonic Y_lm on unit vectors xyz (...,3)."""
    from scipy.special import sph_harm_y
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    Y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * np.real(Y)
    return math.sqrt(2.0) * (-1) ** m * np.imag(Y)


def _star_map(corners, uv, harm):
    p = _flat(corners, uv)
    dirs = p / np.linalg.norm(p, axis=2, keepdims=True)
    r = np.ones(dirs.shape[:2])
    for (l, m, c) in harm:
        r = r + 0.2 * c * _real_sph_harm(l, m, dirs)
    return dirs * r[..., None]


def _torus_map(params, uv, R0=2.0):
    """params: (P,3,2) corner (theta, phi) of a grid triangle."""
    A = params[:, 0, :][:, None, :]
    B = params[:, 1, :][:, None, :]
    C = params[:, 2, :][:, None, :]
    tp = A + uv[None, :, 0:1] * (B - A) + uv[None, :, 1:2] * (C - A)
    th, ph = tp[..., 0], tp[..., 1]
    r = 0.5 + 0.05 * np.sin(3 * th) * np.cos(5 * ph)
    rho = R0 + r * np.cos(ph)
    return np.stack([rho * np.cos(th), rho * np.sin(th), r * np.sin(ph)], axis=-1)


def _lattice(L):
    pts = [(i / L, j / L) for i in range(L + 1) for j in range(L + 1 - i)]
    return np.array(pts, dtype=np.float64)


# --------------------------------------------------------------------------
# Problem container
# --------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    degree: np.ndarray          # (P,) int32
    node_ptr: np.ndarray        # (P+1,) int64
    xyz: np.ndarray             # (N,3) float64, patch nodes, patch-major
    ref_nodes: dict             # d -> (n_d,2) float64
    target_xyz: np.ndarray      # (N_T,3)
    node_of_target: np.ndarray  # (N_T,) int64, node id or -1
    near_row_ptr: np.ndarray    # (N_T+1,) int64  (CSR by target)
    near_patch: np.ndarray      # (nnz,) int32, ascending per row, self excluded
    centers: np.ndarray         # (P,3)
    radii: np.ndarray           # (P,)
    eta: float
    alpha: complex
    beta: complex
    k: complex
    tol: float
    sigma: np.ndarray           # (N,) density (complex128, or float64 if real kernel)
    lam: np.ndarray             # (N_T,) adjoint vector
    meta: dict = field(default_factory=dict)

    @property
    def P(self):
        return int(self.degree.shape[0])

    @property
    def N(self):
        return int(self.xyz.shape[0])

    @property
    def NT(self):
        return int(self.target_xyz.shape[0])

    @property
    def real_kernel(self):
        return (self.k == 0 and self.alpha.imag == 0 and self.beta.imag == 0)

    def subset_targets(self, idx):
        """Copy restricted to the targets `idx` (near rows kept as is)."""
        idx = np.asarray(idx, dtype=np.int64)
        rows = [self.near_patch[self.near_row_ptr[t]:self.near_row_ptr[t + 1]] for t in idx]
        rp = np.zeros(len(idx) + 1, dtype=np.int64)
        rp[1:] = np.cumsum([len(r) for r in rows])
        np_ = np.concatenate(rows).astype(np.int32) if len(rows) else np.zeros(0, np.int32)
        out = Problem(**{**self.__dict__})
        out.target_xyz = self.target_xyz[idx].copy()
        out.node_of_target = self.node_of_target[idx].copy()
        out.near_row_ptr = rp
        out.near_patch = np_
        out.lam = self.lam[idx].copy() if self.lam is not None else None
        out.meta = dict(self.meta, target_subset=True)
        return out


def _assemble(name, degree, mapfn, mapdata, eta, alpha, beta, k, tol, rng,
              sigma_fn, lattice=32, chunk=20000):
    """Sample patches at their nodes, build centres/radii and the near list."""
    degree = np.asarray(degree, dtype=np.int32)
    P = degree.shape[0]
    nn = np.array([n_nodes(int(d)) for d in degree], dtype=np.int64)
    node_ptr = np.zeros(P + 1, dtype=np.int64)
    node_ptr[1:] = np.cumsum(nn)
    N = int(node_ptr[-1])
    xyz = np.empty((N, 3), dtype=np.float64)
    ref = {int(d): reference_nodes(int(d)) for d in np.unique(degree)}
    for d, uv in ref.items():
        sel = np.nonzero(degree == d)[0]
        for s0 in range(0, len(sel), chunk):
            s = sel[s0:s0 + chunk]
            pts = mapfn(mapdata[s], uv)  # (len(s), n_d, 3)
            offs = node_ptr[s][:, None] + np.arange(uv.shape[0])[None, :]
            xyz[offs.reshape(-1)] = pts.reshape(-1, 3)
    lat = _lattice(lattice)
    centers = np.empty((P, 3))
    radii = np.empty(P)
    for s0 in range(0, P, chunk):
        pts = mapfn(mapdata[s0:s0 + chunk], lat)
        c = pts.mean(axis=1)
        centers[s0:s0 + chunk] = c
        radii[s0:s0 + chunk] = np.linalg.norm(pts - c[:, None, :], axis=2).max(axis=1)
    # near lists: targets = all nodes
    target_patch = np.repeat(np.arange(P, dtype=np.int64), nn)
    tree = cKDTree(xyz)
    hits = tree.query_ball_point(centers, eta * radii * (1.0 + 1e-9))
    pair_t, pair_p = [], []
    for j in range(P):
        h = np.asarray(hits[j], dtype=np.int64)
        if h.size == 0:
            continue
        dist = np.linalg.norm(xyz[h] - centers[j], axis=1)
        gap = np.abs(dist - eta * radii[j])
        if np.any(gap <= 1e-12 * radii[j]):
            raise RuntimeError("target on a near-field sphere; perturb the input")
        h = h[(dist < eta * radii[j]) & (target_patch[h] != j)]
        pair_t.append(h)
        pair_p.append(np.full(h.size, j, dtype=np.int64))
    pt = np.concatenate(pair_t) if pair_t else np.zeros(0, np.int64)
    pp = np.concatenate(pair_p) if pair_p else np.zeros(0, np.int64)
    order = np.lexsort((pp, pt))
    pt, pp = pt[order], pp[order]
    counts = np.bincount(pt, minlength=N)
    rp = np.zeros(N + 1, dtype=np.int64)
    rp[1:] = np.cumsum(counts)
    sigma, lam = sigma_fn(xyz, rng)
    return Problem(name=name, degree=degree, node_ptr=node_ptr, xyz=xyz, ref_nodes=ref,
                   target_xyz=xyz.copy(), node_of_target=np.arange(N, dtype=np.int64),
                   near_row_ptr=rp, near_patch=pp.astype(np.int32), centers=centers,
                   radii=radii, eta=eta, alpha=complex(alpha), beta=complex(beta),
                   k=complex(k), tol=float(tol), sigma=sigma, lam=lam, meta={})


def _sphere_quadratic_ctrl(levels):
    v, f = _icosahedron()
    v, f = _subdivide_projected(v, f, levels)
    A, B, C = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]

    def proj(p):
        return p / np.linalg.norm(p, axis=1, keepdims=True)

    ctrl = np.stack([A, B, C, proj(A + B), proj(B + C), proj(C + A)], axis=1)
    return ctrl


def _complex_gauss(rng, n):
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2.0)


def sphere_problem(levels, degree, alpha, beta, k, tol, seed, density="uniform",
                   eta=1.25, name=None):
    """Unit sphere: icosahedron, `levels` projected midpoint subdivisions,
    quadratic patches through the 3 projected vertices and the 3 projected
    flat-edge midpoints, sampled at the degree-`degree` nodes."""
    ctrl = _sphere_quadratic_ctrl(levels)
    P = ctrl.shape[0]
    rng = np.random.default_rng(seed)
    real = (k == 0 and np.imag(alpha) == 0 and np.imag(beta) == 0)

    def sig(xyz, rng):
        N = xyz.shape[0]
        if density == "uniform":
            s = rng.uniform(-1.0, 1.0, N)
            s = s if real else s.astype(np.complex128)
            lam = rng.uniform(-1.0, 1.0, N) if real else _complex_gauss(rng, N)
        elif density == "sph":
            lm = [(l, m) for l in range(7) for m in range(-l, l + 1)]
            pick = rng.choice(len(lm), size=20, replace=False)
            coef = _complex_gauss(rng, 20)
            dirs = xyz / np.linalg.norm(xyz, axis=1, keepdims=True)
            s = np.zeros(N, dtype=np.complex128)
            for c, i in zip(coef, pick):
                l, m = lm[i]
                s += c * _real_sph_harm(l, m, dirs)
            lam = _complex_gauss(rng, N)
        elif density == "gauss":
            s = _complex_gauss(rng, N)
            lam = _complex_gauss(rng, N)
        else:
            raise ValueError(density)
        return s, lam

    return _assemble(name or f"sphere{P}_d{degree}", np.full(P, degree), _quad_map, ctrl,
                     eta, alpha, beta, k, tol, rng, sig)


def mixed_problem(seed=3, tol=1e-8, k=10.0, eta=1.25, ell_freq=10, tor_grid=(80, 25),
                  dmin=2, dmax=8):
    """3:2:1 ellipsoid (frequency-10 geodesic icosphere, 2000 patches) plus a
    perturbed torus (80 x 25 grid, 4000 patches), degrees uniform in
    [dmin, dmax] per patch, combined field D - ik S."""
    rng = np.random.default_rng(seed)
    ell = _geodesic_faces(ell_freq)
    nth, nph = tor_grid
    th = np.linspace(0, 2 * np.pi, nth + 1)
    ph = np.linspace(0, 2 * np.pi, nph + 1)
    tri = []
    for i in range(nth):
        for j in range(nph):
            a, b = (th[i], ph[j]), (th[i + 1], ph[j])
            c, dd = (th[i + 1], ph[j + 1]), (th[i], ph[j + 1])
            tri.append((a, b, c))
            tri.append((a, c, dd))
    tor = np.array(tri, dtype=np.float64)
    # orientation of torus triangles: make the normal outward
    t_test = _torus_map(tor[:1], np.array([[1 / 3, 1 / 3], [1 / 3 + 1e-6, 1 / 3], [1 / 3, 1 / 3 + 1e-6]]))[0]
    nrm = np.cross(t_test[1] - t_test[0], t_test[2] - t_test[0])
    cen = t_test[0]
    axis_pt = 2.0 * np.array([cen[0], cen[1], 0.0]) / np.linalg.norm(cen[:2])
    if np.dot(nrm, cen - axis_pt) < 0:
        tor = tor[:, [0, 2, 1], :]
    P1, P2 = ell.shape[0], tor.shape[0]
    degree = rng.integers(dmin, dmax + 1, size=P1 + P2)
    axes = (1.5, 1.0, 0.5)

    # composite map: index < P1 -> ellipsoid, else torus; mapdata = index array
    class _Data:
        def __getitem__(self, s):
            return np.arange(P1 + P2)[s]

    def mapfn(idx, uv):
        idx = np.asarray(idx)
        out = np.empty((idx.size, uv.shape[0], 3))
        m1 = idx < P1
        if np.any(m1):
            out[m1] = _ellipsoid_map(ell[idx[m1]], uv, axes)
        if np.any(~m1):
            out[~m1] = _torus_map(tor[idx[~m1] - P1], uv)
        return out

    def sig(xyz, rng):
        N = xyz.shape[0]
        return _complex_gauss(rng, N), _complex_gauss(rng, N)

    return _assemble("mixed_ellipsoid_torus", degree, mapfn, _Data(), eta, -1j * k, 1.0, k,
                     tol, rng, sig)


def star_problem(freq=100, degree=6, seed=5, tol=1e-9, k=20.0, eta=1.25, lattice=8):
    """Star-shaped surface r = 1 + 0.2 sum_i c_i Y_i (10 real harmonics of
    degree <= 4, c_i ~ N(0,1)/10) on a frequency-`freq` geodesic icosphere."""
    rng = np.random.default_rng(seed)
    lm = [(l, m) for l in range(5) for m in range(-l, l + 1)]
    pick = rng.choice(len(lm), size=10, replace=False)
    coef = rng.standard_normal(10) / 10.0
    harm = [(lm[i][0], lm[i][1], c) for i, c in zip(pick, coef)]
    faces = _geodesic_faces(freq)
    P = faces.shape[0]

    def mapfn(c, uv):
        return _star_map(c, uv, harm)

    def sig(xyz, rng):
        N = xyz.shape[0]
        return _complex_gauss(rng, N), _complex_gauss(rng, N)

    return _assemble(f"star{P}_d{degree}", np.full(P, degree), mapfn, faces, eta, -1j * k, 1.0,
                     k, tol, rng, sig, lattice=lattice)


CONFIG_NAMES = ("laplace_s_sphere80_d3", "cfie_sphere1280_d4", "mixed_ellipsoid_torus",
                "cfie_sphere320_d4_adjoint", "star200k_d6")


def config(i: int) -> Problem:
    """The five workloads of the measurement plan, 0-based."""
    if i == 0:
        return sphere_problem(1, 3, 1.0, 0.0, 0.0, 1e-6, seed=1, density="uniform",
                              name=CONFIG_NAMES[0])
    if i == 1:
        k = 2.0 * math.pi
        return sphere_problem(3, 4, -1j * k, 1.0, k, 1e-8, seed=2, density="sph",
                              name=CONFIG_NAMES[1])
    if i == 2:
        return mixed_problem()
    if i == 3:
        return sphere_problem(2, 4, -5j, 1.0, 5.0, 1e-10, seed=4, density="gauss",
                              name=CONFIG_NAMES[3])
    if i == 4:
        return star_problem()
    raise ValueError(i)
