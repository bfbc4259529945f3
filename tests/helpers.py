"""Shared helpers for tests: small hand-built problems and the parity norm."""
from __future__ import annotations

import numpy as np

from paper_2006_02545_amd import surfaces as S


def flat_patch_problem(verts, d, targets, alpha=1.0, beta=0.0, k=0.0, tol=1e-10,
                       self_nodes=False):
    """One flat triangular patch with corners `verts` (3x3) sampled at the
    degree-d reference nodes; off-surface targets `targets` (M,3) whose near
    list is that patch; optionally every node as a self target as well."""
    verts = np.asarray(verts, dtype=np.float64)
    uv = S.reference_nodes(d)
    xyz = verts[0] + uv[:, :1] * (verts[1] - verts[0]) + uv[:, 1:2] * (verts[2] - verts[0])
    nd = uv.shape[0]
    targets = np.zeros((0, 3)) if targets is None else np.asarray(targets, dtype=np.float64)
    M = targets.shape[0]
    txyz = targets
    not_ = -np.ones(M, dtype=np.int64)
    rows = [[0] for _ in range(M)]
    if self_nodes:
        txyz = np.concatenate([txyz, xyz], 0)
        not_ = np.concatenate([not_, np.arange(nd, dtype=np.int64)])
        rows += [[] for _ in range(nd)]
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    npat = np.array([p for r in rows for p in r], dtype=np.int32)
    return S.Problem(name="flat", degree=np.array([d], np.int32),
                     node_ptr=np.array([0, nd], np.int64), xyz=xyz, ref_nodes={d: uv},
                     target_xyz=txyz, node_of_target=not_, near_row_ptr=rp, near_patch=npat,
                     centers=verts.mean(0)[None], radii=np.array([1.0]), eta=1.25,
                     alpha=complex(alpha), beta=complex(beta), k=complex(k), tol=tol,
                     sigma=np.ones(nd, np.complex128), lam=np.ones(len(rows), np.complex128))


def all_pairs_problem(prob, targets=None, target_nodes=None):
    """Copy of `prob` whose targets see every patch (near list = all patches
    but the target's own), for assembling the full operator on tiny surfaces.
    `targets`: off-surface points; `target_nodes`: node ids used as targets."""
    P = prob.P
    txyz, not_, rows = [], [], []
    if targets is not None:
        for x in np.asarray(targets, dtype=np.float64):
            txyz.append(x)
            not_.append(-1)
            rows.append(list(range(P)))
    if target_nodes is not None:
        for n in target_nodes:
            own = int(np.searchsorted(prob.node_ptr, n, side="right") - 1)
            txyz.append(prob.xyz[n])
            not_.append(int(n))
            rows.append([j for j in range(P) if j != own])
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    out = S.Problem(**{**prob.__dict__})
    out.target_xyz = np.array(txyz, dtype=np.float64).reshape(-1, 3)
    out.node_of_target = np.array(not_, dtype=np.int64)
    out.near_row_ptr = rp
    out.near_patch = np.array([p for r in rows for p in r], dtype=np.int32)
    out.lam = np.ones(len(rows), np.complex128)
    return out


def wilton_potential(tri, x):
    """Closed form of int_T dA / |x - y| over a flat triangle T (3x3 corners).

    Edge decomposition of the uniformly charged triangle potential (Wilton,
    Rao, Glisson, Schaubert, Al-Bundak, Butler, IEEE TAP 32(3), 1984):
      sum_i  P0_i ln((R+_i + l+_i)/(R-_i + l-_i))
             - |d| [atan(P0_i l+_i / (R0_i^2 + |d| R+_i))
                    - atan(P0_i l-_i / (R0_i^2 + |d| R-_i))]
    with d the signed height of x over the plane, P0_i the signed distance
    (in-plane, positive towards the interior) from the projection of x to
    edge i's line, l+-_i the signed positions of the edge ends along the edge
    measured from the foot, R0_i^2 = P0_i^2 + d^2, R+-_i^2 = R0_i^2 + l+-_i^2.
    """
    tri = np.asarray(tri, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    d = np.dot(x - tri[0], n)
    rho = x - d * n
    tot = 0.0
    for i in range(3):
        a, b = tri[i], tri[(i + 1) % 3]
        s = (b - a) / np.linalg.norm(b - a)
        u = np.cross(s, n)  # in-plane normal to the edge, pointing outward
        lp = np.dot(b - rho, s)
        lm = np.dot(a - rho, s)
        P0 = np.dot(a - rho, u)  # signed distance, > 0 when rho is inside
        R0sq = P0 * P0 + d * d
        Rp = np.sqrt(R0sq + lp * lp)
        Rm = np.sqrt(R0sq + lm * lm)
        if abs(P0) > 0:
            tot += P0 * np.log((Rp + lp) / (Rm + lm))
        tot -= abs(d) * (np.arctan2(P0 * lp, R0sq + abs(d) * Rp)
                         - np.arctan2(P0 * lm, R0sq + abs(d) * Rm))
    return tot


def solid_angle(tri, x):
    """Signed solid angle of a flat triangle seen from x (Van Oosterom and
    Strackee, IEEE TBME 30(2), 1983): tan(Om/2) = a.(b x c) / (abc + (a.b)c
    + (a.c)b + (b.c)a), a, b, c the corners relative to x.  Negative when x
    is on the side the corner-order normal (B-A)x(C-A) points to."""
    a, b, c = (np.asarray(v, dtype=np.float64) - np.asarray(x, dtype=np.float64) for v in tri)
    la, lb, lc = np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)
    num = np.dot(a, np.cross(b, c))
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    return 2.0 * np.arctan2(num, den)


def node_jacobians(run, prob, j):
    """J(u_l, v_l) at the nodes of patch j, from the oracle's chart."""
    d = int(prob.degree[j])
    out = []
    for (u, v) in prob.ref_nodes[d]:
        _, Xu, Xv = run.chart(j, u, v)
        out.append(np.linalg.norm(np.cross(Xu, Xv)))
    return np.array(out)


def dual_norm_error(a, b, Jl, wl):
    """|| W^{-1} (a - b) ||_2 with W = diag(sqrt(J_l |w_l|)): the dual of the
    L2(Gamma_j) norm of a density sampled at the nodes (paper's error
    analysis, Section 4.2)."""
    W = np.sqrt(np.asarray(Jl) * np.abs(np.asarray(wl)))
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)) / W))
