"""Pins of the CPU oracle against facts that do not come from the oracle:
closed forms, library routines, textbook identities and the paper's own
statements.  CPU only.

Each test names the passage of the paper (Greengard, O'Neil, Rachh, Vico,
arXiv 2006.02545) or the external result it checks.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special

import oracle
from paper_2006_02545_amd import surfaces as S
from tests.helpers import (all_pairs_problem, dual_norm_error, flat_patch_problem,
                           node_jacobians, solid_angle, wilton_potential)


def _duffy_gauss(n):
    """Tensor Gauss-Legendre on T0 through u = x(1-y), v = y (numpy's rule,
    independent of the oracle's own rules)."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = (x + 1) / 2
    w = w / 2
    X, Y = np.meshgrid(x, x, indexing="ij")
    WX, WY = np.meshgrid(w, w, indexing="ij")
    u = (X * (1 - Y)).ravel()
    v = Y.ravel()
    wt = (WX * WY * (1 - Y)).ravel()
    return u, v, wt


# ---------------------------------------------------------------- Section 2

@pytest.mark.parametrize("d", [0, 1, 2, 4, 6, 8])
def test_koornwinder_orthonormal(d):
    """Section 2: Koornwinder polynomials are orthonormal on T0 (the paper
    fixes c_nm by unit L2 norm; orthogonality as (n,m) != (n',m'))."""
    u, v, w = _duffy_gauss(16)
    nd = (d + 1) * (d + 2) // 2
    G = np.zeros((nd, nd))
    for ui, vi, wi in zip(u, v, w):
        K, _, _ = oracle.koornwinder(d, ui, vi)
        G += wi * np.outer(K, K)
    assert np.abs(G - np.eye(nd)).max() < 1e-13


@pytest.mark.parametrize("d", [2, 5, 8])
def test_koornwinder_degree_and_derivatives(d):
    """K_nm has total degree n (Section 2); derivatives match central
    differences of the values."""
    rng = np.random.default_rng(d)
    for _ in range(5):
        u, v = rng.uniform(0.05, 0.45, 2)
        K, Ku, Kv = oracle.koornwinder(d, u, v)
        h = 1e-6
        Kp, _, _ = oracle.koornwinder(d, u + h, v)
        Km, _, _ = oracle.koornwinder(d, u - h, v)
        assert np.allclose((Kp - Km) / (2 * h), Ku, atol=1e-7 * (1 + np.abs(Ku).max()))
        Kp, _, _ = oracle.koornwinder(d, u, v + h)
        Km, _, _ = oracle.koornwinder(d, u, v - h)
        assert np.allclose((Kp - Km) / (2 * h), Kv, atol=1e-7 * (1 + np.abs(Kv).max()))
    # total degree: K_nm along a line is a polynomial of degree n -> the
    # (n+1)-th finite difference vanishes
    t = np.linspace(0.0, 0.3, d + 3)
    vals = np.array([oracle.koornwinder(d, 0.1 + 0.5 * s, 0.2 + 0.3 * s)[0] for s in t])
    diffs = np.diff(vals, n=d + 1, axis=0)
    assert np.abs(diffs).max() < 1e-8


@pytest.mark.parametrize("n,a", [(1, 0), (5, 0), (12, 0), (20, 0), (3, 1), (9, 1), (16, 1)])
def test_gauss_jacobi_against_scipy(n, a):
    """Gauss(-Jacobi) rules against scipy.special.roots_jacobi."""
    y, w = oracle.gauss_jacobi(n, a, 0)
    x, wx = scipy.special.roots_jacobi(n, a, 0)
    order = np.argsort(y)
    assert np.allclose(y[order], (x + 1) / 2, atol=1e-14)
    assert np.allclose(w[order], wx / 2 ** (a + 1), rtol=1e-12)


@pytest.mark.parametrize("ng", [1, 3, 6, 8, 10])
def test_conical_rule_exactness(ng):
    """The subtriangle rule integrates u^a v^b exactly for a + b <= 2 ng - 1:
    int_T0 u^a v^b = a! b! / (a + b + 2)!."""
    r = oracle.conical_rule(ng)
    for a in range(2 * ng):
        for b in range(2 * ng - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            q = np.sum(r[:, 2] * r[:, 0] ** a * r[:, 1] ** b)
            assert abs(q - exact) <= 1e-14 * max(1.0, exact) + 1e-16
    assert np.all(r[:, 0] > 0) and np.all(r[:, 1] > 0) and np.all(r[:, 0] + r[:, 1] < 1)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 6, 8])
def test_vandermonde_inverse_and_weights(d):
    """Section 2.1: U_(nm),j = K_nm(u_j,v_j), V = U^{-1} maps node values to
    coefficients; the cardinal functions sum_nm V_(nm),l K_nm are Lagrange
    polynomials; interpolatory weights integrate degree-d polynomials
    exactly and sum to |T0| = 1/2; ||V||_2 equals numpy's spectral norm."""
    uv = S.reference_nodes(d)
    V, nv, w = oracle.reference(d, uv)
    nd = uv.shape[0]
    U = np.stack([oracle.koornwinder(d, u, v)[0] for (u, v) in uv], axis=1)  # [nm][j]
    assert np.abs(V @ U.T - np.eye(nd)).max() < 1e-11 * max(1, np.abs(V).max())
    card = V.T @ U  # card[l][m] = L_l(node m)
    assert np.abs(card - np.eye(nd)).max() < 1e-11
    assert abs(nv - np.linalg.norm(V, 2)) < 1e-12 * nv
    assert abs(w.sum() - 0.5) < 1e-14
    for a in range(d + 1):
        for b in range(d + 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.dot(w, uv[:, 0] ** a * uv[:, 1] ** b) - exact) < 1e-13


# ----------------------------------------- Sections 3-4: flat triangles

TRI = np.array([[0.1, -0.2, 0.05], [1.1, 0.1, -0.1], [0.2, 0.9, 0.2]])


def test_wilton_formula_against_scipy():
    """The closed form used below agrees with scipy's adaptive cubature."""
    n = np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0])
    nh = n / np.linalg.norm(n)
    for x in [TRI.mean(0) + 0.3 * nh, TRI.mean(0) - 0.05 * nh, TRI[0] + np.array([0.7, 0.2, 0.4])]:
        def f(v, u):
            y = TRI[0] + u * (TRI[1] - TRI[0]) + v * (TRI[2] - TRI[0])
            return np.linalg.norm(n) / np.linalg.norm(x - y)
        ref, _ = scipy.integrate.dblquad(f, 0, 1, 0, lambda u: 1 - u, epsabs=1e-13, epsrel=1e-12)
        assert abs(wilton_potential(TRI, x) - ref) < 1e-9 * abs(ref)

        def g(v, u):
            y = TRI[0] + u * (TRI[1] - TRI[0]) + v * (TRI[2] - TRI[0])
            r = x - y
            return np.dot(n, r) / np.linalg.norm(r) ** 3
        ref2, _ = scipy.integrate.dblquad(g, 0, 1, 0, lambda u: 1 - u, epsabs=1e-13, epsrel=1e-12)
        assert abs(-solid_angle(TRI, x) - ref2) < 1e-8 * max(1, abs(ref2))


@pytest.mark.parametrize("dist", [2.0, 0.5, 1e-1, 1e-2, 1e-3, 1e-4])
@pytest.mark.parametrize("mode", [oracle.METHOD, oracle.TRUTH])
def test_flat_single_layer_closed_form(dist, mode):
    """Laplace single layer of a flat patch: since the cardinal functions sum
    to one, sum_l a_l(x) = int_T G_0 dA = wilton / (4 pi), for targets at
    several heights above an interior point and beside an edge."""
    n = np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0])
    nh = n / np.linalg.norm(n)
    edge_mid = 0.5 * (TRI[0] + TRI[1])
    out_dir = np.cross(TRI[1] - TRI[0], nh)
    out_dir /= np.linalg.norm(out_dir)
    targets = [TRI.mean(0) + dist * nh, edge_mid + dist * out_dir, TRI[2] - dist * nh]
    tol = 1e-10
    prob = flat_patch_problem(TRI, 4, targets, alpha=1, beta=0, k=0, tol=tol)
    run = oracle.OracleRun(prob, mode=mode)
    for t, x in enumerate(targets):
        a = run.pair(t, 0)
        exact = wilton_potential(TRI, x) / (4 * math.pi)
        # error bound of Section 4.3 for sigma = 1: eps ||1||_{L2(patch)}
        area = 0.5 * np.linalg.norm(n)
        bound = (1e-12 if mode == oracle.TRUTH else 10 * tol) * math.sqrt(area)
        assert abs(a.sum() - exact) <= bound + 1e-14 * abs(exact), (t, a.sum(), exact)


@pytest.mark.parametrize("dist", [1e-6, 1e-8])
def test_method_rounding_floor_near_coincident(dist):
    """Targets almost on a flat patch (above an interior point, beside an
    edge, above a corner): the method's test reaches its double-precision
    rounding floor there.  The trees stay small (accepted at the floor, not
    refined to the depth limit) and the single and double layers keep the
    Section 4.3 error bound against the closed forms (Wilton et al.;
    Van Oosterom-Strackee)."""
    n = np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0])
    nh = n / np.linalg.norm(n)
    area = 0.5 * np.linalg.norm(n)
    edge_mid = 0.5 * (TRI[0] + TRI[1])
    out_dir = np.cross(TRI[1] - TRI[0], nh)
    out_dir /= np.linalg.norm(out_dir)
    targets = [TRI.mean(0) + dist * nh, edge_mid + dist * out_dir + dist * nh,
               0.9 * TRI[2] + 0.1 * TRI.mean(0) + dist * nh]
    tol = 1e-8
    for al, be, exact_fn in [(1.0, 0.0, lambda x: wilton_potential(TRI, x) / (4 * math.pi)),
                             (0.0, 1.0, lambda x: -solid_angle(TRI, x) / (4 * math.pi))]:
        prob = flat_patch_problem(TRI, 4, targets, alpha=al, beta=be, k=0, tol=tol)
        # depth 30: a point-like near-singularity at height h needs ~log2(1/h) levels
        run = oracle.OracleRun(prob, mode=oracle.METHOD, max_depth=30)
        for t, x in enumerate(targets):
            c0 = run.stats.checks
            a = run.pair(t, 0)
            checks = run.stats.checks - c0
            exact = exact_fn(x)
            assert run.stats.nonconverged == 0
            assert checks < 1000, (t, checks)
            assert abs(a.sum() - exact) <= 10 * tol * math.sqrt(area), (al, be, t, a.sum(), exact)


@pytest.mark.parametrize("dist", [1.0, 1e-1, 1e-2, 1e-3])
def test_flat_double_layer_solid_angle(dist):
    """Laplace double layer n.grad_y G_0 of a flat patch: sum_l a_l(x) equals
    minus the signed solid angle over 4 pi (positive on the side the normal
    X_u x X_v points to, Section 3.1)."""
    n = np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0])
    nh = n / np.linalg.norm(n)
    targets = [TRI.mean(0) + dist * nh, TRI.mean(0) - dist * nh,
               0.5 * (TRI[1] + TRI[2]) + dist * (nh + 0.3 * (TRI[1] - TRI[0]))]
    prob = flat_patch_problem(TRI, 3, targets, alpha=0, beta=1, k=0, tol=1e-10)
    run = oracle.OracleRun(prob, mode=oracle.TRUTH)
    for t, x in enumerate(targets):
        s = run.pair(t, 0).sum()
        exact = -solid_angle(TRI, x) / (4 * math.pi)
        assert abs(s - exact) < 1e-11, (t, s, exact)
    assert run.pair(0, 0).sum().real > 0


@pytest.mark.parametrize("d", [2, 4])
def test_flat_self_patch(d):
    """Self interaction on a flat patch: the double layer vanishes
    identically (n.(x-y) = 0 in-plane); the single layer sums to the
    in-plane potential of the triangle (closed form with zero height)."""
    prob = flat_patch_problem(TRI, d, None, alpha=0, beta=1, k=0, tol=1e-10, self_nodes=True)
    # method mode only: with an exactly vanishing integrand the truth mode's
    # purely relative guards have nothing to hold on to
    run = oracle.OracleRun(prob, mode=oracle.METHOD)
    for t in range(prob.NT):
        assert np.abs(run.pair(t, 0)).max() < 1e-14
    prob = flat_patch_problem(TRI, d, None, alpha=1, beta=0, k=0, tol=1e-10, self_nodes=True)
    run = oracle.OracleRun(prob, mode=oracle.TRUTH)
    for t in range(prob.NT):
        exact = wilton_potential(TRI, prob.target_xyz[t]) / (4 * math.pi)
        assert abs(run.pair(t, 0).sum() - exact) < 1e-11 * abs(exact)


def test_polynomial_density_against_scipy():
    """For a degree-d density p sampled at the nodes, sum_l a_l p_l equals
    int_T G_k p J on the curved chart (interpolation reproduces p): checked
    against scipy's adaptive cubature on a curved sphere patch, Helmholtz
    combined field, near target."""
    prob = S.sphere_problem(1, 3, -2j, 1.0, 2.0, 1e-10, seed=0)
    run = oracle.OracleRun(prob, mode=oracle.TRUTH)
    j = 5
    d = 3
    uv = prob.ref_nodes[d]
    c = prob.centers[j]
    t_far = None
    for t in range(prob.NT):
        if prob.node_of_target[t] // 10 != j and np.linalg.norm(prob.target_xyz[t] - c) < 1.2 * prob.radii[j]:
            t_far = t
            break
    assert t_far is not None
    x = prob.target_xyz[t_far]

    def p(u, v):
        return 1.0 + 2.0 * u - v + 0.5 * u * v - u ** 3 + 0.3 * v ** 2

    a = run.pair(t_far, j)
    lhs = np.sum(a * np.array([p(u, v) for (u, v) in uv]))
    k = 2.0

    def integrand(v, u, part):
        X, Xu, Xv = run.chart(j, u, v)
        n = np.cross(Xu, Xv)
        r = x - X
        rr = np.linalg.norm(r)
        e = np.exp(1j * k * rr)
        val = -2j * e / (4 * np.pi * rr) * np.linalg.norm(n) + np.dot(n, r) * (1 - 1j * k * rr) * e / (4 * np.pi * rr ** 3)
        val *= p(u, v)
        return val.real if part == 0 else val.imag

    re, _ = scipy.integrate.dblquad(integrand, 0, 1, 0, lambda u: 1 - u, args=(0,), epsabs=1e-12, epsrel=1e-11)
    im, _ = scipy.integrate.dblquad(integrand, 0, 1, 0, lambda u: 1 - u, args=(1,), epsabs=1e-12, epsrel=1e-11)
    assert abs(lhs - (re + 1j * im)) < 1e-9 * abs(lhs)


# ------------------------------------ full operator on a closed surface

def test_gauss_identity():
    """Double layer of density 1 over the closed (watertight) quadratic
    sphere: -1 inside, -1/2 on the surface (principal value, Section 3),
    0 outside; exact for the discretised surface, so it tests every
    quadrature path (near, self, far) at once."""
    prob = S.sphere_problem(1, 4, 1.0, 0.0, 0.0, 1e-9, seed=0)
    inside = [np.array([0.1, -0.2, 0.3]), np.array([0.0, 0.0, 0.95])]
    outside = [np.array([0.5, 0.9, 0.2]), np.array([0.0, 0.0, 1.05])]
    nodes = [0, 7, 600]
    full = all_pairs_problem(prob, targets=inside + outside, target_nodes=nodes)
    run = oracle.OracleRun(full, mode=oracle.METHOD, alpha=0.0, beta=1.0, k=0.0, tol=1e-9)
    rp, col, val = run.generate()
    y = oracle.apply(rp, col, val, np.ones(prob.N))
    expect = [-1, -1, 0, 0, -0.5, -0.5, -0.5]
    assert np.allclose(y, expect, atol=1e-7), y


def _real_sph(l, m, xyz):
    return S._real_sph_harm(l, m, xyz / np.linalg.norm(xyz, axis=-1, keepdims=True))


def test_sphere_eigenvalues():
    """Unit sphere, exact-sphere patches (radially projected flat triangles
    sampled at degree-4 nodes): S_k Y_n = i k j_n(k) h_n(k) Y_n and
    D_k Y_n (principal value) = (i k^2 / 2)(j_n h_n' + j_n' h_n) Y_n
    (textbook spectra; D sign per Section 3: n(y).grad_y G).  The error is
    the O(h^{d+1}) geometry error of the discretised sphere."""
    faces = S._geodesic_faces(4)
    prob = S._assemble("sph", np.full(faces.shape[0], 4),
                       lambda c, uv: S._ellipsoid_map(c, uv, (1.0, 1.0, 1.0)), faces, 1.25,
                       1.0, 0.0, 0.0, 1e-9, np.random.default_rng(0),
                       lambda xyz, rng: (np.ones(xyz.shape[0]), np.ones(xyz.shape[0])))
    nodes = [3, 2500]
    full = all_pairs_problem(prob, target_nodes=nodes)
    k = 1.5
    csr = {}
    for (al, be) in [(1.0, 0.0), (0.0, 1.0)]:
        run = oracle.OracleRun(full, mode=oracle.METHOD, alpha=al, beta=be, k=k, tol=1e-7)
        csr[al] = run.generate()
    for (l, m) in [(0, 0), (1, -1), (2, 1), (3, 0)]:
        sig = _real_sph(l, m, prob.xyz)
        jn = scipy.special.spherical_jn(l, k)
        jnp = scipy.special.spherical_jn(l, k, derivative=True)
        hn = jn + 1j * scipy.special.spherical_yn(l, k)
        hnp = jnp + 1j * scipy.special.spherical_yn(l, k, derivative=True)
        lamS = 1j * k * jn * hn
        lamD = 0.5j * k * k * (jn * hnp + jnp * hn)
        for (al, lam) in [(1.0, lamS), (0.0, lamD)]:
            rp, col, val = csr[al]
            y = oracle.apply(rp, col, val, sig)
            expect = lam * sig[nodes]
            assert np.abs(y - expect).max() < 2e-4 * max(1.0, abs(lam)), (l, m, al, y, expect)


# ------------------------------------------------------- invariances

def test_invariances():
    """Weights are unchanged by a rigid motion of patches and targets;
    the combined field equals D - ik S; Helmholtz at k -> 0 tends to
    Laplace (difference O(k))."""
    prob = S.config(0)
    rng = np.random.default_rng(3)
    pairs = [(t, int(j)) for t in rng.choice(prob.NT, 4, replace=False)
             for j in prob.near_patch[prob.near_row_ptr[t]:prob.near_row_ptr[t + 1]]]
    pairs += [(0, 0), (15, 1)]
    k = 3.0
    base = oracle.OracleRun(prob, mode=oracle.TRUTH, alpha=-1j * k, beta=1.0, k=k)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    moved = S.Problem(**{**prob.__dict__})
    shift = np.array([0.3, -1.2, 2.0])
    moved.xyz = prob.xyz @ Q.T + shift
    moved.target_xyz = prob.target_xyz @ Q.T + shift
    mv = oracle.OracleRun(moved, mode=oracle.TRUTH, alpha=-1j * k, beta=1.0, k=k)
    sS = oracle.OracleRun(prob, mode=oracle.TRUTH, alpha=1.0, beta=0.0, k=k)
    sD = oracle.OracleRun(prob, mode=oracle.TRUTH, alpha=0.0, beta=1.0, k=k)
    lap = oracle.OracleRun(prob, mode=oracle.TRUTH, alpha=1.0, beta=0.0, k=0.0)
    small = oracle.OracleRun(prob, mode=oracle.TRUTH, alpha=1.0, beta=0.0, k=1e-6)
    for (t, j) in pairs:
        a = base.pair(t, j)
        scale = np.abs(a).max()
        assert np.abs(mv.pair(t, j) - a).max() < 1e-10 * scale
        assert np.abs(sD.pair(t, j) - 1j * k * sS.pair(t, j) - a).max() < 1e-10 * scale
        lp = lap.pair(t, j)
        assert np.abs(small.pair(t, j) - lp).max() < 1e-5 * np.abs(lp).max()


def test_method_mode_meets_error_bound():
    """Section 4.3 error bound: the adaptive method's weights are within
    eps in the dual norm ||W^{-1}(a - a_true)||_2, W = diag(sqrt(J_l w_l)),
    on near and self pairs of the Laplace sphere workload."""
    prob = S.config(0)
    meth = oracle.OracleRun(prob, mode=oracle.METHOD)
    tru = oracle.OracleRun(prob, mode=oracle.TRUTH)
    rng = np.random.default_rng(7)
    d = 3
    _, _, w = oracle.reference(d, prob.ref_nodes[d])
    worst = 0.0
    for t in rng.choice(prob.NT, 6, replace=False):
        own = int(np.searchsorted(prob.node_ptr, t, side="right") - 1)
        for j in list(prob.near_patch[prob.near_row_ptr[t]:prob.near_row_ptr[t + 1]]) + [own]:
            e = dual_norm_error(meth.pair(t, j), tru.pair(t, j), node_jacobians(meth, prob, j), w)
            worst = max(worst, e)
    assert worst <= prob.tol, worst


def test_oracle_ball_flat_triangle():
    """Ball of a flat patch: the parametric mean of an affine chart is the
    vertex centroid, and the farthest lattice point is a vertex."""
    import oracle
    from tests.helpers import flat_patch_problem
    verts = np.array([[0.3, -0.1, 0.2], [1.4, 0.2, -0.3], [0.1, 0.8, 0.5]])
    for d in (1, 3, 6):
        prob = flat_patch_problem(verts, d, None)
        c, R = oracle.OracleRun(prob, mode=oracle.TRUTH).ball(0)
        g = verts.mean(0)
        assert np.abs(c - g).max() <= 1e-14
        assert abs(R - np.linalg.norm(verts - g, axis=1).max()) <= 1e-14


def test_oracle_near_lists_known_distances():
    """Targets placed at known multiples of eta R from the ball centre; node
    targets of the patch itself are never listed (own patch)."""
    import oracle
    from tests.helpers import flat_patch_problem
    verts = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    g = verts.mean(0)
    R = np.linalg.norm(verts - g, axis=1).max()
    eta = 1.25
    dirn = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    scales = [0.0, 0.5, 0.999, 1.001, 2.0]
    targets = [g + s * eta * R * dirn for s in scales]
    prob = flat_patch_problem(verts, 3, targets, self_nodes=True)
    rp, pp, margin = oracle.near_lists(prob, eta, g[None], np.array([R]))
    rows = [list(pp[rp[t]:rp[t + 1]]) for t in range(prob.NT)]
    assert rows[:5] == [[0], [0], [0], [], []]
    assert all(r == [] for r in rows[5:])          # the patch's own nodes
    assert margin[2] == pytest.approx(0.001 * eta, rel=1e-6)
