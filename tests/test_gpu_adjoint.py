"""GPU checks of the adjoint (gradient of Phi = sum_t conj(lambda_t) (A sigma)_t
with respect to node coordinates, wavenumber and kernel weights), through
the C ABI.

* Central finite differences of Phi computed with the forward generator and
  the sparse apply, on uniform subdivision trees (min_depth = max_depth), where
  the quadrature is a smooth function of the geometry.
* Exact invariances of the frozen quadrature: translating every node (patches
  and targets) or rotating them leaves Phi unchanged, so the gradient sums to
  zero and its moment sum_n x_n x dPhi/dx_n vanishes.
* Phi is linear in alpha and beta: dPhi/dalpha and dPhi/dbeta are the
  single- and double-layer values of Phi.
* Against the oracle: central differences of the oracle's own Phi (method
  mode, uniform depth-2 trees) for off-surface targets, i.e. the near part of
  the gradient with respect to patch nodes and the wavenumber.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2006_02545_amd import nfq
    assert torch.cuda.is_available()
    return nfq.Context(0)


def _phi(ctx, prob, xyz, alpha, beta, k, sigma, lam, **kw):
    import torch
    from paper_2006_02545_amd import nfq
    plan = nfq.Plan(ctx, prob.degree, prob.node_ptr, xyz, xyz, prob.node_of_target,
                    prob.near_row_ptr, prob.near_patch)
    col, val, _ = plan.generate(alpha, beta, k, prob.tol, **kw)
    if val.dtype != torch.complex128:
        val = val.to(torch.complex128)
    y = plan.apply(col, val, torch.as_tensor(sigma)).cpu().numpy()
    return complex(np.sum(np.conj(lam) * y))


def _small(seed=0):
    from paper_2006_02545_amd import surfaces as S
    prob = S.sphere_problem(1, 3, -2j, 1.0, 2.0, 1e-8, seed=seed, density="gauss")
    return prob


def test_adjoint_matches_finite_differences(ctx):
    from paper_2006_02545_amd import nfq
    print("adjoint FD case sphere80_d3 uniform depth 2", flush=True)
    prob = _small()
    rng = np.random.default_rng(5)
    sigma = prob.sigma
    lam = prob.lam
    kw = dict(min_depth=2, max_depth=2)
    plan = nfq.plan_for(ctx, prob)
    grad, gk, da, db = plan.adjoint(prob.alpha, prob.beta, prob.k, prob.tol, sigma, lam, **kw)
    h = 1e-6
    picks = [(int(n), int(c)) for n, c in zip(rng.choice(prob.N, 10, replace=False),
                                            rng.integers(0, 3, 10))]
    scale = np.abs(grad).max()
    for (n, c) in picks:
        xp = prob.xyz.copy()
        xm = prob.xyz.copy()
        xp[n, c] += h
        xm[n, c] -= h
        fd = (_phi(ctx, prob, xp, prob.alpha, prob.beta, prob.k, sigma, lam, **kw)
              - _phi(ctx, prob, xm, prob.alpha, prob.beta, prob.k, sigma, lam, **kw)) / (2 * h)
        assert abs(fd - grad[n, c]) <= 1e-5 * scale, (n, c, fd, grad[n, c], scale)
    k = prob.k
    fdk = (_phi(ctx, prob, prob.xyz, prob.alpha, prob.beta, k + h, sigma, lam, **kw)
           - _phi(ctx, prob, prob.xyz, prob.alpha, prob.beta, k - h, sigma, lam, **kw)) / (2 * h)
    assert abs(fdk - gk) <= 1e-6 * max(1.0, abs(gk)), (fdk, gk)


def test_adjoint_invariances_and_linearity(ctx):
    from paper_2006_02545_amd import nfq, surfaces as S
    print("adjoint invariance case sphere320_d4_k5 adaptive", flush=True)
    prob = S.config(3)
    plan = nfq.plan_for(ctx, prob)
    grad, gk, da, db = plan.adjoint(prob.alpha, prob.beta, prob.k, prob.tol, prob.sigma, prob.lam)
    mag = np.abs(grad).sum(axis=0).max()
    # translation invariance
    assert np.abs(grad.sum(axis=0)).max() <= 1e-9 * mag
    # rotation invariance: sum_n x_n x grad_n = 0
    mom = np.cross(prob.xyz.astype(np.complex128), grad).sum(axis=0)
    assert np.abs(mom).max() <= 1e-9 * mag * np.abs(prob.xyz).max()
    # linearity in alpha, beta
    phiS = _phi(ctx, prob, prob.xyz, 1.0, 0.0, prob.k, prob.sigma, prob.lam)
    phiD = _phi(ctx, prob, prob.xyz, 0.0, 1.0, prob.k, prob.sigma, prob.lam)
    # (the forward with alpha = 1, beta = 0 takes its own adaptive decisions: agreement to ~eps)
    assert abs(da - phiS) <= 1e-7 * abs(phiS), (da, phiS)
    assert abs(db - phiD) <= 1e-7 * abs(phiD), (db, phiD)


def _offsurface_problem():
    """Degree-3 sphere (80 patches) with 40 targets 5 % outside the surface
    and their near lists (|x - c_j| < eta R_j)."""
    from paper_2006_02545_amd import surfaces as S
    prob = S.sphere_problem(1, 3, -3j, 1.0, 3.0, 1e-8, seed=2, density="gauss")
    rng = np.random.default_rng(11)
    pick = rng.choice(prob.NT, 40, replace=False)
    xt = prob.target_xyz[pick] * 1.05
    rows = [np.nonzero(np.linalg.norm(xt[i] - prob.centers, axis=1) < prob.eta * prob.radii)[0]
            for i in range(len(xt))]
    prob.target_xyz = xt
    prob.node_of_target = np.full(len(xt), -1, dtype=np.int64)
    prob.near_row_ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    prob.near_patch = np.concatenate(rows).astype(np.int32)
    prob.lam = prob.lam[pick]
    return prob


def _oracle_phi(prob, xyz, k, depth):
    import oracle
    from dataclasses import replace
    p2 = replace(prob, xyz=xyz)
    run = oracle.OracleRun(p2, mode=oracle.METHOD, tol=1e-300, max_depth=depth, k=k)
    phi = 0j
    for t in range(p2.NT):
        for j in p2.near_patch[p2.near_row_ptr[t]:p2.near_row_ptr[t + 1]]:
            a = run.pair(t, int(j))
            sl = slice(p2.node_ptr[j], p2.node_ptr[j + 1])
            phi += np.conj(p2.lam[t]) * np.dot(a, p2.sigma[sl])
    return phi


def test_adjoint_matches_oracle_gradient(ctx):
    from paper_2006_02545_amd import nfq
    print("adjoint oracle-gradient case sphere80_d3 off-surface depth 2", flush=True)
    prob = _offsurface_problem()
    depth = 2
    plan = nfq.plan_for(ctx, prob)
    grad, gk, _, _ = plan.adjoint(prob.alpha, prob.beta, prob.k, prob.tol, prob.sigma, prob.lam,
                                  min_depth=depth, max_depth=depth)
    # the same uniform quadrature on both sides: the oracle never accepts
    # before the depth limit at tol 1e-300
    h = 1e-5
    rng = np.random.default_rng(3)
    used = np.unique(np.concatenate([np.arange(prob.node_ptr[j], prob.node_ptr[j + 1])
                                     for j in np.unique(prob.near_patch)]))
    scale = np.abs(grad).max()
    for n in rng.choice(used, 4, replace=False):
        c = int(rng.integers(0, 3))
        xp, xm = prob.xyz.copy(), prob.xyz.copy()
        xp[n, c] += h
        xm[n, c] -= h
        fd = (_oracle_phi(prob, xp, prob.k, depth) - _oracle_phi(prob, xm, prob.k, depth)) / (2 * h)
        assert abs(fd - grad[n, c]) <= 1e-6 * scale, (n, c, fd, grad[n, c], scale)
    k = prob.k
    fdk = (_oracle_phi(prob, prob.xyz, k + h, depth) - _oracle_phi(prob, prob.xyz, k - h, depth)) / (2 * h)
    assert abs(fdk - gk) <= 1e-6 * max(1.0, abs(gk)), (fdk, gk)


def _invariances(ctx, prob, tag):
    from paper_2006_02545_amd import nfq
    rng = np.random.default_rng(21)
    prob.sigma = (rng.standard_normal(prob.N) + 1j * rng.standard_normal(prob.N)) / np.sqrt(2)
    prob.lam = (rng.standard_normal(prob.NT) + 1j * rng.standard_normal(prob.NT)) / np.sqrt(2)
    plan = nfq.plan_for(ctx, prob)
    grad, gk, da, db = plan.adjoint(prob.alpha, prob.beta, prob.k, prob.tol, prob.sigma, prob.lam)
    assert np.all(np.isfinite(grad)) and np.isfinite(gk), tag
    mag = np.abs(grad).sum(axis=0).max()
    assert np.abs(grad.sum(axis=0)).max() <= 1e-9 * mag, tag
    mom = np.cross(prob.xyz.astype(np.complex128), grad).sum(axis=0)
    assert np.abs(mom).max() <= 1e-9 * mag * np.abs(prob.xyz).max(), tag
    phiS = _phi(ctx, prob, prob.xyz, 1.0, 0.0, prob.k, prob.sigma, prob.lam)
    phiD = _phi(ctx, prob, prob.xyz, 0.0, 1.0, prob.k, prob.sigma, prob.lam)
    assert abs(da - phiS) <= 1e-7 * abs(phiS), (tag, da, phiS)
    assert abs(db - phiD) <= 1e-7 * abs(phiD), (tag, db, phiD)


def test_adjoint_mixed_degrees_invariances(ctx):
    """Degrees 2..6 on the small ellipsoid + torus, and a degree-8 sphere:
    translation and rotation invariance of the frozen quadrature, and
    dPhi/dalpha, dPhi/dbeta against forward runs."""
    from paper_2006_02545_amd import surfaces as S
    print("adjoint invariance case mixed degrees 2..6", flush=True)
    prob = S.mixed_problem(seed=11, tol=1e-8, k=3.0, ell_freq=3, tor_grid=(16, 6), dmin=2, dmax=6)
    _invariances(ctx, prob, "mixed 2..6")
    print("adjoint invariance case sphere80_d8", flush=True)
    prob = S.sphere_problem(1, 8, -2j, 1.0, 2.0, 1e-8, seed=3, density="gauss")
    _invariances(ctx, prob, "sphere80_d8")


def test_adjoint_degree7_refused(ctx):
    """Near pairs on degree-7 patches: the adjoint is refused (UNSUPPORTED)."""
    from paper_2006_02545_amd import nfq, surfaces as S
    prob = S.sphere_problem(1, 7, -2j, 1.0, 2.0, 1e-8, seed=3, density="gauss")
    plan = nfq.plan_for(ctx, prob)
    with pytest.raises(nfq.NfqError) as e:
        plan.adjoint(prob.alpha, prob.beta, prob.k, prob.tol, prob.sigma, prob.lam)
    assert e.value.status == -7


@pytest.mark.skip(reason="the degree-7 near-pair adjoint kernel returns non-finite values on the GPU "
                         "(degrees 6 and 8 and the degree-7 forward are correct); the library refuses "
                         "it until the cause is found")
def test_adjoint_degree7_values(ctx):
    from paper_2006_02545_amd import surfaces as S
    prob = S.sphere_problem(1, 7, -2j, 1.0, 2.0, 1e-8, seed=3, density="gauss")
    _invariances(ctx, prob, "sphere80_d7")
