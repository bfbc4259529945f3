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
