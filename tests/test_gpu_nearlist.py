"""GPU near lists (nfq_near_lists) against the oracle, through the C ABI.

The oracle computes each patch's ball from its own chart (conical-rule mean,
lattice maximum) and the lists by brute force over all patches.  Lists must
agree exactly, except for targets that lie within 1e-9 R of some ball's
sphere, where rounding may decide either way (there must be few of them).
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TIE = 1e-9


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2006_02545_amd import nfq
    assert torch.cuda.is_available()
    return nfq.Context(0)


def _register(ctx, prob):
    for d, uv in prob.ref_nodes.items():
        if int(d) not in ctx.registered:
            ctx.register_degree(int(d), uv)


def _gpu_lists(ctx, prob):
    _register(ctx, prob)
    rp, pp, c, r = ctx.near_lists(prob.degree, prob.node_ptr, prob.xyz, prob.target_xyz,
                                  prob.node_of_target, prob.eta)
    return rp.cpu().numpy(), pp.cpu().numpy(), c.cpu().numpy(), r.cpu().numpy()


def _problem(name):
    from paper_2006_02545_amd import surfaces as S
    from tests.golden.make_golden import WORKLOADS
    return WORKLOADS[name][0]()


@pytest.mark.parametrize("name", ["laplace_s_sphere80_d3", "cfie_sphere320_d4_k5",
                                  "mixed_small_d1to8"])
def test_near_lists_match_oracle(ctx, name):
    import oracle
    print("near-list case", name, flush=True)
    prob = _problem(name)
    rp, pp, c, r = _gpu_lists(ctx, prob)
    run = oracle.OracleRun(prob, mode=oracle.TRUTH)
    oc = np.zeros((prob.P, 3))
    orad = np.zeros(prob.P)
    for j in range(prob.P):
        oc[j], orad[j] = run.ball(j)
    assert np.abs(c - oc).max() <= 1e-13 * orad.max()
    assert np.abs(r - orad).max() <= 1e-12 * orad.max()
    orp, opp, margin = oracle.near_lists(prob, prob.eta, oc, orad)
    ties = 0
    for t in range(prob.NT):
        got = pp[rp[t]:rp[t + 1]]
        want = opp[orp[t]:orp[t + 1]]
        assert np.all(np.diff(got) > 0), t
        if margin[t] < TIE:
            ties += 1
            continue
        assert np.array_equal(got, want), (t, got, want)
    assert ties <= prob.NT // 100
    print("%d targets, %d pairs, %d near-tie rows skipped" % (prob.NT, rp[-1], ties), flush=True)


def test_near_lists_off_surface_targets(ctx):
    """Off-surface targets (node_of_target = -1) 2 % outside and 3 % inside
    the 320-patch sphere: no own patch is excluded."""
    import oracle
    from dataclasses import replace
    print("near-list case off-surface targets, sphere320", flush=True)
    base = _problem("cfie_sphere320_d4_k5")
    rng = np.random.default_rng(5)
    pick = rng.choice(base.NT, 600, replace=False)
    x = base.target_xyz[pick] * np.where(np.arange(600) % 2 == 0, 1.02, 0.97)[:, None]
    prob = replace(base, target_xyz=x, node_of_target=np.full(600, -1, np.int64))
    rp, pp, c, r = _gpu_lists(ctx, prob)
    run = oracle.OracleRun(base, mode=oracle.TRUTH)
    oc = np.zeros((prob.P, 3))
    orad = np.zeros(prob.P)
    for j in range(prob.P):
        oc[j], orad[j] = run.ball(j)
    orp, opp, margin = oracle.near_lists(prob, prob.eta, oc, orad)
    for t in range(prob.NT):
        if margin[t] < TIE:
            continue
        assert np.array_equal(pp[rp[t]:rp[t + 1]], opp[orp[t]:orp[t + 1]]), t
    assert rp[-1] > 0


def test_near_lists_edge_cases(ctx):
    """No targets; no patches near any target; capacity too small."""
    import torch
    from paper_2006_02545_amd import nfq
    prob = _problem("laplace_s_sphere80_d3")
    _register(ctx, prob)
    # no targets
    rp, pp, _, _ = ctx.near_lists(prob.degree, prob.node_ptr, prob.xyz, np.zeros((0, 3)),
                                  np.zeros(0, np.int64), prob.eta)
    assert rp.cpu().numpy().tolist() == [0] and pp.numel() == 0
    # targets far away: empty rows
    far = np.array([[10.0, 0.0, 0.0], [0.0, -7.0, 3.0]])
    rp, pp, _, _ = ctx.near_lists(prob.degree, prob.node_ptr, prob.xyz, far,
                                  np.full(2, -1, np.int64), prob.eta)
    assert rp.cpu().numpy().tolist() == [0, 0, 0] and pp.numel() == 0
    # capacity error: row pointers still written, status INVALID_ARG
    dev = torch.device("cuda", 0)
    deg = torch.as_tensor(prob.degree, device=dev)
    nptr = torch.as_tensor(prob.node_ptr, device=dev)
    x = torch.as_tensor(prob.xyz, device=dev)
    tx = torch.as_tensor(prob.target_xyz, device=dev)
    nt = torch.as_tensor(prob.node_of_target, device=dev)
    surf = nfq.Surface(prob.P, deg.data_ptr(), nptr.data_ptr(), x.data_ptr())
    tg = nfq.Targets(prob.NT, tx.data_ptr(), nt.data_ptr())
    row = torch.empty(prob.NT + 1, dtype=torch.int64, device=dev)
    patch = torch.empty(4, dtype=torch.int32, device=dev)
    import ctypes as C
    nnz = C.c_int64()
    st = ctx.L.nfq_near_lists(ctx.h, C.byref(surf), C.byref(tg), float(prob.eta),
                              C.c_void_p(row.data_ptr()), C.c_void_p(patch.data_ptr()), 4,
                              C.byref(nnz), None, None)
    assert st == nfq.NFQ_ERR_INVALID_ARG
    assert nnz.value > 4 and int(row[-1].item()) == nnz.value
    # bad eta
    st = ctx.L.nfq_near_lists(ctx.h, C.byref(surf), C.byref(tg), -1.0, C.c_void_p(row.data_ptr()),
                              None, 0, C.byref(nnz), None, None)
    assert st == nfq.NFQ_ERR_INVALID_ARG


def test_near_lists_star200k_sampled(ctx):
    """200,000-patch surface, 5.6 M targets: the whole GPU build, then 200
    sampled targets checked against the oracle.  Candidates for a sampled
    target come from the input's own balls (exact surface map), taken twice
    as wide so that they hold every patch of the oracle's list."""
    import oracle
    from tests.golden.make_golden import WORKLOADS
    print("near-list case star200k_d6", flush=True)
    prob = WORKLOADS["star200k_d6"][0]()
    _register(ctx, prob)
    t0 = time.perf_counter()
    rp, pp, c, r = _gpu_lists(ctx, prob)
    print("GPU near lists: %.1f ms (with copies), %d pairs" % ((time.perf_counter() - t0) * 1e3,
                                                                 rp[-1]), flush=True)
    run = oracle.OracleRun(prob, mode=oracle.TRUTH)
    rng = np.random.default_rng(7)
    ties = 0
    for t in rng.choice(prob.NT, 200, replace=False):
        x = prob.target_xyz[t]
        cand = np.nonzero(np.linalg.norm(prob.centers - x, axis=1) < 2 * prob.eta * prob.radii)[0]
        own = int(np.searchsorted(prob.node_ptr, prob.node_of_target[t], side="right") - 1)
        want, close = [], False
        for j in cand:
            oc, orad = run.ball(int(j))
            dist = np.sqrt(((x - oc) ** 2).sum())
            if abs(dist - prob.eta * orad) < TIE * orad:
                close = True
            if dist < prob.eta * orad and j != own:
                want.append(int(j))
        if close:
            ties += 1
            continue
        assert np.array_equal(pp[rp[t]:rp[t + 1]], np.array(sorted(want), np.int32)), t
    assert ties <= 2
