"""Write the stored expected values of the GPU parity tests.

Calls only the CPU oracle (oracle/, truth mode) on the seeded synthetic
workloads of paper_2006_02545_amd.surfaces; nothing here comes from the HIP
path.  For each workload and each sampled target it stores the full CSR row
(ascending patch blocks, near patches plus the target's own patch) and, per
block, the dual-norm weights W_l = sqrt(J(u_l, v_l) |w_l|) of the patch
(Section 4.2 error analysis), so the tests can apply the paper's bound
||W^{-1}(a_gpu - a_true)||_2 <= 10 eps per pair.

Usage: python tests/golden/make_golden.py [name ...]
"""
from __future__ import annotations

import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2006_02545_amd import surfaces as S  # noqa: E402


def small_mixed():
    """Mixed degrees 2..8 on a small ellipsoid + torus (ragged rows)."""
    return S.mixed_problem(seed=11, tol=1e-8, k=3.0, ell_freq=3, tor_grid=(16, 6), dmin=2,
                           dmax=8)


WORKLOADS = {
    # name: (builder, number of sampled targets or None for all)
    "laplace_s_sphere80_d3": (lambda: S.config(0), None),
    "cfie_sphere1280_d4": (lambda: S.config(1), 160),
    "cfie_sphere320_d4_k5": (lambda: S.config(3), 120),
    "mixed_small_d1to8": (small_mixed, 160),
    # smallest degrees, real double layer and a tighter tolerance
    "laplace_d_sphere80_d1": (lambda: S.sphere_problem(1, 1, 0.0, 1.0, 0.0, 1e-6, seed=8,
                                                       density="uniform"), None),
    "cfie_sphere80_d2_k3": (lambda: S.sphere_problem(1, 2, -3j, 1.0, 3.0, 1e-9, seed=9,
                                                     density="gauss"), 160),
    # real Laplace double layer on the small mixed-degree fixture (real-kernel
    # instances of every degree)
    "laplace_d_mixed_small": (lambda: S.mixed_problem(seed=11, tol=1e-8, k=0.0, ell_freq=3,
                                                      tor_grid=(16, 6), dmin=2, dmax=8), 160),
    # full-size workloads, sampled rows
    "mixed_ellipsoid_torus": (lambda: S.config(2), 48),
    "star200k_d6": (lambda: S.config(4), 24),
}


def _rows(args):
    name, targets = args
    prob = WORKLOADS[name][0]()
    run = oracle.OracleRun(prob, mode=oracle.TRUTH)
    out = []
    for t in targets:
        t = int(t)
        own = int(np.searchsorted(prob.node_ptr, t, side="right") - 1)
        pats = sorted([int(j) for j in prob.near_patch[prob.near_row_ptr[t]:prob.near_row_ptr[t + 1]]]
                      + [own])
        vals, Ws = [], []
        for j in pats:
            vals.append(run.pair(t, j))
            d = int(prob.degree[j])
            _, _, w = oracle.reference(d, prob.ref_nodes[d])
            J = []
            for (u, v) in prob.ref_nodes[d]:
                _, Xu, Xv = run.chart(j, u, v)
                J.append(np.linalg.norm(np.cross(Xu, Xv)))
            Ws.append(np.sqrt(np.array(J) * np.abs(w)))
        out.append((t, pats, np.concatenate(vals), np.concatenate(Ws)))
    return out


def make(name, workers=8):
    build, nsamp = WORKLOADS[name]
    prob = build()
    if nsamp is None:
        targets = np.arange(prob.NT)
    else:
        targets = np.sort(np.random.default_rng(12345).choice(prob.NT, nsamp, replace=False))
    # large surfaces take a while to build: one chunk per worker there
    nchunk = workers if prob.P > 50000 else workers * 4
    chunks = [(name, c) for c in np.array_split(targets, nchunk) if len(c)]
    with ProcessPoolExecutor(workers) as ex:
        res = [r for part in ex.map(_rows, chunks) for r in part]
    res.sort(key=lambda r: r[0])
    t_ids = np.array([r[0] for r in res], dtype=np.int64)
    row_len = np.array([len(r[2]) for r in res], dtype=np.int64)
    patches = np.concatenate([np.array(r[1], dtype=np.int32) for r in res])
    npat = np.array([len(r[1]) for r in res], dtype=np.int64)
    vals = np.concatenate([r[2] for r in res])
    W = np.concatenate([r[3] for r in res])
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, targets=t_ids, row_len=row_len, patches=patches, npat=npat,
                        vals=vals, W=W, tol=prob.tol)
    print("wrote", path, "targets", len(t_ids), "entries", vals.size)


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    for n in names:
        make(n)
