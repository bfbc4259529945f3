"""CPU checks of the C ABI and of the host logic (no compute calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2006_02545_amd import nfq, surfaces

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nfq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nfq_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_names():
    decl = _declared()
    assert decl == sorted(nfq.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(nfq.LIB_PATH):
        pytest.skip("libnfq.so not built")
    lib = ctypes.CDLL(nfq.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.nfq_status_str  # callable without a device
    lib.nfq_status_str.restype = ctypes.c_char_p
    assert lib.nfq_status_str(-4) == b"NFQ_ERR_SINGULAR_PAIR"
    assert lib.nfq_status_str(1) == b"NFQ_WARN_NONCONVERGED"


def test_context_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        nfq.Context(0)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
def test_reference_nodes_interior_unisolvent(d):
    uv = surfaces.reference_nodes(d)
    nd = (d + 1) * (d + 2) // 2
    assert uv.shape == (nd, 2)
    assert np.all(uv > 0) and np.all(uv.sum(1) < 1)
    # unisolvent: the monomial Vandermonde is nonsingular
    M = np.stack([uv[:, 0] ** a * uv[:, 1] ** b for a in range(d + 1) for b in range(d + 1 - a)], 1)
    assert np.linalg.cond(M) < 1e10


@pytest.mark.parametrize("cfg", [0, 1, 3])
def test_near_lists_well_formed(cfg):
    """Rows strictly ascending, own patch excluded, strict ball test."""
    p = surfaces.config(cfg)
    own = np.repeat(np.arange(p.P), np.diff(p.node_ptr))
    for t in range(0, p.NT, max(1, p.NT // 300)):
        row = p.near_patch[p.near_row_ptr[t]:p.near_row_ptr[t + 1]]
        assert np.all(np.diff(row) > 0)
        assert own[t] not in row
        for j in row:
            assert np.linalg.norm(p.target_xyz[t] - p.centers[j]) < p.eta * p.radii[j]


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; --gpus above 1 exits with a message."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
