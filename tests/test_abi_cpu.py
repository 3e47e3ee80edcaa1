"""The C ABI library loads on a CPU-only host, exports every declared entry
point, and its host-only parts work (no compute calls need a GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pts.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pts_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(ptslib):
    names = _declared()
    assert len(names) >= 30
    L = ctypes.CDLL(ptslib.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the Python binding covers the whole ABI with the same names
    assert set(names) <= set(ptslib.SIGNATURES)


def test_create_without_gpu_fails_cleanly(ptslib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = ptslib.lib().pts_create(ctypes.byref(h), 0, None, None)
    assert rc == ptslib.PTS_ERR_UNSUPPORTED
    assert not h.value
    assert ptslib.lib().pts_last_error(None)


def test_null_context_is_an_argument_error(ptslib):
    L = ptslib.lib()
    assert L.pts_estep(None, None, 8, 8, None, None, None, None) == ptslib.PTS_ERR_ARG
    assert L.pts_mstep(None, None, None, None, 8, 8, None) == ptslib.PTS_ERR_ARG
    assert L.pts_eig_sym_top(None, 4, 2, None, None, 0) == ptslib.PTS_ERR_ARG


@pytest.mark.parametrize("n,d,seed", [(40, 40, 0), (257, 16, 1), (700, 64, 2)])
def test_host_eigensolver_against_numpy(ptslib, n, d, seed):
    r = np.random.default_rng(seed)
    A = r.normal(size=(n, n)) * np.linspace(3.0, 0.01, n)
    C = A @ A.T / n
    ev, V = ptslib.eig_sym_top(C, d)
    lam, U = np.linalg.eigh(C)
    lam, U = lam[::-1], U[:, ::-1]
    assert np.abs(ev - lam[:d]).max() <= 1e-12 * lam[0]
    assert np.abs(V.T @ V - np.eye(d)).max() <= 1e-12
    assert np.abs(V @ V.T - U[:, :d] @ U[:, :d].T).max() <= 1e-10
    assert np.abs(C @ V - V * ev).max() <= 1e-12 * lam[0]
    for j in range(d):  # sign rule
        assert V[np.argmax(np.abs(V[:, j])), j] > 0


def test_host_eigensolver_degenerate_spectrum(ptslib):
    # repeated eigenvalues: the subspace is unique, the basis is not
    r = np.random.default_rng(5)
    Q, _ = np.linalg.qr(r.normal(size=(60, 60)))
    lam = np.concatenate([np.full(5, 4.0), np.full(10, 1.0), np.linspace(0.5, 0.01, 45)])
    C = (Q * lam) @ Q.T
    ev, V = ptslib.eig_sym_top(C, 15)
    assert np.allclose(ev, lam[:15], atol=1e-12)
    P = Q[:, :15] @ Q[:, :15].T
    assert np.abs(V @ V.T - P).max() <= 1e-10
    assert np.abs(V.T @ V - np.eye(15)).max() <= 1e-10
