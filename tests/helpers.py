"""Shared helpers for the tests (no method arithmetic: conversions and gating)."""

import os
import sys

import numpy as np
import pytest


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def announce(msg):
    """Name the case before any GPU work (flushed, so a crash still shows it)."""
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def csr_to_dense(rowptr, col, val, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, col[rowptr[i]:rowptr[i + 1]]] = val[rowptr[i]:rowptr[i + 1]]
    return A


def dense_to_csr(A):
    n = A.shape[0]
    rows, cols = np.nonzero(A)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols.astype(np.int32), A[rows, cols].astype(np.float64)


def check_csr_valid(rowptr, col, val, n):
    assert rowptr[0] == 0 and rowptr[-1] == col.size == val.size
    assert np.all(np.diff(rowptr) >= 0)
    for i in range(n):
        c = col[rowptr[i]:rowptr[i + 1]]
        assert np.all(np.diff(c) > 0), f"row {i} columns not strictly sorted"
        assert np.all((c >= 0) & (c < n))
    assert np.all(val != 0)
