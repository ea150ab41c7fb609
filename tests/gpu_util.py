"""Helpers shared by the GPU parity tests (test harness only)."""

from __future__ import annotations

import sys

import numpy as np

REL = 1e-5  # floats and gradients: within 1e-5 relative of the FP64 oracle


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def assert_close(name: str, got, ref, A, rel: float = REL) -> dict:
    """Pass rule: |got - ref| <= rel (|ref| + A) elementwise, A the oracle's
    absolute-value evaluation; also normwise ||got - ref|| / ||ref|| <= rel."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.isfinite(got).all(), f"{name}: non-finite output"
    err = np.abs(got - ref)
    denom = np.abs(ref) + A
    worst = float((err / np.where(denom > 0, denom, 1.0)).max()) if err.size else 0.0
    nref = float(np.linalg.norm(ref))
    normwise = float(np.linalg.norm(err) / nref) if nref > 0 else float(np.linalg.norm(err))
    say(f"[{name}] elementwise max err/(|ref|+A) = {worst:.3e}  normwise = {normwise:.3e}  "
        f"max|err| = {float(err.max()) if err.size else 0.0:.3e}")
    bad = err > rel * denom
    assert not bad.any(), f"{name}: {int(bad.sum())} elements beyond tolerance (worst {worst:.3e})"
    assert normwise <= rel, f"{name}: normwise error {normwise:.3e}"
    return {"elementwise": worst, "normwise": normwise}


def pack_rows(a: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Packed order: row i of the result is row perm[i] of a."""
    return np.ascontiguousarray(a[perm])


def unpack_rows(a: np.ndarray, perm: np.ndarray) -> np.ndarray:
    out = np.empty_like(a)
    out[perm] = a
    return out
