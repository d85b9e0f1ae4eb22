"""Helpers for the GPU parity tests (comparison rules and input staging)."""

from __future__ import annotations

import sys

import numpy as np

# Periodogram tolerance (normwise): max|P_gpu - P_ref| / max|P_ref|.
P_TOL_FP32 = 1e-5
# Two cells whose oracle values differ by less than this (relative) are a
# near-tie: FP32 rounding may rank them either way.
NEAR_TIE = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rounded(x):
    """The complex64 values the GPU sees, back in complex128 for the oracle."""
    return np.asarray(x).astype(np.complex64).astype(np.complex128)


def normwise_error(P_gpu, P_ref):
    P_gpu = np.asarray(P_gpu, dtype=np.float64)
    P_ref = np.asarray(P_ref, dtype=np.float64)
    return float(np.max(np.abs(P_gpu - P_ref)) / np.max(np.abs(P_ref)))


def oracle_ranked(oracle, P, k):
    """Oracle peaks as (s, r, value), s signed."""
    m_pad = P.shape[0]
    return [(row - m_pad // 2, r, v) for row, r, v in oracle.find_peaks(P, k)]


def compare_peak_indices(gpu, ref, P_ref, near_tie=NEAR_TIE):
    """Compare GPU peak cells with the oracle's, rank by rank.

    gpu: [(s, r), ...]; ref: oracle [(s, r, value), ...] of the same length.
    A differing cell at rank i is accepted only as a near-tie: the oracle's
    own value at the GPU's cell must lie within NEAR_TIE (relative) of the
    oracle's i-th peak value.  Returns the number of near-tie exclusions, or
    None on a real mismatch.
    """
    if len(gpu) != len(ref):
        return None
    m_pad = P_ref.shape[0]
    excluded = 0
    for (gs, gr), (rs, rr, rv) in zip(gpu, ref):
        if (gs, gr) == (rs, rr):
            continue
        vg = P_ref[gs + m_pad // 2, gr]
        if abs(vg - rv) <= near_tie * rv:
            excluded += 1
            continue
        return None
    return excluded


def check_topk_property(P, peaks, k):
    """The reported peaks are exactly the top-k 3x3 cyclic local maxima of P.

    Written from the definition (a cell >= its 8 cyclic neighbours; rank by
    value descending, flat index ascending), independently of the oracle's
    peak finder.  P: float32 [M'][N'] (row s + M'/2 holds Doppler s);
    peaks: [(s, r, p, ...)].  Returns an error string, or None.
    """
    P = np.asarray(P, dtype=np.float32)
    m_pad, n_pad = P.shape
    is_max = np.ones(P.shape, dtype=bool)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di or dj:
                is_max &= P >= np.roll(np.roll(P, di, axis=0), dj, axis=1)
    rows, cols = np.nonzero(is_max)
    vals = P[rows, cols]
    flat = rows.astype(np.int64) * n_pad + cols
    order = np.lexsort((flat, -vals.astype(np.float64)))[:k]
    want = [(int(rows[i]) - m_pad // 2, int(cols[i]), float(vals[i])) for i in order]
    got = [(int(s), int(r), float(np.float32(p))) for s, r, p, *_ in peaks]
    if got != want:
        return f"top-{k} mismatch: got {got[:4]}..., want {want[:4]}..."
    return None
