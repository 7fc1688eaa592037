"""Small test-side helpers: re-scoring a CIGAR and textbook special cases.

These are written from the definitions (affine gap cost o + (k-1)e, local
alignment) and share nothing with the oracle or the GPU library.
"""
from __future__ import annotations

import numpy as np


def rescore(q, r, matrix, o, e, qbeg, rbeg, cigar):
    """Score of the alignment described by (qbeg, rbeg, cigar) and the spans
    it consumes: returns (score, query_consumed, ref_consumed)."""
    i, j, s = qbeg, rbeg, 0
    for n, op in cigar:
        if op == "M":
            for _ in range(n):
                s += int(matrix[q[i], r[j]])
                i += 1
                j += 1
        elif op == "I":
            s -= o + (n - 1) * e
            i += n
        elif op == "D":
            s -= o + (n - 1) * e
            j += n
        else:
            raise ValueError(op)
    return s, i - qbeg, j - rbeg


def score2_from_maxcol(maxcol, ref_begin1, ref_end1, m):
    """Second-best score by its definition on the max array (mask
    [ref_begin1 - m, ref_end1 + m])."""
    best, at = 0, -1
    for j, v in enumerate(maxcol):
        if ref_begin1 - m <= j <= ref_end1 + m:
            continue
        if v > best:
            best, at = int(v), j
    return best, at


def kadane_local(q, r, matrix):
    """Best ungapped local alignment by Kadane's maximum subarray along every
    diagonal.  Returns (score1, maxcol, end, begin) with the stated tie-breaks
    (end: smallest column then row; begin: latest start on the diagonal)."""
    lq, lr = len(q), len(r)
    S = matrix[np.asarray(q)[:, None], np.asarray(r)[None, :]].astype(np.int64)
    run = np.zeros((lq, lr), dtype=np.int64)   # best segment sum ending at (i, j)
    for i in range(lq):
        for j in range(lr):
            prev = run[i - 1, j - 1] if i > 0 and j > 0 else 0
            run[i, j] = max(prev, 0) + S[i, j]
    H = np.maximum(run, 0)
    maxcol = H.max(axis=0) if lq else np.zeros(lr, dtype=np.int64)
    score1 = int(H.max()) if H.size else 0
    if score1 <= 0:
        return 0, maxcol, (-1, -1), (-1, -1)
    je = int(np.nonzero((H == score1).any(axis=0))[0][0])
    ie = int(np.nonzero(H[:, je] == score1)[0][0])
    # latest start whose segment sum to (ie, je) equals score1
    acc = 0
    begin = None
    for k in range(0, min(ie, je) + 1):
        acc += int(S[ie - k, je - k])
        if acc == score1:
            begin = (ie - k, je - k)
            break
    return score1, maxcol, (ie, je), begin


def textbook_linear_sw(q, r, matrix, g):
    """One-matrix Smith-Waterman with linear gap cost g per symbol.
    Returns (score1, maxcol)."""
    lq, lr = len(q), len(r)
    H = np.zeros((lq + 1, lr + 1), dtype=np.int64)
    for i in range(1, lq + 1):
        for j in range(1, lr + 1):
            H[i, j] = max(0, H[i - 1, j - 1] + int(matrix[q[i - 1], r[j - 1]]),
                          H[i - 1, j] - g, H[i, j - 1] - g)
    maxcol = H[1:, 1:].max(axis=0) if lq else np.zeros(lr, dtype=np.int64)
    return int(H.max()), maxcol
