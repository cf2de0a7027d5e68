"""Chunk sizes of the loop-scheduling techniques and a schedule simulator.

TEST INFRASTRUCTURE ONLY.

Section 2.2 of the paper describes the techniques in words:
  * STATIC -- the iterations are divided once, up front, about N/P per worker
    (Section 2.1 and the related-work discussion of the earlier PSIA); here as
    balanced contiguous blocks: the first N mod P workers get ceil(N/P), the
    rest floor(N/P);
  * SS     -- self-scheduling, one iteration per request;
  * GSS    -- guided self-scheduling: every step hands out the remaining
    iterations divided by the number of workers, c = ceil(R/P)
    (Polychronopoulos and Kuck, cited by the paper);
  * FAC    -- factoring: batches of P equal chunks; the paper prints no formula,
    so the FAC2 rule of Hummel et al. (cited by the paper) is used: batch b
    has P chunks of ceil(R_b / (x P)) with x = 2, the last chunks clamped to
    what remains.
Two later techniques of the same family, which the paper leaves to future
work (more complex dynamic loop scheduling), follow their authors' papers:
  * FAC_PROB -- probabilistic factoring (Hummel, Schonberg and Flynn 1992):
    batch j of P chunks of ceil(R_j / (x_j P)), where with
    b_j = P cv / (2 sqrt(R_j)) and cv = sigma / mu of the iteration cost,
    x_0 = 1 + b_0^2 + b_0 sqrt(b_0^2 + 2) for the first batch and
    x_j = 2 + b_j^2 + b_j sqrt(b_j^2 + 4) for the later ones;
  * TSS      -- trapezoid self-scheduling (Tzen and Ni 1993): chunk sizes fall
    linearly from F = ceil(N / (2P)) towards L = 1 over
    C = ceil(2N / (F + L)) chunks: chunk i has ceil(F - i delta) iterations
    (never below L) with the real step delta = (F - L) / (C - 1), the last
    chunk clamped to what remains.  An integer step would be 0 whenever
    C - 1 > F - L, which is the case for a GPU's P (N = 2M, P = 1280 gives
    delta = 0.15), and TSS would degenerate to fixed chunks of N / (2P).
``min_chunk`` raises every dynamic chunk to at least that many iterations.

Chunks are half-open [start, end) ranges of the iteration space in order; a
table is the list of chunk sizes, and ``starts`` its exclusive prefix sum with
N appended.

``simulate`` is a discrete-event model of the master-worker protocol of
Section 3 (request, assign, compute, request again) on P identical workers with
known per-iteration costs; it is used to test the qualitative claims of
Section 2.2 without a cluster or a GPU.
"""
from __future__ import annotations

import heapq
import math

import numpy as np

STATIC, SS, GSS, FAC = 0, 1, 2, 3
TSS, FAC_PROB = 5, 6


def static_sizes(N: int, P: int) -> list[int]:
    q, r = divmod(N, P)
    return [q + 1] * r + [q] * (P - r)


def ss_sizes(N: int, min_chunk: int = 1) -> list[int]:
    c = max(1, min_chunk)
    out, R = [], N
    while R > 0:
        k = min(c, R)
        out.append(k)
        R -= k
    return out


def gss_sizes(N: int, P: int, min_chunk: int = 1) -> list[int]:
    out, R = [], N
    while R > 0:
        c = min(max(-(-R // P), min_chunk, 1), R)
        out.append(c)
        R -= c
    return out


def fac_sizes(N: int, P: int, divisor: float = 2.0, min_chunk: int = 1) -> list[int]:
    out, R = [], N
    x = float(np.float32(divisor))
    while R > 0:
        c = max(int(math.ceil(R / (x * P))), min_chunk, 1)
        for _ in range(P):
            if R == 0:
                break
            k = min(c, R)
            out.append(k)
            R -= k
    return out


def fac_prob_ratio(R: int, P: int, cv: float, first: bool) -> float:
    """Hummel's x_j of a batch with R iterations remaining."""
    b = P * cv / (2.0 * math.sqrt(R))
    if first:
        return 1.0 + b * b + b * math.sqrt(b * b + 2.0)
    return 2.0 + b * b + b * math.sqrt(b * b + 4.0)


def fac_prob_sizes(N: int, P: int, cv: float, min_chunk: int = 1) -> list[int]:
    out, R = [], N
    cv = float(np.float32(cv))
    first = True
    while R > 0:
        x = fac_prob_ratio(R, P, cv, first)
        first = False
        c = max(int(math.ceil(R / (x * P))), min_chunk, 1)
        for _ in range(P):
            if R == 0:
                break
            k = min(c, R)
            out.append(k)
            R -= k
    return out


def tss_sizes(N: int, P: int, min_chunk: int = 1) -> list[int]:
    if N <= 0:
        return []
    last = max(1, min_chunk)
    first = max(-(-N // (2 * P)), last)
    n = -(-2 * N // (first + last))
    delta = (first - last) / (n - 1) if n > 1 else 0.0
    out, R, i = [], N, 0
    while R > 0:
        c = max(int(math.ceil(first - i * delta)), last)
        k = min(c, R)
        out.append(k)
        R -= k
        i += 1
    return out


def sizes(kind: int, N: int, P: int, min_chunk: int = 1, divisor: float = 2.0) -> list[int]:
    if kind == STATIC:
        return static_sizes(N, P)
    if kind == SS:
        return ss_sizes(N, min_chunk)
    if kind == GSS:
        return gss_sizes(N, P, min_chunk)
    if kind == FAC:
        return fac_sizes(N, P, divisor, min_chunk)
    if kind == TSS:
        return tss_sizes(N, P, min_chunk)
    if kind == FAC_PROB:
        return fac_prob_sizes(N, P, divisor, min_chunk)
    raise ValueError(kind)


def starts(sz) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(np.asarray(sz, dtype=np.int64))]).astype(np.int64)


def simulate(costs, sz, P: int, static: bool = False, overhead: float = 0.0):
    """Finish time of each of P workers.

    Dynamic: a free worker (earliest free time, lowest id on ties) takes the
    next chunk in order and is busy for the chunk's summed cost plus
    ``overhead``.  Static: worker k executes chunk k.
    """
    costs = np.asarray(costs, dtype=np.float64)
    st = starts(sz)
    per_chunk = [float(costs[st[i]:st[i + 1]].sum()) for i in range(len(sz))]
    if static:
        fin = np.zeros(P)
        for k, c in enumerate(per_chunk):
            fin[k % P] += c + overhead
        return fin
    heap = [(0.0, w) for w in range(P)]
    heapq.heapify(heap)
    fin = np.zeros(P)
    for c in per_chunk:
        t, w = heapq.heappop(heap)
        t = t + c + overhead
        fin[w] = t
        heapq.heappush(heap, (t, w))
    return fin
