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


# ---------------------------------------------------------------------------
# Techniques whose chunk depends on the requesting worker (the paper's future
# work, "more complex" dynamic loop scheduling).  Each is restated from its
# authors' definition; the readings are marked.
#
# WF  -- weighted factoring (Hummel, Schmidt, Uma and Wein 1996): factoring's
#        batches, each request scaled by the requester's relative speed w_i
#        (sum of the w_i = P).  Reading: the r-th request (counting from 0)
#        belongs to batch b = r // P, whose base is FAC2's chunk of batch b,
#        c_b = ceil(R_b / (x P)) with R_b following FAC2's own schedule; the
#        request gets max(min_chunk, ceil(w_i c_b)) iterations, clamped to
#        what remains.  Past FAC2's last batch the base is min_chunk.
# AWF -- adaptive weighted factoring (Banicescu, Velusamy and Devaprasad 2003;
#        the variant that adapts after every chunk, Carino and Banicescu
#        2008): WF whose weights come from measured performance.  Worker i's
#        time per iteration pi_i = (sum_k k t_ik) / (sum_k k n_ik) over its
#        completed chunks k = 1, 2, ... (later chunks count more);
#        w_i = P (1 / pi_i) / sum_j (1 / pi_j).  Reading: the sum runs over
#        the workers that have completed a chunk, scaled by P over their
#        number; a worker with no completed chunk has weight 1.
# AF  -- adaptive factoring (Banicescu and Liu 2000): a request by worker i
#        with R iterations left gets
#            K_i = (D + 2 T R - sqrt(D^2 + 4 D T R)) / (2 mu_i),
#        D = sum_j sigma_j^2 / mu_j, T = 1 / sum_j (1 / mu_j), from the mean
#        mu_j and standard deviation sigma_j of worker j's iteration times.
#        Readings: a worker's first request (no estimate yet) gets FAC2's
#        first-batch chunk ceil(N / (2P)); the sums run over the workers with
#        an estimate, scaled by P over their number; K_i is rounded up and
#        kept in [min_chunk, R].  With every sigma = 0, K_i = T R / mu_i, so
#        P equal workers get ceil(R / P): guided self-scheduling.
# ---------------------------------------------------------------------------
WF, AWF, AF = 7, 8, 9


def fac_bases(N: int, P: int, divisor: float = 2.0, min_chunk: int = 1) -> list[int]:
    """FAC2's base chunk of each batch, c_b = max(ceil(R_b / (x P)), min_chunk)."""
    out, R = [], N
    x = float(np.float32(divisor))
    while R > 0:
        c = max(int(math.ceil(R / (x * P))), min_chunk, 1)
        out.append(c)
        R -= min(R, c * P)
    return out


def wf_chunk(w: float, base: int, remaining: int, min_chunk: int = 1) -> int:
    """WF: a request of weight w in a batch of base chunk ``base``."""
    return min(max(int(math.ceil(w * base)), min_chunk, 1), remaining)


def awf_weights(A, B, P: int):
    """AWF weights from each worker's sums A_i = sum_k k n_ik, B_i = sum_k k t_ik
    (A_i = 0: no completed chunk, weight 1)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    meas = A > 0
    w = np.ones(len(A))
    if meas.any():
        rate = np.where(meas, A / np.where(meas, B, 1.0), 0.0)   # 1 / pi_i
        total = rate[meas].sum() * P / meas.sum()
        w[meas] = P * rate[meas] / total
    return w


def af_chunk(D: float, T: float, R: int, mu: float, min_chunk: int = 1) -> int:
    """AF: chunk of a worker with mean iteration time mu, R iterations left."""
    k = (D + 2.0 * T * R - math.sqrt(D * D + 4.0 * D * T * R)) / (2.0 * mu)
    return min(max(int(math.ceil(k)), min_chunk, 1), R)


def af_sums(mu, sigma, P: int):
    """(D, T) over the workers with an estimate (mu > 0), scaled to P workers."""
    mu = np.asarray(mu, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    meas = mu > 0
    n = int(meas.sum())
    D = float((sigma[meas] ** 2 / mu[meas]).sum()) * P / n
    T = 1.0 / (float((1.0 / mu[meas]).sum()) * P / n)
    return D, T


def simulate_adaptive(kind: int, costs, P: int, speeds=None, divisor: float = 2.0,
                      min_chunk: int = 1, weights=None):
    """Discrete-event run of the master-worker protocol with a technique whose
    chunk depends on the requester.

    costs: per-iteration cost (time on a speed-1 worker); speeds: per-worker
    speed (iteration time = cost / speed), default 1.  A free worker
    (earliest free time, lowest id on ties) requests; the master sizes its
    chunk from what it has measured so far (AWF: each worker's completed
    chunks; AF: each worker's completed iterations, one time sample per
    iteration); WF takes ``weights`` (default: the speeds scaled to sum P).
    Returns (chunks as (worker, start, size) in request order, finish times).
    """
    costs = np.asarray(costs, dtype=np.float64)
    N = len(costs)
    speeds = np.ones(P) if speeds is None else np.asarray(speeds, dtype=np.float64)
    if weights is None:
        weights = speeds * P / speeds.sum()
    bases = fac_bases(N, P, divisor, min_chunk)
    A = np.zeros(P); B = np.zeros(P); nchunk = np.zeros(P, dtype=np.int64)
    cnt = np.zeros(P); mean = np.zeros(P); m2 = np.zeros(P)
    heap = [(0.0, w) for w in range(P)]
    heapq.heapify(heap)
    fin = np.zeros(P)
    chunks, nxt, r = [], 0, 0
    while nxt < N:
        t, w = heapq.heappop(heap)
        R = N - nxt
        b = r // P
        base = bases[b] if b < len(bases) else max(1, min_chunk)
        if kind == WF:
            k = wf_chunk(float(weights[w]), base, R, min_chunk)
        elif kind == AWF:
            k = wf_chunk(float(awf_weights(A, B, P)[w]), base, R, min_chunk)
        elif kind == AF:
            if cnt[w] < 2 or not (cnt > 1).any():
                k = min(max(bases[0], min_chunk, 1), R)
            else:
                mu = np.where(cnt > 1, mean, 0.0)
                sd = np.sqrt(np.where(cnt > 1, m2 / np.maximum(cnt - 1, 1), 0.0))
                D, T = af_sums(mu, sd, P)
                k = af_chunk(D, T, R, float(mean[w]), min_chunk)
        else:
            raise ValueError(kind)
        it = costs[nxt:nxt + k] / speeds[w]
        dt = float(it.sum())
        chunks.append((w, nxt, k))
        nxt += k
        r += 1
        nchunk[w] += 1
        A[w] += nchunk[w] * k
        B[w] += nchunk[w] * dt
        for v in it:  # Welford over the worker's iteration times
            cnt[w] += 1
            d = v - mean[w]
            mean[w] += d / cnt[w]
            m2[w] += d * (v - mean[w])
        t += dt
        fin[w] = t
        heapq.heappush(heap, (t, w))
    return chunks, fin
