"""Checkpointed reversal of the time loop and the gradient's parametrisation.

TEST INFRASTRUCTURE ONLY (part of the oracle).

Reversal model.  The forward state after step k is S_k = (u^{k-1}, u^k);
S_0 (the initial data) is always available.  The adjoint iteration k
(k = nt, ..., 1, in that order) needs u^k, i.e. the current state must be
S_k.  One forward step turns the current state S_k into S_{k+1} and costs 1;
a snapshot slot holds one state; storing the current state into a slot,
restoring a slot's state as the current one, and the adjoint iteration cost
nothing.  With s slots (S_0 not counted) the least number of forward steps
that reverses nt steps is

  optimal_cost       the recursion of binomial checkpointing taken as a
                     definition: advance from S_a to S_{a+m} and store it,
                     reverse (a+m, b] with one slot fewer, run iteration a+m
                     on the stored S_{a+m}, then reverse (a, a+m-1] from S_a
                     with every slot, minimised over m;
  exhaustive_cost    the same number found by searching every sequence of
                     actions of the model above (small cases only);
  binomial_cost      the closed form of Griewank & Walther (ACM TOMS 26,
                     2000, Algorithm 799 "revolve"): reversing l steps whose
                     reverse step i needs state i, with r stored states
                     counting the initial one, takes t l - C(r + t, r + 1)
                     forward steps, t the least integer with C(r + t, r) >= l.
                     Our nt iterations need S_nt .. S_1 and S_0 is stored,
                     which is their problem with l = nt + 1 and r = s + 1.

simulate_plan checks an action list (as the product library emits it)
against the model and returns its forward-step count.

Parametrisation (the gradient is taken with respect to the velocity c by the
adjoint; the slowness s = 1/c and m = 1/c^2 follow by the chain rule):
  dJ/ds = -c^2 dJ/dc,   dJ/dm = -(c^3 / 2) dJ/dc.
"""
from __future__ import annotations

import heapq
from functools import lru_cache
from math import comb
from typing import List, Sequence, Tuple

import numpy as np

ADVANCE, STORE, RESTORE, ADJOINT = 0, 1, 2, 3


def optimal_cost(L: int, s: int) -> int:
    """Least forward steps to reverse L steps from a stored start with s free slots."""
    if L < 0 or s < 0:
        raise ValueError("L and s must be >= 0")

    @lru_cache(maxsize=None)
    def C(l: int, k: int) -> int:
        if l <= 0:
            return 0
        if l == 1:
            return 1
        if k == 0:
            return l * (l + 1) // 2   # restore the start before each iteration
        return min(m + C(l - m, k - 1) + C(m - 1, k) for m in range(1, l + 1))

    return C(L, s)


def binomial_cost(L: int, s: int) -> int:
    """Griewank & Walther's closed form for l = L + 1 reverse steps and
    r = s + 1 stored states."""
    if L == 0:
        return 0
    r, l = s + 1, L + 1
    t = 0
    while comb(r + t, r) < l:
        t += 1
    return t * l - comb(r + t, r + 1)


def exhaustive_cost(L: int, s: int) -> int:
    """0-1 shortest path over (current state, stored states, next iteration)."""
    start = (0, frozenset(), L)   # current S_0, no slot used, iteration L next
    dist = {start: 0}
    heap = [(0, 0, start)]
    tie = 1
    while heap:
        d, _, node = heapq.heappop(heap)
        if dist.get(node, None) != d:
            continue
        cur, stored, k = node
        if k == 0:
            return d
        moves: List[Tuple[int, tuple]] = []
        if cur == k:
            moves.append((0, (cur, stored, k - 1)))        # adjoint iteration k
        if cur < k:
            moves.append((1, (cur + 1, stored, k)))        # one forward step
        if cur != 0 and cur not in stored and len(stored) < s:
            moves.append((0, (cur, stored | {cur}, k)))    # store
        for j in stored | {0}:
            if j != cur:
                moves.append((0, (j, stored, k)))          # restore
        for j in stored:
            moves.append((0, (cur, stored - {j}, k)))      # free a slot
        for w, nxt in moves:
            nd = d + w
            if nd < dist.get(nxt, 1 << 60):
                dist[nxt] = nd
                heapq.heappush(heap, (nd, tie, nxt))
                tie += 1
    raise RuntimeError("no reversal found")


def simulate_plan(ops: Sequence[Tuple[int, int]], nt: int, nsnap: int) -> int:
    """Check that the action list reverses nt steps within nsnap slots (slot
    -1 is S_0) and return its number of forward steps."""
    cur = 0
    slots = {-1: 0}
    k_next = nt
    steps = 0
    for op, arg in ops:
        if op == ADVANCE:
            if not (cur < arg <= nt):
                raise AssertionError(f"advance from {cur} to {arg}")
            steps += arg - cur
            cur = arg
        elif op == STORE:
            if not (0 <= arg < nsnap):
                raise AssertionError(f"slot {arg} outside 0..{nsnap - 1}")
            slots[arg] = cur
        elif op == RESTORE:
            if arg not in slots:
                raise AssertionError(f"restore of empty slot {arg}")
            cur = slots[arg]
        elif op == ADJOINT:
            if arg != k_next or cur != arg:
                raise AssertionError(f"adjoint {arg} with state {cur}, expected {k_next}")
            k_next -= 1
        else:
            raise AssertionError(f"unknown op {op}")
    if k_next != 0:
        raise AssertionError(f"iterations {k_next}..1 missing")
    return steps


def gradient_param(g_c: np.ndarray, c: np.ndarray, param: str) -> np.ndarray:
    """dJ/d(param) from dJ/dc (FP64)."""
    g_c = np.asarray(g_c, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    if param == "velocity":
        return g_c.copy()
    if param == "slowness":
        return -c * c * g_c
    if param == "m":
        return -0.5 * c ** 3 * g_c
    raise ValueError(f"unknown parameter {param!r}")
