"""Deterministic SI simulation from every node (TEST INFRASTRUCTURE).

Sec. 1 of the paper: seed a single node at its first appearance; a
susceptible node becomes infected when it has an event with an infected one;
the infected set at the end is the seed's maximum out-component.  Events at
one time step are not adjacent (Sec. 2.1), so infection spreads by at most one
hop per time step: the newly infected set at a step is computed from the
infected set as it was before that step.  Pure Python, O(n m): tiny inputs only.
"""
from __future__ import annotations


def _steps(src, dst, t, sequential):
    m = len(src)
    i = 0
    while i < m:
        j = i + 1
        if not sequential:
            while j < m and int(t[j]) == int(t[i]):
                j += 1
        yield int(t[i]), [(int(src[e]), int(dst[e])) for e in range(i, j)]
        i = j


def first_appearance(n, src, dst, t):
    first = [None] * n
    for e in range(len(src)):
        for x in (int(src[e]), int(dst[e])):
            if first[x] is None:
                first[x] = int(t[e])
    return first


def out_components(n, src, dst, t, directed=False, sequential=False):
    """List of sets: OC[s] = nodes infected by an SI process seeded at s."""
    first = first_appearance(n, src, dst, t)
    steps = list(_steps(src, dst, t, sequential))
    result = []
    for s in range(n):
        infected = {s}
        if first[s] is not None:
            started = False
            for k, (tau, evs) in enumerate(steps):
                if not started:
                    # first step containing an event of s (ties: the whole step)
                    if tau < first[s]:
                        continue
                    started = True
                newly = set()
                for x, y in evs:
                    if x in infected:
                        newly.add(y)
                    if not directed and y in infected:
                        newly.add(x)
                infected |= newly
        result.append(infected)
    return result
