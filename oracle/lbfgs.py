"""Plain FP64 oracle of the limited-memory BFGS direction (TEST
INFRASTRUCTURE ONLY: only the tests use this module).

The paper names L-BFGS-B as the optimizer of its inversions (Applications,
FWI); the bounds are applied here by clipping the model after each step.
What this module fixes is the search direction: the two-loop recursion of
Nocedal and Wright (Numerical Optimization, Algorithm 7.4) over the stored
pairs s_i = m_{i+1} - m_i, y_i = g_{i+1} - g_i, newest first, with the
initial inverse Hessian gamma I, gamma = s^T y / y^T y of the newest pair:

    q = g;  for i = newest .. oldest:  a_i = rho_i s_i^T q;  q -= a_i y_i
    r = gamma q;  for i = oldest .. newest:  b = rho_i y_i^T r;  r += (a_i - b) s_i
    p = -r,   rho_i = 1 / (y_i^T s_i).

With no stored pair, p = -g.
"""
from __future__ import annotations

import numpy as np


def two_loop(g, S, Y):
    """p = -H g for the pairs S[i], Y[i] given oldest first."""
    g = np.asarray(g, dtype=np.float64)
    if len(S) == 0:
        return -g
    S = [np.asarray(s, dtype=np.float64) for s in S]
    Y = [np.asarray(y, dtype=np.float64) for y in Y]
    rho = [1.0 / float(y @ s) for s, y in zip(S, Y)]
    q = g.copy()
    alpha = [0.0] * len(S)
    for i in reversed(range(len(S))):
        alpha[i] = rho[i] * float(S[i] @ q)
        q -= alpha[i] * Y[i]
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
    r = gamma * q
    for i in range(len(S)):
        b = rho[i] * float(Y[i] @ r)
        r += (alpha[i] - b) * S[i]
    return -r


def bfgs_inverse(S, Y, n):
    """The dense inverse-Hessian approximation the same pairs build:
    H_0 = gamma I, H_{i+1} = (I - rho s y^T) H_i (I - rho y s^T) + rho s s^T."""
    S = [np.asarray(s, dtype=np.float64) for s in S]
    Y = [np.asarray(y, dtype=np.float64) for y in Y]
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
    H = gamma * np.eye(n)
    I = np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / float(y @ s)
        H = (I - rho * np.outer(s, y)) @ H @ (I - rho * np.outer(y, s)) + rho * np.outer(s, s)
    return H
