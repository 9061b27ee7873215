"""Conditional value functions (CVFs) of the parallel-scan LQR, in NumPy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A CVF from stage k to stage i (Sec. II-A, eq. sol_min) is the tuple
(A, c, C, P, p) of

    V_{k->i}(x_k, x_i) = max_lam  1/2 x_k^T P x_k + p^T x_k
                                  - 1/2 lam^T C lam + lam^T (x_i - A x_k - c)

(up to a constant).  Two consecutive CVFs compose by minimising over the
intermediate state (eq. V_ki_min).  The composition printed in eq. comb_rule
has sign slips (with C = 0 it must reduce to plain affine composition
A_{k,i} = A_{j,i} A_{k,j}, and its p-rule names an undefined b_{k,j});
``combine`` implements the composition derived from eq. V_ki_min, which is
the rule of Sarkka and Garcia-Fernandez with their eta equal to -p:

    E = I + C_kj P_ji
    A_ki = A_ji E^-1 A_kj
    c_ki = A_ji E^-1 (c_kj - C_kj p_ji) + c_ji
    C_ki = A_ji E^-1 C_kj A_ji^T + C_ji
    p_ki = A_kj^T E^-T (p_ji + P_ji c_kj) + p_kj
    P_ki = A_kj^T E^-T P_ji A_kj + P_kj

One-step elements are not printed either (they are the input array of the
scan, Sec. II-A).  Minimising the stage cost over u subject to the dynamics
x' = A x + B u + c gives

    A_el = A - B R^-1 M,  c_el = c - B R^-1 r,  C_el = B R^-1 B^T,
    P_el = Q - M^T R^-1 M,  p_el = q - M^T R^-1 r,

and a value function V(x) = 1/2 x^T P x + p^T x is the element
(0, 0, 0, P, p).
"""
from __future__ import annotations

import numpy as np


def element(A, B, c, Q, R, M, q, r):
    Ri = np.linalg.inv(R)
    return (A - B @ Ri @ M, c - B @ Ri @ r, B @ Ri @ B.T, Q - M.T @ Ri @ M, q - M.T @ Ri @ r)


def value_element(P, p):
    n = len(p)
    return (np.zeros((n, n)), np.zeros(n), np.zeros((n, n)), P, p)


def combine(a, b):
    """a = V_{k->j}, b = V_{j->i}; returns V_{k->i}."""
    A1, c1, C1, P1, p1 = a
    A2, c2, C2, P2, p2 = b
    n = len(c1)
    E = np.eye(n) + C1 @ P2
    Ei = np.linalg.inv(E)
    A = A2 @ Ei @ A1
    c = A2 @ Ei @ (c1 - C1 @ p2) + c2
    C = A2 @ Ei @ C1 @ A2.T + C2
    EiT = Ei.T
    p = A1.T @ EiT @ (p2 + P2 @ c1) + p1
    P = A1.T @ EiT @ P2 @ A1 + P1
    return (A, c, C, P, p)


def combine_as_printed(a, b):
    """The composition exactly as printed (minus sign on A, minus sign on
    c_kj, b_kj read as c_kj); kept only to show that it is not the
    minimisation of eq. V_ki_min."""
    A1, c1, C1, P1, p1 = a
    A2, c2, C2, P2, p2 = b
    n = len(c1)
    Ei = np.linalg.inv(np.eye(n) + C1 @ P2)
    A = -A2 @ Ei @ A1
    c = A2 @ Ei @ (-c1 + C1 @ p2) + c2
    C = A2 @ Ei @ C1 @ A2.T + C2
    p = A1.T @ Ei.T @ (p2 + P2 @ c1) + p1
    P = A1.T @ Ei.T @ P2 @ A1 + P1
    return (A, c, C, P, p)


def suffix_scan(elems, op=combine):
    """All suffix compositions [e_0 + ... + e_N, ..., e_N] by a sequential
    right-to-left fold."""
    out = [None] * len(elems)
    acc = elems[-1]
    out[-1] = acc
    for k in range(len(elems) - 2, -1, -1):
        acc = op(elems[k], acc)
        out[k] = acc
    return out


def balanced_fold(elems, op=combine):
    """Composition of all elements by a balanced binary tree (the order a
    parallel scan uses)."""
    if len(elems) == 1:
        return elems[0]
    h = len(elems) // 2
    return op(balanced_fold(elems[:h], op), balanced_fold(elems[h:], op))
