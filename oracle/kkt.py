"""Optimality error of the original (unlifted) problem, eq. (8).

Written independently of the interior-point code: it takes a candidate point
(y, lam, omega_d, zL, zU) and evaluates the first-order KKT conditions of

    min f(y)  s.t.  c(y) = 0,  d(y) <= 0,  lb <= y <= ub

with the Lagrangian f + lam^T c + omega_d^T d - zL^T (y - lb) - zU^T (ub - y):
stationarity, primal feasibility, complementarity and dual sign conditions,
each as an infinity norm.  Returns a dict of the parts and their maximum.
"""
from __future__ import annotations

import numpy as np


def kkt_error(nlp, y, lam, omega_d, zL, zU):
    y = np.asarray(y, float)
    hasL, hasU = np.isfinite(nlp.lb), np.isfinite(nlp.ub)
    stat = nlp.grad(y) + nlp.jac_c(y).T @ lam - np.where(hasL, zL, 0.0) + np.where(hasU, zU, 0.0)
    if nlp.m_d:
        stat = stat + nlp.jac_d(y).T @ omega_d
    c = nlp.cons_c(y)
    parts = {"stationarity": float(np.max(np.abs(stat))),
             "equality": float(np.max(np.abs(c))) if len(c) else 0.0}
    if nlp.m_d:
        d = nlp.cons_d(y)
        parts["inequality"] = float(max(0.0, np.max(d)))
        parts["ineq_compl"] = float(np.max(np.abs(d * omega_d)))
        parts["ineq_sign"] = float(max(0.0, -np.min(omega_d)))
    gl = np.where(hasL, y - nlp.lb, 0.0)
    gu = np.where(hasU, nlp.ub - y, 0.0)
    parts["bound"] = float(max(0.0, -np.min(gl), -np.min(gu)))
    parts["bound_compl"] = float(max(np.max(np.abs(gl * np.where(hasL, zL, 0.0))),
                                     np.max(np.abs(gu * np.where(hasU, zU, 0.0)))))
    parts["bound_sign"] = float(max(0.0, -np.min(np.where(hasL, zL, 0.0)),
                                    -np.min(np.where(hasU, zU, 0.0))))
    parts["max"] = max(parts.values())
    return parts
