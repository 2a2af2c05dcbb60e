"""Sensitivities of the NMPC solution (oracle side).

At the returned iterate z* of the lifted barrier problem (fixed final mu) the
primal-dual conditions F(z; p) = 0 of Section 3.2 (eqs. 8-9 for the lifted
problem of eq. 16, with bound multipliers) define z*(p).  The implicit function
theorem gives dz/dp = -(dF/dz)^{-1} dF/dp; eliminating ds, domega, dbeta and the
bound-multiplier directions exactly as the condensation of eqs. (14) and (17)
leaves

    K dy/dp = b(p),   K = W + Sigma + J_c^T (Q+ + Q-) J_c + J_d^T Q_d J_d,
    b(p) = - d(grad f)/dp - J_c^T (Q+ + Q-) dc/dp - J_d^T Q_d dd/dp,

with Q = beta / s on the lifted rows (the two lifted copies of an equality act
as one penalty of weight Q+ + Q-).  Then du_1/dp = S_u dy/dp and
df*/dp = df/dp + grad f^T dy/dp.

Near the solution the lifted weights are of order mu / gamma^2, so the
condensed matrix formed in floating point carries the curvature W only to an
absolute precision of about eps |J^T Q J|, which shows in the sensitivities at
the 1e-5 level.  The oracle therefore solves the equivalent uncondensed system
(the step before the elimination of the multiplier directions)

    [ W + Sigma    J^T    ] [dy/dp ]   [ -d(grad f)/dp ]
    [ J          -Q^{-1}  ] [dlam/dp] = [ -d(c, d)/dp   ]

with a sparse LU factorization, independently of the interior-point code.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def condensed_matrix(ipm, st):
    """K at the iterate st (no regularization) and the lifted weights."""
    nlp, mc = ipm.nlp, ipm.mc
    lam = st.omega[:mc] - st.omega[mc:2 * mc]
    lam_d = st.omega[2 * mc:]
    W = nlp.hess(st.y, lam, lam_d)
    gL, gU = ipm.gaps(st.y)
    sig = np.where(ipm.hasL, st.zL / gL, 0.0) + np.where(ipm.hasU, st.zU / gU, 0.0)
    Q = st.beta / st.s
    Qc = Q[:mc] + Q[mc:2 * mc]
    Qd = Q[2 * mc:]
    Jc, Jd = nlp.jac_c(st.y), nlp.jac_d(st.y)
    K = W + sp.diags(sig) + Jc.T @ sp.diags(Qc) @ Jc
    if ipm.md:
        K = K + Jd.T @ sp.diags(Qd) @ Jd
    return K.toarray(), Jc, Jd, Qc, Qd


def augmented_matrix(ipm, st):
    """[[W + Sigma, J^T], [J, -Q^{-1}]] at st, J = [J_c; J_d], Q = (Q+ + Q-, Q_d)."""
    nlp, mc = ipm.nlp, ipm.mc
    lam = st.omega[:mc] - st.omega[mc:2 * mc]
    W = nlp.hess(st.y, lam, st.omega[2 * mc:])
    gL, gU = ipm.gaps(st.y)
    sig = np.where(ipm.hasL, st.zL / gL, 0.0) + np.where(ipm.hasU, st.zU / gU, 0.0)
    Q = st.beta / st.s
    Qa = np.concatenate([Q[:mc] + Q[mc:2 * mc], Q[2 * mc:]])
    J = sp.vstack([nlp.jac_c(st.y), nlp.jac_d(st.y)]).tocsr()
    A = sp.bmat([[W + sp.diags(sig), J.T], [J, sp.diags(-1.0 / Qa)]]).tocsc()
    return A, J, Qa


def sensitivities(ipm, st):
    """dy/dp, du1/dp and df*/dp for every parameter group of the model."""
    nlp = ipm.nlp
    A, J, _ = augmented_matrix(ipm, st)
    lu = spla.splu(A)
    gf = nlp.grad(st.y)
    iu = nlp.u1_index()
    n = nlp.n
    out = {}
    for name, (dc, dd, dgrad, dfp) in nlp.parameter_derivatives(st.y).items():
        rhs = -np.vstack([dgrad, dc, dd])
        dy = lu.solve(np.asarray(rhs, dtype=np.float64))[:n, :]
        out[name] = dict(dy=dy, du1=dy[iu, :], df=dfp + gf @ dy)
    return out


def vjp(ipm, st, seed_u1, seed_obj):
    """Gradient of seed_u1 . u1* + seed_obj f* with respect to every parameter group."""
    sens = sensitivities(ipm, st)
    return {k: np.asarray(seed_u1) @ v["du1"] + seed_obj * v["df"] for k, v in sens.items()}
