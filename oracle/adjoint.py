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
df*/dp = df/dp + grad f^T dy/dp.  K is formed and factored here on its own
(dense Cholesky), independently of the interior-point iterations.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


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


def sensitivities(ipm, st):
    """dy/dp, du1/dp and df*/dp for every parameter group of the model."""
    nlp = ipm.nlp
    K, Jc, Jd, Qc, Qd = condensed_matrix(ipm, st)
    Lc = np.linalg.cholesky(K)
    gf = nlp.grad(st.y)
    iu = nlp.u1_index()
    out = {}
    for name, (dc, dd, dgrad, dfp) in nlp.parameter_derivatives(st.y).items():
        b = -dgrad - Jc.T @ (Qc[:, None] * dc)
        if ipm.md:
            b = b - Jd.T @ (Qd[:, None] * dd)
        dy = np.linalg.solve(Lc.T, np.linalg.solve(Lc, b))
        out[name] = dict(dy=dy, du1=dy[iu, :], df=dfp + gf @ dy)
    return out


def vjp(ipm, st, seed_u1, seed_obj):
    """Gradient of seed_u1 . u1* + seed_obj f* with respect to every parameter group."""
    sens = sensitivities(ipm, st)
    return {k: np.asarray(seed_u1) @ v["du1"] + seed_obj * v["df"] for k, v in sens.items()}
