"""Reverse-mode gradient of an edge-readout loss (oracle, full storage).

TEST INFRASTRUCTURE ONLY.

The paper has no adjoint; this is the exact transpose of the forward step of
oracle.lbm, written from the chain rule.  With
  X_t = S_t + e dt J                  (e = 1 split form, 0 fused Taylor)
  Y_t = alpha X_t + beta M X_t + (1 - e) dt J
  S_{t+1} = L(Y_t) + ghost constants
and lambda_T = dLoss/dS_T, for t = T-1 .. 0:
  mu_t     = L^T lambda_{t+1}          (dLoss/dY_t)
  nu_t     = M^T mu_t                  (with a per-cell phase mixture, whose
             scattering is (1 - sum f_k) M X + sum f_k M_k X: the same
             fractions of M^T mu_t and M_k^T mu_t)
  lambda_t = alpha mu_t + beta nu_t    (dLoss/dX_t = dLoss/dS_t)
  g_alpha += <mu_t, X_t>,  g_beta += <nu_t, X_t>   (per cell, over d and s)
  g_emis  += dt <e lambda_t + (1 - e) mu_t, jprof>
then g_tau = g_alpha dalpha/dtau + g_beta dbeta/dtau and likewise for albedo.
With dichroic absorption the scattering acts on X_d = D(xi) X, xi = (1 - albedo)
tau eta, so the sums above take X_d, lambda_t = D^T (alpha mu_t + beta nu_t),
g_xi += <alpha mu_t + beta nu_t, dD/dxi X_t>, and g_tau, g_albedo gain
g_xi dxi/dtau = g_xi (1 - albedo) eta and g_xi dxi/dalbedo = -g_xi tau eta.
All states are stored in float64 (no checkpointing).
"""
import numpy as np

from . import lbm


def adjoint(S0, prob, nsteps, lam_T):
    """Returns dict(lambda0, g_alpha, g_beta, g_tau, g_albedo, g_emis)."""
    n, C = prob.n, prob.nx * prob.ny
    J = prob.emission_field()
    e = 0.0 if prob.fused_taylor else 1.0
    _, hist = lbm.run(S0, prob, nsteps, keep=True)
    jp = prob.jprof.reshape(n, 4, 1)
    lam = np.array(lam_T, dtype=np.float64).reshape(prob.shape)
    al = prob.alpha.reshape(C)
    be = prob.beta.reshape(C)
    g_al = np.zeros(C)
    g_be = np.zeros(C)
    g_em = np.zeros(C)
    g_xi = np.zeros(C)
    for t in range(nsteps - 1, -1, -1):
        X = (hist[t] + e * prob.dt * J).reshape(4 * n, C)
        X0 = X
        if prob.eta is not None:
            X = lbm.dichroic_absorption(X0, prob)
        mu = lbm.stream_transpose(lam, prob).reshape(4 * n, C)
        nu = lbm.scatter_product(prob, mu, transpose=True)
        g_al += np.sum(mu * X, axis=0)
        g_be += np.sum(nu * X, axis=0)
        lam_x = al[None, :] * mu + be[None, :] * nu
        if prob.eta is not None:
            g_xi += np.sum(lam_x * dichroic_derivative(X0, prob), axis=0)
            lam_x = lbm.dichroic_absorption(lam_x, prob)   # D^T = D (symmetric in I, Q)
        src = e * lam_x + (1.0 - e) * mu
        g_em += prob.dt * np.sum(src.reshape(n, 4, C) * jp, axis=(0, 1))
        lam = lam_x.reshape(prob.shape)
    dal_dt, dal_dw, dbe_dt, dbe_dw = lbm.coefficient_derivatives(
        prob.tau, prob.albedo, prob.abs_taylor, prob.scat_exp, prob.fused_taylor)
    shp = (prob.ny, prob.nx)
    g_al = g_al.reshape(shp)
    g_be = g_be.reshape(shp)
    g_xi = g_xi.reshape(shp)
    eta = 0.0 if prob.eta is None else prob.eta
    return {
        "lambda0": lam,
        "g_alpha": g_al,
        "g_beta": g_be,
        "g_tau": g_al * dal_dt + g_be * dbe_dt + g_xi * (1.0 - prob.albedo) * eta,
        "g_albedo": g_al * dal_dw + g_be * dbe_dw - g_xi * prob.tau * eta,
        "g_emis": g_em.reshape(shp),
    }


def dichroic_derivative(X, prob):
    """d/dxi of the dichroic factors applied to X (xi = tau_abs eta per cell):
    I + Q scales by exp(-xi w_d), I - Q by exp(xi w_d), so their derivatives
    are -w_d and +w_d times the scaled sums."""
    xi = ((1.0 - prob.albedo) * prob.tau * prob.eta).reshape(1, -1)
    w = np.sin(prob.dirs.theta) ** 2
    Xd = X.reshape(prob.n, 4, -1)
    dplus = -w[:, None] * (Xd[:, 0] + Xd[:, 1]) * np.exp(-xi * w[:, None])
    dminus = w[:, None] * (Xd[:, 0] - Xd[:, 1]) * np.exp(xi * w[:, None])
    out = np.zeros_like(Xd)
    out[:, 0] = 0.5 * (dplus + dminus)
    out[:, 1] = 0.5 * (dplus - dminus)
    return out.reshape(X.shape)


def edge_loss_of(params, base_prob, S0, nsteps, edge):
    """Forward loss for a modified (tau, albedo, emis) triple (for finite differences)."""
    tau, alb, em = params
    p = lbm.Problem(base_prob.nx, base_prob.ny, base_prob.dirs, base_prob.shifts,
                    base_prob.M, base_prob.dt, base_prob.bc, tau, alb, em,
                    base_prob.jprof, base_prob.inflow_cells, base_prob.abs_taylor,
                    base_prob.scat_exp, base_prob.fused_taylor, M2=base_prob.mix_M, frac=base_prob.mix_f,
                    dichroism=base_prob.eta)
    S = lbm.run(S0, p, nsteps)
    return lbm.edge_loss(S, p, edge)[0]


def central_difference(base_prob, S0, nsteps, edge, which, cell, rel_h=1e-6):
    """FP64 central difference of the edge loss wrt one per-cell parameter."""
    y, x = cell
    arrs = [base_prob.tau.copy(), base_prob.albedo.copy(), base_prob.emis.copy()]
    k = {"tau": 0, "albedo": 1, "emis": 2}[which]
    v = arrs[k][y, x]
    h = rel_h * max(abs(v), 1e-3)
    plus = [a.copy() for a in arrs]
    minus = [a.copy() for a in arrs]
    plus[k][y, x] = v + h
    minus[k][y, x] = v - h
    lp = edge_loss_of(plus, base_prob, S0, nsteps, edge)
    lm = edge_loss_of(minus, base_prob, S0, nsteps, edge)
    return (lp - lm) / (2.0 * h)
