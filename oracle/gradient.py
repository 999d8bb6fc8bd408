"""Derivative of the transport cost with respect to the two marginals.

The relaxed problem is the barrier minimisation of Sec. 2.4,
    P_mu(rho_in, rho_f) = min_rho KE(rho) - mu dt sum_k sum_i a'_i log rho_i^k,
under the per-slice mass constraints, and the reported cost is KE at the
minimiser.  The envelope theorem gives dP_mu/dtheta as the partial
derivative of KE at fixed optimal (phi, rho):
    d/d rho_in = -Omega^T phi^1     - dt/4 R_T (grad phi^1)^2
    d/d rho_f  =  Omega^T phi^{K+1} - dt/4 R_T (grad phi^{K+1})^2.
cost = P_mu + mu dt sum a' log rho*, so dcost = envelope + dt (a' s)^T drho*.
The last term comes from one adjoint solve with the transposed KKT matrix;
after eliminating the slack rows it is the same symmetric J_s:
    J_s (q_phi; q_rho) = (0; dt a' s),
and the correction is -q_phi^T dF_phi/dtheta, where only F_phi^1 depends on
rho_in and only F_phi^{K+1} on rho_f.  Gradients are defined modulo a'
(global constant of phi, mass constraint) and returned Euclidean-projected
orthogonal to a'.

Pins (tests/test_oracle_gradient.py): central finite differences of the
oracle cost along mass-preserving directions on small meshes.
"""

from __future__ import annotations

import numpy as np

from .ipm import Problem, saddle_matrix, solve_saddle_direct


def _project_out(v, ac):
    return v - ac * float(v @ ac) / float(ac @ ac)


def envelope_gradient(prob: Problem, phi):
    o, dt = prob.ops, prob.dt
    g1 = o.grad @ phi[0]
    gK = o.grad @ phi[-1]
    g_in = -(o.Om.T @ phi[0]) - 0.25 * dt * (o.RT @ (g1 * g1))
    g_f = (o.Om.T @ phi[-1]) - 0.25 * dt * (o.RT @ (gK * gK))
    return g_in, g_f


def cost_gradient(prob: Problem, phi, rho, s):
    """(d cost/d rho_in, d cost/d rho_f) at a converged solution."""
    o, K, dt = prob.ops, prob.K, prob.dt
    g_in, g_f = envelope_gradient(prob, phi)
    J = saddle_matrix(prob, phi, rho, s)
    rhs = np.concatenate([np.zeros((K + 1) * prob.nf), (dt * o.ac[None, :] * s).ravel()])
    q = solve_saddle_direct(J, rhs)
    qphi = q[: (K + 1) * prob.nf].reshape(K + 1, prob.nf)
    g1 = o.grad @ phi[0]
    gK = o.grad @ phi[-1]
    # dF_phi^1/d rho_in = Omega/dt + 1/2 grad^T W Diag(grad phi^1) R_E
    corr_in = -((o.Om.T @ qphi[0]) / dt + 0.5 * (o.RT @ (g1 * (o.grad @ qphi[0]))))
    # dF_phi^{K+1}/d rho_f = -Omega/dt + 1/2 grad^T W Diag(grad phi^{K+1}) R_E
    corr_f = -(-(o.Om.T @ qphi[-1]) / dt + 0.5 * (o.RT @ (gK * (o.grad @ qphi[-1]))))
    return _project_out(g_in + corr_in, o.ac), _project_out(g_f + corr_f, o.ac)
