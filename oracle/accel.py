"""Sketch-and-project with acceleration (Alg. 3, Sec. 9).

Three iterate sequences w, z, v and their residuals r_w = A w - b, r_z = A z - b,
r_v = A v - b. With mu in (0, 1] and nu in [1, 1/mu] (the parameters the paper sets
from spectral quantities, eq:mu+nu; here they are inputs),
    beta = 1 - sqrt(mu / nu),  gamma = sqrt(1 / (mu nu)),  alpha = 1 / (1 + sqrt(nu / mu)).
One iteration k:
    r_z^k = alpha r_v^k + (1 - alpha) r_w^k        (formed before it is sketched)
    delta = least-norm solution of (S^T A S) delta = S^T r_z^k,  g = S delta
    z^k = alpha v^k + (1 - alpha) w^k
    w^{k+1} = z^k - g,            r_w^{k+1} = r_z^k - A g
    v^{k+1} = beta v^k + (1 - beta) z^k - gamma g,
    r_v^{k+1} = beta r_v^k + (1 - beta) r_z^k - gamma A g
starting from w = v = 0 and r_w = r_v = -b. The loop runs while
||r_v^k|| / ||r_v^0|| > tol and k < max_iter; the output is w. With mu = nu = 1
(beta = 0, gamma = 1, alpha = 1/2) the iterates are those of Alg. 1.

Part of the oracle: test infrastructure only.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from .linalg import least_norm_solution
from .solver import draw_sketch, sketched_products


def accel_constants(mu, nu):
    """(alpha, beta, gamma) of Alg. 3, in this FP64 operation order."""
    if not (0.0 < mu <= 1.0) or not (1.0 <= nu <= 1.0 / mu):
        raise ValueError("need 0 < mu <= 1 and 1 <= nu <= 1 / mu")
    beta = 1.0 - math.sqrt(mu / nu)
    gamma = math.sqrt(1.0 / (mu * nu))
    alpha = 1.0 / (1.0 + math.sqrt(nu / mu))
    return alpha, beta, gamma


@dataclass
class AccelState:
    w: np.ndarray
    v: np.ndarray
    r_w: np.ndarray
    r_v: np.ndarray
    k: int
    r0_norm: float
    history: list = field(default_factory=list)   # ||r_v^k|| / ||r_v^0||


def accel_init(system):
    r0 = -system.b.copy()
    return AccelState(w=np.zeros(system.m), v=np.zeros(system.m), r_w=r0, r_v=r0.copy(), k=0,
                      r0_norm=float(np.linalg.norm(r0)), history=[1.0])


def accel_step(system, state, opts, mu, nu, sketch=None):
    """One iteration of Alg. 3 in place; returns (delta, sketch)."""
    alpha, beta, gamma = accel_constants(mu, nu)
    if sketch is None:
        sketch = draw_sketch(system, opts, state.k)
    S, AS, G, active = sketched_products(system, sketch)
    r_z = alpha * state.r_v + (1.0 - alpha) * state.r_w
    rho = np.asarray(S.T @ r_z).ravel()
    delta = least_norm_solution(G, rho, active)
    g = np.asarray(S @ delta).ravel()
    Ag = AS @ delta
    z = alpha * state.v + (1.0 - alpha) * state.w
    w_next = z - g
    v_next = beta * state.v + (1.0 - beta) * z - gamma * g
    state.r_w, state.r_v = r_z - Ag, beta * state.r_v + (1.0 - beta) * r_z - gamma * Ag
    state.w, state.v = w_next, v_next
    state.k += 1
    state.history.append(float(np.linalg.norm(state.r_v)) / state.r0_norm)
    return delta, sketch


def accel_solve(system, opts, mu, nu, state=None):
    if state is None:
        state = accel_init(system)
    if state.r0_norm == 0.0:
        return state
    while state.history[-1] > opts.tol and state.k < opts.max_iter:
        accel_step(system, state, opts, mu, nu)
    return state
