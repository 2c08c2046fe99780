"""Sketch-and-project with momentum for ridge regression (Alg. 1, Alg. 2).

One iteration k (Alg. 2, with Alg. 1 as the case beta_k = 0, gamma_k = 1):

1. gamma_k, beta_k from the momentum schedule;
2. draw S_k ~ D (see ``sketch``);
3. AS_k = A S_k = Z (Z^T S_k) + lambda S_k (kernel ridge: K (K S_k) + lambda K S_k);
4. the sketched system G = S_k^T A S_k and sketched residual rho = S_k^T r^k;
5. delta_k = least-norm solution of G delta = rho (eq:sketched_system);
6. w^{k+1} = (1 + beta_k) w^k - beta_k w^{k-1} - gamma_k S_k delta_k;
7. r^{k+1} = (1 + beta_k) r^k - beta_k r^{k-1} - gamma_k AS_k delta_k
   (eq:res_update_mom; the residual is r = A w - b, Sec. 3).

Initialisation w^{-1} = w^0 = 0 and r^{-1} = r^0 = -b. The loop runs while
||r^k|| / ||r^0|| > epsilon and k < max_iter (the paper prints the loop test
with the inequality reversed and has no iteration cap).

Momentum schedules:

* "none":      gamma_k = 1, beta_k = 0 (Alg. 1);
* "constant":  gamma_k = 1, beta_k = 0.5, the constant setting compared in
  Sec. 8.1;
* "heuristic": gamma_k = 1 and beta_k = 1 - (2 - eta) / ((k+1)(1 - eta) + 1)
  (eq:parametersheurististic, the beta of eq:cst_eta_lambda_to_gamma_beta_formula),
  capped at beta_max. eta = 0.995 and beta_max = 0.5 by default: the paper
  fixes neither for this rule, but says beta_k rises from 0 to about 0.5.
  The operations are evaluated in exactly this order in FP64.
* "theory": the increasing-momentum rule of eq:parameterswitchtheory in the
  iterate-averaging parameters of Thm 6.2: eta_k = eta (0.995) before the switch
  and 1 from it on, zeta_k = (1 / eta_k) sum_{t<k} eta_t (1 - eta_t)
  (eq:zeta_kaptheo, zeta_0 = 0), gamma_k = eta_k / (zeta_{k+1} + 1) and
  beta_k = zeta_k / (zeta_{k+1} + 1) (eq:etalambdatogammbetagen). The paper
  switches when beta_k reaches 0.5, but beta_k itself depends on eta_{k+1}; the
  switch index K is read as the first k at which the constant-eta momentum of
  Cor 6.3 (eq:cst_eta_lambda_to_gamma_beta_formula) reaches beta_max (0.5), so that
  the schedule is a function of k alone. With eta = 0.995, K = 201 and gamma_k,
  beta_k settle at 0.5 from there on. The sum is min(k, K) * (eta (1 - eta)).

Part of the oracle: test infrastructure only.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import sketch as sk
from .linalg import least_norm_solution


@dataclass
class Options:
    sketch: str = "subsample"       # subsample | count | subcount | weighted
    tau: int = 50
    sum_size: int = 0               # SubCount k; 0 = the paper's rule
    momentum: str = "none"          # none | constant | heuristic | theory
    eta: float = 0.995
    beta_max: float = 0.5
    gamma_const: float = 1.0
    beta_const: float = 0.5
    tol: float = 1e-6
    max_iter: int = 10000
    seed: int = 1
    problem_id: int = 0
    slot: int = 0


def schedule(opts, k):
    """(gamma_k, beta_k) for iteration k >= 0."""
    if opts.momentum == "none":
        return 1.0, 0.0
    if opts.momentum == "constant":
        return float(opts.gamma_const), float(opts.beta_const)
    if opts.momentum == "heuristic":
        eta = float(opts.eta)
        denom = float(k + 1) * (1.0 - eta)
        denom = denom + 1.0
        beta = 1.0 - (2.0 - eta) / denom
        return 1.0, min(float(opts.beta_max), beta)
    if opts.momentum == "theory":
        eta = float(opts.eta)
        K = theory_switch(eta, float(opts.beta_max))
        c = eta * (1.0 - eta)
        eta_k = eta if k < K else 1.0
        eta_k1 = eta if k + 1 < K else 1.0
        zeta_k = float(min(k, K)) * c / eta_k
        zeta_k1 = float(min(k + 1, K)) * c / eta_k1
        return eta_k / (zeta_k1 + 1.0), zeta_k / (zeta_k1 + 1.0)
    raise ValueError(f"unknown momentum {opts.momentum!r}")


SWITCH_NEVER = 1 << 40


def theory_switch(eta, threshold):
    """First k at which beta_k = 1 - (2 - eta) / ((k+1)(1 - eta) + 1), the constant-eta
    momentum of Cor 6.3, reaches threshold; SWITCH_NEVER when it never does."""
    if not (eta < 1.0) or not (threshold < 1.0):
        return SWITCH_NEVER
    def reached(k):
        denom = float(k + 1) * (1.0 - eta)
        denom = denom + 1.0
        return 1.0 - (2.0 - eta) / denom >= threshold

    # (k+1)(1 - eta) + 1 >= (2 - eta) / (1 - threshold) gives a start near K; beta_k
    # increases with k, so step down while the threshold is already reached, then up
    k = max(0, int(((2.0 - eta) / (1.0 - threshold) - 1.0) / (1.0 - eta)) - 3)
    while k > 0 and reached(k - 1):
        k -= 1
    while not reached(k):
        k += 1
    return k


@dataclass
class State:
    w: np.ndarray
    w_prev: np.ndarray
    r: np.ndarray
    r_prev: np.ndarray
    k: int
    r0_norm: float
    history: list = field(default_factory=list)   # ||r^k|| / ||r^0||, k = 0, 1, ...


def init_state(system):
    m = system.m
    r0 = -system.b.copy()
    r0n = float(np.linalg.norm(r0))
    return State(w=np.zeros(m), w_prev=np.zeros(m), r=r0, r_prev=r0.copy(), k=0,
                 r0_norm=r0n, history=[1.0])


def draw_sketch(system, opts, k, q=None):
    return sk.draw(opts.sketch, opts.seed, opts.problem_id, k, system.m, opts.tau,
                   sum_size=opts.sum_size, slot=opts.slot, q=q)


def sketched_products(system, sketch):
    """AS = Z (Z^T S) + lambda S (m x tau, dense), G = S^T AS, and the column mask."""
    S = sketch.matrix()
    if hasattr(system, "sketched_AS"):      # kernel ridge: A S = K (K S) + lambda K S
        AS = system.sketched_AS(S)
    else:
        T = system.Z.T @ S                  # K x tau
        AS = system.Z @ T                   # m x tau
        AS = (AS.toarray() if sp.issparse(AS) else np.asarray(AS)) + system.lam * S.toarray()
    G = np.asarray(S.T @ AS)
    active = np.zeros(sketch.tau, dtype=bool)
    active[sketch.cols] = True
    return S, AS, G, active


def step(system, state, opts, sketch=None, q=None):
    """Advance one iteration of Alg. 2 in place and return (delta, sketch, AS)."""
    k = state.k
    gamma, beta = schedule(opts, k)
    if sketch is None:
        sketch = draw_sketch(system, opts, k, q=q)
    S, AS, G, active = sketched_products(system, sketch)
    rho = np.asarray(S.T @ state.r).ravel()
    delta = least_norm_solution(G, rho, active)
    Sdelta = np.asarray(S @ delta).ravel()
    ASdelta = AS @ delta
    w_next = (1.0 + beta) * state.w - beta * state.w_prev - gamma * Sdelta
    r_next = (1.0 + beta) * state.r - beta * state.r_prev - gamma * ASdelta
    state.w_prev, state.w = state.w, w_next
    state.r_prev, state.r = state.r, r_next
    state.k = k + 1
    state.history.append(float(np.linalg.norm(r_next)) / state.r0_norm)
    return delta, sketch, AS


def solve(system, opts, state=None):
    """Iterate until ||r^k|| / ||r^0|| <= tol or k = max_iter; returns the state."""
    if state is None:
        state = init_state(system)
    if state.r0_norm == 0.0:
        return state
    while state.history[-1] > opts.tol and state.k < opts.max_iter:
        step(system, state, opts)
    return state


def true_residual(system, w):
    """A w - b computed from Z directly (not from the recursion)."""
    return system.matvec(w) - system.b
