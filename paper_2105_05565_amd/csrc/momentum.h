// Momentum schedules (Sec. 6, Sec. 8.1) on the host, shared by the single and the batched
// solver: gamma_k and beta_k of iteration k in a fixed FP64 operation order.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/rs.h"

namespace rs {

constexpr int64_t kSwitchNever = int64_t(1) << 40;

// The switch index of the theoretical rule (eq:parameterswitchtheory): the first k at which
// the constant-eta momentum of Cor 6.3, 1 - (2 - eta) / ((k+1)(1 - eta) + 1), reaches
// threshold; kSwitchNever when it never does (eta >= 1 or threshold >= 1).
inline int64_t momentum_switch(double eta, double threshold) {
#pragma clang fp contract(off)
  if (!(eta < 1.0) || !(threshold < 1.0)) return kSwitchNever;
  auto reached = [&](int64_t k) {
    double denom = (double)(k + 1) * (1.0 - eta);
    denom = denom + 1.0;
    return 1.0 - (2.0 - eta) / denom >= threshold;
  };
  // beta grows with k: start just below the crossing solved for k, then walk to it
  const double est = ((2.0 - eta) / (1.0 - threshold) - 1.0) / (1.0 - eta);
  if (!(est < (double)kSwitchNever)) return kSwitchNever;
  int64_t k = std::max<int64_t>(0, (int64_t)est - 3);
  while (k > 0 && reached(k - 1)) --k;
  while (!reached(k)) ++k;
  return k;
}

// gamma_k, beta_k of iteration k. sw: momentum_switch(o.eta, o.beta_max), used by THEORY.
inline void momentum_schedule(const rs_options& o, int64_t sw, int64_t k, double* gamma, double* beta) {
#pragma clang fp contract(off)
  switch (o.momentum) {
    case RS_MOMENTUM_NONE:
      *gamma = 1.0;
      *beta = 0.0;
      return;
    case RS_MOMENTUM_CONSTANT:
      *gamma = o.gamma;
      *beta = o.beta;
      return;
    case RS_MOMENTUM_THEORY: {
      // iterate-averaging parameters of Thm 6.2 with eta_k = eta before the switch and 1
      // from it on: zeta_k = (1 / eta_k) sum_{t<k} eta_t (1 - eta_t) (eq:zeta_kaptheo),
      // gamma_k = eta_k / (zeta_{k+1} + 1), beta_k = zeta_k / (zeta_{k+1} + 1)
      // (eq:etalambdatogammbetagen); the sum is min(k, switch) eta (1 - eta)
      const double eta = o.eta;
      const double c = eta * (1.0 - eta);
      const double eta_k = k < sw ? eta : 1.0;
      const double eta_k1 = k + 1 < sw ? eta : 1.0;
      const double zeta_k = (double)std::min(k, sw) * c / eta_k;
      const double zeta_k1 = (double)std::min(k + 1, sw) * c / eta_k1;
      *gamma = eta_k / (zeta_k1 + 1.0);
      *beta = zeta_k / (zeta_k1 + 1.0);
      return;
    }
    default: {
      // HEURISTIC (eq:parametersheurististic)
      const double eta = o.eta;
      double denom = (double)(k + 1) * (1.0 - eta);
      denom = denom + 1.0;
      const double bt = 1.0 - (2.0 - eta) / denom;
      *gamma = 1.0;
      *beta = std::min(o.beta_max, bt);
      return;
    }
  }
}

// Constants of the accelerated method (Alg. 3) for 0 < mu <= 1 <= nu <= 1 / mu, in this
// FP64 order: beta = 1 - sqrt(mu / nu), gamma = sqrt(1 / (mu nu)), alpha = 1 / (1 + sqrt(nu / mu)).
inline void accel_constants(double mu, double nu, double* alpha, double* beta, double* gamma) {
#pragma clang fp contract(off)
  *beta = 1.0 - std::sqrt(mu / nu);
  *gamma = std::sqrt(1.0 / (mu * nu));
  *alpha = 1.0 / (1.0 + std::sqrt(nu / mu));
}

// Validation of the momentum settings; returns nullptr when they are usable.
inline const char* momentum_invalid(const rs_options& o) {
  if (o.momentum < RS_MOMENTUM_NONE || o.momentum > RS_MOMENTUM_THEORY) return "unknown momentum";
  if (o.momentum == RS_MOMENTUM_THEORY && !(o.eta > 0.0 && o.eta <= 1.0))
    return "the theoretical momentum rule needs 0 < eta <= 1";
  if (o.momentum == RS_MOMENTUM_THEORY && !(o.beta_max == o.beta_max)) return "beta_max is NaN";
  return nullptr;
}

}  // namespace rs
