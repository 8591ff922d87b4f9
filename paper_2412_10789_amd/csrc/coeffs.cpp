// Host FP64 Chebyshev coefficients and truncation steps.
//
//  PPR  (Lemma 2): gamma = alpha / sqrt(2 alpha - alpha^2),
//                  beta  = (1 - sqrt(2 alpha - alpha^2)) / (1 - alpha),
//                  c_0 = gamma, c_k = 2 gamma beta^k; tail(K) = sum_{k>K} c_k
//                  = 2 gamma beta^{K+1} / (1 - beta) (Lemma 4 proof).
//  HKPR (Lemma 3): c_0 = e^{-t} I_0(t), c_k = 2 e^{-t} I_k(t).  The ratios
//                  I_k(t) / I_0(t) come from Miller's backward recurrence
//                  I_{k-1} = (2k/t) I_k + I_{k+1} (J.C.P. Miller, 1952),
//                  started far above the last wanted order; the result is
//                  normalised with e^{-t} (I_0 + 2 sum_{k>=1} I_k) = 1, the
//                  coefficient-sum identity of the Lemma 4 proof.  Backward
//                  recurrence keeps every order accurate to a few ulps
//                  relative, so tiny tail coefficients are reliable.
//  K selection: see cp_kmode in chebyprop.h.
//
//  Taylor weights of PwMethod (Def. 3, Def. 4, Alg. 1): PPR zeta_k =
//  alpha (1 - alpha)^k, HKPR zeta_k = e^{-t} t^k / k! (evaluated through
//  logarithms).  Every P^k e_s is a probability vector, so the l1 error
//  of N terms is exactly the tail sum_{k>=N} zeta_k: (1 - alpha)^N for PPR,
//  the Poisson(t) upper tail for HKPR (summed term by term from the far end).

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace cp {
namespace {

bool valid_kind_param(int32_t kind, double param) {
  if (kind == CP_PPR) return param > 0.0 && param < 1.0;
  if (kind == CP_HKPR) return param > 0.0 && std::isfinite(param);
  return false;
}

// e^{-t} I_k(t) style coefficients c_0..c_K (already including the factor 2
// for k >= 1), by backward recurrence from order `top`.
std::vector<double> hkpr_coeffs(double t, int32_t K) {
  const int32_t top = 2 * (K + (int32_t)std::ceil(t)) + 64;
  std::vector<double> J(top + 2, 0.0);
  J[top + 1] = 0.0;
  J[top] = 1e-300;
  for (int32_t k = top; k >= 1; --k) {
    J[k - 1] = (2.0 * k / t) * J[k] + J[k + 1];
    if (J[k - 1] > 1e250) {  // rescale the part computed so far
      for (int32_t j = k - 1; j <= top; ++j) J[j] *= 1e-250;
    }
  }
  // normalisation: J_0 + 2 sum_{k>=1} J_k, summed from the small end
  double s = 0.0;
  for (int32_t k = top; k >= 1; --k) s += J[k];
  s = J[0] + 2.0 * s;
  std::vector<double> c(K + 1);
  c[0] = J[0] / s;
  for (int32_t k = 1; k <= K; ++k) c[k] = 2.0 * J[k] / s;
  return c;
}

}  // namespace

cp_status coeffs_impl(int32_t kind, double param, int32_t K, double* c) {
  if (!c || K < 0 || !valid_kind_param(kind, param)) return CP_EINVAL;
  if (kind == CP_PPR) {
    const double root = std::sqrt(2.0 * param - param * param);
    const double gamma = param / root;
    const double beta = (1.0 - root) / (1.0 - param);
    c[0] = gamma;
    double bk = 1.0;
    for (int32_t k = 1; k <= K; ++k) {
      bk *= beta;
      c[k] = 2.0 * gamma * bk;
    }
    return CP_OK;
  }
  std::vector<double> h = hkpr_coeffs(param, K);
  std::copy(h.begin(), h.end(), c);
  return CP_OK;
}

cp_status choose_K_impl(int32_t kind, double param, double tol, int32_t kmode, int32_t K_fixed,
                        double vol, double d_s, int32_t K_max, int32_t* K_out, double* tail_out) {
  if (!K_out || !valid_kind_param(kind, param)) return CP_EINVAL;
  if (K_max <= 0) K_max = kDefaultKMax;
  const bool ppr = kind == CP_PPR;
  double gamma = 0, beta = 0;
  if (ppr) {
    const double root = std::sqrt(2.0 * param - param * param);
    gamma = param / root;
    beta = (1.0 - root) / (1.0 - param);
  }
  // tail(K) for a given K
  std::vector<double> hk;  // HKPR coefficients up to a horizon, filled lazily
  auto tail = [&](int32_t K) -> double {
    if (ppr) return 2.0 * gamma * std::pow(beta, (double)K + 1.0) / (1.0 - beta);
    const int32_t H = K + 64 + (int32_t)std::ceil(4.0 * std::sqrt(param)) + (int32_t)std::ceil(param);
    if ((int32_t)hk.size() < H + 1) hk = hkpr_coeffs(param, H + 64);
    double s = 0.0;
    for (int32_t k = (int32_t)hk.size() - 1; k > K; --k) s += std::fabs(hk[k]);
    return s;
  };

  int32_t K = 0;
  if (kmode == CP_K_FIXED) {
    if (K_fixed < 1) return CP_EINVAL;
    K = K_fixed;
    if (K > K_max) return CP_EKMAX;
  } else {
    if (!(tol > 0.0 && tol < 1.0)) return CP_EINVAL;
    if (kmode == CP_K_PAPER) {
      const double k = ppr ? std::log(1.0 / tol) / std::sqrt(param) : std::sqrt(param) * std::log(1.0 / tol);
      K = std::max<int32_t>(1, (int32_t)std::ceil(k));
      if (K > K_max) return CP_EKMAX;
    } else if (kmode == CP_K_CERTIFIED || kmode == CP_K_TAIL) {
      double L = 1.0;
      if (kmode == CP_K_CERTIFIED) {
        if (!(vol > 0.0 && d_s > 0.0)) return CP_EINVAL;
        L = std::sqrt(vol / d_s);
      }
      if (ppr) {
        // closed-form start, then adjust by one step either way
        double kk = std::log(tol * (1.0 - beta) / (2.0 * gamma * L)) / std::log(beta) - 1.0;
        K = std::max<int32_t>(1, (int32_t)std::floor(std::max(0.0, kk)));
        while (K > 1 && tail(K - 1) * L <= tol) --K;
        while (tail(K) * L > tol) {
          if (++K > K_max) return CP_EKMAX;
        }
      } else {
        K = 1;
        // coarse doubling then linear scan keeps the Miller recurrence short
        int32_t hi = 8;
        while (tail(hi) * L > tol) {
          if (hi >= K_max) return CP_EKMAX;
          hi = std::min(K_max, hi * 2);
        }
        int32_t lo = std::max(1, hi / 2);
        if (hi <= 8) lo = 1;
        for (K = lo; K < hi && tail(K) * L > tol; ++K) {
        }
      }
    } else {
      return CP_EINVAL;
    }
  }
  *K_out = K;
  if (tail_out) *tail_out = tail(K);
  return CP_OK;
}

namespace {

double hkpr_taylor_term(double t, int64_t k) {
  return std::exp(-t + (double)k * std::log(t) - std::lgamma((double)k + 1.0));
}

}  // namespace

cp_status taylor_impl(int32_t kind, double param, int32_t N, double* zeta) {
  if (!zeta || N < 0 || !valid_kind_param(kind, param)) return CP_EINVAL;
  if (kind == CP_PPR) {
    double q = 1.0;
    for (int32_t k = 0; k < N; ++k) {
      zeta[k] = param * q;
      q *= 1.0 - param;
    }
    return CP_OK;
  }
  for (int32_t k = 0; k < N; ++k) zeta[k] = hkpr_taylor_term(param, k);
  return CP_OK;
}

cp_status choose_N_impl(int32_t kind, double param, double tol, int32_t kmode, int32_t N_fixed,
                        int32_t N_max, int32_t* N_out, double* tail_out) {
  if (!N_out || !valid_kind_param(kind, param)) return CP_EINVAL;
  if (N_max <= 0) N_max = kDefaultKMax;
  const bool ppr = kind == CP_PPR;
  if (kmode != CP_K_FIXED && !(tol > 0.0 && tol < 1.0)) return CP_EINVAL;
  if (kmode != CP_K_FIXED && kmode != CP_K_CERTIFIED && kmode != CP_K_TAIL && kmode != CP_K_PAPER)
    return CP_EINVAL;
  // HKPR: suffix sums S[N] = sum_{k>=N} zeta_k up to a horizon past which the
  // Poisson mass is below 1e-30 of the total
  std::vector<double> S;
  if (!ppr) {
    const double t = param;
    if (t - 12.0 * std::sqrt(t) > (double)N_max) return CP_EKMAX;  // tail(N_max) is ~1
    const int64_t H = (int64_t)std::ceil(std::max((double)N_max, t + 12.0 * std::sqrt(t))) + 64;
    S.assign((size_t)H + 2, 0.0);
    for (int64_t k = H; k >= 0; --k) S[(size_t)k] = S[(size_t)k + 1] + hkpr_taylor_term(t, k);
  }
  auto tail = [&](int32_t N) -> double {
    return ppr ? std::pow(1.0 - param, (double)N) : S[(size_t)N];
  };
  int32_t N = 0;
  if (kmode == CP_K_FIXED) {
    if (N_fixed < 1) return CP_EINVAL;
    if (N_fixed > N_max) return CP_EKMAX;
    N = N_fixed;
  } else if (ppr) {
    const double guess = std::ceil(std::log(tol) / std::log(1.0 - param));
    if (!(guess <= (double)N_max + 1.0)) return CP_EKMAX;
    N = std::max<int32_t>(1, (int32_t)guess);
    while (N > 1 && tail(N - 1) <= tol) --N;
    while (tail(N) > tol) {
      if (++N > N_max) return CP_EKMAX;
    }
  } else {
    N = 1;
    while (tail(N) > tol) {
      if (++N > N_max) return CP_EKMAX;
    }
  }
  *N_out = N;
  if (tail_out) *tail_out = tail(N);
  return CP_OK;
}

}  // namespace cp
