// sabr_oracle.cpp -- CPU reference for SA calibration of SABR/LIBOR models.
//
// TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the CPU
// baseline leg of the benchmark, never by the product path.  FP64 throughout,
// glibc libm, no fast-math, no FMA contraction (-ffp-contract=off).  Every
// function is written for readability, not speed; each cites the passage of
// arXiv 2408.01470 it follows.  The one scalar template parameter S is either
// double or a forward-mode dual number, so the same code yields exact
// gradients (to rounding) for the adjoint checks.
//
// Parity status: the cost, maps, Black, Philox, SA and LM functions are pinned
// by tests (paper worked example, closed forms, library references, brute
// force).  See the test-suite for each pin.
#include "sabr_oracle.h"

#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

thread_local std::string g_err;
int32_t fail(const std::string &msg) {
  g_err = msg;
  return -1;
}
const double kInf = std::numeric_limits<double>::infinity();

// ---------------------------------------------------------------------------
// Forward-mode dual numbers: value plus N partial derivatives.
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) {
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
  Dual(double x) : v(x) {  // NOLINT: implicit promotion of constants
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
};

inline double val(double x) { return x; }
template <int N>
inline double val(const Dual<N> &x) { return x.v; }

template <int N>
Dual<N> chain(double v, double dv, const Dual<N> &a) {  // f(a) with f'(a) = dv
  Dual<N> r(v);
  for (int i = 0; i < N; ++i) r.d[i] = dv * a.d[i];
  return r;
}
template <int N>
Dual<N> operator+(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r(a.v + b.v);
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N>
Dual<N> operator-(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r(a.v - b.v);
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N>
Dual<N> operator-(const Dual<N> &a) {
  Dual<N> r(-a.v);
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N>
Dual<N> operator*(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r(a.v * b.v);
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N>
Dual<N> operator/(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r(a.v / b.v);
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
template <int N> Dual<N> operator+(const Dual<N> &a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N> &b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N> &a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N> &b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N> &a, double b) { return a * Dual<N>(b); }
template <int N> Dual<N> operator*(double a, const Dual<N> &b) { return Dual<N>(a) * b; }
template <int N> Dual<N> operator/(const Dual<N> &a, double b) { return a / Dual<N>(b); }
template <int N> Dual<N> operator/(double a, const Dual<N> &b) { return Dual<N>(a) / b; }
template <int N> Dual<N> &operator+=(Dual<N> &a, const Dual<N> &b) { return a = a + b; }

template <int N>
Dual<N> exp(const Dual<N> &a) {
  double e = std::exp(a.v);
  return chain(e, e, a);
}
template <int N>
Dual<N> log(const Dual<N> &a) { return chain(std::log(a.v), 1.0 / a.v, a); }
template <int N>
Dual<N> log1p(const Dual<N> &a) { return chain(std::log1p(a.v), 1.0 / (1.0 + a.v), a); }
template <int N>
Dual<N> sqrt(const Dual<N> &a) {
  double s = std::sqrt(a.v);
  return chain(s, 0.5 / s, a);
}
template <int N>
Dual<N> erfc(const Dual<N> &a) {
  // d/dx erfc(x) = -2/sqrt(pi) exp(-x^2)
  return chain(std::erfc(a.v), -2.0 / std::sqrt(M_PI) * std::exp(-a.v * a.v), a);
}
// base^e for a constant base (market data) and a parameter-dependent exponent
template <int N>
Dual<N> pow(double base, const Dual<N> &e) {
  double p = std::pow(base, e.v);
  return chain(p, p * std::log(base), e);
}

using std::erfc;
using std::exp;
using std::log;
using std::log1p;
using std::pow;
using std::sqrt;

// ---------------------------------------------------------------------------
// Hagan 2002 lognormal implied volatility (the formula the paper cites for
// the SABR model, with z / x(z) and the O(T) correction; Sec. 2.1 cites Hagan
// et al. and Obloj).  Written out from its textbook definition:
//   L = ln(f/K), q = (f K)^((1-beta)/2), z = (nu/alpha) q L,
//   x(z) = ln((sqrt(1 - 2 rho z + z^2) + z - rho) / (1 - rho)),
//   sigma = alpha / (q D1) * z/x(z) * corr,
//   D1 = 1 + (1-beta)^2 L^2/24 + (1-beta)^4 L^4/1920,
//   corr = 1 + [(1-beta)^2 alpha^2/(24 q^2) + rho beta nu alpha/(4 q)
//              + (2 - 3 rho^2) nu^2/24] T.
// ---------------------------------------------------------------------------
template <class S>
S chi(const S &z, const S &rho) {
  // z / x(z) with the removable singularity chi(0) = 1.  x(z) is evaluated in
  // one of three algebraically identical forms so that no branch subtracts
  // nearly equal numbers:  with s = sqrt(1 - 2 rho z + z^2),
  //   (s + z - rho)/(1 - rho) = 1 + 2z/(s + 1 - z) = (1 + rho)/(s - z + rho).
  if (val(z) == 0.0) return S(1.0);
  S s = sqrt(1.0 - 2.0 * rho * z + z * z);
  S x;
  if (val(z) > 1.0)
    x = log((s + z - rho) / (1.0 - rho));
  else if (val(z) < -1.0)
    x = log((1.0 + rho) / (s - z + rho));
  else
    x = log1p(2.0 * z / (s + 1.0 - z));
  return z / x;
}

template <class S>
S hagan2002_vol(double f, double K, double T, const S &alpha, const S &beta, const S &rho,
                const S &nu) {
  const double L = log(f / K);
  S omb = 1.0 - beta;
  S q = pow(f * K, 0.5 * omb);
  S z = (nu / alpha) * q * L;
  S ch = chi(z, rho);
  S omb2 = omb * omb;
  S D1 = 1.0 + omb2 * (L * L) / 24.0 + omb2 * omb2 * (L * L * L * L) / 1920.0;
  S corr = 1.0 + (omb2 * alpha * alpha / (24.0 * q * q) + rho * beta * nu * alpha / (4.0 * q) +
                  (2.0 - 3.0 * rho * rho) * nu * nu / 24.0) *
                     T;
  return alpha / (q * D1) * ch * corr;
}

// Paper eq. (sigmaHagan), Sec. 2.1, exactly as printed: second order in the
// moneyness k = ln(K/f), omega = f^(1-beta)/alpha, no expiry dependence.
template <class S>
S paper_eq3_vol(double f, double K, const S &alpha, const S &beta, const S &rho, const S &nu) {
  S omb = 1.0 - beta;
  S fpow = pow(f, omb);
  S omega = fpow / alpha;
  const double k = log(K / f);
  S rso = rho * nu * omega;
  S bracket = 1.0 - 0.5 * (omb - rso) * k +
              (omb * omb + (2.0 - 3.0 * rho * rho) * nu * nu * omega * omega +
               3.0 * (omb - rso)) *
                  (k * k) / 12.0;
  return alpha / fpow * bracket;
}

// ---------------------------------------------------------------------------
// Black-76 (named for caplets and swaptions in Sec. 1 and in f_s, Sec. 3):
//   call = D [f N(d1) - K N(d2)], put = D [K N(-d2) - f N(-d1)],
//   d1,2 = (ln(f/K) +- sigma^2 T/2) / (sigma sqrt T), N(x) = erfc(-x/sqrt 2)/2.
// The out-of-the-money side is evaluated directly and the other side through
// put-call parity, call - put = D (f - K).
// ---------------------------------------------------------------------------
template <class S>
S norm_cdf(const S &x) { return 0.5 * erfc(-x / std::sqrt(2.0)); }

// Out-of-the-money side: the call when K >= f, else the put.
template <class S>
S black_otm(double f, double K, double T, const S &sigma, double D) {
  S sd = sigma * std::sqrt(T);
  S d1 = (log(f / K) + 0.5 * sigma * sigma * T) / sd;
  S d2 = d1 - sd;
  return (K >= f) ? D * (f * norm_cdf(d1) - K * norm_cdf(d2))
                  : D * (K * norm_cdf(-d2) - f * norm_cdf(-d1));
}

template <class S>
S black_price(int kind, double f, double K, double T, const S &sigma, double D) {
  S v = black_otm(f, K, T, sigma, D);
  const bool otm_call = K >= f;
  const bool want_call = (kind == 0);
  if (want_call == otm_call) return v;
  return want_call ? v + D * (f - K) : v + D * (K - f);
}

double black_vega(double f, double K, double T, double sigma, double D) {
  const double sd = sigma * std::sqrt(T);
  const double d1 = (std::log(f / K) + 0.5 * sigma * sigma * T) / sd;
  return D * f * std::exp(-0.5 * d1 * d1) / std::sqrt(2.0 * M_PI) * std::sqrt(T);
}

// ---------------------------------------------------------------------------
// Market data of one instance and the market-only quantities of each
// underlying: caplet on forward i = swap over the single period i.  For a
// swap over forwards k in [e, e+n): annuity A = sum tau_k P_k, weights
// w_k = tau_k P_k / A, swap rate S0 = sum w_k F_k, expiry T_e.
// ---------------------------------------------------------------------------
struct Fwd {
  double T, tau, F, P;
};
struct Und {
  int first, len;
  double A, S0, Te;
  std::vector<double> w;
};
struct Quote {
  int und, kind;
  double K, vol, w;
  double target, weight;  // market value of the quoted instrument, weight
  double target_otm;      // price mode: market price of the out-of-the-money side
};
struct Inst {
  int model, formula, residual;
  double beta;
  std::vector<Fwd> f;
  std::vector<Und> u;
  std::vector<Quote> q;
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int32_t build_inst(const oracle_market *m, int i, Inst &I) {
  if (!m) return fail("null market");
  if (i < 0 || i >= m->n_inst) return fail("instance index out of range");
  if (m->model < 0 || m->model > 4) return fail("unknown model");
  if (m->formula < 0 || m->formula > 1) return fail("unknown vol formula");
  if (m->residual < 0 || m->residual > 1) return fail("unknown residual mode");
  I.model = m->model;
  I.formula = m->formula;
  I.residual = m->residual;
  I.beta = m->beta;
  if (m->model != 0 && !(m->beta >= 0.0 && m->beta <= 1.0)) return fail("beta outside [0,1]");
  const int f0 = m->fwd_off[i], f1 = m->fwd_off[i + 1];
  const int u0 = m->und_off[i], u1 = m->und_off[i + 1];
  const int q0 = m->q_off[i], q1 = m->q_off[i + 1];
  if (f1 < f0 || u1 < u0 || q1 < q0) return fail("offsets not monotone");
  I.f.clear();
  I.u.clear();
  I.q.clear();
  for (int k = f0; k < f1; ++k) {
    Fwd F{m->fwd_T[k], m->fwd_tau[k], m->fwd_F[k], m->fwd_P[k]};
    if (!(std::isfinite(F.T) && F.T >= 0.0) || !finite_pos(F.tau) || !finite_pos(F.F) ||
        !finite_pos(F.P))
      return fail("bad forward data");
    I.f.push_back(F);
  }
  const int nf = f1 - f0;
  for (int k = u0; k < u1; ++k) {
    Und U;
    U.first = m->und_first[k];
    U.len = m->und_len[k];
    if (U.len < 1 || U.first < 0 || U.first + U.len > nf) return fail("bad underlying range");
    if (m->model != 1 && U.len != 1) return fail("only LMM12 markets hold swaptions");
    U.A = 0.0;
    for (int j = U.first; j < U.first + U.len; ++j) U.A += I.f[j].tau * I.f[j].P;
    U.S0 = 0.0;
    for (int j = U.first; j < U.first + U.len; ++j) {
      const double wk = I.f[j].tau * I.f[j].P / U.A;
      U.w.push_back(wk);
      U.S0 += wk * I.f[j].F;
    }
    U.Te = I.f[U.first].T;
    if (!(U.Te > 0.0)) return fail("underlying expiry must be positive");
    I.u.push_back(U);
  }
  const int nu = u1 - u0;
  int prev = 0;
  for (int k = q0; k < q1; ++k) {
    Quote Q;
    Q.und = m->q_und[k];
    Q.kind = m->q_kind[k];
    Q.K = m->q_K[k];
    Q.vol = m->q_vol[k];
    Q.w = m->q_w[k];
    if (Q.und < 0 || Q.und >= nu) return fail("quote underlying out of range");
    if (Q.und < prev) return fail("quotes not sorted by underlying");
    prev = Q.und;
    if (Q.kind != 0 && Q.kind != 1) return fail("bad quote kind");
    if (!finite_pos(Q.K) || !finite_pos(Q.vol) || !(std::isfinite(Q.w) && Q.w >= 0.0))
      return fail("bad quote data");
    const Und &U = I.u[Q.und];
    if (I.residual == 0) {
      Q.target = Q.vol;
      Q.weight = Q.w;
    } else {
      // Price residuals: market price from Black at the market vol; weight
      // divided by vega^2 so the cost is close to vol units.
      Q.target = black_price<double>(Q.kind, U.S0, Q.K, U.Te, Q.vol, U.A);
      Q.target_otm = black_otm<double>(U.S0, Q.K, U.Te, Q.vol, U.A);
      const double vg = black_vega(U.S0, Q.K, U.Te, Q.vol, U.A);
      if (!finite_pos(vg)) return fail("zero market vega");
      Q.weight = Q.w / (vg * vg);
    }
    I.q.push_back(Q);
  }
  return 0;
}

int num_params(int model) { return model == 0 ? 4 : (model == 1 ? 12 : -1); }

// Parameters per point of a market: 4 or 12; 3 per forward for PERFWD; 2
// per forward plus one for MM.  PERFWD and MM instances must all hold the
// same number of forwards; -1 otherwise.
int market_params(const oracle_market *m) {
  if (m->model < 2) return num_params(m->model);
  if (m->model > 4) return -1;
  if (m->n_inst < 1) return -1;
  const int nf = m->fwd_off[1] - m->fwd_off[0];
  for (int i = 1; i < m->n_inst; ++i)
    if (m->fwd_off[i + 1] - m->fwd_off[i] != nf) return -1;
  if (nf < 1) return -1;
  return m->model == 2 ? 3 * nf : (m->model == 3 ? 2 * nf + 1 : 2 * nf + 8);
}

// ---------------------------------------------------------------------------
// Helpers of the Rebonato map.
// Moments I_m(k, x) = int_0^x u^m e^{-k u} du, m = 0, 1, 2, k >= 0: the
// series x^{m+1} sum_j (-kx)^j / (j! (m + j + 1)) for kx < 1/2, else
//   I_0 = (1 - e)/k, I_1 = (1 - e (1 + z))/k^2, I_2 = 2 (1 - e (1 + z + z^2/2))/k^3,
// e = exp(-z), z = kx.
// ---------------------------------------------------------------------------
template <class S>
void exp_moments(const S &k, double x, S I[3]) {
  const S z = k * x;
  if (val(z) < 0.5) {
    S term(1.0), s0(0.0), s1(0.0), s2(0.0);
    for (int j = 0; j < 40; ++j) {
      s0 += term / double(j + 1);
      s1 += term / double(j + 2);
      s2 += term / double(j + 3);
      term = term * (-z) / double(j + 1);
    }
    I[0] = s0 * x;
    I[1] = s1 * (x * x);
    I[2] = s2 * (x * x * x);
  } else {
    const S e = exp(-z);
    I[0] = (1.0 - e) / k;
    I[1] = (1.0 - e * (1.0 + z)) / (k * k);
    I[2] = 2.0 * (1.0 - e * (1.0 + z + 0.5 * z * z)) / (k * k * k);
  }
}

// int_0^x ((a + b u) e^{-c u} + d)^2 du
template <class S>
S abcd_square_integral(const S &a, const S &b, const S &c, const S &d, double x) {
  S I2[3], I1[3];
  exp_moments(2.0 * c, x, I2);
  exp_moments(c, x, I1);
  return a * a * I2[0] + 2.0 * a * b * I2[1] + b * b * I2[2] +
         2.0 * d * (a * I1[0] + b * I1[1]) + d * d * x;
}

// Nodes and weights of the 64-point Gauss-Legendre rule on [-1, 1]: roots of
// P_64 by Newton's method from cos(pi (k - 1/4) / (64 + 1/2)), weights
// 2 / ((1 - x^2) P_64'(x)^2).
struct GaussLegendre64 {
  double x[64], w[64];
  GaussLegendre64() {
    const int n = 64;
    for (int k = 1; k <= n; ++k) {
      double t = std::cos(M_PI * (k - 0.25) / (n + 0.5)), dp = 0.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = t;   // P_0, P_1, then the three-term recurrence
        for (int j = 2; j <= n; ++j) {
          const double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (t * p1 - p0) / (t * t - 1.0);
        const double step = p1 / dp;
        t -= step;
        if (std::fabs(step) < 1e-16) break;
      }
      x[k - 1] = t;
      w[k - 1] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
  }
};
const GaussLegendre64 &gl64() {
  static const GaussLegendre64 g;
  return g;
}

// ---------------------------------------------------------------------------
// Parameter maps: model parameters -> SABR (alpha, beta, rho, nu) per
// underlying.
//  GLOBAL4: p = (alpha, beta, rho, nu) shared by every forward (the Hagan
//    model with common parameters; the paper's x = (phi_ii, sigma_i, alpha_i)
//    with phi_ii = rho, sigma_i = nu).
//  PERFWD: p = (alpha_1, rho_1, nu_1, ..., alpha_n, rho_n, nu_n), one
//    triple per forward, beta fixed: the Hagan model of Sec. 3 with its
//    per-forward parameters x = (phi_ii, sigma_i, alpha_i) (phi_ii = rho_i,
//    sigma_i = nu_i), the model calibrated to caplets in Sec. 4.1.1.  Every
//    triple must lie in the domain, quoted or not.
//  MM: p = (alpha_1, phi_1, ..., alpha_n, phi_n, sigma), beta fixed: the
//    Mercurio-Morini model of Sec. 2.2, x = (phi_i, sigma, alpha_i), with the
//    SABR parameters of eq. (haganForMercurio): beta_i = beta, rho_i =
//    phi_i, nu_i = sigma, alpha_i^SABR = alpha_i exp(int_0^{T_i} M_i(s) ds),
//    M_i(s) = -sigma sum_j tau_j phi_j alpha_j F_j^beta / (1 + tau_j F_j)
//    over the forwards j <= i of the drift sum at s.  The drift sum starts
//    at the forward after h(s) (reading: this reproduces the paper's
//    printed ATM levels), so forward j enters while s < T_{j-1}, the fixing
//    of the forward before it (0 for the first):
//      int_0^{T_i} M_i = -sigma sum_{j<=i} c_j T_{j-1},
//      c_j = tau_j phi_j alpha_j F_j^beta / (1 + tau_j F_j).
//    Every (alpha_j, phi_j) must lie in the domain (alpha > 0, |phi| < 1),
//    and sigma >= 0.
//  REB: p = (kappa_1, phi_1, ..., kappa_n, phi_n, a, b, c, d, a_h, b_h, c_h,
//    d_h), beta fixed: the Rebonato model of Sec. 2.2, x = (phi_ii, kappa_i,
//    the parameters of g and h), with the SABR parameters of eq.
//    (haganForRebonato) for the caplet on forward i (expiry T = T_i):
//      alpha_i = kappa_i sqrt(G / T),  G = int_0^T g_i(t)^2 dt,
//      nu_i = sqrt(2 J / (T G)),  J = int_0^T g_i(t)^2 H_i(t) dt,
//      H_i(t) = int_0^t h_i(s)^2 ds = t hhat_i(t)^2,  rho_i = phi_i,
//    g_i(t) = (a + b (T - t)) e^{-c (T - t)} + d and h_i likewise in the h
//    parameters.  With tau = T - t: G = Qg(T) and J = int_0^T g(tau)^2
//    (Qh(T) - Qh(tau)) dtau, Q(x) the closed-form square integral of the
//    abcd function over [0, x]; J by the 64-point Gauss-Legendre rule.
//    Domain: kappa_i > 0, |phi_i| < 1, c >= 0, c_h >= 0, G > 0.
//  LMM12: p = (a, b, c, d, a_n, b_n, c_n, d_n, rho, lambda1, eta2, lambda2),
//    beta fixed.  alpha_i = (a + b T_i) e^{-c T_i} + d and
//    nu_i = (a_n + b_n T_i) e^{-c_n T_i} + d_n are the abcd forms of Sec. 2.3
//    at t = 0; phi_ii = rho; rho_ij from eq. (rhoij) with eta1 = 0; theta_ij
//    from eq. (thetaij); phi_ij from eq. (phiij) with lambda3 = 0 (= rho).
//    A swap rate over several forwards gets SABR parameters from a
//    first-order freeze of dS = sum w_k dF_k at t = 0 with u_k = w_k F_k^beta:
//      V = sum_kl u_k u_l alpha_k alpha_l rho_kl,  alpha_S = sqrt(V)/S0^beta,
//      c_k = u_k alpha_k sum_l u_l alpha_l rho_kl / V,
//      nu_S^2 = sum_kl c_k c_l nu_k nu_l theta_kl,
//      rho_S = sum_kl (u_k alpha_k)(c_l nu_l) phi_kl / (alpha_S S0^beta nu_S).
// Returns false when the point is outside the model's domain.
// ---------------------------------------------------------------------------
template <class S>
struct Theta {
  S alpha, beta, rho, nu;
};

template <class S>
bool map_params(const Inst &I, const S *p, std::vector<Theta<S>> &th) {
  th.assign(I.u.size(), Theta<S>());
  if (I.model == 0) {
    const S &alpha = p[0], &beta = p[1], &rho = p[2], &nu = p[3];
    if (!(val(alpha) > 0.0) || !(val(beta) >= 0.0 && val(beta) <= 1.0) ||
        !(std::fabs(val(rho)) < 1.0) || !(val(nu) >= 0.0))
      return false;
    for (size_t u = 0; u < I.u.size(); ++u) th[u] = Theta<S>{alpha, beta, rho, nu};
    return true;
  }
  if (I.model == 4) {
    const size_t nf = I.f.size();
    const S *q = p + 2 * nf;   // a, b, c, d, a_h, b_h, c_h, d_h
    if (!(val(q[2]) >= 0.0) || !(val(q[6]) >= 0.0)) return false;
    for (size_t k = 0; k < nf; ++k)
      if (!(val(p[2 * k]) > 0.0) || !(std::fabs(val(p[2 * k + 1])) < 1.0)) return false;
    const GaussLegendre64 &gl = gl64();
    for (size_t u = 0; u < I.u.size(); ++u) {
      const int k = I.u[u].first;
      const double T = I.u[u].Te;
      const S G = abcd_square_integral(q[0], q[1], q[2], q[3], T);
      const S QT = abcd_square_integral(q[4], q[5], q[6], q[7], T);
      S J(0.0);
      for (int j = 0; j < 64; ++j) {
        const double tau = 0.5 * T * (1.0 + gl.x[j]);
        const S g = (q[0] + q[1] * tau) * exp(-(q[2] * tau)) + q[3];
        J += (0.5 * T * gl.w[j]) * (g * g) * (QT - abcd_square_integral(q[4], q[5], q[6], q[7], tau));
      }
      if (!(val(G) > 0.0) || !(val(J) >= 0.0)) return false;
      const S alpha = p[2 * k] * sqrt(G / T);
      const S nu = sqrt(2.0 * J / (T * G));
      th[u] = Theta<S>{alpha, S(I.beta), p[2 * k + 1], nu};
    }
    return true;
  }
  if (I.model == 3) {
    const size_t nf = I.f.size();
    const S &sigma = p[2 * nf];
    if (!(val(sigma) >= 0.0)) return false;
    for (size_t k = 0; k < nf; ++k)
      if (!(val(p[2 * k]) > 0.0) || !(std::fabs(val(p[2 * k + 1])) < 1.0)) return false;
    std::vector<S> aS(nf);
    S D(0.0);   // sum_{j<=k} c_j T_{j-1}
    for (size_t k = 0; k < nf; ++k) {
      const Fwd &F = I.f[k];
      const double Tprev = (k == 0) ? 0.0 : I.f[k - 1].T;
      const S c = F.tau * p[2 * k + 1] * p[2 * k] * std::pow(F.F, I.beta) / (1.0 + F.tau * F.F);
      D += c * Tprev;
      aS[k] = p[2 * k] * exp(-(sigma * D));
    }
    for (size_t u = 0; u < I.u.size(); ++u) {
      const int k = I.u[u].first;
      th[u] = Theta<S>{aS[k], S(I.beta), p[2 * k + 1], sigma};
    }
    return true;
  }
  if (I.model == 2) {
    for (size_t k = 0; k < I.f.size(); ++k)
      if (!(val(p[3 * k]) > 0.0) || !(std::fabs(val(p[3 * k + 1])) < 1.0) ||
          !(val(p[3 * k + 2]) >= 0.0))
        return false;
    for (size_t u = 0; u < I.u.size(); ++u) {
      const int k = I.u[u].first;
      th[u] = Theta<S>{p[3 * k], S(I.beta), p[3 * k + 1], p[3 * k + 2]};
    }
    return true;
  }
  const S &a = p[0], &b = p[1], &c = p[2], &d = p[3];
  const S &an = p[4], &bn = p[5], &cn = p[6], &dn = p[7];
  const S &rho = p[8], &lam1 = p[9], &eta2 = p[10], &lam2 = p[11];
  if (!(std::fabs(val(rho)) < 1.0) || !(val(lam1) >= 0.0) || !(val(lam2) >= 0.0) ||
      !(val(eta2) >= 0.0 && val(eta2) <= 1.0))
    return false;
  const S beta(I.beta);
  const size_t nf = I.f.size();
  std::vector<S> al(nf), nv(nf);
  for (size_t k = 0; k < nf; ++k) {
    const double T = I.f[k].T;
    al[k] = (a + b * T) * exp(-(c * T)) + d;
    nv[k] = (an + bn * T) * exp(-(cn * T)) + dn;
  }
  for (size_t ui = 0; ui < I.u.size(); ++ui) {
    const Und &U = I.u[ui];
    for (int k = U.first; k < U.first + U.len; ++k)
      if (!(val(al[k]) > 0.0) || !(val(nv[k]) >= 0.0)) return false;
    if (U.len == 1) {
      th[ui] = Theta<S>{al[U.first], beta, rho, nv[U.first]};
      continue;
    }
    const int n = U.len;
    std::vector<S> ua(n);  // u_k alpha_k
    for (int k = 0; k < n; ++k) {
      const Fwd &Fk = I.f[U.first + k];
      ua[k] = U.w[k] * std::pow(Fk.F, I.beta) * al[U.first + k];
    }
    std::vector<S> R(n, S(0.0));  // R_k = sum_l u_l alpha_l rho_kl
    for (int k = 0; k < n; ++k)
      for (int l = 0; l < n; ++l) {
        const double dT = std::fabs(I.f[U.first + k].T - I.f[U.first + l].T);
        R[k] += ua[l] * exp(-(lam1 * dT));
      }
    S V(0.0);
    for (int k = 0; k < n; ++k) V += ua[k] * R[k];
    if (!(val(V) > 0.0)) return false;
    const double S0b = std::pow(U.S0, I.beta);
    S alphaS = sqrt(V) / S0b;
    std::vector<S> cnu(n);  // c_k nu_k
    for (int k = 0; k < n; ++k) cnu[k] = ua[k] * R[k] / V * nv[U.first + k];
    S nu2(0.0);
    for (int k = 0; k < n; ++k)
      for (int l = 0; l < n; ++l) {
        const double dT = std::fabs(I.f[U.first + k].T - I.f[U.first + l].T);
        S theta = eta2 + (1.0 - eta2) * exp(-(lam2 * dT));
        nu2 += cnu[k] * cnu[l] * theta;
      }
    S nuS = sqrt(nu2);
    S rhoS(0.0);
    if (val(nuS) > 0.0) {
      S acc(0.0);
      for (int k = 0; k < n; ++k)
        for (int l = 0; l < n; ++l) acc += ua[k] * cnu[l] * rho;
      rhoS = acc / (alphaS * S0b * nuS);
    }
    if (!(std::fabs(val(rhoS)) < 1.0)) return false;
    th[ui] = Theta<S>{alphaS, beta, rhoS, nuS};
  }
  return true;
}

// Model value of every quote (vol or Black price of the quoted instrument)
// and its residual r_q = m_q - mkt_q; false on domain failure (model vol not
// finite and positive, or price not finite).  In price mode the residual is
// taken between the out-of-the-money sides: by put-call parity it equals the
// quoted side's difference exactly, without cancelling the intrinsic value.
template <class S>
bool model_values(const Inst &I, const S *p, std::vector<S> &mv, std::vector<S> &rv) {
  std::vector<Theta<S>> th;
  if (!map_params(I, p, th)) return false;
  mv.assign(I.q.size(), S(0.0));
  rv.assign(I.q.size(), S(0.0));
  for (size_t k = 0; k < I.q.size(); ++k) {
    const Quote &Q = I.q[k];
    const Und &U = I.u[Q.und];
    const Theta<S> &t = th[Q.und];
    S sig = (I.formula == 0) ? hagan2002_vol(U.S0, Q.K, U.Te, t.alpha, t.beta, t.rho, t.nu)
                             : paper_eq3_vol(U.S0, Q.K, t.alpha, t.beta, t.rho, t.nu);
    if (!(std::isfinite(val(sig)) && val(sig) > 0.0)) return false;
    if (I.residual == 0) {
      mv[k] = sig;
      rv[k] = sig - Q.target;
    } else {
      mv[k] = black_price(Q.kind, U.S0, Q.K, U.Te, sig, U.A);
      rv[k] = black_otm(U.S0, Q.K, U.Te, sig, U.A) - Q.target_otm;
    }
    if (!std::isfinite(val(mv[k])) || !std::isfinite(val(rv[k]))) return false;
  }
  return true;
}

// Cost f = sum_q w_q (m_q - mkt_q)^2 (f_c and f_s of Sec. 3 with weights);
// +inf on a domain failure or a non-finite sum.
template <class S>
S cost_point(const Inst &I, const S *p, double *resid) {
  std::vector<S> mv, rv;
  if (!model_values(I, p, mv, rv)) {
    if (resid)
      for (size_t k = 0; k < I.q.size(); ++k) resid[k] = std::nan("");
    return S(kInf);
  }
  S f(0.0);
  for (size_t k = 0; k < I.q.size(); ++k) {
    const S &r = rv[k];
    if (resid) resid[k] = val(r);
    f += I.q[k].weight * r * r;
  }
  if (!std::isfinite(val(f))) return S(kInf);
  return f;
}

double cost_d(const Inst &I, const double *p) { return cost_point<double>(I, p, nullptr); }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): 10 rounds of two 64x64->128 multiplies with the
// published multipliers and Weyl key increments.
// ---------------------------------------------------------------------------
void philox4x64_10(const uint64_t in[4], const uint64_t key_in[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c[4] = {in[0], in[1], in[2], in[3]};
  uint64_t k[2] = {key_in[0], key_in[1]};
  for (int r = 0; r < 10; ++r) {
    const unsigned __int128 p0 = (unsigned __int128)M0 * c[0];
    const unsigned __int128 p1 = (unsigned __int128)M1 * c[2];
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    const uint64_t n0 = hi1 ^ c[1] ^ k[0], n1 = lo1, n2 = hi0 ^ c[3] ^ k[1], n3 = lo0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
    k[0] += W0;
    k[1] += W1;
  }
  for (int j = 0; j < 4; ++j) out[j] = c[j];
}

// u_j, j = 0..P, for (instance, level, step, chain): words of consecutive
// Philox blocks b = 0, 1, ... at counter (l*N + s, chain, b, 0), key
// (seed, instance); u = (word >> 11) * 2^-53 in [0, 1).
void sa_uniforms(uint64_t seed, int inst, int l, int N, int s, int chain, int P, double *u) {
  const int nblk = (P + 1 + 3) / 4;
  for (int b = 0; b < nblk; ++b) {
    const uint64_t ctr[4] = {(uint64_t)l * (uint64_t)N + (uint64_t)s, (uint64_t)chain,
                             (uint64_t)b, 0};
    const uint64_t key[2] = {seed, (uint64_t)inst};
    uint64_t w[4];
    philox4x64_10(ctr, key, w);
    for (int j = 0; j < 4; ++j) {
      const int idx = 4 * b + j;
      if (idx <= P) u[idx] = (double)(w[j] >> 11) * 0x1.0p-53;
    }
  }
}

// Neighbour (the paper leaves ComputeNeighbour undefined; reading: every
// coordinate moves uniformly by at most step_frac (ub - lb), is mirrored
// back into the box, then clamped).
void propose(int P, const double *x, const double *u, const double *lb, const double *ub,
             double step_frac, double *xp) {
  for (int k = 0; k < P; ++k) {
    const double delta = step_frac * (ub[k] - lb[k]);
    double y = x[k] + delta * (2.0 * u[k] - 1.0);
    if (y > ub[k]) y = 2.0 * ub[k] - y;
    if (y < lb[k]) y = 2.0 * lb[k] - y;
    if (y > ub[k]) y = ub[k];
    if (y < lb[k]) y = lb[k];
    xp[k] = y;
  }
}

// Dense Cholesky solve of the (small) symmetric positive-definite system
// M x = rhs; false if M is not positive definite.
bool cholesky_solve(int P, std::vector<double> M, const double *rhs, double *x) {
  for (int j = 0; j < P; ++j) {
    double s = M[j * P + j];
    for (int k = 0; k < j; ++k) s -= M[j * P + k] * M[j * P + k];
    if (!(s > 0.0) || !std::isfinite(s)) return false;
    const double ljj = std::sqrt(s);
    M[j * P + j] = ljj;
    for (int i = j + 1; i < P; ++i) {
      double t = M[i * P + j];
      for (int k = 0; k < j; ++k) t -= M[i * P + k] * M[j * P + k];
      M[i * P + j] = t / ljj;
    }
  }
  std::vector<double> y(P);
  for (int i = 0; i < P; ++i) {
    double t = rhs[i];
    for (int k = 0; k < i; ++k) t -= M[i * P + k] * y[k];
    y[i] = t / M[i * P + i];
  }
  for (int i = P - 1; i >= 0; --i) {
    double t = y[i];
    for (int k = i + 1; k < P; ++k) t -= M[k * P + i] * x[k];
    x[i] = t / M[i * P + i];
  }
  return true;
}

// Residuals r_q = m_q - mkt_q, J_q = dm_q/dp and f; false on domain failure.
template <int P>
bool residual_jacobian(const Inst &I, const double *p, std::vector<double> &r,
                       std::vector<double> &J, double &f) {
  std::vector<Dual<P>> pd(P);
  for (int k = 0; k < P; ++k) {
    pd[k] = Dual<P>(p[k]);
    pd[k].d[k] = 1.0;
  }
  std::vector<Dual<P>> mv, rv;
  const size_t nq = I.q.size();
  r.assign(nq, 0.0);
  J.assign(nq * P, 0.0);
  if (!model_values(I, pd.data(), mv, rv)) return false;
  f = 0.0;
  for (size_t q = 0; q < nq; ++q) {
    r[q] = rv[q].v;
    for (int k = 0; k < P; ++k) J[q * P + k] = rv[q].d[k];
    f += I.q[q].weight * r[q] * r[q];
  }
  return std::isfinite(f);
}

template <int P>
void normal_equations(const Inst &I, const std::vector<double> &r, const std::vector<double> &J,
                      double *jtwj, double *jtwr) {
  for (int a = 0; a < P; ++a) {
    jtwr[a] = 0.0;
    for (int b = 0; b < P; ++b) jtwj[a * P + b] = 0.0;
  }
  for (size_t q = 0; q < I.q.size(); ++q) {
    const double w = I.q[q].weight;
    for (int a = 0; a < P; ++a) {
      jtwr[a] += w * J[q * P + a] * r[q];
      for (int b = 0; b < P; ++b) jtwj[a * P + b] += w * J[q * P + a] * J[q * P + b];
    }
  }
}

// Projected Levenberg-Marquardt (the gradient polish of the annealing's best
// points; the paper polishes with Nelder-Mead after SA, Sec. 3):
//   (J^T W J + mu diag(J^T W J)) delta = -J^T W r, trial = clamp(p + delta),
//   accept if f decreases (mu /= 10, stop when the relative decrease < tol),
//   else mu *= 10 (stop once mu > 1e16).  A zero diagonal entry is replaced by
//   1.  Coordinates that
//   are fixed (lb = ub) or sit on a bound the descent direction -J^T W r
//   points out of are frozen for the iteration (their row and column of the
//   system become the identity, their right-hand side 0).
template <int P>
void lm_one(const Inst &I, double *p, const double *lb, const double *ub, int max_iter,
            double mu0, double tol, double *f_out, int *it_out) {
  std::vector<double> r, J;
  double f;
  if (!residual_jacobian<P>(I, p, r, J, f)) {
    *f_out = kInf;
    *it_out = 0;
    return;
  }
  double mu = mu0;
  int it = 0;
  std::vector<double> A(P * P), g(P), M(P * P), delta(P), trial(P);
  for (; it < max_iter; ++it) {
    normal_equations<P>(I, r, J, A.data(), g.data());
    M = A;
    for (int k = 0; k < P; ++k) {
      const double dk = A[k * P + k] > 0.0 ? A[k * P + k] : 1.0;
      M[k * P + k] = A[k * P + k] + mu * dk;
    }
    std::vector<double> rhs(P);
    for (int k = 0; k < P; ++k) rhs[k] = -g[k];
    for (int k = 0; k < P; ++k) {
      const bool frozen = (lb[k] == ub[k]) || (p[k] <= lb[k] && g[k] > 0.0) ||
                          (p[k] >= ub[k] && g[k] < 0.0);
      if (!frozen) continue;
      for (int j = 0; j < P; ++j) M[k * P + j] = M[j * P + k] = 0.0;
      M[k * P + k] = 1.0;
      rhs[k] = 0.0;
    }
    if (!cholesky_solve(P, M, rhs.data(), delta.data())) {
      mu *= 10.0;
      continue;
    }
    for (int k = 0; k < P; ++k) {
      double y = p[k] + delta[k];
      if (y > ub[k]) y = ub[k];
      if (y < lb[k]) y = lb[k];
      trial[k] = y;
    }
    const double ft = cost_d(I, trial.data());
    if (ft < f) {
      const double rel = (f - ft) / f;
      for (int k = 0; k < P; ++k) p[k] = trial[k];
      double fnew;
      residual_jacobian<P>(I, p, r, J, fnew);
      f = ft;
      mu /= 10.0;
      if (rel < tol) {
        ++it;
        break;
      }
    } else {
      mu *= 10.0;
      if (mu > 1e16) {  // steps no longer change p: converged to rounding
        ++it;
        break;
      }
    }
  }
  *f_out = f;
  *it_out = it;
}

// ---------------------------------------------------------------------------
// Nelder-Mead polish of one point (the paper's local minimizer, Sec. 3, after
// the annealing), in the standard form with reflection 1, expansion 2,
// contraction 1/2 and shrink 1/2, every trial point clamped into the box.
// Initial simplex: x0 and x0 + d_k e_k, d_k = step (ub_k - lb_k) (x0 - d_k
// if that leaves the box).  Each iteration orders the vertices (best: lowest
// cost, lowest index on ties; worst: highest cost, highest index on ties;
// second worst likewise among the rest), stops when f_worst - f_best <=
// tol |f_best|, and otherwise
//   c = mean of the vertices other than the worst (summed in index order),
//   x_r = c + (c - x_w):  f_r < f_b      -> x_e = c + 2 (c - x_w), keep the
//                                           better of x_e and x_r;
//                         f_r < f_sw     -> keep x_r;
//                         f_r < f_w      -> x_c = c + (x_r - c)/2, keep it if
//                                           f_c <= f_r, else shrink;
//                         otherwise      -> x_c = c + (x_w - c)/2, keep it if
//                                           f_c < f_w, else shrink;
//   shrink: x_v <- x_b + (x_v - x_b)/2 for every v != b, re-evaluated.
// Returns the best vertex, its cost and the iterations taken.
// ---------------------------------------------------------------------------
void nm_one(const Inst &I, int P, double *p, const double *lb, const double *ub, int max_iter,
            double step, double tol, double *f_out, int *it_out) {
  std::vector<std::vector<double>> S(P + 1, std::vector<double>(p, p + P));
  std::vector<double> F(P + 1);
  for (int k = 0; k < P; ++k) {
    const double d = step * (ub[k] - lb[k]);
    S[k + 1][k] = (p[k] + d <= ub[k]) ? p[k] + d : p[k] - d;
  }
  auto clampk = [&](double y, int k) { return std::min(std::max(y, lb[k]), ub[k]); };
  for (int v = 0; v <= P; ++v) F[v] = cost_point<double>(I, S[v].data(), nullptr);
  std::vector<double> c(P), xr(P), xe(P), xc(P);
  int it = 0;
  while (it < max_iter) {
    int b = 0, w = 0;
    for (int v = 1; v <= P; ++v) {
      if (F[v] < F[b]) b = v;
      if (F[v] >= F[w]) w = v;
    }
    int sw = (w == 0) ? 1 : 0;
    for (int v = 0; v <= P; ++v)
      if (v != w && F[v] >= F[sw]) sw = v;
    if (F[w] - F[b] <= tol * std::fabs(F[b])) break;
    ++it;
    for (int k = 0; k < P; ++k) {
      double sum = 0.0;
      for (int v = 0; v <= P; ++v)
        if (v != w) sum += S[v][k];
      c[k] = sum / P;
    }
    for (int k = 0; k < P; ++k) xr[k] = clampk(c[k] + (c[k] - S[w][k]), k);
    const double fr = cost_point<double>(I, xr.data(), nullptr);
    bool shrink = false;
    if (fr < F[b]) {
      for (int k = 0; k < P; ++k) xe[k] = clampk(c[k] + 2.0 * (c[k] - S[w][k]), k);
      const double fe = cost_point<double>(I, xe.data(), nullptr);
      if (fe < fr) {
        S[w] = xe;
        F[w] = fe;
      } else {
        S[w] = xr;
        F[w] = fr;
      }
    } else if (fr < F[sw]) {
      S[w] = xr;
      F[w] = fr;
    } else if (fr < F[w]) {
      for (int k = 0; k < P; ++k) xc[k] = clampk(c[k] + 0.5 * (xr[k] - c[k]), k);
      const double fc = cost_point<double>(I, xc.data(), nullptr);
      if (fc <= fr) {
        S[w] = xc;
        F[w] = fc;
      } else {
        shrink = true;
      }
    } else {
      for (int k = 0; k < P; ++k) xc[k] = clampk(c[k] + 0.5 * (S[w][k] - c[k]), k);
      const double fc = cost_point<double>(I, xc.data(), nullptr);
      if (fc < F[w]) {
        S[w] = xc;
        F[w] = fc;
      } else {
        shrink = true;
      }
    }
    if (shrink) {
      for (int v = 0; v <= P; ++v) {
        if (v == b) continue;
        for (int k = 0; k < P; ++k) S[v][k] = S[b][k] + 0.5 * (S[v][k] - S[b][k]);
        F[v] = cost_point<double>(I, S[v].data(), nullptr);
      }
    }
  }
  int b = 0;
  for (int v = 1; v <= P; ++v)
    if (F[v] < F[b]) b = v;
  for (int k = 0; k < P; ++k) p[k] = S[b][k];
  *f_out = F[b];
  *it_out = it;
}

}  // namespace

// ===========================================================================
// Monte Carlo pricing under the Hagan SABR/LIBOR dynamics (Sec. 2.1: eqs.
// (dinamicasHagan1), (dinamicasHagan2), the spot-measure drifts with the
// first unfixed index h(t) of eq. (h_t), the bank-account numeraire, and the
// correlations of eqs. (rhoij), (thetaij), (phiij)); the pricer the paper
// nests in its swaption cost S_MC (Sec. 3) and times in Table
// (haganMCpricer).  The paper gives no discretisation; the readings below
// are this oracle's definition.
//
//  - Forwards k = 0..M-1: F_k fixes at T_k and accrues tau_k until the next
//    date; during [T_{j-1}, T_j) (T_{-1} = 0) the alive forwards are k >= j.
//  - Each interval [T_{j-1}, T_j) is cut into n_j = ceil(len / dt) (at least
//    one) equal steps of h = len / n_j; global step counter s = 0, 1, ...
//  - Step, for alive k with pre-step values:
//      s_k = V_k max(F_k, 0)^beta_k,  d_i = tau_i s_i / (1 + tau_i F_i),
//      F_k <- max(F_k + s_k h sum_{i=j..k} rho_{k,i} d_i + s_k x_k, 0),
//      V_k <- V_k exp((sigma_k sum_{i=j..k} phi_{i,k} d_i - sigma_k^2 / 2) h
//                     + sigma_k x_{M+k}),
//    with phi_{i,k} = E[dW_i dZ_k] (the covariance of Z_k with the
//    numeraire's drivers) and x = sqrt(h) B xi, B (2M x 2M, rows W_0..W_{M-1},
//    Z_0..Z_{M-1}) the correlation factor given by the caller, whose alive
//    rows vanish beyond column 2(M - j), xi the step's first 2(M - j)
//    standard normals (M - j pairs).
//  - Normals: pairs 2b and 2b + 1 of step s on path p are Box-Muller of the
//    Philox4x32-10 block (counter (b, s, p mod 2^32, p / 2^32), key (seed mod
//    2^32, seed / 2^32)): words (w0, w1) for pair 2b, (w2, w3) for pair
//    2b + 1, u1 = (w_first + 1) 2^-32, u2 = w_second 2^-32;  r = sqrt(-2 ln u1),
//    t = 2 pi u2, xi_{2m} = r cos t, xi_{2m+1} = r sin t.
//  - Deflator D = P(0, T_0) at t = 0, divided by (1 + tau_j F_j(T_j)) at each
//    fixing T_j after the payoffs expiring there are taken.
//  - Option (a, b, K): payer swaption expiring at T_a on forwards a..b-1
//    (b = a + 1: the caplet on F_a), value at T_a
//      max(1 - P(T_a, T_b) - K sum_{i=a}^{b-1} tau_i P(T_a, T_{i+1}), 0),
//    P(T_a, T_{i+1}) = prod_{l=a}^{i} 1 / (1 + tau_l F_l(T_a)); the path's
//    discounted payoff is D times that.
// ===========================================================================
namespace {

void philox4x32_10(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c[4] = {in[0], in[1], in[2], in[3]};
  uint32_t k[2] = {key_in[0], key_in[1]};
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k[0];
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
    k[0] += W0;
    k[1] += W1;
  }
  for (int j = 0; j < 4; ++j) out[j] = c[j];
}

void mc_normals(uint64_t seed, int64_t path, int64_t step, int M, double *xi) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4] = {0, 0, 0, 0};
  for (int m = 0; m < M; ++m) {
    if (m % 2 == 0) {
      const uint32_t ctr[4] = {(uint32_t)(m / 2), (uint32_t)step, (uint32_t)path,
                               (uint32_t)((uint64_t)path >> 32)};
      philox4x32_10(ctr, key, w);
    }
    const uint32_t wa = w[2 * (m % 2)], wb = w[2 * (m % 2) + 1];
    const double u1 = ((double)wa + 1.0) * 0x1.0p-32;
    const double u2 = (double)wb * 0x1.0p-32;
    const double r = std::sqrt(-2.0 * std::log(u1));
    const double t = 6.283185307179586 * u2;
    xi[2 * m] = r * std::cos(t);
    xi[2 * m + 1] = r * std::sin(t);
  }
}

int mc_steps(double len, double dt) {
  const double n = std::ceil(len / dt);
  return n < 1.0 ? 1 : (int)n;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *oracle_last_error(void) { return g_err.c_str(); }
int32_t oracle_num_params(int32_t model) { return num_params(model); }
int32_t oracle_market_num_params(const oracle_market *m) { return m ? market_params(m) : -1; }

void oracle_set_threads(int32_t n) {
  if (n > 0) omp_set_num_threads(n);
}

int32_t oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

double oracle_hagan2002_vol(double f, double K, double T, double alpha, double beta, double rho,
                            double nu) {
  return hagan2002_vol<double>(f, K, T, alpha, beta, rho, nu);
}
double oracle_paper_eq3_vol(double f, double K, double alpha, double beta, double rho,
                            double nu) {
  return paper_eq3_vol<double>(f, K, alpha, beta, rho, nu);
}
double oracle_chi(double z, double rho) { return chi<double>(z, rho); }
double oracle_black(int32_t kind, double f, double K, double T, double sigma, double D) {
  return black_price<double>(kind, f, K, T, sigma, D);
}
double oracle_black_vega(double f, double K, double T, double sigma, double D) {
  return black_vega(f, K, T, sigma, D);
}
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  philox4x64_10(ctr, key, out);
}
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox4x32_10(ctr, key, out);
}
void oracle_mc_normals(uint64_t seed, int64_t path, int64_t step, int32_t M, double *xi) {
  mc_normals(seed, path, step, M, xi);
}
int32_t oracle_mc_steps(double len, double dt) { return mc_steps(len, dt); }

int32_t oracle_mc_paths(int32_t M, const double *T, const double *tau, const double *F0,
                        const double *alpha, const double *beta, const double *phi,
                        const double *sigma, const double *y, double P0, const double *B,
                        int32_t n_opt, const int32_t *opt_a, const int32_t *opt_b,
                        const double *opt_K, int64_t path0, int64_t n_paths, double dt,
                        uint64_t seed, double *X) {
  if (M < 1) return fail("mc: need at least one forward");
  if (!(dt > 0.0)) return fail("mc: dt must be positive");
  if (n_paths < 0 || path0 < 0) return fail("mc: bad path range");
  int amax = -1;
  for (int o = 0; o < n_opt; ++o) {
    if (opt_a[o] < 0 || opt_b[o] <= opt_a[o] || opt_b[o] > M)
      return fail("mc: option " + std::to_string(o) + " needs 0 <= a < b <= M");
    if (opt_a[o] > amax) amax = opt_a[o];
  }
  const double eta1 = y[0], lam1 = y[1], lam3 = y[4];
  // rho_{k,i} (eq. rhoij) and phi_{i,k} = E[dW_i dZ_k] (eq. phiij)
  std::vector<double> rho((size_t)M * M), phw((size_t)M * M);
  for (int k = 0; k < M; ++k)
    for (int i = 0; i < M; ++i) {
      const double dT = std::fabs(T[k] - T[i]);
      rho[(size_t)k * M + i] = eta1 + (1.0 - eta1) * std::exp(-lam1 * dT);
      const double sg = phi[i] > 0.0 ? 1.0 : (phi[i] < 0.0 ? -1.0 : 0.0);
      phw[(size_t)i * M + k] = sg * std::sqrt(std::fabs(phi[i] * phi[k])) * std::exp(-lam3 * dT);
    }
  const int n2 = 2 * M;
#pragma omp parallel for schedule(static)
  for (int64_t pp = 0; pp < n_paths; ++pp) {
    const int64_t path = path0 + pp;
    std::vector<double> F(F0, F0 + M), V(alpha, alpha + M), Fn(M), Vn(M), s(M), d(M);
    std::vector<double> xi(n2), x(n2);
    double D = P0;
    int64_t step = 0;
    double *Xp = X + pp * n_opt;
    for (int j = 0; j <= amax; ++j) {
      const double len = T[j] - (j > 0 ? T[j - 1] : 0.0);
      const int n = mc_steps(len, dt);
      const double h = len / n, sh = std::sqrt(h);
      for (int st = 0; st < n; ++st, ++step) {
        // the alive forwards' increments take the step's first 2(M - j)
        // normals (the factor's columns beyond are zero on their rows)
        const int na = 2 * (M - j);
        mc_normals(seed, path, step, M - j, xi.data());
        for (int r = 0; r < n2; ++r) {
          double acc = 0.0;
          for (int c = 0; c < na; ++c) acc += B[(size_t)r * n2 + c] * xi[c];
          x[r] = sh * acc;
        }
        for (int k = j; k < M; ++k) {
          s[k] = V[k] * std::pow(std::fmax(F[k], 0.0), beta[k]);
          d[k] = tau[k] * s[k] / (1.0 + tau[k] * F[k]);
        }
        for (int k = j; k < M; ++k) {
          double sr = 0.0, sv = 0.0;
          for (int i = j; i <= k; ++i) {
            sr += rho[(size_t)k * M + i] * d[i];
            sv += phw[(size_t)i * M + k] * d[i];
          }
          Fn[k] = std::fmax(F[k] + s[k] * sr * h + s[k] * x[k], 0.0);
          Vn[k] = V[k] * std::exp((sigma[k] * sv - 0.5 * sigma[k] * sigma[k]) * h +
                                  sigma[k] * x[M + k]);
        }
        for (int k = j; k < M; ++k) {
          F[k] = Fn[k];
          V[k] = Vn[k];
        }
      }
      // fixing of F_j at T_j: payoffs expiring here, then the numeraire
      for (int o = 0; o < n_opt; ++o) {
        if (opt_a[o] != j) continue;
        double Pb = 1.0, A = 0.0;
        for (int i = j; i < opt_b[o]; ++i) {
          Pb /= (1.0 + tau[i] * F[i]);
          A += tau[i] * Pb;
        }
        Xp[o] = D * std::fmax(1.0 - Pb - opt_K[o] * A, 0.0);
      }
      D /= (1.0 + tau[j] * F[j]);
    }
  }
  return 0;
}

int32_t oracle_underlyings(const oracle_market *m, int32_t inst, double *S0, double *A,
                           double *T) {
  Inst I;
  if (build_inst(m, inst, I)) return -1;
  for (size_t u = 0; u < I.u.size(); ++u) {
    S0[u] = I.u[u].S0;
    A[u] = I.u[u].A;
    T[u] = I.u[u].Te;
  }
  return 0;
}

int32_t oracle_map_params(const oracle_market *m, int32_t inst, const double *p, double *out) {
  Inst I;
  if (build_inst(m, inst, I)) return -1;
  std::vector<Theta<double>> th;
  if (!map_params(I, p, th)) {
    for (size_t u = 0; u < I.u.size() * 4; ++u) out[u] = std::nan("");
    return 1;
  }
  for (size_t u = 0; u < th.size(); ++u) {
    out[4 * u + 0] = th[u].alpha;
    out[4 * u + 1] = th[u].beta;
    out[4 * u + 2] = th[u].rho;
    out[4 * u + 3] = th[u].nu;
  }
  return 0;
}

int32_t oracle_model_values(const oracle_market *m, int32_t inst, const double *p,
                            double *model, double *target, double *weight) {
  Inst I;
  if (build_inst(m, inst, I)) return -1;
  std::vector<double> mv, rv;
  const bool ok = model_values(I, p, mv, rv);
  for (size_t q = 0; q < I.q.size(); ++q) {
    if (model) model[q] = ok ? mv[q] : std::nan("");
    if (target) target[q] = I.q[q].target;
    if (weight) weight[q] = I.q[q].weight;
  }
  return ok ? 0 : 1;
}

int32_t oracle_cost_batch(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                          const double *params, double *cost, double *resid,
                          int32_t resid_stride) {
  if (!m) return fail("null market");
  std::vector<Inst> insts(m->n_inst);
  for (int i = 0; i < m->n_inst; ++i)
    if (build_inst(m, i, insts[i])) return -1;
  const int P = market_params(m);
  if (P < 0) return fail("unknown model or PERFWD instances of unequal size");
  for (int i = 0; i < n_pts; ++i)
    if (pt_inst[i] < 0 || pt_inst[i] >= m->n_inst) return fail("point instance out of range");
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < n_pts; ++i) {
    const Inst &I = insts[pt_inst[i]];
    cost[i] = cost_point<double>(I, params + (size_t)i * P,
                                 resid ? resid + (size_t)i * resid_stride : nullptr);
  }
  return 0;
}

int32_t oracle_cost_grad(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                         const double *params, double *cost, double *grad, double *jtwj,
                         double *jtwr) {
  if (!m) return fail("null market");
  std::vector<Inst> insts(m->n_inst);
  for (int i = 0; i < m->n_inst; ++i)
    if (build_inst(m, i, insts[i])) return -1;
  const int P = market_params(m);
  if (m->model >= 2 || P < 0) return fail("gradients and LM need GLOBAL4 or LMM12");
  for (int i = 0; i < n_pts; ++i)
    if (pt_inst[i] < 0 || pt_inst[i] >= m->n_inst) return fail("point instance out of range");
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < n_pts; ++i) {
    const Inst &I = insts[pt_inst[i]];
    const double *p = params + (size_t)i * P;
    if (P == 4) {
      Dual<4> pd[4];
      for (int k = 0; k < 4; ++k) {
        pd[k] = Dual<4>(p[k]);
        pd[k].d[k] = 1.0;
      }
      Dual<4> f = cost_point<Dual<4>>(I, pd, nullptr);
      cost[i] = f.v;
      for (int k = 0; k < 4; ++k) grad[(size_t)i * 4 + k] = std::isfinite(f.v) ? f.d[k] : 0.0;
      if (jtwj || jtwr) {
        std::vector<double> r, J, A(16), g(4);
        double ff;
        const bool ok = residual_jacobian<4>(I, p, r, J, ff);
        if (ok) normal_equations<4>(I, r, J, A.data(), g.data());
        for (int k = 0; k < 16; ++k)
          if (jtwj) jtwj[(size_t)i * 16 + k] = ok ? A[k] : 0.0;
        for (int k = 0; k < 4; ++k)
          if (jtwr) jtwr[(size_t)i * 4 + k] = ok ? g[k] : 0.0;
      }
    } else {
      Dual<12> pd[12];
      for (int k = 0; k < 12; ++k) {
        pd[k] = Dual<12>(p[k]);
        pd[k].d[k] = 1.0;
      }
      Dual<12> f = cost_point<Dual<12>>(I, pd, nullptr);
      cost[i] = f.v;
      for (int k = 0; k < 12; ++k)
        grad[(size_t)i * 12 + k] = std::isfinite(f.v) ? f.d[k] : 0.0;
      if (jtwj || jtwr) {
        std::vector<double> r, J, A(144), g(12);
        double ff;
        const bool ok = residual_jacobian<12>(I, p, r, J, ff);
        if (ok) normal_equations<12>(I, r, J, A.data(), g.data());
        for (int k = 0; k < 144; ++k)
          if (jtwj) jtwj[(size_t)i * 144 + k] = ok ? A[k] : 0.0;
        for (int k = 0; k < 12; ++k)
          if (jtwr) jtwr[(size_t)i * 12 + k] = ok ? g[k] : 0.0;
      }
    }
  }
  return 0;
}

// Mirrors of the library's cost entry points on host pointers (no stream,
// no workspace): sabr_cost_batch and sabr_cost_vjp, argument for argument.
int32_t oracle_sabr_cost_batch(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                               const double *params, double *cost, double *resid, double *model,
                               int32_t stride) {
  if (!m) return fail("null market");
  std::vector<Inst> insts(m->n_inst);
  for (int i = 0; i < m->n_inst; ++i)
    if (build_inst(m, i, insts[i])) return -1;
  const int P = market_params(m);
  if (P < 0) return fail("unknown model or PERFWD instances of unequal size");
  if ((resid || model) && stride < 1) return fail("stride below the quote count");
  for (int i = 0; i < m->n_inst; ++i)
    if ((resid || model) && (int)insts[i].q.size() > stride)
      return fail("stride below the quote count");
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < n_pts; ++i) {
    if (pt_inst[i] < 0 || pt_inst[i] >= m->n_inst) {   // out of range: NaN, as on the device
      cost[i] = std::nan("");
      continue;
    }
    const Inst &I = insts[pt_inst[i]];
    const double *p = params + (size_t)i * P;
    cost[i] = cost_point<double>(I, p, resid ? resid + (size_t)i * stride : nullptr);
    if (model) {
      std::vector<double> mv, rv;
      const bool ok = model_values(I, p, mv, rv);
      for (size_t q = 0; q < I.q.size(); ++q)
        model[(size_t)i * stride + q] = ok ? mv[q] : std::nan("");
    }
  }
  return 0;
}

int32_t oracle_sabr_cost_vjp(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                             const double *params, const double *g_cost, double *cost,
                             double *g_params, double *jtwj, double *jtwr) {
  if (!m) return fail("null market");
  const int P = market_params(m);
  if (m->model >= 2 || P < 0) return fail("gradients need GLOBAL4 or LMM12");
  std::vector<double> c((size_t)n_pts), g((size_t)n_pts * P);
  if (oracle_cost_grad(m, n_pts, pt_inst, params, c.data(), g.data(), jtwj, jtwr)) return -1;
  for (int i = 0; i < n_pts; ++i) {
    if (cost) cost[i] = c[i];
    const double s = g_cost ? g_cost[i] : 1.0;
    for (int k = 0; k < P; ++k) g_params[(size_t)i * P + k] = s * g[(size_t)i * P + k];
  }
  return 0;
}

// Synchronous parallel simulated annealing (Sec. 3: the boxed SA loop, run by
// many Markov chains; at the end of every temperature level all chains
// restart from the final point with the lowest cost).
// One chain's N Metropolis steps of level l at temperature T: proposal from
// the level's uniforms, cost, acceptance test, best-ever update.  x, F, bx,
// BF are the chain's state (updated); accept flags go to acc[s * stride].
// key: Philox key word 1 of the instance.  Per-step detail (nullable):
// proposal xp_out[s][P], its cost fp_out[s], acceptance uniform u_out[s].
// Returns the number of accepted proposals.
static int chain_level(const Inst &I, const oracle_sa_config &cfg, int key, int l, int c,
                       double T, int P, const double *lo, const double *hi, double *x, double &F,
                       double *bx, double &BF, uint8_t *acc, int64_t stride,
                       double *xp_out = nullptr, double *fp_out = nullptr,
                       double *u_out = nullptr) {
  const int N = cfg.n_steps;
  std::vector<double> u(P + 1), xp(P);
  int na = 0;
  for (int s = 0; s < N; ++s) {
    sa_uniforms(cfg.seed, key, l, N, s, c, P, u.data());
    propose(P, x, u.data(), lo, hi, cfg.step_frac, xp.data());
    double fp = cost_d(I, xp.data());
    if (std::isnan(fp)) fp = kInf;
    const double dE = fp - F;
    const bool a = (dE <= 0.0) || (u[P] < std::exp(-dE / T));
    if (xp_out)
      for (int k = 0; k < P; ++k) xp_out[(size_t)s * P + k] = xp[k];
    if (fp_out) fp_out[s] = fp;
    if (u_out) u_out[s] = u[P];
    if (a) {
      for (int k = 0; k < P; ++k) x[k] = xp[k];
      F = fp;
      ++na;
    }
    if (acc) acc[(int64_t)s * stride] = a ? 1 : 0;
    if (fp < BF) {
      BF = fp;
      for (int k = 0; k < P; ++k) bx[k] = xp[k];
    }
  }
  return na;
}

// Doubles of one instance's annealing state with C chains of P parameters:
// X [C][P], F [C], BX [C][P], BF [C], T.
static size_t state_doubles(int C, int P) { return 2 * (size_t)C * (P + 1) + 1; }

int32_t oracle_sa_calibrate(const oracle_market *m, const oracle_sa_config *cfg,
                            const int32_t *chains, const double *lb, const double *ub,
                            const double *x0, double *best_x, double *best_f,
                            double *chain_best_x, double *chain_best_f, uint8_t *accept,
                            double *level_trace, int32_t *level_best, int64_t *n_evals) {
  if (!m || !cfg) return fail("null argument");
  const int P = market_params(m);
  if (P < 0) return fail("unknown model or PERFWD instances of unequal size");
  if (cfg->n_levels < 0 || cfg->n_steps < 0) return fail("negative level or step count");
  if (!(cfg->cool > 0.0 && cfg->cool <= 1.0) || !(cfg->T0 > 0.0)) return fail("bad schedule");
  const int L = cfg->n_levels, N = cfg->n_steps;
  if (cfg->level0 < 0) return fail("negative first level");
  int64_t chain_base = 0, acc_base = 0;
  size_t state_off = 0;
  for (int i = 0; i < m->n_inst; ++i) {
    Inst I;
    if (build_inst(m, i, I)) return -1;
    const int C = chains[i];
    if (C < 1) return fail("need at least one chain per instance");
    const double *lo = lb + (size_t)i * P, *hi = ub + (size_t)i * P;
    for (int k = 0; k < P; ++k)
      if (!(lo[k] <= hi[k])) return fail("lb > ub");
    const int key = cfg->inst_key ? cfg->inst_key[i] : i;
    std::vector<double> X((size_t)C * P), F(C), BX((size_t)C * P), BF(C);
    double T;
    int64_t evals = 0;
    if (cfg->state_in) {
      // resume: the state a run of levels 0..level0-1 left
      const double *st = cfg->state_in + state_off;
      std::copy(st, st + (size_t)C * P, X.begin());
      std::copy(st + (size_t)C * P, st + (size_t)C * (P + 1), F.begin());
      std::copy(st + (size_t)C * (P + 1), st + (size_t)C * (2 * P + 1), BX.begin());
      std::copy(st + (size_t)C * (2 * P + 1), st + (size_t)C * (2 * P + 2), BF.begin());
      T = st[(size_t)C * (2 * P + 2)];
    } else {
      // 1. every chain starts at x0 (default: box midpoint) and evaluates it
      std::vector<double> start(P);
      for (int k = 0; k < P; ++k) start[k] = x0 ? x0[(size_t)i * P + k] : 0.5 * (lo[k] + hi[k]);
      for (int c = 0; c < C; ++c) {
        for (int k = 0; k < P; ++k) X[(size_t)c * P + k] = start[k];
        F[c] = cost_d(I, start.data());
        for (int k = 0; k < P; ++k) BX[(size_t)c * P + k] = start[k];
        BF[c] = F[c];
      }
      evals = C;
      T = (cfg->T0_per_inst ? cfg->T0_per_inst[i] : cfg->T0);
      for (int l = 0; l < cfg->level0; ++l) T = cfg->cool * T;
    }
    std::vector<int> nacc(C);
    for (int l = 0; l < L; ++l) {
      // 2. N Metropolis steps per chain at temperature T (chains independent)
      const int lg = cfg->level0 + l;
#pragma omp parallel for schedule(static)
      for (int c = 0; c < C; ++c)
        nacc[c] = chain_level(I, *cfg, key, lg, c, T, P, lo, hi, &X[(size_t)c * P], F[c],
                              &BX[(size_t)c * P], BF[c],
                              accept ? accept + acc_base + (int64_t)l * N * C + c : nullptr, C);
      evals += (int64_t)C * N;
      // 3. level end: restart every chain at the lowest final cost (ties ->
      //    lowest chain index); the restart point is copied, not re-evaluated
      int bstar = 0;
      for (int c = 1; c < C; ++c)
        if (F[c] < F[bstar]) bstar = c;
      for (int c = 0; c < C; ++c) {
        if (c == bstar) continue;
        for (int k = 0; k < P; ++k) X[(size_t)c * P + k] = X[(size_t)bstar * P + k];
        F[c] = F[bstar];
      }
      if (level_best) level_best[(size_t)i * L + l] = bstar;
      if (level_trace) {
        int gb = 0;
        for (int c = 1; c < C; ++c)
          if (BF[c] < BF[gb]) gb = c;
        int64_t tot = 0;
        for (int c = 0; c < C; ++c) tot += nacc[c];
        double *tr = level_trace + ((size_t)i * L + l) * 3;
        tr[0] = BF[gb];
        tr[1] = N > 0 ? (double)tot / ((double)C * N) : 0.0;
        tr[2] = 0.0;
      }
      T = cfg->cool * T;
    }
    // 4. best ever over all chains (ties -> lowest chain index)
    int gb = 0;
    for (int c = 1; c < C; ++c)
      if (BF[c] < BF[gb]) gb = c;
    for (int k = 0; k < P; ++k) best_x[(size_t)i * P + k] = BX[(size_t)gb * P + k];
    best_f[i] = BF[gb];
    if (chain_best_x)
      for (size_t k = 0; k < (size_t)C * P; ++k) chain_best_x[chain_base * P + k] = BX[k];
    if (chain_best_f)
      for (int c = 0; c < C; ++c) chain_best_f[chain_base + c] = BF[c];
    if (n_evals) n_evals[i] = evals;
    if (cfg->state_out) {
      double *st = cfg->state_out + state_off;
      std::copy(X.begin(), X.end(), st);
      std::copy(F.begin(), F.end(), st + (size_t)C * P);
      std::copy(BX.begin(), BX.end(), st + (size_t)C * (P + 1));
      std::copy(BF.begin(), BF.end(), st + (size_t)C * (2 * P + 1));
      st[(size_t)C * (2 * P + 2)] = T;
    }
    state_off += state_doubles(C, P);
    chain_base += C;
    acc_base += (int64_t)L * N * C;
  }
  return 0;
}

// Level 0 of the same annealing for a sample of chains (chains are
// independent until the first level end): chain sample_chain[j] of
// instance sample_inst[j] starts at x0 (default: box midpoint) and takes the
// level's N steps at T0.  Outputs per sample: accept [n][N], final cost F,
// best-ever cost BF and point BX [n][P].
int32_t oracle_sa_level0_sample(const oracle_market *m, const oracle_sa_config *cfg,
                                const int32_t *chains, const double *lb, const double *ub,
                                const double *x0, int32_t n_sample, const int32_t *sample_inst,
                                const int32_t *sample_chain, uint8_t *accept, double *F_out,
                                double *BF_out, double *BX_out) {
  if (!m || !cfg) return fail("null argument");
  const int P = market_params(m);
  if (P < 0) return fail("unknown model or PERFWD instances of unequal size");
  if (cfg->n_steps < 0) return fail("negative step count");
  if (!(cfg->T0 > 0.0)) return fail("bad schedule");
  const int N = cfg->n_steps;
  std::vector<Inst> insts(m->n_inst);
  std::vector<char> built(m->n_inst, 0);
  for (int j = 0; j < n_sample; ++j) {
    const int i = sample_inst[j];
    if (i < 0 || i >= m->n_inst) return fail("sample instance out of range");
    if (sample_chain[j] < 0 || sample_chain[j] >= chains[i]) return fail("sample chain out of range");
    if (!built[i]) {
      if (build_inst(m, i, insts[i])) return -1;
      built[i] = 1;
    }
  }
#pragma omp parallel for schedule(dynamic)
  for (int j = 0; j < n_sample; ++j) {
    const int i = sample_inst[j];
    const double *lo = lb + (size_t)i * P, *hi = ub + (size_t)i * P;
    std::vector<double> x(P);
    for (int k = 0; k < P; ++k) x[k] = x0 ? x0[(size_t)i * P + k] : 0.5 * (lo[k] + hi[k]);
    double F = cost_d(insts[i], x.data());
    double BF = F;
    double *bx = BX_out + (size_t)j * P;
    for (int k = 0; k < P; ++k) bx[k] = x[k];
    const double T = cfg->T0_per_inst ? cfg->T0_per_inst[i] : cfg->T0;
    chain_level(insts[i], *cfg, cfg->inst_key ? cfg->inst_key[i] : i, 0, sample_chain[j], T, P,
                lo, hi, x.data(), F, bx, BF, accept + (size_t)j * N, 1);
    F_out[j] = F;
    BF_out[j] = BF;
  }
  return 0;
}

// The N steps of one chain in one level, step by step: chain `chain` of
// instance `inst` at level `level` (Philox counter level N + s) and
// temperature T, from point x (cost f).  Outputs per step s: proposal
// xp_out[s][P], its cost fp_out[s], acceptance uniform u_out[s], accept flag
// acc_out[s].  For locating where two runs of the same annealing part.
int32_t oracle_sa_chain_steps(const oracle_market *m, const oracle_sa_config *cfg, int32_t inst,
                              int32_t chain, int32_t level, double T, const double *lb,
                              const double *ub, const double *x, double f, double *xp_out,
                              double *fp_out, double *u_out, uint8_t *acc_out) {
  if (!m || !cfg || !x || !lb || !ub) return fail("null argument");
  const int P = market_params(m);
  if (P < 0) return fail("unknown model or PERFWD instances of unequal size");
  if (inst < 0 || inst >= m->n_inst) return fail("instance out of range");
  if (cfg->n_steps < 0 || level < 0 || chain < 0) return fail("negative step, level or chain");
  Inst I;
  if (build_inst(m, inst, I)) return -1;
  std::vector<double> xc(x, x + P), bx(x, x + P);
  double F = f, BF = f;
  chain_level(I, *cfg, cfg->inst_key ? cfg->inst_key[inst] : inst, level, chain, T, P,
              lb + (size_t)inst * P, ub + (size_t)inst * P, xc.data(), F, bx.data(), BF, acc_out,
              1, xp_out, fp_out, u_out);
  return 0;
}

int32_t oracle_lm_polish(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                         double *params, const double *lb, const double *ub, int32_t max_iter,
                         double mu0, double tol, double *cost_out, int32_t *iters_out) {
  if (!m) return fail("null market");
  std::vector<Inst> insts(m->n_inst);
  for (int i = 0; i < m->n_inst; ++i)
    if (build_inst(m, i, insts[i])) return -1;
  const int P = market_params(m);
  if (m->model >= 2 || P < 0) return fail("gradients and LM need GLOBAL4 or LMM12");
  for (int i = 0; i < n_pts; ++i)
    if (pt_inst[i] < 0 || pt_inst[i] >= m->n_inst) return fail("point instance out of range");
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < n_pts; ++i) {
    const int inst = pt_inst[i];
    const Inst &I = insts[inst];
    double f;
    int it;
    if (P == 4)
      lm_one<4>(I, params + (size_t)i * 4, lb + (size_t)inst * 4, ub + (size_t)inst * 4,
                max_iter, mu0, tol, &f, &it);
    else
      lm_one<12>(I, params + (size_t)i * 12, lb + (size_t)inst * 12, ub + (size_t)inst * 12,
                 max_iter, mu0, tol, &f, &it);
    if (cost_out) cost_out[i] = f;
    if (iters_out) iters_out[i] = it;
  }
  return 0;
}

int32_t oracle_nm_polish(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                         double *params, const double *lb, const double *ub, int32_t max_iter,
                         double step, double tol, double *cost_out, int32_t *iters_out) {
  if (!m) return fail("null market");
  std::vector<Inst> insts(m->n_inst);
  for (int i = 0; i < m->n_inst; ++i)
    if (build_inst(m, i, insts[i])) return -1;
  const int P = market_params(m);
  if (P < 0) return fail("unknown model or PERFWD instances of unequal size");
  for (int i = 0; i < n_pts; ++i)
    if (pt_inst[i] < 0 || pt_inst[i] >= m->n_inst) return fail("point instance out of range");
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < n_pts; ++i) {
    const int inst = pt_inst[i];
    double f;
    int it;
    nm_one(insts[inst], P, params + (size_t)i * P, lb + (size_t)inst * P, ub + (size_t)inst * P,
           max_iter, step, tol, &f, &it);
    if (cost_out) cost_out[i] = f;
    if (iters_out) iters_out[i] = it;
  }
  return 0;
}

}  // extern "C"
