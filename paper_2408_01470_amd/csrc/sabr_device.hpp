// sabr_device.hpp -- device-side building blocks of the SA calibrator
// (gfx950, FP64 vector ALU).
//
// Market layout, Philox4x64-10, the Hagan 2002 lognormal implied vol, the
// paper's eq. (sigmaHagan), Black-76 and wavefront helpers.  Everything here
// is written for a 64-lane wavefront in which the lanes of one wave either
// share one parameter point (lanes over quotes) or hold one quote each.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sabr {

constexpr int kWave = 64;
constexpr double kInf = __builtin_huge_val();

// ---------------------------------------------------------------------------
// Packed market (device image).  All arrays are structure-of-arrays over the
// whole batch; per-instance ranges come from DevInst.  Indices stored in the
// arrays (underlying of a quote, first forward of an underlying) are local to
// their instance.
// ---------------------------------------------------------------------------
struct DevInst {
  int f0, nf;   // forward range
  int u0, nu;   // underlying range
  int q0, nq;   // quote range
  int maxlen;   // longest underlying (forwards per swap)
  int pad;
};

struct DevMarket {
  int n_inst, model, formula, residual;
  double beta;           // fixed beta (LMM12)
  int max_nq, max_nu, max_nf, max_len;
  const DevInst *inst;
  // forwards
  const double *f_T;     // fixing time T_k
  const double *f_v;     // tau_k P_k F_k^beta (fixed beta)
  // underlyings (caplet = one-period swap)
  const int *u_first, *u_len;
  const double *u_S0, *u_A, *u_invA, *u_S0b;  // swap rate, annuity, 1/A, S0^beta
  // quotes
  const int *q_und, *q_kind;
  const double *q_f, *q_K, *q_T, *q_sqrtT, *q_D;
  const double *q_L;      // ln(f/K)
  const double *q_lfk;    // ln(f K)
  const double *q_lnf;    // ln f
  const double *q_qfix;   // (f K)^((1-beta)/2), fixed beta
  const double *q_D1fix;  // 1 + (1-b)^2 L^2/24 + (1-b)^4 L^4/1920, fixed beta
  const double *q_fpfix;  // f^(1-beta), fixed beta
  const double *q_tgt;    // market vol or market Black price
  const double *q_w;      // weight (price mode: user weight / vega^2)
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC 2011).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__device__ __forceinline__ double u53(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

// ---------------------------------------------------------------------------
// Wavefront helpers.  Butterfly sums give bitwise-identical totals in every
// lane (each pairwise add is commutative).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Orders LDS traffic of one wavefront: a wave's LDS operations execute in
// issue order, so only the compiler must be kept from reordering them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// SABR constants of one (alpha, beta, rho, nu): everything in the Hagan
// formula that does not depend on the quote.
// ---------------------------------------------------------------------------
struct SabrConst {
  double alpha, rho, nua;   // nu / alpha
  double omb, omb2;         // 1 - beta, (1 - beta)^2
  double ca, cb, cc;        // corr q^2 = q^2 + (ca + cb q + cc q^2) T
  double s1, s2, s3, s4, s5;  // series of z / x(z) around z = 0
  double a_fp;              // alpha (eq3 scale numerator)
  double nu;
};

__device__ __forceinline__ SabrConst sabr_const(double alpha, double beta, double rho, double nu) {
  SabrConst k;
  k.alpha = alpha;
  k.rho = rho;
  k.nu = nu;
  k.nua = nu / alpha;
  k.omb = 1.0 - beta;
  k.omb2 = k.omb * k.omb;
  k.ca = k.omb2 * alpha * alpha * (1.0 / 24.0);
  k.cb = rho * beta * nu * alpha * 0.25;
  const double r2 = rho * rho;
  k.cc = (2.0 - 3.0 * r2) * nu * nu * (1.0 / 24.0);
  // z / x(z) = 1 + s1 z + ... + s5 z^5 + O(z^6)  (coefficients from the
  // Taylor expansion of x(z) = ln((sqrt(1 - 2 rho z + z^2) + z - rho)/(1 - rho)))
  k.s1 = -0.5 * rho;
  k.s2 = (2.0 - 3.0 * r2) * (1.0 / 12.0);
  k.s3 = -rho * (6.0 * r2 - 5.0) * (1.0 / 24.0);
  k.s4 = -((225.0 * r2 - 240.0) * r2 + 34.0) * (1.0 / 720.0);
  k.s5 = -rho * ((210.0 * r2 - 275.0) * r2 + 74.0) * (1.0 / 480.0);
  k.a_fp = alpha;
  return k;
}

constexpr double kZSeries = 0x1.0p-10;  // |z| below which z/x(z) uses the series

// Hagan 2002 lognormal vol given L = ln(f/K), q = (f K)^((1-beta)/2),
// D1 = 1 + (1-b)^2 L^2/24 + (1-b)^4 L^4/1920 and expiry T:
//   sigma = alpha chi(z) corr / (q D1),  corr q^2 = q^2 + (ca + cb q + cc q^2) T,
// evaluated as one division.  x(z) = log1p(t) with t = num/den chosen so that
// neither num nor den cancels:
//   |z| <= 1:  t = 2z / (s + 1 - z)
//   z  >  1:   t = (s + z - 1) / (1 - rho)
//   z  < -1:   t = (1 + z - s) / (s - z + rho),      s = sqrt(1 - 2 rho z + z^2);
// for |z| < 2^-10 the series of z/x(z) replaces the quotient (removable
// singularity at z = 0, truncation error below 1e-17).
__device__ __forceinline__ double hagan2002(const SabrConst &k, double L, double q, double D1,
                                            double T) {
  const double z = k.nua * q * L;
  const double s = sqrt(fma(z, z - 2.0 * k.rho, 1.0));
  const double az = fabs(z);
  const bool mid = az <= 1.0;
  const double num = mid ? 2.0 * z : (z > 0.0 ? (s + z) - 1.0 : (1.0 + z) - s);
  const double den = mid ? (s + 1.0) - z : (z > 0.0 ? 1.0 - k.rho : (s - z) + k.rho);
  const double x = log1p(num / den);
  const bool small = az < kZSeries;
  const double ser = fma(z, fma(z, fma(z, fma(z, fma(z, k.s5, k.s4), k.s3), k.s2), k.s1), 1.0);
  const double Pq = fma(q, q, T * fma(q, fma(q, k.cc, k.cb), k.ca));
  const double numer = k.alpha * Pq * (small ? ser : z);
  const double denom = q * q * q * D1 * (small ? 1.0 : x);
  return numer / denom;
}

__device__ __forceinline__ double d1_term(double omb2, double L) {
  const double u = omb2 * L * L;
  return fma(u, fma(u, 1.0 / 1920.0, 1.0 / 24.0), 1.0);
}

// Paper eq. (sigmaHagan): sigma = (alpha/f^(1-b)) [1 - (1/2)(1-b - rho nu w) k
//   + (1/12)((1-b)^2 + (2 - 3 rho^2) nu^2 w^2 + 3((1-b) - rho nu w)) k^2],
// w = f^(1-b)/alpha, k = ln(K/f) = -L, fp = f^(1-b).
__device__ __forceinline__ double paper_eq3(const SabrConst &k, double L, double fp) {
  const double w = fp / k.alpha;
  const double rnw = k.rho * k.nu * w;
  const double kk = -L;
  const double c1 = -0.5 * (k.omb - rnw);
  const double c2 = (k.omb2 + (2.0 - 3.0 * k.rho * k.rho) * k.nu * k.nu * w * w +
                     3.0 * (k.omb - rnw)) * (1.0 / 12.0);
  return k.alpha / fp * fma(kk, fma(kk, c2, c1), 1.0);
}

// ---------------------------------------------------------------------------
// Black-76.  The out-of-the-money side (call when K >= f, i.e. L <= 0) is
// evaluated directly, the other side through put-call parity.  Price
// residuals are taken between out-of-the-money sides (equal to the quoted
// side's difference by parity, without cancelling the intrinsic value).
//   call = D [f N(d1) - K N(d2)],  put = D [K N(-d2) - f N(-d1)],
//   d1 = L/(sigma sqrt T) + sigma sqrt T / 2,  N(x) = erfc(-x/sqrt 2)/2.
// ---------------------------------------------------------------------------
// Price of the out-of-the-money side (call when L <= 0).
__device__ __forceinline__ double black_otm(double f, double K, double L, double sqrtT,
                                            double sigma, double D) {
  const double sd = sigma * sqrtT;
  const double d1 = L / sd + 0.5 * sd;
  const double d2 = d1 - sd;
  const bool otm_call = L <= 0.0;
  const double sg = otm_call ? 1.0 : -1.0;  // N(sg d) with sg = -1 for the put
  const double n1 = 0.5 * erfc(-sg * d1 * M_SQRT1_2);
  const double n2 = 0.5 * erfc(-sg * d2 * M_SQRT1_2);
  return otm_call ? D * (f * n1 - K * n2) : D * (K * n2 - f * n1);
}

// Intrinsic value to add to the out-of-the-money price to get the quoted side.
__device__ __forceinline__ double parity_shift(int kind, double f, double K, double L, double D) {
  const bool otm_call = L <= 0.0;
  const bool want_call = (kind == 0);
  if (want_call == otm_call) return 0.0;
  return want_call ? D * (f - K) : D * (K - f);
}

__device__ __forceinline__ double black(int kind, double f, double K, double L, double sqrtT,
                                        double sigma, double D) {
  const double v = black_otm(f, K, L, sqrtT, sigma, D);
  const double sh = parity_shift(kind, f, K, L, D);
  return sh == 0.0 ? v : v + sh;
}

__device__ __forceinline__ double black_vega(double f, double L, double sqrtT, double sigma,
                                             double D) {
  const double sd = sigma * sqrtT;
  const double d1 = L / sd + 0.5 * sd;
  return D * f * exp(-0.5 * d1 * d1) * (0.39894228040143267794 * sqrtT);
}

}  // namespace sabr
