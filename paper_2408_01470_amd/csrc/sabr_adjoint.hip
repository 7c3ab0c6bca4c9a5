// sabr_adjoint.hip -- hand-written adjoint of the calibration cost and the
// Levenberg-Marquardt polish (gfx950).
//
// Per quote, a reverse sweep of the implied-vol formula and of Black-76
// gives dm/d(alpha, beta, rho, nu) of the quote's underlying.  For LMM12 the
// Jacobian M_u (3 x 12) of each underlying's SABR parameters (alpha_u, rho_u,
// nu_u) with respect to the model parameters comes from a reverse sweep of
// the parameter map, and J_q = dm_q/dp = M_u^T dm_q/dtheta_u.  With r_q the
// residual and w_q its weight:
//   d cost/dp = 2 sum_q w_q r_q J_q,  J^T W J = sum_q w_q J_q J_q^T,
//   J^T W r = sum_q w_q r_q J_q.
// One wavefront per point, lanes over quotes, per-lane accumulators reduced
// across the wave in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sabr_adjoint.hpp"
#include "sabr_cost.hpp"

namespace sabr {

namespace {

// sigma and d sigma/d(alpha, beta, rho, nu) of one quote (after quote_grad:
// the model value m and dm/d(...), with the vol kept in vol).
struct SigGrad {
  double sig, da, db, dr, dn, vol;
};

// Hagan 2002 (see hagan2002_frac) with its reverse sweep.  beta_param: q and
// D1 depend on beta through qa = ln(f K); otherwise qa = q, qb = D1 are fixed.
__device__ __forceinline__ SigGrad hagan2002_grad(double alpha, double beta, double rho,
                                                  double nu, double L, double T, double qa,
                                                  double qb, bool beta_param) {
  const double omb = 1.0 - beta;
  const double q = beta_param ? exp(0.5 * omb * qa) : qa;
  const double uL = omb * omb * L * L;
  const double D1 = beta_param ? fma(uL, fma(uL, 1.0 / 1920.0, 1.0 / 24.0), 1.0) : qb;
  const double nua = nu / alpha;
  const double z = nua * q * L;
  const double s = sqrt(fma(z, z - 2.0 * rho, 1.0));
  const double az = fabs(z);
  const bool mid = az <= 1.0;
  const double num = mid ? 2.0 * z : (z > 0.0 ? (s + z) - 1.0 : (1.0 + z) - s);
  const double den = mid ? (s + 1.0) - z : (z > 0.0 ? 1.0 - rho : (s - z) + rho);
  const double t = num / den;
  const double x = log1p(t);
  const double r2 = rho * rho;
  const double s2 = (2.0 - 3.0 * r2) * (1.0 / 12.0);
  const bool small = az < kZSeries;
  const double chi = small ? fma(z, fma(z, s2, -0.5 * rho), 1.0) : z / x;
  const double ca = omb * omb * alpha * alpha * (1.0 / 24.0);
  const double cb = rho * beta * nu * alpha * 0.25;
  const double cc = (2.0 - 3.0 * r2) * nu * nu * (1.0 / 24.0);
  const double Pq = fma(q, q, T * fma(q, fma(q, cc, cb), ca));
  const double sig = alpha * Pq * chi / (q * q * q * D1);
  // chi derivatives: five-term series near 0, else x_z = 1/s and the
  // rho-derivative of the log1p argument of the branch in use
  double chi_z, chi_r;
  if (az < 0x1.0p-10) {
    const double s3 = -rho * (6.0 * r2 - 5.0) * (1.0 / 24.0);
    const double s4 = -((225.0 * r2 - 240.0) * r2 + 34.0) * (1.0 / 720.0);
    const double s5 = -rho * ((210.0 * r2 - 275.0) * r2 + 74.0) * (1.0 / 480.0);
    chi_z = fma(z, fma(z, fma(z, fma(z, 5.0 * s5, 4.0 * s4), 3.0 * s3), 2.0 * s2), -0.5 * rho);
    const double d2 = -0.5 * rho;
    const double d3 = -(18.0 * r2 - 5.0) * (1.0 / 24.0);
    const double d4 = -(900.0 * r2 - 480.0) * rho * (1.0 / 720.0);
    const double d5 = -((1050.0 * r2 - 825.0) * r2 + 74.0) * (1.0 / 480.0);
    chi_r = z * fma(z, fma(z, fma(z, fma(z, d5, d4), d3), d2), -0.5);
  } else {
    const double zs = z / s;
    double x_r;
    if (mid)
      x_r = t * zs / (den * (1.0 + t));
    else if (z > 0.0)
      x_r = (t - zs) / (den * (1.0 + t));
    else
      x_r = (zs - t * (1.0 - zs)) / (den * (1.0 + t));
    const double ix2 = 1.0 / (x * x);
    chi_z = (x - zs) * ix2;
    chi_r = -z * x_r * ix2;
  }
  // reverse sweep with sigma-bar = 1
  const double a_direct = sig / alpha;
  const double Pb = sig / Pq;
  const double chib = sig / chi;
  double qb_ = -3.0 * sig / q;
  const double D1b = -sig / D1;
  qb_ += Pb * (2.0 * q + T * (cb + 2.0 * cc * q));
  const double cab = Pb * T, cbb = Pb * T * q, ccb = Pb * T * q * q;
  const double zb = chib * chi_z;
  double rb = chib * chi_r;
  const double nuab = zb * q * L;
  qb_ += zb * nua * L;
  double ab = a_direct + cab * omb * omb * alpha * (1.0 / 12.0) + cbb * rho * beta * nu * 0.25 -
              nuab * nu / (alpha * alpha);
  rb += cbb * beta * nu * alpha * 0.25 - ccb * rho * nu * nu * 0.25;
  const double nb = cbb * rho * beta * alpha * 0.25 + ccb * (2.0 - 3.0 * r2) * nu * (1.0 / 12.0) +
                    nuab / alpha;
  double ombb = cab * omb * alpha * alpha * (1.0 / 12.0);
  if (beta_param) {
    ombb += qb_ * 0.5 * qa * q;
    ombb += D1b * (1.0 / 12.0 + uL * (1.0 / 480.0)) * omb * L * L;
  }
  const double bb = cbb * rho * nu * alpha * 0.25 - ombb;
  return SigGrad{sig, ab, bb, rb, nb, sig};
}

// Paper eq. (sigmaHagan) with its derivatives; fp = f^(1-beta) (fixed beta)
// or qc = ln f (beta a parameter).
__device__ __forceinline__ SigGrad eq3_grad(double alpha, double beta, double rho, double nu,
                                            double L, double qc, bool beta_param) {
  const double omb = 1.0 - beta;
  const double lnf = qc;
  const double fp = beta_param ? exp(omb * lnf) : qc;
  const double w = fp / alpha;
  const double k = -L;
  const double rnw = rho * nu * w;
  const double g2 = 2.0 - 3.0 * rho * rho;
  const double c1 = -0.5 * (omb - rnw);
  const double c2 = (omb * omb + g2 * nu * nu * w * w + 3.0 * (omb - rnw)) * (1.0 / 12.0);
  const double B = fma(k, fma(k, c2, c1), 1.0);
  const double A = alpha / fp;
  const double sig = A * B;
  auto dB = [&](double c1d, double c2d) { return k * (c1d + k * c2d); };
  // alpha: w_a = -w/alpha
  const double wa = -w / alpha;
  const double da = B / fp + A * dB(0.5 * rho * nu * wa,
                                    (2.0 * g2 * nu * nu * w * wa - 3.0 * rho * nu * wa) / 12.0);
  const double dr = A * dB(0.5 * nu * w, (-6.0 * rho * nu * nu * w * w - 3.0 * nu * w) / 12.0);
  const double dn = A * dB(0.5 * rho * w, (2.0 * g2 * nu * w * w - 3.0 * rho * w) / 12.0);
  double db = 0.0;
  if (beta_param) {
    // omb_b = -1, fp_b = -fp ln f, w_b = -w ln f, A_b = A ln f
    const double wb = -w * lnf;
    const double c1b = -0.5 * (-1.0 - rho * nu * wb);
    const double c2b = (-2.0 * omb + 2.0 * g2 * nu * nu * w * wb + 3.0 * (-1.0 - rho * nu * wb)) /
                       12.0;
    db = A * lnf * B + A * dB(c1b, c2b);
  }
  return SigGrad{sig, da, db, dr, dn, sig};
}

// Model value m (vol, or out-of-the-money Black price) of one quote and
// dm/d(alpha, beta, rho, nu).
template <int FORMULA, int RESID>
__device__ __forceinline__ SigGrad quote_grad(double alpha, double beta, double rho, double nu,
                                              const QuoteRec &R, const UndMkt &U,
                                              bool beta_param) {
  SigGrad g = (FORMULA == 0)
                  ? hagan2002_grad(alpha, beta, rho, nu, R.L, U.T, R.qa, R.qb, beta_param)
                  : eq3_grad(alpha, beta, rho, nu, R.L, R.qc, beta_param);
  if (RESID == 1) {
    const double sig = g.sig;
    const double m = black_otm(U.f, R.K, R.L, U.sqrtT, U.isqrtT, sig, 1.0 / sig, U.D);
    // vega: D f phi(d1) sqrt(T), the same for both sides
    const double sd = sig * U.sqrtT;
    const double d1 = fma(R.L / sig, U.isqrtT, 0.5 * sd);
    const double vega = U.D * U.f * exp(-0.5 * d1 * d1) * (0.39894228040143267794 * U.sqrtT);
    g.sig = m;
    g.da *= vega;
    g.db *= vega;
    g.dr *= vega;
    g.dn *= vega;
  }
  return g;
}

// Accumulates the cost, gradient and (optionally) normal equations of one
// GLOBAL4 point over the wave's quotes (J_q = dm_q/d(alpha, beta, rho, nu)).
// Out-of-domain points give cost +inf and zero derivatives.  grad, jtwr: P
// values; jtwj: P(P+1)/2 (upper triangle).  (LMM12 takes lmm_normal and
// grad_kernel below: per-underlying seeds and sweeps of the map.)
template <int FORMULA, int RESID, bool NORMAL>
__device__ double point_normal(const DevMarket &m, const DevInst &in, const UndMkt *um,
                               const double *p, double *grad, double *jtwj, double *jtwr) {
  constexpr int P = 4;
  constexpr int NT = P * (P + 1) / 2;
  const int lane = lane_id();
  bool bad = !(p[0] > 0.0) || !(p[1] >= 0.0 && p[1] <= 1.0) || !(fabs(p[2]) < 1.0) ||
             !(p[3] >= 0.0);
  const double beta = p[1];
  double g[P], jr[P], jj[NORMAL ? NT : 1];
#pragma unroll
  for (int k = 0; k < P; ++k) g[k] = jr[k] = 0.0;
#pragma unroll
  for (int k = 0; k < (NORMAL ? NT : 1); ++k) jj[k] = 0.0;
  double acc = 0.0;
  for (int q = lane; q < in.nq; q += kWave) {
    const QuoteRec &R = m.q[in.q0 + q];
    const UndMkt U = um[R.und];
    const SigGrad sg = quote_grad<FORMULA, RESID>(p[0], beta, p[2], p[3], R, U, true);
    bad |= !(sg.vol > 0.0) || !(sg.vol < kInf) || !(fabs(sg.sig) < kInf);
    const double r = sg.sig - R.tgt;
    acc = fma(R.w * r, r, acc);
    const double J[P] = {sg.da, sg.db, sg.dr, sg.dn};
    const double wr = R.w * r;
#pragma unroll
    for (int k = 0; k < P; ++k) g[k] = fma(wr, J[k], g[k]);
    if (NORMAL) {
      int t = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const double wj = R.w * J[i];
#pragma unroll
        for (int j = i; j < P; ++j, ++t) jj[t] = fma(wj, J[j], jj[t]);
      }
    }
  }
  const double tot = wave_sum(acc);
  const bool any_bad = __any(bad) || !(tot < kInf);
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const double s = wave_sum(g[k]);
    grad[k] = any_bad ? 0.0 : 2.0 * s;
    jtwr[k] = any_bad ? 0.0 : s;
  }
  if (NORMAL) {
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const double s = wave_sum(jj[k]);
      jtwj[k] = any_bad ? 0.0 : s;
    }
  }
  return any_bad ? kInf : tot;
}

// sabr_cost_vjp on GLOBAL4 plans: one wave per point (grid-stride), the
// instance's market values in LDS.
template <int FORMULA, int RESID, bool NORMAL>
__global__ __launch_bounds__(64) void vjp_kernel(DevMarket m, int n_pts, const int *pt_inst,
                                                 const double *params, const double *g_cost,
                                                 double *cost, double *g_params, double *jtwj,
                                                 double *jtwr) {
  extern __shared__ double smem[];
  constexpr int P = 4;
  constexpr int NT = P * (P + 1) / 2;
  const int lane = lane_id();
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  for (int pt = blockIdx.x; pt < n_pts; pt += gridDim.x) {
    const int inst = __builtin_amdgcn_readfirstlane(pt_inst[pt]);
    if (inst < 0 || inst >= m.n_inst) {
      if (lane == 0 && cost) cost[pt] = __builtin_nan("");
      continue;
    }
    const DevInst in = m.inst[inst];
    wave_lds_sync();
    for (int u = lane; u < in.nu; u += kWave) um[u] = und_mkt(m, in.u0 + u);
    wave_lds_sync();
    double p[P];
#pragma unroll
    for (int k = 0; k < P; ++k) p[k] = params[(size_t)pt * P + k];
    double grad[P], jr[P], jj[NORMAL ? NT : 1];
    const double f = point_normal<FORMULA, RESID, NORMAL>(m, in, um, p, grad, jj, jr);
    if (lane == 0) {
      const double gc = g_cost ? g_cost[pt] : 1.0;
      if (cost) cost[pt] = f;
#pragma unroll
      for (int k = 0; k < P; ++k) g_params[(size_t)pt * P + k] = gc * grad[k];
      if (jtwr)
        for (int k = 0; k < P; ++k) jtwr[(size_t)pt * P + k] = jr[k];
      if (NORMAL && jtwj) {
        int t = 0;
        for (int i = 0; i < P; ++i)
          for (int j = i; j < P; ++j, ++t) {
            jtwj[((size_t)pt * P + i) * P + j] = jj[t];
            jtwj[((size_t)pt * P + j) * P + i] = jj[t];
          }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Gradient of the LMM12 cost without the map Jacobian.  With J_q = M_u^T s_q
// (s_q = dm_q/d(alpha_u, rho_u, nu_u) of the quote's underlying u):
//   sum_q w_q r_q J_q = sum_u M_u^T t_u,   t_u = sum_{q of u} w_q r_q s_q,
// and M_u^T t_u is one reverse sweep of u's map with the seed t_u.  Per chunk
// of kGradChunk underlyings (the map's order, quotes contiguous per
// underlying): the SABR constants into LDS, the quotes (lanes over quotes;
// each lane's w r s summed per underlying by a segmented scan across the
// wave, the segment ends adding into the chunk's t table in LDS), then one
// lane per underlying runs the reverse sweep into per-lane gradient
// accumulators.  Up to kGradWaves points per workgroup share one LDS copy of
// the per-underlying market values.
// ---------------------------------------------------------------------------
constexpr int kGradChunk = kWave;
constexpr int kGradWaves = 8;

// Per-forward values the reverse sweep needs besides the map's record:
// e^{-c T}, e^{-c_n T}, T and the frozen weight v = tau P F^beta.
struct FwdAux {
  double E, En, T, v;
};

// Black-76 out-of-the-money price (black_otm) and its vega D f phi(d1)
// sqrt(T), sharing the exponential.
__device__ __forceinline__ double black_otm_vega(double f, double K, double L, double sqrtT,
                                                 double isqrtT, double sigma, double isigma,
                                                 double D, double &vega) {
  const double sd = sigma * sqrtT;
  const double d1 = fma(L * isigma, isqrtT, 0.5 * sd);
  const double d2 = d1 - sd;
  double E, X1, X2;
  const double x1 = fabs(d1) * M_SQRT1_2;   // black_otm's arithmetic
  exp_erfcx2(-(x1 * x1), x1, fabs(d2) * M_SQRT1_2, E, X1, X2);
  const double hE = 0.5 * f * E;
  vega = D * f * E * (0.39894228040143267794 * sqrtT);
  if (L <= 0.0)
    return D * (d1 <= 0.0 ? hE * (X1 - X2) : fma(-hE, X1 + X2, f));
  return D * (d2 >= 0.0 ? hE * (X2 - X1) : fma(-hE, X1 + X2, K));
}

// Relative sensitivities of sigma for one quote (Hagan 2002, beta fixed:
// q = R.qa, q^3 D1 = R.qb), d sigma/d(alpha, rho, nu) = sigma (ra, rr, rn), with
// k the underlying's SABR constants:
//   sigma = alpha Pq chi / (q^3 D1),  Pq = q^2 + T (ca + cb q + cc q^2),
//   chi = z/x(z),  z = (nu/alpha) q L;
//   ra = [1 + T (2 ca + cb q)/Pq - z chi_z/chi] / alpha,
//   rr = T q nu (beta alpha - rho nu q)/(4 Pq) + chi_rho/chi,
//   rn = T q (rho beta alpha/4 + (2 - 3 rho^2) nu q/12)/Pq + (q L/alpha) chi_z/chi;
// chi_z and chi_rho by the log1p form, or by their series below |z| = 2^-10
// (as hagan2002_grad).  sigma itself comes from hagan2002_frac, as in the
// cost kernels (these lines repeat its intermediate values, which the
// compiler shares).
struct SigRatio {
  double ra, rr, rn;
};

__device__ __forceinline__ SigRatio hagan_ratios(const SabrConst &k, double beta, double L,
                                                 double q, double T) {
  const double al = k.alpha, rho = k.rho, nua = k.nua;
  const double z = nua * q * L;
  const double s = sqrt_gs(fma(z, z - 2.0 * rho, 1.0));
  const double az = fabs(z);
  const bool mid = az <= 1.0;
  const double num = mid ? 2.0 * z : (z > 0.0 ? (s + z) - 1.0 : (1.0 + z) - s);
  const double den = mid ? (s + 1.0) - z : (z > 0.0 ? 1.0 - rho : (s - z) + rho);
  const double t = num * rcp_nr(den);
  const double x = log1p_tang(t);
  const double ix = rcp_nr(x);
  const double r2 = rho * rho;
  const double s2 = fma(-0.25, r2, 1.0 / 6.0);   // (2 - 3 rho^2)/12
  const double chi = az < kZSeries ? fma(z, fma(z, s2, -0.5 * rho), 1.0) : z * ix;
  double chi_z, chi_r;
  if (az < 0x1.0p-10) {
    const double s3 = -rho * (6.0 * r2 - 5.0) * (1.0 / 24.0);
    const double s4 = -((225.0 * r2 - 240.0) * r2 + 34.0) * (1.0 / 720.0);
    const double s5 = -rho * ((210.0 * r2 - 275.0) * r2 + 74.0) * (1.0 / 480.0);
    chi_z = fma(z, fma(z, fma(z, fma(z, 5.0 * s5, 4.0 * s4), 3.0 * s3), 2.0 * s2), -0.5 * rho);
    const double d3 = -(18.0 * r2 - 5.0) * (1.0 / 24.0);
    const double d4 = -(900.0 * r2 - 480.0) * rho * (1.0 / 720.0);
    const double d5 = -((1050.0 * r2 - 825.0) * r2 + 74.0) * (1.0 / 480.0);
    chi_r = z * fma(z, fma(z, fma(z, fma(z, d5, d4), d3), -0.5 * rho), -0.5);
  } else {
    const double zs = z * rcp_nr(s);
    const double x_num = mid ? t * zs : (z > 0.0 ? t - zs : zs - t * (1.0 - zs));
    const double x_r = x_num * rcp_nr(den * (1.0 + t));
    const double ix2 = ix * ix;
    chi_z = (x - zs) * ix2;
    chi_r = -z * x_r * ix2;
  }
  const double Pq = fma(q, q, T * fma(q, fma(q, k.cc, k.cb), k.ca));
  const double iPq = rcp_nr(Pq);
  const double ichi = rcp_nr(chi);
  const double ia = rcp_nr(al);
  const double nu = nua * al;
  const double cz = chi_z * ichi;
  SigRatio o;
  o.ra = ia * (1.0 + T * fma(k.cb, q, 2.0 * k.ca) * iPq - z * cz);
  o.rr = fma(T * q * 0.25 * nu * fma(-rho * nu, q, beta * al), iPq, chi_r * ichi);
  o.rn = fma(T * q * fma(rho * beta * al, 0.25, (2.0 - 3.0 * r2) * nu * q * (1.0 / 12.0)), iPq,
             q * L * ia * cz);
  return o;
}

// Model value m of one LMM12 quote (vol, or the out-of-the-money Black price:
// the same operations as the cost kernels) and dm/d(alpha, rho, nu) of its
// underlying.
struct QuoteSens {
  double m, sa, sr, sn;
  bool bad;
};

template <int FORMULA, int RESID>
__device__ __forceinline__ QuoteSens quote_sens(const SabrConst &k, double beta,
                                                const QuoteRec &R, const UndMkt &U) {
  VolFrac vf;
  double da, dr, dn;   // d sigma/d(alpha, rho, nu)
  if (FORMULA == 0) {
    vf = hagan2002_frac(k, R.L, R.qa, R.qb, U.T);
  } else {   // eq. (sigmaHagan), beta fixed: the quadratic in k = -L itself
    vf.numer = fma(-R.L, fma(-R.L, k.cc, k.cb), k.ca);
    vf.denom = 1.0;
  }
  QuoteSens o;
  double sig, sc = 1.0;
  if (RESID == 0) {
    sig = FORMULA == 1 ? vf.numer : vf.numer * rcp_nr(vf.denom);
    o.m = sig;
    o.bad = !(sig > 0.0) || !(sig < kInf);
  } else {
    const double rr = rcp_nr(vf.numer * vf.denom);
    sig = FORMULA == 1 ? vf.numer : vf.numer * (vf.numer * rr);
    const double isig = FORMULA == 1 ? rr : vf.denom * (vf.denom * rr);
    o.m = black_otm_vega(U.f, R.K, R.L, U.sqrtT, U.isqrtT, sig, isig, U.D, sc);
    o.bad = !(sig > 0.0) || !(sig < kInf) || !(fabs(o.m) < kInf);
  }
  if (FORMULA == 0) {
    const SigRatio h = hagan_ratios(k, beta, R.L, R.qa, U.T);
    const double ss = sig * sc;
    da = ss * h.ra;
    dr = ss * h.rr;
    dn = ss * h.rn;
  } else {
    const SigGrad e3 = eq3_grad(k.alpha, beta, k.rho, k.nua * k.alpha, R.L, U.fp, false);
    da = sc * e3.da;
    dr = sc * e3.dr;
    dn = sc * e3.dn;
  }
  o.sa = da;
  o.sr = dr;
  o.sn = dn;
  return o;
}

// Register or LDS storage of the two per-lane columns of the reverse sweep.
template <int NMAX>
struct SweepCols {
  double c1[NMAX], c2[NMAX];
  __device__ __forceinline__ double &a(int j) { return c1[j]; }
  __device__ __forceinline__ double &b(int j) { return c2[j]; }
};
template <>
struct SweepCols<0> {
  double *c1, *c2;   // stride kWave
  __device__ __forceinline__ double &a(int j) { return c1[j * kWave]; }
  __device__ __forceinline__ double &b(int j) { return c2[j * kWave]; }
};

// g += M_u^T (tA, tR, tN) for the swap of forwards [e, e + n) (n >= 2): the
// frozen-weight map forward (a_j = v_j alpha_j, R_j = sum_l a_l rho_jl,
// V = sum a_j R_j, s_a = sum a_j, b_j = a_j R_j nu_j, S_b = sum b_j,
// Be_j = sum_l b_l e_jl, Nb = eta2 S_b^2 + (1 - eta2) sum_j b_j Be_j,
// alpha_S = c0 sqrt V, nu_S = sqrt(Nb)/V, rho_S = rho s_a S_b/sqrt(V Nb)),
// then its reverse sweep with that seed.  Pair sums with an exp(-lambda |dT|)
// kernel are left plus right recursions over the gap factors; |dT|-weighted
// pair sums (the lambda derivatives) take the time-weighted left sums.
// Columns: c1 holds the left a sums, then R_j, then the a-bar terms the
// last pass completes; c2 the right b sums, then Be_j, then b-bar_j.
template <int NMAX>
__device__ __forceinline__ void swap_vjp(const FwdMap *fw, const FwdAux *fx, int n, double c0,
                                         const double *p, double tA, double tR, double tN,
                                         SweepCols<NMAX> &col, double *g) {
  constexpr bool REG = NMAX > 0;
  const int J = REG ? NMAX : n;
  const double rho = p[8], eta2 = p[10];
  double La = 0.0, sa = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (REG && j >= n) continue;
    col.a(j) = La;
    sa += fw[j].a;
    La = fw[j].g1 * (La + fw[j].a);
  }
  double Ra = 0.0, Rb = 0.0, V = 0.0, Sb = 0.0;
#pragma unroll
  for (int j = J - 1; j >= 0; --j) {
    if (REG && j >= n) continue;
    const FwdMap F = fw[j];
    const double Rj = col.a(j) + F.a + Ra;
    col.a(j) = Rj;
    V = fma(F.a, Rj, V);
    const double bj = F.a * Rj * F.nv;
    Sb += bj;
    col.b(j) = Rb;
    if (j > 0) {
      Ra = fw[j - 1].g1 * (Ra + F.a);
      Rb = fw[j - 1].g2 * (Rb + bj);
    }
  }
  double Lb = 0.0, LbT = 0.0, bBe = 0.0, lam2h = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (REG && j >= n) continue;
    const FwdMap F = fw[j];
    const double T = fx[j].T;
    const double bj = F.a * col.a(j) * F.nv;
    const double Be = Lb + bj + col.b(j);
    col.b(j) = Be;
    bBe = fma(bj, Be, bBe);
    lam2h = fma(bj, fma(T, Lb, -LbT), lam2h);
    Lb = F.g2 * (Lb + bj);
    LbT = F.g2 * fma(bj, T, LbT);
  }
  const double Nb = fma(eta2 * Sb, Sb, (1.0 - eta2) * bBe);
  const double sV = sqrt_gs(V), sN = sqrt_gs(Nb);
  double Vb = tA * c0 * 0.5 * rcp_nr(sV);
  double Nbb = 0.0, sab = 0.0, Sbb = 0.0;
  if (sN > 0.0) {
    const double iV = rcp_nr(V), inv = rcp_nr(sV * sN);
    const double rhoS = rho * sa * Sb * inv;
    Vb -= iV * fma(tN * sN, iV, 0.5 * tR * rhoS);
    Nbb = 0.5 * fma(tN, inv * sV * iV, -tR * rhoS * rcp_nr(Nb));
    sab = tR * rho * Sb * inv;
    Sbb = tR * rho * sa * inv;
    g[8] = fma(tR, sa * Sb * inv, g[8]);
  }
  g[10] = fma(Nbb, fma(Sb, Sb, -bBe), g[10]);
  g[11] = fma(-2.0 * Nbb * (1.0 - eta2), lam2h, g[11]);
  const double an = p[4], bn = p[5];
  double RR = 0.0;
#pragma unroll
  for (int j = J - 1; j >= 0; --j) {
    if (REG && j >= n) continue;
    const FwdMap F = fw[j];
    const FwdAux X = fx[j];
    const double bb = fma(2.0 * Nbb, fma(eta2, Sb, (1.0 - eta2) * col.b(j)), Sbb);
    const double Rj = col.a(j);
    const double Rbar = F.a * fma(bb, F.nv, Vb);
    const double nub = bb * F.a * Rj;
    g[4] = fma(nub, X.En, g[4]);
    g[5] = fma(nub * X.T, X.En, g[5]);
    g[6] = fma(-nub * X.T * fma(bn, X.T, an), X.En, g[6]);
    g[7] += nub;
    col.a(j) = fma(fma(bb, F.nv, Vb), Rj, sab) + (Rbar + RR);
    col.b(j) = bb;
    if (j > 0) RR = fw[j - 1].g1 * (RR + Rbar);
  }
  const double a = p[0], b = p[1];
  double LR = 0.0, LRT = 0.0, Lx = 0.0, LxT = 0.0, l1 = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (REG && j >= n) continue;
    const FwdMap F = fw[j];
    const FwdAux X = fx[j];
    const double Rbar = F.a * fma(col.b(j), F.nv, Vb);
    const double alb = (col.a(j) + LR) * X.v;
    g[0] = fma(alb, X.E, g[0]);
    g[1] = fma(alb * X.T, X.E, g[1]);
    g[2] = fma(-alb * X.T * fma(b, X.T, a), X.E, g[2]);
    g[3] += alb;
    l1 -= fma(Rbar, fma(X.T, Lx, -LxT), F.a * fma(X.T, LR, -LRT));
    LR = F.g1 * (LR + Rbar);
    LRT = F.g1 * fma(Rbar, X.T, LRT);
    Lx = F.g1 * (Lx + F.a);
    LxT = F.g1 * fma(F.a, X.T, LxT);
  }
  g[9] += l1;
}

// The wave's LDS of the gradient kernel: the map's forward records and the
// sweep's per-forward values, the chunk's SABR constants and t table, and
// (swaps longer than 24 forwards) the sweep's two per-lane columns.
__host__ __device__ inline int grad_wave_doubles(const DevMarket &m) {
  return kFwdMapDoubles * m.max_nf + 4 * m.max_nf + (kSabrConstDoubles + 3) * kGradChunk +
         (m.max_len > 24 ? 2 * kWave * m.max_len : 0);
}

// Segmented inclusive sum over the wave's lanes: segments are runs of equal
// key (heads: bit l set where lane l starts a run); afterwards the last lane
// of each run holds the run's sum.
__device__ __forceinline__ double seg_scan(double v, int lane, int start) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double w = __shfl_up(v, o, kWave);
    if (lane - o >= start) v += w;
  }
  return v;
}

template <int FORMULA, int RESID, int REG>
__global__ __launch_bounds__(kWave *kGradWaves) void grad_kernel(DevMarket m, int n_pts,
                                                                 const int *pt_inst,
                                                                 const double *params,
                                                                 const double *g_cost,
                                                                 double *cost, double *g_params,
                                                                 double *jtwr, int lds_per_wave) {
  extern __shared__ double smem[];
  __shared__ int s_inst[kGradWaves];
  constexpr int P = 12;
  const int nw = blockDim.x / kWave;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = lane_id();
  const int pt = blockIdx.x * nw + wid;
  int inst = -1;
  if (pt < n_pts) inst = __builtin_amdgcn_readfirstlane(pt_inst[pt]);
  const bool valid = pt < n_pts && inst >= 0 && inst < m.n_inst;
  if (pt < n_pts && !valid && lane == 0 && cost) cost[pt] = __builtin_nan("");
  if (lane == 0) s_inst[wid] = valid ? inst : -1;
  __syncthreads();
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  double *wb = smem + 6 * m.max_nu + (size_t)wid * lds_per_wave;
  WaveLds w;
  w.fw = reinterpret_cast<FwdMap *>(wb);
  FwdAux *fx = reinterpret_cast<FwdAux *>(wb + kFwdMapDoubles * m.max_nf);
  w.th = reinterpret_cast<SabrConst *>(wb + (kFwdMapDoubles + 4) * m.max_nf);
  double *tt = wb + (kFwdMapDoubles + 4) * m.max_nf + kSabrConstDoubles * kGradChunk;
  w.lk = tt + 3 * kGradChunk;   // the map's LDS column (swaps beyond 24 forwards)
  for (int r = 0; r < nw; ++r) {   // one round per distinct instance (see cost_kernel)
    const int ri = s_inst[r];
    bool first = ri >= 0;
    for (int q = 0; q < r; ++q) first = first && s_inst[q] != ri;
    if (!first) continue;
    const DevInst rin = m.inst[ri];
    for (int u = threadIdx.x; u < rin.nu; u += blockDim.x) um[u] = und_mkt(m, rin.u0 + u);
    __syncthreads();
    if (valid && inst == ri) {
      const DevInst in = m.inst[inst];
      double p[P];
#pragma unroll
      for (int k = 0; k < P; ++k) p[k] = params[(size_t)pt * P + k];
      bool bad = lmm12_fwd(m, in, p, w);
      for (int k = lane; k < in.nf; k += kWave) {
        const double T = m.f_T[in.f0 + k];
        fx[k] = FwdAux{exp_neg(-(p[2] * T)), exp_neg(-(p[6] * T)), T, m.f_v[in.f0 + k]};
      }
      wave_lds_sync();
      double g[P];
#pragma unroll
      for (int k = 0; k < P; ++k) g[k] = 0.0;
      double acc = 0.0;
      const int *uq0 = m.u_q0 + in.u0;
      const UndMap *umap = m.u_map + in.u0;
      const QuoteRec *qrec = m.q + in.q0;
      const double beta = m.beta;
      for (int c0 = 0; c0 < in.nu; c0 += kGradChunk) {
        const int c1 = min(in.nu, c0 + kGradChunk);
        bad |= lmm12_und<FORMULA, (REG > 0 ? REG : kMapRegLen)>(m, in, um, p, w, c0, c1);
        for (int k = lane; k < 3 * kGradChunk; k += kWave) tt[k] = 0.0;
        wave_lds_sync();
        const int qa = uq0[c0], qb = c1 < in.nu ? uq0[c1] : in.nq;
        for (int q0 = qa; q0 < qb; q0 += kWave) {   // wave-uniform trip count
          const int q = q0 + lane;
          int key = -1 - lane;                        // no quote: a run of its own
          double v0 = 0.0, v1 = 0.0, v2 = 0.0;
          if (q < qb) {
            const QuoteRec R = qrec[q];
            const UndMkt U = um[R.und];
            const SabrConst k = w.th[R.und - c0];
            key = R.und;
            const QuoteSens qs = quote_sens<FORMULA, RESID>(k, beta, R, U);
            bad |= qs.bad;
            const double r = qs.m - R.tgt;
            acc = fma(R.w * r, r, acc);
            const double wr = R.w * r;
            v0 = wr * qs.sa;
            v1 = wr * qs.sr;
            v2 = wr * qs.sn;
          }
          const int prev = __shfl_up(key, 1, kWave);
          const unsigned long long heads = __ballot(lane == 0 || prev != key);
          const unsigned long long upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
          const int start = kWave - 1 - __clzll(heads & upto);
          v0 = seg_scan(v0, lane, start);
          v1 = seg_scan(v1, lane, start);
          v2 = seg_scan(v2, lane, start);
          const bool tail = key >= 0 && (lane == kWave - 1 || ((heads >> (lane + 1)) & 1));
          if (tail) {
            double *t = tt + 3 * (key - c0);
            t[0] += v0;
            t[1] += v1;
            t[2] += v2;
          }
        }
        wave_lds_sync();
        const int i = c0 + lane;   // one underlying per lane (kGradChunk = kWave)
        if (i < c1) {
          const UndMap un = umap[i];
          const double tA = tt[3 * lane], tR = tt[3 * lane + 1], tN = tt[3 * lane + 2];
          if (un.n == 1) {
            const FwdAux X = fx[un.e];
            g[0] = fma(tA, X.E, g[0]);
            g[1] = fma(tA * X.T, X.E, g[1]);
            g[2] = fma(-tA * X.T * fma(p[1], X.T, p[0]), X.E, g[2]);
            g[3] += tA;
            g[4] = fma(tN, X.En, g[4]);
            g[5] = fma(tN * X.T, X.En, g[5]);
            g[6] = fma(-tN * X.T * fma(p[5], X.T, p[4]), X.En, g[6]);
            g[7] += tN;
            g[8] += tR;
          } else {
            SweepCols<REG> col;
            if constexpr (REG == 0) {
              col.c1 = w.lk + lane;
              col.c2 = w.lk + (size_t)m.max_len * kWave + lane;
            }
            swap_vjp<REG>(w.fw + un.e, fx + un.e, un.n, m.u_c0[in.u0 + un.u], p, tA, tR, tN,
                          col, g);
          }
        }
        wave_lds_sync();   // the next chunk overwrites the constants and the t table
      }
      const double tot = wave_sum(acc);
      const bool any_bad = __any(bad) || !(tot < kInf);
      const double gc = g_cost ? g_cost[pt] : 1.0;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const double s = wave_sum(g[k]);
        if (lane == 0) {
          g_params[(size_t)pt * P + k] = any_bad ? 0.0 : gc * (2.0 * s);
          if (jtwr) jtwr[(size_t)pt * P + k] = any_bad ? 0.0 : s;
        }
      }
      if (lane == 0 && cost) cost[pt] = any_bad ? kInf : tot;
    }
    __syncthreads();   // the next round overwrites the market values
  }
}

// ---------------------------------------------------------------------------
// Projected Levenberg-Marquardt, one wave per point for all iterations:
//   (J^T W J + mu diag(J^T W J)) delta = -J^T W r, trial = clamp(p + delta),
//   accept if the cost decreases (mu /= 10; stop when the relative decrease
//   < tol), else mu *= 10 (stop once mu > 1e16).  A zero diagonal entry is
//   replaced by 1; coordinates fixed by the box (lb = ub) or on a bound that
//   -J^T W r points out of are frozen for the iteration.
// ---------------------------------------------------------------------------
template <int P>
__device__ bool cholesky_solve_lds(double *A, double *rhs, double *x) {
  // A: P x P row-major in LDS (overwritten by L), rhs: P
  for (int j = 0; j < P; ++j) {
    double s = A[j * P + j];
    for (int k = 0; k < j; ++k) s -= A[j * P + k] * A[j * P + k];
    if (!(s > 0.0) || !(s < kInf)) return false;
    const double ljj = sqrt(s);
    A[j * P + j] = ljj;
    for (int i = j + 1; i < P; ++i) {
      double t = A[i * P + j];
      for (int k = 0; k < j; ++k) t -= A[i * P + k] * A[j * P + k];
      A[i * P + j] = t / ljj;
    }
  }
  for (int i = 0; i < P; ++i) {
    double t = rhs[i];
    for (int k = 0; k < i; ++k) t -= A[i * P + k] * x[k];
    x[i] = t / A[i * P + i];
  }
  for (int i = P - 1; i >= 0; --i) {
    double t = x[i];
    for (int k = i + 1; k < P; ++k) t -= A[k * P + i] * x[k];
    x[i] = t / A[i * P + i];
  }
  return true;
}

// The GLOBAL4 LM (LMM12: lm12_kernel below).
template <int FORMULA, int RESID>
__global__ __launch_bounds__(64) void lm_kernel(DevMarket m, int n_pts, const int *pt_inst,
                                                double *params, const double *lb,
                                                const double *ub, int max_iter, double mu0,
                                                double tol, double *cost_out, int *iters_out) {
  extern __shared__ double smem[];
  constexpr int P = 4;
  constexpr int NT = P * (P + 1) / 2;
  const int lane = lane_id();
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  const WaveLds w{};   // no map
  double *sys = smem + 6 * m.max_nu;   // P*P + 3P doubles
  for (int pt = blockIdx.x; pt < n_pts; pt += gridDim.x) {
    const int inst = __builtin_amdgcn_readfirstlane(pt_inst[pt]);
    if (inst < 0 || inst >= m.n_inst) {
      if (lane == 0) {
        if (cost_out) cost_out[pt] = __builtin_nan("");
        if (iters_out) iters_out[pt] = 0;
      }
      continue;
    }
    const DevInst in = m.inst[inst];
    wave_lds_sync();
    for (int u = lane; u < in.nu; u += kWave) um[u] = und_mkt(m, in.u0 + u);
    wave_lds_sync();
    double p[P], lo[P], hi[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      p[k] = params[(size_t)pt * P + k];
      lo[k] = lb[(size_t)inst * P + k];
      hi[k] = ub[(size_t)inst * P + k];
    }
    double grad[P], g[P], jj[NT];
    double f = point_normal<FORMULA, RESID, true>(m, in, um, p, grad, jj, g);
    double mu = mu0;
    int it = 0;
    if (f < kInf) {
      for (; it < max_iter; ++it) {
        // damped, frozen system into LDS; lane 0 solves
        double *A = sys, *rhs = sys + P * P, *dl = sys + P * P + P;
        wave_lds_sync();
        if (lane == 0) {
          int t = 0;
          for (int i = 0; i < P; ++i)
            for (int j = i; j < P; ++j, ++t) A[i * P + j] = A[j * P + i] = jj[t];
          for (int k = 0; k < P; ++k) {
            const double akk = A[k * P + k];
            A[k * P + k] = akk + mu * (akk > 0.0 ? akk : 1.0);
            rhs[k] = -g[k];
          }
          for (int k = 0; k < P; ++k) {
            const bool frozen = (lo[k] == hi[k]) || (p[k] <= lo[k] && g[k] > 0.0) ||
                                (p[k] >= hi[k] && g[k] < 0.0);
            if (!frozen) continue;
            for (int j = 0; j < P; ++j) A[k * P + j] = A[j * P + k] = 0.0;
            A[k * P + k] = 1.0;
            rhs[k] = 0.0;
          }
          sys[P * P + 2 * P] = cholesky_solve_lds<P>(A, rhs, dl) ? 1.0 : 0.0;
        }
        wave_lds_sync();
        const bool solved = sys[P * P + 2 * P] != 0.0;
        if (!solved) {
          mu *= 10.0;
          continue;
        }
        double trial[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
          double y = p[k] + dl[k];
          if (y > hi[k]) y = hi[k];
          if (y < lo[k]) y = lo[k];
          trial[k] = y;
        }
        const double ft = point_cost<0, FORMULA, RESID>(m, in, um, trial, 0.0, w, nullptr, nullptr);
        if (ft < f) {
          const double rel = (f - ft) / f;
#pragma unroll
          for (int k = 0; k < P; ++k) p[k] = trial[k];
          point_normal<FORMULA, RESID, true>(m, in, um, p, grad, jj, g);
          f = ft;
          mu /= 10.0;
          if (rel < tol) {
            ++it;
            break;
          }
        } else {
          mu *= 10.0;
          if (mu > 1e16) {
            ++it;
            break;
          }
        }
      }
    }
    if (lane == 0) {
      for (int k = 0; k < P; ++k) params[(size_t)pt * P + k] = p[k];
      if (cost_out) cost_out[pt] = f;
      if (iters_out) iters_out[pt] = it;
    }
  }
}

// ---------------------------------------------------------------------------
// LMM12 normal equations without a per-quote Jacobian.  With J_q = M_u^T s_q:
//   J^T W r = sum_u M_u^T t_u,       t_u = sum_{q of u} w_q r_q s_q,
//   J^T W J = sum_u M_u^T S_u M_u,   S_u = sum_{q of u} w_q s_q s_q^T (3 x 3).
// Per chunk of kGradChunk underlyings: the SABR constants, then the quotes
// (lanes over quotes; w r s and the six entries of w s s^T summed per
// underlying by the segmented scan), then one lane per underlying runs three
// reverse sweeps of the map (unit seeds: the rows of M_u), adds M_u^T t_u to
// its J^T W r accumulators and stores M_u and S_u in LDS, and last the lanes
// take the 78 entries of the upper triangle of J^T W J (lane l entry l, lanes
// 0..13 also entry 64 + l) and add sum_u m_i^T S_u m_j over the chunk.
// ---------------------------------------------------------------------------
constexpr int kNormP = 12;
constexpr int kNormT = kNormP * (kNormP + 1) / 2;   // 78
constexpr int kMSDoubles = 3 * kNormP + 6;          // M_u rows and S_u

// Upper-triangle entry t (row-major, i <= j) of a kNormP x kNormP matrix.
__device__ __forceinline__ void tri_ij(int t, int &i, int &j) {
  i = 0;
  int rem = t;
  while (rem >= kNormP - i) {
    rem -= kNormP - i;
    ++i;
  }
  j = i + rem;
}

struct NormLds {
  WaveLds w;     // map records, SABR constants (>= kGradChunk entries), LDS columns
  FwdAux *fx;    // [max_nf]
  double *ts;    // [kGradChunk][9]: t_u (3) and S_u (6)
  double *ms;    // [kGradChunk][kMSDoubles]
  double *sys;   // 2 kNormP^2 + 6 kNormP: the LM system and its inputs
};

__host__ __device__ inline int norm_th_entries(const DevMarket &m) {
  const int t = th_entries(m, false);
  return t > kGradChunk ? t : kGradChunk;
}

// Two LDS columns per lane: the sweep's beyond 24 forwards (the map's own
// column, for the cost of a trial point, is the first of them).
__host__ __device__ inline bool norm_lds_columns(const DevMarket &m) {
  return m.max_len > 24 || lds_column(m, false);
}

__host__ __device__ inline int norm_wave_doubles(const DevMarket &m) {
  return kFwdMapDoubles * m.max_nf + kSabrConstDoubles * norm_th_entries(m) +
         (norm_lds_columns(m) ? 2 * kWave * m.max_len : 0) + 4 * m.max_nf + 9 * kGradChunk +
         kMSDoubles * kGradChunk + 2 * kNormP * kNormP + 6 * kNormP;
}

__device__ __forceinline__ NormLds norm_lds(const DevMarket &m, double *base) {
  NormLds L;
  L.w.fw = reinterpret_cast<FwdMap *>(base);
  double *o = base + kFwdMapDoubles * m.max_nf;
  L.w.th = reinterpret_cast<SabrConst *>(o);
  o += kSabrConstDoubles * norm_th_entries(m);
  L.w.lk = o;
  o += norm_lds_columns(m) ? 2 * kWave * m.max_len : 0;
  L.fx = reinterpret_cast<FwdAux *>(o);
  o += 4 * m.max_nf;
  L.ts = o;
  o += 9 * kGradChunk;
  L.ms = o;
  o += kMSDoubles * kGradChunk;
  L.sys = o;
  return L;
}

// The map Jacobian rows of one underlying, row r = M_u^T e_r for
// r = (alpha_u, rho_u, nu_u) over the 12 parameters, one at a time into
// ms[12 r ..]; g += sum_r t_r row_r.
template <int REG>
__device__ __forceinline__ void und_rows(const UndMap &un, const NormLds &L, int max_len,
                                         const double *p, double c0, const double *t,
                                         double *ms, double (&g)[kNormP]) {
  if (un.n == 1) {
    const FwdAux X = L.fx[un.e];
    double M[3][kNormP];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < kNormP; ++k) M[r][k] = 0.0;
    M[0][0] = X.E;
    M[0][1] = X.T * X.E;
    M[0][2] = -X.T * fma(p[1], X.T, p[0]) * X.E;
    M[0][3] = 1.0;
    M[1][8] = 1.0;
    M[2][4] = X.En;
    M[2][5] = X.T * X.En;
    M[2][6] = -X.T * fma(p[5], X.T, p[4]) * X.En;
    M[2][7] = 1.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < kNormP; ++k) {
        ms[r * kNormP + k] = M[r][k];
        g[k] = fma(t[r], M[r][k], g[k]);
      }
    return;
  }
  for (int r = 0; r < 3; ++r) {
    double row[kNormP];
#pragma unroll
    for (int k = 0; k < kNormP; ++k) row[k] = 0.0;
    SweepCols<REG> col;
    if constexpr (REG == 0) {
      col.c1 = L.w.lk + lane_id();
      col.c2 = L.w.lk + (size_t)max_len * kWave + lane_id();
    }
    swap_vjp<REG>(L.w.fw + un.e, L.fx + un.e, un.n, c0, p, r == 0 ? 1.0 : 0.0,
                  r == 1 ? 1.0 : 0.0, r == 2 ? 1.0 : 0.0, col, row);
#pragma unroll
    for (int k = 0; k < kNormP; ++k) {
      ms[r * kNormP + k] = row[k];
      g[k] = fma(t[r], row[k], g[k]);
    }
  }
}

// Cost, J^T W r (wave-uniform, jr) and J^T W J (lane l holds entries l and,
// for l < kNormT - kWave, 64 + l: h[0], h[1]) of one LMM12 point; +inf cost
// and zero derivatives outside the domain.
template <int FORMULA, int RESID, int REG>
__device__ double lmm_normal(const DevMarket &m, const DevInst &in, const UndMkt *um,
                             const double *p, const NormLds &L, double (&jr)[kNormP],
                             double (&h)[2]) {
  const int lane = lane_id();
  bool bad = lmm12_fwd(m, in, p, L.w);
  for (int k = lane; k < in.nf; k += kWave) {
    const double T = m.f_T[in.f0 + k];
    L.fx[k] = FwdAux{exp_neg(-(p[2] * T)), exp_neg(-(p[6] * T)), T, m.f_v[in.f0 + k]};
  }
  wave_lds_sync();
  double g[kNormP];
#pragma unroll
  for (int k = 0; k < kNormP; ++k) g[k] = 0.0;
  h[0] = h[1] = 0.0;
  int hi0, hj0, hi1 = 0, hj1 = 0;
  tri_ij(lane, hi0, hj0);
  const bool two = lane + kWave < kNormT;
  if (two) tri_ij(lane + kWave, hi1, hj1);
  double acc = 0.0;
  const int *uq0 = m.u_q0 + in.u0;
  const UndMap *umap = m.u_map + in.u0;
  const QuoteRec *qrec = m.q + in.q0;
  const double beta = m.beta;
  for (int c0 = 0; c0 < in.nu; c0 += kGradChunk) {
    const int c1 = min(in.nu, c0 + kGradChunk);
    bad |= lmm12_und<FORMULA, (REG > 0 ? REG : kMapRegLen)>(m, in, um, p, L.w, c0, c1);
    for (int k = lane; k < 9 * kGradChunk; k += kWave) L.ts[k] = 0.0;
    wave_lds_sync();
    const int qa = uq0[c0], qb = c1 < in.nu ? uq0[c1] : in.nq;
    for (int q0 = qa; q0 < qb; q0 += kWave) {   // wave-uniform trip count
      const int q = q0 + lane;
      int key = -1 - lane;                        // no quote: a run of its own
      double v[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = 0.0;
      if (q < qb) {
        const QuoteRec R = qrec[q];
        const QuoteSens qs = quote_sens<FORMULA, RESID>(L.w.th[R.und - c0], beta, R, um[R.und]);
        key = R.und;
        bad |= qs.bad;
        const double r = qs.m - R.tgt;
        acc = fma(R.w * r, r, acc);
        const double wr = R.w * r;
        v[0] = wr * qs.sa;
        v[1] = wr * qs.sr;
        v[2] = wr * qs.sn;
        const double wa = R.w * qs.sa, wrh = R.w * qs.sr;
        v[3] = wa * qs.sa;
        v[4] = wa * qs.sr;
        v[5] = wa * qs.sn;
        v[6] = wrh * qs.sr;
        v[7] = wrh * qs.sn;
        v[8] = R.w * qs.sn * qs.sn;
      }
      const int prev = __shfl_up(key, 1, kWave);
      const unsigned long long heads = __ballot(lane == 0 || prev != key);
      const unsigned long long upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
      const int start = kWave - 1 - __clzll(heads & upto);
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = seg_scan(v[k], lane, start);
      const bool tail = key >= 0 && (lane == kWave - 1 || ((heads >> (lane + 1)) & 1));
      if (tail) {
        double *t = L.ts + 9 * (key - c0);
#pragma unroll
        for (int k = 0; k < 9; ++k) t[k] += v[k];
      }
    }
    wave_lds_sync();
    const int i = c0 + lane;   // one underlying per lane (kGradChunk = kWave)
    if (i < c1) {
      const UndMap un = umap[i];
      const double *t = L.ts + 9 * lane;
      double *ms = L.ms + kMSDoubles * lane;
      und_rows<REG>(un, L, m.max_len, p, m.u_c0[in.u0 + un.u], t, ms, g);
#pragma unroll
      for (int k = 0; k < 6; ++k) ms[3 * kNormP + k] = t[3 + k];
    }
    wave_lds_sync();
    // J^T W J entries: sum over the chunk's underlyings of m_i^T S m_j,
    // S = [[s0 s1 s2], [s1 s3 s4], [s2 s4 s5]]
    for (int u = 0; u < c1 - c0; ++u) {
      const double *ms = L.ms + kMSDoubles * u;
      const double *S = ms + 3 * kNormP;
      {
        const double a0 = ms[hi0], a1 = ms[kNormP + hi0], a2 = ms[2 * kNormP + hi0];
        const double b0 = ms[hj0], b1 = ms[kNormP + hj0], b2 = ms[2 * kNormP + hj0];
        const double Sb0 = fma(S[0], b0, fma(S[1], b1, S[2] * b2));
        const double Sb1 = fma(S[1], b0, fma(S[3], b1, S[4] * b2));
        const double Sb2 = fma(S[2], b0, fma(S[4], b1, S[5] * b2));
        h[0] = fma(a0, Sb0, fma(a1, Sb1, fma(a2, Sb2, h[0])));
      }
      if (two) {
        const double a0 = ms[hi1], a1 = ms[kNormP + hi1], a2 = ms[2 * kNormP + hi1];
        const double b0 = ms[hj1], b1 = ms[kNormP + hj1], b2 = ms[2 * kNormP + hj1];
        const double Sb0 = fma(S[0], b0, fma(S[1], b1, S[2] * b2));
        const double Sb1 = fma(S[1], b0, fma(S[3], b1, S[4] * b2));
        const double Sb2 = fma(S[2], b0, fma(S[4], b1, S[5] * b2));
        h[1] = fma(a0, Sb0, fma(a1, Sb1, fma(a2, Sb2, h[1])));
      }
    }
    wave_lds_sync();   // the next chunk overwrites the constants and both tables
  }
  const double tot = wave_sum(acc);
  const bool any_bad = __any(bad) || !(tot < kInf);
#pragma unroll
  for (int k = 0; k < kNormP; ++k) {
    const double s = wave_sum(g[k]);
    jr[k] = any_bad ? 0.0 : s;
  }
  if (any_bad) h[0] = h[1] = 0.0;
  return any_bad ? kInf : tot;
}

// Writes the lanes' J^T W J entries into a full kNormP x kNormP row-major
// matrix A (both triangles).
__device__ __forceinline__ void scatter_jtwj(double *A, const double (&h)[2]) {
  const int lane = lane_id();
  int i, j;
  tri_ij(lane, i, j);
  A[i * kNormP + j] = h[0];
  A[j * kNormP + i] = h[0];
  if (lane + kWave < kNormT) {
    tri_ij(lane + kWave, i, j);
    A[i * kNormP + j] = h[1];
    A[j * kNormP + i] = h[1];
  }
}

// sabr_cost_vjp with J^T W J on LMM12 plans: one wave per point, up to
// kGradWaves points per workgroup sharing the market values (rounds per
// distinct instance, as cost_kernel).
template <int FORMULA, int RESID, int REG>
__global__ __launch_bounds__(kWave *kGradWaves) void normal_kernel(DevMarket m, int n_pts,
                                                                   const int *pt_inst,
                                                                   const double *params,
                                                                   const double *g_cost,
                                                                   double *cost, double *g_params,
                                                                   double *jtwj, double *jtwr,
                                                                   int lds_per_wave) {
  extern __shared__ double smem[];
  __shared__ int s_inst[kGradWaves];
  const int nw = blockDim.x / kWave;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = lane_id();
  const int pt = blockIdx.x * nw + wid;
  int inst = -1;
  if (pt < n_pts) inst = __builtin_amdgcn_readfirstlane(pt_inst[pt]);
  const bool valid = pt < n_pts && inst >= 0 && inst < m.n_inst;
  if (pt < n_pts && !valid && lane == 0 && cost) cost[pt] = __builtin_nan("");
  if (lane == 0) s_inst[wid] = valid ? inst : -1;
  __syncthreads();
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  const NormLds L = norm_lds(m, smem + 6 * m.max_nu + (size_t)wid * lds_per_wave);
  for (int r = 0; r < nw; ++r) {
    const int ri = s_inst[r];
    bool first = ri >= 0;
    for (int q = 0; q < r; ++q) first = first && s_inst[q] != ri;
    if (!first) continue;
    const DevInst rin = m.inst[ri];
    for (int u = threadIdx.x; u < rin.nu; u += blockDim.x) um[u] = und_mkt(m, rin.u0 + u);
    __syncthreads();
    if (valid && inst == ri) {
      const DevInst in = m.inst[inst];
      double p[kNormP], jr[kNormP], h[2];
#pragma unroll
      for (int k = 0; k < kNormP; ++k) p[k] = params[(size_t)pt * kNormP + k];
      const double f = lmm_normal<FORMULA, RESID, REG>(m, in, um, p, L, jr, h);
      const double gc = g_cost ? g_cost[pt] : 1.0;
      if (lane == 0) {
        if (cost) cost[pt] = f;
#pragma unroll
        for (int k = 0; k < kNormP; ++k) {
          g_params[(size_t)pt * kNormP + k] = gc * (2.0 * jr[k]);
          if (jtwr) jtwr[(size_t)pt * kNormP + k] = jr[k];
        }
      }
      if (jtwj) scatter_jtwj(jtwj + (size_t)pt * kNormP * kNormP, h);
    }
    __syncthreads();
  }
}

// Projected Levenberg-Marquardt (as lm_kernel) for LMM12 plans with the
// normal equations of lmm_normal; one wave per point for all its
// iterations, up to kGradWaves points per workgroup.
template <int FORMULA, int RESID, int REG>
__global__ __launch_bounds__(kWave *kGradWaves) void lm12_kernel(DevMarket m, int n_pts,
                                                                 const int *pt_inst,
                                                                 double *params, const double *lb,
                                                                 const double *ub, int max_iter,
                                                                 double mu0, double tol,
                                                                 double *cost_out,
                                                                 int *iters_out,
                                                                 int lds_per_wave) {
  extern __shared__ double smem[];
  __shared__ int s_inst[kGradWaves];
  constexpr int P = kNormP;
  constexpr int CM = (REG == 24) ? 5 : 1;   // the cost kernels' model variant
  const int nw = blockDim.x / kWave;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = lane_id();
  const int pt = blockIdx.x * nw + wid;
  int inst = -1;
  if (pt < n_pts) inst = __builtin_amdgcn_readfirstlane(pt_inst[pt]);
  const bool valid = pt < n_pts && inst >= 0 && inst < m.n_inst;
  if (pt < n_pts && !valid && lane == 0) {
    if (cost_out) cost_out[pt] = __builtin_nan("");
    if (iters_out) iters_out[pt] = 0;
  }
  if (lane == 0) s_inst[wid] = valid ? inst : -1;
  __syncthreads();
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  const NormLds L = norm_lds(m, smem + 6 * m.max_nu + (size_t)wid * lds_per_wave);
  for (int r = 0; r < nw; ++r) {
    const int ri = s_inst[r];
    bool first = ri >= 0;
    for (int q = 0; q < r; ++q) first = first && s_inst[q] != ri;
    if (!first) continue;
    const DevInst rin = m.inst[ri];
    for (int u = threadIdx.x; u < rin.nu; u += blockDim.x) um[u] = und_mkt(m, rin.u0 + u);
    __syncthreads();
    if (valid && inst == ri) {
      const DevInst in = m.inst[inst];
      // LDS: A (P x P, overwritten by its factor), rhs, solution, solved
      // flag, J^T W r, box, J^T W J
      double *A = L.sys, *rhs = A + P * P, *dl = rhs + P, *flag = dl + P;
      double *gj = flag + P, *lo = gj + P, *hi = lo + P, *Hs = hi + P;
      double p[P];
#pragma unroll
      for (int k = 0; k < P; ++k) p[k] = params[(size_t)pt * P + k];
      if (lane < P) {
        lo[lane] = lb[(size_t)inst * P + lane];
        hi[lane] = ub[(size_t)inst * P + lane];
      }
      double f = kInf, mu = mu0;
      int it = 0;
      bool need = true, start = true;
      // one call site each for the normal equations (at the start and after
      // every accepted step) and for the trial cost
      for (;;) {
        if (need) {
          double g[P], h[2];
          const double fn = lmm_normal<FORMULA, RESID, REG>(m, in, um, p, L, g, h);
          wave_lds_sync();
          if (lane == 0)
            for (int k = 0; k < P; ++k) gj[k] = g[k];
          scatter_jtwj(Hs, h);
          wave_lds_sync();
          need = false;
          if (start) {
            start = false;
            f = fn;
            if (!(f < kInf)) break;
          }
        }
        if (it >= max_iter) break;
        // damped, frozen system from the stored J^T W J; lane 0 solves
        if (lane == 0) {
          for (int k = 0; k < P * P; ++k) A[k] = Hs[k];
          for (int k = 0; k < P; ++k) {
            const double akk = A[k * P + k];
            A[k * P + k] = akk + mu * (akk > 0.0 ? akk : 1.0);
            rhs[k] = -gj[k];
          }
          for (int k = 0; k < P; ++k) {
            const bool frozen = (lo[k] == hi[k]) || (p[k] <= lo[k] && gj[k] > 0.0) ||
                                (p[k] >= hi[k] && gj[k] < 0.0);
            if (!frozen) continue;
            for (int j = 0; j < P; ++j) A[k * P + j] = A[j * P + k] = 0.0;
            A[k * P + k] = 1.0;
            rhs[k] = 0.0;
          }
          flag[0] = cholesky_solve_lds<P>(A, rhs, dl) ? 1.0 : 0.0;
        }
        wave_lds_sync();
        const bool solved = flag[0] != 0.0;
        double trial[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
          double y = p[k] + dl[k];
          if (y > hi[k]) y = hi[k];
          if (y < lo[k]) y = lo[k];
          trial[k] = y;
        }
        ++it;
        bool accept = false, stop = false;
        if (solved) {
          const double ft = point_cost<CM, FORMULA, RESID>(m, in, um, trial, 0.0, L.w, nullptr,
                                                            nullptr);
          if (ft < f) {
            const double rel = (f - ft) / f;
            f = ft;
            mu /= 10.0;
            accept = true;
            stop = rel < tol;
          } else {
            mu *= 10.0;
            stop = mu > 1e16;
          }
        } else {
          mu *= 10.0;
        }
        if (accept) {
#pragma unroll
          for (int k = 0; k < P; ++k) p[k] = trial[k];
          need = true;
        }
        if (stop) break;
        wave_lds_sync();   // the next pass overwrites A, rhs and dl
      }
      if (lane == 0) {
        for (int k = 0; k < P; ++k) params[(size_t)pt * P + k] = p[k];
        if (cost_out) cost_out[pt] = f;
        if (iters_out) iters_out[pt] = it;
      }
    }
    __syncthreads();
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
#define SABR_SELECT_FR(FORMULA_, RESID_, CALL)                      \
  do {                                                              \
    if ((FORMULA_) == 0) {                                          \
      if ((RESID_) == 0) { CALL(0, 0); } else { CALL(0, 1); }       \
    } else {                                                        \
      if ((RESID_) == 0) { CALL(1, 0); } else { CALL(1, 1); }       \
    }                                                               \
  } while (0)

// LDS of the GLOBAL4 vjp and LM kernels: the market values and the LM system.
size_t adjoint_lds_bytes(const DevMarket &m) {
  constexpr int P = 4;
  return (size_t)(6 * m.max_nu + P * P + 3 * P) * 8;
}

int adjoint_waves(int n_pts) { return n_pts < kAdjointMaxWaves ? n_pts : kAdjointMaxWaves; }

// Waves per workgroup of the gradient kernel: the most waves per CU that
// 160 KB of LDS holds (each workgroup stages the market values once), ties
// to the larger workgroup; 0 if not even one wave fits.
int grad_waves(const DevMarket &m) {
  const long per_cu = 160 * 1024;
  int best = 0, best_res = 0;
  for (int w = kGradWaves; w >= 1; w >>= 1) {
    const long bytes = (long)(6 * m.max_nu + (long)w * grad_wave_doubles(m)) * 8;
    if (bytes > lds_budget_bytes()) continue;
    const int res = (int)std::min<long>(per_cu / bytes * w, 16);
    if (res > best_res) {
      best_res = res;
      best = w;
    }
  }
  return best;
}

// Waves per workgroup of the normal-equation kernels, by the same rule.
int norm_waves(const DevMarket &m) {
  const long per_cu = 160 * 1024;
  int best = 0, best_res = 0;
  for (int w = kGradWaves; w >= 1; w >>= 1) {
    const long bytes = (long)(6 * m.max_nu + (long)w * norm_wave_doubles(m)) * 8;
    if (bytes > lds_budget_bytes()) continue;
    const int res = (int)std::min<long>(per_cu / bytes * w, 16);
    if (res > best_res) {
      best_res = res;
      best = w;
    }
  }
  return best;
}

#define SABR_REG_SELECT(LAUNCH, B, C)   \
  do {                                 \
    if (m.max_len <= kMapRegLen)       \
      LAUNCH(B, C, 16);                \
    else if (m.max_len <= 24)          \
      LAUNCH(B, C, 24);                \
    else                               \
      LAUNCH(B, C, 0);                 \
  } while (0)
#define SABR_FR_SELECT(LAUNCH)                                                  \
  do {                                                                          \
    if (m.formula == 0) {                                                       \
      if (m.residual == 0) SABR_REG_SELECT(LAUNCH, 0, 0); else SABR_REG_SELECT(LAUNCH, 0, 1); \
    } else {                                                                    \
      if (m.residual == 0) SABR_REG_SELECT(LAUNCH, 1, 0); else SABR_REG_SELECT(LAUNCH, 1, 1); \
    }                                                                           \
  } while (0)

hipError_t launch_normal(const DevMarket &m, int n_pts, const int *pt_inst, const double *params,
                         const double *g_cost, double *cost, double *g_params, double *jtwj,
                         double *jtwr, hipStream_t s) {
  const int waves = norm_waves(m);
  if (waves == 0) return hipErrorInvalidValue;
  const int ld = norm_wave_doubles(m);
  const size_t lds = (size_t)(6 * m.max_nu + waves * ld) * 8;
  const dim3 grid((n_pts + waves - 1) / waves), block(kWave * waves);
#define LAUNCH(B, C, R)                                                                       \
  hipLaunchKernelGGL((normal_kernel<B, C, R>), grid, block, lds, s, m, n_pts, pt_inst, params, \
                     g_cost, cost, g_params, jtwj, jtwr, ld)
  SABR_FR_SELECT(LAUNCH);
#undef LAUNCH
  return hipGetLastError();
}

hipError_t launch_lm12(const DevMarket &m, int n_pts, const int *pt_inst, double *params,
                       const double *lb, const double *ub, int max_iter, double mu0, double tol,
                       double *cost_out, int *iters_out, hipStream_t s) {
  const int waves = norm_waves(m);
  if (waves == 0) return hipErrorInvalidValue;
  const int ld = norm_wave_doubles(m);
  const size_t lds = (size_t)(6 * m.max_nu + waves * ld) * 8;
  const dim3 grid((n_pts + waves - 1) / waves), block(kWave * waves);
#define LAUNCH(B, C, R)                                                                     \
  hipLaunchKernelGGL((lm12_kernel<B, C, R>), grid, block, lds, s, m, n_pts, pt_inst, params, \
                     lb, ub, max_iter, mu0, tol, cost_out, iters_out, ld)
  SABR_FR_SELECT(LAUNCH);
#undef LAUNCH
  return hipGetLastError();
}

hipError_t launch_grad(const DevMarket &m, int n_pts, const int *pt_inst, const double *params,
                       const double *g_cost, double *cost, double *g_params, double *jtwr,
                       hipStream_t s) {
  const int waves = grad_waves(m);
  if (waves == 0) return hipErrorInvalidValue;
  const int ld = grad_wave_doubles(m);
  const size_t lds = (size_t)(6 * m.max_nu + waves * ld) * 8;
  const dim3 grid((n_pts + waves - 1) / waves), block(kWave * waves);
#define LAUNCH(B, C, R)                                                                     \
  hipLaunchKernelGGL((grad_kernel<B, C, R>), grid, block, lds, s, m, n_pts, pt_inst, params, \
                     g_cost, cost, g_params, jtwr, ld)
#define CALL(B, C)                     \
  do {                                 \
    if (m.max_len <= kMapRegLen)       \
      LAUNCH(B, C, 16);                \
    else if (m.max_len <= 24)          \
      LAUNCH(B, C, 24);                \
    else                               \
      LAUNCH(B, C, 0);                 \
  } while (0)
  if (m.formula == 0) {
    if (m.residual == 0) CALL(0, 0); else CALL(0, 1);
  } else {
    if (m.residual == 0) CALL(1, 0); else CALL(1, 1);
  }
#undef CALL
#undef LAUNCH
  return hipGetLastError();
}

hipError_t launch_vjp(const DevMarket &m, int n_pts, const int *pt_inst, const double *params,
                      const double *g_cost, double *cost, double *g_params, double *jtwj,
                      double *jtwr, hipStream_t s) {
  if (n_pts == 0) return hipSuccess;
  if (m.model != 0 && m.model != 1) return hipErrorInvalidValue;   // GLOBAL4 and LMM12 only
  // LMM12: per-underlying seeds and map sweeps (the gradient alone: one
  // sweep each; with J^T W J: the three rows of M_u)
  if (m.model == 1 && !jtwj)
    return launch_grad(m, n_pts, pt_inst, params, g_cost, cost, g_params, jtwr, s);
  if (m.model == 1)
    return launch_normal(m, n_pts, pt_inst, params, g_cost, cost, g_params, jtwj, jtwr, s);
  const size_t lds = adjoint_lds_bytes(m);
  const int waves = adjoint_waves(n_pts);
#define CALL(B, C)                                                                           \
  do {                                                                                       \
    if (jtwj)                                                                                \
      hipLaunchKernelGGL((vjp_kernel<B, C, true>), dim3(waves), dim3(kWave), lds, s, m,      \
                         n_pts, pt_inst, params, g_cost, cost, g_params, jtwj, jtwr);          \
    else                                                                                     \
      hipLaunchKernelGGL((vjp_kernel<B, C, false>), dim3(waves), dim3(kWave), lds, s, m,     \
                         n_pts, pt_inst, params, g_cost, cost, g_params, jtwj, jtwr);          \
  } while (0)
  SABR_SELECT_FR(m.formula, m.residual, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t launch_lm(const DevMarket &m, int n_pts, const int *pt_inst, double *params,
                     const double *lb, const double *ub, int max_iter, double mu0, double tol,
                     double *cost_out, int *iters_out, hipStream_t s) {
  if (n_pts == 0) return hipSuccess;
  if (m.model != 0 && m.model != 1) return hipErrorInvalidValue;   // GLOBAL4 and LMM12 only
  if (m.model == 1)
    return launch_lm12(m, n_pts, pt_inst, params, lb, ub, max_iter, mu0, tol, cost_out,
                       iters_out, s);
  const size_t lds = adjoint_lds_bytes(m);
  const int waves = adjoint_waves(n_pts);
#define CALL(B, C)                                                                          \
  hipLaunchKernelGGL((lm_kernel<B, C>), dim3(waves), dim3(kWave), lds, s, m, n_pts, pt_inst,   \
                     params, lb, ub, max_iter, mu0, tol, cost_out, iters_out)
  SABR_SELECT_FR(m.formula, m.residual, CALL);
#undef CALL
  return hipGetLastError();
}

}  // namespace sabr
