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

// ---------------------------------------------------------------------------
// Jacobian of the LMM12 map.  Row 0: alpha_u, row 1: rho_u, row 2: nu_u, each
// over the 12 parameters, written to M[u*36 ..] (global scratch of the wave).
// Caplet (forward e): alpha_e = (a + b T) E + d, E = e^{-cT}; nu_e alike;
// rho_u = rho.  Swap: reverse sweep of the O(n^2) form of the frozen-weight
// map (pair factors by running products of the gap factors g1, g2):
//   a_j = v_j alpha_j, R_j = sum_l a_l rho_jl, V = sum a_j R_j, s_a = sum a_j,
//   b_j = a_j R_j nu_j, S_b = sum b_j, Be_j = sum_l b_l e_jl (e = theta's
//   exponential), Btheta_j = eta2 S_b + (1 - eta2) Be_j, Nb = sum b_j Btheta_j,
//   alpha_S = sqrt(V)/(A S0^b), nu_S = sqrt(Nb)/V, rho_S = rho s_a S_b/sqrt(V Nb).
// ---------------------------------------------------------------------------
struct FwdExp {
  double E, En;  // e^{-c T_k}, e^{-c_n T_k}
};

__device__ void lmm12_jacobian(const DevMarket &m, const DevInst &in, const double *p, WaveLds w,
                               const FwdExp *ef, double *col, double *M) {
  const int lane = lane_id();
  const double a = p[0], b = p[1];
  const double an = p[4], bn = p[5];
  const double rho = p[8], eta2 = p[10];
  const int ML = m.max_len;
  // per-lane columns (stride kWave): R_j, b_j, Be_j, and two scratch columns
  double *cR = col + lane;
  double *cb = col + ML * kWave + lane;
  double *cB = col + 2 * ML * kWave + lane;
  double *c3 = col + 3 * ML * kWave + lane;
  double *c4 = col + 4 * ML * kWave + lane;
  const double *fT = m.f_T + in.f0;
  const double *fv = m.f_v + in.f0;
  for (int u = lane; u < in.nu; u += kWave) {
    double *Mu = M + (size_t)u * 36;
    const int e = m.u_first[in.u0 + u];
    const int n = m.u_len[in.u0 + u];
    if (n == 1) {
      for (int j = 0; j < 36; ++j) Mu[j] = 0.0;
      const double T = fT[e];
      const double E = ef[e].E, En = ef[e].En;
      Mu[0] = E;
      Mu[1] = T * E;
      Mu[2] = -T * fma(b, T, a) * E;
      Mu[3] = 1.0;
      Mu[12 + 8] = 1.0;
      Mu[24 + 4] = En;
      Mu[24 + 5] = T * En;
      Mu[24 + 6] = -T * fma(bn, T, an) * En;
      Mu[24 + 7] = 1.0;
      continue;
    }
    const FwdMap *fw = w.fw + e;
    // Forward values in O(n): every sum over pairs with a factor
    // exp(-lambda |T_j - T_l|) is a left plus a right recursion over the gap
    // factors (g1 for rho_jl, g2 for the theta kernel e_jl); the |T_l - T_j|
    // weighted sums add a time-weighted recursion (sum x_l k_jl (T_j - T_l)
    // over l < j = T_j L_j - LT_j, and symmetrically on the right).
    double sa = 0.0, V = 0.0, Sb = 0.0;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {        // left sums of a (g1)
      cR[j * kWave] = acc;
      const double aj = fw[j].a;
      sa += aj;
      acc = fw[j].g1 * (acc + aj);
    }
    acc = 0.0;
    for (int j = n - 1; j >= 0; --j) {   // R_j = left + a_j + right; b_j
      const double aj = fw[j].a;
      const double Rj = cR[j * kWave] + aj + acc;
      cR[j * kWave] = Rj;
      V = fma(aj, Rj, V);
      const double bj = aj * Rj * fw[j].nv;
      cb[j * kWave] = bj;
      Sb += bj;
      if (j > 0) acc = fw[j - 1].g1 * (acc + aj);
    }
    double Lb = 0.0, LbT = 0.0;
    for (int j = 0; j < n; ++j) {        // left sums of b (g2), plain and time-weighted
      const double bj = cb[j * kWave], T = fT[e + j];
      cB[j * kWave] = Lb;
      c3[j * kWave] = fma(T, Lb, -LbT);
      const double g2 = fw[j].g2;
      Lb = g2 * (Lb + bj);
      LbT = g2 * fma(bj, T, LbT);
    }
    double Nb = 0.0, bBe = 0.0, lam2_pairs = 0.0, Rb = 0.0, RbT = 0.0;
    for (int j = n - 1; j >= 0; --j) {   // Be_j, sum_l b_l e_jl |T_l - T_j|
      const double bj = cb[j * kWave], T = fT[e + j];
      const double Be = cB[j * kWave] + bj + Rb;
      cB[j * kWave] = Be;
      const double dBe = c3[j * kWave] + fma(-T, Rb, RbT);
      Nb = fma(bj, fma(eta2, Sb, (1.0 - eta2) * Be), Nb);
      bBe = fma(bj, Be, bBe);
      lam2_pairs = fma(bj, dBe, lam2_pairs);
      if (j > 0) {
        const double g2 = fw[j - 1].g2;
        Rb = g2 * (Rb + bj);
        RbT = g2 * fma(bj, T, RbT);
      }
    }
    const double sV = sqrt(V), sN = sqrt(Nb);
    const double c0 = m.u_invA[in.u0 + u] / m.u_S0b[in.u0 + u];
    const double rhoS = (sN > 0.0) ? rho * sa * Sb / (sV * sN) : 0.0;
    for (int row = 0; row < 3; ++row) {
      const double sA = row == 0 ? 1.0 : 0.0, sR = row == 1 ? 1.0 : 0.0,
                   sNu = row == 2 ? 1.0 : 0.0;
      double Vb = sA * c0 / (2.0 * sV);
      double Nbb = 0.0, sab = 0.0, Sbb = 0.0, rb = 0.0;
      if (sN > 0.0) {
        Vb += -sNu * sN / (V * V) - sR * rhoS / (2.0 * V);
        Nbb = sNu / (2.0 * sN * V) - sR * rhoS / (2.0 * Nb);
        const double inv = 1.0 / (sV * sN);
        sab = sR * rho * Sb * inv;
        Sbb = sR * rho * sa * inv;
        rb = sR * sa * Sb * inv;
      }
      // R-bar_j = a_j (b-bar_j nu_j + V-bar), b-bar_j = 2 Nb-bar Btheta_j + S_b-bar;
      // right sums of R-bar (g1), plain (cb) and time-weighted (c4)
      double RR = 0.0, RRT = 0.0;
      for (int j = n - 1; j >= 0; --j) {
        const double T = fT[e + j];
        const double bbj = fma(2.0 * Nbb, fma(eta2, Sb, (1.0 - eta2) * cB[j * kWave]), Sbb);
        const double Rbj = fw[j].a * fma(bbj, fw[j].nv, Vb);
        c3[j * kWave] = Rbj;
        cb[j * kWave] = RR;
        c4[j * kWave] = fma(-T, RR, RRT);
        if (j > 0) {
          const double g1 = fw[j - 1].g1;
          RR = g1 * (RR + Rbj);
          RRT = g1 * fma(Rbj, T, RRT);
        }
      }
      // a-bar_j = b-bar_j nu_j R_j + V-bar R_j + s_a-bar + sum_m R-bar_m rho_mj, and
      // the lambda1 term -sum_j a_j sum_l R-bar_l rho_jl |T_l - T_j|
      double LR = 0.0, LRT = 0.0, l1 = 0.0;
      double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0, m5 = 0.0, m6 = 0.0, m7 = 0.0;
      for (int j = 0; j < n; ++j) {
        const FwdMap F = fw[j];
        const double T = fT[e + j];
        const double aj = F.a, Rj = cR[j * kWave], Rbj = c3[j * kWave];
        const double bbj = fma(2.0 * Nbb, fma(eta2, Sb, (1.0 - eta2) * cB[j * kWave]), Sbb);
        const double abar =
            fma(bbj * F.nv, Rj, fma(Vb, Rj, sab)) + ((LR + Rbj) + cb[j * kWave]);
        l1 = fma(-aj, fma(T, LR, -LRT) + c4[j * kWave], l1);
        const double alb = abar * fv[e + j];   // alpha-bar_j
        const double nub = bbj * aj * Rj;      // nu-bar_j
        const double E = ef[e + j].E, En = ef[e + j].En;
        m0 = fma(alb, E, m0);
        m1 = fma(alb * T, E, m1);
        m2 = fma(-alb * T * fma(b, T, a), E, m2);
        m3 += alb;
        m4 = fma(nub, En, m4);
        m5 = fma(nub * T, En, m5);
        m6 = fma(-nub * T * fma(bn, T, an), En, m6);
        m7 += nub;
        LR = F.g1 * (LR + Rbj);
        LRT = F.g1 * fma(Rbj, T, LRT);
      }
      double *Mr = Mu + row * 12;
      Mr[0] = m0;
      Mr[1] = m1;
      Mr[2] = m2;
      Mr[3] = m3;
      Mr[4] = m4;
      Mr[5] = m5;
      Mr[6] = m6;
      Mr[7] = m7;
      Mr[8] = rb;
      Mr[9] = l1;                                     // lambda1
      Mr[10] = Nbb * (Sb * Sb - bBe);                 // eta2
      Mr[11] = -Nbb * (1.0 - eta2) * lam2_pairs;      // lambda2 (ordered pairs)
    }
  }
}

// Accumulates the cost, gradient and (optionally) normal equations of one
// point over the wave's quotes.  Out-of-domain points give cost +inf and
// zero derivatives.  grad, jtwr: P values; jtwj: P(P+1)/2 (upper triangle).
template <int MODEL, int FORMULA, int RESID, bool NORMAL>
__device__ double point_normal(const DevMarket &m, const DevInst &in, const UndMkt *um,
                               const double *p, WaveLds w, FwdExp *ef, double *col,
                               double *M, double *grad, double *jtwj, double *jtwr) {
  constexpr int P = NP<MODEL>::P;
  constexpr int NT = P * (P + 1) / 2;
  const int lane = lane_id();
  bool bad;
  double beta;
  if (MODEL == 0) {
    bad = !(p[0] > 0.0) || !(p[1] >= 0.0 && p[1] <= 1.0) || !(fabs(p[2]) < 1.0) ||
          !(p[3] >= 0.0);
    beta = p[1];
  } else {
    bad = lmm12_map<FORMULA>(m, in, um, p, w);
    beta = m.beta;
    for (int k = lane; k < in.nf; k += kWave) {
      const double T = m.f_T[in.f0 + k];
      ef[k] = FwdExp{exp(-(p[2] * T)), exp(-(p[6] * T))};
    }
    wave_lds_sync();
    if (!bad) lmm12_jacobian(m, in, p, w, ef, col, M);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  double g[P], jr[P], jj[NORMAL ? NT : 1];
#pragma unroll
  for (int k = 0; k < P; ++k) g[k] = jr[k] = 0.0;
#pragma unroll
  for (int k = 0; k < (NORMAL ? NT : 1); ++k) jj[k] = 0.0;
  double acc = 0.0;
  for (int q = lane; q < in.nq; q += kWave) {
    const QuoteRec &R = m.q[in.q0 + q];
    const UndMkt U = um[R.und];
    double al, rh, nu;
    if (MODEL == 0) {
      al = p[0];
      rh = p[2];
      nu = p[3];
    } else {
      const SabrConst &K = w.th[R.und];
      al = K.alpha;
      rh = K.rho;
      nu = K.nua * K.alpha;
    }
    const SigGrad sg = quote_grad<FORMULA, RESID>(al, beta, rh, nu, R, U, MODEL == 0);
    bad |= !(sg.vol > 0.0) || !(sg.vol < kInf) || !(fabs(sg.sig) < kInf);
    const double r = sg.sig - R.tgt;
    acc = fma(R.w * r, r, acc);
    double J[P];
    if (MODEL == 0) {
      J[0] = sg.da;
      J[1] = sg.db;
      J[2] = sg.dr;
      J[3] = sg.dn;
    } else {
      const double *Mu = M + (size_t)R.und * 36;
#pragma unroll
      for (int k = 0; k < P; ++k) J[k] = sg.da * Mu[k] + sg.dr * Mu[12 + k] + sg.dn * Mu[24 + k];
    }
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

__device__ __forceinline__ size_t vjp_lds_doubles(const DevMarket &m) {
  return 6 * m.max_nu + wave_lds_doubles(m, true) + (m.model == 1 ? 2 * m.max_nf + 5 * m.max_len * kWave : 0);
}

// sabr_cost_vjp: one wave per point (grid-stride), private M_u scratch per wave.
template <int MODEL, int FORMULA, int RESID, bool NORMAL>
__global__ __launch_bounds__(64) void vjp_kernel(DevMarket m, int n_pts, const int *pt_inst,
                                                 const double *params, const double *g_cost,
                                                 double *cost, double *g_params, double *jtwj,
                                                 double *jtwr, double *scratch) {
  extern __shared__ double smem[];
  constexpr int P = NP<MODEL>::P;
  constexpr int NT = P * (P + 1) / 2;
  const int lane = lane_id();
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  WaveLds w = wave_lds(m, smem + 6 * m.max_nu, true);
  FwdExp *ef = reinterpret_cast<FwdExp *>(smem + 6 * m.max_nu + wave_lds_doubles(m, true));
  double *col = smem + 6 * m.max_nu + wave_lds_doubles(m, true) + 2 * m.max_nf;
  double *M = scratch + (size_t)blockIdx.x * m.max_nu * 36;
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
    const double f = point_normal<MODEL, FORMULA, RESID, NORMAL>(m, in, um, p, w, ef, col, M,
                                                                 grad, jj, jr);
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

template <int MODEL, int FORMULA, int RESID>
__global__ __launch_bounds__(64) void lm_kernel(DevMarket m, int n_pts, const int *pt_inst,
                                                double *params, const double *lb,
                                                const double *ub, int max_iter, double mu0,
                                                double tol, double *cost_out, int *iters_out,
                                                double *scratch) {
  extern __shared__ double smem[];
  constexpr int P = NP<MODEL>::P;
  constexpr int NT = P * (P + 1) / 2;
  const int lane = lane_id();
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  WaveLds w = wave_lds(m, smem + 6 * m.max_nu, true);
  FwdExp *ef = reinterpret_cast<FwdExp *>(smem + 6 * m.max_nu + wave_lds_doubles(m, true));
  double *col = smem + 6 * m.max_nu + wave_lds_doubles(m, true) + 2 * m.max_nf;
  double *sys = col + (MODEL == 1 ? 5 * m.max_len * kWave : 0);  // P*P + 3P doubles
  double *M = scratch + (size_t)blockIdx.x * m.max_nu * 36;
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
    double f = point_normal<MODEL, FORMULA, RESID, true>(m, in, um, p, w, ef, col, M, grad, jj,
                                                          g);
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
        const double ft = point_cost<MODEL, FORMULA, RESID>(m, in, um, trial, 0.0, w, nullptr, nullptr);
        if (ft < f) {
          const double rel = (f - ft) / f;
#pragma unroll
          for (int k = 0; k < P; ++k) p[k] = trial[k];
          point_normal<MODEL, FORMULA, RESID, true>(m, in, um, p, w, ef, col, M, grad, jj, g);
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

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
#define SABR_SELECT3(MODEL_, FORMULA_, RESID_, CALL)                  \
  do {                                                                \
    if ((MODEL_) == 0) {                                              \
      if ((FORMULA_) == 0) {                                          \
        if ((RESID_) == 0) { CALL(0, 0, 0); } else { CALL(0, 0, 1); } \
      } else {                                                        \
        if ((RESID_) == 0) { CALL(0, 1, 0); } else { CALL(0, 1, 1); } \
      }                                                               \
    } else {                                                          \
      if ((FORMULA_) == 0) {                                          \
        if ((RESID_) == 0) { CALL(1, 0, 0); } else { CALL(1, 0, 1); } \
      } else {                                                        \
        if ((RESID_) == 0) { CALL(1, 1, 0); } else { CALL(1, 1, 1); } \
      }                                                               \
    }                                                                 \
  } while (0)

size_t adjoint_lds_bytes(const DevMarket &m) {
  const int P = m.model == 0 ? 4 : 12;
  return (size_t)(6 * m.max_nu + wave_lds_doubles(m, true) + 2 * m.max_nf +
                  (m.model == 1 ? 5 * m.max_len * kWave : 0) + P * P + 3 * P) *
         8;
}

size_t adjoint_scratch_bytes(const DevMarket &m, int n_waves) {
  return m.model == 1 ? (size_t)n_waves * m.max_nu * 36 * 8 : 0;
}

int adjoint_waves(int n_pts) { return n_pts < kAdjointMaxWaves ? n_pts : kAdjointMaxWaves; }

hipError_t launch_vjp(const DevMarket &m, int n_pts, const int *pt_inst, const double *params,
                      const double *g_cost, double *cost, double *g_params, double *jtwj,
                      double *jtwr, double *scratch, hipStream_t s) {
  if (n_pts == 0) return hipSuccess;
  if (m.model != 0 && m.model != 1) return hipErrorInvalidValue;   // GLOBAL4 and LMM12 only
  const size_t lds = adjoint_lds_bytes(m);
  const int waves = adjoint_waves(n_pts);
#define CALL(A, B, C)                                                                        \
  do {                                                                                       \
    if (jtwj)                                                                                \
      hipLaunchKernelGGL((vjp_kernel<A, B, C, true>), dim3(waves), dim3(kWave), lds, s, m,   \
                         n_pts, pt_inst, params, g_cost, cost, g_params, jtwj, jtwr, scratch); \
    else                                                                                     \
      hipLaunchKernelGGL((vjp_kernel<A, B, C, false>), dim3(waves), dim3(kWave), lds, s, m,  \
                         n_pts, pt_inst, params, g_cost, cost, g_params, jtwj, jtwr, scratch); \
  } while (0)
  SABR_SELECT3(m.model, m.formula, m.residual, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t launch_lm(const DevMarket &m, int n_pts, const int *pt_inst, double *params,
                     const double *lb, const double *ub, int max_iter, double mu0, double tol,
                     double *cost_out, int *iters_out, double *scratch, hipStream_t s) {
  if (n_pts == 0) return hipSuccess;
  if (m.model != 0 && m.model != 1) return hipErrorInvalidValue;   // GLOBAL4 and LMM12 only
  const size_t lds = adjoint_lds_bytes(m);
  const int waves = adjoint_waves(n_pts);
#define CALL(A, B, C)                                                                       \
  hipLaunchKernelGGL((lm_kernel<A, B, C>), dim3(waves), dim3(kWave), lds, s, m, n_pts, pt_inst, \
                     params, lb, ub, max_iter, mu0, tol, cost_out, iters_out, scratch)
  SABR_SELECT3(m.model, m.formula, m.residual, CALL);
#undef CALL
  return hipGetLastError();
}

}  // namespace sabr
