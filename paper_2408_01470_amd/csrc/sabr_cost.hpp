// sabr_cost.hpp -- the per-point cost evaluation shared by the annealing,
// cost, adjoint and Levenberg-Marquardt kernels: LDS layout of a wavefront,
// the LMM12 parameter map and the quote loop.
#pragma once
#include "gauss_legendre.hpp"
#include "sabr_internal.hpp"

namespace sabr {

template <int MODEL>
struct NP;
template <>
struct NP<0> {
  static constexpr int P = 4;
};
template <>
struct NP<1> {
  static constexpr int P = 12;
};
// PERFWD (three parameters per forward) and MM (two per forward and one):
// known at run time (DevMarket::np).
template <>
struct NP<2> {
  static constexpr int P = 0;
};
template <>
struct NP<3> {
  static constexpr int P = 0;
};
template <>
struct NP<4> {   // REB: two per forward and eight
  static constexpr int P = 0;
};
template <>
struct NP<5> {   // LMM12, the swap column in 24 registers
  static constexpr int P = 12;
};

// Per-wave LDS scratch of the LMM12 map: per forward {alpha, nu, g1, g2, a}
// (g1, g2: correlation factors of the gap to the next forward; a = v alpha,
// the forward's term of the swap recursions) and the count of forwards
// outside the domain (alpha > 0, nu >= 0) before it and up to it (two 32-bit
// counts in one word, so a swap's check is one difference); per underlying
// its SABR constants; a per-lane column for long swap recursions.
struct FwdMap {
  double al, nv, g1, g2, a, nbad;
};
__device__ __forceinline__ double pack_counts(int before, int upto) {
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)upto << 32) | (unsigned)before);
}
__device__ __forceinline__ int count_before(double c) {
  return (int)(unsigned)__builtin_bit_cast(unsigned long long, c);
}
__device__ __forceinline__ int count_upto(double c) {
  return (int)(unsigned)(__builtin_bit_cast(unsigned long long, c) >> 32);
}
static_assert(sizeof(FwdMap) == 48, "16-byte aligned LDS record");
constexpr int kFwdMapDoubles = 6;

struct WaveLds {
  FwdMap *fw;      // [max_nf]
  SabrConst *th;   // [max_nu]
  double *lk;      // [max_len][64], used for swaps longer than kMapRegLen
};

__device__ __forceinline__ WaveLds wave_lds(const DevMarket &m, double *base,
                                            bool full = false) {
  WaveLds w;
  w.fw = reinterpret_cast<FwdMap *>(base);
  w.th = reinterpret_cast<SabrConst *>(base + kFwdMapDoubles * m.max_nf);
  w.lk = base + kFwdMapDoubles * m.max_nf + kSabrConstDoubles * th_entries(m, full);
  return w;
}

__device__ __forceinline__ UndMkt und_mkt(const DevMarket &m, int g) {
  const double T = m.u_T[g];
  const double sT = sqrt(T);
  return UndMkt{m.u_S0[g], m.u_A[g], T, sT, 1.0 / sT, m.model != 0 ? m.u_fp[g] : 0.0};
}

// The forward records of a swap from forward e on, as an LDS pointer: the
// unrolled recursions below then address them with constant offsets.
using FwdLds = __attribute__((address_space(3))) const FwdMap *;
__device__ __forceinline__ FwdLds fwd_at(const FwdMap *fw, int e) {
  using lcp = __attribute__((address_space(3))) const char *;
  return (FwdLds)((lcp)fw + __umul24((unsigned)e, (unsigned)sizeof(FwdMap)));
}

// Moments of the frozen-weight map of one swap over forwards [e, e+n),
// n >= 2, with a_j = v_j alpha_j and R_j = sum_l a_l rho_jl:
//   V = sum_j a_j R_j, suma = sum_j a_j, b_j = a_j R_j nu_j, Sb = sum_j b_j,
//   Sbb = sum_kl b_k b_l exp(-lambda2 |T_k - T_l|).
// R_j = (left sum) + a_j + (right sum); the left sums come from a forward
// recursion and are kept per lane, the right sums and the b recursion run
// backward.  Two storage variants of the per-lane column: registers for
// swaps of up to kMapRegLen forwards (loops unrolled so every index is
// static), an LDS column of max_len doubles per lane beyond that.
// The forwards' domain (alpha > 0, nu >= 0) is checked once per forward by
// the map (FwdMap::nbad), not here.
struct SwapMoments {
  double V, suma, Sb, Sbb;
};

template <int NMAX>
__device__ __forceinline__ SwapMoments swap_moments_reg(const FwdMap *fw, int e, int n) {
  const FwdLds f = fwd_at(fw, e);
  double Lk[NMAX];
  double Lacc = 0.0, suma = 0.0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    if (j < n) {
      const double aj = f[j].a;
      Lk[j] = Lacc;
      suma += aj;
      Lacc = f[j].g1 * (Lacc + aj);
    }
  }
  double Rr = 0.0, Rb = 0.0, V = 0.0, Sb = 0.0, Sbb = 0.0;
#pragma unroll
  for (int j = NMAX - 1; j >= 0; --j) {
    if (j < n) {
      const double aj = f[j].a;
      const double Rj = Lk[j] + aj + Rr;
      const double ar = aj * Rj;
      V += ar;
      const double bj = ar * f[j].nv;
      Sb += bj;
      Sbb = fma(bj, fma(2.0, Rb, bj), Sbb);
      if (j > 0) {
        Rr = f[j - 1].g1 * (Rr + aj);
        Rb = f[j - 1].g2 * (Rb + bj);
      }
    }
  }
  return SwapMoments{V, suma, Sb, Sbb};
}

__device__ __forceinline__ SwapMoments swap_moments_lds(const FwdMap *fw, int e, int n,
                                                        double *lk) {
  double Lacc = 0.0, suma = 0.0;
  for (int j = 0; j < n; ++j) {
    const FwdMap F = fw[e + j];
    const double aj = F.a;
    lk[j * kWave] = Lacc;
    suma += aj;
    Lacc = F.g1 * (Lacc + aj);
  }
  double Rr = 0.0, Rb = 0.0, V = 0.0, Sb = 0.0, Sbb = 0.0;
  for (int j = n - 1; j >= 0; --j) {
    const FwdMap F = fw[e + j];
    const double aj = F.a;
    const double Rj = lk[j * kWave] + aj + Rr;
    const double ar = aj * Rj;
    V += ar;
    const double bj = ar * F.nv;
    Sb += bj;
    Sbb = fma(bj, fma(2.0, Rb, bj), Sbb);
    if (j > 0) {
      const FwdMap G = fw[e + j - 1];
      Rr = G.g1 * (Rr + aj);
      Rb = G.g2 * (Rb + bj);
    }
  }
  return SwapMoments{V, suma, Sb, Sbb};
}

// SABR constants of one underlying with SABR parameters (alpha, rho, nu) and
// beta fixed; fp = f^(1-beta).  Hagan 2002 (FORMULA 0): alpha, rho,
// nu/alpha and the expiry-correction coefficients
//   ca = (1-b)^2 alpha^2/24, cb = rho b nu alpha/4, cc = (2 - 3 rho^2) nu^2/24.
// Paper eq. (sigmaHagan) (FORMULA 1): its vol is a quadratic in k = ln(K/f)
// whose coefficients depend on the underlying only, so ca, cb, cc hold them:
//   sigma = ca + cb k + cc k^2,  ca = alpha/fp,  cb = -ca (1-b - rho nu w)/2,
//   cc = ca ((1-b)^2 + (2 - 3 rho^2) nu^2 w^2 + 3 (1-b - rho nu w))/12,
//   w = fp/alpha.
template <int FORMULA>
__device__ __forceinline__ SabrConst und_const(double ta, double tr, double tn, double beta,
                                               double fp) {
  const double omb = 1.0 - beta;
  const double ia = rcp_nr(ta);
  SabrConst K;
  K.alpha = ta;
  K.rho = tr;
  K.nua = tn * ia;
  if (FORMULA == 0) {
    K.ca = omb * omb * ta * ta * (1.0 / 24.0);
    K.cb = tr * beta * tn * ta * 0.25;
    K.cc = (2.0 - 3.0 * (tr * tr)) * tn * tn * (1.0 / 24.0);
  } else {
    const double wv = fp * ia;
    const double e0 = ta * rcp_nr(fp);
    const double d = omb - tr * tn * wv;
    const double nw = tn * wv;
    K.ca = e0;
    K.cb = -0.5 * e0 * d;
    K.cc = e0 * ((omb * omb + (2.0 - 3.0 * (tr * tr)) * nw * nw + 3.0 * d) * (1.0 / 12.0));
  }
  return K;
}

// LMM12 parameter map of one point into the wave's LDS.  Returns true when
// the point lies outside the model's domain (wave-uniform).
//   alpha_k = (a + b T_k) e^{-c T_k} + d, nu_k likewise (abcd forms);
//   rho_kl = exp(-lambda1 |T_k - T_l|) = product of per-gap factors g1,
//   theta_kl = eta2 + (1 - eta2) exp(-lambda2 |T_k - T_l|), phi_kl = rho.
// Swap of forwards [e, e+n) with a_k = v_k alpha_k (v_k = tau_k P_k F_k^b;
// the weights w_k = tau_k P_k / A enter through the common factor 1/A):
//   R_k = sum_l a_l rho_kl (forward and backward recursions, O(n)),
//   V = sum a_k R_k, b_k = a_k R_k nu_k,
//   Nb = eta2 (sum b)^2 + (1 - eta2) sum_kl b_k b_l exp(-lambda2 |dT|),
//   alpha_S = sqrt(V)/(A S0^b), nu_S = sqrt(Nb)/V,
//   rho_S = rho (sum a)(sum b) / (sqrt(V) sqrt(Nb))   (0 if Nb = 0).
// Underlyings are visited in decreasing length (the u_map table) so the lanes
// of a pass run recursions of similar length.
// Forward part: the parameter domain and the per-forward records.
__device__ inline bool lmm12_fwd(const DevMarket &m, const DevInst &in, const double *p,
                                 WaveLds w) {
  const int lane = lane_id();
  const double a = p[0], b = p[1], c = p[2], d = p[3];
  const double an = p[4], bn = p[5], cn = p[6], dn = p[7];
  const double rho = p[8], lam1 = p[9], eta2 = p[10], lam2 = p[11];
  const bool bad = !(fabs(rho) < 1.0) || !(lam1 >= 0.0) || !(lam2 >= 0.0) ||
                   !(eta2 >= 0.0 && eta2 <= 1.0);
  int carry = 0;   // forwards outside the domain in earlier passes
  for (int k0 = 0; k0 < in.nf; k0 += kWave) {   // wave-uniform: the counts need every lane
    const int k = k0 + lane;
    const bool live = k < in.nf;
    FwdMap F{};
    if (live) {
      const double T = m.f_T[in.f0 + k];
      F.al = fma(b, T, a) * exp_neg(-(c * T)) + d;
      F.nv = fma(bn, T, an) * exp_neg(-(cn * T)) + dn;
      F.a = m.f_v[in.f0 + k] * F.al;
      if (k + 1 < in.nf) {
        const double dT = m.f_T[in.f0 + k + 1] - T;
        F.g1 = exp_neg(-(lam1 * dT));
        F.g2 = exp_neg(-(lam2 * dT));
      }
    }
    const bool out = live && (!(F.al > 0.0) || !(F.nv >= 0.0));
    const uint64_t mask = __ballot(out);
    const int before =
        carry + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                               __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
    F.nbad = pack_counts(before, before + (out ? 1 : 0));
    if (live) w.fw[k] = F;
    carry += __popcll(mask);
  }
  wave_lds_sync();
  return bad;
}

// Whether a forward of [e, e+n) lies outside the domain (the map's counts).
__device__ __forceinline__ bool fwd_out_of_domain(const FwdMap *fw, int e, int n) {
  return count_upto(fw[e + n - 1].nbad) > count_before(fw[e].nbad);
}

// Underlying part for the underlyings [i0, i1) of the map's visiting order
// (the internal order): their SABR constants go to w.th[u - i0].  Returns
// this lane's domain failure.
template <int FORMULA, int REG = kMapRegLen>
__device__ inline bool lmm12_und(const DevMarket &m, const DevInst &in, const UndMkt *um,
                                 const double *p, WaveLds w, int i0, int i1) {
  const int lane = lane_id();
  const double rho = p[8], eta2 = p[10];
  const double beta = m.beta;
  bool bad = false;
  const UndMap *umap = m.u_map + in.u0;
  UndMap un{0, 0, 1, 0};
  if (i0 + lane < i1) un = umap[i0 + lane];
  double *lk = w.lk + lane;
  for (int i = i0 + lane; i < i1; i += kWave) {
    const int u = un.u, e = un.e, n = un.n;
    if (i + kWave < i1) un = umap[i + kWave];   // next pass's entry
    double ta, tr, tn;
    if (n == 1) {
      const FwdMap F = w.fw[e];
      ta = F.al;
      tr = rho;
      tn = F.nv;
      bad |= !(ta > 0.0) || !(tn >= 0.0);
    } else {
      const SwapMoments S = (m.max_len <= REG) ? swap_moments_reg<REG>(w.fw, e, n)
                                               : swap_moments_lds(w.fw, e, n, lk);
      const double V = S.V, suma = S.suma, Sb = S.Sb, Sbb = S.Sbb;
      bad |= fwd_out_of_domain(w.fw, e, n);
      const double Nb = fma(eta2 * Sb, Sb, (1.0 - eta2) * Sbb);
      const double sV = sqrt_gs(V), sN = sqrt_gs(Nb);
      ta = sV * m.u_c0[in.u0 + u];
      tn = sN * rcp_nr(V);
      tr = (sN > 0.0) ? rho * suma * Sb * rcp_nr(sV * sN) : 0.0;
      bad |= !(V > 0.0) || !(fabs(tr) < 1.0);
    }
    w.th[u - i0] = und_const<FORMULA>(ta, tr, tn, beta, um[u].fp);
  }
  wave_lds_sync();
  return bad;
}

// The whole map into the wave's LDS (a full-size underlying table).
template <int FORMULA>
__device__ inline bool lmm12_map(const DevMarket &m, const DevInst &in, const UndMkt *um,
                                 const double *p, WaveLds w) {
  bool bad = lmm12_fwd(m, in, p, w);
  bad |= lmm12_und<FORMULA>(m, in, um, p, w, 0, in.nu);
  return __any(bad);
}

// PERFWD map (the Hagan model of Sec. 3 with per-forward parameters, as
// calibrated to caplets in Sec. 4.1.1): lane k < np holds coordinate k of
// (alpha_1, rho_1, nu_1, alpha_2, ...), beta is fixed.  Each caplet's SABR
// constants come from its forward's triple, fetched across lanes.  Every
// triple must lie in the domain (alpha > 0, |rho| < 1, nu >= 0).  Returns
// true (wave-uniform) on a domain failure.
template <int FORMULA>
__device__ bool perfwd_map(const DevMarket &m, const DevInst &in, const UndMkt *um, double xl,
                           WaveLds w) {
  const int lane = lane_id();
  const double beta = m.beta;
  const int role = lane % 3;
  bool bad = false;
  if (lane < m.np)
    bad = (role == 0) ? !(xl > 0.0) : (role == 1) ? !(fabs(xl) < 1.0) : !(xl >= 0.0);
  const UndMap *umap = m.u_map + in.u0;
  for (int i0 = 0; i0 < in.nu; i0 += kWave) {   // wave-uniform trip count: every lane shuffles
    const int i = i0 + lane;
    UndMap un{0, 0, 1, 0};
    if (i < in.nu) un = umap[i];
    const int src = 3 * un.e;
    const double ta = __shfl(xl, src, kWave);
    const double tr = __shfl(xl, src + 1, kWave);
    const double tn = __shfl(xl, src + 2, kWave);
    if (i < in.nu) w.th[un.u] = und_const<FORMULA>(ta, tr, tn, beta, um[un.u].fp);
  }
  wave_lds_sync();
  return __any(bad);
}

// MM map (the Mercurio-Morini model of Sec. 2.2 with the SABR parameters of
// eq. (haganForMercurio)): lane k < np holds coordinate k of
// (alpha_1, phi_1, ..., alpha_n, phi_n, sigma), beta fixed.  Lane j < n
// computes alpha_j^SABR = alpha_j exp(-sigma D_j), D_j = sum_{l<=j} phi_l
// alpha_l w_l with the plan's drift weights w_l = T_{l-1} tau_l F_l^beta /
// (1 + tau_l F_l) (T_{-1} = 0: the drift sum starts at the forward after the
// first unfixed one), by a prefix sum over the lanes; each caplet fetches
// its forward's alpha^SABR and phi across lanes, nu = sigma.  Domain:
// alpha_j > 0, |phi_j| < 1, sigma >= 0.  Returns true (wave-uniform) on a
// domain failure.
template <int FORMULA>
__device__ bool mm_map(const DevMarket &m, const DevInst &in, const UndMkt *um, double xl,
                       WaveLds w) {
  const int lane = lane_id();
  const int np = m.np;   // 2 nf + 1
  const double beta = m.beta;
  bool bad = false;
  if (lane < np)
    bad = (lane == np - 1) ? !(xl >= 0.0) : ((lane & 1) == 0) ? !(xl > 0.0) : !(fabs(xl) < 1.0);
  const double sigma = readlane_d(xl, np - 1);
  const double al = __shfl(xl, 2 * lane, kWave);       // lanes j < nf: alpha_j, phi_j
  const double ph = __shfl(xl, 2 * lane + 1, kWave);
  double d = (lane < in.nf) ? ph * al * m.f_mmw[in.f0 + lane] : 0.0;
#pragma unroll
  for (int o = 1; o < kWave / 2; o <<= 1) {   // inclusive prefix sum over lanes 0..31
    const double t = __shfl_up(d, o, kWave);
    if (lane >= o) d += t;
  }
  const double aS = al * exp_cw(-(sigma * d));
  const UndMap *umap = m.u_map + in.u0;
  for (int i0 = 0; i0 < in.nu; i0 += kWave) {   // wave-uniform trip count: every lane shuffles
    const int i = i0 + lane;
    UndMap un{0, 0, 1, 0};
    if (i < in.nu) un = umap[i];
    const double ta = __shfl(aS, un.e, kWave);
    const double tr = __shfl(ph, un.e, kWave);
    if (i < in.nu) w.th[un.u] = und_const<FORMULA>(ta, tr, sigma, beta, um[un.u].fp);
  }
  wave_lds_sync();
  return __any(bad);
}

// Square integral of an abcd function, Q(x) = int_0^x ((a + b u) e^{-c u} +
// d)^2 du for c >= 0, x >= 0, from the moments I_m(k, x) = int_0^x u^m
// e^{-k u} du (m = 0, 1, 2) at k = c and k = 2c.  With psi_m(z) =
// int_0^1 s^m e^{-z s} ds, I_m = x^{m+1} psi_m(kx); psi_2 by its series
// sum_j (-z)^j / (j! (j + 3)) when z < 1/2 (17 terms: truncation < 1e-19),
// a polynomial in -z evaluated by Horner's rule, else
// (2 - e^{-z} (2 + 2z + z^2)) / z^3, and psi_1, psi_0 by the downward
// recurrence psi_{m-1} = (z psi_m + e^{-z}) / m, stable for every z >= 0.
// e1 = e^{-c x} is passed in (e^{-2cx} = e1^2).
constexpr double psi2_series_coef(int j) {
  double f = 1.0;   // j!, exact in double for j <= 16
  for (int i = 2; i <= j; ++i) f *= i;
  return 1.0 / (f * (j + 3));
}
constexpr int kPsi2Deg = 16;
constexpr double kPsi2Series[kPsi2Deg + 1] = {
    psi2_series_coef(0),  psi2_series_coef(1),  psi2_series_coef(2),  psi2_series_coef(3),
    psi2_series_coef(4),  psi2_series_coef(5),  psi2_series_coef(6),  psi2_series_coef(7),
    psi2_series_coef(8),  psi2_series_coef(9),  psi2_series_coef(10), psi2_series_coef(11),
    psi2_series_coef(12), psi2_series_coef(13), psi2_series_coef(14), psi2_series_coef(15),
    psi2_series_coef(16)};

// psi_0, psi_1, psi_2 at z >= 0 given e = e^{-z} and the series value s.
__device__ __forceinline__ void psi012(double z, double e, double s, double &p0, double &p1,
                                       double &p2) {
  const double iz = rcp_nr(z);
  const double big = (2.0 - e * fma(z, z + 2.0, 2.0)) * (iz * iz * iz);
  p2 = (z < 0.5) ? s : big;
  p1 = fma(z, p2, e) * 0.5;
  p0 = fma(z, p1, e);
}

__device__ __forceinline__ double abcd_sq_int(double a, double b, double c, double d, double x,
                                              double e1) {
  const double z2 = 2.0 * c * x, z1 = c * x;
  double s2, s1;   // the two series, their Horner chains interleaved
  horner2_s<kPsi2Series, kPsi2Deg>(-z2, -z1, s2, s1, std::make_index_sequence<kPsi2Deg>{});
  double p0, p1, p2, q0, q1, q2;
  psi012(z2, e1 * e1, s2, p0, p1, p2);
  psi012(z1, e1, s1, q0, q1, q2);
  // a^2 I0(2c) + 2ab I1(2c) + b^2 I2(2c) + 2d (a I0(c) + b I1(c)) + d^2 x
  const double t2 = x * fma(a * a, p0, x * fma(2.0 * a * b, p1, x * (b * b) * p2));
  const double t1 = 2.0 * d * x * fma(a, q0, b * x * q1);
  return fma(d * d, x, t2 + t1);
}

// Rebonato map (the Rebonato model of Sec. 2.2 with the SABR parameters of
// eq. (haganForRebonato)): lane k < np holds coordinate k of (kappa_1,
// phi_1, ..., kappa_n, phi_n, a, b, c, d, a_h, b_h, c_h, d_h), beta fixed.
// For the caplet on forward e with expiry T:
//   alpha = kappa_e sqrt(G / T), G = Qg(T);  nu = sqrt(2 J / (T G)),
//   J = int_0^T g(tau)^2 (Qh(T) - Qh(tau)) dtau  (tau = T - t),
// Qg, Qh the square integrals of g and h (abcd_sq_int), J by the 32-point
// Gauss-Legendre rule.  First pass (lanes over underlyings): G and Qh(T)
// into the underlying's LDS record; second pass (lanes over underlying x
// node pairs, 32 lanes per underlying): the quadrature terms, summed over
// the 32 lanes, and the SABR constants.  Domain: kappa_e > 0, |phi_e| < 1,
// c >= 0, c_h >= 0, G > 0.
template <int FORMULA>
__device__ bool reb_map(const DevMarket &m, const DevInst &in, const UndMkt *um, double xl,
                        WaveLds w) {
  const int lane = lane_id();
  const int np = m.np;   // 2 nf + 8
  const int q0 = np - 8;
  const double beta = m.beta;
  bool bad = false;
  if (lane < q0) bad = ((lane & 1) == 0) ? !(xl > 0.0) : !(fabs(xl) < 1.0);
  const double a = readlane_d(xl, q0), b = readlane_d(xl, q0 + 1);
  const double c = readlane_d(xl, q0 + 2), d = readlane_d(xl, q0 + 3);
  const double ah = readlane_d(xl, q0 + 4), bh = readlane_d(xl, q0 + 5);
  const double ch = readlane_d(xl, q0 + 6), dh = readlane_d(xl, q0 + 7);
  bad |= !(c >= 0.0) || !(ch >= 0.0);
  const UndMap *umap = m.u_map + in.u0;
  for (int i = lane; i < in.nu; i += kWave) {
    const UndMap un = umap[i];
    const double T = um[un.u].T;
    SabrConst K{};
    K.ca = abcd_sq_int(a, b, c, d, T, exp_neg(-(c * T)));
    K.cb = abcd_sq_int(ah, bh, ch, dh, T, exp_neg(-(ch * T)));
    bad |= !(K.ca > 0.0);
    w.th[un.u] = K;
  }
  wave_lds_sync();
  const int half = lane >> 5, j = lane & 31;
  const double node = kGLNode[j], weight = kGLWeight[j];
  for (int i0 = 0; i0 < in.nu; i0 += 2) {   // two underlyings a pass, one per half-wave
    const int i = i0 + half;
    double term = 0.0;
    UndMap un{0, 0, 1, 0};
    if (i < in.nu) {
      un = umap[i];
      const double T = um[un.u].T;
      const double QT = w.th[un.u].cb;
      const double ht = 0.5 * T;
      const double tau = fma(ht, node, ht);
      const double g = fma(b, tau, a) * exp_neg(-(c * tau)) + d;
      const double Qt = abcd_sq_int(ah, bh, ch, dh, tau, exp_neg(-(ch * tau)));
      term = (ht * weight) * (g * g) * (QT - Qt);
    }
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) term += __shfl_xor(term, o, kWave);   // within the half
    const double kap = __shfl(xl, 2 * un.e, kWave);
    const double phi = __shfl(xl, 2 * un.e + 1, kWave);
    wave_lds_sync();
    if (i < in.nu && j == 0) {
      const double T = um[un.u].T;
      const double G = w.th[un.u].ca;
      const double iT = rcp_nr(T);
      const double ta = kap * sqrt_gs(G * iT);
      const double tn = sqrt_gs(2.0 * term * iT * rcp_nr(G));
      w.th[un.u] = und_const<FORMULA>(ta, phi, tn, beta, um[un.u].fp);
    }
    bad |= (i < in.nu) && !(term >= 0.0);
    wave_lds_sync();
  }
  return __any(bad);
}

// Cost of one point for the wave: f = sum_q w_q r_q^2, +inf on a domain
// failure.  p[] is wave-uniform (GLOBAL4, LMM12); PERFWD, MM and REB read
// the point from the lanes instead (xl: lane k holds coordinate k).  Optional
// per-quote residual and model outputs (the quoted side in price mode).
// Split evaluation: with nsub > 1 waves sharing the point, wave sub takes
// the quotes of every nsub-th block of 64 (from block sub on) and returns
// their partial sum (+inf on a domain failure); the map is every wave's.
// PAIR (GLOBAL4 only): each half of the wave evaluates its own point (p[]
// holds the half's coordinates) over the instance's quotes, 32 at a time,
// and every lane gets its half's cost, bit for bit the cost one wave gives:
// half-lane l stands for wave lanes l (the even passes) and l + 32 (the odd
// ones), keeps their two partial sums apart and adds them in wave_sum's
// order (half_sum2).
template <int MODEL, int FORMULA, int RESID, bool PAIR = false>
__device__ double point_cost(const DevMarket &m, const DevInst &in, const UndMkt *um,
                             const double *p, double xl, WaveLds w, double *resid,
                             double *model, int sub = 0, int nsub = 1) {
  static_assert(!PAIR || MODEL == 0, "paired chains: the map must be per-lane arithmetic");
  constexpr bool LMM = (MODEL == 1 || MODEL == 5);   // 5: LMM12, 24-register swap column
  constexpr int REG = (MODEL == 5) ? 24 : kMapRegLen;
  // the lane's place among the lanes of its point
  const int lane = PAIR ? (lane_id() & (kHalf - 1)) : lane_id();
  bool bad = false;
  SabrConst g{};
  double omb, omb2 = 0.0;
  if (MODEL == 0) {
    bad = !(p[0] > 0.0) || !(p[1] >= 0.0 && p[1] <= 1.0) || !(fabs(p[2]) < 1.0) ||
          !(p[3] >= 0.0);
    g = sabr_const(p[0], p[1], p[2], p[3]);
    omb = 1.0 - p[1];
    omb2 = omb * omb;
  } else if (LMM) {
    bad = lmm12_fwd(m, in, p, w);   // the underlyings follow chunk by chunk
    omb = 1.0 - m.beta;
  } else if (MODEL == 2) {
    bad = perfwd_map<FORMULA>(m, in, um, xl, w);
    omb = 1.0 - m.beta;
  } else if (MODEL == 3) {
    bad = mm_map<FORMULA>(m, in, um, xl, w);
    omb = 1.0 - m.beta;
  } else {
    bad = reb_map<FORMULA>(m, in, um, xl, w);
    omb = 1.0 - m.beta;
  }
  double acc = 0.0, acc_hi = 0.0;   // acc_hi: PAIR's odd passes (wave lanes 32-63)
  const int *qx = m.q_ext + in.q0;   // per-quote outputs go to the caller's order
  auto quote = [&](const QuoteRec &R, int q, int toff, double &acc) {
    const double L = R.L;
    const int u = R.und;
    const UndMkt U = lds_elem(um, u);
    const SabrConst k = (MODEL == 0) ? g : lds_elem(w.th, u - toff);
    // eq. (sigmaHagan) with beta fixed: the vol itself, a quadratic in
    // k = ln(K/f) = -L with the underlying's coefficients
    constexpr bool direct = (FORMULA == 1 && MODEL != 0);
    VolFrac vf;
    if (FORMULA == 0) {
      const double qv = (MODEL == 0) ? exp_cw(0.5 * omb * R.qa) : R.qa;
      const double q3D1 = (MODEL == 0) ? qv * qv * qv * d1_term(omb2, L) : R.qb;
      vf = hagan2002_frac(k, L, qv, q3D1, U.T);
    } else if (direct) {
      vf.numer = fma(-L, fma(-L, k.cc, k.cb), k.ca);
      vf.denom = 1.0;
    } else {
      vf = paper_eq3_frac(k, omb, L, exp_cw(omb * R.qc));
    }
    double mv;
    if (RESID == 0) {
      mv = direct ? vf.numer : vf.numer * rcp_nr(vf.denom);
      bad |= !(mv > 0.0) || !(mv < kInf);
      if (model) model[qx[q]] = mv;
    } else {
      // one reciprocal gives sigma = numer/denom and 1/sigma = denom/numer
      const double rr = rcp_nr(vf.numer * vf.denom);
      const double sig = direct ? vf.numer : vf.numer * (vf.numer * rr);
      const double isig = direct ? rr : vf.denom * (vf.denom * rr);
      bad |= !(sig > 0.0) || !(sig < kInf);
      mv = black_otm(U.f, R.K, L, U.sqrtT, U.isqrtT, sig, isig, U.D);
      bad |= !(fabs(mv) < kInf);
      if (model) {
        const double sh = parity_shift(R.kind, U.f, R.K, L, U.D);
        model[qx[q]] = sh == 0.0 ? mv : mv + sh;
      }
    }
    const double r = mv - R.tgt;
    acc = fma(R.w * r, r, acc);
    if (resid) resid[qx[q]] = r;
  };
  // Quotes [qa, qb) (this wave's blocks of them) with two record buffers in
  // turn: the next pass's record is loaded while this pass computes (the
  // global load latency hides behind the arithmetic), and no register copies
  // are needed between passes.
  const QuoteRec *qrec = m.q + in.q0;
  const int qs = PAIR ? kHalf : nsub * kWave;
  auto quotes = [&](int qa, int qb, int toff) {
    QuoteRec Ra{}, Rb{};
    const int q0 = qa + sub * kWave + lane;
    if (q0 < qb) Ra = glb_elem(qrec, q0);
    for (int q = q0; q < qb; q += 2 * qs) {
      if (q + qs < qb) Rb = glb_elem(qrec, q + qs);
      quote(Ra, q, toff, acc);
      if (q + qs >= qb) break;
      if (q + 2 * qs < qb) Ra = glb_elem(qrec, q + 2 * qs);
      quote(Rb, q + qs, toff, PAIR ? acc_hi : acc);
    }
  };
  if (LMM) {
    // LMM12: the underlyings' SABR constants chunk by chunk (thchunk of
    // them in LDS at a time), each followed by its underlyings' quotes (a
    // contiguous range in the internal order)
    const int *uq0 = m.u_q0 + in.u0;
    const int chunk = m.thchunk;
    for (int c0 = 0; c0 < in.nu; c0 += chunk) {
      const int c1 = min(in.nu, c0 + chunk);
      bad |= lmm12_und<FORMULA, REG>(m, in, um, p, w, c0, c1);
      quotes(uq0[c0], c1 < in.nu ? uq0[c1] : in.nq, c0);
      wave_lds_sync();   // the next chunk overwrites the constants
    }
  } else {
    quotes(0, in.nq, 0);
  }
  const double tot = PAIR ? half_sum2(acc, acc_hi) : wave_sum(acc);
  const bool any_bad = PAIR ? half_any(bad) : __any(bad);
  return (any_bad || !(tot < kInf)) ? kInf : tot;
}

}  // namespace sabr
