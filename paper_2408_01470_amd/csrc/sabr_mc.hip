// sabr_mc.hip -- Monte Carlo pricer of caplets and swaptions under the Hagan
// SABR/LIBOR dynamics (Sec. 2.1: eqs. (dinamicasHagan1), (dinamicasHagan2)
// with their spot-measure drifts and the first unfixed index of eq. (h_t),
// the bank-account numeraire, the correlations of eqs. (rhoij), (thetaij),
// (phiij)): the pricer S_MC of the swaption cost (Sec. 3) and of Table
// (haganMCpricer).
//
// Scheme (the paper gives none): within each fixing interval [T_{j-1}, T_j)
// equal steps of at most dt; per step, with the alive forwards k >= j,
//   s_k = V_k max(F_k, 0)^beta_k,  d_i = tau_i s_i / (1 + tau_i F_i),
//   F_k <- max(F_k + s_k h sum_{i=j..k} rho_{k,i} d_i + s_k x_k, 0)      (Euler)
//   V_k <- V_k exp((sigma_k sum_{i=j..k} phi_{i,k} d_i - sigma_k^2/2) h
//                  + sigma_k x_{M+k})                                   (log-Euler)
// with x = sqrt(h) B xi, B the correlation factor of the plan (lower
// triangular with the alive forwards leading) and xi the step's first 2n
// normals, n = M - j alive forwards (Box-Muller of Philox4x32-10 blocks, two
// pairs a block from 32-bit uniforms, counter (block, step, path), key
// seed).  Both sums are O(M) recursions over the gaps:
// rho_{k,i} = eta1 + (1 - eta1) prod_{l=i+1..k} g1_l and phi_{i,k} =
// sgn(phi_i) sqrt|phi_i| sqrt|phi_k| prod_{l=i+1..k} g3_l, g = exp(-lambda
// (T_l - T_{l-1})).  At each fixing T_j the payoffs of the options expiring
// there are taken (payer swaption on forwards a..b-1, b = a + 1 the caplet)
// and the deflator is divided by 1 + tau_j F_j(T_j).
//
// Layout: one path per lane (2, 4 or 8 lanes per path when there are few
// paths), 4 waves per block; the forwards, their volatilities and the step's
// increments in registers (at most 24 forwards); the factor (column-major,
// rows by decreasing forward, W_k and Z_k interleaved) and the per-forward
// constants are wave-uniform and read through the scalar cache.  Logarithms,
// exponentials and the sine and cosine of the Box-Muller angle are the
// library's branch-free polynomial versions.  Each wave reduces its paths'
// payoffs and squares per option (register lane moves) into a slot of the
// workspace; a second kernel sums the slots in a fixed order, so prices do
// not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/sabr.h"
#include "sabr_device.hpp"
#include "sabr_mc_internal.h"

namespace sabr {
namespace {

constexpr int kMcMaxFwd = 24;
constexpr int kMcWavesPerBlock = 4;
constexpr int kMcReduceThreads = 256;

// Per-forward constants: rows of the plan image's forward table.
enum { MC_T, MC_TAU, MC_F0, MC_ALPHA, MC_BETA, MC_SIGMA, MC_PHS, MC_PHA, MC_G1, MC_G3, MC_ROWS };

struct McArgs {
  int M, n_opt, amax;
  long long n_paths;
  unsigned seed_lo, seed_hi;
  double eta1, P0;
  const double *fw;   // [MC_ROWS][M]
  const double *B;    // factor, column-major [2M][2M], rows W_k at 2k, Z_k at 2k + 1
  const int *opt_a, *opt_b, *opt_off;   // options grouped by expiry; opt_off [M + 1]
  const double *opt_K;
  double *part;       // [n_opt][2][n_waves]
  long long n_waves;
  int nst[kMcMaxFwd];
  double h[kMcMaxFwd], sh[kMcMaxFwd];
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011).
__device__ __forceinline__ void philox4x32_10(unsigned c0, unsigned c1, unsigned c2, unsigned c3,
                                              unsigned k0, unsigned k1, unsigned out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const unsigned hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const unsigned n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// log(x) for a positive x (method of log1p_tang with v = x exactly):
// x = 2^k m, m in [sqrt(1/2), sqrt(2)), f = m - 1, s = f/(2 + f),
// log m = f - s (f - s^2 P(s^2)).  Branch-free; 0 gives a finite garbage
// value that callers select away.
__device__ __forceinline__ double mc_log(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);
  int k = __builtin_amdgcn_frexp_exp(x);
  const bool up = m < M_SQRT1_2;
  m = up ? m + m : m;
  k = up ? k - 1 : k;
  const double f = m - 1.0;
  const double s = f * rcp_nr(2.0 + f);
  const double z = s * s;
  const double p = horner_s<kLog1pPoly, kLog1pDeg>(z);
  const double lf = fma(-s, fma(-z, p, f), f);
  const double kd = (double)k;
  return fma(kd, kLn2Hi, fma(kd, kLn2Lo, lf));
}

// Taylor coefficients of sin x / x and (cos x - 1) / x^2 in z = x^2, for
// |x| <= pi/4 (truncation below 2^-60 relative).
constexpr double inv_fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return 1.0 / f;
}
constexpr int kMcSinDeg = 8, kMcCosDeg = 8;
constexpr double kMcSinPoly[kMcSinDeg + 1] = {
    -inv_fact(3), inv_fact(5), -inv_fact(7), inv_fact(9), -inv_fact(11),
    inv_fact(13), -inv_fact(15), inv_fact(17), -inv_fact(19)};
constexpr double kMcCosPoly[kMcCosDeg + 1] = {
    -inv_fact(2), inv_fact(4), -inv_fact(6), inv_fact(8), -inv_fact(10),
    inv_fact(12), -inv_fact(14), inv_fact(16), -inv_fact(18)};

// (sin, cos)(2 pi u) for u in [0, 1): q = rint(4u) and r = u - q/4 (exact)
// give 2 pi u = 2 pi r + q pi/2 with |2 pi r| <= pi/4; the quadrant swaps
// and signs the pair.
__device__ __forceinline__ void mc_sincos_2pi(double u, double &sn, double &cs) {
  const double q = rint(4.0 * u);
  const double x = 6.283185307179586 * (u - 0.25 * q);
  const double z = x * x;
  const double sx = fma(x * z, horner_s<kMcSinPoly, kMcSinDeg>(z), x);
  const double cx = fma(z, horner_s<kMcCosPoly, kMcCosDeg>(z), 1.0);
  const int iq = (int)q & 3;
  const double a = (iq & 1) ? cx : sx, b = (iq & 1) ? sx : cx;
  sn = (iq & 2) ? -a : a;
  cs = ((iq + 1) & 2) ? -b : b;
}

// Sum of v over the LPP consecutive lanes of a group (LPP = 2: a pair; 4: a
// quad; 8: a half row), by register lane moves; every lane of the group
// ends with the same bits (each step adds two partial sums, in either
// order).
template <int LPP>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (LPP >= 2) v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  if constexpr (LPP >= 4) v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  if constexpr (LPP >= 8) v += dpp_d<0x141>(v);   // row_half_mirror
  return v;
}

// MF = the problem's forward count (one instantiation per count keeps every
// register index and loop bound static); LPP lanes per path: with few paths
// (LPP = 2, 4 or 8) lane g of a path's group draws the Philox blocks b = g,
// g + LPP, ... (normal pairs 2b and 2b + 1) and adds their factor columns
// (a copy of the factor in LDS) into its partial increments, the group sums
// them, and every lane of the group moves the same forwards.  Per step: the increments x of the alive
// rows are
// accumulated column by column (pair m of normals, columns 2m and 2m + 1 of
// the factor, stored column-major with rows W_k, Z_k interleaved), then the
// forwards move in increasing k with the drift recursions.
// Register budget: 4 waves per SIMD up to 13 forwards (measured faster on the
// paper's 13-forward market despite a few spilled registers), 3 up to 16, 2
// beyond.
template <int MF, int LPP>
__global__ __launch_bounds__(kWave *kMcWavesPerBlock, (MF <= 13 ? 4 : (MF <= 16 ? 3 : 2)))
void mc_kernel(McArgs a) {
  constexpr int MMAX = MF;
  constexpr int M = MF, n2 = 2 * MF;
  __shared__ double Bs[LPP > 1 ? n2 * n2 : 1];
  if constexpr (LPP > 1) {   // before any wave leaves: the barrier needs them all
    for (int i = threadIdx.x; i < n2 * n2; i += blockDim.x) Bs[i] = a.B[i];
    __syncthreads();
  }
  const int lane = lane_id();
  const long long wave = (long long)blockIdx.x * kMcWavesPerBlock + threadIdx.x / kWave;
  if (wave >= a.n_waves) return;   // whole waves only
  const int g = lane % LPP;
  const long long path = wave * (kWave / LPP) + lane / LPP;
  const bool live = path < a.n_paths;
  const double *__restrict__ fw = a.fw;
  const double *__restrict__ Bc = a.B;
  const double eta1 = a.eta1;

  double F[MMAX], V[MMAX];
#pragma unroll
  for (int k = 0; k < MMAX; ++k) {
    F[k] = k < M ? fw[MC_F0 * M + k] : 0.0;
    V[k] = k < M ? fw[MC_ALPHA * M + k] : 0.0;
  }
  double D = a.P0;
  unsigned step = 0;
  const unsigned p_lo = (unsigned)path, p_hi = (unsigned)((unsigned long long)path >> 32);

  for (int j = 0; j <= a.amax; ++j) {
    const int n = a.nst[j];
    const double h = a.h[j], sh = a.sh[j];
    for (int st = 0; st < n; ++st, ++step) {
      double x[2 * MMAX];
#pragma unroll
      for (int r = 0; r < 2 * MMAX; ++r) x[r] = 0.0;
      const int na = M - j;   // alive forwards: pairs 0..na-1, rows 0..2na-1
      // normal pair m from words (wa, wb): its two factor columns into x
      // (lower triangular: rows 2m..2na-1)
      auto pair = [&](int m, unsigned wa, unsigned wb) {
        const double u1 = ((double)wa + 1.0) * 0x1.0p-32;
        const double u2 = (double)wb * 0x1.0p-32;
        const double rr = sqrt_gs(-2.0 * mc_log(u1));
        double sn, cs;
        mc_sincos_2pi(u2, sn, cs);
        const double z0 = u1 < 1.0 ? rr * cs : 0.0, z1 = u1 < 1.0 ? rr * sn : 0.0;
        const double *c0 = (LPP > 1 ? Bs : Bc) + (size_t)(2 * m) * n2, *c1 = c0 + n2;
#pragma unroll
        for (int r = 0; r < 2 * MMAX; ++r)
          if (r >= 2 * m && r < 2 * na) x[r] = fma(c1[r], z1, fma(c0[r], z0, x[r]));
      };
      constexpr int NB = (M + 1) / 2;   // Philox blocks a step at most: two pairs each
      const int nb = (na + 1) / 2;
      for (int i = 0; i < (NB + LPP - 1) / LPP; ++i) {
        const int b = i * LPP + g;
        if (b < nb) {
          unsigned w[4];
          philox4x32_10((unsigned)b, step, p_lo, p_hi, a.seed_lo, a.seed_hi, w);
          pair(2 * b, w[0], w[1]);
          if (2 * b + 1 < na) pair(2 * b + 1, w[2], w[3]);
        }
      }
      if constexpr (LPP > 1) {
#pragma unroll
        for (int r = 0; r < 2 * MMAX; ++r)
          if (r < 2 * na) x[r] = group_sum<LPP>(x[r]);
      }
      double Ds = 0.0, E = 0.0, G = 0.0;
#pragma unroll
      for (int k = 0; k < MMAX; ++k) {
        if (k >= j && k < M) {
          const double f = F[k], v = V[k];
          const double tk = fw[MC_TAU * M + k], bk = fw[MC_BETA * M + k];
          const double fp = fmax(f, 0.0);
          double fb;   // F^beta; beta is wave-uniform: a scalar branch
          if (bk == 0.5)
            fb = fp > 0.0 ? sqrt_gs(fp) : 0.0;
          else if (bk == 1.0)
            fb = fp;
          else
            fb = fp > 0.0 ? exp_cw(bk * mc_log(fp)) : (bk == 0.0 ? 1.0 : 0.0);
          const double s = v * fb;
          const double d = tk * s * rcp_nr(fma(tk, f, 1.0));
          Ds += d;
          E = fma(fw[MC_G1 * M + k], E, d);
          G = fma(fw[MC_G3 * M + k], G, fw[MC_PHS * M + k] * d);
          const double sg = fw[MC_SIGMA * M + k];
          const int pk = 2 * (M - 1 - k);   // this forward's rows
          F[k] = fmax(f + s * (eta1 * Ds + (1.0 - eta1) * E) * h + s * (sh * x[pk]), 0.0);
          V[k] = v * exp_cw((sg * fw[MC_PHA * M + k] * G - 0.5 * sg * sg) * h +
                            sg * (sh * x[pk + 1]));
        }
      }
    }
    // fixing of F_j: the options expiring at T_j, then the deflator
    for (int o = a.opt_off[j]; o < a.opt_off[j + 1]; ++o) {
      const int ob = a.opt_b[o];
      const double K = a.opt_K[o];
      double Pb = 1.0, A = 0.0;
#pragma unroll
      for (int i = 0; i < MMAX; ++i) {
        if (i >= j && i < ob) {
          Pb /= (1.0 + fw[MC_TAU * M + i] * F[i]);
          A += fw[MC_TAU * M + i] * Pb;
        }
      }
      const double xo = (live && g == 0) ? D * fmax(1.0 - Pb - K * A, 0.0) : 0.0;
      const double s1 = wave_sum(xo), s2 = wave_sum(xo * xo);
      if (lane == 0) {
        a.part[(2 * (long long)o) * a.n_waves + wave] = s1;
        a.part[(2 * (long long)o + 1) * a.n_waves + wave] = s2;
      }
    }
    double Fj = 0.0;
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
      if (i == j) Fj = F[i];
    D /= (1.0 + fw[MC_TAU * M + j] * Fj);
  }
}

// Mean and standard error per option: block o sums its slots in a fixed
// order (strided partial sums, then a tree).
__global__ __launch_bounds__(kMcReduceThreads) void mc_reduce_kernel(const double *part,
                                                                     long long n_waves,
                                                                     long long n_paths,
                                                                     const int *ext,
                                                                     double *price, double *se) {
  __shared__ double s1[kMcReduceThreads], s2[kMcReduceThreads];
  const int o = blockIdx.x, t = threadIdx.x;
  const double *p1 = part + (2 * (long long)o) * n_waves, *p2 = p1 + n_waves;
  double a = 0.0, b = 0.0;
  for (long long w = t; w < n_waves; w += kMcReduceThreads) {
    a += p1[w];
    b += p2[w];
  }
  s1[t] = a;
  s2[t] = b;
  __syncthreads();
  for (int w = kMcReduceThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      s1[t] += s1[t + w];
      s2[t] += s2[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double n = (double)n_paths;
    const double mean = s1[0] / n;
    double var = n > 1.0 ? (s2[0] - s1[0] * mean) / (n - 1.0) : 0.0;
    if (!(var > 0.0)) var = 0.0;
    price[ext[o]] = mean;
    if (se) se[ext[o]] = sqrt(var / n);
  }
}

// The swaption cost of Sec. 3 over the options' prices: sum_o w_o (price_o -
// target_o)^2 (w = 1 without weights), one block, a fixed order.
__global__ __launch_bounds__(kMcReduceThreads) void mc_cost_kernel(const double *price,
                                                                   const double *target,
                                                                   const double *weight, int n,
                                                                   double *cost) {
  __shared__ double s1[kMcReduceThreads];
  const int t = threadIdx.x;
  double a = 0.0;
  for (int o = t; o < n; o += kMcReduceThreads) {
    const double r = price[o] - target[o];
    a += (weight ? weight[o] : 1.0) * r * r;
  }
  s1[t] = a;
  __syncthreads();
  for (int w = kMcReduceThreads / 2; w > 0; w >>= 1) {
    if (t < w) s1[t] += s1[t + w];
    __syncthreads();
  }
  if (t == 0) cost[0] = s1[0];
}

// ---------------------------------------------------------------------------
// Host: the correlation factor.  The 2M x 2M matrix of eqs. (rhoij),
// (thetaij), (phiij) (rows W_0..W_{M-1}, Z_0..Z_{M-1}; entry (k, M + l) =
// phi_{k,l} = E[dW_k dZ_l]) need not be positive semi-definite (the paper's
// calibrated Hagan parameters give an indefinite one); it is repaired
// spectrally (Rebonato and Jaeckel, 1999: eigenvalues clipped at zero, unit
// diagonal restored), and the factor is the Cholesky factor of the repaired
// matrix with the components ordered W_{M-1}, Z_{M-1}, ..., W_0, Z_0, so
// that the forwards alive after a fixing are a leading block drawing on the
// first normals only.  Eigen-decomposition by cyclic Jacobi rotations
// (Rutishauser's formulation).
// ---------------------------------------------------------------------------
void corr_matrix(int M, const double *T, const double *phi, const double y[5], double *C) {
  const int n = 2 * M;
  for (int k = 0; k < M; ++k)
    for (int l = 0; l < M; ++l) {
      const double dT = std::fabs(T[k] - T[l]);
      C[k * n + l] = y[0] + (1.0 - y[0]) * std::exp(-y[1] * dT);
      C[(M + k) * n + (M + l)] = y[2] + (1.0 - y[2]) * std::exp(-y[3] * dT);
      const double sg = phi[k] > 0.0 ? 1.0 : (phi[k] < 0.0 ? -1.0 : 0.0);
      const double ph = sg * std::sqrt(std::fabs(phi[k] * phi[l])) * std::exp(-y[4] * dT);
      C[k * n + (M + l)] = ph;
      C[(M + l) * n + k] = ph;
    }
}

void jacobi_eigen(int n, std::vector<double> A, std::vector<double> &lam, std::vector<double> &Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        tot += A[(size_t)p * n + q] * A[(size_t)p * n + q];
        if (p != q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
      }
    if (off <= 1e-34 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) /
                         (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c, tau = s / (1.0 + c);
        A[(size_t)p * n + p] = app - t * apq;
        A[(size_t)q * n + q] = aqq + t * apq;
        A[(size_t)p * n + q] = A[(size_t)q * n + p] = 0.0;
        for (int r = 0; r < n; ++r) {
          if (r == p || r == q) continue;
          const double arp = A[(size_t)r * n + p], arq = A[(size_t)r * n + q];
          const double nrp = arp - s * (arq + tau * arp), nrq = arq + s * (arp - tau * arq);
          A[(size_t)r * n + p] = A[(size_t)p * n + r] = nrp;
          A[(size_t)r * n + q] = A[(size_t)q * n + r] = nrq;
        }
        for (int r = 0; r < n; ++r) {
          const double qrp = Q[(size_t)r * n + p], qrq = Q[(size_t)r * n + q];
          Q[(size_t)r * n + p] = qrp - s * (qrq + tau * qrp);
          Q[(size_t)r * n + q] = qrq + s * (qrp - tau * qrq);
        }
      }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = A[(size_t)i * n + i];
}

void corr_factor(int M, const double *T, const double *phi, const double y[5], double *B) {
  const int n = 2 * M;
  std::vector<double> C((size_t)n * n), lam, Q;
  corr_matrix(M, T, phi, y, C.data());
  jacobi_eigen(n, C, lam, Q);
  // the repaired matrix Q max(Lambda, 0) Q^T at unit diagonal
  std::vector<double> R((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      double acc = 0.0;
      for (int e = 0; e < n; ++e)
        acc += Q[(size_t)r * n + e] * std::max(lam[e], 0.0) * Q[(size_t)c * n + e];
      R[(size_t)r * n + c] = acc;
    }
  std::vector<double> d(n);
  for (int r = 0; r < n; ++r) {
    const double v = std::sqrt(R[(size_t)r * n + r]);
    d[r] = v > 0.0 ? v : 1.0;
  }
  // Cholesky in the order W_{M-1}, Z_{M-1}, ..., W_0, Z_0 (semi-definite: a
  // pivot at or below 1e-9 leaves its column zero; the zero pivots of a
  // clipped spectrum come out as rounding noise of order 1e-12)
  std::vector<int> rows(n);
  for (int k = M - 1, p = 0; k >= 0; --k) {
    rows[p++] = k;
    rows[p++] = M + k;
  }
  std::vector<double> L((size_t)n * n, 0.0);
  auto A = [&](int p, int q) {
    return R[(size_t)rows[p] * n + rows[q]] / (d[rows[p]] * d[rows[q]]);
  };
  for (int c = 0; c < n; ++c) {
    double dd = A(c, c);
    for (int i = 0; i < c; ++i) dd -= L[(size_t)c * n + i] * L[(size_t)c * n + i];
    if (dd <= 1e-9) continue;
    const double lc = std::sqrt(dd);
    L[(size_t)c * n + c] = lc;
    for (int r = c + 1; r < n; ++r) {
      double v = A(r, c);
      for (int i = 0; i < c; ++i) v -= L[(size_t)r * n + i] * L[(size_t)c * n + i];
      L[(size_t)r * n + c] = v / lc;
    }
  }
  for (int p = 0; p < n; ++p)
    for (int c = 0; c < n; ++c) B[(size_t)rows[p] * n + c] = L[(size_t)p * n + c];
}

}  // namespace

// Lanes per path: with few paths a path's normal pairs spread over a quad or
// a row of lanes, so more waves share the steps' latency.
int mc_lanes_per_path(int M, long long n_paths) {
  const int nb = (M + 1) / 2;   // Philox blocks a step
  if (n_paths <= 4096 && nb >= 5) return 8;
  if (n_paths <= 16384 && nb >= 3) return 4;
  if (n_paths <= 131072 && nb >= 2) return 2;
  return 1;
}

}  // namespace sabr

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
struct sabr_mc_plan {
  int M = 0, n_opt = 0, amax = 0;
  double eta1 = 0.0, P0 = 0.0;
  std::vector<double> T;          // fixing times (host copy, for the step grid)
  std::vector<double> B;          // factor [2M][2M], rows W_0..W_{M-1}, Z_0..Z_{M-1}
  std::vector<double> img_d;      // fw [MC_ROWS][M], B [2M][2M], opt_K [n_opt]
  std::vector<int> img_i;         // opt_a, opt_b [n_opt], opt_off [M + 1], ext [n_opt]
  size_t off_B = 0, off_K = 0;    // in doubles
  size_t off_a = 0, off_b = 0, off_off = 0, off_ext = 0;   // in ints
  void *dev = nullptr;            // caller-owned image
  size_t dev_bytes = 0;
};

namespace {

bool is_fin(double v) { return std::isfinite(v); }

size_t image_bytes(const sabr_mc_plan *p) {
  return p->img_d.size() * sizeof(double) + p->img_i.size() * sizeof(int);
}

}  // namespace

extern "C" {

sabr_status sabr_mc_plan_create(const sabr_mc_problem *pr, sabr_mc_plan **out) {
  using namespace sabr;
  if (!pr || !out) return mc_fail(SABR_EINVAL, "null argument");
  *out = nullptr;
  const int M = pr->n_fwd;
  if (M < 1 || M > kMcMaxFwd)
    return mc_fail(SABR_EINVAL, "mc: n_fwd must be 1.." + std::to_string(kMcMaxFwd));
  if (!pr->T || !pr->tau || !pr->F0 || !pr->alpha || !pr->beta || !pr->phi || !pr->sigma)
    return mc_fail(SABR_EINVAL, "mc: null forward array");
  for (int k = 0; k < M; ++k) {
    const double prev = k > 0 ? pr->T[k - 1] : 0.0;
    if (!is_fin(pr->T[k]) || !(pr->T[k] > prev))
      return mc_fail(SABR_EINVAL, "mc: fixing times must be positive and increasing");
    if (!is_fin(pr->tau[k]) || !(pr->tau[k] > 0.0) || !is_fin(pr->F0[k]) || !(pr->F0[k] > 0.0) ||
        !is_fin(pr->alpha[k]) || !(pr->alpha[k] > 0.0))
      return mc_fail(SABR_EINVAL, "mc: tau, F0 and alpha must be positive");
    if (!(pr->beta[k] >= 0.0 && pr->beta[k] <= 1.0))
      return mc_fail(SABR_EINVAL, "mc: beta outside [0, 1]");
    if (!(std::fabs(pr->phi[k]) <= 1.0)) return mc_fail(SABR_EINVAL, "mc: |phi_ii| > 1");
    if (!is_fin(pr->sigma[k]) || !(pr->sigma[k] >= 0.0))
      return mc_fail(SABR_EINVAL, "mc: sigma must be >= 0");
  }
  const double y[5] = {pr->eta1, pr->lambda1, pr->eta2, pr->lambda2, pr->lambda3};
  if (!(y[0] >= 0.0 && y[0] <= 1.0) || !(y[2] >= 0.0 && y[2] <= 1.0))
    return mc_fail(SABR_EINVAL, "mc: eta1 and eta2 must lie in [0, 1]");
  if (!(y[1] >= 0.0) || !(y[3] >= 0.0) || !(y[4] >= 0.0) || !is_fin(y[1]) || !is_fin(y[3]) ||
      !is_fin(y[4]))
    return mc_fail(SABR_EINVAL, "mc: lambdas must be finite and >= 0");
  if (!is_fin(pr->P0) || !(pr->P0 > 0.0)) return mc_fail(SABR_EINVAL, "mc: P0 must be positive");
  const int n_opt = pr->n_opt;
  if (n_opt < 1) return mc_fail(SABR_EINVAL, "mc: need at least one option");
  if (!pr->opt_a || !pr->opt_b || !pr->opt_K) return mc_fail(SABR_EINVAL, "mc: null option array");
  int amax = 0;
  for (int o = 0; o < n_opt; ++o) {
    if (pr->opt_a[o] < 0 || pr->opt_b[o] <= pr->opt_a[o] || pr->opt_b[o] > M)
      return mc_fail(SABR_EINVAL, "mc: option " + std::to_string(o) + " needs 0 <= a < b <= n_fwd");
    if (!is_fin(pr->opt_K[o])) return mc_fail(SABR_EINVAL, "mc: option strike not finite");
    amax = std::max(amax, pr->opt_a[o]);
  }
  sabr_mc_plan *P = new (std::nothrow) sabr_mc_plan;
  if (!P) return mc_fail(SABR_ENOMEM, "out of host memory");
  P->M = M;
  P->n_opt = n_opt;
  P->amax = amax;
  P->eta1 = y[0];
  P->P0 = pr->P0;
  P->T.assign(pr->T, pr->T + M);
  const int n2 = 2 * M;
  P->off_B = (size_t)MC_ROWS * M;
  P->off_K = P->off_B + (size_t)n2 * n2;
  P->img_d.assign(P->off_K + n_opt, 0.0);
  double *fw = P->img_d.data();
  for (int k = 0; k < M; ++k) {
    fw[MC_T * M + k] = pr->T[k];
    fw[MC_TAU * M + k] = pr->tau[k];
    fw[MC_F0 * M + k] = pr->F0[k];
    fw[MC_ALPHA * M + k] = pr->alpha[k];
    fw[MC_BETA * M + k] = pr->beta[k];
    fw[MC_SIGMA * M + k] = pr->sigma[k];
    const double ap = std::sqrt(std::fabs(pr->phi[k]));
    fw[MC_PHS * M + k] = pr->phi[k] > 0.0 ? ap : (pr->phi[k] < 0.0 ? -ap : 0.0);
    fw[MC_PHA * M + k] = ap;
    const double gap = k > 0 ? pr->T[k] - pr->T[k - 1] : 0.0;
    fw[MC_G1 * M + k] = std::exp(-y[1] * gap);
    fw[MC_G3 * M + k] = std::exp(-y[4] * gap);
  }
  P->B.assign((size_t)n2 * n2, 0.0);
  corr_factor(M, pr->T, pr->phi, y, P->B.data());
  // device layout: column-major, rows by decreasing forward (W_k at
  // 2(M - 1 - k), Z_k at 2(M - 1 - k) + 1): the alive rows lead
  for (int c = 0; c < n2; ++c)
    for (int k = 0; k < M; ++k) {
      const int pos = 2 * (M - 1 - k);
      P->img_d[P->off_B + (size_t)c * n2 + pos] = P->B[(size_t)k * n2 + c];
      P->img_d[P->off_B + (size_t)c * n2 + pos + 1] = P->B[(size_t)(M + k) * n2 + c];
    }
  // options grouped by expiry (stable), outputs back to the caller's order
  std::vector<int> ord(n_opt);
  for (int o = 0; o < n_opt; ++o) ord[o] = o;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int x, int z) { return pr->opt_a[x] < pr->opt_a[z]; });
  P->off_a = 0;
  P->off_b = n_opt;
  P->off_off = 2 * (size_t)n_opt;
  P->off_ext = P->off_off + M + 1;
  P->img_i.assign(P->off_ext + n_opt, 0);
  std::vector<int> cnt(M + 1, 0);
  for (int i = 0; i < n_opt; ++i) {
    const int o = ord[i];
    P->img_i[P->off_a + i] = pr->opt_a[o];
    P->img_i[P->off_b + i] = pr->opt_b[o];
    P->img_d[P->off_K + i] = pr->opt_K[o];
    P->img_i[P->off_ext + i] = o;
    cnt[pr->opt_a[o] + 1] += 1;
  }
  for (int j = 0; j < M; ++j) cnt[j + 1] += cnt[j];
  for (int j = 0; j <= M; ++j) P->img_i[P->off_off + j] = cnt[j];
  *out = P;
  return SABR_OK;
}

void sabr_mc_plan_destroy(sabr_mc_plan *plan) { delete plan; }

size_t sabr_mc_plan_device_bytes(const sabr_mc_plan *plan) { return plan ? image_bytes(plan) : 0; }

sabr_status sabr_mc_plan_upload(sabr_mc_plan *plan, void *dev_buf, size_t bytes, void *stream) {
  using namespace sabr;
  if (!plan || !dev_buf) return mc_fail(SABR_EINVAL, "null argument");
  const size_t need = image_bytes(plan);
  if (bytes < need) return mc_fail(SABR_EWORKSPACE, "mc: plan buffer too small");
  if (reinterpret_cast<uintptr_t>(dev_buf) % 8 != 0)
    return mc_fail(SABR_EINVAL, "mc: plan buffer must be 8-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t nd = plan->img_d.size() * sizeof(double);
  hipError_t e = hipMemcpyAsync(dev_buf, plan->img_d.data(), nd, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(static_cast<char *>(dev_buf) + nd, plan->img_i.data(),
                       plan->img_i.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return mc_hip_fail(e, "mc plan upload");
  plan->dev = dev_buf;
  plan->dev_bytes = need;
  return SABR_OK;
}

sabr_status sabr_mc_factor(const sabr_mc_plan *plan, double *B) {
  using namespace sabr;
  if (!plan || !B) return mc_fail(SABR_EINVAL, "null argument");
  const size_t n2 = 2 * (size_t)plan->M;
  std::copy(plan->B.begin(), plan->B.begin() + n2 * n2, B);
  return SABR_OK;
}

size_t sabr_mc_workspace_size(const sabr_mc_plan *plan, int64_t n_paths) {
  if (!plan || n_paths < 1 || n_paths > (int64_t(1) << 38)) return 0;
  const long long lanes = n_paths * sabr::mc_lanes_per_path(plan->M, n_paths);
  const long long n_waves = (lanes + sabr::kWave - 1) / sabr::kWave;
  // per-wave partial sums, then one price per option (used by sabr_mc_cost)
  return ((size_t)plan->n_opt * 2 * (size_t)n_waves + (size_t)plan->n_opt) * sizeof(double);
}

sabr_status sabr_mc_price(const sabr_mc_plan *plan, int64_t n_paths, double dt, uint64_t seed,
                          double *price, double *stderr_out, void *workspace, size_t ws_bytes,
                          void *stream) {
  using namespace sabr;
  if (!plan || !price) return mc_fail(SABR_EINVAL, "null argument");
  if (!plan->dev) return mc_fail(SABR_EINVAL, "mc: plan not uploaded");
  // 2^38 paths = 2^32 waves = 2^30 blocks of four waves: within one grid dimension
  if (n_paths < 1 || n_paths > (int64_t(1) << 38))
    return mc_fail(SABR_EINVAL, "mc: n_paths must be 1..2^38");
  if (!is_fin(dt) || !(dt > 0.0)) return mc_fail(SABR_EINVAL, "mc: dt must be positive");
  const size_t need = sabr_mc_workspace_size(plan, n_paths);
  if (!workspace || ws_bytes < need) return mc_fail(SABR_EWORKSPACE, "mc: workspace too small");
  McArgs a{};
  a.M = plan->M;
  a.n_opt = plan->n_opt;
  a.amax = plan->amax;
  a.n_paths = n_paths;
  a.seed_lo = (unsigned)seed;
  a.seed_hi = (unsigned)(seed >> 32);
  a.eta1 = plan->eta1;
  a.P0 = plan->P0;
  double total = 0.0;
  for (int j = 0; j <= plan->amax; ++j) {
    const double len = plan->T[j] - (j > 0 ? plan->T[j - 1] : 0.0);
    const double n = std::ceil(len / dt);
    total += n < 1.0 ? 1.0 : n;
    if (total > 2147483647.0) return mc_fail(SABR_EINVAL, "mc: more than 2^31 time steps");
    a.nst[j] = n < 1.0 ? 1 : (int)n;
    a.h[j] = len / a.nst[j];
    a.sh[j] = std::sqrt(a.h[j]);
  }
  const double *dd = static_cast<const double *>(plan->dev);
  const int *di = reinterpret_cast<const int *>(dd + plan->img_d.size());
  a.fw = dd;
  a.B = dd + plan->off_B;
  a.opt_K = dd + plan->off_K;
  a.opt_a = di + plan->off_a;
  a.opt_b = di + plan->off_b;
  a.opt_off = di + plan->off_off;
  a.part = static_cast<double *>(workspace);
  const int lpp = mc_lanes_per_path(plan->M, n_paths);
  a.n_waves = (n_paths * lpp + kWave - 1) / kWave;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long blocks = (a.n_waves + kMcWavesPerBlock - 1) / kMcWavesPerBlock;
  switch (plan->M) {
#define SABR_MC_LAUNCH(N, L)                                                                   \
  hipLaunchKernelGGL((mc_kernel<N, L>), dim3((unsigned)blocks), dim3(kWave * kMcWavesPerBlock), \
                     0, s, a)
#define SABR_MC_CASE(N)                                                \
  case N:                                                              \
    if (N >= 9 && lpp == 8) SABR_MC_LAUNCH(N, (N >= 9 ? 8 : 1));       \
    else if (N >= 5 && lpp == 4) SABR_MC_LAUNCH(N, (N >= 5 ? 4 : 1));  \
    else if (N >= 3 && lpp == 2) SABR_MC_LAUNCH(N, (N >= 3 ? 2 : 1));  \
    else SABR_MC_LAUNCH(N, 1);                                         \
    break;
    SABR_MC_CASE(1) SABR_MC_CASE(2) SABR_MC_CASE(3) SABR_MC_CASE(4) SABR_MC_CASE(5)
    SABR_MC_CASE(6) SABR_MC_CASE(7) SABR_MC_CASE(8) SABR_MC_CASE(9) SABR_MC_CASE(10)
    SABR_MC_CASE(11) SABR_MC_CASE(12) SABR_MC_CASE(13) SABR_MC_CASE(14) SABR_MC_CASE(15)
    SABR_MC_CASE(16) SABR_MC_CASE(17) SABR_MC_CASE(18) SABR_MC_CASE(19) SABR_MC_CASE(20)
    SABR_MC_CASE(21) SABR_MC_CASE(22) SABR_MC_CASE(23) SABR_MC_CASE(24)
#undef SABR_MC_CASE
#undef SABR_MC_LAUNCH
    default: return mc_fail(SABR_EINVAL, "mc: bad forward count");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mc_hip_fail(e, "mc kernel launch");
  hipLaunchKernelGGL(mc_reduce_kernel, dim3(plan->n_opt), dim3(kMcReduceThreads), 0, s, a.part,
                     a.n_waves, (long long)n_paths, di + plan->off_ext, price, stderr_out);
  e = hipGetLastError();
  if (e != hipSuccess) return mc_hip_fail(e, "mc reduce launch");
  return SABR_OK;
}

sabr_status sabr_mc_cost(const sabr_mc_plan *plan, int64_t n_paths, double dt, uint64_t seed,
                         const double *target, const double *weight, double *price,
                         double *cost, void *workspace, size_t ws_bytes, void *stream) {
  using namespace sabr;
  if (!plan || !target || !cost) return mc_fail(SABR_EINVAL, "null argument");
  const size_t need = sabr_mc_workspace_size(plan, n_paths);
  if (need == 0) return mc_fail(SABR_EINVAL, "mc: n_paths must be 1..2^38");
  if (!workspace || ws_bytes < need) return mc_fail(SABR_EWORKSPACE, "mc: workspace too small");
  double *p = price ? price
                    : reinterpret_cast<double *>(static_cast<char *>(workspace) + need) -
                          plan->n_opt;
  const sabr_status st =
      sabr_mc_price(plan, n_paths, dt, seed, p, nullptr, workspace, ws_bytes, stream);
  if (st != SABR_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(mc_cost_kernel, dim3(1), dim3(kMcReduceThreads), 0, s, p, target, weight,
                     plan->n_opt, cost);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mc_hip_fail(e, "mc cost launch");
  return SABR_OK;
}

}  // extern "C"
