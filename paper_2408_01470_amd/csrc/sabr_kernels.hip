// sabr_kernels.hip -- HIP kernels of the SA calibrator for gfx950.
//
// Mapping: one 64-lane wavefront evaluates one parameter point (one Markov
// chain) with its lanes spread over the market's quotes; the per-quote
// squared errors are summed per lane and reduced across the wave.  The
// FP64 vector ALU bounds every kernel here (no dense contraction: no MFMA).
#include <hip/hip_runtime.h>

#include "sabr_internal.hpp"

namespace sabr {

namespace {

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

struct WaveLds {
  double *al, *nv, *g1, *g2;  // per forward
  double *ta, *tr, *tn, *tq;  // per underlying
  double *lk;                 // per-lane recursion column
};

__device__ __forceinline__ WaveLds wave_lds(const DevMarket &m, double *base) {
  WaveLds w;
  w.al = base;
  w.nv = w.al + m.max_nf;
  w.g1 = w.nv + m.max_nf;
  w.g2 = w.g1 + m.max_nf;
  w.ta = w.g2 + m.max_nf;
  w.tr = w.ta + m.max_nu;
  w.tn = w.tr + m.max_nu;
  w.tq = w.tn + m.max_nu;
  w.lk = w.tq + m.max_nu;
  return w;
}

// LMM12 parameter map of one point into the wave's LDS.  Returns true when
// the point lies outside the model's domain (wave-uniform).
//   alpha_k = (a + b T_k) e^{-c T_k} + d, nu_k likewise (abcd forms);
//   rho_kl = exp(-lambda1 |T_k - T_l|) = product of per-gap factors g1,
//   theta_kl = eta2 + (1 - eta2) exp(-lambda2 |T_k - T_l|), phi_kl = rho.
// Swap of forwards [e, e+n) with a_k = u_k alpha_k (u_k = tau_k P_k F_k^b / A):
//   R_k = sum_l a_l rho_kl (forward and backward recursions, O(n)),
//   V = sum a_k R_k, b_k = a_k R_k nu_k,
//   Nb = eta2 (sum b)^2 + (1 - eta2) sum_kl b_k b_l exp(-lambda2 |dT|),
//   alpha_S = sqrt(V)/S0^b, nu_S = sqrt(Nb)/V,
//   rho_S = rho (sum a)(sum b) / (sqrt(V) sqrt(Nb))   (0 if Nb = 0).
__device__ bool lmm12_map(const DevMarket &m, const DevInst &in, const double *p, WaveLds w) {
  const int lane = lane_id();
  const double a = p[0], b = p[1], c = p[2], d = p[3];
  const double an = p[4], bn = p[5], cn = p[6], dn = p[7];
  const double rho = p[8], lam1 = p[9], eta2 = p[10], lam2 = p[11];
  bool bad = !(fabs(rho) < 1.0) || !(lam1 >= 0.0) || !(lam2 >= 0.0) ||
             !(eta2 >= 0.0 && eta2 <= 1.0);
  for (int k = lane; k < in.nf; k += kWave) {
    const double T = m.f_T[in.f0 + k];
    w.al[k] = (a + b * T) * exp(-(c * T)) + d;
    w.nv[k] = (an + bn * T) * exp(-(cn * T)) + dn;
    if (k + 1 < in.nf) {
      const double dT = m.f_T[in.f0 + k + 1] - T;
      w.g1[k] = exp(-(lam1 * dT));
      w.g2[k] = exp(-(lam2 * dT));
    }
  }
  wave_lds_sync();
  double *lk = w.lk + lane;
  for (int u = lane; u < in.nu; u += kWave) {
    const int e = m.u_first[in.u0 + u];
    const int n = m.u_len[in.u0 + u];
    for (int k = e; k < e + n; ++k) bad |= !(w.al[k] > 0.0) || !(w.nv[k] >= 0.0);
    double ta, tr, tn;
    if (n == 1) {
      ta = w.al[e];
      tr = rho;
      tn = w.nv[e];
    } else {
      const double invA = m.u_invA[in.u0 + u];
      const double S0b = m.u_S0b[in.u0 + u];
      const double *v = m.f_v + in.f0;
      double Lacc = 0.0, suma = 0.0;
      for (int j = 0; j < n; ++j) {
        const int k = e + j;
        const double aj = v[k] * invA * w.al[k];
        lk[j * kWave] = Lacc;
        suma += aj;
        Lacc = w.g1[k] * (Lacc + aj);
      }
      double Rr = 0.0, Rb = 0.0, V = 0.0, Sb = 0.0, Sbb = 0.0;
      for (int j = n - 1; j >= 0; --j) {
        const int k = e + j;
        const double aj = v[k] * invA * w.al[k];
        const double Rj = lk[j * kWave] + aj + Rr;
        const double ar = aj * Rj;
        V += ar;
        const double bj = ar * w.nv[k];
        Sb += bj;
        Sbb += bj * (bj + 2.0 * Rb);
        if (j > 0) {
          Rr = w.g1[k - 1] * (Rr + aj);
          Rb = w.g2[k - 1] * (Rb + bj);
        }
      }
      const double Nb = eta2 * Sb * Sb + (1.0 - eta2) * Sbb;
      const double sV = sqrt(V), sN = sqrt(Nb);
      ta = sV / S0b;
      tn = sN / V;
      tr = (sN > 0.0) ? rho * suma * Sb / (sV * sN) : 0.0;
      bad |= !(V > 0.0) || !(fabs(tr) < 1.0);
    }
    w.ta[u] = ta;
    w.tr[u] = tr;
    w.tn[u] = tn;
    w.tq[u] = tn / ta;
  }
  wave_lds_sync();
  return __any(bad);
}

// Cost of one point for the wave: f = sum_q w_q (m_q - mkt_q)^2, +inf on a
// domain failure.  Optional per-quote residual and model outputs.
template <int MODEL, int FORMULA, int RESID>
__device__ double point_cost(const DevMarket &m, int inst, const double *p, WaveLds w,
                             double *resid, double *model) {
  const DevInst in = m.inst[inst];
  const int lane = lane_id();
  bool bad = false;
  SabrConst g{};
  if (MODEL == 0) {
    bad = !(p[0] > 0.0) || !(p[1] >= 0.0 && p[1] <= 1.0) || !(fabs(p[2]) < 1.0) ||
          !(p[3] >= 0.0);
    g = sabr_const(p[0], p[1], p[2], p[3]);
  } else {
    bad = lmm12_map(m, in, p, w);
  }
  const double beta = (MODEL == 0) ? p[1] : m.beta;
  double acc = 0.0;
  for (int q = lane; q < in.nq; q += kWave) {
    const int gq = in.q0 + q;
    const double L = m.q_L[gq];
    const double T = m.q_T[gq];
    SabrConst k;
    double qv = 1.0, D1 = 1.0, fp = 1.0;
    if (MODEL == 0) {
      k = g;
      if (FORMULA == 0) {
        qv = exp(0.5 * k.omb * m.q_lfk[gq]);
        D1 = d1_term(k.omb2, L);
      } else {
        fp = exp(k.omb * m.q_lnf[gq]);
      }
    } else {
      const int u = m.q_und[gq];
      k = sabr_const(w.ta[u], beta, w.tr[u], w.tn[u]);
      k.nua = w.tq[u];
      if (FORMULA == 0) {
        qv = m.q_qfix[gq];
        D1 = m.q_D1fix[gq];
      } else {
        fp = m.q_fpfix[gq];
      }
    }
    const double sig = (FORMULA == 0) ? hagan2002(k, L, qv, D1, T) : paper_eq3(k, L, fp);
    bad |= !(sig > 0.0) || !(fabs(sig) < kInf);
    double mv = sig;
    if (RESID == 1) {
      const double f = m.q_f[gq], K = m.q_K[gq], D = m.q_D[gq];
      mv = black_otm(f, K, L, m.q_sqrtT[gq], sig, D);
      bad |= !(fabs(mv) < kInf);
      if (model) {
        const double sh = parity_shift(m.q_kind[gq], f, K, L, D);
        model[q] = sh == 0.0 ? mv : mv + sh;
      }
    } else if (model) {
      model[q] = mv;
    }
    const double r = mv - m.q_tgt[gq];
    acc += m.q_w[gq] * r * r;
    if (resid) resid[q] = r;
  }
  const double tot = wave_sum(acc);
  const bool any_bad = __any(bad);
  return (any_bad || !(tot < kInf)) ? kInf : tot;
}

// ---------------------------------------------------------------------------
// Market precompute (market-only quantities, once per upload).
// ---------------------------------------------------------------------------
__global__ void prep_kernel(DevMarket m, double *q_tgt, double *q_w, double *q_L, double *q_lfk,
                            double *q_lnf, double *q_sqrtT, double *q_qfix, double *q_D1fix,
                            double *q_fpfix, double *f_v, double *u_S0b, const double *q_vol,
                            const double *q_wuser, const double *f_tauP, const double *f_F,
                            int n_q, int n_f, int n_u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double beta = m.beta, omb = 1.0 - beta;
  if (i < n_f) f_v[i] = f_tauP[i] * pow(f_F[i], beta);
  if (i < n_u) u_S0b[i] = pow(m.u_S0[i], beta);
  if (i >= n_q) return;
  const double f = m.q_f[i], K = m.q_K[i], T = m.q_T[i];
  const double L = log(f / K);
  const double sT = sqrt(T);
  q_L[i] = L;
  q_lfk[i] = log(f * K);
  q_lnf[i] = log(f);
  q_sqrtT[i] = sT;
  q_qfix[i] = pow(f * K, 0.5 * omb);
  q_D1fix[i] = d1_term(omb * omb, L);
  q_fpfix[i] = pow(f, omb);
  const double vol = q_vol[i];
  if (m.residual == 0) {
    q_tgt[i] = vol;
    q_w[i] = q_wuser[i];
  } else {
    q_tgt[i] = black_otm(f, K, L, sT, vol, m.q_D[i]);
    const double vg = black_vega(f, L, sT, vol, m.q_D[i]);
    q_w[i] = q_wuser[i] / (vg * vg);
  }
}

// ---------------------------------------------------------------------------
// sabr_cost_batch: one wave per point.
// ---------------------------------------------------------------------------
template <int MODEL, int FORMULA, int RESID>
__global__ __launch_bounds__(256) void cost_kernel(DevMarket m, int n_pts, const int *pt_inst,
                                                   const double *params, double *cost,
                                                   double *resid, double *model, int stride,
                                                   int lds_per_wave) {
  extern __shared__ double smem[];
  constexpr int P = NP<MODEL>::P;
  const int wid = threadIdx.x / kWave;
  const int pt = blockIdx.x * (blockDim.x / kWave) + wid;
  if (pt >= n_pts) return;
  const int inst = pt_inst[pt];
  if (inst < 0 || inst >= m.n_inst) {
    if (lane_id() == 0) cost[pt] = __builtin_nan("");
    return;
  }
  double p[P];
#pragma unroll
  for (int k = 0; k < P; ++k) p[k] = params[(size_t)pt * P + k];
  WaveLds w = wave_lds(m, smem + (size_t)wid * lds_per_wave);
  const double c = point_cost<MODEL, FORMULA, RESID>(
      m, inst, p, w, resid ? resid + (size_t)pt * stride : nullptr,
      model ? model + (size_t)pt * stride : nullptr);
  if (lane_id() == 0) cost[pt] = c;
}

// ---------------------------------------------------------------------------
// Simulated annealing (Sec. 3): synchronous parallel chains.  One wave per
// chain, W chains of one instance per workgroup, one launch per temperature
// level; the level-end kernel restarts every chain at the best final point.
// ---------------------------------------------------------------------------

// Neighbour: x' = x + delta (2u - 1), delta = step_frac (ub - lb), mirrored
// into [lb, ub] then clamped.  No contraction, so x' is bitwise reproducible.
__device__ __forceinline__ double propose1(double x, double u, double lo, double hi,
                                          double step_frac) {
#pragma clang fp contract(off)
  const double delta = step_frac * (hi - lo);
  double y = x + delta * (2.0 * u - 1.0);
  if (y > hi) y = 2.0 * hi - y;
  if (y < lo) y = 2.0 * lo - y;
  if (y > hi) y = hi;
  if (y < lo) y = lo;
  return y;
}

template <int MODEL, int FORMULA, int RESID>
__global__ __launch_bounds__(256) void sa_init_kernel(DevMarket m, SAArgs a, int lds_per_wave) {
  extern __shared__ double smem[];
  constexpr int P = NP<MODEL>::P;
  const int wid = threadIdx.x / kWave;
  const int inst = a.tile_inst[blockIdx.x];
  const int c = a.tile_chain[blockIdx.x] + wid;
  if (c >= a.chains[inst]) return;
  double x[P];
#pragma unroll
  for (int k = 0; k < P; ++k) x[k] = a.x0[(size_t)inst * P + k];
  WaveLds w = wave_lds(m, smem + (size_t)wid * lds_per_wave);
  const double f = point_cost<MODEL, FORMULA, RESID>(m, inst, x, w, nullptr, nullptr);
  if (lane_id() == 0) {
    const int64_t gc = a.chain_base[inst] + c;
    for (int k = 0; k < P; ++k) {
      a.X[gc * P + k] = x[k];
      a.BX[gc * P + k] = x[k];
    }
    a.F[gc] = f;
    a.BF[gc] = f;
    if (c == 0) {
      for (int k = 0; k < P; ++k) a.RX[(size_t)inst * P + k] = x[k];
      a.RF[inst] = f;
      a.Tcur[inst] = a.T0[inst];
      if (inst == 0) a.t_start[0] = wall_clock64();
    }
  }
}

template <int MODEL, int FORMULA, int RESID>
__global__ __launch_bounds__(256) void sa_level_kernel(DevMarket m, SAArgs a, int level,
                                                       int lds_per_wave) {
  extern __shared__ double smem[];
  constexpr int P = NP<MODEL>::P;
  constexpr int NBLK = (P + 1 + 3) / 4;
  const int wid = threadIdx.x / kWave;
  const int lane = lane_id();
  const int inst = a.tile_inst[blockIdx.x];
  const int C = a.chains[inst];
  const int c = a.tile_chain[blockIdx.x] + wid;
  if (c >= C) return;
  const int64_t gc = a.chain_base[inst] + c;
  double x[P], lo[P], hi[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    x[k] = a.RX[(size_t)inst * P + k];
    lo[k] = a.lb[(size_t)inst * P + k];
    hi[k] = a.ub[(size_t)inst * P + k];
  }
  double f = a.RF[inst];
  double bf = a.BF[gc];
  const double T = a.Tcur[inst];
  WaveLds w = wave_lds(m, smem + (size_t)wid * lds_per_wave);
  int nacc = 0;
  for (int s = 0; s < a.N; ++s) {
    double u[4 * NBLK];
    const uint64_t ctr0 = (uint64_t)level * (uint64_t)a.N + (uint64_t)s;
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
      uint64_t wds[4];
      philox4x64_10(ctr0, (uint64_t)c, (uint64_t)b, 0, a.seed, (uint64_t)inst, wds);
#pragma unroll
      for (int j = 0; j < 4; ++j) u[4 * b + j] = u53(wds[j]);
    }
    double xp[P];
#pragma unroll
    for (int k = 0; k < P; ++k) xp[k] = propose1(x[k], u[k], lo[k], hi[k], a.step_frac);
    double fp = point_cost<MODEL, FORMULA, RESID>(m, inst, xp, w, nullptr, nullptr);
    if (fp != fp) fp = kInf;
    const double dE = fp - f;
    const bool acc = (dE <= 0.0) || (u[P] < exp(-dE / T));
    if (acc) {
#pragma unroll
      for (int k = 0; k < P; ++k) x[k] = xp[k];
      f = fp;
      ++nacc;
    }
    if (a.accept && lane == 0)
      a.accept[a.acc_base[inst] + ((int64_t)level * a.N + s) * C + c] = acc ? 1 : 0;
    if (fp < bf) {
      bf = fp;
      if (lane == 0)
        for (int k = 0; k < P; ++k) a.BX[gc * P + k] = xp[k];
    }
  }
  if (lane == 0) {
    for (int k = 0; k < P; ++k) a.X[gc * P + k] = x[k];
    a.F[gc] = f;
    a.BF[gc] = bf;
    a.NACC[gc] = nacc;
  }
}

// Level end, one workgroup per instance: argmin of the final costs (ties ->
// lowest chain), restart point, best-ever trace, next temperature.
__global__ __launch_bounds__(256) void sa_level_end_kernel(SAArgs a, int level) {
  __shared__ double sf[256], sb[256];
  __shared__ int si[256], sj[256];
  __shared__ long long sn[256];
  const int inst = blockIdx.x;
  const int C = a.chains[inst];
  const int64_t base = a.chain_base[inst];
  double bestf = kInf, bestb = kInf;
  int bi = C, bj = C;
  long long na = 0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    const double fc = a.F[base + c], bc = a.BF[base + c];
    if (bi == C || fc < bestf) {  // strict: the lowest chain wins ties
      bestf = fc;
      bi = c;
    }
    if (bj == C || bc < bestb) {
      bestb = bc;
      bj = c;
    }
    na += a.NACC[base + c];
  }
  sf[threadIdx.x] = bestf;
  si[threadIdx.x] = bi;
  sb[threadIdx.x] = bestb;
  sj[threadIdx.x] = bj;
  sn[threadIdx.x] = na;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const int t = threadIdx.x + o;
      // lexicographic (f, chain) minimum; chain C marks an empty slot
      if (si[t] < C && (si[threadIdx.x] == C || sf[t] < sf[threadIdx.x] ||
                        (sf[t] == sf[threadIdx.x] && si[t] < si[threadIdx.x]))) {
        sf[threadIdx.x] = sf[t];
        si[threadIdx.x] = si[t];
      }
      if (sj[t] < C && (sj[threadIdx.x] == C || sb[t] < sb[threadIdx.x] ||
                        (sb[t] == sb[threadIdx.x] && sj[t] < sj[threadIdx.x]))) {
        sb[threadIdx.x] = sb[t];
        sj[threadIdx.x] = sj[t];
      }
      sn[threadIdx.x] += sn[t];
    }
    __syncthreads();
  }
  const int bstar = si[0];
  const int P = a.P;
  if (threadIdx.x < P) a.RX[(size_t)inst * P + threadIdx.x] = a.X[(base + bstar) * P + threadIdx.x];
  if (threadIdx.x == 0) {
    a.RF[inst] = a.F[base + bstar];
    if (a.level_best) a.level_best[(size_t)inst * a.L + level] = bstar;
    if (a.trace) {
      double *tr = a.trace + ((size_t)inst * a.L + level) * 3;
      tr[0] = sb[0];
      tr[1] = a.N > 0 ? (double)sn[0] / ((double)C * a.N) : 0.0;
      tr[2] = (double)(wall_clock64() - a.t_start[0]) * a.ns_per_tick;
    }
    a.Tcur[inst] = a.cool * a.Tcur[inst];
  }
}

// Best ever over all chains of each instance (ties -> lowest chain).
__global__ __launch_bounds__(256) void sa_final_kernel(SAArgs a) {
  __shared__ double sb[256];
  __shared__ int sj[256];
  const int inst = blockIdx.x;
  const int C = a.chains[inst];
  const int64_t base = a.chain_base[inst];
  const int P = a.P;
  double bestb = kInf;
  int bj = C;
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    const double bc = a.BF[base + c];
    if (bj == C || bc < bestb) {
      bestb = bc;
      bj = c;
    }
    if (a.chain_best_f) a.chain_best_f[base + c] = bc;
    if (a.chain_best_x)
      for (int k = 0; k < P; ++k) a.chain_best_x[(base + c) * P + k] = a.BX[(base + c) * P + k];
  }
  sb[threadIdx.x] = bestb;
  sj[threadIdx.x] = bj;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const int t = threadIdx.x + o;
      if (sj[t] < C && (sj[threadIdx.x] == C || sb[t] < sb[threadIdx.x] ||
                        (sb[t] == sb[threadIdx.x] && sj[t] < sj[threadIdx.x]))) {
        sb[threadIdx.x] = sb[t];
        sj[threadIdx.x] = sj[t];
      }
    }
    __syncthreads();
  }
  const int g = sj[0];
  if (threadIdx.x < P) a.best_x[(size_t)inst * P + threadIdx.x] = a.BX[(base + g) * P + threadIdx.x];
  if (threadIdx.x == 0) a.best_f[inst] = a.BF[base + g];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_prep(const DevMarket &m, double *q_tgt, double *q_w, double *q_L,
                       double *q_lfk, double *q_lnf, double *q_sqrtT, double *q_qfix,
                       double *q_D1fix, double *q_fpfix, double *f_v, double *u_S0b,
                       const double *q_vol, const double *q_wuser, const double *f_tauP,
                       const double *f_F, int n_q, int n_f, int n_u, hipStream_t s) {
  int n = n_q;
  if (n_f > n) n = n_f;
  if (n_u > n) n = n_u;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(prep_kernel, dim3((n + 255) / 256), dim3(256), 0, s, m, q_tgt, q_w, q_L,
                     q_lfk, q_lnf, q_sqrtT, q_qfix, q_D1fix, q_fpfix, f_v, u_S0b, q_vol, q_wuser,
                     f_tauP, f_F, n_q, n_f, n_u);
  return hipGetLastError();
}

#define SABR_SELECT(MODEL_, FORMULA_, RESID_, CALL)                  \
  do {                                                               \
    if ((MODEL_) == 0) {                                             \
      if ((FORMULA_) == 0) {                                         \
        if ((RESID_) == 0) { CALL(0, 0, 0); } else { CALL(0, 0, 1); } \
      } else {                                                       \
        if ((RESID_) == 0) { CALL(0, 1, 0); } else { CALL(0, 1, 1); } \
      }                                                              \
    } else {                                                         \
      if ((FORMULA_) == 0) {                                         \
        if ((RESID_) == 0) { CALL(1, 0, 0); } else { CALL(1, 0, 1); } \
      } else {                                                       \
        if ((RESID_) == 0) { CALL(1, 1, 0); } else { CALL(1, 1, 1); } \
      }                                                              \
    }                                                                \
  } while (0)

static int waves_for_lds(int lds_doubles, int want) {
  if (lds_doubles == 0) return want;
  int w = (64 * 1024) / (lds_doubles * 8);
  if (w > want) w = want;
  return w < 1 ? 1 : w;
}

hipError_t launch_cost(const DevMarket &m, int n_pts, const int *pt_inst, const double *params,
                       double *cost, double *resid, double *model, int stride, hipStream_t s) {
  if (n_pts == 0) return hipSuccess;
  const int ld = wave_lds_doubles(m);
  const int waves = waves_for_lds(ld, 4);
  const dim3 grid((n_pts + waves - 1) / waves), block(kWave * waves);
  const size_t lds = (size_t)ld * 8 * waves;
#define CALL(A, B, C)                                                                      \
  hipLaunchKernelGGL((cost_kernel<A, B, C>), grid, block, lds, s, m, n_pts, pt_inst, params, \
                     cost, resid, model, stride, ld)
  SABR_SELECT(m.model, m.formula, m.residual, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t launch_sa_init(const DevMarket &m, const SAArgs &a, int n_tiles, int waves,
                          hipStream_t s) {
  const int ld = wave_lds_doubles(m);
  const size_t lds = (size_t)ld * 8 * waves;
#define CALL(A, B, C)                                                                    \
  hipLaunchKernelGGL((sa_init_kernel<A, B, C>), dim3(n_tiles), dim3(kWave * waves), lds, s, \
                     m, a, ld)
  SABR_SELECT(m.model, m.formula, m.residual, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t launch_sa_level(const DevMarket &m, const SAArgs &a, int level, int n_tiles,
                           int waves, hipStream_t s) {
  const int ld = wave_lds_doubles(m);
  const size_t lds = (size_t)ld * 8 * waves;
#define CALL(A, B, C)                                                                     \
  hipLaunchKernelGGL((sa_level_kernel<A, B, C>), dim3(n_tiles), dim3(kWave * waves), lds, s, \
                     m, a, level, ld)
  SABR_SELECT(m.model, m.formula, m.residual, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t launch_sa_level_end(const SAArgs &a, int level, hipStream_t s) {
  hipLaunchKernelGGL(sa_level_end_kernel, dim3(a.n_inst), dim3(256), 0, s, a, level);
  return hipGetLastError();
}

hipError_t launch_sa_final(const SAArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(sa_final_kernel, dim3(a.n_inst), dim3(256), 0, s, a);
  return hipGetLastError();
}

int sa_waves_per_group(const DevMarket &m, int want) { return waves_for_lds(wave_lds_doubles(m), want); }

}  // namespace sabr
