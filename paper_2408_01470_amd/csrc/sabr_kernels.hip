// sabr_kernels.hip -- HIP kernels of the SA calibrator for gfx950.
//
// Mapping: one 64-lane wavefront evaluates one parameter point (one Markov
// chain) with its lanes spread over the market's quotes; each lane sums its
// quotes' weighted squared errors and the wave reduces the sums.  A
// workgroup holds W chains of one instance and stages that instance's
// per-underlying market values in LDS.  Parameter vectors live distributed
// over lanes (lane k holds coordinate k) and are broadcast to scalar
// registers when the cost needs them.  The FP64 vector ALU bounds every
// kernel here (no dense contraction: no MFMA).
#include <hip/hip_runtime.h>

#include <mutex>

#include "sabr_cost.hpp"

namespace sabr {

namespace {

// ---------------------------------------------------------------------------
// Market precompute (market-only quantities, once per upload).  The host has
// written und, kind and K of every quote record; this fills the rest.
// ---------------------------------------------------------------------------
__global__ void prep_kernel(DevMarket m, QuoteRec *q, double *f_v, double *u_S0b, double *u_c0,
                            double *u_fp,
                            const double *q_vol, const double *q_wuser, const int *q_und_g,
                            const double *f_tauP, const double *f_F, int n_q, int n_f, int n_u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double beta = m.beta, omb = 1.0 - beta;
  if (i < n_f) f_v[i] = f_tauP[i] * pow(f_F[i], beta);
  if (i < n_u) {
    const double S0b = pow(m.u_S0[i], beta);
    u_S0b[i] = S0b;
    u_c0[i] = m.u_invA[i] / S0b;
    u_fp[i] = pow(m.u_S0[i], omb);
  }
  if (i >= n_q) return;
  const int gu = q_und_g[i];
  QuoteRec R = q[i];
  const double f = m.u_S0[gu], K = R.K, T = m.u_T[gu], D = m.u_A[gu];
  const double L = log(f / K);
  const double sT = sqrt(T);
  R.L = L;
  if (m.model == 0) {
    R.qa = log(f * K);
    R.qb = 0.0;
    R.qc = log(f);
  } else {
    const double q = pow(f * K, 0.5 * omb);
    R.qa = q;
    R.qb = q * q * q * d1_term(omb * omb, L);
    R.qc = pow(f, omb);
  }
  const double vol = q_vol[i];
  if (m.residual == 0) {
    R.tgt = vol;
    R.w = q_wuser[i];
  } else {
    R.tgt = black_otm(f, K, L, sT, 1.0 / sT, vol, 1.0 / vol, D);
    const double vg = black_vega(f, L, sT, vol, D);
    R.w = q_wuser[i] / (vg * vg);
  }
  q[i] = R;
}

// ---------------------------------------------------------------------------
// sabr_cost_batch: one wave per point, up to kCostWaves points per workgroup.
// ---------------------------------------------------------------------------
constexpr int kCostWaves = 8;

template <int MODEL, int FORMULA, int RESID>
__global__ __launch_bounds__(kWave *kCostWaves, 4) void cost_kernel(DevMarket m, int n_pts,
                                                                   const int *pt_inst,
                                                                   const double *params,
                                                                   double *cost, double *resid,
                                                                   double *model, int stride,
                                                                   int lds_per_wave) {
  extern __shared__ double smem[];
  __shared__ int s_inst[kCostWaves];
  constexpr int PC = NP<MODEL>::P;       // 0: known at run time (PERFWD)
  const int P = PC > 0 ? PC : m.np;
  const int nw = blockDim.x / kWave;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int pt = blockIdx.x * nw + wid;
  int inst = -1;
  if (pt < n_pts) inst = __builtin_amdgcn_readfirstlane(pt_inst[pt]);
  const bool valid = pt < n_pts && inst >= 0 && inst < m.n_inst;
  if (pt < n_pts && !valid && lane_id() == 0) cost[pt] = __builtin_nan("");
  if (lane_id() == 0) s_inst[wid] = valid ? inst : -1;
  __syncthreads();
  // The workgroup's waves share one copy of the per-underlying market values:
  // one round per distinct instance among them (one round when the points of
  // a workgroup belong to one instance, the usual batch layout).  Every wave
  // takes part in every round's barriers.
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  double *wbase = smem + 6 * m.max_nu + (size_t)wid * lds_per_wave;
  for (int r = 0; r < nw; ++r) {
    const int ri = s_inst[r];
    bool first = ri >= 0;
    for (int q = 0; q < r; ++q) first = first && s_inst[q] != ri;
    if (!first) continue;   // the same for the whole workgroup
    const DevInst rin = m.inst[ri];
    for (int u = threadIdx.x; u < rin.nu; u += blockDim.x) um[u] = und_mkt(m, rin.u0 + u);
    __syncthreads();
    if (valid && inst == ri) {
      const DevInst in = m.inst[inst];
      double p[PC > 0 ? PC : 1];
#pragma unroll
      for (int k = 0; k < PC; ++k) p[k] = params[(size_t)pt * PC + k];
      const double xl = (PC == 0 && lane_id() < P) ? params[(size_t)pt * P + lane_id()] : 0.0;
      WaveLds w = wave_lds(m, wbase);
      const double c = point_cost<MODEL, FORMULA, RESID>(
          m, in, um, p, xl, w, resid ? resid + (size_t)pt * stride : nullptr,
          model ? model + (size_t)pt * stride : nullptr);
      if (lane_id() == 0) cost[pt] = c;
    }
    __syncthreads();   // the next round overwrites the market values
  }
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

template <int P>
__device__ __forceinline__ void broadcast_params(double xl, double *p) {
#pragma unroll
  for (int k = 0; k < P; ++k) p[k] = readlane_d(xl, k);
}

__device__ __forceinline__ UndMkt *stage_underlyings(const DevMarket &m, const DevInst &in,
                                                     double *smem) {
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  for (int u = threadIdx.x; u < in.nu; u += blockDim.x) um[u] = und_mkt(m, in.u0 + u);
  __syncthreads();
  return um;
}

// Lexicographic (f, chain) minimum over the wavefront; chain C marks an empty
// slot.  Every lane ends with the minimum.
__device__ __forceinline__ void wave_argmin(double &f, int &i, int C) {
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const double f2 = __shfl_xor(f, o, kWave);
    const int i2 = __shfl_xor(i, o, kWave);
    if (i2 < C && (i == C || f2 < f || (f2 == f && i2 < i))) {
      f = f2;
      i = i2;
    }
  }
}

// Level-end partial of one workgroup's chains (its waves hold consecutive
// chains of one instance; with PAIR each half-wave holds one, in lane
// order): lowest final cost (ties: lowest chain), lowest best-ever cost,
// accepted moves.  Every wave of the workgroup calls it; a wave (half)
// without a chain passes c = C.
template <bool PAIR = false>
__device__ void tile_partial(const SAArgs &a, int C, int c, double f, double bf, int nacc) {
  constexpr int S = PAIR ? 2 : 1;   // chain slots per wave
  __shared__ double red_f[S * kMaxWavesPerGroup], red_b[S * kMaxWavesPerGroup];
  __shared__ int red_c[S * kMaxWavesPerGroup], red_n[S * kMaxWavesPerGroup];
  const int wid = threadIdx.x / kWave;
  const int lane = lane_id();
  if (lane == 0 || (PAIR && lane == kHalf)) {
    const int v = S * wid + (PAIR ? lane / kHalf : 0);
    red_f[v] = f;
    red_b[v] = bf;
    red_c[v] = c;
    red_n[v] = nacc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bestf = kInf, bestb = kInf;
    int bi = C, bj = C, na = 0;
    for (int v = 0; v < S * (int)(blockDim.x / kWave); ++v) {   // chains in increasing order
      const int cv = red_c[v];
      if (cv >= C) continue;
      if (bi == C || red_f[v] < bestf) {   // strict: the lowest chain wins ties
        bestf = red_f[v];
        bi = cv;
      }
      if (bj == C || red_b[v] < bestb) {
        bestb = red_b[v];
        bj = cv;
      }
      na += red_n[v];
    }
    const int t = blockIdx.x;
    a.TF[t] = bestf;
    a.TI[t] = bi;
    a.TB[t] = bestb;
    a.TJ[t] = bj;
    a.TN[t] = na;
  }
}

// Level end of one instance by one workgroup, from its tiles' partials: the
// chain with the lowest final cost (ties: lowest chain) becomes every
// chain's restart point; the trace gets the best-ever cost, the acceptance
// rate and the device time; T is cooled.  scratch: 5 doubles per wave + 1 of
// LDS.
__device__ void level_end_block(const SAArgs &a, int inst, int level, double *scratch) {
  const int C = a.chains[inst];
  const int64_t base = a.chain_base[inst];
  const int t0 = a.tile_off[inst], t1 = a.tile_off[inst + 1];
  double bestf = kInf, bestb = kInf, na = 0.0;
  int bi = C, bj = C;
  // four tiles per thread and pass, their loads issued together
  const int stride = blockDim.x;
  for (int k0 = t0 + (int)threadIdx.x; k0 < t1; k0 += 4 * stride) {
    double fc[4], bc[4];
    int ic[4], jc[4], nc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + j * stride;
      const bool in = k < t1;
      fc[j] = in ? a.TF[k] : kInf;
      bc[j] = in ? a.TB[k] : kInf;
      ic[j] = in ? a.TI[k] : C;
      jc[j] = in ? a.TJ[k] : C;
      nc[j] = in ? a.TN[k] : 0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {   // tiles, hence chains, in increasing order
      if (ic[j] < C && (bi == C || fc[j] < bestf)) {  // strict: the lowest chain wins ties
        bestf = fc[j];
        bi = ic[j];
      }
      if (jc[j] < C && (bj == C || bc[j] < bestb)) {
        bestb = bc[j];
        bj = jc[j];
      }
      na += (double)nc[j];
    }
  }
  wave_argmin(bestf, bi, C);
  wave_argmin(bestb, bj, C);
  na = wave_sum(na);
  const int wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (lane_id() == 0) {
    scratch[5 * wid + 0] = bestf;
    scratch[5 * wid + 1] = (double)bi;
    scratch[5 * wid + 2] = bestb;
    scratch[5 * wid + 3] = (double)bj;
    scratch[5 * wid + 4] = na;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < nw; ++v) {
      const double f2 = scratch[5 * v], b2 = scratch[5 * v + 2];
      const int i2 = (int)scratch[5 * v + 1], j2 = (int)scratch[5 * v + 3];
      if (i2 < C && (bi == C || f2 < bestf || (f2 == bestf && i2 < bi))) {
        bestf = f2;
        bi = i2;
      }
      if (j2 < C && (bj == C || b2 < bestb || (b2 == bestb && j2 < bj))) {
        bestb = b2;
        bj = j2;
      }
      na += scratch[5 * v + 4];
    }
    scratch[5 * nw] = (double)bi;
    a.RF[inst] = bestf;
    if (a.level_best) a.level_best[(size_t)inst * a.L + level] = bi;
    if (a.trace) {
      double *tr = a.trace + ((size_t)inst * a.L + level) * 3;
      tr[0] = bestb;
      tr[1] = a.N > 0 ? na / ((double)C * a.N) : 0.0;
      tr[2] = (double)(wall_clock64() - a.t_start[0]) * a.ns_per_tick;
    }
    a.Tcur[inst] = a.cool * a.Tcur[inst];
  }
  __syncthreads();
  const int bstar = (int)scratch[5 * nw];
  const int P = a.P;
  if (threadIdx.x < P) a.RX[(size_t)inst * P + threadIdx.x] = a.X[(base + bstar) * P + threadIdx.x];
}

// Cost of a point whose quotes the nsub waves of a one-chain workgroup split
// (point_cost with sub, nsub): each wave's partial goes to LDS slot
// [parity][sub]; after the barrier every wave sums the slots in sub order,
// so all of them hold the same total and take the same Metropolis decision.
// Alternating the parity between calls makes one barrier per call enough:
// a wave writes a slot again only after every wave passed the barrier that
// followed its last read of it.
__device__ __forceinline__ double split_total(double part, int sub, int nsub, int parity) {
  __shared__ double xs[2][kMaxWavesPerGroup];
  if (lane_id() == 0) xs[parity][sub] = part;
  __syncthreads();
  double t = xs[parity][0];
  for (int k = 1; k < nsub; ++k) t += xs[parity][k];
  return t;
}

// The coordinates of the point whose lane k < P holds coordinate k, for
// every lane of the chain: wave-uniform, or per half-wave with PAIR.
template <int PC, bool PAIR>
__device__ __forceinline__ void chain_params(double xl, double *p) {
  if constexpr (PAIR) {
#pragma unroll
    for (int k = 0; k < PC; ++k) p[k] = half_lane(xl, k);
  } else {
    broadcast_params<PC>(xl, p);
  }
}

// SPLIT: compiled for chains split over the waves of their workgroup
// (a.wpc > 1); PAIR: two chains per wave, one per half (a.cpw = 2); the
// one-wave-per-chain variant keeps no trace of either.
template <int MODEL, int FORMULA, int RESID, bool SPLIT, bool PAIR>
__global__ __launch_bounds__(kWave * kMaxWavesPerGroup) void sa_init_kernel(DevMarket m, SAArgs a,
                                                                             int lds_per_wave) {
  static_assert(!(SPLIT && PAIR), "a chain spans waves or shares one, not both");
  extern __shared__ double smem[];
  constexpr int PC = NP<MODEL>::P;       // 0: known at run time (PERFWD)
  const int P = PC > 0 ? PC : a.P;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  // the lane's place among its chain's lanes (the wave, or its half)
  const int lane = PAIR ? (lane_id() & (kHalf - 1)) : lane_id();
  const int inst = a.tile_inst[blockIdx.x];
  const DevInst in = m.inst[inst];
  const UndMkt *um = stage_underlyings(m, in, smem);
  const int C = a.chains[inst];
  // SPLIT: the workgroup is one chain, its wpc waves split the quotes
  const int wpc = SPLIT ? a.wpc : 1;
  // the wave's first chain; with PAIR the upper half takes the next one
  const int c0 = a.tile_chain[blockIdx.x] + (SPLIT ? 0 : (PAIR ? 2 * wid : wid));
  const int c = c0 + (PAIR ? lane_id() / kHalf : 0);
  const int sub = SPLIT ? wid : 0;
  // resume: the state that the levels before level0 left (every chain of an
  // instance at its restart point) in place of the evaluation of x0
  const double *st =
      a.state_in ? a.state_in + 2 * (size_t)(P + 1) * a.chain_base[inst] + inst : nullptr;
  double f = kInf, bf = kInf;
  if (st) {
    if (c < C) {
      f = st[(size_t)C * P + c];
      bf = st[(size_t)C * (2 * P + 1) + c];
    }
  } else if (c0 < C) {   // wave-uniform (workgroup-uniform when wpc > 1)
    const double xl = (lane < P) ? a.x0[(size_t)inst * P + lane] : 0.0;
    double x[PC > 0 ? PC : 1];
    chain_params<PC, PAIR>(xl, x);
    WaveLds w = wave_lds(m, smem + 6 * m.max_nu + (size_t)wid * lds_per_wave);
    f = point_cost<MODEL, FORMULA, RESID, PAIR>(m, in, um, x, xl, w, nullptr, nullptr, sub,
                                                 wpc);
    if (SPLIT) f = split_total(f, sub, wpc, 0);
    bf = f;
  }
  if (c < C && sub == 0) {
    const bool own = lane < P;
    const double xl = own ? (st ? st[(size_t)c * P + lane] : a.x0[(size_t)inst * P + lane]) : 0.0;
    const double bxl = own && st ? st[(size_t)C * (P + 1) + (size_t)c * P + lane] : xl;
    const int64_t gc = a.chain_base[inst] + c;
    if (own) {
      a.X[gc * P + lane] = xl;
      a.BX[gc * P + lane] = bxl;
      if (c == 0) a.RX[(size_t)inst * P + lane] = xl;
    }
    if (lane == 0) {
      a.BF[gc] = bf;
      if (c == 0) {
        a.RF[inst] = f;
        double T = a.T0[inst];   // T0 cool^level0 by repeated multiplication
        for (int l = 0; l < a.level0; ++l) T = a.cool * T;
        a.Tcur[inst] = st ? st[(size_t)C * (2 * P + 2)] : T;
        if (inst == 0) a.t_start[0] = wall_clock64();
      }
    }
  }
  tile_partial<PAIR>(a, C, (c < C && sub == 0) ? c : C, f, bf, 0);
}

// OCC: minimum waves per SIMD the register allocation must allow (1 = the
// compiler's choice); a tuning knob traded against spills.  SPLIT and PAIR
// as for sa_init_kernel.
template <int MODEL, int FORMULA, int RESID, int OCC, bool SPLIT, bool PAIR>
__global__ __launch_bounds__(kWave * kMaxWavesPerGroup, OCC) void sa_level_kernel(DevMarket m,
                                                                                 SAArgs a,
                                                                                 int level,
                                                            int lds_per_wave) {
  static_assert(!(SPLIT && PAIR), "a chain spans waves or shares one, not both");
  extern __shared__ double smem[];
  constexpr int PC = NP<MODEL>::P;       // 0: known at run time (PERFWD)
  const int P = PC > 0 ? PC : a.P;
  const int nb = uni_blocks(P), spp = uni_steps(P, PAIR ? kHalf : kWave);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  // the lane's place among its chain's lanes (the wave, or its half)
  const int lane = PAIR ? (lane_id() & (kHalf - 1)) : lane_id();
  const int half = PAIR ? lane_id() / kHalf : 0;
  const int inst = a.tile_inst[blockIdx.x];
  const DevInst in = m.inst[inst];
  const UndMkt *um = stage_underlyings(m, in, smem);
  const int C = a.chains[inst];
  // SPLIT: the workgroup is one chain, its wpc waves split the quotes and
  // take the same steps; wave sub = 0 writes the chain's results
  const int wpc = SPLIT ? a.wpc : 1;
  // the wave's first chain; with PAIR the upper half takes the next one
  const int c0 = a.tile_chain[blockIdx.x] + (SPLIT ? 0 : (PAIR ? 2 * wid : wid));
  const int c = c0 + half;
  // PAIR: the upper half of an instance's last wave may hold no chain; it
  // steps along on its partner's records and writes nothing
  const bool live = c < C;
  const int sub = SPLIT ? wid : 0;
  double f_end = kInf, bf_end = kInf;
  int nacc_end = 0;
  if (c0 < C) {   // wave-uniform: waves past the instance's last chain have no work
    const int64_t gc = a.chain_base[inst] + (live ? c : c0);
    // lane k < P holds coordinate k of the chain's point, best point and box
    const bool own = lane < P;
    double x = own ? a.RX[(size_t)inst * P + lane] : 0.0;
    const double lo = own ? a.lb[(size_t)inst * P + lane] : 0.0;
    const double hi = own ? a.ub[(size_t)inst * P + lane] : 0.0;
    double bx = own ? a.BX[gc * P + lane] : 0.0;
    double f = a.RF[inst];
    double bf = a.BF[gc];
    const double T = a.Tcur[inst];
    double *wbase = smem + 6 * m.max_nu + (size_t)wid * lds_per_wave;
    WaveLds w = wave_lds(m, wbase);
    // [spp][P + 1] uniforms of the chain (each half's own with PAIR)
    double *uw = wbase + wave_lds_doubles(m) + half * spp * (P + 1);
    int nacc = 0;
    for (int s0 = 0; s0 < a.N; s0 += spp) {
      // Uniforms u_0..u_P of step s are the words of Philox blocks 0..P/4 of
      // counter (level N + s, chain, block, 0): word k mod 4 of block k/4.  One
      // pass over the lanes makes those of spp steps.
      {
        // the lane index is re-read each pass so nothing derived from it
        // stays live in registers across the steps
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const int sl = ln / nb, blk = ln - sl * nb;
        if (sl < spp && s0 + sl < a.N) {
          uint64_t wds[4];
          philox4x64_10((uint64_t)(a.level0 + level) * (uint64_t)a.N + (uint64_t)(s0 + sl),
                        (uint64_t)c,
                        (uint64_t)blk, 0, a.seed, (uint64_t)inst, wds);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (4 * blk + j <= P) uw[sl * (P + 1) + 4 * blk + j] = u53(wds[j]);
        }
      }
      wave_lds_sync();
      const int s1 = min(a.N, s0 + spp);
      for (int s = s0; s < s1; ++s) {
        const double *us = uw + (s - s0) * (P + 1);
        const double u = lane <= P ? us[lane] : 0.0;
        const double xp = own ? propose1(x, u, lo, hi, a.step_frac) : 0.0;
        double p[PC > 0 ? PC : 1];
        chain_params<PC, PAIR>(xp, p);
        double fp = point_cost<MODEL, FORMULA, RESID, PAIR>(m, in, um, p, xp, w, nullptr,
                                                             nullptr, sub, wpc);
        if (SPLIT) fp = split_total(fp, sub, wpc, s & 1);
        if (fp != fp) fp = kInf;
        const double uP = us[P];
        const double dE = fp - f;
        // dE > 0 here: the argument is <= 0 (or NaN when both costs are +inf,
        // which exp_neg maps to 0: a rejection, as exp(NaN) would give).  The
        // exponent is the correctly rounded quotient -dE/T, one division a
        // step, so it carries no rounding beyond that of dE itself.
        // (dE is uniform over the chain's lanes: the exponential runs for
        // uphill moves only)
        bool acc = dE <= 0.0;
        if (!acc) acc = uP < exp_neg(-dE / T);
        if (acc) {
          x = xp;
          f = fp;
          ++nacc;
        }
        if (a.accept && lane == 0 && sub == 0 && live)
          a.accept[a.acc_base[inst] + ((int64_t)level * a.N + s) * C + c] = acc ? 1 : 0;
        if (fp < bf) {
          bf = fp;
          bx = xp;
        }
      }
      wave_lds_sync();   // the next chunk overwrites the uniforms
    }
    if (own && sub == 0 && live) {
      a.X[gc * P + lane] = x;
      a.BX[gc * P + lane] = bx;
    }
    if (lane == 0 && sub == 0 && live) {
      a.BF[gc] = bf;
    }
    f_end = f;
    bf_end = bf;
    nacc_end = nacc;
  }
  tile_partial<PAIR>(a, C, (live && sub == 0) ? c : C, f_end, bf_end, nacc_end);
}

// Level end, one workgroup per instance: argmin of the final costs (ties ->
// lowest chain), restart point, best-ever trace, next temperature.
constexpr int kLevelEndThreads = 1024;
__global__ __launch_bounds__(kLevelEndThreads) void sa_level_end_kernel(SAArgs a, int level) {
  __shared__ double scratch[5 * (kLevelEndThreads / kWave) + 1];
  level_end_block(a, blockIdx.x, level, scratch);
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

// The annealing state after the last level (layout of SAArgs::state_out):
// every chain at the instance's restart point with its cost, the chains'
// best-ever points and costs, the next level's temperature.
__global__ __launch_bounds__(256) void sa_state_out_kernel(SAArgs a) {
  const int inst = blockIdx.x;
  const int C = a.chains[inst];
  const int P = a.P;
  const int64_t base = a.chain_base[inst];
  double *st = a.state_out + 2 * (size_t)(P + 1) * base + inst;
  const size_t CP = (size_t)C * P;
  for (size_t k = threadIdx.x; k < CP; k += blockDim.x) {
    st[k] = a.RX[(size_t)inst * P + k % P];
    st[(size_t)C * (P + 1) + k] = a.BX[(size_t)base * P + k];
  }
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    st[CP + c] = a.RF[inst];
    st[(size_t)C * (2 * P + 1) + c] = a.BF[base + c];
  }
  if (threadIdx.x == 0) st[(size_t)C * (2 * P + 2)] = a.Tcur[inst];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_prep(const DevMarket &m, QuoteRec *q, double *f_v, double *u_S0b, double *u_c0,
                       double *u_fp,
                       const double *q_vol, const double *q_wuser, const int *q_und_g,
                       const double *f_tauP, const double *f_F, int n_q, int n_f, int n_u,
                       hipStream_t s) {
  int n = n_q;
  if (n_f > n) n = n_f;
  if (n_u > n) n = n_u;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(prep_kernel, dim3((n + 255) / 256), dim3(256), 0, s, m, q, f_v, u_S0b, u_c0,
                     u_fp,
                     q_vol, q_wuser, q_und_g, f_tauP, f_F, n_q, n_f, n_u);
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
    } else if ((MODEL_) == 1) {                                      \
      if ((FORMULA_) == 0) {                                         \
        if ((RESID_) == 0) { CALL(1, 0, 0); } else { CALL(1, 0, 1); } \
      } else {                                                       \
        if ((RESID_) == 0) { CALL(1, 1, 0); } else { CALL(1, 1, 1); } \
      }                                                              \
    } else if ((MODEL_) == 2) {                                      \
      if ((FORMULA_) == 0) {                                         \
        if ((RESID_) == 0) { CALL(2, 0, 0); } else { CALL(2, 0, 1); } \
      } else {                                                       \
        if ((RESID_) == 0) { CALL(2, 1, 0); } else { CALL(2, 1, 1); } \
      }                                                              \
    } else if ((MODEL_) == 5) {                                      \
      if ((FORMULA_) == 0) {                                         \
        if ((RESID_) == 0) { CALL(5, 0, 0); } else { CALL(5, 0, 1); } \
      } else {                                                       \
        if ((RESID_) == 0) { CALL(5, 1, 0); } else { CALL(5, 1, 1); } \
      }                                                              \
    } else if ((MODEL_) == 3) {                                      \
      if ((FORMULA_) == 0) {                                         \
        if ((RESID_) == 0) { CALL(3, 0, 0); } else { CALL(3, 0, 1); } \
      } else {                                                       \
        if ((RESID_) == 0) { CALL(3, 1, 0); } else { CALL(3, 1, 1); } \
      }                                                              \
    } else {                                                         \
      if ((FORMULA_) == 0) {                                         \
        if ((RESID_) == 0) { CALL(4, 0, 0); } else { CALL(4, 0, 1); } \
      } else {                                                       \
        if ((RESID_) == 0) { CALL(4, 1, 0); } else { CALL(4, 1, 1); } \
      }                                                              \
    }                                                                \
  } while (0)

// The LDS budget of one workgroup, read from the device once (0: not yet).
static int g_lds_budget = 0;

int lds_budget_bytes() {
  int bytes = __atomic_load_n(&g_lds_budget, __ATOMIC_RELAXED);
  if (bytes == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      bytes = v;
    else
      bytes = 64 * 1024;
    __atomic_store_n(&g_lds_budget, bytes, __ATOMIC_RELAXED);
  }
  return bytes;
}

size_t sa_lds_bytes(const DevMarket &m, int waves, bool pair) {
  return (size_t)(6 * m.max_nu + waves * sa_wave_doubles(m, pair)) * 8;
}

int sa_waves_per_group(const DevMarket &m, int want, bool pair) {
  int w = want;
  while (w > 1 && (long)sa_lds_bytes(m, w, pair) > lds_budget_bytes()) --w;
  return w;
}

hipError_t launch_cost(const DevMarket &m, int n_pts, const int *pt_inst, const double *params,
                       double *cost, double *resid, double *model, int stride, hipStream_t s) {
  if (n_pts == 0) return hipSuccess;
  // one shared copy of the per-underlying market values, a wave-private
  // region per wave
  const int ld = wave_lds_doubles(m);
  auto bytes = [&](int w) { return (long)(6 * m.max_nu + (long)w * ld) * 8; };
  if (bytes(1) > lds_budget_bytes()) return hipErrorInvalidValue;
  int waves = kCostWaves;
  while (waves > 1 && bytes(waves) > lds_budget_bytes()) --waves;
  const dim3 grid((n_pts + waves - 1) / waves), block(kWave * waves);
  const size_t lds = (size_t)bytes(waves);
#define CALL(A, B, C)                                                                      \
  hipLaunchKernelGGL((cost_kernel<A, B, C>), grid, block, lds, s, m, n_pts, pt_inst, params, \
                     cost, resid, model, stride, ld)
  SABR_SELECT(kernel_model(m), m.formula, m.residual, CALL);
#undef CALL
  return hipGetLastError();
}

// One annealing kernel launch; the paired-chain variants exist for GLOBAL4
// only (the host refuses two chains per wave for the other models).
template <int A, int B, int C, bool SP, bool PR>
hipError_t init_launch(dim3 g, dim3 blk, size_t lds, hipStream_t s, const DevMarket &m,
                       const SAArgs &a, int ld) {
  if constexpr (PR && A != 0) {
    return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((sa_init_kernel<A, B, C, SP, PR>), g, blk, lds, s, m, a, ld);
    return hipGetLastError();
  }
}

template <int A, int B, int C, int O, bool SP, bool PR>
hipError_t level_launch(dim3 g, dim3 blk, size_t lds, hipStream_t s, const DevMarket &m,
                        const SAArgs &a, int level, int ld) {
  if constexpr (PR && A != 0) {
    return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((sa_level_kernel<A, B, C, O, SP, PR>), g, blk, lds, s, m, a, level, ld);
    return hipGetLastError();
  }
}

hipError_t launch_sa_init(const DevMarket &m, const SAArgs &a, int n_tiles, int waves,
                          hipStream_t s) {
  const bool pair = a.cpw == 2;
  const int ld = sa_wave_doubles(m, pair);
  const size_t lds = sa_lds_bytes(m, waves, pair);
  const dim3 g(n_tiles), blk(kWave * waves);
  hipError_t e = hipSuccess;
#define CALL(A, B, C)                                                \
  do {                                                               \
    if (a.wpc > 1)                                                   \
      e = init_launch<A, B, C, true, false>(g, blk, lds, s, m, a, ld); \
    else if (pair)                                                   \
      e = init_launch<A, B, C, false, true>(g, blk, lds, s, m, a, ld); \
    else                                                             \
      e = init_launch<A, B, C, false, false>(g, blk, lds, s, m, a, ld); \
  } while (0)
  SABR_SELECT(kernel_model(m), m.formula, m.residual, CALL);
#undef CALL
  return e;
}

hipError_t launch_sa_level(const DevMarket &m, const SAArgs &a, int level, int n_tiles,
                           int waves, int occupancy, hipStream_t s) {
  const bool pair = a.cpw == 2;
  const int ld = sa_wave_doubles(m, pair);
  const size_t lds = sa_lds_bytes(m, waves, pair);
  const dim3 g(n_tiles), blk(kWave * waves);
  hipError_t e = hipSuccess;
#define LAUNCH(A, B, C, O, SP, PR) \
  e = level_launch<A, B, C, O, SP, PR>(g, blk, lds, s, m, a, level, ld)
  // split chains are few (latency-bound): one register budget serves them
#define BY_OCC(A, B, C, PR)             \
  do {                                  \
    if (occupancy >= 4)                 \
      LAUNCH(A, B, C, 4, false, PR);    \
    else if (occupancy == 3)            \
      LAUNCH(A, B, C, 3, false, PR);    \
    else                                \
      LAUNCH(A, B, C, 1, false, PR);    \
  } while (0)
#define CALL(A, B, C)                   \
  do {                                  \
    if (a.wpc > 1)                      \
      LAUNCH(A, B, C, 1, true, false);  \
    else if (pair)                      \
      BY_OCC(A, B, C, true);            \
    else                                \
      BY_OCC(A, B, C, false);           \
  } while (0)
  SABR_SELECT(kernel_model(m), m.formula, m.residual, CALL);
#undef CALL
#undef BY_OCC
#undef LAUNCH
  return e;
}

hipError_t launch_sa_level_end(const SAArgs &a, int level, int max_tiles, hipStream_t s) {
  const int threads = max_tiles > 1024 ? kLevelEndThreads : 256;
  hipLaunchKernelGGL(sa_level_end_kernel, dim3(a.n_inst), dim3(threads), 0, s, a, level);
  return hipGetLastError();
}

hipError_t launch_sa_final(const SAArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(sa_final_kernel, dim3(a.n_inst), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sa_state_out(const SAArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(sa_state_out_kernel, dim3(a.n_inst), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free annealing entry point
// (sa_calibrate_noalloc): one copy of this array per device, held until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: host code uses only the address hipGetSymbolAddress returns
// for the current device, looked up once per device and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kSaNoallocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices] = {};   // the array's address on each device

hipError_t sa_noalloc_scratch(void **ptr) {
  auto &mu = g_scratch_mu;
  auto &per_dev = g_scratch_dev;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(mu);
  if (per_dev[dev] == nullptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr || reinterpret_cast<uintptr_t>(p) % 256) return hipErrorInvalidSymbol;
    per_dev[dev] = p;
  }
  *ptr = per_dev[dev];
  return hipSuccess;
}

void forget_process_caches() {
  __atomic_store_n(&g_lds_budget, 0, __ATOMIC_RELAXED);
  std::lock_guard<std::mutex> guard(g_scratch_mu);
  for (void *&p : g_scratch_dev) p = nullptr;
}

}  // namespace sabr
