// sabr_nm.hip -- Nelder-Mead polish of annealed points (the local minimizer
// the paper runs after its annealing, Sec. 3), for every model.
//
// One wavefront per point.  The simplex (P + 1 vertices) and its costs live
// in LDS; lane k owns coordinate k of every vertex, so the vertex arithmetic
// (centroid, reflection, expansion, contractions, shrink) is one lane per
// coordinate with no cross-lane traffic, and each cost evaluation is the
// whole wave's quote loop (point_cost).  Vertex arithmetic is evaluated
// without contraction, so the simplex follows a plain IEEE evaluation of the
// same steps whenever the cost comparisons agree.
#include <hip/hip_runtime.h>

#include "sabr_adjoint.hpp"
#include "sabr_cost.hpp"

namespace sabr {

namespace {

// clamp(c + t d) into [lo, hi], no fma contraction
__device__ __forceinline__ double nm_affine(double c, double t, double d, double lo, double hi) {
#pragma clang fp contract(off)
  const double y = c + t * d;
  return fmin(fmax(y, lo), hi);
}

// b + (v - b) / 2, no fma contraction
__device__ __forceinline__ double nm_half(double b, double v) {
#pragma clang fp contract(off)
  return b + 0.5 * (v - b);
}

// Lexicographic (f, i) minimum over the wavefront; i == C marks an empty
// lane.  Every lane ends with the minimum.
__device__ __forceinline__ void nm_argmin(double &f, int &i, int C) {
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

// Cost of the point whose coordinate k sits in lane k.
template <int MODEL, int FORMULA, int RESID>
__device__ __forceinline__ double nm_cost(const DevMarket &m, const DevInst &in,
                                          const UndMkt *um, double xl, WaveLds w) {
  constexpr int PC = NP<MODEL>::P;
  double p[PC > 0 ? PC : 1];
#pragma unroll
  for (int k = 0; k < PC; ++k) p[k] = readlane_d(xl, k);
  return point_cost<MODEL, FORMULA, RESID>(m, in, um, p, xl, w, nullptr, nullptr);
}

// Best (lowest cost, lowest index), worst (highest cost, highest index) and
// second-worst vertex of the simplex F[0..P].
struct NmOrder {
  int b, w;
  double fb, fw, fsw;
};

__device__ __forceinline__ NmOrder nm_order(const double *F, int P) {
  const int lane = lane_id();
  const int C = P + 1;
  const bool in = lane <= P;
  const double fv = in ? F[lane] : kInf;
  NmOrder o;
  double f = fv;
  int i = in ? lane : C;
  nm_argmin(f, i, C);
  o.b = i;
  o.fb = f;
  // the worst: minimum of (-f, P - v)
  f = in ? -fv : kInf;
  i = in ? P - lane : C;
  nm_argmin(f, i, C);
  o.w = P - i;
  o.fw = -f;
  f = (in && lane != o.w) ? -fv : kInf;
  i = (in && lane != o.w) ? P - lane : C;
  nm_argmin(f, i, C);
  o.fsw = -f;
  return o;
}

template <int MODEL, int FORMULA, int RESID>
__global__ __launch_bounds__(64) void nm_kernel(DevMarket m, int n_pts, const int *pt_inst,
                                                double *params, const double *lb,
                                                const double *ub, int max_iter, double step,
                                                double tol, double *cost_out, int *iters_out) {
  extern __shared__ double smem[];
  const int pt = blockIdx.x;
  const int lane = lane_id();
  const int P = m.np;
  const int inst = __builtin_amdgcn_readfirstlane(pt_inst[pt]);
  if (inst < 0 || inst >= m.n_inst) {
    if (lane == 0) {
      if (cost_out) cost_out[pt] = __builtin_nan("");
      if (iters_out) iters_out[pt] = 0;
    }
    return;
  }
  const DevInst in = m.inst[inst];
  UndMkt *um = reinterpret_cast<UndMkt *>(smem);
  for (int u = lane; u < in.nu; u += kWave) um[u] = und_mkt(m, in.u0 + u);
  WaveLds w = wave_lds(m, smem + 6 * m.max_nu);
  double *S = smem + 6 * m.max_nu + wave_lds_doubles(m);   // [P + 1][P]
  double *F = S + (size_t)(P + 1) * P;                       // [P + 1]
  wave_lds_sync();

  const bool own = lane < P;
  const double lo = own ? lb[(size_t)inst * P + lane] : 0.0;
  const double hi = own ? ub[(size_t)inst * P + lane] : 0.0;
  const double x0 = own ? params[(size_t)pt * P + lane] : 0.0;
  // initial simplex: x0 and x0 + d_k e_k (x0 - d_k when that leaves the box)
  for (int v = 0; v <= P; ++v) {
    double xv = x0;
    if (v > 0 && lane == v - 1) {
      double d, up;
      {
#pragma clang fp contract(off)
        d = step * (hi - lo);
        up = x0 + d;
      }
      xv = (up <= hi) ? up : x0 - d;
    }
    if (own) S[v * P + lane] = xv;
    const double f = nm_cost<MODEL, FORMULA, RESID>(m, in, um, xv, w);
    if (lane == 0) F[v] = f;
  }
  wave_lds_sync();

  int it = 0;
  while (it < max_iter) {
    const NmOrder o = nm_order(F, P);
    if (o.fw - o.fb <= tol * fabs(o.fb)) break;
    ++it;
    double sum = 0.0;
    if (own)
      for (int v = 0; v <= P; ++v)
        if (v != o.w) sum += S[v * P + lane];
    const double c = sum / (double)P;
    const double xw = own ? S[o.w * P + lane] : 0.0;
    const double xr = own ? nm_affine(c, 1.0, c - xw, lo, hi) : 0.0;
    const double fr = nm_cost<MODEL, FORMULA, RESID>(m, in, um, xr, w);
    double xn = xr, fn = fr;
    bool keep = true;
    if (fr < o.fb) {
      const double xe = own ? nm_affine(c, 2.0, c - xw, lo, hi) : 0.0;
      const double fe = nm_cost<MODEL, FORMULA, RESID>(m, in, um, xe, w);
      if (fe < fr) {
        xn = xe;
        fn = fe;
      }
    } else if (fr < o.fsw) {
      // keep the reflection
    } else if (fr < o.fw) {
      const double xc = own ? nm_affine(c, 0.5, xr - c, lo, hi) : 0.0;
      const double fc = nm_cost<MODEL, FORMULA, RESID>(m, in, um, xc, w);
      keep = fc <= fr;
      xn = xc;
      fn = fc;
    } else {
      const double xc = own ? nm_affine(c, 0.5, xw - c, lo, hi) : 0.0;
      const double fc = nm_cost<MODEL, FORMULA, RESID>(m, in, um, xc, w);
      keep = fc < o.fw;
      xn = xc;
      fn = fc;
    }
    if (keep) {
      if (own) S[o.w * P + lane] = xn;
      if (lane == 0) F[o.w] = fn;
    } else {   // shrink towards the best vertex
      const double xb = own ? S[o.b * P + lane] : 0.0;
      for (int v = 0; v <= P; ++v) {
        if (v == o.b) continue;
        const double xv = own ? nm_half(xb, S[v * P + lane]) : 0.0;
        if (own) S[v * P + lane] = xv;
        const double f = nm_cost<MODEL, FORMULA, RESID>(m, in, um, xv, w);
        if (lane == 0) F[v] = f;
      }
    }
    wave_lds_sync();
  }
  const NmOrder o = nm_order(F, P);
  if (own) params[(size_t)pt * P + lane] = S[o.b * P + lane];
  if (lane == 0) {
    if (cost_out) cost_out[pt] = o.fb;
    if (iters_out) iters_out[pt] = it;
  }
}

}  // namespace

size_t nm_lds_bytes(const DevMarket &m) {
  return (size_t)(6 * m.max_nu + wave_lds_doubles(m) + (m.np + 1) * m.np + m.np + 1) * 8;
}

hipError_t launch_nm(const DevMarket &m, int n_pts, const int *pt_inst, double *params,
                     const double *lb, const double *ub, int max_iter, double step, double tol,
                     double *cost_out, int *iters_out, hipStream_t s) {
  if (n_pts == 0) return hipSuccess;
  const size_t lds = nm_lds_bytes(m);
  int dev = 0, cap = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      cap <= 0)
    cap = 64 * 1024;
  if (lds > (size_t)cap) return hipErrorInvalidValue;
#define CALL(A, B, C)                                                                          \
  hipLaunchKernelGGL((nm_kernel<A, B, C>), dim3(n_pts), dim3(kWave), lds, s, m, n_pts, pt_inst, \
                     params, lb, ub, max_iter, step, tol, cost_out, iters_out)
#define SEL_FR(A)                                         \
  do {                                                    \
    if (m.formula == 0) {                                 \
      if (m.residual == 0) CALL(A, 0, 0); else CALL(A, 0, 1); \
    } else {                                              \
      if (m.residual == 0) CALL(A, 1, 0); else CALL(A, 1, 1); \
    }                                                     \
  } while (0)
  switch (kernel_model(m)) {
    case 0: SEL_FR(0); break;
    case 1: SEL_FR(1); break;
    case 2: SEL_FR(2); break;
    case 3: SEL_FR(3); break;
    case 4: SEL_FR(4); break;
    case 5: SEL_FR(5); break;
    default: return hipErrorInvalidValue;
  }
#undef SEL_FR
#undef CALL
  return hipGetLastError();
}

}  // namespace sabr
