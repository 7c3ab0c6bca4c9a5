// elementary_calib.hip -- prices the FP64 elementary functions the
// calibrator calls, for the algorithmic FLOP count of the roofline.
//
// Each kernel evaluates one function once per thread over n inputs drawn
// from the ranges the cost kernels see (the device library's exp, log1p,
// sqrt and division, and the kernels' own erfcx, exp, log1p, sqrt and
// reciprocal, and the exp + erfcx pair of the Black price); under
//   rocprofv3 --pmc SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64
//                   SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64
// the FP64 FLOP per call is 64 (ADD + MUL + TRANS + 2 FMA) / n minus the
// identical counts of the "copy" kernel (load, store, no arithmetic).  The
// last kernel adds its three results (2 FLOP beyond the call).
//
// Then the FP64 rate the chip delivers: fma_peak_kernel runs eight
// independent FMA chains per lane (enough to keep the VALU issuing every
// cycle at any wave count) over a grid of many waves per SIMD; HIP events
// time each launch and the program prints TFLOP/s next to the device's CU
// count and rated clock.  Under rocprofv3 --kernel-trace --pmc GRBM_COUNT
// the same launches give the clock the chip holds under pure FMA work.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sabr_device.hpp"
#include <cstdio>
#include <vector>

#define CHECK(x)                                                             \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) {                                                  \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
      return 1;                                                              \
    }                                                                        \
  } while (0)

template <int FN>
__global__ void elem_kernel(const double *__restrict__ x, const double *__restrict__ y,
                            double *__restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[i], b = y[i];
  double r;
  if (FN == 0) r = a;                 // copy: the baseline
  else if (FN == 1) r = exp(a);
  else if (FN == 2) r = log1p(a);
  else if (FN == 3) r = sqrt(a);
  else if (FN == 4) r = a / b;
  else if (FN == 5) r = sabr::erfcx_pos(a);   // the kernels' own functions from here on
  else if (FN == 6) r = sabr::exp_cw(a);
  else if (FN == 7) r = sabr::log1p_tang(a);
  else if (FN == 8) r = sabr::sqrt_gs(a);
  else if (FN == 9) r = a * sabr::rcp_nr(b);
  else {
    double E, X1, X2;
    sabr::exp_erfcx2(-a, a, b, E, X1, X2);
    r = E + X1 + X2;
  }
  out[i] = r;
}

constexpr int kPeakChains = 8;
constexpr int kPeakIters = 4096;

// 2 kPeakChains kPeakIters FLOP per lane: a <- a b + c on every chain, with
// b just below 1 and c small so the values stay normal and bounded.  x holds
// at least 512 doubles; every lane stores (so no chain is dead code) to
// out[i mod n], n a power of two.
__global__ void __launch_bounds__(256) fma_peak_kernel(const double *__restrict__ x,
                                                       double *__restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double b = 1.0 - 0x1.0p-30 * x[threadIdx.x];
  const double c = 0x1.0p-20 * x[threadIdx.x + 256];
  double a[kPeakChains];
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) a[k] = x[(threadIdx.x + 37 * k) & 511];
  for (int it = 0; it < kPeakIters; ++it) {
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) a[k] = fma(a[k], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) s += a[k];
  out[i & (n - 1)] = s;
}

int fma_peak(double *dx, double *dout, int n) {
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int blocks = 16384, threads = 256;   // 65536 waves: 64 per SIMD of 1024
  const double flop = 2.0 * kPeakChains * kPeakIters * (double)blocks * threads;
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  // about 2 s of launches: the clock ramps up over the first ones, so the
  // figures are the mean and best of the second half
  const int reps = 400;
  std::vector<double> tfs(reps);
  for (int r = 0; r < reps; ++r) {
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(fma_peak_kernel, dim3(blocks), dim3(threads), 0, 0, dx, dout, n);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    tfs[r] = flop / (ms * 1e-3) / 1e12;
    if (r % 50 == 0 || r == reps - 1)
      std::printf("fma_peak launch %d: %.3f ms, %.2f TFLOP/s\n", r, ms, tfs[r]);
  }
  double best = 0.0, sum = 0.0;
  for (int r = reps / 2; r < reps; ++r) {
    sum += tfs[r];
    best = tfs[r] > best ? tfs[r] : best;
  }
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  std::printf("fma_peak: %s (%s), %d CUs, rated clock %.0f MHz; FP64 FMA %.2f TFLOP/s mean, %.2f best "
              "over the last %d of the launches (%.3e FLOP each)\n",
              prop.name, prop.gcnArchName, prop.multiProcessorCount, prop.clockRate * 1e-3,
              sum / (reps - reps / 2), best, reps - reps / 2, flop);
  return 0;
}

int main() {
  const int n = 1 << 20;
  // inputs per function: exp in [-12, 0], log1p in [-0.6, 1.5], sqrt in
  // [0.2, 4], div in [0.1, 10]/[0.1, 10], erfcx in [0, 8]; the library
  // functions (1-4), then the kernels' own (5-10)
  constexpr int NF = 11;
  const double lo[NF] = {0.0, -12.0, -0.6, 0.2, 0.1, 0.0, -12.0, -0.6, 0.2, 0.1, 0.0};
  const double hi[NF] = {1.0, 0.0, 1.5, 4.0, 10.0, 8.0, 0.0, 1.5, 4.0, 10.0, 8.0};
  const char *names[NF] = {"copy",   "exp",        "log1p",   "sqrt",     "div",       "erfcx_pos",
                           "exp_cw", "log1p_tang", "sqrt_gs", "rcp_nr*x", "exp_erfcx2"};
  double *dx, *dy, *dout;
  CHECK(hipMalloc(&dx, n * sizeof(double)));
  CHECK(hipMalloc(&dy, n * sizeof(double)));
  CHECK(hipMalloc(&dout, n * sizeof(double)));
  std::vector<double> hx(n), hy(n);
  for (int f = 0; f < NF; ++f) {
    unsigned long long s = 88172645463325252ULL + f;
    for (int i = 0; i < n; ++i) {
      s ^= s << 13;
      s ^= s >> 7;
      s ^= s << 17;
      const double u = (double)(s >> 11) * 0x1.0p-53;
      s ^= s << 13;
      s ^= s >> 7;
      s ^= s << 17;
      const double v = (double)(s >> 11) * 0x1.0p-53;
      hx[i] = lo[f] + (hi[f] - lo[f]) * u;
      hy[i] = lo[f] + (hi[f] - lo[f]) * v;
    }
    CHECK(hipMemcpy(dx, hx.data(), n * sizeof(double), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(dy, hy.data(), n * sizeof(double), hipMemcpyHostToDevice));
    const dim3 grid(n / 256), block(256);
    switch (f) {
      case 0: hipLaunchKernelGGL(elem_kernel<0>, grid, block, 0, 0, dx, dy, dout, n); break;
      case 1: hipLaunchKernelGGL(elem_kernel<1>, grid, block, 0, 0, dx, dy, dout, n); break;
      case 2: hipLaunchKernelGGL(elem_kernel<2>, grid, block, 0, 0, dx, dy, dout, n); break;
      case 3: hipLaunchKernelGGL(elem_kernel<3>, grid, block, 0, 0, dx, dy, dout, n); break;
      case 4: hipLaunchKernelGGL(elem_kernel<4>, grid, block, 0, 0, dx, dy, dout, n); break;
      case 5: hipLaunchKernelGGL(elem_kernel<5>, grid, block, 0, 0, dx, dy, dout, n); break;
      case 6: hipLaunchKernelGGL(elem_kernel<6>, grid, block, 0, 0, dx, dy, dout, n); break;
      case 7: hipLaunchKernelGGL(elem_kernel<7>, grid, block, 0, 0, dx, dy, dout, n); break;
      case 8: hipLaunchKernelGGL(elem_kernel<8>, grid, block, 0, 0, dx, dy, dout, n); break;
      case 9: hipLaunchKernelGGL(elem_kernel<9>, grid, block, 0, 0, dx, dy, dout, n); break;
      default: hipLaunchKernelGGL(elem_kernel<10>, grid, block, 0, 0, dx, dy, dout, n); break;
    }
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    std::printf("%s: %d calls\n", names[f], n);
  }
  if (fma_peak(dx, dout, n) != 0) return 1;   // n = 2^20 >= 512, a power of two
  CHECK(hipFree(dx));
  CHECK(hipFree(dy));
  CHECK(hipFree(dout));
  return 0;
}
