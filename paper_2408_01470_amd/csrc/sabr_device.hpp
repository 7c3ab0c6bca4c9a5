// sabr_device.hpp -- device-side building blocks of the SA calibrator
// (gfx950, FP64 vector ALU).
//
// Market layout, Philox4x64-10, the Hagan 2002 lognormal implied vol, the
// paper's eq. (sigmaHagan), Black-76 and wavefront helpers.  The kernels run
// one 64-lane wavefront per parameter point with the lanes spread over the
// market's quotes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "erfcx_poly.hpp"
#include "exp_poly.hpp"
#include "log1p_poly.hpp"

namespace sabr {

constexpr int kWave = 64;
constexpr double kInf = __builtin_huge_val();

// ---------------------------------------------------------------------------
// Packed market (device image).  Arrays are structure-of-arrays over the
// whole batch except the quote records, which are 64-byte array-of-structs
// entries read with 16-byte loads.  Indices stored in the image (underlying
// of a quote, first forward of an underlying) are local to their instance.
// ---------------------------------------------------------------------------
struct DevInst {
  int f0, nf;   // forward range
  int u0, nu;   // underlying range
  int q0, nq;   // quote range
  int maxlen;   // longest underlying (forwards per swap)
  int pad;
};

// One quote.  qa/qb/qc hold the market-only factors of the vol formula:
//   beta a parameter (GLOBAL4): qa = ln(f K), qb = 0, qc = ln f;
//   beta fixed (LMM12):         qa = q = (f K)^((1-b)/2), qb = q^3 D1(L),
//                               qc = f^(1-b).
struct QuoteRec {
  double L;     // ln(f/K)
  double qa, qb;
  double tgt;   // market vol, or out-of-the-money Black price of the market vol
  double w;     // weight (price mode: user weight / market vega^2)
  double qc;
  int und;      // underlying (local index)
  int kind;     // 0 call, 1 put
  double K;     // strike
};
static_assert(sizeof(QuoteRec) == 64, "quote record must be 64 bytes");

// One underlying in the order the map visits them (per instance, decreasing
// swap length): local index, first forward, length.
struct alignas(16) UndMap {
  int u, e, n, pad;
};

struct DevMarket {
  int n_inst, model, formula, residual;
  int np;                // parameters per point (3 per forward for PERFWD)
  int thchunk;           // LMM12: underlyings whose SABR constants the cost kernels
                         // hold in LDS at a time
  int reglen;            // LMM12: swaps of up to this many forwards keep the map's
                         // recursion column in registers in the cost kernels
                         // (16 or 24; longer ones use an LDS column)
  double beta;           // fixed beta (LMM12, PERFWD)
  int max_nq, max_nu, max_nf, max_len;
  const DevInst *inst;
  // forwards
  const double *f_T;     // fixing time T_k
  const double *f_v;     // tau_k P_k F_k^beta (fixed beta)
  const double *f_mmw;   // MM drift weight T_{k-1} tau_k F_k^beta / (1 + tau_k F_k)
  // underlyings (caplet = one-period swap)
  const int *u_first, *u_len;
  const int *u_order;    // per instance: the map's visiting order (the internal order)
  const int *u_q0;       // per underlying: its first quote (local index)
  const int *q_ext;      // per quote: its index in the caller's order (local)
  const double *u_S0, *u_A, *u_invA, *u_S0b, *u_T;  // swap rate, annuity, 1/A, S0^beta, expiry
  const UndMap *u_map;   // per instance: u_order[i] with its first forward and length
  const double *u_c0;    // 1/(A S0^beta) per underlying
  const double *u_fp;    // S0^(1-beta) per underlying (fixed beta)
  // quotes
  const QuoteRec *q;
};

// Per-underlying market values staged in LDS by every workgroup.
struct UndMkt {
  double f, D, T, sqrtT, isqrtT;
  double fp;   // f^(1-beta) for a fixed beta (LMM12, PERFWD), else 0
};
static_assert(sizeof(UndMkt) == 48, "16-byte aligned LDS record");

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
// Wavefront helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Value of lane l as a wave-uniform (scalar) register.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// A double moved across lanes by a DPP pattern (both halves); lanes whose
// row is not in ROW_MASK read 0.  With every row enabled the pattern writes
// every lane, so no old value is needed (no zeroing moves).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  int lo, hi;
  if constexpr (ROW_MASK == 0xf) {
    lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  } else {
    lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROW_MASK, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  }
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes (all active), returned wave-uniform.  Register-to-
// register lane moves only: quad swaps (lane ^ 1, lane ^ 2), the half-row and
// row mirrors (every lane of a 16-lane row then holds the row's sum), then
// the row broadcasts of lanes 15 and 31 fold the four rows into lane 63.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);        // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);        // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);       // row_half_mirror
  v += dpp_d<0x140>(v);       // row_mirror
  v += dpp_d<0x142, 0xa>(v);  // row_bcast15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);  // row_bcast31 into rows 2 and 3
  return readlane_d(v, kWave - 1);
}

// Paired chains: lanes 0-31 serve one chain, lanes 32-63 another.
constexpr int kHalf = kWave / 2;

// The value of lane k of the caller's half (k < 32), in every lane of it.
__device__ __forceinline__ double half_lane(double v, int k) {
  const double lo = readlane_d(v, k), hi = readlane_d(v, kHalf + k);
  return (threadIdx.x & kHalf) ? hi : lo;
}

// Sums over the 16-lane rows (all lanes active): the first four moves of
// wave_sum, after which every lane of a row holds the row's sum.
__device__ __forceinline__ double row_sums(double v) {
  v += dpp_d<0xB1>(v);        // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);        // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);       // row_half_mirror
  v += dpp_d<0x140>(v);       // row_mirror
  return v;
}

// For each half of the wave, the wave_sum of the 64 values whose lanes 0-31
// are the half's lo and lanes 32-63 its hi, bit for bit (IEEE addition
// commutes): wave_sum adds rows 0 + 1 and rows 2 + 3 (row_bcast15), then the
// two pairs (row_bcast31); here lo's and hi's rows stand for rows 0, 1 and
// 2, 3.  Every lane of the half gets its total.
__device__ __forceinline__ double half_sum2(double lo, double hi) {
  lo = row_sums(lo);
  hi = row_sums(hi);
  lo += dpp_d<0x142, 0xa>(lo);  // row_bcast15 into rows 1 and 3
  hi += dpp_d<0x142, 0xa>(hi);
  return half_lane(hi + lo, kHalf - 1);
}

// Whether any lane of the caller's half has b set.
__device__ __forceinline__ bool half_any(bool b) {
  const unsigned long long m = __ballot(b);
  return ((threadIdx.x & kHalf) ? (m >> kHalf) : (m & 0xffffffffULL)) != 0;
}

// Element i of an array the caller knows to lie in LDS, addressed in 32 bits
// (one 24-bit multiply, where the generic pointer's index takes a 64-bit
// multiply-add); i * sizeof(T) < 2^24 always holds in LDS.
template <class T>
__device__ __forceinline__ T lds_elem(const T *p, int i) {
  static_assert(sizeof(T) % sizeof(double) == 0, "records of doubles");
  using lcp = __attribute__((address_space(3))) const char *;
  using ldp = __attribute__((address_space(3))) const double *;
  const ldp src = (ldp)((lcp)p + __umul24((unsigned)i, (unsigned)sizeof(T)));
  T v;
  double *dst = reinterpret_cast<double *>(&v);
#pragma unroll
  for (size_t k = 0; k < sizeof(T) / sizeof(double); ++k) dst[k] = src[k];
  return v;
}

// Element i >= 0 of a global array by a 32-bit byte offset from its base
// (the scalar-base form of the global load; i * sizeof(T) < 2^32).
template <class T>
__device__ __forceinline__ T glb_elem(const T *p, int i) {
  return *(const T *)((const char *)p + (unsigned)i * (unsigned)sizeof(T));
}

// Orders LDS traffic of one wavefront: a wave's LDS operations execute in
// issue order, so only the compiler must be kept from reordering them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Elementary functions of the quote loop, branch-free.
// ---------------------------------------------------------------------------
// A double constant materialized in a scalar register pair where it is used.
// Left alone, the compiler hoists the polynomial coefficients below out of
// the quote loop into vector registers, where they stay pinned for the whole
// loop and cost occupancy; volatile scalar moves keep each coefficient local
// to its use (SALU work, which issues beside other waves' vector work).
template <unsigned long long BITS>
__device__ __forceinline__ double sconst() {
  unsigned lo, hi;
  asm volatile("s_mov_b32 %0, %1" : "=s"(lo) : "i"((unsigned)(BITS & 0xffffffffull)));
  asm volatile("s_mov_b32 %0, %1" : "=s"(hi) : "i"((unsigned)(BITS >> 32)));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
#define SABR_SCONST(x) ::sabr::sconst<__builtin_bit_cast(unsigned long long, (x))>()

// h t + c with c in a scalar register pair, as one VOP3 v_fma_f64.  Written
// as fma() the compiler emits the two-address v_fmac_f64 instead, which
// needs c copied into the destination vector register first (two extra
// vector moves per Horner step).
__device__ __forceinline__ double fma_s(double h, double t, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(h), "v"(t), "s"(c));
  return r;
}

// Horner's rule on the coefficients C[0..DEG] (constant arrays), one chain
// or two interleaved chains sharing each coefficient.  Each step's
// coefficient is materialized one step ahead: a vector instruction may not
// read a scalar register the instruction just before it wrote (the hardware
// then needs a wait state, one s_nop per step).
template <const double *C, int DEG, size_t I>
__device__ __forceinline__ double next_coef(double c) {
  if constexpr (I + 1 < DEG) return SABR_SCONST(C[DEG - 2 - I]);
  return c;
}
template <const double *C, int DEG, size_t I>
__device__ __forceinline__ void horner_step(double t, double &h, double &c) {
  const double cn = next_coef<C, DEG, I>(c);
  h = fma_s(h, t, c);
  c = cn;
}
// The leading step t C[DEG] + C[DEG-1] of a single chain as a multiply and
// an add, each reading its constant from scalar registers (an fma would need
// C[DEG] copied to vector registers first: two more vector instructions).
__device__ __forceinline__ double lead_step(double t, double c0, double c1) {
#pragma clang fp contract(off)
  return t * c0 + c1;
}
template <const double *C, int DEG, size_t... I>
__device__ __forceinline__ double horner_s(double t, std::index_sequence<I...>) {
  const double c0 = SABR_SCONST(C[DEG]);
  const double c1 = SABR_SCONST(C[DEG - 1]);
  double c = SABR_SCONST(C[DEG - 2]);
  double h = lead_step(t, c0, c1);
  (horner_step<C, DEG, I + 1>(t, h, c), ...);
  return h;
}
template <const double *C, int DEG>
__device__ __forceinline__ double horner_s(double t) {
  static_assert(DEG >= 2, "a leading step and at least one more");
  return horner_s<C, DEG>(t, std::make_index_sequence<DEG - 1>{});
}
template <const double *C, int DEG, size_t I>
__device__ __forceinline__ void horner2_step(double t1, double t2, double &h1, double &h2,
                                             double &c) {
  const double cn = next_coef<C, DEG, I>(c);
  h1 = fma_s(h1, t1, c);
  h2 = fma_s(h2, t2, c);
  c = cn;
}
template <const double *C, int DEG, size_t... I>
__device__ __forceinline__ void horner2_s(double t1, double t2, double &h1, double &h2,
                                          std::index_sequence<I...>) {
  h1 = SABR_SCONST(C[DEG]);
  h2 = h1;
  double c = SABR_SCONST(C[DEG - 1]);
  (horner2_step<C, DEG, I>(t1, t2, h1, h2, c), ...);
}

// 1/d for a normal, finite d.  The v_rcp_f64 seed r0 has a relative error
// below 2^-24 on MI355X (measured over 4M inputs: 4.6e-8); with
// e = 1 - d r0 (exact to 2^-77 in one fma), 1/d = r0 (1 + e + e^2 + ...) and
// r0 + r0 (e + e^2) leaves a truncation error e^3 < 2^-72: within an ulp or
// so of the rounded quotient.  A zero, infinite or NaN d gives NaN, which
// every caller treats as a domain failure.
__device__ __forceinline__ double rcp_nr(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// sqrt(a) for a positive normal a: Goldschmidt iteration (Markstein, IA-64
// and Elementary Functions, 2000) from the v_rsq_f64 seed (relative error
// below 2^-24 on MI355X, measured: 5.3e-8), g -> sqrt(a), h -> 1/(2 sqrt(a)):
// one pass (error ~2^-47) and a final Newton correction g + (a - g^2) h.
// Zero, infinite, negative or NaN a gives NaN.
__device__ __forceinline__ double sqrt_gs(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  return fma(fma(-g, g, a), h, g);
}

// exp(x) (method of exp_poly.hpp): k = rint(x/ln2), r = x - k ln2 in two fma
// steps, 2^k p(r).  Underflows to 0 below -746, overflows to +inf above 710,
// NaN stays NaN.  exp_neg below is the same for finite x <= 0 without the
// upper clamp and the NaN test.
__device__ __forceinline__ double exp_cw(double x) {
  const double xc = fmin(fmax(x, -746.0), 710.0);
  const double kd = rint(xc * kExpInvLn2);
  double r = fma(-kd, kExpLn2Hi, xc);
  r = fma(-kd, kExpLn2Lo, r);
  const double p = horner_s<kExpPoly, kExpDeg>(r);
  const double e = ldexp(p, (int)kd);
  return x == x ? e : x;
}

__device__ __forceinline__ double exp_neg(double x) {
  const double xc = fmax(x, -746.0);
  const double kd = rint(xc * kExpInvLn2);
  double r = fma(-kd, kExpLn2Hi, xc);
  r = fma(-kd, kExpLn2Lo, r);
  return ldexp(horner_s<kExpPoly, kExpDeg>(r), (int)kd);
}

// log1p(t) for t > -1 (method of log1p_poly.hpp): v = 1 + t rounded with its
// exact error e (two-sum), v = 2^k m with m in [sqrt(1/2), sqrt(2)),
// f = (m - 1) + e 2^-k (so 1 + f = (1 + t)/2^k), s = f/(2 + f),
// log(1 + f) = f - s (f - s^2 P(s^2)), and log1p(t) = k ln2 + log(1 + f).
// NaN for t <= -1, t = +inf or NaN t; branch-free.  CHECKED = false leaves
// out the select of NaN for t <= -1, for callers whose t >= 0 (NaN and +inf
// still give NaN).
template <bool CHECKED = true>
__device__ __forceinline__ double log1p_tang(double t) {
  const double v = 1.0 + t;
  const double vv = v - 1.0;
  const double e = (1.0 - (v - vv)) + (t - vv);
  double m = __builtin_amdgcn_frexp_mant(v);
  int k = __builtin_amdgcn_frexp_exp(v);
  const bool up = m < M_SQRT1_2;
  m = up ? m + m : m;
  k = up ? k - 1 : k;
  // 1 + t = 2^k (m + e 2^-k) exactly: the rounding error of v joins f (it is
  // below 2^-53 of m, so f's own rounding stays relative to f)
  const double f = (m - 1.0) + ldexp(e, -k);
  const double s = f * rcp_nr(2.0 + f);
  const double z = s * s;
  const double p = horner_s<kLog1pPoly, kLog1pDeg>(z);
  const double lf = fma(-s, fma(-z, p, f), f);
  const double kd = (double)k;
  const double res = fma(kd, kLn2Hi, lf + kd * kLn2Lo);
  if constexpr (!CHECKED) return res;
  return v > 0.0 ? res : __builtin_nan("");
}

// erfcx(x) = exp(x^2) erfc(x) for x >= 0 (method of erfcx_poly.hpp): one
// reciprocal r = 1/(x + K) (x + K >= K, so no range scaling is needed),
// t = (x - K) r, erfcx = h(t) r with h a degree-24 polynomial; branch-free,
// no tables.  Arguments above 1e100 (and NaN) are taken as 1e100: callers
// multiply the result by exp(-x^2), which is zero there.
__device__ __forceinline__ double erfcx_pos(double x) {
  x = fmin(x, 1e100);
  const double r = rcp_nr(x + kErfcxK);
  const double t = (x - kErfcxK) * r;
  return horner_s<kErfcxPoly, kErfcxDeg>(t) * r;
}

// One step of three interleaved Horner chains: step I of the two chains on
// C (degree DEG) and, over its last DEG2 steps, of a third chain on C2
// (degree DEG2 <= DEG).  The coefficients reach the scalar registers in
// program order, one step ahead of their use (see horner_step), so the
// interleaving is written out here rather than left to the scheduler.
template <const double *C, int DEG, const double *C2, int DEG2, size_t I>
__device__ __forceinline__ void horner3_step(double t1, double t2, double t3, double &h1,
                                             double &h2, double &h3, double &c, double &c2) {
  const double cn = next_coef<C, DEG, I>(c);
  // the third chain's step J = I - (DEG - DEG2) uses C2[DEG2 - 1 - J]; its
  // first coefficient is materialized with the step before its first use
  double c2n = c2;
  if constexpr (I + 1 + DEG2 == DEG) c2n = SABR_SCONST(C2[DEG2 - 1]);
  if constexpr (I + DEG2 >= DEG && I + 1 < DEG) c2n = SABR_SCONST(C2[DEG - 2 - I]);
  h1 = fma_s(h1, t1, c);
  h2 = fma_s(h2, t2, c);
  if constexpr (I + DEG2 >= DEG) h3 = fma_s(h3, t3, c2);
  c = cn;
  c2 = c2n;
}
template <const double *C, int DEG, const double *C2, int DEG2, size_t... I>
__device__ __forceinline__ void horner3_s(double t1, double t2, double t3, double &h1, double &h2,
                                          double &h3, std::index_sequence<I...>) {
  static_assert(DEG2 < DEG, "the third chain rides along the last steps");
  h1 = SABR_SCONST(C[DEG]);
  h2 = h1;
  h3 = SABR_SCONST(C2[DEG2]);
  double c = SABR_SCONST(C[DEG - 1]), c2 = 0.0;
  (horner3_step<C, DEG, C2, DEG2, I>(t1, t2, t3, h1, h2, h3, c, c2), ...);
}

// erfcx_pos of two arguments, the two polynomial chains interleaved.
__device__ __forceinline__ void erfcx_pos2(double x1, double x2, double &X1, double &X2) {
  x1 = fmin(x1, 1e100);
  x2 = fmin(x2, 1e100);
  const double r1 = rcp_nr(x1 + kErfcxK), r2 = rcp_nr(x2 + kErfcxK);
  double h1, h2;
  horner2_s<kErfcxPoly, kErfcxDeg>((x1 - kErfcxK) * r1, (x2 - kErfcxK) * r2, h1, h2,
                                    std::make_index_sequence<kErfcxDeg>{});
  X1 = h1 * r1;
  X2 = h2 * r2;
}

// exp_neg(xe) and erfcx_pos of x1 and x2 (as those functions compute them),
// the exponential's Horner chain interleaved with the last steps of the two
// erfcx chains.
__device__ __forceinline__ void exp_erfcx2(double xe, double x1, double x2, double &E, double &X1,
                                           double &X2) {
  const double xc = fmax(xe, -746.0);
  const double kd = rint(xc * kExpInvLn2);
  double r = fma(-kd, kExpLn2Hi, xc);
  r = fma(-kd, kExpLn2Lo, r);
  x1 = fmin(x1, 1e100);
  x2 = fmin(x2, 1e100);
  // one reciprocal for both: 1/a1 = a2/(a1 a2), 1/a2 = a1/(a1 a2)
  const double a1 = x1 + kErfcxK, a2 = x2 + kErfcxK;
  const double ip = rcp_nr(a1 * a2);
  const double r1 = a2 * ip, r2 = a1 * ip;
  double h1, h2, he;
  horner3_s<kErfcxPoly, kErfcxDeg, kExpPoly, kExpDeg>((x1 - kErfcxK) * r1, (x2 - kErfcxK) * r2, r,
                                                       h1, h2, he,
                                                       std::make_index_sequence<kErfcxDeg>{});
  X1 = h1 * r1;
  X2 = h2 * r2;
  E = ldexp(he, (int)kd);
}

// ---------------------------------------------------------------------------
// SABR constants of one (alpha, beta, rho, nu): everything in the Hagan
// formula that does not depend on the quote.
//   corr q^2 = q^2 + (ca + cb q + cc q^2) T, ca = (1-b)^2 alpha^2/24,
//   cb = rho beta nu alpha/4, cc = (2 - 3 rho^2) nu^2/24;
//   z/x(z) = 1 - (rho/2) z + ((2 - 3 rho^2)/12) z^2 + O(z^3)   (near z = 0).
// ---------------------------------------------------------------------------
struct SabrConst {
  double alpha, rho, nua;   // nua = nu / alpha
  double ca, cb, cc;
};
static_assert(sizeof(SabrConst) == 48, "16-byte aligned LDS record");
constexpr int kSabrConstDoubles = 6;

__device__ __forceinline__ SabrConst sabr_const(double alpha, double beta, double rho, double nu) {
  SabrConst k;
  const double omb = 1.0 - beta;
  const double r2 = rho * rho;
  k.alpha = alpha;
  k.rho = rho;
  k.nua = nu * rcp_nr(alpha);
  k.ca = omb * omb * alpha * alpha * (1.0 / 24.0);
  k.cb = rho * beta * nu * alpha * 0.25;
  k.cc = (2.0 - 3.0 * r2) * nu * nu * (1.0 / 24.0);
  return k;
}

// |z| below which the adjoint's chi = z/x(z) takes its series (three terms
// leave a truncation error below 1e-17 here).
constexpr double kZSeries = 0x1.0p-18;
// Smallest |z| the cost kernels' quotient form takes (see hagan2002_frac).
constexpr double kZFloor = 0x1.0p-60;

// Hagan 2002 lognormal vol given L = ln(f/K), q = (f K)^((1-beta)/2),
// q3D1 = q^3 D1 with D1 = 1 + (1-b)^2 L^2/24 + (1-b)^4 L^4/1920 (a quote's
// constant when beta is fixed) and expiry T, as a fraction
//   sigma = numer / denom,  numer = alpha corr q^2 chi_num,
//                           denom = q^3 D1 chi_den,
// with chi = z/x(z) = chi_num/chi_den.  s = sqrt(1 - 2 rho z + z^2) is
// unchanged and x(z) changes sign under (z, rho) -> (-z, -rho), so with
// a = |z| and r = sign(z) rho, chi = a / log1p(t) with t = num/den chosen so
// that neither num nor den cancels:
//   a <= 1:  t = 2a / (s + (1 - a))
//   a >  1:  t = (s + (a - 1)) / (1 - r).
// At the removable singularity z = 0 (chi -> 1) the quotient a/log1p(t)
// stays accurate to a few ulps for every a > 0 (t has no cancellation and
// log1p is accurate for small t), so a is kept at kZFloor = 2^-60 or above
// instead of switching to the series: below it chi = 1 - rho z/2 + O(z^2)
// rounds to 1, and at a = kZFloor the quotient gives chi = 1 exactly
// (s + (1 - a) rounds to 2, t = a, log1p(t) rounds to t).  The floor keeps
// numer and denom (both carry the factor a) far from underflow, also in
// their product.  t >= 0 in the domain (|rho| < 1).
struct VolFrac {
  double numer, denom;
};

__device__ __forceinline__ VolFrac hagan2002_frac(const SabrConst &k, double L, double q,
                                                  double q3D1, double T) {
  const double z = k.nua * q * L;
  const double s = sqrt_gs(fma(z, z - 2.0 * k.rho, 1.0));
  const double az = fmax(fabs(z), kZFloor);
  const bool mid = az <= 1.0;
  const double num = mid ? 2.0 * az : s + (az - 1.0);
  const double den = mid ? s + (1.0 - az) : fma(-copysign(1.0, z), k.rho, 1.0);
  const double cn = az, cd = log1p_tang<false>(num * rcp_nr(den));   // chi = cn / cd
  const double Pq = fma(q, q, T * fma(q, fma(q, k.cc, k.cb), k.ca));
  VolFrac v;
  v.numer = k.alpha * Pq * cn;
  v.denom = q3D1 * cd;
  return v;
}

__device__ __forceinline__ double d1_term(double omb2, double L) {
  const double u = omb2 * L * L;
  return fma(u, fma(u, 1.0 / 1920.0, 1.0 / 24.0), 1.0);
}

// Paper eq. (sigmaHagan): sigma = (alpha/f^(1-b)) [1 - (1/2)(1-b - rho nu w) k
//   + (1/12)((1-b)^2 + (2 - 3 rho^2) nu^2 w^2 + 3((1-b) - rho nu w)) k^2],
// w = f^(1-b)/alpha, k = ln(K/f) = -L, fp = f^(1-b); as a fraction
// numer/denom like the Hagan 2002 form.
__device__ __forceinline__ VolFrac paper_eq3_frac(const SabrConst &k, double omb, double L,
                                                  double fp) {
  const double nu = k.nua * k.alpha;
  const double w = fp / k.alpha;
  const double rnw = k.rho * nu * w;
  const double kk = -L;
  const double c1 = -0.5 * (omb - rnw);
  const double c2 = (omb * omb + (2.0 - 3.0 * k.rho * k.rho) * nu * nu * w * w +
                     3.0 * (omb - rnw)) * (1.0 / 12.0);
  VolFrac v;
  v.numer = k.alpha * fma(kk, fma(kk, c2, c1), 1.0);
  v.denom = fp;
  return v;
}

// ---------------------------------------------------------------------------
// Black-76 on the out-of-the-money side (the call when K >= f, i.e. L <= 0;
// the other side follows by put-call parity, call - put = D (f - K)):
//   call = D [f N(d1) - K N(d2)],  put = D [K N(-d2) - f N(-d1)],
//   d1 = L/(sigma sqrt T) + sigma sqrt T / 2,  d2 = d1 - sigma sqrt T.
// With E = exp(-d1^2/2), K exp(-d2^2/2) = f E, and N(y) = E(y) X(y)/2 for
// y <= 0, 1 - E(y) X(y)/2 for y > 0, X(y) = erfcx(|y|/sqrt 2), one
// exponential serves both normal tails:
//   call (d2 < 0 always):  D f [d1 <= 0 ? E (X1 - X2)/2 : 1 - E (X1 + X2)/2]
//   put  (-d1 < 0 always): D [-d2 <= 0 ? f E (X2 - X1)/2 : K - f E (X1 + X2)/2].
// Takes 1/sigma so the caller can share one division between sigma and 1/sigma.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double black_otm(double f, double K, double L, double sqrtT,
                                            double isqrtT, double sigma, double isigma,
                                            double D) {
  const double sd = sigma * sqrtT;
  const double d1 = fma(L * isigma, isqrtT, 0.5 * sd);
  const double d2 = d1 - sd;
  double E, X1, X2;
  const double x1 = fabs(d1) * M_SQRT1_2;   // -d1^2/2 = -x1^2
  exp_erfcx2(-(x1 * x1), x1, fabs(d2) * M_SQRT1_2, E, X1, X2);
  const double hE = 0.5 * f * E;
  if (L <= 0.0)
    return D * (d1 <= 0.0 ? hE * (X1 - X2) : fma(-hE, X1 + X2, f));
  return D * (d2 >= 0.0 ? hE * (X2 - X1) : fma(-hE, X1 + X2, K));
}

// Intrinsic value to add to the out-of-the-money price to get the quoted side.
__device__ __forceinline__ double parity_shift(int kind, double f, double K, double L, double D) {
  const bool otm_call = L <= 0.0;
  const bool want_call = (kind == 0);
  if (want_call == otm_call) return 0.0;
  return want_call ? D * (f - K) : D * (K - f);
}

__device__ __forceinline__ double black_vega(double f, double L, double sqrtT, double sigma,
                                             double D) {
  const double sd = sigma * sqrtT;
  const double d1 = L / sd + 0.5 * sd;
  return D * f * exp(-0.5 * d1 * d1) * (0.39894228040143267794 * sqrtT);
}

}  // namespace sabr
