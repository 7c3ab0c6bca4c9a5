// sabr_internal.hpp -- interface between the C-ABI runtime (sabr_api.cpp) and
// the kernels (sabr_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sabr_device.hpp"

namespace sabr {

// Swaps of up to this many forwards keep the map's per-lane recursion column
// in registers; longer ones in LDS.
constexpr int kMapRegLen = 16;

// Doubles of LDS one wavefront needs for the LMM12 and PERFWD maps: a 48-byte
// record per forward (alpha, nu, the two correlation gap factors, v alpha;
// unused by PERFWD), a 48-byte record of SABR constants per underlying, and
// (for swaps longer than kMapRegLen) a per-lane column of max_len doubles for
// the swap recursion.
// Each workgroup adds 6 doubles per underlying of market values.
// The cost evaluation (point_cost) takes the LMM12 underlyings thchunk at a
// time (128, or 64 for markets of more than 128 underlyings), so its table
// holds min(max_nu, thchunk) records; the adjoint's whole-map table (full)
// holds max_nu.
__host__ __device__ inline int th_chunk_for(int max_nu) { return max_nu <= 128 ? 128 : 64; }
// Waves (chains) per annealing workgroup at most: the instance's market
// values staged in LDS are shared by the workgroup's waves.
constexpr int kMaxWavesPerGroup = 8;
__host__ __device__ inline int th_entries(const DevMarket &m, bool full) {
  return (m.model == 1 && !full && m.max_nu > m.thchunk) ? m.thchunk : m.max_nu;
}

// Whether the wave's layout holds the per-lane LDS column of the swap
// recursion: swaps longer than kMapRegLen, unless the cost kernels keep them
// in registers (reglen; the adjoint's whole map always uses the column).
__host__ __device__ inline bool lds_column(const DevMarket &m, bool full) {
  return m.max_len > kMapRegLen && (full || m.reglen < m.max_len);
}

__host__ __device__ inline int wave_lds_doubles(const DevMarket &m, bool full = false) {
  if (m.model == 0) return 0;
  return 6 * m.max_nf + kSabrConstDoubles * th_entries(m, full) +
         (lds_column(m, full) ? kWave * m.max_len : 0);
}

// Kernel variant of a plan: the model, or 5 for LMM12 with the swap column in
// 24 registers (swaps of 17 to 24 forwards).
__host__ __device__ inline int kernel_model(const DevMarket &m) {
  return (m.model == 1 && m.reglen == 24) ? 5 : m.model;
}

// Steps whose uniforms one Philox pass of the annealing kernel produces: a
// step takes P + 1 uniforms, the words of (P + 4) / 4 Philox blocks; lane l
// of the chain's lanes (the wave, or its half for paired chains) computes
// block l mod nb of step l / nb, at most kUniSteps steps a pass, and the
// uniforms wait in LDS.
constexpr int kUniSteps = 16;
__host__ __device__ constexpr int uni_blocks(int P) { return (P + 4) / 4; }
__host__ __device__ constexpr int uni_steps(int P, int lanes = kWave) {
  return lanes / uni_blocks(P) < kUniSteps ? lanes / uni_blocks(P) : kUniSteps;
}

// Doubles of LDS per wave of the annealing kernels: the map's scratch and
// uni_steps(P) x (P + 1) uniforms per chain of the wave (two with pair).
__host__ __device__ inline int sa_wave_doubles(const DevMarket &m, bool pair = false) {
  return wave_lds_doubles(m) +
         (pair ? 2 * uni_steps(m.np, kHalf) : uni_steps(m.np)) * (m.np + 1);
}

// Paired chains (two chains per wave, one per half) need a map that is plain
// per-lane arithmetic of the point and at most 32 coordinates: GLOBAL4.
__host__ __device__ inline bool pair_capable(const DevMarket &m) { return m.model == 0; }

struct SAArgs {
  int n_inst, P, N, L;
  int wpc;                      // waves per chain: 1, or every wave of a one-chain workgroup
  int cpw;                      // chains per wave: 1, or 2 (one per half-wave; GLOBAL4)
  int level0;                   // index of the first level (Philox counters, temperature)
  uint64_t seed;
  double step_frac, cool, ns_per_tick;
  const int *chains;            // [n_inst]
  const int64_t *chain_base;    // [n_inst] first global chain of each instance
  const int64_t *acc_base;      // [n_inst] offset of each instance's accept flags
  const int *tile_inst;         // [n_tiles]
  const int *tile_chain;        // [n_tiles] first chain of the tile
  const int *tile_off;          // [n_inst + 1] each instance's tiles, in chain order
  // per-tile partials of the level end, written by the init and level
  // kernels: lowest final cost and its chain (ties: lowest chain), lowest
  // best-ever cost and its chain, accepted moves of the level
  double *TF, *TB;
  int *TI, *TJ, *TN;
  const double *lb, *ub, *x0;   // [n_inst][P]
  const double *T0;             // [n_inst]
  double *X, *BX, *BF;          // per-chain final point, best-ever point and cost
  double *RX, *RF, *Tcur;       // per-instance restart point and temperature
  uint64_t *t_start;            // wall clock at initialisation
  uint8_t *accept;              // nullable: [inst][level][step][chain]
  double *trace;                // nullable: [inst][level][3]
  int *level_best;              // nullable: [inst][level]
  double *best_x, *best_f;      // [n_inst][P], [n_inst]
  double *chain_best_x, *chain_best_f;  // nullable
  // nullable: the annealing state to resume from, and the state after the
  // last level; per instance X [C][P], F [C], BX [C][P], BF [C], T, i.e.
  // 2 C (P + 1) + 1 doubles from 2 (P + 1) chain_base + instance index
  const double *state_in;
  double *state_out;
};

hipError_t launch_prep(const DevMarket &m, QuoteRec *q, double *f_v, double *u_S0b, double *u_c0,
                       double *u_fp,
                       const double *q_vol, const double *q_wuser, const int *q_und_g,
                       const double *f_tauP, const double *f_F, int n_q, int n_f, int n_u,
                       hipStream_t s);

hipError_t launch_cost(const DevMarket &m, int n_pts, const int *pt_inst, const double *params,
                       double *cost, double *resid, double *model, int stride, hipStream_t s);

hipError_t launch_sa_init(const DevMarket &m, const SAArgs &a, int n_tiles, int waves,
                          hipStream_t s);
hipError_t launch_sa_level(const DevMarket &m, const SAArgs &a, int level, int n_tiles,
                           int waves, int occupancy, hipStream_t s);
// max_tiles: the most workgroups (tiles) any instance has; sizes the
// level-end block (256 threads, 1024 beyond 1024 tiles).
hipError_t launch_sa_level_end(const SAArgs &a, int level, int max_tiles, hipStream_t s);
hipError_t launch_sa_final(const SAArgs &a, hipStream_t s);
hipError_t launch_sa_state_out(const SAArgs &a, hipStream_t s);

// Bytes of the fixed per-device scratch array of the allocation-free
// annealing entry point, and the current device's address of it (looked up
// on the first call on each device).
constexpr size_t kSaNoallocBytes = (size_t)64 << 20;
hipError_t sa_noalloc_scratch(void **ptr);

// Wavefronts per SA/cost workgroup that fit the LDS budget (at most `want`),
// with one chain per wave or two (pair).
int sa_waves_per_group(const DevMarket &m, int want, bool pair = false);

}  // namespace sabr
