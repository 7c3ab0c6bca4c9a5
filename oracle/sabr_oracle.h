/*
 * sabr_oracle.h -- CPU reference ("oracle") for SA calibration of SABR/LIBOR
 * market models to caplet and swaption quotes.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct FP64 code used to
 * check the GPU library.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code with the GPU
 * library: no headers, helpers, tables or kernels.
 *
 * Source of every formula: Ferreiro, Garcia, Lopez-Salas, Vazquez,
 * "SABR/LIBOR market models: pricing and calibration for some interest rate
 * derivatives" (arXiv 2408.01470):
 *   - Hagan second-order moneyness formula, eq. (sigmaHagan), Sec. 2.1;
 *   - correlation parameterisations eq. (rhoij), (thetaij), (phiij), Sec. 2.1;
 *   - abcd volatility functions g_i, h_i, Sec. 2.3 (Rebonato model);
 *   - caplet cost f_c and swaption cost f_s, Sec. 3;
 *   - simulated annealing loop (boxed pseudocode) and the synchronous
 *     one-GPU parallel variant (restart of all chains at the best final
 *     point of each temperature level), Sec. 3.
 * Where the paper names a formula without printing it (the full Hagan 2002
 * lognormal expansion with z/x(z), Black-76) the oracle writes out the
 * textbook definition.  Items the paper leaves open (neighbour rule, search
 * box, swaption closed form, LM polish) follow the readings listed in the
 * design notes of the repository.
 *
 * All arrays are HOST memory owned by the caller.  Return 0 on success,
 * negative on invalid input (message via oracle_last_error()).
 */
#ifndef SABR_ORACLE_H
#define SABR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* CSR batch of independent markets (instances); indices are local to the
 * instance (und_first into its forwards, q_und into its underlyings). */
typedef struct {
  int32_t n_inst;
  const int32_t *fwd_off;                 /* [n_inst+1] */
  const double *fwd_T, *fwd_tau, *fwd_F, *fwd_P; /* fixing, accrual, F_i(0), P(0,T_i+tau_i) */
  const int32_t *und_off;                 /* [n_inst+1] */
  const int32_t *und_first, *und_len;     /* forward range [first, first+len) */
  const int32_t *q_off;                   /* [n_inst+1] */
  const int32_t *q_und, *q_kind;          /* underlying, 0 = call/payer, 1 = put/receiver */
  const double *q_K, *q_vol, *q_w;        /* strike, market implied vol, user weight */
  int32_t model;                          /* 0 GLOBAL4, 1 LMM12, 2 PERFWD, 3 MM, 4 REB */
  int32_t formula;                        /* 0 = Hagan 2002, 1 = paper eq. (sigmaHagan) */
  int32_t residual;                       /* 0 = vol residuals, 1 = Black price residuals */
  double beta;                            /* fixed beta (all but GLOBAL4) */
} oracle_market;

const char *oracle_last_error(void);
int32_t oracle_num_params(int32_t model);
/* Parameters per point of a market (3 per forward for PERFWD, 2 per forward
 * plus one for MM, 2 per forward plus 8 for REB, whose instances must hold
 * equally many forwards); -1 if invalid.  Gradients and LM take GLOBAL4 and
 * LMM12 markets only. */
int32_t oracle_market_num_params(const oracle_market *m);
/* OpenMP threads of the calls below (n > 0); for timing on one core. */
void oracle_set_threads(int32_t n);
int32_t oracle_max_threads(void);   /* OpenMP threads the parallel loops use */

/* Single-quote primitives (pins). */
double oracle_hagan2002_vol(double f, double K, double T, double alpha, double beta,
                            double rho, double nu);
double oracle_paper_eq3_vol(double f, double K, double alpha, double beta, double rho,
                            double nu);
double oracle_chi(double z, double rho);               /* z / x(z), chi(0) = 1 */
double oracle_black(int32_t kind, double f, double K, double T, double sigma, double D);
double oracle_black_vega(double f, double K, double T, double sigma, double D);
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Per-underlying SABR parameters (alpha, beta, rho, nu) of one parameter
 * point for instance `inst`: out[4*n_und]. */
int32_t oracle_map_params(const oracle_market *m, int32_t inst, const double *p, double *out);

/* Market-derived quantities per underlying: S0, annuity A, expiry T. */
int32_t oracle_underlyings(const oracle_market *m, int32_t inst, double *S0, double *A,
                           double *T);

/* Model values (vol or price, per residual mode) and the effective market
 * target and weight used by the cost: per quote of instance `inst`. */
int32_t oracle_model_values(const oracle_market *m, int32_t inst, const double *p,
                            double *model, double *target, double *weight);

/* cost[i] = sum_q w_q (m_q - mkt_q)^2 for point i of instance pt_inst[i];
 * resid (nullable) gets r_q, row stride = max quotes per instance. */
int32_t oracle_cost_batch(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                          const double *params, double *cost, double *resid,
                          int32_t resid_stride);

/* Exact gradient of the cost (forward-mode dual numbers):
 * grad[i*P + k] = d cost_i / d p_k.  jtwj [n_pts][P][P], jtwr [n_pts][P] nullable. */
int32_t oracle_cost_grad(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                         const double *params, double *cost, double *grad, double *jtwj,
                         double *jtwr);

typedef struct {
  double T0;          /* initial temperature */
  double cool;        /* T_{l+1} = cool * T_l */
  double step_frac;   /* neighbour half-width as a fraction of (ub - lb) */
  int32_t n_levels;   /* L */
  int32_t n_steps;    /* N */
  uint64_t seed;      /* Philox key word 0; key word 1 = instance id */
  const double *T0_per_inst; /* nullable */
  int32_t level0;            /* first level index: the Philox counter of step s of run level l
                                is (level0 + l) N + s; without state_in, T starts at
                                T0 cool^level0 (repeated multiplication) */
  const int32_t *inst_key;   /* nullable [n_inst]: Philox key word 1 per instance (default: the
                                instance index), so one instance of a batch runs alone */
  const double *state_in;    /* nullable: resume from this state (no initial evaluation) */
  double *state_out;         /* nullable: the state after the last level (its restart done,
                                T cooled) */
} oracle_sa_config;
/* State layout (state_in, state_out): per instance, in order, with C its
 * chains: X [C][P], F [C], BX [C][P], BF [C] (current and best-ever points
 * and costs), T (the next level's temperature): 2 C (P + 1) + 1 doubles. */

/* Mirrors of sabr_cost_batch and sabr_cost_vjp (include/sabr.h) with the
 * same argument lists on host pointers, without stream and workspace:
 * cost[i] (+inf on a domain failure, NaN for an out-of-range pt_inst[i]),
 * resid and model (nullable) at [i*stride + q] in the caller's quote order
 * (stride >= the largest instance's quote count); g_params[i*P + k] =
 * g_cost[i] (nullable -> 1) * d cost_i / d p_k, jtwj and jtwr (nullable) as
 * oracle_cost_grad.  oracle_sa_calibrate is the mirror of sa_calibrate (its
 * last argument, n_evals, in place of the workspace and the stream). */
int32_t oracle_sabr_cost_batch(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                               const double *params, double *cost, double *resid, double *model,
                               int32_t stride);
int32_t oracle_sabr_cost_vjp(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                             const double *params, const double *g_cost, double *cost,
                             double *g_params, double *jtwj, double *jtwr);

/* Synchronous parallel SA, chains[i] chains on instance i.
 * best_x [n_inst][P], best_f [n_inst]; nullable outputs:
 *   chain_best_x [sum chains][P], chain_best_f [sum chains]   (per-chain best ever)
 *   accept      [n_inst] blocks of [L][N][chains[i]] bytes  (offset by prefix sums)
 *   level_trace [n_inst][L][3] = {best-ever f, acceptance rate, 0}
 *   level_best  [n_inst][L] = level-end argmin chain (restart point index)
 * n_evals [n_inst] nullable: cost evaluations performed. */
int32_t oracle_sa_calibrate(const oracle_market *m, const oracle_sa_config *cfg,
                            const int32_t *chains, const double *lb, const double *ub,
                            const double *x0, double *best_x, double *best_f,
                            double *chain_best_x, double *chain_best_f, uint8_t *accept,
                            double *level_trace, int32_t *level_best, int64_t *n_evals);

/* Level 0 of the same annealing for sampled chains (chains are independent
 * until the first level end): sample j is chain sample_chain[j] of instance
 * sample_inst[j]; accept [n_sample][N], F_out / BF_out [n_sample] (final and
 * best-ever cost), BX_out [n_sample][P] (best-ever point). */
int32_t oracle_sa_level0_sample(const oracle_market *m, const oracle_sa_config *cfg,
                                const int32_t *chains, const double *lb, const double *ub,
                                const double *x0, int32_t n_sample, const int32_t *sample_inst,
                                const int32_t *sample_chain, uint8_t *accept, double *F_out,
                                double *BF_out, double *BX_out);

/* One chain's N steps of one level, step by step (proposal xp_out [N][P],
 * its cost fp_out [N], acceptance uniform u_out [N], accept flag acc_out
 * [N]) from point x with cost f at temperature T; lb, ub [n_inst][P]. */
int32_t oracle_sa_chain_steps(const oracle_market *m, const oracle_sa_config *cfg, int32_t inst,
                              int32_t chain, int32_t level, double T, const double *lb,
                              const double *ub, const double *x, double f, double *xp_out,
                              double *fp_out, double *u_out, uint8_t *acc_out);

/* Projected Levenberg-Marquardt polish of n_pts points (in place). */
int32_t oracle_lm_polish(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                         double *params, const double *lb, const double *ub,
                         int32_t max_iter, double mu0, double tol, double *cost_out,
                         int32_t *iters_out);

/* Nelder-Mead polish in place (reflection 1, expansion 2, contraction 1/2,
 * shrink 1/2, trial points clamped into the box; initial simplex x0 and
 * x0 + step (ub_k - lb_k) e_k; stop when f_worst - f_best <= tol |f_best|
 * or after max_iter iterations).  Every model. */
int32_t oracle_nm_polish(const oracle_market *m, int32_t n_pts, const int32_t *pt_inst,
                         double *params, const double *lb, const double *ub, int32_t max_iter,
                         double step, double tol, double *cost_out, int32_t *iters_out);

/* Philox4x32-10 block (Salmon et al., SC 2011). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The 2M standard normals of Monte Carlo step `step` on path `path`. */
void oracle_mc_normals(uint64_t seed, int64_t path, int64_t step, int32_t M, double *xi);

/* Steps of a fixing interval of length len at step size dt. */
int32_t oracle_mc_steps(double len, double dt);

/* Monte Carlo under the Hagan SABR/LIBOR dynamics (Sec. 2.1) under the spot
 * measure: X[p][o] = discounted payoff of option o (payer swaption
 * (opt_a, opt_b, opt_K); opt_b = opt_a + 1: caplet) on path path0 + p.
 * Forward arrays [M]; y = (eta1, lambda1, eta2, lambda2, lambda3); B [2M][2M]
 * the correlation factor (rows W_0..W_{M-1}, Z_0..Z_{M-1}; the rows of
 * forwards k >= j vanish beyond column 2(M - j)); P0 = P(0, T_0). */
int32_t oracle_mc_paths(int32_t M, const double *T, const double *tau, const double *F0,
                        const double *alpha, const double *beta, const double *phi,
                        const double *sigma, const double *y, double P0, const double *B,
                        int32_t n_opt, const int32_t *opt_a, const int32_t *opt_b,
                        const double *opt_K, int64_t path0, int64_t n_paths, double dt,
                        uint64_t seed, double *X);

#ifdef __cplusplus
}
#endif
#endif
