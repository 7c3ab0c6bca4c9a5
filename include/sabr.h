/*
 * sabr.h -- C ABI of the MI355X (gfx950) simulated-annealing calibrator of
 * SABR/LIBOR market models to caplet and swaption quotes.
 *
 * Method: Ferreiro, Garcia, Lopez-Salas, Vazquez, "SABR/LIBOR market models:
 * pricing and calibration for some interest rate derivatives"
 * (arXiv 2408.01470).  The library minimises the weighted quote cost
 *     f(p) = sum_q w_q (m_q(p) - mkt_q)^2
 * (the caplet cost f_c and swaption cost f_s of Sec. 3, with weights) over a
 * box by synchronous parallel simulated annealing (Sec. 3: the boxed SA loop
 * T <- rho T, N Metropolis steps per level, all chains restarted at the best
 * final point of each level), where m_q is the Hagan implied vol of quote q
 * (Sec. 2.1, eq. (sigmaHagan), or the full Hagan 2002 lognormal expansion the
 * paper cites) or its Black-76 price.
 *
 * Conventions
 *  - Market data enter once, as HOST arrays, through sabr_plan_create (which
 *    validates everything before any GPU work) and sabr_plan_upload (which
 *    copies a packed image into caller-owned DEVICE memory).
 *  - Every other array argument is DEVICE memory owned by the caller unless
 *    marked [host].  The library never frees or retains caller pointers
 *    beyond the plan's device image (valid until the plan is destroyed or
 *    re-uploaded).
 *  - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL
 *    = default stream); results are valid after the stream is synchronised.
 *  - Return values: SABR_OK, or a negative sabr_status; sabr_last_error()
 *    gives a thread-local message.  Invalid arguments are reported before
 *    anything is enqueued.
 *  - Domain failures are not errors: a point whose parameters leave the
 *    model's domain (alpha <= 0, |rho| >= 1, nu < 0, a model vol that is not
 *    finite and positive, ...) gets cost +inf.
 *  - All arithmetic is IEEE FP64.
 */
#ifndef SABR_H
#define SABR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SABR_OK = 0,
  SABR_EINVAL = -1,        /* invalid argument or market data */
  SABR_ENOMEM = -2,        /* host allocation failed */
  SABR_EHIP = -3,          /* HIP runtime error */
  SABR_EUNSUPPORTED = -4,  /* combination not supported */
  SABR_EWORKSPACE = -5     /* device buffer too small */
} sabr_status;

/* Parameter layouts.
 *  GLOBAL4: p = (alpha, beta, rho, nu) shared by every forward (the Hagan
 *           model with common parameters: x = (phi_ii, sigma_i, alpha_i) of
 *           Sec. 3 with phi_ii = rho, sigma_i = nu).  Caplet markets only.
 *  LMM12:   p = (a, b, c, d, a_nu, b_nu, c_nu, d_nu, rho, lambda1, eta2,
 *           lambda2), beta fixed (sabr_problem.beta):
 *             alpha_i = (a + b T_i) exp(-c T_i) + d   (abcd form, Sec. 2.3)
 *             nu_i    = (a_nu + b_nu T_i) exp(-c_nu T_i) + d_nu
 *             phi_ii = rho, rho_ij = exp(-lambda1 |T_i - T_j|)  (eq. (rhoij), eta1 = 0)
 *             theta_ij = eta2 + (1 - eta2) exp(-lambda2 |T_i - T_j|)  (eq. (thetaij))
 *             phi_ij = rho  (eq. (phiij), lambda3 = 0).
 *           A swaption on forwards [e, e+n) gets SABR parameters from a
 *           first-order freeze of dS = sum_k w_k dF_k at t = 0 (the paper
 *           prices swaptions by Monte Carlo; this closed-form map replaces it):
 *             u_k = w_k F_k^beta, a_k = u_k alpha_k, R_k = sum_l a_l rho_kl,
 *             V = sum_k a_k R_k, alpha_S = sqrt(V) / S0^beta,
 *             c_k = a_k R_k / V, nu_S^2 = sum_kl c_k c_l nu_k nu_l theta_kl,
 *             rho_S = sum_kl a_k c_l nu_l phi_kl / (alpha_S S0^beta nu_S).
 *  PERFWD:  p = (alpha_1, rho_1, nu_1, ..., alpha_n, rho_n, nu_n), one triple
 *           per forward of the instance, beta fixed (sabr_problem.beta): the
 *           Hagan model of Sec. 3 with per-forward parameters
 *           x = (phi_ii, sigma_i, alpha_i) (phi_ii = rho_i, sigma_i = nu_i),
 *           calibrated to caplets in Sec. 4.1.1.  Caplet markets only; every
 *           instance holds the same number n <= 21 of forwards, P = 3 n.
 *           Every triple must lie in the domain, quoted or not.  The adjoint
 *           and LM entry points return SABR_EUNSUPPORTED for it (its cost
 *           separates per forward: polish each forward as a GLOBAL4 instance
 *           with beta frozen by lb = ub).
 *  MM:      p = (alpha_1, phi_1, ..., alpha_n, phi_n, sigma), beta fixed: the
 *           Mercurio-Morini model of Sec. 2.2 (x = (phi_i, sigma, alpha_i)) with
 *           the SABR parameters of eq. (haganForMercurio): rho_i = phi_i,
 *           nu_i = sigma, alpha_i^SABR = alpha_i exp(-sigma D_i),
 *           D_i = sum_{j<=i} T_{j-1} tau_j phi_j alpha_j F_j^beta / (1 + tau_j F_j)
 *           with T_{j-1} the previous forward's fixing (0 for the first): the
 *           drift sum runs from the forward after the first unfixed one.
 *           Caplet markets only; every instance holds the same number
 *           n <= 31 of forwards, P = 2 n + 1.  Domain: alpha_j > 0,
 *           |phi_j| < 1, sigma >= 0.  The adjoint and LM entry points return
 *           SABR_EUNSUPPORTED for it.
 *  REB:     p = (kappa_1, phi_1, ..., kappa_n, phi_n, a, b, c, d, a_h, b_h,
 *           c_h, d_h), beta fixed: the Rebonato model of Sec. 2.2 (x = (phi_ii,
 *           kappa_i, the parameters of g and h)) with the SABR parameters of
 *           eq. (haganForRebonato) for the caplet on forward i, expiry T:
 *             alpha_i = kappa_i sqrt(G / T), G = int_0^T g_i(t)^2 dt,
 *             nu_i = sqrt(2 J / (T G)), J = int_0^T g_i(t)^2 H_i(t) dt,
 *             H_i(t) = int_0^t h_i(s)^2 ds, rho_i = phi_i,
 *           g_i(t) = (a + b (T - t)) e^{-c (T - t)} + d, h_i likewise; G and
 *           H in closed form, J by the 32-point Gauss-Legendre rule.
 *           Caplet markets only; every instance holds the same number
 *           n <= 27 of forwards, P = 2 n + 8.  Domain: kappa_i > 0,
 *           |phi_i| < 1, c >= 0, c_h >= 0, G > 0.  The adjoint and LM entry
 *           points return SABR_EUNSUPPORTED for it. */
typedef enum {
  SABR_MODEL_GLOBAL4 = 0,
  SABR_MODEL_LMM12 = 1,
  SABR_MODEL_PERFWD = 2,
  SABR_MODEL_MM = 3,
  SABR_MODEL_REB = 4
} sabr_model;

/* Implied-vol formula.
 *  HAGAN2002: L = ln(f/K), q = (fK)^((1-beta)/2), z = (nu/alpha) q L,
 *    sigma = alpha/(q D1) * z/x(z) * [1 + ((1-beta)^2 alpha^2/(24 q^2)
 *            + rho beta nu alpha/(4q) + (2 - 3 rho^2) nu^2/24) T],
 *    x(z) = ln((sqrt(1 - 2 rho z + z^2) + z - rho)/(1 - rho)),
 *    D1 = 1 + (1-beta)^2 L^2/24 + (1-beta)^4 L^4/1920.
 *  PAPER_EQ3: eq. (sigmaHagan) of Sec. 2.1 exactly as printed (second order
 *    in ln(K/f), no expiry dependence). */
typedef enum { SABR_VOL_HAGAN2002 = 0, SABR_VOL_PAPER_EQ3 = 1 } sabr_vol_formula;

/* Residual: model vol minus market vol, or Black-76 price minus the Black
 * price of the market vol (weight divided by the market vega squared). */
typedef enum { SABR_RES_VOL = 0, SABR_RES_PRICE = 1 } sabr_residual;

/* Quote kinds: call (caplet, payer swaption) or put (floorlet, receiver). */
typedef enum { SABR_Q_CALL = 0, SABR_Q_PUT = 1 } sabr_quote_kind;

/* A CSR batch of n_inst independent markets (instances), all [host].
 * Instance i owns forwards [fwd_off[i], fwd_off[i+1]), underlyings
 * [und_off[i], und_off[i+1]) and quotes [q_off[i], q_off[i+1]).  Indices
 * stored in und_first and q_und are local to the instance.  An underlying is
 * the swap over forwards [first, first+len): len = 1 is a caplet on that
 * forward, with expiry T_first, annuity A = sum tau_k P_k, weights
 * w_k = tau_k P_k / A and swap rate S0 = sum w_k F_k.  Quotes must be sorted
 * by underlying within each instance. */
typedef struct {
  int32_t n_inst;
  const int32_t *fwd_off;                         /* [n_inst+1] */
  const double *fwd_T, *fwd_tau, *fwd_F, *fwd_P;  /* fixing, accrual, F(0), P(0, T+tau) */
  const int32_t *und_off;                         /* [n_inst+1] */
  const int32_t *und_first, *und_len;
  const int32_t *q_off;                           /* [n_inst+1] */
  const int32_t *q_und, *q_kind;
  const double *q_K, *q_vol, *q_w;                /* strike, market implied vol, weight */
  int32_t model, vol_formula, residual;
  double beta;                                    /* fixed beta (LMM12, PERFWD, MM), in [0, 1] */
} sabr_problem;

typedef struct sabr_plan sabr_plan; /* opaque; host memory only */

/* Validate the market (offsets monotone and in range, positive finite
 * forwards, strikes, accruals, discounts and vols, non-negative weights,
 * positive expiries, quotes sorted by underlying, swaps in LMM12 markets
 * only, PERFWD, MM and REB instances of equal size) and
 * build its packed image.  On success *out owns host memory only. */
sabr_status sabr_plan_create(const sabr_problem *prob /*[host]*/, sabr_plan **out /*[host]*/);
void sabr_plan_destroy(sabr_plan *plan);

/* Bytes of device memory the plan's image needs (256-byte aligned blocks). */
size_t sabr_plan_device_bytes(const sabr_plan *plan);

/* Copy the image into dev_buf (device, >= sabr_plan_device_bytes) and run the
 * market precompute kernel (logs, square roots, fixed-beta powers, Black
 * market prices and vegas in price mode).  The plan keeps dev_buf. */
sabr_status sabr_plan_upload(sabr_plan *plan, void *dev_buf, size_t bytes, void *stream);

int32_t sabr_num_params(int32_t model);  /* 4 or 12; -1 if unknown, PERFWD, MM or REB */
/* P of the plan (PERFWD 3 n, MM 2 n + 1, REB 2 n + 8) */
int32_t sabr_plan_num_params(const sabr_plan *plan);
int32_t sabr_plan_num_inst(const sabr_plan *plan);
int32_t sabr_plan_max_quotes(const sabr_plan *plan); /* largest quotes per instance */

/* Swap rate S0, annuity A and expiry T of every underlying [host out,
 * concatenated over instances in CSR order]. */
sabr_status sabr_plan_underlyings(const sabr_plan *plan, double *S0, double *A, double *T);

/* Cost of n_pts points: point i belongs to instance pt_inst[i] and has
 * parameters params[i*P .. i*P+P).  cost[i] = sum_q w_q (m_q - mkt_q)^2 over
 * that instance's quotes, +inf on a domain failure, NaN if pt_inst[i] is out
 * of range.  resid (nullable) receives r_q = m_q - mkt_q at
 * resid[i*stride + q]; model (nullable) receives m_q (vol or price, per the
 * residual mode) at model[i*stride + q].  stride >= max quotes per instance
 * when either is given.  (Sec. 3, f_c and f_s.) */
sabr_status sabr_cost_batch(const sabr_plan *plan, int32_t n_pts, const int32_t *pt_inst,
                            const double *params, double *cost, double *resid, double *model,
                            int32_t stride, void *stream);

/* Annealing schedule and options (Sec. 3 boxed SA loop: T_0 = T0,
 * T_{l+1} = cool * T_l by FP64 multiplication, N = n_steps Metropolis steps
 * per level, n_levels levels). */
typedef struct {
  double T0;             /* initial temperature (> 0) */
  double cool;           /* cooling factor in (0, 1] */
  double step_frac;      /* neighbour half-width as a fraction of (ub - lb), (0, 1] */
  int32_t n_levels;      /* L >= 0 */
  int32_t n_steps;       /* N >= 0 */
  uint64_t seed;         /* Philox key word 0; key word 1 = instance index */
  const double *T0_per_inst; /* [host] nullable [n_inst] per-instance T0 */
  int32_t waves_per_group;   /* chains per workgroup, at most 8 (0 = library default 4) */
  int32_t use_graph;         /* 1: capture the launch sequence in a hipGraph and replay it */
  void *const *level_events; /* [host] nullable: 2 * n_levels hipEvent_t recorded on `stream`
                                just before and just after each level's annealing kernel
                                (eager launches only; ignored when use_graph = 1); a null
                                pair skips that level */
  int32_t occupancy;         /* register budget of the level kernel: minimum waves per SIMD
                                (0 or 1 = compiler's choice, 3, 4); a tuning knob */
  int32_t waves_per_chain;   /* 0 or 1: one wave per chain; 2..8: each chain is a workgroup of
                                that many waves splitting its quotes (blocks of 64, round
                                robin), for few chains of many quotes; waves_per_group is then
                                ignored.  The cost sums the waves' partials in wave order, so
                                it may differ from the one-wave sum in the last bits.
                                SABR_EINVAL when the waves' LDS does not fit a workgroup */
  int32_t chains_per_wave;   /* 0 or 1: one chain per wave; 2: two chains per wave, one per
                                half (32 lanes): each half proposes, prices the quotes 32 at a
                                time and takes its Metropolis decision on its own, for many
                                chains of few quotes (the per-step work and the last, partial
                                pass of quotes are shared by two chains).  Same Philox streams
                                and accept rules, and the same results bit for bit: each half
                                keeps the partial sums of the 64 lanes one wave would use and
                                adds them in the same order.  GLOBAL4 plans only, and not with
                                waves_per_chain > 1: SABR_EINVAL */
  int32_t level0;            /* index of the first level (>= 0, else SABR_EINVAL): step s of run
                                level l draws the Philox counter (level0 + l) N + s, and without
                                state_in the temperature starts at T0 cool^level0 (repeated
                                multiplication).  A run of L levels equals a run of l levels
                                with state_out followed by L - l levels from level0 = l with
                                that state as state_in, bit for bit */
  const double *state_in;    /* [device] nullable: resume from this annealing state (layout
                                below) instead of evaluating x0; T is the state's.  Every chain
                                of an instance must sit at one point with one cost, as in every
                                state sa_calibrate or the CPU oracle writes; x0 is then unused */
  double *state_out;         /* [device] nullable: the state after the last level (its restart
                                done, T cooled).  Layout, per instance i in order with C its
                                chains: X [C][P], F [C] (every chain's point and cost), BX [C][P],
                                BF [C] (best-ever points and costs), T: 2 C (P + 1) + 1 doubles,
                                starting at 2 (P + 1) (chains of instances before i) + i */
} sa_config;

/* Device workspace bytes sa_calibrate needs for these chain counts. */
size_t sa_workspace_size(const sabr_plan *plan, const sa_config *cfg /*[host]*/,
                         const int32_t *chains /*[host][n_inst]*/);

/* Synchronous parallel simulated annealing on every instance at once.
 * Instance i runs chains[i] >= 1 Markov chains in the box [lb, ub]
 * ([host][n_inst][P], lb <= ub) from x0 ([host] nullable -> box midpoint).
 * Step s of level l of chain c of instance i draws u_0..u_P from
 * Philox4x64-10 with counter (l N + s, c, b, 0) and key (seed, i), block b =
 * 0, 1, ..., word j of the concatenation, u = (word >> 11) 2^-53; the
 * proposal is x'_k = x_k + step_frac (ub_k - lb_k)(2 u_k - 1) mirrored into
 * the box then clamped; it is accepted iff f' - f <= 0 or
 * u_P < exp(-(f' - f)/T_l).  At each level end every chain restarts at the
 * final point of lowest cost (ties -> lowest chain index).
 * Outputs (device): best_x [n_inst][P], best_f [n_inst] = best point ever
 * evaluated; nullable: chain_best_x [sum chains][P] / chain_best_f [sum
 * chains] (per-chain best ever), accept [sum_i L N chains[i]] bytes in
 * (instance, level, step, chain) order, level_trace [n_inst][L][3] =
 * {best-ever f, acceptance rate, ns since start}, level_best [n_inst][L] =
 * restart chain of each level.  Cost evaluations: chains[i] (1 + N L). */
sabr_status sa_calibrate(const sabr_plan *plan, const sa_config *cfg /*[host]*/,
                         const int32_t *chains /*[host]*/, const double *lb /*[host]*/,
                         const double *ub /*[host]*/, const double *x0 /*[host] nullable*/,
                         double *best_x, double *best_f, double *chain_best_x,
                         double *chain_best_f, uint8_t *accept, double *level_trace,
                         int32_t *level_best, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of the fixed device scratch of sa_calibrate_noalloc (64 MiB). */
#define SA_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/* sa_calibrate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, results and errors as sa_calibrate, without the
 * workspace.  The scratch is a fixed array of SA_NOALLOC_MAX_BYTES bytes in
 * the library's device code, one per device, held until the process ends;
 * its address for the current device is looked up on the first call there.
 * A call whose sa_workspace_size exceeds SA_NOALLOC_MAX_BYTES fails with
 * SABR_EWORKSPACE; use_graph must be 0 (SABR_EINVAL otherwise).  The call
 * allocates no device memory (the small host tables go through the plan's
 * own staging buffer, as in sa_calibrate).  Every call on one device shares
 * that device's array and leaves its contents there: calls that overlap on
 * one device (concurrent streams or threads) race and must be serialised by
 * the caller.  Nothing in the array needs to start at zero: every word is
 * written by the call before it is read. */
sabr_status sa_calibrate_noalloc(const sabr_plan *plan, const sa_config *cfg /*[host]*/,
                                 const int32_t *chains /*[host]*/, const double *lb /*[host]*/,
                                 const double *ub /*[host]*/,
                                 const double *x0 /*[host] nullable*/, double *best_x,
                                 double *best_f, double *chain_best_x, double *chain_best_f,
                                 uint8_t *accept, double *level_trace, int32_t *level_best,
                                 void *stream);

/* Device workspace bytes sabr_lm_polish needs (the box tables; independent
 * of n_pts).  sabr_cost_vjp needs none. */
size_t sabr_adjoint_workspace_size(const sabr_plan *plan, int32_t n_pts);

/* Hand-written adjoint of the cost (reverse sweep of the implied-vol formula,
 * Black-76 and the parameter map): for point i,
 *   g_params[i*P + k] = g_cost[i] * d cost_i / d p_k   (g_cost nullable -> 1),
 *   cost[i] (nullable)   = cost_i,
 *   jtwj[i*P*P ..] (nullable) = J^T W J,  jtwr[i*P ..] (nullable) = J^T W r,
 * with r_q the residuals, W = diag(w_q) and J_q = d r_q / d p; note
 * d cost/d p = 2 J^T W r.  Out-of-domain points give cost +inf and zero
 * derivatives.  The derivative of the cost follows from the paper's f_c and
 * f_s (Sec. 3); the paper itself polishes with Nelder-Mead and has no
 * gradient.  GLOBAL4 and LMM12 plans (PERFWD, MM, REB: SABR_EUNSUPPORTED).
 * workspace, ws_bytes: unused (may be null and 0; kept for ABI stability). */
sabr_status sabr_cost_vjp(const sabr_plan *plan, int32_t n_pts, const int32_t *pt_inst,
                          const double *params, const double *g_cost, double *cost,
                          double *g_params, double *jtwj, double *jtwr, void *workspace,
                          size_t ws_bytes, void *stream);

/* Projected Levenberg-Marquardt polish of n_pts points in place (the local
 * refinement after annealing; the paper uses Nelder-Mead there, Sec. 3):
 *   (J^T W J + mu diag(J^T W J)) delta = -J^T W r, trial = clamp(p + delta),
 *   accept if the cost decreases (mu /= 10; stop when the relative decrease
 *   is below tol), else mu *= 10 (stop once mu > 1e16); mu starts at mu0.
 * A zero diagonal entry is replaced by 1; coordinates with lb = ub, or on a
 * bound that -J^T W r points out of, are frozen for the iteration.  lb, ub:
 * [host][n_inst][P].  cost_out [n_pts] and iters_out [n_pts] nullable.
 * GLOBAL4 and LMM12 plans (PERFWD, MM, REB: SABR_EUNSUPPORTED). */
sabr_status sabr_lm_polish(const sabr_plan *plan, int32_t n_pts, const int32_t *pt_inst,
                           double *params, const double *lb, const double *ub, int32_t max_iter,
                           double mu0, double tol, double *cost_out, int32_t *iters_out,
                           void *workspace, size_t ws_bytes, void *stream);

/* Device workspace bytes sabr_nm_polish needs (the box tables). */
size_t sabr_nm_workspace_size(const sabr_plan *plan);

/* Nelder-Mead polish of n_pts points in place: the local minimizer the paper
 * runs on the annealing's result (Sec. 3), for every model.  Standard
 * coefficients (reflection 1, expansion 2, contraction 1/2, shrink 1/2),
 * every trial point clamped into [lb, ub]; initial simplex x0 and
 * x0 + step (ub_k - lb_k) e_k (x0 - that step when it leaves the box);
 * vertices ordered by cost (best: lowest index on ties; worst: highest);
 * stop when f_worst - f_best <= tol |f_best| or after max_iter iterations.
 * One wavefront per point with the simplex in LDS ((P + 1)(P + 2) doubles
 * beside the cost's own LDS; SABR_EUNSUPPORTED if that exceeds the LDS of a
 * workgroup).  params: [n_pts][P] device, in/out (the best vertex); lb, ub:
 * [host][n_inst][P] with 0 < step <= 1; cost_out [n_pts] and iters_out
 * [n_pts] (device, nullable): the best cost (NaN for an invalid pt_inst)
 * and the iterations taken. */
sabr_status sabr_nm_polish(const sabr_plan *plan, int32_t n_pts, const int32_t *pt_inst,
                           double *params, const double *lb, const double *ub, int32_t max_iter,
                           double step, double tol, double *cost_out, int32_t *iters_out,
                           void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Monte Carlo pricer of caplets and swaptions under the Hagan SABR/LIBOR
 * dynamics (Sec. 2.1: eqs. (dinamicasHagan1), (dinamicasHagan2) under the
 * spot measure with the drifts mu^F, mu^V, the first unfixed index h(t) of
 * eq. (h_t) and the bank-account numeraire; correlations eqs. (rhoij),
 * (thetaij), (phiij)): the pricer S_MC that the paper nests in its swaption
 * cost (Sec. 3) and times in Table (haganMCpricer).
 *
 * Forward k (k = 0..n_fwd-1) fixes at T[k] and accrues tau[k]; during
 * [T[j-1], T[j]) (T[-1] = 0) the alive forwards are k >= j.  Each such
 * interval is cut into ceil(length / dt) (at least one) equal steps; a step
 * moves F_k by Euler (floored at 0) and V_k by log-Euler, driven by
 * x = sqrt(h) B xi where B is the plan's correlation factor (below) and xi
 * the step's first 2n standard normals, n = the alive forwards (the factor's
 * alive rows vanish beyond column 2n): pairs 2b and 2b + 1 of step s on
 * path p are the Box-Muller transforms of the Philox4x32-10 block at
 * counter (b, s, p mod 2^32, p / 2^32) and key (seed mod 2^32, seed / 2^32),
 * words (w0, w1) for pair 2b and (w2, w3) for pair 2b + 1, each giving
 * u1 = (w_first + 1) 2^-32 and u2 = w_second 2^-32.  The drift of V_k takes the
 * covariance of Z_k with W_i, phi_{i,k}.  At T[a] option (a, b, K) pays
 * max(1 - P(T_a, T_b) - K sum_{i=a}^{b-1} tau_i P(T_a, T_{i+1}), 0)
 * (a payer swaption on forwards a..b-1; b = a + 1 is the caplet on F_a),
 * deflated by P0 / prod_{j<a} (1 + tau_j F_j(T_j)).
 *
 * Correlation factor: the 2 n_fwd x 2 n_fwd matrix of (W_0.., Z_0..) need
 * not be positive semi-definite (the paper's calibrated Hagan parameters
 * give an indefinite one); it is repaired spectrally (Rebonato and Jaeckel
 * 1999: eigenvalues clipped at 0, unit diagonal restored) and B is the
 * Cholesky factor of the repaired matrix with the components ordered
 * W_{n_fwd-1}, Z_{n_fwd-1}, ..., W_0, Z_0 (a pivot at or below 1e-9 leaves its
 * column zero), rows returned in the order W_0.., Z_0..; computed on the
 * host when the plan is created.  B B^T is the matrix itself when it is
 * positive semi-definite.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_fwd;             /* 1..24 */
  const double *T;           /* [n_fwd] fixing times, 0 < T[0] < T[1] < ... */
  const double *tau;         /* [n_fwd] accrual fractions > 0 */
  const double *F0;          /* [n_fwd] initial forwards > 0 */
  const double *alpha;       /* [n_fwd] V_k(0) > 0 */
  const double *beta;        /* [n_fwd] in [0, 1] */
  const double *phi;         /* [n_fwd] phi_kk, |phi_kk| <= 1 */
  const double *sigma;       /* [n_fwd] vol of vol >= 0 */
  double eta1, lambda1, eta2, lambda2, lambda3;  /* eta in [0, 1], lambda >= 0 */
  double P0;                 /* P(0, T[0]) > 0 */
  int32_t n_opt;             /* >= 1 */
  const int32_t *opt_a;      /* [n_opt] expiry index a */
  const int32_t *opt_b;      /* [n_opt] end index b, a < b <= n_fwd */
  const double *opt_K;       /* [n_opt] strike */
} sabr_mc_problem;           /* every array [host] */

typedef struct sabr_mc_plan sabr_mc_plan; /* opaque; host memory only */

/* Validate the problem and build its image (host only: no GPU call). */
sabr_status sabr_mc_plan_create(const sabr_mc_problem *prob /*[host]*/, sabr_mc_plan **out);
void sabr_mc_plan_destroy(sabr_mc_plan *plan);
/* Bytes of the device image; sabr_mc_plan_upload copies it into the
 * caller's 8-byte aligned device buffer and synchronises the stream. */
size_t sabr_mc_plan_device_bytes(const sabr_mc_plan *plan);
sabr_status sabr_mc_plan_upload(sabr_mc_plan *plan, void *dev_buf, size_t bytes, void *stream);
/* The correlation factor B [2 n_fwd][2 n_fwd] (row-major, [host]). */
sabr_status sabr_mc_factor(const sabr_mc_plan *plan, double *B);
/* Workspace bytes of sabr_mc_price for n_paths paths (0 if n_paths is out
 * of range). */
size_t sabr_mc_workspace_size(const sabr_mc_plan *plan, int64_t n_paths);
/* Price every option over paths 0..n_paths-1 (1 <= n_paths <= 2^38; at
 * most 2^31 time steps): price[o] the mean discounted payoff, stderr_out[o]
 * (may be NULL) its standard error (sample standard deviation / sqrt(n)),
 * both [n_opt] device arrays in the caller's option order.  The results
 * depend only on the problem, n_paths, dt and seed. */
sabr_status sabr_mc_price(const sabr_mc_plan *plan, int64_t n_paths, double dt, uint64_t seed,
                          double *price, double *stderr_out, void *workspace, size_t ws_bytes,
                          void *stream);

/* The swaption cost f_s of Sec. 3 by this pricer: cost[0] = sum_o w_o
 * (price_o - target_o)^2 with price as sabr_mc_price computes it over the
 * same paths (target, weight [n_opt] device arrays in the caller's option
 * order; weight NULL = 1; price [n_opt] device, or NULL to keep the prices
 * in the workspace).  The sum runs in a fixed order on the device. */
sabr_status sabr_mc_cost(const sabr_mc_plan *plan, int64_t n_paths, double dt, uint64_t seed,
                         const double *target, const double *weight, double *price,
                         double *cost, void *workspace, size_t ws_bytes, void *stream);

/* Last error message of the calling thread ("" if none). */
const char *sabr_last_error(void);

/* Forget the library's process-wide state: the per-device address of the
 * no-allocation scratch array (looked up again on the next
 * sa_calibrate_noalloc), the cached LDS budget and the calling thread's last
 * error.  Nothing else is process-wide: each plan owns its device image and
 * its captured graph and releases them in sabr_plan_destroy (Monte Carlo
 * plans in sabr_mc_plan_destroy); the scratch array itself is a static
 * device variable held until the process ends.  Call it with no other call
 * of the library in flight.  Always SABR_OK. */
sabr_status sabr_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* SABR_H */
