// sabr_api.cpp -- C ABI of the SA calibrator (see include/sabr.h): host-side
// validation, packed device image, workspace layout, launch sequence and the
// hipGraph replay cache.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sabr.h"
#include "sabr_adjoint.hpp"
#include "sabr_internal.hpp"
#include "sabr_mc_internal.h"

using sabr::DevInst;
using sabr::DevMarket;

namespace {

thread_local std::string g_err;

sabr_status fail(sabr_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

sabr_status hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return SABR_EHIP;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

namespace sabr {
sabr_status mc_fail(sabr_status st, const std::string &msg) { return fail(st, msg); }
sabr_status mc_hip_fail(hipError_t e, const char *what) { return hip_fail(e, what); }
}  // namespace sabr

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bump allocator over one device buffer: every block is 256-byte aligned.
struct Layout {
  size_t off = 0;
  template <class T>
  size_t take(size_t n) {
    const size_t o = off;
    off = align256(off + n * sizeof(T));
    return o;
  }
};

// Register column length of the LMM12 swap recursion in the cost kernels:
// 16 or 24 forwards, or 0 (an LDS column) for longer swaps.
int reglen_for(int max_len) {
  return max_len <= sabr::kMapRegLen ? sabr::kMapRegLen : (max_len <= 24 ? 24 : 0);
}

}  // namespace

struct sabr_plan {
  int n_inst = 0, model = 0, formula = 0, residual = 0;
  int np = 0;  // parameters per point
  double beta = 0.5;
  int nF = 0, nU = 0, nQ = 0;
  int max_nq = 0, max_nu = 0, max_nf = 0, max_len = 0;
  // host copies of the uploaded arrays
  std::vector<DevInst> inst;
  std::vector<double> f_T, f_tauP, f_F, f_mmw;
  std::vector<int> u_first, u_len, u_order, u_ext, u_q0;
  std::vector<sabr::UndMap> u_map;
  std::vector<double> u_S0, u_A, u_invA, u_T;
  std::vector<sabr::QuoteRec> q;  // und, kind, K filled on the host
  std::vector<int> q_und_g, q_ext;
  std::vector<double> q_vol, q_wuser;
  // device image offsets
  size_t o_uq0, o_qext;
  size_t o_inst, o_fT, o_ftauP, o_fF, o_fmmw, o_ufirst, o_ulen, o_uorder, o_uS0, o_uA, o_uinvA, o_uT,
      o_q, o_qundg, o_qvol, o_qwuser;  // uploaded (contiguous prefix)
  size_t upload_bytes = 0;
  size_t o_fv, o_uS0b, o_uc0, o_ufp, o_umap;
  size_t total_bytes = 0;
  std::vector<unsigned char> staging;
  char *dev = nullptr;
  DevMarket dm{};
  // host staging of per-call tables (kept until the next call)
  std::vector<unsigned char> sa_staging, lm_staging, nm_staging;
  std::mutex mu;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uint64_t> graph_key;
  ~sabr_plan() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  }
};

extern "C" {

const char *sabr_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace sabr {
// Clears the process-wide caches (LDS budget, scratch addresses; in the
// kernels' file); the next use looks them up again.
void forget_process_caches();
}  // namespace sabr

extern "C" {

sabr_status sabr_shutdown(void) {
  sabr::forget_process_caches();
  g_err.clear();
  return SABR_OK;
}

int32_t sabr_num_params(int32_t model) { return model == 0 ? 4 : (model == 1 ? 12 : -1); }

sabr_status sabr_plan_create(const sabr_problem *pr, sabr_plan **out) {
  if (!pr || !out) return fail(SABR_EINVAL, "null argument");
  *out = nullptr;
  if (pr->n_inst < 1) return fail(SABR_EINVAL, "n_inst must be >= 1");
  if (pr->model < 0 || pr->model > 4) return fail(SABR_EINVAL, "unknown model");
  if (pr->vol_formula < 0 || pr->vol_formula > 1) return fail(SABR_EINVAL, "unknown formula");
  if (pr->residual < 0 || pr->residual > 1) return fail(SABR_EINVAL, "unknown residual mode");
  if (!(pr->beta >= 0.0 && pr->beta <= 1.0)) return fail(SABR_EINVAL, "beta outside [0, 1]");
  if (!pr->fwd_off || !pr->und_off || !pr->q_off || !pr->fwd_T || !pr->fwd_tau || !pr->fwd_F ||
      !pr->fwd_P || !pr->und_first || !pr->und_len || !pr->q_und || !pr->q_kind || !pr->q_K ||
      !pr->q_vol || !pr->q_w)
    return fail(SABR_EINVAL, "null market array");
  const int n = pr->n_inst;
  for (const int32_t *off : {pr->fwd_off, pr->und_off, pr->q_off}) {
    if (off[0] != 0) return fail(SABR_EINVAL, "CSR offsets must start at 0");
    for (int i = 0; i < n; ++i)
      if (off[i + 1] < off[i]) return fail(SABR_EINVAL, "CSR offsets not monotone");
  }
  sabr_plan *P = new (std::nothrow) sabr_plan;
  if (!P) return fail(SABR_ENOMEM, "out of host memory");
  P->n_inst = n;
  P->model = pr->model;
  P->formula = pr->vol_formula;
  P->residual = pr->residual;
  P->beta = pr->beta;
  P->np = sabr_num_params(pr->model);
  if (pr->model >= 2) {
    // PERFWD: one (alpha, rho, nu) per forward; MM: one (alpha, phi) per
    // forward and sigma; REB: one (kappa, phi) per forward and the eight
    // parameters of g and h.  Lanes k < P of a wave hold the point next to
    // the Metropolis uniform, so every instance has the same nf with P <= 63.
    const char *name = pr->model == 2 ? "PERFWD" : (pr->model == 3 ? "MM" : "REB");
    const int nf = pr->fwd_off[1] - pr->fwd_off[0];
    for (int i = 1; i < n; ++i)
      if (pr->fwd_off[i + 1] - pr->fwd_off[i] != nf) {
        delete P;
        return fail(SABR_EINVAL, std::string(name) + " instances must hold equally many forwards");
      }
    const int np = pr->model == 2 ? 3 * nf : (pr->model == 3 ? 2 * nf + 1 : 2 * nf + 8);
    if (nf < 1 || np > sabr::kWave - 1) {
      delete P;
      const int most = pr->model == 2 ? 21 : (pr->model == 3 ? 31 : 27);
      return fail(SABR_EINVAL, std::string(name) + " needs 1.." + std::to_string(most) +
                                   " forwards per instance");
    }
    P->np = np;
  }
  P->nF = pr->fwd_off[n];
  P->nU = pr->und_off[n];
  P->nQ = pr->q_off[n];
  auto bad = [&](const std::string &m) {
    delete P;
    return fail(SABR_EINVAL, m);
  };
  for (int k = 0; k < P->nF; ++k) {
    const double T = pr->fwd_T[k], tau = pr->fwd_tau[k], F = pr->fwd_F[k], Pk = pr->fwd_P[k];
    if (!(std::isfinite(T) && T >= 0.0) || !finite_pos(tau) || !finite_pos(F) || !finite_pos(Pk))
      return bad("forward " + std::to_string(k) + ": bad T, tau, F or P");
    P->f_T.push_back(T);
    P->f_tauP.push_back(tau * Pk);
    P->f_F.push_back(F);
  }
  // MM drift weights T_{k-1} tau_k F_k^beta / (1 + tau_k F_k), T_{-1} = 0 per instance
  P->f_mmw.assign(P->nF, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = pr->fwd_off[i] + 1; k < pr->fwd_off[i + 1]; ++k) {
      const double tau = pr->fwd_tau[k], F = pr->fwd_F[k];
      P->f_mmw[k] = pr->fwd_T[k - 1] * tau * std::pow(F, pr->beta) / (1.0 + tau * F);
    }
  for (int i = 0; i < n; ++i) {
    DevInst d{};
    d.f0 = pr->fwd_off[i];
    d.nf = pr->fwd_off[i + 1] - d.f0;
    d.u0 = pr->und_off[i];
    d.nu = pr->und_off[i + 1] - d.u0;
    d.q0 = pr->q_off[i];
    d.nq = pr->q_off[i + 1] - d.q0;
    if (d.nq < 1) return bad("instance " + std::to_string(i) + " has no quotes");
    d.maxlen = 1;
    // underlyings in the caller's order: validation and market values
    std::vector<int> ufirst(d.nu), ulen(d.nu);
    std::vector<double> uS0(d.nu), uA(d.nu), uT(d.nu);
    for (int j = 0; j < d.nu; ++j) {
      const int u = d.u0 + j;
      const int first = pr->und_first[u], len = pr->und_len[u];
      if (len < 1 || first < 0 || first + len > d.nf)
        return bad("underlying " + std::to_string(u) + ": forward range out of bounds");
      if (pr->model != 1 && len != 1) return bad("only LMM12 markets hold swaptions");
      if (len > d.maxlen) d.maxlen = len;
      // annuity, weights and swap rate, summed in forward order
      double A = 0.0;
      for (int k = first; k < first + len; ++k)
        A += pr->fwd_tau[d.f0 + k] * pr->fwd_P[d.f0 + k];
      double S0 = 0.0;
      for (int k = first; k < first + len; ++k) {
        const double wk = pr->fwd_tau[d.f0 + k] * pr->fwd_P[d.f0 + k] / A;
        S0 += wk * pr->fwd_F[d.f0 + k];
      }
      const double Te = pr->fwd_T[d.f0 + first];
      if (!(Te > 0.0)) return bad("underlying " + std::to_string(u) + ": expiry must be > 0");
      ufirst[j] = first;
      ulen[j] = len;
      uS0[j] = S0;
      uA[j] = A;
      uT[j] = Te;
    }
    int prev = 0;
    for (int q = d.q0; q < d.q0 + d.nq; ++q) {
      const int u = pr->q_und[q], kind = pr->q_kind[q];
      const double K = pr->q_K[q], vol = pr->q_vol[q], w = pr->q_w[q];
      if (u < 0 || u >= d.nu) return bad("quote " + std::to_string(q) + ": underlying out of range");
      if (u < prev) return bad("quotes of instance " + std::to_string(i) + " not sorted by underlying");
      prev = u;
      if (kind != 0 && kind != 1) return bad("quote " + std::to_string(q) + ": bad kind");
      if (!finite_pos(K) || !finite_pos(vol) || !(std::isfinite(w) && w >= 0.0))
        return bad("quote " + std::to_string(q) + ": bad strike, vol or weight");
    }
    // Internal order: underlyings by decreasing length (stable), so a pass of
    // the swap map over consecutive underlyings runs swaps of similar length,
    // and the quotes grouped by that order, so the underlyings of a chunk own
    // a contiguous range of quotes.  Per-quote outputs and the underlyings
    // query go back to the caller's order.
    std::vector<int> ord(d.nu), pos(d.nu);
    for (int j = 0; j < d.nu; ++j) ord[j] = j;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return ulen[x] > ulen[y]; });
    for (int p = 0; p < d.nu; ++p) pos[ord[p]] = p;
    for (int p = 0; p < d.nu; ++p) {
      const int j = ord[p];
      P->u_first.push_back(ufirst[j]);
      P->u_len.push_back(ulen[j]);
      P->u_S0.push_back(uS0[j]);
      P->u_A.push_back(uA[j]);
      P->u_invA.push_back(1.0 / uA[j]);
      P->u_T.push_back(uT[j]);
      P->u_ext.push_back(d.u0 + j);
      P->u_order.push_back(p);
      P->u_map.push_back(sabr::UndMap{p, ufirst[j], ulen[j], 0});
    }
    std::vector<int> qord(d.nq);
    for (int j = 0; j < d.nq; ++j) qord[j] = j;
    std::stable_sort(qord.begin(), qord.end(), [&](int x, int y) {
      return pos[pr->q_und[d.q0 + x]] < pos[pr->q_und[d.q0 + y]];
    });
    std::vector<int> uq0(d.nu + 1, d.nq);
    for (int j = d.nq - 1; j >= 0; --j) uq0[pos[pr->q_und[d.q0 + qord[j]]]] = j;
    for (int p = d.nu - 1; p >= 0; --p) uq0[p] = std::min(uq0[p], uq0[p + 1]);
    for (int p = 0; p < d.nu; ++p) P->u_q0.push_back(uq0[p]);
    for (int j = 0; j < d.nq; ++j) {
      const int q = d.q0 + qord[j];
      sabr::QuoteRec R{};
      R.und = pos[pr->q_und[q]];
      R.kind = pr->q_kind[q];
      R.K = pr->q_K[q];
      P->q.push_back(R);
      P->q_und_g.push_back(d.u0 + R.und);
      P->q_vol.push_back(pr->q_vol[q]);
      P->q_wuser.push_back(pr->q_w[q]);
      P->q_ext.push_back(qord[j]);
    }
    if (d.nq > P->max_nq) P->max_nq = d.nq;
    if (d.nu > P->max_nu) P->max_nu = d.nu;
    if (d.nf > P->max_nf) P->max_nf = d.nf;
    if (d.maxlen > P->max_len) P->max_len = d.maxlen;
    P->inst.push_back(d);
  }
  // device image: uploaded prefix, then the precomputed arrays
  Layout L;
  P->o_inst = L.take<DevInst>(n);
  P->o_fT = L.take<double>(P->nF);
  P->o_ftauP = L.take<double>(P->nF);
  P->o_fF = L.take<double>(P->nF);
  P->o_fmmw = L.take<double>(P->nF);
  P->o_ufirst = L.take<int>(P->nU);
  P->o_ulen = L.take<int>(P->nU);
  P->o_uorder = L.take<int>(P->nU);
  P->o_uq0 = L.take<int>(P->nU);
  P->o_uS0 = L.take<double>(P->nU);
  P->o_uA = L.take<double>(P->nU);
  P->o_uinvA = L.take<double>(P->nU);
  P->o_uT = L.take<double>(P->nU);
  P->o_umap = L.take<sabr::UndMap>(P->nU);
  P->o_q = L.take<sabr::QuoteRec>(P->nQ);
  P->o_qundg = L.take<int>(P->nQ);
  P->o_qext = L.take<int>(P->nQ);
  P->o_qvol = L.take<double>(P->nQ);
  P->o_qwuser = L.take<double>(P->nQ);
  P->upload_bytes = L.off;
  P->o_fv = L.take<double>(P->nF);
  P->o_uS0b = L.take<double>(P->nU);
  P->o_ufp = L.take<double>(P->nU);
  P->o_uc0 = L.take<double>(P->nU);
  P->total_bytes = L.off;
  P->staging.assign(P->upload_bytes, 0);
  auto put = [&](size_t off, const void *src, size_t bytes) {
    if (bytes) std::memcpy(P->staging.data() + off, src, bytes);
  };
  put(P->o_inst, P->inst.data(), n * sizeof(DevInst));
  put(P->o_fT, P->f_T.data(), P->nF * 8);
  put(P->o_ftauP, P->f_tauP.data(), P->nF * 8);
  put(P->o_fF, P->f_F.data(), P->nF * 8);
  put(P->o_fmmw, P->f_mmw.data(), P->nF * 8);
  put(P->o_ufirst, P->u_first.data(), P->nU * 4);
  put(P->o_ulen, P->u_len.data(), P->nU * 4);
  put(P->o_uq0, P->u_q0.data(), P->nU * 4);
  put(P->o_uorder, P->u_order.data(), P->nU * 4);
  put(P->o_uS0, P->u_S0.data(), P->nU * 8);
  put(P->o_uA, P->u_A.data(), P->nU * 8);
  put(P->o_uinvA, P->u_invA.data(), P->nU * 8);
  put(P->o_uT, P->u_T.data(), P->nU * 8);
  put(P->o_umap, P->u_map.data(), P->nU * sizeof(sabr::UndMap));
  put(P->o_q, P->q.data(), P->nQ * sizeof(sabr::QuoteRec));
  put(P->o_qundg, P->q_und_g.data(), P->nQ * 4);
  put(P->o_qext, P->q_ext.data(), P->nQ * 4);
  put(P->o_qvol, P->q_vol.data(), P->nQ * 8);
  put(P->o_qwuser, P->q_wuser.data(), P->nQ * 8);
  *out = P;
  return SABR_OK;
}

void sabr_plan_destroy(sabr_plan *plan) { delete plan; }

size_t sabr_plan_device_bytes(const sabr_plan *plan) { return plan ? plan->total_bytes : 0; }
int32_t sabr_plan_num_params(const sabr_plan *plan) { return plan ? plan->np : -1; }
int32_t sabr_plan_num_inst(const sabr_plan *plan) { return plan ? plan->n_inst : -1; }
int32_t sabr_plan_max_quotes(const sabr_plan *plan) { return plan ? plan->max_nq : -1; }

sabr_status sabr_plan_underlyings(const sabr_plan *plan, double *S0, double *A, double *T) {
  if (!plan) return fail(SABR_EINVAL, "null plan");
  for (int g = 0; g < plan->nU; ++g) {   // internal order -> the caller's
    const int u = plan->u_ext[g];
    if (S0) S0[u] = plan->u_S0[g];
    if (A) A[u] = plan->u_A[g];
    if (T) T[u] = plan->u_T[g];
  }
  return SABR_OK;
}

sabr_status sabr_plan_upload(sabr_plan *P, void *dev_buf, size_t bytes, void *stream) {
  if (!P || !dev_buf) return fail(SABR_EINVAL, "null argument");
  if (bytes < P->total_bytes) return fail(SABR_EWORKSPACE, "device buffer smaller than the image");
  if (reinterpret_cast<uintptr_t>(dev_buf) % 256) return fail(SABR_EINVAL, "device buffer not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *d = static_cast<char *>(dev_buf);
  hipError_t e = hipMemcpyAsync(d, P->staging.data(), P->upload_bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "upload");
  DevMarket m{};
  m.n_inst = P->n_inst;
  m.model = P->model;
  m.np = P->np;
  m.formula = P->formula;
  m.residual = P->residual;
  m.beta = P->beta;
  m.max_nq = P->max_nq;
  m.max_nu = P->max_nu;
  m.max_nf = P->max_nf;
  m.max_len = P->max_len;
  m.reglen = reglen_for(P->max_len);
  m.thchunk = sabr::th_chunk_for(P->max_nu);
  m.inst = reinterpret_cast<const DevInst *>(d + P->o_inst);
  auto D = [&](size_t o) { return reinterpret_cast<double *>(d + o); };
  auto I = [&](size_t o) { return reinterpret_cast<int *>(d + o); };
  m.f_T = D(P->o_fT);
  m.f_v = D(P->o_fv);
  m.f_mmw = D(P->o_fmmw);
  m.u_first = I(P->o_ufirst);
  m.u_len = I(P->o_ulen);
  m.u_order = I(P->o_uorder);
  m.u_q0 = I(P->o_uq0);
  m.q_ext = I(P->o_qext);
  m.u_S0 = D(P->o_uS0);
  m.u_A = D(P->o_uA);
  m.u_invA = D(P->o_uinvA);
  m.u_S0b = D(P->o_uS0b);
  m.u_fp = D(P->o_ufp);
  m.u_T = D(P->o_uT);
  m.u_map = reinterpret_cast<const sabr::UndMap *>(d + P->o_umap);
  m.u_c0 = D(P->o_uc0);
  m.q = reinterpret_cast<const sabr::QuoteRec *>(d + P->o_q);
  e = sabr::launch_prep(m, reinterpret_cast<sabr::QuoteRec *>(d + P->o_q), D(P->o_fv),
                        D(P->o_uS0b), D(P->o_uc0), D(P->o_ufp), D(P->o_qvol), D(P->o_qwuser),
                        I(P->o_qundg),
                        D(P->o_ftauP), D(P->o_fF), P->nQ, P->nF, P->nU, s);
  if (e != hipSuccess) return hip_fail(e, "market precompute launch");
  P->dev = d;
  P->dm = m;
  std::lock_guard<std::mutex> g(P->mu);
  if (P->graph_exec) {
    (void)hipGraphExecDestroy(P->graph_exec);
    P->graph_exec = nullptr;
    P->graph_key.clear();
  }
  return SABR_OK;
}

sabr_status sabr_cost_batch(const sabr_plan *P, int32_t n_pts, const int32_t *pt_inst,
                            const double *params, double *cost, double *resid, double *model,
                            int32_t stride, void *stream) {
  if (!P) return fail(SABR_EINVAL, "null plan");
  if (!P->dev) return fail(SABR_EINVAL, "plan not uploaded");
  if (n_pts < 0) return fail(SABR_EINVAL, "n_pts < 0");
  if (n_pts == 0) return SABR_OK;
  if (!pt_inst || !params || !cost) return fail(SABR_EINVAL, "null pt_inst, params or cost");
  if ((resid || model) && stride < P->max_nq) return fail(SABR_EINVAL, "stride < max quotes");
  hipError_t e = sabr::launch_cost(P->dm, n_pts, pt_inst, params, cost, resid, model, stride,
                                   static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "cost launch");
  return SABR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Simulated annealing
// ---------------------------------------------------------------------------
namespace {

struct SALayout {
  size_t o_chains, o_cbase, o_abase, o_tinst, o_tchain, o_toff, o_lb, o_ub, o_x0, o_T0;
  size_t upload_bytes;
  size_t o_X, o_BX, o_BF, o_RX, o_RF, o_Tcur, o_tstart;
  size_t o_TF, o_TB, o_TI, o_TJ, o_TN;
  size_t total;
  int n_tiles, waves, wpc, cpw, max_tiles;
  int64_t tot_chains;
};

SALayout sa_layout(const sabr_plan *P, const sa_config *cfg, const int32_t *chains) {
  SALayout S{};
  const int n = P->n_inst;
  const int Pn = P->np;
  int want = cfg && cfg->waves_per_group > 0 ? cfg->waves_per_group : 4;
  if (want > sabr::kMaxWavesPerGroup) want = sabr::kMaxWavesPerGroup;
  DevMarket shape{};  // LDS budget depends on the market's shape only
  shape.model = P->model;
  shape.np = P->np;
  shape.max_nf = P->max_nf;
  shape.max_nu = P->max_nu;
  shape.max_len = P->max_len;
  shape.reglen = reglen_for(P->max_len);
  shape.thchunk = sabr::th_chunk_for(P->max_nu);
  // waves_per_chain > 1: one chain per workgroup, its waves split the quotes;
  // chains_per_wave = 2: two chains per wave, one per half
  S.wpc = cfg && cfg->waves_per_chain > 1 ? cfg->waves_per_chain : 1;
  S.cpw = cfg && cfg->chains_per_wave == 2 ? 2 : 1;
  S.waves = S.wpc > 1 ? S.wpc : sabr::sa_waves_per_group(shape, want, S.cpw == 2);
  const int cpt = S.waves / S.wpc * S.cpw;   // chains per tile
  S.n_tiles = 0;
  S.max_tiles = 0;
  S.tot_chains = 0;
  for (int i = 0; i < n; ++i) {
    const int ti = (chains[i] + cpt - 1) / cpt;
    S.n_tiles += ti;
    if (ti > S.max_tiles) S.max_tiles = ti;
    S.tot_chains += chains[i];
  }
  Layout L;
  S.o_chains = L.take<int>(n);
  S.o_cbase = L.take<int64_t>(n);
  S.o_abase = L.take<int64_t>(n);
  S.o_tinst = L.take<int>(S.n_tiles);
  S.o_tchain = L.take<int>(S.n_tiles);
  S.o_toff = L.take<int>(n + 1);
  S.o_lb = L.take<double>((size_t)n * Pn);
  S.o_ub = L.take<double>((size_t)n * Pn);
  S.o_x0 = L.take<double>((size_t)n * Pn);
  S.o_T0 = L.take<double>(n);
  S.upload_bytes = L.off;
  S.o_X = L.take<double>(S.tot_chains * Pn);
  S.o_BX = L.take<double>(S.tot_chains * Pn);
  S.o_BF = L.take<double>(S.tot_chains);
  S.o_RX = L.take<double>((size_t)n * Pn);
  S.o_RF = L.take<double>(n);
  S.o_Tcur = L.take<double>(n);
  S.o_tstart = L.take<uint64_t>(1);
  S.o_TF = L.take<double>(S.n_tiles);
  S.o_TB = L.take<double>(S.n_tiles);
  S.o_TI = L.take<int>(S.n_tiles);
  S.o_TJ = L.take<int>(S.n_tiles);
  S.o_TN = L.take<int>(S.n_tiles);
  S.total = L.off;
  return S;
}

sabr_status check_sa_args(const sabr_plan *P, const sa_config *cfg, const int32_t *chains) {
  if (!P) return fail(SABR_EINVAL, "null plan");
  if (!cfg || !chains) return fail(SABR_EINVAL, "null config or chains");
  if (!(cfg->T0 > 0.0) || !std::isfinite(cfg->T0)) return fail(SABR_EINVAL, "T0 must be > 0");
  if (!(cfg->cool > 0.0 && cfg->cool <= 1.0)) return fail(SABR_EINVAL, "cool outside (0, 1]");
  if (!(cfg->step_frac > 0.0 && cfg->step_frac <= 1.0))
    return fail(SABR_EINVAL, "step_frac outside (0, 1]");
  if (cfg->n_levels < 0 || cfg->n_steps < 0) return fail(SABR_EINVAL, "negative L or N");
  if (cfg->waves_per_chain < 0 || cfg->waves_per_chain > sabr::kMaxWavesPerGroup)
    return fail(SABR_EINVAL, "waves_per_chain outside [0, 8]");
  if (cfg->waves_per_chain > 1) {
    DevMarket shape{};
    shape.model = P->model;
    shape.np = P->np;
    shape.max_nf = P->max_nf;
    shape.max_nu = P->max_nu;
    shape.max_len = P->max_len;
    shape.reglen = reglen_for(P->max_len);
    shape.thchunk = sabr::th_chunk_for(P->max_nu);
    if (sabr::sa_waves_per_group(shape, cfg->waves_per_chain) != cfg->waves_per_chain)
      return fail(SABR_EINVAL, "waves_per_chain: the waves' LDS exceeds one workgroup's");
  }
  if (cfg->level0 < 0) return fail(SABR_EINVAL, "level0 must be >= 0");
  if (cfg->chains_per_wave < 0 || cfg->chains_per_wave > 2)
    return fail(SABR_EINVAL, "chains_per_wave outside [0, 2]");
  if (cfg->chains_per_wave == 2) {
    if (P->model != 0) return fail(SABR_EINVAL, "chains_per_wave = 2 needs a GLOBAL4 plan");
    if (cfg->waves_per_chain > 1)
      return fail(SABR_EINVAL, "chains_per_wave = 2 with waves_per_chain > 1");
  }
  for (int i = 0; i < P->n_inst; ++i) {
    if (chains[i] < 1) return fail(SABR_EINVAL, "every instance needs >= 1 chain");
    if (cfg->T0_per_inst && !(cfg->T0_per_inst[i] > 0.0 && std::isfinite(cfg->T0_per_inst[i])))
      return fail(SABR_EINVAL, "T0_per_inst must be > 0");
  }
  return SABR_OK;
}

}  // namespace

extern "C" {

size_t sa_workspace_size(const sabr_plan *P, const sa_config *cfg, const int32_t *chains) {
  if (check_sa_args(P, cfg, chains) != SABR_OK) return 0;
  return sa_layout(P, cfg, chains).total;
}

}  // extern "C"

namespace {

// Validation of the arguments sa_calibrate and sa_calibrate_noalloc share
// (everything but the workspace).
sabr_status check_sa_call(const sabr_plan *Pc, const sa_config *cfg, const int32_t *chains,
                          const double *lb, const double *ub, const double *x0,
                          const double *best_x, const double *best_f) {
  sabr_status st = check_sa_args(Pc, cfg, chains);
  if (st != SABR_OK) return st;
  if (!Pc->dev) return fail(SABR_EINVAL, "plan not uploaded");
  if (!lb || !ub) return fail(SABR_EINVAL, "null box");
  if (!best_x || !best_f) return fail(SABR_EINVAL, "null best_x or best_f");
  const int n = Pc->n_inst;
  const int Pn = Pc->np;
  for (int i = 0; i < n * Pn; ++i) {
    if (!std::isfinite(lb[i]) || !std::isfinite(ub[i]) || !(lb[i] <= ub[i]))
      return fail(SABR_EINVAL, "box bound " + std::to_string(i) + ": need finite lb <= ub");
    if (x0 && !(x0[i] >= lb[i] && x0[i] <= ub[i]))
      return fail(SABR_EINVAL, "x0 outside the box");
  }
  return SABR_OK;
}

// The annealing run of sa_calibrate on a validated call with a workspace of
// at least sa_layout(...).total bytes.
sabr_status sa_run(sabr_plan *P, const sa_config *cfg, const int32_t *chains, const double *lb,
                   const double *ub, const double *x0, double *best_x, double *best_f,
                   double *chain_best_x, double *chain_best_f, uint8_t *accept,
                   double *level_trace, int32_t *level_best, const SALayout &S, void *workspace,
                   void *stream) {
  const int n = P->n_inst;
  const int Pn = P->np;
  const int L = cfg->n_levels, N = cfg->n_steps;
  // host-side tables
  std::lock_guard<std::mutex> guard(P->mu);
  std::vector<unsigned char> &stg = P->sa_staging;
  stg.assign(S.upload_bytes, 0);
  int *h_chains = reinterpret_cast<int *>(stg.data() + S.o_chains);
  int64_t *h_cbase = reinterpret_cast<int64_t *>(stg.data() + S.o_cbase);
  int64_t *h_abase = reinterpret_cast<int64_t *>(stg.data() + S.o_abase);
  int *h_tinst = reinterpret_cast<int *>(stg.data() + S.o_tinst);
  int *h_tchain = reinterpret_cast<int *>(stg.data() + S.o_tchain);
  int *h_toff = reinterpret_cast<int *>(stg.data() + S.o_toff);
  double *h_lb = reinterpret_cast<double *>(stg.data() + S.o_lb);
  double *h_ub = reinterpret_cast<double *>(stg.data() + S.o_ub);
  double *h_x0 = reinterpret_cast<double *>(stg.data() + S.o_x0);
  double *h_T0 = reinterpret_cast<double *>(stg.data() + S.o_T0);
  int64_t cb = 0, ab = 0;
  int t = 0;
  for (int i = 0; i < n; ++i) {
    h_chains[i] = chains[i];
    h_cbase[i] = cb;
    h_abase[i] = ab;
    h_toff[i] = t;
    cb += chains[i];
    ab += (int64_t)L * N * chains[i];
    for (int c = 0; c < chains[i]; c += S.waves / S.wpc * S.cpw) {
      h_tinst[t] = i;
      h_tchain[t] = c;
      ++t;
    }
    h_T0[i] = cfg->T0_per_inst ? cfg->T0_per_inst[i] : cfg->T0;
    for (int k = 0; k < Pn; ++k) {
      const size_t j = (size_t)i * Pn + k;
      h_lb[j] = lb[j];
      h_ub[j] = ub[j];
      h_x0[j] = x0 ? x0[j] : 0.5 * (lb[j] + ub[j]);
    }
  }
  h_toff[n] = t;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *w = static_cast<char *>(workspace);
  hipError_t e = hipMemcpyAsync(w, stg.data(), S.upload_bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "SA table upload");
  int rate_khz = 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      rate_khz <= 0)
    rate_khz = 100000;
  sabr::SAArgs a{};
  a.n_inst = n;
  a.wpc = S.wpc;
  a.cpw = S.cpw;
  a.level0 = cfg->level0;
  a.state_in = cfg->state_in;
  a.state_out = cfg->state_out;
  a.P = Pn;
  a.N = N;
  a.L = L;
  a.seed = cfg->seed;
  a.step_frac = cfg->step_frac;
  a.cool = cfg->cool;
  a.ns_per_tick = 1.0e6 / (double)rate_khz;
  a.chains = reinterpret_cast<const int *>(w + S.o_chains);
  a.chain_base = reinterpret_cast<const int64_t *>(w + S.o_cbase);
  a.acc_base = reinterpret_cast<const int64_t *>(w + S.o_abase);
  a.tile_inst = reinterpret_cast<const int *>(w + S.o_tinst);
  a.tile_chain = reinterpret_cast<const int *>(w + S.o_tchain);
  a.tile_off = reinterpret_cast<const int *>(w + S.o_toff);
  a.TF = reinterpret_cast<double *>(w + S.o_TF);
  a.TB = reinterpret_cast<double *>(w + S.o_TB);
  a.TI = reinterpret_cast<int *>(w + S.o_TI);
  a.TJ = reinterpret_cast<int *>(w + S.o_TJ);
  a.TN = reinterpret_cast<int *>(w + S.o_TN);
  a.lb = reinterpret_cast<const double *>(w + S.o_lb);
  a.ub = reinterpret_cast<const double *>(w + S.o_ub);
  a.x0 = reinterpret_cast<const double *>(w + S.o_x0);
  a.T0 = reinterpret_cast<const double *>(w + S.o_T0);
  a.X = reinterpret_cast<double *>(w + S.o_X);
  a.BX = reinterpret_cast<double *>(w + S.o_BX);
  a.BF = reinterpret_cast<double *>(w + S.o_BF);
  a.RX = reinterpret_cast<double *>(w + S.o_RX);
  a.RF = reinterpret_cast<double *>(w + S.o_RF);
  a.Tcur = reinterpret_cast<double *>(w + S.o_Tcur);
  a.t_start = reinterpret_cast<uint64_t *>(w + S.o_tstart);
  a.accept = accept;
  a.trace = level_trace;
  a.level_best = level_best;
  a.best_x = best_x;
  a.best_f = best_f;
  a.chain_best_x = chain_best_x;
  a.chain_best_f = chain_best_f;

  void *const *events = cfg->level_events;
  auto enqueue = [&](hipStream_t q) -> hipError_t {
    hipError_t r = sabr::launch_sa_init(P->dm, a, S.n_tiles, S.waves, q);
    if (r != hipSuccess) return r;
    const bool ev = events && !cfg->use_graph;
    for (int l = 0; l < L; ++l) {
      if (N > 0) {
        const bool evl = ev && events[2 * l] && events[2 * l + 1];
        if (evl && (r = hipEventRecord(static_cast<hipEvent_t>(events[2 * l]), q)) != hipSuccess)
          return r;
        r = sabr::launch_sa_level(P->dm, a, l, S.n_tiles, S.waves, cfg->occupancy, q);
        if (r != hipSuccess) return r;
        if (evl && (r = hipEventRecord(static_cast<hipEvent_t>(events[2 * l + 1]), q)) !=
                       hipSuccess)
          return r;
      }
      r = sabr::launch_sa_level_end(a, l, S.max_tiles, q);
      if (r != hipSuccess) return r;
    }
    r = sabr::launch_sa_final(a, q);
    if (r != hipSuccess || !cfg->state_out) return r;
    return sabr::launch_sa_state_out(a, q);
  };

  if (!cfg->use_graph) {
    e = enqueue(s);
    if (e != hipSuccess) return hip_fail(e, "SA launch");
    return SABR_OK;
  }
  if (s == nullptr) return fail(SABR_EINVAL, "graph replay needs a non-default stream");
  // replay key: every pointer and scalar baked into the captured kernels
  std::vector<uint64_t> key = {(uint64_t)(uintptr_t)P->dev, (uint64_t)(uintptr_t)w,
                               (uint64_t)(uintptr_t)best_x, (uint64_t)(uintptr_t)best_f,
                               (uint64_t)(uintptr_t)chain_best_x,
                               (uint64_t)(uintptr_t)chain_best_f, (uint64_t)(uintptr_t)accept,
                               (uint64_t)(uintptr_t)level_trace, (uint64_t)(uintptr_t)level_best,
                               (uint64_t)L, (uint64_t)N, cfg->seed, (uint64_t)S.waves,
                               (uint64_t)S.n_tiles, (uint64_t)cfg->occupancy,
                               (uint64_t)S.wpc, (uint64_t)S.cpw, (uint64_t)cfg->level0,
                               (uint64_t)(uintptr_t)cfg->state_in,
                               (uint64_t)(uintptr_t)cfg->state_out};
  uint64_t bits;
  std::memcpy(&bits, &cfg->step_frac, 8);
  key.push_back(bits);
  std::memcpy(&bits, &cfg->cool, 8);
  key.push_back(bits);
  for (int i = 0; i < n; ++i) key.push_back((uint64_t)chains[i]);
  if (!P->graph_exec || key != P->graph_key) {
    if (P->graph_exec) {
      (void)hipGraphExecDestroy(P->graph_exec);
      P->graph_exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    hipError_t er = enqueue(s);
    e = hipStreamEndCapture(s, &graph);
    if (er != hipSuccess) return hip_fail(er, "SA capture");
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&P->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      P->graph_exec = nullptr;
      return hip_fail(e, "graph instantiate");
    }
    P->graph_key = key;
  }
  e = hipGraphLaunch(P->graph_exec, s);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return SABR_OK;
}

}  // namespace

extern "C" {

sabr_status sa_calibrate(const sabr_plan *Pc, const sa_config *cfg, const int32_t *chains,
                         const double *lb, const double *ub, const double *x0, double *best_x,
                         double *best_f, double *chain_best_x, double *chain_best_f,
                         uint8_t *accept, double *level_trace, int32_t *level_best,
                         void *workspace, size_t ws_bytes, void *stream) {
  sabr_status st = check_sa_call(Pc, cfg, chains, lb, ub, x0, best_x, best_f);
  if (st != SABR_OK) return st;
  if (!workspace) return fail(SABR_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(SABR_EINVAL, "workspace not 256-byte aligned");
  sabr_plan *P = const_cast<sabr_plan *>(Pc);
  const SALayout S = sa_layout(P, cfg, chains);
  if (ws_bytes < S.total) return fail(SABR_EWORKSPACE, "workspace too small");
  return sa_run(P, cfg, chains, lb, ub, x0, best_x, best_f, chain_best_x, chain_best_f, accept,
                level_trace, level_best, S, workspace, stream);
}

sabr_status sa_calibrate_noalloc(const sabr_plan *Pc, const sa_config *cfg,
                                 const int32_t *chains, const double *lb, const double *ub,
                                 const double *x0, double *best_x, double *best_f,
                                 double *chain_best_x, double *chain_best_f, uint8_t *accept,
                                 double *level_trace, int32_t *level_best, void *stream) {
  sabr_status st = check_sa_call(Pc, cfg, chains, lb, ub, x0, best_x, best_f);
  if (st != SABR_OK) return st;
  if (cfg->use_graph)
    return fail(SABR_EINVAL, "sa_calibrate_noalloc: use_graph must be 0 (instantiating a graph "
                             "allocates; capture the eager launches instead)");
  sabr_plan *P = const_cast<sabr_plan *>(Pc);
  const SALayout S = sa_layout(P, cfg, chains);
  if (S.total > SA_NOALLOC_MAX_BYTES)
    return fail(SABR_EWORKSPACE, "sa_calibrate_noalloc: this call needs " +
                                     std::to_string(S.total) + " bytes of scratch, more than "
                                     "the fixed " + std::to_string(SA_NOALLOC_MAX_BYTES) +
                                     " (use sa_calibrate with a workspace)");
  void *scratch_ptr = nullptr;
  hipError_t e = sabr::sa_noalloc_scratch(&scratch_ptr);
  if (e != hipSuccess) return hip_fail(e, "sa_calibrate_noalloc: scratch lookup");
  return sa_run(P, cfg, chains, lb, ub, x0, best_x, best_f, chain_best_x, chain_best_f, accept,
                level_trace, level_best, S, scratch_ptr, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adjoint and Levenberg-Marquardt
// ---------------------------------------------------------------------------
namespace {

// Device workspace of the LM polish: the box tables (the adjoint needs none).
struct AdjLayout {
  size_t o_lb, o_ub, total;
};

AdjLayout adj_layout(const sabr_plan *P) {
  AdjLayout A{};
  Layout L;
  const int Pn = P->np;
  A.o_lb = L.take<double>((size_t)P->n_inst * Pn);
  A.o_ub = L.take<double>((size_t)P->n_inst * Pn);
  A.total = L.off;
  return A;
}

sabr_status check_points(const sabr_plan *P, int32_t n_pts) {
  if (!P) return fail(SABR_EINVAL, "null plan");
  if (!P->dev) return fail(SABR_EINVAL, "plan not uploaded");
  if (n_pts < 0) return fail(SABR_EINVAL, "n_pts < 0");
  return SABR_OK;
}

}  // namespace

extern "C" {

size_t sabr_adjoint_workspace_size(const sabr_plan *P, int32_t n_pts) {
  if (!P || n_pts < 0) return 0;
  return adj_layout(P).total;
}

sabr_status sabr_cost_vjp(const sabr_plan *P, int32_t n_pts, const int32_t *pt_inst,
                          const double *params, const double *g_cost, double *cost,
                          double *g_params, double *jtwj, double *jtwr, void *workspace,
                          size_t ws_bytes, void *stream) {
  sabr_status st = check_points(P, n_pts);
  if (st != SABR_OK) return st;
  if (n_pts == 0) return SABR_OK;
  if (!pt_inst || !params || !g_params) return fail(SABR_EINVAL, "null pt_inst, params or g_params");
  if (P->model >= 2) return fail(SABR_EUNSUPPORTED, "the adjoint takes GLOBAL4 and LMM12 plans");
  (void)workspace;   // no device scratch: the kernels keep everything in LDS
  (void)ws_bytes;
  hipError_t e = sabr::launch_vjp(P->dm, n_pts, pt_inst, params, g_cost, cost, g_params, jtwj,
                                  jtwr, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  return SABR_OK;
}

sabr_status sabr_lm_polish(const sabr_plan *Pc, int32_t n_pts, const int32_t *pt_inst,
                           double *params, const double *lb, const double *ub, int32_t max_iter,
                           double mu0, double tol, double *cost_out, int32_t *iters_out,
                           void *workspace, size_t ws_bytes, void *stream) {
  sabr_status st = check_points(Pc, n_pts);
  if (st != SABR_OK) return st;
  if (n_pts == 0) return SABR_OK;
  if (!pt_inst || !params || !lb || !ub) return fail(SABR_EINVAL, "null argument");
  if (max_iter < 0 || !(mu0 > 0.0) || !(tol >= 0.0)) return fail(SABR_EINVAL, "bad LM settings");
  if (Pc->model >= 2) return fail(SABR_EUNSUPPORTED, "LM takes GLOBAL4 and LMM12 plans");
  sabr_plan *P = const_cast<sabr_plan *>(Pc);
  const int Pn = P->np;
  for (int i = 0; i < P->n_inst * Pn; ++i)
    if (!std::isfinite(lb[i]) || !std::isfinite(ub[i]) || !(lb[i] <= ub[i]))
      return fail(SABR_EINVAL, "box bound " + std::to_string(i) + ": need finite lb <= ub");
  const AdjLayout A = adj_layout(P);
  if (!workspace || ws_bytes < A.total) return fail(SABR_EWORKSPACE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(SABR_EINVAL, "workspace not 256-byte aligned");
  char *w = static_cast<char *>(workspace);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> guard(P->mu);
  std::vector<unsigned char> &stg = P->lm_staging;
  stg.assign(A.total, 0);
  std::memcpy(stg.data() + A.o_lb, lb, sizeof(double) * P->n_inst * Pn);
  std::memcpy(stg.data() + A.o_ub, ub, sizeof(double) * P->n_inst * Pn);
  hipError_t e = hipMemcpyAsync(w, stg.data(), A.total, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "LM box upload");
  e = sabr::launch_lm(P->dm, n_pts, pt_inst, params, reinterpret_cast<const double *>(w + A.o_lb),
                      reinterpret_cast<const double *>(w + A.o_ub), max_iter, mu0, tol, cost_out,
                      iters_out, s);
  if (e != hipSuccess) return hip_fail(e, "LM launch");
  return SABR_OK;
}

size_t sabr_nm_workspace_size(const sabr_plan *P) {
  if (!P) return 0;
  Layout L;
  L.take<double>((size_t)P->n_inst * P->np);
  L.take<double>((size_t)P->n_inst * P->np);
  return L.off;
}

sabr_status sabr_nm_polish(const sabr_plan *Pc, int32_t n_pts, const int32_t *pt_inst,
                           double *params, const double *lb, const double *ub, int32_t max_iter,
                           double step, double tol, double *cost_out, int32_t *iters_out,
                           void *workspace, size_t ws_bytes, void *stream) {
  sabr_status st = check_points(Pc, n_pts);
  if (st != SABR_OK) return st;
  if (n_pts == 0) return SABR_OK;
  if (!pt_inst || !params || !lb || !ub) return fail(SABR_EINVAL, "null argument");
  if (max_iter < 0 || !(step > 0.0 && step <= 1.0) || !(tol >= 0.0))
    return fail(SABR_EINVAL, "bad Nelder-Mead settings");
  sabr_plan *P = const_cast<sabr_plan *>(Pc);
  const int Pn = P->np;
  for (int i = 0; i < P->n_inst * Pn; ++i)
    if (!std::isfinite(lb[i]) || !std::isfinite(ub[i]) || !(lb[i] <= ub[i]))
      return fail(SABR_EINVAL, "box bound " + std::to_string(i) + ": need finite lb <= ub");
  const size_t need = sabr_nm_workspace_size(P);
  if (!workspace || ws_bytes < need) return fail(SABR_EWORKSPACE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(SABR_EINVAL, "workspace not 256-byte aligned");
  if (sabr::nm_lds_bytes(P->dm) > 160 * 1024) return fail(SABR_EUNSUPPORTED, "simplex does not fit in LDS");
  Layout L;
  const size_t o_lb = L.take<double>((size_t)P->n_inst * Pn);
  const size_t o_ub = L.take<double>((size_t)P->n_inst * Pn);
  char *w = static_cast<char *>(workspace);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> guard(P->mu);
  std::vector<unsigned char> &stg = P->nm_staging;
  stg.assign(L.off, 0);
  std::memcpy(stg.data() + o_lb, lb, sizeof(double) * P->n_inst * Pn);
  std::memcpy(stg.data() + o_ub, ub, sizeof(double) * P->n_inst * Pn);
  hipError_t e = hipMemcpyAsync(w, stg.data(), L.off, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "Nelder-Mead box upload");
  e = sabr::launch_nm(P->dm, n_pts, pt_inst, params, reinterpret_cast<const double *>(w + o_lb),
                      reinterpret_cast<const double *>(w + o_ub), max_iter, step, tol, cost_out,
                      iters_out, s);
  if (e != hipSuccess) return hip_fail(e, "Nelder-Mead launch");
  return SABR_OK;
}

}  // extern "C"
