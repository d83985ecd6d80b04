// Host side of libpr: argument checking, workspace, the captured-graph
// solve loop, and the C ABI declared in include/pr.h.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/pr.h"
#include "pr_internal.h"

using namespace pr;

#define PR_TRY(expr)                          \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return PR_EDEVICE;  \
  } while (0)

namespace {

int vec_of(int xdt) { return xdt == kF64 ? 2 : (xdt == kF32 ? 4 : 8); }
size_t esize(int xdt) { return xdt == kF64 ? 8 : (xdt == kF32 ? 4 : 2); }

template <typename T>
hipError_t dalloc(T **p, size_t count) {
  return hipMalloc((void **)p, sizeof(T) * (count > 0 ? count : 1));
}

constexpr int kLanczosMax = 512;   // Lanczos steps for ||X||_2^2 at most
constexpr int kLanczosCheck = 8;   // steps between convergence checks on the host
constexpr int kUnionRebuilds = 16;  // checks for new coordinates of the batch's support union per solve

}  // namespace

struct pr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream used only for graph capture
  Problem P{};
  double norm2 = 0.0;
  int32_t max_batch = 1;
  NodeParams *d_prm = nullptr;
  NodeState *d_state = nullptr;
  NodeState *h_state = nullptr;  // pinned, 2 slots
  int8_t *d_status = nullptr;
  uint32_t *d_stp = nullptr;     // the status packed 2 bits per entry (NodeParams::stp)
  std::vector<uint32_t> h_stp;
  NodeBufs nb{};
  ProbBufs B{};
  int32_t *iota = nullptr;
  int32_t *d_np = nullptr;       // holds p (dense column list length)
  double *d_u = nullptr;         // n
  double *d_v = nullptr;         // p
  double *d_w = nullptr;         // p
  double *d_scal = nullptr;      // small scalars
  double *d_lam = nullptr;       // Lanczos coefficients: alpha [kLanczosMax], beta [kLanczosMax]
  double *d_vprev = nullptr;     // p: previous Lanczos vector
  double *d_regscratch = nullptr;  // 3p
  hipGraphExec_t gexec = nullptr;
  hipGraphExec_t gtail = nullptr;  // the same iterations, kTailUnits of them (the last ones of a solve)
  int32_t graph_units = 0;
  bool graph_gram = false;  // the iteration graph was captured in Gram mode
  bool step_bt = false;     // the next solve's step is the backtracking variant
  bool graph_bt = false;    // ... and the captured graph's is
  int32_t debug = 0;        // pr_ctx_set_debug flags
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t tev[2] = {nullptr, nullptr};
  // batched path (both losses, X in any storage type, n and p multiples of 128, p <= 16384)
  bool batch_ok = false;
  int32_t KS = 1, KSF = 1, nfb = 0;
  int32_t fmaxF = 1, fmaxT = 1;  // largest extra split factors of the two GEMMs
  int32_t rs = 1;            // rows of the second product per node (logistic: zeta and the momentum gradient)
  void *Xrow = nullptr;      // row-major copy of X (n x p), X's storage type
  double *Bx = nullptr;      // [cap padded][p] FP64 current iterates
  double *Rd = nullptr;      // [rs cap padded][n] FP64 residual / loss rows
  double *CF = nullptr;      // [KSF][cap padded][n]
  double *CT = nullptr;      // [KS][rs cap padded][p]
  double *Uprev = nullptr;   // logistic: [cap][n] X x of each node's previous (backtracking: last accepted) iterate
  double *Ucur = nullptr, *Uy = nullptr;  // logistic backtracking: X x of the last evaluation, X y of the pending trial
  double *bdsum = nullptr;   // logistic backtracking: [cap][nfb] Bregman remainder sums
  double *bybt = nullptr, *bgbt = nullptr;  // backtracking: [cap][p] momentum point and grad f there
  int32_t *d_rowmap2 = nullptr;  // logistic: [2 cap padded] rows of the second product of the nodes still iterating
  double *fsum = nullptr;    // [cap][nfb][2]
  double *bx0 = nullptr, *bx1 = nullptr, *bxbest = nullptr, *bhprev = nullptr, *bsval = nullptr;
  int32_t *bsidx = nullptr;
  int8_t *bstatus = nullptr;
  NodeParams *d_bprm = nullptr;
  NodeState *d_bstate = nullptr;
  NodeState *h_bstate = nullptr;  // pinned, cap
  int32_t *d_active = nullptr;
  int32_t *d_rowmap = nullptr;    // [cap padded] slots of the nodes still iterating
  int32_t *d_split = nullptr;     // {rows still iterating, forward split, transpose split, compacted Gram split, tile counters x2}
  int32_t *d_ftab = nullptr;      // [kTuneTables][kTuneMax] tuned split factors per active row-tile count
  int32_t h_ftab[kTuneTables * kTuneMax] = {};
  double h_tbest[kTuneTables * kTuneMax] = {};  // measured ms of the chosen split per active row-tile count
  double t_gemv_ms = 0.0;                       // one X^T pass of the single-node iteration (measured)
  // batched Gram mode: U = G X_it planes [KSG * f][cap padded][p] (CT's storage when it is large enough)
  int32_t KSG = 1, fmaxG = 1;
  double *CG = nullptr;
  bool cg_own = false, gram_batch_ok = false;
  uint32_t *bstp = nullptr;        // [cap][stpw] packed node status of the batch
  std::vector<uint32_t> h_bstp;
  int32_t *h_active = nullptr;    // pinned, 2 slots
  hipGraphExec_t bgexec = nullptr;
  int32_t bgraph_units = 0, bgraph_m = 0;
  int64_t bgraph_kp = 0, bgraph_ku = 0;
  // support-union compaction of the batched product with the iterates (built per pr_solve_batch)
  bool union_on = false;
  int64_t ku = 0, kp = 0;           // union size, padded to the GEMM's reduction granule
  int64_t union_nout = 0;           // nonzeros outside the union at the nodes' last iterates
  int32_t *d_umask = nullptr;       // [p]
  int32_t *d_ulist = nullptr;       // [p] union coordinates, ascending
  int32_t *d_olist = nullptr;       // [p] the other coordinates
  int32_t *d_ocnt = nullptr;        // [cap padded] nonzeros outside the union per node
  int32_t *d_oidx = nullptr;        // [cap padded][p]
  double *d_oval = nullptr;         // [cap padded][p]
  double *BxU = nullptr;            // [cap padded][kp max] compacted iterates
  double *GU = nullptr;             // [p][3p/4] union columns of G (Gram mode)
  void *XrU = nullptr;              // [n][3p/4] union columns of the row-major X copy (products over X)
  // batched certification: per-node scratch [cap padded][p] and {Psi, Phi} per node
  double *cert_a = nullptr, *d_cert = nullptr;
  // least squares from the Gram matrix (pr_ctx_enable_gram)
  bool gram = false;
  double *G = nullptr;   // [p][p] X^T X over the stored X, FP64
  double *gb = nullptr;  // [p] X^T y
  double gyy = 0.0;      // y^T y
  Problem PG{};          // G viewed as the "design" of the column-list GEMV (n = p, y = b)
  ProbBufs BG{};         // its partial sums; h goes to B.h1
  // iteration variants (AC-FGM, LASSO; allocated on first use) and their graph
  AcState *d_ac = nullptr;
  AcBufs ab{};
  LassoState *d_lx = nullptr;
  hipGraphExec_t vgexec = nullptr;
  int32_t vgraph_units = 0;
  int32_t vgraph_kind = -1;   // 0 AC-FGM, 1 + LASSO kind
  double vgraph_key[3] = {0.0, 0.0, 0.0};
  // learned warm start (allocated on first use)
  uint16_t *mF = nullptr;  // [p][8] features of one node
  float *mout = nullptr;   // [p] network outputs
  double *mnz = nullptr;   // [p] compacted nonzero magnitudes
  double *mfs = nullptr;   // {max |w|, nnz}
  double *mvhat = nullptr, *mx = nullptr;  // [p] proposal before / after the prox step
  // batched warm start: proposals, w = X^T zeta at the parents [max_batch padded][p],
  // feature rows [..][p][8], network outputs [..][p]
  double *mVb = nullptr, *mWb = nullptr, *mPb = nullptr;  // mPb: prox(beta_parent) rows
  uint16_t *mFb = nullptr;
  float *moutb = nullptr;
};

namespace {

// Status in the packed layout of NodeParams::stp (3 = beyond p).
void pack_status(const std::vector<int8_t> &st, std::vector<uint32_t> &w) {
  const int64_t p = (int64_t)st.size();
  const int64_t T = kNodeThreads;
  for (size_t k = 0; k < w.size(); k++) {
    const int64_t q = (int64_t)k / T, t = (int64_t)k % T;
    uint32_t v = 0u;
    for (int i = 0; i < 16; i++) {
      const int64_t j = t + (16 * q + i) * T;
      const uint32_t code = (j < p) ? (uint32_t)st[(size_t)j] : 3u;
      v |= code << (2 * i);
    }
    w[k] = v;
  }
}

void free_ctx(pr_ctx *c) {
  if (!c) return;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->gtail) (void)hipGraphExecDestroy(c->gtail);
  if (c->bgexec) (void)hipGraphExecDestroy(c->bgexec);
  if (c->vgexec) (void)hipGraphExecDestroy(c->vgexec);
  {
    void *vb[] = {c->d_ac, c->d_lx, c->ab.xb, c->ab.gb, c->ab.yb, c->ab.xc, c->ab.yc, c->ab.z, c->ab.sidx2,
                  c->ab.sval2, c->ab.uz, c->ab.ucur};
    for (void *b : vb)
      if (b) (void)hipFree(b);
  }
  if (c->cg_own && c->CG) (void)hipFree(c->CG);
  {
    void *ub[] = {c->d_umask, c->d_ulist, c->d_olist, c->d_ocnt, c->d_oidx, c->d_oval, c->BxU, c->GU, c->XrU,
                  c->cert_a, c->d_cert};
    for (void *b : ub)
      if (b) (void)hipFree(b);
  }
  void *bb[] = {c->bstp, c->Xrow, c->Uprev, c->Ucur, c->Uy, c->bdsum, c->bybt, c->bgbt, c->d_rowmap2, c->Bx, c->Rd, c->CF, c->CT, c->fsum, c->bx0, c->bx1, c->bxbest, c->bhprev,
                c->bsval, c->bsidx, c->bstatus, c->d_bprm, c->d_bstate, c->d_active, c->d_rowmap, c->d_split, c->d_ftab, c->mF, c->mout, c->mnz, c->mfs, c->mvhat, c->mx, c->G, c->gb, c->BG.part, c->nb.xlb, c->mVb, c->mWb, c->mFb, c->moutb, c->mPb};
  for (void *b : bb)
    if (b) (void)hipFree(b);
  if (c->h_bstate) (void)hipHostFree(c->h_bstate);
  if (c->h_active) (void)hipHostFree(c->h_active);
  for (int i = 0; i < 2; i++) {
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->tev[i]) (void)hipEventDestroy(c->tev[i]);
  }
  if (c->cap) (void)hipStreamDestroy(c->cap);
  void *bufs[] = {c->d_prm, c->d_state, c->d_status, c->d_stp, c->nb.x0, c->nb.x1, c->nb.xbest, c->nb.hprev, c->nb.vbuf,
                  c->nb.abuf, c->nb.sidx, c->nb.sval, c->nb.ybt, c->nb.gbt, c->B.uy, c->B.dsum, c->B.r, c->B.gm,
                  c->B.ucur, c->B.uprev,
                  c->B.zbest, c->B.h1, c->B.h2, c->B.part, c->B.rbsum, c->iota,
                  c->d_np, c->d_u, c->d_v, c->d_w, c->d_scal, c->d_lam, c->d_vprev, c->d_regscratch};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (c->h_state) (void)hipHostFree(c->h_state);
  delete c;
}

}  // namespace

// Validate a node and build its status vector.  Returns PR_OK, or an error;
// *infeasible is set when |J1| > k.
int pr::build_status(const pr_node *node, int64_t p, std::vector<int8_t> &st, int64_t &n1, int64_t &pbar,
                 int32_t &kbar, bool &infeasible) {
  if (!node) return PR_EINVAL;
  if (node->k < 1 || !(node->lambda2 > 0.0) || !isfinite(node->lambda2) || !(node->M > 0.0))
    return PR_EINVAL;
  if (node->n0 < 0 || node->n1 < 0 || (node->n0 > 0 && !node->J0) || (node->n1 > 0 && !node->J1))
    return PR_EINVAL;
  st.assign((size_t)p, (int8_t)kFree);
  for (int64_t i = 0; i < node->n0; i++) {
    int64_t j = node->J0[i];
    if (j < 0 || j >= p) return PR_EINVAL;
    st[(size_t)j] = (int8_t)kZero;
  }
  for (int64_t i = 0; i < node->n1; i++) {
    int64_t j = node->J1[i];
    if (j < 0 || j >= p) return PR_EINVAL;
    if (st[(size_t)j] == kZero) return PR_EOVERLAP;
    st[(size_t)j] = (int8_t)kOne;
  }
  n1 = 0;
  int64_t nf = 0;
  for (int64_t j = 0; j < p; j++) {
    if (st[(size_t)j] == kOne) n1++;
    else if (st[(size_t)j] == kFree) nf++;
  }
  pbar = nf;
  infeasible = n1 > (int64_t)node->k;
  int64_t kb = infeasible ? 0 : (int64_t)node->k - n1;
  if (kb > nf) kb = nf;
  kbar = (int32_t)kb;
  return PR_OK;
}

const Problem &pr::ctx_problem(const pr_ctx *c) { return c->P; }
hipStream_t pr::ctx_stream(const pr_ctx *c) { return c->stream; }
int32_t pr::ctx_max_batch(const pr_ctx *c) { return c->max_batch; }

namespace {

int check_opts(const pr_opts *o) {
  if (!o) return PR_OK;
  if (!(o->rel_gap_tol >= 0.0) || !(o->eta > 1.0) || o->max_iter < 0 || o->check_every < 1 ||
      !(o->L >= 0.0) || !isfinite(o->L) || o->method < kFistaGap || o->method > kFistaBt)
    return PR_EINVAL;
  if ((o->method == kAcfgmGap || o->method == kAcfgm) &&
      (!(o->acfgm_b > 0.0) || !(o->acfgm_b < 1.0) || !(o->acfgm_c > 1.0) || !isfinite(o->acfgm_c) ||
       !(o->L0 >= 0.0) || !isfinite(o->L0)))
    return PR_EINVAL;
  if (is_bt(o->method) && (!(o->acfgm_c > 1.0) || !isfinite(o->acfgm_c) || !(o->L0 >= 0.0) || !isfinite(o->L0)))
    return PR_EINVAL;
  return PR_OK;
}

double curvature(int loss) { return loss == kLsq ? 2.0 : 0.25; }

// One iteration unit: column-list GEMV + loss epilogue, X^T pass, node step.
// `unit` is the unit's position in the captured graph (its parity selects the
// x buffers; see StepArgs).
hipError_t enqueue_unit(pr_ctx *c, hipStream_t s, int unit) {
  const StepArgs a{c->P.p, c->d_stp, c->gram ? c->gb : nullptr, unit & 1, c->step_bt ? 1 : 0};
  if (c->gram) {
    // h = b - G x over the support of x, then the node step
    hipError_t e = launch_spfwd(c->PG, c->BG, c->nb.sidx, c->nb.sval, &c->d_state->nsupp, kSpGram, c->d_state,
                                nullptr, s);
    if (e != hipSuccess) return e;
    return launch_node_step(c->d_prm, c->d_state, c->nb, c->B, c->P.p, s, &a);
  }
  const int mode = c->P.loss == kLsq ? kSpLsq : kSpLogistic;
  hipError_t e = launch_spfwd(c->P, c->B, c->nb.sidx, c->nb.sval, &c->d_state->nsupp, mode, c->d_state,
                              nullptr, s);
  if (e != hipSuccess) return e;
  // the register-resident node step leaves g_N of its new iterate to an extra
  // workgroup of this product (the strided step evaluates it itself)
  const bool reg = node_ept(c->P.p) != 0;
  e = launch_gemv_t(c->P, c->B.r, c->P.loss == kLsq ? nullptr : c->B.gm, c->B.h1, c->B.h2,
                    &c->d_state->done, s, reg ? c->d_prm : nullptr, c->d_state, c->nb.sidx, c->nb.sval,
                    &c->d_state->nsupp, (reg && c->step_bt) ? c->B.dsum : nullptr, c->B.nfin);
  if (e != hipSuccess) return e;
  return launch_node_step(c->d_prm, c->d_state, c->nb, c->B, c->P.p, s, &a);
}

// Captured iterations of a solve after the node is done still cost their
// launches (each kernel exits at once, ~20 us per iteration): the last ones run
// as launches of a short graph.
constexpr int32_t kTailUnits = 8;

// Capture `units` iteration units into an executable graph.
int capture_units(pr_ctx *c, int32_t units, hipGraphExec_t *out) {
  hipGraph_t g = nullptr;
  PR_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < units && e == hipSuccess; i++) e = enqueue_unit(c, c->cap, i);
  hipError_t e2 = hipStreamEndCapture(c->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return PR_EDEVICE;
  }
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *out = nullptr;
    return PR_EDEVICE;
  }
  return PR_OK;
}

// The iteration graph: `units` iterations rounded up to an even count, so that
// every launch starts with x^k in the first buffer (iterations after the node
// is done exit at once), and the short tail graph when it is shorter.
int ensure_graph(pr_ctx *c, int32_t units) {
  units += units & 1;
  if (c->gexec && c->graph_units == units && c->graph_gram == c->gram && c->graph_bt == c->step_bt) return PR_OK;
  for (hipGraphExec_t *ge : {&c->gexec, &c->gtail})
    if (*ge) {
      (void)hipGraphExecDestroy(*ge);
      *ge = nullptr;
    }
  c->graph_units = 0;
  int rc = capture_units(c, units, &c->gexec);
  if (rc == PR_OK && units > kTailUnits) rc = capture_units(c, kTailUnits, &c->gtail);
  if (rc != PR_OK) return rc;
  c->graph_units = units;
  c->graph_gram = c->gram;
  c->graph_bt = c->step_bt;
  return PR_OK;
}

// Launch a captured iteration graph of `units` iterations until the node state
// reports done or `max_units` iterations have been launched.  Each launch is
// followed by a copy of the node state into its own pinned slot and an event;
// at most two launches are in flight.  Iterations launched after the stop
// still cost their launches, so the host predicts the stop from the rate at
// which the relative gap fell over the last `units` or more evaluations: no
// further launch is queued behind launches that are predicted to reach it, and
// the last iterations run as launches of the short graph `gs` (`sunits`
// iterations) when there is one.  The prediction only decides how much is
// queued; the iterates do not depend on it.
hipError_t run_graph(pr_ctx *c, hipGraphExec_t g, int32_t units, int64_t max_units, double tol,
                     hipGraphExec_t gs = nullptr, int32_t sunits = 0) {
  int slot = 0, head = 0, inflight = 0;
  int32_t qunits[2] = {0, 0};
  int64_t issued = 0;
  auto issue = [&](bool small) -> hipError_t {
    hipError_t e = hipGraphLaunch(small ? gs : g, c->stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&c->h_state[slot], c->d_state, sizeof(NodeState), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return e;
    e = hipEventRecord(c->ev[slot], c->stream);
    if (e != hipSuccess) return e;
    qunits[slot] = small ? sunits : units;
    issued += qunits[slot];
    slot ^= 1;
    inflight++;
    return hipSuccess;
  };
  hipError_t e = issue(false);
  if (e != hipSuccess) return e;
  if (issued < max_units) {
    e = issue(false);
    if (e != hipSuccess) return e;
  }
  // (evaluations, relative gap) at each observation with a finite gap
  std::vector<std::pair<int64_t, double>> hist;
  while (inflight > 0) {
    e = hipEventSynchronize(c->ev[head]);
    if (e != hipSuccess) return e;
    const NodeState h = c->h_state[head];
    head ^= 1;
    inflight--;
    if (h.done) break;
    // evaluations predicted before the stop (infinite while the gap has not
    // fallen over the window)
    const int64_t ev = (int64_t)h.iter + h.trials;
    double rem = INFINITY;
    if (isfinite(h.rel_gap) && h.rel_gap > 0.0) {
      const std::pair<int64_t, double> *base = nullptr;
      for (const auto &o : hist)
        if (ev - o.first >= units || !base) base = &o;
      if (base && ev > base->first && h.rel_gap < base->second && tol > 0.0)
        rem = log(h.rel_gap / tol) * (double)(ev - base->first) / log(base->second / h.rel_gap);
      hist.emplace_back(ev, h.rel_gap);
    }
    double queued = inflight ? (double)qunits[head] : 0.0;
    while (inflight < 2 && issued < max_units) {
      const double need = rem - queued;
      if (inflight > 0 && need <= 0.0) break;
      const bool small = gs && need < (double)units;
      e = issue(small);
      if (e != hipSuccess) return e;
      queued += small ? sunits : units;
    }
  }
  return hipStreamSynchronize(c->stream);
}

// Buffers of the iteration variants, allocated on first use.
int ensure_variant_bufs(pr_ctx *c) {
  if (c->d_ac) return PR_OK;
  const int64_t n = c->P.n, p = c->P.p;
  AcBufs &a = c->ab;
  bool ok = dalloc(&c->d_lx, 1) == hipSuccess;
  ok = ok && dalloc(&a.xb, p) == hipSuccess && dalloc(&a.gb, p) == hipSuccess && dalloc(&a.yb, p) == hipSuccess;
  ok = ok && dalloc(&a.xc, p) == hipSuccess && dalloc(&a.yc, p) == hipSuccess && dalloc(&a.z, p) == hipSuccess;
  ok = ok && dalloc(&a.sidx2, p) == hipSuccess && dalloc(&a.sval2, p) == hipSuccess;
  ok = ok && dalloc(&a.uz, n) == hipSuccess && dalloc(&a.ucur, n) == hipSuccess;
  ok = ok && dalloc(&c->d_ac, 1) == hipSuccess;  // last: marks the set complete
  if (!ok) return PR_ENOMEM;
  PR_TRY(hipMemsetAsync(a.ucur, 0, sizeof(double) * n, c->stream));
  return PR_OK;
}

// One unit of an iteration variant: AC-FGM (kind 0) or LASSO (kind 1 + form).
hipError_t enqueue_variant_unit(pr_ctx *c, hipStream_t s, int kind, const double *key) {
  if (kind == 0) {
    hipError_t e = launch_spfwd(c->P, c->B, c->nb.sidx, c->nb.sval, &c->d_state->nsupp, kSpPlain, c->d_state,
                                c->ab.uz, s);
    if (e == hipSuccess) e = launch_ac_resid(c->P, c->B, c->ab.uz, c->ab.ucur, c->d_state, c->d_ac, s);
    if (e == hipSuccess) e = launch_gemv_t(c->P, c->B.r, nullptr, c->B.h1, nullptr, &c->d_state->done, s);
    if (e == hipSuccess)
      e = launch_ac_step(c->d_prm, c->d_state, c->d_ac, c->ab, c->nb, c->B, key[0], key[1], (int32_t)key[2], s);
    return e;
  }
  hipError_t e = launch_spfwd(c->P, c->B, c->nb.sidx, c->nb.sval, &c->d_state->nsupp, kSpLsq, c->d_state, nullptr,
                              s);
  if (e == hipSuccess) e = launch_gemv_t(c->P, c->B.r, nullptr, c->B.h1, nullptr, &c->d_state->done, s);
  if (e == hipSuccess) e = launch_lasso_step(c->d_prm, c->d_state, c->d_lx, c->nb, c->B, kind - 1, key[0], s);
  return e;
}

// The captured graph of `units` variant iterations; the step parameters that
// the kernels take as arguments are part of the cache key.
int ensure_variant_graph(pr_ctx *c, int kind, const double *key, int32_t units) {
  if (c->vgexec && c->vgraph_units == units && c->vgraph_kind == kind && c->vgraph_key[0] == key[0] &&
      c->vgraph_key[1] == key[1] && c->vgraph_key[2] == key[2])
    return PR_OK;
  if (c->vgexec) {
    (void)hipGraphExecDestroy(c->vgexec);
    c->vgexec = nullptr;
  }
  hipGraph_t g = nullptr;
  PR_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < units && e == hipSuccess; i++) e = enqueue_variant_unit(c, c->cap, kind, key);
  hipError_t e2 = hipStreamEndCapture(c->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return PR_EDEVICE;
  }
  e = hipGraphInstantiate(&c->vgexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->vgexec = nullptr;
    return PR_EDEVICE;
  }
  c->vgraph_units = units;
  c->vgraph_kind = kind;
  for (int i = 0; i < 3; i++) c->vgraph_key[i] = key[i];
  return PR_OK;
}

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal
// a[0..m) and off-diagonal b[0..m-1), by bisection on the Sturm count (the
// number of negative pivots of T - x I = L D L^T is the number of eigenvalues
// below x), started from the Gershgorin interval.  Returns the upper end of
// the final interval.
double tridiag_max_eig(const double *a, const double *b, int m) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; i++) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  hi += 1e-15 * fabs(hi) + 1e-300;
  auto below = [&](double x) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < m; i++) {
      d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) cnt++;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 2e-16 * std::max(fabs(lo), fabs(hi)); it++) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) == m) hi = mid;
    else lo = mid;
  }
  return hi;
}

// ||X||_2^2 = lambda_max(X^T X) by the Lanczos recurrence on X^T X from a
// fixed pseudo-random direction: each step is one product X v, one X^T u and one
// single-workgroup update, with no host round trip; every kLanczosCheck steps
// the host takes the top eigenvalue of the tridiagonal matrix of the
// recurrence coefficients (a lower bound that rises to lambda_max) and stops
// once it moved by at most 1e-13 relative over the last check interval, when
// the recurrence breaks down (an invariant subspace that holds every
// eigenvector the start direction touches, generically all: the value is
// exact), or
// after min(p, kLanczosMax) steps.  Without reorthogonalisation the extreme
// value still converges; lost orthogonality only repeats converged values.
int lanczos_norm2(pr_ctx *c) {
  const int64_t n = c->P.n, p = c->P.p;
  // start vector: fixed pseudo-random entries (splitmix64 of the index) with
  // random signs, so that no structure of X^T X (an eigenvector orthogonal to
  // the all-ones direction, say) can hide its top eigenvector from the
  // recurrence; the same vector on every run
  std::vector<double> v0((size_t)p);
  double nv = 0.0;
  for (int64_t j = 0; j < p; j++) {
    uint64_t z = (uint64_t)j * 0x9E3779B97F4A7C15ull + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = 0.5 + (double)(z >> 11) * 0x1.0p-53;   // [0.5, 1.5)
    v0[(size_t)j] = (z & 1u) ? -u : u;
    nv += u * u;
  }
  nv = 1.0 / sqrt(nv);
  for (double &x : v0) x *= nv;
  PR_TRY(hipMemcpyAsync(c->d_v, v0.data(), sizeof(double) * p, hipMemcpyHostToDevice, c->stream));
  double *alpha = c->d_lam, *beta = c->d_lam + kLanczosMax;
  std::vector<double> ha(kLanczosMax), hb(kLanczosMax);
  const int mmax = (int)std::min<int64_t>(kLanczosMax, p);
  double prev = -1.0;
  for (int j = 0; j < mmax; j++) {
    if (launch_spfwd(c->P, c->B, c->iota, c->d_v, c->d_np, kSpPlain, nullptr, c->d_u, c->stream) != hipSuccess)
      return PR_EDEVICE;
    PR_TRY(launch_sumsq(c->d_u, n, alpha + j, c->stream));
    PR_TRY(launch_gemv_t(c->P, c->d_u, nullptr, c->d_w, nullptr, nullptr, c->stream));
    PR_TRY(launch_lanczos(c->d_w, c->d_v, c->d_vprev, alpha + j, j > 0 ? beta + j - 1 : nullptr, beta + j, p,
                          c->stream));
    const int m = j + 1;
    if (m % kLanczosCheck != 0 && m != mmax) continue;
    PR_TRY(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * m, hipMemcpyDeviceToHost, c->stream));
    PR_TRY(hipMemcpyAsync(hb.data(), beta, sizeof(double) * m, hipMemcpyDeviceToHost, c->stream));
    PR_TRY(hipStreamSynchronize(c->stream));
    const double th = tridiag_max_eig(ha.data(), hb.data(), m);
    c->norm2 = th;
    if (!(hb[(size_t)m - 1] > 1e-14 * th)) return PR_OK;
    if (prev > 0.0 && th - prev <= 1e-13 * th) return PR_OK;
    prev = th;
  }
  return PR_OK;
}

int nr_of(int32_t m) { return (m + 63) / 64 * 64; }

// Autotuner of the batched GEMMs (run once per context).  For every count of
// active 64-row tiles, each extra split factor f of each GEMM (a tile's extent
// along the reduction dimension is K / (base * f)) is timed with HIP events in
// the solve's launch configuration (persistent grid, row map, tile counter);
// the chosen f minimises the measured time plus the modelled cost of the
// split partial planes that the next kernel reads (bytes / kTunePlaneBW).
// The table goes to the device, where the per-iteration row-map kernel reads
// it.
int tune_batch(pr_ctx *c) {
  const int64_t n = c->P.n, p = c->P.p;
  const int NrMax = nr_of(c->max_batch), NrMaxT = nr_of(c->rs * c->max_batch);
  hipStream_t s = c->stream;
  PR_TRY(launch_iota(c->d_rowmap, NrMax, s));
  if (c->d_rowmap2) PR_TRY(launch_iota(c->d_rowmap2, NrMaxT, s));
  int32_t *cnt = c->d_split + 4;
  for (int g = 0; g < 2; g++) {
    const bool fwd = g == 0;
    const int base = fwd ? c->KSF : c->KS, fmax = fwd ? c->fmaxF : c->fmaxT;
    const double plane_bytes = 8.0 * (double)(fwd ? n : p);  // per row and split plane
    // the second product has rs rows per node: its table is indexed by its own row-tile count
    const int rows = fwd ? c->max_batch : c->rs * c->max_batch;
    const int nrmax = fwd ? NrMax : NrMaxT;
    const int ntmax = nrmax / 64 < kTuneMax - 1 ? nrmax / 64 : kTuneMax - 1;
    int32_t *rmap = (!fwd && c->d_rowmap2) ? c->d_rowmap2 : c->d_rowmap;
    for (int nta = 1; nta <= ntmax; nta++) {
      const int32_t nrow = nta * 64 < rows ? nta * 64 : rows;
      double best = INFINITY;
      int bestf = 1;
      for (int f = 1; f <= fmax; f *= 2) {
        const int32_t sp[3] = {nrow, base * f, base * f};
        PR_TRY(hipMemcpyAsync(c->d_split, sp, sizeof(sp), hipMemcpyHostToDevice, s));
        auto launch = [&]() -> hipError_t {
          hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t), s);
          if (e != hipSuccess) return e;
          if (fwd)
            return launch_gemm_any(c->P.xdt, c->Xrow, p, kF64, c->Bx, p, c->CF, n, NrMax, p, base, nullptr,
                                   c->d_rowmap, c->d_split, c->d_split + 1, base * fmax, cnt, s);
          return launch_gemm_any(c->P.xdt, c->P.X, n, kF64, c->Rd, n, c->CT, p, NrMaxT, n, base, nullptr, rmap,
                                 c->d_split, c->d_split + 2, base * fmax, cnt, s);
        };
        PR_TRY(launch());
        PR_TRY(hipEventRecord(c->tev[0], s));
        for (int r = 0; r < kTuneReps; r++) PR_TRY(launch());
        PR_TRY(hipEventRecord(c->tev[1], s));
        PR_TRY(hipEventSynchronize(c->tev[1]));
        float ms = 0.0f;
        PR_TRY(hipEventElapsedTime(&ms, c->tev[0], c->tev[1]));
        const double cost = ms / kTuneReps + 1e3 * (double)(base * f) * nrow * plane_bytes / kTunePlaneBW;
        if (cost < best) {
          best = cost;
          bestf = f;
        }
      }
      c->h_ftab[g * kTuneMax + nta] = bestf;
      c->h_tbest[g * kTuneMax + nta] = best;
    }
    for (int nta = ntmax + 1; nta < kTuneMax; nta++) {
      c->h_ftab[g * kTuneMax + nta] = c->h_ftab[g * kTuneMax + ntmax];
      c->h_tbest[g * kTuneMax + nta] = c->h_tbest[g * kTuneMax + ntmax];
    }
    c->h_ftab[g * kTuneMax] = 1;
  }
  PR_TRY(hipMemcpyAsync(c->d_ftab, c->h_ftab, sizeof(c->h_ftab), hipMemcpyHostToDevice, s));
  // one X^T pass of the single-node path (its form for this loss), for the
  // choice between the batched and the one-at-a-time path (batch_pays)
  {
    const bool two = c->P.loss == kLogistic;
    auto pass = [&]() {
      return launch_gemv_t(c->P, c->B.r, two ? c->B.gm : nullptr, c->B.h1, two ? c->B.h2 : nullptr, nullptr, s);
    };
    PR_TRY(pass());
    PR_TRY(hipEventRecord(c->tev[0], s));
    for (int r = 0; r < kTuneReps; r++) PR_TRY(pass());
    PR_TRY(hipEventRecord(c->tev[1], s));
    PR_TRY(hipEventSynchronize(c->tev[1]));
    float ms = 0.0f;
    PR_TRY(hipEventElapsedTime(&ms, c->tev[0], c->tev[1]));
    c->t_gemv_ms = (double)ms / kTuneReps;
  }
  PR_TRY(hipStreamSynchronize(s));
  return PR_OK;
}

// Whether m nodes go faster through the batched iteration than one at a time:
// per iteration, the batch costs its two GEMMs at m active rows (the tuned
// times; Gram mode its one product) plus the node steps, the single-node path
// m times one X^T pass plus the product over the support and the step
// (Gram mode: the product over the support's Gram columns and the step).  A
// 64-row MFMA tile costs the same for 1 node as for 64, so small rounds
// (typically the first levels of a branch-and-bound tree) run one at a time.
bool batch_pays(const pr_ctx *c, int32_t m) {
  int nta = nr_of(m) / 64, nta2 = nr_of(c->rs * m) / 64;
  if (nta >= kTuneMax) nta = kTuneMax - 1;
  if (nta2 >= kTuneMax) nta2 = kTuneMax - 1;
  const double step = 0.03;  // ms: the batched node steps / one single-node step
  double t_batch, t_single;
  if (c->gram && c->gram_batch_ok) {
    t_batch = c->h_tbest[2 * kTuneMax + nta] + step;
    t_single = 0.4 * c->t_gemv_ms + step;
  } else {
    t_batch = c->h_tbest[nta] + c->h_tbest[kTuneMax + nta2] + step;
    t_single = 1.3 * c->t_gemv_ms + step;
  }
  return (double)m * t_single >= t_batch;
}

// Split factor of the second product (X^T R) for a batch of m nodes: the
// tuned factor for its row-tile count (rs rows per node).
int32_t kst_for(const pr_ctx *c, int32_t m) {
  int nta = nr_of(c->rs * m) / 64;
  if (nta >= kTuneMax) nta = kTuneMax - 1;
  return c->KS * c->h_ftab[kTuneMax + nta];
}

int alloc_batch(pr_ctx *c) {
  const int64_t n = c->P.n, p = c->P.p;
  const int cap = c->max_batch;
  c->rs = c->P.loss == kLogistic ? 2 : 1;
  const int NrMax = nr_of(cap), NrMaxT = nr_of(c->rs * cap);
  // split the reductions so that each GEMM has >= ~1024 workgroups at full batch
  const int tiles_t = (int)(p / 128) * (NrMaxT / 64);
  int KS = 1;
  while (KS < 16 && tiles_t * KS < 512 && (n / (2 * KS)) % 32 == 0) KS *= 2;
  const int tiles_f = (int)(n / 128) * (NrMax / 64);
  int KSF = 1;
  while (KSF < 16 && tiles_f * KSF < 512 && (p / (2 * KSF)) % 32 == 0) KSF *= 2;
  // extra split factors of the two GEMMs (chosen per iteration from the
  // number of active row tiles), up to 16 while the split stays a multiple of 32
  int fF = 1, fT = 1;
  while (2 * fF <= 16 && (p / (2 * fF * KSF)) % 32 == 0 && p % (2 * fF * KSF) == 0) fF *= 2;
  while (2 * fT <= 16 && (n / (2 * fT * KS)) % 32 == 0 && n % (2 * fT * KS) == 0) fT *= 2;
  c->KS = KS;
  c->KSF = KSF;
  c->fmaxF = fF;
  c->fmaxT = fT;
  c->nfb = batch_resid_blocks(n);
  bool ok = hipMalloc(&c->Xrow, esize(c->P.xdt) * (size_t)n * p) == hipSuccess;
  ok = ok && dalloc(&c->Bx, (size_t)NrMax * p) == hipSuccess;
  ok = ok && dalloc(&c->Rd, (size_t)NrMaxT * n) == hipSuccess;
  ok = ok && dalloc(&c->CF, (size_t)KSF * fF * NrMax * n) == hipSuccess;
  ok = ok && dalloc(&c->CT, (size_t)KS * fT * NrMaxT * p) == hipSuccess;
  if (c->rs == 2) {
    ok = ok && dalloc(&c->Uprev, (size_t)cap * n) == hipSuccess;
    ok = ok && dalloc(&c->Ucur, (size_t)cap * n) == hipSuccess && dalloc(&c->Uy, (size_t)cap * n) == hipSuccess;
    ok = ok && dalloc(&c->bdsum, (size_t)cap * batch_resid_blocks(n)) == hipSuccess;
    ok = ok && dalloc(&c->d_rowmap2, NrMaxT) == hipSuccess;
  }
  ok = ok && dalloc(&c->bybt, (size_t)cap * p) == hipSuccess && dalloc(&c->bgbt, (size_t)cap * p) == hipSuccess;
  ok = ok && dalloc(&c->fsum, (size_t)2 * cap * c->nfb) == hipSuccess;
  ok = ok && dalloc(&c->bx0, (size_t)cap * p) == hipSuccess && dalloc(&c->bx1, (size_t)cap * p) == hipSuccess;
  ok = ok && dalloc(&c->bxbest, (size_t)cap * p) == hipSuccess && dalloc(&c->bhprev, (size_t)cap * p) == hipSuccess;
  ok = ok && dalloc(&c->bsval, (size_t)cap * p) == hipSuccess && dalloc(&c->bsidx, (size_t)cap * p) == hipSuccess;
  ok = ok && dalloc(&c->bstatus, (size_t)cap * p) == hipSuccess;
  ok = ok && dalloc(&c->bstp, (size_t)cap * c->h_stp.size()) == hipSuccess;
  ok = ok && dalloc(&c->d_bprm, cap) == hipSuccess && dalloc(&c->d_bstate, cap) == hipSuccess;
  ok = ok && dalloc(&c->d_active, 2) == hipSuccess;
  // d_split: {rows iterating, forward split, second split, compacted split, tile counters x2,
  // certification split, -, rows of the second product}
  ok = ok && dalloc(&c->d_rowmap, NrMax) == hipSuccess && dalloc(&c->d_split, 12) == hipSuccess;
  ok = ok && dalloc(&c->d_ftab, kTuneTables * kTuneMax) == hipSuccess;
  ok = ok && hipHostMalloc((void **)&c->h_bstate, sizeof(NodeState) * cap, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void **)&c->h_active, 2 * sizeof(int32_t), hipHostMallocDefault) == hipSuccess;
  if (!ok) return PR_ENOMEM;
  ok = hipMemsetAsync(c->Bx, 0, sizeof(double) * NrMax * p, c->stream) == hipSuccess;
  ok = ok && hipMemsetAsync(c->Rd, 0, sizeof(double) * NrMaxT * n, c->stream) == hipSuccess;
  for (double *u : {c->Uprev, c->Ucur, c->Uy})
    if (u) ok = ok && hipMemsetAsync(u, 0, sizeof(double) * cap * n, c->stream) == hipSuccess;
  ok = ok && launch_transpose(c->P.xdt, c->P.X, c->Xrow, n, p, c->stream) == hipSuccess;
  ok = ok && hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) return PR_EDEVICE;
  int rc = tune_batch(c);
  if (rc != PR_OK) return rc;
  c->batch_ok = true;
  return PR_OK;
}

// Batched Gram mode (least squares, after pr_ctx_enable_gram): one product
// U = G X_it per iteration in place of the two products with X.  Its base
// split, plane storage and autotuned split table (ftab row 2, same cost model
// as tune_batch).
int tune_gram_batch(pr_ctx *c) {
  const int64_t p = c->P.p;
  const int NrMax = nr_of(c->max_batch);
  const int tiles = (int)(p / 128) * (NrMax / 64);
  int KSG = 1;
  while (KSG < 16 && tiles * KSG < 512 && (p / (2 * KSG)) % 32 == 0) KSG *= 2;
  int fG = 1;
  while (2 * fG <= 16 && (p / (2 * fG * KSG)) % 32 == 0 && p % (2 * fG * KSG) == 0) fG *= 2;
  c->KSG = KSG;
  c->fmaxG = fG;
  if (KSG * fG <= c->KS * c->fmaxT) {
    c->CG = c->CT;
    c->cg_own = false;
  } else {
    if (dalloc(&c->CG, (size_t)KSG * fG * NrMax * p) != hipSuccess) return PR_ENOMEM;
    c->cg_own = true;
  }
  const int ntmax = NrMax / 64 < kTuneMax - 1 ? NrMax / 64 : kTuneMax - 1;
  hipStream_t s = c->stream;
  PR_TRY(launch_iota(c->d_rowmap, NrMax, s));
  int32_t *cnt = c->d_split + 4;
  const double plane_bytes = 8.0 * (double)p;
  for (int nta = 1; nta <= ntmax; nta++) {
    const int32_t nrow = nta * 64 < c->max_batch ? nta * 64 : c->max_batch;
    double best = INFINITY;
    int bestf = 1;
    for (int f = 1; f <= fG; f *= 2) {
      const int32_t sp[3] = {nrow, KSG * f, KSG * f};
      PR_TRY(hipMemcpyAsync(c->d_split, sp, sizeof(sp), hipMemcpyHostToDevice, s));
      auto launch = [&]() -> hipError_t {
        hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t), s);
        if (e != hipSuccess) return e;
        return launch_gemm_any(kF64, c->G, p, kF64, c->Bx, p, c->CG, p, NrMax, p, KSG, nullptr, c->d_rowmap,
                               c->d_split, c->d_split + 2, KSG * fG, cnt, s);
      };
      PR_TRY(launch());
      PR_TRY(hipEventRecord(c->tev[0], s));
      for (int r = 0; r < kTuneReps; r++) PR_TRY(launch());
      PR_TRY(hipEventRecord(c->tev[1], s));
      PR_TRY(hipEventSynchronize(c->tev[1]));
      float ms = 0.0f;
      PR_TRY(hipEventElapsedTime(&ms, c->tev[0], c->tev[1]));
      const double cost = ms / kTuneReps + 1e3 * (double)(KSG * f) * nrow * plane_bytes / kTunePlaneBW;
      if (cost < best) {
        best = cost;
        bestf = f;
      }
    }
    c->h_ftab[2 * kTuneMax + nta] = bestf;
    c->h_tbest[2 * kTuneMax + nta] = best;
  }
  for (int nta = ntmax + 1; nta < kTuneMax; nta++) {
    c->h_ftab[2 * kTuneMax + nta] = c->h_ftab[2 * kTuneMax + ntmax];
    c->h_tbest[2 * kTuneMax + nta] = c->h_tbest[2 * kTuneMax + ntmax];
  }
  c->h_ftab[2 * kTuneMax] = 1;
  PR_TRY(hipMemcpyAsync(c->d_ftab, c->h_ftab, sizeof(c->h_ftab), hipMemcpyHostToDevice, s));
  PR_TRY(hipStreamSynchronize(s));
  c->gram_batch_ok = true;
  return PR_OK;
}

BatchBufs batch_bufs(pr_ctx *c, int32_t m) {
  BatchBufs bb{};
  bb.m = m;
  bb.Nr = nr_of(m);
  bb.rs = c->gram ? 1 : c->rs;
  bb.NrT = c->gram ? bb.Nr : nr_of(c->rs * m);
  bb.loss = c->P.loss;
  bb.ksp = c->d_split + (c->gram && c->union_on ? 3 : 2);  // planes of the product the step sums
  bb.nfb = c->nfb;
  bb.x0 = c->bx0;
  bb.x1 = c->bx1;
  bb.xbest = c->bxbest;
  bb.hprev = c->bhprev;
  bb.sidx = c->bsidx;
  bb.sval = c->bsval;
  bb.CT = c->gram ? c->CG : c->CT;
  bb.fsum = c->fsum;
  bb.Bx = c->Bx;
  bb.active = c->d_active;
  bb.gap_factor = 0.99;
  bb.p = c->P.p;
  bb.stp = c->bstp;
  bb.stpw = (int64_t)c->h_stp.size();
  bb.gb = c->gram ? c->gb : nullptr;
  bb.gyy = c->gyy;
  bb.ybt = c->bybt;
  bb.gbt = c->bgbt;
  bb.dsum = c->bdsum;
  return bb;
}

// One batched iteration: forward GEMM, residual split, X^T R GEMM, node steps
// (Gram mode: the product G X_it, node steps).
hipError_t enqueue_batch_unit(pr_ctx *c, int32_t m, hipStream_t s) {
  const int64_t n = c->P.n, p = c->P.p;
  const int Nr = nr_of(m);
  hipError_t e;
  if (c->gram) {
    e = launch_batch_rowmap(c->d_bstate, m, c->d_rowmap, c->d_split, c->d_split + 4, c->d_ftab, c->KSF, c->KSG, 2,
                            c->union_on ? c->kp : p, p, 1, nullptr, s);
    if (e != hipSuccess) return e;
    if (c->union_on) {
      e = launch_union_compact(c->Bx, p, c->d_rowmap, c->d_split, Nr, c->d_ulist, c->ku, c->kp, c->d_olist,
                               p - c->ku, c->BxU, c->d_ocnt, c->d_oidx, c->d_oval, c->d_active, s);
      if (e != hipSuccess) return e;
      e = launch_gemm_any(kF64, c->GU, c->kp, kF64, c->BxU, c->kp, c->CG, p, Nr, c->kp, c->KSG, c->d_active,
                          c->d_rowmap, c->d_split, c->d_split + 3, c->KSG * c->fmaxG, c->d_split + 4, s);
      if (e != hipSuccess) return e;
      e = launch_union_fix(c->G, p, c->d_rowmap, c->d_split, Nr, c->d_ocnt, c->d_oidx, c->d_oval, c->CG,
                           c->d_active, s);
    } else {
      e = launch_gemm_any(kF64, c->G, p, kF64, c->Bx, p, c->CG, p, Nr, p, c->KSG, c->d_active, c->d_rowmap,
                          c->d_split, c->d_split + 2, c->KSG * c->fmaxG, c->d_split + 4, s);
    }
    if (e != hipSuccess) return e;
    return launch_batch_step(c->d_bprm, c->d_bstate, batch_bufs(c, m), p, s);
  }
  const int xdt = c->P.xdt;
  const bool two = c->rs == 2;
  e = launch_batch_rowmap(c->d_bstate, m, c->d_rowmap, c->d_split, c->d_split + 4, c->d_ftab, c->KSF, c->KS, 1,
                          c->union_on ? c->kp : p, p, c->rs, c->d_rowmap2, s);
  if (e != hipSuccess) return e;
  if (c->union_on) {
    e = launch_union_compact(c->Bx, p, c->d_rowmap, c->d_split, Nr, c->d_ulist, c->ku, c->kp, c->d_olist, p - c->ku,
                             c->BxU, c->d_ocnt, c->d_oidx, c->d_oval, c->d_active, s);
    if (e != hipSuccess) return e;
    e = launch_gemm_any(xdt, c->XrU, c->kp, kF64, c->BxU, c->kp, c->CF, n, Nr, c->kp, c->KSF, c->d_active,
                        c->d_rowmap, c->d_split, c->d_split + 3, c->KSF * c->fmaxF, c->d_split + 4, s);
    if (e != hipSuccess) return e;
    e = launch_union_fix_x(xdt, c->P.X, n, p, c->d_rowmap, c->d_split, Nr, c->d_ocnt, c->d_oidx, c->d_oval, c->CF,
                           c->d_active, s);
  } else {
    e = launch_gemm_any(xdt, c->Xrow, p, kF64, c->Bx, p, c->CF, n, Nr, p, c->KSF, c->d_active, c->d_rowmap,
                        c->d_split, c->d_split + 1, c->KSF * c->fmaxF, c->d_split + 4, s);
  }
  if (e != hipSuccess) return e;
  e = launch_batch_resid(c->CF, c->union_on ? c->d_split + 3 : c->d_split + 1, n, m, Nr, c->P.y, c->Rd, c->fsum,
                         c->d_bstate, c->P.loss, c->Uprev, s, c->Ucur, c->Uy, c->bdsum);
  if (e != hipSuccess) return e;
  e = launch_gemm_any(xdt, c->P.X, n, kF64, c->Rd, n, c->CT, p, nr_of(c->rs * m), n, c->KS, c->d_active,
                      two ? c->d_rowmap2 : c->d_rowmap, two ? c->d_split + 8 : c->d_split, c->d_split + 2,
                      c->KS * c->fmaxT, c->d_split + 5, s);
  if (e != hipSuccess) return e;
  return launch_batch_step(c->d_bprm, c->d_bstate, batch_bufs(c, m), p, s);
}

int ensure_batch_graph(pr_ctx *c, int32_t m, int32_t units) {
  // the union sizes are kernel arguments of the captured launches
  const int64_t kp = c->union_on ? c->kp : 0, ku = c->union_on ? c->ku : 0;
  if (c->bgexec && c->bgraph_units == units && c->bgraph_m == m && c->bgraph_kp == kp && c->bgraph_ku == ku)
    return PR_OK;
  if (c->bgexec) {
    (void)hipGraphExecDestroy(c->bgexec);
    c->bgexec = nullptr;
  }
  hipGraph_t g = nullptr;
  PR_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < units && e == hipSuccess; i++) e = enqueue_batch_unit(c, m, c->cap);
  hipError_t e2 = hipStreamEndCapture(c->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return PR_EDEVICE;
  }
  e = hipGraphInstantiate(&c->bgexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->bgexec = nullptr;
    return PR_EDEVICE;
  }
  c->bgraph_units = units;
  c->bgraph_m = m;
  c->bgraph_kp = kp;
  c->bgraph_ku = ku;
  return PR_OK;
}

// Support union of the batch's current iterates (rows 0..m-1 of Bx) for the
// product with the iterates (G X_it in Gram mode, else the forward product
// X_it X^T).  fresh: a new union, compaction on when its padded size is at
// most 3/4 of p.  Otherwise the current iterates' supports are joined to
// the union in use, unless the join would not fit (the union in use stays,
// its misses go through the correction kernel).  *changed tells whether the
// lists and G[:, U] were rebuilt.  Runs between graph launches, with nothing
// else in flight.
int build_union(pr_ctx *c, int32_t m, bool fresh, bool *changed) {
  const int64_t n = c->P.n, p = c->P.p;
  const int NrMax = nr_of(c->max_batch);
  // every split count the tuned table may pick must divide kp into whole
  // reduction steps of the tile: 16 indices (FP64 x FP64, Gram mode) with
  // splits KSG * f, f <= fmaxG; 32 (BF16 x FP64) with KSF * f, f <= fmaxF
  const int64_t gran = c->gram ? 16LL * c->KSG * c->fmaxG : 32LL * c->KSF * c->fmaxF;
  const int64_t kpmax = (3 * p / 4) / gran * gran;
  *changed = false;
  if (fresh) c->union_on = false;
  if (kpmax < gran) return PR_OK;
  if (!c->d_umask) {
    bool ok = dalloc(&c->d_umask, p) == hipSuccess && dalloc(&c->d_ulist, p) == hipSuccess;
    ok = ok && dalloc(&c->d_olist, p) == hipSuccess && dalloc(&c->d_ocnt, NrMax) == hipSuccess;
    ok = ok && dalloc(&c->d_oidx, (size_t)NrMax * p) == hipSuccess;
    ok = ok && dalloc(&c->d_oval, (size_t)NrMax * p) == hipSuccess;
    ok = ok && dalloc(&c->BxU, (size_t)NrMax * (3 * p / 4)) == hipSuccess;
    if (!ok) return PR_ENOMEM;
  }
  if (c->gram && !c->GU && dalloc(&c->GU, (size_t)p * (3 * p / 4)) != hipSuccess) return PR_ENOMEM;
  if (!c->gram && !c->XrU && hipMalloc(&c->XrU, esize(c->P.xdt) * (size_t)n * (3 * p / 4)) != hipSuccess)
    return PR_ENOMEM;
  hipStream_t s = c->stream;
  if (fresh) PR_TRY(hipMemsetAsync(c->d_umask, 0, sizeof(int32_t) * p, s));
  PR_TRY(launch_union_mask(c->Bx, m, p, c->d_umask, s));
  std::vector<int32_t> mask((size_t)p);
  PR_TRY(hipMemcpyAsync(mask.data(), c->d_umask, sizeof(int32_t) * p, hipMemcpyDeviceToHost, s));
  PR_TRY(hipStreamSynchronize(s));
  std::vector<int32_t> ul, ol;
  for (int64_t j = 0; j < p; j++) (mask[(size_t)j] ? ul : ol).push_back((int32_t)j);
  const int64_t ku = (int64_t)ul.size();
  const int64_t kp = (ku + gran - 1) / gran * gran;
  if (ku == 0 || kp > kpmax) return PR_OK;
  if (!fresh && ku == c->ku) return PR_OK;
  PR_TRY(hipMemcpyAsync(c->d_ulist, ul.data(), sizeof(int32_t) * ku, hipMemcpyHostToDevice, s));
  if (!ol.empty())
    PR_TRY(hipMemcpyAsync(c->d_olist, ol.data(), sizeof(int32_t) * ol.size(), hipMemcpyHostToDevice, s));
  if (c->gram) PR_TRY(launch_gather_cols(c->G, p, c->d_ulist, ku, kp, c->GU, s));
  else PR_TRY(launch_gather_cols_x(c->P.xdt, c->Xrow, n, p, c->d_ulist, ku, kp, c->XrU, s));
  if (fresh) PR_TRY(hipMemsetAsync(c->d_ocnt, 0, sizeof(int32_t) * NrMax, s));
  PR_TRY(hipStreamSynchronize(s));  // the host lists go out of scope
  c->ku = ku;
  c->kp = kp;
  c->union_on = true;
  *changed = true;
  return PR_OK;
}

// FP64 values of the m batched nodes at their stopping iterates (rows of
// bxbest), over the stored X, for every node at once: the forward product
// X_it X^T and the transposed product R X on the batch's FP64-accumulated
// GEMMs (split as the iteration splits them), residual rows and loss sums,
// then one workgroup per node for g_N(x) and g_N*(X^T zeta / (2 lambda2)).
// lb[q] = Psi(zeta_q) with zeta_q = 2 (y - X x_q), ub[q] = Phi(x_q).
int certify_batch(pr_ctx *c, int32_t m, std::vector<double> &lb, std::vector<double> &ub, int32_t *kst_out = nullptr) {
  const int64_t n = c->P.n, p = c->P.p;
  const int NrMax = nr_of(c->max_batch), Nr = nr_of(m), NrT = nr_of(c->rs * m);
  hipStream_t s = c->stream;
  if (!c->cert_a) {
    bool ok = dalloc(&c->cert_a, (size_t)NrMax * p) == hipSuccess && dalloc(&c->d_cert, 2 * (size_t)NrMax) == hipSuccess;
    if (!ok) return PR_ENOMEM;
  }
  int nta = Nr / 64;
  if (nta >= kTuneMax) nta = kTuneMax - 1;
  static_assert(kTuneTables >= 2, "forward and transpose split tables");
  const int32_t ksf = c->KSF * c->h_ftab[nta];
  const int32_t kst = kst_for(c, m);
  PR_TRY(hipMemcpyAsync(c->Bx, c->bxbest, sizeof(double) * m * p, hipMemcpyDeviceToDevice, s));
  PR_TRY(hipMemcpyAsync(c->d_split + 6, &ksf, sizeof(int32_t), hipMemcpyHostToDevice, s));
  PR_TRY(launch_gemm_any(c->P.xdt, c->Xrow, p, kF64, c->Bx, p, c->CF, n, Nr, p, ksf, nullptr, nullptr, nullptr,
                         nullptr, ksf, nullptr, s));
  PR_TRY(launch_batch_resid(c->CF, c->d_split + 6, n, m, Nr, c->P.y, c->Rd, c->fsum, nullptr, c->P.loss, nullptr,
                            s));
  PR_TRY(launch_gemm_any(c->P.xdt, c->P.X, n, kF64, c->Rd, n, c->CT, p, NrT, n, kst, nullptr, nullptr, nullptr,
                         nullptr, kst, nullptr, s));
  PR_TRY(launch_cert_batch(c->d_bprm, c->bxbest, c->CT, kst, NrT, c->rs, c->fsum, c->nfb, p, c->cert_a, c->bsidx,
                           c->bsval, c->d_cert, m, s));
  if (kst_out) *kst_out = kst;
  std::vector<double> h((size_t)2 * m);
  PR_TRY(hipMemcpyAsync(h.data(), c->d_cert, sizeof(double) * 2 * m, hipMemcpyDeviceToHost, s));
  PR_TRY(hipStreamSynchronize(s));
  lb.resize((size_t)m);
  ub.resize((size_t)m);
  for (int32_t q = 0; q < m; q++) {
    lb[(size_t)q] = h[2 * (size_t)q];
    ub[(size_t)q] = h[2 * (size_t)q + 1];
  }
  return PR_OK;
}

}  // namespace

extern "C" {

void pr_opts_default(pr_opts *o) {
  if (!o) return;
  o->rel_gap_tol = 1e-6;
  o->eta = exp(3.0);
  o->cutoff = NAN;
  o->L = 0.0;
  o->max_iter = 100000;
  o->check_every = 32;
  o->method = PR_FISTA_GAP;
  o->pad0 = 0;
  o->trace = nullptr;
  o->acfgm_b = 0.1;
  o->acfgm_c = 2.0;
  o->L0 = 0.0;
}

const char *pr_strerror(int code) {
  switch (code) {
    case PR_OK: return "ok";
    case PR_EINVAL: return "invalid argument";
    case PR_EOVERLAP: return "J0 and J1 overlap";
    case PR_EDEVICE: return "HIP runtime error";
    case PR_ENOMEM: return "out of memory";
    default: return "unknown error";
  }
}

int pr_ctx_create(pr_ctx **out, const pr_problem *prob, int32_t max_batch, void *stream) {
  if (!out || !prob || !prob->X || !prob->y || prob->n < 1 || prob->p < 1 || prob->p >= kJ0Flag || max_batch < 1)
    return PR_EINVAL;
  if (prob->xdtype < PR_F64 || prob->xdtype > PR_BF16) return PR_EINVAL;
  if (prob->loss != PR_LSQ && prob->loss != PR_LOGISTIC) return PR_EINVAL;
  if (prob->p >= (int64_t)1 << 31 || prob->n >= (int64_t)1 << 40) return PR_EINVAL;
  const int vec = vec_of(prob->xdtype);
  if (prob->n % vec != 0) return PR_EINVAL;
  if (((uintptr_t)prob->X) % 16 != 0 || ((uintptr_t)prob->y) % 8 != 0) return PR_EINVAL;
  pr_ctx *c = new (std::nothrow) pr_ctx();
  if (!c) return PR_ENOMEM;
  c->stream = (hipStream_t)stream;
  c->max_batch = max_batch;
  c->P.X = prob->X;
  c->P.xdt = prob->xdtype;
  c->P.loss = prob->loss;
  c->P.y = prob->y;
  c->P.n = prob->n;
  c->P.p = prob->p;
  const int64_t n = prob->n, p = prob->p;
  c->B.rows = kSpThreads * vec;
  c->B.rb = (int32_t)((n + c->B.rows - 1) / c->B.rows);
  // column chunks of the column-list product: 16 at most (fewer planes for
  // the summing kernel; on the 16384 x 8192 root 16 chunks beat 8, 12 and 32
  // per iteration, and the 500 x 200 root ran 8% faster than with 64), but
  // enough for one workgroup per compute unit where the design has few row
  // blocks and the columns to fill them, at least 64 per chunk (BF16
  // 16000 x 16000: 8 row blocks of 2048 rows, 32 chunks instead of 16: the
  // dense product 93 -> 82 us, its root solves 6% faster)
  int nch = 512 / c->B.rb;
  if (nch < 1) nch = 1;
  if (nch > kSpChunksMax) nch = kSpChunksMax;
  int fill = (kCUs + c->B.rb - 1) / c->B.rb;
  if (fill > kSpChunksFill) fill = kSpChunksFill;
  if (fill > nch && (int64_t)fill * 64 <= p) nch = fill;
  if (nch > p) nch = (int)p;
  c->B.nch = nch;
  c->B.nfin = spfwd_final_blocks(n);
  bool ok = hipGetDevice(&c->device) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) == hipSuccess;
  ok = ok && dalloc(&c->d_prm, 1) == hipSuccess && dalloc(&c->d_state, 1) == hipSuccess;
  ok = ok && hipHostMalloc((void **)&c->h_state, 2 * sizeof(NodeState), hipHostMallocDefault) == hipSuccess;
  ok = ok && dalloc(&c->d_status, p) == hipSuccess;
  c->h_stp.assign((size_t)kNodeThreads * (size_t)((p + 16 * kNodeThreads - 1) / (16 * kNodeThreads)), 0u);
  ok = ok && dalloc(&c->d_stp, c->h_stp.size()) == hipSuccess;
  ok = ok && dalloc(&c->nb.x0, p) == hipSuccess && dalloc(&c->nb.x1, p) == hipSuccess;
  ok = ok && dalloc(&c->nb.xbest, p) == hipSuccess && dalloc(&c->nb.xlb, p) == hipSuccess;
  ok = ok && dalloc(&c->nb.hprev, p) == hipSuccess && dalloc(&c->nb.vbuf, p) == hipSuccess;
  ok = ok && dalloc(&c->nb.abuf, p) == hipSuccess && dalloc(&c->nb.sidx, p) == hipSuccess;
  ok = ok && dalloc(&c->nb.sval, p) == hipSuccess;
  ok = ok && dalloc(&c->nb.ybt, p) == hipSuccess && dalloc(&c->nb.gbt, p) == hipSuccess;
  ok = ok && dalloc(&c->B.r, n) == hipSuccess && dalloc(&c->B.gm, n) == hipSuccess;
  ok = ok && dalloc(&c->B.ucur, n) == hipSuccess && dalloc(&c->B.uprev, n) == hipSuccess;
  ok = ok && dalloc(&c->B.zbest, n) == hipSuccess;
  ok = ok && dalloc(&c->B.h1, p) == hipSuccess && dalloc(&c->B.h2, p) == hipSuccess;
  ok = ok && dalloc(&c->B.part, (size_t)nch * n) == hipSuccess;
  ok = ok && dalloc(&c->B.rbsum, 2 * (size_t)c->B.nfin) == hipSuccess;
  ok = ok && dalloc(&c->B.dsum, (size_t)c->B.nfin) == hipSuccess && dalloc(&c->B.uy, n) == hipSuccess;
  ok = ok && dalloc(&c->iota, p) == hipSuccess && dalloc(&c->d_np, 1) == hipSuccess;
  ok = ok && dalloc(&c->d_u, n) == hipSuccess && dalloc(&c->d_v, p) == hipSuccess;
  ok = ok && dalloc(&c->d_w, p) == hipSuccess && dalloc(&c->d_scal, 8) == hipSuccess;
  ok = ok && dalloc(&c->d_lam, 2 * kLanczosMax) == hipSuccess && dalloc(&c->d_vprev, p) == hipSuccess;
  ok = ok && dalloc(&c->d_regscratch, 3 * (size_t)p) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreate(&c->tev[0]) == hipSuccess && hipEventCreate(&c->tev[1]) == hipSuccess;
  if (!ok) {
    free_ctx(c);
    return PR_ENOMEM;
  }
  int32_t pp = (int32_t)p;
  ok = hipMemsetAsync(c->B.ucur, 0, sizeof(double) * n, c->stream) == hipSuccess;
  ok = ok && hipMemsetAsync(c->B.uprev, 0, sizeof(double) * n, c->stream) == hipSuccess;
  ok = ok && hipMemsetAsync(c->B.r, 0, sizeof(double) * n, c->stream) == hipSuccess;
  ok = ok && hipMemsetAsync(c->B.gm, 0, sizeof(double) * n, c->stream) == hipSuccess;
  ok = ok && hipMemsetAsync(c->B.uy, 0, sizeof(double) * n, c->stream) == hipSuccess;
  ok = ok && hipMemcpyAsync(c->d_np, &pp, sizeof(int32_t), hipMemcpyHostToDevice, c->stream) == hipSuccess;
  ok = ok && launch_iota(c->iota, p, c->stream) == hipSuccess;
  ok = ok && hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) {
    free_ctx(c);
    return PR_EDEVICE;
  }
  int rc = lanczos_norm2(c);
  if (rc != PR_OK) {
    free_ctx(c);
    return rc;
  }
  if (max_batch > 1 && n % 128 == 0 && p % 128 == 0 && p <= 16384) {
    rc = alloc_batch(c);
    if (rc != PR_OK) {
      free_ctx(c);
      return rc;
    }
  }
  *out = c;
  return PR_OK;
}

int pr_ctx_destroy(pr_ctx *c) {
  if (!c) return PR_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  free_ctx(c);
  return PR_OK;
}

int pr_ctx_set_debug(pr_ctx *c, int32_t flags) {
  if (!c || (flags & ~(PR_DEBUG_GRAM_RECHECK | PR_DEBUG_FORCE_BATCH))) return PR_EINVAL;
  c->debug = flags;
  return PR_OK;
}

int pr_ctx_norm2(pr_ctx *c, double *out) {
  if (!c || !out) return PR_EINVAL;
  *out = c->norm2;
  return PR_OK;
}

int pr_solve(pr_ctx *c, const pr_node *node, const pr_opts *opts_in, const double *beta0, double *beta_out,
             double *zeta_out, pr_result *out);

// End of a Gram-mode solve: the bounds the iteration computed from G are
// recomputed over the stored X (pr_dual_bound): Psi at the dual vectors of the
// iterate with the best Psi and of the iterate with the best Phi, and Phi at
// the latter.  A decision (converged / prune / branch) these values do not
// confirm is redone on the matrix-vector path from the best iterate.
static int gram_certify(pr_ctx *c, const pr_node *node, const pr_opts *opts, const NodeState &hs, double *beta_out,
                        double *zeta_out, pr_result *out) {
  const int64_t n = c->P.n, p = c->P.p;
  hipStream_t s = c->stream;
  double lb1 = -INFINITY, ub1 = INFINITY, lb2 = -INFINITY, ub2 = INFINITY;
  int rc = pr_dual_bound(c, node, nullptr, c->nb.xlb, &lb1, &ub1);  // leaves zeta(x_lb) in B.gm
  if (rc != PR_OK) return rc;
  if (zeta_out) PR_TRY(hipMemcpyAsync(zeta_out, c->B.gm, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  rc = pr_dual_bound(c, node, nullptr, c->nb.xbest, &lb2, &ub2);
  if (rc != PR_OK) return rc;
  if (zeta_out && lb2 > lb1) PR_TRY(hipMemcpyAsync(zeta_out, c->B.gm, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  const double lb = lb2 > lb1 ? lb2 : lb1, ub = ub2;
  const double rel = (ub - lb) / fmax(fabs(ub), 1e-300);
  const int st = hs.done ? hs.status : kMaxIter;
  bool confirmed = true;
  if (st == kConverged) confirmed = rel <= opts->rel_gap_tol;
  else if (st == kCutoffPrune) confirmed = lb >= opts->cutoff;
  else if (st == kCutoffBranch) confirmed = ub <= opts->cutoff;
  if (c->debug & PR_DEBUG_GRAM_RECHECK) confirmed = false;
  if (!confirmed) {
    // rare: redo on the matrix-vector path (its own iteration graph, see
    // ensure_graph), warm-started from the best iterate.  Its bounds are the
    // FP64 values over the stored X of that run, returned with its own zeta.
    PR_TRY(hipMemcpyAsync(c->nb.vbuf, c->nb.xbest, sizeof(double) * p, hipMemcpyDeviceToDevice, s));
    c->gram = false;
    pr_opts o2 = *opts;
    rc = pr_solve(c, node, &o2, c->nb.vbuf, beta_out, zeta_out, out);
    c->gram = true;
    if (rc == PR_OK) {
      out->iters += hs.iter;
      out->restarts += hs.restarts;
      out->trials += hs.trials;
    }
    return rc;
  }
  if (beta_out) PR_TRY(hipMemcpyAsync(beta_out, c->nb.xbest, sizeof(double) * p, hipMemcpyDeviceToDevice, s));
  PR_TRY(hipStreamSynchronize(s));
  out->lower_bound = lb;
  out->primal = ub;
  out->rel_gap = rel;
  out->L = hs.L;
  out->iters = hs.iter;
  out->restarts = hs.restarts;
  out->trials = hs.trials;
  out->status = st;
  return PR_OK;
}

// AC-FGM on the node whose parameters are already on the device (pr_solve).
static int solve_acfgm(pr_ctx *c, const pr_opts *opts, double L, const double *beta0, double *beta_out,
                       double *zeta_out, pr_result *out) {
  const int64_t n = c->P.n, p = c->P.p;
  int rc = ensure_variant_bufs(c);
  if (rc != PR_OK) return rc;
  const double L0 = opts->L0 > 0.0 ? opts->L0 : L / 64.0;
  PR_TRY(launch_ac_init(c->d_prm, c->d_state, c->d_ac, c->ab, c->nb, beta0, L0, c->stream));
  const double key[3] = {opts->acfgm_b, opts->acfgm_c, opts->method == kAcfgmGap ? 1.0 : 0.0};
  rc = ensure_variant_graph(c, 0, key, opts->check_every);
  if (rc != PR_OK) return rc;
  PR_TRY(run_graph(c, c->vgexec, c->vgraph_units,
                   ((int64_t)opts->max_iter / opts->check_every + 3) * c->vgraph_units, opts->rel_gap_tol));
  PR_TRY(launch_zbest_final(c->d_state, c->B, c->P.loss, n, c->stream));
  NodeState hs;
  AcState ha;
  PR_TRY(hipMemcpyAsync(&hs, c->d_state, sizeof(hs), hipMemcpyDeviceToHost, c->stream));
  PR_TRY(hipMemcpyAsync(&ha, c->d_ac, sizeof(ha), hipMemcpyDeviceToHost, c->stream));
  if (beta_out)
    PR_TRY(hipMemcpyAsync(beta_out, c->nb.xbest, sizeof(double) * p, hipMemcpyDeviceToDevice, c->stream));
  if (zeta_out)
    PR_TRY(hipMemcpyAsync(zeta_out, c->B.zbest, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  PR_TRY(hipStreamSynchronize(c->stream));
  out->lower_bound = hs.lb;
  out->primal = hs.ub;
  out->rel_gap = hs.rel_gap;
  out->L = ha.L1;
  out->iters = hs.iter;
  out->restarts = hs.restarts;
  out->status = hs.done ? hs.status : PR_MAXITER;
  out->trials = ha.rejected;
  return PR_OK;
}

int pr_lasso_solve(pr_ctx *c, const pr_lasso *lp, const pr_opts *opts_in, const double *beta0, double *beta_out,
                   double *zeta_out, pr_result *out) {
  if (!c || !lp || !out) return PR_EINVAL;
  pr_opts opts;
  pr_opts_default(&opts);
  if (opts_in) opts = *opts_in;
  if (check_opts(&opts) != PR_OK) return PR_EINVAL;
  if (c->P.loss != kLsq || (lp->kind != PR_L1_REG && lp->kind != PR_L1_BALL) || !(lp->lam > 0.0) ||
      !isfinite(lp->lam) || (opts.method != kFistaGap && opts.method != kFista))
    return PR_EINVAL;
  const int64_t n = c->P.n, p = c->P.p;
  int rc = ensure_variant_bufs(c);
  if (rc != PR_OK) return rc;
  memset(out, 0, sizeof(*out));
  const double L = opts.L > 0.0 ? opts.L : 1.01 * curvature(kLsq) * c->norm2;
  NodeParams prm{};
  prm.st = c->d_status;
  prm.p = p;
  prm.loss = kLsq;
  prm.eta = opts.eta;
  prm.tol = opts.rel_gap_tol;
  prm.cutoff = NAN;
  prm.max_iter = opts.max_iter;
  prm.method = opts.method;
  prm.trace = opts.trace;
  PR_TRY(hipMemcpyAsync(c->d_prm, &prm, sizeof(prm), hipMemcpyHostToDevice, c->stream));
  PR_TRY(launch_lasso_init(c->d_state, c->d_lx, c->nb, beta0, p, lp->kind, lp->lam, L, c->stream));
  const double key[3] = {lp->lam, 0.0, 0.0};
  rc = ensure_variant_graph(c, 1 + lp->kind, key, opts.check_every);
  if (rc != PR_OK) return rc;
  PR_TRY(run_graph(c, c->vgexec, c->vgraph_units,
                   ((int64_t)opts.max_iter / opts.check_every + 3) * c->vgraph_units, opts.rel_gap_tol));
  PR_TRY(launch_zbest_final(c->d_state, c->B, kLsq, n, c->stream));
  NodeState hs;
  LassoState hl;
  PR_TRY(hipMemcpyAsync(&hs, c->d_state, sizeof(hs), hipMemcpyDeviceToHost, c->stream));
  PR_TRY(hipMemcpyAsync(&hl, c->d_lx, sizeof(hl), hipMemcpyDeviceToHost, c->stream));
  PR_TRY(hipStreamSynchronize(c->stream));
  if (beta_out)
    PR_TRY(hipMemcpyAsync(beta_out, c->nb.xbest, sizeof(double) * p, hipMemcpyDeviceToDevice, c->stream));
  if (zeta_out) PR_TRY(launch_scale_copy(c->B.zbest, zeta_out, hl.zscale_best, n, c->stream));
  PR_TRY(hipStreamSynchronize(c->stream));
  out->lower_bound = hs.lb;
  out->primal = hs.ub;
  out->rel_gap = hs.rel_gap;
  out->L = L;
  out->iters = hs.iter;
  out->restarts = hs.restarts;
  out->status = hs.done ? hs.status : PR_MAXITER;
  return PR_OK;
}

int pr_ctx_enable_gram(pr_ctx *c) {
  if (!c) return PR_EINVAL;
  const int64_t n = c->P.n, p = c->P.p;
  if (c->P.loss != kLsq || p % 128 != 0 || n % 32 != 0 || p > 16384) return PR_EINVAL;
  if (c->gram) return PR_OK;
  hipStream_t s = c->stream;
  bool ok = dalloc(&c->G, (size_t)p * p) == hipSuccess && dalloc(&c->gb, (size_t)p) == hipSuccess;
  c->PG.X = c->G;
  c->PG.xdt = kF64;
  c->PG.loss = kLsq;
  c->PG.y = c->gb;
  c->PG.n = p;
  c->PG.p = p;
  c->BG = c->B;
  c->BG.rows = kSpThreads * 2;  // FP64 "design": 2 rows per 16-byte load
  c->BG.rb = (int32_t)((p + c->BG.rows - 1) / c->BG.rows);
  int nch = 512 / c->BG.rb;
  if (nch < 1) nch = 1;
  if (nch > kSpChunksMax) nch = kSpChunksMax;
  c->BG.nch = nch;
  c->BG.nfin = spfwd_final_blocks(p);
  c->BG.part = nullptr;
  ok = ok && dalloc(&c->BG.part, (size_t)nch * p) == hipSuccess;
  if (!ok) return PR_ENOMEM;
  // G = X^T X on FP64 MFMA (operands converted exactly, FP64 sums); b = X^T y
  PR_TRY(launch_gemm_any(c->P.xdt, c->P.X, n, c->P.xdt, c->P.X, n, c->G, p, p, n, 1, nullptr, nullptr, nullptr,
                         nullptr, 0, nullptr, s));
  PR_TRY(launch_gemv_t(c->P, c->P.y, nullptr, c->gb, nullptr, nullptr, s));
  std::vector<double> yh((size_t)n);
  PR_TRY(hipMemcpyAsync(yh.data(), c->P.y, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  PR_TRY(hipStreamSynchronize(s));
  double yy = 0.0;
  for (double v : yh) yy += v * v;
  c->gyy = yy;
  if (c->batch_ok) {
    const int rc = tune_gram_batch(c);
    if (rc != PR_OK) return rc;
  }
  c->gram = true;
  for (hipGraphExec_t *ge : {&c->gexec, &c->gtail})  // the captured iterations change
    if (*ge) {
      (void)hipGraphExecDestroy(*ge);
      *ge = nullptr;
    }
  c->graph_units = 0;
  if (c->bgexec) {
    (void)hipGraphExecDestroy(c->bgexec);
    c->bgexec = nullptr;
    c->bgraph_units = 0;
  }
  return PR_OK;
}

int pr_solve(pr_ctx *c, const pr_node *node, const pr_opts *opts_in, const double *beta0,
             double *beta_out, double *zeta_out, pr_result *out) {
  if (!c || !out) return PR_EINVAL;
  pr_opts opts;
  pr_opts_default(&opts);
  if (opts_in) opts = *opts_in;
  if (check_opts(&opts) != PR_OK) return PR_EINVAL;
  const int64_t n = c->P.n, p = c->P.p;
  std::vector<int8_t> st;
  int64_t n1, pbar;
  int32_t kbar;
  bool infeasible;
  int rc = build_status(node, p, st, n1, pbar, kbar, infeasible);
  if (rc != PR_OK) return rc;
  memset(out, 0, sizeof(*out));
  if (infeasible) {
    out->lower_bound = INFINITY;
    out->primal = INFINITY;
    out->rel_gap = NAN;
    out->status = PR_INFEASIBLE;
    if (beta_out) PR_TRY(hipMemsetAsync(beta_out, 0, sizeof(double) * p, c->stream));
    PR_TRY(hipStreamSynchronize(c->stream));
    return PR_OK;
  }
  const double L = opts.L > 0.0 ? opts.L : 1.01 * curvature(c->P.loss) * c->norm2;
  NodeParams prm{};
  prm.st = c->d_status;
  prm.p = p;
  prm.pbar = pbar;
  prm.kbar = kbar;
  prm.loss = c->P.loss;
  prm.lambda2 = node->lambda2;
  prm.M = node->M;
  prm.eta = opts.eta;
  prm.tol = opts.rel_gap_tol;
  prm.cutoff = opts.cutoff;
  prm.max_iter = opts.max_iter;
  prm.method = opts.method;
  prm.trace = opts.trace;
  prm.gram_b = c->gram ? c->gb : nullptr;
  prm.gram_yy = c->gyy;
  prm.stp = c->d_stp;
  double L_init = L;
  if (is_bt(opts.method)) {
    // backtracking from L0 (default L / 16), capped at L; register-resident steps only
    if (node_ept(p) == 0) return PR_EINVAL;
    prm.Lmax = L;
    prm.L0 = opts.L0 > 0.0 ? fmin(opts.L0, L) : L / 16.0;
    prm.ls_c = opts.acfgm_c;
    L_init = prm.L0;
  }
  pack_status(st, c->h_stp);
  PR_TRY(hipMemcpyAsync(c->d_status, st.data(), (size_t)p, hipMemcpyHostToDevice, c->stream));
  PR_TRY(hipMemcpyAsync(c->d_stp, c->h_stp.data(), sizeof(uint32_t) * c->h_stp.size(), hipMemcpyHostToDevice,
                        c->stream));
  PR_TRY(hipMemcpyAsync(c->d_prm, &prm, sizeof(prm), hipMemcpyHostToDevice, c->stream));
  if (opts.method == kAcfgmGap || opts.method == kAcfgm)
    return solve_acfgm(c, &opts, L, beta0, beta_out, zeta_out, out);
  PR_TRY(launch_node_init(c->d_prm, c->d_state, c->nb, beta0, L_init, p, c->stream));
  c->step_bt = is_bt(opts.method);
  rc = ensure_graph(c, opts.check_every);
  if (rc != PR_OK) return rc;
  // backtracking: rejected trials take evaluations beyond the iteration budget
  const int64_t launches = (int64_t)opts.max_iter / opts.check_every + 3;
  PR_TRY(run_graph(c, c->gexec, c->graph_units, (is_bt(opts.method) ? 2 * launches : launches) * c->graph_units,
                   opts.rel_gap_tol, c->gtail, kTailUnits));
  NodeState hs;
  if (c->gram) {
    PR_TRY(hipMemcpyAsync(&hs, c->d_state, sizeof(hs), hipMemcpyDeviceToHost, c->stream));
    PR_TRY(hipStreamSynchronize(c->stream));
    return gram_certify(c, node, &opts, hs, beta_out, zeta_out, out);
  }
  PR_TRY(launch_zbest_final(c->d_state, c->B, c->P.loss, n, c->stream));
  PR_TRY(hipMemcpyAsync(&hs, c->d_state, sizeof(hs), hipMemcpyDeviceToHost, c->stream));
  PR_TRY(hipStreamSynchronize(c->stream));
  if (beta_out)
    PR_TRY(hipMemcpyAsync(beta_out, c->nb.xbest, sizeof(double) * p, hipMemcpyDeviceToDevice, c->stream));
  if (zeta_out)
    PR_TRY(hipMemcpyAsync(zeta_out, c->B.zbest, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  PR_TRY(hipStreamSynchronize(c->stream));
  out->lower_bound = hs.lb;
  out->primal = hs.ub;
  out->rel_gap = hs.rel_gap;
  out->L = hs.L;
  out->iters = hs.iter;
  out->restarts = hs.restarts;
  out->trials = hs.trials;
  out->status = hs.done ? hs.status : PR_MAXITER;
  return PR_OK;
}

int pr_gemm(void *stream, const uint16_t *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t Mc,
            int64_t Nr, int64_t K, int32_t KS) {
  if (!A || !B || !C || Mc < 128 || Nr < 64 || K < 32 || KS < 1 || Mc % 128 || Nr % 64 ||
      K % (32 * (int64_t)KS) || lda < K || ldb < K || lda % 8 || ldb % 2)
    return PR_EINVAL;
  if (((uintptr_t)A) % 16 || ((uintptr_t)B) % 16 || ((uintptr_t)C) % 8) return PR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  PR_TRY(launch_gemm_f64(A, lda, B, ldb, C, Mc, Nr, K, KS, nullptr, nullptr, nullptr, nullptr, 0, nullptr, s));
  return PR_OK;
}

int pr_prox(void *stream, const double *v, int64_t p, double rho, int32_t k, double M,
            const int8_t *status, double *out) {
  if (!v || !out || !status || p < 1 || p >= ((int64_t)1 << 31) || !(rho > 0.0) || !isfinite(rho) ||
      !(M > 0.0) || k < 1)
    return PR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int8_t> st((size_t)p);
  PR_TRY(hipMemcpyAsync(st.data(), status, (size_t)p, hipMemcpyDeviceToHost, s));
  PR_TRY(hipStreamSynchronize(s));
  int64_t n1 = 0, nf = 0;
  for (int64_t j = 0; j < p; j++) {
    if (st[(size_t)j] == kOne) n1++;
    else if (st[(size_t)j] == kFree) nf++;
    else if (st[(size_t)j] != kZero) return PR_EINVAL;
  }
  if (n1 > k) return PR_EINVAL;
  int64_t kb = (int64_t)k - n1;
  if (kb > nf) kb = nf;
  double *abuf = nullptr;
  if (hipMalloc((void **)&abuf, sizeof(double) * p) != hipSuccess) return PR_ENOMEM;
  hipError_t e = launch_prox(v, out, p, rho, (int32_t)kb, M, status, abuf, nullptr, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(abuf);
  return e == hipSuccess ? PR_OK : PR_EDEVICE;
}

int pr_time_prox(void *stream, const double *v, int64_t p, double rho, int32_t k, double M, const int8_t *status,
                 double *out, int32_t reps, double *ms_prox, double *ms_g) {
  if (!v || !out || !status || p < 1 || p >= ((int64_t)1 << 31) || !(rho > 0.0) || !isfinite(rho) ||
      !(M > 0.0) || k < 1 || reps < 1 || !ms_prox || !ms_g)
    return PR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int8_t> st((size_t)p);
  PR_TRY(hipMemcpyAsync(st.data(), status, (size_t)p, hipMemcpyDeviceToHost, s));
  PR_TRY(hipStreamSynchronize(s));
  int64_t n1 = 0, nf = 0;
  for (int64_t j = 0; j < p; j++) {
    if (st[(size_t)j] == kOne) n1++;
    else if (st[(size_t)j] == kFree) nf++;
    else if (st[(size_t)j] != kZero) return PR_EINVAL;
  }
  if (n1 > k) return PR_EINVAL;
  int64_t kb = (int64_t)k - n1;
  if (kb > nf) kb = nf;
  double *abuf = nullptr, *g2 = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMalloc((void **)&abuf, sizeof(double) * 3 * p) != hipSuccess) return PR_ENOMEM;
  if (hipMalloc((void **)&g2, sizeof(double) * 2) != hipSuccess) {
    (void)hipFree(abuf);
    return PR_ENOMEM;
  }
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms = 0.0f;
  // prox: one untimed launch, then `reps` timed ones
  if (e == hipSuccess) e = launch_prox(v, out, p, rho, (int32_t)kb, M, status, abuf, nullptr, s);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int32_t i = 0; i < reps && e == hipSuccess; i++) e = launch_prox(v, out, p, rho, (int32_t)kb, M, status, abuf, nullptr, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) *ms_prox = (double)ms / reps;
  // g_N at the prox output (a point of dom g_N)
  if (e == hipSuccess) e = launch_regularizer(out, nullptr, p, (int32_t)kb, M, status, abuf, g2, s);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int32_t i = 0; i < reps && e == hipSuccess; i++) e = launch_regularizer(out, nullptr, p, (int32_t)kb, M, status, abuf, g2, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) *ms_g = (double)ms / reps;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(g2);
  (void)hipFree(abuf);
  return e == hipSuccess ? PR_OK : PR_EDEVICE;
}

int pr_regularizer(void *stream, const double *beta, const double *alpha, int64_t p, int32_t k,
                   double M, const int8_t *status, double *g_out, double *gstar_out) {
  if ((!beta && !alpha) || !status || p < 1 || p >= ((int64_t)1 << 31) || !(M > 0.0) || k < 1)
    return PR_EINVAL;
  if ((beta && !g_out) || (alpha && !gstar_out)) return PR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int8_t> st((size_t)p);
  PR_TRY(hipMemcpyAsync(st.data(), status, (size_t)p, hipMemcpyDeviceToHost, s));
  PR_TRY(hipStreamSynchronize(s));
  int64_t n1 = 0, nf = 0;
  for (int64_t j = 0; j < p; j++) {
    if (st[(size_t)j] == kOne) n1++;
    else if (st[(size_t)j] == kFree) nf++;
    else if (st[(size_t)j] != kZero) return PR_EINVAL;
  }
  if (n1 > k) {
    if (g_out) *g_out = INFINITY;
    if (gstar_out) *gstar_out = -INFINITY;
    return PR_OK;
  }
  int64_t kb = (int64_t)k - n1;
  if (kb > nf) kb = nf;
  double *scr = nullptr;
  if (hipMalloc((void **)&scr, sizeof(double) * (3 * p + 2)) != hipSuccess) return PR_ENOMEM;
  double res[2] = {0.0, 0.0};
  hipError_t e = launch_regularizer(beta, alpha, p, (int32_t)kb, M, status, scr, scr + 3 * p, s);
  if (e == hipSuccess) e = hipMemcpyAsync(res, scr + 3 * p, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(scr);
  if (e != hipSuccess) return PR_EDEVICE;
  if (g_out) *g_out = res[0];
  if (gstar_out) *gstar_out = res[1];
  return PR_OK;
}

int pr_gemv(pr_ctx *c, const double *b, double *u) {
  if (!c || !b || !u) return PR_EINVAL;
  if (launch_spfwd(c->P, c->B, c->iota, b, c->d_np, kSpPlain, nullptr, u, c->stream) != hipSuccess)
    return PR_EDEVICE;
  PR_TRY(hipStreamSynchronize(c->stream));
  return PR_OK;
}

int pr_gemv_t(pr_ctx *c, const double *r, double *h) {
  if (!c || !r || !h) return PR_EINVAL;
  PR_TRY(launch_gemv_t(c->P, r, nullptr, h, nullptr, nullptr, c->stream));
  PR_TRY(hipStreamSynchronize(c->stream));
  return PR_OK;
}

int pr_gemv_t2(pr_ctx *c, const double *r1, const double *r2, double *h1, double *h2) {
  if (!c || !r1 || !r2 || !h1 || !h2) return PR_EINVAL;
  PR_TRY(launch_gemv_t(c->P, r1, r2, h1, h2, nullptr, c->stream));
  PR_TRY(hipStreamSynchronize(c->stream));
  return PR_OK;
}

int pr_time_gemv_t(pr_ctx *c, const double *r, double *h, int32_t reps, double *ms_avg) {
  if (!c || !r || !h || reps < 1 || !ms_avg) return PR_EINVAL;
  // logistic solves run the two-right-hand-side form: [X^T r, X^T r2] with r2
  // the context's gradient buffer (here a copy of r) and its output buffer
  const bool two = c->P.loss == kLogistic;
  const double *r2 = two ? c->B.gm : nullptr;
  double *h2 = two ? c->B.h2 : nullptr;
  if (two) PR_TRY(hipMemcpyAsync(c->B.gm, r, sizeof(double) * c->P.n, hipMemcpyDeviceToDevice, c->stream));
  PR_TRY(launch_gemv_t(c->P, r, r2, h, h2, nullptr, c->stream));
  PR_TRY(hipEventRecord(c->tev[0], c->stream));
  for (int i = 0; i < reps; i++) PR_TRY(launch_gemv_t(c->P, r, r2, h, h2, nullptr, c->stream));
  PR_TRY(hipEventRecord(c->tev[1], c->stream));
  PR_TRY(hipEventSynchronize(c->tev[1]));
  float ms = 0.0f;
  PR_TRY(hipEventElapsedTime(&ms, c->tev[0], c->tev[1]));
  *ms_avg = (double)ms / reps;
  return PR_OK;
}

int pr_time_gemv(pr_ctx *c, const double *b, double *u, int32_t reps, double *ms_avg) {
  if (!c || !b || !u || reps < 1 || !ms_avg) return PR_EINVAL;
  auto fwd = [&]() { return launch_spfwd(c->P, c->B, c->iota, b, c->d_np, kSpPlain, nullptr, u, c->stream); };
  PR_TRY(fwd());
  PR_TRY(hipEventRecord(c->tev[0], c->stream));
  for (int i = 0; i < reps; i++) PR_TRY(fwd());
  PR_TRY(hipEventRecord(c->tev[1], c->stream));
  PR_TRY(hipEventSynchronize(c->tev[1]));
  float ms = 0.0f;
  PR_TRY(hipEventElapsedTime(&ms, c->tev[0], c->tev[1]));
  *ms_avg = (double)ms / reps;
  return PR_OK;
}

int pr_time_read(const void *buf, int64_t bytes, int32_t blocks, int32_t unroll, int32_t reps, void *stream,
                 double *ms_avg) {
  if (!buf || ((uintptr_t)buf) % 16 || bytes < 16 || bytes % 16 || blocks < 1 || blocks > (1 << 20) ||
      (unroll != 1 && unroll != 4) || reps < 1 || !ms_avg)
    return PR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int rc = PR_OK;
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) rc = PR_EDEVICE;
  const int64_t n16 = bytes / 16;
  if (rc == PR_OK && launch_read_stream(buf, n16, blocks, unroll, s) != hipSuccess) rc = PR_EDEVICE;
  if (rc == PR_OK && hipEventRecord(ev[0], s) != hipSuccess) rc = PR_EDEVICE;
  for (int i = 0; rc == PR_OK && i < reps; i++)
    if (launch_read_stream(buf, n16, blocks, unroll, s) != hipSuccess) rc = PR_EDEVICE;
  if (rc == PR_OK && hipEventRecord(ev[1], s) != hipSuccess) rc = PR_EDEVICE;
  if (rc == PR_OK && hipEventSynchronize(ev[1]) != hipSuccess) rc = PR_EDEVICE;
  float ms = 0.0f;
  if (rc == PR_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) rc = PR_EDEVICE;
  if (rc == PR_OK) *ms_avg = (double)ms / reps;
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  return rc;
}

int pr_batch_tuning(pr_ctx *c, int32_t len, int32_t *ksf_out, int32_t *kst_out) {
  if (!c || !c->batch_ok || len < 1 || !ksf_out || !kst_out) return PR_EINVAL;
  for (int32_t i = 0; i < len; i++) {
    const int t = i + 1 < kTuneMax ? i + 1 : kTuneMax - 1;
    ksf_out[i] = c->KSF * c->h_ftab[t];
    kst_out[i] = c->KS * c->h_ftab[kTuneMax + t];
  }
  return PR_OK;
}

int pr_batch_union_size(pr_ctx *c, int64_t *ku, int64_t *kp, int64_t *nout) {
  if (!c || !ku || !kp || !nout) return PR_EINVAL;
  *ku = c->union_on ? c->ku : 0;
  *kp = c->union_on ? c->kp : 0;
  *nout = c->union_on ? c->union_nout : 0;
  return PR_OK;
}

int pr_time_gram_gemm(pr_ctx *c, int32_t m, int32_t reps, double *ms) {
  if (!c || !c->gram_batch_ok || m < 1 || m > c->max_batch || reps < 1 || !ms) return PR_EINVAL;
  const int64_t p = c->P.p;
  const int Nr = nr_of(m);
  hipStream_t s = c->stream;
  int nta = (m + 63) / 64;
  if (nta >= kTuneMax) nta = kTuneMax - 1;
  const int ksg = c->KSG * c->h_ftab[2 * kTuneMax + nta];
  int32_t *cnt = c->d_split + 4;
  auto gemm = [&]() {
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    return launch_gemm_any(kF64, c->G, p, kF64, c->Bx, p, c->CG, p, Nr, p, ksg, nullptr, nullptr, nullptr, nullptr, 0,
                           cnt, s);
  };
  PR_TRY(gemm());
  PR_TRY(hipEventRecord(c->tev[0], s));
  for (int i = 0; i < reps; i++) PR_TRY(gemm());
  PR_TRY(hipEventRecord(c->tev[1], s));
  PR_TRY(hipEventSynchronize(c->tev[1]));
  float e = 0.0f;
  PR_TRY(hipEventElapsedTime(&e, c->tev[0], c->tev[1]));
  *ms = (double)e / reps;
  return PR_OK;
}

int pr_time_batch_gemm(pr_ctx *c, int32_t m, int32_t reps, double *ms_fwd, double *ms_t) {
  if (!c || !c->batch_ok || m < 1 || m > c->max_batch || reps < 1 || !ms_fwd || !ms_t) return PR_EINVAL;
  const int64_t n = c->P.n, p = c->P.p;
  const int Nr = nr_of(m);
  hipStream_t s = c->stream;
  // the split the batched iteration uses with all m rows active
  int nta = (m + 63) / 64;
  if (nta >= kTuneMax) nta = kTuneMax - 1;
  const int ksf = c->KSF * c->h_ftab[nta], kst = kst_for(c, m);
  const int NrT = nr_of(c->rs * m);
  int32_t *cnt = c->d_split + 4;
  auto fwd = [&]() {
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    return launch_gemm_any(c->P.xdt, c->Xrow, p, kF64, c->Bx, p, c->CF, n, Nr, p, ksf, nullptr, nullptr, nullptr,
                           nullptr, 0, cnt, s);
  };
  auto trn = [&]() {
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    return launch_gemm_any(c->P.xdt, c->P.X, n, kF64, c->Rd, n, c->CT, p, NrT, n, kst, nullptr, nullptr, nullptr,
                           nullptr, 0, cnt, s);
  };
  double *outs[2] = {ms_fwd, ms_t};
  for (int w = 0; w < 2; w++) {
    PR_TRY(w ? trn() : fwd());
    PR_TRY(hipEventRecord(c->tev[0], s));
    for (int i = 0; i < reps; i++) PR_TRY(w ? trn() : fwd());
    PR_TRY(hipEventRecord(c->tev[1], s));
    PR_TRY(hipEventSynchronize(c->tev[1]));
    float ms = 0.0f;
    PR_TRY(hipEventElapsedTime(&ms, c->tev[0], c->tev[1]));
    *outs[w] = (double)ms / reps;
  }
  return PR_OK;
}

namespace {

int ensure_mlp(pr_ctx *c) {
  if (c->mF) return PR_OK;
  const int64_t p = c->P.p;
  bool ok = dalloc(&c->mF, (size_t)p * 8) == hipSuccess && dalloc(&c->mout, (size_t)p) == hipSuccess;
  ok = ok && dalloc(&c->mnz, (size_t)p) == hipSuccess && dalloc(&c->mfs, 2) == hipSuccess;
  ok = ok && dalloc(&c->mvhat, (size_t)p) == hipSuccess && dalloc(&c->mx, (size_t)p) == hipSuccess;
  return ok ? PR_OK : PR_ENOMEM;
}

FeatScalars feat_scalars(const pr_node *node, const std::vector<int8_t> &st, int32_t kbar) {
  FeatScalars sc;
  sc.lambda2 = node->lambda2;
  sc.k = node->k;
  sc.n0 = sc.n1 = 0;
  for (int8_t v : st) {
    sc.n0 += v == kZero;
    sc.n1 += v == kOne;
  }
  sc.kbar = kbar;
  return sc;
}

// Status of the node in c->d_status and w = X^T zeta, zeta = -grad F(X beta),
// in c->d_w: the inputs of the feature kernel.
int grad_image(pr_ctx *c, const std::vector<int8_t> &st, const double *beta) {
  const int64_t n = c->P.n, p = c->P.p;
  hipStream_t s = c->stream;
  PR_TRY(hipMemcpyAsync(c->d_status, st.data(), (size_t)p, hipMemcpyHostToDevice, s));
  if (launch_spfwd(c->P, c->B, c->iota, beta, c->d_np, kSpPlain, nullptr, c->d_u, s) != hipSuccess)
    return PR_EDEVICE;
  PR_TRY(launch_loss_terms(c->P.loss, c->d_u, c->P.y, n, c->B.gm, c->d_scal, s));
  PR_TRY(launch_gemv_t(c->P, c->B.gm, nullptr, c->d_w, nullptr, nullptr, s));
  return PR_OK;
}

}  // namespace

int pr_mlp_features(pr_ctx *c, const pr_node *nodes, int32_t m, const double *Bparent, const double *Bchild,
                    uint16_t *F, float *T) {
  if (!c || !nodes || m < 0 || !Bparent || !F || (Bchild && !T) || ((uintptr_t)F) % 16) return PR_EINVAL;
  const int64_t p = c->P.p;
  std::vector<std::vector<int8_t>> sts((size_t)m);
  std::vector<int32_t> kbars((size_t)m);
  for (int32_t i = 0; i < m; i++) {
    int64_t n1, pbar;
    bool inf;
    int rc = build_status(&nodes[i], p, sts[(size_t)i], n1, pbar, kbars[(size_t)i], inf);
    if (rc != PR_OK) return rc;
    if (inf) kbars[(size_t)i] = 0;
  }
  int rc = ensure_mlp(c);
  if (rc != PR_OK) return rc;
  hipStream_t s = c->stream;
  for (int32_t i = 0; i < m; i++) {
    const double *bp = Bparent + (int64_t)i * p;
    rc = grad_image(c, sts[(size_t)i], bp);
    if (rc != PR_OK) return rc;
    PR_TRY(launch_features(bp, c->d_w, c->d_status, p, c->mnz, c->mfs,
                           feat_scalars(&nodes[i], sts[(size_t)i], kbars[(size_t)i]),
                           Bchild ? Bchild + (int64_t)i * p : nullptr, F + (int64_t)i * p * 8,
                           T ? T + (int64_t)i * p : nullptr, s));
  }
  PR_TRY(hipStreamSynchronize(s));
  return PR_OK;
}

int64_t pr_mlp_workspace(int64_t rows) {
  if (rows < 1) return 0;
  int cpb;
  return (int64_t)mlp_grid(rows, &cpb) * kMlpPartStride;
}

int pr_mlp_forward(void *stream, const float *params, const uint16_t *F, int64_t rows, float *out) {
  if (!params || !F || !out || rows < 0 || ((uintptr_t)F) % 16) return PR_EINVAL;
  if (rows == 0) return PR_OK;
  PR_TRY(launch_mlp_forward(params, F, rows, out, (hipStream_t)stream));
  return PR_OK;
}

int pr_mlp_grad(void *stream, const float *params, const uint16_t *F, const float *T, int64_t rows, float *work,
                float *grad) {
  if (!params || !F || !T || !work || !grad || rows < 1 || ((uintptr_t)F) % 16) return PR_EINVAL;
  PR_TRY(launch_mlp_grad(params, F, T, rows, work, grad, (hipStream_t)stream));
  return PR_OK;
}

int pr_mlp_adam(void *stream, float *params, const float *grad, float *m1, float *m2, int32_t step, double lr,
                double beta1, double beta2, double eps) {
  if (!params || !grad || !m1 || !m2 || step < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
      !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return PR_EINVAL;
  const double c1 = 1.0 / (1.0 - pow(beta1, step)), c2 = 1.0 / (1.0 - pow(beta2, step));
  PR_TRY(launch_mlp_adam(params, grad, m1, m2, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1,
                         (float)c2, (hipStream_t)stream));
  return PR_OK;
}

static int stage_batch_nodes(pr_ctx *c, const pr_node *nodes, const std::vector<int32_t> &slot_of,
                             const std::vector<std::vector<int8_t>> &sts, const std::vector<int32_t> &kbars,
                             const std::vector<int64_t> &pbars, const pr_opts &opts, const double *B0,
                             double Lcap = 0.0);

// Batched starting points (batched path, m <= max_batch):
// the parents' certificates and w = X^T zeta at every parent from one pass of
// the batch's two GEMMs; the proximal steps of all children in one launch
// and their certificates from a second pass; with a network, the feature rows
// and outputs of all children in one launch each, the proximal steps of the
// proposals in one launch and their certificates from a third pass.
static int warm_start_batched(pr_ctx *c, const pr_node *nodes, int32_t m, const float *params, const double *Bparent,
                              double *B0, const std::vector<std::vector<int8_t>> &sts,
                              const std::vector<int32_t> &kbars, const std::vector<int64_t> &pbars,
                              const std::vector<char> &infeas, int32_t *choice, double *gaps) {
  const int64_t p = c->P.p;
  hipStream_t s = c->stream;
  std::vector<int32_t> slot_of;
  for (int32_t i = 0; i < m; i++)
    if (!infeas[(size_t)i]) slot_of.push_back(i);
  const int32_t mb = (int32_t)slot_of.size();
  for (int32_t i = 0; i < m; i++) {
    if (!infeas[(size_t)i]) continue;
    PR_TRY(hipMemcpyAsync(B0 + (int64_t)i * p, Bparent + (int64_t)i * p, sizeof(double) * p, hipMemcpyDeviceToDevice,
                          s));
    if (choice) choice[i] = 0;
    if (gaps) gaps[3 * i] = gaps[3 * i + 1] = gaps[3 * i + 2] = INFINITY;
  }
  if (mb == 0) {
    PR_TRY(hipStreamSynchronize(s));
    return PR_OK;
  }
  const int NrMax = nr_of(c->max_batch);
  if (!c->mVb) {
    bool ok = dalloc(&c->mVb, (size_t)NrMax * p) == hipSuccess && dalloc(&c->mWb, (size_t)NrMax * p) == hipSuccess;
    ok = ok && dalloc(&c->mFb, (size_t)NrMax * p * 8) == hipSuccess && dalloc(&c->moutb, (size_t)NrMax * p) == hipSuccess;
    ok = ok && dalloc(&c->mPb, (size_t)NrMax * p) == hipSuccess;
    if (!ok) return PR_ENOMEM;
  }
  pr_opts o;
  pr_opts_default(&o);
  int rc = stage_batch_nodes(c, nodes, slot_of, sts, kbars, pbars, o, Bparent);  // parents -> bxbest
  if (rc != PR_OK) return rc;
  std::vector<double> lbP, ubP, lbA, ubA, lbN, ubN;
  int32_t kst = 1;
  rc = certify_batch(c, mb, lbP, ubP, &kst);  // leaves X^T zeta (or X^T r) of every parent in CT's split planes
  if (rc != PR_OK) return rc;
  const double L = 1.01 * curvature(c->P.loss) * c->norm2;
  PR_TRY(hipMemcpyAsync(c->mVb, c->bxbest, sizeof(double) * mb * p, hipMemcpyDeviceToDevice, s));  // parents
  // w = X^T zeta at every parent (least squares: the planes hold X^T r, zeta = 2 r)
  if (params)
    PR_TRY(launch_sum_planes(c->CT, kst, nr_of(c->rs * mb), c->rs, p, mb, c->P.loss == kLsq ? 2.0 : 1.0, c->mWb, s));
  // prox(beta_parent) of every child, then its certificate
  PR_TRY(launch_prox_batch(c->d_bprm, c->mVb, c->bxbest, c->cert_a, p, mb, 1.0 / L, s));
  rc = certify_batch(c, mb, lbA, ubA);
  if (rc != PR_OK) return rc;
  PR_TRY(hipMemcpyAsync(c->mPb, c->bxbest, sizeof(double) * mb * p, hipMemcpyDeviceToDevice, s));
  if (params) {
    for (int32_t q = 0; q < mb; q++) {
      const int32_t i = slot_of[(size_t)q];
      PR_TRY(launch_features(c->mVb + (int64_t)q * p, c->mWb + (int64_t)q * p, c->bstatus + (int64_t)q * p, p,
                             c->mnz, c->mfs, feat_scalars(&nodes[i], sts[(size_t)i], kbars[(size_t)i]), nullptr,
                             c->mFb + (int64_t)q * p * 8, nullptr, s));
    }
    PR_TRY(launch_mlp_forward(params, c->mFb, (int64_t)mb * p, c->moutb, s));
    PR_TRY(launch_mlp_propose(c->mVb, c->moutb, (int64_t)mb * p, c->mVb, s));
    PR_TRY(launch_prox_batch(c->d_bprm, c->mVb, c->bxbest, c->cert_a, p, mb, 1.0 / L, s));
    rc = certify_batch(c, mb, lbN, ubN);
    if (rc != PR_OK) return rc;
  }
  for (int32_t q = 0; q < mb; q++) {
    const int32_t i = slot_of[(size_t)q];
    const double gp = ubP[(size_t)q] - lbP[(size_t)q], ga = ubA[(size_t)q] - lbA[(size_t)q];
    const double gn = params ? ubN[(size_t)q] - lbN[(size_t)q] : INFINITY;
    int use = 0;
    double best = gp;
    if (ga < best) {
      use = 1;
      best = ga;
    }
    if (gn < best) use = 2;
    const double *src = use == 0 ? Bparent + (int64_t)i * p
                                 : (use == 1 ? c->mPb + (int64_t)q * p : c->bxbest + (int64_t)q * p);
    PR_TRY(hipMemcpyAsync(B0 + (int64_t)i * p, src, sizeof(double) * p, hipMemcpyDeviceToDevice, s));
    if (choice) choice[i] = use;
    if (gaps) {
      gaps[3 * i] = gp;
      gaps[3 * i + 1] = ga;
      gaps[3 * i + 2] = gn;
    }
  }
  PR_TRY(hipStreamSynchronize(s));
  return PR_OK;
}

int pr_mlp_warm_start(pr_ctx *c, const pr_node *nodes, int32_t m, const float *params, const double *Bparent,
                      double *B0, int32_t *choice, double *gaps) {
  if (!c || !nodes || m < 0 || !Bparent || !B0) return PR_EINVAL;
  const int64_t p = c->P.p;
  std::vector<std::vector<int8_t>> sts((size_t)m);
  std::vector<int32_t> kbars((size_t)m);
  std::vector<int64_t> pbars((size_t)m);
  std::vector<char> infeas((size_t)m);
  for (int32_t i = 0; i < m; i++) {
    int64_t n1;
    bool inf;
    int rc = build_status(&nodes[i], p, sts[(size_t)i], n1, pbars[(size_t)i], kbars[(size_t)i], inf);
    if (rc != PR_OK) return rc;
    infeas[(size_t)i] = inf;
  }
  int rc = ensure_mlp(c);
  if (rc != PR_OK) return rc;
  if (m == 0) return PR_OK;
  if (c->batch_ok && m <= c->max_batch)
    return warm_start_batched(c, nodes, m, params, Bparent, B0, sts, kbars, pbars, infeas, choice, gaps);
  hipStream_t s = c->stream;
  const double L = 1.01 * curvature(c->P.loss) * c->norm2;
  for (int32_t i = 0; i < m; i++) {
    const double *bp = Bparent + (int64_t)i * p;
    double *x0 = B0 + (int64_t)i * p;
    double gp = INFINITY, ga = INFINITY, gn = INFINITY;
    int use = 0;
    if (!infeas[(size_t)i]) {
      double lb, ub;
      rc = pr_dual_bound(c, &nodes[i], nullptr, bp, &lb, &ub);  // leaves d_status and d_w = X^T zeta(beta)
      if (rc != PR_OK) return rc;
      gp = ub - lb;
      const double rho = 2.0 * nodes[i].lambda2 / L;
      if (params) {  // the network's proposal first: d_w still holds X^T zeta at the parent
        PR_TRY(launch_features(bp, c->d_w, c->d_status, p, c->mnz, c->mfs,
                               feat_scalars(&nodes[i], sts[(size_t)i], kbars[(size_t)i]), nullptr, c->mF, nullptr,
                               s));
        PR_TRY(launch_mlp_forward(params, c->mF, p, c->mout, s));
        PR_TRY(launch_mlp_propose(bp, c->mout, p, c->mvhat, s));
        PR_TRY(launch_prox(c->mvhat, c->mvhat, p, rho, kbars[(size_t)i], nodes[i].M, c->d_status, c->d_regscratch,
                           nullptr, s));
        rc = pr_dual_bound(c, &nodes[i], nullptr, c->mvhat, &lb, &ub);
        if (rc != PR_OK) return rc;
        gn = ub - lb;
      }
      PR_TRY(launch_prox(bp, c->mx, p, rho, kbars[(size_t)i], nodes[i].M, c->d_status, c->d_regscratch, nullptr,
                         s));
      rc = pr_dual_bound(c, &nodes[i], nullptr, c->mx, &lb, &ub);
      if (rc != PR_OK) return rc;
      ga = ub - lb;
      double best = gp;
      if (ga < best) {
        use = 1;
        best = ga;
      }
      if (gn < best) use = 2;
    }
    const double *src = use == 0 ? bp : (use == 1 ? c->mx : c->mvhat);
    PR_TRY(hipMemcpyAsync(x0, src, sizeof(double) * p, hipMemcpyDeviceToDevice, s));
    if (choice) choice[i] = use;
    if (gaps) {
      gaps[3 * i] = gp;
      gaps[3 * i + 1] = ga;
      gaps[3 * i + 2] = gn;
    }
  }
  PR_TRY(hipStreamSynchronize(s));
  return PR_OK;
}

int pr_dual_bound(pr_ctx *c, const pr_node *node, const double *zeta, const double *beta,
                  double *lb_out, double *primal_out) {
  if (!c || !lb_out || (!zeta && !beta)) return PR_EINVAL;
  const int64_t n = c->P.n, p = c->P.p;
  std::vector<int8_t> st;
  int64_t n1, pbar;
  int32_t kbar;
  bool infeasible;
  int rc = build_status(node, p, st, n1, pbar, kbar, infeasible);
  if (rc != PR_OK) return rc;
  if (infeasible) {
    *lb_out = INFINITY;
    if (primal_out) *primal_out = INFINITY;
    return PR_OK;
  }
  hipStream_t s = c->stream;
  PR_TRY(hipMemcpyAsync(c->d_status, st.data(), (size_t)p, hipMemcpyHostToDevice, s));
  const double lam2 = node->lambda2;
  double *scal = c->d_scal;  // [0] F(X beta), [1] -F*(-zeta), [2] g(beta), [3] g*(w)
  const double *z = zeta;
  if (beta) {
    if (launch_spfwd(c->P, c->B, c->iota, beta, c->d_np, kSpPlain, nullptr, c->d_u, s) != hipSuccess)
      return PR_EDEVICE;
    // zeta induced from beta goes to B.zbest's twin: reuse B.gm as scratch
    PR_TRY(launch_loss_terms(c->P.loss, c->d_u, c->P.y, n, c->B.gm, scal, s));
    if (!zeta) z = c->B.gm;
    PR_TRY(launch_regularizer(beta, nullptr, p, kbar, node->M, c->d_status, c->d_regscratch, scal + 2, s));
  }
  if (zeta) PR_TRY(launch_zeta_terms(c->P.loss, zeta, c->P.y, n, scal, s));
  PR_TRY(launch_gemv_t(c->P, z, nullptr, c->d_w, nullptr, nullptr, s));
  PR_TRY(launch_scale_copy(c->d_w, c->d_v, 0.5 / lam2, p, s));
  PR_TRY(launch_regularizer(nullptr, c->d_v, p, kbar, node->M, c->d_status, c->d_regscratch, scal + 2, s));
  double hs[4];
  PR_TRY(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, s));
  PR_TRY(hipStreamSynchronize(s));
  *lb_out = hs[1] - 2.0 * lam2 * hs[3];
  if (primal_out) *primal_out = beta ? hs[0] + 2.0 * lam2 * hs[2] : NAN;
  return PR_OK;
}

// Node parameters, status vectors (plain and packed) of the batch slots
// q -> node slot_of[q] on the device; with B0 each slot's starting row is
// copied into the batch's best-iterate rows.  Lcap: the fixed-step constant,
// the cap of the backtracking line search.
static int stage_batch_nodes(pr_ctx *c, const pr_node *nodes, const std::vector<int32_t> &slot_of,
                             const std::vector<std::vector<int8_t>> &sts, const std::vector<int32_t> &kbars,
                             const std::vector<int64_t> &pbars, const pr_opts &opts, const double *B0,
                             double Lcap) {
  const int64_t p = c->P.p;
  const int32_t mb = (int32_t)slot_of.size();
  hipStream_t s = c->stream;
  std::vector<NodeParams> prm((size_t)mb);
  for (int32_t q = 0; q < mb; q++) {
    const int32_t i = slot_of[(size_t)q];
    NodeParams &pp = prm[(size_t)q];
    pp.st = c->bstatus + (int64_t)q * p;
    pp.p = p;
    pp.pbar = pbars[(size_t)i];
    pp.kbar = kbars[(size_t)i];
    pp.loss = c->P.loss;
    pp.lambda2 = nodes[i].lambda2;
    pp.M = nodes[i].M;
    pp.eta = opts.eta;
    pp.tol = opts.rel_gap_tol;
    pp.cutoff = opts.cutoff;
    pp.max_iter = opts.max_iter;
    pp.method = opts.method;
    pp.trace = nullptr;
    pp.gram_b = c->gram ? c->gb : nullptr;
    pp.gram_yy = c->gyy;
    if (is_bt(opts.method)) {
      pp.Lmax = Lcap;
      pp.L0 = opts.L0 > 0.0 ? fmin(opts.L0, Lcap) : Lcap / 16.0;
      pp.ls_c = opts.acfgm_c;
    }
    PR_TRY(hipMemcpyAsync(c->bstatus + (int64_t)q * p, sts[(size_t)i].data(), (size_t)p, hipMemcpyHostToDevice, s));
    if (B0) PR_TRY(hipMemcpyAsync(c->bxbest + (int64_t)q * p, B0 + (int64_t)i * p, sizeof(double) * p,
                                  hipMemcpyDeviceToDevice, s));
  }
  {
    const size_t W = c->h_stp.size();
    c->h_bstp.assign((size_t)mb * W, 0u);
    std::vector<uint32_t> w(W);
    for (int32_t q = 0; q < mb; q++) {
      pack_status(sts[(size_t)slot_of[(size_t)q]], w);
      std::copy(w.begin(), w.end(), c->h_bstp.begin() + (size_t)q * W);
    }
    PR_TRY(hipMemcpyAsync(c->bstp, c->h_bstp.data(), sizeof(uint32_t) * c->h_bstp.size(), hipMemcpyHostToDevice,
                          s));
  }
  PR_TRY(hipMemcpyAsync(c->d_bprm, prm.data(), sizeof(NodeParams) * mb, hipMemcpyHostToDevice, s));
  return PR_OK;
}

int pr_solve_batch(pr_ctx *c, const pr_node *nodes, int32_t m, const pr_opts *opts_in, const double *B0,
                   double *B_out, pr_result *out) {
  if (!c || !nodes || !out || m < 1 || m > c->max_batch) return PR_EINVAL;
  pr_opts opts;
  pr_opts_default(&opts);
  if (opts_in) opts = *opts_in;
  if (check_opts(&opts) != PR_OK) return PR_EINVAL;
  const int64_t n = c->P.n, p = c->P.p;
  // validate every node first: nothing runs if any node is malformed
  std::vector<std::vector<int8_t>> sts((size_t)m);
  std::vector<int32_t> kbars((size_t)m);
  std::vector<int64_t> pbars((size_t)m);
  std::vector<char> infeas((size_t)m);
  for (int32_t i = 0; i < m; i++) {
    int64_t n1;
    bool inf;
    int rc = build_status(&nodes[i], p, sts[(size_t)i], n1, pbars[(size_t)i], kbars[(size_t)i], inf);
    if (rc != PR_OK) return rc;
    infeas[(size_t)i] = inf;
  }
  // AC-FGM, and rounds too small for the batch to pay (batch_pays), run node by node
  if (!c->batch_ok || opts.method == kAcfgmGap || opts.method == kAcfgm ||
      (!(c->debug & PR_DEBUG_FORCE_BATCH) && !batch_pays(c, m))) {
    for (int32_t i = 0; i < m; i++) {
      int rc = pr_solve(c, &nodes[i], &opts, B0 ? B0 + (int64_t)i * p : nullptr,
                        B_out ? B_out + (int64_t)i * p : nullptr, nullptr, &out[i]);
      if (rc != PR_OK) return rc;
    }
    return PR_OK;
  }
  hipStream_t s = c->stream;
  std::vector<int32_t> slot_of;  // batch slot -> node index
  for (int32_t i = 0; i < m; i++) {
    memset(&out[i], 0, sizeof(pr_result));
    if (infeas[(size_t)i]) {
      out[i].lower_bound = INFINITY;
      out[i].primal = INFINITY;
      out[i].rel_gap = NAN;
      out[i].status = PR_INFEASIBLE;
      if (B_out) PR_TRY(hipMemsetAsync(B_out + (int64_t)i * p, 0, sizeof(double) * p, s));
    } else {
      slot_of.push_back(i);
    }
  }
  const int32_t mb = (int32_t)slot_of.size();
  if (mb == 0) {
    PR_TRY(hipStreamSynchronize(s));
    return PR_OK;
  }
  const double L = opts.L > 0.0 ? opts.L : 1.01 * curvature(c->P.loss) * c->norm2;
  int rcs = stage_batch_nodes(c, nodes, slot_of, sts, kbars, pbars, opts, B0, L);
  if (rcs != PR_OK) return rcs;
  for (double *u : {c->Uprev, c->Ucur, c->Uy})
    if (u) PR_TRY(hipMemsetAsync(u, 0, sizeof(double) * mb * n, s));
  int32_t act = mb;
  PR_TRY(hipMemcpyAsync(c->d_active, &act, sizeof(int32_t), hipMemcpyHostToDevice, s));
  BatchBufs bb = batch_bufs(c, mb);
  const bool bt = is_bt(opts.method);
  const double L_init = bt ? (opts.L0 > 0.0 ? fmin(opts.L0, L) : L / 16.0) : L;
  PR_TRY(launch_batch_init(c->d_bprm, c->d_bstate, bb, B0 ? c->bxbest : nullptr, L_init, p, s));
  c->union_on = false;
  int rc = ensure_batch_graph(c, mb, opts.check_every);
  if (rc != PR_OK) return rc;
  auto issue = [&](int slot) -> hipError_t {
    hipError_t e = hipGraphLaunch(c->bgexec, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&c->h_active[slot], c->d_active, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipEventRecord(c->ev[slot], s);
  };
  // backtracking: rejected trials take evaluations beyond the iteration budget
  const int64_t max_launches = ((int64_t)opts.max_iter / opts.check_every + 3) * (bt ? 2 : 1);
  int64_t launched = 0;
  PR_TRY(issue(0));
  launched++;
  if (launched < max_launches) {
    // after the first launch the supports have settled: compact the product
    // with the iterates to their union for the remaining launches
    PR_TRY(hipEventSynchronize(c->ev[0]));
    if (c->h_active[0] > 0) {
      bool changed = false;
      rc = build_union(c, mb, true, &changed);
      if (rc != PR_OK) return rc;
      if (changed) {
        rc = ensure_batch_graph(c, mb, opts.check_every);
        if (rc != PR_OK) return rc;
      }
    }
  }
  PR_TRY(issue(1));
  launched++;
  int rebuilds = 0;
  // tail handoff: once the nodes still iterating are so few that one node at a
  // time is cheaper per iteration (batch_pays), the batch stops and they
  // continue on the single-node path from their current iterates
  bool handoff = false;
  const bool may_hand_off = !(c->debug & PR_DEBUG_FORCE_BATCH);
  for (int64_t k = 0;; k++) {
    const int slot = (int)(k & 1);
    PR_TRY(hipEventSynchronize(c->ev[slot]));
    if (c->h_active[slot] <= 0) break;
    if (launched >= max_launches) break;
    if (may_hand_off && !batch_pays(c, c->h_active[slot])) {
      handoff = true;
      break;
    }
    if (c->union_on && rebuilds < kUnionRebuilds) {
      // supports still move in the first launches: once the other launch is
      // done, join the coordinates that left the union when there are more
      // than one per four nodes (each costs one matrix column per iteration)
      PR_TRY(hipStreamSynchronize(s));
      std::vector<int32_t> oc((size_t)mb);
      PR_TRY(hipMemcpy(oc.data(), c->d_ocnt, sizeof(int32_t) * mb, hipMemcpyDeviceToHost));
      int64_t nout = 0;
      for (int32_t v : oc) nout += v;
      rebuilds++;
      if (4 * nout > mb) {
        bool changed = false;
        rc = build_union(c, mb, false, &changed);
        if (rc != PR_OK) return rc;
        if (changed) {
          rc = ensure_batch_graph(c, mb, opts.check_every);
          if (rc != PR_OK) return rc;
        } else {
          rebuilds = kUnionRebuilds;  // nothing new fits: keep this union
        }
      }
    }
    PR_TRY(issue(slot));
    launched++;
  }
  PR_TRY(hipStreamSynchronize(s));
  PR_TRY(hipMemcpy(c->h_bstate, c->d_bstate, sizeof(NodeState) * mb, hipMemcpyDeviceToHost));
  c->union_nout = 0;
  if (c->union_on) {
    std::vector<int32_t> oc((size_t)mb);
    PR_TRY(hipMemcpy(oc.data(), c->d_ocnt, sizeof(int32_t) * mb, hipMemcpyDeviceToHost));
    for (int32_t v : oc) c->union_nout += v;
  }
  // FP64 certification of every node over the stored X, at the iterate that
  // stopped it: the decision of the batched step (converged, prune, branch)
  // stands if Phi(x) and Psi(zeta) recomputed over X confirm it; otherwise the
  // node continues on the single-node path.  A node stopped by the iteration
  // limit reports its (valid) recomputed bounds.
  for (int32_t q = 0; q < mb; q++) {
    const NodeState &hs = c->h_bstate[q];
    if (!hs.done)  // the graph loop stopped at the iteration limit before this node did
      PR_TRY(hipMemcpyAsync(c->bxbest + (int64_t)q * p, (hs.parity ? c->bx1 : c->bx0) + (int64_t)q * p,
                            sizeof(double) * p, hipMemcpyDeviceToDevice, s));
  }
  // certify with the dual vector of each stopping iterate, zeta = 2 (y - X x),
  // by Phi(x) and Psi(zeta) recomputed over the stored X, all nodes at once
  std::vector<double> lbs, ubs;
  rc = certify_batch(c, mb, lbs, ubs);
  if (rc != PR_OK) return rc;
  for (int32_t q = 0; q < mb; q++) {
    const int32_t i = slot_of[(size_t)q];
    const NodeState &hs = c->h_bstate[q];
    double *xq = c->bxbest + (int64_t)q * p;
    const int st = hs.done ? hs.status : kMaxIter;
    const double lb = lbs[(size_t)q], ub = ubs[(size_t)q];
    const double rel = (ub - lb) / fmax(fabs(ub), 1e-300);
    bool confirmed = false;
    if (st == kConverged) confirmed = rel <= opts.rel_gap_tol;
    else if (st == kCutoffPrune) confirmed = lb >= opts.cutoff;
    else if (st == kCutoffBranch) confirmed = ub <= opts.cutoff;
    else confirmed = !(handoff && !hs.done);  // iteration limit; a handed-off node continues
    pr_result &r = out[i];
    if (confirmed) {
      r.lower_bound = lb;
      r.primal = ub;
      r.rel_gap = rel;
      r.L = hs.L;
      r.iters = hs.iter;
      r.restarts = hs.restarts;
      r.trials = hs.trials;
      r.status = st;
      if (B_out) PR_TRY(hipMemcpyAsync(B_out + (int64_t)i * p, xq, sizeof(double) * p, hipMemcpyDeviceToDevice, s));
    } else {
      // the single-node FP64 path from the node's iterate: a fresh budget after
      // an unconfirmed decision, the rest of the budget after a handoff
      pr_opts o2 = opts;
      if (!hs.done) o2.max_iter = opts.max_iter > hs.iter ? opts.max_iter - hs.iter : 1;
      rc = pr_solve(c, &nodes[i], &o2, xq, B_out ? B_out + (int64_t)i * p : nullptr, nullptr, &r);
      if (rc != PR_OK) return rc;
      if (r.lower_bound < lb) r.lower_bound = lb;  // both are valid bounds
      r.rel_gap = (r.primal - r.lower_bound) / fmax(fabs(r.primal), 1e-300);
      r.iters += hs.iter;
      r.restarts += hs.restarts;
      r.trials += hs.trials;
    }
  }
  PR_TRY(hipStreamSynchronize(s));
  return PR_OK;
}

}  // extern "C"
