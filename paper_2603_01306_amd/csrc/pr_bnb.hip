// Branch and bound for the k-sparse problem (1) on top of the batched node
// relaxations: every node's certified FP64 lower bound comes from
// pr_solve_batch (perspective relaxation, FISTA with the duality-gap restart,
// dynamic termination against the incumbent as in Section 5.3); this file
// holds the search around it and the incumbent heuristic.
//
// Search: best first over open nodes keyed by their parents' bound; each round
// solves up to max_batch nodes together, warm-started from their parents'
// solutions.  A solved node is fathomed when its bound reaches the incumbent
// (within the relative tolerance); otherwise it branches on the free
// coordinate with the largest |beta_j| of its relaxation solution (children:
// j fixed to one, j fixed to zero).
//
// Incumbent: the support S = J1 + the kbar largest |beta_j| over the free
// coordinates of each node's relaxation solution, and the leaf node J1 = S,
// J0 = the rest.  At that leaf kbar = 0, so g_N is half the squared norm on S
// and the relaxation is problem (1) restricted to S (the box-constrained
// ridge fit for least squares): pr_solve on it (warm-started from the node's
// solution, solved to a 1e-9 relative gap) returns a feasible k-sparse point
// whose primal value, evaluated in FP64 over the stored X, is the objective
// of (1) there.  Each support is tried once.  A node with nothing left to
// branch on is such a leaf itself, so its own problem is always offered as an
// incumbent before it is fathomed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <queue>
#include <set>
#include <vector>

#include "pr_internal.h"

#define PR_TRY(expr)                          \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return PR_EDEVICE;  \
  } while (0)

namespace pr {
namespace {

struct Open {
  double bound;
  int32_t depth;
  int32_t slot;  // arena slot of the parent's solution (-1: cold start)
  std::vector<int32_t> J0, J1;
};
struct OpenCmp {
  bool operator()(const Open &a, const Open &b) const { return a.bound > b.bound; }
};

}  // namespace

struct BnbState {
  pr_ctx *c;
  Problem P;
  hipStream_t s;
  int64_t n, p;
  double *arena = nullptr;  // [slots][p] parent solutions
  int32_t slots = 0;
  std::vector<int32_t> free_slots, refs;
  double *d_B0 = nullptr, *d_Bout = nullptr;
  double *d_cand = nullptr;  // p: incumbent candidate
  double ub = INFINITY;
  std::vector<double> best;  // dense incumbent (host)
  std::set<std::vector<int32_t>> tried;  // supports already solved
};

// Incumbent candidate from a relaxation solution (host copy beta, device copy
// d_beta): the leaf node of its support S solved by pr_solve; updates
// st.ub / st.best when its objective improves.
static int try_incumbent(BnbState &st, const pr_node &node, const std::vector<int8_t> &status,
                         const std::vector<double> &beta, const double *d_beta) {
  const int64_t p = st.p;
  std::vector<int32_t> S;
  int32_t kbar = node.k;
  for (int64_t j = 0; j < p; j++)
    if (status[(size_t)j] == kOne) {
      S.push_back((int32_t)j);
      kbar--;
    }
  std::vector<std::pair<double, int32_t>> fr;
  for (int64_t j = 0; j < p; j++)
    if (status[(size_t)j] == kFree && beta[(size_t)j] != 0.0) fr.push_back({-std::fabs(beta[(size_t)j]), (int32_t)j});
  const size_t take = std::min<size_t>(fr.size(), (size_t)std::max(kbar, 0));
  std::partial_sort(fr.begin(), fr.begin() + take, fr.end());
  for (size_t q = 0; q < take; q++) S.push_back(fr[q].second);
  const int64_t m = (int64_t)S.size();
  std::sort(S.begin(), S.end());
  if (!st.tried.insert(S).second) return PR_OK;
  std::vector<int32_t> J0;
  J0.reserve((size_t)(p - m));
  size_t q = 0;
  for (int64_t j = 0; j < p; j++) {
    if (q < S.size() && S[q] == (int32_t)j) q++;
    else J0.push_back((int32_t)j);
  }
  pr_node leaf = node;
  leaf.J1 = S.empty() ? nullptr : S.data();
  leaf.n1 = m;
  leaf.J0 = J0.empty() ? nullptr : J0.data();
  leaf.n0 = (int64_t)J0.size();
  pr_opts lo;
  pr_opts_default(&lo);
  lo.rel_gap_tol = 1e-9;
  if (node_ept(p) != 0) lo.method = PR_FISTA_BT_GAP;  // the line search where the register-resident step runs
  pr_result r;
  int rc = pr_solve(st.c, &leaf, &lo, d_beta, st.d_cand, nullptr, &r);
  if (rc != PR_OK) return rc;
  if (r.primal < st.ub) {
    st.ub = r.primal;
    st.best.assign((size_t)p, 0.0);
    PR_TRY(hipMemcpyAsync(st.best.data(), st.d_cand, sizeof(double) * p, hipMemcpyDeviceToHost, st.s));
    PR_TRY(hipStreamSynchronize(st.s));
  }
  return PR_OK;
}

}  // namespace pr

using namespace pr;

extern "C" {

void pr_bnb_opts_default(pr_bnb_opts *o) {
  if (!o) return;
  o->rel_gap_tol = 1e-4;
  o->time_limit_s = INFINITY;
  o->max_nodes = 100000;
  o->batch = 0;
  pr_opts_default(&o->node_opts);
}

int pr_bnb(pr_ctx *c, const pr_node *root, const pr_bnb_opts *opts_in, double *beta_best, pr_bnb_result *out) {
  if (!c || !root || !out) return PR_EINVAL;
  pr_bnb_opts o;
  pr_bnb_opts_default(&o);
  if (opts_in) o = *opts_in;
  if (!(o.rel_gap_tol >= 0.0) || o.max_nodes < 1 || o.batch < 0 || !(o.time_limit_s > 0.0)) return PR_EINVAL;
  const Problem &P = ctx_problem(c);
  const auto t0 = std::chrono::steady_clock::now();
  auto elapsed = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
  {
    std::vector<int8_t> st0;
    int64_t n1, pbar;
    int32_t kbar;
    bool inf;
    int rc = build_status(root, P.p, st0, n1, pbar, kbar, inf);
    if (rc != PR_OK) return rc;
  }
  BnbState st;
  st.c = c;
  st.P = P;
  st.s = ctx_stream(c);
  st.n = P.n;
  st.p = P.p;
  const int32_t B = o.batch > 0 ? std::min(o.batch, ctx_max_batch(c)) : ctx_max_batch(c);
  st.slots = std::min<int32_t>(o.max_nodes + 1, 4 * 4096);
  memset(out, 0, sizeof(*out));
  int rc = PR_OK;
  bool ok = hipMalloc((void **)&st.arena, sizeof(double) * st.slots * P.p) == hipSuccess;
  ok = ok && hipMalloc((void **)&st.d_B0, sizeof(double) * B * P.p) == hipSuccess;
  ok = ok && hipMalloc((void **)&st.d_Bout, sizeof(double) * B * P.p) == hipSuccess;
  ok = ok && hipMalloc((void **)&st.d_cand, sizeof(double) * P.p) == hipSuccess;
  auto cleanup = [&]() {
    void *bufs[] = {st.arena, st.d_B0, st.d_Bout, st.d_cand};
    for (void *q : bufs)
      if (q) (void)hipFree(q);
  };
  if (!ok) {
    cleanup();
    return PR_ENOMEM;
  }
  st.refs.assign((size_t)st.slots, 0);
  for (int32_t q = st.slots - 1; q >= 0; q--) st.free_slots.push_back(q);

  std::priority_queue<Open, std::vector<Open>, OpenCmp> open;
  {
    Open r;
    r.bound = -INFINITY;
    r.depth = 0;
    r.slot = -1;
    if (root->n0) r.J0.assign(root->J0, root->J0 + root->n0);
    if (root->n1) r.J1.assign(root->J1, root->J1 + root->n1);
    open.push(r);
  }
  int64_t solved = 0, pruned = 0;
  int32_t maxdepth = 0;
  double relax_s = 0.0;
  std::vector<double> bh((size_t)P.p);
  int status = PR_BNB_OPTIMAL;
  auto gap_closed = [&](double lb) { return std::isfinite(st.ub) && st.ub - lb <= o.rel_gap_tol * std::fabs(st.ub); };
  while (!open.empty()) {
    if (gap_closed(open.top().bound)) break;
    if (solved >= o.max_nodes) {
      status = PR_BNB_NODE_LIMIT;
      break;
    }
    if (elapsed() >= o.time_limit_s) {
      status = PR_BNB_TIME_LIMIT;
      break;
    }
    // next round: up to B open nodes, best bound first
    std::vector<Open> round;
    while (!open.empty() && (int32_t)round.size() < B && solved + (int64_t)round.size() < o.max_nodes) {
      Open nd = open.top();
      open.pop();
      if (gap_closed(nd.bound)) {
        pruned++;
        if (nd.slot >= 0 && --st.refs[(size_t)nd.slot] == 0) st.free_slots.push_back(nd.slot);
        continue;
      }
      round.push_back(std::move(nd));
    }
    if (round.empty()) continue;
    const int32_t m = (int32_t)round.size();
    std::vector<pr_node> nodes((size_t)m);
    for (int32_t i = 0; i < m; i++) {
      pr_node &q = nodes[(size_t)i];
      q = *root;
      q.J0 = round[(size_t)i].J0.empty() ? nullptr : round[(size_t)i].J0.data();
      q.n0 = (int64_t)round[(size_t)i].J0.size();
      q.J1 = round[(size_t)i].J1.empty() ? nullptr : round[(size_t)i].J1.data();
      q.n1 = (int64_t)round[(size_t)i].J1.size();
      double *dst = st.d_B0 + (int64_t)i * P.p;
      if (round[(size_t)i].slot >= 0) {
        if (hipMemcpyAsync(dst, st.arena + (int64_t)round[(size_t)i].slot * P.p, sizeof(double) * P.p,
                           hipMemcpyDeviceToDevice, st.s) != hipSuccess) {
          rc = PR_EDEVICE;
          break;
        }
      } else if (hipMemsetAsync(dst, 0, sizeof(double) * P.p, st.s) != hipSuccess) {
        rc = PR_EDEVICE;
        break;
      }
    }
    if (rc != PR_OK) break;
    pr_opts no = o.node_opts;
    no.cutoff = std::isfinite(st.ub) ? st.ub * (1.0 - o.rel_gap_tol) : NAN;
    no.trace = nullptr;
    std::vector<pr_result> res((size_t)m);
    const double ts = elapsed();
    rc = pr_solve_batch(c, nodes.data(), m, &no, st.d_B0, st.d_Bout, res.data());
    relax_s += elapsed() - ts;
    if (rc != PR_OK) break;
    solved += m;
    for (int32_t i = 0; i < m; i++) {
      Open &nd = round[(size_t)i];
      if (nd.slot >= 0 && --st.refs[(size_t)nd.slot] == 0) st.free_slots.push_back(nd.slot);
      maxdepth = std::max(maxdepth, nd.depth);
      const pr_result &r = res[(size_t)i];
      if (r.status == PR_INFEASIBLE || r.status == PR_CUTOFF_PRUNE) {
        pruned++;
        continue;
      }
      const double bound = std::max(nd.bound, r.lower_bound);
      std::vector<int8_t> sv;
      int64_t n1, pbar;
      int32_t kbar;
      bool inf;
      rc = build_status(&nodes[(size_t)i], P.p, sv, n1, pbar, kbar, inf);
      if (rc != PR_OK) break;
      if (hipMemcpyAsync(bh.data(), st.d_Bout + (int64_t)i * P.p, sizeof(double) * P.p, hipMemcpyDeviceToHost,
                         st.s) != hipSuccess ||
          hipStreamSynchronize(st.s) != hipSuccess) {
        rc = PR_EDEVICE;
        break;
      }
      rc = try_incumbent(st, nodes[(size_t)i], sv, bh, st.d_Bout + (int64_t)i * P.p);
      if (rc != PR_OK) break;
      if (gap_closed(bound)) {
        pruned++;
        continue;
      }
      // branch on the free coordinate with the largest |beta_j|
      int32_t jb = -1;
      double amax = -1.0;
      for (int64_t j = 0; j < P.p; j++)
        if (sv[(size_t)j] == kFree && std::fabs(bh[(size_t)j]) > amax) {
          amax = std::fabs(bh[(size_t)j]);
          jb = (int32_t)j;
        }
      if (jb < 0 || kbar <= 0) {  // a leaf: its own problem was offered as an incumbent above
        pruned++;
        continue;
      }
      int32_t slot = -1;
      if (!st.free_slots.empty()) {
        slot = st.free_slots.back();
        st.free_slots.pop_back();
        st.refs[(size_t)slot] = 2;
        if (hipMemcpyAsync(st.arena + (int64_t)slot * P.p, st.d_Bout + (int64_t)i * P.p, sizeof(double) * P.p,
                           hipMemcpyDeviceToDevice, st.s) != hipSuccess) {
          rc = PR_EDEVICE;
          break;
        }
      }
      Open a, b2;
      a.bound = b2.bound = bound;
      a.depth = b2.depth = nd.depth + 1;
      a.slot = b2.slot = slot;
      a.J0 = nd.J0;
      a.J1 = nd.J1;
      a.J1.push_back(jb);
      b2.J0 = nd.J0;
      b2.J0.push_back(jb);
      b2.J1 = nd.J1;
      open.push(std::move(a));
      open.push(std::move(b2));
    }
    if (rc != PR_OK) break;
  }
  if (rc == PR_OK) {
    double lb = open.empty() ? st.ub : std::min(st.ub, open.top().bound);
    if (open.empty() && status == PR_BNB_OPTIMAL) lb = st.ub;
    out->lower_bound = lb;
    out->upper_bound = st.ub;
    out->rel_gap = (st.ub - lb) / std::fmax(std::fabs(st.ub), 1e-300);
    if (status == PR_BNB_OPTIMAL && !(out->rel_gap <= o.rel_gap_tol)) status = PR_BNB_NODE_LIMIT;
    out->nodes_solved = solved;
    out->nodes_pruned = pruned;
    out->nodes_open = (int64_t)open.size();
    out->max_depth = maxdepth;
    out->status = status;
    out->seconds = elapsed();
    out->relaxation_seconds = relax_s;
    if (beta_best) {
      if (st.best.empty()) st.best.assign((size_t)P.p, 0.0);
      if (hipMemcpy(beta_best, st.best.data(), sizeof(double) * P.p, hipMemcpyHostToDevice) != hipSuccess)
        rc = PR_EDEVICE;
    }
  }
  cleanup();
  return rc;
}

}  // extern "C"
