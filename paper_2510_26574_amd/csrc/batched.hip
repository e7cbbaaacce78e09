// Batched form: many decompositions (rpchol_factor, bistoch_degrees,
// bistoch_eig per job; jobs on shared points factorised together by
// rpchol_factor_group) issued over a pool of streams so that small jobs
// overlap on the chip, optionally captured once into a HIP graph and
// replayed.  Jobs are assigned longest-first to the stream with the least
// estimated work (LPT list scheduling); each stream reuses one slice of the
// caller's workspace for its jobs, which run in sequence on it.
#include <algorithm>
#include <mutex>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "profile.hpp"

namespace {

constexpr int MAX_STREAMS = 32;

struct DevicePool {
  int device;
  int n;
  hipStream_t s[MAX_STREAMS];
  hipEvent_t fork;
  hipEvent_t join[MAX_STREAMS];
};

std::mutex g_mu;
std::vector<DevicePool*> g_pools;  // one per device, kept until the process ends

int pool_for_current(int n, DevicePool** out) {
  int dev = 0;
  RPC_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  DevicePool* p = nullptr;
  for (DevicePool* q : g_pools)
    if (q->device == dev) p = q;
  if (!p) {
    p = new DevicePool();
    p->device = dev;
    p->n = 0;
    RPC_HIP_CHECK(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    for (int i = 0; i < MAX_STREAMS; ++i)
      RPC_HIP_CHECK(hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming));
    g_pools.push_back(p);
  }
  while (p->n < n) {
    RPC_HIP_CHECK(hipStreamCreateWithFlags(&p->s[p->n], hipStreamNonBlocking));
    ++p->n;
  }
  *out = p;
  return RPC_OK;
}

__global__ void k_clear_status(int32_t* st) { *st = 0; }

int job_ws(const rpc_job* j, size_t* bytes) {
  size_t a = 0, b = 0, c = 0;
  int rc = rpchol_factor_workspace_size(&j->X, &j->factor, &a);
  if (rc) return rc;
  rc = bistoch_degrees_workspace_size(j->X.N, j->factor.r, &b);
  if (rc) return rc;
  rc = bistoch_eig_workspace_size(j->X.N, j->factor.r, &j->eig, &c);
  if (rc) return rc;
  *bytes = align_up(std::max(a, std::max(b, c)), 256);
  return RPC_OK;
}

double job_cost(const rpc_job* j) {
  const double N = (double)j->X.N, d = (double)j->X.d, r = (double)j->factor.r;
  return N * r * (2.0 * d + 3.0 * r);
}

// Jobs flagged RPC_FACTOR_SHARED_X that use the same points (pointer, N, d,
// ldx) and the same factor options apart from eps and the uniforms form one
// unit: their factorisations run together (rpchol_factor_group), then each
// job's degrees and eigenpairs in turn.  Every other job is a unit of one.
constexpr int MAX_UNIT = 16;

bool same_group(const rpc_job* a, const rpc_job* b) {
  const rpc_factor_opts &p = a->factor, &q = b->factor;
  return (p.flags & RPC_FACTOR_SHARED_X) && (q.flags & RPC_FACTOR_SHARED_X) && a->X.X == b->X.X &&
         a->X.N == b->X.N && a->X.d == b->X.d && a->X.ldx == b->X.ldx && p.r == q.r &&
         p.b == q.b && p.mode == q.mode && p.mode != RPC_REPLAY && p.gemm_dtype == q.gemm_dtype &&
         p.factor_dtype == q.factor_dtype && p.tau == q.tau && p.flags == q.flags &&
         a->ldf == b->ldf;
}

std::vector<std::vector<int>> make_units(const rpc_job* jobs, int n) {
  std::vector<std::vector<int>> units;
  std::vector<char> used(n, 0);
  for (int i = 0; i < n; ++i) {
    if (used[i]) continue;
    std::vector<int> u{i};
    used[i] = 1;
    for (int j = i + 1; j < n && (int)u.size() < MAX_UNIT; ++j)
      if (!used[j] && same_group(&jobs[i], &jobs[j])) {
        u.push_back(j);
        used[j] = 1;
      }
    units.push_back(u);
  }
  return units;
}

int unit_ws(const rpc_job* jobs, const std::vector<int>& u, size_t* bytes) {
  size_t m = 0;
  for (int j : u) {
    size_t b = 0;
    const int rc = job_ws(&jobs[j], &b);
    if (rc) return rc;
    m = std::max(m, b);
  }
  if (u.size() > 1) {
    size_t g = 0;
    const int rc = rpchol_factor_group_workspace_size(&jobs[u[0]].X, &jobs[u[0]].factor,
                                                      (int32_t)u.size(), &g);
    if (rc) return rc;
    m = std::max(m, align_up(g, 256));
  }
  *bytes = m;
  return RPC_OK;
}

int per_stream_bytes(const rpc_job* jobs, int n, size_t* out) {
  size_t m = 0;
  for (const auto& u : make_units(jobs, n)) {
    size_t b = 0;
    const int rc = unit_ws(jobs, u, &b);
    if (rc) return rc;
    m = std::max(m, b);
  }
  *out = m;
  return RPC_OK;
}

int issue_eig(const rpc_job* j, void* ws, size_t wsb, rpc_stream_t rs) {
  int rc = bistoch_degrees(j->F, j->factor.factor_dtype, j->X.N, j->ldf, j->factor.r, j->k, j->c,
                           j->d_tilde, j->q_tilde, ws, wsb, j->dev_status, rs);
  if (rc) return rc;
  return bistoch_eig(j->F, j->factor.factor_dtype, j->X.N, j->ldf, j->factor.r, j->k, j->c,
                     j->d_tilde, j->q_tilde, &j->eig, j->U, j->ldu, j->lambda, j->ext_E, ws, wsb,
                     j->dev_status, rs);
}

int issue_unit(const rpc_job* jobs, const std::vector<int>& u, void* ws, size_t wsb, hipStream_t s) {
  rpc_stream_t rs = reinterpret_cast<rpc_stream_t>(s);
  for (int j : u) hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, jobs[j].dev_status);
  RPC_LAUNCH_CHECK();
  int rc;
  if (u.size() == 1) {
    const rpc_job* j = &jobs[u[0]];
    rc = rpchol_factor(&j->X, &j->factor, j->F, j->ldf, j->pivots, j->rho, j->k, ws, wsb,
                       j->dev_status, rs);
  } else {
    const int G = (int)u.size();
    double eps[MAX_UNIT];
    const rpc_factor_opts* opts[MAX_UNIT];
    void* F[MAX_UNIT];
    int64_t* piv[MAX_UNIT];
    double* rho[MAX_UNIT];
    int32_t* k[MAX_UNIT];
    int32_t* st[MAX_UNIT];
    for (int g = 0; g < G; ++g) {
      const rpc_job* j = &jobs[u[g]];
      eps[g] = j->X.eps;
      opts[g] = &j->factor;
      F[g] = j->F;
      piv[g] = j->pivots;
      rho[g] = j->rho;
      k[g] = j->k;
      st[g] = j->dev_status;
    }
    rc = rpchol_factor_group(&jobs[u[0]].X, eps, opts, G, F, jobs[u[0]].ldf, piv, rho, k, st, ws,
                             wsb, rs);
  }
  if (rc) return rc;
  for (int j : u) {
    rc = issue_eig(&jobs[j], ws, wsb, rs);
    if (rc) return rc;
  }
  return RPC_OK;
}

int issue_job(const rpc_job* j, void* ws, size_t wsb, hipStream_t s) {
  return issue_unit(j, std::vector<int>{0}, ws, wsb, s);
}

// Fork onto the pool streams, issue every job, join back into `origin`.
// Keeps bistoch_eig from blocking the issuing thread while jobs are issued.
struct NoHostGate {
  NoHostGate() { rpc_internal::set_host_gate_off(true); }
  ~NoHostGate() { rpc_internal::set_host_gate_off(false); }
};

int issue_all(const rpc_job* jobs, int n, int ns, void* ws, size_t wsb, hipStream_t origin) {
  NoHostGate no_gate;
  if (!jobs || n < 1 || ns < 1 || ns > MAX_STREAMS) return RPC_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!jobs[i].dev_status) return RPC_EINVAL;
  size_t per = 0;
  int rc = per_stream_bytes(jobs, n, &per);
  if (rc) return rc;
  if (!ws || wsb < per * (size_t)ns) return RPC_EWORKSPACE;
  DevicePool* p = nullptr;
  rc = pool_for_current(ns, &p);
  if (rc) return rc;
  // units (jobs, or groups of jobs on shared points), longest first onto the
  // least loaded stream
  const std::vector<std::vector<int>> units = make_units(jobs, n);
  const int nu = (int)units.size();
  std::vector<double> cost(nu, 0.0);
  for (int i = 0; i < nu; ++i)
    for (int j : units[i]) cost[i] += job_cost(&jobs[j]);
  std::vector<int> order(nu);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<double> load(ns, 0.0);
  std::vector<std::vector<int>> lists(ns);
  for (int u : order) {
    const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lists[s].push_back(u);
    load[s] += cost[u];
  }
  RPC_HIP_CHECK(hipEventRecord(p->fork, origin));
  for (int s = 0; s < ns; ++s) RPC_HIP_CHECK(hipStreamWaitEvent(p->s[s], p->fork, 0));
  int first_err = RPC_OK;
  for (int s = 0; s < ns; ++s) {
    char* base = (char*)ws + per * (size_t)s;
    for (int u : lists[s]) {
      rc = issue_unit(jobs, units[u], base, per, p->s[s]);
      if (rc && !first_err) first_err = rc;
      if (rc) break;
    }
  }
  // always join, so the origin stream (and a capture) is left consistent
  for (int s = 0; s < ns; ++s) {
    RPC_HIP_CHECK(hipEventRecord(p->join[s], p->s[s]));
    RPC_HIP_CHECK(hipStreamWaitEvent(origin, p->join[s], 0));
  }
  return first_err;
}

}  // namespace

extern "C" {

int rpc_job_workspace_size(const rpc_job* job, size_t* bytes) {
  if (!job || !bytes) return RPC_EINVAL;
  return job_ws(job, bytes);
}

int rpc_batched_workspace_size(const rpc_job* jobs, int32_t n_jobs, int32_t n_streams,
                               size_t* bytes) {
  if (!jobs || !bytes || n_jobs < 1 || n_streams < 1 || n_streams > MAX_STREAMS) return RPC_EINVAL;
  size_t per = 0;
  const int rc = per_stream_bytes(jobs, n_jobs, &per);
  if (rc) return rc;
  *bytes = per * (size_t)n_streams;
  return RPC_OK;
}

int rpc_batched_run(const rpc_job* jobs, int32_t n_jobs, int32_t n_streams, void* workspace,
                    size_t workspace_bytes, rpc_stream_t stream) {
  return issue_all(jobs, n_jobs, n_streams, workspace, workspace_bytes,
                   reinterpret_cast<hipStream_t>(stream));
}

int rpc_batched_graph_create(const rpc_job* jobs, int32_t n_jobs, int32_t n_streams,
                             void* workspace, size_t workspace_bytes, rpc_stream_t stream,
                             rpc_graph* out) {
  if (!out || !stream || prof::enabled()) return RPC_EINVAL;
  *out = nullptr;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  RPC_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const int rc = issue_all(jobs, n_jobs, n_streams, workspace, workspace_bytes, st);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (rc != RPC_OK || e != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return rc != RPC_OK ? rc : RPC_EHIP;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    return RPC_EHIP;
  }
  rpc_graph h = new rpc_graph_s{g, x};
  *out = h;
  return RPC_OK;
}

int rpc_graph_launch(rpc_graph g, rpc_stream_t stream) {
  if (!g) return RPC_EINVAL;
  RPC_HIP_CHECK(hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)));
  return RPC_OK;
}

int rpc_graph_destroy(rpc_graph g) {
  if (!g) return RPC_EINVAL;
  hipGraphExecDestroy(g->exec);
  hipGraphDestroy(g->graph);
  delete g;
  return RPC_OK;
}

int rpc_batched_graph_launch(rpc_graph g, rpc_stream_t stream) { return rpc_graph_launch(g, stream); }

int rpc_batched_graph_destroy(rpc_graph g) { return rpc_graph_destroy(g); }

int rpc_autotune_block(const rpc_job* job, const int32_t* candidates, int32_t n_candidates,
                       int32_t reps, void* workspace, size_t workspace_bytes, rpc_stream_t stream,
                       int32_t* best_b, double* ms) {
  if (!job || !candidates || n_candidates < 1 || reps < 1 || !best_b) return RPC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  RPC_HIP_CHECK(hipEventCreate(&e0));
  RPC_HIP_CHECK(hipEventCreate(&e1));
  double best = 1e300;
  int rc = RPC_OK;
  *best_b = 0;
  for (int c = 0; c < n_candidates && rc == RPC_OK; ++c) {
    rpc_job j = *job;
    j.factor.b = candidates[c];
    size_t need = 0;
    rc = job_ws(&j, &need);
    if (rc) break;
    if (need > workspace_bytes) {
      rc = RPC_EWORKSPACE;
      break;
    }
    rc = issue_job(&j, workspace, workspace_bytes, st);  // warm-up
    double tot = 0.0;
    for (int r = 0; r < reps && rc == RPC_OK; ++r) {
      if (hipEventRecord(e0, st) != hipSuccess) rc = RPC_EHIP;
      if (rc == RPC_OK) rc = issue_job(&j, workspace, workspace_bytes, st);
      if (rc == RPC_OK && hipEventRecord(e1, st) != hipSuccess) rc = RPC_EHIP;
      float t = 0.0f;
      if (rc == RPC_OK && (hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = RPC_EHIP;
      tot += t;
    }
    if (rc) break;
    const double avg = tot / reps;
    if (ms) ms[c] = avg;
    if (avg < best) {
      best = avg;
      *best_b = candidates[c];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
