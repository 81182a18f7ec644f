// Batch scheduler: many transforms of different plans (uneven L and spin)
// issued as one unit, optionally captured once into a HIP graph and
// replayed.
//
// Jobs that share a plan share its workspace, so they run in order on one
// internal stream; jobs of different plans run on different internal
// streams forked from, and joined back into, the caller's stream (in the
// graph: parallel branches), so that small transforms that cannot fill the
// GPU alone overlap.  Internal streams use the default priority.

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "common.hpp"

struct osht_graph {
  std::vector<osht_job_t> jobs;  // the job list the graph was captured for
  std::vector<int64_t> versions;  // workspace version of each job's plan at capture
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~osht_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace osht {

namespace {

constexpr int kMaxStreams = 8;

struct StreamPool {
  int device = -1;
  hipStream_t s[kMaxStreams] = {};
  hipEvent_t fork = nullptr, join[kMaxStreams] = {};
  hipStream_t origin = nullptr;  // capture origin (graphs)
  void init(int dev) {
    if (device == dev) return;
    OSHT_CHECK(device < 0, OSHT_ENOTSUP, "batch scheduler used on two devices in one process thread");
    for (auto& x : s) OSHT_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    OSHT_HIP(hipStreamCreateWithFlags(&origin, hipStreamNonBlocking));
    OSHT_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    for (auto& e : join) OSHT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    device = dev;
  }
};

thread_local StreamPool g_pool;

void run_job(const osht_job_t& j, hipStream_t st) {
  Plan& p = const_cast<osht_plan_t*>(j.plan)->p;
  const double* in = static_cast<const double*>(j.in);
  double* out = static_cast<double*>(j.out);
  switch (j.direction) {
    case OSHT_DIR_INVERSE: run_inverse(p, in, out, j.batch, st); break;
    case OSHT_DIR_FORWARD: run_forward(p, in, out, j.batch, st); break;
    case OSHT_DIR_INVERSE_ADJOINT: run_inverse_adjoint(p, in, out, j.batch, st); break;
    case OSHT_DIR_FORWARD_ADJOINT: run_forward_adjoint(p, in, out, j.batch, st); break;
    default: throw Error{OSHT_EINVAL, "unknown job direction"};
  }
  if (p.flags & OSHT_CHECK_FINITE) launch_finite_scan(p, out, 2 * (int64_t)p.L * p.L * j.batch, st);
}

// Issues every job: fork from `from`, plan-grouped streams, join into `from`.
void issue(const std::vector<osht_job_t>& jobs, hipStream_t from) {
  std::map<const osht_plan_t*, int> lane;
  for (const auto& j : jobs)
    if (!lane.count(j.plan)) lane.emplace(j.plan, (int)(lane.size() % kMaxStreams));
  OSHT_HIP(hipEventRecord(g_pool.fork, from));
  const int nl = std::min<int>((int)lane.size(), kMaxStreams);
  for (int i = 0; i < nl; ++i) OSHT_HIP(hipStreamWaitEvent(g_pool.s[i], g_pool.fork, 0));
  for (const auto& j : jobs) run_job(j, g_pool.s[lane[j.plan]]);
  for (int i = 0; i < nl; ++i) {
    OSHT_HIP(hipEventRecord(g_pool.join[i], g_pool.s[i]));
    OSHT_HIP(hipStreamWaitEvent(from, g_pool.join[i], 0));
  }
}

std::vector<int64_t> versions_of(const std::vector<osht_job_t>& jobs) {
  std::vector<int64_t> v;
  for (const auto& j : jobs) v.push_back(j.plan->p.ws_version);
  return v;
}

// Same jobs, and no plan's workspace or descriptor tables (which the
// captured kernels read) rebuilt since the capture.
bool same_jobs(const osht_graph_t& g, const std::vector<osht_job_t>& b) {
  if (g.jobs.size() != b.size()) return false;
  for (size_t i = 0; i < b.size(); ++i) {
    const osht_job_t& a = g.jobs[i];
    if (a.plan != b[i].plan || a.direction != b[i].direction || a.in != b[i].in || a.out != b[i].out ||
        a.batch != b[i].batch)
      return false;
  }
  return g.versions == versions_of(b);
}

}  // namespace

// Called with the jobs validated; graph_inout may be NULL (direct issue).
void batch_run(const osht_job_t* jobs, int n, hipStream_t stream, osht_graph_t** graph_inout) {
  int dev = 0;
  OSHT_HIP(hipGetDevice(&dev));
  g_pool.init(dev);
  std::vector<osht_job_t> list(jobs, jobs + n);
  // workspaces and descriptor tables are sized before any capture
  std::vector<std::unique_lock<std::mutex>> locks;
  {
    std::vector<Plan*> plans;
    for (const auto& j : list) {
      Plan* p = &const_cast<osht_plan_t*>(j.plan)->p;
      OSHT_CHECK(p->device == dev, OSHT_EINVAL, "job plan lives on another device");
      if (std::find(plans.begin(), plans.end(), p) == plans.end()) plans.push_back(p);
    }
    std::sort(plans.begin(), plans.end());  // fixed lock order
    for (Plan* p : plans) locks.emplace_back(p->mu);
    for (const auto& j : list) prepare_transforms(const_cast<osht_plan_t*>(j.plan)->p, j.batch);
  }
  if (!graph_inout) {
    issue(list, stream);
    return;
  }
  osht_graph_t* g = *graph_inout;
  if (g && g->device == dev && same_jobs(*g, list)) {
    OSHT_HIP(hipGraphLaunch(g->exec, stream));
    return;
  }
  std::unique_ptr<osht_graph_t> ng(new osht_graph_t);
  ng->jobs = list;
  ng->versions = versions_of(list);
  ng->device = dev;
  // kernel timing events are not captured
  std::vector<std::pair<Plan*, bool>> prof;
  for (const auto& j : list) {
    Plan* p = &const_cast<osht_plan_t*>(j.plan)->p;
    prof.emplace_back(p, p->prof.enabled);
    p->prof.enabled = false;
  }
  hipError_t cap = hipStreamBeginCapture(g_pool.origin, hipStreamCaptureModeRelaxed);
  try {
    OSHT_HIP(cap);
    issue(list, g_pool.origin);
  } catch (...) {
    hipGraph_t junk = nullptr;
    if (cap == hipSuccess) (void)hipStreamEndCapture(g_pool.origin, &junk);
    if (junk) (void)hipGraphDestroy(junk);
    for (auto& pr : prof) pr.first->prof.enabled = pr.second;
    throw;
  }
  for (auto& pr : prof) pr.first->prof.enabled = pr.second;
  OSHT_HIP(hipStreamEndCapture(g_pool.origin, &ng->graph));
  OSHT_HIP(hipGraphInstantiate(&ng->exec, ng->graph, nullptr, nullptr, 0));
  OSHT_HIP(hipGraphLaunch(ng->exec, stream));
  delete g;
  *graph_inout = ng.release();
}

}  // namespace osht

extern "C" int osht_graph_destroy(osht_graph_t* graph) {
  delete graph;
  return OSHT_OK;
}
