// Requests captured as HIP graphs: one graph launch replays every kernel of
// a request (steps a1-a9) on a plan's workspace, with the catalogue sizes
// and alpha read from device memory so that one graph serves catalogues of
// any size up to the capacity it was captured with.
#include <cmath>

#include "frsd_internal.h"

struct frsd_graph {
  frsd_plan *plan = nullptr;  // request 0's (a batch graph: n requests on plans of one shape)
  void *ws = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n = 1;                  // requests
  void *wss[frsd::kMaxBatch] = {};
  int64_t cap_g[frsd::kMaxBatch] = {}, cap_r[frsd::kMaxBatch] = {};  // catalogue capacities per request
};

namespace frsd {

// {N_g, N_r, alpha} of the next replay, written by a kernel on the replay's
// stream just before the graph (no memset or copy node in the graph).
__global__ void k_set_dyn(double *dyn, double ng, double nr, double alpha) {
  if (threadIdx.x == 0) {
    dyn[0] = ng;
    dyn[1] = nr;
    dyn[2] = alpha;
  }
}

// The same for every request of a batch graph (one workgroup per request;
// dyn is request 0's and moves by each request's workspace distance).
struct DynSet {
  double ng[kMaxBatch], nr[kMaxBatch], alpha[kMaxBatch];
};
__global__ void k_set_dyn_batch(double *dyn, DynSet d, Batch bt) {
  if (threadIdx.x != 0) return;
  const int r = blockIdx.x;
  double *p = moved(dyn, bt.delta[r]);
  p[0] = d.ng[r];
  p[1] = d.nr[r];
  p[2] = d.alpha[r];
}

}  // namespace frsd

using namespace frsd;

extern "C" int frsd_graph_create(frsd_plan *plan, void *ws, const frsd_catalog *gal, const frsd_catalog *ran,
                                 double alpha, const frsd_pk_out *pk, const frsd_bk_out *bk, void *stream,
                                 frsd_graph **out) {
  clear_error();
  if (!plan || !ws || !out) return fail(FRSD_EINVAL, "null argument");
  if (plan->state < 1 || plan->init_ws != ws) return fail(FRSD_ESTATE, "workspace not initialised by frsd_plan_init");
  if (prof_on()) return fail(FRSD_ESTATE, "per-kernel profiling must be off while a request is captured");
  if (plan->p.stream_moments) return fail(FRSD_EINVAL, "streamed plans are not captured");
  int rc;
  if ((rc = check_catalog(gal, false, "galaxies"))) return rc;
  if ((rc = check_catalog(ran, true, "randoms"))) return rc;
  if (gal->n + ran->n > plan->p.max_objects) return fail(FRSD_ENOMEM, "galaxies + randoms exceed max_objects");
  if (gal->n + ran->n > (int64_t)0x7fffffff) return fail(FRSD_EINVAL, "more than 2^31-1 objects");
  if (!std::isfinite(alpha)) return fail(FRSD_EINVAL, "alpha must be finite");
  if (!pk || !pk->n_modes || !pk->k_eff || !pk->p0 || !pk->p2 || !pk->p4 || !pk->s00 || !pk->s20 || !pk->s40 ||
      !pk->scalars)
    return fail(FRSD_EINVAL, "null power-spectrum output array");
  const bool do_bk = bk != nullptr && plan->p.bk_nbins > 0;
  if (do_bk && (!bk->nt || !bk->t0 || !bk->t2 || !bk->t4 || !bk->b0 || !bk->b2 || !bk->b4 || !bk->sn0 || !bk->sn2 ||
                !bk->sn4))
    return fail(FRSD_EINVAL, "null bispectrum output array");
  frsd_catalog gd, rd;
  frsd_pk_out pkd;
  frsd_bk_out bkd;
  if ((rc = device_view(gal, &gd)) || (rc = device_view(ran, &rd)) || (rc = device_view(pk, &pkd))) return rc;
  gal = &gd;
  ran = &rd;
  pk = &pkd;
  if (do_bk) {
    if ((rc = device_view(bk, &bkd))) return rc;
    bk = &bkd;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!s) return fail(FRSD_EINVAL, "capture needs an explicit (non-null) stream");
  double *dyn = ws_ptr<double>(ws, plan->L.dyn);
  hipLaunchKernelGGL(k_set_dyn, dim3(1), dim3(64), 0, s, dyn, (double)gal->n, (double)ran->n, alpha);
  FRSD_LAUNCH_CHECK();
  FRSD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const bool f64 = plan->p.precision == FRSD_F64;
  rc = f64 ? run_mesh_assign<double>(plan, ws, gal, ran, alpha, s, dyn)
           : run_mesh_assign<float>(plan, ws, gal, ran, alpha, s, dyn);
  if (!rc) rc = f64 ? run_pk<double>(plan, ws, pk, s, false) : run_pk<float>(plan, ws, pk, s, false);
  if (!rc && do_bk) rc = f64 ? run_bk<double>(plan, ws, bk, s) : run_bk<float>(plan, ws, bk, s);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(FRSD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t ge = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(FRSD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  frsd_graph *gr = new frsd_graph();
  gr->plan = plan;
  gr->ws = ws;
  gr->graph = g;
  gr->exec = ge;
  gr->wss[0] = ws;
  gr->cap_g[0] = gal->n;
  gr->cap_r[0] = ran->n;
  *out = gr;
  return FRSD_OK;
}

extern "C" int frsd_graph_launch(frsd_graph *gr, int64_t n_gal, int64_t n_ran, double alpha, void *stream) {
  clear_error();
  if (!gr) return fail(FRSD_EINVAL, "null graph");
  if (gr->n != 1) return fail(FRSD_EINVAL, "a batch graph is replayed with frsd_graph_launch_batch");
  if (n_gal < 0 || n_ran < 0 || n_gal > gr->cap_g[0] || n_ran > gr->cap_r[0])
    return fail(FRSD_ENOMEM, "catalogue sizes beyond the capacity the graph was captured with");
  if (!std::isfinite(alpha)) return fail(FRSD_EINVAL, "alpha must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_set_dyn, dim3(1), dim3(64), 0, s, ws_ptr<double>(gr->ws, gr->plan->L.dyn), (double)n_gal,
                     (double)n_ran, alpha);
  FRSD_LAUNCH_CHECK();
  FRSD_HIP(hipGraphLaunch(gr->exec, s));
  return FRSD_OK;
}

extern "C" void frsd_graph_destroy(frsd_graph *gr) {
  if (!gr) return;
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  if (gr->graph) (void)hipGraphDestroy(gr->graph);
  delete gr;
}

// A batch of requests captured as one graph: the launches of frsd_pk_batch
// (catalogues with randoms, no random cache) with every request's sizes and
// alpha read from its workspace.
extern "C" int frsd_graph_create_batch(frsd_plan *const *plans, void *const *workspaces, int32_t n,
                                       const frsd_catalog *gal, const frsd_catalog *ran, const double *alpha,
                                       const frsd_pk_out *out, void *stream, frsd_graph **graph) {
  clear_error();
  if (!graph) return fail(FRSD_EINVAL, "null argument");
  if (!ran) return fail(FRSD_EINVAL, "a batch graph needs random catalogues (no random cache)");
  if (prof_on()) return fail(FRSD_ESTATE, "per-kernel profiling must be off while a request is captured");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!s) return fail(FRSD_EINVAL, "capture needs an explicit (non-null) stream");
  frsd_catalog gd[kMaxBatch], rd[kMaxBatch];
  frsd_pk_out od[kMaxBatch];
  int rc = batch_views(plans, workspaces, n, gal, ran, alpha, out, gd, rd, od);
  if (rc) return rc;
  const bool f64 = plans[0]->p.precision == FRSD_F64;
  DynSet d{};
  for (int r = 0; r < n; ++r) {
    d.ng[r] = (double)gd[r].n;
    d.nr[r] = (double)rd[r].n;
    d.alpha[r] = alpha[r];
  }
  const Batch bt = batch_of(workspaces, n);
  double *dyn = ws_ptr<double>(workspaces[0], plans[0]->L.dyn);
  hipLaunchKernelGGL(k_set_dyn_batch, dim3(n), dim3(64), 0, s, dyn, d, bt);
  FRSD_LAUNCH_CHECK();
  FRSD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  rc = f64 ? run_mesh_assign_batch<double>(plans, workspaces, n, gd, rd, alpha, s, dyn)
           : run_mesh_assign_batch<float>(plans, workspaces, n, gd, rd, alpha, s, dyn);
  if (!rc) rc = f64 ? run_pk_batch<double>(plans, workspaces, n, od, s, false)
                    : run_pk_batch<float>(plans, workspaces, n, od, s, false);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(FRSD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t ge = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(FRSD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  frsd_graph *gr = new frsd_graph();
  gr->plan = plans[0];
  gr->ws = workspaces[0];
  gr->graph = g;
  gr->exec = ge;
  gr->n = n;
  for (int r = 0; r < n; ++r) {
    gr->wss[r] = workspaces[r];
    gr->cap_g[r] = gd[r].n;
    gr->cap_r[r] = rd[r].n;
  }
  *graph = gr;
  return FRSD_OK;
}

extern "C" int frsd_graph_launch_batch(frsd_graph *gr, const int64_t *n_gal, const int64_t *n_ran,
                                       const double *alpha, void *stream) {
  clear_error();
  if (!gr || !n_gal || !n_ran || !alpha) return fail(FRSD_EINVAL, "null argument");
  DynSet d{};
  for (int r = 0; r < gr->n; ++r) {
    if (n_gal[r] < 0 || n_ran[r] < 0 || n_gal[r] > gr->cap_g[r] || n_ran[r] > gr->cap_r[r])
      return fail(FRSD_ENOMEM, "catalogue sizes beyond the capacity the graph was captured with");
    if (!std::isfinite(alpha[r])) return fail(FRSD_EINVAL, "alpha must be finite");
    d.ng[r] = (double)n_gal[r];
    d.nr[r] = (double)n_ran[r];
    d.alpha[r] = alpha[r];
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_set_dyn_batch, dim3(gr->n), dim3(64), 0, s, ws_ptr<double>(gr->ws, gr->plan->L.dyn), d,
                     batch_of(gr->wss, gr->n));
  FRSD_LAUNCH_CHECK();
  FRSD_HIP(hipGraphLaunch(gr->exec, s));
  return FRSD_OK;
}
