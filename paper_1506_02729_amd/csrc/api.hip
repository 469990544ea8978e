// C ABI entry points (include/fastrsd.h): argument validation, call order,
// and dispatch to the FP32 or FP64 kernel instantiations.
#include <cstring>

#include "frsd_internal.h"

using namespace frsd;

static int check_ws(const frsd_plan *pl, const void *ws) {
  if (!pl) return fail(FRSD_EINVAL, "null plan");
  if (!ws) return fail(FRSD_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(FRSD_EINVAL, "workspace must be 256-byte aligned");
  return FRSD_OK;
}

static int host_to_device(void *p, int where, void **out) {
  *out = p;
  if (!p || where == FRSD_DEVICE) return FRSD_OK;
  if (where != FRSD_HOST) return fail(FRSD_EINVAL, "where must be FRSD_DEVICE or FRSD_HOST");
  void *d = nullptr;
  if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess || !d) {
    (void)hipGetLastError();
    return fail(FRSD_EINVAL, "a host array is not page-locked (allocate it with hipHostMalloc)");
  }
  *out = d;
  return FRSD_OK;
}

int frsd::device_view(const frsd_catalog *in, frsd_catalog *out) {
  *out = *in;
  if (in->n == 0) return FRSD_OK;
  int rc;
  void *d;
  if ((rc = host_to_device(const_cast<void *>(in->pos), in->where, &d))) return rc;
  out->pos = d;
  if ((rc = host_to_device(const_cast<void *>(in->w), in->where, &d))) return rc;
  out->w = d;
  if ((rc = host_to_device(const_cast<void *>(in->nbar), in->where, &d))) return rc;
  out->nbar = d;
  out->where = FRSD_DEVICE;
  return FRSD_OK;
}

int frsd::device_view(const frsd_pk_out *in, frsd_pk_out *out) {
  *out = *in;
  double **f[] = {&out->k_eff, &out->p0, &out->p2, &out->p4, &out->s00, &out->s20, &out->s40, &out->scalars,
                  &out->p4b, &out->s22};
  int rc;
  void *d;
  if ((rc = host_to_device(out->n_modes, in->where, &d))) return rc;
  out->n_modes = static_cast<int64_t *>(d);
  for (double **p : f) {
    if ((rc = host_to_device(*p, in->where, &d))) return rc;
    *p = static_cast<double *>(d);
  }
  out->where = FRSD_DEVICE;
  return FRSD_OK;
}

int frsd::device_view(const frsd_bk_out *in, frsd_bk_out *out) {
  *out = *in;
  double **f[] = {&out->nt, &out->t0, &out->t2, &out->t4, &out->b0, &out->b2, &out->b4, &out->sn0, &out->sn2,
                  &out->sn4, &out->t220, &out->b4za};
  int rc;
  void *d;
  for (double **p : f) {
    if ((rc = host_to_device(*p, in->where, &d))) return rc;
    *p = static_cast<double *>(d);
  }
  out->where = FRSD_DEVICE;
  return FRSD_OK;
}

int frsd::check_catalog(const frsd_catalog *c, bool need_nbar, const char *what) {
  if (!c) return fail(FRSD_EINVAL, std::string("null catalogue: ") + what);
  if (c->n < 0) return fail(FRSD_EINVAL, std::string("negative size: ") + what);
  if (c->n == 0) return FRSD_OK;
  if (c->dtype != FRSD_F32 && c->dtype != FRSD_F64) return fail(FRSD_EINVAL, std::string("dtype must be 32 or 64: ") + what);
  if (!c->pos || !c->w) return fail(FRSD_EINVAL, std::string("null pos or w: ") + what);
  if (need_nbar && !c->nbar) return fail(FRSD_EINVAL, std::string("randoms need nbar: ") + what);
  return FRSD_OK;
}

extern "C" int frsd_plan_init(frsd_plan *plan, void *ws, size_t ws_bytes, void *stream) {
  clear_error();
  int rc = check_ws(plan, ws);
  if (rc) return rc;
  if (ws_bytes < plan->L.total) return fail(FRSD_ENOMEM, "workspace smaller than frsd_plan_workspace_bytes");
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = upload_tables(plan, ws, s, false);
  if (rc) return rc;
  rc = run_bin_geometry(plan, ws, s);
  if (rc) return rc;
  if (plan->p.bk_nbins > 0) {
    rc = run_nt(plan, ws, s);
    if (rc) return rc;
  }
  plan->state = 1;
  plan->init_ws = ws;
  plan->cache_ready = false;
  plan->assigned_cached = false;
  plan->mesh_live = false;
  return FRSD_OK;
}

extern "C" int frsd_mesh_assign(frsd_plan *plan, void *ws, const frsd_catalog *gal, const frsd_catalog *ran,
                                double alpha, void *stream) {
  clear_error();
  int rc = check_ws(plan, ws);
  if (rc) return rc;
  if (plan->state < 1 || plan->init_ws != ws) return fail(FRSD_ESTATE, "workspace not initialised by frsd_plan_init");
  if ((rc = check_catalog(gal, false, "galaxies"))) return rc;
  if ((rc = check_catalog(ran, true, "randoms"))) return rc;
  if (!std::isfinite(alpha)) return fail(FRSD_EINVAL, "alpha must be finite");
  if (gal->n + ran->n > plan->p.max_objects)
    return fail(FRSD_ENOMEM, "galaxies + randoms exceed max_objects of the plan");
  if (gal->n + ran->n > (int64_t)0x7fffffff) return fail(FRSD_EINVAL, "more than 2^31-1 objects");
  frsd_catalog gd, rd;
  if ((rc = device_view(gal, &gd)) || (rc = device_view(ran, &rd))) return rc;
  gal = &gd;
  ran = &rd;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->p.stream_moments) {
    if (plan->p.precision == FRSD_F64) rc = run_stream_assign<double>(plan, ws, gal, ran, alpha, s);
    else rc = run_stream_assign<float>(plan, ws, gal, ran, alpha, s);
  } else if (plan->p.precision == FRSD_F64) {
    rc = run_mesh_assign<double>(plan, ws, gal, ran, alpha, s);
  } else {
    rc = run_mesh_assign<float>(plan, ws, gal, ran, alpha, s);
  }
  if (rc) return rc;
  plan->state = 2;
  plan->assigned_cached = false;
  plan->mesh_live = true;
  return FRSD_OK;
}

extern "C" int frsd_random_cache(frsd_plan *plan, void *ws, const frsd_catalog *ran, void *stream) {
  clear_error();
  int rc = check_ws(plan, ws);
  if (rc) return rc;
  if (!plan->p.random_cache) return fail(FRSD_EINVAL, "plan was created without random_cache");
  if (plan->state < 1 || plan->init_ws != ws) return fail(FRSD_ESTATE, "workspace not initialised by frsd_plan_init");
  if ((rc = check_catalog(ran, true, "randoms"))) return rc;
  if (ran->n > plan->p.max_objects) return fail(FRSD_ENOMEM, "randoms exceed max_objects of the plan");
  if (ran->n > (int64_t)0x7fffffff) return fail(FRSD_EINVAL, "more than 2^31-1 objects");
  frsd_catalog rd;
  if ((rc = device_view(ran, &rd))) return rc;
  ran = &rd;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->p.precision == FRSD_F64) rc = run_random_cache<double>(plan, ws, ran, s);
  else rc = run_random_cache<float>(plan, ws, ran, s);
  if (rc) return rc;
  plan->cache_ready = true;
  plan->state = 1;  // the mesh region holds no mock
  plan->mesh_live = false;
  return FRSD_OK;
}

extern "C" int frsd_mesh_assign_cached(frsd_plan *plan, void *ws, const frsd_catalog *gal, double alpha,
                                       void *stream) {
  clear_error();
  int rc = check_ws(plan, ws);
  if (rc) return rc;
  if (!plan->cache_ready || plan->init_ws != ws)
    return fail(FRSD_ESTATE, "frsd_mesh_assign_cached needs frsd_random_cache on this workspace first");
  if ((rc = check_catalog(gal, false, "galaxies"))) return rc;
  if (!std::isfinite(alpha)) return fail(FRSD_EINVAL, "alpha must be finite");
  if (gal->n > plan->p.max_objects) return fail(FRSD_ENOMEM, "galaxies exceed max_objects of the plan");
  if (gal->n > (int64_t)0x7fffffff) return fail(FRSD_EINVAL, "more than 2^31-1 objects");
  frsd_catalog gd;
  if ((rc = device_view(gal, &gd))) return rc;
  gal = &gd;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->p.precision == FRSD_F64) rc = run_mesh_assign_cached<double>(plan, ws, gal, alpha, s);
  else rc = run_mesh_assign_cached<float>(plan, ws, gal, alpha, s);
  if (rc) return rc;
  plan->state = 2;
  plan->mesh_live = true;
  plan->assigned_cached = true;
  plan->cached_alpha = alpha;
  return FRSD_OK;
}

extern "C" int frsd_pk_multipoles(frsd_plan *plan, void *ws, const frsd_pk_out *out, void *stream) {
  clear_error();
  int rc = check_ws(plan, ws);
  if (rc) return rc;
  if (plan->state < 2 || plan->init_ws != ws) return fail(FRSD_ESTATE, "frsd_pk_multipoles needs frsd_mesh_assign first");
  if (!plan->mesh_live)
    return fail(FRSD_ESTATE, "the meshes were overwritten by frsd_bk_multipoles: call frsd_mesh_assign again");
  if (!out || !out->n_modes || !out->k_eff || !out->p0 || !out->p2 || !out->p4 || !out->s00 || !out->s20 ||
      !out->s40 || !out->scalars)
    return fail(FRSD_EINVAL, "null output array");
  frsd_pk_out od;
  if ((rc = device_view(out, &od))) return rc;
  out = &od;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->p.stream_moments) rc = plan->p.precision == FRSD_F64 ? run_stream_pk<double>(plan, ws, out, s)
                                                                  : run_stream_pk<float>(plan, ws, out, s);
  else if (plan->p.precision == FRSD_F64) rc = run_pk<double>(plan, ws, out, s, plan->assigned_cached);
  else rc = run_pk<float>(plan, ws, out, s, plan->assigned_cached);
  if (rc) return rc;
  plan->state = 3;
  return FRSD_OK;
}

extern "C" int frsd_bk_multipoles(frsd_plan *plan, void *ws, const frsd_bk_out *out, void *stream) {
  clear_error();
  int rc = check_ws(plan, ws);
  if (rc) return rc;
  if (plan->p.bk_nbins == 0) return fail(FRSD_EINVAL, "plan has no bispectrum bins");
  if (plan->state < 3 || plan->init_ws != ws) return fail(FRSD_ESTATE, "frsd_bk_multipoles needs frsd_pk_multipoles first");
  if (!out || !out->nt || !out->t0 || !out->t2 || !out->t4 || !out->b0 || !out->b2 || !out->b4 || !out->sn0 ||
      !out->sn2 || !out->sn4)
    return fail(FRSD_EINVAL, "null output array");
  frsd_bk_out od;
  if ((rc = device_view(out, &od))) return rc;
  out = &od;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (plan->p.precision == FRSD_F64) rc = run_bk<double>(plan, ws, out, s);
  else rc = run_bk<float>(plan, ws, out, s);
  // the shell buffers (and the w^2-weighted moments) may take the mesh region
  if (plan->L.buf1 == plan->L.mesh || plan->n_wmom > 0) plan->mesh_live = false;
  return rc;
}

extern "C" int frsd_status(frsd_plan *plan, void *ws, int64_t *n_rejected, void *stream) {
  clear_error();
  int rc = check_ws(plan, ws);
  if (rc) return rc;
  if (!n_rejected) return fail(FRSD_EINVAL, "null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  FRSD_HIP(hipStreamSynchronize(s));
  unsigned long long v = 0;
  FRSD_HIP(hipMemcpy(&v, ws_ptr<void>(ws, plan->L.reject), sizeof(v), hipMemcpyDeviceToHost));
  *n_rejected = (int64_t)v;
  if (v) return fail(FRSD_EDOM, "objects outside [0, L)^3 or at the observer were rejected");
  return FRSD_OK;
}

// Plans of one shape: equal parameters, hence equal workspace layouts.
static bool same_params(const frsd_params &a, const frsd_params &b) {
  bool eq = a.n_grid == b.n_grid && a.order == b.order && a.interlace == b.interlace &&
            a.compensate == b.compensate && a.ell_max == b.ell_max && a.precision == b.precision &&
            a.box == b.box && a.pk_kmin == b.pk_kmin && a.pk_dk == b.pk_dk && a.pk_nbins == b.pk_nbins &&
            a.bk_kmin == b.bk_kmin && a.bk_dk == b.bk_dk && a.bk_nbins == b.bk_nbins && a.bk_grid == b.bk_grid &&
            a.max_objects == b.max_objects && a.bk_ell_max == b.bk_ell_max && a.bk_shot_noise == b.bk_shot_noise &&
            a.bk_zero_area == b.bk_zero_area && a.random_cache == b.random_cache &&
            a.stream_moments == b.stream_moments && a.stream_slots == b.stream_slots;
  for (int d = 0; d < 3; ++d) eq = eq && a.observer[d] == b.observer[d];
  return eq;
}

// Validation of a batch (every request before any device work) and the
// device views of its catalogues and outputs (ran null: no randoms).
int frsd::batch_views(frsd_plan *const *plans, void *const *workspaces, int n, const frsd_catalog *gal,
                      const frsd_catalog *ran, const double *alpha, const frsd_pk_out *out, frsd_catalog *gd,
                      frsd_catalog *rd, frsd_pk_out *od) {
  if (n < 1 || n > kMaxBatch) return fail(FRSD_EINVAL, "batch size must be 1..FRSD_MAX_BATCH");
  if (!plans || !workspaces || !gal || !alpha || !out) return fail(FRSD_EINVAL, "null argument");
  const bool cached = ran == nullptr;
  int rc;
  for (int r = 0; r < n; ++r) {
    if ((rc = check_ws(plans[r], workspaces[r]))) return rc;
    if (!same_params(plans[r]->p, plans[0]->p) || std::memcmp(&plans[r]->L, &plans[0]->L, sizeof(Layout)) != 0)
      return fail(FRSD_EINVAL, "the plans of a batch must have equal parameters");
    for (int q = 0; q < r; ++q)
      if (workspaces[q] == workspaces[r] || plans[q] == plans[r])
        return fail(FRSD_EINVAL, "a plan or workspace appears twice in the batch");
  }
  if (plans[0]->p.stream_moments) return fail(FRSD_EINVAL, "streamed plans are not batched");
  for (int r = 0; r < n; ++r) {
    frsd_plan *pl = plans[r];
    if (pl->state < 1 || pl->init_ws != workspaces[r])
      return fail(FRSD_ESTATE, "workspace not initialised by frsd_plan_init");
    if (cached && !pl->cache_ready)
      return fail(FRSD_ESTATE, "a batch without randoms needs frsd_random_cache on every workspace");
    if ((rc = check_catalog(&gal[r], false, "galaxies"))) return rc;
    if (!cached && (rc = check_catalog(&ran[r], true, "randoms"))) return rc;
    if (!std::isfinite(alpha[r])) return fail(FRSD_EINVAL, "alpha must be finite");
    const int64_t nobj = gal[r].n + (cached ? 0 : ran[r].n);
    if (nobj > pl->p.max_objects) return fail(FRSD_ENOMEM, "a catalogue exceeds max_objects of the plan");
    if (nobj > (int64_t)0x7fffffff) return fail(FRSD_EINVAL, "more than 2^31-1 objects");
    const frsd_pk_out &o = out[r];
    if (!o.n_modes || !o.k_eff || !o.p0 || !o.p2 || !o.p4 || !o.s00 || !o.s20 || !o.s40 || !o.scalars)
      return fail(FRSD_EINVAL, "null output array");
  }
  for (int r = 0; r < n; ++r) {
    if ((rc = device_view(&gal[r], &gd[r])) || (rc = device_view(&out[r], &od[r]))) return rc;
    if (!cached && (rc = device_view(&ran[r], &rd[r]))) return rc;
  }
  return FRSD_OK;
}

extern "C" int frsd_pk_batch(frsd_plan *const *plans, void *const *workspaces, int32_t n, const frsd_catalog *gal,
                             const frsd_catalog *ran, const double *alpha, const frsd_pk_out *out, void *stream) {
  clear_error();
  frsd_catalog gd[kMaxBatch], rd[kMaxBatch];
  frsd_pk_out od[kMaxBatch];
  int rc = batch_views(plans, workspaces, n, gal, ran, alpha, out, gd, rd, od);
  if (rc) return rc;
  const bool cached = ran == nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool f64 = plans[0]->p.precision == FRSD_F64;
  rc = f64 ? run_mesh_assign_batch<double>(plans, workspaces, n, gd, cached ? nullptr : rd, alpha, s)
           : run_mesh_assign_batch<float>(plans, workspaces, n, gd, cached ? nullptr : rd, alpha, s);
  if (rc) return rc;
  for (int r = 0; r < n; ++r) {
    plans[r]->state = 2;
    plans[r]->mesh_live = true;
    plans[r]->assigned_cached = cached;
    if (cached) plans[r]->cached_alpha = alpha[r];
  }
  rc = f64 ? run_pk_batch<double>(plans, workspaces, n, od, s, cached)
           : run_pk_batch<float>(plans, workspaces, n, od, s, cached);
  if (rc) return rc;
  for (int r = 0; r < n; ++r) plans[r]->state = 3;
  return FRSD_OK;
}
