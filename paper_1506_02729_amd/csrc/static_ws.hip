// The entry point that allocates nothing (frsd_run_static): one whole
// request on a static device scratch instead of a caller-provided
// workspace, for callers that cannot allocate device memory.
//
// `scratch` below is a file-scope device array; each device that runs the
// entry point holds its own copy until the process ends.  Its device address
// is fetched once per device (hipGetSymbolAddress, with that device current)
// and every kernel takes that address as its workspace; host code never
// passes the array's own name.
#include <cmath>
#include <mutex>
#include <string>

#include "frsd_internal.h"

namespace frsd {
constexpr size_t kScratchBytes = (size_t)128 << 20;  // 128 MiB per device
constexpr int kMaxDevices = 64;
}  // namespace frsd

static __device__ __align__(256) unsigned char scratch[frsd::kScratchBytes];

namespace frsd {
namespace {
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch (fetched on the first call
// on that device).
int scratch_address(void **out) {
  int dev = 0;
  FRSD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FRSD_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    FRSD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(FRSD_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return FRSD_OK;
}
}  // namespace
}  // namespace frsd

using namespace frsd;

extern "C" int frsd_run_static(frsd_plan *plan, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                               const frsd_pk_out *pk, const frsd_bk_out *bk, void *stream) {
  clear_error();
  if (!plan) return fail(FRSD_EINVAL, "null plan");
  if (plan->p.stream_moments || plan->p.random_cache)
    return fail(FRSD_EINVAL, "frsd_run_static takes plans without stream_moments and random_cache");
  if (plan->L.total > kScratchBytes)
    return fail(FRSD_ENOMEM, "the plan's workspace (" + std::to_string(plan->L.total) +
                                 " bytes) exceeds the static scratch (" + std::to_string(kScratchBytes) + " bytes)");
  int rc;
  if ((rc = check_catalog(gal, false, "galaxies"))) return rc;
  if ((rc = check_catalog(ran, true, "randoms"))) return rc;
  if (!std::isfinite(alpha)) return fail(FRSD_EINVAL, "alpha must be finite");
  if (gal->n + ran->n > plan->p.max_objects)
    return fail(FRSD_ENOMEM, "galaxies + randoms exceed max_objects of the plan");
  if (gal->n + ran->n > (int64_t)0x7fffffff) return fail(FRSD_EINVAL, "more than 2^31-1 objects");
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
  void *ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // Tables first (the scratch holds whatever the last call left): from the
  // plan's page-locked image if frsd_plan_init made one, else straight from
  // its host image; neither allocates.
  if ((rc = upload_tables(plan, ws, s, plan->tab_pinned == nullptr))) return rc;
  if ((rc = run_bin_geometry(plan, ws, s))) return rc;
  if (plan->p.bk_nbins > 0 && (rc = run_nt(plan, ws, s))) return rc;
  const bool f64 = plan->p.precision == FRSD_F64;
  if ((rc = f64 ? run_mesh_assign<double>(plan, ws, gal, ran, alpha, s)
                : run_mesh_assign<float>(plan, ws, gal, ran, alpha, s)))
    return rc;
  if ((rc = f64 ? run_pk<double>(plan, ws, pk, s, false) : run_pk<float>(plan, ws, pk, s, false))) return rc;
  if (do_bk && (rc = f64 ? run_bk<double>(plan, ws, bk, s) : run_bk<float>(plan, ws, bk, s))) return rc;
  return FRSD_OK;
}
