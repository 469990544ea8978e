// Host side of the library: parameter validation, bins, triangle list, FFT
// radix schedules, workspace layout and the thread-local error string.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "frsd_internal.h"

namespace frsd {

static thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}
void clear_error() { g_err.clear(); }
const char *last_error() { return g_err.c_str(); }

bool make_fft_len(int n, FftLen *out) {
  FftLen f{};
  f.n = n;
  int m = n;
  int ns = 0;
  while (m % 3 == 0) { f.radix[ns++] = 3; m /= 3; }
  while (m % 5 == 0) { f.radix[ns++] = 5; m /= 5; }
  while (m % 7 == 0) { f.radix[ns++] = 7; m /= 7; }
  while (m % 8 == 0) { f.radix[ns++] = 8; m /= 8; }
  if (m % 4 == 0) { f.radix[ns++] = 4; m /= 4; }
  if (m % 2 == 0) { f.radix[ns++] = 2; m /= 2; }
  if (m != 1 || ns > 12) return false;
  f.nstage = ns;
  *out = f;
  return true;
}

static bool is_smooth(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  while (n % 7 == 0) n /= 7;
  return n == 1;
}

static int smallest_smooth_at_least(int n) {
  for (int m = n;; ++m)
    if (is_smooth(m)) return m;
}

// squared edges in k_f units, snapped to integers within 1e-9 relative
static std::vector<double> squared_edges(double kmin, double dk, int nb, double kf) {
  std::vector<double> e2(nb + 1);
  for (int b = 0; b <= nb; ++b) {
    const double e = (kmin + dk * b) / kf;
    double v = e * e;
    const double r = std::nearbyint(v);
    if (std::fabs(v - r) <= 1e-9 * std::fmax(r, 1.0)) v = r;
    e2[b] = v;
  }
  return e2;
}

// largest integer strictly below sqrt(e2top)
static int max_component(double e2top) {
  int c = (int)std::floor(std::sqrt(e2top));
  while ((double)c * c >= e2top && c > 0) --c;
  while ((double)(c + 1) * (c + 1) < e2top) ++c;
  return c;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace frsd

using namespace frsd;

extern "C" const char *frsd_last_error(void) { return frsd::last_error(); }

extern "C" int frsd_plan_create(const frsd_params *params, frsd_plan **plan_out) {
  clear_error();
  if (!params || !plan_out) return fail(FRSD_EINVAL, "null argument");
  const frsd_params &p = *params;
  if (p.n_grid < 32 || p.n_grid > 1024 || p.n_grid % 16 != 0 || !is_smooth(p.n_grid))
    return fail(FRSD_EINVAL, "n_grid must be 2^a 3^b 5^c 7^d, a multiple of 16, in [32, 1024]");
  if (p.order < 1 || p.order > 4) return fail(FRSD_EINVAL, "order must be 1 (NGP), 2 (CIC), 3 (TSC) or 4 (PCS)");
  if (p.ell_max != 0 && p.ell_max != 2 && p.ell_max != 4) return fail(FRSD_EINVAL, "ell_max must be 0, 2 or 4");
  if (p.precision != FRSD_F32 && p.precision != FRSD_F64) return fail(FRSD_EINVAL, "precision must be 32 or 64");
  if (!(p.box > 0) || !std::isfinite(p.box)) return fail(FRSD_EINVAL, "box must be positive");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(p.observer[d])) return fail(FRSD_EINVAL, "observer must be finite");
  if (p.pk_nbins < 1 || !(p.pk_dk > 0) || p.pk_kmin < 0) return fail(FRSD_EINVAL, "invalid power-spectrum bins");
  if (p.bk_nbins < 0 || (p.bk_nbins > 0 && (!(p.bk_dk > 0) || p.bk_kmin < 0)))
    return fail(FRSD_EINVAL, "invalid bispectrum bins");
  if (p.max_objects < 0) return fail(FRSD_EINVAL, "max_objects must be >= 0");
  const int bk_ell = p.bk_ell_max < 0 ? p.ell_max : p.bk_ell_max;
  if (p.bk_ell_max < -1 || (bk_ell != 0 && bk_ell != 2 && bk_ell != 4) || bk_ell > p.ell_max)
    return fail(FRSD_EINVAL, "bk_ell_max must be -1, 0, 2 or 4 and at most ell_max");
  if (p.bk_shot_noise != 0 && p.bk_shot_noise != 1) return fail(FRSD_EINVAL, "bk_shot_noise must be 0 or 1");
  if (p.bk_zero_area != 0 && p.bk_zero_area != 1) return fail(FRSD_EINVAL, "bk_zero_area must be 0 or 1");
  if (p.bk_zero_area && bk_ell < 2) return fail(FRSD_EINVAL, "bk_zero_area needs the quadrupole (bk_ell_max >= 2)");
  if (p.random_cache != 0 && p.random_cache != 1) return fail(FRSD_EINVAL, "random_cache must be 0 or 1");
  if (p.random_cache && p.bk_shot_noise && p.bk_nbins > 0)
    return fail(FRSD_EINVAL, "random_cache does not combine with bk_shot_noise (its second pass grids every object)");
  if (p.stream_moments != 0 && p.stream_moments != 1) return fail(FRSD_EINVAL, "stream_moments must be 0 or 1");
  if (p.stream_moments && (p.bk_nbins > 0 || p.random_cache))
    return fail(FRSD_EINVAL, "stream_moments plans compute P_ell only (no bispectrum, no random cache)");
  if (p.stream_slots < 0 || (p.stream_slots != 0 && !p.stream_moments))
    return fail(FRSD_EINVAL, "stream_slots must be >= 0, and 0 unless stream_moments is set");

  frsd_plan *pl = new frsd_plan();
  pl->p = p;
  pl->N = p.n_grid;
  pl->h = p.box / p.n_grid;
  pl->kf = 2.0 * M_PI / p.box;
  const int N = pl->N;
  const double ny2 = (double)(N / 2) * (N / 2);

  pl->pk_e2 = squared_edges(p.pk_kmin, p.pk_dk, p.pk_nbins, pl->kf);
  if (pl->pk_e2.back() > ny2 * (1 + 1e-12)) { delete pl; return fail(FRSD_EINVAL, "pk k_max beyond Nyquist"); }
  if (pl->pk_e2.back() <= 1.0) { delete pl; return fail(FRSD_EINVAL, "pk bins contain no mode"); }
  pl->nc_p = max_component(pl->pk_e2.back());
  pl->nmax = pl->nc_p;
  if (p.bk_nbins > 0) {
    pl->bk_e2 = squared_edges(p.bk_kmin, p.bk_dk, p.bk_nbins, pl->kf);
    if (pl->bk_e2.back() > ny2 * (1 + 1e-12)) { delete pl; return fail(FRSD_EINVAL, "bk k_max beyond Nyquist"); }
    if (pl->bk_e2.back() <= 1.0) { delete pl; return fail(FRSD_EINVAL, "bk bins contain no mode"); }
    pl->nc_b = max_component(pl->bk_e2.back());
    if (pl->nc_b > pl->nmax) pl->nmax = pl->nc_b;
    pl->D = 2 * pl->nc_b + 1;
    const int need = 3 * pl->nc_b + 1;
    if (p.bk_grid) {
      if (p.bk_grid < need || !is_smooth(p.bk_grid) || p.bk_grid > 1024) {
        delete pl;
        return fail(FRSD_EINVAL, "bk_grid must be 2^a 3^b 5^c 7^d > 3 n_c and <= 1024");
      }
      pl->M = p.bk_grid;
    } else {
      pl->M = smallest_smooth_at_least(need);
    }
    if (pl->M > 1024) { delete pl; return fail(FRSD_EINVAL, "bispectrum grid would exceed 1024"); }
    // triangle list: b1 >= b2 >= b3 with lo(b1) < hi(b2) + hi(b3)
    std::vector<double> e(p.bk_nbins + 1);
    for (int b = 0; b <= p.bk_nbins; ++b) e[b] = std::sqrt(pl->bk_e2[b]);
    for (int b1 = 0; b1 < p.bk_nbins; ++b1)
      for (int b2 = 0; b2 <= b1; ++b2)
        for (int b3 = 0; b3 <= b2; ++b3)
          if (e[b1] < e[b2 + 1] + e[b3 + 1]) {
            pl->tri.push_back(b1); pl->tri.push_back(b2); pl->tri.push_back(b3);
          }
    pl->ntri = (int64_t)pl->tri.size() / 3;
    pl->bk_ell = bk_ell;
    pl->n_ell = bk_ell / 2 + 1;
    pl->n_out = (int)(pl->ntri * pl->n_ell);
    pl->n_wmom = (p.bk_shot_noise && bk_ell >= 2) ? (bk_ell == 2 ? kMomRank2 : kMomRank4) : 0;
  }

  // moments in slot order, and their packing into complex meshes
  SlotDesc &sd = pl->slots;
  int nm = 0;
  const int nmom_ell = p.ell_max == 0 ? 1 : (p.ell_max == 2 ? kMomRank2 : kMomRank4);
  for (int m = 0; m < nmom_ell; ++m) sd.mom_id[nm++] = m;
  if (p.bk_nbins > 0) sd.mom_id[nm++] = kMomW;
  sd.n_mom = nm;
  int ns = 0;
  if (p.interlace) {
    for (int m = 0; m < nm; ++m) {
      sd.re_mom[ns] = m; sd.im_mom[ns] = m; sd.im_shift[ns] = 1; ++ns;
    }
  } else {
    for (int m = 0; m < nm; m += 2) {
      sd.re_mom[ns] = m; sd.im_mom[ns] = (m + 1 < nm) ? m + 1 : -1; sd.im_shift[ns] = 0; ++ns;
    }
  }
  sd.n_slot = ns;

  if (!make_fft_len(N, &pl->fft_n)) { delete pl; return fail(FRSD_EINVAL, "no radix schedule for n_grid"); }
  if (pl->M && !make_fft_len(pl->M, &pl->fft_m)) { delete pl; return fail(FRSD_EINVAL, "no radix schedule for M"); }

  // workspace layout
  const size_t T = (p.precision == FRSD_F64) ? 8 : 4;
  const size_t NNN = (size_t)N * N * N;
  const size_t nobj = (size_t)(p.max_objects > 0 ? p.max_objects : 1);
  Layout &L = pl->L;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.tw_fwd = take(2 * T * N);
  L.tw_inv = take(2 * T * (pl->M ? pl->M : 1));
  L.tw_inv64 = take(16 * (size_t)(pl->M ? pl->M : 1));
  L.scal_part = take(8 * 6 * kIngestBlocks);
  L.scal = take(8 * 16);
  L.reject = take(8);
  L.dyn = take(8 * 4);
  L.cnt = take(4 * (2 * NNN + 1));  // half-cell counts / offsets
  L.scan_blk = take(4 * ((2 * NNN + 1 + 4095) / 4096 + 1));
  L.colmask = take((size_t)N * N);
  L.xmask = take((size_t)N);
  L.colocc = take((size_t)N * N);
  L.slot = take(4 * nobj);
  L.cellkey = take(4 * nobj);
  L.sorted = take(sorted_bytes(nobj, T));
  pl->stream_slots = p.stream_moments ? std::min(p.stream_slots > 0 ? p.stream_slots : kStreamSlots, sd.n_slot) : 0;
  const size_t slots_resident = p.stream_moments ? (size_t)pl->stream_slots : (size_t)sd.n_slot;
  // the complex meshes and the assignment planes are adjacent: together they
  // are the scratch region of the bispectrum call (below)
  L.mesh = take(2 * T * NNN * slots_resident);
  L.planar = take(2 * T * NNN * slots_resident);
  const size_t scratch_end = off;
  if (p.stream_moments) L.acc = take(stream_acc_bytes(pl, T));
  if (p.random_cache) {
    L.rcache = take(2 * T * NNN * sd.n_slot);
    L.rcache_sums = take(8 * 4);
  }
  const int nbins_all = p.pk_nbins + p.bk_nbins;
  L.bin_part = take(8 * (size_t)kBinSums * nbins_all * kMaxBinBlocks);
  L.bin_sum = take(8 * (size_t)kBinSums * nbins_all);
  if (p.bk_nbins > 0) {
    const size_t D = pl->D, M = pl->M;
    const size_t npair_batch = kMaxPairBatch;
    L.lowk = take(2 * T * 3 * D * D * D);
    // intermediates sized for FP64 (the N^T indicator fields are FP64 for every plan)
    const size_t buf1_bytes = 16 * npair_batch * D * D * M, buf2_bytes = 16 * npair_batch * D * M * M;
    const size_t nfield = (size_t)pl->n_ell * p.bk_nbins;
    const size_t shell_bytes = std::max(T * nfield, (size_t)8 * p.bk_nbins) * M * M * M;
    // The assignment planes are dead after the first FFT pass and the
    // complex meshes after the binning of frsd_pk_multipoles (the bispectrum
    // reads the low-k cube); the shell intermediates and fields live only
    // inside one bispectrum call (and plan init).  Calls on a workspace are
    // ordered on one stream, so the shell buffers take the mesh and planar
    // regions when they fit in them (frsd_pk_multipoles then needs a new
    // frsd_mesh_assign).
    if (align256(buf1_bytes) + align256(buf2_bytes) + align256(shell_bytes) <= scratch_end - L.mesh) {
      L.buf1 = L.mesh;
      L.buf2 = L.buf1 + align256(buf1_bytes);
      L.shells = L.buf2 + align256(buf2_bytes);
    } else {
      L.buf1 = take(buf1_bytes);
      L.buf2 = take(buf2_bytes);
      L.shells = take(shell_bytes);
    }
    L.tri_tab = take(16 * (size_t)pl->n_out + 16 * (size_t)pl->ntri + 12 * (size_t)pl->ntri);
    // contraction partials: the vector contraction's (per output and
    // workgroup) only for the sums that do not fit the matrix-core tables
    size_t vec_part = 0;
    if (!triple_mfma_supported(pl)) vec_part = std::max(vec_part, 8 * (size_t)pl->n_out * kTriBlocks);
    if (!triple_mfma_supported(pl, 1)) vec_part = std::max(vec_part, 8 * (size_t)pl->ntri * kTriBlocks);
    L.tri_part = take(std::max(vec_part, triple_mfma_part_bytes(pl, kMaxTriWg)));
    L.pair_tab = take(8 * (size_t)p.bk_nbins * (p.bk_nbins + 1) / 2);
    L.tri_dense = take(triple_mfma_dense_bytes());
    L.pair_tab_nt = take(8 * (size_t)p.bk_nbins * (p.bk_nbins + 1) / 2);
    L.tri_dense_nt = take(triple_mfma_dense_bytes());
    L.tri_sum = take(8 * (size_t)std::max(pl->n_out, (int)pl->ntri));
    L.nt = take(8 * (size_t)pl->ntri);
    L.bk_ctr = take(8 * (size_t)p.bk_nbins);
    if (p.bk_zero_area) {
      L.pair_tab_220 = take(8 * (size_t)p.bk_nbins * (p.bk_nbins + 1) / 2);
      L.tri_sum220 = take(8 * (size_t)pl->ntri);
      L.tri_tab220 = take(16 * (size_t)pl->ntri);
    }
  }
  // bin lookup tables |n|^2 -> bin (int16)
  pl->pk_lut_len = (int)std::ceil(pl->pk_e2.back());
  L.pk_lut = take(2 * (size_t)pl->pk_lut_len);
  if (p.bk_nbins > 0) {
    pl->bk_lut_len = (int)std::ceil(pl->bk_e2.back());
    L.bk_lut = take(2 * (size_t)pl->bk_lut_len);
    L.bk_m2 = take(8 * (size_t)p.bk_nbins);
  }
  L.total = off;
  *plan_out = pl;
  return FRSD_OK;
}

// The page-locked table image may still be the source of uploads queued by
// frsd_plan_init: wait for them before it is freed.
frsd_plan::~frsd_plan() {
  if (tab_done) {
    (void)hipEventSynchronize(tab_done);
    (void)hipEventDestroy(tab_done);
  }
  if (tab_pinned) (void)hipHostFree(tab_pinned);
}

extern "C" void frsd_plan_destroy(frsd_plan *plan) { delete plan; }

extern "C" int frsd_plan_workspace_bytes(const frsd_plan *plan, size_t *bytes) {
  clear_error();
  if (!plan || !bytes) return fail(FRSD_EINVAL, "null argument");
  *bytes = plan->L.total;
  return FRSD_OK;
}

extern "C" int frsd_bk_ntriangles(const frsd_plan *plan, int64_t *ntri) {
  clear_error();
  if (!plan || !ntri) return fail(FRSD_EINVAL, "null argument");
  *ntri = plan->ntri;
  return FRSD_OK;
}

extern "C" int frsd_plan_set_tuning(frsd_plan *plan, const frsd_tuning *t) {
  clear_error();
  if (!plan || !t) return fail(FRSD_EINVAL, "null argument");
  if (t->tri_wg < 256 || t->tri_wg > kMaxTriWg || t->row_grid < 256 || t->row_grid > kMaxRowGrid ||
      t->bin_blocks < 256 || t->bin_blocks > kMaxBinBlocks || t->pair_batch < 1 || t->pair_batch > kMaxPairBatch ||
      (t->sweep_x != 0 && t->sweep_x != 16 && t->sweep_x != 32 && t->sweep_x != 64))
    return fail(FRSD_EINVAL, "tuning value out of range");
  plan->tune = *t;
  return FRSD_OK;
}

extern "C" int frsd_plan_get_tuning(const frsd_plan *plan, frsd_tuning *t) {
  clear_error();
  if (!plan || !t) return fail(FRSD_EINVAL, "null argument");
  *t = plan->tune;
  return FRSD_OK;
}

extern "C" int frsd_bk_grid(const frsd_plan *plan, int32_t *m) {
  clear_error();
  if (!plan || !m) return fail(FRSD_EINVAL, "null argument");
  *m = plan->M;
  return FRSD_OK;
}

extern "C" int frsd_bk_triangles(const frsd_plan *plan, int32_t *b123) {
  clear_error();
  if (!plan || (!b123 && plan->ntri > 0)) return fail(FRSD_EINVAL, "null argument");
  if (plan->ntri > 0) std::memcpy(b123, plan->tri.data(), sizeof(int32_t) * plan->tri.size());
  return FRSD_OK;
}
