// Internal declarations of the fastrsd HIP library (gfx950).
//
// Layout of the device workspace, the host-side plan, and the kernel launch
// wrappers shared by the translation units.  Nothing here is part of the
// C ABI in include/fastrsd.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/fastrsd.h"

namespace frsd {

// ---------------------------------------------------------------------------
// Moments.  The line-of-sight moments Q_ab = sum w xhat_a xhat_b and
// Q_abcd (Sec. II.B eqs. delta2b, delta4b) of a unit vector obey the trace
// relations sum_a Q_aa = Q_0 and sum_a Q_aabc = Q_bc, so 1 + 5 + 9 of the
// 1 + 6 + 15 components determine the rest:
//   Q_zz = Q_0 - Q_xx - Q_yy,
//   Q_zzxx = Q_xx - Q_xxxx - Q_xxyy,  Q_zzyy = Q_yy - Q_xxyy - Q_yyyy,
//   Q_zzzz = Q_zz - Q_zzxx - Q_zzyy,  Q_zzxy = Q_xy - Q_xxxy - Q_yyyx,
//   Q_zzzy = Q_yz - Q_xxyz - Q_yyyz,  Q_zzzx = Q_zx - Q_xxxz - Q_yyxz.
// Only the 15 kept components are gridded and transformed; the binning
// folds the eliminated ones into the coefficients of the kept ones
// (class_coeffs in device.h).  IDs: 0 the monopole; 1-5 xx yy xy yz zx;
// 6-14 xxxx yyyy xxxy xxxz yyyx yyyz xxyy xxyz yyxz; 15 the w^2-weighted
// monopole F_0^w (Sec. III.B, the definition below eq. SNbisp2).
// ---------------------------------------------------------------------------
constexpr int kMomRank2 = 6;   // moments of l_max = 2 (IDs 0-5)
constexpr int kMomRank4 = 15;  // moments of l_max = 4 (IDs 0-14)
constexpr int kMomW = 15;
constexpr int kMaxMom = 16;
constexpr int kMaxSlots = 16;

// ---------------------------------------------------------------------------
// FFT plan for one length: radix schedule (factors 8, 4, 2, 3).
// ---------------------------------------------------------------------------
struct FftLen {
  int n = 0;
  int nstage = 0;
  int radix[12] = {0};
};
bool make_fft_len(int n, FftLen *out);

// Device-visible kernel arguments describing the mesh planes.
struct SlotDesc {
  int n_slot;                 // complex meshes
  int re_mom[kMaxSlots];      // moment position (index into mom list) in the real part
  int im_mom[kMaxSlots];      // moment position in the imaginary part, -1 if empty
  int im_shift[kMaxSlots];    // 1: imaginary part is the interlaced twin (nodes at +1/2)
  int mom_id[kMaxMom];        // moment ID of each position
  int n_mom;
};

// Byte offsets of the workspace regions (all 256-byte aligned).
struct Layout {
  size_t tw_fwd = 0, tw_inv = 0, tw_inv64 = 0;  // twiddle tables
  size_t scal_part = 0, scal = 0, reject = 0;    // scalar reductions
  size_t cnt = 0, scan_blk = 0;                  // per-cell counts / offsets, scan partials
  size_t colmask = 0, xmask = 0;                 // occupied node columns (x, y) and x slabs (uint8)
  size_t colocc = 0;                             // cell columns (x, y) holding an object (uint8)
  size_t slot = 0, cellkey = 0;                  // per-object rank within its cell, cell id
  size_t sorted = 0;                             // sorted object records
  size_t mesh = 0;                               // n_slot complex N^3 meshes
  size_t planar = 0;                             // 2 n_slot real N^3 assignment planes
  size_t bin_part = 0, bin_sum = 0;              // shell-sum partials and totals
  size_t lowk = 0;                               // A_0, A_2, A_4 on |n| < top bk edge
  size_t buf1 = 0, buf2 = 0;                     // inverse-FFT intermediates
  size_t shells = 0;                             // shell fields on M^3
  size_t tri_tab = 0, tri_part = 0, tri_sum = 0; // contraction tables and partials
  size_t pair_tab = 0, tri_dense = 0;             // (b2, b3) of each row; dense sums of the MFMA path
  size_t pair_tab_nt = 0, tri_dense_nt = 0;       // the same for the N^T indicator sums
  size_t nt = 0;                                 // N^T per triangle
  size_t pk_lut = 0, bk_lut = 0;                 // |n|^2 -> bin index (int16, -1 outside)
  size_t bk_m2 = 0;                              // |n|^2 range of every bispectrum bin (int2)
  size_t bk_ctr = 0;                             // centre of every bispectrum bin, k_f units (double)
  size_t pair_tab_220 = 0, tri_sum220 = 0;       // pairs (F_2 b2, F_0 b3) and sums of T_220
  size_t tri_tab220 = 0;                         // vector-contraction outputs of T_220 (F_2 b1, F_2 b2, F_0 b3)
  size_t rcache = 0, rcache_sums = 0;            // cached random spectra (mesh layout) and their sums
  size_t dyn = 0;                                // {N_g, N_r, alpha} of graph replays (double)
  size_t acc = 0;                                // streamed plans: class-sum accumulators R_0, R_2, R_4
  size_t total = 0;
};

// Sorted object records: one record of four T per object, ordered by cell
// (x-major, z fastest): fx, fy, fz (fraction of the grid coordinate inside
// its cell, in [0, 1)) and t0 (the signed weight s w).  The w^2 weight of
// F_0^w is t0^2 and the line of sight is rebuilt from the position.
template <typename T> struct alignas(4 * sizeof(T)) Rec4 { T x, y, z, w; };
inline size_t sorted_bytes(size_t nobj, size_t tbytes) { return ((nobj * 4 * tbytes) + 255) & ~(size_t)255; }

constexpr int kBinSums = 8;     // per bin: count, sum|k|, then S00 S20 S40 S22 (P bins) or -, -, -, S0w S2w S4w (B bins)
constexpr int kScalars = 4;     // I22, N0, I33, W3
constexpr int kIngestBlocks = 1024;
constexpr int kBinBlocks = 2048;       // default of the tunable bin_blocks (tuning limits below)
constexpr int kTriBlocks = 1024;
constexpr int kTriMfmaBlocks = 1024;
constexpr int kPairBatch = 8;   // default shell-field pairs per inverse-FFT batch
constexpr int kStreamSlots = 2;  // default complex slots gridded and transformed per pass of a streamed plan
// Tunable launch parameters (frsd_plan_set_tuning); the workspace is sized for
// the largest values so that a plan can be retuned at any time.
constexpr int kMaxTriWg = 2048, kMaxRowGrid = 16384, kMaxBinBlocks = 4096, kMaxPairBatch = 16;

// Request batches (frsd_pk_batch): the forward FFT and the binning of up to
// kMaxBatch requests run as one launch each.  The requests' plans have one
// shape and so one workspace layout: a kernel takes request 0's pointers and
// adds delta[r], the byte distance from request 0's workspace to request r's,
// to those of the regions that belong to a request (constant tables are read
// from request 0's workspace).  A single request is a batch of one.
constexpr int kMaxBatch = FRSD_MAX_BATCH;
struct Batch {
  long long delta[kMaxBatch];
  int n;
};
inline Batch batch_one() {
  Batch b{};
  b.n = 1;
  return b;
}
inline Batch batch_of(void *const *ws, int n) {
  Batch b{};
  b.n = n;
  for (int r = 0; r < n; ++r) b.delta[r] = static_cast<char *>(ws[r]) - static_cast<char *>(ws[0]);
  return b;
}
// p moved by d bytes.  Byte-pointer arithmetic, not an integer round trip:
// the compiler then still knows a kernel argument moved this way points to
// global memory and keeps global (not flat) loads and stores.
template <typename P>
__host__ __device__ __forceinline__ P *moved(P *p, long long d) {
  using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P *>(reinterpret_cast<B *>(p) + d);
}
// the same for an optional region (a null p stays null)
template <typename P>
__host__ __device__ __forceinline__ P *shifted(P *p, long long d) {
  return p ? moved(p, d) : p;
}

// One constant table of a plan: bytes at host_off of the plan's host table
// image go to workspace offset ws_off.
struct TabSeg {
  size_t host_off, ws_off, bytes;
};

}  // namespace frsd

struct frsd_plan {
  frsd_params p{};
  frsd_tuning tune{frsd::kTriMfmaBlocks, 4096, frsd::kBinBlocks, frsd::kPairBatch, 0};
  int N = 0;
  double h = 0, kf = 0;
  frsd::SlotDesc slots{};
  // bins (squared edges in k_f units)
  std::vector<double> pk_e2, bk_e2;
  int nc_p = 0, nc_b = 0, nmax = 0;   // largest integer component inside the P / B spheres
  int pk_lut_len = 0, bk_lut_len = 0; // entries of the |n|^2 -> bin tables
  int M = 0;                          // real-space triangle-search grid
  int D = 0;                          // low-k cube side 2 nc_b + 1
  std::vector<int32_t> tri;           // 3 * ntri
  int64_t ntri = 0;
  int n_out = 0;                      // contraction outputs (ntri * n_ell)
  int n_ell = 0;                      // multipoles in the bispectrum (1, 2 or 3)
  int bk_ell = 0;                     // highest bispectrum multipole (0, 2 or 4)
  int n_wmom = 0;                     // w^2-weighted moments of the complete l > 0 shot noise (0, 6 or 15)
  frsd::FftLen fft_n, fft_m;
  frsd::Layout L;
  int state = 0;                      // 0 created, 1 initialised, 2 assigned, 3 pk done
  void *init_ws = nullptr;
  bool cache_ready = false;           // init_ws holds a random cache
  bool assigned_cached = false;       // the last assignment used the random cache
  int stream_slots = 0;               // streamed plans: complex slots resident per group
  bool mesh_live = false;             // the mesh region holds the last assignment's spectra
  double cached_alpha = 0;            // its alpha
  // Constant tables (twiddles, bin lookups, triangle and contraction tables),
  // built on the host once per plan and copied into a workspace at init.
  std::vector<unsigned char> tab_host;
  std::vector<frsd::TabSeg> tab_seg;
  bool tab_built = false;
  void *tab_pinned = nullptr;          // page-locked copy of tab_host: the uploads are asynchronous
  hipEvent_t tab_done = nullptr;       // recorded on the stream after the last upload from tab_pinned
  ~frsd_plan();
};

namespace frsd {

// error handling ------------------------------------------------------------
int fail(int code, const std::string &msg);
void clear_error();
// FRSD_EINVAL unless c is a valid catalogue (randoms need nbar)
int check_catalog(const frsd_catalog *c, bool need_nbar, const char *what);
// Device-visible copies of catalogues and output structs: page-locked host
// arrays (where = FRSD_HOST) replaced by their device pointers.
int device_view(const frsd_catalog *in, frsd_catalog *out);
int device_view(const frsd_pk_out *in, frsd_pk_out *out);
int device_view(const frsd_bk_out *in, frsd_bk_out *out);

#define FRSD_HIP(call)                                                       \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::frsd::fail(FRSD_EHIP, std::string(#call) + ": " +            \
                                         hipGetErrorString(e_));             \
  } while (0)

#define FRSD_LAUNCH_CHECK()                                                  \
  do {                                                                       \
    hipError_t e_ = hipGetLastError();                                       \
    if (e_ != hipSuccess)                                                    \
      return ::frsd::fail(FRSD_EHIP, std::string("kernel launch: ") +        \
                                         hipGetErrorString(e_));             \
  } while (0)

// Optional per-kernel timing (frsd_profile): events recorded on the launch
// stream around each wrapped launch.
bool prof_on();
class ProfScope {
 public:
  ProfScope(const char *name, hipStream_t s);
  ~ProfScope();

 private:
  const char *name_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};
#define FRSD_TIMED(name, stream, ...)          \
  do {                                         \
    ::frsd::ProfScope prof_scope_(name, stream); \
    __VA_ARGS__;                               \
  } while (0)

template <typename T>
inline T *ws_ptr(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// launch wrappers (defined in the .hip translation units) --------------------
// dyn (may be null): device {N_g, N_r, alpha} read by the ingest kernels in
// place of the catalogue sizes and alpha (graph replays)
template <typename T>
int run_mesh_assign(frsd_plan *pl, void *ws, const frsd_catalog *gal,
                    const frsd_catalog *ran, double alpha, hipStream_t s, const double *dyn = nullptr);
// cached: the meshes hold galaxies alone, combined here with the random cache
template <typename T>
int run_pk(frsd_plan *pl, void *ws, const frsd_pk_out *out, hipStream_t s, bool cached);
// Batches of n plans of one shape (frsd_pk_batch): per request the ingest,
// sort and assignment, then one forward FFT over every request's meshes
// (ran null: galaxies against each plan's random cache); one binning over
// every request's meshes, then each request's P_ell
// (dyn: request 0's {N_g, N_r, alpha}, each request's read from its own
// workspace, for graph replays)
template <typename T>
int run_mesh_assign_batch(frsd_plan *const *pl, void *const *ws, int n, const frsd_catalog *gal,
                          const frsd_catalog *ran, const double *alpha, hipStream_t s, const double *dyn = nullptr);
// Checks a batch (FRSD_E* before any device work) and fills the device views
// gd, rd (ran non-null) and od of its n requests.
int batch_views(frsd_plan *const *plans, void *const *workspaces, int n, const frsd_catalog *gal,
                const frsd_catalog *ran, const double *alpha, const frsd_pk_out *out, frsd_catalog *gd,
                frsd_catalog *rd, frsd_pk_out *od);
template <typename T>
int run_pk_batch(frsd_plan *const *pl, void *const *ws, int n, const frsd_pk_out *out, hipStream_t s, bool cached);
// streamed plans (stream.hip): moment groups accumulated into R_0, R_2, R_4
template <typename T>
int run_stream_assign(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                      hipStream_t s);
template <typename T>
int run_stream_pk(frsd_plan *pl, void *ws, const frsd_pk_out *out, hipStream_t s);
size_t stream_acc_bytes(const frsd_plan *pl, size_t tbytes);
// random cache (grid.hip): spectra of the randoms alone; galaxies against it
template <typename T>
int run_random_cache(frsd_plan *pl, void *ws, const frsd_catalog *ran, hipStream_t s);
template <typename T>
int run_mesh_assign_cached(frsd_plan *pl, void *ws, const frsd_catalog *gal, double alpha, hipStream_t s);
int run_bin_geometry(frsd_plan *pl, void *ws, hipStream_t s);
// complete l > 0 shot noise: w^2-weighted moments (grid.hip), their sums (pk.hip)
template <typename T>
int run_w_moments(frsd_plan *pl, void *ws, hipStream_t s);
template <typename T>
int run_bin_w(frsd_plan *pl, void *ws, hipStream_t s);
template <typename T>
int run_bk(frsd_plan *pl, void *ws, const frsd_bk_out *out, hipStream_t s);
int run_nt(frsd_plan *pl, void *ws, hipStream_t s);
// Host table image of the plan (once per plan), then its upload into ws on
// stream s: from page-locked memory (asynchronous; allocates it on the first
// call) or, with `pageable`, straight from the host image (no allocation).
int build_tables(frsd_plan *pl);
void tab_add(frsd_plan *pl, size_t ws_off, const void *src, size_t bytes);
int upload_tables(frsd_plan *pl, void *ws, hipStream_t s, bool pageable);

// FFT passes (fft.hip) --------------------------------------------------------
// Forward c2c FFT of n_batch N^3 complex meshes given as planar real arrays
// (re of mesh s = array 2s, im = array 2s+1); output interleaved complex.
// Node columns (x, y) with colmask 0 and x slabs with xmask 0 are zero in
// every mesh: they are read as zero, never from memory.  Only modes with
// |n|^2 <= m2max are guaranteed in the output.  With a batch of several
// requests, planar, mesh and the masks are request 0's (each request's
// n_batch meshes, masks from its own workspace).
template <typename T>
int fft3d_forward(const FftLen &f, const void *tw, const void *planar, void *mesh, int n_batch, int nmax, int m2max,
                  const uint8_t *colmask, const uint8_t *xmask, hipStream_t s, int row_grid,
                  const Batch &batch = batch_one());

// Triple-product contraction on the matrix cores (triple_mfma.hip).
bool triple_mfma_supported(const frsd_plan *pl);
bool triple_mfma_supported(const frsd_plan *pl, int ne);
size_t triple_mfma_part_bytes(const frsd_plan *pl, int nwg);
size_t triple_mfma_dense_bytes();
int triple_mfma(frsd_plan *pl, void *ws, const float *fields, hipStream_t s);
int triple_mfma64(frsd_plan *pl, void *ws, const double *fields, hipStream_t s);
int triple_mfma64_nt(frsd_plan *pl, void *ws, const double *indicators, hipStream_t s);
// T_220 = sum_x F_{2,b1} F_{2,b2} F_{0,b3} on the N^T job tiles (when those fit)
int triple_mfma_220(frsd_plan *pl, void *ws, const float *fields, hipStream_t s);
int triple_mfma64_220(frsd_plan *pl, void *ws, const double *fields, hipStream_t s);
void triple_mfma_tables_220(frsd_plan *pl);
// Job and pair tables of the contraction for ne column groups (n_ell for
// T_ell; 1 and for_nt for the N^T indicator sums), added to the plan's
// table image.
int triple_mfma_tables(frsd_plan *pl, int ne, bool for_nt);

// Shell-filtered inverse FFTs on the M^3 grid (bk.hip).
template <typename T>
int shell_fields(frsd_plan *pl, void *ws, bool indicators, hipStream_t s);

}  // namespace frsd
