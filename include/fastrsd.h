/*
 * fastrsd -- FFT multipole estimators for redshift-space clustering on
 * AMD Instinct MI355X (gfx950).
 *
 * Implements the power-spectrum and bispectrum multipole estimators of
 * R. Scoccimarro, "Fast Estimators for Redshift-Space Clustering",
 * arXiv:1506.02729:
 *
 *   F_0(k)   = (sum_g - alpha sum_r) w_j exp(i k.x_j)               Sec. III.A eq. (F0)
 *   Q^{ab}   = (sum_g - alpha sum_r) xhat^a xhat^b w_j exp(i k.x_j)  Sec. III.A eq. (Qab)
 *   F_2      = 3/2 khat_a khat_b Q^{ab} - 1/2 F_0                    Sec. III.A eq. (F2)
 *   F_4      = 35/8 khat^4 Q^{abcd} - 5/2 F_2 - 7/8 F_0              Sec. II.B eqs. (delta4),(delta4b)
 *   P_ell    = (2 ell + 1) <F_ell F_0^*>_shell / I22  (- N_0 for ell=0)  Sec. III.A eqs. (P0_impl)-(P4_impl)
 *   B_ell    = (2 ell + 1) <F_ell F_0 F_0>_T / (N^T I33) - N^(ell)   Sec. III.B eqs. (BispMono),(BispQuad)
 *
 * with the triangle sum done by shell-filtered inverse FFTs and a grid sum
 * of triple products (Sec. III.B eqs. (Factorize),(F_k)).
 *
 * Conventions shared by every call:
 *  - Positions are in the box frame [0, L)^3 (Mpc/h).  An object outside the
 *    box, or exactly at the observer, is rejected: it contributes nothing and
 *    is counted (see frsd_status), never wrapped.
 *  - Integer wave-vectors n use the fftfreq convention; k = (2 pi / L) n.
 *  - A bin b covers [kmin + b dk, kmin + (b+1) dk); membership is decided on
 *    the integer |n|^2 against squared edges in units of k_f = 2 pi / L,
 *    snapped to the nearest integer when within 1e-9 relative.  DC is never
 *    binned.  Mode counts are over the full grid (n and -n both counted).
 *  - All device memory is owned by the caller.  The library never allocates
 *    device memory: every call works inside the caller's workspace `ws`
 *    (device pointer, 256-byte aligned, at least frsd_plan_workspace_bytes).
 *    Catalogues and outputs may also be page-locked host memory (`where`).
 *  - `stream` is a hipStream_t passed as void*.  Device calls only enqueue
 *    work on it and return; results are valid once the stream is
 *    synchronised.  Calls on one workspace must be ordered on one stream.
 *  - Every call returns FRSD_OK (0) or a negative error code, and then
 *    frsd_last_error() describes the failure (thread-local).  No call
 *    throws or exits.
 */
#ifndef FASTRSD_H
#define FASTRSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FRSD_OK = 0,
  FRSD_EINVAL = -1,  /* invalid parameter, size or pointer              */
  FRSD_EDOM = -2,    /* objects outside the box or at the observer       */
  FRSD_ENOMEM = -3,  /* workspace or catalogue capacity too small        */
  FRSD_EHIP = -4,    /* a HIP runtime call failed                        */
  FRSD_ESTATE = -5   /* calls out of order (e.g. bk before pk)           */
};

enum { FRSD_F32 = 32, FRSD_F64 = 64 };
enum { FRSD_DEVICE = 0, FRSD_HOST = 1 };  /* where an array lives */
#define FRSD_MAX_BATCH 16  /* requests of one frsd_pk_batch call */

typedef struct frsd_plan frsd_plan;

/* Estimator parameters (host struct, copied by frsd_plan_create). */
typedef struct {
  int32_t n_grid;      /* N, FFT mesh side: 2^a 3^b 5^c 7^d, multiple of 16, 32..1024 */
  int32_t order;       /* mass assignment order p: 1 NGP, 2 CIC, 3 TSC, 4 PCS          */
  int32_t interlace;   /* 1: interlaced twin grid at half-cell offset (Sec. III.A)    */
  int32_t compensate;  /* 1: divide by prod_d sinc(pi n_d / N)^p                      */
  int32_t ell_max;     /* 0, 2 or 4: multipoles computed (1, 6 or 15 moment meshes:
                          the 1, 7 or 22 moments of Sec. II.B less those fixed by the
                          trace relations of a unit line of sight)                  */
  int32_t precision;   /* FRSD_F32 (served) or FRSD_F64 (plain) arithmetic            */
  double box;          /* L, box side (Mpc/h)                                         */
  double observer[3];  /* observer position in the box frame (may lie outside)        */
  double pk_kmin, pk_dk; /* power-spectrum bins (h/Mpc); top edge <= k_Nyquist        */
  int32_t pk_nbins;      /* >= 1                                                      */
  double bk_kmin, bk_dk; /* bispectrum bins (h/Mpc); top edge <= k_Nyquist            */
  int32_t bk_nbins;      /* 0: no bispectrum                                          */
  int32_t bk_grid;       /* M, real-space grid of the triangle search; 0: smallest
                            2^a 3^b 5^c 7^d with M > 3 n_c (n_c = largest integer below the
                            top bispectrum edge in k_f units), which makes the grid
                            sum equal to the exact closed-triangle sum              */
  int64_t max_objects;   /* capacity: galaxies + randoms per frsd_mesh_assign call    */
  int32_t bk_ell_max;    /* bispectrum multipoles: 0, 2 or 4 (<= ell_max); -1: ell_max */
  int32_t bk_shot_noise; /* l > 0 shot noise of eq. (SNbisp2thin): 0 its q1 term only;
                            1 complete, with the w^2-weighted multipoles F^w_2, F^w_4
                            (the moment meshes gridded again with weight w^2 inside
                            frsd_bk_multipoles, transformed to the bispectrum sphere) */
  int32_t bk_zero_area;  /* 1: also T_220 and the zero-area hexadecapole B4za of
                            Sec. II.C eq. (Bhexa2) (needs bk_ell_max >= 2)          */
  int32_t random_cache;  /* 1: the workspace also holds the Fourier moment meshes of
                            one random catalogue (frsd_random_cache), so that mocks
                            sharing it run frsd_mesh_assign_cached on their galaxies
                            alone (not with bk_shot_noise = 1)                      */
  int32_t stream_moments;/* 1: P_ell only, for meshes whose moment meshes do not fit at
                            once (N = 1024): the moments are gridded, transformed and
                            accumulated into A_0, A_2, A_4 stream_slots complex slots
                            at a time (no bispectrum, no random cache)              */
  int32_t stream_slots;  /* streamed plans: complex slots resident at once, each
                            4 T N^3 bytes (T = 4 or 8: the complex mesh and its two
                            assignment planes); 0: 2; values above the number of
                            slots are clamped to it.  Must be 0 without stream_moments */
} frsd_params;

/* A catalogue.  pos is n x 3 interleaved (x, y, z); w and nbar have n
 * entries.  nbar may be NULL for galaxies (it only enters I22 and I33
 * through the randoms).  dtype is FRSD_F32 or FRSD_F64 and applies to all
 * three arrays.  where: FRSD_DEVICE (device memory) or FRSD_HOST
 * (page-locked host memory from hipHostMalloc, read by the ingest kernels
 * over the host link, twice per call; other host memory gives FRSD_EINVAL). */
typedef struct {
  const void *pos;
  const void *w;
  const void *nbar;
  int64_t n;
  int32_t dtype;
  int32_t where;
} frsd_catalog;

/* Power-spectrum outputs: caller-owned arrays of pk_nbins entries (scalars:
 * 4 entries), in device memory or, with where = FRSD_HOST, in page-locked
 * host memory (written by the kernels over the host link).  Written by
 * frsd_pk_multipoles. */
typedef struct {
  int64_t *n_modes;  /* N_b, full-grid mode count                                  */
  double *k_eff;     /* mean |k| over the modes of the bin                          */
  double *p0, *p2, *p4;   /* P_ell of eqs. (P0_impl)-(P4_impl); NaN if I22 == 0   */
  double *s00, *s20, *s40; /* raw shell sums sum_b Re[F_ell F_0^*]                */
  double *scalars;   /* [I22, N_0, I33, W3]: I22 = alpha sum_r nbar w^2 (eq. I22def),
                        N_0 = (sum_g + alpha^2 sum_r) w^2 (eq. N0true),
                        I33 = alpha sum_r nbar^2 w^3, W3 = (sum_g - alpha^3 sum_r) w^3 */
  double *p4b;       /* optional (NULL: not written).  Split hexadecapole of Sec. II.B
                        eqs. (factorizeL4), (split), (P4fast): (35/2 S22 - 5 S20 -
                        7/2 S00) / (N_b I22) with the raw S00; needs ell_max >= 2 only
                        (the quadrupole's moments), NaN for ell_max 0                */
  double *s22;       /* optional (NULL: not written).  Raw sum_b |F_2|^2              */
  int32_t where;     /* FRSD_DEVICE or FRSD_HOST, for every array above               */
} frsd_pk_out;

/* Bispectrum outputs: caller-owned arrays of ntri entries, one per triangle
 * of frsd_bk_triangles (in that order), in device memory or (where =
 * FRSD_HOST) page-locked host memory. */
typedef struct {
  double *nt;             /* N^T, exact count of closed lattice triangles (eq. NT)  */
  double *t0, *t2, *t4;   /* raw triangle sums sum_T Re F_ell(q1) F_0(q2) F_0(q3)   */
  double *b0, *b2, *b4;   /* (2 ell + 1) T_ell / (N^T I33); NaN when N^T == 0        */
  double *sn0, *sn2, *sn4;/* thin-shell shot noise (eq. SNbisp2thin), N^(ell): sn0
                             complete; sn2/sn4 complete with bk_shot_noise = 1, else
                             the q1 term (2l+1) S_lw(b1)/(N_b1 I33).  The cosines
                             qhat1.qhat_i come from the law of cosines at the bin
                             centres (clamped to [-1, 1]).  B_ell = b_ell - sn_ell;
                             NaN for ell > bk_ell_max                               */
  double *t220;           /* optional (bk_zero_area): sum_T Re F_2(q1) F_2(q2) F_0(q3) */
  double *b4za;           /* optional (bk_zero_area): (35/2 T_220 - 5 T_2 - 7/2 T_0) /
                             (N^T I33), eq. (Bhexa2), no shot noise subtracted      */
  int32_t where;          /* FRSD_DEVICE or FRSD_HOST, for every array above        */
} frsd_bk_out;

/* Launch parameters chosen by the autotuner (paper_1506_02729_amd/autotune.py,
 * cached as JSON per plan shape); any value in range gives the same results
 * up to rounding order.  frsd_plan_set_tuning may be called at any time
 * between requests (the workspace is sized for the largest values);
 * FRSD_EINVAL outside the ranges. */
typedef struct {
  int32_t tri_wg;      /* workgroups of the matrix-core contraction, 256..2048 (1024)      */
  int32_t row_grid;    /* workgroups of the persistent forward z pass, 256..16384 (4096)   */
  int32_t bin_blocks;  /* workgroups of the binning kernel, 256..4096 (2048)               */
  int32_t pair_batch;  /* shell-field pairs per inverse-FFT launch, 1..16 (8)              */
  int32_t sweep_x;     /* x nodes per workgroup of the x-sweep assignment: 16, 32 or 64;
                          0 (default): 16, or 64 for streamed plans                    */
} frsd_tuning;
int frsd_plan_set_tuning(frsd_plan *plan, const frsd_tuning *tuning);
int frsd_plan_get_tuning(const frsd_plan *plan, frsd_tuning *tuning);

/* Validates parameters and builds the host-side plan: bins, triangle list,
 * FFT radix schedules and the workspace layout.  Host only. */
int frsd_plan_create(const frsd_params *params, frsd_plan **plan);
void frsd_plan_destroy(frsd_plan *plan);

/* Exact device workspace size for this plan (bytes). */
int frsd_plan_workspace_bytes(const frsd_plan *plan, size_t *bytes);

/* Uploads tables into ws and, with a bispectrum, computes N^T for every
 * listed triangle (FP64, exact to rounding).  Required once per workspace
 * before any other device call.  Asynchronous on `stream`. */
int frsd_plan_init(frsd_plan *plan, void *ws, size_t ws_bytes, void *stream);

/* Steps a1-a4: line of sight, sort by cell, interlaced B-spline assignment
 * of the moment meshes (weights w, w xhat_i xhat_j, w xhat_i xhat_j xhat_k
 * xhat_l and, with a bispectrum, the w^2 mesh of F_0^w) and their forward
 * FFTs (Sec. III.A eq. (mapFFT)).  Galaxies enter with sign +1, randoms
 * with -alpha; ran may have n == 0.  alpha is explicit (the paper's
 * N_g / N_r is the usual choice).  Also reduces I22, N_0, I33, W3.
 * FRSD_ENOMEM if gal->n + ran->n > max_objects. */
int frsd_mesh_assign(frsd_plan *plan, void *ws, const frsd_catalog *gal,
                     const frsd_catalog *ran, double alpha, void *stream);

/* Random-catalogue cache, for many mocks over one survey mask (the paper
 * caches what depends only on the mask and grid, Sec. III.B; its randoms
 * dominate the assignment time, Sec. III.C).  Needs a plan with
 * random_cache = 1.  frsd_random_cache grids ran alone (weight +w for the
 * moments, w^2 for F_0^w), transforms it and keeps the spectra and the
 * randoms' sums of nbar w^2, nbar^2 w^3, w^2, w^3 in ws.
 * frsd_mesh_assign_cached then runs steps a1-a4 on the galaxies alone; the
 * following frsd_pk_multipoles combines every mesh as F = F_gal - alpha
 * F_ran (F_0^w: + alpha^2 F_ran^w), and I22, N_0, I33, W3 use the cached
 * sums: the results are those of frsd_mesh_assign(gal, ran, alpha) up to
 * rounding.  The cache stays valid until frsd_random_cache is called again
 * or the workspace is initialised again.  Rejected randoms are counted by
 * frsd_status after frsd_random_cache.  Asynchronous on `stream`. */
int frsd_random_cache(frsd_plan *plan, void *ws, const frsd_catalog *ran, void *stream);
int frsd_mesh_assign_cached(frsd_plan *plan, void *ws, const frsd_catalog *gal, double alpha, void *stream);

/* Steps a5-a6: multipole combination and shell binning into P_0, P_2, P_4.
 * Requires a preceding frsd_mesh_assign (or frsd_mesh_assign_cached) on ws
 * and no frsd_bk_multipoles since then (FRSD_ESTATE otherwise).  Also
 * extracts the low-k multipole fields that frsd_bk_multipoles uses. */
int frsd_pk_multipoles(frsd_plan *plan, void *ws, const frsd_pk_out *out, void *stream);

/* Steps a1-a6 for a batch of n requests of one shape, the many-mock case of
 * the paper's covariance use (Sec. III.C): plans[r] and workspaces[r] are n
 * plans created with equal frsd_params, each initialised on its own
 * workspace (distinct).  Request r is frsd_mesh_assign(gal[r], ran[r],
 * alpha[r]) followed by frsd_pk_multipoles into out[r] (Sec. III.A eqs.
 * (mapFFT), (P0_impl)-(P4_impl)), and every kernel of those steps (ingest,
 * sort, assignment, each forward FFT pass, binning) is ONE launch over all n
 * requests, so that small meshes share launches that fill the device
 * (catalogues of one role that differ in dtype are ingested one request at a
 * time).  ran == NULL: every plan holds a random
 * cache (frsd_random_cache) and the galaxies are assigned against it, as
 * frsd_mesh_assign_cached.  gal, ran, alpha and out are host arrays of n
 * entries.  Results equal those of n calls of frsd_mesh_assign (or
 * frsd_mesh_assign_cached) and frsd_pk_multipoles up to rounding order, and
 * leave every plan in the same state as that sequence (frsd_bk_multipoles
 * and frsd_status may follow per plan).  FRSD_EINVAL: n outside
 * 1..FRSD_MAX_BATCH, a null pointer, plans whose parameters differ, a
 * streamed plan, a workspace given twice; FRSD_ESTATE: a workspace not
 * initialised by its plan, or without a random cache when ran is NULL;
 * FRSD_ENOMEM: a catalogue beyond max_objects.  Validation covers every
 * request before any device work.  Asynchronous on `stream`. */
int frsd_pk_batch(frsd_plan *const *plans, void *const *workspaces, int32_t n, const frsd_catalog *gal,
                  const frsd_catalog *ran, const double *alpha, const frsd_pk_out *out, void *stream);

/* Number of listed triangles and the list itself (host array of 3*ntri
 * int32: b1 >= b2 >= b3 with lo(b1) < hi(b2) + hi(b3), lexicographic). */
int frsd_bk_ntriangles(const frsd_plan *plan, int64_t *ntri);
int frsd_bk_triangles(const frsd_plan *plan, int32_t *b123);

/* Side M of the real-space grid of the triangle search (Sec. III.B eqs.
 * (Factorize),(F_k)): params.bk_grid, or the smallest 2^a 3^b 5^c 7^d above
 * 3 n_c; 0 without bispectrum.  FRSD_EINVAL on a null argument. */
int frsd_bk_grid(const frsd_plan *plan, int32_t *m);

/* Steps a7-a9: shell-filtered inverse FFTs of F_0, F_2, F_4 on the M^3 grid,
 * triple-product contraction over all listed triangles and normalisation
 * (Sec. III.B).  Requires a preceding frsd_pk_multipoles on ws.  Its shell
 * buffers reuse the workspace's mesh region, so the next
 * frsd_pk_multipoles needs a new assignment; it may be called again on
 * the same assignment. */
int frsd_bk_multipoles(frsd_plan *plan, void *ws, const frsd_bk_out *out, void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid allocation): one whole
 * request -- the plan's tables and N^T, then the steps of frsd_mesh_assign,
 * frsd_pk_multipoles and, when bk is non-NULL and the plan has bispectrum
 * bins, frsd_bk_multipoles -- with the library's static device scratch as
 * the workspace instead of a caller-provided one.  Same arguments, outputs
 * and results as that sequence; the caller passes the catalogues and the
 * output arrays only.  Allocates nothing: no hipMalloc, hipFree or
 * page-locked allocation (tables are copied from the plan's host image, or
 * from its page-locked copy if frsd_plan_init made one).
 * Limit: the plan's workspace (frsd_plan_workspace_bytes) must fit the
 * scratch of 128 MiB (e.g. FP32 plans up to N = 64 with a few bispectrum
 * bins); larger plans get FRSD_ENOMEM before any device work.  The scratch
 * (one per device, held until the process ends) keeps the last call's
 * contents; every region a call reads is written by that call first.  All
 * calls on one device share it: calls that overlap in time on one device
 * (other streams or threads) race and give undefined results.  The count
 * of rejected objects is not reported (frsd_status needs a workspace).
 * Asynchronous on `stream`. */
int frsd_run_static(frsd_plan *plan, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                    const frsd_pk_out *pk, const frsd_bk_out *bk, void *stream);

/* A request captured as a HIP graph (serving loops that replay one plan):
 * frsd_graph_create records every kernel of frsd_mesh_assign,
 * frsd_pk_multipoles and (bk non-NULL, plan with bispectrum bins)
 * frsd_bk_multipoles for these catalogue buffers, outputs and workspace on
 * `stream` (non-null; stream capture, so nothing runs then) and
 * instantiates it.  The catalogue sizes given here are capacities: the
 * ingest kernels read N_g, N_r and alpha from device memory, which
 * frsd_graph_launch sets (with a kernel, not a copy) before each replay, so a
 * replay takes the first n_gal / n_ran objects of the same buffers with any
 * contents.  Replays on one workspace must be ordered on one stream, as any
 * call.  The graph owns no device memory; destroy it before the plan or the
 * workspace.  FRSD_ESTATE while frsd_profile is on. */
typedef struct frsd_graph frsd_graph;
int frsd_graph_create(frsd_plan *plan, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                      const frsd_pk_out *pk, const frsd_bk_out *bk, void *stream, frsd_graph **graph);
int frsd_graph_launch(frsd_graph *graph, int64_t n_gal, int64_t n_ran, double alpha, void *stream);
void frsd_graph_destroy(frsd_graph *graph);

/* A batch of requests captured as one graph: the launches of frsd_pk_batch
 * (same arguments and checks; ran non-NULL: no random cache) recorded on
 * `stream` (non-null) for these catalogue buffers, whose sizes are
 * capacities, and outputs.  frsd_graph_launch_batch replays it with request
 * r taking the first n_gal[r] / n_ran[r] objects of its buffers and alpha[r]
 * (host arrays of the captured batch size; the sizes and alpha are written
 * into each workspace by a kernel before the replay).  FRSD_ENOMEM for sizes
 * beyond the capacities, FRSD_EINVAL for frsd_graph_launch on a batch
 * graph; frsd_graph_launch_batch also replays a graph of one request.
 * Destroyed with frsd_graph_destroy. */
int frsd_graph_create_batch(frsd_plan *const *plans, void *const *workspaces, int32_t n, const frsd_catalog *gal,
                            const frsd_catalog *ran, const double *alpha, const frsd_pk_out *out, void *stream,
                            frsd_graph **graph);
int frsd_graph_launch_batch(frsd_graph *graph, const int64_t *n_gal, const int64_t *n_ran, const double *alpha,
                            void *stream);

/* Synchronises `stream` and reports the number of objects rejected by the
 * last frsd_mesh_assign (outside [0, L)^3 or at the observer).  Returns
 * FRSD_EDOM when that number is non-zero. */
int frsd_status(frsd_plan *plan, void *ws, int64_t *n_rejected, void *stream);

/* Per-kernel timing with HIP events recorded on each call's stream.  Off
 * by default.  frsd_profile(1) makes every later kernel launch of every plan
 * record a start and a stop event; frsd_profile_report waits for the
 * recorded events, writes one line "name launches total_ms" per kernel name
 * into buf (NUL-terminated, truncated to len), and clears the records. */
int frsd_profile(int enable);
int frsd_profile_report(char *buf, size_t len);

/* Thread-local description of the last failure ("" if none). */
const char *frsd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTRSD_H */
