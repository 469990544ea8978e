// Step a3: B-spline assignment of the moment meshes (Sec. III.A eq. mapFFT
// and the paragraph after it), and the driver of steps a1-a4.
//
// Owner-computes gather, no atomics.  Each thread owns one node of the main
// grid (integer grid coordinates) and the node half a cell above it on the
// interlaced twin grid, and accumulates every moment plane of both nodes in
// registers:
//   mesh_m(i) = sum_j t0_j T_m(xhat_j) prod_d W_p(u_jd - i_d),
// with T_m in {1, xhat_a xhat_b, xhat_a xhat_b xhat_c xhat_d} (the 15 kept
// components of frsd_internal.h) and the w^2 plane of F_0^w (weight t0^2).  A workgroup owns a block of 4 x 8 x 16
// nodes; it stages the objects of every cell that can reach the block (the
// block grown by the kernel support) in LDS, in cell order, and each thread
// walks the contiguous runs of objects in the RW^3 cells around its node
// (RW = 4 for TSC: floor cells i-2..i+1 reach the main node i and i-1..i+1
// the twin node i+1/2; RW = 5 for PCS: i-2..i+1 and i-2..i+2).  Plans of
// orders 1-3 with N a multiple of 64 use the x-sweep form below instead.
// The line of sight of an object is rebuilt from its
// position and the observer (the true position, not the periodic image,
// for blocks at the box faces).
//
// Blocks whose grown region holds more objects than LDS can stage are
// processed in several chunks of the staged order; the accumulators carry
// over.  Blocks with no object write zeros.
//
// Only node columns (x, y) within reach of some object (colmask, built
// from the cell offsets before the assignment) are written; the FFT passes
// read every other column as zero.  Blocks with no such column return at
// once, so the empty part of the box around a survey costs neither
// assignment nor memory traffic.
//
// Output packing: plane array 2s holds the real part and 2s+1 the
// imaginary part of complex slot s.  With interlacing, the main-grid plane
// of moment m is the real part and the twin plane the imaginary part of
// slot m; without interlacing, moments 2s and 2s+1 share slot s.  The first
// FFT pass reads the planar arrays and writes interleaved complex meshes.
#include <algorithm>
#include <type_traits>

#include "device.h"
#include "frsd_internal.h"

namespace frsd {

constexpr int kBX = 4, kBY = 8, kBZ = 16;
constexpr int kGThreads = kBX * kBY * kBZ;  // one (main, twin) node pair per thread
constexpr int kGCellsMax = 1920;            // cells of a grown block (96 columns x 20 for PCS, 77 x 19 for TSC)
constexpr int kGStageBytes = 65536;         // staged object records (two workgroups per CU)

template <typename T>
int ingest_and_sort(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                    hipStream_t s, const double *dyn);
template <typename T>
int ingest_and_sort_batch(frsd_plan *pl, void *const *wss, int nreq, const frsd_catalog *gal,
                          const frsd_catalog *ran, const double *alpha, hipStream_t s, const double *dyn);
void scal_keep(frsd_plan *pl, void *ws, hipStream_t s);
void scal_cached(frsd_plan *pl, void *ws, double alpha, hipStream_t s);
void scal_cached_batch(frsd_plan *pl, void *const *wss, int nreq, const double *alpha, hipStream_t s);

// Floor cells that reach the main node i (at i) or the twin node (at i + 1/2),
// relative to i: [LO, HI].
template <int P> struct Win;
template <> struct Win<1> { static constexpr int LO = -1, HI = 0; };
template <> struct Win<2> { static constexpr int LO = -1, HI = 1; };
template <> struct Win<3> { static constexpr int LO = -2, HI = 1; };
template <> struct Win<4> { static constexpr int LO = -2, HI = 2; };  // main i-2..i+1, twin i-2..i+2

// Assignment kernel of order P at distance d (grid units); NGP is the
// half-open cell [-1/2, 1/2).
template <typename T, int P>
__device__ __forceinline__ T kernel_w(T d) {
  if constexpr (P == 1) {
    return (d >= T(-0.5) && d < T(0.5)) ? T(1) : T(0);
  } else if constexpr (P == 2) {
    return fmax(T(1) - fabs(d), T(0));
  } else if constexpr (P == 3) {
    // both pieces evaluated, then selected: no divergent branch
    const T a = fabs(d);
    const T b = fmax(T(1.5) - a, T(0));
    const T inner = T(0.75) - a * a, outer = T(0.5) * b * b;
    return a < T(0.5) ? inner : outer;
  } else {
    // cubic B-spline (PCS): (4 - 6 a^2 + 3 a^3) / 6 for a < 1, (2 - a)^3 / 6 for 1 <= a < 2
    static_assert(P == 4, "orders 1..4");
    const T a = fabs(d);
    const T b = fmax(T(2) - a, T(0));
    const T inner = (T(4) + a * a * (T(3) * a - T(6))) * T(1.0 / 6.0), outer = b * b * b * T(1.0 / 6.0);
    return a < T(1) ? inner : outer;
  }
}

// r^2 is at least ~1e-12 grid units^2 here, far from the denormal range, so
// the bare hardware reciprocal square root (about 1 ulp) is used.
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

struct GridArgs {
  int N;
  int n_ell_mom;       // moments of the multipoles: 1, 6 or 15 (ell_max 0, 2, 4)
  int has_w;           // w^2 plane present (position n_ell_mom)
  int interlace;
  int wsq;             // 1: every object weighs t0^2 (the w^2-weighted moments of F^w_l)
  int m0;              // first moment position written (streamed plans grid a group of positions
                       // m0..n_ell_mom-1 per pass; planes are numbered from m0)
  double ou[3];        // observer in grid units
  long long plane_stride;
  int sx;              // x-sweep: nodes along x per workgroup (16, 32 or 64)
};

// Add the moment-weighted contribution s of one object to the 16
// accumulators (the 15 kept moments of frsd_internal.h and the w^2 plane):
// q holds the kept rank-2 monomials of the line of sight in ID order (xx yy
// xy yz zx), q4 the kept rank-4 ones.  Moments below m0 (not written by
// this pass of a streamed plan) are accumulated all the same (and not
// written): per-rank tests here cost the FP64 gather more than they save.
template <typename T>
__device__ __forceinline__ void add_moments(T *acc, T s, T t0, const T *q, const T *q4, int n_ell_mom, bool has_w) {
  acc[0] += s;
  if (n_ell_mom > 1) {
#pragma unroll
    for (int i = 0; i < 5; ++i) acc[1 + i] += s * q[i];
    if (n_ell_mom > kMomRank2) {
#pragma unroll
      for (int i = 0; i < 9; ++i) acc[kMomRank2 + i] += s * q4[i];
    }
  }
  if (has_w) acc[kMomW] += s * t0;
}

// Kept rank-4 monomials (IDs 6-14: xxxx yyyy xxxy xxxz yyyx yyyz xxyy xxyz
// yyxz) from the kept rank-2 ones: each is xx or yy times a rank-2 monomial.
template <typename T>
__device__ __forceinline__ void rank4_from_rank2(const T *q, T *q4) {
  q4[0] = q[0] * q[0]; q4[1] = q[1] * q[1]; q4[2] = q[0] * q[2]; q4[3] = q[0] * q[4]; q4[4] = q[1] * q[2];
  q4[5] = q[1] * q[3]; q4[6] = q[0] * q[1]; q4[7] = q[0] * q[3]; q4[8] = q[1] * q[4];
}

// Node columns within reach of an object: colmask[x N + y] = 1 when some
// cell column (cx, cy) with cx - x and cy - y in [LO, HI] (periodic) holds
// an object, i.e. offs[2 (cx N + cy + 1) N] > offs[2 (cx N + cy) N] for the
// exclusive scan offs of the half-cell counts (colocc[cx N + cy]); xmask[x]
// = 1 when any column of slab x is set.  One workgroup per (x, request of
// the batch); every pointer is request 0's.
template <int P>
__global__ __launch_bounds__(256) void k_col_mask(const int *__restrict__ offs, int N, uint8_t *colmask,
                                                  uint8_t *xmask, uint8_t *colocc, Batch bt) {
  constexpr int LO = Win<P>::LO, HI = Win<P>::HI;
  const long long dr = bt.delta[blockIdx.y];
  offs = shifted(offs, dr);
  colmask = shifted(colmask, dr);
  xmask = shifted(xmask, dr);
  colocc = shifted(colocc, dr);
  const int x = blockIdx.x;
  int any = 0;
  for (int y = threadIdx.x; y < N; y += 256) {
    const long long c0 = 2 * ((long long)x * N + y) * N;
    colocc[(long long)x * N + y] = offs[c0 + 2 * N] > offs[c0] ? 1 : 0;
    int m = 0;
#pragma unroll
    for (int dx = LO; dx <= HI; ++dx) {
      int cx = x + dx;
      cx += cx < 0 ? N : (cx >= N ? -N : 0);
#pragma unroll
      for (int dy = LO; dy <= HI; ++dy) {
        int cy = y + dy;
        cy += cy < 0 ? N : (cy >= N ? -N : 0);
        const long long c0 = 2 * ((long long)cx * N + cy) * N;
        m |= offs[c0 + 2 * N] > offs[c0] ? 1 : 0;
      }
    }
    colmask[(long long)x * N + y] = (uint8_t)m;
    any |= m;
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) xmask[x] = any ? 1 : 0;
}

// The same sum with the rank-4 monomials taken as (s xx) q_b and (s yy) q_b:
// no rank-4 table is held across a ring of nodes.
template <typename T>
__device__ __forceinline__ void add_moments_u(T *acc, T s, T t0, const T *q, int n_ell_mom, bool has_w, int m0) {
  if (m0 == 0) acc[0] += s;
  if (n_ell_mom > 1) {
    const T u0 = s * q[0], u1 = s * q[1];
    if (m0 < kMomRank2) {
      acc[1] += u0; acc[2] += u1;
      acc[3] += s * q[2]; acc[4] += s * q[3]; acc[5] += s * q[4];
    }
    if (n_ell_mom > kMomRank2) {
      // xxxx yyyy xxxy xxxz yyyx yyyz xxyy xxyz yyxz
      acc[6] += u0 * q[0]; acc[7] += u1 * q[1]; acc[8] += u0 * q[2];
      acc[9] += u0 * q[4]; acc[10] += u1 * q[2]; acc[11] += u1 * q[3];
      acc[12] += u0 * q[1]; acc[13] += u0 * q[3]; acc[14] += u1 * q[4];
    }
  }
  if (has_w) acc[kMomW] += s * t0;
}

// Grid (blocks, request of the batch); every pointer is request 0's.
template <typename T, int P>
__global__ __launch_bounds__(kGThreads) void k_grid(const int *__restrict__ offs, const Rec4<T> *__restrict__ recs,
                                                     const uint8_t *__restrict__ colmask, GridArgs ga,
                                                     T *__restrict__ planar, Batch bt) {
  {
    const long long dr = bt.delta[blockIdx.y];
    offs = shifted(offs, dr);
    recs = shifted(recs, dr);
    colmask = shifted(colmask, dr);
    planar = shifted(planar, dr);
  }
  constexpr int LO = Win<P>::LO, RW = Win<P>::HI - Win<P>::LO + 1;
  constexpr int CY = kBY + RW - 1, CZ = kBZ + RW - 1;
  constexpr int NCELL = (kBX + RW - 1) * CY * CZ;
  static_assert(NCELL <= kGCellsMax, "grown block too large");
  constexpr int CAP = kGStageBytes / (int)sizeof(Rec4<T>);

  extern __shared__ unsigned char smem_raw[];
  Rec4<T> *st = reinterpret_cast<Rec4<T> *>(smem_raw);  // staged records, block-relative coordinates
  __shared__ int cst[NCELL + 1];                         // staged start of each grown-block cell
  __shared__ int gsrc[NCELL];                            // first sorted record of each cell
  __shared__ int scan_tmp[kGThreads];

  const int N = ga.N;
  const int nby = N / kBY, nbz = N / kBZ;
  const int bx = blockIdx.x / (nby * nbz), by = (blockIdx.x / nbz) % nby, bz = blockIdx.x % nbz;
  const int X0 = bx * kBX, Y0 = by * kBY, Z0 = bz * kBZ;
  const int lx = threadIdx.x / (kBY * kBZ), ly = (threadIdx.x / kBZ) % kBY, lz = threadIdx.x % kBZ;
  const bool live = colmask[(long long)(X0 + lx) * N + (Y0 + ly)] != 0;
  if (!__syncthreads_or(live)) return;  // no object within reach of any node of the block

  // cell table of the grown block: cell e = (ix * CY + iy) * CZ + k is the
  // floor cell (X0 + LO + ix, Y0 + LO + iy, Z0 + LO + k), periodic
  constexpr int PER = (NCELL + kGThreads - 1) / kGThreads;
  int cnt[PER];
  int mysum = 0;
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = threadIdx.x * PER + r;
    cnt[r] = 0;
    if (e < NCELL) {
      const int col = e / CZ, k = e - col * CZ;
      int cx = X0 + LO + col / CY, cy = Y0 + LO + col % CY, cz = Z0 + LO + k;
      cx += cx < 0 ? N : (cx >= N ? -N : 0);
      cy += cy < 0 ? N : (cy >= N ? -N : 0);
      cz += cz < 0 ? N : (cz >= N ? -N : 0);
      const long long idx = 2 * (((long long)cx * N + cy) * N + cz);  // both halves of the cell
      const int a = offs[idx];
      gsrc[e] = a;
      cnt[r] = offs[idx + 2] - a;
      mysum += cnt[r];
    }
  }
  scan_tmp[threadIdx.x] = mysum;
  __syncthreads();
  for (int o = 1; o < kGThreads; o <<= 1) {
    const int t = threadIdx.x >= o ? scan_tmp[threadIdx.x - o] : 0;
    __syncthreads();
    scan_tmp[threadIdx.x] += t;
    __syncthreads();
  }
  const int total = scan_tmp[kGThreads - 1];
  int run = scan_tmp[threadIdx.x] - mysum;
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = threadIdx.x * PER + r;
    if (e < NCELL) cst[e] = run;
    run += cnt[r];
  }
  if (threadIdx.x == 0) cst[NCELL] = total;

  T am[kMaxMom], at[kMaxMom];
#pragma unroll
  for (int m = 0; m < kMaxMom; ++m) { am[m] = T(0); at[m] = T(0); }

  const T fx = (T)lx, fy = (T)ly, fz = (T)lz;
  const T bxo = (T)((double)X0 - ga.ou[0]), byo = (T)((double)Y0 - ga.ou[1]), bzo = (T)((double)Z0 - ga.ou[2]);
  const bool has_w = ga.has_w != 0;
  // blocks whose grown region crosses the periodic boundary: staged
  // coordinates are periodic images, the line of sight needs the true ones
  constexpr int HI = Win<P>::HI;
  const bool edge = X0 + LO < 0 || Y0 + LO < 0 || Z0 + LO < 0 || X0 + kBX - 1 + HI >= N ||
                    Y0 + kBY - 1 + HI >= N || Z0 + kBZ - 1 + HI >= N;
  const T nf = (T)N;
  const T lox = (T)(-X0), loy = (T)(-Y0), loz = (T)(-Z0), hix = (T)(N - X0), hiy = (T)(N - Y0), hiz = (T)(N - Z0);

  for (int s0 = 0; s0 < total; s0 += CAP) {
    const int s1 = min(total, s0 + CAP);
    __syncthreads();  // cell table ready / previous chunk consumed
    for (int i = s0 + (int)threadIdx.x; i < s1; i += kGThreads) {
      int lo = 0, hi = NCELL;  // cst[lo] <= i < cst[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cst[mid] <= i) lo = mid; else hi = mid;
      }
      const Rec4<T> g = recs[gsrc[lo] + (i - cst[lo])];
      const int col = lo / CZ, k = lo - col * CZ;
      Rec4<T> r;
      r.x = (T)(LO + col / CY) + g.x;
      r.y = (T)(LO + col % CY) + g.y;
      r.z = (T)(LO + k) + g.z;
      r.w = ga.wsq ? g.w * g.w : g.w;
      st[i - s0] = r;
    }
    __syncthreads();

    // walk the RW x RW columns of the node's window; in each, the RW cells
    // starting at this node's z are one contiguous run of staged records
    // one flat stream per thread (the columns' runs back to back); the
    // wavefront runs a uniform trip count, the longest stream among its
    // threads, and finished threads add zero
    int mine = 0;
#pragma unroll 1
    for (int wi = 0; wi < RW * RW; ++wi) {
      const int e = ((lx + wi / RW) * CY + (ly + wi % RW)) * CZ + lz;
      mine += max(0, min(cst[e + RW], s1) - max(cst[e], s0));
    }
    int trips = mine;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) trips = max(trips, __shfl_xor(trips, o, 64));
    int wi = 0, j = 0, je = 0;
    auto advance = [&]() {
#pragma unroll 1
      while (j >= je && wi < RW * RW) {
        const int e = ((lx + wi / RW) * CY + (ly + wi % RW)) * CZ + lz;
        j = max(cst[e], s0) - s0;
        je = min(cst[e + RW], s1) - s0;
        ++wi;
      }
    };
    advance();
    bool nvalid = j < je;
    Rec4<T> nr = st[nvalid ? j : 0];
#pragma unroll 1
    for (int t = 0; t < trips; ++t) {
      // the next record is read while this one is processed
      Rec4<T> r = nr;
      if (!nvalid) r.w = T(0);
      j += nvalid ? 1 : 0;
      advance();
      nvalid = j < je;
      nr = st[nvalid ? j : 0];
      const T dx = r.x - fx, dy = r.y - fy, dz = r.z - fz;
      const T sm = r.w * (kernel_w<T, P>(dx) * kernel_w<T, P>(dy) * kernel_w<T, P>(dz));
      T stw = T(0);
      if (ga.interlace)
        stw = r.w * (kernel_w<T, P>(dx - T(0.5)) * kernel_w<T, P>(dy - T(0.5)) * kernel_w<T, P>(dz - T(0.5)));
      // line of sight (computed even when only the monopole is gridded)
      T q[5], q4[9];
      {
        T px = r.x + bxo, py = r.y + byo, pz = r.z + bzo;
        if (edge) {
          px += r.x < lox ? nf : (r.x >= hix ? -nf : T(0));
          py += r.y < loy ? nf : (r.y >= hiy ? -nf : T(0));
          pz += r.z < loz ? nf : (r.z >= hiz ? -nf : T(0));
        }
        const T r2 = px * px + py * py + pz * pz;
        const T ir = r2 > T(0) ? rsqrt_t(r2) : T(0);
        const T hx = px * ir, hy = py * ir, hz = pz * ir;
        q[0] = hx * hx; q[1] = hy * hy; q[2] = hx * hy; q[3] = hy * hz; q[4] = hz * hx;
      }
      rank4_from_rank2(q, q4);
      add_moments<T>(am, sm, r.w, q, q4, ga.n_ell_mom, has_w);
      if (ga.interlace) add_moments<T>(at, stw, r.w, q, q4, ga.n_ell_mom, has_w);
    }
  }

  // write every plane of both nodes (contiguous z-runs of the planar output)
  if (!live) return;
  const long long g = ((long long)(X0 + lx) * N + (Y0 + ly)) * N + (Z0 + lz);
  const long long ps = ga.plane_stride;
  const int n_mom = ga.n_ell_mom + ga.has_w - ga.m0;
#pragma unroll
  for (int id = 0; id < kMaxMom; ++id) {
    const bool present = (id < ga.n_ell_mom && id >= ga.m0) || (id == kMomW && ga.has_w);
    if (!present) continue;
    const int pos = (id < ga.n_ell_mom ? id : ga.n_ell_mom) - ga.m0;  // position of the moment in the slot list
    if (ga.interlace) {
      planar[(2LL * pos) * ps + g] = am[id];
      planar[(2LL * pos + 1) * ps + g] = at[id];
    } else {
      planar[(long long)pos * ps + g] = am[id];  // array pos = slot pos / 2, part pos % 2
    }
  }
  if (!ga.interlace && (n_mom & 1)) planar[(long long)n_mom * ps + g] = T(0);
}

// ---------------------------------------------------------------------------
// x-sweep assignment (orders 1-3, N a multiple of 64; FP32 and FP64 plans).
//
// A workgroup owns a 4 (y) x 32 (z) patch of node columns and sweeps it
// along x over 64 nodes.  At each cell slab x = c it stages the objects of
// the slab cells that reach the patch, and every thread adds each object of
// its window to the ring of the RING nodes of its column that the slab
// reaches (nodes c - HI .. c - LO); the lowest ring node is then complete
// and is written out.  Per visit the line of sight, the moments and the y
// and z kernel weights are computed once for all ring nodes, which makes the
// sweep several times cheaper in instructions than the per-node gather
// above.  Staged records stay 16 bytes (each lane reads its own record, so
// LDS bandwidth, not arithmetic, decides the record size).  Main and twin
// grids are separate passes (separate windows and rings).  The ring slots
// are compile-time indices: the cell loop is unrolled by RING.
// ---------------------------------------------------------------------------
constexpr int kSY = 4, kSZ = 32, kSX = 64;  // kSX: the longest x run of a workgroup (runs of 16, 32 or 64)
constexpr int kSThreads = kSY * kSZ;                   // one node column per thread
constexpr int kSCap = 1024;                            // staged objects per chunk (16 B each)
constexpr int kSCellsMax = (kSY + 3) * (kSZ + 3);      // slab cells for a ring of 4
constexpr int kSStepsMax = kSX + 3;
static_assert(kSCellsMax <= 2 * kSThreads, "two slab cells per thread");

// Cells [LO, HI] (relative to node n) reaching the main node n or the twin
// node n + 1/2 of each assignment order.
template <int P, bool TWIN> struct SweepWin;
template <> struct SweepWin<3, false> { static constexpr int LO = -2, HI = 1; };
template <> struct SweepWin<3, true> { static constexpr int LO = -1, HI = 1; };
template <> struct SweepWin<2, false> { static constexpr int LO = -1, HI = 0; };
template <> struct SweepWin<2, true> { static constexpr int LO = -1, HI = 1; };
template <> struct SweepWin<1, false> { static constexpr int LO = -1, HI = 0; };
template <> struct SweepWin<1, true> { static constexpr int LO = 0, HI = 0; };

// Staged object: x fraction in cell c, y and z relative to the patch origin,
// t0 (16 bytes in FP32 plans, 32 in FP64 plans).
template <typename T> struct alignas(4 * sizeof(T)) SweepRec {
  T x, y, z, w;
};

// FP32 plans run 4 waves per SIMD (128 VGPRs); FP64 plans hold twice the
// accumulator registers and run 2.  Grid (patches, request of the batch);
// every pointer is request 0's.
template <typename T, int P, bool TWIN>
__global__ __launch_bounds__(kSThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) void k_grid_sweep(
    const int *__restrict__ offs, const Rec4<T> *__restrict__ recs, const uint8_t *__restrict__ colmask,
    const uint8_t *__restrict__ colocc, GridArgs ga, T *__restrict__ planar, Batch bt) {
  {
    const long long dr = bt.delta[blockIdx.y];
    offs = moved(offs, dr);
    recs = moved(recs, dr);
    colmask = moved(colmask, dr);
    colocc = moved(colocc, dr);
    planar = moved(planar, dr);
  }
  using Wn = SweepWin<P, TWIN>;
  constexpr int LO = Wn::LO, HI = Wn::HI, RING = HI - LO + 1;
  constexpr int CY = kSY + RING - 1, CZ = kSZ + RING - 1, NSC = CY * CZ;
  static_assert(NSC <= kSCellsMax && RING <= 4, "slab too large");
  constexpr T SH = TWIN ? T(0.5) : T(0);  // node offset of the pass
  // TSC main and CIC twin nodes: the support ends mid-cell in z, where the
  // kernel weight is zero, so the window's z run skips the far halves of
  // its first and last cells (the records of a cell are ordered by z half)
  constexpr bool TRIM = (P == 3 && !TWIN) || (P == 2 && TWIN);
  __shared__ SweepRec<T> st[kSCap];
  __shared__ int cst[kSCellsMax + 1];  // staged start of each slab cell (e = iy * CZ + iz)
  __shared__ int clo[kSCellsMax];      // records of the cell's lower z half (those come first)
  __shared__ int gsrc[kSCellsMax];     // first sorted record of each slab cell
  __shared__ int wtot[kSThreads / 64];
  __shared__ uint8_t step_live[kSStepsMax];  // slab of the step holds an object in the patch's y range

  const int N = ga.N, SX = ga.sx;
  const int nyb = N / kSY, nzb = N / kSZ;
  const int bz = blockIdx.x % nzb, by = (blockIdx.x / nzb) % nyb, bx = blockIdx.x / (nzb * nyb);
  const int X0 = bx * SX, Y0 = by * kSY, Z0 = bz * kSZ;
  const int ly = threadIdx.x / kSZ, lz = threadIdx.x % kSZ;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  const int NSTEP = SX + RING - 1;  // <= kSStepsMax
  for (int i = threadIdx.x; i < NSTEP; i += kSThreads) step_live[i] = 0;
  {  // patches with no node in reach of an object write nothing
    int live = 0;
    for (int t = threadIdx.x; t < SX * kSY; t += kSThreads)
      live |= colmask[(long long)(X0 + t / kSY) * N + (Y0 + t % kSY)];
    if (!__syncthreads_or(live)) return;
  }
  // steps whose slab has no object in the y range of the patch skip the
  // staging and the visits (the ring is still flushed)
  for (int t = threadIdx.x; t < NSTEP * CY; t += kSThreads) {
    const int sx = t / CY, iy = t - sx * CY;
    int c = X0 + LO + sx, cy = Y0 + LO + iy;
    c += c < 0 ? N : (c >= N ? -N : 0);
    cy += cy < 0 ? N : (cy >= N ? -N : 0);
    if (colocc[(long long)c * N + cy]) step_live[sx] = 1;
  }
  __syncthreads();
  const bool has_w = ga.has_w != 0;
  const int nmom = ga.n_ell_mom, m0 = ga.m0;
  const T ny_ = (T)ly + SH, nz_ = (T)lz + SH;  // node position relative to (Y0, Z0)
  const T nf = (T)N;
  const T oyr = (T)((double)Y0 - ga.ou[1]), ozr = (T)((double)Z0 - ga.ou[2]);
  // patches whose slab crosses the periodic boundary in y or z rebuild the
  // true position of the object for the line of sight
  const bool edge = Y0 + LO < 0 || Z0 + LO < 0 || Y0 + kSY - 1 + HI >= N || Z0 + kSZ - 1 + HI >= N;
  const T loy = (T)(-Y0), loz = (T)(-Z0), hiy = (T)(N - Y0), hiz = (T)(N - Z0);

  T acc[RING][kMaxMom];
#pragma unroll
  for (int r = 0; r < RING; ++r)
#pragma unroll
    for (int m = 0; m < kMaxMom; ++m) acc[r][m] = T(0);

  const long long ps = ga.plane_stride;

  auto step = [&](const int sidx, auto kc) {
    constexpr int k = decltype(kc)::value;  // sidx % RING
    const int c = X0 + LO + sidx;            // cell slab (unwrapped)
    const int cw = c < 0 ? c + N : (c >= N ? c - N : c);
    const T xo = (T)((double)cw - ga.ou[0]);

    if (step_live[sidx]) {
    // ---- slab cell table and exclusive scan of the counts ----
    int cnt[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + h * kSThreads;
      if (e < NSC) {
        const int iy = e / CZ, iz = e - iy * CZ;
        int cy = Y0 + LO + iy, cz = Z0 + LO + iz;
        cy += cy < 0 ? N : (cy >= N ? -N : 0);
        cz += cz < 0 ? N : (cz >= N ? -N : 0);
        const long long idx = 2 * (((long long)cw * N + cy) * N + cz);
        const int a0 = offs[idx];
        gsrc[e] = a0;
        cnt[h] = offs[idx + 2] - a0;
        if (TRIM) clo[e] = offs[idx + 1] - a0;
      }
    }
    // thread t holds cells t and t + 256: scan the 512 slots in two halves
    int incl0 = cnt[0], incl1 = cnt[1];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t0 = __shfl_up(incl0, o, 64), t1 = __shfl_up(incl1, o, 64);
      if (lane >= o) { incl0 += t0; incl1 += t1; }
    }
    if (lane == 63) wtot[wave] = incl0;
    __syncthreads();
    int pre0 = 0, tot0 = 0;
#pragma unroll
    for (int w = 0; w < kSThreads / 64; ++w) {
      const int v = wtot[w];
      pre0 += w < wave ? v : 0;
      tot0 += v;
    }
    __syncthreads();
    if (lane == 63) wtot[wave] = incl1;
    __syncthreads();
    int pre1 = tot0, total = tot0;
#pragma unroll
    for (int w = 0; w < kSThreads / 64; ++w) {
      const int v = wtot[w];
      pre1 += w < wave ? v : 0;
      total += v;
    }
    {
      const int e0 = threadIdx.x, e1 = threadIdx.x + kSThreads;
      if (e0 < NSC) cst[e0] = pre0 + incl0 - cnt[0];
      if (e1 < NSC) cst[e1] = pre1 + incl1 - cnt[1];
      if (threadIdx.x == 0) cst[NSC] = total;
    }

    for (int s0 = 0; s0 < total; s0 += kSCap) {
      const int s1 = min(total, s0 + kSCap);
      __syncthreads();  // cell table ready / previous chunk consumed
      for (int i = s0 + (int)threadIdx.x; i < s1; i += kSThreads) {
        int lo = 0, hi = NSC;  // cst[lo] <= i < cst[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (cst[mid] <= i) lo = mid; else hi = mid;
        }
        const Rec4<T> g = recs[gsrc[lo] + (i - cst[lo])];
        const int iy = lo / CZ, iz = lo - iy * CZ;
        SweepRec<T> r;
        r.x = g.x;
        r.y = (T)(LO + iy) + g.y;
        r.z = (T)(LO + iz) + g.z;
        r.w = ga.wsq ? g.w * g.w : g.w;
        st[i - s0] = r;
      }
      __syncthreads();

      // this thread's window: RING runs (y cells ly..ly+RING-1), each the
      // RING z cells lz..lz+RING-1; one flat stream, uniform trip count per
      // wavefront (finished threads add zero)
      // (TRIM: from the upper half of the first cell to the lower half of
      // the last one, the z extent of the kernel's support)
      auto run_begin = [&](int e) { return TRIM ? cst[e] + clo[e] : cst[e]; };
      auto run_end = [&](int e) { return TRIM ? cst[e + RING - 1] + clo[e + RING - 1] : cst[e + RING]; };
      int mine = 0;
#pragma unroll
      for (int j = 0; j < RING; ++j) {
        const int e = (ly + j) * CZ + lz;
        mine += max(0, min(run_end(e), s1) - max(run_begin(e), s0));
      }
      int trips = mine;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) trips = max(trips, __shfl_xor(trips, o, 64));
      int wi = 0, j = 0, je = 0;
      auto advance = [&]() {
#pragma unroll 1
        while (j >= je && wi < RING) {
          const int e = (ly + wi) * CZ + lz;
          j = max(run_begin(e), s0) - s0;
          je = min(run_end(e), s1) - s0;
          ++wi;
        }
      };
      advance();
      bool nvalid = j < je;
      SweepRec<T> nr = st[nvalid ? j : 0];
#pragma unroll 1
      for (int t = 0; t < trips; ++t) {
        SweepRec<T> r = nr;
        if (!nvalid) r.w = T(0);
        j += nvalid ? 1 : 0;
        advance();
        nvalid = j < je;
        nr = st[nvalid ? j : 0];
        const T wyz = kernel_w<T, P>(r.y - ny_) * kernel_w<T, P>(r.z - nz_);
        // line of sight from the true position
        T px = xo + r.x, py = oyr + r.y, pz = ozr + r.z;
        if (edge) {
          py += r.y < loy ? nf : (r.y >= hiy ? -nf : T(0));
          pz += r.z < loz ? nf : (r.z >= hiz ? -nf : T(0));
        }
        const T r2 = px * px + py * py + pz * pz;
        const T ir = r2 > T(0) ? rsqrt_t(r2) : T(0);
        const T hx = px * ir, hy = py * ir, hz = pz * ir;
        const T q[5] = {hx * hx, hy * hy, hx * hy, hy * hz, hz * hx};
        T wr[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < RING; ++q) wr[q] = r.w * kernel_w<T, P>(r.x + (T)(HI - q) - SH);
#pragma unroll
        for (int rr = 0; rr < RING; ++rr) add_moments_u<T>(acc[(k + rr) % RING], wyz * wr[rr], r.w, q, nmom, has_w, m0);
      }
    }
    }  // step_live

    // the lowest ring node (c - HI) is complete: written when it belongs to
    // the workgroup (the first RING - 1 steps only warm the ring up), and its
    // slot is cleared for the node entering the ring at the next step
    T *a = acc[k % RING];
    if (sidx >= RING - 1) {
      const int n = X0 + sidx - (RING - 1);
      if (colmask[(long long)n * N + Y0 + ly]) {
        const long long g = ((long long)n * N + (Y0 + ly)) * N + (Z0 + lz);
        // streaming stores: the planes are read again only by the FFT, after
        // far more data than the caches hold has passed
#pragma unroll
        for (int id = 0; id < kMaxMom; ++id) {
          const bool present = (id < nmom && id >= ga.m0) || (id == kMomW && has_w);
          if (!present) continue;
          const int pos = (id < nmom ? id : nmom) - ga.m0;
          if (ga.interlace) __builtin_nontemporal_store(a[id], &planar[(2LL * pos + (TWIN ? 1 : 0)) * ps + g]);
          else __builtin_nontemporal_store(a[id], &planar[(long long)pos * ps + g]);
        }
        const int nw = nmom + (has_w ? 1 : 0) - ga.m0;
        if (!TWIN && !ga.interlace && (nw & 1)) planar[(long long)nw * ps + g] = T(0);
      }
    }
#pragma unroll
    for (int m = 0; m < kMaxMom; ++m) a[m] = T(0);
    __syncthreads();  // slab buffers are rewritten by the next step
  };

#pragma unroll 1
  for (int s0 = 0; s0 < NSTEP; s0 += RING) {
    if (s0 + 0 < NSTEP) step(s0 + 0, std::integral_constant<int, 0>{});
    if constexpr (RING > 1) if (s0 + 1 < NSTEP) step(s0 + 1, std::integral_constant<int, 1>{});
    if constexpr (RING > 2) if (s0 + 2 < NSTEP) step(s0 + 2, std::integral_constant<int, 2>{});
    if constexpr (RING > 3) if (s0 + 3 < NSTEP) step(s0 + 3, std::integral_constant<int, 3>{});
  }
}

// Assignment of n_ell_mom moment planes (and the w^2 plane when has_w);
// wsq: weights t0^2 instead of t0 (a second pass after the first, whose
// occupancy masks it reuses).
template <typename T, int P>
static int launch_grid(frsd_plan *pl, void *ws, hipStream_t s, int n_ell_mom, int has_w, int wsq, int m0,
                       const Batch &bt) {
  const Layout &L = pl->L;
  const int N = pl->N;
  GridArgs ga{};
  ga.N = N;
  ga.n_ell_mom = n_ell_mom;
  ga.has_w = has_w;
  ga.wsq = wsq;
  ga.m0 = m0;
  ga.interlace = pl->p.interlace;
  for (int d = 0; d < 3; ++d) ga.ou[d] = pl->p.observer[d] / pl->h;
  ga.plane_stride = (long long)N * N * N;
  if (!wsq && m0 == 0)
    FRSD_TIMED("col_mask", s, hipLaunchKernelGGL(k_col_mask<P>, dim3((unsigned)N, bt.n), dim3(256), 0, s,
                                                 ws_ptr<const int>(ws, L.cnt), N, ws_ptr<uint8_t>(ws, L.colmask),
                                                 ws_ptr<uint8_t>(ws, L.xmask), ws_ptr<uint8_t>(ws, L.colocc), bt));
  if constexpr (P <= 3) {
    if (N % kSX == 0 && N % kSZ == 0) {
      // x nodes per workgroup: the plan's tuning, else 16 (short runs spread
      // a clustered mock over more workgroups, and small meshes get enough
      // of them; each run re-stages 3 slabs of its neighbour's), or 64 for
      // streamed plans, whose passes grid a few moments per visit, so that
      // the re-staging weighs more
      ga.sx = pl->tune.sweep_x ? pl->tune.sweep_x : (pl->p.stream_moments ? 64 : 16);
      const unsigned nblk = (unsigned)((N / ga.sx) * (N / kSY) * (N / kSZ));
      FRSD_TIMED("grid", s, hipLaunchKernelGGL((k_grid_sweep<T, P, false>), dim3(nblk, bt.n), dim3(kSThreads), 0, s,
                                               ws_ptr<const int>(ws, L.cnt), ws_ptr<const Rec4<T>>(ws, L.sorted),
                                               ws_ptr<const uint8_t>(ws, L.colmask), ws_ptr<const uint8_t>(ws, L.colocc),
                                               ga, ws_ptr<T>(ws, L.planar), bt));
      if (ga.interlace)
        FRSD_TIMED("grid_twin", s, hipLaunchKernelGGL((k_grid_sweep<T, P, true>), dim3(nblk, bt.n), dim3(kSThreads), 0,
                                                      s, ws_ptr<const int>(ws, L.cnt),
                                                      ws_ptr<const Rec4<T>>(ws, L.sorted),
                                                      ws_ptr<const uint8_t>(ws, L.colmask),
                                                      ws_ptr<const uint8_t>(ws, L.colocc), ga,
                                                      ws_ptr<T>(ws, L.planar), bt));
      FRSD_LAUNCH_CHECK();
      return FRSD_OK;
    }
  }
  auto kern = k_grid<T, P>;
  FRSD_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kGStageBytes));
  const unsigned nblk = (unsigned)((N / kBX) * (N / kBY) * (N / kBZ));
  FRSD_TIMED("grid", s, hipLaunchKernelGGL(kern, dim3(nblk, bt.n), dim3(kGThreads), kGStageBytes, s,
                                           ws_ptr<const int>(ws, L.cnt), ws_ptr<const Rec4<T>>(ws, L.sorted),
                                           ws_ptr<const uint8_t>(ws, L.colmask), ga, ws_ptr<T>(ws, L.planar), bt));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template <typename T>
static int grid_order(frsd_plan *pl, void *ws, hipStream_t s, int n_ell_mom, int has_w, int wsq, int m0 = 0,
                      const Batch &bt = batch_one()) {
  switch (pl->p.order) {
    case 1: return launch_grid<T, 1>(pl, ws, s, n_ell_mom, has_w, wsq, m0, bt);
    case 2: return launch_grid<T, 2>(pl, ws, s, n_ell_mom, has_w, wsq, m0, bt);
    case 3: return launch_grid<T, 3>(pl, ws, s, n_ell_mom, has_w, wsq, m0, bt);
    default: return launch_grid<T, 4>(pl, ws, s, n_ell_mom, has_w, wsq, m0, bt);
  }
}

// Moment positions m0..m1-1 only (streamed plans), planes numbered from m0.
template <typename T>
int run_grid_group(frsd_plan *pl, void *ws, int m0, int m1, hipStream_t s) {
  return grid_order<T>(pl, ws, s, m1, 0, 0, m0);
}
template int run_grid_group<float>(frsd_plan *, void *, int, int, hipStream_t);
template int run_grid_group<double>(frsd_plan *, void *, int, int, hipStream_t);

// Assignment of the sorted records into every moment plane of the plan
// (of every request of the batch; ws: request 0's workspace).
template <typename T>
static int grid_all(frsd_plan *pl, void *ws, hipStream_t s, const Batch &bt = batch_one()) {
  const SlotDesc &sd = pl->slots;
  int n_ell_mom = 0, has_w = 0;
  for (int m = 0; m < sd.n_mom; ++m) {
    if (sd.mom_id[m] == kMomW) has_w = 1;
    else ++n_ell_mom;
  }
  return grid_order<T>(pl, ws, s, n_ell_mom, has_w, 0, 0, bt);
}

// Forward transforms of the assignment planes into the complex meshes at
// mesh_off (the mesh region, or the random cache) of the batch's requests
// (ws: request 0's workspace).
template <typename T>
static int transform(frsd_plan *pl, void *ws, size_t mesh_off, hipStream_t s, const Batch &bt = batch_one()) {
  return fft3d_forward<T>(pl->fft_n, ws_ptr<void>(ws, pl->L.tw_fwd), ws_ptr<const void>(ws, pl->L.planar),
                          ws_ptr<void>(ws, mesh_off), pl->slots.n_slot, pl->nmax,
                          std::max(pl->pk_lut_len, pl->p.bk_nbins > 0 ? pl->bk_lut_len : 0) - 1,
                          ws_ptr<const uint8_t>(ws, pl->L.colmask), ws_ptr<const uint8_t>(ws, pl->L.xmask), s,
                          pl->tune.row_grid, bt);
}

template <typename T>
static int grid_and_transform(frsd_plan *pl, void *ws, size_t mesh_off, hipStream_t s) {
  const int rc = grid_all<T>(pl, ws, s);
  return rc ? rc : transform<T>(pl, ws, mesh_off, s);
}

template <typename T>
int run_mesh_assign(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                    hipStream_t s, const double *dyn) {
  int rc = ingest_and_sort<T>(pl, ws, gal, ran, alpha, s, dyn);
  if (rc) return rc;
  return grid_and_transform<T>(pl, ws, pl->L.mesh, s);
}

// Random cache: the randoms alone with weight +w (ingested as "randoms" with
// alpha = -1, so each record carries -alpha w = w), their moment meshes
// transformed into the cache region and their raw sums kept.
template <typename T>
int run_random_cache(frsd_plan *pl, void *ws, const frsd_catalog *ran, hipStream_t s) {
  const frsd_catalog none{nullptr, nullptr, nullptr, 0, FRSD_F64};
  int rc = ingest_and_sort<T>(pl, ws, &none, ran, -1.0, s, nullptr);
  if (rc) return rc;
  scal_keep(pl, ws, s);
  return grid_and_transform<T>(pl, ws, pl->L.rcache, s);
}

// Galaxies alone against the random cache: their meshes into the mesh
// region (the binning combines them with the cached ones), and the scalar
// sums folded with the cached random sums for this alpha.
template <typename T>
int run_mesh_assign_cached(frsd_plan *pl, void *ws, const frsd_catalog *gal, double alpha, hipStream_t s) {
  const frsd_catalog none{nullptr, nullptr, nullptr, 0, FRSD_F64};
  int rc = ingest_and_sort<T>(pl, ws, gal, &none, alpha, s, nullptr);
  if (rc) return rc;
  scal_cached(pl, ws, alpha, s);
  return grid_and_transform<T>(pl, ws, pl->L.mesh, s);
}

// A batch of requests on plans of one shape: the ingest and sort, the
// occupancy masks, the assignment (main and twin grids) and each forward
// FFT pass run as one launch over every request.  ran null: the galaxies
// against each plan's random cache.
template <typename T>
int run_mesh_assign_batch(frsd_plan *const *pls, void *const *wss, int n, const frsd_catalog *gal,
                          const frsd_catalog *ran, const double *alpha, hipStream_t s, const double *dyn) {
  int rc = ingest_and_sort_batch<T>(pls[0], wss, n, gal, ran, alpha, s, dyn);
  if (rc) return rc;
  if (!ran) scal_cached_batch(pls[0], wss, n, alpha, s);
  const Batch bt = batch_of(wss, n);
  rc = grid_all<T>(pls[0], wss[0], s, bt);
  return rc ? rc : transform<T>(pls[0], wss[0], pls[0]->L.mesh, s, bt);
}

template int run_mesh_assign_batch<float>(frsd_plan *const *, void *const *, int, const frsd_catalog *,
                                          const frsd_catalog *, const double *, hipStream_t, const double *);
template int run_mesh_assign_batch<double>(frsd_plan *const *, void *const *, int, const frsd_catalog *,
                                           const frsd_catalog *, const double *, hipStream_t, const double *);
template int run_random_cache<float>(frsd_plan *, void *, const frsd_catalog *, hipStream_t);
template int run_random_cache<double>(frsd_plan *, void *, const frsd_catalog *, hipStream_t);
template int run_mesh_assign_cached<float>(frsd_plan *, void *, const frsd_catalog *, double, hipStream_t);
template int run_mesh_assign_cached<double>(frsd_plan *, void *, const frsd_catalog *, double, hipStream_t);

// The w^2-weighted moment meshes of F^w_2, F^w_4 (Sec. III.B, the definition
// of F^w_l below eq. SNbisp2): the first n_wmom moments gridded again from
// the sorted records with weight t0^2 (w^2 for galaxies, alpha^2 w^2 for
// randoms), then transformed with the forward passes pruned to the
// bispectrum sphere.  Overwrites the planar and mesh regions (the
// multipole fields of the bispectrum already sit in the low-k cube).
template <typename T>
int run_w_moments(frsd_plan *pl, void *ws, hipStream_t s) {
  int rc = grid_order<T>(pl, ws, s, pl->n_wmom, 0, 1);
  if (rc) return rc;
  const int n_slot = pl->p.interlace ? pl->n_wmom : (pl->n_wmom + 1) / 2;
  return fft3d_forward<T>(pl->fft_n, ws_ptr<void>(ws, pl->L.tw_fwd), ws_ptr<const void>(ws, pl->L.planar),
                          ws_ptr<void>(ws, pl->L.mesh), n_slot, pl->nc_b, pl->bk_lut_len - 1,
                          ws_ptr<const uint8_t>(ws, pl->L.colmask), ws_ptr<const uint8_t>(ws, pl->L.xmask), s,
                          pl->tune.row_grid);
}

template int run_w_moments<float>(frsd_plan *, void *, hipStream_t);
template int run_w_moments<double>(frsd_plan *, void *, hipStream_t);

template int run_mesh_assign<float>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                    hipStream_t, const double *);
template int run_mesh_assign<double>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                     hipStream_t, const double *);

}  // namespace frsd
