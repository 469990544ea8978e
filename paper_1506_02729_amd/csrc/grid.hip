// Step a3: B-spline assignment of the moment meshes (Sec. III.A eq. mapFFT
// and the paragraph after it), and the driver of steps a1-a4.
//
// Owner-computes gather with LDS privatisation.  A workgroup owns one
// 8 x 4 x 16 tile of output nodes of one grid (the main grid, nodes at
// integer grid coordinates, or the interlaced twin grid, nodes at
// half-integer coordinates) and accumulates all moment planes of that grid
// for the tile in LDS.  It walks the cells whose objects can reach the tile
// (the tile grown by the kernel support; objects are sorted by cell, so
// each z-run of cells is one contiguous segment of the sorted records).
//
// Lane mapping: each half-wavefront (32 lanes) takes one object and each of
// its lanes owns one moment plane (w, w xhat_i xhat_j, w xhat^4 ..., w^2).
// For a given node the 23 lanes of an object therefore add into 23
// different planes, at addresses one plane stride (tile size + 1) apart,
// and no two lanes of an object ever hit the same word.  The LDS
// accumulators are FP64 for every precision: on gfx950 the LDS FP64 atomic
// add (ds_add_f64) runs at ~7 lanes/clk/CU while the FP32 one runs at
// ~0.3, so FP64 is both ~25x faster here and more accurate.
// Each tile is written once, with contiguous z-runs, to a planar output
// (one real N^3 array per plane); tiles whose 27-tile neighbourhood holds
// no object skip the scan and write zeros.  No separate zero fill and no
// global atomics are needed.
//
// Output packing: plane array 2s holds the real part and 2s+1 the
// imaginary part of complex slot s.  With interlacing, the main-grid plane
// of moment m is the real part and the twin plane the imaginary part of
// slot m; without interlacing, moments 2s and 2s+1 share slot s.  The first
// FFT pass reads the planar arrays and writes interleaved complex meshes.
#include "device.h"
#include "frsd_internal.h"

namespace frsd {

constexpr int kGX = 8, kGY = 4, kGZ = 16, kGCells = kGX * kGY * kGZ;
constexpr int kPlaneStride = kGCells + 1;
constexpr int kGridThreads = 1024;  // one workgroup fills a CU's LDS: 16 waves hide latency
constexpr int kMaxSeg = kGridThreads;  // one segment per thread at most
// Object records of one chunk, staged in LDS (1024 FP32 or 512 FP64 records).
template <typename T>
struct Staged {
  static constexpr int n = sizeof(T) == 4 ? 1024 : 512;
  int cell[n];
  T f[3][n];
  T t0[n], tw[n];
  T h[3][n];
};

template <typename T>
int ingest_and_sort(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                    hipStream_t s);

struct PlaneDesc {
  int n_groups;           // 1 (no interlacing) or 2 (main, twin)
  int n_planes[2];
  int twin[2];            // group uses the twin grid
  int mom[2][32];         // moment ID of each plane
  int out_slot[2][32];    // complex slot written by each plane
  int out_im[2][32];      // 0: real part, 1: imaginary part
  int zero_slot;          // slot whose imaginary part has no plane (odd count, no interlacing), or -1
  int8_t idx[kMaxMom][4]; // moment components
  int8_t rank[kMaxMom];
};

// Kernel weights of order P along one axis for an object at cell c with
// fractional offset f in [0, 1): first node and P weights, main grid or
// twin grid (twin nodes at +1/2, i.e. the object's coordinate is u - 1/2).
template <typename T, int P, bool TWIN>
__device__ __forceinline__ int axis_weights(int c, T f, T *wt) {
  const T half = T(0.5);
  if constexpr (P == 1) {
    wt[0] = T(1);
    return TWIN ? c : c + (f >= half ? 1 : 0);
  } else if constexpr (P == 2) {
    if (!TWIN) { wt[0] = T(1) - f; wt[1] = f; return c; }
    const bool up = f >= half;
    const T d = up ? f - half : f + half;
    wt[0] = T(1) - d; wt[1] = d;
    return up ? c : c - 1;
  } else {
    // nearest node m and offset d in [-1/2, 1/2)
    const bool up = f >= half;
    const int m = TWIN ? c : c + (up ? 1 : 0);
    const T d = TWIN ? f - half : (up ? f - T(1) : f);
    const T a = half - d, b = half + d;
    wt[0] = half * a * a; wt[1] = T(0.75) - d * d; wt[2] = half * b * b;
    return m - 1;
  }
}

// Nodes reached from cell c: [c - LO, c + HI] (main / twin grid, order P).
template <int P, bool TWIN> struct Reach;
template <> struct Reach<1, false> { static constexpr int LO = 0, HI = 1; };
template <> struct Reach<1, true> { static constexpr int LO = 0, HI = 0; };
template <> struct Reach<2, false> { static constexpr int LO = 0, HI = 1; };
template <> struct Reach<2, true> { static constexpr int LO = 1, HI = 1; };
template <> struct Reach<3, false> { static constexpr int LO = 1, HI = 2; };
template <> struct Reach<3, true> { static constexpr int LO = 1, HI = 1; };

template <typename T, int P, bool TWIN>
__device__ void grid_tile(const int *__restrict__ offs, const int *__restrict__ r_cell,
                          const T *__restrict__ r_f, size_t fstride, int N, const PlaneDesc &pd, int group,
                          int X0, int Y0, int Z0, double *acc, int *seg_start, int *seg_pref, Staged<T> &st) {
  constexpr int LO = Reach<P, TWIN>::LO, HI = Reach<P, TWIN>::HI;
  // cells that can reach the tile: [T0 - HI, T0 + 7 + LO] per axis
  constexpr int nxr = kGX + LO + HI, nyr = kGY + LO + HI;
  constexpr int nseg = nxr * nyr * 2;
  static_assert(nseg <= kMaxSeg, "too many segments");
  const int zlo = Z0 - HI, zhi = Z0 + kGZ - 1 + LO;
  int my_len = 0, my_start = 0;
  if (threadIdx.x < nseg) {
    const int part = threadIdx.x & 1;
    const int col = threadIdx.x >> 1;
    const int cx = ((X0 - HI + col / nyr) % N + N) % N;
    const int cy = ((Y0 - HI + col % nyr) % N + N) % N;
    int a, e;  // inclusive z range of this part of the periodic run; a > e: empty
    if (zlo < 0) { if (part == 0) { a = 0; e = zhi; } else { a = N + zlo; e = N - 1; } }
    else if (zhi >= N) { if (part == 0) { a = zlo; e = N - 1; } else { a = 0; e = zhi - N; } }
    else { if (part == 0) { a = zlo; e = zhi; } else { a = 1; e = 0; } }
    if (a <= e) {
      const long long rowc = ((long long)cx * N + cy) * N;
      my_start = offs[rowc + a];
      my_len = offs[rowc + e + 1] - my_start;
    }
  }
  seg_pref[threadIdx.x + 1] = my_len;
  if (threadIdx.x == 0) seg_pref[0] = 0;
  seg_start[threadIdx.x] = my_start;
  __syncthreads();
  for (int o = 1; o < kGridThreads; o <<= 1) {
    const int t = (threadIdx.x >= o) ? seg_pref[threadIdx.x + 1 - o] : 0;
    __syncthreads();
    seg_pref[threadIdx.x + 1] += t;
    __syncthreads();
  }
  const int total = seg_pref[kGridThreads];

  // this lane's moment plane
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, pl = lane & 31;
  const int np = pd.n_planes[group];
  const bool active = pl < np;
  const int mom = active ? pd.mom[group][pl] : 0;
  const bool is_w = mom == kMomW;
  const int rank = is_w ? 0 : pd.rank[mom];
  int comp[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) comp[k] = is_w ? 0 : pd.idx[mom][k];

  const T *fx = r_f, *fy = r_f + fstride, *fz = r_f + 2 * fstride, *t0p = r_f + 3 * fstride,
          *twp = r_f + 4 * fstride, *hxp = r_f + 5 * fstride, *hyp = r_f + 6 * fstride, *hzp = r_f + 7 * fstride;
  double *myacc = acc + pl * kPlaneStride;
  const int wave = threadIdx.x >> 6;
  constexpr int nwaves = kGridThreads / 64;

  constexpr int kStage = Staged<T>::n;
  for (int cbase = 0; cbase < total; cbase += kStage) {
    const int n = min(kStage, total - cbase);
    __syncthreads();  // previous chunk consumed
    // stage the chunk's records in LDS: coalesced runs of the sorted arrays
    for (int i = threadIdx.x; i < n; i += kGridThreads) {
      const int it = cbase + i;
      int lo = 0, hi = kGridThreads;  // seg_pref[lo] <= it < seg_pref[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg_pref[mid] <= it) lo = mid; else hi = mid;
      }
      const int o = seg_start[lo] + (it - seg_pref[lo]);
      st.cell[i] = r_cell[o];
      st.f[0][i] = fx[o]; st.f[1][i] = fy[o]; st.f[2][i] = fz[o];
      st.t0[i] = t0p[o]; st.tw[i] = twp[o];
      st.h[0][i] = hxp[o]; st.h[1][i] = hyp[o]; st.h[2][i] = hzp[o];
    }
    __syncthreads();
    if (!active) continue;
    for (int base = 2 * wave; base < n; base += 2 * nwaves) {
      const int i = base + half;
      if (i >= n) continue;
      const int pc = st.cell[i];
      // offset of the object's cell from the tile origin, unwrapped into the
      // grown range [-HI, 7 + LO] (the periodic seam is crossed at most once)
      int rx = (pc >> 20) - X0, ry = ((pc >> 10) & 1023) - Y0, rz = (pc & 1023) - Z0;
      rx += rx < -HI ? N : (rx > kGX - 1 + LO ? -N : 0);
      ry += ry < -HI ? N : (ry > kGY - 1 + LO ? -N : 0);
      rz += rz < -HI ? N : (rz > kGZ - 1 + LO ? -N : 0);
      const T hx = st.h[0][i], hy = st.h[1][i], hz = st.h[2][i];
      T t = is_w ? st.tw[i] : st.t0[i];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < rank) t *= comp[k] == 0 ? hx : (comp[k] == 1 ? hy : hz);
      T wx[P], wy[P], wz[P];
      const int nx0 = axis_weights<T, P, TWIN>(rx, st.f[0][i], wx);
      const int ny0 = axis_weights<T, P, TWIN>(ry, st.f[1][i], wy);
      const int nz0 = axis_weights<T, P, TWIN>(rz, st.f[2][i], wz);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        const int lx = nx0 + a;
        if ((unsigned)lx >= (unsigned)kGX) continue;
#pragma unroll
        for (int b = 0; b < P; ++b) {
          const int ly = ny0 + b;
          if ((unsigned)ly >= (unsigned)kGY) continue;
          const T wab = wx[a] * wy[b] * t;
#pragma unroll
          for (int c = 0; c < P; ++c) {
            const int lz = nz0 + c;
            if ((unsigned)lz >= (unsigned)kGZ) continue;
            atomicAdd(&myacc[(lx * kGY + ly) * kGZ + lz], (double)(wab * wz[c]));
          }
        }
      }
    }
  }
}

template <typename T, int P>
__global__ __launch_bounds__(kGridThreads) void k_grid(const int *__restrict__ offs, const int *__restrict__ r_cell,
                                                        const T *__restrict__ r_f, size_t fstride, int N,
                                                        const int *__restrict__ tile_cnt, PlaneDesc pd, T *planar,
                                                        long long plane_stride) {
  extern __shared__ unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);  // [n_planes][kPlaneStride]
  __shared__ int seg_start[kMaxSeg];
  __shared__ int seg_pref[kMaxSeg + 1];
  __shared__ Staged<T> st;
  __shared__ int any_obj;
  const int group = blockIdx.x % pd.n_groups;
  const int tile = blockIdx.x / pd.n_groups;
  const int ntx = N / kGX, nty = N / kGY, ntz = N / kGZ;
  const int tx = tile / (ntz * nty), ty = (tile / ntz) % nty, tz = tile % ntz;
  const int X0 = tx * kGX, Y0 = ty * kGY, Z0 = tz * kGZ;
  const int np = pd.n_planes[group];

  // objects can only come from this tile and its 26 neighbours (the kernel
  // support is shorter than a tile side)
  if (threadIdx.x == 0) any_obj = 0;
  __syncthreads();
  if (threadIdx.x < 27) {
    const int dx = threadIdx.x / 9 - 1, dy = (threadIdx.x / 3) % 3 - 1, dz = threadIdx.x % 3 - 1;
    const int nx = (tx + dx + ntx) % ntx, ny = (ty + dy + nty) % nty, nz = (tz + dz + ntz) % ntz;
    if (tile_cnt[(nx * nty + ny) * ntz + nz] > 0) any_obj = 1;
  }
  __syncthreads();
  if (any_obj) {
    for (int i = threadIdx.x; i < np * kPlaneStride; i += kGridThreads) acc[i] = 0.0;
    // (the segment scan inside starts with a barrier)
    if (pd.twin[group])
      grid_tile<T, P, true>(offs, r_cell, r_f, fstride, N, pd, group, X0, Y0, Z0, acc, seg_start, seg_pref, st);
    else
      grid_tile<T, P, false>(offs, r_cell, r_f, fstride, N, pd, group, X0, Y0, Z0, acc, seg_start, seg_pref, st);
    __syncthreads();
  }
  // write the planes of the tile as contiguous z-runs of the planar output
  for (int p = 0; p < np; ++p) {
    T *dst = planar + (long long)(2 * pd.out_slot[group][p] + pd.out_im[group][p]) * plane_stride;
    const double *src = acc + p * kPlaneStride;
    for (int idx = threadIdx.x; idx < kGCells; idx += kGridThreads) {
      const int lz = idx % kGZ, ly = (idx / kGZ) % kGY, lx = idx / (kGZ * kGY);
      const long long g = ((long long)(X0 + lx) * N + (Y0 + ly)) * N + (Z0 + lz);
      dst[g] = any_obj ? (T)src[idx] : T(0);
    }
  }
  if (group == 0 && pd.zero_slot >= 0) {
    T *dst = planar + (long long)(2 * pd.zero_slot + 1) * plane_stride;
    for (int idx = threadIdx.x; idx < kGCells; idx += kGridThreads) {
      const int lz = idx % kGZ, ly = (idx / kGZ) % kGY, lx = idx / (kGZ * kGY);
      const long long g = ((long long)(X0 + lx) * N + (Y0 + ly)) * N + (Z0 + lz);
      dst[g] = T(0);
    }
  }
}

static PlaneDesc make_planes(const frsd_plan *pl) {
  PlaneDesc pd{};
  const SlotDesc &sd = pl->slots;
  const MomentTable &tab = moment_table();
  for (int i = 0; i < kMaxMom; ++i) {
    pd.rank[i] = tab.rank[i];
    for (int k = 0; k < 4; ++k) pd.idx[i][k] = tab.idx[i][k];
  }
  pd.zero_slot = -1;
  if (pl->p.interlace) {
    pd.n_groups = 2;
    for (int g = 0; g < 2; ++g) {
      pd.twin[g] = g;
      pd.n_planes[g] = sd.n_mom;
      for (int m = 0; m < sd.n_mom; ++m) {
        pd.mom[g][m] = sd.mom_id[m];
        pd.out_slot[g][m] = m;
        pd.out_im[g][m] = g;
      }
    }
  } else {
    pd.n_groups = 1;
    pd.twin[0] = 0;
    pd.n_planes[0] = sd.n_mom;
    for (int m = 0; m < sd.n_mom; ++m) {
      pd.mom[0][m] = sd.mom_id[m];
      pd.out_slot[0][m] = m / 2;
      pd.out_im[0][m] = m % 2;
    }
    if (sd.n_mom % 2) pd.zero_slot = sd.n_mom / 2;
  }
  return pd;
}

template <typename T, int P>
static int launch_grid(frsd_plan *pl, void *ws, hipStream_t s) {
  const Layout &L = pl->L;
  const int N = pl->N;
  const size_t nobj = (size_t)(pl->p.max_objects > 0 ? pl->p.max_objects : 1);
  const size_t cstride = sorted_stride(nobj, 4);
  const size_t fstride = sorted_stride(nobj, sizeof(T)) / sizeof(T);
  const PlaneDesc pd = make_planes(pl);
  const int npmax = pd.n_planes[0];
  const size_t shmem = sizeof(double) * (size_t)npmax * kPlaneStride;
  auto kern = k_grid<T, P>;
  FRSD_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const unsigned ntiles = (unsigned)((N / kGX) * (N / kGY) * (N / kGZ));
  FRSD_TIMED("grid", s, hipLaunchKernelGGL(kern, dim3(ntiles * pd.n_groups), dim3(kGridThreads), shmem, s,
                                           ws_ptr<const int>(ws, L.cnt), ws_ptr<const int>(ws, L.sorted),
                                           ws_ptr<const T>(ws, L.sorted + cstride), fstride, N,
                                           ws_ptr<const int>(ws, L.tile_cnt), pd, ws_ptr<T>(ws, L.planar),
                                           (long long)N * N * N));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template <typename T>
int run_mesh_assign(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                    hipStream_t s) {
  int rc = ingest_and_sort<T>(pl, ws, gal, ran, alpha, s);
  if (rc) return rc;
  switch (pl->p.order) {
    case 1: rc = launch_grid<T, 1>(pl, ws, s); break;
    case 2: rc = launch_grid<T, 2>(pl, ws, s); break;
    default: rc = launch_grid<T, 3>(pl, ws, s); break;
  }
  if (rc) return rc;
  return fft3d_forward<T>(pl->fft_n, ws_ptr<void>(ws, pl->L.tw_fwd), ws_ptr<const void>(ws, pl->L.planar),
                          ws_ptr<void>(ws, pl->L.mesh), pl->slots.n_slot, pl->nmax, s);
}

template int run_mesh_assign<float>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                    hipStream_t);
template int run_mesh_assign<double>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                     hipStream_t);

}  // namespace frsd
