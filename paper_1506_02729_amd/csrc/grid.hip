// Step a3: B-spline assignment of the moment meshes (Sec. III.A eq. mapFFT
// and the paragraph after it), and the driver of steps a1-a4.
//
// Owner-computes gather: a workgroup owns one 8 x 8 x 16 tile of output
// nodes for a group of complex mesh slots.  It walks the cells whose
// objects can reach the tile (the tile grown by the kernel support; objects
// are sorted by cell so each z-run of cells is one contiguous segment),
// accumulates every (object, node, moment) contribution that lands inside
// the tile with LDS atomics, and finally writes the tile once with plain
// coalesced stores.  No global atomics, no separate zero fill: empty tiles
// are written as zeros.
//
// Each complex slot holds two real planes: the real part is a moment on the
// main grid (nodes at integer grid coordinates); the imaginary part is the
// same moment on the interlaced twin grid (nodes at half-integer
// coordinates) or, without interlacing, the next moment on the main grid.
#include "device.h"
#include "frsd_internal.h"

namespace frsd {

constexpr int kTX = 8, kTY = 8, kTZ = 16, kTCells = kTX * kTY * kTZ;
constexpr int kGridThreads = 256;
constexpr int kMaxSeg = 256;

template <typename T>
int ingest_and_sort(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                    hipStream_t s);

struct MomArgs {
  int8_t idx[kMaxMom][4];
  int8_t rank[kMaxMom];
};

// Kernel weights of order P along one axis for an object at cell c with
// fractional offset f in [0, 1).  Writes the first node and P weights for
// the main grid (shift 0) or the twin grid (nodes at +1/2, i.e. u - 1/2).
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

template <typename T, int P, bool TWIN>
__device__ __forceinline__ void node_set(int c, T f, int t0, int tdim, int N, T *wt, int *loc) {
  const int first = axis_weights<T, P, TWIN>(c, f, wt);
#pragma unroll
  for (int a = 0; a < P; ++a) {
    int l = first + a - t0;
    l = (l % N + N) % N;  // periodic
    loc[a] = (l < tdim) ? l : -1;
  }
}

template <typename T, int P, int GMAX>
__global__ __launch_bounds__(kGridThreads) void k_grid(const int *__restrict__ offs, const int *__restrict__ r_cell,
                                                        const T *__restrict__ r_f, size_t fstride, int N,
                                                        SlotDesc sd, MomArgs mt, cplx_t<T> *mesh,
                                                        long long slot_stride) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char smem_raw[];
  T *acc = reinterpret_cast<T *>(smem_raw);  // [GMAX][2][kTCells]
  __shared__ int seg_start[kMaxSeg];
  __shared__ int seg_pref[kMaxSeg + 1];

  constexpr int LO = (P == 1) ? 0 : 1;   // nodes reached from cell c: [c - LO, c + HI]
  constexpr int HI = (P == 3) ? 2 : 1;
  const int ntz = N / kTZ, nty = N / kTY;
  const int b = blockIdx.x;
  const int X0 = (b / (ntz * nty)) * kTX, Y0 = ((b / ntz) % nty) * kTY, Z0 = (b % ntz) * kTZ;
  const int slot0 = blockIdx.y * GMAX;
  const int gs = min(GMAX, sd.n_slot - slot0);

  for (int i = threadIdx.x; i < GMAX * 2 * kTCells; i += kGridThreads) acc[i] = T(0);

  // cell segments: every (cx, cy) column of the grown tile, z-run split at the periodic seam
  const int nxr = kTX + LO + HI, nyr = kTY + LO + HI;
  const int nseg = nxr * nyr * 2;
  const int zlo = Z0 - HI, zhi = Z0 + kTZ - 1 + LO;
  int my_len = 0, my_start = 0;
  if (threadIdx.x < nseg) {
    const int part = threadIdx.x & 1;
    const int col = threadIdx.x >> 1;
    const int cx = ((X0 - HI + col / nyr) % N + N) % N;
    const int cy = ((Y0 - HI + col % nyr) % N + N) % N;
    int a, e;  // inclusive z range of this part, a > e means empty
    if (zlo < 0) { if (part == 0) { a = 0; e = zhi; } else { a = N + zlo; e = N - 1; } }
    else if (zhi >= N) { if (part == 0) { a = zlo; e = N - 1; } else { a = 0; e = zhi - N; } }
    else { if (part == 0) { a = zlo; e = zhi; } else { a = 1; e = 0; } }
    if (a <= e) {
      const long long rowc = ((long long)cx * N + cy) * N;
      my_start = offs[rowc + a];
      my_len = offs[rowc + e + 1] - my_start;
    }
  }
  // inclusive scan of segment lengths (nseg <= 256 = block size)
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

  const T *fx = r_f, *fy = r_f + fstride, *fz = r_f + 2 * fstride, *t0p = r_f + 3 * fstride,
          *twp = r_f + 4 * fstride, *hxp = r_f + 5 * fstride, *hyp = r_f + 6 * fstride, *hzp = r_f + 7 * fstride;

  for (int it = threadIdx.x; it < total; it += kGridThreads) {
    // segment containing flat index `it`
    int lo = 0, hi = kGridThreads;  // seg_pref[lo] <= it < seg_pref[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (seg_pref[mid] <= it) lo = mid; else hi = mid;
    }
    const int o = seg_start[lo] + (it - seg_pref[lo]);
    const int cell = r_cell[o];
    const int cz = cell % N, cy = (cell / N) % N, cx = cell / (N * N);
    const T f0 = fx[o], f1 = fy[o], f2 = fz[o];
    const T t0 = t0p[o], tw = twp[o];
    const T hv[3] = {hxp[o], hyp[o], hzp[o]};

    T wx[P], wy[P], wz[P];
    int lx[P], ly[P], lz[P];
    node_set<T, P, false>(cx, f0, X0, kTX, N, wx, lx);
    node_set<T, P, false>(cy, f1, Y0, kTY, N, wy, ly);
    node_set<T, P, false>(cz, f2, Z0, kTZ, N, wz, lz);
    T vx[P], vy[P], vz[P];
    int mx[P], my[P], mz[P];
    node_set<T, P, true>(cx, f0, X0, kTX, N, vx, mx);
    node_set<T, P, true>(cy, f1, Y0, kTY, N, vy, my);
    node_set<T, P, true>(cz, f2, Z0, kTZ, N, vz, mz);

    T tre[GMAX], tim[GMAX];
    bool shift[GMAX];
#pragma unroll
    for (int j = 0; j < GMAX; ++j) {
      tre[j] = T(0); tim[j] = T(0); shift[j] = false;
      if (j < gs) {
        const int sl = slot0 + j;
        int id = sd.mom_id[sd.re_mom[sl]];
        T v = (id == kMomW) ? tw : t0;
        if (id != kMomW)
          for (int k = 0; k < mt.rank[id]; ++k) v *= hv[mt.idx[id][k]];
        tre[j] = v;
        const int im = sd.im_mom[sl];
        if (im >= 0) {
          id = sd.mom_id[im];
          T u = (id == kMomW) ? tw : t0;
          if (id != kMomW)
            for (int k = 0; k < mt.rank[id]; ++k) u *= hv[mt.idx[id][k]];
          tim[j] = u;
          shift[j] = sd.im_shift[sl] != 0;
        }
      }
    }

    // main grid: real parts, and imaginary parts of unshifted slots
#pragma unroll
    for (int a = 0; a < P; ++a) {
      if (lx[a] < 0) continue;
#pragma unroll
      for (int bb = 0; bb < P; ++bb) {
        if (ly[bb] < 0) continue;
        const T wab = wx[a] * wy[bb];
        const int base = (lx[a] * kTY + ly[bb]) * kTZ;
#pragma unroll
        for (int c = 0; c < P; ++c) {
          if (lz[c] < 0) continue;
          const T W = wab * wz[c];
          const int idx = base + lz[c];
#pragma unroll
          for (int j = 0; j < GMAX; ++j) {
            if (j < gs) {
              atomicAdd(&acc[(2 * j) * kTCells + idx], W * tre[j]);
              if (!shift[j] && tim[j] != T(0)) atomicAdd(&acc[(2 * j + 1) * kTCells + idx], W * tim[j]);
            }
          }
        }
      }
    }
    // twin grid: imaginary parts of interlaced slots
    bool any_shift = false;
#pragma unroll
    for (int j = 0; j < GMAX; ++j) any_shift |= (j < gs) && shift[j];
    if (any_shift) {
#pragma unroll
      for (int a = 0; a < P; ++a) {
        if (mx[a] < 0) continue;
#pragma unroll
        for (int bb = 0; bb < P; ++bb) {
          if (my[bb] < 0) continue;
          const T wab = vx[a] * vy[bb];
          const int base = (mx[a] * kTY + my[bb]) * kTZ;
#pragma unroll
          for (int c = 0; c < P; ++c) {
            if (mz[c] < 0) continue;
            const T W = wab * vz[c];
            const int idx = base + mz[c];
#pragma unroll
            for (int j = 0; j < GMAX; ++j)
              if (j < gs && shift[j]) atomicAdd(&acc[(2 * j + 1) * kTCells + idx], W * tim[j]);
          }
        }
      }
    }
  }
  __syncthreads();

  // write the tile: consecutive threads cover consecutive z
  for (int idx = threadIdx.x; idx < kTCells; idx += kGridThreads) {
    const int lz0 = idx % kTZ, ly0 = (idx / kTZ) % kTY, lx0 = idx / (kTZ * kTY);
    const long long g = ((long long)(X0 + lx0) * N + (Y0 + ly0)) * N + (Z0 + lz0);
    for (int j = 0; j < gs; ++j) {
      C v;
      v.x = acc[(2 * j) * kTCells + idx];
      v.y = acc[(2 * j + 1) * kTCells + idx];
      mesh[(long long)(slot0 + j) * slot_stride + g] = v;
    }
  }
}

template <typename T, int P, int GMAX>
static int launch_grid(frsd_plan *pl, void *ws, hipStream_t s) {
  const Layout &L = pl->L;
  const int N = pl->N;
  const size_t nobj = (size_t)(pl->p.max_objects > 0 ? pl->p.max_objects : 1);
  const size_t cstride = sorted_stride(nobj, 4);
  const size_t fstride = sorted_stride(nobj, sizeof(T)) / sizeof(T);
  MomArgs mt{};
  const MomentTable &tab = moment_table();
  for (int i = 0; i < kMaxMom; ++i) {
    mt.rank[i] = tab.rank[i];
    for (int k = 0; k < 4; ++k) mt.idx[i][k] = tab.idx[i][k];
  }
  const size_t shmem = sizeof(T) * GMAX * 2 * kTCells;
  auto kern = k_grid<T, P, GMAX>;
  FRSD_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const unsigned ntiles = (unsigned)((N / kTX) * (N / kTY) * (N / kTZ));
  const unsigned ngroups = (unsigned)((pl->slots.n_slot + GMAX - 1) / GMAX);
  FRSD_TIMED("grid", s, hipLaunchKernelGGL(kern, dim3(ntiles, ngroups), dim3(kGridThreads), shmem, s, ws_ptr<const int>(ws, L.cnt),
                     ws_ptr<const int>(ws, L.sorted), ws_ptr<const T>(ws, L.sorted + cstride), fstride, N,
                     pl->slots, mt, ws_ptr<cplx_t<T>>(ws, L.mesh), (long long)N * N * N));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template <typename T>
int run_mesh_assign(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                    hipStream_t s) {
  int rc = ingest_and_sort<T>(pl, ws, gal, ran, alpha, s);
  if (rc) return rc;
  constexpr int G = sizeof(T) == 4 ? 8 : 4;
  switch (pl->p.order) {
    case 1: rc = launch_grid<T, 1, G>(pl, ws, s); break;
    case 2: rc = launch_grid<T, 2, G>(pl, ws, s); break;
    default: rc = launch_grid<T, 3, G>(pl, ws, s); break;
  }
  if (rc) return rc;
  return fft3d_forward<T>(pl->fft_n, ws_ptr<void>(ws, pl->L.tw_fwd), ws_ptr<void>(ws, pl->L.mesh),
                          pl->slots.n_slot, s);
}

template int run_mesh_assign<float>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                    hipStream_t);
template int run_mesh_assign<double>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                     hipStream_t);

}  // namespace frsd
