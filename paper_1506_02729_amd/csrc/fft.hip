// Batched 3D complex FFTs of the packed moment meshes (step a4).
//
// Each moment mesh is a complex N^3 array [x][y][z] (z fastest) whose real
// part holds one real assignment plane and whose imaginary part holds a
// second one (the interlaced twin, or the next moment without
// interlacing), so one complex transform yields two real-input transforms.
// The 3D forward DFT sum_i m[i] exp(-2 pi i n.i / N) is done as three
// passes of 1D transforms along z, y and x.  A workgroup stages P pencils
// in LDS: for the z pass the pencils are contiguous rows; for the y and x
// passes the P pencils are P consecutive z columns, so every global row
// access is a contiguous run of P complex values.  Common lengths get a
// kernel with the length and radix schedule fixed at compile time.
//
// Pruning: the binning step reads only modes whose signed frequencies all
// satisfy |n_d| <= n_max (the largest component of any mode in a bin), so
// each pass keeps only those frequencies of the axis it transforms: the z
// pass writes kept z, the y pass transforms only kept-z columns and writes
// kept y, the x pass transforms only columns with kept y and z and writes
// kept x.  Kept indices form two runs, [0, ka) and [N - kb, N).  Entries
// outside the kept set are never written and never read.
//
// Sphere: the binning reads only modes with |n|^2 <= m2max.  The y pass
// writes only (n_y, n_z) with n_y^2 + n_z^2 <= m2max, the x pass transforms
// only those columns and writes only modes inside the sphere.
//
// Survey sparsity: a survey fills a fraction of the box, and every node
// column (x, y) out of reach of all objects (colmask 0) is zero in every
// plane, as is every x slab with no such column (xmask 0).  The z pass skips
// those rows (no read, no write), the y pass takes them as zero and skips
// empty x slabs, and the x pass takes empty slabs as zero.  Exact zeros in
// the butterflies change no rounding, so the result is the dense one.
#include <algorithm>

#include "device.h"
#include "frsd_internal.h"

namespace frsd {

// streaming store of one complex value (not kept in the caches)
template <typename C>
__device__ __forceinline__ void st_nt(C *p, C v) {
  using T = decltype(v.x);
  typedef T V2 __attribute__((ext_vector_type(2)));
  V2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<V2 *>(p));
}


struct Keep {
  int ka, kb;    // kept runs [0, ka) and [N - kb, N) (kb = 0: one run [0, ka))
  int nba, nbb;  // workgroups of P columns over each run
  int m2max;     // largest |n|^2 read after the transform (compiled-length passes)
};

// Signed frequency of index e of a length-N axis.
__device__ __forceinline__ int sfreq(int e, int N) { return 2 * e <= N ? e : e - N; }

__device__ __forceinline__ bool kept(int e, int N, const Keep &k) { return e < k.ka || e >= N - k.kb; }

// Column block b of the kept runs: first column and number of columns.
__device__ __forceinline__ void column_block(int b, int P, int N, const Keep &k, int &z0, int &nz) {
  if (b < k.nba) {
    z0 = b * P;
    nz = min(P, k.ka - z0);
  } else {
    z0 = N - k.kb + (b - k.nba) * P;
    nz = min(P, N - z0);
  }
}

// Run-time length kernel (lengths without a compiled kernel).  AXIS 2
// reads the planar real arrays `planar` (re, im of mesh b at arrays 2b,
// 2b+1) and writes `data`; AXIS 1 and 0 work in place on `data`.
// Grid: AXIS 2 (N^2 / P rows, mesh); AXIS 1 (x * (nba + nbb) + column
// block, mesh); AXIS 0 (kept y * (nba + nbb) + column block, mesh), with
// mesh = request * n_mesh + mesh of the request.
template <typename T, int AXIS>
__global__ __launch_bounds__(FftTune<T>::threads) void k_fft_axis(cplx_t<T> *data, const T *planar, int N, int P,
                                                           StageList st, const cplx_t<T> *tw_g,
                                                           long long batch_stride, Keep keep,
                                                           const uint8_t *__restrict__ colmask,
                                                           const uint8_t *__restrict__ xmask, Batch bt,
                                                           int n_mesh) {
  using C = cplx_t<T>;
  constexpr int NT = FftTune<T>::threads;
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + N;
  const int ld = N + 1;

  const int req = bt.n > 1 ? (int)blockIdx.y / n_mesh : 0, mi = (int)blockIdx.y - req * n_mesh;
  const long long dr = bt.n > 1 ? bt.delta[req] : 0;
  colmask = moved(colmask, dr);
  xmask = moved(xmask, dr);
  C *mesh = moved(data, dr) + (long long)mi * batch_stride;
  const long long NN = (long long)N * N;

  if (AXIS == 2) {
    const long long q0 = (long long)blockIdx.x * P;
    const int npen = (int)((q0 + P <= NN) ? P : (NN - q0));
    int any = 0;
    for (int p = threadIdx.x; p < npen; p += NT) any |= colmask[q0 + p];
    if (!__syncthreads_or(any)) return;  // every row of the block is empty
    for (int i = threadIdx.x; i < N; i += NT) tw[i] = tw_g[i];
    const int tot = npen * N;
    const T *re = moved(planar, dr) + 2 * (long long)mi * batch_stride + q0 * N;
    const T *im = re + batch_stride;
    for (int f = threadIdx.x; f < tot; f += NT) {
      const int p = f / N, e = f - p * N;
      lds[p * ld + e] = colmask[q0 + p] ? cmake<C>(re[f], im[f]) : cmake<C>(T(0), T(0));
    }
    __syncthreads();
    lds_fft<C, false, NT, FftTune<T>::pn>(lds, ld, N, npen, st, tw);
    C *dst = mesh + q0 * N;
    for (int f = threadIdx.x; f < tot; f += NT) {
      const int p = f / N, e = f - p * N;
      if (colmask[q0 + p] && kept(e, N, keep)) dst[f] = lds[p * ld + e];
    }
    return;
  }

  const int nzb = keep.nba + keep.nbb;
  const int outer_i = blockIdx.x / nzb;
  int z0, npen;
  column_block(blockIdx.x - outer_i * nzb, P, N, keep, z0, npen);
  const int outer = (AXIS == 1) ? outer_i : (outer_i < keep.ka ? outer_i : N - keep.kb + (outer_i - keep.ka));
  if (AXIS == 1 && !xmask[outer]) return;  // empty x slab: its y-pass output is never read
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = tw_g[i];
  const long long es = (AXIS == 1) ? N : NN;
  C *col = mesh + ((AXIS == 1) ? (long long)outer * NN : (long long)outer * N) + z0;
  // rows read as zero: empty node columns (y pass), empty x slabs (x pass)
  const uint8_t *live = (AXIS == 1) ? colmask + (long long)outer * N : xmask;
  for (int f = threadIdx.x; f < P * N; f += NT) {
    const int e = f / P, p = f - e * P;
    if (p < npen) lds[p * ld + e] = live[e] ? col[e * es + p] : cmake<C>(T(0), T(0));
  }
  __syncthreads();
  lds_fft<C, false, NT, FftTune<T>::pn>(lds, ld, N, npen, st, tw);
  for (int f = threadIdx.x; f < P * N; f += NT) {
    const int e = f / P, p = f - e * P;
    if (p < npen && kept(e, N, keep)) col[e * es + p] = lds[p * ld + e];
  }
}

// Compiled-length kernels on the register-resident core (fft_pencils).
// Row pass (z): P_ROW contiguous rows per workgroup.  Column passes (y, x):
// P_COL consecutive z columns per workgroup, so every global access is a run
// of P_COL complex values.
template <typename T> struct FwdTune {
  static constexpr int nt_row = 256, nt_col = sizeof(T) == 4 ? 512 : 256;
  static constexpr int row_elems = sizeof(T) == 4 ? 8192 : 2048;  // rows per workgroup x length (16 rows of 512 measured 6% faster than 8)
  static constexpr int p_col = sizeof(T) == 4 ? 16 : 8;
};
template <typename T, int LEN> constexpr int p_row() {
  return fit_pencils<cplx_t<T>, LEN, (FwdTune<T>::row_elems / LEN > 0 ? FwdTune<T>::row_elems / LEN : 1)>();
}
// column pencils: 16 (FP32) or 8 (FP64), fewer where the LDS would not fit (N >= 768)
template <typename T, int LEN> constexpr int p_col() { return fit_pencils<cplx_t<T>, LEN, FwdTune<T>::p_col>(); }

// Row pass (z), persistent: a fixed grid of workgroups walks the groups of
// P_ROW rows, mesh by mesh (every request's n_mesh meshes), and moves on at
// once from groups whose rows are all empty, so the empty part of the box
// costs no workgroup launches.

template <typename T, int LEN>
__global__ __launch_bounds__(FwdTune<T>::nt_row) void k_fft_row(cplx_t<T> *data, const T *planar,
                                                                const cplx_t<T> *tw_g, long long batch_stride,
                                                                Keep keep, const uint8_t *__restrict__ colmask,
                                                                int n_mesh, Batch bt) {
  using C = cplx_t<T>;
  constexpr int P = p_row<T, LEN>(), NT = FwdTune<T>::nt_row;
  constexpr long long NN = (long long)LEN * LEN;
  constexpr long long NG = (NN + P - 1) / P;  // row groups per mesh
  __shared__ unsigned char live[P];            // rows of the current group that hold data
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + LEN;
  for (int i = threadIdx.x; i < LEN; i += NT) tw[i] = tw_g[i];
  const int n_all = n_mesh * bt.n;
  for (long long it = blockIdx.x; it < NG * n_all; it += gridDim.x) {
    const long long grp = it / n_all;
    const int slot = (int)(it - grp * n_all);
    const int req = slot / n_mesh, mi = slot - req * n_mesh;
    // (a single request loads no distance: nothing waits on it before the mask loads)
    const long long dr = bt.n > 1 ? bt.delta[req] : 0;
    const uint8_t *cm = moved(colmask, dr);
    const long long q0 = grp * P;
    const int npen = (int)((q0 + P <= NN) ? P : (NN - q0));
    int any = 0;
    for (int p = threadIdx.x; p < P; p += NT) {
      live[p] = p < npen ? cm[q0 + p] : 0;
      any |= live[p];
    }
    if (!__syncthreads_or(any)) continue;  // (the barrier also publishes tw and live)
    const T *re = moved(planar, dr) + 2 * (long long)mi * batch_stride + q0 * LEN;
    const T *im = re + batch_stride;
    C *dst = moved(data, dr) + (long long)mi * batch_stride + q0 * LEN;
    fft_pencils<C, LEN, P, NT, false, false>(
        lds, tw, npen,
        [&](int p, int e) {
          return live[p] ? cmake<C>(re[p * LEN + e], im[p * LEN + e]) : cmake<C>(T(0), T(0));
        },
        [&](int p, int e, C v) {
          if (live[p] && kept(e, LEN, keep)) st_nt(&dst[p * LEN + e], v);
        });
    __syncthreads();  // pencils and live are rewritten by the next group
  }
}

// Column passes (y, x): grid (column blocks, mesh), mesh = request *
// n_mesh + mesh of the request.
template <typename T, int AXIS, int LEN>
__global__ __launch_bounds__(FwdTune<T>::nt_col) void k_fft_col(cplx_t<T> *data, const cplx_t<T> *tw_g,
                                                                long long batch_stride, Keep keep,
                                                                const uint8_t *__restrict__ colmask,
                                                                const uint8_t *__restrict__ xmask, Batch bt,
                                                                int n_mesh) {
  using C = cplx_t<T>;
  constexpr int P = p_col<T, LEN>(), NT = FwdTune<T>::nt_col;
  constexpr long long NN = (long long)LEN * LEN;
  const int req = bt.n > 1 ? (int)blockIdx.y / n_mesh : 0, mi = (int)blockIdx.y - req * n_mesh;
  const long long dr = bt.n > 1 ? bt.delta[req] : 0;
  colmask = moved(colmask, dr);
  xmask = moved(xmask, dr);
  const int nzb = keep.nba + keep.nbb;
  const int outer_i = blockIdx.x / nzb;
  int z0, npen;
  column_block(blockIdx.x - outer_i * nzb, P, LEN, keep, z0, npen);
  const int outer = (AXIS == 1) ? outer_i : (outer_i < keep.ka ? outer_i : LEN - keep.kb + (outer_i - keep.ka));
  if (AXIS == 1 && !xmask[outer]) return;  // empty x slab: its y-pass output is never read
  // x pass: n_y of the block and the smallest n_z^2 of its columns; a block
  // wholly outside the sphere's (n_y, n_z) disc has nothing to transform
  const int ny2 = (AXIS == 0) ? sfreq(outer, LEN) * sfreq(outer, LEN) : 0;
  if (AXIS == 0) {
    int nz2min = 1 << 30;
    for (int p = 0; p < npen; ++p) nz2min = min(nz2min, sfreq(z0 + p, LEN) * sfreq(z0 + p, LEN));
    if (ny2 + nz2min > keep.m2max) return;
  }
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + LEN;
  // rows read as zero: empty node columns (y pass), empty x slabs (x pass);
  // the flags sit in LDS so that no load waits on another
  __shared__ unsigned char live[LEN];
  const uint8_t *lsrc = (AXIS == 1) ? colmask + (long long)outer * LEN : xmask;
  for (int i = threadIdx.x; i < LEN; i += NT) {
    tw[i] = tw_g[i];
    live[i] = lsrc[i];
  }
  __syncthreads();
  constexpr long long es = (AXIS == 1) ? LEN : NN;
  C *col = moved(data, dr) + (long long)mi * batch_stride +
           ((AXIS == 1) ? (long long)outer * NN : (long long)outer * LEN) + z0;
  // in place: every load happens in the first stage, every store in the last
  // (y pass: columns (n_y = e, n_z) outside the disc are not written; x
  // pass: those columns are read as zero and only modes inside the sphere
  // are written)
  fft_pencils<C, LEN, P, NT, false, true>(
      lds, tw, npen,
      [&](int p, int e) {
        const int nz = sfreq(z0 + p, LEN);
        const bool in = AXIS == 1 || ny2 + nz * nz <= keep.m2max;
        return live[e] && in ? col[e * es + p] : cmake<C>(T(0), T(0));
      },
      [&](int p, int e, C v) {
        const int nz = sfreq(z0 + p, LEN), ne = sfreq(e, LEN);
        if (kept(e, LEN, keep) && ny2 + nz * nz + ne * ne <= keep.m2max) st_nt(&col[e * es + p], v);
      });
}

static StageList stages_of(const FftLen &f) {
  StageList s{};
  s.nstage = f.nstage;
  for (int i = 0; i < f.nstage; ++i) s.radix[i] = f.radix[i];
  return s;
}

static Keep make_keep(int N, int P, int nmax) {
  // kept runs [0, nmax] and [N - nmax, N), widened to whole blocks of P columns
  Keep k{};
  k.m2max = 3 * N * N;  // no sphere limit unless the caller sets one
  k.ka = std::min(N, (nmax + 1 + P - 1) / P * P);
  const int b0 = std::max(k.ka, (N - nmax) / P * P);
  k.kb = N - b0;
  if (k.ka + k.kb >= N || 2 * nmax + 1 >= N) { k.ka = N; k.kb = 0; }
  k.nba = (k.ka + P - 1) / P;
  k.nbb = (k.kb + P - 1) / P;
  return k;
}

template <typename T, int LEN>
static int fft3d_forward_ct(const void *tw, const void *planar, void *mesh, int n_batch, int nmax, int m2max,
                            const uint8_t *colmask, const uint8_t *xmask, hipStream_t s, int row_grid,
                            const Batch &bt) {
  using C = cplx_t<T>;
  constexpr int PR = p_row<T, LEN>(), PC = p_col<T, LEN>();
  constexpr long long NN = (long long)LEN * LEN;
  Keep k = make_keep(LEN, PC, nmax);
  k.m2max = m2max;
  const unsigned nzb = (unsigned)(k.nba + k.nbb);
  constexpr size_t sh_row = fft_pencils_lds<C, LEN, PR>(), sh_col = fft_pencils_lds<C, LEN, PC>();
  FRSD_HIP(hipFuncSetAttribute((const void *)k_fft_row<T, LEN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_row));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_fft_col<T, 1, LEN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_col));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_fft_col<T, 0, LEN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_col));
  const long long bs = NN * LEN;
  const unsigned nm = (unsigned)(n_batch * bt.n);
  const dim3 gz((unsigned)row_grid), gy((unsigned)LEN * nzb, nm), gx((unsigned)(k.ka + k.kb) * nzb, nm);
  FRSD_TIMED("fft_z", s, hipLaunchKernelGGL((k_fft_row<T, LEN>), gz, dim3(FwdTune<T>::nt_row), sh_row, s, (C *)mesh,
                                            (const T *)planar, (const C *)tw, bs, k, colmask, n_batch, bt));
  FRSD_TIMED("fft_y", s, hipLaunchKernelGGL((k_fft_col<T, 1, LEN>), gy, dim3(FwdTune<T>::nt_col), sh_col, s, (C *)mesh,
                                            (const C *)tw, bs, k, colmask, xmask, bt, n_batch));
  FRSD_TIMED("fft_x", s, hipLaunchKernelGGL((k_fft_col<T, 0, LEN>), gx, dim3(FwdTune<T>::nt_col), sh_col, s, (C *)mesh,
                                            (const C *)tw, bs, k, colmask, xmask, bt, n_batch));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template <typename T>
static int fft3d_forward_rt(const FftLen &f, const void *tw, const void *planar, void *mesh, int n_batch, int nmax,
                            const uint8_t *colmask, const uint8_t *xmask, hipStream_t s, const Batch &bt) {
  using C = cplx_t<T>;
  const int N = f.n;
  const int P = FftTune<T>::pn / N;
  const long long NN = (long long)N * N;
  const Keep k = make_keep(N, P, nmax);
  const unsigned nzb = (unsigned)(k.nba + k.nbb);
  const size_t shmem = sizeof(C) * ((size_t)N + (size_t)P * (N + 1));
  const StageList st = stages_of(f);
  const long long bs = NN * N;
  FRSD_HIP(hipFuncSetAttribute((const void *)k_fft_axis<T, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_fft_axis<T, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_fft_axis<T, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const unsigned nm = (unsigned)(n_batch * bt.n);
  const dim3 gz((unsigned)((NN + P - 1) / P), nm), gy((unsigned)N * nzb, nm), gx((unsigned)(k.ka + k.kb) * nzb, nm);
  FRSD_TIMED("fft_z", s, hipLaunchKernelGGL((k_fft_axis<T, 2>), gz, dim3(FftTune<T>::threads), shmem, s, (C *)mesh,
                                            (const T *)planar, N, P, st, (const C *)tw, bs, k, colmask, xmask, bt,
                                            n_batch));
  FRSD_TIMED("fft_y", s, hipLaunchKernelGGL((k_fft_axis<T, 1>), gy, dim3(FftTune<T>::threads), shmem, s, (C *)mesh,
                                            (const T *)planar, N, P, st, (const C *)tw, bs, k, colmask, xmask, bt,
                                            n_batch));
  FRSD_TIMED("fft_x", s, hipLaunchKernelGGL((k_fft_axis<T, 0>), gx, dim3(FftTune<T>::threads), shmem, s, (C *)mesh,
                                            (const T *)planar, N, P, st, (const C *)tw, bs, k, colmask, xmask, bt,
                                            n_batch));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template <typename T>
int fft3d_forward(const FftLen &f, const void *tw, const void *planar, void *mesh, int n_batch, int nmax, int m2max,
                  const uint8_t *colmask, const uint8_t *xmask, hipStream_t s, int row_grid, const Batch &bt) {
  switch (f.n) {
#define FRSD_CASE(L) \
  case L: return fft3d_forward_ct<T, L>(tw, planar, mesh, n_batch, nmax, m2max, colmask, xmask, s, row_grid, bt);
    FRSD_FFT_LENGTHS(FRSD_CASE)
#undef FRSD_CASE
    default: return fft3d_forward_rt<T>(f, tw, planar, mesh, n_batch, nmax, colmask, xmask, s, bt);
  }
}

template int fft3d_forward<float>(const FftLen &, const void *, const void *, void *, int, int, int, const uint8_t *,
                                  const uint8_t *, hipStream_t, int, const Batch &);
template int fft3d_forward<double>(const FftLen &, const void *, const void *, void *, int, int, int, const uint8_t *,
                                   const uint8_t *, hipStream_t, int, const Batch &);

}  // namespace frsd
