// Triple-product contraction on the matrix cores (FP32 plans).
//
// The bispectrum triangle sums T_ell(b1,b2,b3) = sum_x F_{ell,b1}(x)
// F_{0,b2}(x) F_{0,b3}(x) (Sec. III.B eq. Factorize) are entries of one
// product C = A B summed over the M^3 cells x, with
//   rows  r = (b2, b3), b2 >= b3, r = b2 (b2 + 1) / 2 + b3:  A[r][x] = F_{0,b2}(x) F_{0,b3}(x)
//   cols  c = n_ell b1 + l (b1-major):                       B[x][c] = F_{ell_l,b1}(x)
// A is formed on the fly from the staged F_0 shells, so only the shell
// fields themselves are read from HBM.  Only the 16 x 16 tiles of C that
// hold a listed triangle are computed (block sparsity: b1 >= b2 and
// lo(b1) < hi(b2) + hi(b3) keep about a third of the tiles).
//
// Precision: each FP32 operand is split into two bfloat16 values,
// v = hi + lo with hi = bf16(v) and lo = bf16(v - hi), and each product is
// hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 (the dropped lo*lo
// term is below 2^-16 relative).  Accumulation is FP32 inside a
// workgroup's range of cells; workgroup partials are summed in FP64.
//
// Work split: 8 wavefronts per workgroup; wavefront w owns up to 16 output
// tiles ("jobs", sorted by row tile) in 64 accumulator registers.  Every
// workgroup covers all jobs for its own contiguous range of cells.
#include <vector>

#include "device.h"
#include "frsd_internal.h"

namespace frsd {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kXThreads = 512;
constexpr int kXWaves = kXThreads / 64;
constexpr int kXMaxJobs = 16;     // output tiles per wavefront
constexpr int kXCols = 112;       // columns (7 tiles)
constexpr int kXMaxRows = 768;    // pairs
constexpr int kXKC = 64;          // cells per LDS stage (2 MFMA k-steps)
constexpr int kXUPad = kXKC + 4;  // FP32 row stride of the staged F_0 shells
constexpr int kXBPad = kXKC + 8;  // bf16 row stride of the staged B operand
constexpr int kXMaxB = 37;        // bins

struct XJobs {
  uint8_t rt[kXWaves][kXMaxJobs];
  uint8_t ct[kXWaves][kXMaxJobs];
  int first[kXWaves];   // index of the wave's first job in the global job list
  int nj[kXWaves];
};

struct XArgs {
  long long ncell;
  long long cells_per_wg;
  int nb, n_ell, ncol, npair, njobs;
};

__device__ __forceinline__ void split_bf16(float v, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

__global__ __launch_bounds__(kXThreads, 2) void k_triple_mfma(const float *__restrict__ f, XArgs a, XJobs jobs,
                                                               const int2 *__restrict__ pairs,
                                                               float *__restrict__ part) {
  __shared__ float U[kXMaxB][kXUPad];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[kXCols][kXBPad];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[kXCols][kXBPad];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;     // row (A) / column (B) inside a 16-tile
  const int lk = lane >> 4;     // 8-wide k group of the 32-wide k-step
  const int nj = jobs.nj[wave];

  f32x4_t acc[kXMaxJobs];
#pragma unroll
  for (int j = 0; j < kXMaxJobs; ++j) acc[j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  // padding columns stay zero
  for (int i = threadIdx.x; i < (kXCols - a.ncol) * kXBPad; i += kXThreads) {
    const int c = a.ncol + i / kXBPad, k = i % kXBPad;
    Bh[c][k] = (__bf16)0.f;
    Bl[c][k] = (__bf16)0.f;
  }

  const long long c_begin = (long long)blockIdx.x * a.cells_per_wg;
  const long long c_end = min(a.ncell, c_begin + a.cells_per_wg);
  for (long long c0 = c_begin; c0 < c_end; c0 += kXKC) {
    const int len = (int)min((long long)kXKC, c_end - c0);
    __syncthreads();  // previous stage fully consumed
    for (int i = threadIdx.x; i < a.ncol * kXKC; i += kXThreads) {
      const int fl = i / kXKC, k = i - fl * kXKC;  // field fl = l * nb + b1
      const float v = (k < len) ? f[(long long)fl * a.ncell + c0 + k] : 0.f;
      const int l = fl / a.nb, b1 = fl - l * a.nb;
      const int col = b1 * a.n_ell + l;
      __bf16 h, lo;
      split_bf16(v, h, lo);
      Bh[col][k] = h;
      Bl[col][k] = lo;
      if (fl < a.nb) U[fl][k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kXKC / 32; ++ks) {
      const int k0 = ks * 32 + lk * 8;
      int cur_rt = -1;
      bf16x8_t ah, al;
#pragma unroll
      for (int j = 0; j < kXMaxJobs; ++j) {
        if (j < nj) {
          const int rt = jobs.rt[wave][j], ct = jobs.ct[wave][j];
          if (rt != cur_rt) {
            cur_rt = rt;
            const int r = rt * 16 + li;
            const bool ok = r < a.npair;
            const int2 p = pairs[ok ? r : 0];
            const float *u2 = &U[p.x][k0];
            const float *u3 = &U[p.y][k0];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float v = ok ? u2[e] * u3[e] : 0.f;
              __bf16 h, lo;
              split_bf16(v, h, lo);
              ah[e] = h;
              al[e] = lo;
            }
          }
          const bf16x8_t bh = *reinterpret_cast<const bf16x8_t *>(&Bh[ct * 16 + li][k0]);
          const bf16x8_t bl = *reinterpret_cast<const bf16x8_t *>(&Bl[ct * 16 + li][k0]);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[j], 0, 0, 0);
        }
      }
    }
  }

  // C[i][j] of a 16x16 tile: lane holds rows 4 (lane / 16) + v, column lane % 16
  float *out = part + (long long)blockIdx.x * a.njobs * 256;
#pragma unroll
  for (int j = 0; j < kXMaxJobs; ++j) {
    if (j < nj) {
      float *t = out + (long long)(jobs.first[wave] + j) * 256;
#pragma unroll
      for (int v = 0; v < 4; ++v) t[(4 * lk + v) * 16 + li] = acc[j][v];
    }
  }
}

// Sum over workgroups (FP64) of the partial tiles, one thread per entry.
__global__ void k_triple_mfma_reduce(const float *__restrict__ part, int nwg, int nvals, double *__restrict__ sum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvals) return;
  double s = 0.0;
  for (int w = 0; w < nwg; ++w) s += (double)part[(long long)w * nvals + i];
  sum[i] = s;
}

// Gather the listed outputs (triangle t, multipole l) from the job tiles.
__global__ void k_triple_mfma_gather(const double *__restrict__ dense, const int4 *__restrict__ otab,
                                     const int16_t *__restrict__ tile_job, int nb, int n_ell, int nout,
                                     double *__restrict__ tsum) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  const int4 e = otab[o];  // (field l * nb + b1, b2, b3)
  const int l = e.x / nb, b1 = e.x - l * nb;
  const int r = e.y * (e.y + 1) / 2 + e.z;
  const int c = b1 * n_ell + l;
  const int job = tile_job[(r / 16) * 7 + c / 16];
  tsum[o] = dense[(long long)job * 256 + (r % 16) * 16 + (c % 16)];
}

// Host-side job list: every (row tile, column tile) holding a listed output.
static bool make_jobs(const frsd_plan *pl, XJobs *jobs, std::vector<int16_t> *tile_job, int *njobs) {
  const int nb = pl->p.bk_nbins, ne = pl->n_ell;
  const int nrt = (nb * (nb + 1) / 2 + 15) / 16;
  std::vector<char> need((size_t)nrt * 7, 0);
  for (int64_t t = 0; t < pl->ntri; ++t) {
    const int b1 = pl->tri[3 * t], b2 = pl->tri[3 * t + 1], b3 = pl->tri[3 * t + 2];
    const int r = b2 * (b2 + 1) / 2 + b3;
    for (int l = 0; l < ne; ++l) need[(r / 16) * 7 + (b1 * ne + l) / 16] = 1;
  }
  std::vector<std::pair<int, int>> list;
  for (int rt = 0; rt < nrt; ++rt)
    for (int ct = 0; ct < 7; ++ct)
      if (need[rt * 7 + ct]) list.emplace_back(rt, ct);
  const int n = (int)list.size();
  if (n > kXWaves * kXMaxJobs) return false;
  *jobs = XJobs{};
  tile_job->assign((size_t)kXMaxRows / 16 * 7, (int16_t)-1);
  const int per = (n + kXWaves - 1) / kXWaves;
  for (int w = 0; w < kXWaves; ++w) {
    const int a = std::min(n, w * per), b = std::min(n, (w + 1) * per);
    jobs->first[w] = a;
    jobs->nj[w] = b - a;
    for (int j = a; j < b; ++j) {
      jobs->rt[w][j - a] = (uint8_t)list[j].first;
      jobs->ct[w][j - a] = (uint8_t)list[j].second;
      (*tile_job)[list[j].first * 7 + list[j].second] = (int16_t)j;
    }
  }
  *njobs = n;
  return true;
}

bool triple_mfma_supported(const frsd_plan *pl) {
  const int nb = pl->p.bk_nbins;
  if (nb > kXMaxB || nb * (nb + 1) / 2 > kXMaxRows || pl->n_ell * nb > kXCols) return false;
  XJobs j;
  std::vector<int16_t> tj;
  int n;
  return make_jobs(pl, &j, &tj, &n);
}

size_t triple_mfma_part_bytes(int nwg) { return sizeof(float) * (size_t)nwg * kXWaves * kXMaxJobs * 256; }
size_t triple_mfma_dense_bytes() {
  return sizeof(double) * (size_t)kXWaves * kXMaxJobs * 256 + sizeof(int16_t) * (kXMaxRows / 16) * 7 + 256;
}

int triple_mfma(frsd_plan *pl, void *ws, const float *fields, hipStream_t s) {
  const Layout &L = pl->L;
  XArgs a{};
  a.ncell = (long long)pl->M * pl->M * pl->M;
  a.nb = pl->p.bk_nbins;
  a.n_ell = pl->n_ell;
  a.ncol = pl->n_ell * a.nb;
  a.npair = a.nb * (a.nb + 1) / 2;
  XJobs jobs;
  std::vector<int16_t> tile_job;
  int njobs = 0;
  if (!make_jobs(pl, &jobs, &tile_job, &njobs)) return fail(FRSD_EINVAL, "too many contraction tiles");
  a.njobs = njobs;
  const int nwg = kTriMfmaBlocks;
  long long per = (a.ncell + nwg - 1) / nwg;
  per = (per + kXKC - 1) / kXKC * kXKC;
  a.cells_per_wg = per;
  double *dense = ws_ptr<double>(ws, L.tri_dense);
  const int16_t *tj = reinterpret_cast<const int16_t *>(dense + (size_t)kXWaves * kXMaxJobs * 256);
  FRSD_TIMED("triple", s, hipLaunchKernelGGL(k_triple_mfma, dim3(nwg), dim3(kXThreads), 0, s, fields, a, jobs,
                                             ws_ptr<const int2>(ws, L.pair_tab), ws_ptr<float>(ws, L.tri_part)));
  const int nvals = njobs * 256;
  FRSD_TIMED("tri_reduce", s,
             hipLaunchKernelGGL(k_triple_mfma_reduce, dim3((nvals + 255) / 256), dim3(256), 0, s,
                                ws_ptr<const float>(ws, L.tri_part), nwg, nvals, dense));
  FRSD_TIMED("tri_gather", s,
             hipLaunchKernelGGL(k_triple_mfma_gather, dim3((pl->n_out + 255) / 256), dim3(256), 0, s, dense,
                                ws_ptr<const int4>(ws, L.tri_tab), tj, a.nb, a.n_ell, pl->n_out,
                                ws_ptr<double>(ws, L.tri_sum)));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

// Uploads the (row tile, column tile) -> job table (synchronous; plan init).
int triple_mfma_upload(frsd_plan *pl, void *ws) {
  XJobs jobs;
  std::vector<int16_t> tile_job;
  int njobs = 0;
  if (!make_jobs(pl, &jobs, &tile_job, &njobs)) return fail(FRSD_EINVAL, "too many contraction tiles");
  double *dense = ws_ptr<double>(ws, pl->L.tri_dense);
  int16_t *tj = reinterpret_cast<int16_t *>(dense + (size_t)kXWaves * kXMaxJobs * 256);
  FRSD_HIP(hipMemcpy(tj, tile_job.data(), tile_job.size() * sizeof(int16_t), hipMemcpyHostToDevice));
  return FRSD_OK;
}

}  // namespace frsd
