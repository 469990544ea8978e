// Triple-product contraction on the matrix cores: BF16 hi/lo for FP32 plans,
// FP64 MFMA for FP64 plans and for the N^T indicator sums of plan init.
//
// The bispectrum triangle sums T_ell(b1,b2,b3) = sum_x F_{ell,b1}(x)
// F_{0,b2}(x) F_{0,b3}(x) (Sec. III.B eq. Factorize) are entries of one
// product C = A B summed over the M^3 cells x, with
//   rows  r = the pairs (b2, b3), b2 >= b3, in the order of pair_rows below:  A[r][x] = F_{0,b2}(x) F_{0,b3}(x)
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
// Work split: 16 wavefronts per workgroup (one workgroup per CU); wavefront
// w owns up to 8 output tiles ("jobs", sorted by row tile) in 32 accumulator
// registers.  Every workgroup covers all jobs for its own contiguous range
// of cells.
#include <algorithm>
#include <vector>

#include "device.h"
#include "frsd_internal.h"

namespace frsd {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

constexpr int kXThreads = 1024;
constexpr int kXWaves = kXThreads / 64;
constexpr int kXMaxJobs = 8;      // output tiles per wavefront
constexpr int kXCols = 112;       // columns (7 tiles)
constexpr int kXMaxRows = 768;    // pairs
constexpr int kXKC = 64;          // cells per LDS stage (2 MFMA k-steps)
constexpr int kXUPad = kXKC + 4;  // FP32 row stride of the staged F_0 shells (16-byte aligned rows)
constexpr int kXBPad = kXKC + 16; // bf16 row stride of the staged B operand (16-byte aligned rows; 40 dwords measured fastest)
constexpr int kXMaxB = 37;        // bins
constexpr int kXMaxU = 2 * kXMaxB + 1;  // staged pair-product rows: F_0 and F_2 shells of every bin, then a zero row
constexpr int kXPf = (kXCols * (kXKC / 2) + kXThreads - 1) / kXThreads;  // cell pairs per thread per stage

struct XJobs {
  uint8_t rt[kXWaves][kXMaxJobs];
  uint8_t ct[kXWaves][kXMaxJobs];
  int first[kXWaves];   // index of the wave's first job in the global job list
  int nj[kXWaves];
};

// ncol: columns of the product (B fields); nload: fields read per stage
// (fields 0..nload-1 of the shell array); nu: fields staged for the pair
// products (0..nu-1).  t220: the columns are the F_2 fields (nb..2nb-1)
// and the pair rows hold F_{2,b2} F_{0,b3} (Sec. II.C eq. Bhexa2);
// otherwise field l nb + b1 is column b1 n_ell + l.
struct XArgs {
  long long ncell;
  long long cells_per_wg;
  int nb, n_ell, ncol, npair, njobs;
  int nload, nu, t220;
};

// Split of FP32 values into bfloat16 pairs, two values at once: one packed
// rounding gives both hi parts, which are widened back to FP32 by a byte
// permute (low half moved up) and a mask of the packed word (no second
// rounding per value), and the residuals x - hi are packed the same way.
// For a product a*b the residual is formed by an FMA, so it is exact.
__device__ __forceinline__ void widen2_bf16(bf16x2_t hi, float &h0, float &h1) {
  const unsigned u = __builtin_bit_cast(unsigned, hi);
  // bytes (0, 0, u.b0, u.b1): the low bfloat16 as an FP32 bit pattern
  h0 = __uint_as_float(__builtin_amdgcn_perm(u, u, 0x01000c0cu));
  h1 = __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ void split2_bf16(float x0, float x1, bf16x2_t &hi, bf16x2_t &lo) {
  hi = bf16x2_t{(__bf16)x0, (__bf16)x1};
  float h0, h1;
  widen2_bf16(hi, h0, h1);
  lo = bf16x2_t{(__bf16)(x0 - h0), (__bf16)(x1 - h1)};
}
__device__ __forceinline__ void split2_prod_bf16(float a0, float b0, float a1, float b1, bf16x2_t &hi,
                                                 bf16x2_t &lo) {
  hi = bf16x2_t{(__bf16)(a0 * b0), (__bf16)(a1 * b1)};
  float h0, h1;
  widen2_bf16(hi, h0, h1);
  lo = bf16x2_t{(__bf16)__builtin_fmaf(a0, b0, -h0), (__bf16)__builtin_fmaf(a1, b1, -h1)};
}

// One workgroup: a contiguous range of cells, all jobs.  Per stage of kXKC
// cells every field is read once from HBM (two adjacent cells per thread),
// split into bf16 hi/lo for the B operand, and the F_0 fields are kept in
// FP32 for the on-the-fly pair products.  Stages alternate between two LDS
// buffers: the global loads of stage s + 1 are issued before the MFMAs of
// stage s and stored into the other buffer after them.
// NU: staged rows (F_0 of every bin and a zero row for T_ell; F_0 and F_2
// of every bin and a zero row for T_220).
template <int NU>
__global__ __launch_bounds__(kXThreads) void k_triple_mfma(const float *__restrict__ f, XArgs a, XJobs jobs,
                                                               const int2 *__restrict__ pairs,
                                                               float *__restrict__ part) {
  // two stage buffers; row kXMaxB of U stays zero.  B2[buffer][0] holds the
  // hi parts, B2[buffer][1] the lo parts, at a fixed byte distance so one
  // address serves both reads.
  __shared__ __attribute__((aligned(16))) float U2[2][NU][kXUPad];
  __shared__ __attribute__((aligned(16))) __bf16 B2[2][2][kXCols][kXBPad];
  __shared__ uint32_t prs[kXMaxRows];  // byte offsets in U of rows b2 (low half) and b3 (high half)
  __shared__ uint8_t cmap[kXCols];     // staged field -> column (0xff: not a column)
  constexpr int kURow = kXUPad * 4, kUBuf = NU * kURow;  // bytes
  constexpr int kBRow = kXBPad * 2, kBHalf = kXCols * kBRow, kBBuf = 2 * kBHalf;
  constexpr int kZeroRow = NU - 1;
  static_assert(kZeroRow * kURow < 65536 && kBHalf < 65536, "offsets must fit 16 bits / the DS immediate");

  const int lane = threadIdx.x & 63;
  // wave-uniform (scalar) so the job table is read with scalar loads and the
  // row-tile test below is a scalar branch
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15;     // row (A) / column (B) inside a 16-tile
  const int lk = lane >> 4;     // 8-wide k group of the 32-wide k-step
  const int nj = jobs.nj[wave];
  // the wave's job tiles, read once into scalar registers
  // (scalar): row offset into prs, B byte offset of the column tile, and one
  // word whose bit j marks job j present and bit 8 + j marks job j as the
  // first of its row tile (jobs are sorted by row tile, so each row tile's
  // pair products are formed once per k-step)
  int jrt[kXMaxJobs], jcb[kXMaxJobs];
  int jbits = 0;
#pragma unroll
  for (int j = 0; j < kXMaxJobs; ++j) {
    jrt[j] = __builtin_amdgcn_readfirstlane((int)jobs.rt[wave][j]) * 16;
    jcb[j] = __builtin_amdgcn_readfirstlane((int)jobs.ct[wave][j]) * 16 * kBRow;
    if (j < nj) jbits |= 1 << j;
    if (j < nj && (j == 0 || jrt[j] != jrt[j - 1])) jbits |= 1 << (8 + j);
  }
  jbits = __builtin_amdgcn_readfirstlane(jbits);

  // one FP32 accumulator per job takes all three products (an MFMA whose
  // accumulator input is the previous MFMA's result issues back to back)
  f32x4_t acc[kXMaxJobs];
#pragma unroll
  for (int j = 0; j < kXMaxJobs; ++j) acc[j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  // rows past the last pair read the zero row of U
  for (int i = threadIdx.x; i < kXMaxRows; i += kXThreads) {
    uint32_t v = (uint32_t)(kZeroRow * kURow) * 0x10001u;
    if (i < a.npair) { const int2 p = pairs[i]; v = (uint32_t)(p.x * kURow) | ((uint32_t)(p.y * kURow) << 16); }
    prs[i] = v;
  }
  for (int i = threadIdx.x; i < 2 * kXUPad; i += kXThreads) U2[i / kXUPad][kZeroRow][i % kXUPad] = 0.f;
  for (int i = threadIdx.x; i < a.nload; i += kXThreads) {
    const int l = i / a.nb, b1 = i - l * a.nb;
    cmap[i] = a.t220 ? (uint8_t)(l == 1 ? b1 : 0xff) : (uint8_t)(b1 * a.n_ell + l);
  }
  // padding columns stay zero
  for (int i = threadIdx.x; i < 2 * (kXCols - a.ncol) * kXBPad; i += kXThreads) {
    const int bsel = i & 1, ii = i >> 1;
    const int c = a.ncol + ii / kXBPad, k = ii % kXBPad;
    B2[bsel][0][c][k] = (__bf16)0.f;
    B2[bsel][1][c][k] = (__bf16)0.f;
  }

  const long long c_begin = (long long)blockIdx.x * a.cells_per_wg;
  const long long c_end = min(a.ncell, c_begin + a.cells_per_wg);
  const int npe = a.nload * (kXKC / 2);  // cell pairs per stage
  const bool even = (a.ncell & 1) == 0;
  float2 pf[kXPf];

  auto load = [&](long long c0) {
    const int len = (int)min((long long)kXKC, c_end - c0);
#pragma unroll
    for (int q = 0; q < kXPf; ++q) {
      const int e = threadIdx.x + q * kXThreads;
      const int fl = e / (kXKC / 2), k = 2 * (e % (kXKC / 2));
      float2 v = make_float2(0.f, 0.f);
      if (e < npe) {
        const float *src = f + (long long)fl * a.ncell + c0 + k;
        if (k + 1 < len) {
          if (even) v = *reinterpret_cast<const float2 *>(src);
          else v = make_float2(src[0], src[1]);
        } else if (k < len) {
          v.x = src[0];
        }
      }
      pf[q] = v;
    }
  };
  auto store = [&](int bsel) {
    float(*U)[kXUPad] = U2[bsel];
    __bf16(*Bh)[kXBPad] = B2[bsel][0];
    __bf16(*Bl)[kXBPad] = B2[bsel][1];
#pragma unroll
    for (int q = 0; q < kXPf; ++q) {
      const int e = threadIdx.x + q * kXThreads;
      if (e < npe) {
        const int fl = e / (kXKC / 2), k = 2 * (e % (kXKC / 2));
        const int col = cmap[fl];
        if (col != 0xff) {
          bf16x2_t h, l;
          split2_bf16(pf[q].x, pf[q].y, h, l);
          *reinterpret_cast<bf16x2_t *>(&Bh[col][k]) = h;
          *reinterpret_cast<bf16x2_t *>(&Bl[col][k]) = l;
        }
        if (fl < a.nu) *reinterpret_cast<float2 *>(&U[fl][k]) = pf[q];
      }
    }
  };

  // stages alternate between the two buffers: the loads of stage s + 1 are
  // in flight during the MFMAs of stage s and are stored into the other
  // buffer after them; one barrier per stage
  if (c_begin < c_end) {
    load(c_begin);
    __syncthreads();  // tables above written
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (long long c0 = c_begin; c0 < c_end; c0 += kXKC, cur ^= 1) {
    const bool more = c0 + kXKC < c_end;
    if (more) load(c0 + kXKC);
    // the job word is re-read as an opaque scalar each stage so the job tests
    // stay scalar compare-and-branch (not hoisted as per-lane masks)
    int jb = jbits;
    asm volatile("" : "+s"(jb));
    const char *Ub = reinterpret_cast<const char *>(&U2[0][0][0]) + cur * kUBuf;
    const char *Bb = reinterpret_cast<const char *>(&B2[0][0][0][0]) + cur * kBBuf;
#pragma unroll
    for (int ks = 0; ks < kXKC / 32; ++ks) {
      const int k0 = ks * 32 + lk * 8;
      const char *Ul = Ub + 4 * k0;               // this lane's 8 cells of a U row
      const char *Bl_ = Bb + li * kBRow + 2 * k0;  // this lane's B row and 8 cells
      bf16x8_t ah, al;
#pragma unroll
      for (int j = 0; j < kXMaxJobs; ++j) {
        if ((jb >> j) & 1) {
          if ((jb >> (8 + j)) & 1) {
            const unsigned pr = prs[jrt[j] + li];
            const char *px = Ul + (pr & 0xffffu), *py = Ul + (pr >> 16);
            const float4 x0 = *reinterpret_cast<const float4 *>(px);
            const float4 x1 = *reinterpret_cast<const float4 *>(px + 16);
            const float4 y0 = *reinterpret_cast<const float4 *>(py);
            const float4 y1 = *reinterpret_cast<const float4 *>(py + 16);
            bf16x2_t h[4], l[4];
            split2_prod_bf16(x0.x, y0.x, x0.y, y0.y, h[0], l[0]);
            split2_prod_bf16(x0.z, y0.z, x0.w, y0.w, h[1], l[1]);
            split2_prod_bf16(x1.x, y1.x, x1.y, y1.y, h[2], l[2]);
            split2_prod_bf16(x1.z, y1.z, x1.w, y1.w, h[3], l[3]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              ah[2 * e] = h[e][0]; ah[2 * e + 1] = h[e][1];
              al[2 * e] = l[e][0]; al[2 * e + 1] = l[e][1];
            }
          }
          const char *pb = Bl_ + jcb[j];
          const bf16x8_t bh = *reinterpret_cast<const bf16x8_t *>(pb);
          const bf16x8_t bl = *reinterpret_cast<const bf16x8_t *>(pb + kBHalf);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[j], 0, 0, 0);
        }
      }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
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

// FP64 plans: the same block-sparse product on v_mfma_f64_16x16x4_f64, with
// no operand splitting.  Lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]
// of a 16 x 4 by 4 x 16 step and C[l / 16 + 4 v][l % 16] in accumulator
// register v.  A = F_0,b2 F_0,b3 is formed per lane from the staged
// monopole shells (one product per lane and k-step); partials stay FP64.
typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr int kZKC = 32;         // cells per LDS stage (8 MFMA k-steps of 4)
constexpr int kZPad = kZKC + 2;  // doubles per staged row: rows 68 dwords apart keep 8-byte reads conflict-free
constexpr int kZPf = (kXCols * (kZKC / 2) + kXThreads - 1) / kXThreads;  // cell pairs per thread per stage

template <int NU>
__global__ __launch_bounds__(kXThreads) void k_triple_mfma64(const double *__restrict__ f, XArgs a, XJobs jobs,
                                                               const int2 *__restrict__ pairs,
                                                               double *__restrict__ part) {
  __shared__ __attribute__((aligned(16))) double U2[2][NU][kZPad];  // the last row stays zero
  __shared__ __attribute__((aligned(16))) double B2[2][kXCols][kZPad];
  __shared__ uint32_t prs[kXMaxRows];  // U row offsets (doubles) of b2 (low half) and b3 (high half)
  __shared__ uint8_t cmap[kXCols];     // staged field -> column (0xff: not a column)
  constexpr int kZeroRow = NU - 1;
  static_assert(kZeroRow * kZPad < 65536, "row offsets must fit 16 bits");

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15;  // row of A, column of B and C
  const int lk = lane >> 4;  // k of A and B
  const int nj = jobs.nj[wave];
  int jrt[kXMaxJobs], jcb[kXMaxJobs];
  int jbits = 0;  // bit j: job j present; bit 8 + j: job j starts a row tile
#pragma unroll
  for (int j = 0; j < kXMaxJobs; ++j) {
    jrt[j] = __builtin_amdgcn_readfirstlane((int)jobs.rt[wave][j]) * 16;
    jcb[j] = __builtin_amdgcn_readfirstlane((int)jobs.ct[wave][j]) * 16 * kZPad;
    if (j < nj) jbits |= 1 << j;
    if (j < nj && (j == 0 || jrt[j] != jrt[j - 1])) jbits |= 1 << (8 + j);
  }
  jbits = __builtin_amdgcn_readfirstlane(jbits);
  f64x4_t acc[kXMaxJobs];
#pragma unroll
  for (int j = 0; j < kXMaxJobs; ++j) acc[j] = f64x4_t{0.0, 0.0, 0.0, 0.0};

  for (int i = threadIdx.x; i < kXMaxRows; i += kXThreads) {
    uint32_t v = (uint32_t)(kZeroRow * kZPad) * 0x10001u;
    if (i < a.npair) { const int2 p = pairs[i]; v = (uint32_t)(p.x * kZPad) | ((uint32_t)(p.y * kZPad) << 16); }
    prs[i] = v;
  }
  for (int i = threadIdx.x; i < 2 * kZPad; i += kXThreads) U2[i / kZPad][kZeroRow][i % kZPad] = 0.0;
  for (int i = threadIdx.x; i < a.nload; i += kXThreads) {
    const int l = i / a.nb, b1 = i - l * a.nb;
    cmap[i] = a.t220 ? (uint8_t)(l == 1 ? b1 : 0xff) : (uint8_t)(b1 * a.n_ell + l);
  }
  for (int i = threadIdx.x; i < 2 * (kXCols - a.ncol) * kZPad; i += kXThreads) {
    const int bsel = i & 1, ii = i >> 1;
    B2[bsel][a.ncol + ii / kZPad][ii % kZPad] = 0.0;
  }

  const long long c_begin = (long long)blockIdx.x * a.cells_per_wg;
  const long long c_end = min(a.ncell, c_begin + a.cells_per_wg);
  const int npe = a.nload * (kZKC / 2);  // cell pairs per stage
  const bool even = (a.ncell & 1) == 0;
  double2 pf[kZPf];
  auto load = [&](long long c0) {
    const int len = (int)min((long long)kZKC, c_end - c0);
#pragma unroll
    for (int q = 0; q < kZPf; ++q) {
      const int e = threadIdx.x + q * kXThreads;
      const int fl = e >> 4, k = 2 * (e & 15);
      double2 v = make_double2(0.0, 0.0);
      if (e < npe) {
        const double *src = f + (long long)fl * a.ncell + c0 + k;
        if (k + 1 < len) {
          if (even) v = *reinterpret_cast<const double2 *>(src);
          else v = make_double2(src[0], src[1]);
        } else if (k < len) {
          v.x = src[0];
        }
      }
      pf[q] = v;
    }
  };
  auto store = [&](int bsel) {
#pragma unroll
    for (int q = 0; q < kZPf; ++q) {
      const int e = threadIdx.x + q * kXThreads;
      if (e < npe) {
        const int fl = e >> 4, k = 2 * (e & 15);
        const int col = cmap[fl];
        if (col != 0xff) *reinterpret_cast<double2 *>(&B2[bsel][col][k]) = pf[q];
        if (fl < a.nu) *reinterpret_cast<double2 *>(&U2[bsel][fl][k]) = pf[q];
      }
    }
  };

  if (c_begin < c_end) {
    load(c_begin);
    __syncthreads();  // tables above written
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (long long c0 = c_begin; c0 < c_end; c0 += kZKC, cur ^= 1) {
    const bool more = c0 + kZKC < c_end;
    if (more) load(c0 + kZKC);
    int jb = jbits;
    asm volatile("" : "+s"(jb));  // job tests stay scalar branches
    const double *Ub = &U2[cur][0][0];
    const double *Bb = &B2[cur][0][0] + li * kZPad;
#pragma unroll
    for (int ks = 0; ks < kZKC / 4; ++ks) {
      const int kk = ks * 4 + lk;
      double av = 0.0;
#pragma unroll
      for (int j = 0; j < kXMaxJobs; ++j) {
        if ((jb >> j) & 1) {
          if ((jb >> (8 + j)) & 1) {
            const unsigned pr = prs[jrt[j] + li];
            av = Ub[(pr & 0xffffu) + kk] * Ub[(pr >> 16) + kk];
          }
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bb[jcb[j] + kk], acc[j], 0, 0, 0);
        }
      }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
  }

  double *out = part + (long long)blockIdx.x * a.njobs * 256;
#pragma unroll
  for (int j = 0; j < kXMaxJobs; ++j) {
    if (j < nj) {
      double *t = out + (long long)(jobs.first[wave] + j) * 256;
#pragma unroll
      for (int v = 0; v < 4; ++v) t[(lk + 4 * v) * 16 + li] = acc[j][v];
    }
  }
}


// Sum over workgroups (FP64) of the partial tiles, one thread per entry.
template <typename TP>
__global__ void k_triple_mfma_reduce(const TP *__restrict__ part, int nwg, int nvals, double *__restrict__ sum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvals) return;
  // four interleaved sums keep several loads in flight
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int w = 0;
  for (; w + 4 <= nwg; w += 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] += (double)part[(long long)(w + k) * nvals + i];
  }
  for (; w < nwg; ++w) s[0] += (double)part[(long long)w * nvals + i];
  sum[i] = (s[0] + s[1]) + (s[2] + s[3]);
}

// Gather the listed outputs (triangle t, multipole l) from the job tiles.
// tile_job holds the (row tile, column tile) -> job table followed by the
// row of each pair b2 (b2 + 1) / 2 + b3.
__global__ void k_triple_mfma_gather(const double *__restrict__ dense, const int4 *__restrict__ otab,
                                     const int16_t *__restrict__ tile_job, int nb, int n_ell, int nout,
                                     double *__restrict__ tsum) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  const int4 e = otab[o];  // (field l * nb + b1, b2, b3)
  const int l = e.x / nb, b1 = e.x - l * nb;
  const int r = tile_job[(kXMaxRows / 16) * 7 + e.y * (e.y + 1) / 2 + e.z];
  const int c = b1 * n_ell + l;
  const int job = tile_job[(r / 16) * 7 + c / 16];
  tsum[o] = dense[(long long)job * 256 + (r % 16) * 16 + (c % 16)];
}

// Row of each pair p = b2 (b2 + 1) / 2 + b3 in the product: pairs sorted by
// the last 16-column tile they need, then by their first needed column, so
// that the 16 pairs of a row tile need similar column ranges (103 instead
// of 114 output tiles for 37 bins).  Pairs in no listed triangle go last.
static std::vector<int> pair_rows(const frsd_plan *pl, int ne) {
  const int nb = pl->p.bk_nbins, np = nb * (nb + 1) / 2;
  std::vector<int> lo(np, 1 << 30), hi(np, 1 << 30);
  for (int64_t t = 0; t < pl->ntri; ++t) {
    const int b1 = pl->tri[3 * t], b2 = pl->tri[3 * t + 1], b3 = pl->tri[3 * t + 2];
    const int p = b2 * (b2 + 1) / 2 + b3;
    lo[p] = std::min(lo[p], b1 * ne);
    hi[p] = hi[p] == (1 << 30) ? b1 * ne + ne - 1 : std::max(hi[p], b1 * ne + ne - 1);
  }
  std::vector<int> order(np);
  for (int p = 0; p < np; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int ha = hi[a] / 16, hb = hi[b] / 16;
    return ha != hb ? ha < hb : lo[a] < lo[b];
  });
  std::vector<int> row(np);
  for (int r = 0; r < np; ++r) row[order[r]] = r;
  return row;
}

// Host-side job list: every (row tile, column tile) holding a listed output,
// for ne column groups (the multipoles of T_ell, or 1 for the N^T indicator
// sums).
static bool make_jobs(const frsd_plan *pl, int ne, XJobs *jobs, std::vector<int16_t> *tile_job, int *njobs) {
  const int nb = pl->p.bk_nbins;
  const int nrt = (nb * (nb + 1) / 2 + 15) / 16;
  const std::vector<int> row = pair_rows(pl, ne);
  std::vector<char> need((size_t)nrt * 7, 0);
  for (int64_t t = 0; t < pl->ntri; ++t) {
    const int b1 = pl->tri[3 * t], b2 = pl->tri[3 * t + 1], b3 = pl->tri[3 * t + 2];
    const int r = row[b2 * (b2 + 1) / 2 + b3];
    for (int l = 0; l < ne; ++l) need[(r / 16) * 7 + (b1 * ne + l) / 16] = 1;
  }
  std::vector<std::pair<int, int>> list;
  for (int rt = 0; rt < nrt; ++rt)
    for (int ct = 0; ct < 7; ++ct)
      if (need[rt * 7 + ct]) list.emplace_back(rt, ct);
  const int n = (int)list.size();
  if (n > kXWaves * kXMaxJobs) return false;
  *jobs = XJobs{};
  tile_job->assign((size_t)kXMaxRows / 16 * 7 + kXMaxRows, (int16_t)-1);
  for (size_t p = 0; p < row.size(); ++p) (*tile_job)[(size_t)kXMaxRows / 16 * 7 + p] = (int16_t)row[p];

  // Preferred: whole row tiles per wavefront (each row tile's pair products
  // formed by one wavefront only), balanced over the four SIMDs (wavefront w
  // runs on SIMD w % 4) by longest-first placement; the cost of a row tile
  // is 3 MFMAs per column tile plus about 3 MFMA-times of VALU for its pair
  // products.
  std::vector<std::vector<std::pair<int, int>>> wl(kXWaves);
  {
    std::vector<std::vector<std::pair<int, int>>> groups;
    for (const auto &e : list) {
      if (groups.empty() || groups.back()[0].first != e.first) groups.emplace_back();
      groups.back().push_back(e);
    }
    std::vector<int> order(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) order[g] = (int)g;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return groups[a].size() > groups[b].size(); });
    double simd_cost[4] = {0, 0, 0, 0};
    bool ok = true;
    for (int g : order) {
      const int len = (int)groups[g].size();
      int best_w = -1;
      double best_c = 1e300;
      for (int sidx = 0; sidx < 4; ++sidx) {
        int w_fit = -1;
        for (int k = 0; k < kXWaves / 4; ++k) {
          const int w = 4 * k + sidx;
          if ((int)wl[w].size() + len <= kXMaxJobs && (w_fit < 0 || wl[w].size() < wl[w_fit].size())) w_fit = w;
        }
        if (w_fit >= 0 && simd_cost[sidx] < best_c) { best_c = simd_cost[sidx]; best_w = w_fit; }
      }
      if (best_w < 0) { ok = false; break; }
      for (const auto &e : groups[g]) wl[best_w].push_back(e);
      simd_cost[best_w % 4] += 3.0 * len + 3.0;
    }
    if (ok)
      for (auto &w : wl) std::sort(w.begin(), w.end());
    else {
      // fallback: contiguous runs of the sorted list
      for (auto &w : wl) w.clear();
      const int base = n / kXWaves, extra = n % kXWaves;
      int a = 0;
      for (int w = 0; w < kXWaves; ++w) {
        const int b = a + base + (w < extra ? 1 : 0);
        for (int j = a; j < b; ++j) wl[w].push_back(list[j]);
        a = b;
      }
    }
  }
  int first = 0;
  for (int w = 0; w < kXWaves; ++w) {
    jobs->first[w] = first;
    jobs->nj[w] = (int)wl[w].size();
    for (int j = 0; j < (int)wl[w].size(); ++j) {
      jobs->rt[w][j] = (uint8_t)wl[w][j].first;
      jobs->ct[w][j] = (uint8_t)wl[w][j].second;
      (*tile_job)[wl[w][j].first * 7 + wl[w][j].second] = (int16_t)(first + j);
    }
    first += (int)wl[w].size();
  }
  *njobs = n;
  return true;
}

bool triple_mfma_supported(const frsd_plan *pl, int ne) {
  const int nb = pl->p.bk_nbins;
  if (nb > kXMaxB || nb * (nb + 1) / 2 > kXMaxRows || ne * nb > kXCols) return false;
  XJobs j;
  std::vector<int16_t> tj;
  int n;
  return make_jobs(pl, ne, &j, &tj, &n);
}
bool triple_mfma_supported(const frsd_plan *pl) { return triple_mfma_supported(pl, pl->n_ell); }

// Workgroup partials of the contractions that run on the matrix cores: nwg
// workgroups x the larger job count of T_ell and N^T x one 16 x 16 tile,
// FP64 (FP32 plans store FP32 partials in the same region).
size_t triple_mfma_part_bytes(const frsd_plan *pl, int nwg) {
  int most = 0;
  for (const int ne : {pl->n_ell, 1}) {
    XJobs j;
    std::vector<int16_t> tj;
    int n = 0;
    const int nb = pl->p.bk_nbins;
    if (nb > kXMaxB || nb * (nb + 1) / 2 > kXMaxRows || ne * nb > kXCols) continue;
    if (make_jobs(pl, ne, &j, &tj, &n)) most = std::max(most, n);
  }
  return sizeof(double) * (size_t)nwg * (size_t)most * 256;
}
size_t triple_mfma_dense_bytes() {
  return sizeof(double) * (size_t)kXWaves * kXMaxJobs * 256 + sizeof(int16_t) * ((kXMaxRows / 16) * 7 + kXMaxRows) +
         256;
}

// FP32 plans: T_ell (t220 = false) with the job tables at tri_dense and the
// pairs (F_0 b2, F_0 b3) at pair_tab, or T_220 (t220) with the job tables
// of the N^T sums (one column group) and the pairs (F_2 b2, F_0 b3).
static int triple_mfma_run(frsd_plan *pl, void *ws, const float *fields, bool t220, hipStream_t s) {
  const Layout &L = pl->L;
  XArgs a{};
  a.ncell = (long long)pl->M * pl->M * pl->M;
  a.nb = pl->p.bk_nbins;
  const int ne = t220 ? 1 : pl->n_ell;
  a.n_ell = ne;
  a.ncol = ne * a.nb;
  a.nload = t220 ? 2 * a.nb : a.ncol;
  a.nu = t220 ? 2 * a.nb : a.nb;
  a.t220 = t220 ? 1 : 0;
  a.npair = a.nb * (a.nb + 1) / 2;
  XJobs jobs;
  std::vector<int16_t> tile_job;
  int njobs = 0;
  if (!make_jobs(pl, ne, &jobs, &tile_job, &njobs)) return fail(FRSD_EINVAL, "too many contraction tiles");
  a.njobs = njobs;
  const int nwg = pl->tune.tri_wg;
  long long per = (a.ncell + nwg - 1) / nwg;
  per = (per + kXKC - 1) / kXKC * kXKC;
  a.cells_per_wg = per;
  double *dense = ws_ptr<double>(ws, t220 ? L.tri_dense_nt : L.tri_dense);
  const int16_t *tj = reinterpret_cast<const int16_t *>(dense + (size_t)kXWaves * kXMaxJobs * 256);
  auto kern = t220 ? k_triple_mfma<kXMaxU> : k_triple_mfma<kXMaxB + 1>;
  FRSD_TIMED(t220 ? "triple_220" : "triple", s,
             hipLaunchKernelGGL(kern, dim3(nwg), dim3(kXThreads), 0, s, fields, a, jobs,
                                ws_ptr<const int2>(ws, t220 ? L.pair_tab_220 : L.pair_tab),
                                ws_ptr<float>(ws, L.tri_part)));
  const int nvals = njobs * 256;
  FRSD_TIMED("tri_reduce", s,
             hipLaunchKernelGGL(k_triple_mfma_reduce<float>, dim3((nvals + 255) / 256), dim3(256), 0, s,
                                ws_ptr<const float>(ws, L.tri_part), nwg, nvals, dense));
  const int nout = t220 ? (int)pl->ntri : pl->n_out;
  const int4 *otab = ws_ptr<const int4>(ws, L.tri_tab) + (t220 ? pl->n_out : 0);
  FRSD_TIMED("tri_gather", s,
             hipLaunchKernelGGL(k_triple_mfma_gather, dim3((nout + 255) / 256), dim3(256), 0, s, dense, otab, tj,
                                a.nb, a.n_ell, nout, ws_ptr<double>(ws, t220 ? L.tri_sum220 : L.tri_sum)));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

int triple_mfma(frsd_plan *pl, void *ws, const float *fields, hipStream_t s) {
  return triple_mfma_run(pl, ws, fields, false, s);
}
int triple_mfma_220(frsd_plan *pl, void *ws, const float *fields, hipStream_t s) {
  return triple_mfma_run(pl, ws, fields, true, s);
}

// FP64 on the matrix cores: ne column groups of fields (n_ell for T_ell,
// 1 for the N^T indicator sums), with the job tables at `dense_off` and the
// pair table at `pair_off`; writes tsum[o] for the nout outputs of otab.
static int triple_mfma64_run(frsd_plan *pl, void *ws, const double *fields, int ne, size_t dense_off,
                             size_t pair_off, const int4 *otab, int nout, size_t sum_off, bool t220,
                             hipStream_t s) {
  const Layout &L = pl->L;
  XArgs a{};
  a.ncell = (long long)pl->M * pl->M * pl->M;
  a.nb = pl->p.bk_nbins;
  a.n_ell = ne;
  a.ncol = ne * a.nb;
  a.nload = t220 ? 2 * a.nb : a.ncol;
  a.nu = t220 ? 2 * a.nb : a.nb;
  a.t220 = t220 ? 1 : 0;
  a.npair = a.nb * (a.nb + 1) / 2;
  XJobs jobs;
  std::vector<int16_t> tile_job;
  int njobs = 0;
  if (!make_jobs(pl, ne, &jobs, &tile_job, &njobs)) return fail(FRSD_EINVAL, "too many contraction tiles");
  a.njobs = njobs;
  const int nwg = pl->tune.tri_wg;
  long long per = (a.ncell + nwg - 1) / nwg;
  per = (per + kZKC - 1) / kZKC * kZKC;
  a.cells_per_wg = per;
  double *dense = ws_ptr<double>(ws, dense_off);
  const int16_t *tj = reinterpret_cast<const int16_t *>(dense + (size_t)kXWaves * kXMaxJobs * 256);
  auto kern = t220 ? k_triple_mfma64<kXMaxU> : k_triple_mfma64<kXMaxB + 1>;
  FRSD_TIMED(t220 ? "triple_220" : "triple", s,
             hipLaunchKernelGGL(kern, dim3(nwg), dim3(kXThreads), 0, s, fields, a, jobs,
                                ws_ptr<const int2>(ws, pair_off), ws_ptr<double>(ws, L.tri_part)));
  const int nvals = njobs * 256;
  FRSD_TIMED("tri_reduce", s,
             hipLaunchKernelGGL(k_triple_mfma_reduce<double>, dim3((nvals + 255) / 256), dim3(256), 0, s,
                                ws_ptr<const double>(ws, L.tri_part), nwg, nvals, dense));
  FRSD_TIMED("tri_gather", s,
             hipLaunchKernelGGL(k_triple_mfma_gather, dim3((nout + 255) / 256), dim3(256), 0, s, dense, otab, tj,
                                a.nb, ne, nout, ws_ptr<double>(ws, sum_off)));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

// FP64 plans: T_ell on the same job tiles as the FP32 path.
int triple_mfma64(frsd_plan *pl, void *ws, const double *fields, hipStream_t s) {
  return triple_mfma64_run(pl, ws, fields, pl->n_ell, pl->L.tri_dense, pl->L.pair_tab,
                           ws_ptr<const int4>(ws, pl->L.tri_tab), pl->n_out, pl->L.tri_sum, false, s);
}

// N^T indicator sums (plan init): one column group, the triangle list as outputs.
int triple_mfma64_nt(frsd_plan *pl, void *ws, const double *indicators, hipStream_t s) {
  return triple_mfma64_run(pl, ws, indicators, 1, pl->L.tri_dense_nt, pl->L.pair_tab_nt,
                           ws_ptr<const int4>(ws, pl->L.tri_tab) + pl->n_out, (int)pl->ntri, pl->L.tri_sum, false, s);
}

// T_220 of FP64 plans: the N^T job tiles (their dense region is free after
// plan init), pairs (F_2 b2, F_0 b3), one output per triangle.
int triple_mfma64_220(frsd_plan *pl, void *ws, const double *fields, hipStream_t s) {
  return triple_mfma64_run(pl, ws, fields, 1, pl->L.tri_dense_nt, pl->L.pair_tab_220,
                           ws_ptr<const int4>(ws, pl->L.tri_tab) + pl->n_out, (int)pl->ntri, pl->L.tri_sum220, true,
                           s);
}

// The (row tile, column tile) -> job table, the row of each pair and the
// pair (b2, b3) of each row for ne column groups, added to the plan's table
// image: those of T_ell (ne = n_ell) at tri_dense / pair_tab, those of the
// N^T indicator sums (for_nt, ne = 1) at tri_dense_nt / pair_tab_nt.
// Pairs (F_2 b2, F_0 b3) of the T_220 rows, in the row order of the N^T
// job tables (staged rows nb + b2 and b3).
void triple_mfma_tables_220(frsd_plan *pl) {
  const int nb = pl->p.bk_nbins;
  const std::vector<int> row = pair_rows(pl, 1);
  std::vector<int2> pairs(row.size());
  for (int b2 = 0; b2 < nb; ++b2)
    for (int b3 = 0; b3 <= b2; ++b3) pairs[row[b2 * (b2 + 1) / 2 + b3]] = make_int2(nb + b2, b3);
  tab_add(pl, pl->L.pair_tab_220, pairs.data(), pairs.size() * sizeof(int2));
}

int triple_mfma_tables(frsd_plan *pl, int ne, bool for_nt) {
  XJobs jobs;
  std::vector<int16_t> tile_job;
  int njobs = 0;
  if (!make_jobs(pl, ne, &jobs, &tile_job, &njobs)) return fail(FRSD_EINVAL, "too many contraction tiles");
  const size_t dense_off = for_nt ? pl->L.tri_dense_nt : pl->L.tri_dense;
  const size_t pair_off = for_nt ? pl->L.pair_tab_nt : pl->L.pair_tab;
  tab_add(pl, dense_off + sizeof(double) * (size_t)kXWaves * kXMaxJobs * 256, tile_job.data(),
          tile_job.size() * sizeof(int16_t));
  const int nb = pl->p.bk_nbins;
  const std::vector<int> row = pair_rows(pl, ne);
  std::vector<int2> pairs(row.size());
  for (int b2 = 0; b2 < nb; ++b2)
    for (int b3 = 0; b3 <= b2; ++b3) pairs[row[b2 * (b2 + 1) / 2 + b3]] = make_int2(b2, b3);
  tab_add(pl, pair_off, pairs.data(), pairs.size() * sizeof(int2));
  return FRSD_OK;
}

}  // namespace frsd
