// Steps a7-a9: bispectrum multipoles by the FFT triangle search
// (Sec. III.B eqs. Factorize, F_k, BispMono, BispQuad, SNbisp2thin).
//
// For every bispectrum bin b and multipole field F_ell (ell = 0, 2, 4) the
// shell field F_{ell,b}(x) = sum_{n in b} F_ell(n) exp(+2 pi i n.x / M) is
// built on an M^3 grid by a pruned 3D inverse FFT: the input is non-zero
// only on |n_d| <= n_c, so the z pass runs on the (2 n_c + 1)^2 columns of
// the low-k cube, the y pass on (2 n_c + 1) x M rows and only the x pass on
// all M^2 rows.  Two real shell fields are packed in one complex transform
// (their spectra are Hermitian, so the real and imaginary parts of the
// output separate them).
//
// The triangle sums T_ell(b1,b2,b3) = M^-3 sum_x F_{ell,b1} F_{0,b2} F_{0,b3}
// equal the sums over closed triangles when M > 3 n_c.  N^T is the same sum
// of indicator fields, done once per plan in FP64 and rounded.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.h"
#include "frsd_internal.h"

namespace frsd {

constexpr int kTriThreads = 256;
constexpr int kTriKO = 32;     // outputs per thread
constexpr int kTriChunk = 64;  // cells staged per step

struct ShellArgs {
  int M, D, nc, nb, nfield;
  int pair0, npair;
  int lut_len;
};

static StageList stage_list(const FftLen &f) {
  StageList s{};
  s.nstage = f.nstage;
  for (int i = 0; i < f.nstage; ++i) s.radix[i] = f.radix[i];
  return s;
}

// z pass: pencils (pair, ix, iy) of the low-k cube, output buf1[pair][ix][iy][z]
template <typename T, bool IND>
__global__ __launch_bounds__(FftTune<T>::threads) void k_shell_z(const cplx_t<T> *__restrict__ lowk,
                                                        const int16_t *__restrict__ lut, ShellArgs a, int P,
                                                        StageList st, const cplx_t<T> *tw_g, cplx_t<T> *buf1) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + a.M;
  const int M = a.M, ld = M + 1, D = a.D, nc = a.nc;
  for (int i = threadIdx.x; i < M; i += FftTune<T>::threads) tw[i] = tw_g[i];
  const long long DD = (long long)D * D;
  const long long npen_all = (long long)a.npair * DD;
  const long long q0 = (long long)blockIdx.x * P;
  const int npen = (int)((q0 + P <= npen_all) ? P : (npen_all - q0));
  for (int i = threadIdx.x; i < npen * ld; i += FftTune<T>::threads) lds[i] = cmake<C>(T(0), T(0));
  __syncthreads();
  const long long DDD = DD * D;
  for (int f = threadIdx.x; f < npen * D; f += FftTune<T>::threads) {
    const int p = f / D, kz = f - p * D;
    const long long q = q0 + p;
    const int pair = (int)(q / DD);
    const int col = (int)(q - (long long)pair * DD);
    const int ix = col / D, iy = col - ix * D;
    const int nx = ix - nc, ny = iy - nc, nz = kz - nc;
    const long long m2 = (long long)nx * nx + (long long)ny * ny + (long long)nz * nz;
    const int b = (m2 > 0 && m2 < a.lut_len) ? lut[m2] : -1;
    const int fa = 2 * (a.pair0 + pair), fb = fa + 1;
    T ar = 0, ai = 0, br = 0, bi = 0;
    if (b >= 0) {
      if (fa % a.nb == b) {
        if (IND) ar = T(1);
        else { const C v = lowk[(fa / a.nb) * DDD + ((long long)ix * D + iy) * D + kz]; ar = v.x; ai = v.y; }
      }
      if (fb < a.nfield && fb % a.nb == b) {
        if (IND) br = T(1);
        else { const C v = lowk[(fb / a.nb) * DDD + ((long long)ix * D + iy) * D + kz]; br = v.x; bi = v.y; }
      }
    }
    // Z = A + i B
    lds[p * ld + (nz + M) % M] = cmake<C>(ar - bi, ai + br);
  }
  __syncthreads();
  lds_fft<C, true, FftTune<T>::threads, FftTune<T>::pn>(lds, ld, M, npen, st, tw);
  C *dst = buf1 + q0 * M;
  for (int f = threadIdx.x; f < npen * M; f += FftTune<T>::threads) {
    const int p = f / M, e = f - p * M;
    dst[f] = lds[p * ld + e];
  }
}

// y pass: pencils (pair, ix, z); input buf1[pair][ix][iy][z], output buf2[pair][ix][y][z]
template <typename T>
__global__ __launch_bounds__(FftTune<T>::threads) void k_shell_y(const cplx_t<T> *__restrict__ buf1, ShellArgs a, int P,
                                                        StageList st, const cplx_t<T> *tw_g, cplx_t<T> *buf2) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + a.M;
  const int M = a.M, ld = M + 1, D = a.D, nc = a.nc;
  for (int i = threadIdx.x; i < M; i += FftTune<T>::threads) tw[i] = tw_g[i];
  const long long npen_all = (long long)a.npair * D * M;
  const long long q0 = (long long)blockIdx.x * P;
  const int npen = (int)((q0 + P <= npen_all) ? P : (npen_all - q0));
  for (int i = threadIdx.x; i < npen * ld; i += FftTune<T>::threads) lds[i] = cmake<C>(T(0), T(0));
  __syncthreads();
  for (int f = threadIdx.x; f < npen * D; f += FftTune<T>::threads) {
    const int iy = f / npen, p = f - iy * npen;
    const long long q = q0 + p;               // q = (pair * D + ix) * M + z
    const long long pix = q / M;
    const int z = (int)(q - pix * M);
    lds[p * ld + (iy - nc + M) % M] = buf1[(pix * D + iy) * M + z];
  }
  __syncthreads();
  lds_fft<C, true, FftTune<T>::threads, FftTune<T>::pn>(lds, ld, M, npen, st, tw);
  for (int f = threadIdx.x; f < npen * M; f += FftTune<T>::threads) {
    const int y = f / npen, p = f - y * npen;
    const long long q = q0 + p;
    const long long pix = q / M;
    const int z = (int)(q - pix * M);
    buf2[(pix * M + y) * M + z] = lds[p * ld + y];
  }
}

// x pass: pencils (pair, y, z); input buf2[pair][ix][y][z]; output the two
// real shell fields of the pair, shells[f][y][z][x] (the contraction only needs one cell order for all fields)
template <typename T, typename TO>
__global__ __launch_bounds__(FftTune<T>::threads) void k_shell_x(const cplx_t<T> *__restrict__ buf2, ShellArgs a, int P,
                                                        StageList st, const cplx_t<T> *tw_g, TO *shells) {
  using C = cplx_t<T>;
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + a.M;
  const int M = a.M, ld = M + 1, D = a.D, nc = a.nc;
  for (int i = threadIdx.x; i < M; i += FftTune<T>::threads) tw[i] = tw_g[i];
  const long long MM = (long long)M * M;
  const long long npen_all = (long long)a.npair * MM;
  const long long q0 = (long long)blockIdx.x * P;
  const int npen = (int)((q0 + P <= npen_all) ? P : (npen_all - q0));
  for (int i = threadIdx.x; i < npen * ld; i += FftTune<T>::threads) lds[i] = cmake<C>(T(0), T(0));
  __syncthreads();
  for (int f = threadIdx.x; f < npen * D; f += FftTune<T>::threads) {
    const int ix = f / npen, p = f - ix * npen;
    const long long q = q0 + p;               // q = pair * M^2 + (y * M + z)
    const long long pair = q / MM;
    const long long yz = q - pair * MM;
    lds[p * ld + (ix - nc + M) % M] = buf2[(pair * D + ix) * MM + yz];
  }
  __syncthreads();
  lds_fft<C, true, FftTune<T>::threads, FftTune<T>::pn>(lds, ld, M, npen, st, tw);
  const long long MMM = MM * M;
  for (int f = threadIdx.x; f < npen * M; f += FftTune<T>::threads) {
    const int x = f / npen, p = f - x * npen;
    const long long q = q0 + p;
    const long long pair = q / MM;
    const long long yz = q - pair * MM;
    const int fa = 2 * (a.pair0 + (int)pair), fb = fa + 1;
    const C v = lds[p * ld + x];
    shells[(long long)fa * MMM + yz * M + x] = (TO)v.x;
    if (fb < a.nfield) shells[(long long)fb * MMM + yz * M + x] = (TO)v.y;
  }
}

// Compiled-length shell passes on the register-resident core (fft_pencils);
// same pencils and buffers as the run-time kernels above.  A pencil element
// e holds frequency e (e <= nc) or e - M (e >= M - nc) and is zero between.
// Pencils per workgroup: the y and x passes of FP32 plans take 32 pencils
// (1024 threads) when their LDS fits, the z pass and FP64 plans 16 or 8.
template <typename T, int LEN, int PASS> struct ShellTune {
  static constexpr bool wide =
      sizeof(T) == 4 && PASS != 0 && fft_pencils_lds<cplx_t<T>, LEN, 32>() <= (size_t)112 * 1024;
  static constexpr int nt = wide ? 1024 : (sizeof(T) == 4 ? 512 : 256);
  static constexpr int p = wide ? 32 : fit_pencils<cplx_t<T>, LEN, (sizeof(T) == 4 ? 16 : 8)>();
};

__device__ __forceinline__ int band_index(int e, int M, int nc) {
  return e <= nc ? e + nc : (e >= M - nc ? e - M + nc : -1);
}

// Shell radius bound of pair `pair` of the batch: the largest |n|^2 in the
// bins of its two fields.  A column (n_x, n_y) with n_x^2 + n_y^2 above it
// is zero after the z pass, and a row n_x with n_x^2 above it is zero after
// the y pass; those are neither written nor read (each pass tests the same
// bound), so the passes skip them.
__device__ __forceinline__ int pair_m2max(const int2 *bin_m2, const ShellArgs &a, int pair) {
  int h = -1;
  for (int k = 0; k < 2; ++k) {
    const int f = 2 * (a.pair0 + pair) + k;
    if (f < a.nfield) {
      const int2 r = bin_m2[f % a.nb];
      if (r.x <= r.y) h = max(h, r.y);
    }
  }
  return h;
}

// Per-pencil values of a compiled-length shell pass, set up once per
// workgroup in LDS so that no element recomputes them.
struct ShellPenZ {
  int m2xy;      // n_x^2 + n_y^2 of the pencil's column
  int col;       // offset of the column in a low-k multipole cube
  int off[2];    // multipole cube of field a / field b of the pair
  int lo[2], hi[2];  // |n|^2 range of the field's bin (empty: lo > hi)
  int live;      // column within the pair's shell radius
};

template <typename T, bool IND, int LEN>
__global__ __launch_bounds__((ShellTune<T, LEN, 0>::nt)) void k_shell_z_ct(const cplx_t<T> *__restrict__ lowk,
                                                                 const int2 *__restrict__ bin_m2, ShellArgs a,
                                                                 const cplx_t<T> *tw_g, cplx_t<T> *buf1) {
  using C = cplx_t<T>;
  constexpr int P = ShellTune<T, LEN, 0>::p, NT = ShellTune<T, LEN, 0>::nt;
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + LEN;
  __shared__ ShellPenZ pen[P];
  const int D = a.D, nc = a.nc;
  const int DD = D * D;
  const int DDD = DD * D;
  const long long npen_all = (long long)a.npair * DD;
  const long long q0 = (long long)blockIdx.x * P;
  const int npen = (int)((q0 + P <= npen_all) ? P : (npen_all - q0));
  int live = 0;
  if (threadIdx.x < P) {
    // pencil q = (pair * D + ix) * D + iy of the batch
    const int p = threadIdx.x;
    ShellPenZ v{};
    v.lo[0] = v.lo[1] = 1;
    v.hi[0] = v.hi[1] = 0;
    if (p < npen) {
      const long long q = q0 + p;
      const int pair = (int)(q / DD);
      const int colq = (int)(q - (long long)pair * DD);
      const int ix = colq / D, iy = colq - ix * D;
      v.m2xy = (ix - nc) * (ix - nc) + (iy - nc) * (iy - nc);
      v.col = colq * D;
      for (int h = 0; h < 2; ++h) {
        const int f = 2 * (a.pair0 + pair) + h;
        if (f < a.nfield) {
          const int2 r = bin_m2[f % a.nb];
          v.off[h] = (f / a.nb) * DDD;
          v.lo[h] = r.x;
          v.hi[h] = r.y;
        }
      }
      v.live = v.m2xy <= pair_m2max(bin_m2, a, pair) ? 1 : 0;
    }
    pen[p] = v;
    live = v.live;
  }
  if (!__syncthreads_or(live)) return;  // every column of the block lies outside its shells
  for (int i = threadIdx.x; i < LEN; i += NT) tw[i] = tw_g[i];
  __syncthreads();
  fft_pencils<C, LEN, P, NT, true, false>(
      lds, tw, npen,
      [&](int p, int e) {
        const int kz = band_index(e, LEN, nc);
        if (kz < 0) return cmake<C>(T(0), T(0));
        const ShellPenZ &v = pen[p];
        if (!v.live) return cmake<C>(T(0), T(0));
        const int m2 = v.m2xy + (kz - nc) * (kz - nc);
        T ar = 0, ai = 0, br = 0, bi = 0;
        if (m2 >= v.lo[0] && m2 <= v.hi[0]) {
          if (IND) ar = T(1);
          else { const C z = lowk[v.off[0] + v.col + kz]; ar = z.x; ai = z.y; }
        }
        if (m2 >= v.lo[1] && m2 <= v.hi[1]) {
          if (IND) br = T(1);
          else { const C z = lowk[v.off[1] + v.col + kz]; br = z.x; bi = z.y; }
        }
        return cmake<C>(ar - bi, ai + br);  // Z = A + i B
      },
      [&](int p, int e, C v) {
        if (pen[p].live) buf1[(q0 + p) * LEN + e] = v;
      });
}

template <typename T, int LEN>
__global__ __launch_bounds__((ShellTune<T, LEN, 1>::nt)) void k_shell_y_ct(const cplx_t<T> *__restrict__ buf1,
                                                                 const int2 *__restrict__ bin_m2, ShellArgs a,
                                                                 const cplx_t<T> *tw_g, cplx_t<T> *buf2) {
  using C = cplx_t<T>;
  constexpr int P = ShellTune<T, LEN, 1>::p, NT = ShellTune<T, LEN, 1>::nt;
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + LEN;
  // per pencil q = (pair * D + ix) * M + z: its first input element (buf1
  // row iy = 0), first output element (buf2 row y = 0), n_x^2 and the
  // pair's shell radius bound (rows with n_x^2 + n_y^2 above it are zero;
  // a pencil with n_x^2 above it is zero and not written)
  __shared__ long long src0[P], dst0[P];
  __shared__ int nx2[P], hmax[P];
  const int D = a.D, nc = a.nc;
  const long long npen_all = (long long)a.npair * D * LEN;
  const long long q0 = (long long)blockIdx.x * P;  // q = (pair * D + ix) * M + z
  const int npen = (int)((q0 + P <= npen_all) ? P : (npen_all - q0));
  int live = 0;
  if (threadIdx.x < P) {
    const int p = threadIdx.x;
    const long long q = q0 + p, pix = q / LEN, z = q - pix * LEN;
    const int pair = (int)(pix / D), ix = (int)(pix - (long long)pair * D);
    src0[p] = pix * D * LEN + z;
    dst0[p] = pix * LEN * LEN + z;
    nx2[p] = (ix - nc) * (ix - nc);
    hmax[p] = p < npen ? pair_m2max(bin_m2, a, pair) : -1;
    live = nx2[p] <= hmax[p];
  }
  if (!__syncthreads_or(live)) return;
  for (int i = threadIdx.x; i < LEN; i += NT) tw[i] = tw_g[i];
  __syncthreads();
  fft_pencils<C, LEN, P, NT, true, true>(
      lds, tw, npen,
      [&](int p, int e) {
        const int iy = band_index(e, LEN, nc);
        if (iy < 0 || nx2[p] + (iy - nc) * (iy - nc) > hmax[p]) return cmake<C>(T(0), T(0));
        return buf1[src0[p] + (long long)iy * LEN];
      },
      [&](int p, int e, C v) {
        if (nx2[p] <= hmax[p]) buf2[dst0[p] + (long long)e * LEN] = v;
      });
}

template <typename T, typename TO, int LEN>
__global__ __launch_bounds__((ShellTune<T, LEN, 2>::nt)) void k_shell_x_ct(const cplx_t<T> *__restrict__ buf2,
                                                                 const int2 *__restrict__ bin_m2, ShellArgs a,
                                                                 const cplx_t<T> *tw_g, TO *shells) {
  using C = cplx_t<T>;
  constexpr int P = ShellTune<T, LEN, 2>::p, NT = ShellTune<T, LEN, 2>::nt;
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + LEN;
  for (int i = threadIdx.x; i < LEN; i += NT) tw[i] = tw_g[i];
  __syncthreads();
  const int D = a.D, nc = a.nc;
  constexpr long long MM = (long long)LEN * LEN, MMM = MM * LEN;
  const long long npen_all = (long long)a.npair * MM;
  const long long q0 = (long long)blockIdx.x * P;  // q = pair * M^2 + (y * M + z)
  const int npen = (int)((q0 + P <= npen_all) ? P : (npen_all - q0));
  // rows n_x beyond the pair's shell radius were not written by the y pass.
  // The P pencils span at most two pairs (P < M^2): their bounds are kept
  // in registers, h0 below pencil index qb and h1 from it on.
  const int pair0 = (int)(q0 / MM);
  const long long qb = (long long)(pair0 + 1) * MM;
  const int h0 = pair_m2max(bin_m2, a, pair0);
  const int h1 = pair0 + 1 < a.npair ? pair_m2max(bin_m2, a, pair0 + 1) : -1;
  // output cell order [y][z][x] (x fastest): contiguous rows of M values
  // (divisions by the compiled M^2 are multiplications)
  fft_pencils<C, LEN, P, NT, true, true, false>(
      lds, tw, npen,
      [&](int p, int e) {
        const int ix = band_index(e, LEN, nc);
        const long long q = q0 + p;
        const int hm = q < qb ? h0 : h1;
        if (ix < 0 || (ix - nc) * (ix - nc) > hm) return cmake<C>(T(0), T(0));
        const long long pair = q / MM;
        return buf2[(pair * D + ix) * MM + (q - pair * MM)];
      },
      [&](int p, int e, C v) {
        const long long q = q0 + p, pair = q / MM, yz = q - pair * MM;
        const int fa = 2 * (a.pair0 + (int)pair), fb = fa + 1;
        shells[(long long)fa * MMM + yz * LEN + e] = (TO)v.x;
        if (fb < a.nfield) shells[(long long)fb * MMM + yz * LEN + e] = (TO)v.y;
      });
}

template <typename T, typename TO, bool IND, int LEN>
static int shell_pipeline_ct(frsd_plan *pl, void *ws, int nfield, const void *tw, TO *shells, hipStream_t s) {
  using C = cplx_t<T>;
  const Layout &L = pl->L;
  ShellArgs a{};
  a.M = LEN; a.D = pl->D; a.nc = pl->nc_b; a.nb = pl->p.bk_nbins; a.nfield = nfield;
  a.lut_len = pl->bk_lut_len;
  const int D = a.D;
  constexpr int PZ = ShellTune<T, LEN, 0>::p, NTZ = ShellTune<T, LEN, 0>::nt;
  constexpr int PY = ShellTune<T, LEN, 1>::p, NTY = ShellTune<T, LEN, 1>::nt;
  constexpr int PX = ShellTune<T, LEN, 2>::p, NTX = ShellTune<T, LEN, 2>::nt;
  constexpr size_t shz = fft_pencils_lds<C, LEN, PZ>(), shy = fft_pencils_lds<C, LEN, PY>(),
                   shx = fft_pencils_lds<C, LEN, PX>();
  FRSD_HIP(hipFuncSetAttribute((const void *)k_shell_z_ct<T, IND, LEN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shz));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_shell_y_ct<T, LEN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shy));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_shell_x_ct<T, TO, LEN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shx));
  const int npairs = (nfield + 1) / 2;
  const int pb = pl->tune.pair_batch;
  for (int p0 = 0; p0 < npairs; p0 += pb) {
    a.pair0 = p0;
    a.npair = std::min(pb, npairs - p0);
    const long long nz = (long long)a.npair * D * D, ny = (long long)a.npair * D * LEN,
                    nx = (long long)a.npair * LEN * LEN;
    FRSD_TIMED("shell_z", s, hipLaunchKernelGGL((k_shell_z_ct<T, IND, LEN>), dim3((unsigned)((nz + PZ - 1) / PZ)), dim3(NTZ), shz, s,
                       ws_ptr<const C>(ws, L.lowk), ws_ptr<const int2>(ws, L.bk_m2), a, (const C *)tw,
                       ws_ptr<C>(ws, L.buf1)));
    FRSD_TIMED("shell_y", s, hipLaunchKernelGGL((k_shell_y_ct<T, LEN>), dim3((unsigned)((ny + PY - 1) / PY)), dim3(NTY), shy, s,
                       ws_ptr<const C>(ws, L.buf1), ws_ptr<const int2>(ws, L.bk_m2), a, (const C *)tw,
                       ws_ptr<C>(ws, L.buf2)));
    FRSD_TIMED("shell_x", s, hipLaunchKernelGGL((k_shell_x_ct<T, TO, LEN>), dim3((unsigned)((nx + PX - 1) / PX)), dim3(NTX), shx, s,
                       ws_ptr<const C>(ws, L.buf2), ws_ptr<const int2>(ws, L.bk_m2), a, (const C *)tw, shells));
    FRSD_LAUNCH_CHECK();
  }
  return FRSD_OK;
}

template <typename T, typename TO, bool IND>
static int shell_pipeline_rt(frsd_plan *pl, void *ws, int nfield, const void *tw, TO *shells, hipStream_t s) {
  using C = cplx_t<T>;
  const Layout &L = pl->L;
  ShellArgs a{};
  a.M = pl->M; a.D = pl->D; a.nc = pl->nc_b; a.nb = pl->p.bk_nbins; a.nfield = nfield;
  a.lut_len = pl->bk_lut_len;
  const int M = a.M, D = a.D;
  const int P = FftTune<T>::pn / M;
  const StageList st = stage_list(pl->fft_m);
  const size_t shmem = sizeof(C) * ((size_t)M + (size_t)P * (M + 1));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_shell_z<T, IND>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_shell_y<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_shell_x<T, TO>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const int npairs = (nfield + 1) / 2;
  const int pb = pl->tune.pair_batch;
  for (int p0 = 0; p0 < npairs; p0 += pb) {
    a.pair0 = p0;
    a.npair = std::min(pb, npairs - p0);
    const long long nz = (long long)a.npair * D * D, ny = (long long)a.npair * D * M,
                    nx = (long long)a.npair * M * M;
    FRSD_TIMED("shell_z", s, hipLaunchKernelGGL((k_shell_z<T, IND>), dim3((unsigned)((nz + P - 1) / P)), dim3(FftTune<T>::threads), shmem, s,
                       ws_ptr<const C>(ws, L.lowk), ws_ptr<const int16_t>(ws, L.bk_lut), a, P, st, (const C *)tw,
                       ws_ptr<C>(ws, L.buf1)));
    FRSD_TIMED("shell_y", s, hipLaunchKernelGGL((k_shell_y<T>), dim3((unsigned)((ny + P - 1) / P)), dim3(FftTune<T>::threads), shmem, s,
                       ws_ptr<const C>(ws, L.buf1), a, P, st, (const C *)tw, ws_ptr<C>(ws, L.buf2)));
    FRSD_TIMED("shell_x", s, hipLaunchKernelGGL((k_shell_x<T, TO>), dim3((unsigned)((nx + P - 1) / P)), dim3(FftTune<T>::threads), shmem, s,
                       ws_ptr<const C>(ws, L.buf2), a, P, st, (const C *)tw, shells));
    FRSD_LAUNCH_CHECK();
  }
  return FRSD_OK;
}

template <typename T, typename TO, bool IND>
static int shell_pipeline(frsd_plan *pl, void *ws, int nfield, const void *tw, TO *shells, hipStream_t s) {
  switch (pl->M) {
#define FRSD_CASE(L) \
  case L: return shell_pipeline_ct<T, TO, IND, L>(pl, ws, nfield, tw, shells, s);
    FRSD_SHELL_LENGTHS(FRSD_CASE)
#undef FRSD_CASE
    default: return shell_pipeline_rt<T, TO, IND>(pl, ws, nfield, tw, shells, s);
  }
}

// ---------------------------------------------------------------------------
// Triple-product contraction (vector FMA version): out[o] = sum_x
// F[ta](x) F[tb](x) F[tc](x) for every output o = (ta, tb, tc), as per-block
// FP64 partials over grid-strided chunks of cells.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kTriThreads) void k_triple(const T *__restrict__ f, long long ncell, int nfield,
                                                        const int4 *__restrict__ otab, int nout, double *part) {
  extern __shared__ unsigned char smem_raw[];
  T *st = reinterpret_cast<T *>(smem_raw);  // [nfield][kTriChunk]
  int ta[kTriKO], tb[kTriKO], tc[kTriKO];
  double acc[kTriKO];
  const int obase = blockIdx.y * (kTriThreads * kTriKO);
#pragma unroll
  for (int j = 0; j < kTriKO; ++j) {
    const int o = obase + threadIdx.x + j * kTriThreads;
    acc[j] = 0.0;
    if (o < nout) { const int4 e = otab[o]; ta[j] = e.x; tb[j] = e.y; tc[j] = e.z; }
    else { ta[j] = 0; tb[j] = 0; tc[j] = 0; }
  }
  for (long long c0 = (long long)blockIdx.x * kTriChunk; c0 < ncell; c0 += (long long)gridDim.x * kTriChunk) {
    const int len = (int)((c0 + kTriChunk <= ncell) ? kTriChunk : (ncell - c0));
    __syncthreads();
    for (int i = threadIdx.x; i < nfield * kTriChunk; i += kTriThreads) {
      const int fl = i / kTriChunk, c = i - fl * kTriChunk;
      st[i] = (c < len) ? f[(long long)fl * ncell + c0 + c] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kTriKO; ++j) {
      if (obase + threadIdx.x + j * kTriThreads < nout) {
        const T *pa = st + ta[j] * kTriChunk, *pb = st + tb[j] * kTriChunk, *pc = st + tc[j] * kTriChunk;
        T sacc = T(0);
        for (int c = 0; c < kTriChunk; ++c) sacc += pa[c] * pb[c] * pc[c];
        acc[j] += (double)sacc;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kTriKO; ++j) {
    const int o = obase + threadIdx.x + j * kTriThreads;
    if (o < nout) part[(long long)o * gridDim.x + blockIdx.x] = acc[j];
  }
}

__global__ void k_sum_part(const double *part, int nblk, int nvals, double *sum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvals) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += part[(long long)i * nblk + b];
  sum[i] = s;
}

__global__ void k_nt_final(const double *sum, int ntri, double inv_m3, double *nt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntri) nt[t] = rint(sum[t] * inv_m3);
}

struct BkFinalArgs {
  int ntri, n_ell, pk_nb;
  int full_sn;   // complete l > 0 shot noise (Q_lw sums present)
  double inv_m3;
};

__device__ __forceinline__ double legendre_even(int ell, double mu) {
  const double m2 = mu * mu;
  return ell == 2 ? 1.5 * m2 - 0.5 : (35.0 * m2 * m2 - 30.0 * m2 + 3.0) * 0.125;
}

// B_ell^raw = (2 ell + 1) T_ell / (N^T I33) (eqs. BispMono, BispQuad), the
// thin-shell shot noise of eq. SNbisp2thin and, with t220, the zero-area
// hexadecapole of eq. Bhexa2.  Shot noise for l > 0: the q1 term
// (2l+1) S_lw(b1) / (N_b1 I33) and, with full_sn, the q2 and q3 terms
// (2l+1) L_l(qhat1 . qhat_i) Q_lw(b_i) / (N_bi I33), the cosines from the
// law of cosines at the bin centres ctr (k_f units), clamped to [-1, 1].
__global__ void k_bk_final(const int *tri, const double *tsum, const double *nt, const double *bin_sum,
                           const double *scal, const double *ctr, const double *t220, BkFinalArgs a,
                           frsd_bk_out out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.ntri) return;
  const double I33 = scal[2], W3 = scal[3];
  const double NT = nt[t];
  const int b[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
  const double nan = __builtin_nan("");
  double *tp[3] = {out.t0, out.t2, out.t4};
  double *bp[3] = {out.b0, out.b2, out.b4};
  double *sp[3] = {out.sn0, out.sn2, out.sn4};
  double Tl[3] = {nan, nan, nan};
  out.nt[t] = NT;
  for (int li = 0; li < 3; ++li) {
    const double ell = 2.0 * li;
    if (li < a.n_ell) {
      const double T = tsum[t * a.n_ell + li] * a.inv_m3;
      Tl[li] = T;
      tp[li][t] = T;
      bp[li][t] = NT > 0 ? (2 * ell + 1) * T / (NT * I33) : nan;
    } else {
      tp[li][t] = nan; bp[li][t] = nan;
    }
  }
  // bin sums of the bispectrum bins: [count, sum|k|, Q2w, Q4w, -, S0w, S2w, S4w]
  auto bs = [&](int bin, int q) { return bin_sum[(a.pk_nb + bin) * kBinSums + q]; };
  double sn0 = 0;
  for (int i = 0; i < 3; ++i) sn0 += bs(b[i], 5) / bs(b[i], 0);
  sp[0][t] = sn0 / I33 - 2.0 * W3 / I33;
  const double k1 = ctr[b[0]], k2 = ctr[b[1]], k3 = ctr[b[2]];
  const double c12 = fmin(1.0, fmax(-1.0, (k3 * k3 - k1 * k1 - k2 * k2) / (2.0 * k1 * k2)));
  const double c13 = fmin(1.0, fmax(-1.0, (k2 * k2 - k1 * k1 - k3 * k3) / (2.0 * k1 * k3)));
  for (int li = 1; li < 3; ++li) {
    const int ell = 2 * li;
    if (li >= a.n_ell) { sp[li][t] = nan; continue; }
    double v = bs(b[0], 5 + li) / bs(b[0], 0);
    if (a.full_sn)
      v += legendre_even(ell, c12) * bs(b[1], 1 + li) / bs(b[1], 0) +
           legendre_even(ell, c13) * bs(b[2], 1 + li) / bs(b[2], 0);
    sp[li][t] = (2 * ell + 1) * v / I33;
  }
  if (t220) {
    const double T = t220[t] * a.inv_m3;
    if (out.t220) out.t220[t] = T;
    if (out.b4za) out.b4za[t] = NT > 0 ? (17.5 * T - 5.0 * Tl[1] - 3.5 * Tl[0]) / (NT * I33) : nan;
  }
}

template <typename T>
static int contract(frsd_plan *pl, void *ws, const T *fields, int nfield, const int4 *otab, int nout,
                    hipStream_t s, size_t sum_off = (size_t)-1) {
  const Layout &L = pl->L;
  const long long M3 = (long long)pl->M * pl->M * pl->M;
  const size_t shmem = sizeof(T) * (size_t)nfield * kTriChunk;
  FRSD_HIP(hipFuncSetAttribute((const void *)k_triple<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const unsigned ny = (unsigned)((nout + kTriThreads * kTriKO - 1) / (kTriThreads * kTriKO));
  FRSD_TIMED("triple", s, hipLaunchKernelGGL(k_triple<T>, dim3(kTriBlocks, ny), dim3(kTriThreads), shmem, s, fields, M3, nfield, otab, nout,
                     ws_ptr<double>(ws, L.tri_part)));
  FRSD_TIMED("tri_reduce", s, hipLaunchKernelGGL(k_sum_part, dim3((nout + 255) / 256), dim3(256), 0, s, ws_ptr<const double>(ws, L.tri_part),
                     kTriBlocks, nout, ws_ptr<double>(ws, sum_off == (size_t)-1 ? L.tri_sum : sum_off)));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

// N^T of every listed triangle from FP64 indicator fields.
int run_nt(frsd_plan *pl, void *ws, hipStream_t s) {
  const Layout &L = pl->L;
  double *shells = ws_ptr<double>(ws, L.shells);
  int rc = shell_pipeline<double, double, true>(pl, ws, pl->p.bk_nbins, ws_ptr<void>(ws, L.tw_inv64), shells, s);
  if (rc) return rc;
  const int4 *otab = ws_ptr<const int4>(ws, L.tri_tab) + pl->n_out;
  if (triple_mfma_supported(pl, 1)) rc = triple_mfma64_nt(pl, ws, shells, s);
  else rc = contract<double>(pl, ws, shells, pl->p.bk_nbins, otab, (int)pl->ntri, s);
  if (rc) return rc;
  const double inv_m3 = 1.0 / ((double)pl->M * pl->M * pl->M);
  FRSD_TIMED("nt_final", s, hipLaunchKernelGGL(k_nt_final, dim3((unsigned)((pl->ntri + 255) / 256)), dim3(256), 0, s,
                     ws_ptr<const double>(ws, L.tri_sum), (int)pl->ntri, inv_m3, ws_ptr<double>(ws, L.nt)));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template <typename T>
int run_bk(frsd_plan *pl, void *ws, const frsd_bk_out *out, hipStream_t s) {
  const Layout &L = pl->L;
  const int nfield = pl->n_ell * pl->p.bk_nbins;
  int rc;
  // complete l > 0 shot noise: the w^2-weighted moments and their Q_lw sums
  // (they use the planar and mesh regions before the shell fields take them)
  if (pl->n_wmom > 0) {
    if ((rc = run_w_moments<T>(pl, ws, s))) return rc;
    if ((rc = run_bin_w<T>(pl, ws, s))) return rc;
  }
  T *shells = ws_ptr<T>(ws, L.shells);
  rc = shell_pipeline<T, T, false>(pl, ws, nfield, ws_ptr<void>(ws, L.tw_inv), shells, s);
  if (rc) return rc;
  const bool z220 = pl->p.bk_zero_area != 0;
  const int4 *otab220 = ws_ptr<const int4>(ws, L.tri_tab220);
  if constexpr (sizeof(T) == 4) {
    if (triple_mfma_supported(pl)) rc = triple_mfma(pl, ws, reinterpret_cast<const float *>(shells), s);
    else rc = contract<T>(pl, ws, shells, nfield, ws_ptr<const int4>(ws, L.tri_tab), pl->n_out, s);
    if (!rc && z220) {
      if (triple_mfma_supported(pl, 1)) rc = triple_mfma_220(pl, ws, reinterpret_cast<const float *>(shells), s);
      else rc = contract<T>(pl, ws, shells, nfield, otab220, (int)pl->ntri, s, L.tri_sum220);
    }
  } else {
    if (triple_mfma_supported(pl)) rc = triple_mfma64(pl, ws, reinterpret_cast<const double *>(shells), s);
    else rc = contract<T>(pl, ws, shells, nfield, ws_ptr<const int4>(ws, L.tri_tab), pl->n_out, s);
    if (!rc && z220) {
      if (triple_mfma_supported(pl, 1)) rc = triple_mfma64_220(pl, ws, reinterpret_cast<const double *>(shells), s);
      else rc = contract<T>(pl, ws, shells, nfield, otab220, (int)pl->ntri, s, L.tri_sum220);
    }
  }
  if (rc) return rc;
  BkFinalArgs a{};
  a.ntri = (int)pl->ntri; a.n_ell = pl->n_ell; a.pk_nb = pl->p.pk_nbins;
  a.full_sn = pl->n_wmom > 0 ? 1 : 0;
  a.inv_m3 = 1.0 / ((double)pl->M * pl->M * pl->M);
  // the triangle list is kept in the tail of the table region as int32 triples
  const int *tri = reinterpret_cast<const int *>(ws_ptr<const int4>(ws, L.tri_tab) + pl->n_out + pl->ntri);
  FRSD_TIMED("bk_final", s, hipLaunchKernelGGL(k_bk_final, dim3((unsigned)((pl->ntri + 255) / 256)), dim3(256), 0, s, tri,
                     ws_ptr<const double>(ws, L.tri_sum), ws_ptr<const double>(ws, L.nt),
                     ws_ptr<const double>(ws, L.bin_sum), ws_ptr<const double>(ws, L.scal),
                     ws_ptr<const double>(ws, L.bk_ctr), z220 ? ws_ptr<const double>(ws, L.tri_sum220) : nullptr,
                     a, *out));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template int run_bk<float>(frsd_plan *, void *, const frsd_bk_out *, hipStream_t);
template int run_bk<double>(frsd_plan *, void *, const frsd_bk_out *, hipStream_t);

// ---------------------------------------------------------------------------
// Tables uploaded by frsd_plan_init.
// ---------------------------------------------------------------------------
// Stage twiddle table of a length-n transform (radix schedule of
// make_fft_len): for every stage s > 0 with Ns = product of the earlier
// radices, W_{Ns R}^{r k} = exp(-2 pi i r k / (Ns R)) at (Ns - 1) + k (R - 1)
// + (r - 1), k < Ns, 1 <= r < R; the entries fill [R_0 - 1, n - 1).
template <typename T>
static std::vector<T> twiddles(int n) {
  std::vector<T> t(2 * (size_t)n, T(0));
  FftLen f;
  if (!make_fft_len(n, &f)) return t;
  const long double two_pi = 6.283185307179586476925286766559005768L;
  int ns = 1;
  for (int s = 0; s < f.nstage; ++s) {
    const int R = f.radix[s];
    if (s > 0) {
      for (int k = 0; k < ns; ++k)
        for (int r = 1; r < R; ++r) {
          const size_t idx = (size_t)(ns - 1) + (size_t)k * (R - 1) + (r - 1);
          const long double a = two_pi * (long double)(r * k) / (long double)(ns * R);
          t[2 * idx] = (T)cosl(a);
          t[2 * idx + 1] = (T)(-sinl(a));
        }
    }
    ns *= R;
  }
  return t;
}

static std::vector<int16_t> bin_lut(const std::vector<double> &e2, int len) {
  std::vector<int16_t> lut(len, -1);
  const int nb = (int)e2.size() - 1;
  for (int m = 1; m < len; ++m) {
    for (int b = 0; b < nb; ++b)
      if ((double)m >= e2[b] && (double)m < e2[b + 1]) { lut[m] = (int16_t)b; break; }
  }
  return lut;
}

void tab_add(frsd_plan *pl, size_t ws_off, const void *src, size_t bytes) {
  const size_t off = (pl->tab_host.size() + 255) & ~(size_t)255;
  pl->tab_host.resize(off + bytes);
  std::memcpy(pl->tab_host.data() + off, src, bytes);
  pl->tab_seg.push_back(TabSeg{off, ws_off, bytes});
}

// Every constant table of the plan, in one host image: stage twiddles of
// the forward and inverse transforms, the |n|^2 -> bin lookups, the |n|^2
// range of each bispectrum bin, the contraction output tables and triangle
// list, and the matrix-core job tables of the T_ell and N^T contractions
// (each only when that contraction runs on the matrix cores: run_bk and
// run_nt take the same predicates).
int build_tables(frsd_plan *pl) {
  if (pl->tab_built) return FRSD_OK;
  pl->tab_host.clear();
  pl->tab_seg.clear();
  const Layout &L = pl->L;
  const bool f64 = pl->p.precision == FRSD_F64;
  if (f64) {
    auto t = twiddles<double>(pl->N);
    tab_add(pl, L.tw_fwd, t.data(), t.size() * sizeof(double));
  } else {
    auto t = twiddles<float>(pl->N);
    tab_add(pl, L.tw_fwd, t.data(), t.size() * sizeof(float));
  }
  auto lp = bin_lut(pl->pk_e2, pl->pk_lut_len);
  tab_add(pl, L.pk_lut, lp.data(), lp.size() * sizeof(int16_t));
  if (pl->p.bk_nbins > 0) {
    if (f64) {
      auto t = twiddles<double>(pl->M);
      tab_add(pl, L.tw_inv, t.data(), t.size() * sizeof(double));
    } else {
      auto t = twiddles<float>(pl->M);
      tab_add(pl, L.tw_inv, t.data(), t.size() * sizeof(float));
    }
    auto t64 = twiddles<double>(pl->M);
    tab_add(pl, L.tw_inv64, t64.data(), t64.size() * sizeof(double));
    auto lb = bin_lut(pl->bk_e2, pl->bk_lut_len);
    tab_add(pl, L.bk_lut, lb.data(), lb.size() * sizeof(int16_t));
    // |n|^2 range [lo, hi] of every bispectrum bin (bins hold consecutive
    // integers; an empty bin gets lo > hi)
    std::vector<int2> m2r(pl->p.bk_nbins, make_int2(1, 0));
    for (int m = 1; m < pl->bk_lut_len; ++m) {
      const int b = lb[m];
      if (b < 0) continue;
      if (m2r[b].x > m2r[b].y) m2r[b] = make_int2(m, m);
      else m2r[b].y = m;
    }
    for (int m = 1; m < pl->bk_lut_len; ++m)
      if (lb[m] >= 0 && (m < m2r[lb[m]].x || m > m2r[lb[m]].y)) return fail(FRSD_EINVAL, "bin lookup not monotone");
    tab_add(pl, L.bk_m2, m2r.data(), m2r.size() * sizeof(int2));
    // contraction tables: data outputs (field of b1 for each ell, b2, b3), then
    // indicator outputs (b1, b2, b3), then the raw int32 triangle list
    const int nb = pl->p.bk_nbins;
    std::vector<int4> tab((size_t)pl->n_out + (size_t)pl->ntri);
    for (int64_t t = 0; t < pl->ntri; ++t) {
      const int b1 = pl->tri[3 * t], b2 = pl->tri[3 * t + 1], b3 = pl->tri[3 * t + 2];
      for (int li = 0; li < pl->n_ell; ++li) tab[t * pl->n_ell + li] = make_int4(li * nb + b1, b2, b3, 0);
      tab[pl->n_out + t] = make_int4(b1, b2, b3, 0);
    }
    tab_add(pl, L.tri_tab, tab.data(), tab.size() * sizeof(int4));
    tab_add(pl, L.tri_tab + tab.size() * sizeof(int4), pl->tri.data(), pl->tri.size() * sizeof(int32_t));
    // bin centres in k_f units (the thin-shell cosines of the shot noise)
    std::vector<double> ctr(nb);
    for (int b = 0; b < nb; ++b) ctr[b] = 0.5 * (std::sqrt(pl->bk_e2[b]) + std::sqrt(pl->bk_e2[b + 1]));
    tab_add(pl, L.bk_ctr, ctr.data(), ctr.size() * sizeof(double));
    if (pl->p.bk_zero_area) {
      // vector-contraction outputs of T_220: (F_2 of b1, F_2 of b2, F_0 of b3)
      std::vector<int4> t220((size_t)pl->ntri);
      for (int64_t t = 0; t < pl->ntri; ++t)
        t220[t] = make_int4(nb + pl->tri[3 * t], nb + pl->tri[3 * t + 1], pl->tri[3 * t + 2], 0);
      tab_add(pl, L.tri_tab220, t220.data(), t220.size() * sizeof(int4));
      if (triple_mfma_supported(pl, 1)) triple_mfma_tables_220(pl);
    }
    if (triple_mfma_supported(pl)) {
      const int rc = triple_mfma_tables(pl, pl->n_ell, false);
      if (rc) return rc;
    }
    if (triple_mfma_supported(pl, 1)) {
      const int rc = triple_mfma_tables(pl, 1, true);
      if (rc) return rc;
    }
  }
  pl->tab_built = true;
  return FRSD_OK;
}

int upload_tables(frsd_plan *pl, void *ws, hipStream_t s, bool pageable) {
  int rc = build_tables(pl);
  if (rc) return rc;
  const unsigned char *src = pl->tab_host.data();
  if (!pageable) {
    if (!pl->tab_pinned) {
      FRSD_HIP(hipHostMalloc(&pl->tab_pinned, std::max<size_t>(pl->tab_host.size(), 1), hipHostMallocDefault));
      std::memcpy(pl->tab_pinned, pl->tab_host.data(), pl->tab_host.size());
      FRSD_HIP(hipEventCreateWithFlags(&pl->tab_done, hipEventDisableTiming));
    }
    src = static_cast<const unsigned char *>(pl->tab_pinned);
  }
  for (const TabSeg &g : pl->tab_seg)
    FRSD_HIP(hipMemcpyAsync(ws_ptr<void>(ws, g.ws_off), src + g.host_off, g.bytes, hipMemcpyHostToDevice, s));
  if (!pageable) FRSD_HIP(hipEventRecord(pl->tab_done, s));
  return FRSD_OK;
}

}  // namespace frsd
