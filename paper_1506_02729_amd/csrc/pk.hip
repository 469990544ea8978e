// Steps a5-a6: multipole combination and |k|-shell binning, fused
// (Sec. II.B eqs. delta2b, delta4b; Sec. III.A eqs. F2, P0_impl-P4_impl).
//
// One thread per wave-vector n of the half space (n and -n give complex-
// conjugate contributions, so each half-space mode is counted twice).  For
// every complex slot the thread reads Z(n) and Z(-n), and accumulates the
// real-coefficient combinations needed for F_0, F_2, F_4 and F_0^w:
//   R_2 = sum_ab khat_a khat_b Q_ab,  R_4 = sum_abcd khat_a khat_b khat_c khat_d Q_abcd
// over the kept moments (class_coeffs), F_2 = 3/2 R_2 - 1/2 F_0,
//   F_4 = 35/8 R_4 - 5/2 F_2 - 7/8 F_0.
// Because every step after the FFT is linear with real coefficients, the
// unpacking of the two real planes of a slot (X = [Z(n) + Z(-n)^*] / 2,
// Y = [Z(n) - Z(-n)^*] / 2i), the interlacing 1/2 [X + exp(-i pi sum n / N) Y]
// and the window compensation prod sinc(pi n_d / N)^p are applied once per
// multipole to the combined sums.  Shell sums are reduced per wavefront by
// bin key and accumulated in FP64: three data sums per bin, since the mode
// counts and sum |k| of every bin do not depend on the data and are summed
// once per plan by the same kernel in its geometry mode.
#include <cmath>
#include <utility>

#include "device.h"
#include "frsd_internal.h"

namespace frsd {

constexpr int kBinThreads = 256;
constexpr int kMaxBinsAll = 512;
constexpr int kBinTab = 513;  // |n| <= N/2 for N <= 1024

struct BinArgs {
  int N, nmax, order, interlace, compensate;
  int pk_nb, bk_nb, pk_lut_len, bk_lut_len;
  int nc_b, D;  // low-k cube
  int n_slot, n_ell, has_w;
  double kf;
  // random cache: slot s is Z_gal + cx[s] X_ran + i cy[s] Y_ran, with X_ran and
  // Y_ran the real-plane spectra of the cached slot (cx = cy: one factor);
  // the factor of a plane is 0 (empty), -alpha (kind 1: the moments of eqs.
  // F0, Qab) or +alpha^2 (kind 2: the w^2 weights of F_0^w), alpha[r] that
  // of request r of the batch
  int cached;
  int8_t kx[kMaxSlots], ky[kMaxSlots];
  double alpha[kMaxBatch];
};

__device__ __forceinline__ double cache_factor(int kind, double al) {
  return kind == 1 ? -al : (kind == 2 ? al * al : 0.0);
}

// Sum v[NV] over every run of equal keys among consecutive lanes (a
// segmented inclusive scan), and let the last lane of each run whose key is
// >= 0 add the run's sums to lds_bins[key * NV + *].  Lanes are assigned
// consecutive modes along n_z, so keys come in a few long runs; a key that
// forms several runs adds each run's sum separately.  Every lane of the
// wavefront takes part.
template <int NV>
__device__ __forceinline__ void wave_run_add(int key, double *v, double *lds_bins) {
  if (__ballot(key >= 0) == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  const int next = __shfl_down(key, 1, 64);
  int start = (lane == 0 || prev != key) ? lane : 0;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) start = max(start, __shfl_up(start, o, 64));
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const bool take = lane - o >= start;
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const double t = __shfl_up(v[s], o, 64);
      v[s] += take ? t : 0.0;
    }
  }
  if (key >= 0 && (lane == 63 || next != key)) {
#pragma unroll
    for (int s = 0; s < NV; ++s) atomicAdd(&lds_bins[key * NV + s], v[s]);
  }
}

// Per-mode sums reduced by the binning kernel: GEOM (once per plan) the
// mode count and sum |k| of every bin; otherwise the data sums, (S00, S20,
// S40, S22) for the P_ell bins and (S0w, S2w, S4w, unused) for the
// bispectrum bins.  S22 = sum |F_2|^2 feeds the split hexadecapole P_4b
// (Sec. II.B eq. P4fast).
template <bool GEOM> struct BinValues { static constexpr int n = GEOM ? 2 : 4; };

// Add the moment at position p of the moment list (moments 0..n_ell-1 in
// ID order, then the w^2 moment if has_w) with Fourier values z(n), z(-n)
// to the class sums r[cls][+-]: class 0 the monopole, 1 R_2, 2 R_4 (each
// kept moment with its class_coeffs coefficient), 3 the w^2 moment.
template <typename C, typename T, int p>
__device__ __forceinline__ void add_position(int n_ell, int has_w, const T *c2, const T *c4, C zp, C zm,
                                             C (&r)[4][2]) {
  if (p < n_ell) {
    if (p == 0) {
      r[0][0] = cadd(r[0][0], zp);
      r[0][1] = cadd(r[0][1], zm);
    }
    if (p < kMomRank2 && n_ell > 1) {
      const T c = c2[p < kMomRank2 ? p : 0];
      r[1][0] = cadd(r[1][0], cscale(zp, c));
      r[1][1] = cadd(r[1][1], cscale(zm, c));
    }
    if (n_ell > kMomRank2) {
      const T c = c4[p < kMomRank4 ? p : 0];
      r[2][0] = cadd(r[2][0], cscale(zp, c));
      r[2][1] = cadd(r[2][1], cscale(zm, c));
    }
  } else if (p == n_ell && has_w) {
    r[3][0] = cadd(r[3][0], zp);
    r[3][1] = cadd(r[3][1], zm);
  }
}

// All slots of one mode, unrolled so that every position is a constant.
template <typename C, typename T, bool IL, int... S>
__device__ __forceinline__ void add_slots(std::integer_sequence<int, S...>, int n_slot, int n_ell, int has_w,
                                          const T *c2, const T *c4, const C *zp, const C *zm, C (&rr)[4][2],
                                          C (&ri)[4][2]) {
  if constexpr (IL) {
    ((S < n_slot ? add_position<C, T, S>(n_ell, has_w, c2, c4, zp[S], zm[S], rr) : void()), ...);
  } else {
    ((S < n_slot ? add_position<C, T, 2 * S>(n_ell, has_w, c2, c4, zp[S], zm[S], rr) : void()), ...);
    ((S < n_slot ? add_position<C, T, 2 * S + 1>(n_ell, has_w, c2, c4, zp[S], zm[S], ri) : void()), ...);
  }
}

// IL: slot s holds moment position s on the main grid (real part) and on
// the twin grid (imaginary part); otherwise positions 2s and 2s+1.
// WP: the slots hold the w^2-weighted moments (a second assignment pass),
// whose combinations are F^w_0, F^w_2, F^w_4; only bispectrum bins are
// summed, Q_lw = sum Re[F_0 (F^w_l)^*] for l = 2, 4, with F_0 read from the
// low-k cube written by the first pass.
// Grid (blocks, request): mesh, lowk, part and rcache are request 0's and
// move by the request's workspace distance.
template <typename T, bool GEOM, bool IL, bool WP = false>
__global__ __launch_bounds__(kBinThreads) void k_bin(const cplx_t<T> *__restrict__ mesh, long long slot_stride,
                                                      BinArgs a, const int16_t *__restrict__ pk_lut,
                                                      const int16_t *__restrict__ bk_lut, cplx_t<T> *lowk,
                                                      double *part, const cplx_t<T> *__restrict__ rcache, Batch bt) {
  using C = cplx_t<T>;
  constexpr int NV = BinValues<GEOM>::n;
  const long long dr = bt.delta[blockIdx.y];
  mesh = shifted(mesh, dr);
  lowk = shifted(lowk, dr);
  part = shifted(part, dr);
  rcache = shifted(rcache, dr);
  const double al = a.alpha[blockIdx.y];
  __shared__ double bins[kMaxBinsAll * NV];
  // per-axis factors for |n| <= nmax: interlacing phase exp(-i pi n / N)
  // (cos, sin) and the inverse window 1 / sinc(pi n / N)^p
  __shared__ double tcos[kBinTab], tsin[kBinTab], tiw[kBinTab];
  const int nall = a.pk_nb + a.bk_nb;
  const int N = a.N, nm = a.nmax;
  for (int i = threadIdx.x; i < nall * NV; i += kBinThreads) bins[i] = 0.0;
  if (!GEOM) {
    for (int n = threadIdx.x; n <= nm; n += kBinThreads) {
      const double x = (double)n / N;
      double sn, cs;
      sincospi(x, &sn, &cs);
      tcos[n] = cs;
      tsin[n] = -sn;
      double iw = 1.0;
      if (a.compensate && n != 0) {
        const double sc = sn / (M_PI * x);
        double wp = sc;
        for (int q = 1; q < a.order; ++q) wp *= sc;
        iw = 1.0 / wp;
      }
      tiw[n] = iw;
    }
  }
  __syncthreads();

  const int side = 2 * nm + 1;
  const long long total = (long long)side * side * (nm + 1);
  const long long stride = (long long)gridDim.x * kBinThreads;
  // every lane runs the same number of iterations so the wavefront
  // reductions see all lanes
  const long long iters = (total + stride - 1) / stride;
  for (long long itn = 0; itn < iters; ++itn) {
    const long long t = blockIdx.x * (long long)kBinThreads + threadIdx.x + itn * stride;
    int kp = -1, kb = -1;
    double vp[NV], vb[NV];
#pragma unroll
    for (int s = 0; s < NV; ++s) { vp[s] = 0; vb[s] = 0; }
    int ix = 0, iy = 0, iz = 0;
    long long m2 = 0;
    if (t < total) {
      iz = (int)(t % (nm + 1));
      const long long r = t / (nm + 1);
      iy = (int)(r % side) - nm;
      ix = (int)(r / side) - nm;
      const bool half = (iz > 0) || (iy > 0) || (iy == 0 && ix > 0);
      m2 = (long long)ix * ix + (long long)iy * iy + (long long)iz * iz;
      if (half) {
        kp = (!WP && m2 < a.pk_lut_len) ? pk_lut[m2] : -1;
        kb = (a.bk_nb > 0 && m2 < a.bk_lut_len) ? bk_lut[m2] : -1;
      }
    }
    if (GEOM) {
      if (kp >= 0 || kb >= 0) {
        const double kmag = a.kf * sqrt((double)m2);
        vp[0] = 2.0; vp[1] = 2.0 * kmag;
        vb[0] = 2.0; vb[1] = 2.0 * kmag;
      }
    } else if (kp >= 0 || kb >= 0) {
      const long long gp = ((long long)((ix + N) % N) * N + (iy + N) % N) * N + iz;
      const long long gm = ((long long)((N - ix) % N) * N + (N - iy) % N) * N + (N - iz) % N;
      // every slot's Z(n) and Z(-n) are requested before any is used
      C zp[kMaxSlots], zm[kMaxSlots];
#pragma unroll
      for (int sl = 0; sl < kMaxSlots; ++sl) {
        if (sl < a.n_slot) {
          zp[sl] = mesh[sl * slot_stride + gp];
          zm[sl] = mesh[sl * slot_stride + gm];
        }
      }
      if (!GEOM && !WP && a.cached) {
        // F = F_gal + c F_ran per real plane: c X_ran(n) + i c' Y_ran(n) =
        // (c + c')/2 Z_ran(n) + (c - c')/2 Z_ran(-n)^*
#pragma unroll
        for (int sl = 0; sl < kMaxSlots; ++sl) {
          if (sl < a.n_slot) {
            const C rp = rcache[sl * slot_stride + gp], rm = rcache[sl * slot_stride + gm];
            const double fx = cache_factor(a.kx[sl], al), fy = cache_factor(a.ky[sl], al);
            const T ca = (T)(0.5 * (fx + fy)), cb = (T)(0.5 * (fx - fy));
            zp[sl] = cadd(zp[sl], cadd(cscale(rp, ca), cscale(cmake<C>(rm.x, -rm.y), cb)));
            zm[sl] = cadd(zm[sl], cadd(cscale(rm, ca), cscale(cmake<C>(rp.x, -rp.y), cb)));
          }
        }
      }
      const T ik = (T)(1.0 / sqrt((double)m2));
      T c2[kMomRank2], c4[kMomRank4];
      class_coeffs<T>((T)ix * ik, (T)iy * ik, (T)iz * ik, c2, c4);
      // class sums [class][n / -n] of the real-part and imaginary-part planes
      C rr[4][2], ri[4][2];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int q = 0; q < 2; ++q) { rr[c][q] = cmake<C>(T(0), T(0)); ri[c][q] = cmake<C>(T(0), T(0)); }
      add_slots<C, T, IL>(std::make_integer_sequence<int, kMaxSlots>{}, a.n_slot, a.n_ell, a.has_w, c2, c4, zp, zm,
                          rr, ri);
      // multipole combinations (Sec. II.B): F_0 = R0, F_2 = 3/2 R2 - 1/2 R0,
      // F_4 = 35/8 R4 - 15/4 R2 + 3/8 R0, and F_0^w
      auto multipoles = [&](C (&r)[4][2], C (&z)[4][2]) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          z[0][q] = r[0][q];
          z[1][q] = cadd(cscale(r[1][q], T(1.5)), cscale(r[0][q], T(-0.5)));
          z[2][q] = cadd(cadd(cscale(r[2][q], T(4.375)), cscale(r[1][q], T(-3.75))), cscale(r[0][q], T(0.375)));
          z[3][q] = r[3][q];
        }
      };
      C zr[4][2], zi[4][2];
      multipoles(rr, zr);
      if constexpr (IL) {
#pragma unroll
        for (int l = 0; l < 4; ++l) { zi[l][0] = zr[l][0]; zi[l][1] = zr[l][1]; }
      } else {
        multipoles(ri, zi);
      }
      // unpack, interlace, compensate
      const int ax = ix < 0 ? -ix : ix, ay = iy < 0 ? -iy : iy;
      double ph_re = 1.0, ph_im = 0.0, s = 1.0;
      if (a.interlace) {
        // exp(-i pi (n_x + n_y + n_z) / N) as a product of per-axis factors
        const double cx = tcos[ax], sx = ix < 0 ? -tsin[ax] : tsin[ax];
        const double cy = tcos[ay], sy = iy < 0 ? -tsin[ay] : tsin[ay];
        const double cz = tcos[iz], sz = tsin[iz];
        const double cxy = cx * cy - sx * sy, sxy = cx * sy + sx * cy;
        ph_re = cxy * cz - sxy * sz;
        ph_im = cxy * sz + sxy * cz;
        s = 0.5;
      }
      const double scale = s * (tiw[ax] * tiw[ay] * tiw[iz]);
      double A[4][2];
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        // X = (zr(n) + conj zr(-n)) / 2 ;  Y = (zi(n) - conj zi(-n)) / 2i
        const double xr = 0.5 * ((double)zr[l][0].x + (double)zr[l][1].x);
        const double xi = 0.5 * ((double)zr[l][0].y - (double)zr[l][1].y);
        const double yr = 0.5 * ((double)zi[l][0].y + (double)zi[l][1].y);
        const double yi = -0.5 * ((double)zi[l][0].x - (double)zi[l][1].x);
        const double pr = ph_re * yr - ph_im * yi, pi = ph_re * yi + ph_im * yr;
        A[l][0] = scale * (xr + pr);
        A[l][1] = scale * (xi + pi);
      }
      const double S00 = A[0][0] * A[0][0] + A[0][1] * A[0][1];
      const double S20 = A[1][0] * A[0][0] + A[1][1] * A[0][1];
      const double S40 = A[2][0] * A[0][0] + A[2][1] * A[0][1];
      const double S0w = A[0][0] * A[3][0] + A[0][1] * A[3][1];
      const double S2w = A[1][0] * A[3][0] + A[1][1] * A[3][1];
      const double S4w = A[2][0] * A[3][0] + A[2][1] * A[3][1];
      const double S22 = A[1][0] * A[1][0] + A[1][1] * A[1][1];
      // each half-space mode stands for n and -n
      if constexpr (WP) {
        if (kb >= 0) {
          const int D = a.D, nc = a.nc_b;
          const C f0 = lowk[((long long)(ix + nc) * D + (iy + nc)) * D + (iz + nc)];
          vb[0] = 2.0 * ((double)f0.x * A[1][0] + (double)f0.y * A[1][1]);
          vb[1] = 2.0 * ((double)f0.x * A[2][0] + (double)f0.y * A[2][1]);
        }
      } else if constexpr (NV == 4) {
        vp[0] = 2.0 * S00; vp[1] = 2.0 * S20; vp[2] = 2.0 * S40; vp[3] = 2.0 * S22;
        vb[0] = 2.0 * S0w; vb[1] = 2.0 * S2w; vb[2] = 2.0 * S4w; vb[3] = 0.0;
      }
      if (!WP && kb >= 0 && lowk) {
        // A_0, A_2, A_4 at n and -n on the low-k cube [-nc, nc]^3
        const int D = a.D, nc = a.nc_b;
        const long long DDD = (long long)D * D * D;
        const long long ip = ((long long)(ix + nc) * D + (iy + nc)) * D + (iz + nc);
        const long long im = ((long long)(nc - ix) * D + (nc - iy)) * D + (nc - iz);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          lowk[l * DDD + ip] = cmake<C>((T)A[l][0], (T)A[l][1]);
          lowk[l * DDD + im] = cmake<C>((T)A[l][0], (T)(-A[l][1]));
        }
      }
    }
    wave_run_add<NV>(kp, vp, bins);
    wave_run_add<NV>(kb >= 0 ? a.pk_nb + kb : -1, vb, bins);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nall * NV; i += kBinThreads) part[(long long)i * gridDim.x + blockIdx.x] = bins[i];
}

// Sum of the per-block partials, one wavefront per (bin, quantity) reading
// its nblk contiguous partials, into the kBinSums slots of the bin.  mode 1
// (geometry): slots 0-1; mode 0 (data): slots 2-5 (P_ell bins: S00 S20 S40
// S22) or 5-7 (bispectrum bins: S0w S2w S4w; their fourth quantity is not
// kept); mode 2 (w^2-weighted pass): slots 2-3 of the bispectrum bins (Q2w,
// Q4w).  Grid (wavefront groups, request), as k_bin.
__global__ __launch_bounds__(256) void k_bin_reduce(const double *part, int nblk, int nv, int nall, int pk_nb,
                                                    int mode, double *sum, Batch bt) {
  part = shifted(part, bt.delta[blockIdx.y]);
  sum = shifted(sum, bt.delta[blockIdx.y]);
  const int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= nall * nv) return;  // whole wavefronts
  double s = 0;
  for (int b = lane; b < nblk; b += 64) s += part[(long long)i * nblk + b];
  s = wave_sum(s);
  const int bin = i / nv, q = i - bin * nv;
  const bool keep = mode == 1 || (mode == 0 && (bin < pk_nb || q < 3)) || (mode == 2 && bin >= pk_nb && q < 2);
  if (lane == 0 && keep) {
    const int slot = mode == 1 ? q : (mode == 2 ? 2 + q : (bin < pk_nb ? 2 + q : 5 + q));
    sum[bin * kBinSums + slot] = s;
  }
}

// Output arrays of every request of a batch (device views).
struct PkOuts {
  frsd_pk_out o[kMaxBatch];
};

// Grid (bin blocks, request of the batch); sum and scal are request 0's.
__global__ void k_pk_final(const double *sum, const double *scal, int nb, int ell_max, PkOuts outs, Batch bt) {
  const int r = blockIdx.y;
  sum = moved(sum, bt.delta[r]);
  scal = moved(scal, bt.delta[r]);
  const frsd_pk_out &o = outs.o[r];
  int64_t *n_modes = o.n_modes;
  double *k_eff = o.k_eff, *p0 = o.p0, *p2 = o.p2, *p4 = o.p4, *s00 = o.s00, *s20 = o.s20, *s40 = o.s40,
         *scal_out = o.scalars, *p4b = o.p4b, *s22 = o.s22;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const double I22 = scal[0], N0 = scal[1];
  if (b == 0 && scal_out)
    for (int k = 0; k < kScalars; ++k) scal_out[k] = scal[k];
  if (b >= nb) return;
  const double *v = sum + b * kBinSums;
  const double cnt = v[0];
  n_modes[b] = (int64_t)llrint(cnt);
  k_eff[b] = cnt > 0 ? v[1] / cnt : 0.0;
  s00[b] = v[2]; s20[b] = v[3]; s40[b] = v[4];
  p0[b] = (v[2] / cnt - N0) / I22;
  p2[b] = ell_max >= 2 ? 5.0 * v[3] / (cnt * I22) : __builtin_nan("");
  p4[b] = ell_max >= 4 ? 9.0 * v[4] / (cnt * I22) : __builtin_nan("");
  // split hexadecapole (Sec. II.B eqs. factorizeL4, split, P4fast):
  // L_4 = 35/18 L_2^2 - 5/9 L_2 - 7/18 with L_2^2 split over the pair, times
  // 9, over N_b I22; the raw S00 keeps the self pairs' term the same as in P_4
  if (s22) s22[b] = v[5];
  if (p4b) p4b[b] = ell_max >= 2 ? (17.5 * v[5] - 5.0 * v[3] - 3.5 * v[2]) / (cnt * I22) : __builtin_nan("");
}

static BinArgs bin_args(const frsd_plan *pl) {
  const frsd_params &p = pl->p;
  const SlotDesc &sd = pl->slots;
  BinArgs a{};
  a.N = pl->N; a.nmax = pl->nmax; a.order = p.order; a.interlace = p.interlace; a.compensate = p.compensate;
  a.pk_nb = p.pk_nbins; a.bk_nb = p.bk_nbins; a.pk_lut_len = pl->pk_lut_len; a.bk_lut_len = pl->bk_lut_len;
  a.nc_b = pl->nc_b; a.D = pl->D; a.kf = pl->kf;
  a.n_slot = sd.n_slot;
  for (int m = 0; m < sd.n_mom; ++m) {
    if (sd.mom_id[m] == kMomW) a.has_w = 1;
    else ++a.n_ell;
  }
  return a;
}

// The binning kernel takes the slot layout the plan builds: moment
// positions 0..n_ell-1 in table order, then w^2; with interlacing slot s
// holds position s on both grids, without it positions 2s and 2s+1.
static bool slot_layout_ok(const SlotDesc &sd, const BinArgs &a, bool interlace) {
  if (sd.n_mom != a.n_ell + a.has_w) return false;
  for (int m = 0; m < sd.n_mom; ++m)
    if (sd.mom_id[m] != (m < a.n_ell ? m : kMomW)) return false;
  for (int s = 0; s < sd.n_slot; ++s) {
    const int re = interlace ? s : 2 * s;
    const int im = interlace ? s : (2 * s + 1 < sd.n_mom ? 2 * s + 1 : -1);
    if (sd.re_mom[s] != re || sd.im_mom[s] != im) return false;
  }
  return sd.n_slot == (interlace ? sd.n_mom : (sd.n_mom + 1) / 2);
}

// Mode counts and sum |k| of every bin (data independent; once per plan).
int run_bin_geometry(frsd_plan *pl, void *ws, hipStream_t s) {
  const Layout &L = pl->L;
  const frsd_params &p = pl->p;
  const int nall = p.pk_nbins + p.bk_nbins;
  if (nall > kMaxBinsAll) return fail(FRSD_EINVAL, "too many bins (pk + bk > 512)");
  const BinArgs a = bin_args(pl);
  constexpr int NV = BinValues<true>::n;
  FRSD_TIMED("bin_geom", s, hipLaunchKernelGGL((k_bin<float, true, true>), dim3(pl->tune.bin_blocks), dim3(kBinThreads), 0, s,
                                               (const float2 *)nullptr, 0LL, a,
                                               ws_ptr<const int16_t>(ws, L.pk_lut),
                                               p.bk_nbins > 0 ? ws_ptr<const int16_t>(ws, L.bk_lut) : nullptr,
                                               (float2 *)nullptr, ws_ptr<double>(ws, L.bin_part),
                                               (const float2 *)nullptr, batch_one()));
  FRSD_TIMED("bin_reduce", s, hipLaunchKernelGGL(k_bin_reduce, dim3((nall * NV + 3) / 4), dim3(256), 0, s,
                                                 ws_ptr<const double>(ws, L.bin_part), pl->tune.bin_blocks, NV, nall,
                                                 p.pk_nbins, 1, ws_ptr<double>(ws, L.bin_sum), batch_one()));  // geometry
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

int run_pk_final(frsd_plan *pl, void *const *wss, int n, const frsd_pk_out *out, hipStream_t s);

// Binning of n requests of one shape in one launch (grid y = request), then
// each request's P_ell.  cached: every request's meshes hold galaxies alone,
// combined with its plan's random cache for its own alpha.
template <typename T>
int run_pk_batch(frsd_plan *const *pls, void *const *wss, int n, const frsd_pk_out *out, hipStream_t s,
                 bool cached) {
  frsd_plan *pl = pls[0];
  void *ws = wss[0];
  const Layout &L = pl->L;
  const frsd_params &p = pl->p;
  const int nall = p.pk_nbins + p.bk_nbins;
  if (nall > kMaxBinsAll) return fail(FRSD_EINVAL, "too many bins (pk + bk > 512)");
  if (n < 1 || n > kMaxBatch) return fail(FRSD_EINVAL, "batch size out of range");
  BinArgs a = bin_args(pl);
  if (a.nmax >= kBinTab) return fail(FRSD_EINVAL, "k range too large for the binning tables");
  if (cached) {
    const SlotDesc &sd = pl->slots;
    auto kind = [&](int pos) -> int8_t { return pos < 0 || pos >= sd.n_mom ? 0 : (sd.mom_id[pos] == kMomW ? 2 : 1); };
    a.cached = 1;
    for (int sl = 0; sl < sd.n_slot; ++sl) {
      a.kx[sl] = kind(sd.re_mom[sl]);
      a.ky[sl] = kind(sd.im_mom[sl]);
    }
    for (int r = 0; r < n; ++r) a.alpha[r] = pls[r]->cached_alpha;
  }
  if (!slot_layout_ok(pl->slots, a, p.interlace != 0)) return fail(FRSD_EINVAL, "unexpected slot layout");
  const Batch bt = batch_of(wss, n);
  using C = cplx_t<T>;
  const long long NNN = (long long)pl->N * pl->N * pl->N;
  constexpr int NV = BinValues<false>::n;
  auto kern = p.interlace ? k_bin<T, false, true> : k_bin<T, false, false>;
  FRSD_TIMED("bin", s, hipLaunchKernelGGL(kern, dim3(pl->tune.bin_blocks, n), dim3(kBinThreads), 0, s,
                                          ws_ptr<const C>(ws, L.mesh), NNN, a, ws_ptr<const int16_t>(ws, L.pk_lut),
                                          p.bk_nbins > 0 ? ws_ptr<const int16_t>(ws, L.bk_lut) : nullptr,
                                          p.bk_nbins > 0 ? ws_ptr<C>(ws, L.lowk) : nullptr,
                                          ws_ptr<double>(ws, L.bin_part),
                                          a.cached ? ws_ptr<const C>(ws, L.rcache) : nullptr, bt));
  FRSD_TIMED("bin_reduce", s, hipLaunchKernelGGL(k_bin_reduce, dim3((nall * NV + 3) / 4, n), dim3(256), 0, s,
                                                 ws_ptr<const double>(ws, L.bin_part), pl->tune.bin_blocks, NV, nall,
                                                 p.pk_nbins, 0, ws_ptr<double>(ws, L.bin_sum), bt));
  FRSD_LAUNCH_CHECK();
  return run_pk_final(pl, wss, n, out, s);
}

template <typename T>
int run_pk(frsd_plan *pl, void *ws, const frsd_pk_out *out, hipStream_t s, bool cached) {
  return run_pk_batch<T>(&pl, &ws, 1, out, s, cached);
}

// P_ell from the bin sums (slots 0-5 of every P_ell bin) and the scalars,
// for the n requests of a batch (out: their device views).
int run_pk_final(frsd_plan *pl, void *const *wss, int n, const frsd_pk_out *out, hipStream_t s) {
  const Layout &L = pl->L;
  const frsd_params &p = pl->p;
  PkOuts po{};
  for (int r = 0; r < n; ++r) po.o[r] = out[r];
  FRSD_TIMED("pk_final", s, hipLaunchKernelGGL(k_pk_final, dim3((p.pk_nbins + 255) / 256, n), dim3(256), 0, s,
                                               ws_ptr<const double>(wss[0], L.bin_sum),
                                               ws_ptr<const double>(wss[0], L.scal), p.pk_nbins, p.ell_max, po,
                                               batch_of(wss, n)));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}
int run_pk_final(frsd_plan *pl, void *ws, const frsd_pk_out *out, hipStream_t s) {
  return run_pk_final(pl, &ws, 1, out, s);
}

template int run_pk<float>(frsd_plan *, void *, const frsd_pk_out *, hipStream_t, bool);
template int run_pk<double>(frsd_plan *, void *, const frsd_pk_out *, hipStream_t, bool);
template int run_pk_batch<float>(frsd_plan *const *, void *const *, int, const frsd_pk_out *, hipStream_t, bool);
template int run_pk_batch<double>(frsd_plan *const *, void *const *, int, const frsd_pk_out *, hipStream_t, bool);

// Q_lw = sum_b Re[F_0 (F^w_l)^*] (l = 2, 4) of every bispectrum bin from the
// w^2-weighted moment meshes of run_w_moments (the q_2, q_3 terms of Sec. III.B
// eq. SNbisp2thin), into slots 2-3 of the bispectrum bins' sums.
template <typename T>
int run_bin_w(frsd_plan *pl, void *ws, hipStream_t s) {
  const Layout &L = pl->L;
  const frsd_params &p = pl->p;
  const int nall = p.pk_nbins + p.bk_nbins;
  BinArgs a = bin_args(pl);
  a.nmax = pl->nc_b;
  a.n_ell = pl->n_wmom;
  a.has_w = 0;
  a.n_slot = p.interlace ? pl->n_wmom : (pl->n_wmom + 1) / 2;
  using C = cplx_t<T>;
  const long long NNN = (long long)pl->N * pl->N * pl->N;
  constexpr int NV = BinValues<false>::n;
  auto kern = p.interlace ? k_bin<T, false, true, true> : k_bin<T, false, false, true>;
  FRSD_TIMED("bin_w", s, hipLaunchKernelGGL(kern, dim3(pl->tune.bin_blocks), dim3(kBinThreads), 0, s, ws_ptr<const C>(ws, L.mesh),
                                            NNN, a, ws_ptr<const int16_t>(ws, L.pk_lut),
                                            ws_ptr<const int16_t>(ws, L.bk_lut), ws_ptr<C>(ws, L.lowk),
                                            ws_ptr<double>(ws, L.bin_part), (const C *)nullptr, batch_one()));
  FRSD_TIMED("bin_reduce", s, hipLaunchKernelGGL(k_bin_reduce, dim3((nall * NV + 3) / 4), dim3(256), 0, s,
                                                 ws_ptr<const double>(ws, L.bin_part), pl->tune.bin_blocks, NV, nall,
                                                 p.pk_nbins, 2, ws_ptr<double>(ws, L.bin_sum), batch_one()));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template int run_bin_w<float>(frsd_plan *, void *, hipStream_t);
template int run_bin_w<double>(frsd_plan *, void *, hipStream_t);

}  // namespace frsd
