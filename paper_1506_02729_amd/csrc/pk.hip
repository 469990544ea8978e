// Steps a5-a6: multipole combination and |k|-shell binning, fused
// (Sec. II.B eqs. delta2b, delta4b; Sec. III.A eqs. F2, P0_impl-P4_impl).
//
// One thread per wave-vector n of the half space (n and -n give complex-
// conjugate contributions, so each half-space mode is counted twice).  For
// every complex slot the thread reads Z(n) and Z(-n), and accumulates the
// real-coefficient combinations needed for F_0, F_2, F_4 and F_0^w:
//   F_2 = 3/2 sum_m mult_m khat^m Q_m - 1/2 F_0,
//   F_4 = 35/8 sum_m mult_m khat^m Q_m - 5/2 F_2 - 7/8 F_0.
// Because every step after the FFT is linear with real coefficients, the
// unpacking of the two real planes of a slot (X = [Z(n) + Z(-n)^*] / 2,
// Y = [Z(n) - Z(-n)^*] / 2i), the interlacing 1/2 [X + exp(-i pi sum n / N) Y]
// and the window compensation prod sinc(pi n_d / N)^p are applied once per
// multipole to the combined sums.  Shell sums are reduced per wavefront by
// bin key and accumulated in FP64: three data sums per bin, since the mode
// counts and sum |k| of every bin do not depend on the data and are summed
// once per plan by the same kernel in its geometry mode.
#include <cmath>

#include "device.h"
#include "frsd_internal.h"

namespace frsd {

constexpr int kBinThreads = 256;
constexpr int kMaxBinsAll = 512;

struct BinArgs {
  int N, nmax, order, interlace, compensate;
  int pk_nb, bk_nb, pk_lut_len, bk_lut_len;
  int nc_b, D;  // low-k cube
  int ell_max, has_w;
  double kf;
};

struct CoefArgs {  // per moment position: rank, components, multiplicity
  int8_t idx[kMaxMom][4];
  int8_t rank[kMaxMom];
  float mult[kMaxMom];
};

// Reduce v[NV] over the lanes of the wavefront that share `key`, one
// distinct key at a time, and add the sums to lds_bins[key * NV + *].
template <int NV>
__device__ __forceinline__ void wave_bin_add(int key, const double *v, double *lds_bins) {
  const int lane = threadIdx.x & 63;
  bool pending = key >= 0;
  while (true) {
    const unsigned long long mask = __ballot(pending);
    if (mask == 0ull) break;
    const int leader = __ffsll((long long)mask) - 1;
    const int k = __shfl(key, leader, 64);
    const bool mine = pending && key == k;
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const double t = wave_sum(mine ? v[s] : 0.0);
      if (lane == leader) atomicAdd(&lds_bins[k * NV + s], t);
    }
    if (mine) pending = false;
  }
}

// Per-mode sums reduced by the binning kernel: GEOM (once per plan) the
// mode count and sum |k| of every bin; otherwise the data sums, (S00, S20,
// S40) for the P_ell bins and (S0w, S2w, S4w) for the bispectrum bins.
template <bool GEOM> struct BinValues { static constexpr int n = GEOM ? 2 : 3; };

template <typename T, bool GEOM>
__global__ __launch_bounds__(kBinThreads) void k_bin(const cplx_t<T> *__restrict__ mesh, long long slot_stride,
                                                      SlotDesc sd, CoefArgs ca, BinArgs a,
                                                      const int16_t *__restrict__ pk_lut,
                                                      const int16_t *__restrict__ bk_lut, cplx_t<T> *lowk,
                                                      double *part) {
  using C = cplx_t<T>;
  constexpr int NV = BinValues<GEOM>::n;
  __shared__ double bins[kMaxBinsAll * 3];
  const int nall = a.pk_nb + a.bk_nb;
  for (int i = threadIdx.x; i < nall * NV; i += kBinThreads) bins[i] = 0.0;
  __syncthreads();

  const int N = a.N, nm = a.nmax;
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
    if (t < total) {
      const int iz = (int)(t % (nm + 1));
      const long long r = t / (nm + 1);
      const int iy = (int)(r % side) - nm;
      const int ix = (int)(r / side) - nm;
      const bool half = (iz > 0) || (iy > 0) || (iy == 0 && ix > 0);
      const long long m2 = (long long)ix * ix + (long long)iy * iy + (long long)iz * iz;
      if (half) {
        kp = (m2 < a.pk_lut_len) ? pk_lut[m2] : -1;
        kb = (a.bk_nb > 0 && m2 < a.bk_lut_len) ? bk_lut[m2] : -1;
      }
      if (GEOM && (kp >= 0 || kb >= 0)) {
        const double kmag = a.kf * sqrt((double)m2);
        vp[0] = 2.0; vp[1] = 2.0 * kmag;
        vb[0] = 2.0; vb[1] = 2.0 * kmag;
      }
      if (!GEOM && (kp >= 0 || kb >= 0)) {
        const T kk = (T)sqrt((double)m2);
        const T kh[3] = {(T)ix / kk, (T)iy / kk, (T)iz / kk};
        const long long gp = ((long long)((ix + N) % N) * N + (iy + N) % N) * N + iz;
        const long long gm = ((long long)((N - ix) % N) * N + (N - iy) % N) * N + (N - iz) % N;
        // accumulators [ell: 0, 2, 4, w][re-plane / im-plane][n / -n]
        C zr[4][2], zi[4][2];
#pragma unroll
        for (int l = 0; l < 4; ++l)
#pragma unroll
          for (int q = 0; q < 2; ++q) { zr[l][q] = cmake<C>(T(0), T(0)); zi[l][q] = cmake<C>(T(0), T(0)); }
        for (int sl = 0; sl < sd.n_slot; ++sl) {
          const C zp = mesh[sl * slot_stride + gp];
          const C zm = mesh[sl * slot_stride + gm];
#pragma unroll
          for (int part2 = 0; part2 < 2; ++part2) {
            const int mp = part2 == 0 ? sd.re_mom[sl] : sd.im_mom[sl];
            if (mp < 0) continue;
            const int id = sd.mom_id[mp];
            T c[4] = {T(0), T(0), T(0), T(0)};
            if (id == kMomW) {
              c[3] = T(1);
            } else {
              T mono = T(ca.mult[id]);
              for (int k = 0; k < ca.rank[id]; ++k) mono *= kh[ca.idx[id][k]];
              if (ca.rank[id] == 0) { c[0] = T(1); c[1] = T(-0.5); c[2] = T(0.375); }
              else if (ca.rank[id] == 2) { c[1] = T(1.5) * mono; c[2] = T(-3.75) * mono; }
              else { c[2] = T(4.375) * mono; }
            }
            C(*acc)[2] = part2 == 0 ? zr : zi;
#pragma unroll
            for (int l = 0; l < 4; ++l) {
              acc[l][0] = cadd(acc[l][0], cscale(zp, c[l]));
              acc[l][1] = cadd(acc[l][1], cscale(zm, c[l]));
            }
          }
        }
        // unpack, interlace, compensate
        double ph_re = 1.0, ph_im = 0.0, s = 1.0;
        if (a.interlace) {
          sincospi(-(double)(ix + iy + iz) / N, &ph_im, &ph_re);
          s = 0.5;
        }
        double win = 1.0;
        if (a.compensate) {
          const int nn[3] = {ix, iy, iz};
          for (int d = 0; d < 3; ++d) {
            if (nn[d] != 0) {
              const double x = (double)nn[d] / N;
              const double sc = sinpi(x) / (M_PI * x);
              double wp = sc;
              for (int q = 1; q < a.order; ++q) wp *= sc;
              win *= wp;
            }
          }
        }
        const double scale = s / win;
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
        // each half-space mode stands for n and -n
        vp[0] = 2.0 * S00; vp[NV > 1 ? 1 : 0] = 2.0 * S20; vp[NV - 1] = 2.0 * S40;
        vb[0] = 2.0 * S0w; vb[NV > 1 ? 1 : 0] = 2.0 * S2w; vb[NV - 1] = 2.0 * S4w;
        if (kb >= 0 && lowk) {
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
    }
    wave_bin_add<NV>(kp, vp, bins);
    wave_bin_add<NV>(kb >= 0 ? a.pk_nb + kb : -1, vb, bins);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nall * NV; i += kBinThreads) part[(long long)i * gridDim.x + blockIdx.x] = bins[i];
}

// Sum of the per-block partials, one thread per (bin, quantity), into the
// kBinSums slots of the bin: geometry into slots 0-1, data sums into 2-4
// (P_ell bins) or 5-7 (bispectrum bins).
__global__ void k_bin_reduce(const double *part, int nblk, int nv, int nall, int pk_nb, int geom, double *sum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nall * nv) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += part[(long long)i * nblk + b];
  const int bin = i / nv, q = i - bin * nv;
  const int slot = geom ? q : (bin < pk_nb ? 2 + q : 5 + q);
  sum[bin * kBinSums + slot] = s;
}

__global__ void k_pk_final(const double *sum, const double *scal, int nb, int ell_max, int64_t *n_modes, double *k_eff,
                           double *p0, double *p2, double *p4, double *s00, double *s20, double *s40,
                           double *scal_out) {
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
}

static BinArgs bin_args(const frsd_plan *pl) {
  const frsd_params &p = pl->p;
  BinArgs a{};
  a.N = pl->N; a.nmax = pl->nmax; a.order = p.order; a.interlace = p.interlace; a.compensate = p.compensate;
  a.pk_nb = p.pk_nbins; a.bk_nb = p.bk_nbins; a.pk_lut_len = pl->pk_lut_len; a.bk_lut_len = pl->bk_lut_len;
  a.nc_b = pl->nc_b; a.D = pl->D; a.ell_max = p.ell_max; a.has_w = p.bk_nbins > 0; a.kf = pl->kf;
  return a;
}

// Mode counts and sum |k| of every bin (data independent; once per plan).
int run_bin_geometry(frsd_plan *pl, void *ws, hipStream_t s) {
  const Layout &L = pl->L;
  const frsd_params &p = pl->p;
  const int nall = p.pk_nbins + p.bk_nbins;
  if (nall > kMaxBinsAll) return fail(FRSD_EINVAL, "too many bins (pk + bk > 512)");
  const BinArgs a = bin_args(pl);
  constexpr int NV = BinValues<true>::n;
  FRSD_TIMED("bin_geom", s, hipLaunchKernelGGL((k_bin<float, true>), dim3(kBinBlocks), dim3(kBinThreads), 0, s,
                                               (const float2 *)nullptr, 0LL, pl->slots, CoefArgs{}, a,
                                               ws_ptr<const int16_t>(ws, L.pk_lut),
                                               p.bk_nbins > 0 ? ws_ptr<const int16_t>(ws, L.bk_lut) : nullptr,
                                               (float2 *)nullptr, ws_ptr<double>(ws, L.bin_part)));
  FRSD_TIMED("bin_reduce", s, hipLaunchKernelGGL(k_bin_reduce, dim3((nall * NV + 255) / 256), dim3(256), 0, s,
                                                 ws_ptr<const double>(ws, L.bin_part), kBinBlocks, NV, nall,
                                                 p.pk_nbins, 1, ws_ptr<double>(ws, L.bin_sum)));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template <typename T>
int run_pk(frsd_plan *pl, void *ws, const frsd_pk_out *out, hipStream_t s) {
  const Layout &L = pl->L;
  const frsd_params &p = pl->p;
  const int nall = p.pk_nbins + p.bk_nbins;
  if (nall > kMaxBinsAll) return fail(FRSD_EINVAL, "too many bins (pk + bk > 512)");
  const BinArgs a = bin_args(pl);
  CoefArgs ca{};
  const MomentTable &tab = moment_table();
  for (int i = 0; i < kMaxMom; ++i) {
    ca.rank[i] = tab.rank[i]; ca.mult[i] = tab.mult[i];
    for (int k = 0; k < 4; ++k) ca.idx[i][k] = tab.idx[i][k];
  }
  using C = cplx_t<T>;
  const long long NNN = (long long)pl->N * pl->N * pl->N;
  constexpr int NV = BinValues<false>::n;
  FRSD_TIMED("bin", s, hipLaunchKernelGGL((k_bin<T, false>), dim3(kBinBlocks), dim3(kBinThreads), 0, s, ws_ptr<const C>(ws, L.mesh), NNN,
                     pl->slots, ca, a, ws_ptr<const int16_t>(ws, L.pk_lut),
                     p.bk_nbins > 0 ? ws_ptr<const int16_t>(ws, L.bk_lut) : nullptr,
                     p.bk_nbins > 0 ? ws_ptr<C>(ws, L.lowk) : nullptr, ws_ptr<double>(ws, L.bin_part)));
  FRSD_TIMED("bin_reduce", s, hipLaunchKernelGGL(k_bin_reduce, dim3((nall * NV + 255) / 256), dim3(256), 0, s,
                                                 ws_ptr<const double>(ws, L.bin_part), kBinBlocks, NV, nall,
                                                 p.pk_nbins, 0, ws_ptr<double>(ws, L.bin_sum)));
  FRSD_TIMED("pk_final", s, hipLaunchKernelGGL(k_pk_final, dim3((p.pk_nbins + 255) / 256), dim3(256), 0, s, ws_ptr<const double>(ws, L.bin_sum),
                     ws_ptr<const double>(ws, L.scal), p.pk_nbins, p.ell_max, out->n_modes, out->k_eff, out->p0, out->p2,
                     out->p4, out->s00, out->s20, out->s40, out->scalars));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template int run_pk<float>(frsd_plan *, void *, const frsd_pk_out *, hipStream_t);
template int run_pk<double>(frsd_plan *, void *, const frsd_pk_out *, hipStream_t);

}  // namespace frsd
