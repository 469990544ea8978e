// Streamed power-spectrum multipoles for meshes whose full set of moment
// meshes does not fit the device (e.g. N = 1024: 15 interlaced complex FP32
// meshes take 129 GB, twice that with the assignment planes).
//
// The moment meshes are gridded, transformed and consumed a group of
// stream_slots complex slots at a time: after each group's forward FFTs,
// k_stream_acc adds that group's part of the class sums
//   R_0 = Q_0,  R_2 = sum_ab khat_a khat_b Q_ab,  R_4 (rank 4), over the
//   kept moments with their class_coeffs coefficients
// (Sec. II.B eqs. delta2b, delta4b, with Q_m unpacked from the packed slot,
// interlaced and compensated as in the binning kernel) into accumulators on
// the half space of kept frequencies.  Everything after the FFT is linear, so
// the sums over groups are the sums over all moments.  k_stream_bin then
// forms A_0 = R_0, A_2 = 3/2 R_2 - 1/2 R_0, A_4 = 35/8 R_4 - 15/4 R_2 +
// 3/8 R_0 per mode and the FP64 shell sums S_00, S_20, S_40, S_22 of P_ell
// (Sec. III.A eqs. P0_impl-P4_impl) and P_4b.
//
// Resident at once: the records, stream_slots slots of assignment planes and
// of complex meshes (2 unless the plan asks for more), and three accumulators
// of (2 n_max + 1)^2 (n_max + 1) modes.
#include <algorithm>
#include <cmath>

#include "device.h"
#include "frsd_internal.h"

namespace frsd {

template <typename T>
int run_grid_group(frsd_plan *pl, void *ws, int m0, int m1, hipStream_t s);
template <typename T>
int ingest_and_sort(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                    hipStream_t s, const double *dyn);

constexpr int kAccThreads = 256;
constexpr int kAccTab = 513;  // |n| <= N/2 for N <= 1024

struct AccArgs {
  int N, nm, m2max, pk_lut_len;
  int order, interlace, compensate;
  int pos0, npos, n_mom, nslot;  // first moment position of the group, positions in it, all positions, slots
  int first;                     // the first group writes the accumulators instead of adding
  long long acc_stride;          // elements per accumulator
};

// Per-axis interlacing phase exp(-i pi n / N) and inverse window, |n| <= nm.
__device__ void axis_tables(int nm, int N, int order, int compensate, double *tcos, double *tsin, double *tiw) {
  for (int n = threadIdx.x; n <= nm; n += blockDim.x) {
    const double x = (double)n / N;
    double sn, cs;
    sincospi(x, &sn, &cs);
    tcos[n] = cs;
    tsin[n] = -sn;
    double iw = 1.0;
    if (compensate && n != 0) {
      const double sc = sn / (M_PI * x);
      double wp = sc;
      for (int q = 1; q < order; ++q) wp *= sc;
      iw = 1.0 / wp;
    }
    tiw[n] = iw;
  }
}

// Half-space mode t of the box [-nm, nm]^2 x [0, nm] (z fastest).
__device__ __forceinline__ void acc_mode(long long t, int nm, int &ix, int &iy, int &iz) {
  iz = (int)(t % (nm + 1));
  const long long r = t / (nm + 1);
  const int side = 2 * nm + 1;
  iy = (int)(r % side) - nm;
  ix = (int)(r / side) - nm;
}

template <typename T>
__global__ __launch_bounds__(kAccThreads) void k_stream_acc(const cplx_t<T> *__restrict__ mesh, long long slot_stride,
                                                            const int16_t *__restrict__ lut, AccArgs a,
                                                            cplx_t<T> *__restrict__ acc) {
  using C = cplx_t<T>;
  __shared__ double tcos[kAccTab], tsin[kAccTab], tiw[kAccTab];
  axis_tables(a.nm, a.N, a.order, a.compensate, tcos, tsin, tiw);
  __syncthreads();
  const int N = a.N, nm = a.nm;
  for (long long t = blockIdx.x * (long long)kAccThreads + threadIdx.x; t < a.acc_stride;
       t += (long long)gridDim.x * kAccThreads) {
    int ix, iy, iz;
    acc_mode(t, nm, ix, iy, iz);
    const bool half = (iz > 0) || (iy > 0) || (iy == 0 && ix > 0);
    const long long m2 = (long long)ix * ix + (long long)iy * iy + (long long)iz * iz;
    if (!half || m2 >= a.pk_lut_len || lut[m2] < 0) continue;  // only modes of a P_ell bin
    const long long gp = ((long long)((ix + N) % N) * N + (iy + N) % N) * N + iz;
    const long long gm = ((long long)((N - ix) % N) * N + (N - iy) % N) * N + (N - iz) % N;
    const double ik = 1.0 / sqrt((double)m2);
    double c2[kMomRank2], c4[kMomRank4];
    class_coeffs<double>(ix * ik, iy * ik, iz * ik, c2, c4);
    const int ax = ix < 0 ? -ix : ix, ay = iy < 0 ? -iy : iy;
    double ph_re = 1.0, ph_im = 0.0, sc = 1.0;
    if (a.interlace) {
      const double cx = tcos[ax], sx = ix < 0 ? -tsin[ax] : tsin[ax];
      const double cy = tcos[ay], sy = iy < 0 ? -tsin[ay] : tsin[ay];
      const double cz = tcos[iz], sz = tsin[iz];
      const double cxy = cx * cy - sx * sy, sxy = cx * sy + sx * cy;
      ph_re = cxy * cz - sxy * sz;
      ph_im = cxy * sz + sxy * cz;
      sc = 0.5;
    }
    const double win = tiw[ax] * tiw[ay] * tiw[iz];
    double r[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    // moment p into R_0, R_2, R_4 with its class coefficients (plans with
    // l_max = 4: every moment reaches R_4, the monopole and rank-2 ones R_2)
    auto add = [&](int p, double qr, double qi) {
      if (p == 0) {
        r[0][0] += qr;
        r[0][1] += qi;
      }
      if (p < kMomRank2 && a.n_mom > 1) {
        r[1][0] += c2[p] * qr;
        r[1][1] += c2[p] * qi;
      }
      if (a.n_mom > kMomRank2) {
        r[2][0] += c4[p] * qr;
        r[2][1] += c4[p] * qi;
      }
    };
    for (int g = 0; g < a.nslot; ++g) {
      const C zp = mesh[g * slot_stride + gp], zm = mesh[g * slot_stride + gm];
      // X = (Z(n) + Z(-n)^*) / 2, Y = (Z(n) - Z(-n)^*) / 2i
      const double xr = 0.5 * ((double)zp.x + (double)zm.x), xi = 0.5 * ((double)zp.y - (double)zm.y);
      const double yr = 0.5 * ((double)zp.y + (double)zm.y), yi = -0.5 * ((double)zp.x - (double)zm.x);
      if (a.interlace) {
        const int p = a.pos0 + g;
        if (p >= a.pos0 + a.npos) continue;
        const double pr = ph_re * yr - ph_im * yi, pi = ph_re * yi + ph_im * yr;
        add(p, sc * win * (xr + pr), sc * win * (xi + pi));
      } else {
        const int p0 = a.pos0 + 2 * g, p1 = p0 + 1;
        if (p0 < a.pos0 + a.npos) add(p0, win * xr, win * xi);
        if (p1 < a.pos0 + a.npos) add(p1, win * yr, win * yi);
      }
    }
#pragma unroll
    for (int cl = 0; cl < 3; ++cl) {
      C *dst = acc + cl * a.acc_stride + t;
      const C v = a.first ? cmake<C>(T(0), T(0)) : *dst;
      *dst = cmake<C>((T)(v.x + r[cl][0]), (T)(v.y + r[cl][1]));
    }
  }
}

// Sum v[4] over runs of equal keys in the wavefront into lds bins (the same
// segmented reduction as the binning kernel).
__device__ __forceinline__ void run_add4(int key, double *v, double *lds_bins) {
  if (__ballot(key >= 0) == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64), next = __shfl_down(key, 1, 64);
  int start = (lane == 0 || prev != key) ? lane : 0;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) start = max(start, __shfl_up(start, o, 64));
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const bool take = lane - o >= start;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double t = __shfl_up(v[s], o, 64);
      v[s] += take ? t : 0.0;
    }
  }
  if (key >= 0 && (lane == 63 || next != key)) {
#pragma unroll
    for (int s = 0; s < 4; ++s) atomicAdd(&lds_bins[key * 4 + s], v[s]);
  }
}

constexpr int kMaxStreamBins = 1024;

template <typename T>
__global__ __launch_bounds__(kAccThreads) void k_stream_bin(const cplx_t<T> *__restrict__ acc, long long acc_stride,
                                                            int nm, int pk_lut_len, const int16_t *__restrict__ lut,
                                                            int nb, double *part) {
  using C = cplx_t<T>;
  __shared__ double bins[kMaxStreamBins * 4];
  for (int i = threadIdx.x; i < nb * 4; i += kAccThreads) bins[i] = 0.0;
  __syncthreads();
  const long long stride = (long long)gridDim.x * kAccThreads;
  const long long iters = (acc_stride + stride - 1) / stride;  // uniform trip count for the wavefront sums
  for (long long it = 0; it < iters; ++it) {
    const long long t = blockIdx.x * (long long)kAccThreads + threadIdx.x + it * stride;
    int key = -1;
    double v[4] = {0, 0, 0, 0};
    if (t < acc_stride) {
      int ix, iy, iz;
      acc_mode(t, nm, ix, iy, iz);
      const bool half = (iz > 0) || (iy > 0) || (iy == 0 && ix > 0);
      const long long m2 = (long long)ix * ix + (long long)iy * iy + (long long)iz * iz;
      if (half && m2 < pk_lut_len) key = lut[m2];
      if (key >= 0) {
        const C r0 = acc[t], r2 = acc[acc_stride + t], r4 = acc[2 * acc_stride + t];
        const double a0r = r0.x, a0i = r0.y;
        const double a2r = 1.5 * r2.x - 0.5 * r0.x, a2i = 1.5 * r2.y - 0.5 * r0.y;
        const double a4r = 4.375 * r4.x - 3.75 * r2.x + 0.375 * r0.x, a4i = 4.375 * r4.y - 3.75 * r2.y + 0.375 * r0.y;
        // each half-space mode stands for n and -n
        v[0] = 2.0 * (a0r * a0r + a0i * a0i);
        v[1] = 2.0 * (a2r * a0r + a2i * a0i);
        v[2] = 2.0 * (a4r * a0r + a4i * a0i);
        v[3] = 2.0 * (a2r * a2r + a2i * a2i);
      }
    }
    run_add4(key, v, bins);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb * 4; i += kAccThreads) part[(long long)i * gridDim.x + blockIdx.x] = bins[i];
}

// Sum of the per-block partials into slots 2-5 of each bin (S00 S20 S40 S22).
__global__ __launch_bounds__(256) void k_stream_reduce(const double *part, int nblk, int nb, double *sum) {
  const int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= nb * 4) return;
  double s = 0;
  for (int b = lane; b < nblk; b += 64) s += part[(long long)i * nblk + b];
  s = wave_sum(s);
  if (lane == 0) sum[(i / 4) * kBinSums + 2 + (i % 4)] = s;
}

static AccArgs acc_args(const frsd_plan *pl) {
  AccArgs a{};
  a.N = pl->N;
  a.nm = pl->nc_p;
  a.pk_lut_len = pl->pk_lut_len;
  a.order = pl->p.order;
  a.interlace = pl->p.interlace;
  a.compensate = pl->p.compensate;
  a.n_mom = pl->slots.n_mom;
  const long long side = 2LL * a.nm + 1;
  a.acc_stride = side * side * (a.nm + 1);
  return a;
}

size_t stream_acc_bytes(const frsd_plan *pl, size_t tbytes) {
  const size_t side = 2 * (size_t)pl->nc_p + 1;
  return 3 * 2 * tbytes * side * side * ((size_t)pl->nc_p + 1);
}

template <typename T>
int run_stream_assign(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                      hipStream_t s) {
  using C = cplx_t<T>;
  int rc = ingest_and_sort<T>(pl, ws, gal, ran, alpha, s, nullptr);
  if (rc) return rc;
  const Layout &L = pl->L;
  AccArgs a = acc_args(pl);
  const int per_slot = pl->p.interlace ? 1 : 2;          // moment positions per complex slot
  const int pos_per_group = pl->stream_slots * per_slot;
  const long long NNN = (long long)pl->N * pl->N * pl->N;
  for (int p0 = 0; p0 < a.n_mom; p0 += pos_per_group) {
    const int p1 = std::min(a.n_mom, p0 + pos_per_group);
    if ((rc = run_grid_group<T>(pl, ws, p0, p1, s))) return rc;
    const int nslot = (p1 - p0 + per_slot - 1) / per_slot;
    if ((rc = fft3d_forward<T>(pl->fft_n, ws_ptr<void>(ws, L.tw_fwd), ws_ptr<const void>(ws, L.planar),
                               ws_ptr<void>(ws, L.mesh), nslot, pl->nmax, pl->pk_lut_len - 1,
                               ws_ptr<const uint8_t>(ws, L.colmask), ws_ptr<const uint8_t>(ws, L.xmask), s,
                               pl->tune.row_grid)))
      return rc;
    a.pos0 = p0;
    a.npos = p1 - p0;
    a.nslot = nslot;
    a.first = p0 == 0;
    FRSD_TIMED("stream_acc", s, hipLaunchKernelGGL(k_stream_acc<T>, dim3(4096), dim3(kAccThreads), 0, s,
                                                   ws_ptr<const C>(ws, L.mesh), NNN,
                                                   ws_ptr<const int16_t>(ws, L.pk_lut), a, ws_ptr<C>(ws, L.acc)));
    FRSD_LAUNCH_CHECK();
  }
  return FRSD_OK;
}

int run_pk_final(frsd_plan *pl, void *ws, const frsd_pk_out *out, hipStream_t s);

template <typename T>
int run_stream_pk(frsd_plan *pl, void *ws, const frsd_pk_out *out, hipStream_t s) {
  using C = cplx_t<T>;
  const Layout &L = pl->L;
  const int nb = pl->p.pk_nbins;
  if (nb > kMaxStreamBins) return fail(FRSD_EINVAL, "too many power-spectrum bins for a streamed plan");
  const AccArgs a = acc_args(pl);
  const int nblk = pl->tune.bin_blocks;
  FRSD_TIMED("stream_bin", s, hipLaunchKernelGGL(k_stream_bin<T>, dim3(nblk), dim3(kAccThreads), 0, s,
                                                 ws_ptr<const C>(ws, L.acc), a.acc_stride, a.nm, a.pk_lut_len,
                                                 ws_ptr<const int16_t>(ws, L.pk_lut), nb, ws_ptr<double>(ws, L.bin_part)));
  FRSD_TIMED("bin_reduce", s, hipLaunchKernelGGL(k_stream_reduce, dim3((nb * 4 + 3) / 4), dim3(256), 0, s,
                                                 ws_ptr<const double>(ws, L.bin_part), nblk, nb,
                                                 ws_ptr<double>(ws, L.bin_sum)));
  FRSD_LAUNCH_CHECK();
  return run_pk_final(pl, ws, out, s);
}

template int run_stream_assign<float>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                      hipStream_t);
template int run_stream_assign<double>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                       hipStream_t);
template int run_stream_pk<float>(frsd_plan *, void *, const frsd_pk_out *, hipStream_t);
template int run_stream_pk<double>(frsd_plan *, void *, const frsd_pk_out *, hipStream_t);

}  // namespace frsd
