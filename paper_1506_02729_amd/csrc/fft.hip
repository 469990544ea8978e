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
#include "device.h"
#include "frsd_internal.h"

namespace frsd {


// AXIS 2 reads the planar real arrays `planar` (re, im of mesh b at arrays
// 2b, 2b+1) and writes `data`; AXIS 1 and 0 work in place on `data`.
template <typename T, int AXIS, int LEN>
__global__ __launch_bounds__(FftTune<T>::threads) void k_fft_axis(cplx_t<T> *data, const T *planar, int n_rt, int P_rt,
                                                           StageList st, const cplx_t<T> *tw_g,
                                                           long long batch_stride) {
  using C = cplx_t<T>;
  const int N = LEN ? LEN : n_rt;
  const int P = LEN ? FftTune<T>::pn / LEN : P_rt;
  extern __shared__ unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *lds = tw + N;
  const int ld = N + 1;
  for (int i = threadIdx.x; i < N; i += FftTune<T>::threads) tw[i] = tw_g[i];

  C *mesh = data + (long long)blockIdx.y * batch_stride;
  const long long NN = (long long)N * N;
  const long long q0 = (long long)blockIdx.x * P;  // first pencil of this workgroup
  const int npen = (int)((q0 + P <= NN) ? P : (NN - q0));
  const int tot = npen * N;

  if (AXIS == 2) {
    // pencil q: row q of length N, contiguous in both planar arrays
    const T *re = planar + 2 * (long long)blockIdx.y * batch_stride + q0 * N;
    const T *im = re + batch_stride;
    for (int f = threadIdx.x; f < tot; f += FftTune<T>::threads) {
      const int p = f / N, e = f - p * N;
      lds[p * ld + e] = cmake<C>(re[f], im[f]);
    }
  } else {
    // pencil q = (outer, z) with z fastest; element stride N (AXIS 1) or N^2 (AXIS 0)
    const long long es = (AXIS == 1) ? N : NN;
    for (int f = threadIdx.x; f < tot; f += FftTune<T>::threads) {
      const int e = f / npen, p = f - e * npen;
      const long long q = q0 + p;
      const long long base = (AXIS == 1) ? ((q / N) * NN + (q % N)) : q;
      lds[p * ld + e] = mesh[base + e * es];
    }
  }
  __syncthreads();
  lds_fft_any<C, false, FftTune<T>::threads, FftTune<T>::pn, LEN>(lds, ld, N, npen, st, tw);

  if (AXIS == 2) {
    C *dst = mesh + q0 * N;
    for (int f = threadIdx.x; f < tot; f += FftTune<T>::threads) {
      const int p = f / N, e = f - p * N;
      dst[f] = lds[p * ld + e];
    }
  } else {
    const long long es = (AXIS == 1) ? N : NN;
    for (int f = threadIdx.x; f < tot; f += FftTune<T>::threads) {
      const int e = f / npen, p = f - e * npen;
      const long long q = q0 + p;
      const long long base = (AXIS == 1) ? ((q / N) * NN + (q % N)) : q;
      mesh[base + e * es] = lds[p * ld + e];
    }
  }
}

static StageList stages_of(const FftLen &f) {
  StageList s{};
  s.nstage = f.nstage;
  for (int i = 0; i < f.nstage; ++i) s.radix[i] = f.radix[i];
  return s;
}

template <typename T, int LEN>
static int fft3d_forward_len(const FftLen &f, const void *tw, const void *planar, void *mesh, int n_batch,
                             hipStream_t s) {
  using C = cplx_t<T>;
  const int N = f.n;
  const int P = FftTune<T>::pn / N;
  const long long NN = (long long)N * N;
  const unsigned nblk = (unsigned)((NN + P - 1) / P);
  const size_t shmem = sizeof(C) * ((size_t)N + (size_t)P * (N + 1));
  const StageList st = stages_of(f);
  const long long bs = NN * N;
  dim3 grid(nblk, n_batch);
  FRSD_HIP(hipFuncSetAttribute((const void *)k_fft_axis<T, 2, LEN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_fft_axis<T, 1, LEN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  FRSD_HIP(hipFuncSetAttribute((const void *)k_fft_axis<T, 0, LEN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  FRSD_TIMED("fft_z", s, hipLaunchKernelGGL((k_fft_axis<T, 2, LEN>), grid, dim3(FftTune<T>::threads), shmem, s, (C *)mesh,
                                            (const T *)planar, N, P, st, (const C *)tw, bs));
  FRSD_TIMED("fft_y", s, hipLaunchKernelGGL((k_fft_axis<T, 1, LEN>), grid, dim3(FftTune<T>::threads), shmem, s, (C *)mesh,
                                            (const T *)planar, N, P, st, (const C *)tw, bs));
  FRSD_TIMED("fft_x", s, hipLaunchKernelGGL((k_fft_axis<T, 0, LEN>), grid, dim3(FftTune<T>::threads), shmem, s, (C *)mesh,
                                            (const T *)planar, N, P, st, (const C *)tw, bs));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

template <typename T>
int fft3d_forward(const FftLen &f, const void *tw, const void *planar, void *mesh, int n_batch, hipStream_t s) {
  switch (f.n) {
#define FRSD_CASE(L) \
  case L: return fft3d_forward_len<T, L>(f, tw, planar, mesh, n_batch, s);
    FRSD_FFT_LENGTHS(FRSD_CASE)
#undef FRSD_CASE
    default: return fft3d_forward_len<T, 0>(f, tw, planar, mesh, n_batch, s);
  }
}

template int fft3d_forward<float>(const FftLen &, const void *, const void *, void *, int, hipStream_t);
template int fft3d_forward<double>(const FftLen &, const void *, const void *, void *, int, hipStream_t);

}  // namespace frsd
