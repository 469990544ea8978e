// Device helpers: complex arithmetic, wavefront reductions and the
// LDS-resident mixed-radix Stockham FFT used by every transform in the
// library (forward moment-mesh FFTs and shell-filtered inverse FFTs).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace frsd {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };
template <typename T> using cplx_t = typename Cplx<T>::type;

template <typename C> __device__ __forceinline__ C cmake(decltype(C{}.x) a, decltype(C{}.x) b) {
  C r; r.x = a; r.y = b; return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return cmake<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) {
  return cmake<C>(a.x * s, a.y * s);
}
// multiply by -i (forward) or +i (inverse)
template <typename C, bool INV> __device__ __forceinline__ C cmul_mi(C a) {
  return INV ? cmake<C>(-a.y, a.x) : cmake<C>(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Wavefront (64-lane) sum of a double.
// ---------------------------------------------------------------------------
// Coefficients of the kept moments (IDs 0-14, see frsd_internal.h) in the
// class sums R_2 = sum_j w_j (khat.xhat_j)^2 = sum_ab khat_a khat_b Q_ab and
// R_4 = sum_j w_j (khat.xhat_j)^4, with the eliminated components folded in
// through the trace relations: c2[p] for R_2 (p = 0-5), c4[p] for R_4
// (p = 0-14).  (R_0 = Q_0.)
template <typename T>
__device__ __forceinline__ void class_coeffs(T hx, T hy, T hz, T *c2, T *c4) {
  const T xx = hx * hx, yy = hy * hy, zz = hz * hz, xy = hx * hy, yz = hy * hz, zx = hz * hx;
  const T z4 = zz * zz, zzxx = zz * xx, zzyy = zz * yy;
  c2[0] = zz;
  c2[1] = xx - zz;
  c2[2] = yy - zz;
  c2[3] = T(2) * xy;
  c2[4] = T(2) * yz;
  c2[5] = T(2) * zx;
  c4[0] = z4;
  c4[1] = T(6) * zzxx - T(2) * z4;
  c4[2] = T(6) * zzyy - T(2) * z4;
  c4[3] = T(12) * zz * xy;
  c4[4] = T(4) * zz * yz;
  c4[5] = T(4) * zz * zx;
  c4[6] = xx * xx + z4 - T(6) * zzxx;                        // xxxx
  c4[7] = yy * yy + z4 - T(6) * zzyy;                        // yyyy
  c4[8] = T(4) * xx * xy - T(12) * zz * xy;                  // xxxy
  c4[9] = T(4) * xx * zx - T(4) * zz * zx;                   // xxxz
  c4[10] = T(4) * yy * xy - T(12) * zz * xy;                 // yyyx
  c4[11] = T(4) * yy * yz - T(4) * zz * yz;                  // yyyz
  c4[12] = T(6) * xx * yy + T(2) * z4 - T(6) * (zzxx + zzyy);  // xxyy
  c4[13] = T(12) * xx * yz - T(4) * zz * yz;                 // xxyz
  c4[14] = T(12) * yy * zx - T(4) * zz * zx;                 // yyxz
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Small DFTs.  Forward uses exp(-2 pi i r k / R); INV uses exp(+...).
// ---------------------------------------------------------------------------
template <typename C, bool INV> __device__ __forceinline__ void dft2(C &a, C &b) {
  C t = a; a = cadd(t, b); b = csub(t, b);
}

template <typename C, bool INV> __device__ __forceinline__ void dft4(C &x0, C &x1, C &x2, C &x3) {
  C t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3);
  C t3 = cmul_mi<C, INV>(csub(x1, x3));
  x0 = cadd(t0, t2); x2 = csub(t0, t2); x1 = cadd(t1, t3); x3 = csub(t1, t3);
}

template <typename C, bool INV> __device__ __forceinline__ void dft3(C &x0, C &x1, C &x2) {
  using S = decltype(C{}.x);
  const S h = S(0.8660254037844386467637231707529361834714);  // sqrt(3)/2
  C t = cadd(x1, x2);
  C m = csub(x0, cscale(t, S(0.5)));
  C d = csub(x1, x2);
  // s = d * (-i sqrt3/2) forward, d * (+i sqrt3/2) inverse
  C s = cscale(cmul_mi<C, INV>(d), h);
  x0 = cadd(x0, t); x1 = cadd(m, s); x2 = csub(m, s);
}

// 5-point DFT from the real/imaginary split of the 2 conjugate pairs of
// fifth roots of unity: with t1 = x1 + x4, t2 = x2 + x3, t3 = x1 - x4,
// t4 = x2 - x3, c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5),
//   X1, X4 = x0 + c1 t1 + c2 t2 -/+ i (s1 t3 + s2 t4),
//   X2, X3 = x0 + c2 t1 + c1 t2 -/+ i (s2 t3 - s1 t4)
// (signs of i swapped for INV).
template <typename C, bool INV> __device__ __forceinline__ void dft5(C *v) {
  using S = decltype(C{}.x);
  const S c1 = S(0.3090169943749474241022934171828190588602);   // cos(2 pi / 5)
  const S c2 = S(-0.8090169943749474241022934171828190588602);  // cos(4 pi / 5)
  const S s1 = S(0.9510565162951535721164393333793821434057);   // sin(2 pi / 5)
  const S s2 = S(0.5877852522924731291687059546390727685977);   // sin(4 pi / 5)
  const C x0 = v[0];
  const C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  const C t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  const C a1 = cadd(x0, cadd(cscale(t1, c1), cscale(t2, c2)));
  const C a2 = cadd(x0, cadd(cscale(t1, c2), cscale(t2, c1)));
  const C b1 = cmul_mi<C, INV>(cadd(cscale(t3, s1), cscale(t4, s2)));
  const C b2 = cmul_mi<C, INV>(csub(cscale(t3, s2), cscale(t4, s1)));
  v[0] = cadd(x0, cadd(t1, t2));
  v[1] = cadd(a1, b1); v[4] = csub(a1, b1);
  v[2] = cadd(a2, b2); v[3] = csub(a2, b2);
}

// 7-point DFT, the same split over the 3 conjugate pairs: with t_j =
// x_j + x_{7-j}, d_j = x_j - x_{7-j} (j = 1, 2, 3), c_k = cos(2 pi k / 7),
// s_k = sin(2 pi k / 7),
//   X_m, X_{7-m} = x0 + sum_j c_{mj} t_j -/+ i sum_j s_{mj} d_j   (m = 1, 2, 3),
// indices mj taken mod 7 with c_{7-k} = c_k and s_{7-k} = -s_k (signs of i
// swapped for INV).
template <typename C, bool INV> __device__ __forceinline__ void dft7(C *v) {
  using S = decltype(C{}.x);
  const S c1 = S(0.6234898018587335305250048840042398106323);   // cos(2 pi / 7)
  const S c2 = S(-0.2225209339563144042889025644967947594664);  // cos(4 pi / 7)
  const S c3 = S(-0.9009688679024191262361023195074450511659);  // cos(6 pi / 7)
  const S s1 = S(0.7818314824680298087084445266740577502323);   // sin(2 pi / 7)
  const S s2 = S(0.9749279121818236070181316829939312172327);   // sin(4 pi / 7)
  const S s3 = S(0.4338837391175581204757683328483587546099);   // sin(6 pi / 7)
  const C x0 = v[0];
  const C t1 = cadd(v[1], v[6]), t2 = cadd(v[2], v[5]), t3 = cadd(v[3], v[4]);
  const C d1 = csub(v[1], v[6]), d2 = csub(v[2], v[5]), d3 = csub(v[3], v[4]);
  const C a1 = cadd(x0, cadd(cadd(cscale(t1, c1), cscale(t2, c2)), cscale(t3, c3)));
  const C a2 = cadd(x0, cadd(cadd(cscale(t1, c2), cscale(t2, c3)), cscale(t3, c1)));
  const C a3 = cadd(x0, cadd(cadd(cscale(t1, c3), cscale(t2, c1)), cscale(t3, c2)));
  const C b1 = cmul_mi<C, INV>(cadd(cadd(cscale(d1, s1), cscale(d2, s2)), cscale(d3, s3)));
  const C b2 = cmul_mi<C, INV>(csub(csub(cscale(d1, s2), cscale(d2, s3)), cscale(d3, s1)));
  const C b3 = cmul_mi<C, INV>(cadd(csub(cscale(d1, s3), cscale(d2, s1)), cscale(d3, s2)));
  v[0] = cadd(x0, cadd(cadd(t1, t2), t3));
  v[1] = cadd(a1, b1); v[6] = csub(a1, b1);
  v[2] = cadd(a2, b2); v[5] = csub(a2, b2);
  v[3] = cadd(a3, b3); v[4] = csub(a3, b3);
}

template <typename C, bool INV> __device__ __forceinline__ void dft8(C *v) {
  using S = decltype(C{}.x);
  const S r = S(0.7071067811865475244008443621048490392848);  // 1/sqrt(2)
  // even / odd 4-point transforms
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<C, INV>(e0, e1, e2, e3);
  dft4<C, INV>(o0, o1, o2, o3);
  // twiddles W8^k, k = 1, 2, 3 (conjugated for INV)
  C w1 = INV ? cmake<C>(r * (o1.x - o1.y), r * (o1.x + o1.y))
             : cmake<C>(r * (o1.x + o1.y), r * (o1.y - o1.x));
  C w2 = cmul_mi<C, INV>(o2);
  C w3 = INV ? cmake<C>(-r * (o3.x + o3.y), r * (o3.x - o3.y))
             : cmake<C>(r * (o3.y - o3.x), -r * (o3.x + o3.y));
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1); v[5] = csub(e1, w1);
  v[2] = cadd(e2, w2); v[6] = csub(e2, w2);
  v[3] = cadd(e3, w3); v[7] = csub(e3, w3);
}

template <typename C, int R, bool INV> __device__ __forceinline__ void dftR(C *v) {
  if constexpr (R == 2) dft2<C, INV>(v[0], v[1]);
  else if constexpr (R == 3) dft3<C, INV>(v[0], v[1], v[2]);
  else if constexpr (R == 4) dft4<C, INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 5) dft5<C, INV>(v);
  else if constexpr (R == 7) dft7<C, INV>(v);
  else dft8<C, INV>(v);
}

// ---------------------------------------------------------------------------
// One Stockham stage of radix R on P pencils of length n held in LDS
// (pencil p at lds[p * ld .. p * ld + n)).  Ns is the product of the radices
// already applied.  Each butterfly j reads x[j + r n/R], applies the twiddle
// W_{Ns R}^{r (j mod Ns)}, does an R-point DFT and writes the results to
// (j / Ns) Ns R + (j mod Ns) + r Ns.  All reads of the stage complete
// (barrier) before any write, so the stage runs in place.
// tw is the stage twiddle table (fill order of the host's stage_twiddles):
// W_{Ns R}^{r k} at (Ns - 1) + k (R - 1) + (r - 1), for every stage but the
// first, in LDS.
// ---------------------------------------------------------------------------
template <typename C, int R, bool INV, int THREADS, int PN>
__device__ __forceinline__ void stockham_stage(C *lds, int ld, int n, int P, int Ns, const C *tw) {
  constexpr int MAXB = (PN + R * THREADS - 1) / (R * THREADS);
  const int nbf = n / R;
  const int total = P * nbf;
  C v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = threadIdx.x + q * THREADS;
    if (b < total) {
      const int p = b / nbf;
      const int j = b - p * nbf;
      const int k = j % Ns;
      const C *src = lds + p * ld + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[r * nbf];
      if (Ns > 1) {
        const C *w = tw + (Ns - 1) + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = INV ? cmulc(v[q][r], w[r - 1]) : cmul(v[q][r], w[r - 1]);
      }
      dftR<C, R, INV>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = threadIdx.x + q * THREADS;
    if (b < total) {
      const int p = b / nbf;
      const int j = b - p * nbf;
      const int k = j % Ns;
      C *dst = lds + p * ld + (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

struct StageList {
  int nstage;
  int radix[12];
};

// Compile-time radix schedule of a length LEN = 2^a 3^b 5^c 7^d (same order
// as the host schedule: all factors 3, then 5s, then 7s, then 8s, then one 4
// and/or one 2).
constexpr int ct_radix(int len, int s) {
  int m = len, k = 0;
  while (m % 3 == 0) { if (k == s) return 3; m /= 3; ++k; }
  while (m % 5 == 0) { if (k == s) return 5; m /= 5; ++k; }
  while (m % 7 == 0) { if (k == s) return 7; m /= 7; ++k; }
  while (m % 8 == 0) { if (k == s) return 8; m /= 8; ++k; }
  if (m % 4 == 0) { if (k == s) return 4; m /= 4; ++k; }
  if (m % 2 == 0) { if (k == s) return 2; m /= 2; ++k; }
  return 0;
}
constexpr int ct_nstage(int len) {
  int s = 0;
  while (ct_radix(len, s) != 0) ++s;
  return s;
}

// Full transform of P pencils in LDS.  Caller synchronises before the call
// (data loaded) and may read results right after it returns.
template <typename C, bool INV, int THREADS, int PN>
__device__ void lds_fft(C *lds, int ld, int n, int P, const StageList &st, const C *tw) {
  int Ns = 1;
  for (int s = 0; s < st.nstage; ++s) {
    const int R = st.radix[s];
    if (R == 8) stockham_stage<C, 8, INV, THREADS, PN>(lds, ld, n, P, Ns, tw);
    else if (R == 4) stockham_stage<C, 4, INV, THREADS, PN>(lds, ld, n, P, Ns, tw);
    else if (R == 2) stockham_stage<C, 2, INV, THREADS, PN>(lds, ld, n, P, Ns, tw);
    else if (R == 5) stockham_stage<C, 5, INV, THREADS, PN>(lds, ld, n, P, Ns, tw);
    else if (R == 7) stockham_stage<C, 7, INV, THREADS, PN>(lds, ld, n, P, Ns, tw);
    else stockham_stage<C, 3, INV, THREADS, PN>(lds, ld, n, P, Ns, tw);
    Ns *= R;
  }
}

// ---------------------------------------------------------------------------
// Register-resident Stockham transform of P pencils of length LEN (radix
// schedule ct_radix).  Each stage keeps its butterflies' operands in
// registers; LDS is used only to exchange data between stages, with one pad
// slot per 8 elements and an odd pencil stride so that the strided stage
// writes and the pencil-strided accesses spread over the banks.  The first
// stage reads its operands straight from global memory through load(p, e)
// and the last stage writes its results through store(p, e, v), so a pass
// touches LDS 4 times per element for three stages.  With PFAST (first
// stage) / PFAST_OUT (last stage), consecutive threads take consecutive
// pencils (global rows strided by pencil, e.g. y and x passes over z
// columns); otherwise consecutive elements (contiguous rows).  load / store are called only for
// pencils p < npen.  twst is the stage twiddle table of fill_stage_twiddles.
// ---------------------------------------------------------------------------
__device__ __forceinline__ constexpr int fpad(int i) { return i + (i >> 3); }
template <int LEN> constexpr int fft_ld() { return LEN + LEN / 8 + 1; }

template <typename C, int LEN, int P, int NT, bool INV, bool PFAST, bool PFAST_OUT, int STAGE, int NS, class Load,
          class Store>
__device__ __forceinline__ void fft_stage(C *lds, const C *twst, int npen, Load &load, Store &store) {
  constexpr int S = ct_nstage(LEN);
  constexpr int R = ct_radix(LEN, STAGE);
  constexpr bool FIRST = STAGE == 0, LAST = STAGE == S - 1;
  constexpr int NBF = LEN / R;
  constexpr int TOT = P * NBF;
  constexpr int MAXB = (TOT + NT - 1) / NT;
  constexpr int LD = fft_ld<LEN>();
  constexpr bool PMAP = FIRST ? PFAST : (LAST ? PFAST_OUT : false);
  C v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = threadIdx.x + q * NT;
    if (b < TOT) {
      const int p = PMAP ? b % P : b / NBF;
      const int j = PMAP ? b / P : b % NBF;
      if constexpr (FIRST) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = p < npen ? load(p, j + r * NBF) : cmake<C>(0, 0);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = lds[p * LD + fpad(j + r * NBF)];
      }
      if constexpr (NS > 1) {
        const int k = j % NS;
        const C *w = twst + (NS - 1) + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = INV ? cmulc(v[q][r], w[r - 1]) : cmul(v[q][r], w[r - 1]);
      }
      dftR<C, R, INV>(v[q]);
    }
  }
  if constexpr (!FIRST) __syncthreads();  // every read of the stage precedes the in-place writes
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = threadIdx.x + q * NT;
    if (b < TOT) {
      const int p = PMAP ? b % P : b / NBF;
      const int j = PMAP ? b / P : b % NBF;
      if constexpr (LAST) {
        if (p < npen) {
#pragma unroll
          for (int r = 0; r < R; ++r) store(p, j + r * NS, v[q][r]);
        }
      } else {
        const int base = (j / NS) * NS * R + j % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[p * LD + fpad(base + r * NS)] = v[q][r];
      }
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
    fft_stage<C, LEN, P, NT, INV, PFAST, PFAST_OUT, STAGE + 1, NS * R>(lds, twst, npen, load, store);
  }
}

template <typename C, int LEN, int P, int NT, bool INV, bool PFAST, bool PFAST_OUT = PFAST, class Load, class Store>
__device__ __forceinline__ void fft_pencils(C *lds, const C *twst, int npen, Load &&load, Store &&store) {
  static_assert(ct_nstage(LEN) >= 2, "length too short");
  fft_stage<C, LEN, P, NT, INV, PFAST, PFAST_OUT, 0, 1>(lds, twst, npen, load, store);
}

// LDS bytes of fft_pencils: stage twiddles (LEN) + P padded pencils.
template <typename C, int LEN, int P> constexpr size_t fft_pencils_lds() {
  return sizeof(C) * ((size_t)LEN + (size_t)P * fft_ld<LEN>());
}

// Dynamic LDS one workgroup of the compiled-length transforms may take:
// P pencils are halved until P padded pencils and the twiddles fit.
constexpr size_t kFftLdsBudget = 100 * 1024;
template <typename C, int LEN, int P> constexpr int fit_pencils() {
  if constexpr (P > 1) {
    if (fft_pencils_lds<C, LEN, P>() > kFftLdsBudget) return fit_pencils<C, LEN, P / 2>();
  }
  return P;
}

// Pencil batching of the LDS transforms: P = pn / n pencils per workgroup.
// FP32 stages 8192 complex values with 512 threads so that the strided
// passes move rows of >= 16 consecutive complex values (>= 128 bytes).
template <typename T> struct FftTune {
  static constexpr int threads = sizeof(T) == 4 ? 512 : 256;
  static constexpr int pn = sizeof(T) == 4 ? 8192 : 4096;
};

// Lengths with a compile-time kernel; other 2^a 3^b 5^c 7^d lengths use the
// run-time one.  Forward mesh sides (multiples of 16) and the real-space
// grids of the triangle search.
#define FRSD_FFT_LENGTHS(X) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
#define FRSD_SHELL_LENGTHS(X) FRSD_FFT_LENGTHS(X) X(343) X(360)

}  // namespace frsd
