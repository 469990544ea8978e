// Steps a1-a2: catalogue ingest, line of sight, counting sort by cell, and
// the FP64 scalar reductions I22, N_0, I33, W3 (Sec. III.A eqs. I22def,
// N0true; Sec. III.B eq. Noise0).
//
// Pass 1 (k_count) validates every object, finds its cell floor(x / h) and
// the half of the cell in z its fraction lies in, and takes a rank inside
// that half cell with an atomic increment of its count.  An exclusive scan
// of the counts gives each half cell's first slot; pass 2 (k_scatter)
// re-reads the catalogue and writes the object's record at offset + rank,
// so objects end up grouped by cell in row-major cell order (x slowest, z
// fastest), and inside a cell those with z fraction below 1/2 first (half
// cell 2 c_z, then 2 c_z + 1).  The offsets of cell c are offs[2 c] (first
// record) and offs[2 c + 2] (end); offs[2 c + 1] splits the halves.  The
// half is decided on the fraction as the record stores it (FP32 or FP64),
// so the assignment kernels see the same split.
//
// Every kernel here serves a batch of requests on plans of one shape (grid y
// = request): workspace pointers are request 0's and move by the request's
// workspace distance; catalogue arrays, sizes and alpha come per request.
#include "device.h"
#include "frsd_internal.h"

namespace frsd {

constexpr int kIngestThreads = 256;
constexpr int kScanChunk = 4096;   // elements per scan block (256 threads x 16)

__global__ void k_fill_i32(int *p, long long n, int v, Batch bt) {
  p = moved(p, bt.delta[blockIdx.y]);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_zero_u64(unsigned long long *p, Batch bt) { moved(p, bt.delta[blockIdx.y])[threadIdx.x] = 0ull; }

// The catalogues of one role (galaxies or randoms) of the requests of a
// batch, and each request's alpha.
struct CatArgs {
  const void *pos[kMaxBatch], *w[kMaxBatch], *nbar[kMaxBatch];
  long long n[kMaxBatch];
  long long off[kMaxBatch];  // first object slot (the randoms follow the galaxies)
};
struct Alphas {
  double v[kMaxBatch];
};

struct GeomArgs {
  double inv_h, L, ox, oy, oz;
  int N;
  int rec_f32;  // records hold FP32 fractions
};

constexpr double kOneMinus = 1.0 - 1e-15;  // largest fraction kept in a cell

// Fraction of u in cell c, clamped to [0, 1).
__device__ __forceinline__ double cell_fraction(double u, int c) {
  const double f = u - c;
  return f < 0 ? 0 : (f > kOneMinus ? kOneMinus : f);
}

// Cell of an in-box position; u = x / h rounded up to N near the upper edge
// is folded back into the last cell.
__device__ __forceinline__ int cell_coord(double u, int N) {
  int c = (int)floor(u);
  return c < 0 ? 0 : (c > N - 1 ? N - 1 : c);
}

template <typename TIN>
__device__ __forceinline__ bool load_pos(const TIN *pos, long long i, const GeomArgs &g, double &x,
                                         double &y, double &z) {
  x = (double)pos[3 * i];
  y = (double)pos[3 * i + 1];
  z = (double)pos[3 * i + 2];
  const bool inbox = (x >= 0.0) && (x < g.L) && (y >= 0.0) && (y < g.L) && (z >= 0.0) && (z < g.L);
  const double rx = x - g.ox, ry = y - g.oy, rz = z - g.oz;
  return inbox && (rx * rx + ry * ry + rz * rz > 0.0);
}

// Block sum of up to four doubles into part[col * nblk + blockIdx.x].
__device__ void block_sum4(double v0, double v1, double v2, double v3, double *part, int col0, int ncol) {
  __shared__ double red[4][kIngestThreads / 64];
  v0 = wave_sum(v0); v1 = wave_sum(v1); v2 = wave_sum(v2); v3 = wave_sum(v3);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) { red[0][w] = v0; red[1][w] = v1; red[2][w] = v2; red[3][w] = v3; }
  __syncthreads();
  if (threadIdx.x < ncol) {
    double s = 0;
    for (int k = 0; k < kIngestThreads / 64; ++k) s += red[threadIdx.x][k];
    part[(col0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
}

// Pass 1.  Galaxies write partial columns 0,1 (sum w^2, sum w^3); randoms
// write columns 2..5 (sum nbar w^2, sum nbar^2 w^3, sum w^2, sum w^3).
// dyn (graph replays, may be null): {N_g, N_r, alpha} in device memory,
// which then replace the launch's n and offset (and alpha below).
__device__ __forceinline__ void dyn_sizes(const double *dyn, int is_ran, long long &n, long long &obj_off) {
  if (dyn) {
    n = (long long)dyn[is_ran ? 1 : 0];
    obj_off = is_ran ? (long long)dyn[0] : 0;
  }
}

template <typename TIN>
__global__ __launch_bounds__(kIngestThreads) void k_count(CatArgs c, int is_ran, GeomArgs g, int *cnt, int *slot,
                                                           int *cellkey, double *part,
                                                           unsigned long long *reject, const double *dyn,
                                                           Batch bt) {
  const int r = blockIdx.y;
  const long long dr = bt.delta[r];
  cnt = moved(cnt, dr);
  slot = moved(slot, dr);
  cellkey = moved(cellkey, dr);
  part = moved(part, dr);
  reject = moved(reject, dr);
  dyn = shifted(dyn, dr);
  const TIN *pos = static_cast<const TIN *>(c.pos[r]), *w = static_cast<const TIN *>(c.w[r]),
            *nbar = static_cast<const TIN *>(c.nbar[r]);
  long long n = c.n[r], obj_off = c.off[r];
  dyn_sizes(dyn, is_ran, n, obj_off);
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double x, y, z;
    const bool ok = load_pos(pos, i, g, x, y, z);
    if (ok) {
      const double uz = z * g.inv_h;
      const int cx = cell_coord(x * g.inv_h, g.N), cy = cell_coord(y * g.inv_h, g.N), cz = cell_coord(uz, g.N);
      const double fz = cell_fraction(uz, cz);
      const int hz = g.rec_f32 ? ((float)fz >= 0.5f) : (fz >= 0.5);
      const int cell = 2 * ((cx * g.N + cy) * g.N + cz) + hz;  // half-cell key, < 2 N^3 <= 2^31
      slot[obj_off + i] = atomicAdd(&cnt[cell], 1);
      cellkey[obj_off + i] = cell;
      const double wi = (double)w[i];
      const double w2 = wi * wi, w3 = w2 * wi;
      if (is_ran) {
        const double nb = (double)nbar[i];
        s0 += nb * w2; s1 += nb * nb * w3; s2 += w2; s3 += w3;
      } else {
        s0 += w2; s1 += w3;
      }
    } else {
      cellkey[obj_off + i] = -1;
      atomicAdd(reject, 1ull);
    }
  }
  if (is_ran) block_sum4(s0, s1, s2, s3, part, 2, 4);
  else block_sum4(s0, s1, 0.0, 0.0, part, 0, 2);
}

// Pass 2: write the record of each accepted object at its sorted slot.
template <typename TIN, typename T>
__global__ __launch_bounds__(kIngestThreads) void k_scatter(CatArgs c, int is_ran, Alphas al, GeomArgs g,
                                                             const int *offs, const int *slot, const int *cellkey,
                                                             Rec4<T> *rec, const double *dyn, Batch bt) {
  const int r = blockIdx.y;
  const long long dr = bt.delta[r];
  offs = moved(offs, dr);
  slot = moved(slot, dr);
  cellkey = moved(cellkey, dr);
  rec = moved(rec, dr);
  dyn = shifted(dyn, dr);
  const TIN *pos = static_cast<const TIN *>(c.pos[r]), *w = static_cast<const TIN *>(c.w[r]);
  long long n = c.n[r], obj_off = c.off[r];
  double alpha = al.v[r];
  dyn_sizes(dyn, is_ran, n, obj_off);
  if (dyn) alpha = dyn[2];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int cell = cellkey[obj_off + i];
    if (cell < 0) continue;
    const long long dst = (long long)offs[cell] + slot[obj_off + i];
    const double ux = (double)pos[3 * i] * g.inv_h, uy = (double)pos[3 * i + 1] * g.inv_h,
                 uz = (double)pos[3 * i + 2] * g.inv_h;
    const int cx = cell_coord(ux, g.N), cy = cell_coord(uy, g.N), cz = cell_coord(uz, g.N);
    const double f0 = cell_fraction(ux, cx), f1 = cell_fraction(uy, cy), f2 = cell_fraction(uz, cz);
    const double wi = (double)w[i];
    Rec4<T> r;
    r.x = (T)f0; r.y = (T)f1; r.z = (T)f2;
    r.w = (T)(is_ran ? -alpha * wi : wi);
    rec[dst] = r;
  }
}

// I22 = alpha S_r[nbar w^2], N0 = S_g[w^2] + alpha^2 S_r[w^2],
// I33 = alpha S_r[nbar^2 w^3], W3 = S_g[w^3] - alpha^3 S_r[w^3].
// One wavefront per partial column (6 columns, 384 threads), then the
// scalars.
__global__ __launch_bounds__(384) void k_scal_final(const double *part, int nblk, Alphas al, double *scal,
                                                    const double *dyn, Batch bt) {
  const long long dr = bt.delta[blockIdx.x];
  part = moved(part, dr);
  scal = moved(scal, dr);
  dyn = shifted(dyn, dr);
  double alpha = al.v[blockIdx.x];
  if (dyn) alpha = dyn[2];
  __shared__ double col[6];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double s = 0;
  for (int b = lane; b < nblk; b += 64) s += part[w * nblk + b];
  s = wave_sum(s);
  if (lane == 0) col[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    scal[0] = alpha * col[2];
    scal[1] = col[0] + alpha * alpha * col[4];
    scal[2] = alpha * col[3];
    scal[3] = col[1] - alpha * alpha * alpha * col[5];
    for (int k = 0; k < 6; ++k) scal[4 + k] = col[k];
  }
}

// Random cache: keep the randoms' raw sums (columns 2-5: nbar w^2, nbar^2 w^3,
// w^2, w^3) at cache time; for a cached assignment, fold them with the
// galaxies' sums (columns 0-1) into I22, N_0, I33, W3 for this alpha.
__global__ void k_scal_keep(const double *scal, double *keep) {
  if (threadIdx.x < 4) keep[threadIdx.x] = scal[6 + threadIdx.x];
}
// one workgroup per request of the batch
__global__ void k_scal_cached(const double *keep, Alphas al, double *scal, Batch bt) {
  if (threadIdx.x != 0) return;
  keep = moved(keep, bt.delta[blockIdx.x]);
  scal = moved(scal, bt.delta[blockIdx.x]);
  const double alpha = al.v[blockIdx.x];
  const double g0 = scal[4], g1 = scal[5];
  scal[0] = alpha * keep[0];
  scal[1] = g0 + alpha * alpha * keep[2];
  scal[2] = alpha * keep[1];
  scal[3] = g1 - alpha * alpha * alpha * keep[3];
  for (int k = 0; k < 4; ++k) scal[6 + k] = keep[k];
}

void scal_keep(frsd_plan *pl, void *ws, hipStream_t s) {
  FRSD_TIMED("scalars", s, hipLaunchKernelGGL(k_scal_keep, dim3(1), dim3(64), 0, s, ws_ptr<const double>(ws, pl->L.scal),
                                              ws_ptr<double>(ws, pl->L.rcache_sums)));
}
void scal_cached_batch(frsd_plan *pl, void *const *wss, int nreq, const double *alpha, hipStream_t s) {
  Alphas al{};
  for (int r = 0; r < nreq; ++r) al.v[r] = alpha[r];
  FRSD_TIMED("scalars", s, hipLaunchKernelGGL(k_scal_cached, dim3(nreq), dim3(64), 0, s,
                                              ws_ptr<const double>(wss[0], pl->L.rcache_sums), al,
                                              ws_ptr<double>(wss[0], pl->L.scal), batch_of(wss, nreq)));
}
void scal_cached(frsd_plan *pl, void *ws, double alpha, hipStream_t s) { scal_cached_batch(pl, &ws, 1, &alpha, s); }

// ---------------------------------------------------------------------------
// Exclusive scan of int32 counts, in place (three kernels).
// ---------------------------------------------------------------------------
// Four consecutive counts from index i (16-byte aligned), zero past n.
__device__ __forceinline__ int4 load4(const int *a, long long i, long long n) {
  if (i + 3 < n) return *reinterpret_cast<const int4 *>(a + i);
  int4 v = make_int4(0, 0, 0, 0);
  if (i < n) v.x = a[i];
  if (i + 1 < n) v.y = a[i + 1];
  if (i + 2 < n) v.z = a[i + 2];
  return v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const int *a, long long n, int *blk, Batch bt) {
  a = moved(a, bt.delta[blockIdx.y]);
  blk = moved(blk, bt.delta[blockIdx.y]);
  const long long base = (long long)blockIdx.x * kScanChunk;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanChunk / 1024; ++k) {
    const int4 v = load4(a, base + 4 * (k * 256 + (int)threadIdx.x), n);
    s += v.x + v.y + v.z + v.w;
  }
  __shared__ int red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) blk[blockIdx.x] = red[0];
}

// Exclusive scan of the 256 per-thread values v of a block (wavefront
// shuffles, then the 4 wavefront totals); returns the exclusive prefix and
// the block total.
__device__ __forceinline__ int block_exscan256_fast(int v, int *wtot, int &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  int pre = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int t = wtot[k];
    pre += k < w ? t : 0;
    total += t;
  }
  __syncthreads();
  return pre + incl - v;
}

// Block partials: thread t owns a contiguous run of them.
__global__ __launch_bounds__(256) void k_scan_top(int *blk, int nb, Batch bt) {
  blk = moved(blk, bt.delta[blockIdx.x]);
  __shared__ int wtot[4];
  const int per = (nb + 255) / 256;
  const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += blk[i];
  int total;
  int run = block_exscan256_fast(s, wtot, total);
  for (int i = b0; i < b1; ++i) {
    const int v = blk[i];
    blk[i] = run;
    run += v;
  }
}

// One chunk of 4096 counts per block: read and written as 16-byte vectors
// through LDS (one pad word per 16 so that each thread's 16 consecutive
// counts sit in distinct banks), scanned per thread and per block.
__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 4); }

__global__ __launch_bounds__(256) void k_scan_down(int *a, long long n, const int *blk, Batch bt) {
  a = moved(a, bt.delta[blockIdx.y]);
  blk = moved(blk, bt.delta[blockIdx.y]);
  __shared__ int buf[kScanChunk + kScanChunk / 16];
  __shared__ int wtot[4];
  const long long base = (long long)blockIdx.x * kScanChunk;
#pragma unroll
  for (int k = 0; k < kScanChunk / 1024; ++k) {
    const int e = 4 * (k * 256 + (int)threadIdx.x);
    const int4 v = load4(a, base + e, n);
    buf[scan_pad(e)] = v.x;
    buf[scan_pad(e + 1)] = v.y;
    buf[scan_pad(e + 2)] = v.z;
    buf[scan_pad(e + 3)] = v.w;
  }
  __syncthreads();
  int v[16];
  int s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = buf[scan_pad(threadIdx.x * 16 + k)];
    s += v[k];
  }
  int total;
  int run = block_exscan256_fast(s, wtot, total) + blk[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    buf[scan_pad(threadIdx.x * 16 + k)] = run;
    run += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanChunk / 1024; ++k) {
    const int e = 4 * (k * 256 + (int)threadIdx.x);
    const long long i = base + e;
    const int4 v = make_int4(buf[scan_pad(e)], buf[scan_pad(e + 1)], buf[scan_pad(e + 2)], buf[scan_pad(e + 3)]);
    if (i + 3 < n) {
      *reinterpret_cast<int4 *>(a + i) = v;
    } else {
      if (i < n) a[i] = v.x;
      if (i + 1 < n) a[i + 1] = v.y;
      if (i + 2 < n) a[i + 2] = v.z;
    }
  }
}

// ---------------------------------------------------------------------------
// Catalogues of role k (0 galaxies, 1 randoms) of every request: one dtype
// per launch.  Empty catalogues take any dtype.
static bool role_dtype(const frsd_catalog *const *cat, int nreq, int *dtype) {
  *dtype = FRSD_F64;
  bool seen = false;
  for (int r = 0; r < nreq; ++r) {
    if (cat[r]->n == 0) continue;
    if (seen && cat[r]->dtype != *dtype) return false;
    *dtype = cat[r]->dtype;
    seen = true;
  }
  return true;
}

template <typename T>
static int ingest_launches(frsd_plan *pl, void *const *wss, int nreq, const frsd_catalog *const *gal,
                           const frsd_catalog *const *ran, const double *alpha, hipStream_t s, const double *dyn,
                           int dt_gal, int dt_ran) {
  const Layout &L = pl->L;
  void *ws = wss[0];
  const Batch bt = batch_of(wss, nreq);
  const int N = pl->N;
  const long long ncell = 2LL * N * N * N;  // half cells
  const GeomArgs g{1.0 / pl->h, pl->p.box, pl->p.observer[0], pl->p.observer[1], pl->p.observer[2], N,
                   sizeof(T) == 4 ? 1 : 0};
  CatArgs cat[2] = {};
  Alphas al{};
  for (int r = 0; r < nreq; ++r) {
    const frsd_catalog *c2[2] = {gal[r], ran[r]};
    for (int k = 0; k < 2; ++k) {
      cat[k].pos[r] = c2[k]->pos;
      cat[k].w[r] = c2[k]->w;
      cat[k].nbar[r] = c2[k]->nbar;
      cat[k].n[r] = c2[k]->n;
      cat[k].off[r] = k == 0 ? 0 : gal[r]->n;
    }
    al.v[r] = alpha[r];
  }
  const int dts[2] = {dt_gal, dt_ran};
  const unsigned nr = (unsigned)nreq;

  FRSD_TIMED("fill", s, hipLaunchKernelGGL(k_fill_i32, dim3(2048, nr), dim3(256), 0, s, ws_ptr<int>(ws, L.cnt),
                                           ncell + 1, 0, bt));
  FRSD_TIMED("fill", s, hipLaunchKernelGGL(k_zero_u64, dim3(1, nr), dim3(1), 0, s,
                                           ws_ptr<unsigned long long>(ws, L.reject), bt));
  for (int k = 0; k < 2; ++k) {
    auto kern = dts[k] == FRSD_F64 ? (void (*)(CatArgs, int, GeomArgs, int *, int *, int *, double *,
                                              unsigned long long *, const double *, Batch))k_count<double>
                                   : k_count<float>;
    FRSD_TIMED("count", s, hipLaunchKernelGGL(kern, dim3(kIngestBlocks, nr), dim3(kIngestThreads), 0, s, cat[k], k,
                                              g, ws_ptr<int>(ws, L.cnt), ws_ptr<int>(ws, L.slot),
                                              ws_ptr<int>(ws, L.cellkey), ws_ptr<double>(ws, L.scal_part),
                                              ws_ptr<unsigned long long>(ws, L.reject), dyn, bt));
  }
  FRSD_LAUNCH_CHECK();
  const long long n = ncell + 1;
  const int nb = (int)((n + kScanChunk - 1) / kScanChunk);
  FRSD_TIMED("scan", s, hipLaunchKernelGGL(k_scan_reduce, dim3(nb, nr), dim3(256), 0, s, ws_ptr<int>(ws, L.cnt), n,
                                           ws_ptr<int>(ws, L.scan_blk), bt));
  FRSD_TIMED("scan", s, hipLaunchKernelGGL(k_scan_top, dim3(nr), dim3(256), 0, s, ws_ptr<int>(ws, L.scan_blk), nb, bt));
  FRSD_TIMED("scan", s, hipLaunchKernelGGL(k_scan_down, dim3(nb, nr), dim3(256), 0, s, ws_ptr<int>(ws, L.cnt), n,
                                           ws_ptr<int>(ws, L.scan_blk), bt));
  for (int k = 0; k < 2; ++k) {
    auto kern = dts[k] == FRSD_F64 ? (void (*)(CatArgs, int, Alphas, GeomArgs, const int *, const int *,
                                              const int *, Rec4<T> *, const double *, Batch))k_scatter<double, T>
                                   : k_scatter<float, T>;
    FRSD_TIMED("scatter", s, hipLaunchKernelGGL(kern, dim3(kIngestBlocks, nr), dim3(kIngestThreads), 0, s, cat[k], k,
                                                al, g, ws_ptr<int>(ws, L.cnt), ws_ptr<int>(ws, L.slot),
                                                ws_ptr<int>(ws, L.cellkey), ws_ptr<Rec4<T>>(ws, L.sorted), dyn, bt));
  }
  FRSD_TIMED("scalars", s, hipLaunchKernelGGL(k_scal_final, dim3(nr), dim3(384), 0, s,
                                              ws_ptr<double>(ws, L.scal_part), kIngestBlocks, al,
                                              ws_ptr<double>(ws, L.scal), dyn, bt));
  FRSD_LAUNCH_CHECK();
  return FRSD_OK;
}

// Steps a1-a2 for the requests of a batch (ran null: no randoms); requests
// whose catalogues of one role differ in dtype go one at a time.  dyn (may
// be null): request 0's {N_g, N_r, alpha}, each request's in its workspace.
template <typename T>
int ingest_and_sort_batch(frsd_plan *pl, void *const *wss, int nreq, const frsd_catalog *gal,
                          const frsd_catalog *ran, const double *alpha, hipStream_t s, const double *dyn) {
  const frsd_catalog none{nullptr, nullptr, nullptr, 0, FRSD_F64};
  const frsd_catalog *gp[kMaxBatch], *rp[kMaxBatch];
  for (int r = 0; r < nreq; ++r) {
    gp[r] = &gal[r];
    rp[r] = ran ? &ran[r] : &none;
  }
  int dg, dr;
  if (role_dtype(gp, nreq, &dg) && role_dtype(rp, nreq, &dr))
    return ingest_launches<T>(pl, wss, nreq, gp, rp, alpha, s, dyn, dg, dr);
  for (int r = 0; r < nreq; ++r) {
    const int dgr = gp[r]->n ? gp[r]->dtype : FRSD_F64, drr = rp[r]->n ? rp[r]->dtype : FRSD_F64;
    const double *dyn_r = dyn ? ws_ptr<const double>(wss[r], pl->L.dyn) : nullptr;
    const int rc = ingest_launches<T>(pl, &wss[r], 1, &gp[r], &rp[r], &alpha[r], s, dyn_r, dgr, drr);
    if (rc) return rc;
  }
  return FRSD_OK;
}

template <typename T>
int ingest_and_sort(frsd_plan *pl, void *ws, const frsd_catalog *gal, const frsd_catalog *ran, double alpha,
                    hipStream_t s, const double *dyn) {
  const int dg = gal->n ? gal->dtype : FRSD_F64, dr = ran->n ? ran->dtype : FRSD_F64;
  return ingest_launches<T>(pl, &ws, 1, &gal, &ran, &alpha, s, dyn, dg, dr);
}

template int ingest_and_sort<float>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                    hipStream_t, const double *);
template int ingest_and_sort<double>(frsd_plan *, void *, const frsd_catalog *, const frsd_catalog *, double,
                                     hipStream_t, const double *);
template int ingest_and_sort_batch<float>(frsd_plan *, void *const *, int, const frsd_catalog *,
                                          const frsd_catalog *, const double *, hipStream_t, const double *);
template int ingest_and_sort_batch<double>(frsd_plan *, void *const *, int, const frsd_catalog *,
                                           const frsd_catalog *, const double *, hipStream_t, const double *);

}  // namespace frsd
