/*
 * Plain-C mass assignment for the FP64 oracle (test infrastructure only).
 *
 * mesh[i] = sum_j weight_j prod_d W_p(u_jd - i_d), periodic, with the
 * B-spline kernels of order p of Sec. III.A (the paragraph after eq.
 * Nelltrue): NGP on the half-open cell, CIC, TSC, PCS.  The same definition
 * as oracle.estimator.assign_mesh, written as a loop so that catalogues of
 * 10^7-10^8 objects stay tractable.  OpenMP threads take x-slabs of
 * objects in two colours so that no two threads ever write the same node.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double bspline(int p, double d) {
  const double a = fabs(d);
  switch (p) {
    case 1: return (d >= -0.5 && d < 0.5) ? 1.0 : 0.0;
    case 2: return a < 1.0 ? 1.0 - a : 0.0;
    case 3: return a < 0.5 ? 0.75 - a * a : (a < 1.5 ? 0.5 * (1.5 - a) * (1.5 - a) : 0.0);
    default:
      return a < 1.0 ? (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0
                     : (a < 2.0 ? (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0 : 0.0);
  }
}

static int64_t first_node(double u, int p) {
  if (p % 2 == 1) return (int64_t)floor(u + 0.5) - (p - 1) / 2;
  return (int64_t)floor(u) - (p / 2 - 1);
}

static void add_object(const double *u, double w, int N, int p, double *mesh) {
  int64_t i0[3];
  double wt[3][4];
  for (int d = 0; d < 3; ++d) {
    i0[d] = first_node(u[d], p);
    for (int a = 0; a < p; ++a) wt[d][a] = bspline(p, u[d] - (double)(i0[d] + a));
  }
  for (int a = 0; a < p; ++a) {
    const int64_t ix = ((i0[0] + a) % N + N) % N;
    for (int b = 0; b < p; ++b) {
      const int64_t iy = ((i0[1] + b) % N + N) % N;
      const double wab = w * wt[0][a] * wt[1][b];
      for (int c = 0; c < p; ++c) {
        const int64_t iz = ((i0[2] + c) % N + N) % N;
        mesh[(ix * N + iy) * N + iz] += wab * wt[2][c];
      }
    }
  }
}

/*
 * u: n x 3 grid coordinates, w: n weights, order: first-node x-slab order of
 * the objects (an argsort of floor(u_x)), slab_start: N + 1 offsets into
 * `order` per x-slab.  mesh: N^3 doubles, overwritten.
 */
void oracle_assign(const double *u, const double *w, const int64_t *order, const int64_t *slab_start, int64_t n,
                   int N, int p, double *mesh, int nthreads) {
  (void)n;
  memset(mesh, 0, sizeof(double) * (size_t)N * N * N);
  /* blocks of B slabs: objects in a block reach at most 2 slabs beyond it, so
     blocks of the same colour (every other block) never share a node when
     B >= 4 and there are at least 2 blocks of each colour */
  const int B = 8;
  const int nblk = (N + B - 1) / B;
  if (nblk < 4) {
    for (int64_t k = 0; k < slab_start[N]; ++k) add_object(u + 3 * order[k], w[order[k]], N, p, mesh);
    return;
  }
  /* with an odd block count the last block touches block 0 through the
     periodic seam: it is done alone after the two colours */
  const int ncol = (nblk % 2) ? nblk - 1 : nblk;
  for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int blk = colour; blk < ncol; blk += 2) {
      const int s0 = blk * B, s1 = (blk + 1) * B < N ? (blk + 1) * B : N;
      for (int64_t k = slab_start[s0]; k < slab_start[s1]; ++k)
        add_object(u + 3 * order[k], w[order[k]], N, p, mesh);
    }
  }
  for (int blk = ncol; blk < nblk; ++blk) {
    const int s0 = blk * B, s1 = (blk + 1) * B < N ? (blk + 1) * B : N;
    for (int64_t k = slab_start[s0]; k < slab_start[s1]; ++k) add_object(u + 3 * order[k], w[order[k]], N, p, mesh);
  }
}
