// Vector kernels of the restarted GMRES solver (double precision Arnoldi).
//
// The paper solves its symmetric Galerkin system by CG with one H-matrix
// product per step (Sec. 4.1); the collocation matrix is not symmetric, so
// its solve is GMRES with the same product.  Both are here.  All reductions
// write per-tile partial sums that a second kernel adds in a fixed order, so
// the solve is bitwise reproducible.
#include "hm_internal.h"

namespace hm {

namespace {
constexpr int kRowsPerTile = 2048;
constexpr int kGT = 256;
}

int gmres_tiles(int64_t n) { return (int)ceil_div(n, kRowsPerTile); }

// part[(k * tiles + tile) * nr + c] = sum over the tile's rows of
// Q[k][i][c] * w[i][c]   (Q: nk vectors of n*nr doubles, stride ldq)
__global__ __launch_bounds__(kGT) void k_dots(const double* __restrict__ Q, int64_t ldq,
                                              const double* __restrict__ w, int64_t n, int nr,
                                              int tiles, double* __restrict__ part) {
  __shared__ double lds[kGT];
  const int tile = blockIdx.x, k = blockIdx.y;
  const double* q = Q + (int64_t)k * ldq;
  const int per = kGT / nr;               // threads per column (nr <= 256)
  const int c = threadIdx.x % nr, r0 = threadIdx.x / nr;
  double acc = 0.0;
  if (r0 < per) {
    const int64_t beg = (int64_t)tile * kRowsPerTile;
    const int64_t end = min(beg + kRowsPerTile, n);
    for (int64_t i = beg + r0; i < end; i += per) acc += q[i * nr + c] * w[i * nr + c];
  }
  lds[threadIdx.x] = (r0 < per) ? acc : 0.0;
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    double s = 0.0;
    for (int t = 0; t < per; ++t) s += lds[t * nr + threadIdx.x];
    part[((int64_t)k * tiles + tile) * nr + threadIdx.x] = s;
  }
}

// out[k * nr + c] = sum_tile part[(k * tiles + tile) * nr + c]: one
// wavefront per output, lane l adding tiles l, l + 64, ... in order, then a
// fixed shuffle tree (the same order every call).
__device__ inline double tile_sum(const double* __restrict__ part, int k, int c, int tiles,
                                  int nr) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int t = lane; t < tiles; t += 64) s += part[((int64_t)k * tiles + t) * nr + c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  return s;
}
__global__ __launch_bounds__(256) void k_dots_final(const double* __restrict__ part, int nk,
                                                    int tiles, int nr,
                                                    double* __restrict__ out) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= nk * nr) return;                          // uniform over the wavefront
  const double s = tile_sum(part, e / nr, e % nr, tiles, nr);
  if ((threadIdx.x & 63) == 0) out[e] = s;
}

// w[i][c] -= sum_{k < nk} Q[k][i][c] h[k][c]   (h on the device)
__global__ void k_orth_update(const double* __restrict__ Q, int64_t ldq, const double* __restrict__ h,
                              int nk, int64_t n, int nr, double* __restrict__ w) {
  const int64_t tot = n * nr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % nr);
    double v = w[e];
    for (int k = 0; k < nk; ++k) v -= Q[(int64_t)k * ldq + e] * h[k * nr + c];
    w[e] = v;
  }
}

// x[i][c] += sum_{k < nk} Q[k][i][c] y[k][c]
__global__ void k_combine(const double* __restrict__ Q, int64_t ldq, const double* __restrict__ y,
                          int nk, int64_t n, int nr, double* __restrict__ x) {
  const int64_t tot = n * nr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % nr);
    double v = x[e];
    for (int k = 0; k < nk; ++k) v += Q[(int64_t)k * ldq + e] * y[k * nr + c];
    x[e] = v;
  }
}

// out[i][c] = a[i][c] * s[c]
__global__ void k_scale_cols(const double* __restrict__ a, const double* __restrict__ s, int64_t n,
                             int nr, double* __restrict__ out) {
  const int64_t tot = n * nr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = a[e] * s[e % nr];
}

// out = a + b
__global__ void k_add(const double* __restrict__ a, const double* __restrict__ b, int64_t tot,
                      double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = a[e] + b[e];
}

// out = a - b
__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b, int64_t tot,
                      double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = a[e] - b[e];
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ a, int64_t tot, D* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (D)a[e];
}

// Variants for graph replays: the Arnoldi step j is read from device memory
// (jd[0]); the grids cover the largest step, blocks past it return at once.
__global__ __launch_bounds__(kGT) void k_dots_dev(const double* __restrict__ Q, int64_t ldq,
                                                  const int* __restrict__ jd,
                                                  const double* __restrict__ w, int64_t n, int nr,
                                                  int tiles, double* __restrict__ part) {
  if ((int)blockIdx.y > jd[0]) return;               // uniform over the block
  __shared__ double lds[kGT];
  const int tile = blockIdx.x, k = blockIdx.y;
  const double* q = Q + (int64_t)k * ldq;
  const int per = kGT / nr;
  const int c = threadIdx.x % nr, r0 = threadIdx.x / nr;
  double acc = 0.0;
  if (r0 < per) {
    const int64_t beg = (int64_t)tile * kRowsPerTile;
    const int64_t end = min(beg + kRowsPerTile, n);
    for (int64_t i = beg + r0; i < end; i += per) acc += q[i * nr + c] * w[i * nr + c];
  }
  lds[threadIdx.x] = (r0 < per) ? acc : 0.0;
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    double s = 0.0;
    for (int t = 0; t < per; ++t) s += lds[t * nr + threadIdx.x];
    part[((int64_t)k * tiles + tile) * nr + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(256) void k_dots_final_dev(const double* __restrict__ part,
                                                        const int* __restrict__ jd, int nkmax,
                                                        int tiles, int nr,
                                                        double* __restrict__ out) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nk = jd[0] + 1;
  if (e >= nk * nr || e >= nkmax * nr) return;       // uniform over the wavefront
  const double s = tile_sum(part, e / nr, e % nr, tiles, nr);
  if ((threadIdx.x & 63) == 0) out[e] = s;
}

__global__ void k_orth_update_dev(const double* __restrict__ Q, int64_t ldq,
                                  const double* __restrict__ h, const int* __restrict__ jd,
                                  int64_t n, int nr, double* __restrict__ w) {
  const int nk = jd[0] + 1;
  const int64_t tot = n * nr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % nr);
    double v = w[e];
    for (int k = 0; k < nk; ++k) v -= Q[(int64_t)k * ldq + e] * h[k * nr + c];
    w[e] = v;
  }
}

// out = Q[jd[0]] (the Arnoldi vector of step j, into a fixed buffer)
__global__ void k_copy_col(const double* __restrict__ Q, int64_t ldq, const int* __restrict__ jd,
                           double* __restrict__ out) {
  const double* q = Q + (int64_t)jd[0] * ldq;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ldq;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = q[e];
}

// out = (float) Q[jd[0]]: the Arnoldi vector of step j rounded to single
// precision, the input of a product with float vectors
__global__ void k_copy_col_f32(const double* __restrict__ Q, int64_t ldq, const int* __restrict__ jd,
                               float* __restrict__ out) {
  const double* q = Q + (int64_t)jd[0] * ldq;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ldq;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (float)q[e];
}

// ---- conjugate gradients (Sec. 4.1), every column its own recurrence.
// alpha_c = rr[c] / pq[c] for active columns (0 for inactive ones and for
// pq = 0); x += alpha p, r -= alpha q.
__global__ void k_cg_update(double* __restrict__ x, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ q,
                            const double* __restrict__ rr, const double* __restrict__ pq,
                            const double* __restrict__ active, int64_t n, int nr) {
  const int64_t tot = n * nr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % nr);
    const double a = (active[c] != 0.0 && pq[c] != 0.0) ? rr[c] / pq[c] : 0.0;
    x[e] += a * p[e];
    r[e] -= a * q[e];
  }
}

// p = r + beta p with beta_c = rr_new[c] / rr_old[c], active columns only.
__global__ void k_cg_dir(double* __restrict__ p, const double* __restrict__ r,
                         const double* __restrict__ rr_new, const double* __restrict__ rr_old,
                         const double* __restrict__ active, int64_t n, int nr) {
  const int64_t tot = n * nr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % nr);
    if (active[c] != 0.0 && rr_old[c] != 0.0) p[e] = r[e] + (rr_new[c] / rr_old[c]) * p[e];
  }
}

// ------------------------------------------------------------------ launchers
void cg_update(double* x, double* r, const double* p, const double* q, const double* rr,
               const double* pq, const double* active, int64_t n, int nr, hipStream_t s) {
  k_cg_update<<<grid_for(n * nr, 256, 8192), 256, 0, s>>>(x, r, p, q, rr, pq, active, n, nr);
  HM_LAUNCH_CHECK();
}
void cg_dir(double* p, const double* r, const double* rr_new, const double* rr_old,
            const double* active, int64_t n, int nr, hipStream_t s) {
  k_cg_dir<<<grid_for(n * nr, 256, 8192), 256, 0, s>>>(p, r, rr_new, rr_old, active, n, nr);
  HM_LAUNCH_CHECK();
}
void gmres_dots_dev(const double* Q, int64_t ldq, const int* jd, int nkmax, const double* w,
                    int64_t n, int nr, double* part, double* out, hipStream_t s) {
  const int tiles = gmres_tiles(n);
  dim3 grid(tiles, nkmax);
  k_dots_dev<<<grid, kGT, 0, s>>>(Q, ldq, jd, w, n, nr, tiles, part);
  HM_LAUNCH_CHECK();
  k_dots_final_dev<<<(unsigned)ceil_div(nkmax * nr, 4), 256, 0, s>>>(part, jd, nkmax, tiles, nr,
                                                                      out);
  HM_LAUNCH_CHECK();
}
void gmres_orth_update_dev(const double* Q, int64_t ldq, const double* h, const int* jd,
                           int64_t n, int nr, double* w, hipStream_t s) {
  k_orth_update_dev<<<grid_for(n * nr, 256, 8192), 256, 0, s>>>(Q, ldq, h, jd, n, nr, w);
  HM_LAUNCH_CHECK();
}
void gmres_copy_col(const double* Q, int64_t ldq, const int* jd, double* out, hipStream_t s) {
  k_copy_col<<<grid_for(ldq, 256, 8192), 256, 0, s>>>(Q, ldq, jd, out);
  HM_LAUNCH_CHECK();
}
void gmres_copy_col_f32(const double* Q, int64_t ldq, const int* jd, float* out, hipStream_t s) {
  k_copy_col_f32<<<grid_for(ldq, 256, 8192), 256, 0, s>>>(Q, ldq, jd, out);
  HM_LAUNCH_CHECK();
}
void gmres_dots(const double* Q, int64_t ldq, int nk, const double* w, int64_t n, int nr,
                double* part, double* out, hipStream_t s) {
  const int tiles = gmres_tiles(n);
  dim3 grid(tiles, nk);
  k_dots<<<grid, kGT, 0, s>>>(Q, ldq, w, n, nr, tiles, part);
  HM_LAUNCH_CHECK();
  k_dots_final<<<(unsigned)ceil_div(nk * nr, 4), 256, 0, s>>>(part, nk, tiles, nr, out);
  HM_LAUNCH_CHECK();
}
void gmres_orth_update(const double* Q, int64_t ldq, const double* h, int nk, int64_t n, int nr,
                       double* w, hipStream_t s) {
  k_orth_update<<<grid_for(n * nr, 256, 8192), 256, 0, s>>>(Q, ldq, h, nk, n, nr, w);
  HM_LAUNCH_CHECK();
}
void gmres_combine(const double* Q, int64_t ldq, const double* y, int nk, int64_t n, int nr,
                   double* x, hipStream_t s) {
  k_combine<<<grid_for(n * nr, 256, 8192), 256, 0, s>>>(Q, ldq, y, nk, n, nr, x);
  HM_LAUNCH_CHECK();
}
void gmres_scale_cols(const double* a, const double* sc, int64_t n, int nr, double* out,
                      hipStream_t s) {
  k_scale_cols<<<grid_for(n * nr, 256, 8192), 256, 0, s>>>(a, sc, n, nr, out);
  HM_LAUNCH_CHECK();
}
void gmres_sub(const double* a, const double* b, int64_t tot, double* out, hipStream_t s) {
  k_sub<<<grid_for(tot, 256, 8192), 256, 0, s>>>(a, b, tot, out);
  HM_LAUNCH_CHECK();
}
void gmres_add(const double* a, const double* b, int64_t tot, double* out, hipStream_t s) {
  k_add<<<grid_for(tot, 256, 8192), 256, 0, s>>>(a, b, tot, out);
  HM_LAUNCH_CHECK();
}
void convert_f32_to_f64(const float* a, int64_t tot, double* out, hipStream_t s) {
  k_convert<float, double><<<grid_for(tot, 256, 8192), 256, 0, s>>>(a, tot, out);
  HM_LAUNCH_CHECK();
}
void convert_f64_to_f32(const double* a, int64_t tot, float* out, hipStream_t s) {
  k_convert<double, float><<<grid_for(tot, 256, 8192), 256, 0, s>>>(a, tot, out);
  HM_LAUNCH_CHECK();
}

}  // namespace hm
