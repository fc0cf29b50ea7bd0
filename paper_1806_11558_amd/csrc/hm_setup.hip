// H-matrix setup kernels: entry evaluation, near-field assembly, batched
// adaptive cross approximation, packing of the factors into leaf slices, and
// the per-leaf item lists used by the matrix-vector products.
//
// Storage layout (device, Morton order):
//   Every stored block is cut along the leaf clusters of its row cluster
//   ("row slices") -- dense blocks and the U factors -- or of its column
//   cluster ("column slices") -- the V factors.  A slice is column-major with
//   leading dimension ld = size of its leaf rounded up to 4 (padding rows are
//   zero), so one leaf's share of a block is one contiguous run of memory.
//   A leaf cluster then streams its dense blocks and its U slices in the
//   product y = H x (Sec. 2.3, last paragraph), and its V slices in the
//   first phase t = V^T x.
#include <cmath>

#include "hm_internal.h"

namespace hm {

// ------------------------------------------------------------------ entries
template <typename T>
struct Src {
  double cx, cy, cz;
  T ox[kNQ], oy[kNQ], oz[kNQ];
  T aw, sf;
};

template <typename T>
__device__ inline void load_src(const Geom<T>& g, int j, Src<T>& s) {
  s.cx = g.c[j];
  s.cy = g.c[g.n + j];
  s.cz = g.c[2 * g.n + j];
#pragma unroll
  for (int q = 0; q < kNQ; ++q) {
    s.ox[q] = g.o[(int64_t)q * g.n + j];
    s.oy[q] = g.o[(int64_t)(kNQ + q) * g.n + j];
    s.oz[q] = g.o[(int64_t)(2 * kNQ + q) * g.n + j];
  }
  s.aw = g.aw[j];
  s.sf = g.sf[j];
}

__device__ inline float rsq(float x) { return rsqrtf(x); }
__device__ inline double rsq(double x) { return 1.0 / sqrt(x); }

// a(i, j) = |T_j|/(4 pi) sum_q w_q / |x_i - y_jq| for i != j (seven-point
// Radon rule on the single-layer kernel of Sec. 2.1), the analytic self-term
// for i == j.  Positions i, j are Morton positions; (xi, yi, zi) = x_i.
template <typename T>
__device__ inline T eval_entry(double xi, double yi, double zi, int i, const Src<T>& s, int j) {
  if (i == j) return s.sf;
  const T dx = (T)(xi - s.cx), dy = (T)(yi - s.cy), dz = (T)(zi - s.cz);
  T acc[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < kNQ; ++q) {
    const T ex = dx - s.ox[q], ey = dy - s.oy[q], ez = dz - s.oz[q];
    const T r = rsq(ex * ex + ey * ey + ez * ez);
    acc[q == 0 ? 0 : (q <= 3 ? 1 : 2)] += r;
  }
  const T w =
      (T)Radon7::w0 * acc[0] + (T)Radon7::w1 * acc[1] + (T)Radon7::w2 * acc[2];
  return w * s.aw;
}

template <typename T>
__device__ inline T entry_at(const Geom<T>& g, int i, int j) {
  Src<T> s;
  load_src(g, j, s);
  return eval_entry(g.c[i], g.c[g.n + i], g.c[2 * g.n + i], i, s, j);
}

// Entries at arbitrary (application) index pairs, for checking.
template <typename T>
__global__ void k_entries(Geom<T> g, const int32_t* __restrict__ inv_perm,
                          const int32_t* __restrict__ rows, const int32_t* __restrict__ cols,
                          int64_t cnt, double* __restrict__ out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < cnt;
       k += (int64_t)gridDim.x * blockDim.x)
    out[k] = (double)entry_at(g, inv_perm[rows[k]], inv_perm[cols[k]]);
}

__global__ void k_inverse_perm(const int32_t* __restrict__ perm, int64_t n,
                               int32_t* __restrict__ inv) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    inv[perm[p]] = (int32_t)p;
}

// ------------------------------------------------------------------ near field
// Dense leaves of Algorithm 1, assembled in one batch (Sec. 3.3): one
// workgroup per block, entries written straight into the block's row slices.
struct LeafTab {
  const int32_t* lo;     // first position of leaf
  const int32_t* m;      // size
  const int64_t* ldpre;  // prefix of ld over leaves (nleaf + 1 entries)
  const int2* cl_leaves; // per cluster: first and last leaf
};

__device__ inline int leaf_ld(const LeafTab& L, int lf) {
  return (int)(L.ldpre[lf + 1] - L.ldpre[lf]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_near(Geom<T> g, const int2* __restrict__ dns, int64_t nd,
                                              const Cluster* __restrict__ cl, LeafTab L,
                                              const int64_t* __restrict__ doff, T* __restrict__ D) {
  for (int64_t b = blockIdx.x; b < nd; b += gridDim.x) {
    const int2 ts = dns[b];
    const Cluster tau = cl[ts.x], sig = cl[ts.y];
    const int n = sig.y - sig.x;
    const int2 lv = L.cl_leaves[ts.x];
    const int64_t base0 = doff[b];
    for (int lf = lv.x; lf <= lv.y; ++lf) {
      const int ld = leaf_ld(L, lf), m = L.m[lf], lo = L.lo[lf];
      T* dst = D + base0 + (int64_t)n * (L.ldpre[lf] - L.ldpre[lv.x]);
      for (int e = threadIdx.x; e < ld * n; e += blockDim.x) {
        const int i = e % ld, j = e / ld;
        T v = 0;
        if (i < m) v = entry_at(g, lo + i, sig.x + j);
        dst[e] = v;
      }
    }
    (void)tau;
  }
}

// ------------------------------------------------------------------ ACA
// Reductions over a wavefront.  argmax keys: larger key wins, ties go to the
// smaller index; the signed value travels with its key.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <typename T>
struct ArgMax {
  T key;
  int idx;
  T val;
};

template <typename T>
__device__ inline void argmax_merge(ArgMax<T>& a, const ArgMax<T>& b) {
  if (b.key > a.key || (b.key == a.key && b.idx < a.idx)) a = b;
}

// The result is taken from lane 0 so that every lane holds the same value
// even when a key is NaN (NaN keys never win a comparison).
template <typename T>
__device__ inline ArgMax<T> wave_argmax(ArgMax<T> a) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    ArgMax<T> b;
    b.key = __shfl_xor(a.key, d, 64);
    b.idx = __shfl_xor(a.idx, d, 64);
    b.val = __shfl_xor(a.val, d, 64);
    argmax_merge(a, b);
  }
  a.key = __shfl(a.key, 0, 64);
  a.idx = __shfl(a.idx, 0, 64);
  a.val = __shfl(a.val, 0, 64);
  return a;
}

template <typename T>
struct AcaArgs {
  Geom<T> g;
  const int2* blk;       // (tau, sigma) of the chunk's blocks
  const Cluster* cl;
  const int64_t* slot;   // element offset of every block's working slot in pool
  int64_t slot0;         // slot offset of the chunk's first block (pool[0])
  T* pool;
  const int32_t* big;    // blocks handled by a whole workgroup
  int64_t nbig;
  const int32_t* small;  // blocks handled by one wavefront each (m, n <= 64)
  int64_t nsmall;
  int kmax;
  double eps;
  int32_t* rank;         // out: rank per block
  int32_t* info;         // out: bit 0 cap hit, bits 1.. number of row evaluations
};

// Stop test shared by both variants: keep term r, then stop when
// |u_r||v_r| <= eps |S_r|_F, or r reached the cap, or every row was used.
__device__ inline bool aca_stop(double uu, double vv, double s2, double eps) {
  return sqrt(uu) * sqrt(vv) <= eps * sqrt(fmax(s2, 0.0));
}

// One block per wavefront; lane k owns row k and column k (m, n <= 64).
// The working factors live in the block's slot: U column-major m x kcap,
// then V n x kcap.  Every lane only touches its own row / column of them;
// values of other lanes arrive by shuffles.
template <typename T>
__device__ void aca_wave(const AcaArgs<T>& A, int b) {
  const int lane = threadIdx.x & 63;
  const int2 ts = A.blk[b];
  const Cluster tau = A.cl[ts.x], sig = A.cl[ts.y];
  const int r0 = tau.x, m = tau.y - tau.x, c0 = sig.x, n = sig.y - sig.x;
  const int kcap = min(A.kmax, min(m, n));
  T* U = A.pool + (A.slot[b] - A.slot0);
  T* V = U + (int64_t)kcap * m;
  const Geom<T>& g = A.g;
  const bool has_row = lane < m, has_col = lane < n;

  Src<T> my_src;
  if (has_col) load_src(g, c0 + lane, my_src);
  double my_x = 0, my_y = 0, my_z = 0;
  if (has_row) {
    my_x = g.c[r0 + lane];
    my_y = g.c[g.n + r0 + lane];
    my_z = g.c[2 * g.n + r0 + lane];
  }
  bool used = false;
  int nused = 0, r = 0, istar = 0, rows_eval = 0;
  double s2 = 0.0;
  bool cap_hit = false;
  while (true) {
    // residual row v~ = a(i*, :) - sum_l u_l[i*] v_l
    const double xi = __shfl(my_x, istar, 64), yi = __shfl(my_y, istar, 64),
                 zi = __shfl(my_z, istar, 64);
    T val = 0;
    if (has_col) val = eval_entry(xi, yi, zi, r0 + istar, my_src, c0 + lane);
    for (int l = 0; l < r; ++l) {
      const T ul = has_row ? U[(int64_t)l * m + lane] : (T)0;
      const T ui = __shfl(ul, istar, 64);
      if (has_col) val -= ui * V[(int64_t)l * n + lane];
    }
    ++rows_eval;
    if (lane == istar) used = true;
    ++nused;
    ArgMax<T> am{has_col ? (T)fabs(val) : (T)-1, has_col ? lane : 1 << 30, has_col ? val : (T)0};
    am = wave_argmax(am);
    if (am.val == (T)0 || am.idx < 0 || am.idx >= n) {
      if (nused >= m) break;
      ArgMax<T> nx{(T)-1, 1 << 30, (T)0};
      if (has_row && !used) {
        nx.key = (r > 0) ? (T)fabs(U[(int64_t)(r - 1) * m + lane]) : (T)0;
        nx.idx = lane;
      }
      istar = wave_argmax(nx).idx;
      if (istar < 0 || istar >= m) break;
      continue;
    }
    const int jstar = am.idx;
    const T v = has_col ? val / am.val : (T)0;
    if (has_col) V[(int64_t)r * n + lane] = v;
    // residual column u = a(:, j*) - sum_l v_l[j*] u_l
    Src<T> s;
    load_src(g, c0 + jstar, s);
    T u = 0;
    if (has_row) u = eval_entry(my_x, my_y, my_z, r0 + lane, s, c0 + jstar);
    for (int l = 0; l < r; ++l) {
      const T vl = has_col ? V[(int64_t)l * n + lane] : (T)0;
      const T vj = __shfl(vl, jstar, 64);
      if (has_row) u -= vj * U[(int64_t)l * m + lane];
    }
    if (has_row) U[(int64_t)r * m + lane] = u;
    // |S_r|_F^2 update
    double cross = 0.0;
    for (int l = 0; l < r; ++l) {
      const double pu = has_row ? (double)U[(int64_t)l * m + lane] * (double)u : 0.0;
      const double pv = has_col ? (double)V[(int64_t)l * n + lane] * (double)v : 0.0;
      cross += wave_sum(pu) * wave_sum(pv);
    }
    const double uu = wave_sum((double)u * (double)u);
    const double vv = wave_sum((double)v * (double)v);
    s2 += 2.0 * cross + uu * vv;
    ++r;
    if (aca_stop(uu, vv, s2, A.eps)) break;
    if (r >= kcap) {
      cap_hit = kcap < min(m, n);
      break;
    }
    if (nused >= m) break;
    ArgMax<T> nx{(T)-1, 1 << 30, (T)0};
    if (has_row && !used) {
      nx.key = (T)fabs(u);
      nx.idx = lane;
    }
    istar = wave_argmax(nx).idx;
    if (istar < 0 || istar >= m) break;
  }
  if (lane == 0) {
    A.rank[b] = r;
    A.info[b] = (cap_hit ? 1 : 0) | (rows_eval << 1);
  }
}

// One block per workgroup of 256 threads.  Cross-thread reads of the working
// factors happen only after a barrier.  The used-row flags are bytes placed
// after V in the slot.
constexpr int kAcaThreads = 256;
constexpr int kAcaWaves = kAcaThreads / 64;

template <typename T>
struct AcaShared {
  T a[kMaxRank];             // u_l[i*] or v_l[j*] of the previous terms
  double du[kMaxRank][kAcaWaves], dv[kMaxRank][kAcaWaves];
  ArgMax<T> am[kAcaWaves];
  double red[3][kAcaWaves];
  ArgMax<T> am_out;
  double out[3];
};

template <typename T>
__device__ ArgMax<T> wg_argmax(ArgMax<T> a, AcaShared<T>& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  a = wave_argmax(a);
  if (lane == 0) sh.am[wave] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    ArgMax<T> r = sh.am[0];
    for (int w = 1; w < kAcaWaves; ++w) argmax_merge(r, sh.am[w]);
    sh.am_out = r;
  }
  __syncthreads();
  ArgMax<T> r = sh.am_out;
  __syncthreads();
  return r;
}

template <typename T>
__device__ void aca_wg(const AcaArgs<T>& A, int b, AcaShared<T>& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int2 ts = A.blk[b];
  const Cluster tau = A.cl[ts.x], sig = A.cl[ts.y];
  const int r0 = tau.x, m = tau.y - tau.x, c0 = sig.x, n = sig.y - sig.x;
  const int kcap = min(A.kmax, min(m, n));
  T* U = A.pool + (A.slot[b] - A.slot0);
  T* V = U + (int64_t)kcap * m;
  uint8_t* used = reinterpret_cast<uint8_t*>(V + (int64_t)kcap * n);
  const Geom<T>& g = A.g;
  for (int i = tid; i < m; i += kAcaThreads) used[i] = 0;
  __syncthreads();
  int nused = 0, r = 0, istar = 0, rows_eval = 0;
  double s2 = 0.0;
  bool cap_hit = false;
  while (true) {
    if (tid < r) sh.a[tid] = U[(int64_t)tid * m + istar];
    __syncthreads();
    const double xi = g.c[r0 + istar], yi = g.c[g.n + r0 + istar], zi = g.c[2 * g.n + r0 + istar];
    ArgMax<T> am{(T)-1, 1 << 30, (T)0};
    for (int j = tid; j < n; j += kAcaThreads) {
      Src<T> s;
      load_src(g, c0 + j, s);
      T val = eval_entry(xi, yi, zi, r0 + istar, s, c0 + j);
      for (int l = 0; l < r; ++l) val -= sh.a[l] * V[(int64_t)l * n + j];
      V[(int64_t)r * n + j] = val;
      const T k = (T)fabs(val);
      if (k > am.key) am = ArgMax<T>{k, j, val};
    }
    if (tid == 0) used[istar] = 1;
    ++rows_eval;
    ++nused;
    am = wg_argmax(am, sh);
    if (am.val == (T)0 || am.idx < 0 || am.idx >= n) {
      if (nused >= m) break;
      ArgMax<T> nx{(T)-1, 1 << 30, (T)0};
      for (int i = tid; i < m; i += kAcaThreads) {
        if (used[i]) continue;
        const T k = (r > 0) ? (T)fabs(U[(int64_t)(r - 1) * m + i]) : (T)0;
        if (k > nx.key) nx = ArgMax<T>{k, i, (T)0};
      }
      istar = wg_argmax(nx, sh).idx;
      if (istar < 0 || istar >= m) break;
      continue;
    }
    const int jstar = am.idx;
    const T delta = am.val;
    double vv = 0.0;
    for (int j = tid; j < n; j += kAcaThreads) {
      const T v = V[(int64_t)r * n + j] / delta;
      V[(int64_t)r * n + j] = v;
      vv += (double)v * (double)v;
    }
    if (tid < r) sh.a[tid] = V[(int64_t)tid * n + jstar];
    __syncthreads();
    Src<T> s;
    load_src(g, c0 + jstar, s);
    double uu = 0.0;
    ArgMax<T> nx{(T)-1, 1 << 30, (T)0};
    for (int i = tid; i < m; i += kAcaThreads) {
      T u = eval_entry(g.c[r0 + i], g.c[g.n + r0 + i], g.c[2 * g.n + r0 + i], r0 + i, s, c0 + jstar);
      for (int l = 0; l < r; ++l) u -= sh.a[l] * U[(int64_t)l * m + i];
      U[(int64_t)r * m + i] = u;
      uu += (double)u * (double)u;
      if (!used[i]) {
        const T k = (T)fabs(u);
        if (k > nx.key) nx = ArgMax<T>{k, i, (T)0};
      }
    }
    __syncthreads();
    // cross terms (u_l . u_r)(v_l . v_r) for l < r
    for (int l = 0; l < r; ++l) {
      double pu = 0.0, pv = 0.0;
      for (int i = tid; i < m; i += kAcaThreads)
        pu += (double)U[(int64_t)l * m + i] * (double)U[(int64_t)r * m + i];
      for (int j = tid; j < n; j += kAcaThreads)
        pv += (double)V[(int64_t)l * n + j] * (double)V[(int64_t)r * n + j];
      pu = wave_sum(pu);
      pv = wave_sum(pv);
      if (lane == 0) {
        sh.du[l][wave] = pu;
        sh.dv[l][wave] = pv;
      }
    }
    uu = wave_sum(uu);
    vv = wave_sum(vv);
    nx = wave_argmax(nx);
    if (lane == 0) {
      sh.red[0][wave] = uu;
      sh.red[1][wave] = vv;
      sh.am[wave] = nx;
    }
    __syncthreads();
    if (wave == 0) {
      double c = 0.0;
      for (int l = lane; l < r; l += 64) {
        double a = 0.0, bb = 0.0;
        for (int w = 0; w < kAcaWaves; ++w) {
          a += sh.du[l][w];
          bb += sh.dv[l][w];
        }
        c += a * bb;
      }
      c = wave_sum(c);
      if (lane == 0) {
        double tu = 0.0, tv = 0.0;
        ArgMax<T> best = sh.am[0];
        for (int w = 0; w < kAcaWaves; ++w) {
          tu += sh.red[0][w];
          tv += sh.red[1][w];
          if (w) argmax_merge(best, sh.am[w]);
        }
        sh.out[0] = tu;
        sh.out[1] = tv;
        sh.out[2] = c;
        sh.am_out = best;
      }
    }
    __syncthreads();
    uu = sh.out[0];
    vv = sh.out[1];
    const double cross = sh.out[2];
    const int inext = sh.am_out.idx;
    __syncthreads();
    s2 += 2.0 * cross + uu * vv;
    ++r;
    if (aca_stop(uu, vv, s2, A.eps)) break;
    if (r >= kcap) {
      cap_hit = kcap < min(m, n);
      break;
    }
    if (nused >= m) break;
    if (inext < 0 || inext >= m) break;
    istar = inext;
  }
  if (tid == 0) {
    A.rank[b] = r;
    A.info[b] = (cap_hit ? 1 : 0) | (rows_eval << 1);
  }
}

// Task t < nbig: big block; otherwise four small blocks, one per wavefront.
template <typename T>
__global__ __launch_bounds__(kAcaThreads) void k_aca(AcaArgs<T> A) {
  __shared__ AcaShared<T> sh;
  const int64_t ntask = A.nbig + (A.nsmall + kAcaWaves - 1) / kAcaWaves;
  for (int64_t t = blockIdx.x; t < ntask; t += gridDim.x) {
    if (t < A.nbig) {
      aca_wg(A, A.big[t], sh);
      __syncthreads();
    } else {
      const int64_t k = (t - A.nbig) * kAcaWaves + (threadIdx.x >> 6);
      if (k < A.nsmall) aca_wave(A, A.small[k]);
    }
  }
}

// Working-slot size (elements) of every block and its workgroup/wavefront class.
template <typename T>
__global__ void k_aca_slots(const int2* __restrict__ blk, int64_t nb, const Cluster* __restrict__ cl,
                            int kmax, int64_t* __restrict__ slot, int64_t* __restrict__ is_big) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const Cluster t = cl[ts.x], s = cl[ts.y];
    const int64_t m = t.y - t.x, n = s.y - s.x;
    const int64_t kcap = min((int64_t)kmax, min(m, n));
    const int64_t flag_elems = (m + (int64_t)sizeof(T) - 1) / (int64_t)sizeof(T);
    slot[b] = ((kcap * (m + n) + flag_elems) + 3) & ~(int64_t)3;
    is_big[b] = (m > 64 || n > 64) ? 1 : 0;
  }
}

__global__ void k_split_lists(const int64_t* __restrict__ is_big, const int64_t* __restrict__ ob,
                              int64_t nb, int32_t* __restrict__ big, int32_t* __restrict__ small) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    if (is_big[b])
      big[ob[b]] = (int32_t)b;
    else
      small[b - ob[b]] = (int32_t)b;
  }
}

// ------------------------------------------------------------------ packing
// Packed size of a factorised block: r * (LD(tau) + LD(sigma)).
__global__ void k_packed_sizes(const int2* __restrict__ blk, int64_t nb, const int32_t* __restrict__ rank,
                               LeafTab L, int64_t* __restrict__ sz) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const int2 lt = L.cl_leaves[ts.x], ls = L.cl_leaves[ts.y];
    const int64_t ldt = L.ldpre[lt.y + 1] - L.ldpre[lt.x];
    const int64_t lds = L.ldpre[ls.y + 1] - L.ldpre[ls.x];
    sz[b] = (int64_t)rank[b] * (ldt + lds);
  }
}

// Copy the working factors of each block into its leaf slices: U slices of
// the row leaves, then V slices of the column leaves.
template <typename T>
__global__ __launch_bounds__(256) void k_pack(const int2* __restrict__ blk, int64_t nb,
                                              const Cluster* __restrict__ cl, LeafTab L,
                                              const int32_t* __restrict__ rank,
                                              const int64_t* __restrict__ slot, int64_t slot0,
                                              const T* __restrict__ pool, int kmax, const int64_t* __restrict__ fo, T* __restrict__ arena,
                                              uint64_t* __restrict__ ptr_out) {
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int2 ts = blk[b];
    const Cluster tau = cl[ts.x], sig = cl[ts.y];
    const int m = tau.y - tau.x, n = sig.y - sig.x;
    const int r = rank[b];
    const int kcap = min(kmax, min(m, n));
    const T* U = pool + (slot[b] - slot0);
    const T* Vw = U + (int64_t)kcap * m;
    T* dst = arena + fo[b];
    if (threadIdx.x == 0) ptr_out[b] = (uint64_t)(uintptr_t)dst;
    const int2 lt = L.cl_leaves[ts.x], ls = L.cl_leaves[ts.y];
    const int64_t ldt = L.ldpre[lt.y + 1] - L.ldpre[lt.x];
    for (int lf = lt.x; lf <= lt.y; ++lf) {
      const int ld = leaf_ld(L, lf), ml = L.m[lf], off = L.lo[lf] - tau.x;
      T* d = dst + (int64_t)r * (L.ldpre[lf] - L.ldpre[lt.x]);
      for (int e = threadIdx.x; e < ld * r; e += blockDim.x) {
        const int i = e % ld, l = e / ld;
        d[e] = (i < ml) ? U[(int64_t)l * m + off + i] : (T)0;
      }
    }
    T* dv = dst + (int64_t)r * ldt;
    for (int lf = ls.x; lf <= ls.y; ++lf) {
      const int ld = leaf_ld(L, lf), ml = L.m[lf], off = L.lo[lf] - sig.x;
      T* d = dv + (int64_t)r * (L.ldpre[lf] - L.ldpre[ls.x]);
      for (int e = threadIdx.x; e < ld * r; e += blockDim.x) {
        const int i = e % ld, l = e / ld;
        d[e] = (i < ml) ? Vw[(int64_t)l * n + off + i] : (T)0;
      }
    }
  }
}

// ------------------------------------------------------------------ items
// Number of slices every block contributes to the row lists and column lists.
__global__ void k_item_counts(const int2* __restrict__ dns, int64_t nd, const int2* __restrict__ lr,
                              int64_t nl, LeafTab L, int64_t* __restrict__ crow,
                              int64_t* __restrict__ ccol) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nd + nl;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = (b < nd) ? dns[b] : lr[b - nd];
    const int2 lt = L.cl_leaves[ts.x], ls = L.cl_leaves[ts.y];
    const int64_t nt = lt.y - lt.x + 1, ns = ls.y - ls.x + 1;
    crow[b] = nt;
    ccol[b] = (b < nd) ? nt * ns : ns;
  }
}

template <typename T>
__global__ void k_item_expand(const int2* __restrict__ dns, int64_t nd, const int2* __restrict__ lr,
                              int64_t nl, const Cluster* __restrict__ cl, LeafTab L,
                              const int64_t* __restrict__ doff, const T* __restrict__ D,
                              const uint64_t* __restrict__ lrptr, const int32_t* __restrict__ rank,
                              const int64_t* __restrict__ toff, const int64_t* __restrict__ pslot,
                              const int64_t* __restrict__ orow, const int64_t* __restrict__ ocol,
                              Item* __restrict__ irow, uint64_t* __restrict__ krow,
                              Item* __restrict__ icol, uint64_t* __restrict__ kcol) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nd + nl;
       b += (int64_t)gridDim.x * blockDim.x) {
    const bool dense = b < nd;
    const int64_t bl = dense ? b : b - nd;
    const int2 ts = dense ? dns[bl] : lr[bl];
    const Cluster tau = cl[ts.x], sig = cl[ts.y];
    const int2 lt = L.cl_leaves[ts.x], ls = L.cl_leaves[ts.y];
    const int64_t ldt = L.ldpre[lt.y + 1] - L.ldpre[lt.x];
    int64_t pr = orow[b], pc = ocol[b];
    if (dense) {
      const int n = sig.y - sig.x;
      const T* base = D + doff[bl];
      for (int lf = lt.x; lf <= lt.y; ++lf, ++pr) {
        const T* d = base + (int64_t)n * (L.ldpre[lf] - L.ldpre[lt.x]);
        irow[pr] = Item{(uint64_t)(uintptr_t)d, n, sig.x, -1, 0, 0, 0};
        krow[pr] = (uint64_t)lf;
        for (int cf = ls.x; cf <= ls.y; ++cf, ++pc) {
          const int ld = leaf_ld(L, lf);
          const T* dt = d + (int64_t)(L.lo[cf] - sig.x) * ld;
          icol[pc] = Item{(uint64_t)(uintptr_t)dt, L.m[cf], L.lo[lf], lf, 0, 0, 0};
          kcol[pc] = (uint64_t)cf;
        }
      }
    } else {
      const int r = rank[bl];
      const T* base = reinterpret_cast<const T*>((uintptr_t)lrptr[bl]);
      const int to = (int)toff[bl];
      const int64_t ps = pslot[bl];
      for (int lf = lt.x; lf <= lt.y; ++lf, ++pr) {
        const T* d = base + (int64_t)r * (L.ldpre[lf] - L.ldpre[lt.x]);
        irow[pr] = Item{(uint64_t)(uintptr_t)d, r, to, (int)(ps + (int64_t)(lf - lt.x) * r), 1, 0, 0};
        krow[pr] = (uint64_t)lf;
      }
      const T* bv = base + (int64_t)r * ldt;
      for (int cf = ls.x; cf <= ls.y; ++cf, ++pc) {
        const T* d = bv + (int64_t)r * (L.ldpre[cf] - L.ldpre[ls.x]);
        icol[pc] = Item{(uint64_t)(uintptr_t)d, r, to, (int)(ps + (int64_t)(cf - ls.x) * r), 1, 0, 0};
        kcol[pc] = (uint64_t)cf;
      }
    }
    (void)tau;
  }
}

__global__ void k_iota(int32_t* __restrict__ v, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    v[k] = (int32_t)k;
}

__global__ void k_gather_items(const Item* __restrict__ in, const int32_t* __restrict__ idx, int64_t n,
                               Item* __restrict__ out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    out[k] = in[idx[k]];
}

__global__ void k_leaf_counts(const uint64_t* __restrict__ keys, int64_t n, int64_t* __restrict__ cnt) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd((unsigned long long*)&cnt[keys[k]], 1ull);
}

// Per-block values derived from the ranks.
__global__ void k_lr_meta(const int2* __restrict__ lr, int64_t nl, const int32_t* __restrict__ rank,
                          LeafTab L, int64_t* __restrict__ rk, int64_t* __restrict__ psz) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nl;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = lr[b];
    const int2 lt = L.cl_leaves[ts.x], ls = L.cl_leaves[ts.y];
    const int64_t nk = max(lt.y - lt.x + 1, ls.y - ls.x + 1);
    rk[b] = rank[b];
    psz[b] = (int64_t)rank[b] * nk;
  }
}

// Dense block sizes: n * LD(tau).
__global__ void k_dense_sizes(const int2* __restrict__ dns, int64_t nd, const Cluster* __restrict__ cl,
                              LeafTab L, int64_t* __restrict__ sz) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nd;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = dns[b];
    const Cluster s = cl[ts.y];
    const int2 lt = L.cl_leaves[ts.x];
    sz[b] = (int64_t)(s.y - s.x) * (L.ldpre[lt.y + 1] - L.ldpre[lt.x]);
  }
}

// Unpack one factorised block back into plain column-major U (m x r), V (n x r).
template <typename T>
__global__ void k_unpack(const int2* __restrict__ lr, int64_t b, const Cluster* __restrict__ cl,
                         LeafTab L, const int32_t* __restrict__ rank,
                         const uint64_t* __restrict__ lrptr, T* __restrict__ out) {
  const int2 ts = lr[b];
  const Cluster tau = cl[ts.x], sig = cl[ts.y];
  const int m = tau.y - tau.x, n = sig.y - sig.x, r = rank[b];
  const T* base = reinterpret_cast<const T*>((uintptr_t)lrptr[b]);
  const int2 lt = L.cl_leaves[ts.x], ls = L.cl_leaves[ts.y];
  const int64_t ldt = L.ldpre[lt.y + 1] - L.ldpre[lt.x];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)(m + n) * r;
       e += (int64_t)gridDim.x * blockDim.x) {
    const bool isu = e < (int64_t)m * r;
    const int64_t ee = isu ? e : e - (int64_t)m * r;
    const int rows = isu ? m : n;
    const int i = (int)(ee % rows), l = (int)(ee / rows);
    const int pos = (isu ? tau.x : sig.x) + i;
    int lf0 = isu ? lt.x : ls.x, lf1 = isu ? lt.y : ls.y;
    int lf = lf0;
    while (lf < lf1 && L.lo[lf + 1] <= pos) ++lf;
    const T* sl = (isu ? base : base + (int64_t)r * ldt) + (int64_t)r * (L.ldpre[lf] - L.ldpre[lf0]);
    out[e] = sl[(int64_t)l * leaf_ld(L, lf) + (pos - L.lo[lf])];
  }
}

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_entries(const Geom<T>& g, const int32_t* inv, const int32_t* rows, const int32_t* cols,
                    int64_t cnt, double* out, hipStream_t s) {
  k_entries<T><<<grid_for(cnt, 256), 256, 0, s>>>(g, inv, rows, cols, cnt, out);
  HM_LAUNCH_CHECK();
}
void launch_inverse_perm(const int32_t* perm, int64_t n, int32_t* inv, hipStream_t s) {
  k_inverse_perm<<<grid_for(n, 256), 256, 0, s>>>(perm, n, inv);
  HM_LAUNCH_CHECK();
}

template <typename T>
void launch_near(const Geom<T>& g, const int2* dns, int64_t nd, const Cluster* cl,
                 const int32_t* leaf_lo, const int32_t* leaf_m, const int64_t* ldpre,
                 const int2* cl_leaves, const int64_t* doff, T* D, hipStream_t s) {
  if (nd == 0) return;
  LeafTab L{leaf_lo, leaf_m, ldpre, cl_leaves};
  k_near<T><<<grid_for(nd, 1, 1 << 20), 256, 0, s>>>(g, dns, nd, cl, L, doff, D);
  HM_LAUNCH_CHECK();
}

void launch_dense_sizes(const int2* dns, int64_t nd, const Cluster* cl, const int32_t* leaf_lo,
                        const int32_t* leaf_m, const int64_t* ldpre, const int2* cl_leaves,
                        int64_t* sz, hipStream_t s) {
  if (nd == 0) return;
  LeafTab L{leaf_lo, leaf_m, ldpre, cl_leaves};
  k_dense_sizes<<<grid_for(nd, 256), 256, 0, s>>>(dns, nd, cl, L, sz);
  HM_LAUNCH_CHECK();
}

// Batched ACA of the blocks blk[0..nb) followed by packing into `arena`
// (allocated here, exact size) -- see the host orchestration for chunking.
template <typename T>
void launch_aca_slots(const int2* blk, int64_t nb, const Cluster* cl, int kmax, int64_t* slot,
                      int64_t* is_big, hipStream_t s) {
  k_aca_slots<T><<<grid_for(nb, 256), 256, 0, s>>>(blk, nb, cl, kmax, slot, is_big);
  HM_LAUNCH_CHECK();
}
template void launch_aca_slots<float>(const int2*, int64_t, const Cluster*, int, int64_t*, int64_t*,
                                      hipStream_t);
template void launch_aca_slots<double>(const int2*, int64_t, const Cluster*, int, int64_t*, int64_t*,
                                       hipStream_t);

void launch_split_lists(const int64_t* is_big, const int64_t* ob, int64_t nb, int32_t* big,
                        int32_t* small, hipStream_t s) {
  k_split_lists<<<grid_for(nb, 256), 256, 0, s>>>(is_big, ob, nb, big, small);
  HM_LAUNCH_CHECK();
}

template <typename T>
void launch_aca(const Geom<T>& g, const int2* blk, const Cluster* cl, const int64_t* slot,
                int64_t slot0, T* pool, const int32_t* big, int64_t nbig, const int32_t* small,
                int64_t nsmall, int kmax, double eps, int32_t* rank, int32_t* info, hipStream_t s) {
  AcaArgs<T> A{g, blk, cl, slot, slot0, pool, big, nbig, small, nsmall, kmax, eps, rank, info};
  const int64_t ntask = nbig + ceil_div(nsmall, kAcaWaves);
  if (ntask == 0) return;
  int dev = 0, ncu = 0;
  HM_HIP(hipGetDevice(&dev));
  HM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t grid = std::min<int64_t>(ntask, (int64_t)std::max(ncu, 1) * 16);
  k_aca<T><<<(unsigned)grid, kAcaThreads, 0, s>>>(A);
  HM_LAUNCH_CHECK();
}

void launch_packed_sizes(const int2* blk, int64_t nb, const int32_t* rank, const int32_t* leaf_lo,
                         const int32_t* leaf_m, const int64_t* ldpre, const int2* cl_leaves,
                         int64_t* sz, hipStream_t s) {
  LeafTab L{leaf_lo, leaf_m, ldpre, cl_leaves};
  k_packed_sizes<<<grid_for(nb, 256), 256, 0, s>>>(blk, nb, rank, L, sz);
  HM_LAUNCH_CHECK();
}

template <typename T>
void launch_pack(const int2* blk, int64_t nb, const Cluster* cl, const int32_t* leaf_lo,
                 const int32_t* leaf_m, const int64_t* ldpre, const int2* cl_leaves,
                 const int32_t* rank, const int64_t* slot, int64_t slot0, const T* pool, int kmax,
                 const int64_t* fo, T* arena, uint64_t* ptr_out, hipStream_t s) {
  LeafTab L{leaf_lo, leaf_m, ldpre, cl_leaves};
  k_pack<T><<<grid_for(nb, 1, 1 << 20), 256, 0, s>>>(blk, nb, cl, L, rank, slot, slot0, pool, kmax,
                                                     fo, arena, ptr_out);
  HM_LAUNCH_CHECK();
}

void launch_lr_meta(const int2* lr, int64_t nl, const int32_t* rank, const int32_t* leaf_lo,
                    const int32_t* leaf_m, const int64_t* ldpre, const int2* cl_leaves, int64_t* rk,
                    int64_t* psz, hipStream_t s) {
  if (nl == 0) return;
  LeafTab L{leaf_lo, leaf_m, ldpre, cl_leaves};
  k_lr_meta<<<grid_for(nl, 256), 256, 0, s>>>(lr, nl, rank, L, rk, psz);
  HM_LAUNCH_CHECK();
}

void launch_item_counts(const int2* dns, int64_t nd, const int2* lr, int64_t nl,
                        const int32_t* leaf_lo, const int32_t* leaf_m, const int64_t* ldpre,
                        const int2* cl_leaves, int64_t* crow, int64_t* ccol, hipStream_t s) {
  LeafTab L{leaf_lo, leaf_m, ldpre, cl_leaves};
  k_item_counts<<<grid_for(nd + nl, 256), 256, 0, s>>>(dns, nd, lr, nl, L, crow, ccol);
  HM_LAUNCH_CHECK();
}

template <typename T>
void launch_item_expand(const int2* dns, int64_t nd, const int2* lr, int64_t nl, const Cluster* cl,
                        const int32_t* leaf_lo, const int32_t* leaf_m, const int64_t* ldpre,
                        const int2* cl_leaves, const int64_t* doff, const T* D,
                        const uint64_t* lrptr, const int32_t* rank, const int64_t* toff,
                        const int64_t* pslot, const int64_t* orow, const int64_t* ocol, Item* irow,
                        uint64_t* krow, Item* icol, uint64_t* kcol, hipStream_t s) {
  LeafTab L{leaf_lo, leaf_m, ldpre, cl_leaves};
  k_item_expand<T><<<grid_for(nd + nl, 64), 64, 0, s>>>(dns, nd, lr, nl, cl, L, doff, D, lrptr,
                                                         rank, toff, pslot, orow, ocol, irow, krow,
                                                         icol, kcol);
  HM_LAUNCH_CHECK();
}

void launch_iota(int32_t* v, int64_t n, hipStream_t s) {
  k_iota<<<grid_for(n, 256), 256, 0, s>>>(v, n);
  HM_LAUNCH_CHECK();
}
void launch_gather_items(const Item* in, const int32_t* idx, int64_t n, Item* out, hipStream_t s) {
  k_gather_items<<<grid_for(n, 256), 256, 0, s>>>(in, idx, n, out);
  HM_LAUNCH_CHECK();
}
void launch_leaf_counts(const uint64_t* keys, int64_t n, int64_t* cnt, hipStream_t s) {
  k_leaf_counts<<<grid_for(n, 256), 256, 0, s>>>(keys, n, cnt);
  HM_LAUNCH_CHECK();
}

template <typename T>
void launch_unpack(const int2* lr, int64_t b, const Cluster* cl, const int32_t* leaf_lo,
                   const int32_t* leaf_m, const int64_t* ldpre, const int2* cl_leaves,
                   const int32_t* rank, const uint64_t* lrptr, T* out, int64_t total, hipStream_t s) {
  LeafTab L{leaf_lo, leaf_m, ldpre, cl_leaves};
  k_unpack<T><<<grid_for(total, 256), 256, 0, s>>>(lr, b, cl, L, rank, lrptr, out);
  HM_LAUNCH_CHECK();
}

#define HM_INST(T)                                                                                 \
  template void launch_entries<T>(const Geom<T>&, const int32_t*, const int32_t*, const int32_t*,  \
                                  int64_t, double*, hipStream_t);                                  \
  template void launch_near<T>(const Geom<T>&, const int2*, int64_t, const Cluster*,               \
                               const int32_t*, const int32_t*, const int64_t*, const int2*,        \
                               const int64_t*, T*, hipStream_t);                                   \
  template void launch_aca<T>(const Geom<T>&, const int2*, const Cluster*, const int64_t*, int64_t, \
                              T*, const int32_t*, int64_t, const int32_t*, int64_t, int, double,   \
                              int32_t*, int32_t*, hipStream_t);                                    \
  template void launch_pack<T>(const int2*, int64_t, const Cluster*, const int32_t*,               \
                               const int32_t*, const int64_t*, const int2*, const int32_t*,        \
                               const int64_t*, int64_t, const T*, int, const int64_t*, T*,         \
                               uint64_t*, hipStream_t);                                            \
  template void launch_item_expand<T>(const int2*, int64_t, const int2*, int64_t, const Cluster*,  \
                                      const int32_t*, const int32_t*, const int64_t*, const int2*, \
                                      const int64_t*, const T*, const uint64_t*, const int32_t*,   \
                                      const int64_t*, const int64_t*, const int64_t*,              \
                                      const int64_t*, Item*, uint64_t*, Item*, uint64_t*,          \
                                      hipStream_t);                                                \
  template void launch_unpack<T>(const int2*, int64_t, const Cluster*, const int32_t*,             \
                                 const int32_t*, const int64_t*, const int2*, const int32_t*,      \
                                 const uint64_t*, T*, int64_t, hipStream_t);
HM_INST(float)
HM_INST(double)
#undef HM_INST

}  // namespace hm
