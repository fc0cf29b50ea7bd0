// Geometry preparation, Morton codes, cluster tree, bounding boxes and the
// level-wise block cluster tree traversal.
//
// Compiled with -ffp-contract=off: the Morton quantisation, the boxes and the
// admissibility test of Sec. 2.3 (eq. admissibilityCondition) must round
// exactly like the plain FP64 definition, so that the block partition is
// bit-identical to it.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "hm_internal.h"

namespace hm {

// ------------------------------------------------------------------ geometry
// Collocation points x_i = ((v0 + v1) + v2) / 3 (element centres, Sec. 4.1),
// application order, SoA double[3][n].
__global__ void k_centroids(const double* __restrict__ V, const int32_t* __restrict__ T, int64_t n,
                            double* __restrict__ C) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = T[3 * t], b = T[3 * t + 1], c = T[3 * t + 2];
#pragma unroll
    for (int d = 0; d < 3; ++d) C[d * n + t] = ((V[3 * a + d] + V[3 * b + d]) + V[3 * c + d]) / 3.0;
  }
}

// Per-block partial min/max of the centroids: out[blk][6].
__global__ __launch_bounds__(256) void k_minmax_partial(const double* __restrict__ C, int64_t n,
                                                        int64_t off, int64_t cnt,
                                                        double* __restrict__ out) {
  __shared__ double lds[6][256];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t t = off + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < off + cnt;
       t += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double v = C[d * n + t];
      mn[d] = fmin(mn[d], v);
      mx[d] = fmax(mx[d], v);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lds[d][threadIdx.x] = mn[d];
    lds[3 + d][threadIdx.x] = mx[d];
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lds[d][threadIdx.x] = fmin(lds[d][threadIdx.x], lds[d][threadIdx.x + s]);
        lds[3 + d][threadIdx.x] = fmax(lds[3 + d][threadIdx.x], lds[3 + d][threadIdx.x + s]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) out[blockIdx.x * 6 + threadIdx.x] = lds[threadIdx.x][0];
}

__global__ void k_minmax_final(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double r[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int b = 0; b < nblk; ++b)
    for (int d = 0; d < 3; ++d) {
      r[d] = fmin(r[d], part[b * 6 + d]);
      r[3 + d] = fmax(r[3 + d], part[b * 6 + 3 + d]);
    }
  for (int d = 0; d < 6; ++d) out[d] = r[d];
}

// Spread the low 21 bits of x to every third bit.
__device__ inline uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// Morton code of the collocation points of one geometry, positions
// [off, off + cnt) of the SoA array C (Sec. 3.1 "Spatial data structure"):
// q_d = min(floor((c_d - a_d) * scale), 2^21 - 1); x is the most significant
// bit of every triple.  Also initialises the value array of the sort.
__global__ void k_morton(const double* __restrict__ C, int64_t n, int64_t off, int64_t cnt,
                         double ax, double ay, double az, double scale,
                         uint64_t* __restrict__ keys, int32_t* __restrict__ idx) {
  const double a[3] = {ax, ay, az};
  for (int64_t t = off + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < off + cnt;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint64_t q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double v = floor((C[d * n + t] - a[d]) * scale);
      v = fmin(v, (double)((1 << kMortonBits) - 1));
      q[d] = (uint64_t)v;
    }
    keys[t] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    idx[t] = (int32_t)t;
  }
}

// Quadrature data and self-terms in Morton order.  For position p the source
// triangle is t = perm[p]; its vertex offsets d_k = v_k - c are stored in
// the storage type, and the nodes of the rule are c and c + beta d_k (beta1
// for nodes 1..3, beta2 for 4..6), so that a distance |x_i - y_jq| is formed
// as (x_i - c_j) - beta d_k with the large part in double.  Nine values per
// triangle instead of the 21 node offsets: the entry kernels, which stream
// these records, read 64 bytes per source in FP32 instead of 116.
//
// Self-term (x_i inside the flat triangle): the triangle is split at x_i over
// its edges; with h the distance of x_i to an edge line and l_a, l_b the
// signed coordinates of the edge's end points along it, measured from the
// foot point, the edge contributes h * (asinh(l_b / h) - asinh(l_a / h)).
template <typename T>
__global__ void k_geom_sorted(const double* __restrict__ V, const int32_t* __restrict__ Tri,
                              const int32_t* __restrict__ perm, int64_t n, double* __restrict__ c,
                              T* __restrict__ o, T* __restrict__ aw, T* __restrict__ sf) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = perm[p];
    double v[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int32_t vi = Tri[3 * t + k];
#pragma unroll
      for (int d = 0; d < 3; ++d) v[k][d] = V[3 * (int64_t)vi + d];
    }
    double cc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      cc[d] = ((v[0][d] + v[1][d]) + v[2][d]) / 3.0;
      c[d * n + p] = cc[d];
    }
    // vertex offsets d_k = v_k - c; the rule's nodes are c and c + beta d_k
#pragma unroll
    for (int k = 0; k < kNV; ++k)
#pragma unroll
      for (int d = 0; d < 3; ++d) o[(int64_t)(d * kNV + k) * n + p] = (T)(v[k][d] - cc[d]);
    const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                          e1[0] * e2[1] - e1[1] * e2[0]};
    const double area = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    const double inv4pi = 0.079577471545947667884441881686257181;  // 1/(4 pi)
    aw[p] = (T)(area * inv4pi);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double* A = v[k];
      const double* B = v[(k + 1) % 3];
      double e[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      double le = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
      double tt[3] = {e[0] / le, e[1] / le, e[2] / le};
      double ax = A[0] - cc[0], ay = A[1] - cc[1], az = A[2] - cc[2];
      double bx = B[0] - cc[0], by = B[1] - cc[1], bz = B[2] - cc[2];
      double la = ax * tt[0] + ay * tt[1] + az * tt[2];
      double lb = bx * tt[0] + by * tt[1] + bz * tt[2];
      double fx = ax - la * tt[0], fy = ay - la * tt[1], fz = az - la * tt[2];
      double h = sqrt(fx * fx + fy * fy + fz * fz);
      s += h * (asinh(lb / h) - asinh(la / h));
    }
    sf[p] = (T)(s * inv4pi);
  }
}

// ------------------------------------------------------------------ cluster tree
// Node [lo, hi) splits iff hi - lo > leaf (Sec. 2.3, (C3)/(C4), CBC).
__global__ void k_cluster_flags(const Cluster* __restrict__ cl, int64_t beg, int64_t cnt, int leaf,
                                int64_t* __restrict__ flag) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < cnt;
       k += (int64_t)gridDim.x * blockDim.x) {
    Cluster c = cl[beg + k];
    flag[k] = (c.y - c.x > leaf) ? 1 : 0;
  }
}

__global__ void k_cluster_emit(Cluster* __restrict__ cl, int64_t beg, int64_t cnt,
                               const int64_t* __restrict__ flag, const int64_t* __restrict__ off,
                               int64_t next) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < cnt;
       k += (int64_t)gridDim.x * blockDim.x) {
    Cluster c = cl[beg + k];
    if (flag[k]) {
      const int64_t ch = next + 2 * off[k];
      const int mid = c.x + (c.y - c.x) / 2;
      cl[ch] = make_int4(c.x, mid, -1, c.w + 1);
      cl[ch + 1] = make_int4(mid, c.y, -1, c.w + 1);
      c.z = (int)ch;
      cl[beg + k] = c;
    }
  }
}

// Mark the first position of every leaf cluster.
__global__ void k_leaf_marks(const Cluster* __restrict__ cl, int64_t ncl, int64_t* __restrict__ mark) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncl;
       k += (int64_t)gridDim.x * blockDim.x) {
    Cluster c = cl[k];
    if (c.z < 0) mark[c.x] = 1;
  }
}

// pos_leaf[p] = leaf index (Morton order of leaves) of position p, from the
// exclusive scan of the marks: leaf = excl[p] + mark[p] - 1.
__global__ void k_pos_leaf(const int64_t* __restrict__ mark, const int64_t* __restrict__ excl,
                           int64_t n, int32_t* __restrict__ pos_leaf) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    pos_leaf[p] = (int32_t)(excl[p] + mark[p] - 1);
}

// Leaf table (Morton order) and the leaf range of every cluster.
__global__ void k_leaf_table(const Cluster* __restrict__ cl, int64_t ncl,
                             const int32_t* __restrict__ pos_leaf, int32_t* __restrict__ leaf_lo,
                             int32_t* __restrict__ leaf_m, int32_t* __restrict__ leaf_cl,
                             int64_t* __restrict__ leaf_ld, int2* __restrict__ cl_leaves) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncl;
       k += (int64_t)gridDim.x * blockDim.x) {
    Cluster c = cl[k];
    const int first = pos_leaf[c.x], last = pos_leaf[c.y - 1];
    cl_leaves[k] = make_int2(first, last);
    if (c.z < 0) {
      leaf_lo[first] = c.x;
      leaf_m[first] = c.y - c.x;
      leaf_cl[first] = (int32_t)k;
      leaf_ld[first] = ((c.y - c.x) + 3) & ~3;
    }
  }
}

// ------------------------------------------------------------------ boxes
// Box of every leaf cluster from its members (Sec. 2.3: per-axis min / max).
__global__ void k_leaf_boxes(const Cluster* __restrict__ cl, const int32_t* __restrict__ leaf_cl,
                             int64_t nleaf, const double* __restrict__ c, int64_t n,
                             double* __restrict__ box) {
  for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < nleaf;
       l += (int64_t)gridDim.x * blockDim.x) {
    const int k = leaf_cl[l];
    Cluster cc = cl[k];
    double b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int p = cc.x; p < cc.y; ++p)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double v = c[d * n + p];
        b[d] = fmin(b[d], v);
        b[3 + d] = fmax(b[3 + d], v);
      }
#pragma unroll
    for (int d = 0; d < 6; ++d) box[6 * (int64_t)k + d] = b[d];
  }
}

// Union of the two children for the internal nodes in [beg, beg + cnt).
__global__ void k_parent_boxes(const Cluster* __restrict__ cl, int64_t beg, int64_t cnt,
                               double* __restrict__ box) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < cnt;
       k += (int64_t)gridDim.x * blockDim.x) {
    Cluster c = cl[beg + k];
    if (c.z < 0) continue;
    const double* b1 = box + 6 * (int64_t)c.z;
    const double* b2 = box + 6 * ((int64_t)c.z + 1);
    double* b = box + 6 * (beg + k);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      b[d] = fmin(b1[d], b2[d]);
      b[3 + d] = fmax(b1[3 + d], b2[3 + d]);
    }
  }
}

// ------------------------------------------------------------------ traversal
// eq. admissibilityCondition squared: min(diam^2) <= eta^2 dist^2, with the
// evaluation order (a*a + b*b) + c*c and no contraction.
__device__ inline bool admissible(const double* bt, const double* bs, double eta2) {
  double dx = bt[3] - bt[0], dy = bt[4] - bt[1], dz = bt[5] - bt[2];
  const double dt2 = (dx * dx + dy * dy) + dz * dz;
  dx = bs[3] - bs[0];
  dy = bs[4] - bs[1];
  dz = bs[5] - bs[2];
  const double ds2 = (dx * dx + dy * dy) + dz * dz;
  double g[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double g1 = bs[d] - bt[3 + d];
    const double g2 = bt[d] - bs[3 + d];
    g[d] = fmax(fmax(g1, g2), 0.0);
  }
  const double dist2 = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
  return fmin(dt2, ds2) <= eta2 * dist2;
}

// Squared distance of two boxes.
__device__ inline double box_dist2(const double* bt, const double* bs) {
  double g[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) g[d] = fmax(fmax(bs[d] - bt[3 + d], bt[d] - bs[3 + d]), 0.0);
  return (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
}

// Does a triangle of cluster t share a vertex with one of cluster s?  Walks
// the triangles around the vertices of the smaller cluster.
__device__ inline bool share_vertex(const GalTouch& gt, Cluster t, Cluster s) {
  const Cluster a = (t.y - t.x <= s.y - s.x) ? t : s;
  const Cluster b = (t.y - t.x <= s.y - s.x) ? s : t;
  for (int i = a.x; i < a.y; ++i)
    for (int k = 0; k < 3; ++k) {
      const int32_t v = gt.vid[k * gt.n + i];
      for (int32_t q = gt.vbeg[v]; q < gt.vbeg[v + 1]; ++q) {
        const int32_t p = gt.vpos[q];
        if (b.x <= p && p < b.y) return true;
      }
    }
  return false;
}

// Algorithm 1 for one level of candidate blocks: admissible leaf, dense
// leaf, or subdivide (not admissible, both clusters > leaf).  The class of
// every candidate pair is packed for one scan: 1 = admissible (low 32
// bits), 1 << 32 = dense leaf (high 32 bits), 0 = subdivide.  The exclusive
// prefix then holds the admissible and dense offsets in its two halves, and
// the split offset is k minus both.  With gt.vid (Galerkin) an admissible
// pair whose triangles share a vertex is not admissible: its entries include
// singular integrals, which the ACA does not evaluate.  Only pairs whose
// boxes are within the reach of touching triangles are searched.
__global__ void k_classify(const int2* __restrict__ cand, int64_t ncand,
                           const Cluster* __restrict__ cl, const double* __restrict__ box,
                           double eta2, int leaf, GalTouch gt, int64_t* __restrict__ f) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncand;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = cand[k];
    const Cluster t = cl[ts.x], s = cl[ts.y];
    const double* bt = box + 6 * (int64_t)ts.x;
    const double* bs = box + 6 * (int64_t)ts.y;
    bool adm = admissible(bt, bs, eta2);
    if (adm && gt.vid && box_dist2(bt, bs) <= gt.reach2) adm = !share_vertex(gt, t, s);
    const bool split = !adm && (t.y - t.x > leaf) && (s.y - s.x > leaf);
    f[k] = adm ? 1 : (split ? 0 : (int64_t(1) << 32));
  }
}

// Children in the order (t1,s1), (t1,s2), (t2,s1), (t2,s2).
__global__ void k_emit(const int2* __restrict__ cand, int64_t ncand, const Cluster* __restrict__ cl,
                       const int64_t* __restrict__ f, const int64_t* __restrict__ off,
                       int2* __restrict__ adm_out, int2* __restrict__ dns_out,
                       int2* __restrict__ next) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncand;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = cand[k];
    const int64_t c = f[k], o = off[k];
    const int64_t oa = o & 0xffffffffLL, od = o >> 32;
    if (c == 1) {
      adm_out[oa] = ts;
    } else if (c != 0) {
      dns_out[od] = ts;
    } else {
      const int t1 = cl[ts.x].z, s1 = cl[ts.y].z;
      int2* q = next + 4 * (k - oa - od);
      q[0] = make_int2(t1, s1);
      q[1] = make_int2(t1, s1 + 1);
      q[2] = make_int2(t1 + 1, s1);
      q[3] = make_int2(t1 + 1, s1 + 1);
    }
  }
}

// ------------------------------------------------------------------ launchers
namespace {
constexpr int kT = 256;
}

void launch_centroids(const double* V, const int32_t* T, int64_t n, double* C, hipStream_t s) {
  k_centroids<<<grid_for(n, kT), kT, 0, s>>>(V, T, n, C);
  HM_LAUNCH_CHECK();
}

void launch_minmax(const double* C, int64_t n, int64_t off, int64_t cnt, double* out6,
                   hipStream_t s) {
  const int nblk = (int)std::min<int64_t>(grid_for(cnt, kT), 1024);
  double* part = dalloc_t<double>(6 * (size_t)nblk, s);
  k_minmax_partial<<<nblk, kT, 0, s>>>(C, n, off, cnt, part);
  HM_LAUNCH_CHECK();
  k_minmax_final<<<1, 64, 0, s>>>(part, nblk, out6);
  HM_LAUNCH_CHECK();
  dfree(part, s);
}

void launch_morton(const double* C, int64_t n, int64_t off, int64_t cnt, const double* a,
                   double scale, uint64_t* keys, int32_t* idx, hipStream_t s) {
  k_morton<<<grid_for(cnt, kT), kT, 0, s>>>(C, n, off, cnt, a[0], a[1], a[2], scale, keys, idx);
  HM_LAUNCH_CHECK();
}

template <typename T>
void launch_geom_sorted(const double* V, const int32_t* Tri, const int32_t* perm, int64_t n,
                        double* c, T* o, T* aw, T* sf, hipStream_t s) {
  k_geom_sorted<T><<<grid_for(n, kT), kT, 0, s>>>(V, Tri, perm, n, c, o, aw, sf);
  HM_LAUNCH_CHECK();
}
template void launch_geom_sorted<float>(const double*, const int32_t*, const int32_t*, int64_t,
                                        double*, float*, float*, float*, hipStream_t);
template void launch_geom_sorted<double>(const double*, const int32_t*, const int32_t*, int64_t,
                                         double*, double*, double*, double*, hipStream_t);

// Vertices and vertex indices of every triangle in Morton order (the
// Galerkin operator's singular entries and its touching test):
// v[(3 k + d) n + p] = coordinate d of vertex k of triangle perm[p],
// vid[k n + p] = its vertex index.
__global__ void k_tri_sorted(const double* __restrict__ V, const int32_t* __restrict__ Tri,
                             const int32_t* __restrict__ perm, int64_t n, double* __restrict__ v,
                             int32_t* __restrict__ vid) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = perm[p];
    for (int k = 0; k < 3; ++k) {
      const int32_t a = Tri[3 * t + k];
      vid[k * n + p] = a;
      for (int d = 0; d < 3; ++d) v[(3 * k + d) * n + p] = V[3 * (int64_t)a + d];
    }
  }
}
void launch_tri_sorted(const double* V, const int32_t* Tri, const int32_t* perm, int64_t n,
                       double* v, int32_t* vid, hipStream_t s) {
  k_tri_sorted<<<grid_for(n, kT), kT, 0, s>>>(V, Tri, perm, n, v, vid);
  HM_LAUNCH_CHECK();
}

// Largest centroid-to-vertex distance (squared, as the bits of a
// non-negative double, which order like the values).
__global__ void k_tri_reach(const double* __restrict__ c, const double* __restrict__ tv, int64_t n,
                            unsigned long long* __restrict__ out) {
  double r2 = 0.0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    for (int k = 0; k < 3; ++k) {
      double d2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double e = tv[(3 * k + d) * n + p] - c[d * n + p];
        d2 += e * e;
      }
      r2 = fmax(r2, d2);
    }
  atomicMax(out, (unsigned long long)__double_as_longlong(r2));
}

// (vertex, position) pairs of every triangle corner.
__global__ void k_corner_pairs(const int32_t* __restrict__ vid, int64_t n,
                               uint64_t* __restrict__ key, int32_t* __restrict__ pos) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 3 * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    key[e] = (uint64_t)(uint32_t)vid[e];
    pos[e] = (int32_t)(e % n);
  }
}

// vbeg[v] = first sorted entry with key >= v, for v = 0..nv.
__global__ void k_vertex_begins(const uint64_t* __restrict__ key, int64_t ne, int64_t nv,
                                int32_t* __restrict__ vbeg) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e <= ne;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lo = e == 0 ? 0 : (int64_t)key[e - 1] + 1;
    const int64_t hi = e == ne ? nv : (int64_t)key[e];
    for (int64_t v = lo; v <= hi; ++v) vbeg[v] = (int32_t)e;
  }
}

GalTouch make_gal_touch(const double* c, const double* tv, const int32_t* vid, int64_t n,
                        int64_t nv, hipStream_t s) {
  if (3 * n >= INT32_MAX) throw Error{HM_ERR_STATE, "too many triangle corners"};
  GalTouch t;
  t.vid = vid;
  t.n = n;
  unsigned long long* r = dalloc_t<unsigned long long>(1, s);
  HM_HIP(hipMemsetAsync(r, 0, sizeof(unsigned long long), s));
  k_tri_reach<<<std::min<unsigned>(grid_for(n, kT), 1024), kT, 0, s>>>(c, tv, n, r);
  HM_LAUNCH_CHECK();
  uint64_t* key = dalloc_t<uint64_t>(3 * n, s);
  t.vpos = dalloc_t<int32_t>(3 * n, s);
  t.vbeg = dalloc_t<int32_t>(nv + 1, s);
  k_corner_pairs<<<grid_for(3 * n, kT), kT, 0, s>>>(vid, n, key, t.vpos);
  HM_LAUNCH_CHECK();
  int bits = 1;
  while ((int64_t(1) << bits) < nv) ++bits;
  radix_sort_u64_i32(key, t.vpos, 3 * n, bits, s);
  k_vertex_begins<<<grid_for(3 * n + 1, kT), kT, 0, s>>>(key, 3 * n, nv, t.vbeg);
  HM_LAUNCH_CHECK();
  unsigned long long rb = 0;
  HM_HIP(hipMemcpyAsync(&rb, r, sizeof(rb), hipMemcpyDeviceToHost, s));
  HM_HIP(hipStreamSynchronize(s));
  dfree(key, s);
  dfree(r, s);
  double r2 = 0.0;
  std::memcpy(&r2, &rb, sizeof(r2));
  // the centroids of two touching triangles are at most 2 r_max apart; the
  // margin covers the rounding of the boxes
  t.reach2 = 4.0 * r2 * (1.0 + 1e-9);
  return t;
}

void free_gal_touch(GalTouch& t, hipStream_t s) {
  if (t.vbeg) dfree(t.vbeg, s);
  if (t.vpos) dfree(t.vpos, s);
  t = GalTouch{};
}

// Builds the CBC tree level by level on the device.  Returns the number of
// clusters; level_beg receives the first cluster of every level (plus end).
int64_t build_cluster_tree(const std::vector<int64_t>& goff, int leaf, Cluster* cl, int64_t cap,
                           std::vector<int64_t>& level_beg, hipStream_t s) {
  // one root per geometry, [goff[g], goff[g + 1]), all at level 0
  const int64_t G = (int64_t)goff.size() - 1;
  std::vector<Cluster> roots(G);
  for (int64_t g = 0; g < G; ++g) roots[g] = make_int4((int)goff[g], (int)goff[g + 1], -1, 0);
  if (G > cap) throw Error{HM_ERR_STATE, "cluster capacity exceeded"};
  HM_HIP(hipMemcpyAsync(cl, roots.data(), G * sizeof(Cluster), hipMemcpyHostToDevice, s));
  HM_HIP(hipStreamSynchronize(s));
  level_beg.assign(1, 0);
  int64_t beg = 0, cnt = G;
  int64_t* flag = dalloc_t<int64_t>(cap, s);
  int64_t* off = dalloc_t<int64_t>(cap, s);
  int64_t* tot = dalloc_t<int64_t>(1, s);
  while (cnt > 0) {
    level_beg.push_back(beg + cnt);
    k_cluster_flags<<<grid_for(cnt, kT), kT, 0, s>>>(cl, beg, cnt, leaf, flag);
    HM_LAUNCH_CHECK();
    scan_excl_i64(flag, off, cnt, tot, s);
    const int64_t nsplit = d2h_i64(tot, s);
    if (nsplit == 0) break;
    if (beg + cnt + 2 * nsplit > cap) throw Error{HM_ERR_STATE, "cluster capacity exceeded"};
    k_cluster_emit<<<grid_for(cnt, kT), kT, 0, s>>>(cl, beg, cnt, flag, off, beg + cnt);
    HM_LAUNCH_CHECK();
    beg += cnt;
    cnt = 2 * nsplit;
  }
  dfree(flag, s);
  dfree(off, s);
  dfree(tot, s);
  return level_beg.back();
}

void launch_leaf_marks(const Cluster* cl, int64_t ncl, int64_t* mark, hipStream_t s) {
  k_leaf_marks<<<grid_for(ncl, kT), kT, 0, s>>>(cl, ncl, mark);
  HM_LAUNCH_CHECK();
}
void launch_pos_leaf(const int64_t* mark, const int64_t* excl, int64_t n, int32_t* pos_leaf,
                     hipStream_t s) {
  k_pos_leaf<<<grid_for(n, kT), kT, 0, s>>>(mark, excl, n, pos_leaf);
  HM_LAUNCH_CHECK();
}
void launch_leaf_table(const Cluster* cl, int64_t ncl, const int32_t* pos_leaf, int32_t* leaf_lo,
                       int32_t* leaf_m, int32_t* leaf_cl, int64_t* leaf_ld, int2* cl_leaves,
                       hipStream_t s) {
  k_leaf_table<<<grid_for(ncl, kT), kT, 0, s>>>(cl, ncl, pos_leaf, leaf_lo, leaf_m, leaf_cl,
                                                leaf_ld, cl_leaves);
  HM_LAUNCH_CHECK();
}
void launch_boxes(const Cluster* cl, const std::vector<int64_t>& level_beg, const int32_t* leaf_cl,
                  int64_t nleaf, const double* c, int64_t n, double* box, hipStream_t s) {
  k_leaf_boxes<<<grid_for(nleaf, 64), 64, 0, s>>>(cl, leaf_cl, nleaf, c, n, box);
  HM_LAUNCH_CHECK();
  for (int64_t L = (int64_t)level_beg.size() - 2; L >= 0; --L) {
    const int64_t beg = level_beg[L], cnt = level_beg[L + 1] - level_beg[L];
    if (cnt <= 0) continue;
    k_parent_boxes<<<grid_for(cnt, kT), kT, 0, s>>>(cl, beg, cnt, box);
    HM_LAUNCH_CHECK();
  }
}

// Level-wise Algorithm 1, started from the root pair of every geometry.
// Returns the admissible and dense leaf lists (device, owned by the caller)
// in level order.
void build_block_tree(const Cluster* cl, int64_t nroots, const double* box, double eta, int leaf,
                      const GalTouch& gt, int2** adm_out, int64_t* nadm, int2** dns_out,
                      int64_t* ndns, int64_t* depth, hipStream_t s) {
  std::vector<std::pair<int2*, int64_t>> adm_lv, dns_lv;
  // traversal from (root_g, root_g) of every geometry: geometries never
  // interact, so the operator is block diagonal over them
  int2* cand = dalloc_t<int2>(nroots, s);
  std::vector<int2> rp(nroots);
  for (int64_t g = 0; g < nroots; ++g) rp[g] = make_int2((int)g, (int)g);
  HM_HIP(hipMemcpyAsync(cand, rp.data(), nroots * sizeof(int2), hipMemcpyHostToDevice, s));
  HM_HIP(hipStreamSynchronize(s));
  int64_t ncand = nroots;
  const double eta2 = eta * eta;
  int64_t* tot = dalloc_t<int64_t>(1, s);
  int64_t lv = 0;
  while (ncand > 0) {
    // the packed scan keeps each count in 32 bits
    if (ncand >= (int64_t(1) << 32)) throw Error{HM_ERR_STATE, "block tree level too large"};
    int64_t* f = dalloc_t<int64_t>(2 * ncand, s);
    int64_t* off = f + ncand;
    k_classify<<<grid_for(ncand, kT), kT, 0, s>>>(cand, ncand, cl, box, eta2, leaf, gt, f);
    HM_LAUNCH_CHECK();
    scan_excl_i64(f, off, ncand, tot, s);
    const int64_t packed = d2h_i64(tot, s);
    int64_t h[3];
    h[0] = packed & 0xffffffffLL;                       // admissible
    h[1] = packed >> 32;                                // dense leaves
    h[2] = ncand - h[0] - h[1];                         // split
    int2* a = dalloc_t<int2>(h[0], s);
    int2* d = dalloc_t<int2>(h[1], s);
    int2* nx = dalloc_t<int2>(4 * h[2], s);
    k_emit<<<grid_for(ncand, kT), kT, 0, s>>>(cand, ncand, cl, f, off, a, d, nx);
    HM_LAUNCH_CHECK();
    adm_lv.push_back({a, h[0]});
    dns_lv.push_back({d, h[1]});
    dfree(f, s);
    dfree(cand, s);
    cand = nx;
    ncand = 4 * h[2];
    ++lv;
  }
  dfree(cand, s);
  dfree(tot, s);
  auto concat = [&](std::vector<std::pair<int2*, int64_t>>& parts, int2** out, int64_t* cnt) {
    int64_t tot_n = 0;
    for (auto& p : parts) tot_n += p.second;
    *out = dalloc_t<int2>(tot_n, s);
    int64_t o = 0;
    for (auto& p : parts) {
      if (p.second)
        HM_HIP(hipMemcpyAsync(*out + o, p.first, p.second * sizeof(int2),
                              hipMemcpyDeviceToDevice, s));
      o += p.second;
      dfree(p.first, s);
    }
    *cnt = tot_n;
  };
  concat(adm_lv, adm_out, nadm);
  concat(dns_lv, dns_out, ndns);
  *depth = lv;
}

}  // namespace hm
