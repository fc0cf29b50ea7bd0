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
#include <chrono>
#include <cmath>
#include <type_traits>

#include "hm_internal.h"

namespace hm {

// ------------------------------------------------------------------ entries
// Source triangle j: centroid, vertex offsets d_k = v_k - c (the nodes of
// the rule are c and c + beta d_k), |T_j| / (4 pi) and the self-term.
template <typename T>
struct Src {
  double cx, cy, cz;
  T dx[kNV], dy[kNV], dz[kNV];
  T aw, sf;
};

// base[k] at a byte offset of 32 bits from a wavefront-uniform base: the
// load then takes the base in scalar registers and one vector offset, with
// no 64-bit address arithmetic per load
template <typename T>
__device__ inline T ld_at(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ inline void st_at(T* base, uint32_t byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

template <typename T>
__device__ inline void load_src(const Geom<T>& g, int j, Src<T>& s) {
  s.cx = g.c[j];
  s.cy = g.c[g.n + j];
  s.cz = g.c[2 * g.n + j];
#pragma unroll
  for (int k = 0; k < kNV; ++k) {
    s.dx[k] = g.o[(int64_t)k * g.n + j];
    s.dy[k] = g.o[(int64_t)(kNV + k) * g.n + j];
    s.dz[k] = g.o[(int64_t)(2 * kNV + k) * g.n + j];
  }
  s.aw = g.aw[j];
  s.sf = g.sf[j];
}

// The same through uniform bases and one 32-bit offset: fewer vector
// instructions per entry, more scalar registers held (used where one
// column is loaded at a time)
template <typename T>
__device__ inline void load_src_u(const Geom<T>& g, int j, Src<T>& s) {
  const uint32_t bd = (uint32_t)j * 8u, bt = (uint32_t)j * (uint32_t)sizeof(T);
  s.cx = ld_at(g.c, bd);
  s.cy = ld_at(g.c + g.n, bd);
  s.cz = ld_at(g.c + 2 * g.n, bd);
#pragma unroll
  for (int k = 0; k < kNV; ++k) {
    s.dx[k] = ld_at(g.o + (int64_t)k * g.n, bt);
    s.dy[k] = ld_at(g.o + (int64_t)(kNV + k) * g.n, bt);
    s.dz[k] = ld_at(g.o + (int64_t)(2 * kNV + k) * g.n, bt);
  }
  s.aw = ld_at(g.aw, bt);
  s.sf = ld_at(g.sf, bt);
}

// The hardware reciprocal square root.  Its argument is the squared distance
// between a collocation point and a quadrature node of another triangle, far
// above the subnormal range for any mesh of distinct triangles; there the
// instruction gives the result of rsqrtf, whose extra steps only rescale
// subnormal arguments.
__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// In double: the device math library's reciprocal square root (a hardware
// estimate refined to double precision), one refinement sequence where
// 1.0 / sqrt(x) runs two (the square root's and the division's).  FP64
// setup at N = 1,310,720: near field 32 -> 18 ms, ACA 305 -> 271 ms; the
// Galerkin form, 49 of them per entry, 1.39 -> 0.88 s.
__device__ inline double rsq(double x) { return rsqrt(x); }

// sum_q w_q / |p - y_q| over the seven nodes of source s, with p the point
// minus the source's centroid: node 0 at offset 0, nodes 1..3 at beta1 d_k
// and 4..6 at beta2 d_k (k = 2, 1, 0: the vertex that carries weight b).
template <typename T>
__device__ inline T rule7(T px, T py, T pz, const Src<T>& s) {
  const T b1 = (T)Radon7::beta1, b2 = (T)Radon7::beta2;
  const T a0 = rsq(px * px + py * py + pz * pz);
  T a1 = 0, a2 = 0;
#pragma unroll
  for (int k = kNV - 1; k >= 0; --k) {
    const T ex = px - b1 * s.dx[k], ey = py - b1 * s.dy[k], ez = pz - b1 * s.dz[k];
    a1 += rsq(ex * ex + ey * ey + ez * ez);
  }
#pragma unroll
  for (int k = kNV - 1; k >= 0; --k) {
    const T ex = px - b2 * s.dx[k], ey = py - b2 * s.dy[k], ez = pz - b2 * s.dz[k];
    a2 += rsq(ex * ex + ey * ey + ez * ez);
  }
  return (T)Radon7::w0 * a0 + (T)Radon7::w1 * a1 + (T)Radon7::w2 * a2;
}

// a(i, j) = |T_j|/(4 pi) sum_q w_q / |x_i - y_jq| for i != j (seven-point
// Radon rule on the single-layer kernel of Sec. 2.1), the analytic self-term
// for i == j.  Positions i, j are Morton positions; (xi, yi, zi) = x_i.
template <typename T>
__device__ inline T eval_entry(double xi, double yi, double zi, int i, const Src<T>& s, int j) {
  if (i == j) return s.sf;
  const T dx = (T)(xi - s.cx), dy = (T)(yi - s.cy), dz = (T)(zi - s.cz);
  return rule7(dx, dy, dz, s) * s.aw;
}

// ---- wavefront primitives (gfx9 DPP).  The row-of-16 butterfly (quad
// permutes, half mirror, mirror) followed by the two row broadcasts leaves
// the full result in lane 63; readlane makes it uniform.  Masked rows of a
// DPP move read 0.
template <int CTRL, int ROWMASK>
__device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xF, false);
}
__device__ inline int rdl_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
template <int C, int RM>
__device__ inline float dpp_v(float v) {
  return __int_as_float(dpp_i<C, RM>(__float_as_int(v)));
}
template <int C, int RM>
__device__ inline double dpp_v(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)dpp_i<C, RM>((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_i<C, RM>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline float rdl_v(float v, int l) { return __int_as_float(rdl_i(__float_as_int(v), l)); }
__device__ inline double rdl_v(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)rdl_i((int)(unsigned)b, l);
  const unsigned hi = (unsigned)rdl_i((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the wavefront, uniform result, fixed order.
template <typename A>
__device__ inline A wsum(A v) {
  v += dpp_v<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_v<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp_v<0x141, 0xF>(v);   // row_half_mirror
  v += dpp_v<0x140, 0xF>(v);   // row_mirror
  v += dpp_v<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_v<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return rdl_v(v, 63);
}

// ---- row side of an entry.  Collocation: the collocation point x_i.
// Galerkin: the whole triangle T_i (centroid, node offsets, |T_i| / 4 pi).
template <typename T, int OP>
struct Tgt;
template <typename T>
struct Tgt<T, kOpColloc> {
  double x, y, z;
};
template <typename T>
struct Tgt<T, kOpGalerkin> {
  double x, y, z;
  T dx[kNV], dy[kNV], dz[kNV];     // vertex offsets, as in Src
  T aw;
};

// Row i = base + k, base wavefront-uniform (one 32-bit offset per load).
template <typename T>
__device__ inline void load_tgt(const Geom<T>& g, int base, int k, Tgt<T, kOpColloc>& t) {
  const uint32_t b8 = (uint32_t)k * 8u;
  t.x = ld_at(g.c + base, b8);
  t.y = ld_at(g.c + g.n + base, b8);
  t.z = ld_at(g.c + 2 * g.n + base, b8);
}
template <typename T>
__device__ inline void load_tgt(const Geom<T>& g, int base, int k, Tgt<T, kOpGalerkin>& t) {
  const uint32_t b8 = (uint32_t)k * 8u, bt = (uint32_t)k * (uint32_t)sizeof(T);
  t.x = ld_at(g.c + base, b8);
  t.y = ld_at(g.c + g.n + base, b8);
  t.z = ld_at(g.c + 2 * g.n + base, b8);
#pragma unroll
  for (int k = 0; k < kNV; ++k) {
    t.dx[k] = ld_at(g.o + (int64_t)k * g.n + base, bt);
    t.dy[k] = ld_at(g.o + (int64_t)(kNV + k) * g.n + base, bt);
    t.dz[k] = ld_at(g.o + (int64_t)(2 * kNV + k) * g.n + base, bt);
  }
  t.aw = ld_at(g.aw + base, bt);
}

// Galerkin entry of two triangles that share no vertex:
// |T_i| |T_j| / (4 pi) sum_p w_p sum_q w_q / |x_ip - y_jq| (Radon's rule on
// both triangles, Sec. 2.2), the centroid difference in double.
template <typename T>
__device__ inline T eval_far_g(const Tgt<T, kOpGalerkin>& t, const Src<T>& s) {
  const T dx = (T)(t.x - s.cx), dy = (T)(t.y - s.cy), dz = (T)(t.z - s.cz);
  const T b1 = (T)Radon7::beta1, b2 = (T)Radon7::beta2;
  // outer nodes of T_i in the same order as the inner ones
  const T o0 = rule7(dx, dy, dz, s);
  T o1 = 0, o2 = 0;
#pragma unroll
  for (int k = kNV - 1; k >= 0; --k)
    o1 += rule7(dx + b1 * t.dx[k], dy + b1 * t.dy[k], dz + b1 * t.dz[k], s);
#pragma unroll
  for (int k = kNV - 1; k >= 0; --k)
    o2 += rule7(dx + b2 * t.dx[k], dy + b2 * t.dy[k], dz + b2 * t.dz[k], s);
  const T sum = (T)Radon7::w0 * o0 + (T)Radon7::w1 * o1 + (T)Radon7::w2 * o2;
  return sum * (t.aw * s.aw) * (T)12.566370614359172954;   // |T_i||T_j|/(4 pi) = 4 pi aw_i aw_j
}

// Entry of row t (position i) and source s (position j).  Galerkin pairs
// that touch are not evaluated here (see galerkin_singular); they never lie
// in an admissible block, so the ACA meets only this form.
template <typename T>
__device__ inline T op_entry(const Tgt<T, kOpColloc>& t, int i, const Src<T>& s, int j) {
  return eval_entry(t.x, t.y, t.z, i, s, j);
}
template <typename T>
__device__ inline T op_entry(const Tgt<T, kOpGalerkin>& t, int i, const Src<T>& s, int j) {
  (void)i;
  (void)j;
  return eval_far_g(t, s);
}

// ---- singular Galerkin entries (Sec. 4.1: higher-order quadrature and the
// Duffy trick), in double.
// int_T dsigma_y / |x - y| for the flat triangle T with vertices v[0..2]
// and any point x: T is the signed sum of the triangles (x', a, b) over its
// edges, x' the projection of x onto the plane of T at signed height d; in
// polar coordinates about x' every edge gives, between its end points,
// h asinh(l / c) + |d| atan(|d| l / (h R)) - |d| atan(l / h)
// (h distance of x' to the edge line, l coordinate along it, c^2 = h^2 + d^2,
// R distance from x to the end point).  Evaluated here in an equivalent
// form with one logarithm and two arc tangents per edge:
//   asinh(l_b / c) - asinh(l_a / c) = log((l_b + R_b) / (l_a + R_a))  (l_a >= 0),
//   = log((|l_a| + R_a) / (|l_b| + R_b)) (l_b <= 0), and
//   log((l_b + R_b)(|l_a| + R_a) / c^2) when the edge spans the foot point
//   (R^2 = l^2 + c^2; no cancellation in any case);
//   atan(|d| l / (h R)) - atan(l / h) = atan(z),
//   z = -l h (l^2 + h^2) / ((R + |d|)(h^2 R + |d| l^2))
//   (the two arguments have a non-negative product, and R - |d| is written
//   as (l^2 + h^2) / (R + |d|)).
// What depends only on T -- its unit normal, the unit edge tangents t_k,
// the in-plane edge normals m_k = t_k x n and the edge lengths -- is set up
// once per pair.
struct TriJ {
  double v[3][3], n[3], t[3][3], m[3][3], le[3];
};

__device__ inline void tri_setup(const double v[3][3], TriJ& J) {
  double e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    e1[k] = v[1][k] - v[0][k];
    e2[k] = v[2][k] - v[0][k];
    for (int c = 0; c < 3; ++c) J.v[k][c] = v[k][c];
  }
  double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                 e1[0] * e2[1] - e1[1] * e2[0]};
  const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int c = 0; c < 3; ++c) J.n[c] = n[c] / nn;
  for (int k = 0; k < 3; ++k) {
    const double* a = v[k];
    const double* b = v[(k + 1) % 3];
    double e[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double le = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    J.le[k] = le;
    for (int c = 0; c < 3; ++c) J.t[k][c] = e[c] / le;
    J.m[k][0] = J.t[k][1] * J.n[2] - J.t[k][2] * J.n[1];
    J.m[k][1] = J.t[k][2] * J.n[0] - J.t[k][0] * J.n[2];
    J.m[k][2] = J.t[k][0] * J.n[1] - J.t[k][1] * J.n[0];
  }
}

__device__ inline double tri_inner_integral(const double x[3], const TriJ& J) {
  const double d = (x[0] - J.v[0][0]) * J.n[0] + (x[1] - J.v[0][1]) * J.n[1] +
                   (x[2] - J.v[0][2]) * J.n[2];
  const double ad = fabs(d);
  double R[3];
  for (int k = 0; k < 3; ++k) {
    const double dx = x[0] - J.v[k][0], dy = x[1] - J.v[k][1], dz = x[2] - J.v[k][2];
    R[k] = sqrt(dx * dx + dy * dy + dz * dz);
  }
  double total = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double ax = J.v[k][0] - x[0], ay = J.v[k][1] - x[1], az = J.v[k][2] - x[2];
    // signed distance of x' to the edge line (positive: x' on the inner side)
    const double hs = ax * J.m[k][0] + ay * J.m[k][1] + az * J.m[k][2];
    const double h = fabs(hs);
    if (!(h > 0.0)) continue;                            // x' on the edge line
    const double la = ax * J.t[k][0] + ay * J.t[k][1] + az * J.t[k][2];
    const double lb = la + J.le[k];
    const double Ra = R[k], Rb = R[(k + 1) % 3];
    double lg;
    if (la >= 0.0)
      lg = log((lb + Rb) / (la + Ra));
    else if (lb <= 0.0)
      lg = log((Ra - la) / (Rb - lb));
    else
      lg = log((lb + Rb) * (Ra - la) / (h * h + d * d));
    double val = h * lg;
    if (ad > 0.0) {
      const double h2 = h * h;
      const double za = -la * h * (la * la + h2) / ((Ra + ad) * (h2 * Ra + ad * la * la));
      const double zb = -lb * h * (lb * lb + h2) / ((Rb + ad) * (h2 * Rb + ad * lb * lb));
      val += ad * (atan(zb) - atan(za));
    }
    total += hs > 0.0 ? val : -val;
  }
  return total;
}

template <typename T>
__device__ inline void load_tri(const Geom<T>& g, int i, double v[3][3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[k][c] = g.v[(int64_t)(3 * k + c) * g.n + i];
}

// a_ij of touching triangles: kGalQ x kGalQ Gauss points on T_i in collapsed coordinates
// x = v0 + s (v1 - v0) + s t (v2 - v1), weight w_s w_t s |(v1 - v0) x (v2 - v1)|,
// the inner integral over T_j in closed form.
template <typename T>
__device__ inline double galerkin_singular_part(const Geom<T>& g, const GaussRule& R, int i, int j,
                                                int k0, int step) {
  double ti[3][3], tj[3][3];
  load_tri(g, i, ti);
  load_tri(g, j, tj);
  TriJ J;
  tri_setup(tj, J);
  double a[3], b[3];
  for (int c = 0; c < 3; ++c) {
    a[c] = ti[1][c] - ti[0][c];
    b[c] = ti[2][c] - ti[1][c];
  }
  const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2],
               cz = a[0] * b[1] - a[1] * b[0];
  const double jac = sqrt(cx * cx + cy * cy + cz * cz);
  double acc = 0.0;
  for (int k = k0; k < kGalQ * kGalQ; k += step) {
    const int ks = k / kGalQ, kt = k % kGalQ;
    const double s = R.x[ks], t = R.x[kt];
    double x[3];
    for (int c = 0; c < 3; ++c) x[c] = ti[0][c] + s * a[c] + s * t * b[c];
    acc += R.w[ks] * R.w[kt] * s * jac * tri_inner_integral(x, J);
  }
  return acc * 0.079577471545947667884441881686257181;   // 1/(4 pi)
}
template <typename T>
__device__ inline double galerkin_singular(const Geom<T>& g, const GaussRule& R, int i, int j) {
  return wsum(galerkin_singular_part(g, R, i, j, threadIdx.x & 63, 64));
}


// Do triangles i and j share a vertex (or coincide)?
template <typename T>
__device__ inline bool touching(const Geom<T>& g, int i, int j) {
  if (i == j) return true;
  const int32_t a0 = g.vid[i], a1 = g.vid[g.n + i], a2 = g.vid[2 * g.n + i];
  const int32_t b0 = g.vid[j], b1 = g.vid[g.n + j], b2 = g.vid[2 * g.n + j];
  return a0 == b0 || a0 == b1 || a0 == b2 || a1 == b0 || a1 == b1 || a1 == b2 || a2 == b0 ||
         a2 == b1 || a2 == b2;
}

// Entries at arbitrary (application) index pairs, for checking: one
// wavefront per pair (the singular Galerkin entries sum over its lanes).
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_entries(Geom<T> g, GaussRule R,
                                                 const int32_t* __restrict__ inv_perm,
                                                 const int32_t* __restrict__ rows,
                                                 const int32_t* __restrict__ cols, int64_t cnt,
                                                 double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  for (int64_t k = blockIdx.x * 4 + (threadIdx.x >> 6); k < cnt; k += (int64_t)gridDim.x * 4) {
    const int i = inv_perm[rows[k]], j = inv_perm[cols[k]];
    double v;
    if (OP == kOpGalerkin && touching(g, i, j)) {
      v = galerkin_singular(g, R, i, j);
    } else {
      Tgt<T, OP> t;
      load_tgt(g, i, 0, t);
      Src<T> s;
      load_src(g, j, s);
      v = (double)op_entry(t, i, s, j);
    }
    if (lane == 0) out[k] = v;
  }
}

__global__ void k_inverse_perm(const int32_t* __restrict__ perm, int64_t n,
                               int32_t* __restrict__ inv) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    inv[perm[p]] = (int32_t)p;
}

// ------------------------------------------------------------------ near field
// Dense leaves of Algorithm 1, assembled in one batch (Sec. 3.3): one
// workgroup per (dense block, row leaf) slice, written straight into the row
// leaf's panel (ld x n, column-major, zero padding rows).
struct LeafTab {
  const int32_t* lo;     // first position of leaf
  const int32_t* m;      // size
  const int64_t* ldpre;  // prefix of ld over leaves (nleaf + 1 entries)
  const int2* cl_leaves; // per cluster: first and last leaf
};

__device__ inline int leaf_ld(const LeafTab& L, int lf) {
  return (int)(L.ldpre[lf + 1] - L.ldpre[lf]);
}

template <typename T, int OP>
__global__ __launch_bounds__(256) void k_near(Geom<T> g, const int32_t* __restrict__ sidx,
                                              const int32_t* __restrict__ ib,
                                              const int32_t* __restrict__ ilf, int64_t np,
                                              const int2* __restrict__ dns,
                                              const Cluster* __restrict__ cl, LeafTab L,
                                              const int64_t* __restrict__ offI, T* __restrict__ D) {
  // the slice's source triangles (columns, at most a leaf) and rows are
  // staged in LDS once; entries read them from there.  Galerkin pairs that
  // touch get 0 here and their value from k_near_singular.
  constexpr bool GAL = OP == kOpGalerkin;
  __shared__ Src<T> src[kMaxLeaf];
  __shared__ Tgt<T, OP> tr[kMaxLeaf];
  __shared__ int32_t vr[GAL ? 3 : 1][kMaxLeaf], vc[GAL ? 3 : 1][kMaxLeaf];
  for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
    const int32_t u = sidx[p];
    const int b = ib[u], lf = ilf[u];
    const Cluster sig = cl[dns[b].y];
    const int n = sig.y - sig.x;
    const int ld = leaf_ld(L, lf), m = L.m[lf], lo = L.lo[lf];
    T* dst = D + offI[p];
    if (n <= kMaxLeaf) {                                // dense blocks are leaf pairs
      for (int j = threadIdx.x; j < n; j += blockDim.x) {
        load_src_u(g, sig.x + j, src[j]);
        if (GAL)
          for (int k = 0; k < 3; ++k) vc[k][j] = g.vid[(int64_t)k * g.n + sig.x + j];
      }
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        load_tgt(g, lo, i, tr[i]);
        if (GAL)
          for (int k = 0; k < 3; ++k) vr[k][i] = g.vid[(int64_t)k * g.n + lo + i];
      }
      __syncthreads();
      // entry e = i + ld j; (i, j) advance by a fixed step instead of a
      // division per entry
      const int di = (int)blockDim.x % ld, dj = (int)blockDim.x / ld;
      int i = (int)threadIdx.x % ld, j = (int)threadIdx.x / ld;
      for (int e = threadIdx.x; e < ld * n; e += blockDim.x) {
        T v = 0;
        if (i < m) {
          bool skip = false;
          if (GAL) {
            skip = lo + i == sig.x + j;
            for (int a = 0; a < 3; ++a)
              for (int c = 0; c < 3; ++c) skip = skip || vr[a][i] == vc[c][j];
          }
          if (!skip) {
            const Src<T> sj = src[j];
            v = op_entry(tr[i], lo + i, sj, sig.x + j);
          }
        }
        dst[e] = v;
        i += di;
        j += dj;
        if (i >= ld) {
          i -= ld;
          ++j;
        }
      }
      __syncthreads();                                  // before the next slice is staged
    } else {
      for (int e = threadIdx.x; e < ld * n; e += blockDim.x) {
        const int i = e % ld, j = e / ld;
        T v = 0;
        if (i < m && !(GAL && touching(g, lo + i, sig.x + j))) {
          Tgt<T, OP> t;
          load_tgt(g, lo, i, t);
          Src<T> sj;
          load_src(g, sig.x + j, sj);
          v = op_entry(t, lo + i, sj, sig.x + j);
        }
        dst[e] = v;
      }
    }
  }
}

// Singular Galerkin entries of the near field (pairs that share a vertex,
// left at 0 by k_near): one workgroup per slice as in k_near.  Every
// wavefront looks at 64 consecutive entries at a time and evaluates the
// touching ones among them one after the other, all its lanes together
// (the trip count of its loop is the same for all lanes).
template <typename T>
__global__ __launch_bounds__(256) void k_near_singular(Geom<T> g, GaussRule R,
                                                       const int32_t* __restrict__ sidx,
                                                       const int32_t* __restrict__ ib,
                                                       const int32_t* __restrict__ ilf, int64_t np,
                                                       const int2* __restrict__ dns,
                                                       const Cluster* __restrict__ cl, LeafTab L,
                                                       const int64_t* __restrict__ offI,
                                                       T* __restrict__ D) {
  __shared__ int32_t vr[3][kMaxLeaf], vc[3][kMaxLeaf];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
    const int32_t u = sidx[p];
    const int b = ib[u], lf = ilf[u];
    const Cluster sig = cl[dns[b].y];
    const int n = sig.y - sig.x;
    const int ld = leaf_ld(L, lf), m = L.m[lf], lo = L.lo[lf];
    T* dst = D + offI[p];
    const bool staged = n <= kMaxLeaf;
    if (staged) {
      for (int j = threadIdx.x; j < n; j += blockDim.x)
        for (int k = 0; k < 3; ++k) vc[k][j] = g.vid[(int64_t)k * g.n + sig.x + j];
      for (int i = threadIdx.x; i < m; i += blockDim.x)
        for (int k = 0; k < 3; ++k) vr[k][i] = g.vid[(int64_t)k * g.n + lo + i];
    }
    __syncthreads();
    for (int e0 = wave * 64; e0 < ld * n; e0 += blockDim.x) {
      const int e = e0 + lane;
      const int i = e % ld, j = e / ld;
      bool t = false;
      if (e < ld * n && i < m) {
        if (staged) {
          t = lo + i == sig.x + j;
          for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) t = t || vr[a][i] == vc[c][j];
        } else {
          t = touching(g, lo + i, sig.x + j);
        }
      }
      unsigned long long mask = __ballot(t);
      while (mask) {
        const int l = __ffsll(mask) - 1;
        mask &= mask - 1;
        const int el = e0 + l;
        const double v = galerkin_singular(g, R, lo + el % ld, sig.x + el / ld);
        if (lane == 0) dst[el] = (T)v;
      }
    }
    __syncthreads();                                  // before the next slice is staged
  }
}

// ------------------------------------------------------------------ ACA
// Values that are equal in every lane, moved to scalar registers, so that
// the compiler sees the branches on them as uniform.  The workgroup ACA and
// the work queue branch only on such values: a barrier then never sits in
// control flow that the compiler treats as divergent (it may otherwise let
// some lanes run ahead to a barrier while others still hold pending work).
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float uni(float v) { return __int_as_float(uni(__float_as_int(v))); }
__device__ inline double uni(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)uni((int)(unsigned)b), hi = (unsigned)uni((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Pivot search: key = bit pattern of |value| (monotone for non-negative
// floats), larger key wins, ties go to the smaller index (stored as ~index,
// larger wins).  {0, 0} is the "no candidate" sentinel and loses to every
// real candidate, including a zero value.
struct Piv {
  unsigned long long k;
  unsigned ni;
};
__device__ inline unsigned long long key_bits(float a) { return (unsigned)__float_as_int(a); }
__device__ inline unsigned long long key_bits(double a) {
  return (unsigned long long)__double_as_longlong(a);
}
__device__ inline void piv_merge(Piv& a, unsigned long long k, unsigned ni) {
  if (k > a.k || (k == a.k && ni > a.ni)) {
    a.k = k;
    a.ni = ni;
  }
}
template <int C, int RM>
__device__ inline void piv_step(Piv& a) {
  const unsigned lo = (unsigned)dpp_i<C, RM>((int)(unsigned)a.k);
  const unsigned hi = (unsigned)dpp_i<C, RM>((int)(unsigned)(a.k >> 32));
  const unsigned ni = (unsigned)dpp_i<C, RM>((int)a.ni);
  piv_merge(a, ((unsigned long long)hi << 32) | lo, ni);
}
__device__ inline Piv wpiv(Piv a) {
  piv_step<0xB1, 0xF>(a);
  piv_step<0x4E, 0xF>(a);
  piv_step<0x141, 0xF>(a);
  piv_step<0x140, 0xF>(a);
  piv_step<0x142, 0xA>(a);
  piv_step<0x143, 0xC>(a);
  Piv r;
  r.k = ((unsigned long long)(unsigned)rdl_i((int)(unsigned)(a.k >> 32), 63) << 32) |
        (unsigned)rdl_i((int)(unsigned)a.k, 63);
  r.ni = (unsigned)rdl_i((int)a.ni, 63);
  return r;
}
// index of the winner, or -1 when there was no candidate
__device__ inline int piv_index(const Piv& p) {
  return (p.k == 0 && p.ni == 0) ? -1 : (int)(~p.ni);
}

// Kernel classes of the batched ACA: 0 one 1,024-thread workgroup per
// block, 1 one 256-thread workgroup, 2..4 one wavefront per block with
// Q = 4, 2, 1 rows and columns per lane (up to 256, 128, 64), 5 one
// 128-thread workgroup.  Each class is its own kernel (its own register
// allocation) and its own work queue; the size bins of the blocks are mapped
// to classes by an AcaBins table.
constexpr int kAcaClasses = 6;
constexpr int kAcaThreads = 256;
constexpr int kAcaWaves = kAcaThreads / 64;

// Working slot of a block: U column-major m x kc, then V n x kc, then m
// bytes of used-row flags (workgroup variant); kc = the block's rank cap in
// the pass that owns the slot.
struct AcaSlot {
  uint64_t ptr;
  int32_t kc;
  int32_t pad;
};

template <typename T>
struct AcaArgs {
  Geom<T> g;
  const int2* blk;       // (tau, sigma) of the chunk's blocks
  const Cluster* cl;
  const AcaSlot* slot;   // working slot of every block of the chunk
  const int32_t* list[kAcaClasses];  // block indices of each class, largest first
  int64_t cnt[kAcaClasses];
  int* head;             // queue position of each class (zero before the launches)
  int kmax;              // rank cap of this pass
  double eps;
  int32_t* rank;         // out: rank per block
  int32_t* info;         // out: bit 0 cap hit, bits 1.. number of row evaluations
};

// Stop test shared by both variants: keep term r, then stop when
// |u_r||v_r| <= eps |S_r|_F, or r reached the cap, or every row was used.
__device__ inline bool aca_stop(double uu, double vv, double s2, double eps) {
  return sqrt(uu) * sqrt(vv) <= eps * sqrt(fmax(s2, 0.0));
}

template <typename X, int Q>
__device__ inline X pick(const X (&a)[Q], int q) {
  X v = a[0];
#pragma unroll
  for (int k = 1; k < Q; ++k)
    if (q == k) v = a[k];
  return v;
}

// One block per wavefront (m, n <= 64 Q).  Lane L owns rows and columns
// L + 64 q, q < Q.  The working factors live in the block's slot: U
// column-major m x kcap, then V n x kcap; a lane only reads and writes its
// own rows / columns of them, other lanes' values arrive by readlane.

template <typename T, int Q, int OP>
__device__ void aca_wave(const AcaArgs<T>& A, int b) {
  constexpr int KB = Q == 4 ? 4 : 8;   // previous terms per batch of loads
  const int lane = threadIdx.x & 63;
  const int2 ts = A.blk[b];
  const Cluster tau = A.cl[ts.x], sig = A.cl[ts.y];
  const int r0 = tau.x, m = tau.y - tau.x, c0 = sig.x, n = sig.y - sig.x;
  const int kcap = min(A.kmax, min(m, n));
  T* U = reinterpret_cast<T*>((uintptr_t)A.slot[b].ptr);
  T* V = U + (int64_t)kcap * m;
  const Geom<T>& g = A.g;
  bool hr[Q], hc[Q], used[Q];
  double px[Q], py[Q], pz[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = lane + 64 * q;
    hr[q] = i < m;
    hc[q] = i < n;
    used[q] = false;
    px[q] = hr[q] ? g.c[r0 + i] : 0.0;
    py[q] = hr[q] ? g.c[g.n + r0 + i] : 0.0;
    pz[q] = hr[q] ? g.c[2 * g.n + r0 + i] : 0.0;
  }
  int nused = 0, r = 0, istar = 0, rows_eval = 0;
  double s2 = 0.0;
  bool cap_hit = false;
  while (true) {
    const int iq = istar >> 6, il = istar & 63;
    Tgt<T, OP> ti;
    if constexpr (OP == kOpColloc)
      ti = Tgt<T, OP>{rdl_v(pick(px, iq), il), rdl_v(pick(py, iq), il), rdl_v(pick(pz, iq), il)};
    else
      load_tgt(g, r0 + istar, 0, ti);
    // residual row  v~ = a(i*, :) - sum_l u_l[i*] v_l
    T val[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      val[q] = 0;
      if (hc[q]) {
        Src<T> s;
        load_src(g, c0 + lane + 64 * q, s);
        val[q] = op_entry(ti, r0 + istar, s, c0 + lane + 64 * q);
      }
    }
    // the previous terms KB at a time: their loads are issued together (an
    // index past r - 1 reads term r - 1 and is not used)
    const bool ownr = lane + 64 * iq < m;
    for (int l0 = 0; l0 < r; l0 += KB) {
      T ub[KB], vb[KB][Q];
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int l = min(l0 + k, r - 1);
        ub[k] = ownr ? U[(int64_t)l * m + lane + 64 * iq] : (T)0;
#pragma unroll
        for (int q = 0; q < Q; ++q) vb[k][q] = hc[q] ? V[(int64_t)l * n + lane + 64 * q] : (T)0;
      }
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (l0 + k < r) {
          const T ui = rdl_v(ub[k], il);
#pragma unroll
          for (int q = 0; q < Q; ++q)
            if (hc[q]) val[q] -= ui * vb[k][q];
        }
      }
    }
    ++rows_eval;
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (q == iq && lane == il) used[q] = true;
    ++nused;
    Piv pv{0, 0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (hc[q]) piv_merge(pv, key_bits((T)fabs(val[q])), ~(unsigned)(lane + 64 * q));
    const int jstar = piv_index(wpiv(pv));
    T delta = 0;
    if (jstar >= 0 && jstar < n) delta = rdl_v(pick(val, jstar >> 6), jstar & 63);
    if (delta == (T)0) {
      if (nused >= m) break;
      Piv nx{0, 0};
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (hr[q] && !used[q]) {
          const T k = (r > 0) ? (T)fabs(U[(int64_t)(r - 1) * m + lane + 64 * q]) : (T)0;
          piv_merge(nx, key_bits(k), ~(unsigned)(lane + 64 * q));
        }
      istar = piv_index(wpiv(nx));
      if (istar < 0 || istar >= m) break;
      continue;
    }
    T v[Q];
    double vv = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      v[q] = hc[q] ? val[q] / delta : (T)0;
      if (hc[q]) V[(int64_t)r * n + lane + 64 * q] = v[q];
      vv += (double)v[q] * (double)v[q];
    }
    // residual column  u = a(:, j*) - sum_l v_l[j*] u_l.  The cross terms of
    // |S_r|_F^2, sum_l (u_l . u)(v_l . v), equal u . w with w = sum_l u_l
    // (v_l . v), accumulated in the same pass over the previous terms.
    const int jq = jstar >> 6, jl = jstar & 63;
    Src<T> s;
    load_src(g, c0 + jstar, s);
    T u[Q];
    double wv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      u[q] = 0;
      if (hr[q]) {
        Tgt<T, OP> tq;
        if constexpr (OP == kOpColloc)
          tq = Tgt<T, OP>{px[q], py[q], pz[q]};
        else
          load_tgt(g, r0, lane + 64 * q, tq);
        u[q] = op_entry(tq, r0 + lane + 64 * q, s, c0 + jstar);
      }
      wv[q] = 0.0;
    }
    for (int l0 = 0; l0 < r; l0 += KB) {
      T vo[KB][Q], uo[KB][Q];
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int l = min(l0 + k, r - 1);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          vo[k][q] = hc[q] ? V[(int64_t)l * n + lane + 64 * q] : (T)0;
          uo[k][q] = hr[q] ? U[(int64_t)l * m + lane + 64 * q] : (T)0;
        }
      }
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (l0 + k < r) {
          double pvl = 0.0;
#pragma unroll
          for (int q = 0; q < Q; ++q) pvl += (double)vo[k][q] * (double)v[q];
          const T vj = rdl_v(pick(vo[k], jq), jl);
          const double dv = wsum(pvl);
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            u[q] -= vj * uo[k][q];
            wv[q] += dv * (double)uo[k][q];
          }
        }
      }
    }
    double uu = 0.0, cw = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (hr[q]) U[(int64_t)r * m + lane + 64 * q] = u[q];
      uu += (double)u[q] * (double)u[q];
      cw += (double)u[q] * wv[q];
    }
    const double cross = wsum(cw);
    uu = wsum(uu);
    vv = wsum(vv);
    s2 += 2.0 * cross + uu * vv;
    ++r;
    if (aca_stop(uu, vv, s2, A.eps)) break;
    if (r >= kcap) {
      cap_hit = kcap < min(m, n);
      break;
    }
    if (nused >= m) break;
    Piv nx{0, 0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (hr[q] && !used[q]) piv_merge(nx, key_bits((T)fabs(u[q])), ~(unsigned)(lane + 64 * q));
    istar = piv_index(wpiv(nx));
    if (istar < 0 || istar >= m) break;
  }
  if (lane == 0) {
    A.rank[b] = r;
    A.info[b] = (cap_hit ? 1 : 0) | (rows_eval << 1);
  }
}

// One block per workgroup of NT threads (blocks larger than the wavefront
// classes: NT = 256, and NT = 1024 for the largest blocks, whose sequential
// steps are the critical path of their chunk).  Cross-thread reads of the working factors happen only after a
// barrier.  The used-row flags are bytes placed after V in the slot.
template <typename T, int NT>
struct AcaShared {
  static constexpr int kW = NT / 64;
  T a[kMaxRank];             // u_l[i*] or v_l[j*] of the previous terms
  double dv[kMaxRank][kW];   // per-wave partial dots v_l . v_r
  double dt[kMaxRank];       // their totals
  Piv pv[kW];
  double red[3][kW];
  Piv pv_out;
  double out[3];
};

template <int NT>
__device__ inline Piv wg_piv(Piv a, Piv* lds, Piv* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  a = wpiv(a);
  if (lane == 0) lds[wave] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    Piv r = lds[0];
    for (int w = 1; w < (NT / 64); ++w) piv_merge(r, lds[w].k, lds[w].ni);
    *out = r;
  }
  __syncthreads();
  Piv r = *out;
  __syncthreads();
  return r;
}

// previous terms per batch of loads, and columns (rows) per thread at a
// time, in the workgroup variant
constexpr int kTermBatch = 8;
constexpr int kColUnroll = 1;

template <typename T, int NT, int OP>
__device__ void aca_wg(const AcaArgs<T>& A, int b, AcaShared<T, NT>& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int2 ts = A.blk[b];
  const Cluster tau = A.cl[ts.x], sig = A.cl[ts.y];
  const int r0 = tau.x, m = tau.y - tau.x, c0 = sig.x, n = sig.y - sig.x;
  const int kcap = min(A.kmax, min(m, n));
  T* U = reinterpret_cast<T*>((uintptr_t)A.slot[b].ptr);
  T* V = U + (int64_t)kcap * m;
  uint8_t* used = reinterpret_cast<uint8_t*>(V + (int64_t)kcap * n);
  const Geom<T>& g = A.g;
  for (int i = tid; i < m; i += NT) used[i] = 0;
  __syncthreads();
  int nused = 0, r = 0, istar = 0, rows_eval = 0;
  double s2 = 0.0;
  bool cap_hit = false;
  while (true) {
    if (tid < r) sh.a[tid] = U[(int64_t)tid * m + istar];
    __syncthreads();
    Tgt<T, OP> ti;
    if constexpr (OP == kOpColloc)
      ti = Tgt<T, OP>{g.c[r0 + istar], g.c[g.n + r0 + istar], g.c[2 * g.n + r0 + istar]};
    else
      load_tgt(g, r0 + istar, 0, ti);
    Piv pv{0, 0};
    // kColUnroll columns per thread at a time, so that their loads overlap
    // (indices past n - 1 are clamped and their results dropped)
    for (int j0 = tid; j0 < n; j0 += kColUnroll * NT) {
      Src<T> sj[kColUnroll];
      T val[kColUnroll];
      int jj[kColUnroll];
#pragma unroll
      for (int u = 0; u < kColUnroll; ++u) {
        jj[u] = min(j0 + u * NT, n - 1);
        load_src_u(g, c0 + jj[u], sj[u]);
      }
#pragma unroll
      for (int u = 0; u < kColUnroll; ++u)
        val[u] = op_entry(ti, r0 + istar, sj[u], c0 + jj[u]);
      for (int l0 = 0; l0 < r; l0 += kTermBatch) {
        T vb[kColUnroll][kTermBatch];
#pragma unroll
        for (int u = 0; u < kColUnroll; ++u)
#pragma unroll
          for (int k = 0; k < kTermBatch; ++k)
            vb[u][k] = ld_at(V + (int64_t)min(l0 + k, r - 1) * n, (uint32_t)jj[u] * (uint32_t)sizeof(T));
#pragma unroll
        for (int k = 0; k < kTermBatch; ++k)
          if (l0 + k < r)
#pragma unroll
            for (int u = 0; u < kColUnroll; ++u) val[u] -= sh.a[l0 + k] * vb[u][k];
      }
#pragma unroll
      for (int u = 0; u < kColUnroll; ++u) {
        if (j0 + u * NT < n) {
          V[(int64_t)r * n + jj[u]] = val[u];
          piv_merge(pv, key_bits((T)fabs(val[u])), ~(unsigned)jj[u]);
        }
      }
    }
    if (tid == 0) used[istar] = 1;
    ++rows_eval;
    ++nused;
    const int jstar = uni(piv_index(wg_piv<NT>(pv, sh.pv, &sh.pv_out)));
    // every thread may read V[r][j*] now (barriers in wg_piv)
    const T delta = uni((jstar >= 0 && jstar < n) ? V[(int64_t)r * n + jstar] : (T)0);
    // every thread holds delta before the owner of j* overwrites that entry
    __syncthreads();
    if (delta == (T)0) {
      if (nused >= m) break;
      Piv nx{0, 0};
      for (int i = tid; i < m; i += NT) {
        if (used[i]) continue;
        const T k = (r > 0) ? (T)fabs(U[(int64_t)(r - 1) * m + i]) : (T)0;
        piv_merge(nx, key_bits(k), ~(unsigned)i);
      }
      istar = uni(piv_index(wg_piv<NT>(nx, sh.pv, &sh.pv_out)));
      if (istar < 0 || istar >= m) break;
      continue;
    }
    // v_r = v~ / delta, then the dots v_l . v_r of the previous terms.  Each
    // thread reads back only the entries of v_r it wrote itself.
    double vv = 0.0;
    for (int j = tid; j < n; j += NT) {
      const T v = V[(int64_t)r * n + j] / delta;
      V[(int64_t)r * n + j] = v;
      vv += (double)v * (double)v;
    }
    for (int l0 = 0; l0 < r; l0 += kTermBatch) {
      double pvv[kTermBatch];
#pragma unroll
      for (int k = 0; k < kTermBatch; ++k) pvv[k] = 0.0;
      for (int j = tid; j < n; j += NT) {
        const uint32_t jb = (uint32_t)j * (uint32_t)sizeof(T);
        const double vr = (double)ld_at(V + (int64_t)r * n, jb);
        T vb[kTermBatch];
#pragma unroll
        for (int k = 0; k < kTermBatch; ++k) vb[k] = ld_at(V + (int64_t)min(l0 + k, r - 1) * n, jb);
#pragma unroll
        for (int k = 0; k < kTermBatch; ++k) pvv[k] += (double)vb[k] * vr;
      }
#pragma unroll
      for (int k = 0; k < kTermBatch; ++k) {
        if (l0 + k < r) {
          const double t = wsum(pvv[k]);
          if (lane == 0) sh.dv[l0 + k][wave] = t;
        }
      }
    }
    if (tid < r) sh.a[tid] = V[(int64_t)tid * n + jstar];
    __syncthreads();
    if (tid < r) {
      double t = 0.0;
      for (int w = 0; w < (NT / 64); ++w) t += sh.dv[tid][w];
      sh.dt[tid] = t;
    }
    __syncthreads();
    // residual column u_r; the cross terms sum_l (u_l . u_r)(v_l . v_r) are
    // u_r . w with w = sum_l (v_l . v_r) u_l, built in the same pass.
    Src<T> s;
    load_src(g, c0 + jstar, s);
    double uu = 0.0, cw = 0.0;
    Piv nx{0, 0};
    for (int i0 = tid; i0 < m; i0 += kColUnroll * NT) {
      T u[kColUnroll];
      double w[kColUnroll];
      int ii[kColUnroll];
#pragma unroll
      for (int q = 0; q < kColUnroll; ++q) {
        ii[q] = min(i0 + q * NT, m - 1);
        const int i = ii[q];
        Tgt<T, OP> tq;
        load_tgt(g, r0, i, tq);
        u[q] = op_entry(tq, r0 + i, s, c0 + jstar);
        w[q] = 0.0;
      }
      for (int l0 = 0; l0 < r; l0 += kTermBatch) {
        T ub[kColUnroll][kTermBatch];
#pragma unroll
        for (int q = 0; q < kColUnroll; ++q)
#pragma unroll
          for (int k = 0; k < kTermBatch; ++k)
            ub[q][k] = ld_at(U + (int64_t)min(l0 + k, r - 1) * m, (uint32_t)ii[q] * (uint32_t)sizeof(T));
#pragma unroll
        for (int k = 0; k < kTermBatch; ++k) {
          if (l0 + k < r) {
#pragma unroll
            for (int q = 0; q < kColUnroll; ++q) {
              u[q] -= sh.a[l0 + k] * ub[q][k];
              w[q] += sh.dt[l0 + k] * (double)ub[q][k];
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < kColUnroll; ++q) {
        if (i0 + q * NT < m) {
          const int i = ii[q];
          U[(int64_t)r * m + i] = u[q];
          uu += (double)u[q] * (double)u[q];
          cw += (double)u[q] * w[q];
          if (!used[i]) piv_merge(nx, key_bits((T)fabs(u[q])), ~(unsigned)i);
        }
      }
    }
    uu = wsum(uu);
    vv = wsum(vv);
    cw = wsum(cw);
    nx = wpiv(nx);
    if (lane == 0) {
      sh.red[0][wave] = uu;
      sh.red[1][wave] = vv;
      sh.red[2][wave] = cw;
      sh.pv[wave] = nx;
    }
    __syncthreads();
    if (tid == 0) {
      double tu = 0.0, tv = 0.0, tc = 0.0;
      Piv best = sh.pv[0];
      for (int w = 0; w < (NT / 64); ++w) {
        tu += sh.red[0][w];
        tv += sh.red[1][w];
        tc += sh.red[2][w];
        if (w) piv_merge(best, sh.pv[w].k, sh.pv[w].ni);
      }
      sh.out[0] = tu;
      sh.out[1] = tv;
      sh.out[2] = tc;
      sh.pv_out = best;
    }
    __syncthreads();
    uu = uni(sh.out[0]);
    vv = uni(sh.out[1]);
    const double cross = uni(sh.out[2]);
    const int inext = uni(piv_index(sh.pv_out));
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

// The batched ACA (Sec. 3.1, "Batching"): every class is one persistent
// launch over a work queue of its blocks, largest first, so that blocks of
// uneven size and rank are taken up by whichever workgroup or wavefront is
// free (the load imbalance of fixed assignments).  A workgroup or wavefront
// leaves when the queue position passes the last block.
//
// Classes 0 (NT = 1,024) and 1 (NT = 256): one block per workgroup.  One
// latch, no early continue: every block ends at the barrier below, so the
// thread that fetches the next position has finished the current block (its
// result stores included) before any thread reads the next position.
// Galerkin entries (49 kernel values each) hold the whole row triangle in
// registers: half the occupancy, no spills.
template <typename T, int NT, int CLS, int OP>
__global__ __launch_bounds__(NT, NT == 1024 ? 1 : (OP == kOpGalerkin ? 2 : 4)) void k_aca_wg(AcaArgs<T> A) {
  __shared__ AcaShared<T, NT> sh;
  __shared__ int item_sh;
  while (true) {
    if (threadIdx.x == 0) item_sh = atomicAdd(A.head + CLS, 1);
    __syncthreads();
    const int64_t it = uni(item_sh);
    if (it >= A.cnt[CLS]) break;
    aca_wg<T, NT, OP>(A, A.list[CLS][it], sh);
    __syncthreads();
  }
}

// Classes 2..4: one block per wavefront; every wavefront takes its own
// blocks from the queue, NB consecutive (similar) blocks per fetch for the
// small classes, which have millions of blocks (no barriers).  Galerkin
// entries hold the row triangle in registers: two waves per SIMD for one
// row per lane, one (with the accumulation registers as spill space) for
// two and four.
template <typename T, int Q, int OP>
__global__ __launch_bounds__(kAcaThreads, OP == kOpGalerkin ? (Q == 1 ? 2 : 1) : (Q == 1 ? 4 : (Q == 2 ? 3 : 2)))
void k_aca_wave(AcaArgs<T> A) {
  constexpr int c = Q == 4 ? 2 : (Q == 2 ? 3 : 4);
  constexpr int NB = Q == 4 ? 1 : (Q == 2 ? 2 : 4);
  const int lane = threadIdx.x & 63;
  const int64_t cnt = A.cnt[c];
  while (true) {
    int it = 0;
    if (lane == 0) it = atomicAdd(A.head + c, NB);
    it = uni(it);
    if (it >= cnt) break;
    const int64_t end = std::min<int64_t>(it + NB, cnt);
    for (int64_t k = it; k < end; ++k) aca_wave<T, Q, OP>(A, A.list[c][k]);
  }
}

__device__ inline int aca_bin(int64_t mx) {
  int k = 0;
  while (k < kAcaBins - 1 && mx > kAcaBinEdge[k]) ++k;
  return k;
}

// Largest max(m, n) a kernel class takes (the wavefront classes hold 64 Q
// rows and columns).
__host__ __device__ inline int64_t aca_class_cap(int c) {
  return c == 2 ? 256 : (c == 3 ? 128 : (c == 4 ? 64 : INT64_MAX));
}

// Class of every block: the class of its size bin.  With mask, only blocks
// whose mask entry is set get a class.  flags[c * nb + b] = (class == c).
__global__ void k_aca_classes(const int2* __restrict__ blk, int64_t nb,
                              const Cluster* __restrict__ cl, const int64_t* __restrict__ mask,
                              AcaBins bins, int64_t* __restrict__ flags) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const Cluster t = cl[ts.x], s = cl[ts.y];
    const int64_t mx = max(t.y - t.x, s.y - s.x);
    int c = bins.cls[aca_bin(mx)];
    if (mx > aca_class_cap(c)) c = 1;                  // never with a valid binning
    if (mask && !mask[b]) c = -1;
#pragma unroll
    for (int k = 0; k < kAcaClasses; ++k) flags[k * nb + b] = (k == c) ? 1 : 0;
  }
}

// list_c[offs_c[b]] = b for the class c of block b.
__global__ void k_split_lists(const int64_t* __restrict__ flags, const int64_t* __restrict__ offs,
                              int64_t nb, int32_t* __restrict__ lists) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < kAcaClasses; ++k)
      if (flags[k * nb + b]) lists[k * nb + offs[k * nb + b]] = (int32_t)b;
  }
}

// ------------------------------------------------------------------ panels
// Items are (block, leaf) pairs: the slice of a block that belongs to one leaf
// of its row cluster (dense slices, U slices) or column cluster.  Sorting the
// items by leaf (stable, so block order is kept inside a leaf) and scanning
// their widths gives every row leaf one contiguous panel per item set.

__global__ void k_count_leaves(const int2* __restrict__ blk, int64_t nb,
                               const int2* __restrict__ cl_leaves, int which,
                               int64_t* __restrict__ cnt) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const int2 lv = cl_leaves[which ? ts.y : ts.x];
    cnt[b] = lv.y - lv.x + 1;
  }
}

__global__ void k_expand_leaves(const int2* __restrict__ blk, int64_t nb,
                                const int2* __restrict__ cl_leaves, int which,
                                const int64_t* __restrict__ off, uint64_t* __restrict__ key,
                                int32_t* __restrict__ ib, int32_t* __restrict__ ilf,
                                int32_t* __restrict__ idx) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const int2 lv = cl_leaves[which ? ts.y : ts.x];
    int64_t o = off[b];
    for (int lf = lv.x; lf <= lv.y; ++lf, ++o) {
      key[o] = (uint64_t)lf;
      ib[o] = (int32_t)b;
      ilf[o] = lf;
      idx[o] = (int32_t)o;
    }
  }
}

// Width of every sorted item: the number of columns of the block (dense) or
// its rank (U slices).
__global__ void k_item_width(const int32_t* __restrict__ sidx, const int32_t* __restrict__ ib,
                             int64_t np, const int2* __restrict__ blk,
                             const Cluster* __restrict__ cl, const int32_t* __restrict__ rank,
                             int64_t* __restrict__ wid) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int b = ib[sidx[p]];
    if (rank) {
      wid[p] = rank[b];
    } else {
      const Cluster s = cl[blk[b].y];
      wid[p] = s.y - s.x;
    }
  }
}

// Leaf panels: first column col0[c] (in the item set's column space), width
// W[c] and size ld_c * W[c].  ibeg holds the first sorted item of each leaf.
__global__ void k_leaf_panels(const int64_t* __restrict__ ibeg, const int64_t* __restrict__ gcol,
                              int64_t np, int64_t total, const int64_t* __restrict__ ldpre,
                              int64_t nleaf, int64_t* __restrict__ col0, int64_t* __restrict__ W,
                              int64_t* __restrict__ psize) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nleaf;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = ibeg[c] < np ? gcol[ibeg[c]] : total;
    const int64_t e = ibeg[c + 1] < np ? gcol[ibeg[c + 1]] : total;
    col0[c] = a;
    W[c] = e - a;
    psize[c] = (ldpre[c + 1] - ldpre[c]) * (e - a);
  }
}

// Element offset of every sorted item inside the panel arena, and the
// inverse of the sort permutation.
__global__ void k_item_offsets(const int32_t* __restrict__ sidx, const int32_t* __restrict__ ilf,
                               int64_t np, const int64_t* __restrict__ gcol,
                               const int64_t* __restrict__ col0, const int64_t* __restrict__ poff,
                               const int64_t* __restrict__ ldpre, int64_t* __restrict__ offI,
                               int32_t* __restrict__ inv) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = sidx[p];
    const int lf = ilf[u];
    offI[p] = poff[lf] + (gcol[p] - col0[lf]) * (ldpre[lf + 1] - ldpre[lf]);
    inv[u] = (int32_t)p;
  }
}

// Column maps: a dense column multiplies x at Morton position sigma_lo + j,
// a U column multiplies t at n + toff_b + l.
__global__ void k_colmap(const int32_t* __restrict__ sidx, const int32_t* __restrict__ ib,
                         int64_t np, const int64_t* __restrict__ gcol,
                         const int64_t* __restrict__ wid, const int2* __restrict__ blk,
                         const Cluster* __restrict__ cl, const int64_t* __restrict__ toff,
                         int64_t tbase, int64_t n, int32_t* __restrict__ colmap) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int b = ib[sidx[p]];
    const int64_t base = toff ? n + tbase + toff[b] : (int64_t)cl[blk[b].y].x;
    const int64_t w = wid[p];
    for (int64_t j = 0; j < w; ++j) colmap[gcol[p] + j] = (int32_t)(base + j);
  }
}

__global__ void k_runs(const int64_t* __restrict__ col0, const int64_t* __restrict__ W,
                       const int64_t* __restrict__ poff, int64_t nleaf, uint64_t base, int esize,
                       int64_t colbase, Run* __restrict__ runs) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nleaf;
       c += (int64_t)gridDim.x * blockDim.x) {
    runs[c] = Run{base + (uint64_t)(poff[c] * esize), colbase + col0[c], (int32_t)W[c], 0};
  }
}

// ------------------------------------------------------------------ packing
// U slice of every sorted U item: the rows of leaf lf of block b, ld x r
// column-major, at its place in the leaf panel, converted to the factor
// storage type TL (divided by the term's scale when su is given).
template <typename T, typename TL>
__global__ __launch_bounds__(256) void k_pack_u(const int32_t* __restrict__ sidx,
                                                const int32_t* __restrict__ ib,
                                                const int32_t* __restrict__ ilf, int64_t np,
                                                const int2* __restrict__ blk,
                                                const Cluster* __restrict__ cl, LeafTab L,
                                                const int32_t* __restrict__ rank,
                                                const AcaSlot* __restrict__ slot,
                                                const int64_t* __restrict__ offI,
                                                const float* __restrict__ su,
                                                const int64_t* __restrict__ toff, int64_t tbase,
                                                TL* __restrict__ arena) {
  // one wavefront per item (slices are a few hundred values); wave-uniform
  // index, so the descriptors come in by scalar loads
  const int lane = threadIdx.x & 63;
  const int64_t wid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t p = wid; p < np; p += (int64_t)gridDim.x * 4) {
    const int32_t u = sidx[p];
    const int b = ib[u], lf = ilf[u];
    const int2 ts = blk[b];
    const Cluster tau = cl[ts.x];
    const int m = tau.y - tau.x, r = rank[b];
    const T* U = reinterpret_cast<const T*>((uintptr_t)slot[b].ptr);
    const int ld = leaf_ld(L, lf), ml = L.m[lf], off = L.lo[lf] - tau.x;
    TL* d = arena + offI[p];
    const int tot = ld * r;
    // eight values per lane in flight
    for (int e0 = lane; e0 < tot; e0 += 512) {
      T v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + 64 * k, i = e % ld, l = e / ld;
        v[k] = (e < tot && i < ml) ? U[(int64_t)l * m + off + i] : (T)0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e = e0 + 64 * k;
        if (e < tot) {
          T x = v[k];
          if (su) x = x / (T)su[tbase + toff[b] + e / ld];
          d[e] = (TL)x;
        }
      }
    }
  }
}

// Per-term scale of the U factors stored in FP16: max_i |U[i][l]| (1 for a
// zero column).  One wavefront per block.
template <typename T>
__global__ __launch_bounds__(256) void k_u_scales(const int2* __restrict__ blk, int64_t nb,
                                                  const Cluster* __restrict__ cl,
                                                  const int32_t* __restrict__ rank,
                                                  const AcaSlot* __restrict__ slot,
                                                  const int64_t* __restrict__ toff, int64_t tbase,
                                                  float* __restrict__ su) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t b = blockIdx.x * 4 + (threadIdx.x >> 6); b < nb; b += nw) {
    const Cluster tau = cl[blk[b].x];
    const int m = tau.y - tau.x, r = rank[b];
    const T* U = reinterpret_cast<const T*>((uintptr_t)slot[b].ptr);
    for (int l = 0; l < r; ++l) {
      float mx = 0.f;
      for (int i = lane; i < m; i += 64) mx = fmaxf(mx, fabsf((float)U[(int64_t)l * m + i]));
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d, 64));
      if (lane == 0) su[tbase + toff[b] + l] = mx > 0.f ? mx : 1.f;
    }
  }
}

// V factor of every block: its column-leaf slices (ld x r, column-major)
// at varena + vbase[b] + vw[b] (ldpre[lf] - ldpre[sf]), converted to TL
// (|v| <= 1 by the pivot normalisation, so no scale).
template <typename T, typename TL>
__global__ __launch_bounds__(256) void k_pack_v(const int2* __restrict__ blk, int64_t nb,
                                                const Cluster* __restrict__ cl, LeafTab L,
                                                const int32_t* __restrict__ rank,
                                                const AcaSlot* __restrict__ slot,
                                                const int64_t* __restrict__ vbase,
                                                const int32_t* __restrict__ vw,
                                                TL* __restrict__ varena,
                                                uint64_t* __restrict__ vptr) {
  // one wavefront per block (most are a few hundred values)
  const int lane = threadIdx.x & 63;
  const int64_t wid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t b = wid; b < nb; b += (int64_t)gridDim.x * 4) {
    const int2 ts = blk[b];
    const Cluster tau = cl[ts.x], sig = cl[ts.y];
    const int m = tau.y - tau.x, n = sig.y - sig.x, r = rank[b];
    const T* Vw = reinterpret_cast<const T*>((uintptr_t)slot[b].ptr) + (int64_t)slot[b].kc * m;
    TL* dst = varena + vbase[b];
    if (lane == 0) vptr[b] = (uint64_t)(uintptr_t)dst;
    const int2 ls = L.cl_leaves[ts.y];
    const int w = vw[b];
    for (int lf = ls.x; lf <= ls.y; ++lf) {
      const int ld = leaf_ld(L, lf), ml = L.m[lf], off = L.lo[lf] - sig.x;
      TL* d = dst + (int64_t)w * (L.ldpre[lf] - L.ldpre[ls.x]);
      const int tot = ld * r;
      for (int e0 = lane; e0 < tot; e0 += 512) {
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int e = e0 + 64 * k, i = e % ld, l = e / ld;
          v[k] = (e < tot && i < ml) ? Vw[(int64_t)l * n + off + i] : (T)0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int e = e0 + 64 * k;
          if (e < tot) d[e] = (TL)v[k];
        }
      }
    }
  }
}

// ---- column-cluster groups of the V factors.  The blocks of a chunk are
// sorted by column cluster; blocks that share it (and whose column leaves
// share one ld) form a group whose V slices lie side by side in one panel
// per column leaf (ld x W, W = the group's terms), in sorted order, with
// consecutive terms in t.  Blocks whose column leaves differ in ld stay
// alone (W = r).

// Sort key of every block: its column cluster, or 2^31 + b (alone).
__global__ void k_group_keys(const int2* __restrict__ blk, int64_t nb,
                             const int2* __restrict__ cl_leaves, const int64_t* __restrict__ ldpre,
                             uint64_t* __restrict__ key, int32_t* __restrict__ idx) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int sg = blk[b].y;
    const int2 ls = cl_leaves[sg];
    const int64_t ld0 = ldpre[ls.x + 1] - ldpre[ls.x];
    bool uni = true;
    for (int lf = ls.x + 1; lf <= ls.y && uni; ++lf) uni = (ldpre[lf + 1] - ldpre[lf]) == ld0;
    key[b] = uni ? (uint64_t)sg : ((uint64_t)1 << 31) + (uint64_t)b;
    idx[b] = (int32_t)b;
  }
}

// Ranks in sorted order, and 1 at the first position of every group.
__global__ void k_group_marks(const uint64_t* __restrict__ key, const int32_t* __restrict__ idx,
                              int64_t nb, const int32_t* __restrict__ rank,
                              int64_t* __restrict__ rk, int64_t* __restrict__ first) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nb;
       k += (int64_t)gridDim.x * blockDim.x) {
    rk[k] = rank[idx[k]];
    first[k] = (k == 0 || key[k] != key[k - 1]) ? 1 : 0;
  }
}

// Group table: first sorted position of every group (gpos[k] = groups
// before position k).
__global__ void k_group_starts(const int64_t* __restrict__ first, const int64_t* __restrict__ gpos,
                               int64_t nb, int64_t* __restrict__ gstart) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nb;
       k += (int64_t)gridDim.x * blockDim.x)
    if (first[k]) gstart[gpos[k]] = k;
}

// Per group: its width W (terms) and the size of its panels, W * LD(sigma).
__global__ void k_group_sizes(const int64_t* __restrict__ gstart, int64_t ng, int64_t nb,
                              const int64_t* __restrict__ tsort, const int32_t* __restrict__ idx,
                              const int2* __restrict__ blk, const int2* __restrict__ cl_leaves,
                              const int64_t* __restrict__ ldpre, int64_t* __restrict__ gw,
                              int64_t* __restrict__ gsz) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = gstart[g], e = g + 1 < ng ? gstart[g + 1] : nb;
    const int64_t w = tsort[e] - tsort[a];
    const int2 ls = cl_leaves[blk[idx[a]].y];
    gw[g] = w;
    gsz[g] = w * (ldpre[ls.y + 1] - ldpre[ls.x]);
  }
}

// Per block: its term offset (sorted order), the start of its first slice
// in the V arena and the slice width of its group.
__global__ void k_block_vlayout(const int32_t* __restrict__ idx, const int64_t* __restrict__ gpos,
                                const int64_t* __restrict__ first, int64_t nb,
                                const int64_t* __restrict__ tsort,
                                const int64_t* __restrict__ gstart, const int64_t* __restrict__ gw,
                                const int64_t* __restrict__ goff, const int2* __restrict__ blk,
                                const int2* __restrict__ cl_leaves,
                                const int64_t* __restrict__ ldpre, int64_t* __restrict__ toff,
                                int64_t* __restrict__ vbase, int32_t* __restrict__ vw) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nb;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int b = idx[k];
    const int64_t g = gpos[k] + first[k] - 1;
    const int64_t col = tsort[k] - tsort[gstart[g]];
    const int2 ls = cl_leaves[blk[b].y];
    toff[b] = tsort[k];
    vbase[b] = goff[g] + col * (ldpre[ls.x + 1] - ldpre[ls.x]);
    vw[b] = (int32_t)gw[g];
  }
}

// Work units of the forward phase 1 per group: its panel columns in chunks
// of at most uw(ld) (a group whose leaves differ in ld is one block: one
// unit).  uw is the widest chunk that the one-pass form of the one-column
// phase-1 kernel takes: R = ld / gran lanes per column, C = 64 / R columns
// per load (rounded down), `passes` loads per lane.  (A width of 1024 / ld
// that ignored the rounding sent every full unit of ld = 40, 48 or 60 to
// the slice-by-slice form.)
__device__ inline int unit_cols(int64_t ld, int gran, int passes) {
  const int64_t R = ld / gran > 0 ? ld / gran : 1;
  return (int)min((int64_t)64, passes * (64 / R));
}
__global__ void k_group_units(const int64_t* __restrict__ gstart, int64_t ng,
                              const uint64_t* __restrict__ key, const int32_t* __restrict__ idx,
                              const int64_t* __restrict__ gw, const int2* __restrict__ blk,
                              const int2* __restrict__ cl_leaves, const int64_t* __restrict__ ldpre,
                              int gran, int passes, int64_t* __restrict__ cnt) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = gstart[g];
    const int64_t w = gw[g];
    if (key[a] >= ((uint64_t)1 << 31)) {
      cnt[g] = w > 0 ? 1 : 0;
    } else {
      const int2 ls = cl_leaves[blk[idx[a]].y];
      const int uw = unit_cols(ldpre[ls.x + 1] - ldpre[ls.x], gran, passes);
      cnt[g] = (w + uw - 1) / uw;
    }
  }
}

__global__ void k_emit_units(const int64_t* __restrict__ gstart, int64_t ng,
                             const uint64_t* __restrict__ key, const int32_t* __restrict__ idx,
                             const int64_t* __restrict__ gw, const int64_t* __restrict__ goff,
                             const int64_t* __restrict__ uoff, const int64_t* __restrict__ tsort,
                             int64_t toff_base, const LrMeta* __restrict__ meta, int gran, int passes,
                             uint64_t varena, int esize, LrMeta* __restrict__ units) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = gstart[g];
    const int64_t w = gw[g];
    if (w == 0) continue;
    const LrMeta B = meta[idx[a]];                      // the group's first block
    if (key[a] >= ((uint64_t)1 << 31)) {
      units[uoff[g]] = B;
      continue;
    }
    const int64_t ld = B.vld;
    const int uw = unit_cols(ld, gran, passes);
    int64_t o = uoff[g];
    for (int64_t c0 = 0; c0 < w; c0 += uw, ++o) {
      LrMeta U = B;
      U.vptr = varena + (uint64_t)((goff[g] + c0 * ld) * esize);
      U.r = (int32_t)min((int64_t)uw, w - c0);
      U.toff = (int32_t)(toff_base + tsort[a] + c0);
      U.tf = U.tl = 0;
      U.ub = 0;
      U.vw = (int32_t)w;
      units[o] = U;
    }
  }
}

// Per U item: its global panel column (for the transposed block sums) and
// the address of its slice (for unpacking), indexed by (block, row leaf).
__global__ void k_urec(const int32_t* __restrict__ sidx, const int32_t* __restrict__ ib,
                       const int32_t* __restrict__ ilf, int64_t np, const int2* __restrict__ blk,
                       const int2* __restrict__ cl_leaves, const int64_t* __restrict__ ub,
                       const int64_t* __restrict__ gcol, int64_t colbase,
                       const int64_t* __restrict__ offI, uint64_t base, int esize,
                       int64_t* __restrict__ ucol, uint64_t* __restrict__ uptr) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = sidx[p];
    const int b = ib[u], lf = ilf[u];
    const int64_t q = ub[b] + (lf - cl_leaves[blk[b].x].x);
    ucol[q] = colbase + gcol[p];
    uptr[q] = base + (uint64_t)(offI[p] * esize);
  }
}

// Address of every dense item's slice, indexed by (block, row leaf) (for
// reading the stored near field back).
__global__ void k_drec(const int32_t* __restrict__ sidx, const int32_t* __restrict__ ib,
                       const int32_t* __restrict__ ilf, int64_t np, const int2* __restrict__ blk,
                       const int2* __restrict__ cl_leaves, const int64_t* __restrict__ ub,
                       const int64_t* __restrict__ offI, uint64_t base, int esize,
                       uint64_t* __restrict__ dptr) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = sidx[p];
    const int b = ib[u], lf = ilf[u];
    dptr[ub[b] + (lf - cl_leaves[blk[b].x].x)] = base + (uint64_t)(offI[p] * esize);
  }
}

__global__ void k_lr_meta(const int2* __restrict__ blk, int64_t nb, const int2* __restrict__ cl_leaves,
                          const int64_t* __restrict__ ldpre, const int32_t* __restrict__ rank,
                          const int64_t* __restrict__ toff, int64_t toff_base,
                          const uint64_t* __restrict__ vptr, const int32_t* __restrict__ vw,
                          const int64_t* __restrict__ ub, LrMeta* __restrict__ meta) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const int2 lt = cl_leaves[ts.x], ls = cl_leaves[ts.y];
    LrMeta M;
    M.vptr = vptr[b];
    M.r = rank[b];
    M.toff = (int32_t)(toff_base + toff[b]);
    M.sf = ls.x;
    M.sl = ls.y;
    M.tf = lt.x;
    M.tl = lt.y;
    M.ub = ub[b];
    const int64_t ld0 = ldpre[ls.x + 1] - ldpre[ls.x];
    bool uni = true;
    for (int lf = ls.x + 1; lf <= ls.y && uni; ++lf) uni = (ldpre[lf + 1] - ldpre[lf]) == ld0;
    M.vld = uni ? (int32_t)ld0 : 0;
    M.vw = vw[b];
    meta[b] = M;
  }
}

// ------------------------------------------------------------------ transposed items
// Per column leaf: every dense block whose column cluster contains it gives
// one item per row leaf (its columns' partial dots in w), every admissible
// block one V slice.
// The V side comes from the phase-1 units (column chunks of the V panels:
// wider items than single blocks, with consecutive terms).
__global__ void k_titem_counts(const int2* __restrict__ dns, int64_t nd, const LrMeta* __restrict__ units,
                               int64_t nl, const int2* __restrict__ cl_leaves,
                               int64_t* __restrict__ cnt) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nd + nl;
       b += (int64_t)gridDim.x * blockDim.x) {
    if (b < nd) {
      const int2 ts = dns[b];
      const int2 lt = cl_leaves[ts.x], ls = cl_leaves[ts.y];
      cnt[b] = (int64_t)(lt.y - lt.x + 1) * (ls.y - ls.x + 1);
    } else {
      const LrMeta& U = units[b - nd];
      cnt[b] = U.sl - U.sf + 1;
    }
  }
}

__global__ void k_titem_expand(const int2* __restrict__ dns, int64_t nd, int64_t nl,
                               const Cluster* __restrict__ cl, LeafTab L,
                               const int64_t* __restrict__ off, const int32_t* __restrict__ invD,
                               const int64_t* __restrict__ oD, const int64_t* __restrict__ gcolD,
                               const LrMeta* __restrict__ meta, int esize, TItem* __restrict__ out,
                               uint64_t* __restrict__ key, int32_t* __restrict__ idx) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nd + nl;
       b += (int64_t)gridDim.x * blockDim.x) {
    int64_t o = off[b];
    if (b < nd) {
      const int2 ts = dns[b];
      const Cluster sig = cl[ts.y];
      const int2 lt = L.cl_leaves[ts.x], ls = L.cl_leaves[ts.y];
      for (int lf = lt.x; lf <= lt.y; ++lf) {
        const int64_t p = invD[oD[b] + (lf - lt.x)];
        for (int cf = ls.x; cf <= ls.y; ++cf, ++o) {
          out[o] = TItem{0, gcolD[p] + (L.lo[cf] - sig.x), L.m[cf], 0};
          key[o] = (uint64_t)cf;
          idx[o] = (int32_t)o;
        }
      }
    } else {
      const LrMeta M = meta[b - nd];
      for (int cf = M.sf; cf <= M.sl; ++cf, ++o) {
        const uint64_t d = M.vptr + (uint64_t)((int64_t)M.vw * (L.ldpre[cf] - L.ldpre[M.sf]) * esize);
        out[o] = TItem{d, (int64_t)M.toff, M.r, 1};
        key[o] = (uint64_t)cf;
        idx[o] = (int32_t)o;
      }
    }
  }
}

__global__ void k_gather_titems(const TItem* __restrict__ in, const int32_t* __restrict__ idx,
                                int64_t n, TItem* __restrict__ out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    out[k] = in[idx[k]];
}

// beg[c] = first position p of the sorted keys with key[p] >= c, for
// c = 0..nleaf (beg[nleaf] = n): each position fills the leaves between its
// predecessor's key and its own.
__global__ void k_seg_begins(const uint64_t* __restrict__ keys, int64_t n, int64_t nleaf,
                             int64_t* __restrict__ beg) {
  // beg[c] = first position whose key is >= c (keys sorted, all < nleaf), by
  // a binary search per leaf: leaves without items cost no serial loop
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c <= nleaf;
       c += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if ((int64_t)keys[mid] < c)
        lo = mid + 1;
      else
        hi = mid;
    }
    beg[c] = lo;
  }
}

__global__ void k_to_i32(const int64_t* __restrict__ a, int64_t n, int32_t* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (int32_t)a[e];
}

// Unpack one factorised block back into plain column-major U (m x r), V (n x r),
// scales applied.
template <typename TL, typename TO>
__global__ void k_unpack(const int2* __restrict__ lr, int64_t b, const Cluster* __restrict__ cl,
                         LeafTab L, const LrMeta* __restrict__ meta,
                         const uint64_t* __restrict__ uptr, const float* __restrict__ su,
                         TO* __restrict__ out) {
  const int2 ts = lr[b];
  const Cluster tau = cl[ts.x], sig = cl[ts.y];
  const LrMeta M = meta[b];
  const int m = tau.y - tau.x, n = sig.y - sig.x, r = M.r;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)(m + n) * r;
       e += (int64_t)gridDim.x * blockDim.x) {
    const bool isu = e < (int64_t)m * r;
    const int64_t ee = isu ? e : e - (int64_t)m * r;
    const int rows = isu ? m : n;
    const int i = (int)(ee % rows), l = (int)(ee / rows);
    const int pos = (isu ? tau.x : sig.x) + i;
    const int lf0 = isu ? M.tf : M.sf, lf1 = isu ? M.tl : M.sl;
    int lf = lf0;
    while (lf < lf1 && L.lo[lf + 1] <= pos) ++lf;
    const TL* sl;
    if (isu)
      sl = reinterpret_cast<const TL*>((uintptr_t)uptr[M.ub + (lf - lf0)]);
    else
      sl = reinterpret_cast<const TL*>((uintptr_t)M.vptr) + (int64_t)M.vw * (L.ldpre[lf] - L.ldpre[lf0]);
    TO v = (TO)sl[(int64_t)l * leaf_ld(L, lf) + (pos - L.lo[lf])];
    if (isu && su) v *= (TO)su[M.toff + l];
    out[e] = v;
  }
}

// ------------------------------------------------------------------ ACA launchers
// Elements of a working slot at rank cap kcap: U (m x kcap) and V
// (n x kcap), then m bytes of used-row flags, rounded up to 4 elements.
template <typename T>
__host__ __device__ inline int64_t slot_elems(int64_t m, int64_t n, int kcap) {
  const int64_t flag_elems = (m + (int64_t)sizeof(T) - 1) / (int64_t)sizeof(T);
  return (((int64_t)kcap * (m + n) + flag_elems) + 3) & ~(int64_t)3;
}

// One queue launch per kernel class with work, largest class first; A holds
// the class lists and counts (head is zeroed here).
template <typename T, int OP>
void launch_aca_classes(const AcaArgs<T>& A, int* head, hipStream_t s) {
  HM_HIP(hipMemsetAsync(head, 0, kAcaClasses * sizeof(int), s));
  int dev = 0, ncu = 0;
  HM_HIP(hipGetDevice(&dev));
  HM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  ncu = std::max(ncu, 1);
  // grid: as many workgroups as can be resident at once (the queue does the
  // rest), never more than the class has work for
  auto grid = [&](const void* k, int threads, int64_t work) {
    int per_cu = 0;
    HM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, 0));
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(work, (int64_t)ncu * std::max(per_cu, 1)));
  };
  const int64_t* cnt = A.cnt;
  if constexpr (OP == kOpColloc) {
    if (cnt[0] > 0) {
      k_aca_wg<T, 1024, 0, OP><<<grid((const void*)k_aca_wg<T, 1024, 0, OP>, 1024, cnt[0]), 1024,
                                 0, s>>>(A);
      HM_LAUNCH_CHECK();
    }
  }
  if (cnt[1] > 0) {
    k_aca_wg<T, 256, 1, OP><<<grid((const void*)k_aca_wg<T, 256, 1, OP>, 256, cnt[1]), 256, 0, s>>>(A);
    HM_LAUNCH_CHECK();
  }
  if (cnt[5] > 0) {
    k_aca_wg<T, 128, 5, OP><<<grid((const void*)k_aca_wg<T, 128, 5, OP>, 128, cnt[5]), 128, 0, s>>>(A);
    HM_LAUNCH_CHECK();
  }
  {
    if (cnt[2] > 0) {
      k_aca_wave<T, 4, OP><<<grid((const void*)k_aca_wave<T, 4, OP>, kAcaThreads,
                                  ceil_div(cnt[2], kAcaWaves)),
                             kAcaThreads, 0, s>>>(A);
      HM_LAUNCH_CHECK();
    }
    if (cnt[3] > 0) {
      k_aca_wave<T, 2, OP><<<grid((const void*)k_aca_wave<T, 2, OP>, kAcaThreads,
                                  ceil_div(cnt[3], 2 * kAcaWaves)),
                             kAcaThreads, 0, s>>>(A);
      HM_LAUNCH_CHECK();
    }
  }
  if (cnt[4] > 0) {
    k_aca_wave<T, 1, OP><<<grid((const void*)k_aca_wave<T, 1, OP>, kAcaThreads, ceil_div(cnt[4], 4 * kAcaWaves)),
                       kAcaThreads, 0, s>>>(A);
    HM_LAUNCH_CHECK();
  }
}

// The batched ACA over the blocks of a chunk (with mask: only the marked
// ones) at rank cap kmax: class lists from the binning, then the class
// launches.  flags, offs: kAcaClasses * nb int64 scratch; lists:
// kAcaClasses * nb int32; head: kAcaClasses int.
template <typename T, int OP>
void run_aca(const Geom<T>& g, const int2* blk, int64_t nb, const Cluster* cl,
             const AcaSlot* slot, int kmax, double eps, const int64_t* mask, const AcaBins& bins,
             int64_t* flags, int64_t* offs, int32_t* lists, int* head, int32_t* rank,
             int32_t* info, int64_t* tmp, hipStream_t s) {
  if (nb == 0) return;
  if (nb >= INT32_MAX) throw Error{HM_ERR_STATE, "ACA chunk of more than 2^31 blocks"};
  k_aca_classes<<<grid_for(nb, 256), 256, 0, s>>>(blk, nb, cl, mask, bins, flags);
  HM_LAUNCH_CHECK();
  for (int k = 0; k < kAcaClasses; ++k)
    scan_excl_i64(flags + k * nb, offs + k * nb, nb, tmp + k, s);
  int64_t cnt[kAcaClasses];
  HM_HIP(hipMemcpyAsync(cnt, tmp, kAcaClasses * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HM_HIP(hipStreamSynchronize(s));
  k_split_lists<<<grid_for(nb, 256), 256, 0, s>>>(flags, offs, nb, lists);
  HM_LAUNCH_CHECK();
  AcaArgs<T> A{};
  A.g = g;
  A.blk = blk;
  A.cl = cl;
  A.slot = slot;
  for (int k = 0; k < kAcaClasses; ++k) {
    A.list[k] = lists + k * nb;
    A.cnt[k] = cnt[k];
  }
  A.head = head;
  A.kmax = kmax;
  A.eps = eps;
  A.rank = rank;
  A.info = info;
  launch_aca_classes<T, OP>(A, head, s);
}

// The binning the library uses without tuning, from the tuner's choices at
// N = 1,310,720 (FP32): wavefront classes up to 256 (one, two or four rows
// per lane), 128-thread workgroups up to 1,024 (257..512: 1.46 against
// 1.98 ms for 256-thread workgroups on a sample of 16,151 blocks; 513..1,024:
// 2.47 against 2.70 ms), 256-thread workgroups up to 4,096 and 1,024-thread
// workgroups above.  Galerkin entries keep the row triangle in registers:
// one and two rows per lane up to 128, 128-thread workgroups up to 1,024 and
// 256-thread workgroups above (65..128 on two rows per lane 0.96 against
// 1.07 ms for 128 threads and 1.64 for 256; 129..256 on 128 threads 1.56
// against 1.91 for 256 threads and 2.32 for four rows per lane; 257..512
// 2.24 against 2.79; 513..1,024 3.78 against 4.10); the 1,024-thread class
// is not built for them.
AcaBins default_aca_bins(int op) {
  if (op == kOpGalerkin) return AcaBins{{4, 3, 5, 5, 5, 1, 1, 1}};
  return AcaBins{{4, 3, 2, 5, 5, 1, 1, 0}};
}

// Kernel classes the tuner tries for a bin.
std::vector<int> aca_bin_candidates(int bin, int op) {
  if (op == kOpGalerkin) {
    // the wavefront classes with two and four rows per lane run Galerkin
    // entries at one or two waves per SIMD; the 1,024-thread class is not
    // built for them
    if (bin == 0) return {4};
    if (bin == 1) return {1, 3, 5};
    if (bin == 2) return {1, 2, 5};
    if (bin <= 4) return {1, 5};
    return {1};
  }
  switch (bin) {
    case 0: return {4};
    case 1: return {3, 1, 5};
    case 2: return {2, 1, 5};
    case 3:
    case 4: return {1, 5, 0};
    default: return {1, 0, 5};
  }
}

__global__ void k_block_bins(const int2* __restrict__ blk, int64_t nb,
                             const Cluster* __restrict__ cl, int32_t* __restrict__ bin) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const Cluster t = cl[ts.x], s = cl[ts.y];
    bin[b] = aca_bin(max(t.y - t.x, s.y - s.x));
  }
}

// desc[list[k]] = {pool + off[k], kcap} for the blocks of a list.
template <typename T>
__global__ void k_list_desc(const int32_t* __restrict__ list, int64_t cnt,
                            const int2* __restrict__ blk, const Cluster* __restrict__ cl, int kmax,
                            const int64_t* __restrict__ off, T* pool, AcaSlot* __restrict__ desc) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < cnt;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int b = list[k];
    const int2 ts = blk[b];
    const Cluster t = cl[ts.x], s = cl[ts.y];
    AcaSlot d;
    d.ptr = (uint64_t)(uintptr_t)(pool + off[k]);
    d.kc = min(kmax, min(t.y - t.x, s.y - s.x));
    d.pad = 0;
    desc[b] = d;
  }
}

// The binning tuner: for every size bin with more than one candidate class,
// a sample of its blocks (every st-th block in list order, at most
// kTuneSample, and no more than the working pool holds) is run through each
// candidate's kernel at the first-pass rank cap, twice, and the second pass
// is timed with HIP events; the fastest class is kept.  The sample's ranks
// and slots are overwritten by the real run.
constexpr int64_t kTuneSample = 16384;

template <typename T, int OP>
AcaBins tune_aca_bins(const Geom<T>& g, const SetupIn& in, int k1, double eps, T* pool,
                      int64_t pool_elems, AcaSlot* desc, int* head, int32_t* rank, int32_t* info,
                      std::vector<AcaTuneRow>& rows, hipStream_t s) {
  AcaBins bins = default_aca_bins(OP);
  const int64_t nl = in.nl;
  std::vector<int32_t> hb(nl);
  std::vector<int2> hlr(nl);
  std::vector<Cluster> hcl;
  {
    int32_t* db = dalloc_t<int32_t>(nl, s);
    k_block_bins<<<grid_for(nl, 256), 256, 0, s>>>(in.lr, nl, in.cl, db);
    HM_LAUNCH_CHECK();
    HM_HIP(hipMemcpyAsync(hb.data(), db, nl * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HM_HIP(hipMemcpyAsync(hlr.data(), in.lr, nl * sizeof(int2), hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    dfree(db, s);
    int ncl = 0;
    for (const int2& b : hlr) ncl = std::max(ncl, std::max(b.x, b.y) + 1);
    hcl.resize(ncl);
    HM_HIP(hipMemcpyAsync(hcl.data(), in.cl, ncl * sizeof(Cluster), hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
  }
  std::vector<std::vector<int32_t>> members(kAcaBins);
  for (int64_t b = 0; b < nl; ++b) members[hb[b]].push_back((int32_t)b);
  int32_t* dlist = dalloc_t<int32_t>(kTuneSample, s);
  int64_t* doff = dalloc_t<int64_t>(kTuneSample, s);
  hipEvent_t e0, e1;
  HM_HIP(hipEventCreate(&e0));
  HM_HIP(hipEventCreate(&e1));
  for (int bin = 0; bin < kAcaBins; ++bin) {
    const std::vector<int> cand = aca_bin_candidates(bin, OP);
    const std::vector<int32_t>& mem = members[bin];
    if (cand.size() < 2 || mem.empty()) continue;
    // the sample and its slots, laid out from the start of the pool
    const int64_t st = std::max<int64_t>(1, ((int64_t)mem.size() + kTuneSample - 1) / kTuneSample);
    std::vector<int32_t> smp;
    std::vector<int64_t> off;
    int64_t used = 0;
    for (size_t k = 0; k < mem.size(); k += (size_t)st) {
      const int2 ts = hlr[mem[k]];
      const int64_t m = hcl[ts.x].y - hcl[ts.x].x, n = hcl[ts.y].y - hcl[ts.y].x;
      const int64_t e = slot_elems<T>(m, n, (int)std::min<int64_t>(k1, std::min(m, n)));
      if (used + e > pool_elems) break;
      smp.push_back(mem[k]);
      off.push_back(used);
      used += e;
    }
    if (smp.empty()) continue;
    const int64_t ns = (int64_t)smp.size();
    HM_HIP(hipMemcpyAsync(dlist, smp.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HM_HIP(hipMemcpyAsync(doff, off.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice, s));
    k_list_desc<T><<<grid_for(ns, 256), 256, 0, s>>>(dlist, ns, in.lr, in.cl, k1, doff, pool,
                                                      desc);
    HM_LAUNCH_CHECK();
    double best = 0.0;
    for (int c : cand) {
      AcaArgs<T> A{};
      A.g = g;
      A.blk = in.lr;
      A.cl = in.cl;
      A.slot = desc;
      A.list[c] = dlist;
      A.cnt[c] = ns;
      A.head = head;
      A.kmax = k1;
      A.eps = eps;
      A.rank = rank;
      A.info = info;
      launch_aca_classes<T, OP>(A, head, s);            // warm-up (code loading, caches)
      HM_HIP(hipEventRecord(e0, s));
      launch_aca_classes<T, OP>(A, head, s);
      HM_HIP(hipEventRecord(e1, s));
      HM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      HM_HIP(hipEventElapsedTime(&ms, e0, e1));
      rows.push_back(AcaTuneRow{bin, c, ns, (double)ms});
      if (c == cand.front() || ms < best) {
        best = ms;
        bins.cls[bin] = c;
      }
    }
  }
  HM_HIP(hipEventDestroy(e0));
  HM_HIP(hipEventDestroy(e1));
  dfree(dlist, s);
  dfree(doff, s);
  return bins;
}

// Largest possible rank of every block: min(kmax, m, n).
__global__ void k_term_caps(const int2* __restrict__ blk, int64_t nb, const Cluster* __restrict__ cl,
                            int kmax, int64_t* __restrict__ kc) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const Cluster t = cl[ts.x], s = cl[ts.y];
    kc[b] = min((int64_t)kmax, (int64_t)min(t.y - t.x, s.y - s.x));
  }
}

// Working-slot sizes (elements) of all blocks at rank cap kmax.
template <typename T>
__global__ void k_slot_sizes(const int2* __restrict__ blk, int64_t nb, const Cluster* __restrict__ cl,
                             int kmax, int64_t* __restrict__ slot) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const Cluster t = cl[ts.x], s = cl[ts.y];
    const int64_t m = t.y - t.x, n = s.y - s.x;
    slot[b] = slot_elems<T>(m, n, (int)min((int64_t)kmax, min(m, n)));
  }
}

// Slot descriptors of a chunk's blocks: pool + (off[b] - off0) and the rank
// cap kmax of the pass.  With mask, only the marked blocks are written.
template <typename T>
__global__ void k_slot_desc(const int2* __restrict__ blk, int64_t nb, const Cluster* __restrict__ cl,
                            int kmax, const int64_t* __restrict__ off, int64_t off0, T* pool,
                            const int64_t* __restrict__ mask, AcaSlot* __restrict__ desc) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    if (mask && !mask[b]) continue;
    const int2 ts = blk[b];
    const Cluster t = cl[ts.x], s = cl[ts.y];
    const int kcap = min(kmax, min(t.y - t.x, s.y - s.x));
    AcaSlot d;
    d.ptr = (uint64_t)(uintptr_t)(pool + (off[b] - off0));
    d.kc = kcap;
    d.pad = 0;
    desc[b] = d;
  }
}

// Blocks of the first pass that stopped at its rank cap k1 although the full
// cap allows more terms: mark[b] = 1 and their slot size at the full cap.
template <typename T>
__global__ void k_rerun_marks(const int2* __restrict__ blk, int64_t nb, const Cluster* __restrict__ cl,
                              const int32_t* __restrict__ info, int k1, int kmax,
                              int64_t* __restrict__ mark, int64_t* __restrict__ size) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int2 ts = blk[b];
    const Cluster t = cl[ts.x], s = cl[ts.y];
    const int64_t m = t.y - t.x, n = s.y - s.x;
    const int full = (int)min((int64_t)kmax, min(m, n));
    const bool again = (info[b] & 1) && k1 < full;
    mark[b] = again ? 1 : 0;
    size[b] = again ? slot_elems<T>(m, n, full) : 0;
  }
}

// ------------------------------------------------------------------ host side
template <typename T>
void launch_entries(const Geom<T>& g, int op, const int32_t* inv, const int32_t* rows,
                    const int32_t* cols, int64_t cnt, double* out, hipStream_t s) {
  const GaussRule R = gauss_rule01();
  if (op == kOpGalerkin)
    k_entries<T, kOpGalerkin><<<grid_for(cnt, 4, 1 << 20), 256, 0, s>>>(g, R, inv, rows, cols, cnt, out);
  else
    k_entries<T, kOpColloc><<<grid_for(cnt, 4, 1 << 20), 256, 0, s>>>(g, R, inv, rows, cols, cnt, out);
  HM_LAUNCH_CHECK();
}
template void launch_entries<float>(const Geom<float>&, int, const int32_t*, const int32_t*,
                                    const int32_t*, int64_t, double*, hipStream_t);
template void launch_entries<double>(const Geom<double>&, int, const int32_t*, const int32_t*,
                                     const int32_t*, int64_t, double*, hipStream_t);

// Gauss-Legendre nodes and weights on [0, 1]: the roots of the Legendre
// polynomial P_q by Newton's method from the Chebyshev-like first guesses,
// weights 2 / ((1 - x^2) P_q'(x)^2), both mapped from [-1, 1].
GaussRule gauss_rule01() {
  GaussRule R{};
  const int q = kGalQ;
  for (int k = 0; k < q; ++k) {
    double x = std::cos(M_PI * (k + 0.75) / (q + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int l = 2; l <= q; ++l) {
        const double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    R.x[k] = 0.5 * (x + 1.0);
    R.w[k] = 1.0 / ((1.0 - x * x) * dp * dp);   // (2 / ((1 - x^2) P'^2)) / 2
  }
  return R;
}

void launch_inverse_perm(const int32_t* perm, int64_t n, int32_t* inv, hipStream_t s) {
  k_inverse_perm<<<grid_for(n, 256), 256, 0, s>>>(perm, n, inv);
  HM_LAUNCH_CHECK();
}

namespace {
using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}
int64_t scan_total(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
  scan_excl_i64(in, out, n, tmp, s);
  return d2h_i64(tmp, s);
}
int bits_for(int64_t v) {
  int b = 1;
  while ((1ll << b) < v) ++b;
  return b;
}

// Temporary device buffers released together.
struct Temps {
  hipStream_t s;
  std::vector<void*> v;
  template <typename X>
  X* get(int64_t cnt) {
    X* p = dalloc_t<X>(cnt > 0 ? cnt : 1, s);
    v.push_back(p);
    return p;
  }
  void release() {
    for (void* p : v) dfree(p, s);
    v.clear();
  }
  ~Temps() { release(); }
};

// A set of (block, leaf) items sorted by leaf, with leaf panels laid out.
struct PanelSet {
  int64_t np = 0, cols = 0, elems = 0;
  int32_t *ib = nullptr, *ilf = nullptr, *sidx = nullptr, *inv = nullptr;
  int64_t *wid = nullptr, *gcol = nullptr, *col0 = nullptr, *W = nullptr, *poff = nullptr,
          *offI = nullptr;
};

// Expands the row-leaf items of blocks blk[0..nb), sorts them by leaf and lays
// out one panel per leaf (widths: cluster size of sigma, or rank).
void panel_layout(const int2* blk, int64_t nb, const Cluster* cl, const int2* cl_leaves,
                  const int64_t* ldpre, int64_t nleaf, const int32_t* rank, int64_t* off,
                  PanelSet& P, Temps& T, int64_t* tmp, hipStream_t s) {
  int64_t* cnt = T.get<int64_t>(nb);
  k_count_leaves<<<grid_for(nb, 256), 256, 0, s>>>(blk, nb, cl_leaves, 0, cnt);
  HM_LAUNCH_CHECK();
  P.np = scan_total(cnt, off, nb, tmp, s);
  if (P.np >= INT32_MAX) throw Error{HM_ERR_STATE, "more than 2^31 block slices"};
  uint64_t* key = T.get<uint64_t>(P.np);
  P.ib = T.get<int32_t>(P.np);
  P.ilf = T.get<int32_t>(P.np);
  P.sidx = T.get<int32_t>(P.np);
  k_expand_leaves<<<grid_for(nb, 64), 64, 0, s>>>(blk, nb, cl_leaves, 0, off, key, P.ib, P.ilf,
                                                  P.sidx);
  HM_LAUNCH_CHECK();
  radix_sort_u64_i32(key, P.sidx, P.np, bits_for(nleaf), s);
  P.wid = T.get<int64_t>(P.np);
  P.gcol = T.get<int64_t>(P.np);
  k_item_width<<<grid_for(P.np, 256), 256, 0, s>>>(P.sidx, P.ib, P.np, blk, cl, rank, P.wid);
  HM_LAUNCH_CHECK();
  P.cols = scan_total(P.wid, P.gcol, P.np, tmp, s);
  int64_t* ibeg = T.get<int64_t>(nleaf + 1);
  k_seg_begins<<<grid_for(nleaf + 1, 256), 256, 0, s>>>(key, P.np, nleaf, ibeg);
  HM_LAUNCH_CHECK();
  P.col0 = T.get<int64_t>(nleaf);
  P.W = T.get<int64_t>(nleaf);
  int64_t* psize = T.get<int64_t>(nleaf);
  k_leaf_panels<<<grid_for(nleaf, 256), 256, 0, s>>>(ibeg, P.gcol, P.np, P.cols, ldpre, nleaf,
                                                     P.col0, P.W, psize);
  HM_LAUNCH_CHECK();
  P.poff = T.get<int64_t>(nleaf);
  P.elems = scan_total(psize, P.poff, nleaf, tmp, s);
  P.offI = T.get<int64_t>(P.np);
  P.inv = T.get<int32_t>(P.np);
  k_item_offsets<<<grid_for(P.np, 256), 256, 0, s>>>(P.sidx, P.ilf, P.np, P.gcol, P.col0, P.poff,
                                                     ldpre, P.offI, P.inv);
  HM_LAUNCH_CHECK();
}
}  // namespace

// Work units of the per-row-leaf product kernels: every run of every leaf
// cut into pieces of at most ucols columns, grouped by leaf.
void make_units(Storage& out, const int64_t* ldpre, int64_t nleaf, int ucols, const Alloc& alloc,
                hipStream_t s) {
  std::vector<Run> hr((size_t)out.nruns * nleaf);
  std::vector<int64_t> hld(nleaf + 1);
  if (!hr.empty())
    HM_HIP(hipMemcpyAsync(hr.data(), out.runs, hr.size() * sizeof(Run), hipMemcpyDeviceToHost, s));
  HM_HIP(hipMemcpyAsync(hld.data(), ldpre, (nleaf + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HM_HIP(hipStreamSynchronize(s));
  std::vector<Unit> hu;
  std::vector<int32_t> hb(nleaf + 1);
  out.ldmax = 1;
  for (int64_t c = 0; c < nleaf; ++c) {
    hb[c] = (int32_t)hu.size();
    out.ldmax = std::max(out.ldmax, (int)(hld[c + 1] - hld[c]));
    for (int k = 0; k < out.nruns; ++k) {
      const int64_t w = hr[(size_t)k * nleaf + c].w;
      for (int64_t a = 0; a < w; a += ucols)
        hu.push_back(Unit{(int32_t)c, k, (int32_t)a, (int32_t)std::min<int64_t>(ucols, w - a)});
    }
  }
  if (hu.size() >= (size_t)INT32_MAX) throw Error{HM_ERR_STATE, "too many product units"};
  hb[nleaf] = (int32_t)hu.size();
  out.nunits = (int64_t)hu.size();
  out.unit_cols = ucols;
  out.units = static_cast<Unit*>(alloc((hu.size() + 1) * sizeof(Unit)));
  out.ubeg = static_cast<int32_t*>(alloc(hb.size() * sizeof(int32_t)));
  if (!hu.empty())
    HM_HIP(hipMemcpyAsync(out.units, hu.data(), hu.size() * sizeof(Unit), hipMemcpyHostToDevice, s));
  HM_HIP(hipMemcpyAsync(out.ubeg, hb.data(), hb.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HM_HIP(hipStreamSynchronize(s));
}

// Number of units make_units would produce for ucols.
int64_t count_units(const Storage& out, int64_t nleaf, int ucols, hipStream_t s) {
  std::vector<Run> hr((size_t)out.nruns * nleaf);
  if (!hr.empty())
    HM_HIP(hipMemcpyAsync(hr.data(), out.runs, hr.size() * sizeof(Run), hipMemcpyDeviceToHost, s));
  HM_HIP(hipStreamSynchronize(s));
  int64_t cnt = 0;
  for (const Run& r : hr) cnt += (r.w + ucols - 1) / ucols;
  return cnt;
}

template <typename T, typename TL>
void build_storage(const Geom<T>& g, const SetupIn& in, Storage& out, const Alloc& alloc,
                   hipStream_t s) {
  const LeafTab L{in.leaf_lo, in.leaf_m, in.ldpre, in.cl_leaves};
  const int esize = (int)sizeof(T);
  const int lsize = (int)sizeof(TL);
  constexpr bool scaled = !std::is_same<T, TL>::value;
  const int64_t n = in.n, nleaf = in.nleaf;
  Temps keep{s, {}};       // lives until the product plan is complete
  int64_t* tmp = keep.get<int64_t>(8);   // one total per ACA class, scan scratch

  // ---- near field: dense slices in row-leaf panels
  auto t0 = clk::now();
  PanelSet PD;
  int64_t* oD = keep.get<int64_t>(in.nd + 1);
  Temps td{s, {}};
  panel_layout(in.dns, in.nd, in.cl, in.cl_leaves, in.ldpre, nleaf, nullptr, oD, PD, td, tmp, s);
  out.D_elems = PD.elems;
  out.dense_cols = PD.cols;
  T* D = static_cast<T*>(alloc((size_t)PD.elems * esize));
  int32_t* colmapD = keep.get<int32_t>(PD.cols);
  k_colmap<<<grid_for(PD.np, 256), 256, 0, s>>>(PD.sidx, PD.ib, PD.np, PD.gcol, PD.wid, in.dns,
                                                in.cl, nullptr, 0, n, colmapD);
  HM_LAUNCH_CHECK();
  std::vector<Run*> run_parts;
  std::vector<std::pair<int32_t*, int64_t>> colmap_parts;
  std::vector<std::pair<LrMeta*, int64_t>> unit_parts;      // forward phase-1 units per chunk
  Run* runD = keep.get<Run>(nleaf);
  k_runs<<<grid_for(nleaf, 256), 256, 0, s>>>(PD.col0, PD.W, PD.poff, nleaf, (uint64_t)(uintptr_t)D,
                                              esize, 0, runD);
  HM_LAUNCH_CHECK();
  run_parts.push_back(runD);
  colmap_parts.push_back({colmapD, PD.cols});
  if (PD.np > 0) {
    const unsigned gn = grid_for(PD.np, 1, 1 << 20);
    if (in.op == kOpGalerkin) {
      k_near<T, kOpGalerkin><<<gn, 256, 0, s>>>(g, PD.sidx, PD.ib, PD.ilf, PD.np, in.dns, in.cl, L,
                                                PD.offI, D);
      HM_LAUNCH_CHECK();
      k_near_singular<T><<<gn, 256, 0, s>>>(g, gauss_rule01(), PD.sidx, PD.ib, PD.ilf, PD.np,
                                            in.dns, in.cl, L, PD.offI, D);
    } else {
      k_near<T, kOpColloc><<<gn, 256, 0, s>>>(g, PD.sidx, PD.ib, PD.ilf, PD.np, in.dns, in.cl, L,
                                              PD.offI, D);
    }
    HM_LAUNCH_CHECK();
  }
  // slice addresses of the dense items, by (block, row leaf)
  out.dub = static_cast<int64_t*>(alloc((size_t)(in.nd + 1) * sizeof(int64_t)));
  out.dptr = static_cast<uint64_t*>(alloc((size_t)(PD.np + 1) * sizeof(uint64_t)));
  if (in.nd > 0)
    HM_HIP(hipMemcpyAsync(out.dub, oD, in.nd * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  if (PD.np > 0) {
    k_drec<<<grid_for(PD.np, 256), 256, 0, s>>>(PD.sidx, PD.ib, PD.ilf, PD.np, in.dns,
                                                in.cl_leaves, oD, PD.offI,
                                                (uint64_t)(uintptr_t)D, esize, out.dptr);
    HM_LAUNCH_CHECK();
  }
  // keep what the transposed items need
  int32_t* invD = keep.get<int32_t>(PD.np);
  int64_t* gcolD = keep.get<int64_t>(PD.np);
  if (PD.np) {
    HM_HIP(hipMemcpyAsync(invD, PD.inv, PD.np * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HM_HIP(hipMemcpyAsync(gcolD, PD.gcol, PD.np * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  }
  td.release();
  HM_HIP(hipStreamSynchronize(s));
  out.ms_near = ms_since(t0);

  // ---- batched ACA in memory-bounded chunks; U slices in row-leaf panels,
  // V factors block-contiguous
  t0 = clk::now();
  const int kmax = in.kmax;
  const int64_t nl = in.nl;
  out.rank = static_cast<int32_t*>(alloc((nl + 1) * sizeof(int32_t)));
  out.info = static_cast<int32_t*>(alloc((nl + 1) * sizeof(int32_t)));
  out.meta = static_cast<LrMeta*>(alloc((nl + 1) * sizeof(LrMeta)));
  int64_t* ub = static_cast<int64_t*>(alloc((nl + 1) * sizeof(int64_t)));
  {
    int64_t* cnt = keep.get<int64_t>(nl);
    if (nl) {
      k_count_leaves<<<grid_for(nl, 256), 256, 0, s>>>(in.lr, nl, in.cl_leaves, 0, cnt);
      HM_LAUNCH_CHECK();
    }
    out.u_items = scan_total(cnt, ub, nl, tmp, s);
  }
  out.ucol = static_cast<int64_t*>(alloc((out.u_items + 1) * sizeof(int64_t)));
  out.uptr = static_cast<uint64_t*>(alloc((out.u_items + 1) * sizeof(uint64_t)));
  int64_t toff_base = 0, ucols = 0;
  double ms_pack = 0;
  if (nl > 0) {
    Temps ta{s, {}};
    // first pass at the rank cap k1 (slots sized for it); blocks that stop
    // at k1 although kmax allows more are run again with full-size slots
    const int k1 = std::min(kmax, kAcaFirstRank);
    int64_t* slot = ta.get<int64_t>(nl);
    int64_t* slot_off = ta.get<int64_t>(nl + 1);
    k_slot_sizes<T><<<grid_for(nl, 256), 256, 0, s>>>(in.lr, nl, in.cl, k1, slot);
    HM_LAUNCH_CHECK();
    scan_excl_i64(slot, slot_off, nl, slot_off + nl, s);
    // all slots at once when they fit the budget; otherwise chunks of
    // consecutive blocks, cut on the host from the slot offsets
    const int64_t total_slots = d2h_i64(slot_off + nl, s);
    const int64_t budget_elems = std::max<int64_t>(in.pool_budget_bytes / esize, 1);
    std::vector<int64_t> hoff;
    int64_t pool_elems = std::max<int64_t>(total_slots, 1);
    if (total_slots > budget_elems) {
      hoff.resize(nl + 1);
      HM_HIP(hipMemcpyAsync(hoff.data(), slot_off, (nl + 1) * sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
      HM_HIP(hipStreamSynchronize(s));
      int64_t maxslot = 0;
      for (int64_t b = 0; b < nl; ++b) maxslot = std::max(maxslot, hoff[b + 1] - hoff[b]);
      pool_elems = std::max(budget_elems, maxslot);
    }
    auto slot_at = [&](int64_t b) { return hoff.empty() ? (b == 0 ? 0 : total_slots) : hoff[b]; };
    // the working slots come from the block cache and go back to it: handing a
    // block of this size back to the stream-ordered pool made its next
    // operation wait for milliseconds
    size_t pool_bytes = (size_t)pool_elems * esize;
    T* pool = static_cast<T*>(cache_take(pool_bytes, &pool_bytes));
    if (!pool) pool = static_cast<T*>(dalloc(pool_bytes, s));
    if (scaled) {
      // at most min(kmax, m, n) terms per block
      int64_t* kc = ta.get<int64_t>(nl);
      int64_t* ko = ta.get<int64_t>(nl + 1);
      k_term_caps<<<grid_for(nl, 256), 256, 0, s>>>(in.lr, nl, in.cl, kmax, kc);
      HM_LAUNCH_CHECK();
      const int64_t maxterms = scan_total(kc, ko, nl, tmp, s);
      out.su = static_cast<float*>(alloc((size_t)(maxterms + 1) * sizeof(float)));
    }
    int64_t* cflags = ta.get<int64_t>(kAcaClasses * nl);
    int64_t* coffs = ta.get<int64_t>(kAcaClasses * nl);
    int32_t* clists = ta.get<int32_t>(kAcaClasses * nl);
    int64_t* toffc = ta.get<int64_t>(nl + 1);
    int64_t* rk64 = ta.get<int64_t>(nl);
    int64_t* voff = ta.get<int64_t>(nl + 1);
    int32_t* vwid = ta.get<int32_t>(nl + 1);
    uint64_t* vptr = ta.get<uint64_t>(nl);
    int64_t* oU = ta.get<int64_t>(nl + 1);
    AcaSlot* desc = ta.get<AcaSlot>(nl);
    int64_t* rmark = ta.get<int64_t>(nl);
    int64_t* rsize = ta.get<int64_t>(nl);
    int64_t* roff = ta.get<int64_t>(nl + 1);
    int* head = ta.get<int>(kAcaClasses);
    const auto aca = in.op == kOpGalerkin ? run_aca<T, kOpGalerkin> : run_aca<T, kOpColloc>;
    out.bins = default_aca_bins(in.op);
    if (in.tune_aca) {
      const auto tune = in.op == kOpGalerkin ? tune_aca_bins<T, kOpGalerkin>
                                             : tune_aca_bins<T, kOpColloc>;
      out.bins = tune(g, in, k1, in.eps, pool, pool_elems, desc, head, out.rank, out.info,
                      out.aca_tune, s);
    }
    int64_t b0 = 0;
    while (b0 < nl) {
      int64_t b1 = hoff.empty() ? nl : b0 + 1;
      while (b1 < nl && hoff[b1 + 1] - hoff[b0] <= pool_elems) ++b1;
      const int64_t slot0 = slot_at(b0);
      const int64_t nb = b1 - b0;
      k_slot_desc<T><<<grid_for(nb, 256), 256, 0, s>>>(in.lr + b0, nb, in.cl, k1, slot_off + b0,
                                                       slot0, pool, nullptr, desc + b0);
      HM_LAUNCH_CHECK();
      aca(g, in.lr + b0, nb, in.cl, desc + b0, k1, in.eps, nullptr, out.bins, cflags, coffs, clists,
                 head, out.rank + b0, out.info + b0, tmp, s);
      T* pool2 = nullptr;
      if (k1 < kmax) {
        k_rerun_marks<T><<<grid_for(nb, 256), 256, 0, s>>>(in.lr + b0, nb, in.cl, out.info + b0,
                                                           k1, kmax, rmark, rsize);
        HM_LAUNCH_CHECK();
        const int64_t elems2 = scan_total(rsize, roff, nb, tmp, s);
        if (elems2 > 0) {
          pool2 = static_cast<T*>(dalloc((size_t)elems2 * esize, s));
          k_slot_desc<T><<<grid_for(nb, 256), 256, 0, s>>>(in.lr + b0, nb, in.cl, kmax, roff, 0,
                                                           pool2, rmark, desc + b0);
          HM_LAUNCH_CHECK();
          aca(g, in.lr + b0, nb, in.cl, desc + b0, kmax, in.eps, rmark, out.bins, cflags, coffs,
                     clists, head, out.rank + b0, out.info + b0, tmp, s);
          ++out.aca_reruns;
        }
      }
      HM_HIP(hipStreamSynchronize(s));
      const auto tp = clk::now();
      // column-cluster groups: term offsets in t (sorted order) and the V
      // panel layout
      Temps tg{s, {}};
      uint64_t* gkey = tg.get<uint64_t>(nb);
      int32_t* gidx = tg.get<int32_t>(nb);
      int64_t* gfirst = tg.get<int64_t>(nb);
      int64_t* gpos = tg.get<int64_t>(nb + 1);
      int64_t* tsort = tg.get<int64_t>(nb + 1);
      k_group_keys<<<grid_for(nb, 256), 256, 0, s>>>(in.lr + b0, nb, in.cl_leaves, in.ldpre, gkey,
                                                     gidx);
      HM_LAUNCH_CHECK();
      radix_sort_u64_i32(gkey, gidx, nb, 32, s);
      k_group_marks<<<grid_for(nb, 256), 256, 0, s>>>(gkey, gidx, nb, out.rank + b0, rk64, gfirst);
      HM_LAUNCH_CHECK();
      scan_excl_i64(rk64, tsort, nb, tsort + nb, s);
      const int64_t terms = d2h_i64(tsort + nb, s);
      const int64_t ngr = scan_total(gfirst, gpos, nb, tmp, s);
      int64_t* gstart = tg.get<int64_t>(ngr + 1);
      int64_t* gw = tg.get<int64_t>(ngr + 1);
      int64_t* gsz = tg.get<int64_t>(ngr + 1);
      int64_t* goff = tg.get<int64_t>(ngr + 1);
      int64_t* gcnt = tg.get<int64_t>(ngr + 1);
      int64_t* guoff = tg.get<int64_t>(ngr + 1);
      k_group_starts<<<grid_for(nb, 256), 256, 0, s>>>(gfirst, gpos, nb, gstart);
      HM_LAUNCH_CHECK();
      k_group_sizes<<<grid_for(ngr, 256), 256, 0, s>>>(gstart, ngr, nb, tsort, gidx, in.lr + b0,
                                                       in.cl_leaves, in.ldpre, gw, gsz);
      HM_LAUNCH_CHECK();
      const int64_t velems = scan_total(gsz, goff, ngr, tmp, s);
      k_block_vlayout<<<grid_for(nb, 256), 256, 0, s>>>(gidx, gpos, gfirst, nb, tsort, gstart, gw,
                                                        goff, in.lr + b0, in.cl_leaves, in.ldpre,
                                                        toffc, voff, vwid);
      HM_LAUNCH_CHECK();
      // V factors
      TL* varena = static_cast<TL*>(alloc((size_t)velems * lsize));
      k_pack_v<T, TL><<<grid_for(nb, 4, 1 << 20), 256, 0, s>>>(in.lr + b0, nb, in.cl, L,
                                                               out.rank + b0, desc + b0, voff,
                                                               vwid, varena, vptr);
      HM_LAUNCH_CHECK();
      k_lr_meta<<<grid_for(nb, 256), 256, 0, s>>>(in.lr + b0, nb, in.cl_leaves, in.ldpre,
                                                  out.rank + b0, toffc, toff_base, vptr, vwid,
                                                  ub + b0, out.meta + b0);
      HM_LAUNCH_CHECK();
      // phase-1 units of the chunk
      {
        // rows per granule and loads per lane of the one-column phase-1
        // kernel (FP16 slices: eight loads of 8 bytes)
        const int gran = sizeof(TL) == 8 ? 2 : 4;
        const int passes = sizeof(TL) == 2 ? 8 : 4;
        k_group_units<<<grid_for(ngr, 256), 256, 0, s>>>(gstart, ngr, gkey, gidx, gw, in.lr + b0,
                                                         in.cl_leaves, in.ldpre, gran, passes,
                                                         gcnt);
        HM_LAUNCH_CHECK();
        const int64_t nu = scan_total(gcnt, guoff, ngr, tmp, s);
        LrMeta* um = keep.get<LrMeta>(nu + 1);
        k_emit_units<<<grid_for(ngr, 256), 256, 0, s>>>(gstart, ngr, gkey, gidx, gw, goff, guoff,
                                                        tsort, toff_base, out.meta + b0, gran,
                                                        passes, (uint64_t)(uintptr_t)varena, lsize,
                                                        um);
        HM_LAUNCH_CHECK();
        unit_parts.push_back({um, nu});
      }
      HM_HIP(hipStreamSynchronize(s));
      tg.release();
      // U slices in row-leaf panels
      Temps tu{s, {}};
      PanelSet PU;
      panel_layout(in.lr + b0, nb, in.cl, in.cl_leaves, in.ldpre, nleaf, out.rank + b0, oU, PU,
                   tu, tmp, s);
      TL* uarena = static_cast<TL*>(alloc((size_t)PU.elems * lsize));
      if (scaled && nb > 0) {
        k_u_scales<T><<<grid_for(nb, 4, 1 << 20), 256, 0, s>>>(
            in.lr + b0, nb, in.cl, out.rank + b0, desc + b0, toffc, toff_base, out.su);
        HM_LAUNCH_CHECK();
      }
      if (PU.np > 0) {
        k_pack_u<T, TL><<<grid_for(PU.np, 4, 1 << 20), 256, 0, s>>>(
            PU.sidx, PU.ib, PU.ilf, PU.np, in.lr + b0, in.cl, L, out.rank + b0, desc + b0,
            PU.offI, scaled ? out.su : nullptr, toffc, toff_base, uarena);
        HM_LAUNCH_CHECK();
      }
      const int64_t colbase = out.dense_cols + ucols;
      int32_t* cm = keep.get<int32_t>(PU.cols);
      k_colmap<<<grid_for(PU.np, 256), 256, 0, s>>>(PU.sidx, PU.ib, PU.np, PU.gcol, PU.wid,
                                                    in.lr + b0, in.cl, toffc, toff_base, n, cm);
      HM_LAUNCH_CHECK();
      colmap_parts.push_back({cm, PU.cols});
      Run* rc = keep.get<Run>(nleaf);
      k_runs<<<grid_for(nleaf, 256), 256, 0, s>>>(PU.col0, PU.W, PU.poff, nleaf,
                                                  (uint64_t)(uintptr_t)uarena, lsize, colbase, rc);
      HM_LAUNCH_CHECK();
      run_parts.push_back(rc);
      k_urec<<<grid_for(PU.np, 256), 256, 0, s>>>(PU.sidx, PU.ib, PU.ilf, PU.np, in.lr + b0,
                                                  in.cl_leaves, ub + b0, PU.gcol, colbase, PU.offI,
                                                  (uint64_t)(uintptr_t)uarena, lsize, out.ucol,
                                                  out.uptr);
      HM_LAUNCH_CHECK();
      HM_HIP(hipStreamSynchronize(s));
      tu.release();
      if (pool2) dfree(pool2, s);
      ms_pack += ms_since(tp);
      toff_base += terms;
      ucols += PU.cols;
      out.lr_elems += velems + PU.elems;
      ++out.nchunks;
      b0 = b1;
    }
    HM_HIP(hipStreamSynchronize(s));
    cache_put(pool, pool_bytes);
  }
  out.toff_total = toff_base;
  if (toff_base >= INT32_MAX) throw Error{HM_ERR_STATE, "more than 2^31 low-rank terms"};
  {
    int64_t nu = 0;
    for (auto& up : unit_parts) nu += up.second;
    out.nu1 = nu;
    out.meta1 = static_cast<LrMeta*>(alloc((size_t)(nu + 1) * sizeof(LrMeta)));
    int64_t o = 0;
    for (auto& up : unit_parts) {
      if (up.second)
        HM_HIP(hipMemcpyAsync(out.meta1 + o, up.first, up.second * sizeof(LrMeta),
                              hipMemcpyDeviceToDevice, s));
      o += up.second;
    }
  }
  out.ms_aca = ms_since(t0) - ms_pack;

  // ---- product plan: runs, column map, transposed items
  t0 = clk::now();
  out.nruns = (int)run_parts.size();
  out.runs = static_cast<Run*>(alloc((size_t)out.nruns * nleaf * sizeof(Run)));
  for (int k = 0; k < out.nruns; ++k)
    HM_HIP(hipMemcpyAsync(out.runs + (int64_t)k * nleaf, run_parts[k], nleaf * sizeof(Run),
                          hipMemcpyDeviceToDevice, s));
  make_units(out, in.ldpre, nleaf, kUnitCols, alloc, s);
  out.ncols = out.dense_cols + ucols;
  out.colmap = static_cast<int32_t*>(alloc((out.ncols + 1) * sizeof(int32_t)));
  {
    int64_t o = 0;
    for (auto& pc : colmap_parts) {
      if (pc.second)
        HM_HIP(hipMemcpyAsync(out.colmap + o, pc.first, pc.second * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, s));
      o += pc.second;
    }
  }
  {
    Temps tt{s, {}};
    const int64_t nb_all = in.nd + out.nu1;
    int64_t* cnt = tt.get<int64_t>(nb_all);
    int64_t* off = tt.get<int64_t>(nb_all + 1);
    k_titem_counts<<<grid_for(nb_all, 256), 256, 0, s>>>(in.dns, in.nd, out.meta1, out.nu1,
                                                         in.cl_leaves, cnt);
    HM_LAUNCH_CHECK();
    out.ntitems = scan_total(cnt, off, nb_all, tmp, s);
    if (out.ntitems >= INT32_MAX) throw Error{HM_ERR_STATE, "more than 2^31 transposed items"};
    TItem* raw = tt.get<TItem>(out.ntitems);
    uint64_t* key = tt.get<uint64_t>(out.ntitems);
    int32_t* idx = tt.get<int32_t>(out.ntitems);
    k_titem_expand<<<grid_for(nb_all, 64), 64, 0, s>>>(in.dns, in.nd, out.nu1, in.cl, L, off, invD,
                                                       oD, gcolD, out.meta1, lsize, raw, key, idx);
    HM_LAUNCH_CHECK();
    radix_sort_u64_i32(key, idx, out.ntitems, bits_for(nleaf), s);
    out.titems = static_cast<TItem*>(alloc((out.ntitems + 1) * sizeof(TItem)));
    k_gather_titems<<<grid_for(out.ntitems, 256), 256, 0, s>>>(raw, idx, out.ntitems, out.titems);
    HM_LAUNCH_CHECK();
    int64_t* lb = tt.get<int64_t>(nleaf + 1);
    k_seg_begins<<<grid_for(nleaf + 1, 256), 256, 0, s>>>(key, out.ntitems, nleaf, lb);
    HM_LAUNCH_CHECK();
    out.tbeg = static_cast<int32_t*>(alloc((nleaf + 1) * sizeof(int32_t)));
    k_to_i32<<<grid_for(nleaf + 1, 256), 256, 0, s>>>(lb, nleaf + 1, out.tbeg);
    HM_LAUNCH_CHECK();
    HM_HIP(hipStreamSynchronize(s));
  }
  out.ms_pack = ms_pack + ms_since(t0);
  keep.release();
}
template void build_storage<float, float>(const Geom<float>&, const SetupIn&, Storage&,
                                          const Alloc&, hipStream_t);
template void build_storage<double, double>(const Geom<double>&, const SetupIn&, Storage&,
                                            const Alloc&, hipStream_t);
template void build_storage<float, _Float16>(const Geom<float>&, const SetupIn&, Storage&,
                                             const Alloc&, hipStream_t);

template <typename TL, typename TO>
void launch_unpack(const int2* lr, int64_t b, const Cluster* cl, const int32_t* leaf_lo,
                   const int32_t* leaf_m, const int64_t* ldpre, const int2* cl_leaves,
                   const LrMeta* meta, const uint64_t* uptr, const float* su, TO* out,
                   int64_t total, hipStream_t s) {
  LeafTab L{leaf_lo, leaf_m, ldpre, cl_leaves};
  k_unpack<TL, TO><<<grid_for(total, 256), 256, 0, s>>>(lr, b, cl, L, meta, uptr, su, out);
  HM_LAUNCH_CHECK();
}
#define HM_UNPACK(TL, TO)                                                                          \
  template void launch_unpack<TL, TO>(const int2*, int64_t, const Cluster*, const int32_t*,        \
                                      const int32_t*, const int64_t*, const int2*, const LrMeta*, \
                                      const uint64_t*, const float*, TO*, int64_t, hipStream_t);
HM_UNPACK(float, float)
HM_UNPACK(double, double)
HM_UNPACK(_Float16, float)
#undef HM_UNPACK

}  // namespace hm
