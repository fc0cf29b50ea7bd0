// H-matrix-vector products y = H x and y = H^T x (Sec. 2.3, last paragraph:
// dense leaves apply their stored block, admissible leaves the low-rank
// factors), organised per leaf cluster so that every output row is owned by
// exactly one workgroup: no atomics, fixed summation order, bitwise
// reproducible.
//
//   forward    t_b = V_b^T x_sigma            (per column leaf, then per block)
//              y_c = sum dense D x + sum U t  (per row leaf)
//   transposed s_b = U_b^T x_tau              (per row leaf, then per block)
//              y_c = sum D^T x + sum V s      (per column leaf)
//
// A slice is column-major with ld a multiple of 4.  A wavefront reads it in
// 16-byte granules: lane = (column group cg, row granule g) with R = ld/G row
// granules per column and C = 64/R columns per instruction.
#include "hm_internal.h"

namespace hm {

template <typename T>
struct Gran;
template <>
struct Gran<float> {
  using V = float4;
  static constexpr int G = 4;
  __device__ static inline void load(const float* p, float* o) {
    float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct Gran<double> {
  using V = double2;
  static constexpr int G = 2;
  __device__ static inline void load(const double* p, double* o) {
    double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x; o[1] = v.y;
  }
};



// Sum of v over the R lanes g = 0..R-1 of a lane segment; the result is
// valid in the lane with g == 0.  Every lane of the wavefront must call it.
template <typename A>
__device__ inline A seg_sum(A v, int g, int R) {
  for (int s = 1; s < R; s <<= 1) {
    A o = __shfl_down(v, s, 64);
    if (g + s < R) v += o;
  }
  return v;
}

// ------------------------------------------------------------------ gather / scatter
// xp[p][k] = x[perm[p]][k0 + k] for one block of NR right-hand sides.
template <typename VT, typename A>
__global__ void k_gather(const VT* __restrict__ x, int nrhs, int k0, int nr,
                         const int32_t* __restrict__ perm, int64_t n, A* __restrict__ xp) {
  const int64_t tot = n * nr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / nr;
    const int k = (int)(e % nr);
    xp[e] = (A)x[(int64_t)perm[p] * nrhs + k0 + k];
  }
}

// ------------------------------------------------------------------ phase 1
// For every leaf: partial[(aux + j)][k] = sum_i S[j*ld + i] x_leaf[i][k] over
// the low-rank slices (kind 1) of its list.
template <typename T, typename A, int NR>
__global__ __launch_bounds__(256) void k_mv_phase1(const int32_t* __restrict__ beg,
                                                   const Item* __restrict__ items, MvLeaves L,
                                                   const A* __restrict__ xp, A* __restrict__ partial) {
  constexpr int G = Gran<T>::G;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t c = blockIdx.x; c < L.nleaf; c += gridDim.x) {
    const int ld = (int)(L.ldpre[c + 1] - L.ldpre[c]);
    const int R = ld / G, C = 64 / R;
    const int cg = lane / R, g = lane % R;
    const bool act = cg < C;
    const int m = L.m[c], lo = L.lo[c];
    A xg[G][NR];
#pragma unroll
    for (int e = 0; e < G; ++e) {
      const int row = g * G + e;
#pragma unroll
      for (int k = 0; k < NR; ++k)
        xg[e][k] = (act && row < m) ? xp[(int64_t)(lo + row) * NR + k] : (A)0;
    }
    const int b0 = beg[c], b1 = beg[c + 1];
    for (int it = b0 + wave; it < b1; it += 4) {
      const Item I = items[it];
      if (I.kind != 1) continue;
      const T* S = reinterpret_cast<const T*>((uintptr_t)I.data);
      for (int j0 = 0; j0 < I.w; j0 += C) {
        const int j = j0 + cg;
        A p[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) p[k] = 0;
        if (act && j < I.w) {
          T s[G];
          Gran<T>::load(S + (int64_t)j * ld + g * G, s);
#pragma unroll
          for (int e = 0; e < G; ++e)
#pragma unroll
            for (int k = 0; k < NR; ++k) p[k] += (A)s[e] * xg[e][k];
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) p[k] = seg_sum(p[k], g, R);
        if (act && g == 0 && j < I.w) {
#pragma unroll
          for (int k = 0; k < NR; ++k) partial[(int64_t)(I.aux + j) * NR + k] = p[k];
        }
      }
    }
  }
}

// t[(toff + l)][k] = sum_q partial[(pslot + q r + l)][k], q < nk.
// meta[b] = (toff, pslot, r, nk_rows, nk_cols, -) per low-rank block.
template <typename A, int NR>
__global__ void k_mv_sum(const int64_t* __restrict__ meta, int64_t nl, int use_rows,
                         const A* __restrict__ partial, A* __restrict__ t) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nl;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t* M = meta + 6 * b;
    const int64_t toff = M[0], ps = M[1], r = M[2], nk = use_rows ? M[3] : M[4];
    for (int64_t l = 0; l < r; ++l) {
      A acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = 0;
      for (int64_t q = 0; q < nk; ++q)
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] += partial[(ps + q * r + l) * NR + k];
#pragma unroll
      for (int k = 0; k < NR; ++k) t[(toff + l) * NR + k] = acc[k];
    }
  }
}

// ------------------------------------------------------------------ phase 2
// For every leaf c, y_c = sum over its list:
//   kind 1 (and kind 0 when !transposed): y += S z[src ..], z = t (kind 1) or
//     xp (kind 0)                                         ("N" product)
//   kind 0 when transposed: y[j] += sum_i S[j*ld_s + i] xp[lo_s + i] with
//     the slice's own row leaf s = aux                     ("T" product)
// then y[perm[lo + i]][k0 + k] = result.
template <typename T, typename A, typename VT, int NR>
__global__ __launch_bounds__(256) void k_mv_phase2(const int32_t* __restrict__ beg,
                                                   const Item* __restrict__ items, MvLeaves L,
                                                   const A* __restrict__ xp, const A* __restrict__ t,
                                                   int transposed, const int32_t* __restrict__ perm,
                                                   VT* __restrict__ y, int nrhs, int k0) {
  constexpr int G = Gran<T>::G;
  __shared__ A ybuf[4][kMaxLeaf][NR];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t c = blockIdx.x; c < L.nleaf; c += gridDim.x) {
    const int ld = (int)(L.ldpre[c + 1] - L.ldpre[c]);
    const int R = ld / G, C = 64 / R;
    const int cg = lane / R, g = lane % R;
    const bool act = cg < C;
    const int m = L.m[c], lo = L.lo[c];
    A acc[G][NR];
    A yT[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      yT[k] = 0;
#pragma unroll
      for (int e = 0; e < G; ++e) acc[e][k] = 0;
    }
    const int b0 = beg[c], b1 = beg[c + 1];
    for (int it = b0 + wave; it < b1; it += 4) {
      const Item I = items[it];
      const T* S = reinterpret_cast<const T*>((uintptr_t)I.data);
      if (I.kind == 1 || !transposed) {
        const A* z = (I.kind == 1) ? t : xp;
        for (int j0 = 0; j0 < I.w; j0 += C) {
          const int j = j0 + cg;
          if (act && j < I.w) {
            T s[G];
            Gran<T>::load(S + (int64_t)j * ld + g * G, s);
            A zz[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) zz[k] = z[(int64_t)(I.src + j) * NR + k];
#pragma unroll
            for (int e = 0; e < G; ++e)
#pragma unroll
              for (int k = 0; k < NR; ++k) acc[e][k] += (A)s[e] * zz[k];
          }
        }
      } else {
        // dense block seen from its column leaf: T product with the row leaf's x
        const int sl = I.aux;
        const int lds = (int)(L.ldpre[sl + 1] - L.ldpre[sl]);
        const int Rs = lds / G, Cs = 64 / Rs;
        const int cgs = lane / Rs, gs = lane % Rs;
        const bool acts = cgs < Cs;
        const int ms = L.m[sl], los = L.lo[sl];
        A xg[G][NR];
#pragma unroll
        for (int e = 0; e < G; ++e) {
          const int row = gs * G + e;
#pragma unroll
          for (int k = 0; k < NR; ++k)
            xg[e][k] = (acts && row < ms) ? xp[(int64_t)(los + row) * NR + k] : (A)0;
        }
        for (int j0 = 0; j0 < I.w; j0 += Cs) {
          const int j = j0 + cgs;
          A p[NR];
#pragma unroll
          for (int k = 0; k < NR; ++k) p[k] = 0;
          if (acts && j < I.w) {
            T s[G];
            Gran<T>::load(S + (int64_t)j * lds + gs * G, s);
#pragma unroll
            for (int e = 0; e < G; ++e)
#pragma unroll
              for (int k = 0; k < NR; ++k) p[k] += (A)s[e] * xg[e][k];
          }
#pragma unroll
          for (int k = 0; k < NR; ++k) p[k] = seg_sum(p[k], gs, Rs);
          // column j0 + q lives in lane q*Rs; move it to lane (output row) j0 + q
          const int q = lane - j0;
          const int src = (q >= 0 && q < Cs) ? q * Rs : 0;
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            const A v = __shfl(p[k], src, 64);
            if (q >= 0 && q < Cs && q < I.w - j0) yT[k] += v;
          }
        }
      }
    }
    // combine the column groups of the N products (tree over cg, stride R)
#pragma unroll
    for (int e = 0; e < G; ++e)
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        A v = acc[e][k];
        for (int s = 1; s < C; s <<= 1) {
          A o = __shfl_down(v, s * R, 64);
          if (cg + s < C) v += o;
        }
        acc[e][k] = v;
      }
    if (cg == 0) {
#pragma unroll
      for (int e = 0; e < G; ++e) {
        const int row = g * G + e;
        if (row < kMaxLeaf)
#pragma unroll
          for (int k = 0; k < NR; ++k) ybuf[wave][row][k] = acc[e][k];
      }
    }
    __syncthreads();
    if (lane < m) {
#pragma unroll
      for (int k = 0; k < NR; ++k) ybuf[wave][lane][k] += yT[k];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * NR; e += blockDim.x) {
      const int row = e / NR, k = e % NR;
      const A v = ((ybuf[0][row][k] + ybuf[1][row][k]) + ybuf[2][row][k]) + ybuf[3][row][k];
      y[(int64_t)perm[lo + row] * nrhs + k0 + k] = (VT)v;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ host side


template <typename T, typename A, typename VT, int NR>
static void mv_chunk(const MvPlan& P, const VT* x, VT* y, int nrhs, int k0, bool transposed,
                     hipStream_t s) {
  A* xp = static_cast<A*>(P.xp);
  A* partial = static_cast<A*>(P.partial);
  A* t = static_cast<A*>(P.t);
  MvProfile* pr = P.prof;
  if (pr) HM_HIP(hipEventRecord(pr->ev[0], s));
  k_gather<VT, A><<<grid_for(P.n * NR, 256, 4096), 256, 0, s>>>(x, nrhs, k0, NR, P.perm, P.n, xp);
  HM_LAUNCH_CHECK();
  if (pr) HM_HIP(hipEventRecord(pr->ev[1], s));
  const int32_t* b1 = transposed ? P.row_beg : P.col_beg;
  const Item* i1 = transposed ? P.row_items : P.col_items;
  const int32_t* b2 = transposed ? P.col_beg : P.row_beg;
  const Item* i2 = transposed ? P.col_items : P.row_items;
  const unsigned g = (unsigned)std::min<int64_t>(P.L.nleaf, P.grid);
  if (P.nlr > 0) {
    k_mv_phase1<T, A, NR><<<g, 256, 0, s>>>(b1, i1, P.L, xp, partial);
    HM_LAUNCH_CHECK();
  }
  if (pr) HM_HIP(hipEventRecord(pr->ev[2], s));
  if (P.nlr > 0) {
    k_mv_sum<A, NR><<<grid_for(P.nlr, 256), 256, 0, s>>>(P.lr_meta, P.nlr, transposed ? 1 : 0,
                                                          partial, t);
    HM_LAUNCH_CHECK();
  }
  if (pr) HM_HIP(hipEventRecord(pr->ev[3], s));
  k_mv_phase2<T, A, VT, NR><<<g, 256, 0, s>>>(b2, i2, P.L, xp, t, transposed ? 1 : 0, P.perm, y,
                                               nrhs, k0);
  HM_LAUNCH_CHECK();
  if (pr) {
    HM_HIP(hipEventRecord(pr->ev[4], s));
    HM_HIP(hipEventSynchronize(pr->ev[4]));
    for (int k = 0; k < 4; ++k) {
      float ms = 0.f;
      HM_HIP(hipEventElapsedTime(&ms, pr->ev[k], pr->ev[k + 1]));
      pr->ms[k] += ms;
      pr->launches[k] += 1;
    }
  }
}

template <typename T, typename A, typename VT>
void matvec_impl(const MvPlan& P, const VT* x, VT* y, int nrhs, bool transposed, hipStream_t s) {
  int k0 = 0;
  while (k0 < nrhs) {
    const int left = nrhs - k0;
    if (left >= 16) {
      mv_chunk<T, A, VT, 16>(P, x, y, nrhs, k0, transposed, s);
      k0 += 16;
    } else if (left >= 8) {
      mv_chunk<T, A, VT, 8>(P, x, y, nrhs, k0, transposed, s);
      k0 += 8;
    } else if (left >= 4) {
      mv_chunk<T, A, VT, 4>(P, x, y, nrhs, k0, transposed, s);
      k0 += 4;
    } else if (left >= 2) {
      mv_chunk<T, A, VT, 2>(P, x, y, nrhs, k0, transposed, s);
      k0 += 2;
    } else {
      mv_chunk<T, A, VT, 1>(P, x, y, nrhs, k0, transposed, s);
      k0 += 1;
    }
  }
}

// storage T, vectors VT; accumulation in double unless both are float
void matvec_dispatch(const MvPlan& P, int storage_f32, const void* x, void* y, int nrhs, int vec_f32,
                     bool transposed, hipStream_t s) {
  if (storage_f32 && vec_f32)
    matvec_impl<float, float, float>(P, (const float*)x, (float*)y, nrhs, transposed, s);
  else if (storage_f32 && !vec_f32)
    matvec_impl<float, double, double>(P, (const double*)x, (double*)y, nrhs, transposed, s);
  else if (!storage_f32 && vec_f32)
    matvec_impl<double, double, float>(P, (const float*)x, (float*)y, nrhs, transposed, s);
  else
    matvec_impl<double, double, double>(P, (const double*)x, (double*)y, nrhs, transposed, s);
}

}  // namespace hm
