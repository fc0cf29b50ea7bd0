// H-matrix-vector products y = H x and y = H^T x (Sec. 2.3, last paragraph:
// dense leaves apply their stored block, admissible leaves the low-rank
// factors), with every output row owned by exactly one workgroup: no atomics,
// a fixed summation order, bitwise reproducible results.
//
// Storage (built by the setup):
//   row panels  for every row leaf c, its dense slices and (per ACA chunk) its
//               U slices are each one contiguous column-major panel
//               ld_c x W; column j of a panel multiplies z[colmap[col0 + j]]
//               where z = [x in Morton order ; t]
//   V blocks    the V factor of every admissible block is contiguous: its
//               column-leaf slices (ld x r, column-major) one after another
//
//   forward     z[0..n)      = x[perm]                          (gather)
//               z[n + toff_b + l] = sum_i V_b[i][l] x_sigma[i] (one wavefront
//                                                               per block)
//               y_c = sum over the row panels of c of  P z[map]  (per leaf)
//   transposed  w[col] = sum_i P[i][col] x_c[i] for every panel column
//               (per row leaf), s_b[l] = sum over the row leaves of b of the
//               w of its U columns (per block), then per column leaf
//               y_c = sum over dense blocks of the w entries of its columns
//                   + sum over its V slices of V s_b
//
// A wavefront reads a slice in 16-byte granules: lane = (column group cg,
// row granule g), R = ld/G row granules per column, C = 64/R columns per
// instruction.
#include <type_traits>

#include "hm_internal.h"

namespace hm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// Granule loads of G stored values per lane, returned in the arithmetic type
// E; the stored operator is streamed once per product, so the loads are
// non-temporal.  FP32 and FP16 granules both cover 4 rows (16 and 8 bytes),
// so dense and FP16 factor panels of a leaf share one lane layout.
template <typename T>
struct Gran;
template <>
struct Gran<float> {
  using E = float;
  static constexpr int G = 4;
  __device__ static inline void load(const float* p, float* o) {
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct Gran<double> {
  using E = double;
  static constexpr int G = 2;
  __device__ static inline void load(const double* p, double* o) {
    const f64x2 v = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
    o[0] = v.x; o[1] = v.y;
  }
};
template <>
struct Gran<_Float16> {
  using E = float;
  static constexpr int G = 4;
  __device__ static inline void load(const _Float16* p, float* o) {
    const f16x4 v = __builtin_nontemporal_load(reinterpret_cast<const f16x4*>(p));
    o[0] = (float)v.x; o[1] = (float)v.y; o[2] = (float)v.z; o[3] = (float)v.w;
  }
};

// NR consecutive values z[0..NR) (16-byte aligned when NR * sizeof(A) is a
// multiple of 16: z rows are NR values long and the buffer is 256-byte aligned).
template <typename A, int NR>
__device__ inline void load_row(const A* __restrict__ p, A (&o)[NR]) {
  if constexpr (sizeof(A) == 8 && NR % 2 == 0) {
#pragma unroll
    for (int k = 0; k < NR; k += 2) {
      const f64x2 v = *reinterpret_cast<const f64x2*>(p + k);
      o[k] = v.x;
      o[k + 1] = v.y;
    }
  } else if constexpr (sizeof(A) == 4 && NR % 4 == 0) {
#pragma unroll
    for (int k = 0; k < NR; k += 4) {
      const f32x4 v = *reinterpret_cast<const f32x4*>(p + k);
      o[k] = v.x;
      o[k + 1] = v.y;
      o[k + 2] = v.z;
      o[k + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NR; ++k) o[k] = p[k];
  }
}

// Sum of v over the R lanes g = 0..R-1 of a lane segment; valid in the lane
// with g == 0.  Every lane of the wavefront must call it.
template <typename A>
__device__ inline A seg_sum(A v, int g, int R) {
  for (int s = 1; s < R; s <<= 1) {
    const A o = __shfl_down(v, s, 64);
    if (g + s < R) v += o;
  }
  return v;
}

// Workgroup w runs on XCD w mod 8 (8 XCDs, each with its own L2).  Logical
// index li -> item (li mod 8) * per + li / 8 gives every XCD a contiguous
// range of leaves, so neighbouring leaves, which
// gather mostly the same x and t values, share one L2.  A bijection of
// [0, 8 per) onto itself; items >= the count are skipped.
constexpr int kXcds = 8;
__device__ inline int64_t xcd_item(int64_t li, int64_t per) {
  return (li % kXcds) * per + li / kXcds;
}

// ------------------------------------------------------------------ gather
template <typename VT, typename A>
__global__ void k_gather(const VT* __restrict__ x, int nrhs, int k0, int nr,
                         const int32_t* __restrict__ perm, int64_t n, A* __restrict__ z) {
  const int64_t tot = n * nr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / nr;
    const int k = (int)(e % nr);
    z[e] = (A)x[(int64_t)perm[p] * nrhs + k0 + k];
  }
}

// ------------------------------------------------------------------ forward, phase 1
// One wavefront per admissible block: t_b = V_b^T x_sigma (times the U scale
// when the factors are FP16), written to z[n + toff + l].
//
// Lane = (column group cg, row granule g); the P = ceil(r / C) passes of C
// columns each keep a register accumulator.  When all column-leaf slices
// share one ld (the usual case) the x granule is loaded once per slice, the
// accumulators run over all slices, and each pass is reduced once at the
// end; otherwise every slice is reduced on its own.  Column sums move to
// lane l, which owns term l.
template <typename A, int NR>
__device__ inline void fwd1_flush(A (&p)[NR], int g, int R, int j0, int C, int r, int lane,
                                  A (&tl)[NR]) {
#pragma unroll
  for (int k = 0; k < NR; ++k) p[k] = seg_sum(p[k], g, R);
  const int q = lane - j0;
  const bool mine = q >= 0 && q < C && lane < r;
  const int src = mine ? q * R : 0;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const A v = __shfl(p[k], src, 64);
    if (mine) tl[k] += v;
  }
}

// The slices of one block with every column-leaf slice of ld rows: P passes
// of C columns, P known at compile time so that the granules of all passes
// are loaded with no branch between them and the x loads; columns past r
// read column r - 1 into accumulators that are never flushed.
template <typename T, typename A, int NR, int P>
__device__ inline void fwd1_uniform(const LrMeta& M, const MvLeaves& L, const A* __restrict__ z,
                                    int r, int ld, int R, int C, int cg, int g, bool act, int lane,
                                    A (&tl)[NR]) {
  constexpr int G = Gran<T>::G;
  A acc[P][NR];
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[q][k] = 0;
  // 32-bit element offsets of the lane's granule in each pass
  int off[P];
#pragma unroll
  for (int q = 0; q < P; ++q) off[q] = min(q * C + cg, r - 1) * ld + g * G;
  const int sstride = ld * M.vw;
  const T* Sl = reinterpret_cast<const T*>((uintptr_t)M.vptr);
  int lo = L.lo[M.sf];                       // the leaves of sigma are consecutive
  for (int lf = M.sf; lf <= M.sl; ++lf, Sl += sstride) {
    const int m = L.m[lf];
    typename Gran<T>::E sv[P][G];
#pragma unroll
    for (int q = 0; q < P; ++q) Gran<T>::load(Sl + off[q], sv[q]);
    A xg[G][NR];
#pragma unroll
    for (int e = 0; e < G; ++e) {
      // unconditional load of a clamped row, zeroed outside the slice
      const int row = g * G + e;
      const bool in = act && row < m;
      const A* zr = z + (int64_t)(lo + (in ? row : 0)) * NR;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const A v = zr[k];
        xg[e][k] = in ? v : (A)0;
      }
    }
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int e = 0; e < G; ++e)
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[q][k] += (A)sv[q][e] * xg[e][k];
    lo += m;
  }
#pragma unroll
  for (int q = 0; q < P; ++q) fwd1_flush<A, NR>(acc[q], g, R, q * C, C, r, lane, tl);
}

template <typename T, typename A, int NR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_fwd1(const LrMeta* __restrict__ meta, int64_t nl,
                                              MvLeaves L, A* __restrict__ z, int64_t n,
                                              const float* __restrict__ su) {
  constexpr int G = Gran<T>::G;
  // loads per lane of the one-pass form; the phase-1 units of FP16 slices
  // are sized for eight, of FP32 and FP64 ones for four
  constexpr int PMAX = (NR == 1 && sizeof(T) == 2) ? 8 : (NR <= 2 ? 4 : (NR <= 4 ? 2 : 1));
  const int lane = threadIdx.x & 63;
  // wave-uniform block index: descriptors and leaf data come in by scalar loads
  const int64_t wid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  // the next block's descriptor is loaded one iteration ahead
  LrMeta Mn;
  if (wid < nl) Mn = meta[wid];
  for (int64_t b = wid; b < nl; b += nw) {
    const LrMeta M = Mn;
    if (b + nw < nl) Mn = meta[b + nw];
    const int r = M.r;
    if (r == 0) continue;
    A tl[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) tl[k] = 0;
    const T* S = reinterpret_cast<const T*>((uintptr_t)M.vptr);
    const int R0 = M.vld / G, C0 = R0 > 0 ? 64 / R0 : 1;
    if (M.vld > 0 && r <= PMAX * C0 && r <= 64) {
      const int ld = M.vld, R = R0, C = C0;
      // lane / R by a multiply and shift (exact for lane < 64, R <= 64)
      const unsigned mul = (unsigned)(65536.0f / (float)R) + 1u;
      const int cg = (int)(((unsigned)lane * mul) >> 16), g = lane - cg * R;
      const bool act = cg < C;
      const int P = (r + C - 1) / C;
      switch (P) {                                      // uniform over the wavefront
        case 1: fwd1_uniform<T, A, NR, 1>(M, L, z, r, ld, R, C, cg, g, act, lane, tl); break;
        case 2:
          if constexpr (PMAX >= 2) fwd1_uniform<T, A, NR, 2>(M, L, z, r, ld, R, C, cg, g, act, lane, tl);
          break;
        case 3:
          if constexpr (PMAX >= 3) fwd1_uniform<T, A, NR, 3>(M, L, z, r, ld, R, C, cg, g, act, lane, tl);
          break;
        case 4:
          if constexpr (PMAX >= 4) fwd1_uniform<T, A, NR, 4>(M, L, z, r, ld, R, C, cg, g, act, lane, tl);
          break;
        case 5:
          if constexpr (PMAX >= 5) fwd1_uniform<T, A, NR, 5>(M, L, z, r, ld, R, C, cg, g, act, lane, tl);
          break;
        case 6:
          if constexpr (PMAX >= 6) fwd1_uniform<T, A, NR, 6>(M, L, z, r, ld, R, C, cg, g, act, lane, tl);
          break;
        case 7:
          if constexpr (PMAX >= 7) fwd1_uniform<T, A, NR, 7>(M, L, z, r, ld, R, C, cg, g, act, lane, tl);
          break;
        default:
          if constexpr (PMAX >= 8) fwd1_uniform<T, A, NR, 8>(M, L, z, r, ld, R, C, cg, g, act, lane, tl);
          break;
      }
    } else {
      // general path, 64 terms (one per lane) at a time
      for (int t0 = 0; t0 < r; t0 += 64) {
        const int rc = min(64, r - t0);
        const T* Sl = S;
#pragma unroll
        for (int k = 0; k < NR; ++k) tl[k] = 0;
        for (int lf = M.sf; lf <= M.sl; ++lf) {
          const int ld = (int)(L.ldpre[lf + 1] - L.ldpre[lf]);
          const int R = ld / G, C = 64 / R;
          const int cg = lane / R, g = lane % R;
          const bool act = cg < C;
          const int m = L.m[lf], lo = L.lo[lf];
          A xg[G][NR];
#pragma unroll
          for (int e = 0; e < G; ++e) {
            const int row = g * G + e;
#pragma unroll
            for (int k = 0; k < NR; ++k)
              xg[e][k] = (act && row < m) ? z[(int64_t)(lo + row) * NR + k] : (A)0;
          }
          for (int j0 = 0; j0 < rc; j0 += C) {
            const int j = j0 + cg;
            A p[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) p[k] = 0;
            if (act && j < rc) {
              typename Gran<T>::E sv[G];
              Gran<T>::load(Sl + (int64_t)(t0 + j) * ld + g * G, sv);
#pragma unroll
              for (int e = 0; e < G; ++e)
#pragma unroll
                for (int k = 0; k < NR; ++k) p[k] += (A)sv[e] * xg[e][k];
            }
            fwd1_flush<A, NR>(p, g, R, j0, C, rc, lane, tl);
          }
          Sl += (int64_t)ld * M.vw;
        }
        if (t0 + 64 < r && lane < rc) {       // every chunk but the last one
          const A sc = su ? (A)su[M.toff + t0 + lane] : (A)1;
#pragma unroll
          for (int k = 0; k < NR; ++k) z[(n + M.toff + t0 + lane) * NR + k] = tl[k] * sc;
        }
      }
    }
    // terms 64 q + lane of the last chunk q (the only chunk when r <= 64)
    const int tlast = r > 64 ? (r - 1) / 64 * 64 : 0;
    if (tlast + lane < r) {
      const A sc = su ? (A)su[M.toff + tlast + lane] : (A)1;
#pragma unroll
      for (int k = 0; k < NR; ++k) z[(n + M.toff + tlast + lane) * NR + k] = tl[k] * sc;
    }
  }
}

// Several right-hand sides (NR >= 4): lane = (term j, right-hand-side group
// kg) with JG terms per pass and KPL = NR JG / 64 right-hand sides per lane,
// so every lane owns complete sums and no cross-lane reduction is needed.
// All lanes walk the same rows; a lane reads its term's granule (shared by the
// lanes of other groups) and its KPL values of each x row.
template <typename T, typename A, int NR, int JG>
__device__ inline void fwd1m_block(const LrMeta& M, const MvLeaves& L, A* __restrict__ z,
                                   int64_t n, const float* __restrict__ su, int lane) {
  constexpr int G = Gran<T>::G;
  constexpr int KPL = NR * JG / 64;
  static_assert(KPL >= 1 && KPL * (64 / JG) == NR, "lane layout must cover NR");
  const int r = M.r;
  const int jl = lane % JG, k0 = (lane / JG) * KPL;
  const A sc0 = (A)1;
  for (int jp = 0; jp < r; jp += JG) {
    const int j = jp + jl;
    const bool ok = j < r;
    const int jc = ok ? j : r - 1;
    A acc[KPL];
#pragma unroll
    for (int k = 0; k < KPL; ++k) acc[k] = 0;
    const T* S = reinterpret_cast<const T*>((uintptr_t)M.vptr);
    for (int lf = M.sf; lf <= M.sl; ++lf) {
      const int ld = (int)(L.ldpre[lf + 1] - L.ldpre[lf]);
      const int m = L.m[lf], lo = L.lo[lf];
      const T* col = S + (int64_t)jc * ld;
      const A* zr = z + (int64_t)lo * NR + k0;
      for (int i0 = 0; i0 < m; i0 += G) {
        typename Gran<T>::E sv[G];
        Gran<T>::load(col + i0, sv);
#pragma unroll
        for (int e = 0; e < G; ++e) {
          if (i0 + e < m) {                              // uniform over the wavefront
            A xv[KPL];
            load_row<A, KPL>(zr + (int64_t)(i0 + e) * NR, xv);
#pragma unroll
            for (int k = 0; k < KPL; ++k) acc[k] += (A)sv[e] * xv[k];
          }
        }
      }
      S += (int64_t)ld * M.vw;
    }
    if (ok) {
      const A sc = su ? (A)su[M.toff + j] : sc0;
#pragma unroll
      for (int k = 0; k < KPL; ++k) z[(n + M.toff + j) * NR + k0 + k] = acc[k] * sc;
    }
  }
}

template <typename T, typename A, int NR>
__global__ __launch_bounds__(256) void k_fwd1m(const LrMeta* __restrict__ meta, int64_t nl,
                                               MvLeaves L, A* __restrict__ z, int64_t n,
                                               const float* __restrict__ su) {
  const int lane = threadIdx.x & 63;
  // wave-uniform block index: descriptors and leaf data come in by scalar loads
  const int64_t wid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t b = wid; b < nl; b += nw) {
    const LrMeta M = meta[b];
    if (M.r == 0) continue;
    if constexpr (NR >= 8) {
      if (M.r <= 8) {
        fwd1m_block<T, A, NR, 8>(M, L, z, n, su, lane);
        continue;
      }
    }
    fwd1m_block<T, A, NR, 16>(M, L, z, n, su, lane);
  }
}

// ------------------------------------------------------------------ forward, phase 2
// Per row leaf: y_c = sum over its panels of P z[colmap], then scattered to
// application order.  Panel 0 of a leaf holds dense slices (type TD), the
// others U slices (type TL); both share the lane layout.
//
// The workgroup first gathers the z values of a tile of panel columns into
// LDS (one load per column instead of one per lane, and no map -> z
// dependency inside the streaming loop), then streams the tile's columns:
// wavefront w takes column groups w, w + 4, ..., UNR of them at a time.
// Loads are unconditional: a lane without a column of its own reads the
// panel's last column and contributes zero, so the compiler keeps all UNR
// loads in flight instead of waiting inside divergent branches.  A tile
// holds kZTileBytes of z.
constexpr int kZTileBytes = 8192;
template <typename A, int NR>
constexpr int z_tile() { return kZTileBytes / (int)(NR * sizeof(A)); }

template <typename T, typename A, int NR, int G>
__device__ inline void fwd2_run_lds(const Run& rn, int a, int uw, int ld, int C, int cg, int g,
                                    bool act, int wave, const int32_t* __restrict__ colmap,
                                    const A* __restrict__ z, A* __restrict__ zt,
                                    A (&acc)[G][NR]) {
  constexpr int UNR = 4;
  static_assert(Gran<T>::G == G, "panel granules must cover the same rows");
  const T* S = reinterpret_cast<const T*>((uintptr_t)rn.data) + (int64_t)a * ld + g * G;
  const int32_t* map = colmap + rn.col0 + a;
  constexpr int kTile = z_tile<A, NR>();
  for (int t0 = 0; t0 < uw; t0 += kTile) {
    const int tw = min(kTile, uw - t0);
    __syncthreads();                                   // the previous tile is consumed
    for (int c = threadIdx.x; c < tw; c += blockDim.x) {
      A v[NR];
      load_row<A, NR>(z + (int64_t)map[t0 + c] * NR, v);
#pragma unroll
      for (int k = 0; k < NR; ++k) zt[c * NR + k] = v[k];
    }
    __syncthreads();
    const T* St = S + (int64_t)t0 * ld;
    const int ngrp = (tw + C - 1) / C;
    for (int q0 = wave; q0 < ngrp; q0 += 4 * UNR) {
      typename Gran<T>::E s[UNR][G];
      int jl[UNR];
      bool ok[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + 4 * u;
        const int j = q * C + cg;
        ok[u] = act && q < ngrp && j < tw;
        jl[u] = ok[u] ? j : tw - 1;
        Gran<T>::load(St + (int64_t)jl[u] * ld, s[u]);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
#pragma unroll
        for (int e = 0; e < G; ++e) {
          const A sv = ok[u] ? (A)s[u][e] : (A)0;
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[e][k] += sv * zt[jl[u] * NR + k];
        }
      }
    }
  }
}

template <typename TD, typename TL, typename A, int NR>
__global__ __launch_bounds__(256) void k_fwd2(const Run* __restrict__ runs, MvLeaves L,
                                              const Unit* __restrict__ units, int64_t nunits,
                                              const int32_t* __restrict__ colmap,
                                              const A* __restrict__ z, A* __restrict__ ypart,
                                              int ldmax) {
  constexpr int G = Gran<TD>::G;
  __shared__ A ybuf[4][kMaxLeaf][NR];
  __shared__ A zt[z_tile<A, NR>() * NR];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t per = (nunits + kXcds - 1) / kXcds;
  for (int64_t li = blockIdx.x; li < per * kXcds; li += gridDim.x) {
    const int64_t u = xcd_item(li, per);
    if (u >= nunits) continue;                          // uniform over the workgroup
    const Unit U = units[u];
    const int64_t c = U.leaf;
    const int ld = (int)(L.ldpre[c + 1] - L.ldpre[c]);
    const int R = ld / G, C = 64 / R;
    const int cg = lane / R, g = lane % R;
    const bool act = cg < C;
    const int m = L.m[c];
    A acc[G][NR];
#pragma unroll
    for (int e = 0; e < G; ++e)
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[e][k] = 0;
    const Run rn = runs[(int64_t)U.run * L.nleaf + c];
    if (std::is_same<TD, TL>::value || U.run == 0)
      fwd2_run_lds<TD, A, NR, G>(rn, U.a, U.w, ld, C, cg, g, act, wave, colmap, z, zt, acc);
    else
      fwd2_run_lds<TL, A, NR, G>(rn, U.a, U.w, ld, C, cg, g, act, wave, colmap, z, zt, acc);
    // combine the column groups (tree over cg, stride R), then the waves
#pragma unroll
    for (int e = 0; e < G; ++e)
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        A v = acc[e][k];
        for (int s = 1; s < C; s <<= 1) {
          const A o = __shfl_down(v, s * R, 64);
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
    A* yp = ypart + u * ldmax * NR;
    for (int e = threadIdx.x; e < m * NR; e += blockDim.x) {
      const int row = e / NR, k = e % NR;
      yp[e] = ((ybuf[0][row][k] + ybuf[1][row][k]) + ybuf[2][row][k]) + ybuf[3][row][k];
    }
    __syncthreads();
  }
}

// y rows of every leaf = sum of its units' partial rows (in unit order),
// scattered to application order.  One wavefront per leaf (a leaf has at
// most 64 rows).
template <typename A, typename VT, int NR>
__global__ __launch_bounds__(256) void k_fwd2_sum(MvLeaves L, const int32_t* __restrict__ ubeg,
                                                  const A* __restrict__ ypart, int ldmax,
                                                  const int32_t* __restrict__ perm,
                                                  VT* __restrict__ y, int nrhs, int k0) {
  const int lane = threadIdx.x & 63;
  for (int64_t c = blockIdx.x * 4 + (threadIdx.x >> 6); c < L.nleaf; c += (int64_t)gridDim.x * 4) {
    const int m = L.m[c], lo = L.lo[c];
    const int u0 = ubeg[c], u1 = ubeg[c + 1];
    for (int e = lane; e < m * NR; e += 64) {
      const int row = e / NR, k = e % NR;
      A v = 0;
      for (int u = u0; u < u1; ++u) v += ypart[(int64_t)u * ldmax * NR + e];
      y[(int64_t)perm[lo + row] * nrhs + k0 + k] = (VT)v;
    }
  }
}

// ------------------------------------------------------------------ many right-hand sides on MFMA
// With 8 or 16 right-hand sides, both forward phases are small dense
// products with a long inner dimension: phase 1 is T_b = V_b^T X (terms x
// right-hand sides, inner dimension = rows of sigma), phase 2 is
// Y_c += P Z (rows of the leaf x right-hand sides, inner dimension = panel
// columns).  Both run on 16 x 16 x 4 matrix instructions, C[16][16] +=
// A[16][4] B[4][16] with, for lane l, a = A[l % 16][l / 16] and
// b = B[l / 16][l % 16]: v_mfma_f64_16x16x4 for double vectors (item j of
// the accumulator = C[4 j + l / 16][l % 16]), v_mfma_f32_16x16x4 for float
// vectors (item j = C[4 (l / 16) + j][l % 16]).  Stored values are widened
// to the accumulation type, double or float as on the vector path.
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename A>
struct Mfma;
template <>
struct Mfma<double> {
  using V = f64x4;
  // row of accumulator item j in lane group q = l / 16
  __device__ static inline int row(int j, int q) { return 4 * j + q; }
};
template <>
struct Mfma<float> {
  using V = f32x4;
  __device__ static inline int row(int j, int q) { return 4 * q + j; }
};

template <typename A, typename T>
__device__ inline A widen(T v) { return (A)v; }

// Four consecutive stored values (a 16-byte FP32 granule, two FP64
// granules, an 8-byte FP16 granule), widened to A; streamed once per
// product, so the loads are non-temporal.
template <typename A, typename T>
__device__ inline void load4(const T* p, A (&o)[4]) {
  if constexpr (std::is_same<T, double>::value) {
    const f64x2 u = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
    const f64x2 v = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p + 2));
    o[0] = (A)u.x; o[1] = (A)u.y; o[2] = (A)v.x; o[3] = (A)v.y;
  } else if constexpr (std::is_same<T, float>::value) {
    const f32x4 u = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    o[0] = (A)u.x; o[1] = (A)u.y; o[2] = (A)u.z; o[3] = (A)u.w;
  } else {
    const f16x4 u = __builtin_nontemporal_load(reinterpret_cast<const f16x4*>(p));
    o[0] = (A)u.x; o[1] = (A)u.y; o[2] = (A)u.z; o[3] = (A)u.w;
  }
}

// Phase 1 for FP64 and FP16 stored factors: term tiles of 16 (up to four
// per pass), rows in quads (lane group lq takes row 4 i + lq of quad i), two
// quads at a time, every load unconditional (clamped to the slice, the value
// zeroed outside it) and every product issued, so no branch surrounds an
// MFMA; a quad past the slice contributes exact zeros; rows go in in order.
// (For these two the granule form below was slower: 29 against 19 ms (FP64)
// and 10.6 against 10.0 ms (FP16) for the 16-column phase at N = 1,310,720.)
template <typename T, typename A, int NR, int NTL>
__device__ inline void fwd1x_pass_rows(const LrMeta& M, const MvLeaves& L,
                                       const A* __restrict__ zx, int tg, int r, int lr, int lq,
                                       typename Mfma<A>::V (&acc)[4]) {
  constexpr int IU = 2;
  const T* S = reinterpret_cast<const T*>((uintptr_t)M.vptr);
  int lo = L.lo[M.sf];                    // the leaves of sigma are consecutive
  for (int lf = M.sf; lf <= M.sl; ++lf) {
    const int m = L.m[lf];
    const int ld = (int)(L.ldpre[lf + 1] - L.ldpre[lf]);
    for (int i00 = 0; i00 < m; i00 += 4 * IU) {
      A bv[IU], av[IU][NTL];
#pragma unroll
      for (int u = 0; u < IU; ++u) {
        const int i = i00 + 4 * u + lq;
        const bool ok = i < m;
        const int ic = ok ? i : m - 1;
        bv[u] = (ok && lr < NR) ? zx[(int64_t)(lo + ic) * NR + lr] : (A)0;
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
          const int term = tg + t * 16 + lr;
          const T v = S[(int64_t)min(term, r - 1) * ld + ic];
          av[u][t] = (ok && term < r) ? widen<A>(v) : (A)0;
        }
      }
#pragma unroll
      for (int u = 0; u < IU; ++u)
#pragma unroll
        for (int t = 0; t < NTL; ++t) acc[t] = mfma16(av[u][t], bv[u], acc[t]);
    }
    S += (int64_t)ld * M.vw;
    lo += m;
  }
}

// Phase 1 for FP32 stored factors: one wavefront per admissible block, term
// tiles of 16 (up to four per pass), rows in tiles of 16.  The inner dimension may be summed in any
// order, so lane (term lr, quad lq) reads the four consecutive rows
// 4 lq .. 4 lq + 3 of a tile as one granule and feeds them to four
// instructions: step e takes row 4 lq + e of the tile from lane group lq,
// and the x values follow the same rows.  Up to four tiles are in flight,
// every load unconditional (clamped to the slice, the value zeroed outside
// it) and every product issued, so no branch surrounds an MFMA.  Rows in
// [m, ld) of a slice are zero padding; granules that start at or past m
// are zeroed.  A leaf's rows go in groups of four tiles and a last group of
// as many tiles as remain (three for the 40-row leaves of a sphere, where
// a fixed group of four spent a quarter of its loads and products on
// padding).
template <typename T, typename A, int NR, int NTL, int IU>
__device__ inline void fwd1x_tiles_gran(const T* __restrict__ S, int ld, int m, int i00,
                                        const A* __restrict__ zx, int lo, const int (&tc)[NTL],
                                        const bool (&tok)[NTL], bool rhs, int lr, int lq,
                                        typename Mfma<A>::V (&acc)[4]) {
  A av[IU][NTL][4], bv[IU][4];
#pragma unroll
  for (int u = 0; u < IU; ++u) {
    const int i0 = i00 + 16 * u + 4 * lq;       // first row of the lane's granule
    const bool okg = i0 < m;
    const int ig = okg ? i0 : 0;
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
      A v[4];
      load4<A, T>(S + (int64_t)tc[t] * ld + ig, v);
#pragma unroll
      for (int e = 0; e < 4; ++e) av[u][t][e] = (okg && tok[t]) ? v[e] : (A)0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool okr = rhs && i0 + e < m;
      const A x = zx[(int64_t)(lo + (okr ? i0 + e : 0)) * NR + (rhs ? lr : 0)];
      bv[u][e] = okr ? x : (A)0;
    }
  }
#pragma unroll
  for (int u = 0; u < IU; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int t = 0; t < NTL; ++t) acc[t] = mfma16(av[u][t][e], bv[u][e], acc[t]);
}

template <typename T, typename A, int NR, int NTL>
__device__ inline void fwd1x_pass_gran(const LrMeta& M, const MvLeaves& L,
                                       const A* __restrict__ zx, int tg, int r, int lr, int lq,
                                       typename Mfma<A>::V (&acc)[4]) {
  const T* S = reinterpret_cast<const T*>((uintptr_t)M.vptr);
  int lo = L.lo[M.sf];                    // the leaves of sigma are consecutive
  int tc[NTL];                            // clamped term of each tile
  bool tok[NTL];
#pragma unroll
  for (int t = 0; t < NTL; ++t) {
    const int term = tg + t * 16 + lr;
    tok[t] = term < r;
    tc[t] = tok[t] ? term : r - 1;
  }
  const bool rhs = lr < NR;
  for (int lf = M.sf; lf <= M.sl; ++lf) {
    const int m = L.m[lf];
    const int ld = (int)(L.ldpre[lf + 1] - L.ldpre[lf]);
    int i00 = 0;
    for (; i00 + 64 <= m; i00 += 64)
      fwd1x_tiles_gran<T, A, NR, NTL, 4>(S, ld, m, i00, zx, lo, tc, tok, rhs, lr, lq, acc);
    switch ((m - i00 + 15) / 16) {        // uniform over the wavefront
      case 1: fwd1x_tiles_gran<T, A, NR, NTL, 1>(S, ld, m, i00, zx, lo, tc, tok, rhs, lr, lq, acc); break;
      case 2: fwd1x_tiles_gran<T, A, NR, NTL, 2>(S, ld, m, i00, zx, lo, tc, tok, rhs, lr, lq, acc); break;
      case 3: fwd1x_tiles_gran<T, A, NR, NTL, 3>(S, ld, m, i00, zx, lo, tc, tok, rhs, lr, lq, acc); break;
      default: break;
    }
    S += (int64_t)ld * M.vw;
    lo += m;
  }
}

template <typename T, typename A, int NR>
__global__ __launch_bounds__(256) void k_fwd1x(const LrMeta* __restrict__ meta, int64_t nl,
                                               MvLeaves L, const A* __restrict__ zx,
                                               A* __restrict__ zt, int64_t n,
                                               const float* __restrict__ su) {
  using V = typename Mfma<A>::V;
  static_assert(NR == 8 || NR == 16, "MFMA phase 1 takes 8 or 16 right-hand sides");
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lq = lane >> 4;     // a: term lr, row lq; b: row lq, rhs lr
  const int64_t wid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t b = wid; b < nl; b += nw) {
    const LrMeta M = meta[b];
    const int r = M.r;
    if (r == 0) continue;
    for (int tg = 0; tg < r; tg += 64) {
      const int ntile = min(4, (r - tg + 15) / 16);
      V acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = V{0, 0, 0, 0};
      if constexpr (!std::is_same<T, float>::value) {
        switch (ntile) {                      // uniform over the wavefront
          case 1: fwd1x_pass_rows<T, A, NR, 1>(M, L, zx, tg, r, lr, lq, acc); break;
          case 2: fwd1x_pass_rows<T, A, NR, 2>(M, L, zx, tg, r, lr, lq, acc); break;
          case 3: fwd1x_pass_rows<T, A, NR, 3>(M, L, zx, tg, r, lr, lq, acc); break;
          default: fwd1x_pass_rows<T, A, NR, 4>(M, L, zx, tg, r, lr, lq, acc); break;
        }
      } else {
        switch (ntile) {
          case 1: fwd1x_pass_gran<T, A, NR, 1>(M, L, zx, tg, r, lr, lq, acc); break;
          case 2: fwd1x_pass_gran<T, A, NR, 2>(M, L, zx, tg, r, lr, lq, acc); break;
          case 3: fwd1x_pass_gran<T, A, NR, 3>(M, L, zx, tg, r, lr, lq, acc); break;
          default: fwd1x_pass_gran<T, A, NR, 4>(M, L, zx, tg, r, lr, lq, acc); break;
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < ntile) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int term = tg + t * 16 + Mfma<A>::row(j, lq);
            if (term < r && lr < NR) {
              const A sc = su ? (A)su[M.toff + term] : (A)1;
              zt[(n + M.toff + term) * NR + lr] = acc[t][j] * sc;
            }
          }
        }
      }
    }
  }
}

// The column quads of one z tile for a leaf of NT 16-row tiles: KQ quads per
// wavefront at a time, every load unconditional (clamped to the panel, the
// value zeroed outside it) and every product issued, so the loop has no
// branch around an MFMA and the accumulators stay in place.  A quad past the
// tile contributes exact zeros; the products go in in column order.
template <typename E, typename A, int NR, int NT, int KQ>
__device__ inline void fwd2x_tile(const E* __restrict__ P, int64_t cbase, int ld, int tw,
                                  const A* __restrict__ zs, int wave, int lr, int lq,
                                  typename Mfma<A>::V (&acc)[4]) {
  for (int q0 = wave; q0 * 4 < tw; q0 += 4 * KQ) {
    A bv[KQ], av[KQ][NT];
#pragma unroll
    for (int u = 0; u < KQ; ++u) {
      const int col = (q0 + 4 * u) * 4 + lq;
      const bool okc = col < tw;
      const int colc = okc ? col : tw - 1;
      bv[u] = (okc && lr < NR) ? zs[colc * NR + lr] : (A)0;
      const E* pc = P + (cbase + colc) * ld;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int row = t * 16 + lr;
        const E v = pc[min(row, ld - 1)];
        av[u][t] = (okc && row < ld) ? widen<A>(v) : (A)0;
      }
    }
#pragma unroll
    for (int u = 0; u < KQ; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma16(av[u][t], bv[u], acc[t]);
  }
}

template <typename E, typename A, int NR, int KQ>
__device__ inline void fwd2x_tile_nt(int nrt, const E* __restrict__ P, int64_t cbase, int ld,
                                     int tw, const A* __restrict__ zs, int wave, int lr,
                                     int lq, typename Mfma<A>::V (&acc)[4]) {
  switch (nrt) {                                        // uniform over the workgroup
    case 1: fwd2x_tile<E, A, NR, 1, KQ>(P, cbase, ld, tw, zs, wave, lr, lq, acc); break;
    case 2: fwd2x_tile<E, A, NR, 2, KQ>(P, cbase, ld, tw, zs, wave, lr, lq, acc); break;
    case 3: fwd2x_tile<E, A, NR, 3, KQ>(P, cbase, ld, tw, zs, wave, lr, lq, acc); break;
    default: fwd2x_tile<E, A, NR, 4, KQ>(P, cbase, ld, tw, zs, wave, lr, lq, acc); break;
  }
}

// The same with granule loads: lane (i = lr, column lq of a quad) reads
// rows 4 i .. 4 i + 3 of its column at once and gives row 4 i + t to the
// accumulator of tile t, so tile t holds the rows 4 i + t (i = 0..15) and
// every panel column is one contiguous read of 16 lanes.  Lanes with
// 4 i >= ld contribute zeros.
template <typename E, typename A, int NR, int KQ>
__device__ inline void fwd2x_gran(const E* __restrict__ P, int64_t cbase, int ld, int tw,
                                  const A* __restrict__ zs, int wave, int lr, int lq,
                                  typename Mfma<A>::V (&acc)[4]) {
  const bool okr = 4 * lr < ld;
  const int rg = okr ? 4 * lr : 0;
  for (int q0 = wave; q0 * 4 < tw; q0 += 4 * KQ) {
    A bv[KQ], av[KQ][4];
#pragma unroll
    for (int u = 0; u < KQ; ++u) {
      const int col = (q0 + 4 * u) * 4 + lq;
      const bool okc = col < tw;
      const int colc = okc ? col : tw - 1;
      bv[u] = (okc && lr < NR) ? zs[colc * NR + lr] : (A)0;
      A v[4];
      load4<A, E>(P + (cbase + colc) * ld + rg, v);
#pragma unroll
      for (int t = 0; t < 4; ++t) av[u][t] = (okc && okr) ? v[t] : (A)0;
    }
#pragma unroll
    for (int u = 0; u < KQ; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = mfma16(av[u][t], bv[u], acc[t]);
  }
}

// Phase 2: one workgroup per work unit; the unit's z values are staged in
// LDS per tile, each wavefront takes column quads round-robin and keeps one
// accumulator per 16-row tile of the leaf; the four wavefronts are added in
// LDS in a fixed order.
template <typename TD, typename TL, typename A, int NR, bool GR>
__global__ __launch_bounds__(256) void k_fwd2x(const Run* __restrict__ runs, MvLeaves L,
                                               const Unit* __restrict__ units, int64_t nunits,
                                               const int32_t* __restrict__ colmap,
                                               const A* __restrict__ z,
                                               A* __restrict__ ypart, int ldmax) {
  using V = typename Mfma<A>::V;
  static_assert(NR == 8 || NR == 16, "MFMA phase 2 takes 8 or 16 right-hand sides");
  constexpr int kQuads = 4;
  // the z tile and the final combination of the wavefronts share one LDS
  // buffer (the tile is consumed before the combination starts)
  constexpr int kTile = (4 * kMaxLeaf * NR) / NR;     // columns: 256
  __shared__ A lbuf[4 * kMaxLeaf * NR];
  A* zs = lbuf;
  A (*ybuf)[kMaxLeaf][NR] = reinterpret_cast<A (*)[kMaxLeaf][NR]>(lbuf);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;     // a: row lr, column lq; b: column lq, rhs lr
  const int64_t per = (nunits + kXcds - 1) / kXcds;
  for (int64_t li = blockIdx.x; li < per * kXcds; li += gridDim.x) {
    const int64_t u = xcd_item(li, per);
    if (u >= nunits) continue;                          // uniform over the workgroup
    const Unit U = units[u];
    const int64_t c = U.leaf;
    const int ld = (int)(L.ldpre[c + 1] - L.ldpre[c]);
    const int m = L.m[c];
    const int nrt = (ld + 15) / 16;                     // 16-row tiles, at most 4
    const Run rn = runs[(int64_t)U.run * L.nleaf + c];
    const bool dense = std::is_same<TD, TL>::value || U.run == 0;
    const int32_t* map = colmap + rn.col0 + U.a;
    V acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = V{0, 0, 0, 0};
    for (int t0 = 0; t0 < U.w; t0 += kTile) {
      const int tw = min(kTile, U.w - t0);
      __syncthreads();                                  // the previous tile is consumed
      for (int e = threadIdx.x; e < tw * NR; e += blockDim.x) {
        const int col = e / NR, k = e % NR;
        zs[e] = z[(int64_t)map[t0 + col] * NR + k];
      }
      __syncthreads();
      const int64_t cbase = (int64_t)U.a + t0;          // first panel column of the tile
      if constexpr (GR) {
        if (dense)
          fwd2x_gran<TD, A, NR, kQuads>(reinterpret_cast<const TD*>((uintptr_t)rn.data), cbase,
                                        ld, tw, zs, wave, lr, lq, acc);
        else
          fwd2x_gran<TL, A, NR, kQuads>(reinterpret_cast<const TL*>((uintptr_t)rn.data), cbase,
                                        ld, tw, zs, wave, lr, lq, acc);
      } else {
        if (dense)
          fwd2x_tile_nt<TD, A, NR, kQuads>(nrt, reinterpret_cast<const TD*>((uintptr_t)rn.data),
                                           cbase, ld, tw, zs, wave, lr, lq, acc);
        else
          fwd2x_tile_nt<TL, A, NR, kQuads>(nrt, reinterpret_cast<const TL*>((uintptr_t)rn.data),
                                           cbase, ld, tw, zs, wave, lr, lq, acc);
      }
    }
    __syncthreads();                                    // the last tile is consumed
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (GR || t < nrt) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = GR ? 4 * Mfma<A>::row(j, lq) + t : t * 16 + Mfma<A>::row(j, lq);
          if (row < kMaxLeaf && lr < NR) ybuf[wave][row][lr] = acc[t][j];
        }
      }
    }
    __syncthreads();
    A* yp = ypart + u * ldmax * NR;
    for (int e = threadIdx.x; e < m * NR; e += blockDim.x) {
      const int row = e / NR, k = e % NR;
      yp[e] = ((ybuf[0][row][k] + ybuf[1][row][k]) + ybuf[2][row][k]) + ybuf[3][row][k];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ transposed, phase 1
// Per row leaf: w[col0 + j] = sum_i P[i][j] x_c[i] for every panel column.
//
// Lane (cg, g) forms the partial dot of its granule of column group
// cg with x; the R partials of a column are then added by one lane, which
// reads them from the wavefront's own LDS area (a shift-down tree over the
// R lanes cost about four times the instructions per column).  Only the
// wavefront itself reads what it wrote: program order of its LDS
// instructions is enough, and wave_lds_order keeps the compiler from
// moving LDS accesses across the exchange.
template <int NR>
constexpr int tr1_unr() { return NR <= 2 ? 4 : 1; }   // column groups per wavefront in flight

__device__ inline void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, typename A, int NR, int G>
__device__ inline void tr1_run(const Run& rn, int a, int uw, int ld, int R, int C, int cg, int g,
                               bool act, int wave, const A (&xg)[G][NR], A* __restrict__ w,
                               A* __restrict__ red) {
  static_assert(Gran<T>::G == G, "panel granules must cover the same rows");
  constexpr int UNR = tr1_unr<NR>();
  const int lane = threadIdx.x & 63;
  const T* S = reinterpret_cast<const T*>((uintptr_t)rn.data) + (int64_t)a * ld + g * G;
  const int64_t col0 = rn.col0 + a;
  const int ngrp = (uw + C - 1) / C;
  // a step covers the UNR C consecutive columns q0 C ... (q0 + UNR) C - 1;
  // reader t of a step sums column q0 C + t: group u = t / C, segment c
  const int ncol = UNR * C;
  const int ur = lane / C, cr = lane - ur * C;       // the reader's column in the first 64
  for (int q0 = wave * UNR; q0 < ngrp; q0 += 4 * UNR) {
    // UNR consecutive column groups, all granules loaded before any is reduced
    typename Gran<T>::E sv[UNR][G];
    bool ok[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int j = (q0 + u) * C + cg;
      ok[u] = act && q0 + u < ngrp && j < uw;
      Gran<T>::load(S + (int64_t)(ok[u] ? j : uw - 1) * ld, sv[u]);
    }
    A ps[UNR][NR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
#pragma unroll
      for (int k = 0; k < NR; ++k) ps[u][k] = 0;
#pragma unroll
      for (int e = 0; e < G; ++e) {
        const A x = ok[u] ? (A)sv[u][e] : (A)0;
#pragma unroll
        for (int k = 0; k < NR; ++k) ps[u][k] += x * xg[e][k];
      }
    }
    wave_lds_order();                                   // the last step's reads are done
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int k = 0; k < NR; ++k) red[(u * 64 + lane) * NR + k] = ps[u][k];
    wave_lds_order();
    for (int t = lane; t < ncol; t += 64) {
      int u = ur, c = cr;
      if (t >= 64) {
        u = t / C;
        c = t - u * C;
      }
      const A* rp = red + (u * 64 + c * R) * NR;
      A v[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) v[k] = 0;
      // partials added in order of g, read four at a time
      int e = 0;
      for (; e + 4 <= R; e += 4) {
        A r4[4][NR];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < NR; ++k) r4[i][k] = rp[(e + i) * NR + k];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < NR; ++k) v[k] += r4[i][k];
      }
      for (; e < R; ++e)
#pragma unroll
        for (int k = 0; k < NR; ++k) v[k] += rp[e * NR + k];
      const int jj = q0 * C + t;
      if (jj < uw) {
#pragma unroll
        for (int k = 0; k < NR; ++k) w[(col0 + jj) * NR + k] = v[k];
      }
    }
  }
}

template <typename TD, typename TL, typename A, int NR>
__global__ __launch_bounds__(256) void k_tr1(const Run* __restrict__ runs, MvLeaves L,
                                             const Unit* __restrict__ units, int64_t nunits,
                                             const A* __restrict__ z, A* __restrict__ w) {
  constexpr int G = Gran<TD>::G;
  __shared__ A red[4][tr1_unr<NR>() * 64 * NR];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t per = (nunits + kXcds - 1) / kXcds;
  for (int64_t li = blockIdx.x; li < per * kXcds; li += gridDim.x) {
    const int64_t u = xcd_item(li, per);
    if (u >= nunits) continue;
    const Unit U = units[u];
    const int64_t c = U.leaf;
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
        xg[e][k] = (act && row < m) ? z[(int64_t)(lo + row) * NR + k] : (A)0;
    }
    const Run rn = runs[(int64_t)U.run * L.nleaf + c];
    if (std::is_same<TD, TL>::value || U.run == 0)
      tr1_run<TD, A, NR, G>(rn, U.a, U.w, ld, R, C, cg, g, act, wave, xg, w, red[wave]);
    else
      tr1_run<TL, A, NR, G>(rn, U.a, U.w, ld, R, C, cg, g, act, wave, xg, w, red[wave]);
  }
}

// s_b[l] = sum over the row leaves of b of w[ucol + l]  ->  z[n + toff + l].
// The sums of one block, lane = (group, term): with r <= 16 (32) the
// wavefront splits into four (two) groups of 16 (32) lanes; group g adds the
// row leaves q = g, g + groups, ... and the groups are added by shifts at
// the end.  Ranks above 64 take their terms 64 at a time.
template <typename A, int NR>
__device__ inline void tr_sums_block(const LrMeta& M, const int64_t* __restrict__ ucol,
                                     const A* __restrict__ w, A* __restrict__ z, int64_t n,
                                     const float* __restrict__ su, int lane) {
  const int nk = M.tl - M.tf + 1;
  const int gw = M.r <= 16 ? 16 : (M.r <= 32 ? 32 : 64);   // uniform over the wavefront
  const int ng = 64 / gw, grp = lane / gw;
  for (int t0 = 0; t0 < M.r; t0 += 64) {
    const int l = t0 + lane % gw;
    const bool ok = l < M.r;
    A acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = 0;
    if (ok) {
      // four row leaves per step with their loads in flight together
      int q = grp;
      for (; q + 3 * ng < nk; q += 4 * ng) {
        A v[4][NR];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          load_row<A, NR>(w + (ucol[M.ub + q + u * ng] + l) * NR, v[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[k] += v[u][k];
      }
      for (; q < nk; q += ng) {
        const int64_t col = ucol[M.ub + q] + l;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] += w[col * NR + k];
      }
    }
    for (int sh = gw; sh < 64; sh <<= 1) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const A o = __shfl_down(acc[k], sh, 64);
        acc[k] += o;
      }
    }
    if (grp == 0 && ok) {
      const A sc = su ? (A)su[M.toff + l] : (A)1;
#pragma unroll
      for (int k = 0; k < NR; ++k) z[(n + M.toff + l) * NR + k] = acc[k] * sc;
    }
  }
}

// One wavefront per four consecutive blocks.  When all four have rank <= 16
// (most blocks: the small ones), each 16-lane group takes one block and adds
// its row leaves in order, so the four dependent chains (descriptor, column
// offsets, sums, store) overlap; otherwise the wavefront takes the four
// blocks one after another as above.
template <typename A, int NR>
__global__ __launch_bounds__(256) void k_tr_sums(const LrMeta* __restrict__ meta, int64_t nl,
                                                 const int64_t* __restrict__ ucol,
                                                 const A* __restrict__ w, A* __restrict__ z,
                                                 int64_t n, const float* __restrict__ su) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  const int64_t nq = (nl + 3) / 4;
  const int grp = lane >> 4, l = lane & 15;
  for (int64_t qd = wid; qd < nq; qd += nw) {
    const int64_t b = qd * 4 + grp;
    const bool has = b < nl;
    const LrMeta M = meta[has ? b : nl - 1];
    if (__all(!has || M.r <= 16)) {                     // uniform over the wavefront
      if (has && l < M.r) {
        const int nk = M.tl - M.tf + 1;
        A acc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = 0;
        for (int q = 0; q < nk; ++q) {
          const int64_t col = ucol[M.ub + q] + l;
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[k] += w[col * NR + k];
        }
        const A sc = su ? (A)su[M.toff + l] : (A)1;
#pragma unroll
        for (int k = 0; k < NR; ++k) z[(n + M.toff + l) * NR + k] = acc[k] * sc;
      }
    } else {
      for (int g = 0; g < 4; ++g) {
        const int64_t bg = qd * 4 + g;
        if (bg < nl) tr_sums_block<A, NR>(meta[bg], ucol, w, z, n, su, lane);
      }
    }
  }
}

// ------------------------------------------------------------------ transposed, phase 2
// Per column leaf: dense blocks contribute w entries (kind 0, lane = output
// row), V slices contribute V s (kind 1, granule product).  The items of a
// leaf are dealt to S workgroups (item i to workgroup (i / 4) mod S, wavefront
// i mod 4), so that a leaf's few hundred slices are not one long chain of
// dependent loads per wavefront; with S > 1 each workgroup writes its partial
// rows to ypart[c S + s] and k_tr2_sum adds them in order of s.
template <typename T, typename A, typename VT, int NR>
__global__ __launch_bounds__(256) void k_tr2(const int32_t* __restrict__ beg,
                                             const TItem* __restrict__ items, MvLeaves L,
                                             const A* __restrict__ w, const A* __restrict__ z,
                                             int64_t n, const int32_t* __restrict__ perm,
                                             VT* __restrict__ y, int nrhs, int k0, int S,
                                             A* __restrict__ ypart, int ldmax) {
  constexpr int G = Gran<T>::G;
  __shared__ A ybuf[4][kMaxLeaf][NR];
  // wave-uniform index: item descriptors come in by scalar loads
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwork = L.nleaf * S;
  const int64_t per = (nwork + kXcds - 1) / kXcds;
  for (int64_t li = blockIdx.x; li < per * kXcds; li += gridDim.x) {
    const int64_t q = xcd_item(li, per);
    if (q >= nwork) continue;                           // uniform over the workgroup
    const int64_t c = q / S;
    const int sp = (int)(q - c * S);
    const int ld = (int)(L.ldpre[c + 1] - L.ldpre[c]);
    const int R = ld / G, C = 64 / R;
    const int cg = lane / R, g = lane % R;
    const bool act = cg < C;
    const int m = L.m[c], lo = L.lo[c];
    A acc[G][NR], yT[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      yT[k] = 0;
#pragma unroll
      for (int e = 0; e < G; ++e) acc[e][k] = 0;
    }
    const int b0 = beg[c], b1 = beg[c + 1];
    // the next item's descriptor is loaded one iteration ahead
    const int it0 = b0 + 4 * sp + wave;
    TItem In;
    if (it0 < b1) In = items[it0];
    for (int it = it0; it < b1; it += 4 * S) {
      const TItem I = In;
      if (it + 4 * S < b1) In = items[it + 4 * S];
      if (I.kind == 0) {
        if (lane < I.w) {
#pragma unroll
          for (int k = 0; k < NR; ++k) yT[k] += w[(I.src + lane) * NR + k];
        }
      } else {
        const T* S = reinterpret_cast<const T*>((uintptr_t)I.data);
        if constexpr (sizeof(T) < 8) {
          for (int j0 = 0; j0 < I.w; j0 += C) {
            const int j = j0 + cg;
            if (act && j < I.w) {
              typename Gran<T>::E s[G];
              Gran<T>::load(S + (int64_t)j * ld + g * G, s);
              A zz[NR];
              load_row<A, NR>(z + (n + I.src + j) * NR, zz);
#pragma unroll
              for (int e = 0; e < G; ++e)
#pragma unroll
                for (int k = 0; k < NR; ++k) acc[e][k] += (A)s[e] * zz[k];
            }
          }
        } else {
          // FP64 slices: UNR column groups at a time with unconditional loads
          // (a lane without a column reads the slice's last one and adds zero),
          // so all their loads are in flight together (16% faster; slower for
          // FP32 and FP16 slices, which keep the loop above)
          constexpr int UNR = NR <= 2 ? 4 : 1;
          const int ngrp = (I.w + C - 1) / C;
          for (int q0 = 0; q0 < ngrp; q0 += UNR) {
            typename Gran<T>::E s[UNR][G];
            A zz[UNR][NR];
            bool ok[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
              const int j = (q0 + u) * C + cg;
              ok[u] = act && q0 + u < ngrp && j < I.w;
              const int jj = ok[u] ? j : I.w - 1;
              Gran<T>::load(S + (int64_t)jj * ld + g * G, s[u]);
              load_row<A, NR>(z + (n + I.src + jj) * NR, zz[u]);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u)
#pragma unroll
              for (int e = 0; e < G; ++e) {
                const A sv = ok[u] ? (A)s[u][e] : (A)0;
#pragma unroll
                for (int k = 0; k < NR; ++k) acc[e][k] += sv * zz[u][k];
              }
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < G; ++e)
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        A v = acc[e][k];
        for (int s = 1; s < C; s <<= 1) {
          const A o = __shfl_down(v, s * R, 64);
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
    A* yp = ypart + q * ldmax * NR;
    for (int e = threadIdx.x; e < m * NR; e += blockDim.x) {
      const int row = e / NR, k = e % NR;
      const A v = ((ybuf[0][row][k] + ybuf[1][row][k]) + ybuf[2][row][k]) + ybuf[3][row][k];
      if (S == 1)
        y[(int64_t)perm[lo + row] * nrhs + k0 + k] = (VT)v;
      else
        yp[e] = v;
    }
    __syncthreads();
  }
}

// y rows of every column leaf = sum of its S partial rows (in order of s),
// scattered to application order.
template <typename A, typename VT, int NR>
__global__ __launch_bounds__(256) void k_tr2_sum(MvLeaves L, int S, const A* __restrict__ ypart,
                                                 int ldmax, const int32_t* __restrict__ perm,
                                                 VT* __restrict__ y, int nrhs, int k0) {
  const int lane = threadIdx.x & 63;
  for (int64_t c = blockIdx.x * 4 + (threadIdx.x >> 6); c < L.nleaf; c += (int64_t)gridDim.x * 4) {
    const int m = L.m[c], lo = L.lo[c];
    const A* yp = ypart + c * S * ldmax * NR;
    for (int e = lane; e < m * NR; e += 64) {
      const int row = e / NR, k = e % NR;
      A v = 0;
      for (int sp = 0; sp < S; ++sp) v += yp[(int64_t)sp * ldmax * NR + e];
      y[(int64_t)perm[lo + row] * nrhs + k0 + k] = (VT)v;
    }
  }
}

// ------------------------------------------------------------------ host side
template <typename TD, typename TL, typename A, typename VT, int NR>
static void mv_chunk(const MvPlan& P, const VT* x, VT* y, int nrhs, int k0, bool transposed,
                     hipStream_t s) {
  A* z = static_cast<A*>(P.z);
  A* w = static_cast<A*>(P.w);
  MvProfile* pr = P.prof;
  if (pr) HM_HIP(hipEventRecord(pr->ev[0], s));
  k_gather<VT, A><<<grid_for(P.n * NR, 256, 4096), 256, 0, s>>>(x, nrhs, k0, NR, P.perm, P.n, z);
  HM_LAUNCH_CHECK();
  if (pr) HM_HIP(hipEventRecord(pr->ev[1], s));
  if (!transposed) {
    // phase 1 over its work units (column chunks of the V panels)
    const unsigned g1 = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(P.nu1, 4), 1 << 20));
    if (P.nu1 > 0) {
      if constexpr (NR == 8 || NR == 16) {
        k_fwd1x<TL, A, NR><<<g1, 256, 0, s>>>(P.meta1, P.nu1, P.L, z, z, P.n, P.su);
      } else if constexpr (NR >= 4) {
        k_fwd1m<TL, A, NR><<<g1, 256, 0, s>>>(P.meta1, P.nu1, P.L, z, P.n, P.su);
      } else {
        k_fwd1<TL, A, NR><<<g1, 256, 0, s>>>(P.meta1, P.nu1, P.L, z, P.n, P.su);
      }
      HM_LAUNCH_CHECK();
    }
    if (pr) {
      HM_HIP(hipEventRecord(pr->ev[2], s));
      HM_HIP(hipEventRecord(pr->ev[3], s));
    }
    const unsigned gu = (unsigned)std::min<int64_t>(ceil_div(P.nunits, kXcds) * kXcds, P.grid);
    if (P.nunits > 0) {
      // double vectors on the FP64 matrix cores; with float vectors the
      // vector kernel streams the panels faster than the FP32 instructions
      if constexpr (NR == 8 || NR == 16)
        k_fwd2x<TD, TL, A, NR, true><<<gu, 256, 0, s>>>(P.runs, P.L, P.units, P.nunits,
                                                        P.colmap, z, static_cast<A*>(P.ypart),
                                                        P.ldmax);
      else
        k_fwd2<TD, TL, A, NR><<<gu, 256, 0, s>>>(P.runs, P.L, P.units, P.nunits, P.colmap, z,
                                                 static_cast<A*>(P.ypart), P.ldmax);
      HM_LAUNCH_CHECK();
    }
    k_fwd2_sum<A, VT, NR><<<(unsigned)std::min<int64_t>(ceil_div(P.L.nleaf, 4), P.grid), 256, 0, s>>>(
        P.L, P.ubeg, static_cast<const A*>(P.ypart), P.ldmax, P.perm, y, nrhs, k0);
    HM_LAUNCH_CHECK();
  } else {
    if (P.nunits > 0) {
      const unsigned gu = (unsigned)std::min<int64_t>(ceil_div(P.nunits, kXcds) * kXcds, P.grid);
      k_tr1<TD, TL, A, NR><<<gu, 256, 0, s>>>(P.runs, P.L, P.units, P.nunits, z, w);
      HM_LAUNCH_CHECK();
    }
    if (pr) HM_HIP(hipEventRecord(pr->ev[2], s));
    if (P.nlr > 0) {
      // four blocks per wavefront, four wavefronts per workgroup; blocks
      // come largest first and stay round-robin over the XCDs
      const unsigned gq =
          (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(ceil_div(P.nlr, 4), 4), 1 << 20));
      k_tr_sums<A, NR><<<gq, 256, 0, s>>>(P.meta, P.nlr, P.ucol, w, z, P.n, P.su);
      HM_LAUNCH_CHECK();
    }
    if (pr) HM_HIP(hipEventRecord(pr->ev[3], s));
    // workgroups per column leaf: up to 8, as many as the unit workspace
    // holds partial rows (ldmax x NR) for
    const int64_t cap = P.ypart_bytes / ((int64_t)P.ldmax * NR * (int64_t)sizeof(A));
    const int S = (int)std::max<int64_t>(1, std::min<int64_t>(8, cap / std::max<int64_t>(1, P.L.nleaf)));
    // leaves carry similar work: the grid covers the XCD-ordered index range
    const unsigned gt = (unsigned)std::min<int64_t>(ceil_div(P.L.nleaf * S, kXcds) * kXcds, P.grid);
    k_tr2<TL, A, VT, NR><<<gt, 256, 0, s>>>(P.tbeg, P.titems, P.L, w, z, P.n, P.perm, y, nrhs, k0,
                                            S, static_cast<A*>(P.ypart), P.ldmax);
    HM_LAUNCH_CHECK();
    if (S > 1) {
      k_tr2_sum<A, VT, NR><<<(unsigned)std::min<int64_t>(ceil_div(P.L.nleaf, 4), P.grid), 256, 0, s>>>(
          P.L, S, static_cast<const A*>(P.ypart), P.ldmax, P.perm, y, nrhs, k0);
      HM_LAUNCH_CHECK();
    }
  }
  if (pr) {
    HM_HIP(hipEventRecord(pr->ev[4], s));
    HM_HIP(hipEventSynchronize(pr->ev[4]));
    const int base = transposed ? 4 : 0;
    for (int k = 0; k < 4; ++k) {
      float ms = 0.f;
      HM_HIP(hipEventElapsedTime(&ms, pr->ev[k], pr->ev[k + 1]));
      pr->ms[base + k] += ms;
      pr->launches[base + k] += 1;
    }
  }
}

template <typename TD, typename TL, typename A, typename VT>
void matvec_impl(const MvPlan& P, const VT* x, VT* y, int nrhs, bool transposed, hipStream_t s) {
  const int cap = transposed ? P.max_nr_t : 16;
  int k0 = 0;
  while (k0 < nrhs) {
    const int left = nrhs - k0;
    if (left >= 16 && cap >= 16) {
      mv_chunk<TD, TL, A, VT, 16>(P, x, y, nrhs, k0, transposed, s);
      k0 += 16;
    } else if (left >= 8 && cap >= 8) {
      mv_chunk<TD, TL, A, VT, 8>(P, x, y, nrhs, k0, transposed, s);
      k0 += 8;
    } else if (left >= 4 && cap >= 4) {
      mv_chunk<TD, TL, A, VT, 4>(P, x, y, nrhs, k0, transposed, s);
      k0 += 4;
    } else if (left >= 2 && cap >= 2) {
      mv_chunk<TD, TL, A, VT, 2>(P, x, y, nrhs, k0, transposed, s);
      k0 += 2;
    } else {
      mv_chunk<TD, TL, A, VT, 1>(P, x, y, nrhs, k0, transposed, s);
      k0 += 1;
    }
  }
}

// storage 0: FP64, 1: FP32, 2: FP32 dense + FP16 factors.  Vectors VT;
// accumulation in double unless the storage and the vectors are single
// precision.
void matvec_dispatch(const MvPlan& P, int storage, const void* x, void* y, int nrhs, int vec_f32,
                     bool transposed, hipStream_t s) {
  if (storage == 2) {
    if (vec_f32)
      matvec_impl<float, _Float16, float, float>(P, (const float*)x, (float*)y, nrhs, transposed, s);
    else
      matvec_impl<float, _Float16, double, double>(P, (const double*)x, (double*)y, nrhs,
                                                    transposed, s);
  } else if (storage == 1) {
    if (vec_f32)
      matvec_impl<float, float, float, float>(P, (const float*)x, (float*)y, nrhs, transposed, s);
    else
      matvec_impl<float, float, double, double>(P, (const double*)x, (double*)y, nrhs, transposed,
                                                s);
  } else {
    if (vec_f32)
      matvec_impl<double, double, double, float>(P, (const float*)x, (float*)y, nrhs, transposed,
                                                 s);
    else
      matvec_impl<double, double, double, double>(P, (const double*)x, (double*)y, nrhs,
                                                  transposed, s);
  }
}

}  // namespace hm
