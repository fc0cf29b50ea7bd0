// Internal declarations of the gfx950 H-matrix library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/hm.h"

namespace hm {

// ---------------------------------------------------------------- errors
struct Error {
  hm_status code;
  std::string msg;
};
void set_error(const std::string& msg);
#define HM_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw ::hm::Error{HM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)
#define HM_LAUNCH_CHECK() HM_HIP(hipGetLastError())

// ---------------------------------------------------------------- constants
constexpr int kMortonBits = 21;
constexpr int kNQ = 7;              // quadrature nodes of the triangle rule
constexpr int kMaxLeaf = 64;        // leaf clusters fit one wavefront
constexpr int kMaxRank = 256;

// Radon's seven-point degree-5 rule: weights normalised to sum to one.
// Node q = 0 is the centroid; nodes 1..3 use (a1, a1, b1), 4..6 (a2, a2, b2).
struct Radon7 {
  static constexpr double s15 = 3.872983346207416885179265399782399611;  // sqrt(15)
  static constexpr double a1 = (6.0 - s15) / 21.0;
  static constexpr double b1 = (9.0 + 2.0 * s15) / 21.0;
  static constexpr double a2 = (6.0 + s15) / 21.0;
  static constexpr double b2 = (9.0 - 2.0 * s15) / 21.0;
  static constexpr double w0 = 9.0 / 40.0;
  static constexpr double w1 = (155.0 - s15) / 1200.0;
  static constexpr double w2 = (155.0 + s15) / 1200.0;
};

// ---------------------------------------------------------------- device data
// Geometry in Morton order, structure of arrays.
//   c   : double[3][n]     centroids (collocation points)
//   o   : T[3*7][n]        quadrature node minus centroid, x for q=0..6,
//                          then y, then z
//   aw  : T[n]             |T_j| / (4 pi)
//   sf  : T[n]             analytic self-term a_jj
template <typename T>
struct Geom {
  const double* c;
  const T* o;
  const T* aw;
  const T* sf;
  int64_t n;
};

// Cluster record: lo, hi (Morton positions), first child (-1 for a leaf), level.
using Cluster = int4;

// One slice of a stored block, as seen from one leaf cluster.
struct Item {
  uint64_t data;   // device address of the slice (column-major, ld of its row leaf)
  int32_t w;       // columns of the slice
  int32_t src;     // first column's index into the input vector (x or t)
  int32_t aux;     // LR: partial-sum slot; dense transposed: row leaf of the slice
  int32_t kind;    // 0 dense, 1 low rank
  int32_t pad0, pad1;
};
static_assert(sizeof(Item) == 32, "Item layout");

// Leaf table and per-leaf item lists used by the products.
struct MvLeaves {
  const int32_t* lo;
  const int32_t* m;
  const int64_t* ldpre;   // prefix of ld over leaves (nleaf + 1 entries)
  int64_t nleaf;
};
// Optional per-kernel timing of the products (HM_PROFILE).
struct MvProfile {
  hipEvent_t ev[5];
  double ms[4];
  double launches[4];
};
struct MvPlan {
  const int32_t* row_beg;   // leaf -> first row item (nleaf + 1)
  const Item* row_items;    // dense row slices and U slices
  const int32_t* col_beg;
  const Item* col_items;    // V slices and dense blocks seen from a column leaf
  MvLeaves L;
  const int64_t* lr_meta;   // per low-rank block: toff, pslot, r, nk_rows, nk_cols, 0
  int64_t nlr;
  const int32_t* perm;
  int64_t n;
  void* xp;                 // workspace: gathered x
  void* partial;            // workspace: per-slice partial products
  void* t;                  // workspace: V^T x (or U^T x) per block
  int grid;
  MvProfile* prof;          // null unless profiling
};
void matvec_dispatch(const MvPlan& P, int storage_f32, const void* x, void* y, int nrhs,
                     int vec_f32, bool transposed, hipStream_t s);

// ---------------------------------------------------------------- primitives
// Exclusive scan of int64 values; *d_total (device) receives the sum.
void scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* d_total,
                   hipStream_t s);
// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of key.
void radix_sort_u64_i32(uint64_t* keys, int32_t* vals, int64_t n, int bits,
                        hipStream_t s);

// Stream-ordered temporary allocation (throws HM_ERR_OOM).
void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);
template <typename T>
T* dalloc_t(size_t count, hipStream_t s) {
  return static_cast<T*>(dalloc(count * sizeof(T) + 16, s));
}
int64_t d2h_i64(const int64_t* d, hipStream_t s);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline unsigned grid_for(int64_t n, int threads, int64_t cap = 1 << 20) {
  int64_t g = ceil_div(n, threads);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace hm
