// Internal declarations of the gfx950 H-matrix library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <functional>
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
constexpr int kNV = 3;              // vertices of a triangle
constexpr int kMaxLeaf = 64;        // leaf clusters fit one wavefront
constexpr int kMaxRank = 256;
constexpr int64_t kAcaPoolCap = int64_t(40) << 30;  // bytes of ACA working slots at once
constexpr int kAcaFirstRank = 24;   // rank cap of the first ACA pass (slot size)

// Radon's seven-point degree-5 rule: weights normalised to sum to one.
// Node q = 0 is the centroid; nodes 1..3 use (a1, a1, b1), 4..6 (a2, a2, b2).
// A node with barycentric weights (a, a, b), b on vertex v, lies at
// c + (b - a) (v - c) (c the centroid; 2a + b = 1): beta1 = b1 - a1 =
// (1 + sqrt 15) / 7 and beta2 = b2 - a2 = (1 - sqrt 15) / 7.
struct Radon7 {
  static constexpr double s15 = 3.872983346207416885179265399782399611;  // sqrt(15)
  static constexpr double a1 = (6.0 - s15) / 21.0;
  static constexpr double b1 = (9.0 + 2.0 * s15) / 21.0;
  static constexpr double a2 = (6.0 + s15) / 21.0;
  static constexpr double b2 = (9.0 - 2.0 * s15) / 21.0;
  static constexpr double w0 = 9.0 / 40.0;
  static constexpr double w1 = (155.0 - s15) / 1200.0;
  static constexpr double w2 = (155.0 + s15) / 1200.0;
  static constexpr double beta1 = (1.0 + s15) / 7.0;
  static constexpr double beta2 = (1.0 - s15) / 7.0;
};


// ---------------------------------------------------------------- device data
// Geometry in Morton order, structure of arrays.
//   c   : double[3][n]     centroids (collocation points)
//   o   : T[3*3][n]        vertex minus centroid, d_k = v_k - c: x of
//                          k = 0..2, then y, then z (the six outer nodes
//                          of the rule are c + beta d_k)
//   aw  : T[n]             |T_j| / (4 pi)
//   sf  : T[n]             analytic self-term a_jj
//   v   : double[9][n]     vertices (v0 xyz, v1 xyz, v2 xyz), Galerkin only
//   vid : int32[3][n]      global vertex indices, Galerkin only
template <typename T>
struct Geom {
  const double* c;
  const T* o;
  const T* aw;
  const T* sf;
  int64_t n;
  const double* v = nullptr;
  const int32_t* vid = nullptr;
};

// Operator of a handle: collocation at centroids (the default) or the
// paper's Galerkin discretisation (Sec. 2.2, eq. linearSystem).
enum { kOpColloc = 0, kOpGalerkin = 1 };

// Gauss-Legendre rule on [0, 1] for the singular Galerkin entries (outer
// integral in collapsed coordinates, kGalQ x kGalQ points).
constexpr int kGalQ = 12;
struct GaussRule {
  double x[kGalQ];
  double w[kGalQ];
};
GaussRule gauss_rule01();

// Cluster record: lo, hi (Morton positions), first child (-1 for a leaf), level.
using Cluster = int4;

// Galerkin admissibility: the test for triangles of two clusters that share
// a vertex (the supports of their basis functions touch).
//   vid   : int32[3][n]   vertex indices, Morton order
//   vbeg  : int32[nv + 1] vertex -> first entry of vpos
//   vpos  : int32[3 n]    Morton positions of the triangles around each vertex
//   reach2: (2 r_max)^2 with r_max the largest centroid-to-vertex distance;
//           the centroids of two touching triangles are at most 2 r_max apart
struct GalTouch {
  const int32_t* vid = nullptr;
  int32_t* vbeg = nullptr;
  int32_t* vpos = nullptr;
  int64_t n = 0;
  double reach2 = 0.0;
};
GalTouch make_gal_touch(const double* c, const double* tv, const int32_t* vid, int64_t n,
                        int64_t nv, hipStream_t s);
void free_gal_touch(GalTouch& t, hipStream_t s);



// Leaf table and the product plan.
struct MvLeaves {
  const int32_t* lo;
  const int32_t* m;
  const int64_t* ldpre;   // prefix of ld over leaves (nleaf + 1 entries)
  int64_t nleaf;
};
// One contiguous column-major panel (ld of its row leaf x w) of a row leaf;
// its column j multiplies z[colmap[col0 + j]].
struct Run {
  uint64_t data;
  int64_t col0;
  int32_t w;
  int32_t pad;
};
// Per admissible block: V factor address, rank, offset of its terms in t,
// first/last leaf of its column (sf, sl) and row (tf, tl) cluster, and the
// first entry of its U slices in the per-(block, row leaf) records.
// The V factor of a block is stored in column-leaf slices, each ld x r
// column-major; slice lf starts vw * (ldpre[lf] - ldpre[sf]) elements after
// vptr: blocks that share a column cluster (whose leaves share one ld) lie
// side by side in panels of vw = the sum of their ranks columns, a block
// alone has vw = r.  The same record with r = a chunk of a panel's columns
// describes a work unit of the forward phase 1.
struct LrMeta {
  uint64_t vptr;
  int32_t r, toff, sf, sl, tf, tl;
  int64_t ub;
  int32_t vld;   // ld shared by all column-leaf slices, 0 if they differ
  int32_t vw;    // slice width: columns between the slices of one leaf and the next
};
// Column-leaf item of the transposed product: kind 0 = columns of a dense
// slice (partial dots at w[src ..]), kind 1 = V slice at `data` (w = rank,
// src = toff of its block).
struct TItem {
  uint64_t data;
  int64_t src;
  int32_t w;
  int32_t kind;
};
// Optional per-kernel timing of the products (HM_PROFILE): four stages of
// the forward and four of the transposed product.
struct MvProfile {
  hipEvent_t ev[5];
  double ms[8];
  double launches[8];
};
// Unit of the per-row-leaf product kernels: columns [a, a + w) of run `run`
// of row leaf `leaf` (at most kUnitCols columns), so that a leaf with a wide
// panel is shared by several workgroups.  Units of a leaf are consecutive.
struct Unit {
  int32_t leaf, run, a, w;
};
constexpr int kUnitCols = 1024;

struct MvPlan {
  const Run* runs;          // [nruns][nleaf]
  int nruns;
  const Unit* units;        // nunits, grouped by leaf
  int64_t nunits;
  const int32_t* ubeg;      // leaf -> first unit (nleaf + 1)
  void* ypart;              // workspace: per-unit partial rows, ldmax x 16 each
  int64_t ypart_bytes;      // its size (the transposed product reuses it)
  int ldmax;
  const int32_t* colmap;
  const LrMeta* meta;
  int64_t nlr;
  const LrMeta* meta1;      // work units of the forward phase 1 (panel column chunks)
  int64_t nu1;
  const int64_t* ucol;
  const int32_t* tbeg;      // column leaf -> first transposed item (nleaf + 1)
  const TItem* titems;
  MvLeaves L;
  const int32_t* perm;
  int64_t n;
  void* z;                  // workspace: [x in Morton order ; t], 16 columns
  void* w;                  // workspace: panel-column partial dots
  const float* su;          // per-term scales of FP16 U factors (null: none)
  int max_nr_t;             // right-hand sides per transposed pass (w size)
  int grid;
  MvProfile* prof;          // null unless profiling
};

// Binning of the batched ACA: blocks fall into size bins by max(m, n) (upper
// edges kAcaBinEdge), and every bin is run by one kernel class: 0 one
// 1,024-thread workgroup per block, 1 one 256-thread workgroup, 2..4 one
// wavefront with 4, 2, 1 rows and columns per lane (up to 256, 128, 64),
// 5 one 128-thread workgroup.
constexpr int kAcaBins = 8;
constexpr int kAcaBinEdge[kAcaBins] = {64, 128, 256, 512, 1024, 2048, 4096, 0x7fffffff};
struct AcaBins {
  int cls[kAcaBins];
};
// One measured candidate of the binning tuner: bin, kernel class, sampled
// blocks and the time of one pass over them.
struct AcaTuneRow {
  int bin, cls;
  int64_t blocks;
  double ms;
};

// Inputs and outputs of the storage build (near field, ACA, panels).
struct SetupIn {
  int64_t n;
  const Cluster* cl;
  const int2* cl_leaves;
  const int32_t* leaf_lo;
  const int32_t* leaf_m;
  const int64_t* ldpre;
  int64_t nleaf;
  const int2* dns;
  int64_t nd;
  const int2* lr;
  int64_t nl;
  int kmax;
  double eps;
  int64_t pool_budget_bytes;   // upper bound for the ACA working pool
  int op;                      // kOpColloc or kOpGalerkin
  bool tune_aca = false;       // time the ACA kernel classes per size bin, keep the fastest
};
struct Storage {
  int64_t D_elems = 0, dense_cols = 0;
  int32_t* rank = nullptr;
  int32_t* info = nullptr;
  LrMeta* meta = nullptr;
  LrMeta* meta1 = nullptr;   // forward phase-1 units
  int64_t nu1 = 0;
  int64_t* ucol = nullptr;
  uint64_t* uptr = nullptr;
  int64_t lr_elems = 0, toff_total = 0, nchunks = 0, u_items = 0, aca_reruns = 0;
  Run* runs = nullptr;
  int nruns = 0;
  Unit* units = nullptr;
  int64_t nunits = 0;
  int unit_cols = 0;
  int32_t* ubeg = nullptr;
  int ldmax = 0;
  float* su = nullptr;       // per-term scales when the factors are FP16
  int64_t* dub = nullptr;    // dense block -> its first (block, row leaf) item
  uint64_t* dptr = nullptr;  // address of every dense item's slice (ld x n)
  int32_t* colmap = nullptr;
  int64_t ncols = 0;
  TItem* titems = nullptr;
  int32_t* tbeg = nullptr;
  int64_t ntitems = 0;
  double ms_near = 0, ms_aca = 0, ms_pack = 0;
  AcaBins bins{};                       // the binning the ACA ran with
  std::vector<AcaTuneRow> aca_tune;     // the tuner's measurements (empty without it)
};
using Alloc = std::function<void*(size_t)>;
// T: evaluation, ACA and dense storage type; TL: storage type of the
// low-rank factors (T, or _Float16 with per-term scales for U).
template <typename T, typename TL>
void build_storage(const Geom<T>& g, const SetupIn& in, Storage& out, const Alloc& alloc,
                   hipStream_t s);
void make_units(Storage& out, const int64_t* ldpre, int64_t nleaf, int ucols, const Alloc& alloc,
                hipStream_t s);
int64_t count_units(const Storage& out, int64_t nleaf, int ucols, hipStream_t s);
template <typename TL, typename TO>
void launch_unpack(const int2* lr, int64_t b, const Cluster* cl, const int32_t* leaf_lo,
                   const int32_t* leaf_m, const int64_t* ldpre, const int2* cl_leaves,
                   const LrMeta* meta, const uint64_t* uptr, const float* su, TO* out,
                   int64_t total, hipStream_t s);

// storage: 0 FP64, 1 FP32, 2 FP32 dense + FP16 factors
void matvec_dispatch(const MvPlan& P, int storage, const void* x, void* y, int nrhs,
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
// The library's memory pool on the current device; trim_pool() returns what
// it caches (memory not owned by a live handle) to the device.
hipMemPool_t lib_pool();
void trim_pool();
// Cache of device blocks of freed handles on the current device: take one of
// at least `bytes` (and at most 1/8 more; its size in *got) or nullptr; put
// one back; free all.
void* cache_take(size_t bytes, size_t* got);
void cache_put(void* p, size_t bytes);
void cache_release();
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
