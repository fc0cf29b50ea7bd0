// C ABI of the library and the host orchestration of the setup (Sec. 3:
// clustering, level-wise block tree, batched near field, batched ACA), the
// products and the GMRES loop.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hm_internal.h"

namespace hm {

// ---- launchers defined in the other translation units
void launch_centroids(const double* V, const int32_t* T, int64_t n, double* C, hipStream_t s);
void launch_minmax(const double* C, int64_t n, int64_t off, int64_t cnt, double* out6,
                   hipStream_t s);
void launch_morton(const double* C, int64_t n, int64_t off, int64_t cnt, const double* a,
                   double scale, uint64_t* keys, int32_t* idx, hipStream_t s);
template <typename T>
void launch_geom_sorted(const double* V, const int32_t* Tri, const int32_t* perm, int64_t n,
                        double* c, T* o, T* aw, T* sf, hipStream_t s);
int64_t build_cluster_tree(const std::vector<int64_t>& goff, int leaf, Cluster* cl, int64_t cap,
                           std::vector<int64_t>& level_beg, hipStream_t s);
void launch_leaf_marks(const Cluster* cl, int64_t ncl, int64_t* mark, hipStream_t s);
void launch_pos_leaf(const int64_t* mark, const int64_t* excl, int64_t n, int32_t* pos_leaf,
                     hipStream_t s);
void launch_leaf_table(const Cluster* cl, int64_t ncl, const int32_t* pos_leaf, int32_t* leaf_lo,
                       int32_t* leaf_m, int32_t* leaf_cl, int64_t* leaf_ld, int2* cl_leaves,
                       hipStream_t s);
void launch_boxes(const Cluster* cl, const std::vector<int64_t>& level_beg, const int32_t* leaf_cl,
                  int64_t nleaf, const double* c, int64_t n, double* box, hipStream_t s);
void build_block_tree(const Cluster* cl, int64_t nroots, const double* box, double eta, int leaf,
                      const GalTouch& gt, int2** adm_out, int64_t* nadm, int2** dns_out,
                      int64_t* ndns, int64_t* depth, hipStream_t s);
template <typename T>
void launch_entries(const Geom<T>& g, int op, const int32_t* inv, const int32_t* rows,
                    const int32_t* cols, int64_t cnt, double* out, hipStream_t s);
void launch_tri_sorted(const double* V, const int32_t* Tri, const int32_t* perm, int64_t n,
                       double* v, int32_t* vid, hipStream_t s);
void launch_inverse_perm(const int32_t* perm, int64_t n, int32_t* inv, hipStream_t s);

int gmres_tiles(int64_t n);
void gmres_dots(const double* Q, int64_t ldq, int nk, const double* w, int64_t n, int nr,
                double* part, double* out, hipStream_t s);
void gmres_orth_update(const double* Q, int64_t ldq, const double* h, int nk, int64_t n, int nr,
                       double* w, hipStream_t s);
void gmres_combine(const double* Q, int64_t ldq, const double* y, int nk, int64_t n, int nr,
                   double* x, hipStream_t s);
void gmres_scale_cols(const double* a, const double* sc, int64_t n, int nr, double* out,
                      hipStream_t s);
void gmres_sub(const double* a, const double* b, int64_t tot, double* out, hipStream_t s);
void gmres_dots_dev(const double* Q, int64_t ldq, const int* jd, int nkmax, const double* w,
                    int64_t n, int nr, double* part, double* out, hipStream_t s);
void gmres_orth_update_dev(const double* Q, int64_t ldq, const double* h, const int* jd,
                           int64_t n, int nr, double* w, hipStream_t s);
void gmres_copy_col(const double* Q, int64_t ldq, const int* jd, double* out, hipStream_t s);

// Device workspace of a solve.  With HM_SOLVE_GRAPH it stays with the handle
// together with the instantiated graph of one Arnoldi step (product of the
// current basis vector, two Gram-Schmidt passes, norm), which is replayed
// for every step; the step index is read from device memory (jd).
//
// Buffers: Q the basis (m + 1 vectors), fd the right-hand side of the GMRES
// run, x its iterate, w the product / residual, xin the captured step's
// input; with refinement also fo (the caller's right-hand side), xs (the
// refined solution) and the float vectors xf, wf of the inner products.
struct SolveWs {
  int nr = 0, m = 0;
  bool tr = false, f32 = false;
  int64_t n = 0;
  double *Q = nullptr, *fd = nullptr, *x = nullptr, *w = nullptr, *hdev = nullptr,
         *part = nullptr, *scl = nullptr, *ydev = nullptr, *xin = nullptr, *fo = nullptr,
         *xs = nullptr;
  float *xf = nullptr, *wf = nullptr;
  int* jd = nullptr;
  std::vector<void*> mem;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t free_stream = nullptr;
  // Lays the buffers out through get(count of doubles) -> double*.
  template <typename Get>
  void layout(int64_t n_, int nr_, int m_, bool tr_, bool f32_, Get&& get) {
    n = n_, nr = nr_, m = m_, tr = tr_, f32 = f32_;
    const int64_t nv = n * nr;
    Q = get((size_t)(m + 1) * nv);
    fd = get(nv);
    x = get(nv);
    w = get(nv);
    xin = get(nv);
    hdev = get((size_t)(m + 2) * nr * 2 + nr);
    part = get((size_t)(m + 2) * gmres_tiles(n) * nr);
    scl = get(nr);
    ydev = get((size_t)(m + 1) * nr);
    jd = (int*)get(1);
    if (f32) {
      fo = get(nv);
      xs = get(nv);
      xf = (float*)get((nv + 1) / 2);
      wf = (float*)get((nv + 1) / 2);
    }
  }
  // From the library's pool (stream-ordered), freed with the workspace.
  void alloc(int64_t n_, int nr_, int m_, bool tr_, bool f32_, hipStream_t s) {
    layout(n_, nr_, m_, tr_, f32_, [&](size_t cnt) {
      double* q = (double*)dalloc(cnt * sizeof(double), s);
      mem.push_back(q);
      return q;
    });
  }
  ~SolveWs() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (mem.empty()) return;
    for (void* q : mem) (void)hipFreeAsync(q, free_stream);
    (void)hipStreamSynchronize(free_stream);
  }
};
void convert_f32_to_f64(const float* a, int64_t tot, double* out, hipStream_t s);
void convert_f64_to_f32(const double* a, int64_t tot, float* out, hipStream_t s);
void gmres_add(const double* a, const double* b, int64_t tot, double* out, hipStream_t s);
void cg_update(double* x, double* r, const double* p, const double* q, const double* rr,
               const double* pq, const double* active, int64_t n, int nr, hipStream_t s);
void cg_dir(double* p, const double* r, const double* rr_new, const double* rr_old,
            const double* active, int64_t n, int nr, hipStream_t s);
void gmres_copy_col_f32(const double* Q, int64_t ldq, const int* jd, float* out, hipStream_t s);

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

constexpr int kMaxNr = 16;   // right-hand sides per product pass
constexpr int kMaxGeoms = 65536;
// unit widths the product autotuner tries, the smallest first
constexpr int kTuneCols[] = {512, 1024, 2048, 4096, 8192};

// Block statistics of a build, summed on the device: out[0] dense entries,
// [1] low-rank entries sum r (m + n), [2] U entries sum r m, [3] rank sum,
// [4] rank max, [5] cap hits, [6] ACA entry evaluations (rows evaluated n +
// r m).  out must be zero on entry; one atomic per wavefront and value.
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  return v;
}
__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
  for (int s = 32; s > 0; s >>= 1) {
    const unsigned long long o = __shfl_xor(v, s, 64);
    v = o > v ? o : v;
  }
  return v;
}
__global__ __launch_bounds__(256) void k_block_stats(const int2* __restrict__ dns, int64_t nd, const int2* __restrict__ lr,
                              int64_t nl, const int4* __restrict__ cl,
                              const int32_t* __restrict__ rank, const int32_t* __restrict__ info,
                              unsigned long long* __restrict__ out) {
  unsigned long long v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nd + nl;
       b += (int64_t)gridDim.x * blockDim.x) {
    if (b < nd) {
      const int4 t = cl[dns[b].x], sg = cl[dns[b].y];
      v[0] += (unsigned long long)(t.y - t.x) * (unsigned long long)(sg.y - sg.x);
    } else {
      const int64_t k = b - nd;
      const int4 t = cl[lr[k].x], sg = cl[lr[k].y];
      const unsigned long long m = t.y - t.x, nn = sg.y - sg.x, r = rank[k];
      const unsigned long long rows = (unsigned)info[k] >> 1;
      v[1] += r * (m + nn);
      v[2] += r * m;
      v[3] += r;
      v[4] = r > v[4] ? r : v[4];
      v[5] += (unsigned)info[k] & 1u;
      v[6] += rows * nn + r * m;
    }
  }
  // wave reduction, then the 4 waves through LDS: one atomic per value and workgroup
  __shared__ unsigned long long part[4][7];
  const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 7; ++k) v[k] = k == 4 ? wave_max_u64(v[k]) : wave_sum_u64(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 7; ++k) part[wave][k] = v[k];
  }
  __syncthreads();
  if ((int)threadIdx.x < 7) {
    const int k = (int)threadIdx.x;
    unsigned long long a = part[0][k];
    for (int w = 1; w < 4; ++w) a = k == 4 ? (part[w][k] > a ? part[w][k] : a) : a + part[w][k];
    if (k == 4)
      atomicMax(out + k, a);
    else
      atomicAdd(out + k, a);
  }
}

}  // namespace hm

using namespace hm;

// ------------------------------------------------------------------ handle
struct hm_handle {
  int device = 0;
  hm_params p{};
  int64_t n = 0;
  int form = 0;                  // hm_precision
  int f32 = 0;                   // evaluation in float
  size_t ts = 8;                 // bytes per stored value
  std::vector<std::pair<void*, size_t>> owned;   // persistent allocations and sizes
  int64_t bytes = 0;

  double* c = nullptr;           // centroids, Morton order
  void* o = nullptr;
  void* aw = nullptr;
  void* sf = nullptr;
  int op = kOpColloc;            // kOpGalerkin with HM_GALERKIN
  double* tv = nullptr;          // Galerkin: vertices, Morton order [9][n]
  int32_t* vid = nullptr;        // Galerkin: vertex indices [3][n]
  uint64_t* keys = nullptr;      // Morton keys, application order
  int32_t* perm = nullptr;       // Morton position -> triangle
  int32_t* inv = nullptr;

  int64_t ncl = 0, depth = 0;
  Cluster* cl = nullptr;
  double* box = nullptr;
  int2* cl_leaves = nullptr;
  int64_t nleaf = 0;
  int32_t *leaf_lo = nullptr, *leaf_m = nullptr, *leaf_cl = nullptr;
  int64_t* ldpre = nullptr;

  int64_t nd = 0, nl = 0;
  int2 *dns = nullptr, *lr = nullptr;
  Storage sto;

  void *z = nullptr, *w = nullptr, *ypart = nullptr;
  int64_t ypart_bytes = 0;
  std::unique_ptr<SolveWs> sws;         // graph-replay solve workspace
  std::vector<std::array<double, 2>> tune;   // autotuner: (unit columns, ms)
  int max_nr_t = 1;
  int grid = 1024;

  hipStream_t alloc_stream = nullptr;   // stream of the build (owned allocations)
  std::vector<int64_t> goff;            // triangle offsets of the geometries (G + 1)
  hm_stats st{};
  double ms[HM_NPHASE] = {0};
  MvProfile prof{};
  bool profiling = false;

  void* alloc(size_t b) {
    if (b == 0) b = 16;
    if (p.mem_limit_bytes > 0 && bytes + (int64_t)b > p.mem_limit_bytes)
      throw Error{HM_ERR_OOM, "mem_limit_bytes exceeded (" + std::to_string(bytes + b) + " > " +
                                  std::to_string(p.mem_limit_bytes) + ")"};
    // a block of a freed handle, else stream-ordered from the library's pool
    // (on the stream of the build)
    size_t got = b;
    void* q = cache_take(b, &got);
    if (!q) {
      q = dalloc(b, alloc_stream);
      got = b;
    }
    owned.push_back({q, got});
    bytes += (int64_t)b;
    return q;
  }
  template <typename X>
  X* alloc_t(size_t cnt) {
    return static_cast<X*>(alloc(cnt * sizeof(X)));
  }
  ~hm_handle() {
    if (profiling)
      for (auto& e : prof.ev) (void)hipEventDestroy(e);
    // nothing may still use the blocks when they go to the cache (a failed
    // build can leave work in flight; the build stream may no longer exist)
    (void)hipDeviceSynchronize();
    for (auto& q : owned) cache_put(q.first, q.second);
  }
  MvPlan plan() const {
    MvPlan P;
    P.runs = sto.runs;
    P.nruns = sto.nruns;
    P.units = sto.units;
    P.nunits = sto.nunits;
    P.ubeg = sto.ubeg;
    P.ypart = ypart;
    P.ypart_bytes = ypart_bytes;
    P.ldmax = sto.ldmax;
    P.colmap = sto.colmap;
    P.meta = sto.meta;
    P.nlr = nl;
    P.meta1 = sto.meta1;
    P.nu1 = sto.nu1;
    P.ucol = sto.ucol;
    P.tbeg = sto.tbeg;
    P.titems = sto.titems;
    P.L = MvLeaves{leaf_lo, leaf_m, ldpre, nleaf};
    P.perm = perm;
    P.n = n;
    P.z = z;
    P.w = w;
    P.su = sto.su;
    P.max_nr_t = max_nr_t;
    P.grid = grid;
    P.prof = profiling ? const_cast<MvProfile*>(&prof) : nullptr;
    return P;
  }
};

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// The setup's temporaries go back to the library's pool, which keeps them
// cached for the next build (hm_release_memory returns them to the device).
void release_cached_memory(hipStream_t s) {
  HM_HIP(hipStreamSynchronize(s));
}

template <typename F>
hm_status guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const Error& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return HM_ERR_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return HM_ERR_STATE;
  }
}

hm_status arg_error(const std::string& m) {
  g_err = m;
  return HM_ERR_ARG;
}

// Offsets + total of n int64 values (device); returns the total.
int64_t scan_total(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
  scan_excl_i64(in, out, n, tmp, s);
  return d2h_i64(tmp, s);
}

// ---------------------------------------------------------------- the build
// Autotuner of the product schedule: the width of the column units of the
// per-leaf kernels decides how evenly the panels spread over the CUs
// against how many partial rows are summed.  Every candidate is timed on
// this handle's own storage (one untimed and three timed one-column
// products of a zero vector; the work does not depend on the values) and the
// fastest is kept.
void autotune_units(hm_handle* h, hipStream_t s) {
  const int64_t n = h->n;
  double* xt = dalloc_t<double>(n, s);
  double* yt = dalloc_t<double>(n, s);
  HM_HIP(hipMemsetAsync(xt, 0, n * sizeof(double), s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HM_HIP(hipEventCreate(&e0));
  HM_HIP(hipEventCreate(&e1));
  struct Guard {
    hipEvent_t a, b;
    ~Guard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } gd{e0, e1};
  const bool prof = h->profiling;
  h->profiling = false;
  h->tune.clear();
  int best = h->sto.unit_cols;
  float best_ms = 0.f;
  for (int ucols : kTuneCols) {
    make_units(h->sto, h->ldpre, h->nleaf, ucols, [h](size_t b) { return h->alloc(b); }, s);
    const MvPlan P = h->plan();
    matvec_dispatch(P, h->form, xt, yt, 1, 0, false, s);
    HM_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r) matvec_dispatch(P, h->form, xt, yt, 1, 0, false, s);
    HM_HIP(hipEventRecord(e1, s));
    HM_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    HM_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms /= 3.f;
    h->tune.push_back({(double)ucols, (double)ms});
    if (best_ms == 0.f || ms < best_ms) {
      best_ms = ms;
      best = ucols;
    }
  }
  make_units(h->sto, h->ldpre, h->nleaf, best, [h](size_t b) { return h->alloc(b); }, s);
  h->profiling = prof;
  dfree(xt, s);
  dfree(yt, s);
}

template <typename T, typename TL>
void build_impl(hm_handle* h, const double* V_host, int64_t nv, const int32_t* T_host,
                hipStream_t s) {
  const std::vector<int64_t>& goff = h->goff;   // triangle offsets of the geometries
  const int64_t G = (int64_t)goff.size() - 1;
  const int64_t n = h->n;
  const hm_params& p = h->p;
  const auto t_start = clk::now();
  auto t0 = clk::now();
  int64_t* tmp = dalloc_t<int64_t>(4, s);

  // ---- upload + geometry (application order)
  double* V = dalloc_t<double>(3 * nv, s);
  int32_t* Tri = dalloc_t<int32_t>(3 * n, s);
  HM_HIP(hipMemcpyAsync(V, V_host, 3 * nv * sizeof(double), hipMemcpyHostToDevice, s));
  HM_HIP(hipMemcpyAsync(Tri, T_host, 3 * n * sizeof(int32_t), hipMemcpyHostToDevice, s));
  double* Capp = dalloc_t<double>(3 * n, s);
  launch_centroids(V, Tri, n, Capp, s);
  HM_HIP(hipStreamSynchronize(s));
  h->ms[0] = ms_since(t0);

  // ---- Morton codes and sort
  t0 = clk::now();
  // every geometry has its own cube box and is sorted within its own range
  double* mm = dalloc_t<double>(6 * G, s);
  for (int64_t g = 0; g < G; ++g) launch_minmax(Capp, n, goff[g], goff[g + 1] - goff[g], mm + 6 * g, s);
  std::vector<double> mmh(6 * G);
  HM_HIP(hipMemcpyAsync(mmh.data(), mm, 6 * G * sizeof(double), hipMemcpyDeviceToHost, s));
  HM_HIP(hipStreamSynchronize(s));
  h->keys = h->alloc_t<uint64_t>(n);
  h->perm = h->alloc_t<int32_t>(n);
  h->inv = h->alloc_t<int32_t>(n);
  uint64_t* ksort = dalloc_t<uint64_t>(n, s);
  for (int64_t g = 0; g < G; ++g) {
    const double* mg = mmh.data() + 6 * g;
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) ext = std::max(ext, mg[3 + d] - mg[d]);
    const double scale = ext > 0.0 ? 2097152.0 / ext : 0.0;
    launch_morton(Capp, n, goff[g], goff[g + 1] - goff[g], mg, scale, h->keys, h->perm, s);
  }
  HM_HIP(hipMemcpyAsync(ksort, h->keys, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
  for (int64_t g = 0; g < G; ++g)
    radix_sort_u64_i32(ksort + goff[g], h->perm + goff[g], goff[g + 1] - goff[g],
                       3 * kMortonBits, s);
  launch_inverse_perm(h->perm, n, h->inv, s);
  dfree(ksort, s);
  dfree(mm, s);
  dfree(Capp, s);

  // ---- geometry in Morton order
  h->c = h->alloc_t<double>(3 * n);
  h->o = h->alloc(3 * kNV * n * sizeof(T));
  h->aw = h->alloc(n * sizeof(T));
  h->sf = h->alloc(n * sizeof(T));
  launch_geom_sorted<T>(V, Tri, h->perm, n, h->c, (T*)h->o, (T*)h->aw, (T*)h->sf, s);
  if (h->op == kOpGalerkin) {
    h->tv = h->alloc_t<double>(9 * n);
    h->vid = h->alloc_t<int32_t>(3 * n);
    launch_tri_sorted(V, Tri, h->perm, n, h->tv, h->vid, s);
  }
  dfree(V, s);
  dfree(Tri, s);
  HM_HIP(hipStreamSynchronize(s));
  h->ms[1] = ms_since(t0);
  const Geom<T> g{h->c, (const T*)h->o, (const T*)h->aw, (const T*)h->sf, n, h->tv, h->vid};

  // ---- cluster tree, leaves, boxes
  t0 = clk::now();
  const int64_t cap = 2 * n + 2 * G;
  Cluster* cltmp = dalloc_t<Cluster>(cap, s);
  std::vector<int64_t> level_beg;
  h->ncl = build_cluster_tree(goff, p.leaf_size, cltmp, cap, level_beg, s);
  h->cl = h->alloc_t<Cluster>(h->ncl);
  HM_HIP(hipMemcpyAsync(h->cl, cltmp, h->ncl * sizeof(Cluster), hipMemcpyDeviceToDevice, s));
  dfree(cltmp, s);
  int64_t* mark = dalloc_t<int64_t>(n, s);
  int64_t* excl = dalloc_t<int64_t>(n, s);
  HM_HIP(hipMemsetAsync(mark, 0, n * sizeof(int64_t), s));
  launch_leaf_marks(h->cl, h->ncl, mark, s);
  h->nleaf = scan_total(mark, excl, n, tmp, s);
  int32_t* pos_leaf = dalloc_t<int32_t>(n, s);
  launch_pos_leaf(mark, excl, n, pos_leaf, s);
  dfree(mark, s);
  dfree(excl, s);
  h->leaf_lo = h->alloc_t<int32_t>(h->nleaf);
  h->leaf_m = h->alloc_t<int32_t>(h->nleaf);
  h->leaf_cl = h->alloc_t<int32_t>(h->nleaf);
  h->cl_leaves = h->alloc_t<int2>(h->ncl);
  h->ldpre = h->alloc_t<int64_t>(h->nleaf + 1);
  int64_t* leaf_ld = dalloc_t<int64_t>(h->nleaf, s);
  launch_leaf_table(h->cl, h->ncl, pos_leaf, h->leaf_lo, h->leaf_m, h->leaf_cl, leaf_ld,
                    h->cl_leaves, s);
  scan_excl_i64(leaf_ld, h->ldpre, h->nleaf, h->ldpre + h->nleaf, s);
  dfree(leaf_ld, s);
  dfree(pos_leaf, s);
  h->box = h->alloc_t<double>(6 * h->ncl);
  launch_boxes(h->cl, level_beg, h->leaf_cl, h->nleaf, h->c, n, h->box, s);
  HM_HIP(hipStreamSynchronize(s));
  h->ms[2] = ms_since(t0);

  // ---- block cluster tree (Algorithm 1, level-wise)
  t0 = clk::now();
  int2 *adm = nullptr, *dns = nullptr;
  GalTouch gt;
  if (h->op == kOpGalerkin) gt = make_gal_touch(h->c, h->tv, h->vid, n, nv, s);
  build_block_tree(h->cl, G, h->box, p.eta, p.leaf_size, gt, &adm, &h->nl, &dns, &h->nd, &h->depth,
                   s);
  free_gal_touch(gt, s);
  h->lr = h->alloc_t<int2>(h->nl);
  h->dns = h->alloc_t<int2>(h->nd);
  if (h->nl) HM_HIP(hipMemcpyAsync(h->lr, adm, h->nl * sizeof(int2), hipMemcpyDeviceToDevice, s));
  if (h->nd) HM_HIP(hipMemcpyAsync(h->dns, dns, h->nd * sizeof(int2), hipMemcpyDeviceToDevice, s));
  dfree(adm, s);
  dfree(dns, s);
  HM_HIP(hipStreamSynchronize(s));
  h->ms[3] = ms_since(t0);

  // ---- near field, batched ACA, panels and product plan
  {
    size_t freeb = 0, totb = 0;
    HM_HIP(hipMemGetInfo(&freeb, &totb));
    // ACA working pool: at most 40% of the free memory and at most
    // kAcaPoolCap.  A larger pool means fewer chunks (each chunk costs host
    // synchronisations) but a large transient allocation; it comes from the
    // block cache when an earlier build returned one of its size.
    int64_t budget = std::min<int64_t>((int64_t)(0.40 * (double)freeb), kAcaPoolCap);
    if (p.mem_limit_bytes > 0) budget = std::min(budget, (p.mem_limit_bytes - h->bytes) / 3);
    SetupIn in{n, h->cl, h->cl_leaves, h->leaf_lo, h->leaf_m, h->ldpre, h->nleaf,
               h->dns, h->nd, h->lr, h->nl, p.max_rank > 0 ? p.max_rank : 64, p.aca_eps,
               std::max<int64_t>(budget, 1 << 20), h->op,
               (p.flags & HM_AUTOTUNE) != 0};
    build_storage<T, TL>(g, in, h->sto, [h](size_t b) { return h->alloc(b); }, s);
    h->ms[4] = h->sto.ms_near;
    h->ms[5] = h->sto.ms_aca;
    h->ms[6] = h->sto.ms_pack;
  }
  t0 = clk::now();
  // ---- product workspace: z = [x ; t] with 16 columns, w for the
  // transposed product sized to at most 2 GB (fewer columns per pass)
  h->z = h->alloc((size_t)(n + h->sto.toff_total + 1) * kMaxNr * sizeof(double));
  {
    // partial rows for the most units any unit size of the tuner produces
    int64_t nu = h->sto.nunits;
    if (p.flags & HM_AUTOTUNE)
      nu = std::max(nu, count_units(h->sto, h->nleaf, kTuneCols[0], s));
    h->ypart_bytes = (nu + 1) * (int64_t)h->sto.ldmax * kMaxNr * (int64_t)sizeof(double);
    h->ypart = h->alloc((size_t)h->ypart_bytes);
  }
  {
    const int64_t cols = h->sto.ncols + 1;
    int nrt = kMaxNr;
    while (nrt > 1 && (double)cols * nrt * sizeof(double) > 2.0e9) nrt >>= 1;
    h->max_nr_t = nrt;
    h->w = h->alloc((size_t)cols * nrt * sizeof(double));
  }
  int dev = 0, ncu = 0;
  HM_HIP(hipGetDevice(&dev));
  HM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  h->grid = std::max(ncu, 1) * 32;
  HM_HIP(hipStreamSynchronize(s));
  h->ms[6] += ms_since(t0);
  if (p.flags & HM_AUTOTUNE) autotune_units(h, s);
  dfree(tmp, s);
  release_cached_memory(s);

  // ---- statistics: block sums on the device, one small copy back
  hm_stats& st = h->st;
  std::memset(&st, 0, sizeof(st));
  st.n = n;
  st.n_clusters = h->ncl;
  st.n_leaves = h->nleaf;
  st.n_dense = h->nd;
  st.n_lr = h->nl;
  st.depth = h->depth;
  {
    unsigned long long* dsum = static_cast<unsigned long long*>(dalloc(7 * sizeof(unsigned long long), s));
    HM_HIP(hipMemsetAsync(dsum, 0, 7 * sizeof(unsigned long long), s));
    if (h->nd + h->nl > 0) {
      k_block_stats<<<grid_for(h->nd + h->nl, 256, 256), 256, 0, s>>>(
          h->dns, h->nd, h->lr, h->nl, h->cl, h->sto.rank, h->sto.info, dsum);
      HM_LAUNCH_CHECK();
    }
    unsigned long long hs[7];
    HM_HIP(hipMemcpyAsync(hs, dsum, sizeof(hs), hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    dfree(dsum, s);
    st.dense_entries = (int64_t)hs[0];
    st.lr_entries = (int64_t)hs[1];
    st.lr_u_entries = (int64_t)hs[2];
    st.rank_sum = (int64_t)hs[3];
    st.rank_max = (int64_t)hs[4];
    st.cap_hits = (int64_t)hs[5];
    st.aca_entry_evals = (int64_t)hs[6];
  }
  st.stored_bytes = h->sto.D_elems * (int64_t)sizeof(T) + h->sto.lr_elems * (int64_t)sizeof(TL);
  st.n_panel_cols = h->sto.ncols;
  st.n_titems = h->sto.ntitems;
  st.device_bytes = h->bytes;
  st.precision = h->form;
  st.aca_chunks = h->sto.nchunks;
  st.n_geom = (int64_t)h->goff.size() - 1;
  st.unit_cols = h->sto.unit_cols;
  h->ms[7] = ms_since(t_start);
  if ((p.flags & HM_STRICT) && st.cap_hits > 0)
    throw Error{HM_ERR_ACA, std::to_string(st.cap_hits) + " blocks reached max_rank"};
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

// ------------------------------------------------------------------ GMRES core
namespace {
// Restarted GMRES on op(H) x = b for every column of b at once (the columns
// are independent systems).  `apply` computes w = op(H) v for double vectors
// v, w of the solve workspace; the Arnoldi basis, the Gram-Schmidt passes and
// the Givens rotations are in double.  b is ws->fd, the iterate ws->x (read
// as the initial guess, written back).  Returns the number of Arnoldi steps;
// rn receives the explicit residual norms |b - op(H) x| at the end.
// With x_zero the initial guess is known to be zero and the first residual is
// b itself (one product fewer).
template <typename Apply, typename Step>
int gmres_core(SolveWs* ws, int64_t n, int nr, int m, double tol, int max_iter, bool use_graph,
               const Apply& apply, const Step& graph_step, const std::vector<double>& fn,
               std::vector<double>& rn, std::vector<int>& conv, int& restarts, bool x_zero,
               hipStream_t s) {
  const int64_t nv = n * nr;
  double *Q = ws->Q, *fd = ws->fd, *x = ws->x, *w = ws->w, *hdev = ws->hdev, *part = ws->part,
         *scl = ws->scl, *ydev = ws->ydev;
  double* hnorm = hdev + (size_t)(m + 2) * nr * 2;   // |w| of the current step
  std::vector<double> hv((size_t)(m + 2) * nr * 2 + nr);
  auto norms = [&](const double* v, std::vector<double>& out) {
    gmres_dots(v, 0, 1, v, n, nr, part, hdev, s);
    out.resize(nr);
    HM_HIP(hipMemcpyAsync(out.data(), hdev, nr * sizeof(double), hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    for (auto& z : out) z = std::sqrt(std::max(z, 0.0));
  };
  // r = b - op(H) x  (into w)
  auto residual = [&](std::vector<double>& r) {
    apply(x, w);
    gmres_sub(fd, w, nv, w, s);
    norms(w, r);
  };
  auto rel = [&](int c, double r) { return fn[c] > 0 ? r / fn[c] : 0.0; };
  if (x_zero) {
    HM_HIP(hipMemcpyAsync(w, fd, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
    rn = fn;
  } else {
    residual(rn);
  }
  conv.assign(nr, 0);
  for (int c = 0; c < nr; ++c) conv[c] = rel(c, rn[c]) <= tol;
  int total_it = 0;
  // per-column Arnoldi state
  std::vector<double> H((size_t)(m + 1) * m * nr), cs((size_t)m * nr), sn((size_t)m * nr),
      gv((size_t)(m + 1) * nr);
  std::vector<int> kc(nr);
  std::vector<double> sc(nr);
  while (total_it < max_iter) {
    bool all = true;
    for (int c = 0; c < nr; ++c) all = all && conv[c];
    if (all) break;
    // Q0 = r / |r| for active columns
    for (int c = 0; c < nr; ++c) sc[c] = (!conv[c] && rn[c] > 0) ? 1.0 / rn[c] : 0.0;
    HM_HIP(hipMemcpyAsync(scl, sc.data(), nr * sizeof(double), hipMemcpyHostToDevice, s));
    gmres_scale_cols(w, scl, n, nr, Q, s);
    std::vector<int> active(nr);
    for (int c = 0; c < nr; ++c) {
      active[c] = !conv[c];
      kc[c] = 0;
      std::fill(gv.begin() + (size_t)c * (m + 1), gv.begin() + (size_t)(c + 1) * (m + 1), 0.0);
      gv[(size_t)c * (m + 1)] = rn[c];
    }
    for (int j = 0; j < m && total_it < max_iter; ++j) {
      if (use_graph) {
        graph_step(j);
      } else {
        double* qj = Q + (size_t)j * nv;
        apply(qj, w);
        // classical Gram-Schmidt, twice
        for (int pass = 0; pass < 2; ++pass) {
          gmres_dots(Q, nv, j + 1, w, n, nr, part, hdev + (size_t)pass * (m + 2) * nr, s);
          gmres_orth_update(Q, nv, hdev + (size_t)pass * (m + 2) * nr, j + 1, n, nr, w, s);
        }
        gmres_dots(w, 0, 1, w, n, nr, part, hnorm, s);
      }
      HM_HIP(hipMemcpyAsync(hv.data(), hdev, hv.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HM_HIP(hipStreamSynchronize(s));
      ++total_it;
      bool any = false;
      for (int c = 0; c < nr; ++c) {
        const double hn = std::sqrt(std::max(hv[(size_t)(m + 2) * nr * 2 + c], 0.0));
        sc[c] = 0.0;
        if (!active[c]) continue;
        double* Hc = H.data() + (size_t)c * (m + 1) * m;
        for (int k = 0; k <= j; ++k)
          Hc[(size_t)k * m + j] = hv[(size_t)k * nr + c] + hv[(size_t)(m + 2) * nr + (size_t)k * nr + c];
        Hc[(size_t)(j + 1) * m + j] = hn;
        // previous rotations
        double* csc = cs.data() + (size_t)c * m;
        double* snc = sn.data() + (size_t)c * m;
        for (int k = 0; k < j; ++k) {
          const double a = Hc[(size_t)k * m + j], b = Hc[(size_t)(k + 1) * m + j];
          Hc[(size_t)k * m + j] = csc[k] * a + snc[k] * b;
          Hc[(size_t)(k + 1) * m + j] = -snc[k] * a + csc[k] * b;
        }
        const double a = Hc[(size_t)j * m + j], b = Hc[(size_t)(j + 1) * m + j];
        const double rr = std::hypot(a, b);
        csc[j] = rr > 0 ? a / rr : 1.0;
        snc[j] = rr > 0 ? b / rr : 0.0;
        Hc[(size_t)j * m + j] = rr;
        Hc[(size_t)(j + 1) * m + j] = 0.0;
        double* gc = gv.data() + (size_t)c * (m + 1);
        gc[j + 1] = -snc[j] * gc[j];
        gc[j] = csc[j] * gc[j];
        kc[c] = j + 1;
        const double est = rel(c, std::fabs(gc[j + 1]));
        if (est <= tol || hn == 0.0) {
          active[c] = 0;
        } else {
          sc[c] = 1.0 / hn;
          any = true;
        }
      }
      if (!any) break;
      HM_HIP(hipMemcpyAsync(scl, sc.data(), nr * sizeof(double), hipMemcpyHostToDevice, s));
      gmres_scale_cols(w, scl, n, nr, Q + (size_t)(j + 1) * nv, s);
    }
    // x += Q y  (upper triangular solves on the host)
    int kmaxc = 0;
    for (int c = 0; c < nr; ++c) kmaxc = std::max(kmaxc, kc[c]);
    if (kmaxc > 0) {
      std::vector<double> y((size_t)kmaxc * nr, 0.0);
      for (int c = 0; c < nr; ++c) {
        const double* Hc = H.data() + (size_t)c * (m + 1) * m;
        const double* gc = gv.data() + (size_t)c * (m + 1);
        for (int k = kc[c] - 1; k >= 0; --k) {
          double v = gc[k];
          for (int l = k + 1; l < kc[c]; ++l) v -= Hc[(size_t)k * m + l] * y[(size_t)l * nr + c];
          y[(size_t)k * nr + c] = Hc[(size_t)k * m + k] != 0.0 ? v / Hc[(size_t)k * m + k] : 0.0;
        }
      }
      HM_HIP(hipMemcpyAsync(ydev, y.data(), y.size() * sizeof(double), hipMemcpyHostToDevice, s));
      gmres_combine(Q, nv, ydev, kmaxc, n, nr, x, s);
    }
    ++restarts;
    residual(rn);
    for (int c = 0; c < nr; ++c) conv[c] = rel(c, rn[c]) <= tol;
  }
  return total_it;
}

// Conjugate gradients (Sec. 4.1: the solver of the symmetric Galerkin
// system, one product per step) for every column of b = ws->fd at once, each
// with its own step lengths; the iterate ws->x is read as the initial guess
// and written back.  In cycles: the residual b - H x is computed
// explicitly, CG runs on the unconverged columns (r in Q, p in Q + nv, H p
// in w) until their recursively updated residuals reach tol, and the
// explicit residual decides again; a cycle that improves no unconverged
// column by 10% ends the solve.  Returns the steps taken; rn receives the
// explicit residual norms at the end.
template <typename Apply>
int cg_core(SolveWs* ws, int64_t n, int nr, double tol, int max_iter, const Apply& apply,
            const std::vector<double>& fn, std::vector<double>& rn, std::vector<int>& conv,
            int& cycles, hipStream_t s) {
  const int64_t nv = n * nr;
  double *r = ws->Q, *p = ws->Q + nv, *x = ws->x, *q = ws->w, *part = ws->part;
  double* pq = ws->hdev;
  double* rra = ws->hdev + nr;
  double* rrb = ws->hdev + 2 * nr;
  double* active = ws->scl;
  auto rel = [&](int c, double v) { return fn[c] > 0 ? v / fn[c] : 0.0; };
  std::vector<double> rr(nr), act(nr), rprev;
  // r = b - H x, rra = |r|^2 per column, rn = |r|
  auto residual = [&]() {
    apply(x, q);
    gmres_sub(ws->fd, q, nv, r, s);
    gmres_dots(r, 0, 1, r, n, nr, part, rra, s);
    HM_HIP(hipMemcpyAsync(rr.data(), rra, nr * sizeof(double), hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    rn.resize(nr);
    for (int c = 0; c < nr; ++c) rn[c] = std::sqrt(std::max(rr[c], 0.0));
    for (int c = 0; c < nr; ++c) conv[c] = rel(c, rn[c]) <= tol;
  };
  residual();
  int it = 0;
  while (true) {
    bool all = true;
    for (int c = 0; c < nr; ++c) all = all && conv[c];
    if (all || it >= max_iter) break;
    if (!rprev.empty()) {
      bool progress = false;
      for (int c = 0; c < nr; ++c)
        if (!conv[c] && rn[c] < 0.9 * rprev[c]) progress = true;
      if (!progress) break;
    }
    rprev = rn;
    for (int c = 0; c < nr; ++c) act[c] = conv[c] ? 0.0 : 1.0;
    HM_HIP(hipMemcpyAsync(active, act.data(), nr * sizeof(double), hipMemcpyHostToDevice, s));
    HM_HIP(hipMemcpyAsync(p, r, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
    while (it < max_iter) {
      apply(p, q);
      gmres_dots(p, 0, 1, q, n, nr, part, pq, s);
      cg_update(x, r, p, q, rra, pq, active, n, nr, s);
      gmres_dots(r, 0, 1, r, n, nr, part, rrb, s);
      HM_HIP(hipMemcpyAsync(rr.data(), rrb, nr * sizeof(double), hipMemcpyDeviceToHost, s));
      HM_HIP(hipStreamSynchronize(s));
      ++it;
      bool any = false, changed = false;
      for (int c = 0; c < nr; ++c) {
        if (act[c] == 0.0) continue;
        if (rel(c, std::sqrt(std::max(rr[c], 0.0))) <= tol || !(rr[c] > 0.0)) {
          act[c] = 0.0;
          changed = true;
        } else {
          any = true;
        }
      }
      if (!any) break;
      if (changed)
        HM_HIP(hipMemcpyAsync(active, act.data(), nr * sizeof(double), hipMemcpyHostToDevice, s));
      cg_dir(p, r, rrb, rra, active, n, nr, s);
      std::swap(rra, rrb);
    }
    ++cycles;
    residual();
  }
  return it;
}
}  // namespace

// ------------------------------------------------------------------ ABI
extern "C" {

const char* hm_last_error(void) { return g_err.c_str(); }

hm_status hm_params_default(hm_params* p) {
  if (!p) return arg_error("hm_params_default: NULL");
  std::memset(p, 0, sizeof(*p));
  p->leaf_size = 32;
  p->max_rank = 64;
  p->precision = HM_F64;
  p->flags = 0;
  p->eta = 1.0;
  p->aca_eps = 1e-6;
  p->mem_limit_bytes = 0;
  return HM_OK;
}

namespace {
hm_status check_params(const hm_params* p, const char* who) {
  const std::string w(who);
  if (p->leaf_size < 1 || p->leaf_size > kMaxLeaf) return arg_error(w + ": leaf_size must be in 1..64");
  if (p->max_rank < 0 || p->max_rank > kMaxRank) return arg_error(w + ": max_rank must be in 0..256");
  if (p->precision != HM_F64 && p->precision != HM_F32 && p->precision != HM_F32_F16)
    return arg_error(w + ": bad precision");
  if (!(p->eta >= 0.0) || !std::isfinite(p->eta)) return arg_error(w + ": eta must be finite and >= 0");
  if (!(p->aca_eps >= 0.0) || !std::isfinite(p->aca_eps))
    return arg_error(w + ": aca_eps must be finite and >= 0");
  if (p->mem_limit_bytes < 0) return arg_error(w + ": mem_limit_bytes < 0");
  if (p->flags & ~(HM_STRICT | HM_PROFILE | HM_AUTOTUNE | HM_GALERKIN))
    return arg_error(w + ": unknown flag");
  return HM_OK;
}

// Checks one geometry's vertices and triangles (indices local to it).
hm_status check_mesh(const double* vertices, int64_t nv, const int32_t* triangles, int64_t nt,
                     const std::string& w) {
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(vertices[i])) return arg_error(w + ": non-finite vertex coordinate");
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t a = triangles[3 * t], b = triangles[3 * t + 1], c = triangles[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
      return arg_error(w + ": triangle " + std::to_string(t) + " has a vertex index out of range");
    const double* A = vertices + 3 * (int64_t)a;
    const double* B = vertices + 3 * (int64_t)b;
    const double* C = vertices + 3 * (int64_t)c;
    const double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    const double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                          e1[0] * e2[1] - e1[1] * e2[0]};
    if (!(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2] > 0.0))
      return arg_error(w + ": triangle " + std::to_string(t) + " is degenerate");
  }
  return HM_OK;
}

// Builds a handle from validated, concatenated input; `tri` holds global
// vertex indices and goff the triangle offsets of the geometries.
hm_status build_handle(const double* vertices, int64_t n_vertices, const int32_t* tri,
                       std::vector<int64_t> goff, const hm_params* p, void* stream,
                       hm_handle** out) {
  return guarded([&]() -> hm_status {
    std::unique_ptr<hm_handle> h(new hm_handle());
    h->p = *p;
    if (h->p.max_rank == 0) h->p.max_rank = 64;
    h->n = goff.back();
    h->goff = std::move(goff);
    h->form = p->precision;
    h->f32 = (p->precision != HM_F64) ? 1 : 0;
    h->ts = h->f32 ? 4 : 8;
    h->op = (p->flags & HM_GALERKIN) ? kOpGalerkin : kOpColloc;
    HM_HIP(hipGetDevice(&h->device));
    if (p->flags & HM_PROFILE) {
      for (auto& e : h->prof.ev) HM_HIP(hipEventCreate(&e));
      h->profiling = true;
    }
    hipStream_t s = as_stream(stream);
    h->alloc_stream = s;
    if (h->form == HM_F32_F16)
      build_impl<float, _Float16>(h.get(), vertices, n_vertices, tri, s);
    else if (h->form == HM_F32)
      build_impl<float, float>(h.get(), vertices, n_vertices, tri, s);
    else
      build_impl<double, double>(h.get(), vertices, n_vertices, tri, s);
    *out = h.release();
    return HM_OK;
  });
}
}  // namespace

hm_status hm_build(const double* vertices, int64_t n_vertices, const int32_t* triangles,
                   int64_t n_triangles, const hm_params* p, void* stream, hm_handle** out) {
  if (!out) return arg_error("hm_build: out is NULL");
  *out = nullptr;
  if (!vertices || !triangles || !p) return arg_error("hm_build: NULL argument");
  if (n_triangles < 1 || n_triangles > (int64_t)INT32_MAX / 2)
    return arg_error("hm_build: n_triangles out of range");
  if (n_vertices < 3 || n_vertices > (int64_t)INT32_MAX) return arg_error("hm_build: n_vertices out of range");
  hm_status st = check_params(p, "hm_build");
  if (st != HM_OK) return st;
  st = check_mesh(vertices, n_vertices, triangles, n_triangles, "hm_build");
  if (st != HM_OK) return st;
  return build_handle(vertices, n_vertices, triangles, {0, n_triangles}, p, stream, out);
}

hm_status hm_build_batch(const double* vertices, const int64_t* vtx_offsets,
                         const int32_t* triangles, const int64_t* tri_offsets, int32_t n_geom,
                         const hm_params* p, void* stream, hm_handle** out) {
  if (!out) return arg_error("hm_build_batch: out is NULL");
  *out = nullptr;
  if (!vertices || !vtx_offsets || !triangles || !tri_offsets || !p)
    return arg_error("hm_build_batch: NULL argument");
  if (n_geom < 1 || n_geom > kMaxGeoms) return arg_error("hm_build_batch: n_geom must be in 1..65536");
  if (vtx_offsets[0] != 0 || tri_offsets[0] != 0)
    return arg_error("hm_build_batch: offsets must start at 0");
  for (int32_t g = 0; g < n_geom; ++g) {
    if (tri_offsets[g + 1] - tri_offsets[g] < 1)
      return arg_error("hm_build_batch: geometry " + std::to_string(g) + " has no triangle");
    if (vtx_offsets[g + 1] - vtx_offsets[g] < 3)
      return arg_error("hm_build_batch: geometry " + std::to_string(g) + " has fewer than 3 vertices");
  }
  const int64_t nt = tri_offsets[n_geom], nv = vtx_offsets[n_geom];
  if (nt > (int64_t)INT32_MAX / 2) return arg_error("hm_build_batch: too many triangles");
  if (nv > (int64_t)INT32_MAX) return arg_error("hm_build_batch: too many vertices");
  hm_status st = check_params(p, "hm_build_batch");
  if (st != HM_OK) return st;
  std::vector<int32_t> tri((size_t)3 * nt);
  for (int32_t g = 0; g < n_geom; ++g) {
    const int64_t t0 = tri_offsets[g], t1 = tri_offsets[g + 1], v0 = vtx_offsets[g];
    st = check_mesh(vertices + 3 * v0, vtx_offsets[g + 1] - v0, triangles + 3 * t0, t1 - t0,
                    "hm_build_batch: geometry " + std::to_string(g));
    if (st != HM_OK) return st;
    for (int64_t e = 3 * t0; e < 3 * t1; ++e) tri[e] = (int32_t)(triangles[e] + v0);
  }
  return build_handle(vertices, nv, tri.data(),
                      std::vector<int64_t>(tri_offsets, tri_offsets + n_geom + 1), p, stream, out);
}

static hm_status matvec_common(hm_handle* h, const void* x, void* y, int64_t n_rows, int32_t nrhs,
                               int32_t dtype, void* stream, bool transposed) {
  const char* who = transposed ? "hm_matvec_T" : "hm_matvec";
  if (!h) return arg_error(std::string(who) + ": NULL handle");
  if (!x || !y) return arg_error(std::string(who) + ": NULL vector");
  if (n_rows != h->n)
    return arg_error(std::string(who) + ": vectors have " + std::to_string(n_rows) +
                     " rows, the handle " + std::to_string(h->n));
  if (nrhs < 1) return arg_error(std::string(who) + ": nrhs must be >= 1");
  if (dtype != HM_F64 && dtype != HM_F32) return arg_error(std::string(who) + ": bad dtype");
  const size_t vb = (size_t)h->n * nrhs * (dtype == HM_F32 ? 4 : 8);
  const char* xb = (const char*)x;
  const char* yb = (const char*)y;
  if (xb < yb + vb && yb < xb + vb) return arg_error(std::string(who) + ": x and y overlap");
  return guarded([&]() -> hm_status {
    matvec_dispatch(h->plan(), h->form, x, y, nrhs, dtype == HM_F32 ? 1 : 0, transposed,
                    as_stream(stream));
    return HM_OK;
  });
}

hm_status hm_matvec(hm_handle* h, const void* x, void* y, int64_t n, int32_t nrhs, int32_t dtype,
                    void* stream) {
  return matvec_common(h, x, y, n, nrhs, dtype, stream, false);
}

hm_status hm_matvec_T(hm_handle* h, const void* x, void* y, int64_t n, int32_t nrhs, int32_t dtype,
                      void* stream) {
  return matvec_common(h, x, y, n, nrhs, dtype, stream, true);
}

// ------------------------------------------------------------------ GMRES
// Workspace of hm_solve_noalloc: a file-scope device array, one copy per GPU
// for the life of the process.  Host code uses only the address that
// hipGetSymbolAddress returns for it on each device, never the array's name.
constexpr size_t kScratchBytes = HM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

// Device address of `scratch` on the current device, taken once per device.
static double* scratch_address() {
  static std::mutex mu;
  static std::vector<double*> addr;
  int dev = 0;
  HM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      throw Error{HM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                  hipGetErrorString(e)};
    addr[dev] = static_cast<double*>(ptr);
  }
  return addr[dev];
}

// Doubles the solve workspace takes, every buffer rounded up to 256 bytes.
static size_t solve_ws_doubles(int64_t n, int nr, int m, bool refine) {
  size_t tot = 0;
  SolveWs probe;
  probe.layout(n, nr, m, false, refine, [&](size_t cnt) {
    tot += (cnt + 31) & ~(size_t)31;
    return (double*)nullptr;
  });
  return tot;
}

// fixed_ws: null => the workspace comes from the library's pool; else the
// solve runs in that device buffer of fixed_doubles doubles and allocates
// nothing (no graph replay in that mode).
static hm_status solve_common(hm_handle* h, const void* f, void* sigma, int64_t n_rows,
                              int32_t nrhs, int32_t dtype, const hm_solve_params* sp,
                              hm_solve_info* info, void* stream, bool no_alloc) {
  const std::string who = no_alloc ? "hm_solve_noalloc" : "hm_solve";
  if (!h) return arg_error(who + ": NULL handle");
  if (!f || !sigma || !sp) return arg_error(who + ": NULL argument");
  if (n_rows != h->n)
    return arg_error(who + ": vectors have " + std::to_string(n_rows) + " rows, the handle " +
                     std::to_string(h->n));
  if (nrhs < 1 || nrhs > 256) return arg_error(who + ": nrhs must be in 1..256");
  if (dtype != HM_F64 && dtype != HM_F32) return arg_error(who + ": bad dtype");
  if (!(sp->tol > 0.0) || !std::isfinite(sp->tol)) return arg_error(who + ": tol must be > 0");
  if (sp->restart < 0 || sp->restart > 1000) return arg_error(who + ": restart must be in 0..1000");
  if (sp->max_iter < 1) return arg_error(who + ": max_iter must be >= 1");
  if (sp->refine != 0 && sp->refine != 1) return arg_error(who + ": refine must be 0 or 1");
  if (sp->refine && (!(sp->inner_tol >= 0.0) || !(sp->inner_tol < 1.0)))
    return arg_error(who + ": inner_tol must be in [0, 1)");
  if (sp->flags & ~(HM_SOLVE_GRAPH | HM_SOLVE_CG)) return arg_error(who + ": unknown flag");
  const bool cg = (sp->flags & HM_SOLVE_CG) != 0;
  if (cg && (sp->flags & HM_SOLVE_GRAPH))
    return arg_error(who + ": HM_SOLVE_CG does not combine with HM_SOLVE_GRAPH");
  if (cg && sp->refine) return arg_error(who + ": HM_SOLVE_CG does not combine with refine");
  if (cg && sp->transpose) return arg_error(who + ": HM_SOLVE_CG does not combine with transpose");
  if (no_alloc) {
    if (sp->flags & HM_SOLVE_GRAPH)
      return arg_error(who + ": HM_SOLVE_GRAPH is not available without allocation");
    const int mm = cg ? 1 : (sp->restart > 0 ? sp->restart : 100);
    const size_t need = solve_ws_doubles(h->n, nrhs, mm, sp->refine != 0) * sizeof(double);
    if (need > kScratchBytes)
      return arg_error(who + ": the workspace needs " + std::to_string(need) +
                       " bytes, more than the fixed " + std::to_string(kScratchBytes) +
                       " (reduce n * nrhs * (restart + 7))");
  }
  {
    const size_t vb = (size_t)h->n * nrhs * (dtype == HM_F32 ? 4 : 8);
    const char* fb = (const char*)f;
    const char* sb = (const char*)sigma;
    if (fb < sb + vb && sb < fb + vb) return arg_error(who + ": f and sigma overlap");
  }
  return guarded([&]() -> hm_status {
    hipStream_t s = as_stream(stream);
    const int64_t n = h->n;
    const int nr = nrhs;
    const int64_t nv = n * nr;
    // CG keeps r and p where GMRES keeps its basis (two vectors)
    const int m = cg ? 1 : (sp->restart > 0 ? sp->restart : 100);
    const bool tr = sp->transpose != 0;
    const bool refine = sp->refine != 0;
    const double inner_tol = refine ? (sp->inner_tol > 0.0 ? sp->inner_tol : 1e-4) : 0.0;
    const MvPlan P = h->plan();
    // device workspace: per call, or kept with the handle for graph replays
    const bool use_graph = (sp->flags & HM_SOLVE_GRAPH) != 0;
    std::unique_ptr<SolveWs> local;
    SolveWs* ws = nullptr;
    if (no_alloc) {
      // bump allocation in the device's fixed array (size checked above)
      double* base = scratch_address();
      size_t used = 0;
      local.reset(new SolveWs());
      local->free_stream = s;
      local->layout(n, nr, m, tr, refine, [&](size_t cnt) {
        double* q = base + used;
        used += (cnt + 31) & ~(size_t)31;
        return q;
      });
      ws = local.get();
    } else if (use_graph) {
      if (!h->sws || h->sws->nr != nr || h->sws->m != m || h->sws->tr != tr ||
          h->sws->f32 != refine) {
        if (h->sws) h->sws->free_stream = s;
        h->sws.reset(new SolveWs());
        h->sws->alloc(n, nr, m, tr, refine, s);
      }
      ws = h->sws.get();
    } else {
      local.reset(new SolveWs());
      local->free_stream = s;
      local->alloc(n, nr, m, tr, refine, s);
      ws = local.get();
    }
    // op(H) v with double vectors and double accumulation (the plain solve
    // and the refinement residual) ...
    auto apply64 = [&](const double* in, double* out) {
      matvec_dispatch(P, h->form, in, out, nr, 0, tr, s);
    };
    // ... and with float vectors (the inner solve of the refinement): the
    // basis vector is rounded to float, the product accumulates in float for
    // the single-precision forms, the result is widened back to double
    auto apply32 = [&](const double* in, double* out) {
      convert_f64_to_f32(in, nv, ws->xf, s);
      matvec_dispatch(P, h->form, ws->xf, ws->wf, nr, 1, tr, s);
      convert_f32_to_f64(ws->wf, nv, out, s);
    };
    const int mhd = m + 2;
    if (use_graph && !ws->exec) {
      // capture one Arnoldi step on a private stream (the caller's may be the
      // null stream, which cannot capture); no profiling events inside
      MvPlan Pg = P;
      Pg.prof = nullptr;
      hipStream_t cs = nullptr;
      HM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      struct StreamGuard {
        hipStream_t st;
        ~StreamGuard() { (void)hipStreamDestroy(st); }
      } sgd{cs};
      HM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
      if (refine) {
        gmres_copy_col_f32(ws->Q, nv, ws->jd, ws->xf, cs);
        matvec_dispatch(Pg, h->form, ws->xf, ws->wf, nr, 1, tr, cs);
        convert_f32_to_f64(ws->wf, nv, ws->w, cs);
      } else {
        gmres_copy_col(ws->Q, nv, ws->jd, ws->xin, cs);
        matvec_dispatch(Pg, h->form, ws->xin, ws->w, nr, 0, tr, cs);
      }
      for (int pass = 0; pass < 2; ++pass) {
        double* hp = ws->hdev + (size_t)pass * mhd * nr;
        gmres_dots_dev(ws->Q, nv, ws->jd, m + 1, ws->w, n, nr, ws->part, hp, cs);
        gmres_orth_update_dev(ws->Q, nv, hp, ws->jd, n, nr, ws->w, cs);
      }
      gmres_dots(ws->w, 0, 1, ws->w, n, nr, ws->part, ws->hdev + (size_t)mhd * nr * 2, cs);
      HM_HIP(hipStreamEndCapture(cs, &ws->graph));
      HM_HIP(hipGraphInstantiate(&ws->exec, ws->graph, nullptr, nullptr, 0));
    }
    auto graph_step = [&](int j) {
      const int jh = j;
      HM_HIP(hipMemcpyAsync(ws->jd, &jh, sizeof(int), hipMemcpyHostToDevice, s));
      HM_HIP(hipGraphLaunch(ws->exec, s));
    };
    auto norms = [&](const double* v, std::vector<double>& out) {
      gmres_dots(v, 0, 1, v, n, nr, ws->part, ws->hdev, s);
      out.resize(nr);
      HM_HIP(hipMemcpyAsync(out.data(), ws->hdev, nr * sizeof(double), hipMemcpyDeviceToHost, s));
      HM_HIP(hipStreamSynchronize(s));
      for (auto& z : out) z = std::sqrt(std::max(z, 0.0));
    };

    // the right-hand side in double (fo when refining, else fd directly)
    double* fsrc = refine ? ws->fo : ws->fd;
    double* xsol = refine ? ws->xs : ws->x;
    if (dtype == HM_F32) {
      convert_f32_to_f64((const float*)f, nv, fsrc, s);
      if (sp->use_x0) convert_f32_to_f64((const float*)sigma, nv, xsol, s);
    } else {
      HM_HIP(hipMemcpyAsync(fsrc, f, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
      if (sp->use_x0)
        HM_HIP(hipMemcpyAsync(xsol, sigma, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    if (!sp->use_x0) HM_HIP(hipMemsetAsync(xsol, 0, nv * sizeof(double), s));

    std::vector<double> fn, rn;
    std::vector<int> conv(nr, 0);
    norms(fsrc, fn);
    auto rel = [&](int c, double r) { return fn[c] > 0 ? r / fn[c] : 0.0; };
    int total_it = 0, restarts = 0, ir_steps = 0;
    if (cg) {
      total_it = cg_core(ws, n, nr, sp->tol, sp->max_iter, apply64, fn, rn, conv, restarts, s);
    } else if (!refine) {
      total_it = gmres_core(ws, n, nr, m, sp->tol, sp->max_iter, use_graph, apply64, graph_step,
                            fn, rn, conv, restarts, false, s);
    } else {
      // iterative refinement: the residual of the current solution in double
      // (vectors and accumulation), the correction from GMRES with float
      // products to the relative tolerance inner_tol, added in double
      std::vector<double> rprev, rin, zero_fn;
      std::vector<int> cin;
      std::vector<double> keep(nr);
      while (true) {
        apply64(xsol, ws->w);
        gmres_sub(ws->fo, ws->w, nv, ws->fd, s);    // r = f - H sigma  (the inner right-hand side)
        norms(ws->fd, rn);
        for (int c = 0; c < nr; ++c) conv[c] = rel(c, rn[c]) <= sp->tol;
        bool all = true;
        for (int c = 0; c < nr; ++c) all = all && conv[c];
        if (all || total_it >= sp->max_iter) break;
        // stagnation: no column's residual fell below 90% of the previous one
        if (!rprev.empty()) {
          bool progress = false;
          for (int c = 0; c < nr; ++c)
            if (!conv[c] && rn[c] < 0.9 * rprev[c]) progress = true;
          if (!progress) break;
        }
        rprev = rn;
        // converged columns take no part in the correction (zero right-hand side)
        for (int c = 0; c < nr; ++c) keep[c] = conv[c] ? 0.0 : 1.0;
        HM_HIP(hipMemcpyAsync(ws->scl, keep.data(), nr * sizeof(double), hipMemcpyHostToDevice, s));
        gmres_scale_cols(ws->fd, ws->scl, n, nr, ws->fd, s);
        HM_HIP(hipMemsetAsync(ws->x, 0, nv * sizeof(double), s));
        std::vector<double> fin(nr);
        for (int c = 0; c < nr; ++c) fin[c] = conv[c] ? 0.0 : rn[c];
        total_it += gmres_core(ws, n, nr, m, inner_tol, sp->max_iter - total_it, use_graph, apply32,
                               graph_step, fin, rin, cin, restarts, true, s);
        gmres_add(xsol, ws->x, nv, xsol, s);
        ++ir_steps;
      }
    }
    // result
    if (dtype == HM_F32)
      convert_f64_to_f32(xsol, nv, (float*)sigma, s);
    else
      HM_HIP(hipMemcpyAsync(sigma, xsol, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
    HM_HIP(hipStreamSynchronize(s));
    int nconv = 0;
    double worst = 0.0;
    for (int c = 0; c < nr; ++c) {
      nconv += conv[c];
      worst = std::max(worst, rel(c, rn[c]));
    }
    if (info) {
      info->iters = total_it;
      info->restarts = restarts;
      info->converged = nconv;
      info->ir_steps = ir_steps;
      info->rel_residual = worst;
    }
    return nconv == nr ? HM_OK : HM_NOT_CONVERGED;
  });
}

hm_status hm_solve(hm_handle* h, const void* f, void* sigma, int64_t n, int32_t nrhs,
                   int32_t dtype, const hm_solve_params* sp, hm_solve_info* info, void* stream) {
  return solve_common(h, f, sigma, n, nrhs, dtype, sp, info, stream, false);
}

hm_status hm_solve_noalloc(hm_handle* h, const void* f, void* sigma, int64_t n, int32_t nrhs,
                           int32_t dtype, const hm_solve_params* sp, hm_solve_info* info,
                           void* stream) {
  return solve_common(h, f, sigma, n, nrhs, dtype, sp, info, stream, true);
}

void hm_free(hm_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  delete h;
}

hm_status hm_release_memory(void) {
  return guarded([&]() -> hm_status {
    HM_HIP(hipDeviceSynchronize());
    cache_release();
    trim_pool();
    return HM_OK;
  });
}

hm_status hm_query(hm_handle* h, int32_t what, void* dst, int64_t dst_bytes, int64_t* needed) {
  if (!h) return arg_error("hm_query: NULL handle");
  return guarded([&]() -> hm_status {
    HM_HIP(hipDeviceSynchronize());
    int64_t need = 0;
    auto check = [&](int64_t b) -> bool {
      need = b;
      if (needed) *needed = b;
      return dst && dst_bytes >= b;
    };
    auto copy_dev = [&](const void* src, int64_t b) -> hm_status {
      if (!check(b)) return arg_error("hm_query: destination too small");
      if (b) HM_HIP(hipMemcpy(dst, src, b, hipMemcpyDeviceToHost));
      return HM_OK;
    };
    switch (what) {
      case HM_Q_STATS:
        if (!check(sizeof(hm_stats))) return arg_error("hm_query: destination too small");
        std::memcpy(dst, &h->st, sizeof(hm_stats));
        return HM_OK;
      case HM_Q_MORTON: return copy_dev(h->keys, h->n * 8);
      case HM_Q_PERM: return copy_dev(h->perm, h->n * 4);
      case HM_Q_CLUSTERS: return copy_dev(h->cl, h->ncl * 16);
      case HM_Q_BOXES: return copy_dev(h->box, h->ncl * 48);
      case HM_Q_KERNEL_TIMES: {
        if (!h->profiling) return arg_error("hm_query: build without HM_PROFILE");
        if (!check(8 * 2 * HM_NKERNEL)) return arg_error("hm_query: destination too small");
        double* o = (double*)dst;
        for (int k = 0; k < HM_NKERNEL; ++k) {
          o[k] = h->prof.ms[k];
          o[HM_NKERNEL + k] = h->prof.launches[k];
          h->prof.ms[k] = 0;
          h->prof.launches[k] = 0;
        }
        return HM_OK;
      }
      case HM_Q_TUNE: {
        const int64_t b = (int64_t)h->tune.size() * 16;
        if (!check(b)) return arg_error("hm_query: destination too small");
        double* o = (double*)dst;
        for (size_t k = 0; k < h->tune.size(); ++k) {
          o[2 * k] = h->tune[k][0];
          o[2 * k + 1] = h->tune[k][1];
        }
        return HM_OK;
      }
      case HM_Q_ACA_BINS: {
        if (!check(kAcaBins * 8)) return arg_error("hm_query: destination too small");
        int32_t* o = (int32_t*)dst;
        for (int k = 0; k < kAcaBins; ++k) {
          o[2 * k] = kAcaBinEdge[k];
          o[2 * k + 1] = h->sto.bins.cls[k];
        }
        return HM_OK;
      }
      case HM_Q_ACA_TUNE: {
        const int64_t b = (int64_t)h->sto.aca_tune.size() * 32;
        if (!check(b)) return arg_error("hm_query: destination too small");
        double* o = (double*)dst;
        for (size_t k = 0; k < h->sto.aca_tune.size(); ++k) {
          const AcaTuneRow& r = h->sto.aca_tune[k];
          o[4 * k] = r.bin;
          o[4 * k + 1] = r.cls;
          o[4 * k + 2] = (double)r.blocks;
          o[4 * k + 3] = r.ms;
        }
        return HM_OK;
      }
      case HM_Q_TIMINGS:
        if (!check(sizeof(h->ms))) return arg_error("hm_query: destination too small");
        std::memcpy(dst, h->ms, sizeof(h->ms));
        return HM_OK;
      case HM_Q_LEAVES: {
        if (!check(h->nleaf * 12)) return arg_error("hm_query: destination too small");
        std::vector<int32_t> lo(h->nleaf), m(h->nleaf);
        std::vector<int64_t> ld(h->nleaf + 1);
        HM_HIP(hipMemcpy(lo.data(), h->leaf_lo, h->nleaf * 4, hipMemcpyDeviceToHost));
        HM_HIP(hipMemcpy(m.data(), h->leaf_m, h->nleaf * 4, hipMemcpyDeviceToHost));
        HM_HIP(hipMemcpy(ld.data(), h->ldpre, (h->nleaf + 1) * 8, hipMemcpyDeviceToHost));
        int32_t* o = (int32_t*)dst;
        for (int64_t k = 0; k < h->nleaf; ++k) {
          o[3 * k] = lo[k];
          o[3 * k + 1] = m[k];
          o[3 * k + 2] = (int32_t)(ld[k + 1] - ld[k]);
        }
        return HM_OK;
      }
      case HM_Q_DENSE_BLOCKS:
      case HM_Q_LR_BLOCKS: {
        const bool dense = what == HM_Q_DENSE_BLOCKS;
        const int64_t cnt = dense ? h->nd : h->nl;
        if (!check(cnt * 48)) return arg_error("hm_query: destination too small");
        std::vector<int2> bl(cnt);
        std::vector<Cluster> clh(h->ncl);
        std::vector<int32_t> rk(dense ? 0 : cnt), inf(dense ? 0 : cnt);
        if (cnt)
          HM_HIP(hipMemcpy(bl.data(), dense ? h->dns : h->lr, cnt * 8, hipMemcpyDeviceToHost));
        HM_HIP(hipMemcpy(clh.data(), h->cl, h->ncl * 16, hipMemcpyDeviceToHost));
        if (!dense && cnt) {
          HM_HIP(hipMemcpy(rk.data(), h->sto.rank, cnt * 4, hipMemcpyDeviceToHost));
          HM_HIP(hipMemcpy(inf.data(), h->sto.info, cnt * 4, hipMemcpyDeviceToHost));
        }
        int64_t* o = (int64_t*)dst;
        for (int64_t b = 0; b < cnt; ++b) {
          const Cluster t = clh[bl[b].x], sg = clh[bl[b].y];
          o[6 * b] = t.x;
          o[6 * b + 1] = t.y;
          o[6 * b + 2] = sg.x;
          o[6 * b + 3] = sg.y;
          o[6 * b + 4] = dense ? 0 : rk[b];
          o[6 * b + 5] = dense ? 0 : (inf[b] & 1);
        }
        return HM_OK;
      }
      case HM_Q_LR_FACTORS: {
        if (!dst || dst_bytes < 8) return arg_error("hm_query: block index expected in dst");
        const int64_t b = *(const int64_t*)dst;
        if (b < 0 || b >= h->nl) return arg_error("hm_query: block index out of range");
        int2 ts;
        HM_HIP(hipMemcpy(&ts, h->lr + b, 8, hipMemcpyDeviceToHost));
        Cluster t, sg;
        HM_HIP(hipMemcpy(&t, h->cl + ts.x, 16, hipMemcpyDeviceToHost));
        HM_HIP(hipMemcpy(&sg, h->cl + ts.y, 16, hipMemcpyDeviceToHost));
        int32_t r = 0;
        HM_HIP(hipMemcpy(&r, h->sto.rank + b, 4, hipMemcpyDeviceToHost));
        const int64_t total = (int64_t)r * ((t.y - t.x) + (sg.y - sg.x));
        if (!check(total * (int64_t)h->ts)) return arg_error("hm_query: destination too small");
        if (total == 0) return HM_OK;
        void* buf = nullptr;
        HM_HIP(hipMalloc(&buf, total * h->ts));
        if (h->form == HM_F32_F16)
          launch_unpack<_Float16, float>(h->lr, b, h->cl, h->leaf_lo, h->leaf_m, h->ldpre,
                                         h->cl_leaves, h->sto.meta, h->sto.uptr, h->sto.su,
                                         (float*)buf, total, 0);
        else if (h->form == HM_F32)
          launch_unpack<float, float>(h->lr, b, h->cl, h->leaf_lo, h->leaf_m, h->ldpre,
                                      h->cl_leaves, h->sto.meta, h->sto.uptr, nullptr,
                                      (float*)buf, total, 0);
        else
          launch_unpack<double, double>(h->lr, b, h->cl, h->leaf_lo, h->leaf_m, h->ldpre,
                                        h->cl_leaves, h->sto.meta, h->sto.uptr, nullptr,
                                        (double*)buf, total, 0);
        HM_HIP(hipMemcpy(dst, buf, total * h->ts, hipMemcpyDeviceToHost));
        HM_HIP(hipFree(buf));
        return HM_OK;
      }
      case HM_Q_DENSE_ENTRIES: {
        if (!dst || dst_bytes < 8) return arg_error("hm_query: block index expected in dst");
        const int64_t b = *(const int64_t*)dst;
        if (b < 0 || b >= h->nd) return arg_error("hm_query: block index out of range");
        int2 ts;
        HM_HIP(hipMemcpy(&ts, h->dns + b, 8, hipMemcpyDeviceToHost));
        Cluster t, sg;
        HM_HIP(hipMemcpy(&t, h->cl + ts.x, 16, hipMemcpyDeviceToHost));
        HM_HIP(hipMemcpy(&sg, h->cl + ts.y, 16, hipMemcpyDeviceToHost));
        int2 lt;
        HM_HIP(hipMemcpy(&lt, h->cl_leaves + ts.x, 8, hipMemcpyDeviceToHost));
        const int64_t m = t.y - t.x, nc = sg.y - sg.x;
        if (!check(m * nc * 8)) return arg_error("hm_query: destination too small");
        // the block's row slices, one per leaf of its row cluster: ld x nc,
        // column-major, in the dense storage type
        int64_t q0 = 0;
        HM_HIP(hipMemcpy(&q0, h->sto.dub + b, 8, hipMemcpyDeviceToHost));
        const int nlf = lt.y - lt.x + 1;
        std::vector<uint64_t> addr(nlf);
        std::vector<int32_t> llo(nlf), lm(nlf);
        std::vector<int64_t> ld(nlf + 1);
        HM_HIP(hipMemcpy(addr.data(), h->sto.dptr + q0, nlf * 8, hipMemcpyDeviceToHost));
        HM_HIP(hipMemcpy(llo.data(), h->leaf_lo + lt.x, nlf * 4, hipMemcpyDeviceToHost));
        HM_HIP(hipMemcpy(lm.data(), h->leaf_m + lt.x, nlf * 4, hipMemcpyDeviceToHost));
        HM_HIP(hipMemcpy(ld.data(), h->ldpre + lt.x, (nlf + 1) * 8, hipMemcpyDeviceToHost));
        const size_t es = h->f32 ? 4 : 8;
        double* o = (double*)dst;
        for (int k = 0; k < nlf; ++k) {
          const int64_t ldk = ld[k + 1] - ld[k];
          std::vector<char> buf((size_t)ldk * nc * es);
          HM_HIP(hipMemcpy(buf.data(), (const void*)(uintptr_t)addr[k], buf.size(),
                           hipMemcpyDeviceToHost));
          for (int64_t j = 0; j < nc; ++j)
            for (int i = 0; i < lm[k]; ++i) {
              const int64_t e = j * ldk + i;
              const double v = es == 4 ? (double)((const float*)buf.data())[e]
                                       : ((const double*)buf.data())[e];
              o[(int64_t)(llo[k] - t.x + i) * nc + j] = v;
            }
        }
        return HM_OK;
      }
      default:
        return arg_error("hm_query: unknown query kind");
    }
    (void)need;
  });
}

hm_status hm_entries(hm_handle* h, const int32_t* rows, const int32_t* cols, int64_t count,
                     double* out) {
  if (!h) return arg_error("hm_entries: NULL handle");
  if (count < 0 || (count > 0 && (!rows || !cols || !out))) return arg_error("hm_entries: bad arguments");
  for (int64_t k = 0; k < count; ++k)
    if (rows[k] < 0 || rows[k] >= h->n || cols[k] < 0 || cols[k] >= h->n)
      return arg_error("hm_entries: index out of range");
  if (count == 0) return HM_OK;
  return guarded([&]() -> hm_status {
    hipStream_t s = 0;
    int32_t* dr = dalloc_t<int32_t>(count, s);
    int32_t* dc = dalloc_t<int32_t>(count, s);
    double* dout = dalloc_t<double>(count, s);
    HM_HIP(hipMemcpyAsync(dr, rows, count * 4, hipMemcpyHostToDevice, s));
    HM_HIP(hipMemcpyAsync(dc, cols, count * 4, hipMemcpyHostToDevice, s));
    if (h->f32) {
      Geom<float> g{h->c, (const float*)h->o, (const float*)h->aw, (const float*)h->sf, h->n,
                    h->tv, h->vid};
      launch_entries<float>(g, h->op, h->inv, dr, dc, count, dout, s);
    } else {
      Geom<double> g{h->c, (const double*)h->o, (const double*)h->aw, (const double*)h->sf, h->n,
                     h->tv, h->vid};
      launch_entries<double>(g, h->op, h->inv, dr, dc, count, dout, s);
    }
    HM_HIP(hipMemcpyAsync(out, dout, count * 8, hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    dfree(dr, s);
    dfree(dc, s);
    dfree(dout, s);
    HM_HIP(hipStreamSynchronize(s));
    return HM_OK;
  });
}

}  // extern "C"
