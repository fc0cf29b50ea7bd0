/*
 * hm.h -- C ABI of the MI355X (gfx950) H-matrix library for the Laplace
 * single-layer boundary integral equation.
 *
 * The library implements the method of Harbrecht & Zaspel, "A scalable
 * H-matrix approach for the solution of boundary integral equations on
 * multi-GPU clusters" (arXiv 1806.11558), for one GPU:
 *
 *   operator   S u(x) = int_Gamma u(y) / (4 pi |x - y|) dsigma_y = f(x)
 *              (Sec. 2.1, Example 1), discretised by collocation with one
 *              piecewise-constant unknown per flat triangle, collocation
 *              point = centroid (nodes at element centres, Sec. 4.1):
 *              a_ij = int_{T_j} G(x_i, y) dsigma_y, seven-point Radon rule
 *              for i != j, closed form for i == j;
 *   clustering Morton codes + sort, cardinality-based binary cluster tree
 *              (Sec. 2.3 (C1)-(C4); Sec. 3.1 "Spatial data structure");
 *   partition  block cluster tree of Algorithm 1 under the admissibility
 *              condition (Sec. 2.3, eq. admissibilityCondition), built
 *              level by level with scans (Sec. 3.1, "Block cluster tree
 *              traversal");
 *   setup      dense near-field blocks assembled in batches (Sec. 3.3) and
 *              adaptive cross approximation U V^T of every admissible block
 *              (Sec. 2.3), batched (Sec. 3.1, "Batching");
 *   apply      H-matrix-vector product (Sec. 2.3, last paragraph) and its
 *              transpose, used inside restarted GMRES.
 *
 * Conventions shared by every call
 *   - All functions are extern "C" and return hm_status (hm_free excepted).
 *   - Arguments are validated on the host before any HIP call; invalid
 *     arguments return HM_ERR_ARG and leave outputs untouched.
 *   - Unknowns are the triangles in the caller's order ("application
 *     order"); every vector crossing the ABI is in that order.
 *   - Device vectors are [n, nrhs] row-major (rhs index fastest), owned by
 *     the caller, of dtype HM_F64 (double) or HM_F32 (float).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work of a call is issued on that stream.  A handle is not
 *     safe for concurrent calls (it owns workspace); use one stream per
 *     handle.
 *   - hm_last_error() returns a thread-local message for the last failure.
 */
#ifndef HM_H
#define HM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hm_handle hm_handle;

typedef enum {
  HM_OK = 0,
  HM_NOT_CONVERGED = 1,   /* completed; iterative solve missed its tolerance */
  HM_ERR_ARG = -1,        /* invalid argument (checked before any HIP call)  */
  HM_ERR_OOM = -2,        /* device allocation failed or mem_limit exceeded  */
  HM_ERR_HIP = -3,        /* a HIP runtime call failed                       */
  HM_ERR_ACA = -4,        /* HM_STRICT and a block hit the rank cap          */
  HM_ERR_STATE = -5       /* handle in an unusable state                     */
} hm_status;

/* Arithmetic form of the build: kernel evaluation, ACA and storage. */
typedef enum {
  HM_F64 = 0,             /* everything in double                            */
  HM_F32 = 1,             /* evaluation, ACA and storage in float; the
                             geometry (centroids) and the pairwise centroid
                             difference stay double                         */
  HM_F32_F16 = 2          /* as HM_F32, but the low-rank factors are stored
                             in FP16: V as is (|v| <= 1 by the pivot
                             normalisation), every column of U divided by an
                             FP32 max-abs scale; products accumulate in float
                             (or double for double vectors).  Dense blocks
                             stay FP32                                       */
} hm_precision;

/* flags */
#define HM_STRICT 1       /* a block that reaches max_rank without meeting
                             the ACA stopping test fails the build           */
#define HM_PROFILE 2      /* products record HIP events around each kernel on
                             the caller's stream and synchronise it at the
                             end of the call; totals via HM_Q_KERNEL_TIMES   */
#define HM_AUTOTUNE 4     /* the build picks two schedules by measurement:
                             the ACA kernel class of every block size bin
                             (each candidate class timed on a sample of the
                             bin's blocks at the first-pass rank cap; via
                             HM_Q_ACA_BINS / HM_Q_ACA_TUNE), and the
                             column-unit width of the product (512 .. 8192,
                             timed on the handle's own storage; via
                             HM_Q_TUNE).  A tuned binning may change the ACA
                             kernel of some blocks and with it the rounding
                             of their factors (within the ACA tolerance), so
                             two tuned builds need not agree bitwise       */
#define HM_GALERKIN 8     /* the Galerkin matrix of Sec. 2.2 (eq.
                             linearSystem) with piecewise constants instead
                             of collocation at the centroids:
                             a_ij = int_Ti int_Tj 1/(4 pi |x - y|), Radon's
                             seven-point rule on both triangles for pairs
                             that share no vertex; for identical triangles
                             and triangles that share an edge or a vertex
                             (Sec. 4.1: higher-order quadrature and the
                             Duffy trick) a 12 x 12 Gauss rule on T_i in
                             collapsed coordinates with the inner integral
                             over T_j in closed form, in double.  The right
                             side is f_i = int_Ti f; the matrix is symmetric
                             up to quadrature error, so HM_SOLVE_CG applies.
                             Needs the vertex indices to be shared between
                             neighbouring triangles (a conforming mesh)   */

typedef struct {
  int32_t leaf_size;        /* C_leaf of (C3); 1..64.  Paper: 32             */
  int32_t max_rank;         /* ACA rank cap k_max; 1..256; 0 => 64.  The cap
                               is also limited by min(m, n) of each block     */
  int32_t precision;        /* hm_precision                                   */
  int32_t flags;            /* HM_STRICT | HM_PROFILE | HM_AUTOTUNE |
                               HM_GALERKIN                                    */
  double eta;               /* admissibility parameter eta >= 0.  Paper: 1.0 */
  double aca_eps;           /* relative Frobenius stopping tolerance of ACA;
                               0 => fixed-rank mode (every block gets
                               min(max_rank, m, n) terms, as the paper's k)  */
  int64_t mem_limit_bytes;  /* 0 => no limit; a build whose device footprint
                               would exceed it fails with HM_ERR_OOM         */
} hm_params;

/* Fill *p with the defaults: leaf 32, max_rank 64, HM_F64, eta 1, eps 1e-6. */
hm_status hm_params_default(hm_params* p);

/*
 * hm_build -- set up the H-matrix of the collocation operator (or, with
 * HM_GALERKIN, of the Galerkin matrix) of one mesh (Sec. 2.3 and Sec. 3;
 * Algorithm 1).
 *   vertices   host, double[n_vertices][3]
 *   triangles  host, int32[n_triangles][3], vertex indices in [0, n_vertices);
 *              every triangle must have positive area
 *   p          host, build parameters (copied)
 *   stream     hipStream_t
 *   out        receives the new handle (owned by the caller, release with
 *              hm_free); set to NULL on failure
 * The host arrays are copied before return and may be freed afterwards.  The
 * call returns when the handle is ready (it synchronises `stream`).
 * Errors: HM_ERR_ARG (NULL pointers, n_triangles < 1, bad index, degenerate
 * triangle, bad parameter), HM_ERR_OOM, HM_ERR_HIP, HM_ERR_ACA (HM_STRICT).
 */
hm_status hm_build(const double* vertices, int64_t n_vertices,
                   const int32_t* triangles, int64_t n_triangles,
                   const hm_params* p, void* stream, hm_handle** out);

/*
 * hm_build_batch -- one handle for several independent meshes, set up in the
 * same batched launches (the batching of Sec. 3.3 carried over many surfaces
 * at once).  Every geometry gets its own Morton box, cluster tree and block
 * partition (Algorithm 1 starts from each geometry's root pair); geometries
 * do not interact, so the operator is block diagonal over them and a product
 * or solve treats all of them together.
 *   vertices     host, double[vtx_offsets[n_geom]][3], all geometries
 *                concatenated
 *   vtx_offsets  host, int64[n_geom + 1], starts at 0, at least 3 vertices
 *                per geometry
 *   triangles    host, int32[tri_offsets[n_geom]][3]; the indices of
 *                geometry g are local to its vertex range
 *   tri_offsets  host, int64[n_geom + 1], starts at 0, at least 1 triangle
 *                per geometry
 *   n_geom       1..65536
 * Unknowns are the triangles in concatenated order (N = tri_offsets[n_geom]);
 * products and solves take vectors of that length.  Other arguments,
 * ownership and errors as hm_build; n_geom = 1 builds the same handle.
 */
hm_status hm_build_batch(const double* vertices, const int64_t* vtx_offsets,
                         const int32_t* triangles, const int64_t* tri_offsets, int32_t n_geom,
                         const hm_params* p, void* stream, hm_handle** out);

/*
 * hm_matvec -- y = H x, the approximate product of Sec. 2.3 (last
 * paragraph): dense leaves apply their stored block, admissible leaves apply
 * U (V^T x), so a product costs O(k N log N).  It is the one operation the
 * paper's solver needs per iteration (Sec. 3.4, Sec. 4.1).
 *   x, y   device, [n, nrhs] row-major, dtype `dtype` (HM_F64 or HM_F32),
 *          owned by the caller; y is overwritten; x and y must not overlap
 *   n      rows of x and y; must equal the handle's number of unknowns
 *          (else HM_ERR_ARG before any device access)
 *   nrhs   number of right-hand sides, >= 1
 * Accumulation is in double when either the storage or the vectors are
 * double, else in float.  Stream-ordered; no host synchronisation; allocates
 * nothing (the product workspace belongs to the handle).  Deterministic:
 * repeated calls give bitwise identical results.
 * Errors: HM_ERR_ARG (NULL handle or vector, n mismatch, nrhs < 1, bad dtype,
 * overlap), HM_ERR_HIP (launch failure).
 */
hm_status hm_matvec(hm_handle* h, const void* x, void* y, int64_t n, int32_t nrhs,
                    int32_t dtype, void* stream);

/*
 * hm_matvec_T -- y = H^T x with the same storage: the transpose of the
 * product of Sec. 2.3 block by block, (U V^T)^T = V U^T for admissible
 * leaves (U and V swap roles) and D^T for dense leaves.  The collocation
 * matrix is not symmetric, so this is a separate operation; the adjoint
 * solve uses it.  Arguments, ownership and errors as hm_matvec.
 */
hm_status hm_matvec_T(hm_handle* h, const void* x, void* y, int64_t n, int32_t nrhs,
                      int32_t dtype, void* stream);

typedef struct {
  double tol;          /* relative residual |f - H s| / |f| to reach, > 0   */
  int32_t restart;     /* GMRES restart length m, 1..1000; 0 => 100         */
  int32_t max_iter;    /* total Arnoldi steps allowed (inner steps included
                          with refine), >= 1                                */
  int32_t transpose;   /* 1: solve H^T s = f (adjoint), 0: H s = f          */
  int32_t use_x0;      /* 1: sigma holds the initial guess on entry         */
  int32_t flags;       /* HM_SOLVE_GRAPH, HM_SOLVE_CG or 0                  */
  int32_t refine;      /* 0: GMRES with double products throughout;
                          1: iterative refinement -- residual f - H s in
                          double (vectors and accumulation), correction by
                          GMRES whose products take float vectors (float
                          accumulation for the HM_F32 / HM_F32_F16 forms) to
                          the relative residual inner_tol, added in double  */
  double inner_tol;    /* refine = 1: inner relative tolerance in (0, 1);
                          0 => 1e-4.  Ignored when refine = 0               */
} hm_solve_params;

/* hm_solve_params.flags: replay one captured HIP graph per Arnoldi step
   (product, two Gram-Schmidt passes, norm) instead of launching its kernels
   one by one.  The graph and the solve workspace ((restart + 1) basis
   vectors) stay with the handle until the next solve with another nrhs,
   restart, direction or refine mode, or hm_free.  Results are bitwise those
   of flags = 0. */
#define HM_SOLVE_GRAPH 1
/* hm_solve_params.flags: conjugate gradients instead of GMRES, the solver of
   Sec. 4.1 for the symmetric positive definite Galerkin system (HM_GALERKIN
   handles; on a collocation handle CG is not guaranteed to converge).  One
   product per step, every right-hand side with its own step lengths, vectors
   and recurrences in double; stops when the recursively updated residual
   reaches tol relative to |f|, then checks the explicit residual (a column
   whose explicit residual misses tol is reported not converged).  restart is
   ignored; max_iter bounds the steps.  Not combined with HM_SOLVE_GRAPH,
   refine = 1 or transpose = 1 (HM_ERR_ARG). */
#define HM_SOLVE_CG 2

typedef struct {
  int32_t iters;          /* Arnoldi steps taken (max over right-hand sides;
                             summed over the inner solves with refine)      */
  int32_t restarts;       /* completed restart cycles                       */
  int32_t converged;      /* number of right-hand sides that converged      */
  int32_t ir_steps;       /* refinement corrections applied (0 without)     */
  double rel_residual;    /* max over rhs of the explicit |f - H s| / |f|,
                             with double products                            */
} hm_solve_info;

/*
 * hm_solve -- solve H s = f (or H^T s = f) for the density s.  The paper
 * solves its symmetric Galerkin system by CG with one H-matrix product per
 * step, stopped at a relative residual of 1e-8 (Sec. 4.1): HM_SOLVE_CG
 * (info->restarts then counts the explicit-residual cycles).  The
 * collocation matrix is not symmetric, so the default is restarted GMRES
 * with the same product:
 * x0 = 0 unless use_x0, Arnoldi basis in double with classical Gram-Schmidt
 * applied twice, Givens rotations on the host; the residual is recomputed
 * explicitly at every restart and at the end.  With refine = 1 the solve is
 * an iterative refinement around GMRES with float products (see
 * hm_solve_params); it stops when the double residual reaches tol, when
 * max_iter steps are spent, or when a correction no longer reduces the
 * residual of any unconverged column by 10%.  Each right-hand side is an
 * independent system; all are advanced together.
 *   f, sigma  device, [n, nrhs] row-major, dtype `dtype`, owned by the
 *             caller; must not overlap
 *   n         rows of f and sigma; must equal the handle's unknowns
 *   nrhs      1..256
 *   info      host, optional (may be NULL)
 * The solve allocates its workspace ((restart + 1) n nrhs doubles plus a
 * few vectors) from the library's pool for the call (kept with the handle
 * with HM_SOLVE_GRAPH).
 * Returns HM_OK when every column reached tol, HM_NOT_CONVERGED otherwise
 * (sigma then holds the last iterate; info says how far it got).
 * Errors: HM_ERR_ARG (NULL, n mismatch, bad nrhs / dtype / tol / restart /
 * max_iter / refine / inner_tol / flags, overlap), HM_ERR_OOM, HM_ERR_HIP.
 * Synchronises `stream`.
 */
hm_status hm_solve(hm_handle* h, const void* f, void* sigma, int64_t n, int32_t nrhs,
                   int32_t dtype, const hm_solve_params* sp, hm_solve_info* info,
                   void* stream);

/*
 * hm_solve_noalloc -- hm_solve for callers that cannot allocate device
 * memory (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and errors as hm_solve
 * (bitwise the same solution and info), but the solve workspace lives in a
 * fixed device array of HM_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends, and the call allocates
 * nothing (the product workspace already belongs to the handle).
 *   - The workspace needs 8 * (restart + 7) * n * nrhs bytes plus a little;
 *     larger requests fail with HM_ERR_ARG before any device work.
 *   - HM_SOLVE_GRAPH is rejected (HM_ERR_ARG).
 *   - Every call on one GPU shares that GPU's array: calls that overlap in
 *     time on one GPU (other threads, other streams) race and give wrong
 *     results; serialise them.  Nothing in the array is assumed to be zero
 *     or kept from the last call.
 */
#define HM_NOALLOC_SCRATCH_BYTES ((int64_t)128 << 20)
hm_status hm_solve_noalloc(hm_handle* h, const void* f, void* sigma, int64_t n, int32_t nrhs,
                           int32_t dtype, const hm_solve_params* sp, hm_solve_info* info,
                           void* stream);

/* Release every resource of h (NULL-safe); waits for work in flight.  The
   handle's device memory goes back to the library's memory pool on that
   device, which keeps it for later builds (allocating recently freed device
   memory from the driver again costs seconds per tens of GB);
   hm_release_memory returns it to the device. */
void hm_free(hm_handle* h);

/* Return the device memory cached in the library's pool of the current
   device (memory of freed handles and build temporaries) to the device.
   Memory of live handles is not affected.  Synchronises the device. */
hm_status hm_release_memory(void);

/* ---- introspection (tests, benchmarks) --------------------------------- */

typedef enum {
  HM_Q_STATS = 0,         /* hm_stats                                        */
  HM_Q_MORTON = 1,        /* uint64[n] Morton keys, application order        */
  HM_Q_PERM = 2,          /* int32[n] pi: Morton position -> triangle        */
  HM_Q_CLUSTERS = 3,      /* int32[ncl][4] (lo, hi, first child or -1, level),
                             breadth-first order                             */
  HM_Q_BOXES = 4,         /* double[ncl][6] (min xyz, max xyz)               */
  HM_Q_DENSE_BLOCKS = 5,  /* int64[ndense][6] (row_lo,row_hi,col_lo,col_hi,
                             arena offset of its first row slice, 0)          */
  HM_Q_LR_BLOCKS = 6,     /* int64[nlr][6] (row_lo,row_hi,col_lo,col_hi,
                             rank, cap_hit)                                  */
  HM_Q_LEAVES = 7,        /* int32[nleaf][3] (lo, size, ld) in Morton order  */
  HM_Q_TIMINGS = 8,       /* double[HM_NPHASE] milliseconds per setup phase  */
  HM_Q_LR_FACTORS = 9,    /* for LR block b = *(int64*)dst on entry: the
                             dense factors U (m x r) then V (n x r), both
                             column-major, in the build's storage type        */
  HM_Q_KERNEL_TIMES = 10, /* double[2][HM_NKERNEL]: accumulated milliseconds
                             and launch counts of the product stages since
                             the build or the last query (reset on read);
                             needs HM_PROFILE.  Stages: forward gather,
                             forward V^T x, (unused), forward panels, then
                             transposed gather, transposed panel dots,
                             transposed block sums, transposed column leaves */
  HM_Q_TUNE = 11,         /* double[k][2] (unit columns, ms per one-column
                             product) of every width the autotuner timed;
                             k = 0 without HM_AUTOTUNE                       */
  HM_Q_DENSE_ENTRIES = 12,/* for dense block b = *(int64*)dst on entry (the
                             order of HM_Q_DENSE_BLOCKS): its stored entries,
                             double[m][n] row-major, rows and columns in
                             Morton order of the block's clusters           */
  HM_Q_ACA_BINS = 13,     /* int32[8][2] (largest max(m, n) of the size bin,
                             kernel class) the batched ACA ran with; classes:
                             0 one 1,024-thread workgroup per block, 1 one
                             256-thread workgroup, 2, 3, 4 one wavefront with
                             4, 2, 1 rows and columns per lane, 5 one
                             128-thread workgroup                           */
  HM_Q_ACA_TUNE = 14      /* double[k][4] (bin, class, sampled blocks, ms of
                             one pass over them) of every candidate the ACA
                             binning tuner timed; k = 0 without HM_AUTOTUNE */
} hm_query_kind;

#define HM_NPHASE 8        /* geometry, morton+sort, tree+boxes, partition,
                              near field, aca, pack+items, total             */
#define HM_NKERNEL 8       /* product stages, see HM_Q_KERNEL_TIMES          */

typedef struct {
  int64_t n;
  int64_t n_clusters, n_leaves, n_dense, n_lr, depth;
  int64_t dense_entries;   /* sum over dense blocks of m*n                   */
  int64_t lr_entries;      /* sum over admissible blocks of r*(m+n)          */
  int64_t lr_u_entries;    /* sum over admissible blocks of r*m              */
  int64_t stored_bytes;    /* bytes of the stored operator (dense + factors,
                              including leaf padding)                        */
  int64_t rank_sum, rank_max, cap_hits;
  int64_t aca_entry_evals; /* matrix entries evaluated by ACA                */
  int64_t n_panel_cols;     /* columns of all row-leaf panels                 */
  int64_t n_titems;         /* items of the transposed product's column lists */
  int64_t device_bytes;    /* device memory held by the handle               */
  int64_t precision;
  int64_t aca_chunks;
  int64_t n_geom;           /* geometries in the handle                      */
  int64_t unit_cols;        /* column-unit width of the product schedule     */
} hm_stats;

/*
 * hm_query -- copy a piece of the built structure to host memory `dst`
 * (dst_bytes long).  *needed (optional) receives the required size; when
 * dst is NULL or too small, nothing is copied and HM_ERR_ARG is returned
 * (with *needed set).  Synchronises the handle's stream.
 */
hm_status hm_query(hm_handle* h, int32_t what, void* dst, int64_t dst_bytes,
                   int64_t* needed);

/*
 * hm_entries -- evaluate matrix entries a(rows[k], cols[k]) (application
 * indices) on the device with the build's entry kernel and precision (the
 * collocation entries, or with HM_GALERKIN the Galerkin entries, singular
 * pairs included); the result is written to out[k] as double.  rows, cols,
 * out: host arrays of length count.  Used to check the quadrature against
 * the oracle.
 */
hm_status hm_entries(hm_handle* h, const int32_t* rows, const int32_t* cols,
                     int64_t count, double* out);

/* Thread-local description of the last error ("" if none). */
const char* hm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HM_H */
