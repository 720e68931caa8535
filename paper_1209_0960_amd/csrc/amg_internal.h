// Internal declarations of the MI355X aggregation AMG library: the device
// layout of a hierarchy, the allocator, kernel launch wrappers and timing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "amg.h"

namespace amgx {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);

struct Failure {
  amg_status st;
};

#define AMG_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      ::amgx::set_error(std::string(#call) + ": " + hipGetErrorString(e_));                  \
      throw ::amgx::Failure{e_ == hipErrorOutOfMemory ? AMG_ERR_OUT_OF_MEMORY : AMG_ERR_HIP}; \
    }                                                                                        \
  } while (0)

[[noreturn]] void fail(amg_status st, const std::string& msg);

// ------------------------------------------------------------------ memory
// Device allocation through the user hook or the library's block cache.
void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);
// Synchronise a stream; blocks the library freed on it before the call become
// reusable from any stream.
void sync_stream(hipStream_t s);
hipError_t sync_stream_nothrow(hipStream_t s);

// RAII owner of a temporary device buffer.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  DBuf() = default;
  DBuf(size_t b, hipStream_t st) : bytes(b), s(st) { p = b ? dalloc(b, st) : nullptr; }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes), s(o.s) { o.p = nullptr; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      if (p) dfree(p, s);
      p = o.p;
      bytes = o.bytes;
      s = o.s;
      o.p = nullptr;
    }
    return *this;
  }
  ~DBuf() {
    if (p) dfree(p, s);
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// ------------------------------------------------------------------ timing
enum { KIND_NONE = -1 };
bool timing_on();
struct TimingRec {
  int kind;
  double bytes;
  hipEvent_t e0, e1;
};
int g_timing_mask_for_graphs();
// Records an event pair around a launch when timing is enabled.
struct KTimer {
  int kind;
  hipStream_t s;
  double bytes;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  KTimer(int k, hipStream_t st, double b);
  ~KTimer();
};

// ------------------------------------------------------------------ hierarchy
// A level of the hierarchy.  During construction the arrays are in the
// level's natural row order (level 0: the caller's order; level l+1: coarse
// rows numbered tile-major in aggregate creation order).  Once the hierarchy is
// complete, every level except the coarsest is relabelled into colour order
// (rows of colour 0 first, each colour in ascending natural order) and the
// arrays below then hold that "solve order": perm[r] is the natural row of
// solve row r.  The CSR entry order inside each row is unchanged.
struct Level {
  int n = 0, nnz = 0;
  int T = 512, ntiles = 0;
  int nc = 0;  // rows of the next level (0 on the coarsest)
  int ncol = 0;
  int sub = 8;  // lanes per row of the solve kernels (power of two >= mean row length, 4..64)
  // matrix
  int* rowptr = nullptr;
  int* colind = nullptr;
  double* vals = nullptr;
  float* vals32 = nullptr;
  double* l1 = nullptr;  // sum_j |a_ij| for l1-Jacobi
  float* l1_32 = nullptr;
  // aggregation (towards level l+1)
  int* agg = nullptr;       // n: coarse row of each row
  int* members = nullptr;   // n: rows grouped by coarse row, ascending natural order
  int* mptr = nullptr;      // nc+1 (natural coarse order)
  int* cinv = nullptr;      // nc: coarse solve row of each natural coarse row (NULL: identity)
  int* tile_off = nullptr;  // ntiles+1: first coarse row of each tile (natural order only)
  // colouring
  int* colour = nullptr;  // n (natural order only)
  int* crows = nullptr;   // n: rows grouped by colour, ascending (natural order only)
  std::vector<int> cptr;  // host, ncol+1: colour c = solve rows [cptr[c], cptr[c+1])
  int* perm = nullptr;    // n: natural row of each solve row (NULL: identity)
  // Solve-phase matrix in SELL-64 form: slice s holds solve rows
  // [srow[s], srow[s+1]) (at most 64, never across a colour boundary); its
  // off-diagonal entries are stored column-major (entry k of lane t at
  // soff[s] + 64 k + t), padded to the slice's longest row with (row, 0.0);
  // the diagonal is kept apart.  sptr[c] = first slice of colour c.
  int nsl = 0;
  std::vector<int> sptr;  // host, ncol+1
  int* sptr_d = nullptr;  // device copy of sptr
  int* srow = nullptr;    // nsl+1
  std::vector<int> srow_h, soff_h;  // host copies (launch sizes, byte counts)
  int* soff = nullptr;    // nsl+1
  int* scol = nullptr;
  double* sval = nullptr;
  float* sval32 = nullptr;
  double* dg = nullptr;
  float* dg32 = nullptr;
  // smoother of this level (AMG_SMOOTHER_*)
  int sm = AMG_SMOOTHER_MCSGS;
  // tile-ordered multicolour smoother: the level's colours (solve order) and
  // their count, and per tile of T rows the first tile-local row of each
  // colour (ntiles x (tncol + 1)); the solve order takes each tile's rows
  // colour by colour, the slices see one colour of 64 consecutive rows
  int* tcol = nullptr;
  int tncol = 0;
  int* tcb = nullptr;
  // hybrid smoother (natural order, slices of 64 consecutive rows)
  unsigned short* hsf = nullptr;  // n: forward wavefront step inside the tile
  unsigned short* hsb = nullptr;  // n: backward wavefront step
  int hdf = 0, hdb = 0;           // largest steps
  int hw = 0;                     // most in-tile couplings of a row
  int hg = 1;                     // lanes per row of the in-tile sweeps (1, or HS_G when hw > 8)
  // in-tile couplings of each row (tile sweeps): icp (n+1) offsets, icc local
  // column (row - first row of the tile), icv value (FP64, or FP32 on FP32
  // cycles), in SELL entry order; a tile's couplings are contiguous
  int* icp = nullptr;
  unsigned short* icc = nullptr;
  double* icv = nullptr;
  float* icv32 = nullptr;
  // couplings to other tiles (tile sweeps), likewise: ocp (n+1), global
  // column (solve order), value
  int* ocp = nullptr;
  int* occ = nullptr;
  double* ocv = nullptr;
  float* ocv32 = nullptr;
  long long ocn = 0;
  int icmax = 0;                  // most in-tile couplings of one tile
  long long icn = 0;              // in-tile couplings of the level
  // optional setup data (natural order; on point-based levels per node and node-graph entry)
  uint8_t* strong = nullptr;
  uint8_t* iso = nullptr;
  // point-based levels (Sec. 4.2): unknowns per node, and for the block smoother
  // row c of the inverse diagonal block of each row's node (n x bs, solve order)
  int bs = 1;
  int nn = 0, nnzb = 0;  // nodes and node-graph entries (setup data sizes)
  double* dinv = nullptr;
  float* dinv32 = nullptr;
};

struct Batch;

struct Hierarchy {
  amg_params p{};
  int flexible = 0;
  std::vector<Level> lev;
  int nL = 0;
  double* Ainv = nullptr;  // dense inverse of the coarsest matrix (FP64, symmetric)
  double setup_ms = 0.0;
  // Solve context of pcg_solve / amg_precond_apply (one entry, one right-hand
  // side), created on first use and released with the hierarchy.
  Batch* single = nullptr;
  size_t bytes = 0;
  std::vector<std::pair<void*, size_t>> owned;
  std::mutex owned_mu;  // alloc / free_one from the setup's two host threads
  hipStream_t setup_stream = nullptr;
  // Recorded on the caller's stream after each amg_precond_apply (which runs
  // there, asynchronously); release() waits for it before any buffer returns
  // to the allocator.
  hipEvent_t apply_done = nullptr;

  // Frees one buffer obtained from alloc() (no-op for NULL).
  void free_one(void* ptr, hipStream_t s);
  template <typename T>
  T* alloc(size_t count, hipStream_t s) {
    size_t b = count * sizeof(T);
    if (b == 0) b = sizeof(T);
    void* ptr = dalloc(b, s);
    std::lock_guard<std::mutex> g(owned_mu);
    owned.emplace_back(ptr, b);
    bytes += b;
    return static_cast<T*>(ptr);
  }
  void release(hipStream_t s);
};

// Slots of the per-right-hand-side scalar block used by the CG kernels.
enum {
  S_RHO = 0,  // r.z of the current direction
  S_PQ,       // p.A p
  S_ALPHA,
  S_RR,       // r.r after the update
  S_RZ,
  S_ZDR,      // z.(r - r_old) (flexible CG)
  S_BETA,
  S_FLAG,     // 1.0 = breakdown (p.A p <= 0 or r.z <= 0): updates stop
  S_R0,       // r_0.r_0
  S_TMP,      // ||b - A x||^2 at the end
  S_TMP2,     // ||b||^2 at the end
  S_NEWP,     // 1.0 until the first direction is formed (p = z, beta unused)
  S_COUNT = 16
};

// Scalars of a BiCGSTAB solve (device, one right-hand side).
enum {
  BS_RHO = 0,  // r~.r of the current direction
  BS_ALPHA,
  BS_OMEGA,
  BS_BETA,
  BS_SS,       // s.s of the half step
  BS_RR,       // r.r after the update
  BS_RR0,      // r_0.r_0
  BS_FLAG,     // breakdown, updates stop: 1 at alpha, 2 at omega, 3 at beta (x = x_k)
  BS_HALF,     // 1.0 = converged at the half step (x = x + alpha M p): updates stop
  BS_TMP,      // ||b - A x||^2 at the end
  BS_TMP2,     // ||b||^2 at the end
  BS_COUNT = 16
};
// Finish operations of the BiCGSTAB reductions (kk_bcg_finish).
enum { BF_INIT = 0, BF_ALPHA, BF_S, BF_OMEGA, BF_BETA, BF_TRUE, BF_BB };

constexpr int RED_BLOCKS = 8192;  // upper bound on the partial sums of one dot product
constexpr int RED_THREADS = 256;
constexpr int MAX_LEVELS = 32;
constexpr int MAX_RHS = 8;
constexpr int CTL_INTS = 16;  // per entry: [0] active, [1 + k] right-hand side k finished

// ------------------------------------------------------------------ setup kernels
// Validation: returns bit flags 1 = invalid structure/value, 2 = bad diagonal,
// 4 = not symmetric.
int validate_csr(int n, int nnz, const int* rp, const int* ci, const double* v, int check_symmetry,
                 hipStream_t s);
// sym: the level's values are known to be exactly symmetric.
void strength(const Level& L, double delta, double beta, uint8_t* strong, uint8_t* iso, bool sym, hipStream_t s);
// Returns the number of coarse rows; fills agg, members, mptr, tile_off.
int aggregate(Hierarchy& H, Level& L, const uint8_t* strong, const uint8_t* iso, const amg_params& p, hipStream_t s);
// Galerkin product; returns the coarse level's CSR arrays allocated in H.
void galerkin(Hierarchy& H, const Level& L, Level& C, hipStream_t s);
void colour(Hierarchy& H, Level& L, uint32_t seed, hipStream_t s);
// One colour, natural order (the hybrid smoother needs no colouring).
void colour_single(Hierarchy& H, Level& L, hipStream_t s);
// Wavefront steps of the in-tile sweeps of the hybrid smoother (after
// build_sell; the level has one colour).
void hybrid_steps(Hierarchy& H, Level& L, int T, hipStream_t s);
// Colouring of a level of the tile-ordered multicolour smoother: every tile
// of T rows (the level's smoothing tiles) on its own, first fit over its rows ascending on the couplings
// inside the tile (natural order, before relabelling).
void colour_tile_local(Hierarchy& H, Level& L, int T, hipStream_t s);
// After colour_tile_local on a level of the tile-ordered multicolour smoother: the
// solve order takes each tile's rows colour by colour (reorder; the coarsest
// level keeps natural order), one colour for the slices, the colours in
// L.tcol (solve order) and each tile's colour bounds in L.tcb.
void tile_colour_order(Hierarchy& H, Level& L, bool reorder, hipStream_t s);
// The in-tile couplings of a tile-sweep level (after build_sell and
// hybrid_steps, before the FP64 SELL values of an FP32 level are dropped).
void tile_couplings(Hierarchy& H, Level& L, bool f32, hipStream_t s);

// Lanes per row of the in-tile sweeps on levels whose rows have more than 8
// in-tile couplings (the others take one lane per row).
constexpr int HS_G = 4;

// Smoother of level l under parameters p.
inline int level_smoother(const amg_params& p, int l) {
  return p.coarse_smoother >= 0 && l >= p.coarse_from ? p.coarse_smoother : p.smoother;
}
// Process-wide pools of streams and events (reused across calls).
hipStream_t stream_take();
void stream_give(hipStream_t st);  // synchronises the stream first
hipEvent_t event_take();
void event_give(hipEvent_t e);
// Whether level l's smoother runs as tile sweeps (the hybrid smoother, in
// natural or colour order: the same launches, the order is in the steps).
inline bool tile_sweeps(int sm) { return sm == AMG_SMOOTHER_HYBRID_SGS || sm == AMG_SMOOTHER_TILE_MCSGS; }
// Rows per smoothing tile of level l (the blocks of the tile smoothers).
inline int smooth_tile(const amg_params& p, int l) {
  const int fine = p.smooth_tile_rows > 0 ? p.smooth_tile_rows : p.tile_rows;
  return p.coarse_smooth_tile_rows > 0 && l >= p.coarse_from ? p.coarse_smooth_tile_rows : fine;
}
void cast_f32(const double* in, float* out, size_t n, hipStream_t s);
void l1_diag(const Level& L, double* out64, float* out32, hipStream_t s);
// Dense FP64 factorisation of the coarsest level and its explicit inverse.
void coarse_factor(Hierarchy& H, const Level& L, hipStream_t s);
// Relabels level l into colour order (solve order); `next_perm` is the solve
// order of level l+1 (NULL: identity, the coarsest level).  Frees the natural
// order arrays that the solve does not need.
void permute_level(Hierarchy& H, int l, const int* next_perm, hipStream_t s);
// out[r] = in[perm[r]] (gather) and out[perm[r]] = in[r] (scatter); perm NULL: copy.
void gather(int n, const int* perm, const double* in, double* out, hipStream_t s);
// Builds the SELL-64 arrays of a level in solve order from its CSR and frees the CSR.
void build_sell(Hierarchy& H, int l, hipStream_t s);
void scatter(int n, const int* perm, const double* in, double* out, hipStream_t s);
void exclusive_scan(const int* in, int* out, int n, hipStream_t s);  // out has n+1 entries
// Point-based levels: block structure check (returns flag 1 when a node's rows
// are not whole blocks with the diagonal block), the node graph with the block
// weights, expansion of node aggregates and colours to the unknowns, inverses
// of the diagonal blocks (after the level is in solve order, before build_sell).
int validate_blocks(int n, int bs, const int* rp, const int* ci, hipStream_t s);
void node_graph(Hierarchy& H, const Level& L, int bs, Level& S, hipStream_t s);
void release_level(Hierarchy& H, Level& S, hipStream_t s);
void expand_aggregates(Hierarchy& H, const Level& S, int bs, Level& L, hipStream_t s);
void expand_colours(Hierarchy& H, const Level& S, int bs, Level& L, hipStream_t s);
void block_inverses(Hierarchy& H, Level& L, int bs, bool f32, hipStream_t s);

// ------------------------------------------------------------------ solve engine
// Every solve-phase launch is table driven: block b of a launch reads
// tab[b] = {d, lo, hi, part} and works on units [lo, hi) (rows, slices or
// coarse rows, by kernel) of descriptor D[d], one (entry, level) pair of a
// batch; reductions write their block sum to partial index `part` of the
// entry.  The split of an entry's units into blocks depends on that entry
// alone, so its arithmetic is the same in every batch it runs in.
struct Item {
  int d, lo, hi, part;
};

// Device descriptor of one level of one batch entry.  Matrix arrays belong to
// the hierarchy, vectors to the entry (right-hand sides interleaved: value k
// of row i at i * R + k, rows in solve order).
struct BDesc {
  const int *srow, *soff, *scol;
  const double *sval64, *dg64, *l164;
  const float *sval32, *dg32, *l132;
  const int *rowptr, *colind;  // CSR (one-level hierarchies only)
  const double* vals;
  const int *mptr, *members, *agg;  // transfer to level l+1
  const int* cinv;                  // natural -> solve order of level l+1 (NULL: identity)
  const double* Ainv;               // coarsest level: dense inverse (nL x nL)
  void *x, *b, *t;                  // this level's iterate, right-hand side, residual
  void *xc, *bc;                    // level l+1's iterate and right-hand side
  double *r, *z, *p, *q, *rold, *xs, *bs;  // level-0 CG vectors
  double* partial;                  // [2][RED_BLOCKS][R]
  double* scal;                     // [R][S_COUNT]
  const int* sptr;                  // ncol+1: first slice of each colour
  int ncol;
  // hybrid smoother: wavefront step of each row in the forward / backward
  // sweep inside its tile of T rows, and the largest step of each sweep
  const unsigned short *hsf, *hsb;
  int T, hdf, hdb, hw, hg;
  const int* icp;                   // in-tile couplings (tile sweeps): offsets, local column, value
  const unsigned short* icc;
  const double* icv64;
  const float* icv32;
  const int *ocp, *occ;             // couplings to other tiles (tile sweeps): offsets, column, value
  const double* ocv64;
  const float* ocv32;
  const int* tcb;                   // tile-ordered multicolour levels: colour bounds of each tile (tncol + 1)
  const int* tcol;                  //   and the colour of each row (solve order)
  int tncol;
  int sm;                           // AMG_SMOOTHER_* of the level (tile forms: OP_RESID_OFF + OP_HSGS)
  const int* ctl;                   // [CTL_INTS]
  int active;                       // 0: the entry is finished (table launches skip it)
  int n, nc, nsl, nL;
  int nt;                           // 1: SELL entries larger than the last-level cache (streaming loads)
  int blk;                          // unknowns per node (point-based levels > 1)
  const double* dinv64;             // row c of the inverse diagonal block of each row's node (n x bs)
  const float* dinv32;
  double omega;
};

// Kernel selectors of a launch.
enum {
  OP_ZERO = 0,   // x = 0 (rows)
  OP_GS,         // Gauss-Seidel on the slices of one colour
  OP_RESID,      // t = b - A x (slices)
  OP_JACOBI,     // x += t / l1 (rows)
  OP_RESTRICT,   // b_c = P^T t (coarse rows)
  OP_PROLONG,    // x += omega P x_c (rows)
  OP_COARSE,     // x = A_L^{-1} b (rows of the coarsest level, 4 per block)
  OP_TAIL,       // down-leg of levels lt..L-1 of one entry in one workgroup (zero, pre-smooth, restrict)
  OP_R2B,        // FP32 cycle: b_0 = (float) r
  OP_X2Z,        // FP32 cycle: z = (double) x_0
  OP_DOTS_RZ,    // partials of r.z and z.(r - r_old)
  OP_UPDATE_P,   // p = z + beta p
  OP_SPMV_DOT,   // q = A p, partials of p.q (SELL slices)
  OP_SPMV_DOT_CSR,   // same on a CSR level 0 (aux = lanes per row)
  OP_UPDATE_XR,  // x += alpha p, r -= alpha q, partials of r.r
  OP_RESID_DOT,  // out = b - A x, partials of out.out (aux = 0: out = r, 1: out = q)
  OP_RESID_DOT_CSR,  // same on a CSR level 0 (aux2 = lanes per row)
  OP_DOT_BB,     // partials of b.b
  OP_VZERO_ROLD, // r_old = 0 (rows)
  OP_FINISH,     // per entry: reduce partials, scalar update (aux = FIN_*, aux2 = slot)
  OP_GS0,        // first Gauss-Seidel pass from x = 0: x = b / diag on the slices of one colour
  OP_TAIL_UP,    // up-leg of levels L-1..lt of one entry in one workgroup (prolong, post-smooth)
  OP_GS_RESID,   // Gauss-Seidel pass that also writes the residual of its rows
  OP_RESID_OFF,  // hybrid smoother: t = b - (couplings to other tiles) x (slices)
  OP_HSGS,       // hybrid smoother: in-tile forward + backward sweeps (tiles; aux = 1: from b, x = 0)
  OP_BGS,        // point-based level: block Gauss-Seidel on the slices of one colour (whole nodes)
  OP_TSGS,       // tile-ordered multicolour smoother: in-tile sweeps colour by colour (tiles; aux bit 0: from
                 // b, bit 1: also the in-tile sums of the residual into t)
  OP_RESID_TILE, // tile-sweep level: t = b - A x from the compact couplings (rows; aux = 1: in-tile sums in t)
};

// LDS bytes of the LDS-staged colour-ordered tile sweep (tiles of T rows, at
// most C in-tile couplings per tile, R right-hand sides, NC colours, values
// of vb bytes): iterate, source, diagonal; coupling offsets and colour
// bounds (int); then, 8-byte aligned, the couplings' values and 16-bit local
// columns.
__host__ __device__ inline size_t tsgs_fixed_bytes(int T, int R, int NC, size_t vb) {
  const size_t b = (size_t)T * (2 * R + 1) * vb + (size_t)(T + 1 + NC + 1) * sizeof(int);
  return (b + 7) & ~(size_t)7;
}
__host__ __device__ inline size_t tsgs_lds_bytes(int T, int C, int R, int NC, size_t vb) {
  return tsgs_fixed_bytes(T, R, NC, vb) + (size_t)C * (vb + sizeof(unsigned short));
}

// LDS bytes and eligibility of the register form of the colour-ordered tile
// sweep (one thread per row, tiles of at most 256 rows, at most 32 in-tile
// couplings per row W, at most C per tile, one right-hand side).
inline size_t tsgs_reg_lds_bytes(int T, int C, size_t vb) {
  return (size_t)T * vb + (size_t)C * (vb + sizeof(unsigned short));
}
inline bool tsgs_reg_ok(int R, int T, int W, int C, size_t vb) {
  return R == 1 && T <= 256 && W <= 32 && tsgs_reg_lds_bytes(T, C, vb) <= 65536;
}
enum { FIN_STORE = 0, FIN_ALPHA, FIN_BETA_PCG, FIN_BETA_FCG, FIN_INIT };

struct Launch {
  int op = 0, level = 0, aux = 0, aux2 = 0, aux3 = 0;
  size_t off = 0;  // first item in the plan's table
  int nblk = 0;
  int kind = KIND_NONE;
  double bytes = 0.0;  // algorithmic HBM bytes
  // Plans of one entry launch without a table: descriptor direct.d passed by
  // value, units [direct.lo, direct.hi) in pieces of direct.part per block.
  bool use_direct = false;
  Item direct{};
};

// Enqueues launches[i] for i in [first, last) with tables at `tab`.
// Dh: host copy of the descriptors (direct launches pass one by value).
void issue_launches(const std::vector<Launch>& L, size_t first, size_t last, const Item* tab, const BDesc* D,
                    const BDesc* Dh, int R, int fp32, hipStream_t s);
// out = in permuted and interleaved: out[r * R + k] = in[k * n + perm[r]]
// (gather) and its inverse (scatter); perm NULL: identity.
void gather_rhs(int n, int R, const int* perm, const double* in, double* out, hipStream_t s);
void scatter_rhs(int n, int R, const int* perm, const double* in, double* out, hipStream_t s);

// BiCGSTAB level-0 kernels (one right-hand side, FP64, solve order).  Each
// reduction leaves two partial sums per block in part[2 * block + {0, 1}];
// bcg_finish sums them in block order.  Returns the number of blocks.
// y = A x, or y = c - A x (c non-NULL); partials (w.y, y.y), w nullable.
// sub: lanes per CSR row; bytes: algorithmic bytes (kernel timing).
int bcg_spmv(const BDesc& d0, int sub, const double* x, const double* c, double* y, const double* w, double* part,
             double bytes, hipStream_t s);
// s = r - alpha v, x += alpha ph; partials (0, s.s).
int bcg_half(int n, const double* r, const double* v, const double* ph, double* x, double* sv, const double* sc,
             double* part, hipStream_t s);
// x += omega sh, r = s - omega t; partials (r~.r, r.r).
int bcg_full(int n, const double* sv, const double* t, const double* sh, const double* rt, double* x, double* r,
             const double* sc, double* part, hipStream_t s);
// p = r + beta (p - omega v), also into pin; init: p = pin = rt = r.
void bcg_dir(int n, const double* r, const double* v, double* p, double* pin, double* rt, const double* sc,
             int init, hipStream_t s);
// partials (0, u.u)
int bcg_norm2(int n, const double* u, double* part, hipStream_t s);
void bcg_finish(int op, int nb, const double* part, double* sc, double tol2, hipStream_t s);

void batch_destroy(Batch* B);
// pcg_solve / amg_precond_apply / pcg_solve_batched on the engine.
amg_status pcg_run(Hierarchy& H, const double* b, double* x, double rtol, int maxit, amg_solve_info* info,
                   double* res_hist, double* iter_hist, hipStream_t us);
void precond_run(Hierarchy& H, const double* r, double* z, hipStream_t us);
// The same V-cycle with its vectors in the library's fixed per-device scratch
// array (no allocation); fails with AMG_ERR_UNSUPPORTED when they do not fit.
void precond_noalloc_run(Hierarchy& H, const double* r, double* z, hipStream_t us);
size_t precond_noalloc_bytes(const Hierarchy& H);
size_t precond_noalloc_capacity();
// bicgstab_solve (Sec. 5: BiCGSTAB with the V-cycle applied twice per iteration).
amg_status bicgstab_run(Hierarchy& H, const double* b, double* x, double rtol, int maxit, amg_solve_info* info,
                        int* half_step, double* res_hist, double* iter_hist, hipStream_t us);
amg_status pcg_batched_run(Hierarchy* const* hs, int nsys, int nrhs, const double* const* b, double* const* x,
                           double rtol, int maxit, amg_solve_info* info, hipStream_t us);
// Continuous batching: entries are submitted and retired between steps.
Batch* batch_new(int R, int cap, int use_graphs);
int batch_submit(Batch& B, Hierarchy& H, const double* b, double* x, double rtol, int maxit, int64_t tag,
                 hipStream_t us);
void batch_step(Batch& B, int iterations);
int batch_active(const Batch& B);
int batch_poll(Batch& B, int64_t* tags, amg_status* status, amg_solve_info* info, int cap);
size_t batch_entry_bytes(const Batch& B);


}  // namespace amgx
