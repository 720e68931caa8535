// Internal declarations of the MI355X aggregation AMG library: the device
// layout of a hierarchy, the allocator, kernel launch wrappers and timing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
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
// Device allocation through the user hook or stream-ordered hipMallocAsync.
void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);

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
  int* mptr = nullptr;      // nc+1
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
  int* srow = nullptr;    // nsl+1
  std::vector<int> srow_h, soff_h;  // host copies (launch sizes, byte counts)
  int* soff = nullptr;    // nsl+1
  int* scol = nullptr;
  double* sval = nullptr;
  float* sval32 = nullptr;
  double* dg = nullptr;
  float* dg32 = nullptr;
  // optional setup data (natural order)
  uint8_t* strong = nullptr;
  uint8_t* iso = nullptr;
  // V-cycle work vectors (precision of the cycle, solve order)
  double* x64 = nullptr;
  double* b64 = nullptr;
  double* t64 = nullptr;
  float* x32 = nullptr;
  float* b32 = nullptr;
  float* t32 = nullptr;
};

struct Hierarchy {
  amg_params p{};
  int flexible = 0;
  std::vector<Level> lev;
  int nL = 0;
  double* Ainv = nullptr;  // dense inverse of the coarsest matrix (FP64, symmetric)
  // CG work space
  double *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr, *rold = nullptr;
  double *bp = nullptr, *xp = nullptr;  // level-0 right-hand side / iterate in solve order
  double* partial = nullptr;  // reduction partials
  double* scal = nullptr;     // device scalars
  double* host_scal = nullptr;  // pinned
  double setup_ms = 0.0;
  // solve stream and the captured CG iteration
  hipStream_t work = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t iter_exec = nullptr;
  size_t bytes = 0;
  std::vector<std::pair<void*, size_t>> owned;
  hipStream_t setup_stream = nullptr;

  // Frees one buffer obtained from alloc() (no-op for NULL).
  void free_one(void* ptr, hipStream_t s);
  template <typename T>
  T* alloc(size_t count, hipStream_t s) {
    size_t b = count * sizeof(T);
    if (b == 0) b = sizeof(T);
    void* ptr = dalloc(b, s);
    owned.emplace_back(ptr, b);
    bytes += b;
    return static_cast<T*>(ptr);
  }
  void release(hipStream_t s);
};

// Slots of the device scalar block used by the CG kernels.
enum {
  S_RHO = 0,
  S_PQ,
  S_ALPHA,
  S_RR,
  S_RZ,
  S_ZDR,
  S_BETA,
  S_FLAG,  // 1.0 = breakdown
  S_R0,
  S_TMP,
  S_COUNT = 16
};

constexpr int RED_BLOCKS = 1024;  // fixed number of partial sums of every dot product
constexpr int RED_THREADS = 256;

// ------------------------------------------------------------------ setup kernels
// Validation: returns bit flags 1 = invalid structure/value, 2 = bad diagonal,
// 4 = not symmetric.
int validate_csr(int n, int nnz, const int* rp, const int* ci, const double* v, int check_symmetry,
                 hipStream_t s);
void strength(const Level& L, double delta, double beta, uint8_t* strong, uint8_t* iso, hipStream_t s);
// Returns the number of coarse rows; fills agg, members, mptr, tile_off.
int aggregate(Hierarchy& H, Level& L, const uint8_t* strong, const uint8_t* iso, const amg_params& p, hipStream_t s);
// Galerkin product; returns the coarse level's CSR arrays allocated in H.
void galerkin(Hierarchy& H, const Level& L, Level& C, hipStream_t s);
void colour(Hierarchy& H, Level& L, uint32_t seed, hipStream_t s);
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

// ------------------------------------------------------------------ solve kernels
template <typename V>
void vcycle(Hierarchy& H, int l, const V* b, V* x, hipStream_t s);
void precond_apply(Hierarchy& H, const double* r, double* z, hipStream_t s);
// y = A x (FP64) for level 0, fused partial of dot(x, y) when `partial` is set.
void spmv64(const Level& L, const double* x, double* y, double* partial, hipStream_t s, int kind);
void residual64(const Level& L, const double* b, const double* x, double* r, double* partial, hipStream_t s);

// CG vector kernels: each writes RED_BLOCKS partial sums, reduced by finish_*.
void cg_update_xr(int n, double* x, double* r, double* rold, const double* p, const double* q,
                  const double* scal, double* partial, hipStream_t s);
void cg_dots_rz(int n, const double* r, const double* z, const double* rold, double* partial, hipStream_t s);
void cg_update_p(int n, double* p, const double* z, const double* scal, hipStream_t s);
void dot_partial(int n, const double* a, const double* b, double* partial, hipStream_t s);
// Reduces `nparts` partial sums into scal[slot]; op selects the scalar update.
enum { FIN_STORE = 0, FIN_ALPHA, FIN_BETA_PCG, FIN_BETA_FCG, FIN_RHO_INIT };
void finish(double* partial, int nparts, double* scal, int slot, int op, hipStream_t s);

}  // namespace amgx
