// Solve engine: one or many CG solves (entries) advanced together, one CG
// iteration of every active entry per step.  A step is a fixed list of
// table-driven launches (the V-cycle of Sec. 2 level by level over all
// entries, then the CG vector updates), built once per set of entries and
// replayed as a HIP graph while the set is unchanged.  Entries join (after a
// prologue that forms r_0) and leave (after the true residual and the copy of
// x back to the caller) between steps, which gives pcg_solve (one entry),
// pcg_solve_batched (all entries start together) and the continuous-batching
// interface amg_batch_* the same code and the same per-entry arithmetic.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "amg_internal.h"

namespace amgx {

namespace {

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int ROW_CH = 1024;     // rows per block of the row-wise kernels
constexpr int RESTRICT_CH = 256; // coarse rows per block of the restriction
constexpr int SLICES_PB = 4;     // slices per block of the sweep / residual kernels

// Number of partial sums of a reduction over n rows (or slices): depends on
// the entry alone.
// Row reductions stream (threads stride over rows; 4096 blocks keep enough
// waves in flight at 256^3, more measured no faster);
// slice reductions are chains of dependent loads per wavefront (at most 8
// slices per wavefront), so they get more blocks.
int red_blocks_rows(int n) { return std::min(4096, std::max(1, cdiv(n, 2048))); }
int red_blocks_slices(int nsl) { return std::min(RED_BLOCKS, std::max(1, cdiv(nsl, 32))); }

// Process-wide reuse of pinned host buffers, streams and events: creating and
// destroying them costs milliseconds of runtime calls per solve context.
std::mutex g_pool_mu;
std::vector<std::pair<size_t, void*>> g_pinned;  // (bytes, pointer), free
std::vector<std::pair<int, hipStream_t>> g_streams;  // (device, stream), free
std::vector<std::pair<int, hipEvent_t>> g_events;

void* pinned_take(size_t bytes) {
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    size_t best = SIZE_MAX;
    for (size_t i = 0; i < g_pinned.size(); ++i)
      if (g_pinned[i].first >= bytes && g_pinned[i].first <= 4 * bytes + 65536 &&
          (best == SIZE_MAX || g_pinned[i].first < g_pinned[best].first))
        best = i;
    if (best != SIZE_MAX) {
      void* p = g_pinned[best].second;
      g_pinned[best] = g_pinned.back();
      g_pinned.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  AMG_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
  return p;
}
void pinned_give(void* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> g(g_pool_mu);
  g_pinned.emplace_back(bytes, p);
}
int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

}  // namespace

hipStream_t stream_take() {
  const int dev = current_device();
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    for (size_t i = 0; i < g_streams.size(); ++i)
      if (g_streams[i].first == dev) {
        hipStream_t st = g_streams[i].second;
        g_streams[i] = g_streams.back();
        g_streams.pop_back();
        return st;
      }
  }
  hipStream_t st = nullptr;
  AMG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  return st;
}
void stream_give(hipStream_t st) {
  if (!st) return;
  (void)sync_stream_nothrow(st);
  std::lock_guard<std::mutex> g(g_pool_mu);
  g_streams.emplace_back(current_device(), st);
}
hipEvent_t event_take() {
  const int dev = current_device();
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    for (size_t i = 0; i < g_events.size(); ++i)
      if (g_events[i].first == dev) {
        hipEvent_t e = g_events[i].second;
        g_events[i] = g_events.back();
        g_events.pop_back();
        return e;
      }
  }
  hipEvent_t e = nullptr;
  AMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return e;
}
void event_give(hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> g(g_pool_mu);
  g_events.emplace_back(current_device(), e);
}

// Device vectors of one entry (right-hand sides interleaved, solve order),
// carved from one allocation.
struct Ctx {
  void* block = nullptr;
  size_t bytes = 0;
  std::vector<void*> x, b, t;  // per level, precision of the cycle
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *rold = nullptr, *xs = nullptr, *bs = nullptr;
  double* partial = nullptr;
  void release(hipStream_t s) {
    if (block) dfree(block, s);
    block = nullptr;
    bytes = 0;
    x.clear();
    b.clear();
    t.clear();
  }
};

// Two-pass carving: the first pass sums aligned sizes, the second hands out
// pointers into the block.
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  void* take(size_t n) {
    void* p = base ? base + off : nullptr;
    off += (n + 255) & ~(size_t)255;
    return p;
  }
};

struct Result {
  int64_t tag = 0;
  amg_status status = AMG_OK;
  amg_solve_info info[MAX_RHS];
};

struct Entry {
  bool used = false;       // holds a solve (running or awaiting finalisation)
  bool complete = false;   // every right-hand side finished
  Hierarchy* bound = nullptr;  // hierarchy whose vectors and descriptors the slot holds
  Ctx ctx;
  const double* b_user = nullptr;
  double* x_user = nullptr;
  double rtol = 0.0;
  int maxit = 0;
  int64_t tag = 0;
  bool started = false;
  double r0[MAX_RHS], rel[MAX_RHS];
  int it[MAX_RHS];
  amg_status st[MAX_RHS];
  bool done[MAX_RHS];
  double* res_hist = nullptr;   // host, R = 1 only
  double* iter_hist = nullptr;  // device, R = 1 only
  double t0 = 0.0;
};

struct Plan {
  std::vector<Launch> L;
  size_t precond_end = 0;  // launches [0, precond_end) form the V-cycle
  Item* tab_d = nullptr;
  size_t cap = 0;
  hipGraphExec_t exec = nullptr;
  int runs = 0;
  std::vector<int> slots;
  double rows = 0.0;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    runs = 0;
  }
};

struct Batch {
  int R = 1, cap = 0, use_graphs = 1;
  bool single = false;  // the per-hierarchy context of pcg_solve / amg_precond_apply
  // All entries start together and are completed at the end (pcg_solve_batched):
  // finished entries are only switched off, the launch plan is kept.
  bool deferred = false;
  int fp32 = -1, smoother = 0, pre = 0, post = 0, flexible = 0, bs = 1;
  int coarse_smoother = -1, coarse_from = 1;  // per-level smoother choice (shared by the entries)
  int stile[MAX_LEVELS] = {};                  // smoothing tile of each level (shared with a tile smoother)
  hipStream_t work = nullptr;
  hipEvent_t ev = nullptr;
  BDesc* desc_d = nullptr;
  BDesc* desc_h = nullptr;  // pinned host copy, uploaded whole when dirty
  bool desc_dirty = false, ctl_dirty = false;
  double* scal_d = nullptr;
  double* scal_h = nullptr;  // pinned
  int* ctl_d = nullptr;
  int* ctl_h = nullptr;  // pinned
  std::vector<Entry> ent;
  std::vector<int> pending;  // slots awaiting their prologue
  std::vector<Result> results;
  Plan iter, tmp;
  Plan papply;  // the preconditioner alone (amg_precond_apply)
  bool dirty = true;

  size_t scal_count() const { return (size_t)cap * R * S_COUNT; }
  double* scal_of(int slot) const { return scal_d + (size_t)slot * R * S_COUNT; }
  const double* scal_h_of(int slot) const { return scal_h + (size_t)slot * R * S_COUNT; }
  int desc_index(int slot, int l) const { return slot * MAX_LEVELS + l; }
};

namespace {

// ------------------------------------------------------------------ set-up of a batch
void batch_init(Batch& B, int R, int cap, int use_graphs) {
  if (R != 1 && R != 2 && R != 4 && R != 8) fail(AMG_ERR_UNSUPPORTED, "right-hand sides per entry must be 1, 2, 4 or 8");
  if (cap < 1) fail(AMG_ERR_INVALID_ARG, "batch capacity must be positive");
  B.R = R;
  B.cap = cap;
  B.use_graphs = use_graphs;
  B.ent.resize(cap);
  B.work = stream_take();
  B.ev = event_take();
  B.desc_h = static_cast<BDesc*>(pinned_take((size_t)cap * MAX_LEVELS * sizeof(BDesc)));
  for (size_t i = 0; i < (size_t)cap * MAX_LEVELS; ++i) B.desc_h[i] = BDesc{};
  B.desc_d = static_cast<BDesc*>(dalloc((size_t)cap * MAX_LEVELS * sizeof(BDesc), B.work));
  B.scal_d = static_cast<double*>(dalloc(B.scal_count() * sizeof(double), B.work));
  B.ctl_d = static_cast<int*>(dalloc((size_t)cap * CTL_INTS * sizeof(int), B.work));
  B.scal_h = static_cast<double*>(pinned_take(B.scal_count() * sizeof(double)));
  B.ctl_h = static_cast<int*>(pinned_take((size_t)cap * CTL_INTS * sizeof(int)));
  std::memset(B.ctl_h, 0, (size_t)cap * CTL_INTS * sizeof(int));
  AMG_HIP(hipMemsetAsync(B.ctl_d, 0, (size_t)cap * CTL_INTS * sizeof(int), B.work));
  AMG_HIP(hipMemsetAsync(B.scal_d, 0, B.scal_count() * sizeof(double), B.work));
}

void check_uniform(Batch& B, const Hierarchy& H) {
  const int fp32 = H.p.vcycle_fp32 ? 1 : 0;
  if (B.fp32 < 0) {
    B.fp32 = fp32;
    B.smoother = H.p.smoother;
    B.pre = H.p.pre_sweeps;
    B.post = H.p.post_sweeps;
    B.flexible = H.flexible;
    B.bs = H.p.block_size;
    B.coarse_smoother = H.p.coarse_smoother;
    B.coarse_from = H.p.coarse_from;
    for (int l = 0; l < MAX_LEVELS; ++l) B.stile[l] = smooth_tile(H.p, l);
    return;
  }
  const bool same_coarse = B.coarse_smoother == H.p.coarse_smoother &&
                           (B.coarse_smoother < 0 || B.coarse_from == H.p.coarse_from);
  if (B.fp32 != fp32 || B.smoother != H.p.smoother || !same_coarse || B.pre != H.p.pre_sweeps ||
      B.post != H.p.post_sweeps || B.flexible != H.flexible || B.bs != H.p.block_size)
    fail(AMG_ERR_INVALID_ARG,
         "hierarchies of one batch must share vcycle_fp32, the smoothers, pre/post sweeps, block size and the CG "
         "variant");
  bool same_tiles = true;
  for (int l = 0; l < MAX_LEVELS; ++l) same_tiles = same_tiles && B.stile[l] == smooth_tile(H.p, l);
  if ((tile_sweeps(B.smoother) || tile_sweeps(B.coarse_smoother)) && !same_tiles)
    fail(AMG_ERR_INVALID_ARG, "hierarchies of one batch with a tile smoother must share their smoothing tiles");
}

// The fields of a level's descriptor that come from the hierarchy (matrix,
// transfer, smoother and coarsest-solve data); the vectors are the caller's.
void level_desc(BDesc& d, const Hierarchy& H, int l) {
  const int Lc = (int)H.lev.size() - 1;
  const Level& L = H.lev[l];
  d.srow = L.srow;
  d.soff = L.soff;
  d.scol = L.scol;
  d.sval64 = L.sval;
  d.dg64 = L.dg;
  d.l164 = L.l1;
  d.sval32 = L.sval32;
  d.dg32 = L.dg32;
  d.l132 = L.l1_32;
  d.rowptr = L.rowptr;
  d.colind = L.colind;
  d.vals = L.vals;
  if (l < Lc) {
    d.mptr = L.mptr;
    d.members = L.members;
    d.agg = L.agg;
    d.cinv = L.cinv;
  } else {
    d.Ainv = H.Ainv;
  }
  d.sptr = L.sptr_d;
  d.ncol = L.ncol;
  d.hsf = L.hsf;
  d.hsb = L.hsb;
  d.T = L.T;
  d.hdf = L.hdf;
  d.hdb = L.hdb;
  d.hw = L.hw;
  d.hg = L.hg;
  d.icp = L.icp;
  d.icc = L.icc;
  d.icv64 = L.icv;
  d.icv32 = L.icv32;
  d.ocp = L.ocp;
  d.occ = L.occ;
  d.ocv64 = L.ocv;
  d.ocv32 = L.ocv32;
  d.tcb = L.tcb;
  d.tcol = L.tcol;
  d.tncol = L.tncol;
  d.sm = L.sm;
  d.n = L.n;
  d.nc = L.nc;
  d.nsl = L.nsl;
  d.nL = H.nL;
  d.omega = H.p.omega;
  // entries of at least 8 B each (FP32 value and column) beyond the 256 MB
  // last-level cache: every pass streams them from HBM
  d.nt = (L.scol && (double)L.soff_h[L.nsl] * 8.0 > 256.0 * (1 << 20)) ? 1 : 0;
  d.blk = L.bs;
  d.dinv64 = L.dinv;
  d.dinv32 = L.dinv32;
}

// Allocates the vectors of `slot` for hierarchy H and writes its descriptors.
void bind_slot(Batch& B, int slot, Hierarchy& H) {
  Entry& E = B.ent[slot];
  hipStream_t s = B.work;
  E.ctx.release(s);
  E.bound = nullptr;
  const int R = B.R;
  const int Lc = (int)H.lev.size() - 1;
  if (Lc >= MAX_LEVELS) fail(AMG_ERR_UNSUPPORTED, "too many levels");
  const size_t vb = B.fp32 ? 4 : 8;
  Ctx& C = E.ctx;
  const size_t n0 = (size_t)H.lev[0].n;
  auto carve = [&](Carver& cv) {
    auto vec64 = [&](size_t n) { return static_cast<double*>(cv.take(n * R * sizeof(double))); };
    C.r = vec64(n0);
    C.z = vec64(n0);
    C.p = vec64(n0);
    C.q = vec64(n0);
    C.xs = vec64(n0);
    C.bs = vec64(n0);
    C.rold = H.flexible ? vec64(n0) : nullptr;
    C.partial = static_cast<double*>(cv.take(2 * (size_t)RED_BLOCKS * R * sizeof(double)));
    C.x.assign(Lc + 1, nullptr);
    C.b.assign(Lc + 1, nullptr);
    C.t.assign(Lc + 1, nullptr);
    for (int l = 0; l <= Lc; ++l) {
      const size_t n = (size_t)H.lev[l].n;
      if (l == 0 && !B.fp32) {  // the FP64 cycle works on r and z directly
        C.b[0] = C.r;
        C.x[0] = C.z;
      } else {
        C.x[l] = cv.take(n * R * vb);
        C.b[l] = cv.take(n * R * vb);
      }
      if (l < Lc) C.t[l] = cv.take(n * R * vb);
    }
  };
  Carver sizing;
  carve(sizing);
  C.block = dalloc(sizing.off, s);
  C.bytes = sizing.off;
  Carver cv;
  cv.base = static_cast<char*>(C.block);
  carve(cv);
  for (int l = 0; l < MAX_LEVELS; ++l) {
    BDesc& d = B.desc_h[B.desc_index(slot, l)];
    d = BDesc{};
    if (l > Lc) continue;
    level_desc(d, H, l);
    if (l < Lc) {
      d.xc = C.x[l + 1];
      d.bc = C.b[l + 1];
    }
    d.x = C.x[l];
    d.b = C.b[l];
    d.t = C.t[l];
    d.r = C.r;
    d.z = C.z;
    d.p = C.p;
    d.q = C.q;
    d.rold = C.rold;
    d.xs = C.xs;
    d.bs = C.bs;
    d.partial = C.partial;
    d.scal = B.scal_of(slot);
    d.ctl = B.ctl_d + (size_t)slot * CTL_INTS;
    d.active = 0;
  }
  B.desc_dirty = true;
  E.bound = &H;
  B.dirty = true;
}

// Marks the entry of `slot` active or finished in its descriptors.
void set_active(Batch& B, int slot, int v, hipStream_t s) {
  (void)s;
  for (int l = 0; l < MAX_LEVELS; ++l) B.desc_h[B.desc_index(slot, l)].active = v;
  B.desc_dirty = true;
}

void upload_ctl(Batch& B, hipStream_t s) {
  (void)s;
  B.ctl_dirty = true;
}

// Uploads the host copies changed since the last launch sequence (pinned
// memory, one copy each).  The host changes them only between
// synchronisations, and every change is followed by a flush before the next
// launch on the stream, so the device sees the latest state.
void flush(Batch& B, hipStream_t s) {
  if (B.desc_dirty)
    AMG_HIP(hipMemcpyAsync(B.desc_d, B.desc_h, (size_t)B.cap * MAX_LEVELS * sizeof(BDesc), hipMemcpyHostToDevice,
                           s));
  if (B.ctl_dirty)
    AMG_HIP(hipMemcpyAsync(B.ctl_d, B.ctl_h, (size_t)B.cap * CTL_INTS * sizeof(int), hipMemcpyHostToDevice, s));
  B.desc_dirty = B.ctl_dirty = false;
}

// ------------------------------------------------------------------ launch lists
// Collects the launches of a program and their tables.  Every launch is a
// list of segments, one per entry, each a regular split of a unit range; a
// plan of a single entry launches its (single-segment) launches directly.
struct Builder {
  const Batch& B;
  const bool single;
  std::vector<Item> items;
  std::vector<Launch> L;
  Launch cur;
  int segs = 0;
  Builder(const Batch& b, bool single_entry) : B(b), single(single_entry) {}
  void begin(int op, int level, int kind, int aux = 0, int aux2 = 0, int aux3 = 0) {
    cur = Launch{};
    cur.op = op;
    cur.level = level;
    cur.kind = kind;
    cur.aux = aux;
    cur.aux2 = aux2;
    cur.aux3 = aux3;
    cur.off = items.size();
    segs = 0;
  }
  void add(int d, int lo, int hi, int part, double bytes) {
    items.push_back(Item{d, lo, hi, part});
    cur.bytes += bytes;
  }
  void segment(int d, int lo0, int hi, int ch) {
    if (segs++ == 0) cur.direct = Item{d, lo0, hi, ch};
  }
  void end() {
    cur.nblk = (int)(items.size() - cur.off);
    cur.use_direct = single && segs == 1;
    if (cur.nblk > 0) L.push_back(cur);
  }
  // Fixed-size pieces of [lo0, hi).
  void pieces(int d, int lo0, int hi, int ch, double bytes_per_unit) {
    if (lo0 >= hi) return;
    segment(d, lo0, hi, ch);
    for (int lo = lo0; lo < hi; lo += ch) {
      const int h = std::min(hi, lo + ch);
      add(d, lo, h, 0, bytes_per_unit * (h - lo));
    }
  }
  void pieces(int d, int n, int ch, double bytes_per_unit) { pieces(d, 0, n, ch, bytes_per_unit); }
  // nb contiguous chunks of [0, n), partial index = chunk index; returns nb.
  int chunks(int d, int n, int nb, double bytes_per_unit) {
    const int ch = cdiv(n, nb);
    segment(d, 0, n, ch);
    for (int i = 0; i < nb; ++i) {
      const int lo = std::min(n, i * ch), hi = std::min(n, lo + ch);
      add(d, lo, hi, i, bytes_per_unit * (hi - lo));
    }
    return nb;
  }
  // One item for entry d whose lo carries a partial count (finish kernels).
  void one(int d, int np) {
    segment(d, np, np, 0);
    add(d, np, np, 0, 0.0);
  }
};

inline const Hierarchy& hier(const Batch& B, int slot) { return *B.ent[slot].bound; }
inline int coarsest(const Batch& B, int slot) { return (int)hier(B, slot).lev.size() - 1; }
inline bool sell0(const Batch& B, int slot) { return hier(B, slot).lev[0].scol != nullptr; }
// The outer product (and residual) of CG reads level 0 as SELL-64 slices,
// unless the hierarchy keeps the CSR form for it (spmv_format 1).
inline bool outer_sell(const Batch& B, int slot) { return sell0(B, slot) && hier(B, slot).p.spmv_format == 0; }
// First level cycled by the single-workgroup tail: the first with at most
// tail_rows rows (the coarsest if none).
inline int tail_start(const Batch& B, int slot) {
  const Hierarchy& H = hier(B, slot);
  const int Lc = (int)H.lev.size() - 1;
  for (int l = 0; l < Lc; ++l)
    if (H.lev[l].n <= H.p.tail_rows) return l;
  return Lc;
}

int kind_at(int l, int k) { return l == 0 ? k : AMG_KIND_COARSE_LEVELS; }

// Algorithmic bytes of one pass over slices [s0, s1) of level L: matrix once,
// diagonal, and R x (b read, x read, x written) per row.
double pass_bytes(const Level& L, int s0, int s1, int R, double vb) {
  const double ent = (double)(L.soff_h[s1] - L.soff_h[s0]);
  const double rows = (double)(L.srow_h[s1] - L.srow_h[s0]);
  return ent * (4.0 + vb) + rows * (vb + 3.0 * R * vb) + (s1 - s0) * 8.0;
}

// extra_writes: further R-vectors written per row (the residual variant: 1).
void add_slices(Builder& b, const Batch& B, int slot, int l, int s0, int s1, double extra_writes = 0.0) {
  if (s0 >= s1) return;
  const Level& L = hier(B, slot).lev[l];
  const double vb = B.fp32 ? 4 : 8;
  const int d = B.desc_index(slot, l);
  b.segment(d, s0, s1, SLICES_PB);
  for (int lo = s0; lo < s1; lo += SLICES_PB) {
    const int hi = std::min(s1, lo + SLICES_PB);
    const double rows = (double)(L.srow_h[hi] - L.srow_h[lo]);
    b.add(d, lo, hi, 0, pass_bytes(L, lo, hi, B.R, vb) + extra_writes * rows * B.R * vb);
  }
}

// Colours of the passes of `sweeps` symmetric multicolour Gauss-Seidel sweeps
// (forward, then backward over the colours).  A pass on the colour updated by
// the pass before is left out: rows of one colour depend only on the other
// colours, so it would recompute the same values.
std::vector<int> sgs_passes(int ncol, int sweeps) {
  std::vector<int> q;
  for (int k = 0; k < sweeps; ++k) {
    for (int c = 0; c < ncol; ++c)
      if (q.empty() || q.back() != c) q.push_back(c);
    for (int c = ncol - 1; c >= 0; --c)
      if (q.empty() || q.back() != c) q.push_back(c);
  }
  return q;
}

// Algorithmic bytes of a pass from x = 0 over slices [s0, s1): diagonal, and
// R x (b read, x written) per row.
double pass0_bytes(const Level& L, int s0, int s1, int R, double vb) {
  const double rows = (double)(L.srow_h[s1] - L.srow_h[s0]);
  return rows * (vb + 2.0 * R * vb) + (s1 - s0) * 8.0;
}

// Multicolour smoothing of entry e's level l starts and ends on colour 0 and
// takes more than one pass: the zero fill and the prolongation can skip the
// colour-0 rows (their values are written by the first pass before any read),
// and the last pre-smoothing pass writes the residual of its rows.
bool colour0_shortcuts(const Batch& B, int e, int l) {
  const Level& L = hier(B, e).lev[l];
  return L.sm == AMG_SMOOTHER_MCSGS && L.ncol >= 2 && L.bs == 1;
}

// Smoother of level l of the batch's entries (they share the choice).
int sm_at(const Batch& B, int l) {
  return B.coarse_smoother >= 0 && l >= B.coarse_from ? B.coarse_smoother : B.smoother;
}
// First row after colour 0 (solve order).
int colour0_rows(const Level& L) { return L.srow_h[L.sptr[1]]; }

// Launch limits of the tile sweeps of level l over entries E: the most
// in-tile couplings of a row (W) and of a tile (C), the most wavefront steps
// of a sweep + 1 (S) and the most colours (NC).
struct TileLimits {
  int W = 0, S = 0, C = 0, NC = 0;
};
TileLimits tile_limits(const Batch& B, const std::vector<int>& E, int l) {
  TileLimits t;
  for (int e : E) {
    const Level& L = hier(B, e).lev[l];
    t.W = std::max(t.W, L.hw);
    t.S = std::max(t.S, std::max(L.hdf, L.hdb) + 1);
    t.C = std::max(t.C, L.icmax);
    t.NC = std::max(t.NC, L.tncol);
  }
  return t;
}
// Level l sweeps colour by colour (bounds in one wavefront register).
bool colour_sweeps(const Batch& B, const std::vector<int>& E, int l) {
  return sm_at(B, l) == AMG_SMOOTHER_TILE_MCSGS && tile_limits(B, E, l).NC < 64;
}
// The last pre-smoothing sweep of level l also leaves the in-tile sums of
// the residual in t (register form of the colour-ordered sweep).
bool fused_resid(const Batch& B, const std::vector<int>& E, int l) {
  if (B.pre == 0 || !colour_sweeps(B, E, l)) return false;
  const TileLimits t = tile_limits(B, E, l);
  return tsgs_reg_ok(B.R, hier(B, E[0]).lev[l].T, t.W, std::max(t.C, 1), B.fp32 ? 4 : 8);
}

// `sweeps` smoothing steps on level l; from_zero: the iterate is zero before,
// and (pre-smoothing) each entry's last pass also writes its residual rows.
void build_smooth(Builder& b, const Batch& B, const std::vector<int>& E, int l, int sweeps, bool from_zero) {
  const double vb = B.fp32 ? 4 : 8;
  const int sm = sm_at(B, l);
  if (sm == AMG_SMOOTHER_MCSGS) {
    std::vector<std::vector<int>> seq(E.size());
    size_t len = 0;
    for (size_t i = 0; i < E.size(); ++i) {
      seq[i] = sgs_passes(hier(B, E[i]).lev[l].ncol, sweeps);
      len = std::max(len, seq[i].size());
    }
    for (size_t j = 0; j < len; ++j) {
      const bool zero = from_zero && j == 0;
      // entries whose last pre-smoothing pass this is: the residual variant
      auto last = [&](size_t i) {
        return from_zero && !zero && j + 1 == seq[i].size() && colour0_shortcuts(B, E[i], l);
      };
      bool any_last = false;
      for (size_t i = 0; i < E.size(); ++i) any_last = any_last || (j < seq[i].size() && last(i));
      if (any_last) {
        b.begin(OP_GS_RESID, l, kind_at(l, AMG_KIND_RESTRICT));
        for (size_t i = 0; i < E.size(); ++i) {
          if (j >= seq[i].size() || !last(i)) continue;
          const Level& L = hier(B, E[i]).lev[l];
          const int c = seq[i][j];
          add_slices(b, B, E[i], l, L.sptr[c], L.sptr[c + 1], 1.0);
        }
        b.end();
      }
      // point-based levels (every entry of a batch shares the block size):
      // block passes only, the first one too (the iterate was zero-filled)
      const bool blk = B.bs > 1;
      b.begin(blk ? OP_BGS : zero ? OP_GS0 : OP_GS, l, kind_at(l, zero ? AMG_KIND_OTHER : AMG_KIND_SWEEP));
      for (size_t i = 0; i < E.size(); ++i) {
        if (j >= seq[i].size() || last(i)) continue;
        const int e = E[i];
        const Level& L = hier(B, e).lev[l];
        const int c = seq[i][j];
        if (!zero || blk) {  // a block pass also reads the bs values of its row of the inverse block
          add_slices(b, B, e, l, L.sptr[c], L.sptr[c + 1], blk ? (double)L.bs / B.R : 0.0);
          continue;
        }
        const int s0 = L.sptr[c], s1 = L.sptr[c + 1];
        if (s0 >= s1) continue;
        const int d = B.desc_index(e, l);
        b.segment(d, s0, s1, SLICES_PB);
        for (int lo = s0; lo < s1; lo += SLICES_PB) {
          const int hi = std::min(s1, lo + SLICES_PB);
          b.add(d, lo, hi, 0, pass0_bytes(L, lo, hi, B.R, vb));
        }
      }
      b.end();
    }
  } else if (tile_sweeps(sm)) {
    // per step: t = b - (couplings to other tiles) x, then the in-tile sweeps
    // (from x = 0: src = b, no residual pass); natural or colour order is in
    // the steps of the rows
    for (int k = 0; k < sweeps; ++k) {
      const bool zero = from_zero && k == 0;
      if (!zero) {
        b.begin(OP_RESID_OFF, l, kind_at(l, AMG_KIND_SWEEP));
        for (int e : E) {
          const Level& L = hier(B, e).lev[l];
          // per row the offset, its couplings to other tiles (column, value, gathered x), b read, t written
          b.pieces(B.desc_index(e, l), L.n, 256,  // one row per thread (blocks of 256 threads)
                   4.0 + (double)L.ocn / L.n * (4.0 + vb + B.R * vb) + 2.0 * B.R * vb);
        }
        b.end();
      }
      // LDS layout of the launch: limits over its entries
      const TileLimits tl = tile_limits(B, E, l);
      const int W = tl.W, S = tl.S, C = tl.C, NC = tl.NC;
      const bool emit = from_zero && k + 1 == sweeps && fused_resid(B, E, l);
      if (colour_sweeps(B, E, l))  // colour by colour (at least one coupling slot in LDS)
        b.begin(OP_TSGS, l, kind_at(l, AMG_KIND_SWEEP), (zero ? 1 : 0) | (emit ? 2 : 0), std::max(C, 1),
                NC | (std::min(W, 0x7fff) << 16));
      else  // wavefront steps of the solve order (natural, or colour by colour in each tile)
        b.begin(OP_HSGS, l, kind_at(l, AMG_KIND_SWEEP), zero ? 1 : 0, W | (S << 16), C);
      for (int e : E) {
        const Level& L = hier(B, e).lev[l];
        // in-tile couplings once (value, 16-bit column), per row the coupling
        // offset, two steps, diagonal, source, x read (not from zero) and written
        const double per_tile = (double)L.icn / L.n * L.T * (2.0 + vb) +
                                L.T * (8.0 + vb + B.R * vb + (zero ? 1.0 : 2.0) * B.R * vb);
        b.pieces(B.desc_index(e, l), 0, cdiv(L.n, L.T), 1, per_tile);
      }
      b.end();
    }
  } else {
    for (int k = 0; k < sweeps; ++k) {
      b.begin(OP_RESID, l, kind_at(l, AMG_KIND_SWEEP));
      for (int e : E) add_slices(b, B, e, l, 0, hier(B, e).lev[l].nsl);
      b.end();
      b.begin(OP_JACOBI, l, kind_at(l, AMG_KIND_SWEEP));
      for (int e : E) b.pieces(B.desc_index(e, l), hier(B, e).lev[l].n, ROW_CH, vb + 3.0 * B.R * vb);
      b.end();
    }
  }
}

// z = M r for every entry of S (Sec. 2: V-cycle), level by level over the
// entries that have the level; all coarsest solves in one launch.  convert:
// FP32 cycle with r -> b_0 and x_0 -> z conversions of its own (the CG
// iteration writes b_0 where r is produced and reads x_0 as z).
void build_precond(Builder& b, const Batch& B, const std::vector<int>& S, bool convert) {
  const double vb = B.fp32 ? 4 : 8;
  const int R = B.R;
  int maxLc = 0;  // deepest level cycled by separate launches
  for (int e : S) maxLc = std::max(maxLc, tail_start(B, e));
  if (B.fp32 && convert) {
    b.begin(OP_R2B, 0, AMG_KIND_CG_VEC);
    for (int e : S) b.pieces(B.desc_index(e, 0), hier(B, e).lev[0].n, ROW_CH, 12.0 * R);
    b.end();
  }
  std::vector<std::vector<int>> below(maxLc);
  for (int l = 0; l < maxLc; ++l)
    for (int e : S)
      if (tail_start(B, e) > l) below[l].push_back(e);
  for (int l = 0; l < maxLc; ++l) {
    const std::vector<int>& E = below[l];
    b.begin(OP_ZERO, l, l == 0 ? AMG_KIND_OTHER : AMG_KIND_COARSE_LEVELS);
    for (int e : E) {
      if (tile_sweeps(sm_at(B, l)) && B.pre > 0) continue;  // the first step writes every row
      const Level& L = hier(B, e).lev[l];
      const int r0 = B.pre > 0 && colour0_shortcuts(B, e, l) ? colour0_rows(L) : 0;
      b.pieces(B.desc_index(e, l), r0, L.n, ROW_CH, R * vb);
    }
    b.end();
    build_smooth(b, B, E, l, B.pre, true);
    if (tile_sweeps(sm_at(B, l))) {  // from the compact couplings (in-tile part from the sweep if fused)
      const bool fused = fused_resid(B, E, l);
      b.begin(OP_RESID_TILE, l, kind_at(l, AMG_KIND_RESTRICT), fused ? 1 : 0);
      for (int e : E) {
        const Level& L = hier(B, e).lev[l];
        const double in = fused ? B.R * vb : 4.0 + (double)L.icn / L.n * (2.0 + vb + B.R * vb);
        b.pieces(B.desc_index(e, l), L.n, 256,
                 in + 4.0 + (double)L.ocn / L.n * (4.0 + vb + B.R * vb) + vb + 3.0 * B.R * vb);
      }
      b.end();
    } else {
      b.begin(OP_RESID, l, kind_at(l, AMG_KIND_RESTRICT));
      for (int e : E) {
        const Level& L = hier(B, e).lev[l];
        add_slices(b, B, e, l, B.pre > 0 && colour0_shortcuts(B, e, l) ? L.sptr[1] : 0, L.nsl);
      }
      b.end();
    }
    b.begin(OP_RESTRICT, l, kind_at(l, AMG_KIND_RESTRICT));
    for (int e : E) {
      const Level& L = hier(B, e).lev[l];
      // members and fine residual once, coarse pointers and result once
      const double per_coarse = (double)L.n / std::max(1, L.nc) * (4.0 + R * vb) + 4.0 + R * vb;
      b.pieces(B.desc_index(e, l), L.nc, RESTRICT_CH, per_coarse);
    }
    b.end();
  }
  // Levels from tail_start down: one workgroup per entry (down-leg, then
  // up-leg); the coarsest solves of all entries in between, spread over many
  // workgroups.
  auto tail_leg = [&](int op, bool up) {
    b.begin(op, maxLc, AMG_KIND_COARSE_LEVELS, 0, (B.pre << 8) | B.post);
    for (int e : S) {
      const Hierarchy& H = hier(B, e);
      const int lt = tail_start(B, e), lc = coarsest(B, e);
      if (lt == lc) continue;
      double bytes = 0.0;
      for (int l = lt; l < lc; ++l) {
        const Level& L = H.lev[l];
        const double pass = pass_bytes(L, 0, L.nsl, R, vb);
        const int k = up ? B.post : B.pre;
        const double sweeps = L.sm == AMG_SMOOTHER_MCSGS
                                  ? (double)sgs_passes(L.ncol, k).size() / std::max(1, L.ncol)
                                  : 2.0 * k;
        bytes += up ? sweeps * pass + L.n * (4.0 + 2.0 * R * vb)
                    : (sweeps + 1.0) * pass + L.n * (4.0 + 2.0 * R * vb);
      }
      const int d = B.desc_index(e, lt);
      b.segment(d, lt, lc, 0);
      b.add(d, lt, lc, 0, bytes);
    }
    b.end();
  };
  tail_leg(OP_TAIL, false);
  b.begin(OP_COARSE, maxLc, AMG_KIND_COARSE_LEVELS);
  for (int e : S) {
    const Hierarchy& H = hier(B, e);
    b.pieces(B.desc_index(e, coarsest(B, e)), H.nL, 4, 8.0 * H.nL + 2.0 * R * vb);
  }
  b.end();
  tail_leg(OP_TAIL_UP, true);
  for (int l = maxLc - 1; l >= 0; --l) {
    const std::vector<int>& E = below[l];
    b.begin(OP_PROLONG, l, kind_at(l, AMG_KIND_PROLONG));
    for (int e : E) {
      const Level& L = hier(B, e).lev[l];
      const double per_row = 4.0 + 2.0 * R * vb + R * vb * (double)L.nc / L.n;
      const int r0 = B.post > 0 && colour0_shortcuts(B, e, l) ? colour0_rows(L) : 0;
      b.pieces(B.desc_index(e, l), r0, L.n, ROW_CH, per_row);
    }
    b.end();
    build_smooth(b, B, E, l, B.post, false);
  }
  if (B.fp32 && convert) {
    b.begin(OP_X2Z, 0, AMG_KIND_CG_VEC);
    for (int e : S) b.pieces(B.desc_index(e, 0), hier(B, e).lev[0].n, ROW_CH, 12.0 * R);
    b.end();
  }
}

// out = b - A x with partials (which: 0 -> r, 1 -> q); returns per-slot partial counts.
std::vector<int> build_resid_dot(Builder& b, const Batch& B, const std::vector<int>& S, int which, int kind) {
  std::vector<int> np(S.size());
  const int R = B.R;
  b.begin(OP_RESID_DOT, 0, kind, which);
  for (size_t i = 0; i < S.size(); ++i) {
    const int e = S[i];
    if (!outer_sell(B, e)) continue;
    const Level& L = hier(B, e).lev[0];
    const double per_slice = ((double)L.soff_h[L.nsl] * 12.0 + (double)L.n * (8.0 + 24.0 * R)) / L.nsl + 8.0;
    np[i] = b.chunks(B.desc_index(e, 0), L.nsl, red_blocks_slices(L.nsl), per_slice);
  }
  b.end();
  for (int sub = 4; sub <= 64; sub *= 2) {
    b.begin(OP_RESID_DOT_CSR, 0, kind, which, sub);
    for (size_t i = 0; i < S.size(); ++i) {
      const int e = S[i];
      const Level& L = hier(B, e).lev[0];
      if (outer_sell(B, e) || L.sub != sub) continue;
      const double per_row = (double)L.nnz / L.n * 12.0 + 4.0 + 24.0 * R;
      np[i] = b.chunks(B.desc_index(e, 0), L.n, red_blocks_rows(L.n), per_row);
    }
    b.end();
  }
  return np;
}

void build_finish(Builder& b, const Batch& B, const std::vector<int>& S, const std::vector<int>& np, int op,
                  int slot_ = 0) {
  b.begin(OP_FINISH, 0, KIND_NONE, op, slot_);
  for (size_t i = 0; i < S.size(); ++i) b.one(B.desc_index(S[i], 0), np[i]);
  b.end();
}

// One CG iteration (Sec. 2): z = M r, beta, p, q = A p, alpha, x and r, ||r||^2.
void build_iter(Builder& b, const Batch& B, const std::vector<int>& S, size_t* precond_end) {
  const int R = B.R;
  const double zb = B.fp32 ? 4.0 : 8.0;  // bytes per value of z (read as the FP32 x_0)
  build_precond(b, B, S, false);
  *precond_end = b.L.size();
  std::vector<int> nr(S.size());
  b.begin(OP_DOTS_RZ, 0, AMG_KIND_CG_VEC, B.fp32);
  for (size_t i = 0; i < S.size(); ++i) {
    const int n = hier(B, S[i]).lev[0].n;
    nr[i] = b.chunks(B.desc_index(S[i], 0), n, red_blocks_rows(n), (zb + (B.flexible ? 16.0 : 8.0)) * R);
  }
  b.end();
  build_finish(b, B, S, nr, B.flexible ? FIN_BETA_FCG : FIN_BETA_PCG);
  b.begin(OP_UPDATE_P, 0, AMG_KIND_CG_VEC, B.fp32);
  for (int e : S) b.pieces(B.desc_index(e, 0), hier(B, e).lev[0].n, ROW_CH, (zb + 16.0) * R);
  b.end();
  std::vector<int> ns(S.size());
  b.begin(OP_SPMV_DOT, 0, AMG_KIND_SPMV_F64);
  for (size_t i = 0; i < S.size(); ++i) {
    const int e = S[i];
    if (!outer_sell(B, e)) continue;
    const Level& L = hier(B, e).lev[0];
    const double per_slice = ((double)L.soff_h[L.nsl] * 12.0 + (double)L.n * (8.0 + 16.0 * R)) / L.nsl + 8.0;
    ns[i] = b.chunks(B.desc_index(e, 0), L.nsl, red_blocks_slices(L.nsl), per_slice);
  }
  b.end();
  for (int sub = 4; sub <= 64; sub *= 2) {
    b.begin(OP_SPMV_DOT_CSR, 0, AMG_KIND_SPMV_F64, sub);
    for (size_t i = 0; i < S.size(); ++i) {
      const int e = S[i];
      const Level& L = hier(B, e).lev[0];
      if (outer_sell(B, e) || L.sub != sub) continue;
      const double per_row = (double)L.nnz / L.n * 12.0 + 4.0 + 16.0 * R;
      ns[i] = b.chunks(B.desc_index(e, 0), L.n, red_blocks_rows(L.n), per_row);
    }
    b.end();
  }
  build_finish(b, B, S, ns, FIN_ALPHA);
  b.begin(OP_UPDATE_XR, 0, AMG_KIND_CG_VEC, B.fp32);
  for (size_t i = 0; i < S.size(); ++i) {
    const int n = hier(B, S[i]).lev[0].n;
    nr[i] = b.chunks(B.desc_index(S[i], 0), n, red_blocks_rows(n),
                     ((B.flexible ? 56.0 : 48.0) + (B.fp32 ? 4.0 : 0.0)) * R);
  }
  b.end();
  build_finish(b, B, S, nr, FIN_STORE, S_RR);
}

// r = b - A x, ||r_0||^2 and the CG scalars of a starting entry.
void build_prologue(Builder& b, const Batch& B, const std::vector<int>& S) {
  if (B.flexible) {
    b.begin(OP_VZERO_ROLD, 0, AMG_KIND_CG_VEC);
    for (int e : S) b.pieces(B.desc_index(e, 0), hier(B, e).lev[0].n, ROW_CH, 8.0 * B.R);
    b.end();
  }
  // r = b - A x, and in the FP32 cycle also its right-hand side (float) r
  const std::vector<int> np = build_resid_dot(b, B, S, B.fp32 ? 2 : 0, AMG_KIND_CG_VEC);
  build_finish(b, B, S, np, FIN_INIT);
}

// ||b - A x||^2 and ||b||^2 of finishing entries.
void build_final(Builder& b, const Batch& B, const std::vector<int>& S) {
  const std::vector<int> np = build_resid_dot(b, B, S, 1, AMG_KIND_CG_VEC);
  build_finish(b, B, S, np, FIN_STORE, S_TMP);
  std::vector<int> nb(S.size());
  b.begin(OP_DOT_BB, 0, AMG_KIND_CG_VEC);
  for (size_t i = 0; i < S.size(); ++i) {
    const int n = hier(B, S[i]).lev[0].n;
    nb[i] = b.chunks(B.desc_index(S[i], 0), n, red_blocks_rows(n), 8.0 * B.R);
  }
  b.end();
  build_finish(b, B, S, nb, FIN_STORE, S_TMP2);
}

void upload_plan(Plan& P, Builder& b, hipStream_t s) {
  P.drop_graph();
  P.L = std::move(b.L);
  // Direct launches (the plans of one entry) take their ranges from the block
  // index: the table is uploaded only if some launch reads it (a plan of a
  // 256^3 system holds about 12 MB of items, which would cost a staged copy
  // from pageable memory on every new hierarchy).
  bool table = false;
  for (const Launch& L : P.L) table = table || !L.use_direct;
  if (!table) return;
  if (b.items.size() > P.cap) {
    if (P.tab_d) dfree(P.tab_d, s);
    P.cap = std::max(b.items.size(), (size_t)1024);
    P.tab_d = static_cast<Item*>(dalloc(P.cap * sizeof(Item), s));
  }
  if (!b.items.empty())
    AMG_HIP(hipMemcpyAsync(P.tab_d, b.items.data(), b.items.size() * sizeof(Item), hipMemcpyHostToDevice, s));
}

// Plans over at least this many rows x right-hand sides are launched
// directly: their kernels outlast the host's launch calls, so a graph only
// adds its capture and instantiation (measured on lognormal systems: graphs
// 9% faster at 96^3, launches 5% faster at 128^3 and equal at 256^3).
constexpr double GRAPH_MAX_ROWS = 1.5e6;

void run_plan(Batch& B, Plan& P, hipStream_t s, bool graph) {
  flush(B, s);
  if (!graph || !B.use_graphs || g_timing_mask_for_graphs() != 0 || P.rows * B.R >= GRAPH_MAX_ROWS) {
    issue_launches(P.L, 0, P.L.size(), P.tab_d, B.desc_d, B.desc_h, B.R, B.fp32, s);
    return;
  }
  if (!P.exec) {
    hipGraph_t g = nullptr;
    AMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      issue_launches(P.L, 0, P.L.size(), P.tab_d, B.desc_d, B.desc_h, B.R, B.fp32, s);
    } catch (...) {
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    AMG_HIP(hipStreamEndCapture(s, &g));
    hipError_t e = hipGraphInstantiate(&P.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    AMG_HIP(e);
  }
  AMG_HIP(hipGraphLaunch(P.exec, s));
}

void read_scal(Batch& B) {
  AMG_HIP(hipMemcpyAsync(B.scal_h, B.scal_d, B.scal_count() * sizeof(double), hipMemcpyDeviceToHost, B.work));
  sync_stream(B.work);
}

// ------------------------------------------------------------------ entry life cycle
void start_entry(Batch& B, int slot, Hierarchy& H, const double* b, double* x, double rtol, int maxit, int64_t tag,
                 double* res_hist, double* iter_hist, hipStream_t us) {
  check_uniform(B, H);
  Entry& E = B.ent[slot];
  if (E.bound != &H) bind_slot(B, slot, H);
  hipStream_t s = B.work;
  E.used = true;
  E.complete = false;
  E.started = false;
  E.b_user = b;
  E.x_user = x;
  E.rtol = rtol;
  E.maxit = maxit;
  E.tag = tag;
  E.res_hist = res_hist;
  E.iter_hist = iter_hist;
  for (int k = 0; k < MAX_RHS; ++k) {
    E.r0[k] = 0.0;
    E.rel[k] = 1.0;
    E.it[k] = 0;
    E.st[k] = AMG_ERR_NOT_CONVERGED;
    E.done[k] = false;
  }
  int* c = B.ctl_h + (size_t)slot * CTL_INTS;
  std::memset(c, 0, CTL_INTS * sizeof(int));
  c[0] = 1;
  for (int k = 0; k < B.R; ++k) c[1 + k] = maxit == 0 ? 1 : 0;
  AMG_HIP(hipEventRecord(B.ev, us));
  AMG_HIP(hipStreamWaitEvent(s, B.ev, 0));
  AMG_HIP(hipMemsetAsync(B.scal_of(slot), 0, (size_t)B.R * S_COUNT * sizeof(double), s));
  upload_ctl(B, s);
  set_active(B, slot, 1, s);
  const Level& L0 = H.lev[0];
  gather_rhs(L0.n, B.R, L0.perm, b, E.ctx.bs, s);
  gather_rhs(L0.n, B.R, L0.perm, x, E.ctx.xs, s);
  if (iter_hist) scatter_rhs(L0.n, 1, L0.perm, E.ctx.xs, iter_hist, s);
  if (res_hist) res_hist[0] = 1.0;
  if (std::find(B.iter.slots.begin(), B.iter.slots.end(), slot) == B.iter.slots.end()) B.dirty = true;
  B.pending.push_back(slot);
  E.t0 = now_ms();
}

// True residual, copy-out and result record of the finishing slots.
void finalise(Batch& B, const std::vector<int>& S) {
  if (S.empty()) return;
  hipStream_t s = B.work;
  Builder b(B, S.size() == 1);
  build_final(b, B, S);
  upload_plan(B.tmp, b, s);
  run_plan(B, B.tmp, s, false);
  for (int e : S) {
    const Entry& E = B.ent[e];
    const Level& L0 = E.bound->lev[0];
    scatter_rhs(L0.n, B.R, L0.perm, E.ctx.xs, E.x_user, s);
  }
  read_scal(B);
  const double t = now_ms();
  for (int e : S) {
    Entry& E = B.ent[e];
    Result res;
    res.tag = E.tag;
    res.status = AMG_OK;
    for (int k = 0; k < B.R; ++k) {
      const double* sc = B.scal_h_of(e) + k * S_COUNT;
      const double rn = std::sqrt(sc[S_TMP]), bn = std::sqrt(sc[S_TMP2]);
      amg_solve_info& in = res.info[k];
      in.iterations = E.it[k];
      in.converged = E.st[k] == AMG_OK ? 1 : 0;
      in.levels = (int)E.bound->lev.size();
      in.rel_residual = E.rel[k];
      in.true_rel_residual = bn > 0.0 ? rn / bn : 0.0;
      in.setup_ms = E.bound->setup_ms;
      in.solve_ms = t - E.t0;
      if (E.st[k] == AMG_ERR_BREAKDOWN)
        res.status = AMG_ERR_BREAKDOWN;
      else if (E.st[k] != AMG_OK && res.status == AMG_OK)
        res.status = E.st[k];
    }
    B.results.push_back(res);
    B.ctl_h[(size_t)e * CTL_INTS] = 0;
    set_active(B, e, 0, s);
    E.used = false;
    E.complete = false;
    if (!B.single) {  // a batch slot gives its memory back; the single context keeps it
      E.ctx.release(s);
      E.bound = nullptr;
    }
  }
  upload_ctl(B, s);
}

void finish_rhs(Entry& E, int k, amg_status st, int* c) {
  E.done[k] = true;
  E.st[k] = st;
  c[1 + k] = 1;
}

// One CG iteration of every active entry.
void step(Batch& B) {
  hipStream_t s = B.work;
  if (!B.pending.empty()) {
    Builder b(B, B.pending.size() == 1);
    build_prologue(b, B, B.pending);
    upload_plan(B.tmp, b, s);
    run_plan(B, B.tmp, s, false);
    B.pending.clear();
  }
  std::vector<int> act;
  double act_rows = 0.0;
  for (int e = 0; e < B.cap; ++e)
    if (B.ent[e].used && !B.ent[e].complete) {
      act.push_back(e);
      act_rows += B.ent[e].bound->lev[0].n;
    }
  if (act.empty()) return;
  bool rebuild = B.dirty || B.iter.L.empty() || (!B.deferred && act_rows < 0.7 * B.iter.rows);
  if (!rebuild)
    for (int e : act)
      if (std::find(B.iter.slots.begin(), B.iter.slots.end(), e) == B.iter.slots.end()) rebuild = true;
  if (rebuild) {
    Builder b(B, act.size() == 1);
    build_iter(b, B, act, &B.iter.precond_end);
    const size_t pe = B.iter.precond_end;
    upload_plan(B.iter, b, s);
    B.iter.precond_end = pe;
    B.iter.slots = act;
    B.iter.rows = act_rows;
    B.dirty = false;
  }
  run_plan(B, B.iter, s, B.iter.runs >= 1);
  B.iter.runs++;
  read_scal(B);
  std::vector<int> fin;
  bool ctl_changed = false;
  for (int e : act) {
    Entry& E = B.ent[e];
    int* c = B.ctl_h + (size_t)e * CTL_INTS;
    const double* sc0 = B.scal_h_of(e);
    bool all = true;
    for (int k = 0; k < B.R; ++k) {
      if (E.done[k]) continue;
      const double* sc = sc0 + k * S_COUNT;
      if (!E.started) {
        E.r0[k] = std::sqrt(sc[S_R0]);
        if (E.r0[k] == 0.0) {
          E.rel[k] = 0.0;
          finish_rhs(E, k, AMG_OK, c);
          ctl_changed = true;
          continue;
        }
        if (E.maxit == 0) {
          finish_rhs(E, k, AMG_ERR_NOT_CONVERGED, c);
          continue;
        }
      }
      if (sc[S_FLAG] != 0.0) {
        finish_rhs(E, k, AMG_ERR_BREAKDOWN, c);
        ctl_changed = true;
        continue;
      }
      E.it[k] += 1;
      E.rel[k] = std::sqrt(sc[S_RR]) / E.r0[k];
      if (E.res_hist) E.res_hist[E.it[k]] = E.rel[k];
      if (E.rel[k] <= E.rtol) {
        finish_rhs(E, k, AMG_OK, c);
        ctl_changed = true;
      } else if (E.it[k] >= E.maxit) {
        finish_rhs(E, k, AMG_ERR_NOT_CONVERGED, c);
        ctl_changed = true;
      }
    }
    E.started = true;
    if (E.iter_hist) {
      const Level& L0 = E.bound->lev[0];
      scatter_rhs(L0.n, 1, L0.perm, E.ctx.xs, E.iter_hist + (size_t)E.it[0] * L0.n, s);
    }
    for (int k = 0; k < B.R; ++k) all = all && E.done[k];
    if (all) {
      E.complete = true;
      fin.push_back(e);
    }
  }
  if (!fin.empty() && !B.deferred) {
    finalise(B, fin);
  } else {
    for (int e : fin) set_active(B, e, 0, s);
    if (ctl_changed) upload_ctl(B, s);
  }
}

void batch_release(Batch& B) {
  if (B.work) (void)sync_stream_nothrow(B.work);
  hipStream_t s = B.work;
  B.iter.drop_graph();
  B.tmp.drop_graph();
  for (auto& E : B.ent) E.ctx.release(s);
  if (B.iter.tab_d) dfree(B.iter.tab_d, s);
  if (B.tmp.tab_d) dfree(B.tmp.tab_d, s);
  if (B.papply.tab_d) dfree(B.papply.tab_d, s);
  B.papply.tab_d = nullptr;
  if (B.desc_d) dfree(B.desc_d, s);
  if (B.scal_d) dfree(B.scal_d, s);
  if (B.ctl_d) dfree(B.ctl_d, s);
  B.iter.tab_d = B.tmp.tab_d = nullptr;
  B.desc_d = nullptr;
  B.scal_d = nullptr;
  B.ctl_d = nullptr;
  if (s) (void)sync_stream_nothrow(s);
  pinned_give(B.desc_h, (size_t)B.cap * MAX_LEVELS * sizeof(BDesc));
  B.desc_h = nullptr;
  pinned_give(B.scal_h, B.scal_count() * sizeof(double));
  pinned_give(B.ctl_h, (size_t)B.cap * CTL_INTS * sizeof(int));
  B.scal_h = nullptr;
  B.ctl_h = nullptr;
  event_give(B.ev);
  B.ev = nullptr;
  stream_give(s);
  B.work = nullptr;
}

Batch& single_of(Hierarchy& H) {
  if (!H.single) {
    Batch* B = new Batch();
    B->single = true;
    try {
      batch_init(*B, 1, 1, H.p.use_graphs);
      check_uniform(*B, H);
      bind_slot(*B, 0, H);
    } catch (...) {
      batch_release(*B);
      delete B;
      throw;
    }
    H.single = B;
  }
  return *H.single;
}

}  // namespace

void batch_destroy(Batch* B) {
  if (!B) return;
  batch_release(*B);
  delete B;
}

// ------------------------------------------------------------------ entry points
amg_status pcg_run(Hierarchy& H, const double* b, double* x, double rtol, int maxit, amg_solve_info* info,
                   double* res_hist, double* iter_hist, hipStream_t us) {
  Batch& B = single_of(H);
  B.results.clear();
  B.pending.clear();
  start_entry(B, 0, H, b, x, rtol, maxit, 0, res_hist, iter_hist, us);
  while (B.results.empty()) step(B);
  const Result res = B.results.back();
  B.results.clear();
  AMG_HIP(hipEventRecord(B.ev, B.work));
  AMG_HIP(hipStreamWaitEvent(us, B.ev, 0));
  if (info) *info = res.info[0];
  if (res.status == AMG_ERR_NOT_CONVERGED) set_error("maximum number of iterations reached");
  if (res.status == AMG_ERR_BREAKDOWN) set_error("CG breakdown (p^T A p <= 0 or r^T z <= 0)");
  return res.status;
}

void precond_run(Hierarchy& H, const double* r, double* z, hipStream_t us) {
  Batch& B = single_of(H);
  hipStream_t s = B.work;
  if (B.papply.L.empty()) {
    Builder b(B, true);
    build_precond(b, B, {0}, true);
    upload_plan(B.papply, b, s);
  }
  sync_stream(s);  // descriptors and tables are written on the work stream
  flush(B, us);
  const Level& L0 = H.lev[0];
  const Entry& E = B.ent[0];
  gather_rhs(L0.n, 1, L0.perm, r, E.ctx.r, us);
  issue_launches(B.papply.L, 0, B.papply.L.size(), B.papply.tab_d, B.desc_d, B.desc_h, 1, B.fp32, us);
  scatter_rhs(L0.n, 1, L0.perm, E.ctx.z, z, us);
  if (!H.apply_done) AMG_HIP(hipEventCreateWithFlags(&H.apply_done, hipEventDisableTiming));
  AMG_HIP(hipEventRecord(H.apply_done, us));
}

// BiCGSTAB (van der Vorst; the outer solver of Sec. 5) with right
// preconditioning by the V-cycle of the hierarchy's solve context, in FP64 on
// level-0 vectors in solve order.  The preconditioner reads the context's r
// and writes its z; the direction p and then s are written into r, the
// products M p and M s are consumed from z before the next application.  The
// scalars stay on the device (the finish kernels compute alpha, omega, beta
// and the stop flags); the host reads them once per iteration.
amg_status bicgstab_run(Hierarchy& H, const double* b, double* x, double rtol, int maxit, amg_solve_info* info,
                        int* half_step, double* res_hist, double* iter_hist, hipStream_t us) {
  Batch& B = single_of(H);
  hipStream_t s = B.work;
  const double t0 = now_ms();
  if (B.papply.L.empty()) {
    Builder bl(B, true);
    build_precond(bl, B, {0}, true);
    upload_plan(B.papply, bl, s);
  }
  const Level& L0 = H.lev[0];
  const int n = L0.n;
  const Ctx& C = B.ent[0].ctx;
  const BDesc d0 = B.desc_h[B.desc_index(0, 0)];
  AMG_HIP(hipEventRecord(B.ev, us));
  AMG_HIP(hipStreamWaitEvent(s, B.ev, 0));
  flush(B, s);
  // r, r~, p, v, t, the partial sums and the scalars
  Carver sizing;
  for (int k = 0; k < 5; ++k) sizing.take((size_t)n * sizeof(double));
  sizing.take(2 * (size_t)RED_BLOCKS * sizeof(double));
  sizing.take(BS_COUNT * sizeof(double));
  struct Owned {
    void* blk = nullptr;
    double* host = nullptr;
    hipStream_t s;
    ~Owned() {
      if (blk) dfree(blk, s);
      pinned_give(host, BS_COUNT * sizeof(double));
    }
  } own;
  own.s = s;
  own.blk = dalloc(sizing.off, s);
  own.host = static_cast<double*>(pinned_take(BS_COUNT * sizeof(double)));
  Carver cv;
  cv.base = static_cast<char*>(own.blk);
  auto vec = [&] { return static_cast<double*>(cv.take((size_t)n * sizeof(double))); };
  double *r = vec(), *rt = vec(), *p = vec(), *v = vec(), *t = vec();
  double* part = static_cast<double*>(cv.take(2 * (size_t)RED_BLOCKS * sizeof(double)));
  double* sc = static_cast<double*>(cv.take(BS_COUNT * sizeof(double)));
  double* sh = own.host;
  // algorithmic bytes of y = A x (+ c read, + w read)
  const double mat = L0.scol ? (double)L0.soff_h[L0.nsl] * 12.0 + 8.0 * n : (double)L0.nnz * 12.0 + 4.0 * (n + 1);
  auto spmv = [&](const double* xin, const double* c, double* y, const double* w) {
    return bcg_spmv(d0, L0.sub, xin, c, y, w, part, mat + n * (16.0 + (c ? 8.0 : 0.0) + (w ? 8.0 : 0.0)), s);
  };
  auto precond = [&] { issue_launches(B.papply.L, 0, B.papply.L.size(), B.papply.tab_d, B.desc_d, B.desc_h, 1, B.fp32, s); };
  auto read = [&] {
    AMG_HIP(hipMemcpyAsync(sh, sc, BS_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    sync_stream(s);
  };
  gather_rhs(n, 1, L0.perm, b, C.bs, s);
  gather_rhs(n, 1, L0.perm, x, C.xs, s);
  if (iter_hist) scatter_rhs(n, 1, L0.perm, C.xs, iter_hist, s);
  if (res_hist) res_hist[0] = 1.0;
  int nb = spmv(C.xs, C.bs, r, nullptr);
  bcg_finish(BF_INIT, nb, part, sc, 0.0, s);
  bcg_dir(n, r, v, p, C.r, rt, sc, 1, s);
  read();
  const double r0 = std::sqrt(sh[BS_RR0]);
  const double tol2 = (rtol * r0) * (rtol * r0);
  amg_status st = AMG_ERR_NOT_CONVERGED;
  int it = 0, half = 0;
  double rel = r0 == 0.0 ? 0.0 : 1.0;
  if (r0 == 0.0) st = AMG_OK;
  for (int k = 1; st == AMG_ERR_NOT_CONVERGED && k <= maxit; ++k) {
    precond();  // z = M p
    nb = spmv(C.z, nullptr, v, rt);
    bcg_finish(BF_ALPHA, nb, part, sc, tol2, s);
    nb = bcg_half(n, r, v, C.z, C.xs, C.r, sc, part, s);
    bcg_finish(BF_S, nb, part, sc, tol2, s);
    precond();  // z = M s
    nb = spmv(C.z, nullptr, t, C.r);
    bcg_finish(BF_OMEGA, nb, part, sc, tol2, s);
    nb = bcg_full(n, C.r, t, C.z, rt, C.xs, r, sc, part, s);
    bcg_finish(BF_BETA, nb, part, sc, tol2, s);
    bcg_dir(n, r, v, p, C.r, rt, sc, 0, s);
    read();
    // a breakdown at beta comes after iteration k is complete (as in the
    // oracle, it counts and is recorded); earlier ones leave it uncounted
    if (sh[BS_FLAG] != 0.0 && sh[BS_FLAG] != 3.0) {
      st = AMG_ERR_BREAKDOWN;
      break;
    }
    it = k;
    if (iter_hist) scatter_rhs(n, 1, L0.perm, C.xs, iter_hist + (size_t)k * n, s);
    if (sh[BS_HALF] != 0.0) {
      half = 1;
      rel = std::sqrt(sh[BS_SS]) / r0;
      st = AMG_OK;
    } else {
      rel = std::sqrt(sh[BS_RR]) / r0;
      if (sh[BS_RR] <= tol2)
        st = AMG_OK;
      else if (sh[BS_FLAG] != 0.0)
        st = AMG_ERR_BREAKDOWN;
    }
    if (res_hist) res_hist[k] = rel;
  }
  nb = spmv(C.xs, C.bs, t, nullptr);
  bcg_finish(BF_TRUE, nb, part, sc, 0.0, s);
  nb = bcg_norm2(n, C.bs, part, s);
  bcg_finish(BF_BB, nb, part, sc, 0.0, s);
  scatter_rhs(n, 1, L0.perm, C.xs, x, s);
  read();
  if (info) {
    info->iterations = it;
    info->converged = st == AMG_OK ? 1 : 0;
    info->levels = (int)H.lev.size();
    info->rel_residual = rel;
    info->true_rel_residual = sh[BS_TMP2] > 0.0 ? std::sqrt(sh[BS_TMP]) / std::sqrt(sh[BS_TMP2]) : 0.0;
    info->setup_ms = H.setup_ms;
    info->solve_ms = now_ms() - t0;
  }
  if (half_step) *half_step = half;
  AMG_HIP(hipEventRecord(B.ev, s));
  AMG_HIP(hipStreamWaitEvent(us, B.ev, 0));
  if (st == AMG_ERR_NOT_CONVERGED) set_error("maximum number of iterations reached");
  if (st == AMG_ERR_BREAKDOWN) set_error("BiCGSTAB breakdown (r~.v, t.t, omega or r~.r zero or not finite)");
  return st;
}

amg_status pcg_batched_run(Hierarchy* const* hs, int nsys, int nrhs, const double* const* b, double* const* x,
                           double rtol, int maxit, amg_solve_info* info, hipStream_t us) {
  Batch B;
  amg_status worst = AMG_OK;
  try {
    batch_init(B, nrhs, nsys, hs[0]->p.use_graphs);
    B.deferred = true;
    for (int i = 0; i < nsys; ++i) start_entry(B, i, *hs[i], b[i], x[i], rtol, maxit, i, nullptr, nullptr, us);
    auto running = [&] {
      for (const Entry& E : B.ent)
        if (E.used && !E.complete) return true;
      return false;
    };
    while (running()) step(B);
    std::vector<int> all(nsys);
    for (int i = 0; i < nsys; ++i) {
      all[i] = i;
      set_active(B, i, 1, B.work);
    }
    finalise(B, all);
    for (const Result& r : B.results) {
      if (info)
        for (int k = 0; k < nrhs; ++k) info[(size_t)r.tag * nrhs + k] = r.info[k];
      if (r.status == AMG_ERR_BREAKDOWN)
        worst = AMG_ERR_BREAKDOWN;
      else if (r.status != AMG_OK && worst == AMG_OK)
        worst = r.status;
    }
    AMG_HIP(hipEventRecord(B.ev, B.work));
    AMG_HIP(hipStreamWaitEvent(us, B.ev, 0));
  } catch (...) {
    batch_release(B);
    throw;
  }
  batch_release(B);
  if (worst == AMG_ERR_NOT_CONVERGED) set_error("maximum number of iterations reached for some system");
  if (worst == AMG_ERR_BREAKDOWN) set_error("CG breakdown in some system");
  return worst;
}

// ------------------------------------------------------------------ continuous batching
Batch* batch_new(int R, int cap, int use_graphs) {
  Batch* B = new Batch();
  try {
    batch_init(*B, R, cap, use_graphs);
  } catch (...) {
    batch_release(*B);
    delete B;
    throw;
  }
  return B;
}

int batch_submit(Batch& B, Hierarchy& H, const double* b, double* x, double rtol, int maxit, int64_t tag,
                 hipStream_t us) {
  int slot = -1;
  for (int e = 0; e < B.cap && slot < 0; ++e)
    if (!B.ent[e].used) slot = e;
  if (slot < 0) fail(AMG_ERR_INVALID_ARG, "batch is full");
  start_entry(B, slot, H, b, x, rtol, maxit, tag, nullptr, nullptr, us);
  return slot;
}

void batch_step(Batch& B, int iterations) {
  for (int i = 0; i < iterations; ++i) step(B);
}

int batch_active(const Batch& B) {
  int a = 0;
  for (const Entry& E : B.ent) a += E.used ? 1 : 0;
  return a;
}

int batch_poll(Batch& B, int64_t* tags, amg_status* status, amg_solve_info* info, int cap) {
  const int n = std::min<int>(cap, (int)B.results.size());
  for (int i = 0; i < n; ++i) {
    const Result& r = B.results[i];
    if (tags) tags[i] = r.tag;
    if (status) status[i] = r.status;
    if (info)
      for (int k = 0; k < B.R; ++k) info[(size_t)i * B.R + k] = r.info[k];
  }
  B.results.erase(B.results.begin(), B.results.begin() + n);
  return n;
}

size_t batch_entry_bytes(const Batch& B) {
  size_t s = 0;
  for (const Entry& E : B.ent) s += E.ctx.bytes;
  return s;
}

// ------------------------------------------------------------------ fixed scratch
// amg_precond_apply_noalloc takes the V-cycle's vectors (level-0 r and z in
// solve order; per level the iterate, right-hand side and residual) from this
// file-scope array instead of the allocator.  Each device that the library
// runs on holds its own copy until the process ends.  In host code `scratch`
// is only the host-side name of the symbol: its device address comes from
// hipGetSymbolAddress, once per device (with that device current), and only
// that address is handed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device: device address of `scratch`

void* scratch_device_ptr() {
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    AMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(AMG_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// The vectors of one V-cycle application, laid out as in a solve context of
// one right-hand side (the FP64 cycle works on r and z directly at level 0).
struct CycleVecs {
  double *r = nullptr, *z = nullptr;
  void *x[MAX_LEVELS] = {}, *b[MAX_LEVELS] = {}, *t[MAX_LEVELS] = {};
};

void carve_cycle(const Hierarchy& H, bool fp32, Carver& cv, CycleVecs& v) {
  const int Lc = (int)H.lev.size() - 1;
  const size_t vb = fp32 ? 4 : 8;
  const size_t n0 = (size_t)H.lev[0].n;
  v.r = static_cast<double*>(cv.take(n0 * sizeof(double)));
  v.z = static_cast<double*>(cv.take(n0 * sizeof(double)));
  for (int l = 0; l <= Lc; ++l) {
    const size_t n = (size_t)H.lev[l].n;
    if (l == 0 && !fp32) {
      v.b[0] = v.r;
      v.x[0] = v.z;
    } else {
      v.x[l] = cv.take(n * vb);
      v.b[l] = cv.take(n * vb);
    }
    v.t[l] = l < Lc ? cv.take(n * vb) : nullptr;
  }
}
}  // namespace

size_t precond_noalloc_bytes(const Hierarchy& H) {
  Carver sizing;
  CycleVecs v;
  carve_cycle(H, H.p.vcycle_fp32 != 0, sizing, v);
  return sizing.off;
}

size_t precond_noalloc_capacity() { return NOALLOC_SCRATCH_BYTES; }

void precond_noalloc_run(Hierarchy& H, const double* r, double* z, hipStream_t us) {
  const int Lc = (int)H.lev.size() - 1;
  if (Lc >= MAX_LEVELS) fail(AMG_ERR_UNSUPPORTED, "too many levels");
  const size_t need = precond_noalloc_bytes(H);
  if (need > NOALLOC_SCRATCH_BYTES)
    fail(AMG_ERR_UNSUPPORTED, "the V-cycle of this hierarchy needs " + std::to_string(need) +
                                  " bytes of vectors, more than the fixed scratch array of " +
                                  std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes");
  // A host-side description of a one-entry batch: it only feeds the launch
  // builder (no device memory, stream or event of its own).
  Batch B;
  B.R = 1;
  B.cap = 1;
  B.single = true;
  B.ent.resize(1);
  B.ent[0].bound = &H;
  check_uniform(B, H);
  if (tail_start(B, 0) != Lc)
    fail(AMG_ERR_UNSUPPORTED, "amg_precond_apply_noalloc does not run the one-workgroup tail (tail_rows > 0)");
  Carver cv;
  cv.base = static_cast<char*>(scratch_device_ptr());
  CycleVecs v;
  carve_cycle(H, B.fp32 != 0, cv, v);
  BDesc desc[MAX_LEVELS];
  for (int l = 0; l <= Lc; ++l) {
    BDesc& d = desc[l];
    d = BDesc{};
    level_desc(d, H, l);
    d.x = v.x[l];
    d.b = v.b[l];
    d.t = v.t[l];
    if (l < Lc) {
      d.xc = v.x[l + 1];
      d.bc = v.b[l + 1];
    }
    d.r = v.r;
    d.z = v.z;
    d.active = 1;
  }
  Builder bl(B, true);
  build_precond(bl, B, {0}, true);
  for (const Launch& L : bl.L)
    if (!L.use_direct || L.op == OP_TAIL || L.op == OP_TAIL_UP)
      fail(AMG_ERR_UNSUPPORTED, "launch without a by-value descriptor in the fixed-scratch V-cycle");
  const Level& L0 = H.lev[0];
  gather_rhs(L0.n, 1, L0.perm, r, v.r, us);
  issue_launches(bl.L, 0, bl.L.size(), nullptr, nullptr, desc, 1, B.fp32, us);
  scatter_rhs(L0.n, 1, L0.perm, v.z, z, us);
}

}  // namespace amgx
