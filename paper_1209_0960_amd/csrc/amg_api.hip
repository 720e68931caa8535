// C interface of the MI355X aggregation AMG-PCG: hierarchy construction,
// preconditioner application, (flexible) preconditioned CG, introspection.
#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstring>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <unordered_map>
#include <mutex>
#include <thread>

#include "amg_internal.h"

namespace amgx {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
void fail(amg_status st, const std::string& msg) {
  set_error(msg);
  throw Failure{st};
}

// ------------------------------------------------------------------ allocator
static amg_alloc_fn g_alloc = nullptr;
static amg_free_fn g_free = nullptr;
static void* g_ctx = nullptr;

// Default allocator: a cache of hipMalloc blocks.  A freed block is kept for
// the stream that freed it, whose order puts any reuse after the block's last
// use; once the library has synchronised that stream after the free, the
// block is idle and any stream may take it.  No stream waits on an event of
// another stream, which may be under graph capture meanwhile.  Blocks are
// rounded (256 B below 1 MiB, 2 MiB above) and reused best fit within 25% +
// 2 MiB of the request; they return to the device only when a hipMalloc fails
// (then the calling stream is synchronised, every idle block is released and
// the allocation retried).  The stream-ordered runtime pool was measured at
// milliseconds of runtime calls per hierarchy; this keeps setup and release
// to a map lookup per buffer once warm.
namespace {
constexpr uintptr_t ANY_STREAM = ~(uintptr_t)0;
struct CKey {
  int dev;
  uintptr_t s;  // freeing stream, or ANY_STREAM once idle
  size_t bytes;
  bool operator<(const CKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (s != o.s) return s < o.s;
    return bytes < o.bytes;
  }
};
struct CVal {
  void* p;
  unsigned long long gen;  // order of the free
};
std::mutex g_cmu;
std::multimap<CKey, CVal> g_cache;
std::unordered_map<void*, std::pair<int, size_t>> g_live;  // live block -> (device, bytes)
unsigned long long g_gen = 0;

size_t round_bytes(size_t b) {
  const size_t MB2 = (size_t)2 << 20;
  return b < ((size_t)1 << 20) ? (b + 255) & ~(size_t)255 : (b + MB2 - 1) / MB2 * MB2;
}

// The cache's runtime calls (hipMalloc, hipFree) concern only memory that no
// stream uses.  Other threads may be capturing graphs meanwhile; the relaxed
// interaction mode keeps these calls from invalidating those captures.
struct RelaxedCapture {
  hipStreamCaptureMode m = hipStreamCaptureModeRelaxed;
  RelaxedCapture() { (void)hipThreadExchangeStreamCaptureMode(&m); }
  ~RelaxedCapture() { (void)hipThreadExchangeStreamCaptureMode(&m); }
};

// Takes the smallest fitting block kept for (dev, s); the lock is held.
void* take_block(int dev, uintptr_t s, size_t need) {
  const size_t limit = need + need / 4 + ((size_t)2 << 20);
  auto it = g_cache.lower_bound(CKey{dev, s, need});
  if (it == g_cache.end() || it->first.dev != dev || it->first.s != s || it->first.bytes > limit) return nullptr;
  void* p = it->second.p;
  g_live[p] = {dev, it->first.bytes};
  g_cache.erase(it);
  return p;
}

// Blocks freed on s up to free number `gen` become idle (s has been
// synchronised after those frees).
void promote(hipStream_t s, unsigned long long gen) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(g_cmu);
  auto it = g_cache.lower_bound(CKey{dev, (uintptr_t)s, 0});
  while (it != g_cache.end() && it->first.dev == dev && it->first.s == (uintptr_t)s) {
    if (it->second.gen <= gen) {
      g_cache.insert({CKey{dev, ANY_STREAM, it->first.bytes}, it->second});
      it = g_cache.erase(it);
    } else {
      ++it;
    }
  }
}

unsigned long long free_count() {
  std::lock_guard<std::mutex> g(g_cmu);
  return g_gen;
}

void release_idle(int dev, hipStream_t s) {
  const unsigned long long gen = free_count();
  if (hipStreamSynchronize(s) == hipSuccess) promote(s, gen);
  (void)hipGetLastError();
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> g(g_cmu);
    auto it = g_cache.lower_bound(CKey{dev, ANY_STREAM, 0});
    while (it != g_cache.end() && it->first.dev == dev && it->first.s == ANY_STREAM) {
      drop.push_back(it->second.p);
      it = g_cache.erase(it);
    }
  }
  for (void* p : drop) (void)hipFree(p);
}
}  // namespace

// Frees every cached block of the current device after a device-wide
// synchronisation (no stream can still use a freed block then).
void release_cached_blocks() {
  int dev = 0;
  AMG_HIP(hipGetDevice(&dev));
  AMG_HIP(hipDeviceSynchronize());
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> g(g_cmu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
      if (it->first.dev == dev) {
        drop.push_back(it->second.p);
        it = g_cache.erase(it);
      } else {
        ++it;
      }
    }
  }
  RelaxedCapture relaxed;
  for (void* p : drop) (void)hipFree(p);
}

hipError_t sync_stream_nothrow(hipStream_t s) {
  const unsigned long long gen = free_count();
  const hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) promote(s, gen);
  return e;
}

void sync_stream(hipStream_t s) {
  const unsigned long long gen = free_count();
  AMG_HIP(hipStreamSynchronize(s));
  promote(s, gen);
}

void* dalloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 16;
  if (g_alloc) {
    void* p = g_alloc(bytes, (void*)s, g_ctx);
    if (!p) fail(AMG_ERR_OUT_OF_MEMORY, "allocator hook returned NULL for " + std::to_string(bytes) + " bytes");
    return p;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  const size_t need = round_bytes(bytes);
  {
    std::lock_guard<std::mutex> g(g_cmu);
    void* p = take_block(dev, (uintptr_t)s, need);
    if (!p) p = take_block(dev, ANY_STREAM, need);
    if (p) return p;
  }
  RelaxedCapture relaxed;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, need);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    release_idle(dev, s);
    e = hipMalloc(&p, need);
  }
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? AMG_ERR_OUT_OF_MEMORY : AMG_ERR_HIP,
         std::string("hipMalloc(") + std::to_string(need) + "): " + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> g(g_cmu);
  g_live[p] = {dev, need};
  return p;
}

void dfree(void* p, hipStream_t s) {
  if (!p) return;
  if (g_free) {
    g_free(p, (void*)s, g_ctx);
    return;
  }
  std::lock_guard<std::mutex> g(g_cmu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;  // not ours
  const CKey key{it->second.first, (uintptr_t)s, it->second.second};
  g_live.erase(it);
  g_cache.insert({key, CVal{p, ++g_gen}});
}

void Hierarchy::free_one(void* ptr, hipStream_t s) {
  if (!ptr) return;
  {
    std::lock_guard<std::mutex> g(owned_mu);
    size_t k = 0;
    while (k < owned.size() && owned[k].first != ptr) ++k;
    if (k == owned.size()) return;
    bytes -= owned[k].second;
    owned[k] = owned.back();
    owned.pop_back();
  }
  dfree(ptr, s);
}

void Hierarchy::release(hipStream_t s) {
  if (apply_done) {  // the last preconditioner application may still read the arrays below
    (void)hipEventSynchronize(apply_done);
    (void)hipEventDestroy(apply_done);
    apply_done = nullptr;
  }
  if (single) {  // its launch tables and graph refer to the arrays below
    batch_destroy(single);
    single = nullptr;
  }
  for (auto& o : owned) dfree(o.first, s);
  owned.clear();
  bytes = 0;
}

// ------------------------------------------------------------------ timing
static std::mutex g_tmu;

static int g_timing = 0;  // bit mask of enabled kinds
static std::vector<TimingRec> g_pending;
static std::vector<hipEvent_t> g_event_pool;
static double g_ms[AMG_KIND_COUNT];
static int64_t g_launches[AMG_KIND_COUNT];
static double g_bytes[AMG_KIND_COUNT];

bool timing_on() { return g_timing != 0; }
int g_timing_mask_for_graphs() { return g_timing; }

static hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  AMG_HIP(hipEventCreate(&e));
  return e;
}

KTimer::KTimer(int k, hipStream_t st, double b) : kind(k), s(st), bytes(b) {
  if (k < 0 || !(g_timing & (1 << k))) return;
  std::lock_guard<std::mutex> g(g_tmu);
  e0 = take_event();
  e1 = take_event();
  AMG_HIP(hipEventRecord(e0, s));
}

KTimer::~KTimer() {
  if (!e0) return;
  (void)hipEventRecord(e1, s);
  std::lock_guard<std::mutex> g(g_tmu);
  g_pending.push_back(TimingRec{kind, bytes, e0, e1});
}

static void drain_timing() {
  for (auto& r : g_pending) {
    float ms = 0.f;
    (void)hipEventSynchronize(r.e1);
    (void)hipEventElapsedTime(&ms, r.e0, r.e1);
    g_ms[r.kind] += ms;
    g_launches[r.kind] += 1;
    g_bytes[r.kind] += r.bytes;
    g_event_pool.push_back(r.e0);
    g_event_pool.push_back(r.e1);
  }
  g_pending.clear();
}

}  // namespace amgx

using namespace amgx;

struct amg_hierarchy {
  Hierarchy H;
};

struct amg_batch {
  Batch* B = nullptr;
};

namespace {

template <typename F>
amg_status guarded(F&& f) {
  try {
    f();
    return AMG_OK;
  } catch (const Failure& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return AMG_ERR_OUT_OF_MEMORY;
  }
}

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void check_params(const amg_params& p) {
  if (!(p.strength_threshold > 0.0 && p.strength_threshold < 1.0)) fail(AMG_ERR_INVALID_ARG, "strength_threshold");
  if (!(p.isolated_threshold >= 0.0)) fail(AMG_ERR_INVALID_ARG, "isolated_threshold");
  if (p.agg_min < 1 || p.agg_max < p.agg_min) fail(AMG_ERR_INVALID_ARG, "agg_min/agg_max");
  if (p.agg_max > 32) fail(AMG_ERR_UNSUPPORTED, "agg_max above 32");
  if (p.agg_diameter < 1) fail(AMG_ERR_INVALID_ARG, "agg_diameter");
  if (p.tile_rows < 64 || p.tile_rows > 1024) fail(AMG_ERR_UNSUPPORTED, "tile_rows outside 64..1024");
  if (p.coarse_max < 1 || p.max_levels < 1) fail(AMG_ERR_INVALID_ARG, "coarse_max/max_levels");
  if (p.max_levels > MAX_LEVELS) fail(AMG_ERR_UNSUPPORTED, "max_levels above 32");
  if (p.smoother < AMG_SMOOTHER_MCSGS || p.smoother > AMG_SMOOTHER_TILE_MCSGS) fail(AMG_ERR_INVALID_ARG, "smoother");
  if (p.coarse_smoother < -1 || p.coarse_smoother > AMG_SMOOTHER_TILE_MCSGS)
    fail(AMG_ERR_INVALID_ARG, "coarse_smoother");
  if ((p.coarse_smoother >= 0 || p.coarse_smooth_tile_rows > 0) && p.coarse_from < 1)
    fail(AMG_ERR_INVALID_ARG, "coarse_from");
  if (p.smooth_tile_rows < 0 || p.coarse_smooth_tile_rows < 0) fail(AMG_ERR_INVALID_ARG, "smooth_tile_rows");
  if ((p.smooth_tile_rows > 0 && (p.smooth_tile_rows < 64 || p.smooth_tile_rows > 1024)) ||
      (p.coarse_smooth_tile_rows > 0 && (p.coarse_smooth_tile_rows < 64 || p.coarse_smooth_tile_rows > 1024)))
    fail(AMG_ERR_UNSUPPORTED, "smoothing tiles outside 64..1024 rows");
  if (p.pre_sweeps < 0 || p.post_sweeps < 0) fail(AMG_ERR_INVALID_ARG, "sweeps");
  if (p.tail_rows < 0) fail(AMG_ERR_INVALID_ARG, "tail_rows");
  if (p.colour_tile_rows < 64 || p.colour_tile_rows > 1024) fail(AMG_ERR_UNSUPPORTED, "colour_tile_rows outside 64..1024");
  if (p.spmv_format != 0 && p.spmv_format != 1) fail(AMG_ERR_INVALID_ARG, "spmv_format");
  if (p.block_size < 1) fail(AMG_ERR_INVALID_ARG, "block_size");
  if (p.block_size > 4) fail(AMG_ERR_UNSUPPORTED, "block_size above 4");
  if (p.block_size > 1 && (p.smoother != AMG_SMOOTHER_MCSGS ||
                           (p.coarse_smoother >= 0 && p.coarse_smoother != AMG_SMOOTHER_MCSGS)))
    fail(AMG_ERR_UNSUPPORTED, "point-based levels (block_size > 1) take the multicolour smoother only");
  if (p.block_size > 1 && p.tail_rows > 0)
    fail(AMG_ERR_UNSUPPORTED, "point-based levels (block_size > 1) are not cycled by the one-workgroup tail");
}

// Colouring of level l for its smoother (the colour-ordered relabelling comes
// later, once the coarsest level is known).
void colour_level(Hierarchy& H, int l, hipStream_t s) {
  const amg_params& p = H.p;
  Level& L = H.lev[l];
  const int sm = level_smoother(p, l), bs = p.block_size;
  if (sm == AMG_SMOOTHER_HYBRID_SGS) {
    colour_single(H, L, s);
  } else if (sm == AMG_SMOOTHER_TILE_MCSGS) {  // tile-local colours set the sweep order inside a tile
    colour_tile_local(H, L, smooth_tile(p, l), s);
  } else if (bs > 1) {  // node colours, shared by each node's unknowns
    Level S;
    node_graph(H, L, bs, S, s);
    colour(H, S, p.colour_seed + (uint32_t)l, s);
    expand_colours(H, S, bs, L, s);
    release_level(H, S, s);
  } else {
    colour(H, L, p.colour_seed + (uint32_t)l, s);
  }
}

// Setup work beside the coarsening: a second host thread, with a stream of
// its own, colours level l as soon as its matrix exists (level 0 at once,
// level l + 1 after its Galerkin product) and factorises the coarsest level
// once it is known, so that these chains of small launches and host round
// trips overlap the coarsening and the relabelling of the finer levels.  The
// two threads touch different fields of a level; the level vector is
// reserved in full beforehand so that it never moves.  threaded = false: every
// task runs at once on the caller's thread and stream.
class SideThread {
 public:
  SideThread(Hierarchy& H, bool threaded) : H_(H), threaded_(threaded) {
    if (!threaded_) return;
    (void)hipGetDevice(&dev_);
    s2_ = stream_take();
    th_ = std::thread([this] { run(); });
  }
  ~SideThread() { stop(); }
  SideThread(const SideThread&) = delete;
  SideThread& operator=(const SideThread&) = delete;
  // Colour level l (its matrix is complete once stream s reaches this point).
  void colour(int l, hipStream_t s) { push(COLOUR, l, s); }
  // Dense factorisation of the coarsest level l.
  void factor(int l, hipStream_t s) { push(FACTOR, l, s); }
  // Waits until every level pushed so far is coloured; raises the first
  // failure.
  void wait_colours() {
    if (!threaded_) return;
    std::unique_lock<std::mutex> g(mu_);
    done_cv_.wait(g, [&] { return coloured_ == colours_; });
    if (st_ != AMG_OK) {
      g.unlock();
      stop();
      fail(st_, msg_);
    }
  }
  // Waits for every task; raises the first failure.
  void finish() {
    stop();
    if (st_ != AMG_OK) fail(st_, msg_);
  }

 private:
  enum Kind { COLOUR, FACTOR };
  struct Task {
    Kind kind;
    int l;
    hipEvent_t ready;
  };
  void run_task(Kind kind, int l, hipStream_t s) {
    if (kind == COLOUR)
      colour_level(H_, l, s);
    else
      coarse_factor(H_, H_.lev[l], s);
  }
  void push(Kind kind, int l, hipStream_t s) {
    if (!threaded_) {
      run_task(kind, l, s);
      return;
    }
    hipEvent_t e = event_take();
    AMG_HIP(hipEventRecord(e, s));
    {
      std::lock_guard<std::mutex> g(mu_);
      q_.push_back({kind, l, e});
      if (kind == COLOUR) ++colours_;
    }
    cv_.notify_one();
  }
  void stop() {
    if (!th_.joinable()) return;
    {
      std::lock_guard<std::mutex> g(mu_);
      done_ = true;
    }
    cv_.notify_one();
    th_.join();
    stream_give(s2_);
  }
  void run() {
    (void)hipSetDevice(dev_);
    for (;;) {
      Task t;
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&] { return done_ || !q_.empty(); });
        if (q_.empty()) break;
        t = q_.front();
        q_.pop_front();
      }
      amg_status st = AMG_OK;
      std::string msg;
      if (st_ == AMG_OK) {
        try {
          AMG_HIP(hipStreamWaitEvent(s2_, t.ready, 0));
          run_task(t.kind, t.l, s2_);
          if (t.kind == COLOUR) sync_stream(s2_);  // the colours are complete when counted
        } catch (const Failure& e) {
          st = e.st;
          msg = amg_last_error();
        } catch (const std::bad_alloc&) {
          st = AMG_ERR_OUT_OF_MEMORY;
          msg = "host allocation failed";
        }
      }
      event_give(t.ready);
      {
        std::lock_guard<std::mutex> g(mu_);
        if (st != AMG_OK && st_ == AMG_OK) {
          st_ = st;
          msg_ = msg;
        }
        if (t.kind == COLOUR) ++coloured_;
      }
      done_cv_.notify_all();
    }
    (void)sync_stream_nothrow(s2_);
  }
  Hierarchy& H_;
  bool threaded_;
  int dev_ = 0;
  hipStream_t s2_ = nullptr;
  std::thread th_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<Task> q_;
  bool done_ = false;
  int colours_ = 0, coloured_ = 0;  // colouring tasks pushed / done
  amg_status st_ = AMG_OK;
  std::string msg_;
};

void setup_impl(const amg_csr* A, const amg_params* pp, hipStream_t s, Hierarchy& H, bool overlap) {
  const double t0 = now_ms();
  if (!A || !pp) fail(AMG_ERR_INVALID_ARG, "NULL argument");
  H.p = *pp;
  check_params(H.p);
  H.flexible = H.p.flexible < 0 ? (H.p.vcycle_fp32 ? 1 : 0) : (H.p.flexible ? 1 : 0);
  H.setup_stream = s;
  if (A->n <= 0 || A->nnz < A->n || !A->rowptr || !A->colind || !A->vals)
    fail(AMG_ERR_INVALID_ARG, "invalid CSR header (n, nnz or NULL arrays)");
  const int fl = validate_csr(A->n, A->nnz, A->rowptr, A->colind, A->vals, H.p.check_symmetry, s);
  if (fl & 1) fail(AMG_ERR_INVALID_ARG, "malformed CSR (row pointers, column order/range or non-finite value)");
  if (fl & 2) fail(AMG_ERR_BAD_DIAGONAL, "missing or non-positive diagonal");
  if (fl & 4) fail(AMG_ERR_NOT_SYMMETRIC, "matrix is not symmetric");
  const int bs = H.p.block_size;
  if (bs > 1 && validate_blocks(A->n, bs, A->rowptr, A->colind, s))
    fail(AMG_ERR_INVALID_ARG, "block_size > 1 needs every node's rows to hold whole blocks, the diagonal block included");

  H.lev.clear();
  H.lev.reserve(MAX_LEVELS + 1);  // never reallocated while the colouring thread reads it
  H.lev.emplace_back();
  {
    Level& L0 = H.lev[0];
    L0.n = A->n;
    L0.nnz = A->nnz;
    L0.rowptr = H.alloc<int>((size_t)A->n + 1, s);
    L0.colind = H.alloc<int>((size_t)A->nnz, s);
    L0.vals = H.alloc<double>((size_t)A->nnz, s);
    AMG_HIP(hipMemcpyAsync(L0.rowptr, A->rowptr, ((size_t)A->n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(L0.colind, A->colind, (size_t)A->nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(L0.vals, A->vals, (size_t)A->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  const amg_params& p = H.p;
  H.lev[0].T = p.tile_rows;
  H.lev[0].ntiles = (H.lev[0].n + p.tile_rows - 1) / p.tile_rows;
  SideThread side(H, overlap);
  side.colour(0, s);
  for (;;) {
    const int l = (int)H.lev.size() - 1;
    if (H.lev[l].n <= p.coarse_max || l == p.max_levels - 1) break;
    uint8_t *strong, *iso;
    DBuf ts, ti;
    // point-based levels: strength and aggregation on the node graph
    Level S;
    if (bs > 1) node_graph(H, H.lev[l], bs, S, s);
    Level& G = bs > 1 ? S : H.lev[l];
    const int n = G.n, nnz = G.nnz;
    if (p.keep_setup_data) {
      strong = H.alloc<uint8_t>((size_t)nnz, s);
      iso = H.alloc<uint8_t>((size_t)n, s);
      H.lev[l].strong = strong;
      H.lev[l].iso = iso;
      H.lev[l].nn = n;
      H.lev[l].nnzb = nnz;
    } else {
      ts = DBuf((size_t)nnz, s);
      ti = DBuf((size_t)n, s);
      strong = ts.as<uint8_t>();
      iso = ti.as<uint8_t>();
    }
    // level 0's values were checked exactly symmetric; Galerkin sums of a
    // coarse level need not be (their terms are added in different orders),
    // nor are the block norms of the node graph
    strength(G, p.strength_threshold, p.isolated_threshold, strong, iso, bs == 1 && l == 0 && p.check_symmetry != 0,
             s);
    const int nc = aggregate(H, G, strong, iso, p, s);
    if ((double)nc > 0.9 * (double)n) {
      if (bs > 1) release_level(H, S, s);
      H.lev[l].nc = 0;  // stalled: this level becomes the coarsest
      break;
    }
    if (bs > 1) {
      expand_aggregates(H, S, bs, H.lev[l], s);
      release_level(H, S, s);
    }
    H.lev.emplace_back();
    galerkin(H, H.lev[l], H.lev[l + 1], s);
    H.lev[l + 1].T = p.tile_rows;
    H.lev[l + 1].ntiles = (H.lev[l + 1].n + p.tile_rows - 1) / p.tile_rows;
    side.colour(l + 1, s);
  }
  const int Lc = (int)H.lev.size() - 1;
  if (H.lev[Lc].n > 4096)
    fail(AMG_ERR_COARSENING_STALLED, "coarsest level has " + std::to_string(H.lev[Lc].n) + " rows");
  side.factor(Lc, s);
  side.wait_colours();
  H.lev[Lc].nc = 0;
  const bool f32 = p.vcycle_fp32 != 0;
  for (int l = 0; l <= Lc; ++l) {
    H.lev[l].bs = bs;
    H.lev[l].sm = level_smoother(p, l);
    // from here on a level's tiles are its smoothing tiles (aggregation is done)
    H.lev[l].T = smooth_tile(p, l);
    H.lev[l].ntiles = (H.lev[l].n + H.lev[l].T - 1) / H.lev[l].T;
    if (H.lev[l].sm == AMG_SMOOTHER_TILE_MCSGS) tile_colour_order(H, H.lev[l], l < Lc, s);
  }
  // Relabel every level above the coarsest into colour order (the coarsest
  // keeps its natural order for the dense solve).
  for (int l = Lc - 1; l >= 0; --l) permute_level(H, l, l + 1 < Lc ? H.lev[l + 1].perm : nullptr, s);
  for (int l = 0; l <= Lc; ++l) {
    Level& L = H.lev[l];
    const double mean = (double)L.nnz / L.n;
    L.sub = 4;
    while (L.sub < 64 && L.sub < mean) L.sub *= 2;
  }
  for (int l = 0; l < Lc; ++l) {
    Level& L = H.lev[l];
    if (L.sm == AMG_SMOOTHER_L1_JACOBI) {
      if (f32) {
        L.l1_32 = H.alloc<float>((size_t)L.n, s);
        l1_diag(L, nullptr, L.l1_32, s);
      } else {
        L.l1 = H.alloc<double>((size_t)L.n, s);
        l1_diag(L, L.l1, nullptr, s);
      }
    }
    if (bs > 1) block_inverses(H, L, bs, f32, s);
    build_sell(H, l, s);
    if (tile_sweeps(L.sm)) {
      tile_couplings(H, L, f32, s);
      // Wavefront steps: for the hybrid smoother, and on colour-ordered
      // levels for the sweeps that use them (the one-workgroup tail, levels
      // of 64 colours or more, tiles whose staged sweep exceeds 64 KiB of
      // LDS at 8 right-hand sides); the colour-by-colour sweeps need none.
      const bool steps = L.sm == AMG_SMOOTHER_HYBRID_SGS || p.tail_rows > 0 || L.tncol >= 64 ||
                         tsgs_lds_bytes(L.T, std::max(L.icmax, 1), 8, L.tncol, 8) > 65536;
      if (steps) hybrid_steps(H, L, L.T, s);
    }
    L.sptr_d = H.alloc<int>(L.sptr.size(), s);
    AMG_HIP(hipMemcpyAsync(L.sptr_d, L.sptr.data(), L.sptr.size() * sizeof(int), hipMemcpyHostToDevice, s));
    if (f32) {
      const size_t ent = (size_t)L.soff_h[L.nsl];
      L.sval32 = H.alloc<float>(ent, s);
      cast_f32(L.sval, L.sval32, ent, s);
      L.dg32 = H.alloc<float>((size_t)L.n, s);
      cast_f32(L.dg, L.dg32, (size_t)L.n, s);
      if (l > 0) {  // level 0 keeps FP64 values for the outer CG product
        H.free_one(L.sval, s);
        L.sval = nullptr;
      }
    }
  }
  side.finish();
  sync_stream(s);
  H.setup_ms = now_ms() - t0;
}

}  // namespace

extern "C" {

amg_status amg_default_params(amg_params* p) {
  if (!p) return AMG_ERR_INVALID_ARG;
  std::memset(p, 0, sizeof(*p));
  p->strength_threshold = 0.08;
  p->isolated_threshold = 1e-5;
  p->agg_min = 8;
  p->agg_max = 12;
  p->agg_diameter = 3;
  p->omega = 1.6;
  p->coarse_max = 500;
  p->max_levels = 25;
  p->tile_rows = 128;
  p->smoother = AMG_SMOOTHER_MCSGS;
  p->pre_sweeps = 1;
  p->post_sweeps = 1;
  p->vcycle_fp32 = 0;
  p->flexible = -1;
  p->colour_seed = 0;
  p->check_symmetry = 1;
  p->keep_setup_data = 0;
  p->use_graphs = 1;
  p->tail_rows = 0;
  p->colour_tile_rows = 128;
  p->block_size = 1;
  p->spmv_format = 0;
  p->coarse_smoother = -1;
  p->coarse_from = 1;
  p->smooth_tile_rows = 0;
  p->coarse_smooth_tile_rows = 0;
  return AMG_OK;
}

namespace {
// overlap: colour the levels from a second host thread beside the coarsening
// (a single setup); the setups of a batch already overlap one another.
amg_status setup_one(const amg_csr* A, const amg_params* p, hipStream_t stream, amg_hierarchy** out, bool overlap) {
  if (!out) {
    set_error("out is NULL");
    return AMG_ERR_INVALID_ARG;
  }
  *out = nullptr;
  amg_hierarchy* h = nullptr;
  try {
    h = new amg_hierarchy();
  } catch (...) {
    set_error("host allocation failed");
    return AMG_ERR_OUT_OF_MEMORY;
  }
  amg_status st = guarded([&] { setup_impl(A, p, stream, h->H, overlap); });
  if (st != AMG_OK) {
    (void)sync_stream_nothrow(stream);
    h->H.release(stream);
    (void)sync_stream_nothrow(stream);
    delete h;
    return st;
  }
  *out = h;
  return AMG_OK;
}
}  // namespace

amg_status amg_setup(const amg_csr* A, const amg_params* p, void* stream, amg_hierarchy** out) {
  return setup_one(A, p, S(stream), out, true);
}

amg_status amg_precond_apply(amg_hierarchy* h, const double* r, double* z, void* stream) {
  if (!h || !r || !z || r == z) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  return guarded([&] { precond_run(h->H, r, z, S(stream)); });
}

amg_status amg_precond_apply_noalloc(amg_hierarchy* h, const double* r, double* z, void* stream) {
  if (!h || !r || !z || r == z) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  return guarded([&] { precond_noalloc_run(h->H, r, z, S(stream)); });
}

amg_status pcg_solve(amg_hierarchy* h, const double* b, double* x, double rtol, int32_t maxit, amg_solve_info* info,
                     double* res_hist, double* iter_hist, void* stream) {
  if (!h || !b || !x || maxit < 0 || !(rtol >= 0.0)) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  amg_status st = AMG_OK;
  amg_status g = guarded([&] { st = pcg_run(h->H, b, x, rtol, maxit, info, res_hist, iter_hist, S(stream)); });
  return g != AMG_OK ? g : st;
}

amg_status bicgstab_solve(amg_hierarchy* h, const double* b, double* x, double rtol, int32_t maxit,
                          amg_solve_info* info, int32_t* half_step, double* res_hist, double* iter_hist,
                          void* stream) {
  if (!h || !b || !x || maxit < 0 || !(rtol >= 0.0)) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  amg_status st = AMG_OK;
  amg_status g = guarded(
      [&] { st = bicgstab_run(h->H, b, x, rtol, maxit, info, half_step, res_hist, iter_hist, S(stream)); });
  return g != AMG_OK ? g : st;
}

void amg_free(amg_hierarchy* h) {
  if (!h) return;
  hipStream_t s = h->H.setup_stream;
  (void)sync_stream_nothrow(s);
  h->H.release(s);
  (void)sync_stream_nothrow(s);
  delete h;
}

const char* amg_status_string(amg_status s) {
  switch (s) {
    case AMG_OK: return "AMG_OK";
    case AMG_ERR_INVALID_ARG: return "AMG_ERR_INVALID_ARG";
    case AMG_ERR_BAD_DIAGONAL: return "AMG_ERR_BAD_DIAGONAL";
    case AMG_ERR_NOT_SYMMETRIC: return "AMG_ERR_NOT_SYMMETRIC";
    case AMG_ERR_NOT_SPD: return "AMG_ERR_NOT_SPD";
    case AMG_ERR_COARSENING_STALLED: return "AMG_ERR_COARSENING_STALLED";
    case AMG_ERR_OUT_OF_MEMORY: return "AMG_ERR_OUT_OF_MEMORY";
    case AMG_ERR_BREAKDOWN: return "AMG_ERR_BREAKDOWN";
    case AMG_ERR_NOT_CONVERGED: return "AMG_ERR_NOT_CONVERGED";
    case AMG_ERR_HIP: return "AMG_ERR_HIP";
    case AMG_ERR_UNSUPPORTED: return "AMG_ERR_UNSUPPORTED";
  }
  return "unknown status";
}

const char* amg_last_error(void) { return g_err.c_str(); }

amg_status amg_release_cached_memory(void) {
  return guarded([&] { release_cached_blocks(); });
}

amg_status amg_set_allocator(amg_alloc_fn alloc, amg_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    set_error("allocator and free must both be set or both be NULL");
    return AMG_ERR_INVALID_ARG;
  }
  g_alloc = alloc;
  g_free = free_fn;
  g_ctx = ctx;
  return AMG_OK;
}

amg_status amg_hierarchy_bytes(const amg_hierarchy* h, size_t* bytes) {
  if (!h || !bytes) return AMG_ERR_INVALID_ARG;
  *bytes = h->H.bytes;
  return AMG_OK;
}

amg_status amg_num_levels(const amg_hierarchy* h, int32_t* levels) {
  if (!h || !levels) return AMG_ERR_INVALID_ARG;
  *levels = (int32_t)h->H.lev.size();
  return AMG_OK;
}

amg_status amg_level_info(const amg_hierarchy* h, int32_t l, int32_t* n, int32_t* nnz, int32_t* ncolours,
                          int32_t* n_next) {
  if (!h || l < 0 || l >= (int32_t)h->H.lev.size()) {
    set_error("level out of range");
    return AMG_ERR_INVALID_ARG;
  }
  const Level& L = h->H.lev[l];
  if (n) *n = L.n;
  if (nnz) *nnz = L.nnz;
  if (ncolours) *ncolours = L.tcol ? L.tncol : L.ncol;
  if (n_next) *n_next = L.nc;
  return AMG_OK;
}

amg_status amg_copy_level(const amg_hierarchy* h, int32_t l, int32_t* agg, int32_t* colour, int32_t* rowptr,
                          int32_t* colind, double* vals, uint8_t* strong, uint8_t* iso) {
  if (!h || l < 0 || l >= (int32_t)h->H.lev.size()) {
    set_error("level out of range");
    return AMG_ERR_INVALID_ARG;
  }
  const Hierarchy& H = h->H;
  const Level& L = H.lev[l];
  return guarded([&] {
    AMG_HIP(hipDeviceSynchronize());
    const int n = L.n, nnz = L.nnz;
    const size_t sflags = L.bs > 1 ? (size_t)L.nnzb : (size_t)nnz, iflags = L.bs > 1 ? (size_t)L.nn : (size_t)n;
    if (strong && L.strong) AMG_HIP(hipMemcpy(strong, L.strong, sflags, hipMemcpyDeviceToHost));
    if (iso && L.iso) AMG_HIP(hipMemcpy(iso, L.iso, iflags, hipMemcpyDeviceToHost));
    if (!L.perm) {  // natural order (the coarsest level, or a one-level hierarchy)
      if (agg && L.agg && L.nc > 0) AMG_HIP(hipMemcpy(agg, L.agg, (size_t)n * sizeof(int), hipMemcpyDeviceToHost));
      if (colour)
        AMG_HIP(hipMemcpy(colour, L.tcol ? L.tcol : L.colour, (size_t)n * sizeof(int), hipMemcpyDeviceToHost));
      if (rowptr) AMG_HIP(hipMemcpy(rowptr, L.rowptr, ((size_t)n + 1) * sizeof(int), hipMemcpyDeviceToHost));
      if (colind) AMG_HIP(hipMemcpy(colind, L.colind, (size_t)nnz * sizeof(int), hipMemcpyDeviceToHost));
      if (vals) AMG_HIP(hipMemcpy(vals, L.vals, (size_t)nnz * sizeof(double), hipMemcpyDeviceToHost));
      return;
    }
    // Solve order (SELL-64 + diagonal) -> natural-order CSR on the host.
    std::vector<int> perm(n), pinv(n), srp(n + 1), scol(L.soff_h[L.nsl]);
    std::vector<double> sval(L.soff_h[L.nsl]), dg(n);
    AMG_HIP(hipMemcpy(perm.data(), L.perm, (size_t)n * sizeof(int), hipMemcpyDeviceToHost));
    AMG_HIP(hipMemcpy(srp.data(), L.rowptr, ((size_t)n + 1) * sizeof(int), hipMemcpyDeviceToHost));
    AMG_HIP(hipMemcpy(scol.data(), L.scol, scol.size() * sizeof(int), hipMemcpyDeviceToHost));
    if (L.sval) {
      AMG_HIP(hipMemcpy(sval.data(), L.sval, sval.size() * sizeof(double), hipMemcpyDeviceToHost));
    } else {  // FP32 levels above 0 keep only the FP32 copy: values are not recoverable exactly
      std::vector<float> f(sval.size());
      AMG_HIP(hipMemcpy(f.data(), L.sval32, f.size() * sizeof(float), hipMemcpyDeviceToHost));
      for (size_t q = 0; q < f.size(); ++q) sval[q] = f[q];
    }
    AMG_HIP(hipMemcpy(dg.data(), L.dg, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    for (int r = 0; r < n; ++r) pinv[perm[r]] = r;
    std::vector<int> rp(n + 1, 0);
    for (int i = 0; i < n; ++i) rp[i + 1] = rp[i] + (srp[pinv[i] + 1] - srp[pinv[i]]);
    std::vector<std::pair<int, double>> row;
    for (int sl = 0; sl < L.nsl; ++sl) {
      const int w = (L.soff_h[sl + 1] - L.soff_h[sl]) / 64;
      for (int r = L.srow_h[sl]; r < L.srow_h[sl + 1]; ++r) {
        const int lane = r - L.srow_h[sl];
        const int i = perm[r];
        row.clear();
        row.emplace_back(i, dg[r]);
        for (int k = 0; k < srp[r + 1] - srp[r] - 1 && k < w; ++k) {
          const size_t q = (size_t)L.soff_h[sl] + 64 * (size_t)k + lane;
          row.emplace_back(perm[scol[q]], sval[q]);
        }
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int, double>& a, const std::pair<int, double>& b) { return a.first < b.first; });
        for (size_t q = 0; q < row.size(); ++q) {
          if (colind) colind[rp[i] + q] = row[q].first;
          if (vals) vals[rp[i] + q] = row[q].second;
        }
      }
    }
    if (rowptr) std::memcpy(rowptr, rp.data(), ((size_t)n + 1) * sizeof(int));
    if (colour && L.tcol) {  // colours of the tile sweep order (solve order)
      std::vector<int> tc(n);
      AMG_HIP(hipMemcpy(tc.data(), L.tcol, (size_t)n * sizeof(int), hipMemcpyDeviceToHost));
      for (int r = 0; r < n; ++r) colour[perm[r]] = tc[r];
    } else if (colour) {
      for (int c = 0; c < L.ncol; ++c)
        for (int r = L.cptr[c]; r < L.cptr[c + 1]; ++r) colour[perm[r]] = c;
    }
    if (agg && L.nc > 0) {
      std::vector<int> pagg(n), nperm;
      AMG_HIP(hipMemcpy(pagg.data(), L.agg, (size_t)n * sizeof(int), hipMemcpyDeviceToHost));
      const Level& N = H.lev[l + 1];
      if (N.perm) {
        nperm.resize(N.n);
        AMG_HIP(hipMemcpy(nperm.data(), N.perm, (size_t)N.n * sizeof(int), hipMemcpyDeviceToHost));
      }
      for (int i = 0; i < n; ++i) {
        const int a = pagg[pinv[i]];
        agg[i] = N.perm ? nperm[a] : a;
      }
    }
  });
}

amg_status amg_setup_batched(const amg_csr* A, int32_t nsys, const amg_params* p, void* stream,
                             amg_hierarchy** out) {
  if (!out || !A || !p || nsys < 1) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  for (int i = 0; i < nsys; ++i) out[i] = nullptr;
  // Setups are independent and end in host synchronisations (level sizes,
  // colour counts), so several run at once, each from its own host thread on
  // its own stream; their kernels overlap on the device.
  hipStream_t us = S(stream);
  if (sync_stream_nothrow(us) != hipSuccess) {
    set_error("caller stream failed");
    return AMG_ERR_HIP;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int nthreads = std::max(1, std::min<int>(nsys, 16));
  // largest systems first, so that the last setups to start are short ones
  std::vector<int> order(nsys);
  for (int i = 0; i < nsys; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return A[a].nnz > A[b].nnz; });
  std::atomic<int> next{0};
  std::vector<amg_status> st(nsys, AMG_OK);
  std::vector<std::string> msg(nsys);
  auto worker = [&]() {
    (void)hipSetDevice(dev);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    for (int k = next++; k < nsys; k = next++) {
      const int i = order[k];
      if (!s) {
        st[i] = AMG_ERR_HIP;
        msg[i] = "stream creation failed";
        continue;
      }
      st[i] = setup_one(&A[i], p, s, &out[i], false);
      if (st[i] != AMG_OK) msg[i] = amg_last_error();
      if (out[i]) out[i]->H.setup_stream = us;
    }
    if (s) {
      (void)sync_stream_nothrow(s);
      (void)hipStreamDestroy(s);
    }
  };
  std::vector<std::thread> pool;
  try {
    for (int t = 1; t < nthreads; ++t) pool.emplace_back(worker);
  } catch (...) {
  }
  worker();
  for (auto& t : pool) t.join();
  for (int i = 0; i < nsys; ++i)
    if (st[i] != AMG_OK) {
      for (int j = 0; j < nsys; ++j) {
        amg_free(out[j]);
        out[j] = nullptr;
      }
      set_error("system " + std::to_string(i) + ": " + msg[i]);
      return st[i];
    }
  return AMG_OK;
}

amg_status pcg_solve_batched(amg_hierarchy* const* h, int32_t nsys, int32_t nrhs, const double* const* b,
                             double* const* x, double rtol, int32_t maxit, amg_solve_info* info, void* stream) {
  if (!h || !b || !x || nsys < 1 || maxit < 0 || !(rtol >= 0.0)) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  std::vector<Hierarchy*> hs(nsys);
  for (int i = 0; i < nsys; ++i) {
    if (!h[i] || !b[i] || !x[i]) {
      set_error("NULL hierarchy or vector for system " + std::to_string(i));
      return AMG_ERR_INVALID_ARG;
    }
    hs[i] = &h[i]->H;
  }
  amg_status st = AMG_OK;
  amg_status g = guarded([&] { st = pcg_batched_run(hs.data(), nsys, nrhs, b, x, rtol, maxit, info, S(stream)); });
  return g != AMG_OK ? g : st;
}

amg_status amg_batch_create(int32_t nrhs, int32_t max_entries, int32_t use_graphs, amg_batch** out) {
  if (!out) {
    set_error("out is NULL");
    return AMG_ERR_INVALID_ARG;
  }
  *out = nullptr;
  amg_batch* b = nullptr;
  amg_status st = guarded([&] {
    b = new amg_batch();
    b->B = batch_new(nrhs, max_entries, use_graphs);
  });
  if (st != AMG_OK) {
    delete b;
    return st;
  }
  *out = b;
  return AMG_OK;
}

amg_status amg_batch_submit(amg_batch* b, amg_hierarchy* h, const double* rhs, double* x, double rtol,
                            int32_t maxit, int64_t tag, void* stream) {
  if (!b || !h || !rhs || !x || maxit < 0 || !(rtol >= 0.0)) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  return guarded([&] { (void)batch_submit(*b->B, h->H, rhs, x, rtol, maxit, tag, S(stream)); });
}

amg_status amg_batch_step(amg_batch* b, int32_t iterations) {
  if (!b || iterations < 0) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  return guarded([&] { batch_step(*b->B, iterations); });
}

amg_status amg_batch_poll(amg_batch* b, int64_t* tags, amg_status* status, amg_solve_info* info, int32_t cap,
                          int32_t* count) {
  if (!b || !count || cap < 0) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  *count = batch_poll(*b->B, tags, status, info, cap);
  return AMG_OK;
}

amg_status amg_batch_active(const amg_batch* b, int32_t* active) {
  if (!b || !active) return AMG_ERR_INVALID_ARG;
  *active = batch_active(*b->B);
  return AMG_OK;
}

amg_status amg_batch_bytes(const amg_batch* b, size_t* bytes) {
  if (!b || !bytes) return AMG_ERR_INVALID_ARG;
  *bytes = batch_entry_bytes(*b->B);
  return AMG_OK;
}

void amg_batch_free(amg_batch* b) {
  if (!b) return;
  batch_destroy(b->B);
  delete b;
}

amg_status amg_estimate_bytes(int32_t n, int32_t nnz, const amg_params* p, int32_t nrhs, size_t* setup_peak,
                              size_t* hierarchy, size_t* context) {
  if (n <= 0 || nnz < n || !p || nrhs < 1) {
    set_error("invalid argument");
    return AMG_ERR_INVALID_ARG;
  }
  const double N = n, Z = nnz;
  const bool f32 = p->vcycle_fp32 != 0;
  const bool flex = p->flexible < 0 ? f32 : p->flexible != 0;
  const double vb = f32 ? 4.0 : 8.0;
  // Level 0 in solve order: SELL-64 off-diagonals (column + FP64 value, + FP32
  // copy), diagonal(s), permutation, row pointers, aggregate map and members.
  // The hybrid smoother adds two 16-bit wavefront steps per row, its
  // colour-ordered form the colours as well.
  // The CSR form of the outer product (spmv_format 1) keeps 12 B per entry more;
  // point-based levels keep bs values of the inverse diagonal block per row.
  const double bs = std::max(1, p->block_size);
  const double lev0 = (f32 ? 16.0 * Z + 12.0 * N : 12.0 * Z + 16.0 * N) +
                      (p->smoother == AMG_SMOOTHER_HYBRID_SGS ? 4.0 * N : 0.0) +
                      (p->smoother == AMG_SMOOTHER_TILE_MCSGS ? 8.0 * N : 0.0) +
                      (p->spmv_format == 1 ? 12.0 * Z : 0.0) + (bs > 1 ? (f32 ? 12.0 : 8.0) * bs * N : 0.0);
  // Coarser levels and slice padding stay below 35% of level 0 for aggregates
  // of 8-12 rows; the dense coarsest inverse and its factorisation workspace.
  const double cm = std::min<double>(std::max(p->coarse_max, 1), 4096);
  const double dense = 3.0 * 8.0 * cm * cm;
  const double hier = 1.35 * lev0 + dense;
  // Setup holds the input copy, strength flags, aggregation and Galerkin
  // temporaries and the relabelled copies of a level at once.
  const double peak = std::max(36.0 * Z + 8.0 * N, hier) + dense;
  // Per solve: CG vectors (x, b, r, z, p, q, and r_old for flexible CG) and the
  // cycle's x, b, t on every level (levels below 0 add at most 20%).
  const double ctx = nrhs * N * (8.0 * (6 + (flex ? 1 : 0)) + 3.6 * vb) + 2.0 * RED_BLOCKS * nrhs * 8.0 + 65536.0;
  if (setup_peak) *setup_peak = (size_t)peak;
  if (hierarchy) *hierarchy = (size_t)hier;
  if (context) *context = (size_t)ctx;
  return AMG_OK;
}

amg_status amg_set_kernel_timing(int32_t kind_mask) {
  std::lock_guard<std::mutex> g(g_tmu);
  g_timing = kind_mask;
  return AMG_OK;
}

amg_status amg_get_kernel_timing(int32_t kind, double* ms, int64_t* launches, double* bytes) {
  if (kind < 0 || kind >= AMG_KIND_COUNT) return AMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(g_tmu);
  drain_timing();
  if (ms) *ms = g_ms[kind];
  if (launches) *launches = g_launches[kind];
  if (bytes) *bytes = g_bytes[kind];
  return AMG_OK;
}

amg_status amg_reset_kernel_timing(void) {
  std::lock_guard<std::mutex> g(g_tmu);
  drain_timing();
  for (int k = 0; k < AMG_KIND_COUNT; ++k) {
    g_ms[k] = 0.0;
    g_launches[k] = 0;
    g_bytes[k] = 0.0;
  }
  return AMG_OK;
}

}  // extern "C"
