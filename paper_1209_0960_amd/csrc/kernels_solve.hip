// Solve-phase kernels for gfx950, table driven (see Item / BDesc): SELL-64
// multicolour Gauss-Seidel and l1-Jacobi sweeps, residual, restriction by
// aggregate member lists, prolongation with the over-correction factor, the
// coarsest-level product with the explicit inverse, the FP64 outer product
// and the CG vector kernels.  Each kernel handles R right-hand sides at once
// (interleaved vectors): a lane owns one row and keeps R accumulators, so the
// matrix is read once for all of them and the arithmetic of right-hand side
// k is the same for every R.  Contraction is off and every multiply-add is an
// explicit fma, so the code generated for different R rounds identically.
// Reductions: each block writes one partial sum per right-hand side; the
// per-entry finish kernel adds an entry's partials in a fixed order.
#pragma clang fp contract(off)

#include "amg_internal.h"

namespace amgx {

namespace {

constexpr int WAVE = 64;
constexpr int NT = 256;  // threads of every solve kernel

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

__device__ inline float madd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double madd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// R consecutive values as one vector access.
template <typename V, int R>
__device__ inline void ldv(const V* p, V (&o)[R]) {
  if constexpr (R == 1) {
    o[0] = p[0];
  } else {
    typedef V vt __attribute__((ext_vector_type(R)));
    const vt t = *reinterpret_cast<const vt*>(p);
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = t[k];
  }
}
template <typename V, int R>
__device__ inline void stv(V* p, const V (&o)[R]) {
  if constexpr (R == 1) {
    p[0] = o[0];
  } else {
    typedef V vt __attribute__((ext_vector_type(R)));
    vt t;
#pragma unroll
    for (int k = 0; k < R; ++k) t[k] = o[k];
    *reinterpret_cast<vt*>(p) = t;
  }
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Deterministic block sums of R values (valid in thread 0): per-wave
// butterfly, then the wave sums in wave order.
template <int R>
__device__ inline void block_sums(double (&v)[R]) {
  __shared__ double ws[NT / WAVE][R];
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = wave_sum_d(v[k]);
  const int w = threadIdx.x / WAVE;
  if (__lane_id() == 0)
#pragma unroll
    for (int k = 0; k < R; ++k) ws[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < R; ++k) {
      double s = 0.0;
      for (int i = 0; i < NT / WAVE; ++i) s += ws[i][k];
      v[k] = s;
    }
  __syncthreads();
}

template <int R>
__device__ inline void write_partials(const BDesc& d, int set, int part, const double (&v)[R]) {
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < R; ++k) d.partial[((size_t)set * RED_BLOCKS + part) * R + k] = v[k];
}

// Right-hand side k of the entry takes no more CG updates (finished or broken down).
__device__ inline bool frozen(const BDesc& d, int k) {
  return d.ctl[1 + k] != 0 || d.scal[k * S_COUNT + S_FLAG] != 0.0;
}

template <typename V>
struct Mat;
template <>
struct Mat<double> {
  __device__ static const double* sval(const BDesc& d) { return d.sval64; }
  __device__ static const double* dg(const BDesc& d) { return d.dg64; }
  __device__ static const double* l1(const BDesc& d) { return d.l164; }
  __device__ static const double* dinv(const BDesc& d) { return d.dinv64; }
  __device__ static const double* icv(const BDesc& d) { return d.icv64; }
  __device__ static const double* ocv(const BDesc& d) { return d.ocv64; }
};
template <>
struct Mat<float> {
  __device__ static const float* sval(const BDesc& d) { return d.sval32; }
  __device__ static const float* dg(const BDesc& d) { return d.dg32; }
  __device__ static const float* l1(const BDesc& d) { return d.l132; }
  __device__ static const float* dinv(const BDesc& d) { return d.dinv32; }
  __device__ static const float* icv(const BDesc& d) { return d.icv32; }
  __device__ static const float* ocv(const BDesc& d) { return d.ocv32; }
};

// Work item of this block.  Table launches read it from tab[blockIdx.x] and
// the descriptor from D (an inactive entry -- finished, awaiting removal from
// the batch -- returns at once); direct launches (a plan of one entry) get the
// descriptor by value and split [base.lo, base.hi) into pieces of base.part
// units per block, the same split the table would hold.
__device__ inline Item direct_item(const Item& base) {
  Item it;
  it.d = base.d;
  it.lo = base.lo + (int)blockIdx.x * base.part;
  it.hi = min(base.hi, it.lo + base.part);
  it.part = (int)blockIdx.x;
  return it;
}

#define AMG_KARGS const Item *__restrict__ tab, const BDesc *__restrict__ D, const BDesc dv, const Item base
#define AMG_BODY(BODY, ...)            \
  if constexpr (DIRECT) {              \
    const Item it = direct_item(base); \
    BODY(it, dv, ##__VA_ARGS__);       \
  } else {                             \
    const Item it = tab[blockIdx.x];   \
    const BDesc& d = D[it.d];          \
    if (d.active == 0) return;         \
    BODY(it, d, ##__VA_ARGS__);        \
  }

// ---------------------------------------------------------------- SELL-64
// Lane t of the wavefront owning slice s reads its off-diagonal entry e at
// soff[s] + 64 e + t: every matrix load is one contiguous 64-wide access;
// padding entries are (row, 0).
// Matrix entries of a level larger than the last-level cache are loaded with
// the non-temporal hint (nt): they are read once per pass and would otherwise
// push the gathered iterate values out of L2.  Smaller levels keep the
// ordinary loads, since their entries are re-read from the cache by the next
// passes.
// (A run-time choice between the two loads of one address is folded into
// one plain load by the compiler, so the choice is a template parameter and
// callers branch on the level's flag around whole loops.)
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <typename V, int R, bool NT>
__device__ inline void sell_offdiag_t(const int* __restrict__ scol, const V* __restrict__ sval, int base, int w,
                                      int lane, const V* x, V (&acc)[R]) {
  const int* cp = scol + base + lane;
  const V* vp = sval + base + lane;
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0;
  int e = 0;
  if constexpr (R * sizeof(V) <= 8) {
    // Long rows (coarse levels): chunks of 8 entries with all their loads,
    // then all their gathers, in flight together; same summation order.
    for (; w > 8 && e + 8 <= w; e += 8) {
      int j[8];
      V a[8], xv[8][R];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        j[q] = ld_stream<NT>(cp + 64 * (e + q));
        a[q] = ld_stream<NT>(vp + 64 * (e + q));
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) ldv<V, R>(x + (size_t)j[q] * R, xv[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = madd(a[q], xv[q][k], acc[k]);
    }
  }
  for (; e + 2 <= w; e += 2) {
    const int j0 = ld_stream<NT>(cp + 64 * e), j1 = ld_stream<NT>(cp + 64 * (e + 1));
    const V a0 = ld_stream<NT>(vp + 64 * e), a1 = ld_stream<NT>(vp + 64 * (e + 1));
    V x0[R], x1[R];
    ldv<V, R>(x + (size_t)j0 * R, x0);
    ldv<V, R>(x + (size_t)j1 * R, x1);
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = madd(a0, x0[k], acc[k]);
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = madd(a1, x1[k], acc[k]);
  }
  if (e < w) {
    const int j0 = ld_stream<NT>(cp + 64 * e);
    const V a0 = ld_stream<NT>(vp + 64 * e);
    V x0[R];
    ldv<V, R>(x + (size_t)j0 * R, x0);
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = madd(a0, x0[k], acc[k]);
  }
}

template <typename V, int R>
__device__ __forceinline__ void sell_offdiag(const int* __restrict__ scol, const V* __restrict__ sval, int base,
                                             int w, int lane, const V* x, V (&acc)[R], bool nt) {
  if (nt)
    sell_offdiag_t<V, R, true>(scol, sval, base, w, lane, x, acc);
  else
    sell_offdiag_t<V, R, false>(scol, sval, base, w, lane, x, acc);
}

// Gauss-Seidel update of the slices [lo, hi) (one per wavefront) of one
// colour: x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii.  Rows of one colour do
// not couple, so the in-place update is race free.  RES (the last pass before
// the residual): also t_i = b_i - (a_ii x_i + sum), from the same sum, which
// is what the residual kernel would compute for these rows.
template <typename V, int R, bool RES, bool NT>
__device__ __forceinline__ void kb_gs_body_t(const Item& it, const BDesc& d) {
  const int sl = it.lo + (int)(threadIdx.x / WAVE);
  if (sl >= it.hi) return;
  const int lane = __lane_id();
  const int r = d.srow[sl] + lane;
  const int base = d.soff[sl], w = (d.soff[sl + 1] - base) >> 6;
  V* x = static_cast<V*>(d.x);
  V acc[R];
  sell_offdiag_t<V, R, NT>(d.scol, Mat<V>::sval(d), base, w, lane, x, acc);
  if (r < d.srow[sl + 1]) {
    V bb[R], o[R];
    if constexpr (R == 1)
      bb[0] = ld_stream<NT>(static_cast<const V*>(d.b) + r);
    else
      ldv<V, R>(static_cast<const V*>(d.b) + (size_t)r * R, bb);
    const V dg = ld_stream<NT>(Mat<V>::dg(d) + r);
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = (bb[k] - acc[k]) / dg;
    stv<V, R>(x + (size_t)r * R, o);
    if constexpr (RES) {
      V t[R];
#pragma unroll
      for (int k = 0; k < R; ++k) t[k] = bb[k] - madd(dg, o[k], acc[k]);
      stv<V, R>(static_cast<V*>(d.t) + (size_t)r * R, t);
    }
  }
}
template <typename V, int R, bool RES = false>
__device__ __forceinline__ void kb_gs_body(const Item& it, const BDesc& d) {
  if (d.nt)
    kb_gs_body_t<V, R, RES, true>(it, d);
  else
    kb_gs_body_t<V, R, RES, false>(it, d);
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_gs(AMG_KARGS) {
  AMG_BODY((kb_gs_body<V, R>))
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_gsr(AMG_KARGS) {
  AMG_BODY((kb_gs_body<V, R, true>))
}

// Block Gauss-Seidel pass of a point-based level (Sec. 4.2): the slices
// [lo, hi) of one colour hold whole nodes of bs consecutive rows (a slice
// starts at a node and the rows of a node never straddle two slices or two
// wavefronts).  Row r of node rows [r0, r0 + bs): t_r = b_r - sum of a_rj x_j
// over its entries outside the node's own block (entry order), then
// x_r = sum_d dinv[r][d] t_(r0 + d), the node's t exchanged between its
// lanes.  Nodes of one colour do not couple, so the update is race free.
template <typename V, int R>
__device__ __forceinline__ void kb_bgs_body(const Item& it, const BDesc& d) {
  const int sl = it.lo + (int)(threadIdx.x / WAVE);
  if (sl >= it.hi) return;  // whole wavefronts only: the shuffles below see every lane
  const int lane = __lane_id();
  const int r = d.srow[sl] + lane;
  const bool act = r < d.srow[sl + 1];
  const int bs = d.blk, comp = r % bs, r0 = r - comp;
  const int base = d.soff[sl], w = (d.soff[sl + 1] - base) >> 6;
  const V* x = static_cast<const V*>(d.x);
  const V* sv = Mat<V>::sval(d);
  V t[R];
#pragma unroll
  for (int k = 0; k < R; ++k) t[k] = 0;
  for (int e = 0; e < w; ++e) {
    const int j = d.scol[base + 64 * e + lane];
    if (j < r0 || j >= r0 + bs) {  // outside the node's own block (padding names the row itself)
      const V a = sv[base + 64 * e + lane];
      V xv[R];
      ldv<V, R>(x + (size_t)j * R, xv);
#pragma unroll
      for (int k = 0; k < R; ++k) t[k] = madd(a, xv[k], t[k]);
    }
  }
  if (act) {
    V bb[R];
    ldv<V, R>(static_cast<const V*>(d.b) + (size_t)r * R, bb);
#pragma unroll
    for (int k = 0; k < R; ++k) t[k] = bb[k] - t[k];
  }
  V o[R];
#pragma unroll
  for (int k = 0; k < R; ++k) o[k] = 0;
  const V* dinv = Mat<V>::dinv(d) + (size_t)(act ? r : 0) * bs;
  for (int q = 0; q < bs; ++q) {
    const int src = act ? lane - comp + q : lane;  // lane of row r0 + q (same wavefront)
    const V dq = act ? dinv[q] : (V)0;
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = madd(dq, __shfl(t[k], src, WAVE), o[k]);
  }
  if (act) stv<V, R>(static_cast<V*>(d.x) + (size_t)r * R, o);
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_bgs(AMG_KARGS) {
  AMG_BODY((kb_bgs_body<V, R>))
}

// The first Gauss-Seidel pass from x = 0: every off-diagonal product is a
// zero, the sum stays +0 and the update is b_i / a_ii, so the pass reads no
// matrix entries and gives the same values bit for bit.
template <typename V, int R>
__device__ __forceinline__ void kb_gs0_body(const Item& it, const BDesc& d) {
  const int sl = it.lo + (int)(threadIdx.x / WAVE);
  if (sl >= it.hi) return;
  const int r = d.srow[sl] + __lane_id();
  if (r < d.srow[sl + 1]) {
    V bb[R], o[R];
    ldv<V, R>(static_cast<const V*>(d.b) + (size_t)r * R, bb);
    const V dg = Mat<V>::dg(d)[r];
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = bb[k] / dg;
    stv<V, R>(static_cast<V*>(d.x) + (size_t)r * R, o);
  }
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_gs0(AMG_KARGS) {
  AMG_BODY((kb_gs0_body<V, R>))
}

// t = b - A x on the slices [lo, hi).
template <typename V, int R, bool NT>
__device__ __forceinline__ void kb_resid_body_t(const Item& it, const BDesc& d) {
  const int sl = it.lo + (int)(threadIdx.x / WAVE);
  if (sl >= it.hi) return;
  const int lane = __lane_id();
  const int r = d.srow[sl] + lane;
  const int base = d.soff[sl], w = (d.soff[sl + 1] - base) >> 6;
  const V* x = static_cast<const V*>(d.x);
  V acc[R];
  sell_offdiag_t<V, R, NT>(d.scol, Mat<V>::sval(d), base, w, lane, x, acc);
  if (r < d.srow[sl + 1]) {
    V bb[R], xr[R], o[R];
    if constexpr (R == 1)
      bb[0] = ld_stream<NT>(static_cast<const V*>(d.b) + r);
    else
      ldv<V, R>(static_cast<const V*>(d.b) + (size_t)r * R, bb);
    ldv<V, R>(x + (size_t)r * R, xr);
    const V dg = ld_stream<NT>(Mat<V>::dg(d) + r);
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = bb[k] - madd(dg, xr[k], acc[k]);
    stv<V, R>(static_cast<V*>(d.t) + (size_t)r * R, o);
  }
}
template <typename V, int R>
__device__ __forceinline__ void kb_resid_body(const Item& it, const BDesc& d) {
  if (d.nt)
    kb_resid_body_t<V, R, true>(it, d);
  else
    kb_resid_body_t<V, R, false>(it, d);
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_resid(AMG_KARGS) {
  AMG_BODY((kb_resid_body<V, R>))
}

// ---------------------------------------------------------------- hybrid smoother
// Hybrid symmetric Gauss-Seidel (Sec. 3.2): block-Jacobi over the tiles of T
// rows of a level in natural order, one forward and one backward sequential
// Gauss-Seidel sweep inside each tile.  A step first forms, for every row,
// t_i = b_i - sum over the couplings to other tiles of a_ij x_j (the iterate
// from before the step); the in-tile sweeps then use t and the tile's own
// current values only, so tiles never read each other's updates.

// t = b - (couplings to other tiles) x on rows [lo, hi) (one thread per row,
// the level's compact list of each row's couplings to other tiles, SELL
// entry order).
template <typename V, int R>
__device__ __forceinline__ void kb_resid_off_body(const Item& it, const BDesc& d) {
  const V* x = static_cast<const V*>(d.x);
  const V* ocv = Mat<V>::ocv(d);
  for (int r = it.lo + (int)threadIdx.x; r < it.hi; r += (int)blockDim.x) {
    V acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0;
    const int e1 = d.ocp[r + 1];
    // four entries at a time: their loads, then their gathers, in flight together
    for (int e0 = d.ocp[r]; e0 < e1; e0 += 4) {
      V a[4], xv[4][R];
      int j[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u, e1 - 1);
        a[u] = ocv[e];
        j[u] = d.occ[e];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) ldv<V, R>(x + (size_t)j[u] * R, xv[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u < e1)
#pragma unroll
          for (int k = 0; k < R; ++k) acc[k] = madd(a[u], xv[u][k], acc[k]);
    }
    V bb[R], o[R];
    ldv<V, R>(static_cast<const V*>(d.b) + (size_t)r * R, bb);
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = bb[k] - acc[k];
    stv<V, R>(static_cast<V*>(d.t) + (size_t)r * R, o);
  }
}
// Residual of a tile-sweep level, t = b - (a_ii x_i + acc) on rows [lo, hi)
// (one thread per row), acc the sum over the row's in-tile couplings (compact
// order), then on over its couplings to other tiles.  from_t: the in-tile
// part is already in t (written by the last smoothing sweep, which holds the
// couplings and the final iterate); every path that forms this residual
// follows the same order, so all give the same bits.
template <typename V, int R>
__device__ __forceinline__ void kb_resid_tile_body(const Item& it, const BDesc& d, int from_t) {
  const V* x = static_cast<const V*>(d.x);
  V* t = static_cast<V*>(d.t);
  const V* icv = Mat<V>::icv(d);
  const V* ocv = Mat<V>::ocv(d);
  for (int r = it.lo + (int)threadIdx.x; r < it.hi; r += (int)blockDim.x) {
    V acc[R];
    if (from_t) {
      ldv<V, R>(t + (size_t)r * R, acc);
    } else {
#pragma unroll
      for (int k = 0; k < R; ++k) acc[k] = 0;
      const int lo = r - r % d.T, e1 = d.icp[r + 1];
      for (int e0 = d.icp[r]; e0 < e1; e0 += 4) {
        V a[4], xv[4][R];
        int j[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + u, e1 - 1);
          a[u] = icv[e];
          j[u] = lo + (int)d.icc[e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) ldv<V, R>(x + (size_t)j[u] * R, xv[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (e0 + u < e1)
#pragma unroll
            for (int k = 0; k < R; ++k) acc[k] = madd(a[u], xv[u][k], acc[k]);
      }
    }
    const int e1 = d.ocp[r + 1];
    for (int e0 = d.ocp[r]; e0 < e1; e0 += 4) {
      V a[4], xv[4][R];
      int j[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u, e1 - 1);
        a[u] = ocv[e];
        j[u] = d.occ[e];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) ldv<V, R>(x + (size_t)j[u] * R, xv[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u < e1)
#pragma unroll
          for (int k = 0; k < R; ++k) acc[k] = madd(a[u], xv[u][k], acc[k]);
    }
    V bb[R], xr[R], o[R];
    ldv<V, R>(static_cast<const V*>(d.b) + (size_t)r * R, bb);
    ldv<V, R>(x + (size_t)r * R, xr);
    const V dg = Mat<V>::dg(d)[r];
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = bb[k] - madd(dg, xr[k], acc[k]);
    stv<V, R>(t + (size_t)r * R, o);
  }
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_resid_tile(AMG_KARGS, int from_t) {
  AMG_BODY((kb_resid_tile_body<V, R>), from_t)
}

template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_resid_off(AMG_KARGS) {
  AMG_BODY((kb_resid_off_body<V, R>))
}

// The forward then the backward sweep over rows [lo, hi) of one tile by the
// lanes of one wavefront: x_i = (src_i - sum over in-tile j != i of a_ij x_j)
// / a_ii, rows of one wavefront step together (their couplings lie in earlier
// steps of the sweep, whose values are final, or in later ones, not yet
// touched), steps separated by sync().  Rows of backward step 0 have no
// coupling after them in the sweep order, so the backward sweep would
// recompute their forward values bit for bit: it starts at step 1.
// xt[(i - lo) * R + k] is the tile's iterate (LDS copy or the level's vector
// itself).  Every caller runs the same number of steps, so sync() may be a
// workgroup barrier.
//
// Each row is summed by a group of d.hg lanes (1 or HS_G): lane `sub` of the
// group adds the row's in-tile couplings sub, sub + hg, ... (SELL entry
// order) from zero, then group_sum adds the partial sums of lanes at distance
// 1, then 2.  Every kernel that sweeps tiles uses this order, so the launch
// path, its LDS-staged form and the one-workgroup tail give the same bits.
static_assert(HS_G == 4, "group_sum adds lanes at distance 1 and 2");

// Value of the lane at quad position given by the DPP quad permutation
// CTRL (0xB1: lanes 1,0,3,2 of each quad, i.e. lane ^ 1; 0x4E: 2,3,0,1,
// lane ^ 2); every lane of the quad must be active.
template <int CTRL>
__device__ __forceinline__ float quad_swap(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, 0xF, 0xF, false);
  p.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, p);
}

template <typename V, int R>
__device__ __forceinline__ void group_sum(V (&acc)[R], int G) {
  if (G == 1) return;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    acc[k] = acc[k] + quad_swap<0xB1>(acc[k]);
    acc[k] = acc[k] + quad_swap<0x4E>(acc[k]);
  }
}

template <typename V, int R, typename Sync>
__device__ inline void hybrid_tile(const BDesc& d, int lo, int hi, const V* __restrict__ src, V* xt, int lane,
                                   Sync sync) {
  const V* icv = Mat<V>::icv(d);
  const V* dg = Mat<V>::dg(d);
  const int G = d.hg, sub = lane % G, ng = WAVE / G;
  for (int dir = 0; dir < 2; ++dir) {
    const unsigned short* st = dir == 0 ? d.hsf : d.hsb;
    const int depth = dir == 0 ? d.hdf : d.hdb;
    for (int step = dir; step <= depth; ++step) {
      for (int i0 = lo; i0 < hi; i0 += ng) {
        const int i = i0 + lane / G;
        const bool on = i < hi && st[i] == step;  // the same in every lane of a group
        V acc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] = 0;
        if (on) {
          for (int e = d.icp[i] + sub; e < d.icp[i + 1]; e += G) {
            const V a = icv[e];
            const int j = d.icc[e];
#pragma unroll
            for (int k = 0; k < R; ++k) acc[k] = madd(a, xt[(size_t)j * R + k], acc[k]);
          }
        }
        group_sum<V, R>(acc, G);
        if (on && sub == 0) {
          V sr[R];
          ldv<V, R>(src + (size_t)i * R, sr);
          const V di = dg[i];
#pragma unroll
          for (int k = 0; k < R; ++k) xt[(size_t)(i - lo) * R + k] = (sr[k] - acc[k]) / di;
        }
      }
      sync();
    }
  }
}

// One tile per block of one wavefront (it.lo = tile), its iterate staged in
// LDS (T * R values).  from_b: the iterate before the step is zero, src = b.
template <typename V, int R>
__device__ __forceinline__ void kb_hsgs_body(const Item& it, const BDesc& d, int from_b) {
  extern __shared__ double hs_lds[];
  V* xt = reinterpret_cast<V*>(hs_lds);
  const int lo = it.lo * d.T, hi = min(d.n, lo + d.T);
  const int lane = (int)threadIdx.x;
  V* x = static_cast<V*>(d.x);
  const int m = (hi - lo) * R;
  for (int q = lane; q < m; q += WAVE) xt[q] = from_b ? (V)0 : x[(size_t)lo * R + q];
  __syncthreads();
  hybrid_tile<V, R>(d, lo, hi, static_cast<const V*>(from_b ? d.b : d.t), xt, lane, [] { __syncthreads(); });
  for (int q = lane; q < m; q += WAVE) x[(size_t)lo * R + q] = xt[q];
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(WAVE) void kb_hsgs(AMG_KARGS, int from_b) {
  AMG_BODY((kb_hsgs_body<V, R>), from_b)
}

// In-tile sum of one row from LDS couplings ev/ec over [e0, e1): lane `sub`
// of a group of G adds entries e0 + sub, e0 + sub + G, ... in that order (as
// hybrid_tile does), eight at a time with their loads and gathers in flight
// together.
template <typename V, int R>
__device__ __forceinline__ void lds_row_sum(const V* __restrict__ ev, const unsigned short* __restrict__ ec,
                                            const V* xt, int e0, int e1, int sub, int G, V (&acc)[R]) {
  for (int eb = e0 + sub; eb < e1; eb += 8 * G) {
    V a[8], xv[8][R];
    int j[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool v = eb + u * G < e1;
      a[u] = v ? ev[eb + u * G] : (V)0;
      j[u] = v ? (int)ec[eb + u * G] : 0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r) xv[u][r] = xt[(size_t)j[u] * R + r];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (eb + u * G < e1)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = madd(a[u], xv[u][r], acc[r]);
  }
}

// LDS layout of the staged sweep of a tile of T rows, at most C in-tile
// couplings per tile and at most S wavefront steps per sweep: iterate,
// source, diagonal (V); step bounds, coupling offsets (int); steps and
// rows by step (16 bit); then, 8-byte aligned, the couplings' values (V) and
// local columns (16 bit).
__host__ __device__ inline size_t hsgs_fixed_bytes(int T, int R, int S, size_t vb) {
  const size_t b = (size_t)T * (2 * R + 1) * vb + (size_t)(2 * (S + 1) + T + 1) * sizeof(int) +
                   (size_t)4 * T * sizeof(unsigned short);
  return (b + 7) & ~(size_t)7;
}
template <typename V>
__host__ __device__ inline size_t hsgs_lds_bytes(int T, int C, int R, int S) {
  return hsgs_fixed_bytes(T, R, S, sizeof(V)) + (size_t)C * (sizeof(V) + sizeof(unsigned short));
}

// Exclusive prefix sum of c[0..m) in place by one wavefront (returns the total).
__device__ inline int wave_exclusive_scan(int* c, int m, int lane) {
  int carry = 0;
  for (int b0 = 0; b0 < m; b0 += WAVE) {
    const int s = b0 + lane;
    const int v = s < m ? c[s] : 0;
    int inc = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int y = __shfl_up(inc, o, WAVE);
      if (lane >= o) inc += y;
    }
    if (s < m) c[s] = carry + inc - v;
    carry += __shfl(inc, WAVE - 1, WAVE);
  }
  return carry;
}

// The same sweeps with everything a step reads staged in LDS first, by
// contiguous copies: the tile's iterate and source, its diagonal, its rows'
// in-tile couplings (the level's compact lists, SELL entry order, as in
// hybrid_tile) and, for each sweep, the tile's rows listed step by step
// (counting sort on the step), so that a step's rows sit side by side on the
// lane groups.  W: the most in-tile couplings of a row, C: of a tile, S: the
// most steps of a sweep + 1 (over the launch's entries).
template <typename V, int R>
__device__ __forceinline__ void kb_hsgs_lds_body(const Item& it, const BDesc& d, int from_b, int W, int S, int C) {
  extern __shared__ double hs_lds[];
  const int T = d.T;
  V* xt = reinterpret_cast<V*>(hs_lds);
  V* sr = xt + (size_t)T * R;
  V* dl = sr + (size_t)T * R;
  int* so = reinterpret_cast<int*>(dl + T);  // [2][S + 1] step bounds
  int* cp = so + 2 * (S + 1);                // [T + 1] coupling offsets
  unsigned short* stf = reinterpret_cast<unsigned short*>(cp + T + 1);
  unsigned short* stb = stf + T;
  unsigned short* lst = stb + T;  // [2][T] rows by step
  V* ev = reinterpret_cast<V*>(reinterpret_cast<char*>(hs_lds) + hsgs_fixed_bytes(T, R, S, sizeof(V)));
  unsigned short* ec = reinterpret_cast<unsigned short*>(ev + C);
  const int lo = it.lo * T, hi = min(d.n, lo + T), nt = hi - lo;
  const int lane = (int)threadIdx.x;
  V* x = static_cast<V*>(d.x);
  const V* src = static_cast<const V*>(from_b ? d.b : d.t);
  const V* icv = Mat<V>::icv(d);
  const V* dg = Mat<V>::dg(d);
  const int c0 = d.icp[lo], m = d.icp[hi] - c0;
  for (int q = lane; q < 2 * (S + 1); q += WAVE) so[q] = 0;
  // couplings: four loads of each kind in flight per lane
  for (int k0 = 0; k0 < m; k0 += 4 * WAVE) {
    V a[4];
    unsigned short j[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * WAVE + lane;
      a[u] = k < m ? icv[c0 + k] : (V)0;
      j[u] = k < m ? d.icc[c0 + k] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * WAVE + lane;
      if (k < m) {
        ev[k] = a[u];
        ec[k] = j[u];
      }
    }
  }
  for (int q = lane; q <= nt; q += WAVE) cp[q] = d.icp[lo + q] - c0;
  for (int q = lane; q < nt; q += WAVE) {
    const int i = lo + q;
    stf[q] = d.hsf[i];
    stb[q] = d.hsb[i];
    dl[q] = dg[i];
  }
  for (int q = lane; q < nt * R; q += WAVE) {
    sr[q] = src[(size_t)lo * R + q];
    xt[q] = from_b ? (V)0 : x[(size_t)lo * R + q];
  }
  __syncthreads();
  // this tile's deepest steps (the sweeps stop there)
  int df = 0, db = 0;
  for (int q = lane; q < nt; q += WAVE) {
    df = max(df, (int)stf[q]);
    db = max(db, (int)stb[q]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    df = max(df, __shfl_xor(df, o, WAVE));
    db = max(db, __shfl_xor(db, o, WAVE));
  }
  if (T <= 2 * WAVE && W <= 8 && d.hg == 1) {
    // Small tiles with few couplings (the finest levels): each lane keeps its
    // two rows' couplings, steps, source and diagonal in registers, so a step
    // is one round of LDS gathers; same entry order and arithmetic.
    int cq[2], sfq[2], sbq[2];
    V aq[2][8], sq[2][R], dq[2];
    int jq[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = lane + h * WAVE;
      const bool on = q < nt;
      const int e0 = on ? cp[q] : 0;
      cq[h] = on ? cp[q + 1] - e0 : 0;
      sfq[h] = on ? (int)stf[q] : -1;
      sbq[h] = on ? (int)stb[q] : -1;
      dq[h] = on ? dl[q] : (V)1;
#pragma unroll
      for (int k = 0; k < R; ++k) sq[h][k] = on ? sr[(size_t)q * R + k] : (V)0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool e = u < cq[h];
        aq[h][u] = e ? ev[e0 + u] : (V)0;
        jq[h][u] = e ? (int)ec[e0 + u] : 0;
      }
    }
    for (int dir = 0; dir < 2; ++dir) {
      const int depth = dir == 0 ? df : db;
      for (int step = dir; step <= depth; ++step) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if ((dir == 0 ? sfq[h] : sbq[h]) != step) continue;
          const int q = lane + h * WAVE;
          V acc[R];
#pragma unroll
          for (int k = 0; k < R; ++k) acc[k] = 0;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (u < cq[h])
#pragma unroll
              for (int k = 0; k < R; ++k) acc[k] = madd(aq[h][u], xt[(size_t)jq[h][u] * R + k], acc[k]);
#pragma unroll
          for (int k = 0; k < R; ++k) xt[(size_t)q * R + k] = (sq[h][k] - acc[k]) / dq[h];
        }
        __syncthreads();
      }
    }
  } else {
    // rows by step: counts, bounds, placement (the order inside a step is free)
    for (int dir = 0; dir < 2; ++dir) {
      const unsigned short* st = dir == 0 ? stf : stb;
      int* c = so + dir * (S + 1);
      for (int q = lane; q < nt; q += WAVE) atomicAdd(&c[st[q]], 1);
      __syncthreads();
      wave_exclusive_scan(c, S + 1, lane);
      __syncthreads();
      for (int q = lane; q < nt; q += WAVE) lst[dir * T + atomicAdd(&c[st[q]], 1)] = (unsigned short)q;
    }
    __syncthreads();  // c[s] is now the end of step s's rows
    const int G = d.hg, sub = lane % G, ng = WAVE / G;
    for (int dir = 0; dir < 2; ++dir) {
      const int depth = dir == 0 ? df : db;
      const int* c = so + dir * (S + 1);
      const unsigned short* ls = lst + dir * T;
      for (int step = dir; step <= depth; ++step) {
        const int r1 = c[step];
        for (int p0 = step == 0 ? 0 : c[step - 1]; p0 < r1; p0 += ng) {
          const int p = p0 + lane / G;
          const bool on = p < r1;
          const int q = on ? (int)ls[p] : 0;
          V acc[R];
#pragma unroll
          for (int k = 0; k < R; ++k) acc[k] = 0;
          if (on) lds_row_sum<V, R>(ev, ec, xt, cp[q], cp[q + 1], sub, G, acc);
          group_sum<V, R>(acc, G);
          if (on && sub == 0)
#pragma unroll
            for (int k = 0; k < R; ++k) xt[(size_t)q * R + k] = (sr[(size_t)q * R + k] - acc[k]) / dl[q];
        }
        __syncthreads();
      }
    }
  }
  for (int q = lane; q < nt * R; q += WAVE) x[(size_t)lo * R + q] = xt[q];
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(WAVE) void kb_hsgs_lds(AMG_KARGS, int from_b, int W, int S, int C) {
  AMG_BODY((kb_hsgs_lds_body<V, R>), from_b, W, S, C)
}

// The tile-ordered multicolour smoother on one tile (one wavefront, it.lo =
// tile): the level's solve order takes each tile's rows colour by colour, so
// the rows of a colour are one contiguous range and the sweeps go colour by
// colour, forward then backward (the backward sweep starts below the tile's
// last colour, whose rows it would recompute bit for bit).  Rows of one
// colour are not coupled, so this is the sequential sweep in (colour, row)
// order.  Everything is staged in LDS by contiguous copies; rows are summed
// by groups of d.hg lanes as in hybrid_tile (same couplings, same order), so
// the one-workgroup tail, which sweeps such a level by its wavefront steps,
// gives the same bits.  C: the most in-tile couplings of a tile, NC: the
// most colours (over the launch's entries, below WAVE).
template <typename V, int R>
__device__ __forceinline__ void kb_tsgs_body(const Item& it, const BDesc& d, int from_b, int C, int NC) {
  extern __shared__ double hs_lds[];
  const int T = d.T;
  V* xt = reinterpret_cast<V*>(hs_lds);
  V* sr = xt + (size_t)T * R;
  V* dl = sr + (size_t)T * R;
  int* cp = reinterpret_cast<int*>(dl + T);  // [T + 1] coupling offsets
  int* cb = cp + T + 1;                      // [ncol + 1] colour bounds
  V* ev = reinterpret_cast<V*>(reinterpret_cast<char*>(hs_lds) + tsgs_fixed_bytes(T, R, NC, sizeof(V)));
  unsigned short* ec = reinterpret_cast<unsigned short*>(ev + C);
  const int lo = it.lo * T, hi = min(d.n, lo + T), nt = hi - lo;
  const int lane = (int)threadIdx.x, ncol = d.tncol;
  V* x = static_cast<V*>(d.x);
  const V* src = static_cast<const V*>(from_b ? d.b : d.t);
  const V* icv = Mat<V>::icv(d);
  const V* dg = Mat<V>::dg(d);
  const int c0 = d.icp[lo], m = d.icp[hi] - c0;
  // row data two rows per lane at a time, then couplings sixteen per lane at
  // a time: each batch's loads in flight together, then its LDS stores
  for (int q0 = 0; q0 <= nt; q0 += 2 * WAVE) {
    int cv[2];
    V dv[2], sv[2][R], xv[2][R];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = q0 + h * WAVE + lane;
      const int qr = min(q, nt - 1);  // clamped: loads without branches, stores guarded
      cv[h] = d.icp[lo + min(q, nt)];
      dv[h] = dg[lo + qr];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        sv[h][r] = src[(size_t)(lo + qr) * R + r];
        xv[h][r] = from_b ? (V)0 : x[(size_t)(lo + qr) * R + r];
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = q0 + h * WAVE + lane;
      if (q <= nt) cp[q] = cv[h] - c0;
      if (q < nt) {
        dl[q] = dv[h];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          sr[(size_t)q * R + r] = sv[h][r];
          xt[(size_t)q * R + r] = xv[h][r];
        }
      }
    }
  }
  for (int q = lane; q <= ncol; q += WAVE) cb[q] = d.tcb[(size_t)it.lo * (ncol + 1) + q];
  if (m == 0 && lane == 0) {  // no couplings: the clamped reads below find a valid slot
    ev[0] = (V)0;
    ec[0] = 0;
  }
  for (int k0 = 0; k0 < m; k0 += 16 * WAVE) {
    V a[16];
    unsigned short j[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = c0 + min(k0 + u * WAVE + lane, m - 1);
      a[u] = icv[k];
      j[u] = d.icc[k];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + u * WAVE + lane;
      if (k < m) {
        ev[k] = a[u];
        ec[k] = j[u];
      }
    }
  }
  __syncthreads();
  // Work units: the rows of a colour in groups of ng (one row per lane
  // group), forward colours 0..last then backward last-1..0, the tile's last
  // colour with rows being `last`.  The read-only data of the next unit (row
  // bounds, source, diagonal, the first eight couplings of each lane) is
  // loaded while the current unit sums, so a unit waits on its gathers of
  // the iterate alone; units of one colour need no barrier between them.
  const int G = d.hg, sub = lane % G, ng = WAVE / G;
  // colour bounds in one register (lane c holds bound c; ncol < WAVE): the
  // loop control reads them without waiting on LDS
  const int cbv = lane <= ncol ? cb[lane] : 0;
  auto cbu = [&](int c) { return __builtin_amdgcn_readlane(cbv, c); };
  int last = ncol - 1;
  while (last > 0 && cbu(last) == cbu(last + 1)) --last;
  const int K = 2 * last + 1;
  auto col = [&](int k) { return k <= last ? k : 2 * last - k; };
  auto first_unit = [&](int k, int& p0) {  // first colour at or after k with rows
    while (k < K && cbu(col(k)) == cbu(col(k) + 1)) ++k;
    if (k < K) p0 = cbu(col(k));
    return k;
  };
  struct Unit {
    int q, e0, e1;
    bool on;
    V s[R], dv, a[8];
    int j[8];
  };
  auto load_unit = [&](int c, int p0, Unit& u) {
    const int r1 = cbu(c + 1);
    u.q = p0 + lane / G;
    u.on = u.q < r1;
    const int qq = u.on ? u.q : r1 - 1;  // a row of the colour: every read stays in range
    u.e0 = cp[qq];
    u.e1 = cp[qq + 1];
    u.dv = dl[qq];
#pragma unroll
    for (int r = 0; r < R; ++r) u.s[r] = sr[(size_t)qq * R + r];
    const int el = u.e1 > 0 ? u.e1 - 1 : 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = min(u.e0 + sub + t * G, el);
      u.a[t] = ev[e];
      u.j[t] = ec[e];
    }
  };
  int p0 = 0;
  int k = first_unit(0, p0);
  Unit cur, nxt;
  if (k < K) load_unit(col(k), p0, cur);
  while (k < K) {
    const int c = col(k);
    int np0 = p0 + ng, nk = k;
    if (np0 >= cbu(c + 1)) nk = first_unit(k + 1, np0);
    if (nk < K) load_unit(col(nk), np0, nxt);
    V acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;
    {
      V xv[8][R];
#pragma unroll
      for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int r = 0; r < R; ++r) xv[t][r] = xt[(size_t)cur.j[t] * R + r];
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (cur.on && cur.e0 + sub + t * G < cur.e1)
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = madd(cur.a[t], xv[t][r], acc[r]);
      // rows with more than 8 G couplings go on in the same order
      if (cur.on && cur.e1 - cur.e0 > 8 * G) lds_row_sum<V, R>(ev, ec, xt, cur.e0 + 8 * G, cur.e1, sub, G, acc);
    }
    group_sum<V, R>(acc, G);
    if (cur.on && sub == 0)
#pragma unroll
      for (int r = 0; r < R; ++r) xt[(size_t)cur.q * R + r] = (cur.s[r] - acc[r]) / cur.dv;
    if (nk != k) __syncthreads();
    cur = nxt;
    k = nk;
    p0 = np0;
  }
  for (int q = lane; q < nt * R; q += WAVE) x[(size_t)lo * R + q] = xt[q];
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(WAVE) void kb_tsgs(AMG_KARGS, int from_b, int C, int NC) {
  AMG_BODY((kb_tsgs_body<V, R>), from_b, C, NC)
}

// Register form of the colour-ordered tile sweep (one right-hand side,
// tiles of at most 256 rows, at most WM in-tile couplings per row): one
// thread per row for the whole sweep, keeping the row's couplings, source,
// diagonal and colour in registers, so a colour step waits on the gathers of
// the iterate (in LDS, sixteen in flight) alone.  Each row sums its
// couplings one after another in SELL entry order (the level's lanes per
// row is 1), as hybrid_tile does.  The couplings pass through LDS once, by
// contiguous copies, on their way to the registers.
template <typename V, int WM>
__device__ __forceinline__ void kb_tsgs_reg_body(const Item& it, const BDesc& d, int mode, int C) {
  // mode bit 0: the iterate is zero before the sweep (source b); bit 1: also
  // write each row's in-tile sum with the final iterate to t (the first part
  // of kb_resid_tile's residual)
  const int from_b = mode & 1;
  extern __shared__ double hs_lds[];
  const int T = d.T, nthr = (int)blockDim.x;
  V* xt = reinterpret_cast<V*>(hs_lds);
  V* ev = xt + T;
  unsigned short* ec = reinterpret_cast<unsigned short*>(ev + C);
  const int lo = it.lo * T, hi = min(d.n, lo + T), nt = hi - lo;
  const int q = (int)threadIdx.x, lane = __lane_id();
  V* x = static_cast<V*>(d.x);
  const V* src = static_cast<const V*>(from_b ? d.b : d.t);
  const V* icv = Mat<V>::icv(d);
  const V* dg = Mat<V>::dg(d);
  const int c0 = d.icp[lo], m = d.icp[hi] - c0;
  const bool on = q < nt;
  const int qr = min(q, nt - 1);  // clamped: loads without branches
  const int a0 = d.icp[lo + qr], a1 = d.icp[lo + qr + 1];
  const int e0 = a0 - c0, cnt = on ? a1 - a0 : 0;
  const int cl = on ? d.tcol[lo + qr] : -1;
  const V sv = src[lo + qr], dv = dg[lo + qr];
  const V x0 = from_b ? (V)0 : x[lo + qr];
  // the tile's last colour with rows (bounds of colour `lane`, every wavefront alike)
  const int ncol = d.tncol;
  const int* cbt = d.tcb + (size_t)it.lo * (ncol + 1);
  const bool ne = lane < ncol && cbt[lane] < cbt[lane + 1];
  const unsigned long long nem = __builtin_amdgcn_ballot_w64(ne);
  const int last = nem ? 63 - __builtin_clzll(nem) : 0;
  if (on) xt[q] = x0;
  if (m == 0 && q == 0) {
    ev[0] = (V)0;
    ec[0] = 0;
  }
  for (int k0 = 0; k0 < m; k0 += 16 * nthr) {
    V a[16];
    unsigned short j[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = c0 + min(k0 + u * nthr + q, m - 1);
      a[u] = icv[k];
      j[u] = d.icc[k];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + u * nthr + q;
      if (k < m) {
        ev[k] = a[u];
        ec[k] = j[u];
      }
    }
  }
  __syncthreads();
  V a[WM];
  int j[WM];
#pragma unroll
  for (int u = 0; u < WM; ++u) {
    const int e = u < cnt ? e0 + u : 0;
    a[u] = ev[e];
    j[u] = ec[e];
  }
  for (int k = 0; k < 2 * last + 1; ++k) {
    const int c = k <= last ? k : 2 * last - k;
    const bool act = cl == c;
    V acc = 0;
    constexpr int CH = WM % 16 == 0 ? 16 : 8;  // gathers in flight per round
#pragma unroll
    for (int u0 = 0; u0 < WM; u0 += CH) {
      if (!__builtin_amdgcn_ballot_w64(act && cnt > u0)) break;  // no row of this wavefront and colour has more
      V xv[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) xv[u] = xt[j[u0 + u]];
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (u0 + u < cnt) acc = madd(a[u0 + u], xv[u], acc);
    }
    if (act) xt[q] = (sv - acc) / dv;
    __syncthreads();
  }
  if (on) x[lo + q] = xt[q];
  if (mode & 2) {
    V acc = 0;
#pragma unroll
    for (int u0 = 0; u0 < WM; u0 += 8) {
      if (!__builtin_amdgcn_ballot_w64(cnt > u0)) break;
      V xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = xt[j[u0 + u]];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u0 + u < cnt) acc = madd(a[u0 + u], xv[u], acc);
    }
    if (on) static_cast<V*>(d.t)[lo + q] = acc;
  }
}
template <typename V, int WM, bool DIRECT>
__global__ __launch_bounds__(256) void kb_tsgs_reg(AMG_KARGS, int mode, int C) {
  AMG_BODY((kb_tsgs_reg_body<V, WM>), mode, C)
}

template <typename V, int R>
__device__ __forceinline__ void kb_zero_body(const Item& it, const BDesc& d) {
  V* x = static_cast<V*>(d.x);
  V z[R];
#pragma unroll
  for (int k = 0; k < R; ++k) z[k] = 0;
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += (int)blockDim.x) stv<V, R>(x + (size_t)i * R, z);
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_zero(AMG_KARGS) {
  AMG_BODY((kb_zero_body<V, R>))
}

template <typename V, int R>
__device__ __forceinline__ void kb_jacobi_body(const Item& it, const BDesc& d) {
  V* x = static_cast<V*>(d.x);
  const V* t = static_cast<const V*>(d.t);
  const V* l1 = Mat<V>::l1(d);
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += (int)blockDim.x) {
    V xv[R], tv[R];
    ldv<V, R>(x + (size_t)i * R, xv);
    ldv<V, R>(t + (size_t)i * R, tv);
    const V di = l1[i];
#pragma unroll
    for (int k = 0; k < R; ++k) xv[k] = xv[k] + tv[k] / di;
    stv<V, R>(x + (size_t)i * R, xv);
  }
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_jacobi(AMG_KARGS) {
  AMG_BODY((kb_jacobi_body<V, R>))
}

// b_c[I] = sum of t over the members of aggregate I (ascending), coarse rows
// [lo, hi) in natural coarse order (neighbouring threads gather neighbouring
// fine rows); the sum goes to I's solve row.
template <typename V, int R>
__device__ __forceinline__ void kb_restrict_body(const Item& it, const BDesc& d) {
  const int I = it.lo + (int)threadIdx.x;
  if (I >= it.hi) return;
  const V* t = static_cast<const V*>(d.t);
  V s[R];
#pragma unroll
  for (int k = 0; k < R; ++k) s[k] = 0;
  // members eight at a time: their indices, then their residuals, in flight
  // together; the sum keeps the member order
  const int p1 = d.mptr[I + 1];
  for (int p0 = d.mptr[I]; p0 < p1; p0 += 8) {
    int m[8];
    V tv[8][R];
#pragma unroll
    for (int u = 0; u < 8; ++u) m[u] = d.members[min(p0 + u, p1 - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) ldv<V, R>(t + (size_t)m[u] * R, tv[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (p0 + u < p1)
#pragma unroll
        for (int k = 0; k < R; ++k) s[k] += tv[u][k];
  }
  stv<V, R>(static_cast<V*>(d.bc) + (size_t)(d.cinv ? d.cinv[I] : I) * R, s);
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_restrict(AMG_KARGS) {
  AMG_BODY((kb_restrict_body<V, R>))
}

// x_i += omega x_c[agg_i], rows [lo, hi).
template <typename V, int R>
__device__ __forceinline__ void kb_prolong_body(const Item& it, const BDesc& d) {
  V* x = static_cast<V*>(d.x);
  const V* xc = static_cast<const V*>(d.xc);
  const V om = (V)d.omega;
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += (int)blockDim.x) {
    V xv[R], cv[R];
    ldv<V, R>(x + (size_t)i * R, xv);
    ldv<V, R>(xc + (size_t)d.agg[i] * R, cv);
#pragma unroll
    for (int k = 0; k < R; ++k) xv[k] = madd(om, cv[k], xv[k]);
    stv<V, R>(x + (size_t)i * R, xv);
  }
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_prolong(AMG_KARGS) {
  AMG_BODY((kb_prolong_body<V, R>))
}

// x = A_L^{-1} b on the coarsest level: one wavefront per row (rows
// [lo, hi), at most 4), lanes over the contiguous row, FP64 accumulation.
template <typename V, int R>
__device__ __forceinline__ void kb_coarse_body(const Item& it, const BDesc& d) {
  const int i = it.lo + (int)(threadIdx.x / WAVE);
  if (i >= it.hi) return;
  const int lane = __lane_id(), n = d.nL;
  const V* b = static_cast<const V*>(d.b);
  const double* row = d.Ainv + (size_t)i * n;
  double s[R];
#pragma unroll
  for (int k = 0; k < R; ++k) s[k] = 0.0;
  for (int j = lane; j < n; j += WAVE) {
    const double a = row[j];
    V bv[R];
    ldv<V, R>(b + (size_t)j * R, bv);
#pragma unroll
    for (int k = 0; k < R; ++k) s[k] = madd(a, (double)bv[k], s[k]);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) s[k] = wave_sum_d(s[k]);
  if (lane == 0) {
    V o[R];
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = (V)s[k];
    stv<V, R>(static_cast<V*>(d.x) + (size_t)i * R, o);
  }
}
template <typename V, int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_coarse(AMG_KARGS) {
  AMG_BODY((kb_coarse_body<V, R>))
}

// ---------------------------------------------------------------- coarse tail
// The V-cycle below level lt of one entry in one workgroup (TAIL_NT threads):
// levels lt..lc-1 and the coarsest solve, passes separated by workgroup
// barriers instead of kernel launches.  Every pass applies the same per-row
// bodies as the launches of the larger levels (one wavefront per slice, one
// thread per row), so the result does not depend on where the tail starts.
constexpr int TAIL_NT = 1024;

// op: 0 residual, 1 Gauss-Seidel pass, 2 Gauss-Seidel pass from x = 0.
template <typename V, int R>
__device__ inline void tail_slices(const BDesc& d, int s0, int s1, int op) {
  const int nw = (int)blockDim.x / WAVE;
  for (int lo = s0; lo < s1; lo += nw) {
    const Item it{0, lo, min(s1, lo + nw), 0};
    if (op == 1)
      kb_gs_body<V, R>(it, d);
    else if (op == 2)
      kb_gs0_body<V, R>(it, d);
    else
      kb_resid_body<V, R>(it, d);
  }
  __syncthreads();
}

// The colour passes of the separate launches, in the same order (d.sm: the
// level's smoother).
template <typename V, int R>
__device__ inline void tail_smooth(const BDesc& d, int sweeps, bool from_zero) {
  int prev = -1;  // a pass on the colour just updated would repeat its values
  for (int k = 0; k < sweeps; ++k) {
    if (d.sm == AMG_SMOOTHER_MCSGS) {
      for (int dir = 0; dir < 2; ++dir)
        for (int q = 0; q < d.ncol; ++q) {
          const int c = dir == 0 ? q : d.ncol - 1 - q;
          if (c == prev) continue;
          tail_slices<V, R>(d, d.sptr[c], d.sptr[c + 1], from_zero && prev < 0 ? 2 : 1);
          prev = c;
        }
    } else if (d.sm == AMG_SMOOTHER_HYBRID_SGS || d.sm == AMG_SMOOTHER_TILE_MCSGS) {
      // wavefronts take tiles; the sweeps work on the level's vector in
      // place (tiles only read their own rows), steps separated by barriers
      const bool zero = from_zero && k == 0;
      if (!zero) {
        kb_resid_off_body<V, R>(Item{0, 0, d.n, 0}, d);
        __syncthreads();
      }
      const int nw = (int)blockDim.x / WAVE, wv = (int)threadIdx.x / WAVE;
      const int ntl = (d.n + d.T - 1) / d.T;
      const V* src = static_cast<const V*>(zero ? d.b : d.t);
      for (int t0 = 0; t0 < ntl; t0 += nw) {
        const int lo = min(d.n, (t0 + wv) * d.T), hi = min(d.n, lo + d.T);
        hybrid_tile<V, R>(d, lo, hi, src, static_cast<V*>(d.x) + (size_t)lo * R, __lane_id(),
                          [] { __syncthreads(); });
      }
    } else {
      tail_slices<V, R>(d, 0, d.nsl, 0);
      kb_jacobi_body<V, R>(Item{0, 0, d.n, 0}, d);
      __syncthreads();
    }
  }
}

// Levels lt..lc-1 of one entry by one workgroup, where launches would be
// latency bound: the down-leg (up = 0: x = 0, pre-smoothing, residual,
// restriction) or the up-leg (up = 1: prolongation, post-smoothing).  The
// coarsest solve between them is a separate many-block launch.
// it.d: descriptor of level lt (level l at D[it.d + l - lt]); it.lo = lt, it.hi = lc.
template <typename V, int R>
__global__ __launch_bounds__(TAIL_NT) void kb_tail(const Item* __restrict__ tab, const BDesc* __restrict__ D,
                                                    const Item base, int pre, int post, int direct,
                                                    int up) {
  const Item it = direct ? base : tab[blockIdx.x];
  const BDesc* dl = D + it.d;
  if (!direct && dl->active == 0) return;
  const int lt = it.lo, lc = it.hi;
  const int nt = (int)blockDim.x;
  if (!up) {
    for (int l = lt; l < lc; ++l) {
      const BDesc& d = dl[l - lt];
      kb_zero_body<V, R>(Item{0, 0, d.n, 0}, d);
      __syncthreads();
      tail_smooth<V, R>(d, pre, true);
      if (d.sm == AMG_SMOOTHER_HYBRID_SGS || d.sm == AMG_SMOOTHER_TILE_MCSGS) {
        kb_resid_tile_body<V, R>(Item{0, 0, d.n, 0}, d, 0);
        __syncthreads();
      } else {
        tail_slices<V, R>(d, 0, d.nsl, 0);
      }
      for (int lo = 0; lo < d.nc; lo += nt) kb_restrict_body<V, R>(Item{0, lo, min(d.nc, lo + nt), 0}, d);
      __syncthreads();
    }
  } else {
    for (int l = lc - 1; l >= lt; --l) {
      const BDesc& d = dl[l - lt];
      kb_prolong_body<V, R>(Item{0, 0, d.n, 0}, d);
      __syncthreads();
      tail_smooth<V, R>(d, post, false);
    }
  }
}

// FP32 cycle: level-0 right-hand side = (float) r; z = (double) x.
template <int R>
__device__ __forceinline__ void kb_r2b_body(const Item& it, const BDesc& d) {
  float* b = static_cast<float*>(d.b);
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += NT) {
    double rv[R];
    float o[R];
    ldv<double, R>(d.r + (size_t)i * R, rv);
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = (float)rv[k];
    stv<float, R>(b + (size_t)i * R, o);
  }
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_r2b(AMG_KARGS) {
  AMG_BODY((kb_r2b_body<R>))
}

template <int R>
__device__ __forceinline__ void kb_x2z_body(const Item& it, const BDesc& d) {
  const float* x = static_cast<const float*>(d.x);
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += NT) {
    float xv[R];
    double o[R];
    ldv<float, R>(x + (size_t)i * R, xv);
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = (double)xv[k];
    stv<double, R>(d.z + (size_t)i * R, o);
  }
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_x2z(AMG_KARGS) {
  AMG_BODY((kb_x2z_body<R>))
}

// ---------------------------------------------------------------- CG vectors
// zx: z is the FP32 level-0 iterate of the cycle, widened here (exactly), so
// the FP64 z is never stored during the iterations.
template <int R>
__device__ inline void load_z(const BDesc& d, int i, int zx, double (&zv)[R]) {
  if (zx) {
    float xv[R];
    ldv<float, R>(static_cast<const float*>(d.x) + (size_t)i * R, xv);
#pragma unroll
    for (int k = 0; k < R; ++k) zv[k] = (double)xv[k];
  } else {
    ldv<double, R>(d.z + (size_t)i * R, zv);
  }
}

// b32: the FP32 right-hand side of the cycle's level 0 is (float) r, written
// where r is produced, so the next cycle needs no separate conversion.
template <int R>
__device__ inline void store_b32(const BDesc& d, int i, const double (&rv)[R]) {
  float o[R];
#pragma unroll
  for (int k = 0; k < R; ++k) o[k] = (float)rv[k];
  stv<float, R>(static_cast<float*>(d.b) + (size_t)i * R, o);
}

// Partials of r.z and (flexible) z.(r - r_old) over the rows [lo, hi).
template <int R>
__device__ __forceinline__ void kb_dots_rz_body(const Item& it, const BDesc& d, int zx) {
  double a[R], c[R];
#pragma unroll
  for (int k = 0; k < R; ++k) a[k] = c[k] = 0.0;
  const bool flex = d.rold != nullptr;
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += NT) {
    double rv[R], zv[R];
    ldv<double, R>(d.r + (size_t)i * R, rv);
    load_z<R>(d, i, zx, zv);
#pragma unroll
    for (int k = 0; k < R; ++k) a[k] = madd(rv[k], zv[k], a[k]);
    if (flex) {
      double ov[R];
      ldv<double, R>(d.rold + (size_t)i * R, ov);
#pragma unroll
      for (int k = 0; k < R; ++k) c[k] = madd(zv[k], rv[k] - ov[k], c[k]);
    }
  }
  block_sums<R>(a);
  block_sums<R>(c);
  write_partials<R>(d, 0, it.part, a);
  write_partials<R>(d, 1, it.part, c);
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_dots_rz(AMG_KARGS, int zx) {
  AMG_BODY((kb_dots_rz_body<R>), zx)
}

// p = z (first direction) or p = z + beta p, rows [lo, hi).
template <int R>
__device__ __forceinline__ void kb_update_p_body(const Item& it, const BDesc& d, int zx) {
  bool skip[R], first[R];
  double beta[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    skip[k] = frozen(d, k);
    first[k] = d.scal[k * S_COUNT + S_NEWP] != 0.0;
    beta[k] = d.scal[k * S_COUNT + S_BETA];
  }
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += NT) {
    double pv[R], zv[R];
    ldv<double, R>(d.p + (size_t)i * R, pv);
    load_z<R>(d, i, zx, zv);
#pragma unroll
    for (int k = 0; k < R; ++k)
      if (!skip[k]) pv[k] = first[k] ? zv[k] : madd(beta[k], pv[k], zv[k]);
    stv<double, R>(d.p + (size_t)i * R, pv);
  }
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_update_p(AMG_KARGS, int zx) {
  AMG_BODY((kb_update_p_body<R>), zx)
}

// q = A p (FP64, SELL slices [lo, hi), wavefront w takes lo + w, lo + w + 4, ...)
// with partials of p.q.  (STREAM: the level's entries and diagonal exceed the
// last-level cache and are loaded with the non-temporal hint, as in the
// colour passes.)
template <int R, bool STREAM>
__device__ __forceinline__ void kb_spmv_dot_body_t(const Item& it, const BDesc& d) {
  const int lane = __lane_id();
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0.0;
  for (int sl = it.lo + (int)(threadIdx.x / WAVE); sl < it.hi; sl += NT / WAVE) {
    const int r = d.srow[sl] + lane;
    const int base = d.soff[sl], w = (d.soff[sl + 1] - base) >> 6;
    double off[R];
    sell_offdiag_t<double, R, STREAM>(d.scol, d.sval64, base, w, lane, d.p, off);
    if (r < d.srow[sl + 1]) {
      double pr[R], y[R];
      ldv<double, R>(d.p + (size_t)r * R, pr);
      const double dg = ld_stream<STREAM>(d.dg64 + r);
#pragma unroll
      for (int k = 0; k < R; ++k) {
        y[k] = madd(dg, pr[k], off[k]);
        acc[k] = madd(pr[k], y[k], acc[k]);
      }
      stv<double, R>(d.q + (size_t)r * R, y);
    }
  }
  block_sums<R>(acc);
  write_partials<R>(d, 0, it.part, acc);
}
template <int R>
__device__ __forceinline__ void kb_spmv_dot_body(const Item& it, const BDesc& d) {
  if (d.nt)
    kb_spmv_dot_body_t<R, true>(it, d);
  else
    kb_spmv_dot_body_t<R, false>(it, d);
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_spmv_dot(AMG_KARGS) {
  AMG_BODY((kb_spmv_dot_body<R>))
}

// out = b - A x (FP64, SELL) with partials of out.out; out is r (which = 0)
// or q (which = 1), b and x the entry's right-hand side and iterate.
template <int R, bool STREAM>
__device__ __forceinline__ void kb_resid_dot_body_t(const Item& it, const BDesc& d, int which) {
  const int lane = __lane_id();
  const bool b32 = (which & 2) != 0;
  double* out = (which & 1) ? d.q : d.r;
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0.0;
  for (int sl = it.lo + (int)(threadIdx.x / WAVE); sl < it.hi; sl += NT / WAVE) {
    const int r = d.srow[sl] + lane;
    const int base = d.soff[sl], w = (d.soff[sl + 1] - base) >> 6;
    double off[R];
    sell_offdiag_t<double, R, STREAM>(d.scol, d.sval64, base, w, lane, d.xs, off);
    if (r < d.srow[sl + 1]) {
      double xr[R], br[R], o[R];
      ldv<double, R>(d.xs + (size_t)r * R, xr);
      ldv<double, R>(d.bs + (size_t)r * R, br);
      const double dg = ld_stream<STREAM>(d.dg64 + r);
#pragma unroll
      for (int k = 0; k < R; ++k) {
        o[k] = br[k] - madd(dg, xr[k], off[k]);
        acc[k] = madd(o[k], o[k], acc[k]);
      }
      stv<double, R>(out + (size_t)r * R, o);
      if (b32) store_b32<R>(d, r, o);
    }
  }
  block_sums<R>(acc);
  write_partials<R>(d, 0, it.part, acc);
}
template <int R>
__device__ __forceinline__ void kb_resid_dot_body(const Item& it, const BDesc& d, int which) {
  if (d.nt)
    kb_resid_dot_body_t<R, true>(it, d, which);
  else
    kb_resid_dot_body_t<R, false>(it, d, which);
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_resid_dot(AMG_KARGS, int which) {
  AMG_BODY((kb_resid_dot_body<R>), which)
}

// CSR level 0 (one-level hierarchies): SUB lanes per row read the row as one
// contiguous stream and combine with a SUB-wide butterfly.
template <int SUB>
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int o = SUB / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, SUB);
  return v;
}

template <int R, int SUB>
__device__ inline void csr_row(const BDesc& d, int i, int sl, const double* x, double (&s)[R]) {
#pragma unroll
  for (int k = 0; k < R; ++k) s[k] = 0.0;
  for (int e = d.rowptr[i] + sl; e < d.rowptr[i + 1]; e += SUB) {
    const double a = d.vals[e];
    double xv[R];
    ldv<double, R>(x + (size_t)d.colind[e] * R, xv);
#pragma unroll
    for (int k = 0; k < R; ++k) s[k] = madd(a, xv[k], s[k]);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) s[k] = group_sum<SUB>(s[k]);
}

template <int R, int SUB>
__device__ __forceinline__ void kb_spmv_dot_csr_body(const Item& it, const BDesc& d) {
  const int sl = threadIdx.x % SUB;
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0.0;
  for (int i = it.lo + (int)threadIdx.x / SUB; i < it.hi; i += NT / SUB) {
    double s[R];
    csr_row<R, SUB>(d, i, sl, d.p, s);
    if (sl == 0) {
      double pr[R];
      ldv<double, R>(d.p + (size_t)i * R, pr);
#pragma unroll
      for (int k = 0; k < R; ++k) acc[k] = madd(pr[k], s[k], acc[k]);
      stv<double, R>(d.q + (size_t)i * R, s);
    }
  }
  block_sums<R>(acc);
  write_partials<R>(d, 0, it.part, acc);
}
template <int R, int SUB, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_spmv_dot_csr(AMG_KARGS) {
  AMG_BODY((kb_spmv_dot_csr_body<R, SUB>))
}

template <int R, int SUB>
__device__ __forceinline__ void kb_resid_dot_csr_body(const Item& it, const BDesc& d, int which) {
  const int sl = threadIdx.x % SUB;
  const bool b32 = (which & 2) != 0;
  double* out = (which & 1) ? d.q : d.r;
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0.0;
  for (int i = it.lo + (int)threadIdx.x / SUB; i < it.hi; i += NT / SUB) {
    double s[R];
    csr_row<R, SUB>(d, i, sl, d.xs, s);
    if (sl == 0) {
      double br[R], o[R];
      ldv<double, R>(d.bs + (size_t)i * R, br);
#pragma unroll
      for (int k = 0; k < R; ++k) {
        o[k] = br[k] - s[k];
        acc[k] = madd(o[k], o[k], acc[k]);
      }
      stv<double, R>(out + (size_t)i * R, o);
      if (b32) store_b32<R>(d, i, o);
    }
  }
  block_sums<R>(acc);
  write_partials<R>(d, 0, it.part, acc);
}
template <int R, int SUB, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_resid_dot_csr(AMG_KARGS, int which) {
  AMG_BODY((kb_resid_dot_csr_body<R, SUB>), which)
}

// x += alpha p; r_old = r (flexible); r -= alpha q; partials of r.r, rows
// [lo, hi).  A frozen right-hand side keeps x, r and r_old.
template <int R>
__device__ __forceinline__ void kb_update_xr_body(const Item& it, const BDesc& d, int b32) {
  bool skip[R], anyskip = false;
  double alpha[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    skip[k] = frozen(d, k);
    anyskip |= skip[k];
    alpha[k] = d.scal[k * S_COUNT + S_ALPHA];
  }
  const bool flex = d.rold != nullptr;
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0.0;
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += NT) {
    double xv[R], rv[R], pv[R], qv[R], ov[R];
    ldv<double, R>(d.xs + (size_t)i * R, xv);
    ldv<double, R>(d.r + (size_t)i * R, rv);
    ldv<double, R>(d.p + (size_t)i * R, pv);
    ldv<double, R>(d.q + (size_t)i * R, qv);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      ov[k] = rv[k];
      if (!skip[k]) {
        xv[k] = madd(alpha[k], pv[k], xv[k]);
        rv[k] = madd(-alpha[k], qv[k], rv[k]);
      }
      acc[k] = madd(rv[k], rv[k], acc[k]);
    }
    stv<double, R>(d.xs + (size_t)i * R, xv);
    stv<double, R>(d.r + (size_t)i * R, rv);
    if (b32) store_b32<R>(d, i, rv);
    if (flex) {
      if (anyskip) {
        double keep[R];
        ldv<double, R>(d.rold + (size_t)i * R, keep);
#pragma unroll
        for (int k = 0; k < R; ++k)
          if (!skip[k]) keep[k] = ov[k];
        stv<double, R>(d.rold + (size_t)i * R, keep);
      } else {
        stv<double, R>(d.rold + (size_t)i * R, ov);
      }
    }
  }
  block_sums<R>(acc);
  write_partials<R>(d, 0, it.part, acc);
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_update_xr(AMG_KARGS, int b32) {
  AMG_BODY((kb_update_xr_body<R>), b32)
}

template <int R>
__device__ __forceinline__ void kb_dot_bb_body(const Item& it, const BDesc& d) {
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0.0;
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += NT) {
    double bv[R];
    ldv<double, R>(d.bs + (size_t)i * R, bv);
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = madd(bv[k], bv[k], acc[k]);
  }
  block_sums<R>(acc);
  write_partials<R>(d, 0, it.part, acc);
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_dot_bb(AMG_KARGS) {
  AMG_BODY((kb_dot_bb_body<R>))
}

template <int R>
__device__ __forceinline__ void kb_vzero_rold_body(const Item& it, const BDesc& d) {
  double z[R];
#pragma unroll
  for (int k = 0; k < R; ++k) z[k] = 0.0;
  for (int i = it.lo + (int)threadIdx.x; i < it.hi; i += NT) stv<double, R>(d.rold + (size_t)i * R, z);
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_vzero_rold(AMG_KARGS) {
  AMG_BODY((kb_vzero_rold_body<R>))
}

// One block per entry: sums the entry's it.lo partials per right-hand side in
// index order (fixed tree) and applies the scalar step `op`.
template <int R>
__device__ __forceinline__ void kb_finish_body(const Item& it, const BDesc& d, int op, int slot) {
  const int nparts = it.lo;
  double a[R], c[R];
#pragma unroll
  for (int k = 0; k < R; ++k) a[k] = c[k] = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NT) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      a[k] += d.partial[(size_t)i * R + k];
      if (op == FIN_BETA_FCG) c[k] += d.partial[((size_t)RED_BLOCKS + i) * R + k];
    }
  }
  block_sums<R>(a);
  block_sums<R>(c);
  if (threadIdx.x != 0) return;
  for (int k = 0; k < R; ++k) {
    double* sc = d.scal + k * S_COUNT;
    switch (op) {
      case FIN_STORE:
        sc[slot] = a[k];
        break;
      case FIN_INIT:
        sc[S_R0] = a[k];
        sc[S_RR] = a[k];
        sc[S_NEWP] = 1.0;
        sc[S_FLAG] = 0.0;
        break;
      case FIN_ALPHA:
        if (d.ctl[1 + k] != 0) break;
        sc[S_PQ] = a[k];
        if (!(a[k] > 0.0)) sc[S_FLAG] = 1.0;
        sc[S_ALPHA] = sc[S_RHO] / a[k];
        sc[S_NEWP] = 0.0;
        break;
      case FIN_BETA_PCG:
      case FIN_BETA_FCG: {
        if (d.ctl[1 + k] != 0) break;
        sc[S_RZ] = a[k];
        sc[S_ZDR] = c[k];
        if (!(a[k] > 0.0)) sc[S_FLAG] = 1.0;
        if (sc[S_NEWP] != 0.0)
          sc[S_BETA] = 0.0;
        else if (a[k] > 0.0)
          sc[S_BETA] = (op == FIN_BETA_FCG ? c[k] : a[k]) / sc[S_RHO];
        sc[S_RHO] = a[k];
        break;
      }
    }
  }
}
template <int R, bool DIRECT>
__global__ __launch_bounds__(NT) void kb_finish(AMG_KARGS, int op, int slot) {
  AMG_BODY((kb_finish_body<R>), op, slot)
}

// ---------------------------------------------------------------- user vectors
// out[r * R + k] = in[k * n + perm[r]]
__global__ void k_gather_rhs(int n, int R, const int* __restrict__ perm, const double* __restrict__ in,
                             double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * R) return;
  const int r = (int)(e / R), k = (int)(e % R);
  out[e] = in[(size_t)k * n + (perm ? perm[r] : r)];
}

__global__ void k_scatter_rhs(int n, int R, const int* __restrict__ perm, const double* __restrict__ in,
                              double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * R) return;
  const int r = (int)(e / R), k = (int)(e % R);
  out[(size_t)k * n + (perm ? perm[r] : r)] = in[e];
}

#define AMG_SUB_DISPATCH(SUBV, CALL) \
  switch (SUBV) {                    \
    case 4: {                        \
      constexpr int SUB = 4;         \
      CALL;                          \
    } break;                         \
    case 8: {                        \
      constexpr int SUB = 8;         \
      CALL;                          \
    } break;                         \
    case 16: {                       \
      constexpr int SUB = 16;        \
      CALL;                          \
    } break;                         \
    case 32: {                       \
      constexpr int SUB = 32;        \
      CALL;                          \
    } break;                         \
    default: {                       \
      constexpr int SUB = 64;        \
      CALL;                          \
    } break;                         \
  }

#define AMG_STRIP(...) __VA_ARGS__
// Launches the direct or the table variant of kernel KNAME<TARGS..., DIRECT>.
#define AMG_LAUNCH(KNAME, TARGS, ...)                                                                  \
  do {                                                                                                 \
    if (L.use_direct)                                                                                  \
      hipLaunchKernelGGL((KNAME<AMG_STRIP TARGS, true>), g, b, 0, s, nullptr, nullptr, Dh[L.direct.d], \
                         L.direct, ##__VA_ARGS__);                                                     \
    else                                                                                               \
      hipLaunchKernelGGL((KNAME<AMG_STRIP TARGS, false>), g, b, 0, s, t, D, BDesc{}, Item{}, ##__VA_ARGS__); \
  } while (0)

template <typename V, int R>
void launch_cycle_op(const Launch& L, const Item* t, const BDesc* D, const BDesc* Dh, hipStream_t s) {
  const dim3 g(L.nblk), b(NT);
  switch (L.op) {
    case OP_ZERO: AMG_LAUNCH(kb_zero, (V, R)); break;
    case OP_GS: AMG_LAUNCH(kb_gs, (V, R)); break;
    case OP_GS0: AMG_LAUNCH(kb_gs0, (V, R)); break;
    case OP_GS_RESID: AMG_LAUNCH(kb_gsr, (V, R)); break;
    case OP_RESID: AMG_LAUNCH(kb_resid, (V, R)); break;
    case OP_RESID_OFF: AMG_LAUNCH(kb_resid_off, (V, R)); break;
    case OP_HSGS: {
      // one wavefront per tile: everything staged in LDS when it fits in
      // 64 KiB (aux2 = W | S << 16: the most in-tile couplings of a row, the
      // most steps of a sweep + 1; aux3: the most in-tile couplings of a
      // tile), else the iterate alone
      const dim3 bw(WAVE);
      const int T = Dh[L.direct.d].T;
      const int W = L.aux2 & 0xffff, S = L.aux2 >> 16, C = L.aux3;
      const size_t full = hsgs_lds_bytes<V>(T, C, R, S);
      if (full <= 65536) {
        if (L.use_direct)
          hipLaunchKernelGGL((kb_hsgs_lds<V, R, true>), g, bw, full, s, nullptr, nullptr, Dh[L.direct.d], L.direct,
                             L.aux, W, S, C);
        else
          hipLaunchKernelGGL((kb_hsgs_lds<V, R, false>), g, bw, full, s, t, D, BDesc{}, Item{}, L.aux, W, S, C);
        break;
      }
      const size_t lds = (size_t)T * R * sizeof(V);
      if (L.use_direct)
        hipLaunchKernelGGL((kb_hsgs<V, R, true>), g, bw, lds, s, nullptr, nullptr, Dh[L.direct.d], L.direct, L.aux);
      else
        hipLaunchKernelGGL((kb_hsgs<V, R, false>), g, bw, lds, s, t, D, BDesc{}, Item{}, L.aux);
    } break;
    case OP_TSGS: {
      // one thread per row for one right-hand side, tiles of at most 256
      // rows and at most 32 in-tile couplings per row (aux3 >> 16: the most
      // of the launch's entries); else one wavefront per tile, staged in LDS
      // when it fits in 64 KiB (aux2: the most in-tile couplings of a tile,
      // aux3 & 0xffff: the most colours), else the hybrid sweeps by
      // wavefront steps on the iterate alone
      const dim3 bw(WAVE);
      const int T = Dh[L.direct.d].T, C = L.aux2, NC = L.aux3 & 0xffff, W = L.aux3 >> 16;
      if (tsgs_reg_ok(R, T, W, C, sizeof(V))) {
        const size_t lds = tsgs_reg_lds_bytes(T, C, sizeof(V));
        const dim3 bt((T + WAVE - 1) / WAVE * WAVE);  // one thread per row
#define AMG_TSGS_REG(WM)                                                                                        \
  do {                                                                                                         \
    if (L.use_direct)                                                                                          \
      hipLaunchKernelGGL((kb_tsgs_reg<V, WM, true>), g, bt, lds, s, nullptr, nullptr, Dh[L.direct.d], L.direct, \
                         L.aux, C);                                                                            \
    else                                                                                                       \
      hipLaunchKernelGGL((kb_tsgs_reg<V, WM, false>), g, bt, lds, s, t, D, BDesc{}, Item{}, L.aux, C);         \
  } while (0)
        if (W <= 16)
          AMG_TSGS_REG(16);
        else if (W <= 24)
          AMG_TSGS_REG(24);
        else
          AMG_TSGS_REG(32);
#undef AMG_TSGS_REG
        break;
      }
      const size_t full = tsgs_lds_bytes(T, C, R, NC, sizeof(V));
      if (full <= 65536) {
        if (L.use_direct)
          hipLaunchKernelGGL((kb_tsgs<V, R, true>), g, bw, full, s, nullptr, nullptr, Dh[L.direct.d], L.direct,
                             L.aux & 1, C, NC);
        else
          hipLaunchKernelGGL((kb_tsgs<V, R, false>), g, bw, full, s, t, D, BDesc{}, Item{}, L.aux & 1, C, NC);
        break;
      }
      const size_t lds = (size_t)T * R * sizeof(V);
      if (L.use_direct)
        hipLaunchKernelGGL((kb_hsgs<V, R, true>), g, bw, lds, s, nullptr, nullptr, Dh[L.direct.d], L.direct,
                           L.aux & 1);
      else
        hipLaunchKernelGGL((kb_hsgs<V, R, false>), g, bw, lds, s, t, D, BDesc{}, Item{}, L.aux & 1);
    } break;
    case OP_RESID_TILE: AMG_LAUNCH(kb_resid_tile, (V, R), L.aux); break;
    case OP_JACOBI: AMG_LAUNCH(kb_jacobi, (V, R)); break;
    case OP_BGS: AMG_LAUNCH(kb_bgs, (V, R)); break;
    case OP_RESTRICT: AMG_LAUNCH(kb_restrict, (V, R)); break;
    case OP_PROLONG: AMG_LAUNCH(kb_prolong, (V, R)); break;
    case OP_COARSE: AMG_LAUNCH(kb_coarse, (V, R)); break;
    case OP_TAIL:
    case OP_TAIL_UP: {
      const int up = L.op == OP_TAIL_UP ? 1 : 0;
      if (L.use_direct)
        hipLaunchKernelGGL((kb_tail<V, R>), dim3(1), dim3(TAIL_NT), 0, s, nullptr, D, L.direct, L.aux2 >> 8,
                           L.aux2 & 255, 1, up);
      else
        hipLaunchKernelGGL((kb_tail<V, R>), dim3(L.nblk), dim3(TAIL_NT), 0, s, t, D, Item{}, L.aux2 >> 8,
                           L.aux2 & 255, 0, up);
    } break;
    default: fail(AMG_ERR_HIP, "unknown cycle launch");
  }
}

template <int R>
void launch_r(const Launch& L, const Item* t, const BDesc* D, const BDesc* Dh, int fp32, hipStream_t s) {
  const dim3 g(L.nblk), b(NT);
  switch (L.op) {
    case OP_ZERO:
    case OP_GS:
    case OP_GS0:
    case OP_GS_RESID:
    case OP_RESID:
    case OP_RESID_OFF:
    case OP_HSGS:
    case OP_TSGS:
    case OP_RESID_TILE:
    case OP_BGS:
    case OP_JACOBI:
    case OP_RESTRICT:
    case OP_PROLONG:
    case OP_COARSE:
    case OP_TAIL:
    case OP_TAIL_UP:
      if (fp32)
        launch_cycle_op<float, R>(L, t, D, Dh, s);
      else
        launch_cycle_op<double, R>(L, t, D, Dh, s);
      break;
    case OP_R2B: AMG_LAUNCH(kb_r2b, (R)); break;
    case OP_X2Z: AMG_LAUNCH(kb_x2z, (R)); break;
    case OP_DOTS_RZ: AMG_LAUNCH(kb_dots_rz, (R), L.aux); break;
    case OP_UPDATE_P: AMG_LAUNCH(kb_update_p, (R), L.aux); break;
    case OP_SPMV_DOT: AMG_LAUNCH(kb_spmv_dot, (R)); break;
    case OP_SPMV_DOT_CSR: AMG_SUB_DISPATCH(L.aux, AMG_LAUNCH(kb_spmv_dot_csr, (R, SUB))); break;
    case OP_UPDATE_XR: AMG_LAUNCH(kb_update_xr, (R), L.aux); break;
    case OP_RESID_DOT: AMG_LAUNCH(kb_resid_dot, (R), L.aux); break;
    case OP_RESID_DOT_CSR: AMG_SUB_DISPATCH(L.aux2, AMG_LAUNCH(kb_resid_dot_csr, (R, SUB), L.aux)); break;
    case OP_DOT_BB: AMG_LAUNCH(kb_dot_bb, (R)); break;
    case OP_VZERO_ROLD: AMG_LAUNCH(kb_vzero_rold, (R)); break;
    case OP_FINISH: AMG_LAUNCH(kb_finish, (R), L.aux, L.aux2); break;
    default: fail(AMG_ERR_HIP, "unknown launch");
  }
}

}  // namespace

void issue_launches(const std::vector<Launch>& Ls, size_t first, size_t last, const Item* tab, const BDesc* D,
                    const BDesc* Dh, int R, int fp32, hipStream_t s) {
  for (size_t i = first; i < last; ++i) {
    const Launch& L = Ls[i];
    if (L.nblk <= 0) continue;
    KTimer tm(L.kind, s, L.bytes);
    const Item* t = L.use_direct ? nullptr : tab + L.off;  // direct launches take no table
    switch (R) {
      case 1: launch_r<1>(L, t, D, Dh, fp32, s); break;
      case 2: launch_r<2>(L, t, D, Dh, fp32, s); break;
      case 4: launch_r<4>(L, t, D, Dh, fp32, s); break;
      case 8: launch_r<8>(L, t, D, Dh, fp32, s); break;
      default: fail(AMG_ERR_UNSUPPORTED, "right-hand sides per entry must be 1, 2, 4 or 8");
    }
  }
  AMG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- BiCGSTAB
// Level-0 kernels of the BiCGSTAB iteration (Sec. 5), one right-hand side in
// FP64 and solve order.  A reduction splits its rows (or slices) into nb fixed
// chunks, one per block, and leaves two partial sums per block; the finish
// kernel adds them in block order, so results do not depend on scheduling.
// The scalars (BS_*) stay on the device: a block reads them once, and an
// update kernel does nothing after a breakdown or a half-step exit.
namespace {

__device__ inline void bcg_partials(double* part, double a0, double a1) {
  double a[2] = {a0, a1};
  block_sums<2>(a);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a[0];
    part[2 * blockIdx.x + 1] = a[1];
  }
}

// y = A x (SELL-64 slices [lo, lo + ch) of the block), or c - A x.
__global__ __launch_bounds__(NT) void kk_spmv_sell(const BDesc d, int ch, const double* __restrict__ x,
                                                   const double* __restrict__ c, double* __restrict__ y,
                                                   const double* __restrict__ w, double* __restrict__ part) {
  const int lo = (int)blockIdx.x * ch, hi = min(d.nsl, lo + ch);
  const int lane = __lane_id();
  double wy = 0.0, yy = 0.0;
  for (int sl = lo + (int)(threadIdx.x / WAVE); sl < hi; sl += NT / WAVE) {
    const int r = d.srow[sl] + lane;
    const int base = d.soff[sl], wd = (d.soff[sl + 1] - base) >> 6;
    double off[1];
    sell_offdiag<double, 1>(d.scol, d.sval64, base, wd, lane, x, off, d.nt != 0);
    if (r < d.srow[sl + 1]) {
      double v = madd(d.dg64[r], x[r], off[0]);
      if (c) v = c[r] - v;
      y[r] = v;
      if (w) wy = madd(w[r], v, wy);
      yy = madd(v, v, yy);
    }
  }
  bcg_partials(part, wy, yy);
}

// The same over CSR rows [lo, lo + ch), SUB lanes per row.
template <int SUB>
__global__ __launch_bounds__(NT) void kk_spmv_csr(const BDesc d, int ch, const double* __restrict__ x,
                                                  const double* __restrict__ c, double* __restrict__ y,
                                                  const double* __restrict__ w, double* __restrict__ part) {
  const int lo = (int)blockIdx.x * ch, hi = min(d.n, lo + ch);
  const int sl = threadIdx.x % SUB;
  double wy = 0.0, yy = 0.0;
  for (int i = lo + (int)threadIdx.x / SUB; i < hi; i += NT / SUB) {
    double sum[1];
    csr_row<1, SUB>(d, i, sl, x, sum);
    if (sl == 0) {
      const double v = c ? c[i] - sum[0] : sum[0];
      y[i] = v;
      if (w) wy = madd(w[i], v, wy);
      yy = madd(v, v, yy);
    }
  }
  bcg_partials(part, wy, yy);
}

__device__ inline bool bcg_stopped(const double* sc) { return sc[BS_FLAG] != 0.0 || sc[BS_HALF] != 0.0; }

__global__ __launch_bounds__(NT) void kk_bcg_half(int n, int ch, const double* __restrict__ r,
                                                  const double* __restrict__ v, const double* __restrict__ ph,
                                                  double* __restrict__ x, double* __restrict__ sv,
                                                  const double* __restrict__ sc, double* __restrict__ part) {
  if (bcg_stopped(sc)) return;
  const double alpha = sc[BS_ALPHA];
  const int lo = (int)blockIdx.x * ch, hi = min(n, lo + ch);
  double ss = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += NT) {
    const double si = madd(-alpha, v[i], r[i]);
    sv[i] = si;
    x[i] = madd(alpha, ph[i], x[i]);
    ss = madd(si, si, ss);
  }
  bcg_partials(part, 0.0, ss);
}

__global__ __launch_bounds__(NT) void kk_bcg_full(int n, int ch, const double* __restrict__ sv,
                                                  const double* __restrict__ t, const double* __restrict__ sh,
                                                  const double* __restrict__ rt, double* __restrict__ x,
                                                  double* __restrict__ r, const double* __restrict__ sc,
                                                  double* __restrict__ part) {
  if (bcg_stopped(sc)) return;
  const double omega = sc[BS_OMEGA];
  const int lo = (int)blockIdx.x * ch, hi = min(n, lo + ch);
  double tr = 0.0, rr = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += NT) {
    x[i] = madd(omega, sh[i], x[i]);
    const double ri = madd(-omega, t[i], sv[i]);
    r[i] = ri;
    tr = madd(rt[i], ri, tr);
    rr = madd(ri, ri, rr);
  }
  bcg_partials(part, tr, rr);
}

__global__ __launch_bounds__(NT) void kk_bcg_dir(int n, const double* __restrict__ r, const double* __restrict__ v,
                                                 double* __restrict__ p, double* __restrict__ pin,
                                                 double* __restrict__ rt, const double* __restrict__ sc,
                                                 int init) {
  const int i = (int)blockIdx.x * NT + (int)threadIdx.x;
  if (i >= n) return;
  if (init) {
    const double ri = r[i];
    p[i] = ri;
    pin[i] = ri;
    rt[i] = ri;
    return;
  }
  if (bcg_stopped(sc)) return;
  const double pi = madd(sc[BS_BETA], madd(-sc[BS_OMEGA], v[i], p[i]), r[i]);
  p[i] = pi;
  pin[i] = pi;
}

__global__ __launch_bounds__(NT) void kk_norm2(int n, int ch, const double* __restrict__ u,
                                               double* __restrict__ part) {
  const int lo = (int)blockIdx.x * ch, hi = min(n, lo + ch);
  double uu = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += NT) uu = madd(u[i], u[i], uu);
  bcg_partials(part, 0.0, uu);
}

__device__ inline bool is_finite_d(double v) { return v - v == 0.0; }

// One block: sums the partials in block order, then the scalar step of `op`.
// Convergence is tested as in the oracle: ||.||^2 <= tol2 = (rtol ||r_0||)^2.
__global__ __launch_bounds__(NT) void kk_bcg_finish(int op, int nb, const double* __restrict__ part,
                                                    double* __restrict__ sc, double tol2) {
  double a0 = 0.0, a1 = 0.0;
  for (int i = (int)threadIdx.x; i < nb; i += NT) {
    a0 += part[2 * i];
    a1 += part[2 * i + 1];
  }
  double a[2] = {a0, a1};
  block_sums<2>(a);
  if (threadIdx.x != 0) return;
  switch (op) {
    case BF_INIT:  // r_0 = b - A x_0; r~ = r_0, so rho = r_0.r_0
      for (int k = 0; k < BS_COUNT; ++k) sc[k] = 0.0;
      sc[BS_RR0] = sc[BS_RR] = sc[BS_RHO] = a[1];
      break;
    case BF_ALPHA:
      if (bcg_stopped(sc)) break;
      if (!(a[0] != 0.0) || !is_finite_d(a[0]))
        sc[BS_FLAG] = 1.0;  // x unchanged
      else
        sc[BS_ALPHA] = sc[BS_RHO] / a[0];
      break;
    case BF_S:
      if (bcg_stopped(sc)) break;
      sc[BS_SS] = a[1];
      if (a[1] <= tol2) sc[BS_HALF] = 1.0;
      break;
    case BF_OMEGA: {
      if (bcg_stopped(sc)) break;
      const double om = a[0] / a[1];
      if (!(a[1] > 0.0) || !is_finite_d(a[1]) || !(om != 0.0) || !is_finite_d(om))
        sc[BS_FLAG] = 2.0;  // x holds the half step
      else
        sc[BS_OMEGA] = om;
    } break;
    case BF_BETA:
      if (bcg_stopped(sc)) break;
      sc[BS_RR] = a[1];
      if (a[1] <= tol2) break;  // converged: the host stops
      if (!(a[0] != 0.0) || !is_finite_d(a[0])) {
        sc[BS_FLAG] = 3.0;  // after the full iteration
      } else {
        sc[BS_BETA] = (a[0] / sc[BS_RHO]) * (sc[BS_ALPHA] / sc[BS_OMEGA]);
        sc[BS_RHO] = a[0];
      }
      break;
    case BF_TRUE: sc[BS_TMP] = a[1]; break;
    default: sc[BS_TMP2] = a[1]; break;
  }
}

int bcg_row_blocks(int n) { return std::min(1024, std::max(1, cdiv(n, 2048))); }

}  // namespace

int bcg_spmv(const BDesc& d0, int sub, const double* x, const double* c, double* y, const double* w, double* part,
             double bytes, hipStream_t s) {
  int nb;
  if (d0.scol) {
    nb = std::min(RED_BLOCKS, std::max(1, cdiv(d0.nsl, 32)));
    const int ch = cdiv(d0.nsl, nb);
    KTimer tm(AMG_KIND_SPMV_F64, s, bytes);
    hipLaunchKernelGGL(kk_spmv_sell, dim3(nb), dim3(NT), 0, s, d0, ch, x, c, y, w, part);
  } else {
    nb = bcg_row_blocks(d0.n);
    const int ch = cdiv(d0.n, nb);
    KTimer tm(AMG_KIND_SPMV_F64, s, bytes);
    AMG_SUB_DISPATCH(sub, hipLaunchKernelGGL((kk_spmv_csr<SUB>), dim3(nb), dim3(NT), 0, s, d0, ch, x, c, y, w,
                                                part));
  }
  AMG_HIP(hipGetLastError());
  return nb;
}

int bcg_half(int n, const double* r, const double* v, const double* ph, double* x, double* sv, const double* sc,
             double* part, hipStream_t s) {
  const int nb = bcg_row_blocks(n);
  KTimer tm(AMG_KIND_CG_VEC, s, 48.0 * n);
  hipLaunchKernelGGL(kk_bcg_half, dim3(nb), dim3(NT), 0, s, n, cdiv(n, nb), r, v, ph, x, sv, sc, part);
  AMG_HIP(hipGetLastError());
  return nb;
}

int bcg_full(int n, const double* sv, const double* t, const double* sh, const double* rt, double* x, double* r,
             const double* sc, double* part, hipStream_t s) {
  const int nb = bcg_row_blocks(n);
  KTimer tm(AMG_KIND_CG_VEC, s, 56.0 * n);
  hipLaunchKernelGGL(kk_bcg_full, dim3(nb), dim3(NT), 0, s, n, cdiv(n, nb), sv, t, sh, rt, x, r, sc, part);
  AMG_HIP(hipGetLastError());
  return nb;
}

void bcg_dir(int n, const double* r, const double* v, double* p, double* pin, double* rt, const double* sc,
             int init, hipStream_t s) {
  KTimer tm(AMG_KIND_CG_VEC, s, init ? 32.0 * n : 40.0 * n);
  hipLaunchKernelGGL(kk_bcg_dir, dim3(cdiv(n, NT)), dim3(NT), 0, s, n, r, v, p, pin, rt, sc, init);
  AMG_HIP(hipGetLastError());
}

int bcg_norm2(int n, const double* u, double* part, hipStream_t s) {
  const int nb = bcg_row_blocks(n);
  KTimer tm(AMG_KIND_CG_VEC, s, 8.0 * n);
  hipLaunchKernelGGL(kk_norm2, dim3(nb), dim3(NT), 0, s, n, cdiv(n, nb), u, part);
  AMG_HIP(hipGetLastError());
  return nb;
}

void bcg_finish(int op, int nb, const double* part, double* sc, double tol2, hipStream_t s) {
  KTimer tm(AMG_KIND_CG_VEC, s, 16.0 * nb);
  hipLaunchKernelGGL(kk_bcg_finish, dim3(1), dim3(NT), 0, s, op, nb, part, sc, tol2);
  AMG_HIP(hipGetLastError());
}

void gather_rhs(int n, int R, const int* perm, const double* in, double* out, hipStream_t s) {
  const long long e = (long long)n * R;
  hipLaunchKernelGGL(k_gather_rhs, dim3(cdiv(e, 256)), dim3(256), 0, s, n, R, perm, in, out);
  AMG_HIP(hipGetLastError());
}

void scatter_rhs(int n, int R, const int* perm, const double* in, double* out, hipStream_t s) {
  const long long e = (long long)n * R;
  hipLaunchKernelGGL(k_scatter_rhs, dim3(cdiv(e, 256)), dim3(256), 0, s, n, R, perm, in, out);
  AMG_HIP(hipGetLastError());
}

}  // namespace amgx
