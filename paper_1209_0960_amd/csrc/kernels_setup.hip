// Setup kernels of the aggregation AMG hierarchy for gfx950 (wave64).
//
// Integer outputs (strong flags, aggregates, colours, coarse sparsity) are
// deterministic and independent of scheduling; the Galerkin values are ordered
// sequential sums, so the whole setup is reproducible bit for bit.  Floating
// point contraction is disabled in this file so that every FP64 operation of
// the strength test is rounded once.
#include <algorithm>
#include <climits>
#include <initializer_list>

#include "amg_internal.h"

#pragma clang fp contract(off)

namespace amgx {

namespace {

constexpr int WAVE = 64;

__device__ inline uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// Calls f(k, j) for the stored entries k of row i (column j), loading them in
// chunks of 8 whose loads are issued together.  The per-tile kernels walk
// their rows one per lane of a single wavefront, where entry-by-entry loads
// would be a chain of dependent memory round trips.
template <typename F>
__device__ __forceinline__ void for_entries(const int* __restrict__ rp, const int* __restrict__ ci, int i, F f) {
  const int b = rp[i], e = rp[i + 1];
  for (int k0 = b; k0 < e; k0 += 8) {
    int jj[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) jj[q] = k0 + q < e ? ci[k0 + q] : -1;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (jj[q] >= 0) f(k0 + q, jj[q]);
  }
}

__device__ inline int wave_incl_scan(int v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    int t = __shfl_up(v, d, WAVE);
    if (lane >= d) v += t;
  }
  return v;
}

// Wave reductions with DPP: two quad permutations and two row rotations give
// every lane its 16-lane row's result, then the four rows are combined from
// lanes 15, 31, 47 and 63.  Called with all 64 lanes active; the result is
// wave-uniform.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <typename Op>
__device__ __forceinline__ unsigned wave_reduce(unsigned v, Op op) {
  v = op(v, dpp_u32<0xB1>(v));   // quad_perm [1,0,3,2]
  v = op(v, dpp_u32<0x4E>(v));   // quad_perm [2,3,0,1]
  v = op(v, dpp_u32<0x124>(v));  // row_ror:4
  v = op(v, dpp_u32<0x128>(v));  // row_ror:8
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 15), b = (unsigned)__builtin_amdgcn_readlane((int)v, 31);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 47), d = (unsigned)__builtin_amdgcn_readlane((int)v, 63);
  return op(op(a, b), op(c, d));
}
__device__ inline int wave_sum(int v) {
  return (int)wave_reduce((unsigned)v, [](unsigned x, unsigned y) { return x + y; });
}
__device__ inline int wave_max(int v) {
  return (int)wave_reduce((unsigned)v, [](unsigned x, unsigned y) { return (unsigned)max((int)x, (int)y); });
}
__device__ inline int wave_min(int v) {
  return (int)wave_reduce((unsigned)v, [](unsigned x, unsigned y) { return (unsigned)min((int)x, (int)y); });
}
__device__ inline unsigned wave_or(unsigned v) {
  return wave_reduce(v, [](unsigned x, unsigned y) { return x | y; });
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_max_u64(unsigned long long v) {
  const unsigned lo = dpp_u32<CTRL>((unsigned)v), hi = dpp_u32<CTRL>((unsigned)(v >> 32));
  const unsigned long long o = ((unsigned long long)hi << 32) | lo;
  return o > v ? o : v;
}
__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
  v = dpp_max_u64<0xB1>(v);
  v = dpp_max_u64<0x4E>(v);
  v = dpp_max_u64<0x124>(v);
  v = dpp_max_u64<0x128>(v);
  unsigned long long r = 0;
#pragma unroll
  for (int l = 15; l < WAVE; l += 16) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    const unsigned long long x = ((unsigned long long)hi << 32) | lo;
    r = x > r ? x : r;
  }
  return r;
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// ============================================================== scan
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ int block_excl_scan(int v, int* total) {
  __shared__ int ws[SCAN_THREADS / WAVE];
  const int lane = __lane_id(), w = threadIdx.x / WAVE;
  int inc = wave_incl_scan(v);
  if (lane == WAVE - 1) ws[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_THREADS / WAVE; ++i) {
    int s = ws[i];
    off += (i < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(const int* __restrict__ in, int n, int* __restrict__ bsum) {
  const long long base = (long long)blockIdx.x * SCAN_TILE;
  int s = 0;
#pragma unroll
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    long long i = base + (long long)r * SCAN_THREADS + threadIdx.x;
    if (i < n) s += in[i];
  }
  int tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of nb block sums in place, single workgroup; bsum[nb] = total.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_top(int* bsum, int nb) {
  int carry = 0;
  for (int base = 0; base < nb; base += SCAN_THREADS) {
    int i = base + threadIdx.x;
    int v = i < nb ? bsum[i] : 0;
    int tot;
    int ex = block_excl_scan(v, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_final(const int* __restrict__ in, int n,
                                                             const int* __restrict__ bsum, int nb,
                                                             int* __restrict__ out) {
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int s = 0;
#pragma unroll
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    long long i = base + r;
    v[r] = i < n ? in[i] : 0;
    s += v[r];
  }
  int tot;
  int ex = block_excl_scan(s, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    long long i = base + r;
    if (i < n) out[i] = ex;
    ex += v[r];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = bsum[nb];
}

// ============================================================== validation
__global__ void k_validate_struct(int n, int nnz, const int* __restrict__ rp, const int* __restrict__ ci,
                                  const double* __restrict__ v, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f = 0;
  const int b = rp[i], e = rp[i + 1];
  if (i == 0 && b != 0) f |= 1;
  if (i == n - 1 && e != nnz) f |= 1;
  if (b < 0 || e < b || e > nnz) {
    atomicOr(flags, 1);
    return;
  }
  bool has_diag = false;
  double d = 0.0;
  for (int k = b; k < e; ++k) {
    const int j = ci[k];
    const double a = v[k];
    if (j < 0 || j >= n) f |= 1;
    if (k > b && ci[k - 1] >= j) f |= 1;
    if (!__builtin_isfinite(a)) f |= 1;
    if (j == i) {
      has_diag = true;
      d = a;
    }
  }
  if (!has_diag || !(d > 0.0)) f |= 2;
  if (f) atomicOr(flags, f);
}

__device__ inline int find_in_row(const int* __restrict__ rp, const int* __restrict__ ci, int row, int col) {
  int lo = rp[row], hi = rp[row + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int c = ci[mid];
    if (c == col) return mid;
    if (c < col)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

// The row kernels below give each row STR_SUB consecutive lanes, which take
// its entries in turn (a row's entries are read by neighbouring lanes), and
// each group of lanes STR_ROWS rows, 32 rows apart: the first STR_SUB entries
// of all of them (most rows have no more) are loaded together, so that their
// chains of dependent loads overlap; longer rows finish in a plain loop.
constexpr int STR_SUB = 8;
constexpr int STR_ROWS = 4;
constexpr int STR_GROUPS = 256 / STR_SUB;  // lane groups per block
constexpr int STR_BLOCK_ROWS = STR_GROUPS * STR_ROWS;
__device__ inline int str_row(int u) { return ((int)blockIdx.x * STR_ROWS + u) * STR_GROUPS + (int)threadIdx.x / STR_SUB; }

// Every off-diagonal a_ij has a stored a_ji (equal to it when `check`): the
// binary searches of a group's rows advance together.
__global__ __launch_bounds__(256) void k_validate_sym(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const double* __restrict__ v, int check, int* flags) {
  const int q0 = (int)threadIdx.x % STR_SUB;
  int i[STR_ROWS], b[STR_ROWS], e[STR_ROWS];
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    i[u] = str_row(u);
    b[u] = i[u] < n ? rp[i[u]] : 0;
    e[u] = i[u] < n ? rp[i[u] + 1] : 0;
  }
  int j[STR_ROWS], lo[STR_ROWS], hi[STR_ROWS], q[STR_ROWS];
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    const int k = b[u] + q0;
    j[u] = k < e[u] ? ci[k] : i[u];
  }
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    const bool act = j[u] != i[u];
    lo[u] = act ? rp[j[u]] : 0;
    hi[u] = act ? rp[j[u] + 1] - 1 : -1;
    q[u] = -1;
  }
  for (;;) {
    bool any = false;
#pragma unroll
    for (int u = 0; u < STR_ROWS; ++u) {
      if (lo[u] > hi[u]) continue;
      any = true;
      const int mid = (lo[u] + hi[u]) >> 1;
      const int c = ci[mid];
      if (c == i[u]) {
        q[u] = mid;
        lo[u] = 1;
        hi[u] = 0;
      } else if (c < i[u]) {
        lo[u] = mid + 1;
      } else {
        hi[u] = mid - 1;
      }
    }
    if (!any) break;
  }
  bool bad = false;
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u)
    if (j[u] != i[u] && (q[u] < 0 || (check && v[q[u]] != v[b[u] + q0]))) bad = true;
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    if (i[u] >= n) continue;
    for (int k = b[u] + q0 + STR_SUB; k < e[u] && !bad; k += STR_SUB) {
      const int jj = ci[k];
      if (jj == i[u]) continue;
      const int qq = find_in_row(rp, ci, jj, i[u]);
      if (qq < 0 || (check && v[qq] != v[k])) bad = true;
    }
  }
  if (bad) atomicOr(flags, 4);
}

// ============================================================== strength
// Sec. 2.1, eqs. (symmetric_strong1)/(symmetric_strong2) on in-tile edges:
// w_E(i,j) = max(-a_ij, 0), w_V(i) = a_ii, s_ij = w_E(i,j) w_E(j,i) / (a_ii a_jj).
// sym: the values are known to be exactly symmetric (checked at setup), so
// a_ji is a_ij and the transposed entry need not be looked up.
__device__ inline double s_edge_v(double aij, double aji, double di, double dj) {
  const double wij = (-aij > 0.0) ? -aij : 0.0;
  const double wji = (-aji > 0.0) ? -aji : 0.0;
  const double num = wij * wji;
  const double den = di * dj;
  return num / den;
}
__device__ inline double a_ji(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                              int i, int j, double aij, bool sym) {
  if (sym) return aij;
  const int q = find_in_row(rp, ci, j, i);
  return q >= 0 ? v[q] : 0.0;
}
__device__ inline double s_edge(const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ v, const double* __restrict__ d, int i, int j,
                                double aij, bool sym) {
  double aji = aij;
  if (!sym) {
    const int q = find_in_row(rp, ci, j, i);
    aji = q >= 0 ? v[q] : 0.0;
  }
  return s_edge_v(aij, aji, d[i], d[j]);
}

__global__ __launch_bounds__(256) void k_diag(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                              const double* __restrict__ v, double* __restrict__ d) {
  const int q0 = (int)threadIdx.x % STR_SUB;
  int i[STR_ROWS], b[STR_ROWS], e[STR_ROWS], c[STR_ROWS];
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    i[u] = str_row(u);
    b[u] = i[u] < n ? rp[i[u]] : 0;
    e[u] = i[u] < n ? rp[i[u] + 1] : 0;
  }
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) c[u] = b[u] + q0 < e[u] ? ci[b[u] + q0] : -1;
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    if (c[u] == i[u]) d[i[u]] = v[b[u] + q0];
    for (int k = b[u] + q0 + STR_SUB; k < e[u]; k += STR_SUB)
      if (ci[k] == i[u]) d[i[u]] = v[k];
  }
}

// Whether the entry (i, j) is an edge of row i's tile subgraph, the edges whose
// strength eq. (symmetric_strong2) tests.
__device__ inline bool in_tile_edge(int n, int T, int i, int j) {
  const int lo = (i / T) * T, hi = min(lo + T, n);
  return j != i && j >= lo && j < hi;
}

__global__ __launch_bounds__(256) void k_eta(int n, int T, const int* __restrict__ rp, const int* __restrict__ ci,
                                             const double* __restrict__ v, const double* __restrict__ d,
                                             double* __restrict__ eta, int sym) {
  const int q0 = (int)threadIdx.x % STR_SUB;
  int i[STR_ROWS], b[STR_ROWS], e[STR_ROWS], j[STR_ROWS];
  double a[STR_ROWS], di[STR_ROWS], dj[STR_ROWS], em[STR_ROWS];
  bool in[STR_ROWS];
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    i[u] = str_row(u);
    b[u] = i[u] < n ? rp[i[u]] : 0;
    e[u] = i[u] < n ? rp[i[u] + 1] : 0;
  }
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    const int k = b[u] + q0;
    j[u] = k < e[u] ? ci[k] : i[u];
    a[u] = k < e[u] ? v[k] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    in[u] = i[u] < n && in_tile_edge(n, T, i[u], j[u]);
    di[u] = in[u] ? d[i[u]] : 1.0;
    dj[u] = in[u] ? d[j[u]] : 1.0;
  }
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    em[u] = 0.0;
    if (in[u]) {
      const double s = s_edge_v(a[u], a_ji(rp, ci, v, i[u], j[u], a[u], sym != 0), di[u], dj[u]);
      if (s > em[u]) em[u] = s;
    }
    if (i[u] < n)
      for (int k = b[u] + q0 + STR_SUB; k < e[u]; k += STR_SUB) {
        const int jj = ci[k];
        if (!in_tile_edge(n, T, i[u], jj)) continue;
        const double s = s_edge(rp, ci, v, d, i[u], jj, v[k], sym != 0);
        if (s > em[u]) em[u] = s;
      }
  }
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    double x = em[u];
#pragma unroll
    for (int o = STR_SUB / 2; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, STR_SUB));
    if (i[u] < n && q0 == 0) eta[i[u]] = x;
  }
}

__global__ __launch_bounds__(256) void k_strong(int n, int T, const int* __restrict__ rp, const int* __restrict__ ci,
                                                const double* __restrict__ v, const double* __restrict__ d,
                                                const double* __restrict__ eta, double delta, double beta,
                                                uint8_t* __restrict__ strong, uint8_t* __restrict__ iso, int sym) {
  const int q0 = (int)threadIdx.x % STR_SUB;
  int i[STR_ROWS], b[STR_ROWS], e[STR_ROWS], j[STR_ROWS];
  double a[STR_ROWS], ei[STR_ROWS], ej[STR_ROWS], di[STR_ROWS], dj[STR_ROWS];
  bool in[STR_ROWS];
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    i[u] = str_row(u);
    b[u] = i[u] < n ? rp[i[u]] : 0;
    e[u] = i[u] < n ? rp[i[u] + 1] : 0;
    ei[u] = i[u] < n ? eta[i[u]] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    const int k = b[u] + q0;
    j[u] = k < e[u] ? ci[k] : i[u];
    a[u] = k < e[u] ? v[k] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    in[u] = i[u] < n && in_tile_edge(n, T, i[u], j[u]);
    ej[u] = in[u] ? eta[j[u]] : 0.0;
    di[u] = in[u] ? d[i[u]] : 1.0;
    dj[u] = in[u] ? d[j[u]] : 1.0;
  }
#pragma unroll
  for (int u = 0; u < STR_ROWS; ++u) {
    if (i[u] >= n) continue;
    const int k0 = b[u] + q0;
    if (k0 < e[u]) {
      uint8_t f = 0;
      if (in[u]) {
        const double m = ei[u] < ej[u] ? ei[u] : ej[u];
        const double s = s_edge_v(a[u], a_ji(rp, ci, v, i[u], j[u], a[u], sym != 0), di[u], dj[u]);
        f = (s > delta * m) ? 1 : 0;
      }
      strong[k0] = f;
    }
    for (int k = k0 + STR_SUB; k < e[u]; k += STR_SUB) {
      const int jj = ci[k];
      uint8_t f = 0;
      if (in_tile_edge(n, T, i[u], jj)) {
        const double ejj = eta[jj];
        const double m = ei[u] < ejj ? ei[u] : ejj;
        const double s = s_edge(rp, ci, v, d, i[u], jj, v[k], sym != 0);
        f = (s > delta * m) ? 1 : 0;
      }
      strong[k] = f;
    }
    if (q0 == 0) iso[i[u]] = (ei[u] < beta) ? 1 : 0;
  }
}

// ============================================================== aggregation
// One wavefront per tile of T rows runs the greedy aggregation of Sec. 2.1
// (Alg. 1 with Alg. 2 and Alg. 3, singleton merge, isolated phase) on the tile
// subgraph (Alg. 4).  The tile graph lives in LDS as a local CSR of 16-bit
// neighbour indices with the strong flag in bit 15, and each vertex has one
// packed 32-bit state word.  Each selection step scores all front candidates
// in parallel (one per lane) and picks the winner with a butterfly reduction
// over a strict total order.
constexpr int AGG_MAX_T = 1024;
constexpr int AGG_MAX_SLOTS = 32;
// state word: bits 0-15 aggregate id (0xFFFF = none), 16-21 member slot of
// the current aggregate (63 = none), bit 22 isolated, bit 23 on the front.
constexpr unsigned ST_AGG = 0xFFFFu, ST_SLOT_SHIFT = 16, ST_SLOT_NONE = 63u << 16, ST_SLOT_MASK = 63u << 16;
constexpr unsigned ST_ISO = 1u << 22, ST_FRONT = 1u << 23;
// bits 24-29 of a front vertex: its strong links into the current aggregate
// (cons2), kept up to date as members are added.
constexpr unsigned ST_C2_SHIFT = 24, ST_C2_MASK = 63u << 24;

__device__ inline int st_agg(unsigned w) { return (int)(short)(w & ST_AGG); }
__device__ inline int st_slot(unsigned w) { return (int)((w >> ST_SLOT_SHIFT) & 63u); }

struct AggLayout {
  size_t lptr, st, cmm, niso, adjb, madj, nna, front, adjl, mem, ladj, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline AggLayout agg_layout(int T, int E) {
  AggLayout L;
  size_t o = 0;
  L.lptr = o; o = align16(o + 4 * (size_t)(T + 1));
  L.st = o; o = align16(o + 4 * (size_t)T);
  L.cmm = o; o = align16(o + 4 * (size_t)T);
  L.niso = o; o = align16(o + 2 * (size_t)T);
  L.adjb = o; o = align16(o + 4 * (size_t)((T + 31) / 32));
  L.madj = o; o = align16(o + 4 * (size_t)AGG_MAX_SLOTS);
  L.nna = o; o = align16(o + 2 * (size_t)T);
  L.front = o; o = align16(o + 2 * (size_t)T);
  L.adjl = o; o = align16(o + 2 * (size_t)T);
  L.mem = o; o = align16(o + 2 * (size_t)AGG_MAX_SLOTS);
  L.ladj = o; o = align16(o + 2 * (size_t)(E > 0 ? E : 1));
  L.total = o;
  return L;
}

struct AggSh {
  int* lptr;
  unsigned* st;
  unsigned* cmm;     // front vertex: mask of the member slots it is adjacent to
  short* niso;       // isolated in-tile neighbours per vertex
  unsigned* adjbits; // bit a: aggregate a is adjacent to the current aggregate
  unsigned* madj;
  short* nna;
  short* front;
  short* adjl;
  short* mem;
  unsigned short* ladj;
};

// Per-aggregate state, uniform across the wave.
struct AggState {
  int asize;   // members of the current aggregate
  int fcount;  // entries appended to the front list (candidates in N(a))
  int acount;  // entries appended to the adjacent-aggregate list
};

// Adds vertex c to aggregate `id`: marks it, updates the unaggregated
// neighbour counts, the member adjacency masks, the candidate front and the
// set of adjacent aggregates.  Phase 1 fronts hold non-isolated vertices and
// track every adjacent aggregate; the isolated phase fronts hold isolated
// vertices and track only aggregates of phase 1 (ids < P1).
__device__ void add_member(const AggSh& S, AggState& as, int c, int id, bool iso_phase, int P1) {
  const int lane = __lane_id();
  const int s = as.asize;
  if (lane == 0) {
    S.st[c] = (S.st[c] & ST_ISO) | ((unsigned)s << ST_SLOT_SHIFT) | ((unsigned)id & ST_AGG);
    S.mem[s] = (short)c;
  }
  __syncthreads();
  const int b = S.lptr[c], e = S.lptr[c + 1];
  unsigned bits = 0;
  for (int base = b; base < e; base += WAVE) {
    const int k = base + lane;
    int j = 0, aj = 0;
    bool appF = false, appA = false;
    if (k < e) {
      j = S.ladj[k] & 0x7FFF;
      if (!iso_phase) S.nna[j] = (short)(S.nna[j] - 1);
      const unsigned wj = S.st[j];
      aj = st_agg(wj);
      if (aj == id) {
        const int sj = st_slot(wj);
        bits |= 1u << sj;
        S.madj[sj] |= 1u << s;
      } else if (aj < 0) {
        const bool elig = iso_phase ? (wj & ST_ISO) != 0 : (wj & ST_ISO) == 0;
        if (elig) {
          // on the front: one more member slot adjacent, one more strong link
          // (strong flags are symmetric, so c's flag for j is j's for c)
          S.st[j] = (wj | ST_FRONT) + ((S.ladj[k] >> 15) << ST_C2_SHIFT);
          S.cmm[j] |= 1u << s;
          appF = !(wj & ST_FRONT);
        }
      } else {
        const bool track = iso_phase ? (aj < P1) : true;
        const unsigned bit = 1u << (aj & 31);
        if (track && (atomicOr(&S.adjbits[aj >> 5], bit) & bit) == 0) appA = true;
      }
    }
    const uint64_t mF = __ballot(appF);
    if (appF) S.front[as.fcount + __popcll(mF & lanemask_lt())] = (short)j;
    as.fcount += __popcll(mF);
    const uint64_t mA = __ballot(appA);
    if (appA) S.adjl[as.acount + __popcll(mA & lanemask_lt())] = (short)aj;
    as.acount += __popcll(mA);
  }
  bits = wave_or(bits);
  if (lane == 0) S.madj[s] = bits;
  as.asize = s + 1;
  __syncthreads();
}

__device__ void clear_aggregate(const AggSh& S, AggState& as) {
  const int lane = __lane_id();
  for (int p = lane; p < as.fcount; p += WAVE) {
    const int c = S.front[p];
    S.st[c] &= ~(ST_FRONT | ST_C2_MASK);
    S.cmm[c] = 0;
  }
  for (int p = lane; p < as.acount; p += WAVE) {
    const int a = S.adjl[p];
    atomicAnd(&S.adjbits[a >> 5], ~(1u << (a & 31)));
  }
  __syncthreads();
  if (lane < as.asize) {
    const int v = S.mem[lane];
    S.st[v] = (S.st[v] & ~ST_SLOT_MASK) | ST_SLOT_NONE;
    S.madj[lane] = 0;
  }
  as.asize = as.fcount = as.acount = 0;
  __syncthreads();
}

// Eccentricity test of a candidate within a+{c}: every member reachable in at
// most dmax hops (paths through members only; c is the source).  Because every
// earlier addition passed the same test, this equals diam(a+{c}) <= dmax.
__device__ inline bool ecc_ok(const AggSh& S, unsigned mm, int asize, int dmax) {
  const unsigned full = asize >= 32 ? 0xFFFFFFFFu : ((1u << asize) - 1u);
  unsigned reach = mm, fr = mm;
  for (int d = 1; d < dmax && reach != full; ++d) {
    unsigned nx = 0, f = fr;
    while (f) {
      const int u = __builtin_ctz(f);
      f &= f - 1;
      nx |= S.madj[u];
    }
    fr = nx & ~reach;
    reach |= nx;
  }
  return reach == full;
}

// Scores of a candidate c from state kept up to date by add_member.  The
// strong flags are symmetric: s_ij and s_ji are the same products (w_ij w_ji
// and a_ii a_jj commute) compared with the same delta*min(eta_i, eta_j), so
// every strong link is two-way: cons2 (strong links into a) is the count in
// c's status word and cons1 is zero.  The sparsity pattern is symmetric
// (checked at setup), so the member mask of c is cmm[c], and in phase 1
// |N(c) n U| is the unaggregated neighbour count nna[c] less the isolated
// neighbours niso[c] (isolated vertices are all unaggregated then).
// Tie-break scores: connect(c,a) (strong neighbours outside a, weight 2 when
// in an aggregate adjacent to a) and neighbors(c,a) = |(N(c) n U) \ N(a)|.
// Entries are read in chunks of 8 so that their loads are in flight together.
__device__ inline void score_b(const AggSh& S, int c, int id, int& conn, int& nb) {
  conn = 0;
  nb = 0;
  const int b = S.lptr[c], e = S.lptr[c + 1];
  for (int k0 = b; k0 < e; k0 += 8) {
    unsigned w[8], wj[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) w[q] = k0 + q < e ? S.ladj[k0 + q] : 0u;
#pragma unroll
    for (int q = 0; q < 8; ++q) wj[q] = k0 + q < e ? S.st[w[q] & 0x7FFF] : 0u;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (k0 + q >= e) break;
      const int aj = st_agg(wj[q]);
      if (aj == id) continue;
      if (w[q] >> 15) conn += (aj >= 0 && ((S.adjbits[aj >> 5] >> (aj & 31)) & 1u)) ? 2 : 1;
      if (aj < 0 && !(wj[q] & (ST_ISO | ST_FRONT))) ++nb;
    }
  }
}

// Grow key of an admissible candidate: the lexicographic order (cons2,
// connect/|N|, neighbors, -index) as one unsigned integer.  |N| <= T-1 < 2^10
// and connect <= 2|N|, so floor(connect * 2^20 / |N|) orders the ratios
// exactly (two distinct ratios differ by at least 2^-20) and fits 22 bits.
__device__ inline unsigned long long grow_key(int c2, int conn, int deg, int nb, int c) {
  const unsigned r = ((unsigned)conn << 20) / (unsigned)deg;
  return ((unsigned long long)c2 << 58) | ((unsigned long long)r << 22) | ((unsigned long long)nb << 11) |
         (unsigned long long)(2047 - c);
}

// Strict total order of grow candidates with equal cons2: larger
// connect/|N| (exact cross multiplication), then larger neighbors, then
// smaller index.  c < 0 marks "no candidate".
__device__ inline bool better(int ca, int conna, int dega, int nba, int cb, int connb, int degb, int nbb) {
  if (ca < 0) return false;
  if (cb < 0) return true;
  const long long l = (long long)conna * degb, r = (long long)connb * dega;
  if (l != r) return l > r;
  if (nba != nbb) return nba > nbb;
  return ca < cb;
}

__global__ __launch_bounds__(WAVE) void k_aggregate(int n, int T, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const uint8_t* __restrict__ strong,
                                                    const uint8_t* __restrict__ isov, int smin, int smax, int dmax,
                                                    int Ecap, int* __restrict__ agg_local, int* __restrict__ tile_cnt,
                                                    int* __restrict__ members, int* __restrict__ mstart) {
  extern __shared__ __align__(16) unsigned char sm[];
  const AggLayout Lo = agg_layout(T, Ecap);
  AggSh S;
  S.lptr = (int*)(sm + Lo.lptr);
  S.st = (unsigned*)(sm + Lo.st);
  S.cmm = (unsigned*)(sm + Lo.cmm);
  S.niso = (short*)(sm + Lo.niso);
  S.adjbits = (unsigned*)(sm + Lo.adjb);
  S.madj = (unsigned*)(sm + Lo.madj);
  S.nna = (short*)(sm + Lo.nna);
  S.front = (short*)(sm + Lo.front);
  S.adjl = (short*)(sm + Lo.adjl);
  S.mem = (short*)(sm + Lo.mem);
  S.ladj = (unsigned short*)(sm + Lo.ladj);

  const int lane = __lane_id();
  const int t = blockIdx.x;
  const int lo = t * T;
  const int nt = min(T, n - lo);

  // ---- tile graph: local CSR of the in-tile off-diagonal entries
  int carry = 0;
  for (int base = 0; base < nt; base += WAVE) {
    const int v = base + lane;
    int cnt = 0;
    if (v < nt) {
      const int i = lo + v;
      for_entries(rp, ci, i, [&](int, int j) { cnt += (j != i && j >= lo && j < lo + nt) ? 1 : 0; });
    }
    const int inc = wave_incl_scan(cnt);
    if (v < nt) S.lptr[v] = carry + inc - cnt;
    carry += __shfl(inc, WAVE - 1, WAVE);
  }
  if (lane == 0) S.lptr[nt] = carry;
  __syncthreads();
  int nonIso = 0;
  for (int v = lane; v < nt; v += WAVE) {
    const int i = lo + v;
    int pos = S.lptr[v];
    for_entries(rp, ci, i, [&](int k, int j) {
      if (j != i && j >= lo && j < lo + nt) S.ladj[pos++] = (unsigned short)((j - lo) | (strong[k] ? 0x8000 : 0));
    });
    const bool is = isov[i] != 0;
    S.st[v] = ST_AGG | ST_SLOT_NONE | (is ? ST_ISO : 0u);
    S.cmm[v] = 0;
    S.nna[v] = (short)(pos - S.lptr[v]);
    nonIso += is ? 0 : 1;
  }
  for (int w = lane; w < (T + 31) / 32; w += WAVE) S.adjbits[w] = 0;
  if (lane < AGG_MAX_SLOTS) S.madj[lane] = 0;
  int nU = wave_sum(nonIso);
  __syncthreads();
  for (int v = lane; v < nt; v += WAVE) {
    int c = 0;
    for (int k = S.lptr[v]; k < S.lptr[v + 1]; ++k) c += (S.st[S.ladj[k] & 0x7FFF] & ST_ISO) ? 1 : 0;
    S.niso[v] = (short)c;
  }
  __syncthreads();

  AggState as{0, 0, 0};
  int id = 0;

  // ---- phase 1: non-isolated vertices (Alg. 1)
  int seed = INT_MAX;
  if (nU > 0) {
    int key = INT_MAX;
    for (int v = lane; v < nt; v += WAVE)
      if (!(S.st[v] & ST_ISO)) key = min(key, ((int)S.nna[v] << 16) | v);
    seed = wave_min(key) & 0xFFFF;
  }
  while (nU > 0) {
    add_member(S, as, seed, id, false, 0);
    --nU;
    // Grow (Alg. 2): among the unaggregated front candidates with cons2 > 0
    // whose addition keeps the diameter within dmax, the one with the largest
    // cons2, ties broken by connect/|N|, then neighbors, then the smaller
    // index: the maximum grow key.
    while (as.asize < smin) {
      unsigned long long key = 0;
      for (int base = 0; base < as.fcount; base += WAVE) {
        const int p = base + lane;
        if (p < as.fcount) {
          const int c = S.front[p];
          const unsigned wc = S.st[c];
          const int c2 = (int)((wc & ST_C2_MASK) >> ST_C2_SHIFT);
          if (st_agg(wc) < 0 && c2 > 0 && ecc_ok(S, S.cmm[c], as.asize, dmax)) {
            int conn, nb;
            score_b(S, c, id, conn, nb);
            const unsigned long long k = grow_key(c2, conn, S.lptr[c + 1] - S.lptr[c], nb, c);
            key = k > key ? k : key;
          }
        }
      }
      key = wave_max_u64(key);
      if (key == 0) break;
      add_member(S, as, 2047 - (int)(key & 2047), id, false, 0);
      --nU;
    }
    // Round (Alg. 3): the smallest candidate with cons2 > 0 adjacent to more
    // members than unaggregated non-isolated vertices.
    while (as.asize < smax) {
      int best = INT_MAX;
      for (int base = 0; base < as.fcount; base += WAVE) {
        const int p = base + lane;
        if (p < as.fcount) {
          const int c = S.front[p];
          const unsigned wc = S.st[c];
          if (st_agg(wc) < 0 && (wc & ST_C2_MASK) != 0 && __popc(S.cmm[c]) > S.nna[c] - S.niso[c])
            best = min(best, c);
        }
      }
      best = wave_min(best);
      if (best == INT_MAX) break;
      add_member(S, as, best, id, false, 0);
      --nU;
    }
    // One-vertex aggregate: join the aggregate holding most strong neighbours.
    bool merged = false;
    if (as.asize == 1) {
      const int v = S.mem[0];
      const int b = S.lptr[v], e = S.lptr[v + 1];
      int bk = INT_MAX, bcnt = 0;
      for (int base = b; base < e; base += WAVE) {
        const int k = base + lane;
        if (k < e) {
          const unsigned w = S.ladj[k];
          const int aj = st_agg(S.st[w & 0x7FFF]);
          if ((w >> 15) && aj >= 0 && aj != id) {
            int cnt = 0;
            for (int q = b; q < e; ++q) {
              const unsigned wq = S.ladj[q];
              cnt += ((wq >> 15) && st_agg(S.st[wq & 0x7FFF]) == aj) ? 1 : 0;
            }
            if (cnt > bcnt || (cnt == bcnt && aj < bk)) {
              bcnt = cnt;
              bk = aj;
            }
          }
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const int ok = __shfl_xor(bk, o, WAVE), oc = __shfl_xor(bcnt, o, WAVE);
        if (oc > bcnt || (oc == bcnt && ok < bk)) {
          bcnt = oc;
          bk = ok;
        }
      }
      if (bcnt > 0) {
        if (lane == 0) S.st[v] = (S.st[v] & ~ST_AGG) | ((unsigned)bk & ST_AGG);
        merged = true;
      }
      __syncthreads();
    }
    if (!merged) ++id;
    // Next seed: fewest unaggregated neighbours on the front, else over U.
    if (nU > 0) {
      int key = INT_MAX;
      for (int p = lane; p < as.fcount; p += WAVE) {
        const int c = S.front[p];
        if (st_agg(S.st[c]) < 0) key = min(key, ((int)S.nna[c] << 16) | c);
      }
      key = wave_min(key);
      if (key == INT_MAX) {
        for (int v = lane; v < nt; v += WAVE) {
          const unsigned wv = S.st[v];
          if (st_agg(wv) < 0 && !(wv & ST_ISO)) key = min(key, ((int)S.nna[v] << 16) | v);
        }
        key = wave_min(key);
      }
      seed = key & 0xFFFF;
    }
    clear_aggregate(S, as);
  }

  // ---- phase 2: isolated vertices (GrowIsoAggregate reading)
  const int P1 = id;
  for (int base = 0; base < nt; base += WAVE) {
    for (;;) {
      const int v = base + lane;
      bool cand = false;
      if (v < nt) {
        const unsigned wv = S.st[v];
        cand = (wv & ST_ISO) && st_agg(wv) < 0;
      }
      const uint64_t m = __ballot(cand);
      if (!m) break;
      const int s0 = base + (int)__builtin_ctzll(m);
      const int myid = id++;
      add_member(S, as, s0, myid, true, P1);
      while (as.asize < smin) {
        int best = INT_MAX;
        for (int b2 = 0; b2 < as.fcount; b2 += WAVE) {
          const int p = b2 + lane;
          if (p < as.fcount) {
            const int c = S.front[p];
            if (st_agg(S.st[c]) < 0) {
              bool common = false;
              unsigned mm = 0;
              for (int k = S.lptr[c]; k < S.lptr[c + 1]; ++k) {
                const unsigned wj = S.st[S.ladj[k] & 0x7FFF];
                const int aj = st_agg(wj);
                if (aj == myid)
                  mm |= 1u << st_slot(wj);
                else if (aj >= 0 && aj < P1 && ((S.adjbits[aj >> 5] >> (aj & 31)) & 1u))
                  common = true;
              }
              if (common && ecc_ok(S, mm, as.asize, dmax)) best = min(best, c);
            }
          }
        }
        best = wave_min(best);
        if (best == INT_MAX) break;
        add_member(S, as, best, myid, true, P1);
      }
      clear_aggregate(S, as);
    }
  }

  // ---- outputs: local ids, count, member lists grouped by aggregate (rows
  // ascending inside each).  The adjacency is no longer needed: lptr holds the
  // per-aggregate counters, front the rank of each row inside its aggregate.
  __syncthreads();
  for (int v = lane; v < nt; v += WAVE) agg_local[lo + v] = st_agg(S.st[v]);
  const int na = id;
  if (lane == 0) tile_cnt[t] = na;
  int* cnt = S.lptr;
  for (int k = lane; k < na; k += WAVE) cnt[k] = 0;
  __syncthreads();
  for (int base = 0; base < nt; base += WAVE) {
    const int v = base + lane;
    const int k = v < nt ? st_agg(S.st[v]) : -1;
    uint64_t left = __ballot(v < nt);
    while (left) {
      const int leader = (int)__builtin_ctzll(left);
      const int kl = __shfl(k, leader, WAVE);
      const uint64_t m = __ballot(k == kl) & left;
      const int c0 = cnt[kl];
      if (k == kl && ((m >> lane) & 1ull)) S.front[v] = (short)(c0 + __popcll(m & lanemask_lt()));
      __syncthreads();
      if (lane == leader) cnt[kl] = c0 + __popcll(m);
      __syncthreads();
      left &= ~m;
    }
  }
  carry = 0;
  for (int base = 0; base < na; base += WAVE) {
    const int k = base + lane;
    const int c = k < na ? cnt[k] : 0;
    const int inc = wave_incl_scan(c);
    if (k < na) {
      cnt[k] = carry + inc - c;
      mstart[lo + k] = carry + inc - c;
    }
    carry += __shfl(inc, WAVE - 1, WAVE);
  }
  __syncthreads();
  for (int v = lane; v < nt; v += WAVE) members[lo + cnt[st_agg(S.st[v])] + S.front[v]] = lo + v;
}

__global__ void k_tile_nnz_max(int n, int T, int ntiles, const int* __restrict__ rp, int* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  const int lo = t * T, hi = min(lo + T, n);
  atomicMax(out, rp[hi] - rp[lo]);
}

__global__ void k_agg_finalize(int n, int T, const int* __restrict__ agg_local, const int* __restrict__ tile_off,
                               const int* __restrict__ tile_cnt, const int* __restrict__ mstart,
                               int* __restrict__ agg, int* __restrict__ mptr, int nc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = i / T;
  const int off = tile_off[t];
  agg[i] = off + agg_local[i];
  const int k = i - t * T;
  if (k < tile_cnt[t]) mptr[off + k] = t * T + mstart[i];
  if (i == 0) mptr[nc] = n;
}

// ============================================================== Galerkin
// A_c(I,J) = sum over members i of a_I (ascending) and stored (i,j) in CSR
// order with agg[j] = J of a_ij, summed sequentially from the first term.
// One wavefront per coarse row: the row's terms are gathered in that order,
// ranked by (J, position) (a stable counting sort), and equal-J runs summed.
constexpr int GAL_CAP = 256;
constexpr int GAL_WAVES = 4;

__global__ void k_term_count(int nc, const int* __restrict__ mptr, const int* __restrict__ members,
                             const int* __restrict__ rp, int* __restrict__ tcount, int* maxm) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int s = 0;
  const int p1 = mptr[I + 1];
  for (int p0 = mptr[I]; p0 < p1; p0 += 8) {  // 8 members per step, their loads in flight together
    int mi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) mi[u] = p0 + u < p1 ? members[p0 + u] : -1;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (mi[u] >= 0) s += rp[mi[u] + 1] - rp[mi[u]];
  }
  tcount[I] = s;
  atomicMax(maxm, s);
}

// A group of W lanes (W = 64: the wavefront; W = 32: half of it) per coarse
// row; gl = lane inside the group.  The ballots are taken over the wavefront
// and cut to the group's bits.
template <int W>
__device__ __forceinline__ int group_incl_scan(int v, int gl) {
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    const int t = __shfl_up(v, d, W);
    if (gl >= d) v += t;
  }
  return v;
}
template <int W>
__device__ __forceinline__ uint64_t group_ballot(bool p) {
  const uint64_t b = __ballot(p);
  if (W == 64) return b;
  return (b >> (__lane_id() & ~(W - 1))) & ((1ull << W) - 1);
}

template <typename IdxT, int W>
__device__ void galerkin_row(int I, int m, int tb, const int* __restrict__ mptr, const int* __restrict__ members,
                             const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ va,
                             const int* __restrict__ agg, int* J, double* V, IdxT* Sx, int* __restrict__ tcol,
                             double* __restrict__ tval, int* __restrict__ ucount) {
  const int gl = __lane_id() & (W - 1);
  const uint64_t lt = (1ull << gl) - 1ull;
  // Terms in member order, CSR order inside a member: lane q takes member q,
  // finds its first term by a scan of the row lengths and copies its entries
  // with their loads in flight together.
  const int p0 = mptr[I], nm = mptr[I + 1] - p0;
  int pos = 0;
  for (int base = 0; base < nm; base += W) {
    const int q = base + gl;
    int b = 0, len = 0;
    if (q < nm) {
      const int i = members[p0 + q];
      b = rp[i];
      len = rp[i + 1] - b;
    }
    const int inc = group_incl_scan<W>(len, gl);
    const int off = pos + inc - len;
    for (int k0 = 0; k0 < len; k0 += 8) {
      int cc[8];
      double vv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        cc[u] = k0 + u < len ? ci[b + k0 + u] : 0;
        vv[u] = k0 + u < len ? va[b + k0 + u] : 0.0;
      }
      int aa[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) aa[u] = k0 + u < len ? agg[cc[u]] : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + u < len) {
          J[off + k0 + u] = aa[u];
          V[off + k0 + u] = vv[u];
        }
    }
    pos += __shfl(inc, W - 1, W);
  }
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  // Rank of term t among the terms ordered by (J, position): a stable
  // counting sort, reading 8 terms per step with their loads in flight together.
  for (int t = gl; t < m; t += W) {
    const int Jt = J[t];
    int r = 0, u = 0;
    for (; u + 8 <= m; u += 8) {
      int Ju[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) Ju[k] = J[u + k];
#pragma unroll
      for (int k = 0; k < 8; ++k) r += (Ju[k] < Jt || (Ju[k] == Jt && u + k < t)) ? 1 : 0;
    }
    for (; u < m; ++u) {
      const int Ju = J[u];
      r += (Ju < Jt || (Ju == Jt && u < t)) ? 1 : 0;
    }
    Sx[r] = (IdxT)t;
  }
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  // Equal-J runs in rank order, each summed sequentially from its first term
  // by the run's head; the run's end inside this chunk of W ranks comes from
  // the ballot of heads, so its loads are independent of the additions.
  int cnt = 0;
  for (int base = 0; base < m; base += W) {
    const int r = base + gl;
    bool head = false;
    int Jr = 0;
    if (r < m) {
      Jr = J[Sx[r]];
      head = (r == 0) || (J[Sx[r - 1]] != Jr);
    }
    const uint64_t hm = group_ballot<W>(head);
    if (head) {
      const int o = cnt + __popcll(hm & lt);
      const uint64_t after = gl == W - 1 ? 0ull : (hm >> (gl + 1));
      const int end = after ? r + 1 + (int)__builtin_ctzll(after) : min(m, base + W);
      double acc = V[Sx[r]];
#pragma unroll 4
      for (int q = r + 1; q < end; ++q) acc = acc + V[Sx[q]];
      if (!after)  // the run may go on in the next chunk
        for (int q = end; q < m && J[Sx[q]] == Jr; ++q) acc = acc + V[Sx[q]];
      tcol[tb + o] = Jr;
      tval[tb + o] = acc;
    }
    cnt += __popcll(hm);
  }
  if (gl == 0) ucount[I] = cnt;
}

__global__ __launch_bounds__(GAL_WAVES* WAVE, 8) void k_galerkin_rows(
    int nc, const int* __restrict__ mptr, const int* __restrict__ members, const int* __restrict__ rp,
    const int* __restrict__ ci, const double* __restrict__ va, const int* __restrict__ agg,
    const int* __restrict__ toff, int* gJ, double* gV, int* gS, int* __restrict__ tcol, double* __restrict__ tval,
    int* __restrict__ ucount) {
  __shared__ int sJ[GAL_WAVES][GAL_CAP];
  __shared__ double sV[GAL_WAVES][GAL_CAP];
  __shared__ short sS[GAL_WAVES][GAL_CAP];
  const int w = threadIdx.x / WAVE;
  const int I = blockIdx.x * GAL_WAVES + w;
  if (I >= nc) return;
  const int tb = toff[I];
  const int m = toff[I + 1] - tb;
  if (m <= GAL_CAP)
    galerkin_row<short, WAVE>(I, m, tb, mptr, members, rp, ci, va, agg, sJ[w], sV[w], sS[w], tcol, tval, ucount);
  else
    galerkin_row<int, WAVE>(I, m, tb, mptr, members, rp, ci, va, agg, gJ + tb, gV + tb, gS + tb, tcol, tval, ucount);
}

// The same with half a wavefront per coarse row, for levels whose rows all
// have at most GAL_CAP / 2 terms: twice the rows in flight in the same LDS.
__global__ __launch_bounds__(GAL_WAVES* WAVE) void k_galerkin_rows_half(
    int nc, const int* __restrict__ mptr, const int* __restrict__ members, const int* __restrict__ rp,
    const int* __restrict__ ci, const double* __restrict__ va, const int* __restrict__ agg,
    const int* __restrict__ toff, int* __restrict__ tcol, double* __restrict__ tval, int* __restrict__ ucount) {
  constexpr int HW = WAVE / 2, CAP = GAL_CAP / 2;
  __shared__ int sJ[2 * GAL_WAVES][CAP];
  __shared__ double sV[2 * GAL_WAVES][CAP];
  __shared__ short sS[2 * GAL_WAVES][CAP];
  const int w = threadIdx.x / HW;
  const int I = blockIdx.x * 2 * GAL_WAVES + w;
  if (I >= nc) return;
  const int tb = toff[I];
  const int m = toff[I + 1] - tb;
  galerkin_row<short, HW>(I, m, tb, mptr, members, rp, ci, va, agg, sJ[w], sV[w], sS[w], tcol, tval, ucount);
}

// 16 lanes per coarse row, so the copies are contiguous across lanes.
__global__ __launch_bounds__(256) void k_compact(int nc, const int* __restrict__ toff, const int* __restrict__ crp,
                                                 const int* __restrict__ tcol, const double* __restrict__ tval,
                                                 int* __restrict__ ccol, double* __restrict__ cval) {
  const int I = blockIdx.x * 16 + (int)threadIdx.x / 16, q0 = (int)threadIdx.x % 16;
  if (I >= nc) return;
  const int src = toff[I], dst = crp[I], cnt = crp[I + 1] - dst;
  for (int q = q0; q < cnt; q += 16) {
    ccol[dst + q] = tcol[src + q];
    cval[dst + q] = tval[src + q];
  }
}

// ============================================================== colouring
// Greedy first-fit colouring in a fixed order: tiles by descending key
// (fmix32(t ^ seed), t) -- fmix32 being the MurmurHash3 32-bit finaliser --
// and rows ascending inside a tile; each row takes the smallest colour that
// none of its already coloured neighbours has.  In parallel, a tile is
// coloured once every neighbour of its rows that lies in a tile of higher key
// is coloured (such tiles precede it in the order; neighbours in tiles of
// lower key wait for it), and inside the tile a row is coloured once all its
// smaller in-tile neighbours are.  Either way a row sees exactly the neighbours
// that precede it in the sequential order, so the result is that order's.
__device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__device__ inline bool tile_before(int ta, int tb, uint32_t seed) {  // ta precedes tb
  const uint32_t ka = fmix32((uint32_t)ta ^ seed), kb = fmix32((uint32_t)tb ^ seed);
  return ka > kb || (ka == kb && ta > tb);
}

__global__ void k_fill(int n, int* p, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

constexpr int COL_MAX_T = 1024;
constexpr int TSET = 2048;  // LDS hash set of the neighbour tiles of one tile

// Distinct neighbour tiles of each tile (tiles holding an off-tile neighbour of
// one of its rows).  Count pass (adj == NULL): cnt[t] and pending[t] = number
// of neighbour tiles that precede t.  Fill pass: adj[tptr[t] ...].
__global__ __launch_bounds__(WAVE) void k_tile_nbrs(int n, int T, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, uint32_t seed,
                                                    const int* __restrict__ tptr, int* __restrict__ adj,
                                                    int* __restrict__ cnt, int* __restrict__ pending,
                                                    int* overflow) {
  __shared__ int hs[TSET];
  const int lane = __lane_id();
  const int t = blockIdx.x;
  const int lo = t * T, hi = min(lo + T, n), nt = hi - lo;
  for (int q = lane; q < TSET; q += WAVE) hs[q] = -1;
  __syncthreads();
  for (int v = lane; v < nt; v += WAVE) {
    const int i = lo + v;
    for_entries(rp, ci, i, [&](int, int j) {
      if (j >= lo && j < hi) return;
      const int u = j / T;
      int h = (int)(fmix32((uint32_t)u) & (TSET - 1));
      for (int probe = 0;; ++probe) {
        if (probe == TSET) {
          atomicOr(overflow, 1);
          break;
        }
        const int old = atomicCAS(&hs[h], -1, u);
        if (old == -1 || old == u) break;
        h = (h + 1) & (TSET - 1);
      }
    });
  }
  __syncthreads();
  if (!adj) {
    int c = 0, pr = 0;
    for (int q = lane; q < TSET; q += WAVE)
      if (hs[q] >= 0) {
        ++c;
        pr += tile_before(hs[q], t, seed) ? 1 : 0;
      }
    c = wave_sum(c);
    pr = wave_sum(pr);
    if (lane == 0) {
      cnt[t] = c;
      pending[t] = pr;
    }
    return;
  }
  int pos = tptr[t];
  for (int base = 0; base < TSET; base += WAVE) {
    const int u = hs[base + lane];
    const uint64_t m = __ballot(u >= 0);
    if (u >= 0) adj[pos + __popcll(m & lanemask_lt())] = u;
    pos += __popcll(m);
  }
}

__global__ void k_ready0(int ntiles, const int* __restrict__ pending, int* __restrict__ list, int* cnt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ready = t < ntiles && pending[t] == 0;
  const uint64_t m = __ballot(ready);
  if (!m) return;
  const int lane = __lane_id(), leader = (int)__builtin_ctzll(m);
  int base = 0;
  if (lane == leader) base = atomicAdd(cnt, __popcll(m));
  base = __shfl(base, leader, WAVE);
  if (ready) list[base + __popcll(m & lanemask_lt())] = t;
}

// Dynamic LDS of k_colour_tiles: lptr[T+1], col[T], mask[T] (64-bit), big[T],
// qcur[T], adj[E] (local indices of the smaller in-tile neighbours).
__host__ __device__ inline size_t col_smem(int T, int E) {
  return align16(4 * (size_t)(T + 1)) + align16(4 * (size_t)T) + align16(8 * (size_t)T) + align16((size_t)T) +
         align16(4 * (size_t)T) + align16(2 * (size_t)(E > 0 ? E : 1));
}

// Colours the tiles of `work` (all their preceding neighbour tiles are
// finished), then releases the neighbour tiles they precede.
__device__ void colour_tile(int t, int n, int T, const int* __restrict__ rp, const int* __restrict__ ci,
                            const int* __restrict__ tptr, const int* __restrict__ tadj, int* pending, uint32_t seed,
                            int* colour, int* maxcol) {
  extern __shared__ __align__(16) unsigned char sm[];
  int* lptr = (int*)sm;
  int* col = (int*)(sm + align16(4 * (size_t)(T + 1)));
  uint64_t* mask = (uint64_t*)((unsigned char*)col + align16(4 * (size_t)T));
  unsigned char* big = (unsigned char*)mask + align16(8 * (size_t)T);
  int* qcur = (int*)(big + align16((size_t)T));  // first smaller neighbour not yet seen coloured
  unsigned short* adj = (unsigned short*)((unsigned char*)qcur + align16(4 * (size_t)T));
  const int lane = __lane_id();
  const int lo = t * T, hi = min(lo + T, n), nt = hi - lo;
  // Colours already taken by off-tile neighbours (all in preceding tiles) and
  // the smaller in-tile neighbours of each row.
  int carry = 0;
  for (int base = 0; base < nt; base += WAVE) {
    const int v = base + lane;
    int cnt = 0;
    if (v < nt) {
      const int i = lo + v;
      uint64_t m = 0;
      unsigned char bg = 0;
      for_entries(rp, ci, i, [&](int, int j) {
        if (j >= lo && j < hi) {
          cnt += (j < i) ? 1 : 0;
          return;
        }
        const int cj = colour[j];
        if (cj >= 64)
          bg = 1;
        else if (cj >= 0)
          m |= 1ull << cj;
      });
      mask[v] = m;
      big[v] = bg;
    }
    const int inc = wave_incl_scan(cnt);
    if (v < nt) lptr[v] = carry + inc - cnt;
    carry += __shfl(inc, WAVE - 1, WAVE);
  }
  if (lane == 0) lptr[nt] = carry;
  __syncthreads();
  for (int v = lane; v < nt; v += WAVE) {
    const int i = lo + v;
    int pos = lptr[v];
    qcur[v] = pos;
    for_entries(rp, ci, i, [&](int, int j) {
      if (j >= lo && j < i) adj[pos++] = (unsigned short)(j - lo);
    });
    col[v] = -1;
  }
  __syncthreads();
  // First-fit colour of a row depends only on the colours of its smaller
  // neighbours, so rows whose smaller in-tile neighbours are all coloured can
  // be coloured at once: wavefront rounds (one lane per row) while the rate
  // would finish the tile in a few dozen rounds, then rows in ascending order
  // for the rest of a long chain.  Both give the sequential first-fit colouring.
  // Colours never change once set, so a waiting row keeps where its scan
  // stopped (qcur) and the colours seen so far (OR-ed into mask, big).
  int cmax = -1;
  int first = 0;  // every row below `first` is coloured
  int total = 0;  // rows coloured by the rounds
  for (int round = 0; round < 64; ++round) {
    int made = 0;
    for (int v = first + lane; v < nt; v += WAVE) {
      if (col[v] >= 0) continue;
      uint64_t m = mask[v];
      bool ready = true, bg = big[v] != 0;
      int q = qcur[v];
      for (const int qe = lptr[v + 1]; q < qe; ++q) {  // stops at the first uncoloured one
        const int cj = col[adj[q]];
        if (cj < 0) {
          ready = false;
          break;
        }
        if (cj < 64)
          m |= 1ull << cj;
        else
          bg = true;
      }
      if (!ready) {
        qcur[v] = q;
        mask[v] = m;
        big[v] = bg ? 1 : 0;
        continue;
      }
      if (bg || m == ~0ull) continue;  // colours beyond 63: left to the ordered pass
      const int c = (int)__builtin_ctzll(~m);
      col[v] = c;
      cmax = max(cmax, c);
      ++made;
    }
    __syncthreads();
    made = wave_sum(made);
    total += made;
    while (first < nt) {  // first uncoloured row, 64 rows per step
      const int v = first + lane;
      const uint64_t done = __ballot(v >= nt || col[v] >= 0);
      if (done != ~0ull) {
        first += (int)__builtin_ctzll(~done);
        break;
      }
      first += WAVE;
    }
    first = min(first, nt);
    if (first >= nt || made == 0) break;
    // A long dependency chain (few rows per round) is faster row by row.
    if (round >= 7 && (long long)(nt - total) * (round + 1) > 40LL * total) break;
  }
  __syncthreads();
  // Rows in ascending order; the lanes read one row's smaller in-tile
  // neighbours together and OR their colours into the forbidden mask.
  for (int v = first; v < nt; ++v) {
    if (col[v] >= 0) continue;
    uint64_t m = 0;
    bool bg = false;
    for (int q = lptr[v] + lane; q < lptr[v + 1]; q += WAVE) {
      const int cj = col[adj[q]];
      if (cj < 64)
        m |= 1ull << cj;
      else
        bg = true;
    }
    unsigned lo32 = (unsigned)m, hi32 = (unsigned)(m >> 32);
    lo32 = wave_or(lo32);
    hi32 = wave_or(hi32);
    m = ((uint64_t)hi32 << 32 | lo32) | mask[v];
    bg = (__ballot(bg) != 0) || big[v] != 0;
    int c;
    if (!bg && m != ~0ull) {
      c = (int)__builtin_ctzll(~m);
    } else {  // colours beyond 63 among the neighbours: search directly
      const int i = lo + v;
      c = 0;
      for (;;) {
        bool used = false;
        for (int k = rp[i] + lane; k < rp[i + 1]; k += WAVE) {
          const int j = ci[k];
          if (j == i || (j >= lo && j > i)) continue;
          if (((j >= lo && j < hi) ? col[j - lo] : colour[j]) == c) used = true;
        }
        if (!__ballot(used)) break;
        ++c;
      }
    }
    if (lane == 0) col[v] = c;
    cmax = max(cmax, c);
    __syncthreads();
  }
  for (int v = lane; v < nt; v += WAVE) colour[lo + v] = col[v];
  cmax = wave_max(cmax);
  if (lane == 0) atomicMax(maxcol, cmax);
  // Tiles after this one wait for one neighbour less; k_ready0 lists those
  // that reach zero for the next launch, which sees these colours.  This tile
  // is marked done (-1): no tile before it is left to decrement it.
  for (int q = tptr[t] + lane; q < tptr[t + 1]; q += WAVE) {
    const int u = tadj[q];
    if (tile_before(t, u, seed)) atomicSub(&pending[u], 1);
  }
  if (lane == 0) pending[t] = -1;
  __syncthreads();  // the next tile of this block reuses the shared arrays
}

// The tiles of work[0, *count) (all their preceding neighbour tiles are
// finished), block b taking entries b, b + gridDim.x, ...: the grid does not
// depend on the count, so rounds are enqueued without a host round trip.
__global__ __launch_bounds__(WAVE) void k_colour_tiles(int n, int T, const int* __restrict__ work,
                                                       const int* __restrict__ count, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const int* __restrict__ tptr,
                                                       const int* __restrict__ tadj, int* pending, uint32_t seed,
                                                       int* colour, int* maxcol) {
  const int c = *count;
  for (int w = blockIdx.x; w < c; w += gridDim.x)
    colour_tile(work[w], n, T, rp, ci, tptr, tadj, pending, seed, colour, maxcol);
}

// Number of tiles not yet coloured (pending != -1), added to *out.
__global__ void k_count_pending(int ntiles, const int* __restrict__ pending, int* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t m = __ballot(t < ntiles && pending[t] != -1);
  if (m && __lane_id() == (int)__builtin_ctzll(m)) atomicAdd(out, __popcll(m));
}

constexpr int CL_THREADS = 256;

__global__ __launch_bounds__(CL_THREADS) void k_colour_hist(int n, const int* __restrict__ colour, int C,
                                                            int nblk, int* __restrict__ bcnt) {
  extern __shared__ int h[];
  for (int c = threadIdx.x; c < C; c += CL_THREADS) h[c] = 0;
  __syncthreads();
  const int i = blockIdx.x * CL_THREADS + threadIdx.x;
  if (i < n) atomicAdd(&h[colour[i]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += CL_THREADS) bcnt[(size_t)c * nblk + blockIdx.x] = h[c];
}

__global__ __launch_bounds__(CL_THREADS) void k_colour_place(int n, const int* __restrict__ colour, int C, int nblk,
                                                             const int* __restrict__ gofs, int* __restrict__ crows) {
  extern __shared__ int wc[];  // [CL_THREADS/WAVE][C]
  const int nw = CL_THREADS / WAVE;
  for (int q = threadIdx.x; q < nw * C; q += CL_THREADS) wc[q] = 0;
  __syncthreads();
  const int lane = __lane_id(), w = threadIdx.x / WAVE;
  const int i = blockIdx.x * CL_THREADS + threadIdx.x;
  const bool valid = i < n;
  const int c = valid ? colour[i] : -1;
  uint64_t active = __ballot(valid);
  int rank = 0;
  while (active) {
    const int leader = (int)__builtin_ctzll(active);
    const int cl = __shfl(c, leader, WAVE);
    const uint64_t m = __ballot(valid && c == cl);
    if (valid && c == cl) rank = __popcll(m & lanemask_lt());
    if (lane == 0) wc[w * C + cl] = __popcll(m);
    active &= ~m;
  }
  __syncthreads();
  if (!valid) return;
  int off = 0;
  for (int q = 0; q < w; ++q) off += wc[q * C + c];
  crows[gofs[(size_t)c * nblk + blockIdx.x] + off + rank] = i;
}

__global__ void k_gather_cptr(int C, int nblk, const int* __restrict__ gofs, int n, int* __restrict__ cptr) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) cptr[c] = gofs[(size_t)c * nblk];
  if (c == C) cptr[C] = n;
}

// ============================================================== casts etc.
__global__ void k_cast(size_t n, const double* __restrict__ in, float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void k_l1(int n, const int* __restrict__ rp, const double* __restrict__ v, double* __restrict__ o64,
                     float* __restrict__ o32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) s = s + fabs(v[k]);
  if (o64) o64[i] = s;
  if (o32) o32[i] = (float)s;
}

// ============================================================== coarsest level
__global__ void k_densify(int nL, const int* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ v, double* __restrict__ D) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nL) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) D[(size_t)i * nL + ci[k]] = v[k];
}

// Blocked dense Cholesky A = L L^T and inverse A^-1 = L^-T L^-1 (FP64) with
// 64x64 blocks.  D is row-major n x n; blocks past the edge are handled with
// bounds checks (entries outside the matrix read as identity padding).
constexpr int CB = 64;

__device__ inline void load_block(const double* __restrict__ D, int n, int bi, int bj, double (*B)[CB + 1]) {
  for (int q = threadIdx.x; q < CB * CB; q += blockDim.x) {
    const int r = q / CB, c = q % CB, i = bi * CB + r, j = bj * CB + c;
    B[r][c] = (i < n && j < n) ? D[(size_t)i * n + j] : (i == j ? 1.0 : 0.0);
  }
}
__device__ inline void store_block(double* __restrict__ D, int n, int bi, int bj, double (*B)[CB + 1]) {
  for (int q = threadIdx.x; q < CB * CB; q += blockDim.x) {
    const int r = q / CB, c = q % CB, i = bi * CB + r, j = bj * CB + c;
    if (i < n && j < n) D[(size_t)i * n + j] = B[r][c];
  }
}

// The triangular kernels run one wavefront per block with a row (or column)
// of the block per lane in registers; the block products give each of 256
// threads a 4 x 4 set of entries (rows tr + 16a, columns tc + 16b).  Every
// entry is computed with the same operations in the same order as a plain
// per-entry loop over k.
__device__ inline void load_row(const double* __restrict__ D, int n, int bi, int bj, int r, double (&x)[CB]) {
  const int i = bi * CB + r;
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int j = bj * CB + c;
    x[c] = (i < n && j < n) ? D[(size_t)i * n + j] : (i == j ? 1.0 : 0.0);
  }
}
__device__ inline void store_row(double* __restrict__ D, int n, int bi, int bj, int r, const double (&x)[CB]) {
  const int i = bi * CB + r;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < CB; ++c)
    if (bj * CB + c < n) D[(size_t)i * n + bj * CB + c] = x[c];
}

// The triangular kernels below are fully unrolled so that the block's rows
// stay in registers, with their updates as fused multiply-adds; barriers
// between steps (one wavefront: cheap) keep the compiler from issuing the
// LDS reads of later steps early, which would not fit in registers.
//
// Cholesky steps k = J0 .. J0+31 on columns J0 .. J0+31 of a diagonal block
// (b[jj] = B_i,J0+jj on lane i): the pivot sqrt(B_kk) from lane k, column k
// divided by it and broadcast through LDS, then B_ij -= B_ik B_jk for
// k < j <= i.
template <int J0>
__device__ __forceinline__ void chol_steps(double (&b)[CB / 2], int i, double* col, int* fail) {
#pragma unroll
  for (int kk = 0; kk < CB / 2; ++kk) {
    const int k = J0 + kk;
    const double d = __shfl(b[kk], k, WAVE);
    const bool ok = d > 0.0;
    if (!ok && i == 0) *fail = 1;
    const double piv = ok ? sqrt(d) : 1.0;
    if (i == k) b[kk] = piv;
    else if (i > k) b[kk] = b[kk] / piv;
    col[i] = b[kk];
    __syncthreads();
#pragma unroll
    for (int jj = kk + 1; jj < CB / 2; ++jj)
      if (J0 + jj <= i) b[jj] = fma(-b[kk], col[J0 + jj], b[jj]);
    __syncthreads();
  }
}

// Factor the diagonal block p (lower triangle), one wavefront, lane i holding
// row i, 32 columns at a time: the first half takes its steps; then the
// second half takes the first half's terms (k ascending, as the steps would
// have applied them) and its own steps.
__global__ __launch_bounds__(WAVE) void k_chol_diag(int n, int p, double* D, int* fail) {
  __shared__ double col[CB];
  __shared__ double Lf[CB][CB / 2 + 1];  // columns 0..31 after their steps
  constexpr int H = CB / 2;
  const int i = threadIdx.x, gi = p * CB + i;
  auto elem = [&](int gj) { return (gi < n && gj < n) ? D[(size_t)gi * n + gj] : (gi == gj ? 1.0 : 0.0); };
  double b[H], b2[H];
#pragma unroll
  for (int jj = 0; jj < H; ++jj) b[jj] = elem(p * CB + jj);
  chol_steps<0>(b, i, col, fail);
#pragma unroll
  for (int jj = 0; jj < H; ++jj) Lf[i][jj] = b[jj];
#pragma unroll
  for (int jj = 0; jj < H; ++jj) b2[jj] = elem(p * CB + H + jj);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < H; ++k) {
#pragma unroll
    for (int jj = 0; jj < H; ++jj)
      if (H + jj <= i) b2[jj] = fma(-b[k], Lf[H + jj][k], b2[jj]);
    __syncthreads();  // (one wavefront: cheap) bounds the LDS reads issued ahead
  }
  chol_steps<H>(b2, i, col, fail);
  if (gi < n) {
#pragma unroll
    for (int jj = 0; jj < H; ++jj) {
      if (p * CB + jj < n) D[(size_t)gi * n + p * CB + jj] = b[jj];
      if (p * CB + H + jj < n) D[(size_t)gi * n + p * CB + H + jj] = b2[jj];
    }
  }
}

// Panel: L_ip = A_ip L_pp^{-T} for the block rows i > p (one wavefront each,
// lane r solving row r by forward substitution, k ascending).
__global__ __launch_bounds__(WAVE) void k_chol_trsm(int n, int p, double* D) {
  __shared__ double Lp[CB][CB + 1];
  const int bi = p + 1 + blockIdx.x, r = threadIdx.x, gr = bi * CB + r;
  load_block(D, n, p, p, Lp);
  double x[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int gc = p * CB + c;
    x[c] = (gr < n && gc < n) ? D[(size_t)gr * n + gc] : 0.0;  // off the diagonal: no identity padding
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    double v = x[c];
#pragma unroll
    for (int k = 0; k < c; ++k) v = fma(-x[k], Lp[c][k], v);
    x[c] = v / Lp[c][c];
    __syncthreads();  // (one wavefront: cheap) row c + 1's LDS reads are not issued ahead of row c
  }
  if (gr < n) {
#pragma unroll
    for (int c = 0; c < CB; ++c)
      if (p * CB + c < n) D[(size_t)gr * n + p * CB + c] = x[c];
  }
}

// 4 x 4 entries per thread of a 64 x 64 block product: rows tr + 16a, columns
// tc + 16b; a(k, a) and b(k, b) read the operands from LDS.
template <typename FA, typename FB>
__device__ __forceinline__ void block_dot(FA a, FB b, double (&s)[4][4]) {
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) s[x][y] = 0.0;
  for (int k = 0; k < CB; ++k) {
    double av[4], bv[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) av[x] = a(k, x);
#pragma unroll
    for (int y = 0; y < 4; ++y) bv[y] = b(k, y);
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) s[x][y] += av[x] * bv[y];
  }
}

// Trailing update A_ij -= L_ip L_jp^T for p < j <= i (one workgroup per pair).
__global__ __launch_bounds__(256) void k_chol_update(int n, int p, double* D) {
  __shared__ double Li[CB][CB + 1];
  __shared__ double Lj[CB][CB + 1];
  int q = blockIdx.x, bi = 0;  // pairs (i, j), i >= j, over the trailing blocks
  const int nt = (n + CB - 1) / CB - (p + 1);
  while (q >= bi + 1) {
    q -= bi + 1;
    ++bi;
  }
  const int I = p + 1 + bi, J = p + 1 + q;
  if (bi >= nt) return;
  load_block(D, n, I, p, Li);
  load_block(D, n, J, p, Lj);
  __syncthreads();
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double s[4][4];
  block_dot([&](int k, int x) { return Li[tr + 16 * x][k]; }, [&](int k, int y) { return Lj[tc + 16 * y][k]; }, s);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int r = tr + 16 * x, c = tc + 16 * y, i = I * CB + r, j = J * CB + c;
      if (i >= n || j >= n || (I == J && c > r)) continue;
      D[(size_t)i * n + j] -= s[x][y];
    }
}

// W = L^{-1}: diagonal blocks W_ii = L_ii^{-1} (one wavefront each; lane c
// computes column c by forward substitution).
__global__ __launch_bounds__(WAVE) void k_trinv_diag(int n, const double* __restrict__ D, double* __restrict__ W) {
  __shared__ double L[CB][CB + 1];
  const int b = blockIdx.x, c = threadIdx.x;
  load_block(D, n, b, b, L);
  __syncthreads();
  double x[CB];
#pragma unroll
  for (int r = 0; r < CB; ++r) {
    double v = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < r; ++k)
      if (k >= c) v = fma(-L[r][k], x[k], v);
    x[r] = r < c ? 0.0 : v / L[r][r];
  }
  const int j = b * CB + c;
#pragma unroll
  for (int r = 0; r < CB; ++r)
    if (b * CB + r < n && j < n) W[(size_t)(b * CB + r) * n + j] = x[r];
}

// Block row i of W: W_ij = -W_ii sum_{k=j}^{i-1} L_ik W_kj for j < i.
__global__ __launch_bounds__(256) void k_trinv_row(int n, int bi, const double* __restrict__ D,
                                                   double* __restrict__ W) {
  __shared__ double A[CB][CB + 1];
  __shared__ double Bm[CB][CB + 1];
  const int bj = blockIdx.x, tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double S[4][4], s[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) S[x][y] = 0.0;
  for (int bk = bj; bk < bi; ++bk) {
    __syncthreads();
    load_block(D, n, bi, bk, A);
    load_block(W, n, bk, bj, Bm);
    __syncthreads();
    block_dot([&](int k, int x) { return A[tr + 16 * x][k]; }, [&](int k, int y) { return Bm[k][tc + 16 * y]; }, s);
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) S[x][y] += s[x][y];
  }
  __syncthreads();
  load_block(W, n, bi, bi, A);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) Bm[tr + 16 * x][tc + 16 * y] = S[x][y];
  __syncthreads();
  block_dot([&](int k, int x) { return A[tr + 16 * x][k]; }, [&](int k, int y) { return Bm[k][tc + 16 * y]; }, s);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = bi * CB + tr + 16 * x, j = bj * CB + tc + 16 * y;
      if (i < n && j < n) W[(size_t)i * n + j] = -s[x][y];
    }
}

// A^-1 = W^T W: block (I, J), I >= J, sum over k >= I of W_kI^T W_kJ; written
// to both (I, J) and (J, I) so the result is exactly symmetric.
__global__ __launch_bounds__(256) void k_wtw_blocks(int n, const double* __restrict__ W, double* __restrict__ Ainv) {
  __shared__ double Wi[CB][CB + 1];
  __shared__ double Wj[CB][CB + 1];
  int q = blockIdx.x, bi = 0;
  while (q >= bi + 1) {
    q -= bi + 1;
    ++bi;
  }
  const int I = bi, J = q;
  const int nb = (n + CB - 1) / CB;
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double acc[4][4], s[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
  for (int bk = I; bk < nb; ++bk) {
    __syncthreads();
    load_block(W, n, bk, I, Wi);
    load_block(W, n, bk, J, Wj);
    __syncthreads();
    block_dot([&](int k, int x) { return Wi[k][tr + 16 * x]; }, [&](int k, int y) { return Wj[k][tc + 16 * y]; }, s);
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] += s[x][y];
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int r = tr + 16 * x, c = tc + 16 * y, i = I * CB + r, j = J * CB + c;
      if (i < n && j < n && (I != J || c <= r)) {
        Ainv[(size_t)i * n + j] = acc[x][y];
        Ainv[(size_t)j * n + i] = acc[x][y];
      }
    }
}

// ============================================================== solve order
__global__ void k_invperm(int n, const int* __restrict__ perm, int* __restrict__ pinv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) pinv[perm[r]] = r;
}

__global__ void k_perm_rowlen(int n, const int* __restrict__ perm, const int* __restrict__ rp, int* __restrict__ len) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) {
    const int i = perm[r];
    len[r] = rp[i + 1] - rp[i];
  }
}

// Copy each solve row's entries (same order) with the columns relabelled.
// `sub` consecutive threads (a power of two <= 64) copy one row, PERM_ROWS
// rows per group (`per` rows apart) with the first `sub` entries of all of
// them loaded together; grid-stride over rows, so the grid stays within the
// dispatch limits at any n.
constexpr int PERM_ROWS = 4;
__global__ __launch_bounds__(256) void k_perm_rows(int n, int sub, const int* __restrict__ perm,
                                                   const int* __restrict__ pinv, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const double* __restrict__ v,
                                                   const int* __restrict__ prp, int* __restrict__ pci,
                                                   double* __restrict__ pv) {
  const int per = 256 / sub;
  const int q0 = (int)threadIdx.x % sub;
  const long long step = (long long)gridDim.x * per * PERM_ROWS;
  for (long long r0 = (long long)blockIdx.x * per * PERM_ROWS + threadIdx.x / sub; r0 < n; r0 += step) {
    int i[PERM_ROWS], b[PERM_ROWS], len[PERM_ROWS], d[PERM_ROWS], c[PERM_ROWS], pc[PERM_ROWS];
    double x[PERM_ROWS];
#pragma unroll
    for (int u = 0; u < PERM_ROWS; ++u) {
      const long long r = r0 + (long long)u * per;
      i[u] = r < n ? perm[r] : -1;
    }
#pragma unroll
    for (int u = 0; u < PERM_ROWS; ++u) {
      const long long r = r0 + (long long)u * per;
      b[u] = i[u] >= 0 ? rp[i[u]] : 0;
      len[u] = i[u] >= 0 ? rp[i[u] + 1] - b[u] : 0;
      d[u] = i[u] >= 0 ? prp[r] : 0;
    }
#pragma unroll
    for (int u = 0; u < PERM_ROWS; ++u) {
      c[u] = q0 < len[u] ? ci[b[u] + q0] : 0;
      x[u] = q0 < len[u] ? v[b[u] + q0] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PERM_ROWS; ++u) pc[u] = q0 < len[u] ? pinv[c[u]] : 0;
#pragma unroll
    for (int u = 0; u < PERM_ROWS; ++u) {
      if (q0 < len[u]) {
        pci[d[u] + q0] = pc[u];
        pv[d[u] + q0] = x[u];
      }
      for (int q = q0 + sub; q < len[u]; q += sub) {
        pci[d[u] + q] = pinv[ci[b[u] + q]];
        pv[d[u] + q] = v[b[u] + q];
      }
    }
  }
}

__global__ void k_perm_agg(int n, const int* __restrict__ perm, const int* __restrict__ agg,
                           const int* __restrict__ next_pinv, int* __restrict__ pagg) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) {
    const int a = agg[perm[r]];
    pagg[r] = next_pinv ? next_pinv[a] : a;
  }
}

__global__ void k_perm_mcount(int nc, const int* __restrict__ next_perm, const int* __restrict__ mptr,
                              int* __restrict__ cnt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) {
    const int I = next_perm ? next_perm[c] : c;
    cnt[c] = mptr[I + 1] - mptr[I];
  }
}

__global__ void k_perm_members(int nc, const int* __restrict__ next_perm, const int* __restrict__ mptr,
                               const int* __restrict__ members, const int* __restrict__ pinv,
                               const int* __restrict__ pmptr, int* __restrict__ pmem) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) {
    const int I = next_perm ? next_perm[c] : c;
    const int b = mptr[I], len = mptr[I + 1] - b, d = pmptr[c];
    for (int q = 0; q < len; ++q) pmem[d + q] = pinv[members[b + q]];
  }
}

__global__ void k_gather(int n, const int* __restrict__ perm, const double* __restrict__ in, double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] = in[perm[r]];
}

__global__ void k_scatter(int n, const int* __restrict__ perm, const double* __restrict__ in,
                          double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[perm[r]] = in[r];
}

// ============================================================== SELL-64
__global__ void k_sell_width(int nsl, const int* __restrict__ srow, const int* __restrict__ rp,
                             int* __restrict__ w64) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nsl) return;
  int w = 0;
  for (int r = srow[sl]; r < srow[sl + 1]; ++r) w = max(w, rp[r + 1] - rp[r] - 1);
  w64[sl] = 64 * w;
}

// One wavefront per slice.  The slice's rows are consecutive in the
// (colour-ordered) CSR, so their entries are one contiguous range: it is
// staged through shared memory with contiguous loads when it has at most
// SF_CAP entries, and each lane then scans its row there.
constexpr int SF_CAP = 512;
__global__ __launch_bounds__(256) void k_sell_fill(int nsl, const int* __restrict__ srow, const int* __restrict__ soff,
                                                   const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const double* __restrict__ v, int* __restrict__ scol,
                                                   double* __restrict__ sval, double* __restrict__ dg) {
  __shared__ int sc[4][SF_CAP];
  __shared__ double sv[4][SF_CAP];
  const int wv = (int)threadIdx.x / WAVE;
  const int sl = blockIdx.x * 4 + wv;
  if (sl >= nsl) return;
  const int lane = __lane_id();
  const int r0 = srow[sl], r1 = srow[sl + 1], r = r0 + lane;
  const bool valid = r < r1;
  const int base = soff[sl], w = (soff[sl + 1] - base) / 64;
  const int e0 = rp[r0], ne = rp[r1] - e0;
  const bool staged = ne <= SF_CAP;
  if (staged) {
    for (int k = lane; k < ne; k += WAVE) {
      sc[wv][k] = ci[e0 + k];
      sv[wv][k] = v[e0 + k];
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
  int k = 0;
  if (valid) {
    for (int q = rp[r]; q < rp[r + 1]; ++q) {
      const int j = staged ? sc[wv][q - e0] : ci[q];
      const double a = staged ? sv[wv][q - e0] : v[q];
      if (j == r) {
        dg[r] = a;
      } else {
        scol[base + 64 * k + lane] = j;
        sval[base + 64 * k + lane] = a;
        ++k;
      }
    }
  }
  for (; k < w; ++k) {
    scol[base + 64 * k + lane] = valid ? r : r0;
    sval[base + 64 * k + lane] = 0.0;
  }
}


// ============================================================== point-based levels
// A level of bs-component nodes (point-based AMG for systems, Sec. 4.2) is a
// scalar CSR in which node i owns rows i*bs .. i*bs+bs-1 (natural order) and
// every stored block is full: its bs rows hold the columns J*bs .. J*bs+bs-1
// side by side.  Coarsening and colouring run on the node graph, weighted by
// row-sum norms of the blocks (Sec. 2.1); the decisions are expanded to the
// bs unknowns of each node.
constexpr int BLK_MAX = 4;  // largest supported block size

// Every node's rows share one pattern of whole blocks, the diagonal block
// included (flag 1 otherwise).  Runs after the structural checks.
__global__ void k_validate_blocks(int nn, int bs, const int* __restrict__ rp, const int* __restrict__ ci, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int r0 = i * bs, len = rp[r0 + 1] - rp[r0];
  bool ok = len % bs == 0, diag = false;
  for (int c = 0; c < bs && ok; ++c) {
    if (rp[r0 + c + 1] - rp[r0 + c] != len) {
      ok = false;
      break;
    }
    for (int q = 0; q < len / bs && ok; ++q) {
      const int J = ci[rp[r0] + q * bs] / bs;
      for (int d = 0; d < bs; ++d)
        if (ci[rp[r0 + c] + q * bs + d] != J * bs + d) ok = false;
      if (J == i) diag = true;
    }
  }
  if (!ok || !diag) atomicOr(flags, 1);
}

__global__ void k_node_count(int nn, int bs, const int* __restrict__ rp, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) cnt[i] = (rp[i * bs + 1] - rp[i * bs]) / bs;
}

// Node graph with the block weights where the scalar criterion reads them:
// off-diagonal -||A_iJ||_inf (so w_E = max(-a, 0) is the norm), diagonal
// ||A_ii||_inf; row sums added in column order, then the largest taken.
__global__ void k_node_fill(int nn, int bs, const int* __restrict__ rp, const int* __restrict__ ci,
                            const double* __restrict__ v, const int* __restrict__ nrp, int* __restrict__ nci,
                            double* __restrict__ nv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int r0 = i * bs, nb = nrp[i + 1] - nrp[i];
  for (int q = 0; q < nb; ++q) {
    const int J = ci[rp[r0] + q * bs] / bs;
    double nrm = 0.0;
    for (int c = 0; c < bs; ++c) {
      double rs = 0.0;
      for (int d = 0; d < bs; ++d) rs = rs + fabs(v[rp[r0 + c] + q * bs + d]);
      nrm = fmax(nrm, rs);
    }
    nci[nrp[i] + q] = J;
    nv[nrp[i] + q] = J == i ? nrm : -nrm;
  }
}

// Prolongation P (x) I: unknown c of node i goes to unknown c of the node's
// aggregate; member lists of coarse unknown (I, c): the members of I, ascending.
__global__ void k_expand_agg(int n, int bs, const int* __restrict__ nagg, int* __restrict__ agg) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) agg[r] = nagg[r / bs] * bs + r % bs;
}

__global__ void k_expand_members(int ncn, int bs, const int* __restrict__ nmptr, const int* __restrict__ nmem,
                                 int* __restrict__ mptr, int* __restrict__ mem) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= ncn) return;
  const int b = nmptr[I], cnt = nmptr[I + 1] - b;
  for (int c = 0; c < bs; ++c) {
    mptr[I * bs + c] = bs * b + c * cnt;
    for (int k = 0; k < cnt; ++k) mem[bs * b + c * cnt + k] = nmem[b + k] * bs + c;
  }
  if (I == ncn - 1) mptr[ncn * bs] = bs * nmptr[ncn];
}

__global__ void k_expand_colour(int n, int bs, const int* __restrict__ ncol, const int* __restrict__ ncrows,
                                int* __restrict__ col, int* __restrict__ crows) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  col[r] = ncol[r / bs];
  crows[r] = ncrows[r / bs] * bs + r % bs;
}

// Inverse of every node's diagonal block (solve order: node q owns rows
// q*bs .. q*bs+bs-1), Gauss-Jordan with partial pivoting (largest magnitude,
// first on ties); row c of the inverse goes to dinv[(q*bs + c)*bs ..].
// Flag 1: a zero pivot.
__global__ void k_block_dinv(int nn, int bs, const int* __restrict__ rp, const int* __restrict__ ci,
                             const double* __restrict__ v, double* __restrict__ dinv, int* __restrict__ flag) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nn) return;
  double m[BLK_MAX * BLK_MAX], e[BLK_MAX * BLK_MAX];
  for (int k = 0; k < bs * bs; ++k) {
    m[k] = 0.0;
    e[k] = 0.0;
  }
  for (int c = 0; c < bs; ++c) {
    e[c * bs + c] = 1.0;
    const int r = q * bs + c;
    for (int k = rp[r]; k < rp[r + 1]; ++k) {
      const int j = ci[k];
      if (j >= q * bs && j < q * bs + bs) m[c * bs + (j - q * bs)] = v[k];
    }
  }
  for (int c = 0; c < bs; ++c) {
    int piv = c;
    for (int r = c + 1; r < bs; ++r)
      if (fabs(m[r * bs + c]) > fabs(m[piv * bs + c])) piv = r;
    if (m[piv * bs + c] == 0.0) {
      atomicOr(flag, 1);
      return;
    }
    if (piv != c)
      for (int k = 0; k < bs; ++k) {
        double t = m[c * bs + k];
        m[c * bs + k] = m[piv * bs + k];
        m[piv * bs + k] = t;
        t = e[c * bs + k];
        e[c * bs + k] = e[piv * bs + k];
        e[piv * bs + k] = t;
      }
    const double p = m[c * bs + c];
    for (int k = 0; k < bs; ++k) {
      m[c * bs + k] = m[c * bs + k] / p;
      e[c * bs + k] = e[c * bs + k] / p;
    }
    for (int r = 0; r < bs; ++r) {
      if (r == c) continue;
      const double f = m[r * bs + c];
      for (int k = 0; k < bs; ++k) {
        m[r * bs + k] = m[r * bs + k] - f * m[c * bs + k];
        e[r * bs + k] = e[r * bs + k] - f * e[c * bs + k];
      }
    }
  }
  for (int k = 0; k < bs * bs; ++k) dinv[(size_t)q * bs * bs + k] = e[k];
}

template <typename T>
T read1(const T* dptr, hipStream_t s) {
  T v;
  AMG_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
  sync_stream(s);
  return v;
}

// Several device ints with one host round trip.
void read_ints(hipStream_t s, std::initializer_list<std::pair<int*, const int*>> dst_src) {
  for (const auto& d : dst_src) AMG_HIP(hipMemcpyAsync(d.first, d.second, sizeof(int), hipMemcpyDeviceToHost, s));
  sync_stream(s);
}

}  // namespace

// ================================================================== host side
void exclusive_scan(const int* in, int* out, int n, hipStream_t s) {
  const int nb = std::max(1, cdiv(n, SCAN_TILE));
  DBuf bs((size_t)(nb + 1) * sizeof(int), s);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, bs.as<int>());
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_THREADS), 0, s, bs.as<int>(), nb);
  hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, bs.as<int>(), nb, out);
  AMG_HIP(hipGetLastError());
}

int validate_csr(int n, int nnz, const int* rp, const int* ci, const double* v, int check_symmetry, hipStream_t s) {
  DBuf f(sizeof(int), s);
  AMG_HIP(hipMemsetAsync(f.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_validate_struct, dim3(cdiv(n, 256)), dim3(256), 0, s, n, nnz, rp, ci, v, f.as<int>());
  AMG_HIP(hipGetLastError());
  int flags = read1(f.as<int>(), s);
  if (flags) return flags;
  hipLaunchKernelGGL(k_validate_sym, dim3(cdiv(n, STR_BLOCK_ROWS)), dim3(256), 0, s, n, rp, ci, v, check_symmetry,
                     f.as<int>());
  AMG_HIP(hipGetLastError());
  return read1(f.as<int>(), s);
}

void strength(const Level& L, double delta, double beta, uint8_t* strong, uint8_t* iso, bool sym, hipStream_t s) {
  DBuf d((size_t)L.n * sizeof(double), s), eta((size_t)L.n * sizeof(double), s);
  const int g = cdiv(L.n, STR_BLOCK_ROWS);
  AMG_HIP(hipMemsetAsync(d.p, 0, (size_t)L.n * sizeof(double), s));  // rows without a stored diagonal
  hipLaunchKernelGGL(k_diag, dim3(g), dim3(256), 0, s, L.n, L.rowptr, L.colind, L.vals, d.as<double>());
  hipLaunchKernelGGL(k_eta, dim3(g), dim3(256), 0, s, L.n, L.T, L.rowptr, L.colind, L.vals, d.as<double>(),
                     eta.as<double>(), sym ? 1 : 0);
  hipLaunchKernelGGL(k_strong, dim3(g), dim3(256), 0, s, L.n, L.T, L.rowptr, L.colind, L.vals, d.as<double>(),
                     eta.as<double>(), delta, beta, strong, iso, sym ? 1 : 0);
  AMG_HIP(hipGetLastError());
}

int aggregate(Hierarchy& H, Level& L, const uint8_t* strong, const uint8_t* iso, const amg_params& p, hipStream_t s) {
  const int n = L.n, T = L.T;
  const int ntiles = cdiv(n, T);
  L.ntiles = ntiles;
  DBuf mx(sizeof(int), s);
  AMG_HIP(hipMemsetAsync(mx.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_tile_nnz_max, dim3(cdiv(ntiles, 256)), dim3(256), 0, s, n, T, ntiles, L.rowptr, mx.as<int>());
  AMG_HIP(hipGetLastError());
  const int Ecap = read1(mx.as<int>(), s);
  const AggLayout lay = agg_layout(T, Ecap);
  if (lay.total > 160 * 1024)
    fail(AMG_ERR_UNSUPPORTED, "aggregation tile graph exceeds LDS (" + std::to_string(lay.total) +
                                  " bytes); use smaller tile_rows");
  AMG_HIP(hipFuncSetAttribute((const void*)k_aggregate, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lay.total));
  DBuf agg_local((size_t)n * sizeof(int), s), tile_cnt((size_t)ntiles * sizeof(int), s),
      mstart((size_t)n * sizeof(int), s);
  int* members = H.alloc<int>((size_t)n, s);
  hipLaunchKernelGGL(k_aggregate, dim3(ntiles), dim3(WAVE), lay.total, s, n, T, L.rowptr, L.colind, strong, iso,
                     p.agg_min, p.agg_max, p.agg_diameter, Ecap, agg_local.as<int>(), tile_cnt.as<int>(), members,
                     mstart.as<int>());
  AMG_HIP(hipGetLastError());
  int* tile_off = H.alloc<int>((size_t)ntiles + 1, s);
  exclusive_scan(tile_cnt.as<int>(), tile_off, ntiles, s);
  const int nc = read1(tile_off + ntiles, s);
  int* agg = H.alloc<int>((size_t)n, s);
  int* mptr = H.alloc<int>((size_t)nc + 1, s);
  hipLaunchKernelGGL(k_agg_finalize, dim3(cdiv(n, 256)), dim3(256), 0, s, n, T, agg_local.as<int>(), tile_off,
                     tile_cnt.as<int>(), mstart.as<int>(), agg, mptr, nc);
  AMG_HIP(hipGetLastError());
  L.members = members;
  L.tile_off = tile_off;
  L.agg = agg;
  L.mptr = mptr;
  L.nc = nc;
  return nc;
}

void galerkin(Hierarchy& H, const Level& L, Level& C, hipStream_t s) {
  const int nc = L.nc;
  DBuf tcount((size_t)nc * sizeof(int), s), mx(sizeof(int), s);
  AMG_HIP(hipMemsetAsync(mx.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_term_count, dim3(cdiv(nc, 256)), dim3(256), 0, s, nc, L.mptr, L.members, L.rowptr,
                     tcount.as<int>(), mx.as<int>());
  DBuf toff((size_t)(nc + 1) * sizeof(int), s);
  exclusive_scan(tcount.as<int>(), toff.as<int>(), nc, s);
  int maxm = 0, total = 0;
  read_ints(s, {{&maxm, mx.as<int>()}, {&total, toff.as<int>() + nc}});
  if (total != L.nnz) fail(AMG_ERR_HIP, "Galerkin term count mismatch");
  DBuf tcol((size_t)total * sizeof(int), s), tval((size_t)total * sizeof(double), s),
      ucount((size_t)nc * sizeof(int), s);
  DBuf gJ, gV, gS;
  if (maxm > GAL_CAP) {
    gJ = DBuf((size_t)total * sizeof(int), s);
    gV = DBuf((size_t)total * sizeof(double), s);
    gS = DBuf((size_t)total * sizeof(int), s);
  }
  if (maxm <= GAL_CAP / 2)
    hipLaunchKernelGGL(k_galerkin_rows_half, dim3(cdiv(nc, 2 * GAL_WAVES)), dim3(GAL_WAVES * WAVE), 0, s, nc, L.mptr,
                       L.members, L.rowptr, L.colind, L.vals, L.agg, toff.as<int>(), tcol.as<int>(),
                       tval.as<double>(), ucount.as<int>());
  else
    hipLaunchKernelGGL(k_galerkin_rows, dim3(cdiv(nc, GAL_WAVES)), dim3(GAL_WAVES * WAVE), 0, s, nc, L.mptr,
                       L.members, L.rowptr, L.colind, L.vals, L.agg, toff.as<int>(), gJ.as<int>(), gV.as<double>(),
                       gS.as<int>(), tcol.as<int>(), tval.as<double>(), ucount.as<int>());
  AMG_HIP(hipGetLastError());
  C.n = nc;
  C.rowptr = H.alloc<int>((size_t)nc + 1, s);
  exclusive_scan(ucount.as<int>(), C.rowptr, nc, s);
  C.nnz = read1(C.rowptr + nc, s);
  C.colind = H.alloc<int>((size_t)C.nnz, s);
  C.vals = H.alloc<double>((size_t)C.nnz, s);
  hipLaunchKernelGGL(k_compact, dim3(cdiv(nc, 16)), dim3(256), 0, s, nc, toff.as<int>(), C.rowptr, tcol.as<int>(),
                     tval.as<double>(), C.colind, C.vals);
  AMG_HIP(hipGetLastError());
}

void colour(Hierarchy& H, Level& L, uint32_t seed, hipStream_t s) {
  const int n = L.n, T = H.p.colour_tile_rows;
  if (T > COL_MAX_T) fail(AMG_ERR_UNSUPPORTED, "colour_tile_rows above 1024");
  const int ntiles = cdiv(n, T);
  L.colour = H.alloc<int>((size_t)n, s);
  DBuf cnt(4 * sizeof(int), s), w0((size_t)ntiles * sizeof(int), s);
  DBuf tcnt((size_t)ntiles * sizeof(int), s), pend((size_t)ntiles * sizeof(int), s),
      tptr(((size_t)ntiles + 1) * sizeof(int), s);
  hipLaunchKernelGGL(k_fill, dim3(cdiv(n, 256)), dim3(256), 0, s, n, L.colour, -1);
  AMG_HIP(hipMemsetAsync(cnt.p, 0, 4 * sizeof(int), s));
  // tile graph
  hipLaunchKernelGGL(k_tile_nbrs, dim3(ntiles), dim3(WAVE), 0, s, n, T, L.rowptr, L.colind, seed, nullptr, nullptr,
                     tcnt.as<int>(), pend.as<int>(), cnt.as<int>());
  exclusive_scan(tcnt.as<int>(), tptr.as<int>(), ntiles, s);
  DBuf mx(sizeof(int), s);
  AMG_HIP(hipMemsetAsync(mx.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_tile_nnz_max, dim3(cdiv(ntiles, 256)), dim3(256), 0, s, n, T, ntiles, L.rowptr, mx.as<int>());
  // neighbour-tile entries, the hash-set overflow flag of the counting pass
  // (the listing pass hashes the same keys) and the largest tile's entries
  int nadj = 0, overflow = 0, Ecap = 0;
  read_ints(s, {{&nadj, tptr.as<int>() + ntiles}, {&overflow, cnt.as<int>()}, {&Ecap, mx.as<int>()}});
  if (overflow) fail(AMG_ERR_UNSUPPORTED, "a tile has more than 2048 neighbour tiles");
  DBuf tadj((size_t)std::max(nadj, 1) * sizeof(int), s);
  hipLaunchKernelGGL(k_tile_nbrs, dim3(ntiles), dim3(WAVE), 0, s, n, T, L.rowptr, L.colind, seed, tptr.as<int>(),
                     tadj.as<int>(), nullptr, nullptr, cnt.as<int>());
  AMG_HIP(hipGetLastError());
  const size_t shm = col_smem(T, Ecap);
  if (shm > 160 * 1024) fail(AMG_ERR_UNSUPPORTED, "colouring tile exceeds LDS; use smaller tile_rows");
  AMG_HIP(hipFuncSetAttribute((const void*)k_colour_tiles, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  // Rounds: list the tiles whose neighbours before them are all done (ballot
  // compaction, one atomic per wavefront), then colour them.  Rounds are
  // enqueued 8 at a time; the host then checks whether any tile is left.
  // Every round colours at least one tile while any is left (the tile order
  // is acyclic), so ntiles rounds always suffice.
  int* list = w0.as<int>();
  int* lcnt = cnt.as<int>() + 2;
  const int grid = std::min(ntiles, 8192);
  for (int done = 0; done < ntiles;) {
    for (int k = 0; k < 8; ++k) {
      AMG_HIP(hipMemsetAsync(lcnt, 0, sizeof(int), s));
      hipLaunchKernelGGL(k_ready0, dim3(cdiv(ntiles, 256)), dim3(256), 0, s, ntiles, pend.as<int>(), list, lcnt);
      hipLaunchKernelGGL(k_colour_tiles, dim3(grid), dim3(WAVE), shm, s, n, T, list, lcnt, L.rowptr, L.colind,
                         tptr.as<int>(), tadj.as<int>(), pend.as<int>(), seed, L.colour, cnt.as<int>() + 1);
    }
    AMG_HIP(hipGetLastError());
    done += 8;
    AMG_HIP(hipMemsetAsync(lcnt, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_count_pending, dim3(cdiv(ntiles, 256)), dim3(256), 0, s, ntiles, pend.as<int>(), lcnt);
    if (read1(lcnt, s) == 0) break;
    if (done >= ntiles) fail(AMG_ERR_HIP, "tile colouring did not reach every tile");
  }
  const int C = read1(cnt.as<int>() + 1, s) + 1;
  if (C > 4096) fail(AMG_ERR_UNSUPPORTED, "more than 4096 colours");
  L.ncol = C;
  const int nblk = cdiv(n, CL_THREADS);
  DBuf bcnt((size_t)C * nblk * sizeof(int), s), gofs(((size_t)C * nblk + 1) * sizeof(int), s);
  hipLaunchKernelGGL(k_colour_hist, dim3(nblk), dim3(CL_THREADS), C * sizeof(int), s, n, L.colour, C, nblk,
                     bcnt.as<int>());
  exclusive_scan(bcnt.as<int>(), gofs.as<int>(), C * nblk, s);
  L.crows = H.alloc<int>((size_t)n, s);
  hipLaunchKernelGGL(k_colour_place, dim3(nblk), dim3(CL_THREADS), (CL_THREADS / WAVE) * C * sizeof(int), s, n,
                     L.colour, C, nblk, gofs.as<int>(), L.crows);
  DBuf cp((size_t)(C + 1) * sizeof(int), s);
  hipLaunchKernelGGL(k_gather_cptr, dim3(cdiv(C + 1, 256)), dim3(256), 0, s, C, nblk, gofs.as<int>(), n, cp.as<int>());
  AMG_HIP(hipGetLastError());
  L.cptr.assign(C + 1, 0);
  AMG_HIP(hipMemcpyAsync(L.cptr.data(), cp.p, (C + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
  sync_stream(s);
}

// ---------------------------------------------------------------- hybrid smoother
__global__ void k_iota(int n, int* p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

void colour_single(Hierarchy& H, Level& L, hipStream_t s) {
  const int n = L.n;
  L.colour = H.alloc<int>((size_t)n, s);
  L.crows = H.alloc<int>((size_t)n, s);
  hipLaunchKernelGGL(k_fill, dim3(cdiv(n, 256)), dim3(256), 0, s, n, L.colour, 0);
  hipLaunchKernelGGL(k_iota, dim3(cdiv(n, 256)), dim3(256), 0, s, n, L.crows);
  AMG_HIP(hipGetLastError());
  L.ncol = 1;
  L.cptr = {0, n};
}

constexpr int HS_MAX_T = 1024;

// Wavefront steps of the sequential Gauss-Seidel sweeps inside one tile (one
// wavefront per tile, SELL slices of 64 consecutive rows, rows swept in solve
// order: natural order, or (colour, row) order on levels that sort each
// tile's rows by colour).  Forward: step(i) = 1 + the largest step of the
// rows j < i of the tile coupled to i (a_ij or a_ji stored), 0 without any;
// backward the same with j > i.  A row's step exceeds those of all its
// earlier-swept couplings, so updating the rows step by step reproduces the
// sequential sweep.  Found by monotone relaxation from 0 (each row pulls from
// its own entries and pushes to the rows its entries name); it stops at the
// fixed point, reached after at most nt rounds (a longest path has fewer than
// nt edges).
__global__ __launch_bounds__(64) void k_hybrid_steps(int n, int T, const int* __restrict__ soff,
                                                     const int* __restrict__ scol, unsigned short* __restrict__ sf,
                                                     unsigned short* __restrict__ sb, int* __restrict__ mx) {
  __shared__ int st[HS_MAX_T];
  const int lo = (int)blockIdx.x * T, hi = min(n, lo + T), nt = hi - lo;
  const int lane = (int)threadIdx.x;
  for (int dir = 0; dir < 2; ++dir) {
    for (int q = lane; q < nt; q += 64) st[q] = 0;
    __syncthreads();
    bool conv = false;
    for (int round = 0; round <= nt && !conv; ++round) {
      bool ch = false;
      for (int q = lane; q < nt; q += 64) {
        const int i = lo + q, sl = i >> 6, t = i & 63;
        const int base = soff[sl], w = (soff[sl + 1] - base) >> 6;
        int m = st[q];
        for (int k = 0; k < w; ++k) {
          const int j = scol[base + 64 * k + t];
          if (j >= lo && j < hi && (dir == 0 ? j < i : j > i)) m = max(m, st[j - lo] + 1);
        }
        if (m > st[q]) {
          st[q] = m;
          ch = true;
        }
        for (int k = 0; k < w; ++k) {
          const int j = scol[base + 64 * k + t];
          if (j >= lo && j < hi && (dir == 0 ? j > i : j < i) && atomicMax(&st[j - lo], m + 1) < m + 1) ch = true;
        }
      }
      __syncthreads();
      conv = __ballot(ch) == 0;
    }
    if (!conv) atomicOr(mx + 2, 1);
    if (dir == 0) {  // the most in-tile couplings of a row (LDS layout of the sweeps)
      int cmax = 0;
      for (int q = lane; q < nt; q += 64) {
        const int i = lo + q, sl = i >> 6, t = i & 63;
        const int base = soff[sl], w = (soff[sl + 1] - base) >> 6;
        int c = 0;
        for (int k = 0; k < w; ++k) {
          const int j = scol[base + 64 * k + t];
          c += (j >= lo && j < hi && j != i) ? 1 : 0;
        }
        cmax = max(cmax, c);
      }
      cmax = wave_max(cmax);
      if (lane == 0) atomicMax(mx + 3, cmax);
    }
    int dmax = 0;
    for (int q = lane; q < nt; q += 64) {
      (dir == 0 ? sf : sb)[lo + q] = (unsigned short)st[q];
      dmax = max(dmax, st[q]);
    }
    dmax = wave_max(dmax);
    if (lane == 0) atomicMax(mx + dir, dmax);
    __syncthreads();
  }
}

// Colouring of a level of the tile-ordered multicolour smoother: each tile of
// T rows (natural order) on its own, first fit over its rows in ascending
// order on the couplings inside the tile (one wavefront per tile).  A row
// takes its colour once every earlier coupled row of the tile has one, so
// rows are coloured in rounds; the result is the sequential first fit.  The
// tile's couplings to earlier rows are staged in LDS first (16-bit local
// indices, TL_STAGE_PER_ROW per row of the tile on average; a tile with more
// reads the matrix in every round instead), so that a round costs a few LDS
// reads per row.  LDS: colours and offsets (2T + 1 ints), then the staging.
// mx[0]: most colours, mx[1]: set when a row would need more than 256.
constexpr int TL_MAXC = 256;
constexpr int TL_STAGE_PER_ROW = 16;
inline size_t tile_local_lds_bytes(int T) {
  return (size_t)(2 * T + 1) * sizeof(int) + (size_t)T * TL_STAGE_PER_ROW * sizeof(unsigned short);
}
__global__ __launch_bounds__(64) void k_colour_tile_local(int n, int T, const int* __restrict__ rowptr,
                                                          const int* __restrict__ colind, int* __restrict__ colour,
                                                          int* __restrict__ mx) {
  extern __shared__ int tl_lds[];
  int* cl = tl_lds;
  int* lp = tl_lds + T;
  unsigned short* la = reinterpret_cast<unsigned short*>(tl_lds + 2 * T + 1);
  const int lo = (int)blockIdx.x * T, hi = min(n, lo + T), nt = hi - lo;
  const int lane = (int)threadIdx.x;
  // earlier in-tile couplings per row, their offsets
  int carry = 0;
  for (int base = 0; base < nt; base += 64) {
    const int q = base + lane;
    int cnt = 0;
    if (q < nt) {
      const int i = lo + q;
      for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int j = colind[k];
        cnt += (j >= lo && j < i) ? 1 : 0;
      }
    }
    const int inc = wave_incl_scan(cnt);
    if (q < nt) lp[q] = carry + inc - cnt;
    carry += __shfl(inc, 63, 64);
  }
  if (lane == 0) lp[nt] = carry;
  const bool staged = carry <= T * TL_STAGE_PER_ROW;
  for (int q = lane; q < nt; q += 64) cl[q] = -1;
  __syncthreads();
  if (staged) {
    for (int q = lane; q < nt; q += 64) {
      const int i = lo + q;
      int pos = lp[q];
      for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int j = colind[k];
        if (j >= lo && j < i) la[pos++] = (unsigned short)(j - lo);
      }
    }
    __syncthreads();
  }
  for (int round = 0; round <= nt; ++round) {
    bool left = false;
    for (int q = lane; q < nt; q += 64) {
      if (cl[q] >= 0) continue;
      const int i = lo + q;
      unsigned long long used[TL_MAXC / 64] = {0, 0, 0, 0};
      bool ready = true;
      if (staged) {
        const int e = lp[q + 1];
        for (int k0 = lp[q]; k0 < e && ready; k0 += 8) {
          int c8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) c8[u] = k0 + u < e ? cl[la[k0 + u]] : TL_MAXC;  // past the row: no colour
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (c8[u] < 0) ready = false;
            else if (c8[u] < TL_MAXC) used[c8[u] >> 6] |= 1ull << (c8[u] & 63);
          }
        }
      } else {
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
          const int j = colind[k];
          if (j < lo || j >= i) continue;
          const int c = cl[j - lo];
          if (c < 0) {
            ready = false;
            break;
          }
          used[c >> 6] |= 1ull << (c & 63);
        }
      }
      if (!ready) {
        left = true;
        continue;
      }
      int c = 0;
      while (c < TL_MAXC && ((used[c >> 6] >> (c & 63)) & 1ull)) ++c;
      if (c == TL_MAXC) {
        atomicOr(mx + 1, 1);
        c = TL_MAXC - 1;
      }
      cl[q] = c;
    }
    __syncthreads();
    if (!__ballot(left)) break;
  }
  int cmax = 0;
  for (int q = lane; q < nt; q += 64) {
    colour[lo + q] = cl[q];
    cmax = max(cmax, cl[q] + 1);
  }
  cmax = wave_max(cmax);
  if (lane == 0) atomicMax(mx, cmax);
}

void colour_tile_local(Hierarchy& H, Level& L, int T, hipStream_t s) {
  const int n = L.n, ntiles = cdiv(n, T);
  if (T > HS_MAX_T) fail(AMG_ERR_UNSUPPORTED, "tile sweeps take tiles of at most 1024 rows");
  L.colour = H.alloc<int>((size_t)n, s);
  DBuf mx(2 * sizeof(int), s);
  AMG_HIP(hipMemsetAsync(mx.p, 0, 2 * sizeof(int), s));
  hipLaunchKernelGGL(k_colour_tile_local, dim3(ntiles), dim3(64), tile_local_lds_bytes(T), s, n, T, L.rowptr,
                     L.colind, L.colour, mx.as<int>());
  AMG_HIP(hipGetLastError());
  int bad = 0;
  read_ints(s, {{&L.ncol, mx.as<int>()}, {&bad, mx.as<int>() + 1}});
  if (bad) fail(AMG_ERR_UNSUPPORTED, "a tile row needs more than 256 colours");
}

// Rows of each tile of T rows grouped by colour (one wavefront per tile,
// ballot compaction, colour by colour, ascending row inside a colour): the
// solve order, the colour of each solve row, and each tile's colour bounds
// (tcb[t * (C + 1) + c] = first tile-local solve row of colour c).
__global__ __launch_bounds__(64) void k_tile_colour_order(int n, int T, int C, const int* __restrict__ colour,
                                                          int* __restrict__ crows, int* __restrict__ tcol,
                                                          int* __restrict__ tcb) {
  const int t = blockIdx.x, lo = t * T, hi = min(n, lo + T), nt = hi - lo;
  const int lane = (int)threadIdx.x;
  int base = 0;
  for (int c = 0; c < C; ++c) {
    if (lane == 0) tcb[(size_t)t * (C + 1) + c] = base;
    for (int q0 = 0; q0 < nt; q0 += 64) {
      const int q = q0 + lane;
      const bool f = q < nt && colour[lo + q] == c;
      const unsigned long long m = __ballot(f);
      if (f) {
        const int p = base + __popcll(m & ((1ull << lane) - 1ull));
        crows[lo + p] = lo + q;
        tcol[lo + p] = c;
      }
      base += __popcll(m);
    }
  }
  if (lane == 0) tcb[(size_t)t * (C + 1) + C] = base;
}

void tile_colour_order(Hierarchy& H, Level& L, bool reorder, hipStream_t s) {
  const int n = L.n, T = L.T, C = L.ncol, ntiles = cdiv(n, T);
  L.tncol = C;
  H.free_one(L.crows, s);
  L.crows = nullptr;
  if (!reorder) {  // the coarsest level keeps its natural order: colours as they are
    L.tcol = L.colour;
    L.colour = nullptr;
    colour_single(H, L, s);
    return;
  }
  L.tcol = H.alloc<int>((size_t)n, s);
  L.crows = H.alloc<int>((size_t)n, s);
  L.tcb = H.alloc<int>((size_t)ntiles * (C + 1), s);
  hipLaunchKernelGGL(k_tile_colour_order, dim3(ntiles), dim3(64), 0, s, n, T, C, L.colour, L.crows, L.tcol, L.tcb);
  AMG_HIP(hipGetLastError());
  L.ncol = 1;
  L.cptr = {0, n};
}

void hybrid_steps(Hierarchy& H, Level& L, int T, hipStream_t s) {
  if (T > HS_MAX_T) fail(AMG_ERR_UNSUPPORTED, "the hybrid smoother takes tiles of at most 1024 rows");
  if (L.ncol != 1) fail(AMG_ERR_INVALID_ARG, "hybrid smoother level must have one colour");
  for (int q = 0; q < L.nsl; ++q)
    if (L.srow_h[q] != 64 * q) fail(AMG_ERR_HIP, "hybrid smoother expects slices of 64 consecutive rows");
  const int n = L.n, ntiles = cdiv(n, T);
  L.hsf = H.alloc<unsigned short>((size_t)n, s);
  L.hsb = H.alloc<unsigned short>((size_t)n, s);
  DBuf mx(4 * sizeof(int), s);
  AMG_HIP(hipMemsetAsync(mx.p, 0, 4 * sizeof(int), s));
  hipLaunchKernelGGL(k_hybrid_steps, dim3(ntiles), dim3(64), 0, s, n, T, L.soff, L.scol, L.hsf, L.hsb, mx.as<int>());
  AMG_HIP(hipGetLastError());
  int bad = 0;
  read_ints(s, {{&L.hdf, mx.as<int>()}, {&L.hdb, mx.as<int>() + 1}, {&bad, mx.as<int>() + 2}, {&L.hw, mx.as<int>() + 3}});
  if (bad) fail(AMG_ERR_HIP, "hybrid smoother step relaxation did not converge");
  if (std::max(L.hdf, L.hdb) >= 0xffff || L.hw >= 0xffff) fail(AMG_ERR_UNSUPPORTED, "hybrid smoother tile too deep");
}

// In-tile (ext = 0) or other-tile (ext = 1) couplings of row i (one thread
// per row; tiles of T rows): count, then (ptr set) columns (relative to the
// tile, or global) and values in SELL entry order.
__global__ void k_tile_rows(int n, int T, int ext, const int* __restrict__ soff, const int* __restrict__ scol,
                            const double* __restrict__ sval, const int* __restrict__ ptr, int* __restrict__ cnt,
                            unsigned short* __restrict__ col16, int* __restrict__ col32, double* __restrict__ v64,
                            float* __restrict__ v32, int* __restrict__ cmax) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int lo = i - i % T, hi = min(n, lo + T);
  const int t = i & 63, base = soff[i >> 6], w = (soff[(i >> 6) + 1] - base) >> 6;
  int c = ptr ? ptr[i] : 0;
  const bool vals = v64 || v32;
  for (int e0 = 0; e0 < w; e0 += 8) {  // 8 slots of the row per step, their loads in flight together
    int jj[8];
    double vv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) jj[u] = e0 + u < w ? scol[base + 64 * (e0 + u) + t] : -1;
#pragma unroll
    for (int u = 0; u < 8; ++u) vv[u] = vals && e0 + u < w ? sval[base + 64 * (e0 + u) + t] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (e0 + u >= w) break;
      const int j = jj[u];
      const bool in = j >= lo && j < hi;
      if (ext ? in : (!in || j == i)) continue;
      if (ptr) {
        if (col16) col16[c] = (unsigned short)(j - lo);
        if (col32) col32[c] = j;
        if (v64) v64[c] = vv[u];
        if (v32) v32[c] = (float)vv[u];
      }
      ++c;
    }
  }
  if (!ptr) {
    cnt[i] = c;
    if (cmax) atomicMax(cmax, c);
  }
}

__global__ void k_ic_tile_max(int n, int T, int ntiles, const int* __restrict__ icp, int* __restrict__ mx) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  atomicMax(mx, icp[min(n, (t + 1) * T)] - icp[t * T]);
}

void tile_couplings(Hierarchy& H, Level& L, bool f32, hipStream_t s) {
  const int n = L.n, T = L.T, g = cdiv(n, 256);
  DBuf cnt((size_t)n * sizeof(int), s), mx(2 * sizeof(int), s);
  AMG_HIP(hipMemsetAsync(mx.p, 0, 2 * sizeof(int), s));
  for (int ext = 0; ext < 2; ++ext) {
    int*& ptr = ext ? L.ocp : L.icp;
    hipLaunchKernelGGL(k_tile_rows, dim3(g), dim3(256), 0, s, n, T, ext, L.soff, L.scol, L.sval, nullptr,
                       cnt.as<int>(), nullptr, nullptr, nullptr, nullptr, ext ? nullptr : mx.as<int>() + 1);
    ptr = H.alloc<int>((size_t)n + 1, s);
    exclusive_scan(cnt.as<int>(), ptr, n, s);
    const int tot = read1(ptr + n, s);
    const size_t m = (size_t)std::max(tot, 1);
    unsigned short* c16 = ext ? nullptr : (L.icc = H.alloc<unsigned short>(m, s));
    int* c32 = ext ? (L.occ = H.alloc<int>(m, s)) : nullptr;
    double* v64 = nullptr;
    float* v32 = nullptr;
    if (f32)
      v32 = (ext ? L.ocv32 : L.icv32) = H.alloc<float>(m, s);
    else
      v64 = (ext ? L.ocv : L.icv) = H.alloc<double>(m, s);
    hipLaunchKernelGGL(k_tile_rows, dim3(g), dim3(256), 0, s, n, T, ext, L.soff, L.scol, L.sval, ptr, nullptr, c16,
                       c32, v64, v32, nullptr);
    (ext ? L.ocn : L.icn) = tot;
  }
  const int ntiles = cdiv(n, T);
  hipLaunchKernelGGL(k_ic_tile_max, dim3(cdiv(ntiles, 256)), dim3(256), 0, s, n, T, ntiles, L.icp, mx.as<int>());
  AMG_HIP(hipGetLastError());
  read_ints(s, {{&L.icmax, mx.as<int>()}, {&L.hw, mx.as<int>() + 1}});
  // rows with many in-tile couplings are summed by groups of lanes, except on
  // levels of the tile-ordered multicolour smoother (one lane per row:
  // the register form of its sweep keeps each row's couplings in one lane)
  L.hg = L.hw > 8 && !L.tcb ? HS_G : 1;
}

void cast_f32(const double* in, float* out, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_cast, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, in, out);
  AMG_HIP(hipGetLastError());
}

void l1_diag(const Level& L, double* o64, float* o32, hipStream_t s) {
  hipLaunchKernelGGL(k_l1, dim3(cdiv(L.n, 256)), dim3(256), 0, s, L.n, L.rowptr, L.vals, o64, o32);
  AMG_HIP(hipGetLastError());
}

void coarse_factor(Hierarchy& H, const Level& L, hipStream_t s) {
  const int n = L.n;
  H.nL = n;
  const size_t nn = (size_t)n * n;
  const int nb = cdiv(n, CB);
  DBuf D(nn * sizeof(double), s), W(nn * sizeof(double), s), f(sizeof(int), s);
  AMG_HIP(hipMemsetAsync(D.p, 0, nn * sizeof(double), s));
  AMG_HIP(hipMemsetAsync(W.p, 0, nn * sizeof(double), s));
  AMG_HIP(hipMemsetAsync(f.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_densify, dim3(cdiv(n, 256)), dim3(256), 0, s, n, L.rowptr, L.colind, L.vals, D.as<double>());
  for (int p = 0; p < nb; ++p) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(WAVE), 0, s, n, p, D.as<double>(), f.as<int>());
    const int rest = nb - p - 1;
    if (rest > 0) {
      hipLaunchKernelGGL(k_chol_trsm, dim3(rest), dim3(WAVE), 0, s, n, p, D.as<double>());
      hipLaunchKernelGGL(k_chol_update, dim3(rest * (rest + 1) / 2), dim3(256), 0, s, n, p, D.as<double>());
    }
  }
  AMG_HIP(hipGetLastError());
  if (read1(f.as<int>(), s)) fail(AMG_ERR_NOT_SPD, "coarsest-level Cholesky pivot <= 0");
  hipLaunchKernelGGL(k_trinv_diag, dim3(nb), dim3(WAVE), 0, s, n, D.as<double>(), W.as<double>());
  for (int bi = 1; bi < nb; ++bi)
    hipLaunchKernelGGL(k_trinv_row, dim3(bi), dim3(256), 0, s, n, bi, D.as<double>(), W.as<double>());
  H.Ainv = H.alloc<double>(nn, s);
  hipLaunchKernelGGL(k_wtw_blocks, dim3(nb * (nb + 1) / 2), dim3(256), 0, s, n, W.as<double>(), H.Ainv);
  AMG_HIP(hipGetLastError());
}

void gather(int n, const int* perm, const double* in, double* out, hipStream_t s) {
  if (!perm) {
    if (in != out) AMG_HIP(hipMemcpyAsync(out, in, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    return;
  }
  hipLaunchKernelGGL(k_gather, dim3(cdiv(n, 256)), dim3(256), 0, s, n, perm, in, out);
  AMG_HIP(hipGetLastError());
}

void scatter(int n, const int* perm, const double* in, double* out, hipStream_t s) {
  if (!perm) {
    if (in != out) AMG_HIP(hipMemcpyAsync(out, in, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    return;
  }
  hipLaunchKernelGGL(k_scatter, dim3(cdiv(n, 256)), dim3(256), 0, s, n, perm, in, out);
  AMG_HIP(hipGetLastError());
}

void permute_level(Hierarchy& H, int l, const int* next_perm, hipStream_t s) {
  Level& L = H.lev[l];
  const int n = L.n, nnz = L.nnz, nc = L.nc;
  const int g = cdiv(n, 256);
  int* perm = L.crows;  // rows grouped by colour, ascending: the solve order
  DBuf pinv((size_t)n * sizeof(int), s), len((size_t)n * sizeof(int), s);
  hipLaunchKernelGGL(k_invperm, dim3(g), dim3(256), 0, s, n, perm, pinv.as<int>());
  hipLaunchKernelGGL(k_perm_rowlen, dim3(g), dim3(256), 0, s, n, perm, L.rowptr, len.as<int>());
  int* prp = H.alloc<int>((size_t)n + 1, s);
  exclusive_scan(len.as<int>(), prp, n, s);
  int* pci = H.alloc<int>((size_t)nnz, s);
  double* pv = H.alloc<double>((size_t)nnz, s);
  int sub = 4;
  while (sub < 64 && (long long)sub * n < 2LL * nnz) sub *= 2;  // about the mean row length
  hipLaunchKernelGGL(k_perm_rows, dim3(std::min(cdiv(n, 256 / sub * PERM_ROWS), 1 << 20)), dim3(256), 0, s, n, sub,
                     perm,
                     pinv.as<int>(), L.rowptr, L.colind,
                     L.vals, prp, pci, pv);
  // Coarse solve index of each natural coarse row (NULL: the next level is the
  // coarsest and keeps its natural order).
  int* npinv = next_perm ? H.alloc<int>((size_t)nc, s) : nullptr;
  if (next_perm) hipLaunchKernelGGL(k_invperm, dim3(cdiv(nc, 256)), dim3(256), 0, s, nc, next_perm, npinv);
  int* pagg = H.alloc<int>((size_t)n, s);
  hipLaunchKernelGGL(k_perm_agg, dim3(g), dim3(256), 0, s, n, perm, L.agg, npinv, pagg);
  // Member lists stay in natural coarse order (the restriction walks
  // neighbouring aggregates together); members become fine solve rows.
  int* pmem = H.alloc<int>((size_t)n, s);
  hipLaunchKernelGGL(k_perm_members, dim3(cdiv(nc, 256)), dim3(256), 0, s, nc, nullptr, L.mptr, L.members,
                     pinv.as<int>(), L.mptr, pmem);
  AMG_HIP(hipGetLastError());
  sync_stream(s);
  for (void* p : {(void*)L.rowptr, (void*)L.colind, (void*)L.vals, (void*)L.agg, (void*)L.members,
                  (void*)L.tile_off, (void*)L.colour})
    H.free_one(p, s);
  L.rowptr = prp;
  L.colind = pci;
  L.vals = pv;
  L.agg = pagg;
  L.members = pmem;
  L.cinv = npinv;
  L.tile_off = nullptr;
  L.colour = nullptr;
  L.perm = perm;
  L.crows = nullptr;
}

void build_sell(Hierarchy& H, int l, hipStream_t s) {
  Level& L = H.lev[l];
  std::vector<int> srow_h;
  L.sptr.assign(L.ncol + 1, 0);
  const int step = L.bs > 1 ? 64 - 64 % L.bs : 64;  // slices hold whole nodes on point-based levels
  for (int c = 0; c < L.ncol; ++c) {
    L.sptr[c] = (int)srow_h.size();
    for (int r = L.cptr[c]; r < L.cptr[c + 1]; r += step) srow_h.push_back(r);
  }
  L.sptr[L.ncol] = (int)srow_h.size();
  srow_h.push_back(L.n);
  L.nsl = (int)srow_h.size() - 1;
  L.srow = H.alloc<int>(srow_h.size(), s);
  AMG_HIP(hipMemcpyAsync(L.srow, srow_h.data(), srow_h.size() * sizeof(int), hipMemcpyHostToDevice, s));
  DBuf w((size_t)L.nsl * sizeof(int), s);
  hipLaunchKernelGGL(k_sell_width, dim3(cdiv(L.nsl, 256)), dim3(256), 0, s, L.nsl, L.srow, L.rowptr, w.as<int>());
  L.soff = H.alloc<int>((size_t)L.nsl + 1, s);
  exclusive_scan(w.as<int>(), L.soff, L.nsl, s);
  L.srow_h = srow_h;
  L.soff_h.assign(L.nsl + 1, 0);
  AMG_HIP(hipMemcpyAsync(L.soff_h.data(), L.soff, ((size_t)L.nsl + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
  sync_stream(s);
  const int tot = L.soff_h[L.nsl];
  if (tot < 0) fail(AMG_ERR_UNSUPPORTED, "padded matrix exceeds 2^31 entries");
  L.scol = H.alloc<int>((size_t)tot, s);
  L.sval = H.alloc<double>((size_t)tot, s);
  L.dg = H.alloc<double>((size_t)L.n, s);
  hipLaunchKernelGGL(k_sell_fill, dim3(cdiv(L.nsl, 4)), dim3(256), 0, s, L.nsl, L.srow, L.soff, L.rowptr, L.colind,
                     L.vals, L.scol, L.sval, L.dg);
  AMG_HIP(hipGetLastError());
  sync_stream(s);
  if (l == 0 && H.p.spmv_format == 1) return;  // the outer product reads the CSR arrays (solve order)
  H.free_one(L.colind, s);
  H.free_one(L.vals, s);
  L.colind = nullptr;
  L.vals = nullptr;
}

// ---------------------------------------------------------------- point-based levels (host)
int validate_blocks(int n, int bs, const int* rp, const int* ci, hipStream_t s) {
  if (bs <= 1) return 0;
  if (bs > BLK_MAX) fail(AMG_ERR_UNSUPPORTED, "block_size above 4");
  if (n % bs) return 1;
  DBuf f(sizeof(int), s);
  AMG_HIP(hipMemsetAsync(f.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_validate_blocks, dim3(cdiv(n / bs, 256)), dim3(256), 0, s, n / bs, bs, rp, ci, f.as<int>());
  AMG_HIP(hipGetLastError());
  return read1(f.as<int>(), s);
}

void node_graph(Hierarchy& H, const Level& L, int bs, Level& S, hipStream_t s) {
  const int nn = L.n / bs;
  S = Level{};
  S.n = nn;
  S.T = L.T;
  S.rowptr = H.alloc<int>((size_t)nn + 1, s);
  DBuf cnt((size_t)nn * sizeof(int), s);
  hipLaunchKernelGGL(k_node_count, dim3(cdiv(nn, 256)), dim3(256), 0, s, nn, bs, L.rowptr, cnt.as<int>());
  exclusive_scan(cnt.as<int>(), S.rowptr, nn, s);
  S.nnz = read1(S.rowptr + nn, s);
  S.colind = H.alloc<int>((size_t)S.nnz, s);
  S.vals = H.alloc<double>((size_t)S.nnz, s);
  hipLaunchKernelGGL(k_node_fill, dim3(cdiv(nn, 256)), dim3(256), 0, s, nn, bs, L.rowptr, L.colind, L.vals,
                     S.rowptr, S.colind, S.vals);
  AMG_HIP(hipGetLastError());
}

void release_level(Hierarchy& H, Level& S, hipStream_t s) {
  for (void* p : {(void*)S.rowptr, (void*)S.colind, (void*)S.vals, (void*)S.agg, (void*)S.members, (void*)S.mptr,
                  (void*)S.tile_off, (void*)S.colour, (void*)S.crows})
    H.free_one(p, s);
  S = Level{};
}

void expand_aggregates(Hierarchy& H, const Level& S, int bs, Level& L, hipStream_t s) {
  const int n = L.n, ncn = S.nc;
  L.nc = ncn * bs;
  L.agg = H.alloc<int>((size_t)n, s);
  L.mptr = H.alloc<int>((size_t)L.nc + 1, s);
  L.members = H.alloc<int>((size_t)n, s);
  L.tile_off = nullptr;
  L.ntiles = S.ntiles;
  hipLaunchKernelGGL(k_expand_agg, dim3(cdiv(n, 256)), dim3(256), 0, s, n, bs, S.agg, L.agg);
  hipLaunchKernelGGL(k_expand_members, dim3(cdiv(ncn, 256)), dim3(256), 0, s, ncn, bs, S.mptr, S.members, L.mptr,
                     L.members);
  AMG_HIP(hipGetLastError());
}

void expand_colours(Hierarchy& H, const Level& S, int bs, Level& L, hipStream_t s) {
  const int n = L.n;
  L.colour = H.alloc<int>((size_t)n, s);
  L.crows = H.alloc<int>((size_t)n, s);
  hipLaunchKernelGGL(k_expand_colour, dim3(cdiv(n, 256)), dim3(256), 0, s, n, bs, S.colour, S.crows, L.colour,
                     L.crows);
  AMG_HIP(hipGetLastError());
  L.ncol = S.ncol;
  L.cptr.resize(S.cptr.size());
  for (size_t c = 0; c < S.cptr.size(); ++c) L.cptr[c] = S.cptr[c] * bs;
}

void block_inverses(Hierarchy& H, Level& L, int bs, bool f32, hipStream_t s) {
  const int nn = L.n / bs;
  L.dinv = H.alloc<double>((size_t)L.n * bs, s);
  DBuf f(sizeof(int), s);
  AMG_HIP(hipMemsetAsync(f.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_block_dinv, dim3(cdiv(nn, 128)), dim3(128), 0, s, nn, bs, L.rowptr, L.colind, L.vals, L.dinv,
                     f.as<int>());
  AMG_HIP(hipGetLastError());
  if (read1(f.as<int>(), s)) fail(AMG_ERR_BAD_DIAGONAL, "singular diagonal block");
  if (f32) {
    L.dinv32 = H.alloc<float>((size_t)L.n * bs, s);
    cast_f32(L.dinv, L.dinv32, (size_t)L.n * bs, s);
  }
}

}  // namespace amgx
