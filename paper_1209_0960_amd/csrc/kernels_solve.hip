// Solve-phase kernels for gfx950: CSR products, multicolour Gauss-Seidel and
// l1-Jacobi sweeps, fused residual + restriction per aggregation tile,
// prolongation with the over-correction factor, the coarsest-level product
// with the explicit inverse, and the CG vector kernels.  All reductions use a
// fixed number of partial sums and a fixed tree, so results are reproducible
// run to run and independent of other work on the device.
#include "amg_internal.h"

namespace amgx {

namespace {

constexpr int WAVE = 64;

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Deterministic block sum (RED_THREADS threads): per-wave butterfly, then the
// wave sums in wave order.
__device__ inline double block_sum(double v) {
  __shared__ double ws[RED_THREADS / WAVE];
  v = wave_sum_d(v);
  const int w = threadIdx.x / WAVE;
  if (__lane_id() == 0) ws[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < RED_THREADS / WAVE; ++i) s += ws[i];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- products
template <typename V>
__global__ void k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ va,
                       const V* __restrict__ x, V* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  V s = 0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) s += va[k] * x[ci[k]];
  y[i] = s;
}

// y = A x with partial sums of x.y (grid-stride over a fixed grid).
__global__ __launch_bounds__(RED_THREADS) void k_spmv_dot(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci, const double* __restrict__ va,
                                                          const double* __restrict__ x, double* __restrict__ y,
                                                          double* __restrict__ partial) {
  double acc = 0.0;
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) {
    double s = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) s += va[k] * x[ci[k]];
    y[i] = s;
    acc += x[i] * s;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// r = b - A x with partial sums of r.r.
__global__ __launch_bounds__(RED_THREADS) void k_residual_dot(int n, const int* __restrict__ rp,
                                                              const int* __restrict__ ci,
                                                              const double* __restrict__ va,
                                                              const double* __restrict__ b,
                                                              const double* __restrict__ x, double* __restrict__ r,
                                                              double* __restrict__ partial) {
  double acc = 0.0;
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) {
    double s = b[i];
    for (int k = rp[i]; k < rp[i + 1]; ++k) s -= va[k] * x[ci[k]];
    r[i] = s;
    acc += s * s;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// ---------------------------------------------------------------- smoothers
// Gauss-Seidel update of the rows of one colour, which occupy the contiguous
// solve rows [lo, lo+cnt): x_i = (b_i - sum_{j!=i} a_ij x_j) / a_ii.
template <typename V>
__global__ void k_gs_colour(int lo, int cnt, const int* __restrict__ rp, const int* __restrict__ ci,
                            const V* __restrict__ va, const V* __restrict__ b, V* __restrict__ x) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const int i = lo + t;
  V acc = b[i], d = 1;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = ci[k];
    const V a = va[k];
    if (j == i)
      d = a;
    else
      acc -= a * x[j];
  }
  x[i] = acc / d;
}

template <typename V>
__global__ void k_resid(int n, const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ va,
                        const V* __restrict__ b, const V* __restrict__ x, V* __restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  V acc = b[i];
  for (int k = rp[i]; k < rp[i + 1]; ++k) acc -= va[k] * x[ci[k]];
  t[i] = acc;
}

template <typename V>
__global__ void k_jacobi_update(int n, const V* __restrict__ t, const V* __restrict__ d, V* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += t[i] / d[i];
}

// ---------------------------------------------------------------- sub-wave rows
// SUB consecutive lanes own one row: they read the row's entries as one
// contiguous stream (a wavefront covers 64/SUB consecutive rows in one
// coalesced load per entry block) and combine with a SUB-wide butterfly.
template <int SUB, typename V>
__device__ inline V group_sum(V v) {
#pragma unroll
  for (int o = SUB / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, SUB);
  return v;
}

// ---------------------------------------------------------------- SELL-64
// One wavefront per slice of 64 solve rows: lane t owns row srow[s] + t and
// reads its off-diagonal entry k at soff[s] + 64 k + t, so every load of the
// matrix is one contiguous 64-wide access; padding entries are (row, 0).
template <typename V>
__device__ inline V sell_offdiag(const int* __restrict__ scol, const V* __restrict__ sval, int base, int w, int lane,
                                 const V* __restrict__ x) {
  const int* cp = scol + base + lane;
  const V* vp = sval + base + lane;
  V acc = 0;
  int k = 0;
  for (; k + 2 <= w; k += 2) {
    const int j0 = cp[64 * k], j1 = cp[64 * (k + 1)];
    const V a0 = vp[64 * k], a1 = vp[64 * (k + 1)];
    acc += a0 * x[j0];
    acc += a1 * x[j1];
  }
  if (k < w) acc += vp[64 * k] * x[cp[64 * k]];
  return acc;
}

// Gauss-Seidel on the slices [s0, s0+ns) of one colour.
template <typename V>
__global__ __launch_bounds__(256) void k_gs_sell(int s0, int ns, const int* __restrict__ srow,
                                                 const int* __restrict__ soff, const int* __restrict__ scol,
                                                 const V* __restrict__ sval, const V* __restrict__ dg,
                                                 const V* __restrict__ b, V* __restrict__ x) {
  const int sl = s0 + (int)(blockIdx.x * 4 + threadIdx.x / WAVE);
  if (sl >= s0 + ns) return;
  const int lane = __lane_id();
  const int r = srow[sl] + lane;
  const int base = soff[sl], w = (soff[sl + 1] - base) >> 6;
  const V acc = sell_offdiag<V>(scol, sval, base, w, lane, x);
  if (r < srow[sl + 1]) x[r] = (b[r] - acc) / dg[r];
}

// t = b - A x over all slices.
template <typename V>
__global__ __launch_bounds__(256) void k_resid_sell(int nsl, const int* __restrict__ srow,
                                                    const int* __restrict__ soff, const int* __restrict__ scol,
                                                    const V* __restrict__ sval, const V* __restrict__ dg,
                                                    const V* __restrict__ b, const V* __restrict__ x,
                                                    V* __restrict__ t) {
  const int sl = (int)(blockIdx.x * 4 + threadIdx.x / WAVE);
  if (sl >= nsl) return;
  const int lane = __lane_id();
  const int r = srow[sl] + lane;
  const int base = soff[sl], w = (soff[sl + 1] - base) >> 6;
  const V acc = sell_offdiag<V>(scol, sval, base, w, lane, x);
  if (r < srow[sl + 1]) t[r] = b[r] - (dg[r] * x[r] + acc);
}

// y = A x (FP64) with deterministic partial sums of x.y over a fixed grid.
__global__ __launch_bounds__(RED_THREADS) void k_spmv_dot_sell(int nsl, const int* __restrict__ srow,
                                                               const int* __restrict__ soff,
                                                               const int* __restrict__ scol,
                                                               const double* __restrict__ sval,
                                                               const double* __restrict__ dg,
                                                               const double* __restrict__ x, double* __restrict__ y,
                                                               double* __restrict__ partial) {
  const int lane = __lane_id();
  const int wpb = RED_THREADS / WAVE;
  double acc = 0.0;
  for (int sl = blockIdx.x * wpb + threadIdx.x / WAVE; sl < nsl; sl += RED_BLOCKS * wpb) {
    const int r = srow[sl] + lane;
    const int base = soff[sl], w = (soff[sl + 1] - base) >> 6;
    const double off = sell_offdiag<double>(scol, sval, base, w, lane, x);
    if (r < srow[sl + 1]) {
      const double xr = x[r];
      const double yr = dg[r] * xr + off;
      y[r] = yr;
      acc += xr * yr;
    }
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// r = b - A x (FP64) with deterministic partial sums of r.r.
__global__ __launch_bounds__(RED_THREADS) void k_residual_dot_sell(int nsl, const int* __restrict__ srow,
                                                                   const int* __restrict__ soff,
                                                                   const int* __restrict__ scol,
                                                                   const double* __restrict__ sval,
                                                                   const double* __restrict__ dg,
                                                                   const double* __restrict__ b,
                                                                   const double* __restrict__ x,
                                                                   double* __restrict__ r,
                                                                   double* __restrict__ partial) {
  const int lane = __lane_id();
  const int wpb = RED_THREADS / WAVE;
  double acc = 0.0;
  for (int sl = blockIdx.x * wpb + threadIdx.x / WAVE; sl < nsl; sl += RED_BLOCKS * wpb) {
    const int i = srow[sl] + lane;
    const int base = soff[sl], w = (soff[sl + 1] - base) >> 6;
    const double off = sell_offdiag<double>(scol, sval, base, w, lane, x);
    if (i < srow[sl + 1]) {
      const double ri = b[i] - (dg[i] * x[i] + off);
      r[i] = ri;
      acc += ri * ri;
    }
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// y = A x with deterministic partial sums of x.y over a fixed grid.
template <int SUB>
__global__ __launch_bounds__(RED_THREADS) void k_spmv_dot_sub(int n, const int* __restrict__ rp,
                                                              const int* __restrict__ ci,
                                                              const double* __restrict__ va,
                                                              const double* __restrict__ x, double* __restrict__ y,
                                                              double* __restrict__ partial) {
  const int sl = threadIdx.x % SUB;
  const int gpb = RED_THREADS / SUB;
  double acc = 0.0;
  for (int i = blockIdx.x * gpb + threadIdx.x / SUB; i < n; i += RED_BLOCKS * gpb) {
    double s = 0.0;
    for (int k = rp[i] + sl; k < rp[i + 1]; k += SUB) s += va[k] * x[ci[k]];
    s = group_sum<SUB>(s);
    if (sl == 0) {
      y[i] = s;
      acc += x[i] * s;
    }
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// r = b - A x with deterministic partial sums of r.r.
template <int SUB>
__global__ __launch_bounds__(RED_THREADS) void k_residual_dot_sub(int n, const int* __restrict__ rp,
                                                                  const int* __restrict__ ci,
                                                                  const double* __restrict__ va,
                                                                  const double* __restrict__ b,
                                                                  const double* __restrict__ x,
                                                                  double* __restrict__ r, double* __restrict__ partial) {
  const int sl = threadIdx.x % SUB;
  const int gpb = RED_THREADS / SUB;
  double acc = 0.0;
  for (int i = blockIdx.x * gpb + threadIdx.x / SUB; i < n; i += RED_BLOCKS * gpb) {
    double s = 0.0;
    for (int k = rp[i] + sl; k < rp[i + 1]; k += SUB) s += va[k] * x[ci[k]];
    s = group_sum<SUB>(s);
    if (sl == 0) {
      const double ri = b[i] - s;
      r[i] = ri;
      acc += ri * ri;
    }
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Dispatch on the lanes-per-row width chosen for a level.
#define AMG_SUB_DISPATCH(SUBV, KERNEL_CALL) \
  switch (SUBV) {                           \
    case 4: {                               \
      constexpr int SUB = 4;                \
      KERNEL_CALL;                          \
    } break;                                \
    case 8: {                               \
      constexpr int SUB = 8;                \
      KERNEL_CALL;                          \
    } break;                                \
    case 16: {                              \
      constexpr int SUB = 16;               \
      KERNEL_CALL;                          \
    } break;                                \
    case 32: {                              \
      constexpr int SUB = 32;               \
      KERNEL_CALL;                          \
    } break;                                \
    default: {                              \
      constexpr int SUB = 64;               \
      KERNEL_CALL;                          \
    } break;                                \
  }

// ---------------------------------------------------------------- transfers
// b_c[I] = sum over the members of aggregate I (ascending natural order) of the
// residual t computed by k_resid.
template <typename V>
__global__ void k_restrict(int nc, const int* __restrict__ mptr, const int* __restrict__ members,
                           const V* __restrict__ t, V* __restrict__ bc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  V s = 0;
  for (int p = mptr[I]; p < mptr[I + 1]; ++p) s += t[members[p]];
  bc[I] = s;
}

template <typename V>
__global__ void k_prolong(int n, const int* __restrict__ agg, const V* __restrict__ xc, V* __restrict__ x, V omega) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += omega * xc[agg[i]];
}

// x = A_L^{-1} b with the explicit inverse: one wavefront per row, lanes over
// the (contiguous) row, butterfly sum.
template <typename Vin, typename Vout>
__global__ __launch_bounds__(256) void k_coarse_gemv(int n, const double* __restrict__ Ainv,
                                                     const Vin* __restrict__ b, Vout* __restrict__ x) {
  const int i = blockIdx.x * 4 + threadIdx.x / WAVE;
  if (i >= n) return;
  const int lane = __lane_id();
  double s = 0.0;
  const double* row = Ainv + (size_t)i * n;
  for (int j = lane; j < n; j += WAVE) s += row[j] * (double)b[j];
  s = wave_sum_d(s);
  if (lane == 0) x[i] = (Vout)s;
}

template <typename V>
__global__ void k_zero(int n, V* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

template <typename A, typename B>
__global__ void k_convert(int n, const A* __restrict__ in, B* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (B)in[i];
}

// ---------------------------------------------------------------- CG vectors
// x += alpha p; r_old = r (flexible); r -= alpha q; partial sums of r.r.
// A set breakdown flag turns the update into a no-op.
__global__ __launch_bounds__(RED_THREADS) void k_cg_update_xr(int n, double* __restrict__ x, double* __restrict__ r,
                                                              double* __restrict__ rold,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ q,
                                                              const double* __restrict__ scal,
                                                              double* __restrict__ partial) {
  const bool skip = scal[S_FLAG] != 0.0;
  const double alpha = scal[S_ALPHA];
  double acc = 0.0;
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) {
    double ri = r[i];
    if (!skip) {
      x[i] += alpha * p[i];
      if (rold) rold[i] = ri;
      ri -= alpha * q[i];
      r[i] = ri;
    }
    acc += ri * ri;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// partial sums of r.z and (flexible) z.(r - r_old) into partial[0..B) and [B..2B).
__global__ __launch_bounds__(RED_THREADS) void k_cg_dots_rz(int n, const double* __restrict__ r,
                                                            const double* __restrict__ z,
                                                            const double* __restrict__ rold,
                                                            double* __restrict__ partial) {
  double a = 0.0, c = 0.0;
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) {
    const double zi = z[i], ri = r[i];
    a += ri * zi;
    if (rold) c += zi * (ri - rold[i]);
  }
  const double ta = block_sum(a);
  const double tc = block_sum(c);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = ta;
    partial[RED_BLOCKS + blockIdx.x] = tc;
  }
}

__global__ void k_cg_update_p(int n, double* __restrict__ p, const double* __restrict__ z,
                              const double* __restrict__ scal) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || scal[S_FLAG] != 0.0) return;
  p[i] = z[i] + scal[S_BETA] * p[i];
}

__global__ __launch_bounds__(RED_THREADS) void k_dot(int n, const double* __restrict__ a,
                                                     const double* __restrict__ b, double* __restrict__ partial) {
  double acc = 0.0;
  for (int i = blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += RED_BLOCKS * RED_THREADS) acc += a[i] * b[i];
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(RED_THREADS) void k_finish(const double* __restrict__ partial, int nparts,
                                                        double* __restrict__ scal, int slot, int op) {
  double a = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nparts; i += RED_THREADS) {
    a += partial[i];
    if (op == FIN_BETA_FCG) c += partial[RED_BLOCKS + i];
  }
  a = block_sum(a);
  c = block_sum(c);
  if (threadIdx.x != 0) return;
  switch (op) {
    case FIN_STORE:
      scal[slot] = a;
      break;
    case FIN_ALPHA:
      scal[S_PQ] = a;
      if (!(a > 0.0)) scal[S_FLAG] = 1.0;
      scal[S_ALPHA] = scal[S_RHO] / a;
      break;
    case FIN_RHO_INIT:
      scal[S_RHO] = a;
      if (!(a > 0.0)) scal[S_FLAG] = 1.0;
      break;
    case FIN_BETA_PCG:
    case FIN_BETA_FCG: {
      scal[S_RZ] = a;
      scal[S_ZDR] = c;
      if (!(a > 0.0)) {
        scal[S_FLAG] = 1.0;
        break;
      }
      const double rho = scal[S_RHO];
      scal[S_BETA] = (op == FIN_BETA_FCG ? c : a) / rho;
      scal[S_RHO] = a;
      break;
    }
  }
}

// ---------------------------------------------------------------- level access
template <typename V>
struct LV;
template <>
struct LV<double> {
  static const double* svals(const Level& L) { return L.sval; }
  static const double* diag(const Level& L) { return L.dg; }
  static const double* vals(const Level& L) { return L.vals; }
  static double* x(Level& L) { return L.x64; }
  static double* b(Level& L) { return L.b64; }
  static double* t(Level& L) { return L.t64; }
  static const double* l1(const Level& L) { return L.l1; }
};
template <>
struct LV<float> {
  static const float* svals(const Level& L) { return L.sval32; }
  static const float* diag(const Level& L) { return L.dg32; }
  static const float* vals(const Level& L) { return L.vals32; }
  static float* x(Level& L) { return L.x32; }
  static float* b(Level& L) { return L.b32; }
  static float* t(Level& L) { return L.t32; }
  static const float* l1(const Level& L) { return L.l1_32; }
};

inline int kind_of(int l, int k) { return l == 0 ? k : AMG_KIND_COARSE_LEVELS; }

template <typename V>
double slice_bytes(const Level& L, int s0, int s1) {  // algorithmic bytes of a pass over slices [s0, s1)
  const double vb = sizeof(V);
  const double ent = (double)(L.soff_h[s1] - L.soff_h[s0]);
  const double rows = (double)(L.srow_h[s1] - L.srow_h[s0]);
  return ent * (4.0 + vb) + rows * 4.0 * vb + (s1 - s0) * 8.0;  // entries; b, diag, x read, x write; slice headers
}

template <typename V>
void smooth(Hierarchy& H, int l, const V* b, V* x, hipStream_t s) {
  Level& L = H.lev[l];
  const V* va = LV<V>::svals(L);
  const V* dg = LV<V>::diag(L);
  if (H.p.smoother == AMG_SMOOTHER_MCSGS) {
    for (int dir = 0; dir < 2; ++dir)
      for (int q = 0; q < L.ncol; ++q) {
        const int c = dir == 0 ? q : L.ncol - 1 - q;
        const int s0 = L.sptr[c], ns = L.sptr[c + 1] - s0;
        if (!ns) continue;
        KTimer tm(kind_of(l, AMG_KIND_SWEEP), s, slice_bytes<V>(L, s0, s0 + ns));
        hipLaunchKernelGGL(k_gs_sell<V>, dim3(cdiv(ns, 4)), dim3(256), 0, s, s0, ns, L.srow, L.soff, L.scol, va, dg, b,
                           x);
      }
  } else {
    V* t = LV<V>::t(L);
    {
      KTimer tm(kind_of(l, AMG_KIND_SWEEP), s, slice_bytes<V>(L, 0, L.nsl));
      hipLaunchKernelGGL(k_resid_sell<V>, dim3(cdiv(L.nsl, 4)), dim3(256), 0, s, L.nsl, L.srow, L.soff, L.scol, va, dg,
                         b, x, t);
    }
    {
      KTimer tm(kind_of(l, AMG_KIND_SWEEP), s, L.n * 4.0 * sizeof(V));
      hipLaunchKernelGGL(k_jacobi_update<V>, dim3(cdiv(L.n, 256)), dim3(256), 0, s, L.n, t, LV<V>::l1(L), x);
    }
  }
  AMG_HIP(hipGetLastError());
}

}  // namespace

template <typename V>
void vcycle(Hierarchy& H, int l, const V* b, V* x, hipStream_t s) {
  const int Lc = (int)H.lev.size() - 1;
  Level& L = H.lev[l];
  if (l == Lc) {
    KTimer tm(kind_of(l, AMG_KIND_COARSE_LEVELS), s, 8.0 * H.nL * H.nL);
    hipLaunchKernelGGL((k_coarse_gemv<V, V>), dim3(cdiv(H.nL, 4)), dim3(256), 0, s, H.nL, H.Ainv, b, x);
    AMG_HIP(hipGetLastError());
    return;
  }
  const double vb = sizeof(V);
  hipLaunchKernelGGL(k_zero<V>, dim3(cdiv(L.n, 256)), dim3(256), 0, s, L.n, x);
  for (int k = 0; k < H.p.pre_sweeps; ++k) smooth<V>(H, l, b, x, s);
  Level& C = H.lev[l + 1];
  {
    KTimer tm(kind_of(l, AMG_KIND_RESTRICT), s, slice_bytes<V>(L, 0, L.nsl));
    hipLaunchKernelGGL(k_resid_sell<V>, dim3(cdiv(L.nsl, 4)), dim3(256), 0, s, L.nsl, L.srow, L.soff, L.scol,
                       LV<V>::svals(L), LV<V>::diag(L), b, x, LV<V>::t(L));
  }
  {
    KTimer tm(kind_of(l, AMG_KIND_RESTRICT), s, L.n * (4.0 + vb) + L.nc * (4.0 + vb));
    hipLaunchKernelGGL(k_restrict<V>, dim3(cdiv(L.nc, 256)), dim3(256), 0, s, L.nc, L.mptr, L.members, LV<V>::t(L),
                       LV<V>::b(C));
    AMG_HIP(hipGetLastError());
  }
  vcycle<V>(H, l + 1, LV<V>::b(C), LV<V>::x(C), s);
  {
    KTimer tm(kind_of(l, AMG_KIND_PROLONG), s, L.n * (4.0 + 2 * vb) + L.nc * vb);
    hipLaunchKernelGGL(k_prolong<V>, dim3(cdiv(L.n, 256)), dim3(256), 0, s, L.n, L.agg, LV<V>::x(C), x,
                       (V)H.p.omega);
    AMG_HIP(hipGetLastError());
  }
  for (int k = 0; k < H.p.post_sweeps; ++k) smooth<V>(H, l, b, x, s);
}

template void vcycle<double>(Hierarchy&, int, const double*, double*, hipStream_t);
template void vcycle<float>(Hierarchy&, int, const float*, float*, hipStream_t);

void precond_apply(Hierarchy& H, const double* r, double* z, hipStream_t s) {
  if (!H.p.vcycle_fp32) {
    vcycle<double>(H, 0, r, z, s);
    return;
  }
  Level& L = H.lev[0];
  const int n = L.n;
  {
    KTimer tm(AMG_KIND_CG_VEC, s, 12.0 * n);
    hipLaunchKernelGGL((k_convert<double, float>), dim3(cdiv(n, 256)), dim3(256), 0, s, n, r, L.b32);
  }
  vcycle<float>(H, 0, L.b32, L.x32, s);
  {
    KTimer tm(AMG_KIND_CG_VEC, s, 12.0 * n);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(cdiv(n, 256)), dim3(256), 0, s, n, L.x32, z);
  }
  AMG_HIP(hipGetLastError());
}

void spmv64(const Level& L, const double* x, double* y, double* partial, hipStream_t s, int kind) {
  KTimer tm(kind, s, 12.0 * L.nnz + 4.0 * (L.n + 1) + 16.0 * L.n);
  if (!partial && L.scol) fail(AMG_ERR_HIP, "spmv64 on SELL level needs a partial buffer");
  if (L.scol) {
    hipLaunchKernelGGL(k_spmv_dot_sell, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, L.nsl, L.srow, L.soff, L.scol,
                       L.sval, L.dg, x, y, partial);
  } else if (partial) {
    AMG_SUB_DISPATCH(L.sub, hipLaunchKernelGGL(k_spmv_dot_sub<SUB>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, L.n,
                                               L.rowptr, L.colind, L.vals, x, y, partial));
  } else
    hipLaunchKernelGGL(k_spmv<double>, dim3(cdiv(L.n, 256)), dim3(256), 0, s, L.n, L.rowptr, L.colind, L.vals, x, y);
  AMG_HIP(hipGetLastError());
}

void residual64(const Level& L, const double* b, const double* x, double* r, double* partial, hipStream_t s) {
  KTimer tm(AMG_KIND_CG_VEC, s, 12.0 * L.nnz + 4.0 * (L.n + 1) + 24.0 * L.n);
  if (L.scol) {
    hipLaunchKernelGGL(k_residual_dot_sell, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, L.nsl, L.srow, L.soff, L.scol,
                       L.sval, L.dg, b, x, r, partial);
  } else {
    AMG_SUB_DISPATCH(L.sub, hipLaunchKernelGGL(k_residual_dot_sub<SUB>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, L.n,
                                               L.rowptr, L.colind, L.vals, b, x, r, partial));
  }
  AMG_HIP(hipGetLastError());
}

void cg_update_xr(int n, double* x, double* r, double* rold, const double* p, const double* q, const double* scal,
                  double* partial, hipStream_t s) {
  KTimer tm(AMG_KIND_CG_VEC, s, (rold ? 56.0 : 48.0) * n);
  hipLaunchKernelGGL(k_cg_update_xr, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, n, x, r, rold, p, q, scal, partial);
  AMG_HIP(hipGetLastError());
}

void cg_dots_rz(int n, const double* r, const double* z, const double* rold, double* partial, hipStream_t s) {
  KTimer tm(AMG_KIND_CG_VEC, s, (rold ? 24.0 : 16.0) * n);
  hipLaunchKernelGGL(k_cg_dots_rz, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, n, r, z, rold, partial);
  AMG_HIP(hipGetLastError());
}

void cg_update_p(int n, double* p, const double* z, const double* scal, hipStream_t s) {
  KTimer tm(AMG_KIND_CG_VEC, s, 24.0 * n);
  hipLaunchKernelGGL(k_cg_update_p, dim3(cdiv(n, 256)), dim3(256), 0, s, n, p, z, scal);
  AMG_HIP(hipGetLastError());
}

void dot_partial(int n, const double* a, const double* b, double* partial, hipStream_t s) {
  KTimer tm(AMG_KIND_CG_VEC, s, 16.0 * n);
  hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, n, a, b, partial);
  AMG_HIP(hipGetLastError());
}

void finish(double* partial, int nparts, double* scal, int slot, int op, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(RED_THREADS), 0, s, partial, nparts, scal, slot, op);
  AMG_HIP(hipGetLastError());
}

}  // namespace amgx
