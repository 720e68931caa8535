// Plain, slow CPU oracle of the non-smoothed aggregation AMG preconditioned CG
// and BiCGSTAB
// (Blatt, Ippisch, Bastian: "A Massively Parallel Algebraic Multigrid
// Preconditioner based on Aggregation for Elliptic Problems with
// Heterogeneous Coefficients").
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library may link, load or
// call this file; only the tests, the smoke check and the CPU baseline leg of
// the benchmark use it.  It shares no code, header or table with the HIP path.
//
// Style: single-threaded, IEEE FP64 (built with -O2 -ffp-contract=off so that
// every multiply and add is rounded separately), set-based code that follows
// the paper's definitions and algorithm steps in their order.  Where the paper
// is silent, garbled or ambiguous the reading used here is stated next to the
// code; the same readings are listed with the design notes of the library.
//
// Parity status of each function (what pins it) is stated in its comment.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <set>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Status codes of the oracle (its own numbering).
enum {
  ORC_OK = 0,
  ORC_INVALID = 1,
  ORC_BAD_DIAGONAL = 2,
  ORC_NOT_SYMMETRIC = 3,
  ORC_NOT_SPD = 4,
  ORC_STALLED = 5,
  ORC_BREAKDOWN = 7,
  ORC_NOT_CONVERGED = 8,
};

struct Csr {
  int n = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
  int nnz() const { return (int)col.size(); }
};

// Stored entry a_ij, or 0 (with found=false) when (i,j) is not stored.
double entry(const Csr& A, int i, int j, bool* found) {
  for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
    if (A.col[k] == j) {
      if (found) *found = true;
      return A.val[k];
    }
  if (found) *found = false;
  return 0.0;
}

double diag_of(const Csr& A, int i) { return entry(A, i, i, nullptr); }

// ---------------------------------------------------------------------------
// Tiles: contiguous row ranges [t*T, min((t+1)*T, n)).  They play the role of
// the paper's non-overlapping index sets I_(p): aggregation only sees edges
// with both ends inside one tile (Sec. 3.3, Alg. 4, restriction of the graph to
// the edges E_(p)); one tile covering a whole small level stands in for the
// agglomeration onto one process (Sec. 3.3.1).
int tile_lo(int t, int T) { return t * T; }
int tile_hi(int t, int T, int n) { return std::min((t + 1) * T, n); }

// ---------------------------------------------------------------------------
// Strength of connection (Sec. 2.1, eqs. (symmetric_strong1), (symmetric_strong2)).
//
// Edge weight w_E((i,j)) = (a_ij - |a_ij|)/2 in the paper is <= 0 while the text
// calls it "the absolute value otherwise"; the reading is w_E = max(-a_ij, 0).
// Vertex weight w_V(i) = a_ii.
// s_ij = w_E(i,j) w_E(j,i) / (w_V(i) w_V(j)), evaluated as num/den with
// num = wij*wji and den = aii*ajj (each rounded once).
// eta_max(i) = max of s_ij over in-tile neighbours j (0 if none).
// (i,j) strong  iff s_ij > delta * min(eta_max(i), eta_max(j)).
// i isolated    iff eta_max(i) < beta.
double wE(double a) { return (-a > 0.0) ? -a : 0.0; }

double s_ij(const Csr& A, int i, int j) {
  double aij = entry(A, i, j, nullptr);
  double aji = entry(A, j, i, nullptr);
  double num = wE(aij) * wE(aji);
  double den = diag_of(A, i) * diag_of(A, j);
  return num / den;
}

void strength(const Csr& A, int T, double delta, double beta, std::vector<uint8_t>& strong,
              std::vector<uint8_t>& iso) {
  const int n = A.n;
  std::vector<double> eta(n, 0.0);
  for (int i = 0; i < n; ++i) {
    int t = i / T, lo = tile_lo(t, T), hi = tile_hi(t, T, n);
    double e = 0.0;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      int j = A.col[k];
      if (j == i || j < lo || j >= hi) continue;
      double s = s_ij(A, i, j);
      if (s > e) e = s;
    }
    eta[i] = e;
  }
  strong.assign(A.nnz(), 0);
  iso.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    int t = i / T, lo = tile_lo(t, T), hi = tile_hi(t, T, n);
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      int j = A.col[k];
      if (j == i || j < lo || j >= hi) continue;
      double m = eta[i] < eta[j] ? eta[i] : eta[j];
      strong[k] = (s_ij(A, i, j) > delta * m) ? 1 : 0;
    }
    iso[i] = (eta[i] < beta) ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// Greedy aggregation of one tile (Sec. 2.1, Alg. 1 "Build Aggregates" with
// Alg. 2 "Grow Aggregate" and Alg. 3 "Round Aggregate", run on the tile
// subgraph as in Alg. 4).  Readings of silent or garbled points:
//  * N(i) = stored off-diagonal in-tile columns of row i (the pattern is
//    structurally symmetric, so this equals the in-neighbour set of the paper).
//  * U = unaggregated non-isolated vertices (no Dirichlet rows exist: the
//    boundary is eliminated).  N_na(u) counts unaggregated in-tile neighbours.
//  * First seed and every "select v in S": smallest N_na, ties to smallest index.
//  * The next-seed front is S = N(a) n U; if it is empty, S = U.
//  * Grow: while |a| < s_min; candidates C0 = {c in N(a) n U : diam(a+c) <= d_max};
//    C1 = argmax of cons2 over C0 if that maximum is > 0, else argmax of cons1 if
//    > 0, else stop; ties by connect(c,a)/|N(c)| (exact integer cross
//    multiplication), then by neighbors(c,a), then by smallest index.
//  * connect(c,a) = sum over strong neighbours j of c outside a of 2 if j lies
//    in an aggregate that is already adjacent to a (has a vertex in N(a)), else 1.
//  * neighbors(c,a) = |(N(c) n U) \ N(a)|: the new candidates c would bring.
//  * Round: while |a| < s_max; D = {c in N(a) n U with a strong connection to a};
//    C = {c in D : |N(c) n a| > |N(c) n U|}; stop when C is empty, else add the
//    smallest index.  No diameter test.
//  * Single-vertex aggregate a = {v}: move v to the existing aggregate holding
//    the most strong neighbours of v (ties: smallest id); its id is freed.
//  * Isolated vertices (GrowIsoAggregate, not given in the paper): seed at the
//    smallest unaggregated isolated vertex; while |a| < s_min add the smallest
//    unaggregated isolated c in N(a) with diam(a+c) <= d_max whose set of
//    adjacent non-isolated aggregates meets that of a.
// Aggregate ids are dense per tile, in creation order.
struct TileGraph {
  int lo = 0, m = 0;
  std::vector<std::vector<int>> N;                 // local in-tile neighbours (ascending)
  std::vector<std::vector<uint8_t>> Nstrong;       // strong flag of each entry of N
  std::vector<uint8_t> iso;
};

TileGraph tile_graph(const Csr& A, const std::vector<uint8_t>& strong,
                     const std::vector<uint8_t>& iso, int t, int T) {
  TileGraph G;
  G.lo = tile_lo(t, T);
  int hi = tile_hi(t, T, A.n);
  G.m = hi - G.lo;
  G.N.resize(G.m);
  G.Nstrong.resize(G.m);
  G.iso.resize(G.m);
  for (int v = 0; v < G.m; ++v) {
    int i = G.lo + v;
    G.iso[v] = iso[i];
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      int j = A.col[k];
      if (j == i || j < G.lo || j >= hi) continue;
      G.N[v].push_back(j - G.lo);
      G.Nstrong[v].push_back(strong[k]);
    }
  }
  return G;
}

struct TileAggregator {
  const TileGraph& G;
  int smin, smax, dmax;
  std::vector<int> agg;  // local aggregate id, -1 = unaggregated
  int next_id = 0;

  TileAggregator(const TileGraph& g, int a, int b, int c) : G(g), smin(a), smax(b), dmax(c) {
    agg.assign(G.m, -1);
  }

  bool adjacent(int u, int w) const {
    for (int x : G.N[u])
      if (x == w) return true;
    return false;
  }
  bool strong_edge(int u, int w) const {  // edge (u,w) stored in row u and strong
    for (size_t k = 0; k < G.N[u].size(); ++k)
      if (G.N[u][k] == w) return G.Nstrong[u][k] != 0;
    return false;
  }
  bool inU(int v) const { return agg[v] < 0 && !G.iso[v]; }
  int Nna(int v) const {
    int c = 0;
    for (int j : G.N[v])
      if (agg[j] < 0) ++c;
    return c;
  }
  std::set<int> Nset(const std::set<int>& a) const {  // N(a): neighbours of a outside a
    std::set<int> s;
    for (int u : a)
      for (int j : G.N[u])
        if (!a.count(j)) s.insert(j);
    return s;
  }
  // Graph diameter of the subgraph induced by S (all tile edges); INT_MAX if
  // S is disconnected.
  int diameter(const std::set<int>& S) const {
    int best = 0;
    for (int src : S) {
      std::map<int, int> dist;
      std::vector<int> queue{src};
      dist[src] = 0;
      for (size_t h = 0; h < queue.size(); ++h) {
        int u = queue[h];
        for (int j : G.N[u])
          if (S.count(j) && !dist.count(j)) {
            dist[j] = dist[u] + 1;
            queue.push_back(j);
          }
      }
      if (dist.size() != S.size()) return std::numeric_limits<int>::max();
      for (auto& kv : dist) best = std::max(best, kv.second);
    }
    return best;
  }
  int cons2(int c, const std::set<int>& a) const {
    int k = 0;
    for (int j : a)
      if (strong_edge(c, j) && strong_edge(j, c)) ++k;
    return k;
  }
  int cons1(int c, const std::set<int>& a) const {
    int k = 0;
    for (int j : a)
      if (strong_edge(c, j) != strong_edge(j, c)) ++k;
    return k;
  }
  // connect(c,a) with adj = aggregates adjacent to a.
  long connect(int c, const std::set<int>& a, const std::set<int>& adj) const {
    long s = 0;
    for (size_t k = 0; k < G.N[c].size(); ++k) {
      int j = G.N[c][k];
      if (!G.Nstrong[c][k] || a.count(j)) continue;
      s += (agg[j] >= 0 && adj.count(agg[j])) ? 2 : 1;
    }
    return s;
  }
  // neighbors(c,a) with Na = N(a).
  long neighbors(int c, const std::set<int>& Na) const {
    long s = 0;
    for (int j : G.N[c])
      if (inU(j) && !Na.count(j)) ++s;
    return s;
  }
  void add(std::set<int>& a, int c, int id) {
    a.insert(c);
    agg[c] = id;
  }

  void grow(std::set<int>& a, int id) {
    while ((int)a.size() < smin) {
      const std::set<int> Na = Nset(a);
      std::vector<int> C0;
      for (int c : Na) {
        if (!inU(c)) continue;
        std::set<int> ac = a;
        ac.insert(c);
        if (diameter(ac) <= dmax) C0.push_back(c);
      }
      if (C0.empty()) break;
      int m2 = 0, m1 = 0;
      std::map<int, int> c2, c1;
      for (int c : C0) {
        c2[c] = cons2(c, a);
        c1[c] = cons1(c, a);
        m2 = std::max(m2, c2[c]);
        m1 = std::max(m1, c1[c]);
      }
      std::vector<int> C1;
      if (m2 > 0) {
        for (int c : C0)
          if (c2[c] == m2) C1.push_back(c);
      } else if (m1 > 0) {
        for (int c : C0)
          if (c1[c] == m1) C1.push_back(c);
      } else {
        break;
      }
      if (C1.size() > 1) {  // maximal connect(c,a)/|N(c)|, compared exactly
        std::set<int> adj;
        for (int w : Na)
          if (agg[w] >= 0) adj.insert(agg[w]);
        std::map<int, long> con;
        for (int c : C1) con[c] = connect(c, a, adj);
        std::vector<int> keep;
        for (int c : C1) {
          bool best = true;
          for (int w : C1)
            if (con[w] * (long)G.N[c].size() > con[c] * (long)G.N[w].size()) best = false;
          if (best) keep.push_back(c);
        }
        C1 = keep;
      }
      if (C1.size() > 1) {  // maximal neighbors(c,a)
        std::map<int, long> nb;
        long mx = -1;
        for (int c : C1) {
          nb[c] = neighbors(c, Na);
          mx = std::max(mx, nb[c]);
        }
        std::vector<int> keep;
        for (int c : C1)
          if (nb[c] == mx) keep.push_back(c);
        C1 = keep;
      }
      int c = *std::min_element(C1.begin(), C1.end());
      add(a, c, id);
    }
  }

  void round(std::set<int>& a, int id) {
    while ((int)a.size() < smax) {
      std::vector<int> C;
      for (int c : Nset(a)) {
        if (!inU(c)) continue;
        if (!(cons2(c, a) > 0 || cons1(c, a) > 0)) continue;
        int in_a = 0, in_U = 0;
        for (int j : G.N[c]) {
          if (a.count(j)) ++in_a;
          if (inU(j)) ++in_U;
        }
        if (in_a > in_U) C.push_back(c);
      }
      if (C.empty()) break;
      add(a, *std::min_element(C.begin(), C.end()), id);
    }
  }

  int pick_min_nna(const std::vector<int>& S) const {
    int best = -1, bn = 0;
    for (int v : S) {
      int k = Nna(v);
      if (best < 0 || k < bn || (k == bn && v < best)) {
        best = v;
        bn = k;
      }
    }
    return best;
  }

  void run() {
    // Phase 1: non-isolated vertices.
    auto U_list = [&]() {
      std::vector<int> u;
      for (int v = 0; v < G.m; ++v)
        if (inU(v)) u.push_back(v);
      return u;
    };
    std::vector<int> U = U_list();
    int v = U.empty() ? -1 : pick_min_nna(U);
    while (!U_list().empty()) {
      int id = next_id;
      std::set<int> a;
      add(a, v, id);
      grow(a, id);
      round(a, id);
      bool merged = false;
      if (a.size() == 1) {
        std::map<int, int> cnt;  // aggregate id -> number of strong neighbours of v in it
        for (size_t k = 0; k < G.N[v].size(); ++k) {
          int w = G.N[v][k];
          if (G.Nstrong[v][k] && agg[w] >= 0 && agg[w] != id) cnt[agg[w]]++;
        }
        if (!cnt.empty()) {
          int bk = -1, bc = -1;
          for (auto& kv : cnt)
            if (kv.second > bc) {  // ascending ids: strict '>' keeps the smallest on ties
              bc = kv.second;
              bk = kv.first;
            }
          agg[v] = bk;
          merged = true;
        }
      }
      if (!merged) ++next_id;
      std::vector<int> S;
      for (int w : Nset(a))
        if (inU(w)) S.push_back(w);
      std::vector<int> Ucur = U_list();
      if (!Ucur.empty()) {
        if (S.empty()) S = Ucur;
        v = pick_min_nna(S);
      }
    }
    const int phase1_ids = next_id;
    // Phase 2: isolated vertices.
    auto na_ids = [&](int x) {  // adjacent non-isolated (phase-1) aggregates of x
      std::set<int> s;
      for (int w : G.N[x])
        if (agg[w] >= 0 && agg[w] < phase1_ids) s.insert(agg[w]);
      return s;
    };
    for (int s0 = 0; s0 < G.m; ++s0) {
      if (!G.iso[s0] || agg[s0] >= 0) continue;
      int id = next_id++;
      std::set<int> a;
      add(a, s0, id);
      while ((int)a.size() < smin) {
        std::set<int> NAa;
        for (int u : a)
          for (int k : na_ids(u)) NAa.insert(k);
        int pick = -1;
        for (int c : Nset(a)) {  // ascending
          if (!G.iso[c] || agg[c] >= 0) continue;
          bool common = false;
          for (int k : na_ids(c))
            if (NAa.count(k)) common = true;
          if (!common) continue;
          std::set<int> ac = a;
          ac.insert(c);
          if (diameter(ac) > dmax) continue;
          pick = c;
          break;
        }
        if (pick < 0) break;
        add(a, pick, id);
      }
    }
  }
};

int aggregate_all(const Csr& A, const std::vector<uint8_t>& strong, const std::vector<uint8_t>& iso,
                  int T, int smin, int smax, int dmax, std::vector<int>& agg,
                  std::vector<int>* tile_counts) {
  const int n = A.n;
  const int ntiles = (n + T - 1) / T;
  agg.assign(n, -1);
  if (tile_counts) tile_counts->assign(ntiles, 0);
  int offset = 0;
  for (int t = 0; t < ntiles; ++t) {
    TileGraph G = tile_graph(A, strong, iso, t, T);
    TileAggregator ag(G, smin, smax, dmax);
    ag.run();
    for (int v = 0; v < G.m; ++v) agg[G.lo + v] = offset + ag.agg[v];
    if (tile_counts) (*tile_counts)[t] = ag.next_id;
    offset += ag.next_id;
  }
  return offset;
}

// ---------------------------------------------------------------------------
// Galerkin coarse operator (Sec. 2.1, eq. (prolongation) and the product
// P^T A P).  P(i,J) = 1 iff fine row i belongs to aggregate J (the paper's
// indices are swapped).  A_c(I,J) = sum over members i of a_I (ascending) and
// stored entries (i,j) of row i (CSR order) with agg[j] = J of a_ij, summed
// sequentially from the first term.  The pattern keeps explicit zeros.
// The paper scales by 1/omega; here A_c is stored unscaled and omega multiplies
// the prolongated correction on every level instead, which gives the same
// V-cycle by linearity.
Csr galerkin(const Csr& A, const std::vector<int>& agg, int nc) {
  std::vector<std::vector<int>> members(nc);
  for (int i = 0; i < A.n; ++i) members[agg[i]].push_back(i);  // ascending i
  Csr C;
  C.n = nc;
  C.ptr.assign(nc + 1, 0);
  for (int I = 0; I < nc; ++I) {
    std::map<int, double> row;
    for (int i : members[I])
      for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        int J = agg[A.col[k]];
        auto it = row.find(J);
        if (it == row.end())
          row[J] = A.val[k];
        else
          it->second = it->second + A.val[k];
      }
    for (auto& kv : row) {
      C.col.push_back(kv.first);
      C.val.push_back(kv.second);
    }
    C.ptr[I + 1] = (int)C.col.size();
  }
  return C;
}

// ---------------------------------------------------------------------------
// Multicolouring (not in the paper: the hot path replaces the hybrid smoother
// by multicolour symmetric Gauss-Seidel).  Greedy first-fit colouring in a
// fixed vertex order: the tiles (the same row ranges as the aggregation) are
// taken in descending key (fmix32(t xor s), t), with fmix32 the 32-bit
// finaliser of MurmurHash3 (public domain) and s the colour seed plus the
// level; inside a tile the rows are taken in ascending order.  Each row gets
// the smallest colour c >= 0 that none of its already coloured neighbours
// (stored off-diagonals, any tile) has.
uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

uint64_t tile_key(int t, uint32_t s) {
  return ((uint64_t)fmix32((uint32_t)t ^ s) << 32) | (uint32_t)t;
}

int colour_rows(const Csr& A, int T, uint32_t s, std::vector<int>& colour) {
  const int n = A.n;
  const int ntiles = (n + T - 1) / T;
  std::vector<int> tiles(ntiles);
  for (int t = 0; t < ntiles; ++t) tiles[t] = t;
  std::sort(tiles.begin(), tiles.end(), [&](int a, int b) { return tile_key(a, s) > tile_key(b, s); });
  colour.assign(n, -1);
  int ncol = 0;
  for (int t : tiles)
    for (int i = tile_lo(t, T); i < tile_hi(t, T, n); ++i) {
      std::set<int> used;
      for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        int j = A.col[k];
        if (j != i && colour[j] >= 0) used.insert(colour[j]);
      }
      int c = 0;
      while (used.count(c)) ++c;
      colour[i] = c;
      ncol = std::max(ncol, c + 1);
    }
  return ncol;
}

// Colouring of the tile-ordered multicolour smoother (not in the paper): each
// tile of T consecutive rows is coloured on its own, first fit over its rows
// in ascending order, looking only at couplings inside the tile (the smoother
// is block-Jacobi across tiles, so a colouring proper inside every tile
// orders each tile's sweep).  Returns the number of colours.
int colour_tile_local(const Csr& A, int T, std::vector<int>& colour) {
  const int n = A.n;
  colour.assign(n, -1);
  int ncol = 0;
  for (int lo = 0; lo < n; lo += T) {
    const int hi = std::min(n, lo + T);
    for (int i = lo; i < hi; ++i) {
      std::set<int> used;
      for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const int j = A.col[k];
        if (j != i && j >= lo && j < hi && colour[j] >= 0) used.insert(colour[j]);
      }
      int c = 0;
      while (used.count(c)) ++c;
      colour[i] = c;
      ncol = std::max(ncol, c + 1);
    }
  }
  return ncol;
}

// ---------------------------------------------------------------------------
// Dense FP64 Cholesky (Cholesky-Banachiewicz, lower triangle of A is read)
// for the coarsest level (the paper factorises it with a sparse direct solver).
int cholesky(int n, const std::vector<double>& Ad, std::vector<double>& L) {
  L.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = Ad[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s = s - L[(size_t)i * n + k] * L[(size_t)j * n + k];
      if (i == j) {
        if (!(s > 0.0)) return ORC_NOT_SPD;
        L[(size_t)i * n + i] = std::sqrt(s);
      } else {
        L[(size_t)i * n + j] = s / L[(size_t)j * n + j];
      }
    }
  return ORC_OK;
}

void chol_solve(int n, const std::vector<double>& L, const double* b, double* x) {
  std::vector<double> y(n);
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s = s - L[(size_t)i * n + k] * y[k];
    y[i] = s / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < n; ++k) s = s - L[(size_t)k * n + i] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
}

// ---------------------------------------------------------------------------
// Hierarchy and V-cycle (Sec. 2: smooth, restrict the residual with P^T,
// recurse, direct solve when small, prolongate, smooth).
struct Params {
  double delta, beta;
  int smin, smax, dmax;
  double omega;
  int coarse_max, max_levels, tile_rows;
  int smoother, pre, post, fp32, flexible;
  uint32_t colour_seed;
  int check_symmetry;
  int colour_tile_rows;  // rows per tile of the colouring order
  int block_size;        // unknowns per node (point-based AMG for systems); 1: scalar
  int coarse_smoother;   // smoother of the levels from coarse_from on (-1: `smoother` on every level)
  int coarse_from;
  // Blocks of the hybrid forms (Sec. 3.2: the matrices A_(p) of the block-
  // Jacobi) above level coarse_from and from it on; 0: tile_rows, and the
  // finer levels' size respectively.  They need not match the aggregation
  // tiles.
  int smooth_tile_rows, coarse_smooth_tile_rows;
};

// SMOOTH_TILE_MCSGS (not in the paper): the hybrid form of Sec. 3.2
// (block-Jacobi over tiles of smooth_tile() rows, one symmetric Gauss-Seidel
// step inside each) with the rows of each tile taken in the order of the
// level's multicolouring (colour, then row), meant for coarse levels.
enum { SMOOTH_MCSGS = 0, SMOOTH_L1JACOBI = 1, SMOOTH_HYBRID = 2, SMOOTH_TILE_MCSGS = 3 };

// Smoother of level l.
int smoother_of(const Params& p, int l) {
  return (p.coarse_smoother >= 0 && l >= p.coarse_from) ? p.coarse_smoother : p.smoother;
}

// Rows per block of the hybrid smoothers on level l.
int smooth_tile(const Params& p, int l) {
  const int fine = p.smooth_tile_rows > 0 ? p.smooth_tile_rows : p.tile_rows;
  return (p.coarse_smooth_tile_rows > 0 && l >= p.coarse_from) ? p.coarse_smooth_tile_rows : fine;
}

struct Level {
  Csr A;
  std::vector<float> val32;
  std::vector<uint8_t> strong, iso;
  std::vector<int> agg;  // to level l+1 (empty on the coarsest level)
  int nc = 0;
  std::vector<int> colour;
  int ncol = 0;
  std::vector<std::vector<int>> rows_of_colour;  // ascending rows per colour
  std::vector<double> l1;                        // sum_j |a_ij|
  // point-based levels (block size bs > 1): inverse of every node's diagonal
  // block, row-major bs x bs per node, in FP64 and rounded to FP32
  std::vector<double> dinv;
  std::vector<float> dinv32;
  std::vector<std::vector<int>> nodes_of_colour;  // ascending nodes per colour
};

// ---------------------------------------------------------------------------
// Point-based AMG for systems (Sec. 4.2, with the block weights of Sec. 2.1).
// A level whose unknowns come in nodes of bs components is kept in scalar form:
// node i owns rows i*bs .. i*bs+bs-1, and every stored block A_ij is stored in
// full (its bs rows hold the bs columns j*bs .. j*bs+bs-1 side by side, in
// ascending column order).  The coarsening graph is the node graph with the
// row-sum norms of the blocks as weights: w_E((i,j)) = ||A_ij||_inf,
// w_V(i) = ||A_ii||_inf; strength, aggregation and colouring run on it and
// every decision holds for all bs unknowns of a node.  The prolongation is
// P (x) I_bs, so the Galerkin block (I,J) is the sum of the blocks A_ij over
// i in a_I, j in a_J (the scalar product P^T A P of the expanded P).

// Node graph with the block weights in the places the scalar criterion reads
// them: off-diagonal entry -||A_ij||_inf (so w_E = max(-a, 0) = the norm) and
// diagonal ||A_ii||_inf.
Csr node_weights(const Csr& A, int bs) {
  Csr S;
  S.n = A.n / bs;
  S.ptr.assign(S.n + 1, 0);
  for (int i = 0; i < S.n; ++i) {
    const int r0 = i * bs;
    const int nblk = (A.ptr[r0 + 1] - A.ptr[r0]) / bs;
    for (int q = 0; q < nblk; ++q) {
      const int J = A.col[A.ptr[r0] + q * bs] / bs;
      double nrm = 0.0;
      for (int c = 0; c < bs; ++c) {
        double rs = 0.0;
        for (int d = 0; d < bs; ++d) rs = rs + std::fabs(A.val[A.ptr[r0 + c] + q * bs + d]);
        nrm = std::max(nrm, rs);
      }
      S.col.push_back(J);
      S.val.push_back(J == i ? nrm : -nrm);
    }
    S.ptr[i + 1] = (int)S.col.size();
  }
  return S;
}

// Every node's rows have one pattern of whole blocks, the diagonal block
// included.
bool block_structure_ok(const Csr& A, int bs) {
  if (bs < 1 || A.n % bs) return false;
  for (int i = 0; i < A.n / bs; ++i) {
    const int r0 = i * bs, len = A.ptr[r0 + 1] - A.ptr[r0];
    if (len % bs) return false;
    bool diag = false;
    for (int c = 0; c < bs; ++c) {
      if (A.ptr[r0 + c + 1] - A.ptr[r0 + c] != len) return false;
      for (int q = 0; q < len / bs; ++q) {
        const int J = A.col[A.ptr[r0] + q * bs] / bs;
        for (int d = 0; d < bs; ++d)
          if (A.col[A.ptr[r0 + c] + q * bs + d] != J * bs + d) return false;
        if (J == i) diag = true;
      }
    }
    if (!diag) return false;
  }
  return true;
}

// Gauss-Jordan inverse with partial pivoting (largest magnitude, first on
// ties) of a bs x bs row-major block; false if a pivot is zero.
bool invert_block(int bs, const double* a, double* inv) {
  std::vector<double> m(a, a + bs * bs), e(bs * bs, 0.0);
  for (int c = 0; c < bs; ++c) e[c * bs + c] = 1.0;
  for (int c = 0; c < bs; ++c) {
    int piv = c;
    for (int r = c + 1; r < bs; ++r)
      if (std::fabs(m[r * bs + c]) > std::fabs(m[piv * bs + c])) piv = r;
    if (m[piv * bs + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < bs; ++k) {
        std::swap(m[c * bs + k], m[piv * bs + k]);
        std::swap(e[c * bs + k], e[piv * bs + k]);
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
  std::copy(e.begin(), e.end(), inv);
  return true;
}

// Block Gauss-Seidel update of node i (the smoother becomes a block smoother,
// Sec. 4.2): t_c = b_(i,c) - sum over the entries of row (i,c) outside the
// node's own block (CSR order) of a x; x_(i,c) = sum_d Dinv_i[c][d] t_d.
template <typename V>
void block_gs_node(const Csr& A, const V* val, const V* dinv, int bs, int i, const V* b, V* x) {
  V t[16];
  for (int c = 0; c < bs; ++c) {
    const int r = i * bs + c;
    V acc = b[r];
    for (int k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
      const int j = A.col[k];
      if (j / bs != i) acc = acc - val[k] * x[j];
    }
    t[c] = acc;
  }
  for (int c = 0; c < bs; ++c) {
    V s = 0;
    for (int d = 0; d < bs; ++d) s = s + dinv[(size_t)i * bs * bs + c * bs + d] * t[d];
    x[i * bs + c] = s;
  }
}

struct Hier {
  Params p;
  std::vector<Level> lev;
  std::vector<double> L;  // Cholesky factor of the coarsest matrix
  int nL = 0;
};

template <typename V>
struct Vec {
  std::vector<V> v;
};

// Gauss-Seidel update of row i with values `val` (double or float) and
// accumulation in type V: acc = b_i - sum_{j != i} a_ij x_j in CSR order,
// x_i = acc / a_ii.
template <typename V>
void gs_row(const Csr& A, const V* val, int i, const V* b, V* x) {
  V acc = b[i];
  V d = 0;
  for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
    int j = A.col[k];
    if (j == i)
      d = val[k];
    else
      acc = acc - val[k] * x[j];
  }
  x[i] = acc / d;
}

// One hybrid symmetric Gauss-Seidel step (Sec. 3.2, parallel smoothers):
// block-Jacobi over the tiles [tT, min((t+1)T, n)), and inside each tile one
// sequential Gauss-Seidel step, a forward then a backward sweep over its rows.
// Couplings to other tiles use the iterate from before the step (the defect
// is formed once, before any tile changes); couplings inside the tile use the
// current values.  Row update: acc = b_i - (couplings to other tiles, CSR
// order) - (couplings inside the tile except a_ii, CSR order); x_i = acc/a_ii.
// Rows of a tile are swept in natural order, or, given a colouring, in the
// order (colour, row) forward and its reverse backward.
// Parity pin: x + M^-1 (b - A x) with M = (D + L_B) D^-1 (D + U_B), L_B and
// U_B the strict triangles, in the sweep order, of the tile-block-diagonal
// part of A.
template <typename V>
void hybrid_sgs(const Csr& A, const V* val, int T, const V* b, V* x, const int* colour = nullptr) {
  const int n = A.n;
  const std::vector<V> xold(x, x + n);
  auto row = [&](int i, int lo, int hi) {
    V acc = b[i];
    V d = 0;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int j = A.col[k];
      if (j < lo || j >= hi) acc = acc - val[k] * xold[j];
    }
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int j = A.col[k];
      if (j == i)
        d = val[k];
      else if (j >= lo && j < hi)
        acc = acc - val[k] * x[j];
    }
    x[i] = acc / d;
  };
  for (int lo = 0; lo < n; lo += T) {
    const int hi = std::min(n, lo + T);
    std::vector<int> ord;  // the tile's rows in sweep order: natural, or (colour, row)
    for (int i = lo; i < hi; ++i) ord.push_back(i);
    if (colour) std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return colour[a] < colour[c]; });
    for (size_t q = 0; q < ord.size(); ++q) row(ord[q], lo, hi);
    for (size_t q = ord.size(); q-- > 0;) row(ord[q], lo, hi);
  }
}

template <typename V>
const V* level_vals(const Level& L);
template <>
const double* level_vals<double>(const Level& L) { return L.A.val.data(); }
template <>
const float* level_vals<float>(const Level& L) { return L.val32.data(); }

template <typename V>
const V* level_dinv(const Level& L);
template <>
const double* level_dinv<double>(const Level& L) { return L.dinv.data(); }
template <>
const float* level_dinv<float>(const Level& L) { return L.dinv32.data(); }

template <typename V>
void smooth(const Hier& H, int l, const V* b, V* x) {
  const Level& L = H.lev[l];
  const V* val = level_vals<V>(L);
  const int bs = H.p.block_size;
  if (bs > 1) {  // multicolour block symmetric Gauss-Seidel over the nodes
    const V* dinv = level_dinv<V>(L);
    for (int c = 0; c < L.ncol; ++c)
      for (int i : L.nodes_of_colour[c]) block_gs_node<V>(L.A, val, dinv, bs, i, b, x);
    for (int c = L.ncol - 1; c >= 0; --c)
      for (int i : L.nodes_of_colour[c]) block_gs_node<V>(L.A, val, dinv, bs, i, b, x);
    return;
  }
  const int sm = smoother_of(H.p, l);
  if (sm == SMOOTH_MCSGS) {
    for (int c = 0; c < L.ncol; ++c)  // forward sweep
      for (int i : L.rows_of_colour[c]) gs_row<V>(L.A, val, i, b, x);
    for (int c = L.ncol - 1; c >= 0; --c)  // backward sweep
      for (int i : L.rows_of_colour[c]) gs_row<V>(L.A, val, i, b, x);
  } else if (sm == SMOOTH_HYBRID) {
    hybrid_sgs<V>(L.A, val, smooth_tile(H.p, l), b, x);
  } else if (sm == SMOOTH_TILE_MCSGS) {
    hybrid_sgs<V>(L.A, val, smooth_tile(H.p, l), b, x, L.colour.data());
  } else {
    // l1-Jacobi (Baker, Falgout, Kolev, Yang 2011, pointwise): x += (b - A x) / d
    const int n = L.A.n;
    std::vector<V> r(n);
    for (int i = 0; i < n; ++i) {
      V acc = b[i];
      for (int k = L.A.ptr[i]; k < L.A.ptr[i + 1]; ++k) acc = acc - val[k] * x[L.A.col[k]];
      r[i] = acc;
    }
    for (int i = 0; i < n; ++i) x[i] = x[i] + r[i] / (V)L.l1[i];
  }
}

template <typename V>
void vcycle(const Hier& H, int l, const V* b, V* x) {
  const int Lc = (int)H.lev.size() - 1;
  const Level& L = H.lev[l];
  const int n = L.A.n;
  if (l == Lc) {
    std::vector<double> bd(n), xd(n);
    for (int i = 0; i < n; ++i) bd[i] = (double)b[i];
    chol_solve(n, H.L, bd.data(), xd.data());
    for (int i = 0; i < n; ++i) x[i] = (V)xd[i];
    return;
  }
  const V* val = level_vals<V>(L);
  for (int i = 0; i < n; ++i) x[i] = 0;
  for (int s = 0; s < H.p.pre; ++s) smooth<V>(H, l, b, x);
  // b_c[I] = sum over members i of a_I (ascending) of (b_i - A_i x)
  std::vector<V> bc(L.nc, (V)0), xc(L.nc, (V)0);
  for (int i = 0; i < n; ++i) {
    V acc = b[i];
    for (int k = L.A.ptr[i]; k < L.A.ptr[i + 1]; ++k) acc = acc - val[k] * x[L.A.col[k]];
    bc[L.agg[i]] = bc[L.agg[i]] + acc;
  }
  vcycle<V>(H, l + 1, bc.data(), xc.data());
  const V om = (V)H.p.omega;
  for (int i = 0; i < n; ++i) x[i] = x[i] + om * xc[L.agg[i]];
  for (int s = 0; s < H.p.post; ++s) smooth<V>(H, l, b, x);
}

void precond(const Hier& H, const double* r, double* z) {
  const int n = H.lev[0].A.n;
  if (H.p.fp32) {
    std::vector<float> rf(n), zf(n);
    for (int i = 0; i < n; ++i) rf[i] = (float)r[i];
    vcycle<float>(H, 0, rf.data(), zf.data());
    for (int i = 0; i < n; ++i) z[i] = (double)zf[i];
  } else {
    vcycle<double>(H, 0, r, z);
  }
}

double dot(int n, const double* a, const double* b) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s = s + a[i] * b[i];
  return s;
}

void spmv(const Csr& A, const double* x, double* y) {
  for (int i = 0; i < A.n; ++i) {
    double s = 0.0;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) s = s + A.val[k] * x[A.col[k]];
    y[i] = s;
  }
}

int validate(const Csr& A, int check_symmetry) {
  const int n = A.n;
  if (n <= 0 || (int)A.ptr.size() != n + 1 || A.ptr[0] != 0 || A.ptr[n] != A.nnz())
    return ORC_INVALID;
  for (int i = 0; i < n; ++i) {
    if (A.ptr[i + 1] < A.ptr[i]) return ORC_INVALID;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      int j = A.col[k];
      if (j < 0 || j >= n) return ORC_INVALID;
      if (k > A.ptr[i] && A.col[k - 1] >= j) return ORC_INVALID;
      if (!std::isfinite(A.val[k])) return ORC_INVALID;
    }
  }
  for (int i = 0; i < n; ++i) {
    bool f = false;
    double d = entry(A, i, i, &f);
    if (!f || !(d > 0.0)) return ORC_BAD_DIAGONAL;
  }
  for (int i = 0; i < n; ++i)
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      bool f = false;
      double t = entry(A, A.col[k], i, &f);
      if (!f) return ORC_NOT_SYMMETRIC;  // structural symmetry is always required
      if (check_symmetry && t != A.val[k]) return ORC_NOT_SYMMETRIC;
    }
  return ORC_OK;
}

bool finish_level(Level& L, const Params& p, int l) {
  const int bs = p.block_size;
  if (bs > 1) {  // colours of the node graph, each node's unknowns share its colour
    const Csr S = node_weights(L.A, bs);
    std::vector<int> nc;
    L.ncol = colour_rows(S, p.colour_tile_rows, p.colour_seed + (uint32_t)l, nc);
    L.colour.assign(L.A.n, 0);
    L.nodes_of_colour.assign(L.ncol, {});
    for (int i = 0; i < S.n; ++i) {
      L.nodes_of_colour[nc[i]].push_back(i);
      for (int c = 0; c < bs; ++c) L.colour[i * bs + c] = nc[i];
    }
    L.dinv.assign((size_t)S.n * bs * bs, 0.0);
    std::vector<double> blk(bs * bs);
    for (int i = 0; i < S.n; ++i) {
      for (int c = 0; c < bs; ++c)
        for (int k = L.A.ptr[i * bs + c]; k < L.A.ptr[i * bs + c + 1]; ++k)
          if (L.A.col[k] / bs == i) blk[c * bs + L.A.col[k] % bs] = L.A.val[k];
      if (!invert_block(bs, blk.data(), &L.dinv[(size_t)i * bs * bs])) return false;
    }
    L.dinv32.resize(L.dinv.size());
    for (size_t k = 0; k < L.dinv.size(); ++k) L.dinv32[k] = (float)L.dinv[k];
  } else if (smoother_of(p, l) == SMOOTH_HYBRID) {  // no multicolouring: one colour, natural order
    L.colour.assign(L.A.n, 0);
    L.ncol = 1;
  } else if (smoother_of(p, l) == SMOOTH_TILE_MCSGS) {
    L.ncol = colour_tile_local(L.A, smooth_tile(p, l), L.colour);
  } else {
    L.ncol = colour_rows(L.A, p.colour_tile_rows, p.colour_seed + (uint32_t)l, L.colour);
  }
  L.rows_of_colour.assign(L.ncol, {});
  for (int i = 0; i < L.A.n; ++i) L.rows_of_colour[L.colour[i]].push_back(i);
  L.val32.resize(L.A.nnz());
  for (int k = 0; k < L.A.nnz(); ++k) L.val32[k] = (float)L.A.val[k];
  L.l1.assign(L.A.n, 0.0);
  for (int i = 0; i < L.A.n; ++i) {
    double s = 0.0;
    for (int k = L.A.ptr[i]; k < L.A.ptr[i + 1]; ++k) s = s + std::fabs(L.A.val[k]);
    L.l1[i] = s;
  }
  return true;
}

int build(Hier& H, const Csr& A0) {
  const Params& p = H.p;
  const int bs = p.block_size;
  if (p.smoother < 0 || p.smoother > SMOOTH_TILE_MCSGS || p.coarse_smoother < -1 ||
      p.coarse_smoother > SMOOTH_TILE_MCSGS || p.smooth_tile_rows < 0 || p.coarse_smooth_tile_rows < 0 ||
      ((p.coarse_smoother >= 0 || p.coarse_smooth_tile_rows > 0) && p.coarse_from < 1))
    return ORC_INVALID;
  if (bs > 1 && (bs > 16 || p.smoother != SMOOTH_MCSGS || (p.coarse_smoother >= 0 && p.coarse_smoother != SMOOTH_MCSGS) ||
                 !block_structure_ok(A0, bs)))
    return ORC_INVALID;
  int st = validate(A0, p.check_symmetry);
  if (st) return st;
  H.lev.clear();
  H.lev.emplace_back();
  H.lev[0].A = A0;
  for (;;) {
    int l = (int)H.lev.size() - 1;
    Level& L = H.lev[l];
    if (L.A.n <= p.coarse_max || l == p.max_levels - 1) break;
    std::vector<int> agg;
    int nc = 0;
    if (bs > 1) {  // strength and aggregation of the node graph; P = P_nodes (x) I_bs
      const Csr S = node_weights(L.A, bs);
      strength(S, p.tile_rows, p.delta, p.beta, L.strong, L.iso);
      std::vector<int> nagg;
      const int ncn = aggregate_all(S, L.strong, L.iso, p.tile_rows, p.smin, p.smax, p.dmax, nagg, nullptr);
      if ((double)ncn > 0.9 * (double)S.n) break;  // coarsening stalled
      agg.assign(L.A.n, 0);
      for (int i = 0; i < S.n; ++i)
        for (int c = 0; c < bs; ++c) agg[i * bs + c] = nagg[i] * bs + c;
      nc = ncn * bs;
    } else {
      strength(L.A, p.tile_rows, p.delta, p.beta, L.strong, L.iso);
      nc = aggregate_all(L.A, L.strong, L.iso, p.tile_rows, p.smin, p.smax, p.dmax, agg, nullptr);
      if ((double)nc > 0.9 * (double)L.A.n) break;  // coarsening stalled
    }
    L.agg = agg;
    L.nc = nc;
    Csr C = galerkin(L.A, agg, nc);
    H.lev.emplace_back();
    H.lev.back().A = C;
  }
  for (size_t l = 0; l < H.lev.size(); ++l)
    if (!finish_level(H.lev[l], p, (int)l)) return ORC_BAD_DIAGONAL;  // singular diagonal block
  Level& Lc = H.lev.back();
  Lc.agg.clear();
  Lc.nc = 0;
  if (Lc.A.n > 4096) return ORC_STALLED;
  H.nL = Lc.A.n;
  std::vector<double> D((size_t)H.nL * H.nL, 0.0);
  for (int i = 0; i < H.nL; ++i)
    for (int k = Lc.A.ptr[i]; k < Lc.A.ptr[i + 1]; ++k) D[(size_t)i * H.nL + Lc.A.col[k]] = Lc.A.val[k];
  return cholesky(H.nL, D, H.L);
}

Csr make_csr(int n, int nnz, const int* ptr, const int* col, const double* val) {
  Csr A;
  A.n = n;
  A.ptr.assign(ptr, ptr + n + 1);
  A.col.assign(col, col + nnz);
  A.val.assign(val, val + nnz);
  return A;
}

}  // namespace

// ===========================================================================
// C interface for the tests (ctypes).  All pointers are host pointers.
extern "C" {

struct orc_params {
  double strength_threshold, isolated_threshold;
  int agg_min, agg_max, agg_diameter;
  double omega;
  int coarse_max, max_levels, tile_rows;
  int smoother, pre_sweeps, post_sweeps, vcycle_fp32, flexible;
  uint32_t colour_seed;
  int check_symmetry;
  int colour_tile_rows;
  int block_size;
  int coarse_smoother, coarse_from;
  int smooth_tile_rows, coarse_smooth_tile_rows;
};

static Params to_params(const orc_params* q) {
  Params p;
  p.delta = q->strength_threshold;
  p.beta = q->isolated_threshold;
  p.smin = q->agg_min;
  p.smax = q->agg_max;
  p.dmax = q->agg_diameter;
  p.omega = q->omega;
  p.coarse_max = q->coarse_max;
  p.max_levels = q->max_levels;
  p.tile_rows = q->tile_rows;
  p.smoother = q->smoother;
  p.pre = q->pre_sweeps;
  p.post = q->post_sweeps;
  p.fp32 = q->vcycle_fp32;
  p.flexible = q->flexible < 0 ? q->vcycle_fp32 : q->flexible;
  p.colour_seed = q->colour_seed;
  p.check_symmetry = q->check_symmetry;
  p.colour_tile_rows = q->colour_tile_rows;
  p.block_size = q->block_size < 1 ? 1 : q->block_size;
  p.coarse_smoother = q->coarse_smoother;
  p.coarse_from = q->coarse_from;
  p.smooth_tile_rows = q->smooth_tile_rows;
  p.coarse_smooth_tile_rows = q->coarse_smooth_tile_rows;
  return p;
}

int orc_validate(int n, int nnz, const int* ptr, const int* col, const double* val, int check_symmetry) {
  if (n <= 0 || !ptr || ptr[0] != 0 || ptr[n] != nnz) return ORC_INVALID;
  return validate(make_csr(n, nnz, ptr, col, val), check_symmetry);
}

void orc_strength(int n, int nnz, const int* ptr, const int* col, const double* val, int tile_rows,
                  double delta, double beta, uint8_t* strong, uint8_t* iso) {
  Csr A = make_csr(n, nnz, ptr, col, val);
  std::vector<uint8_t> s, is;
  strength(A, tile_rows, delta, beta, s, is);
  std::memcpy(strong, s.data(), s.size());
  std::memcpy(iso, is.data(), is.size());
}

// Aggregates of selected tiles: local ids written to agg_local[row] for rows of
// the listed tiles, and the aggregate count of each listed tile to counts[k].
void orc_aggregate_tiles(int n, int nnz, const int* ptr, const int* col, const uint8_t* strong,
                         const uint8_t* iso, int tile_rows, int smin, int smax, int dmax, int ntiles,
                         const int* tiles, int* agg_local, int* counts) {
  Csr A;
  A.n = n;
  A.ptr.assign(ptr, ptr + n + 1);
  A.col.assign(col, col + nnz);
  std::vector<uint8_t> s(strong, strong + nnz), is(iso, iso + n);
  for (int k = 0; k < ntiles; ++k) {
    TileGraph G = tile_graph(A, s, is, tiles[k], tile_rows);
    TileAggregator ag(G, smin, smax, dmax);
    ag.run();
    for (int v = 0; v < G.m; ++v) agg_local[G.lo + v] = ag.agg[v];
    counts[k] = ag.next_id;
  }
}

int orc_aggregate(int n, int nnz, const int* ptr, const int* col, const uint8_t* strong, const uint8_t* iso,
                  int tile_rows, int smin, int smax, int dmax, int* agg, int* tile_counts) {
  Csr A;
  A.n = n;
  A.ptr.assign(ptr, ptr + n + 1);
  A.col.assign(col, col + nnz);
  std::vector<uint8_t> s(strong, strong + nnz), is(iso, iso + n);
  std::vector<int> a, tc;
  int nc = aggregate_all(A, s, is, tile_rows, smin, smax, dmax, a, &tc);
  std::memcpy(agg, a.data(), sizeof(int) * n);
  if (tile_counts) std::memcpy(tile_counts, tc.data(), sizeof(int) * tc.size());
  return nc;
}

// Two calls: with ccol == NULL only cptr (nc+1) is filled; then ccol/cval.
int orc_galerkin(int n, int nnz, const int* ptr, const int* col, const double* val, const int* agg, int nc,
                 int* cptr, int* ccol, double* cval) {
  Csr A = make_csr(n, nnz, ptr, col, val);
  std::vector<int> a(agg, agg + n);
  Csr C = galerkin(A, a, nc);
  std::memcpy(cptr, C.ptr.data(), sizeof(int) * (nc + 1));
  if (ccol) std::memcpy(ccol, C.col.data(), sizeof(int) * C.col.size());
  if (cval) std::memcpy(cval, C.val.data(), sizeof(double) * C.val.size());
  return C.nnz();
}

int orc_colour(int n, int nnz, const int* ptr, const int* col, int tile_rows, uint32_t seed, int* colour) {
  Csr A;
  A.n = n;
  A.ptr.assign(ptr, ptr + n + 1);
  A.col.assign(col, col + nnz);
  std::vector<int> c;
  int k = colour_rows(A, tile_rows, seed, c);
  std::memcpy(colour, c.data(), sizeof(int) * n);
  return k;
}

uint32_t orc_fmix32(uint32_t h) { return fmix32(h); }

int orc_cholesky(int n, const double* A, double* L) {
  std::vector<double> a(A, A + (size_t)n * n), l;
  int st = cholesky(n, a, l);
  std::memcpy(L, l.data(), sizeof(double) * l.size());
  return st;
}

// One multicolour SGS step (forward then backward colour sweep) on x in place.
void orc_mcsgs(int n, int nnz, const int* ptr, const int* col, const double* val, const int* colour, int ncol,
               const double* b, double* x) {
  Csr A = make_csr(n, nnz, ptr, col, val);
  std::vector<std::vector<int>> rows(ncol);
  for (int i = 0; i < n; ++i) rows[colour[i]].push_back(i);
  for (int c = 0; c < ncol; ++c)
    for (int i : rows[c]) gs_row<double>(A, A.val.data(), i, b, x);
  for (int c = ncol - 1; c >= 0; --c)
    for (int i : rows[c]) gs_row<double>(A, A.val.data(), i, b, x);
}

// One hybrid SGS step with tiles of T rows on x in place.
// colour: NULL (natural order inside each tile) or n colours (tile rows
// taken in (colour, row) order).
void orc_hybrid_sgs(int n, int nnz, const int* ptr, const int* col, const double* val, int T, const double* b,
                    double* x, const int* colour) {
  Csr A = make_csr(n, nnz, ptr, col, val);
  hybrid_sgs<double>(A, A.val.data(), T, b, x, colour);
}

void* orc_setup(int n, int nnz, const int* ptr, const int* col, const double* val, const orc_params* q,
                int* status) {
  Hier* H = new Hier();
  H->p = to_params(q);
  if (n <= 0 || ptr[0] != 0 || ptr[n] != nnz) {
    *status = ORC_INVALID;
    delete H;
    return nullptr;
  }
  int st = build(*H, make_csr(n, nnz, ptr, col, val));
  *status = st;
  if (st) {
    delete H;
    return nullptr;
  }
  return H;
}

void orc_free(void* h) { delete (Hier*)h; }

int orc_num_levels(void* h) { return (int)((Hier*)h)->lev.size(); }

void orc_level_info(void* h, int l, int* n, int* nnz, int* ncol) {
  Level& L = ((Hier*)h)->lev[l];
  *n = L.A.n;
  *nnz = L.A.nnz();
  *ncol = L.ncol;
}

void orc_copy_level(void* h, int l, int* agg, int* colour, int* ptr, int* col, double* val, uint8_t* strong,
                    uint8_t* iso) {
  Level& L = ((Hier*)h)->lev[l];
  if (agg && !L.agg.empty()) std::memcpy(agg, L.agg.data(), sizeof(int) * L.A.n);
  if (colour) std::memcpy(colour, L.colour.data(), sizeof(int) * L.A.n);
  if (ptr) std::memcpy(ptr, L.A.ptr.data(), sizeof(int) * (L.A.n + 1));
  if (col) std::memcpy(col, L.A.col.data(), sizeof(int) * L.A.nnz());
  if (val) std::memcpy(val, L.A.val.data(), sizeof(double) * L.A.nnz());
  if (strong && !L.strong.empty()) std::memcpy(strong, L.strong.data(), L.strong.size());
  if (iso && !L.iso.empty()) std::memcpy(iso, L.iso.data(), L.iso.size());
}

void orc_coarse_factor(void* h, double* L) {
  Hier* H = (Hier*)h;
  std::memcpy(L, H->L.data(), sizeof(double) * H->L.size());
}

void orc_vcycle(void* h, const double* r, double* z) { precond(*(Hier*)h, r, z); }

// One application of level l's smoother (one symmetric Gauss-Seidel step, one
// l1-Jacobi sweep or one hybrid step, as the hierarchy's parameters select) to
// x in place, in FP64 (fp32 = 0) or with the level's FP32 values (fp32 = 1:
// b and x are rounded to float first and the result widened back).
void orc_smooth(void* h, int l, int fp32, const double* b, double* x) {
  const Hier& H = *(const Hier*)h;
  const int n = H.lev[l].A.n;
  if (fp32) {
    std::vector<float> bf(n), xf(n);
    for (int i = 0; i < n; ++i) {
      bf[i] = (float)b[i];
      xf[i] = (float)x[i];
    }
    smooth<float>(H, l, bf.data(), xf.data());
    for (int i = 0; i < n; ++i) x[i] = (double)xf[i];
  } else {
    smooth<double>(H, l, b, x);
  }
}

// Preconditioned CG (x0 given in x) or flexible CG (Polak-Ribiere beta).
// res_hist[k] = ||r_k|| / ||r_0||; iter_hist (n*(maxit+1), nullable) = x_k.
int orc_pcg(void* h, const double* b, double* x, double rtol, int maxit, int* iters, double* res_hist,
            double* iter_hist, double* true_rel) {
  Hier& H = *(Hier*)h;
  const Csr& A = H.lev[0].A;
  const int n = A.n;
  std::vector<double> r(n), z(n), p(n), q(n), rold(n), d(n);
  spmv(A, x, q.data());
  for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
  const double r0 = std::sqrt(dot(n, r.data(), r.data()));
  if (res_hist) res_hist[0] = 1.0;
  if (iter_hist) std::memcpy(iter_hist, x, sizeof(double) * n);
  *iters = 0;
  auto finish = [&](int st) {
    spmv(A, x, q.data());
    for (int i = 0; i < n; ++i) d[i] = b[i] - q[i];
    double bn = std::sqrt(dot(n, b, b));
    *true_rel = bn > 0.0 ? std::sqrt(dot(n, d.data(), d.data())) / bn : 0.0;
    return st;
  };
  if (r0 == 0.0) return finish(ORC_OK);
  precond(H, r.data(), z.data());
  p = z;
  double rho = dot(n, r.data(), z.data());
  if (!(rho > 0.0)) return finish(ORC_BREAKDOWN);
  for (int k = 1; k <= maxit; ++k) {
    spmv(A, p.data(), q.data());
    double pq = dot(n, p.data(), q.data());
    if (!(pq > 0.0)) return finish(ORC_BREAKDOWN);
    double alpha = rho / pq;
    for (int i = 0; i < n; ++i) {
      x[i] = x[i] + alpha * p[i];
      rold[i] = r[i];
      r[i] = r[i] - alpha * q[i];
    }
    double res = std::sqrt(dot(n, r.data(), r.data()));
    *iters = k;
    if (res_hist) res_hist[k] = res / r0;
    if (iter_hist) std::memcpy(iter_hist + (size_t)k * n, x, sizeof(double) * n);
    if (res <= rtol * r0) return finish(ORC_OK);
    precond(H, r.data(), z.data());
    double rz = dot(n, r.data(), z.data());
    if (!(rz > 0.0)) return finish(ORC_BREAKDOWN);
    double beta;
    if (H.p.flexible) {
      for (int i = 0; i < n; ++i) d[i] = r[i] - rold[i];
      beta = dot(n, z.data(), d.data()) / rho;
    } else {
      beta = rz / rho;
    }
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    rho = rz;
  }
  return finish(ORC_NOT_CONVERGED);
}

}  // extern "C"

namespace {

// Preconditioned BiCGSTAB (van der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992),
// the outer solver of the paper's experiments (Sec. 5; it applies the
// preconditioner twice per iteration).  Right preconditioning: M is applied to
// the search directions p and s, so r stays the residual b - A x of the
// iterate and the stopping test ||r||^2 <= (rtol ||r_0||)^2 is on it.  The
// test is made twice per iteration, on s (x then holds x + alpha M p) and on
// r.  res_hist[k] and iter_hist[k] hold the residual norm ratio and the
// iterate where iteration k stopped (at s for a half-step exit; *half = 1).
// Breakdown: r~.v = 0, t.t = 0, omega = 0, or r~.r = 0 before convergence,
// or any of them not finite.  Parity pins: iterates equal to those of a
// library BiCGSTAB with the same preconditioner; exact preconditioner ->
// convergence at the first half step; recurrence residual equal to the
// residual of the iterate; a hand-built breakdown.
template <typename Prec>
int bicgstab(const Csr& A, const Prec& M, const double* b, double* x, double rtol, int maxit, int* iters,
             int* half, double* res_hist, double* iter_hist, double* true_rel) {
  const int n = A.n;
  std::vector<double> r(n), rt(n), p(n), ph(n), v(n), s(n), sh(n), t(n), d(n);
  spmv(A, x, t.data());
  for (int i = 0; i < n; ++i) r[i] = b[i] - t[i];
  const double rr0 = dot(n, r.data(), r.data());
  const double r0 = std::sqrt(rr0);
  const double tol2 = (rtol * r0) * (rtol * r0);
  if (res_hist) res_hist[0] = 1.0;
  if (iter_hist) std::memcpy(iter_hist, x, sizeof(double) * n);
  *iters = 0;
  *half = 0;
  auto finish = [&](int st) {
    spmv(A, x, t.data());
    for (int i = 0; i < n; ++i) d[i] = b[i] - t[i];
    const double bn = std::sqrt(dot(n, b, b));
    *true_rel = bn > 0.0 ? std::sqrt(dot(n, d.data(), d.data())) / bn : 0.0;
    return st;
  };
  auto record = [&](int k, double nrm2) {
    *iters = k;
    if (res_hist) res_hist[k] = std::sqrt(nrm2) / r0;
    if (iter_hist) std::memcpy(iter_hist + (size_t)k * n, x, sizeof(double) * n);
  };
  if (r0 == 0.0) return finish(ORC_OK);
  rt = r;  // shadow residual r~ = r_0
  p = r;
  double rho = rr0;  // r~ . r_0
  for (int k = 1; k <= maxit; ++k) {
    M(p.data(), ph.data());
    spmv(A, ph.data(), v.data());
    const double rv = dot(n, rt.data(), v.data());
    if (!(rv != 0.0) || !std::isfinite(rv)) return finish(ORC_BREAKDOWN);
    const double alpha = rho / rv;
    for (int i = 0; i < n; ++i) {
      s[i] = r[i] - alpha * v[i];
      x[i] = x[i] + alpha * ph[i];
    }
    const double ss = dot(n, s.data(), s.data());
    if (ss <= tol2) {
      *half = 1;
      record(k, ss);
      return finish(ORC_OK);
    }
    M(s.data(), sh.data());
    spmv(A, sh.data(), t.data());
    const double ts = dot(n, t.data(), s.data());
    const double tt = dot(n, t.data(), t.data());
    if (!(tt > 0.0) || !std::isfinite(tt)) return finish(ORC_BREAKDOWN);
    const double omega = ts / tt;
    if (!(omega != 0.0) || !std::isfinite(omega)) return finish(ORC_BREAKDOWN);
    for (int i = 0; i < n; ++i) {
      x[i] = x[i] + omega * sh[i];
      r[i] = s[i] - omega * t[i];
    }
    const double rr = dot(n, r.data(), r.data());
    record(k, rr);
    if (rr <= tol2) return finish(ORC_OK);
    const double rho_new = dot(n, rt.data(), r.data());
    if (!(rho_new != 0.0) || !std::isfinite(rho_new)) return finish(ORC_BREAKDOWN);
    const double beta = (rho_new / rho) * (alpha / omega);
    for (int i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
    rho = rho_new;
  }
  return finish(ORC_NOT_CONVERGED);
}

}  // namespace

extern "C" {

// BiCGSTAB preconditioned by one V-cycle of hierarchy h (x0 given in x).
int orc_bicgstab(void* h, const double* b, double* x, double rtol, int maxit, int* iters, int* half,
                 double* res_hist, double* iter_hist, double* true_rel) {
  const Hier& H = *(const Hier*)h;
  auto M = [&](const double* in, double* out) { precond(H, in, out); };
  return bicgstab(H.lev[0].A, M, b, x, rtol, maxit, iters, half, res_hist, iter_hist, true_rel);
}

// Unpreconditioned BiCGSTAB (M = I) on any CSR matrix (square, not
// necessarily symmetric), for the checks of the iteration itself.
int orc_bicgstab_plain(int n, int nnz, const int* ptr, const int* col, const double* val, const double* b,
                       double* x, double rtol, int maxit, int* iters, int* half, double* res_hist,
                       double* iter_hist, double* true_rel) {
  const Csr A = make_csr(n, nnz, ptr, col, val);
  auto M = [&](const double* in, double* out) { std::memcpy(out, in, sizeof(double) * A.n); };
  return bicgstab(A, M, b, x, rtol, maxit, iters, half, res_hist, iter_hist, true_rel);
}

}  // extern "C"
