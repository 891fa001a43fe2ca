// Host planner: quadtree, ring orderings, merge index maps, workspace layout
// and batched-launch descriptors for one (n, leaf, convection) build shape.
#include <map>
#include <mutex>
#include <cctype>
#include "plan.h"
#include "kernels.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <sstream>
#include <stdexcept>
#include <unordered_map>

namespace dtn {

static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

int user_depth(int n, int leaf) {
  int L = 0;
  while (ceil_div(n, 1 << L) > leaf) ++L;
  return L;
}

// Node at position r of a box ring listed counter-clockwise from the box's SW corner.
static void ring_node(const Rect& b, int r, int& i, int& j) {
  const int sx1 = b.sx() - 1, sy1 = b.sy() - 1;
  if (r < sx1) { i = b.x0 + r; j = b.y0; return; }
  r -= sx1;
  if (r < sy1) { i = b.x1 - 1; j = b.y0 + r; return; }
  r -= sy1;
  if (r < sx1) { i = b.x1 - 1 - r; j = b.y1 - 1; return; }
  r -= sx1;
  i = b.x0; j = b.y1 - 1 - r;
}

// Inverse of ring_node; -1 if (i, j) is not on the ring.
static int ring_pos(const Rect& b, int i, int j) {
  const int sx1 = b.sx() - 1, sy1 = b.sy() - 1;
  if (j == b.y0 && i >= b.x0 && i < b.x1 - 1) return i - b.x0;
  if (i == b.x1 - 1 && j >= b.y0 && j < b.y1 - 1) return sx1 + (j - b.y0);
  if (j == b.y1 - 1 && i > b.x0 && i <= b.x1 - 1) return sx1 + sy1 + (b.x1 - 1 - i);
  if (i == b.x0 && j > b.y0 && j <= b.y1 - 1) return 2 * sx1 + sy1 + (b.y1 - 1 - j);
  return -1;
}

// A node is eliminated by a merge when all four of its neighbours exist and lie in the union.
static bool interior_to(const Rect& u, int n, int i, int j) {
  const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
  for (int q = 0; q < 4; ++q) {
    int a = i + di[q], c = j + dj[q];
    if (a < 0 || a >= n || c < 0 || c >= n) return false;
    if (a < u.x0 || a >= u.x1 || c < u.y0 || c >= u.y1) return false;
  }
  return true;
}

// Node encoding of the index pool: (j << 16) | i (no divisions on the device).
static inline int enc(int i, int j) { return (j << 16) | i; }
static inline int enc_i(int p) { return p & 0xFFFF; }
static inline int enc_j(int p) { return p >> 16; }

// Standard normal samples for the range finder's test matrix: splitmix64 (Steele, Lea and
// Flood, 2014) drives the Box-Muller transform; deterministic for a given seed.
static void gaussian_fill(double* out, size_t cnt, unsigned long long seed) {
  unsigned long long x = seed;
  auto next = [&]() {
    unsigned long long z = (x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  };
  auto unif = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };   // (0, 1)
  const double two_pi = 6.283185307179586476925286766559;
  for (size_t q = 0; q < cnt; q += 2) {
    const double r = std::sqrt(-2.0 * std::log(unif())), t = two_pi * unif();
    out[q] = r * std::cos(t);
    if (q + 1 < cnt) out[q + 1] = r * std::sin(t);
  }
}

static bool adjacent(int, int p, int q) {
  return std::abs(enc_i(p) - enc_i(q)) + std::abs(enc_j(p) - enc_j(q)) == 1;
}

namespace {

struct Builder {
  Plan& P;
  // the problem whose tasks are being built
  int n = 0, sym = 0, definite = 0, net = 0;
  int cur_level = 1 << 30;   // quadtree level of the boxes the tasks being built produce
  double h2 = 0.0, cs = 0.0;
  long long coef_off = 0;
  explicit Builder(Plan& p) : P(p) {}

  void set_problem(const ProbPlan& pp) {
    n = pp.n;
    const double h = 1.0 / (pp.n - 1);
    h2 = h * h;
    cs = pp.conv == 1 ? h : 0.5 * h;
    coef_off = pp.coef_off;
    sym = pp.sym;
    definite = pp.definite;
    net = pp.net;
  }

  void stamp(SchurTask& t) const {
    t.cn = n;
    t.h2 = h2;
    t.cs = cs;
    t.coef = coef_off;
    // mirrored Schur products: every level of a definite problem; otherwise they are kept off the top
    // levels, where the interface blocks are worst conditioned
    t.sym = sym && (definite || cur_level >= kSymMinLevel);
    t.net = net;
  }

  GemmDesc gd(int M, int N, int K, int bA, long long oA, int lda, int bB, long long oB, int ldb,
              int bC, long long oC, int ldc, double alpha, double beta, int rmap, int cmap, int kmap) {
    GemmDesc g{};
    g.M = M; g.N = N; g.K = K;
    g.bufA = bA; g.bufB = bB; g.bufC = bC;
    g.offA = oA; g.offB = oB; g.offC = oC;
    g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.rmapC = rmap; g.cmapC = cmap; g.kmapA = kmap;
    g.tiles_m = ceil_div(M, kGemmBM);
    g.tiles_n = ceil_div(N, kGemmBN);
    g.alpha = alpha; g.beta = beta;
    g.kee = 0;
    return g;
  }

  void push(LaunchGemm& L, const GemmDesc& g0) {
    if (g0.M <= 0 || g0.N <= 0) return;
    GemmDesc g = g0;
    if (L.count == 0) L.first = (int)P.gemms.size();
    if (L.first + L.count != (int)P.gemms.size()) throw std::logic_error("non-contiguous launch descriptors");
    const double part = g.tri ? 0.5 : 1.0;   // a triangular block computes (about) half its entries
    L.flops += part * 2.0 * g.M * (double)g.N * g.K;
    L.bytes += 8.0 * ((double)g.M * g.K + (double)g.K * g.N + part * (g.beta != 0.0 ? 2.0 : 1.0) * g.M * (double)g.N);
    L.count++;
    P.gemms.push_back(g);
  }

  // Autotuner key of a launch: what its tile choice depends on.
  std::string launch_signature(const LaunchGemm& L, int tiles64) const {
    int M = 0, N = 0, K = 0, kee = 0, sym = 0, beta = 0;
    for (int q = 0; q < L.count; ++q) {
      const GemmDesc& g = P.gemms[L.first + q];
      M = std::max(M, g.M);
      N = std::max(N, g.N);
      K = std::max(K, g.K);
      kee |= g.kee > 0;
      sym |= g.tri || g.mirror;
      beta |= g.beta != 0.0;
    }
    return "d" + std::to_string(L.count) + "t" + std::to_string(tiles64) + "M" + std::to_string(M) + "N" +
           std::to_string(N) + "K" + std::to_string(K) + "a" + std::to_string(L.mode) + "e" + std::to_string(kee) +
           "s" + std::to_string(sym) + "b" + std::to_string(beta) + "f" + (P.fast ? "1" : "0");
  }

  // Pick the launch's workgroup tile and lay out its tiles.
  void finalize(LaunchGemm& L) {
    if (L.count == 0) return;
    int big_tiles = 0;
    bool all_wide = true;
    for (int q = 0; q < L.count; ++q) {
      const GemmDesc& g = P.gemms[L.first + q];
      big_tiles += ceil_div(g.M, 128) * ceil_div(g.N, 128);
      all_wide = all_wide && g.M >= 128 && g.N >= 128;
    }
    // tile per launch, by how many workgroups it would give: 128 x 128 (8 waves) when there are
    // at least kBigTileMin of them (half the operand traffic per flop of 64 x 64), 64 x 64 when
    // there are at least kSmallTileBelow of those, else 32 x 32 (4x the workgroups of 64 x 64).
    // FP32 launches of mixed-precision plans take 128 x 128 by the same rule (no tuned override), else 64 x 64.
    int tiles64 = 0;
    for (int q = 0; q < L.count; ++q) {
      const GemmDesc& g = P.gemms[L.first + q];
      tiles64 += ceil_div(g.M, 64) * ceil_div(g.N, 64);
    }
    bool any_plain = false, any_kmap = false, any_trans = false;
    for (int q = 0; q < L.count; ++q) {
      const GemmDesc& g = P.gemms[L.first + q];
      if (g.transA) any_trans = true;
      else if (g.kmapA >= 0) any_kmap = true;
      else any_plain = true;
    }
    L.mode = (int)any_plain + (int)any_kmap + (int)any_trans > 1 ? 3 : any_kmap ? 1 : any_trans ? 2 : 0;
    if (L.prec != 0) L.cfg = all_wide && big_tiles >= kBigTileMin && force_cfg < 0 ? 2 : 0;
    else if (all_wide && big_tiles >= kBigTileMin) L.cfg = 2;
    else L.cfg = tiles64 < kSmallTileBelow ? 3 : 0;
    // 32 x 32 tiles of a small launch walk K in chunks of 64 (latency: a quarter of the round trips)
    if (L.cfg == 3) {
      int t32 = 0;
      for (int q = 0; q < L.count; ++q) {
        const GemmDesc& g = P.gemms[L.first + q];
        t32 += ceil_div(g.M, 32) * ceil_div(g.N, 32);
      }
      if (t32 <= kDeepChunkTiles) L.cfg = 4;
    }
    L.sig = launch_signature(L, tiles64);
    if (force_cfg < 0 && L.prec == 0) {
      // autotuned tile (or the tile of a tuning run) when it suits the launch
      auto fits = [&](int c) { return c == 0 || c == 3 || c == 4 || (c == 2 && all_wide); };
      int c = -1;
      if (P.tune_force >= 0) {
        c = P.tune_force;
      } else if (tune_enabled()) {
        int t;
        if (tune_get(L.sig, t)) c = t;
      }
      if (c >= 0 && fits(c)) L.cfg = c;
    }
    if (force_cfg >= 0 && L.prec == 0) L.cfg = force_cfg;
    const int tm = L.cfg == 3 || L.cfg == 4 ? 32 : L.cfg == 2 ? 128 : 64, tn = tm;
    int out_tiles = 0, kmin = 1 << 30;
    for (int q = 0; q < L.count; ++q) {
      const GemmDesc& g = P.gemms[L.first + q];
      out_tiles += ceil_div(g.M, tm) * ceil_div(g.N, tn);
      kmin = std::min(kmin, g.K);
    }
    // split K when the output tiles alone would leave most CUs idle on a long K loop (fast-path plans
    // of phases with merge scratch: the partial tiles follow it, the counters are fresh int scratch)
    int S = 1;
    bool sym_blocks = false;   // triangular or mirrored blocks are not split
    for (int q = 0; q < L.count; ++q) sym_blocks = sym_blocks || P.gemms[L.first + q].tri || P.gemms[L.first + q].mirror;
    if (split_ok && P.fast && L.prec == 0 && !sym_blocks && out_tiles < kSplitTilesBelow && kmin >= kSplitMinK)
      S = std::max(1, std::min({kSplitMax, 2 * kSplitTilesBelow / std::max(out_tiles, 1), kmin / kSplitMinSlice}));
    L.tiles = 0;
    long long part = split_ws;
    for (int q = 0; q < L.count; ++q) {
      GemmDesc& g = P.gemms[L.first + q];
      g.tiles_m = ceil_div(g.M, tm);
      g.tiles_n = ceil_div(g.N, tn);
      const int dt = g.tri ? g.tiles_m * (g.tiles_m + 1) / 2 : g.tiles_m * g.tiles_n;   // tiles that run
      g.tile_start = L.tiles;
      g.ksplit = S;
      g.kcnt = -1;
      g.kpart = 0;
      if (S > 1) {
        g.kcnt = (int)P.int_ws;
        P.int_ws += (size_t)g.tiles_m * g.tiles_n;
        g.kpart = part;
        part += (long long)g.tiles_m * g.tiles_n * S * tm * tn;
      }
      L.tiles += dt * S;
    }
    if (S > 1) P.ws_doubles = std::max(P.ws_doubles, (size_t)part);
  }
  bool split_ok = false;     // set while finalizing a phase whose partials can follow its scratch
  int force_cfg = -1;        // >= 0: the tile configuration of the next finalized FP64 launch
  long long split_ws = 0;

  void finalize_phase(Phase& ph) {
    // mixed precision: the X and Schur products of every dense merge run on FP32 MFMA, and so do the
    // products of the recursive inversion below the top kMixedFp64Levels levels (the base-block
    // inverses, and the whole inversion of the largest interface blocks, stay FP64)
    if (P.mixed && P.fast) {
      if (ph.min_level >= kMixedFp64Levels)
        for (auto& op : ph.inv_ops) op.gemm.prec = 1;
      ph.xgemm.prec = 1;
      ph.sgemm.prec = 1;
      ph.sgemm_tri.prec = 1;
    }
    split_ok = P.fast && ph.ws_end > 0;
    split_ws = (ph.ws_end + 31) & ~31LL;
    for (auto& L : ph.gje_update) finalize(L);
    for (auto& op : ph.inv_ops) finalize(op.gemm);
    finalize(ph.xgemm);
    finalize(ph.sgemm);
    force_cfg = 0;   // lower-tile blocks on 64 x 64 tiles: finer rounds than 128 x 128 for half-full launches
    finalize(ph.sgemm_tri);
    force_cfg = -1;
    for (auto& op : ph.comp_ops) finalize(op.gemm);
    split_ok = false;
  }

  // Base box: K = M'[P, P] in the order [ring; interior], S written with leading dimension e.
  SchurTask base_task(const Rect& b, int dst, long long out) {
    SchurTask t{};
    t.kind = 0;
    const int e = b.ring();
    const int mi = std::max(0, b.sx() - 2) * std::max(0, b.sy() - 2);
    t.e = e; t.i = mi; t.e1 = e; t.i1 = mi;
    t.m1 = t.m2 = 0;
    t.idx = (int)P.ipool.size();
    t.src = -1; t.dst = dst; t.s1 = t.s2 = 0; t.out = out;
    const int tot = e + mi;
    std::vector<int> cpos(tot, 0), node(tot), pmap(e);
    for (int r = 0; r < e; ++r) {
      int i, j; ring_node(b, r, i, j);
      node[r] = enc(i, j);
      pmap[r] = r;
    }
    int q = e;
    for (int j = b.y0 + 1; j < b.y1 - 1; ++j)
      for (int i = b.x0 + 1; i < b.x1 - 1; ++i) node[q++] = enc(i, j);
    P.ipool.insert(P.ipool.end(), cpos.begin(), cpos.end());
    P.ipool.insert(P.ipool.end(), node.begin(), node.end());
    P.ipool.insert(P.ipool.end(), pmap.begin(), pmap.end());
    stamp(t);
    return t;
  }

  // Pairwise merge of child c1 (west or south) and c2 (east or north), Section 3.2.
  bool merge_task(const Rect& c1, int src, long long s1, const Rect& c2, long long s2,
                  int dst, long long out, SchurTask& t, std::string& err) {
    Rect u{std::min(c1.x0, c2.x0), std::max(c1.x1, c2.x1), std::min(c1.y0, c2.y0), std::max(c1.y1, c2.y1)};
    const int m1 = c1.ring(), m2 = c2.ring();
    std::vector<int> p1, p3, p2, p4;   // child ring positions
    for (int r = 0; r < m1; ++r) {
      int i, j; ring_node(c1, r, i, j);
      (interior_to(u, n, i, j) ? p3 : p1).push_back(r);
    }
    for (int r = 0; r < m2; ++r) {
      int i, j; ring_node(c2, r, i, j);
      (interior_to(u, n, i, j) ? p4 : p2).push_back(r);
    }
    t = SchurTask{};
    t.kind = 1;
    t.e1 = (int)p1.size(); t.i1 = (int)p3.size();
    t.e = t.e1 + (int)p2.size(); t.i = t.i1 + (int)p4.size();
    t.m1 = m1; t.m2 = m2;
    t.src = src; t.dst = dst; t.s1 = s1; t.s2 = s2; t.out = out;
    t.idx = (int)P.ipool.size();
    if (t.e != u.ring()) { err = "merge exterior does not match the union ring"; return false; }
    const int tot = t.e + t.i;
    std::vector<int> cpos(tot), node(tot), pmap(t.e);
    auto fill = [&](int at, const std::vector<int>& pos, const Rect& c) {
      for (size_t k = 0; k < pos.size(); ++k) {
        int i, j; ring_node(c, pos[k], i, j);
        cpos[at + (int)k] = pos[k];
        node[at + (int)k] = enc(i, j);
      }
    };
    fill(0, p1, c1);
    fill(t.e1, p2, c2);
    fill(t.e, p3, c1);
    fill(t.e + t.i1, p4, c2);
    for (int a = 0; a < t.e; ++a) {
      const int p = node[a];
      pmap[a] = ring_pos(u, enc_i(p), enc_j(p));
      if (pmap[a] < 0) { err = "exterior node not on the union ring"; return false; }
    }
    // Five-point structure: P3 never touches P2 and P4 never touches P1, so the
    // coupling blocks A32, A41 (and A14, A23) vanish and both K_ie and K_ei are
    // block diagonal (the remark after the merge formula in Section 3.2).
    for (int a = t.e; a < t.e + t.i1; ++a)
      for (int b = t.e1; b < t.e; ++b)
        if (adjacent(n, node[a], node[b])) { err = "unexpected P3-P2 coupling"; return false; }
    for (int a = t.e + t.i1; a < tot; ++a)
      for (int b = 0; b < t.e1; ++b)
        if (adjacent(n, node[a], node[b])) { err = "unexpected P4-P1 coupling"; return false; }
    P.ipool.insert(P.ipool.end(), cpos.begin(), cpos.end());
    P.ipool.insert(P.ipool.end(), node.begin(), node.end());
    P.ipool.insert(P.ipool.end(), pmap.begin(), pmap.end());
    stamp(t);
    return true;
  }

  bool is_small(const SchurTask& t) const {
    if (P.fast)
      return t.i <= kFastMaxI && t.e <= kFastMaxCols && t.i + t.e <= kFastMaxCols &&
             ((size_t)t.i * t.e + 64) * 8 <= (size_t)kSmallFastLds;
    return t.i <= kSmallImax && (size_t)t.i * (t.i + t.e) * 8 <= kSmallLdsMax;
  }

  // For a merge whose block inversion splits K_ii first at the children's interface (h1 = i1), the
  // off-diagonal blocks A12 = A34 and A21 = A43 couple the two interface lines through the five-point
  // stencil (Section 3): match[c] is the first child's interior node coupled to the second child's
  // interior node c (or -1).  False when some node couples to more than one (then dense products).
  bool coupling_match(const SchurTask& t, std::vector<int>& match) const {
    const int e = t.e, i = t.i, i1 = t.i1, i2 = i - i1;
    const int* node = P.ipool.data() + t.idx + e + i;
    std::unordered_map<int, int> first;
    for (int r = 0; r < i1; ++r) first[node[e + r]] = r;
    std::vector<char> used(i1, 0);
    match.assign(i2, -1);
    for (int c = 0; c < i2; ++c) {
      const int q = node[e + i1 + c], qi = q & 0xFFFF, qj = q >> 16;
      const int nb[4][2] = {{qi - 1, qj}, {qi + 1, qj}, {qi, qj - 1}, {qi, qj + 1}};
      int hit = -1, cnt = 0;
      for (const auto& d : nb) {
        if (d[0] < 0 || d[1] < 0) continue;
        const auto it = first.find((d[1] << 16) | d[0]);
        if (it != first.end()) { hit = it->second; ++cnt; }
      }
      if (cnt > 1) return false;
      if (hit >= 0) {
        if (used[hit]) return false;
        used[hit] = 1;
        match[c] = hit;
      }
    }
    return true;
  }

  // Recursive 2x2 block inversion of every merge's K_ii (at m.inv, leading dimension i),
  // batched over the phase's merges; rng[q] is merge q's index range at this node:
  //   X11 = inv(A11); Wb = X11 A12; Wc = A21 X11; A22 <- A22 - A21 Wb; X22 = inv(A22);
  //   X12 = -Wb X22; X21 = -X22 Wc; X11 <- X11 - X12 Wc.
  void rbi(Phase& ph, int depth, int D, const std::vector<std::pair<int, int>>& rng,
           const std::vector<std::vector<long long>>& wb, const std::vector<std::vector<long long>>& wc) {
    const int nlm = ph.large_count;
    if (depth == D) {
      InvOp op;
      op.base_first = (int)P.bases.size();
      for (int q = 0; q < nlm; ++q) {
        const LargeMerge& m = P.large[ph.large_first + q];
        const int lo = rng[q].first, hi = rng[q].second;
        if (hi <= lo) continue;
        BaseBlock b{};
        b.off = m.inv + lo + (long long)lo * m.t.i;
        b.scale = m.scale;
        b.ld = m.t.i;
        b.bs = hi - lo;
        P.bases.push_back(b);
      }
      op.base_count = (int)P.bases.size() - op.base_first;
      if (op.base_count > 0) ph.inv_ops.push_back(op);
      return;
    }
    std::vector<std::pair<int, int>> left(nlm), right(nlm);
    for (int q = 0; q < nlm; ++q) {
      const int lo = rng[q].first, hi = rng[q].second, mid = lo + (hi - lo + 1) / 2;
      left[q] = {lo, mid};
      right[q] = {mid, hi};
    }
    rbi(ph, depth + 1, D, left, wb, wc);
    auto A = [](const LargeMerge& m, int r, int c) { return m.inv + r + (long long)c * m.t.i; };
    struct Sz { int i, lo, mid, hi, h1, h2; };
    auto sz = [&](int q) {
      const LargeMerge& m = P.large[ph.large_first + q];
      Sz s{m.t.i, left[q].first, left[q].second, right[q].second, 0, 0};
      s.h1 = s.mid - s.lo;
      s.h2 = s.hi - s.mid;
      return s;
    };
    InvOp s1, s2, s3, s4;
    // top split at the children's interface: Wb, Wc and A22 - A21 Wb are copies and scalings of X11
    // entries (one coupled pair per row and column of A12), done by one elementwise launch
    std::vector<char> cpl(nlm, 0);
    if (depth == 0) {
      InvOp c;
      c.couple_first = (int)P.couples.size();
      std::vector<int> match;
      for (int q = 0; q < nlm; ++q) {
        const LargeMerge& m = P.large[ph.large_first + q];
        const Sz s = sz(q);
        if (s.h1 <= 0 || s.h2 <= 0 || s.h1 != m.t.i1 || !coupling_match(m.t, match)) continue;
        cpl[q] = 1;
        CoupleDesc d{};
        d.inv = m.inv;
        d.wb = wb[q][0];
        d.wc = wc[q][0];
        d.i = s.i; d.h1 = s.h1; d.h2 = s.h2;
        d.match = (int)P.ipool.size();
        P.ipool.insert(P.ipool.end(), match.begin(), match.end());
        P.couples.push_back(d);
      }
      c.couple_count = (int)P.couples.size() - c.couple_first;
      if (c.couple_count > 0) ph.inv_ops.push_back(c);
    }
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < nlm; ++q) {
        const LargeMerge& m = P.large[ph.large_first + q];
        const Sz s = sz(q);
        if (s.h1 <= 0 || s.h2 <= 0 || cpl[q]) continue;
        if (pass == 0)   // Wb = X11 A12
          push(s1.gemm, gd(s.h1, s.h2, s.h1, BUF_WS, A(m, s.lo, s.lo), s.i, BUF_WS, A(m, s.lo, s.mid), s.i,
                           BUF_WS, wb[q][depth], s.h1, 1.0, 0.0, -1, -1, -1));
        else             // Wc = A21 X11
          push(s1.gemm, gd(s.h2, s.h1, s.h1, BUF_WS, A(m, s.mid, s.lo), s.i, BUF_WS, A(m, s.lo, s.lo), s.i,
                           BUF_WS, wc[q][depth], s.h2, 1.0, 0.0, -1, -1, -1));
      }
    ph.inv_ops.push_back(s1);
    for (int q = 0; q < nlm; ++q) {     // A22 <- A22 - A21 Wb
      const LargeMerge& m = P.large[ph.large_first + q];
      const Sz s = sz(q);
      if (s.h1 <= 0 || s.h2 <= 0 || cpl[q]) continue;
      push(s2.gemm, gd(s.h2, s.h2, s.h1, BUF_WS, A(m, s.mid, s.lo), s.i, BUF_WS, wb[q][depth], s.h1,
                       BUF_WS, A(m, s.mid, s.mid), s.i, -1.0, 1.0, -1, -1, -1));
    }
    ph.inv_ops.push_back(s2);
    rbi(ph, depth + 1, D, right, wb, wc);
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < nlm; ++q) {
        const LargeMerge& m = P.large[ph.large_first + q];
        const Sz s = sz(q);
        if (s.h1 <= 0 || s.h2 <= 0) continue;
        if (pass == 0)   // X12 = -Wb X22
          push(s3.gemm, gd(s.h1, s.h2, s.h2, BUF_WS, wb[q][depth], s.h1, BUF_WS, A(m, s.mid, s.mid), s.i,
                           BUF_WS, A(m, s.lo, s.mid), s.i, -1.0, 0.0, -1, -1, -1));
        else             // X21 = -X22 Wc
          push(s3.gemm, gd(s.h2, s.h1, s.h2, BUF_WS, A(m, s.mid, s.mid), s.i, BUF_WS, wc[q][depth], s.h2,
                           BUF_WS, A(m, s.mid, s.lo), s.i, -1.0, 0.0, -1, -1, -1));
      }
    ph.inv_ops.push_back(s3);
    for (int q = 0; q < nlm; ++q) {     // X11 <- X11 - X12 Wc
      const LargeMerge& m = P.large[ph.large_first + q];
      const Sz s = sz(q);
      if (s.h1 <= 0 || s.h2 <= 0) continue;
      push(s4.gemm, gd(s.h1, s.h1, s.h2, BUF_WS, A(m, s.lo, s.mid), s.i, BUF_WS, wc[q][depth], s.h2,
                       BUF_WS, A(m, s.lo, s.lo), s.i, -1.0, 1.0, -1, -1, -1));
    }
    ph.inv_ops.push_back(s4);
  }

  void finish_fast_large(Phase& ph, std::vector<SchurTask>& large, int limax, bool comp) {
    int D = 0;
    while (ceil_div(limax, 1 << D) > kBaseBlock) ++D;
    long long ws = 0;
    std::vector<std::vector<long long>> wb, wc;
    for (auto& t : large) {
      LargeMerge m{};
      m.t = t;
      m.W = 0;
      m.piv = -1;
      const long long e = t.e, i = t.i, e1 = t.e1, i1 = t.i1, e2 = t.e - t.e1, i2 = t.i - t.i1;
      m.inv = ws; ws += i * i;
      std::vector<long long> b(D), c(D);
      long long n_ = i;
      for (int d = 0; d < D; ++d) {
        const long long h1 = (n_ + 1) / 2, h2 = n_ - h1;
        b[d] = ws; ws += h1 * h2;
        c[d] = ws; ws += h2 * h1;
        n_ = h1;   // the larger half bounds every node of the next depth
      }
      wb.push_back(b);
      wc.push_back(c);
      m.q = m.r = -1;
      m.b31 = ws; ws += i1 * e1;
      m.b42 = ws; ws += i2 * e2;
      m.a13 = ws; ws += e1 * i1;
      m.a24 = ws; ws += e2 * i2;
      m.x = -1;
      if (!comp) { m.x = ws; ws += i * e; }
      m.scale = ws; ws += 1;
      ws = (ws + 31) & ~31LL;
      if (comp) {
        CompMerge cm;
        const long long mrow[4] = {i1, i2, e1, e2}, ncol[4] = {e1, e2, i1, i2};
        const long long asrc[4] = {m.b31, m.b42, m.a13, m.a24};
        for (int b = 0; b < 4; ++b) {
          CompBlock& B = cm.blk[b];
          B.A = asrc[b]; B.m = (int)mrow[b]; B.n = (int)ncol[b];
          B.qb = ws; ws += mrow[b] * kCompCols;
          B.yb = ws; ws += mrow[b] * kCompPass1;
          B.bmat = ws; ws += (long long)kCompCols * ncol[b];
          B.g = ws; ws += kCompPass1 * kCompPass1;
          B.mm = ws; ws += kCompPass1 * kCompPass1;
          B.h = ws; ws += kCompPass1 * kCompPass2;
          B.dmax = ws; ws += 1;
          ws = (ws + 31) & ~31LL;
          P.aux_rows = std::max(P.aux_rows, B.n);
        }
        cm.w1 = ws; ws += i * kCompCols;
        cm.w2 = ws; ws += i * kCompCols;
        for (int c = 0; c < 4; ++c) { cm.c[c] = ws; ws += (long long)kCompCols * kCompCols; }
        cm.d1 = ws; ws += (long long)kCompCols * e;
        cm.d2 = ws; ws += (long long)kCompCols * e;
        ws = (ws + 31) & ~31LL;
        comp_merges.push_back(cm);
      }
      P.large.push_back(m);
    }
    P.ws_doubles = std::max(P.ws_doubles, (size_t)ws);
    ph.ws_end = ws;
    ph.large_count = (int)large.size();
    for (auto& t : large) {
      const double e = t.e, i = t.i;
      ph.gather_bytes += 8.0 * 2.0 * (i * i + 2.0 * i * e + e * e);
    }
    std::vector<std::pair<int, int>> rng;
    for (auto& t : large) rng.push_back({0, t.i});
    rbi(ph, 0, D, rng, wb, wc);
    if (comp) {
      ph.compressed = true;
      push_compressed(ph);
      comp_merges.clear();
    } else {
      push_products(ph, false);
    }
  }

  // ------------------------------------------------------------------------------------------
  // Compressed merge (Section 6, Step 2).  Each off-diagonal block A (S31, S42 of K_ie; S13,
  // S24 of K_ei; m x n) is factored A ~= Q B with Q (m x kCompCols) orthonormal and B = Q^T A:
  //   pass 1: Y = A W1 (Gaussian W1, kCompPass1 columns), G = Y^T Y, pivoted Cholesky truncated
  //           at max(tol, 1e-7) relative -> Q1 = Y M, re-orthogonalised by a second Cholesky QR;
  //   pass 2: Y = A W2 with Q1 projected out twice, truncated at tol -> Q2, re-orthogonalised.
  // Columns of Q past the rank are exactly zero, so every product below has a fixed shape.
  // Then X = K_ii^{-1} K_ie is never formed:
  //   W1 = K_ii^{-1}[:, P3] Q31, W2 = K_ii^{-1}[:, P4] Q42,
  //   S[P1, :] -= Q13 [(B13 W1[P3]) B31 | (B13 W2[P3]) B42],
  //   S[P2, :] -= Q24 [(B24 W1[P4]) B31 | (B24 W2[P4]) B42].
  // ------------------------------------------------------------------------------------------
  struct CompBlock { long long A = 0, qb = 0, yb = 0, bmat = 0, g = 0, mm = 0, h = 0, dmax = 0; int m = 0, n = 0; };
  struct CompMerge { CompBlock blk[4]; long long w1 = 0, w2 = 0, c[4] = {0, 0, 0, 0}, d1 = 0, d2 = 0; };
  std::vector<CompMerge> comp_merges;
  std::vector<int> omega_descs;   // descriptors reading the Gaussian matrix: offB holds its column

  template <class F> void comp_gemm(Phase& ph, F fill) {
    CompOp op;
    for (size_t q = 0; q < comp_merges.size(); ++q) fill(op.gemm, comp_merges[q], P.large[ph.large_first + q]);
    if (op.gemm.count > 0) ph.comp_ops.push_back(op);
  }
  void comp_pchol(Phase& ph, int k, int mode, int pass_slot) {
    CompOp op;
    op.pchol_first = (int)P.pchols.size();
    for (size_t q = 0; q < comp_merges.size(); ++q)
      for (int b = 0; b < 4; ++b) {
        const CompBlock& B = comp_merges[q].blk[b];
        PcholDesc d{};
        d.g = B.g; d.m = B.mm; d.dmax = B.dmax; d.k = k; d.mode = mode; d.tol = P.tol;
        d.rank = (int)P.int_ws++;
        if (pass_slot >= 0) {
          if (pass_slot == 0) {
            RankSlot rs;
            rs.level = ph.level;
            rs.first = d.rank;
            P.rank_slots.push_back(rs);
          } else {
            P.rank_slots[P.rank_slots.size() - comp_merges.size() * 4 + q * 4 + b].second = d.rank;
          }
        }
        P.pchols.push_back(d);
      }
    op.pchol_count = (int)P.pchols.size() - op.pchol_first;
    ph.comp_ops.push_back(op);
  }

  void push_compressed(Phase& ph) {
    const int K1 = kCompPass1, K2 = kCompPass2, KC = kCompCols;
    // pass 1
    comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge&) {
      for (const CompBlock& B : cm.blk) {
        const size_t at = P.gemms.size();
        push(L, gd(B.m, K1, B.n, BUF_WS, B.A, B.m, BUF_AUX, 0, 0, BUF_WS, B.yb, B.m, 1.0, 0.0, -1, -1, -1));
        if (P.gemms.size() > at) omega_descs.push_back((int)at);
      }
    });
    auto gram = [&](int k) {
      comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge&) {
        for (const CompBlock& B : cm.blk) {
          GemmDesc g = gd(k, k, B.m, BUF_WS, B.yb, B.m, BUF_WS, B.yb, B.m, BUF_WS, B.g, k, 1.0, 0.0, -1, -1, -1);
          g.transA = 1;
          push(L, g);
        }
      });
    };
    auto gram_q = [&](int k, int col0) {
      comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge&) {
        for (const CompBlock& B : cm.blk) {
          const long long q = B.qb + (long long)col0 * B.m;
          GemmDesc g = gd(k, k, B.m, BUF_WS, q, B.m, BUF_WS, q, B.m, BUF_WS, B.g, k, 1.0, 0.0, -1, -1, -1);
          g.transA = 1;
          push(L, g);
        }
      });
    };
    // C = (Y or Q columns) * M into (Q columns or Y)
    auto apply_m = [&](int k, bool from_y, int col0) {
      comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge&) {
        for (const CompBlock& B : cm.blk) {
          const long long q = B.qb + (long long)col0 * B.m;
          push(L, gd(B.m, k, k, BUF_WS, from_y ? B.yb : q, B.m, BUF_WS, B.mm, k, BUF_WS, from_y ? q : B.yb, B.m,
                     1.0, 0.0, -1, -1, -1));
        }
      });
    };
    auto copy_y_to_q = [&](int k, int col0) {
      comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge&) {
        for (const CompBlock& B : cm.blk)
          push(L, gd(B.m, k, k, BUF_WS, B.yb, B.m, BUF_AUX, 0, kCompCols, BUF_WS, B.qb + (long long)col0 * B.m, B.m,
                     1.0, 0.0, -1, -1, -1));   // times the identity at the start of BUF_AUX
      });
    };
    gram(K1);
    comp_pchol(ph, K1, 0, 0);
    apply_m(K1, true, 0);        // Q1 = Y M
    gram_q(K1, 0);
    comp_pchol(ph, K1, 2, -1);
    apply_m(K1, false, 0);       // Y = Q1 M'
    copy_y_to_q(K1, 0);          // Q1 = Y
    // pass 2: sketch of the residual
    comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge&) {
      for (const CompBlock& B : cm.blk) {
        const size_t at = P.gemms.size();
        push(L, gd(B.m, K2, B.n, BUF_WS, B.A, B.m, BUF_AUX, K1, 0, BUF_WS, B.yb, B.m, 1.0, 0.0, -1, -1, -1));
        if (P.gemms.size() > at) omega_descs.push_back((int)at);
      }
    });
    for (int rep = 0; rep < 2; ++rep) {
      comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge&) {   // H = Q1^T Y
        for (const CompBlock& B : cm.blk) {
          GemmDesc g = gd(K1, K2, B.m, BUF_WS, B.qb, B.m, BUF_WS, B.yb, B.m, BUF_WS, B.h, K1, 1.0, 0.0, -1, -1, -1);
          g.transA = 1;
          push(L, g);
        }
      });
      comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge&) {   // Y -= Q1 H
        for (const CompBlock& B : cm.blk)
          push(L, gd(B.m, K2, K1, BUF_WS, B.qb, B.m, BUF_WS, B.h, K1, BUF_WS, B.yb, B.m, -1.0, 1.0, -1, -1, -1));
      });
    }
    gram(K2);
    comp_pchol(ph, K2, 1, 1);
    apply_m(K2, true, K1);       // Q2 = Y M
    gram_q(K2, K1);
    comp_pchol(ph, K2, 2, -1);
    apply_m(K2, false, K1);      // Y = Q2 M'
    copy_y_to_q(K2, K1);         // Q2 = Y
    // B = Q^T A
    comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge&) {
      for (const CompBlock& B : cm.blk) {
        GemmDesc g = gd(KC, B.n, B.m, BUF_WS, B.qb, B.m, BUF_WS, B.A, B.m, BUF_WS, B.bmat, KC, 1.0, 0.0, -1, -1, -1);
        g.transA = 1;
        push(L, g);
      }
    });
    // W1 = inv[:, P3] Q31, W2 = inv[:, P4] Q42
    comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge& m) {
      const int i = m.t.i, i1 = m.t.i1, i2 = i - i1;
      push(L, gd(i, KC, i1, BUF_WS, m.inv, i, BUF_WS, cm.blk[0].qb, i1, BUF_WS, cm.w1, i, 1.0, 0.0, -1, -1, -1));
      push(L, gd(i, KC, i2, BUF_WS, m.inv + (long long)i1 * i, i, BUF_WS, cm.blk[1].qb, i2, BUF_WS, cm.w2, i,
                 1.0, 0.0, -1, -1, -1));
    });
    // C11 = B13 W1[P3], C12 = B13 W2[P3], C21 = B24 W1[P4], C22 = B24 W2[P4]
    comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge& m) {
      const int i = m.t.i, i1 = m.t.i1, i2 = i - i1;
      push(L, gd(KC, KC, i1, BUF_WS, cm.blk[2].bmat, KC, BUF_WS, cm.w1, i, BUF_WS, cm.c[0], KC, 1.0, 0.0, -1, -1, -1));
      push(L, gd(KC, KC, i1, BUF_WS, cm.blk[2].bmat, KC, BUF_WS, cm.w2, i, BUF_WS, cm.c[1], KC, 1.0, 0.0, -1, -1, -1));
      push(L, gd(KC, KC, i2, BUF_WS, cm.blk[3].bmat, KC, BUF_WS, cm.w1 + i1, i, BUF_WS, cm.c[2], KC, 1.0, 0.0, -1, -1, -1));
      push(L, gd(KC, KC, i2, BUF_WS, cm.blk[3].bmat, KC, BUF_WS, cm.w2 + i1, i, BUF_WS, cm.c[3], KC, 1.0, 0.0, -1, -1, -1));
    });
    // D1 = [C11 B31 | C12 B42], D2 = [C21 B31 | C22 B42]
    comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge& m) {
      const int e = m.t.e, e1 = m.t.e1, e2 = e - e1;
      push(L, gd(KC, e1, KC, BUF_WS, cm.c[0], KC, BUF_WS, cm.blk[0].bmat, KC, BUF_WS, cm.d1, KC, 1.0, 0.0, -1, -1, -1));
      push(L, gd(KC, e2, KC, BUF_WS, cm.c[1], KC, BUF_WS, cm.blk[1].bmat, KC, BUF_WS, cm.d1 + (long long)e1 * KC, KC,
                 1.0, 0.0, -1, -1, -1));
      push(L, gd(KC, e1, KC, BUF_WS, cm.c[2], KC, BUF_WS, cm.blk[0].bmat, KC, BUF_WS, cm.d2, KC, 1.0, 0.0, -1, -1, -1));
      push(L, gd(KC, e2, KC, BUF_WS, cm.c[3], KC, BUF_WS, cm.blk[1].bmat, KC, BUF_WS, cm.d2 + (long long)e1 * KC, KC,
                 1.0, 0.0, -1, -1, -1));
    });
    // S[P1, :] -= Q13 D1, S[P2, :] -= Q24 D2 (scattered into the parent's ring order)
    comp_gemm(ph, [&](LaunchGemm& L, const CompMerge& cm, const LargeMerge& m) {
      const int e = m.t.e, i = m.t.i, e1 = m.t.e1, e2 = e - e1;
      const int pm = m.t.idx + 2 * (e + i);
      push(L, gd(e1, e, KC, BUF_WS, cm.blk[2].qb, e1, BUF_WS, cm.d1, KC, m.t.dst, m.t.out, e, -1.0, 1.0, pm, pm, -1));
      push(L, gd(e2, e, KC, BUF_WS, cm.blk[3].qb, e2, BUF_WS, cm.d2, KC, m.t.dst, m.t.out, e, -1.0, 1.0, pm + e1, pm,
                 -1));
    });
  }

  // X = K_ii^{-1} diag(S31, S42) and S[pmap, pmap] -= diag(S13, S24) X.  Each launch's
  // descriptors must be contiguous, so the two products are listed in separate passes.
  // with_kmap: the inverse is stored row-permuted (pivoted path) and read through a column map.
  void push_products(Phase& ph, bool with_kmap) {
    for (int q = 0; q < ph.large_count; ++q) {
      const LargeMerge& m = P.large[ph.large_first + q];
      const int e = m.t.e, i = m.t.i, e1 = m.t.e1, i1 = m.t.i1, e2 = e - e1, i2 = i - i1;
      const int kmap = with_kmap ? m.piv + i : -1;
      if (i1 > 0) push(ph.xgemm, gd(i, e1, i1, BUF_WS, m.inv, i, BUF_WS, m.b31, i1,
                                    BUF_WS, m.x, i, 1.0, 0.0, -1, -1, kmap));
      if (i2 > 0) push(ph.xgemm, gd(i, e2, i2, BUF_WS, with_kmap ? m.inv : m.inv + (long long)i1 * i, i,
                                    BUF_WS, m.b42, i2, BUF_WS, m.x + (long long)e1 * i, i, 1.0, 0.0, -1, -1,
                                    with_kmap ? kmap + i1 : -1));
    }
    std::vector<GemmDesc> tri;   // the symmetric merges' diagonal blocks: their own launch, after the loop
    // The off-diagonal blocks of symmetric merges join that launch when on their own they would run on
    // 64 x 64 tiles too: one launch fills the CUs' last round of tiles once instead of twice.
    int d2_big = 0, d2_t64 = 0;
    bool d2_wide = true;
    for (int q = 0; q < ph.large_count; ++q) {
      const LargeMerge& m = P.large[ph.large_first + q];
      const int e1 = m.t.e1, e2 = m.t.e - e1, i1 = m.t.i1, i2 = m.t.i - i1;
      if (with_kmap || !m.t.sym || i1 <= 0 || i2 <= 0) continue;
      d2_big += ceil_div(e2, 128) * ceil_div(e1, 128);
      d2_t64 += ceil_div(e2, 64) * ceil_div(e1, 64);
      d2_wide = d2_wide && e1 >= 128 && e2 >= 128;
    }
    const bool d2_joins = P.mixed == 0 && !(d2_wide && d2_big >= kBigTileMin) && d2_t64 >= kSmallTileBelow;
    for (int q = 0; q < ph.large_count; ++q) {
      const LargeMerge& m = P.large[ph.large_first + q];
      const int e = m.t.e, i = m.t.i, e1 = m.t.e1, i1 = m.t.i1, e2 = e - e1, i2 = i - i1;
      const int pm = m.t.idx + 2 * (e + i);
      // the dense path forms K_ee in these products' epilogue (the gather leaves it out); both
      // blocks of rows are pushed so that every entry of the parent's S is written
      const bool kee = !with_kmap && i1 > 0 && i2 > 0;
      P.large[ph.large_first + q].kee_gemm = kee ? 1 : 0;
      GemmDesc g1 = gd(e1, e, i1, BUF_WS, m.a13, e1, BUF_WS, m.x, i, m.t.dst, m.t.out, e, -1.0, 1.0, pm, pm, -1);
      GemmDesc g2 = gd(e2, e, i2, BUF_WS, m.a24, e2, BUF_WS, m.x + i1, i, m.t.dst, m.t.out, e, -1.0, 1.0,
                       pm + e1, pm, -1);
      if (kee && m.t.sym) {
        // symmetric S: the child-1 diagonal block (lower tiles), the child-2 x child-1 block and the
        // child-2 diagonal block (lower tiles), each entry also written at its mirror position
        // (S13 = S31^T and S24 = S42^T: the products read S31 and S42 transposed, the gather skips S13, S24)
        GemmDesc d1 = gd(e1, e1, i1, BUF_WS, m.b31, i1, BUF_WS, m.x, i, m.t.dst, m.t.out, e, -1.0, 1.0, pm, pm, -1);
        GemmDesc d2 = gd(e2, e1, i2, BUF_WS, m.b42, i2, BUF_WS, m.x + i1, i, m.t.dst, m.t.out, e, -1.0, 1.0,
                         pm + e1, pm, -1);
        GemmDesc d3 = gd(e2, e2, i2, BUF_WS, m.b42, i2, BUF_WS, m.x + i1 + (long long)e1 * i, i, m.t.dst, m.t.out,
                         e, -1.0, 1.0, pm + e1, pm + e1, -1);
        d1.transA = d2.transA = d3.transA = 1;
        P.large[ph.large_first + q].kee_gemm = 2;
        d1.kee = d2.kee = d3.kee = ph.large_first + q + 1;
        d1.kee_row0 = 0;  d1.kee_col0 = 0;
        d2.kee_row0 = e1; d2.kee_col0 = 0;
        d3.kee_row0 = e1; d3.kee_col0 = e1;
        d1.tri = d3.tri = 1;
        d1.mirror = d2.mirror = d3.mirror = 1;
        tri.push_back(d1);
        if (d2_joins) tri.push_back(d2);
        else push(ph.sgemm, d2);
        tri.push_back(d3);
        continue;
      }
      if (kee) {
        g1.kee = g2.kee = ph.large_first + q + 1;
        g1.kee_row0 = 0;
        g2.kee_row0 = e1;
      }
      if (i1 > 0) push(ph.sgemm, g1);
      if (i2 > 0) push(ph.sgemm, g2);
    }
    for (const GemmDesc& g : tri) push(ph.sgemm_tri, g);
  }

  // Distribute the tasks of one phase over the small and large paths.
  void finish_phase(Phase& ph, std::vector<SchurTask>& tasks, const std::vector<TaskTag>& tags) {
    split_phase(ph, tasks, tags);
    finalize_phase(ph);
  }

  void split_phase(Phase& ph, std::vector<SchurTask>& tasks, const std::vector<TaskTag>& tags) {
    ph.small_first = (int)P.tasks.size();
    ph.large_first = (int)P.large.size();
    std::vector<SchurTask> large;
    for (size_t tq = 0; tq < tasks.size(); ++tq) {
      const SchurTask& t = tasks[tq];
      (is_small(t) ? P.task_tags : P.large_tags).push_back(tags[tq]);
      ph.imax = std::max(ph.imax, t.i);
      ph.emax = std::max(ph.emax, t.e);
      if (t.kind == 1) {
        const double e = t.e, i = t.i;
        ph.model_flops += 2.0 / 3.0 * i * i * i + 2.0 * i * i * e + e * e * i;
      }
      if (is_small(t)) {
        const double e = t.e, i = t.i;
        ph.small_flops += 2.0 / 3.0 * i * i * i + 2.0 * i * i * e + e * e * i;
        ph.small_bytes += 8.0 * ((i + e) * (i + e) + e * e);
        P.tasks.push_back(t);
        if (!P.fast) ph.small_lds = std::max(ph.small_lds, (size_t)t.i * (t.i + t.e) * 8);
      } else {
        large.push_back(t);
      }
    }
    ph.small_count = (int)P.tasks.size() - ph.small_first;
    for (int q = ph.small_first; q < (int)P.tasks.size(); ++q) {
      ph.small_threads = std::max(ph.small_threads, P.tasks[q].i + P.tasks[q].e);   // columns of [K_ii | K_ie]
      if (P.fast) {
        ph.small_lds = std::max(ph.small_lds, ((size_t)P.tasks[q].i * P.tasks[q].e + 64) * 8);
        ph.small_imax = std::max(ph.small_imax, P.tasks[q].i);
      }
    }
    if (large.empty()) return;
    int limax = 0;
    for (auto& t : large) limax = std::max(limax, t.i);
    if (P.fast) {
      bool comp = P.tol > 0.0;
      if (comp) {
        if (P.hbs_level >= 0) {
          comp = ph.min_level <= P.hbs_level;
        } else {
          for (auto& t : large) comp = comp && std::min(t.m1, t.m2) >= kCompMinChild;
        }
      }
      finish_fast_large(ph, large, limax, comp);
      return;
    }
    if (limax <= 256)       { ph.gje_nt = 256;  ph.gje_r = 1; ph.gje_w = 32; }
    else if (limax <= 1024) { ph.gje_nt = 512;  ph.gje_r = 2; ph.gje_w = 32; }
    else if (limax <= 2048) { ph.gje_nt = 1024; ph.gje_r = 2; ph.gje_w = 16; }
    else if (limax <= 4096) { ph.gje_nt = 1024; ph.gje_r = 4; ph.gje_w = 8; }
    else                    { ph.gje_nt = 1024; ph.gje_r = 8; ph.gje_w = 4; }
    const int W = ph.gje_w;
    long long ws = 0;
    size_t iws = 0;                // int scratch, relative; relocated after the constant pool
    size_t iws0 = iws;
    for (auto& t : large) {
      LargeMerge m{};
      m.t = t;
      m.W = W;
      const long long e = t.e, i = t.i, e1 = t.e1, i1 = t.i1, e2 = t.e - t.e1, i2 = t.i - t.i1;
      m.inv = ws; ws += i * i;
      m.q = ws; ws += i * W;
      m.r = ws; ws += (long long)W * i;
      m.b31 = ws; ws += i1 * e1;
      m.b42 = ws; ws += i2 * e2;
      m.a13 = ws; ws += e1 * i1;
      m.a24 = ws; ws += e2 * i2;
      m.x = ws; ws += i * e;
      m.scale = ws; ws += 1;
      ws = (ws + 31) & ~31LL;   // 256-byte alignment of every merge's scratch
      m.piv = (int)iws; iws += 2 * (size_t)i;
      P.large.push_back(m);
    }
    P.ws_doubles = std::max(P.ws_doubles, (size_t)ws);
    P.int_ws = std::max(P.int_ws, iws - iws0);
    ph.large_count = (int)large.size();
    for (auto& t : large) {
      const double e = t.e, i = t.i;
      ph.gather_bytes += 8.0 * 2.0 * (i * i + 2.0 * i * e + e * e);
    }
    // Gauss-Jordan update products, one launch per block step.
    const int steps = ceil_div(limax, W);
    ph.gje_update.resize(steps);
    for (int k = 0; k < steps; ++k) {
      const int c0 = k * W;
      for (int q = 0; q < ph.large_count; ++q) {
        const LargeMerge& m = P.large[ph.large_first + q];
        const int i = m.t.i;
        if (c0 >= i) continue;
        const int Wk = std::min(W, i - c0);
        // A[:, cols] -= Q' R[:, cols] for the columns left and right of the block
        push(ph.gje_update[k], gd(i, c0, Wk, BUF_WS, m.q, i, BUF_WS, m.r, W,
                                  BUF_WS, m.inv, i, -1.0, 1.0, -1, -1, -1));
        const int c1 = c0 + Wk;
        push(ph.gje_update[k], gd(i, i - c1, Wk, BUF_WS, m.q, i, BUF_WS, m.r + (long long)c1 * W, W,
                                  BUF_WS, m.inv + (long long)c1 * i, i, -1.0, 1.0, -1, -1, -1));
      }
    }
    push_products(ph, true);
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// Autotuner table
// ---------------------------------------------------------------------------
namespace {
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
int g_tune_gen = 0;
bool g_tune_on = true;
}  // namespace

void tune_put(const std::string& sig, int cfg) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[sig] = cfg;
  ++g_tune_gen;
}

bool tune_get(const std::string& sig, int& cfg) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(sig);
  if (it == g_tune.end()) return false;
  cfg = it->second;
  return true;
}

void tune_clear() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.clear();
  ++g_tune_gen;
}

int tune_generation() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_tune_gen * 2 + (g_tune_on ? 1 : 0);
}

void tune_enable(bool on) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  if (g_tune_on != on) ++g_tune_gen;
  g_tune_on = on;
}

bool tune_enabled() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_tune_on;
}

size_t tune_size() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_tune.size();
}

// {"arch": "gfx950", "tiles": {"<signature>": <cfg>, ...}}
std::string tune_json(const std::string& arch) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  std::ostringstream o;
  o << "{\"arch\": \"" << arch << "\", \"tiles\": {";
  bool first = true;
  for (const auto& kv : g_tune) {
    o << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
    first = false;
  }
  o << "}}\n";
  return o.str();
}

bool tune_load_json(const std::string& text, const std::string& arch, std::string& err) {
  // a flat reader for the format tune_json writes: quoted keys, integer values
  auto skip = [&](size_t& i) { while (i < text.size() && std::isspace((unsigned char)text[i])) ++i; };
  auto str = [&](size_t& i, std::string& out) {
    skip(i);
    if (i >= text.size() || text[i] != '"') return false;
    const size_t j = text.find('"', i + 1);
    if (j == std::string::npos) return false;
    out = text.substr(i + 1, j - i - 1);
    i = j + 1;
    return true;
  };
  auto expect = [&](size_t& i, char c) { skip(i); if (i < text.size() && text[i] == c) { ++i; return true; } return false; };
  size_t i = 0;
  std::string key, val;
  std::map<std::string, int> tiles;
  std::string got_arch;
  if (!expect(i, '{')) { err = "tune cache: expected an object"; return false; }
  for (;;) {
    if (expect(i, '}')) break;
    if (!str(i, key) || !expect(i, ':')) { err = "tune cache: expected a key"; return false; }
    if (key == "arch") {
      if (!str(i, got_arch)) { err = "tune cache: arch must be a string"; return false; }
    } else if (key == "tiles") {
      if (!expect(i, '{')) { err = "tune cache: tiles must be an object"; return false; }
      for (;;) {
        if (expect(i, '}')) break;
        std::string sig;
        if (!str(i, sig) || !expect(i, ':')) { err = "tune cache: bad tile entry"; return false; }
        skip(i);
        size_t j = i;
        while (j < text.size() && std::isdigit((unsigned char)text[j])) ++j;
        if (j == i) { err = "tune cache: tile must be an integer"; return false; }
        const int c = std::atoi(text.substr(i, j - i).c_str());
        if (c != 0 && c != 2 && c != 3 && c != 4) { err = "tune cache: unknown tile " + std::to_string(c); return false; }
        tiles[sig] = c;
        i = j;
        if (!expect(i, ',')) { if (expect(i, '}')) break; err = "tune cache: bad tiles object"; return false; }
      }
    } else {
      err = "tune cache: unknown key " + key;
      return false;
    }
    if (!expect(i, ',')) { if (expect(i, '}')) break; err = "tune cache: bad object"; return false; }
  }
  if (got_arch != arch) { err = "tune cache: written for " + got_arch + ", this device is " + arch; return false; }
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto& kv : tiles) g_tune[kv.first] = kv.second;
  ++g_tune_gen;
  return true;
}

bool plan_make(int n, int leaf, int conv, bool fast, Plan& P, std::string& err) {
  ProbSpec sp;
  sp.n = n; sp.leaf = leaf; sp.conv = conv;
  return plan_make_many({sp}, fast, P, err);
}

namespace {

// The quadtree of one problem and its buffer regions.
struct Tree {
  ProbPlan pp;
  std::vector<std::vector<Rect>> boxes;        // children of box q at level l: 4q..4q+3 (SW, SE, NW, NE)
  std::vector<std::vector<long long>> off;     // S offsets within the level buffer region
  long long lva_base = 0, lvb_base = 0, half_base = 0;
  size_t lva_need = 0, lvb_need = 0, half_need = 0;
  std::vector<Rect> halves;                    // results of the latest west+east phase
  std::vector<long long> hoff;
};

int merge_phases(const Tree& T) { return 1 + 2 * T.pp.Lr; }

}  // namespace

void quadtree_levels(int n, int Lr, std::vector<std::vector<Rect>>& boxes) {
  boxes.assign(Lr + 1, {});
  boxes[0].push_back(Rect{0, n, 0, n});
  for (int l = 0; l < Lr; ++l) {
    for (const Rect& b : boxes[l]) {
      const int xm = b.x0 + b.sx() / 2, ym = b.y0 + b.sy() / 2;
      boxes[l + 1].push_back(Rect{b.x0, xm, b.y0, ym});
      boxes[l + 1].push_back(Rect{xm, b.x1, b.y0, ym});
      boxes[l + 1].push_back(Rect{b.x0, xm, ym, b.y1});
      boxes[l + 1].push_back(Rect{xm, b.x1, ym, b.y1});
    }
  }
}

bool plan_make_many(const std::vector<ProbSpec>& specs, bool fast, Plan& P, std::string& err, bool mixed,
                    double tol, int hbs_level, int tune_force) {
  P = Plan{};
  P.tune_force = tune_force;
  P.fast = fast;
  P.mixed = mixed;
  P.tol = tol;
  P.hbs_level = hbs_level;
  if (specs.empty()) { err = "no problems"; return false; }
  Builder B(P);
  std::vector<Tree> trees(specs.size());
  size_t lva = 0, lvb = 0, half = 0, coef = 0;
  for (size_t p = 0; p < specs.size(); ++p) {
    const int n = specs[p].n, leaf = specs[p].leaf;
    if (n < 3) { err = "n must be >= 3"; return false; }
    if (leaf < 4) { err = "leaf must be >= 4"; return false; }
    if (n > 65536) { err = "n too large"; return false; }
    Tree& T = trees[p];
    ProbPlan& pp = T.pp;
    pp.n = n; pp.leaf = leaf; pp.conv = specs[p].conv; pp.sym = specs[p].sym;
    pp.definite = specs[p].sym && specs[p].definite;
    pp.net = specs[p].net;
    pp.nb = 4 * (n - 1);
    pp.L = user_depth(n, leaf);
    pp.Lr = std::max(pp.L, user_depth(n, kBaseSide));
    const int Lr = pp.Lr;
    quadtree_levels(n, Lr, T.boxes);
    for (auto& lv : T.boxes)
      for (auto& b : lv)
        if (b.sx() < 2 || b.sy() < 2) { err = "box narrower than 2 nodes"; return false; }
    // Schur complements of level l live in LVA (l even) or LVB (l odd), in this problem's region.
    T.off.assign(Lr + 1, {});
    for (int l = 0; l <= Lr; ++l) {
      long long o = 0;
      for (auto& b : T.boxes[l]) { T.off[l].push_back(o); o += (long long)b.ring() * b.ring(); }
      size_t& need = (l % 2 == 0) ? T.lva_need : T.lvb_need;
      need = std::max(need, (size_t)o);
    }
    for (int l = 0; l < Lr; ++l) {
      long long o = 0;
      for (size_t q = 0; q < T.boxes[l].size(); ++q)
        for (int h = 0; h < 2; ++h) {
          const Rect& w = T.boxes[l + 1][4 * q + 2 * h];
          const Rect& e = T.boxes[l + 1][4 * q + 2 * h + 1];
          Rect u{w.x0, e.x1, w.y0, w.y1};
          o += (long long)u.ring() * u.ring();
        }
      T.half_need = std::max(T.half_need, (size_t)o);
    }
    T.lva_base = (long long)lva; lva += T.lva_need;
    T.lvb_base = (long long)lvb; lvb += T.lvb_need;
    pp.lva_base = T.lva_base;
    pp.lvb_base = T.lvb_base;
    T.half_base = (long long)half; half += T.half_need;
    pp.coef_off = (long long)coef; coef += 3 * (size_t)n * n;
    // Algorithmic flops: banded leaf model at the user's leaves, merge model above.
    pp.level_model_flops.assign(pp.L + 1, 0.0);
    for (auto& b : T.boxes[pp.L]) {
      const double mx = std::max(0, b.sx() - 2), my = std::max(0, b.sy() - 2);
      const double nrhs = std::max(0.0, 2 * (mx + my) - 4);
      pp.level_model_flops[pp.L] += 2.0 * mx * my * mx * mx + 4.0 * mx * my * mx * nrhs;
    }
    pp.root_buf = BUF_LVA;
    pp.root_off = T.lva_base;
  }
  P.lva_doubles = lva;
  P.lvb_doubles = lvb;
  P.half_doubles = half;
  P.coef_doubles = coef;
  auto lvbuf = [](int l) { return (l % 2 == 0) ? BUF_LVA : BUF_LVB; };
  auto lvoff = [](const Tree& T, int l, size_t q) {
    return (l % 2 == 0 ? T.lva_base : T.lvb_base) + T.off[l][q];
  };
  auto merge_flops = [](const SchurTask& t) {
    const double e = t.e, i = t.i;
    return 2.0 / 3.0 * i * i * i + 2.0 * i * i * e + e * e * i;
  };

  int K = 0;
  for (const Tree& T : trees) K = std::max(K, merge_phases(T));
  for (int k = 0; k < K; ++k) {
    Phase ph;
    ph.kind = k == 0 ? PH_BASE : (k % 2 == 1 ? PH_WE : PH_SN);
    std::vector<SchurTask> tasks;
    std::vector<TaskTag> tags;
    for (size_t pi = 0; pi < trees.size(); ++pi) {
      Tree& T = trees[pi];
      if (k >= merge_phases(T)) continue;
      ProbPlan& pp = T.pp;
      B.set_problem(pp);
      const int Lr = pp.Lr;
      if (k == 0) {
        B.cur_level = Lr;
        ph.level = Lr;
        ph.min_level = std::min(ph.min_level, Lr);
        ph.in_leaf = Lr > pp.L;
        for (size_t q = 0; q < T.boxes[Lr].size(); ++q) {
          tasks.push_back(B.base_task(T.boxes[Lr][q], lvbuf(Lr), lvoff(T, Lr, q)));
          tags.push_back({PH_BASE, Lr, (int)q, (int)pi});
        }
        continue;
      }
      const int l = Lr - (k + 1) / 2, cl = l + 1;
      B.cur_level = l;
      ph.level = l;
      ph.min_level = std::min(ph.min_level, l);
      ph.in_leaf = l >= pp.L;
      double fl = 0.0;
      if (ph.kind == PH_WE) {
        // (SW, SE) -> bottom half, (NW, NE) -> top half
        T.halves.clear();
        T.hoff.clear();
        long long ho = T.half_base;
        for (size_t q = 0; q < T.boxes[l].size(); ++q)
          for (int h = 0; h < 2; ++h) {
            const Rect& w = T.boxes[cl][4 * q + 2 * h];
            const Rect& e = T.boxes[cl][4 * q + 2 * h + 1];
            Rect u{w.x0, e.x1, w.y0, w.y1};
            SchurTask t;
            if (!B.merge_task(w, lvbuf(cl), lvoff(T, cl, 4 * q + 2 * h), e, lvoff(T, cl, 4 * q + 2 * h + 1),
                              BUF_HALF, ho, t, err)) return false;
            tasks.push_back(t);
            tags.push_back({PH_WE, l, (int)(2 * q + h), (int)pi});
            fl += merge_flops(t);
            T.halves.push_back(u);
            T.hoff.push_back(ho);
            ho += (long long)u.ring() * u.ring();
          }
      } else {
        // (bottom, top) -> box
        for (size_t q = 0; q < T.boxes[l].size(); ++q) {
          SchurTask t;
          if (!B.merge_task(T.halves[2 * q], BUF_HALF, T.hoff[2 * q], T.halves[2 * q + 1], T.hoff[2 * q + 1],
                            lvbuf(l), lvoff(T, l, q), t, err)) return false;
          tasks.push_back(t);
          tags.push_back({PH_SN, l, (int)q, (int)pi});
          fl += merge_flops(t);
        }
      }
      if (l < pp.L) pp.level_model_flops[l] += fl;
    }
    B.finish_phase(ph, tasks, tags);
    if (ph.kind == PH_BASE) ph.model_flops = 0;
    P.phases.push_back(std::move(ph));
  }
  // The int scratch (pivots, column maps) follows the constant index pool on the device.
  const int ibase = (int)P.ipool.size();
  for (auto& m : P.large)
    if (m.piv >= 0) m.piv += ibase;
  for (auto& g : P.gemms) {
    if (g.kmapA >= 0) g.kmapA += ibase;
    if (g.kcnt >= 0) g.kcnt += ibase;
  }
  for (auto& d : P.pchols) d.rank += ibase;
  for (auto& r : P.rank_slots) { r.first += ibase; r.second += ibase; }
  // BUF_AUX: identity (kCompCols x kCompCols), then the Gaussian test matrix (aux_rows x kCompCols)
  if (!P.pchols.empty()) {
    const long long KC = kCompCols, rows = P.aux_rows;
    P.aux.assign(KC * KC + rows * KC, 0.0);
    for (long long q = 0; q < KC; ++q) P.aux[q + q * KC] = 1.0;
    gaussian_fill(P.aux.data() + KC * KC, (size_t)(rows * KC), 0x243F6A8885A308D3ULL);
    for (int q : B.omega_descs) {
      GemmDesc& g = P.gemms[q];
      g.offB = KC * KC + g.offB * rows;   // offB held the first column of the test matrix
      g.ldb = (int)rows;
    }
  }
  for (Tree& T : trees) {
    T.pp.model_flops = 0;
    for (double f : T.pp.level_model_flops) T.pp.model_flops += f;
    P.probs.push_back(T.pp);
  }
  const ProbPlan& p0 = P.probs[0];
  P.n = p0.n; P.leaf = p0.leaf; P.conv = p0.conv; P.nb = p0.nb; P.L = p0.L; P.Lr = p0.Lr;
  P.root_buf = p0.root_buf;
  P.root_off = p0.root_off;
  P.level_model_flops = p0.level_model_flops;
  P.model_flops = 0;
  for (const ProbPlan& pp : P.probs) P.model_flops += pp.model_flops;
  if (P.ws_doubles == 0) P.ws_doubles = 32;
  if (P.half_doubles == 0) P.half_doubles = 32;
  if (P.lvb_doubles == 0) P.lvb_doubles = 32;
  return true;
}

std::string Plan::describe() const {
  std::ostringstream o;
  o << "plan n=" << n << " leaf=" << leaf << " L=" << L << " Lr=" << Lr << " nb=" << nb
    << " tasks=" << tasks.size() << " large=" << large.size() << " gemms=" << gemms.size()
    << " ws=" << ws_doubles * 8 / 1e6 << "MB lva=" << lva_doubles * 8 / 1e6 << "MB lvb="
    << lvb_doubles * 8 / 1e6 << "MB half=" << half_doubles * 8 / 1e6 << "MB model_flops=" << model_flops
    << "\n";
  for (const auto& ph : phases) {
    o << "  phase kind=" << ph.kind << " level=" << ph.level << (ph.in_leaf ? " (leaf)" : "")
      << " small=" << ph.small_count << " large=" << ph.large_count << " imax=" << ph.imax
      << " emax=" << ph.emax << " gje=" << ph.gje_nt << "/" << ph.gje_r << "/" << ph.gje_w
      << " steps=" << ph.gje_update.size() << " xgemm_tiles=" << ph.xgemm.tiles
      << " sgemm_tiles=" << ph.sgemm.tiles << "\n";
  }
  return o.str();
}

}  // namespace dtn

namespace dtn {

// Host-side consistency check of a plan: every device descriptor addresses only the buffers the
// runtime allocates for the plan (sizes from the plan itself), every int-pool reference lies inside
// the pool and its scratch, and every launch's tiles are numbered without gaps.  Column maps that
// the pivoted path fills on the device are not known here and are not followed.
bool plan_check(const Plan& P, std::string& err) {
  const long long ipn = (long long)P.ipool.size() + (long long)P.int_ws + 1;
  auto size_of = [&](int buf) -> long long {
    switch (buf) {
      case BUF_WS: return (long long)P.ws_doubles;
      case BUF_LVA: return (long long)P.lva_doubles;
      case BUF_LVB: return (long long)P.lvb_doubles;
      case BUF_HALF: return (long long)P.half_doubles;
      case BUF_COEF: return (long long)P.coef_doubles;
      case BUF_AUX: return (long long)P.aux.size();
      default: return -1;
    }
  };
  std::ostringstream os;
  auto fail = [&](const std::string& what) { err = what; return false; };
  auto in_buf = [&](int buf, long long lo, long long hi) {   // [lo, hi] inside buffer buf
    const long long n = size_of(buf);
    return n >= 0 && lo >= 0 && hi < n && lo <= hi + 1;
  };
  auto pool_max = [&](int off, int cnt, int& mx) {           // largest constant-pool entry of a map
    if (off < 0 || (long long)off + cnt > (long long)P.ipool.size()) return false;
    mx = 0;
    for (int q = 0; q < cnt; ++q) mx = std::max(mx, P.ipool[off + q]);
    return true;
  };
  for (size_t d = 0; d < P.gemms.size(); ++d) {
    const GemmDesc& g = P.gemms[d];
    os.str("");
    os << "gemm descriptor " << d << " (" << g.M << "x" << g.N << "x" << g.K << "): ";
    if (g.M <= 0 || g.N <= 0 || g.K < 0) return fail(os.str() + "empty or negative shape");
    if (g.K > 0) {
      long long hiA;
      if (g.transA) hiA = g.offA + (g.K - 1) + (long long)(g.M - 1) * g.lda;
      else if (g.kmapA >= 0) hiA = g.offA + (g.M - 1);   // columns from a device-filled map
      else hiA = g.offA + (g.M - 1) + (long long)(g.K - 1) * g.lda;
      if (!in_buf(g.bufA, g.offA, hiA)) return fail(os.str() + "A outside its buffer");
      if (!in_buf(g.bufB, g.offB, g.offB + (g.K - 1) + (long long)(g.N - 1) * g.ldb))
        return fail(os.str() + "B outside its buffer");
    }
    int rmax = g.M - 1, cmax = g.N - 1;
    if (g.rmapC >= 0 && !pool_max(g.rmapC, g.M, rmax)) return fail(os.str() + "row map outside the pool");
    if (g.cmapC >= 0 && !pool_max(g.cmapC, g.N, cmax)) return fail(os.str() + "column map outside the pool");
    if (!in_buf(g.bufC, g.offC, g.offC + rmax + (long long)cmax * g.ldc)) return fail(os.str() + "C outside its buffer");
    if (g.mirror && !in_buf(g.bufC, g.offC, g.offC + cmax + (long long)rmax * g.ldc))
      return fail(os.str() + "mirrored C outside its buffer");
    if (g.tri && (g.M != g.N || g.rmapC != g.cmapC)) return fail(os.str() + "triangular block is not symmetric in shape");
    if ((g.tri || g.mirror) && g.ksplit > 1) return fail(os.str() + "symmetric blocks are not split");
    if (g.kee > 0) {
      if ((size_t)(g.kee - 1) >= P.large.size()) return fail(os.str() + "K_ee source is not a large merge");
      const SchurTask& t = P.large[g.kee - 1].t;
      if (g.kee_row0 < 0 || g.kee_row0 + g.M > t.e || g.kee_col0 < 0 || g.kee_col0 + g.N > t.e)
        return fail(os.str() + "K_ee block outside the merge");
    }
    if (g.ksplit > 1) {
      const long long tiles = (long long)g.tiles_m * g.tiles_n;
      if (g.kcnt < (long long)P.ipool.size() || g.kcnt + tiles > ipn) return fail(os.str() + "split counters outside the int scratch");
      if (g.kpart < 0 || g.kpart >= (long long)P.ws_doubles) return fail(os.str() + "split partials outside ws");
    }
  }
  auto check_launch = [&](const LaunchGemm& L, const char* what) {
    if (L.count == 0) return true;
    const int tm = (L.cfg == 3 || L.cfg == 4) ? 32 : L.cfg == 2 || L.cfg == 1 ? 128 : 64;
    long long tiles = 0;
    for (int q = 0; q < L.count; ++q) {
      const GemmDesc& g = P.gemms[L.first + q];
      if (g.tile_start != tiles) { err = std::string(what) + ": tiles not numbered contiguously"; return false; }
      if (g.tiles_m != (g.M + tm - 1) / tm || g.tiles_n != (g.N + tm - 1) / tm) {
        err = std::string(what) + ": tile counts do not match the launch's tile";
        return false;
      }
      const long long ot = g.tri ? (long long)g.tiles_m * (g.tiles_m + 1) / 2 : (long long)g.tiles_m * g.tiles_n;
      if (g.ksplit > 1 && g.kpart + ot * g.ksplit * tm * tm > (long long)P.ws_doubles) {
        err = std::string(what) + ": split partials outside ws";
        return false;
      }
      tiles += ot * std::max(1, g.ksplit);
    }
    if (tiles != L.tiles) { err = std::string(what) + ": launch tile total mismatch"; return false; }
    return true;
  };
  for (size_t q = 0; q < P.phases.size(); ++q) {
    const Phase& ph = P.phases[q];
    for (const auto& L : ph.gje_update) if (!check_launch(L, "block Gauss-Jordan update")) return false;
    for (const auto& op : ph.inv_ops) if (!check_launch(op.gemm, "block inversion product")) return false;
    if (!check_launch(ph.xgemm, "X product") || !check_launch(ph.sgemm, "Schur product") ||
        !check_launch(ph.sgemm_tri, "Schur product (diagonal blocks)"))
      return false;
    for (const auto& op : ph.comp_ops) if (!check_launch(op.gemm, "compression product")) return false;
  }
  for (size_t b = 0; b < P.bases.size(); ++b) {
    const BaseBlock& bb = P.bases[b];
    if (bb.bs <= 0 || bb.bs > kBaseBlock || !in_buf(BUF_WS, bb.off, bb.off + (bb.bs - 1) + (long long)(bb.bs - 1) * bb.ld) ||
        !in_buf(BUF_WS, bb.scale, bb.scale))
      return fail("diagonal block " + std::to_string(b) + " outside ws");
  }
  for (size_t c = 0; c < P.couples.size(); ++c) {
    const CoupleDesc& d = P.couples[c];
    int mx = 0;
    if (d.h1 + d.h2 != d.i || !pool_max(d.match, d.h2, mx) || mx >= d.h1 ||
        !in_buf(BUF_WS, d.inv, d.inv + (long long)d.i * d.i - 1) ||
        !in_buf(BUF_WS, d.wb, d.wb + (long long)d.h1 * d.h2 - 1) || !in_buf(BUF_WS, d.wc, d.wc + (long long)d.h1 * d.h2 - 1))
      return fail("coupling step " + std::to_string(c) + " outside its buffers");
    for (int q = 0; q < d.h2; ++q)
      if (P.ipool[d.match + q] < -1) return fail("coupling step " + std::to_string(c) + ": bad match entry");
  }
  for (size_t q = 0; q < P.tasks.size(); ++q) {
    const SchurTask& t = P.tasks[q];
    const long long e = t.e, i = t.i;
    if (t.idx < 0 || t.idx + 3 * e + 2 * i > (long long)P.ipool.size()) return fail("small task " + std::to_string(q) + ": maps outside the pool");
    if (!in_buf(t.dst, t.out, t.out + e * e - 1)) return fail("small task " + std::to_string(q) + ": output outside its buffer");
    if (t.kind == 1 && (!in_buf(t.src, t.s1, t.s1 + (long long)t.m1 * t.m1 - 1) || !in_buf(t.src, t.s2, t.s2 + (long long)t.m2 * t.m2 - 1)))
      return fail("small task " + std::to_string(q) + ": children outside their buffer");
  }
  for (size_t q = 0; q < P.large.size(); ++q) {
    const LargeMerge& m = P.large[q];
    const SchurTask& t = m.t;
    const long long e = t.e, i = t.i;
    if (t.idx < 0 || t.idx + 3 * e + 2 * i > (long long)P.ipool.size()) return fail("large merge " + std::to_string(q) + ": maps outside the pool");
    if (!in_buf(t.dst, t.out, t.out + e * e - 1) || !in_buf(t.src, t.s1, t.s1 + (long long)t.m1 * t.m1 - 1) ||
        !in_buf(t.src, t.s2, t.s2 + (long long)t.m2 * t.m2 - 1))
      return fail("large merge " + std::to_string(q) + ": output or children outside their buffers");
    if (!in_buf(BUF_WS, m.inv, m.inv + i * i - 1) || !in_buf(BUF_WS, m.scale, m.scale))
      return fail("large merge " + std::to_string(q) + ": K_ii outside ws");
  }
  for (size_t q = 0; q < P.pchols.size(); ++q) {
    const PcholDesc& d = P.pchols[q];
    const long long k2 = (long long)d.k * d.k;
    if (!in_buf(BUF_WS, d.g, d.g + k2 - 1) || !in_buf(BUF_WS, d.m, d.m + k2 - 1) || !in_buf(BUF_WS, d.dmax, d.dmax) ||
        d.rank < (int)P.ipool.size() || d.rank >= ipn)
      return fail("range-finder step " + std::to_string(q) + " outside its buffers");
  }
  return true;
}

}  // namespace dtn
