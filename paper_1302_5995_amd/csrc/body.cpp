// Body loads (Section 7.3): planning of the right-hand-side updates that carry loads at fixed interior
// nodes through the nested-dissection build (the leaf's update, then Section 3.2's update at every
// pairwise merge), so that the root's condensed right-hand sides give the operator F from loads to
// boundary fluxes.
#include <algorithm>
#include <map>
#include <numeric>
#include <tuple>

#include "plan.h"

namespace dtn {

namespace {

constexpr int kBodyTile = 64;   // the body products run on 64 x 64 tiles

GemmDesc body_gd(int M, int N, int K, int bA, long long oA, int lda, int kmap, int bB, long long oB, int ldb,
                 int bC, long long oC, int ldc, int rmap, double alpha, double beta) {
  GemmDesc g{};
  g.M = M; g.N = N; g.K = K;
  g.bufA = bA; g.bufB = bB; g.bufC = bC;
  g.offA = oA; g.offB = oB; g.offC = oC;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.rmapC = rmap; g.cmapC = -1; g.kmapA = kmap;
  g.kcnt = -1;
  g.tiles_m = (M + kBodyTile - 1) / kBodyTile;
  g.tiles_n = (N + kBodyTile - 1) / kBodyTile;
  g.alpha = alpha; g.beta = beta;
  return g;
}

}  // namespace

bool body_plan_make(const Plan& P, const std::vector<int>& nodes, int (*class_of)(int), BodyPlan& B,
                    std::string& err) {
  B = BodyPlan{};
  if (P.probs.size() != 1) { err = "body loads: single-problem builds only"; return false; }
  if (P.tol > 0.0) { err = "body loads: dense builds only (tol = 0)"; return false; }
  const ProbPlan& pp = P.probs[0];
  const int n = pp.n, Lr = pp.Lr;
  if (P.task_tags.size() != P.tasks.size() || P.large_tags.size() != P.large.size()) {
    err = "body loads: plan without task boxes";
    return false;
  }
  std::vector<std::vector<Rect>> boxes;
  quadtree_levels(n, Lr, boxes);
  std::vector<int> base_of((size_t)n * n, -1);
  for (size_t q = 0; q < boxes[Lr].size(); ++q) {
    const Rect& r = boxes[Lr][q];
    for (int j = r.y0; j < r.y1; ++j)
      for (int i = r.x0; i < r.x1; ++i) base_of[(size_t)i + (size_t)n * j] = (int)q;
  }
  const int cnt = (int)nodes.size();
  std::vector<long long> key(cnt);
  for (int q = 0; q < cnt; ++q) {
    const int i = nodes[q] & 0xFFFF, j = nodes[q] >> 16;
    if (nodes[q] < 0 || i <= 0 || j <= 0 || i >= n - 1 || j >= n - 1) {
      err = "body loads: node " + std::to_string(q) + " is not an interior node of the grid";
      return false;
    }
    key[q] = ((long long)base_of[(size_t)i + (size_t)n * j] << 32) | (long long)nodes[q];
  }
  B.user.resize(cnt);
  std::iota(B.user.begin(), B.user.end(), 0);
  std::sort(B.user.begin(), B.user.end(), [&](int a, int b) { return key[a] < key[b]; });
  for (int s = 1; s < cnt; ++s)
    if (key[B.user[s]] == key[B.user[s - 1]]) { err = "body loads: a node is listed twice"; return false; }
  B.count = cnt;
  B.nodes.resize(cnt);
  std::vector<int> base_sorted(cnt);
  for (int s = 0; s < cnt; ++s) {
    B.nodes[s] = nodes[B.user[s]];
    base_sorted[s] = (int)(key[B.user[s]] >> 32);
  }
  // the loads of base boxes [b0, b1)
  auto cols = [&](long long b0, long long b1) {
    const int lo = (int)(std::lower_bound(base_sorted.begin(), base_sorted.end(), b0) - base_sorted.begin());
    const int hi = (int)(std::lower_bound(base_sorted.begin(), base_sorted.end(), b1) - base_sorted.begin());
    return std::make_pair(lo, hi);
  };
  auto span = [&](int l) { return 1LL << (2 * (Lr - l)); };   // base boxes under one box of level l
  auto box_cols = [&](int l, long long q) { return cols(q * span(l), (q + 1) * span(l)); };
  auto half_cols = [&](int l, long long q) { return cols(2 * q * span(l + 1), (2 * q + 2) * span(l + 1)); };

  // C buffers: (0, l, q) the level box, (1, l, q) the half
  std::map<std::tuple<int, int, long long>, long long> coff;
  long long body = 0;
  bool have_root = false;
  B.phases.resize(P.phases.size());
  for (size_t k = 0; k < P.phases.size(); ++k) {
    const Phase& ph = P.phases[k];
    BodyPhase& bp = B.phases[k];
    bp.job_first = (int)B.jobs.size();
    long long scr = 0;
    std::vector<GemmDesc> zg, ug;
    std::vector<HbsGj> gj;
    auto add_task = [&](const SchurTask& t, const TaskTag& g, const LargeMerge* m) -> bool {
      std::pair<int, int> c, c1{0, 0}, c2{0, 0};
      std::tuple<int, int, long long> out_key, k1, k2;
      if (g.kind == PH_BASE) {
        c = box_cols(g.l, g.q);
        out_key = std::make_tuple(0, g.l, (long long)g.q);
      } else if (g.kind == PH_WE) {
        c = half_cols(g.l, g.q);
        c1 = box_cols(g.l + 1, 2LL * g.q);
        c2 = box_cols(g.l + 1, 2LL * g.q + 1);
        out_key = std::make_tuple(1, g.l, (long long)g.q);
        k1 = std::make_tuple(0, g.l + 1, 2LL * g.q);
        k2 = std::make_tuple(0, g.l + 1, 2LL * g.q + 1);
      } else {
        c = box_cols(g.l, g.q);
        c1 = half_cols(g.l, 2LL * g.q);
        c2 = half_cols(g.l, 2LL * g.q + 1);
        out_key = std::make_tuple(0, g.l, (long long)g.q);
        k1 = std::make_tuple(1, g.l, 2LL * g.q);
        k2 = std::make_tuple(1, g.l, 2LL * g.q + 1);
      }
      if (c.second <= c.first) return true;
      const int nbs = c.second - c.first, e = t.e, i = t.i;
      BodyJob j{};
      j.t = t;
      j.lo = c.first; j.hi = c.second;
      j.lo1 = c1.first; j.hi1 = c1.second; j.lo2 = c2.first; j.hi2 = c2.second;
      j.c1 = j.c2 = 0;
      if (g.kind != PH_BASE) {
        if (c1.first != c.first || c1.second != c2.first || c2.second != c.second) {
          err = "body loads: children's loads are not contiguous";
          return false;
        }
        if (c1.second > c1.first) {
          auto it = coff.find(k1);
          if (it == coff.end()) { err = "body loads: a child's right-hand sides were not formed"; return false; }
          j.c1 = it->second;
        }
        if (c2.second > c2.first) {
          auto it = coff.find(k2);
          if (it == coff.end()) { err = "body loads: a child's right-hand sides were not formed"; return false; }
          j.c2 = it->second;
        }
      }
      j.out = body;
      coff[out_key] = body;
      body += (long long)e * nbs;
      body = (body + 31) & ~31LL;
      j.kii = -1;
      if (!m && i > 0) {
        if (!class_of || (class_of(i) == 0 && i > 256)) { err = "body loads: interface block too large"; return false; }
        j.kii = scr; scr += (long long)i * i;
      }
      j.cint = scr; scr += (long long)i * nbs;
      j.kei = scr; scr += (long long)e * i;
      j.z = scr; scr += (long long)i * nbs;
      scr = (scr + 31) & ~31LL;
      j.elems = (long long)e * nbs + (long long)i * nbs + (long long)e * i + (j.kii >= 0 ? (long long)i * i : 0);
      j.bodies = j.lo;
      bp.elems_max = std::max(bp.elems_max, j.elems);
      if (i > 0) {
        if (j.kii >= 0) gj.push_back({2, i, j.kii});
        if (m) {
          const int kmap = P.fast ? -1 : m->piv + i;
          zg.push_back(body_gd(i, nbs, i, BUF_WS, m->inv, i, kmap, BUF_BSCR, j.cint, i, BUF_BSCR, j.z, i, -1, 1.0, 0.0));
        } else {
          zg.push_back(body_gd(i, nbs, i, BUF_BSCR, j.kii, i, -1, BUF_BSCR, j.cint, i, BUF_BSCR, j.z, i, -1, 1.0, 0.0));
        }
        ug.push_back(body_gd(e, nbs, i, BUF_BSCR, j.kei, e, -1, BUF_BSCR, j.z, i, BUF_BODY, j.out, e,
                             t.idx + 2 * (e + i), -1.0, 1.0));
      }
      if (g.l == 0 && g.kind != PH_WE) {
        B.root_off = j.out;
        have_root = true;
      }
      B.jobs.push_back(j);
      return true;
    };
    for (int q = 0; q < ph.small_count; ++q)
      if (!add_task(P.tasks[ph.small_first + q], P.task_tags[ph.small_first + q], nullptr)) return false;
    for (int q = 0; q < ph.large_count; ++q)
      if (!add_task(P.large[ph.large_first + q].t, P.large_tags[ph.large_first + q], &P.large[ph.large_first + q]))
        return false;
    bp.job_count = (int)B.jobs.size() - bp.job_first;
    B.scr_doubles = std::max(B.scr_doubles, (size_t)scr);
    // Gauss-Jordan launches, one per size class
    std::stable_sort(gj.begin(), gj.end(), [](const HbsGj& a, const HbsGj& b) { return a.n < b.n; });
    for (size_t g = 0; g < gj.size();) {
      const int cls = class_of(gj[g].n);
      size_t e = g;
      while (e < gj.size() && class_of(gj[e].n) == cls) ++e;
      bp.gj_first.push_back((int)B.gjs.size() + (int)g);
      bp.gj_count.push_back((int)(e - g));
      bp.gj_cls.push_back(cls);
      g = e;
    }
    B.gjs.insert(B.gjs.end(), gj.begin(), gj.end());
    auto place = [&](std::vector<GemmDesc>& v, int& first, int& count, int& tiles) {
      first = (int)B.gemms.size();
      count = (int)v.size();
      tiles = 0;
      for (auto& g : v) {
        g.tile_start = tiles;
        tiles += g.tiles_m * g.tiles_n;
      }
      B.gemms.insert(B.gemms.end(), v.begin(), v.end());
    };
    place(zg, bp.zg_first, bp.zg_count, bp.zg_tiles);
    bool any_kmap = false, any_plain = false;
    for (auto& g : zg) (g.kmapA >= 0 ? any_kmap : any_plain) = true;
    bp.zg_mode = any_kmap && any_plain ? 3 : any_kmap ? 1 : 0;
    place(ug, bp.ug_first, bp.ug_count, bp.ug_tiles);
  }
  if (!have_root && cnt > 0) { err = "body loads: the root box carried no loads"; return false; }
  B.body_doubles = (size_t)std::max<long long>(body, 1);
  return true;
}

bool body_plan_check(const Plan& P, const BodyPlan& B, std::string& err) {
  auto fail = [&](const std::string& m) { err = "body plan: " + m; return false; };
  std::map<long long, std::pair<int, int>> formed;   // C offset -> (ld, columns)
  for (size_t k = 0; k < B.phases.size(); ++k) {
    const BodyPhase& ph = B.phases[k];
    if (ph.job_first < 0 || ph.job_first + ph.job_count > (int)B.jobs.size()) return fail("job range");
    for (int q = ph.job_first; q < ph.job_first + ph.job_count; ++q) {
      const BodyJob& j = B.jobs[q];
      const SchurTask& t = j.t;
      const long long e = t.e, i = t.i, nbs = j.hi - j.lo;
      if (nbs <= 0 || j.lo < 0 || j.hi > B.count) return fail("columns");
      if (j.out < 0 || j.out + e * nbs > (long long)B.body_doubles) return fail("output C");
      if (t.idx < 0 || (size_t)t.idx + 2 * (e + i) + e > P.ipool.size()) return fail("index maps");
      const int* cpos = P.ipool.data() + t.idx;
      const int* pmap = cpos + 2 * (e + i);
      for (long long r = 0; r < e; ++r)
        if (pmap[r] < 0 || pmap[r] >= e) return fail("parent ring position");
      if (t.kind == 1) {
        for (int side = 0; side < 2; ++side) {
          const int lo = side ? j.lo2 : j.lo1, hi = side ? j.hi2 : j.hi1;
          const long long off = side ? j.c2 : j.c1;
          const int m = side ? t.m2 : t.m1;
          if (hi <= lo) continue;
          auto it = formed.find(off);
          if (it == formed.end() || it->second.first != m || it->second.second != hi - lo)
            return fail("a child's C is missing or of another shape");
          for (long long a = 0; a < e + i; ++a) {
            const bool first = a < t.e1 || (a >= e && a < e + t.i1);
            if (first == (side == 0) && (cpos[a] < 0 || cpos[a] >= m)) return fail("child ring position");
          }
        }
      } else if (t.kind != 0) {
        return fail("task kind");
      }
      const long long scr = (long long)B.scr_doubles;
      if (j.cint < 0 || j.cint + i * nbs > scr || j.kei < 0 || j.kei + e * i > scr || j.z < 0 || j.z + i * nbs > scr)
        return fail("scratch");
      if (j.kii >= 0 && j.kii + i * i > scr) return fail("K_ii scratch");
      formed[j.out] = std::make_pair((int)e, (int)nbs);
    }
    for (size_t g = 0; g < ph.gj_first.size(); ++g)
      for (int q = ph.gj_first[g]; q < ph.gj_first[g] + ph.gj_count[g]; ++q) {
        if (q < 0 || q >= (int)B.gjs.size()) return fail("inversion job");
        const HbsGj& gj = B.gjs[q];
        if (gj.n <= 0 || gj.n > 256 || gj.off < 0 || gj.off + (long long)gj.n * gj.n > (long long)B.scr_doubles)
          return fail("inversion block");
      }
    for (int q = 0; q < ph.zg_count + ph.ug_count; ++q) {
      const int gi = q < ph.zg_count ? ph.zg_first + q : ph.ug_first + q - ph.zg_count;
      if (gi < 0 || gi >= (int)B.gemms.size()) return fail("product");
      const GemmDesc& g = B.gemms[gi];
      auto inside = [&](int buf, long long off, long long ld, long long rows, long long cols) {
        const long long cap = buf == BUF_WS ? (long long)P.ws_doubles : buf == BUF_BSCR ? (long long)B.scr_doubles
                                              : buf == BUF_BODY ? (long long)B.body_doubles : -1;
        return off >= 0 && ld >= rows && off + ld * (cols - 1) + rows <= cap;
      };
      const long long Crows = g.rmapC >= 0 ? g.ldc : g.M;
      if (!inside(g.bufA, g.offA, g.lda, g.M, g.K) || !inside(g.bufB, g.offB, g.ldb, g.K, g.N) ||
          !inside(g.bufC, g.offC, g.ldc, Crows, g.N))
        return fail("product operand outside its buffer");
    }
  }
  if (B.count > 0) {
    auto it = formed.find(B.root_off);
    if (it == formed.end() || it->second.first != P.probs[0].nb || it->second.second != B.count)
      return fail("root right-hand sides");
  }
  return true;
}

}  // namespace dtn
