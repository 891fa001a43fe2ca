// Host planner of the DtN build: quadtree (Section 2), per-level merge schedule
// (Section 3.3), index maps of the pairwise merge (Section 3.2), workspace
// layout and the descriptors of every batched launch.  A plan depends only on
// (n, leaf, convection form); coefficient values enter at build time.
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace dtn {

struct Rect {
  int x0, x1, y0, y1;
  int sx() const { return x1 - x0; }
  int sy() const { return y1 - y0; }
  int ring() const { return 2 * (sx() - 1) + 2 * (sy() - 1); }
};

struct LaunchGemm {
  int first = 0;     // first descriptor in Plan::gemms
  int count = 0;     // descriptors in this launch
  int tiles = 0;     // total tiles (workgroups)
  double flops = 0;  // 2*M*N*K summed over the descriptors
  double bytes = 0;  // algorithmic operand traffic: A, B read once, C read (beta != 0) and written
  int cfg = 0;       // workgroup tile: 0 = 64 x 64, 2 = 128 x 128 (8 waves), 3 = 32 x 32
  int prec = 0;      // 0: FP64 MFMA; 1: FP32 MFMA (mixed-precision plans, lower levels)
  int mode = 3;      // form of A shared by the descriptors: 0 plain, 1 gathered columns, 2 transposed, 3 mixed
  std::string sig;   // autotuner key: the launch's shape (descriptor count, tiles, largest M, N, K, A form, flags)
};

enum PhaseKind { PH_BASE = 0, PH_WE = 1, PH_SN = 2 };

// One step of a compressed merge: a pivoted-Cholesky launch (pchol_first >= 0) or a product.
struct CompOp {
  int pchol_first = -1, pchol_count = 0;
  LaunchGemm gemm;
};

// Where the range finder of one compressed block leaves its ranks (int scratch slots).
struct RankSlot {
  int level = 0;
  int first = 0, second = 0;   // slots of the first and residual pass
};

// One launch of the recursive block inversion of a phase's interface blocks.
struct InvOp {
  int base_first = -1, base_count = 0;   // >= 0: diagonal-block inversion launch (Plan::bases)
  int couple_first = -1, couple_count = 0;   // >= 0: interface-coupling step launch (Plan::couples)
  LaunchGemm gemm;                       // otherwise one batched product
};

struct Phase {
  int kind = PH_BASE;
  int level = 0;          // refined-tree level of the boxes this phase produces
  int min_level = 1 << 30;  // smallest such level over the phase's problems
  bool in_leaf = false;   // below the user's leaf level (part of leaf elimination)
  int small_first = 0, small_count = 0;
  size_t small_lds = 0;   // dynamic LDS bytes of the small-merge kernel
  int large_first = 0, large_count = 0;
  int gje_nt = 0, gje_r = 0, gje_w = 0;
  int imax = 0, emax = 0;
  std::vector<LaunchGemm> gje_update;  // one per Gauss-Jordan block step
  LaunchGemm xgemm, sgemm;
  LaunchGemm sgemm_tri;   // symmetric merges: the triangular diagonal blocks of the Schur products
  std::vector<InvOp> inv_ops;          // fast path: recursive block inversion schedule
  int small_threads = 0;               // fast path: largest i + e of the small tasks
  int small_imax = 0;                  // fast path: largest i of the small tasks
  long long ws_end = 0;                // end of the phase's merge scratch in ws (split-K partials follow)
  bool compressed = false;             // large merges use low-rank factored off-diagonal blocks
  std::vector<CompOp> comp_ops;        // compressed merges: range finder and factored products
  double model_flops = 0;              // merge model 2/3 i^3 + 2 i^2 e + e^2 i summed
  double small_flops = 0, small_bytes = 0;   // work of the small-task launch
  double gather_bytes = 0;                   // large-merge gather traffic
};

// One problem of a (possibly multi-problem) plan.
struct ProbSpec {
  int n = 0, leaf = 0, conv = 0;
  int sym = 0;       // 1: no convection (b = c = 0): symmetric operator (the Schur products run half)
  int definite = 0;  // with sym: d >= 0 at every interior node, so every interface block is positive
                     // definite and well conditioned; the mirrored products then run at every level
  int nonneg = 0;    // d >= 0 at every interior node (known on the host): no interior resonance
  int net = 0;       // network form (conductances of the east and north links in b and c)
};

struct ProbPlan {
  int n = 0, leaf = 0, conv = 0, nb = 0;
  int sym = 0, definite = 0, net = 0;
  int L = 0, Lr = 0;
  long long coef_off = 0;          // b, c, d fields (3 n^2 doubles) in the coefficient buffer
  int root_buf = BUF_LVA;
  long long root_off = 0;          // the root Schur complement (nb x nb)
  double model_flops = 0;
  std::vector<double> level_model_flops;   // per user level (leaves at L)
  long long lva_base = 0, lvb_base = 0;    // this problem's region in the level buffers
};

// Boxes of every quadtree level (level 0 the root) down to level Lr, split as the planner splits them
// (floor halves, children SW, SE, NW, NE).  The Schur complements of level l lie in LVA (l even) or LVB
// (l odd) from the problem's base, box after box (ring x ring each), and are complete after phase 0
// (l = Lr) or phase 2 (Lr - l).
void quadtree_levels(int n, int Lr, std::vector<std::vector<Rect>>& boxes);

// Where a task's output box sits in its problem's quadtree: PH_BASE (base box q of level l), PH_WE (half
// q = 2 p + h of level l's box p: the merge of children 4 p + 2 h and 4 p + 2 h + 1 of level l + 1) or PH_SN
// (box q of level l: the merge of halves 2 q and 2 q + 1).
struct TaskTag {
  int kind, l, q, prob;
};

struct Plan {
  // problem 0 (the only one of a single-problem plan)
  int n = 0, leaf = 0, conv = 0;
  bool fast = true;  // true: unpivoted fast path (monitored); false: partial pivoting throughout
  bool mixed = false;  // FP32 MFMA X and Schur products (and inversion products below kMixedFp64Levels)
  int L = 0;        // user tree depth: leaves (side <= leaf) at level L
  int Lr = 0;       // refined depth: base boxes (side <= kBaseSide) at level Lr
  int nb = 0;
  std::vector<SchurTask> tasks;    // small-path tasks of all phases
  std::vector<LargeMerge> large;   // large-path merges of all phases
  std::vector<TaskTag> task_tags, large_tags;   // the box of each (host only)
  std::vector<GemmDesc> gemms;
  std::vector<BaseBlock> bases;
  std::vector<CoupleDesc> couples;
  std::vector<int> ipool;          // constant index data (cpos, node, pmap)
  size_t int_ws = 0;               // ints of scratch after ipool (pivots, column maps)
  size_t ws_doubles = 0, lva_doubles = 0, lvb_doubles = 0, half_doubles = 0;
  std::vector<Phase> phases;
  int root_buf = BUF_LVA;
  long long root_off = 0;
  double model_flops = 0;          // algorithmic flops: banded leaf model + merge model
  std::vector<double> level_model_flops;   // per user level (leaves at L)
  // every problem: phase k of the plan holds phase k (counted from the base boxes up) of
  // each problem that has one, so merges of equal height share launches across problems
  std::vector<ProbPlan> probs;
  size_t coef_doubles = 0;
  // low-rank compression of the top merges (Section 6, Step 2)
  double tol = 0.0;
  int hbs_level = -1;              // compress parents at levels <= this; -1: children's S >= 1000
  std::vector<PcholDesc> pchols;
  std::vector<RankSlot> rank_slots;
  std::vector<double> aux;         // BUF_AUX contents: Gaussian test matrix (aux_rows x kCompCols), identity
  int aux_rows = 0;
  int tune_force = -1;             // >= 0: every FP64 launch that can take this tile does (tuning runs)
  std::string describe() const;
};

constexpr int kBaseSide = 8;            // base boxes eliminated densely in one workgroup
constexpr int kMixedFp64Levels = 2;     // mixed precision: levels 0 .. 1 invert their interface blocks in FP64
#ifndef DTN_SYM_MIN_LEVEL
#define DTN_SYM_MIN_LEVEL 2
#endif
// Symmetric problems that are not known to be definite (d < 0 somewhere, e.g. Helmholtz) take the mirrored
// Schur products only at levels >= this: at the top levels, where the interface blocks are worst
// conditioned, the rounding error of one computed triangle copied to its mirror is amplified well beyond
// that of the two independently computed triangles.
constexpr int kSymMinLevel = DTN_SYM_MIN_LEVEL;
constexpr int kCompPass1 = 64, kCompPass2 = 32;   // range finder: sketch columns per pass
constexpr int kCompCols = kCompPass1 + kCompPass2;  // rank cap of a compressed block
constexpr int kCompMinChild = 1000;     // default: compress merges whose children's S >= 1000
constexpr size_t kSmallLdsMax = 150 * 1024;
constexpr int kSmallImax = 256;
constexpr int kGemmBM = 64, kGemmBN = 64;
constexpr int kSmallTileBelow = 1024;   // products with fewer 64 x 64 tiles than this use 32 x 32 tiles
constexpr int kBigTileMin = 512;
constexpr int kDeepChunkTiles = 512;    // 32 x 32 launches with at most this many tiles take K in chunks of 64        // products with at least this many 128 x 128 tiles use them
constexpr int kSplitTilesBelow = 256;   // launches with fewer tiles than this (and K >= kSplitMinK) split K
constexpr int kSplitMinK = 512;
constexpr int kSplitMinSlice = 128;     // each K slice at least this deep
constexpr int kSplitMax = 16;

int user_depth(int n, int leaf);
bool plan_make(int n, int leaf, int conv, bool fast, Plan& out, std::string& err);
bool plan_make_many(const std::vector<ProbSpec>& specs, bool fast, Plan& out, std::string& err,
                    bool mixed = false, double tol = 0.0, int hbs_level = -1, int tune_force = -1);

// Autotuned tile choice: a process-wide table from launch signature to tile configuration (0: 64 x 64,
// 2: 128 x 128, 3: 32 x 32, 4: 32 x 32 with K in chunks of 64), filled by timing runs (dtn_tune) or
// loaded from a JSON cache keyed by the GPU architecture.  When enabled, the planner takes a launch's
// tile from the table (if the tile suits the launch) instead of its fixed thresholds.
void tune_put(const std::string& sig, int cfg);
bool tune_get(const std::string& sig, int& cfg);
void tune_clear();
int tune_generation();           // changes whenever the table or the switch changes
void tune_enable(bool on);
bool tune_enabled();
size_t tune_size();
std::string tune_json(const std::string& arch);
bool tune_load_json(const std::string& text, const std::string& arch, std::string& err);
// Host-side check that every device descriptor of a plan stays inside the plan's buffers.
bool plan_check(const Plan& P, std::string& err);

// Body loads (Section 7.3) of a single-problem plan: the right-hand-side updates of every task whose box
// holds loads, phase by phase, with their buffers.  Loads are given as interior node codes (j << 16) | i
// and sorted so that every box's loads are contiguous (by base box, in the planner's box order).
struct BodyPhase {
  int job_first = 0, job_count = 0;
  long long elems_max = 0;                 // largest gather of one job
  std::vector<int> gj_first, gj_count, gj_cls;   // Gauss-Jordan launches (one per size class)
  int zg_first = 0, zg_count = 0, zg_tiles = 0, zg_mode = 0;   // Z = K_ii^{-1} C_int products
  int ug_first = 0, ug_count = 0, ug_tiles = 0;                // C -= K_ei Z products
};

struct BodyPlan {
  int count = 0;                   // loads
  std::vector<int> user;           // sorted position -> caller's index
  std::vector<int> nodes;          // sorted node codes
  std::vector<BodyJob> jobs;
  std::vector<HbsGj> gjs;
  std::vector<GemmDesc> gemms;
  std::vector<BodyPhase> phases;   // parallel to Plan::phases
  size_t body_doubles = 0, scr_doubles = 0;
  long long root_off = 0;          // the root box's C (nb x count) in BUF_BODY
};

// class_of(n): launch class of an n x n Gauss-Jordan block (0 for n beyond the kernels' 256).
bool body_plan_make(const Plan& P, const std::vector<int>& nodes, int (*class_of)(int), BodyPlan& B, std::string& err);
// Host check that every gather, inversion and product of a body plan stays inside its buffers.
bool body_plan_check(const Plan& P, const BodyPlan& B, std::string& err);

}  // namespace dtn
