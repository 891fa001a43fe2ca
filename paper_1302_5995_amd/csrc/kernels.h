// Launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace dtn {

// A pivot whose magnitude is at most this fraction of the largest entry of the
// block being factored marks the build as singular (DTN_ESINGULAR).
constexpr double kPivotRtol = 1e-11;
// The fast path eliminates without cross-row pivoting (the Schur complements of the
// build are strongly diagonally dominant); a pivot below this fraction of its block's
// largest entry sends the build back to the partially pivoted path.
constexpr double kWeakPivotRtol = 1e-5;
// Unpivoted path: element growth of a 128-block inverse (largest entry of the block or of its
// half-level Schur complement over the merge's largest K_ii entry) above which the build is redone
// with partial pivoting.
constexpr double kGrowthLimit = 16.0;
constexpr int kFastMaxI = 64;        // small fast tasks: i <= 64 and i + e <= 256 (one column per thread)
constexpr int kFastMaxCols = 256;
constexpr int kSmallFastLds = 100 * 1024;   // dynamic LDS limit of the small fast kernel (X = i x e + 64)
constexpr int kSmallWaveLds = 32 * 1024;    // one-wave small kernel: LDS per task (pivot column + X)
constexpr int kBaseBlock = 128;      // diagonal blocks of the recursive inversion (its bottom levels fused)
constexpr int kPcholMax = 96;        // largest Gram matrix of the range finder

hipError_t launch_small(const SchurTask* tasks, int count, size_t lds, const int* ip, const DevBufs& B,
                        DevStatus* st, hipStream_t s);
hipError_t launch_reset(const LargeMerge* lm, int nlm, const DevBufs& B, DevStatus* st, hipStream_t s);
hipError_t launch_large_gather(const LargeMerge* lm, int nlm, int blocks_per, const int* ip, const DevBufs& B,
                               hipStream_t s);
hipError_t launch_gje_panel(int nt, int r, int w, const LargeMerge* lm, int nlm, int c0, int* ip, const DevBufs& B,
                            DevStatus* st, hipStream_t s);
hipError_t launch_gje_swap(const LargeMerge* lm, int nlm, int imax, int c0, const int* ip, const DevBufs& B,
                           hipStream_t s);
hipError_t launch_gje_kmap(const LargeMerge* lm, int nlm, int imax, int* ip, hipStream_t s);
// cfg 0: 64 x 64 workgroup tiles (4 waves); cfg 2 (and 1): 128 x 128 (8 waves of 64 x 32, 512
// threads); cfg 3: 32 x 32 (4 waves of 16 x 16); cfg 4: 32 x 32 with K in chunks of 64 (small
// launches of short products).  The launch runs tiles tile_base ..
// tile_base + tiles - 1 of the descriptor list (tile_start numbering).  prec 0: FP64 MFMA;
// prec 1: FP32 MFMA on FP32-rounded operands (64 x 64 tiles), FP64 epilogue.  mode: the form of
// A shared by every descriptor of the launch (0 plain, 1 gathered columns through kmapA,
// 2 transposed, 3 mixed: read from each descriptor).
hipError_t launch_gemm_batched(const GemmDesc* descs, int ndesc, int tiles, int cfg, const DevBufs& B,
                               const int* ip, hipStream_t s, int tile_base = 0, int prec = 0, int mode = 3,
                               const LargeMerge* lm = nullptr);
hipError_t launch_gemm_single(GemmDesc D, int cfg, const DevBufs& B, hipStream_t s);
int gemm_tile_m(int cfg);
int gemm_tile_n(int cfg);
hipError_t launch_scale_copy(const double* S, double* T, long long cnt, double scale, hipStream_t s);
// Body loads: the gathers of a phase's right-hand-side updates (count jobs, chunks workgroups each) and
// the final F[:, user[c]] = scale * C[:, c].
hipError_t launch_body_gather(const BodyJob* jobs, int count, int chunks, const int* ip, const int* bnodes,
                              const DevBufs& B, double h2, hipStream_t s);
hipError_t launch_body_out(const double* C, int nb, int cnt, const int* user, double scale, double* F, int ldf,
                           hipStream_t s);

// Root output T = (ring-row change of S') / h for the R2 (reading 1) and R3 (reading 2) ring rows.
hipError_t launch_root_rows(const double* S, double* T, int n, int reading, const double* coef, double h2, double cs,
                            hipStream_t s);
// imax: largest i of the launch's tasks; cols: largest i + e; lds: largest i * e * 8 + 512 bytes.
// base: every task is a base box (kind 0), else every task is a merge (kind 1).
hipError_t launch_small_fast(const SchurTask* tasks, int count, bool base, int imax, int cols, size_t lds,
                             const int* ip, const DevBufs& B, DevStatus* st, hipStream_t s);
hipError_t launch_base_inv(const BaseBlock* blocks, int count, const DevBufs& B, DevStatus* st, hipStream_t s);
// Top step of the block inversion of merges split at the children's interface (CoupleDesc).
hipError_t launch_couple(const CoupleDesc* cd, int count, int blocks_per, const int* ip, const DevBufs& B,
                         hipStream_t s);
// Split-K apply for narrow right-hand sides (bitwise independent of how columns are batched).
// Partial-sum bytes of a launch of up to `cols` columns (capped at apply_splitk_max_cols()).
size_t apply_splitk_workspace(int nb, int cols);
int apply_splitk_max_cols();
// dtn_apply_device uses the split-K kernels up to this many columns and the MFMA GEMM above.
constexpr int kApplySplitkMaxK = 64;
hipError_t launch_apply_splitk(const double* T, int nb, const double* G, int ldg, int k, double* Y, int ldy,
                               double* part, hipStream_t s, int chunk = kApplySplitkMaxK);
// Allocation-free apply: a file-scope device array holds the split-K partials of operators with up to
// kNoAllocMaxNb ring rows, in column chunks of kNoAllocCols.
constexpr int kNoAllocMaxNb = 8188;   // 4 (n - 1) for n = 2048
constexpr int kNoAllocCols = 32;
// Device address of that array on the current device (call with the device current, once per device).
hipError_t noalloc_scratch_address(double** p);
size_t noalloc_scratch_bytes();
hipError_t launch_pchol(const PcholDesc* descs, int count, const DevBufs& B, int* ip, DevStatus* st, hipStream_t s);
hipError_t kernels_init();

}  // namespace dtn
