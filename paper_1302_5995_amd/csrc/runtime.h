// Internals of the runtime shared with the serving layer (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/dtn.h"
#include "common.h"

namespace dtn { struct HbsRep; }

struct dtn_op {
  int device = 0;
  int n = 0, nb = 0, leaf = 0;
  double* T = nullptr;              // nb x nb, column-major, owned (device caching allocator); NULL once
                                    // dropped in favour of the HBS factors
  dtn::HbsRep* hbs = nullptr;       // HBS (telescoping) factors of T, if compressed
  dtn::HbsRep* hbsi = nullptr;      // factors of T^{-1} (Section 5.1, Algorithm 1), if inverted
  double* hbs_work = nullptr;       // workspace of the HBS applies (hbs_work_bytes bytes)
  size_t hbs_work_cap = 0;
  hipEvent_t hbs_ev = nullptr;      // orders HBS applies of this handle on different streams
  bool hbs_ev_recorded = false;
  dtn_stats stats{};
  // Schur complements of one quadtree level captured during the build (capture_level)
  double* body = nullptr;           // body loads: F (nb x body_count), column-major, owned
  int body_count = 0;
  double* cap = nullptr;
  std::vector<int> cap_rects;       // 4 ints per box: x0, x1, y0, y1
  std::vector<long long> cap_offs;  // offset of each box's S in cap (ring x ring)
  // split-K apply partial sums (allocated on the first narrow apply); applies of this handle on
  // different streams are ordered through part_ev so they never share the buffer concurrently
  double* part = nullptr;
  hipEvent_t part_ev = nullptr;
  bool part_ev_recorded = false;
  std::mutex part_mu;
};

namespace dtn {

void set_err(const std::string& s);
const std::string& last_err();
int device_ready(int dev);
void* dev_alloc(int dev, size_t bytes);
void dev_release(int dev, void* p);
// Device bytes of the plans a build with this descriptor may allocate: the plan it runs on and,
// for DTN_PIVOT_AUTO, the partial-pivoting plan it falls back to on a weak pivot.  Plans already
// cached on the device count zero.
int plan_footprint(int dev, const dtn_build_desc& D, size_t& bytes);
// HBS form of a handle's operator (hbs.hip).
int hbs_compress(dtn_op* op, double tol, int leaf, hipStream_t s);
// Equal-rank HBS factors of T and the factors of T^{-1} by Algorithm 1 (the forward factors are not kept).
int hbs_invert(dtn_op* op, double tol, int leaf, hipStream_t s);
// The same for an nb x nb device matrix A (ld nb) on device dev: *out owns the inverse factors.
int hbs_invert_matrix(int dev, const double* A, int nb, double tol, int leaf, hipStream_t s, HbsRep** out);
void hbs_rep_free(int dev, HbsRep* H);
// In-place inverses of square blocks (HbsGj jobs on the device, every block in buf) by the HBS inversion's
// Gauss-Jordan kernels: gj_block_class(n) gives the launch class of an n x n block (4, 8, 10: register
// tiles, n <= 160; 0: global memory, n <= 256); a launch holds blocks of one class.
int gj_block_class(int n);
hipError_t launch_gj_blocks(const HbsGj* jobs, int count, int cls, double* buf, DevStatus* st, hipStream_t s);
// X = K^{-1} diag(Z1, Z2) for an i x i device matrix K (ld i) taken in the order src (row r of the
// reordered matrix is row src[r] of K): K(src, src) in equal-rank HBS form, inverted by Algorithm 1,
// applied by Algorithm 2, the result's rows put back in K's order.  Z1 is i1 x e1 (ld i1), Z2 is
// (i - i1) x e2 (ld i - i1), X is i x (e1 + e2) (ld ldx).  Synchronous on s.
int hbs_perm_solve(int dev, const double* K, int i, const std::vector<int>& src, const double* Z1, int i1, int e1,
                   const double* Z2, int e2, double tol, int leaf, double* X, int ldx, hipStream_t s);
void hbs_release(dtn_op* op);
size_t hbs_bytes(const dtn_op* op);   // both representations
size_t hbs_work_bytes(const HbsRep* H, int k);
hipError_t hbs_apply(const HbsRep* H, const double* X, int ldx, int k, double* Y, int ldy, double* work, hipStream_t s);
void hbs_info(const HbsRep* H, dtn_hbs_info* out);
// Apply of op->hbs (Y = T X) or of op->hbsi (Y = T^{-1} X, `inverse`) with the handle's workspace
// (grown on demand, ordered across streams).
int hbs_apply_handle(dtn_op* op, const double* X, int ldx, int k, double* Y, int ldy, hipStream_t s,
                     bool inverse = false);
// The plan-cache key of the plan a build with this descriptor runs on (problem size, leaf,
// convection form, symmetry, pivoting, precision, tol, compressed levels).
std::string plan_cache_key(int dev, const dtn_build_desc& D);

}  // namespace dtn
