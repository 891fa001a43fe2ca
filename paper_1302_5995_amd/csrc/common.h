// Shared plain-old-data structures of the DtN build: written by the host
// planner, read by the gfx950 kernels.  Offsets are in elements of the buffer
// they index; buffers are named by small integer ids and bound to device
// pointers per build through a DevBufs table that lives in device memory.
#pragma once

#include <cstdint>

namespace dtn {

// Buffer ids of the DevBufs table.
enum BufId : int {
  BUF_WS = 0,     // plan workspace (doubles): merge scratch (T_ii / inverse, panels, X, operands)
  BUF_LVA = 1,    // level buffer A (doubles): Schur complements of one quadtree level
  BUF_LVB = 2,    // level buffer B (doubles)
  BUF_HALF = 3,   // half-level buffer (doubles): results of the west+east merges
  BUF_OUT = 4,    // the handle's operator T (nb x nb), written by the final scaling
  BUF_COEF = 5,   // b, c, d fields (3 * n * n doubles, in that order)
  BUF_G = 6,      // apply: right-hand sides
  BUF_Y = 7,      // apply: results
  BUF_AUX = 8,    // plan constants (doubles): Gaussian test matrix and identity of the range finder
  BUF_BODY = 9,   // body loads: condensed right-hand sides of every box holding loads (ring x its loads)
  BUF_BSCR = 10,  // body loads: per-phase scratch (K_ii of small tasks, C_int, K_ei, Z)
  BUF_COUNT = 11
};

struct DevBufs {
  double* p[BUF_COUNT];
};

// Stencil data needed to evaluate entries of the h^2-scaled five-point matrix M'.
struct Coef {
  int n;
  int net;        // 1: network form (b, c hold the conductances of the east and north links)
  int pad0, pad1;
  double h2;      // h^2
  double cs;      // convection coefficient scale: h/2 (centred) or h (paper's printed form)
};

// One dense Schur complement S = K_ee - K_ei K_ii^{-1} K_ie of an (e+i) x (e+i) matrix K
// whose local ordering is [P1; P2; P3; P4] for a merge (P1,P3 on the first child's ring,
// P2,P4 on the second's; e = |P1|+|P2|, i = |P3|+|P4|) or [ring; interior] for a base box.
struct SchurTask {
  int kind;            // 0: base box (all entries from the stencil); 1: pairwise merge
  int e, i;            // exterior (kept) and interior (eliminated) sizes
  int e1, i1;          // merge: |P1|, |P3|; base box: e1 = e, i1 = i
  int m1, m2;          // merge: ring sizes (leading dimensions) of the two children's S
  int idx;             // int-pool offset of cpos[e+i], node[e+i], pmap[e]
  int src, dst;        // buffer ids: children's S (merge), output S
  long long s1, s2;    // element offsets of the children's S in `src`
  long long out;       // element offset of the output S (e x e, leading dimension e) in `dst`
  // the task's problem (a launch may hold tasks of several problems)
  int cn;              // grid size n (nodes per side)
  int sym;             // 1: no convection (b = c = 0), so every K and Schur complement is symmetric
  int net;             // 1: network form: row k is sum over links of sigma (u_k - u_l) + h^2 d u_k, with the
                       //    conductance of link (i,j)-(i+1,j) in b and of (i,j)-(i,j+1) in c
  int pad_net;
  double h2;           // h^2, h = 1/(n-1)
  double cs;           // convection scale: h/2 (centred) or h (the paper's printed form)
  long long coef;      // element offset of the problem's b, c, d fields (3 n^2) in BUF_COEF
};

// Extra data of a merge that goes through the multi-workgroup path
// (explicit inverse of K_ii by blocked Gauss-Jordan, then two batched products).
struct LargeMerge {
  SchurTask t;
  int W;               // Gauss-Jordan panel width
  int piv;             // int-workspace offset: pivots (i ints), then column map (i ints)
  long long inv;       // ws offset: K_ii, overwritten by its row-permuted inverse (i x i, ld i)
  long long q;         // ws offset: panel multipliers Q' (i x W, ld i)
  long long r;         // ws offset: pivot row block R (W x i, ld W)
  long long b31, b42;  // ws offsets: S31 (i1 x e1), S42 (i2 x e2)
  long long a13, a24;  // ws offsets: S13 (e1 x i1), S24 (e2 x i2)
  long long x;         // ws offset: X = K_ii^{-1} K_ie (i x e, ld i)
  long long scale;     // ws offset: one double, max |K_ii| (singularity threshold)
  int kee_gemm;        // 1: K_ee is formed in the Schur product's epilogue (the gather skips it);
                       // 2: besides, the product reads S31, S42 transposed (the gather skips S13, S24)
  int pad;
};

// One product C[rmap(r), cmap(c)] = alpha * sum_k A[r, kmap(k)] B[k, c] + beta * C[...]
// over r < M, c < N (column-major operands).
struct GemmDesc {
  int M, N, K;
  int bufA, bufB, bufC;
  long long offA, offB, offC;
  int lda, ldb, ldc;
  int rmapC, cmapC, kmapA;   // int-pool offsets, or -1 for the identity
  int tiles_m, tiles_n;
  int tile_start;            // first tile index of this descriptor within its launch
  int transA;                // 1: A is stored transposed (A[r, k] at offA + k + r * lda)
  int ksplit;                // > 1: K is cut into ksplit slices, one workgroup each per output tile
  int kcnt;                  // ksplit > 1: int-pool offset of one arrival counter per output tile
  int kee;                   // > 0: C's old values are K_ee of merge kee - 1 (the launch's LargeMerge array),
  int kee_row0;              //   rows kee_row0 + r, columns kee_col0 + c, evaluated from the children
  int kee_col0;              //   (C is not read)
  int tri;                   // 1: square block with rmapC == cmapC: only tiles on or below the diagonal run
  int mirror;                // 1: each entry (r, c) is also written at (c, r) (symmetric result; on diagonal
  int pad2;                  //   tiles the lower half is written and mirrored, so every entry is written once)
  long long kpart;           // ksplit > 1: ws offset of the slices' partial tiles
  double alpha, beta;
};

// One Gram matrix G = Y^T Y (k x k, k <= kPcholMax) factored by pivoted Cholesky with
// truncation; the kernel writes M (k x k) with Y M = orthonormal columns spanning the kept
// directions (columns of M past the rank are zero) and the rank.
struct PcholDesc {
  long long g;               // ws offset of G (ld k)
  long long m;               // ws offset of M (ld k)
  long long dmax;            // ws offset of the block's pass-1 largest diagonal (written in mode 0)
  int k;
  int rank;                  // int-pool slot receiving the rank
  int mode;                  // 0: first pass, 1: residual pass, 2: re-orthogonalisation
  int pad;
  double tol;                // compression tolerance (relative)
};

// One diagonal block inverted in place by the recursive block inversion (one wave per block).
struct BaseBlock {
  long long off;             // ws offset of the block's (0,0) entry
  long long scale;           // ws offset of the merge's max |K_ii|
  int ld;                    // leading dimension (the merge's i)
  int bs;                    // block size (<= kBaseBlock)
};

// Top step of the recursive block inversion of a merge whose K_ii splits at the children's interface
// (h1 = i1): A12 and A21 are then the stencil coupling of the two interface lines, one entry per coupled
// pair of nodes.
struct CoupleDesc {
  long long inv;             // ws offset of K_ii (ld i): X11 at (0, 0), A12, A21 and A22 around it
  long long wb, wc;          // ws offsets of Wb = X11 A12 (h1 x h2, ld h1) and Wc = A21 X11 (h2 x h1, ld h2)
  int i, h1, h2;
  int match;                 // int-pool offset: per second-child interface node, the coupled first-child one or -1
};

// Device status word of a build.
// Body loads (Section 7.3): one task's right-hand-side update (Section 3.2; the leaf's update for a base
// box).  The loads are sorted so that every box's loads are a contiguous range [lo, hi) of columns; the
// box's condensed right-hand sides C (ring x (hi - lo), ld its ring size) are
//   C = C_ext - K_ei K_ii^{-1} C_int,
// C_ext and C_int the rows of [C1 0; 0 C2] (the children's, zero outside their columns) at the exterior
// and interior nodes of the merge, or for a base box the loads themselves (h^2 at the loaded node).
struct BodyJob {
  SchurTask t;               // the task: index maps, children's S, coefficients
  int lo, hi;                // the box's load columns
  int lo1, hi1, lo2, hi2;    // the children's load columns (merges)
  long long c1, c2;          // BUF_BODY offsets of the children's C (ld t.m1, t.m2)
  long long out;             // BUF_BODY offset of the box's C (ld t.e)
  long long kii;             // BUF_BSCR offset of K_ii (i x i), gathered and inverted here; -1: the
                             // merge's inverse in the plan workspace
  long long cint, kei, z;    // BUF_BSCR offsets: C_int (i x cols), K_ei (e x i), Z = K_ii^{-1} C_int
  long long elems;           // elements the gather writes: e cols + i cols + e i (+ i i)
  int bodies;                // offset of the sorted load nodes (node codes) in the job's int array
  int pad;
};

// One square block inverted in place (n x n, ld n) at element offset off of a buffer.
struct HbsGj {
  int buf, n;
  long long off;
};

struct DevStatus {
  int singular;              // set when a pivot falls below DTN_PIVOT_RTOL * scale
  int nonfinite;             // set when a pivot is NaN/Inf
  int weak;                  // unpivoted fast path: a pivot fell below kWeakPivotRtol * scale
  int rank_capped;           // a compressed block kept every column of its residual sketch (rank cap reached)
  unsigned long long min_ratio_bits;   // bits of the smallest |pivot| / scale (positive double)
  unsigned long long max_growth_bits;  // bits of the largest |entry| / scale seen by the 128-block inverses
};

}  // namespace dtn
