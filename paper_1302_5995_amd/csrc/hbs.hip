// Hierarchically block-separable (HBS) form of a built operator T (Section 4) and the telescoping
// apply (tele1-tele3).
//
// Tree (Section 4.2.1): the ring positions [0, nb) split into floor/ceil halves until an interval holds
// at most `leaf` positions; levels count from the root.  Factors (Section 4.3, def1-def6): each leaf tau
// holds D_tau = T(I_tau, I_tau); each node below the root holds a row basis U_tau and a column basis
// V_tau; each parent holds its two sibling blocks.  The paper defers the construction to other work;
// this one uses interpolative decompositions from randomized samples, from the leaves up:
//   * a node's candidate rows R_tau are its positions at a leaf and its children's skeleton rows at a
//     parent; its off-diagonal block row T(R_tau, complement of I_tau) is sampled as
//     Y = (T Omega)(R_tau, :) - T(R_tau, I_tau) Omega(I_tau, :) with a Gaussian Omega (nb x s);
//   * a column-pivoted Householder QR of Y^T, truncated at the first |r_tt| <= tol |r_00|, selects the
//     skeleton rows J_tau and gives U_tau = P [I; (R11^{-1} R12)^T] with T(R_tau, :) ~= U_tau T(J_tau, :)
//     on the complement;
//   * columns the same way from (Omega^T T)(:, C_tau) - Omega(I_tau, :)^T T(I_tau, C_tau);
//   * the sibling blocks are then T(J_s1, J'_s2) and T(J_s2, J'_s1), the leaf blocks T(I, I).
// Apply Y = T X: upward pass xh_tau = V_tau^T x, sibling products, downward pass with U_tau, leaf blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dtn.h"
#include "kernels.h"
#include "runtime.h"

namespace dtn {

constexpr int kHbsSamples = 160;    // random samples per node side (rank cap + oversampling)
constexpr int kHbsMaxRank = 128;    // rank cap of a row or column basis
constexpr int kHbsMaxCand = 2 * kHbsMaxRank;   // candidates of a parent: both children's skeletons
constexpr int kHbsMaxLeaf = 64;     // leaf intervals hold at most this many positions
constexpr int kHbsTile = 32;        // sample kernel: 32 candidates x 32 samples per workgroup

struct HbsTreeNode {
  int lo, hi;       // index interval
  int c1, c2;       // children (-1 at a leaf)
};

// Construction scratch of one node side (side 0: rows, 1: columns).
struct HbsSide {
  int node, side;
};

// One product C[M x N] = op(A)[M x K] B[K x N] (+ beta C) of the apply; N is the apply's column count.
// Buffers: 0 the factors, 1 the input X, 2 the output Y, 3 the workspace of the passes.
struct HbsMm {
  int M, K;
  int bufA, bufB, bufC;
  int transA;        // 1: A[r, k] = stored[k + r * lda]
  long long offA, offB, offC;
  int lda, ldb, ldc; // ldb / ldc < 0: the caller's leading dimension of X / Y
  double beta;
};

// One gathered copy dst[r + c * rows] = src[row(r) + col(c) * ld] of the packing step.
struct HbsCopy {
  int src;           // 0: T, 1: basis scratch
  long long soff;    // element offset in src
  int ld;
  int ridx, cidx;    // int-scratch offsets of row / column index lists, or -1: contiguous
  int rows, cols;
  long long dst;     // element offset in the packed factors
};

struct HbsRep {
  int nb = 0, leaf = 0, depth = 0;
  double tol = 0.0;
  std::vector<HbsTreeNode> nodes;
  std::vector<int> level_of;
  std::vector<int> k, kc;            // row / column ranks per node (root: 0)
  double* fac = nullptr;             // packed factors (of T, or of T^{-1} for an inverse representation)
  size_t fac_doubles = 0;
  HbsMm* d_mm = nullptr;             // apply products, grouped into launches
  std::vector<std::pair<int, int>> launches;   // (first, count) in d_mm
  size_t work_rows = 0;              // workspace rows per apply column (upward and downward passes)
  std::vector<int> level_rank;
  // factor offsets in fac per node (-1: none): bases, leaf blocks, sibling blocks
  std::vector<long long> offU, offV, offD, offB12, offB21;
};

// One block copy dst[r + c dld] = src[r + c sld] of the inversion (buffers: 0 the factors of T,
// 1 the inverse factors, 2 the inversion scratch).
struct HbsBlk {
  int src, dst;
  long long soff, doff;
  int sld, dld, rows, cols;
};

// HbsGj (common.h): one square matrix inverted in place (n x n, ld n) in buffer `buf` (1 or 2, as in HbsBlk).
constexpr int kHbsGjMax = 2 * kHbsMaxRank;   // largest block the inversion kernel takes
constexpr int kHbsIdCols = 4;   // columns a wave reflects together in the ID kernel
constexpr int kHbsIdThreads = 512;   // threads of an ID workgroup (eight waves share the reflections)
// register tile (rows and columns per thread) of the register-resident inversion for an n x n block,
// or 0 for the global-memory kernel
static inline int gj_class(int n) { return n <= 64 ? 4 : n <= 128 ? 8 : n <= 160 ? 10 : 0; }

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Candidate c of node `nd` on side `side`: its own position at a leaf, else the children's skeletons.
__device__ inline int hbs_cand(const HbsTreeNode* nodes, const int* skel, const int* cnt, int nd, int side, int c) {
  const HbsTreeNode t = nodes[nd];
  if (t.c1 < 0) return t.lo + c;
  const int k1 = cnt[2 * t.c1 + side];
  return c < k1 ? skel[(2 * t.c1 + side) * kHbsMaxRank + c] : skel[(2 * t.c2 + side) * kHbsMaxRank + (c - k1)];
}

__device__ inline int hbs_ncand(const HbsTreeNode* nodes, const int* cnt, int nd, int side) {
  const HbsTreeNode t = nodes[nd];
  return t.c1 < 0 ? t.hi - t.lo : cnt[2 * t.c1 + side] + cnt[2 * t.c2 + side];
}

// Samples of the off-diagonal block row (side 0) or column (side 1) of one node:
//   side 0: Y[c, s] = Z[cand c, s] - sum_{j in I} T[cand c, j] Om[j, s]        (Z = T Om, nb x S)
//   side 1: Y[c, s] = Zt[s, cand c] - sum_{j in I} T[j, cand c] Om[j, s]      (Zt = Om^T T, S x nb)
// stored as Y^T: ybuf[slot * S * kHbsMaxCand + s + c * S].  Block (slot, candidate tile, sample tile).
// joint: the two sides of a node (consecutive entries of `sides`) share one slot, rows 0..S-1 the
// block row's samples and S..2S-1 the block column's: ybuf[node slot * 2S * kHbsMaxCand + side S + s
// + c * 2S].
// The Gaussian test matrix Om (nb x S, column-major) and its transpose: standard normal numbers from
// splitmix64 (Steele, Lea and Flood) taken as a counter-based generator (output q is the mix of
// seed + (q + 1) * 0x9e3779b97f4a7c15) driving the Box-Muller transform, entries 2m and 2m + 1 of Om in
// column-major order from outputs 2m and 2m + 1.
__device__ __forceinline__ unsigned long long splitmix_at(unsigned long long seed, unsigned long long q) {
  unsigned long long z = seed + (q + 1ULL) * 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_hbs_gauss(double* __restrict__ om, double* __restrict__ omt, int nb, int S,
                                                   unsigned long long seed) {
  const long long tot = (long long)nb * S, pairs = (tot + 1) / 2;
  for (long long m = blockIdx.x * 256LL + threadIdx.x; m < pairs; m += (long long)gridDim.x * 256) {
    const double u1 = ((splitmix_at(seed, 2 * m) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (splitmix_at(seed, 2 * m + 1) >> 11) * (1.0 / 9007199254740992.0);
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    const double g[2] = {r * cs, r * sn};
    for (int h = 0; h < 2; ++h) {
      const long long e = 2 * m + h;
      if (e >= tot) break;
      const int j = (int)(e % nb), c = (int)(e / nb);
      om[e] = g[h];
      omt[c + (long long)j * S] = g[h];
    }
  }
}

__global__ __launch_bounds__(256) void k_hbs_sample(const HbsSide* __restrict__ sides, const HbsTreeNode* __restrict__ nodes,
                                                    const int* __restrict__ skel, const int* __restrict__ cnt,
                                                    const double* __restrict__ T, int nb, const double* __restrict__ Om,
                                                    const double* __restrict__ Z, const double* __restrict__ Zt,
                                                    double* __restrict__ ybuf, int joint) {
  __shared__ double Ts[kHbsTile][kHbsTile + 1];   // [candidate][j]
  __shared__ double Os[kHbsTile][kHbsTile + 1];   // [j][sample]
  __shared__ int cand[kHbsTile];
  const HbsSide sd = sides[blockIdx.x];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.y * kHbsTile, s0 = blockIdx.z * kHbsTile;
  const int p = hbs_ncand(nodes, cnt, sd.node, sd.side);
  if (c0 >= p) return;
  const HbsTreeNode t = nodes[sd.node];
  if (tid < kHbsTile) cand[tid] = c0 + tid < p ? hbs_cand(nodes, skel, cnt, sd.node, sd.side, c0 + tid) : 0;
  __syncthreads();
  // four outputs per thread: candidate cc, samples ss .. ss + 3 * 8
  const int cc = tid % kHbsTile, sq = tid / kHbsTile;   // sq in 0..7
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j0 = t.lo; j0 < t.hi; j0 += kHbsTile) {
    __syncthreads();
    for (int x = tid; x < kHbsTile * kHbsTile; x += 256) {
      const int a = x % kHbsTile, b = x / kHbsTile;   // a fastest
      const int j = j0 + b;
      // side 0: Ts[a][b] = T[cand a, j] (reads stride nb along a); side 1: T[j, cand a]
      double tv = 0.0;
      if (j < t.hi && c0 + a < p)
        tv = sd.side == 0 ? T[cand[a] + (long long)j * nb] : T[j + (long long)cand[a] * nb];
      Ts[a][b] = tv;
      const int jj = j0 + a, ss = s0 + b;
      Os[a][b] = (jj < t.hi) ? Om[jj + (long long)ss * nb] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int b = 0; b < kHbsTile; ++b) {
      const double tv = Ts[cc][b];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = fma(tv, Os[b][sq + 8 * q], acc[q]);
    }
  }
  if (c0 + cc < p) {
    const int ld = joint ? 2 * kHbsSamples : kHbsSamples;
    const long long base = joint ? (long long)(blockIdx.x >> 1) * ld * kHbsMaxCand + sd.side * kHbsSamples
                                 : (long long)blockIdx.x * ld * kHbsMaxCand;
    for (int q = 0; q < 4; ++q) {
      const int s = s0 + sq + 8 * q;
      const double z = sd.side == 0 ? Z[cand[cc] + (long long)s * nb] : Zt[s + (long long)cand[cc] * kHbsSamples];
      ybuf[base + s + (long long)(c0 + cc) * ld] = z - acc[q];
    }
  }
}

// Interpolative decomposition of one node side from its samples (one workgroup): column-pivoted
// Householder QR of Y^T (SX x p, column c = candidate c), truncated at the first |r_tt| <= tol |r_00|
// (or at kHbsMaxRank: then st->rank_capped is raised when the next column is still above the
// threshold).  JOINT (SX = 2S): one workgroup per node on the stacked samples of its block row and block
// column, so that one skeleton set and one interpolation matrix serve both sides (equal ranks, U = V).
// Works in place on the samples in global memory (at most SX x 256 doubles, L2-resident).  A step is two
// phases: wave 0 picks the pivot column, swaps it into place and forms its Householder vector from
// registers; then each wave reflects whole columns held in registers (lanes over the rows), writes them
// once and leaves their squared norms below the next row for the next pivot choice, so the trailing
// columns are read and written once per step.  Writes the skeleton positions, the rank and the basis
// (p x k, column-major, ld kHbsMaxCand) of the side, or of both sides.
template <int SX, bool JOINT>
__global__ __launch_bounds__(kHbsIdThreads) void k_hbs_id(const HbsSide* __restrict__ sides, const HbsTreeNode* __restrict__ nodes,
                                                int* __restrict__ skel, int* __restrict__ cnt, double* __restrict__ ybuf,
                                                double* __restrict__ basis, double tol, DevStatus* __restrict__ st) {
  constexpr int R = (SX + 63) / 64;   // rows per lane
  __shared__ double v[SX];
  __shared__ double nrm[kHbsMaxCand];
  __shared__ int perm[kHbsMaxCand];
  __shared__ int s_stop;
  __shared__ double s_beta;
  const HbsSide sd = sides[JOINT ? 2 * blockIdx.x : blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = hbs_ncand(nodes, cnt, sd.node, sd.side);
  double* A = ybuf + (long long)blockIdx.x * SX * kHbsMaxCand;     // SX x p, column-major
  constexpr int NW = kHbsIdThreads / 64;
  for (int j = tid; j < p; j += kHbsIdThreads) perm[j] = j;
  for (int j = wave; j < p; j += NW) {
    double s2 = 0.0;
    for (int i = lane; i < SX; i += 64) s2 = fma(A[i + j * SX], A[i + j * SX], s2);
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
    if (lane == 0) nrm[j] = s2;
  }
  if (tid == 0) s_stop = 0;
  __syncthreads();
  const int tmax = min(min(p, SX), kHbsMaxRank);
  double r00 = 0.0;   // |r_00|, kept by wave 0
  int t = 0;
  for (;; ++t) {
    if (wave == 0) {
      double best = -1.0;
      int bi = t;
      for (int j = t + lane; j < p; j += 64)
        if (nrm[j] > best) { best = nrm[j]; bi = j; }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      const double r = sqrt(fmax(best, 0.0));
      if (t == 0) r00 = r;
      const bool done = t >= p || best <= 0.0 || r <= tol * r00;
      if (done || t == tmax) {
        if (lane == 0) {
          s_stop = 1;
          if (!done) atomicOr(&st->rank_capped, 1);   // the basis is full and a column above the threshold remains
        }
      } else {
        // the pivot column bi becomes column t (whole columns, rows 0 .. SX-1)
        double ct[R], cb[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = lane + 64 * q;
          ct[q] = i < SX ? A[i + t * SX] : 0.0;
          cb[q] = (i < SX && bi != t) ? A[i + bi * SX] : ct[q];
        }
        if (bi != t) {
#pragma unroll
          for (int q = 0; q < R; ++q) {
            const int i = lane + 64 * q;
            if (i < SX) A[i + bi * SX] = ct[q];
          }
          if (lane == 0) {
            const int pq = perm[t];
            perm[t] = perm[bi];
            perm[bi] = pq;
            nrm[bi] = nrm[t];
          }
        }
        // Householder vector of the new column t (rows t .. SX-1)
        double s2 = 0.0, x0 = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = lane + 64 * q;
          if (i >= t && i < SX) s2 = fma(cb[q], cb[q], s2);
          if (q == (t >> 6)) x0 = cb[q];
        }
        for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
        x0 = __shfl(x0, t & 63);
        const double alpha = x0 >= 0.0 ? -sqrt(s2) : sqrt(s2);
        const double v0 = x0 - alpha;
        const double vn2 = s2 - x0 * x0 + v0 * v0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = lane + 64 * q;
          if (i < SX) {
            if (i > t) v[i] = cb[q];
            if (i == t) { v[i] = v0; cb[q] = alpha; }
            A[i + t * SX] = cb[q];
          }
        }
        if (lane == 0) s_beta = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      }
    }
    __syncthreads();
    if (s_stop) break;
    const double beta = s_beta;
    // reflect the columns right of t, each wave kHbsIdCols columns at a time held in registers (their
    // loads and reductions in flight together); their norms below row t+1
    double vi[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = lane + 64 * q;
      vi[q] = (i >= t && i < SX) ? v[i] : 0.0;
    }
    for (int jb = t + 1 + wave * kHbsIdCols; jb < p; jb += NW * kHbsIdCols) {
      double a[kHbsIdCols][R], w[kHbsIdCols], s2[kHbsIdCols];
#pragma unroll
      for (int u = 0; u < kHbsIdCols; ++u) {
        const int j = jb + u;
        w[u] = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = lane + 64 * q;
          a[u][q] = (j < p && i >= t && i < SX) ? A[i + j * SX] : 0.0;
          w[u] = fma(vi[q], a[u][q], w[u]);
        }
      }
      for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int u = 0; u < kHbsIdCols; ++u) w[u] += __shfl_xor(w[u], o);
#pragma unroll
      for (int u = 0; u < kHbsIdCols; ++u) {
        const int j = jb + u;
        const double wb = w[u] * beta;
        s2[u] = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = lane + 64 * q;
          if (j < p && i >= t && i < SX) {
            a[u][q] = fma(-wb, vi[q], a[u][q]);
            A[i + j * SX] = a[u][q];
            if (i > t) s2[u] = fma(a[u][q], a[u][q], s2[u]);
          }
        }
      }
      for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int u = 0; u < kHbsIdCols; ++u) s2[u] += __shfl_xor(s2[u], o);
      if (lane == 0)
#pragma unroll
        for (int u = 0; u < kHbsIdCols; ++u)
          if (jb + u < p) nrm[jb + u] = s2[u];
    }
    __syncthreads();
  }
  const int k = t;
  // X = R11^{-1} R12 by back substitution, one column of R12 per thread (R12 overwritten by X)
  for (int j = k + tid; j < p; j += kHbsIdThreads) {
    for (int r = k - 1; r >= 0; --r) {
      double x = A[r + j * SX];
      for (int q = r + 1; q < k; ++q) x = fma(-A[r + q * SX], A[q + j * SX], x);
      A[r + j * SX] = x / A[r + r * SX];
    }
  }
  __syncthreads();
  // basis rows: candidate perm[q] gets e_q for q < k and X(:, q) for q >= k
  for (int side = JOINT ? 0 : sd.side; side <= (JOINT ? 1 : sd.side); ++side) {
    const int slot = 2 * sd.node + side;
    double* U = basis + (long long)slot * kHbsMaxCand * kHbsMaxRank;
    for (int x = tid; x < p * k; x += kHbsIdThreads) {
      const int q = x % p, c = x / p;
      const double val = q < k ? (q == c ? 1.0 : 0.0) : A[c + q * SX];
      U[perm[q] + (long long)c * kHbsMaxCand] = val;
    }
    if (tid < k) skel[slot * kHbsMaxRank + tid] = hbs_cand(nodes, skel, cnt, sd.node, sd.side, perm[tid]);
  }
  __syncthreads();
  if (tid == 0) {
    cnt[2 * sd.node + sd.side] = k;
    if (JOINT) cnt[2 * sd.node + 1] = k;
  }
}

__global__ __launch_bounds__(256) void k_hbs_blk(const HbsBlk* __restrict__ jobs, const double* fac, double* ifac,
                                                 double* scr) {
  const HbsBlk j = jobs[blockIdx.x];
  const double* S = (j.src == 0 ? fac : j.src == 1 ? (const double*)ifac : (const double*)scr) + j.soff;
  double* D = (j.dst == 1 ? ifac : scr) + j.doff;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < j.cols; c += 4)
    for (int r = lane; r < j.rows; r += 64) D[r + (long long)c * j.dld] = S[r + (long long)c * j.sld];
}

// In-place inverse of one n x n block (n <= kHbsGjMax) by Gauss-Jordan elimination with partial
// (row) pivoting, one workgroup per block, the matrix in global memory (L2-resident at these sizes).
// Step t: the row with the largest |a_it| (i >= t) is swapped into row t; row t becomes
// (row t with a_tt replaced by 1) / a_tt and every other row i loses a_it times it (its column-t entry
// starting from 0), so that the stored matrix holds the inverse's columns for the eliminated
// positions.  At the end the row interchanges are undone as column interchanges, last first.  A
// zero or non-finite pivot raises st->singular.
__global__ __launch_bounds__(256) void k_hbs_gj(const HbsGj* __restrict__ jobs, double* ifac, double* scr,
                                                DevStatus* __restrict__ st) {
  __shared__ double rowv[kHbsGjMax];
  __shared__ double colv[kHbsGjMax];
  __shared__ int piv[kHbsGjMax];
  __shared__ int s_p;
  const HbsGj j = jobs[blockIdx.x];
  const int n = j.n;
  if (n <= 0 || n > kHbsGjMax) return;
  double* A = (j.buf == 1 ? ifac : scr) + j.off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int t = 0; t < n; ++t) {
    if (wave == 0) {
      double best = -1.0;
      int bi = t;
      for (int i = t + lane; i < n; i += 64) {
        const double v = fabs(A[i + (long long)t * n]);
        if (v > best) { best = v; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        if (!(best > 0.0) || !isfinite(best)) atomicOr(&st->singular, 1);
        s_p = bi;
        piv[t] = bi;
      }
    }
    __syncthreads();
    const int pr = s_p;
    if (pr != t)
      for (int c = tid; c < n; c += 256) {
        const double a = A[t + (long long)c * n];
        A[t + (long long)c * n] = A[pr + (long long)c * n];
        A[pr + (long long)c * n] = a;
      }
    __syncthreads();
    const double pv = A[t + (long long)t * n];
    const double ipv = pv != 0.0 ? 1.0 / pv : 0.0;
    for (int c = tid; c < n; c += 256) rowv[c] = (c == t ? 1.0 : A[t + (long long)c * n]) * ipv;
    for (int i = tid; i < n; i += 256) colv[i] = i == t ? 0.0 : A[i + (long long)t * n];
    __syncthreads();
    for (int c = wave; c < n; c += 4) {
      const double rc = rowv[c];
      double* Ac = A + (long long)c * n;
      for (int i = lane; i < n; i += 64) {
        const double a = c == t ? 0.0 : Ac[i];
        Ac[i] = i == t ? rc : fma(-colv[i], rc, a);
      }
    }
    __syncthreads();
  }
  for (int t = n - 1; t >= 0; --t) {
    const int pr = piv[t];
    if (pr != t)
      for (int i = tid; i < n; i += 256) {
        const double a = A[i + (long long)t * n];
        A[i + (long long)t * n] = A[i + (long long)pr * n];
        A[i + (long long)pr * n] = a;
      }
    __syncthreads();
  }
}

// The same inverse with the block held in registers, for n <= 16 K: a 16 x 16 grid of threads, thread
// (tr, tc) holding rows tr + 16 x and columns tc + 16 y (x, y < K), so that each step costs K^2 FMAs per
// thread and two barriers.  Rows are not moved: step t takes as pivot the largest |a_it| among the rows
// not yet used (partial pivoting by row choice), so the stored matrix ends as the inverse with its rows
// and columns permuted: entry (i, c) of the result is entry (step at which row i was the pivot, pivot row
// of step c) of the inverse, which the final stores put in place.  A zero or non-finite pivot raises
// st->singular.
template <int K>
__global__ __launch_bounds__(256) void k_hbs_gjr(const HbsGj* __restrict__ jobs, double* ifac, double* scr,
                                                 DevStatus* __restrict__ st) {
  constexpr int NM = 16 * K;
  __shared__ double colb[2][NM];     // column t of the step (all rows), double-buffered
  __shared__ double rowb[2][NM];     // the pivot row (all columns)
  __shared__ int s_piv[2];
  __shared__ int rowof[NM];          // pivot row of each step
  __shared__ int stepof[NM];         // step at which each row was the pivot
  const HbsGj jb = jobs[blockIdx.x];
  const int n = jb.n;
  if (n <= 0 || n > NM) return;
  double* A = (jb.buf == 1 ? ifac : scr) + jb.off;
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;   // a column group's 16 threads are adjacent lanes
  double a[K][K];
#pragma unroll
  for (int x = 0; x < K; ++x)
#pragma unroll
    for (int y = 0; y < K; ++y) {
      const int i = tr + 16 * x, c = tc + 16 * y;
      a[x][y] = (i < n && c < n) ? A[i + (long long)c * n] : 0.0;
    }
  unsigned used = 0;   // bit x: row tr + 16 x already taken (or past n)
#pragma unroll
  for (int x = 0; x < K; ++x)
    if (tr + 16 * x >= n) used |= 1u << x;
  for (int t = 0; t < n; ++t) {
    const int b = t & 1, yt = t >> 4;
    if (tc == (t & 15)) {
      // publish column t and choose its pivot among the unused rows
      double best = -1.0;
      int bi = -1;
#pragma unroll
      for (int y = 0; y < K; ++y)
        if (y == yt) {
#pragma unroll
          for (int x = 0; x < K; ++x) {
            const double v = a[x][y];
            colb[b][tr + 16 * x] = v;
            if (!((used >> x) & 1u) && fabs(v) > best) { best = fabs(v); bi = tr + 16 * x; }
          }
        }
      for (int o = 8; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 16);
        const int oi = __shfl_xor(bi, o, 16);
        if (ob > best || (ob == best && oi >= 0 && (bi < 0 || oi < bi))) { best = ob; bi = oi; }
      }
      if (tr == 0) {
        if (!(best > 0.0) || !isfinite(best) || bi < 0) {
          atomicOr(&st->singular, 1);
          if (bi < 0) bi = t;   // unreachable for n <= NM: an unused row always remains
        }
        s_piv[b] = bi;
        rowof[t] = bi;
        stepof[bi] = t;
      }
    }
    __syncthreads();
    const int r = s_piv[b], xr = r >> 4;
    const bool own_row = tr == (r & 15);
    if (own_row) {
#pragma unroll
      for (int x = 0; x < K; ++x)
        if (x == xr) {
#pragma unroll
          for (int y = 0; y < K; ++y) rowb[b][tc + 16 * y] = a[x][y];
        }
      used |= 1u << xr;
    }
    __syncthreads();
    const double pv = colb[b][r];
    const double ipv = pv != 0.0 ? 1.0 / pv : 0.0;
    double rs[K], ci[K];
#pragma unroll
    for (int y = 0; y < K; ++y) {
      const int c = tc + 16 * y;
      rs[y] = (c == t ? 1.0 : rowb[b][c]) * ipv;
    }
#pragma unroll
    for (int x = 0; x < K; ++x) ci[x] = colb[b][tr + 16 * x];
    // column t starts from 0; the pivot row becomes rs: zero it and take ci = -1 there
#pragma unroll
    for (int y = 0; y < K; ++y)
      if (y == yt && tc == (t & 15)) {
#pragma unroll
        for (int x = 0; x < K; ++x) a[x][y] = 0.0;
      }
#pragma unroll
    for (int x = 0; x < K; ++x)
      if (x == xr && own_row) {
        ci[x] = -1.0;
#pragma unroll
        for (int y = 0; y < K; ++y) a[x][y] = 0.0;
      }
#pragma unroll
    for (int x = 0; x < K; ++x)
#pragma unroll
      for (int y = 0; y < K; ++y) a[x][y] = fma(-ci[x], rs[y], a[x][y]);
  }
  __syncthreads();
#pragma unroll
  for (int x = 0; x < K; ++x)
#pragma unroll
    for (int y = 0; y < K; ++y) {
      const int i = tr + 16 * x, c = tc + 16 * y;
      if (i < n && c < n) A[stepof[i] + (long long)rowof[c] * n] = a[x][y];
    }
}

__global__ __launch_bounds__(256) void k_hbs_pack(const HbsCopy* __restrict__ jobs, const double* __restrict__ T,
                                                  const double* __restrict__ basis, const int* __restrict__ iws,
                                                  double* __restrict__ fac) {
  const HbsCopy jb = jobs[blockIdx.x];
  const double* src = jb.src == 0 ? T : basis;
  const long long tot = (long long)jb.rows * jb.cols;
  for (long long x = threadIdx.x; x < tot; x += 256) {
    const int r = (int)(x % jb.rows), c = (int)(x / jb.rows);
    const long long rr = jb.ridx >= 0 ? iws[jb.ridx + r] : r;
    const long long ci = jb.cidx >= 0 ? iws[jb.cidx + c] : c;
    fac[jb.dst + x] = src[jb.soff + rr + ci * jb.ld];
  }
}

// Products of one apply step: block (product, 32-column chunk).  The chunk of B (K x 32) goes through
// LDS 64 rows of K at a time; wave w computes columns 8w .. 8w+7 of C for all M rows (lanes over the
// rows, up to four rows per lane), so each A element loaded feeds eight FMAs and each B element is an
// LDS broadcast.  Chunks of at most 8 columns (latency-bound narrow applies) take one output per thread.
__global__ __launch_bounds__(256) void k_hbs_mm(const HbsMm* __restrict__ mm, int N, const double* __restrict__ fac,
                                                const double* __restrict__ X, int ldx, double* __restrict__ Y, int ldy,
                                                double* __restrict__ W, int ldw) {
  constexpr int KC = 64, MR = kHbsMaxCand / 64;
  __shared__ double Bs[KC][32];
  const HbsMm d = mm[blockIdx.x];
  const int c0 = blockIdx.y * 32;
  if (c0 >= N || d.M <= 0) return;
  const int nc = min(32, N - c0);
  auto base = [&](int buf) -> const double* {
    return buf == 0 ? fac : buf == 1 ? X : buf == 2 ? Y : W;
  };
  auto ldof = [&](int buf, int ld) { return ld >= 0 ? ld : (buf == 1 ? ldx : buf == 2 ? ldy : ldw); };
  const double* A = base(d.bufA) + d.offA;
  const double* B = base(d.bufB) + d.offB + (long long)c0 * ldof(d.bufB, d.ldb);
  double* C = (d.bufC == 2 ? Y : W) + d.offC + (long long)c0 * ldof(d.bufC, d.ldc);
  const int ldb = ldof(d.bufB, d.ldb), ldc = ldof(d.bufC, d.ldc);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, cw = wave * 8;
  if (nc <= 8) {
    // narrow applies (a few columns): one output per thread, the K loop straight from memory
    for (int o = tid; o < d.M * nc; o += 256) {
      const int r = o % d.M, c = o / d.M;
      double acc = 0.0;
      if (d.transA) {
        for (int k = 0; k < d.K; ++k) acc = fma(A[k + (long long)r * d.lda], B[k + (long long)c * ldb], acc);
      } else {
        for (int k = 0; k < d.K; ++k) acc = fma(A[r + (long long)k * d.lda], B[k + (long long)c * ldb], acc);
      }
      double* cp = C + r + (long long)c * ldc;
      *cp = d.beta != 0.0 ? fma(d.beta, *cp, acc) : acc;
    }
    return;
  }
  double acc[MR][8];
#pragma unroll
  for (int m = 0; m < MR; ++m)
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) acc[m][cc] = 0.0;
  for (int k0 = 0; k0 < d.K; k0 += KC) {
    const int kc = min(KC, d.K - k0);
    for (int x = tid; x < KC * 32; x += 256) {
      const int kk = x % KC, c = x / KC;
      Bs[kk][c] = (kk < kc && c < nc) ? B[k0 + kk + (long long)c * ldb] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < kc; ++kk) {
      double b[8];
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) b[cc] = Bs[kk][cw + cc];
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int r = lane + 64 * m;
        if (64 * m < d.M) {
          const long long ai = d.transA ? (k0 + kk) + (long long)r * d.lda : r + (long long)(k0 + kk) * d.lda;
          const double a = r < d.M ? A[ai] : 0.0;
#pragma unroll
          for (int cc = 0; cc < 8; ++cc) acc[m][cc] = fma(a, b[cc], acc[m][cc]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const int r = lane + 64 * m;
    if (r < d.M)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int c = cw + cc;
        if (c < nc) {
          double* cp = C + r + (long long)c * ldc;
          *cp = d.beta != 0.0 ? fma(d.beta, *cp, acc[m][cc]) : acc[m][cc];
        }
      }
  }
}

// ---------------------------------------------------------------------------
// Host
// ---------------------------------------------------------------------------

#define HBSCHK(expr, code)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      set_err(std::string(#expr) + " failed: " + hipGetErrorString(e_));                   \
      return code;                                                                          \
    }                                                                                       \
  } while (0)

// Every apply product fits k_hbs_mm: at most kHbsMaxCand rows (four per lane).
static bool mm_shapes_ok(const std::vector<HbsMm>& mm) {
  for (const HbsMm& d : mm)
    if (d.M > kHbsMaxCand || d.M < 0 || d.K < 0) return false;
  return true;
}

// Scratch allocations of one construction, released on every exit path once the work queued on the
// stream has finished (a released block may be handed to another thread's stream at once).
struct DevScratch {
  int dev;
  hipStream_t s;
  std::vector<void*> ptrs;
  DevScratch(int d, hipStream_t st) : dev(d), s(st) {}
  void* get(size_t bytes) {
    void* p = dev_alloc(dev, std::max<size_t>(bytes, 256));
    if (p) ptrs.push_back(p);
    return p;
  }
  ~DevScratch() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(s);
    for (void* p : ptrs) dev_release(dev, p);
  }
};

static void rep_free(int dev, HbsRep* H) {
  if (!H) return;
  dev_release(dev, H->fac);
  dev_release(dev, H->d_mm);
  delete H;
}

void hbs_release(dtn_op* op) {
  if (!op) return;
  rep_free(op->device, op->hbs);
  op->hbs = nullptr;
  rep_free(op->device, op->hbsi);
  op->hbsi = nullptr;
}

static void build_tree(int nb, int leaf, std::vector<HbsTreeNode>& nodes, std::vector<int>& level, int& depth) {
  nodes.clear();
  level.clear();
  nodes.push_back({0, nb, -1, -1});
  level.push_back(0);
  for (size_t q = 0; q < nodes.size(); ++q) {
    const int lo = nodes[q].lo, hi = nodes[q].hi;
    if (hi - lo > leaf) {
      const int mid = lo + (hi - lo) / 2;
      nodes[q].c1 = (int)nodes.size();
      nodes.push_back({lo, mid, -1, -1});
      level.push_back(level[q] + 1);
      nodes[q].c2 = (int)nodes.size();
      nodes.push_back({mid, hi, -1, -1});
      level.push_back(level[q] + 1);
    }
  }
  depth = *std::max_element(level.begin(), level.end());
}

// HBS factors of the handle's T at tolerance tol.  With `square` each node takes one skeleton set and one
// interpolation matrix for its block row and block column together (the ID of both sides' stacked
// samples), so that its ranks are equal and U = V, as the inversion of Section 5.1 needs (separate
// skeletons with ranks raised to the larger one leave V^T Dt^{-1} U nearly singular on convection
// problems).  On success *out owns the factors and the forward-apply products.
static int hbs_construct(int dev, const double* A, int nb, double tol, int leaf, bool square, hipStream_t s,
                         HbsRep** out) {
  *out = nullptr;
  if (!(tol > 0.0) || !std::isfinite(tol)) { set_err("hbs: tol must be finite and > 0"); return DTN_EINVAL; }
  if (leaf < 8 || leaf > kHbsMaxLeaf) { set_err("hbs: leaf must be in [8, 64]"); return DTN_EINVAL; }
  if (!A) { set_err("hbs: no dense matrix to compress"); return DTN_EINVAL; }
  auto H = std::make_unique<HbsRep>();
  H->nb = nb;
  H->leaf = leaf;
  H->tol = tol;
  build_tree(nb, leaf, H->nodes, H->level_of, H->depth);
  const int nn = (int)H->nodes.size();
  DevScratch sc(dev, s);
  const int S = kHbsSamples;
  HbsTreeNode* d_nodes = (HbsTreeNode*)sc.get(nn * sizeof(HbsTreeNode));
  int* d_int = (int*)sc.get((size_t)(2 * nn * kHbsMaxRank + 2 * nn) * sizeof(int));
  double* d_om = (double*)sc.get((size_t)nb * S * sizeof(double));
  double* d_omt = (double*)sc.get((size_t)nb * S * sizeof(double));
  double* d_z = (double*)sc.get((size_t)nb * S * sizeof(double));
  double* d_zt = (double*)sc.get((size_t)nb * S * sizeof(double));
  double* d_basis = (double*)sc.get((size_t)2 * nn * kHbsMaxCand * kHbsMaxRank * sizeof(double));
  DevStatus* d_st = (DevStatus*)sc.get(sizeof(DevStatus));
  if (!d_nodes || !d_int || !d_om || !d_omt || !d_z || !d_zt || !d_basis || !d_st) {
    set_err("hbs: device allocation failed (construction scratch)");
    return DTN_ENOMEM;
  }
  int* d_skel = d_int;
  int* d_cnt = d_int + 2 * nn * kHbsMaxRank;
  HBSCHK(hipMemcpyAsync(d_nodes, H->nodes.data(), nn * sizeof(HbsTreeNode), hipMemcpyHostToDevice, s), DTN_EDEVICE);
  HBSCHK(hipMemsetAsync(d_int, 0, (size_t)(2 * nn * kHbsMaxRank + 2 * nn) * sizeof(int), s), DTN_EDEVICE);
  HBSCHK(hipMemsetAsync(d_st, 0, sizeof(DevStatus), s), DTN_EDEVICE);
  {
    const long long pairs = ((long long)nb * S + 1) / 2;
    hipLaunchKernelGGL(k_hbs_gauss, dim3((unsigned)std::min<long long>(2048, (pairs + 255) / 256)), dim3(256), 0, s,
                       d_om, d_omt, nb, S, 0x48425321ULL + (uint64_t)nb);
    HBSCHK(hipGetLastError(), DTN_EDEVICE);
  }
  // Z = T Om (nb x S), Zt = Om^T T (S x nb) on the MFMA GEMM
  {
    DevBufs B{};
    B.p[BUF_OUT] = const_cast<double*>(A);
    B.p[BUF_G] = d_om;
    B.p[BUF_Y] = d_z;
    GemmDesc g{};
    g.M = nb; g.N = S; g.K = nb;
    g.bufA = BUF_OUT; g.bufB = BUF_G; g.bufC = BUF_Y;
    g.lda = nb; g.ldb = nb; g.ldc = nb;
    g.rmapC = g.cmapC = g.kmapA = -1;
    g.alpha = 1.0; g.beta = 0.0;
    HBSCHK(launch_gemm_single(g, 0, B, s), DTN_EDEVICE);
    DevBufs B2{};
    B2.p[BUF_OUT] = d_omt;
    B2.p[BUF_G] = const_cast<double*>(A);
    B2.p[BUF_Y] = d_zt;
    GemmDesc g2 = g;
    g2.M = S; g2.N = nb; g2.K = nb;
    g2.lda = S; g2.ldb = nb; g2.ldc = S;
    HBSCHK(launch_gemm_single(g2, 0, B2, s), DTN_EDEVICE);
  }
  // levels from the leaves up; each level's node sides in one launch of each kernel
  std::vector<HbsSide> sides;
  std::vector<std::pair<int, int>> lev_range;
  for (int lev = H->depth; lev >= 1; --lev) {
    const int first = (int)sides.size();
    for (int q = 0; q < nn; ++q)
      if (H->level_of[q] == lev) { sides.push_back({q, 0}); sides.push_back({q, 1}); }
    lev_range.push_back({first, (int)sides.size() - first});
  }
  size_t max_level_sides = 0;
  for (auto& r : lev_range) max_level_sides = std::max(max_level_sides, (size_t)r.second);
  HbsSide* d_sides = (HbsSide*)sc.get(std::max<size_t>(1, sides.size()) * sizeof(HbsSide));
  double* d_y = (double*)sc.get(std::max<size_t>(1, max_level_sides) * S * kHbsMaxCand * sizeof(double));
  if (!d_sides || !d_y) { set_err("hbs: device allocation failed (samples)"); return DTN_ENOMEM; }
  if (!sides.empty())
    HBSCHK(hipMemcpyAsync(d_sides, sides.data(), sides.size() * sizeof(HbsSide), hipMemcpyHostToDevice, s), DTN_EDEVICE);
  for (auto& r : lev_range) {
    const dim3 grid(r.second, kHbsMaxCand / kHbsTile, S / kHbsTile);
    hipLaunchKernelGGL(k_hbs_sample, grid, dim3(256), 0, s, d_sides + r.first, d_nodes, d_skel, d_cnt, A, nb,
                       d_om, d_z, d_zt, d_y, square ? 1 : 0);
    HBSCHK(hipGetLastError(), DTN_EDEVICE);
    if (square)
      hipLaunchKernelGGL((k_hbs_id<2 * kHbsSamples, true>), dim3(r.second / 2), dim3(kHbsIdThreads), 0, s, d_sides + r.first,
                         d_nodes, d_skel, d_cnt, d_y, d_basis, tol, d_st);
    else
      hipLaunchKernelGGL((k_hbs_id<kHbsSamples, false>), dim3(r.second), dim3(kHbsIdThreads), 0, s, d_sides + r.first, d_nodes,
                         d_skel, d_cnt, d_y, d_basis, tol, d_st);
    HBSCHK(hipGetLastError(), DTN_EDEVICE);
  }
  std::vector<int> cnt(2 * nn);
  DevStatus hs{};
  HBSCHK(hipMemcpyAsync(cnt.data(), d_cnt, cnt.size() * sizeof(int), hipMemcpyDeviceToHost, s), DTN_EDEVICE);
  HBSCHK(hipMemcpyAsync(&hs, d_st, sizeof(hs), hipMemcpyDeviceToHost, s), DTN_EDEVICE);
  HBSCHK(hipStreamSynchronize(s), DTN_EDEVICE);
  if (hs.rank_capped) {
    set_err("hbs: a basis reached the rank cap (" + std::to_string(kHbsMaxRank) + ") at this tol: raise tol");
    return DTN_ERANK;
  }
  H->k.assign(nn, 0);
  H->kc.assign(nn, 0);
  H->level_rank.assign(H->depth + 1, 0);
  for (int q = 1; q < nn; ++q) {
    H->k[q] = cnt[2 * q];
    H->kc[q] = cnt[2 * q + 1];
    H->level_rank[H->level_of[q]] = std::max(H->level_rank[H->level_of[q]], std::max(H->k[q], H->kc[q]));
  }
  // packed layout and the copies that fill it
  auto ncand = [&](int q, int side) {
    const HbsTreeNode& t = H->nodes[q];
    if (t.c1 < 0) return t.hi - t.lo;
    return side == 0 ? H->k[t.c1] + H->k[t.c2] : H->kc[t.c1] + H->kc[t.c2];
  };
  if (square)
    for (int q = 1; q < nn; ++q)
      if (H->k[q] != H->kc[q]) { set_err("hbs: equal-rank construction left unequal ranks"); return DTN_EDEVICE; }
  H->offU.assign(nn, -1);
  H->offV.assign(nn, -1);
  H->offD.assign(nn, -1);
  H->offB12.assign(nn, -1);
  H->offB21.assign(nn, -1);
  auto& offU = H->offU;
  auto& offV = H->offV;
  auto& offD = H->offD;
  auto& offB12 = H->offB12;
  auto& offB21 = H->offB21;
  std::vector<HbsCopy> jobs;
  long long at = 0;
  const int skel_base = 0;
  auto skel_off = [&](int q, int side) { return skel_base + (2 * q + side) * kHbsMaxRank; };
  for (int q = 0; q < nn; ++q) {
    const HbsTreeNode& t = H->nodes[q];
    if (q > 0) {
      for (int side = 0; side < 2; ++side) {
        const int p = ncand(q, side), k = side == 0 ? H->k[q] : H->kc[q];
        if (p * k == 0) continue;
        (side == 0 ? offU : offV)[q] = at;
        jobs.push_back({1, (long long)(2 * q + side) * kHbsMaxCand * kHbsMaxRank, kHbsMaxCand, -1, -1, p, k, at});
        at += (long long)p * k;
      }
    }
    if (t.c1 < 0) {
      const int m = t.hi - t.lo;
      offD[q] = at;
      jobs.push_back({0, (long long)t.lo + (long long)t.lo * nb, nb, -1, -1, m, m, at});
      at += (long long)m * m;
    } else {
      if (H->k[t.c1] * H->kc[t.c2] > 0) {
        offB12[q] = at;
        jobs.push_back({0, 0, nb, skel_off(t.c1, 0), skel_off(t.c2, 1), H->k[t.c1], H->kc[t.c2], at});
        at += (long long)H->k[t.c1] * H->kc[t.c2];
      }
      if (H->k[t.c2] * H->kc[t.c1] > 0) {
        offB21[q] = at;
        jobs.push_back({0, 0, nb, skel_off(t.c2, 0), skel_off(t.c1, 1), H->k[t.c2], H->kc[t.c1], at});
        at += (long long)H->k[t.c2] * H->kc[t.c1];
      }
    }
  }
  H->fac_doubles = (size_t)at;
  H->fac = (double*)dev_alloc(dev, std::max<size_t>(1, H->fac_doubles) * sizeof(double));
  HbsCopy* d_jobs = (HbsCopy*)sc.get(std::max<size_t>(1, jobs.size()) * sizeof(HbsCopy));
  if (!H->fac || !d_jobs) {
    dev_release(dev, H->fac);
    set_err("hbs: device allocation failed (factors)");
    return DTN_ENOMEM;
  }
  if (!jobs.empty()) {
    HBSCHK(hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(HbsCopy), hipMemcpyHostToDevice, s), DTN_EDEVICE);
    hipLaunchKernelGGL(k_hbs_pack, dim3((unsigned)jobs.size()), dim3(256), 0, s, d_jobs, A, d_basis, d_int, H->fac);
    HBSCHK(hipGetLastError(), DTN_EDEVICE);
  }
  // apply products: workspace rows per column = for every parent, its children's xh then yh blocks
  std::vector<long long> ox(nn, -1), oy(nn, -1);
  long long w = 0;
  for (int q = 0; q < nn; ++q) {
    const HbsTreeNode& t = H->nodes[q];
    if (t.c1 < 0) continue;
    ox[q] = w; w += H->kc[t.c1] + H->kc[t.c2];
    oy[q] = w; w += H->k[t.c1] + H->k[t.c2];
  }
  H->work_rows = (size_t)std::max<long long>(w, 1);
  std::vector<int> parent(nn, -1);
  for (int q = 0; q < nn; ++q)
    if (H->nodes[q].c1 >= 0) { parent[H->nodes[q].c1] = q; parent[H->nodes[q].c2] = q; }
  // rows of node q's xh / yh inside its parent's block
  auto xrow = [&](int q) { const int pq = parent[q]; return ox[pq] + (H->nodes[pq].c2 == q ? H->kc[H->nodes[pq].c1] : 0); };
  auto yrow = [&](int q) { const int pq = parent[q]; return oy[pq] + (H->nodes[pq].c2 == q ? H->k[H->nodes[pq].c1] : 0); };
  std::vector<HbsMm> mm;
  auto launch = [&](std::vector<HbsMm>& v) {
    if (v.empty()) return;
    H->launches.push_back({(int)mm.size(), (int)v.size()});
    mm.insert(mm.end(), v.begin(), v.end());
    v.clear();
  };
  std::vector<HbsMm> cur;
  // leaves: xh = V^T x(I), y(I) = D x(I)
  for (int q = 0; q < nn; ++q) {
    const HbsTreeNode& t = H->nodes[q];
    if (t.c1 >= 0) continue;
    const int m = t.hi - t.lo;
    if (q > 0 && H->kc[q] > 0)
      cur.push_back({H->kc[q], m, 0, 1, 3, 1, offV[q], t.lo, xrow(q), m, -1, -1, 0.0});
    cur.push_back({m, m, 0, 1, 2, 0, offD[q], t.lo, t.lo, m, -1, -1, 0.0});
  }
  launch(cur);
  // upward: parents below the root, deepest first
  for (int lev = H->depth - 1; lev >= 1; --lev) {
    for (int q = 1; q < nn; ++q) {
      const HbsTreeNode& t = H->nodes[q];
      if (H->level_of[q] != lev || t.c1 < 0 || H->kc[q] == 0) continue;
      const int pcols = H->kc[t.c1] + H->kc[t.c2];
      cur.push_back({H->kc[q], pcols, 0, 3, 3, 1, offV[q], ox[q], xrow(q), pcols, -1, -1, 0.0});
    }
    launch(cur);
  }
  // sibling blocks of every parent (they initialise yh)
  for (int q = 0; q < nn; ++q) {
    const HbsTreeNode& t = H->nodes[q];
    if (t.c1 < 0) continue;
    const int k1 = H->k[t.c1], k2 = H->k[t.c2], c1 = H->kc[t.c1], c2 = H->kc[t.c2];
    if (k1 > 0) {
      if (c2 > 0) cur.push_back({k1, c2, 0, 3, 3, 0, offB12[q], ox[q] + c1, oy[q], k1, -1, -1, 0.0});
      else cur.push_back({k1, 0, 0, 3, 3, 0, 0, 0, oy[q], 1, -1, -1, 0.0});
    }
    if (k2 > 0) {
      if (c1 > 0) cur.push_back({k2, c1, 0, 3, 3, 0, offB21[q], ox[q], oy[q] + k1, k2, -1, -1, 0.0});
      else cur.push_back({k2, 0, 0, 3, 3, 0, 0, 0, oy[q] + k1, 1, -1, -1, 0.0});
    }
  }
  launch(cur);
  // downward: parents below the root, top first: [yh_c1; yh_c2] += U yh
  for (int lev = 1; lev <= H->depth - 1; ++lev) {
    for (int q = 1; q < nn; ++q) {
      const HbsTreeNode& t = H->nodes[q];
      if (H->level_of[q] != lev || t.c1 < 0 || H->k[q] == 0) continue;
      const int prow = H->k[t.c1] + H->k[t.c2];
      if (prow == 0) continue;
      cur.push_back({prow, H->k[q], 0, 3, 3, 0, offU[q], yrow(q), oy[q], prow, -1, -1, 1.0});
    }
    launch(cur);
  }
  // leaves: y(I) += U yh
  for (int q = 1; q < nn; ++q) {
    const HbsTreeNode& t = H->nodes[q];
    if (t.c1 >= 0 || H->k[q] == 0) continue;
    const int m = t.hi - t.lo;
    cur.push_back({m, H->k[q], 0, 3, 2, 0, offU[q], yrow(q), t.lo, m, -1, -1, 1.0});
  }
  launch(cur);
  if (!mm_shapes_ok(mm)) { set_err("hbs: an apply product has more rows than the apply kernel takes"); return DTN_EINVAL; }
  H->d_mm = (HbsMm*)dev_alloc(dev, std::max<size_t>(1, mm.size()) * sizeof(HbsMm));
  if (!H->d_mm) {
    dev_release(dev, H->fac);
    set_err("hbs: device allocation failed (apply descriptors)");
    return DTN_ENOMEM;
  }
  if (!mm.empty())
    HBSCHK(hipMemcpyAsync(H->d_mm, mm.data(), mm.size() * sizeof(HbsMm), hipMemcpyHostToDevice, s), DTN_EDEVICE);
  HBSCHK(hipStreamSynchronize(s), DTN_EDEVICE);   // scratch is released on return
  *out = H.release();
  return DTN_OK;
}

int hbs_compress(dtn_op* op, double tol, int leaf, hipStream_t s) {
  if (!op->T) { set_err("hbs: the handle holds no dense operator to compress"); return DTN_EINVAL; }
  HbsRep* H = nullptr;
  const int rc = hbs_construct(op->device, op->T, op->nb, tol, leaf, false, s, &H);
  if (rc != DTN_OK) return rc;
  rep_free(op->device, op->hbs);
  op->hbs = H;
  return DTN_OK;
}

// Section 5.1, Algorithm 1: factors of T^{-1} from the equal-rank HBS factors {U, V, D, B} of T, levels
// finer to coarser.  A node tau with block Dt (its leaf block D, or at a parent the children's reduced
// blocks Dh joined by the sibling blocks B12, B21) gets
//   Dh = (V^T Dt^{-1} U)^{-1},  E = Dt^{-1} U Dh,  F* = Dh V^T Dt^{-1},  G = Dt^{-1} - E V^T Dt^{-1},
// and the root keeps G = (its joined block)^{-1}.  Per level: the blocks Dt are assembled in the G
// slots (k_hbs_blk) and inverted in place (k_hbs_gj); W1 = Dt^{-1} U and W2 = V^T Dt^{-1}, then
// V^T W1, inverted in place into Dh; E = W1 Dh and F* = Dh W2; G -= E W2 (FP64 MFMA products of
// every node of the level in one launch each).  Algorithm 2's apply products follow.
int hbs_invert_matrix(int dev, const double* A, int nb, double tol, int leaf, hipStream_t s, HbsRep** out) {
  *out = nullptr;
  HbsRep* Fraw = nullptr;
  int rc = hbs_construct(dev, A, nb, tol, leaf, true, s, &Fraw);
  if (rc != DTN_OK) return rc;
  struct RepGuard {
    int dev;
    HbsRep* H;
    ~RepGuard() { rep_free(dev, H); }
  } fguard{dev, Fraw};
  const HbsRep& F = *Fraw;
  const int nn = (int)F.nodes.size();
  auto H = std::make_unique<HbsRep>();
  H->nb = F.nb;
  H->leaf = F.leaf;
  H->depth = F.depth;
  H->tol = F.tol;
  H->nodes = F.nodes;
  H->level_of = F.level_of;
  H->k = F.k;
  H->kc = F.kc;
  H->level_rank = F.level_rank;
  const auto& nodes = F.nodes;
  // size of each node's block Dt and its rank
  std::vector<int> pdim(nn), rk(nn);
  for (int q = 0; q < nn; ++q) {
    const HbsTreeNode& t = nodes[q];
    pdim[q] = t.c1 < 0 ? t.hi - t.lo : F.k[t.c1] + F.k[t.c2];
    rk[q] = q > 0 ? F.k[q] : 0;
    if (pdim[q] > kHbsGjMax) { set_err("hbs: a block exceeds the inversion kernel's size"); return DTN_EINVAL; }
  }
  // inverse factors E, F*, G per node (root: G only), and the scratch W1, W2, Dh
  std::vector<long long> oE(nn, -1), oFs(nn, -1), oG(nn, -1), oW1(nn, -1), oW2(nn, -1), oDh(nn, -1);
  long long at = 0, sat = 0;
  for (int q = 0; q < nn; ++q) {
    const long long p = pdim[q], k = rk[q];
    if (q > 0) {
      oE[q] = at; at += p * k;
      oFs[q] = at; at += k * p;
      oW1[q] = sat; sat += p * k;
      oW2[q] = sat; sat += k * p;
      oDh[q] = sat; sat += k * k;
    }
    oG[q] = at; at += p * p;
  }
  H->fac_doubles = (size_t)at;
  H->fac = (double*)dev_alloc(dev, std::max<size_t>(1, H->fac_doubles) * sizeof(double));
  if (!H->fac) { set_err("hbs: device allocation failed (inverse factors)"); return DTN_ENOMEM; }
  struct FacGuard {
    int dev;
    HbsRep* H;
    bool armed = true;
    ~FacGuard() { if (armed) { dev_release(dev, H->fac); dev_release(dev, H->d_mm); } }
  } hguard{dev, H.get()};
  DevScratch sc(dev, s);
  double* scr = (double*)sc.get((size_t)std::max<long long>(sat, 1) * sizeof(double));
  DevStatus* d_st = (DevStatus*)sc.get(sizeof(DevStatus));
  if (!scr || !d_st) { set_err("hbs: device allocation failed (inversion scratch)"); return DTN_ENOMEM; }
  HBSCHK(hipMemsetAsync(d_st, 0, sizeof(DevStatus), s), DTN_EDEVICE);

  // host-side job lists, one group per (level, step)
  std::vector<HbsBlk> blks;
  std::vector<HbsGj> gjs;
  std::vector<GemmDesc> gds;
  struct Step { int kind, first, count, tiles; };   // kind 0: blk, 1: gj (tiles: register tile, 0: global), 2: gemm
  std::vector<Step> steps;
  constexpr int kCfg = 3;
  const int tm = gemm_tile_m(kCfg), tn = gemm_tile_n(kCfg);
  enum { FAC = 0, IFAC = 1, SCR = 2 };
  std::vector<GemmDesc> cur;
  auto gemm = [&](int M, int N, int K, int bA, long long oA, int lda, int tA, int bB, long long oB, int ldb, int bC,
                  long long oC, int ldc, double alpha, double beta) {
    if (M <= 0 || N <= 0) return;
    GemmDesc g{};
    g.M = M; g.N = N; g.K = K;
    g.bufA = bA; g.bufB = bB; g.bufC = bC;
    g.offA = oA; g.offB = oB; g.offC = oC;
    g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.rmapC = g.cmapC = g.kmapA = -1;
    g.transA = tA;
    g.alpha = alpha; g.beta = beta;
    cur.push_back(g);
  };
  auto flush_gemm = [&]() {
    if (cur.empty()) return;
    int tiles = 0;
    for (auto& g : cur) {
      g.tiles_m = (g.M + tm - 1) / tm;
      g.tiles_n = (g.N + tn - 1) / tn;
      g.tile_start = tiles;
      tiles += g.tiles_m * g.tiles_n;
    }
    steps.push_back({2, (int)gds.size(), (int)cur.size(), tiles});
    gds.insert(gds.end(), cur.begin(), cur.end());
    cur.clear();
  };
  // the inversions pushed since g0, one step per kernel size class (register tiles of 4, 8 or 10 rows
  // per thread, else the global-memory kernel), ordered by size
  auto push_gj_step = [&](int g0) {
    std::stable_sort(gjs.begin() + g0, gjs.end(), [](const HbsGj& a, const HbsGj& b) { return a.n < b.n; });
    for (int g = g0; g < (int)gjs.size();) {
      const int cls = gj_class(gjs[g].n);
      int e = g;
      while (e < (int)gjs.size() && gj_class(gjs[e].n) == cls) ++e;
      steps.push_back({1, g, e - g, cls});
      g = e;
    }
  };
  // assemble the joined block of parent q (or the leaf block) into G_q and invert it
  auto assemble_invert = [&](const std::vector<int>& qs) {
    const int b0 = (int)blks.size(), g0 = (int)gjs.size();
    for (int q : qs) {
      const HbsTreeNode& t = nodes[q];
      const int p = pdim[q];
      if (p == 0) continue;
      if (t.c1 < 0) {
        blks.push_back({FAC, IFAC, F.offD[q], oG[q], p, p, p, p});
      } else {
        const int k1 = F.k[t.c1], k2 = F.k[t.c2];
        if (k1) blks.push_back({SCR, IFAC, oDh[t.c1], oG[q], k1, p, k1, k1});
        if (k2) blks.push_back({SCR, IFAC, oDh[t.c2], oG[q] + k1 + (long long)k1 * p, k2, p, k2, k2});
        if (k1 && k2) {
          blks.push_back({FAC, IFAC, F.offB12[q], oG[q] + (long long)k1 * p, k1, p, k1, k2});
          blks.push_back({FAC, IFAC, F.offB21[q], oG[q] + k1, k2, p, k2, k1});
        }
      }
      gjs.push_back({IFAC, p, oG[q]});
    }
    if ((int)blks.size() > b0) steps.push_back({0, b0, (int)blks.size() - b0, 0});
    push_gj_step(g0);
  };
  for (int lev = F.depth; lev >= 1; --lev) {
    std::vector<int> qs;
    for (int q = 1; q < nn; ++q)
      if (F.level_of[q] == lev) qs.push_back(q);
    assemble_invert(qs);
    for (int q : qs) {   // W1 = Dt^{-1} U (p x k), W2 = V^T Dt^{-1} (k x p)
      const int p = pdim[q], k = rk[q];
      if (!k || !p) continue;
      gemm(p, k, p, IFAC, oG[q], p, 0, FAC, F.offU[q], p, SCR, oW1[q], p, 1.0, 0.0);
      gemm(k, p, p, FAC, F.offV[q], p, 1, IFAC, oG[q], p, SCR, oW2[q], k, 1.0, 0.0);
    }
    flush_gemm();
    for (int q : qs) {   // V^T W1 (k x k)
      const int p = pdim[q], k = rk[q];
      if (!k || !p) continue;
      gemm(k, k, p, FAC, F.offV[q], p, 1, SCR, oW1[q], p, SCR, oDh[q], k, 1.0, 0.0);
    }
    flush_gemm();
    {
      const int g0 = (int)gjs.size();
      for (int q : qs)
        if (rk[q] && pdim[q]) gjs.push_back({SCR, rk[q], oDh[q]});
      push_gj_step(g0);
    }
    for (int q : qs) {   // E = W1 Dh (p x k), F* = Dh W2 (k x p)
      const int p = pdim[q], k = rk[q];
      if (!k || !p) continue;
      gemm(p, k, k, SCR, oW1[q], p, 0, SCR, oDh[q], k, IFAC, oE[q], p, 1.0, 0.0);
      gemm(k, p, k, SCR, oDh[q], k, 0, SCR, oW2[q], k, IFAC, oFs[q], k, 1.0, 0.0);
    }
    flush_gemm();
    for (int q : qs) {   // G = Dt^{-1} - E W2
      const int p = pdim[q], k = rk[q];
      if (!k || !p) continue;
      gemm(p, p, k, IFAC, oE[q], p, 0, SCR, oW2[q], k, IFAC, oG[q], p, -1.0, 1.0);
    }
    flush_gemm();
  }
  assemble_invert({0});

  HbsBlk* d_blk = (HbsBlk*)sc.get(std::max<size_t>(1, blks.size()) * sizeof(HbsBlk));
  HbsGj* d_gj = (HbsGj*)sc.get(std::max<size_t>(1, gjs.size()) * sizeof(HbsGj));
  GemmDesc* d_gd = (GemmDesc*)sc.get(std::max<size_t>(1, gds.size()) * sizeof(GemmDesc));
  if (!d_blk || !d_gj || !d_gd) { set_err("hbs: device allocation failed (inversion jobs)"); return DTN_ENOMEM; }
  if (!blks.empty())
    HBSCHK(hipMemcpyAsync(d_blk, blks.data(), blks.size() * sizeof(HbsBlk), hipMemcpyHostToDevice, s), DTN_EDEVICE);
  if (!gjs.empty())
    HBSCHK(hipMemcpyAsync(d_gj, gjs.data(), gjs.size() * sizeof(HbsGj), hipMemcpyHostToDevice, s), DTN_EDEVICE);
  if (!gds.empty())
    HBSCHK(hipMemcpyAsync(d_gd, gds.data(), gds.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, s), DTN_EDEVICE);
  DevBufs B{};
  B.p[FAC] = F.fac;
  B.p[IFAC] = H->fac;
  B.p[SCR] = scr;
  for (const Step& st : steps) {
    if (st.kind == 0) {
      hipLaunchKernelGGL(k_hbs_blk, dim3(st.count), dim3(256), 0, s, d_blk + st.first, (const double*)F.fac, H->fac, scr);
      HBSCHK(hipGetLastError(), DTN_EDEVICE);
    } else if (st.kind == 1) {
      const HbsGj* jg = d_gj + st.first;
      if (st.tiles == 4)
        hipLaunchKernelGGL(k_hbs_gjr<4>, dim3(st.count), dim3(256), 0, s, jg, H->fac, scr, d_st);
      else if (st.tiles == 8)
        hipLaunchKernelGGL(k_hbs_gjr<8>, dim3(st.count), dim3(256), 0, s, jg, H->fac, scr, d_st);
      else if (st.tiles == 10)
        hipLaunchKernelGGL(k_hbs_gjr<10>, dim3(st.count), dim3(256), 0, s, jg, H->fac, scr, d_st);
      else
        hipLaunchKernelGGL(k_hbs_gj, dim3(st.count), dim3(256), 0, s, jg, H->fac, scr, d_st);
      HBSCHK(hipGetLastError(), DTN_EDEVICE);
    } else {
      HBSCHK(launch_gemm_batched(d_gd + st.first, st.count, st.tiles, kCfg, B, nullptr, s, 0, 0, 3, nullptr), DTN_EDEVICE);
    }
  }
  DevStatus hs{};
  HBSCHK(hipMemcpyAsync(&hs, d_st, sizeof(hs), hipMemcpyDeviceToHost, s), DTN_EDEVICE);
  HBSCHK(hipStreamSynchronize(s), DTN_EDEVICE);
  if (hs.singular) {
    set_err("hbs: a block of the inversion (Dt, V^T Dt^{-1} U or the root block) is singular");
    return DTN_ESINGULAR;
  }

  // Algorithm 2: y = T^{-1} x.  Workspace per column: for every parent its children's xh, then yh.
  std::vector<long long> ox(nn, -1), oy(nn, -1);
  long long w = 0;
  for (int q = 0; q < nn; ++q) {
    const HbsTreeNode& t = nodes[q];
    if (t.c1 < 0) continue;
    ox[q] = w; w += F.k[t.c1] + F.k[t.c2];
    oy[q] = w; w += F.k[t.c1] + F.k[t.c2];
  }
  H->work_rows = (size_t)std::max<long long>(w, 1);
  std::vector<int> parent(nn, -1);
  for (int q = 0; q < nn; ++q)
    if (nodes[q].c1 >= 0) { parent[nodes[q].c1] = q; parent[nodes[q].c2] = q; }
  auto xrow = [&](int q) { const int pq = parent[q]; return ox[pq] + (nodes[pq].c2 == q ? F.k[nodes[pq].c1] : 0); };
  auto yrow = [&](int q) { const int pq = parent[q]; return oy[pq] + (nodes[pq].c2 == q ? F.k[nodes[pq].c1] : 0); };
  std::vector<HbsMm> mm, mcur;
  auto launch = [&]() {
    if (mcur.empty()) return;
    H->launches.push_back({(int)mm.size(), (int)mcur.size()});
    mm.insert(mm.end(), mcur.begin(), mcur.end());
    mcur.clear();
  };
  if (nodes[0].c1 < 0) {   // the root is a leaf: y = G x
    mcur.push_back({pdim[0], pdim[0], 0, 1, 2, 0, oG[0], 0, 0, pdim[0], -1, -1, 0.0});
    launch();
  } else {
    for (int q = 1; q < nn; ++q)   // leaves: xh = F* x(I)
      if (nodes[q].c1 < 0 && rk[q] > 0)
        mcur.push_back({rk[q], pdim[q], 0, 1, 3, 0, oFs[q], nodes[q].lo, xrow(q), rk[q], -1, -1, 0.0});
    launch();
    for (int lev = F.depth - 1; lev >= 1; --lev) {   // upward: xh = F* [xh_c1; xh_c2]
      for (int q = 1; q < nn; ++q)
        if (F.level_of[q] == lev && nodes[q].c1 >= 0 && rk[q] > 0)
          mcur.push_back({rk[q], pdim[q], 0, 3, 3, 0, oFs[q], ox[q], xrow(q), rk[q], -1, -1, 0.0});
      launch();
    }
    mcur.push_back({pdim[0], pdim[0], 0, 3, 3, 0, oG[0], ox[0], oy[0], pdim[0], -1, -1, 0.0});   // root
    launch();
    for (int lev = 1; lev <= F.depth - 1; ++lev) {   // downward: [yh_c1; yh_c2] = E yh + G [xh_c1; xh_c2]
      for (int q = 1; q < nn; ++q)
        if (F.level_of[q] == lev && nodes[q].c1 >= 0 && pdim[q] > 0)
          mcur.push_back({pdim[q], rk[q], 0, 3, 3, 0, rk[q] ? oE[q] : 0, rk[q] ? yrow(q) : 0, oy[q], pdim[q], -1, -1, 0.0});
      launch();
      for (int q = 1; q < nn; ++q)
        if (F.level_of[q] == lev && nodes[q].c1 >= 0 && pdim[q] > 0)
          mcur.push_back({pdim[q], pdim[q], 0, 3, 3, 0, oG[q], ox[q], oy[q], pdim[q], -1, -1, 1.0});
      launch();
    }
    for (int q = 1; q < nn; ++q)   // leaves: y(I) = E yh + G x(I)
      if (nodes[q].c1 < 0)
        mcur.push_back({pdim[q], rk[q], 0, 3, 2, 0, rk[q] ? oE[q] : 0, rk[q] ? yrow(q) : 0, nodes[q].lo, pdim[q], -1, -1, 0.0});
    launch();
    for (int q = 1; q < nn; ++q)
      if (nodes[q].c1 < 0)
        mcur.push_back({pdim[q], pdim[q], 0, 1, 2, 0, oG[q], nodes[q].lo, nodes[q].lo, pdim[q], -1, -1, 1.0});
    launch();
  }
  if (!mm_shapes_ok(mm)) { set_err("hbs: an apply product has more rows than the apply kernel takes"); return DTN_EINVAL; }
  H->d_mm = (HbsMm*)dev_alloc(dev, std::max<size_t>(1, mm.size()) * sizeof(HbsMm));
  if (!H->d_mm) { set_err("hbs: device allocation failed (inverse apply descriptors)"); return DTN_ENOMEM; }
  HBSCHK(hipMemcpyAsync(H->d_mm, mm.data(), mm.size() * sizeof(HbsMm), hipMemcpyHostToDevice, s), DTN_EDEVICE);
  HBSCHK(hipStreamSynchronize(s), DTN_EDEVICE);
  hguard.armed = false;
  *out = H.release();
  return DTN_OK;
}

int hbs_invert(dtn_op* op, double tol, int leaf, hipStream_t s) {
  if (!op->T) { set_err("hbs: the handle holds no dense operator to invert"); return DTN_EINVAL; }
  HbsRep* H = nullptr;
  const int rc = hbs_invert_matrix(op->device, op->T, op->nb, tol, leaf, s, &H);
  if (rc != DTN_OK) return rc;
  rep_free(op->device, op->hbsi);
  op->hbsi = H;
  return DTN_OK;
}

void hbs_rep_free(int dev, HbsRep* H) { rep_free(dev, H); }

size_t hbs_bytes(const dtn_op* op) {
  return (op->hbs ? op->hbs->fac_doubles * sizeof(double) : 0) + (op->hbsi ? op->hbsi->fac_doubles * sizeof(double) : 0);
}

size_t hbs_work_bytes(const HbsRep* H, int k) { return H ? H->work_rows * (size_t)k * sizeof(double) : 0; }

hipError_t hbs_apply(const HbsRep* H, const double* X, int ldx, int k, double* Y, int ldy, double* work,
                     hipStream_t s) {
  for (const auto& L : H->launches) {
    const dim3 grid((unsigned)L.second, (unsigned)((k + 31) / 32));
    hipLaunchKernelGGL(k_hbs_mm, grid, dim3(256), 0, s, H->d_mm + L.first, k, H->fac, X, ldx, Y, ldy, work,
                       (int)H->work_rows);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Row and column reordering of a merge's interface block: Kp = K(src, src), i x i, both ld i.
__global__ __launch_bounds__(256) void k_perm_square(const double* __restrict__ K, int i, const int* __restrict__ src,
                                                     double* __restrict__ Kp) {
  const long long tot = (long long)i * i;
  for (long long q = blockIdx.x * 256LL + threadIdx.x; q < tot; q += (long long)gridDim.x * 256) {
    const int r = (int)(q % i), c = (int)(q / i);
    Kp[q] = K[src[r] + (long long)src[c] * i];
  }
}

// Zp = rows src of diag(Z1, Z2): Z1 is i1 x e1 (ld i1), Z2 is (i - i1) x e2 (ld i - i1), Zp is i x (e1 + e2), ld i.
__global__ __launch_bounds__(256) void k_perm_rhs(const double* __restrict__ Z1, const double* __restrict__ Z2, int i,
                                                  int i1, int e1, int e2, const int* __restrict__ src,
                                                  double* __restrict__ Zp) {
  const long long tot = (long long)i * (e1 + e2);
  const int i2 = i - i1;
  for (long long q = blockIdx.x * 256LL + threadIdx.x; q < tot; q += (long long)gridDim.x * 256) {
    const int r = (int)(q % i), c = (int)(q / i), sr = src[r];
    double v = 0.0;
    if (sr < i1) {
      if (c < e1) v = Z1[sr + (long long)c * i1];
    } else if (c >= e1) {
      v = Z2[(sr - i1) + (long long)(c - e1) * i2];
    }
    Zp[q] = v;
  }
}

// X(src, :) = Xp: Xp is i x e (ld i), X has leading dimension ldx.
__global__ __launch_bounds__(256) void k_perm_scatter(const double* __restrict__ Xp, int i, int e,
                                                      const int* __restrict__ src, double* __restrict__ X, int ldx) {
  const long long tot = (long long)i * e;
  for (long long q = blockIdx.x * 256LL + threadIdx.x; q < tot; q += (long long)gridDim.x * 256) {
    const int r = (int)(q % i), c = (int)(q / i);
    X[src[r] + (long long)c * ldx] = Xp[q];
  }
}

static unsigned perm_grid(long long tot) { return (unsigned)std::min<long long>(4096, std::max<long long>(1, (tot + 255) / 256)); }

int hbs_perm_solve(int dev, const double* K, int i, const std::vector<int>& src, const double* Z1, int i1, int e1,
                   const double* Z2, int e2, double tol, int leaf, double* X, int ldx, hipStream_t s) {
  const int e = e1 + e2;
  if (i <= 0 || i1 < 0 || i1 > i || e1 < 0 || e2 < 0 || ldx < i || (int)src.size() != i) {
    set_err("hbs: interface solve shapes do not match");
    return DTN_EINVAL;
  }
  std::vector<char> seen(i, 0);
  for (int r : src) {
    if (r < 0 || r >= i || seen[r]) { set_err("hbs: interface order is not a permutation"); return DTN_EINVAL; }
    seen[r] = 1;
  }
  DevScratch sc(dev, s);
  int* d_src = (int*)sc.get((size_t)i * sizeof(int));
  double* Kp = (double*)sc.get((size_t)i * i * sizeof(double));
  double* Zp = (double*)sc.get((size_t)i * std::max(e, 1) * sizeof(double));
  double* Xp = (double*)sc.get((size_t)i * std::max(e, 1) * sizeof(double));
  if (!d_src || !Kp || !Zp || !Xp) { set_err("hbs: device allocation failed (interface solve)"); return DTN_ENOMEM; }
  HBSCHK(hipMemcpyAsync(d_src, src.data(), (size_t)i * sizeof(int), hipMemcpyHostToDevice, s), DTN_EDEVICE);
  hipLaunchKernelGGL(k_perm_square, dim3(perm_grid((long long)i * i)), dim3(256), 0, s, K, i, d_src, Kp);
  HBSCHK(hipGetLastError(), DTN_EDEVICE);
  HbsRep* H = nullptr;
  int rc = hbs_invert_matrix(dev, Kp, i, tol, leaf, s, &H);
  if (rc != DTN_OK) return rc;
  struct RepGuard {
    int dev;
    hipStream_t s;
    HbsRep* H;
    ~RepGuard() {
      (void)hipStreamSynchronize(s);   // the applies below read the factors
      rep_free(dev, H);
    }
  } guard{dev, s, H};
  if (e == 0) {
    HBSCHK(hipStreamSynchronize(s), DTN_EDEVICE);
    return DTN_OK;
  }
  double* W = (double*)sc.get(std::max<size_t>(hbs_work_bytes(H, e), 8));
  if (!W) { set_err("hbs: device allocation failed (interface solve)"); return DTN_ENOMEM; }
  hipLaunchKernelGGL(k_perm_rhs, dim3(perm_grid((long long)i * e)), dim3(256), 0, s, Z1, Z2, i, i1, e1, e2, d_src, Zp);
  HBSCHK(hipGetLastError(), DTN_EDEVICE);
  HBSCHK(hbs_apply(H, Zp, i, e, Xp, i, W, s), DTN_EDEVICE);
  hipLaunchKernelGGL(k_perm_scatter, dim3(perm_grid((long long)i * e)), dim3(256), 0, s, Xp, i, e, d_src, X, ldx);
  HBSCHK(hipGetLastError(), DTN_EDEVICE);
  HBSCHK(hipStreamSynchronize(s), DTN_EDEVICE);   // the scratch is released on return
  return DTN_OK;
}

int gj_block_class(int n) { return gj_class(n); }

hipError_t launch_gj_blocks(const HbsGj* jobs, int count, int cls, double* buf, DevStatus* st, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (cls == 4) hipLaunchKernelGGL(k_hbs_gjr<4>, dim3(count), dim3(256), 0, s, jobs, buf, buf, st);
  else if (cls == 8) hipLaunchKernelGGL(k_hbs_gjr<8>, dim3(count), dim3(256), 0, s, jobs, buf, buf, st);
  else if (cls == 10) hipLaunchKernelGGL(k_hbs_gjr<10>, dim3(count), dim3(256), 0, s, jobs, buf, buf, st);
  else hipLaunchKernelGGL(k_hbs_gj, dim3(count), dim3(256), 0, s, jobs, buf, buf, st);
  return hipGetLastError();
}

void hbs_info(const HbsRep* H, dtn_hbs_info* out) {
  std::memset(out, 0, sizeof(*out));
  if (!H) return;
  out->leaf = H->leaf;
  out->levels = H->depth;
  out->nodes = (int)H->nodes.size();
  out->tol = H->tol;
  out->bytes = H->fac_doubles * sizeof(double);
  out->launches = (int)H->launches.size();
  for (int l = 0; l <= H->depth && l < 32; ++l) out->max_rank[l] = H->level_rank[l];
}

}  // namespace dtn
