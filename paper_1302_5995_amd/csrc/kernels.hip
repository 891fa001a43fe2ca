// gfx950 kernels of the DtN build and apply.
//
// Every Schur complement of the build - a base box (Section 3.1) or a pairwise
// merge (Section 3.2) - is S = K_ee - K_ei K_ii^{-1} K_ie for a matrix K whose
// entries are read through `KAcc` from the children's Schur complements and
// the h^2-scaled five-point stencil (Section 7).  Small tasks run whole in one
// workgroup out of LDS; large merges use an explicit inverse of K_ii by
// blocked Gauss-Jordan elimination with partial pivoting followed by two
// batched FP64 matrix-core products.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <algorithm>
#include <utility>

#include "common.h"
#include "kernels.h"

namespace dtn {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Entries of M' = h^2 * (five-point operator); boundary-ring rows are the
// one-sided difference u(b) - u(b_in); corner rows are zero.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double mcoef(const Coef& C, const double* __restrict__ coef, int p, int q) {
  // nodes are encoded (j << 16) | i
  const int n = C.n;
  const int ip = p & 0xFFFF, jp = p >> 16, iq = q & 0xFFFF, jq = q >> 16;
  const bool rx = (ip == 0) || (ip == n - 1);
  const bool ry = (jp == 0) || (jp == n - 1);
  if (rx && ry) return 0.0;
  if (rx || ry) {
    // one-sided difference toward the inward neighbour; for a network, the current through that link
    double w = 1.0;
    if (C.net) {
      const size_t nn = (size_t)n * n;
      if (jp == 0)          w = coef[nn + ip];                              // link (i,0)-(i,1)
      else if (jp == n - 1) w = coef[nn + ip + (size_t)n * (n - 2)];        // link (i,n-2)-(i,n-1)
      else if (ip == 0)     w = coef[(size_t)n * jp];                       // link (0,j)-(1,j)
      else                  w = coef[(size_t)(n - 2) + (size_t)n * jp];     // link (n-2,j)-(n-1,j)
    }
    if (p == q) return w;
    const int ii = ip == 0 ? 1 : (ip == n - 1 ? n - 2 : ip);
    const int jj = jp == 0 ? 1 : (jp == n - 1 ? n - 2 : jp);
    return (iq == ii && jq == jj) ? -w : 0.0;
  }
  const size_t nn = (size_t)n * n;
  const size_t k = (size_t)ip + (size_t)n * jp;
  if (C.net) {
    // network form: -sigma toward each linked neighbour, their sum (+ h^2 d) on the diagonal
    const double se = coef[k], sw = coef[k - 1], sn = coef[nn + k], ss = coef[nn + k - n];
    if (p == q) return se + sw + sn + ss + C.h2 * coef[2 * nn + k];
    if (jq == jp) {
      if (iq == ip + 1) return -se;
      if (iq == ip - 1) return -sw;
    } else if (iq == ip) {
      if (jq == jp + 1) return -sn;
      if (jq == jp - 1) return -ss;
    }
    return 0.0;
  }
  if (p == q) return 4.0 + C.h2 * coef[2 * nn + k];
  if (jq == jp) {
    if (iq == ip + 1) return -1.0 + C.cs * coef[k];        // east
    if (iq == ip - 1) return -1.0 - C.cs * coef[k];        // west
  } else if (iq == ip) {
    if (jq == jp + 1) return -1.0 + C.cs * coef[nn + k];   // north
    if (jq == jp - 1) return -1.0 - C.cs * coef[nn + k];   // south
  }
  return 0.0;
}

// Entry (a, b) of K in the task's local ordering [P1; P2; P3; P4] (merge) or [ring; interior].
struct KAcc {
  int kind, e, e1, i1, m1, m2;
  const int* cpos;
  const int* node;
  const double* S1;
  const double* S2;
  const double* coef;
  Coef C;
  __device__ __forceinline__ bool first(int a) const { return a < e1 || (a >= e && a < e + i1); }
  __device__ __forceinline__ double operator()(int a, int b) const {
    if (kind == 0) return mcoef(C, coef, node[a], node[b]);
    const bool fa = first(a), fb = first(b);
    if (fa && fb) return S1[cpos[a] + (long long)m1 * cpos[b]];
    if (!fa && !fb) return S2[cpos[a] + (long long)m2 * cpos[b]];
    // nodes of different children: a stencil entry, nonzero only for neighbours (a ring node's
    // entries are toward itself and its inward neighbour)
    const int p = node[a], q = node[b];
    const int di = (q & 0xFFFF) - (p & 0xFFFF), dj = (q >> 16) - (p >> 16);
    return abs(di) + abs(dj) <= 1 ? mcoef(C, coef, p, q) : 0.0;
  }
};

__device__ __forceinline__ KAcc make_acc(const SchurTask& t, const int* ip, const DevBufs& B) {
  KAcc K;
  K.kind = t.kind; K.e = t.e; K.e1 = t.e1; K.i1 = t.i1; K.m1 = t.m1; K.m2 = t.m2;
  K.cpos = ip + t.idx;
  K.node = K.cpos + t.e + t.i;
  // base boxes read no child S: point at valid memory so that masked-off loads stay in bounds
  K.S1 = t.kind ? B.p[t.src] + t.s1 : B.p[BUF_COEF] + t.coef;
  K.S2 = t.kind ? B.p[t.src] + t.s2 : B.p[BUF_COEF] + t.coef;
  K.coef = B.p[BUF_COEF] + t.coef;
  K.C = Coef{t.cn, t.net, 0, 0, t.h2, t.cs};
  return K;
}


// Pivot statistics gathered in registers during an elimination and published once at the
// end of the kernel (a global atomic per step would stall every barrier behind it).
struct PivotWatch {
  double min_ratio = 1.0e300;
  int nonfinite = 0;
  __device__ __forceinline__ void note(double piv, double scale) {
    const double a = fabs(piv);
    if (!(a == a) || a > 1.79e308) { nonfinite = 1; return; }
    const double ratio = scale > 0.0 ? a / scale : 0.0;
    min_ratio = fmin(min_ratio, ratio);
  }
  // branch-free variant with the reciprocal scale precomputed
  __device__ __forceinline__ void note_scaled(double piv, double inv_scale) {
    const double a = fabs(piv);
    nonfinite |= !(a <= 1.79e308);          // NaN or Inf
    min_ratio = fmin(min_ratio, a * inv_scale);
  }
  // weak: the unpivoted path's threshold; strict: singular threshold of the pivoted path
  __device__ __forceinline__ void publish(DevStatus* st, bool fast) const {
    if (nonfinite) { atomicOr(&st->nonfinite, 1); if (fast) atomicOr(&st->weak, 1); }
    if (min_ratio < 1.0e300) {
      if (fast && min_ratio <= kWeakPivotRtol) atomicOr(&st->weak, 1);
      if (!fast && min_ratio <= kPivotRtol) atomicOr(&st->singular, 1);
      atomicMin(&st->min_ratio_bits, (unsigned long long)__double_as_longlong(min_ratio));
    }
  }
};

// Wave-level argmax of (value, index); ties go to the smaller index.
__device__ __forceinline__ void wave_argmax(double& v, int& ix) {
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oi = __shfl_xor(ix, off, 64);
    if (ov > v || (ov == v && oi < ix)) { v = ov; ix = oi; }
  }
}

// ---------------------------------------------------------------------------
// Small tasks: one workgroup, K_ii | K_ie in LDS, Gauss-Jordan on the
// augmented matrix (X = K_ii^{-1} K_ie appears in the right block), then
// S = K_ee - K_ei X with K_ei staged through the freed left block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_small_schur(const SchurTask* __restrict__ tasks,
                                                      const int* __restrict__ ip, DevBufs B,
                                                      DevStatus* st) {
  extern __shared__ double sm[];
  __shared__ double redv[4];
  __shared__ int redi[4];
  __shared__ double s_scale;
  const SchurTask t = tasks[blockIdx.x];
  const int e = t.e, i = t.i, ncol = i + e;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const KAcc K = make_acc(t, ip, B);
  const int* pmap = ip + t.idx + 2 * (e + i);
  double* out = B.p[t.dst] + t.out;

  if (i > 0) {
    double mx = 0.0;
    for (int idx = tid; idx < i * ncol; idx += 256) {
      const int r = idx % i, c = idx / i;
      const double v = (c < i) ? K(e + r, e + c) : K(e + r, c - i);
      sm[idx] = v;
      if (c < i) mx = fmax(mx, fabs(v));
    }
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) redv[wave] = mx;
    __syncthreads();
    if (tid == 0) s_scale = fmax(fmax(redv[0], redv[1]), fmax(redv[2], redv[3]));
    __syncthreads();
    const double scale = s_scale;
    PivotWatch pw;
    for (int c = 0; c < i; ++c) {
      double best = -1.0;
      int bi = INT_MAX;
      for (int r = c + tid; r < i; r += 256) {
        const double v = fabs(sm[r + c * i]);
        if (v > best) { best = v; bi = r; }
      }
      wave_argmax(best, bi);
      if (lane == 0) { redv[wave] = best; redi[wave] = bi; }
      __syncthreads();
      int p = redi[0];
      double pb = redv[0];
      for (int w = 1; w < 4; ++w)
        if (redv[w] > pb || (redv[w] == pb && redi[w] < p)) { pb = redv[w]; p = redi[w]; }
      const double piv = sm[p + c * i];
      pw.note(piv, scale);
      const double rp = 1.0 / piv;
      // every thread holds the pivot before the swap below rewrites column c (entry (p, c) included)
      __syncthreads();
      // swap rows c and p (columns >= c) and normalise the new row c
      for (int j = c + tid; j < ncol; j += 256) {
        const double vc = sm[c + j * i], vp = sm[p + j * i];
        sm[c + j * i] = vp * rp;
        if (p != c) sm[p + j * i] = vc;
      }
      __syncthreads();
      // eliminate column c from every other row
      const int nj = ncol - c - 1;
      for (int idx = tid; idx < nj * i; idx += 256) {
        const int r = idx % i, j = c + 1 + idx / i;
        if (r != c) sm[r + j * i] -= sm[r + c * i] * sm[c + j * i];
      }
      __syncthreads();
    }
    if (tid == 0) pw.publish(st, false);
  }

  // S = K_ee - K_ei X; rows staged in chunks of i through the left block of sm.
  const int ch = i > 0 ? i : e;
  const double* X = sm + (size_t)i * i;   // X(r, b) = X[r + b*i]
  for (int a0 = 0; a0 < e; a0 += ch) {
    const int rows = min(ch, e - a0);
    if (i > 0) {
      for (int idx = tid; idx < rows * i; idx += 256) {
        const int aa = idx % rows, r = idx / rows;
        sm[aa + r * rows] = K(a0 + aa, e + r);
      }
      __syncthreads();
    }
    for (int idx = tid; idx < rows * e; idx += 256) {
      const int aa = idx % rows, b = idx / rows;
      const int a = a0 + aa;
      double v = K(a, b);
      if (i > 0) {
        int rlo = 0, rhi = i;
        if (t.kind == 1) { if (a < t.e1) rhi = t.i1; else rlo = t.i1; }
        double acc = 0.0;
        for (int r = rlo; r < rhi; ++r) acc += sm[aa + r * rows] * X[r + (size_t)b * i];
        v -= acc;
      }
      out[pmap[a] + (long long)e * pmap[b]] = v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Fast path (no cross-row pivoting).  Thread j keeps column j of the matrix in
// registers; the pivot column of each step is broadcast through LDS by its
// owner, so each elimination step costs one barrier and i FMAs per thread.
// ---------------------------------------------------------------------------



// Gauss-Jordan elimination of an nr x nc matrix held in registers by a TR x TC thread grid
// (TC a multiple of TR): thread (tr, tc) = (tid / TC, tid % TC) owns rows tr + TR a (a < EA) and
// columns tc + TC b (b < EB), nr <= TR EA.  The pivot row, the pivot column and the reciprocal of
// the pivot are broadcast through double-buffered LDS by their owners (the owner of the next pivot
// divides once, after its own update), so a step costs one barrier and, per entry, one FMA.
// Pivot c lives in row slot Q = c / TR and column slot (Q TR) / TC; the steps are generated once
// per row slot, so every register index is static and no per-entry select is issued.
//   INVERT = false: reduce the first nr columns to the identity (solve form; columns
//                   nr..nc-1 end up holding M[:, :nr]^{-1} M[:, nr:], columns < nr are left
//                   with values nobody reads);
//   INVERT = true : in-place inverse of the nr x nr matrix (nc == nr).
// Only thread 0's pivot watch is kept (it is the one that publishes).
template <int TR, int TC, int EA, int EB>
struct GjeLds {
  double (*prow)[TC * EB];
  double (*pcol)[TR * EA];
  double* rps;
  double* pivs;              // pivot c before scaling, for the pivot watch after the last step
};

// 1 / v from the hardware reciprocal estimate and two Newton-Raphson steps x <- x + x (1 - v x)
// (within an ulp of the correctly rounded quotient for normal v; five dependent operations
// instead of the eleven of the IEEE division sequence, on the critical path of every step).
__device__ __forceinline__ double recip_nr(double v) {
  double x = __builtin_amdgcn_rcp(v);
  double e = fma(-v, x, 1.0);
  x = fma(x, e, x);
  e = fma(-v, x, 1.0);
  return fma(x, e, x);
}

// Owners of pivot row/column c + 1 (row slot QR at row position cr, column slot QC at column
// position cc) publish them, and the owner of the pivot itself its reciprocal.
template <int TR, int TC, int EA, int EB, int QR, int QC>
__device__ __forceinline__ void gje_publish(const double (&m)[EA][EB], const GjeLds<TR, TC, EA, EB>& L, int nbuf,
                                            int tr, int tc, int cr, int cc, int c) {
  if (tr == cr) {
#pragma unroll
    for (int b = 0; b < EB; ++b) L.prow[nbuf][tc + TC * b] = m[QR][b];
  }
  if (tc == cc) {
#pragma unroll
    for (int a = 0; a < EA; ++a) L.pcol[nbuf][tr + TR * a] = m[a][QC];
    if (tr == cr) {
      L.rps[nbuf] = recip_nr(m[QR][QC]);
      L.pivs[c] = m[QR][QC];
    }
  }
}

// The steps whose pivots sit in row slot Q.
template <int TR, int TC, int EA, int EB, bool INVERT, int Q>
__device__ __forceinline__ void gje_slot(double (&m)[EA][EB], int nr, const GjeLds<TR, TC, EA, EB>& L,
                                         double inv_scale, PivotWatch& pw) {
  (void)inv_scale;
  (void)pw;
  constexpr int QC = Q * TR / TC, C0 = Q * TR % TC;   // column slot and first column position
  const int tid = threadIdx.x, tr = tid / TC, tc = tid % TC;
  const int ce = min(TR, nr - Q * TR);
#pragma unroll 1
  for (int cr = 0; cr < ce; ++cr) {
    const int c = Q * TR + cr, buf = c & 1;
    const double rp = L.rps[buf];
    double lr[EA], pj[EB];
#pragma unroll
    for (int a = 0; a < EA; ++a) lr[a] = L.pcol[buf][tr + TR * a];
#pragma unroll
    for (int b = 0; b < EB; ++b) pj[b] = L.prow[buf][tc + TC * b] * rp;
    const bool own_r = tr == cr, own_c = tc == C0 + cr;
#pragma unroll
    for (int a = 0; a < EA; ++a) {
      if (a == Q && own_r) {                      // the pivot row is scaled, not eliminated
#pragma unroll
        for (int b = 0; b < EB; ++b) m[a][b] *= rp;
      } else {
#pragma unroll
        for (int b = 0; b < EB; ++b) m[a][b] = fma(-lr[a], pj[b], m[a][b]);
      }
    }
    if (INVERT && own_c) {                        // the pivot column becomes column c of the inverse
#pragma unroll
      for (int a = 0; a < EA; ++a) m[a][QC] = (a == Q && own_r) ? rp : -lr[a] * rp;
    }
    if (c + 1 < nr) {
      constexpr int QN = Q + 1 < EA ? Q + 1 : Q;
      constexpr int QNC = QN * TR / TC, CN0 = QN * TR % TC;
      if (cr + 1 < TR) gje_publish<TR, TC, EA, EB, Q, QC>(m, L, buf ^ 1, tr, tc, cr + 1, C0 + cr + 1, c + 1);
      else gje_publish<TR, TC, EA, EB, QN, QNC>(m, L, buf ^ 1, tr, tc, 0, CN0, c + 1);
    }
    __syncthreads();
  }
}

template <int TR, int TC, int EA, int EB, bool INVERT, int... Qs>
__device__ __forceinline__ void gje_slots(std::integer_sequence<int, Qs...>, double (&m)[EA][EB], int nr,
                                          const GjeLds<TR, TC, EA, EB>& L, double inv_scale, PivotWatch& pw) {
  (gje_slot<TR, TC, EA, EB, INVERT, Qs>(m, nr, L, inv_scale, pw), ...);
}

// prow, pcol, rps: double-buffered broadcast slots; pivs: room for nr pivots.
template <int TR, int TC, int EA, int EB, bool INVERT>
__device__ __forceinline__ void gje2d(double (&m)[EA][EB], int nr, double (*prow)[TC * EB], double (*pcol)[TR * EA],
                                      double* rps, double* pivs, double scale, PivotWatch& pw) {
  static_assert(TC % TR == 0, "column grid a multiple of the row grid");
  static_assert(TR * EA <= TC * EB || !INVERT, "square inverse");
  const int tid = threadIdx.x, tr = tid / TC, tc = tid % TC;
  const GjeLds<TR, TC, EA, EB> L{prow, pcol, rps, pivs};
  if (nr <= 0) return;
  gje_publish<TR, TC, EA, EB, 0, 0>(m, L, 0, tr, tc, 0, 0, 0);
  __syncthreads();
  const double inv_scale = scale > 0.0 ? 1.0 / scale : 0.0;
  gje_slots<TR, TC, EA, EB, INVERT>(std::make_integer_sequence<int, EA>(), m, nr, L, inv_scale, pw);
  // the last step ended with a barrier: every pivot is in pivs; wave 0 reduces them for thread 0
  if (tid < 64) {
    PivotWatch w;
    for (int c = tid; c < nr; c += 64) w.note_scaled(pivs[c], inv_scale);
    for (int o = 32; o > 0; o >>= 1) {
      w.min_ratio = fmin(w.min_ratio, __shfl_xor(w.min_ratio, o, 64));
      w.nonfinite |= __shfl_xor(w.nonfinite, o, 64);
    }
    if (tid == 0) {
      pw.min_ratio = fmin(pw.min_ratio, w.min_ratio);
      pw.nonfinite |= w.nonfinite;
    }
  }
}

// Entry of M' in the row of a node p that is not on the boundary ring, toward node q (both
// encoded (j << 16) | i): 4 + h^2 d on the diagonal, -1 -/+ cs b toward west/east, -1 -/+ cs c
// toward south/north, 0 otherwise.  Branch-free; one coefficient load (always in bounds).
__device__ __forceinline__ double mrow(const Coef& C, const double* __restrict__ coef, int p, int q) {
  if (C.net) return mcoef(C, coef, p, q);   // network form: conductances of the node's four links
  const int ip = p & 0xFFFF, jp = p >> 16, iq = q & 0xFFFF, jq = q >> 16;
  const int di = iq - ip, dj = jq - jp;
  const bool diag = (di == 0) & (dj == 0);
  const bool horiz = (dj == 0) & ((di == 1) | (di == -1));
  const bool vert = (di == 0) & ((dj == 1) | (dj == -1));
  const long long nn = (long long)C.n * C.n;
  const long long k = ip + (long long)C.n * jp;
  const double f = coef[(diag ? 2 * nn : (vert ? nn : 0)) + k];
  const double sgn = (double)(di + dj);
  return diag ? fma(C.h2, f, 4.0) : ((horiz | vert) ? fma(sgn * C.cs, f, -1.0) : 0.0);
}

// Entry (r, j) of [K_ii | K_ie] of a small task: r an interior row (P3/P4 of a merge, an
// interior node of a base box), j < i a column of K_ii, j >= i column j - i of K_ie.  Merges
// read the children's Schur complements for same-child entries; the only stencil entries are
// the interface coupling A34 (rows P3/P4 are never on the boundary ring), and K_ie has no
// cross-child entries (A32 = A41 = 0 for the five-point stencil).  Base boxes are all stencil.
__device__ __forceinline__ double fill_entry(const KAcc& K, int i, int r, int j) {
  const int e = K.e;
  const int a = e + r;
  const int bcol = j < i ? e + j : j - i;
  const bool fa = r < K.i1;
  const bool fb = j < i ? j < K.i1 : bcol < K.e1;
  const bool same = K.kind != 0 && fa == fb;
  const double* S = fa ? K.S1 : K.S2;
  const long long m = fa ? K.m1 : K.m2;
  const long long idx = same ? K.cpos[a] + m * K.cpos[bcol] : 0;
  const double sv = S[idx];
  const bool stencil = K.kind == 0 || j < i;
  const double cv = stencil ? mrow(K.C, K.coef, K.node[a], K.node[bcol]) : 0.0;
  return same ? sv : cv;
}

// Entry (r, j) of the transposed system [K_ii^T | K_ei^T] of a merge (not a base box): K(c, e + r)
// with c = e + j (j < i) or c = j - i, i.e. row r of the transposed system is column e + r of K.
// Consecutive j read consecutive rows of a child's (column-major) S, so a wave's gathers are
// contiguous; the interface coupling A34 comes from the stencil (row of interior node c), and
// K_ei has no cross-child entries.
__device__ __forceinline__ double fill_entry_t(const KAcc& K, int i, int r, int j) {
  const int e = K.e;
  const int b = e + r;
  const int c = j < i ? e + j : j - i;
  const bool fb = r < K.i1;
  const bool fc = j < i ? j < K.i1 : c < K.e1;
  const bool same = fc == fb;
  const double* S = fc ? K.S1 : K.S2;
  const long long m = fc ? K.m1 : K.m2;
  const long long idx = same ? K.cpos[c] + m * K.cpos[b] : 0;
  double v = S[idx];
  if (!same) {
    // interface coupling: nonzero only between stencil neighbours, whose coefficient is read
    v = 0.0;
    if (j < i) {
      const int p = K.node[c], q = K.node[b];
      const int di = (q & 0xFFFF) - (p & 0xFFFF), dj = (q >> 16) - (p >> 16);
      if (abs(di) + abs(dj) == 1) v = mrow(K.C, K.coef, p, q);
    }
  }
  return v;
}

// Row a of S = K_ee - K_ei X for columns b = b0, b0 + bstep, ... < e, with X (i x e, ld i,
// followed by 64 zeros) in LDS.  Merges keep row a of K_ei (S13 or S24: zero toward the other
// child) in registers and read X columns as LDS broadcasts; a base-box ring node couples to at
// most one interior node (its inward neighbour), so its row of K_ei X is one scaled row of X.
// Reads of the children's S and writes of the parent's S are coalesced across the lanes (rows).
template <int IM, bool BASE>
__device__ __forceinline__ void small_output_row(const KAcc& K, int e, int i, const double* xs, const int* pmap,
                                                 double* out, int a, int b0, int bstep) {
  static_assert(BASE || (IM % 8 == 0 && IM <= 64), "rows of K_ei are processed 8 at a time");
  const long long prow_a = pmap[a];
  if (!BASE) {
    const bool fa = a < K.e1;
    const double* S = fa ? K.S1 : K.S2;
    const long long mm = fa ? K.m1 : K.m2;
    const long long ca = K.cpos[a];
    double kr[IM];
#pragma unroll
    for (int r = 0; r < IM; ++r) {
      const bool use = r < i && (fa == (r < K.i1));
      const long long ix = use ? ca + mm * K.cpos[e + (use ? r : 0)] : 0;
      kr[r] = use ? S[ix] : 0.0;
      if ((r & 15) == 15) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll 1
    for (int b = b0; b < e; b += bstep) {
      const double* xb = xs + b * i;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int r0 = 0; r0 < IM; r0 += 8) {
        double xv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) xv[q] = xb[r0 + q];
#pragma unroll
        for (int q = 0; q < 8; q += 2) {
          s0 = fma(kr[r0 + q], xv[q], s0);
          s1 = fma(kr[r0 + q + 1], xv[q + 1], s1);
        }
        // keep each chunk's LDS reads and FMAs together (bounds the live operands to 8): the
        // sums pass through an empty asm that also orders the next chunk's reads after it
        asm volatile("" : "+v"(s0), "+v"(s1) : : "memory");
      }
      const bool same = fa == (b < K.e1);
      const long long ib = same ? ca + mm * K.cpos[b] : 0;
      const double kee = same ? S[ib] : mcoef(K.C, K.coef, K.node[a], K.node[b]);
      out[prow_a + (long long)e * pmap[b]] = kee - (s0 + s1);
    }
  } else {
    const int pa = K.node[a];
    int ra = 0;
    double va = 0.0;
    for (int r = 0; r < i; ++r) {
      const double v = mcoef(K.C, K.coef, pa, K.node[e + r]);
      if (v != 0.0) { ra = r; va = v; }
    }
    for (int b = b0; b < e; b += bstep) {
      const double s = va * xs[ra + b * i];
      out[prow_a + (long long)e * pmap[b]] = mcoef(K.C, K.coef, pa, K.node[b]) - s;
    }
  }
}

// S = K_ee - X'^T K_ie of a merge (not a base box) on FP64 MFMA, X' = K_ii^{-T} K_ei^T (i x e, ld i,
// then 64 zeros) in LDS.  The product is formed transposed, D = K_ie^T X': the MFMA rows are output
// columns b and its columns output rows a, so each store instruction writes 16 consecutive rows of
// the parent's S in each of four columns (K_ee is read the same way).  The calling wave takes the
// 16-column tiles tb0, tb0 + tstep, ... of the output; per tile it keeps its columns of K_ie (S31 or
// S42: zero toward the other child and past i; each load covers four consecutive rows of a child's S)
// in registers as the A operand and streams X' from LDS as the B operand, one 16-row tile at a time.
// B-operand columns past e are clamped to e - 1 and rows past i read finite X' entries (or the zeros)
// against zero K_ie entries; those outputs are not stored.
template <int IM>
__device__ __forceinline__ void small_output_mfma(const KAcc& K, int e, int i, const double* xs, const int* pmap,
                                                  double* out, int tb0, int tstep) {
  static_assert(IM % 4 == 0, "K_ie held in groups of four rows");
  constexpr int KQ = IM / 4;
  const int lane = threadIdx.x & 63, lr = lane >> 4, lc = lane & 15;
  const int nkq = (i + 3) >> 2, ntile = (e + 15) >> 4;
  for (int tb = tb0; tb < ntile; tb += tstep) {
    double ka[KQ];
    {
      const int b = 16 * tb + lc;
      const bool bv = b < e;
      const int bc = bv ? b : 0;
      const bool fb = bc < K.e1;
      const double* SB = fb ? K.S1 : K.S2;
      const long long mb = fb ? K.m1 : K.m2;
      const long long cb = mb * K.cpos[bc];
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const int r = 4 * q + lr;
        const bool use = bv && r < i && (fb == (r < K.i1));
        ka[q] = use ? SB[K.cpos[e + (use ? r : 0)] + cb] : 0.0;
      }
    }
    // the output columns b = 16 tb + 4 j + lr of this lane's D entries
    bool okb[4], fbj[4];
    long long cbj[4], obj[4];
    int nbj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int b = 16 * tb + 4 * j + lr;
      okb[j] = b < e;
      const int bc = okb[j] ? b : 0;
      fbj[j] = bc < K.e1;
      cbj[j] = K.cpos[bc];
      obj[j] = (long long)e * pmap[bc];
      nbj[j] = K.node[bc];
    }
    for (int ta = 0; ta < ntile; ++ta) {
      const int a = 16 * ta + lc;
      const bool av = a < e;
      const int ac = av ? a : 0;
      const bool fa = ac < K.e1;
      const double* S = fa ? K.S1 : K.S2;
      const long long mm = fa ? K.m1 : K.m2;
      const long long ca = K.cpos[ac];
      const long long pa = pmap[ac];
      const int na = K.node[ac];
      // the tile's K_ee gathers are issued before its MFMA chain
      double kee[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) kee[j] = av && okb[j] && fa == fbj[j] ? S[ca + mm * cbj[j]] : 0.0;
      const double* xa = xs + (long long)min(a, e - 1) * i + lr;
      d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < KQ; ++q)
        if (q < nkq) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ka[q], xa[4 * q], acc, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (av && okb[j]) out[pa + obj[j]] = (fa == fbj[j] ? kee[j] : mcoef(K.C, K.coef, na, nbj[j])) - acc[j];
    }
  }
}

// One small task per wave (i <= IMAX <= 48, i + e <= 64 EB): lane l holds columns l + 64 q of
// [K_ii | K_ie] for a base box, of the transposed system [K_ii^T | K_ei^T] for a merge (whose
// fill then reads contiguous rows of the children's S), rows in registers.  Each elimination step
// publishes the pivot column through a wave-private LDS slot (no workgroup barrier), and the rows
// rotate by one register so that the next pivot row is always register 0 (no dynamic register
// indexing): after i steps row r of X = K_ii^{-1} K_ie (base box) or X' = K_ii^{-T} K_ei^T (merge)
// sits in register IMAX - i + r.  No cross-row pivoting (the transposed system has the same
// pivots); pivots monitored.
template <int IMAX, int EB, bool BASE>
__global__ __launch_bounds__(64) void k_small_wave(const SchurTask* __restrict__ tasks, const int* __restrict__ ip,
                                                    DevBufs B, DevStatus* st) {
  extern __shared__ double lds[];               // [IMAX] pivot column, then X (i x e) and 64 zeros
  double* wcol = lds;
  double* xs = lds + IMAX;
  const SchurTask t = tasks[blockIdx.x];
  const int e = t.e, i = t.i, ncol = i + e;
  const int lane = threadIdx.x;
  KAcc K = make_acc(t, ip, B);
  K.kind = BASE ? 0 : 1;
  const int* pmap = ip + t.idx + 2 * (e + i);
  double* out = B.p[t.dst] + t.out;

  double col[EB][IMAX];
#pragma unroll
  for (int q = 0; q < EB; ++q)
#pragma unroll
    for (int p = 0; p < IMAX; ++p) col[q][p] = 0.0;
  double mx = 0.0;
  if (BASE && i > 0) {
    // stencil entries only: row r straight to register r, unrolled, so that a lane's coefficient
    // loads are all in flight together
#pragma unroll
    for (int r = 0; r < IMAX; ++r) {
#pragma unroll
      for (int q = 0; q < EB; ++q) {
        const int j = lane + 64 * q;
        const bool in = r < i && j < ncol;
        const double v = fill_entry(K, i, in ? r : 0, in ? j : 0);
        col[q][r] = in ? v : 0.0;
        if (j < i) mx = fmax(mx, fabs(col[q][r]));
      }
    }
  } else if (i > 0) {
    // merges read the children's S: fill by rotation, four rows at a time (rows r0 .. r0 + 3 enter
    // at the bottom, so after IMAX / 4 shifts row r is register r), which keeps the register count
    // and the occupancy while four rows of gathers are in flight together
    static_assert(IMAX % 4 == 0, "rows enter four at a time");
#pragma unroll 1
    for (int r0 = 0; r0 < IMAX; r0 += 4) {
      double v[4][EB];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < EB; ++q) {
          const int r = r0 + u, j = lane + 64 * q;
          const bool in = r < i && j < ncol;
          double x = 0.0;
          if (in) x = fill_entry_t(K, i, r, j);
          if (j < i) mx = fmax(mx, fabs(x));
          v[u][q] = x;
        }
#pragma unroll
      for (int q = 0; q < EB; ++q) {
#pragma unroll
        for (int p = 0; p + 4 < IMAX; ++p) col[q][p] = col[q][p + 4];
#pragma unroll
        for (int u = 0; u < 4; ++u) col[q][IMAX - 4 + u] = v[u][q];
      }
    }
  }
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  const double inv_scale = mx > 0.0 ? 1.0 / mx : 0.0;
  if (lane < 64) xs[i * e + lane] = 0.0;
  PivotWatch pw;
#pragma unroll 1
  for (int c = 0; c < i; ++c) {
    if (lane == c) {
#pragma unroll
      for (int p = 0; p < IMAX; ++p) wcol[p] = col[0][p];
    }
    __builtin_amdgcn_wave_barrier();
    double mult[IMAX];
#pragma unroll
    for (int p = 0; p < IMAX; ++p) mult[p] = wcol[p];
    const double piv = mult[0];
    pw.note_scaled(piv, inv_scale);
    const double rp = recip_nr(piv);
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      const double pr = col[q][0] * rp;
#pragma unroll
      for (int p = 1; p < IMAX; ++p) col[q][p - 1] = fma(-mult[p], pr, col[q][p]);
      col[q][IMAX - 1] = pr;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (lane == 0) pw.publish(st, true);
  // X (or X') to LDS: column b = j - i, row r in register IMAX - i + r
#pragma unroll
  for (int q = 0; q < EB; ++q) {
    const int j = lane + 64 * q;
    if (j >= i && j < ncol) {
      const int b = j - i;
#pragma unroll
      for (int p = 0; p < IMAX; ++p) {
        const int r = p - (IMAX - i);
        if (r >= 0) xs[r + b * i] = col[q][p];
      }
    }
  }
  __syncthreads();
  if constexpr (BASE) {
    for (int a = lane; a < e; a += 64) small_output_row<IMAX, BASE>(K, e, i, xs, pmap, out, a, 0, 1);
  } else {
    small_output_mfma<(IMAX + 3) / 4 * 4>(K, e, i, xs, pmap, out, 0, 1);
  }
}

// S = K_ee - K_ei K_ii^{-1} K_ie for one small task per workgroup (i <= 16 EA, i + e <= 16 BC,
// e <= 256): [K_ii | K_ie] (base box) or [K_ii^T | K_ei^T] (merge) in registers on a 16 x 16
// thread grid, eliminated by gje2d (no cross-row pivoting; pivots monitored), X = K_ii^{-1} K_ie
// or X' = K_ii^{-T} K_ei^T to LDS; base boxes then write one output row per thread (column groups
// when e <= 128), merges form S = K_ee - X'^T K_ie on FP64 MFMA, one 16-column tile per wave.
template <int EA, int BC, bool BASE>
__global__ __launch_bounds__(256) void k_small_fast(const SchurTask* __restrict__ tasks, const int* __restrict__ ip,
                                                     DevBufs B, DevStatus* st) {
  constexpr int IM = 16 * EA;
  extern __shared__ double xs[];                // X, i x e, column-major (ld i), + 64 zeros
  __shared__ double prow[2][16 * BC];
  __shared__ double pcol[2][IM];
  __shared__ double rps[2];
  __shared__ double pivs[IM];
  __shared__ unsigned long long s_scale;
  const SchurTask t = tasks[blockIdx.x];
  const int e = t.e, i = t.i, ncol = i + e;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15, lane = tid & 63;
  KAcc K = make_acc(t, ip, B);
  K.kind = BASE ? 0 : 1;
  const int* pmap = ip + t.idx + 2 * (e + i);
  double* out = B.p[t.dst] + t.out;

  double m[EA][BC];
  double mx = 0.0;
#pragma unroll
  for (int a = 0; a < EA; ++a)
#pragma unroll
    for (int b = 0; b < BC; ++b) m[a][b] = 0.0;
  // one register row at a time (a runtime loop: the entry code is emitted BC times, not EA * BC);
  // nothing to fill without interior rows (entry (0, 0) would then not exist)
#pragma unroll 1
  for (int ar = 0; ar < (i > 0 ? EA : 0); ++ar) {
    const int r = tr + 16 * ar;
    double row[BC];
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      const int j = tc + 16 * b;
      const bool in = r < i && j < ncol;
      const double v = BASE ? fill_entry(K, i, in ? r : 0, in ? j : 0) : fill_entry_t(K, i, in ? r : 0, in ? j : 0);
      row[b] = in ? v : 0.0;
      if (j < i) mx = fmax(mx, fabs(row[b]));
    }
#pragma unroll
    for (int a = 0; a < EA; ++a)
#pragma unroll
      for (int b = 0; b < BC; ++b) m[a][b] = (a == ar) ? row[b] : m[a][b];
  }
  if (tid == 0) s_scale = 0ULL;
  if (tid < 64) xs[i * e + tid] = 0.0;
  __syncthreads();
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) atomicMax(&s_scale, (unsigned long long)__double_as_longlong(mx));
  __syncthreads();
  const double scale = __longlong_as_double((long long)s_scale);
  PivotWatch pw;
  gje2d<16, 16, EA, BC, false>(m, i, prow, pcol, rps, pivs, scale, pw);
  if (tid == 0) pw.publish(st, true);
#pragma unroll
  for (int a = 0; a < EA; ++a)
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      const int r = tr + 16 * a, j = tc + 16 * b;
      if (r < i && j >= i && j < ncol) xs[r + (j - i) * i] = m[a][b];
    }
  __syncthreads();

  if constexpr (BASE) {
    const int E64 = (e + 63) & ~63;
    const int G = E64 >= 256 ? 1 : 256 / E64;
    const int a = tid % E64, g = tid / E64;
    if (g >= G || a >= e) return;
    small_output_row<IM, BASE>(K, e, i, xs, pmap, out, a, g, G);
  } else {
    small_output_mfma<IM>(K, e, i, xs, pmap, out, tid >> 6, 4);
  }
}

// Top step of the recursive block inversion of a merge whose K_ii splits at the children's interface
// (h1 = i1), after X11 = inv(A11): A12 and A21 hold the stencil coupling of the two interface lines,
// one entry per coupled pair (k = match[c] is the first child's node coupled to the second child's
// node c, or -1), so with X the K_ii block (ld i)
//   Wb = X11 A12:        column c is column k of X11 times A12[k, c];
//   Wc = A21 X11:        row c is row k of X11 times A21[c, k];
//   A22 <- A22 - A21 Wb: entry (r, c) less A21[r, k_r] Wb[k_r, c].
// The same products as the dense form, each a single term.  One thread per entry, column-major
// walks of the three outputs; blockIdx.y is the merge.
__global__ __launch_bounds__(256) void k_couple(const CoupleDesc* __restrict__ cd, const int* __restrict__ ip,
                                                DevBufs B) {
  const CoupleDesc d = cd[blockIdx.y];
  double* ws = B.p[BUF_WS];
  double* X = ws + d.inv;
  const long long i = d.i;
  const int h1 = d.h1, h2 = d.h2;
  const int* match = ip + d.match;
  const long long n0 = (long long)h1 * h2, n1 = 2 * n0, n2 = n1 + (long long)h2 * h2;
  for (long long x = blockIdx.x * 256LL + threadIdx.x; x < n2; x += (long long)gridDim.x * 256) {
    if (x < n0) {
      const int r = (int)(x % h1), c = (int)(x / h1);
      const int k = match[c];
      ws[d.wb + x] = k >= 0 ? X[r + k * i] * X[k + (h1 + c) * i] : 0.0;
    } else if (x < n1) {
      const long long y = x - n0;
      const int r = (int)(y % h2), c = (int)(y / h2);
      const int k = match[r];
      ws[d.wc + y] = k >= 0 ? X[h1 + r + k * i] * X[k + c * i] : 0.0;
    } else {
      const long long y = x - n1;
      const int r = (int)(y % h2), c = (int)(y / h2);
      const int kr = match[r], kc = match[c];
      if (kr >= 0 && kc >= 0) {
        const double wbv = X[kr + kc * i] * X[kc + (h1 + c) * i];
        double* a = X + h1 + r + (h1 + c) * i;
        *a = fma(-X[h1 + r + kr * i], wbv, *a);
      }
    }
  }
}

// In-place inverse of one diagonal block of up to 2 x 64 = 128 rows: the bottom level of the
// recursive block inversion fused into one workgroup of eight waves (the same arithmetic as the
// recursion: 64-wide register Gauss-Jordan leaves, FP64 MFMA block products).  The block (split
// h1 = ceil(bs/2), h2) sits in LDS as four zero-padded 64 x 64 quadrants:
//   X11 = inv(A11); Wb = X11 A12; S = A22 - A21 Wb; Wc = A21 X11; X22 = inv(S);
//   X12 = -Wb X22; X11 <- X11 - X12 Wc; X21 = -X22 Wc.
// A Gauss-Jordan step is bound by per-step latency and by the instructions each SIMD issues:
// eight waves (two per SIMD, 4 x 2 entries per thread) sit between the four-wave layout, whose
// latency is exposed, and the sixteen-wave one, which issues twice the per-step overhead.  In the
// products each wave owns two 16 x 16 tiles of a 64 x 64 quadrant.
constexpr int kInv2Ld = 2 * 64 + 1;
constexpr size_t kInv2Lds = (size_t)2 * 64 * kInv2Ld * sizeof(double);
constexpr int kInv2Threads = 512;

struct Quad2 {
  d4 t[2];
};

// Tiles (ti, tj0) and (ti, tj0 + 1) of P(a) * Q(b) over a 64-deep sum, plus acc; quadrant
// origins (ra, ca), (rb, cb) in Ls.
__device__ __forceinline__ Quad2 quad_mul(const double* Ls, int ra, int ca, int rb, int cb, int ti, int tj0, int lane,
                                          double sign, Quad2 acc) {
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll 4
  for (int k4 = 0; k4 < 16; ++k4) {
    const double a = sign * Ls[(ra + 16 * ti + lc) * kInv2Ld + ca + 4 * k4 + lr];
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const double b = Ls[(rb + 4 * k4 + lr) * kInv2Ld + cb + 16 * (tj0 + y) + lc];
      acc.t[y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc.t[y], 0, 0, 0);
    }
  }
  return acc;
}

__device__ __forceinline__ void quad_store(double* Ls, int r0, int c0, int ti, int tj0, int lane, const Quad2& v) {
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int j = 0; j < 4; ++j) Ls[(r0 + 16 * ti + 4 * j + lr) * kInv2Ld + c0 + 16 * (tj0 + y) + lc] = v.t[y][j];
}

__device__ __forceinline__ Quad2 quad_load(const double* Ls, int r0, int c0, int ti, int tj0, int lane) {
  const int lr = lane >> 4, lc = lane & 15;
  Quad2 v;
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int j = 0; j < 4; ++j) v.t[y][j] = Ls[(r0 + 16 * ti + 4 * j + lr) * kInv2Ld + c0 + 16 * (tj0 + y) + lc];
  return v;
}

// One group of Gauss-Jordan steps of block_invert_wave: pivots k = 8 AK + kr, whose row and column
// sit in register row AK and register column AK of the lanes with lr == kr and lc == kr.
template <int NR, int AK>
__device__ __forceinline__ void wave_gj_group(double (&m)[NR][NR], int nr, double* piv, int lr, int lc) {
  const int ke = min(8, nr - 8 * AK);
#pragma unroll 1
  for (int kr = 0; kr < ke; ++kr) {
    const bool R = lr == kr, C = lc == kr;
    // every lane reads the pivot-row entries of its columns from lane (kr, lc), the pivot-column
    // entries of its rows from lane (lr, kr) and the pivot from lane (kr, kr), register to register
    double p[NR], l[NR];
#pragma unroll
    for (int b = 0; b < NR; ++b) p[b] = __shfl(m[AK][b], 8 * kr + lc, 64);
#pragma unroll
    for (int a = 0; a < NR; ++a) l[a] = __shfl(m[a][AK], 8 * lr + kr, 64);
    const double d = __shfl(m[AK][AK], 9 * kr, 64);
    if (R && C) piv[8 * AK + kr] = d;
    const double rd = recip_nr(d);
    double q[NR];
#pragma unroll
    for (int b = 0; b < NR; ++b) q[b] = p[b] * rd;
    // the pivot row and column are left out of the rank-1 update and scaled instead
    if (R) l[AK] = 0.0;
    if (C) q[AK] = 0.0;
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
      for (int b = 0; b < NR; ++b) m[a][b] = fma(-l[a], q[b], m[a][b]);
    const double fr = R ? rd : 1.0, fc = C ? -rd : 1.0;
#pragma unroll
    for (int b = 0; b < NR; ++b) m[AK][b] *= fr;
#pragma unroll
    for (int a = 0; a < NR; ++a) m[a][AK] *= fc;
    if (R && C) m[AK][AK] = rd;
  }
}

template <int NR, int... As>
__device__ __forceinline__ void wave_gj_groups(std::integer_sequence<int, As...>, double (&m)[NR][NR], int nr,
                                               double* piv, int lr, int lc) {
  (wave_gj_group<NR, As>(m, nr, piv, lr, lc), ...);
}

// In-place inverse of the leading nr x nr part (nr <= 32) of the 32 x 32 block at (q0, q0) of Ls by
// Gauss-Jordan elimination without pivoting, done by the calling wave alone (no workgroup barrier per
// step).  Lane (lr, lc) = (lane / 8, lane % 8) holds rows lr + 8 a and columns lc + 8 b (a, b < 4).
// Each step every lane takes the pivot row's entries in its columns and the pivot column's entries in its
// rows straight from the owner lanes' registers (cross-lane permutes, no LDS), and forms the pivot's
// reciprocal itself.  Per entry the arithmetic is that of gje2d: a_ij - a_ik (a_kj / d) off the pivot
// row and column, (a_kj / d) on the row, -(a_ik / d) on the column and 1 / d at the pivot; the pivot
// d of step k goes to piv[k].  Entries outside the leading part are zero and stay zero.
__device__ __forceinline__ void block_invert_wave(double* Ls, int q0, int nr, double* piv) {
  constexpr int NR = 4;
  const int lane = threadIdx.x & 63, lr = lane >> 3, lc = lane & 7;
  double m[NR][NR];
#pragma unroll
  for (int a = 0; a < NR; ++a)
#pragma unroll
    for (int b = 0; b < NR; ++b) m[a][b] = Ls[(q0 + lr + 8 * a) * kInv2Ld + q0 + lc + 8 * b];
  wave_gj_groups<NR>(std::make_integer_sequence<int, NR>(), m, nr, piv, lr, lc);
#pragma unroll
  for (int a = 0; a < NR; ++a)
#pragma unroll
    for (int b = 0; b < NR; ++b) {
      const int r = lr + 8 * a, c = lc + 8 * b;
      if (r < nr && c < nr) Ls[(q0 + r) * kInv2Ld + q0 + c] = m[a][b];
    }
}

// One 16 x 16 tile (ti, tj) of sign * P(a) Q(b) over a 32-deep sum plus acc, blocks at (ra, ca) and
// (rb, cb) of Ls.
__device__ __forceinline__ d4 blk_mul(const double* Ls, int ra, int ca, int rb, int cb, int ti, int tj, int lane,
                                      double sign, d4 acc) {
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int k4 = 0; k4 < 8; ++k4) {
    const double a = sign * Ls[(ra + 16 * ti + lc) * kInv2Ld + ca + 4 * k4 + lr];
    const double b = Ls[(rb + 4 * k4 + lr) * kInv2Ld + cb + 16 * tj + lc];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ d4 blk_load(const double* Ls, int r0, int c0, int ti, int tj, int lane) {
  const int lr = lane >> 4, lc = lane & 15;
  d4 v;
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = Ls[(r0 + 16 * ti + 4 * j + lr) * kInv2Ld + c0 + 16 * tj + lc];
  return v;
}

__device__ __forceinline__ void blk_store(double* Ls, int r0, int c0, int ti, int tj, int lane, const d4& v) {
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int j = 0; j < 4; ++j) Ls[(r0 + 16 * ti + 4 * j + lr) * kInv2Ld + c0 + 16 * tj + lc] = v[j];
}

// In-place inverse of the leading nr x nr part of the 64 x 64 quadrant at (q0, q0): the same block
// recursion one level further down, 32 x 32 leaves inverted by wave 0 and 32 x 32 x 32 products on
// FP64 MFMA (waves 0-3 one product, waves 4-7 an independent one, a 16 x 16 tile per wave):
//   X11 = inv(B11); Wb = X11 B12, Wc = B21 X11; S = B22 - B21 Wb; X22 = inv(S);
//   X12 = -Wb X22, X21 = -X22 Wc; X11 <- X11 - X12 Wc.
// Called by the whole workgroup (ends with a barrier); pivots to piv[0 .. nr).
__device__ __forceinline__ void quad_invert(double* Ls, int q0, int nr, double* piv) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n1 = min(32, nr), n2 = nr - n1;
  const int h = wave >> 2, ti = wave & 1, tj = (wave >> 1) & 1;   // product half, 16 x 16 tile
  const int b0 = q0, b1 = q0 + 32;
  if (wave == 0) block_invert_wave(Ls, b0, n1, piv);
  __syncthreads();
  if (n2 <= 0) return;
  const d4 z{0.0, 0.0, 0.0, 0.0};
  d4 v = h == 0 ? blk_mul(Ls, b0, b0, b0, b1, ti, tj, lane, 1.0, z)     // Wb = X11 B12
                : blk_mul(Ls, b1, b0, b0, b0, ti, tj, lane, 1.0, z);    // Wc = B21 X11
  __syncthreads();
  if (h == 0) blk_store(Ls, b0, b1, ti, tj, lane, v);                   // Wb over B12
  __syncthreads();
  d4 s = z;
  if (h == 0) s = blk_mul(Ls, b1, b0, b0, b1, ti, tj, lane, -1.0, blk_load(Ls, b1, b1, ti, tj, lane));   // S
  __syncthreads();
  if (h == 0) blk_store(Ls, b1, b1, ti, tj, lane, s);
  else blk_store(Ls, b1, b0, ti, tj, lane, v);                          // Wc over B21
  __syncthreads();
  if (wave == 0) block_invert_wave(Ls, b1, n2, piv + 32);               // X22 = inv(S)
  __syncthreads();
  v = h == 0 ? blk_mul(Ls, b0, b1, b1, b1, ti, tj, lane, -1.0, z)       // X12 = -Wb X22
             : blk_mul(Ls, b1, b1, b1, b0, ti, tj, lane, -1.0, z);      // X21 = -X22 Wc
  __syncthreads();
  if (h == 0) blk_store(Ls, b0, b1, ti, tj, lane, v);                   // X12 over Wb
  __syncthreads();
  if (h == 0) s = blk_mul(Ls, b0, b1, b1, b0, ti, tj, lane, -1.0, blk_load(Ls, b0, b0, ti, tj, lane));   // X11
  __syncthreads();
  if (h == 0) blk_store(Ls, b0, b0, ti, tj, lane, s);
  else blk_store(Ls, b1, b0, ti, tj, lane, v);                          // X21 over Wc
  __syncthreads();
}

__global__ __launch_bounds__(kInv2Threads) void k_base_inv2(const BaseBlock* __restrict__ blocks, DevBufs B,
                                                            DevStatus* st) {
  extern __shared__ double Ls[];                  // 128 x kInv2Ld, row-major: Ls[r * kInv2Ld + c]
  __shared__ double pivs[128];                    // the block's pivots, watched once at the end
  __shared__ double wmax[kInv2Threads / 64];      // per wave: largest |entry| of the block and of S
  const BaseBlock bb = blocks[blockIdx.x];
  double* A = B.p[BUF_WS] + bb.off;
  const int ld = bb.ld, bs = bb.bs, h1 = (bs + 1) / 2, h2 = bs - h1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, ti = wave & 3, tj0 = 2 * (wave >> 2);
  const double scale = B.p[BUF_WS][bb.scale];
  double amax = 0.0;        // element growth: largest |entry| of the block and of its Schur complement S
  {
    // column-major walk (coalesced global reads); every load is issued before the first LDS store
    constexpr int NL = 128 * 128 / kInv2Threads;
    double v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int x = tid + kInv2Threads * q, r = x & 127, c = x >> 7;
      const int gr = r < 64 ? r : r - 64 + h1, gc = c < 64 ? c : c - 64 + h1;
      const bool in = (r < 64 ? r < h1 : r - 64 < h2) && (c < 64 ? c < h1 : c - 64 < h2);
      v[q] = in ? A[gr + (long long)gc * ld] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int x = tid + kInv2Threads * q;
      Ls[(x & 127) * kInv2Ld + (x >> 7)] = v[q];
      amax = fmax(amax, fabs(v[q]));
    }
  }
  __syncthreads();
  quad_invert(Ls, 0, h1, pivs);                                                   // X11
  if (h2 > 0) {
    const Quad2 z{{d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}}};
    Quad2 v = quad_mul(Ls, 0, 0, 0, 64, ti, tj0, lane, 1.0, z);           // Wb = X11 A12
    __syncthreads();
    quad_store(Ls, 0, 64, ti, tj0, lane, v);
    __syncthreads();
    v = quad_mul(Ls, 64, 0, 0, 64, ti, tj0, lane, -1.0, quad_load(Ls, 64, 64, ti, tj0, lane));   // S = A22 - A21 Wb
    quad_store(Ls, 64, 64, ti, tj0, lane, v);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) amax = fmax(amax, fabs(v.t[t][j]));
    v = quad_mul(Ls, 64, 0, 0, 0, ti, tj0, lane, 1.0, z);              // Wc = A21 X11
    __syncthreads();
    quad_store(Ls, 64, 0, ti, tj0, lane, v);
    __syncthreads();
    quad_invert(Ls, 64, h2, pivs + 64);                                           // X22 = inv(S)
    v = quad_mul(Ls, 0, 64, 64, 64, ti, tj0, lane, -1.0, z);           // X12 = -Wb X22
    __syncthreads();
    quad_store(Ls, 0, 64, ti, tj0, lane, v);
    __syncthreads();
    v = quad_mul(Ls, 0, 64, 64, 0, ti, tj0, lane, -1.0, quad_load(Ls, 0, 0, ti, tj0, lane));     // X11 -= X12 Wc
    quad_store(Ls, 0, 0, ti, tj0, lane, v);
    v = quad_mul(Ls, 64, 64, 64, 0, ti, tj0, lane, -1.0, z);           // X21 = -X22 Wc
    __syncthreads();
    quad_store(Ls, 64, 0, ti, tj0, lane, v);
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
  if (lane == 0) wmax[wave] = amax;
  __syncthreads();
  if (tid < 64) {
    // pivot watch: wave 0 reduces the block's pivots, lane 0 publishes
    PivotWatch pw;
    const double inv_scale = scale > 0.0 ? 1.0 / scale : 0.0;
    if (tid < h1) pw.note_scaled(pivs[tid], inv_scale);
    if (tid < h2) pw.note_scaled(pivs[64 + tid], inv_scale);
    for (int o = 32; o > 0; o >>= 1) {
      pw.min_ratio = fmin(pw.min_ratio, __shfl_xor(pw.min_ratio, o, 64));
      pw.nonfinite |= __shfl_xor(pw.nonfinite, o, 64);
    }
    if (tid == 0) {
      pw.publish(st, true);
      double g = 0.0;
      for (int w = 0; w < kInv2Threads / 64; ++w) g = fmax(g, wmax[w]);
      g *= inv_scale;
      if (g <= 1.79e308) atomicMax(&st->max_growth_bits, (unsigned long long)__double_as_longlong(g));
    }
  }
#pragma unroll
  for (int q = 0; q < 128 * 128 / kInv2Threads; ++q) {
    const int x = tid + kInv2Threads * q, r = x & 127, c = x >> 7;
    const int gr = r < 64 ? r : r - 64 + h1, gc = c < 64 ? c : c - 64 + h1;
    const bool in = (r < 64 ? r < h1 : r - 64 < h2) && (c < 64 ? c < h1 : c - 64 < h2);
    if (in) A[gr + (long long)gc * ld] = Ls[r * kInv2Ld + c];
  }
}

// ---------------------------------------------------------------------------
// Large merges.
// ---------------------------------------------------------------------------
__global__ void k_reset(const LargeMerge* __restrict__ lm, int nlm, DevBufs B, DevStatus* st) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nlm) B.p[BUF_WS][lm[q].scale] = 0.0;
  if (q == 0 && st) {
    st->singular = 0; st->nonfinite = 0; st->weak = 0; st->rank_capped = 0;
    st->min_ratio_bits = 0x7FF0000000000000ULL;
    st->max_growth_bits = 0;
  }
}

// Gather K_ii (-> inverse buffer), S31, S42, S13, S24 into scratch and K_ee into the parent S.
__global__ __launch_bounds__(256) void k_large_gather(const LargeMerge* __restrict__ lm,
                                                       const int* __restrict__ ip, DevBufs B) {
  const LargeMerge m = lm[blockIdx.y];
  const SchurTask& t = m.t;
  const KAcc K = make_acc(t, ip, B);
  const int e = t.e, i = t.i, e1 = t.e1, i1 = t.i1, e2 = e - e1, i2 = i - i1;
  double* ws = B.p[BUF_WS];
  double* out = B.p[t.dst] + t.out;
  const int* pmap = ip + t.idx + 2 * (e + i);
  // the six destination blocks, column by column: K_ii (i cols of i), S31 (e1 cols of i1), S42 (e2
  // of i2), S13 (i1 cols of e1), S24 (i2 cols of e2), K_ee (e cols of e, scattered to the parent);
  // a workgroup takes whole columns (found by comparing the column index with the block
  // boundaries), its threads walk the rows: coalesced, and no division per element
  const int skip_t = m.kee_gemm == 2;   // S13, S24 read as S31^T, S42^T by the Schur product
  const int c0 = i, c1 = c0 + e1, c2 = c1 + e2, c3 = c2 + (skip_t ? 0 : i1), c4 = c3 + (skip_t ? 0 : i2),
            c5 = c4 + (m.kee_gemm ? 0 : e);
  double mx = 0.0;
  for (int col = blockIdx.x; col < c5; col += gridDim.x) {
    if (col < c0) {
      double* dst = ws + m.inv + (long long)col * i;
      for (int r = threadIdx.x; r < i; r += 256) {
        const double v = K(e + r, e + col);
        dst[r] = v;
        mx = fmax(mx, fabs(v));
      }
    } else if (col < c1) {
      const int c = col - c0;
      double* dst = ws + m.b31 + (long long)c * i1;
      for (int r = threadIdx.x; r < i1; r += 256) dst[r] = K(e + r, c);
    } else if (col < c2) {
      const int c = col - c1;
      double* dst = ws + m.b42 + (long long)c * i2;
      for (int r = threadIdx.x; r < i2; r += 256) dst[r] = K(e + i1 + r, e1 + c);
    } else if (col < c3) {
      const int c = col - c2;
      double* dst = ws + m.a13 + (long long)c * e1;
      for (int r = threadIdx.x; r < e1; r += 256) dst[r] = K(r, e + c);
    } else if (col < c4) {
      const int c = col - c3;
      double* dst = ws + m.a24 + (long long)c * e2;
      for (int r = threadIdx.x; r < e2; r += 256) dst[r] = K(e1 + r, e + i1 + c);
    } else {
      const int c = col - c4;
      double* dst = out + (long long)e * pmap[c];
      for (int r = threadIdx.x; r < e; r += 256) dst[pmap[r]] = K(r, c);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0 && mx > 0.0)
    atomicMax((unsigned long long*)(ws + m.scale), (unsigned long long)__double_as_longlong(mx));
}

// Gauss-Jordan block step, panel part: rows r = tid + NT*q of columns [c0, c0+Wk) in registers.
template <int NT, int R, int W>
__global__ __launch_bounds__(NT) void k_gje_panel(const LargeMerge* __restrict__ lm, int c0, int* __restrict__ ip,
                                                   DevBufs B, DevStatus* st) {
  constexpr int NW = NT / 64;
  __shared__ double redv[2][NW];
  __shared__ int redi[2][NW];
  __shared__ double rowb[2][2][W];
  __shared__ double LU[W][W + 1];
  __shared__ double Linv[W][W + 1];
  __shared__ double Tm[W][W + 1];
  const LargeMerge& m = lm[blockIdx.x];
  const int i = m.t.i;
  if (c0 >= i) return;
  const int Wk = min(W, i - c0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* ws = B.p[BUF_WS];
  double* A = ws + m.inv;
  double* Q = ws + m.q;
  int* piv = ip + m.piv;
  const double scale = ws[m.scale];

  double v[R][W];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = tid + NT * q;
#pragma unroll
    for (int w = 0; w < W; ++w) v[q][w] = (r < i && w < Wk) ? A[r + (long long)(c0 + w) * i] : 0.0;
  }

  PivotWatch pw;
  for (int j = 0; j < Wk; ++j) {
    const int col = c0 + j;
    const int par = j & 1;
    double best = -1.0;
    int bi = INT_MAX;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = tid + NT * q;
      double x = 0.0;
#pragma unroll
      for (int w = 0; w < W; ++w) if (w == j) x = v[q][w];
      if (r >= col && r < i && fabs(x) > best) { best = fabs(x); bi = r; }
    }
    wave_argmax(best, bi);
    if (lane == 0) { redv[par][wave] = best; redi[par][wave] = bi; }
    __syncthreads();
    int p = redi[par][0];
    double pb = redv[par][0];
    for (int w = 1; w < NW; ++w)
      if (redv[par][w] > pb || (redv[par][w] == pb && redi[par][w] < p)) { pb = redv[par][w]; p = redi[par][w]; }
    // exchange rows col and p through LDS
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = tid + NT * q;
      if (r == p) {
#pragma unroll
        for (int w = 0; w < W; ++w) rowb[par][1][w] = v[q][w];
      }
      if (r == col && p != col) {
#pragma unroll
        for (int w = 0; w < W; ++w) rowb[par][0][w] = v[q][w];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = tid + NT * q;
      if (r == col) {
#pragma unroll
        for (int w = 0; w < W; ++w) v[q][w] = rowb[par][1][w];
      } else if (r == p) {
#pragma unroll
        for (int w = 0; w < W; ++w) v[q][w] = rowb[par][0][w];
      }
    }
    const double pv = rowb[par][1][j];
    pw.note(pv, scale);
    if (tid == 0) piv[col] = p;
    const double rp = 1.0 / pv;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = tid + NT * q;
      if (r > col && r < i) {
        double l = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) if (w == j) l = v[q][w] * rp;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          if (w == j) v[q][w] = l;
          else if (w > j) v[q][w] -= l * rowb[par][1][w];
        }
      }
    }
  }
  if (tid == 0) pw.publish(st, false);
  // diagonal block: L1 (unit lower) and U
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = tid + NT * q;
    if (r >= c0 && r < c0 + Wk) {
#pragma unroll
      for (int w = 0; w < W; ++w) LU[r - c0][w] = v[q][w];
    }
  }
  __syncthreads();
  // Linv = L1^{-1} and T = U^{-1} L1^{-1}; lane w handles column w
  if (tid < Wk) {
    const int w = tid;
    for (int a = 0; a < Wk; ++a) {
      double s = (a == w) ? 1.0 : 0.0;
      if (a > w) for (int b = w; b < a; ++b) s -= LU[a][b] * Linv[b][w];
      Linv[a][w] = (a < w) ? 0.0 : s;
    }
    for (int a = Wk - 1; a >= 0; --a) {
      double s = Linv[a][w];
      for (int b = a + 1; b < Wk; ++b) s -= LU[a][b] * Tm[b][w];
      Tm[a][w] = s / LU[a][a];
    }
  }
  __syncthreads();
  // Q' rows and the new block column, one column at a time
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = tid + NT * q;
    if (r >= i) continue;
    const bool above = r < c0, below = r >= c0 + Wk;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if (w >= Wk) continue;
      double s = 0.0;
      if (above) {
#pragma unroll
        for (int b = 0; b < W; ++b) if (b < Wk) s += v[q][b] * Tm[b][w];
      } else if (below) {
#pragma unroll
        for (int b = 0; b < W; ++b) if (b < Wk && b >= w) s += v[q][b] * Linv[b][w];
      } else {
        s = ((r - c0) == w ? 1.0 : 0.0) - Tm[r - c0][w];
      }
      Q[r + (long long)w * i] = s;
      A[r + (long long)(c0 + w) * i] = (above || below) ? -s : Tm[r - c0][w];
    }
  }
}

// Apply the block's row exchanges to every other column and copy its pivot rows into R.
__global__ __launch_bounds__(256) void k_gje_swap(const LargeMerge* __restrict__ lm, int c0,
                                                   const int* __restrict__ ip, DevBufs B) {
  const LargeMerge& m = lm[blockIdx.y];
  const int i = m.t.i;
  if (c0 >= i) return;
  const int W = m.W;
  const int Wk = min(W, i - c0);
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= i || (j >= c0 && j < c0 + Wk)) return;
  double* ws = B.p[BUF_WS];
  double* col = ws + m.inv + (long long)j * i;
  const int* piv = ip + m.piv;
  for (int s = c0; s < c0 + Wk; ++s) {
    const int p = piv[s];
    if (p != s) { const double a = col[s]; col[s] = col[p]; col[p] = a; }
  }
  double* R = ws + m.r + (long long)j * W;
  for (int w = 0; w < Wk; ++w) R[w] = col[c0 + w];
}

// Column map of the true inverse: inv(K_ii)[:, c] = inv(P K_ii)[:, kmap[c]].
__global__ void k_gje_kmap(const LargeMerge* __restrict__ lm, int* __restrict__ ip) {
  extern __shared__ int perm[];
  const LargeMerge& m = lm[blockIdx.x];
  const int i = m.t.i;
  const int* piv = ip + m.piv;
  int* kmap = ip + m.piv + i;
  for (int p = threadIdx.x; p < i; p += blockDim.x) perm[p] = p;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int s = 0; s < i; ++s) {
      const int p = piv[s];
      const int a = perm[s]; perm[s] = perm[p]; perm[p] = a;
    }
  __syncthreads();
  for (int p = threadIdx.x; p < i; p += blockDim.x) kmap[perm[p]] = p;
}

// ---------------------------------------------------------------------------
// Batched FP64 GEMM on the matrix cores.  A workgroup of 4 or 8 waves computes a BM x BN
// tile; wave w owns a WM x WN sub-tile of (WM/16) x (WN/16) v_mfma_f64_16x16x4 blocks.
// K is staged through double-buffered LDS in chunks of 16 (one barrier per chunk), with two
// chunks of global loads in flight (two register sets used alternately, so a load has two
// chunks of MFMA work to land).  In LDS both operands are stored row by row (A[m][k'],
// B[n][k']) with k' = (k % 4) * 4 + k / 4: the four k values a lane feeds to the four MFMAs of a
// chunk (k = 4 j + lane / 16) are then contiguous and come in two 128-bit reads; the MFMA sums
// are the same as with any other layout.
// ---------------------------------------------------------------------------
// MFMA 16 x 16 x 4 in the compute type CT; operands and results stay FP64 in memory.
//   double: v_mfma_f64_16x16x4f64, accumulator item j of lane l is row 4 j + l / 16;
//   float:  v_mfma_f32_16x16x4f32 (twice the FP64 rate), accumulator item j of lane l is row
//           4 (l / 16) + j; operands are rounded to FP32 when staged, sums kept in FP32.
template <typename CT> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int j, int lane) { return 4 * j + (lane >> 4); }
};
typedef float f4 __attribute__((ext_vector_type(4)));
template <> struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t zero() { return f4{0.0f, 0.0f, 0.0f, 0.0f}; }
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int j, int lane) { return 4 * (lane >> 4) + j; }
};

// MODE: the form of every A in the launch (uniform per launch, so no branch in the K loop)
//   0: column-major, A[r, k] at A[r + k lda]
//   1: column-major with gathered columns, A[r, k] at A[r + kmap[k] lda]
//   2: transposed, A[r, k] at A[k + r lda]
//   3: any of the above, chosen per descriptor
// Split K (D.ksplit = S > 1): slice ks of output tile tt covers K range [ks Kc, (ks + 1) Kc); its
// partial tile goes to ws at D.kpart, then the slice takes a ticket from the tile's counter (device
// scope, after a release fence); the slice that arrives last sums the S partials in slice order
// (the result does not depend on arrival order), resets the counter and runs the epilogue.  No
// workgroup waits for another.
template <int BM, int BN, int WM, int WN, int BK, typename CT, int MODE>
__device__ __forceinline__ void gemm_tile(const GemmDesc& D, int tm, int tn, int ks, int tt, const DevBufs& Bf,
                                          const int* __restrict__ ip, const LargeMerge* __restrict__ lm) {
  typedef Mfma<CT> MF;
  constexpr int PAD = 2, KQ = BK / 4;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int WGM = BM / WM;                    // waves along M
  constexpr int NT = 64 * (BM / WM) * (BN / WN);  // threads per workgroup
  static_assert(NT == 256 || NT == 512, "four or eight waves per tile");
  static_assert(NT % BM == 0 && NT % BK == 0, "staging layout");
  constexpr int LA = BM * BK / NT, LB = BK * BN / NT;   // elements each thread stages per chunk
  // operand staging; after the K loop the same bytes stage the output (EP doubles per row of a
  // wave's 16-column slab, odd so that the column-wise reads spread over the banks)
  constexpr int EP = 17;
  constexpr size_t kOperandBytes = (size_t)2 * (BM + BN) * (BK + PAD) * sizeof(CT);
  constexpr size_t kSlabBytes = (size_t)(NT / 64) * WM * EP * sizeof(double);
  constexpr size_t kLdsBytes = kSlabBytes > kOperandBytes ? kSlabBytes : kOperandBytes;   // FP32 128 x 128: slabs
  __shared__ __align__(16) unsigned char lds_raw[kLdsBytes];
  CT (*As)[BM][BK + PAD] = reinterpret_cast<CT (*)[BM][BK + PAD]>(lds_raw);
  CT (*Bs)[BN][BK + PAD] = reinterpret_cast<CT (*)[BN][BK + PAD]>(lds_raw + (size_t)2 * BM * (BK + PAD) * sizeof(CT));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int m0 = tm * BM, n0 = tn * BN;
  const int M = D.M, N = D.N;
  const int S = D.ksplit > 1 ? D.ksplit : 1;
  const int Kc = ((D.K + S - 1) / S + BK - 1) / BK * BK;   // slice depth, whole chunks
  const int kbeg = ks * Kc, K = min(D.K, kbeg + Kc);        // this slice: [kbeg, K)
  auto kp = [](int k) { return (k & 3) * KQ + (k >> 2); };
  const bool tA = MODE == 2 || (MODE == 3 && D.transA);
  const int* kmap = (MODE == 1 || MODE == 3) && D.kmapA >= 0 ? ip + D.kmapA : nullptr;
  // staging coordinates: slot s of thread tid holds A (row, kk) and B (kk, col)
  //   A column-major: row = tid % BM, kk = tid / BM + s NT / BM
  //   A transposed:   kk = tid % BK, row = tid / BK + s NT / BK (consecutive threads walk k)
  //   B:              kk = tid % BK, col = tid / BK + s NT / BK
  const int a_row0 = tA ? tid / BK : tid % BM, a_kk0 = tA ? tid % BK : tid / BM;
  const int a_rstep = tA ? NT / BK : 0, a_kstep = tA ? 0 : NT / BM;
  const int b_kk = tid % BK, b_col0 = tid / BK;
  const double* __restrict__ pa = Bf.p[D.bufA] + D.offA + (tA ? a_kk0 + (long long)(m0 + a_row0) * D.lda
                                                               : m0 + a_row0 + (long long)a_kk0 * D.lda);
  const double* __restrict__ pb = Bf.p[D.bufB] + D.offB + b_kk + (long long)(n0 + b_col0) * D.ldb;
  const long long a_sstride = tA ? (long long)a_rstep * D.lda : (long long)a_kstep * D.lda;
  const long long b_sstride = (long long)(NT / BK) * D.ldb;
  double* C = Bf.p[D.bufC] + D.offC;

  // A Schur product of a dense merge takes its old values K_ee(a, b) from the children's S and the
  // stencil (the parent's S is written, never read).  They do not depend on the product, so this
  // thread's entries of the epilogue (row m0 + wm WM + lane % WM, the columns of its slab passes) are
  // loaded here, in flight during the K loop: the same-child entries in one branch-free batch, then
  // the few stencil entries between the children (nonzero only for neighbouring nodes).
  constexpr int EP_CG = 64 / WM, EP_NC = 16 / EP_CG;
  const bool from_kee = D.kee > 0 && D.beta != 0.0;
  double kold[FN][EP_NC];
  if (from_kee) {
    const KAcc Kee = make_acc(lm[D.kee - 1].t, ip, Bf);
    const int grow = m0 + wm * WM + lane % WM, ec = lane / WM;
    const int a = grow < M ? D.kee_row0 + grow : 0;
    const bool fa = a < Kee.e1;
    const double* Sa = fa ? Kee.S1 : Kee.S2;
    const long long ma = fa ? Kee.m1 : Kee.m2, ca = Kee.cpos[a];
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int k = 0; k < EP_NC; ++k) {
        const int col = n0 + wn * WN + b * 16 + ec + EP_CG * k;
        const int cb = D.kee_col0 + (col < N ? col : 0);
        kold[b][k] = Sa[fa == (cb < Kee.e1) ? ca + ma * Kee.cpos[cb] : 0];
      }
    const int na = Kee.node[a];
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int k = 0; k < EP_NC; ++k) {
        const int col = n0 + wn * WN + b * 16 + ec + EP_CG * k;
        const int cb = D.kee_col0 + (col < N ? col : 0);
        if (fa == (cb < Kee.e1)) continue;
        const int nb = Kee.node[cb];
        const int di = (nb & 0xFFFF) - (na & 0xFFFF), dj = (nb >> 16) - (na >> 16);
        kold[b][k] = abs(di) + abs(dj) <= 1 ? mcoef(Kee.C, Kee.coef, na, nb) : 0.0;
      }
  }

  typename MF::acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = MF::zero();

  double ra0[LA], rb0[LB], ra1[LA], rb1[LB];
  auto load = [&](int k0, double (&ra)[LA], double (&rb)[LB]) {
    const bool tail = k0 + BK > K;
#pragma unroll
    for (int s = 0; s < LA; ++s) {
      const int row = a_row0 + a_rstep * s, kk = a_kk0 + a_kstep * s;
      const bool ok = m0 + row < M && (!tail || k0 + kk < K);
      double v = 0.0;
      if (ok) {
        if (kmap && !tA) v = Bf.p[D.bufA][D.offA + m0 + row + (long long)kmap[k0 + kk] * D.lda];
        else v = pa[(tA ? (long long)k0 : (long long)k0 * D.lda) + a_sstride * s];
      }
      ra[s] = v;
    }
#pragma unroll
    for (int s = 0; s < LB; ++s) {
      const int col = b_col0 + (NT / BK) * s;
      const bool ok = n0 + col < N && (!tail || k0 + b_kk < K);
      rb[s] = ok ? pb[k0 + b_sstride * s] : 0.0;
    }
  };
  auto store = [&](int buf, const double (&ra)[LA], const double (&rb)[LB]) {
#pragma unroll
    for (int s = 0; s < LA; ++s) As[buf][a_row0 + a_rstep * s][kp(a_kk0 + a_kstep * s)] = (CT)ra[s];
#pragma unroll
    for (int s = 0; s < LB; ++s) Bs[buf][b_col0 + (NT / BK) * s][kp(b_kk)] = (CT)rb[s];
  };
  auto compute = [&](int buf) {
    const int g = lane >> 4;
    CT fa[FM][KQ], fb[FN][KQ];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int j = 0; j < KQ; ++j) fa[a][j] = As[buf][wm * WM + a * 16 + (lane & 15)][g * KQ + j];
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int j = 0; j < KQ; ++j) fb[b][j] = Bs[buf][wn * WN + b * 16 + (lane & 15)][g * KQ + j];
#pragma unroll
    for (int j = 0; j < KQ; ++j)
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = MF::mac(fa[a][j], fb[b][j], acc[a][b]);
  };
  const int nk = K > kbeg ? (K - kbeg + BK - 1) / BK : 0;
  // chunk 0 to LDS buffer 0 and chunk 1 to register set 1; each pass of the loop computes chunks
  // kt (buffer 0) and kt + 1 (buffer 1) while chunks kt + 2 and kt + 3 load
  if (nk > 0) {
    load(kbeg, ra0, rb0);
    store(0, ra0, rb0);
    if (nk > 1) load(kbeg + BK, ra1, rb1);
    __syncthreads();
  }
  for (int kt = 0; kt < nk; kt += 2) {
    if (kt + 2 < nk) load(kbeg + (kt + 2) * BK, ra0, rb0);
    compute(0);
    if (kt + 1 < nk) store(1, ra1, rb1);
    __syncthreads();
    if (kt + 1 >= nk) break;
    if (kt + 3 < nk) load(kbeg + (kt + 3) * BK, ra1, rb1);
    compute(1);
    if (kt + 2 < nk) store(0, ra0, rb0);
    __syncthreads();
  }
  if (S > 1) {
    constexpr int NACC = FM * FN * 4;
    double* part = Bf.p[BUF_WS] + D.kpart;
    const long long slot = (long long)tt * S;
    double* mine = part + (slot + ks) * NACC * NT;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int j = 0; j < 4; ++j) mine[((a * FN + b) * 4 + j) * NT + tid] = (double)acc[a][b][j];
    __threadfence();
    __syncthreads();
    __shared__ int s_last;
    int* cnt = const_cast<int*>(ip) + D.kcnt + tt;
    if (tid == 0) s_last = atomicAdd(cnt, 1) == S - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double sum = 0.0;
          for (int q = 0; q < S; ++q) sum += part[(slot + q) * NACC * NT + ((a * FN + b) * 4 + j) * NT + tid];
          acc[a][b][j] = (CT)sum;
        }
    if (tid == 0) __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // Epilogue: each wave passes its WM x WN block through LDS one 16-column slab at a time and
  // writes whole columns: lane l takes row l % WM of column l / WM (+ 64 / WM per pass), so a
  // store covers consecutive rows of the parent (512 bytes when WM = 64) instead of 16 columns x 4
  // rows.  The last K chunk ended with a barrier, so the staging bytes are free.
  const int* rmap = D.rmapC >= 0 ? ip + D.rmapC : nullptr;
  const int* cmap = D.cmapC >= 0 ? ip + D.cmapC : nullptr;
  double* slab = reinterpret_cast<double*>(lds_raw) + (size_t)wave * WM * EP;
  constexpr int CG = 64 / WM;                     // columns one pass of the wave covers
  const int er = lane % WM, ec = lane / WM;
  const int grow = m0 + wm * WM + er;
  const bool row_ok = grow < M;
  const long long crow = row_ok ? (rmap ? rmap[grow] : grow) : 0;
#pragma unroll
  for (int b = 0; b < FN; ++b) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int j = 0; j < 4; ++j) slab[(a * 16 + MF::row(j, lane)) * EP + (lane & 15)] = (double)acc[a][b][j];
    __syncthreads();
    // addresses and (beta != 0) the old values of the slab first, so that the loads are in flight
    // together rather than each waiting behind the previous column's store
    constexpr int NC = 16 / CG;
    long long off[NC];
    bool ok[NC];
    double old[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int col = n0 + wn * WN + b * 16 + ec + CG * k;
      ok[k] = row_ok && col < N;
      off[k] = ok[k] ? crow + (long long)(cmap ? cmap[col] : col) * D.ldc : 0;
      old[k] = 0.0;
    }
    if (from_kee) {
#pragma unroll
      for (int k = 0; k < NC; ++k) old[k] = kold[b][k];
    } else if (D.beta != 0.0) {
#pragma unroll
      for (int k = 0; k < NC; ++k)
        if (ok[k]) old[k] = C[off[k]];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (ok[k]) {
        const double val = D.alpha * slab[er * EP + ec + CG * k];
        const double res = (D.beta != 0.0) ? val + D.beta * old[k] : val;
        if (!D.mirror) {
          C[off[k]] = res;
        } else {
          // symmetric result: (r, c) and (c, r); a diagonal tile writes its lower half and mirrors
          // the strictly lower part, so every entry is written exactly once
          const int col = n0 + wn * WN + b * 16 + ec + CG * k;
          const bool diag = D.tri && tm == tn;
          if (!diag || grow >= col) C[off[k]] = res;
          if (!diag || grow > col) C[(long long)(cmap ? cmap[col] : col) + crow * D.ldc] = res;
        }
      }
    }
    __syncthreads();
  }
}

// Tile configurations: 0 = 64 x 64 (waves 32 x 32), 1 = 128 x 128 (waves 64 x 64).
template <int CFG> struct TileCfg;
template <> struct TileCfg<0> { static constexpr int BM = 64, BN = 64, WM = 32, WN = 32, BK = 16; };
template <> struct TileCfg<1> { static constexpr int BM = 128, BN = 128, WM = 64, WN = 64, BK = 16; };
// 128 x 128 with eight waves of 64 x 32: twice the operand reuse of cfg 0 at ~100 registers per thread
template <> struct TileCfg<2> { static constexpr int BM = 128, BN = 128, WM = 64, WN = 32, BK = 16; };
// 32 x 32 with four waves of 16 x 16: four times the workgroups of cfg 0 for small products
template <> struct TileCfg<3> { static constexpr int BM = 32, BN = 32, WM = 16, WN = 16, BK = 16; };
// 32 x 32 with K in chunks of 64: small launches of short products (K <= a few hundred) are latency
// bound, and a quarter of the chunks means a quarter of the load-store-barrier round trips
template <> struct TileCfg<4> { static constexpr int BM = 32, BN = 32, WM = 16, WN = 16, BK = 64; };
template <int CFG> constexpr int tile_threads() {
  return 64 * (TileCfg<CFG>::BM / TileCfg<CFG>::WM) * (TileCfg<CFG>::BN / TileCfg<CFG>::WN);
}

// waves per SIMD the compiler must leave room for: three 64 x 64 workgroups per CU
template <int CFG> constexpr int tile_min_waves() { return CFG == 0 ? 3 : 1; }

template <int CFG, typename CT, int MODE>
__global__ __launch_bounds__(tile_threads<CFG>(), tile_min_waves<CFG>()) void k_gemm_batched(const GemmDesc* __restrict__ descs, int ndesc, int tile_base,
                                                       DevBufs Bf, const int* __restrict__ ip,
                                                       const LargeMerge* __restrict__ lm) {
  using T = TileCfg<CFG>;
  const int tile = blockIdx.x + tile_base;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
  }
  const GemmDesc D = descs[lo];
  const int t = tile - D.tile_start;
  const int S = D.ksplit > 1 ? D.ksplit : 1;
  const int ks = t % S, tt = t / S;
  int tm = tt % D.tiles_m, tn = tt / D.tiles_m;
  if (D.tri) {   // tiles on or below the diagonal, row by row: tt = tm (tm + 1) / 2 + tn, tn <= tm
    tm = (int)((sqrtf(8.0f * tt + 1.0f) - 1.0f) * 0.5f);
    while (tm * (tm + 1) / 2 > tt) --tm;
    while ((tm + 1) * (tm + 2) / 2 <= tt) ++tm;
    tn = tt - tm * (tm + 1) / 2;
  }
  gemm_tile<T::BM, T::BN, T::WM, T::WN, T::BK, CT, MODE>(D, tm, tn, ks, tt, Bf, ip, lm);
}

template <int CFG>
__global__ __launch_bounds__(tile_threads<CFG>()) void k_gemm_single(GemmDesc D, DevBufs Bf) {
  using T = TileCfg<CFG>;
  const int t = blockIdx.x;
  gemm_tile<T::BM, T::BN, T::WM, T::WN, T::BK, double, 0>(D, t % D.tiles_m, t / D.tiles_m, 0, t, Bf, nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// Range finding for the low-rank factorisations of the merge's off-diagonal blocks
// (Section 6, Step 2): G = Y^T Y of a sketch Y, pivoted Cholesky P^T G P = L L^T stopped at the
// first remaining diagonal <= thr, then M = P(:, 1:r) L_r^{-T} so that Y M has orthonormal
// columns spanning the kept directions; columns of M past the rank r are zero.
//   mode 0 (first pass):   thr = max(tol, 1e-7)^2 * max diag(G); max diag(G) saved at dmax
//   mode 1 (residual pass): thr = tol^2 * (saved max diag of the first pass)
//   mode 2 (re-orthogonalisation of an orthonormal-to-1e-4 Q): thr = 1e-24 * max diag(G)
// The Gram matrix keeps each pass's dynamic range within what FP64 Cholesky resolves
// (1e-7 relative to the pass's largest column); the residual pass reaches tol.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pchol(const PcholDesc* __restrict__ descs, DevBufs B, int* __restrict__ ip,
                                                   DevStatus* __restrict__ st) {
  __shared__ double G[kPcholMax][kPcholMax + 1];   // G, then L in its pivot columns
  __shared__ double Li[kPcholMax][kPcholMax + 1];  // L_r^{-1}
  __shared__ int piv[kPcholMax], ipv[kPcholMax];
  __shared__ int s_rank, s_stop;
  __shared__ double s_thr;
  const PcholDesc d = descs[blockIdx.x];
  const int k = d.k, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* ws = B.p[BUF_WS];
  for (int x = tid; x < k * k; x += 256) G[x % k][x / k] = ws[d.g + x];
  if (tid < k) piv[tid] = tid;
  __syncthreads();
  if (tid == 0) {
    double dm = 0.0;
    for (int j = 0; j < k; ++j) dm = fmax(dm, G[j][j]);
    double thr;
    if (d.mode == 0) {
      const double t = fmax(d.tol, 1e-7);
      thr = t * t * dm;
      ws[d.dmax] = dm;
    } else if (d.mode == 1) {
      thr = d.tol * d.tol * ws[d.dmax];
    } else {
      thr = 1e-24 * dm;
    }
    s_thr = thr;
    s_rank = k;
    s_stop = 0;
  }
  __syncthreads();
  const double thr = s_thr;
  for (int st = 0; st < k; ++st) {
    if (wave == 0) {
      // argmax of the remaining diagonal (pivot order positions st .. k-1)
      double v = -1.0;
      int ix = 0x7fffffff;
      for (int q = st + lane; q < k; q += 64) {
        const double dv = G[piv[q]][piv[q]];
        if (dv > v) { v = dv; ix = q; }
      }
      wave_argmax(v, ix);
      if (lane == 0) {
        if (!(v > thr)) {
          s_rank = st;
          s_stop = 1;
        } else {
          const int t = piv[st];
          piv[st] = piv[ix];
          piv[ix] = t;
        }
      }
    }
    __syncthreads();
    if (s_stop) break;
    const int c = piv[st];
    const double dp = sqrt(G[c][c]);
    // pivot column of L (rows in pivot order st + 1 .. k - 1), stored in column c
    for (int q = st + 1 + tid; q < k; q += 256) G[piv[q]][c] /= dp;
    __syncthreads();
    if (tid == 0) G[c][c] = dp;
    // trailing update of the remaining block
    const int rem = k - st - 1;
    for (int x = tid; x < rem * rem; x += 256) {
      const int a = piv[st + 1 + x % rem], b = piv[st + 1 + x / rem];
      G[a][b] -= G[a][c] * G[b][c];
    }
    __syncthreads();
  }
  const int r = s_rank;
  // L_r^{-1} (lower triangular), one column per thread
  if (tid < r) {
    const int cc = tid;
    for (int j = cc; j < r; ++j) {
      double sum = (j == cc) ? 1.0 : 0.0;
      for (int t = cc; t < j; ++t) sum -= G[piv[j]][piv[t]] * Li[t][cc];
      Li[j][cc] = sum / G[piv[j]][piv[j]];
    }
  }
  if (tid < k) ipv[piv[tid]] = tid;
  __syncthreads();
  for (int x = tid; x < k * k; x += 256) {
    const int row = x % k, col = x / k, sp = ipv[row];
    ws[d.m + x] = (sp < r && col < r && col >= sp) ? Li[col][sp] : 0.0;
  }
  if (tid == 0) {
    ip[d.rank] = r;
    // the residual pass kept all of its columns: the block's rank at tol may exceed the cap
    if (d.mode == 1 && !s_stop) atomicOr(&st->rank_capped, 1);
  }
}

// ---------------------------------------------------------------------------
// Apply Y = T G for a few columns, split over K (T streamed from HBM once per launch).
// Workgroup (rb, s, g) owns RPL row blocks of 64 (lane = row within each), the K range of split s and
// column group g (KC columns); wave w takes the range's rows w, w + 4, ... in ascending order, reading
// G (transposed beforehand by k_apply_transpose) with scalar loads.  Launches of at most 8 columns run
// k_apply_narrow instead (same order, G in place).  The four wave sums are combined in LDS in wave order and the split sums by k_apply_reduce in split
// order.  The number of splits depends on nb only, so the summation order of a column never depends
// on k or on the other columns of the launch: a column's result is bitwise the same alone or batched.
// A wide launch (up to kApplyMaxCols columns) has several column groups; the 1-D grid is renumbered
// so that the groups sharing a T tile are dispatched one after another on the same XCD (workgroups go
// to the eight XCDs in turn), where they run together and read the tile through one L2: T leaves HBM
// once per launch however many groups it has.
// ---------------------------------------------------------------------------
constexpr int kApplyGroup = 32;     // columns per workgroup of a wide launch
constexpr int kApplyMaxCols = 256;  // columns per launch
constexpr int kXcds = 8;

__host__ __device__ inline int apply_splits(int nb) { return nb >= 4096 ? 16 : (nb + 255) / 256; }

// Workgroups of a launch with `tiles` row tiles, S splits and `groups` column groups, padded to a
// multiple of the XCD count.
__host__ __device__ inline int apply_grid(int tiles, int S, int groups) {
  const int n = tiles * S * groups;
  return (n + kXcds - 1) / kXcds * kXcds;
}

// G transposed for the split-K kernels: Gt[kk * gld + c] = G[kk + c ldg] for c < k, 0 for k <= c < gld.
// Workgroup (row tile, column tile) of 64 x 64 through LDS; reads and writes are both coalesced.
__global__ __launch_bounds__(256) void k_apply_transpose(const double* __restrict__ G, int ldg, int nb, int k, int gld,
                                                         double* __restrict__ Gt) {
  __shared__ double tile[64][65];
  const int k0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int c = ty; c < 64; c += 4) {
    const int kk = k0 + tx, cc = c0 + c;
    tile[c][tx] = (kk < nb && cc < k) ? G[kk + (long long)cc * ldg] : 0.0;
  }
  __syncthreads();
  for (int q = ty; q < 64; q += 4) {
    const int kk = k0 + q, cc = c0 + tx;
    if (kk < nb && cc < gld) Gt[(long long)kk * gld + cc] = tile[tx][q];
  }
}

template <int KC, int RPL>
__global__ __launch_bounds__(256) void k_apply_splitk(const double* __restrict__ T, int nb, const double* __restrict__ Gt,
                                                       int gld, int groups, double* __restrict__ part) {
  __shared__ double red[64][KC + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int S = apply_splits(nb), tiles = (nb + 64 * RPL - 1) / (64 * RPL);
  // XCD-aware renumbering: block b runs on XCD b % 8; ids of one XCD are made consecutive
  const int per_xcd = gridDim.x / kXcds;
  const int id = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (id >= tiles * S * groups) return;                 // grid padding: the whole workgroup leaves
  const int g = id % groups, rb = (id / groups) % tiles, s = id / (groups * tiles);
  const double* Gg = Gt + g * KC;                       // this group's columns (zero past k)
  part += (long long)g * KC * nb;
  const int r0 = rb * 64 * RPL + lane;                  // lane rows r0, r0 + 64, ...
  const int per = (nb + S - 1) / S;
  const int k0 = s * per, k1 = min(nb, k0 + per);
  const double* Tr[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) Tr[q] = T + min(r0 + 64 * q, nb - 1);
  double acc[RPL][KC];
#pragma unroll
  for (int q = 0; q < RPL; ++q)
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[q][c] = 0.0;
  // wave w takes K rows k0 + w, k0 + w + 4, ... in ascending order.  The row index is wave-uniform,
  // so the G row is read with scalar loads and every FMA takes its G operand from scalar registers;
  // each G value serves the lane's RPL rows.
  constexpr int U = 8 / RPL;                            // K rows per step
  int kk = k0 + wave;
  for (; kk + 4 * (U - 1) < k1; kk += 4 * U) {
    double t[U][RPL];
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int q = 0; q < RPL; ++q) t[j][q] = Tr[q][(long long)(kk + 4 * j) * nb];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const double* gr = Gg + (long long)(kk + 4 * j) * gld;
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const double gv = gr[c];
#pragma unroll
        for (int q = 0; q < RPL; ++q) acc[q][c] = fma(t[j][q], gv, acc[q][c]);
      }
    }
  }
  for (; kk < k1; kk += 4) {
    double t[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) t[q] = Tr[q][(long long)kk * nb];
    const double* gr = Gg + (long long)kk * gld;
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const double gv = gr[c];
#pragma unroll
      for (int q = 0; q < RPL; ++q) acc[q][c] = fma(t[q], gv, acc[q][c]);
    }
  }
  // ((w0 + w1) + w2) + w3 through one LDS buffer, one row block of the lane at a time
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    for (int w = 0; w < 4; ++w) {
      __syncthreads();
      if (wave == w) {
#pragma unroll
        for (int c = 0; c < KC; ++c) red[lane][c] = w == 0 ? acc[q][c] : red[lane][c] + acc[q][c];
      }
    }
    __syncthreads();
    const int r = r0 + 64 * q;
    if (r < nb) {
      for (int c = wave; c < KC; c += 4) part[((long long)s * groups * KC + c) * nb + r] = red[lane][c];
    }
  }
}

// Narrow launches (k <= 8): the same per-column summation order with G read in place.  Each 64-row
// chunk of the split's K range is staged in LDS (column-major G is not contiguous along a K row);
// T streaming bounds these launches, not the LDS reads.
template <int KC>
__global__ __launch_bounds__(256) void k_apply_narrow(const double* __restrict__ T, int nb, const double* __restrict__ G,
                                                      int ldg, int k, double* __restrict__ part) {
  __shared__ double gs[64][KC + 1];
  __shared__ double red[64][KC + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int S = apply_splits(nb), tiles = (nb + 63) / 64;
  const int per_xcd = gridDim.x / kXcds;
  const int id = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (id >= tiles * S) return;                          // grid padding: the whole workgroup leaves
  const int rb = id % tiles, s = id / tiles;
  const int r = rb * 64 + lane;
  const int per = (nb + S - 1) / S;
  const int k0 = s * per, k1 = min(nb, k0 + per);
  const double* Tr = T + min(r, nb - 1);
  double acc[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) acc[c] = 0.0;
  for (int kc = k0; kc < k1; kc += 64) {
    const int kn = min(64, k1 - kc);
    __syncthreads();
    for (int x = tid; x < 64 * KC; x += 256) {
      const int kk = x % 64, c = x / 64;
      gs[kk][c] = (kk < kn && c < k) ? G[(kc + kk) + (long long)c * ldg] : 0.0;
    }
    __syncthreads();
#pragma unroll 1
    for (int j0 = 0; j0 < 16; j0 += 8) {
      double t[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int kk = wave + 4 * (j0 + j);
        t[j] = kk < kn ? Tr[(long long)(kc + kk) * nb] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int kk = wave + 4 * (j0 + j);
        if (kk < kn) {                                  // rows past the range add nothing, as in the wide kernels
#pragma unroll
          for (int c = 0; c < KC; ++c) acc[c] = fma(t[j], gs[kk][c], acc[c]);
        }
      }
    }
  }
  for (int w = 0; w < 4; ++w) {
    __syncthreads();
    if (wave == w) {
#pragma unroll
      for (int c = 0; c < KC; ++c) red[lane][c] = w == 0 ? acc[c] : red[lane][c] + acc[c];
    }
  }
  __syncthreads();
  if (r < nb) {
    for (int c = wave; c < KC; c += 4) part[((long long)s * KC + c) * nb + r] = red[lane][c];
  }
}

__global__ void k_apply_reduce(const double* __restrict__ part, int nb, int k, int kc, int S, double* __restrict__ Y,
                               int ldy) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (long long)nb * k) return;
  const int r = (int)(x % nb), c = (int)(x / nb);
  double v = part[(long long)c * nb + r];
  for (int s = 1; s < S; ++s) v += part[((long long)s * kc + c) * nb + r];
  Y[r + (long long)c * ldy] = v;
}

__global__ void k_scale_copy(const double* __restrict__ S, double* __restrict__ T, long long cnt, double s) {
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < cnt; x += (long long)gridDim.x * blockDim.x)
    T[x] = S[x] * s;
}

// Body loads (Section 7.3): the gathers of one phase's right-hand-side updates, workgroup (job, chunk).
// The stacked right-hand sides of a merge are [C1 0; 0 C2] at the merge's local rows (a child's C at
// its ring position cpos, its own columns); a base box's are h^2 at the loaded nodes.  C_ext goes into
// the box's C at the parent's ring positions (pmap), C_int, K_ei and, for tasks inverted here, K_ii into
// the phase scratch.
__global__ __launch_bounds__(256) void k_body_gather(const BodyJob* __restrict__ jobs, const int* __restrict__ ip,
                                                     const int* __restrict__ bnodes, DevBufs B, double h2) {
  const BodyJob J = jobs[blockIdx.x];
  const SchurTask& t = J.t;
  const KAcc K = make_acc(t, ip, B);
  const int e = t.e, i = t.i, nbs = J.hi - J.lo;
  const int* pmap = ip + t.idx + 2 * (e + i);
  double* body = B.p[BUF_BODY];
  double* scr = B.p[BUF_BSCR];
  auto rhs = [&](int a, int c) -> double {
    const int col = J.lo + c;
    if (t.kind == 0) return K.node[a] == bnodes[col] ? h2 : 0.0;
    if (K.first(a))
      return (col >= J.lo1 && col < J.hi1) ? body[J.c1 + K.cpos[a] + (long long)t.m1 * (col - J.lo1)] : 0.0;
    return (col >= J.lo2 && col < J.hi2) ? body[J.c2 + K.cpos[a] + (long long)t.m2 * (col - J.lo2)] : 0.0;
  };
  const long long n_ext = (long long)e * nbs, n_int = (long long)i * nbs, n_kei = (long long)e * i;
  for (long long x = blockIdx.y * 256LL + threadIdx.x; x < J.elems; x += (long long)gridDim.y * 256) {
    if (x < n_ext) {
      const int r = (int)(x % e), c = (int)(x / e);
      body[J.out + pmap[r] + (long long)e * c] = rhs(r, c);
    } else if (x < n_ext + n_int) {
      const long long y = x - n_ext;
      scr[J.cint + y] = rhs(e + (int)(y % i), (int)(y / i));
    } else if (x < n_ext + n_int + n_kei) {
      const long long y = x - n_ext - n_int;
      scr[J.kei + y] = K((int)(y % e), e + (int)(y / e));
    } else {
      const long long y = x - n_ext - n_int - n_kei;
      scr[J.kii + y] = K(e + (int)(y % i), e + (int)(y / i));
    }
  }
}

// F[:, user[c]] = scale * C[:, c] (nb rows).
__global__ __launch_bounds__(256) void k_body_out(const double* __restrict__ C, int nb, int cnt,
                                                  const int* __restrict__ user, double scale, double* __restrict__ F,
                                                  int ldf) {
  const long long tot = (long long)nb * cnt;
  for (long long x = blockIdx.x * 256LL + threadIdx.x; x < tot; x += (long long)gridDim.x * 256) {
    const int r = (int)(x % nb), c = (int)(x / nb);
    F[r + (long long)ldf * user[c]] = scale * C[x];
  }
}

// Node (i, j) of ring position r of the n x n grid: counter-clockwise from (0, 0), sides of n - 1 nodes.
__device__ inline void ring_ij(int n, int r, int& i, int& j) {
  const int m = n - 1, side = r / m, t = r - side * m;
  if (side == 0)      { i = t;         j = 0; }
  else if (side == 1) { i = m;         j = t; }
  else if (side == 2) { i = m - t;     j = m; }
  else                { i = 0;         j = m - t; }
}

// The root output with the ring rows of another reading: from the root Schur complement S' (rows of the
// one-sided differences u(b) - u(b_in), zero rows at the corners) to
//   R3: T = (S' + L) / h, L the Laplacian of the cycle through the ring nodes;
//   R2: T = (M2 - diag(beta) (S' - M1)) / h, where M2 holds the full five-point rows of the ring nodes
//       restricted to ring columns (couplings to nodes outside the grid dropped), beta_r is the coupling of
//       ring row r to its inward neighbour (0 at corners) and M1 the identity on non-corner rows.  The
//       interior rows and the couplings to the inward neighbours are the same in every reading, so the
//       change of ring rows is this exact rank-structured update of the Schur complement.
// coef: the problem's b, c, d fields (n^2 each, node (i, j) at i + n j); cs: convection scale; h2 = h^2.
__global__ void k_root_rows(const double* __restrict__ S, double* __restrict__ T, int n, int reading,
                            const double* __restrict__ coef, double h2, double cs, double inv_h) {
  const int nb = 4 * (n - 1);
  const long long cnt = (long long)nb * nb;
  const long long nn = (long long)n * n;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < cnt; x += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(x % nb), c = (int)(x / nb);
    const double v = S[x];
    double out;
    if (reading == 2) {   // R3
      const int d = c - r;
      const double L = (d == 0) ? 2.0 : (d == 1 || d == -1 || d == nb - 1 || d == 1 - nb) ? -1.0 : 0.0;
      out = v + L;
    } else {              // R2
      int ir, jr, ic, jc;
      ring_ij(n, r, ir, jr);
      ring_ij(n, c, ic, jc);
      const long long k = ir + (long long)n * jr;
      const double bk = coef[k], ck = coef[nn + k];
      const bool corner = (ir == 0 || ir == n - 1) && (jr == 0 || jr == n - 1);
      double beta = 0.0;
      if (!corner) {
        if (jr == 0)          beta = -1.0 + cs * ck;   // inward neighbour north
        else if (ir == n - 1) beta = -1.0 - cs * bk;   // west
        else if (jr == n - 1) beta = -1.0 - cs * ck;   // south
        else                  beta = -1.0 + cs * bk;   // east
      }
      const int di = ic - ir, dj = jc - jr;
      double m2 = 0.0;
      if (di == 0 && dj == 0)       m2 = 4.0 + h2 * coef[2 * nn + k];
      else if (di == 1 && dj == 0)  m2 = -1.0 + cs * bk;
      else if (di == -1 && dj == 0) m2 = -1.0 - cs * bk;
      else if (di == 0 && dj == 1)  m2 = -1.0 + cs * ck;
      else if (di == 0 && dj == -1) m2 = -1.0 - cs * ck;
      const double m1 = (r == c && !corner) ? 1.0 : 0.0;
      out = m2 - beta * (v - m1);
    }
    T[x] = out * inv_h;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
hipError_t launch_small(const SchurTask* tasks, int count, size_t lds, const int* ip, const DevBufs& B,
                        DevStatus* st, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_small_schur, dim3(count), dim3(256), lds, s, tasks, ip, B, st);
  return hipGetLastError();
}

hipError_t launch_small_fast(const SchurTask* tasks, int count, bool base, int imax, int cols, size_t lds,
                             const int* ip, const DevBufs& B, DevStatus* st, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (imax <= 48 && cols <= 128 && lds + 48 * 8 <= (size_t)kSmallWaveLds) {
    const int im = imax <= 16 ? 16 : imax <= 32 ? 32 : imax <= 36 ? 36 : imax <= 40 ? 40 : 48;
    const int eb = cols <= 64 ? 1 : 2;
    const size_t wl = lds + (size_t)im * 8;
#define DTN_WAVE(IM_, EB_)                                                                                        \
  if (im == IM_ && eb == EB_) {                                                                                    \
    if (base)                                                                                                      \
      hipLaunchKernelGGL((k_small_wave<IM_, EB_, true>), dim3(count), dim3(64), wl, s, tasks, ip, B, st);       \
    else                                                                                                           \
      hipLaunchKernelGGL((k_small_wave<IM_, EB_, false>), dim3(count), dim3(64), wl, s, tasks, ip, B, st);      \
  }
    DTN_WAVE(16, 1) DTN_WAVE(16, 2) DTN_WAVE(32, 1) DTN_WAVE(32, 2) DTN_WAVE(36, 1) DTN_WAVE(36, 2)
    DTN_WAVE(40, 1) DTN_WAVE(40, 2) DTN_WAVE(48, 1) DTN_WAVE(48, 2)
#undef DTN_WAVE
    return hipGetLastError();
  }
  const int ea = imax <= 16 ? 1 : imax <= 32 ? 2 : imax <= 64 ? 4 : 0;
  const int bc = cols <= 64 ? 4 : cols <= 128 ? 8 : cols <= 256 ? 16 : 0;
  if (!ea || !bc) return hipErrorInvalidValue;
#define DTN_SMALL(EA_, BC_)                                                                                \
  if (ea == EA_ && bc == BC_) {                                                                             \
    if (base)                                                                                               \
      hipLaunchKernelGGL((k_small_fast<EA_, BC_, true>), dim3(count), dim3(256), lds, s, tasks, ip, B, st); \
    else                                                                                                    \
      hipLaunchKernelGGL((k_small_fast<EA_, BC_, false>), dim3(count), dim3(256), lds, s, tasks, ip, B, st); \
  }
  DTN_SMALL(1, 4) DTN_SMALL(1, 8) DTN_SMALL(1, 16)
  DTN_SMALL(2, 4) DTN_SMALL(2, 8) DTN_SMALL(2, 16)
  DTN_SMALL(4, 4) DTN_SMALL(4, 8) DTN_SMALL(4, 16)
#undef DTN_SMALL
  return hipGetLastError();
}

hipError_t launch_couple(const CoupleDesc* cd, int count, int blocks_per, const int* ip, const DevBufs& B,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_couple, dim3(blocks_per, count), dim3(256), 0, s, cd, ip, B);
  return hipGetLastError();
}

hipError_t launch_base_inv(const BaseBlock* blocks, int count, const DevBufs& B, DevStatus* st, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_base_inv2, dim3(count), dim3(kInv2Threads), kInv2Lds, s, blocks, B, st);
  return hipGetLastError();
}

hipError_t launch_reset(const LargeMerge* lm, int nlm, const DevBufs& B, DevStatus* st, hipStream_t s) {
  const int n = nlm > 0 ? nlm : 1;
  hipLaunchKernelGGL(k_reset, dim3((n + 255) / 256), dim3(256), 0, s, lm, nlm, B, st);
  return hipGetLastError();
}

hipError_t launch_large_gather(const LargeMerge* lm, int nlm, int blocks_per, const int* ip, const DevBufs& B,
                               hipStream_t s) {
  if (nlm <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_large_gather, dim3(blocks_per, nlm), dim3(256), 0, s, lm, ip, B);
  return hipGetLastError();
}

hipError_t launch_gje_panel(int nt, int r, int w, const LargeMerge* lm, int nlm, int c0, int* ip, const DevBufs& B,
                            DevStatus* st, hipStream_t s) {
  if (nlm <= 0) return hipSuccess;
  if (nt == 256 && r == 1 && w == 32)
    hipLaunchKernelGGL((k_gje_panel<256, 1, 32>), dim3(nlm), dim3(256), 0, s, lm, c0, ip, B, st);
  else if (nt == 512 && r == 2 && w == 32)
    hipLaunchKernelGGL((k_gje_panel<512, 2, 32>), dim3(nlm), dim3(512), 0, s, lm, c0, ip, B, st);
  else if (nt == 1024 && r == 2 && w == 16)
    hipLaunchKernelGGL((k_gje_panel<1024, 2, 16>), dim3(nlm), dim3(1024), 0, s, lm, c0, ip, B, st);
  else if (nt == 1024 && r == 4 && w == 8)
    hipLaunchKernelGGL((k_gje_panel<1024, 4, 8>), dim3(nlm), dim3(1024), 0, s, lm, c0, ip, B, st);
  else if (nt == 1024 && r == 8 && w == 4)
    hipLaunchKernelGGL((k_gje_panel<1024, 8, 4>), dim3(nlm), dim3(1024), 0, s, lm, c0, ip, B, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gje_swap(const LargeMerge* lm, int nlm, int imax, int c0, const int* ip, const DevBufs& B,
                           hipStream_t s) {
  if (nlm <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gje_swap, dim3((imax + 255) / 256, nlm), dim3(256), 0, s, lm, c0, ip, B);
  return hipGetLastError();
}

hipError_t launch_gje_kmap(const LargeMerge* lm, int nlm, int imax, int* ip, hipStream_t s) {
  if (nlm <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gje_kmap, dim3(nlm), dim3(256), (size_t)imax * sizeof(int), s, lm, ip);
  return hipGetLastError();
}

hipError_t launch_gemm_batched(const GemmDesc* descs, int ndesc, int tiles, int cfg, const DevBufs& B,
                               const int* ip, hipStream_t s, int tile_base, int prec, int mode, const LargeMerge* lm) {
  if (ndesc <= 0 || tiles <= 0) return hipSuccess;
  if (mode < 0 || mode > 3) return hipErrorInvalidValue;
#define DTN_GEMM(CFG_, CT_, MODE_, NT_) \
  hipLaunchKernelGGL((k_gemm_batched<CFG_, CT_, MODE_>), dim3(tiles), dim3(NT_), 0, s, descs, ndesc, tile_base, B, ip, lm)
#define DTN_GEMM_MODES(CFG_, CT_, NT_)          \
  switch (mode) {                               \
    case 0: DTN_GEMM(CFG_, CT_, 0, NT_); break; \
    case 1: DTN_GEMM(CFG_, CT_, 1, NT_); break; \
    case 2: DTN_GEMM(CFG_, CT_, 2, NT_); break; \
    default: DTN_GEMM(CFG_, CT_, 3, NT_); break; \
  }
  if (prec == 1) {   // FP32 MFMA (mixed-precision plans), 128 x 128 or 64 x 64 tiles; plain A or the generic form
    if (cfg == 2) {
      if (mode == 0) DTN_GEMM(2, float, 0, 512);
      else DTN_GEMM(2, float, 3, 512);
    } else {
      if (mode == 0) DTN_GEMM(0, float, 0, 256);
      else DTN_GEMM(0, float, 3, 256);
    }
  } else if (cfg == 2 || cfg == 1) {
    DTN_GEMM_MODES(2, double, 512)
  } else if (cfg == 3) {
    DTN_GEMM_MODES(3, double, 256)
  } else if (cfg == 4) {
    DTN_GEMM_MODES(4, double, 256)
  } else {
    DTN_GEMM_MODES(0, double, 256)
  }
#undef DTN_GEMM_MODES
#undef DTN_GEMM
  return hipGetLastError();
}

int gemm_tile_m(int cfg) { return cfg == 0 ? 64 : cfg == 3 || cfg == 4 ? 32 : 128; }
int gemm_tile_n(int cfg) { return cfg == 0 ? 64 : cfg == 3 || cfg == 4 ? 32 : 128; }

hipError_t launch_gemm_single(GemmDesc D, int cfg, const DevBufs& B, hipStream_t s) {
  D.tiles_m = (D.M + gemm_tile_m(cfg) - 1) / gemm_tile_m(cfg);
  D.tiles_n = (D.N + gemm_tile_n(cfg) - 1) / gemm_tile_n(cfg);
  const int tiles = D.tiles_m * D.tiles_n;
  if (tiles <= 0) return hipSuccess;
  if (D.transA || D.kmapA >= 0 || D.ksplit > 1) return hipErrorInvalidValue;   // plain A, whole K only
  if (cfg == 2 || cfg == 1)
    hipLaunchKernelGGL(k_gemm_single<2>, dim3(tiles), dim3(512), 0, s, D, B);
  else
    hipLaunchKernelGGL(k_gemm_single<0>, dim3(tiles), dim3(256), 0, s, D, B);
  return hipGetLastError();
}

// Partial sums of a launch of up to `cols` columns (cols is rounded up the way the launcher pads it).
size_t apply_splitk_workspace(int nb, int cols) {
  cols = std::max(1, std::min(cols, kApplyMaxCols));
  const int padded = cols <= 4 ? 4 : cols <= 8 ? 8 : cols <= 16 ? 16 : cols <= 32 ? 32
                                 : (cols + kApplyGroup - 1) / kApplyGroup * kApplyGroup;
  return (size_t)(apply_splits(nb) + 1) * nb * padded * sizeof(double);   // partial sums + G transposed
}

int apply_splitk_max_cols() { return kApplyMaxCols; }

// Split-K workspace of the allocation-free apply (dtn_apply_device_noalloc): one array per device,
// resident until the process ends, sized for kNoAllocMaxNb ring rows and kNoAllocCols columns per chunk
// in every split (16 at most) plus the transposed G chunk.  Host code never passes this name to a kernel: it takes the device address returned
// by noalloc_scratch_address.
static __device__ __align__(256) double scratch[17 * kNoAllocCols * kNoAllocMaxNb];
static_assert(sizeof(scratch) == (size_t)17 * kNoAllocCols * kNoAllocMaxNb * sizeof(double), "scratch size");

hipError_t noalloc_scratch_address(double** p) {
  *p = nullptr;
  return hipGetSymbolAddress((void**)p, HIP_SYMBOL(scratch));
}

size_t noalloc_scratch_bytes() { return sizeof(scratch); }

// Y[:, 0:k] = T G[:, 0:k] in launches of at most `chunk` (<= kApplyMaxCols) columns; part holds
// apply_splitk_workspace(nb, chunk) bytes: the split sums (apply_splits(nb) x nb x gld) followed by G
// transposed (nb x gld), gld = the launch's columns rounded up to its column groups.  A column's
// summation order depends on nb only.
hipError_t launch_apply_splitk(const double* T, int nb, const double* G, int ldg, int k, double* Y, int ldy,
                               double* part, hipStream_t s, int chunk) {
  const int S = apply_splits(nb), tiles = (nb + 63) / 64;
  chunk = std::max(1, std::min(chunk, kApplyMaxCols));
  for (int c0 = 0; c0 < k; c0 += chunk) {
    const int kk = std::min(chunk, k - c0);
    const int kc = kk <= 4 ? 4 : kk <= 8 ? 8 : kk <= 16 ? 16 : kApplyGroup;
    const int groups = (kk + kc - 1) / kc;
    const int gld = groups * kc;
    const double* Gc = G + (long long)c0 * ldg;
    if (kc <= 8) {
      // narrow: G read in place, no transpose pass
      const dim3 grid((unsigned)apply_grid(tiles, S, 1));
      if (kc == 4) hipLaunchKernelGGL(k_apply_narrow<4>, grid, dim3(256), 0, s, T, nb, Gc, ldg, kk, part);
      else hipLaunchKernelGGL(k_apply_narrow<8>, grid, dim3(256), 0, s, T, nb, Gc, ldg, kk, part);
    } else {
      // wider: G transposed into the workspace first, two rows per lane
      double* Gt = part + (long long)S * nb * gld;
      hipLaunchKernelGGL(k_apply_transpose, dim3((unsigned)tiles, (unsigned)((gld + 63) / 64)), dim3(256), 0, s,
                         Gc, ldg, nb, kk, gld, Gt);
      const dim3 grid((unsigned)apply_grid((nb + 127) / 128, S, groups));
      if (kc == 16) hipLaunchKernelGGL((k_apply_splitk<16, 2>), grid, dim3(256), 0, s, T, nb, Gt, gld, groups, part);
      else hipLaunchKernelGGL((k_apply_splitk<kApplyGroup, 2>), grid, dim3(256), 0, s, T, nb, Gt, gld, groups, part);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long cnt = (long long)nb * kk;
    hipLaunchKernelGGL(k_apply_reduce, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, part, nb, kk,
                       gld, S, Y + (long long)c0 * ldy, ldy);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pchol(const PcholDesc* descs, int count, const DevBufs& B, int* ip, DevStatus* st, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pchol, dim3(count), dim3(256), 0, s, descs, B, ip, st);
  return hipGetLastError();
}

hipError_t launch_root_rows(const double* S, double* T, int n, int reading, const double* coef, double h2, double cs,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_root_rows, dim3(1024), dim3(256), 0, s, S, T, n, reading, coef, h2, cs, (double)(n - 1));
  return hipGetLastError();
}

hipError_t launch_body_gather(const BodyJob* jobs, int count, int chunks, const int* ip, const int* bnodes,
                              const DevBufs& B, double h2, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_body_gather, dim3(count, std::max(1, chunks)), dim3(256), 0, s, jobs, ip, bnodes, B, h2);
  return hipGetLastError();
}

hipError_t launch_body_out(const double* C, int nb, int cnt, const int* user, double scale, double* F, int ldf,
                           hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  const long long tot = (long long)nb * cnt;
  hipLaunchKernelGGL(k_body_out, dim3((unsigned)std::min<long long>(2048, (tot + 255) / 256)), dim3(256), 0, s, C, nb,
                     cnt, user, scale, F, ldf);
  return hipGetLastError();
}

hipError_t launch_scale_copy(const double* S, double* T, long long cnt, double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(1024), dim3(256), 0, s, S, T, cnt, scale);
  return hipGetLastError();
}

}  // namespace dtn

namespace dtn {
hipError_t kernels_init() {
  hipError_t e = hipFuncSetAttribute((const void*)k_small_schur, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(152 * 1024));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_base_inv2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kInv2Lds);
  if (e != hipSuccess) return e;
#define DTN_SMALL_PAIR(EA_, BC_) (const void*)k_small_fast<EA_, BC_, true>, (const void*)k_small_fast<EA_, BC_, false>
  for (const void* f : {DTN_SMALL_PAIR(1, 4), DTN_SMALL_PAIR(1, 8), DTN_SMALL_PAIR(1, 16), DTN_SMALL_PAIR(2, 4),
                        DTN_SMALL_PAIR(2, 8), DTN_SMALL_PAIR(2, 16), DTN_SMALL_PAIR(4, 4), DTN_SMALL_PAIR(4, 8),
                        DTN_SMALL_PAIR(4, 16)}) {
#undef DTN_SMALL_PAIR
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kSmallFastLds));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace dtn
