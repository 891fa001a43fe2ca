/*
 * dtn.h - build and apply the boundary Dirichlet-to-Neumann (DtN) operator of
 *         -Lap u + b u_x + c u_y + d u = 0 on the unit square, on one AMD
 *         Instinct MI355X (gfx950).
 *
 * Method: Gillman & Martinsson, "An O(N) algorithm for constructing the
 * solution operator to 2D elliptic boundary value problems in the absence of
 * body loads".  The problem statement is the paper's Section 1.1 (only the
 * normal derivative on the boundary is sought, for many Dirichlet data g);
 * the build is the nested-dissection scheme of Section 3 (quadtree of
 * Section 2, leaf Schur complements of Section 3.1, pairwise merges of
 * Section 3.2, full algorithm of Section 3.3) with the structured-matrix
 * acceleration of Section 6 at the top levels; the solve stage applies the
 * operator (Section 1.1, step 2).
 *
 * Discretisation (Section 7): n x n grid of nodes (i h, j h), h = 1/(n-1),
 * five-point stencil.  Node (i, j) has linear index i + n*j.  The boundary
 * ring has nb = 4(n-1) nodes, listed counter-clockwise from the corner (0,0):
 * ring index r = s*(n-1) + t, t = 0..n-2, with side s = 0 south (t, 0),
 * 1 east (n-1, t), 2 north (n-1-t, n-1), 3 west (0, n-1-t).  The operator T
 * maps Dirichlet values g on the ring to (g(b) - u(b_in))/h at every
 * non-corner ring node b (b_in its inward neighbour, u the discrete solution
 * with u = g on the ring); rows and columns of the four corners are zero.
 * Convection uses the centred difference (u_e - u_w)/(2h) unless
 * DTN_CONV_PAPER selects the paper's printed (u_e - u_w)/h.
 *
 * Conventions for every call:
 *   - matrices are column-major (Fortran order) float64;
 *   - a "host" pointer is ordinary CPU memory, a "device" pointer is memory
 *     on the handle's GPU (hipMalloc / torch CUDA tensor);
 *   - inputs are borrowed for the duration of the call and never retained;
 *   - calls return DTN_OK (0) or a negative DTN_E* code, builds return NULL
 *     on failure; dtn_last_error() then describes the failure (thread-local).
 *   - distinct handles are independent; a handle is read-only after its
 *     build, so applies on one handle may run concurrently on different
 *     streams.
 */
#ifndef DTN_H
#define DTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DTN_OK          0
#define DTN_EINVAL     (-1)   /* bad argument: n, leaf, k, pointer, leading dimension, NaN/Inf data */
#define DTN_ENOMEM     (-2)   /* device or host allocation failed / memory budget exceeded          */
#define DTN_ESINGULAR  (-3)   /* a leaf interior or merge interface block has a pivot of magnitude
                                 <= DTN_PIVOT_RTOL times the block's largest entry                   */
#define DTN_EDEVICE    (-4)   /* HIP runtime error, or no gfx950 device                             */
#define DTN_EBUSY      (-5)   /* serving: request cannot be admitted now                            */
#define DTN_ENOTSUP    (-6)   /* option combination not supported                                   */
#define DTN_ERANK      (-7)   /* tol > 0: an off-diagonal block still had sketch directions above tol
                                 when its range finder reached the 96-column rank cap, so the
                                 factored block could not be certified to tol (no handle returned) */

#define DTN_PIVOT_RTOL 1e-11

enum dtn_precision { DTN_FP64 = 0, DTN_MIXED = 1 };
enum dtn_batching  { DTN_FUSED = 0, DTN_PLAIN = 1 };
enum dtn_conv      { DTN_CONV_CENTRAL = 0, DTN_CONV_PAPER = 1 };
enum dtn_memspace  { DTN_MEM_HOST = 0, DTN_MEM_DEVICE = 1 };
enum dtn_pivoting  { DTN_PIVOT_AUTO = 0, DTN_PIVOT_PARTIAL = 1 };
enum dtn_ring_rows { DTN_RING_R1 = 0, DTN_RING_R2 = 1, DTN_RING_R3 = 2 };
enum dtn_coef_form { DTN_COEF_PDE = 0, DTN_COEF_NETWORK = 1 };

typedef struct dtn_op dtn_op;

/* Build options.  Initialise with dtn_build_desc_init() and then set fields. */
typedef struct dtn_build_desc {
    int n;                 /* grid nodes per side, >= 3                                            */
    const double* b;       /* n*n coefficients at the nodes, index i + n*j; NULL means 0.          */
    const double* c;       /*   Values on the boundary ring are used only by DTN_RING_R2.          */
    const double* d;
    int coeff_mem;         /* DTN_MEM_HOST or DTN_MEM_DEVICE: where b, c, d live                   */
    int leaf;              /* maximum leaf box side in nodes, >= 4 (Section 2's N_leaf as a side)   */
    double tol;            /* 0: uncompressed merges.  > 0: the off-diagonal blocks S13, S31, S24,
                              S42 of the top merges are replaced by low-rank factors Q B (a
                              randomized range finder truncated where a sketch column falls to
                              tol times the block's largest one) and the Schur update uses the
                              factored products (Section 6, Step 2; Section 7's local tolerance).
                              Ranks are capped at 96 per block: a block that reaches the cap with
                              directions still above tol fails the build with DTN_ERANK.  The
                              unpivoted fast path only (a build that falls back to partial
                              pivoting is uncompressed)                                           */
    int hbs_min_level;     /* with tol > 0: compress merges whose parent box is at quadtree level
                              <= hbs_min_level (root = 0); -1: compress the merges whose children's
                              Schur complements are at least 1000 x 1000 (Section 6, closing
                              remark)                                                             */
    int precision;         /* DTN_FP64, or DTN_MIXED: the X and Schur products of every large merge,
                              and the products of the interface-block inversions below the two top
                              levels, run on FP32 matrix cores (FP64 operands rounded to FP32,
                              FP32 sums, FP64 results); the 128-block inverses and the top two
                              levels' inversions stay FP64.  Relative error ~1e-7 times the
                              problem's conditioning.  Applied only when d >= 0 at every interior node (d
                              NULL, or host arrays checked at build time): with d < 0 somewhere
                              the interface blocks can be near-resonant and FP32 products at any
                              level exceed a relative error of 1e-6, so such builds run in FP64.
                              dtn_stats.precision reports the precision that ran.              */
    int batching;          /* DTN_FUSED: every merge of a level in shared launches (default);
                              DTN_PLAIN: one merge at a time                                      */
    int conv;              /* DTN_CONV_CENTRAL (default) or DTN_CONV_PAPER                         */
    int device;            /* HIP device ordinal (default 0)                                       */
    void* stream;          /* hipStream_t to build on; NULL uses the library's stream              */
    int pivoting;          /* DTN_PIVOT_AUTO (default): eliminate without cross-row pivoting (the
                              Schur complements are strongly diagonally dominant, Section 3.2's
                              remark) while monitoring every pivot and the element growth of the
                              large merges' block inverses; if a pivot falls below 1e-5 of its
                              block's largest entry, or an entry of a 128-block or of its half-level
                              Schur complement exceeds 16 times the merge's largest K_ii entry, the
                              build is redone with DTN_PIVOT_PARTIAL.
                              DTN_PIVOT_PARTIAL: Gauss-Jordan with partial pivoting throughout.   */
    int ring_rows;         /* Equations of the ring nodes, whose Schur complement S' (times 1/h) is the
                              output.  Section 3.1 keeps as boundary set the outermost ring of
                              unknowns with their full equations; Section 1.1 asks for the normal
                              derivative.  DTN_RING_R1 (default): one-sided differences
                              u(b) - u(b_in) on the non-corner ring nodes, zero corner rows: T is
                              the DtN map (T 1 = 0 when d = 0).  DTN_RING_R2: every ring node keeps
                              its full h^2-scaled five-point row of the n x n grid with the
                              couplings to nodes outside the grid dropped (the ring as outermost
                              ring of unknowns, zero data beyond it); this reading uses b, c, d at
                              the ring nodes.  DTN_RING_R3: the R1 rows plus the ring-cycle
                              Laplacian (weight 1 between consecutive ring nodes).  R2 and R3 are
                              formed from the R1 Schur complement by an exact row update after the
                              root merge (same build cost).                                        */
    int coef_form;         /* DTN_COEF_PDE (default): the five-point discretisation of the PDE.
                              DTN_COEF_NETWORK: an equilibrium problem on the grid's network of
                              links (Section 7.1's random Laplacians): the equation of an interior
                              node k is sum over its four links of sigma (u_k - u_l) + h^2 d_k u_k
                              = 0, with b[i + n j] the conductance of link (i,j)-(i+1,j) and
                              c[i + n j] that of (i,j)-(i,j+1) (both required); a ring node's R1
                              row is the current sigma (u(b) - u(b_in)) through its inward link,
                              so the operator is symmetric and annihilates constants; conv is
                              ignored; ring_rows R1 or R3.                                          */
    int capture_level;     /* -1 (default): none.  L >= 0: keep a device copy of the Schur complement
                              of every box of quadtree level L (level 0 the whole grid; below the
                              user's leaves the boxes of the in-leaf dissection, down to sides of
                              8 nodes) as the build forms it, for dtn_level_count / dtn_level_box
                              (checks of intermediate levels, Section 3.3).  DTN_EINVAL if L is
                              deeper than the dissection.                                          */
    int pad0;
    size_t budget_bytes;   /* 0 (default): no limit.  > 0: device bytes the build may allocate (plans
                              not yet cached, including the partial-pivoting fallback plan of
                              DTN_PIVOT_AUTO, the operator T and captured levels); a build that
                              would need more returns DTN_ENOMEM before allocating anything.  For
                              dtn_build_many the first descriptor's budget covers the group,
                              checked against the sum of the problems' single-build needs.        */
    double kii_tol;        /* 0 (default): interface blocks K_ii inverted densely.  > 0: at the merges
                              the compression rule selects (hbs_min_level >= 0: parent levels <=
                              it; -1: both children's Schur complements >= 1000 x 1000), K_ii is
                              put in equal-rank HBS form at this local tolerance and inverted by
                              Algorithm 1 of Section 5.1, and X = K_ii^{-1} K_ie is formed by
                              Algorithm 2 (Section 6, Step 1), instead of the dense recursive
                              inverse.  The HBS tree runs over the interface nodes in pairs (each
                              node of the first child followed by its neighbour across the shared
                              edge), the order in which K_ii's off-diagonal blocks have low rank;
                              a basis reaching the rank cap (128) fails the build with DTN_ERANK.
                              Indefinite K_ii (d < 0) amplify kii_tol in the result about a
                              thousandfold.  Dense off-diagonal products only: requires tol = 0 and
                              DTN_FP64 (DTN_EINVAL otherwise); the partial-pivoting fallback stays
                              dense.  The structured merges of a phase run concurrently on the
                              library's own streams after the work queued on the build's stream,
                              which waits for them.  dtn_stats.structured_merges counts the merges
                              covered (in dtn_build_many, those of all its problems).              */
    int n_body;            /* 0 (default): no body loads.  > 0: also build the operator F of Section
                              7.3 from loads at n_body interior nodes to the boundary fluxes
                              (v = T g + F f_hat, the load f_hat_q entering node q's equation as
                              the right-hand side f): each box's condensed right-hand sides are
                              carried through the leaf elimination and every merge (Section 3.2's
                              update).  Single-problem builds with tol = 0, kii_tol = 0 and the R1
                              ring rows (DTN_EINVAL otherwise).  The loads' buffers (every loaded
                              box's right-hand sides, a phase's scratch, F) are not charged
                              against budget_bytes.                                              */
    int pad1;
    const int* body_nodes; /* n_body host ints: node i + n j of each load, 0 < i, j < n - 1, no
                              repeats (borrowed for the call); F's column q is body_nodes[q]'s   */
} dtn_build_desc;

/* HBS (telescoping) form of a handle's operator (Section 4), see dtn_hbs_compress. */
typedef struct dtn_hbs_info {
    int leaf;                       /* largest leaf interval of the index tree                     */
    int levels;                     /* depth of the index tree (root = level 0)                    */
    int nodes;                      /* tree nodes                                                  */
    int launches;                   /* kernel launches of one HBS apply                            */
    double tol;                     /* local tolerance of the interpolative decompositions         */
    size_t bytes;                   /* device bytes of the factors (D, U, V and sibling blocks)    */
    int max_rank[32];               /* largest row or column rank per tree level (root: 0)         */
} dtn_hbs_info;

/* Per-handle statistics of the build that produced it. */
typedef struct dtn_stats {
    int n, nb, leaf, levels;        /* levels = quadtree depth L                                  */
    int precision, batching;        /* precision that ran (DTN_MIXED may run DTN_FP64)            */
    double build_ms;                /* wall time of the build on its stream (device sync included) */
    double flops;                   /* algorithmic flops of the build (merge and leaf models)      */
    double level_ms[32];            /* per quadtree level, leaves at index L                      */
    double level_flops[32];         /* algorithmic flops per quadtree level, leaves at index L    */
    int    max_rank[32];            /* largest compressed off-diagonal rank per level (0: dense)  */
    double min_pivot_ratio;         /* smallest |pivot| / block max seen in the build             */
    int pivoting_used;              /* DTN_PIVOT_AUTO if the unpivoted path was accepted          */
    size_t op_bytes;                /* device bytes held by the handle                            */
    size_t peak_workspace_bytes;    /* device workspace used during the build                     */
    int structured_merges;          /* merges of the build whose K_ii went through HBS (kii_tol)   */
    double max_growth;              /* element growth of the large merges' 128-block inverses: the
                                       largest |entry| of a block or of its half-level Schur
                                       complement over the merge's largest |K_ii| entry (0: none,
                                       or a build that ran with partial pivoting)                  */
} dtn_stats;

/* Fill a descriptor with defaults (FP64, fused, central convection, device 0, tol 0, host b,c,d). */
void dtn_build_desc_init(dtn_build_desc* desc);

/* Build T for the problem of Section 1.1 (host coefficient arrays, library stream, device 0).
 * Returns a handle owning the device-resident operator, or NULL (see dtn_last_error). */
dtn_op* dtn_build(int n, const double* b, const double* c, const double* d, int leaf, double tol);

/* Build with explicit options. */
dtn_op* dtn_build_ex(const dtn_build_desc* desc);

/* Build `count` problems together in one plan (the fused form of Section 3.3's level-by-level
 * merges across problems): phase k of every problem, counted from its base boxes up, runs in the
 * same launches, so problems of different n and leaf share kernels level by level.  Every
 * descriptor must name the same device, stream, batching, precision and pivoting (DTN_EINVAL
 * otherwise).  A weak pivot in any problem redoes the whole group with partial pivoting.
 * out[q] receives the handle of descs[q].  Returns DTN_OK, or an error code with every out[q]
 * NULL. */
int dtn_build_many(int count, const dtn_build_desc* descs, dtn_op** out);

/* Y = T G for k Dirichlet vectors (the paper's solve stage).  Host pointers: G is nb x k with
 * leading dimension nb, Y is nb x k with leading dimension nb, caller-allocated, not aliasing G.
 * Synchronous.  k >= 1. */
int dtn_apply(dtn_op* op, const double* G, int k, double* Y);

/* Device variant: dG (ldg >= nb) and dY (ldy >= nb) on the handle's device; enqueued on `stream`
 * (hipStream_t; NULL = library stream); asynchronous with respect to the host. */
int dtn_apply_device(dtn_op* op, const double* dG, int ldg, int k, double* dY, int ldy, void* stream);

/* Allocation-free variant of dtn_apply_device, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, layout and result: bitwise the same Y as dtn_apply_device (a column's summation order
 * depends on nb only).  It calls no allocator: the split-K partial sums and transposed G of k <= 64
 * live in one library-owned device array per GPU (17 x 32 x 8188 doubles = 35.6 MB, held until the
 * process ends), and k > 64 runs the MFMA GEMM, which needs no workspace.  Limit: nb <= 8188 (n <= 2048);
 * larger operators return DTN_EINVAL.  Every call on one GPU shares that array: calls that overlap
 * on one GPU (other streams, other host threads) race and must be ordered by the caller.  The
 * device must have been initialised by a build on it (DTN_EDEVICE otherwise).  Asynchronous. */
int dtn_apply_device_noalloc(dtn_op* op, const double* dG, int ldg, int k, double* dY, int ldy, void* stream);

/* Compress the handle's operator T into hierarchically block-separable form (Section 4: binary tree over
 * the ring positions, leaves of at most `leaf` positions, 8 <= leaf <= 64; factors D, U, V and sibling
 * blocks B of def1-def6).  The bases are interpolative decompositions from 160 random samples per
 * node, truncated at the local tolerance tol (> 0) relative to each block row's or column's largest
 * pivot; ranks are capped at 128 (DTN_ERANK if a basis would need more).  The factors stay on the
 * device with the handle.  drop_dense != 0 releases the dense T: every later apply of the handle
 * (dtn_apply, dtn_apply_device, the serving loop) then runs the telescoping apply, dtn_export_dense
 * returns the matrix the factors stand for, and dtn_apply_device_noalloc returns DTN_EINVAL.
 * Synchronous.  Returns DTN_OK or a negative code. */
int dtn_hbs_compress(dtn_op* op, double tol, int leaf, int drop_dense);

/* Describe the handle's HBS factors (DTN_EINVAL if it has none). */
int dtn_hbs_get(const dtn_op* op, dtn_hbs_info* out);

/* Y = T_HBS G through the telescoping factorisation (tele1-tele3): upward pass with the V bases,
 * sibling blocks, downward pass with the U bases, leaf blocks; 2 L + 1 batched launches for a tree of
 * depth L.  Device pointers and stream as dtn_apply_device; the handle keeps a workspace for it. */
int dtn_apply_hbs_device(dtn_op* op, const double* dG, int ldg, int k, double* dY, int ldy, void* stream);

/* Inverse of the handle's operator in HBS form (Section 5.1, Algorithm 1; with ring_rows R2, h^{-1}
 * times the result is the paper's solution operator G = S^{-1} of Section 7).  First equal-rank HBS
 * factors of T are built as in dtn_hbs_compress (same tree, samples and rank cap) but with one skeleton
 * set and one interpolation matrix per node for its block row and block column together (the
 * interpolative decomposition of both sides' stacked samples at tol, so U = V); then, finer levels first, each node's
 * block (its leaf block, or its children's reduced blocks joined by the sibling blocks) is inverted
 * by Gauss-Jordan elimination with partial pivoting (blocks of at most 256 rows), giving the node's
 * E, F* and G factors and its reduced block (V^T Dt^{-1} U)^{-1} for the parent; the root keeps the
 * inverse of its joined block.  The forward factors are released; the inverse factors stay on the
 * device with the handle (replacing earlier ones).  Needs the dense T (DTN_EINVAL after
 * drop_dense).  DTN_ESINGULAR if a block to invert has a zero or non-finite pivot; DTN_ERANK as
 * dtn_hbs_compress.  Synchronous. */
int dtn_hbs_invert(dtn_op* op, double tol, int leaf);

/* Describe the handle's inverse factors (bytes: E, F* and G of every node and the root block;
 * max_rank: the equal ranks per level).  DTN_EINVAL if it has none. */
int dtn_hbs_inverse_get(const dtn_op* op, dtn_hbs_info* out);

/* Y = T^{-1} X through Algorithm 2 (Section 5.1): upward pass with F*, the root block, downward pass
 * with E and G, leaves; 3 L + 1 batched launches for a tree of depth L >= 1.  Device pointers (ldx,
 * ldy >= nb, X and Y not aliasing) and stream as dtn_apply_device; uses the handle's HBS apply
 * workspace (applies of the handle on different streams are ordered).  Asynchronous. */
int dtn_apply_hbs_inverse_device(dtn_op* op, const double* dX, int ldx, int k, double* dY, int ldy, void* stream);

/* nb = 4(n-1) of the handle, or a negative error code. */
int dtn_nb(const dtn_op* op);

/* Boxes captured by a build with capture_level >= 0 (Section 3.3: the Schur complements of one
 * quadtree level, each of its box's ring), or a negative code (DTN_EINVAL: none captured). */
int dtn_level_count(const dtn_op* op);

/* Box q (0 <= q < dtn_level_count) of the captured level: rect = {x0, x1, y0, y1}, the nodes
 * x0 <= i < x1, y0 <= j < y1; S (host, may be NULL to query rect only) receives its Schur complement,
 * m x m column-major with lds >= m, m = 2(x1 - x0 - 1) + 2(y1 - y0 - 1), rows and columns in ring
 * order counter-clockwise from the box's south-west corner (node (x0, y0)).  The box's own matrix is
 * M' restricted to its nodes (ring nodes of the grid keep the ring-row reading R1).  Synchronous. */
int dtn_level_box(const dtn_op* op, int q, int rect[4], double* S, int lds);

/* Copy the dense operator (nb x nb) to host memory T with leading dimension ldt >= nb. */
int dtn_export_dense(const dtn_op* op, double* T, int ldt);

/* A handle holding a given dense operator: T is an nb x nb column-major host matrix (leading dimension
 * ldt >= nb, borrowed, copied) placed on `device`.  The handle takes the calls a built handle takes
 * apart from the build's own records (dtn_level_*; its stats hold n and nb only): applies, HBS
 * compression and inversion (Sections 4 and 5.1, on any square matrix), export, serving.  n is
 * nb / 4 + 1 when 4 divides nb (the ring of that grid), else 0.  With dtn_export_dense it keeps an
 * operator across processes.  Synchronous; NULL on error (dtn_last_error). */
dtn_op* dtn_import_dense(int nb, const double* T, int ldt, int device);

/* Body loads (a build with n_body > 0, Section 7.3): the number of loads (0 without), the operator
 * F (nb x n_body, column-major) copied to host memory with leading dimension ldf >= nb, and its device
 * pointer (leading dimension nb, owned by the handle, NULL without loads). */
int dtn_body_count(const dtn_op* op);
int dtn_body_get(const dtn_op* op, double* F, int ldf);
const double* dtn_body_ptr(const dtn_op* op);

/* Y = T G + F Q on device memory (Section 7.3's solution operator applied to Dirichlet data G, nb x k,
 * and body loads Q, n_body x k, column-major with leading dimensions ldg, ldq, ldy) on `stream`
 * (NULL: the library's).  DTN_EINVAL for a handle built without loads. */
int dtn_apply_body_device(dtn_op* op, const double* dG, int ldg, const double* dQ, int ldq, int k, double* dY,
                          int ldy, void* stream);

/* Device pointer to the resident dense operator (column-major, leading dimension nb), or NULL.
 * Owned by the handle; valid until dtn_free. */
const double* dtn_device_ptr(const dtn_op* op);

/* Statistics of the handle's build. */
int dtn_stats_get(const dtn_op* op, dtn_stats* out);

/* Release the handle and its device memory.  NULL is a no-op. */
void dtn_free(dtn_op* op);

/* Description of the last error on the calling thread ("" if none). */
const char* dtn_last_error(void);

/* The code (DTN_OK or a negative DTN_E* value) of the last dtn_build / dtn_build_ex call on the
 * calling thread; those calls return NULL on failure, and this says why. */
int dtn_last_build_code(void);

/* Kernel-level profiling.  When enabled, every kernel launch of builds and applies on the
 * calling process is bracketed by HIP events on the stream it runs on; per kernel family the
 * library accumulates the number of launches, the summed event time and the algorithmic work
 * of those launches (flops of the dense contractions they perform, bytes they must move).
 * Enabling adds two event records per recorded launch.  Counters are process-wide. */
typedef struct dtn_prof_entry {
    char name[32];                  /* kernel family, e.g. "gemm_schur", "gje_panel"                */
    long long launches;
    double total_ms;                /* summed launch durations (HIP events)                         */
    double flops;                   /* algorithmic flops of those launches                          */
    double bytes;                   /* algorithmic HBM bytes of those launches                      */
} dtn_prof_entry;

int dtn_profile_enable(int on);              /* returns DTN_OK                                      */
/* Restrict recording to the named families (comma-separated, e.g. "gemm_x_t128,gemm_schur_t128");
 * NULL or "" records every family.  Launches of other families then carry no events, so a
 * measurement of one kernel adds nothing to the launches around it.  Returns DTN_OK. */
int dtn_profile_select(const char* families);
int dtn_profile_reset(void);                 /* zero all counters                                   */

/* Host-only self-check of the execution plan for an n x n problem with the given leaf, tol (0:
 * dense; > 0: compressed top levels, Section 6), mixed (nonzero: FP32 products at the lower levels),
 * fast (nonzero: the unpivoted batched path; 0: the pivoted path) and sym (0: a problem with
 * convection; 1: without convection, b = c = NULL, and d >= 0, whose Schur products run half at every
 * level; 2: without convection but d < 0 somewhere, mirrored products below the two top levels only):
 * builds the plan of the
 * quadtree build (Section 5) on the host, touches no device, and checks that every device
 * descriptor (products, diagonal-block inverses, coupling steps, small tasks, large merges,
 * range-finder steps) addresses only the buffers the plan allocates and that every launch's tiles
 * are numbered without gaps.  Returns DTN_OK, or DTN_EINVAL with the first violation in
 * dtn_last_error(). */
int dtn_plan_check(int n, int leaf, double tol, int mixed, int fast, int sym);

/* dtn_plan_check with every FP64 product launch that can take it forced to one tile configuration
 * (tile 0: 64 x 64, 2: 128 x 128 where both sides of every product reach 128, 3: 32 x 32, 4: 32 x 32 with
 * K in chunks of 64; -1: the planner's own choice), as the autotuner may choose.  Host-only. */
int dtn_plan_check_tiles(int n, int leaf, double tol, int mixed, int fast, int sym, int tile);

/* Host-only: plan the body loads of a single-problem build (n, leaf, fast or partially pivoted path,
 * sym as in dtn_plan_check) at the nodes i + n j in nodes[0 .. n_body) and check that every gather,
 * inversion and product of their right-hand-side updates stays inside its buffers. */
int dtn_body_plan_check(int n, int leaf, int fast, int sym, int n_body, const int* nodes);

/* Autotuner of the build's product tiles.  dtn_tune builds the problem of desc (fused batching) reps
 * times under each tile configuration (64 x 64, 128 x 128, 32 x 32, 32 x 32 with deep K chunks, and the
 * planner's fixed thresholds) with HIP events around every product launch, and records for every launch
 * shape (signature: descriptor count, tiles, largest M, N, K, operand form, epilogue flags) the fastest
 * tile in a process-wide table.  Later plans take their tiles from the table while it is enabled
 * (dtn_tune_enable, default on); plans built before are rebuilt.  If the environment variable
 * DTN_TUNE_CACHE names a file, the table is read from it when a device is first used and written to
 * it after each dtn_tune (JSON: {"arch": "gfx950", "tiles": {signature: tile}}).  Returns the number of
 * launch shapes timed (>= 0) or a negative code; report (if non-NULL) receives a JSON description
 * of the timings, cut to len - 1 characters. */
int dtn_tune(const dtn_build_desc* desc, int reps, char* report, int len);
int dtn_tune_enable(int on);             /* 0: plans use the fixed thresholds; nonzero: the table      */
int dtn_tune_clear(void);                /* empty the table                                           */
int dtn_tune_save(const char* path);     /* write the table as JSON                                   */
int dtn_tune_load(const char* path);     /* merge a JSON table (DTN_EINVAL: unreadable, malformed, or
                                            written for another architecture)                        */
int dtn_tune_size(void);                 /* entries in the table                                      */

/* Host-only: the device bytes of the build plans a dtn_build_ex(desc) call may allocate (its plan
 * and, for DTN_PIVOT_AUTO, the partial-pivoting plan it falls back to; plans already cached in
 * this process count zero) in *bytes, and the plan-cache key of its plan (NUL-terminated, cut to
 * keylen - 1 characters) in key.  Builds whose keys differ hold separate workspaces; the serving
 * loop charges each key's bytes once against its HBM budget.  Touches no device.  Returns DTN_OK or
 * DTN_EINVAL (NULL desc or bytes, bad n or leaf). */
int dtn_plan_footprint(const dtn_build_desc* desc, size_t* bytes, char* key, int keylen);
int dtn_profile_read(dtn_prof_entry* out, int max);   /* fills up to max entries, returns count */

/* ------------------------------------------------------------------------------------------
 * Serving: resident operators and continuous batching of applies (the solve stage of
 * Section 1.1 run as a service: many Dirichlet data arriving over time against operators that
 * stay in HBM).  One server drives one device with its own threads and streams:
 *   - applies are queued per operator; a scheduler thread repeatedly takes the operator with the
 *     oldest pending request and concatenates the columns of its pending requests (arrival order,
 *     whole requests, at most max_batch_cols columns) into one pass over T (256 columns per pass;
 *     wider batches take one pass per 256); four pipeline slots
 *     on four streams overlap the host staging of one batch, the device work of the batches
 *     after it and the completion of the ones before it (a completer thread copies results out;
 *     a small pool of helper threads splits each batch's host copies);
 *   - every batch runs the same split-K apply kernels, whose per-column summation order does not
 *     depend on the batch: a request's Y is bitwise the same whether it ran alone or batched;
 *   - builds submitted to the server run on a builder thread and stream of their own, so applies
 *     continue while they run;
 *   - admission by HBM footprint: resident operators (nb^2 * 8 bytes each), the build plans'
 *     workspaces and the staging buffers are charged against budget_bytes.  A build or operator
 *     that can never fit is refused (DTN_EBUSY); a build that does not fit now waits in the build
 *     queue until operators are removed.
 * Host pointers G and Y of a submitted apply are borrowed until dtn_srv_wait returns for its
 * ticket.  All dtn_srv_* calls are thread-safe.
 * ------------------------------------------------------------------------------------------ */
typedef struct dtn_srv dtn_srv;

typedef struct dtn_srv_result {
    int status;                     /* DTN_OK or the request's error code                          */
    int op_id;                      /* apply: its operator; build: id of the new resident operator */
    int k;                          /* apply: number of columns                                    */
    int batch_cols;                 /* apply: columns of the batch it ran in                       */
    long long t_arrival_ns;         /* scheduled arrival (dtn_srv_now_ns clock)                    */
    long long t_start_ns;           /* its batch was formed                                        */
    long long t_done_ns;            /* Y copied back to the caller's buffer / build finished       */
} dtn_srv_result;

typedef struct dtn_srv_stats {
    long long applies_done, builds_done, solves_done, batches, refused;
    size_t budget_bytes, resident_bytes;
    int resident_ops;
    double p50_ms, p99_ms, mean_ms;   /* apply latency, scheduled arrival to completion             */
    double mean_batch_cols;
    double span_s;                    /* first arrival to last completion of the counted applies    */
    double solves_per_s;              /* solves_done / span_s                                       */
    double build_p50_ms, build_p99_ms;   /* build latency, arrival to the operator being resident  */
} dtn_srv_stats;

/* One request of a replayed arrival schedule: an apply, or a build when `build` is non-NULL (then
 * op_id, k, G and Y are ignored and the new operator becomes resident when the build completes). */
typedef struct dtn_srv_request {
    long long t_offset_ns;          /* arrival time after the start of the replay                  */
    int op_id;
    int k;
    const double* G;                /* host, nb x k, leading dimension nb                          */
    double* Y;                      /* host, nb x k, leading dimension nb                          */
    const dtn_build_desc* build;    /* non-NULL: a build request (host coefficient arrays)         */
} dtn_srv_request;

/* Create a server on `device` charging at most budget_bytes of HBM; max_batch_cols >= 1 caps the
 * columns of one batch (and of one request).  Returns NULL on error. */
dtn_srv* dtn_srv_create(size_t budget_bytes, int device, int max_batch_cols);

/* Make a built operator resident (the server borrows it; the caller frees it after removing it
 * or after dtn_srv_destroy).  Returns op_id >= 0, DTN_EBUSY if its footprint exceeds the remaining
 * budget, or another negative code. */
int dtn_srv_add_op(dtn_srv* srv, dtn_op* op);

/* Remove a resident operator.  DTN_EBUSY while requests on it are pending.  Operators built by
 * the server are freed; borrowed ones are returned to the caller's ownership. */
int dtn_srv_remove_op(dtn_srv* srv, int op_id);

/* nb of a resident operator, or a negative code. */
int dtn_srv_op_nb(dtn_srv* srv, int op_id);

/* Queue Y = T_op G (host pointers, nb x k, 1 <= k <= max_batch_cols).  Returns a ticket >= 0 or a
 * negative code.  The arrival time is the time of the call. */
long long dtn_srv_submit_apply(dtn_srv* srv, int op_id, const double* G, int k, double* Y);

/* Queue a build (host or device coefficients as in dtn_build_ex; the descriptor's device and
 * stream are ignored).  The coefficient arrays are borrowed until the ticket completes.  Returns a
 * ticket >= 0, or DTN_EBUSY when the operator and its workspace can never fit the budget. */
long long dtn_srv_submit_build(dtn_srv* srv, const dtn_build_desc* desc);

/* 1 if the ticket has completed, 0 if pending, negative for an unknown ticket. */
int dtn_srv_poll(dtn_srv* srv, long long ticket);

/* Block until the ticket completes, fill *out (may be NULL) and release the ticket.  Returns the
 * request's status. */
int dtn_srv_wait(dtn_srv* srv, long long ticket, dtn_srv_result* out);

/* Submit `count` apply requests at their scheduled arrival times (open loop: the calling thread
 * sleeps until each arrival; latency counts from the scheduled time even when submission lags).
 * tickets[q] receives the ticket of reqs[q].  Returns DTN_OK or the first submission error. */
int dtn_srv_replay(dtn_srv* srv, int count, const dtn_srv_request* reqs, long long* tickets);

/* Latency/throughput statistics of the applies completed since the last reset. */
int dtn_srv_stats_get(dtn_srv* srv, dtn_srv_stats* out);
int dtn_srv_stats_reset(dtn_srv* srv);

/* The server's clock (steady, nanoseconds). */
long long dtn_srv_now_ns(void);

/* Drain every queued request, stop the threads and release the server's memory and the operators
 * it built.  NULL is a no-op. */
void dtn_srv_destroy(dtn_srv* srv);

/* Library version string. */
const char* dtn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DTN_H */
