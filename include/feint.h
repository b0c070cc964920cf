/*
 * feint.h -- C interface of libfeint, element-by-element numerical
 * integration for geometrically bilinear prismatic finite elements of degree
 * p = 1..7 on AMD Instinct MI355X (gfx950).
 *
 * Method: Krużel & Banaś, "Vectorized OpenCL implementation of numerical
 * integration for higher order finite elements" (arXiv 1310.1194), Sec. 2
 * (eqs. (1)-(2), Algorithm 1) and Sec. 4 (bilinear prism).  The Laplace term
 * of the paper is generalised to convection-diffusion-reaction with a load
 * vector: for every element e with constant D (3x3), beta (3), c and f,
 *
 *   A_ab = sum_q w_q det J_q [ grad phi_a . D grad phi_b
 *                              + phi_a (beta . grad phi_b) + c phi_a phi_b ]
 *   b_a  = sum_q w_q det J_q f phi_a
 *
 * (row a = test function, grad phi = J^{-T} times the reference gradient,
 * signed det J).  Quadrature: Duffy-collapsed Gauss-Legendre with p+1 points
 * per direction, (p+1)^3 points.  Basis: Lagrange on the equispaced triangle
 * lattice (i/p, j/p), i+j <= p (j outer, i inner) times 1D Lagrange on the
 * p+1 Gauss-Lobatto nodes (ascending); shape function a = k*ntri + t.
 * Prism vertices: v0..v2 the bottom triangle (zeta = -1), v3..v5 the top one
 * (zeta = +1), v(a+3) above v(a).
 *
 * Conventions for every entry point below:
 *   - Array arguments are DEVICE pointers owned by the caller, element-major,
 *     C-contiguous.  The library never frees or retains them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call is asynchronous on that stream and allocates nothing; the
 *     reference tables of a degree are built and uploaded by
 *     feint_prepare() (called implicitly on first use when the stream is
 *     not capturing).
 *   - Host-detectable errors (null pointer, bad degree or form, ne < 0, a
 *     capturing stream with unprepared tables) are returned before any work is
 *     enqueued.  ne == 0 is a no-op that returns FEINT_OK.
 *   - Device-detected conditions do not abort: bit 0 of *dev_status is set
 *     (atomic OR) when some det J <= 0; results still use the signed det J.
 *   - Calls are safe from several host threads on distinct streams.
 */
#ifndef FEINT_H
#define FEINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FEINT_OK = 0,
    FEINT_ERR_INVALID_ARG = -1,
    FEINT_ERR_UNSUPPORTED_DEGREE = -2,
    FEINT_ERR_UNSUPPORTED_FORM = -3,
    FEINT_ERR_NOT_PREPARED = -4,
    FEINT_ERR_HIP = -5,
    FEINT_ERR_TOO_LARGE = -6
} feint_status;

/* Arithmetic of the contraction A_e = sum_q B_q^T W_q B_q.  The Jacobian,
   its determinant and inverse and the per-point coefficient block W_q are
   always computed in FP64.  The load vector is formed by the same
   contraction (a spare padded column carries w det J f), so it carries the
   form's precision; where a kernel has no spare column (the point-by-point
   kernels at p = 7, the factorised hexahedral kernel at p = 3 and 7) it is
   accumulated in FP64. */
typedef enum {
    FEINT_FP64 = 0,    /* FP64 MFMA, FP64 outputs */
    FEINT_FP32 = 1,    /* FP32 MFMA, FP32 outputs */
    FEINT_BF16X3 = 2,  /* split bf16 hi+lo, 3 MFMA products, FP32 accumulate/outputs */
    FEINT_FP16X3 = 3   /* split fp16 hi+lo with power-of-two scaling, FP32 outputs */
} feint_form;

/* Per-element inputs, FP64, ne elements. */
typedef struct {
    const double *coords;  /* [ne][6][3] prism vertices */
    const double *D;       /* [ne][3][3] row-major diffusion tensor, used as
                              grad phi_a^T D grad phi_b (need not be symmetric) */
    const double *beta;    /* [ne][3] convection vector */
    const double *c;       /* [ne] reaction coefficient */
    const double *f;       /* [ne] source */
    int64_t ne;
} feint_elements;

/* (p+1)^2 (p+2)/2 shape functions (the paper's Table 1, prism row) and
   (p+1)^3 quadrature points; -1 when p is outside [1,7]. */
int feint_nshp(int p);
int feint_nq(int p);

/* Size in bytes of one output element of a form (8 for FP64, else 4);
   0 for an unknown form. */
size_t feint_elem_size(feint_form form);

/* Build and upload the reference tables of degree p (quadrature points and
   weights; shape-function values and reference gradients at every point, in
   every precision the forms use).  Idempotent and thread-safe.  Must be
   called before a stream that will be captured into a graph starts
   capturing.  Library-owned memory; released by feint_shutdown(). */
feint_status feint_prepare(int p);

/* Forward integration (Algorithm 1 generalised to CDR + load vector; the
   paper's eq. (2) as a sum over quadrature points).
     A          [ne][n][n]  row a = test function; double for FEINT_FP64,
                            float otherwise
     b          [ne][n]     same dtype as A
     xq         nullable, [ne][nq][3] double: mapped quadrature points
     dev_status nullable, one uint32 on the device, OR-ed with 1 if some
                det J <= 0 (the caller clears it). */
feint_status feint_integrate(const feint_elements *el, int p, feint_form form,
                             void *A, void *b, double *xq, uint32_t *dev_status,
                             void *stream);

/* Spatially varying coefficients: the same integration with D, beta, c and f
   given at each element's six vertices and evaluated at every quadrature
   point with the geometry shape functions, D(x_q) = sum_a N_a(xi_q) D_a
   (N_a = lambda_a (1-zeta)/2, N_{a+3} = lambda_a (1+zeta)/2; a field in the
   bilinear space of the geometry, continuous across elements when the
   vertex values are shared).  Outputs, forms, variants and errors as
   feint_integrate; all inputs are device pointers, FP64. */
typedef struct {
    const double *coords;  /* [ne][6][3] prism vertices */
    const double *D;       /* [ne][6][3][3] diffusion tensor at each vertex */
    const double *beta;    /* [ne][6][3] convection vector at each vertex */
    const double *c;       /* [ne][6] reaction at each vertex */
    const double *f;       /* [ne][6] source at each vertex */
    int64_t ne;
} feint_fields;
feint_status feint_integrate_fields(const feint_fields *el, int p, feint_form form,
                                    void *A, void *b, double *xq, uint32_t *dev_status,
                                    void *stream);

/* Adjoint of feint_integrate: gradients of
       L = sum_e <G_e, A_e> + <g_e, b_e>
   with respect to every element's inputs.  G [ne][n][n] and g [ne][n] have
   the form's output dtype (double for FEINT_FP64, float for FEINT_FP32; the
   split forms are not differentiated: FEINT_ERR_UNSUPPORTED_FORM).
   Outputs (overwritten, FP64): dcoords [ne][6][3], dD [ne][3][3] (all nine
   entries treated as independent), dbeta [ne][3], dc [ne], df [ne].  The
   per-point Jacobians are recomputed, never stored. */
feint_status feint_integrate_adjoint(const feint_elements *el, int p, feint_form form,
                                     const void *G, const void *g,
                                     double *dcoords, double *dD, double *dbeta,
                                     double *dc, double *df, void *stream);

/* Block shapes of the adjoint kernel: each wave holds a TA x TB block of
   16x16 tiles of G_e (several waves per element for large n, their partial
   gradients summed with FP64 atomics).  feint_adjoint_autotune times every
   compiled shape on the caller's buffers (`reps` repetitions, HIP events on
   `stream`, synchronising on it), keeps the fastest for later calls of this
   (p, form) and returns its time in *best_ms (nullable); ne = 0 or reps < 1
   gives INVALID_ARG.  tile_get/set read or force the choice; tile_describe
   writes "TAxTB" (16x16 tiles of G per wave) or "TKxTBf" (the kernel
   factorised along zeta: TK row indices k by TB column tiles).  Count is 0 and get is -1 for unsupported (p, form). */
int feint_adjoint_tile_count(int p, feint_form form);
int feint_adjoint_tile_get(int p, feint_form form);
feint_status feint_adjoint_tile_set(int p, feint_form form, int tile);
feint_status feint_adjoint_tile_describe(int p, feint_form form, int tile, char *buf, size_t len);
feint_status feint_adjoint_autotune(const feint_elements *el, int p, feint_form form,
                                    const void *G, const void *g, double *dcoords, double *dD,
                                    double *dbeta, double *dc, double *df, int reps, double *best_ms,
                                    void *stream);

/* ---- Mixed-degree batches -------------------------------------------------
   Elements of degrees 1..6 in any order run as one persistent,
   degree-bucketed launch (the paper's Sec. 2.2 advice to group elements by
   type and degree so that reference data is fetched once per group).
   Outputs are packed in element order: element e's matrix starts at
   offA[e] elements of the output dtype, its vector at offb[e], where offA
   and offb are the exclusive prefix sums of n(p_e)^2 and n(p_e). */
typedef struct feint_mixed_plan feint_mixed_plan;

/* Create a plan for at most ne_max elements of form FEINT_FP32 or
   FEINT_FP64.  Allocates the plan's device scratch (bucket counters,
   permutation, work queue: about 40 bytes per element) and prepares the
   tables of degrees 1..6. */
feint_status feint_mixed_plan_create(int64_t ne_max, feint_form form, feint_mixed_plan **plan);

/* Degree bucketing for a batch: histogram of p[ne] (int8, device), stable
   scatter into degree order (heaviest degree first), and the packed output
   offsets offA[ne+1], offb[ne+1] (int64, device; entry ne holds the totals).
   Enqueued on `stream`; elements with p outside [1,6] are an error reported
   through bit 1 of *dev_status (nullable) and get empty outputs. */
feint_status feint_mixed_bucket(feint_mixed_plan *plan, const int8_t *p, int64_t ne,
                                int64_t *offA, int64_t *offb, uint32_t *dev_status,
                                void *stream);

/* The persistent degree-bucketed launch over the bucketing of the last
   feint_mixed_bucket call on this plan (same ne, same p). */
feint_status feint_integrate_mixed(feint_mixed_plan *plan, const feint_elements *el,
                                   void *A_packed, void *b_packed,
                                   const int64_t *offA, const int64_t *offb,
                                   uint32_t *dev_status, void *stream);

/* Capture bucketing + persistent launch for fixed pointers into a HIP graph
   held by the plan (replaces any previous one), then instantiate it.
   Capturing runs nothing: the captured bucketing first happens when the
   graph is launched, so until then feint_integrate_mixed and
   feint_mixed_autotune still see only the last eager feint_mixed_bucket
   (INVALID_ARG, with no launch, if there was none for this ne).  The
   pointers are baked into the graph: the caller keeps every captured
   buffer alive until the plan is destroyed or captures again. */
feint_status feint_mixed_graph_capture(feint_mixed_plan *plan, const feint_elements *el,
                                       const int8_t *p, void *A_packed, void *b_packed,
                                       int64_t *offA, int64_t *offb, uint32_t *dev_status,
                                       void *stream);
/* Replay the captured graph on `stream`. */
feint_status feint_mixed_graph_launch(feint_mixed_plan *plan, void *stream);
/* Time each compiled set of per-degree tile shapes of the persistent launch
   (`reps` launches each, after bucketing with feint_mixed_bucket) and keep
   the fastest in the plan; *best_ms receives its mean launch time. */
feint_status feint_mixed_autotune(feint_mixed_plan *plan, const feint_elements *el,
                                  void *A_packed, void *b_packed, const int64_t *offA,
                                  const int64_t *offb, int reps, double *best_ms, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the
   mixed-degree integration of a batch -- bucketing of p[ne] (int8, device)
   into offA[ne+1], offb[ne+1] and the persistent launch into the packed
   A_packed, b_packed, as feint_mixed_bucket followed by
   feint_integrate_mixed with the first compiled tile set -- without a plan
   and without allocating.  Its bucketing scratch is a fixed device array of
   the library (about 4.3 MB per GPU, held until the process ends) that
   every call on a GPU shares and that keeps the last call's contents;
   calls that overlap on one GPU (two streams, two threads) race on it and
   must be serialised by the caller.  At most FEINT_NOALLOC_MAX_NE elements
   (FEINT_ERR_TOO_LARGE beyond, before any launch, with the reason in
   feint_last_error).  The tables of degrees 1..6 must have been prepared
   (feint_prepare) on the current device: otherwise FEINT_ERR_NOT_PREPARED,
   since preparing them would allocate.  The caller sizes A_packed and
   b_packed (sum of n(p_e)^2 and n(p_e) values of the form's dtype).  form
   is FEINT_FP32 or FEINT_FP64; errors otherwise as for feint_integrate_mixed
   (elements with p outside [1,6] set bit 1 of *dev_status). */
#define FEINT_NOALLOC_MAX_NE 1048576
feint_status feint_integrate_mixed_noalloc(const feint_elements *el, const int8_t *p, feint_form form,
                                           void *A_packed, void *b_packed, int64_t *offA, int64_t *offb,
                                           uint32_t *dev_status, void *stream);
/* Number of compiled tile sets of the plan's form, the one in use, and a
   forced choice. */
int feint_mixed_tile_count(const feint_mixed_plan *plan);
int feint_mixed_tile_get(const feint_mixed_plan *plan);
feint_status feint_mixed_tile_set(feint_mixed_plan *plan, int tile);
/* Describe tile set `tile` into buf: the per-degree shapes for p = 1..6,
   comma-separated, each "TMxTN" (16x16 MFMA tiles per wave) or "vL"
   (vector-ALU kernel, L lanes per element).  INVALID_ARG for a null plan or
   buffer or an index out of range. */
feint_status feint_mixed_tile_describe(const feint_mixed_plan *plan, int tile, char *buf, size_t len);
void feint_mixed_plan_destroy(feint_mixed_plan *plan);

/* ---- Tile autotuning -------------------------------------------------------
   Each (degree, form) has several compiled variants: tile shapes of the MFMA
   kernels (16x16 output tiles per wave), for FP64 and FP32 the kernels that
   contract per triangle point (the rule and the basis factorised along
   zeta: fewer flops, the default from p = 3), and for FP64 and FP32 at
   p <= 3 vector-ALU kernels that give each element a group of lanes (Sec.
   2.2's operation counts make the contraction too small at low degree to
   fill MFMA tiles; which side of the crossover a degree falls on is what
   the autotuner measures).  All variants compute the same A and b to the
   form's rounding.  feint_autotune times each candidate with HIP
   events on the caller's inputs and outputs (ne elements, `reps`
   repetitions) and keeps the fastest for later calls; feint_tile_get/set
   read or force the choice (index into the candidate list). */
int feint_tile_count(int p, feint_form form);
int feint_tile_get(int p, feint_form form);
feint_status feint_tile_set(int p, feint_form form, int tile);
/* Describe candidate `tile` into buf: "TMxTN" output tiles per wave, with
   "s" (table staged in LDS), "sa" (A operands staged), "p" (K loop
   software-pipelined) or "c" (shape functions computed at each point from
   their tensor-product factors, no table read: the paper's SC strategy,
   Sec. 4), or "KxTNf" (contraction per triangle point, or per plane point
   for hexahedra: K zeta rows of shape functions by TN column tiles per
   wave, FP64 and FP32),
   or "vL" (vector-ALU kernel, L lanes per element); "o2" marks a
   two-waves-per-SIMD register budget. */
feint_status feint_tile_describe(int p, feint_form form, int tile, char *buf, size_t len);
feint_status feint_autotune(const feint_elements *el, int p, feint_form form,
                            void *A, void *b, int reps, double *best_ms, void *stream);

/* ---- Quadrature rules (Sec. 2, Table 3) -------------------------------------
   The entry points above integrate with the collapsed Gauss rule, (p+1)^3
   points.  The paper's Table 3 counts N_I = 6, 18, 48, 80, 150, 231, 336
   points for p = 1..7, which is a fully symmetric triangle rule of degree 2p
   (3, 6, 12, 16, 25, 33, 42 points, positive weights, interior points)
   times p+1 Gauss-Legendre points in zeta: products of shape functions are
   integrated exactly on affine prisms (the paper's accuracy requirement)
   with 36-52 % fewer points.  Point q = k * ntri + t (Gauss point k in zeta
   ascending, triangle point t in orbit order: centroid, 3-orbits, 6-orbits). */
typedef enum {
    FEINT_RULE_COLLAPSED = 0,  /* (p+1)^3 collapsed Gauss-Legendre */
    FEINT_RULE_SYMMETRIC = 1   /* symmetric triangle rule of degree 2p x (p+1) Gauss */
} feint_rule;

/* Number of points of a rule; -1 for p outside [1,7] or an unknown rule. */
int feint_nq_rule(int p, feint_rule rule);
/* Host copy of a rule's points: pts [nq][4] = (xi1, xi2, zeta, w), host
   memory owned by the caller with room for cap points (INVALID_ARG if too
   small).  No device work. */
feint_status feint_rule_points(int p, feint_rule rule, double *pts, int64_t cap);
/* feint_prepare for the tables of degree p on `rule`. */
feint_status feint_prepare_rule(int p, feint_rule rule);
/* Forward integration on `rule`: exactly one of el (element-constant
   coefficients) and fl (vertex fields) is non-null, else INVALID_ARG.
   Outputs, forms, errors and the det J flag as feint_integrate; xq, when
   given, is [ne][feint_nq_rule(p, rule)][3]. */
feint_status feint_integrate_rule(const feint_elements *el, const feint_fields *fl, int p, feint_form form,
                                  feint_rule rule, void *A, void *b, double *xq, uint32_t *dev_status,
                                  void *stream);
/* Compiled variants per (degree, form, rule), chosen and described as for
   the collapsed rule (feint_tile_*; those calls are these with
   FEINT_RULE_COLLAPSED).  feint_autotune_rule takes el or fl as
   feint_integrate_rule does. */
int feint_rule_tile_count(int p, feint_form form, feint_rule rule);
int feint_rule_tile_get(int p, feint_form form, feint_rule rule);
feint_status feint_rule_tile_set(int p, feint_form form, feint_rule rule, int tile);
feint_status feint_rule_tile_describe(int p, feint_form form, feint_rule rule, int tile, char *buf,
                                      size_t len);
feint_status feint_autotune_rule(const feint_elements *el, const feint_fields *fl, int p, feint_form form,
                                 feint_rule rule, void *A, void *b, int reps, double *best_ms, void *stream);
/* The adjoint on quadrature rule `rule` (the gradients of the forward pass
   feint_integrate_rule computes with element-constant coefficients);
   arguments, outputs and errors otherwise as feint_integrate_adjoint.  The
   adjoint block-shape choice (feint_adjoint_tile_*) serves both rules. */
feint_status feint_integrate_adjoint_rule(const feint_elements *el, int p, feint_form form, feint_rule rule,
                                          const void *G, const void *g, double *dcoords, double *dD,
                                          double *dbeta, double *dc, double *df, void *stream);

/* ---- Hexahedral elements (Table 1, tensor-product basis) --------------------
   The same integration (CDR element matrix and load vector, W_q in FP64) on
   geometrically trilinear hexahedra: reference cube [-1,1]^3, vertex v =
   i + 2j + 4k at (2i-1, 2j-1, 2k-1); shape functions phi_a = L_i(xi)
   L_j(eta) L_k(zeta), a = (k (p+1) + j) (p+1) + i, L the Lagrange basis on
   the p+1 Gauss-Lobatto nodes; (p+1)^3 Gauss-Legendre points, q = (k n1 +
   j) n1 + i.  Inputs as feint_elements with coords [ne][8][3]; outputs
   A [ne][n][n] (row = test function), b [ne][n], n = (p+1)^3; xq (nullable)
   [ne][(p+1)^3][3]; dev_status as feint_integrate.  All four forms (FP64
   and FP32 on the 16x16x4 MFMA kernels, point by point or factorised along
   zeta per plane point; bf16x3 and fp16x3 on the 16x16x32 split kernel).
   Variants, tile selection and autotuning as for prisms. */
int feint_hex_nshp(int p);
int feint_hex_nq(int p);
feint_status feint_prepare_hex(int p);
feint_status feint_integrate_hex(const feint_elements *el, int p, feint_form form, void *A, void *b,
                                 double *xq, uint32_t *dev_status, void *stream);
int feint_hex_tile_count(int p, feint_form form);
int feint_hex_tile_get(int p, feint_form form);
feint_status feint_hex_tile_set(int p, feint_form form, int tile);
feint_status feint_hex_tile_describe(int p, feint_form form, int tile, char *buf, size_t len);
feint_status feint_hex_autotune(const feint_elements *el, int p, feint_form form, void *A, void *b, int reps,
                                double *best_ms, void *stream);

/* ---- Tetrahedral elements (Table 1, complete basis) -------------------------
   The same integration on affine tetrahedra: reference tetrahedron {xi >= 0,
   xi1 + xi2 + xi3 <= 1}, vertices v0..v3 at 0, e1, e2, e3, x = v0 + J xi with
   the edge vectors v_i - v0 as the columns of J; Lagrange basis on the
   lattice (i/p, j/p, k/p), i + j + k <= p, k outer, j, i inner (n = (p+1)
   (p+2)(p+3)/6); (p+2)^3 collapsed Gauss points, q = (k n1 + j) n1 + i with
   zeta = (1+c)/2, eta = (1+b)(1-zeta)/2, xi = (1+a)(1-eta-zeta)/2 (products
   of shape functions integrated exactly).  Inputs as feint_elements with
   coords [ne][4][3]; outputs, forms, errors and variants as for hexahedra. */
int feint_tet_nshp(int p);
int feint_tet_nq(int p);
feint_status feint_prepare_tet(int p);
feint_status feint_integrate_tet(const feint_elements *el, int p, feint_form form, void *A, void *b,
                                 double *xq, uint32_t *dev_status, void *stream);
int feint_tet_tile_count(int p, feint_form form);
int feint_tet_tile_get(int p, feint_form form);
feint_status feint_tet_tile_set(int p, feint_form form, int tile);
feint_status feint_tet_tile_describe(int p, feint_form form, int tile, char *buf, size_t len);
feint_status feint_tet_autotune(const feint_elements *el, int p, feint_form form, void *A, void *b, int reps,
                                double *best_ms, void *stream);

/* ---- The paper's own term (eq. (1), Sec. 2) on its quadrature ---------------
   The stiffness matrix of the Laplace operator alone,
     A_ab = sum_q w_q det J_q grad phi_a . grad phi_b,
   with no coefficients and no load vector (the paper integrates exactly this
   term, Sec. 2, and counts its work in Table 2), on the symmetric prism rule
   of feint_integrate_rule (the N_I points of Table 3).  coords [ne][6][3]
   FP64 (device); A [ne][n][n], row-major, double for FEINT_FP64 and float
   for FEINT_FP32 (the paper's precision); the split forms give
   UNSUPPORTED_FORM.  xq (nullable) [ne][N_I][3] mapped points; dev_status
   bit 0 as for feint_integrate.  ne == 0 is a no-op; null coords or A with
   ne > 0 give INVALID_ARG.  Tile calls and the autotuner as for the other
   element types ("vL", "KxTNf"). */
feint_status feint_integrate_laplace(const double *coords, int64_t ne, int p, feint_form form, void *A,
                                     double *xq, uint32_t *dev_status, void *stream);
int feint_laplace_tile_count(int p, feint_form form);
int feint_laplace_tile_get(int p, feint_form form);
feint_status feint_laplace_tile_set(int p, feint_form form, int tile);
feint_status feint_laplace_tile_describe(int p, feint_form form, int tile, char *buf, size_t len);
feint_status feint_laplace_autotune(const double *coords, int64_t ne, int p, feint_form form, void *A, int reps,
                                    double *best_ms, void *stream);

/* ---- Global assembly (Sec. 2) ----------------------------------------------
   The element matrices and load vectors of one degree are summed into a CSR
   matrix and a right-hand side through the element-to-global dof map.
   Elements are coloured so that no two elements of a colour share a global
   dof; each colour is one launch and adds its entries without atomics.

   feint_asm_plan_create: dofs is a HOST array [ne][n] (int32, n = nshp(p)):
   the global dof of every local shape function, in the library's local
   order (a = k*ntri + t: triangle lattice node t = (i/p, j/p), j outer, i
   inner; Gauss-Lobatto node k in zeta, ascending).  ndof bounds the ids
   (0 <= dof < ndof < 2^31).  Builds, on the host, the CSR pattern (row i
   holds every dof sharing an element with i, columns ascending), the
   offsets of each element entry inside its row and a greedy colouring, and
   uploads them to the current device (plan-owned memory).  INVALID_ARG for
   null pointers, ne <= 0, an n that is no prism size, ids out of range or a
   dof repeated within an element; TOO_LARGE if a row exceeds 65535 columns.

   feint_assemble: A [ne][n][n] and b [ne][n] as produced by feint_integrate
   with `form` (double for FEINT_FP64, float otherwise), values [nnz] and rhs
   [ndof] of the same dtype; all device pointers owned by the caller.
   values and rhs are cleared first unless `accumulate` is nonzero.  Entry
   (i, j) receives the contributions of the elements in colour order.
   Asynchronous on `stream`; the plan must outlive the work it enqueues. */
typedef struct feint_asm_plan feint_asm_plan;
feint_status feint_asm_plan_create(const int32_t *dofs, int64_t ne, int n, int64_t ndof,
                                   feint_asm_plan **plan);
/* nnz of the pattern and number of colours (either output nullable). */
feint_status feint_asm_plan_info(const feint_asm_plan *plan, int64_t *nnz, int *ncolors);
/* Copy the pattern into caller device buffers row_ptr [ndof+1] (int64) and
   col_idx [nnz] (int32), asynchronously on `stream`. */
feint_status feint_asm_plan_pattern(const feint_asm_plan *plan, int64_t *row_ptr, int32_t *col_idx,
                                    void *stream);
/* Colour of every element into a host array [ne]. */
feint_status feint_asm_plan_colors(const feint_asm_plan *plan, int32_t *color_of);
feint_status feint_assemble(feint_asm_plan *plan, feint_form form, const void *A, const void *b,
                            void *values, void *rhs, int accumulate, void *stream);
void feint_asm_plan_destroy(feint_asm_plan *plan);

const char *feint_status_string(feint_status s);
/* Last HIP error text seen by the library on this thread ("" if none). */
const char *feint_last_error(void);
/* Release every library-owned table (after all work has completed). */
void feint_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* FEINT_H */
