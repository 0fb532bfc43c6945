/*
 * nsmf.h -- matrix-free Newton-Stokes operator engine for AMD MI355X (gfx950).
 *
 * C ABI of the engine that applies, matrix-free on hexahedral Q_k x P_{k-1}^disc or
 * Q_k x Q_{k-2}^disc meshes (k = 2, 3, 4; Sec. 3.2.2) with 2:1 hanging nodes:
 *   - the nonlinear residual of the Glen-law Stokes problem, eq. (weak) with the
 *     viscosity of eq. (glen) (Sec. 2.1-2.2 of the paper);
 *   - the Newton-linearised saddle-point operator A(u) = [[F(u), B^T], [B, 0]]
 *     of Sec. 4.1, F built from the 4th-order tensor of eq. (rank4) and the basal
 *     Robin term of eq. (robin) (eq. (newton), Sec. 2.3);
 *   - the vector-Jacobian product of the residual with respect to u, p, the
 *     per-element log rate factor and the per-face basal friction.
 *
 * Conventions (all entry points):
 *   - Every vector argument is a DEVICE pointer on the context's device, owned by
 *     the caller, contiguous and at least 8-byte aligned; it must stay alive until
 *     the work enqueued on the context's stream has completed.  Host arrays appear
 *     only in nsmf_mesh and are copied during nsmf_upload_mesh.
 *   - Velocity vectors are structure-of-arrays [3][n_nodes] (x, y, z components),
 *     pressure vectors are element-major [n_el][n_p] on each element's reference cube:
 *       P_{k-1} (nsmf_mesh.pspace = NSMF_PSPACE_P): n_p = k(k+1)(k+2)/6, basis of
 *         normalised Legendre products Lhat_i(xi) Lhat_j(eta) Lhat_l(zeta), i+j+l <= k-1,
 *         ordered by (i+j+l, l, j, i);
 *       Q_{k-2} (NSMF_PSPACE_Q): n_p = (k-1)^3, the Lagrange basis on the tensor product
 *         of the k-1 Gauss points per direction (Sec. 6), mode i + (k-1)(j + (k-1) l).
 *   - Work is enqueued asynchronously on the stream given by nsmf_set_stream
 *     (default: the null stream); no call synchronises except nsmf_upload_mesh
 *     (which validates the geometry on the device) and nsmf_kernel_time.
 *   - Errors are returned as nsmf_status codes; a message is kept per context
 *     (nsmf_last_error).  Argument and mesh errors are detected before any work is
 *     enqueued.  A device fault surfaces as NSMF_EHIP on the same or a later call.
 *   - Calls on one context are not thread-safe.
 *
 * Normal Dirichlet condition (eq. (robin), second line): velocity components flagged
 * in nsmf_mesh.dmask are eliminated.  The state and residual use P u (P zeroes the
 * flagged components), residual rows of flagged components equal u itself, and
 * the Jacobian is J_c = P K P + (I - P), which keeps it symmetric.
 */
#ifndef NSMF_H
#define NSMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nsmf_ctx nsmf_ctx;

typedef enum {
  NSMF_OK = 0,
  NSMF_EINVAL = -1,  /* bad argument: NULL pointer, size or precision out of range   */
  NSMF_EHIP = -2,    /* HIP runtime error (allocation, launch, device fault)          */
  NSMF_EMESH = -3,   /* invalid mesh: node id out of range, inconsistent hanging mask,
                        inverted element (det J <= 0 at a quadrature point)            */
  NSMF_ESTATE = -4,  /* call order: no mesh uploaded or no state set                   */
  NSMF_EUNSUP = -5,  /* unsupported: k outside 2..4, geometry that is not column-mapped */
  NSMF_ENOMEM = -6   /* device memory exhausted                                        */
} nsmf_status;

typedef enum {
  NSMF_FP64 = 0,          /* double vectors, FP64 arithmetic                              */
  NSMF_FP32 = 1,          /* float vectors; quadrature-point data rounded once from FP64;
                             FP32 contractions and FP32 accumulation                       */
  NSMF_FP32_BF16OPS = 2   /* as NSMF_FP32 with the 1D reference-element operators (basis
                             values and derivatives at Gauss points) rounded to bfloat16  */
} nsmf_prec;

/* Mesh description (host memory, copied by nsmf_upload_mesh).
 *
 * Elements are hexahedra with (k+1)^3 Gauss-Lobatto nodes each (Sec. 3.2.1); element
 * slot a = a0 + P*(a1 + P*a2), P = k+1, a_d the node index along reference axis d.
 * The isoparametric map of an element is its Q_k interpolant of the slot coordinates
 * obtained through the same restriction R_e as the velocity (so hanging faces follow
 * the coarse neighbour: the mesh is watertight).
 *
 * Hanging nodes (Sec. 3.2.1, figure "hanging"): a slot lying on a face or edge of a
 * coarser neighbour holds in elem_nodes the id of the neighbour's node at the SAME
 * local index along the face/edge tangent directions; the engine interpolates those
 * values in place with the 1D child-interval interpolation matrices.  cmask bits:
 *   0..2   child position (hx, hy, hz) of the element inside its refined parent;
 *   3..8   hanging face -x, +x, -y, +y, -z, +z;
 *   9..20  hanging edge 4*dir + s0 + 2*s1, dir 0/1/2 = parallel to x/y/z, (s0, s1)
 *          the side (0 low / 1 high) along the two other axes in increasing order.
 *
 * Periodic lateral boundaries (the slab problem of Sec. 4.3): nodes on opposite periodic
 * boundaries are one node (one id in elem_nodes; hanging faces across the boundary name the
 * neighbour's nodes as usual) and coords holds one position per node.  period[d] > 0 is the
 * translation between the identified boundaries along axis d (x or y); the engine moves every
 * slot coordinate of an element by a multiple of it to within half a period of the element's
 * first slot before building the geometry, so an element must be shorter than half a period
 * along a periodic axis.  period = {0, 0, 0}: no periodic axis.
 *
 * Nodal frames (eq. (robin), second line, u . n = 0 on a curved base): a node listed in
 * frame_nodes holds its velocity unknowns in the local frame Q of frames (u = Q u_hat, the
 * columns of Q the local axes); its dmask bits and every vector entry of the node (x_u, y_u,
 * residual rows, f_u, the diagonal and the line blocks) refer to the local components.  With
 * the unit normal as third column and dmask set on component 2 this imposes u . n = 0 by
 * rotation.  Every slot naming such a node must be a bottom slot (a2 = 0): basal nodes, which
 * elements above the base may name through hanging faces.  Q must be orthonormal to 1e-12.
 * Errors: NSMF_EINVAL (n_frames < 0, NULL arrays), NSMF_EMESH (id out of range or repeated,
 * Q not orthonormal, a framed node in a slot with a2 > 0).
 */
typedef enum { NSMF_PSPACE_P = 0, NSMF_PSPACE_Q = 1 } nsmf_pspace;

typedef struct {
  int32_t k;                    /* polynomial degree of velocity: 2, 3 or 4                 */
  int64_t n_el;                 /* number of elements (> 0)                                  */
  int64_t n_nodes;              /* number of independent (global) velocity nodes, < 2^28     */
  int64_t n_bface;              /* number of basal faces (>= 0)                              */
  const int32_t *elem_nodes;    /* [n_el][(k+1)^3] global node ids (see above)               */
  const uint32_t *cmask;        /* [n_el] hanging-constraint bits (see above)                */
  const double *coords;         /* [3][n_nodes] node coordinates                             */
  const int32_t *bface_elem;    /* [n_bface] elements whose zeta = -1 face lies on the base  */
  const uint8_t *dmask;         /* [3][n_nodes] 1 = Dirichlet-constrained component; may be NULL */
  int32_t pspace;               /* pressure space, nsmf_pspace (0 = P_{k-1}, 1 = Q_{k-2})    */
  double period[3];             /* periodic translation per axis, 0 = not periodic; z must be 0 */
  int64_t n_frames;             /* number of nodes with a local frame (>= 0)                 */
  const int32_t *frame_nodes;   /* [n_frames] node ids, each at most once (NULL if none)     */
  const double *frames;         /* [n_frames][3][3] row-major orthonormal Q (NULL if none)   */
} nsmf_mesh;

/* Glen law (eq. (glen)): mu = B0 * exp(-logA_e / n) * (II + eps)^((1-n)/(2n)),
 * II = D(u):D(u)/2; constant body-force density b gives f(v) = int b.v. */
typedef struct {
  double n;        /* flow-law exponent, >= 1          */
  double eps;      /* regularisation, > 0              */
  double B0;       /* rate-factor scale, > 0           */
  double body[3];  /* body-force density (b_x, b_y, b_z) */
} nsmf_params;

/* Create a context on HIP device `hip_device`.  *out is set to NULL on failure. */
int nsmf_create(nsmf_ctx **out, int hip_device);
/* Release all device memory owned by the context (waits for its stream). */
void nsmf_destroy(nsmf_ctx *ctx);
/* Stream on which all subsequent work is enqueued (a hipStream_t, e.g. torch's
 * current stream handle); NULL selects the null stream. */
int nsmf_set_stream(nsmf_ctx *ctx, void *hip_stream);

/* Copy and validate the mesh, build the per-element/per-quadrature-point geometry in
 * FP64 on the device (Sec. 3.2.1 isoparametric map; Gauss quadrature with k+1 points
 * per direction).  Synchronises.  Errors: NSMF_EINVAL, NSMF_EUNSUP (k, or geometry not
 * column-mapped: x and y must depend only on (xi, eta) affinely per element),
 * NSMF_EMESH (ids out of range, hanging bits on a level without parent, det J <= 0). */
int nsmf_upload_mesh(nsmf_ctx *ctx, const nsmf_mesh *mesh);

/* Flow-law parameters, per-element logA [n_el] and per-basal-face beta [n_bface]
 * (DEVICE pointers, FP64; NULL means all zeros; copied).  Invalidates the state. */
int nsmf_set_params(nsmf_ctx *ctx, const nsmf_params *params, const double *logA, const double *beta);

/* Linearisation of the operator that nsmf_set_state prepares (Sec. 2.3):
 *   NSMF_NEWTON (default): the Newton Jacobian with the tensor C(u) of eq. (rank4);
 *   NSMF_PICARD: the Picard operator, which keeps the viscosity mu(u) and drops the
 *     anisotropic (D (x) D) part of C(u); J_c is then the Stokes operator with frozen mu.
 * Discards the stored state (call nsmf_set_state again).  nsmf_residual, nsmf_jacobi_diag and
 * the line blocks follow the choice; nsmf_residual_vjp needs NSMF_NEWTON (its velocity part is
 * the exact derivative J^T w) and fails with NSMF_ESTATE otherwise.  Errors: NSMF_EINVAL. */
typedef enum { NSMF_NEWTON = 0, NSMF_PICARD = 1 } nsmf_linearization;
int nsmf_set_linearization(nsmf_ctx *ctx, int kind);

/* Linearisation point (u [3][n_nodes], p [n_el][n_p]; DEVICE, FP64; copied).  Computes
 * per quadrature point, in FP64, the viscosity and Newton-tensor data of eq. (rank4)
 * (and their FP32 roundings for the mixed path).  Requires mesh and params. */
int nsmf_set_state(nsmf_ctx *ctx, const double *u, const double *p);

/* Residual at the state (eq. (weak)), FP64: r_u [3][n_nodes], r_p [n_el][n_p].
 * f_u (nullable, [3][n_nodes]) is an extra load subtracted from the momentum rows. */
int nsmf_residual(nsmf_ctx *ctx, const double *f_u, double *r_u, double *r_p);

/* y = J_c x with J_c the Newton Jacobian at the state (eq. (newton), eq. (rank4)).
 * x_u, y_u [3][n_nodes]; x_p, y_p [n_el][n_p]; double for NSMF_FP64, float otherwise.
 * x and y must not overlap. */
int nsmf_jacobian_apply(nsmf_ctx *ctx, int prec, const void *x_u, const void *x_p, void *y_u, void *y_p);

/* Allocation-free variant of nsmf_jacobian_apply, for callers that cannot allocate device memory
 * during the call (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, same result, same kernels: y = J_c x.  The per-node partial sums
 * that nsmf_jacobian_apply keeps in the context's element vector are kept instead in a
 * library-wide device array of 64 MiB (one copy per GPU, held until the process ends), whose
 * device address nsmf_create resolves once per device; the call itself allocates nothing (no
 * hipMalloc, hipFree, events or library allocation).  The mesh must fit: 3 * (stored entries) *
 * (8 bytes for NSMF_FP64, 4 otherwise) <= 64 MiB, else NSMF_EINVAL with the sizes in
 * nsmf_last_error (e.g. the slab 64x64x8 Q3 workload fits in FP32, not in FP64).  All calls on
 * one GPU share the array and it keeps the last call's contents (nothing has to start at zero:
 * every entry is written before it is read): calls that may overlap on one GPU -- contexts on
 * different streams or threads -- race and must be serialised by the caller.  Not counted by
 * nsmf_set_kernel_timing.  Errors: NSMF_EINVAL (NULL vector, prec out of range, mesh too large),
 * NSMF_ESTATE (no state), NSMF_EHIP. */
int nsmf_jacobian_apply_noalloc(nsmf_ctx *ctx, int prec, const void *x_u, const void *x_p, void *y_u, void *y_p);

/* Pressure gradient y_u = B^T x_p: the discrete form of the term -int p div v of eq. (weak),
 * i.e. the velocity rows of nsmf_jacobian_apply at zero velocity (Dirichlet rows 0, nodal frames
 * applied).  It depends on the mesh only (no state needed).  x_p [n_el][n_p] and y_u [3][n_nodes]
 * DEVICE, of the precision prec (0 FP64, 1 FP32, 2 FP32 with bfloat16-rounded 1D operators).  Used
 * by the block upper-triangular preconditioner of Sec. 4.2.  Errors: NSMF_EINVAL, NSMF_ESTATE (no
 * mesh). */
int nsmf_gradient_apply(nsmf_ctx *ctx, int prec, const void *x_p, void *y_u);

/* Vector-Jacobian product of the residual at the state for cotangent w = (w_u, w_p).
 * Sec. 2.3: the adjoint (transposed) linearisation of eq. (weak) uses the same fourth-order
 * tensor of eq. (rank4) as the Newton step, and A(u) is symmetric (Sec. 4.1), so
 *   g_u, g_p = J_c^T w = J_c w;
 * the parameter derivatives differentiate eq. (weak) through the rate factor of eq. (glen)
 * (B_e = B0 exp(-logA_e / n), so d mu / d logA_e = -mu / n) and through the basal term of
 * eq. (robin):
 *   g_logA[e] = d<w, r>/dlogA_e = -(1/n) sum over the element's points of w detJ mu D(u):D(w_u);
 *   g_beta[f] = d<w, r>/dbeta_f = int_f (T u).(T w_u), T = I - n n^T.
 * w and g_u/g_p are DEVICE double for NSMF_FP64, float otherwise; g_logA [n_el] and
 * g_beta [n_bface] are always DEVICE double (FP64 accumulation).  Any g_* may be NULL.
 * Errors: NSMF_EINVAL (prec out of range, w NULL), NSMF_ESTATE (no state, or the Picard
 * linearisation is selected), NSMF_EHIP. */
int nsmf_residual_vjp(nsmf_ctx *ctx, int prec, const void *w_u, const void *w_p, void *g_u, void *g_p,
                      double *g_logA, double *g_beta);

/* Block-Jacobi preconditioner data at the state (FP64, DEVICE outputs), used by the Newton-Krylov
 * driver (Sec. 4.2).  d_u [3][n_nodes]: the diagonal of the velocity block F per component
 * (eq. (rank4) tested with each basis function, plus the basal Robin term), hanging nodes
 * collecting their children's diagonals with squared interpolation weights; 1 on Dirichlet rows.
 * d_p [n_el][n_p]: minus the lumped 1/mu-weighted pressure mass, the Schur-complement
 * approximation of Sec. 6.  With invert != 0 both outputs hold the reciprocals (the
 * preconditioner's action).  Requires a state. */
int nsmf_jacobi_diag(nsmf_ctx *ctx, int invert, double *d_u, double *d_p);

/* Low-order approximation of the velocity block on the Gauss-Lobatto sub-grid (Sec. 5, "Construction
 * of low-order approximation F~"), the matrix the paper builds its velocity preconditioner from:
 *   y_u = J~_c x_u,  J~_c = P Q^T F~ Q P + (I - P),  F~ = sum_e R_e^T F~_e R_e,
 * where F~_e treats the element's (k+1)^3 nodes as corners of k^3 trilinear sub-cells and integrates
 * the bilinear form of F (the tensor of eq. (rank4), or the Picard operator; the basal term of
 * eq. (robin)) on them with the 2-point Gauss-Lobatto rule per direction (the paper's F~_GL: the
 * quadrature points are the element's nodes, and the basal term is lumped on the base nodes).  The
 * coefficients mu, (n-1)/(2n) mu/(II+eps) and D(u) are taken at each node from the high-order state
 * differentiated inside the element (computed on the first call after nsmf_set_state); R_e is the
 * high-order restriction (figure "interp" (a) at nonconforming faces).  FP64; x_u, y_u [3][n_nodes]
 * DEVICE doubles, not overlapping; Q, P as for the Jacobian.  Requires a state.
 * Errors: NSMF_EINVAL, NSMF_ESTATE, NSMF_EHIP. */
int nsmf_lowo_apply(nsmf_ctx *ctx, const double *x_u, double *y_u);

/* Horizontal coarse space of a two-level velocity preconditioner (a plain stand-in for the coarse
 * levels of the paper's AMG on F~, Sec. 4.2 and Sec. 5; the vertical-line blocks act as the smoother).
 * A coarse function is, per velocity component, the bilinear hat of one point of a coarse lattice in
 * (x, y) times one of three profiles in the node's relative height zeta: 1 - zeta, zeta,
 * 4 zeta (1 - zeta).  Coarse vectors are DEVICE doubles [3][n_cpts][3] (component, lattice point,
 * profile).  nsmf_coarse_setup copies, per node, the 4 lattice points of its coarse cell node_cpt
 * [n_nodes][4], their bilinear weights node_w [n_nodes][4] and zeta node_zeta [n_nodes] in [0, 1]
 * (host arrays; the caller defines the lattice); it synchronises.
 *   nsmf_coarse_prolong:  x_u = P_mask (P_c xc), masked components 0 (x_u double for prec 0, float for 1);
 *   nsmf_coarse_restrict: rc = P_c^T P_mask r_u (FP64 accumulation in a fixed order; r_u double or float).
 * With A_c = P_c^T J~_c P_c (e.g. probed with nsmf_lowo_apply) the coarse correction is
 * P_c A_c^-1 P_c^T.  Errors: NSMF_EINVAL (sizes, indices, zeta), NSMF_ESTATE (no mesh / no coarse space),
 * NSMF_EUNSUP (mesh with nodal frames), NSMF_EHIP. */
int nsmf_coarse_setup(nsmf_ctx *ctx, int64_t n_cpts, const int32_t *node_cpt, const double *node_w,
                      const double *node_zeta);
int nsmf_coarse_prolong(nsmf_ctx *ctx, int prec, const double *xc, void *x_u);
int nsmf_coarse_restrict(nsmf_ctx *ctx, int prec, const void *r_u, double *rc);

/* Vertical-line block preconditioner for the velocity block (a plain fallback beside the
 * block-diagonal preconditioner of Sec. 4.2, whose AMG for F is not part of this engine).
 * The mesh's nodes form vertical lines: chains linked through the z-lines of the elements
 * (Sec. 3.1 column structure), built at upload.  For every line and velocity component,
 * nsmf_line_setup forms the block of F restricted to the line at the current state (eq. (rank4)
 * tested with the line's basis functions, plus the basal Robin term; couplings through hanging
 * slots are left out; Dirichlet rows are unit rows) -- banded with bandwidth k, symmetric
 * positive definite -- and factors it by banded Cholesky in FP64 (with an FP32 copy).
 * *n_lines (may be NULL) receives the number of lines.  Requires a state; the factors are
 * invalidated by nsmf_set_state and nsmf_set_params.  Returns NSMF_EUNSUP if the mesh's lines
 * are not consistent (a node linked to two different nodes above or below it). */
int nsmf_line_setup(nsmf_ctx *ctx, int64_t *n_lines);
/* y_u = (line blocks)^{-1} x_u, per component, by forward and backward substitution along each
 * line.  x_u, y_u [3][n_nodes] DEVICE, double (prec 0, FP64 factors) or float (prec 1, FP32
 * factors); x_u and y_u must not overlap.  Requires nsmf_line_setup at the current state. */
int nsmf_line_apply(nsmf_ctx *ctx, int prec, const void *x_u, void *y_u);

/* Vector kernels of the Krylov driver (classical Gram-Schmidt FGMRES, Sec. 4.2) on DEVICE
 * vectors of length n; prec 0: double vectors, 1: float vectors.  Inner products always
 * accumulate in FP64 with a fixed reduction order (deterministic).
 *   nsmf_vec_dots:  h[i] = sum_r V[i*ldv + r] w[r], i < k <= 64 (h: DEVICE doubles [k])
 *   nsmf_vec_gemv:  w[r] += alpha sum_i V[i*ldv + r] h[i] (h: DEVICE doubles [k])
 *   nsmf_vec_axpby: y = a x + b y (b == 0: y is written without being read, BLAS convention)
 *   nsmf_vec_mul:   z = d .* x (d: DEVICE doubles [n])
 *   nsmf_vec_normalize: x = x / sqrt(nrm2[0]), nrm2 a DEVICE double (e.g. from nsmf_vec_dots of x with
 *                   itself); x = 0 when nrm2[0] <= 0.  Lets the Arnoldi step normalise without the host.
 *   nsmf_vec_convert: out = in, double -> float (to_fp32 != 0) or float -> double */
int nsmf_vec_dots(nsmf_ctx *ctx, int prec, int64_t n, int k, const void *V, int64_t ldv, const void *w, double *h);
int nsmf_vec_gemv(nsmf_ctx *ctx, int prec, int64_t n, int k, const void *V, int64_t ldv, const double *h,
                  double alpha, void *w);
int nsmf_vec_axpby(nsmf_ctx *ctx, int prec, int64_t n, double a, const void *x, double b, void *y);
int nsmf_vec_mul(nsmf_ctx *ctx, int prec, int64_t n, const double *d, const void *x, void *z);
int nsmf_vec_normalize(nsmf_ctx *ctx, int prec, int64_t n, const double *nrm2, void *x);

/* Second Gram-Schmidt pass decided on the device (no host round trip in the Arnoldi step).
 *   nsmf_vec_dots_if, nsmf_vec_gemv_if: nsmf_vec_dots / nsmf_vec_gemv when flag[0] != 0; when
 *       flag[0] == 0, dots_if writes h[i] = 0 (i < k) and gemv_if leaves w unchanged.  flag: DEVICE int32.
 *   nsmf_gs_norm: h: DEVICE doubles [k + 1], the dots of rows V_0..V_{k-1} and of w itself with w
 *       (h[k] = |w|^2) taken before the projection w -= V h.  Writes nrm2[0] = h[k] - sum_{i<k} h[i]^2,
 *       the squared norm of the projected w when the rows are orthonormal (DEVICE double), and, if
 *       flag_out is not NULL, flag_out[0] = (nrm2[0] < eta2 h[k]): the criterion of Daniel, Gragg,
 *       Kaufman and Stewart (1976) for a second pass, eta2 = 1/2 in the driver.  If flag_in is not
 *       NULL and flag_in[0] == 0, nothing is written.  0 <= k < 64, 0 <= eta2 <= 1. */
int nsmf_vec_dots_if(nsmf_ctx *ctx, const int32_t *flag, int prec, int64_t n, int k, const void *V, int64_t ldv,
                     const void *w, double *h);
int nsmf_vec_gemv_if(nsmf_ctx *ctx, const int32_t *flag, int prec, int64_t n, int k, const void *V, int64_t ldv,
                     const double *h, double alpha, void *w);
int nsmf_gs_norm(nsmf_ctx *ctx, int k, const double *h, double eta2, const int32_t *flag_in, int32_t *flag_out,
                 double *nrm2);
int nsmf_vec_convert(nsmf_ctx *ctx, int64_t n, int to_fp32, const void *in, void *out);

/* Sizes of the uploaded mesh; any pointer may be NULL. */
int nsmf_query(nsmf_ctx *ctx, int64_t *n_nodes, int64_t *n_el, int64_t *n_p, int64_t *n_dof, int64_t *n_bface);

/* Geometry kind chosen at upload: 0 affine axis-aligned boxes, 1 column-mapped. */
int nsmf_geometry_kind(nsmf_ctx *ctx);

/* Event timing of jacobian_apply / residual_vjp.  While enabled, each such call records a
 * HIP event pair on the context's stream around its device work (the element kernel and
 * the node assembly kernel); nsmf_kernel_time synchronises and returns the summed
 * milliseconds and the number of timed calls since enabling, then resets. */
int nsmf_set_kernel_timing(nsmf_ctx *ctx, int enable);
int nsmf_kernel_time(nsmf_ctx *ctx, double *ms_total, int64_t *launches);

/* Last error message of the context (never NULL). */
const char *nsmf_last_error(const nsmf_ctx *ctx);
/* Library version string. */
const char *nsmf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NSMF_H */
