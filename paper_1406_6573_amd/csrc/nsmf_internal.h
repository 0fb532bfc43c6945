// Internal declarations shared by the host API (nsmf_api.cpp) and the kernels (nsmf_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsmf {

// Geometry kinds detected at upload.
enum GeoKind { GEO_AFFINE = 0, GEO_COLUMN = 1 };

// Node-id word of the device connectivity: bits 0..27 node id, bits 28..30 the
// Dirichlet mask of components x, y, z of that node, bit 31 a node with a local frame.
// per-point geometry fields of column-mapped elements: d zeta/dx, d zeta/dy, d zeta/dz
constexpr int NGEOQP = 3;
constexpr uint32_t NODE_MASK = 0x0FFFFFFFu;
constexpr int MASK_SHIFT = 28;
constexpr uint32_t ROT_BIT = 1u << 31;   // the slot's node has its unknowns in a local frame

// Largest number of simultaneous dot products of nsmf_vec_dots (Krylov basis size + 1).
constexpr int MAX_DOTS = 64;
constexpr int DOT_BLOCKS = 2048;   // blocks of the multi-dot's first stage (partial sums per block)

// Threads per block and elements per block for P = k+1 nodes per direction.  One
// thread owns one line of P values of an element, so an element occupies P*P threads.
// E elements per block; NT rounds E*P*P up to whole wavefronts.
#ifndef NSMF_E3
#define NSMF_E3 7
#endif
#ifndef NSMF_E4
#define NSMF_E4 4
#endif
#ifndef NSMF_E5
#define NSMF_E5 5
#endif
template <int P> struct Launch;
template <> struct Launch<3> { static constexpr int E = NSMF_E3; static constexpr int NT = (E * 9 + 63) / 64 * 64; };
template <> struct Launch<4> { static constexpr int E = NSMF_E4; static constexpr int NT = (E * 16 + 63) / 64 * 64; };
template <> struct Launch<5> { static constexpr int E = NSMF_E5; static constexpr int NT = (E * 25 + 63) / 64 * 64; };
// element-vector store entries per block: the block's E P^3 slots, padded to a multiple of NT
template <int P> constexpr int store_slots() { return (Launch<P>::E * P * P * P + Launch<P>::NT - 1) / Launch<P>::NT * Launch<P>::NT; }

// Reference-element tables (device memory, read through a restrict pointer).  Indices: q =
// Gauss point, a = Gauss-Lobatto node.
template <typename T, int P> struct Tab {
  T B[P][P];        // B[q][a]  = l_a(g_q)         Lagrange basis at Gauss points
  T D[P][P];        // D[q][a]  = l_a'(g_q)        its derivative
  T I[P][P];        // I[i][m] = l_m(child node i of the lower half [-1, 0]); the upper half is its
                    // mirror image, I_upper[i][m] = I[P-1-i][P-1-m] (symmetric nodes)
  T L[P - 1][P];    // 1D pressure factors at the Gauss points: P_{k-1} space, L[j][q] =
                    // sqrt((2j+1)/2) P_j(g_q) (normalised Legendre, j < k); Q_{k-2} space,
                    // L[j][q] = lambda_j(g_q), the Lagrange basis on the k-1 Gauss points (j < k-1)
  T w[P];           // Gauss weights
  T G[P][P];        // G[i][a] = l_a'(xi_i): derivative of the Lagrange basis at the Gauss-Lobatto nodes
  // Even/odd folded forms of M = B, D, B^T, D^T (K = 0..3) for output rows q < (P+1)/2 and
  // m < P/2: Ke[K][q][m] = (M[q][m] + M[q][P-1-m]) / 2, Ko[K][q][m] = (M[q][m] - M[q][P-1-m]) / 2,
  // Kc[K][q] = M[q][P/2] (odd P; the centre column).
  T Ke[4][(P + 1) / 2][P / 2];
  T Ko[4][(P + 1) / 2][P / 2];
  T Kc[4][(P + 1) / 2];
};

// Pressure spaces (Sec. 3.2.2): P_{k-1} with normalised Legendre products, or Q_{k-2} with the
// Lagrange basis on the tensor Gauss points (Sec. 6).
enum PSpace { PS_P = 0, PS_Q = 1 };

// FP64 tables for degree k = P-1 computed on the host (Newton iterations for the nodes).
struct HostTables {
  int P;
  double xi[5], g[5], w[5];
  double B[5][5], D[5][5], I[2][5][5], L[4][5], G[5][5];
  int n_p;
};
void build_tables(int k, int pspace, HostTables *t);

template <typename T, int P> Tab<T, P> make_tab(const HostTables &h, bool bf16_ops);

// All table variants of one degree, kept once per context in device memory and passed to the
// kernels by pointer: uniform entries are read through the scalar cache, lane-dependent ones
// (quadrature weights, Legendre values at a thread's own points) by ordinary vector loads.
template <int P> struct TabSet {
  Tab<double, P> d;     // FP64 operators
  Tab<float, P> f;      // FP32 operators
  Tab<float, P> fb;     // FP32 arithmetic, B and D rounded to bfloat16
  Tab<double, P> dsq;   // FP64 with squared child-interval weights (diagonal of R^T F R)
};
size_t tabset_bytes(int P);
void fill_tabset(const HostTables &h, void *host_buf);   // host_buf holds tabset_bytes(h.P) bytes

// Device views used by the kernels.
struct MeshView {
  const uint32_t *en;        // [n_el][P^3] node word (id | mask bits)
  const uint32_t *cmask;     // [n_el]
  const int32_t *bface_of;   // [n_el] basal face id or -1
  const int32_t *rot_of;     // [n_el] row of the element's bottom-slot frames in GeoView::rot, or -1
  // entries of the element slots in the node-ordered element vector.  P = 4: pos[e][a] per slot.
  // P = 3, 5: per block, the entries of its slots in ascending order (spos, -1 = padding) with the
  // slot's index in the block's LDS staging order (sslot), [nblocks][store_slots]
  const int32_t *pos;
  const int32_t *spos;
  const uint16_t *sslot;
  int64_t n_el, n_nodes, n_inc;   // n_inc = n_el P^3 element slots
  int64_t n_ent;                  // stored entries of the element vector per component (its plane stride)
  int nblocks;
  int any_hang;                   // 1 if some element has a hanging face or edge (cmask bits above 2)
};

template <typename T> struct GeoView {
  const T *el;     // AFFINE: [n_el][4] (1/J00, 1/J11, 1/J22, detJ); COLUMN: [n_el][2] (1/J00, 1/J11)
  const T *qp;     // COLUMN: [nblocks][4][P][NT] (dzeta/dx, dzeta/dy, dzeta/dz, w detJ)
  const T *face;   // [n_bface][4][P*P] (w |S|, n_x, n_y, n_z) at the face Gauss points
  const T *rot;    // [n_rot][9][P*P] local frame Q (row-major) of the node in each bottom slot of the
                   // elements with a framed node (MeshView::rot_of), or null
};

// Launchers (defined in nsmf_kernels.hip).  Return hipError_t of the launch.
hipError_t launch_geometry_impl(int P, int mode, hipStream_t s, const MeshView &m, const void *tabs,
                                const double *coords, const double period[3], double *el_out, double *qp_out,
                                double *face_out, unsigned *flags);
hipError_t launch_state(int P, int geo, hipStream_t s, const MeshView &m, const GeoView<double> &g,
                        const void *tabs, const double *u, const double *logA, double n, double eps,
                        double B0, bool picard, double *st64, float *st32, double *fst64, float *fst32);
hipError_t launch_apply(int P, int geo, int ps, int prec, bool vjp, hipStream_t s, const MeshView &m, const void *geo_view,
                        const void *tabs, const void *state, const void *fstate, const void *beta,
                        const void *x_u, const void *x_p, void *y_u, void *y_p, double inv_n,
                        double *g_logA, double *g_beta);
// y_u = B^T x_p into the element vector (prec 0, 1, 2 as launch_apply)
hipError_t launch_grad_p(int P, int geo, int ps, int prec, hipStream_t s, const MeshView &m, const void *gview,
                         const void *tabs, const void *xp, void *yu);
hipError_t launch_residual(int P, int geo, int ps, hipStream_t s, const MeshView &m, const GeoView<double> &g,
                           const void *tabs, const double *st64, const double *fst64, const double *beta,
                           const double *p, const double *body, double *r_u, double *r_p);
hipError_t launch_diag(int P, int geo, int ps, hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                       const double *st, const double *beta, double *ev, double *dp);
hipError_t launch_fill(hipStream_t s, void *ptr, int64_t n_words32);
// low-order approximation F~ on the Gauss-Lobatto sub-grid: nodal coefficients (once per state) and
// the matrix-free action (element vector, assembled by launch_assemble)
constexpr int NLOWO = 11;   // per element node: x_rel (3), mu, kappa', D0 (xx, yy, zz, xy, xz, yz)
hipError_t launch_lowo_coef(int P, hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                            const double *X, const double period[3], const double *u, const double *logA, double n,
                            double eps, double B0, bool picard, double *lo);
hipError_t launch_lowo(int P, hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                       const double *lo, const double *beta, const double *x, double *ev);
// vertical-line block preconditioner: element line blocks, node assembly, banded Cholesky
hipError_t launch_lines(int P, int geo, hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                        const double *st, const double *beta, const int32_t *lptr, const int32_t *lslot,
                        const uint8_t *dm, const int32_t *line_ptr, const int32_t *line_node,
                        const int32_t *prow, const int32_t *lrow, int64_t NR, int64_t n_lines, double *buf,
                        double *fac64, float *fac32);
// Line-block rows are interleaved by groups of LINE_GROUP consecutive lines: node i of line l sits at
// row lrow[l] + LINE_GROUP i, lrow[l] = (row offset of l's group) + l mod LINE_GROUP; prow[n] is node
// n's row, NR the rows per component (the groups padded to their longest line).  line_first[l]: id
// of the first node of line l if the line's node ids are consecutive, else -1.  The factorisation
// and the solves run one thread per (line, component), the lines of a component padded to a
// multiple of LINE_GROUP so that a group is one wavefront.
constexpr int LINE_GROUP = 64;
__host__ __device__ inline int64_t line_threads(int64_t n_lines) {
  return (n_lines + LINE_GROUP - 1) / LINE_GROUP * LINE_GROUP;
}
hipError_t launch_line_apply(hipStream_t s, int prec, int P, int64_t N, const int32_t *line_ptr, const int32_t *line_node,
                             const int32_t *lrow, int64_t NR, const int32_t *line_first, int64_t n_lines,
                             const void *fac, const void *x, void *y);

// The run of independent slots z = lo..hi on the z-line (x = i, y = j) of an element, false when
// every slot of the line is dependent.  A hanging face or edge that contains the line makes all of
// it dependent; a hanging z-normal face, or an x/y-parallel hanging edge through an end slot, makes
// only that end slot dependent.  cmask bits: 3..8 faces -x, +x, -y, +y, -z, +z; 9 + 4 dir + s0 +
// 2 s1 edge parallel to axis dir with sides (s0, s1) along the other two axes in increasing order.
inline bool zline_run_host(uint32_t cm, int P, int i, int j, int &lo, int &hi) {
  const uint32_t f = cm >> 3;
  auto side = [P](int a) { return a == 0 ? 0 : (a == P - 1 ? 1 : -1); };
  auto edge = [&](int dir, int a, int b) {
    const int s0 = side(a), s1 = side(b);
    return s0 >= 0 && s1 >= 0 && ((cm >> (9 + 4 * dir + s0 + 2 * s1)) & 1u);
  };
  if (((f >> 0) & 1u) && i == 0) return false;
  if (((f >> 1) & 1u) && i == P - 1) return false;
  if (((f >> 2) & 1u) && j == 0) return false;
  if (((f >> 3) & 1u) && j == P - 1) return false;
  if (edge(2, i, j)) return false;                        // z-parallel edge along the line
  lo = (((f >> 4) & 1u) || edge(0, j, 0) || edge(1, i, 0)) ? 1 : 0;
  hi = (((f >> 5) & 1u) || edge(0, j, P - 1) || edge(1, i, P - 1)) ? P - 2 : P - 1;
  return true;
}
// mval: value of the Dirichlet rows when xm is null
hipError_t launch_assemble(hipStream_t s, int prec, int64_t N, const int32_t *ptr, const void *ev, int64_t n_ent,
                           const uint8_t *dm, const void *xm, const void *f, void *y, double mval = 1.0);
hipError_t launch_d2f(hipStream_t s, const double *in, float *out, int64_t n);
hipError_t launch_f2d(hipStream_t s, const float *in, double *out, int64_t n);
hipError_t launch_recip(hipStream_t s, int64_t n, double *x);
// flag (DEVICE, may be null): when flag[0] == 0 the call is not taken (dots write h = 0)
hipError_t launch_dots(hipStream_t s, int prec, int64_t n, int k, const void *V, int64_t ldv, const void *w,
                       double *partial, double *h, const int32_t *flag = nullptr);
hipError_t launch_gemv(hipStream_t s, int prec, int64_t n, int k, const void *V, int64_t ldv, const double *h,
                       double alpha, void *w, const int32_t *flag = nullptr);
hipError_t launch_gs_norm(hipStream_t s, int k, const double *h, double eta2, const int32_t *flag_in, int32_t *flag_out,
                          double *nrm2);
hipError_t launch_axpby(hipStream_t s, int prec, int64_t n, double a, const void *x, double b, void *y);
hipError_t launch_mul(hipStream_t s, int prec, int64_t n, const double *d, const void *x, void *z);
hipError_t launch_normalize(hipStream_t s, int prec, int64_t n, const double *nrm2, void *x);
// horizontal coarse space of the two-level velocity preconditioner (NCZ vertical profiles)
hipError_t launch_prolong(hipStream_t s, int prec, int64_t N, int64_t nc, const int32_t *cpt, const double *cw,
                          const double *zeta, const uint8_t *dm, const double *xc, void *x);
hipError_t launch_restrict(hipStream_t s, int prec, int64_t N, int64_t nc, const int64_t *cptr, const int32_t *cnode,
                           const double *cwt, const double *zeta, const uint8_t *dm, const void *r, double *rc);

}  // namespace nsmf
