// Element kernels of the matrix-free Newton-Stokes operator for gfx950.
//
// Work decomposition: a block of NT threads processes E elements; an element owns P*P
// threads (P = k+1), each holding one line of P values of a 3D tensor-product field in
// registers.  A 1D contraction along the line a thread holds runs in registers; the
// other directions are reached by passing the field through LDS, where each thread
// picks up a line in the next direction (Sec. 3.3: all element work reduces to
// repeated 1D kernels, and the same 1D kernels apply the hanging-node restriction).
//
// Thread t of an element holds, depending on the phase,
//   z-line  (i, j) = (t % P, t / P): points (i, j, 0..P-1)   -- gather / scatter layout
//   y-line  (i, z) = (t % P, t / P): points (i, 0..P-1, z)
//   x-line  (j, z) = (t % P, t / P): points (0..P-1, j, z)   -- quadrature-point layout
// with point (x, y, z) stored at LDS offset x + P*y + SZ*z (SZ >= P*P, padded against bank
// conflicts).
//
// Per-quadrature-point data are stored in the x-line layout of the kernel itself (qp_at):
// thread-major for P = 4 (one wide load per field and thread), point-major for P = 3, 5 (each
// scalar load one contiguous span across the wavefront).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "nsmf_internal.h"

namespace nsmf {

constexpr int NSTATE = 8;   // mu', kappa, Sigma_xx, Sigma_yy, Sigma_zz, Sigma_xy, Sigma_xz, Sigma_yz
// FP32 apply: mu' and Sigma_hat = sqrt(kappa) Sigma0 (kappa >= 0 for n >= 1), so that the Newton term
// kappa (Sigma0 : D) Sigma0 = (Sigma_hat : D) Sigma_hat takes one value less per point
constexpr int NSTATE32 = 7;
constexpr int NFACEGEO = 4; // w|S|, n_x, n_y, n_z
constexpr int NFACEST = 3;  // w|S| T u

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous range of
// element groups so neighbouring elements (sharing nodes) hit the same L2.
__device__ __forceinline__ int logical_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int q = nb >> 3, r = nb & 7, x = b & 7, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

// Element of slot el of block lb (-1: none): blocks take runs of E consecutive elements.
template <int E> __device__ __forceinline__ int64_t tile_elem(const MeshView &m, int lb, int el) {
  if (el >= E) return -1;
  const int64_t e = (int64_t)lb * E + el;
  return e < m.n_el ? e : -1;
}

template <int P> __device__ __forceinline__ int side_of(int a) { return a == 0 ? 0 : (a == P - 1 ? 1 : -1); }

template <int P> __device__ __forceinline__ bool edge_on(uint32_t cm, int dir, int a, int b) {
  const int s0 = side_of<P>(a), s1 = side_of<P>(b);
  if (s0 < 0 || s1 < 0) return false;
  return (cm >> (9 + 4 * dir + s0 + 2 * s1)) & 1u;
}
// Lines of the element that lie on a hanging face or edge having the line's direction
// as a tangent direction; those are interpolated from the parent values.
template <int P> __device__ __forceinline__ bool xline_hanging(uint32_t cm, int j, int z) {
  const uint32_t f = cm >> 3;
  return ((f >> 2) & 1u && j == 0) || ((f >> 3) & 1u && j == P - 1) || ((f >> 4) & 1u && z == 0) ||
         ((f >> 5) & 1u && z == P - 1) || edge_on<P>(cm, 0, j, z);
}
template <int P> __device__ __forceinline__ bool yline_hanging(uint32_t cm, int i, int z) {
  const uint32_t f = cm >> 3;
  return ((f >> 0) & 1u && i == 0) || ((f >> 1) & 1u && i == P - 1) || ((f >> 4) & 1u && z == 0) ||
         ((f >> 5) & 1u && z == P - 1) || edge_on<P>(cm, 1, i, z);
}
template <int P> __device__ __forceinline__ bool zline_hanging(uint32_t cm, int i, int j) {
  const uint32_t f = cm >> 3;
  return ((f >> 0) & 1u && i == 0) || ((f >> 1) & 1u && i == P - 1) || ((f >> 2) & 1u && j == 0) ||
         ((f >> 3) & 1u && j == P - 1) || edge_on<P>(cm, 2, i, j);
}

// Child-interval interpolation of a line (half h of the parent interval) and its transpose.
// The upper half is the mirror image of the lower one, so h = 1 reverses the line, applies the
// lower-half matrix and reverses the result: the table is indexed statically and stays in scalar
// registers.  The reversal selects between values read at static indices (a conditional between
// two array elements would select their address, a runtime index into a register array, which
// compiles to select chains over the whole array).
template <typename T, int P> __device__ __forceinline__ void mirror_if(bool h, T *v) {
#pragma unroll
  for (int m = 0; m < P / 2; ++m) {
    const T a = v[m], b = v[P - 1 - m];
    v[m] = h ? b : a;
    v[P - 1 - m] = h ? a : b;
  }
}
template <typename T, int P> __device__ __forceinline__ void interp_line(const Tab<T, P> &tb, int h, T *v) {
  T r[P], o[P];
#pragma unroll
  for (int m = 0; m < P; ++m) r[m] = v[m];
  mirror_if<T, P>(h != 0, r);
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T a = 0;
#pragma unroll
    for (int m = 0; m < P; ++m) a += tb.I[i][m] * r[m];
    o[i] = a;
  }
  mirror_if<T, P>(h != 0, o);
#pragma unroll
  for (int i = 0; i < P; ++i) v[i] = o[i];
}
template <typename T, int P> __device__ __forceinline__ void interp_line_t(const Tab<T, P> &tb, int h, T *v) {
  T r[P], o[P];
#pragma unroll
  for (int i = 0; i < P; ++i) r[i] = v[i];
  mirror_if<T, P>(h != 0, r);
#pragma unroll
  for (int m = 0; m < P; ++m) {
    T a = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) a += tb.I[i][m] * r[i];
    o[m] = a;
  }
  mirror_if<T, P>(h != 0, o);
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = o[m];
}

// LDS strides chosen against bank conflicts: the z-plane stride SZ spreads the P lines of a
// y-line access over distinct banks, and the element pad PADE shifts the elements that share a
// wavefront onto disjoint banks.  The values minimise the summed conflict cost of the z-, y- and
// x-line accesses of one block under 32- and 64-bank models of 4-byte banks.
template <typename T, int P> struct LdsShape { static constexpr int SZ = P * P, PADE = 0; };
template <typename T> struct LdsShape<T, 4> { static constexpr int SZ = 20, PADE = sizeof(T) == 8 ? 8 : 0; };
template <typename T> struct LdsShape<T, 5> { static constexpr int SZ = 25, PADE = sizeof(T) == 8 ? 12 : 8; };

// Element workspace: NB buffers of P planes each; point (x, y, z) at x + P*y + SZ*z.
template <typename T, int P> struct Ws {
  static constexpr int P2 = P * P, NB = 5;
  static constexpr int SZ = LdsShape<T, P>::SZ;          // z-plane stride
  static constexpr int BS = SZ * P;                      // buffer size
  static constexpr int ES = NB * BS + LdsShape<T, P>::PADE;   // element stride
  T *s;
  __device__ T *b(int k) const { return s + k * BS; }
  // start of the z-line of thread t = x + P*y, and of the x-line of thread t = y + P*z
  __device__ static int zl(int t, int z) { return t + SZ * z; }
  __device__ static int xl(int t) { return P * (t % P) + SZ * (t / P); }
};

// ---------------------------------------------------------------- hanging restriction R_e
// In: v[c][z] = the values named by elem_nodes on the z-line (parent values in hanging
// slots).  Out: R_e x on the z-line.  Interpolates along x, then y (through LDS), then z
// (in registers), each on the flagged lines only.  All threads of the block must call.
template <typename T, int P>
__device__ void hang_fwd(T (&v)[3][P], uint32_t cm, Ws<T, P> w, const Tab<T, P> &tb, int t, bool act) {
  constexpr int P2 = P * P;
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int z = 0; z < P; ++z) w.b(c)[w.zl(t, z)] = v[c][z];
  __syncthreads();
  if (act) {
    const int j = t % P, z = t / P;
    if (xline_hanging<P>(cm, j, z)) {
      const int h = cm & 1u;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T l[P];
#pragma unroll
        for (int m = 0; m < P; ++m) l[m] = w.b(c)[m + w.xl(t)];
        interp_line<T, P>(tb, h, l);
#pragma unroll
        for (int m = 0; m < P; ++m) w.b(c)[m + w.xl(t)] = l[m];
      }
    }
  }
  __syncthreads();
  if (act) {
    const int i = t % P, z = t / P;
    if (yline_hanging<P>(cm, i, z)) {
      const int h = (cm >> 1) & 1u;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T l[P];
#pragma unroll
        for (int m = 0; m < P; ++m) l[m] = w.b(c)[i + P * m + w.SZ * z];
        interp_line<T, P>(tb, h, l);
#pragma unroll
        for (int m = 0; m < P; ++m) w.b(c)[i + P * m + w.SZ * z] = l[m];
      }
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int z = 0; z < P; ++z) v[c][z] = w.b(c)[w.zl(t, z)];
    const int i = t % P, j = t / P;
    if (zline_hanging<P>(cm, i, j)) {
      const int h = (cm >> 2) & 1u;
#pragma unroll
      for (int c = 0; c < 3; ++c) interp_line<T, P>(tb, h, v[c]);
    }
  }
  __syncthreads();
}

// Transpose R_e^T on the z-line: z (registers), then y, then x (through LDS).
template <typename T, int P>
__device__ void hang_bwd(T (&v)[3][P], uint32_t cm, Ws<T, P> w, const Tab<T, P> &tb, int t, bool act) {
  constexpr int P2 = P * P;
  if (act) {
    const int i = t % P, j = t / P;
    if (zline_hanging<P>(cm, i, j)) {
      const int h = (cm >> 2) & 1u;
#pragma unroll
      for (int c = 0; c < 3; ++c) interp_line_t<T, P>(tb, h, v[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int z = 0; z < P; ++z) w.b(c)[w.zl(t, z)] = v[c][z];
  }
  __syncthreads();
  if (act) {
    const int i = t % P, z = t / P;
    if (yline_hanging<P>(cm, i, z)) {
      const int h = (cm >> 1) & 1u;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T l[P];
#pragma unroll
        for (int m = 0; m < P; ++m) l[m] = w.b(c)[i + P * m + w.SZ * z];
        interp_line_t<T, P>(tb, h, l);
#pragma unroll
        for (int m = 0; m < P; ++m) w.b(c)[i + P * m + w.SZ * z] = l[m];
      }
    }
  }
  __syncthreads();
  if (act) {
    const int j = t % P, z = t / P;
    if (xline_hanging<P>(cm, j, z)) {
      const int h = cm & 1u;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T l[P];
#pragma unroll
        for (int m = 0; m < P; ++m) l[m] = w.b(c)[m + w.xl(t)];
        interp_line_t<T, P>(tb, h, l);
#pragma unroll
        for (int m = 0; m < P; ++m) w.b(c)[m + w.xl(t)] = l[m];
      }
    }
  }
  __syncthreads();
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int z = 0; z < P; ++z) v[c][z] = w.b(c)[w.zl(t, z)];
  __syncthreads();
}

// ---------------------------------------------------------------- folded 1D products
// Gauss points and Gauss-Lobatto nodes are symmetric about 0, so M[P-1-q][P-1-m] = s M[q][m] with
// s = +1 for B and B^T and s = -1 for D and D^T.  With the input split into even and odd parts
// about its centre, e_m = v_m + v_{P-1-m} and o_m = v_m - v_{P-1-m}, the output pair (q, P-1-q)
// is E_q +- O_q (s = +1) or O_q +- E_q (s = -1), where E_q = sum_m Ke[q][m] e_m (+ Kc[q] v_c)
// and O_q = sum_m Ko[q][m] o_m: about 2/3 of the multiply-adds of the plain P x P product.
template <typename T, int P> struct Fold {
  T e[P / 2], o[P / 2], c;
};
template <typename T, int P>
__device__ __forceinline__ Fold<T, P> fold(const T (&v)[P]) {
  Fold<T, P> f;
#pragma unroll
  for (int m = 0; m < P / 2; ++m) {
    f.e[m] = v[m] + v[P - 1 - m];
    f.o[m] = v[m] - v[P - 1 - m];
  }
  f.c = (P % 2) ? v[P / 2] : T(0);
  return f;
}
// An output in folded form: out[q] = ev[q] + od[q], out[P-1-q] = ev[q] - od[q] (q < P/2), and
// out[P/2] = ev[P/2] for odd P.
template <typename T, int P> struct Acc {
  T ev[(P + 1) / 2], od[P / 2];
  __device__ __forceinline__ Acc() {
#pragma unroll
    for (int q = 0; q < (P + 1) / 2; ++q) ev[q] = 0;
#pragma unroll
    for (int q = 0; q < P / 2; ++q) od[q] = 0;
  }
  __device__ __forceinline__ void unfold(T (&out)[P]) const {
#pragma unroll
    for (int q = 0; q < P / 2; ++q) {
      out[q] = ev[q] + od[q];
      out[P - 1 - q] = ev[q] - od[q];
    }
    if (P % 2) out[P / 2] = ev[P / 2];
  }
};
// a += M v for the folded table K (0 = B, 1 = D, 2 = B^T, 3 = D^T) of symmetry sign S
template <int K, typename T, int P>
__device__ __forceinline__ void acc_mv(Acc<T, P> &a, const Tab<T, P> &tb, const Fold<T, P> &f) {
  constexpr int H = P / 2;
  constexpr bool EVEN = K % 2 == 0;   // B, B^T: s = +1
#pragma unroll
  for (int q = 0; q < H; ++q) {
    T &te = EVEN ? a.ev[q] : a.od[q];   // receives E_q
    T &to = EVEN ? a.od[q] : a.ev[q];   // receives O_q
#pragma unroll
    for (int m = 0; m < H; ++m) te += tb.Ke[K][q][m] * f.e[m];
    if (P % 2) te += tb.Kc[K][q] * f.c;
#pragma unroll
    for (int m = 0; m < H; ++m) to += tb.Ko[K][q][m] * f.o[m];
  }
  if (P % 2) {
    // centre row: only the even part survives for s = +1, only the odd part for s = -1
    if (EVEN) {
#pragma unroll
      for (int m = 0; m < H; ++m) a.ev[H] += tb.Ke[K][H][m] * f.e[m];
      a.ev[H] += tb.Kc[K][H] * f.c;
    } else {
#pragma unroll
      for (int m = 0; m < H; ++m) a.ev[H] += tb.Ko[K][H][m] * f.o[m];
    }
  }
}
enum { KB = 0, KD = 1, KBT = 2, KDT = 3 };

// ---------------------------------------------------------------- sum-factorised gradient
// z-line nodal values -> reference gradient at the x-line's quadrature points:
//   gx = (D x B x B) v, gy = (B x D x B) v, gz = (B x B x D) v  (x fastest in the Kronecker order).
// Two barriers; buffers 0..4.  All threads call.
template <typename T, int P>
__device__ void grad_fwd(const T (&v)[P], T (&gx)[P], T (&gy)[P], T (&gz)[P], Ws<T, P> w, const Tab<T, P> &tb,
                         int t, bool act) {
  if (act) {
    const Fold<T, P> f = fold<T, P>(v);
    Acc<T, P> ab, ad;
    acc_mv<KB>(ab, tb, f);
    acc_mv<KD>(ad, tb, f);
    T a[P], d[P];
    ab.unfold(a);
    ad.unfold(d);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      w.b(0)[w.zl(t, q)] = a[q];
      w.b(1)[w.zl(t, q)] = d[q];
    }
  }
  __syncthreads();
  if (act) {
    const int i = t % P, z = t / P;
    T a[P], b[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      a[m] = w.b(0)[i + P * m + w.SZ * z];
      b[m] = w.b(1)[i + P * m + w.SZ * z];
    }
    const Fold<T, P> fa = fold<T, P>(a), fb = fold<T, P>(b);
    Acc<T, P> a0, a1, a2;
    acc_mv<KB>(a0, tb, fa);
    acc_mv<KD>(a1, tb, fa);
    acc_mv<KB>(a2, tb, fb);
    T s0[P], s1[P], s2[P];
    a0.unfold(s0);
    a1.unfold(s1);
    a2.unfold(s2);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      w.b(2)[i + P * q + w.SZ * z] = s0[q];
      w.b(3)[i + P * q + w.SZ * z] = s1[q];
      w.b(4)[i + P * q + w.SZ * z] = s2[q];
    }
  }
  __syncthreads();
  if (act) {
    T a[P], b[P], c[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      a[m] = w.b(2)[m + w.xl(t)];
      b[m] = w.b(3)[m + w.xl(t)];
      c[m] = w.b(4)[m + w.xl(t)];
    }
    Acc<T, P> x0, x1, x2;
    acc_mv<KD>(x0, tb, fold<T, P>(a));
    acc_mv<KB>(x1, tb, fold<T, P>(b));
    acc_mv<KB>(x2, tb, fold<T, P>(c));
    x0.unfold(gx);
    x1.unfold(gy);
    x2.unfold(gz);
  }
}

// Transpose: x-line quadrature values (fx, fy, fz tested against d/dxi, d/deta, d/dzeta of
// the basis, f0 against the basis itself) -> z-line nodal values.  Two barriers; buffers 0..4.
template <typename T, int P, bool VALUE>
__device__ void grad_bwd(const T (&fx)[P], const T (&fy)[P], const T (&fz)[P], const T (&f0)[P], T (&out)[P],
                         Ws<T, P> w, const Tab<T, P> &tb, int t, bool act) {
  if (act) {
    Acc<T, P> h0, h1, h2;
    acc_mv<KDT>(h0, tb, fold<T, P>(fx));
    if (VALUE) acc_mv<KBT>(h0, tb, fold<T, P>(f0));
    acc_mv<KBT>(h1, tb, fold<T, P>(fy));
    acc_mv<KBT>(h2, tb, fold<T, P>(fz));
    T o0[P], o1[P], o2[P];
    h0.unfold(o0);
    h1.unfold(o1);
    h2.unfold(o2);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      w.b(0)[i + w.xl(t)] = o0[i];
      w.b(1)[i + w.xl(t)] = o1[i];
      w.b(2)[i + w.xl(t)] = o2[i];
    }
  }
  __syncthreads();
  if (act) {
    const int i = t % P, z = t / P;
    T a[P], b[P], c[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      a[q] = w.b(0)[i + P * q + w.SZ * z];
      b[q] = w.b(1)[i + P * q + w.SZ * z];
      c[q] = w.b(2)[i + P * q + w.SZ * z];
    }
    Acc<T, P> k0, k1;
    acc_mv<KBT>(k0, tb, fold<T, P>(a));
    acc_mv<KDT>(k0, tb, fold<T, P>(b));
    acc_mv<KBT>(k1, tb, fold<T, P>(c));
    T o0[P], o1[P];
    k0.unfold(o0);
    k1.unfold(o1);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      w.b(3)[i + P * j + w.SZ * z] = o0[j];
      w.b(4)[i + P * j + w.SZ * z] = o1[j];
    }
  }
  __syncthreads();
  if (act) {
    T a[P], b[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      a[q] = w.b(3)[w.zl(t, q)];
      b[q] = w.b(4)[w.zl(t, q)];
    }
    Acc<T, P> o;
    acc_mv<KBT>(o, tb, fold<T, P>(a));
    acc_mv<KDT>(o, tb, fold<T, P>(b));
    o.unfold(out);
  }
}

// Per-quadrature-point field f of point i on the x-line of thread tid in block lb.  P = 4:
// thread-major, the thread's 4 points contiguous, read as one 16/32-byte line.  P = 3, 5:
// point-major, so that each of the thread's scalar loads is one contiguous span across the
// wavefront.  All with the non-temporal hint: the stream is read once per launch and would
// otherwise displace from L2 the reused lines, gathered nodal values and partially written
// element-vector lines (FP32 apply 11% faster on the Q3 slab, element kernel 3% faster on the
// Q4 terrain and 6% on the Q2 dome).  The hint does not pay on the smaller read-once streams
// (node words, store positions, pressure coefficients): their lines straddle elements of
// neighbouring blocks.
template <int P, int NT, int F>
__device__ __forceinline__ size_t qp_at(int lb, int f, int tid, int i) {
  if constexpr (P == 4) return (((size_t)lb * F + f) * NT + tid) * P + i;
  else return (((size_t)lb * F + f) * P + i) * NT + tid;
}
// Store of a per-point value: point-major layouts (P = 3, 5) write whole lines per instruction and
// take the non-temporal hint (the state is written once per Newton step and read by the next
// kernels from HBM; 7% faster linearisation on the Q4 terrain); the thread-major P = 4 layout
// fills a line over four instructions and keeps the plain store.
template <int P, typename T> __device__ __forceinline__ void st_store(T *p, T v) {
  if constexpr (P == 4) *p = v;
  else __builtin_nontemporal_store(v, p);
}
template <typename T, int P, int NT, int F>
__device__ __forceinline__ void load_field(const T *__restrict__ base, int lb, int f, int tid, T (&o)[P]) {
  if constexpr (P == 4 && sizeof(T) == 4) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(base + qp_at<P, NT, F>(lb, f, tid, 0)));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else if constexpr (P == 4 && sizeof(T) == 8) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v *q = reinterpret_cast<const d2v *>(base + qp_at<P, NT, F>(lb, f, tid, 0));
    const d2v a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + 1);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  } else {
#pragma unroll
    for (int i = 0; i < P; ++i) o[i] = __builtin_nontemporal_load(base + qp_at<P, NT, F>(lb, f, tid, i));
  }
}

// ---------------------------------------------------------------- geometry access
// Column-mapped elements: x depends on xi and y on eta only (affine per column), z on all three, so
// J^-1 has the constant entries d xi/dx, d eta/dy and the per-point row (d zeta/dx, d zeta/dy,
// d zeta/dz); detJ = (dx/dxi)(dy/deta)(dz/dzeta) = 1 / (jx jy c), so w detJ is formed from c where it
// is used rather than stored (NGEOQP fields per point).
template <typename T> __device__ __forceinline__ T recip(T x) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(x);   // within 1 ulp
  else return T(1) / x;
}
template <typename T, int P, int GEO> struct QpGeo {
  T jx, jy, jz;          // d xi/dx, d eta/dy, (affine) d zeta/dz
  T detJ;                // affine only
  T wjz;                 // product w_j w_z of the Gauss weights of the thread's x-line (j, z)
  T a[P], b[P], c[P];    // column: d zeta/dx, d zeta/dy, d zeta/dz (x-line)
  // quadrature weight times detJ at point i of the x-line
  __device__ __forceinline__ T wdet(const Tab<T, P> &tb, int i) const {
    if (GEO == GEO_AFFINE) return tb.w[i] * wjz * detJ;
    else return tb.w[i] * wjz * recip<T>(jx * jy * c[i]);
  }
};

template <typename T, int P, int GEO, int NT>
__device__ __forceinline__ void load_geo(QpGeo<T, P, GEO> &g, const GeoView<T> &gv, int64_t e, int lb, int tid,
                                         const Tab<T, P> &tb, int t) {
  const int j = t % P, z = t / P;
  g.wjz = tb.w[j] * tb.w[z];
  if (GEO == GEO_AFFINE) {
    const T *p = gv.el + 4 * e;
    g.jx = p[0]; g.jy = p[1]; g.jz = p[2]; g.detJ = p[3];
  } else {
    const T *p = gv.el + 2 * e;
    g.jx = p[0]; g.jy = p[1];
    load_field<T, P, NT, NGEOQP>(gv.qp, lb, 0, tid, g.a);
    load_field<T, P, NT, NGEOQP>(gv.qp, lb, 1, tid, g.b);
    load_field<T, P, NT, NGEOQP>(gv.qp, lb, 2, tid, g.c);
  }
}

// physical gradient G[c][s] = sum_r Gref[c][r] Jinv[r][s] at x-line point i
template <typename T, int P, int GEO>
__device__ __forceinline__ void to_phys(const QpGeo<T, P, GEO> &g, int i, const T (&gr)[3][3], T (&G)[3][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (GEO == GEO_AFFINE) {
      G[c][0] = gr[c][0] * g.jx;
      G[c][1] = gr[c][1] * g.jy;
      G[c][2] = gr[c][2] * g.jz;
    } else {
      G[c][0] = gr[c][0] * g.jx + gr[c][2] * g.a[i];
      G[c][1] = gr[c][1] * g.jy + gr[c][2] * g.b[i];
      G[c][2] = gr[c][2] * g.c[i];
    }
  }
}
// reference flux f[c][r] = sum_s tau[c][s] Jinv[r][s]
template <typename T, int P, int GEO>
__device__ __forceinline__ void to_ref(const QpGeo<T, P, GEO> &g, int i, const T (&tau)[3][3], T (&f)[3][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (GEO == GEO_AFFINE) {
      f[c][0] = tau[c][0] * g.jx;
      f[c][1] = tau[c][1] * g.jy;
      f[c][2] = tau[c][2] * g.jz;
    } else {
      f[c][0] = tau[c][0] * g.jx;
      f[c][1] = tau[c][1] * g.jy;
      f[c][2] = tau[c][0] * g.a[i] + tau[c][1] * g.b[i] + tau[c][2] * g.c[i];
    }
  }
}

// ---------------------------------------------------------------- pressure basis
// Pressure modes: number per element, and the (i, j, l) indices of the 1D factors of each mode,
// as compile-time constants so that register arrays indexed by them stay in registers.
// P_{k-1}: exponents i+j+l <= k-1, ordered by (i+j+l, l, j, i); Q_{k-2}: the k-1 Gauss points
// per direction, i fastest.  psi_m(x_i, y_j, z_l) = L[e0][i] L[e1][j] L[e2][l] at Gauss points.
template <int P, int PS> constexpr int n_pres() { return PS == PS_P ? (P - 1) * P * (P + 1) / 6 : (P - 2) * (P - 2) * (P - 2); }
// per-element stride (in doubles) of the apply kernel's reduction area: P^2 partial sums of the
// parameter gradients, or the element's pressure coefficients while the forward sweeps run
template <int P, int PS> constexpr int red_stride() { return n_pres<P, PS>() > P * P ? n_pres<P, PS>() : P * P; }
template <int P, int PS> struct PExp {
  static constexpr int NP = n_pres<P, PS>();
  int e[NP][3];
  constexpr PExp() : e{} {
    int m = 0;
    if (PS == PS_P) {
      for (int d = 0; d < P - 1; ++d)
        for (int l = 0; l <= d; ++l)
          for (int j = 0; j <= d - l; ++j) {
            e[m][0] = d - l - j;
            e[m][1] = j;
            e[m][2] = l;
            ++m;
          }
    } else {
      for (int l = 0; l < P - 2; ++l)
        for (int j = 0; j < P - 2; ++j)
          for (int i = 0; i < P - 2; ++i) {
            e[m][0] = i;
            e[m][1] = j;
            e[m][2] = l;
            ++m;
          }
    }
  }
};
// The 1D pressure factors at the x-line thread's own (j, z) Gauss points: per-lane table reads,
// requested ahead of their use so that their latency overlaps other work.
template <typename T, int P> struct PRows {
  T j[P - 1], z[P - 1];
};
template <typename T, int P>
__device__ __forceinline__ PRows<T, P> pressure_rows(const Tab<T, P> &tb, int t) {
  PRows<T, P> r;
#pragma unroll
  for (int a = 0; a < P - 1; ++a) {
    r.j[a] = tb.L[a][t % P];
    r.z[a] = tb.L[a][t / P];
  }
  return r;
}
// x-line thread (j, z): p(i) = sum_m xp[m] L_{e0}(g_i) L_{e1}(g_j) L_{e2}(g_z)
template <typename T, int P, int PS>
__device__ __forceinline__ void pressure_interp(const T *xp, const Tab<T, P> &tb, const PRows<T, P> &pr, T (&pq)[P]) {
  constexpr int NP = n_pres<P, PS>();
  constexpr PExp<P, PS> pe{};
  T pa[P - 1];
#pragma unroll
  for (int a = 0; a < P - 1; ++a) pa[a] = 0;
#pragma unroll
  for (int m = 0; m < NP; ++m) pa[pe.e[m][0]] += xp[m] * pr.j[pe.e[m][1]] * pr.z[pe.e[m][2]];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T s = 0;
#pragma unroll
    for (int a = 0; a < P - 1; ++a) s += pa[a] * tb.L[a][i];
    pq[i] = s;
  }
}
template <typename T, int P, int PS>
__device__ __forceinline__ void pressure_interp(const T *xp, const Tab<T, P> &tb, int t, T (&pq)[P]) {
  constexpr int NP = n_pres<P, PS>();
  const int j = t % P, z = t / P;
  constexpr PExp<P, PS> pe{};
  T pa[P - 1];
#pragma unroll
  for (int a = 0; a < P - 1; ++a) pa[a] = 0;
#pragma unroll
  for (int m = 0; m < NP; ++m) pa[pe.e[m][0]] += xp[m] * tb.L[pe.e[m][1]][j] * tb.L[pe.e[m][2]][z];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T s = 0;
#pragma unroll
    for (int a = 0; a < P - 1; ++a) s += pa[a] * tb.L[a][i];
    pq[i] = s;
  }
}
// partial test sums: part[m] = sum_i d[i] psi_m(i, j, z) on the thread's x-line
template <typename T, int P, int PS>
__device__ __forceinline__ void pressure_test(const T (&d)[P], const Tab<T, P> &tb, const PRows<T, P> &pr,
                                              T (&part)[n_pres<P, PS>()]) {
  constexpr int NP = n_pres<P, PS>();
  T qa[P - 1];
#pragma unroll
  for (int a = 0; a < P - 1; ++a) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) s += tb.L[a][i] * d[i];
    qa[a] = s;
  }
  constexpr PExp<P, PS> pe{};
#pragma unroll
  for (int m = 0; m < NP; ++m) part[m] = qa[pe.e[m][0]] * pr.j[pe.e[m][1]] * pr.z[pe.e[m][2]];
}
template <typename T, int P, int PS>
__device__ __forceinline__ void pressure_test(const T (&d)[P], const Tab<T, P> &tb, int t, T (&part)[n_pres<P, PS>()]) {
  constexpr int NP = n_pres<P, PS>();
  const int j = t % P, z = t / P;
  T qa[P - 1];
#pragma unroll
  for (int a = 0; a < P - 1; ++a) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) s += tb.L[a][i] * d[i];
    qa[a] = s;
  }
  constexpr PExp<P, PS> pe{};
#pragma unroll
  for (int m = 0; m < NP; ++m) part[m] = qa[pe.e[m][0]] * tb.L[pe.e[m][1]][j] * tb.L[pe.e[m][2]][z];
}
// Sum the NP partials over the P*P threads of each element and store -sum into y_p[e], in passes
// of as many modes as the element workspace holds.  All threads of the block must call.
template <typename T, int P, int NP>
__device__ void pressure_reduce(const T (&part)[NP], Ws<T, P> w, int t, bool act, T *yp_e) {
  constexpr int P2 = P * P, MC = Ws<T, P>::ES / (P2 + 1);
  static_assert(MC >= 1, "element workspace too small for the pressure reduction");
#pragma unroll
  for (int m0 = 0; m0 < NP; m0 += MC) {
    if (act)
#pragma unroll
      for (int m = m0; m < (m0 + MC < NP ? m0 + MC : NP); ++m) w.s[(m - m0) * (P2 + 1) + t] = part[m];
    __syncthreads();
    if (act && yp_e != nullptr) {
      for (int m = m0 + t; m < (m0 + MC < NP ? m0 + MC : NP); m += P2) {
        T s = 0;
        for (int r = 0; r < P2; ++r) s += w.s[(m - m0) * (P2 + 1) + r];
        yp_e[m] = -s;
      }
    }
    __syncthreads();
  }
}

// double-precision sum over the P*P threads of an element (for parameter gradients)
template <int P>
__device__ double elem_sum64(double v, double *red, int t, bool act) {
  constexpr int P2 = P * P;
  if (act) red[t] = v;
  __syncthreads();
  double s = 0;
  if (act && t == 0)
    for (int r = 0; r < P2; ++r) s += red[r];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- basal face (zeta = -1)
// Face Gauss point (g_i, g_j) <-> thread t = i + P j (the z-line owner of nodes (i, j, .)).
// Interpolates the bottom-node values xb[c] to the face point (B x B).
template <typename T, int P>
__device__ void face_interp(const T (&xb)[3], T (&uq)[3], Ws<T, P> w, const Tab<T, P> &tb, int t, bool act) {
  constexpr int P2 = P * P;
  const int i = t % P, j = t / P;
  // the thread's table rows are requested before the barriers (per-lane table reads)
  T bi[P], bj[P];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    bi[a] = tb.B[i][a];
    bj[a] = tb.B[j][a];
  }
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c) w.b(0)[c * P2 + t] = xb[c];
  __syncthreads();
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < P; ++a) s += bi[a] * w.b(0)[c * P2 + a + P * j];
      w.b(1)[c * P2 + t] = s;
    }
  __syncthreads();
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T s = 0;
#pragma unroll
      for (int b = 0; b < P; ++b) s += bj[b] * w.b(1)[c * P2 + i + P * b];
      uq[c] = s;
    }
}
// Transposed: face-point values tq[c] -> bottom-node contributions out[c] (B^T x B^T).
template <typename T, int P>
__device__ void face_test(const T (&tq)[3], T (&out)[3], Ws<T, P> w, const Tab<T, P> &tb, int t, bool act) {
  constexpr int P2 = P * P;
  const int i = t % P, j = t / P;
  T ci[P], cj[P];   // table columns i and j, requested before the barriers
#pragma unroll
  for (int a = 0; a < P; ++a) {
    ci[a] = tb.B[a][i];
    cj[a] = tb.B[a][j];
  }
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c) w.b(2)[c * P2 + t] = tq[c];
  __syncthreads();
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T s = 0;
#pragma unroll
      for (int jj = 0; jj < P; ++jj) s += cj[jj] * w.b(2)[c * P2 + i + P * jj];
      w.b(3)[c * P2 + t] = s;
    }
  __syncthreads();
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T s = 0;
#pragma unroll
      for (int ii = 0; ii < P; ++ii) s += ci[ii] * w.b(3)[c * P2 + ii + P * j];
      out[c] = s;
    }
  __syncthreads();
}

// ---------------------------------------------------------------- gather / scatter
// Node words of the thread's z-line (node id | Dirichlet mask bits), then the values of x they
// name (0 in masked components).
template <int P>
__device__ __forceinline__ void load_words(const uint32_t *__restrict__ en_e, int t, bool act, uint32_t (&nw)[P]) {
  constexpr int P2 = P * P;
#pragma unroll
  for (int z = 0; z < P; ++z) nw[z] = act ? en_e[t + P2 * z] : 0u;
}
template <typename T, int P>
__device__ __forceinline__ void gather_words(const uint32_t (&nw)[P], const T *x, int64_t N, bool act, bool use_mask,
                                             T (&v)[3][P]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int z = 0; z < P; ++z) {
      const uint32_t wd = nw[z];
      const bool masked = use_mask && ((wd >> (MASK_SHIFT + c)) & 1u);
      v[c][z] = (act && !masked) ? x[c * N + (wd & NODE_MASK)] : T(0);
    }
}
template <typename T, int P>
__device__ __forceinline__ void gather(const uint32_t *en_e, const T *x, int64_t N, int t, bool act, bool use_mask,
                                       T (&v)[3][P], uint32_t (&nw)[P]) {
  load_words<P>(en_e, t, act, nw);
  gather_words<T, P>(nw, x, N, act, use_mask, v);
}

// Nodal frames (u . n = 0 on a curved base, eq. (robin)): a node with a local frame Q holds
// u_hat with u = Q u_hat.  Such nodes are basal and occur only in bottom slots (z = 0): of basal
// elements, and as parents in hanging slots of the elements above them.  Their frames are stored
// per element (row rot_of[e]) and bottom slot.  frame_in turns the gathered local values of the
// bottom slot into Cartesian ones; frame_out applies Q^T to the slot's result.
template <typename T, int P>
__device__ __forceinline__ void frame_load(const T *__restrict__ rot, int row, int t, T (&Q)[9]) {
  constexpr int P2 = P * P;
#pragma unroll
  for (int r = 0; r < 9; ++r) Q[r] = rot[((size_t)row * 9 + r) * P2 + t];
}
template <typename T, int P>
__device__ __forceinline__ void frame_in(T (&v)[3][P], const T (&Q)[9]) {
  const T a = v[0][0], b = v[1][0], c = v[2][0];
  v[0][0] = Q[0] * a + Q[1] * b + Q[2] * c;
  v[1][0] = Q[3] * a + Q[4] * b + Q[5] * c;
  v[2][0] = Q[6] * a + Q[7] * b + Q[8] * c;
}
template <typename T, int P>
__device__ __forceinline__ void frame_out(T (&y)[3][P], const T (&Q)[9]) {
  const T a = y[0][0], b = y[1][0], c = y[2][0];
  y[0][0] = Q[0] * a + Q[3] * b + Q[6] * c;
  y[1][0] = Q[1] * a + Q[4] * b + Q[7] * c;
  y[2][0] = Q[2] * a + Q[5] * b + Q[8] * c;
}

// Element-vector store in node order.  The result of element slot (e, a) for component c goes
// to ev[c * n_inc + pos], pos being the slot's entry in its node's contiguous segment (built at
// upload).  Where two vertically adjacent elements of the block share a z-face, the lower
// element's top slot also takes the upper element's bottom value and the latter is not stored
// (pos = -1): fewer element-vector entries to write and to assemble.  P = 4: each thread stores
// its z-line through pos[e][a]; the block is one wavefront, and the upper element's bottom values
// come from lane + P^2.  P = 3, 5: the block first stages its results in LDS; then lane l writes
// the l-th entry of the block's stored slots sorted by entry, so that adjacent lanes write
// adjacent entries (measured 3% faster there, slower for P = 4).  The staging area reuses the
// block's workspace.
//
// The store positions are read by store_index, separately from the store, so that a kernel can
// request them early and hide their latency behind the element work.
template <int P> struct StoreIndex {
  static constexpr int R = P == 4 ? P : store_slots<P>() / Launch<P>::NT;
  int32_t pos[R];      // P = 4: the thread's z-line slots; else the thread's sorted entries
  uint32_t code[P == 4 ? 1 : R];
};
template <int P>
__device__ __forceinline__ StoreIndex<P> store_index(const MeshView &m, int lb, int64_t e, int t, bool act) {
  constexpr int E = Launch<P>::E, NT = Launch<P>::NT, P2 = P * P, EP3 = E * P2 * P, SB = store_slots<P>();
  StoreIndex<P> ix;
  if constexpr (P == 4) {
#pragma unroll
    for (int z = 0; z < P; ++z) ix.pos[z] = act ? m.pos[e * EP3 / E + t + P2 * z] : 0;
    ix.code[0] = 0;
  } else {
    const int32_t *sp = m.spos + (size_t)lb * SB;
    const uint16_t *ss = m.sslot + (size_t)lb * SB;
#pragma unroll
    for (int r = 0; r < ix.R; ++r) {
      const int k = r * NT + (int)threadIdx.x;
      ix.pos[r] = sp[k];
      ix.code[r] = ss[k];
    }
  }
  return ix;
}
// All threads of the block must call.
template <typename T, int P>
__device__ __forceinline__ void evec_store(T *ev, const MeshView &m, const StoreIndex<P> &ix, T *stage, int el, int t,
                                           bool act, const T (&v)[3][P]) {
  constexpr int E = Launch<P>::E, NT = Launch<P>::NT, P2 = P * P, EP3 = E * P2 * P;
  if constexpr (P == 4) {
    static_assert(NT == 64 && E * P2 == 64, "one wavefront per block expected");
    // bottom slot of the element above (lane + P^2; lanes past the wavefront read their own)
    const int32_t up_pos = __shfl_down(ix.pos[0], P2);
    T up[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) up[c] = __shfl_down(v[c][0], P2);
    if (!act || ev == nullptr) return;
    const bool take_up = el + 1 < E && up_pos < 0;
#pragma unroll
    for (int z = 0; z < P; ++z) {
      if (ix.pos[z] < 0) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) ev[c * m.n_ent + ix.pos[z]] = (z == P - 1 && take_up) ? v[c][z] + up[c] : v[c][z];
    }
  } else {
    static_assert(3 * EP3 <= E * Ws<T, P>::ES, "staging area exceeds the block workspace");
    __syncthreads();
    if (act)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int z = 0; z < P; ++z) stage[c * EP3 + z * E * P2 + el * P2 + t] = v[c][z];
    __syncthreads();
    if (ev == nullptr) return;
#pragma unroll
    for (int r = 0; r < ix.R; ++r) {
      const int32_t pos = ix.pos[r];
      if (pos >= 0) {
        const int code = (int)ix.code[r], sl = code & 0x7FFF;
        // merged top slot: add the bottom slot (el + 1, x, y, 0) of the element above
        const int below = sl - (P - 1) * E * P2 + P2;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          ev[c * m.n_ent + pos] = (code & 0x8000) ? stage[c * EP3 + sl] + stage[c * EP3 + below] : stage[c * EP3 + sl];
      }
    }
  }
}
template <typename T, int P>
__device__ __forceinline__ void evec_store(T *ev, const MeshView &m, int lb, int64_t e, T *stage, int el, int t,
                                           bool act, const T (&v)[3][P]) {
  evec_store<T, P>(ev, m, store_index<P>(m, lb, e, t, act), stage, el, t, act, v);
}

// ================================================================= kernels
// Jacobian apply (and VJP) of one element: y = J_e x_e at the stored linearisation point for the
// element e of block lb, slot els, given the node words nw of the thread's z-line; writes the
// element's pressure rows (and parameter gradients) and leaves the velocity rows, after R_e^T, in y.
// All threads of the block call it (barriers inside); HANG = false compiles the hanging-node
// interpolation out (meshes without hanging faces).
template <typename T, int P, int GEO, bool VJP, int PS, bool FR, bool HANG>
__device__ __forceinline__ void apply_elem(const MeshView &m, const GeoView<T> &gv, const Tab<T, P> &tb,
                                           const void *__restrict__ st_, const T *__restrict__ fst,
                                           const T *__restrict__ beta, const T *__restrict__ xu,
                                           const T *__restrict__ xp, T *__restrict__ yp, double inv_n,
                                           double *__restrict__ g_logA, double *__restrict__ g_beta, T *smem,
                                           double *red, int lb, int tid, int t, int els, int64_t e, bool act,
                                           const uint32_t (&nw)[P], T (&y)[3][P]) {
  constexpr int NT = Launch<P>::NT, P2 = P * P;
  constexpr int NP = n_pres<P, PS>();
  Ws<T, P> w{smem + els * Ws<T, P>::ES};
  double *redl = red + els * red_stride<P, PS>();
  const int64_t N = m.n_nodes;
  // the linearisation data of the thread's P points are requested right after the connectivity
  // (the caller's) so that their latency overlaps the gather and the forward sweeps, for P = 4 and for
  // FP32 with P = 5.  Elsewhere they are loaded just before the quadrature-point step: in FP64 with
  // P = 3, 5 the extra live registers would cost occupancy, and with FP32 and P = 3 the early request
  // measured 4% slower.  The tile's slice is always allocated, also for threads without an element.
  const uint32_t cm = (HANG && act) ? m.cmask[e] : 0u;
  // basal face of the element, needed after the transposed sweeps: for P = 3, 5 requested here, so
  // that the block does not wait on it at the barrier before the Robin term (element kernel 1% faster
  // on the Q4 terrain, 2% on the Q2 dome); for P = 4 the early request measured 2% slower
  int fid = -1;
  if constexpr (P != 4) fid = act ? m.bface_of[e] : -1;
  // FP32 apply: the 7-value FP32 state; FP64 and the VJP (which needs Sigma0 : D itself for the
  // logA gradient): the 8-value FP64 state
  constexpr bool kS32 = sizeof(T) == 4 && !VJP;
  using ST = std::conditional_t<kS32, float, double>;
  constexpr int NF = kS32 ? NSTATE32 : NSTATE;
  const ST *__restrict__ st = reinterpret_cast<const ST *>(st_);
  constexpr bool kEarlyState = P == 4 || (P == 5 && sizeof(ST) == 4);
  ST stv[NF][P];
  if constexpr (kEarlyState) {
#pragma unroll
    for (int f = 0; f < NF; ++f) load_field<ST, P, NT, NF>(st, lb, f, tid, stv[f]);
  }
  T v[3][P];
  gather_words<T, P>(nw, xu, N, act, true, v);
  const bool rot = FR && act && (nw[0] & ROT_BIT);   // FR: the mesh has nodal frames
  if (rot) {
    T Q[9];
    frame_load<T, P>(gv.rot, m.rot_of[e], t, Q);
    frame_in<T, P>(v, Q);
  }
  // geometry and pressure coefficients are needed only after the forward sweeps; requesting them
  // here hides their latency behind the sweeps (per-point geometry of column-mapped elements).
  // The element's NP pressure coefficients are loaded once each (thread t < NP takes mode t) and
  // passed through LDS (the parameter-gradient reduction area, not in use until after the
  // quadrature-point step), instead of every thread holding all of them through the sweeps.
  constexpr int NPT = (NP + P2 - 1) / P2;   // modes per thread
  QpGeo<T, P, GEO> g;
  T xpt[NPT];
  if (act) {
    load_geo<T, P, GEO, NT>(g, gv, e, lb, tid, tb, t);
#pragma unroll
    for (int r = 0; r < NPT; ++r)
      if (t + r * P2 < NP) xpt[r] = xp[e * NP + t + r * P2];
  }
  if constexpr (HANG)
    if (m.any_hang && __syncthreads_or(act && (cm >> 3) != 0u)) hang_fwd<T, P>(v, cm, w, tb, t, act);
  const T xb[3] = {v[0][0], v[1][0], v[2][0]};

  T gr[3][3][P];
  // FP32 with P = 4, 5: the thread's pressure factors are requested before the forward sweeps and
  // kept for the test (element kernel 2% faster on the Q4 terrain); FP64 and P = 3 read them at
  // each use, where the held registers would cost a wavefront per SIMD
  constexpr bool kRows = sizeof(T) == 4 && P != 3;
  PRows<T, P> pr{};
  if constexpr (kRows) pr = pressure_rows<T, P>(tb, t);
#pragma unroll
  for (int c = 0; c < 3; ++c) grad_fwd<T, P>(v[c], gr[c][0], gr[c][1], gr[c][2], w, tb, t, act);
  T *xps = reinterpret_cast<T *>(redl);
  if (act)
#pragma unroll
    for (int r = 0; r < NPT; ++r)
      if (t + r * P2 < NP) xps[t + r * P2] = xpt[r];
  __syncthreads();

  T pq[P];
  if (act) {
    if constexpr (kRows) pressure_interp<T, P, PS>(xps, tb, pr, pq);
    else pressure_interp<T, P, PS>(xps, tb, t, pq);
  }
  T dw[P];
  double gA = 0.0;
  if constexpr (!kEarlyState) {
#pragma unroll
    for (int f = 0; f < NF; ++f) load_field<ST, P, NT, NF>(st, lb, f, tid, stv[f]);
  }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    if (!act) { dw[i] = 0; continue; }
    T grr[3][3], G[3][3], tau[3][3], f[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 3; ++r) grr[c][r] = gr[c][r][i];
    to_phys<T, P, GEO>(g, i, grr, G);
    constexpr int S0 = kS32 ? 1 : 2;   // first Sigma field
    const T mu = (T)stv[0][i], ka = kS32 ? T(1) : (T)stv[kS32 ? 0 : 1][i];
    const T sxx = (T)stv[S0][i], syy = (T)stv[S0 + 1][i], szz = (T)stv[S0 + 2][i];
    const T sxy = (T)stv[S0 + 3][i], sxz = (T)stv[S0 + 4][i], syz = (T)stv[S0 + 5][i];
    // D = sym(G): off-diagonal entries kept doubled (exy = 2 Dxy) so that Sigma0 : D takes no
    // extra factors; tau = mu' D - kappa (Sigma0 : D) Sigma0 - p w detJ I
    const T dxx = G[0][0], dyy = G[1][1], dzz = G[2][2];
    const T exy = G[0][1] + G[1][0], exz = G[0][2] + G[2][0], eyz = G[1][2] + G[2][1];
    T s = sxx * dxx;
    s += syy * dyy;
    s += szz * dzz;
    s += sxy * exy;
    s += sxz * exz;
    s += syz * eyz;
    if (VJP) gA += (double)s;
    const T ks = kS32 ? s : ka * s, muh = T(0.5) * mu;
    const T wd = g.wdet(tb, i);
    const T pw = pq[i] * wd;
    tau[0][0] = mu * dxx - (ks * sxx + pw);
    tau[1][1] = mu * dyy - (ks * syy + pw);
    tau[2][2] = mu * dzz - (ks * szz + pw);
    tau[0][1] = tau[1][0] = muh * exy - ks * sxy;
    tau[0][2] = tau[2][0] = muh * exz - ks * sxz;
    tau[1][2] = tau[2][1] = muh * eyz - ks * syz;
    dw[i] = (dxx + dyy + dzz) * wd;
    to_ref<T, P, GEO>(g, i, tau, f);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 3; ++r) gr[c][r][i] = f[c][r];
  }
  // pressure rows: y_p[e][m] = -sum_q w detJ psi_m div x
  {
    T part[NP];
    if (act) {
      if constexpr (kRows) pressure_test<T, P, PS>(dw, tb, pr, part);
      else pressure_test<T, P, PS>(dw, tb, t, part);
    }
    pressure_reduce<T, P, NP>(part, w, t, act, (act && yp != nullptr) ? yp + e * NP : nullptr);
  }
  if (VJP) {
    const double sA = elem_sum64<P>(gA, redl, t, act);
    if (act && t == 0 && g_logA != nullptr) g_logA[e] = -inv_n * sA;
  }
  const T zero[P] = {};
#pragma unroll
  for (int c = 0; c < 3; ++c) grad_bwd<T, P, false>(gr[c][0], gr[c][1], gr[c][2], zero, y[c], w, tb, t, act);
  // basal Robin term on the zeta = -1 face: y += int beta (T x).(T v)
  if constexpr (P == 4) fid = act ? m.bface_of[e] : -1;
  if (__syncthreads_or(fid >= 0)) {
    T uq[3], tq[3], out[3];
    // the face point's geometry and beta are requested before the interpolation's barriers
    T ws = 0, n0 = 0, n1 = 0, n2 = 0, bf = 0;
    if (fid >= 0) {
      const T *fg = gv.face + (size_t)fid * NFACEGEO * P2;
      ws = fg[t];
      n0 = fg[P2 + t];
      n1 = fg[2 * P2 + t];
      n2 = fg[3 * P2 + t];
      bf = beta[fid];
    }
    face_interp<T, P>(xb, uq, w, tb, t, act);
    double gb = 0.0;
    if (fid >= 0) {
      const T bw = bf * ws;
      const T nu = n0 * uq[0] + n1 * uq[1] + n2 * uq[2];
      tq[0] = bw * (uq[0] - n0 * nu);
      tq[1] = bw * (uq[1] - n1 * nu);
      tq[2] = bw * (uq[2] - n2 * nu);
      if (VJP) {
        const T *fs = fst + (size_t)fid * NFACEST * P2;
        gb = (double)fs[t] * uq[0] + (double)fs[P2 + t] * uq[1] + (double)fs[2 * P2 + t] * uq[2];
      }
    } else {
      tq[0] = tq[1] = tq[2] = 0;
    }
    face_test<T, P>(tq, out, w, tb, t, act);
    if (fid >= 0)
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c][0] += out[c];
    if (VJP) {
      const double sb = elem_sum64<P>(gb, redl, t, act);
      if (fid >= 0 && t == 0 && g_beta != nullptr) g_beta[fid] = sb;
    }
  }
  if constexpr (HANG)
    if (m.any_hang && __syncthreads_or(act && (cm >> 3) != 0u)) hang_bwd<T, P>(y, cm, w, tb, t, act);
  if (rot) {
    T Q[9];
    frame_load<T, P>(gv.rot, m.rot_of[e], t, Q);
    frame_out<T, P>(y, Q);
  }
}

// Jacobian apply (and VJP): y = J_c x at the stored linearisation point, E consecutive elements per
// block, results through the node-ordered element vector (assembled by k_assemble).
template <typename T, int P, int GEO, bool VJP, int PS, bool FR>
__global__ void __launch_bounds__(Launch<P>::NT)
k_apply(MeshView m, GeoView<T> gv, const Tab<T, P> *__restrict__ tbp, const void *__restrict__ st_, const T *__restrict__ fst,
        const T *__restrict__ beta, const T *__restrict__ xu, const T *__restrict__ xp, T *__restrict__ yu,
        T *__restrict__ yp, double inv_n, double *__restrict__ g_logA, double *__restrict__ g_beta) {
  constexpr int E = Launch<P>::E, P2 = P * P, P3 = P2 * P;
  __shared__ T smem[E * Ws<T, P>::ES];
  __shared__ double red[E * red_stride<P, PS>()];
  const int lb = logical_block();
  const int tid = threadIdx.x, el = tid / P2, t = tid % P2;
  const int64_t e = tile_elem<E>(m, lb, el);
  const bool act = e >= 0;
  const int els = el < E ? el : E - 1;
  // connectivity first: the gather of x waits on it.  The store positions are requested at once
  // too, so that their latency is hidden behind the element work instead of stalling the block's
  // end, except in FP64 with P = 5, where the extra live registers would halve the occupancy.
  constexpr bool kEarlyIndex = !(sizeof(T) == 8 && P == 5);
  uint32_t nw[P];
  load_words<P>(m.en + e * P3, t, act, nw);
  StoreIndex<P> ix;
  if constexpr (kEarlyIndex) ix = store_index<P>(m, lb, e, t, act);
  T y[3][P];
  apply_elem<T, P, GEO, VJP, PS, FR, true>(m, gv, *tbp, st_, fst, beta, xu, xp, yp, inv_n, g_logA, g_beta, smem, red, lb,
                                           tid, t, els, e, act, nw, y);
  if constexpr (!kEarlyIndex) ix = store_index<P>(m, lb, e, t, act);
  evec_store<T, P>(yu, m, ix, smem, els, t, act, y);
}


// Pressure gradient y = B^T x_p (eq. (weak): the term -int p div v), the velocity rows of the
// Jacobian apply at zero velocity: per quadrature point only tau = -p w detJ I, so the gather, the
// forward sweeps, the linearisation data and the basal term drop out; the transposed sweeps, R_e^T,
// the frames and the element-vector store are those of k_apply.
template <typename T, int P, int GEO, int PS, bool FR>
__global__ void __launch_bounds__(Launch<P>::NT)
k_grad_p(MeshView m, GeoView<T> gv, const Tab<T, P> *__restrict__ tbp, const T *__restrict__ xp, T *__restrict__ yu) {
  constexpr int E = Launch<P>::E, NT = Launch<P>::NT, P2 = P * P, P3 = P2 * P;
  constexpr int NP = n_pres<P, PS>(), NPT = (NP + P2 - 1) / P2;
  __shared__ T smem[E * Ws<T, P>::ES];
  __shared__ double red[E * red_stride<P, PS>()];
  const Tab<T, P> &tb = *tbp;
  const int lb = logical_block();
  const int tid = threadIdx.x, el = tid / P2, t = tid % P2;
  const int64_t e = tile_elem<E>(m, lb, el);
  const bool act = e >= 0;
  const int els = el < E ? el : E - 1;
  Ws<T, P> w{smem + els * Ws<T, P>::ES};
  // in order of use: the pressure coefficients and factors (before the barrier), then geometry,
  // then what the transposed sweeps and the store need
  T xpt[NPT];
  if (act)
#pragma unroll
    for (int r = 0; r < NPT; ++r)
      if (t + r * P2 < NP) xpt[r] = xp[e * NP + t + r * P2];
  const PRows<T, P> pr = pressure_rows<T, P>(tb, t);
  QpGeo<T, P, GEO> g;
  if (act) load_geo<T, P, GEO, NT>(g, gv, e, lb, tid, tb, t);
  const StoreIndex<P> ix = store_index<P>(m, lb, e, t, act);
  const uint32_t cm = act ? m.cmask[e] : 0u;
  const bool rot = FR && act && (m.en[e * P3 + t] & ROT_BIT);
  T *xps = reinterpret_cast<T *>(red + els * red_stride<P, PS>());
  if (act)
#pragma unroll
    for (int r = 0; r < NPT; ++r)
      if (t + r * P2 < NP) xps[t + r * P2] = xpt[r];
  __syncthreads();
  T pq[P];
  if (act) pressure_interp<T, P, PS>(xps, tb, pr, pq);
  T f[3][3][P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T tau[3][3], ff[3][3];
    const T pw = act ? pq[i] * g.wdet(tb, i) : T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 3; ++r) tau[c][r] = c == r ? -pw : T(0);
    to_ref<T, P, GEO>(g, i, tau, ff);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 3; ++r) f[c][r][i] = act ? ff[c][r] : T(0);
  }
  T y[3][P];
  const T zero[P] = {};
#pragma unroll
  for (int c = 0; c < 3; ++c) grad_bwd<T, P, false>(f[c][0], f[c][1], f[c][2], zero, y[c], w, tb, t, act);
  if (m.any_hang && __syncthreads_or(act && (cm >> 3) != 0u)) hang_bwd<T, P>(y, cm, w, tb, t, act);
  if (rot) {
    T Q[9];
    frame_load<T, P>(gv.rot, m.rot_of[e], t, Q);
    frame_out<T, P>(y, Q);
  }
  evec_store<T, P>(yu, m, ix, smem, els, t, act, y);
}

// Linearisation point: per quadrature point mu' = w detJ mu, kappa, Sigma0 = mu' D(u)
// (FP64, eq. (glen) and eq. (rank4)); per basal face point w|S| T u.  The Picard operator keeps
// mu and drops the D (x) D part of the tensor: kappa = 0.
template <int P, int GEO>
__global__ void __launch_bounds__(Launch<P>::NT)
k_state(MeshView m, GeoView<double> gv, const Tab<double, P> *__restrict__ tbp, const double *__restrict__ u,
        const double *__restrict__ logA, double n, double eps, double B0, int picard, double *__restrict__ st64,
        float *__restrict__ st32, double *__restrict__ fst64, float *__restrict__ fst32) {
  using T = double;
  const Tab<T, P> &tb = *tbp;
  constexpr int NT = Launch<P>::NT, E = Launch<P>::E, P2 = P * P, P3 = P2 * P;
  __shared__ T smem[E * Ws<T, P>::ES];
  const int lb = logical_block();
  const int tid = threadIdx.x, el = tid / P2, t = tid % P2;
  const int64_t e = tile_elem<E>(m, lb, el);
  const bool act = e >= 0;
  const int els = el < E ? el : E - 1;
  Ws<T, P> w{smem + els * Ws<T, P>::ES};
  const int64_t N = m.n_nodes;
  const uint32_t cm = act ? m.cmask[e] : 0u;
  T v[3][P];
  uint32_t nw[P];
  gather<T, P>(m.en + e * P3, u, N, t, act, true, v, nw);
  if (act && (nw[0] & ROT_BIT)) {
    T Q[9];
    frame_load<T, P>(gv.rot, m.rot_of[e], t, Q);
    frame_in<T, P>(v, Q);
  }
  if (m.any_hang && __syncthreads_or(act && (cm >> 3) != 0u)) hang_fwd<T, P>(v, cm, w, tb, t, act);
  const T xb[3] = {v[0][0], v[1][0], v[2][0]};
  T gr[3][3][P];
#pragma unroll
  for (int c = 0; c < 3; ++c) grad_fwd<T, P>(v[c], gr[c][0], gr[c][1], gr[c][2], w, tb, t, act);
  __syncthreads();
  if (act) {
    QpGeo<T, P, GEO> g;
    load_geo<T, P, GEO, NT>(g, gv, e, lb, tid, tb, t);
    const double Be = B0 * exp(-logA[e] / n);
    const double expo = (1.0 - n) / (2.0 * n), cf = picard ? 0.0 : (n - 1.0) / (2.0 * n);
    double *s64 = st64;
    float *s32 = st32;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      T grr[3][3], G[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) grr[c][r] = gr[c][r][i];
      to_phys<T, P, GEO>(g, i, grr, G);
      const T dxx = G[0][0], dyy = G[1][1], dzz = G[2][2];
      const T dxy = 0.5 * (G[0][1] + G[1][0]), dxz = 0.5 * (G[0][2] + G[2][0]), dyz = 0.5 * (G[1][2] + G[2][1]);
      const T II = 0.5 * (dxx * dxx + dyy * dyy + dzz * dzz) + dxy * dxy + dxz * dxz + dyz * dyz;
      const T mu = Be * pow(II + eps, expo);
      const T mup = g.wdet(tb, i) * mu;
      const T ka = cf / ((II + eps) * mup);
      const T vals[NSTATE] = {mup, ka, mup * dxx, mup * dyy, mup * dzz, mup * dxy, mup * dxz, mup * dyz};
#pragma unroll
      for (int f = 0; f < NSTATE; ++f) st_store<P>(s64 + qp_at<P, NT, NSTATE>(lb, f, tid, i), vals[f]);
      const T sk = sqrt(ka);
      st_store<P>(s32 + qp_at<P, NT, NSTATE32>(lb, 0, tid, i), (float)mup);
#pragma unroll
      for (int f = 0; f < 6; ++f) st_store<P>(s32 + qp_at<P, NT, NSTATE32>(lb, 1 + f, tid, i), (float)(sk * vals[2 + f]));
    }
  }
  const int fid = act ? m.bface_of[e] : -1;
  if (__syncthreads_or(fid >= 0)) {
    T uq[3];
    face_interp<T, P>(xb, uq, w, tb, t, act);
    if (fid >= 0) {
      const T *fg = gv.face + (size_t)fid * NFACEGEO * P2;
      const T ws = fg[t], n0 = fg[P2 + t], n1 = fg[2 * P2 + t], n2 = fg[3 * P2 + t];
      const T nu = n0 * uq[0] + n1 * uq[1] + n2 * uq[2];
      const T b[3] = {ws * (uq[0] - n0 * nu), ws * (uq[1] - n1 * nu), ws * (uq[2] - n2 * nu)};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        fst64[(size_t)fid * NFACEST * P2 + c * P2 + t] = b[c];
        fst32[(size_t)fid * NFACEST * P2 + c * P2 + t] = (float)b[c];
      }
    }
  }
}

// Residual at the linearisation point (FP64): tau = Sigma0 - p w detJ I, body force,
// basal term beta w|S| T u, pressure rows -int psi div u.
template <int P, int GEO, int PS>
__global__ void __launch_bounds__(Launch<P>::NT)
k_residual(MeshView m, GeoView<double> gv, const Tab<double, P> *__restrict__ tbp, const double *__restrict__ st,
           const double *__restrict__ fst, const double *__restrict__ beta, const double *__restrict__ p, double bx,
           double by, double bz, double *__restrict__ ru, double *__restrict__ rp) {
  using T = double;
  const Tab<T, P> &tb = *tbp;
  constexpr int NT = Launch<P>::NT, E = Launch<P>::E, P2 = P * P, P3 = P2 * P;
  constexpr int NP = n_pres<P, PS>();
  __shared__ T smem[E * Ws<T, P>::ES];
  const int lb = logical_block();
  const int tid = threadIdx.x, el = tid / P2, t = tid % P2;
  const int64_t e = tile_elem<E>(m, lb, el);
  const bool act = e >= 0;
  const int els = el < E ? el : E - 1;
  const int fid = act ? m.bface_of[e] : -1;   // basal face, requested with the element's first data
  Ws<T, P> w{smem + els * Ws<T, P>::ES};
  const int64_t N = m.n_nodes;
  const uint32_t cm = act ? m.cmask[e] : 0u;
  uint32_t nw[P];
  load_words<P>(m.en + e * P3, t, act, nw);

  T fr[3][3][P], f0[3][P], dw[P];
  if (act) {
    QpGeo<T, P, GEO> g;
    load_geo<T, P, GEO, NT>(g, gv, e, lb, tid, tb, t);
    T pq[P], xpl[NP];
#pragma unroll
    for (int mm = 0; mm < NP; ++mm) xpl[mm] = p[e * NP + mm];
    pressure_interp<T, P, PS>(xpl, tb, t, pq);
    T stv[NSTATE][P];
#pragma unroll
    for (int f = 0; f < NSTATE; ++f) load_field<T, P, NT, NSTATE>(st, lb, f, tid, stv[f]);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const T mu = stv[0][i];
      const T sxx = stv[2][i], syy = stv[3][i], szz = stv[4][i];
      const T sxy = stv[5][i], sxz = stv[6][i], syz = stv[7][i];
      const T wd = g.wdet(tb, i);
      const T pw = pq[i] * wd;
      T tau[3][3] = {{sxx - pw, sxy, sxz}, {sxy, syy - pw, syz}, {sxz, syz, szz - pw}};
      T f[3][3];
      to_ref<T, P, GEO>(g, i, tau, f);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) fr[c][r][i] = f[c][r];
      f0[0][i] = -bx * wd;
      f0[1][i] = -by * wd;
      f0[2][i] = -bz * wd;
      dw[i] = (sxx + syy + szz) / mu * wd;
    }
  } else {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      dw[i] = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        f0[c][i] = 0;
#pragma unroll
        for (int r = 0; r < 3; ++r) fr[c][r][i] = 0;
      }
    }
  }
  {
    T part[NP];
    if (act) pressure_test<T, P, PS>(dw, tb, t, part);
    pressure_reduce<T, P, NP>(part, w, t, act, act ? rp + e * NP : nullptr);
  }
  T y[3][P];
#pragma unroll
  for (int c = 0; c < 3; ++c) grad_bwd<T, P, true>(fr[c][0], fr[c][1], fr[c][2], f0[c], y[c], w, tb, t, act);
  // the basal term's face data are requested before the vote's barriers
  T tq[3] = {0, 0, 0};
  if (fid >= 0) {
    const T *fs = fst + (size_t)fid * NFACEST * P2;
#pragma unroll
    for (int c = 0; c < 3; ++c) tq[c] = beta[fid] * fs[c * P2 + t];
  }
  if (__syncthreads_or(fid >= 0)) {
    T out[3];
    face_test<T, P>(tq, out, w, tb, t, act);
    if (fid >= 0)
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c][0] += out[c];
  }
  if (m.any_hang && __syncthreads_or(act && (cm >> 3) != 0u)) hang_bwd<T, P>(y, cm, w, tb, t, act);
  if (act && (nw[0] & ROT_BIT)) {
    T Q[9];
    frame_load<T, P>(gv.rot, m.rot_of[e], t, Q);
    frame_out<T, P>(y, Q);
  }
  evec_store<T, P>(ru, m, lb, e, smem, els, t, act, y);
}

// Block-Jacobi data at the linearisation point (FP64).  Velocity: the diagonal of F per
// component, sum over quadrature points of mu'/2 (|grad phi_a|^2 + (d_c phi_a)^2) - kappa
// ((Sigma0 grad phi_a)_c)^2 (eq. (rank4) tested with phi_a e_c), plus the basal term
// beta w|S| phi_a^2 (1 - n_c^2); hanging slots reach their parent nodes through squared
// interpolation weights (tb2), i.e. sum_e sum_a R_e[a,n]^2 F_e[a,a].  Pressure: the lumped
// mass weighted by 1/mu with a minus sign, the Schur-complement approximation of Sec. 6.
// (three wavefronts per SIMD requested: the FP64 Q4 kernel otherwise takes 228 VGPRs, two
// wavefronts; with the bound it spills 4 and runs 5% faster)
template <int P, int GEO, int PS, bool FR>
__global__ void __launch_bounds__(Launch<P>::NT, 3)
k_diag(MeshView m, GeoView<double> gv, const Tab<double, P> *__restrict__ tbp,
       const Tab<double, P> *__restrict__ tb2p, const double *__restrict__ st,
       const double *__restrict__ beta, double *__restrict__ ev, double *__restrict__ dp) {
  using T = double;
  const Tab<T, P> &tb = *tbp, &tb2 = *tb2p;
  constexpr int NT = Launch<P>::NT, E = Launch<P>::E, P2 = P * P, P3 = P2 * P;
  constexpr int NP = n_pres<P, PS>();
  __shared__ T smem[E * Ws<T, P>::ES];
  const int lb = logical_block();
  const int tid = threadIdx.x, el = tid / P2, t = tid % P2;
  const int64_t e = tile_elem<E>(m, lb, el);
  const bool act = e >= 0;
  const int els = el < E ? el : E - 1;
  Ws<T, P> w{smem + els * Ws<T, P>::ES};
  const uint32_t cm = act ? m.cmask[e] : 0u;
  uint32_t nw[P];
  load_words<P>(m.en + e * P3, t, act, nw);
  T y[3][P], yo[3][P];   // yo: off-diagonal entries (xy, xz, yz) of the slot's 3x3 block
  T part[NP];
#pragma unroll
  for (int mm = 0; mm < NP; ++mm) part[mm] = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int z = 0; z < P; ++z) y[c][z] = yo[c][z] = 0;
  // elements with framed bottom slots: the whole 3x3 blocks, so that a node in a local frame Q
  // gets q_c^T (sum_a R[a, n]^2 F_aa) q_c (FR: the mesh has nodal frames)
  const bool offd = FR && act && m.rot_of[e] >= 0;
  const int i = t % P, j = t / P;            // slot (i, j, z) of the z-line
  double jx = 0, jy = 0, jz = 0, detJ = 0;
  if (act) {
    if (GEO == GEO_AFFINE) {
      jx = gv.el[4 * e]; jy = gv.el[4 * e + 1]; jz = gv.el[4 * e + 2]; detJ = gv.el[4 * e + 3];
    } else {
      jx = gv.el[2 * e]; jy = gv.el[2 * e + 1];
    }
  }
  // The element's quadrature points are visited one z-plane (qz) at a time: thread t first stages
  // the state and geometry of point (qx, qy) = (t % P, t / P) of the plane in the element's
  // workspace, then every thread reads the plane from LDS (one load latency per plane instead of
  // one per point).  Points are visited in the same order as a plain loop over (qy + P qz, qx).
  constexpr int NV = NSTATE + NGEOQP;        // staged values per point
  static_assert(NV * P2 <= Ws<T, P>::ES, "plane staging exceeds the element workspace");
  T *stg = w.s;
#pragma unroll 1
  for (int qz = 0; qz < P; ++qz) {
    __syncthreads();
    if (act) {
      const int tidq = el * P2 + j + P * qz;   // x-line (qy, qz) = (j, qz), point qx = i
#pragma unroll
      for (int f = 0; f < NSTATE; ++f) stg[f * P2 + t] = st[qp_at<P, NT, NSTATE>(lb, f, tidq, i)];
      if (GEO != GEO_AFFINE)
#pragma unroll
        for (int f = 0; f < NGEOQP; ++f) stg[(NSTATE + f) * P2 + t] = gv.qp[qp_at<P, NT, NGEOQP>(lb, f, tidq, i)];
    }
    __syncthreads();
    if (act)
#pragma unroll 1
      for (int qy = 0; qy < P; ++qy) {
        const int tq = qy + P * qz;
#pragma unroll 1
        for (int qx = 0; qx < P; ++qx) {
          const int pt = qx + P * qy;
          const double mu = stg[pt];
          const double ka = stg[P2 + pt];
          double S[6];
          for (int f = 0; f < 6; ++f) S[f] = stg[(2 + f) * P2 + pt];
          double a = 0, b = 0, cc = jz, wd;
          if (GEO == GEO_AFFINE) {
            wd = tb.w[qx] * tb.w[qy] * tb.w[qz] * detJ;
          } else {
            a = stg[NSTATE * P2 + pt];
            b = stg[(NSTATE + 1) * P2 + pt];
            cc = stg[(NSTATE + 2) * P2 + pt];
            wd = tb.w[qx] * tb.w[qy] * tb.w[qz] / (jx * jy * cc);
          }
          // pressure: thread (j, z) of the x-line layout owns points (., j, z); here every
          // thread accumulates the points of its own tq = t for the lumped 1/mu mass
          if (tq == t) {
            const double g = wd * wd / mu;
            constexpr PExp<P, PS> pe{};
#pragma unroll
            for (int mm = 0; mm < NP; ++mm) {
              const double psi = tb.L[pe.e[mm][0]][qx] * tb.L[pe.e[mm][1]][qy] * tb.L[pe.e[mm][2]][qz];
              part[mm] += g * psi * psi;
            }
          }
          for (int z = 0; z < P; ++z) {
            const double gr0 = tb.D[qx][i] * tb.B[qy][j] * tb.B[qz][z];
            const double gr1 = tb.B[qx][i] * tb.D[qy][j] * tb.B[qz][z];
            const double gr2 = tb.B[qx][i] * tb.B[qy][j] * tb.D[qz][z];
            double G[3];
            if (GEO == GEO_AFFINE) {
              G[0] = gr0 * jx; G[1] = gr1 * jy; G[2] = gr2 * jz;
            } else {
              G[0] = gr0 * jx + gr2 * a; G[1] = gr1 * jy + gr2 * b; G[2] = gr2 * cc;
            }
            const double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
            const double SG[3] = {S[0] * G[0] + S[3] * G[1] + S[4] * G[2], S[3] * G[0] + S[1] * G[1] + S[5] * G[2],
                                  S[4] * G[0] + S[5] * G[1] + S[2] * G[2]};
            for (int c = 0; c < 3; ++c) y[c][z] += 0.5 * mu * (g2 + G[c] * G[c]) - ka * SG[c] * SG[c];
            if (offd) {
              yo[0][z] += 0.5 * mu * G[0] * G[1] - ka * SG[0] * SG[1];
              yo[1][z] += 0.5 * mu * G[0] * G[2] - ka * SG[0] * SG[2];
              yo[2][z] += 0.5 * mu * G[1] * G[2] - ka * SG[1] * SG[2];
            }
          }
        }
      }
  }
  __syncthreads();   // the workspace is reused below
  if (act) {
    const int fid = m.bface_of[e];
    if (fid >= 0) {
      const double *fg = gv.face + (size_t)fid * NFACEGEO * P2;
      for (int fq = 0; fq < P2; ++fq) {
        const double phi = tb.B[fq % P][i] * tb.B[fq / P][j];
        const double bw = beta[fid] * fg[fq] * phi * phi;
        for (int c = 0; c < 3; ++c) {
          const double nc = fg[(1 + c) * P2 + fq];
          y[c][0] += bw * (1.0 - nc * nc);
        }
        if (offd) {
          const double n0 = fg[P2 + fq], n1 = fg[2 * P2 + fq], n2 = fg[3 * P2 + fq];
          yo[0][0] -= bw * n0 * n1;
          yo[1][0] -= bw * n0 * n2;
          yo[2][0] -= bw * n1 * n2;
        }
      }
    }
  }
  // lumped -M(1/mu): thread t holds the points of x-line t, reduce over the element's threads
  pressure_reduce<T, P, NP>(part, w, t, act, act ? dp + e * NP : nullptr);
  const bool hang = m.any_hang && __syncthreads_or(act && (cm >> 3) != 0u);
  if (hang) hang_bwd<T, P>(y, cm, w, tb2, t, act);
  if constexpr (FR) {
    if (hang && __syncthreads_or(offd)) hang_bwd<T, P>(yo, cm, w, tb2, t, act);
  }
  if (FR && act && (nw[0] & ROT_BIT)) {
    double Q[9];
    frame_load<T, P>(gv.rot, m.rot_of[e], t, Q);
    const double d00 = y[0][0], d11 = y[1][0], d22 = y[2][0], d01 = yo[0][0], d02 = yo[1][0], d12 = yo[2][0];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double a = Q[c], b = Q[3 + c], g = Q[6 + c];   // column c of Q
      y[c][0] = a * a * d00 + b * b * d11 + g * g * d22 + 2.0 * (a * b * d01 + a * g * d02 + b * g * d12);
    }
  }
  evec_store<T, P>(ev, m, lb, e, smem, els, t, act, y);
}

// ---------------------------------------------------------------- vertical-line blocks
// Preconditioner data beside block Jacobi (the paper's AMG is not part of this engine): for every
// vertical line of nodes and velocity component, the block of F restricted to the line.  Thin
// columns couple strongly along z (element aspect ratios 16-300), which point Jacobi cannot
// resolve; the line blocks are banded (bandwidth k) and symmetric positive definite.

// Device twin of zline_run_host: the run lo..hi of independent slots on the z-line (i, j), false
// when the whole line lies on a hanging face or edge.
template <int P> __device__ __forceinline__ bool zline_run(uint32_t cm, int i, int j, int &lo, int &hi) {
  const uint32_t f = cm >> 3;
  if (zline_hanging<P>(cm, i, j)) return false;
  lo = (((f >> 4) & 1u) || edge_on<P>(cm, 0, j, 0) || edge_on<P>(cm, 1, i, 0)) ? 1 : 0;
  hi = (((f >> 5) & 1u) || edge_on<P>(cm, 0, j, P - 1) || edge_on<P>(cm, 1, i, P - 1)) ? P - 2 : P - 1;
  return true;
}

// Element line blocks at the linearisation point (FP64).  For the run lo..hi of independent slots
// on the z-line (i, j) of element e and component c: F_e[(i,j,za,c), (i,j,zb,c)] = sum over the element's quadrature
// points of mu'/2 (grad phi_a . grad phi_b + d_c phi_a d_c phi_b) - kappa (Sigma0 grad phi_a)_c
// (Sigma0 grad phi_b)_c (eq. (rank4) tested with phi_a e_c and phi_b e_c), plus the basal term on
// za = zb = 0.  Each slot stores its row towards the slots below it: buf[(c n_inc + slot) P + d] =
// F_e[zb, zb - d], d = 0..k (0 where zb - d < lo), for zb = lo..hi.  Dependent slots store nothing
// (couplings through hanging constraints are left out of the preconditioner).
template <int P, int GEO, bool FR>
__global__ void __launch_bounds__(Launch<P>::NT)
k_lines(MeshView m, GeoView<double> gv, const Tab<double, P> *__restrict__ tbp, const double *__restrict__ st,
        const double *__restrict__ beta, double *__restrict__ buf) {
  const Tab<double, P> &tb = *tbp;
  constexpr int NT = Launch<P>::NT, E = Launch<P>::E, P2 = P * P, P3 = P2 * P;
  const int lb = logical_block();
  const int tid = threadIdx.x, el = tid / P2, t = tid % P2;
  const int64_t e = tile_elem<E>(m, lb, el);
  const int els = el < E ? el : E - 1;
  const int i = t % P, j = t / P;
  int lo = 0, hi = -1;
  const bool act = e >= 0 && zline_run<P>(m.cmask[e], i, j, lo, hi);   // this thread's z-line has a run
  double rows[3][P][P];                     // rows[c][za][d] = F_e[za, za + d]
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
      for (int d = 0; d < P; ++d) rows[c][a][d] = 0;
  double jx = 0, jy = 0, jz = 0;
  if (e >= 0) {
    if (GEO == GEO_AFFINE) {
      jx = gv.el[4 * e]; jy = gv.el[4 * e + 1]; jz = gv.el[4 * e + 2];
    } else {
      jx = gv.el[2 * e]; jy = gv.el[2 * e + 1];
    }
  }
  // The element's points are visited one z-plane (qz) at a time, staged in LDS by the element's
  // threads (each the point (qx, qy) = (i, j) of the plane), in the order of a plain loop over
  // (qy + P qz, qx): one load latency per plane instead of one per point.
  constexpr int NV = NSTATE + NGEOQP;
  __shared__ double stg[E][NV * P2];
#pragma unroll 1
  for (int qz = 0; qz < P; ++qz) {
    __syncthreads();
    if (e >= 0) {
      const int tidq = el * P2 + j + P * qz;
#pragma unroll
      for (int f = 0; f < NSTATE; ++f) stg[els][f * P2 + t] = st[qp_at<P, NT, NSTATE>(lb, f, tidq, i)];
      if (GEO != GEO_AFFINE)
#pragma unroll
        for (int f = 0; f < NGEOQP; ++f) stg[els][(NSTATE + f) * P2 + t] = gv.qp[qp_at<P, NT, NGEOQP>(lb, f, tidq, i)];
    }
    __syncthreads();
    if (!act) continue;
#pragma unroll 1
    for (int qy = 0; qy < P; ++qy)
#pragma unroll 1
      for (int qx = 0; qx < P; ++qx) {
        const double *sp = &stg[els][qx + P * qy];
        const double mu = sp[0];
        const double ka = sp[P2];
        double S[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) S[f] = sp[(2 + f) * P2];
        double a = 0, b = 0, cc = jz;
        if (GEO != GEO_AFFINE) {
          a = sp[NSTATE * P2];
          b = sp[(NSTATE + 1) * P2];
          cc = sp[(NSTATE + 2) * P2];
        }
        double G[P][3], SG[P][3];
#pragma unroll
        for (int z = 0; z < P; ++z) {
          const double gr0 = tb.D[qx][i] * tb.B[qy][j] * tb.B[qz][z];
          const double gr1 = tb.B[qx][i] * tb.D[qy][j] * tb.B[qz][z];
          const double gr2 = tb.B[qx][i] * tb.B[qy][j] * tb.D[qz][z];
          if (GEO == GEO_AFFINE) {
            G[z][0] = gr0 * jx; G[z][1] = gr1 * jy; G[z][2] = gr2 * jz;
          } else {
            G[z][0] = gr0 * jx + gr2 * a; G[z][1] = gr1 * jy + gr2 * b; G[z][2] = gr2 * cc;
          }
          SG[z][0] = S[0] * G[z][0] + S[3] * G[z][1] + S[4] * G[z][2];
          SG[z][1] = S[3] * G[z][0] + S[1] * G[z][1] + S[5] * G[z][2];
          SG[z][2] = S[4] * G[z][0] + S[5] * G[z][1] + S[2] * G[z][2];
        }
#pragma unroll
        for (int za = 0; za < P; ++za)
#pragma unroll
          for (int d = 0; d < P; ++d) {
            if (za + d >= P) continue;
            const int zb = za + d;
            const double g = G[za][0] * G[zb][0] + G[za][1] * G[zb][1] + G[za][2] * G[zb][2];
#pragma unroll
            for (int c = 0; c < 3; ++c) rows[c][za][d] += 0.5 * mu * (g + G[za][c] * G[zb][c]) - ka * SG[za][c] * SG[zb][c];
          }
      }
  }
  if (!act) return;                         // no barriers below
  const int fid = m.bface_of[e];
  if (fid >= 0) {
    const double *fg = gv.face + (size_t)fid * NFACEGEO * P2;
    for (int fq = 0; fq < P2; ++fq) {
      const double phi = tb.B[fq % P][i] * tb.B[fq / P][j];
      const double bw = beta[fid] * fg[fq] * phi * phi;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double nc = fg[(1 + c) * P2 + fq];
        rows[c][0][0] += bw * (1.0 - nc * nc);
      }
    }
  }
  // bottom slot in a local frame Q (basal node, u . n = 0): its rows couple the local component c
  // with component c of the slots above, F[(c, 0), (c, zb)] = sum_c' Q[c'][c] A[(c', 0), (c, zb)],
  // and its diagonal is q_c^T A[(., 0), (., 0)] q_c, from the cross-component entries
  // A[(c', 0), (c, zb)] = sum over points of mu'/2 (delta_c'c grad phi_0 . grad phi_zb +
  // d_c phi_0 d_c' phi_zb) - kappa (Sigma0 grad phi_0)_c' (Sigma0 grad phi_zb)_c (+ basal term)
  if (FR && lo == 0 && (m.en[e * P3 + t] & ROT_BIT)) {
    double M[3][3][P];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int z = 0; z < P; ++z) M[a][c][z] = 0;
    for (int tq = 0; tq < P2; ++tq) {
      const int qy = tq % P, qz = tq / P, tidq = el * P2 + tq;
      for (int qx = 0; qx < P; ++qx) {
        const double mu = st[qp_at<P, NT, NSTATE>(lb, 0, tidq, qx)];
        const double ka = st[qp_at<P, NT, NSTATE>(lb, 1, tidq, qx)];
        double S[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) S[f] = st[qp_at<P, NT, NSTATE>(lb, 2 + f, tidq, qx)];
        double a = 0, b = 0, cc = jz;
        if (GEO != GEO_AFFINE) {
          a = gv.qp[qp_at<P, NT, NGEOQP>(lb, 0, tidq, qx)];
          b = gv.qp[qp_at<P, NT, NGEOQP>(lb, 1, tidq, qx)];
          cc = gv.qp[qp_at<P, NT, NGEOQP>(lb, 2, tidq, qx)];
        }
        double G[P][3], SG[P][3];
#pragma unroll
        for (int z = 0; z < P; ++z) {
          const double gr0 = tb.D[qx][i] * tb.B[qy][j] * tb.B[qz][z];
          const double gr1 = tb.B[qx][i] * tb.D[qy][j] * tb.B[qz][z];
          const double gr2 = tb.B[qx][i] * tb.B[qy][j] * tb.D[qz][z];
          if (GEO == GEO_AFFINE) {
            G[z][0] = gr0 * jx; G[z][1] = gr1 * jy; G[z][2] = gr2 * jz;
          } else {
            G[z][0] = gr0 * jx + gr2 * a; G[z][1] = gr1 * jy + gr2 * b; G[z][2] = gr2 * cc;
          }
          SG[z][0] = S[0] * G[z][0] + S[3] * G[z][1] + S[4] * G[z][2];
          SG[z][1] = S[3] * G[z][0] + S[1] * G[z][1] + S[5] * G[z][2];
          SG[z][2] = S[4] * G[z][0] + S[5] * G[z][1] + S[2] * G[z][2];
        }
#pragma unroll
        for (int zb = 0; zb < P; ++zb) {
          const double g = G[0][0] * G[zb][0] + G[0][1] * G[zb][1] + G[0][2] * G[zb][2];
#pragma unroll
          for (int ap = 0; ap < 3; ++ap)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              M[ap][c][zb] += 0.5 * mu * ((ap == c ? g : 0.0) + G[0][c] * G[zb][ap]) - ka * SG[0][ap] * SG[zb][c];
        }
      }
    }
    if (fid >= 0) {
      const double *fg = gv.face + (size_t)fid * NFACEGEO * P2;
      for (int fq = 0; fq < P2; ++fq) {
        const double phi = tb.B[fq % P][i] * tb.B[fq / P][j];
        const double bw = beta[fid] * fg[fq] * phi * phi;
        const double nv[3] = {fg[P2 + fq], fg[2 * P2 + fq], fg[3 * P2 + fq]};
#pragma unroll
        for (int ap = 0; ap < 3; ++ap)
#pragma unroll
          for (int c = 0; c < 3; ++c) M[ap][c][0] += bw * ((ap == c ? 1.0 : 0.0) - nv[ap] * nv[c]);
      }
    }
    double Q[9];
    frame_load<double, P>(gv.rot, m.rot_of[e], t, Q);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double dg = 0;
#pragma unroll
      for (int ap = 0; ap < 3; ++ap)
#pragma unroll
        for (int bp = 0; bp < 3; ++bp) dg += Q[3 * ap + c] * Q[3 * bp + c] * M[ap][bp][0];
      rows[c][0][0] = dg;
#pragma unroll
      for (int d = 1; d < P; ++d) {
        double s = 0;
#pragma unroll
        for (int ap = 0; ap < 3; ++ap) s += Q[3 * ap + c] * M[ap][c][d];
        rows[c][0][d] = s;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int zb = 0; zb < P; ++zb)
#pragma unroll
      for (int d = 0; d < P; ++d)
        if (zb >= lo && zb <= hi)
          buf[((size_t)c * m.n_inc + e * P3 + t + P2 * zb) * P + d] = zb - d >= lo ? rows[c][zb - d][d] : 0.0;
}

// Node rows of the line blocks: A[(c NR + prow[n]) W + d] = sum of the rows of the node's conforming
// slots (fixed order, deterministic); entry d couples n with the node d places below it on its line.
// Rows are interleaved by groups of LINE_GROUP lines: node i of line l of group g sits at row
// base[g] + LINE_GROUP i + (l mod LINE_GROUP), so that the threads of one wavefront, which handle
// consecutive lines, read consecutive rows at each step of the factorisation and the solves.
// The node's first MS slot indices are read once (clamped into the node's list; lslot carries one
// sentinel entry past the end, so an empty list reads in bounds), then each component's entries of
// all of them are requested together and summed in slot order; slots past MS (none in a 2:1
// balanced hexahedral mesh) take a plain loop.  Reading slot index and entry per slot in a loop
// waited on two dependent loads per entry (10 ms on the Q4 terrain).
template <int W>
__global__ void k_line_band(int64_t N, int64_t n_inc, int64_t NR, const int32_t *__restrict__ lptr,
                            const int32_t *__restrict__ lslot, const int32_t *__restrict__ prow,
                            const double *__restrict__ buf, double *__restrict__ A) {
  constexpr int MS = 8, MW = W;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int32_t k0 = lptr[n], k1 = lptr[n + 1], cnt = k1 - k0;
  const int64_t q = prow[n];
  int32_t sl[MS];
#pragma unroll
  for (int u = 0; u < MS; ++u) sl[u] = lslot[k0 + (u < cnt ? u : 0)];
  for (int c = 0; c < 3; ++c) {
    double v[MS][MW];
#pragma unroll
    for (int u = 0; u < MS; ++u)
#pragma unroll
      for (int d = 0; d < MW; ++d) v[u][d] = buf[((size_t)c * n_inc + sl[u]) * W + d];
    double s[MW];
#pragma unroll
    for (int d = 0; d < MW; ++d) s[d] = 0.0;
#pragma unroll
    for (int u = 0; u < MS; ++u)
      if (u < cnt)
#pragma unroll
        for (int d = 0; d < MW; ++d) s[d] += v[u][d];
    for (int32_t k = k0 + MS; k < k1; ++k)
      for (int d = 0; d < W; ++d) s[d] += buf[((size_t)c * n_inc + lslot[k]) * W + d];
#pragma unroll
    for (int d = 0; d < MW; ++d) A[((size_t)c * NR + q) * W + d] = s[d];
  }
}

// Banded Cholesky of each line block, one thread per (line, component), in place (interleaved rows,
// see k_line_band): row i of the line holds A[i][i - d] on entry and the factor entry G[i][i - d] on
// exit (A = G G^T), except entry 0, which holds 1 / G[i][i] so that the solves multiply.  Rows of
// Dirichlet-flagged components are unit rows, and couplings with them are dropped (the blocks of
// J_c = P K P + (I - P)).  A non-positive pivot (not expected: the blocks are principal
// submatrices of an SPD matrix) falls back to a diagonal row.
template <int W>
__global__ void k_line_factor(int64_t N, int64_t n_lines, int64_t NR, const int32_t *__restrict__ line_ptr,
                              const int32_t *__restrict__ line_node, const int32_t *__restrict__ lrow,
                              const uint8_t *__restrict__ dm, double *__restrict__ F, float *__restrict__ F32) {
  constexpr int K = W - 1;
  const int64_t L = line_threads(n_lines);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 3 * L) return;
  const int c = (int)(g / L);
  const int64_t l = g % L;
  if (l >= n_lines) return;
  const int32_t b0 = line_ptr[l], len = line_ptr[l + 1] - b0;
  const size_t r0 = (size_t)c * NR + lrow[l];
  double prev[K + 1][W];   // prev[r] = factor row of line row i - r (r = 1..K)
  bool pmask[K + 1];
#pragma unroll
  for (int r = 0; r <= K; ++r) {
    pmask[r] = true;
#pragma unroll
    for (int d = 0; d < W; ++d) prev[r][d] = 0.0;
  }
  for (int32_t i = 0; i < len; ++i) {
    const int32_t n = line_node[b0 + i];
    const bool mi = dm[(size_t)c * N + n] != 0;
    double *row = F + (r0 + (size_t)LINE_GROUP * i) * W;
    double a[W], gi[W];
#pragma unroll
    for (int d = 0; d < W; ++d) {
      const bool keep = d == 0 ? !mi : (!mi && i - d >= 0 && !pmask[d]);
      a[d] = keep ? row[d] : (d == 0 ? 1.0 : 0.0);
      gi[d] = 0.0;
    }
    // G[i][i-d] for d = K..1, then the pivot
#pragma unroll
    for (int d = K; d >= 1; --d) {
      if (i - d < 0) continue;
      double s = a[d];
#pragma unroll
      for (int t2 = 1; t2 + d <= K; ++t2) s -= gi[d + t2] * prev[d][t2];
      gi[d] = s / prev[d][0];
    }
    double s = a[0];
#pragma unroll
    for (int d = 1; d < W; ++d) s -= gi[d] * gi[d];
    if (!(s > 0.0)) {
#pragma unroll
      for (int d = 1; d < W; ++d) gi[d] = 0.0;
      s = a[0] != 0.0 ? (a[0] > 0 ? a[0] : -a[0]) : 1.0;
    }
    gi[0] = sqrt(s);
#pragma unroll
    for (int d = 0; d < W; ++d) {
      const double gv = d == 0 ? 1.0 / gi[0] : gi[d];
      row[d] = gv;
      F32[(r0 + (size_t)LINE_GROUP * i) * W + d] = (float)gv;
    }
#pragma unroll
    for (int r = K; r >= 2; --r) {
      pmask[r] = pmask[r - 1];
#pragma unroll
      for (int d = 0; d < W; ++d) prev[r][d] = prev[r - 1][d];
    }
    pmask[1] = mi;
#pragma unroll
    for (int d = 0; d < W; ++d) prev[1][d] = gi[d];
  }
}

// y = (line blocks)^{-1} x per component: forward G v = x, backward G^T y = v along each line.  One
// block (one wavefront) per group of LINE_GROUP lines and component, one thread per line.  The factor
// rows are interleaved by group (k_line_band), so the wavefront reads consecutive rows at each step.
// x and y are in node order, where the nodes of one line are far apart across the lanes; they pass
// through LDS in chunks of LINE_CH nodes of every line of the group: lane q moves element q mod LINE_CH
// of line q / LINE_CH (+ 4 r lines in round r), so each access is a run of LINE_CH consecutive
// entries of one line (lines with consecutive node ids, first[l] >= 0; others gather through
// line_node).  The backward sweep takes its chunks from each line's end.  Factor rows are loaded LB
// nodes ahead of the recurrence.
constexpr int LINE_CH = 16;
template <typename T, int W>
__global__ void __launch_bounds__(LINE_GROUP)
k_line_apply(int64_t N, int64_t n_lines, int64_t NR, const int32_t *__restrict__ line_ptr,
             const int32_t *__restrict__ line_node, const int32_t *__restrict__ lrow,
             const int32_t *__restrict__ first, const T *__restrict__ F, const T *__restrict__ x,
             T *__restrict__ y) {
  // LB: factor rows requested ahead of the recurrence (16 in FP32: 5% faster on the Q4 terrain; FP64
  // keeps 8 for its registers); LPR: lines per round
  constexpr int K = W - 1, LB = sizeof(T) == 4 ? 16 : 8, CH = LINE_CH, LPR = LINE_GROUP / CH;
  static_assert(LINE_GROUP % CH == 0 && CH % LB == 0, "chunk shape");
  __shared__ T buf[LINE_GROUP][CH + 1];
  __shared__ int32_t mlen[LINE_GROUP], mfirst[LINE_GROUP], mb0[LINE_GROUP];
  const int64_t G = line_threads(n_lines) / LINE_GROUP;
  const int c = (int)(blockIdx.x / G);
  const int lane = (int)threadIdx.x;
  const int64_t l = (blockIdx.x % G) * LINE_GROUP + lane;
  int32_t b0 = 0, len = 0, f0 = 0;   // lanes past the last line: an empty line at node 0
  int64_t r0 = 0;
  if (l < n_lines) {
    b0 = line_ptr[l];
    len = line_ptr[l + 1] - b0;
    f0 = first[l];
    r0 = lrow[l];
  }
  mlen[lane] = len;
  mfirst[lane] = f0;
  mb0[lane] = b0;
  int32_t lmax = len;   // longest line of the group: the chunk loops are uniform over the wavefront
#pragma unroll
  for (int off = LINE_GROUP / 2; off > 0; off >>= 1) lmax = max(lmax, __shfl_xor(lmax, off));
  __syncthreads();
  const T *Fl = F + ((size_t)c * NR + r0) * W;
  const size_t cN = (size_t)c * N;
  const int je = lane / CH, ee = lane % CH;   // this lane's (line, element) in round 0
  // node of entry i of group line j.  Without branches on the lane's line: a lane of a line with
  // consecutive node ids reads line_node[0] and discards it (a branch would make the other lanes'
  // register writes wait for the outstanding load); no read at all when every line of the group
  // has consecutive ids (a wavefront-uniform test).
  const bool all_seq = __all(f0 >= 0);
  // nd[r] = node of entry ent(j) of line j = r LPR + je, for the CH lines of the lane's chunk slot
  auto chunk_nodes = [&](auto ent, int32_t (&nd)[CH]) {
    if (all_seq) {
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        const int j = r * LPR + je;
        nd[r] = mfirst[j] + ent(j);
      }
    } else {
      int32_t ln[CH];
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        const int j = r * LPR + je;
        ln[r] = line_node[mfirst[j] >= 0 ? 0 : mb0[j] + ent(j)];
      }
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        const int j = r * LPR + je;
        nd[r] = mfirst[j] >= 0 ? mfirst[j] + ent(j) : ln[r];
      }
    }
  };
  // forward: v_i = (x_i - sum_d G[i][i-d] v_{i-d}) / G[i][i]
  T v[K + 1];
#pragma unroll
  for (int r = 0; r <= K; ++r) v[r] = 0;
  for (int32_t i0 = 0; i0 < lmax; i0 += CH) {
    // the chunk's nodes first, then all its loads, then the LDS writes: no load waits alone.
    // Entries past a line's end take the line's first node (in bounds); their slots are not read.
    int32_t nd[CH];
    chunk_nodes([&](int j) { const int32_t i = i0 + ee; return i < mlen[j] ? i : 0; }, nd);
    T xv[CH];
#pragma unroll
    for (int r = 0; r < CH; ++r) xv[r] = x[cN + nd[r]];
#pragma unroll
    for (int r = 0; r < CH; ++r) buf[r * LPR + je][ee] = xv[r];
    __syncthreads();
    for (int e0 = 0; e0 < CH; e0 += LB) {
      T rw[LB][W];
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int32_t i = i0 + e0 + u;
        const bool in = i < len;
#pragma unroll
        for (int d = 0; d < W; ++d) rw[u][d] = in ? Fl[(size_t)LINE_GROUP * i * W + d] : T(0);
      }
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int32_t i = i0 + e0 + u;
        if (i >= len) break;
        T s = buf[lane][e0 + u];
#pragma unroll
        for (int d = 1; d < W; ++d)
          if (i - d >= 0) s -= rw[u][d] * v[d];
        s *= rw[u][0];
        buf[lane][e0 + u] = s;
#pragma unroll
        for (int r = K; r >= 2; --r) v[r] = v[r - 1];
        v[1] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      const int j = r * LPR + je;
      if (i0 + ee < mlen[j]) y[cN + nd[r]] = buf[j][ee];
    }
    __syncthreads();
  }
  // backward: z_i = (v_i - sum_d G[i+d][i] z_{i+d}) / G[i][i]; gr[r] holds the row of node i + r.
  // Chunk k holds entries i = len - 1 - (k0 + e) of each line.
  T zr[K + 1], gr[K + 1][W];
#pragma unroll
  for (int r = 0; r <= K; ++r) {
    zr[r] = 0;
#pragma unroll
    for (int d = 0; d < W; ++d) gr[r][d] = 0;
  }
  for (int32_t k0 = 0; k0 < lmax; k0 += CH) {
    int32_t nd[CH];
    chunk_nodes([&](int j) { const int32_t lj = mlen[j], ri = k0 + ee; return ri < lj ? lj - 1 - ri : 0; }, nd);
    T yv[CH];
#pragma unroll
    for (int r = 0; r < CH; ++r) yv[r] = y[cN + nd[r]];
#pragma unroll
    for (int r = 0; r < CH; ++r) buf[r * LPR + je][ee] = yv[r];
    __syncthreads();
    for (int e0 = 0; e0 < CH; e0 += LB) {
      T rw[LB][W];
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int32_t i = len - 1 - (k0 + e0 + u);
        const bool in = i >= 0;
#pragma unroll
        for (int d = 0; d < W; ++d) rw[u][d] = in ? Fl[(size_t)LINE_GROUP * i * W + d] : T(0);
      }
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int32_t i = len - 1 - (k0 + e0 + u);
        if (i < 0) break;
        T s = buf[lane][e0 + u];
#pragma unroll
        for (int d = 1; d < W; ++d)
          if (i + d < len) s -= gr[d][d] * zr[d];
        const T z = s * rw[u][0];
        buf[lane][e0 + u] = z;
#pragma unroll
        for (int r = K; r >= 2; --r) {
          zr[r] = zr[r - 1];
#pragma unroll
          for (int d = 0; d < W; ++d) gr[r][d] = gr[r - 1][d];
        }
        zr[1] = z;
#pragma unroll
        for (int d = 0; d < W; ++d) gr[1][d] = rw[u][d];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      const int j = r * LPR + je;
      if (k0 + ee < mlen[j]) y[cN + nd[r]] = buf[j][ee];
    }
    __syncthreads();
  }
}

// Geometry at upload (FP64).  mode 0: classify (flags bit0 not column-mapped, bit1 not
// affine, bit2 det J <= 0 or not finite, bit3 degenerate basal face).  mode 1: store
// affine data.  mode 2: store column data.  Face data are stored in modes 1 and 2.
template <int P>
__global__ void __launch_bounds__(Launch<P>::NT)
k_geometry(MeshView m, const Tab<double, P> *__restrict__ tbp, const double *__restrict__ X, double px, double py,
           int mode, double *__restrict__ el_out, double *__restrict__ qp_out, double *__restrict__ face_out,
           unsigned *__restrict__ flags) {
  using T = double;
  const Tab<T, P> &tb = *tbp;
  constexpr int NT = Launch<P>::NT, E = Launch<P>::E, P2 = P * P, P3 = P2 * P;
  __shared__ T smem[E * Ws<T, P>::ES];
  __shared__ T ref0[E][3];
  __shared__ T xmag[E];
  const int lb = logical_block();
  const int tid = threadIdx.x, el = tid / P2, t = tid % P2;
  const int64_t e = tile_elem<E>(m, lb, el);
  const bool act = e >= 0;
  const int els = el < E ? el : E - 1;
  Ws<T, P> w{smem + els * Ws<T, P>::ES};
  const int64_t N = m.n_nodes;
  const uint32_t cm = act ? m.cmask[e] : 0u;
  T v[3][P];
  uint32_t nw[P];
  gather<T, P>(m.en + e * P3, X, N, t, act, false, v, nw);
  // work with coordinates relative to the first gathered node: derivatives are unchanged,
  // and neither the hanging interpolation nor the differentiation sees large absolute
  // coordinates (whose rounding would otherwise dominate the Jacobian of distant elements)
  if (act && t == 0) {
    xmag[els] = fabs(v[0][0]) + fabs(v[1][0]) + fabs(v[2][0]);
    for (int c = 0; c < 3; ++c) ref0[els][c] = v[c][0];
  }
  __syncthreads();
  // periodic axes: the periodic image of each slot nearest to the first slot
  if (act)
    for (int c = 0; c < 3; ++c)
      for (int z = 0; z < P; ++z) {
        T d = v[c][z] - ref0[els][c];
        const T per = c == 0 ? px : (c == 1 ? py : 0.0);
        if (per > 0.0) d -= per * rint(d / per);
        v[c][z] = d;
      }
  __syncthreads();
  if (m.any_hang && __syncthreads_or(act && (cm >> 3) != 0u)) hang_fwd<T, P>(v, cm, w, tb, t, act);
  const T xb[3] = {v[0][0], v[1][0], v[2][0]};
  T J[3][3][P];   // J[i][r] = d x_i / d xi_r
#pragma unroll
  for (int c = 0; c < 3; ++c) grad_fwd<T, P>(v[c], J[c][0], J[c][1], J[c][2], w, tb, t, act);
  if (act && t == 0) {
    ref0[els][0] = J[0][0][0];
    ref0[els][1] = J[1][1][0];
    ref0[els][2] = J[2][2][0];
  }
  __syncthreads();
  unsigned fl = 0;
  if (act) {
    const T r00 = ref0[els][0], r11 = ref0[els][1], r22 = ref0[els][2];
    const int j = t % P, z = t / P;
    for (int i = 0; i < P; ++i) {
      T a[3][3];
      for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) a[c][r] = J[c][r][i];
      const T det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                    a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                    a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
      // the input coordinates carry rounding relative to their absolute size (xmag), which
      // the derivatives see amplified by the 1D derivative weights
      const T sc = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]);
      const T tol = 1e-13 * sc + 1e-14 * xmag[els];
      if (!(det > 0) || !isfinite(det)) fl |= 4u;
      if (fabs(a[0][1]) > tol || fabs(a[0][2]) > tol || fabs(a[1][0]) > tol || fabs(a[1][2]) > tol ||
          fabs(a[0][0] - r00) > tol || fabs(a[1][1] - r11) > tol)
        fl |= 1u;
      if (fabs(a[2][0]) > tol || fabs(a[2][1]) > tol || fabs(a[2][2] - r22) > tol) fl |= 2u;
      if (mode == 2) {
        const T j00 = a[0][0], j11 = a[1][1], j22 = a[2][2];
        qp_out[qp_at<P, NT, NGEOQP>(lb, 0, tid, i)] = -a[2][0] / (j00 * j22);
        qp_out[qp_at<P, NT, NGEOQP>(lb, 1, tid, i)] = -a[2][1] / (j11 * j22);
        qp_out[qp_at<P, NT, NGEOQP>(lb, 2, tid, i)] = 1.0 / j22;
      }
    }
    if (t == 0 && mode == 1) {
      el_out[4 * e + 0] = 1.0 / r00;
      el_out[4 * e + 1] = 1.0 / r11;
      el_out[4 * e + 2] = 1.0 / r22;
      el_out[4 * e + 3] = r00 * r11 * r22;
    }
    if (t == 0 && mode == 2) {
      el_out[2 * e + 0] = 1.0 / r00;
      el_out[2 * e + 1] = 1.0 / r11;
    }
  }
  const int fid = act ? m.bface_of[e] : -1;
  if (__syncthreads_or(fid >= 0)) {
    // tangents at face Gauss points: x_xi = (D x B) X, x_eta = (B x D) X over the bottom nodes
    const int i = t % P, j = t / P;
    if (act)
      for (int c = 0; c < 3; ++c) w.b(0)[c * P2 + t] = xb[c];
    __syncthreads();
    if (act)
      for (int c = 0; c < 3; ++c) {
        T sd = 0, sb = 0;
        for (int a = 0; a < P; ++a) {
          sd += tb.D[i][a] * w.b(0)[c * P2 + a + P * j];
          sb += tb.B[i][a] * w.b(0)[c * P2 + a + P * j];
        }
        w.b(1)[c * P2 + t] = sd;
        w.b(2)[c * P2 + t] = sb;
      }
    __syncthreads();
    if (fid >= 0) {
      T xa[3], xe[3];
      for (int c = 0; c < 3; ++c) {
        T s1 = 0, s2 = 0;
        for (int b = 0; b < P; ++b) {
          s1 += tb.B[j][b] * w.b(1)[c * P2 + i + P * b];
          s2 += tb.D[j][b] * w.b(2)[c * P2 + i + P * b];
        }
        xa[c] = s1;
        xe[c] = s2;
      }
      const T cr[3] = {xa[1] * xe[2] - xa[2] * xe[1], xa[2] * xe[0] - xa[0] * xe[2], xa[0] * xe[1] - xa[1] * xe[0]};
      const T area = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      if (!(area > 0) || !isfinite(area)) fl |= 8u;
      if (mode > 0) {
        T *fo = face_out + (size_t)fid * NFACEGEO * P2;
        fo[t] = tb.w[i] * tb.w[j] * area;
        fo[P2 + t] = cr[0] / area;
        fo[2 * P2 + t] = cr[1] / area;
        fo[3 * P2 + t] = cr[2] / area;
      }
    }
  }
  if (mode == 0 && fl) atomicOr(flags, fl);
}

// ---------------------------------------------------------------- low-order F~ on the Gauss-Lobatto sub-grid
// Sec. 5, "Construction of low-order approximation F~": the element's (k+1)^3 nodes are the corners of
// k^3 trilinear sub-cells, and F~_e is the matrix of the bilinear form of F (eq. (rank4), plus the basal
// term of eq. (robin)) on that grid, with the 2-point Gauss-Lobatto rule per sub-cell direction (F~_GL):
// its quadrature points are the sub-cell corners, i.e. the element's nodes, with weight |det J| / 8.
// The coefficients (mu, kappa' = mu (n-1)/(2n)/(II+eps), D0) are taken at each node from the high-order
// state differentiated inside the element.  Globally F~ = sum_e R_e^T F~_e R_e with the high-order
// restriction (figure "interp" (a) at nonconforming faces).

// Reference derivatives of a z-line field at the element's nodes: gz in registers, gx and gy through
// LDS (buffers 0..2).  All threads of the block must call.
template <int P>
__device__ void node_grad(const double (&v)[P], double (&gx)[P], double (&gy)[P], double (&gz)[P], Ws<double, P> w,
                          const Tab<double, P> &tb, int t, bool act) {
  if (act) {
#pragma unroll
    for (int z = 0; z < P; ++z) {
      double a = 0;
#pragma unroll
      for (int m = 0; m < P; ++m) a += tb.G[z][m] * v[m];
      gz[z] = a;
      w.b(0)[w.zl(t, z)] = v[z];
    }
  }
  __syncthreads();
  if (act) {
    const int j = t % P, z = t / P;   // x-line (., j, z) and y-line (j, ., z)
    double lx[P], ly[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      lx[m] = w.b(0)[m + P * j + w.SZ * z];
      ly[m] = w.b(0)[j + P * m + w.SZ * z];
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      double a = 0, b = 0;
#pragma unroll
      for (int m = 0; m < P; ++m) {
        a += tb.G[i][m] * lx[m];
        b += tb.G[i][m] * ly[m];
      }
      w.b(1)[i + P * j + w.SZ * z] = a;
      w.b(2)[j + P * i + w.SZ * z] = b;
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int z = 0; z < P; ++z) {
      gx[z] = w.b(1)[w.zl(t, z)];
      gy[z] = w.b(2)[w.zl(t, z)];
    }
  }
  __syncthreads();
}

// Nodal data of F~ at the state: per element node its coordinates relative to the element's first slot
// (periodic images nearest to it, through R_e) and mu, kappa', D0 from grad u_h at the node.
template <int P>
__global__ void __launch_bounds__(Launch<P>::NT)
k_lowo_coef(MeshView m, GeoView<double> gv, const Tab<double, P> *__restrict__ tbp, const double *__restrict__ X,
            double px, double py, const double *__restrict__ u, const double *__restrict__ logA, double n, double eps,
            double B0, int picard, double *__restrict__ lo) {
  using T = double;
  const Tab<T, P> &tb = *tbp;
  constexpr int NT = Launch<P>::NT, E = Launch<P>::E, P2 = P * P, P3 = P2 * P;
  __shared__ T smem[E * Ws<T, P>::ES];
  __shared__ T ref0[E][3];
  const int lb = logical_block();
  const int tid = threadIdx.x, el = tid / P2, t = tid % P2;
  const int64_t e = tile_elem<E>(m, lb, el);
  const bool act = e >= 0;
  const int els = el < E ? el : E - 1;
  Ws<T, P> w{smem + els * Ws<T, P>::ES};
  const int64_t N = m.n_nodes;
  const uint32_t cm = act ? m.cmask[e] : 0u;
  T xv[3][P];
  uint32_t nw[P];
  gather<T, P>(m.en + e * P3, X, N, t, act, false, xv, nw);
  if (act && t == 0)
    for (int c = 0; c < 3; ++c) ref0[els][c] = xv[c][0];
  __syncthreads();
  if (act)
    for (int c = 0; c < 3; ++c)
      for (int z = 0; z < P; ++z) {
        T d = xv[c][z] - ref0[els][c];
        const T per = c == 0 ? px : (c == 1 ? py : 0.0);
        if (per > 0.0) d -= per * rint(d / per);
        xv[c][z] = d;
      }
  const bool hang = m.any_hang && __syncthreads_or(act && (cm >> 3) != 0u);
  if (hang) hang_fwd<T, P>(xv, cm, w, tb, t, act);
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int z = 0; z < P; ++z) lo[qp_at<P, NT, NLOWO>(lb, c, tid, z)] = xv[c][z];
  // inverse Jacobian of the high-order map at the nodes: Ji[r][i] = d xi_r / d x_i
  T Ji[3][3][P];
  {
    T J[3][3][P];   // J[i][r] = d x_i / d xi_r
#pragma unroll
    for (int c = 0; c < 3; ++c) node_grad<P>(xv[c], J[c][0], J[c][1], J[c][2], w, tb, t, act);
#pragma unroll
    for (int z = 0; z < P; ++z) {
      const T a00 = J[0][0][z], a01 = J[0][1][z], a02 = J[0][2][z];
      const T a10 = J[1][0][z], a11 = J[1][1][z], a12 = J[1][2][z];
      const T a20 = J[2][0][z], a21 = J[2][1][z], a22 = J[2][2][z];
      const T c00 = a11 * a22 - a12 * a21, c01 = a02 * a21 - a01 * a22, c02 = a01 * a12 - a02 * a11;
      const T c10 = a12 * a20 - a10 * a22, c11 = a00 * a22 - a02 * a20, c12 = a02 * a10 - a00 * a12;
      const T c20 = a10 * a21 - a11 * a20, c21 = a01 * a20 - a00 * a21, c22 = a00 * a11 - a01 * a10;
      const T det = a00 * c00 + a01 * c10 + a02 * c20;
      const T id = act ? 1.0 / det : 0.0;
      Ji[0][0][z] = c00 * id; Ji[0][1][z] = c01 * id; Ji[0][2][z] = c02 * id;
      Ji[1][0][z] = c10 * id; Ji[1][1][z] = c11 * id; Ji[1][2][z] = c12 * id;
      Ji[2][0][z] = c20 * id; Ji[2][1][z] = c21 * id; Ji[2][2][z] = c22 * id;
    }
  }
  T uv[3][P];
  gather_words<T, P>(nw, u, N, act, true, uv);
  if (act && (nw[0] & ROT_BIT)) {
    T Q[9];
    frame_load<T, P>(gv.rot, m.rot_of[e], t, Q);
    frame_in<T, P>(uv, Q);
  }
  if (hang) hang_fwd<T, P>(uv, cm, w, tb, t, act);
  T G[3][3][P];   // G[c][i] = d u_c / d x_i at the nodes
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T gr[3][P];
    node_grad<P>(uv[c], gr[0], gr[1], gr[2], w, tb, t, act);
#pragma unroll
    for (int z = 0; z < P; ++z)
#pragma unroll
      for (int i = 0; i < 3; ++i) G[c][i][z] = gr[0][z] * Ji[0][i][z] + gr[1][z] * Ji[1][i][z] + gr[2][z] * Ji[2][i][z];
  }
  if (!act) return;
  const double Be = B0 * exp(-logA[e] / n);
  const double expo = (1.0 - n) / (2.0 * n), cf = picard ? 0.0 : (n - 1.0) / (2.0 * n);
#pragma unroll
  for (int z = 0; z < P; ++z) {
    const T dxx = G[0][0][z], dyy = G[1][1][z], dzz = G[2][2][z];
    const T dxy = 0.5 * (G[0][1][z] + G[1][0][z]), dxz = 0.5 * (G[0][2][z] + G[2][0][z]);
    const T dyz = 0.5 * (G[1][2][z] + G[2][1][z]);
    const T II = 0.5 * (dxx * dxx + dyy * dyy + dzz * dzz) + dxy * dxy + dxz * dxz + dyz * dyz;
    const T mu = Be * pow(II + eps, expo);
    const T vals[8] = {mu, cf * mu / (II + eps), dxx, dyy, dzz, dxy, dxz, dyz};
#pragma unroll
    for (int f = 0; f < 8; ++f) lo[qp_at<P, NT, NLOWO>(lb, 3 + f, tid, z)] = vals[f];
  }
}

// y_e = F~_e x_e for the element's z-lines (thread t = x + P y holds nodes (x, y, 0..P-1)), then R_e^T
// and the element-vector store.  Quadrature point (q, octant s): the sub-cell with corner q and edges
// towards q + s_x e_x, q + s_y e_y, q + s_z e_z; with the edge vectors as columns of J, g_r = J^-T e_r is
// the gradient of the basis function of the r-th edge neighbour, -(g_1 + g_2 + g_3) that of q, and
// f_r = |det J|/8 tau g_r is added to neighbour r and subtracted from q.  Contributions to the x- and
// y-neighbour z-lines pass through LDS (one writer per target entry, fixed summation order).
template <int P> struct LoShape {
  static constexpr int RS = 6 * P * P * P > Ws<double, P>::ES ? 6 * P * P * P : Ws<double, P>::ES;
};
template <int P>
__global__ void __launch_bounds__(Launch<P>::NT)
k_lowo(MeshView m, GeoView<double> gv, const Tab<double, P> *__restrict__ tbp, const double *__restrict__ lo,
       const double *__restrict__ beta, const double *__restrict__ x, double *__restrict__ ev) {
  using T = double;
  const Tab<T, P> &tb = *tbp;
  constexpr int NT = Launch<P>::NT, E = Launch<P>::E, P2 = P * P, P3 = P2 * P, RS = LoShape<P>::RS;
  __shared__ T smem[E * RS];
  const int lb = logical_block();
  const int tid = threadIdx.x, el = tid / P2, t = tid % P2;
  const int64_t e = tile_elem<E>(m, lb, el);
  const bool act = e >= 0;
  const int els = el < E ? el : E - 1;
  T *reg = smem + els * RS;            // element region: V[3][P3], X[3][P3]; later the contributions
  Ws<T, P> w{reg};
  const int64_t N = m.n_nodes;
  const uint32_t cm = act ? m.cmask[e] : 0u;
  const int xi = t % P, yi = t / P;
  T v[3][P];
  uint32_t nw[P];
  gather<T, P>(m.en + e * P3, x, N, t, act, true, v, nw);
  const bool rot = act && (nw[0] & ROT_BIT);
  if (rot) {
    T Q[9];
    frame_load<T, P>(gv.rot, m.rot_of[e], t, Q);
    frame_in<T, P>(v, Q);
  }
  const bool hang = m.any_hang && __syncthreads_or(act && (cm >> 3) != 0u);
  if (hang) hang_fwd<T, P>(v, cm, w, tb, t, act);
  __syncthreads();
  if (act)
#pragma unroll
    for (int z = 0; z < P; ++z)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        reg[c * P3 + t + P2 * z] = v[c][z];
        reg[(3 + c) * P3 + t + P2 * z] = lo[qp_at<P, NT, NLOWO>(lb, c, tid, z)];
      }
  __syncthreads();
  T acc[3][P], cxp[3][P], cxm[3][P], cyp[3][P], cym[3][P];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int z = 0; z < P; ++z) acc[c][z] = cxp[c][z] = cxm[c][z] = cyp[c][z] = cym[c][z] = 0;
  if (act) {
#pragma unroll
    for (int z = 0; z < P; ++z) {
      const int q = t + P2 * z;
      T co[8];
#pragma unroll
      for (int f = 0; f < 8; ++f) co[f] = lo[qp_at<P, NT, NLOWO>(lb, 3 + f, tid, z)];
      const T mu = co[0], ka = co[1];
      const T s00 = co[2], s11 = co[3], s22 = co[4], s01 = co[5], s02 = co[6], s12 = co[7];
#pragma unroll
      for (int oct = 0; oct < 8; ++oct) {
        const int sx = (oct & 1) ? 1 : -1, sy = (oct & 2) ? 1 : -1, sz = (oct & 4) ? 1 : -1;
        if (xi + sx < 0 || xi + sx >= P || yi + sy < 0 || yi + sy >= P || z + sz < 0 || z + sz >= P) continue;
        const int nb[3] = {q + sx, q + P * sy, q + P2 * sz};
        T Jc[3][3], du[3][3];   // Jc[r][i]: edge r (column r of J), du[r][c]: value difference along edge r
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            Jc[r][i] = reg[(3 + i) * P3 + nb[r]] - reg[(3 + i) * P3 + q];
            du[r][i] = reg[i * P3 + nb[r]] - reg[i * P3 + q];
          }
        // J[i][r] = Jc[r][i]; g_r = J^-T e_r = row r of J^-1 = cofactor column / det
        const T a00 = Jc[0][0], a01 = Jc[1][0], a02 = Jc[2][0];
        const T a10 = Jc[0][1], a11 = Jc[1][1], a12 = Jc[2][1];
        const T a20 = Jc[0][2], a21 = Jc[1][2], a22 = Jc[2][2];
        const T c00 = a11 * a22 - a12 * a21, c01 = a02 * a21 - a01 * a22, c02 = a01 * a12 - a02 * a11;
        const T c10 = a12 * a20 - a10 * a22, c11 = a00 * a22 - a02 * a20, c12 = a02 * a10 - a00 * a12;
        const T c20 = a10 * a21 - a11 * a20, c21 = a01 * a20 - a00 * a21, c22 = a00 * a11 - a01 * a10;
        const T det = a00 * c00 + a01 * c10 + a02 * c20;
        const T id = 1.0 / det;
        const T g[3][3] = {{c00 * id, c01 * id, c02 * id}, {c10 * id, c11 * id, c12 * id}, {c20 * id, c21 * id, c22 * id}};
        // G[c][i] = sum_r du[r][c] g[r][i]
        T Gm[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int i = 0; i < 3; ++i) Gm[c][i] = du[0][c] * g[0][i] + du[1][c] * g[1][i] + du[2][c] * g[2][i];
        const T dxx = Gm[0][0], dyy = Gm[1][1], dzz = Gm[2][2];
        const T dxy = 0.5 * (Gm[0][1] + Gm[1][0]), dxz = 0.5 * (Gm[0][2] + Gm[2][0]), dyz = 0.5 * (Gm[1][2] + Gm[2][1]);
        const T sd = s00 * dxx + s11 * dyy + s22 * dzz + 2.0 * (s01 * dxy + s02 * dxz + s12 * dyz);
        const T wd = fabs(det) * 0.125;
        const T tau[3][3] = {{wd * (mu * dxx - ka * sd * s00), wd * (mu * dxy - ka * sd * s01), wd * (mu * dxz - ka * sd * s02)},
                             {wd * (mu * dxy - ka * sd * s01), wd * (mu * dyy - ka * sd * s11), wd * (mu * dyz - ka * sd * s12)},
                             {wd * (mu * dxz - ka * sd * s02), wd * (mu * dyz - ka * sd * s12), wd * (mu * dzz - ka * sd * s22)}};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T f0 = tau[c][0] * g[0][0] + tau[c][1] * g[0][1] + tau[c][2] * g[0][2];
          const T f1 = tau[c][0] * g[1][0] + tau[c][1] * g[1][1] + tau[c][2] * g[1][2];
          const T f2 = tau[c][0] * g[2][0] + tau[c][1] * g[2][1] + tau[c][2] * g[2][2];
          acc[c][z] -= f0 + f1 + f2;
          if (sz > 0) { if (z + 1 < P) acc[c][z + 1] += f2; }
          else { if (z >= 1) acc[c][z - 1] += f2; }
          if (sx > 0) cxp[c][z] += f0; else cxm[c][z] += f0;
          if (sy > 0) cyp[c][z] += f1; else cym[c][z] += f1;
        }
      }
    }
  }
  // basal Robin term, lumped on the sub-faces at the bottom node: 1/4 |t1 x t2| beta (I - n n^T) v
  const int fid = act ? m.bface_of[e] : -1;
  if (fid >= 0) {
    const T bt = beta[fid];
#pragma unroll
    for (int quad = 0; quad < 4; ++quad) {
      const int sx = (quad & 1) ? 1 : -1, sy = (quad & 2) ? 1 : -1;
      if (xi + sx < 0 || xi + sx >= P || yi + sy < 0 || yi + sy >= P) continue;
      T t1[3], t2[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        t1[i] = reg[(3 + i) * P3 + t + sx] - reg[(3 + i) * P3 + t];
        t2[i] = reg[(3 + i) * P3 + t + P * sy] - reg[(3 + i) * P3 + t];
      }
      const T cr[3] = {t1[1] * t2[2] - t1[2] * t2[1], t1[2] * t2[0] - t1[0] * t2[2], t1[0] * t2[1] - t1[1] * t2[0]};
      const T area = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      const T nv[3] = {cr[0] / area, cr[1] / area, cr[2] / area};
      const T nu = nv[0] * v[0][0] + nv[1] * v[1][0] + nv[2] * v[2][0];
      const T wb = 0.25 * area * bt;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c][0] += wb * (v[c][0] - nv[c] * nu);
    }
  }
  // x-neighbour contributions: XP[target] from the source at target - e_x, XM[target] from target + e_x
  __syncthreads();
  if (act)
#pragma unroll
    for (int z = 0; z < P; ++z)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (xi + 1 < P) reg[c * P3 + t + 1 + P2 * z] = cxp[c][z];
        if (xi >= 1) reg[(3 + c) * P3 + t - 1 + P2 * z] = cxm[c][z];
      }
  __syncthreads();
  if (act)
#pragma unroll
    for (int z = 0; z < P; ++z)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (xi >= 1) acc[c][z] += reg[c * P3 + t + P2 * z];
        if (xi + 1 < P) acc[c][z] += reg[(3 + c) * P3 + t + P2 * z];
      }
  __syncthreads();
  if (act)
#pragma unroll
    for (int z = 0; z < P; ++z)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (yi + 1 < P) reg[c * P3 + t + P + P2 * z] = cyp[c][z];
        if (yi >= 1) reg[(3 + c) * P3 + t - P + P2 * z] = cym[c][z];
      }
  __syncthreads();
  if (act)
#pragma unroll
    for (int z = 0; z < P; ++z)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (yi >= 1) acc[c][z] += reg[c * P3 + t + P2 * z];
        if (yi + 1 < P) acc[c][z] += reg[(3 + c) * P3 + t + P2 * z];
      }
  __syncthreads();
  if (hang) hang_bwd<T, P>(acc, cm, w, tb, t, act);
  if (rot) {
    T Q[9];
    frame_load<T, P>(gv.rot, m.rot_of[e], t, Q);
    frame_out<T, P>(acc, Q);
  }
  evec_store<T, P>(ev, m, lb, e, smem, els, t, act, acc);
}

// ---------------------------------------------------------------- assembly  y = sum_e R_e^T y_e
// One thread per node: sums the node's contiguous segment of the node-ordered element vector
// (fixed order, so the result is deterministic).  Rows of Dirichlet-flagged components take the
// value xm (x for the Jacobian, u for the residual), or mval without xm; other rows subtract f when
// given.  y is written with the non-temporal hint: a write-once stream whose dirty lines would
// otherwise be evicted from L2 during the next element kernel (FP32 apply on the Q4 terrain 0.7%
// faster).
constexpr int ASM_NT = 256;
constexpr int ASM_TILE = 4 * ASM_NT;

// FP32: the entries of the block's nodes form one contiguous range [ptr[n0], ptr[n0 + M NT]) of each
// component plane of ev: it is streamed through LDS in tiles with coalesced loads, and each
// thread sums its own nodes' segments (nodes n0 + t + NT j, j < M) from LDS in increasing slot
// order.  A block takes M = 2 node groups when the mesh averages at most two entries per node
// (one tile then covers the block's range, and the two dependent reads of ptr that start a
// block are amortised over twice the nodes); M = 1 otherwise.  Both precisions request each
// node's Dirichlet flags (and f) together with its segment pointers, so that only the element
// vector is waited for before the sums; FP32 clamps the node index instead of guarding the loads,
// since a guarded byte load compiles to a branch with an immediate wait (assembly 144 -> 117 us
// on the Q4 terrain).  FP64: see below.
template <typename T, int M>
__global__ void __launch_bounds__(ASM_NT)
k_assemble(int64_t N, const int32_t *__restrict__ ptr, const T *__restrict__ ev, int64_t n_ent,
           const uint8_t *__restrict__ dm, const T *__restrict__ xm, const T *__restrict__ f, T *__restrict__ y,
           T mval) {
  if constexpr (sizeof(T) == 8) {
    // FP64: the tile would take 24 KiB of LDS per block and cap the occupancy; each thread reads
    // its own segment instead, in predicated chunks of four entries (measured 3% faster there,
    // 2% slower in FP32)
    constexpr int CH = 4;
    const int64_t n = (int64_t)blockIdx.x * ASM_NT + threadIdx.x;
    if (n >= N) return;
    const int32_t k0 = ptr[n], k1 = ptr[n + 1];
    int dv[3];
    T fv[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dv[c] = dm[c * N + n];
      if (f) fv[c] = f[c * N + n];
    }
    T sv[3] = {0, 0, 0};
    for (int32_t k = k0; k < k1; k += CH) {
      T a[3][CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const bool in = k + u < k1;
#pragma unroll
        for (int c = 0; c < 3; ++c) a[c][u] = in ? ev[c * n_ent + k + u] : T(0);
      }
#pragma unroll
      for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int c = 0; c < 3; ++c) sv[c] += a[c][u];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = c * N + n;
      __builtin_nontemporal_store(dv[c] ? (xm ? xm[i] : mval) : sv[c] - fv[c], y + i);
    }
  } else {
    constexpr int NPB = ASM_NT * M;
    __shared__ T tile[3][ASM_TILE];
    const int64_t n0 = (int64_t)blockIdx.x * NPB;
    const int64_t nend = n0 + NPB < N ? n0 + NPB : N;
    const int32_t r0 = ptr[n0], r1 = ptr[nend];
    int32_t k0[M], k1[M];
    int dv[M][3];
    T sv[M][3], fv[M][3];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      // nodes past N sum node N - 1 again (in bounds) and store nothing
      const int64_t n = n0 + threadIdx.x + (int64_t)ASM_NT * j, nc = n < N ? n : N - 1;
      k0[j] = ptr[nc];
      k1[j] = ptr[nc + 1];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dv[j][c] = dm[c * N + nc];
        fv[j][c] = f ? f[c * N + nc] : T(0);
        sv[j][c] = 0;
      }
    }
    for (int32_t c0 = r0; c0 < r1; c0 += ASM_TILE) {
      const int32_t cn = r1 - c0 < ASM_TILE ? r1 - c0 : ASM_TILE;
      T a[3][ASM_TILE / ASM_NT];
#pragma unroll
      for (int u = 0; u < ASM_TILE / ASM_NT; ++u) {
        const int j = (int)threadIdx.x + u * ASM_NT;
        const bool in = j < cn;
        a[0][u] = in ? ev[c0 + j] : T(0);
        a[1][u] = in ? ev[n_ent + c0 + j] : T(0);
        a[2][u] = in ? ev[2 * n_ent + c0 + j] : T(0);
      }
#pragma unroll
      for (int u = 0; u < ASM_TILE / ASM_NT; ++u) {
        const int j = (int)threadIdx.x + u * ASM_NT;
        tile[0][j] = a[0][u];
        tile[1][j] = a[1][u];
        tile[2][j] = a[2][u];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const int32_t kb = k0[j] > c0 ? k0[j] : c0, ke = k1[j] < c0 + cn ? k1[j] : c0 + cn;
        for (int32_t k = kb; k < ke; ++k) {
          sv[j][0] += tile[0][k - c0];
          sv[j][1] += tile[1][k - c0];
          sv[j][2] += tile[2][k - c0];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t n = n0 + threadIdx.x + (int64_t)ASM_NT * j;
      if (n >= N) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t i = c * N + n;
        __builtin_nontemporal_store(dv[j][c] ? (xm ? xm[i] : mval) : sv[j][c] - fv[j][c], y + i);
      }
    }
  }
}

// ---------------------------------------------------------------- small kernels
__global__ void k_fill(uint32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}
__global__ void k_d2f(const double *in, float *out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

static inline int grid1(int64_t n, int nt) { return (int)((n + nt - 1) / nt); }

hipError_t launch_assemble(hipStream_t s, int prec, int64_t N, const int32_t *ptr, const void *ev, int64_t n_ent,
                           const uint8_t *dm, const void *xm, const void *f, void *y, double mval) {
  if (prec == 0)
    hipLaunchKernelGGL((k_assemble<double, 1>), dim3(grid1(N, ASM_NT)), dim3(ASM_NT), 0, s, N, ptr, (const double *)ev,
                       n_ent, dm, (const double *)xm, (const double *)f, (double *)y, mval);
  else if (n_ent <= 2 * N)
    hipLaunchKernelGGL((k_assemble<float, 2>), dim3(grid1(N, 2 * ASM_NT)), dim3(ASM_NT), 0, s, N, ptr, (const float *)ev,
                       n_ent, dm, (const float *)xm, (const float *)f, (float *)y, (float)mval);
  else
    hipLaunchKernelGGL((k_assemble<float, 1>), dim3(grid1(N, ASM_NT)), dim3(ASM_NT), 0, s, N, ptr, (const float *)ev,
                       n_ent, dm, (const float *)xm, (const float *)f, (float *)y, (float)mval);
  return hipGetLastError();
}

hipError_t launch_fill(hipStream_t s, void *ptr, int64_t n) {
  if (n <= 0) return hipSuccess;
  int nb = grid1(n, 256);
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, (uint32_t *)ptr, n);
  return hipGetLastError();
}
hipError_t launch_d2f(hipStream_t s, const double *in, float *out, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_d2f, dim3(grid1(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dispatch
template <int P>
static hipError_t geometry_p(int mode, hipStream_t s, const MeshView &m, const void *tabs, const double *X,
                             const double *per, double *el, double *qp, double *face, unsigned *flags) {
  hipLaunchKernelGGL((k_geometry<P>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, &((const TabSet<P> *)tabs)->d, X, per[0],
                     per[1], mode, el, qp, face, flags);
  return hipGetLastError();
}
hipError_t launch_geometry_impl(int P, int mode, hipStream_t s, const MeshView &m, const void *tabs,
                                const double *X, const double period[3], double *el, double *qp, double *face,
                                unsigned *flags) {
  switch (P) {
    case 3: return geometry_p<3>(mode, s, m, tabs, X, period, el, qp, face, flags);
    case 4: return geometry_p<4>(mode, s, m, tabs, X, period, el, qp, face, flags);
    case 5: return geometry_p<5>(mode, s, m, tabs, X, period, el, qp, face, flags);
  }
  return hipErrorInvalidValue;
}

template <int P, int GEO>
static hipError_t state_pg(hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                           const double *u, const double *logA, double n, double eps, double B0, bool picard,
                           double *st64, float *st32, double *fst64, float *fst32) {
  hipLaunchKernelGGL((k_state<P, GEO>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, g, &((const TabSet<P> *)tabs)->d, u, logA, n, eps, B0,
                     (int)picard, st64, st32, fst64, fst32);
  return hipGetLastError();
}
hipError_t launch_state(int P, int geo, hipStream_t s, const MeshView &m, const GeoView<double> &g,
                        const void *tabs, const double *u, const double *logA, double n, double eps, double B0,
                        bool picard, double *st64, float *st32, double *fst64, float *fst32) {
#define NSMF_ST(PP, GG) \
  if (P == PP && geo == GG) return state_pg<PP, GG>(s, m, g, tabs, u, logA, n, eps, B0, picard, st64, st32, fst64, fst32);
  NSMF_ST(3, GEO_AFFINE) NSMF_ST(3, GEO_COLUMN) NSMF_ST(4, GEO_AFFINE) NSMF_ST(4, GEO_COLUMN)
  NSMF_ST(5, GEO_AFFINE) NSMF_ST(5, GEO_COLUMN)
#undef NSMF_ST
  return hipErrorInvalidValue;
}

template <int P, int GEO, int PS>
static hipError_t residual_pg(hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                              const double *st, const double *fst, const double *beta, const double *p,
                              const double *body, double *ru, double *rp) {
  hipLaunchKernelGGL((k_residual<P, GEO, PS>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, g, &((const TabSet<P> *)tabs)->d, st, fst, beta, p,
                     body[0], body[1], body[2], ru, rp);
  return hipGetLastError();
}
hipError_t launch_residual(int P, int geo, int ps, hipStream_t s, const MeshView &m, const GeoView<double> &g,
                           const void *tabs, const double *st, const double *fst, const double *beta,
                           const double *p, const double *body, double *ru, double *rp) {
#define NSMF_RS(PP, GG)                                                                                  \
  if (P == PP && geo == GG && ps == PS_P) return residual_pg<PP, GG, PS_P>(s, m, g, tabs, st, fst, beta, p, body, ru, rp); \
  if (P == PP && geo == GG && ps == PS_Q) return residual_pg<PP, GG, PS_Q>(s, m, g, tabs, st, fst, beta, p, body, ru, rp);
  NSMF_RS(3, GEO_AFFINE) NSMF_RS(3, GEO_COLUMN) NSMF_RS(4, GEO_AFFINE) NSMF_RS(4, GEO_COLUMN)
  NSMF_RS(5, GEO_AFFINE) NSMF_RS(5, GEO_COLUMN)
#undef NSMF_RS
  return hipErrorInvalidValue;
}

template <int P, int GEO, int PS>
static hipError_t diag_pg(hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                          const double *st, const double *beta, double *ev, double *dp) {
  const TabSet<P> *ts = (const TabSet<P> *)tabs;
  if (g.rot != nullptr)   // nodal frames: the 3x3 slot blocks are formed
    hipLaunchKernelGGL((k_diag<P, GEO, PS, true>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, g, &ts->d, &ts->dsq, st,
                       beta, ev, dp);
  else
    hipLaunchKernelGGL((k_diag<P, GEO, PS, false>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, g, &ts->d, &ts->dsq, st,
                       beta, ev, dp);
  return hipGetLastError();
}
hipError_t launch_diag(int P, int geo, int ps, hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                       const double *st, const double *beta, double *ev, double *dp) {
#define NSMF_DG(PP, GG)                                                                           \
  if (P == PP && geo == GG && ps == PS_P) return diag_pg<PP, GG, PS_P>(s, m, g, tabs, st, beta, ev, dp); \
  if (P == PP && geo == GG && ps == PS_Q) return diag_pg<PP, GG, PS_Q>(s, m, g, tabs, st, beta, ev, dp);
  NSMF_DG(3, GEO_AFFINE) NSMF_DG(3, GEO_COLUMN) NSMF_DG(4, GEO_AFFINE) NSMF_DG(4, GEO_COLUMN)
  NSMF_DG(5, GEO_AFFINE) NSMF_DG(5, GEO_COLUMN)
#undef NSMF_DG
  return hipErrorInvalidValue;
}

template <typename T, int P, int GEO, bool VJP, int PS>
static hipError_t apply_t(hipStream_t s, const MeshView &m, const void *gview, const void *tabs, bool bf16,
                          const void *st, const void *fst, const void *beta, const void *xu, const void *xp, void *yu,
                          void *yp, double inv_n, double *gA, double *gB) {
  const TabSet<P> *ts = (const TabSet<P> *)tabs;
  const Tab<T, P> *tb;
  if constexpr (sizeof(T) == 8) tb = &ts->d;
  else tb = bf16 ? &ts->fb : &ts->f;
  const GeoView<T> &gv = *(const GeoView<T> *)gview;
  if (gv.rot != nullptr)   // nodal frames: the framed-slot variant
    hipLaunchKernelGGL((k_apply<T, P, GEO, VJP, PS, true>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, gv, tb, st,
                       (const T *)fst, (const T *)beta, (const T *)xu, (const T *)xp, (T *)yu, (T *)yp, inv_n, gA, gB);
  else
    hipLaunchKernelGGL((k_apply<T, P, GEO, VJP, PS, false>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, gv, tb, st,
                       (const T *)fst, (const T *)beta, (const T *)xu, (const T *)xp, (T *)yu, (T *)yp, inv_n, gA, gB);
  return hipGetLastError();
}
hipError_t launch_apply(int P, int geo, int ps, int prec, bool vjp, hipStream_t s, const MeshView &m, const void *gview,
                        const void *tabs, const void *st, const void *fst, const void *beta, const void *xu,
                        const void *xp, void *yu, void *yp, double inv_n, double *gA, double *gB) {
  const bool bf = prec == 2;
#define NSMF_AP(TT, PP, GG, VV)                                                                                   \
  if (P == PP && geo == GG && vjp == VV && (sizeof(TT) == 8) == (prec == 0) && ps == PS_P)                       \
    return apply_t<TT, PP, GG, VV, PS_P>(s, m, gview, tabs, bf, st, fst, beta, xu, xp, yu, yp, inv_n, gA, gB);  \
  if (P == PP && geo == GG && vjp == VV && (sizeof(TT) == 8) == (prec == 0) && ps == PS_Q)                       \
    return apply_t<TT, PP, GG, VV, PS_Q>(s, m, gview, tabs, bf, st, fst, beta, xu, xp, yu, yp, inv_n, gA, gB);
#define NSMF_AP2(TT, PP) \
  NSMF_AP(TT, PP, GEO_AFFINE, false) NSMF_AP(TT, PP, GEO_COLUMN, false) NSMF_AP(TT, PP, GEO_AFFINE, true) \
  NSMF_AP(TT, PP, GEO_COLUMN, true)
  NSMF_AP2(double, 3) NSMF_AP2(double, 4) NSMF_AP2(double, 5) NSMF_AP2(float, 3) NSMF_AP2(float, 4)
  NSMF_AP2(float, 5)
#undef NSMF_AP2
#undef NSMF_AP
  return hipErrorInvalidValue;
}

template <typename T, int P, int GEO, int PS>
static hipError_t grad_p_t(hipStream_t s, const MeshView &m, const void *gview, const void *tabs, bool bf16,
                           const void *xp, void *yu) {
  const TabSet<P> *ts = (const TabSet<P> *)tabs;
  const Tab<T, P> *tb;
  if constexpr (sizeof(T) == 8) tb = &ts->d;
  else tb = bf16 ? &ts->fb : &ts->f;
  const GeoView<T> &gv = *(const GeoView<T> *)gview;
  if (gv.rot != nullptr)
    hipLaunchKernelGGL((k_grad_p<T, P, GEO, PS, true>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, gv, tb,
                       (const T *)xp, (T *)yu);
  else
    hipLaunchKernelGGL((k_grad_p<T, P, GEO, PS, false>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, gv, tb,
                       (const T *)xp, (T *)yu);
  return hipGetLastError();
}
hipError_t launch_grad_p(int P, int geo, int ps, int prec, hipStream_t s, const MeshView &m, const void *gview,
                         const void *tabs, const void *xp, void *yu) {
  const bool bf = prec == 2;
#define NSMF_GP(TT, PP, GG)                                                                            \
  if (P == PP && geo == GG && (sizeof(TT) == 8) == (prec == 0) && ps == PS_P)                         \
    return grad_p_t<TT, PP, GG, PS_P>(s, m, gview, tabs, bf, xp, yu);                                 \
  if (P == PP && geo == GG && (sizeof(TT) == 8) == (prec == 0) && ps == PS_Q)                         \
    return grad_p_t<TT, PP, GG, PS_Q>(s, m, gview, tabs, bf, xp, yu);
#define NSMF_GP2(TT, PP) NSMF_GP(TT, PP, GEO_AFFINE) NSMF_GP(TT, PP, GEO_COLUMN)
  NSMF_GP2(double, 3) NSMF_GP2(double, 4) NSMF_GP2(double, 5) NSMF_GP2(float, 3) NSMF_GP2(float, 4) NSMF_GP2(float, 5)
#undef NSMF_GP2
#undef NSMF_GP
  return hipErrorInvalidValue;
}


template <int P, int GEO>
static hipError_t lines_pg(hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                           const double *st, const double *beta, const int32_t *lptr, const int32_t *lslot,
                           const uint8_t *dm, const int32_t *line_ptr, const int32_t *line_node,
                           const int32_t *prow, const int32_t *lrow, int64_t NR, int64_t n_lines, double *buf,
                           double *fac64, float *fac32) {
  if (g.rot != nullptr)   // nodal frames: rotated bottom rows
    hipLaunchKernelGGL((k_lines<P, GEO, true>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, g,
                       &((const TabSet<P> *)tabs)->d, st, beta, buf);
  else
    hipLaunchKernelGGL((k_lines<P, GEO, false>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, g,
                       &((const TabSet<P> *)tabs)->d, st, beta, buf);
  if (P == 3)
    hipLaunchKernelGGL(k_line_band<3>, dim3(grid1(m.n_nodes, 256)), dim3(256), 0, s, m.n_nodes, m.n_inc, NR, lptr,
                       lslot, prow, (const double *)buf, fac64);
  else if (P == 4)
    hipLaunchKernelGGL(k_line_band<4>, dim3(grid1(m.n_nodes, 256)), dim3(256), 0, s, m.n_nodes, m.n_inc, NR, lptr,
                       lslot, prow, (const double *)buf, fac64);
  else
    hipLaunchKernelGGL(k_line_band<5>, dim3(grid1(m.n_nodes, 256)), dim3(256), 0, s, m.n_nodes, m.n_inc, NR, lptr,
                       lslot, prow, (const double *)buf, fac64);
  if (n_lines > 0)
    hipLaunchKernelGGL(k_line_factor<P>, dim3(grid1(3 * line_threads(n_lines), 256)), dim3(256), 0, s, m.n_nodes,
                       n_lines, NR, line_ptr, line_node, lrow, dm, fac64, fac32);
  return hipGetLastError();
}
hipError_t launch_lines(int P, int geo, hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                        const double *st, const double *beta, const int32_t *lptr, const int32_t *lslot,
                        const uint8_t *dm, const int32_t *line_ptr, const int32_t *line_node,
                        const int32_t *prow, const int32_t *lrow, int64_t NR, int64_t n_lines, double *buf,
                        double *fac64, float *fac32) {
#define NSMF_LN(PP, GG)                                                                                          \
  if (P == PP && geo == GG)                                                                                      \
    return lines_pg<PP, GG>(s, m, g, tabs, st, beta, lptr, lslot, dm, line_ptr, line_node, prow, lrow, NR, n_lines, \
                            buf, fac64, fac32);
  NSMF_LN(3, GEO_AFFINE) NSMF_LN(3, GEO_COLUMN) NSMF_LN(4, GEO_AFFINE) NSMF_LN(4, GEO_COLUMN)
  NSMF_LN(5, GEO_AFFINE) NSMF_LN(5, GEO_COLUMN)
#undef NSMF_LN
  return hipErrorInvalidValue;
}
hipError_t launch_line_apply(hipStream_t s, int prec, int P, int64_t N, const int32_t *line_ptr, const int32_t *line_node,
                             const int32_t *lrow, int64_t NR, const int32_t *line_first, int64_t n_lines,
                             const void *fac, const void *x, void *y) {
  if (n_lines <= 0) return hipSuccess;
  const dim3 grid((unsigned)(3 * (line_threads(n_lines) / LINE_GROUP))), blk(LINE_GROUP);
#define NSMF_LA(WW)                                                                                             \
  if (P == WW) {                                                                                                \
    if (prec == 0)                                                                                              \
      hipLaunchKernelGGL((k_line_apply<double, WW>), grid, blk, 0, s, N, n_lines, NR, line_ptr, line_node,      \
                         lrow, line_first, (const double *)fac, (const double *)x, (double *)y);                \
    else                                                                                                        \
      hipLaunchKernelGGL((k_line_apply<float, WW>), grid, blk, 0, s, N, n_lines, NR, line_ptr, line_node,       \
                         lrow, line_first, (const float *)fac, (const float *)x, (float *)y);                   \
    return hipGetLastError();                                                                                   \
  }
  NSMF_LA(3) NSMF_LA(4) NSMF_LA(5)
#undef NSMF_LA
  return hipErrorInvalidValue;
}


template <int P>
static hipError_t lowo_coef_p(hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                              const double *X, const double *per, const double *u, const double *logA, double n,
                              double eps, double B0, bool picard, double *lo) {
  hipLaunchKernelGGL((k_lowo_coef<P>), dim3(m.nblocks), dim3(Launch<P>::NT), 0, s, m, g, &((const TabSet<P> *)tabs)->d, X,
                     per[0], per[1], u, logA, n, eps, B0, (int)picard, lo);
  return hipGetLastError();
}
hipError_t launch_lowo_coef(int P, hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                            const double *X, const double period[3], const double *u, const double *logA, double n,
                            double eps, double B0, bool picard, double *lo) {
  switch (P) {
    case 3: return lowo_coef_p<3>(s, m, g, tabs, X, period, u, logA, n, eps, B0, picard, lo);
    case 4: return lowo_coef_p<4>(s, m, g, tabs, X, period, u, logA, n, eps, B0, picard, lo);
    case 5: return lowo_coef_p<5>(s, m, g, tabs, X, period, u, logA, n, eps, B0, picard, lo);
  }
  return hipErrorInvalidValue;
}
hipError_t launch_lowo(int P, hipStream_t s, const MeshView &m, const GeoView<double> &g, const void *tabs,
                       const double *lo, const double *beta, const double *x, double *ev) {
#define NSMF_LO(PP)                                                                                               \
  if (P == PP) {                                                                                                  \
    hipLaunchKernelGGL((k_lowo<PP>), dim3(m.nblocks), dim3(Launch<PP>::NT), 0, s, m, g,                          \
                       &((const TabSet<PP> *)tabs)->d, lo, beta, x, ev);                                          \
    return hipGetLastError();                                                                                     \
  }
  NSMF_LO(3) NSMF_LO(4) NSMF_LO(5)
#undef NSMF_LO
  return hipErrorInvalidValue;
}

}  // namespace nsmf
