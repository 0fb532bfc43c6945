// Reference-element tables of the engine, computed in FP64 on the host.
//
// Velocity: Q_k Lagrange basis on the Gauss-Lobatto nodes (Sec. 3.2.1): -1, +1 and the
// roots of P_k', found by Newton's method on P_k' with P_k'' from Legendre's equation.
// Quadrature: Gauss-Legendre with k+1 points per direction (roots of P_{k+1} by Newton's
// method, weights 2 / ((1 - x^2) P_{k+1}'(x)^2)).
// Hanging nodes: child-interval interpolation I[h][i][m] = l_m(x_i^h), x_i^0 = (xi_i - 1)/2,
// x_i^1 = (xi_i + 1)/2 -- the tensor-product interpolation of figure "hanging", one
// direction at a time.
// Pressure: normalised Legendre values sqrt((2j+1)/2) P_j(g_q); exponents (i, j, l) with
// i+j+l <= k-1 ordered by (i+j+l, l, j, i).
#include <cmath>
#include <cstring>

#include "nsmf_internal.h"

namespace nsmf {

static void legendre(int n, double x, double *p, double *dp) {
  // P_n and P_n' by the three-term recurrence.
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { *p = 1.0; *dp = 0.0; return; }
  for (int m = 2; m <= n; ++m) {
    double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
    double d2 = d0 + (2.0 * m - 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *p = p1; *dp = d1;
}

static double lagrange(const double *nodes, int n, int a, double x) {
  double v = 1.0;
  for (int b = 0; b < n; ++b)
    if (b != a) v *= (x - nodes[b]) / (nodes[a] - nodes[b]);
  return v;
}

static double lagrange_deriv(const double *nodes, int n, int a, double x) {
  // sum over c != a of 1/(x_a - x_c) * prod_{b != a, c} (x - x_b)/(x_a - x_b); safe at nodes
  double tot = 0.0;
  for (int c = 0; c < n; ++c) {
    if (c == a) continue;
    double term = 1.0 / (nodes[a] - nodes[c]);
    for (int b = 0; b < n; ++b)
      if (b != a && b != c) term *= (x - nodes[b]) / (nodes[a] - nodes[b]);
    tot += term;
  }
  return tot;
}

void build_tables(int k, int pspace, HostTables *t) {
  std::memset(t, 0, sizeof(*t));
  const int P = k + 1;
  t->P = P;
  // Gauss-Lobatto nodes
  t->xi[0] = -1.0;
  t->xi[k] = 1.0;
  for (int i = 1; i < k; ++i) {
    double x = -std::cos(M_PI * i / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, x, &p, &dp);
      double d2 = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
      double dx = dp / d2;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    t->xi[i] = x;
  }
  // Gauss-Legendre points and weights (P = k+1 points)
  for (int i = 0; i < P; ++i) {
    double x = -std::cos(M_PI * (i + 0.75) / (P + 0.5));
    double p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(P, x, &p, &dp);
      double dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    legendre(P, x, &p, &dp);
    t->g[i] = x;
    t->w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  // nodes and weights are symmetric about 0: remove the last-ulp asymmetry of the iterations
  for (int i = 0; i < P / 2; ++i) {
    const double x = 0.5 * (t->xi[k - i] - t->xi[i]), g = 0.5 * (t->g[k - i] - t->g[i]);
    const double w = 0.5 * (t->w[k - i] + t->w[i]);
    t->xi[i] = -x; t->xi[k - i] = x;
    t->g[i] = -g; t->g[k - i] = g;
    t->w[i] = w; t->w[k - i] = w;
  }
  if (P % 2) t->xi[k / 2] = t->g[k / 2] = 0.0;
  for (int q = 0; q < P; ++q)
    for (int a = 0; a < P; ++a) {
      t->B[q][a] = lagrange(t->xi, P, a, t->g[q]);
      t->D[q][a] = lagrange_deriv(t->xi, P, a, t->g[q]);
    }
  for (int i = 0; i < P; ++i)
    for (int a = 0; a < P; ++a) t->G[i][a] = lagrange_deriv(t->xi, P, a, t->xi[i]);
  for (int h = 0; h < 2; ++h)
    for (int i = 0; i < P; ++i) {
      double xc = 0.5 * (t->xi[i] + (h ? 1.0 : -1.0));
      for (int m = 0; m < P; ++m) t->I[h][i][m] = lagrange(t->xi, P, m, xc);
    }
  if (pspace == PS_P) {
    for (int j = 0; j < k; ++j)
      for (int q = 0; q < P; ++q) {
        double p, dp;
        legendre(j, t->g[q], &p, &dp);
        t->L[j][q] = std::sqrt((2.0 * j + 1.0) / 2.0) * p;
      }
    t->n_p = k * (k + 1) * (k + 2) / 6;
  } else {
    // the k-1 Gauss points (roots of P_{k-1}), symmetrised, and their Lagrange basis
    const int m = k - 1;
    double gp[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < m; ++i) {
      double x = -std::cos(M_PI * (i + 0.75) / (m + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p, dp;
        legendre(m, x, &p, &dp);
        const double dx = p / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-17) break;
      }
      gp[i] = x;
    }
    for (int i = 0; i < m / 2; ++i) {
      const double x = 0.5 * (gp[m - 1 - i] - gp[i]);
      gp[i] = -x;
      gp[m - 1 - i] = x;
    }
    if (m % 2) gp[m / 2] = 0.0;
    for (int j = 0; j < m; ++j)
      for (int q = 0; q < P; ++q) t->L[j][q] = lagrange(gp, m, j, t->g[q]);
    t->n_p = m * m * m;
  }
}

static float round_bf16(double v) {
  // round-to-nearest-even of the float value to the 8-bit-mantissa bfloat16 grid
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  uint32_t lsb = (u >> 16) & 1u;
  u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
  std::memcpy(&f, &u, 4);
  return f;
}

template <typename T, int P>
Tab<T, P> make_tab(const HostTables &h, bool bf16_ops) {
  Tab<T, P> t;
  std::memset(&t, 0, sizeof(t));
  for (int q = 0; q < P; ++q)
    for (int a = 0; a < P; ++a) {
      t.B[q][a] = bf16_ops ? (T)round_bf16(h.B[q][a]) : (T)h.B[q][a];
      t.D[q][a] = bf16_ops ? (T)round_bf16(h.D[q][a]) : (T)h.D[q][a];
    }
  for (int i = 0; i < P; ++i)
    for (int m = 0; m < P; ++m) t.I[i][m] = (T)h.I[0][i][m];
  for (int j = 0; j < P - 1; ++j)
    for (int q = 0; q < P; ++q) t.L[j][q] = (T)h.L[j][q];
  for (int q = 0; q < P; ++q) t.w[q] = (T)h.w[q];
  for (int i = 0; i < P; ++i)
    for (int a = 0; a < P; ++a) t.G[i][a] = (T)h.G[i][a];
  // folded forms, from the entries as stored (bfloat16-rounded for the bf16 variant)
  for (int K = 0; K < 4; ++K) {
    auto M = [&](int q, int m) -> double {
      const int r = K < 2 ? q : m, c = K < 2 ? m : q;
      return (K % 2 == 0) ? (double)t.B[r][c] : (double)t.D[r][c];
    };
    for (int q = 0; q < (P + 1) / 2; ++q) {
      for (int m = 0; m < P / 2; ++m) {
        t.Ke[K][q][m] = (T)(0.5 * (M(q, m) + M(q, P - 1 - m)));
        t.Ko[K][q][m] = (T)(0.5 * (M(q, m) - M(q, P - 1 - m)));
      }
      t.Kc[K][q] = (P % 2) ? (T)M(q, P / 2) : T(0);
    }
  }
  return t;
}

template <int P> static void fill_set(const HostTables &h, TabSet<P> *t) {
  t->d = make_tab<double, P>(h, false);
  t->f = make_tab<float, P>(h, false);
  t->fb = make_tab<float, P>(h, true);
  t->dsq = t->d;
  for (int i = 0; i < P; ++i)
    for (int k = 0; k < P; ++k) t->dsq.I[i][k] = t->d.I[i][k] * t->d.I[i][k];
}
size_t tabset_bytes(int P) {
  return P == 3 ? sizeof(TabSet<3>) : (P == 4 ? sizeof(TabSet<4>) : (P == 5 ? sizeof(TabSet<5>) : 0));
}
void fill_tabset(const HostTables &h, void *buf) {
  std::memset(buf, 0, tabset_bytes(h.P));
  if (h.P == 3) fill_set<3>(h, (TabSet<3> *)buf);
  if (h.P == 4) fill_set<4>(h, (TabSet<4> *)buf);
  if (h.P == 5) fill_set<5>(h, (TabSet<5> *)buf);
}

template Tab<double, 3> make_tab<double, 3>(const HostTables &, bool);
template Tab<double, 4> make_tab<double, 4>(const HostTables &, bool);
template Tab<double, 5> make_tab<double, 5>(const HostTables &, bool);
template Tab<float, 3> make_tab<float, 3>(const HostTables &, bool);
template Tab<float, 4> make_tab<float, 4>(const HostTables &, bool);
template Tab<float, 5> make_tab<float, 5>(const HostTables &, bool);

}  // namespace nsmf
