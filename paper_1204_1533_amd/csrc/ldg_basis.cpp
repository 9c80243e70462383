// 1-D operators of the line-DG scheme (Sections 2.1-2.2), host side.
//
// Nodes: Gauss-Lobatto-Legendre (or equispaced) points on [0,1] with s_0 = 0,
// s_p = 1.  Quadrature: Gauss-Legendre with ceil((3p+1)/2) points (exact for
// degree 3p).  From these: interpolation I[g][i] = phi_i(x_g), test-function
// derivative Dg[g][i] = phi_i'(x_g), mass matrix M = I^T W I, and the operators
// the kernels use with the mass solve folded in (Section 2.2): V = M^{-1} Dg^T W,
// L0 = M^{-1} e_0, L1 = M^{-1} e_p; nodal derivative Dn[i][j] = phi_j'(s_i).
// Everything is computed in long double and rounded once to double.
#include <cmath>
#include <cstring>
#include <vector>

#include "ldg_device.hpp"

namespace ldg {

typedef long double R;

static void legendre(int n, R x, R& pn, R& pnm1) {
  R p0 = 1, p1 = x;
  if (n == 0) {
    pn = 1;
    pnm1 = 0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    R p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pnm1 = p0;
}

// zeros of P_n' (interior Lobatto points) on [-1,1] by Newton
static std::vector<R> lobatto(int p) {
  std::vector<R> x(p + 1);
  x[0] = -1;
  x[p] = 1;
  const R pi = 3.141592653589793238462643383279502884L;
  for (int i = 1; i < p; ++i) {
    R z = -cosl(pi * i / p);
    for (int it = 0; it < 100; ++it) {
      R P, Pm;
      legendre(p, z, P, Pm);
      R d1 = p * (Pm - z * P) / (1 - z * z);
      R d2 = (2 * z * d1 - p * (p + 1) * P) / (1 - z * z);
      R step = d1 / d2;
      z -= step;
      if (fabsl(step) < 1e-19L) break;
    }
    x[i] = z;
  }
  return x;
}

static void gauss(int n, std::vector<R>& x, std::vector<R>& w) {
  x.resize(n);
  w.resize(n);
  const R pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    R z = -cosl(pi * (i + 0.75L) / (n + 0.5L));
    R P, Pm, dP;
    for (int it = 0; it < 100; ++it) {
      legendre(n, z, P, Pm);
      dP = n * (Pm - z * P) / (1 - z * z);
      R step = P / dP;
      z -= step;
      if (fabsl(step) < 1e-19L) break;
    }
    legendre(n, z, P, Pm);
    dP = n * (Pm - z * P) / (1 - z * z);
    x[i] = z;
    w[i] = 2 / ((1 - z * z) * dP * dP);
  }
}

static R lag(const std::vector<R>& s, int i, R x) {
  R v = 1;
  for (size_t j = 0; j < s.size(); ++j)
    if ((int)j != i) v *= (x - s[j]) / (s[i] - s[j]);
  return v;
}
static R dlag(const std::vector<R>& s, int i, R x) {
  R acc = 0;
  for (size_t k = 0; k < s.size(); ++k) {
    if ((int)k == i) continue;
    R t = 1 / (s[i] - s[k]);
    for (size_t j = 0; j < s.size(); ++j)
      if ((int)j != i && j != k) t *= (x - s[j]) / (s[i] - s[j]);
    acc += t;
  }
  return acc;
}

// Fills ops; returns false for unsupported p.
bool build_line_ops(int p, int node_family, LineOps& ops, std::vector<double>* nodes_out) {
  if (p < 1 || p > N1MAX - 1) return false;
  const int n1 = p + 1, ng = n_gauss(p);
  std::vector<R> s(n1);
  if (node_family == 0) {
    std::vector<R> x = lobatto(p);
    for (int i = 0; i < n1; ++i) s[i] = (x[i] + 1) / 2;
  } else {
    for (int i = 0; i < n1; ++i) s[i] = (R)i / p;
  }
  s[0] = 0;
  s[p] = 1;
  std::vector<R> xg, wg;
  gauss(ng, xg, wg);
  for (int g = 0; g < ng; ++g) {
    xg[g] = (xg[g] + 1) / 2;
    wg[g] = wg[g] / 2;
  }
  std::memset(&ops, 0, sizeof(ops));
  R I[NGMAX][N1MAX] = {}, Dg[NGMAX][N1MAX] = {};
  for (int g = 0; g < ng; ++g)
    for (int i = 0; i < n1; ++i) {
      I[g][i] = lag(s, i, xg[g]);
      Dg[g][i] = dlag(s, i, xg[g]);
      ops.I[g][i] = (double)I[g][i];
      ops.Dg[g][i] = (double)Dg[g][i];
    }
  // mass matrix and its inverse (Gauss-Jordan with partial pivoting)
  R Mm[N1MAX][2 * N1MAX] = {};
  for (int i = 0; i < n1; ++i) {
    for (int j = 0; j < n1; ++j) {
      R acc = 0;
      for (int g = 0; g < ng; ++g) acc += wg[g] * I[g][i] * I[g][j];
      Mm[i][j] = acc;
    }
    Mm[i][n1 + i] = 1;
  }
  for (int c = 0; c < n1; ++c) {
    int piv = c;
    for (int r = c + 1; r < n1; ++r)
      if (fabsl(Mm[r][c]) > fabsl(Mm[piv][c])) piv = r;
    if (piv != c)
      for (int k = 0; k < 2 * n1; ++k) {
        R t = Mm[c][k];
        Mm[c][k] = Mm[piv][k];
        Mm[piv][k] = t;
      }
    R d = Mm[c][c];
    for (int k = 0; k < 2 * n1; ++k) Mm[c][k] /= d;
    for (int r = 0; r < n1; ++r) {
      if (r == c) continue;
      R f = Mm[r][c];
      for (int k = 0; k < 2 * n1; ++k) Mm[r][k] -= f * Mm[c][k];
    }
  }
  for (int i = 0; i < n1; ++i) {
    ops.L0[i] = (double)Mm[i][n1 + 0];
    ops.L1[i] = (double)Mm[i][n1 + p];
    for (int g = 0; g < ng; ++g) {
      R acc = 0;
      for (int j = 0; j < n1; ++j) acc += Mm[i][n1 + j] * Dg[g][j];
      ops.V[i][g] = (double)(acc * wg[g]);
    }
    for (int j = 0; j < n1; ++j) ops.Dn[i][j] = (double)dlag(s, j, s[i]);
  }
  if (nodes_out) {
    nodes_out->resize(n1);
    for (int i = 0; i < n1; ++i) (*nodes_out)[i] = (double)s[i];
  }
  return true;
}

// Nodes of a (p+1)^D element grouped by level i + j (+ k), ascending within a
// level (the order of the factor rows read by the preconditioner apply).
void build_level_order(int D, int P, LevelOrder& lv) {
  const int N1 = P + 1;
  int NP = 1;
  for (int k = 0; k < D; ++k) NP *= N1;
  auto level = [&](int a) {
    int s = 0;
    for (int k = 0; k < D; ++k) {
      s += a % N1;
      a /= N1;
    }
    return s;
  };
  int pos = 0;
  for (int L = 0; L <= D * P; ++L) {
    lv.off[L] = (int16_t)pos;
    for (int a = 0; a < NP; ++a)
      if (level(a) == L) {
        lv.rank[a] = (int16_t)pos;
        lv.node[pos++] = (int16_t)a;
      }
  }
  lv.off[D * P + 1] = (int16_t)pos;
}

}  // namespace ldg
