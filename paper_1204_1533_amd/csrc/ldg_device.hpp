// Device-side building blocks of the line-DG kernels (gfx950).
//
// * Dual<K>: forward-mode dual numbers (value + K tangents), used to
//   differentiate the flux functions exactly for the Jacobian blocks and for
//   the exact tangent product.
// * Physical fluxes: Euler (ideal gas), Navier-Stokes viscous flux with
//   constant viscosity and Prandtl number (Section 5.2), Poisson F = -q
//   (Section 5.1).
// * Roe's approximate Riemann solver (Section 5.2) in the usual wave form:
//   1/2 (F_L + F_R).n - 1/2 sum_k |lambda_k| alpha_k r_k with Roe averages,
//   no entropy fix; non-unit normals by Fhat.n = |n| Fhat.nbar (Section 2.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldg {

constexpr int N1MAX = 5;  // p <= 4
constexpr int NGMAX = 7;  // ceil((3*4+1)/2)

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
__host__ __device__ constexpr int n_gauss(int p) { return (3 * p + 2) / 2; }

// ---------------------------------------------------------------- 1-D operators
// Passed by value to every kernel (kernel-argument segment).
struct LineOps {
  double I[NGMAX][N1MAX];   // phi_i(x_g)
  double Dg[NGMAX][N1MAX];  // phi_i'(x_g)
  double V[N1MAX][NGMAX];   // (M^{-1} Dg^T W)[i][g]: test-derivative term with mass solve folded in
  double L0[N1MAX];         // M^{-1} e_0  (lifting of the xi = 0 flux)
  double L1[N1MAX];         // M^{-1} e_p  (lifting of the xi = 1 flux)
  double Dn[N1MAX][N1MAX];  // phi_j'(s_i): nodal derivative (mapping gradient)
};

// Nodes of an element sorted by level a_0 + .. + a_{D-1} (the independent
// sets of the block ILU(0) sweeps), ascending node index within a level:
// node[off[L] .. off[L+1]) is level L, rank[a] the position of node a.
constexpr int NPMAX = 125;  // (p+1)^D for p <= 4
struct LevelOrder {
  int16_t node[NPMAX];
  int16_t rank[NPMAX];
  int16_t off[3 * 4 + 2];
};

struct MeshParams {
  int64_t E;
  double gamma, mu, prandtl, c11i, c11d;
  const double* xyz;       // [E][D][Np]
  const int64_t* face_nbr; // [E][2D]
  const int32_t* nbr_node; // [E][2D][Nf]
  const int8_t* sw;        // [E][D]
  const double* gD;        // [E][2D][m][Nf] or null
  const double* gN;        // [E][2D][m][Nf] or null
  const double* S;         // [E][m][Np] or null
  double c22;              // LDG C22 (eqs. ldgflux2, neumann2); 0: the reduced system
  const double* geo;       // per-element geometry record (GeoShape), fixed by the mesh
};

// Kind of a face from its face_nbr entry: a neighbour (interior) or a boundary
// -(kind + 1): Dirichlet (eqs. dirichlet1/2; inviscid: the characteristic
// condition Roe(g_D, u_in)), Neumann (eqs. neumann1/2 with C22 = 0), slip wall.
constexpr int BC_INTERIOR = -1, BC_DIRICHLET = 0, BC_NEUMANN = 1, BC_SLIP = 2;
__host__ __device__ inline int face_kind(int64_t nb) { return nb >= 0 ? BC_INTERIOR : (int)(-nb - 1); }

// ---------------------------------------------------------------- node indexing
// node(n, l, t): position t on line l of direction n.
template <int D, int N1>
__host__ __device__ inline int line_node(int n, int l, int t) {
  int s = 1;
  for (int k = 0; k < n; ++k) s *= N1;
  return (l % s) + t * s + (l / s) * s * N1;
}
template <int N1>
__host__ __device__ inline void node_line(int node, int n, int& l, int& t) {
  int s = 1;
  for (int k = 0; k < n; ++k) s *= N1;
  t = (node / s) % N1;
  l = (node % s) + (node / (s * N1)) * s;
}

// ---------------------------------------------------------------- XCD-aware block order
// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  This
// maps hardware block b of G to a logical block so that every XCD walks one
// contiguous run of blocks (neighbouring elements then share an L2).  It is a
// bijection on [0, G).
constexpr int N_XCD = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
  const int64_t x = b % N_XCD, k = b / N_XCD, per = G / N_XCD, rem = G % N_XCD;
  return x * per + (x < rem ? x : rem) + k;
}

// ---------------------------------------------------------------- line-pattern slots
// A row node a has D p + 1 line-pattern columns: slots 0..p are the nodes of its
// direction-0 line by position (its own position is the diagonal slot); then,
// for each further direction n, p slots for the other nodes of its direction-n line.
// column node of line slot `slot` for row node a (within the element)
template <int D, int P>
__host__ __device__ inline int slot_col(int a, int slot) {
  constexpr int N1 = P + 1;
  if (slot < N1) return line_node<D, N1>(0, a / N1, slot);
  const int n = 1 + (slot - N1) / P, r = (slot - N1) % P;
  int l, t;
  node_line<N1>(a, n, l, t);
  return line_node<D, N1>(n, l, r < t ? r : r + 1);
}
template <int N1>
__host__ __device__ inline int slot_of(int n, int t, int tp, int self) {
  // slot of column position tp on the row's direction-n line; the row sits at t
  if (tp == t) return self;
  return n == 0 ? tp : N1 + (n - 1) * (N1 - 1) + (tp < t ? tp : tp - 1);
}

// ---------------------------------------------------------------- dual numbers
template <int K>
struct Dual {
  double v;
  double d[K];
};

__device__ __forceinline__ double val(double x) { return x; }
template <int K> __device__ __forceinline__ double val(const Dual<K>& x) { return x.v; }

template <int K>
__device__ __forceinline__ Dual<K> mk(double v) {
  Dual<K> r;
  r.v = v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = 0.0;
  return r;
}
template <class T> struct ScalarOf { static __device__ __forceinline__ T make(double v) { return T(v); } };
template <int K> struct ScalarOf<Dual<K>> {
  static __device__ __forceinline__ Dual<K> make(double v) { return mk<K>(v); }
};
template <class T> __device__ __forceinline__ T cst(double v) { return ScalarOf<T>::make(v); }

#define LDG_DUAL_BIN(OP, VEXPR, DEXPR)                                                   \
  template <int K>                                                                       \
  __device__ __forceinline__ Dual<K> operator OP(const Dual<K>& a, const Dual<K>& b) {   \
    Dual<K> r;                                                                           \
    r.v = VEXPR;                                                                         \
    _Pragma("unroll") for (int k = 0; k < K; ++k) r.d[k] = DEXPR;                        \
    return r;                                                                            \
  }
LDG_DUAL_BIN(+, a.v + b.v, a.d[k] + b.d[k])
LDG_DUAL_BIN(-, a.v - b.v, a.d[k] - b.d[k])
LDG_DUAL_BIN(*, a.v * b.v, a.d[k] * b.v + a.v * b.d[k])
#undef LDG_DUAL_BIN
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  double ib = 1.0 / b.v;
  r.v = a.v * ib;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
template <int K> __device__ __forceinline__ Dual<K> operator+(const Dual<K>& a, double b) { Dual<K> r = a; r.v += b; return r; }
template <int K> __device__ __forceinline__ Dual<K> operator+(double b, const Dual<K>& a) { Dual<K> r = a; r.v += b; return r; }
template <int K> __device__ __forceinline__ Dual<K> operator-(const Dual<K>& a, double b) { Dual<K> r = a; r.v -= b; return r; }
template <int K>
__device__ __forceinline__ Dual<K> operator-(double b, const Dual<K>& a) {
  Dual<K> r;
  r.v = b - a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K>& a) {
  Dual<K> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K>& a, double b) {
  Dual<K> r;
  r.v = a.v * b;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b;
  return r;
}
template <int K> __device__ __forceinline__ Dual<K> operator*(double b, const Dual<K>& a) { return a * b; }
template <int K> __device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, double b) { return a * (1.0 / b); }
template <int K>
__device__ __forceinline__ Dual<K> operator/(double a, const Dual<K>& b) {
  Dual<K> r;
  double ib = 1.0 / b.v;
  r.v = a * ib;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = -r.v * b.d[k] * ib;
  return r;
}
template <int K> __device__ __forceinline__ Dual<K>& operator+=(Dual<K>& a, const Dual<K>& b) { a = a + b; return a; }
template <int K> __device__ __forceinline__ Dual<K>& operator-=(Dual<K>& a, const Dual<K>& b) { a = a - b; return a; }

__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
template <int K>
__device__ __forceinline__ Dual<K> dsqrt(const Dual<K>& a) {
  Dual<K> r;
  r.v = sqrt(a.v);
  double h = 0.5 / r.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * h;
  return r;
}
__device__ __forceinline__ double dabs(double x) { return fabs(x); }
// |x| with derivative sign(x), sign(0) = 0
template <int K>
__device__ __forceinline__ Dual<K> dabs(const Dual<K>& a) {
  double s = a.v > 0.0 ? 1.0 : (a.v < 0.0 ? -1.0 : 0.0);
  Dual<K> r;
  r.v = fabs(a.v);
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = s * a.d[k];
  return r;
}

// ---------------------------------------------------------------- physics
constexpr int EQ_POISSON = 0, EQ_EULER = 1, EQ_NS = 2;
template <int D, int EQ> struct Eq {
  static constexpr int M = (EQ == EQ_POISSON) ? 1 : D + 2;
  static constexpr bool INV = (EQ != EQ_POISSON);
  static constexpr bool VIS = (EQ != EQ_EULER);
};

// f[c] = F^inv(u)[c][:] . a
template <int D, class T>
__device__ __forceinline__ void euler_flux_dot(const T* u, const double* a, double gamma, T* f) {
  const T rho = u[0];
  const T irho = 1.0 / rho;
  T vel[D];
  T vn = cst<T>(0.0), ke = cst<T>(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    vel[d] = u[1 + d] * irho;
    vn += vel[d] * a[d];
    ke += u[1 + d] * vel[d];
  }
  const T p = (gamma - 1.0) * (u[D + 1] - 0.5 * ke);
  f[0] = rho * vn;
#pragma unroll
  for (int i = 0; i < D; ++i) f[1 + i] = u[1 + i] * vn + p * a[i];
  f[D + 1] = (u[D + 1] + p) * vn;
}

// f[c] += F^vis(u, q)[c][:] . a  (NS: F^vis = -(0, tau_ij, u_i tau_ij - q_j); q_j = -(mu/Pr) dh/dx_j)
// The gradient may have a different scalar type TQ than the state (e.g. plain
// doubles while the state carries tangents); F^vis is linear in q.
template <int D, int EQ, class T, class TQ = T>
__device__ __forceinline__ void visc_flux_dot_add(const T* u, const TQ* q /*[M][D]*/, const double* a,
                                                  double gamma, double mu, double prandtl, T* f) {
  if constexpr (EQ == EQ_POISSON) {
    T s = cst<T>(0.0);
#pragma unroll
    for (int d = 0; d < D; ++d) s = s + q[d] * a[d];
    f[0] -= s;
  } else {
    const T irho = 1.0 / u[0];
    T vel[D];
#pragma unroll
    for (int d = 0; d < D; ++d) vel[d] = u[1 + d] * irho;
    const T Esp = u[D + 1] * irho;
    T dv[D][D];  // dv[i][j] = d u_i / d x_j
    T dh[D];
    T div = cst<T>(0.0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const TQ dr = q[0 * D + j];
      T dE = (q[(D + 1) * D + j] - Esp * dr) * irho;
      T kin = cst<T>(0.0);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        dv[i][j] = (q[(1 + i) * D + j] - vel[i] * dr) * irho;
        kin += vel[i] * dv[i][j];
      }
      dh[j] = gamma * (dE - kin);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) div += dv[i][i];
    // tau . a and heat . a
    T energy = cst<T>(0.0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T ta = cst<T>(0.0);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T tij = mu * (dv[i][j] + dv[j][i]);
        if (i == j) tij -= (2.0 * mu / 3.0) * div;
        ta += tij * a[j];
      }
      f[1 + i] -= ta;
      energy += vel[i] * ta;
    }
    T qa = cst<T>(0.0);
#pragma unroll
    for (int j = 0; j < D; ++j) qa += dh[j] * a[j];
    f[D + 1] -= energy + (mu / prandtl) * qa;
  }
}

// Fhat.n with uR on the side n points to (outside), uL inside.
template <int D, class T>
__device__ __forceinline__ void roe_flux(const T* uR, const T* uL, const double* n, double gamma, T* F) {
  constexpr int M = D + 2;
  double nn2 = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) nn2 += n[d] * n[d];
  const double nn = sqrt(nn2);
  double nb[D];
#pragma unroll
  for (int d = 0; d < D; ++d) nb[d] = n[d] / nn;
  // primitive states
  const T rL = uL[0], rR = uR[0];
  const T irL = 1.0 / rL, irR = 1.0 / rR;
  T vL[D], vR[D];
  T keL = cst<T>(0.0), keR = cst<T>(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    vL[d] = uL[1 + d] * irL;
    vR[d] = uR[1 + d] * irR;
    keL += uL[1 + d] * vL[d];
    keR += uR[1 + d] * vR[d];
  }
  const T pL = (gamma - 1.0) * (uL[D + 1] - 0.5 * keL);
  const T pR = (gamma - 1.0) * (uR[D + 1] - 0.5 * keR);
  const T HL = (uL[D + 1] + pL) * irL;
  const T HR = (uR[D + 1] + pR) * irR;
  // Roe averages
  const T sL = dsqrt(rL), sR = dsqrt(rR);
  const T isum = 1.0 / (sL + sR);
  T vh[D];
  T q2 = cst<T>(0.0), vnh = cst<T>(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    vh[d] = (sL * vL[d] + sR * vR[d]) * isum;
    q2 += vh[d] * vh[d];
    vnh += vh[d] * nb[d];
  }
  const T Hh = (sL * HL + sR * HR) * isum;
  const T rh = sL * sR;
  const T c2 = (gamma - 1.0) * (Hh - 0.5 * q2);
  const T ch = dsqrt(c2);
  // jumps
  T dvn = cst<T>(0.0);
  T dv[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    dv[d] = vR[d] - vL[d];
    dvn += dv[d] * nb[d];
  }
  const T dp = pR - pL, dr = rR - rL;
  const T l1 = dabs(vnh - ch), l2 = dabs(vnh), l3 = dabs(vnh + ch);
  const T ic2 = 1.0 / c2;
  const T a1 = (dp - rh * ch * dvn) * (0.5 * ic2);
  const T a3 = (dp + rh * ch * dvn) * (0.5 * ic2);
  const T a2 = dr - dp * ic2;
  const T w1 = l1 * a1, w3 = l3 * a3, w2 = l2 * a2, ws = l2 * rh;
  T diss[M];
  diss[0] = w1 + w2 + w3;
  T vdv = cst<T>(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    vdv += vh[d] * dv[d];
    diss[1 + d] = w1 * (vh[d] - ch * nb[d]) + w2 * vh[d] + w3 * (vh[d] + ch * nb[d]) +
                  ws * (dv[d] - dvn * nb[d]);
  }
  diss[D + 1] = w1 * (Hh - ch * vnh) + w2 * (0.5 * q2) + w3 * (Hh + ch * vnh) + ws * (vdv - vnh * dvn);
  // central part
  T vnL = cst<T>(0.0), vnR = cst<T>(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    vnL += vL[d] * nb[d];
    vnR += vR[d] * nb[d];
  }
  F[0] = nn * (0.5 * (rL * vnL + rR * vnR) - 0.5 * diss[0]);
#pragma unroll
  for (int d = 0; d < D; ++d)
    F[1 + d] = nn * (0.5 * (uL[1 + d] * vnL + pL * nb[d] + uR[1 + d] * vnR + pR * nb[d]) - 0.5 * diss[1 + d]);
  F[D + 1] = nn * (0.5 * ((uL[D + 1] + pL) * vnL + (uR[D + 1] + pR) * vnR) - 0.5 * diss[D + 1]);
}

// ---------------------------------------------------------------- metric
// Row n of the cofactor matrix of G (G[a][b] = dx_a/dX_b): a_n = J G^{-T} N_n.
template <int D>
__host__ __device__ inline void cofactor_row(const double G[D][D], int n, double* a) {
  if constexpr (D == 2) {
    // adj(G) = [[G11, -G01], [-G10, G00]]; row n of J G^{-1}
    if (n == 0) { a[0] = G[1][1]; a[1] = -G[0][1]; }
    else        { a[0] = -G[1][0]; a[1] = G[0][0]; }
  } else {
    // row n of adj(G): cross product of columns n+1 and n+2 of G
    const int b1 = (n + 1) % 3, b2 = (n + 2) % 3;
    a[0] = G[1][b1] * G[2][b2] - G[2][b1] * G[1][b2];
    a[1] = G[2][b1] * G[0][b2] - G[0][b1] * G[2][b2];
    a[2] = G[0][b1] * G[1][b2] - G[1][b1] * G[0][b2];
  }
}
template <int D>
__host__ __device__ inline double det(const double G[D][D]) {
  if constexpr (D == 2) return G[0][0] * G[1][1] - G[0][1] * G[1][0];
  else
    return G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) - G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
           G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
}

}  // namespace ldg

namespace ldg {
// Mirror state across a wall with normal n: normal momentum reversed, density
// and energy kept (the outside state of a slip wall).
template <int D, class T>
__device__ __forceinline__ void mirror_state(const T* u, const double* n, T* r) {
  double nn2 = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) nn2 += n[d] * n[d];
  const double inv = 1.0 / sqrt(nn2);
  T mn = cst<T>(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) mn += u[1 + d] * (n[d] * inv);
  r[0] = u[0];
#pragma unroll
  for (int d = 0; d < D; ++d) r[1 + d] = u[1 + d] - (2.0 * n[d] * inv) * mn;
  r[D + 1] = u[D + 1];
}

// Point flux Fhat . n at one face node (Sections 2.2 and 3), by face kind:
//   interior   inviscid Roe(u_out, u_in; n); viscous F^vis of the outside state
//              when the face switch S is +1, of the inside state when S = -1,
//              dotted with n, plus C11 |n| (u_in - u_out);
//   Dirichlet  Roe(g_D, u_in; n) + F^vis(u_in, q_in) . n + C11_D |n| (u_in - g_D)
//              (u_out holds g_D);
//   Neumann    |n| g_N (u_out holds g_N), independent of u and q;
//   slip wall  Roe(u_m, u_in; n) with the mirror state u_m, no viscous flux.
// qsel is the gradient of the side whose viscous flux is taken: the outside
// for an interior face with S = +1, the inside otherwise.  The viscous part is
// evaluated first so the gradient is dead before the Riemann solve.
template <int D, int EQ, class T, bool WITH_INV = true, class TQ = T>
__device__ __forceinline__ void face_flux_point(const T* uin, const T* uout, const TQ* qsel, const double* nrm,
                                                int S, int kind, const MeshParams& mp, T* F) {
  constexpr int M = Eq<D, EQ>::M;
  double nn = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) nn += nrm[d] * nrm[d];
  nn = sqrt(nn);
#pragma unroll
  for (int c = 0; c < M; ++c) F[c] = cst<T>(0.0);
  if (kind == BC_NEUMANN) {
#pragma unroll
    for (int c = 0; c < M; ++c) F[c] = nn * uout[c];
    return;
  }
  if constexpr (Eq<D, EQ>::VIS) {
    if (kind != BC_SLIP) {
      const bool use_out = kind == BC_INTERIOR && S > 0;
      visc_flux_dot_add<D, EQ, T, TQ>(use_out ? uout : uin, qsel, nrm, mp.gamma, mp.mu, mp.prandtl, F);
      const double c11 = kind == BC_DIRICHLET ? mp.c11d : mp.c11i;
#pragma unroll
      for (int c = 0; c < M; ++c) F[c] += (c11 * nn) * (uin[c] - uout[c]);
    }
  }
  if constexpr (Eq<D, EQ>::INV && WITH_INV) {
    T Fr[M];
    if (kind == BC_SLIP) {
      T um[M];
      mirror_state<D, T>(uin, nrm, um);
      roe_flux<D, T>(um, uin, nrm, mp.gamma, Fr);
    } else {
      roe_flux<D, T>(uout, uin, nrm, mp.gamma, Fr);
    }
#pragma unroll
    for (int c = 0; c < M; ++c) F[c] += Fr[c];
  }
}
}  // namespace ldg
