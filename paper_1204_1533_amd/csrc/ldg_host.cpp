// Host side of libldg: context, argument validation, C ABI entry points and
// the Newton-GMRES driver (Section 4.2 of the paper).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/ldg.h"
#include "ldg_ctx.hpp"

namespace ldg {
bool build_line_ops(int p, int node_family, LineOps& ops, std::vector<double>* nodes_out);
void build_level_order(int D, int P, LevelOrder& lv);
}

using namespace ldg;

namespace {

int64_t ipow64(int64_t b, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}

// Node index of position t on line l of direction n (host twin of line_node).
int host_line_node(int n, int l, int t, int N1) {
  int s = 1;
  for (int k = 0; k < n; ++k) s *= N1;
  return (l % s) + t * s + (l / s) * s * N1;
}
bool host_node_on_face(int node, int n, int side, int N1, int p, int* lidx) {
  int s = 1;
  for (int k = 0; k < n; ++k) s *= N1;
  int t = (node / s) % N1;
  if (t != (side ? p : 0)) return false;
  *lidx = (node % s) + (node / (s * N1)) * s;
  return true;
}

}  // namespace

extern "C" {

static void rk4_drop_graph(ldg_ctx c);

const char* ldg_status_string(ldg_status s) {
  switch (s) {
    case LDG_OK: return "ok";
    case LDG_E_INVALID: return "invalid argument";
    case LDG_E_SHAPE: return "inconsistent shape or connectivity";
    case LDG_E_UNSUPPORTED: return "unsupported configuration";
    case LDG_E_HIP: return "HIP runtime error";
    case LDG_E_NOMEM: return "out of device memory";
    case LDG_E_NOT_ASSEMBLED: return "operators not assembled";
    case LDG_E_NOT_CONVERGED: return "linear solver did not converge";
    case LDG_E_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

// Message of the last failed call without a context on this thread
// (ldg_create, ldg_assign_switches).
static thread_local std::string g_create_err;
}  // extern "C"
namespace ldg_host {
void set_host_error(const std::string& m) { g_create_err = m; }
}  // namespace ldg_host
extern "C" {

const char* ldg_last_error(ldg_ctx ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int64_t ldg_num_dofs(ldg_ctx ctx) { return ctx ? ctx->ndof : -1; }

void ldg_destroy(ldg_ctx c) {
  if (!c) return;
  void* ptrs[] = {c->d_xyz, c->d_face_nbr, c->d_nbr_node, c->d_sw, c->d_gD, c->d_gN, c->d_S, c->d_Q, c->d_W, c->d_W2,
                  c->d_K11, c->d_K12, c->d_F, c->d_Fem, c->d_Ua, c->d_Qa, c->d_V, c->d_Z, c->d_R, c->d_G, c->d_x, c->d_r, c->d_z,
                  c->d_tmp, c->d_Un, c->d_partial, c->d_h, c->d_Uold, c->d_st_Un, c->d_st_comb, c->d_st_K,
                  c->d_K21w, c->d_Dense, c->d_geo, c->d_Jwork, c->d_cwork, c->d_K21f};
  for (void* p : ptrs)
    if (p) hipFree(p);
  learned_free(c);
  rk4_drop_graph(c);
  if (c->rk_stream) hipStreamDestroy(c->rk_stream);
  for (hipEvent_t e : c->rk_ev)
    if (e) hipEventDestroy(e);
  for (auto& t : c->tm)
    for (hipEvent_t e : t.ev) hipEventDestroy(e);
  delete c;
}

ldg_status ldg_create(const ldg_problem_desc* d, void* stream, ldg_ctx* out) {
  g_create_err.clear();
  if (!out) {
    g_create_err = "null output handle";
    return LDG_E_INVALID;
  }
  *out = nullptr;
  if (!d) {
    g_create_err = "null problem description";
    return LDG_E_INVALID;
  }
  ldg_ctx c = new ldg_ctx_s();
  auto bad = [&](ldg_status s, const std::string& m) {
    g_create_err = "ldg_create: " + m + (c->err.empty() ? std::string() : " (" + c->err + ")");
    ldg_destroy(c);
    return s;
  };
  if (d->dim != 2 && d->dim != 3) return bad(LDG_E_UNSUPPORTED, "dim must be 2 or 3");
  if (d->p < 1 || d->p > 4) return bad(LDG_E_UNSUPPORTED, "p must be in 1..4");
  if (d->equation < 0 || d->equation > 2) return bad(LDG_E_UNSUPPORTED, "equation must be 0 (Poisson), 1 (Euler) or 2 (Navier-Stokes)");
  if (d->node_family != 0 && d->node_family != 1) return bad(LDG_E_INVALID, "node_family must be 0 or 1");
  if (d->n_elem < 1) return bad(LDG_E_INVALID, "n_elem must be positive");
  if (!d->node_xyz_host || !d->face_nbr_host || !d->nbr_node_host || !d->switch_plus_host)
    return bad(LDG_E_INVALID, "null mesh array");
  if (d->equation != LDG_POISSON && !(d->gamma > 1.0)) return bad(LDG_E_INVALID, "gamma must exceed 1");
  if (d->equation == LDG_NS && (d->mu < 0.0 || !(d->prandtl > 0.0))) return bad(LDG_E_INVALID, "mu must be >= 0 and prandtl > 0");
  if (d->c11_interior < 0.0 || d->c11_dirichlet < 0.0) return bad(LDG_E_INVALID, "c11 penalties must be >= 0");
  const int D = d->dim, P = d->p, N1 = P + 1;
  const int NP = (int)ipow64(N1, D), NL = (int)ipow64(N1, D - 1);
  const int64_t E = d->n_elem;
  const int M = d->equation == LDG_POISSON ? 1 : D + 2;
  // connectivity checks: neighbour index range, node range, reciprocity and switch signs
  bool any_dirichlet = false;
  for (int64_t e = 0; e < E; ++e) {
    for (int n = 0; n < D; ++n) {
      const int8_t sp = d->switch_plus_host[e * D + n];
      if (sp != 1 && sp != -1)
        return bad(LDG_E_INVALID, "switch_plus must be +-1 (element " + std::to_string(e) + ")");
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * n + s;
        const int64_t nb = d->face_nbr_host[e * 2 * D + f];
        if (nb >= E) return bad(LDG_E_SHAPE, std::string("face_nbr out of range") + " (element " + std::to_string(e) + ", face " + std::to_string(f) + ")");
        if (nb < 0) {
          const int kind = face_kind(nb);
          if (kind > BC_SLIP)
            return bad(LDG_E_UNSUPPORTED, "boundary kinds are 0 (Dirichlet), 1 (Neumann), 2 (slip wall) (element " +
                                              std::to_string(e) + ", face " + std::to_string(f) + ")");
          if (kind == BC_SLIP && d->equation == LDG_POISSON)
            return bad(LDG_E_INVALID, "a slip wall needs the Euler or Navier-Stokes equations (element " +
                                          std::to_string(e) + ", face " + std::to_string(f) + ")");
          if (kind == BC_DIRICHLET) any_dirichlet = true;
          continue;
        }
        for (int l = 0; l < NL; ++l) {
          const int nd = d->nbr_node_host[(e * 2 * D + f) * NL + l];
          if (nd < 0 || nd >= NP) return bad(LDG_E_SHAPE, std::string("nbr_node out of range") + " (element " + std::to_string(e) + ", face " + std::to_string(f) + ")");
          const int mine = host_line_node(n, l, s ? P : 0, N1);
          // find the neighbour face that holds nd and maps back to us
          bool found = false;
          for (int f2 = 0; f2 < 2 * D && !found; ++f2) {
            if (d->face_nbr_host[nb * 2 * D + f2] != e) continue;
            int l2;
            if (!host_node_on_face(nd, f2 / 2, f2 % 2, N1, P, &l2)) continue;
            if (d->nbr_node_host[(nb * 2 * D + f2) * NL + l2] != mine) continue;
            const int Smine = s ? sp : -sp;
            const int8_t sp2 = d->switch_plus_host[nb * D + f2 / 2];
            const int Sther = (f2 % 2) ? sp2 : -sp2;
            if (Smine != -Sther)
              return bad(LDG_E_SHAPE, std::string("switch signs must be opposite across a face") + " (element " + std::to_string(e) + ", face " + std::to_string(f) + ")");
            found = true;
          }
          if (!found) return bad(LDG_E_SHAPE, std::string("face connectivity is not reciprocal") + " (element " + std::to_string(e) + ", face " + std::to_string(f) + ")");
        }
      }
    }
  }
  if (any_dirichlet && !(d->c11_dirichlet > 0.0) && d->equation != LDG_EULER)
    return bad(LDG_E_INVALID, "c11_dirichlet must be positive with Dirichlet faces");
  DevCtx& dc = c->dc;
  dc.D = D;
  dc.P = P;
  dc.EQ = d->equation;
  dc.M = M;
  dc.N1 = N1;
  dc.NP = NP;
  dc.NL = NL;
  dc.NG = n_gauss(P);
  dc.E = E;
  dc.stream = (hipStream_t)stream;
  if (!build_line_ops(P, d->node_family, dc.ops, nullptr)) return bad(LDG_E_UNSUPPORTED, "1-D operators for this p");
  build_level_order(D, P, dc.lev);
  c->ndof = E * M * NP;
  c->nq = c->ndof * D;
  c->nnode = E * NP;
  ldg_status st = LDG_OK;
  if ((st = dev_alloc(c, &c->d_xyz, (size_t)E * D * NP)) != LDG_OK ||
      (st = dev_alloc(c, &c->d_face_nbr, (size_t)E * 2 * D)) != LDG_OK ||
      (st = dev_alloc(c, &c->d_nbr_node, (size_t)E * 2 * D * NL)) != LDG_OK ||
      (st = dev_alloc(c, &c->d_sw, (size_t)E * D)) != LDG_OK || (st = dev_alloc(c, &c->d_Q, (size_t)c->nq)) != LDG_OK)
    return bad(st, "device allocation of the mesh arrays");
  if (hipMemcpy(c->d_xyz, d->node_xyz_host, sizeof(double) * E * D * NP, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_face_nbr, d->face_nbr_host, sizeof(int64_t) * E * 2 * D, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_nbr_node, d->nbr_node_host, sizeof(int32_t) * E * 2 * D * NL, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(c->d_sw, d->switch_plus_host, sizeof(int8_t) * E * D, hipMemcpyHostToDevice) != hipSuccess)
    return bad(LDG_E_HIP, "copy of the mesh arrays to the device");
  MeshParams& mp = dc.mp;
  mp.E = E;
  mp.gamma = d->gamma;
  mp.mu = d->mu;
  mp.prandtl = d->prandtl > 0 ? d->prandtl : 1.0;
  mp.c11i = d->c11_interior;
  mp.c11d = d->c11_dirichlet;
  mp.xyz = c->d_xyz;
  mp.face_nbr = c->d_face_nbr;
  mp.nbr_node = c->d_nbr_node;
  mp.sw = c->d_sw;
  mp.gD = nullptr;
  mp.gN = nullptr;
  mp.S = nullptr;
  mp.c22 = 0.0;
  // Gauss-point metrics, line-end normals and -1/J: fixed by the mesh, read by
  // the residual, gradient and Jacobian kernels
  if (dev_alloc(c, &c->d_geo, jacobian_geometry_doubles(dc)) != LDG_OK)
    return bad(LDG_E_NOMEM, "device allocation of the geometry record");
  if (launch_jacobian_geometry(dc, c->d_geo) != hipSuccess) return bad(LDG_E_HIP, "geometry record");
  mp.geo = c->d_geo;
  *out = c;
  return LDG_OK;
}

ldg_status ldg_set_source(ldg_ctx c, const double* S) {
  if (!c) return LDG_E_INVALID;
  if (!S) {
    c->dc.mp.S = nullptr;
    return LDG_OK;
  }
  TRY(dev_alloc(c, &c->d_S, (size_t)c->ndof));
  HIPCK(c, hipMemcpyAsync(c->d_S, S, sizeof(double) * c->ndof, hipMemcpyDeviceToDevice, c->dc.stream));
  c->dc.mp.S = c->d_S;
  return LDG_OK;
}

ldg_status ldg_set_dirichlet(ldg_ctx c, const double* gD) {
  if (!c) return LDG_E_INVALID;
  if (!gD) {
    c->dc.mp.gD = nullptr;
    return LDG_OK;
  }
  const size_t n = (size_t)c->dc.E * 2 * c->dc.D * c->dc.M * c->dc.NL;
  TRY(dev_alloc(c, &c->d_gD, n));
  HIPCK(c, hipMemcpyAsync(c->d_gD, gD, sizeof(double) * n, hipMemcpyDeviceToDevice, c->dc.stream));
  c->dc.mp.gD = c->d_gD;
  return LDG_OK;
}

ldg_status ldg_set_neumann(ldg_ctx c, const double* gN) {
  if (!c) return LDG_E_INVALID;
  if (!gN) {
    c->dc.mp.gN = nullptr;
    return LDG_OK;
  }
  const size_t n = (size_t)c->dc.E * 2 * c->dc.D * c->dc.M * c->dc.NL;
  TRY(dev_alloc(c, &c->d_gN, n));
  HIPCK(c, hipMemcpyAsync(c->d_gN, gN, sizeof(double) * n, hipMemcpyDeviceToDevice, c->dc.stream));
  c->dc.mp.gN = c->d_gN;
  return LDG_OK;
}

ldg_status ldg_gradient(ldg_ctx c, const double* U, double* Q, int32_t homogeneous) {
  if (!c) return LDG_E_INVALID;
  if (!U || !Q) return fail(c, LDG_E_INVALID, "null pointer");
  if ((const void*)U == (const void*)Q) return fail(c, LDG_E_INVALID, "U and Q alias");
  HIPCK(c, launch_gradient(c->dc, U, Q, homogeneous != 0));
  return LDG_OK;
}

ldg_status ldg_residual(ldg_ctx c, const double* U, double* R, double* Q) {
  if (!c) return LDG_E_INVALID;
  if (!U || !R) return fail(c, LDG_E_INVALID, "null pointer");
  if ((const void*)U == (const void*)R) return fail(c, LDG_E_INVALID, "U and R alias");
  double* q = Q ? Q : c->d_Q;
  const bool vis = c->dc.EQ != LDG_EULER;
  if (vis) HIPCK(c, launch_gradient(c->dc, U, q, false));
  HIPCK(c, launch_residual(c->dc, U, vis ? q : nullptr, R));
  return LDG_OK;
}

// R_at_U: the residual at U when the caller has it (features of the learned correction)
static ldg_status assemble(ldg_ctx c, const double* U, double alpha, double gamma, int32_t prec,
                           const double* R_at_U) {
  if (!c) return LDG_E_INVALID;
  if (!U) return fail(c, LDG_E_INVALID, "null pointer");
  if (prec < 0 || prec > 2) return fail(c, LDG_E_INVALID, "storage_prec");
  if (!std::isfinite(alpha) || !std::isfinite(gamma)) return fail(c, LDG_E_INVALID, "alpha/gamma");
  const DevCtx& dc = c->dc;
  const size_t es = elem_size(prec);
  const int ns11 = dc.D * dc.P + 1 + 2 * dc.D, ns12 = dc.D * dc.P + 1 + dc.D, nsF = dc.D * dc.P + 1;
  TRY(grow(c, &c->d_K11, &c->capK11, es * (size_t)ns11 * dc.M * dc.M * c->nnode));
  TRY(grow(c, &c->d_K12, &c->capK12, es * (size_t)ns12 * dc.M * dc.M * dc.D * c->nnode));
  if (dc.EQ != LDG_EULER && !c->d_K21w) {
    // K21 = dD/dU depends on the geometry only: its weights are computed at the
    // first assembly and serve every product after it
    TRY(dev_alloc(c, &c->d_K21w, (size_t)(dc.D * dc.P + 1 + dc.D) * dc.D * c->nnode));
    HIPCK(c, launch_k21_weights(dc, c->d_K21w));
    TRY(dev_alloc(c, &c->d_K21f, (size_t)(dc.D * dc.P + 1 + dc.D) * dc.D * c->nnode));
    HIPCK(c, launch_k21_weights_f32(dc, c->d_K21w, c->d_K21f));
  }
  const int fprec = prec;
  const size_t nF = (size_t)nsF * dc.M * dc.M * c->nnode;
  // A~ is formed node-fastest in d_F (FP64 for FP64 storage, FP32 otherwise),
  // factorised in an element-major copy after it, and the factors are stored
  // in d_Fem in the apply layout (rows padded to a multiple of 4 entries)
  const size_t fbytes = (fprec == LDG_F64 ? 8 : 4) * 2 * nF;
  const size_t nFac = (size_t)dc.E * dc.NP * dc.M * ((nsF * dc.M + 3) / 4 * 4);
  TRY(grow(c, &c->d_F, &c->capF, fbytes));
  TRY(grow(c, &c->d_Fem, &c->capFem, elem_size(fprec) * nFac));
  TRY(dev_alloc(c, &c->d_Ua, (size_t)c->ndof));
  TRY(dev_alloc(c, &c->d_Qa, (size_t)c->nq));
  HIPCK(c, hipMemcpyAsync(c->d_Ua, U, sizeof(double) * c->ndof, hipMemcpyDeviceToDevice, dc.stream));
  const bool vis = dc.EQ != LDG_EULER;
  if (vis) HIPCK(c, launch_gradient(dc, U, c->d_Qa, false));
  if (!c->d_geo) {
    // Gauss-point metrics, line-end normals and -1/J: fixed by the mesh
    TRY(dev_alloc(c, &c->d_geo, jacobian_geometry_doubles(dc)));
    HIPCK(c, launch_jacobian_geometry(dc, c->d_geo));
  }
  TRY(grow(c, (void**)&c->d_Jwork, &c->capJwork, sizeof(double) * jacobian_workspace_doubles(dc)));
  HIPCK(c, launch_jacobian(dc, U, vis ? c->d_Qa : nullptr, c->d_K11, c->d_K12, prec, c->d_geo, c->d_Jwork));
  const bool block_lu = c->precond_kind == LDG_PRECOND_BLOCK_LU;
  const bool keep = !block_lu && (c->learned_collect || (c->net && c->learned_enabled));
  if (keep) TRY(dev_alloc(c, &c->d_At, nF));
  c->learned_kept = keep;
  c->learned_active = false;
  if (block_lu) {
    const size_t NR = (size_t)dc.NP * dc.M;
    TRY(grow(c, (void**)&c->d_Dense, &c->capDense, sizeof(double) * dc.E * NR * NR));
  }
  HIPCK(c, launch_precond_factor(dc, c->d_K11, c->d_K12, c->d_K21w, prec, alpha, gamma, c->d_F, fprec, c->d_Fem,
                                 keep ? c->d_At : nullptr, block_lu ? c->d_Dense : nullptr));
  c->assembled_kind = c->precond_kind;
  c->assembled = true;
  c->prec = prec;
  c->alpha = alpha;
  c->gamma = gamma;
  TRY(learned_after_form(c, R_at_U, gamma));
  return LDG_OK;
}

ldg_status ldg_jacobian_assemble(ldg_ctx c, const double* U, double alpha, double gamma, int32_t prec) {
  return assemble(c, U, alpha, gamma, prec, nullptr);
}

ldg_status ldg_set_c22(ldg_ctx c, double c22) {
  if (!c) return LDG_E_INVALID;
  if (!std::isfinite(c22) || c22 < 0.0) return fail(c, LDG_E_INVALID, "c22 must be finite and >= 0");
  if (c22 != 0.0 && c->dc.EQ != LDG_POISSON)
    return fail(c, LDG_E_UNSUPPORTED, "the coupled system with C22 != 0 is built for the Poisson equation");
  c->dc.mp.c22 = c22;
  return LDG_OK;
}

ldg_status ldg_set_preconditioner(ldg_ctx c, int32_t kind) {
  if (!c) return LDG_E_INVALID;
  if (kind != LDG_PRECOND_BILU0 && kind != LDG_PRECOND_BLOCK_LU) return fail(c, LDG_E_INVALID, "preconditioner kind");
  if (kind == LDG_PRECOND_BLOCK_LU && c->dc.NP * c->dc.M > 768)
    return fail(c, LDG_E_UNSUPPORTED, "block LU needs Np m <= 768");
  if (kind != c->precond_kind) c->assembled = false;  // the factors must be rebuilt
  c->precond_kind = kind;
  return LDG_OK;
}

}  // extern "C"

namespace ldg_host {
// y = (alpha I - gamma A) x with w = K21 x held in W (nq doubles, unused for Euler).
ldg_status apply_op_with(ldg_ctx c, const double* x, double* y, bool exact, double* W) {
  const DevCtx& dc = c->dc;
  const bool vis = dc.EQ != LDG_EULER;
  if (vis) {
    Span sp(c, 1);
    // the stored low-precision operator takes the FP32 weights; FP64 storage and
    // the exact tangent the FP64 ones
    if (c->d_K21f && !exact && c->prec != LDG_F64)
      HIPCK(c, launch_k21_apply_f32(dc, c->d_K21f, x, W));
    else if (c->d_K21w)
      HIPCK(c, launch_k21_apply(dc, c->d_K21w, x, W));
    else
      HIPCK(c, launch_gradient(dc, x, W, true));
  }
  if (exact) {
    // y = alpha x - gamma dR/dU x  (tangent of the FP64 residual at the assembled state)
    HIPCK(c, launch_residual_tangent(dc, c->d_Ua, x, vis ? c->d_Qa : nullptr, vis ? W : nullptr, y));
    HIPCK(c, launch_axpby(y, c->alpha, x, -c->gamma, c->ndof, dc.stream));
  } else {
    Span sp(c, 0);
    HIPCK(c, launch_jacvec(dc, c->d_K11, c->d_K12, c->prec, c->alpha, c->gamma, x, vis ? W : nullptr, y));
  }
  return LDG_OK;
}
}  // namespace ldg_host

extern "C" {

static ldg_status apply_op(ldg_ctx c, const double* x, double* y, bool exact) {
  TRY(dev_alloc(c, &c->d_W, (size_t)c->nq));
  return apply_op_with(c, x, y, exact, c->d_W);
}

ldg_status ldg_jacvec(ldg_ctx c, const double* x, double* y, int32_t exact) {
  if (!c) return LDG_E_INVALID;
  if (!x || !y) return fail(c, LDG_E_INVALID, "null pointer");
  if ((const void*)x == (const void*)y) return fail(c, LDG_E_INVALID, "x and y alias");
  if (!c->assembled) return fail(c, LDG_E_NOT_ASSEMBLED, "call ldg_jacobian_assemble first");
  return apply_op(c, x, y, exact != 0);
}

ldg_status ldg_precond_apply(ldg_ctx c, const double* r, double* z) {
  if (!c) return LDG_E_INVALID;
  if (!r || !z) return fail(c, LDG_E_INVALID, "null pointer");
  if ((const void*)r == (const void*)z) return fail(c, LDG_E_INVALID, "r and z alias");
  if (!c->assembled) return fail(c, LDG_E_NOT_ASSEMBLED, "call ldg_jacobian_assemble first");
  return precond_apply_any(c, r, z);
}

ldg_status ldg_export_operators(ldg_ctx c, double* K11, double* K12, double* F) {
  if (!c) return LDG_E_INVALID;
  if (!c->assembled) return fail(c, LDG_E_NOT_ASSEMBLED, "call ldg_jacobian_assemble first");
  const DevCtx& dc = c->dc;
  const int ns11 = dc.D * dc.P + 1 + 2 * dc.D, ns12 = dc.D * dc.P + 1 + dc.D;
  if (K11) HIPCK(c, launch_export_blocks(dc, c->d_K11, c->prec, ns11, dc.M, K11));
  if (K12) HIPCK(c, launch_export_blocks(dc, c->d_K12, c->prec, ns12, dc.M * dc.D, K12));
  if (F && c->assembled_kind == LDG_PRECOND_BLOCK_LU)
    return fail(c, LDG_E_UNSUPPORTED, "F: the preconditioner is the dense element-block LU");
  if (F) HIPCK(c, launch_factors_to_f64(dc, c->d_Fem, c->prec, F));
  return LDG_OK;
}

// ------------------------------------------------------------------ Krylov helpers
// V_j . w for j < k (columns of length n, stored one after another), to the host
static ldg_status dots(ldg_ctx c, int64_t n, const double* V, int k, const double* w, double* host_out) {
  const DevCtx& dc = c->dc;
  // one block per 1024 entries (four per thread), at most nblk_dot: small systems
  // then reduce over a few blocks instead of many nearly empty ones
  const int nb = (int)std::min<int64_t>(c->nblk_dot, std::max<int64_t>(1, (n + 1023) / 1024));
  HIPCK(c, launch_multidot(V, n, k, w, n, c->d_partial, nb, dc.stream));
  HIPCK(c, launch_multidot_finish(c->d_partial, nb, k, c->d_h, dc.stream));
  HIPCK(c, hipMemcpyAsync(host_out, c->d_h, sizeof(double) * k, hipMemcpyDeviceToHost, dc.stream));
  HIPCK(c, hipStreamSynchronize(dc.stream));
  return LDG_OK;
}

static ldg_status norm2(ldg_ctx c, int64_t n, const double* w, double* out) {
  double v;
  TRY(dots(c, n, w, 1, w, &v));
  *out = std::sqrt(v);
  return LDG_OK;
}

// A linear system for GMRES: vectors of length n, the operator, the
// preconditioner, and the work space (V: restart + 1 columns, Z: restart
// columns, r and tmp: one each).
struct KrylovSystem {
  int64_t n;
  double *V, *Z, *r, *tmp;
  std::function<ldg_status(const double*, double*)> op, prec;
};

// Right-preconditioned GMRES(restart) on A x = b, x0 = 0, classical
// Gram-Schmidt with a selective second pass.  true_res: end with the true
// residual ||b - A x|| in *est_res (else the Arnoldi estimate; the refinement
// loop computes the exact residual itself).
static ldg_status gmres_on(ldg_ctx c, const KrylovSystem& K, const double* b, double* x, double rtol_abs, int restart,
                           int max_iters, int* iters, double* est_res, bool true_res) {
  const DevCtx& dc = c->dc;
  const int64_t n = K.n;
  HIPCK(c, hipMemsetAsync(x, 0, sizeof(double) * n, dc.stream));
  std::vector<double> H((restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), h(restart + 1),
      h2(restart + 1), y(restart);
  int its = 0;
  double beta;
  // r = b - A x
  HIPCK(c, hipMemcpyAsync(K.r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, dc.stream));
  bool first = true;
  while (true) {
    if (!first) {
      TRY(K.op(x, K.tmp));
      HIPCK(c, hipMemcpyAsync(K.r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, dc.stream));
      HIPCK(c, launch_axpby(K.r, -1.0, K.tmp, 1.0, n, dc.stream));
    }
    first = false;
    TRY(norm2(c, n, K.r, &beta));
    *est_res = beta;
    if (!std::isfinite(beta)) return fail(c, LDG_E_NONFINITE, "non-finite GMRES residual");
    if (beta <= rtol_abs || its >= max_iters) break;
    HIPCK(c, hipMemcpyAsync(K.V, K.r, sizeof(double) * n, hipMemcpyDeviceToDevice, dc.stream));
    HIPCK(c, launch_axpby(K.V, 0.0, K.r, 1.0 / beta, n, dc.stream));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k_used = 0;
    for (int k = 0; k < restart; ++k) {
      double* vk = K.V + (int64_t)k * n;
      double* w = K.V + (int64_t)(k + 1) * n;
      double* zk = K.Z + (int64_t)k * n;  // z_k = P^{-1} v_k is kept for the update of x
      TRY(K.prec(vk, zk));
      TRY(K.op(zk, w));
      // Classical Gram-Schmidt, repeated once when the projection removed more
      // than half of |w|^2 (the Daniel-Gragg-Kaufman-Stewart criterion with
      // eta = 1/sqrt 2).  w = V_{k+1} follows V_k in memory, so one pass gives
      // V_j . w (j <= k) and w . w; with V orthonormal, |w - V h|^2 = w.w - |h|^2,
      // and the normalisation is folded into the update.
      double hn = 0.0;
      bool done = false;
      std::fill(h2.begin(), h2.end(), 0.0);
      for (int pass = 0; pass < 2 && !done; ++pass) {
        double* hp = pass == 0 ? h.data() : h2.data();
        TRY(dots(c, n, K.V, k + 2, w, hp));
        double hh = 0.0;
        for (int j = 0; j <= k; ++j) hh += hp[j] * hp[j];
        const double ww = hp[k + 1], rest = ww - hh;
        HIPCK(c, hipMemcpyAsync(c->d_h, hp, sizeof(double) * (k + 1), hipMemcpyHostToDevice, dc.stream));
        if (rest > 0.5 * ww) {
          hn = std::sqrt(rest);
          HIPCK(c, launch_update(w, K.V, n, k + 1, c->d_h, n, dc.stream, 1.0 / hn));
          done = true;
        } else {
          HIPCK(c, launch_update(w, K.V, n, k + 1, c->d_h, n, dc.stream));
        }
      }
      if (!done) {
        // near breakdown (or non-finite values): the norm is taken explicitly
        TRY(norm2(c, n, w, &hn));
        if (hn > 0 && std::isfinite(hn)) HIPCK(c, launch_axpby(w, 0.0, w, 1.0 / hn, n, dc.stream));
      }
      for (int j = 0; j <= k; ++j) H[j * restart + k] = h[j] + h2[j];
      H[(k + 1) * restart + k] = hn;
      if (!std::isfinite(hn)) return fail(c, LDG_E_NONFINITE, "non-finite Arnoldi vector");
      for (int j = 0; j < k; ++j) {
        double t = cs[j] * H[j * restart + k] + sn[j] * H[(j + 1) * restart + k];
        H[(j + 1) * restart + k] = -sn[j] * H[j * restart + k] + cs[j] * H[(j + 1) * restart + k];
        H[j * restart + k] = t;
      }
      double den = std::hypot(H[k * restart + k], H[(k + 1) * restart + k]);
      cs[k] = H[k * restart + k] / den;
      sn[k] = H[(k + 1) * restart + k] / den;
      H[k * restart + k] = den;
      H[(k + 1) * restart + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      ++its;
      k_used = k + 1;
      *est_res = std::fabs(g[k + 1]);
      if (std::fabs(g[k + 1]) <= rtol_abs || its >= max_iters || hn == 0.0) break;
    }
    c->krylov_avail = k_used;
    for (int i = k_used - 1; i >= 0; --i) {
      double s = g[i];
      for (int j = i + 1; j < k_used; ++j) s -= H[i * restart + j] * y[j];
      y[i] = s / H[i * restart + i];
    }
    // x += P^{-1} (V y) = Z y  (P^{-1} is linear and the z_k were kept)
    HIPCK(c, hipMemcpyAsync(c->d_h, y.data(), sizeof(double) * k_used, hipMemcpyHostToDevice, dc.stream));
    HIPCK(c, launch_lincomb(x, K.Z, n, k_used, c->d_h, n, dc.stream));
    if ((*est_res <= rtol_abs || its >= max_iters) && !true_res) break;
    if (*est_res <= rtol_abs || its >= max_iters) {
      // true residual for the report
      TRY(K.op(x, K.tmp));
      HIPCK(c, hipMemcpyAsync(K.r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, dc.stream));
      HIPCK(c, launch_axpby(K.r, -1.0, K.tmp, 1.0, n, dc.stream));
      TRY(norm2(c, n, K.r, est_res));
      break;
    }
  }
  *iters = its;
  return LDG_OK;
}

// GMRES on the Newton system (alpha I - gamma A) x = b: the stored split
// product (exact = false) or the exact tangent (exact = true), preconditioned
// by the assembled preconditioner.
static ldg_status gmres(ldg_ctx c, const double* b, double* x, double rtol_abs, int restart, int max_iters,
                        bool exact, int* iters, double* est_res, bool true_res = true) {
  KrylovSystem K;
  K.n = c->ndof;
  K.V = c->d_V;
  K.Z = c->d_Z;
  K.r = c->d_r;
  K.tmp = c->d_tmp;
  K.op = [c, exact](const double* in, double* out) { return apply_op(c, in, out, exact); };
  K.prec = [c](const double* in, double* out) {
    Span sp(c, 2);
    return precond_apply_any(c, in, out);
  };
  return gmres_on(c, K, b, x, rtol_abs, restart, max_iters, iters, est_res, true_res);
}

static ldg_status ensure_krylov(ldg_ctx c, int restart) {
  const int64_t n = c->ndof;
  if (restart < 1 || restart > 120) return fail(c, LDG_E_INVALID, "restart must be in 1..120");
  if (c->cap_restart < restart) {
    if (c->d_V) hipFree(c->d_V);
    if (c->d_Z) hipFree(c->d_Z);
    c->d_V = nullptr;
    c->d_Z = nullptr;
    c->cap_restart = 0;
    TRY(dev_alloc(c, &c->d_V, (size_t)(restart + 1) * n));
    TRY(dev_alloc(c, &c->d_Z, (size_t)restart * n));
    c->cap_restart = restart;
  }
  TRY(dev_alloc(c, &c->d_R, (size_t)n));
  TRY(dev_alloc(c, &c->d_G, (size_t)n));
  TRY(dev_alloc(c, &c->d_x, (size_t)n));
  TRY(dev_alloc(c, &c->d_r, (size_t)n));
  TRY(dev_alloc(c, &c->d_z, (size_t)n));
  TRY(dev_alloc(c, &c->d_tmp, (size_t)n));
  TRY(dev_alloc(c, &c->d_Un, (size_t)n));
  c->nblk_dot = 1024;
  TRY(dev_alloc(c, &c->d_partial, (size_t)c->nblk_dot * 128));
  TRY(dev_alloc(c, &c->d_h, (size_t)128));
  return LDG_OK;
}

// Steady solve of the coupled (U, Q) system of a linear problem:
// F(U, Q) = [-R(U, Q); Q - G(U, Q)] = 0 with G the gradient whose trace
// carries the C22 jump.  Flexible GMRES on A [U; Q] = -F(0) with
//   A [xU; xQ] = [-R_h(xU, xQ); xQ - G_h(xU, xQ)]        (h: no source, no boundary data),
// preconditioned by an approximate inverse of the C22 = 0 matrix
// A0 = [[-K11, -K12], [-K21, I]]: zU solves S zU = rU + K12 rQ with
// S = -(K11 + K12 K21) by inner GMRES (the reduced system's operator and
// element-block preconditioner) to inner_rtol, and zQ = rQ + K21 zU.  The
// inner solve is needed: with zU = P^{-1} (rU + K12 rQ) for the element-block
// P alone, the C22 coupling of neighbouring Q leaves A M^{-1} with eigenvalues
// far in the left half plane and the iteration stalls.  The outer iteration
// keeps z_k = M^{-1} v_k, so a preconditioner that changes from one
// application to the next is allowed.
static ldg_status coupled_solve(ldg_ctx c, double* U, double* Q, double rtol, double inner_rtol, int restart,
                                int max_iters, int* iters, int* inner_iters, double* relres) {
  const DevCtx& dc = c->dc;
  const int64_t nu = c->ndof, nq = c->nq, N = nu + nq;
  TRY(ensure_krylov(c, restart));  // the inner solves use the reduced system's Krylov space
  // work: V (restart + 1) N, Z restart N, r, tmp, b, x (N each), zero (N), t (nu)
  const size_t need = (size_t)(2 * restart + 6) * N + nu;
  TRY(grow(c, (void**)&c->d_cwork, &c->cap_cwork, sizeof(double) * need));
  double* V = c->d_cwork;
  double* Z = V + (size_t)(restart + 1) * N;
  double* r = Z + (size_t)restart * N;
  double* tmp = r + N;
  double* b = tmp + N;
  double* x = b + N;
  double* zero = x + N;
  double* t = zero + N;
  HIPCK(c, hipMemsetAsync(zero, 0, sizeof(double) * N, dc.stream));
  // K11, K12, K21 weights and the preconditioner of S: alpha = 0, gamma = 1
  TRY(assemble(c, zero, 0.0, 1.0, LDG_F64, nullptr));
  // b = -F(0) = [R(0, 0); G(0, 0)]
  HIPCK(c, launch_residual(dc, zero, zero + nu, b));
  HIPCK(c, launch_gradient(dc, zero, b + nu, false, zero + nu));
  DevCtx dh = dc;
  dh.mp.S = nullptr;
  dh.mp.gD = nullptr;
  dh.mp.gN = nullptr;
  KrylovSystem K;
  K.n = N;
  K.V = V;
  K.Z = Z;
  K.r = r;
  K.tmp = tmp;
  K.op = [c, dh, nu, nq](const double* in, double* out) -> ldg_status {
    HIPCK(c, launch_residual(dh, in, in + nu, out));
    HIPCK(c, launch_axpby(out, 0.0, out, -1.0, nu, dh.stream));
    HIPCK(c, launch_gradient(dh, in, out + nu, true, in + nu));
    HIPCK(c, launch_axpby(out + nu, 1.0, in + nu, -1.0, nq, dh.stream));
    return LDG_OK;
  };
  int inner_total = 0;
  K.prec = [c, nu, nq, zero, t, inner_rtol, restart, &inner_total](const double* in, double* out) -> ldg_status {
    const DevCtx& d = c->dc;
    // t = rU + K12 rQ (the split product with alpha = 0, gamma = 1 and x = 0 gives -K12 rQ)
    HIPCK(c, launch_jacvec(d, c->d_K11, c->d_K12, LDG_F64, 0.0, 1.0, zero, in + nu, t));
    HIPCK(c, launch_axpby(t, 1.0, in, -1.0, nu, d.stream));
    double tn = 0.0, est = 0.0;
    TRY(norm2(c, nu, t, &tn));
    int its = 0;
    if (tn > 0.0) {
      TRY(gmres(c, t, out, inner_rtol * tn, restart, restart, false, &its, &est, false));
    } else {
      HIPCK(c, hipMemsetAsync(out, 0, sizeof(double) * nu, d.stream));
    }
    inner_total += its;
    HIPCK(c, launch_k21_apply(d, c->d_K21w, out, out + nu));
    HIPCK(c, launch_axpby(out + nu, 1.0, in + nu, 1.0, nq, d.stream));
    return LDG_OK;
  };
  double bn = 0.0, res = 0.0;
  TRY(norm2(c, N, b, &bn));
  if (!std::isfinite(bn)) return fail(c, LDG_E_NONFINITE, "non-finite right-hand side");
  int its = 0;
  if (bn == 0.0) {
    HIPCK(c, hipMemsetAsync(x, 0, sizeof(double) * N, dc.stream));
  } else {
    const ldg_status st = gmres_on(c, K, b, x, rtol * bn, restart, max_iters, &its, &res, true);
    c->krylov_avail = 0;  // the Arnoldi vectors left are those of an inner solve
    TRY(st);
  }
  HIPCK(c, hipMemcpyAsync(U, x, sizeof(double) * nu, hipMemcpyDeviceToDevice, dc.stream));
  HIPCK(c, hipMemcpyAsync(Q, x + nu, sizeof(double) * nq, hipMemcpyDeviceToDevice, dc.stream));
  HIPCK(c, hipStreamSynchronize(dc.stream));
  *iters = its;
  *inner_iters = inner_total;
  *relres = bn > 0 ? res / bn : 0.0;
  if (bn > 0 && !(res <= rtol * bn)) return fail(c, LDG_E_NOT_CONVERGED, "coupled GMRES did not reach rtol");
  return LDG_OK;
}

ldg_status ldg_coupled_solve(ldg_ctx c, double* U, double* Q, double rtol, double inner_rtol, int32_t restart,
                             int32_t max_iters, int32_t* iters, int32_t* inner_iters, double* relres) {
  if (!c) return LDG_E_INVALID;
  if (!U || !Q) return fail(c, LDG_E_INVALID, "null pointer");
  if ((const void*)U == (const void*)Q) return fail(c, LDG_E_INVALID, "U and Q alias");
  if (c->dc.EQ != LDG_POISSON) return fail(c, LDG_E_UNSUPPORTED, "the coupled solve is built for the Poisson equation");
  if (!(rtol > 0.0) || !(inner_rtol > 0.0) || !(inner_rtol < 1.0) || restart < 1 || restart > 120 || max_iters < 1)
    return fail(c, LDG_E_INVALID, "rtol > 0, 0 < inner_rtol < 1, restart in 1..120, max_iters >= 1");
  int its = 0, inner = 0;
  double rr = 0.0;
  const ldg_status st = coupled_solve(c, U, Q, rtol, inner_rtol, restart, max_iters, &its, &inner, &rr);
  if (iters) *iters = its;
  if (inner_iters) *inner_iters = inner;
  if (relres) *relres = rr;
  return st;
}

// G(U) = alpha (U - Ucomb) - gamma R(U) into G (R(U) into d_R) and ||G||_2.
static ldg_status eval_G(ldg_ctx c, const double* U, const double* Ucomb, double alpha, double gamma, double* G,
                         double* gnorm) {
  const DevCtx& dc = c->dc;
  const int64_t n = c->ndof;
  TRY(ldg_residual(c, U, c->d_R, nullptr));
  HIPCK(c, launch_copy(G, U, n, dc.stream));
  if (Ucomb) HIPCK(c, launch_axpby(G, -1.0, Ucomb, 1.0, n, dc.stream));
  HIPCK(c, launch_axpby(G, -gamma, c->d_R, alpha, n, dc.stream));
  TRY(norm2(c, c->ndof, G, gnorm));
  return LDG_OK;
}

// Internal controls of one Newton iteration (the public ldg_newton_step uses
// the defaults; the time-step driver sets them).
struct NewtonCtl {
  bool G_current = false;       // d_R = R(U) and d_G = G(U) already hold on entry
  bool accept_inexact = false;  // update U even when the linear solve stops short of rtol
  bool refine = true;           // FP64 refinement around low-precision storage
  bool true_res = true;         // end the (unrefined) GMRES with the true residual
};

// Solves (alpha I - gamma A) x = b with b = d_G into d_x: plain GMRES on the
// stored operator (FP64 storage, or no refinement asked), otherwise FP64
// iterative refinement with the exact tangent around GMRES on the stored one.
static ldg_status linear_solve(ldg_ctx c, const ldg_solver_opts* o, const NewtonCtl& ctl, double bnorm,
                               int* total_its, int* sweeps_out, double* res_out, bool* ok_out) {
  const DevCtx& dc = c->dc;
  const int64_t n = c->ndof;
  const double target = o->rtol * bnorm;
  if (c->prec == LDG_F64 || !ctl.refine) {
    int its;
    double res;
    TRY(gmres(c, c->d_G, c->d_x, target, o->restart, o->max_iters, false, &its, &res, ctl.true_res));
    *total_its = its;
    *sweeps_out = 0;
    *res_out = res;
    *ok_out = res <= target;
    return LDG_OK;
  }
  TRY(dev_alloc(c, &c->d_Un, (size_t)n));
  double* xacc = c->d_Un;  // accumulated correction
  HIPCK(c, hipMemsetAsync(xacc, 0, sizeof(double) * n, dc.stream));
  double* rr = c->d_R;  // refinement residual (R(U) is not needed any more)
  HIPCK(c, hipMemcpyAsync(rr, c->d_G, sizeof(double) * n, hipMemcpyDeviceToDevice, dc.stream));
  double rn = bnorm;
  const int max_ref = o->max_refine > 0 ? o->max_refine : 10;
  const double inner = o->inner_rtol > 0 ? o->inner_rtol : 1e-3;
  int sweeps = 0, tot = 0;
  bool ok = false;
  for (; sweeps < max_ref; ++sweeps) {
    int its;
    double est;
    TRY(gmres(c, rr, c->d_x, inner * rn, o->restart, o->max_iters - tot, false, &its, &est, false));
    tot += its;
    HIPCK(c, launch_axpby(xacc, 1.0, c->d_x, 1.0, n, dc.stream));
    // exact residual rr = b - (alpha I - gamma A) xacc
    TRY(apply_op(c, xacc, c->d_tmp, true));
    HIPCK(c, hipMemcpyAsync(rr, c->d_G, sizeof(double) * n, hipMemcpyDeviceToDevice, dc.stream));
    HIPCK(c, launch_axpby(rr, -1.0, c->d_tmp, 1.0, n, dc.stream));
    TRY(norm2(c, c->ndof, rr, &rn));
    if (!std::isfinite(rn)) return fail(c, LDG_E_NONFINITE, "non-finite refinement residual");
    if (rn <= target) {
      ++sweeps;
      ok = true;
      break;
    }
    if (tot >= o->max_iters) {
      ++sweeps;
      break;
    }
  }
  HIPCK(c, hipMemcpyAsync(c->d_x, xacc, sizeof(double) * n, hipMemcpyDeviceToDevice, dc.stream));
  *total_its = tot;
  *sweeps_out = sweeps;
  *res_out = rn;
  *ok_out = ok;
  return LDG_OK;
}

// One Newton iteration on G(U) = alpha (U - Ucomb) - gamma R(U).  On return
// after an update, d_R = R(U_new) and d_G = G(U_new).
static ldg_status newton_core(ldg_ctx c, double* U, const double* Ucomb, double alpha, double gamma,
                              const ldg_solver_opts* o, ldg_solver_report* rep, const NewtonCtl& ctl) {
  if (!c) return LDG_E_INVALID;
  if (!U || !o) return fail(c, LDG_E_INVALID, "null pointer");
  if (!(o->rtol > 0) || o->max_iters < 1 || o->storage_prec < 0 || o->storage_prec > 2)
    return fail(c, LDG_E_INVALID, "solver options: need rtol > 0, max_iters >= 1, storage_prec in 0..2");
  if (!std::isfinite(alpha) || !std::isfinite(gamma)) return fail(c, LDG_E_INVALID, "alpha/gamma");
  if (o->use_learned && !c->net) return fail(c, LDG_E_INVALID, "use_learned without an attached network");
  if ((const void*)U == (const void*)Ucomb) return fail(c, LDG_E_INVALID, "U and Ucomb alias");
  const DevCtx& dc = c->dc;
  const int64_t n = c->ndof;
  ldg_solver_report r{};
  TRY(ensure_krylov(c, o->restart));
  c->timing = rep != nullptr;
  for (auto& t : c->tm) t.used = 0;
  hipEvent_t ev[5];
  for (auto& e : ev) HIPCK(c, hipEventCreate(&e));
  auto t_start = std::chrono::steady_clock::now();
  HIPCK(c, hipEventRecord(ev[0], dc.stream));
  double g0;
  if (ctl.G_current)
    TRY(norm2(c, c->ndof, c->d_G, &g0));
  else
    TRY(eval_G(c, U, Ucomb, alpha, gamma, c->d_G, &g0));
  HIPCK(c, hipEventRecord(ev[1], dc.stream));
  r.newton_res_before = g0;
  if (!std::isfinite(g0)) return fail(c, LDG_E_NONFINITE, "non-finite Newton residual");
  const bool reassemble = o->reassemble || !c->assembled || c->alpha != alpha || c->gamma != gamma ||
                          c->prec != o->storage_prec;
  if (reassemble) {
    c->learned_enabled = c->net && o->use_learned;
    TRY(assemble(c, U, alpha, gamma, o->storage_prec, c->d_R));
    c->n_assemblies++;
  }
  r.fallback_used = c->learned_fallback;
  HIPCK(c, hipEventRecord(ev[2], dc.stream));
  // b = -G  (kept in d_G during the solve)
  HIPCK(c, launch_axpby(c->d_G, 0.0, c->d_G, -1.0, n, dc.stream));
  int its = 0, sweeps = 0;
  double res = 0.0;
  bool ok = false;
  TRY(linear_solve(c, o, ctl, g0, &its, &sweeps, &res, &ok));
  r.gmres_iters = its;
  // the learned correction is judged by the outcome: a solve that misses the
  // tolerance is repeated with the plain BILU(0) factors
  if (!ok && c->learned_active) {
    c->learned_active = false;
    c->learned_fallback = 1;
    r.fallback_used = 1;
    TRY(linear_solve(c, o, ctl, g0, &its, &sweeps, &res, &ok));
    r.gmres_iters += its;
  }
  HIPCK(c, hipEventRecord(ev[3], dc.stream));
  r.refine_steps = sweeps;
  r.lin_relres = g0 > 0 ? res / g0 : 0.0;
  r.converged = ok ? 1 : 0;
  const bool update = ok || ctl.accept_inexact;
  if (update) {
    TRY(dev_alloc(c, &c->d_Uold, (size_t)n));
    HIPCK(c, launch_copy(c->d_Uold, U, n, dc.stream));
    HIPCK(c, launch_axpby(U, 1.0, c->d_x, 1.0, n, dc.stream));
    double g1;
    TRY(eval_G(c, U, Ucomb, alpha, gamma, c->d_tmp, &g1));
    if (c->learned_active && !(g1 < g0)) {
      // the corrected step did not lower ||G||: undo it and solve again with plain BILU(0)
      c->learned_active = false;
      c->learned_fallback = 1;
      r.fallback_used = 1;
      HIPCK(c, launch_copy(U, c->d_Uold, n, dc.stream));
      TRY(linear_solve(c, o, ctl, g0, &its, &sweeps, &res, &ok));
      r.gmres_iters += its;
      r.refine_steps = sweeps;
      r.lin_relres = g0 > 0 ? res / g0 : 0.0;
      r.converged = ok ? 1 : 0;
      if (ok || ctl.accept_inexact) {
        HIPCK(c, launch_axpby(U, 1.0, c->d_x, 1.0, n, dc.stream));
        TRY(eval_G(c, U, Ucomb, alpha, gamma, c->d_tmp, &g1));
      } else {
        g1 = g0;
      }
    }
    r.newton_res_after = g1;
    HIPCK(c, launch_copy(c->d_G, c->d_tmp, n, dc.stream));
  } else {
    r.newton_res_after = g0;
  }
  HIPCK(c, hipEventRecord(ev[4], dc.stream));
  HIPCK(c, hipEventSynchronize(ev[4]));
  float ms;
  hipEventElapsedTime(&ms, ev[0], ev[1]);
  r.t_resid_ms = ms;
  hipEventElapsedTime(&ms, ev[1], ev[2]);
  r.t_assemble_ms = ms;
  hipEventElapsedTime(&ms, ev[2], ev[3]);
  r.t_solve_ms = ms;
  r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  double* tot[3] = {&r.t_jacvec_ms, &r.t_k21_ms, &r.t_precond_ms};
  int32_t* cnt[3] = {&r.n_jacvec, &r.n_k21, &r.n_precond};
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (size_t i = 0; i + 1 < c->tm[k].used; i += 2) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, c->tm[k].ev[i], c->tm[k].ev[i + 1]) == hipSuccess) acc += t;
    }
    *tot[k] = acc;
    *cnt[k] = (int32_t)(c->tm[k].used / 2);
  }
  c->timing = false;
  for (auto& e : ev) hipEventDestroy(e);
  if (rep) *rep = r;
  if (!update) return fail(c, LDG_E_NOT_CONVERGED, "linear solve did not reach rtol");
  return LDG_OK;
}

ldg_status ldg_newton_step(ldg_ctx c, double* U, const double* Ucomb, double alpha, double gamma,
                           const ldg_solver_opts* o, ldg_solver_report* rep) {
  return newton_core(c, U, Ucomb, alpha, gamma, o, rep, NewtonCtl{});
}

// ------------------------------------------------------------------ implicit time steps
// Alexander's L-stable three-stage DIRK (Section 4.1): diagonal alpha, c_2 = tau_2.
static const double kDirkAlpha = 0.435866521508459;

ldg_status ldg_implicit_step(ldg_ctx c, double* U, double* Uprev, double dt, const ldg_step_opts* so,
                             const ldg_solver_opts* lo, ldg_step_report* rep) {
  if (!c) return LDG_E_INVALID;
  if (!U || !so || !lo) return fail(c, LDG_E_INVALID, "null pointer");
  if (so->scheme < LDG_BDF2 || so->scheme > LDG_BACKWARD_EULER) return fail(c, LDG_E_INVALID, "scheme");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(c, LDG_E_INVALID, "dt must be positive and finite");
  if (so->max_newton < 1) return fail(c, LDG_E_INVALID, "max_newton must be >= 1");
  if (!(so->newton_rtol >= 0) || !(so->newton_atol >= 0))
    return fail(c, LDG_E_INVALID, "need newton_rtol >= 0 and newton_atol >= 0");
  const bool fixed = so->newton_rtol == 0 && so->newton_atol == 0;  // exactly max_newton iterations
  if (so->gmres_per_newton < 0) return fail(c, LDG_E_INVALID, "gmres_per_newton must be >= 0");
  if ((const void*)U == (const void*)Uprev) return fail(c, LDG_E_INVALID, "U and Uprev alias");
  const DevCtx& dc = c->dc;
  const int64_t n = c->ndof;
  auto t_start = std::chrono::steady_clock::now();
  TRY(ensure_krylov(c, lo->restart));
  TRY(dev_alloc(c, &c->d_st_Un, (size_t)n));
  TRY(dev_alloc(c, &c->d_st_comb, (size_t)n));
  TRY(dev_alloc(c, &c->d_st_K, (size_t)2 * n));
  double* Un = c->d_st_Un;
  double* comb = c->d_st_comb;
  double* dK1 = c->d_st_K;  // dt K_1 (DIRK)
  double* dK2 = c->d_st_K + n;
  HIPCK(c, launch_copy(Un, U, n, dc.stream));
  ldg_step_report r{};
  // linear solves: a fixed number of GMRES iterations per Newton iteration
  // (the stored operator, no refinement: the FP64 Newton residual corrects
  // it), or GMRES to lo->rtol as in ldg_newton_step
  ldg_solver_opts lin = *lo;
  NewtonCtl ctl;
  ctl.accept_inexact = true;
  if (so->gmres_per_newton > 0) {
    lin.max_iters = so->gmres_per_newton;
    lin.restart = lo->restart > so->gmres_per_newton ? so->gmres_per_newton : lo->restart;
    ctl.refine = false;
    ctl.true_res = false;
  }
  const int nstage = so->scheme == LDG_DIRK3 ? 3 : 1;
  double gamma;
  if (so->scheme == LDG_BDF2)
    gamma = 2.0 * dt / 3.0;
  else if (so->scheme == LDG_BACKWARD_EULER)
    gamma = dt;
  else
    gamma = kDirkAlpha * dt;
  const double a = kDirkAlpha, tau2 = 0.5 * (1.0 + a);
  const double b1 = -(6 * a * a - 16 * a + 1) / 4, b2 = (6 * a * a - 20 * a + 5) / 4;
  const int n_asm0 = c->n_assemblies;
  bool all_ok = true;
  for (int st = 0; st < nstage && all_ok; ++st) {
    // Ucomb of the stage: the explicit part of the stage equation
    if (so->scheme == LDG_BDF2) {
      // (4 U^n - U^{n-1}) / 3, with U^{n-1} = U^n when no history is given
      HIPCK(c, launch_copy(comb, Un, n, dc.stream));
      if (Uprev) {
        HIPCK(c, launch_axpby(comb, -1.0 / 3.0, Uprev, 4.0 / 3.0, n, dc.stream));
      }
    } else if (so->scheme == LDG_BACKWARD_EULER || st == 0) {
      HIPCK(c, launch_copy(comb, Un, n, dc.stream));
    } else if (st == 1) {
      HIPCK(c, launch_copy(comb, Un, n, dc.stream));
      HIPCK(c, launch_axpby(comb, tau2 - a, dK1, 1.0, n, dc.stream));
    } else {
      HIPCK(c, launch_copy(comb, Un, n, dc.stream));
      HIPCK(c, launch_axpby(comb, b1, dK1, 1.0, n, dc.stream));
      HIPCK(c, launch_axpby(comb, b2, dK2, 1.0, n, dc.stream));
    }
    // Newton iterations on Y - Ucomb - gamma F(Y) = 0 starting from the current U
    double g_first = 0.0, g = 0.0;
    TRY(eval_G(c, U, comb, 1.0, gamma, c->d_G, &g_first));
    if (!std::isfinite(g_first)) {
      c->err = "non-finite residual at the start of stage " + std::to_string(st + 1);
      all_ok = false;
      break;
    }
    g = g_first;
    const double tol = std::max(so->newton_rtol * g_first, so->newton_atol);
    int k = 0, since = 0;
    bool conv = !fixed && g <= tol;
    while (!conv && k < so->max_newton) {
      lin.reassemble = (!so->reuse) || (so->reassemble_after > 0 && since >= so->reassemble_after) ? 1 : 0;
      if (lin.reassemble) since = 0;
      ldg_solver_report nr{};
      ctl.G_current = true;
      ldg_status s = newton_core(c, U, comb, 1.0, gamma, &lin, &nr, ctl);
      if (s != LDG_OK) {
        all_ok = false;
        break;
      }
      ++k;
      ++since;
      r.gmres_iters += nr.gmres_iters;
      r.fallback_used |= nr.fallback_used;
      r.lin_relres_max = std::max(r.lin_relres_max, nr.lin_relres);
      r.t_assemble_ms += nr.t_assemble_ms;
      r.t_solve_ms += nr.t_solve_ms;
      g = nr.newton_res_after;
      if (!std::isfinite(g)) {
        c->err = "non-finite Newton residual in stage " + std::to_string(st + 1);
        all_ok = false;
        break;
      }
      conv = fixed ? k >= so->max_newton : g <= tol;
    }
    r.newton_iters += k;
    if (k > r.max_stage_newton) r.max_stage_newton = k;
    if (st == 0) r.newton_res_first = g_first;
    r.newton_res_final = g;
    ++r.stages;
    if (all_ok && !conv) {
      char buf[160];
      std::snprintf(buf, sizeof(buf), "stage %d: ||G|| = %.3e after %d Newton iterations, tolerance %.3e", st + 1, g,
                    k, tol);
      c->err = buf;
      all_ok = false;
      break;
    }
    if (so->scheme == LDG_DIRK3 && st < 2) {
      // dt K_i = (Y_i - Ucomb_i) / alpha
      double* dK = st == 0 ? dK1 : dK2;
      HIPCK(c, launch_copy(dK, U, n, dc.stream));
      HIPCK(c, launch_axpby(dK, -1.0 / a, comb, 1.0 / a, n, dc.stream));
    }
  }
  r.assemblies = c->n_assemblies - n_asm0;
  r.converged = all_ok ? 1 : 0;
  if (all_ok) {
    if (so->scheme == LDG_BDF2 && Uprev) HIPCK(c, launch_copy(Uprev, Un, n, dc.stream));
  } else {
    HIPCK(c, launch_copy(U, Un, n, dc.stream));  // U unchanged on failure
  }
  HIPCK(c, hipStreamSynchronize(dc.stream));
  r.t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (rep) *rep = r;
  if (!all_ok) return LDG_E_NOT_CONVERGED;
  return LDG_OK;
}

// One classical RK4 step as kernel launches on dc.stream (kernels only, so the
// sequence can be captured: the two copies are kernels, not copy nodes).
static ldg_status rk4_step_launches(ldg_ctx c, double* U, double dt) {
  const DevCtx& dc = c->dc;
  const int64_t n = c->ndof;
  double* Us = c->d_tmp;
  double* acc = c->d_Un;
  const double a[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};
  const double b[4] = {dt / 6, dt / 3, dt / 3, dt / 6};
  HIPCK(c, launch_copy(acc, U, n, dc.stream));
  const double* cur = U;
  for (int k = 0; k < 4; ++k) {
    TRY(ldg_residual(c, cur, c->d_R, nullptr));
    HIPCK(c, launch_rk4_stage(k < 3 ? Us : nullptr, U, c->d_R, a[k], acc, b[k], n, dc.stream));
    cur = Us;
  }
  HIPCK(c, launch_copy(U, acc, n, dc.stream));
  return LDG_OK;
}

static void rk4_drop_graph(ldg_ctx c) {
  if (c->rk_exec) hipGraphExecDestroy(c->rk_exec);
  if (c->rk_graph) hipGraphDestroy(c->rk_graph);
  c->rk_exec = nullptr;
  c->rk_graph = nullptr;
}

ldg_status ldg_rk4(ldg_ctx c, double* U, double dt, int32_t nsteps) {
  if (!c) return LDG_E_INVALID;
  if (!U || nsteps < 0 || !std::isfinite(dt)) return fail(c, LDG_E_INVALID, "arguments");
  const int64_t n = c->ndof;
  TRY(dev_alloc(c, &c->d_R, (size_t)n));
  TRY(dev_alloc(c, &c->d_tmp, (size_t)n));
  TRY(dev_alloc(c, &c->d_Un, (size_t)n));
  if (nsteps == 0) return LDG_OK;
  if (!c->rk_stream) {
    HIPCK(c, hipStreamCreateWithFlags(&c->rk_stream, hipStreamNonBlocking));
    HIPCK(c, hipEventCreateWithFlags(&c->rk_ev[0], hipEventDisableTiming));
    HIPCK(c, hipEventCreateWithFlags(&c->rk_ev[1], hipEventDisableTiming));
  }
  // (re)capture one step when its kernel arguments change
  if (!c->rk_exec || c->rk_U != U || c->rk_dt != dt || c->rk_S != c->dc.mp.S || c->rk_gD != c->dc.mp.gD ||
      c->rk_gN != c->dc.mp.gN) {
    rk4_drop_graph(c);
    const hipStream_t caller = c->dc.stream;
    c->dc.stream = c->rk_stream;
    hipError_t e = hipStreamBeginCapture(c->rk_stream, hipStreamCaptureModeThreadLocal);
    ldg_status st = e == hipSuccess ? rk4_step_launches(c, U, dt) : LDG_E_HIP;
    hipGraph_t g = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(c->rk_stream, &g) : e;
    c->dc.stream = caller;
    if (st != LDG_OK || e2 != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return st != LDG_OK ? st : fail(c, LDG_E_HIP, std::string("RK4 graph capture: ") + hipGetErrorString(e2));
    }
    c->rk_graph = g;
    HIPCK(c, hipGraphInstantiate(&c->rk_exec, g, nullptr, nullptr, 0));
    c->rk_U = U;
    c->rk_dt = dt;
    c->rk_S = c->dc.mp.S;
    c->rk_gD = c->dc.mp.gD;
    c->rk_gN = c->dc.mp.gN;
  }
  // caller's stream -> graph stream -> caller's stream
  HIPCK(c, hipEventRecord(c->rk_ev[0], c->dc.stream));
  HIPCK(c, hipStreamWaitEvent(c->rk_stream, c->rk_ev[0], 0));
  for (int s = 0; s < nsteps; ++s) HIPCK(c, hipGraphLaunch(c->rk_exec, c->rk_stream));
  HIPCK(c, hipEventRecord(c->rk_ev[1], c->rk_stream));
  HIPCK(c, hipStreamWaitEvent(c->dc.stream, c->rk_ev[1], 0));
  return LDG_OK;
}

}  // extern "C"
