// Internal: the context object behind ldg_ctx and host helpers shared by the
// host translation units of libldg.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/ldg.h"
#include "ldg_kernels.hpp"

using namespace ldg;

struct ldg_ctx_s {
  DevCtx dc{};
  std::string err;
  int64_t ndof = 0, nq = 0, nnode = 0;
  double* d_xyz = nullptr;
  int64_t* d_face_nbr = nullptr;
  int32_t* d_nbr_node = nullptr;
  int8_t* d_sw = nullptr;
  double* d_gD = nullptr;
  double* d_gN = nullptr;
  double* d_S = nullptr;
  double* d_Q = nullptr;   // Q scratch (residual)
  double* d_W = nullptr;   // K21 x scratch
  double* d_W2 = nullptr;  // tangent Q scratch
  int precond_kind = 0;       // ldg_precond_kind: 0 BILU(0), 1 exact element-block LU
  double* d_Dense = nullptr;  // [E][NR][NR] dense L\U of A~ (block LU)
  size_t capDense = 0;
  double* d_cwork = nullptr;  // coupled (U, Q) solve: Krylov space and vectors
  size_t cap_cwork = 0;
  double* d_geo = nullptr;    // per-element geometry record of the Jacobian assembly
  double* d_Jwork = nullptr;  // point flux Jacobians of the assembly
  size_t capJwork = 0;
  double* d_K21w = nullptr;  // stored K21 weights [slot][d][E Np], computed on first use
  float* d_K21f = nullptr;  // FP32 copy of the K21 weights
  // assembled state
  bool assembled = false;
  int assembled_kind = 0;  // preconditioner built by the last assembly
  int prec = 0;
  double alpha = 1.0, gamma = 0.0;
  void* d_K11 = nullptr;
  void* d_K12 = nullptr;
  void* d_F = nullptr;
  void* d_Fem = nullptr;  // element-major copy of the factors (read by the apply)
  size_t capFem = 0;
  size_t capK11 = 0, capK12 = 0, capF = 0;
  double* d_Ua = nullptr;  // state at assembly
  double* d_Qa = nullptr;  // D(U) at assembly
  // Newton / Krylov workspace
  double* d_V = nullptr;
  double* d_Z = nullptr;  // preconditioned Arnoldi vectors z_k = P^{-1} v_k
  int cap_restart = 0;
  double* d_R = nullptr;
  double* d_G = nullptr;
  double* d_x = nullptr;
  double* d_r = nullptr;
  double* d_z = nullptr;
  double* d_tmp = nullptr;
  double* d_Un = nullptr;
  double* d_Uold = nullptr;  // state before a Newton update (undone when the learned correction is rejected)
  int n_assemblies = 0;      // Jacobian assemblies since creation
  // implicit time-step driver: U^n, the stage's explicit part, dt K_1 and dt K_2 (DIRK)
  double* d_st_Un = nullptr;
  double* d_st_comb = nullptr;
  double* d_st_K = nullptr;
  double* d_partial = nullptr;
  double* d_h = nullptr;
  int nblk_dot = 0;
  // optional per-kernel event timing inside ldg_newton_step
  struct Timed {
    std::vector<hipEvent_t> ev;  // start/stop pairs
    size_t used = 0;
  };
  bool timing = false;
  Timed tm[3];  // 0 jacvec, 1 K21 gradient, 2 precond apply
  int krylov_avail = 0;  // Arnoldi vectors of the last GMRES cycle left in d_V
  // RK4: one step captured as a HIP graph and replayed (launch-bound on small meshes)
  hipStream_t rk_stream = nullptr;
  hipEvent_t rk_ev[2] = {nullptr, nullptr};
  hipGraph_t rk_graph = nullptr;
  hipGraphExec_t rk_exec = nullptr;
  const double* rk_U = nullptr;
  const double* rk_S = nullptr;
  const double* rk_gD = nullptr;
  const double* rk_gN = nullptr;
  double rk_dt = 0.0;
  // learned correction of the preconditioner
  ldg_net net = nullptr;         // attached network (owned by the caller)
  int infer_prec = 2;            // precision of the network evaluation (F32 or BF16)
  bool learned_enabled = false;  // apply the correction at the next assembly
  bool learned_collect = false;  // keep A~, features and D^{-1} for sampling
  bool learned_kept = false;     // the current assembly kept them
  bool learned_active = false;   // the current assembly applies the correction
  int learned_fallback = 0;      // the last assembly found non-finite network output
  float* d_At = nullptr;         // FP32 copy of A~, factor layout
  float* d_Xf = nullptr;         // features [E][n_in]
  uint16_t* d_Xb = nullptr;      // BF16 features
  float* d_Dinv = nullptr;       // [E Np][m][m]
  float* d_Y = nullptr;          // network output [E][Np m m]
  float* d_C = nullptr;          // correction blocks [m][m][E Np]
  double* d_z0 = nullptr;        // ILU(0) result before the correction
  double* d_Rl = nullptr;        // residual at the assembly state (direct assembly calls)
  int* d_bad = nullptr;
};

// Network of the learned correction: two tanh hidden layers, FP32 master
// weights with a BF16 copy, Adam state and activation workspace.
struct ldg_net_s {
  int dim = 0, p = 0, m = 0, np = 0, nin = 0, nh = 0, nout = 0;
  DevCtx dc{};  // shape information for the loss kernel (D, P, EQ, M, NP)
  hipStream_t stream = nullptr;
  std::string err;
  int64_t nparam = 0, off[6] = {0, 0, 0, 0, 0, 0};
  float* w = nullptr;
  uint16_t* wb = nullptr;
  float* g = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  int step = 0;
  int64_t cap = 0;  // rows of the activation workspace
  uint16_t *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dYb = nullptr, *dA2b = nullptr, *dA1b = nullptr;
  float *H1 = nullptr, *H2 = nullptr, *Y = nullptr, *dY = nullptr, *dH = nullptr, *dA2 = nullptr, *dA1 = nullptr;
  double* loss_part = nullptr;
};

namespace ldg_host {

// Records a start/stop event pair around a launch when timing is on.
struct Span {
  ldg_ctx c;
  int which;
  hipEvent_t stop = nullptr;
  Span(ldg_ctx c_, int w) : c(c_), which(w) {
    if (!c->timing) return;
    auto& t = c->tm[which];
    if (t.used + 2 > t.ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
      t.ev.push_back(a);
      t.ev.push_back(b);
    }
    hipEventRecord(t.ev[t.used], c->dc.stream);
    stop = t.ev[t.used + 1];
    t.used += 2;
  }
  ~Span() {
    if (stop) hipEventRecord(stop, c->dc.stream);
  }
};

inline ldg_status fail(ldg_ctx c, ldg_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCK(ctx, call)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(ctx, LDG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
ldg_status dev_alloc(ldg_ctx c, T** p, size_t count) {
  if (*p) return LDG_OK;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, LDG_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  return LDG_OK;
}

inline ldg_status grow(ldg_ctx c, void** p, size_t* cap, size_t bytes) {
  if (*cap >= bytes && *p) return LDG_OK;
  if (*p) hipFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return fail(c, LDG_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  *cap = bytes;
  return LDG_OK;
}

inline size_t elem_size(int prec) { return prec == LDG_F64 ? 8 : (prec == LDG_F32 ? 4 : 2); }

#define TRY(x)                     \
  do {                             \
    ldg_status s_ = (x);           \
    if (s_ != LDG_OK) return s_;   \
  } while (0)

// y = (alpha I - gamma A) x with the caller's buffer W for w = K21 x (ldg_host.cpp)
ldg_status apply_op_with(ldg_ctx c, const double* x, double* y, bool exact, double* W);

// learned-correction hooks (ldg_learned.cpp)
ldg_status learned_after_form(ldg_ctx c, const double* R_at_U, double gamma);
ldg_status precond_apply_any(ldg_ctx c, const double* r, double* z);
void learned_free(ldg_ctx c);
void set_host_error(const std::string& m);  // message for ldg_last_error(NULL)
ldg_status net_forward(ldg_net net, const float* X, const uint16_t* Xb, int64_t n, int prec, float* Y);

}  // namespace ldg_host
using namespace ldg_host;
