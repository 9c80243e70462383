// Host side of the learned preconditioner correction: the network object
// (parameters, Adam state, forward / backward on matrix cores), its
// evaluation at assembly, the corrected preconditioner apply and the
// extraction of training samples.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ldg_ctx.hpp"

namespace {

ldg_status nfail(ldg_net n, ldg_status s, const std::string& m) {
  if (n) n->err = m;
  return s;
}

#define NHIP(net, call)                                                                                       \
  do {                                                                                                        \
    hipError_t e_ = (call);                                                                                   \
    if (e_ != hipSuccess) return nfail(net, LDG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
ldg_status nalloc(ldg_net n, T** p, size_t count) {
  if (*p) hipFree(*p);
  *p = nullptr;
  if (hipMalloc((void**)p, (count ? count : 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return nfail(n, LDG_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  return LDG_OK;
}

// splitmix64 (Steele, Lea and Flood): the seeded stream of the initial weights
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void net_free_work(ldg_net n) {
  void* ps[] = {n->Xb, n->H1b, n->H2b, n->dYb, n->dA2b, n->dA1b, n->H1, n->H2, n->Y, n->dY, n->dH, n->dA2, n->dA1,
                n->loss_part};
  for (void* p : ps)
    if (p) hipFree(p);
  n->Xb = n->H1b = n->H2b = n->dYb = n->dA2b = n->dA1b = nullptr;
  n->H1 = n->H2 = n->Y = n->dY = n->dH = n->dA2 = n->dA1 = nullptr;
  n->loss_part = nullptr;
  n->cap = 0;
}

ldg_status ensure_work(ldg_net n, int64_t rows) {
  if (rows <= n->cap) return LDG_OK;
  net_free_work(n);
  const size_t r = (size_t)rows, H = (size_t)n->nh;
  TRY(nalloc(n, &n->Xb, r * n->nin));
  TRY(nalloc(n, &n->H1b, r * H));
  TRY(nalloc(n, &n->H2b, r * H));
  TRY(nalloc(n, &n->dYb, r * n->nout));
  TRY(nalloc(n, &n->dA2b, r * H));
  TRY(nalloc(n, &n->dA1b, r * H));
  TRY(nalloc(n, &n->H1, r * H));
  TRY(nalloc(n, &n->H2, r * H));
  TRY(nalloc(n, &n->Y, r * n->nout));
  TRY(nalloc(n, &n->dY, r * n->nout));
  TRY(nalloc(n, &n->dH, r * H));
  TRY(nalloc(n, &n->dA2, r * H));
  TRY(nalloc(n, &n->dA1, r * H));
  TRY(nalloc(n, &n->loss_part, r));
  n->cap = rows;
  return LDG_OK;
}

const float* P(ldg_net n, int k) { return n->w + n->off[k]; }
const uint16_t* PB(ldg_net n, int k) { return n->wb + n->off[k]; }

// Backward pass from n->dY (FP32, [rows][n_out]) into n->g.
ldg_status net_backward(ldg_net net, const float* X, int64_t rows, int prec) {
  const int M = (int)rows, H = net->nh, NI = net->nin, NO = net->nout;
  hipStream_t s = net->stream;
  float* g = net->g;
  if (prec == LDG_BF16) {
    NHIP(net, launch_to_bf16(net->dY, net->dYb, rows * NO, s));
    NHIP(net, launch_gemm_bf16(H, NO, M, net->H2b, 1, H, net->dYb, NO, 1, g + net->off[4], NO, nullptr, nullptr, 0,
                               0.f, s));
    NHIP(net, launch_colsum(net->dY, M, NO, g + net->off[5], s));
    NHIP(net, launch_gemm_bf16(M, H, NO, net->dYb, NO, 1, PB(net, 4), 1, NO, net->dH, H, nullptr, nullptr, 0, 0.f, s));
    NHIP(net, launch_tanh_backward(net->dH, net->H2, net->dA2, net->dA2b, rows * H, s));
    NHIP(net, launch_gemm_bf16(H, H, M, net->H1b, 1, H, net->dA2b, H, 1, g + net->off[2], H, nullptr, nullptr, 0, 0.f,
                               s));
    NHIP(net, launch_colsum(net->dA2, M, H, g + net->off[3], s));
    NHIP(net, launch_gemm_bf16(M, H, H, net->dA2b, H, 1, PB(net, 2), 1, H, net->dH, H, nullptr, nullptr, 0, 0.f, s));
    NHIP(net, launch_tanh_backward(net->dH, net->H1, net->dA1, net->dA1b, rows * H, s));
    NHIP(net, launch_gemm_bf16(NI, H, M, net->Xb, 1, NI, net->dA1b, H, 1, g + net->off[0], H, nullptr, nullptr, 0,
                               0.f, s));
    NHIP(net, launch_colsum(net->dA1, M, H, g + net->off[1], s));
  } else {
    NHIP(net, launch_gemm_f32(H, NO, M, net->H2, 1, H, net->dY, NO, 1, g + net->off[4], NO, nullptr, nullptr, 0, 0.f,
                              s));
    NHIP(net, launch_colsum(net->dY, M, NO, g + net->off[5], s));
    NHIP(net, launch_gemm_f32(M, H, NO, net->dY, NO, 1, P(net, 4), 1, NO, net->dH, H, nullptr, nullptr, 0, 0.f, s));
    NHIP(net, launch_tanh_backward(net->dH, net->H2, net->dA2, nullptr, rows * H, s));
    NHIP(net, launch_gemm_f32(H, H, M, net->H1, 1, H, net->dA2, H, 1, g + net->off[2], H, nullptr, nullptr, 0, 0.f, s));
    NHIP(net, launch_colsum(net->dA2, M, H, g + net->off[3], s));
    NHIP(net, launch_gemm_f32(M, H, H, net->dA2, H, 1, P(net, 2), 1, H, net->dH, H, nullptr, nullptr, 0, 0.f, s));
    NHIP(net, launch_tanh_backward(net->dH, net->H1, net->dA1, nullptr, rows * H, s));
    NHIP(net, launch_gemm_f32(NI, H, M, X, 1, NI, net->dA1, H, 1, g + net->off[0], H, nullptr, nullptr, 0, 0.f, s));
    NHIP(net, launch_colsum(net->dA1, M, H, g + net->off[1], s));
  }
  return LDG_OK;
}

}  // namespace

namespace ldg_host {

// Y = network(X); Xb (BF16 features) may be given to skip the conversion.
ldg_status net_forward(ldg_net net, const float* X, const uint16_t* Xb, int64_t rows, int prec, float* Y) {
  if (rows <= 0) return LDG_OK;
  TRY(ensure_work(net, rows));
  const int M = (int)rows, H = net->nh, NI = net->nin, NO = net->nout;
  hipStream_t s = net->stream;
  if (prec == LDG_BF16) {
    if (!Xb) {  // the backward pass reads the converted features from net->Xb
      NHIP(net, launch_to_bf16(X, net->Xb, rows * NI, s));
      Xb = net->Xb;
    }
    NHIP(net, launch_gemm_bf16(M, H, NI, Xb, NI, 1, PB(net, 0), H, 1, net->H1, H, net->H1b, P(net, 1), 2, 0.f, s));
    NHIP(net, launch_gemm_bf16(M, H, H, net->H1b, H, 1, PB(net, 2), H, 1, net->H2, H, net->H2b, P(net, 3), 2, 0.f, s));
    NHIP(net, launch_gemm_bf16(M, NO, H, net->H2b, H, 1, PB(net, 4), NO, 1, Y, NO, nullptr, P(net, 5), 1, 0.f, s));
  } else {
    NHIP(net, launch_gemm_f32(M, H, NI, X, NI, 1, P(net, 0), H, 1, net->H1, H, nullptr, P(net, 1), 2, 0.f, s));
    NHIP(net, launch_gemm_f32(M, H, H, net->H1, H, 1, P(net, 2), H, 1, net->H2, H, nullptr, P(net, 3), 2, 0.f, s));
    NHIP(net, launch_gemm_f32(M, NO, H, net->H2, H, 1, P(net, 4), NO, 1, Y, NO, nullptr, P(net, 5), 1, 0.f, s));
  }
  return LDG_OK;
}

void learned_free(ldg_ctx c) {
  void* ps[] = {c->d_At, c->d_Xf, c->d_Xb, c->d_Dinv, c->d_Y, c->d_C, c->d_z0, c->d_Rl, c->d_bad};
  for (void* p : ps)
    if (p) hipFree(p);
}

// Called by the assembly after the preconditioner is formed and factorised
// (A~ copied to d_At when kept).  Computes features, evaluates the network
// and the blocks C when the correction is enabled.
ldg_status learned_after_form(ldg_ctx c, const double* R_at_U, double gamma) {
  const DevCtx& dc = c->dc;
  const int64_t NN = c->nnode;
  const bool want = c->net && c->learned_enabled;
  c->learned_active = false;
  c->learned_fallback = 0;
  if (!c->learned_kept) return LDG_OK;
  const int nin = dc.NP * dc.M * dc.M + dc.NP * dc.M, nout = dc.NP * dc.M * dc.M;
  TRY(dev_alloc(c, &c->d_Xf, (size_t)dc.E * nin));
  TRY(dev_alloc(c, &c->d_Xb, (size_t)dc.E * nin));
  TRY(dev_alloc(c, &c->d_Dinv, (size_t)NN * dc.M * dc.M));
  const double* R = R_at_U;
  if (!R) {
    TRY(dev_alloc(c, &c->d_Rl, (size_t)c->ndof));
    TRY(ldg_residual(c, c->d_Ua, c->d_Rl, nullptr));
    R = c->d_Rl;
  }
  HIPCK(c, launch_learned_features(dc, c->d_At, R, -gamma, c->d_Xf, c->d_Xb, c->d_Dinv));
  if (!want) return LDG_OK;
  TRY(dev_alloc(c, &c->d_Y, (size_t)dc.E * nout));
  TRY(dev_alloc(c, &c->d_C, (size_t)NN * dc.M * dc.M));
  TRY(dev_alloc(c, &c->d_z0, (size_t)c->ndof));
  TRY(dev_alloc(c, &c->d_bad, 1));
  if (net_forward(c->net, c->d_Xf, c->infer_prec == LDG_BF16 ? c->d_Xb : nullptr, dc.E, c->infer_prec, c->d_Y) !=
      LDG_OK)
    return fail(c, LDG_E_HIP, "network evaluation: " + c->net->err);
  HIPCK(c, hipMemsetAsync(c->d_bad, 0, sizeof(int), dc.stream));
  HIPCK(c, launch_learned_cblocks(dc, c->d_Y, c->d_Dinv, c->d_C, c->d_bad));
  int bad = 0;
  HIPCK(c, hipMemcpyAsync(&bad, c->d_bad, sizeof(int), hipMemcpyDeviceToHost, dc.stream));
  HIPCK(c, hipStreamSynchronize(dc.stream));
  c->learned_fallback = bad ? 1 : 0;
  c->learned_active = !bad;
  return LDG_OK;
}

ldg_status precond_apply_any(ldg_ctx c, const double* r, double* z) {
  const DevCtx& dc = c->dc;
  if (c->assembled_kind == LDG_PRECOND_BLOCK_LU) {
    HIPCK(c, launch_blocklu_apply(dc, c->d_Dense, r, z));
    return LDG_OK;
  }
  if (!c->learned_active) {
    HIPCK(c, launch_precond_apply(dc, c->d_Fem, c->prec, r, z));
    return LDG_OK;
  }
  HIPCK(c, launch_precond_apply(dc, c->d_Fem, c->prec, r, c->d_z0));
  HIPCK(c, launch_learned_apply(dc, c->d_At, c->d_C, r, c->d_z0, z));
  return LDG_OK;
}

}  // namespace ldg_host

extern "C" {

ldg_status ldg_net_create(int32_t dim, int32_t p, int32_t m, int32_t hidden, uint64_t seed, void* stream,
                          ldg_net* out) {
  if (!out) return LDG_E_INVALID;
  *out = nullptr;
  if ((dim != 2 && dim != 3) || p < 1 || p > 4 || !(m == 1 || m == dim + 2) || hidden < 1 || hidden > 4096)
    return LDG_E_INVALID;
  ldg_net n = new ldg_net_s();
  n->dim = dim;
  n->p = p;
  n->m = m;
  int np = 1;
  for (int k = 0; k < dim; ++k) np *= p + 1;
  n->np = np;
  n->nin = np * m * m + np * m;
  n->nh = hidden;
  n->nout = np * m * m;
  n->stream = (hipStream_t)stream;
  DevCtx& dc = n->dc;
  dc.D = dim;
  dc.P = p;
  dc.EQ = m == 1 ? LDG_POISSON : LDG_NS;
  dc.M = m;
  dc.N1 = p + 1;
  dc.NP = np;
  dc.stream = n->stream;
  const int64_t sz[6] = {(int64_t)n->nin * hidden, hidden, (int64_t)hidden * hidden, hidden,
                         (int64_t)hidden * n->nout, n->nout};
  int64_t o = 0;
  for (int k = 0; k < 6; ++k) {
    n->off[k] = o;
    o += sz[k];
  }
  n->nparam = o;
  std::vector<float> host((size_t)o, 0.f);
  uint64_t st = seed;
  auto glorot = [&](int64_t off, int64_t fan_in, int64_t fan_out) {
    const double a = std::sqrt(6.0 / (double)(fan_in + fan_out));
    for (int64_t i = 0; i < fan_in * fan_out; ++i) {
      const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
      host[(size_t)(off + i)] = (float)((2.0 * u - 1.0) * a);
    }
  };
  glorot(n->off[0], n->nin, hidden);
  glorot(n->off[2], hidden, hidden);
  ldg_status s;
  if ((s = nalloc(n, &n->w, o)) != LDG_OK || (s = nalloc(n, &n->wb, o)) != LDG_OK ||
      (s = nalloc(n, &n->g, o)) != LDG_OK || (s = nalloc(n, &n->m1, o)) != LDG_OK ||
      (s = nalloc(n, &n->m2, o)) != LDG_OK) {
    ldg_net_destroy(n);
    return s;
  }
  if (hipMemcpy(n->w, host.data(), sizeof(float) * o, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(n->m1, 0, sizeof(float) * o) != hipSuccess || hipMemset(n->m2, 0, sizeof(float) * o) != hipSuccess ||
      hipMemset(n->g, 0, sizeof(float) * o) != hipSuccess || launch_to_bf16(n->w, n->wb, o, n->stream) != hipSuccess ||
      hipStreamSynchronize(n->stream) != hipSuccess) {
    ldg_net_destroy(n);
    return LDG_E_HIP;
  }
  *out = n;
  return LDG_OK;
}

void ldg_net_destroy(ldg_net n) {
  if (!n) return;
  net_free_work(n);
  void* ps[] = {n->w, n->wb, n->g, n->m1, n->m2};
  for (void* p : ps)
    if (p) hipFree(p);
  delete n;
}

int64_t ldg_net_num_params(ldg_net n) { return n ? n->nparam : -1; }

const char* ldg_net_last_error(ldg_net n) { return n ? n->err.c_str() : "null network"; }

ldg_status ldg_net_set_params(ldg_net n, const float* params) {
  if (!n) return LDG_E_INVALID;
  if (!params) return nfail(n, LDG_E_INVALID, "null pointer");
  const size_t b = sizeof(float) * n->nparam;
  NHIP(n, hipMemcpyAsync(n->w, params, b, hipMemcpyDeviceToDevice, n->stream));
  NHIP(n, launch_to_bf16(n->w, n->wb, n->nparam, n->stream));
  NHIP(n, hipMemsetAsync(n->m1, 0, b, n->stream));
  NHIP(n, hipMemsetAsync(n->m2, 0, b, n->stream));
  n->step = 0;
  return LDG_OK;
}

ldg_status ldg_net_get_params(ldg_net n, float* params) {
  if (!n) return LDG_E_INVALID;
  if (!params) return nfail(n, LDG_E_INVALID, "null pointer");
  NHIP(n, hipMemcpyAsync(params, n->w, sizeof(float) * n->nparam, hipMemcpyDeviceToDevice, n->stream));
  return LDG_OK;
}

ldg_status ldg_net_forward(ldg_net n, const float* X, int64_t rows, int32_t prec, float* Y) {
  if (!n) return LDG_E_INVALID;
  if (!X || !Y || rows < 0) return nfail(n, LDG_E_INVALID, "arguments");
  if (prec != LDG_F32 && prec != LDG_BF16) return nfail(n, LDG_E_INVALID, "prec must be LDG_F32 or LDG_BF16");
  if (rows > 0x7fffffff / 64) return nfail(n, LDG_E_INVALID, "too many rows");
  return net_forward(n, X, nullptr, rows, prec, Y);
}

ldg_status ldg_net_loss_grad(ldg_net n, const ldg_sample_batch* b, int32_t prec, float* grad, double* loss) {
  if (!n) return LDG_E_INVALID;
  if (!b || !b->X_dev || !b->A_dev || !b->S_dev || !b->T_dev || b->n < 1 || b->n_probe < 1)
    return nfail(n, LDG_E_INVALID, "batch");
  if (prec != LDG_F32 && prec != LDG_BF16) return nfail(n, LDG_E_INVALID, "prec must be LDG_F32 or LDG_BF16");
  if (b->n > 0x7fffffff / 64) return nfail(n, LDG_E_INVALID, "batch too large");
  if (!learned_supported(n->dc)) return nfail(n, LDG_E_UNSUPPORTED, "element too large for the loss kernel");
  // the workspace (n->Y among it) must exist before its pointers are taken
  TRY(ensure_work(n, b->n));
  TRY(net_forward(n, b->X_dev, nullptr, b->n, prec, n->Y));
  const float scale = (float)(1.0 / ((double)b->n * b->n_probe));
  NHIP(n, launch_learned_loss(n->dc, b->n, b->n_probe, b->A_dev, b->S_dev, b->T_dev, n->Y, scale, n->dY,
                              n->loss_part));
  TRY(net_backward(n, b->X_dev, b->n, prec));
  if (grad) NHIP(n, hipMemcpyAsync(grad, n->g, sizeof(float) * n->nparam, hipMemcpyDeviceToDevice, n->stream));
  if (loss) {
    std::vector<double> part((size_t)b->n);
    NHIP(n, hipMemcpyAsync(part.data(), n->loss_part, sizeof(double) * b->n, hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    double acc = 0.0;
    for (double v : part) acc += v;
    *loss = acc;
  }
  return LDG_OK;
}

ldg_status ldg_net_adam_step(ldg_net n, double lr) {
  if (!n) return LDG_E_INVALID;
  if (!(lr > 0.0) || !std::isfinite(lr)) return nfail(n, LDG_E_INVALID, "lr");
  n->step += 1;
  NHIP(n, launch_adam(n->w, n->wb, n->g, n->m1, n->m2, n->nparam, (float)lr, 0.9f, 0.999f, 1e-8f, n->step, n->stream));
  return LDG_OK;
}

ldg_status ldg_learned_attach(ldg_ctx c, ldg_net n, int32_t infer_prec) {
  if (!c) return LDG_E_INVALID;
  if (!n) {
    c->net = nullptr;
    c->learned_enabled = false;
    c->learned_active = false;
    return LDG_OK;
  }
  if (infer_prec != LDG_F32 && infer_prec != LDG_BF16) return fail(c, LDG_E_INVALID, "infer_prec");
  if (n->dim != c->dc.D || n->p != c->dc.P || n->m != c->dc.M) return fail(c, LDG_E_SHAPE, "network shape");
  if (!learned_supported(c->dc)) return fail(c, LDG_E_UNSUPPORTED, "element too large for the learned correction");
  if (n->stream != c->dc.stream) return fail(c, LDG_E_INVALID, "network and context must share the stream");
  c->net = n;
  c->infer_prec = infer_prec;
  c->learned_enabled = true;
  return LDG_OK;
}

ldg_status ldg_learned_collect(ldg_ctx c, int32_t on) {
  if (!c) return LDG_E_INVALID;
  if (on && !learned_supported(c->dc)) return fail(c, LDG_E_UNSUPPORTED, "element too large for the learned correction");
  c->learned_collect = on != 0;
  return LDG_OK;
}

int32_t ldg_learned_active(ldg_ctx c) { return c && c->learned_active ? 1 : 0; }

ldg_status ldg_learned_samples(ldg_ctx c, const int64_t* elems, int64_t n, const double* V, int32_t K, float* X,
                               float* A, float* S, float* T) {
  if (!c) return LDG_E_INVALID;
  if (!elems || n < 1 || K < 1 || !X || !A || !S || !T) return fail(c, LDG_E_INVALID, "arguments");
  if (!c->assembled || !c->learned_kept) return fail(c, LDG_E_NOT_ASSEMBLED, "no assembly kept A~ (collect or attach)");
  for (int64_t i = 0; i < n; ++i)
    if (elems[i] < 0 || elems[i] >= c->dc.E) return fail(c, LDG_E_INVALID, "element index out of range");
  const DevCtx& dc = c->dc;
  const int64_t nd = c->ndof;
  if (!V) {
    if (K > c->krylov_avail) return fail(c, LDG_E_INVALID, "fewer Arnoldi vectors than probes");
    V = c->d_V;
  }
  double* Z0 = nullptr;
  int64_t* d_el = nullptr;
  if (hipMalloc((void**)&Z0, sizeof(double) * nd * K) != hipSuccess) return fail(c, LDG_E_NOMEM, "probe workspace");
  if (hipMalloc((void**)&d_el, sizeof(int64_t) * n) != hipSuccess) {
    hipFree(Z0);
    return fail(c, LDG_E_NOMEM, "element list");
  }
  ldg_status st = LDG_OK;
  hipError_t e = hipMemcpyAsync(d_el, elems, sizeof(int64_t) * n, hipMemcpyHostToDevice, dc.stream);
  for (int k = 0; k < K && e == hipSuccess; ++k)
    e = launch_precond_apply(dc, c->d_Fem, c->prec, V + (int64_t)k * nd, Z0 + (int64_t)k * nd);
  if (e == hipSuccess)
    e = launch_learned_samples(dc, d_el, n, K, c->d_At, c->d_Xf, c->d_Dinv, V, Z0, nd, X, A, S, T);
  if (e == hipSuccess) e = hipStreamSynchronize(dc.stream);
  if (e != hipSuccess) st = fail(c, LDG_E_HIP, std::string("sample extraction: ") + hipGetErrorString(e));
  hipFree(Z0);
  hipFree(d_el);
  return st;
}

}  // extern "C"
