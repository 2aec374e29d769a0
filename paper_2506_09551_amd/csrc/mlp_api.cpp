// C ABI of the surrogate network (learned form): create, parameters,
// gradient, training (captured in a hipGraph per step), ensemble prediction
// and the solver-fallback rule.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "msb_internal.h"
#include "mlp_internal.h"

using namespace msb;


struct msb_mlp {
  int members = 0;
  int64_t pstride = 0;            // floats per member in params/grads/m/v
  float out_scale = 1.0f;
  float* d_in = nullptr;          // [12]: shift[6], scale[6]
  float* params = nullptr;
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  __bf16* w2b = nullptr;          // [members][512][512] bfloat16 operand copies [in][out]
  __bf16* w3b = nullptr;
  __bf16* w2t = nullptr;          // and [out][in]
  __bf16* w3t = nullptr;
  int* step = nullptr;            // device Adam step counter (since the last set_params)
  int* call_step = nullptr;       // device step within the current training call
  int* zero_step = nullptr;       // device 0 (offset for calls without a permutation)
  // activations for `cap` rows per member
  int cap = 0;
  void* act = nullptr;
  size_t act_bytes = 0;
  hipStream_t stream = nullptr;   // private, default priority
};

namespace {

int max_parts(int cap) { return (cap + kRowsPerPart - 1) / kRowsPerPart; }

struct ActView {
  float *z1, *z2, *z3, *y, *g, *part, *splitk;
  __bf16 *h1, *h2, *h3, *dz1, *dz2, *dz3;
  __bf16 *h1T, *h2T, *dz2T, *dz3T;
  double* loss_part;
  int64_t act_stride, y_stride;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t act_need(int members, int cap) {
  const size_t a = (size_t)cap * kMlpH;
  size_t n = 0;
  n += 3 * align256(members * a * sizeof(float));        // gelu'(z1)..gelu'(z3)
  n += 10 * align256(members * a * sizeof(__bf16));      // h1..h3, dz1..dz3, four transposed copies
  n += 2 * align256((size_t)members * cap * sizeof(float));   // y, g
  n += align256((size_t)members * max_parts(cap) * kMlpIn * kMlpH * sizeof(float));   // partials
  n += align256((size_t)members * (cap / 4 + 1) * sizeof(double));
  n += align256((size_t)kMaxSplitK * members * kMlpH * kMlpH * sizeof(float));   // split-K partials
  return n;
}

ActView carve(msb_mlp* m) {
  ActView v;
  char* p = (char*)m->act;
  const size_t a = (size_t)m->cap * kMlpH;
  auto take = [&](size_t bytes) { char* r = p; p += align256(bytes); return r; };
  v.z1 = (float*)take(m->members * a * sizeof(float));
  v.z2 = (float*)take(m->members * a * sizeof(float));
  v.z3 = (float*)take(m->members * a * sizeof(float));
  v.h1 = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.h2 = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.h3 = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.dz1 = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.dz2 = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.dz3 = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.h1T = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.h2T = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.dz2T = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.dz3T = (__bf16*)take(m->members * a * sizeof(__bf16));
  v.y = (float*)take((size_t)m->members * m->cap * sizeof(float));
  v.g = (float*)take((size_t)m->members * m->cap * sizeof(float));
  v.part = (float*)take((size_t)m->members * max_parts(m->cap) * kMlpIn * kMlpH * sizeof(float));
  v.loss_part = (double*)take((size_t)m->members * (m->cap / 4 + 1) * sizeof(double));
  v.splitk = (float*)take((size_t)kMaxSplitK * m->members * kMlpH * kMlpH * sizeof(float));
  v.act_stride = (int64_t)a;
  v.y_stride = m->cap;
  return v;
}

msb_status ensure_cap(msb_mlp* m, int rows) {
  if (rows <= m->cap) return MSB_OK;
  const size_t need = act_need(m->members, rows);
  if (m->act) {
    MSB_HIP(hipFree(m->act));
    m->act = nullptr;
    m->cap = 0;
  }
  if (hipMalloc(&m->act, need) != hipSuccess) {
    (void)hipGetLastError();
    m->act = nullptr;
    return fail(MSB_ENOMEM, "surrogate: activation buffers do not fit");
  }
  m->act_bytes = need;
  m->cap = rows;
  return MSB_OK;
}

MlpFwdArgs fwd_args(msb_mlp* m, const ActView& v, const float* X, const float* T, int batch, int valid) {
  MlpFwdArgs a;
  std::memset(&a, 0, sizeof(a));
  a.X = X;
  a.T = T;
  a.perm = nullptr;
  a.step = m->zero_step;
  a.batch = batch;
  a.valid = valid;
  a.in_shift = m->d_in;
  a.in_scale = m->d_in + kMlpIn;
  a.out_scale = m->out_scale;
  a.params = m->params;
  a.pstride = m->pstride;
  a.z1 = v.z1; a.z2 = v.z2; a.z3 = v.z3;
  a.h1 = v.h1; a.h2 = v.h2; a.h3 = v.h3;
  a.dz1 = v.dz1; a.dz2 = v.dz2; a.dz3 = v.dz3;
  a.act_stride = v.act_stride;
  a.h1T = v.h1T; a.h2T = v.h2T; a.dz2T = v.dz2T; a.dz3T = v.dz3T;
  a.actT_stride = v.act_stride;
  a.ldT = m->cap;
  a.y = v.y; a.g = v.g; a.y_stride = v.y_stride;
  a.loss_part = v.loss_part;
  return a;
}

GemmArgs gemm_base() {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  return g;
}

// forward of `members` networks (member offset `mem0`) on a.batch rows
hipError_t forward(msb_mlp* m, int mem0, int members, const MlpFwdArgs& a0, hipStream_t st) {
  MlpFwdArgs a = a0;
  const int64_t ps = m->pstride;
  a.params = m->params + mem0 * ps;
  hipError_t e = launch_layer1_fwd(a, members, st);
  const __bf16* hin[2] = {a.h1, a.h2};
  float* zout[2] = {a.z2, a.z3};
  __bf16* hout[2] = {a.h2, a.h3};
  // B[n][k] = W[k][n]: the [out][in] copies
  const __bf16* wt[2] = {m->w2t + (int64_t)mem0 * kMlpH * kMlpH, m->w3t + (int64_t)mem0 * kMlpH * kMlpH};
  __bf16* hT[2] = {a.h2T, nullptr};             // h2 feeds the layer-3 weight gradient
  const int64_t boff[2] = {kOffB2, kOffB3};
  for (int l = 0; l < 2 && e == hipSuccess; ++l) {
    GemmArgs g = gemm_base();
    g.A = hin[l]; g.lda = kMlpH; g.sA = a.act_stride;
    g.B = wt[l]; g.ldb = kMlpH; g.sB = (int64_t)kMlpH * kMlpH;
    g.M = a.batch; g.N = kMlpH; g.K = kMlpH;
    g.C = zout[l]; g.ldc = kMlpH; g.sC = a.act_stride;
    g.bias = a.params + boff[l]; g.sBias = ps;
    g.H = hout[l]; g.ldh = kMlpH; g.sH = a.act_stride;
    g.HT = hT[l]; g.ldht = a.ldT; g.sHT = a.actT_stride;
    e = launch_gemm(kEpiFwd, g, members, st);
  }
  if (e == hipSuccess) e = launch_layer4_fwd(a, members, st);
  return e;
}

// backward into m->grads (members from mem0), after forward with targets
hipError_t backward(msb_mlp* m, int mem0, int members, const MlpFwdArgs& a0, const ActView& v, hipStream_t st) {
  MlpFwdArgs a = a0;
  const int64_t ps = m->pstride;
  a.params = m->params + mem0 * ps;
  float* grads = m->grads + mem0 * ps;
  hipError_t e = launch_layer4_bwd(a, members, st);
  // output layer: dW4 = h3^T g, db4 = sum g
  ColSumArgs c;
  std::memset(&c, 0, sizeof(c));
  c.src_bf16 = a.h3; c.src_stride = a.act_stride; c.ld = kMlpH;
  c.wgt = a.g; c.wgt_stride = a.y_stride;
  c.nrows = a.valid; c.ncols = kMlpH; c.rows_per_part = kRowsPerPart; c.max_parts = max_parts(m->cap);
  c.part = v.part; c.out = grads + kOffW4; c.out_stride = ps;
  if (e == hipSuccess) e = launch_colsum(c, members, st);
  ColSumArgs cb = c;
  cb.src_bf16 = nullptr; cb.src_f32 = a.g; cb.src_stride = a.y_stride; cb.ld = 1;
  cb.wgt = nullptr; cb.ncols = 1; cb.out = grads + kOffB4;
  if (e == hipSuccess) e = launch_colsum(cb, members, st);
  // hidden layers 3 and 2: dW = h^T dz, db = sum dz, dz_prev = (dz W^T) * gelu'(z_prev)
  const __bf16* hinT[2] = {a.h2T, a.h1T};
  const __bf16* dzs[2] = {a.dz3, a.dz2};
  const __bf16* dzsT[2] = {a.dz3T, a.dz2T};
  __bf16* dzp[2] = {a.dz2, a.dz1};
  __bf16* dzpT[2] = {a.dz2T, nullptr};
  const float* zp[2] = {a.z2, a.z1};
  const __bf16* wb[2] = {m->w3b + (int64_t)mem0 * kMlpH * kMlpH, m->w2b + (int64_t)mem0 * kMlpH * kMlpH};
  const int64_t woff[2] = {kOffW3, kOffW2}, boff[2] = {kOffB3, kOffB2};
  for (int l = 0; l < 2 && e == hipSuccess; ++l) {
    GemmArgs g = gemm_base();
    g.A = hinT[l]; g.lda = a.ldT; g.sA = a.actT_stride;    // A[in][b] = h^T
    g.B = dzsT[l]; g.ldb = a.ldT; g.sB = a.actT_stride;    // B[out][b] = dz^T
    g.M = kMlpH; g.N = kMlpH; g.K = a.batch;
    // the 512 x 512 output has only 16 tiles per member: split K so that
    // enough workgroups run, then add the slices
    int splits = 1;
    while (splits < kMaxSplitK && a.batch % (2 * splits * 64) == 0 && a.batch / (2 * splits) >= 512) splits *= 2;
    g.splitk = splits;
    if (splits > 1) {
      g.C = v.splitk; g.ldc = kMlpH; g.sC = (int64_t)kMlpH * kMlpH; g.sCk = (int64_t)members * kMlpH * kMlpH;
      e = launch_gemm(kEpiStore, g, members, st);
      if (e == hipSuccess)
        e = launch_splitk_sum(v.splitk, g.sCk, splits, grads + woff[l], ps, (int64_t)kMlpH * kMlpH, members, st);
    } else {
      g.C = grads + woff[l]; g.ldc = kMlpH; g.sC = ps;
      e = launch_gemm(kEpiStore, g, members, st);
    }
    ColSumArgs cz = c;
    cz.src_bf16 = dzs[l]; cz.src_f32 = nullptr; cz.src_stride = a.act_stride; cz.ld = kMlpH;
    cz.wgt = nullptr; cz.ncols = kMlpH; cz.out = grads + boff[l];
    if (e == hipSuccess) e = launch_colsum(cz, members, st);
    GemmArgs d = gemm_base();
    d.A = dzs[l]; d.lda = kMlpH; d.sA = a.act_stride;      // A[b][out] = dz
    d.B = wb[l]; d.ldb = kMlpH; d.sB = (int64_t)kMlpH * kMlpH;   // B[in][out] = W
    d.M = a.batch; d.N = kMlpH; d.K = kMlpH;
    d.H = dzp[l]; d.ldh = kMlpH; d.sH = a.act_stride;
    d.HT = dzpT[l]; d.ldht = a.ldT; d.sHT = a.actT_stride;
    d.Zp = zp[l]; d.ldz = kMlpH; d.sZ = a.act_stride;
    if (e == hipSuccess) e = launch_gemm(kEpiDh, d, members, st);
  }
  // first layer
  ColSumArgs c1 = c;
  c1.src_bf16 = a.dz1; c1.src_stride = a.act_stride; c1.ld = kMlpH; c1.wgt = nullptr; c1.ncols = kMlpH;
  c1.out = grads + kOffB1;
  if (e == hipSuccess) e = launch_colsum(c1, members, st);
  if (e == hipSuccess) e = launch_layer1_bwd(a, v.part, max_parts(m->cap), grads, ps, members, st);
  return e;
}

bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

extern "C" int64_t msb_mlp_num_params(void) { return kMlpParams; }

extern "C" msb_status msb_mlp_create(int members, const double* in_shift, const double* in_scale,
                                     double out_scale, msb_mlp** out) {
  (void)hipGetLastError();
  if (!out || !in_shift || !in_scale) return fail(MSB_EINVAL, "msb_mlp_create: null argument");
  *out = nullptr;
  if (members < 1 || members > 64) return fail(MSB_EINVAL, "msb_mlp_create: members must lie in [1, 64]");
  if (!(std::isfinite(out_scale) && out_scale > 0)) return fail(MSB_EINVAL, "msb_mlp_create: out_scale must be positive");
  float hin[2 * kMlpIn];
  for (int k = 0; k < kMlpIn; ++k) {
    if (!std::isfinite(in_shift[k]) || !std::isfinite(in_scale[k]))
      return fail(MSB_EINVAL, "msb_mlp_create: non-finite input normalisation");
    hin[k] = (float)in_shift[k];
    hin[kMlpIn + k] = (float)in_scale[k];
  }
  msb_mlp* m = new msb_mlp();
  m->members = members;
  m->pstride = (kMlpParams + 63) / 64 * 64;
  m->out_scale = (float)out_scale;
  const size_t pb = (size_t)members * m->pstride * sizeof(float);
  const size_t wb = (size_t)members * kMlpH * kMlpH * sizeof(__bf16);
  hipError_t e = hipMalloc(&m->d_in, sizeof(hin));
  if (e == hipSuccess) e = hipMalloc(&m->params, pb);
  if (e == hipSuccess) e = hipMalloc(&m->grads, pb);
  if (e == hipSuccess) e = hipMalloc(&m->adam_m, pb);
  if (e == hipSuccess) e = hipMalloc(&m->adam_v, pb);
  if (e == hipSuccess) e = hipMalloc(&m->w2b, wb);
  if (e == hipSuccess) e = hipMalloc(&m->w3b, wb);
  if (e == hipSuccess) e = hipMalloc(&m->w2t, wb);
  if (e == hipSuccess) e = hipMalloc(&m->w3t, wb);
  if (e == hipSuccess) e = hipMalloc(&m->step, sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&m->zero_step, sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&m->call_step, sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(m->d_in, hin, sizeof(hin), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->params, 0, pb);
  if (e == hipSuccess) e = hipMemset(m->grads, 0, pb);
  if (e == hipSuccess) e = hipMemset(m->adam_m, 0, pb);
  if (e == hipSuccess) e = hipMemset(m->adam_v, 0, pb);
  if (e == hipSuccess) e = hipMemset(m->step, 0, sizeof(int));
  if (e == hipSuccess) e = hipMemset(m->zero_step, 0, sizeof(int));
  if (e == hipSuccess) e = hipMemset(m->call_step, 0, sizeof(int));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = launch_weights_bf16(m->params, m->pstride, m->w2b, m->w3b, m->w2t, m->w3t, members, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    msb_mlp_destroy(m);
    return fail(MSB_EHIP, std::string("msb_mlp_create: ") + hipGetErrorString(e));
  }
  *out = m;
  return MSB_OK;
}

extern "C" void msb_mlp_destroy(msb_mlp* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  for (void* p : {(void*)m->d_in, (void*)m->params, (void*)m->grads, (void*)m->adam_m, (void*)m->adam_v,
                  (void*)m->w2b, (void*)m->w3b, (void*)m->w2t, (void*)m->w3t, (void*)m->step, (void*)m->zero_step, (void*)m->call_step,
                  m->act})
    if (p) (void)hipFree(p);
  if (m->stream) (void)hipStreamDestroy(m->stream);
  delete m;
}

extern "C" msb_status msb_mlp_set_params(msb_mlp* m, int member, const float* params) {
  (void)hipGetLastError();
  if (!m || !params) return fail(MSB_EINVAL, "msb_mlp_set_params: null argument");
  if (member < 0 || member >= m->members) return fail(MSB_EINVAL, "msb_mlp_set_params: member out of range");
  if (!finite_all(params, kMlpParams)) return fail(MSB_EINVAL, "msb_mlp_set_params: non-finite parameter");
  const int64_t o = (int64_t)member * m->pstride;
  MSB_HIP(hipMemcpy(m->params + o, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice));
  MSB_HIP(hipMemset(m->adam_m + o, 0, kMlpParams * sizeof(float)));
  MSB_HIP(hipMemset(m->adam_v + o, 0, kMlpParams * sizeof(float)));
  MSB_HIP(hipMemset(m->step, 0, sizeof(int)));
  MSB_HIP(launch_weights_bf16(m->params, m->pstride, m->w2b, m->w3b, m->w2t, m->w3t, m->members, m->stream));
  MSB_HIP(hipStreamSynchronize(m->stream));
  return MSB_OK;
}

extern "C" msb_status msb_mlp_get_params(const msb_mlp* m, int member, float* params) {
  (void)hipGetLastError();
  if (!m || !params) return fail(MSB_EINVAL, "msb_mlp_get_params: null argument");
  if (member < 0 || member >= m->members) return fail(MSB_EINVAL, "msb_mlp_get_params: member out of range");
  MSB_HIP(hipMemcpy(params, m->params + (int64_t)member * m->pstride, kMlpParams * sizeof(float),
                    hipMemcpyDeviceToHost));
  return MSB_OK;
}

extern "C" msb_status msb_mlp_grad(msb_mlp* m, int member, const float* X, const float* T, int n,
                                   double* loss, float* grad) {
  (void)hipGetLastError();
  if (!m || !X || !T || !grad) return fail(MSB_EINVAL, "msb_mlp_grad: null argument");
  if (member < 0 || member >= m->members) return fail(MSB_EINVAL, "msb_mlp_grad: member out of range");
  if (n < 1 || n > kMaxRows) return fail(MSB_EINVAL, "msb_mlp_grad: n out of range");
  const int rows = (n + 127) / 128 * 128;
  msb_status r = ensure_cap(m, rows);
  if (r != MSB_OK) return r;
  hipStream_t st = m->stream;
  ActView v = carve(m);
  MlpFwdArgs a = fwd_args(m, v, X, T, rows, n);
  MSB_HIP(forward(m, member, 1, a, st));
  MSB_HIP(backward(m, member, 1, a, v, st));
  std::vector<double> lp(rows / 4);
  MSB_HIP(hipMemcpyAsync(lp.data(), v.loss_part, lp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  MSB_HIP(hipMemcpyAsync(grad, m->grads + (int64_t)member * m->pstride, kMlpParams * sizeof(float),
                         hipMemcpyDeviceToHost, st));
  MSB_HIP(hipStreamSynchronize(st));
  if (loss) {
    double s = 0.0;
    for (double x : lp) s += x;
    *loss = s / n;
  }
  return MSB_OK;
}

extern "C" msb_status msb_mlp_train(msb_mlp* m, const float* X, const float* T, int64_t n_points,
                                    const int* perm, int batch, int steps, double lr, double* loss_hist,
                                    void* stream) {
  (void)hipGetLastError();
  if (!m || !X || !T || !perm) return fail(MSB_EINVAL, "msb_mlp_train: null argument");
  if (batch < 128 || batch % 128 || batch > kMaxRows)
    return fail(MSB_EINVAL, "msb_mlp_train: batch must be a multiple of 128 in [128, 131072]");
  if (steps < 1 || n_points < 1) return fail(MSB_EINVAL, "msb_mlp_train: steps and n_points must be positive");
  if (!(lr > 0) || !std::isfinite(lr)) return fail(MSB_EINVAL, "msb_mlp_train: lr must be positive");
  msb_status r = ensure_cap(m, batch);
  if (r != MSB_OK) return r;
  MSB_HIP(hipStreamSynchronize((hipStream_t)stream));   // inputs complete on the caller's stream
  hipStream_t st = m->stream;
  ActView v = carve(m);
  MlpFwdArgs a = fwd_args(m, v, X, T, batch, batch);
  a.perm = perm;
  a.perm_stride = (int64_t)steps * batch;
  MSB_HIP(hipMemsetAsync(m->call_step, 0, sizeof(int), st));
  a.step = m->call_step;
  double* d_hist = nullptr;
  MSB_HIP(hipMalloc(&d_hist, (size_t)m->members * steps * sizeof(double)));
  struct Free {
    double* p;
    ~Free() { if (p) (void)hipFree(p); }
  } free_hist{d_hist};
  AdamArgs ad;
  ad.params = m->params; ad.grads = m->grads; ad.m = m->adam_m; ad.v = m->adam_v; ad.pstride = m->pstride;
  ad.w2b = m->w2b; ad.w3b = m->w3b; ad.w2t = m->w2t; ad.w3t = m->w3t;
  ad.step = m->step; ad.call_step = m->call_step;
  ad.lr = (float)lr; ad.b1 = 0.9f; ad.b2 = 0.999f; ad.eps = 1e-8f;
  auto enqueue_step = [&]() -> hipError_t {
    hipError_t e = forward(m, 0, m->members, a, st);
    if (e == hipSuccess) e = launch_loss_record(a, d_hist, steps, m->members, st);
    if (e == hipSuccess) e = backward(m, 0, m->members, a, v, st);
    if (e == hipSuccess) e = launch_adam(ad, m->members, st);
    return e;
  };
  // one step captured in a hipGraph and replayed: the step counter on the
  // device selects the permutation slice, the loss slot and Adam's step
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  MSB_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const hipError_t e_launch = enqueue_step();
  const hipError_t e_end = hipStreamEndCapture(st, &g);
  hipError_t e_inst = hipSuccess;
  if (e_launch == hipSuccess && e_end == hipSuccess) e_inst = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  MSB_HIP(e_launch);
  MSB_HIP(e_end);
  MSB_HIP(e_inst);
  hipError_t e = hipSuccess;
  for (int s = 0; s < steps && e == hipSuccess; ++s) e = hipGraphLaunch(ge, st);
  (void)hipGraphExecDestroy(ge);
  MSB_HIP(e);
  if (loss_hist)
    MSB_HIP(hipMemcpyAsync(loss_hist, d_hist, (size_t)m->members * steps * sizeof(double), hipMemcpyDeviceToHost, st));
  MSB_HIP(hipStreamSynchronize(st));
  return MSB_OK;
}

extern "C" msb_status msb_mlp_predict(msb_mlp* m, const float* X, int64_t n, float* mean, float* sd,
                                      void* stream) {
  (void)hipGetLastError();
  if (!m || !X || !mean || !sd) return fail(MSB_EINVAL, "msb_mlp_predict: null argument");
  if (n < 1) return fail(MSB_EINVAL, "msb_mlp_predict: n must be positive");
  const int chunk = 32768;
  msb_status r = ensure_cap(m, std::max(m->cap, chunk));
  if (r != MSB_OK) return r;
  MSB_HIP(hipStreamSynchronize((hipStream_t)stream));
  hipStream_t st = m->stream;
  ActView v = carve(m);
  for (int64_t b0 = 0; b0 < n; b0 += chunk) {
    const int valid = (int)std::min<int64_t>(chunk, n - b0);
    const int rows = (valid + 127) / 128 * 128;
    MlpFwdArgs a = fwd_args(m, v, X, nullptr, rows, valid);
    a.base = b0;
    a.z1 = a.z2 = a.z3 = nullptr;     // inference keeps neither gelu'(z) nor transposed copies
    a.h1T = a.h2T = nullptr;
    MSB_HIP(forward(m, 0, m->members, a, st));
    MSB_HIP(launch_ensemble_stats(v.y, v.y_stride, m->members, valid, 1.0f / m->out_scale, mean + b0, sd + b0, st));
  }
  MSB_HIP(hipStreamSynchronize(st));
  return MSB_OK;
}

extern "C" msb_status msb_mlp_fallback(const float* mean, const float* sd, int n_rows, int n_cols, double frac,
                                       int* row_mask) {
  if (!mean || !sd || !row_mask) return fail(MSB_EINVAL, "msb_mlp_fallback: null argument");
  if (n_rows < 1 || n_cols < 1 || !(frac > 0)) return fail(MSB_EINVAL, "msb_mlp_fallback: bad sizes");
  float peak = -INFINITY;
  for (int64_t i = 0; i < (int64_t)n_rows * n_cols; ++i) peak = std::max(peak, mean[i]);
  const double thr = frac * (double)peak;
  for (int r = 0; r < n_rows; ++r) {
    int f = 0;
    for (int c = 0; c < n_cols && !f; ++c) f = (double)sd[(int64_t)r * n_cols + c] > thr;
    row_mask[r] = f;
  }
  return MSB_OK;
}
