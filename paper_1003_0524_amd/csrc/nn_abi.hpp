// Host runtime and C ABI of the learned V^x extrapolator (included by
// exchange.hip after the exchange-matrix entry points; shares its context,
// error and allocation helpers). Kernels: nn.hpp.
#pragma once
#include "nn.hpp"

struct NnState {
  int I = 0, H = 0, O = 0;
  long off[7] = {0, 0, 0, 0, 0, 0, 0};       // [W1, b1, W2, b2, W3, b3, end]
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
  int32_t* step = nullptr;
  int cap = 0;                               // batch capacity of the buffers below
  float *X = nullptr, *T = nullptr, *h1 = nullptr, *h2 = nullptr, *y = nullptr, *dy = nullptr;
  float *dz2 = nullptr, *dz1 = nullptr;
  hipGraphExec_t gexec = nullptr;            // one training epoch
  int g_n = -1;
  float g_lr = 0.f;
};

struct LearnScratch {
  // eigensolver
  double2* work = nullptr; size_t work_n = 0;
  int64_t *z_off = nullptr, *w_off = nullptr;
  int32_t* sweeps = nullptr;
  // pointer tables [n_k]
  const void** tabA = nullptr; const void** tabB = nullptr; void** tabC = nullptr;
  // sketch partials
  double* part = nullptr; size_t part_n = 0;
};

namespace {

void free_nn(NnState* s) {
  if (!s) return;
  if (s->gexec) hipGraphExecDestroy(s->gexec);
  void* p[] = {s->theta, s->grad, s->m, s->v, s->loss, s->step, s->X, s->T,
               s->h1, s->h2, s->y, s->dy, s->dz2, s->dz1};
  for (void* q : p) if (q) hipFree(q);
  delete s;
}

void release_learned(exc_ctx* c) {
  free_nn(c->nn);
  c->nn = nullptr;
  if (LearnScratch* l = c->ls) {
    void* p[] = {l->work, l->z_off, l->w_off, l->sweeps, (void*)l->tabA, (void*)l->tabB,
                 (void*)l->tabC, l->part};
    for (void* q : p) if (q) hipFree(q);
    delete l;
  }
  c->ls = nullptr;
}

exc_status nn_reserve(exc_ctx* c, int n) {
  NnState* s = c->nn;
  if (n <= s->cap) return EXC_OK;
  float** bufs[] = {&s->X, &s->T, &s->h1, &s->h2, &s->y, &s->dy, &s->dz2, &s->dz1};
  for (float** b : bufs) { if (*b) hipFree(*b); *b = nullptr; }
  if (s->gexec) { hipGraphExecDestroy(s->gexec); s->gexec = nullptr; s->g_n = -1; }
  const size_t n_ = (size_t)n;
  TRY(dalloc(c, &s->X, n_ * s->I));
  TRY(dalloc(c, &s->T, n_ * s->O));
  TRY(dalloc(c, &s->h1, n_ * s->H));
  TRY(dalloc(c, &s->h2, n_ * s->H));
  TRY(dalloc(c, &s->y, n_ * s->O));
  TRY(dalloc(c, &s->dy, n_ * s->O));
  TRY(dalloc(c, &s->dz2, n_ * s->H));
  TRY(dalloc(c, &s->dz1, n_ * s->H));
  s->cap = n;
  return EXC_OK;
}

template <bool TA, bool TB, int EPI>
void gemm(hipStream_t st, const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N,
          int K, const float* bias = nullptr, const float* aux = nullptr, int ldaux = 0) {
  GemmArgs g{A, B, C, bias, aux, lda, ldb, ldc, ldaux, M, N, K};
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((nn_gemm<TA, TB, EPI>), grid, dim3(256), 0, st, g);
}

void nn_forward(NnState* s, hipStream_t st, const float* X, int n, float* y) {
  const float* th = s->theta;
  gemm<false, true, EPI_BIAS_TANH>(st, X, s->I, th + s->off[0], s->I, s->h1, s->H, n, s->H, s->I, th + s->off[1]);
  gemm<false, true, EPI_BIAS_TANH>(st, s->h1, s->H, th + s->off[2], s->H, s->h2, s->H, n, s->H, s->H, th + s->off[3]);
  gemm<false, true, EPI_BIAS>(st, s->h2, s->H, th + s->off[4], s->H, y, s->O, n, s->O, s->H, th + s->off[5]);
}

// forward, loss and dL/dtheta into s->grad (inputs in s->X, s->T)
void nn_backward(NnState* s, hipStream_t st, int n, int advance) {
  const float* th = s->theta;
  float* g = s->grad;
  nn_forward(s, st, s->X, n, s->y);
  hipLaunchKernelGGL(nn_loss_grad, dim3(1), dim3(256), 0, st, s->y, s->T, s->dy, (long)n * s->O, s->loss,
                     s->step, advance);
  // output layer
  gemm<true, false, EPI_NONE>(st, s->dy, s->O, s->h2, s->H, g + s->off[4], s->H, s->O, s->H, n);
  hipLaunchKernelGGL(nn_colsum, dim3((s->O + 255) / 256), dim3(256), 0, st, s->dy, s->O, n, s->O, g + s->off[5]);
  // second hidden layer
  gemm<false, false, EPI_DTANH>(st, s->dy, s->O, th + s->off[4], s->H, s->dz2, s->H, n, s->H, s->O, nullptr,
                                s->h2, s->H);
  gemm<true, false, EPI_NONE>(st, s->dz2, s->H, s->h1, s->H, g + s->off[2], s->H, s->H, s->H, n);
  hipLaunchKernelGGL(nn_colsum, dim3((s->H + 255) / 256), dim3(256), 0, st, s->dz2, s->H, n, s->H, g + s->off[3]);
  // first hidden layer
  gemm<false, false, EPI_DTANH>(st, s->dz2, s->H, th + s->off[2], s->H, s->dz1, s->H, n, s->H, s->H, nullptr,
                                s->h1, s->H);
  gemm<true, false, EPI_NONE>(st, s->dz1, s->H, s->X, s->I, g + s->off[0], s->I, s->H, s->I, n);
  hipLaunchKernelGGL(nn_colsum, dim3((s->H + 255) / 256), dim3(256), 0, st, s->dz1, s->H, n, s->H, g + s->off[1]);
}

void nn_epoch(NnState* s, hipStream_t st, int n, float lr) {
  nn_backward(s, st, n, 1);
  const long np = s->off[6];
  hipLaunchKernelGGL(nn_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, s->theta, s->grad, s->m, s->v,
                     np, s->step, lr);
}

exc_status nn_check(exc_ctx* c) {
  TRY(check_ctx(c));
  if (!c->nn) return fail(c, EXC_ESTATE, "exchange_nn_init has not been called");
  return EXC_OK;
}

exc_status nn_stage(exc_ctx* c, float* dst, const float* src, size_t count, int on_device, hipStream_t st) {
  HIPCHK(c, hipMemcpyAsync(dst, src, count * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  return EXC_OK;
}

exc_status learn_scratch(exc_ctx* c) {
  if (c->ls) return EXC_OK;
  c->ls = new LearnScratch();
  LearnScratch* l = c->ls;
  std::vector<int64_t> zo(c->n_k), wo(c->n_k);
  int64_t z = 0, w = 0;
  for (int k = 0; k < c->n_k; ++k) { zo[k] = z; wo[k] = w; z += (int64_t)c->nb[k] * c->nb[k]; w += c->nb[k]; }
  l->work_n = (size_t)z;
  TRY(dalloc(c, &l->work, l->work_n));
  TRY(upload(c, &l->z_off, zo));
  TRY(upload(c, &l->w_off, wo));
  TRY(dalloc(c, &l->sweeps, (size_t)c->n_k));
  TRY(dalloc(c, (void***)&l->tabA, (size_t)c->n_k));
  TRY(dalloc(c, (void***)&l->tabB, (size_t)c->n_k));
  TRY(dalloc(c, &l->tabC, (size_t)c->n_k));
  return EXC_OK;
}

// Copies a host array of n_k device pointers into a device table. The stream
// is drained first: a previous call's kernels may still read the table.
exc_status put_table(exc_ctx* c, void* dtab, const void* const* h, hipStream_t st) {
  if (!h) return fail(c, EXC_EINVAL, "pointer table is NULL");
  for (int k = 0; k < c->n_k; ++k)
    if (!h[k]) return fail(c, EXC_EINVAL, "pointer for k=%d is NULL", k);
  HIPCHK(c, hipStreamSynchronize(st));
  HIPCHK(c, hipMemcpy(dtab, h, c->n_k * sizeof(void*), hipMemcpyHostToDevice));
  return EXC_OK;
}

}  // namespace

extern "C" {

exc_status exchange_nn_init(exc_ctx* c, int32_t in_dim, int32_t hidden, int32_t out_dim, uint64_t seed) {
  TRY(check_ctx(c));
  if (in_dim < 1 || hidden < 1 || out_dim < 1 || in_dim > 65536 || hidden > 8192 || out_dim > (1 << 20))
    return fail(c, EXC_EINVAL, "network sizes out of range (in %d, hidden %d, out %d)", in_dim, hidden, out_dim);
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipDeviceSynchronize());
  free_nn(c->nn);
  c->nn = new NnState();
  NnState* s = c->nn;
  s->I = in_dim; s->H = hidden; s->O = out_dim;
  const long sz[6] = {(long)hidden * in_dim, hidden, (long)hidden * hidden, hidden, (long)out_dim * hidden, out_dim};
  s->off[0] = 0;
  for (int i = 0; i < 6; ++i) s->off[i + 1] = s->off[i] + sz[i];
  const size_t np = (size_t)s->off[6];
  exc_status st = EXC_OK;
  if ((st = dalloc(c, &s->theta, np)) || (st = dalloc(c, &s->grad, np)) || (st = dalloc(c, &s->m, np)) ||
      (st = dalloc(c, &s->v, np)) || (st = dalloc(c, &s->loss, 1)) || (st = dalloc(c, &s->step, 1))) {
    free_nn(c->nn);
    c->nn = nullptr;
    return st;
  }
  HIPCHK(c, hipMemset(s->m, 0, np * sizeof(float)));
  HIPCHK(c, hipMemset(s->v, 0, np * sizeof(float)));
  HIPCHK(c, hipMemset(s->step, 0, sizeof(int32_t)));
  InitArgs a;
  for (int i = 0; i < 7; ++i) a.off[i] = s->off[i];
  a.fan[0] = in_dim; a.fan[1] = hidden; a.fan[2] = hidden;
  hipLaunchKernelGGL(nn_init_params, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, nullptr, s->theta, a, seed);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipDeviceSynchronize());
  return EXC_OK;
}

exc_status exchange_nn_params(exc_ctx* c, float* params, int64_t n, int32_t set, int32_t on_device) {
  TRY(nn_check(c));
  NnState* s = c->nn;
  if (!params || n != s->off[6])
    return fail(c, EXC_EINVAL, "params must hold exactly %ld floats", s->off[6]);
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipDeviceSynchronize());
  const size_t b = (size_t)n * sizeof(float);
  if (set) {
    HIPCHK(c, hipMemcpy(s->theta, params, b, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    HIPCHK(c, hipMemset(s->m, 0, b));       // a new starting point: Adam starts afresh
    HIPCHK(c, hipMemset(s->v, 0, b));
    HIPCHK(c, hipMemset(s->step, 0, sizeof(int32_t)));
  } else {
    HIPCHK(c, hipMemcpy(params, s->theta, b, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  }
  return EXC_OK;
}

exc_status exchange_nn_grad(exc_ctx* c, const float* X, const float* Y, int32_t n, int32_t on_device,
                            float* grad_out, float* loss_out) {
  TRY(nn_check(c));
  NnState* s = c->nn;
  if (!X || !Y || !grad_out || n < 1) return fail(c, EXC_EINVAL, "X, Y, grad_out non-NULL and n >= 1 required");
  HIPCHK(c, hipSetDevice(c->device));
  TRY(nn_reserve(c, n));
  hipStream_t st = c->own;
  TRY(nn_stage(c, s->X, X, (size_t)n * s->I, on_device, st));
  TRY(nn_stage(c, s->T, Y, (size_t)n * s->O, on_device, st));
  nn_backward(s, st, n, 0);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(grad_out, s->grad, s->off[6] * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  float l = 0.f;
  HIPCHK(c, hipMemcpyAsync(&l, s->loss, sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if (loss_out) *loss_out = l;
  return EXC_OK;
}

exc_status exchange_nn_train(exc_ctx* c, const float* X, const float* Y, int32_t n, int32_t epochs, float lr,
                             int32_t on_device, float* loss_out) {
  TRY(nn_check(c));
  NnState* s = c->nn;
  if (!X || !Y || n < 1 || epochs < 0 || !(lr > 0.f))
    return fail(c, EXC_EINVAL, "X, Y non-NULL, n >= 1, epochs >= 0 and lr > 0 required");
  HIPCHK(c, hipSetDevice(c->device));
  TRY(nn_reserve(c, n));
  hipStream_t st = c->own;
  TRY(nn_stage(c, s->X, X, (size_t)n * s->I, on_device, st));
  TRY(nn_stage(c, s->T, Y, (size_t)n * s->O, on_device, st));
  if (epochs > 0 && (!s->gexec || s->g_n != n || s->g_lr != lr)) {
    // one epoch (forward, loss, backward, Adam: kernels only) as a graph, replayed per epoch
    if (s->gexec) { hipGraphExecDestroy(s->gexec); s->gexec = nullptr; }
    HIPCHK(c, hipStreamSynchronize(st));
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    nn_epoch(s, st, n, lr);
    const hipError_t e1 = hipStreamEndCapture(st, &g);
    if (e1 != hipSuccess) return fail(c, EXC_EHIP, "capturing the training epoch failed: %s", hipGetErrorString(e1));
    const hipError_t e2 = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e2 != hipSuccess) {
      s->gexec = nullptr;
      return fail(c, EXC_EHIP, "instantiating the training graph failed: %s", hipGetErrorString(e2));
    }
    s->g_n = n;
    s->g_lr = lr;
  }
  for (int e = 0; e < epochs; ++e) HIPCHK(c, hipGraphLaunch(s->gexec, st));
  float l = 0.f;
  HIPCHK(c, hipMemcpyAsync(&l, s->loss, sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  if (loss_out) *loss_out = l;
  return EXC_OK;
}

exc_status exchange_nn_predict(exc_ctx* c, const float* X, int32_t n, float* Y_out, int32_t on_device,
                               void* stream) {
  TRY(nn_check(c));
  NnState* s = c->nn;
  if (!X || !Y_out || n < 1) return fail(c, EXC_EINVAL, "X, Y_out non-NULL and n >= 1 required");
  HIPCHK(c, hipSetDevice(c->device));
  TRY(nn_reserve(c, n));
  hipStream_t st = stream ? (hipStream_t)stream : c->own;
  if (stream) HIPCHK(c, hipStreamSynchronize(c->own));   // a training run may still use the buffers
  TRY(nn_stage(c, s->X, X, (size_t)n * s->I, on_device, st));
  nn_forward(s, st, s->X, n, s->y);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(Y_out, s->y, (size_t)n * s->O * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  if (!on_device || !stream) HIPCHK(c, hipStreamSynchronize(st));
  return EXC_OK;
}

exc_status exchange_nn_features(exc_ctx* c, const double* P_new, const double* P_old, int64_t n_real,
                                uint64_t seed, int32_t m, float* x_out, double* norm_out, void* stream) {
  TRY(check_ctx(c));
  if (!P_new || !P_old || !x_out || !norm_out || n_real < 1 || m < 1 || m > SK_MMAX)
    return fail(c, EXC_EINVAL, "device pointers non-NULL, n_real >= 1 and 1 <= m <= %d required", SK_MMAX);
  HIPCHK(c, hipSetDevice(c->device));
  TRY(learn_scratch(c));
  LearnScratch* l = c->ls;
  hipStream_t st = stream ? (hipStream_t)stream : c->own;
  const long nchunk = (long)((n_real + SK_CHUNK - 1) / SK_CHUNK);
  const size_t need = (size_t)nchunk * (m + 1);
  if (need > l->part_n) {
    HIPCHK(c, hipStreamSynchronize(st));
    if (l->part) hipFree(l->part);
    l->part = nullptr;
    l->part_n = 0;
    TRY(dalloc(c, &l->part, need));
    l->part_n = need;
  }
  hipLaunchKernelGGL(nn_sketch_partial, dim3((unsigned)nchunk), dim3(256), 0, st, P_new, P_old, (long)n_real, m,
                     seed, l->part);
  hipLaunchKernelGGL(nn_sketch_final, dim3(1), dim3(128), 0, st, l->part, (int)nchunk, m, x_out, norm_out);
  HIPCHK(c, hipGetLastError());
  if (!stream) HIPCHK(c, hipStreamSynchronize(st));
  return EXC_OK;
}

exc_status exchange_eigh(exc_ctx* c, const void* const* A_k, double* w_out, void* Z_out, void* stream) {
  TRY(check_ctx(c));
  if (!A_k || !w_out || !Z_out) return fail(c, EXC_EINVAL, "A_k, w_out and Z_out must be non-NULL");
  if (c->nb_max > EIGH_NMAX) return fail(c, EXC_EUNSUPPORTED, "eigensolver limited to n_b <= %d", EIGH_NMAX);
  HIPCHK(c, hipSetDevice(c->device));
  TRY(learn_scratch(c));
  LearnScratch* l = c->ls;
  hipStream_t st = stream ? (hipStream_t)stream : c->own;
  TRY(put_table(c, (void*)l->tabA, A_k, st));
  EighArgs a{(const double2* const*)l->tabA, c->d_knb, l->work, (double2*)Z_out, l->z_off, w_out, l->w_off,
             l->sweeps};
  hipLaunchKernelGGL(eigh_jacobi, dim3(c->n_k), dim3(256), 0, st, a);
  HIPCHK(c, hipGetLastError());
  if (!stream) HIPCHK(c, hipStreamSynchronize(st));
  return EXC_OK;
}

exc_status exchange_nn_project(exc_ctx* c, const void* const* Va_k, const void* const* Vb_k, const void* Z,
                               int32_t n_blk, double scale, float* y_out, void* stream) {
  TRY(check_ctx(c));
  if (!Z || !y_out || n_blk < 1) return fail(c, EXC_EINVAL, "Z, y_out non-NULL and n_blk >= 1 required");
  if ((size_t)c->nb_max * n_blk * sizeof(double2) > 65536)
    return fail(c, EXC_EUNSUPPORTED, "n_b * n_blk = %d * %d exceeds the 4096 complex entries staged in LDS",
                c->nb_max, n_blk);
  for (int k = 0; k < c->n_k; ++k)
    if (n_blk > c->nb[k]) return fail(c, EXC_EINVAL, "n_blk %d exceeds n_b(k=%d) = %d", n_blk, k, c->nb[k]);
  HIPCHK(c, hipSetDevice(c->device));
  TRY(learn_scratch(c));
  LearnScratch* l = c->ls;
  hipStream_t st = stream ? (hipStream_t)stream : c->own;
  TRY(put_table(c, (void*)l->tabA, Va_k, st));
  TRY(put_table(c, (void*)l->tabB, Vb_k, st));
  ProjArgs a{(const double2* const*)l->tabA, (const double2* const*)l->tabB, (const double2*)Z, l->z_off,
             c->d_knb, n_blk, scale, y_out, nullptr, nullptr};
  const size_t lds = (size_t)c->nb_max * n_blk * sizeof(double2);
  hipLaunchKernelGGL(nn_project, dim3(c->n_k), dim3(256), lds, st, a);
  HIPCHK(c, hipGetLastError());
  if (!stream) HIPCHK(c, hipStreamSynchronize(st));
  return EXC_OK;
}

exc_status exchange_nn_expand(exc_ctx* c, const void* const* Vanchor_k, const void* Z, int32_t n_blk,
                              const float* y, double scale, void* const* Vout_k, void* stream) {
  TRY(check_ctx(c));
  if (!Z || !y || n_blk < 1) return fail(c, EXC_EINVAL, "Z, y non-NULL and n_blk >= 1 required");
  if ((size_t)c->nb_max * n_blk * sizeof(double2) > 65536)
    return fail(c, EXC_EUNSUPPORTED, "n_b * n_blk = %d * %d exceeds the 4096 complex entries staged in LDS",
                c->nb_max, n_blk);
  for (int k = 0; k < c->n_k; ++k)
    if (n_blk > c->nb[k]) return fail(c, EXC_EINVAL, "n_blk %d exceeds n_b(k=%d) = %d", n_blk, k, c->nb[k]);
  HIPCHK(c, hipSetDevice(c->device));
  TRY(learn_scratch(c));
  LearnScratch* l = c->ls;
  hipStream_t st = stream ? (hipStream_t)stream : c->own;
  TRY(put_table(c, (void*)l->tabA, Vanchor_k, st));
  TRY(put_table(c, (void*)l->tabC, (const void* const*)Vout_k, st));
  ProjArgs a{nullptr, nullptr, (const double2*)Z, l->z_off, c->d_knb, n_blk, scale, const_cast<float*>(y),
             (const double2* const*)l->tabA, (double2* const*)l->tabC};
  const size_t lds = (size_t)c->nb_max * n_blk * sizeof(double2);
  hipLaunchKernelGGL(nn_expand, dim3(c->n_k), dim3(256), lds, st, a);
  HIPCHK(c, hipGetLastError());
  if (!stream) HIPCHK(c, hipStreamSynchronize(st));
  return EXC_OK;
}

}  // extern "C"
