// Host side of the learned surrogate: parameter layout, workspace, and the
// forward, backward and Adam sequences of the Eq. 6.10 layers.
#include "../../include/lsfft_fno.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "fno_launch.hpp"

using namespace lsfft_fno;

namespace {

constexpr int kMaxLayers = 8;

int round_up(int v, int m) { return (v + m - 1) / m * m; }

bool arch_ok(const lsfft_fno_arch* a) {
  if (!a) return false;
  if (a->n != 8 && a->n != 16 && a->n != 32) return false;
  if (a->modes < 1 || 2 * a->modes > a->n) return false;
  if (a->width != kWidth) return false;
  if (a->hidden < 32 || a->hidden > 256 || a->hidden % 32) return false;
  if (a->cin < 1 || a->cin > 32 || a->cout < 1 || a->cout > 32) return false;
  if (a->layers < 1 || a->layers > kMaxLayers) return false;
  return true;
}

// A pointwise layer: packed offsets of w [O][I] and b [O], and its bf16
// copies for the forward product (w, [opad][ipad]) and the backward data
// product (w^T, [t_opad][t_ipad]).
struct Pw {
  long long w_off = 0, b_off = 0;
  int O = 0, I = 0;
  int opad = 0, ipad = 0, t_opad = 0, t_ipad = 0;
  __hip_bfloat16* wb = nullptr;
  __hip_bfloat16* wbt = nullptr;
};

struct Layout {
  Pw lift, hid[kMaxLayers], proj1, proj2;
  long long r_off[kMaxLayers] = {0};
  long long nparam = 0;
  int nmodes = 0;
};

Layout make_layout(const lsfft_fno_arch& a) {
  Layout L;
  long long off = 0;
  auto pw = [&](Pw& p, int O, int I) {
    p.O = O;
    p.I = I;
    p.w_off = off;
    off += (long long)O * I;
    p.b_off = off;
    off += O;
    p.opad = round_up(O, 32);
    p.ipad = round_up(I, 16);
    p.t_opad = round_up(I, 32);
    p.t_ipad = round_up(O, 16);
  };
  L.nmodes = 4 * a.modes * a.modes * a.modes;
  pw(L.lift, a.width, a.cin);
  for (int l = 0; l < a.layers; ++l) {
    pw(L.hid[l], a.width, a.width);
    L.r_off[l] = off;
    off += (long long)L.nmodes * a.width * a.width * 2;
  }
  pw(L.proj1, a.hidden, a.width);
  pw(L.proj2, a.cout, a.hidden);
  L.nparam = off;
  return L;
}

}  // namespace

struct lsfft_fno_s {
  lsfft_fno_arch a{};
  int max_batch = 0;
  hipStream_t stream = nullptr;
  long long V = 0;
  Layout L;
  int step = 0;
  float *params = nullptr, *grads = nullptr, *mom = nullptr, *vel = nullptr;
  __hip_bfloat16* rb[kMaxLayers] = {nullptr};
  // activations and temporaries for max_batch samples
  float* h[kMaxLayers + 1] = {nullptr};
  float* pre[kMaxLayers] = {nullptr};
  float2* Hm[kMaxLayers] = {nullptr};
  float *p1 = nullptr, *z = nullptr, *y = nullptr, *dy = nullptr, *dz = nullptr, *sbuf = nullptr;
  float* dbuf[2] = {nullptr, nullptr};
  float2 *t1 = nullptr, *t2 = nullptr, *ym = nullptr, *gm = nullptr, *tw = nullptr;
  float* wpart = nullptr;
  int wblk = 0;
  double* lpart = nullptr;
  double* loss_dev = nullptr;
  int nchunk = 0;
  std::vector<void*> allocs;
};

namespace {

#define FNO_TRY(expr)                            \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return LSFFT_E_DEVICE; \
  } while (0)

template <typename T>
bool alloc(lsfft_fno_s* f, T** p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
  f->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return true;
}

void release(lsfft_fno_s* f) {
  if (f->stream) (void)hipStreamSynchronize(f->stream);
  for (void* p : f->allocs) (void)hipFree(p);
  f->allocs.clear();
}

// bf16 operand copies of the master parameters
hipError_t prep_weights(lsfft_fno_s* f) {
  auto pw = [&](Pw& p) -> hipError_t {
    const float* w = f->params + p.w_off;
    hipError_t e = launch_cast_pad(w, p.O, p.I, p.I, 1, p.wb, p.opad, p.ipad, f->stream);
    if (e != hipSuccess) return e;
    return launch_cast_pad(w, p.I, p.O, 1, p.I, p.wbt, p.t_opad, p.t_ipad, f->stream);
  };
  hipError_t e;
  if ((e = pw(f->L.lift)) != hipSuccess) return e;
  for (int l = 0; l < f->a.layers; ++l) {
    if ((e = pw(f->L.hid[l])) != hipSuccess) return e;
    if ((e = launch_cast(f->params + f->L.r_off[l], f->rb[l], (long long)f->L.nmodes * kWidth * kWidth * 2,
                         f->stream)) != hipSuccess)
      return e;
  }
  if ((e = pw(f->L.proj1)) != hipSuccess) return e;
  return pw(f->L.proj2);
}

PwArgs pw_args(lsfft_fno_s* f, const Pw& p, bool transposed, const float* in, int B) {
  PwArgs a{};
  a.in = in;
  a.B = B;
  a.V = f->V;
  if (!transposed) {
    a.w = p.wb;
    a.I = p.I;
    a.ipad = p.ipad;
    a.O = p.O;
    a.opad = p.opad;
    a.bias = f->params + p.b_off;
  } else {
    a.w = p.wbt;
    a.I = p.O;
    a.ipad = p.t_ipad;
    a.O = p.I;
    a.opad = p.t_opad;
    a.bias = nullptr;
  }
  return a;
}

hipError_t wgrad(lsfft_fno_s* f, const Pw& p, const float* g, const float* h, int B) {
  WgArgs w{};
  w.g = g;
  w.h = h;
  w.part = f->wpart;
  w.O = p.O;
  w.I = p.I;
  w.opad = round_up(p.O, 32);
  w.ipad = round_up(p.I, 32);
  w.B = B;
  w.V = f->V;
  w.nblk = wgrad_blocks(B, f->V);
  return launch_wgrad(w, f->grads + p.w_off, f->grads + p.b_off, f->stream);
}

// forward pass; the output goes to `y`, the tape to the handle's buffers
hipError_t forward(lsfft_fno_s* f, int B, const float* x, float* y) {
  const lsfft_fno_arch& a = f->a;
  const int n = a.n, M = a.modes, BC = B * kWidth;
  const float inv_n3 = 1.0f / float(n * n * n);
  hipError_t e;
  PwArgs p = pw_args(f, f->L.lift, false, x, B);
  p.out = f->h[0];
  if ((e = launch_pointwise(p, f->stream)) != hipSuccess) return e;
  for (int l = 0; l < a.layers; ++l) {
    if ((e = launch_dft_forward(n, M, BC, f->h[l], f->t1, f->t2, f->Hm[l], 1.0f, 1.0f, f->tw, f->stream)) != hipSuccess)
      return e;
    if ((e = launch_modemix(0, f->Hm[l], f->rb[l], nullptr, reinterpret_cast<float*>(f->ym), f->L.nmodes, B,
                            f->stream)) != hipSuccess)
      return e;
    if ((e = launch_dft_inverse(n, M, BC, f->ym, f->t2, f->t1, f->sbuf, inv_n3, 2.0f * inv_n3, f->tw, f->stream)) !=
        hipSuccess)
      return e;
    p = pw_args(f, f->L.hid[l], false, f->h[l], B);
    p.add = f->sbuf;
    p.out = f->pre[l];
    p.out_act = f->h[l + 1];
    if ((e = launch_pointwise(p, f->stream)) != hipSuccess) return e;
  }
  p = pw_args(f, f->L.proj1, false, f->h[a.layers], B);
  p.out = f->p1;
  p.out_act = f->z;
  if ((e = launch_pointwise(p, f->stream)) != hipSuccess) return e;
  p = pw_args(f, f->L.proj2, false, f->z, B);
  p.out = y;
  return launch_pointwise(p, f->stream);
}

// loss and gradients of every parameter into f->grads
hipError_t backward(lsfft_fno_s* f, int B, const float* x, const float* t) {
  const lsfft_fno_arch& a = f->a;
  const int n = a.n, M = a.modes, BC = B * kWidth;
  const float inv_n3 = 1.0f / float(n * n * n);
  hipError_t e;
  if ((e = launch_loss(f->y, t, f->dy, B, (long long)a.cout * f->V, f->lpart, f->nchunk, f->loss_dev, f->stream)) !=
      hipSuccess)
    return e;
  // projection
  if ((e = wgrad(f, f->L.proj2, f->dy, f->z, B)) != hipSuccess) return e;
  PwArgs p = pw_args(f, f->L.proj2, true, f->dy, B);
  p.aux = f->p1;
  p.out = f->dz;
  if ((e = launch_pointwise(p, f->stream)) != hipSuccess) return e;
  if ((e = wgrad(f, f->L.proj1, f->dz, f->h[a.layers], B)) != hipSuccess) return e;
  int cur = 0;
  p = pw_args(f, f->L.proj1, true, f->dz, B);
  p.aux = f->pre[a.layers - 1];
  p.out = f->dbuf[cur];
  if ((e = launch_pointwise(p, f->stream)) != hipSuccess) return e;
  // hidden layers, last to first; dbuf[cur] holds the gradient of pre[l]
  for (int l = a.layers - 1; l >= 0; --l) {
    const float* dpre = f->dbuf[cur];
    const Pw& hl = f->L.hid[l];
    if ((e = wgrad(f, hl, dpre, f->h[l], B)) != hipSuccess) return e;
    if ((e = launch_dft_forward(n, M, BC, dpre, f->t1, f->t2, f->gm, inv_n3, 2.0f * inv_n3, f->tw, f->stream)) !=
        hipSuccess)
      return e;
    if ((e = launch_modemix(2, f->Hm[l], f->rb[l], f->gm, f->grads + f->L.r_off[l], f->L.nmodes, B, f->stream)) !=
        hipSuccess)
      return e;
    if ((e = launch_modemix(1, f->gm, f->rb[l], nullptr, reinterpret_cast<float*>(f->ym), f->L.nmodes, B,
                            f->stream)) != hipSuccess)
      return e;
    if ((e = launch_dft_inverse(n, M, BC, f->ym, f->t2, f->t1, f->sbuf, 1.0f, 1.0f, f->tw, f->stream)) != hipSuccess)
      return e;
    p = pw_args(f, hl, true, dpre, B);
    p.add = f->sbuf;
    p.aux = (l > 0) ? f->pre[l - 1] : nullptr;
    p.out = f->dbuf[cur ^ 1];
    if ((e = launch_pointwise(p, f->stream)) != hipSuccess) return e;
    cur ^= 1;
  }
  return wgrad(f, f->L.lift, f->dbuf[cur], x, B);
}

}  // namespace

extern "C" {

int64_t lsfft_fno_param_count(const lsfft_fno_arch* arch) {
  if (!arch_ok(arch)) return 0;
  return make_layout(*arch).nparam;
}

lsfft_status lsfft_fno_create(lsfft_fno_t* out, const lsfft_fno_arch* arch, int max_batch, void* hip_stream) {
  if (!out) return LSFFT_E_ARG;
  *out = nullptr;
  if (!arch_ok(arch) || max_batch < 1 || max_batch > 65535) return LSFFT_E_ARG;
  lsfft_fno_s* f = new (std::nothrow) lsfft_fno_s();
  if (!f) return LSFFT_E_ALLOC;
  f->a = *arch;
  f->max_batch = max_batch;
  f->stream = static_cast<hipStream_t>(hip_stream);
  const int n = arch->n, M = arch->modes;
  f->V = (long long)n * n * n;
  f->L = make_layout(*arch);
  const size_t B = (size_t)max_batch, V = (size_t)f->V, C = kWidth, H = (size_t)arch->hidden;
  const size_t nm = (size_t)f->L.nmodes;
  bool ok = alloc(f, &f->params, f->L.nparam) && alloc(f, &f->grads, f->L.nparam) &&
            alloc(f, &f->mom, f->L.nparam) && alloc(f, &f->vel, f->L.nparam);
  auto pwb = [&](Pw& p) {
    return alloc(f, &p.wb, (size_t)p.opad * p.ipad) && alloc(f, &p.wbt, (size_t)p.t_opad * p.t_ipad);
  };
  ok = ok && pwb(f->L.lift) && pwb(f->L.proj1) && pwb(f->L.proj2);
  for (int l = 0; ok && l < arch->layers; ++l)
    ok = pwb(f->L.hid[l]) && alloc(f, &f->rb[l], nm * C * C * 2) && alloc(f, &f->pre[l], B * C * V) &&
         alloc(f, &f->Hm[l], nm * B * C);
  for (int l = 0; ok && l <= arch->layers; ++l) ok = alloc(f, &f->h[l], B * C * V);
  f->wblk = wgrad_blocks(max_batch, f->V);
  f->nchunk = 64;
  ok = ok && alloc(f, &f->p1, B * H * V) && alloc(f, &f->z, B * H * V) && alloc(f, &f->dz, B * H * V) &&
       alloc(f, &f->y, B * (size_t)arch->cout * V) && alloc(f, &f->dy, B * (size_t)arch->cout * V) &&
       alloc(f, &f->sbuf, B * C * V) && alloc(f, &f->dbuf[0], B * C * V) && alloc(f, &f->dbuf[1], B * C * V) &&
       alloc(f, &f->t1, B * C * n * n * M) && alloc(f, &f->t2, B * C * n * 2 * M * M) &&
       alloc(f, &f->ym, nm * B * C) && alloc(f, &f->gm, nm * B * C) && alloc(f, &f->tw, (size_t)n) &&
       alloc(f, &f->wpart, (size_t)f->wblk * (256 * 32 + 256)) &&
       alloc(f, &f->lpart, B * f->nchunk * 2 + B) && alloc(f, &f->loss_dev, 1);
  if (!ok) {
    release(f);
    delete f;
    return LSFFT_E_ALLOC;
  }
  std::vector<float2> tw(n);
  for (int j = 0; j < n; ++j) {
    const double ang = 2.0 * 3.14159265358979323846 * j / n;
    tw[j] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  if (hipMemcpy(f->tw, tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemsetAsync(f->params, 0, sizeof(float) * f->L.nparam, f->stream) != hipSuccess ||
      hipMemsetAsync(f->mom, 0, sizeof(float) * f->L.nparam, f->stream) != hipSuccess ||
      hipMemsetAsync(f->vel, 0, sizeof(float) * f->L.nparam, f->stream) != hipSuccess ||
      prep_weights(f) != hipSuccess || hipStreamSynchronize(f->stream) != hipSuccess) {
    release(f);
    delete f;
    return LSFFT_E_DEVICE;
  }
  *out = f;
  return LSFFT_OK;
}

lsfft_status lsfft_fno_set_params(lsfft_fno_t f, const float* params) {
  if (!f || !params) return LSFFT_E_ARG;
  FNO_TRY(hipMemcpyAsync(f->params, params, sizeof(float) * f->L.nparam, hipMemcpyDeviceToDevice, f->stream));
  FNO_TRY(hipMemsetAsync(f->mom, 0, sizeof(float) * f->L.nparam, f->stream));
  FNO_TRY(hipMemsetAsync(f->vel, 0, sizeof(float) * f->L.nparam, f->stream));
  f->step = 0;
  FNO_TRY(prep_weights(f));
  FNO_TRY(hipStreamSynchronize(f->stream));
  return LSFFT_OK;
}

lsfft_status lsfft_fno_get_params(lsfft_fno_t f, float* params) {
  if (!f || !params) return LSFFT_E_ARG;
  FNO_TRY(hipMemcpyAsync(params, f->params, sizeof(float) * f->L.nparam, hipMemcpyDeviceToDevice, f->stream));
  FNO_TRY(hipStreamSynchronize(f->stream));
  return LSFFT_OK;
}

lsfft_status lsfft_fno_forward(lsfft_fno_t f, int batch, const float* x, float* y) {
  if (!f || !x || !y || batch < 1 || batch > f->max_batch) return LSFFT_E_ARG;
  FNO_TRY(forward(f, batch, x, y));
  FNO_TRY(hipStreamSynchronize(f->stream));
  return LSFFT_OK;
}

lsfft_status lsfft_fno_loss_grad(lsfft_fno_t f, int batch, const float* x, const float* t, float* grad,
                                 double* loss) {
  if (!f || !x || !t || batch < 1 || batch > f->max_batch) return LSFFT_E_ARG;
  FNO_TRY(forward(f, batch, x, f->y));
  FNO_TRY(backward(f, batch, x, t));
  if (grad)
    FNO_TRY(hipMemcpyAsync(grad, f->grads, sizeof(float) * f->L.nparam, hipMemcpyDeviceToDevice, f->stream));
  double l = 0.0;
  FNO_TRY(hipMemcpyAsync(&l, f->loss_dev, sizeof(double), hipMemcpyDeviceToHost, f->stream));
  FNO_TRY(hipStreamSynchronize(f->stream));
  if (loss) *loss = l;
  return LSFFT_OK;
}

lsfft_status lsfft_fno_adam(lsfft_fno_t f, float lr, float beta1, float beta2, float eps) {
  if (!f || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
    return LSFFT_E_ARG;
  f->step += 1;
  const float bc1 = 1.0f - std::pow(beta1, (float)f->step);
  const float bc2 = 1.0f - std::pow(beta2, (float)f->step);
  FNO_TRY(launch_adam(f->params, f->grads, f->mom, f->vel, f->L.nparam, lr, beta1, beta2, eps, bc1, bc2, f->stream));
  FNO_TRY(prep_weights(f));
  FNO_TRY(hipStreamSynchronize(f->stream));
  return LSFFT_OK;
}

lsfft_status lsfft_fno_train_step(lsfft_fno_t f, int batch, const float* x, const float* t, float lr,
                                  double* loss) {
  lsfft_status s = lsfft_fno_loss_grad(f, batch, x, t, nullptr, loss);
  if (s != LSFFT_OK) return s;
  return lsfft_fno_adam(f, lr, 0.9f, 0.999f, 1e-8f);
}

lsfft_status lsfft_fno_destroy(lsfft_fno_t f) {
  if (!f) return LSFFT_OK;
  release(f);
  delete f;
  return LSFFT_OK;
}

}  // extern "C"
