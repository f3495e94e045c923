// Host-side launch interface of the surrogate kernels (fno_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>

namespace lsfft_fno {

constexpr int kWidth = 32;   // channels of the hidden layers (one MFMA tile)

// Pointwise layer out[b][o][v] = sum_i w[o][i] in[b][i][v] (+ bias[o])
// (+ add[b][o][v]); then, if aux, out *= GELU'(aux[b][o][v]); if out_act,
// out_act = GELU(out).  w is bf16 [opad][ipad], zero padded (opad multiple of
// 32, ipad multiple of 16).
struct PwArgs {
  const float* in;
  const __hip_bfloat16* w;
  const float* bias;
  const float* add;
  const float* aux;
  float* out;
  float* out_act;
  int I, ipad, O, opad, B;
  long long V;
};
hipError_t launch_pointwise(const PwArgs& a, hipStream_t s);

// Weight gradient of a pointwise layer: per block partial sums
// part[blk][opad][ipad] and part_b[blk][opad] of sum_{b,v} g[b][o][v] h[b][i][v]
// and sum g[b][o][v]; then the fixed-order reduction into the packed
// gradient gw [O][I], gb [O].
struct WgArgs {
  const float* g;
  const float* h;
  float* part;
  int O, I, opad, ipad, B;
  long long V;
  int nblk;
};
hipError_t launch_wgrad(const WgArgs& a, float* gw, float* gb, hipStream_t s);
int wgrad_blocks(int B, long long V);

// Per-mode complex products on bf16 MFMA, one wave per mode:
//  mode 0: out[m][b][o] = sum_i x[m][b][i] r[m][i][o]
//  mode 1: out[m][b][i] = sum_o x[m][b][o] conj(r[m][i][o])
//  mode 2: out[m][i][o] (fp32 re,im) = sum_b conj(x[m][b][i]) g[m][b][o]
hipError_t launch_modemix(int mode, const float2* x, const __hip_bfloat16* r, const float2* g, float* out,
                          int nmodes, int B, hipStream_t s);

// Truncated transforms over [BC][n][n][n] (x fastest), kept modes as above.
//  forward: modes[m][bc] = scale(kx) * sum_x h e^{-i k.x}, scale = sc0 (kx = 0) or sc1
//  inverse: out[bc][x] = sum_kept c(kx) Re(modes[m][bc] e^{+i k.x}), c = c0 or c1
hipError_t launch_dft_forward(int n, int M, int BC, const float* h, float2* t1, float2* t2, float2* modes,
                              float sc0, float sc1, const float2* tw, hipStream_t s);
hipError_t launch_dft_inverse(int n, int M, int BC, const float2* modes, float2* t2, float2* t1, float* out,
                              float c0, float c1, const float2* tw, hipStream_t s);

// loss = mean_b ||y_b - t_b|| / ||t_b||, dy = (y - t) / (||y_b - t_b|| ||t_b|| B)
hipError_t launch_loss(const float* y, const float* t, float* dy, int B, long long per_sample, double* part,
                       int nchunk, double* loss_dev, hipStream_t s);

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t s);

// dst[r][c] (bf16, drows x dcols) = src[r * sr + c * sc] inside rows x cols, else 0
hipError_t launch_cast_pad(const float* src, int rows, int cols, long long sr, long long sc, __hip_bfloat16* dst,
                           int drows, int dcols, hipStream_t s);
hipError_t launch_cast(const float* src, __hip_bfloat16* dst, long long n, hipStream_t s);

}  // namespace lsfft_fno
