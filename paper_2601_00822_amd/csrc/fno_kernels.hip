// Kernels of the learned surrogate (Eq. 6.10 layers, Fourier-neural-operator
// family): pointwise layers and their gradients on bf16 MFMA
// (v_mfma_f32_32x32x16_bf16, fp32 accumulation), per-mode complex products
// on the same instruction, truncated transforms, loss and Adam in fp32.
//
// MFMA 32x32x16 operand layout used throughout (one wave, lane l):
//   A (32 x 16, row-major operand): row l % 32, columns 8 (l / 32) .. +7
//   B (16 x 32):                    column l % 32, rows 8 (l / 32) .. +7
//   C (32 x 32, 16 floats per lane): element e sits at
//       row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32.
#include <hip/hip_runtime.h>

#include "fft_core.hpp"
#include "fno_launch.hpp"

namespace lsfft_fno {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NTB = 256;   // threads of the elementwise and transform kernels

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752440f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752440f)) + x * 0.39894228040143267794f * expf(-0.5f * x * x);
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 neg8(bf16x8 a) {
  bf16x8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = -a[j];
  return r;
}

// ---------------------------------------------------------------------------
// pointwise layer
// ---------------------------------------------------------------------------
// One wave per block of 32 NT voxels of one sample, computed as NT
// interleaved 32-column MFMA tiles: tile k holds voxels v0 + NT c + k
// (c = lane % 32), so every lane moves NT consecutive voxels, one per tile,
// in one vector access, and each half-wave reads or writes 128 NT
// contiguous bytes of one channel.  The B operand (input channels) is
// converted to bf16 once per block and reused for every 32-row tile of
// output channels.  NT shrinks as the input width grows (register budget).
constexpr int kMaxKs = 16;   // ipad <= 256

template <int NT> struct VecF;
template <> struct VecF<1> { using type = float; };
template <> struct VecF<2> { using type = float2; };
template <> struct VecF<4> { using type = float4; };

template <int NT>
__device__ __forceinline__ void vload(const float* p, float (&v)[NT]) {
  const typename VecF<NT>::type x = *reinterpret_cast<const typename VecF<NT>::type*>(p);
  if constexpr (NT == 1) v[0] = x;
  else if constexpr (NT == 2) { v[0] = x.x; v[1] = x.y; }
  else { v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w; }
}
template <int NT>
__device__ __forceinline__ void vstore(float* p, const float (&v)[NT]) {
  typename VecF<NT>::type x;
  if constexpr (NT == 1) x = v[0];
  else if constexpr (NT == 2) { x.x = v[0]; x.y = v[1]; }
  else { x.x = v[0]; x.y = v[1]; x.z = v[2]; x.w = v[3]; }
  *reinterpret_cast<typename VecF<NT>::type*>(p) = x;
}

template <int KS, int NT>
__global__ __launch_bounds__(256) void k_pointwise(PwArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  constexpr int BV = 32 * NT;   // voxels per wave block
  const long long V = a.V;
  const long long blocks = (long long)a.B * (V / BV);
  const bf16x8* w8 = reinterpret_cast<const bf16x8*>(a.w);
  for (long long t = (long long)blockIdx.x * 4 + wave; t < blocks; t += (long long)gridDim.x * 4) {
    const int b = int(t / (V / BV));
    const long long v = (t % (V / BV)) * BV + NT * col;
    bf16x8 bop[KS][NT];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = s * 16 + half * 8 + j;
        float x[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) x[k] = 0.0f;
        if (i < a.I) vload<NT>(a.in + ((long long)b * a.I + i) * V + v, x);
#pragma unroll
        for (int k = 0; k < NT; ++k) bop[s][k][j] = (__bf16)x[k];
      }
    }
    for (int ot = 0; ot < a.opad / 32; ++ot) {
      f32x16 acc[NT];
#pragma unroll
      for (int k = 0; k < NT; ++k) acc[k] = f32x16{0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const bf16x8 aop = w8[((long long)(ot * 32 + col) * a.ipad + s * 16 + half * 8) / 8];
#pragma unroll
        for (int k = 0; k < NT; ++k) acc[k] = mfma(aop, bop[s][k], acc[k]);
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int o = ot * 32 + 8 * (e / 4) + 4 * half + (e % 4);
        if (o >= a.O) continue;
        const long long idx = ((long long)b * a.O + o) * V + v;
        float val[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) val[k] = acc[k][e];
        if (a.bias) {
          const float bo = a.bias[o];
#pragma unroll
          for (int k = 0; k < NT; ++k) val[k] += bo;
        }
        if (a.add) {
          float ad[NT];
          vload<NT>(a.add + idx, ad);
#pragma unroll
          for (int k = 0; k < NT; ++k) val[k] += ad[k];
        }
        if (a.aux) {
          float ax[NT];
          vload<NT>(a.aux + idx, ax);
#pragma unroll
          for (int k = 0; k < NT; ++k) val[k] *= gelu_grad(ax[k]);
        }
        vstore<NT>(a.out + idx, val);
        if (a.out_act) {
          float g[NT];
#pragma unroll
          for (int k = 0; k < NT; ++k) g[k] = gelu(val[k]);
          vstore<NT>(a.out_act + idx, g);
        }
      }
    }
  }
}

hipError_t launch_pointwise(const PwArgs& a, hipStream_t s) {
  if (a.ipad % 16 || a.opad % 32 || a.ipad > 16 * kMaxKs || a.V % 128) return hipErrorInvalidValue;
  const int ks = a.ipad / 16;
  const int nt = ks <= 2 ? 4 : (ks <= 8 ? 2 : 1);
  const long long nblk = (long long)a.B * (a.V / (32 * nt));
  long long blocks = (nblk + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  const dim3 g((unsigned)blocks);
  switch (ks) {
    case 1: hipLaunchKernelGGL((k_pointwise<1, 4>), g, 256, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_pointwise<2, 4>), g, 256, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_pointwise<4, 2>), g, 256, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_pointwise<6, 2>), g, 256, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_pointwise<8, 2>), g, 256, 0, s, a); break;
    case 10: hipLaunchKernelGGL((k_pointwise<10, 1>), g, 256, 0, s, a); break;
    case 12: hipLaunchKernelGGL((k_pointwise<12, 1>), g, 256, 0, s, a); break;
    case 14: hipLaunchKernelGGL((k_pointwise<14, 1>), g, 256, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_pointwise<16, 1>), g, 256, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pointwise weight gradient: MFMA over 16-voxel chunks, per-block partials
// ---------------------------------------------------------------------------
constexpr int kWgBlocks = 256;
int wgrad_blocks(int B, long long V) {
  const long long chunks = (long long)B * (V / 16);
  long long nb = (chunks + 3) / 4;
  return (int)(nb < kWgBlocks ? (nb < 1 ? 1 : nb) : kWgBlocks);
}

template <int TO, int TI>
__global__ __launch_bounds__(256) void k_wgrad(WgArgs a) {
  __shared__ float red[4][1024 + 32];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5, row = lane & 31;
  const long long V = a.V;
  const long long chunks = (long long)a.B * (V / 16);
  f32x16 acc[TO][TI];
  float bsum[TO];
#pragma unroll
  for (int p = 0; p < TO; ++p) {
    bsum[p] = 0.0f;
#pragma unroll
    for (int q = 0; q < TI; ++q) acc[p][q] = f32x16{0};
  }
  for (long long c = (long long)blockIdx.x * 4 + wave; c < chunks; c += (long long)gridDim.x * 4) {
    const int b = int(c / (V / 16));
    const long long v0 = (c % (V / 16)) * 16 + half * 8;
    // eight consecutive voxels per lane: two 16-byte loads per operand row
    auto load8 = [&](const float* src, bool ok, float (&x)[8]) {
      float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
      if (ok) {
        lo = reinterpret_cast<const float4*>(src)[0];
        hi = reinterpret_cast<const float4*>(src)[1];
      }
      x[0] = lo.x; x[1] = lo.y; x[2] = lo.z; x[3] = lo.w;
      x[4] = hi.x; x[5] = hi.y; x[6] = hi.z; x[7] = hi.w;
    };
    bf16x8 bop[TI];
#pragma unroll
    for (int q = 0; q < TI; ++q) {
      const int i = q * 32 + row;
      float x[8];
      load8(a.h + ((long long)b * a.I + (i < a.I ? i : 0)) * V + v0, i < a.I, x);
#pragma unroll
      for (int j = 0; j < 8; ++j) bop[q][j] = (__bf16)x[j];
    }
#pragma unroll
    for (int p = 0; p < TO; ++p) {
      const int o = p * 32 + row;
      float x[8];
      load8(a.g + ((long long)b * a.O + (o < a.O ? o : 0)) * V + v0, o < a.O, x);
      bf16x8 aop;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        bsum[p] += x[j];
        aop[j] = (__bf16)x[j];
      }
#pragma unroll
      for (int q = 0; q < TI; ++q) acc[p][q] = mfma(aop, bop[q], acc[p][q]);
    }
  }
  // fixed-order sum of the four waves, tile by tile
  float* part = a.part + (size_t)blockIdx.x * (a.opad * a.ipad + a.opad);
#pragma unroll
  for (int p = 0; p < TO; ++p) {
#pragma unroll
    for (int q = 0; q < TI; ++q) {
#pragma unroll
      for (int e = 0; e < 16; ++e) red[wave][e * 64 + lane] = acc[p][q][e];
      if (q == 0) red[wave][1024 + (lane & 31)] = 0.0f;
      __syncthreads();
      if (q == 0) {
        // bias partial: lanes l and l + 32 hold the two halves of row l % 32
        if (half == 0) red[wave][1024 + row] = bsum[p];
        __syncthreads();
        if (half == 1) red[wave][1024 + row] += bsum[p];
        __syncthreads();
      }
      for (int k = threadIdx.x; k < 1024; k += 256) {
        const float s = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        const int e = k / 64, l = k % 64;
        const int o = p * 32 + 8 * (e / 4) + 4 * (l / 32) + (e % 4);
        const int i = q * 32 + (l & 31);
        part[o * a.ipad + i] = s;
      }
      if (q == 0 && threadIdx.x < 32)
        part[a.opad * a.ipad + p * 32 + threadIdx.x] =
            red[0][1024 + threadIdx.x] + red[1][1024 + threadIdx.x] + red[2][1024 + threadIdx.x] +
            red[3][1024 + threadIdx.x];
      __syncthreads();
    }
  }
}

// Fixed-order sum of the per-block partials: a block covers 64 consecutive
// packed outputs, its four waves sum interleaved quarters of the partials,
// and the quarters are added in a fixed order.
__global__ __launch_bounds__(NTB) void k_wgrad_reduce(const float* __restrict__ part, int nblk, int O, int I,
                                                      int opad, int ipad, float* __restrict__ gw,
                                                      float* __restrict__ gb) {
  __shared__ float red[4][64];
  const int n = O * I + O;
  const int stride = opad * ipad + opad;
  const int k = blockIdx.x * 64 + (threadIdx.x & 63);
  const int q = threadIdx.x >> 6;
  float s = 0.0f;
  if (k < n) {
    const int src = (k < O * I) ? (k / I) * ipad + (k % I) : opad * ipad + (k - O * I);
    for (int blk = q; blk < nblk; blk += 4) s += part[(size_t)blk * stride + src];
  }
  red[q][threadIdx.x & 63] = s;
  __syncthreads();
  if (q == 0 && k < n) {
    const float t = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    if (k < O * I) gw[k] = t;
    else gb[k - O * I] = t;
  }
}

hipError_t launch_wgrad(const WgArgs& a, float* gw, float* gb, hipStream_t s) {
  if (a.V % 16 || a.opad % 32 || a.ipad % 32) return hipErrorInvalidValue;
  const dim3 g((unsigned)a.nblk);
  const int to = a.opad / 32, ti = a.ipad / 32;
  if (to == 1 && ti == 1) hipLaunchKernelGGL((k_wgrad<1, 1>), g, 256, 0, s, a);
  else if (to == 2 && ti == 1) hipLaunchKernelGGL((k_wgrad<2, 1>), g, 256, 0, s, a);
  else if (to == 4 && ti == 1) hipLaunchKernelGGL((k_wgrad<4, 1>), g, 256, 0, s, a);
  else if (to == 8 && ti == 1) hipLaunchKernelGGL((k_wgrad<8, 1>), g, 256, 0, s, a);
  else if (to == 1 && ti == 2) hipLaunchKernelGGL((k_wgrad<1, 2>), g, 256, 0, s, a);
  else if (to == 1 && ti == 4) hipLaunchKernelGGL((k_wgrad<1, 4>), g, 256, 0, s, a);
  else if (to == 1 && ti == 8) hipLaunchKernelGGL((k_wgrad<1, 8>), g, 256, 0, s, a);
  else return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = a.O * a.I + a.O;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((n + 63) / 64)), NTB, 0, s, a.part, a.nblk, a.O, a.I,
                     a.opad, a.ipad, gw, gb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-mode complex products (one 64-thread block per mode)
// ---------------------------------------------------------------------------
// Operand tiles are staged in LDS as bf16 planes, A as [row][k] and B
// transposed as [n][k], so every MFMA operand is one 16-byte LDS read.
template <int MODE>
__global__ __launch_bounds__(64) void k_modemix(const float2* __restrict__ x, const __hip_bfloat16* __restrict__ rb,
                                                const float2* __restrict__ g, float* __restrict__ out, int nmodes,
                                                int B) {
  __shared__ __attribute__((aligned(16))) __bf16 Ar[32][32 + 8], Ai[32][32 + 8], Br[32][32 + 8], Bi[32][32 + 8];
  const int lane = threadIdx.x;
  const int half = lane >> 5, col = lane & 31;
  const __bf16* r = reinterpret_cast<const __bf16*>(rb);
  for (int m = blockIdx.x; m < nmodes; m += gridDim.x) {
    const float2* xm = x + (size_t)m * B * 32;
    const __bf16* rm = r + (size_t)m * 32 * 32 * 2;
    if (MODE != 2) {
      // B^T[n][k]: mode 0 -> R[k][n] (n = o, k = i); mode 1 -> conj R[n][k] (n = i, k = o)
      for (int k = lane; k < 1024; k += 64) {
        const int i = k >> 5, o = k & 31;
        const __bf16 re = rm[2 * k], im = rm[2 * k + 1];
        if (MODE == 0) { Br[o][i] = re; Bi[o][i] = im; }
        else { Br[i][o] = re; Bi[i][o] = -im; }
      }
    }
    f32x16 cr = {0}, ci = {0};
    const int nbt = (B + 31) / 32;
    for (int bt = 0; bt < nbt; ++bt) {
      __syncthreads();
      if (MODE != 2) {
        // A[row = b][k]: mode 0 x[b][i], mode 1 g[b][o] (passed in x)
        for (int k = lane; k < 1024; k += 64) {
          const int rr = k >> 5, c = k & 31;
          const int b = bt * 32 + rr;
          const float2 v = (b < B) ? xm[(size_t)b * 32 + c] : make_float2(0.f, 0.f);
          Ar[rr][c] = (__bf16)v.x;
          Ai[rr][c] = (__bf16)v.y;
        }
      } else {
        // A[row = i][k = b] = conj x[b][i]; B^T[n = o][k = b] = g[b][o]
        const float2* gm = g + (size_t)m * B * 32;
        for (int k = lane; k < 1024; k += 64) {
          const int rr = k >> 5, c = k & 31;
          const int b = bt * 32 + rr;
          const float2 v = (b < B) ? xm[(size_t)b * 32 + c] : make_float2(0.f, 0.f);
          const float2 w = (b < B) ? gm[(size_t)b * 32 + c] : make_float2(0.f, 0.f);
          Ar[c][rr] = (__bf16)v.x;
          Ai[c][rr] = (__bf16)(-v.y);
          Br[c][rr] = (__bf16)w.x;
          Bi[c][rr] = (__bf16)w.y;
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int k0 = s * 16 + half * 8;
        const bf16x8 ar = *reinterpret_cast<const bf16x8*>(&Ar[col][k0]);
        const bf16x8 ai = *reinterpret_cast<const bf16x8*>(&Ai[col][k0]);
        const bf16x8 br = *reinterpret_cast<const bf16x8*>(&Br[col][k0]);
        const bf16x8 bi = *reinterpret_cast<const bf16x8*>(&Bi[col][k0]);
        cr = mfma(ar, br, cr);
        cr = mfma(neg8(ai), bi, cr);
        ci = mfma(ar, bi, ci);
        ci = mfma(ai, br, ci);
      }
      if (MODE != 2) {
        float2* om = reinterpret_cast<float2*>(out) + (size_t)m * B * 32;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int rr = 8 * (e / 4) + 4 * half + (e % 4);
          const int b = bt * 32 + rr;
          if (b < B) om[(size_t)b * 32 + col] = make_float2(cr[e], ci[e]);
        }
        cr = f32x16{0};
        ci = f32x16{0};
      }
    }
    if (MODE == 2) {
      float2* om = reinterpret_cast<float2*>(out) + (size_t)m * 32 * 32;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int i = 8 * (e / 4) + 4 * half + (e % 4);
        om[i * 32 + col] = make_float2(cr[e], ci[e]);
      }
    }
    __syncthreads();
  }
}

hipError_t launch_modemix(int mode, const float2* x, const __hip_bfloat16* r, const float2* g, float* out,
                          int nmodes, int B, hipStream_t s) {
  const dim3 grid((unsigned)(nmodes < 65536 ? nmodes : 65536));
  if (mode == 0) hipLaunchKernelGGL(k_modemix<0>, grid, 64, 0, s, x, r, g, out, nmodes, B);
  else if (mode == 1) hipLaunchKernelGGL(k_modemix<1>, grid, 64, 0, s, x, r, g, out, nmodes, B);
  else if (mode == 2) hipLaunchKernelGGL(k_modemix<2>, grid, 64, 0, s, x, r, g, out, nmodes, B);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// truncated transforms: length-N FFTs along one axis at a time, fp32
// ---------------------------------------------------------------------------
// Every kernel transforms a tile of MP pencils with the solver's Stockham
// tile transform (fft_core.hpp): full pencils are loaded (the truncated
// inputs of an inverse as zeros), transformed in registers and LDS, and only
// the kept outputs are stored.  Layouts (BC = batch x channels, P = 2M M):
//   h   [BC][z][y][x]           real
//   t1  [BC][z][y][kx]          kx < M
//   t2  [BC][z][iy][kx]         iy < 2M (signed ky)
//   md  [iz P + iy M + kx][BC]  the kept modes, mode-major
// Kept array index of the signed wavenumber slot s in [0, 2M): s for s < M,
// n - 2M + s for the negative ones; the slot of FFT index k is k for k < M,
// k - n + 2M for k >= n - M, none otherwise.
template <int N> __device__ __forceinline__ int kidx(int s, int M) { return s < M ? s : N - 2 * M + s; }
template <int N> __device__ __forceinline__ int kslot(int k, int M) {
  return k < M ? k : (k >= N - M ? k - N + 2 * M : -1);
}

// twiddles exp(-2 pi i k / N) split into LDS as the tile transform reads
// them, from the (cos, sin) table of the surrogate
template <int N>
__device__ __forceinline__ void load_tw_split(float* twr, float* twi, const float2* twg) {
  for (int k = threadIdx.x; k < N; k += NTB) {
    const float2 w = twg[k];
    twr[k] = w.x;
    twi[k] = -w.y;
  }
}

// x axis: MX rows of N reals per tile, index-fastest butterflies (each
// row's points come from consecutive lanes)
template <int N> struct XT {
  static constexpr int MP = 2048 / N;
  static constexpr int SM = N + 1;
  template <int DIR> using F = lsfft::TileFft<float, N, DIR, false, MP, SM, 1, 1, true, NTB>;
};
// y and z axes: 64 pencils per tile, pencil-fastest butterflies
constexpr int kPen = 64;
template <int N> struct ST {
  static constexpr int SN = kPen + 1;
  template <int DIR> using F = lsfft::TileFft<float, N, DIR, false, kPen, 1, SN, 1, false, NTB>;
};

// x forward: rows of reals -> kx < M
template <int N>
__global__ __launch_bounds__(NTB) void k_dft_x_fwd(const float* __restrict__ h, float2* __restrict__ t1, long long rows,
                                                   int M, const float2* __restrict__ twg) {
  using F = typename XT<N>::template F<-1>;
  constexpr int MP = XT<N>::MP;
  __shared__ float re[MP * XT<N>::SM], im[MP * XT<N>::SM], twr[N], twi[N];
  load_tw_split<N>(twr, twi, twg);
  __syncthreads();
  const int tid = threadIdx.x;
  const long long row0 = (long long)blockIdx.x * MP;
  float in_r[F::B0][F::R0], in_i[F::B0][F::R0];
#pragma unroll
  for (int q = 0; q < F::B0; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::R0>(b, m, j);
    const bool ok = (F::TOT0 % NTB == 0 || b < F::TOT0) && row0 + m < rows;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      in_r[q][r] = ok ? h[(row0 + m) * N + j + r * (N / F::R0)] : 0.0f;
      in_i[q][r] = 0.0f;
    }
  }
  float o_r[F::BL][F::RL], o_i[F::BL][F::RL];
  F::run(in_r, in_i, o_r, o_i, re, im, twr, twi, tid);
#pragma unroll
  for (int q = 0; q < F::BL; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::RL>(b, m, j);
    if ((F::TOTL % NTB == 0 || b < F::TOTL) && row0 + m < rows) {
#pragma unroll
      for (int r = 0; r < F::RL; ++r) {
        const int k = j + r * (N / F::RL);
        if (k < M) t1[(row0 + m) * M + k] = make_float2(o_r[q][r], o_i[q][r]);
      }
    }
  }
}

// x inverse: out[row][x] = sum_kx c(kx) Re(t1[row][kx] e^{+i kx x}),
// c(0) = c0, c(kx > 0) = c1
template <int N>
__global__ __launch_bounds__(NTB) void k_dft_x_inv(const float2* __restrict__ t1, float* __restrict__ out, long long rows,
                                                   int M, float c0, float c1, const float2* __restrict__ twg) {
  using F = typename XT<N>::template F<+1>;
  constexpr int MP = XT<N>::MP;
  __shared__ float re[MP * XT<N>::SM], im[MP * XT<N>::SM], twr[N], twi[N];
  load_tw_split<N>(twr, twi, twg);
  __syncthreads();
  const int tid = threadIdx.x;
  const long long row0 = (long long)blockIdx.x * MP;
  float in_r[F::B0][F::R0], in_i[F::B0][F::R0];
#pragma unroll
  for (int q = 0; q < F::B0; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::R0>(b, m, j);
    const bool ok = (F::TOT0 % NTB == 0 || b < F::TOT0) && row0 + m < rows;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      const int k = j + r * (N / F::R0);
      float2 v = make_float2(0.0f, 0.0f);
      if (ok && k < M) {
        v = t1[(row0 + m) * M + k];
        const float c = (k == 0) ? c0 : c1;
        v.x *= c;
        v.y *= c;
      }
      in_r[q][r] = v.x;
      in_i[q][r] = v.y;
    }
  }
  float o_r[F::BL][F::RL], o_i[F::BL][F::RL];
  F::run(in_r, in_i, o_r, o_i, re, im, twr, twi, tid);
  // real parts through the LDS tile, then coalesced 16-byte stores
  __syncthreads();
#pragma unroll
  for (int q = 0; q < F::BL; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::RL>(b, m, j);
    if (F::TOTL % NTB == 0 || b < F::TOTL) {
#pragma unroll
      for (int r = 0; r < F::RL; ++r) re[m * XT<N>::SM + j + r * (N / F::RL)] = o_r[q][r];
    }
  }
  __syncthreads();
  const int nr = (int)((rows - row0) < MP ? (rows - row0) : MP);
  for (int e = tid; e < nr * N / 4; e += NTB) {
    const int m = (4 * e) / N, x = (4 * e) - m * N;
    const float* sp = re + m * XT<N>::SM + x;
    reinterpret_cast<float4*>(out + row0 * N)[e] = make_float4(sp[0], sp[1], sp[2], sp[3]);
  }
}

// y forward: t1[bz][y][kx] -> t2[bz][iy][kx]; pencil g = bz M + kx
template <int N>
__global__ __launch_bounds__(NTB) void k_dft_y_fwd(const float2* __restrict__ t1, float2* __restrict__ t2, long long nbz,
                                                   int M, const float2* __restrict__ twg) {
  using F = typename ST<N>::template F<-1>;
  __shared__ float re[N * ST<N>::SN], im[N * ST<N>::SN], twr[N], twi[N];
  load_tw_split<N>(twr, twi, twg);
  __syncthreads();
  const int tid = threadIdx.x;
  const long long g0 = (long long)blockIdx.x * kPen, npen = nbz * M;
  float in_r[F::B0][F::R0], in_i[F::B0][F::R0];
#pragma unroll
  for (int q = 0; q < F::B0; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::R0>(b, m, j);
    const long long g = g0 + m;
    const bool ok = (F::TOT0 % NTB == 0 || b < F::TOT0) && g < npen;
    const long long bz = ok ? g / M : 0;
    const int kx = ok ? int(g - bz * M) : 0;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      float2 v = make_float2(0.0f, 0.0f);
      if (ok) v = t1[(bz * N + j + r * (N / F::R0)) * M + kx];
      in_r[q][r] = v.x;
      in_i[q][r] = v.y;
    }
  }
  float o_r[F::BL][F::RL], o_i[F::BL][F::RL];
  F::run(in_r, in_i, o_r, o_i, re, im, twr, twi, tid);
#pragma unroll
  for (int q = 0; q < F::BL; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::RL>(b, m, j);
    const long long g = g0 + m;
    if ((F::TOTL % NTB == 0 || b < F::TOTL) && g < npen) {
      const long long bz = g / M;
      const int kx = int(g - bz * M);
#pragma unroll
      for (int r = 0; r < F::RL; ++r) {
        const int iy = kslot<N>(j + r * (N / F::RL), M);
        if (iy >= 0) t2[(bz * 2 * M + iy) * M + kx] = make_float2(o_r[q][r], o_i[q][r]);
      }
    }
  }
}

// y inverse: t2[bz][iy][kx] -> t1[bz][y][kx]
template <int N>
__global__ __launch_bounds__(NTB) void k_dft_y_inv(const float2* __restrict__ t2, float2* __restrict__ t1, long long nbz,
                                                   int M, const float2* __restrict__ twg) {
  using F = typename ST<N>::template F<+1>;
  __shared__ float re[N * ST<N>::SN], im[N * ST<N>::SN], twr[N], twi[N];
  load_tw_split<N>(twr, twi, twg);
  __syncthreads();
  const int tid = threadIdx.x;
  const long long g0 = (long long)blockIdx.x * kPen, npen = nbz * M;
  float in_r[F::B0][F::R0], in_i[F::B0][F::R0];
#pragma unroll
  for (int q = 0; q < F::B0; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::R0>(b, m, j);
    const long long g = g0 + m;
    const bool ok = (F::TOT0 % NTB == 0 || b < F::TOT0) && g < npen;
    const long long bz = ok ? g / M : 0;
    const int kx = ok ? int(g - bz * M) : 0;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      const int iy = kslot<N>(j + r * (N / F::R0), M);
      float2 v = make_float2(0.0f, 0.0f);
      if (ok && iy >= 0) v = t2[(bz * 2 * M + iy) * M + kx];
      in_r[q][r] = v.x;
      in_i[q][r] = v.y;
    }
  }
  float o_r[F::BL][F::RL], o_i[F::BL][F::RL];
  F::run(in_r, in_i, o_r, o_i, re, im, twr, twi, tid);
#pragma unroll
  for (int q = 0; q < F::BL; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::RL>(b, m, j);
    const long long g = g0 + m;
    if ((F::TOTL % NTB == 0 || b < F::TOTL) && g < npen) {
      const long long bz = g / M;
      const int kx = int(g - bz * M);
#pragma unroll
      for (int r = 0; r < F::RL; ++r)
        t1[(bz * N + j + r * (N / F::RL)) * M + kx] = make_float2(o_r[q][r], o_i[q][r]);
    }
  }
}

// z axis: tiles of kZyx (iy, kx) pairs x kZbc batch-channels, pencil
// m = yx_local + kZyx bc_local: consecutive lanes read runs of kZyx entries
// of t2 and write runs of kZbc entries of md
constexpr int kZyx = 8, kZbc = 8;
static_assert(kZyx * kZbc == kPen, "z tile");

// z forward: t2[bc][z][yx] -> md[(iz P + yx) BC + bc] * scale(kx)
template <int N>
__global__ __launch_bounds__(NTB) void k_dft_z_fwd(const float2* __restrict__ t2, float2* __restrict__ md, int BC, int M,
                                                   float sc0, float sc1, const float2* __restrict__ twg) {
  using F = typename ST<N>::template F<-1>;
  __shared__ float re[N * ST<N>::SN], im[N * ST<N>::SN], twr[N], twi[N];
  load_tw_split<N>(twr, twi, twg);
  __syncthreads();
  const int tid = threadIdx.x;
  const int P = 2 * M * M;
  const int nyx = (P + kZyx - 1) / kZyx;
  const int bc0 = (blockIdx.x / nyx) * kZbc, yx0 = (blockIdx.x % nyx) * kZyx;
  float in_r[F::B0][F::R0], in_i[F::B0][F::R0];
#pragma unroll
  for (int q = 0; q < F::B0; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::R0>(b, m, j);
    const int yx = yx0 + m % kZyx, bc = bc0 + m / kZyx;
    const bool ok = (F::TOT0 % NTB == 0 || b < F::TOT0) && yx < P && bc < BC;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      float2 v = make_float2(0.0f, 0.0f);
      if (ok) v = t2[((long long)bc * N + j + r * (N / F::R0)) * P + yx];
      in_r[q][r] = v.x;
      in_i[q][r] = v.y;
    }
  }
  float o_r[F::BL][F::RL], o_i[F::BL][F::RL];
  F::run(in_r, in_i, o_r, o_i, re, im, twr, twi, tid);
#pragma unroll
  for (int q = 0; q < F::BL; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::RL>(b, m, j);
    const int yx = yx0 + m % kZyx, bc = bc0 + m / kZyx;
    if ((F::TOTL % NTB == 0 || b < F::TOTL) && yx < P && bc < BC) {
      const float sc = (yx % M == 0) ? sc0 : sc1;
#pragma unroll
      for (int r = 0; r < F::RL; ++r) {
        const int iz = kslot<N>(j + r * (N / F::RL), M);
        if (iz >= 0) md[((long long)iz * P + yx) * BC + bc] = make_float2(o_r[q][r] * sc, o_i[q][r] * sc);
      }
    }
  }
}

// z inverse: md -> t2[bc][z][yx]
template <int N>
__global__ __launch_bounds__(NTB) void k_dft_z_inv(const float2* __restrict__ md, float2* __restrict__ t2, int BC, int M,
                                                   const float2* __restrict__ twg) {
  using F = typename ST<N>::template F<+1>;
  __shared__ float re[N * ST<N>::SN], im[N * ST<N>::SN], twr[N], twi[N];
  load_tw_split<N>(twr, twi, twg);
  __syncthreads();
  const int tid = threadIdx.x;
  const int P = 2 * M * M;
  const int nyx = (P + kZyx - 1) / kZyx;
  const int bc0 = (blockIdx.x / nyx) * kZbc, yx0 = (blockIdx.x % nyx) * kZyx;
  float in_r[F::B0][F::R0], in_i[F::B0][F::R0];
#pragma unroll
  for (int q = 0; q < F::B0; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::R0>(b, m, j);
    const int yx = yx0 + m % kZyx, bc = bc0 + m / kZyx;
    const bool ok = (F::TOT0 % NTB == 0 || b < F::TOT0) && yx < P && bc < BC;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      const int iz = kslot<N>(j + r * (N / F::R0), M);
      float2 v = make_float2(0.0f, 0.0f);
      if (ok && iz >= 0) v = md[((long long)iz * P + yx) * BC + bc];
      in_r[q][r] = v.x;
      in_i[q][r] = v.y;
    }
  }
  float o_r[F::BL][F::RL], o_i[F::BL][F::RL];
  F::run(in_r, in_i, o_r, o_i, re, im, twr, twi, tid);
#pragma unroll
  for (int q = 0; q < F::BL; ++q) {
    const int b = tid + q * NTB;
    int m, j;
    F::template bj<F::RL>(b, m, j);
    const int yx = yx0 + m % kZyx, bc = bc0 + m / kZyx;
    if ((F::TOTL % NTB == 0 || b < F::TOTL) && yx < P && bc < BC) {
#pragma unroll
      for (int r = 0; r < F::RL; ++r)
        t2[((long long)bc * N + j + r * (N / F::RL)) * P + yx] = make_float2(o_r[q][r], o_i[q][r]);
    }
  }
}

static unsigned nblocks(long long work, int per) { return (unsigned)((work + per - 1) / per); }

template <int N>
static hipError_t dft_fwd_n(int M, int BC, const float* h, float2* t1, float2* t2, float2* md, float sc0, float sc1,
                            const float2* tw, hipStream_t s) {
  const long long rows = (long long)BC * N * N;
  hipLaunchKernelGGL(k_dft_x_fwd<N>, dim3(nblocks(rows, XT<N>::MP)), NTB, 0, s, h, t1, rows, M, tw);
  const long long nbz = (long long)BC * N;
  hipLaunchKernelGGL(k_dft_y_fwd<N>, dim3(nblocks(nbz * M, kPen)), NTB, 0, s, t1, t2, nbz, M, tw);
  const int P = 2 * M * M;
  const unsigned nz = nblocks(BC, kZbc) * nblocks(P, kZyx);
  hipLaunchKernelGGL(k_dft_z_fwd<N>, dim3(nz), NTB, 0, s, t2, md, BC, M, sc0, sc1, tw);
  return hipGetLastError();
}

template <int N>
static hipError_t dft_inv_n(int M, int BC, const float2* md, float2* t2, float2* t1, float* out, float c0, float c1,
                            const float2* tw, hipStream_t s) {
  const int P = 2 * M * M;
  const unsigned nz = nblocks(BC, kZbc) * nblocks(P, kZyx);
  hipLaunchKernelGGL(k_dft_z_inv<N>, dim3(nz), NTB, 0, s, md, t2, BC, M, tw);
  const long long nbz = (long long)BC * N;
  hipLaunchKernelGGL(k_dft_y_inv<N>, dim3(nblocks(nbz * M, kPen)), NTB, 0, s, t2, t1, nbz, M, tw);
  const long long rows = (long long)BC * N * N;
  hipLaunchKernelGGL(k_dft_x_inv<N>, dim3(nblocks(rows, XT<N>::MP)), NTB, 0, s, t1, out, rows, M, c0, c1, tw);
  return hipGetLastError();
}

hipError_t launch_dft_forward(int n, int M, int BC, const float* h, float2* t1, float2* t2, float2* md, float sc0,
                              float sc1, const float2* tw, hipStream_t s) {
  if (M < 1 || 2 * M > n) return hipErrorInvalidValue;
  switch (n) {
    case 8: return dft_fwd_n<8>(M, BC, h, t1, t2, md, sc0, sc1, tw, s);
    case 16: return dft_fwd_n<16>(M, BC, h, t1, t2, md, sc0, sc1, tw, s);
    case 32: return dft_fwd_n<32>(M, BC, h, t1, t2, md, sc0, sc1, tw, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dft_inverse(int n, int M, int BC, const float2* md, float2* t2, float2* t1, float* out, float c0,
                              float c1, const float2* tw, hipStream_t s) {
  if (M < 1 || 2 * M > n) return hipErrorInvalidValue;
  switch (n) {
    case 8: return dft_inv_n<8>(M, BC, md, t2, t1, out, c0, c1, tw, s);
    case 16: return dft_inv_n<16>(M, BC, md, t2, t1, out, c0, c1, tw, s);
    case 32: return dft_inv_n<32>(M, BC, md, t2, t1, out, c0, c1, tw, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// loss, Adam, casts
// ---------------------------------------------------------------------------
__device__ double block_sum_d(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < NTB / 64; ++k) s += red[k];
  return s;
}

// part[b][chunk][2] = (sum (y - t)^2, sum t^2) over one chunk of sample b
__global__ __launch_bounds__(NTB) void k_loss_part(const float* __restrict__ y, const float* __restrict__ t,
                                                   long long per, int nchunk, double* __restrict__ part) {
  __shared__ double red[NTB / 64];
  const int b = blockIdx.y, c = blockIdx.x;
  const long long len = (per + nchunk - 1) / nchunk;
  const long long lo = c * len, hi = (lo + len < per) ? lo + len : per;
  double e = 0.0, n = 0.0;
  for (long long k = lo + threadIdx.x; k < hi; k += NTB) {
    const double d = (double)y[b * per + k] - (double)t[b * per + k];
    const double tv = (double)t[b * per + k];
    e += d * d;
    n += tv * tv;
  }
  e = block_sum_d(e, red);
  n = block_sum_d(n, red);
  if (threadIdx.x == 0) {
    part[((size_t)b * nchunk + c) * 2] = e;
    part[((size_t)b * nchunk + c) * 2 + 1] = n;
  }
}

// per-sample coefficients 1 / (||e_b|| ||t_b|| B) and the mean loss (one
// block; a thread per sample, then a fixed-order sum)
__global__ __launch_bounds__(NTB) void k_loss_final(const double* __restrict__ part, int B, int nchunk,
                                                    double* __restrict__ coef, double* __restrict__ loss) {
  __shared__ double red[NTB];
  double acc = 0.0;
  for (int b = threadIdx.x; b < B; b += NTB) {
    double e = 0.0, n = 0.0;
    for (int c = 0; c < nchunk; ++c) {
      e += part[((size_t)b * nchunk + c) * 2];
      n += part[((size_t)b * nchunk + c) * 2 + 1];
    }
    const double en = sqrt(e), tn = sqrt(n);
    acc += en / tn;
    coef[b] = 1.0 / (fmax(en, 1e-300) * tn * (double)B);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < NTB; ++k) s += red[k];
    *loss = s / (double)B;
  }
}

__global__ __launch_bounds__(NTB) void k_loss_grad(const float* __restrict__ y, const float* __restrict__ t,
                                                   const double* __restrict__ coef, float* __restrict__ dy, int B,
                                                   long long per) {
  const long long n = (long long)B * per;
  for (long long k = (long long)blockIdx.x * NTB + threadIdx.x; k < n; k += (long long)gridDim.x * NTB)
    dy[k] = (float)(((double)y[k] - (double)t[k]) * coef[k / per]);
}

hipError_t launch_loss(const float* y, const float* t, float* dy, int B, long long per_sample, double* part,
                       int nchunk, double* loss_dev, hipStream_t s) {
  double* coef = part + (size_t)B * nchunk * 2;
  hipLaunchKernelGGL(k_loss_part, dim3((unsigned)nchunk, (unsigned)B), NTB, 0, s, y, t, per_sample, nchunk, part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), NTB, 0, s, part, B, nchunk, coef, loss_dev);
  long long blocks = ((long long)B * per_sample + NTB - 1) / NTB;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)blocks), NTB, 0, s, y, t, coef, dy, B, per_sample);
  return hipGetLastError();
}

__global__ __launch_bounds__(NTB) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, long long n, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2) {
  for (long long k = (long long)blockIdx.x * NTB + threadIdx.x; k < n; k += (long long)gridDim.x * NTB) {
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
  }
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t s) {
  long long blocks = (n + NTB - 1) / NTB;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), NTB, 0, s, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

__global__ __launch_bounds__(NTB) void k_cast_pad(const float* __restrict__ src, int rows, int cols, long long sr,
                                                  long long sc, __hip_bfloat16* __restrict__ dst, int drows, int dcols) {
  __bf16* d = reinterpret_cast<__bf16*>(dst);
  const long long n = (long long)drows * dcols;
  for (long long k = (long long)blockIdx.x * NTB + threadIdx.x; k < n; k += (long long)gridDim.x * NTB) {
    const int r = int(k / dcols), c = int(k % dcols);
    d[k] = (__bf16)((r < rows && c < cols) ? src[r * sr + c * sc] : 0.0f);
  }
}

hipError_t launch_cast_pad(const float* src, int rows, int cols, long long sr, long long sc, __hip_bfloat16* dst,
                           int drows, int dcols, hipStream_t s) {
  long long blocks = ((long long)drows * dcols + NTB - 1) / NTB;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_cast_pad, dim3((unsigned)blocks), NTB, 0, s, src, rows, cols, sr, sc, dst, drows, dcols);
  return hipGetLastError();
}

__global__ __launch_bounds__(NTB) void k_cast(const float* __restrict__ src, __hip_bfloat16* __restrict__ dst,
                                              long long n) {
  __bf16* d = reinterpret_cast<__bf16*>(dst);
  for (long long k = (long long)blockIdx.x * NTB + threadIdx.x; k < n; k += (long long)gridDim.x * NTB)
    d[k] = (__bf16)src[k];
}

hipError_t launch_cast(const float* src, __hip_bfloat16* dst, long long n, hipStream_t s) {
  long long blocks = (n + NTB - 1) / NTB;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_cast, dim3((unsigned)blocks), NTB, 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace lsfft_fno
