// Mixed-radix Stockham FFT building blocks for gfx950 (MI355X).
//
// A workgroup transforms a tile of MP independent pencils of length N held in
// LDS as split real/imaginary arrays.  Element (pencil m, index n) lives at
// m*SM + n*SN, so the same code serves pencils that are strided in HBM (the y
// and z passes: SN = MP, SM = 1, lanes walk consecutive pencils) and pencils
// that are rows in HBM (the x pass: SN = 1, SM = odd row pitch, lanes walk
// rows).  Each pass reads R inputs spaced N/R apart, applies the twiddles of
// the current span, a radix-R butterfly, and writes the autosorted outputs
// (Stockham formulation, no bit reversal).  Transforms are unnormalised:
// forward uses exp(-2 pi i k n / N), inverse exp(+2 pi i k n / N)
// (the DFT of Sec. 4, Eqs. 4.3-4.5; the 1/|N| of Eq. 4.4 is applied once by
// the caller).
//
// Twiddles come from an LDS table tw[k] = exp(-2 pi i k / NT) read with a
// stride TWS, so the table of a length-2N real transform also serves its
// length-N complex core.
#pragma once
#include <hip/hip_runtime.h>

namespace lsfft {

// ---------------------------------------------------------------------------
// radix plans: product of the radices is N, radices in {2, 3, 4, 8}
// ---------------------------------------------------------------------------
template <int N> struct Plan;
#define LSFFT_PLAN(N_, NP_, R0, R1, R2)                                  \
  template <> struct Plan<N_> {                                            \
    static constexpr int np = NP_;                                         \
    static constexpr int r[3] = {R0, R1, R2};                              \
  };
LSFFT_PLAN(2, 1, 2, 1, 1)
LSFFT_PLAN(3, 1, 3, 1, 1)
LSFFT_PLAN(4, 1, 4, 1, 1)
LSFFT_PLAN(6, 2, 3, 2, 1)
LSFFT_PLAN(8, 1, 8, 1, 1)
LSFFT_PLAN(12, 2, 4, 3, 1)
LSFFT_PLAN(16, 2, 4, 4, 1)
LSFFT_PLAN(24, 2, 8, 3, 1)
LSFFT_PLAN(32, 2, 8, 4, 1)
LSFFT_PLAN(48, 3, 4, 4, 3)
LSFFT_PLAN(64, 2, 8, 8, 1)
LSFFT_PLAN(96, 3, 8, 4, 3)
LSFFT_PLAN(128, 3, 8, 4, 4)
LSFFT_PLAN(256, 3, 8, 8, 4)
#undef LSFFT_PLAN

// ---------------------------------------------------------------------------
// complex helpers on split (re, im) scalars
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void cmul(T& ar, T& ai, T br, T bi) {
  T t = ar * br - ai * bi;
  ai = ar * bi + ai * br;
  ar = t;
}

// radix-R butterflies, in place on v[0..R).  DIR = -1 forward, +1 inverse.
template <typename T, int DIR>
__device__ __forceinline__ void bfly2(T* vr, T* vi) {
  T ar = vr[0], ai = vi[0];
  vr[0] = ar + vr[1]; vi[0] = ai + vi[1];
  vr[1] = ar - vr[1]; vi[1] = ai - vi[1];
}

template <typename T, int DIR>
__device__ __forceinline__ void bfly4_vals(T& x0r, T& x0i, T& x1r, T& x1i,
                                          T& x2r, T& x2i, T& x3r, T& x3i) {
  T ar = x0r + x2r, ai = x0i + x2i;
  T br = x0r - x2r, bi = x0i - x2i;
  T cr = x1r + x3r, ci = x1i + x3i;
  T dr = x1r - x3r, di = x1i - x3i;
  // forward: y1 = b - i d, y3 = b + i d ; inverse: y1 = b + i d, y3 = b - i d
  // (-i)*(dr + i di) = di - i dr ; (+i)*(dr + i di) = -di + i dr
  T er, ei;
  if (DIR < 0) { er = di; ei = -dr; } else { er = -di; ei = dr; }
  x0r = ar + cr; x0i = ai + ci;
  x2r = ar - cr; x2i = ai - ci;
  x1r = br + er; x1i = bi + ei;
  x3r = br - er; x3i = bi - ei;
}

template <typename T, int DIR>
__device__ __forceinline__ void bfly4(T* vr, T* vi) {
  bfly4_vals<T, DIR>(vr[0], vi[0], vr[1], vi[1], vr[2], vi[2], vr[3], vi[3]);
}

template <typename T, int DIR>
__device__ __forceinline__ void bfly3(T* vr, T* vi) {
  const T s3 = T(0.86602540378443864676372317075293618);  // sqrt(3)/2
  T sr = vr[1] + vr[2], si = vi[1] + vi[2];
  T dr = vr[1] - vr[2], di = vi[1] - vi[2];
  T mr = vr[0] - T(0.5) * sr, mi = vi[0] - T(0.5) * si;
  // forward: y1 = m - i s3 d ; y2 = m + i s3 d  (inverse swaps)
  T tr, ti;  // (-i s3) * d = s3*di - i s3*dr
  if (DIR < 0) { tr = s3 * di; ti = -s3 * dr; } else { tr = -s3 * di; ti = s3 * dr; }
  vr[0] = vr[0] + sr; vi[0] = vi[0] + si;
  vr[1] = mr + tr; vi[1] = mi + ti;
  vr[2] = mr - tr; vi[2] = mi - ti;
}

template <typename T, int DIR>
__device__ __forceinline__ void bfly8(T* vr, T* vi) {
  const T h = T(0.70710678118654752440084436210484904);  // sqrt(2)/2
  // even and odd radix-4 halves
  bfly4_vals<T, DIR>(vr[0], vi[0], vr[2], vi[2], vr[4], vi[4], vr[6], vi[6]);
  bfly4_vals<T, DIR>(vr[1], vi[1], vr[3], vi[3], vr[5], vi[5], vr[7], vi[7]);
  // twiddle the odd half by W8^k, W8 = exp(DIR * 2 pi i / 8)
  {  // k = 1: (h, DIR*h)
    T r = vr[3], i = vi[3];
    if (DIR < 0) { vr[3] = h * (r + i); vi[3] = h * (i - r); }
    else         { vr[3] = h * (r - i); vi[3] = h * (i + r); }
  }
  {  // k = 2: DIR*i
    T r = vr[5], i = vi[5];
    if (DIR < 0) { vr[5] = i; vi[5] = -r; } else { vr[5] = -i; vi[5] = r; }
  }
  {  // k = 3: (-h, DIR*h)
    T r = vr[7], i = vi[7];
    if (DIR < 0) { vr[7] = h * (i - r); vi[7] = -h * (r + i); }
    else         { vr[7] = -h * (r + i); vi[7] = h * (r - i); }
  }
  // combine: y[k] = E[k] + W^k O[k], y[k+4] = E[k] - W^k O[k]
  // E[k] sits in slot 2k, O[k] (twiddled) in slot 2k+1
  T er[4] = {vr[0], vr[2], vr[4], vr[6]}, ei[4] = {vi[0], vi[2], vi[4], vi[6]};
  T orr[4] = {vr[1], vr[3], vr[5], vr[7]}, oi[4] = {vi[1], vi[3], vi[5], vi[7]};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    vr[k] = er[k] + orr[k];     vi[k] = ei[k] + oi[k];
    vr[k + 4] = er[k] - orr[k]; vi[k + 4] = ei[k] - oi[k];
  }
}

template <typename T, int R, int DIR>
__device__ __forceinline__ void bfly(T* vr, T* vi) {
  if constexpr (R == 2) bfly2<T, DIR>(vr, vi);
  else if constexpr (R == 3) bfly3<T, DIR>(vr, vi);
  else if constexpr (R == 4) bfly4<T, DIR>(vr, vi);
  else if constexpr (R == 8) bfly8<T, DIR>(vr, vi);
}

// ---------------------------------------------------------------------------
// one Stockham pass over an LDS tile
// ---------------------------------------------------------------------------
template <typename T, int N, int R, int NS, int DIR, int MP, int SM, int SN, int TWS, int NT>
__device__ __forceinline__ void stockham_pass(const T* __restrict__ ir, const T* __restrict__ ii,
                                              T* __restrict__ orr, T* __restrict__ oi,
                                              const T* __restrict__ twr, const T* __restrict__ twi,
                                              int tid) {
  constexpr int NB = N / R;
  constexpr int TOT = MP * NB;
  constexpr int TSTEP = N / (NS * R);  // twiddle index step in units of N-th roots
#pragma unroll 2
  for (int b = tid; b < TOT; b += NT) {
    const int m = b % MP;
    const int j = b / MP;
    const int k = j % NS;
    T vr[R], vi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int idx = m * SM + (j + r * NB) * SN;
      vr[r] = ir[idx];
      vi[r] = ii[idx];
    }
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const int t = r * k * TSTEP * TWS;
        const T wr = twr[t];
        const T wi = (DIR < 0) ? twi[t] : -twi[t];
        cmul(vr[r], vi[r], wr, wi);
      }
    }
    bfly<T, R, DIR>(vr, vi);
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int idx = m * SM + (base + r * NS) * SN;
      orr[idx] = vr[r];
      oi[idx] = vi[r];
    }
  }
}

// Full transform of the tile.  Input in buffer 0 (ar, ai); passes ping-pong
// with buffer 1 (br, bi).  Returns 0 if the result is in buffer 0, 1 if in
// buffer 1.  Every pass ends with a workgroup barrier.
template <typename T, int N, int DIR, int MP, int SM, int SN, int TWS, int NT>
__device__ __forceinline__ int fft_tile(T* ar, T* ai, T* br, T* bi,
                                        const T* twr, const T* twi, int tid) {
  using P = Plan<N>;
  constexpr int R0 = P::r[0];
  stockham_pass<T, N, R0, 1, DIR, MP, SM, SN, TWS, NT>(ar, ai, br, bi, twr, twi, tid);
  __syncthreads();
  if constexpr (P::np == 1) {
    return 1;
  } else {
    constexpr int R1 = P::r[1];
    stockham_pass<T, N, R1, R0, DIR, MP, SM, SN, TWS, NT>(br, bi, ar, ai, twr, twi, tid);
    __syncthreads();
    if constexpr (P::np == 2) {
      return 0;
    } else {
      constexpr int R2 = P::r[2];
      stockham_pass<T, N, R2, R0 * R1, DIR, MP, SM, SN, TWS, NT>(ar, ai, br, bi, twr, twi, tid);
      __syncthreads();
      return 1;
    }
  }
}

template <int N> struct PlanCheck {
  static constexpr int prod = Plan<N>::np == 1 ? Plan<N>::r[0]
                            : Plan<N>::np == 2 ? Plan<N>::r[0] * Plan<N>::r[1]
                                               : Plan<N>::r[0] * Plan<N>::r[1] * Plan<N>::r[2];
  static_assert(prod == N, "radix plan does not multiply to N");
};

}  // namespace lsfft
