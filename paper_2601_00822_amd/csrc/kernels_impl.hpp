// HIP kernels of the BFCS Lippmann-Schwinger solver for gfx950.
//
// One basic-scheme iteration is four sweeps over HBM (3D), each a persistent
// kernel walking a device work list of (solve, tile) items:
//
//   ypass<inv>  : inverse y transforms of the strain spectrum (3D only)
//   xpass<ITER> : per x-row: half-spectrum -> real (C2R), Hooke's law
//                 sigma = lam(x) tr(eps) I + 2 mu(x) eps (Eq. 2.2), real ->
//                 half-spectrum (R2C); the real fields never reach HBM
//   ypass<fwd>  : forward y transforms of the stress spectrum (3D only)
//   green<ITER> : along the outermost axis: forward transform of sigma, the
//                 equilibrium residual r = i xi . sigma^ + f^ with its FP64
//                 Parseval partial sum, the update u^ += N0(xi) r (the
//                 displacement form of Eqs. 5.7-5.10, see the solver notes),
//                 the next strain spectrum sym(i xi (x) u^) / |N| and its
//                 inverse transform
//
// followed by a one-block-per-solve FP64 reduction that evaluates the stopping
// rule and retires converged solves.  2D grids skip the y sweeps (the outer
// axis is y).  The same kernels, in other modes, transform the force, form the
// free term u^b = N0 f^ (Eqs. 2.8-2.9), run the conjugate-gradient variant and
// materialize u, eps and sigma.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fft_core.hpp"
#include "lsfft_internal.hpp"

namespace lsfft {

constexpr int NT = kThreads;

// ---------------------------------------------------------------------------
// tile geometry
// ---------------------------------------------------------------------------
constexpr int pow2floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// elements of one component tile held in LDS / registers
template <typename T> struct TileBudget { static constexpr int value = 2048; };
template <> struct TileBudget<double> { static constexpr int value = 1024; };

// pencils per tile for a strided pass of length N
template <typename T, int N> struct StridedGeom {
  static constexpr int MP = clampi(pow2floor(TileBudget<T>::value / N), 1, 64);
  static constexpr int ELEMS = MP * N;
  static constexpr int PPT = (ELEMS + NT - 1) / NT;
};

// rows per tile for the x pass (H = nx / 2 complex points per row); the x
// pass keeps every strain component of its points in registers, so it uses
// half the budget
template <typename T, int H> struct RowGeom {
  static constexpr int MR = clampi(pow2floor(TileBudget<T>::value / 2 / H), 1, 64);
  static constexpr int SM = ((H + 1) % 2 == 1) ? (H + 1) : (H + 2);  // odd pitch
  static constexpr int PPT = (MR * H + NT - 1) / NT;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };

template <typename T>
__device__ __forceinline__ typename C2<T>::type ldc(const void* base, long long i) {
  return reinterpret_cast<const typename C2<T>::type*>(base)[i];
}
template <typename T>
__device__ __forceinline__ void stc(void* base, long long i, T re, T im) {
  typename C2<T>::type v;
  v.x = re;
  v.y = im;
  reinterpret_cast<typename C2<T>::type*>(base)[i] = v;
}

// signed wavevector component of index k on an axis of n points; zero on the
// Nyquist index
__device__ __forceinline__ double wavenum(int k, int n, double scale) {
  const int h = n >> 1;
  if (k == h) return 0.0;
  return scale * double(k < h ? k : k - n);
}

// load exp(-2 pi i k / L), k < L, into LDS from the plan's twiddle table
template <typename T, int L>
__device__ __forceinline__ void load_tw(T* twr, T* twi, const T* table, int tid) {
  constexpr int off = tw_offset(L);
  static_assert(off >= 0, "unsupported transform length");
  for (int k = tid; k < L; k += NT) {
    twr[k] = table[2 * (off + k)];
    twi[k] = table[2 * (off + k) + 1];
  }
}

// block-wide FP64 sum (deterministic for a fixed block size)
__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < NT / 64; ++w) s += red[w];
  }
  return s;  // valid in thread 0
}


// ---------------------------------------------------------------------------
// real <-> half-spectrum folding of a length-NX real row through a
// length-H = NX/2 complex transform (z[n] = a[2n] + i a[2n+1])
// ---------------------------------------------------------------------------

// Z (transform of the packed row, in rr/ri) -> X[k], k = 0..H, written to
// global row `row` of `out` (complex, nxh entries per row).
//   E = (Z[k] + conj Z[H-k]) / 2,  O = -i (Z[k] - conj Z[H-k]) / 2,
//   X[k] = E + exp(-2 pi i k / NX) O
template <typename T, int H, int MR, int SM>
__device__ __forceinline__ void fold_r2c_store(const T* rr, const T* ri, const T* twr, const T* twi,
                                               void* out, int row0, int nrows, int nxh, int tid) {
  for (int e = tid; e < MR * (H + 1); e += NT) {
    const int m = e / (H + 1);
    const int k = e - m * (H + 1);
    const int row = row0 + m;
    if (row >= nrows) continue;
    const int k1 = (k == H) ? 0 : k;
    const int k2 = (k == 0) ? 0 : H - k;
    const T zr = rr[m * SM + k1], zi = ri[m * SM + k1];
    const T wr = rr[m * SM + k2], wi = ri[m * SM + k2];
    const T er = T(0.5) * (zr + wr), ei = T(0.5) * (zi - wi);
    const T dr = T(0.5) * (zr - wr), di = T(0.5) * (zi + wi);
    const T orr = di, oi = -dr;                 // O = -i D
    const T cr = twr[k], ci = twi[k];
    stc<T>(out, (long long)row * nxh + k, er + cr * orr - ci * oi, ei + cr * oi + ci * orr);
  }
}

// X[k] (k = 0..H, rows in ar/ai) -> Z'[k] (k < H) in br/bi such that the
// unnormalised inverse length-H transform of Z' is NX * (a[2n] + i a[2n+1]):
//   Z' = (X[k] + conj X[H-k]) + i exp(+2 pi i k / NX) (X[k] - conj X[H-k])
template <typename T, int H, int MR, int SM>
__device__ __forceinline__ void fold_c2r_prep(const T* ar, const T* ai, T* br, T* bi,
                                              const T* twr, const T* twi, int tid) {
  for (int e = tid; e < MR * H; e += NT) {
    const int m = e / H;
    const int k = e - m * H;
    const T xr = ar[m * SM + k], xi = ai[m * SM + k];
    const T yr = ar[m * SM + (H - k)], yi = -ai[m * SM + (H - k)];   // conj X[H-k]
    const T dr = xr - yr, di = xi - yi;
    const T cr = twr[k], ci = -twi[k];                                // exp(+2 pi i k / NX)
    const T tr = cr * dr - ci * di, ti = cr * di + ci * dr;
    br[m * SM + k] = xr + yr - ti;
    bi[m * SM + k] = xi + yi + tr;
  }
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// ---------------------------------------------------------------------------
// x pass
// ---------------------------------------------------------------------------
template <typename T, int NX, int DIM, int MODE>
__device__ void xpass_item(const InstDesc& D, int local, const double* __restrict__ lame,
                           const T* __restrict__ twtab, unsigned char* smem) {
  constexpr int H = NX / 2;
  using G = RowGeom<T, H>;
  constexpr int MR = G::MR, SM = G::SM, PPT = G::PPT;
  constexpr int TILE = MR * SM;
  constexpr int S = (DIM == 3) ? 6 : 3;
  T* ar = reinterpret_cast<T*>(smem);
  T* ai = ar + TILE;
  T* br = ai + TILE;
  T* bi = br + TILE;
  T* twr = bi + TILE;
  T* twi = twr + NX;
  T* lam_s = twi + NX;
  T* mu_s = lam_s + kMaxPhases;
  const int tid = threadIdx.x;
  load_tw<T, NX>(twr, twi, twtab, tid);
  if constexpr (MODE != M_FT) {
    for (int p = tid; p < D.nphase; p += NT) {
      lam_s[p] = T(lame[2 * (D.lame_off + p)]);
      mu_s[p] = T(lame[2 * (D.lame_off + p) + 1]);
    }
  }
  __syncthreads();
  const int nrows = D.ny * D.nz;
  const int row0 = local * MR;
  const long long P = D.P;
  const int nxh = D.nxh;
  const size_t cbytes = sizeof(T) * 2;

  if constexpr (MODE == M_FT) {
    // forward real-to-half-spectrum of the force rows into F
    for (int c = 0; c < DIM; ++c) {
      const T* src = reinterpret_cast<const T*>(D.f_in) + (long long)c * D.nvox;
      for (int e = tid; e < MR * H; e += NT) {
        const int m = e / H, n = e - (e / H) * H;
        const int row = row0 + m;
        T re = T(0), im = T(0);
        if (row < nrows) {
          const typename C2<T>::type v =
              reinterpret_cast<const typename C2<T>::type*>(src + (long long)row * NX)[n];
          re = v.x;
          im = v.y;
        }
        ar[m * SM + n] = re;
        ai[m * SM + n] = im;
      }
      __syncthreads();
      const int where = fft_tile<T, H, -1, MR, SM, 1, 2, NT>(ar, ai, br, bi, twr, twi, tid);
      fold_r2c_store<T, H, MR, SM>(where ? br : ar, where ? bi : ai, twr, twi,
                                   static_cast<char*>(D.F) + c * P * cbytes, row0, nrows, nxh, tid);
      __syncthreads();
    }
    return;
  } else {
    // strain components of this thread's points, real pairs (x = 2n, 2n + 1)
    T er[S][PPT], ei[S][PPT];
    constexpr int ncu = (MODE == M_MAT) ? S + DIM : S;
#pragma unroll
    for (int c = 0; c < ncu; ++c) {
      const char* src = static_cast<const char*>(D.S) + c * P * cbytes;
      for (int e = tid; e < MR * (H + 1); e += NT) {
        const int m = e / (H + 1), k = e - (e / (H + 1)) * (H + 1);
        const int row = row0 + m;
        T re = T(0), im = T(0);
        if (row < nrows) {
          const typename C2<T>::type v = ldc<T>(src, (long long)row * nxh + k);
          re = v.x;
          im = v.y;
        }
        ar[m * SM + k] = re;
        ai[m * SM + k] = im;
      }
      __syncthreads();
      fold_c2r_prep<T, H, MR, SM>(ar, ai, br, bi, twr, twi, tid);
      __syncthreads();
      const int where = fft_tile<T, H, +1, MR, SM, 1, 2, NT>(br, bi, ar, ai, twr, twi, tid);
      const T* rr = where ? ar : br;
      const T* ri = where ? ai : bi;
      if (c < S) {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const int e = tid + p * NT;
          if (e < MR * H) {
            const int m = e / H, n = e - (e / H) * H;
            er[c][p] = rr[m * SM + n];
            ei[c][p] = ri[m * SM + n];
          }
        }
      } else if (D.out_u) {
        // MAT: displacement component c - S written straight out
        T* dst = reinterpret_cast<T*>(D.out_u) + (long long)(c - S) * D.nvox;
        for (int e = tid; e < MR * H; e += NT) {
          const int m = e / H, n = e - (e / H) * H;
          const int row = row0 + m;
          if (row < nrows) {
            typename C2<T>::type v;
            v.x = rr[m * SM + n];
            v.y = ri[m * SM + n];
            reinterpret_cast<typename C2<T>::type*>(dst + (long long)row * NX)[n] = v;
          }
        }
      }
      __syncthreads();
    }
    if constexpr (MODE == M_MAT) {
      if (D.out_eps) {
#pragma unroll
        for (int c = 0; c < S; ++c) {
          T* dst = reinterpret_cast<T*>(D.out_eps) + (long long)c * D.nvox;
#pragma unroll
          for (int p = 0; p < PPT; ++p) {
            const int e = tid + p * NT;
            const int m = e / H, n = e - (e / H) * H;
            if (e < MR * H && row0 + m < nrows) {
              typename C2<T>::type v;
              v.x = er[c][p];
              v.y = ei[c][p];
              reinterpret_cast<typename C2<T>::type*>(dst + (long long)(row0 + m) * NX)[n] = v;
            }
          }
        }
      }
    }
    // Hooke's law at every point of the tile, microstructure shifted by s
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      const int e = tid + p * NT;
      const int m = e / H, n = e - (e / H) * H;
      const int row = row0 + m;
      if (e < MR * H && row < nrows) {
        const int z = row / D.ny, y = row - (row / D.ny) * D.ny;
        const long long rbase =
            ((long long)wrap(z - D.sz, D.nz) * D.ny + wrap(y - D.sy, D.ny)) * (long long)NX;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const int x = 2 * n + half;
          const int ph = D.phase[rbase + wrap(x - D.sx, NX)];
          const T lam = lam_s[ph], mu2 = T(2) * mu_s[ph];
          T ev[S];
#pragma unroll
          for (int c = 0; c < S; ++c) ev[c] = half ? ei[c][p] : er[c][p];
          T tr = ev[0] + ev[1];
          if constexpr (DIM == 3) tr += ev[2];
#pragma unroll
          for (int c = 0; c < S; ++c) {
            const T sv = mu2 * ev[c] + ((c < DIM) ? lam * tr : T(0));
            if (half) ei[c][p] = sv; else er[c][p] = sv;
          }
        }
      }
    }
    if constexpr (MODE == M_MAT) {
      if (D.out_sig) {
#pragma unroll
        for (int c = 0; c < S; ++c) {
          T* dst = reinterpret_cast<T*>(D.out_sig) + (long long)c * D.nvox;
#pragma unroll
          for (int p = 0; p < PPT; ++p) {
            const int e = tid + p * NT;
            const int m = e / H, n = e - (e / H) * H;
            if (e < MR * H && row0 + m < nrows) {
              typename C2<T>::type v;
              v.x = er[c][p];
              v.y = ei[c][p];
              reinterpret_cast<typename C2<T>::type*>(dst + (long long)(row0 + m) * NX)[n] = v;
            }
          }
        }
      }
      return;
    } else {
      // forward transform of each stress component back to the half spectrum
#pragma unroll
      for (int c = 0; c < S; ++c) {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const int e = tid + p * NT;
          if (e < MR * H) {
            const int m = e / H, n = e - (e / H) * H;
            ar[m * SM + n] = er[c][p];
            ai[m * SM + n] = ei[c][p];
          }
        }
        __syncthreads();
        const int where = fft_tile<T, H, -1, MR, SM, 1, 2, NT>(ar, ai, br, bi, twr, twi, tid);
        fold_r2c_store<T, H, MR, SM>(where ? br : ar, where ? bi : ai, twr, twi,
                                     static_cast<char*>(D.S) + c * P * cbytes, row0, nrows, nxh, tid);
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// y pass (3D): complex transforms along y of `ncomp` components of `buf`
// ---------------------------------------------------------------------------
template <typename T, int NY, int DIR>
__device__ void ypass_item(const InstDesc& D, int local, void* buf, int ncomp,
                           const T* __restrict__ twtab, unsigned char* smem) {
  using G = StridedGeom<T, NY>;
  constexpr int MP = G::MP, E = G::ELEMS;
  T* ar = reinterpret_cast<T*>(smem);
  T* ai = ar + E;
  T* br = ai + E;
  T* bi = br + E;
  T* twr = bi + E;
  T* twi = twr + NY;
  const int tid = threadIdx.x;
  load_tw<T, NY>(twr, twi, twtab, tid);
  __syncthreads();
  const int z = local / D.ntile_y;
  const int kx0 = (local - z * D.ntile_y) * MP;
  const int nxh = D.nxh;
  const long long base = (long long)z * NY * nxh + kx0;
  const size_t cbytes = sizeof(T) * 2;
  for (int c = 0; c < ncomp; ++c) {
    char* cb = static_cast<char*>(buf) + c * D.P * cbytes;
    for (int e = tid; e < E; e += NT) {
      const int m = e % MP, n = e / MP;
      T re = T(0), im = T(0);
      if (kx0 + m < nxh) {
        const typename C2<T>::type v = ldc<T>(cb, base + (long long)n * nxh + m);
        re = v.x;
        im = v.y;
      }
      ar[e] = re;
      ai[e] = im;
    }
    __syncthreads();
    const int where = fft_tile<T, NY, DIR, MP, 1, MP, 1, NT>(ar, ai, br, bi, twr, twi, tid);
    const T* rr = where ? br : ar;
    const T* ri = where ? bi : ai;
    for (int e = tid; e < E; e += NT) {
      const int m = e % MP, n = e / MP;
      if (kx0 + m < nxh) stc<T>(cb, base + (long long)n * nxh + m, rr[e], ri[e]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Green / body-force pass along the outermost axis (z in 3D, y in 2D)
// ---------------------------------------------------------------------------

// N0(xi) v = (v - c0 xi (xi . v) / |xi|^2) / (mu0 |xi|^2); zero where xi = 0
template <typename T, int DIM>
__device__ __forceinline__ void apply_n0(const T* xi, T xi2, T c0, T mu0, T* vr, T* vi) {
  if (xi2 == T(0)) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) { vr[a] = T(0); vi[a] = T(0); }
    return;
  }
  T pr = T(0), pi = T(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) { pr += xi[a] * vr[a]; pi += xi[a] * vi[a]; }
  const T inv = T(1) / xi2;
  const T sc = inv / mu0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    vr[a] = (vr[a] - c0 * xi[a] * pr * inv) * sc;
    vi[a] = (vi[a] - c0 * xi[a] * pi * inv) * sc;
  }
}

// Voigt index pairs, (11,22,33,23,13,12) in 3D and (11,22,12) in 2D
template <int DIM> __device__ __forceinline__ int va(int c) {
  if constexpr (DIM == 3) return c < 3 ? c : (c == 3 ? 1 : 0);
  else return c < 2 ? c : 0;
}
template <int DIM> __device__ __forceinline__ int vb(int c) {
  if constexpr (DIM == 3) return c < 3 ? c : (c == 3 ? 2 : (c == 4 ? 2 : 1));
  else return c < 2 ? c : 1;
}

template <typename T, int NG, int DIM, int MODE>
__device__ void green_item(const InstDesc& D, InstState* __restrict__ St, int local,
                           const T* __restrict__ twtab, unsigned char* smem) {
  using G = StridedGeom<T, NG>;
  constexpr int MP = G::MP, E = G::ELEMS, PPT = G::PPT;
  constexpr int S = (DIM == 3) ? 6 : 3;
  T* ar = reinterpret_cast<T*>(smem);
  T* ai = ar + E;
  T* br = ai + E;
  T* bi = br + E;
  T* twr = bi + E;
  T* twi = twr + NG;
  double* red = reinterpret_cast<double*>(twi + NG + (NG & 1));
  const int tid = threadIdx.x;
  load_tw<T, NG>(twr, twi, twtab, tid);
  __syncthreads();

  const int nxh = D.nxh;
  int ymid = 0, tile;
  long long stride, base;
  if constexpr (DIM == 3) {
    ymid = local / D.ntile_g;
    tile = local - ymid * D.ntile_g;
    stride = (long long)D.ny * nxh;
    base = (long long)ymid * nxh + tile * MP;
  } else {
    tile = local;
    stride = nxh;
    base = (long long)tile * MP;
  }
  const int kx0 = tile * MP;
  const size_t cbytes = sizeof(T) * 2;
  const long long P = D.P;
  const T inv_n = T(D.inv_nvox);
  const T mu0 = T(D.mu0);
  const T c0 = T((D.lam0 + D.mu0) / (D.lam0 + 2.0 * D.mu0));

  // this thread's points: e = tid + p * NT, pencil m = e % MP, index n = e / MP
  T vr[DIM][PPT], vi[DIM][PPT];
  double part = 0.0, part2 = 0.0;

  auto point_xi = [&](int p, T* xi, T& xi2, bool& valid, long long& gidx, T& wgt, int& n) {
    const int e = tid + p * NT;
    const int m = e % MP;
    n = e / MP;
    const int kx = kx0 + m;
    valid = (e < E) && (kx < nxh);
    xi[0] = T(wavenum(kx, D.nx, D.kx));
    if constexpr (DIM == 3) {
      xi[1] = T(wavenum(ymid, D.ny, D.ky));
      xi[2] = T(wavenum(n, D.nz, D.kz));
    } else {
      xi[1] = T(wavenum(n, D.ny, D.ky));
    }
    xi2 = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) xi2 += xi[a] * xi[a];
    gidx = base + (long long)n * stride + m;
    wgt = (kx == 0 || kx == (D.nx >> 1)) ? T(1) : T(2);
  };

  // forward transform of NC components of `src` along the outer axis; calls
  // fn(c, p, re, im) for every point of this thread (c is a compile-time
  // constant after unrolling, so register arrays stay in registers)
  auto forward = [&](const void* src, auto nc_tag, auto&& fn) {
    constexpr int NC = decltype(nc_tag)::value;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const char* cb = static_cast<const char*>(src) + c * P * cbytes;
      for (int e = tid; e < E; e += NT) {
        const int m = e % MP, n = e / MP;
        T re = T(0), im = T(0);
        if (kx0 + m < nxh) {
          const typename C2<T>::type v = ldc<T>(cb, base + (long long)n * stride + m);
          re = v.x;
          im = v.y;
        }
        ar[e] = re;
        ai[e] = im;
      }
      __syncthreads();
      const int where = fft_tile<T, NG, -1, MP, 1, MP, 1, NT>(ar, ai, br, bi, twr, twi, tid);
      const T* rr = where ? br : ar;
      const T* ri = where ? bi : ai;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        const int e = tid + p * NT;
        if (e < E) fn(c, p, rr[e], ri[e]);
      }
      __syncthreads();
    }
  };

  // inverse transform of values produced per point by gen(c, p, re&, im&)
  // into NC components of `dst`
  auto inverse = [&](void* dst, auto nc_tag, auto&& gen) {
    constexpr int NC = decltype(nc_tag)::value;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        const int e = tid + p * NT;
        if (e < E) {
          T re, im;
          gen(c, p, re, im);
          ar[e] = re;
          ai[e] = im;
        }
      }
      __syncthreads();
      const int where = fft_tile<T, NG, +1, MP, 1, MP, 1, NT>(ar, ai, br, bi, twr, twi, tid);
      const T* rr = where ? br : ar;
      const T* ri = where ? bi : ai;
      char* cb = static_cast<char*>(dst) + c * P * cbytes;
      for (int e = tid; e < E; e += NT) {
        const int m = e % MP, n = e / MP;
        if (kx0 + m < nxh) stc<T>(cb, base + (long long)n * stride + m, rr[e], ri[e]);
      }
      __syncthreads();
    }
  };

  // strain spectrum / |N| from the displacement spectrum held in vr/vi:
  // eps^_ab = (i/2)(xi_a u^_b + xi_b u^_a)
  auto strain_gen = [&](int c, int p, T& re, T& im) {
    T xi[DIM], xi2, wgt;
    bool valid;
    long long gidx;
    int n;
    point_xi(p, xi, xi2, valid, gidx, wgt, n);
    const int a = va<DIM>(c), b = vb<DIM>(c);
    // i/2 (xi_a u_b + xi_b u_a) = (-(xi_a ub.i + xi_b ua.i)/2, (xi_a ub.r + xi_b ua.r)/2)
    const T sr = T(0.5) * (xi[a] * vr[b][p] + xi[b] * vr[a][p]);
    const T si = T(0.5) * (xi[a] * vi[b][p] + xi[b] * vi[a][p]);
    re = -si * inv_n;
    im = sr * inv_n;
  };

  const int cur = St->iter & 1;

  if constexpr (MODE == M_FT) {
    // finish the force transform, record the removed mean, project off Z
    forward(D.F, std::integral_constant<int, DIM>{}, [&](int c, int p, T re, T im) { vr[c][p] = re; vi[c][p] = im; });
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      T xi[DIM], xi2, wgt;
      bool valid;
      long long gidx;
      int n;
      point_xi(p, xi, xi2, valid, gidx, wgt, n);
      if (!valid) continue;
      const bool origin = (kx0 + (tid + p * NT) % MP == 0) && n == 0 && (DIM == 2 || ymid == 0);
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        if (origin) St->removed_mean[c] = double(vr[c][p]) * D.inv_nvox;
        if (xi2 == T(0)) { vr[c][p] = T(0); vi[c][p] = T(0); }
        stc<T>(static_cast<char*>(D.F) + c * P * cbytes, gidx, vr[c][p], vi[c][p]);
      }
    }
    return;
  } else if constexpr (MODE == M_INIT || MODE == M_ITER || MODE == M_CG_INIT) {
    if constexpr (MODE == M_INIT) {
#pragma unroll
      for (int p = 0; p < PPT; ++p)
#pragma unroll
        for (int a = 0; a < DIM; ++a) { vr[a][p] = T(0); vi[a][p] = T(0); }
    } else {
      // residual r = i xi . sigma^ accumulated component by component
#pragma unroll
      for (int p = 0; p < PPT; ++p)
#pragma unroll
        for (int a = 0; a < DIM; ++a) { vr[a][p] = T(0); vi[a][p] = T(0); }
      forward(D.S, std::integral_constant<int, S>{}, [&](int c, int p, T re, T im) {
        T xi[DIM], xi2, wgt;
        bool valid;
        long long gidx;
        int n;
        point_xi(p, xi, xi2, valid, gidx, wgt, n);
        const int a = va<DIM>(c), b = vb<DIM>(c);
        // i xi_b s -> (-xi_b im, xi_b re)
        vr[a][p] -= xi[b] * im;
        vi[a][p] += xi[b] * re;
        if (a != b) {
          vr[b][p] -= xi[a] * im;
          vi[b][p] += xi[a] * re;
        }
      });
    }
    // + f^ (already projected off Z), Parseval partial, update
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      T xi[DIM], xi2, wgt;
      bool valid;
      long long gidx;
      int n;
      point_xi(p, xi, xi2, valid, gidx, wgt, n);
      if (!valid) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) { vr[a][p] = T(0); vi[a][p] = T(0); }
        continue;
      }
      T ur[DIM], ui[DIM];
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const typename C2<T>::type f = ldc<T>(static_cast<const char*>(D.F) + a * P * cbytes, gidx);
        vr[a][p] += f.x;
        vi[a][p] += f.y;
        part += double(wgt) * (double(vr[a][p]) * double(vr[a][p]) + double(vi[a][p]) * double(vi[a][p]));
        ur[a] = vr[a][p];
        ui[a] = vi[a][p];
      }
      apply_n0<T, DIM>(xi, xi2, c0, mu0, ur, ui);   // N0 r
      if constexpr (MODE == M_CG_INIT) {
        // r0 stored, z0 = N0 r0 = p0 stored, r.z partial; p0 drives the next
        // operator application
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          stc<T>(static_cast<char*>(D.R) + a * P * cbytes, gidx, vr[a][p], vi[a][p]);
          stc<T>(static_cast<char*>(D.Pd) + a * P * cbytes, gidx, ur[a], ui[a]);
          part2 += double(wgt) * (double(vr[a][p]) * double(ur[a]) + double(vi[a][p]) * double(ui[a]));
          vr[a][p] = ur[a];
          vi[a][p] = ui[a];
        }
      } else {
        const void* uin = D.U[cur];
        void* uout = (MODE == M_INIT) ? D.U[0] : D.U[cur ^ 1];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          T nr = ur[a], ni = ui[a];
          if constexpr (MODE == M_ITER) {
            const typename C2<T>::type u0 = ldc<T>(static_cast<const char*>(uin) + a * P * cbytes, gidx);
            nr += u0.x;
            ni += u0.y;
          }
          stc<T>(static_cast<char*>(uout) + a * P * cbytes, gidx, nr, ni);
          vr[a][p] = nr;
          vi[a][p] = ni;
        }
      }
    }
    // next strain spectrum and its inverse transform
    inverse(D.S, std::integral_constant<int, S>{}, strain_gen);
  } else if constexpr (MODE == M_MAT) {
    const void* uin = D.U[cur];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      T xi[DIM], xi2, wgt;
      bool valid;
      long long gidx;
      int n;
      point_xi(p, xi, xi2, valid, gidx, wgt, n);
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        T re = T(0), im = T(0);
        if (valid) {
          const typename C2<T>::type u0 = ldc<T>(static_cast<const char*>(uin) + a * P * cbytes, gidx);
          re = u0.x;
          im = u0.y;
        }
        vr[a][p] = re;
        vi[a][p] = im;
      }
    }
    inverse(D.S, std::integral_constant<int, S>{}, strain_gen);
    inverse(static_cast<char*>(D.S) + S * P * cbytes, std::integral_constant<int, DIM>{}, [&](int c, int p, T& re, T& im) {
      re = vr[c][p] * inv_n;
      im = vi[c][p] * inv_n;
    });
    return;
  } else if constexpr (MODE == M_CG_AP) {
    // q = A p = -i xi . sigma^(p): stored, and the partial p.q
#pragma unroll
    for (int p = 0; p < PPT; ++p)
#pragma unroll
      for (int a = 0; a < DIM; ++a) { vr[a][p] = T(0); vi[a][p] = T(0); }
    forward(D.S, std::integral_constant<int, S>{}, [&](int c, int p, T re, T im) {
      T xi[DIM], xi2, wgt;
      bool valid;
      long long gidx;
      int n;
      point_xi(p, xi, xi2, valid, gidx, wgt, n);
      const int a = va<DIM>(c), b = vb<DIM>(c);
      // -i xi_b s -> (xi_b im, -xi_b re)
      vr[a][p] += xi[b] * im;
      vi[a][p] -= xi[b] * re;
      if (a != b) {
        vr[b][p] += xi[a] * im;
        vi[b][p] -= xi[a] * re;
      }
    });
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      T xi[DIM], xi2, wgt;
      bool valid;
      long long gidx;
      int n;
      point_xi(p, xi, xi2, valid, gidx, wgt, n);
      if (!valid) continue;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const typename C2<T>::type pd = ldc<T>(static_cast<const char*>(D.Pd) + a * P * cbytes, gidx);
        stc<T>(static_cast<char*>(D.Q) + a * P * cbytes, gidx, vr[a][p], vi[a][p]);
        part += double(wgt) * (double(pd.x) * double(vr[a][p]) + double(pd.y) * double(vi[a][p]));
      }
    }
  } else if constexpr (MODE == M_CG_DIR) {
    // p = N0 r + beta p, stored, then eps^(p) / |N| and its inverse transform
    const T beta = T(St->beta);
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      T xi[DIM], xi2, wgt;
      bool valid;
      long long gidx;
      int n;
      point_xi(p, xi, xi2, valid, gidx, wgt, n);
      if (!valid) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) { vr[a][p] = T(0); vi[a][p] = T(0); }
        continue;
      }
      T zr[DIM], zi[DIM];
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const typename C2<T>::type r = ldc<T>(static_cast<const char*>(D.R) + a * P * cbytes, gidx);
        zr[a] = r.x;
        zi[a] = r.y;
      }
      apply_n0<T, DIM>(xi, xi2, c0, mu0, zr, zi);
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const typename C2<T>::type pd = ldc<T>(static_cast<const char*>(D.Pd) + a * P * cbytes, gidx);
        const T nr = zr[a] + beta * pd.x, ni = zi[a] + beta * pd.y;
        stc<T>(static_cast<char*>(D.Pd) + a * P * cbytes, gidx, nr, ni);
        vr[a][p] = nr;
        vi[a][p] = ni;
      }
    }
    inverse(D.S, std::integral_constant<int, S>{}, strain_gen);
  }

  // FP64 partial sums of this item, one slot per item (fixed order later)
  if constexpr (MODE == M_INIT || MODE == M_ITER || MODE == M_CG_INIT || MODE == M_CG_AP) {
    const double s1 = block_sum(part, red);
    if constexpr (MODE == M_CG_INIT) {
      const double s2 = block_sum(part2, red);
      if (tid == 0) {
        D.partial[2 * local] = s1;
        D.partial[2 * local + 1] = s2;
      }
    } else {
      if (tid == 0) D.partial[2 * local] = s1;
    }
  }
}

// ---------------------------------------------------------------------------
// CG pointwise update: u += alpha p, r -= alpha q, partials r.z and r.r
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__device__ void cg_update_item(const InstDesc& D, InstState* St, int local, unsigned char* smem) {
  // one item = NT * 4 consecutive half-spectrum points
  const int tid = threadIdx.x;
  double* red = reinterpret_cast<double*>(smem);
  const T alpha = T(St->alpha);
  const T mu0 = T(D.mu0);
  const T c0 = T((D.lam0 + D.mu0) / (D.lam0 + 2.0 * D.mu0));
  const size_t cbytes = sizeof(T) * 2;
  const long long P = D.P;
  double prz = 0.0, prr = 0.0;
  for (int q = 0; q < 4; ++q) {
    const long long g = (long long)local * NT * 4 + q * NT + tid;
    if (g >= P) break;
    const int kx = int(g % D.nxh);
    const long long rest = g / D.nxh;
    T xi[DIM];
    xi[0] = T(wavenum(kx, D.nx, D.kx));
    if constexpr (DIM == 3) {
      xi[1] = T(wavenum(int(rest % D.ny), D.ny, D.ky));
      xi[2] = T(wavenum(int(rest / D.ny), D.nz, D.kz));
    } else {
      xi[1] = T(wavenum(int(rest), D.ny, D.ky));
    }
    T xi2 = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) xi2 += xi[a] * xi[a];
    const double wgt = (kx == 0 || kx == (D.nx >> 1)) ? 1.0 : 2.0;
    T rr[DIM], ri[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const typename C2<T>::type u = ldc<T>(static_cast<const char*>(D.U[0]) + a * P * cbytes, g);
      const typename C2<T>::type pd = ldc<T>(static_cast<const char*>(D.Pd) + a * P * cbytes, g);
      const typename C2<T>::type r = ldc<T>(static_cast<const char*>(D.R) + a * P * cbytes, g);
      const typename C2<T>::type qv = ldc<T>(static_cast<const char*>(D.Q) + a * P * cbytes, g);
      stc<T>(static_cast<char*>(D.U[0]) + a * P * cbytes, g, u.x + alpha * pd.x, u.y + alpha * pd.y);
      rr[a] = r.x - alpha * qv.x;
      ri[a] = r.y - alpha * qv.y;
      stc<T>(static_cast<char*>(D.R) + a * P * cbytes, g, rr[a], ri[a]);
      prr += wgt * (double(rr[a]) * double(rr[a]) + double(ri[a]) * double(ri[a]));
    }
    T zr[DIM], zi[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) { zr[a] = rr[a]; zi[a] = ri[a]; }
    apply_n0<T, DIM>(xi, xi2, c0, mu0, zr, zi);
#pragma unroll
    for (int a = 0; a < DIM; ++a) prz += wgt * (double(rr[a]) * double(zr[a]) + double(ri[a]) * double(zi[a]));
  }
  const double s1 = block_sum(prz, red);
  const double s2 = block_sum(prr, red);
  if (tid == 0) {
    D.partial[2 * local] = s1;
    D.partial[2 * local + 1] = s2;
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool gated(int mode) {
  return mode == M_ITER || mode == M_CG_AP || mode == M_CG_UPD || mode == M_CG_DIR || mode == M_CG_INIT;
}

#define LSFFT_LEN_CASES(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(256)

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_xpass(const InstDesc* __restrict__ descs, InstState* __restrict__ states,
                                              const WorkItem* __restrict__ items, const int* __restrict__ nitems,
                                              const double* __restrict__ lame, const T* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n_items = *nitems;
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const WorkItem it = items[w];
    const InstDesc& D = descs[it.inst];
    if (gated(MODE) && states[it.inst].status != ST_RUNNING) continue;
    if (D.dim == 3) {
      switch (D.nx) {
#define X(L) case L: xpass_item<T, L, 3, MODE>(D, it.local, lame, tw, smem); break;
        LSFFT_LEN_CASES(X)
#undef X
        default: break;
      }
    } else {
      switch (D.nx) {
#define X(L) case L: xpass_item<T, L, 2, MODE>(D, it.local, lame, tw, smem); break;
        LSFFT_LEN_CASES(X)
#undef X
        default: break;
      }
    }
    __syncthreads();
  }
}

template <typename T, int DIR>
__global__ __launch_bounds__(NT) void k_ypass(const InstDesc* __restrict__ descs, InstState* __restrict__ states,
                                              const WorkItem* __restrict__ items, const int* __restrict__ nitems,
                                              const T* __restrict__ tw, int which, int ncomp_extra, int gate) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n_items = *nitems;
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const WorkItem it = items[w];
    const InstDesc& D = descs[it.inst];
    if (gate && states[it.inst].status != ST_RUNNING) continue;
    void* buf = (which == 0) ? D.S : D.F;
    const int ncomp = (which == 0) ? D.ncomp_s + ncomp_extra : D.dim;
    switch (D.ny) {
#define X(L) case L: ypass_item<T, L, DIR>(D, it.local, buf, ncomp, tw, smem); break;
      LSFFT_LEN_CASES(X)
#undef X
      default: break;
    }
    __syncthreads();
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_green(const InstDesc* __restrict__ descs, InstState* __restrict__ states,
                                              const WorkItem* __restrict__ items, const int* __restrict__ nitems,
                                              const T* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n_items = *nitems;
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const WorkItem it = items[w];
    const InstDesc& D = descs[it.inst];
    InstState* St = states + it.inst;
    if (gated(MODE) && St->status != ST_RUNNING) continue;
    if (D.dim == 3) {
      switch (D.nz) {
#define X(L) case L: green_item<T, L, 3, MODE>(D, St, it.local, tw, smem); break;
        LSFFT_LEN_CASES(X)
#undef X
        default: break;
      }
    } else {
      switch (D.ny) {
#define X(L) case L: green_item<T, L, 2, MODE>(D, St, it.local, tw, smem); break;
        LSFFT_LEN_CASES(X)
#undef X
        default: break;
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_cg_update(const InstDesc* __restrict__ descs, InstState* __restrict__ states,
                                                  const WorkItem* __restrict__ items, const int* __restrict__ nitems) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n_items = *nitems;
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const WorkItem it = items[w];
    const InstDesc& D = descs[it.inst];
    InstState* St = states + it.inst;
    if (St->status != ST_RUNNING) continue;
    if (D.dim == 3) cg_update_item<T, 3>(D, St, it.local, smem);
    else cg_update_item<T, 2>(D, St, it.local, smem);
    __syncthreads();
  }
}

#ifdef LSFFT_MISC_TU
// Stopping rule and lifecycle of one solve after a residual evaluation.
__device__ void judge(const InstDesc& D, InstState& St, double delta) {
  St.residual = delta;
  if (D.history) D.history[St.iter] = delta;
  if (!(delta == delta) || delta > 1e300) { St.status = ST_DIVERGED; return; }
  if (delta <= D.tol) { St.status = ST_OK; return; }
  if (St.iter >= D.max_iter) { St.status = ST_NOCONV; return; }
  if (delta < 0.99 * St.mark) {
    St.mark = delta;
    St.mark_iter = St.iter;
  } else if (St.iter - St.mark_iter >= 20) {
    St.status = ST_STAGNATED;
    return;
  }
  St.grow = (delta > St.prev) ? St.grow + 1 : 0;
  St.prev = delta;
  if (St.grow > 20) { St.status = ST_DIVERGED; return; }
  St.iter += 1;
}

// One block per solve: fixed-order FP64 sums of the per-item partials.
__global__ __launch_bounds__(NT) void k_reduce(const InstDesc* __restrict__ descs, InstState* __restrict__ states,
                                               const int* __restrict__ inst_list, int ninst, int mode) {
  __shared__ double red[NT / 64];
  if ((int)blockIdx.x >= ninst) return;
  const int i = inst_list[blockIdx.x];
  const InstDesc& D = descs[i];
  InstState& St = states[i];
  if (mode != M_INIT && St.status != ST_RUNNING) return;
  const int nslot = (mode == M_CG_UPD) ? (int)((D.P + NT * 4 - 1) / (NT * 4)) : D.items_g;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nslot; k += NT) {
    a += D.partial[2 * k];
    if (mode == M_CG_INIT || mode == M_CG_UPD) b += D.partial[2 * k + 1];
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x != 0) return;
  if (mode == M_INIT) {
    St.fnorm2 = a;
    St.iter = 0;
    St.mark = 1e308;
    St.mark_iter = 0;
    St.prev = 1e308;
    St.grow = 0;
    if (a == 0.0) {
      St.status = ST_OK;
      St.residual = 0.0;
      if (D.history) D.history[0] = 0.0;
    } else {
      St.status = ST_RUNNING;
    }
  } else if (mode == M_ITER) {
    judge(D, St, sqrt(a / St.fnorm2));
  } else if (mode == M_CG_INIT) {
    St.rz = b;
    const double delta = sqrt(a / St.fnorm2);
    St.residual = delta;
    if (D.history) D.history[0] = delta;
    if (!(delta == delta)) St.status = ST_DIVERGED;
    else if (delta <= D.tol) St.status = ST_OK;
    else if (D.max_iter <= 0) St.status = ST_NOCONV;
  } else if (mode == M_CG_AP) {
    St.pq = a;
    St.alpha = St.rz / a;
  } else if (mode == M_CG_UPD) {
    const double rz_new = a;
    St.beta = rz_new / St.rz;
    St.rz = rz_new;
    // the update produced iterate iter + 1
    St.iter += 1;
    const double delta = sqrt(b / St.fnorm2);
    St.residual = delta;
    if (D.history) D.history[St.iter] = delta;
    if (!(delta == delta) || delta > 1e300) St.status = ST_DIVERGED;
    else if (delta <= D.tol) St.status = ST_OK;
    else if (St.iter >= D.max_iter) St.status = ST_NOCONV;
    else {
      if (delta < 0.99 * St.mark) {
        St.mark = delta;
        St.mark_iter = St.iter;
      } else if (St.iter - St.mark_iter >= 50) {
        St.status = ST_STAGNATED;
      }
    }
  }
}

// Largest phase id of each solve's map (argument validation on the device).
__global__ __launch_bounds__(NT) void k_phase_max(const uint8_t* __restrict__ phase, long long n, int* __restrict__ out) {
  __shared__ int red[NT];
  int m = 0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    m = max(m, (int)phase[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, red[0]);
}

#endif  // LSFFT_MISC_TU

// Translated averaging (Eqs. 3.5-3.6): for every voxel, in the fixed order of
// the group's shifts, sum u, u V, eps, eps V, sigma, sigma V and V, V the
// indicator of the inclusion phase in the shifted microstructure.  Sums are
// added to the FP64 accumulator; no atomics, one thread per voxel.
template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_accumulate(const InstDesc* __restrict__ descs, const GroupDesc* __restrict__ groups,
                                                   int g, const double* __restrict__ lame) {
  constexpr int S = (DIM == 3) ? 6 : 3;
  constexpr int NC = 2 * DIM + 4 * S + 1;
  const GroupDesc G = groups[g];
  const InstDesc& D0 = descs[G.first];
  const long long nvox = D0.nvox;
  for (long long v = (long long)blockIdx.x * NT + threadIdx.x; v < nvox; v += (long long)gridDim.x * NT) {
    const int x = int(v % D0.nx);
    const long long rest = v / D0.nx;
    const int y = int(rest % D0.ny);
    const int z = int(rest / D0.ny);
    double acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0.0;
    for (int i = G.first; i < G.first + G.count; ++i) {
      const InstDesc& D = descs[i];
      const long long pidx = ((long long)wrap(z - D.sz, D.nz) * D.ny + wrap(y - D.sy, D.ny)) * D.nx + wrap(x - D.sx, D.nx);
      const int ph = D.phase[pidx];
      const double ind = (ph == G.incl_phase) ? 1.0 : 0.0;
      const double lam = lame[2 * (D.lame_off + ph)], mu = lame[2 * (D.lame_off + ph) + 1];
      const T* ue = reinterpret_cast<const T*>(D.out_u);
      const T* ee = reinterpret_cast<const T*>(D.out_eps);
      double e[S];
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        const double uv = double(ue[c * nvox + v]);
        acc[c] += uv;
        acc[DIM + c] += uv * ind;
      }
      double tr = 0.0;
#pragma unroll
      for (int c = 0; c < S; ++c) {
        e[c] = double(ee[c * nvox + v]);
        if (c < DIM) tr += e[c];
      }
#pragma unroll
      for (int c = 0; c < S; ++c) {
        const double sg = 2.0 * mu * e[c] + (c < DIM ? lam * tr : 0.0);
        acc[2 * DIM + c] += e[c];
        acc[2 * DIM + S + c] += e[c] * ind;
        acc[2 * DIM + 2 * S + c] += sg;
        acc[2 * DIM + 3 * S + c] += sg * ind;
      }
      acc[NC - 1] += ind;
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) G.avg[k * nvox + v] += acc[k];
  }
}

#ifdef LSFFT_MISC_TU
__global__ __launch_bounds__(NT) void k_scale(double* __restrict__ a, long long n, double s) {
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) a[i] *= s;
}
#endif  // LSFFT_MISC_TU

// ---------------------------------------------------------------------------
// LDS requirements (bytes) of one work item, per precision and length
// ---------------------------------------------------------------------------
template <typename T, int L> constexpr size_t lds_x() {
  using G = RowGeom<T, L / 2>;
  return sizeof(T) * (4 * G::MR * G::SM + 2 * L + 2 * kMaxPhases);
}
template <typename T, int L> constexpr size_t lds_strided() {
  using G = StridedGeom<T, L>;
  return sizeof(T) * (4 * G::ELEMS + 2 * L + 2) + sizeof(double) * 8;
}
template <typename T, int L> constexpr int tiles_strided(int nxh) {
  return (nxh + StridedGeom<T, L>::MP - 1) / StridedGeom<T, L>::MP;
}

}  // namespace lsfft

