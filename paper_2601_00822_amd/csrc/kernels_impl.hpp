// HIP kernels of the BFCS Lippmann-Schwinger solver for gfx950.
//
// One basic-scheme iteration is four sweeps over HBM (3D), each a persistent
// kernel walking a device work list of (solve, tile) items:
//
//   ypass<inv>  : inverse y transforms of the strain spectrum (3D only),
//                 one component per item
//   xpass<ITER> : per block of x rows: half spectrum -> real (C2R), Hooke's
//                 law sigma = lam(x) tr(eps) I + 2 mu(x) eps (Eq. 2.2) on the
//                 real values held in registers, real -> half spectrum (R2C);
//                 the real fields never reach HBM
//   ypass<fwd>  : forward y transforms of the stress spectrum (3D only)
//   green<ITER> : along the outermost axis: forward transform of sigma, the
//                 equilibrium residual r = i xi . sigma^ + f^ with its FP64
//                 Parseval partial sum, the update u^ += N0(xi) r (Algorithm 1
//                 in displacement form), the next strain spectrum
//                 sym(i xi (x) u^) / |N| and its inverse transform
//
// followed by a one-block-per-solve FP64 reduction that evaluates the stopping
// rule and retires converged solves.  2D grids skip the y sweeps (the outer
// axis is y).  The same kernels, in other modes, transform the force, form the
// free term u^b = N0 f^ (Eqs. 2.8-2.9), run the conjugate-gradient variant and
// materialize u, eps and sigma.
//
// Transform stages: the first pass of every transform reads its inputs from
// HBM (or from the pointwise stage) straight into registers, and the last
// pass leaves its outputs in registers, which the next stage consumes where
// they are; only the middle passes go through LDS.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fft_core.hpp"
#include "lsfft_internal.hpp"

namespace lsfft {

// ---------------------------------------------------------------------------
// tile geometry
// ---------------------------------------------------------------------------
constexpr int pow2floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Threads per workgroup and tile elements per component, per kernel family:
// x and y passes hold 8 (FP32) / 4 (FP64) points per thread, the outer pass 4.
template <typename T> struct Cfg;
#ifndef LSFFT_XNTH_F32
#define LSFFT_XNTH_F32 256
#endif
#ifndef LSFFT_XE_F32
#define LSFFT_XE_F32 2048
#endif
#ifndef LSFFT_XNTH_F64
#define LSFFT_XNTH_F64 128
#endif
#ifndef LSFFT_XE_F64
#define LSFFT_XE_F64 512
#endif
template <> struct Cfg<float> {
  static constexpr int NTH = 256, E = 2048;              // y pass
  static constexpr int NTH_X = LSFFT_XNTH_F32, EX = LSFFT_XE_F32;   // x pass
  static constexpr int NTH_G = 256, E_G = 1024;          // outer pass
};
template <> struct Cfg<double> {
  static constexpr int NTH = 128, E = 1024;
  static constexpr int NTH_X = LSFFT_XNTH_F64, EX = LSFFT_XE_F64;
  static constexpr int NTH_G = 256, E_G = 1024;
};

// pencils per strided tile of length N (y pass, outer pass)
template <typename T, int N> struct SGeom {
  static constexpr int MP = clampi(pow2floor(Cfg<T>::E / N), 1, 64);
  // outer pass: FP32 pencils of 256 or more points come 8 to a tile (64-byte
  // runs per line instead of 32), at 2 waves per SIMD (see WavesG)
#ifndef LSFFT_G2_MIN
#define LSFFT_G2_MIN 256
#endif
  static constexpr int MPG = clampi(pow2floor((sizeof(T) == 4 && N >= LSFFT_G2_MIN ? 2 * Cfg<T>::E_G : Cfg<T>::E_G) / N), 1, 64);
};

// LDS rows of pencil-fastest tiles (y pass, outer pass): one row of LP
// words per index.  FP32 tiles of 8 or 16 pencils use unpadded rows plus a
// padding row after every 8 (TileFft SWZ 2); the others pad each row by one
// word.  E is the words of one (re or im) buffer.
template <typename T, int N, int MP> struct PencilRows {
  static constexpr bool pad8 = sizeof(T) == 4 && (MP == 8 || MP == 16);
  static constexpr int SWZ = pad8 ? 2 : 0;
  static constexpr int LP = pad8 ? MP : (MP > 1 ? MP + 1 : 1);
  static constexpr int E = LP * (pad8 ? N + (N - 1) / 8 + 1 : N);
};

// rows per x tile (H = nx / 2 complex points per row); odd LDS pitches.
// DIV divides the tile's entries (schedule variant 1 of the x pass).
template <typename T, int H, int DIV = 1> struct XGeom {
  static constexpr int MR = clampi(pow2floor(Cfg<T>::EX / DIV / H), 1, 64);
  static constexpr int SM = ((H + 1) % 2 == 1) ? (H + 1) : (H + 2);  // fold tile, H + 1 entries
  static constexpr int SKW = H + (H >> 5) + 1;                        // skewed row length
  static constexpr int SM2 = (SKW % 2 == 1) ? SKW : (SKW + 1);         // transform staging
};

// occupancy targets (waves per SIMD) that bound the register allocation
template <typename T, int NG> struct WavesG { static constexpr int value = (NG >= LSFFT_G2_MIN) ? 2 : 3; };
template <int NG> struct WavesG<double, NG> { static constexpr int value = 2; };
#ifndef LSFFT_WAVES_X
#define LSFFT_WAVES_X 3
#endif
#ifndef LSFFT_WAVES_Y
#define LSFFT_WAVES_Y 4
#endif

// ---------------------------------------------------------------------------
// schedules: compiled variants of a pass kernel for one transform length.
// Variant 0 is the hand-tuned default; FP32 3D plans also carry the others
// for lengths of 32 points and more, and lsfft_autotune times them per
// length and keeps the fastest.
//   outer pass: 0 default tile; 1 half the pencils (finer work items, same
//               occupancy target); 2 twice the pencils (512-thread
//               workgroups on 256-point pencils, full 128-byte lines)
//   y pass:     0 default; 1 twice the pencils at 2 waves per SIMD; 2 the
//               other radix order (PlanG instead of Plan)
//   x pass:     0 default; 1 row tiles of half the entries, register-staged
//               (fewer registers per thread, finer items); 2 the other radix
//               order of the core (PlanG instead of Plan)
// The outer pass keeps PlanG (last radix at most 4): its tiles hold the
// points of four pass kinds in registers at once, and the plans ending in
// radix 8 spill there.
// ---------------------------------------------------------------------------
constexpr int kVarG = 3, kVarY = 3, kVarX = 3;
template <typename T, int N, int V> struct GSched {
  static constexpr int MP0 = SGeom<T, N>::MPG;
#ifdef LSFFT_WAVES_G
  static constexpr int W0 = LSFFT_WAVES_G;
#else
  static constexpr int W0 = WavesG<T, N>::value;
#endif
  static constexpr int MP = V == 1 ? (MP0 > 1 ? MP0 / 2 : 1) : V == 2 ? (MP0 < 64 ? 2 * MP0 : 64) : MP0;
  static constexpr int NTH = (V == 2 && N >= 256) ? 2 * Cfg<T>::NTH_G : Cfg<T>::NTH_G;
  static constexpr int WAVES = V == 2 ? 2 : W0;
};
template <typename T, int N, int V> struct YSched {
  static constexpr int MP = V == 1 ? clampi(pow2floor(2 * Cfg<T>::E / N), 1, 64) : SGeom<T, N>::MP;
  static constexpr int WAVES = V == 1 ? 2 : LSFFT_WAVES_Y;
  static constexpr bool ALT = V == 2;
};
template <int V> struct XSched {
  static constexpr int EX_DIV = V == 1 ? 2 : 1;   // row-tile entries: Cfg EX / EX_DIV
  static constexpr bool ALT = V == 2;
};
// radix plan family: the default one or the other
template <bool ALT_IS_G> struct PlanPick;
template <> struct PlanPick<false> { template <int N> using P = Plan<N>; };
template <> struct PlanPick<true> { template <int N> using P = PlanG<N>; };

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// scheduling fence: the compiler may not move instructions across it, which
// bounds how many loads it hoists ahead (and so the live registers)
#define LSFFT_FENCE() __builtin_amdgcn_sched_barrier(0)

template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };

// HBM accesses go through pointers in the global address space.  The
// buffers are reached through pointers stored in the solve descriptor, whose
// address space the compiler cannot infer; generic (flat) accesses would
// also count against the LDS wait counter, so every LDS barrier would wait
// for all loads in flight.
#if defined(__HIP_DEVICE_COMPILE__)
#define LSFFT_GLOBAL __attribute__((address_space(1)))
#else
#define LSFFT_GLOBAL
#endif
template <typename V>
__device__ __forceinline__ V gld(const void* base, long long i) {
  return ((const LSFFT_GLOBAL V*)base)[i];
}
template <typename V>
__device__ __forceinline__ void gst(void* base, long long i, V v) {
  ((LSFFT_GLOBAL V*)base)[i] = v;
}

// Complex entry i of a spectral component.  The byte offset is formed in 32
// bits (a component holds at most 256 x 256 x 128 entries of 16 bytes, and
// no index passed here exceeds the nine components of a work buffer), so
// the access is a uniform 64-bit base plus an unsigned 32-bit lane offset:
// one VGPR per address instead of a 64-bit lane address.
// FP64 keeps a sign-extended 64-bit index: with the 32-bit offset the FP64
// register-staged x pass spills (92 bytes per lane instead of 16).
template <typename T>
__device__ __forceinline__ typename C2<T>::type ldc(const void* base, unsigned i) {
  using V = typename C2<T>::type;
  if constexpr (sizeof(T) == 8) return gld<V>(base, (long long)(int)i);
  const unsigned off = i * (unsigned)sizeof(V);
  return *reinterpret_cast<const LSFFT_GLOBAL V*>((const LSFFT_GLOBAL char*)base + off);
}
template <typename T>
__device__ __forceinline__ void stc(void* base, unsigned i, T re, T im) {
  using V = typename C2<T>::type;
  V v;
  v.x = re;
  v.y = im;
  if constexpr (sizeof(T) == 8) {
    gst<V>(base, (long long)(int)i, v);
    return;
  }
  const unsigned off = i * (unsigned)sizeof(V);
  *reinterpret_cast<LSFFT_GLOBAL V*>((LSFFT_GLOBAL char*)base + off) = v;
}
// the same store, marked non-temporal (streamed past the caches)
template <typename T>
__device__ __forceinline__ void stc_nt(void* base, unsigned i, T re, T im) {
  typedef T V2 __attribute__((ext_vector_type(2)));
  V2 v;
  v.x = re;
  v.y = im;
  __builtin_nontemporal_store(v, reinterpret_cast<LSFFT_GLOBAL V2*>((LSFFT_GLOBAL char*)base + (size_t)i * sizeof(V2)));
}
template <typename T>
__device__ __forceinline__ const char* cptr(const void* base, long long comp_stride, int c) {
  return static_cast<const char*>(base) + (size_t)c * comp_stride * sizeof(T) * 2;
}
template <typename T>
__device__ __forceinline__ char* mptr(void* base, long long comp_stride, int c) {
  return static_cast<char*>(base) + (size_t)c * comp_stride * sizeof(T) * 2;
}

// signed wavevector component of index k on an axis of n points; zero on the
// Nyquist index
__device__ __forceinline__ double wavenum(int k, int n, double scale) {
  const int h = n >> 1;
  if (k == h) return 0.0;
  return scale * double(k < h ? k : k - n);
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// load exp(-2 pi i k / L), k < L, into LDS from the plan's twiddle table
template <typename T, int L, int NTH>
__device__ __forceinline__ void load_tw(T* twr, T* twi, const T* table, int tid) {
  constexpr int off = tw_offset(L);
  static_assert(off >= 0, "unsupported transform length");
  for (int k = tid; k < L; k += NTH) {
    twr[k] = table[2 * (off + k)];
    twi[k] = table[2 * (off + k) + 1];
  }
}

// block-wide FP64 sum (deterministic for a fixed block size), valid in thread 0
template <int NTH>
__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < NTH / 64; ++w) s += red[w];
  }
  return s;
}

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
template <int DIM> __host__ __device__ constexpr int va(int c) {
  if constexpr (DIM == 3) return c < 3 ? c : (c == 3 ? 1 : 0);
  else return c < 2 ? c : 0;
}
template <int DIM> __host__ __device__ constexpr int vb(int c) {
  if constexpr (DIM == 3) return c < 3 ? c : (c == 3 ? 2 : (c == 4 ? 2 : 1));
  else return c < 2 ? c : 1;
}

// ---------------------------------------------------------------------------
// stopping rule and the fused FP64 reduction
// ---------------------------------------------------------------------------
// Lifecycle of one solve after a residual evaluation (basic scheme).
__device__ inline void judge(const InstDesc& D, InstState& St, double delta) {
  St.residual = delta;
  if (D.history) D.history[St.iter] = delta;
  if (!(delta == delta) || delta > 1e300) { St.status = ST_DIVERGED; return; }
  if (delta <= D.tol) { St.status = ST_OK; return; }
  if (St.iter >= D.max_iter) { St.status = ST_NOCONV; return; }
  // a residual that grew over 20 iterations in a row diverges; this is
  // tested before stagnation, which the same 20 iterations would also meet
  St.grow = (delta > St.prev) ? St.grow + 1 : 0;
  St.prev = delta;
  if (St.grow >= 20) { St.status = ST_DIVERGED; return; }
  if (delta < 0.99 * St.mark) {
    St.mark = delta;
    St.mark_iter = St.iter;
  } else if (St.iter - St.mark_iter >= 20) {
    St.status = ST_STAGNATED;
    return;
  }
  St.iter += 1;
}

// Apply the totals (a, b) of a launch's partial sums to the solve's state.
__device__ inline void finalize(const InstDesc& D, InstState& St, int mode, double a, double b) {
  if (mode == M_INIT) {
    St.fnorm2 = a;
    St.iter = 0;
    St.start_step = 0;
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
    else if (D.cg_start) St.start_step = 1;      // Algorithm 3: u1 = b^A first
    else if (delta <= D.tol) St.status = ST_OK;
    else if (D.max_iter <= 0) St.status = ST_NOCONV;
  } else if (mode == M_CG_AP) {
    St.pq = a;
    // the printed start u1 = b^A is the update u1 += 1 * p with p = r = b^A
    St.alpha = St.start_step ? 1.0 : St.rz / a;
  } else if (mode == M_CG_UPD) {
    const double rz_new = a;
    const double delta = sqrt(b / St.fnorm2);
    if (St.start_step) {
      // r = b^A - A(b^A) of the printed start; the next direction is r
      // (beta = 0) and no iteration is counted
      St.start_step = 0;
      St.beta = 0.0;
      St.rz = rz_new;
      St.residual = delta;
      if (D.history) D.history[0] = delta;
      if (!(delta == delta) || delta > 1e300) St.status = ST_DIVERGED;
      else if (delta <= D.tol) St.status = ST_OK;
      else if (D.max_iter <= 0) St.status = ST_NOCONV;
      return;
    }
    St.beta = rz_new / St.rz;
    St.rz = rz_new;
    St.iter += 1;
    St.residual = delta;
    if (D.history) D.history[St.iter] = delta;
    if (!(delta == delta) || delta > 1e300) St.status = ST_DIVERGED;
    else if (delta <= D.tol) St.status = ST_OK;
    else if (St.iter >= D.max_iter) St.status = ST_NOCONV;
    else {
      // the plain CG's residual is far from monotone: a longer window
      const int window = D.precond ? 50 : 1000;
      if (delta < 0.99 * St.mark) {
        St.mark = delta;
        St.mark_iter = St.iter;
      } else if (St.iter - St.mark_iter >= window) {
        St.status = ST_STAGNATED;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// x pass
// ---------------------------------------------------------------------------
// Row block of MR rows (row = z * ny + y).  Per component: the H + 1 half
// spectrum entries of each row (X[0] and X[H] unpacked from the row's first
// entry, which holds X[0] + i X[H]) are staged in LDS; the fold
//   Z'[k] = (X[k] + conj X[H-k]) + i exp(+2 pi i k / NX) (X[k] - conj X[H-k])
// feeds a length-H inverse transform whose output is NX (a[2n] + i a[2n+1]);
// the forward direction is the mirror image:
//   X[k] = E + exp(-2 pi i k / NX) O, E = (Z[k] + conj Z[H-k]) / 2,
//   O = -i (Z[k] - conj Z[H-k]) / 2.
template <typename T, int NX, int DIM, int MODE, int V>
__device__ void xpass_item_std(const InstDesc& D, int local, const double* __restrict__ lame,
                               const T* __restrict__ twtab, unsigned char* smem) {
  constexpr int NTH = Cfg<T>::NTH_X;
  constexpr int H = NX / 2;
  using G = XGeom<T, H, XSched<V>::EX_DIV>;
  constexpr int MR = G::MR, SM = G::SM, SM2 = G::SM2;
  constexpr int S = (DIM == 3) ? 6 : 3;
  using PF = PlanPick<XSched<V>::ALT>;
  using FI = TileFft<T, H, +1, true, MR, SM2, 1, 2, true, NTH, PF::template P, true>;   // C2R core
  using FF = TileFft<T, H, -1, false, MR, SM2, 1, 2, true, NTH, PF::template P, true>;  // R2C core
  static_assert(FI::RL == FF::R0 && FI::BL == FF::B0, "x transforms must chain in registers");
  constexpr int BP = FI::BL, RP = FI::RL;          // points held per thread: BP x RP
  constexpr int TOTP = FI::TOTL;

  T* ar = reinterpret_cast<T*>(smem);              // fold tile MR x SM
  T* ai = ar + MR * SM;
  T* br = ai + MR * SM;                            // transform staging MR x SM2
  T* bi = br + MR * SM2;
  T* twr = bi + MR * SM2;
  T* twi = twr + NX;
  T* lam_s = twi + NX;
  T* mu_s = lam_s + kMaxPhases;
  const int tid = threadIdx.x;
  load_tw<T, NX, NTH>(twr, twi, twtab, tid);
  if constexpr (MODE != M_FT) {
    for (int p = tid; p < D.nphase; p += NTH) {
      lam_s[p] = T(gld<double>(lame, 2 * (D.lame_off + p)));
      mu_s[p] = T(gld<double>(lame, 2 * (D.lame_off + p) + 1));
    }
  }
  __syncthreads();
  const int nrows = D.ny * D.nz;
  // work item = (row tile, part): the part selects the component group, so
  // independent components of one row block run in parallel workgroups
  const int part = local / D.xtiles;
  const int row0 = (local - part * D.xtiles) * MR;
  const long long Pc = D.Pc;

  // forward core on registers `in` (positions j + r H/R0 of butterfly tid + q NTH),
  // then unfold through LDS and store component c of `dst`
  auto forward_store = [&](T (&in_r)[FF::B0][FF::R0], T (&in_i)[FF::B0][FF::R0], void* dst, int c) {
    T o_r[FF::BL][FF::RL], o_i[FF::BL][FF::RL];
    __syncthreads();   // staging buffer free
    FF::run(in_r, in_i, o_r, o_i, br, bi, twr, twi, tid);
    __syncthreads();   // previous users of the fold tile are done
#pragma unroll
    for (int q = 0; q < FF::BL; ++q) {
      const int b = tid + q * NTH;
      if (FF::TOTL % NTH == 0 || b < FF::TOTL) {
        int m, j;
        FF::template bj<FF::RL>(b, m, j);
#pragma unroll
        for (int r = 0; r < FF::RL; ++r) {
          const int n = j + r * (H / FF::RL);
          ar[m * SM + n] = o_r[q][r];
          ai[m * SM + n] = o_i[q][r];
        }
      }
    }
    __syncthreads();
    char* base = mptr<T>(dst, Pc, c);
    for (int e = tid; e < MR * H; e += NTH) {
      const int m = e / H;
      const int k = e - m * H;
      const int row = row0 + m;
      if (row >= nrows) continue;
      const T zr = ar[m * SM + k], zi = ai[m * SM + k];
      if (k == 0) {
        // X[0] = zr + zi and X[H] = zr - zi are real: one packed entry
        stc<T>(base, row * H, zr + zi, zr - zi);
        continue;
      }
      const T wr = ar[m * SM + H - k], wi = ai[m * SM + H - k];
      const T er = T(0.5) * (zr + wr), ei = T(0.5) * (zi - wi);
      const T dr = T(0.5) * (zr - wr), di = T(0.5) * (zi + wi);
      const T orr = di, oi = -dr;
      const T cr = twr[k], ci = twi[k];
      const T xr = er + cr * orr - ci * oi, xi = ei + cr * oi + ci * orr;
      stc<T>(base, row * H + k, xr, xi);
    }
  };

  if constexpr (MODE == M_FT) {
    // real force rows -> half spectrum of F, component `part`
    {
      const int c = part;
      const T* src = reinterpret_cast<const T*>(D.f_in) + (long long)c * D.nvox;
      T in_r[FF::B0][FF::R0], in_i[FF::B0][FF::R0];
#pragma unroll
      for (int q = 0; q < FF::B0; ++q) {
        const int b = tid + q * NTH;
        int m, j;
        FF::template bj<FF::R0>(b, m, j);
        const bool ok = (FF::TOT0 % NTH == 0 || b < FF::TOT0) && row0 + m < nrows;
#pragma unroll
        for (int r = 0; r < FF::R0; ++r) {
          const int n = j + r * (H / FF::R0);
          T re = T(0), im = T(0);
          if (ok) {
            const typename C2<T>::type v =
                gld<typename C2<T>::type>(src + (row0 + m) * NX, n);
            re = v.x;
            im = v.y;
          }
          in_r[q][r] = re;
          in_i[q][r] = im;
        }
      }
      forward_store(in_r, in_i, D.F, c);
    }
    return;
  } else {
    // C2R of component c of S into registers (real pairs at x = 2n, 2n + 1).
    // The H entries of each row of the block (element e = tid + u NTH) are
    // loaded into registers with every load issued before the first use,
    // then staged in LDS for the fold as H + 1 entries: the packed entry
    // Z = X[0] + i X[H] becomes X[0] = (Re Z, 0) and X[H] = (Im Z, 0).
    constexpr int XE = MR * H;
    constexpr int XL = (XE + NTH - 1) / NTH;
    auto c2r = [&](int c, T (&o_r)[BP][RP], T (&o_i)[BP][RP]) {
      const char* src = cptr<T>(D.S, Pc, c);
      T pr[XL], pi[XL];
#pragma unroll
      for (int u = 0; u < XL; ++u) {
        const int e = tid + u * NTH;
        T re = T(0), im = T(0);
        if (XE % NTH == 0 || e < XE) {
          const int m = e / H;
          const int row = row0 + m;
          if (row < nrows) {
            const typename C2<T>::type v = ldc<T>(src, row * H + (e - m * H));
            re = v.x;
            im = v.y;
          }
        }
        pr[u] = re;
        pi[u] = im;
      }
      __syncthreads();   // fold tile and staging free
#pragma unroll
      for (int u = 0; u < XL; ++u) {
        const int e = tid + u * NTH;
        if (XE % NTH == 0 || e < XE) {
          const int m = e / H;
          const int k = e - m * H;
          if (k == 0) {
            ar[m * SM] = pr[u];
            ai[m * SM] = T(0);
            ar[m * SM + H] = pi[u];
            ai[m * SM + H] = T(0);
          } else {
            ar[m * SM + k] = pr[u];
            ai[m * SM + k] = pi[u];
          }
        }
      }
      __syncthreads();
      T in_r[FI::B0][FI::R0], in_i[FI::B0][FI::R0];
#pragma unroll
      for (int q = 0; q < FI::B0; ++q) {
        const int b = tid + q * NTH;
        int m, j;
        FI::template bj<FI::R0>(b, m, j);
        if (FI::TOT0 % NTH != 0 && b >= FI::TOT0) m = 0;
#pragma unroll
        for (int r = 0; r < FI::R0; ++r) {
          const int k = j + r * (H / FI::R0);
          const T xr = ar[m * SM + k], xi = ai[m * SM + k];
          const T yr = ar[m * SM + (H - k)], yi = -ai[m * SM + (H - k)];
          const T dr = xr - yr, di = xi - yi;
          const T cr = twr[k], ci = -twi[k];
          const T tr = cr * dr - ci * di, ti = cr * di + ci * dr;
          in_r[q][r] = xr + yr - ti;
          in_i[q][r] = xi + yi + tr;
        }
      }
      FI::run(in_r, in_i, o_r, o_i, br, bi, twr, twi, tid);
    };
    // write real pairs held in registers to component c of a real field
    auto write_real = [&](void* field, int c, const T (&v_r)[BP][RP], const T (&v_i)[BP][RP]) {
      T* dst = reinterpret_cast<T*>(field) + (long long)c * D.nvox;
#pragma unroll
      for (int q = 0; q < BP; ++q) {
        const int b = tid + q * NTH;
        int m, j;
        FI::template bj<RP>(b, m, j);
        if ((TOTP % NTH == 0 || b < TOTP) && row0 + m < nrows) {
#pragma unroll
          for (int r = 0; r < RP; ++r) {
            const int n = j + r * (H / RP);
            typename C2<T>::type v;
            v.x = v_r[q][r];
            v.y = v_i[q][r];
            gst<typename C2<T>::type>(dst + (row0 + m) * NX, n, v);
          }
        }
      }
    };
    // phase id of the microstructure shifted by s, at real index x of a row
    auto phase_at = [&](int row, int x) -> int {
      const int z = row / D.ny, y = row - (row / D.ny) * D.ny;
      const int rbase = (wrap(z - D.sz, D.nz) * D.ny + wrap(y - D.sy, D.ny)) * NX;
      return gld<uint8_t>(D.phase, rbase + ((D.sx == 0) ? x : wrap(x - D.sx, NX)));
    };
    // apply fn(point value&, lam, mu, half) at every point of this thread
    auto each_point = [&](auto&& fn) {
#pragma unroll
      for (int q = 0; q < BP; ++q) {
        const int b = tid + q * NTH;
        int m, j;
        FI::template bj<RP>(b, m, j);
        const int row = row0 + m;
        if ((TOTP % NTH == 0 || b < TOTP) && row < nrows) {
#pragma unroll
          for (int r = 0; r < RP; ++r) {
            const int n = j + r * (H / RP);
#pragma unroll
            for (int half = 0; half < 2; ++half) {
              const int ph = phase_at(row, 2 * n + half);
              fn(q, r, half, lam_s[ph], mu_s[ph]);
            }
          }
        }
      }
    };

    if (part >= 1 && part <= S - DIM) {
      // shear component: sigma_ab = 2 mu eps_ab
      const int c = DIM + part - 1;
      T e_r[BP][RP], e_i[BP][RP];
      c2r(c, e_r, e_i);
      if constexpr (MODE == M_MAT) {
        if (D.out_eps) write_real(D.out_eps, c, e_r, e_i);
      }
      each_point([&](int q, int r, int half, T lam, T mu) {
        if (half) e_i[q][r] *= T(2) * mu; else e_r[q][r] *= T(2) * mu;
      });
      if constexpr (MODE == M_MAT) {
        if (D.out_sig) write_real(D.out_sig, c, e_r, e_i);
      } else {
        forward_store(e_r, e_i, D.S, c);
      }
      return;
    }
    if constexpr (MODE == M_MAT) {
      if (part > S - DIM) {
        // displacement component, written straight out
        const int c = part - (S - DIM) - 1;
        if (D.out_u) {
          T e_r[BP][RP], e_i[BP][RP];
          c2r(S + c, e_r, e_i);
          write_real(D.out_u, c, e_r, e_i);
        }
        return;
      }
    }
    // part 0: normal components, coupled through the trace
    T n_r[DIM][BP][RP], n_i[DIM][BP][RP];
#pragma unroll
    for (int c = 0; c < DIM; ++c) c2r(c, n_r[c], n_i[c]);
    if constexpr (MODE == M_MAT) {
      if (D.out_eps) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) write_real(D.out_eps, c, n_r[c], n_i[c]);
      }
    }
    each_point([&](int q, int r, int half, T lam, T mu) {
      T ev[DIM];
#pragma unroll
      for (int c = 0; c < DIM; ++c) ev[c] = half ? n_i[c][q][r] : n_r[c][q][r];
      T tr = T(0);
#pragma unroll
      for (int c = 0; c < DIM; ++c) tr += ev[c];
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        const T sv = T(2) * mu * ev[c] + lam * tr;
        if (half) n_i[c][q][r] = sv; else n_r[c][q][r] = sv;
      }
    });
    if constexpr (MODE == M_MAT) {
      if (D.out_sig) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) write_real(D.out_sig, c, n_r[c], n_i[c]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < DIM; ++c) forward_store(n_r[c], n_i[c], D.S, c);
    }
  }
}

// ---------------------------------------------------------------------------
// x pass of the iteration with row tiles staged by direct global->LDS loads
// ---------------------------------------------------------------------------
// FP32 tiles of 2048 complex entries (nx = 64, 128, 256) or 1536 (nx = 48,
// 96: 64 or 32 rows), and with the halved tiles of schedule variant 1 the
// 768-entry tiles of nx = 48 and 96 (32 or 16 rows).  The main block of a row tile (MR rows x H entries) is
// contiguous in HBM; it lands in LDS in 1 KB pieces, one per wave-wide
// 16-byte-per-lane load.  Where rows divide a piece (2048-entry tiles) each
// piece is followed by 64 bytes of padding so that row pairs of consecutive
// pieces fall on different LDS banks; 384-byte rows straddle pieces, so
// those tiles are dense.  Loads bypass the registers, so the
// normal group fetches the next component into the second buffer while the
// current one is transformed.  The buffers double as transform staging and
// fold tiles once their data has been read.
constexpr int kXDmaPhases = kMaxPhases;
constexpr int cmax(int a, int b) { return a > b ? a : b; }
template <typename T, int H, bool ALT = false, int DIV = 1> struct XDma {
  using G = XGeom<T, H, DIV>;
  static constexpr int MR = G::MR;
  // 2048- and 1536-entry tiles; with the halved tiles of schedule variant 1,
  // the 768-entry ones of nx = 48 and 96
  static constexpr bool ok = sizeof(T) == 4 && Cfg<T>::NTH_X == 256 &&
                             (DIV == 1 ? (MR * H == 2048 || MR * H == 1536) : (DIV == 2 && MR * H == 768));
  static constexpr int KB = 1024, PAD = (KB % (H * 8) == 0) ? 64 : 0, PITCH = KB + PAD;
  static constexpr int NCH = MR * H * 8 / KB;                 // 1 KB pieces per tile
  // fold-tile pitch for the unfold: the forward core leaves NB = H / RL
  // consecutive entries of a row in consecutive lanes, so a pitch of NB
  // (mod 32) puts the rows of a wave on disjoint LDS banks
  static constexpr int NB = H / PlanSeq<PlanPick<ALT>::template P, H, false>::last();
  static constexpr int SMF = (H + 1 + ((NB - (H + 1) % 32) % 32 + 32) % 32);
  // transform staging pitch and skew
#ifndef LSFFT_XSTG
#define LSFFT_XSTG 1
#endif
  // The alternate radix order at 128 points (schedule variant 2, the tuned
  // choice at nx = 256) XOR-swizzles the staging index (TileFft SWZ 1) with a
  // pencil pitch of 160 words: a multiple of 32, and rows two apart fall 32
  // words apart, so a wave's two rows of a radix-4 pass also meet different
  // banks where the LDS has 64 of them.  (The default order takes 88 bytes
  // per lane of spills with it.)
  static constexpr bool SWZ = (H == 128) && ALT;
  static constexpr int SMS = (H == 128) ? 160 : (LSFFT_XSTG && H == 64) ? 71 : G::SM2;
  static constexpr bool SKS = !SWZ && !(LSFFT_XSTG && H == 64);
  static constexpr int BUF = (cmax(cmax(NCH * PITCH, 2 * MR * SMS * 4), 2 * MR * SMF * 4) + 15) / 16 * 16;
  // phase ids of the tile: rows of 2H bytes at a pitch of 16 words modulo
  // 32, so two consecutive rows fall on disjoint halves of the LDS banks
  static constexpr int PP = 2 * H + 4 * (((16 - H / 2) % 32 + 32) % 32);
  static_assert(!ok || (PP % 16 == 0 && (PP / 4) % 32 == 16), "phase-id row pitch");
  // per-pass twiddle tables of the inverse (reversed plan) and forward cores
  using PF = PlanPick<ALT>;
  static constexpr int TWPL = twp_len<PF::template P, H, true>() + twp_len<PF::template P, H, false>();
  // dynamic LDS: twiddles (2 x 2H), Lame table, per-pass twiddles (padded to
  // 16 bytes), phase ids of the tile
  static constexpr int TWPB = (8 * TWPL + 15) / 16 * 16;
  static constexpr int DYN = 4 * (2 * 2 * H + 2 * kXDmaPhases) + TWPB + MR * PP;
  static_assert(!ok || (MR * 2 * H == 4096 || MR * 2 * H == 3072 || MR * 2 * H == 1536), "x tile geometry");
  // padded tiles: rows never straddle a piece (a row is 256, 512 or 1024
  // bytes); dense tiles: PAD = 0
  __device__ static __forceinline__ int row_off(int m) {
    const int p = m * H * 8;
    return p + (p >> 10) * PAD;
  }
};

typedef __attribute__((address_space(3))) void* lds_vptr;

// Issue the loads of component `comp` (global base of the component) of row
// tile row0 into LDS buffer `buf`.  Lanes past the last row load nothing.
// Every supported axis length is even, so the component stride (ny nz H
// entries of 8 bytes) keeps every component base 16-byte aligned.
template <typename X, int H>
__device__ __forceinline__ void xdma_issue(const char* comp, int row0, int nrows, unsigned char* buf, int tid) {
  const int wave = tid >> 6, lane = tid & 63;
  const char* mainp = comp + (long long)row0 * H * 8;
  // piece g by wave g mod 4 (768-entry tiles: 6 pieces, two waves take two)
#pragma unroll
  for (int i = 0; i < (X::NCH + 3) / 4; ++i) {
    const int g = i * 4 + wave;
    if (X::NCH % 4 != 0 && g >= X::NCH) break;
    const int b = g * X::KB + lane * 16;
    if (row0 + b / (H * 8) < nrows)
      __builtin_amdgcn_global_load_lds((const void*)(mainp + b), (lds_vptr)(buf + g * X::PITCH), 16, 0, 0);
  }
}

__device__ __forceinline__ void wait_vm_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <typename T, int NX, int DIM, int V>
__device__ void xpass_iter_dma(const InstDesc& D, int local, const double* __restrict__ lame,
                               const T* __restrict__ twtab, unsigned char* smem) {
  constexpr int NTH = 256;
  constexpr int H = NX / 2;
  using G = XGeom<T, H, XSched<V>::EX_DIV>;
  using X = XDma<T, H, XSched<V>::ALT, XSched<V>::EX_DIV>;
  constexpr int MR = G::MR, SM = X::SMF, SM2 = X::SMS;
  constexpr int S = (DIM == 3) ? 6 : 3;
  using PF = PlanPick<XSched<V>::ALT>;
  using FI = TileFft<T, H, +1, true, MR, SM2, 1, 2, true, NTH, PF::template P, X::SKS, true, X::SWZ ? 1 : 0, true>;
  using FF = TileFft<T, H, -1, false, MR, SM2, 1, 2, true, NTH, PF::template P, X::SKS, true, X::SWZ ? 1 : 0, true>;
  static_assert(FI::RL == FF::R0 && FI::BL == FF::B0, "x transforms must chain in registers");
  static_assert(X::NB == H / FF::RL && SM % 32 == X::NB % 32 && SM > H, "fold-tile pitch");
  static_assert(FI::TWPL + FF::TWPL == X::TWPL, "per-pass twiddle tables");
  constexpr int BP = FI::BL, RP = FI::RL;
  constexpr int TOTP = FI::TOTL;
  constexpr int PB = MR * NX / NTH;                // phase bytes per thread

  __shared__ __align__(16) unsigned char xb0[X::BUF];
  __shared__ __align__(16) unsigned char xb1[X::BUF];
  T* twr = reinterpret_cast<T*>(smem);
  T* twi = twr + NX;
  T* lam_s = twi + NX;
  T* mu_s = lam_s + kXDmaPhases;
  T* fir = mu_s + kXDmaPhases;          // per-pass twiddles, inverse core
  T* fii = fir + FI::TWPL;
  T* ffr = fii + FI::TWPL;              // forward core
  T* ffi = ffr + FF::TWPL;
  unsigned char* ptile = reinterpret_cast<unsigned char*>(mu_s + kXDmaPhases) + X::TWPB;
  const int tid = threadIdx.x;
  const int nrows = D.ny * D.nz;
  const int part = local / D.xtiles;
  const int row0 = (local - part * D.xtiles) * MR;
  const long long Pc = D.Pc;
  const int cfirst = (part == 0) ? 0 : DIM + part - 1;

  xdma_issue<X, H>(cptr<T>(D.S, Pc, cfirst), row0, nrows, xb0, tid);
  // phase ids of the tile, PB = 16 (2048-entry tiles), 12 (1536) or 6
  // (768) consecutive x of one row per thread, read at the shifted
  // positions: as one 16-byte load, three 4-byte or three 2-byte loads where
  // the shift keeps the group whole and aligned, byte by byte otherwise
  static_assert(PB == 16 || PB == 12 || PB == 6, "x tile phase map");
  constexpr int PW = PB / 4;
  unsigned phw[4] = {0u, 0u, 0u, 0u};
  {
    const int m = (tid * PB) / NX, x0 = (tid * PB) - m * NX;
    const int row = row0 + m;
    if (row < nrows) {
      const int z = row / D.ny, y = row - (row / D.ny) * D.ny;
      const long long rbase = (long long)(wrap(z - D.sz, D.nz) * D.ny + wrap(y - D.sy, D.ny)) * NX;
      const unsigned long long pa = reinterpret_cast<unsigned long long>(D.phase);
      if (PB == 16 && ((pa | (unsigned)D.sx) & 15ull) == 0) {
        const uint4 v = gld<uint4>(D.phase + rbase + wrap(x0 - D.sx, NX), 0);
        phw[0] = v.x; phw[1] = v.y; phw[2] = v.z; phw[3] = v.w;
      } else if (PB == 12 && (pa & 3ull) == 0 && D.sx % 12 == 0) {
        const uint8_t* g = D.phase + rbase + wrap(x0 - D.sx, NX);
#pragma unroll
        for (int i = 0; i < PW; ++i) phw[i] = gld<unsigned>(g, i);
      } else if (PB == 6 && (pa & 1ull) == 0 && D.sx % 6 == 0) {
        const uint8_t* g = D.phase + rbase + wrap(x0 - D.sx, NX);
#pragma unroll
        for (int i = 0; i < 3; ++i) phw[i >> 1] |= (unsigned)gld<unsigned short>(g, i) << (16 * (i & 1));
      } else {
#pragma unroll
        for (int i = 0; i < PB; ++i)
          phw[i >> 2] |= (unsigned)gld<uint8_t>(D.phase, rbase + wrap(x0 + i - D.sx, NX)) << (8 * (i & 3));
      }
    }
  }
  load_tw<T, NX, NTH>(twr, twi, twtab, tid);
  for (int p = tid; p < D.nphase; p += NTH) {
    lam_s[p] = T(gld<double>(lame, 2 * (D.lame_off + p)));
    mu_s[p] = T(gld<double>(lame, 2 * (D.lame_off + p) + 1));
  }
  {
    const int m = (tid * PB) / NX, x0 = (tid * PB) - m * NX;
    if constexpr (PB == 16) {
      *reinterpret_cast<uint4*>(ptile + m * X::PP + x0) = make_uint4(phw[0], phw[1], phw[2], phw[3]);
    } else if constexpr (PB == 12) {
#pragma unroll
      for (int i = 0; i < PW; ++i) reinterpret_cast<unsigned*>(ptile + m * X::PP + x0)[i] = phw[i];
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i)
        reinterpret_cast<unsigned short*>(ptile + m * X::PP + x0)[i] = (unsigned short)(phw[i >> 1] >> (16 * (i & 1)));
    }
  }
  lds_barrier();   // the length-NX twiddles are in LDS
  FI::twp_fill(fir, fii, twr, twi, tid);
  FF::twp_fill(ffr, ffi, twr, twi, tid);
  wait_vm_all();
  __syncthreads();

  // fold of the tile in `buf` and the length-H inverse core; the buffer then
  // serves as the core's staging
  auto c2r = [&](unsigned char* buf, T (&o_r)[BP][RP], T (&o_i)[BP][RP]) {
    T in_r[FI::B0][FI::R0], in_i[FI::B0][FI::R0];
#pragma unroll
    for (int q = 0; q < FI::B0; ++q) {
      const int b = tid + q * NTH;
      int m, j;
      FI::template bj<FI::R0>(b, m, j);
      if (FI::TOT0 % NTH != 0 && b >= FI::TOT0) m = 0;
      const unsigned char* rowp = buf + X::row_off(m);
#pragma unroll
      for (int r = 0; r < FI::R0; ++r) {
        const int k = j + r * (H / FI::R0);
        const float2 xv = *reinterpret_cast<const float2*>(rowp + 8 * k);
        // at k = 0 this read lands in the next row or the piece's padding
        // (inside the buffer) and is replaced below
        const float2 yv = *reinterpret_cast<const float2*>(rowp + 8 * (H - k));
        T xr = xv.x, xi = xv.y, yr = yv.x, yi = -yv.y;
        if (r == 0 && j == 0) {
          // packed entry Z: X[0] = (Re Z, 0), conj X[H] = (Im Z, 0)
          yr = xi;
          yi = T(0);
          xi = T(0);
        }
        const T dr = xr - yr, di = xi - yi;
        const T cr = twr[k], ci = -twi[k];
        const T tr = cr * dr - ci * di, ti = cr * di + ci * dr;
        in_r[q][r] = xr + yr - ti;
        in_i[q][r] = xi + yi + tr;
      }
    }
    lds_barrier();   // every wave has read the tile
    T* br = reinterpret_cast<T*>(buf);
    FI::run(in_r, in_i, o_r, o_i, br, br + MR * SM2, fir, fii, tid);
  };
  // forward core and unfold (staging in xb1, fold tile in xb0), then the
  // stores of component c of S
  auto forward_store = [&](T (&in_r)[FF::B0][FF::R0], T (&in_i)[FF::B0][FF::R0], int c) {
    T* br = reinterpret_cast<T*>(xb1);
    T* bi = br + MR * SM2;
    T* ar = reinterpret_cast<T*>(xb0);
    T* ai = ar + MR * SM;
    T o_r[FF::BL][FF::RL], o_i[FF::BL][FF::RL];
    lds_barrier();   // staging buffer free
    FF::run(in_r, in_i, o_r, o_i, br, bi, ffr, ffi, tid);
    lds_barrier();   // previous users of the fold tile are done
#pragma unroll
    for (int q = 0; q < FF::BL; ++q) {
      const int b = tid + q * NTH;
      if (FF::TOTL % NTH == 0 || b < FF::TOTL) {
        int m, j;
        FF::template bj<FF::RL>(b, m, j);
#pragma unroll
        for (int r = 0; r < FF::RL; ++r) {
          const int n = j + r * (H / FF::RL);
          ar[m * SM + n] = o_r[q][r];
          ai[m * SM + n] = o_i[q][r];
        }
      }
    }
    lds_barrier();
    char* base = mptr<T>(D.S, Pc, c);
#pragma unroll 1
    for (int u = 0; u < MR * H / NTH; ++u) {
      const int e = tid + u * NTH;
      const int m = e / H;
      const int k = e - m * H;
      const int row = row0 + m;
      if (row >= nrows) continue;
      const T zr = ar[m * SM + k], zi = ai[m * SM + k];
      if (k == 0) {
        // X[0] = zr + zi and X[H] = zr - zi are real: one packed entry
        stc<T>(base, row * H, zr + zi, zr - zi);
        continue;
      }
      const T wr = ar[m * SM + H - k], wi = ai[m * SM + H - k];
      const T er = T(0.5) * (zr + wr), ei = T(0.5) * (zi - wi);
      const T dr = T(0.5) * (zr - wr), di = T(0.5) * (zi + wi);
      const T orr = di, oi = -dr;
      const T cr = twr[k], ci = twi[k];
      const T xr = er + cr * orr - ci * oi, xi = ei + cr * oi + ci * orr;
      stc<T>(base, row * H + k, xr, xi);
    }
  };
  // fn(q, r, half, lam, mu) at every point of this thread
  auto each_point = [&](auto&& fn) {
#pragma unroll
    for (int q = 0; q < BP; ++q) {
      const int b = tid + q * NTH;
      int m, j;
      FI::template bj<RP>(b, m, j);
      if ((TOTP % NTH == 0 || b < TOTP) && row0 + m < nrows) {
#pragma unroll
        for (int r = 0; r < RP; ++r) {
          const int n = j + r * (H / RP);
          const unsigned pp = *reinterpret_cast<const unsigned short*>(ptile + m * X::PP + 2 * n);
#pragma unroll
          for (int half = 0; half < 2; ++half) {
            const int ph = half ? (int)(pp >> 8) : (int)(pp & 0xffu);
            fn(q, r, half, lam_s[ph], mu_s[ph]);
          }
        }
      }
    }
  };

  if (part >= 1) {
    // shear component: sigma_ab = 2 mu eps_ab
    T e_r[BP][RP], e_i[BP][RP];
    c2r(xb0, e_r, e_i);
    each_point([&](int q, int r, int half, T lam, T mu) {
      if (half) e_i[q][r] *= T(2) * mu; else e_r[q][r] *= T(2) * mu;
    });
    forward_store(e_r, e_i, cfirst);
    return;
  }
  // normal components, coupled through the trace; component c + 1 is in
  // flight while component c is transformed
  T n_r[DIM][BP][RP], n_i[DIM][BP][RP];
  xdma_issue<X, H>(cptr<T>(D.S, Pc, 1), row0, nrows, xb1, tid);
  c2r(xb0, n_r[0], n_i[0]);
  wait_vm_all();
  __syncthreads();   // component 1 landed; the staging of component 0 is free
  if constexpr (DIM == 3) xdma_issue<X, H>(cptr<T>(D.S, Pc, 2), row0, nrows, xb0, tid);
  c2r(xb1, n_r[1], n_i[1]);
  if constexpr (DIM == 3) {
    wait_vm_all();
    __syncthreads();
    c2r(xb0, n_r[2], n_i[2]);
  }
  each_point([&](int q, int r, int half, T lam, T mu) {
    T ev[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) ev[c] = half ? n_i[c][q][r] : n_r[c][q][r];
    T tr = T(0);
#pragma unroll
    for (int c = 0; c < DIM; ++c) tr += ev[c];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const T sv = T(2) * mu * ev[c] + lam * tr;
      if (half) n_i[c][q][r] = sv; else n_r[c][q][r] = sv;
    }
  });
#pragma unroll
  for (int c = 0; c < DIM; ++c) forward_store(n_r[c], n_i[c], c);
  (void)S;
}

template <typename T, int NX, int DIM, int MODE, int V>
__device__ __forceinline__ void xpass_item(const InstDesc& D, int local, const double* __restrict__ lame,
                                           const T* __restrict__ twtab, unsigned char* smem) {
#ifndef LSFFT_NO_XDMA
  if constexpr (MODE == M_ITER && XDma<T, NX / 2, XSched<V>::ALT, XSched<V>::EX_DIV>::ok) {
    xpass_iter_dma<T, NX, DIM, V>(D, local, lame, twtab, smem);
    return;
  }
#endif
  xpass_item_std<T, NX, DIM, MODE, V>(D, local, lame, twtab, smem);
}

// ---------------------------------------------------------------------------
// strided tiles (y pass and outer pass)
// ---------------------------------------------------------------------------
// A tile is MP pencils of length N: mpk consecutive kx columns times MP / mpk
// consecutive lines of the other axis.  Element (m, n) of component c lives
// at c Pc + off(m) + n sn.
// Index of spectrum entry (kx, ky, kz) in the layout of D (rows of H
// entries, or 8-wide kx blocks), and the inverse.
__device__ __forceinline__ long long spec_at(const InstDesc& D, int kx, int ky, int kz) {
  if (D.blk) return ((long long)(kx >> 3) * D.ny + ky) * D.bls + kz * 8 + (kx & 7);
  return ((long long)kz * D.ny + ky) * D.H + kx;
}
__device__ __forceinline__ void spec_coords(const InstDesc& D, long long g, int& kx, int& ky, int& kz) {
  if (D.blk) {
    const long long line = g / D.bls, w = g - line * D.bls;
    const long long b = line / D.ny;
    kx = int(b * 8 + (w & 7));
    ky = int(line - b * D.ny);
    kz = int(w >> 3);
  } else {
    kx = int(g % D.H);
    const long long rest = g / D.H;
    ky = int(rest % D.ny);
    kz = int(rest / D.ny);
  }
}

struct TileAddr {
  int sn;              // stride along the pencil (elements)
  int base;            // offset of pencil 0 within a component
  int so;              // stride between lines of the other axis
  int mpk, lg;         // kx pencils per line (power of 2), log2
  int kx0, o0, nother; // first kx, first line, lines in the grid
  int bs = 0;          // kx-blocked layout: stride of 8-wide kx blocks (0: rows)
  __device__ __forceinline__ int off(int m) const {
    if (bs == 0) return base + (m >> lg) * so + (m & (mpk - 1));
    const int k = kx0 + (m & (mpk - 1));
    return base + (k >> 3) * bs + (o0 + (m >> lg)) * so + (k & 7);
  }
  __device__ __forceinline__ bool valid(int m) const { return o0 + (m >> lg) < nother; }
  __device__ __forceinline__ int kx(int m) const { return kx0 + (m & (mpk - 1)); }
  __device__ __forceinline__ int other(int m) const { return o0 + (m >> lg); }
};

// y pass (3D): pencils along y; other axis = z.
__device__ __forceinline__ TileAddr ytile(const InstDesc& D, int local, int MP, bool zfast = false) {
  TileAddr t;
  const int per = MP >> D.lg_y;                    // z lines per tile
  int tz, tk;
  if (zfast) {
    const int nzt = (D.nz + per - 1) / per;
    tk = local / nzt;
    tz = local - tk * nzt;
  } else {
    tz = local / D.ntk_y;
    tk = local - tz * D.ntk_y;
  }
  t.mpk = D.mpk_y;
  t.lg = D.lg_y;
  t.kx0 = tk * D.mpk_y;
  t.o0 = tz * per;
  t.nother = D.nz;
  t.sn = D.H;
  t.so = D.ny * D.H;
  t.base = t.o0 * t.so + t.kx0;
  return t;
}
// the same y tile in the kx-blocked layout: pencil stride bls, z lines 8 apart
__device__ __forceinline__ TileAddr ytile_blk(const InstDesc& D, int local, int MP, bool zfast = false) {
  TileAddr t = ytile(D, local, MP, zfast);
  t.sn = D.bls;
  t.so = 8;
  t.bs = D.ny * D.bls;
  t.base = 0;
  return t;
}

// outer pass: pencils along z (3D, other axis y) or y (2D, no other axis)
template <int DIM>
__device__ __forceinline__ TileAddr gtile(const InstDesc& D, int local, int MP) {
  TileAddr t;
  t.mpk = D.mpk_g;
  t.lg = D.lg_g;
  if constexpr (DIM == 3) {
    const int per = MP >> D.lg_g;
    if (D.blk) {
      // kx-blocked: consecutive tiles cover consecutive y lines of one kx
      // block (each line an 8 x nz block of the layout; tiles narrower than
      // 8 kx take the parts of a line in turn)
      const int nty = (D.ny + per - 1) / per;
      const int sb = D.mpk_g < 8 ? 8 / D.mpk_g : 1;
      const int wk = D.mpk_g < 8 ? 8 : D.mpk_g;
      const int kg = local / (nty * sb), rem = local - kg * (nty * sb);
      const int ty = rem / sb, sub = rem - ty * sb;
      t.kx0 = kg * wk + sub * D.mpk_g;
      t.o0 = ty * per;
      t.nother = D.ny;
      t.sn = 8;
      t.so = D.bls;
      t.bs = D.ny * D.bls;
      t.base = 0;
    } else {
      const int ty = local / D.ntk_g, tk = local - (local / D.ntk_g) * D.ntk_g;
      t.kx0 = tk * D.mpk_g;
      t.o0 = ty * per;
      t.nother = D.ny;
      t.sn = D.ny * D.H;
      t.so = D.H;
      t.base = t.o0 * D.H + t.kx0;
    }
  } else {
    t.kx0 = local * D.mpk_g;
    t.o0 = 0;
    t.nother = 1;                                 // only m < mpk are valid
    t.sn = D.H;
    t.so = D.H;
    t.base = t.kx0;
  }
  return t;
}

template <typename T, int NY, int DIR, int V>
__device__ void ypass_item(const InstDesc& D, int local, int c, const void* src, void* dst,
                           const T* __restrict__ twtab, unsigned char* smem) {
  constexpr int NTH = Cfg<T>::NTH;
  constexpr int MP = YSched<T, NY, V>::MP;
  using PR = PencilRows<T, NY, MP>;
  constexpr int LP = PR::LP;                    // LDS row (one index, all pencils)
  constexpr int E = PR::E;
  using F = TileFft<T, NY, DIR, (DIR > 0), MP, 1, LP, 1, false, NTH, PlanPick<YSched<T, NY, V>::ALT>::template P,
                    false, false, PR::SWZ>;
  static_assert((MP - 1) + (F::ROWS - 1) * LP < E, "y tile staging");
  T* re = reinterpret_cast<T*>(smem);
  T* im = re + E;
  T* twr = im + E;
  T* twi = twr + NY;
  const int tid = threadIdx.x;
  load_tw<T, NY, NTH>(twr, twi, twtab, tid);
  __syncthreads();
  // kx-blocked spectra: the forward transforms leave the row layout for the
  // blocked one, the inverse transforms come back (out of place)
  // The forward pass writes the blocked layout, whose y lines lie 8 nz
  // entries apart.  Where its tiles read runs of at least 128 bytes per row,
  // consecutive tiles take consecutive z lines of one kx group, so that the
  // tiles running together fill those lines and the long stride falls on the
  // row reads instead (strided stores cost more than strided loads here:
  // 207 against 172 us per 256^3 launch in the other order, about 20 us less
  // in this one with 16-kx tiles; with 8-kx tiles, 64-byte row runs, this
  // order took 310 against 208 us).
  const bool zf = D.blk && DIR < 0 && D.mpk_y * 2 * (int)sizeof(T) >= 128;
  const TileAddr t = (D.blk && DIR > 0) ? ytile_blk(D, local, MP) : ytile(D, local, MP, zf);
  const TileAddr td = (D.blk && DIR < 0) ? ytile_blk(D, local, MP, zf) : ytile(D, local, MP);
  const char* cb = cptr<T>(src, D.Pc, c);
  char* db = mptr<T>(dst, D.Pc, c);
  T in_r[F::B0][F::R0], in_i[F::B0][F::R0];
#pragma unroll
  for (int q = 0; q < F::B0; ++q) {
    const int b = tid + q * NTH;
    int m, j;
    F::template bj<F::R0>(b, m, j);
    const bool ok = (F::TOT0 % NTH == 0 || b < F::TOT0) && t.valid(m);
    const int o = t.off(m);
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      T re_ = T(0), im_ = T(0);
      if (ok) {
        const typename C2<T>::type v = ldc<T>(cb, o + (j + r * (NY / F::R0)) * t.sn);
        re_ = v.x;
        im_ = v.y;
      }
      in_r[q][r] = re_;
      in_i[q][r] = im_;
    }
  }
  T o_r[F::BL][F::RL], o_i[F::BL][F::RL];
  F::run(in_r, in_i, o_r, o_i, re, im, twr, twi, tid);
#pragma unroll
  for (int q = 0; q < F::BL; ++q) {
    const int b = tid + q * NTH;
    int m, j;
    F::template bj<F::RL>(b, m, j);
    if ((F::TOTL % NTH == 0 || b < F::TOTL) && td.valid(m)) {
      const int o = td.off(m);
      if (D.blk) {
#pragma unroll
        for (int r = 0; r < F::RL; ++r)
          stc_nt<T>(db, o + (j + r * (NY / F::RL)) * td.sn, o_r[q][r], o_i[q][r]);
      } else {
#pragma unroll
        for (int r = 0; r < F::RL; ++r)
          stc<T>(db, o + (j + r * (NY / F::RL)) * td.sn, o_r[q][r], o_i[q][r]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Green / body-force pass along the outermost axis
// ---------------------------------------------------------------------------
template <typename T, int NG, int DIM, int MODE, int V>
__device__ void green_item(const InstDesc& D, InstState* __restrict__ St, int local,
                           const T* __restrict__ twtab, unsigned char* smem) {
  using GS = GSched<T, NG, V>;
  constexpr int NTH = GS::NTH;
  constexpr int MP = GS::MP;
  using PR = PencilRows<T, NG, MP>;
  constexpr int LP = PR::LP;                    // LDS row
  constexpr int E = PR::E;
  constexpr int S = (DIM == 3) ? 6 : 3;
  using FF = TileFft<T, NG, -1, false, MP, 1, LP, 1, false, NTH, PlanG, false, false, PR::SWZ>;
  using FI = TileFft<T, NG, +1, true, MP, 1, LP, 1, false, NTH, PlanG, false, false, PR::SWZ>;
  static_assert((MP - 1) + (FF::ROWS - 1) * LP < E, "outer tile staging");
  static_assert(FF::RL == FI::R0 && FF::BL == FI::B0, "outer transforms must chain in registers");
  constexpr int BP = FF::BL, RP = FF::RL, TOTP = FF::TOTL;
  constexpr int NSTEP = NG / RP;                 // index step between a butterfly's points

  T* lre[2];
  T* lim[2];
  lre[0] = reinterpret_cast<T*>(smem);
  lim[0] = lre[0] + E;
  lre[1] = lim[0] + E;
  lim[1] = lre[1] + E;
  T* twr = lim[1] + E;
  T* twi = twr + NG;
  double* red = reinterpret_cast<double*>(twi + NG + (NG & 1));
  const int tid = threadIdx.x;
  load_tw<T, NG, NTH>(twr, twi, twtab, tid);
  __syncthreads();

  const TileAddr t = gtile<DIM>(D, local, MP);
  const long long Pc = D.Pc;
  // spectra between the y passes and this one: kx-blocked copies, or in place
  void* const SS = D.blk ? D.S2 : D.S;
  const T inv_n = T(D.inv_nvox);
  const T mu0 = T(D.mu0);
  const T c0 = T((D.lam0 + D.mu0) / (D.lam0 + 2.0 * D.mu0));

  // per last-pass butterfly q of this thread: pencil m, first index j
  bool pv[BP];
  int poff[BP];
  int pj[BP];
  T pxi0[BP], pxi1[BP];   // xi_x, and xi_y in 3D
  T pw[BP];               // Parseval weight
#pragma unroll
  for (int q = 0; q < BP; ++q) {
    const int b = tid + q * NTH;
    int m, j;
    FF::template bj<RP>(b, m, j);
    pv[q] = (TOTP % NTH == 0 || b < TOTP) && t.valid(m);
    poff[q] = t.off(m);
    pj[q] = j;
    const int kx = t.kx(m);
    pxi0[q] = T(wavenum(kx, D.nx, D.kx));
    pxi1[q] = (DIM == 3) ? T(wavenum(t.other(m) < D.ny ? t.other(m) : 0, D.ny, D.ky)) : T(0);
    pw[q] = (kx == 0) ? T(1) : T(2);   // kx = 0 column: the packed kx = 0 and kx = H planes
  }
  auto point_xi = [&](int q, int r, T* xi, T& xi2) {
    const int n = pj[q] + r * NSTEP;
    xi[0] = pxi0[q];
    if constexpr (DIM == 3) {
      xi[1] = pxi1[q];
      xi[2] = T(wavenum(n, D.nz, D.kz));
    } else {
      xi[1] = T(wavenum(n, D.ny, D.ky));
    }
    xi2 = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) xi2 += xi[a] * xi[a];
  };
  auto gidx = [&](int q, int r) -> int { return poff[q] + (pj[q] + r * NSTEP) * t.sn; };

  // first-pass loads of component c of src into (in_r, in_i)
  auto load_first = [&](const void* src, int c, T (&in_r)[FF::B0][FF::R0], T (&in_i)[FF::B0][FF::R0]) {
    const char* cb = cptr<T>(src, Pc, c);
#pragma unroll
    for (int q = 0; q < FF::B0; ++q) {
      const int b = tid + q * NTH;
      int m, j;
      FF::template bj<FF::R0>(b, m, j);
      const bool ok = (FF::TOT0 % NTH == 0 || b < FF::TOT0) && t.valid(m);
      const int o = t.off(m);
#pragma unroll
      for (int r = 0; r < FF::R0; ++r) {
        T re_ = T(0), im_ = T(0);
        if (ok) {
          const typename C2<T>::type v = ldc<T>(cb, o + (j + r * (NG / FF::R0)) * t.sn);
          re_ = v.x;
          im_ = v.y;
        }
        in_r[q][r] = re_;
        in_i[q][r] = im_;
      }
    }
  };

  // forward transforms of NC components of src; fn(c, q, r, re, im) per point
  int buf = 0;
  auto forward_all = [&](const void* src, auto nc_tag, auto&& fn) {
    constexpr int NC = decltype(nc_tag)::value;
    T cur_r[FF::B0][FF::R0], cur_i[FF::B0][FF::R0];
    load_first(src, 0, cur_r, cur_i);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      // the next component's loads are issued before this one's transform
      T nxt_r[FF::B0][FF::R0], nxt_i[FF::B0][FF::R0];
      if (c + 1 < NC) load_first(src, c + 1, nxt_r, nxt_i);
      T o_r[BP][RP], o_i[BP][RP];
      FF::run(cur_r, cur_i, o_r, o_i, lre[buf], lim[buf], twr, twi, tid);
      buf ^= 1;
#pragma unroll
      for (int q = 0; q < BP; ++q)
#pragma unroll
        for (int r = 0; r < RP; ++r) fn(c, q, r, o_r[q][r], o_i[q][r]);
      LSFFT_FENCE();
      if (c + 1 < NC) {
#pragma unroll
        for (int q = 0; q < FF::B0; ++q)
#pragma unroll
          for (int r = 0; r < FF::R0; ++r) { cur_r[q][r] = nxt_r[q][r]; cur_i[q][r] = nxt_i[q][r]; }
      }
    }
  };

  // inverse transforms of NC components produced per point by gen(c, q, r, re&, im&),
  // stored to dst (component offset c0_ in the destination)
  auto inverse_all = [&](void* dst, int cfirst, auto nc_tag, auto&& gen) {
    constexpr int NC = decltype(nc_tag)::value;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T in_r[FI::B0][FI::R0], in_i[FI::B0][FI::R0];
#pragma unroll
      for (int q = 0; q < BP; ++q)
#pragma unroll
        for (int r = 0; r < RP; ++r) gen(c, q, r, in_r[q][r], in_i[q][r]);
      T o_r[FI::BL][FI::RL], o_i[FI::BL][FI::RL];
      FI::run(in_r, in_i, o_r, o_i, lre[buf], lim[buf], twr, twi, tid);
      buf ^= 1;
      char* cb = mptr<T>(dst, Pc, cfirst + c);
      LSFFT_FENCE();
#pragma unroll
      for (int q = 0; q < FI::BL; ++q) {
        const int b = tid + q * NTH;
        int m, j;
        FI::template bj<FI::RL>(b, m, j);
        if ((FI::TOTL % NTH == 0 || b < FI::TOTL) && t.valid(m)) {
          const int o = t.off(m);
          if (D.blk) {
#pragma unroll
            for (int r = 0; r < FI::RL; ++r)
              stc_nt<T>(cb, o + (j + r * (NG / FI::RL)) * t.sn, o_r[q][r], o_i[q][r]);
          } else {
#pragma unroll
            for (int r = 0; r < FI::RL; ++r)
              stc<T>(cb, o + (j + r * (NG / FI::RL)) * t.sn, o_r[q][r], o_i[q][r]);
          }
        }
      }
    }
  };

  // displacement-like vector per point (residual, then state)
  T vr[DIM][BP][RP], vi[DIM][BP][RP];

  // strain spectrum / |N| from the vector held in vr/vi:
  // eps^_ab = (i/2)(xi_a u^_b + xi_b u^_a)
  auto strain_gen = [&](int c, int q, int r, T& re, T& im) {
    T xi[DIM], xi2;
    point_xi(q, r, xi, xi2);
    const int a = va<DIM>(c), b = vb<DIM>(c);
    const T sr = T(0.5) * (xi[a] * vr[b][q][r] + xi[b] * vr[a][q][r]);
    const T si = T(0.5) * (xi[a] * vi[b][q][r] + xi[b] * vi[a][q][r]);
    re = -si * inv_n;
    im = sr * inv_n;
  };
  // accumulate sgn * i xi . sigma^ component c into vr/vi
  auto div_acc = [&](int c, int q, int r, T re, T im, T sgn) {
    T xi[DIM], xi2;
    point_xi(q, r, xi, xi2);
    const int a = va<DIM>(c), b = vb<DIM>(c);
    // i xi_b s -> (-xi_b im, xi_b re)
    vr[a][q][r] -= sgn * xi[b] * im;
    vi[a][q][r] += sgn * xi[b] * re;
    if (a != b) {
      vr[b][q][r] -= sgn * xi[a] * im;
      vi[b][q][r] += sgn * xi[a] * re;
    }
  };
  auto zero_v = [&]() {
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int q = 0; q < BP; ++q)
#pragma unroll
        for (int r = 0; r < RP; ++r) { vr[a][q][r] = T(0); vi[a][q][r] = T(0); }
  };

  double part = 0.0, part2 = 0.0;
  const int cur = St->iter & 1;

  if constexpr (MODE == M_FT) {
    // finish the force transform, record the removed mean, project off Z
    forward_all(D.blk ? D.S2 : D.F, std::integral_constant<int, DIM>{}, [&](int c, int q, int r, T re, T im) {
      vr[c][q][r] = re;
      vi[c][q][r] = im;
    });
#pragma unroll
    for (int q = 0; q < BP; ++q) {
      if (!pv[q]) continue;
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        T xi[DIM], xi2;
        point_xi(q, r, xi, xi2);
        const int g = gidx(q, r);
        const bool origin = (g == 0);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          if (origin) St->removed_mean[c] = double(vr[c][q][r]) * D.inv_nvox;
          if (xi2 == T(0)) { vr[c][q][r] = T(0); vi[c][q][r] = T(0); }
          stc<T>(mptr<T>(D.F, Pc, c), g, vr[c][q][r], vi[c][q][r]);
        }
      }
    }
    return;
  } else if constexpr (MODE == M_INIT || MODE == M_ITER || MODE == M_CG_INIT) {
    zero_v();
    if constexpr (MODE != M_INIT) {
      forward_all(SS, std::integral_constant<int, S>{},
                  [&](int c, int q, int r, T re, T im) { div_acc(c, q, r, re, im, T(1)); });
    }
#pragma unroll
    for (int q = 0; q < BP; ++q) {
      if (!pv[q]) {
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int r = 0; r < RP; ++r) { vr[a][q][r] = T(0); vi[a][q][r] = T(0); }
        continue;
      }
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        T xi[DIM], xi2;
        point_xi(q, r, xi, xi2);
        const int g = gidx(q, r);
        // the force and (basic iteration, FP32) the current state of this
        // point, loaded together: the stores below may alias these buffers
        // as far as the compiler knows, so a load placed after a store would
        // wait for its own round trip.  FP64 tiles have no registers to spare
        // for it and load the state at its use.
        constexpr bool early_u = (MODE == M_ITER) && std::is_same<T, float>::value;
        typename C2<T>::type fv[DIM], u0v[early_u ? DIM : 1];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          fv[a] = ldc<T>(cptr<T>(D.F, Pc, a), g);
          if constexpr (early_u) u0v[a] = ldc<T>(cptr<T>(D.U[cur], Pc, a), g);
        }
        T ur[DIM], ui[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          vr[a][q][r] += fv[a].x;
          vi[a][q][r] += fv[a].y;
          part += double(pw[q]) * (double(vr[a][q][r]) * double(vr[a][q][r]) +
                                   double(vi[a][q][r]) * double(vi[a][q][r]));
          ur[a] = vr[a][q][r];
          ui[a] = vi[a][q][r];
        }
        // N0 r (the plain CG of Algorithm 3 keeps z = r; r vanishes where xi = 0)
        if (MODE != M_CG_INIT || D.precond) apply_n0<T, DIM>(xi, xi2, c0, mu0, ur, ui);
        if constexpr (!early_u) LSFFT_FENCE();
        if constexpr (MODE == M_CG_INIT) {
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            stc<T>(mptr<T>(D.R, Pc, a), g, vr[a][q][r], vi[a][q][r]);
            stc<T>(mptr<T>(D.Pd, Pc, a), g, ur[a], ui[a]);
            part2 += double(pw[q]) * (double(vr[a][q][r]) * double(ur[a]) + double(vi[a][q][r]) * double(ui[a]));
            vr[a][q][r] = ur[a];
            vi[a][q][r] = ui[a];
          }
        } else {
          void* uout = (MODE == M_INIT) ? D.U[0] : D.U[cur ^ 1];
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            T nr = ur[a], ni = ui[a];
            if constexpr (early_u) {
              nr += u0v[a].x;
              ni += u0v[a].y;
            } else if constexpr (MODE == M_ITER) {
              const typename C2<T>::type u0 = ldc<T>(cptr<T>(D.U[cur], Pc, a), g);
              nr += u0.x;
              ni += u0.y;
            }
            stc<T>(mptr<T>(uout, Pc, a), g, nr, ni);
            vr[a][q][r] = nr;
            vi[a][q][r] = ni;
          }
        }
      }
    }
    inverse_all(SS, 0, std::integral_constant<int, S>{}, strain_gen);
  } else if constexpr (MODE == M_MAT) {
#pragma unroll
    for (int q = 0; q < BP; ++q)
#pragma unroll
      for (int r = 0; r < RP; ++r)
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          T re = T(0), im = T(0);
          if (pv[q]) {
            const typename C2<T>::type u0 = ldc<T>(cptr<T>(D.U[cur], Pc, a), gidx(q, r));
            re = u0.x;
            im = u0.y;
          }
          vr[a][q][r] = re;
          vi[a][q][r] = im;
        }
    inverse_all(SS, 0, std::integral_constant<int, S>{}, strain_gen);
    inverse_all(SS, S, std::integral_constant<int, DIM>{}, [&](int c, int q, int r, T& re, T& im) {
      re = vr[c][q][r] * inv_n;
      im = vi[c][q][r] * inv_n;
    });
    return;
  } else if constexpr (MODE == M_CG_AP) {
    // q = A p = -i xi . sigma^(p): stored, and the partial p.q
    zero_v();
    forward_all(SS, std::integral_constant<int, S>{},
                [&](int c, int q, int r, T re, T im) { div_acc(c, q, r, re, im, T(-1)); });
#pragma unroll
    for (int q = 0; q < BP; ++q) {
      if (!pv[q]) continue;
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const int g = gidx(q, r);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          const typename C2<T>::type pd = ldc<T>(cptr<T>(D.Pd, Pc, a), g);
          stc<T>(mptr<T>(D.Q, Pc, a), g, vr[a][q][r], vi[a][q][r]);
          part += double(pw[q]) * (double(pd.x) * double(vr[a][q][r]) + double(pd.y) * double(vi[a][q][r]));
        }
      }
    }
  } else if constexpr (MODE == M_CG_DIR) {
    // p = N0 r + beta p, stored, then eps^(p) / |N| and its inverse transform
    const T beta = T(St->beta);
#pragma unroll
    for (int q = 0; q < BP; ++q) {
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        if (!pv[q]) {
#pragma unroll
          for (int a = 0; a < DIM; ++a) { vr[a][q][r] = T(0); vi[a][q][r] = T(0); }
          continue;
        }
        T xi[DIM], xi2;
        point_xi(q, r, xi, xi2);
        const int g = gidx(q, r);
        T zr[DIM], zi[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          const typename C2<T>::type rv = ldc<T>(cptr<T>(D.R, Pc, a), g);
          zr[a] = rv.x;
          zi[a] = rv.y;
        }
        if (D.precond) apply_n0<T, DIM>(xi, xi2, c0, mu0, zr, zi);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          const typename C2<T>::type pd = ldc<T>(cptr<T>(D.Pd, Pc, a), g);
          const T nr = zr[a] + beta * pd.x, ni = zi[a] + beta * pd.y;
          stc<T>(mptr<T>(D.Pd, Pc, a), g, nr, ni);
          vr[a][q][r] = nr;
          vi[a][q][r] = ni;
        }
      }
    }
    inverse_all(SS, 0, std::integral_constant<int, S>{}, strain_gen);
  } else if constexpr (MODE == M_KCONV) {
    // periodic convolution with a kernel given by its half spectrum:
    // eps^_c = sum_j Kh_cj f^_j / |N| from the (projected) force spectrum,
    // then the inverse outer transforms of the s components
#pragma unroll
    for (int q = 0; q < BP; ++q)
#pragma unroll
      for (int r = 0; r < RP; ++r)
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          T re = T(0), im = T(0);
          if (pv[q]) {
            const typename C2<T>::type fv = ldc<T>(cptr<T>(D.F, Pc, a), gidx(q, r));
            re = fv.x;
            im = fv.y;
          }
          vr[a][q][r] = re;
          vi[a][q][r] = im;
        }
    // The kx = 0 column packs two planes, Z = P0 + i PH (P0, PH the planes'
    // own spectra over (ky, kz)), and a product of two packed spectra is not
    // the packed product: there P0 = (Z + conj Z') / 2 and PH = (Z - conj Z')
    // / (2 i) with Z' the entry at (-ky, -kz), and A0 B0 + i AH BH =
    // ((A + A*)(B + B*) - i (A - A*)(B - B*)) / 4 with X* = conj X'.
    int pk0[BP], pth[BP];
#pragma unroll
    for (int q = 0; q < BP; ++q) {
      int m, j;
      FF::template bj<RP>(tid + q * NTH, m, j);
      pk0[q] = t.kx(m) == 0;
      pth[q] = t.other(m);
    }
    inverse_all(SS, 0, std::integral_constant<int, S>{}, [&](int c, int q, int r, T& re, T& im) {
      re = T(0);
      im = T(0);
      if (!pv[q]) return;
      const int g = gidx(q, r);
      if (pk0[q]) {
        const int n = pj[q] + r * NSTEP;
        const int gp = (DIM == 3) ? (int)spec_at(D, 0, (D.ny - pth[q]) % D.ny, (D.nz - n) % D.nz)
                                  : ((D.ny - n) % D.ny) * D.H;
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          const typename C2<T>::type a = ldc<T>(cptr<T>(D.Kh, Pc, c * DIM + j), g);
          const typename C2<T>::type a2 = ldc<T>(cptr<T>(D.Kh, Pc, c * DIM + j), gp);
          const typename C2<T>::type b2 = ldc<T>(cptr<T>(D.F, Pc, j), gp);
          const T br = vr[j][q][r], bi = vi[j][q][r];
          const T pr = a.x + a2.x, pi = a.y - a2.y;          // A + A*
          const T qr = a.x - a2.x, qi = a.y + a2.y;          // A - A*
          const T rr = br + b2.x, ri = bi - b2.y;            // B + B*
          const T sr = br - b2.x, si = bi + b2.y;            // B - B*
          const T ur = pr * rr - pi * ri, ui = pr * ri + pi * rr;   // (A + A*)(B + B*)
          const T vr_ = qr * sr - qi * si, vi_ = qr * si + qi * sr; // (A - A*)(B - B*)
          re += T(0.25) * (ur + vi_);
          im += T(0.25) * (ui - vr_);
        }
      } else {
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          const typename C2<T>::type kv = ldc<T>(cptr<T>(D.Kh, Pc, c * DIM + j), g);
          re += kv.x * vr[j][q][r] - kv.y * vi[j][q][r];
          im += kv.x * vi[j][q][r] + kv.y * vr[j][q][r];
        }
      }
      re *= inv_n;
      im *= inv_n;
    });
    return;
  } else if constexpr (MODE == M_AA_RES) {
    // Anderson acceleration, first half, at iteration k (state x_k in
    // U[cur], x_{k-1} in the other buffer): the residual r = i xi . sigma^ +
    // f^ with its FP64 norm, F = N0 r (the basic scheme's step), the newest
    // differences dF = F - F_{k-1} and dU = x_k - x_{k-1} into ring slot
    // (k - 1) mod m, F into Fp, and the inner products of the window's dF_j
    // (newest first) with dF and with F.  No inverse transforms.
    zero_v();
    forward_all(SS, std::integral_constant<int, S>{},
                [&](int c, int q, int r, T re, T im) { div_acc(c, q, r, re, im, T(1)); });
    const int k = St->iter;
    const int m = D.aa_m;
    const int nw = k < m ? k : m;
    const int snew = k >= 1 ? (k - 1) % m : 0;
    double pg[kAAMax], pb[kAAMax];
#pragma unroll
    for (int j = 0; j < kAAMax; ++j) {
      pg[j] = 0.0;
      pb[j] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < BP; ++q) {
      if (!pv[q]) continue;
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        T xi[DIM], xi2;
        point_xi(q, r, xi, xi2);
        const int g = gidx(q, r);
        T fr[DIM], fi[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          const typename C2<T>::type fv = ldc<T>(cptr<T>(D.F, Pc, a), g);
          const T rr = vr[a][q][r] + fv.x, ri = vi[a][q][r] + fv.y;
          part += double(pw[q]) * (double(rr) * double(rr) + double(ri) * double(ri));
          fr[a] = rr;
          fi[a] = ri;
        }
        apply_n0<T, DIM>(xi, xi2, c0, mu0, fr, fi);   // F = N0 r
        if (k >= 1) {
          T dfr[DIM], dfi[DIM];
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            const typename C2<T>::type fo = ldc<T>(cptr<T>(D.Fp, Pc, a), g);
            const typename C2<T>::type u0 = ldc<T>(cptr<T>(D.U[cur], Pc, a), g);
            const typename C2<T>::type u1 = ldc<T>(cptr<T>(D.U[cur ^ 1], Pc, a), g);
            dfr[a] = fr[a] - fo.x;
            dfi[a] = fi[a] - fo.y;
            stc<T>(mptr<T>(D.DF, Pc, snew * DIM + a), g, dfr[a], dfi[a]);
            stc<T>(mptr<T>(D.DU, Pc, snew * DIM + a), g, u0.x - u1.x, u0.y - u1.y);
          }
#pragma unroll
          for (int j = 0; j < kAAMax; ++j) {
            if (j >= nw) break;
            const int sj = (snew - j + m) % m;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
              T jr = dfr[a], ji = dfi[a];
              if (j > 0) {
                const typename C2<T>::type v = ldc<T>(cptr<T>(D.DF, Pc, sj * DIM + a), g);
                jr = v.x;
                ji = v.y;
              }
              pg[j] += double(pw[q]) * (double(jr) * double(dfr[a]) + double(ji) * double(dfi[a]));
              pb[j] += double(pw[q]) * (double(jr) * double(fr[a]) + double(ji) * double(fi[a]));
            }
          }
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) stc<T>(mptr<T>(D.Fp, Pc, a), g, fr[a], fi[a]);
      }
    }
    const double s0 = block_sum<NTH>(part, red);
    if (tid == 0) gst<double>(D.partial, (long long)kAAPart * local, s0);
#pragma unroll
    for (int j = 0; j < kAAMax; ++j) {
      if (j >= nw) break;
      const double a1 = block_sum<NTH>(pg[j], red);
      const double a2 = block_sum<NTH>(pb[j], red);
      if (tid == 0) {
        gst<double>(D.partial, (long long)kAAPart * local + 1 + j, a1);
        gst<double>(D.partial, (long long)kAAPart * local + 1 + kAAMax + j, a2);
      }
    }
    return;
  } else if constexpr (MODE == M_AA_UPD) {
    // second half, after the stopping rule advanced the iteration to k + 1:
    // x_{k+1} = x_k + F_k - sum_j gamma_j (dU_j + dF_j) into the buffer of
    // x_{k-1}, then its strain spectrum and the inverse outer transforms
    const int k1 = St->iter;
    const int cur2 = k1 & 1;
    const int k = k1 - 1;
    const int m = D.aa_m;
    const int nw = k < m ? k : m;
    const int snew = k >= 1 ? (k - 1) % m : 0;
    T gam[kAAMax];
#pragma unroll
    for (int j = 0; j < kAAMax; ++j) gam[j] = (j < nw) ? T(D.aa[m * m + j]) : T(0);
#pragma unroll
    for (int q = 0; q < BP; ++q) {
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        if (!pv[q]) {
#pragma unroll
          for (int a = 0; a < DIM; ++a) { vr[a][q][r] = T(0); vi[a][q][r] = T(0); }
          continue;
        }
        const int g = gidx(q, r);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          const typename C2<T>::type xk = ldc<T>(cptr<T>(D.U[cur2 ^ 1], Pc, a), g);
          const typename C2<T>::type fk = ldc<T>(cptr<T>(D.Fp, Pc, a), g);
          T nr = xk.x + fk.x, ni = xk.y + fk.y;
#pragma unroll
          for (int j = 0; j < kAAMax; ++j) {
            if (j >= nw) break;
            const int sj = (snew - j + m) % m;
            const typename C2<T>::type du = ldc<T>(cptr<T>(D.DU, Pc, sj * DIM + a), g);
            const typename C2<T>::type df = ldc<T>(cptr<T>(D.DF, Pc, sj * DIM + a), g);
            nr -= gam[j] * (du.x + df.x);
            ni -= gam[j] * (du.y + df.y);
          }
          stc<T>(mptr<T>(D.U[cur2], Pc, a), g, nr, ni);
          vr[a][q][r] = nr;
          vi[a][q][r] = ni;
        }
      }
    }
    inverse_all(SS, 0, std::integral_constant<int, S>{}, strain_gen);
    return;
  }

  // FP64 partial sums of this item, one slot per item; a separate one-block
  // kernel sums the slots in a fixed order (bitwise reproducible)
  if constexpr (MODE == M_INIT || MODE == M_ITER || MODE == M_CG_INIT || MODE == M_CG_AP) {
    const double s1 = block_sum<NTH>(part, red);
    if constexpr (MODE == M_CG_INIT) {
      const double s2 = block_sum<NTH>(part2, red);
      if (tid == 0) {
        gst<double>(D.partial, 2 * local, s1);
        gst<double>(D.partial, 2 * local + 1, s2);
      }
    } else {
      if (tid == 0) gst<double>(D.partial, 2 * local, s1);
    }
  }
}

// ---------------------------------------------------------------------------
// CG pointwise update: u += alpha p, r -= alpha q, partials r.z and r.r
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__device__ void cg_update_item(const InstDesc& D, InstState* St, int local, unsigned char* smem) {
  constexpr int NTH = Cfg<T>::NTH;
  // entries per batch whose loads are all issued before the batch's stores
  constexpr int QB = (sizeof(T) == 4) ? 4 : 2;
  using V2 = typename C2<T>::type;
  const int tid = threadIdx.x;
  double* red = reinterpret_cast<double*>(smem);
  const T alpha = T(St->alpha);
  const T mu0 = T(D.mu0);
  const T c0 = T((D.lam0 + D.mu0) / (D.lam0 + 2.0 * D.mu0));
  const long long Pc = D.Pc;
  double prz = 0.0, prr = 0.0;
  for (int q0 = 0; q0 < 4; q0 += QB) {
    V2 uv[QB][DIM], pv[QB][DIM], rv[QB][DIM], qv[QB][DIM];
#pragma unroll
    for (int qq = 0; qq < QB; ++qq) {
      const long long g = (long long)local * NTH * 4 + (q0 + qq) * NTH + tid;
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        if (g < Pc) {
          uv[qq][a] = ldc<T>(cptr<T>(D.U[0], Pc, a), g);
          pv[qq][a] = ldc<T>(cptr<T>(D.Pd, Pc, a), g);
          rv[qq][a] = ldc<T>(cptr<T>(D.R, Pc, a), g);
          qv[qq][a] = ldc<T>(cptr<T>(D.Q, Pc, a), g);
        }
      }
    }
#pragma unroll
    for (int qq = 0; qq < QB; ++qq) {
      const long long g = (long long)local * NTH * 4 + (q0 + qq) * NTH + tid;
      if (g >= Pc) continue;
      int kx, ky, kz;
      spec_coords(D, g, kx, ky, kz);
      T xi[DIM];
      xi[0] = T(wavenum(kx, D.nx, D.kx));
      xi[1] = T(wavenum(ky, D.ny, D.ky));
      if constexpr (DIM == 3) xi[2] = T(wavenum(kz, D.nz, D.kz));
      T xi2 = T(0);
#pragma unroll
      for (int a = 0; a < DIM; ++a) xi2 += xi[a] * xi[a];
      const double wgt = (kx == 0) ? 1.0 : 2.0;
      T rr[DIM], ri[DIM];
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        stc<T>(mptr<T>(D.U[0], Pc, a), g, uv[qq][a].x + alpha * pv[qq][a].x, uv[qq][a].y + alpha * pv[qq][a].y);
        rr[a] = rv[qq][a].x - alpha * qv[qq][a].x;
        ri[a] = rv[qq][a].y - alpha * qv[qq][a].y;
        stc<T>(mptr<T>(D.R, Pc, a), g, rr[a], ri[a]);
        prr += wgt * (double(rr[a]) * double(rr[a]) + double(ri[a]) * double(ri[a]));
      }
      T zr[DIM], zi[DIM];
#pragma unroll
      for (int a = 0; a < DIM; ++a) { zr[a] = rr[a]; zi[a] = ri[a]; }
      if (D.precond) apply_n0<T, DIM>(xi, xi2, c0, mu0, zr, zi);
#pragma unroll
      for (int a = 0; a < DIM; ++a) prz += wgt * (double(rr[a]) * double(zr[a]) + double(ri[a]) * double(zi[a]));
    }
  }
  const double s1 = block_sum<NTH>(prz, red);
  const double s2 = block_sum<NTH>(prr, red);
  if (tid == 0) {
    gst<double>(D.partial, 2 * local, s1);
    gst<double>(D.partial, 2 * local + 1, s2);
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// Workgroups are dispatched to the eight XCDs in turn.  Map workgroup b of
// a grid of G to a slot such that each XCD runs one contiguous range of
// slots: neighbouring tiles of the outer pass, which share 128-byte lines
// along kx, then meet in the same L2 instead of each XCD fetching the lines.
__device__ __forceinline__ int xcd_slot(int b, int G) {
  constexpr int X = 8;
  const int q = G / X, r = G - (G / X) * X;
  const int x = b - (b / X) * X, k = b / X;
  return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ bool gated(int mode) {
  return mode == M_ITER || mode == M_CG_AP || mode == M_CG_UPD || mode == M_CG_DIR || mode == M_CG_INIT ||
         mode == M_AA_RES || mode == M_AA_UPD;
}


// The supported axis lengths (the twiddle table's order), split into the
// short ones and those of 32 points and more: the outer-pass launchers of the
// two groups are built in separate translation units.
#define LSFFT_LEN_CASES_SHORT(X) X(4) X(6) X(8) X(12) X(16) X(24)
#define LSFFT_LEN_CASES_LONG(X) X(32) X(48) X(64) X(96) X(128) X(256)
#define LSFFT_LEN_CASES(X) LSFFT_LEN_CASES_SHORT(X) LSFFT_LEN_CASES_LONG(X)

// One kernel per (precision, length, dimension, mode): every work item of a
// launch has the same transform length, so register allocation and LDS
// layout are those of that length alone.
template <typename T, int NX, int DIM, int MODE, int V>
__global__ __launch_bounds__(Cfg<T>::NTH_X) __attribute__((amdgpu_waves_per_eu(LSFFT_WAVES_X))) void k_xpass(
    const InstDesc* __restrict__ descs, InstState* __restrict__ states, const WorkItem* __restrict__ items,
    const int* __restrict__ nitems, const double* __restrict__ lame, const T* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n_items = *nitems;
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const WorkItem it = items[w];
    const InstDesc& D = descs[it.inst];
    if (gated(MODE) && states[it.inst].status != ST_RUNNING) continue;
    xpass_item<T, NX, DIM, MODE, V>(D, it.local, lame, tw, smem);
    __syncthreads();
  }
}

// Fixed-order FP64 sums of one solve's per-item partials, then the stopping
// rule, by one block of NTH threads: thread k adds slots k, k + NTH, ...
// (eight loads issued before their adds), then block_sum.  The order depends
// on NTH only, so every caller with the same block size gets the same bits.
template <int NTH>
__device__ inline void reduce_solve(const InstDesc& D, InstState& St, int mode, double* red) {
  if (mode != M_INIT && St.status != ST_RUNNING) return;
  const int nslot = (mode == M_CG_UPD) ? D.items_cg : D.items_g;
  const bool two = (mode == M_CG_INIT || mode == M_CG_UPD);
  constexpr int U = 8;
  double a = 0.0, b = 0.0;
  for (int k0 = threadIdx.x; k0 < nslot; k0 += NTH * U) {
    double va[U], vb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * NTH;
      va[u] = (k < nslot) ? D.partial[2 * k] : 0.0;
      vb[u] = (two && k < nslot) ? D.partial[2 * k + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a += va[u];
      b += vb[u];
    }
  }
  a = block_sum<NTH>(a, red);
  b = block_sum<NTH>(b, red);
  // thread 0 applies the rule (the state is read here, not kept across the
  // barriers above, where it would live in scratch)
  if (threadIdx.x == 0) {
    InstState loc = St;
    finalize(D, loc, mode, a, b);
    St = loc;
  }
}

// Anderson acceleration's stopping rule and mixing coefficients, by one
// block per solve: fixed-order FP64 sums of the per-item partials of
// M_AA_RES (residual, <dF_j, dF_new>, <dF_j, F>), the stopping rule of the
// basic scheme, then the Gram matrix row and column of the newest ring slot
// and the window's normal equations G gamma = b, solved by Gaussian
// elimination with partial pivoting (a pivot below 1e-30 of the largest
// diagonal entry drops its direction: gamma = 0 there).
template <int NTH>
__device__ inline void reduce_aa(const InstDesc& D, InstState& St, double* red) {
  if (St.status != ST_RUNNING) return;
  const int nslot = D.items_g;
  const int m = D.aa_m;
  const int k = St.iter;
  const int nw = k < m ? k : m;
  double tot[kAAPart];
  for (int c = 0; c < kAAPart; ++c) {
    tot[c] = 0.0;
    if (c != 0 && (c - 1) % kAAMax >= nw) continue;
    double a = 0.0;
    for (int i = threadIdx.x; i < nslot; i += NTH) a += D.partial[(long long)kAAPart * i + c];
    tot[c] = block_sum<NTH>(a, red);
  }
  if (threadIdx.x != 0) return;
  InstState loc = St;
  judge(D, loc, sqrt(tot[0] / loc.fnorm2));
  if (loc.status == ST_RUNNING && nw > 0) {
    double* G = D.aa;
    const int snew = (k - 1) % m;
    int slot[kAAMax];
    for (int j = 0; j < nw; ++j) {
      slot[j] = (snew - j + m) % m;
      G[snew * m + slot[j]] = tot[1 + j];
      G[slot[j] * m + snew] = tot[1 + j];
    }
    double A[kAAMax][kAAMax], b[kAAMax];
    double dmax = 0.0;
    for (int j = 0; j < nw; ++j) {
      for (int l = 0; l < nw; ++l) A[j][l] = G[slot[j] * m + slot[l]];
      b[j] = tot[1 + kAAMax + j];
      dmax = fmax(dmax, fabs(A[j][j]));
    }
    bool live[kAAMax];
    for (int c = 0; c < nw; ++c) {
      int piv = c;
      for (int r = c + 1; r < nw; ++r)
        if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
      live[c] = fabs(A[piv][c]) > 1e-30 * dmax;
      if (!live[c]) continue;
      if (piv != c) {
        for (int l = 0; l < nw; ++l) {
          const double t = A[c][l];
          A[c][l] = A[piv][l];
          A[piv][l] = t;
        }
        const double t = b[c];
        b[c] = b[piv];
        b[piv] = t;
      }
      for (int r = c + 1; r < nw; ++r) {
        const double f = A[r][c] / A[c][c];
        for (int l = c; l < nw; ++l) A[r][l] -= f * A[c][l];
        b[r] -= f * b[c];
      }
    }
    double gam[kAAMax];
    for (int c = nw - 1; c >= 0; --c) {
      if (!live[c]) { gam[c] = 0.0; continue; }
      double v = b[c];
      for (int l = c + 1; l < nw; ++l) v -= A[c][l] * gam[l];
      gam[c] = v / A[c][c];
    }
    for (int j = 0; j < nw; ++j) G[m * m + j] = gam[j];
  }
  St = loc;
}

// one component per work unit: unit w covers item w % n_items, component w / n_items.
// With red_n set, the blocks first apply the stopping rule of the outer pass
// that ran before (basic iteration) to the red_inst[0 .. *red_n) solves; the
// gate below may then see a solve stop while its tiles are being
// transformed, which is harmless (its returned iterate sits in the other
// displacement buffer, and its work spectrum is rewritten before any use)
// as long as each block takes one decision per unit.
template <typename T, int NY, int DIR, int V>
__global__ __launch_bounds__(Cfg<T>::NTH) __attribute__((amdgpu_waves_per_eu((YSched<T, NY, V>::WAVES)))) void k_ypass(
    const InstDesc* __restrict__ descs, InstState* __restrict__ states, const WorkItem* __restrict__ items,
    const int* __restrict__ nitems, const T* __restrict__ tw, int which, int ncomp, int gate,
    const int* __restrict__ red_inst, const int* __restrict__ red_n) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (red_n) {
    __shared__ double red[Cfg<T>::NTH / 64];
    const int nr = *red_n;
    for (int r = blockIdx.x; r < nr; r += gridDim.x) {
      const int i = red_inst[r];
      reduce_solve<Cfg<T>::NTH>(descs[i], states[i], M_ITER, red);
      __syncthreads();
    }
  }
  const int n_items = *nitems;
  const int n_units = n_items * ncomp;
  // XCD-aware order when a tile row is narrower than a 128-byte line
  // (neighbouring tiles then share lines: 8 kx columns of FP32 at ny = 256);
  // with full lines the launch order is kept
  constexpr bool kXcd = YSched<T, NY, V>::MP * 2 * (int)sizeof(T) < 128;
  __shared__ int s_run;
  for (int w = kXcd ? xcd_slot(blockIdx.x, gridDim.x) : (int)blockIdx.x; w < n_units; w += gridDim.x) {
    const int c = w / n_items;
    const WorkItem it = items[w - c * n_items];
    const InstDesc& D = descs[it.inst];
    if (gate) {
      if (red_n) {
        // the prologue of another block may change this solve's status
        // while the block reads it: one read, shared, so that the whole
        // block transforms the unit or skips it (the transform's barriers
        // need every wave)
        if (threadIdx.x == 0) s_run = (states[it.inst].status == ST_RUNNING);
        __syncthreads();
        const bool go = s_run != 0;
        __syncthreads();   // read by every wave before the next unit rewrites it
        if (!go) continue;
      } else if (states[it.inst].status != ST_RUNNING) {
        continue;
      }
    }
    void* src = (which == 0) ? D.S : D.F;
    void* dst = src;
    if (D.blk) {
      if (DIR < 0) dst = D.S2;
      else src = D.S2;
    }
    ypass_item<T, NY, DIR, V>(D, it.local, c, src, dst, tw, smem);
    __syncthreads();
  }
}

template <typename T, int NG, int DIM, int MODE, int V>
__global__ __launch_bounds__((GSched<T, NG, V>::NTH)) __attribute__((amdgpu_waves_per_eu((GSched<T, NG, V>::WAVES)))) void k_green(
    const InstDesc* __restrict__ descs, InstState* __restrict__ states, const WorkItem* __restrict__ items,
    const int* __restrict__ nitems, const T* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n_items = *nitems;
  for (int w = xcd_slot(blockIdx.x, gridDim.x); w < n_items; w += gridDim.x) {
    const WorkItem it = items[w];
    const InstDesc& D = descs[it.inst];
    InstState* St = states + it.inst;
    if (gated(MODE) && St->status != ST_RUNNING) continue;
    green_item<T, NG, DIM, MODE, V>(D, St, it.local, tw, smem);
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(Cfg<T>::NTH) void k_cg_update(const InstDesc* __restrict__ descs,
                                                           InstState* __restrict__ states,
                                                           const WorkItem* __restrict__ items,
                                                           const int* __restrict__ nitems) {
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
constexpr int NTR = 256;   // reduction, validation and averaging kernels

// One block per solve: fixed-order FP64 sums of the per-item partials, then
// the stopping rule.  NTH is the y-pass block size of the plan's precision,
// so that the same sums run as that pass's prologue with the same bits.
template <int NTH>
__global__ __launch_bounds__(NTH) void k_reduce(const InstDesc* __restrict__ descs, InstState* __restrict__ states,
                                                const int* __restrict__ inst_list, const int* __restrict__ ninst,
                                                int mode) {
  __shared__ double red[NTH / 64];
  // the number of listed solves is read on the device: a captured launch
  // keeps its grid while solves retire
  if ((int)blockIdx.x >= *ninst) return;
  const int i = inst_list[blockIdx.x];
  if (mode == M_AA_RES) reduce_aa<NTH>(descs[i], states[i], red);
  else reduce_solve<NTH>(descs[i], states[i], mode, red);
}

// Largest phase id of a phase map (argument validation on the device).
__global__ __launch_bounds__(NTR) void k_phase_max(const uint8_t* __restrict__ phase, long long n, int* __restrict__ out) {
  __shared__ int red[NTR];
  int m = 0;
  for (long long i = (long long)blockIdx.x * NTR + threadIdx.x; i < n; i += (long long)gridDim.x * NTR)
    m = max(m, (int)phase[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = NTR / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, red[0]);
}

// Translated averaging (Eqs. 3.5-3.6): for every voxel, in the fixed order of
// the group's shifts, sum u, u V, eps, eps V, sigma, sigma V and V, V the
// indicator of the inclusion phase in the shifted microstructure.  Sums are
// added to the FP64 accumulator; no atomics, one thread per voxel.
template <typename T, int DIM>
__global__ __launch_bounds__(NTR) void k_accumulate(const InstDesc* __restrict__ descs,
                                                    const GroupDesc* __restrict__ groups, int g,
                                                    const double* __restrict__ lame) {
  constexpr int S = (DIM == 3) ? 6 : 3;
  constexpr int NC = 2 * DIM + 4 * S + 1;
  const GroupDesc G = groups[g];
  const InstDesc& D0 = descs[G.first];
  const long long nvox = D0.nvox;
  for (long long v = (long long)blockIdx.x * NTR + threadIdx.x; v < nvox; v += (long long)gridDim.x * NTR) {
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

// a fill kernel instead of a memset: callers of the allocation-free entry
// points may capture their work in a graph
__global__ __launch_bounds__(NTR) void k_zero_u64(unsigned long long* __restrict__ a, long long n) {
  for (long long i = (long long)blockIdx.x * NTR + threadIdx.x; i < n; i += (long long)gridDim.x * NTR) a[i] = 0ull;
}

__global__ __launch_bounds__(NTR) void k_scale(double* __restrict__ a, long long n, double s) {
  for (long long i = (long long)blockIdx.x * NTR + threadIdx.x; i < n; i += (long long)gridDim.x * NTR) a[i] *= s;
}

// RVE identification (Definition 2.2): radial maxima of the averaged strain
// and stress magnitudes about a centre.  Per voxel: the minimum-image offset
// to the centre (periodic cell, voxel units, then times the spacing), the
// distance r, bin floor(r / dr), and |eps|, |sigma| = sqrt(sum_ab t_ab^2)
// with Voigt shear counted twice.  The arithmetic is pinned to IEEE
// round-to-nearest operations in a fixed order (no contraction).  Bin maxima
// of non-negative doubles are integer maxima of their bit patterns: the
// result does not depend on the order of the updates.
constexpr int kRveMaxBins = 1024;
template <int DIM>
__global__ __launch_bounds__(NTR) void k_radial_max(const double* __restrict__ avg, int nx, int ny, int nz, double hx,
                                                    double hy, double hz, double cx, double cy, double cz, double dr,
                                                    int nbins, unsigned long long* __restrict__ bins) {
#pragma clang fp contract(off)
  constexpr int S = (DIM == 3) ? 6 : 3;
  __shared__ unsigned long long lmax[2 * kRveMaxBins];
  for (int b = threadIdx.x; b < 2 * nbins; b += NTR) lmax[b] = 0ull;
  __syncthreads();
  const long long nvox = (long long)nx * ny * nz;
  const double* eps = avg + (long long)(2 * DIM) * nvox;
  const double* sig = eps + (long long)(2 * S) * nvox;
  for (long long v = (long long)blockIdx.x * NTR + threadIdx.x; v < nvox; v += (long long)gridDim.x * NTR) {
    const int x = (int)(v % nx);
    const int y = (int)((v / nx) % ny);
    const int z = (int)(v / ((long long)nx * ny));
    // minimum-image offsets (voxel units), then times the spacing
    double ox = (double)x - cx, oy = (double)y - cy, oz = (double)z - cz;
    ox = ox - (double)nx * rint(ox / (double)nx);
    oy = oy - (double)ny * rint(oy / (double)ny);
    oz = oz - (double)nz * rint(oz / (double)nz);
    const double dx = ox * hx, dy = oy * hy, dz = oz * hz;
    double r2 = dx * dx;
    r2 = r2 + dy * dy;
    if constexpr (DIM == 3) r2 = r2 + dz * dz;
    int b = (int)floor(sqrt(r2) / dr);
    if (b >= nbins) b = nbins - 1;
    double ae = 0.0, as = 0.0;
#pragma unroll
    for (int c = 0; c < S; ++c) {
      const double e = eps[(long long)c * nvox + v], t = sig[(long long)c * nvox + v];
      const double qe = e * e, qs = t * t;
      ae = ae + ((c < DIM) ? qe : 2.0 * qe);
      as = as + ((c < DIM) ? qs : 2.0 * qs);
    }
    atomicMax(&lmax[b], (unsigned long long)__double_as_longlong(sqrt(ae)));
    atomicMax(&lmax[nbins + b], (unsigned long long)__double_as_longlong(sqrt(as)));
  }
  __syncthreads();
  for (int b = threadIdx.x; b < 2 * nbins; b += NTR)
    if (lmax[b]) atomicMax(&bins[b], lmax[b]);
}

// ---- data kernels of the surrogate's dataset --------------------------------
// Block means: out[f][Z][Y][X] = scale * mean of the fct^d (fct^2 when nz = 1)
// fine voxels of block (X, Y, Z) of field f; FP64 sums in a fixed order.
template <typename T, typename TO>
__global__ __launch_bounds__(NTR) void k_block_mean(const T* __restrict__ in, TO* __restrict__ out, long long nfield,
                                                    int nx, int ny, int nz, int fct, double scale) {
  const int fz = nz > 1 ? fct : 1;
  const int cx = nx / fct, cy = ny / fct, cz = nz / fz;
  const long long ncoarse = (long long)cx * cy * cz;
  const long long total = nfield * ncoarse;
  const double w = scale / double(fct * fct * fz);
  for (long long o = (long long)blockIdx.x * NTR + threadIdx.x; o < total; o += (long long)gridDim.x * NTR) {
    const long long fld = o / ncoarse;
    long long rem = o - fld * ncoarse;
    const int X = int(rem % cx);
    rem /= cx;
    const int Y = int(rem % cy);
    const int Z = int(rem / cy);
    const T* src = in + fld * ((long long)nx * ny * nz);
    double acc = 0.0;
    for (int dz = 0; dz < fz; ++dz)
      for (int dy = 0; dy < fct; ++dy)
        for (int dx = 0; dx < fct; ++dx)
          acc += double(src[((long long)(Z * fz + dz) * ny + (Y * fct + dy)) * nx + (X * fct + dx)]);
    out[o] = TO(acc * w);
  }
}

// Per-sample Euclidean norms, one block per sample, fixed summation order:
// res[2 s] = ||y_s - t_s|| (||t_s|| when y is null), res[2 s + 1] = ||t_s||.
template <typename T>
__global__ __launch_bounds__(NTR) void k_sample_norms(const T* __restrict__ y, const T* __restrict__ t, long long len,
                                                      double* __restrict__ res) {
  __shared__ double red[NTR / 64];
  const long long base = (long long)blockIdx.x * len;
  double dd = 0.0, tt = 0.0;
  for (long long i = threadIdx.x; i < len; i += NTR) {
    const double tv = double(t[base + i]);
    const double dv = y ? double(y[base + i]) - tv : tv;
    dd += dv * dv;
    tt += tv * tv;
  }
  dd = block_sum<NTR>(dd, red);
  tt = block_sum<NTR>(tt, red);
  if (threadIdx.x == 0) {
    res[2 * blockIdx.x] = sqrt(dd);
    res[2 * blockIdx.x + 1] = sqrt(tt);
  }
}

// Bump forces (Eq. 2.5's compact support): force f of a batch is the sum of
// its bumps exp(-1/(1 - r^2/R^2)) d (r < R, minimum-image distance to the
// bump's centre in the periodic cell, voxel units; zero outside).  bumps
// holds per bump (cx, cy, cz, R, dx, dy, dz); first[f] .. first[f + 1] are
// force f's bumps.  One thread per voxel and force.
template <typename T>
__global__ __launch_bounds__(NTR) void k_bump_forces(T* const* __restrict__ fs, const int* __restrict__ first,
                                                     const double* __restrict__ bumps, int nx, int ny, int nz, int dim) {
  const int fi = blockIdx.y;
  const long long nvox = (long long)nx * ny * nz;
  T* f = fs[fi];
  for (long long v = (long long)blockIdx.x * NTR + threadIdx.x; v < nvox; v += (long long)gridDim.x * NTR) {
    const double p[3] = {double(v % nx), double((v / nx) % ny), double(v / ((long long)nx * ny))};
    const double nn[3] = {double(nx), double(ny), double(nz)};
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = first[fi]; b < first[fi + 1]; ++b) {
      const double* B = bumps + 7 * b;
      double r2 = 0.0;
      for (int a = 0; a < dim; ++a) {
        double t = fmod(p[a] - B[a], nn[a]);
        if (t < 0.0) t += nn[a];
        if (t > 0.5 * nn[a]) t -= nn[a];
        r2 += t * t;
      }
      const double q = r2 / (B[3] * B[3]);
      if (q < 1.0) {
        const double e = exp(-1.0 / (1.0 - q));
        for (int a = 0; a < dim; ++a) acc[a] += e * B[4 + a];
      }
    }
    for (int a = 0; a < dim; ++a) f[a * nvox + v] = T(acc[a]);
  }
}

// ---- nonlocal kernel regression (Eqs. 6.5-6.6) ---------------------------
// The operator L_c[u](x) = sum over grid offsets 0 < |r| < delta of
// K_c(|r|) (u(x + r) - u(x)), K_c = sum_m c_m B_m(|r| / delta) in the
// Bernstein basis, and the features Phi_m[u] = sum_r B_m(|r| / delta)
// (u(x + r) - u(x)) of its least-squares fit.  Offsets of equal |r|^2 form a
// shell: Phi_m = sum_q W[m][q] (S_q - n_q u(x)) with S_q the sum of u over
// shell q's offsets and n_q its size.
//
// A workgroup stages one tile of the periodic field and its halo of width R
// (the largest offset component) in LDS, one displacement component at a
// time; each thread owns two voxels of the tile (the second kNlTZ / 2 along z
// in 3D, kNlTY2 / 2 along y in 2D).  Offsets arrive sorted by shell as LDS
// index deltas, so the shell loop and the offset loop are uniform across the
// workgroup.
constexpr int kNlMaxDeg = 8;                                   // degree M
constexpr int kNlMaxR = 6;                                     // horizon <= 7 voxels
constexpr int kNlF = kNlMaxDeg + 1;
constexpr int kNlTri = kNlF * (kNlF + 1) / 2;
constexpr int kNlAcc = kNlTri + kNlF + 1;                      // G (upper), g, Gamma . Gamma
constexpr int kNlTX = 8, kNlTY = 8, kNlTZ = 8;                 // 3D tile
constexpr int kNlTX2 = 16, kNlTY2 = 32;                        // 2D tile
constexpr int kNlGramBlocks = 2048;                            // fixed: the sum order never depends on the device

struct NlGeom {
  int nx, ny, nz, dim;
  int tx, ty, tz;          // tile
  int ntx, nty, ntz;       // tiles per axis
  int R;                   // halo width
  int lx, ly, lz;          // LDS box (tile + 2 R; lz = 1 in 2D)
  int nshell;
  int deg;
  int vpt;                 // voxels per thread: 2, or 1 (tiles of half the voxels)
};

// Matrix form K1(|r|) I + K2(|r|) e e^T: 2 (M + 1) features per component,
// one voxel per thread on tiles of 8 x 8 x 4 (3D) or 16 x 16 (2D), the
// features of a tile in LDS rows of kNlFeatPitch doubles, and one Gram
// entry per thread (the upper triangle row by row, then g, then
// Gamma . Gamma).  The halo of its 3D normal equations is at most kNlMaxR1.
constexpr int kNlF1 = 2 * kNlF;
constexpr int kNlAcc1 = kNlF1 * (kNlF1 + 1) / 2 + kNlF1 + 1;
constexpr int kNlMaxR1 = 4;
constexpr int kNlTZ1 = 4, kNlTY21 = 16;
constexpr int kNlFeatPitch = NTR + 1;
static_assert(kNlAcc1 <= NTR, "one Gram entry per thread");

template <typename T>
__device__ __forceinline__ void nl_stage(const NlGeom& G, const T* __restrict__ ua, int x0, int y0, int z0, T* lds) {
  const int nl = G.lx * G.ly * G.lz;
  for (int i = threadIdx.x; i < nl; i += NTR) {
    const int ix = i % G.lx, rest = i / G.lx;
    const int iy = rest % G.ly, iz = rest / G.ly;
    int gx = (x0 - G.R + ix) % G.nx;
    int gy = (y0 - G.R + iy) % G.ny;
    gx += gx < 0 ? G.nx : 0;
    gy += gy < 0 ? G.ny : 0;
    int gz = 0;
    if (G.dim == 3) {
      gz = (z0 - G.R + iz) % G.nz;
      gz += gz < 0 ? G.nz : 0;
    }
    lds[i] = ua[((long long)gz * G.ny + gy) * G.nx + gx];
  }
}

// tile `tile` of a field: origin and this thread's two voxels (local
// coordinates, LDS index of each voxel's centre, validity)
__device__ __forceinline__ void nl_tile(const NlGeom& G, int tile, int& x0, int& y0, int& z0, int (&vx)[2],
                                        int (&vy)[2], int (&vz)[2], int (&base)[2], bool (&ok)[2]) {
  const int tx = tile % G.ntx, rest = tile / G.ntx;
  const int ty = rest % G.nty, tz = rest / G.nty;
  x0 = tx * G.tx;
  y0 = ty * G.ty;
  z0 = tz * G.tz;
  const int t = threadIdx.x;
  const int lxv = t % G.tx, r2 = t / G.tx;
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const int vv = (G.vpt == 2) ? v : 0;      // one voxel per thread: both slots name it
    int ly, lz;
    if (G.dim == 3) {
      ly = r2 % G.ty;
      lz = r2 / G.ty + vv * (G.tz / 2);
    } else {
      ly = r2 + vv * (G.ty / 2);
      lz = 0;
    }
    vx[v] = x0 + lxv;
    vy[v] = y0 + ly;
    vz[v] = z0 + lz;
    ok[v] = vx[v] < G.nx && vy[v] < G.ny && vz[v] < G.nz && (G.vpt == 2 || v == 0);
    const int R = G.R, Rz = (G.dim == 3) ? G.R : 0;
    base[v] = ((lz + Rz) * G.ly + (ly + R)) * G.lx + (lxv + R);
  }
}

// shell sums minus n_q u(x) of both voxels, handed to fn(q, s0, s1)
template <typename T, typename Fn>
__device__ __forceinline__ void nl_shells(const NlGeom& G, const T* lds, const int (&base)[2],
                                          const int* __restrict__ offs, const int* __restrict__ first, Fn&& fn) {
  const double u0 = double(lds[base[0]]), u1 = double(lds[base[1]]);
  for (int q = 0; q < G.nshell; ++q) {
    const int o0 = first[q], o1 = first[q + 1];
    double s0 = 0.0, s1 = 0.0;
    for (int o = o0; o < o1; ++o) {
      const int d = offs[o];
      s0 += double(lds[base[0] + d]);
      s1 += double(lds[base[1] + d]);
    }
    const double cnt = double(o1 - o0);
    fn(q, s0 - cnt * u0, s1 - cnt * u1);
  }
}

// Normal equations: each workgroup walks items (sample, tile) b, b + grid,
// ... in order, accumulating per thread in FP64 the upper triangle of
// Phi Phi^T, Phi . Gamma and Gamma . Gamma over its voxels and the
// displacement components; the workgroup's sums go to its partial slot
// (kNlAcc doubles, laid out for degree kNlMaxDeg).
template <typename T>
__global__ __launch_bounds__(NTR) void k_nl_gram(NlGeom G, const T* __restrict__ u, const T* __restrict__ gam,
                                                 int nsample, const int* __restrict__ offs,
                                                 const int* __restrict__ first, const double* __restrict__ W,
                                                 double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char nl_smem[];
  T* lds = reinterpret_cast<T*>(nl_smem);
  const long long nvox = (long long)G.nx * G.ny * G.nz;
  const int ntile = G.ntx * G.nty * G.ntz;
  const int nf = G.deg + 1;
  double acc[kNlAcc];
#pragma unroll
  for (int i = 0; i < kNlAcc; ++i) acc[i] = 0.0;
  for (long long item = blockIdx.x; item < (long long)nsample * ntile; item += gridDim.x) {
    const int k = int(item / ntile), tile = int(item % ntile);
    int x0, y0, z0, vx[2], vy[2], vz[2], base[2];
    bool ok[2];
    nl_tile(G, tile, x0, y0, z0, vx, vy, vz, base, ok);
    for (int a = 0; a < G.dim; ++a) {
      const long long comp = ((long long)k * G.dim + a) * nvox;
      __syncthreads();
      nl_stage(G, u + comp, x0, y0, z0, lds);
      __syncthreads();
      double phi[2][kNlF];
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int m = 0; m < kNlF; ++m) phi[v][m] = 0.0;
      nl_shells(G, lds, base, offs, first, [&](int q, double s0, double s1) {
#pragma unroll
        for (int m = 0; m < kNlF; ++m) {
          if (m < nf) {
            const double w = W[m * G.nshell + q];
            phi[0][m] += w * s0;
            phi[1][m] += w * s1;
          }
        }
      });
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        if (!ok[v]) continue;
        const double gv = double(gam[comp + ((long long)vz[v] * G.ny + vy[v]) * G.nx + vx[v]]);
        int i = 0;
#pragma unroll
        for (int m = 0; m < kNlF; ++m)
#pragma unroll
          for (int n2 = m; n2 < kNlF; ++n2, ++i) acc[i] += phi[v][m] * phi[v][n2];
#pragma unroll
        for (int m = 0; m < kNlF; ++m) acc[kNlTri + m] += phi[v][m] * gv;
        acc[kNlTri + kNlF] += gv * gv;
      }
    }
  }
  // workgroup sum in a fixed order: waves by shuffles, then across waves
  // (in the staging LDS, which holds at least kNlAcc NTR / 64 doubles)
  double* red = reinterpret_cast<double*>(nl_smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kNlAcc; ++i) {
    double v = acc[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave * kNlAcc + i] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNlAcc) {
    double s = 0.0;
    for (int w = 0; w < NTR / 64; ++w) s += red[w * kNlAcc + threadIdx.x];
    partial[(long long)blockIdx.x * kNlAcc + threadIdx.x] = s;
  }
}

// fixed-order sum of the partial slots (one workgroup): out[i] = sum over
// slots of partial[slot stride + i], i < nacc
__global__ __launch_bounds__(NTR) void k_nl_gram_sum(const double* __restrict__ partial, int nslot, int stride,
                                                     int nacc, double* __restrict__ out) {
  __shared__ double red[NTR / 64];
  for (int i = 0; i < nacc; ++i) {
    double a = 0.0;
    for (int s = threadIdx.x; s < nslot; s += NTR) a += partial[(long long)s * stride + i];
    const double sum = block_sum<NTR>(a, red);
    if (threadIdx.x == 0) out[i] = sum;
  }
}

// The fitted operator: out = sum_q kw[q] (S_q - n_q u(x)) per component,
// kw[q] = K_c at shell q's radius; one workgroup per (sample, tile).
template <typename T>
__global__ __launch_bounds__(NTR) void k_nl_apply(NlGeom G, const T* __restrict__ u, int nsample,
                                                  const int* __restrict__ offs, const int* __restrict__ first,
                                                  const double* __restrict__ kw, T* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char nl_smem[];
  T* lds = reinterpret_cast<T*>(nl_smem);
  const long long nvox = (long long)G.nx * G.ny * G.nz;
  const int ntile = G.ntx * G.nty * G.ntz;
  const long long item = blockIdx.x;
  if (item >= (long long)nsample * ntile) return;
  const int k = int(item / ntile), tile = int(item % ntile);
  int x0, y0, z0, vx[2], vy[2], vz[2], base[2];
  bool ok[2];
  nl_tile(G, tile, x0, y0, z0, vx, vy, vz, base, ok);
  for (int a = 0; a < G.dim; ++a) {
    const long long comp = ((long long)k * G.dim + a) * nvox;
    __syncthreads();
    nl_stage(G, u + comp, x0, y0, z0, lds);
    __syncthreads();
    double r0 = 0.0, r1 = 0.0;
    nl_shells(G, lds, base, offs, first, [&](int q, double s0, double s1) {
      const double w = kw[q];
      r0 += w * s0;
      r1 += w * s1;
    });
    if (ok[0]) out[comp + ((long long)vz[0] * G.ny + vy[0]) * G.nx + vx[0]] = T(r0);
    if (ok[1]) out[comp + ((long long)vz[1] * G.ny + vy[1]) * G.nx + vx[1]] = T(r1);
  }
}

// Normal equations of the matrix form.  Per staged input component b and
// shell q: S = sum of (u_b(x + r) - u_b(x)) and T_a = sum of e_a e_b
// (u_b(x + r) - u_b(x)), then Phi1[b][m] += W[m][q] S and Phi2[a][m] +=
// W[m][q] T_a.  ee holds e_a e_b per offset as ee[(o 3 + b) 3 + a] (x
// first, zero beyond the dimension).
template <typename T>
__global__ __launch_bounds__(NTR) void k_nl_gram1(NlGeom G, const T* __restrict__ u, const T* __restrict__ gam,
                                                  int nsample, const int* __restrict__ offs,
                                                  const int* __restrict__ first, const double* __restrict__ ee,
                                                  const double* __restrict__ W, double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char nl_smem[];
  double* feat = reinterpret_cast<double*>(nl_smem);          // [kNlF1][kNlFeatPitch]
  double* gt = feat + kNlF1 * kNlFeatPitch;                    // [NTR]
  T* lds = reinterpret_cast<T*>(gt + NTR);                     // staged box
  const long long nvox = (long long)G.nx * G.ny * G.nz;
  const int ntile = G.ntx * G.nty * G.ntz;
  const int nf1 = G.deg + 1, nf = 2 * nf1;
  const int ntri = nf * (nf + 1) / 2;
  const int t = threadIdx.x;
  // the Gram entry this thread owns
  int kind = -1, ei = 0, ej = 0;
  if (t < ntri) {
    int i = 0, rem = t;
    while (rem >= nf - i) {
      rem -= nf - i;
      ++i;
    }
    kind = 0;
    ei = i;
    ej = i + rem;
  } else if (t < ntri + nf) {
    kind = 1;
    ei = t - ntri;
  } else if (t == ntri + nf) {
    kind = 2;
  }
  double acc = 0.0;
  for (long long item = blockIdx.x; item < (long long)nsample * ntile; item += gridDim.x) {
    const int k = int(item / ntile), tile = int(item % ntile);
    int x0, y0, z0, vx[2], vy[2], vz[2], base[2];
    bool ok[2];
    nl_tile(G, tile, x0, y0, z0, vx, vy, vz, base, ok);
    double p1[3][kNlF], p2[3][kNlF];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int m = 0; m < kNlF; ++m) {
        p1[a][m] = 0.0;
        p2[a][m] = 0.0;
      }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (b >= G.dim) break;
      __syncthreads();
      nl_stage(G, u + ((long long)k * G.dim + b) * nvox, x0, y0, z0, lds);
      __syncthreads();
      const double u0 = double(lds[base[0]]);
      for (int q = 0; q < G.nshell; ++q) {
        const int o0 = first[q], o1 = first[q + 1];
        double S = 0.0, T0 = 0.0, T1 = 0.0, T2 = 0.0;
        for (int o = o0; o < o1; ++o) {
          const double dv = double(lds[base[0] + offs[o]]) - u0;
          const double* e = ee + (o * 3 + b) * 3;
          S += dv;
          T0 += e[0] * dv;
          T1 += e[1] * dv;
          T2 += e[2] * dv;
        }
#pragma unroll
        for (int m = 0; m < kNlF; ++m) {
          if (m < nf1) {
            const double w = W[m * G.nshell + q];
            p1[b][m] += w * S;
            p2[0][m] += w * T0;
            p2[1][m] += w * T1;
            p2[2][m] += w * T2;
          }
        }
      }
    }
    // per output component: the tile's features into LDS, then every owner
    // thread adds its entry's sum over the tile's voxels
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= G.dim) break;
      __syncthreads();
#pragma unroll
      for (int m = 0; m < kNlF; ++m) {
        if (m < nf1) {
          feat[m * kNlFeatPitch + t] = ok[0] ? p1[a][m] : 0.0;
          feat[(nf1 + m) * kNlFeatPitch + t] = ok[0] ? p2[a][m] : 0.0;
        }
      }
      gt[t] = ok[0] ? double(gam[((long long)k * G.dim + a) * nvox + ((long long)vz[0] * G.ny + vy[0]) * G.nx + vx[0]])
                    : 0.0;
      __syncthreads();
      if (kind == 0) {
        const double* fi = feat + ei * kNlFeatPitch;
        const double* fj = feat + ej * kNlFeatPitch;
        for (int v = 0; v < NTR; ++v) acc += fi[v] * fj[v];
      } else if (kind == 1) {
        const double* fi = feat + ei * kNlFeatPitch;
        for (int v = 0; v < NTR; ++v) acc += fi[v] * gt[v];
      } else if (kind == 2) {
        for (int v = 0; v < NTR; ++v) acc += gt[v] * gt[v];
      }
    }
  }
  if (t < kNlAcc1) partial[(long long)blockIdx.x * kNlAcc1 + t] = (kind >= 0) ? acc : 0.0;
}

// The fitted matrix-form operator: out_a = sum over b and shells of
// (K1_q delta_ab S_q + K2_q T_aq), kw1 / kw2 the two kernels at each
// shell's radius; one workgroup per (sample, tile), two voxels per thread.
template <typename T>
__global__ __launch_bounds__(NTR) void k_nl_apply1(NlGeom G, const T* __restrict__ u, int nsample,
                                                   const int* __restrict__ offs, const int* __restrict__ first,
                                                   const double* __restrict__ ee, const double* __restrict__ kw1,
                                                   const double* __restrict__ kw2, T* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char nl_smem[];
  T* lds = reinterpret_cast<T*>(nl_smem);
  const long long nvox = (long long)G.nx * G.ny * G.nz;
  const int ntile = G.ntx * G.nty * G.ntz;
  const long long item = blockIdx.x;
  if (item >= (long long)nsample * ntile) return;
  const int k = int(item / ntile), tile = int(item % ntile);
  int x0, y0, z0, vx[2], vy[2], vz[2], base[2];
  bool ok[2];
  nl_tile(G, tile, x0, y0, z0, vx, vy, vz, base, ok);
  double r[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    if (b >= G.dim) break;
    __syncthreads();
    nl_stage(G, u + ((long long)k * G.dim + b) * nvox, x0, y0, z0, lds);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const double u0 = double(lds[base[v]]);
      for (int q = 0; q < G.nshell; ++q) {
        const int o0 = first[q], o1 = first[q + 1];
        double S = 0.0, T0 = 0.0, T1 = 0.0, T2 = 0.0;
        for (int o = o0; o < o1; ++o) {
          const double dv = double(lds[base[v] + offs[o]]) - u0;
          const double* e = ee + (o * 3 + b) * 3;
          S += dv;
          T0 += e[0] * dv;
          T1 += e[1] * dv;
          T2 += e[2] * dv;
        }
        const double w1 = kw1[q], w2 = kw2[q];
        r[v][b] += w1 * S;
        r[v][0] += w2 * T0;
        r[v][1] += w2 * T1;
        r[v][2] += w2 * T2;
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    if (!ok[v]) continue;
    const long long vox = ((long long)vz[v] * G.ny + vy[v]) * G.nx + vx[v];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (a < G.dim) out[((long long)k * G.dim + a) * nvox + vox] = T(r[v][a]);
  }
}

// ---- mixed-precision defect correction: FP64 state, FP32 inner solves ----
// Wavevector of entry g of the packed half spectrum (xi_x = 0 on the kx = 0
// column, which also carries the kx = H plane).
__device__ inline void spectrum_xi(const InstDesc& D, long long g, double xi[3]) {
  int kx, ky, kz;
  spec_coords(D, g, kx, ky, kz);
  xi[0] = wavenum(kx, D.nx, D.kx);
  xi[1] = wavenum(ky, D.ny, D.ky);
  xi[2] = (D.dim == 3) ? wavenum(kz, D.nz, D.kz) : 0.0;
}

__global__ __launch_bounds__(NTR) void k_widen(const float* __restrict__ src, double* __restrict__ dst, long long n) {
  for (long long i = (long long)blockIdx.x * NTR + threadIdx.x; i < n; i += (long long)gridDim.x * NTR)
    dst[i] = double(src[i]);
}

// FP32 force of the inner solve: r = K0 (N0 r), K0 = mu0 |xi|^2 I + (lam0 +
// mu0) xi xi^T the reference acoustic tensor, from the two FP64 state buffers
// of the outer step (u + N0 r and u).  Zero on the xi = 0 set.
__global__ __launch_bounds__(NTR) void k_defect(const InstDesc* __restrict__ d64, const InstState* __restrict__ s64,
                                                const InstDesc* __restrict__ d32, const int* __restrict__ inst) {
  const int i = inst[blockIdx.y];
  const InstDesc& C = d64[i];
  const int cur = s64[i].iter & 1;
  const double2* un = static_cast<const double2*>(C.U[cur]);
  const double2* uo = static_cast<const double2*>(C.U[cur ^ 1]);
  float2* F = static_cast<float2*>(d32[i].F);
  const long long Pc = C.Pc;
  const double b = C.lam0 + C.mu0;
  for (long long g = (long long)blockIdx.x * NTR + threadIdx.x; g < Pc; g += (long long)gridDim.x * NTR) {
    double xi[3];
    spectrum_xi(C, g, xi);
    const double xi2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
    double dr[3] = {0, 0, 0}, di[3] = {0, 0, 0}, pr = 0.0, pi = 0.0;
    for (int a = 0; a < C.dim; ++a) {
      const double2 x = un[a * Pc + g], y = uo[a * Pc + g];
      dr[a] = x.x - y.x;
      di[a] = x.y - y.y;
      pr += xi[a] * dr[a];
      pi += xi[a] * di[a];
    }
    for (int a = 0; a < C.dim; ++a)
      F[a * Pc + g] = make_float2(float(C.mu0 * xi2 * dr[a] + b * xi[a] * pr), float(C.mu0 * xi2 * di[a] + b * xi[a] * pi));
  }
}

// u += d: the FP64 state buffer that the next outer step reads becomes the
// previous state plus the returned iterate of the FP32 inner solve.
__global__ __launch_bounds__(NTR) void k_correct(const InstDesc* __restrict__ d64, const InstState* __restrict__ s64,
                                                 const InstDesc* __restrict__ d32, const InstState* __restrict__ s32,
                                                 const int* __restrict__ inst, int cg) {
  const int i = inst[blockIdx.y];
  const InstDesc& C = d64[i];
  const int cur = s64[i].iter & 1;
  const int sel = cg ? 0 : (s32[i].iter & 1);
  double2* dst = static_cast<double2*>(C.U[cur]);
  const double2* src = static_cast<const double2*>(C.U[cur ^ 1]);
  const float2* d = static_cast<const float2*>(d32[i].U[sel]);
  const long long n = (long long)C.dim * C.Pc;
  for (long long g = (long long)blockIdx.x * NTR + threadIdx.x; g < n; g += (long long)gridDim.x * NTR) {
    const double2 s = src[g];
    const float2 e = d[g];
    dst[g] = make_double2(s.x + double(e.x), s.y + double(e.y));
  }
}

// The returned FP64 iterate rounded once into the FP32 state buffer 0.
__global__ __launch_bounds__(NTR) void k_narrow(const InstDesc* __restrict__ d64, const InstState* __restrict__ s64,
                                                const InstDesc* __restrict__ d32, const int* __restrict__ inst) {
  const int i = inst[blockIdx.y];
  const InstDesc& C = d64[i];
  const double2* src = static_cast<const double2*>(C.U[s64[i].iter & 1]);
  float2* dst = static_cast<float2*>(d32[i].U[0]);
  const long long n = (long long)C.dim * C.Pc;
  for (long long g = (long long)blockIdx.x * NTR + threadIdx.x; g < n; g += (long long)gridDim.x * NTR)
    dst[g] = make_float2(float(src[g].x), float(src[g].y));
}
#endif  // LSFFT_MISC_TU

// ---------------------------------------------------------------------------
// LDS requirements (bytes) of one work item, per precision and length
// ---------------------------------------------------------------------------
template <typename T, int L, int V = 0> constexpr size_t lds_x() {
  using G = XGeom<T, L / 2, XSched<V>::EX_DIV>;
  return sizeof(T) * (2 * G::MR * G::SM + 2 * G::MR * G::SM2 + 2 * L + 2 * kMaxPhases);
}
// the iteration-mode x kernel (dynamic part only when its tiles are staged
// in static LDS buffers)
template <typename T, int L, int V = 0> constexpr size_t lds_xi() {
#ifndef LSFFT_NO_XDMA
  if (XDma<T, L / 2, XSched<V>::ALT, XSched<V>::EX_DIV>::ok) return XDma<T, L / 2, XSched<V>::ALT, XSched<V>::EX_DIV>::DYN;
#endif
  return lds_x<T, L, V>();
}
template <typename T, int L, int V = 0> constexpr size_t lds_y() {
  return sizeof(T) * (2 * PencilRows<T, L, YSched<T, L, V>::MP>::E + 2 * L);
}
template <typename T, int L, int V = 0> constexpr size_t lds_g() {
  return sizeof(T) * (4 * PencilRows<T, L, GSched<T, L, V>::MP>::E + 2 * L + 2) + sizeof(double) * 16;
}

}  // namespace lsfft
