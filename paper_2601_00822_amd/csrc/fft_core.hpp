// Mixed-radix Stockham FFT building blocks for gfx950 (MI355X).
//
// A workgroup transforms a tile of MP independent pencils of length N.  The
// first pass takes its inputs from registers (the caller loads them straight
// from HBM), the middle passes exchange data through one LDS buffer in place
// (gather into registers, barrier, butterfly, scatter, barrier), and the last
// pass leaves its outputs in registers, so a transform costs np - 1 LDS round
// trips for np passes.  Butterfly b of a pass maps to pencil m and index j;
// with JF = false pencils vary fastest across lanes (pencils strided in HBM:
// lanes read runs of consecutive pencils), with JF = true the index varies
// fastest (pencils contiguous in HBM: lanes read runs along the pencil).
//
// A pass of radix R over span NS reads the R inputs j + r N/R, multiplies by
// the twiddles of the current span, applies a radix-R butterfly and writes
// the autosorted outputs (j / NS) NS R + j % NS + r NS (Stockham form, no bit
// reversal).  In the last pass the outputs sit at j + r N/R, which are the
// input positions of a first pass of the same radix: the reversed plan of the
// inverse transform consumes the forward outputs where they are.
// Transforms are unnormalised: forward exp(-2 pi i k n / N), inverse
// exp(+2 pi i k n / N) (the DFT of Sec. 4, Eqs. 4.3-4.5; the 1/|N| of Eq. 4.4
// is applied once by the caller).
//
// Twiddles come from an LDS table tw[k] = exp(-2 pi i k / NTAB) read with
// stride TWS, so the table of a length-2N real transform also serves its
// length-N complex core.
#pragma once
#include <hip/hip_runtime.h>

namespace lsfft {

// ---------------------------------------------------------------------------
// radix plans (forward order): product of the radices is N
// ---------------------------------------------------------------------------
template <int N> struct Plan;
#define LSFFT_PLAN(N_, NP_, R0, R1, R2)                                  \
  template <> struct Plan<N_> {                                            \
    static constexpr int np = NP_;                                         \
    static constexpr int r0 = R0, r1 = R1, r2 = R2;                        \
  };
LSFFT_PLAN(2, 1, 2, 1, 1)
LSFFT_PLAN(3, 1, 3, 1, 1)
LSFFT_PLAN(4, 1, 4, 1, 1)
LSFFT_PLAN(6, 2, 3, 2, 1)
LSFFT_PLAN(8, 1, 8, 1, 1)
LSFFT_PLAN(12, 2, 4, 3, 1)
LSFFT_PLAN(16, 2, 4, 4, 1)
LSFFT_PLAN(24, 2, 8, 3, 1)
LSFFT_PLAN(32, 2, 4, 8, 1)
LSFFT_PLAN(48, 3, 4, 4, 3)
LSFFT_PLAN(64, 2, 8, 8, 1)
LSFFT_PLAN(96, 3, 4, 8, 3)
LSFFT_PLAN(128, 3, 4, 4, 8)
LSFFT_PLAN(256, 3, 4, 8, 8)

// Plans whose last forward radix is at most 4, for tiles held at 4 (or 3)
// points per thread between the forward and the inverse transform.
template <int N> struct PlanG;
#define LSFFT_PLANG(N_, NP_, R0, R1, R2)                                 \
  template <> struct PlanG<N_> {                                           \
    static constexpr int np = NP_;                                         \
    static constexpr int r0 = R0, r1 = R1, r2 = R2;                        \
  };
LSFFT_PLANG(2, 1, 2, 1, 1)
LSFFT_PLANG(3, 1, 3, 1, 1)
LSFFT_PLANG(4, 1, 4, 1, 1)
LSFFT_PLANG(6, 2, 2, 3, 1)
LSFFT_PLANG(8, 2, 2, 4, 1)
LSFFT_PLANG(12, 2, 4, 3, 1)
LSFFT_PLANG(16, 2, 4, 4, 1)
LSFFT_PLANG(24, 2, 8, 3, 1)
LSFFT_PLANG(32, 2, 8, 4, 1)
LSFFT_PLANG(48, 3, 4, 4, 3)
LSFFT_PLANG(64, 3, 4, 4, 4)
LSFFT_PLANG(96, 3, 4, 8, 3)
LSFFT_PLANG(128, 3, 8, 4, 4)
LSFFT_PLANG(256, 3, 8, 8, 4)
#undef LSFFT_PLAN
#undef LSFFT_PLANG

// radix of pass p, in forward order or reversed
template <template <int> class PL, int N, bool REV> struct PlanSeq {
  using P = PL<N>;
  static constexpr int np = P::np;
  static constexpr int fwd(int p) { return p == 0 ? P::r0 : p == 1 ? P::r1 : P::r2; }
  static constexpr int r(int p) { return REV ? fwd(np - 1 - p) : fwd(p); }
  // span before pass p
  static constexpr int ns(int p) {
    int s = 1;
    for (int q = 0; q < p; ++q) s *= r(q);
    return s;
  }
  static constexpr int first() { return r(0); }
  static constexpr int last() { return r(np - 1); }
  static_assert(np == 1 ? P::r0 == N : np == 2 ? P::r0 * P::r1 == N : P::r0 * P::r1 * P::r2 == N,
                "radix plan does not multiply to N");
};

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
  T tr, ti;
  if (DIR < 0) { tr = s3 * di; ti = -s3 * dr; } else { tr = -s3 * di; ti = s3 * dr; }
  vr[0] = vr[0] + sr; vi[0] = vi[0] + si;
  vr[1] = mr + tr; vi[1] = mi + ti;
  vr[2] = mr - tr; vi[2] = mi - ti;
}

template <typename T, int DIR>
__device__ __forceinline__ void bfly8(T* vr, T* vi) {
  const T h = T(0.70710678118654752440084436210484904);  // sqrt(2)/2
  bfly4_vals<T, DIR>(vr[0], vi[0], vr[2], vi[2], vr[4], vi[4], vr[6], vi[6]);
  bfly4_vals<T, DIR>(vr[1], vi[1], vr[3], vi[3], vr[5], vi[5], vr[7], vi[7]);
  {  // W8^1
    T r = vr[3], i = vi[3];
    if (DIR < 0) { vr[3] = h * (r + i); vi[3] = h * (i - r); }
    else         { vr[3] = h * (r - i); vi[3] = h * (i + r); }
  }
  {  // W8^2
    T r = vr[5], i = vi[5];
    if (DIR < 0) { vr[5] = i; vi[5] = -r; } else { vr[5] = -i; vi[5] = r; }
  }
  {  // W8^3
    T r = vr[7], i = vi[7];
    if (DIR < 0) { vr[7] = h * (i - r); vi[7] = -h * (r + i); }
    else         { vr[7] = -h * (r + i); vi[7] = h * (r - i); }
  }
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

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// waits for every direct global->LDS load of the wave still in flight (its
// fence covers LDS, which those loads write); this one lets such loads run on
// across the barrier, for kernels that prefetch a tile into a buffer nobody
// touches until an explicit wait.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}
template <bool LB> __device__ __forceinline__ void tile_sync() {
  if constexpr (LB) lds_barrier();
  else __syncthreads();
}

// Entries of the per-pass twiddle table of a transform (pass p >= 1 holds
// (R_p - 1) NS_p of them, NS_p the span before the pass), and the offset of
// pass p's entries.
template <template <int> class PL, int N, bool REV>
constexpr int twp_off(int p) {
  using S = PlanSeq<PL, N, REV>;
  int o = 0;
  for (int q = 1; q < p; ++q) o += (S::r(q) - 1) * S::ns(q);
  return o;
}
template <template <int> class PL, int N, bool REV>
constexpr int twp_len() { return twp_off<PL, N, REV>(PlanSeq<PL, N, REV>::np); }

// ---------------------------------------------------------------------------
// tile transform with register input and register output
// ---------------------------------------------------------------------------
// T: float/double; N: length; DIR: -1/+1; REV: reversed radix order;
// MP: pencils; SM, SN: LDS strides of pencil and index; TWS: twiddle stride;
// JF: index-fastest butterfly mapping; NTH: threads; PL: radix plan family;
// LB: barriers between passes order LDS only (see lds_barrier);
// SWZ: XOR-swizzled staging index (see lidx); TWP: the twiddles come from a
// per-pass table (twp_fill) instead of the length-N table.
template <typename T, int N, int DIR, bool REV, int MP, int SM, int SN, int TWS, bool JF, int NTH,
          template <int> class PL = Plan, bool SKEW = false, bool LB = false, int SWZ = 0, bool TWP = false>
struct TileFft {
  // LDS word of element (pencil m, index n).  With SKEW one padding word is
  // inserted every 32 indices, which breaks the power-of-two strides of the
  // Stockham scatters across LDS banks.  Two further layouts:
  //  SWZ 1 (index-fastest tiles of 128 points, pencil stride SM a multiple
  //   of 32): the low five bits of n are XORed with a mask built from the
  //   32-entry block h = n / 32 and the pencil's parity e, bits 0-1 <- h,
  //   bits 2-3 <- (h0 ^ e, h1), bit 4 <- h0 ^ e.  n stays inside its block
  //   (a permutation of the pencil), and every gather and scatter of the
  //   radix-4 and radix-8 passes then touches 32 distinct banks per 32
  //   consecutive lanes: a radix-R scatter writes R-strided or NS-grouped
  //   indices, whose blocks h the mask spreads over different low bits, and
  //   a radix-8 pass spans two pencils per 32 lanes, which e separates.
  //  SWZ 2 (pencil-fastest tiles, rows of SN >= MP words): index n lives in
  //   row n + n / 8, one padding row after every 8.  A wave's lanes hold
  //   several consecutive butterflies j, whose first-pass scatters write
  //   rows R apart (R = 4, 8): with rows a power of two of words long those
  //   land on the same banks, and the shifted rows spread them (modelled
  //   bank conflicts of the 8- and 16-pencil tiles' exchanges drop from
  //   about 45 % to 10-20 %).  Every offset stays a compile-time constant
  //   plus a per-butterfly base.
  __device__ static __forceinline__ int lidx(int m, int n) {
    if constexpr (SWZ == 1) {
      const int h0 = (n >> 5) & 1, h1 = (n >> 6) & 1, e = h0 ^ (m & 1);
      return m * SM + (n ^ (h0 | (h1 << 1) | (e << 2) | (h1 << 3) | (e << 4))) * SN;
    } else if constexpr (SWZ == 2) {
      return m * SM + (n + (n >> 3)) * SN;
    } else {
      return m * SM + n * SN + (SKEW ? (n >> 5) : 0);
    }
  }
  // LDS rows (index slots) the layout spans
  static constexpr int ROWS = (SWZ == 2) ? N + (N - 1) / 8 + 1 : N;
  // SWZ 2: row of index n.  A pass touches indices base + r st (r < R):
  // gathers base j < N / R with st = N / R, scatters base
  // (j / NS) NS R + j % NS with st = NS.  When row(base + r st) - row(base)
  // equals row(r st) for every base (no base carries into bit 3 by adding
  // r st), the row is formed once per butterfly and the R elements sit at
  // compile-time offsets from it; checked here over every base.
  static constexpr int row(int n) { return n + (n >> 3); }
  template <int R, int NS, bool SCAT>
  static constexpr bool uniform_rows() {
    if (SWZ != 2) return false;
    const int nb = N / R, st = SCAT ? NS : nb;
    for (int j = 0; j < nb; ++j) {
      const int base = SCAT ? (j / NS) * NS * R + j % NS : j;
      for (int r = 0; r < R; ++r)
        if (row(base + r * st) - row(base) != row(r * st)) return false;
    }
    return true;
  }
  static_assert(SWZ != 1 || (JF && SM % 32 == 0 && N == 128), "swizzled index-fastest layout");
  static_assert(SWZ != 2 || (!JF && SM == 1 && SN >= MP), "padded pencil-fastest layout");
  using S = PlanSeq<PL, N, REV>;
  static constexpr int TWPL = twp_len<PL, N, REV>();
  // Fill the per-pass table (TWPL entries) from the length-N table read with
  // stride TWS: entry twp_off(p) + (r - 1) NS_p + k = w^(r k N / (NS_p R_p)).
  // Consecutive butterflies of an index-fastest tile then read consecutive
  // entries instead of entries r k N / (NS_p R_p) apart.
  __device__ static void twp_fill(T* dr, T* di, const T* twr, const T* twi, int tid) {
    for (int e = tid; e < TWPL; e += NTH) {
      int p = 1, o = 0;
      while (p < S::np - 1 && e >= o + (S::r(p) - 1) * S::ns(p)) {
        o += (S::r(p) - 1) * S::ns(p);
        ++p;
      }
      const int ns = S::ns(p), R = S::r(p);
      const int r = (e - o) / ns + 1, k = (e - o) - (r - 1) * ns;
      const int t = r * k * (N / (ns * R)) * TWS;
      dr[e] = twr[t];
      di[e] = twi[t];
    }
  }
  static constexpr int np = S::np;
  static constexpr int R0 = S::first();
  static constexpr int RL = S::last();
  static constexpr int TOT0 = MP * (N / R0);
  static constexpr int TOTL = MP * (N / RL);
  static constexpr int B0 = (TOT0 + NTH - 1) / NTH;   // butterflies per thread, first pass
  static constexpr int BL = (TOTL + NTH - 1) / NTH;   // last pass

  // butterfly -> (pencil, index)
  template <int R>
  __device__ static __forceinline__ void bj(int b, int& m, int& j) {
    constexpr int NB = N / R;
    if constexpr (JF) { m = b / NB; j = b - m * NB; }
    else { m = b % MP; j = b / MP; }
  }
  // first-pass input position r of butterfly (m, j): index j + r N/R0
  template <int R>
  __device__ static __forceinline__ int in_idx(int j, int r) { return j + r * (N / R); }

  template <int P>
  __device__ static __forceinline__ void twiddle(T* vr, T* vi, int j, const T* twr, const T* twi) {
    constexpr int R = S::r(P), NS = S::ns(P);
    if constexpr (NS > 1) {
      constexpr int TSTEP = N / (NS * R);
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const int t = TWP ? twp_off<PL, N, REV>(P) + (r - 1) * NS + k : r * k * TSTEP * TWS;
        const T wr = twr[t];
        const T wi = (DIR < 0) ? twi[t] : -twi[t];
        cmul(vr[r], vi[r], wr, wi);
      }
    }
  }

  template <int P>
  __device__ static __forceinline__ void scatter_pass(T (&vr)[(MP * N / S::r(P) + NTH - 1) / NTH][S::r(P)],
                                                      T (&vi)[(MP * N / S::r(P) + NTH - 1) / NTH][S::r(P)],
                                                      T* re, T* im, const T* twr, const T* twi, int tid) {
    constexpr int R = S::r(P), NS = S::ns(P), TOT = MP * (N / R), BPT = (TOT + NTH - 1) / NTH;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int b = tid + q * NTH;
      if (TOT % NTH == 0 || b < TOT) {
        int m, j;
        bj<R>(b, m, j);
        twiddle<P>(vr[q], vi[q], j, twr, twi);
        bfly<T, R, DIR>(vr[q], vi[q]);
        const int base = (j / NS) * NS * R + (j % NS);
        if constexpr (uniform_rows<R, NS, true>()) {
          const int i0 = lidx(m, base);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            re[i0 + row(r * NS) * SN] = vr[q][r];
            im[i0 + row(r * NS) * SN] = vi[q][r];
          }
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int idx = lidx(m, base + r * NS);
            re[idx] = vr[q][r];
            im[idx] = vi[q][r];
          }
        }
      }
    }
  }

  template <int P>
  __device__ static __forceinline__ void gather_pass(T (&vr)[(MP * N / S::r(P) + NTH - 1) / NTH][S::r(P)],
                                                     T (&vi)[(MP * N / S::r(P) + NTH - 1) / NTH][S::r(P)],
                                                     const T* re, const T* im, int tid) {
    constexpr int R = S::r(P), TOT = MP * (N / R), BPT = (TOT + NTH - 1) / NTH;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int b = tid + q * NTH;
      if (TOT % NTH == 0 || b < TOT) {
        int m, j;
        bj<R>(b, m, j);
        if constexpr (uniform_rows<R, 1, false>()) {
          const int i0 = lidx(m, j);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            vr[q][r] = re[i0 + row(r * (N / R)) * SN];
            vi[q][r] = im[i0 + row(r * (N / R)) * SN];
          }
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int idx = lidx(m, j + r * (N / R));
            vr[q][r] = re[idx];
            vi[q][r] = im[idx];
          }
        }
      }
    }
  }

  template <int P>
  __device__ static __forceinline__ void compute_pass(T (&vr)[(MP * N / S::r(P) + NTH - 1) / NTH][S::r(P)],
                                                      T (&vi)[(MP * N / S::r(P) + NTH - 1) / NTH][S::r(P)],
                                                      const T* twr, const T* twi, int tid) {
    constexpr int R = S::r(P), NS = S::ns(P), TOT = MP * (N / R), BPT = (TOT + NTH - 1) / NTH;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int b = tid + q * NTH;
      if (TOT % NTH == 0 || b < TOT) {
        int m, j;
        bj<R>(b, m, j);
        twiddle<P>(vr[q], vi[q], j, twr, twi);
        bfly<T, R, DIR>(vr[q], vi[q]);
      }
    }
  }

  // Whole transform.  `in` holds first-pass inputs (position j + r N/R0 of
  // butterfly tid + q NTH), `out` receives last-pass outputs (position
  // j + r N/RL).  Uses LDS (re, im) as staging; contains the barriers it
  // needs between its own passes.  The caller must make sure no thread still
  // reads (re, im) from a previous use when this starts (alternating two
  // buffers between consecutive transforms is enough when np >= 2).
  __device__ static __forceinline__ void run(T (&in_r)[B0][R0], T (&in_i)[B0][R0],
                                             T (&out_r)[BL][RL], T (&out_i)[BL][RL],
                                             T* re, T* im, const T* twr, const T* twi, int tid) {
    if constexpr (np == 1) {
      compute_pass<0>(in_r, in_i, twr, twi, tid);
#pragma unroll
      for (int q = 0; q < BL; ++q)
#pragma unroll
        for (int r = 0; r < RL; ++r) { out_r[q][r] = in_r[q][r]; out_i[q][r] = in_i[q][r]; }
    } else if constexpr (np == 2) {
      scatter_pass<0>(in_r, in_i, re, im, twr, twi, tid);
      tile_sync<LB>();
      gather_pass<1>(out_r, out_i, re, im, tid);
      compute_pass<1>(out_r, out_i, twr, twi, tid);
    } else {
      scatter_pass<0>(in_r, in_i, re, im, twr, twi, tid);
      tile_sync<LB>();
      {
        constexpr int R1 = S::r(1), BP1 = (MP * (N / R1) + NTH - 1) / NTH;
        T mr[BP1][R1], mi[BP1][R1];
        gather_pass<1>(mr, mi, re, im, tid);
        tile_sync<LB>();
        scatter_pass<1>(mr, mi, re, im, twr, twi, tid);
      }
      tile_sync<LB>();
      gather_pass<2>(out_r, out_i, re, im, tid);
      compute_pass<2>(out_r, out_i, twr, twi, tid);
    }
  }
};

}  // namespace lsfft
