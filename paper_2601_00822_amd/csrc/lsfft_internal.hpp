// Internal structures shared by the host orchestration and the HIP kernels.
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

namespace lsfft {

constexpr int kMaxPhases = 256;      // phase ids are uint8
constexpr int kMaxLen = 256;         // longest supported axis

// Supported axis lengths (products of 2 and 3, even).  The twiddle table holds
// exp(-2 pi i k / L) for k < L for each of them, back to back in this order.
constexpr int kNumLens = 12;
__host__ __device__ constexpr int len_at(int i) {
  return i == 0 ? 4 : i == 1 ? 6 : i == 2 ? 8 : i == 3 ? 12 : i == 4 ? 16 : i == 5 ? 24
       : i == 6 ? 32 : i == 7 ? 48 : i == 8 ? 64 : i == 9 ? 96 : i == 10 ? 128 : 256;
}
__host__ __device__ constexpr int tw_offset(int L) {
  int off = 0;
  for (int i = 0; i < kNumLens; ++i) {
    if (len_at(i) == L) return off;
    off += len_at(i);
  }
  return -1;
}
__host__ __device__ constexpr int tw_total() {
  int off = 0;
  for (int i = 0; i < kNumLens; ++i) off += len_at(i);
  return off;
}

// Per-instance lifecycle (device-side, read by every pass kernel).
enum InstStatus : int {
  ST_RUNNING = 2,
  ST_OK = 0,
  ST_STAGNATED = 1,
  ST_NOCONV = -4,
  ST_DIVERGED = -6,
};

// Modes of the pass kernels.
enum PassMode : int {
  M_INIT = 0,    // transform the force, project, free term u^b = N0 f^
  M_ITER = 1,    // one basic-scheme iteration
  M_MAT = 2,     // materialize u, eps, sigma from the state
  M_CG_AP = 3,   // CG: q = A p (forward half) and p.q partials
  M_CG_UPD = 4,  // CG: u += alpha p, r -= alpha q, z = N0 r, r.z partials
  M_CG_DIR = 5,  // CG: p = z + beta p, eps^(p) and its inverse transform
  M_CG_INIT = 6, // CG: r0 = f^ - A u0 from the first operator pass, z0, p0 = z0
  M_FT = 7,      // force transform: R2C along x, y, then the outer axis and projection
  M_AA_RES = 8,  // Anderson: residual, F = N0 r, newest differences, window inner products
  M_AA_UPD = 9,  // Anderson: mixed update of the state and its strain spectrum
  M_KCONV = 10,  // strain spectrum = kernel spectrum x force spectrum, inverse outer transforms
};

// Anderson acceleration: largest memory, and the per-item partial sums of
// M_AA_RES (the residual, then <dF_j, dF_new> and <dF_j, F> for j < kAAMax)
constexpr int kAAMax = 8;
constexpr int kAAPart = 1 + 2 * kAAMax;

// One solve.  All pointers are device pointers; real and complex buffers are
// stored in the plan precision (float or double), complex interleaved.
//
// Spectral layout ("packed half spectrum"): component c of a spectral buffer
// starts at c * Pc and holds the modes kx = 0 .. H-1 (H = nx / 2) as a
// [nz][ny][H] block of Pc = Pm complex entries.  The planes kx = 0 and
// kx = H of a real field are both real after the x transform and both have
// xi_x = 0, so they share the kx = 0 column as Z = F_0 + i F_H: the y and
// outer transforms, the Green operator and the strain map are complex-linear
// and identical on the two planes, and over +k and -k the cross terms of
// |Z|^2 cancel, so the column carries Parseval weight 1.  Rows are H entries
// long, so every tile of the strided passes is full.
struct InstDesc {
  int dim;             // 2 or 3
  int nx, ny, nz;      // nz = 1 in 2D
  int H;               // nx / 2
  int ncomp_s;         // strain components: 3 (2D) or 6 (3D)
  int xtiles;          // x-pass row tiles (work items = row tiles x component groups)
  int items_y;         // y-pass tiles per component
  int mpk_y, lg_y, ntk_y;  // y tiles: kx pencils per tile, log2, kx tiles per plane
  int items_g;         // outer-pass tiles
  int mpk_g, lg_g, ntk_g;  // outer tiles: kx pencils per tile, log2, kx tiles per line
  int items_cg;        // CG update items
  int nphase;
  int lame_off;        // offset (in pairs) into the device Lame table
  int sx, sy, sz;      // microstructure shift: phase read at (x - s) mod n
  int max_iter;
  int group;           // averaging group, -1 if none
  int precond;         // CG: 1 = preconditioned by N0, 0 = plain (Algorithm 3)
  int cg_start;        // CG: 1 = Algorithm 3's printed start u1 = b^A
  int aa_m;            // Anderson memory (1..kAAMax), 0 = not Anderson
  int blk;             // 3D, nx a multiple of 16: kx-blocked layout of S2 (see S2)
  int bls;             // blocked: entries between consecutive y lines of a block (8 nz)
  long long Pm, Pc;    // complex entries: main block, component stride
  long long nvox;      // nx * ny * nz
  double kx, ky, kz;   // 2 pi / (n h) per axis
  double inv_nvox;
  double lam0, mu0;
  double tol;
  const uint8_t* phase;
  const void* f_in;    // real force [d][nvox]
  void* S;             // spectral work [ncomp_s + d][Pc], rows (z, y) of H entries
  // With blk, the spectra between the y passes and the outer pass (stress
  // after the forward y transforms, strain and displacement before the
  // inverse ones, the force before its outer transform) live here instead,
  // kx-blocked: entry (kx, y, z) at ((kx / 8) ny + y) bls + 8 z + kx % 8,
  // so that an outer-pass tile reads and writes whole 8 x nz blocks; the y
  // passes convert between the two layouts (out of place).  The other
  // spectral buffers that only the outer pass and the element-wise kernels
  // touch (state, force, search directions, Anderson history) take the
  // same layout.
  void* S2;            // [ncomp_s + d][Pc] or null
  void* U[2];          // displacement spectrum, double-buffered [d][Pc]
  void* F;             // force spectrum [d][Pc] (may be shared)
  void* R;             // CG residual [d][Pc]
  void* Pd;            // CG direction [d][Pc]
  void* Q;             // CG A p [d][Pc]
  void* Fp;            // Anderson: F of the previous iteration [d][Pc]
  void* DF;            // Anderson: ring of F differences [aa_m][d][Pc]
  void* DU;            // Anderson: ring of state differences [aa_m][d][Pc]
  double* aa;          // Anderson: Gram matrix [aa_m][aa_m] by ring slot, then the coefficients [aa_m]
  const void* Kh;      // kernel convolution: half spectrum of the kernel [s][d][Pc]
  void* out_eps;       // real [s][nvox] or null
  void* out_sig;       // real [s][nvox] or null
  void* out_u;         // real [d][nvox] or null
  double* partial;     // per work item FP64 partial sums [max items][2]
  double* history;     // optional residual history [max_iter + 2] or null
};

struct InstState {
  int iter;
  int status;
  int done;            // reserved
  int start_step;      // CG: 1 while the forced step of the printed start runs
  int mark_iter;       // iteration of the last >= 1% improvement
  int grow;            // consecutive iterations with a growing residual
  double residual;
  double fnorm2;
  double mark;         // residual at mark_iter
  double prev;
  double removed_mean[3];
  double rz;           // CG: r.z of the current iterate
  double alpha;
  double beta;
  double pq;
};

struct WorkItem {
  int inst;
  int local;
};

// Averaging group: solves of one (microstructure, force) pair over shifts.
struct GroupDesc {
  int first;           // first instance index of the group in the batch
  int count;           // number of instances (shifts) of the group
  int incl_phase;
  int pad;
  double* avg;         // [2d + 4s + 1][nvox] FP64 accumulator
};

}  // namespace lsfft
