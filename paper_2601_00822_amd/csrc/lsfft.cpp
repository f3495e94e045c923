// Host side of liblsfft: plans, argument validation, workspace, batch
// scheduling of the pass kernels, convergence polling and reports.
#include "../../include/lsfft.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "launch.hpp"
#include "lsfft_internal.hpp"

using namespace lsfft;

namespace {

constexpr int kMaxGrid = 4096;  // blocks of a persistent launch

bool supported_len(int64_t n) {
  for (int i = 0; i < kNumLens; ++i)
    if (len_at(i) == n) return true;
  return false;
}

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool ensure(size_t bytes) {
    if (bytes <= cap) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
      return false;
    }
    cap = bytes;
    return true;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

// Page-locked host mirror of the plan's metadata buffer: descriptors, states,
// tables, counts and work lists are staged here at the offsets they occupy
// on the device, so an upload is one asynchronous copy per contiguous range.
struct HostBuf {
  char* p = nullptr;
  size_t cap = 0;
  bool ensure(size_t bytes) {
    if (bytes <= cap) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    void* q = nullptr;
    if (hipHostMalloc(&q, bytes, hipHostMallocDefault) != hipSuccess) return false;
    p = static_cast<char*>(q);
    cap = bytes;
    return true;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
};

// One solve of a batch, as resolved on the host.
struct Spec {
  int grid = 0;
  const uint8_t* phase = nullptr;
  const lsfft_phases* tab = nullptr;
  double lam0 = 0, mu0 = 0;
  const void* f = nullptr;
  const void* u_init = nullptr;   // optional starting displacement (real, [d][N])
  void* eps = nullptr;
  void* sig = nullptr;
  void* u = nullptr;
  int shift[3] = {0, 0, 0};
  int group = -1;     // index into the batch's groups
  int leader = -1;    // solve that owns the force spectrum (itself if own)
  int out_index = 0;  // report slot
};

struct BatchGroup {
  double* avg = nullptr;
  int incl_phase = 1;
  int first = 0, count = 0;
};

enum ListId { L_XLEAD, L_YLEAD, L_GLEAD, L_X, L_Y, L_G, L_CG, L_XALL, L_YALL, L_GALL, L_NUM };

// A contiguous run of work items of one list that share the kernel
// specialization (dimension and transform length) and therefore one launch.
struct Seg {
  int dim = 0, len = 0;
  int var = 0;         // schedule variant of the pass kernel
  int off = 0, cap = 0, count = 0;
  size_t lds = 0;
  int cidx = 0;        // slot of its item count in the device count array
};

constexpr int kMaxSegs = 512;

}  // namespace

struct lsfft_plan_s {
  int device = 0;
  hipStream_t ustream = nullptr;  // caller's stream (inputs are ordered on it)
  hipStream_t stream = nullptr;   // plan-owned work stream (capturable)
  hipEvent_t ev_in = nullptr;
  bool graphs = true;
  bool force_timing = false;   // lsfft_autotune: time every launch
  int aa_m = 5;                // Anderson memory (LSFFT_ANDERSON)
  bool f64 = false;
  lsfft_scheme scheme = LSFFT_BASIC;
  unsigned flags = 0;
  std::vector<lsfft_grid> grids;
  int max_batch = 1;
  int poll = 8;
  bool owns_stream = true;
  DevBuf tw, arena, meta, lists;
  HostBuf hmeta;            // host mirror of `meta`
  DevBuf rve;               // radial maxima of lsfft_rve_identify
  DevBuf kspec, zphase;     // lsfft_kernel_convolve: kernel spectrum, all-zero phase map
  bool h2d_inflight = false;  // copies out of `hmeta` may still be queued
  // LSFFT_REFINE64: FP64 companion (same grids, shares the work stream) and
  // the FP64 copies of the forces
  lsfft_plan_s* sub = nullptr;
  DevBuf fwide;
  // timing
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pending;  // (class, index of start event)
  size_t ev_next = 0;
  double kt_ms[LSFFT_K_COUNT] = {0};
  int64_t kt_n[LSFFT_K_COUNT] = {0};
  bool timing_active = false;
  // schedule variant per pass kind (0 x, 1 y, 2 outer) and length index,
  // used by FP32 3D solves (lsfft_autotune, lsfft_schedule_set, the cache)
  int sched[3][kNumLens] = {};
  // spectral layout per grid (index into grids): 1 kx-blocked between the y
  // and outer passes where the grid allows it, 0 rows throughout
  std::vector<int> layout;
};

namespace {

lsfft_status dev_err(hipError_t e) { return e == hipSuccess ? LSFFT_OK : LSFFT_E_DEVICE; }

#define LSFFT_TRY(expr)                          \
  do {                                           \
    hipError_t _e = (expr);                      \
    if (_e != hipSuccess) return LSFFT_E_DEVICE; \
  } while (0)

int grid_dim(const lsfft_grid& g) { return g.dim; }
int64_t gnx(const lsfft_grid& g) { return g.n[0]; }
int64_t gny(const lsfft_grid& g) { return g.n[1]; }
int64_t gnz(const lsfft_grid& g) { return g.dim == 3 ? g.n[2] : 1; }

bool is_fin(double v) { return std::isfinite(v); }

lsfft_status check_table(const lsfft_phases* t, int dim) {
  if (!t || !t->lame || t->nphase < 1 || t->nphase > kMaxPhases) return LSFFT_E_ARG;
  for (int p = 0; p < t->nphase; ++p) {
    const double lam = t->lame[2 * p], mu = t->lame[2 * p + 1];
    if (!is_fin(lam) || !is_fin(mu) || mu <= 0.0 || lam + 2.0 * mu / dim <= 0.0) return LSFFT_E_ARG;
  }
  return LSFFT_OK;
}

// default reference medium: mean of the extreme Lame constants (Algorithm 1 datum)
lsfft_status resolve_ref(const lsfft_phases* t, const lsfft_ref* c0, double* lam0, double* mu0) {
  double lmin = t->lame[0], lmax = t->lame[0], mmin = t->lame[1], mmax = t->lame[1];
  for (int p = 1; p < t->nphase; ++p) {
    lmin = std::min(lmin, t->lame[2 * p]);
    lmax = std::max(lmax, t->lame[2 * p]);
    mmin = std::min(mmin, t->lame[2 * p + 1]);
    mmax = std::max(mmax, t->lame[2 * p + 1]);
  }
  if (c0 && !(std::isnan(c0->lambda0) && std::isnan(c0->mu0))) {
    if (!is_fin(c0->lambda0) || !is_fin(c0->mu0) || c0->mu0 <= 0.0 || c0->lambda0 + 2.0 * c0->mu0 <= 0.0)
      return LSFFT_E_ARG;
    *lam0 = c0->lambda0;
    *mu0 = c0->mu0;
  } else {
    *lam0 = 0.5 * (lmin + lmax);
    *mu0 = 0.5 * (mmin + mmax);
  }
  return LSFFT_OK;
}

struct Geometry {
  int nx, ny, nz, H, dim, s;
  int var_x, var_y, var_g;   // schedule variants of the three passes
  long long Pm, Pc, nvox;
  int xtiles, items_x, items_xall, items_xft, items_y, mpk_y, ntk_y, items_g, mpk_g, ntk_g, items_cg;
  int blk;                              // kx-blocked spectra between the y and outer passes
  int bls;                              // blocked: entries from one y line of a block to the next (8 nz)
  size_t lds_x, lds_xi, lds_y, lds_g;   // lds_xi: x pass of the iteration
};

// the kx-blocked layout needs a 3D grid with nx a multiple of 16
bool blocked_layout_ok(const lsfft_grid& g) { return g.dim == 3 && gnx(g) % 16 == 0; }

int ilog2(int v) {
  int l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}

// largest power of two <= mp that divides h
int kx_pencils(int mp, int h) {
  int k = 1;
  while (k * 2 <= mp && h % (k * 2) == 0) k *= 2;
  return k;
}

int len_index(int L) {
  for (int i = 0; i < kNumLens; ++i)
    if (len_at(i) == L) return i;
  return -1;
}

// schedule variant of pass `kind` on an axis of `len` points in a plan
int plan_variant(const int sched[3][kNumLens], bool f64, int dim, int kind, int len) {
  const int i = len_index(len);
  if (i < 0) return 0;
  const int v = sched[kind][i];
  return (v > 0 && v < schedule_variants(f64, dim, kind, len)) ? v : 0;
}

bool geometry(bool f64, const lsfft_grid& g, const int sched[3][kNumLens], Geometry* o, int layout) {
  o->dim = g.dim;
  o->nx = (int)gnx(g);
  o->ny = (int)gny(g);
  o->nz = (int)gnz(g);
  o->H = o->nx / 2;
  o->s = g.dim == 3 ? 6 : 3;
  // kx = 0 and kx = H share one column (packed half spectrum): no Nyquist plane
  o->Pm = (long long)o->nz * o->ny * o->H;
  o->blk = (layout == 1 && blocked_layout_ok(g)) ? 1 : 0;
  o->bls = o->blk ? 8 * o->nz : 0;
  o->Pc = o->Pm;
  o->nvox = (long long)o->nz * o->ny * o->nx;
  int mr = 0, mpy = 0, mpg = 0;
  const int outer = (g.dim == 3) ? o->nz : o->ny;
  o->var_x = plan_variant(sched, f64, g.dim, 0, o->nx);
  o->var_y = (g.dim == 3) ? plan_variant(sched, f64, g.dim, 1, o->ny) : 0;
  o->var_g = plan_variant(sched, f64, g.dim, 2, outer);
  o->lds_x = query_geometry(f64, 0, o->nx, o->var_x, &mr);
  o->lds_xi = query_geometry(f64, 3, o->nx, o->var_x, nullptr);
  o->lds_y = (g.dim == 3) ? query_geometry(f64, 1, o->ny, o->var_y, &mpy) : 0;
  o->lds_g = query_geometry(f64, 2, outer, o->var_g, &mpg);
  if (!o->lds_x || !o->lds_xi || !o->lds_g || (g.dim == 3 && !o->lds_y)) return false;
  const int rows = o->ny * o->nz;
  o->xtiles = (rows + mr - 1) / mr;
  o->items_x = o->xtiles * (1 + o->s - o->dim);          // normal group + shear components
  o->items_xall = o->xtiles * (1 + o->s);                 // + displacement components
  o->items_xft = o->xtiles * o->dim;                      // force components
  if (g.dim == 3) {
    // blocked: at most 16 kx per z line, so that both layouts see runs of
    // 128 bytes (FP32) or more
    o->mpk_y = kx_pencils(o->blk ? std::min(mpy, 16) : mpy, o->H);
    const int per = mpy / o->mpk_y;
    o->ntk_y = o->H / o->mpk_y;
    o->items_y = o->ntk_y * ((o->nz + per - 1) / per);
  } else {
    o->mpk_y = 1;
    o->ntk_y = 0;
    o->items_y = 0;
  }
  o->mpk_g = kx_pencils(mpg, o->H);
  o->ntk_g = o->H / o->mpk_g;
  if (g.dim == 3) {
    const int per = mpg / o->mpk_g;
    o->items_g = o->ntk_g * ((o->ny + per - 1) / per);
  } else {
    o->items_g = o->ntk_g;
  }
  const int nth = threads_per_block(f64);
  o->items_cg = (int)((o->Pc + nth * 4 - 1) / (nth * 4));
  return true;
}

// -------------------------------------------------------------------------
// timing helpers
// -------------------------------------------------------------------------
// Reserve an event pair for one timed launch of class `cls`; the launch
// itself stamps the pair at the kernel's start and end.  Returns -1 when
// timing is off.
int timed_begin(lsfft_plan_s* p, int cls) {
  if (!p->timing_active) return -1;
  if (p->ev_next + 2 > p->ev_pool.size()) {
    for (int k = 0; k < 256; ++k) {
      hipEvent_t e;
      // device-scope release: no system-scope cache flush after every timed kernel
      if (hipEventCreateWithFlags(&e, hipEventReleaseToDevice) != hipSuccess) return -1;
      p->ev_pool.push_back(e);
    }
  }
  const int idx = (int)p->ev_next;
  p->ev_next += 2;
  p->ev_pending.push_back({cls, idx});
  return idx;
}
LaunchArgs timed(lsfft_plan_s* p, LaunchArgs a, int idx) {
  if (idx >= 0) {
    a.ev0 = p->ev_pool[idx];
    a.ev1 = p->ev_pool[idx + 1];
  }
  return a;
}
void timed_collect(lsfft_plan_s* p) {
  for (auto& pr : p->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev_pool[pr.second], p->ev_pool[pr.second + 1]) == hipSuccess) {
      p->kt_ms[pr.first] += ms;
      p->kt_n[pr.first] += 1;
    }
  }
  p->ev_pending.clear();
  p->ev_next = 0;
}

// -------------------------------------------------------------------------
// the batch engine
// -------------------------------------------------------------------------
struct Batch {
  lsfft_plan_s* p;
  std::vector<Spec> specs;
  std::vector<BatchGroup> groups;
  std::vector<Geometry> geo;
  std::vector<InstDesc> desc;
  std::vector<InstState> state;
  std::vector<double> lame;
  // device views into plan buffers
  InstDesc* d_desc = nullptr;
  InstState* d_state = nullptr;
  double* d_lame = nullptr;
  GroupDesc* d_groups = nullptr;
  int* d_counts = nullptr;
  int* d_inst = nullptr;
  int* d_phasemax = nullptr;
  WorkItem* d_lists[L_NUM] = {nullptr};
  int list_cap[L_NUM] = {0};
  size_t m_state = 0, m_counts = 0, m_inst = 0, m_pmax = 0, m_list[L_NUM] = {0};   // offsets in meta
  std::vector<Seg> segs[L_NUM];   // per list: one segment per (dim, transform length)
  int nseg_total = 0;
  int n_running = 0;
  double tol = 1e-8;
  int max_iter = 0;
  bool averaging = false;
  // the captured polling round, kept for the batch's lifetime (the inner
  // solves of the defect correction replay it once per outer step)
  struct GraphHolder {
    hipGraphExec_t exec = nullptr;
    GraphHolder() = default;
    GraphHolder(const GraphHolder&) {}              // copies start without a graph
    GraphHolder& operator=(const GraphHolder&) { return *this; }
    ~GraphHolder() { if (exec) (void)hipGraphExecDestroy(exec); }
  } graph;
};

// The host mirror may be rewritten only once the copies queued from it ran.
lsfft_status host_fence(lsfft_plan_s* p) {
  if (p->h2d_inflight) {
    LSFFT_TRY(hipStreamSynchronize(p->stream));
    p->h2d_inflight = false;
  }
  return LSFFT_OK;
}
template <typename V> V* hptr(Batch& b, size_t off) { return reinterpret_cast<V*>(b.p->hmeta.p + off); }
// queue one host-mirror -> device copy of meta bytes [off, off + bytes)
lsfft_status h2d(Batch& b, size_t off, size_t bytes) {
  if (bytes == 0) return LSFFT_OK;
  LSFFT_TRY(hipMemcpyAsync(static_cast<char*>(b.p->meta.p) + off, b.p->hmeta.p + off, bytes, hipMemcpyHostToDevice,
                           b.p->stream));
  b.p->h2d_inflight = true;
  return LSFFT_OK;
}
// device -> host copy of the solve states, then into b.state (synchronizes)
lsfft_status d2h_states(Batch& b) {
  const int n = (int)b.specs.size();
  LSFFT_TRY(hipMemcpyAsync(b.p->hmeta.p + b.m_state, b.d_state, sizeof(InstState) * n, hipMemcpyDeviceToHost,
                           b.p->stream));
  LSFFT_TRY(hipStreamSynchronize(b.p->stream));
  b.p->h2d_inflight = false;
  std::memcpy(b.state.data(), hptr<InstState>(b, b.m_state), sizeof(InstState) * n);
  return LSFFT_OK;
}
// b.state -> device (asynchronous)
lsfft_status h2d_states(Batch& b) {
  const int n = (int)b.specs.size();
  if (host_fence(b.p) != LSFFT_OK) return LSFFT_E_DEVICE;
  std::memcpy(hptr<InstState>(b, b.m_state), b.state.data(), sizeof(InstState) * n);
  return h2d(b, b.m_state, sizeof(InstState) * n);
}

LaunchArgs largs(Batch& b, int list, const Seg& sg, int units = 1) {
  LaunchArgs a;
  const int n = std::max(1, sg.count * units);
  a.grid = dim3((unsigned)std::min(n, kMaxGrid));
  a.block = threads_per_block(b.p->f64);
  a.lds = sg.lds;
  a.stream = b.p->stream;
  a.desc = b.d_desc;
  a.state = b.d_state;
  a.items = b.d_lists[list] + sg.off;
  a.count = b.d_counts + sg.cidx;
  a.lame = b.d_lame;
  a.tw = b.p->tw.p;
  return a;
}

LaunchArgs base_args(Batch& b) {
  LaunchArgs a{};
  a.grid = dim3(1);
  a.block = threads_per_block(b.p->f64);
  a.stream = b.p->stream;
  a.desc = b.d_desc;
  a.state = b.d_state;
  a.lame = b.d_lame;
  a.tw = b.p->tw.p;
  return a;
}

// Work-list key of solve i for list l: the kernel specialization it needs.
void list_key(const Batch& b, int l, int i, int* dim, int* len, int* items, size_t* lds, int* var) {
  const Geometry& g = b.geo[i];
  *dim = g.dim;
  switch (l) {
    case L_X: *len = g.nx; *items = g.items_x; *lds = g.lds_xi; *var = g.var_x; break;
    case L_XALL: *len = g.nx; *items = g.items_xall; *lds = g.lds_x; *var = g.var_x; break;
    case L_XLEAD: *len = g.nx; *items = g.items_xft; *lds = g.lds_x; *var = g.var_x; break;
    case L_Y: case L_YALL: case L_YLEAD: *len = g.ny; *items = g.items_y; *lds = g.lds_y; *var = g.var_y; break;
    case L_G: case L_GALL: case L_GLEAD:
      *len = (g.dim == 3) ? g.nz : g.ny; *items = g.items_g; *lds = g.lds_g; *var = g.var_g; break;
    default: *len = 0; *items = g.items_cg; *lds = 0; *var = 0; break;   // L_CG
  }
}

bool is_dynamic(int l) { return l == L_X || l == L_Y || l == L_G || l == L_CG; }

// Lay out every list as segments (first call), then fill the dynamic lists
// with the items of the running solves (every call) and upload lists and
// counts.  Segment offsets and capacities never change within a batch.
// With all_too the whole range from meta offset `from` (0: descriptors
// onward) to the end of the last list goes up in one copy; otherwise the
// counts with the solve list, and the span of the dynamic lists.
lsfft_status upload_lists(Batch& b, const std::vector<int>& running, bool all_too, size_t from = SIZE_MAX) {
  const int n = (int)b.specs.size();
  if (all_too) {
    int cidx = 0;
    for (int l = 0; l < L_NUM; ++l) {
      b.segs[l].clear();
      int off = 0;
      for (int i = 0; i < n; ++i) {
        if ((l == L_XLEAD || l == L_YLEAD || l == L_GLEAD) && b.specs[i].leader != i) continue;
        int dim, len, items, var;
        size_t lds;
        list_key(b, l, i, &dim, &len, &items, &lds, &var);
        if (items == 0) continue;
        Seg* sg = nullptr;
        for (auto& x : b.segs[l])
          if (x.dim == dim && x.len == len) sg = &x;
        if (!sg) {
          b.segs[l].push_back(Seg{});
          sg = &b.segs[l].back();
          sg->dim = dim;
          sg->len = len;
          sg->var = var;
          sg->cidx = cidx++;
        }
        sg->cap += items;
        sg->lds = std::max(sg->lds, lds);
      }
      for (auto& x : b.segs[l]) {
        x.off = off;
        off += x.cap;
      }
      if (off > b.list_cap[l]) return LSFFT_E_ALLOC;
    }
    if (cidx > kMaxSegs - 1) return LSFFT_E_ALLOC;
    b.nseg_total = cidx;
  }
  if (host_fence(b.p) != LSFFT_OK) return LSFFT_E_DEVICE;
  int* counts = hptr<int>(b, b.m_counts);
  std::fill(counts, counts + kMaxSegs, 0);
  size_t lo_b = SIZE_MAX, hi_b = 0;   // meta byte span of the lists written
  for (int l = 0; l < L_NUM; ++l) {
    if (!all_too && !is_dynamic(l)) {
      for (auto& x : b.segs[l]) counts[x.cidx] = x.count;
      continue;
    }
    WorkItem* items = hptr<WorkItem>(b, b.m_list[l]);
    int lo = b.list_cap[l], hi = 0;   // item range written
    for (auto& x : b.segs[l]) {
      int fill = 0;
      const std::vector<int>* src = &running;
      std::vector<int> all_ids;
      if (!is_dynamic(l)) {
        all_ids.resize(n);
        for (int i = 0; i < n; ++i) all_ids[i] = i;
        src = &all_ids;
      }
      for (int i : *src) {
        if ((l == L_XLEAD || l == L_YLEAD || l == L_GLEAD) && b.specs[i].leader != i) continue;
        int dim, len, cnt, var;
        size_t lds;
        list_key(b, l, i, &dim, &len, &cnt, &lds, &var);
        if (cnt == 0 || dim != x.dim || len != x.len) continue;
        for (int k = 0; k < cnt; ++k) items[x.off + fill + k] = WorkItem{i, k};
        fill += cnt;
      }
      x.count = fill;
      counts[x.cidx] = fill;
      if (fill > 0) {
        lo = std::min(lo, x.off);
        hi = std::max(hi, x.off + fill);
      }
    }
    if (hi > lo) {
      lo_b = std::min(lo_b, b.m_list[l] + sizeof(WorkItem) * (size_t)lo);
      hi_b = std::max(hi_b, b.m_list[l] + sizeof(WorkItem) * (size_t)hi);
    }
  }
  int* inst = hptr<int>(b, b.m_inst);
  for (size_t k = 0; k < running.size(); ++k) inst[k] = running[k];
  counts[kMaxSegs - 1] = (int)running.size();   // solves listed for the reduction
  b.n_running = (int)running.size();
  // counts and the solve list are adjacent in the metadata buffer, and the
  // lists follow them
  const size_t end_inst = b.m_inst + sizeof(int) * running.size();
  if (all_too) {
    const size_t lo = std::min(from, b.m_counts);
    return h2d(b, lo, std::max(hi_b, end_inst) - lo);
  }
  lsfft_status ls = h2d(b, b.m_counts, end_inst - b.m_counts);
  if (ls == LSFFT_OK && hi_b > lo_b) ls = h2d(b, lo_b, hi_b - lo_b);
  return ls;
}

// Largest half-spectrum size among the listed solves (grid of the
// defect-correction kernels).
long long max_pc(const Batch& b, const std::vector<int>& ids) {
  long long m = 1;
  for (int i : ids) m = std::max(m, (long long)b.geo[i].Pc);
  return m;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Workspace layout, descriptors, Lame tables, phase validation and the
// initial work lists of a batch.
lsfft_status prepare(Batch& b, bool validate = true) {
  lsfft_plan_s* p = b.p;
  const bool f64 = p->f64;
  const size_t rs = f64 ? 8 : 4;   // real scalar
  const size_t cs = 2 * rs;        // complex scalar
  const int n = (int)b.specs.size();
  const bool cg = p->scheme == LSFFT_CG || p->scheme == LSFFT_CG_PLAIN;

  if (host_fence(p) != LSFFT_OK) return LSFFT_E_DEVICE;
  // geometry, Lame tables
  b.geo.resize(n);
  b.desc.assign(n, InstDesc{});
  b.state.assign(n, InstState{});
  b.lame.clear();
  for (int i = 0; i < n; ++i) {
    if (!geometry(f64, p->grids[b.specs[i].grid], p->sched, &b.geo[i], p->layout[b.specs[i].grid])) return LSFFT_E_ARG;
  }

  // workspace layout
  size_t off = 0;
  const bool aa = p->scheme == LSFFT_ANDERSON;
  const int aam = aa ? p->aa_m : 0;
  std::vector<size_t> o_S(n), o_U0(n), o_U1(n), o_F(n), o_R(n), o_P(n), o_Q(n), o_oe(n), o_ou(n), o_part(n), o_hist(n);
  std::vector<size_t> o_Fp(n), o_DF(n), o_DU(n), o_aa(n), o_S2(n);
  for (int i = 0; i < n; ++i) {
    const Geometry& g = b.geo[i];
    const size_t comp = (size_t)g.Pc * cs;
    o_S[i] = off; off = align_up(off + comp * (g.s + g.dim));
    if (g.blk) { o_S2[i] = off; off = align_up(off + comp * (g.s + g.dim)); }
    o_U0[i] = off; off = align_up(off + comp * g.dim);
    if (!cg) { o_U1[i] = off; off = align_up(off + comp * g.dim); }
    if (b.specs[i].leader == i) { o_F[i] = off; off = align_up(off + comp * g.dim); }
    if (cg) {
      o_R[i] = off; off = align_up(off + comp * g.dim);
      o_P[i] = off; off = align_up(off + comp * g.dim);
      o_Q[i] = off; off = align_up(off + comp * g.dim);
    }
    if (b.averaging) {
      o_oe[i] = off; off = align_up(off + (size_t)g.nvox * rs * g.s);
      o_ou[i] = off; off = align_up(off + (size_t)g.nvox * rs * g.dim);
    }
    if (aa) {
      o_Fp[i] = off; off = align_up(off + comp * g.dim);
      o_DF[i] = off; off = align_up(off + comp * g.dim * aam);
      o_DU[i] = off; off = align_up(off + comp * g.dim * aam);
      o_aa[i] = off; off = align_up(off + sizeof(double) * (size_t)(aam * aam + aam));
    }
    const size_t per_item = aa ? kAAPart : 2;
    o_part[i] = off; off = align_up(off + sizeof(double) * per_item * (size_t)std::max(g.items_g, g.items_cg));
    o_hist[i] = off; off = align_up(off + sizeof(double) * ((size_t)b.max_iter + 2));
  }
  if (!p->arena.ensure(off)) return LSFFT_E_ALLOC;
  char* A = static_cast<char*>(p->arena.p);

  // metadata buffer: desc, state, lame, groups, counts, inst list, phase max, lists
  int list_need[L_NUM] = {0};
  for (int i = 0; i < n; ++i) {
    const Geometry& g = b.geo[i];
    list_need[L_X] += g.items_x; list_need[L_Y] += g.items_y; list_need[L_G] += g.items_g;
    list_need[L_CG] += g.items_cg;
  }
  if (list_need[L_X] == 0) list_need[L_X] = 1;
  list_need[L_XALL] = list_need[L_XLEAD] = 0;
  for (int i = 0; i < n; ++i) {
    list_need[L_XALL] += b.geo[i].items_xall;
    list_need[L_XLEAD] += b.geo[i].items_xft;
  }
  list_need[L_YALL] = list_need[L_YLEAD] = list_need[L_Y];
  list_need[L_GALL] = list_need[L_GLEAD] = list_need[L_G];
  size_t total_lame = 0;
  for (int i = 0; i < n; ++i) total_lame += 2 * (size_t)b.specs[i].tab->nphase;
  size_t moff = 0;
  const size_t m_desc = moff; moff = align_up(moff + sizeof(InstDesc) * n);
  const size_t m_state = moff; moff = align_up(moff + sizeof(InstState) * n);
  const size_t m_lame = moff; moff = align_up(moff + sizeof(double) * total_lame);
  const size_t m_groups = moff; moff = align_up(moff + sizeof(GroupDesc) * std::max<size_t>(1, b.groups.size()));
  const size_t m_counts = moff; moff = align_up(moff + sizeof(int) * kMaxSegs);
  const size_t m_inst = moff; moff = align_up(moff + sizeof(int) * n);
  const size_t m_pmax = moff; moff = align_up(moff + sizeof(int) * n);
  size_t m_list[L_NUM];
  for (int l = 0; l < L_NUM; ++l) {
    m_list[l] = moff;
    moff = align_up(moff + sizeof(WorkItem) * std::max(1, list_need[l]));
  }
  if (!p->meta.ensure(moff) || !p->hmeta.ensure(moff)) return LSFFT_E_ALLOC;
  char* M = static_cast<char*>(p->meta.p);
  b.m_state = m_state;
  b.m_counts = m_counts;
  b.m_inst = m_inst;
  b.m_pmax = m_pmax;
  for (int l = 0; l < L_NUM; ++l) b.m_list[l] = m_list[l];
  b.d_desc = reinterpret_cast<InstDesc*>(M + m_desc);
  b.d_state = reinterpret_cast<InstState*>(M + m_state);
  b.d_lame = reinterpret_cast<double*>(M + m_lame);
  b.d_groups = reinterpret_cast<GroupDesc*>(M + m_groups);
  b.d_counts = reinterpret_cast<int*>(M + m_counts);
  b.d_inst = reinterpret_cast<int*>(M + m_inst);
  b.d_phasemax = reinterpret_cast<int*>(M + m_pmax);
  for (int l = 0; l < L_NUM; ++l) {
    b.d_lists[l] = reinterpret_cast<WorkItem*>(M + m_list[l]);
    b.list_cap[l] = std::max(1, list_need[l]);
  }

  // descriptors
  for (int i = 0; i < n; ++i) {
    const Spec& sp = b.specs[i];
    const Geometry& g = b.geo[i];
    const lsfft_grid& gr = p->grids[sp.grid];
    InstDesc& D = b.desc[i];
    D.dim = g.dim; D.nx = g.nx; D.ny = g.ny; D.nz = g.nz; D.H = g.H; D.ncomp_s = g.s;
    D.xtiles = g.xtiles; D.items_y = g.items_y;
    D.mpk_y = g.mpk_y; D.lg_y = ilog2(g.mpk_y); D.ntk_y = g.ntk_y;
    D.items_g = g.items_g;
    D.mpk_g = g.mpk_g; D.lg_g = ilog2(g.mpk_g); D.ntk_g = g.ntk_g;
    D.items_cg = g.items_cg;
    D.nphase = sp.tab->nphase;
    D.lame_off = (int)(b.lame.size() / 2);
    for (int q = 0; q < 2 * sp.tab->nphase; ++q) b.lame.push_back(sp.tab->lame[q]);
    D.sx = sp.shift[0]; D.sy = sp.shift[1]; D.sz = sp.shift[2];
    D.max_iter = b.max_iter;
    D.group = sp.group;
    D.precond = (p->scheme == LSFFT_CG_PLAIN) ? 0 : 1;
    D.cg_start = (p->scheme == LSFFT_CG_PLAIN) ? 1 : 0;
    D.aa_m = aam;
    D.Fp = aa ? (void*)(A + o_Fp[i]) : nullptr;
    D.DF = aa ? (void*)(A + o_DF[i]) : nullptr;
    D.DU = aa ? (void*)(A + o_DU[i]) : nullptr;
    D.aa = aa ? reinterpret_cast<double*>(A + o_aa[i]) : nullptr;
    D.Pm = g.Pm; D.Pc = g.Pc; D.nvox = g.nvox;
    const double two_pi = 6.283185307179586476925286766559;
    D.kx = two_pi / (g.nx * gr.h[0]);
    D.ky = two_pi / (g.ny * gr.h[1]);
    D.kz = (g.dim == 3) ? two_pi / (g.nz * gr.h[2]) : 0.0;
    D.inv_nvox = 1.0 / (double)g.nvox;
    D.lam0 = sp.lam0; D.mu0 = sp.mu0;
    D.tol = b.tol;
    D.phase = sp.phase;
    D.f_in = sp.f;
    D.S = A + o_S[i];
    D.blk = g.blk;
    D.bls = g.bls;
    D.S2 = g.blk ? (void*)(A + o_S2[i]) : nullptr;
    D.U[0] = A + o_U0[i];
    D.U[1] = cg ? D.U[0] : (void*)(A + o_U1[i]);
    D.F = A + o_F[sp.leader];
    D.R = cg ? (void*)(A + o_R[i]) : nullptr;
    D.Pd = cg ? (void*)(A + o_P[i]) : nullptr;
    D.Q = cg ? (void*)(A + o_Q[i]) : nullptr;
    if (b.averaging) {
      D.out_eps = A + o_oe[i];
      D.out_sig = nullptr;
      D.out_u = A + o_ou[i];
    } else {
      D.out_eps = sp.eps; D.out_sig = sp.sig; D.out_u = sp.u;
    }
    D.partial = reinterpret_cast<double*>(A + o_part[i]);
    D.history = reinterpret_cast<double*>(A + o_hist[i]);
    InstState& S = b.state[i];
    S.status = ST_RUNNING;
    S.iter = 0;
  }
  hipStream_t st = p->stream;
  // descriptors, states, Lame tables and groups: one copy of their range
  char* H = p->hmeta.p;
  std::memcpy(H + m_desc, b.desc.data(), sizeof(InstDesc) * n);
  std::memcpy(H + m_state, b.state.data(), sizeof(InstState) * n);
  if (!b.lame.empty()) std::memcpy(H + m_lame, b.lame.data(), sizeof(double) * b.lame.size());
  GroupDesc* gd = hptr<GroupDesc>(b, m_groups);
  for (size_t g = 0; g < b.groups.size(); ++g)
    gd[g] = GroupDesc{b.groups[g].first, b.groups[g].count, b.groups[g].incl_phase, 0, b.groups[g].avg};

  // phase ids must index the tables: one device max per distinct map (the
  // inner batch of the defect correction reuses the companion's maps)
  if (validate) {
  LSFFT_TRY(hipMemsetAsync(b.d_phasemax, 0, sizeof(int) * n, st));
  for (int i = 0; i < n; ++i) {
    bool seen = false;
    for (int j = 0; j < i && !seen; ++j) seen = (b.specs[j].phase == b.specs[i].phase && b.geo[j].nvox == b.geo[i].nvox);
    if (!seen) LSFFT_TRY(launch_phase_max(b.specs[i].phase, b.geo[i].nvox, b.d_phasemax + i, st));
  }
  LSFFT_TRY(hipMemcpyAsync(H + m_pmax, b.d_phasemax, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  LSFFT_TRY(hipStreamSynchronize(st));
  p->h2d_inflight = false;
  const int* pmax = hptr<int>(b, m_pmax);
  for (int i = 0; i < n; ++i) {
    int m = pmax[i];
    for (int j = 0; j < i; ++j)
      if (b.specs[j].phase == b.specs[i].phase && b.geo[j].nvox == b.geo[i].nvox) m = std::max(m, pmax[j]);
    if (m >= b.specs[i].tab->nphase) return LSFFT_E_ARG;
  }
  }

  // descriptors, states, tables, groups, counts and lists: one copy
  std::vector<int> all(n);
  for (int i = 0; i < n; ++i) all[i] = i;
  return upload_lists(b, all, true, 0);
}

// ---- launches of one pass kind over the segments of a work list ----------
hipError_t pass_x(Batch& b, int list, int mode, int cls) {
  for (const Seg& sg : b.segs[list]) {
    if (sg.count == 0) continue;
    const int t = timed_begin(b.p, cls);
    hipError_t e = launch_xpass(b.p->f64, timed(b.p, largs(b, list, sg), t), mode, sg.dim, sg.len, sg.var);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t pass_reduce(Batch& b, int mode);
// With `reduce`, the first launch also applies the stopping rule of the
// outer pass before it to every running solve (in place of k_reduce).
hipError_t pass_y(Batch& b, int list, int dir, int which, int ncomp, int gate, int cls, bool reduce = false) {
  for (const Seg& sg : b.segs[list]) {
    if (sg.count == 0) continue;
    const int t = timed_begin(b.p, cls);
    LaunchArgs a = largs(b, list, sg, ncomp);
    if (reduce) {
      a.red_inst = b.d_inst;
      a.red_n = b.d_counts + kMaxSegs - 1;
      reduce = false;
    }
    hipError_t e = launch_ypass(b.p->f64, timed(b.p, a, t), dir, which, ncomp, gate, sg.len, sg.var);
    if (e != hipSuccess) return e;
  }
  // no y launch (2D grids only): the rule runs on its own
  if (reduce) return pass_reduce(b, M_ITER);
  return hipSuccess;
}
hipError_t pass_g(Batch& b, int list, int mode, int cls) {
  for (const Seg& sg : b.segs[list]) {
    if (sg.count == 0) continue;
    const int t = timed_begin(b.p, cls);
    hipError_t e = launch_green(b.p->f64, timed(b.p, largs(b, list, sg), t), mode, sg.dim, sg.len, sg.var);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t pass_reduce(Batch& b, int mode) {
  const int t = timed_begin(b.p, LSFFT_K_REDUCE);
  hipError_t e = launch_reduce(timed(b.p, base_args(b), t), b.d_inst, b.d_counts + kMaxSegs - 1, b.n_running, mode);
  return e;
}
hipError_t pass_cg_update(Batch& b) {
  for (const Seg& sg : b.segs[L_CG]) {
    if (sg.count == 0) continue;
    const int t = timed_begin(b.p, LSFFT_K_CGUPD);
    hipError_t e = launch_cg_update(b.p->f64, timed(b.p, largs(b, L_CG, sg), t));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Force transform, free term u^b = N0 P f^ and ||P f||.  With `spectral_force`
// the force spectra are already in place (one per solve) and only the solves
// on the current dynamic lists are (re)started.
lsfft_status setup(Batch& b, bool spectral_force) {
  lsfft_plan_s* p = b.p;
  const int n = (int)b.specs.size();
  p->timing_active = false;
  if (!spectral_force) {
    LSFFT_TRY(pass_x(b, L_XLEAD, M_FT, LSFFT_K_OTHER));
    LSFFT_TRY(pass_y(b, L_YLEAD, -1, 1, 3, 0, LSFFT_K_OTHER));
    LSFFT_TRY(pass_g(b, L_GLEAD, M_FT, LSFFT_K_OTHER));
    LSFFT_TRY(pass_g(b, L_GALL, M_INIT, LSFFT_K_OTHER));
  } else {
    LSFFT_TRY(pass_g(b, L_G, M_INIT, LSFFT_K_OTHER));
  }
  LSFFT_TRY(pass_reduce(b, M_INIT));

  if (!spectral_force && (p->flags & LSFFT_STRICT_EQUIL)) {
    const lsfft_status ls = d2h_states(b);
    if (ls != LSFFT_OK) return ls;
    for (int i = 0; i < n; ++i) {
      const InstState& L = b.state[b.specs[i].leader];
      const double fn = std::sqrt(b.state[i].fnorm2 / (double)b.geo[i].nvox);
      for (int c = 0; c < b.geo[i].dim; ++c) {
        const double sum = std::fabs(L.removed_mean[c]) * (double)b.geo[i].nvox;
        if (sum > 1e-12 * std::sqrt((double)b.geo[i].nvox) * std::max(fn, 1e-300)) return LSFFT_E_NONEQUIL;
      }
    }
  }
  return LSFFT_OK;
}

// Copy the solve states to the host and list the running ones.
lsfft_status read_states(Batch& b, std::vector<int>& running) {
  const int n = (int)b.specs.size();
  const lsfft_status ls = d2h_states(b);
  if (ls != LSFFT_OK) return ls;
  running.clear();
  for (int i = 0; i < n; ++i)
    if (b.state[i].status == ST_RUNNING) running.push_back(i);
  return LSFFT_OK;
}

// Iterate every solve on the dynamic lists until none is running.  With
// `max_rounds` > 0 at most that many single-iteration rounds are run, without
// a graph (the mixed-precision outer step).
lsfft_status iterate(Batch& b, int max_rounds = 0, std::vector<int>* running_out = nullptr) {
  lsfft_plan_s* p = b.p;
  const bool cg = p->scheme == LSFFT_CG || p->scheme == LSFFT_CG_PLAIN;
  hipStream_t st = p->stream;
  const bool timing = (p->flags & LSFFT_TIMING) != 0 || p->force_timing;
  p->timing_active = timing;
  if (cg) {
    // r0 = P f - A u^b from one operator application on u^b
    LSFFT_TRY(pass_y(b, L_Y, +1, 0, 6, 1, LSFFT_K_YPASS));
    LSFFT_TRY(pass_x(b, L_X, M_ITER, LSFFT_K_XPASS));
    LSFFT_TRY(pass_y(b, L_Y, -1, 0, 6, 1, LSFFT_K_YPASS));
    LSFFT_TRY(pass_g(b, L_G, M_CG_INIT, LSFFT_K_GREEN));
    LSFFT_TRY(pass_reduce(b, M_CG_INIT));
  }
  const int per_round = max_rounds > 0 ? 1 : p->poll;
  // Inside a round of the basic scheme the stopping rule of iteration k runs
  // at the start of iteration k + 1's first y pass (same block size and
  // summation order as k_reduce, so the same bits); the round's last
  // iteration keeps k_reduce, since the host reads the states after it.
  // Timed plans keep k_reduce throughout, so that each pass class is timed
  // on its own.
  const bool aa = p->scheme == LSFFT_ANDERSON;
  const bool fuse = !cg && !aa && !timing;
  // one polling round: `per_round` iterations of every running solve
  auto round = [&]() -> hipError_t {
    bool pending = false;
    for (int k = 0; k < per_round; ++k) {
      hipError_t e;
      if ((e = pass_y(b, L_Y, +1, 0, 6, 1, LSFFT_K_YPASS, pending)) != hipSuccess) return e;
      pending = false;
      if ((e = pass_x(b, L_X, M_ITER, LSFFT_K_XPASS)) != hipSuccess) return e;
      if ((e = pass_y(b, L_Y, -1, 0, 6, 1, LSFFT_K_YPASS)) != hipSuccess) return e;
      if (aa) {
        if ((e = pass_g(b, L_G, M_AA_RES, LSFFT_K_GREEN)) != hipSuccess) return e;
        if ((e = pass_reduce(b, M_AA_RES)) != hipSuccess) return e;
        if ((e = pass_g(b, L_G, M_AA_UPD, LSFFT_K_GREEN)) != hipSuccess) return e;
      } else if (!cg) {
        if ((e = pass_g(b, L_G, M_ITER, LSFFT_K_GREEN)) != hipSuccess) return e;
        if (fuse && k + 1 < per_round) pending = true;
        else if ((e = pass_reduce(b, M_ITER)) != hipSuccess) return e;
      } else {
        if ((e = pass_g(b, L_G, M_CG_AP, LSFFT_K_GREEN)) != hipSuccess) return e;
        if ((e = pass_reduce(b, M_CG_AP)) != hipSuccess) return e;
        if ((e = pass_cg_update(b)) != hipSuccess) return e;
        if ((e = pass_reduce(b, M_CG_UPD)) != hipSuccess) return e;
        if ((e = pass_g(b, L_G, M_CG_DIR, LSFFT_K_GREEN)) != hipSuccess) return e;
      }
    }
    return hipSuccess;
  };
  // Without per-launch timing the round is captured once as a HIP graph and
  // replayed: launch grids are fixed at capture (the largest work lists), the
  // kernels read the current item counts from device memory, so retiring
  // solves later needs no recapture.
  hipGraphExec_t& gexec = b.graph.exec;
  const bool use_graph = p->graphs && !timing && max_rounds == 0;
  std::vector<int> running;
  // Rounds launched between two host polls: from each running solve's
  // observed contraction since the previous poll, the iterations it still
  // needs; the earliest finisher sets how many rounds run unpolled (at most
  // kMaxReplays).  Rounds past a solve's end are gated on the device.
  constexpr int kMaxReplays = 8;
  const int n = (int)b.specs.size();
  std::vector<double> last_res(n, -1.0);
  std::vector<int> last_it(n, -1);
  int reps = 1;
  for (int r = 0; max_rounds == 0 || r < max_rounds; r += reps) {
    for (int k = 0; k < reps; ++k) {
      if (use_graph) {
        if (!gexec) {
          hipGraph_t graph = nullptr;
          LSFFT_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          const hipError_t ce = round();
          const hipError_t ee = hipStreamEndCapture(st, &graph);
          if (ce != hipSuccess || ee != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return LSFFT_E_DEVICE;
          }
          const hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
          (void)hipGraphDestroy(graph);
          if (ie != hipSuccess) {
            gexec = nullptr;
            return LSFFT_E_DEVICE;
          }
        }
        LSFFT_TRY(hipGraphLaunch(gexec, st));
      } else {
        LSFFT_TRY(round());
      }
    }
    lsfft_status ls = read_states(b, running);
    if (ls != LSFFT_OK) return ls;
    if (running.empty()) break;
    if ((int)running.size() < b.n_running) {
      ls = upload_lists(b, running, false);
      if (ls != LSFFT_OK) return ls;
    }
    double rem_min = 1e300;
    for (int i : running) {
      const InstState& S = b.state[i];
      double rem = (double)per_round;   // unknown rate: one round
      if (last_it[i] >= 0 && S.iter > last_it[i] && S.residual > 0.0 && S.residual < last_res[i]) {
        const double rho = std::pow(S.residual / last_res[i], 1.0 / (double)(S.iter - last_it[i]));
        const double tol = b.desc[i].tol;
        if (rho < 1.0 && rho > 0.0 && tol < S.residual) rem = std::log(tol / S.residual) / std::log(rho);
        else if (tol >= S.residual) rem = 0.0;
      }
      rem_min = std::min(rem_min, rem);
      last_res[i] = S.residual;
      last_it[i] = S.iter;
    }
    if (max_rounds == 0) {
      reps = (int)std::floor(rem_min / (double)per_round);
      reps = std::max(1, std::min(kMaxReplays, reps));
    }
  }
  if (timing) timed_collect(p);
  p->timing_active = false;
  if (running_out) *running_out = running;
  return LSFFT_OK;
}

// u, eps, sigma of the returned iterates; the averaging accumulation.
lsfft_status materialize(Batch& b) {
  LSFFT_TRY(pass_g(b, L_GALL, M_MAT, LSFFT_K_OTHER));
  LSFFT_TRY(pass_y(b, L_YALL, +1, 0, /*eps + u*/ 9, 0, LSFFT_K_OTHER));
  LSFFT_TRY(pass_x(b, L_XALL, M_MAT, LSFFT_K_OTHER));
  if (b.averaging) {
    for (int g = 0; g < (int)b.groups.size(); ++g) {
      const Geometry& G = b.geo[b.groups[g].first];
      LSFFT_TRY(launch_accumulate(b.p->f64, G.dim, base_args(b), b.d_groups, g, G.nvox));
    }
  }
  LSFFT_TRY(hipStreamSynchronize(b.p->stream));
  return LSFFT_OK;
}

lsfft_status rank_worst(lsfft_status worst, int s) {
  auto rank = [](int v) { return v == LSFFT_E_DIVERGED ? 4 : v == LSFFT_E_NOCONV ? 3 : v == LSFFT_W_STAGNATED ? 1 : 0; };
  return rank(s) > rank(worst) ? (lsfft_status)s : worst;
}

// Starting displacements given by the caller: their spectra (forward
// transforms, projected off the xi = 0 set like the force) are taken into
// U[1] through the force-transform passes, with the descriptors pointed at
// them for the occasion.  Needs every solve to be its own leader (plain
// solves) and the basic scheme (U[1] exists).
lsfft_status transform_starts(Batch& b) {
  const int n = (int)b.specs.size();
  lsfft_plan_s* p = b.p;
  std::vector<InstDesc> keep(b.desc.begin(), b.desc.end());
  if (host_fence(p) != LSFFT_OK) return LSFFT_E_DEVICE;
  for (int i = 0; i < n; ++i) {
    b.desc[i].f_in = b.specs[i].u_init;
    b.desc[i].F = b.desc[i].U[1];
  }
  std::memcpy(hptr<InstDesc>(b, 0), b.desc.data(), sizeof(InstDesc) * n);
  lsfft_status ls = h2d(b, 0, sizeof(InstDesc) * n);
  if (ls != LSFFT_OK) return ls;
  LSFFT_TRY(pass_x(b, L_XLEAD, M_FT, LSFFT_K_OTHER));
  LSFFT_TRY(pass_y(b, L_YLEAD, -1, 1, 3, 0, LSFFT_K_OTHER));
  LSFFT_TRY(pass_g(b, L_GLEAD, M_FT, LSFFT_K_OTHER));
  if (host_fence(p) != LSFFT_OK) return LSFFT_E_DEVICE;
  for (int i = 0; i < n; ++i) b.desc[i] = keep[i];
  std::memcpy(hptr<InstDesc>(b, 0), b.desc.data(), sizeof(InstDesc) * n);
  return h2d(b, 0, sizeof(InstDesc) * n);
}

// After setup: the starting spectra replace the free term as state 0, and
// the strain spectrum of that state is recomputed.
lsfft_status install_starts(Batch& b) {
  const int n = (int)b.specs.size();
  const size_t cs = b.p->f64 ? 16 : 8;
  for (int i = 0; i < n; ++i)
    LSFFT_TRY(hipMemcpyAsync(b.desc[i].U[0], b.desc[i].U[1], cs * (size_t)b.geo[i].dim * (size_t)b.geo[i].Pc,
                             hipMemcpyDeviceToDevice, b.p->stream));
  LSFFT_TRY(pass_g(b, L_G, M_MAT, LSFFT_K_OTHER));
  return LSFFT_OK;
}

lsfft_status run_batch(Batch& b, lsfft_report* rep, double t0_wall) {
  lsfft_status ls = prepare(b);
  if (ls != LSFFT_OK) return ls;
  const bool warm = !b.specs.empty() && b.specs[0].u_init != nullptr;
  if (warm && (ls = transform_starts(b)) != LSFFT_OK) return ls;
  if ((ls = setup(b, false)) != LSFFT_OK) return ls;
  if (warm && (ls = install_starts(b)) != LSFFT_OK) return ls;
  if ((ls = iterate(b)) != LSFFT_OK) return ls;
  if ((ls = materialize(b)) != LSFFT_OK) return ls;
  const double secs = now_s() - t0_wall;
  lsfft_status worst = LSFFT_OK;
  for (int i = 0; i < (int)b.specs.size(); ++i) {
    const InstState& S = b.state[i];
    lsfft_report& r = rep[b.specs[i].out_index];
    r.iters = S.iter;
    r.residual = S.residual;
    const InstState& L = b.state[b.specs[i].leader];
    for (int c = 0; c < 3; ++c) r.removed_mean[c] = (c < b.geo[i].dim) ? L.removed_mean[c] : 0.0;
    r.status = S.status;
    r.seconds = secs;
    worst = rank_worst(worst, S.status);
  }
  return worst;
}

// Mixed-precision defect correction (FP32 plans with LSFFT_REFINE64).  The
// state u lives in FP64 on the companion FP64 plan; each outer step
//   1. evaluates the FP64 residual r = P f + div(L sym grad u) and its norm
//      (one FP64 basic iteration: the stopping test runs on this residual),
//   2. solves A d = r in FP32 with the plan's scheme to a relative residual
//      aimed at 0.3 tol / |r| (A = -div(L sym grad .), the same operator),
//      at least kInnerTol,
//   3. sets u += d in FP64.
// The FP32 floor of the inner solves bounds only the reduction per step, not
// the final accuracy.  The returned fields are materialized in FP32 from the
// FP64 state rounded once.  A floor of 3e-5 reaches 1e-8 in two outer steps
// with about as many FP32 iterations in all as three steps of 1e-3 take, and
// saves one FP64 residual evaluation and one round of host decisions.
#ifndef LSFFT_INNER_TOL
#define LSFFT_INNER_TOL 3e-5
#endif
constexpr double kInnerTol = LSFFT_INNER_TOL;
constexpr int kMaxOuter = 40;

lsfft_status run_refined(Batch& b, lsfft_report* rep, double t0_wall) {
  lsfft_plan_s* p = b.p;
  lsfft_plan_s* q = p->sub;
  const int n = (int)b.specs.size();
  const bool cg = p->scheme == LSFFT_CG || p->scheme == LSFFT_CG_PLAIN;
  hipStream_t st = p->stream;

  // FP64 copies of the forces (exact widening), one per leader
  size_t need = 0;
  std::vector<size_t> foff(n, 0);
  for (int i = 0; i < n; ++i) {
    if (b.specs[i].leader != i) continue;
    const lsfft_grid& g = p->grids[b.specs[i].grid];
    foff[i] = need;
    need = align_up(need + sizeof(double) * (size_t)g.dim * (size_t)(gnx(g) * gny(g) * gnz(g)));
  }
  if (!q->fwide.ensure(need)) return LSFFT_E_ALLOC;
  Batch c;   // FP64 companion: state, force spectrum, residual
  c.p = q;
  c.tol = b.tol;
  c.max_iter = kMaxOuter;
  c.averaging = false;
  c.specs = b.specs;
  for (int i = 0; i < n; ++i) {
    Spec& s = c.specs[i];
    s.eps = s.sig = s.u = nullptr;
    s.group = -1;
    const lsfft_grid& g = p->grids[s.grid];
    const long long cnt = (long long)g.dim * gnx(g) * gny(g) * gnz(g);
    double* w = reinterpret_cast<double*>(static_cast<char*>(q->fwide.p) + foff[s.leader]);
    if (s.leader == i) LSFFT_TRY(launch_widen(static_cast<const float*>(b.specs[i].f), w, cnt, st));
    s.f = w;
  }
  lsfft_status ls = prepare(c);
  if (ls != LSFFT_OK) return ls;
  if ((ls = setup(c, false)) != LSFFT_OK) return ls;

  // FP32 inner solves: one force spectrum per solve (the defects differ)
  Batch in = b;
  in.tol = kInnerTol;
  for (int i = 0; i < n; ++i) in.specs[i].leader = i;
  if ((ls = prepare(in, false)) != LSFFT_OK) return ls;
  std::vector<long long> inner_iters(n, 0);
  std::vector<double> inner_floor(n, 0.0);
  std::vector<int> running, in_listed(n);
  for (int i = 0; i < n; ++i) in_listed[i] = i;   // what prepare() listed for the inner batch
  for (;;) {
    // outer step 1: FP64 residual and stopping test at the current state
    // (iterate reads the states back and shrinks the lists to the running
    // solves)
    if ((ls = iterate(c, 1, &running)) != LSFFT_OK) return ls;
    if (running.empty()) break;
    // inner tolerance per solve: a step leaves about the inner tolerance
    // times the current residual, so aim at 0.3 tol, within [kInnerTol, 0.1],
    // and not below 1.5 times the level where an earlier inner solve of this
    // solve stagnated (its FP32 floor)
    if ((ls = host_fence(p)) != LSFFT_OK) return ls;
    for (int i : running) {
      const double aim = std::max(0.3 * c.tol / std::max(c.state[i].residual, 1e-300), 1.5 * inner_floor[i]);
      in.desc[i].tol = std::min(0.1, std::max(kInnerTol, aim));
    }
    std::memcpy(hptr<InstDesc>(in, 0), in.desc.data(), sizeof(InstDesc) * n);
    if ((ls = h2d(in, 0, sizeof(InstDesc) * n)) != LSFFT_OK) return ls;
    // the inner lists keep their last contents when every inner solve ends;
    // rebuild them only when the set of solves changed
    if (running != in_listed || in.n_running != (int)running.size()) {
      if ((ls = upload_lists(in, running, false)) != LSFFT_OK) return ls;
      in_listed = running;
    }
    // step 2: defect as FP32 force, inner solve
    LSFFT_TRY(launch_defect(c.d_desc, c.d_state, in.d_desc, c.d_inst, c.n_running, max_pc(c, running), st));
    if ((ls = setup(in, true)) != LSFFT_OK) return ls;
    std::vector<int> still;
    if ((ls = iterate(in, 0, &still)) != LSFFT_OK) return ls;
    if (in.n_running != (int)in_listed.size()) in_listed.clear();   // compacted on the way
    for (int i : running) {
      inner_iters[i] += in.state[i].iter;
      if (in.state[i].status == ST_STAGNATED) inner_floor[i] = std::max(inner_floor[i], in.state[i].residual);
    }
    // step 3: u += d in FP64
    LSFFT_TRY(launch_correct(c.d_desc, c.d_state, in.d_desc, in.d_state, c.d_inst, c.n_running, cg,
                             max_pc(c, running), st));
    // strain spectrum of the corrected state, the input of the next residual
    LSFFT_TRY(pass_g(c, L_G, M_MAT, LSFFT_K_OTHER));
  }
  // round the FP64 iterates once and materialize them in FP32
  std::vector<int> all(n);
  for (int i = 0; i < n; ++i) all[i] = i;
  if ((ls = upload_lists(c, all, false)) != LSFFT_OK) return ls;
  LSFFT_TRY(launch_narrow(c.d_desc, c.d_state, in.d_desc, c.d_inst, n, max_pc(c, all), st));
  for (int i = 0; i < n; ++i) {
    in.state[i].iter = 0;
    in.state[i].status = c.state[i].status;
  }
  if ((ls = h2d_states(in)) != LSFFT_OK) return ls;
  if ((ls = materialize(in)) != LSFFT_OK) return ls;
  const double secs = now_s() - t0_wall;
  lsfft_status worst = LSFFT_OK;
  for (int i = 0; i < n; ++i) {
    const InstState& S = c.state[i];
    lsfft_report& r = rep[b.specs[i].out_index];
    r.iters = (int)std::min<long long>(inner_iters[i], 0x7fffffff);
    r.residual = S.residual;
    const InstState& L = c.state[c.specs[i].leader];
    for (int k = 0; k < 3; ++k) r.removed_mean[k] = (k < c.geo[i].dim) ? L.removed_mean[k] : 0.0;
    r.status = S.status;
    r.seconds = secs;
    worst = rank_worst(worst, S.status);
  }
  return worst;
}

lsfft_status check_plan(lsfft_plan_s* p) { return p ? LSFFT_OK : LSFFT_E_ARG; }

// Order the plan's work stream after everything already enqueued on the
// caller's stream (the inputs).
lsfft_status enter(lsfft_plan_s* p) {
  if (hipSetDevice(p->device) != hipSuccess) return LSFFT_E_DEVICE;
  if (hipEventRecord(p->ev_in, p->ustream) != hipSuccess) return LSFFT_E_DEVICE;
  if (hipStreamWaitEvent(p->stream, p->ev_in, 0) != hipSuccess) return LSFFT_E_DEVICE;
  return LSFFT_OK;
}

lsfft_status worse(lsfft_status a, lsfft_status b) {
  auto rank = [](int s) {
    return s < 0 && s != LSFFT_E_NOCONV && s != LSFFT_E_DIVERGED ? 9
         : s == LSFFT_E_DIVERGED ? 4 : s == LSFFT_E_NOCONV ? 3 : s == LSFFT_W_STAGNATED ? 1 : 0;
  };
  return rank(a) >= rank(b) ? a : b;
}

// Twiddle table exp(-2 pi i k / L) for every supported length, long double
// arithmetic rounded once to the plan precision.
bool upload_twiddles(lsfft_plan_s* p) {
  const int total = tw_total();
  std::vector<double> twd(2 * (size_t)total);
  for (int i = 0; i < kNumLens; ++i) {
    const int L = len_at(i), o = tw_offset(L);
    for (int k = 0; k < L; ++k) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)L;
      twd[2 * (o + k)] = (double)cosl(ang);
      twd[2 * (o + k) + 1] = (double)sinl(ang);
    }
  }
  const size_t bytes = (p->f64 ? sizeof(double) : sizeof(float)) * twd.size();
  if (!p->tw.ensure(bytes)) return false;
  hipError_t e;
  if (p->f64) {
    e = hipMemcpy(p->tw.p, twd.data(), bytes, hipMemcpyHostToDevice);
  } else {
    std::vector<float> twf(twd.begin(), twd.end());
    e = hipMemcpy(p->tw.p, twf.data(), bytes, hipMemcpyHostToDevice);
  }
  return e == hipSuccess;
}

// Release a plan, its companion and every buffer they own.
void free_plan(lsfft_plan_s* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (p->sub) free_plan(p->sub);
  p->sub = nullptr;
  if (p->owns_stream) {
    if (p->stream) (void)hipStreamDestroy(p->stream);
    if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  }
  p->tw.release();
  p->arena.release();
  p->meta.release();
  p->hmeta.release();
  p->rve.release();
  p->kspec.release();
  p->zphase.release();
  p->lists.release();
  p->fwide.release();
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  delete p;
}

}  // namespace

// ---------------------------------------------------------------------------
// schedule cache: a flat JSON object {"f32/3d/outer/256": 2, ...}
// ---------------------------------------------------------------------------
const char* kKindName[3] = {"x", "y", "outer"};

std::string tune_key(bool f64, int dim, int kind, int len) {
  char buf[64];
  std::snprintf(buf, sizeof buf, "%s/%dd/%s/%d", f64 ? "f64" : "f32", dim, kKindName[kind], len);
  return buf;
}

// "key": integer pairs of a flat JSON object; anything else is skipped
std::map<std::string, int> parse_tune_cache(const char* text) {
  std::map<std::string, int> out;
  if (!text) return out;
  const char* c = text;
  while (*c) {
    if (*c != '"') { ++c; continue; }
    const char* k0 = ++c;
    while (*c && *c != '"') ++c;
    if (!*c) break;
    std::string key(k0, c - k0);
    ++c;
    while (*c == ' ' || *c == '\t' || *c == '\n' || *c == '\r') ++c;
    if (*c != ':') continue;
    ++c;
    while (*c == ' ' || *c == '\t' || *c == '\n' || *c == '\r') ++c;
    char* end = nullptr;
    const long v = std::strtol(c, &end, 10);
    if (end == c) continue;
    if (v >= 0 && v < 64) out[key] = (int)v;
    c = end;
  }
  return out;
}

bool read_file(const char* path, std::string* text) {
  FILE* fh = std::fopen(path, "rb");
  if (!fh) return false;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, fh)) > 0) text->append(buf, n);
  std::fclose(fh);
  return true;
}

bool write_tune_cache(const char* path, const std::map<std::string, int>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fh = std::fopen(tmp.c_str(), "wb");
  if (!fh) return false;
  std::fprintf(fh, "{\n");
  size_t k = 0;
  for (const auto& kv : m) std::fprintf(fh, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++k < m.size() ? "," : "");
  std::fprintf(fh, "}\n");
  const bool ok = std::fclose(fh) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

// cache key of a grid's spectral layout
std::string layout_key(bool f64, const lsfft_grid& g) {
  char buf[96];
  std::snprintf(buf, sizeof buf, "%s/3d/layout/%lldx%lldx%lld", f64 ? "f64" : "f32", (long long)gnx(g),
                (long long)gny(g), (long long)gnz(g));
  return buf;
}

bool same_shape(const lsfft_grid& a, const lsfft_grid& b) {
  return a.dim == b.dim && gnx(a) == gnx(b) && gny(a) == gny(b) && gnz(a) == gnz(b);
}

// layout of grid gi, in the plan and in its FP64 companion
void set_layout(lsfft_plan_s* p, int gi, int v) {
  p->layout[gi] = v;
  if (p->sub) p->sub->layout[gi] = v;
}

// apply every cache entry that matches one of the plan's grids
void apply_tune_cache(lsfft_plan_s* p, const std::map<std::string, int>& m) {
  for (size_t gi = 0; gi < p->grids.size(); ++gi) {
    if (!blocked_layout_ok(p->grids[gi])) continue;
    const auto it = m.find(layout_key(p->f64, p->grids[gi]));
    if (it != m.end() && it->second <= 1) set_layout(p, (int)gi, it->second);
  }
  for (const lsfft_grid& g : p->grids) {
    const int lens[3] = {(int)gnx(g), (int)gny(g), (int)(g.dim == 3 ? gnz(g) : gny(g))};
    for (int kind = 0; kind < 3; ++kind) {
      if (kind == 1 && g.dim != 3) continue;
      const auto it = m.find(tune_key(p->f64, g.dim, kind, lens[kind]));
      if (it == m.end()) continue;
      const int i = len_index(lens[kind]);
      if (i >= 0 && it->second < schedule_variants(p->f64, g.dim, kind, lens[kind])) p->sched[kind][i] = it->second;
    }
  }
}

std::mutex tune_file_mu;

// ===========================================================================
// C ABI
// ===========================================================================
namespace {

// Accumulation target of one averaging group: FP64 sums of its solves,
// divided by their count at the end.
struct AvgTarget {
  int grid_idx;
  int incl_phase;
  int count;
  double* avg;
};

// Solve `specs` (consecutive solves of one group share a force spectrum) in
// batches of at most max_batch and accumulate every solve into its group's
// target (Eqs. 3.5-3.6 and 3.8).
lsfft_status run_averages(lsfft_plan_t p, const std::vector<Spec>& specs, const std::vector<int>& spec_group,
                          const std::vector<AvgTarget>& groups, double tol, int max_iter, lsfft_report* rep) {
  const int ngroup = (int)groups.size();
  if (enter(p) != LSFFT_OK) return LSFFT_E_DEVICE;
  for (int g = 0; g < ngroup; ++g) {
    const lsfft_grid& gr = p->grids[groups[g].grid_idx];
    const int d = gr.dim, s = d == 3 ? 6 : 3;
    const long long nvox = gr.n[0] * gr.n[1] * (d == 3 ? gr.n[2] : 1);
    if (hipMemsetAsync(groups[g].avg, 0, sizeof(double) * (size_t)(2 * d + 4 * s + 1) * nvox, p->stream) != hipSuccess)
      return LSFFT_E_DEVICE;
  }
  lsfft_status worst = LSFFT_OK;
  const int total = (int)specs.size();
  for (int start = 0; start < total; start += p->max_batch) {
    const int cnt = std::min(p->max_batch, total - start);
    Batch b;
    b.p = p;
    b.tol = tol;
    b.max_iter = max_iter;
    b.averaging = true;
    b.specs.assign(specs.begin() + start, specs.begin() + start + cnt);
    // sub-groups of this batch: consecutive solves of the same group share
    // one force spectrum (the first of them transforms it)
    for (int i = 0; i < cnt; ++i) {
      const int g = spec_group[start + i];
      if (i == 0 || spec_group[start + i - 1] != g) {
        BatchGroup bg;
        bg.avg = groups[g].avg;
        bg.incl_phase = groups[g].incl_phase;
        bg.first = i;
        bg.count = 0;
        b.groups.push_back(bg);
      }
      b.groups.back().count += 1;
      b.specs[i].group = (int)b.groups.size() - 1;
      b.specs[i].leader = b.groups.back().first;
    }
    const double t0 = now_s();
    lsfft_status s = p->sub ? run_refined(b, rep, t0) : run_batch(b, rep, t0);
    if (s == LSFFT_E_ARG || s == LSFFT_E_ALLOC || s == LSFFT_E_DEVICE || s == LSFFT_E_NONEQUIL) return s;
    worst = worse(worst, s);
  }
  for (int g = 0; g < ngroup; ++g) {
    const lsfft_grid& gr = p->grids[groups[g].grid_idx];
    const int d = gr.dim, s = d == 3 ? 6 : 3;
    const long long nvox = gr.n[0] * gr.n[1] * (d == 3 ? gr.n[2] : 1);
    if (launch_scale(groups[g].avg, (long long)(2 * d + 4 * s + 1) * nvox, 1.0 / groups[g].count, p->stream) != hipSuccess)
      return LSFFT_E_DEVICE;
  }
  if (hipStreamSynchronize(p->stream) != hipSuccess) return LSFFT_E_DEVICE;
  return worst;
}

}  // namespace

extern "C" {

const char* lsfft_status_string(int status) {
  switch (status) {
    case LSFFT_OK: return "ok";
    case LSFFT_W_STAGNATED: return "stagnated: residual stopped improving above tol";
    case LSFFT_E_ARG: return "invalid argument";
    case LSFFT_E_ALLOC: return "device allocation failed";
    case LSFFT_E_DEVICE: return "HIP runtime error";
    case LSFFT_E_NOCONV: return "not converged within max_iter";
    case LSFFT_E_NONEQUIL: return "force is not self-equilibrated";
    case LSFFT_E_DIVERGED: return "diverged";
  }
  return "unknown status";
}

lsfft_status lsfft_lame_from_young(int nphase, const double* e_nu, double* lame_out) {
  if (nphase < 1 || !e_nu || !lame_out) return LSFFT_E_ARG;
  for (int p = 0; p < nphase; ++p) {
    const double e = e_nu[2 * p], nu = e_nu[2 * p + 1];
    if (!is_fin(e) || !is_fin(nu) || e <= 0.0 || nu <= -1.0 || nu >= 0.5) return LSFFT_E_ARG;
  }
  for (int p = 0; p < nphase; ++p) {
    const double e = e_nu[2 * p], nu = e_nu[2 * p + 1];
    lame_out[2 * p] = e * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    lame_out[2 * p + 1] = e / (2.0 * (1.0 + nu));
  }
  return LSFFT_OK;
}

lsfft_status lsfft_plan(lsfft_plan_t* out, const lsfft_grid* grids, int ngrid, int max_batch,
                        int prec, int scheme, unsigned flags, void* hip_stream) {
  if (!out) return LSFFT_E_ARG;
  *out = nullptr;
  if (!grids || ngrid < 1 || max_batch < 1) return LSFFT_E_ARG;
  if (prec != LSFFT_F32 && prec != LSFFT_F64) return LSFFT_E_ARG;
  if (scheme < LSFFT_BASIC || scheme > LSFFT_ANDERSON) return LSFFT_E_ARG;
  if (flags & ~(LSFFT_STRICT_EQUIL | LSFFT_TIMING | LSFFT_REFINE64)) return LSFFT_E_ARG;
  if ((flags & LSFFT_REFINE64) && (prec != LSFFT_F32 || max_batch > 65535)) return LSFFT_E_ARG;
  for (int g = 0; g < ngrid; ++g) {
    const lsfft_grid& G = grids[g];
    if (G.dim != 2 && G.dim != 3) return LSFFT_E_ARG;
    for (int a = 0; a < G.dim; ++a) {
      if (!supported_len(G.n[a])) return LSFFT_E_ARG;
      if (!is_fin(G.h[a]) || G.h[a] <= 0.0) return LSFFT_E_ARG;
    }
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LSFFT_E_DEVICE;
  lsfft_plan_s* p = new (std::nothrow) lsfft_plan_s();
  if (!p) return LSFFT_E_ALLOC;
  p->device = dev;
  p->ustream = static_cast<hipStream_t>(hip_stream);
  if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
    delete p;
    return LSFFT_E_DEVICE;
  }
  if (hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(p->stream);
    delete p;
    return LSFFT_E_DEVICE;
  }
  // address of this device's copy of the fixed RVE scratch (once per
  // device); a failed lookup only disables lsfft_rve_identify_noalloc
  (void)rve_scratch_init(dev);
  if (std::getenv("LSFFT_NO_GRAPH")) p->graphs = false;
  p->f64 = (prec == LSFFT_F64);
  p->scheme = static_cast<lsfft_scheme>(scheme);
  p->flags = flags;
  p->grids.assign(grids, grids + ngrid);
  for (auto& G : p->grids)
    if (G.dim == 2) { G.n[2] = 1; G.h[2] = 1.0; }
  // default layout: blocked for FP32 plans; FP64 plans, whose outer tiles
  // are half a kx block wide, start in rows (at 128^3: 21.0 against 23.9 ms
  // per solve)
  p->layout.assign(p->grids.size(), p->f64 ? 0 : 1);
  p->max_batch = max_batch;
  // schedule variants chosen by an earlier lsfft_autotune, if a cache is named
  if (const char* path = std::getenv("LSFFT_TUNE_CACHE")) {
    std::string text;
    std::lock_guard<std::mutex> lock(tune_file_mu);
    if (read_file(path, &text)) apply_tune_cache(p, parse_tune_cache(text.c_str()));
  }
  if (const char* e = std::getenv("LSFFT_POLL")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= 1024) p->poll = v;
  }
  if (!upload_twiddles(p)) {
    free_plan(p);
    return LSFFT_E_ALLOC;
  }
  if (flags & LSFFT_REFINE64) {
    lsfft_plan_s* q = new (std::nothrow) lsfft_plan_s();
    if (!q) {
      free_plan(p);
      return LSFFT_E_ALLOC;
    }
    q->device = dev;
    q->ustream = p->ustream;
    q->stream = p->stream;
    q->owns_stream = false;
    q->graphs = p->graphs;
    q->f64 = true;
    q->scheme = LSFFT_BASIC;
    q->flags = flags & LSFFT_STRICT_EQUIL;   // the force check runs on the FP64 force transform
    q->grids = p->grids;
    q->layout = p->layout;   // the FP64 and FP32 spectra of a solve share one layout
    q->max_batch = p->max_batch;
    p->sub = q;
    if (!upload_twiddles(q)) {
      free_plan(p);
      return LSFFT_E_ALLOC;
    }
  }
  *out = p;
  return LSFFT_OK;
}

lsfft_status lsfft_plan_destroy(lsfft_plan_t p) {
  if (!p) return LSFFT_OK;
  free_plan(p);
  return LSFFT_OK;
}

lsfft_status lsfft_solve_bfcs(lsfft_plan_t p, int nsolve, const int* grid_idx, const uint8_t* const* phase,
                              const lsfft_phases* tab, const lsfft_ref* c0, const void* const* f, double tol,
                              int max_iter, void* const* eps, void* const* sig, void* const* u,
                              const void* const* u_init, lsfft_report* rep) {
  if (check_plan(p) != LSFFT_OK) return LSFFT_E_ARG;
  if (nsolve < 1 || !grid_idx || !phase || !tab || !f || !rep) return LSFFT_E_ARG;
  if (!is_fin(tol) || tol <= 0.0 || max_iter < 0) return LSFFT_E_ARG;
  // warm starts: plain basic-scheme plans, every solve given one
  if (u_init) {
    if (p->sub || p->scheme != LSFFT_BASIC) return LSFFT_E_ARG;
    for (int i = 0; i < nsolve; ++i)
      if (!u_init[i]) return LSFFT_E_ARG;
  }
  std::vector<Spec> specs(nsolve);
  for (int i = 0; i < nsolve; ++i) {
    const int g = grid_idx[i];
    if (g < 0 || g >= (int)p->grids.size()) return LSFFT_E_ARG;
    if (!phase[i] || !f[i]) return LSFFT_E_ARG;
    if (check_table(&tab[i], p->grids[g].dim) != LSFFT_OK) return LSFFT_E_ARG;
    Spec& s = specs[i];
    s.grid = g;
    s.phase = phase[i];
    s.tab = &tab[i];
    if (resolve_ref(&tab[i], c0 ? &c0[i] : nullptr, &s.lam0, &s.mu0) != LSFFT_OK) return LSFFT_E_ARG;
    s.f = f[i];
    s.u_init = u_init ? u_init[i] : nullptr;
    s.eps = eps ? eps[i] : nullptr;
    s.sig = sig ? sig[i] : nullptr;
    s.u = u ? u[i] : nullptr;
    s.out_index = i;
  }
  if (enter(p) != LSFFT_OK) return LSFFT_E_DEVICE;
  lsfft_status worst = LSFFT_OK;
  for (int start = 0; start < nsolve; start += p->max_batch) {
    const int cnt = std::min(p->max_batch, nsolve - start);
    Batch b;
    b.p = p;
    b.tol = tol;
    b.max_iter = max_iter;
    b.specs.assign(specs.begin() + start, specs.begin() + start + cnt);
    for (int i = 0; i < cnt; ++i) b.specs[i].leader = i;
    const double t0 = now_s();
    lsfft_status s = p->sub ? run_refined(b, rep, t0) : run_batch(b, rep, t0);
    if (s == LSFFT_E_ARG || s == LSFFT_E_ALLOC || s == LSFFT_E_DEVICE || s == LSFFT_E_NONEQUIL) return s;
    worst = worse(worst, s);
  }
  return worst;
}

lsfft_status lsfft_translate_average_batch(lsfft_plan_t p, int ngroup, const lsfft_avg_group* groups,
                                           double tol, int max_iter, lsfft_report* rep) {
  if (check_plan(p) != LSFFT_OK) return LSFFT_E_ARG;
  if (ngroup < 1 || !groups || !rep) return LSFFT_E_ARG;
  if (!is_fin(tol) || tol <= 0.0 || max_iter < 0) return LSFFT_E_ARG;
  // expand groups into solves, validating every shift
  std::vector<Spec> specs;
  std::vector<int> spec_group;
  int slot = 0;
  for (int g = 0; g < ngroup; ++g) {
    const lsfft_avg_group& G = groups[g];
    if (G.grid_idx < 0 || G.grid_idx >= (int)p->grids.size()) return LSFFT_E_ARG;
    const lsfft_grid& gr = p->grids[G.grid_idx];
    if (!G.phase || !G.f || !G.avg || !G.shifts || G.nshift < 1) return LSFFT_E_ARG;
    if (check_table(G.tab, gr.dim) != LSFFT_OK) return LSFFT_E_ARG;
    if (G.incl_phase < 0 || G.incl_phase >= G.tab->nphase) return LSFFT_E_ARG;
    double lam0, mu0;
    if (resolve_ref(G.tab, G.c0, &lam0, &mu0) != LSFFT_OK) return LSFFT_E_ARG;
    for (int k = 0; k < G.nshift; ++k) {
      Spec s;
      s.grid = G.grid_idx;
      s.phase = G.phase;
      s.tab = G.tab;
      s.lam0 = lam0;
      s.mu0 = mu0;
      s.f = G.f;
      for (int a = 0; a < gr.dim; ++a) {
        const int v = G.shifts[(size_t)k * gr.dim + a];
        if (v < 0 || v >= gr.n[a]) return LSFFT_E_ARG;
        s.shift[a] = v;
      }
      s.out_index = slot++;
      specs.push_back(s);
      spec_group.push_back(g);
    }
  }
  std::vector<AvgTarget> tg(ngroup);
  for (int g = 0; g < ngroup; ++g) tg[g] = AvgTarget{groups[g].grid_idx, groups[g].incl_phase, groups[g].nshift, groups[g].avg};
  return run_averages(p, specs, spec_group, tg, tol, max_iter, rep);
}

lsfft_status lsfft_translate_average(lsfft_plan_t p, int grid_idx, const uint8_t* phase, const lsfft_phases* tab,
                                     const lsfft_ref* c0, const void* f, const int32_t* shifts, int nshift,
                                     int incl_phase, double tol, int max_iter, double* avg, lsfft_report* rep) {
  lsfft_avg_group g;
  g.grid_idx = grid_idx;
  g.phase = phase;
  g.tab = tab;
  g.c0 = c0;
  g.f = f;
  g.shifts = shifts;
  g.nshift = nshift;
  g.incl_phase = incl_phase;
  g.avg = avg;
  return lsfft_translate_average_batch(p, 1, &g, tol, max_iter, rep);
}

lsfft_status lsfft_realization_average(lsfft_plan_t p, int grid_idx, int nreal, const uint8_t* const* phases,
                                       const lsfft_phases* tab, const lsfft_ref* c0, const void* f, int incl_phase,
                                       double tol, int max_iter, double* avg, lsfft_report* rep) {
  if (check_plan(p) != LSFFT_OK) return LSFFT_E_ARG;
  if (nreal < 1 || !phases || !f || !avg || !rep) return LSFFT_E_ARG;
  if (!is_fin(tol) || tol <= 0.0 || max_iter < 0) return LSFFT_E_ARG;
  if (grid_idx < 0 || grid_idx >= (int)p->grids.size()) return LSFFT_E_ARG;
  const lsfft_grid& gr = p->grids[grid_idx];
  if (check_table(tab, gr.dim) != LSFFT_OK) return LSFFT_E_ARG;
  if (incl_phase < 0 || incl_phase >= tab->nphase) return LSFFT_E_ARG;
  double lam0, mu0;
  if (resolve_ref(tab, c0, &lam0, &mu0) != LSFFT_OK) return LSFFT_E_ARG;
  std::vector<Spec> specs(nreal);
  std::vector<int> spec_group(nreal, 0);
  for (int j = 0; j < nreal; ++j) {
    if (!phases[j]) return LSFFT_E_ARG;
    Spec& s = specs[j];
    s.grid = grid_idx;
    s.phase = phases[j];
    s.tab = tab;
    s.lam0 = lam0;
    s.mu0 = mu0;
    s.f = f;
    s.out_index = j;
  }
  return run_averages(p, specs, spec_group, std::vector<AvgTarget>{AvgTarget{grid_idx, incl_phase, nreal, avg}}, tol,
                      max_iter, rep);
}

}  // extern "C"

namespace {

// Arguments of an RVE identification, checked and resolved on the host.
struct RveArgs {
  int d = 0;
  int n[3] = {1, 1, 1};
  double h[3] = {1.0, 1.0, 1.0};
  double c[3] = {0.0, 0.0, 0.0};
  double box = 0.0;
  int nbins = 0;
};

lsfft_status rve_args(lsfft_plan_t p, int grid_idx, const double* avg, const double* center, double support_radius,
                      double tol, double dr, lsfft_rve* out, RveArgs* a) {
  if (check_plan(p) != LSFFT_OK || !avg || !center || !out) return LSFFT_E_ARG;
  if (grid_idx < 0 || grid_idx >= (int)p->grids.size()) return LSFFT_E_ARG;
  if (!is_fin(tol) || tol <= 0.0 || tol >= 1.0 || !is_fin(dr) || dr <= 0.0) return LSFFT_E_ARG;
  if (!is_fin(support_radius) || support_radius < 0.0) return LSFFT_E_ARG;
  const lsfft_grid& g = p->grids[grid_idx];
  a->d = g.dim;
  double rmax2 = 0.0, box = 1e300;
  for (int k = 0; k < a->d; ++k) {
    if (!is_fin(center[k])) return LSFFT_E_ARG;
    a->n[k] = (int)g.n[k];
    a->h[k] = g.h[k];
    a->c[k] = center[k];
    const double half = 0.5 * a->n[k] * a->h[k];
    rmax2 += half * half;
    box = std::min(box, half);
  }
  a->box = box;
  // the bin count is checked in floating point before the conversion
  const double nb = std::floor(std::sqrt(rmax2) / dr) + 1.0;
  if (!(nb <= (double)kRveBinsMax)) return LSFFT_E_ARG;
  a->nbins = (int)nb;
  return LSFFT_OK;
}

// Radius, fit flag and profile from the bin maxima `hb` (two rows of nbins
// bit patterns of non-negative doubles), Definition 2.2: the smallest bin
// edge beyond which both magnitudes stay below tol times their maxima.
void rve_finish(const unsigned long long* hb, const RveArgs& a, double support_radius, double tol, double dr,
                double* profile, int max_bins, lsfft_rve* out) {
  const int nbins = a.nbins;
  auto me = [&](int b) { double v; std::memcpy(&v, &hb[b], sizeof(double)); return v; };
  auto ms = [&](int b) { double v; std::memcpy(&v, &hb[nbins + b], sizeof(double)); return v; };
  double ge = 0.0, gs = 0.0;
  for (int b = 0; b < nbins; ++b) {
    ge = std::max(ge, me(b));
    gs = std::max(gs, ms(b));
  }
  int first = nbins;   // +inf when the outermost bin is still above tol
  for (int b = nbins - 1; b >= 0; --b) {
    if (me(b) < tol * ge && ms(b) < tol * gs) first = b;
    else break;
  }
  if (ge == 0.0 && gs == 0.0) first = 0;
  out->radius = (first < nbins) ? first * dr : HUGE_VAL;
  out->box_radius = a.box;
  out->fits = (first < nbins && out->radius + 0.5 * support_radius <= a.box) ? 1 : 0;
  out->nbins = nbins;
  out->max_eps = ge;
  out->max_sig = gs;
  if (profile && max_bins >= nbins) {
    for (int b = 0; b < nbins; ++b) {
      profile[b] = me(b);
      profile[max_bins + b] = ms(b);
    }
  }
}

}  // namespace

extern "C" {

lsfft_status lsfft_rve_identify(lsfft_plan_t p, int grid_idx, const double* avg, const double* center,
                                double support_radius, double tol, double dr, double* profile, int max_bins,
                                lsfft_rve* out) {
  RveArgs a;
  lsfft_status ls = rve_args(p, grid_idx, avg, center, support_radius, tol, dr, out, &a);
  if (ls != LSFFT_OK) return ls;
  const int nbins = a.nbins;
  if (!p->rve.ensure(sizeof(unsigned long long) * 2 * (size_t)nbins)) return LSFFT_E_ALLOC;
  if (enter(p) != LSFFT_OK) return LSFFT_E_DEVICE;
  auto* bins = static_cast<unsigned long long*>(p->rve.p);
  std::vector<unsigned long long> hb(2 * (size_t)nbins);
  if (hipMemsetAsync(bins, 0, sizeof(unsigned long long) * hb.size(), p->stream) != hipSuccess) return LSFFT_E_DEVICE;
  if (launch_radial_max(a.d, avg, a.n, a.h, a.c, dr, nbins, bins, p->stream) != hipSuccess) return LSFFT_E_DEVICE;
  if (hipMemcpyAsync(hb.data(), bins, sizeof(unsigned long long) * hb.size(), hipMemcpyDeviceToHost, p->stream) !=
          hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess)
    return LSFFT_E_DEVICE;
  rve_finish(hb.data(), a, support_radius, tol, dr, profile, max_bins, out);
  return LSFFT_OK;
}

lsfft_status lsfft_rve_identify_noalloc(lsfft_plan_t p, int grid_idx, const double* avg, const double* center,
                                        double support_radius, double tol, double dr, double* profile, int max_bins,
                                        lsfft_rve* out) {
  RveArgs a;
  lsfft_status ls = rve_args(p, grid_idx, avg, center, support_radius, tol, dr, out, &a);
  if (ls != LSFFT_OK) return ls;
  // the device's copy of the fixed scratch, looked up when the plan was made
  unsigned long long* bins = rve_scratch_ptr(p->device);
  if (!bins) return LSFFT_E_DEVICE;
  if (enter(p) != LSFFT_OK) return LSFFT_E_DEVICE;
  const long long words = 2 * (long long)a.nbins;
  unsigned long long hb[kRveScratchWords];   // host copy of the bins (stack, no allocation)
  if (launch_zero_u64(bins, words, p->stream) != hipSuccess) return LSFFT_E_DEVICE;
  if (launch_radial_max(a.d, avg, a.n, a.h, a.c, dr, a.nbins, bins, p->stream) != hipSuccess) return LSFFT_E_DEVICE;
  if (hipMemcpyAsync(hb, bins, sizeof(unsigned long long) * (size_t)words, hipMemcpyDeviceToHost, p->stream) !=
          hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess)
    return LSFFT_E_DEVICE;
  rve_finish(hb, a, support_radius, tol, dr, profile, max_bins, out);
  return LSFFT_OK;
}

lsfft_status lsfft_kernel_times(lsfft_plan_t p, int kernel_class, double* total_ms, int64_t* launches) {
  if (!p || kernel_class < 0 || kernel_class >= LSFFT_K_COUNT) return LSFFT_E_ARG;
  if (total_ms) *total_ms = p->kt_ms[kernel_class];
  if (launches) *launches = p->kt_n[kernel_class];
  return LSFFT_OK;
}

lsfft_status lsfft_kernel_times_reset(lsfft_plan_t p) {
  if (!p) return LSFFT_E_ARG;
  for (int k = 0; k < LSFFT_K_COUNT; ++k) {
    p->kt_ms[k] = 0;
    p->kt_n[k] = 0;
  }
  return LSFFT_OK;
}

lsfft_status lsfft_iteration_bytes(lsfft_plan_t p, int grid_idx, int kernel_class, double* bytes) {
  if (!p || !bytes || grid_idx < 0 || grid_idx >= (int)p->grids.size()) return LSFFT_E_ARG;
  if (kernel_class < 0 || kernel_class >= LSFFT_K_COUNT) return LSFFT_E_ARG;
  Geometry g;
  if (!geometry(p->f64, p->grids[grid_idx], p->sched, &g, p->layout[grid_idx])) return LSFFT_E_ARG;
  const double comp = (double)g.Pm * (p->f64 ? 16.0 : 8.0);  // one complex half-spectrum stream
  const double s = g.s, d = g.dim;
  const bool cg = p->scheme == LSFFT_CG || p->scheme == LSFFT_CG_PLAIN;
  double b = 0.0;
  switch (kernel_class) {
    case LSFFT_K_XPASS: b = 2 * s * comp + (double)g.nvox; break;          // eps^ in, sigma^ out, phase
    case LSFFT_K_YPASS: b = (g.dim == 3) ? 4 * s * comp : 0.0; break;       // two sweeps, in and out
    case LSFFT_K_GREEN:
      if (p->scheme == LSFFT_ANDERSON) {
        // residual pass: sigma^, f^, x_k, x_{k-1}, F_{k-1}, m - 1 older dF in;
        // F, dF, dU out; update pass: x_k, F, m dU and m dF in; x_{k+1}, eps^ out
        const double m = p->aa_m;
        b = ((s + 4 * d + (m - 1) * d) + 3 * d + (2 * d + 2 * m * d) + (d + s)) * comp;
      } else {
        b = cg ? (s + 2 * d) * comp + (3 * d + s) * comp                    // A p pass + direction pass
               : (2 * s + 3 * d) * comp;                                     // sigma^, u^, f^ in; u^, eps^ out
      }
      break;
    case LSFFT_K_REDUCE:
      b = 8.0 * (p->scheme == LSFFT_ANDERSON ? kAAPart : 2) * std::max(g.items_g, g.items_cg);
      break;
    case LSFFT_K_CGUPD: b = cg ? 6 * d * comp : 0.0; break;
    default: b = 0.0;
  }
  *bytes = b;
  return LSFFT_OK;
}

lsfft_status lsfft_schedule_get(lsfft_plan_t p, int dim, int kind, int len, int* variant, int* nvariants) {
  if (p && kind == 3) {
    // spectral layout of grid `len`
    if (len < 0 || len >= (int)p->grids.size() || p->grids[len].dim != dim) return LSFFT_E_ARG;
    const bool ok = blocked_layout_ok(p->grids[len]);
    if (variant) *variant = ok ? p->layout[len] : 0;
    if (nvariants) *nvariants = ok ? 2 : 1;
    return LSFFT_OK;
  }
  if (!p || (dim != 2 && dim != 3) || kind < 0 || kind > 2 || len_index(len) < 0) return LSFFT_E_ARG;
  if (variant) *variant = plan_variant(p->sched, p->f64, dim, kind, len);
  if (nvariants) *nvariants = schedule_variants(p->f64, dim, kind, len);
  return LSFFT_OK;
}

lsfft_status lsfft_schedule_set(lsfft_plan_t p, int dim, int kind, int len, int variant) {
  if (p && kind == 3) {
    int cur = 0, nv = 0;
    if (lsfft_schedule_get(p, dim, kind, len, &cur, &nv) != LSFFT_OK || variant < 0 || variant >= nv) return LSFFT_E_ARG;
    if (nv == 2) set_layout(p, len, variant);
    return LSFFT_OK;
  }
  if (!p || (dim != 2 && dim != 3) || kind < 0 || kind > 2 || len_index(len) < 0) return LSFFT_E_ARG;
  if (variant < 0 || variant >= schedule_variants(p->f64, dim, kind, len)) return LSFFT_E_ARG;
  if (dim == 3) p->sched[kind][len_index(len)] = variant;   // 2D grids have the default only
  return LSFFT_OK;
}

int lsfft_tune_cache_lookup(const char* json_text, int prec, int dim, int kind, int len) {
  if (!json_text || (prec != LSFFT_F32 && prec != LSFFT_F64) || (dim != 2 && dim != 3) || kind < 0 || kind > 2)
    return -1;
  const auto m = parse_tune_cache(json_text);
  const auto it = m.find(tune_key(prec == LSFFT_F64, dim, kind, len));
  if (it == m.end() || it->second >= schedule_variants(prec == LSFFT_F64, dim, kind, len)) return -1;
  return it->second;
}

lsfft_status lsfft_autotune(lsfft_plan_t p, int iters, const char* cache_path, lsfft_tune_entry* out, int max_out,
                            int* nout) {
  if (check_plan(p) != LSFFT_OK || iters < 1 || iters > 10000 || max_out < 0 || (max_out > 0 && !out)) return LSFFT_E_ARG;
  if (nout) *nout = 0;
  if (enter(p) != LSFFT_OK) return LSFFT_E_DEVICE;
  const size_t rs = p->f64 ? 8 : 4;
  // the tuning problem: two phases (E = 1 and 10, nu = 0.3) in a pattern of
  // 8-voxel blocks, a deterministic pseudo-random force, `iters` iterations
  double lame[4];
  const double e_nu[4] = {1.0, 0.3, 10.0, 0.3};
  if (lsfft_lame_from_young(2, e_nu, lame) != LSFFT_OK) return LSFFT_E_ARG;
  lsfft_phases tab{2, lame};
  // the distinct 3D grids, each with its synthetic inputs on the device
  struct TuneGrid {
    int gi;
    void* ph = nullptr;
    void* f = nullptr;
  };
  std::vector<TuneGrid> tg;
  struct Release {
    std::vector<TuneGrid>* v;
    ~Release() {
      for (auto& t : *v) {
        if (t.ph) (void)hipFree(t.ph);
        if (t.f) (void)hipFree(t.f);
      }
    }
  } release{&tg};
  for (size_t gi = 0; gi < p->grids.size(); ++gi) {
    const lsfft_grid& g = p->grids[gi];
    if (g.dim != 3) continue;
    bool seen = false;
    for (const auto& t : tg) {
      const lsfft_grid& h = p->grids[t.gi];
      seen = seen || (h.n[0] == g.n[0] && h.n[1] == g.n[1] && h.n[2] == g.n[2]);
    }
    if (seen) continue;
    const int lens[3] = {(int)gnx(g), (int)gny(g), (int)gnz(g)};
    bool tuned = blocked_layout_ok(g);
    for (int k = 0; k < 3; ++k) tuned = tuned || schedule_variants(p->f64, 3, k, lens[k]) > 1;
    if (!tuned) continue;
    const long long nvox = (long long)lens[0] * lens[1] * lens[2];
    std::vector<uint8_t> hph((size_t)nvox);
    std::vector<double> hf(3 * (size_t)nvox);
    unsigned long long st = 0x9e3779b97f4a7c15ull;
    for (long long v = 0; v < nvox; ++v) {
      const long long x = v % lens[0], y = (v / lens[0]) % lens[1], z = v / ((long long)lens[0] * lens[1]);
      hph[(size_t)v] = (uint8_t)(((x / 8) + (y / 8) + (z / 8)) % 3 == 0);
    }
    for (double& q : hf) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      q = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    tg.push_back(TuneGrid{(int)gi});
    TuneGrid& t = tg.back();
    if (hipMalloc(&t.ph, (size_t)nvox) != hipSuccess || hipMalloc(&t.f, 3 * (size_t)nvox * rs) != hipSuccess)
      return LSFFT_E_ALLOC;
    hipError_t he = hipMemcpy(t.ph, hph.data(), (size_t)nvox, hipMemcpyHostToDevice);
    if (he == hipSuccess) {
      if (p->f64) {
        he = hipMemcpy(t.f, hf.data(), 3 * (size_t)nvox * rs, hipMemcpyHostToDevice);
      } else {
        std::vector<float> ff(hf.begin(), hf.end());
        he = hipMemcpy(t.f, ff.data(), 3 * (size_t)nvox * rs, hipMemcpyHostToDevice);
      }
    }
    if (he != hipSuccess) return LSFFT_E_DEVICE;
  }
  // `iters` timed iterations of a batch of identical solves of one grid with
  // the plan's current schedules and layouts: as many solves as fill about
  // 64 M voxels, within the plan's batch size, as a batch of the plan's size
  // would.  A single solve of a small grid leaves most of the 256 CUs idle
  // and times the launch latency instead of the pass (at 96^3 it ranked the
  // tiles the other way round), and a batch whose spectra fit the 256 MB
  // Infinity Cache ranks the layouts differently from one that streams from
  // HBM (at 96^3, 9 solves favoured rows, the 64 of a 512-solve batch the
  // blocked layout).  They share one force spectrum.  The kernel times are
  // left in kt_ms.
  auto time_grid = [&](const TuneGrid& t) -> lsfft_status {
    const lsfft_grid& g = p->grids[t.gi];
    const long long nvox = gnx(g) * gny(g) * gnz(g);
    const int nrep = (int)std::max(1LL, std::min((long long)p->max_batch, (64LL << 20) / nvox));
    Batch b;
    b.p = p;
    b.tol = 1e-300;
    b.max_iter = iters;
    Spec sp;
    sp.grid = t.gi;
    sp.phase = static_cast<const uint8_t*>(t.ph);
    sp.tab = &tab;
    (void)resolve_ref(&tab, nullptr, &sp.lam0, &sp.mu0);
    sp.f = t.f;
    sp.leader = 0;
    for (int k = 0; k < nrep; ++k) {
      sp.out_index = k;
      b.specs.push_back(sp);
    }
    std::vector<lsfft_report> reps((size_t)nrep);
    lsfft_kernel_times_reset(p);
    p->force_timing = true;
    const lsfft_status rs_ = run_batch(b, reps.data(), now_s());
    p->force_timing = false;
    if (rs_ == LSFFT_E_ARG || rs_ == LSFFT_E_ALLOC || rs_ == LSFFT_E_DEVICE) return rs_;
    return LSFFT_OK;
  };
  // Per grid and layout (the kx-blocked one first, then rows, where the
  // grid has both), one round per variant index with
  // every pass of the grid on that variant (or its default where it has
  // fewer): kernel ms per iteration of each pass kind.
  const int cls[3] = {LSFFT_K_XPASS, LSFFT_K_YPASS, LSFFT_K_GREEN};
  const double per_iter[3] = {1.0, 2.0, p->scheme == LSFFT_BASIC ? 1.0 : 2.0};   // CG, Anderson: two outer launches
  struct GridTimes {
    int nl = 1, lay[2] = {0, 0}, nv[3] = {1, 1, 1}, lens[3] = {0, 0, 0}, rounds = 1;
    std::vector<std::array<double, 3>> ms[2];
  };
  std::vector<GridTimes> gt(tg.size());
  for (size_t ti = 0; ti < tg.size(); ++ti) {
    const TuneGrid& t = tg[ti];
    GridTimes& G = gt[ti];
    const lsfft_grid& g = p->grids[t.gi];
    G.lens[0] = (int)gnx(g);
    G.lens[1] = (int)gny(g);
    G.lens[2] = (int)gnz(g);
    for (int k = 0; k < 3; ++k) {
      G.nv[k] = schedule_variants(p->f64, 3, k, G.lens[k]);
      G.rounds = std::max(G.rounds, G.nv[k]);
    }
    const bool two = blocked_layout_ok(g);
    G.nl = two ? 2 : 1;
    G.lay[0] = two ? 1 : p->layout[t.gi];
    int keep[3];
    for (int k = 0; k < 3; ++k) keep[k] = p->sched[k][len_index(G.lens[k])];
    lsfft_status ls = LSFFT_OK;
    for (int l = 0; l < G.nl && ls == LSFFT_OK; ++l) {
      for (size_t gj = 0; gj < p->grids.size(); ++gj)
        if (same_shape(p->grids[gj], g)) set_layout(p, (int)gj, G.lay[l]);
      G.ms[l].assign(G.rounds, std::array<double, 3>{0.0, 0.0, 0.0});
      for (int r = 0; r < G.rounds; ++r) {
        for (int k = 0; k < 3; ++k) p->sched[k][len_index(G.lens[k])] = r < G.nv[k] ? r : 0;
        if ((ls = time_grid(t)) != LSFFT_OK) break;
        for (int k = 0; k < 3; ++k) G.ms[l][r][k] = p->kt_ms[cls[k]] / iters;
      }
    }
    for (int k = 0; k < 3; ++k) p->sched[k][len_index(G.lens[k])] = keep[k];
    lsfft_kernel_times_reset(p);
    if (ls != LSFFT_OK) return ls;
  }
  // Layout per grid: the smaller kernel time of the three passes per
  // iteration, each pass on its fastest variant under that layout (ties go
  // to the blocked layout).
  std::map<std::string, int> chosen;
  std::vector<int> li(tg.size(), 0);
  int n = 0;
  std::vector<lsfft_tune_entry> lay_rows;
  for (size_t ti = 0; ti < tg.size(); ++ti) {
    const GridTimes& G = gt[ti];
    const lsfft_grid& g = p->grids[tg[ti].gi];
    double cost[2] = {0.0, 0.0};
    for (int l = 0; l < G.nl; ++l)
      for (int k = 0; k < 3; ++k) {
        double best = G.ms[l][0][k];
        for (int r = 1; r < G.nv[k]; ++r) best = std::min(best, G.ms[l][r][k]);
        cost[l] += best;
      }
    li[ti] = (G.nl == 2 && cost[1] < cost[0]) ? 1 : 0;
    for (size_t gj = 0; gj < p->grids.size(); ++gj)
      if (same_shape(p->grids[gj], g)) set_layout(p, (int)gj, G.lay[li[ti]]);
    if (G.nl == 2) {
      chosen[layout_key(p->f64, g)] = G.lay[li[ti]];
      for (int l = 0; l < 2; ++l)
        lay_rows.push_back(lsfft_tune_entry{3, tg[ti].gi, G.lay[l], l == li[ti] ? 1 : 0, 1e3 * cost[l]});
    }
  }
  // Variant per (kind, length): mean kernel time per launch, summed over the
  // grids sharing that length, each under its chosen layout.
  std::map<std::pair<int, int>, std::vector<double>> times;
  for (size_t ti = 0; ti < tg.size(); ++ti) {
    const GridTimes& G = gt[ti];
    for (int k = 0; k < 3; ++k) {
      if (G.nv[k] == 1) continue;   // passes with the default only are not tuned
      auto& v = times[{k, G.lens[k]}];
      if ((int)v.size() < G.nv[k]) v.resize(G.nv[k], 0.0);
      for (int r = 0; r < G.nv[k]; ++r) v[r] += 1e3 * G.ms[li[ti]][r][k] / per_iter[k];
    }
  }
  for (const auto& kv : times) {
    const int kind = kv.first.first, len = kv.first.second;
    const auto& v = kv.second;
    int best = 0;
    for (int r = 1; r < (int)v.size(); ++r)
      if (v[r] < v[best]) best = r;
    p->sched[kind][len_index(len)] = best;
    chosen[tune_key(p->f64, 3, kind, len)] = best;
    for (int r = 0; r < (int)v.size(); ++r, ++n)
      if (n < max_out) out[n] = lsfft_tune_entry{kind, len, r, r == best ? 1 : 0, v[r]};
  }
  for (const auto& e : lay_rows) {
    if (n < max_out) out[n] = e;
    ++n;
  }
  if (nout) *nout = n;
  if (cache_path && !chosen.empty()) {
    std::lock_guard<std::mutex> lock(tune_file_mu);
    std::string text;
    std::map<std::string, int> m;
    if (read_file(cache_path, &text)) m = parse_tune_cache(text.c_str());
    for (const auto& kv : chosen) m[kv.first] = kv.second;
    if (!write_tune_cache(cache_path, m)) return LSFFT_E_ARG;
  }
  return LSFFT_OK;
}

lsfft_status lsfft_anderson_memory(lsfft_plan_t p, int m) {
  if (!p || m < 1 || m > kAAMax) return LSFFT_E_ARG;
  p->aa_m = m;
  return LSFFT_OK;
}

lsfft_status lsfft_kernel_convolve(lsfft_plan_t p, int grid_idx, const void* kernel, int nforce,
                                   const void* const* f, void* const* out) {
  if (check_plan(p) != LSFFT_OK || !kernel || nforce < 1 || !f || !out) return LSFFT_E_ARG;
  if (grid_idx < 0 || grid_idx >= (int)p->grids.size()) return LSFFT_E_ARG;
  for (int i = 0; i < nforce; ++i)
    if (!f[i] || !out[i]) return LSFFT_E_ARG;
  const lsfft_grid& gr = p->grids[grid_idx];
  Geometry geo;
  if (!geometry(p->f64, gr, p->sched, &geo, p->layout[grid_idx])) return LSFFT_E_ARG;
  const int d = geo.dim, s = geo.s;
  const size_t rs = p->f64 ? 8 : 4, cs = 2 * rs;
  if (!p->kspec.ensure(cs * (size_t)(s * d) * (size_t)geo.Pc)) return LSFFT_E_ALLOC;
  if (!p->zphase.ensure((size_t)geo.nvox)) return LSFFT_E_ALLOC;
  if (enter(p) != LSFFT_OK) return LSFFT_E_DEVICE;
  // the pass kernels read a phase map (Hooke's law in the x pass runs
  // whatever its output): one phase of unit moduli, unused here
  LSFFT_TRY(hipMemsetAsync(p->zphase.p, 0, (size_t)geo.nvox, p->stream));
  const double lame1[2] = {1.0, 1.0};
  lsfft_phases tab{1, lame1};
  auto spec_of = [&](const void* src, void* eps) {
    Spec sp;
    sp.grid = grid_idx;
    sp.phase = static_cast<const uint8_t*>(p->zphase.p);
    sp.tab = &tab;
    sp.lam0 = 1.0;
    sp.mu0 = 1.0;
    sp.f = src;
    sp.eps = eps;
    return sp;
  };
  // kernel spectrum: the force transform of the s rows [d][N] of the kernel,
  // each as one transform group, into consecutive rows of kspec
  {
    Batch kb;
    kb.p = p;
    kb.max_iter = 0;
    for (int c = 0; c < s; ++c) {
      kb.specs.push_back(spec_of(static_cast<const char*>(kernel) + (size_t)c * d * geo.nvox * rs, nullptr));
      kb.specs.back().leader = c;
    }
    lsfft_status ls = prepare(kb, false);
    if (ls != LSFFT_OK) return ls;
    if (host_fence(p) != LSFFT_OK) return LSFFT_E_DEVICE;
    for (int c = 0; c < s; ++c) kb.desc[c].F = static_cast<char*>(p->kspec.p) + (size_t)c * d * geo.Pc * cs;
    std::memcpy(hptr<InstDesc>(kb, 0), kb.desc.data(), sizeof(InstDesc) * s);
    if ((ls = h2d(kb, 0, sizeof(InstDesc) * s)) != LSFFT_OK) return ls;
    p->timing_active = false;
    LSFFT_TRY(pass_x(kb, L_XLEAD, M_FT, LSFFT_K_OTHER));
    LSFFT_TRY(pass_y(kb, L_YLEAD, -1, 1, 3, 0, LSFFT_K_OTHER));
    LSFFT_TRY(pass_g(kb, L_GLEAD, M_FT, LSFFT_K_OTHER));
    LSFFT_TRY(hipStreamSynchronize(p->stream));
  }
  // the forces, in batches of at most max_batch: force transform, product
  // with the kernel spectrum, inverse transforms of the s strain components
  for (int start = 0; start < nforce; start += p->max_batch) {
    const int cnt = std::min(p->max_batch, nforce - start);
    Batch b;
    b.p = p;
    b.max_iter = 0;
    for (int i = 0; i < cnt; ++i) {
      b.specs.push_back(spec_of(f[start + i], out[start + i]));
      b.specs.back().leader = i;
    }
    lsfft_status ls = prepare(b, false);
    if (ls != LSFFT_OK) return ls;
    if (host_fence(p) != LSFFT_OK) return LSFFT_E_DEVICE;
    for (int i = 0; i < cnt; ++i) b.desc[i].Kh = p->kspec.p;
    std::memcpy(hptr<InstDesc>(b, 0), b.desc.data(), sizeof(InstDesc) * cnt);
    if ((ls = h2d(b, 0, sizeof(InstDesc) * cnt)) != LSFFT_OK) return ls;
    LSFFT_TRY(pass_x(b, L_XLEAD, M_FT, LSFFT_K_OTHER));
    LSFFT_TRY(pass_y(b, L_YLEAD, -1, 1, 3, 0, LSFFT_K_OTHER));
    LSFFT_TRY(pass_g(b, L_GLEAD, M_FT, LSFFT_K_OTHER));
    LSFFT_TRY(pass_g(b, L_GALL, M_KCONV, LSFFT_K_OTHER));
    LSFFT_TRY(pass_y(b, L_YALL, +1, 0, s, 0, LSFFT_K_OTHER));
    LSFFT_TRY(pass_x(b, L_XALL, M_MAT, LSFFT_K_OTHER));
    LSFFT_TRY(hipStreamSynchronize(p->stream));
  }
  return LSFFT_OK;
}

namespace {
// the device a plan-free entry point runs on, and its stream
hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }
}  // namespace

lsfft_status lsfft_block_mean(int prec, int out_prec, int nfield, const int64_t* n, int factor, double scale,
                              const void* in, void* out, void* hip_stream) {
  if ((prec != LSFFT_F32 && prec != LSFFT_F64) || (out_prec != LSFFT_F32 && out_prec != LSFFT_F64)) return LSFFT_E_ARG;
  if (nfield < 1 || !n || !in || !out || factor < 1) return LSFFT_E_ARG;
  if (!is_fin(scale)) return LSFFT_E_ARG;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1 || n[a] > (1 << 20)) return LSFFT_E_ARG;
    if ((a < 2 || n[a] > 1) && n[a] % factor != 0) return LSFFT_E_ARG;
  }
  if (n[0] * n[1] * n[2] > (1ll << 40)) return LSFFT_E_ARG;
  if (launch_block_mean(prec == LSFFT_F64, out_prec == LSFFT_F64, in, out, nfield, (int)n[0], (int)n[1], (int)n[2],
                        factor, scale, as_stream(hip_stream)) != hipSuccess)
    return LSFFT_E_DEVICE;
  return hipStreamSynchronize(as_stream(hip_stream)) == hipSuccess ? LSFFT_OK : LSFFT_E_DEVICE;
}

lsfft_status lsfft_sample_norms(int prec, int nsample, int64_t len, const void* y, const void* t, double* norm_diff,
                                double* norm_t, void* hip_stream) {
  if ((prec != LSFFT_F32 && prec != LSFFT_F64) || nsample < 1 || nsample > (1 << 24) || len < 1 || !t)
    return LSFFT_E_ARG;
  double* dres = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&dres), sizeof(double) * 2 * (size_t)nsample) != hipSuccess)
    return LSFFT_E_ALLOC;
  std::vector<double> h(2 * (size_t)nsample);
  hipStream_t st = as_stream(hip_stream);
  hipError_t e = launch_sample_norms(prec == LSFFT_F64, y, t, nsample, len, dres, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), dres, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dres);
  if (e != hipSuccess) return LSFFT_E_DEVICE;
  for (int i = 0; i < nsample; ++i) {
    if (norm_diff) norm_diff[i] = h[2 * (size_t)i];
    if (norm_t) norm_t[i] = h[2 * (size_t)i + 1];
  }
  return LSFFT_OK;
}

lsfft_status lsfft_bump_forces(int prec, int dim, const int64_t* n, int nforce, const int* nbump,
                               const double* bumps, void* const* f, void* hip_stream) {
  if ((prec != LSFFT_F32 && prec != LSFFT_F64) || (dim != 2 && dim != 3) || !n || nforce < 1 || !nbump || !f)
    return LSFFT_E_ARG;
  if (nforce > 65535) return LSFFT_E_ARG;
  int nz = dim == 3 ? (int)n[2] : 1;
  for (int a = 0; a < dim; ++a)
    if (n[a] < 1 || n[a] > (1 << 16)) return LSFFT_E_ARG;
  std::vector<int> first(nforce + 1, 0);
  for (int i = 0; i < nforce; ++i) {
    if (nbump[i] < 0 || !f[i]) return LSFFT_E_ARG;
    first[i + 1] = first[i] + nbump[i];
  }
  const int total = first[nforce];
  if (total > 0 && !bumps) return LSFFT_E_ARG;
  // per bump (centre x, y, z, radius, direction x, y, z); the caller gives dim + 1 + dim values
  std::vector<double> packed(7 * (size_t)std::max(total, 1), 0.0);
  for (int b = 0; b < total; ++b) {
    const double* src = bumps + (size_t)b * (2 * dim + 1);
    for (int a = 0; a < dim; ++a) packed[7 * (size_t)b + a] = src[a];
    packed[7 * (size_t)b + 3] = src[dim];
    for (int a = 0; a < dim; ++a) packed[7 * (size_t)b + 4 + a] = src[dim + 1 + a];
    if (!is_fin(src[dim]) || src[dim] <= 0.0) return LSFFT_E_ARG;
    for (int k = 0; k < 2 * dim + 1; ++k)
      if (!is_fin(src[k])) return LSFFT_E_ARG;
  }
  hipStream_t st = as_stream(hip_stream);
  char* dbuf = nullptr;
  const size_t b_first = sizeof(int) * first.size(), b_bumps = sizeof(double) * packed.size(),
               b_ptrs = sizeof(void*) * (size_t)nforce;
  const size_t o_bumps = align_up(b_first, 16), o_ptrs = align_up(o_bumps + b_bumps, 16);
  if (hipMalloc(reinterpret_cast<void**>(&dbuf), o_ptrs + b_ptrs) != hipSuccess) return LSFFT_E_ALLOC;
  hipError_t e = hipMemcpy(dbuf, first.data(), b_first, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dbuf + o_bumps, packed.data(), b_bumps, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dbuf + o_ptrs, f, b_ptrs, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = launch_bump_forces(prec == LSFFT_F64, reinterpret_cast<void* const*>(dbuf + o_ptrs),
                           reinterpret_cast<const int*>(dbuf), reinterpret_cast<const double*>(dbuf + o_bumps), nforce,
                           (int)n[0], (int)n[1], nz, dim, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dbuf);
  return e == hipSuccess ? LSFFT_OK : LSFFT_E_DEVICE;
}

}  // extern "C"

namespace {
// The horizon of the nonlocal operator (Eq. 6.5 on the grid, h = 1): the
// offsets r != 0 with |r| < delta (z = 0 in 2D), grouped in shells of equal
// |r|^2 in ascending order, as index deltas of the kernels' LDS box of halo
// R (the largest offset component), with the Bernstein values of degree
// `deg` at each shell's radius.
struct NlHorizon {
  int R = 0;
  std::vector<int> delta, first;   // offsets of shell q: delta[first[q] .. first[q + 1])
  std::vector<double> rho;         // per shell
  std::vector<double> ee;          // per offset, e_a e_b at (o 3 + b) 3 + a (x first)
  int nshell() const { return (int)rho.size(); }
};

// one_voxel: the deltas of the tiles of the matrix-form normal equations
bool nl_horizon(int dim, double delta, bool one_voxel, NlHorizon& h) {
  if (!is_fin(delta) || delta <= 1.0 || delta > kNlMaxHalo + 1) return false;
  const int R = (int)std::ceil(delta) - 1;
  int box[3];
  nl_box(dim, R, one_voxel, box);
  struct Off {
    int delta;
    double e[3];
  };
  std::map<int, std::vector<Off>> shells;   // |r|^2 -> offsets
  const int rz = dim == 3 ? R : 0;
  for (int dz = -rz; dz <= rz; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int rr = dx * dx + dy * dy + dz * dz;
        const double rho = std::sqrt(double(rr));
        if (rr == 0 || !(rho < delta)) continue;
        shells[rr].push_back({(dz * box[1] + dy) * box[0] + dx, {dx / rho, dy / rho, dz / rho}});
      }
  if (shells.empty()) return false;
  h.R = R;
  h.first.push_back(0);
  for (const auto& kv : shells) {
    for (const Off& o : kv.second) {
      h.delta.push_back(o.delta);
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) h.ee.push_back(o.e[a] * o.e[b]);
    }
    h.first.push_back((int)h.delta.size());
    h.rho.push_back(std::sqrt(double(kv.first)));
  }
  return true;
}

// B_{m,M}(rho / delta) for m = 0..M per shell, [M + 1][nshell]
std::vector<double> nl_bernstein(int M, double delta, const NlHorizon& h) {
  std::vector<double> W((size_t)(M + 1) * h.nshell());
  for (int q = 0; q < h.nshell(); ++q) {
    const double t = h.rho[q] / delta;
    double binom = 1.0;
    for (int m = 0; m <= M; ++m) {
      if (m > 0) binom = binom * (M - m + 1) / m;
      W[(size_t)m * h.nshell() + q] = binom * std::pow(t, m) * std::pow(1.0 - t, M - m);
    }
  }
  return W;
}

// device copy of the horizon tables (ints, then the direction products and
// the caller's doubles), freed by the caller
struct NlTables {
  char* buf = nullptr;
  const int* delta = nullptr;
  const int* first = nullptr;
  const double* ee = nullptr;
  const double* vals = nullptr;
  double* work = nullptr;
};

hipError_t nl_upload(const NlHorizon& h, const std::vector<double>& vals, size_t work_doubles, hipStream_t st,
                     NlTables& t) {
  const size_t b_delta = sizeof(int) * h.delta.size(), b_first = sizeof(int) * h.first.size();
  const size_t b_ee = sizeof(double) * h.ee.size();
  const size_t o_first = align_up(b_delta, 16), o_ee = align_up(o_first + b_first, 16);
  const size_t o_vals = align_up(o_ee + b_ee, 16);
  const size_t o_work = align_up(o_vals + sizeof(double) * vals.size(), 256);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&t.buf), o_work + sizeof(double) * std::max<size_t>(work_doubles, 1));
  if (e != hipSuccess) {
    t.buf = nullptr;
    return e;
  }
  t.delta = reinterpret_cast<const int*>(t.buf);
  t.first = reinterpret_cast<const int*>(t.buf + o_first);
  t.ee = reinterpret_cast<const double*>(t.buf + o_ee);
  t.vals = reinterpret_cast<const double*>(t.buf + o_vals);
  t.work = reinterpret_cast<double*>(t.buf + o_work);
  e = hipMemcpyAsync(t.buf, h.delta.data(), b_delta, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(t.buf + o_first, h.first.data(), b_first, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(t.buf + o_ee, h.ee.data(), b_ee, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(t.buf + o_vals, vals.data(), sizeof(double) * vals.size(), hipMemcpyHostToDevice, st);
  return e;
}

lsfft_status nl_check(int prec, int dim, const int64_t* n, int nsample, int n_out[3]) {
  if ((prec != LSFFT_F32 && prec != LSFFT_F64) || (dim != 2 && dim != 3) || !n || nsample < 1) return LSFFT_E_ARG;
  for (int a = 0; a < 3; ++a) n_out[a] = 1;
  long long nvox = 1;
  for (int a = 0; a < dim; ++a) {
    if (n[a] < 1 || n[a] > (1 << 16)) return LSFFT_E_ARG;
    n_out[a] = (int)n[a];
    nvox *= n[a];
  }
  if (nvox * dim * nsample > (1ll << 40)) return LSFFT_E_ARG;
  return LSFFT_OK;
}
}  // namespace

extern "C" {

lsfft_status lsfft_nonlocal_normal_equations(int prec, int dim, const int64_t* n, int nsample, const void* u,
                                             const void* gamma, int degree, int form, double delta, double* G,
                                             double* g, double* gg, void* hip_stream) {
  int nn[3];
  if (nl_check(prec, dim, n, nsample, nn) != LSFFT_OK || !u || !gamma || !G || !g || !gg) return LSFFT_E_ARG;
  if (degree < 0 || degree > kNlMaxDegree || (form != 0 && form != 1)) return LSFFT_E_ARG;
  NlHorizon h;
  if (!nl_horizon(dim, delta, form == 1, h)) return LSFFT_E_ARG;
  if (form == 1 && dim == 3 && h.R > kNlMaxHalo1) return LSFFT_E_ARG;
  const std::vector<double> W = nl_bernstein(degree, delta, h);
  hipStream_t st = as_stream(hip_stream);
  NlTables t;
  const size_t work = (size_t)kNlGramSlots * kNlAccWords1 + kNlAccWords1;
  hipError_t e = nl_upload(h, W, work, st, t);
  if (!t.buf) return LSFFT_E_ALLOC;
  double* out = t.work + (size_t)kNlGramSlots * kNlAccWords1;
  std::vector<double> acc(kNlAccWords1);
  if (e == hipSuccess)
    e = launch_nl_gram(prec == LSFFT_F64, dim, nn, h.R, degree, form, nsample, u, gamma, t.delta, t.first, t.ee,
                       h.nshell(), t.vals, t.work, out, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(acc.data(), out, sizeof(double) * (form == 0 ? kNlAccWords : kNlAccWords1),
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(t.buf);
  if (e != hipSuccess) return LSFFT_E_DEVICE;
  // unpack the upper triangle: form 0 laid out for degree kNlMaxDegree,
  // form 1 for its own nf = 2 (degree + 1) features
  const int nf = (form == 0 ? 1 : 2) * (degree + 1);
  const int F = form == 0 ? kNlMaxDegree + 1 : nf;
  for (int m = 0; m < nf; ++m)
    for (int k = m; k < nf; ++k) {
      const double v = acc[(size_t)(m * F - m * (m - 1) / 2 + (k - m))];
      G[m * nf + k] = v;
      G[k * nf + m] = v;
    }
  const int tri = F * (F + 1) / 2;
  for (int m = 0; m < nf; ++m) g[m] = acc[(size_t)(tri + m)];
  *gg = acc[(size_t)(tri + F)];
  return LSFFT_OK;
}

lsfft_status lsfft_nonlocal_apply(int prec, int dim, const int64_t* n, int nsample, const void* u, int degree,
                                  int form, const double* c, double delta, void* out, void* hip_stream) {
  int nn[3];
  if (nl_check(prec, dim, n, nsample, nn) != LSFFT_OK || !u || !c || !out) return LSFFT_E_ARG;
  if (degree < 0 || degree > kNlMaxDegree || (form != 0 && form != 1)) return LSFFT_E_ARG;
  const int nf1 = degree + 1, nc = (form + 1) * nf1;
  for (int m = 0; m < nc; ++m)
    if (!is_fin(c[m])) return LSFFT_E_ARG;
  NlHorizon h;
  if (!nl_horizon(dim, delta, false, h)) return LSFFT_E_ARG;
  const std::vector<double> W = nl_bernstein(degree, delta, h);
  // K1 (and K2) at each shell's radius, one table after the other
  std::vector<double> kw((size_t)(form + 1) * h.nshell(), 0.0);
  for (int f = 0; f <= form; ++f)
    for (int q = 0; q < h.nshell(); ++q)
      for (int m = 0; m <= degree; ++m)
        kw[(size_t)f * h.nshell() + q] += c[f * nf1 + m] * W[(size_t)m * h.nshell() + q];
  hipStream_t st = as_stream(hip_stream);
  NlTables t;
  hipError_t e = nl_upload(h, kw, 0, st, t);
  if (!t.buf) return LSFFT_E_ALLOC;
  if (e == hipSuccess)
    e = launch_nl_apply(prec == LSFFT_F64, dim, nn, h.R, form, nsample, u, t.delta, t.first, t.ee, h.nshell(),
                        t.vals, t.vals + (form == 1 ? h.nshell() : 0), out, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(t.buf);
  return e == hipSuccess ? LSFFT_OK : LSFFT_E_DEVICE;
}

lsfft_status lsfft_nonlocal_fit(int ncoef, const double* G, const double* g, double lam, int adam_steps, double lr,
                                double* c) {
  if (ncoef < 1 || ncoef > 2 * (kNlMaxDegree + 1) || !G || !g || !c || !is_fin(lam) || lam < 0.0 || adam_steps < 0)
    return LSFFT_E_ARG;
  const int nf = ncoef;
  for (int i = 0; i < nf * nf; ++i)
    if (!is_fin(G[i])) return LSFFT_E_ARG;
  for (int i = 0; i < nf; ++i)
    if (!is_fin(g[i])) return LSFFT_E_ARG;
  if (adam_steps == 0) {
    // (G + lam I) c = g by Cholesky; a pivot that is not positive means the
    // system is singular (or G is not a Gram matrix)
    std::vector<double> L((size_t)nf * nf, 0.0);
    for (int j = 0; j < nf; ++j) {
      double d = G[j * nf + j] + lam;
      for (int k = 0; k < j; ++k) d -= L[j * nf + k] * L[j * nf + k];
      if (!(d > 0.0)) return LSFFT_E_ARG;
      L[j * nf + j] = std::sqrt(d);
      for (int i = j + 1; i < nf; ++i) {
        double v = G[i * nf + j];
        for (int k = 0; k < j; ++k) v -= L[i * nf + k] * L[j * nf + k];
        L[i * nf + j] = v / L[j * nf + j];
      }
    }
    std::vector<double> y(nf);
    for (int i = 0; i < nf; ++i) {
      double v = g[i];
      for (int k = 0; k < i; ++k) v -= L[i * nf + k] * y[k];
      y[i] = v / L[i * nf + i];
    }
    for (int i = nf - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < nf; ++k) v -= L[k * nf + i] * c[k];
      c[i] = v / L[i * nf + i];
    }
    return LSFFT_OK;
  }
  // Adam (Kingma and Ba) on the quadratic loss c^T G c - 2 g . c + lam |c|^2
  // from c = 0: gradient 2 (G c - g + lam c), beta1 0.9, beta2 0.999,
  // eps 1e-12, bias-corrected moments, step lr
  if (!is_fin(lr) || lr <= 0.0) return LSFFT_E_ARG;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-12;
  std::vector<double> m(nf, 0.0), v(nf, 0.0), grad(nf);
  for (int i = 0; i < nf; ++i) c[i] = 0.0;
  for (int k = 1; k <= adam_steps; ++k) {
    for (int i = 0; i < nf; ++i) {
      double gc = 0.0;
      for (int j = 0; j < nf; ++j) gc += G[i * nf + j] * c[j];
      grad[i] = 2.0 * (gc - g[i]) + 2.0 * lam * c[i];
    }
    const double c1 = 1.0 - std::pow(b1, k), c2 = 1.0 - std::pow(b2, k);
    for (int i = 0; i < nf; ++i) {
      m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
      v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
      c[i] -= lr * (m[i] / c1) / (std::sqrt(v[i] / c2) + eps);
    }
  }
  return LSFFT_OK;
}

}  // extern "C"
