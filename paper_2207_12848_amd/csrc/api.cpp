// Host side of the sweep library: the C ABI declared in include/sweep.h.
//
// Validation, DAG construction (count -> Kahn levels -> row lengths -> scan ->
// rows), workspace management and the pass sequences of the forward sweep
// (periodic passes inside source iterations) and of the adjoint (reverse
// iterations with recomputation from the saved direction sums).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "sweep.h"

using sweep::Unit;

namespace {

thread_local std::string g_err;

sweep_status_t fail(sweep_status_t st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

sweep_status_t hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? SWEEP_ERR_OOM : SWEEP_ERR_HIP, "%s: %s", what,
              hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);   \
  } while (0)

#define ST_TRY(expr)                        \
  do {                                      \
    sweep_status_t s_ = (expr);             \
    if (s_ != SWEEP_OK) return s_;          \
  } while (0)

// ---------------------------------------------------------------- device memory
// Building a DAG allocates several large buffers and a caller typically builds,
// sweeps and destroys one DAG after another; hipMalloc/hipFree of gigabytes on
// every build would cost milliseconds (hipFree also synchronises the device).
// Released buffers therefore go to a per-device cache and are handed out again
// to later requests of a similar size.  Stream order is kept with events: a
// buffer is released with an event recorded on the stream that last used it
// (the calling thread's current stream, see StreamScope), and whoever takes it
// from the cache makes its own stream wait for that event first.
thread_local hipStream_t g_cur_stream = nullptr;
thread_local bool g_release_synced = false;  // the device is idle: release without an event

// Sets the calling thread's current stream for allocations and releases.
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(g_cur_stream) { g_cur_stream = s; }
  ~StreamScope() { g_cur_stream = prev; }
};

struct CachedBlock {
  void* p;
  size_t bytes;
  int device;
  hipEvent_t ready;  // recorded when the block was released (may be null)
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;

void cache_trim_all() {
  std::vector<CachedBlock> blocks;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    blocks.swap(g_cache);
  }
  if (!blocks.empty()) (void)hipDeviceSynchronize();
  for (CachedBlock& b : blocks) {
    if (b.ready) (void)hipEventDestroy(b.ready);
    (void)hipFree(b.p);
  }
}

hipError_t cached_malloc(void** p, size_t* bytes, size_t n) {
  // sizes are rounded to 2 KiB (small) or 2 MiB (large) so that repeated builds
  // of similar meshes reuse the same blocks
  n = n <= (8u << 20) ? (n + 2047) / 2048 * 2048 : (n + (2u << 20) - 1) / (2u << 20) * (2u << 20);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    int best = -1;
    for (int i = 0; i < (int)g_cache.size(); ++i) {
      const CachedBlock& b = g_cache[i];
      if (b.device != dev || b.bytes < n || b.bytes > n + n / 4 + (1u << 20)) continue;
      if (best < 0 || b.bytes < g_cache[best].bytes) best = i;
    }
    if (best >= 0) {
      CachedBlock b = g_cache[best];
      g_cache.erase(g_cache.begin() + best);
      if (b.ready) {
        (void)hipStreamWaitEvent(g_cur_stream, b.ready, 0);
        (void)hipEventDestroy(b.ready);
      }
      *p = b.p;
      *bytes = b.bytes;
      return hipSuccess;
    }
  }
  e = hipMalloc(p, n);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    cache_trim_all();
    e = hipMalloc(p, n);
  }
  if (e == hipSuccess) *bytes = n;
  return e;
}

void cached_free(void* p, size_t bytes) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipEvent_t ev = nullptr;
  if (g_release_synced) {
    ev = nullptr;
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
    if (hipEventRecord(ev, g_cur_stream) != hipSuccess) {
      (void)hipEventDestroy(ev);
      ev = nullptr;
      (void)hipDeviceSynchronize();
    }
  } else {
    ev = nullptr;
    (void)hipDeviceSynchronize();
  }
  std::lock_guard<std::mutex> g(g_cache_mu);
  g_cache.push_back({p, bytes, dev, ev});
}

// Device buffer owned by the DAG (or a call); released to the cache.
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  ~Buf() { release(); }
  void release() {
    if (p) cached_free(p, bytes);
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    if (n == 0) n = 16;
    hipError_t e = cached_malloc(&p, &bytes, n);
    if (e != hipSuccess) {
      p = nullptr;
      bytes = 0;
    }
    return e;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- kernel timing
struct ProfRec {
  std::string name;
  hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pool_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

thread_local bool g_capturing = false;  // a pass sequence is being captured into a graph

// Brackets one kernel launch with events when profiling is on (not inside a capture).
struct ProfScope {
  hipEvent_t stop = nullptr;
  hipStream_t s;
  ProfScope(const char* name, hipStream_t stream) : s(stream) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on || g_capturing) return;
    hipEvent_t start = pool_event();
    stop = pool_event();
    if (!start || !stop) {
      stop = nullptr;
      return;
    }
    (void)hipEventRecord(start, s);
    g_prof.push_back({name, start, stop});
  }
  ~ProfScope() {
    if (stop) (void)hipEventRecord(stop, s);
  }
};

constexpr int kRedBlock = 256;
constexpr int kNPart = 9;
constexpr int kMaxG = 64;
constexpr int kMaxLds = 160 * 1024;

}  // namespace

struct sweep_dag_s {
  int32_t n_meshes = 0, D = 0;
  int64_t C_total = 0, T = 0;
  int64_t n_up = 0, n_dn = 0;
  double eps = 1e-12;
  bool has_shift = false;
  int device = 0;
  int cu_count = 256;
  int lds_max = 65536 - 256;  // dynamic LDS bytes available to a sweep workgroup
  std::vector<int32_t> mesh_off, mesh_cells;
  std::vector<Unit> units;
  std::vector<int32_t> order;  // units, deepest first
  std::vector<int32_t> identity;
  Buf units_d, order_d, identity_d, sched, indeg, lp, lev_up, lev_dn, up_ptr, dn_ptr, up, dn,
      aperp, aperp_s, vol_s, bnd, vol, counter, blk_base;
  int32_t n_blocks = 0;  // 256-task blocks over all units (prep kernel)
  int32_t max_depth = 0;
  int32_t max_cells = 0;  // cells of the largest mesh
  int32_t kahn_lds = 0;   // the levels were computed with counters in LDS
  int32_t scheme = SWEEP_SCHEME_AREA;
  Buf flag;               // device error bits (see internal.h) raised by asynchronous calls
  std::vector<int64_t> unit_up, unit_dn;  // row entries of every unit
  // step tables of the level-synchronous sweep, one per workgroup size
  struct StepTable {
    int32_t block = 0, cap_e = 0;  // threads, staged entries per step
    Buf k, eu, ed, base, n;
  };
  std::vector<std::unique_ptr<StepTable>> steps;
  // reduction tables (depend on G)
  int32_t red_G = 0, red_blocks = 0, red_cpb = 0;
  Buf blk_mesh, blk_cell0, mesh_off_d, mesh_cells_d, mesh_blk_base;
  // workspaces
  Buf xpass, lam_b;  // periodic adjoint: recomputed passes, the other pass's lambda
  Buf jpass, jscr;   // merged adjoint: every pass's direction sums; J and absorbed scratch
  Buf phi_a, phi_b, phi_w, jsum_a, jsum_b, partial, lam, gsrc, dk64, de64, tden, tsrc, crec, out_s,
      ion_min;
  // periodic half-faces (built with the DAG; see sweep::PinArgs) and, per call, the
  // periodic tasks' own sources and two passes' periodic inflow sums
  Buf pcell, pf_ptr, pnb, pwf, pwa, ptask, pc_map, pbase, pval, psum_a, psum_b;
  int32_t n_pc = 0;
  int64_t n_pf = 0;
  // captured pass sequences (use_graph): key = every argument and buffer they bake in
  struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;  // capture needs a stream other than the null stream
  ~sweep_dag_s() {
    for (GraphEntry& g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace {

bool dag_ok(sweep_dag_t d) { return d != nullptr && d->T > 0; }

sweep_status_t validate_mesh_host(const sweep_mesh_t& m, int idx) {
  const int32_t C = m.n_cells;
  const int64_t F = m.n_half_faces;
  std::vector<int64_t> fp(C + 1);
  std::vector<int32_t> nbr(F), twin;
  std::vector<int8_t> shift;
  std::vector<double> area(F), nrm(3 * F), vol(C);
  HIP_TRY(hipMemcpy(fp.data(), m.face_ptr, sizeof(int64_t) * (C + 1), hipMemcpyDeviceToHost));
  if (F > 0) {
    HIP_TRY(hipMemcpy(nbr.data(), m.face_nbr, sizeof(int32_t) * F, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(area.data(), m.face_area, sizeof(double) * F, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(nrm.data(), m.face_normal, sizeof(double) * 3 * F, hipMemcpyDeviceToHost));
  }
  HIP_TRY(hipMemcpy(vol.data(), m.cell_volume, sizeof(double) * C, hipMemcpyDeviceToHost));
  if (fp[0] != 0 || fp[C] != F)
    return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: face_ptr must run from 0 to n_half_faces", idx);
  for (int32_t c = 0; c < C; ++c) {
    if (fp[c + 1] < fp[c]) return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: face_ptr not monotone at cell %d", idx, c);
    if (!(vol[c] > 0.0) || !std::isfinite(vol[c]))
      return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: cell %d has volume %g", idx, c, vol[c]);
  }
  for (int64_t f = 0; f < F; ++f) {
    if (nbr[f] < -1 || nbr[f] >= C)
      return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: face %lld neighbour %d out of range", idx, (long long)f, nbr[f]);
    if (!(area[f] >= 0.0) || !std::isfinite(area[f]))
      return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: face %lld area %g", idx, (long long)f, area[f]);
    const double n2 = nrm[3 * f] * nrm[3 * f] + nrm[3 * f + 1] * nrm[3 * f + 1] + nrm[3 * f + 2] * nrm[3 * f + 2];
    if (!(std::fabs(std::sqrt(n2) - 1.0) <= 1e-9))
      return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: face %lld normal is not unit", idx, (long long)f);
  }
  if (m.face_shift) {
    shift.resize(F);
    if (F > 0) HIP_TRY(hipMemcpy(shift.data(), m.face_shift, F, hipMemcpyDeviceToHost));
    for (int64_t f = 0; f < F; ++f)
      if (shift[f] != 0 && nbr[f] < 0)
        return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: wall face %lld has a periodic shift", idx, (long long)f);
  }
  if (m.face_twin) {
    twin.resize(F);
    if (F > 0) HIP_TRY(hipMemcpy(twin.data(), m.face_twin, sizeof(int32_t) * F, hipMemcpyDeviceToHost));
    std::vector<int32_t> owner(F);
    for (int32_t c = 0; c < C; ++c)
      for (int64_t f = fp[c]; f < fp[c + 1]; ++f) owner[f] = c;
    for (int64_t f = 0; f < F; ++f) {
      if (nbr[f] < 0) continue;
      const int64_t t = twin[f];
      if (t < 0 || t >= F || twin[t] != f || owner[t] != nbr[f] || nbr[t] != owner[f])
        return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: half-face %lld has no consistent twin", idx, (long long)f);
      if (area[t] != area[f] || nrm[3 * t] != -nrm[3 * f] || nrm[3 * t + 1] != -nrm[3 * f + 1] ||
          nrm[3 * t + 2] != -nrm[3 * f + 2])
        return fail(SWEEP_ERR_INVALID_ARG,
                    "mesh %d: twin half-faces %lld/%lld need equal areas and opposite normals", idx,
                    (long long)f, (long long)t);
      if (!shift.empty() && shift[t] != -shift[f])
        return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: twin half-faces %lld/%lld need opposite shifts",
                    idx, (long long)f, (long long)t);
    }
  }
  return SWEEP_OK;
}

// Per-mesh first cell and cell count on the device (for the reductions).
sweep_status_t ensure_mesh_tables(sweep_dag_t d) {
  if (d->mesh_off_d.p) return SWEEP_OK;
  HIP_TRY(d->mesh_off_d.alloc(4 * d->mesh_off.size()));
  HIP_TRY(d->mesh_cells_d.alloc(4 * d->mesh_cells.size()));
  HIP_TRY(hipMemcpy(d->mesh_off_d.p, d->mesh_off.data(), 4 * d->mesh_off.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d->mesh_cells_d.p, d->mesh_cells.data(), 4 * d->mesh_cells.size(), hipMemcpyHostToDevice));
  return SWEEP_OK;
}

// Reduction block tables for G groups: blocks never straddle meshes.
sweep_status_t ensure_reduce_tables(sweep_dag_t d, int32_t G) {
  if (d->red_G == G) return SWEEP_OK;
  const int cpb = std::max(1, kRedBlock / G);
  std::vector<int32_t> bm, bc, mbb(d->n_meshes + 1, 0);
  for (int m = 0; m < d->n_meshes; ++m) {
    mbb[m] = (int32_t)bm.size();
    for (int32_t c = 0; c < d->mesh_cells[m]; c += cpb) {
      bm.push_back(m);
      bc.push_back(d->mesh_off[m] + c);
    }
  }
  mbb[d->n_meshes] = (int32_t)bm.size();
  HIP_TRY(d->blk_mesh.alloc(bm.size() * 4));
  HIP_TRY(d->blk_cell0.alloc(bc.size() * 4));
  HIP_TRY(d->mesh_blk_base.alloc(mbb.size() * 4));
  HIP_TRY(hipMemcpy(d->blk_mesh.p, bm.data(), bm.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d->blk_cell0.p, bc.data(), bc.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d->mesh_blk_base.p, mbb.data(), mbb.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(d->partial.alloc(bm.size() * (size_t)G * kNPart * sizeof(double)));
  d->red_G = G;
  d->red_blocks = (int32_t)bm.size();
  d->red_cpb = cpb;
  return SWEEP_OK;
}

struct FwdPlan {
  int32_t boundary, n_pbc, n_scat, form, block, ring, use_graph, law, merge, warm, check, grid, pack;
  float albedo;
  double pbc_tol;
};

sweep_status_t read_opts(const sweep_fwd_opts_t* o, FwdPlan* p) {
  p->boundary = o ? o->boundary : SWEEP_BOUNDARY_VACUUM;
  p->n_pbc = o ? o->n_pbc : 1;
  p->n_scat = o ? o->n_scat : 1;
  p->albedo = o ? (float)o->albedo : 0.0f;
  p->form = o ? o->form : SWEEP_FORM_BATCHED;
  p->block = o ? o->block : 0;
  p->ring = o ? o->ring : 0;
  p->use_graph = o ? o->use_graph : 0;
  p->law = o ? o->law : SWEEP_LAW_UPWIND;
  p->merge = o ? (o->merge != 0) : 0;
  p->warm = o ? (o->warm_start != 0) : 0;
  p->pbc_tol = o ? o->pbc_tol : 0.0;
  p->check = o ? (o->check != 0) : 0;
  p->grid = o ? o->grid : 0;
  if (p->grid < 0) return fail(SWEEP_ERR_INVALID_ARG, "grid must be >= 0");
  p->pack = o ? o->pack : 0;
  if (p->pack < 0 || p->pack > 4) return fail(SWEEP_ERR_INVALID_ARG, "pack must be in [0, 4]");
  if (!(p->pbc_tol >= 0.0) || !std::isfinite(p->pbc_tol))
    return fail(SWEEP_ERR_INVALID_ARG, "pbc_tol must be finite and >= 0");
  if (p->law != SWEEP_LAW_UPWIND && p->law != SWEEP_LAW_EXP)
    return fail(SWEEP_ERR_INVALID_ARG, "unknown cell law %d", p->law);
  if (p->boundary != SWEEP_BOUNDARY_VACUUM && p->boundary != SWEEP_BOUNDARY_PERIODIC)
    return fail(SWEEP_ERR_INVALID_ARG, "unknown boundary %d", p->boundary);
  if (p->n_pbc < 1 || p->n_scat < 1) return fail(SWEEP_ERR_INVALID_ARG, "n_pbc and n_scat must be >= 1");
  if (!(p->albedo >= 0.0f) || !(p->albedo < 1.0f)) return fail(SWEEP_ERR_INVALID_ARG, "albedo must be in [0, 1)");
  if (p->form != SWEEP_FORM_BATCHED && p->form != SWEEP_FORM_PLAIN)
    return fail(SWEEP_ERR_INVALID_ARG, "unknown form %d", p->form);
  if (p->block != 0 && p->block != 256 && p->block != 512 && p->block != 1024)
    return fail(SWEEP_ERR_INVALID_ARG, "block must be 256, 512 or 1024");
  if (p->ring != 0 && (p->ring < 64 || (p->ring & (p->ring - 1)) != 0))
    return fail(SWEEP_ERR_INVALID_ARG, "ring must be a power of two >= 64");
  if (p->boundary == SWEEP_BOUNDARY_VACUUM) p->n_pbc = 1;
  return SWEEP_OK;
}

// Group chunks: groups are independent, a launch packs up to 4 of them per task.
// One sweep launch: groups [g0, g0 + n_chunks x gn) as n_chunks independent
// chunks of gn packed groups.
struct GroupLaunch {
  int g0, gn, n_chunks;
};

// The launches of one sweep of G groups.  Plain form: one group per launch.
// Batched form, packing `pack` (0 = automatic): chunks of pack groups in one
// launch (a unit's chunks are swept side by side on different compute units,
// each with less work per step) and a last launch for the G mod pack groups
// left.  The automatic packing is the smallest one dividing G whose
// n_units x G / pack work items still fit one per compute unit, else 4.
std::vector<GroupLaunch> group_plan(sweep_dag_t d, int G, bool plain, int pack) {
  std::vector<GroupLaunch> ch;
  if (plain) {
    for (int g = 0; g < G; ++g) ch.push_back({g, 1, 1});
    return ch;
  }
  const int64_t n_units = (int64_t)d->units.size();
  int gn = pack;
  for (int c = 1; gn == 0 && c <= std::min(G, 4); ++c)
    if (G % c == 0 && n_units * (G / c) <= d->cu_count) gn = c;
  if (gn == 0) gn = 4;
  gn = std::min(gn, G);
  ch.push_back({0, gn, G / gn});
  if (G % gn != 0) ch.push_back({G - G % gn, G % gn, 1});
  return ch;
}

// The largest ring (a power of two) whose LDS layout fits next to the staging
// buffers and prefetched slots of `block` threads; 0 if none does.
int default_ring(sweep_dag_t d, int gn, int block) {
  int best = 0;
  for (int r = 64; r <= (1 << 20); r *= 2)
    if (sweep::sweep_lds_layout(gn, r, block).bytes <= (size_t)d->lds_max) best = r;
  return best;
}

// The step table of `block`-thread sweeps (built on first use, kept with the DAG).
sweep_status_t ensure_steps(sweep_dag_t d, int block, hipStream_t s, sweep_dag_s::StepTable** out) {
  const int cap_t = block, cap_e = sweep::kStageCh * block - 8;
  for (auto& t : d->steps)
    if (t->block == block && t->cap_e == cap_e) {
      *out = t.get();
      return SWEEP_OK;
    }
  if (g_capturing)  // prepare_steps builds every table a captured sequence needs beforehand
    return fail(SWEEP_ERR_HIP, "step table of %d threads missing during graph capture", block);
  const int n_units = (int)d->units.size();
  // capacity per unit: a level of w tasks and e entries gives at most
  // w / cap_t + 1.15 e / cap_e + 2 steps, and the levels' e sum to at most the
  // unit's upwind plus downwind entries
  std::vector<int64_t> base(n_units + 1, 0);
  for (int u = 0; u < n_units; ++u) {
    const Unit& U = d->units[u];
    const int64_t e = d->unit_up[u] + d->unit_dn[u];
    base[u + 1] = base[u] + 2 * (int64_t)U.depth + U.n_cells / cap_t + (e * 115) / (100LL * cap_e) + 3;
  }
  std::unique_ptr<sweep_dag_s::StepTable> t(new sweep_dag_s::StepTable());
  t->block = block;
  t->cap_e = cap_e;
  const int64_t total = base[n_units];
  HIP_TRY(t->k.alloc(4 * total));
  HIP_TRY(t->eu.alloc(8 * total));
  HIP_TRY(t->ed.alloc(8 * total));
  HIP_TRY(t->base.alloc(8 * (size_t)(n_units + 1)));
  HIP_TRY(t->n.alloc(4 * (size_t)n_units));
  HIP_TRY(hipMemcpyAsync(t->base.p, base.data(), 8 * (size_t)(n_units + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(sweep::launch_steps(d->units_d.as<Unit>(), n_units, d->lp.as<int32_t>(),
                              d->lev_up.as<int64_t>(), d->lev_dn.as<int64_t>(),
                              d->up_ptr.as<int64_t>(), d->dn_ptr.as<int64_t>(),
                              t->base.as<int64_t>(), cap_t, cap_e, t->k.as<int32_t>(),
                              t->eu.as<int64_t>(), t->ed.as<int64_t>(), t->n.as<int32_t>(), s));
  std::vector<int32_t> ns(n_units);
  HIP_TRY(hipMemcpyAsync(ns.data(), t->n.p, 4 * (size_t)n_units, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int u = 0; u < n_units; ++u)
    if (ns[u] < 0) return fail(SWEEP_ERR_HIP, "step table of unit %d overflowed its capacity", u);
  *out = t.get();
  d->steps.push_back(std::move(t));
  return SWEEP_OK;
}

// Builds the step tables the sweeps of a call with these options use (before
// any capture: building one synchronises the stream).
sweep_status_t prepare_steps(sweep_dag_t d, const FwdPlan& p, int32_t G, hipStream_t s) {
  for (const GroupLaunch& c : group_plan(d, G, p.form == SWEEP_FORM_PLAIN, p.pack)) {
    const int block = p.block > 0 ? p.block : sweep::kSweepMaxBlock(c.gn);
    sweep_dag_s::StepTable* t = nullptr;
    ST_TRY(ensure_steps(d, block, s, &t));
  }
  return SWEEP_OK;
}

// Per-task denominators and sources for one sweep (schedule order).
sweep_status_t run_prep(sweep_dag_t d, int32_t G, const float* kappa, const float* emission,
                        const float* gsrc, const float* jsum_prev, float albedo, int32_t law,
                        hipStream_t s) {
  HIP_TRY(d->tden.alloc(4 * (size_t)d->T * G));
  HIP_TRY(d->tsrc.alloc(4 * (size_t)d->T * G));
  HIP_TRY(d->crec.alloc(8 * (size_t)d->C_total * G));
  sweep::PrepArgs q{};
  q.units = d->units_d.as<Unit>();
  q.n_units = (int32_t)d->units.size();
  q.blk_base = d->blk_base.as<int32_t>();
  q.sched = d->sched.as<int32_t>();
  q.aperp_s = d->aperp_s.as<float>();
  q.vol_s = d->vol_s.as<float>();
  q.kappa = kappa;
  q.vol = d->vol.as<float>();
  q.emission = emission;
  q.gsrc = gsrc;
  q.jsum_prev = jsum_prev;
  q.albedo = albedo;
  q.inv_D = 1.0f / (float)d->D;
  q.G = G;
  q.law = law;
  q.C_total = d->C_total;
  q.crec = d->crec.as<float2>();
  q.tden = d->tden.as<float>();
  q.tsrc = d->tsrc.as<float>();
  q.flag = d->flag.as<int32_t>();
  ProfScope ps("prep", s);
  HIP_TRY(sweep::launch_prep(q, d->n_blocks, s));
  return SWEEP_OK;
}

// The direction reduction's arguments that do not change between the passes of
// a call (the reduction tables must be in place: ensure_reduce_tables).
sweep::ReduceArgs reduce_args(sweep_dag_t d, int32_t G, const FwdPlan& p, const float* kappa,
                              const float* emission, float* J, float* absorbed) {
  sweep::ReduceArgs r{};
  r.units = d->units_d.as<Unit>();
  r.D = d->D;
  r.G = G;
  r.C_total = d->C_total;
  r.blk_mesh = d->blk_mesh.as<int32_t>();
  r.blk_cell0 = d->blk_cell0.as<int32_t>();
  r.mesh_off = d->mesh_off_d.as<int32_t>();
  r.mesh_cells = d->mesh_cells_d.as<int32_t>();
  r.bnd = d->bnd.as<float2>();
  r.aperp = d->aperp.as<float>();
  r.law = p.law;
  r.kappa = kappa;
  r.emission = emission;
  r.vol = d->vol.as<float>();
  r.albedo = p.albedo;
  r.J = J;
  r.absorbed = absorbed;
  r.partial = d->partial.as<double>();
  r.cells_per_block = d->red_cpb;
  return r;
}

// Per-call buffers of the periodic fold: the periodic tasks' own sources and the
// inflow sums of two passes.
sweep_status_t alloc_periodic(sweep_dag_t d, int32_t G) {
  const int64_t n = std::max<int64_t>((int64_t)d->n_pc * G, 1);
  HIP_TRY(d->pbase.alloc(4 * (size_t)n * d->D));
  HIP_TRY(d->pval.alloc(4 * (size_t)n * d->D));
  HIP_TRY(d->psum_a.alloc(8 * (size_t)n));
  HIP_TRY(d->psum_b.alloc(8 * (size_t)n));
  return SWEEP_OK;
}

// Folds the periodic coupling of one pass into its sources (sweep::PinArgs):
// forward, the previous pass's exit values through the inflow half-faces
// (their sum over directions into `psum` when given); adjoint, the later pass's
// lambda through the outflow half-faces.  `fresh`: tsrc holds the sources that
// run_prep (or a clear) just wrote, which are saved for the later passes.
sweep_status_t run_pin(sweep_dag_t d, bool adjoint, int32_t G, const float* other, double* psum,
                       bool& fresh, hipStream_t s) {
  sweep::PinArgs q{};
  q.D = d->D;
  q.G = G;
  q.C_total = d->C_total;
  q.n_pc = d->n_pc;
  q.n_pf = d->n_pf;
  q.pf_ptr = d->pf_ptr.as<int32_t>();
  q.pnb = d->pnb.as<int32_t>();
  q.pw = adjoint ? d->pwa.as<float>() : d->pwf.as<float>();
  q.ptask = d->ptask.as<int32_t>();
  q.other = other;
  q.tsrc = d->tsrc.as<float>();
  q.pbase = d->pbase.as<float>();
  q.capture = fresh ? 1 : 0;
  q.pval = psum != nullptr ? d->pval.as<float>() : nullptr;
  q.psum = psum;
  HIP_TRY(sweep::launch_pin(q, s));
  fresh = false;
  return SWEEP_OK;
}

// One sweep of every unit (after run_prep, and run_pin for a periodic pass with
// another pass before it, forward, or after it, adjoint).
sweep_status_t run_sweep(sweep_dag_t d, bool reverse, const FwdPlan& p, int32_t G, float* out,
                         hipStream_t s) {
  sweep::SweepArgs a{};
  a.units = d->units_d.as<Unit>();
  a.sched = d->sched.as<int32_t>();
  a.row_ptr = reverse ? d->dn_ptr.as<int64_t>() : d->up_ptr.as<int64_t>();
  a.ent = reverse ? d->dn.as<int2>() : d->up.as<int2>();
  a.n_ent = reverse ? d->n_dn : d->n_up;
  a.tden = d->tden.as<float>();
  a.tsrc = d->tsrc.as<float>();
  a.out = out;
  HIP_TRY(d->out_s.alloc(4 * (size_t)d->T * G));
  a.out_s = d->out_s.as<float>();
  a.C_total = d->C_total;
  a.G = G;
  a.D = d->D;
  const int n_units = (int)d->units.size();
  for (const GroupLaunch& c : group_plan(d, G, p.form == SWEEP_FORM_PLAIN, p.pack)) {
    const int gn = c.gn;
    const int block = p.block > 0 ? p.block : sweep::kSweepMaxBlock(gn);
    if (block > sweep::kSweepMaxBlock(gn))
      return fail(SWEEP_ERR_INVALID_ARG, "block %d: at most %d threads with %d packed groups", block,
                  sweep::kSweepMaxBlock(gn), gn);
    const int ring = p.ring > 0 ? p.ring : default_ring(d, gn, block);
    const sweep::LdsLayout L = sweep::sweep_lds_layout(gn, std::max(ring, 64), block);
    if (ring == 0 || L.bytes > (size_t)d->lds_max)
      return fail(p.ring > 0 ? SWEEP_ERR_INVALID_ARG : SWEEP_ERR_UNSUPPORTED,
                  "ring %d x %d groups with %d threads needs %zu bytes of LDS, %d available", ring,
                  gn, block, L.bytes, d->lds_max);
    sweep_dag_s::StepTable* stp = nullptr;
    ST_TRY(ensure_steps(d, block, s, &stp));
    a.step_k = stp->k.as<int32_t>();
    a.step_e = reverse ? stp->ed.as<int64_t>() : stp->eu.as<int64_t>();
    a.step_base = stp->base.as<int64_t>();
    a.n_steps = stp->n.as<int32_t>();
    a.g0 = c.g0;
    a.n_chunks = 1;
    a.ring_mask = ring - 1;
    a.stage_off = L.stage_off;
    if (p.form == SWEEP_FORM_PLAIN) {
      a.work_counter = nullptr;
      a.n_units = 1;
      for (int u = 0; u < n_units; ++u) {
        a.unit_order = d->identity_d.as<int32_t>() + u;
        ProfScope ps(reverse ? "sweep_adj" : "sweep_fwd", s);
        hipError_t e = reverse ? sweep::launch_sweep_adj(a, gn, 1, block, L.bytes, s)
                               : sweep::launch_sweep_fwd(a, gn, 1, block, L.bytes, s);
        if (e != hipSuccess) return hip_fail(e, "sweep launch");
      }
    } else {
      int per_cu = std::max(1, (int)((size_t)kMaxLds / (L.bytes + 256)));
      per_cu = std::min(per_cu, std::max(1, 2048 / block));
      a.n_chunks = c.n_chunks;
      int grid = (int)std::min<int64_t>((int64_t)n_units * c.n_chunks, (int64_t)d->cu_count * per_cu);
      if (p.grid > 0) grid = std::min(grid, p.grid);
      a.work_counter = d->counter.as<int32_t>();
      a.unit_order = d->order_d.as<int32_t>();
      a.n_units = n_units;
      HIP_TRY(sweep::launch_fill_i32(a.work_counter, 1, 0, s));
      ProfScope ps(reverse ? "sweep_adj" : "sweep_fwd", s);
      hipError_t e = reverse ? sweep::launch_sweep_adj(a, gn, grid, block, L.bytes, s)
                             : sweep::launch_sweep_fwd(a, gn, grid, block, L.bytes, s);
      if (e != hipSuccess) return hip_fail(e, "sweep launch");
    }
  }
  return SWEEP_OK;
}

// Runs `body(stream)` as a captured graph: the first call with a given key
// captures the sequence on the DAG's capture stream and instantiates it; every
// call launches the instantiated graph on the caller's stream.  `body` must
// only enqueue kernels (every buffer is allocated before).
template <class Body>
sweep_status_t run_graph(sweep_dag_t d, const std::vector<uint64_t>& key, hipStream_t s, Body&& body) {
  for (auto& g : d->graphs)
    if (g.key == key) {
      HIP_TRY(hipGraphLaunch(g.exec, s));
      return SWEEP_OK;
    }
  if (!d->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&d->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(d->cap_stream, hipStreamCaptureModeThreadLocal));
  g_capturing = true;
  const sweep_status_t st = body(d->cap_stream);
  g_capturing = false;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(d->cap_stream, &graph);
  if (st != SWEEP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
  if (d->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(d->graphs.front().exec);
    d->graphs.erase(d->graphs.begin());
  }
  d->graphs.push_back({key, exec});
  HIP_TRY(hipGraphLaunch(exec, s));
  return SWEEP_OK;
}

uint64_t pkey(const void* p) { return (uint64_t)(uintptr_t)p; }

void opts_key(std::vector<uint64_t>& k, const FwdPlan& p) {
  uint32_t ab;
  std::memcpy(&ab, &p.albedo, 4);
  k.insert(k.end(), {(uint64_t)p.boundary, (uint64_t)p.n_pbc, (uint64_t)p.n_scat, (uint64_t)p.form,
                     (uint64_t)p.block, (uint64_t)p.ring, (uint64_t)ab, (uint64_t)p.law,
                     (uint64_t)p.merge, (uint64_t)p.warm, (uint64_t)p.grid, (uint64_t)p.pack});
  uint64_t tb;
  std::memcpy(&tb, &p.pbc_tol, 8);
  k.push_back(tb);
}

sweep_status_t check_common(sweep_dag_t d, int32_t G) {
  if (!dag_ok(d)) return fail(SWEEP_ERR_NOT_BUILT, "DAG handle is NULL or was not built");
  if (G < 1 || G > kMaxG) return fail(SWEEP_ERR_INVALID_ARG, "G must be in [1, %d]", kMaxG);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != d->device) return fail(SWEEP_ERR_INVALID_ARG, "DAG was built on device %d, current is %d", d->device, dev);
  return SWEEP_OK;
}

// Reports (and clears) the invalid inputs the kernels of earlier asynchronous
// calls on `d` flagged; synchronises `s`.
sweep_status_t take_device_error(sweep_dag_t d, hipStream_t s) {
  int32_t bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, d->flag.p, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bits == 0) return SWEEP_OK;
  HIP_TRY(sweep::launch_fill_i32(d->flag.as<int32_t>(), 1, 0, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::string what;
  if (bits & sweep::kErrKappa) what += " kappa negative or not finite;";
  if (bits & sweep::kErrEmission) what += " emission negative or not finite;";
  if (bits & sweep::kErrCell) what += " a cell with Aperp + kappa V not positive and finite;";
  if (bits & sweep::kErrGrad) what += " dL/dJ or dL/dabsorbed not finite;";
  return fail(SWEEP_ERR_INVALID_ARG, "invalid input to an earlier sweep call on this DAG:%s its "
                                     "outputs are not meaningful", what.c_str());
}

// Every array a sweep launch with G groups addresses through a buffer resource
// stays within kMaxBufBytes.
sweep_status_t check_buffer_range(sweep_dag_t d, int32_t G) {
  if ((int64_t)d->max_cells * G * 4 > sweep::kMaxBufBytes)
    return fail(SWEEP_ERR_UNSUPPORTED, "a mesh of %d cells with %d groups exceeds the sweep's "
                "32-bit buffer range (%lld bytes per direction); use fewer groups per call",
                d->max_cells, G, (long long)sweep::kMaxBufBytes);
  return SWEEP_OK;
}

}  // namespace

extern "C" {

const char* sweep_last_error(void) { return g_err.c_str(); }

sweep_status_t sweep_profile_enable(int32_t on) {
  g_err.clear();
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = on != 0;
  return SWEEP_OK;
}

sweep_status_t sweep_profile_reset(void) {
  g_err.clear();
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (ProfRec& r : g_prof) {
    if (hipEventSynchronize(r.stop) == hipSuccess) {
      g_event_pool.push_back(r.start);
      g_event_pool.push_back(r.stop);
    }
  }
  g_prof.clear();
  return SWEEP_OK;
}

sweep_status_t sweep_profile_read(const char* kernel, int64_t* launches, double* total_ms) {
  g_err.clear();
  if (!kernel || !launches || !total_ms) return fail(SWEEP_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> g(g_prof_mu);
  int64_t n = 0;
  double ms = 0.0;
  for (ProfRec& r : g_prof) {
    if (r.name != kernel) continue;
    HIP_TRY(hipEventSynchronize(r.stop));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, r.start, r.stop));
    ms += t;
    ++n;
  }
  *launches = n;
  *total_ms = ms;
  return SWEEP_OK;
}

sweep_status_t sweep_build_dag(const sweep_mesh_t* meshes, int32_t n_meshes, const double* dirs,
                               int32_t n_dirs, const sweep_build_opts_t* opts, void* stream,
                               sweep_dag_t* out) {
  g_err.clear();
  if (out == nullptr) return fail(SWEEP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (meshes == nullptr || n_meshes < 1) return fail(SWEEP_ERR_INVALID_ARG, "need at least one mesh");
  if (dirs == nullptr || n_dirs < 1) return fail(SWEEP_ERR_INVALID_ARG, "need at least one direction");
  const double eps = opts ? opts->eps_tie : 1e-12;
  const int validate = opts ? opts->validate : 1;
  const int kahn_counters = opts ? opts->kahn_counters : 0;
  if (kahn_counters < 0 || kahn_counters > 2)
    return fail(SWEEP_ERR_INVALID_ARG, "kahn_counters must be 0, 1 or 2");
  const int scheme = opts ? opts->scheme : SWEEP_SCHEME_AREA;
  const int n_aligned = opts && opts->n_aligned > 0 ? opts->n_aligned : 3;
  if (scheme != SWEEP_SCHEME_AREA && scheme != SWEEP_SCHEME_ALIGNED)
    return fail(SWEEP_ERR_INVALID_ARG, "unknown transport scheme %d", scheme);
  if (scheme == SWEEP_SCHEME_ALIGNED && (n_aligned < 1 || n_aligned > sweep::kMaxAligned))
    return fail(SWEEP_ERR_INVALID_ARG, "n_aligned must be in [1, %d]", sweep::kMaxAligned);
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(SWEEP_ERR_INVALID_ARG, "eps_tie must be >= 0");
  for (int d = 0; d < n_dirs; ++d) {
    const double n = std::sqrt(dirs[3 * d] * dirs[3 * d] + dirs[3 * d + 1] * dirs[3 * d + 1] +
                               dirs[3 * d + 2] * dirs[3 * d + 2]);
    if (!(std::fabs(n - 1.0) <= 1e-12)) return fail(SWEEP_ERR_INVALID_ARG, "direction %d is not a unit vector", d);
  }
  hipStream_t s = (hipStream_t)stream;
  StreamScope stream_scope(s);
  std::unique_ptr<sweep_dag_s> dag(new sweep_dag_s());
  sweep_dag_s* D = dag.get();
  HIP_TRY(hipGetDevice(&D->device));
  HIP_TRY(hipDeviceGetAttribute(&D->cu_count, hipDeviceAttributeMultiprocessorCount, D->device));
  D->n_meshes = n_meshes;
  D->D = n_dirs;
  D->scheme = scheme;
  D->eps = eps;
  int64_t off = 0;
  for (int m = 0; m < n_meshes; ++m) {
    const sweep_mesh_t& M = meshes[m];
    if (M.n_cells < 1 || M.n_half_faces < 1 || !M.face_ptr || !M.cell_volume || !M.face_nbr ||
        !M.face_area || !M.face_normal)
      return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: missing arrays, no cells or no faces", m);
    if (scheme == SWEEP_SCHEME_ALIGNED && !M.face_twin)
      return fail(SWEEP_ERR_INVALID_ARG, "mesh %d: the aligned transport scheme needs face_twin", m);
    if (validate) ST_TRY(validate_mesh_host(M, m));
    D->mesh_off.push_back((int32_t)off);
    D->mesh_cells.push_back(M.n_cells);
    if (M.face_shift) D->has_shift = true;
    off += M.n_cells;
    if (off > INT32_MAX / 2) return fail(SWEEP_ERR_INVALID_ARG, "too many cells");
  }
  D->mesh_off.push_back((int32_t)off);
  D->C_total = off;
  D->T = off * n_dirs;
  const int64_t T = D->T;
  // the row-pointer scans index tasks with 32-bit counts
  if (T + 1 > INT32_MAX)
    return fail(SWEEP_ERR_UNSUPPORTED, "%lld tasks (cells x directions) in one DAG; at most %d: "
                "split the directions over several DAGs", (long long)T, INT32_MAX - 1);
  const int n_units = n_meshes * n_dirs;
  // units: u = mesh * D + dir; the tasks of unit (m, d) start at D * (first cell
  // of m) + d * cells(m) (k_adj_reduce indexes per-task arrays with this formula)
  std::vector<int32_t> blk_base(n_units + 1, 0);
  for (int m = 0; m < n_meshes; ++m)
    for (int d = 0; d < n_dirs; ++d) {
      Unit U{};
      U.task_base = (int64_t)n_dirs * D->mesh_off[m] + (int64_t)d * D->mesh_cells[m];
      const int u = m * n_dirs + d;
      U.lp_base = U.task_base + 2 * (int64_t)u;
      U.n_cells = D->mesh_cells[m];
      U.dir = d;
      U.mesh = m;
      U.cell_off = D->mesh_off[m];
      D->units.push_back(U);
      blk_base[u + 1] = blk_base[u] + (U.n_cells + 255) / 256;
    }
  const int n_blocks = blk_base[n_units];
  // cell-order tile tables (tiles never straddle meshes)
  std::vector<int32_t> cbm, cbc;
  int max_faces = 1, max_cells = 1;
  // downwind rows are 16 entries wide (one 64-byte line segment each, so the
  // whole row arrives with one line); longer lists continue in an overflow pool
  // of fixed size.  If the pool runs out, the counts are redone with rows of
  // kRowCap entries and a pool sized for every cell with more faces than that
  // ((faces + 2) ints per direction).
  constexpr int kRowNarrow = 16;
  constexpr int kRowCap = 32;
  int64_t ovf_cap = 2;
  {
    // face statistics on the device (one small copy back)
    Buf fstat;
    HIP_TRY(fstat.alloc(16));
    HIP_TRY(hipMemsetAsync(fstat.p, 0, 16, s));
    for (int m = 0; m < n_meshes; ++m)
      HIP_TRY(sweep::launch_face_stats(meshes[m].face_ptr, meshes[m].n_cells, kRowCap, n_dirs,
                                       fstat.as<unsigned long long>(), s));
    unsigned long long fs[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(fs, fstat.p, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    max_faces = std::max<int>(max_faces, (int)fs[0]);
    ovf_cap += (int64_t)fs[1];
  }
  for (int m = 0; m < n_meshes; ++m) {
    for (int32_t c = 0; c < D->mesh_cells[m]; c += sweep::kTileCellsHost) {
      cbm.push_back(m);
      cbc.push_back(c);
    }
    max_cells = std::max(max_cells, meshes[m].n_cells);
  }
  const int n_cblocks = (int)cbm.size();
  // scheme (b) rows hold at most n_aligned <= 4 entries: never any overflow
  int dn_width = scheme == SWEEP_SCHEME_ALIGNED ? sweep::kMaxAligned
                                                : std::min(kRowNarrow, (max_faces + 3) / 4 * 4);
  const int64_t ovf_cap_narrow = std::max<int64_t>(1 << 20, T / 4);
  if (ovf_cap > INT32_MAX / 2)
    return fail(SWEEP_ERR_UNSUPPORTED, "too many cells with more than %d faces", kRowCap);
  std::vector<sweep::MeshDev> md(n_meshes);
  for (int m = 0; m < n_meshes; ++m) {
    md[m].face_ptr = meshes[m].face_ptr;
    md[m].face_twin = meshes[m].face_twin;
    md[m].face_nbr = meshes[m].face_nbr;
    md[m].face_shift = meshes[m].face_shift;
    md[m].face_area = meshes[m].face_area;
    md[m].face_normal = meshes[m].face_normal;
    md[m].cell_volume = meshes[m].cell_volume;
    md[m].n_faces = meshes[m].n_half_faces;
    md[m].n_cells = meshes[m].n_cells;
    md[m].cell_off = D->mesh_off[m];
  }
  // per-face neighbour codes and per-(direction, face) signed weights for the row fill
  int64_t n_faces_total = 0;
  for (int m = 0; m < n_meshes; ++m) n_faces_total += meshes[m].n_half_faces;
  Buf fcode, wface;
  HIP_TRY(fcode.alloc(4 * n_faces_total));
  HIP_TRY(wface.alloc(4 * (size_t)n_faces_total * n_dirs));
  {
    int64_t fo = 0;
    for (int m = 0; m < n_meshes; ++m) {
      md[m].fcode = fcode.as<int32_t>() + fo;
      md[m].face_off = fo;
      HIP_TRY(sweep::launch_face_codes(md[m], fcode.as<int32_t>() + fo, s));
      fo += meshes[m].n_half_faces;
    }
  }
  Buf cblk_mesh_d, cblk_c0_d, dnw, stats_d, meshes_d, dirs_d, rowlen_dn, cnt, inv, depth_d, err_d, len_up, len_dn, scan_tmp;
  HIP_TRY(meshes_d.alloc(sizeof(sweep::MeshDev) * n_meshes));
  HIP_TRY(dirs_d.alloc(sizeof(double) * 3 * n_dirs));
  HIP_TRY(D->blk_base.alloc(sizeof(int32_t) * (n_units + 1)));
  D->n_blocks = n_blocks;
  HIP_TRY(D->units_d.alloc(sizeof(Unit) * n_units));
  HIP_TRY(cblk_mesh_d.alloc(4 * cbm.size()));
  HIP_TRY(cblk_c0_d.alloc(4 * cbc.size()));
  HIP_TRY(hipMemcpyAsync(cblk_mesh_d.p, cbm.data(), 4 * cbm.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(cblk_c0_d.p, cbc.data(), 4 * cbc.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(meshes_d.p, md.data(), sizeof(sweep::MeshDev) * n_meshes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dirs_d.p, dirs, sizeof(double) * 3 * n_dirs, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(D->blk_base.p, blk_base.data(), sizeof(int32_t) * (n_units + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(D->units_d.p, D->units.data(), sizeof(Unit) * n_units, hipMemcpyHostToDevice, s));
  HIP_TRY(D->indeg.alloc(4 * T));
  HIP_TRY(rowlen_dn.alloc(4 * T));
  HIP_TRY(D->aperp.alloc(4 * T));
  HIP_TRY(D->aperp_s.alloc(4 * T));
  HIP_TRY(D->vol_s.alloc(4 * T));
  HIP_TRY(D->bnd.alloc(8 * T));
  HIP_TRY(cnt.alloc(4 * T));  // Kahn's counters in global memory
  HIP_TRY(inv.alloc(4 * T));
  HIP_TRY(D->sched.alloc(4 * T));
  HIP_TRY(D->lp.alloc(4 * (T + 2 * (int64_t)n_units)));
  HIP_TRY(depth_d.alloc(4 * n_units));
  HIP_TRY(err_d.alloc(8));
  HIP_TRY(sweep::launch_fill_i32(err_d.as<int32_t>(), 2, 0, s));
  Buf dn_ovf, dn_ovf_top;
  HIP_TRY(dn_ovf_top.alloc(4));
  Buf ent_tot;  // row entries of all tasks (sizes the row arrays before the schedule exists)
  HIP_TRY(ent_tot.alloc(16));
  Buf big, big_top;  // tasks whose upwind count does not fit a 4-bit counter
  HIP_TRY(big.alloc(8 * T));
  HIP_TRY(big_top.alloc(4));
  HIP_TRY(sweep::launch_fill_i32(big_top.as<int32_t>(), 1, 0, s));
  HIP_TRY(stats_d.alloc(8));
  HIP_TRY(sweep::launch_fill_i32(stats_d.as<int32_t>(), 2, 0, s));
  sweep::DagBuildArgs a{};
  a.units = D->units_d.as<Unit>();
  a.n_units = n_units;
  a.D = n_dirs;
  a.cblk_mesh = cblk_mesh_d.as<int32_t>();
  a.cblk_c0 = cblk_c0_d.as<int32_t>();
  a.max_faces = max_faces;
  a.dn_ovf_top = dn_ovf_top.as<int32_t>();
  a.big = big.as<int64_t>();
  a.big_top = big_top.as<int32_t>();
  a.ent_tot = ent_tot.as<unsigned long long>();
  a.stats = stats_d.as<int32_t>();
  a.meshes = meshes_d.as<sweep::MeshDev>();
  a.dirs = dirs_d.as<double>();
  a.eps = eps;
  a.scheme = scheme;
  a.n_aligned = n_aligned;
  a.blk_base = D->blk_base.as<int32_t>();
  a.indeg = D->indeg.as<int32_t>();
  a.rowlen_dn = rowlen_dn.as<int32_t>();
  a.aperp = D->aperp.as<float>();
  a.aperp_s = D->aperp_s.as<float>();
  a.vol_s = D->vol_s.as<float>();
  a.wface = wface.as<float>();
  a.bnd = D->bnd.as<float2>();
  a.cnt = cnt.as<int32_t>();
  a.inv = inv.as<int32_t>();
  a.sched = D->sched.as<int32_t>();
  a.lp = D->lp.as<int32_t>();
  a.depth = depth_d.as<int32_t>();
  a.err = err_d.as<int32_t>();
  int lds_limit = 65536;
  (void)hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, D->device);
  int32_t stats[2] = {0, 0};
  int32_t n_big = 0;
  for (int attempt = 0;; ++attempt) {
    const int64_t cap = dn_width == kRowNarrow ? ovf_cap_narrow : ovf_cap;
    const int sent_len = std::max(64, dn_width);  // sentinel row of -1 after the rows
    HIP_TRY(dnw.alloc(4 * ((size_t)T * dn_width + sent_len)));
    HIP_TRY(sweep::launch_fill_i32(dnw.as<int32_t>() + (size_t)T * dn_width, sent_len, -1, s));
    // the pool ends with room for one list that is written when it has run out
    HIP_TRY(dn_ovf.alloc(4 * (cap + max_faces + 2)));
    HIP_TRY(sweep::launch_fill_i32(dn_ovf_top.as<int32_t>(), 1, 0, s));
    HIP_TRY(sweep::launch_fill_i32(big_top.as<int32_t>(), 1, 0, s));
    HIP_TRY(sweep::launch_fill_i32(stats_d.as<int32_t>(), 2, 0, s));
    HIP_TRY(sweep::launch_fill_i32(ent_tot.as<int32_t>(), 4, 0, s));
    a.dn_width = dn_width;
    a.dnw = dnw.as<int32_t>();
    a.dn_sentinel = (int64_t)T * dn_width;
    a.dn_ovf = dn_ovf.as<int32_t>();
    a.dn_ovf_cap = cap;
    {
      ProfScope ps("count", s);
      HIP_TRY(sweep::launch_count(a, n_cblocks, lds_limit, s));
    }
    int32_t top = 0;
    int64_t tot[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(tot, ent_tot.p, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(stats, stats_d.p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&n_big, big_top.p, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&top, dn_ovf_top.p, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    D->n_up = tot[0];
    D->n_dn = tot[1];
    if (top <= cap) break;
    if (dn_width >= kRowCap || attempt > 0)
      return fail(SWEEP_ERR_HIP, "downwind overflow pool exhausted (%d > %lld)", top, (long long)cap);
    dn_width = std::min(kRowCap, (max_faces + 3) / 4 * 4);
  }
  // the longest downwind list sets how much of every row Kahn's algorithm loads
  a.dn_chunks = std::max(1, std::min(dn_width / 4, (stats[1] + 3) / 4));
  // row lengths in schedule order (the input of the row-pointer scan)
  HIP_TRY(len_up.alloc(4 * (T + 1)));
  HIP_TRY(len_dn.alloc(4 * (T + 1)));
  a.len_up = len_up.as<int32_t>();
  a.len_dn = len_dn.as<int32_t>();
  HIP_TRY(hipMemsetAsync(a.len_up + T, 0, 4, s));
  HIP_TRY(hipMemsetAsync(a.len_dn + T, 0, 4, s));
  // Kahn counters in LDS as 4-bit fields when the mesh fits the LDS
  // (the kernel's static LDS holds two frontier copies of 2048 cells); the
  // rows' entries of cells with larger counts are flagged first
  const bool lds_fits = (size_t)4 * ((max_cells + 7) / 8 + 64) + 17 * 1024 <= (size_t)lds_limit;
  if (kahn_counters == 1 && !lds_fits)
    return fail(SWEEP_ERR_UNSUPPORTED, "the counters of a %d-cell mesh do not fit in LDS", max_cells);
  const bool lds_cnt = kahn_counters == 2 ? false : lds_fits;
  // counters in global memory are bytes
  if (!lds_cnt && stats[0] > 254)
    return fail(SWEEP_ERR_UNSUPPORTED, "a cell with %d upwind dependencies in one direction "
                "(at most 254 when the mesh's counters do not fit in LDS)", stats[0]);
  D->kahn_lds = lds_cnt ? 1 : 0;
  if (lds_cnt) HIP_TRY(sweep::launch_mark(a, n_big, s));
  {
    ProfScope ps("kahn", s);
    HIP_TRY(sweep::launch_kahn(a, lds_cnt, max_cells, s));
  }
  // (no synchronisation here: the depths and the cycle flag are read once, at the end)
  // the inverse schedule of cells that a cyclic graph leaves out stays -1
  HIP_TRY(sweep::launch_fill_i32(a.inv, T, -1, s));
  HIP_TRY(sweep::launch_sort_levels(a, s));
  HIP_TRY(sweep::launch_gather_len(a, n_blocks, s));
  // row lengths in schedule order -> row pointers
  HIP_TRY(D->up_ptr.alloc(8 * (T + 1)));
  HIP_TRY(D->dn_ptr.alloc(8 * (T + 1)));
  a.up_ptr = D->up_ptr.as<int64_t>();
  a.dn_ptr = D->dn_ptr.as<int64_t>();
  size_t tmp_bytes = 0;
  HIP_TRY(sweep::launch_scan_len(a.len_up, a.up_ptr, T + 1, nullptr, &tmp_bytes, s));
  HIP_TRY(scan_tmp.alloc(tmp_bytes));
  HIP_TRY(sweep::launch_scan_len(a.len_up, a.up_ptr, T + 1, scan_tmp.p, &tmp_bytes, s));
  HIP_TRY(sweep::launch_scan_len(a.len_dn, a.dn_ptr, T + 1, scan_tmp.p, &tmp_bytes, s));
  HIP_TRY(D->up.alloc(8 * std::max<int64_t>(D->n_up, 1)));
  HIP_TRY(D->dn.alloc(8 * std::max<int64_t>(D->n_dn, 1)));
  a.up = D->up.as<int2>();
  a.dn = D->dn.as<int2>();
  {
    ProfScope ps("fill", s);
    HIP_TRY(sweep::launch_fill(a, n_blocks, s));
  }
  HIP_TRY(D->lev_up.alloc(8 * (T + 2 * (int64_t)n_units)));
  HIP_TRY(D->lev_dn.alloc(8 * (T + 2 * (int64_t)n_units)));
  a.lev_up = D->lev_up.as<int64_t>();
  a.lev_dn = D->lev_dn.as<int64_t>();
  HIP_TRY(sweep::launch_level_entries(a, s));
  HIP_TRY(D->vol.alloc(4 * D->C_total));
  for (int m = 0; m < n_meshes; ++m)
    HIP_TRY(sweep::launch_d2f(meshes[m].cell_volume, D->vol.as<float>() + D->mesh_off[m],
                              meshes[m].n_cells, s));
  if (D->has_shift) {
    // the periodic cells and half-faces: counts per cell, two scans, the lists
    const int64_t C1 = (int64_t)D->C_total + 1;
    Buf npf, pflag, pf_off, pc_off, ptmp;
    HIP_TRY(npf.alloc(4 * C1));
    HIP_TRY(pflag.alloc(4 * C1));
    HIP_TRY(pf_off.alloc(8 * C1));
    HIP_TRY(pc_off.alloc(8 * C1));
    a.npf = npf.as<int32_t>();
    a.pflag = pflag.as<int32_t>();
    HIP_TRY(sweep::launch_fill_i32(a.npf + D->C_total, 1, 0, s));
    HIP_TRY(sweep::launch_fill_i32(a.pflag + D->C_total, 1, 0, s));
    for (int m = 0; m < n_meshes; ++m) HIP_TRY(sweep::launch_pcount(a, md[m], s));
    size_t pt_bytes = 0;
    HIP_TRY(sweep::launch_scan_len(a.npf, pf_off.as<int64_t>(), C1, nullptr, &pt_bytes, s));
    HIP_TRY(ptmp.alloc(pt_bytes));
    HIP_TRY(sweep::launch_scan_len(a.npf, pf_off.as<int64_t>(), C1, ptmp.p, &pt_bytes, s));
    HIP_TRY(sweep::launch_scan_len(a.pflag, pc_off.as<int64_t>(), C1, ptmp.p, &pt_bytes, s));
    int64_t totals[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&totals[0], pf_off.as<int64_t>() + D->C_total, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&totals[1], pc_off.as<int64_t>() + D->C_total, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (totals[0] > INT32_MAX)
      return fail(SWEEP_ERR_UNSUPPORTED, "%lld periodic half-faces (at most %d)", (long long)totals[0],
                  INT32_MAX);
    D->n_pf = totals[0];
    D->n_pc = (int32_t)totals[1];
    a.pf_off = pf_off.as<int64_t>();
    a.pc_off = pc_off.as<int64_t>();
    a.n_pc = D->n_pc;
    a.n_pf = D->n_pf;
    HIP_TRY(D->pcell.alloc(4 * std::max<int64_t>(D->n_pc, 1)));
    HIP_TRY(D->pf_ptr.alloc(4 * ((int64_t)D->n_pc + 1)));
    HIP_TRY(D->pnb.alloc(4 * std::max<int64_t>(D->n_pf, 1)));
    HIP_TRY(D->pwf.alloc(4 * std::max<int64_t>(D->n_pf * n_dirs, 1)));
    HIP_TRY(D->pwa.alloc(4 * std::max<int64_t>(D->n_pf * n_dirs, 1)));
    HIP_TRY(D->ptask.alloc(4 * std::max<int64_t>((int64_t)D->n_pc * n_dirs, 1)));
    HIP_TRY(D->pc_map.alloc(4 * (int64_t)D->C_total));
    a.pcell = D->pcell.as<int32_t>();
    a.pf_ptr = D->pf_ptr.as<int32_t>();
    a.pnb = D->pnb.as<int32_t>();
    a.pwf = D->pwf.as<float>();
    a.pwa = D->pwa.as<float>();
    a.ptask = D->ptask.as<int32_t>();
    a.pc_map = D->pc_map.as<int32_t>();
    HIP_TRY(sweep::launch_fill_i32(a.pf_ptr + D->n_pc, 1, (int32_t)D->n_pf, s));
    Buf pface;
    HIP_TRY(pface.alloc(4 * std::max<int64_t>(D->n_pf, 1)));
    a.pface = pface.as<int32_t>();
    for (int m = 0; m < n_meshes; ++m) HIP_TRY(sweep::launch_plist(a, md[m], s));
    for (int m = 0; m < n_meshes; ++m)
      if (md[m].face_shift != nullptr) HIP_TRY(sweep::launch_pdir(a, md[m], m, s));
    HIP_TRY(hipStreamSynchronize(s));  // the local counts and scans are released here
  }
  std::vector<int32_t> depth(n_units);
  int32_t err = 0;
  Buf ue_d;  // row entries per unit (the sweep addresses a unit's rows with 32-bit offsets)
  HIP_TRY(ue_d.alloc(16 * (size_t)n_units));
  HIP_TRY(sweep::launch_unit_entries(D->units_d.as<Unit>(), n_units, D->up_ptr.as<int64_t>(),
                                     D->dn_ptr.as<int64_t>(), ue_d.as<int64_t>(), s));
  std::vector<int64_t> ue(2 * (size_t)n_units);
  HIP_TRY(hipMemcpyAsync(ue.data(), ue_d.p, 16 * (size_t)n_units, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(depth.data(), depth_d.p, 4 * n_units, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&err, err_d.p, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err) return fail(SWEEP_ERR_CYCLE, "a dependency graph is cyclic: some tasks never become ready");
  for (int u = 0; u < n_units; ++u)
    if (8 * std::max(ue[2 * u], ue[2 * u + 1]) > sweep::kMaxBufBytes)
      return fail(SWEEP_ERR_UNSUPPORTED, "mesh %d, direction %d: %lld row entries exceed the sweep's "
                  "32-bit buffer range", D->units[u].mesh, D->units[u].dir,
                  (long long)std::max(ue[2 * u], ue[2 * u + 1]));
  D->max_cells = max_cells;
  D->unit_up.resize(n_units);
  D->unit_dn.resize(n_units);
  for (int u = 0; u < n_units; ++u) {
    D->unit_up[u] = ue[2 * u];
    D->unit_dn[u] = ue[2 * u + 1];
  }
  HIP_TRY(D->flag.alloc(4));
  HIP_TRY(sweep::launch_fill_i32(D->flag.as<int32_t>(), 1, 0, s));
  for (int u = 0; u < n_units; ++u) {
    D->units[u].depth = depth[u];
    D->max_depth = std::max(D->max_depth, depth[u]);
  }
  HIP_TRY(hipMemcpyAsync(D->units_d.p, D->units.data(), sizeof(Unit) * n_units, hipMemcpyHostToDevice, s));
  // schedule of the units: deepest first
  D->order.resize(n_units);
  D->identity.resize(n_units);
  for (int u = 0; u < n_units; ++u) D->order[u] = D->identity[u] = u;
  std::stable_sort(D->order.begin(), D->order.end(), [&](int x, int y) {
    const int64_t wx = (int64_t)D->units[x].depth * 1024 + D->units[x].n_cells / 1024;
    const int64_t wy = (int64_t)D->units[y].depth * 1024 + D->units[y].n_cells / 1024;
    return wx > wy;
  });
  HIP_TRY(D->order_d.alloc(4 * n_units));
  HIP_TRY(D->identity_d.alloc(4 * n_units));
  HIP_TRY(D->counter.alloc(64));
  HIP_TRY(hipMemcpyAsync(D->order_d.p, D->order.data(), 4 * n_units, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(D->identity_d.p, D->identity.data(), 4 * n_units, hipMemcpyHostToDevice, s));
  {
    // LDS a sweep workgroup may use: the device limit less the kernel's static LDS
    int lds_max = 65536;
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, D->device);
    D->lds_max = std::max(65536, std::min(lds_max, kMaxLds)) - 256;
    if (D->lds_max > 65536 - 256 && sweep::set_sweep_lds_limit(D->lds_max) != hipSuccess) {
      (void)hipGetLastError();
      D->lds_max = 65536 - 256;
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  *out = dag.release();
  return SWEEP_OK;
}

sweep_status_t sweep_destroy_dag(sweep_dag_t dag) {
  g_err.clear();
  if (!dag) return SWEEP_OK;
  // the DAG's buffers may still be in use on any stream the caller used; wait for
  // the device once, then hand them to the cache as idle memory
  (void)hipSetDevice(dag->device);
  (void)hipDeviceSynchronize();
  g_release_synced = true;
  delete dag;
  g_release_synced = false;
  return SWEEP_OK;
}

sweep_status_t sweep_dag_info(sweep_dag_t d, sweep_dag_info_t* info) {
  g_err.clear();
  if (!dag_ok(d)) return fail(SWEEP_ERR_NOT_BUILT, "DAG handle is NULL or was not built");
  if (!info) return fail(SWEEP_ERR_INVALID_ARG, "info is NULL");
  std::memset(info, 0, sizeof(*info));
  info->n_meshes = d->n_meshes;
  info->n_dirs = d->D;
  info->n_cells = d->C_total;
  info->n_tasks = d->T;
  info->n_up_entries = d->n_up;
  info->n_down_entries = d->n_dn;
  int mx = 0, mn = INT32_MAX;
  double sum = 0;
  for (const Unit& U : d->units) {
    mx = std::max(mx, U.depth);
    mn = std::min(mn, U.depth);
    sum += U.depth;
  }
  info->max_depth = mx;
  info->min_depth = mn;
  info->mean_depth = sum / d->units.size();
  const Buf* bufs[] = {&d->sched, &d->indeg, &d->lp, &d->lev_up, &d->lev_dn,
                       &d->up_ptr, &d->dn_ptr, &d->up, &d->dn, &d->aperp, &d->aperp_s, &d->vol_s, &d->bnd, &d->vol,
                       &d->pcell, &d->pf_ptr, &d->pnb, &d->pwf, &d->pwa, &d->ptask, &d->pc_map};
  int64_t b = 0;
  for (const Buf* x : bufs) b += (int64_t)x->bytes;
  info->device_bytes = b;
  info->kahn_lds_counters = d->kahn_lds;
  info->scheme = d->scheme;
  return SWEEP_OK;
}

sweep_status_t sweep_dag_export(sweep_dag_t d, int32_t* level, int32_t* order, int32_t* indeg,
                                void* stream) {
  g_err.clear();
  if (!dag_ok(d)) return fail(SWEEP_ERR_NOT_BUILT, "DAG handle is NULL or was not built");
  hipStream_t s = (hipStream_t)stream;
  const int64_t T = d->T;
  if (indeg) HIP_TRY(hipMemcpyAsync(indeg, d->indeg.p, 4 * T, hipMemcpyDeviceToHost, s));
  std::vector<int32_t> sched, lp;
  if (order || level) {
    sched.resize(T);
    lp.resize(T + 2 * d->units.size());
    HIP_TRY(hipMemcpyAsync(sched.data(), d->sched.p, 4 * T, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(lp.data(), d->lp.p, 4 * lp.size(), hipMemcpyDeviceToHost, s));
  }
  ST_TRY(take_device_error(d, s));
  // the schedule groups every unit's cells by level (level k = slots [lp[k], lp[k+1]));
  // the canonical order sorts each level by cell id
  for (const Unit& U : d->units) {
    if (!order && !level) break;
    const int32_t* l = lp.data() + U.lp_base;
    const int32_t* sc = sched.data() + U.task_base;
    for (int k = 0; k < U.depth; ++k) {
      if (level)
        for (int32_t i = l[k]; i < l[k + 1]; ++i) level[U.task_base + sc[i]] = k;
      if (order) {
        int32_t* o = order + U.task_base;
        std::memcpy(o + l[k], sc + l[k], 4 * (size_t)(l[k + 1] - l[k]));
        std::sort(o + l[k], o + l[k + 1]);
      }
    }
  }
  return SWEEP_OK;
}

// Layout of the `saved` workspace in FP32 words: the final pass's phi, the
// direction sums of every iteration, with periodic boundaries (nested order) the
// passes before the last; then, for the adjoint, a warm-started call's inflow
// when the adjoint recomputes the first pass (several source iterations, or the
// merged order: the forward overwrites the final phi it took it from), and with
// pbc_tol the passes each iteration ran.
struct SavedLayout {
  int64_t words = 0;
  int64_t warm = -1;    // offset of the warm start's inflow, -1: none
  int64_t counts = -1;  // offset of the pass counts ([n_scat] FP32), -1: none
};

static SavedLayout saved_layout(sweep_dag_t d, int32_t G, const sweep_fwd_opts_t* opts) {
  SavedLayout L;
  const int n_scat = opts ? std::max(1, opts->n_scat) : 1;
  const bool periodic = opts && opts->boundary == SWEEP_BOUNDARY_PERIODIC;
  const bool merge = periodic && opts->merge && n_scat > 1;
  const int64_t CG = d->C_total * G, DCG = CG * d->D;
  const int64_t extra = periodic && !merge ? (int64_t)std::max(0, opts->n_pbc - 1) * DCG : 0;
  L.words = DCG + n_scat * CG + extra;
  if (periodic && opts->warm_start && n_scat > 1) {
    L.warm = L.words;
    L.words += DCG;
  }
  if (periodic && !merge && opts->pbc_tol > 0.0 && opts->n_pbc > 1) {
    L.counts = L.words;
    L.words += n_scat;
  }
  return L;
}

size_t sweep_saved_bytes(sweep_dag_t d, int32_t G, const sweep_fwd_opts_t* opts) {
  if (!dag_ok(d) || G < 1) return 0;
  return sizeof(float) * (size_t)saved_layout(d, G, opts).words;
}

sweep_status_t sweep_forward(sweep_dag_t d, int32_t G, const float* kappa, const float* emission,
                             const sweep_fwd_opts_t* opts, float* J, float* absorbed,
                             double* totals, void* saved, size_t saved_bytes, void* stream) {
  g_err.clear();
  ST_TRY(check_common(d, G));
  ST_TRY(check_buffer_range(d, G));
  FwdPlan p;
  ST_TRY(read_opts(opts, &p));
  if (!kappa || !emission || !J || !absorbed || !totals)
    return fail(SWEEP_ERR_INVALID_ARG, "kappa, emission, J, absorbed and totals are required");
  const bool periodic = p.boundary == SWEEP_BOUNDARY_PERIODIC;
  if (periodic && !d->has_shift)
    return fail(SWEEP_ERR_INVALID_ARG, "periodic boundaries need meshes built with face_shift");
  const size_t need = sweep_saved_bytes(d, G, opts);
  if (saved && saved_bytes < need)
    return fail(SWEEP_ERR_INVALID_ARG, "saved workspace has %zu bytes, %zu needed", saved_bytes, need);
  // merged: periodic passes and source iterations advance together, max(n_pbc, n_scat)
  // passes, each taking its scattering source and its periodic inflow from the one
  // before (the same as the nested order unless both are iterated)
  const bool merge = p.merge && periodic && p.n_scat > 1;
  const int n_outer = merge ? 1 : p.n_scat;
  const int n_inner = merge ? std::max(p.n_pbc, p.n_scat) : p.n_pbc;
  const bool warm = p.warm && periodic;
  if (warm && !saved)
    return fail(SWEEP_ERR_INVALID_ARG, "warm_start takes the periodic inflow from `saved`, which is NULL");
  // convergence threshold (sec. 2.7): after every pass from the second on, E is read
  // back and the passes of the iteration stop once it is below pbc_tol everywhere
  const bool tol = periodic && p.pbc_tol > 0.0 && n_inner > 1;
  if (tol && merge)
    return fail(SWEEP_ERR_INVALID_ARG, "pbc_tol applies to the nested order, not to merge");
  if (tol && p.use_graph)
    return fail(SWEEP_ERR_INVALID_ARG, "pbc_tol stops on values read back each pass; it cannot be "
                                       "captured in a graph (use_graph)");
  hipStream_t s = (hipStream_t)stream;
  StreamScope stream_scope(s);
  const int64_t CG = d->C_total * G;
  const int64_t DCG = CG * d->D;
  ST_TRY(ensure_reduce_tables(d, G));
  ST_TRY(prepare_steps(d, p, G, s));
  if (!saved) HIP_TRY(d->phi_a.alloc(4 * DCG));
  if (periodic && n_inner > 1) HIP_TRY(d->phi_b.alloc(4 * DCG));
  if (warm) HIP_TRY(d->phi_w.alloc(4 * DCG));
  if (periodic) ST_TRY(alloc_periodic(d, G));
  const int64_t n_tot = (int64_t)d->n_meshes * G * 8;
  std::vector<double> tot_host(tol ? n_tot : 0);
  if (!saved || merge) {
    HIP_TRY(d->jsum_a.alloc(4 * CG));
    HIP_TRY(d->jsum_b.alloc(4 * CG));
  }
  float* phi_final = saved ? (float*)saved : d->phi_a.as<float>();
  auto ckpt = [&](int it) -> float* {
    if (saved) return (float*)saved + DCG + (int64_t)it * CG;
    return (it % 2 == 0) ? d->jsum_a.as<float>() : d->jsum_b.as<float>();
  };
  // direction sums of merged pass k (alternating buffers)
  auto jm = [&](int k) -> float* { return (k % 2 == 0) ? d->jsum_a.as<float>() : d->jsum_b.as<float>(); };
  // with `saved`, the periodic passes before the last keep their phi there (after the
  // checkpoints) for the adjoint
  const bool store_passes = saved && periodic && !merge;
  auto pass_slot = [&](int ps) -> float* {
    return (float*)saved + DCG + (int64_t)p.n_scat * CG + (int64_t)ps * DCG;
  };
  ST_TRY(ensure_mesh_tables(d));
  HIP_TRY(d->tden.alloc(4 * (size_t)d->T * G));
  HIP_TRY(d->tsrc.alloc(4 * (size_t)d->T * G));
  HIP_TRY(d->crec.alloc(8 * (size_t)d->C_total * G));
  HIP_TRY(d->out_s.alloc(4 * (size_t)d->T * G));
  const sweep::ReduceArgs r = reduce_args(d, G, p, kappa, emission, J, absorbed);
  // source iterations, each made of the periodic passes (or the merged sequence),
  // then the totals
  // the inflow of a warm start kept for the adjoint's recomputation, and the
  // pass counts of pbc_tol (see saved_layout)
  const SavedLayout lay = saved_layout(d, G, opts);
  float* warm_saved = saved && warm && lay.warm >= 0 ? (float*)saved + lay.warm : nullptr;
  float* counts_saved = saved && tol && lay.counts >= 0 ? (float*)saved + lay.counts : nullptr;
  auto body = [&](hipStream_t st) -> sweep_status_t {
    if (warm)  // the previous call's final phi, before this call overwrites `saved`
      HIP_TRY(hipMemcpyAsync(d->phi_w.p, saved, 4 * DCG, hipMemcpyDeviceToDevice, st));
    if (warm_saved != nullptr)
      HIP_TRY(hipMemcpyAsync(warm_saved, d->phi_w.p, 4 * DCG, hipMemcpyDeviceToDevice, st));
    bool fresh = false;  // tsrc holds the sources run_prep just wrote
    for (int it = 0; it < n_outer; ++it) {
      const float* jprev_it = it > 0 ? ckpt(it - 1) : nullptr;
      float* prev = (warm && it == 0) ? d->phi_w.as<float>() : nullptr;
      // the periodic inflow of the last two passes, summed over directions
      // (nullptr: a pass without a previous one, zero inflow)
      const double* psum_last = nullptr;
      const double* psum_before = nullptr;
      for (int ps = 0; ps < n_inner; ++ps) {
        float* dst = store_passes ? (ps == n_inner - 1 ? phi_final : pass_slot(ps))
                     : ((n_inner - 1 - ps) % 2 == 0) ? phi_final : d->phi_b.as<float>();
        const float* jprev = merge ? (ps > 0 ? jm(ps - 1) : nullptr) : jprev_it;
        const bool final_pass = ps + 1 == n_inner;
        if (ps == 0 || merge) {
          ST_TRY(run_prep(d, G, kappa, emission, nullptr, jprev, p.albedo, p.law, st));
          fresh = true;
        }
        double* psum_ps = nullptr;
        if (periodic && prev != nullptr) {
          psum_ps = (ps % 2 == 0) ? d->psum_a.as<double>() : d->psum_b.as<double>();
          ST_TRY(run_pin(d, false, G, prev, psum_ps, fresh, st));
        }
        psum_before = psum_last;
        psum_last = psum_ps;
        ST_TRY(run_sweep(d, false, p, G, dst, st));
        if (tol) {
          // the full reduction after every pass: E against the previous pass's
          // inflow, then the totals read back
          sweep::ReduceArgs q = r;
          q.phi = dst;
          q.pc_map = d->pc_map.as<int32_t>();
          q.psum = psum_last;
          q.psum_prev = psum_before;
          q.with_e = ps > 0 ? 1 : 0;
          q.jsum_prev = jprev;
          q.jsum = ckpt(it);
          {
            ProfScope pr("reduce", st);
            HIP_TRY(sweep::launch_reduce(q, d->red_blocks, st));
          }
          bool stop = final_pass;
          if (ps > 0 && !final_pass) {
            HIP_TRY(sweep::launch_totals(d->partial.as<double>(), d->mesh_blk_base.as<int32_t>(),
                                         d->n_meshes, G, totals, st));
            HIP_TRY(hipMemcpyAsync(tot_host.data(), totals, 8 * n_tot, hipMemcpyDeviceToHost, st));
            ST_TRY(take_device_error(d, st));
            double emax = 0.0;
            for (int64_t i = 6; i < n_tot; i += 8) emax = std::max(emax, tot_host[i]);
            stop = emax < p.pbc_tol;
          }
          if (stop) {
            if (dst != phi_final)
              HIP_TRY(hipMemcpyAsync(phi_final, dst, 4 * DCG, hipMemcpyDeviceToDevice, st));
            if (counts_saved != nullptr)
              HIP_TRY(sweep::launch_fill_f32(counts_saved + it, 1, (float)(ps + 1), st));
            break;
          }
          prev = dst;
          continue;
        }
        if (!final_pass && merge) {
          // the direction sums that feed the next merged pass's source
          sweep::ReduceArgs q = r;
          q.phi = dst;
          q.jsum_prev = jprev;
          q.jsum = jm(ps);
          HIP_TRY(sweep::launch_reduce(q, d->red_blocks, st));
        }
        prev = dst;
      }
      if (tol) continue;  // the last pass's reduction is done
      sweep::ReduceArgs q = r;
      q.phi = phi_final;
      q.pc_map = periodic ? d->pc_map.as<int32_t>() : nullptr;
      q.psum = psum_last;
      q.psum_prev = psum_before;
      q.with_e = periodic && n_inner > 1 ? 1 : 0;
      q.jsum_prev = merge ? (n_inner > 1 ? jm(n_inner - 2) : nullptr) : jprev_it;
      q.jsum = merge ? jm(n_inner - 1) : ckpt(it);
      {
        ProfScope ps("reduce", st);
        HIP_TRY(sweep::launch_reduce(q, d->red_blocks, st));
      }
      // merged: the final pass's sums are the last iteration's checkpoint
      if (merge && saved)
        HIP_TRY(hipMemcpyAsync(ckpt(p.n_scat - 1), jm(n_inner - 1), 4 * CG, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(sweep::launch_totals(d->partial.as<double>(), d->mesh_blk_base.as<int32_t>(),
                                 d->n_meshes, G, totals, st));
    return SWEEP_OK;
  };
  if (!p.use_graph) {
    ST_TRY(body(s));
  } else {
    std::vector<uint64_t> key = {1, (uint64_t)G, pkey(kappa), pkey(emission), pkey(J), pkey(absorbed),
                                 pkey(totals), pkey(saved), (uint64_t)saved_bytes};
    opts_key(key, p);
    for (const Buf* b : {&d->phi_a, &d->phi_b, &d->phi_w, &d->pbase, &d->pval, &d->psum_a, &d->psum_b,
                         &d->jsum_a, &d->jsum_b, &d->partial, &d->tden, &d->tsrc, &d->crec, &d->out_s,
                         &d->mesh_blk_base, &d->blk_mesh, &d->blk_cell0})
      key.push_back(pkey(b->p));
    ST_TRY(run_graph(d, key, s, body));
  }
  return p.check ? take_device_error(d, s) : SWEEP_OK;
}

sweep_status_t sweep_adjoint(sweep_dag_t d, int32_t G, const float* kappa,
                             const float* emission, const sweep_fwd_opts_t* opts,
                             const void* saved, size_t saved_bytes, const float* dL_dJ,
                             const float* dL_dabsorbed, float* dL_dkappa, float* dL_demission,
                             void* stream) {
  g_err.clear();
  ST_TRY(check_common(d, G));
  ST_TRY(check_buffer_range(d, G));
  FwdPlan p;
  ST_TRY(read_opts(opts, &p));
  const bool periodic = p.boundary == SWEEP_BOUNDARY_PERIODIC;
  // merged order (sec. 2.7): one sequence of max(n_pbc, n_scat) passes
  const bool merge = periodic && p.merge && p.n_scat > 1;
  // pbc_tol: the forward keeps the passes each iteration ran (held fixed here)
  const bool tol = periodic && !merge && p.pbc_tol > 0.0 && p.n_pbc > 1;
  if (tol && p.use_graph)
    return fail(SWEEP_ERR_INVALID_ARG, "the adjoint of pbc_tol takes its pass counts from `saved`; "
                                       "it cannot be captured in a graph (use_graph)");
  if (periodic && !d->has_shift)
    return fail(SWEEP_ERR_INVALID_ARG, "periodic boundaries need meshes built with face_shift");
  if (!kappa || !emission || !saved || !dL_dJ || !dL_dabsorbed || !dL_dkappa || !dL_demission)
    return fail(SWEEP_ERR_INVALID_ARG, "missing array argument");
  const size_t need = sweep_saved_bytes(d, G, opts);
  if (saved_bytes < need)
    return fail(SWEEP_ERR_INVALID_ARG, "saved workspace has %zu bytes, %zu needed", saved_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  StreamScope stream_scope(s);
  const int64_t CG = d->C_total * G;
  const int64_t DCG = CG * d->D;
  // P passes per iteration: x^0..x^{P-1}; the last iteration's are in `saved`
  // (x^{P-1} first, the others after the checkpoints), earlier iterations'
  // are recomputed into phi_a (x^{P-1}) and xpass (the others)
  const int P = merge ? std::max(p.n_pbc, p.n_scat) : periodic ? p.n_pbc : 1;
  ST_TRY(ensure_mesh_tables(d));
  ST_TRY(prepare_steps(d, p, G, s));
  HIP_TRY(d->lam.alloc(4 * DCG));
  HIP_TRY(d->gsrc.alloc(4 * CG));
  HIP_TRY(d->dk64.alloc(8 * CG));
  HIP_TRY(d->de64.alloc(8 * CG));
  if (merge) {
    ST_TRY(ensure_reduce_tables(d, G));
    HIP_TRY(d->xpass.alloc(4 * DCG * P));
    HIP_TRY(d->jpass.alloc(4 * CG * P));
    HIP_TRY(d->jscr.alloc(8 * CG));
  } else {
    if (p.n_scat > 1) HIP_TRY(d->phi_a.alloc(4 * DCG));
    if (p.n_scat > 1 && P > 1) HIP_TRY(d->xpass.alloc(4 * DCG * (P - 1)));
  }
  if (P > 1) HIP_TRY(d->lam_b.alloc(4 * DCG));
  if (periodic) ST_TRY(alloc_periodic(d, G));
  HIP_TRY(d->tden.alloc(4 * (size_t)d->T * G));
  HIP_TRY(d->tsrc.alloc(4 * (size_t)d->T * G));
  HIP_TRY(d->crec.alloc(8 * (size_t)d->C_total * G));
  HIP_TRY(d->out_s.alloc(4 * (size_t)d->T * G));
  const float* phi_final = (const float*)saved;
  auto ckpt = [&](int it) -> const float* { return (const float*)saved + DCG + (int64_t)it * CG; };
  // a warm start's inflow (the forward kept it in `saved` when the first pass has
  // to be recomputed; held fixed: no gradient flows into it), and with pbc_tol
  // the passes of every iteration
  const SavedLayout lay = saved_layout(d, G, opts);
  const float* warm_saved = periodic && p.warm && lay.warm >= 0 ? (const float*)saved + lay.warm : nullptr;
  std::vector<int> passes(p.n_scat, P);
  if (tol) {
    std::vector<float> cf(p.n_scat);
    HIP_TRY(hipMemcpyAsync(cf.data(), (const float*)saved + lay.counts, 4 * (size_t)p.n_scat,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int it = 0; it < p.n_scat; ++it) {
      const int n = (int)cf[it];
      if (!((float)n == cf[it] && n >= 1 && n <= P))
        return fail(SWEEP_ERR_INVALID_ARG, "`saved` holds no pass counts of a forward call with pbc_tol");
      passes[it] = n;
    }
  }
  auto xp = [&](int it, int ps) -> float* {
    const bool last = it == p.n_scat - 1;
    if (ps == passes[it] - 1) return last ? (float*)saved : d->phi_a.as<float>();
    return last ? (float*)saved + DCG + (int64_t)p.n_scat * CG + (int64_t)ps * DCG
                : d->xpass.as<float>() + (int64_t)ps * DCG;
  };
  // reverse iterations: recompute the passes of iteration `it` (all but the last,
  // which were saved), run the reverse passes (the last with the loss source, the
  // earlier ones fed through the periodic faces by the later pass's adjoint),
  // accumulate the gradients and the adjoint source of iteration it - 1
  auto body_nested = [&](hipStream_t st) -> sweep_status_t {
    HIP_TRY(sweep::launch_adj_init(dL_dJ, dL_dabsorbed, kappa, d->vol.as<float>(),
                                   ckpt(p.n_scat - 1), p.albedo, G, d->C_total,
                                   d->gsrc.as<float>(), d->dk64.as<double>(),
                                   d->de64.as<double>(), d->flag.as<int32_t>(), st));
    bool fresh = false;  // tsrc holds the sources run_prep (or the clear) just wrote
    for (int it = p.n_scat - 1; it >= 0; --it) {
      const float* jprev = it > 0 ? ckpt(it - 1) : nullptr;
      const int Pi = passes[it];  // the passes the forward ran in this iteration
      if (it != p.n_scat - 1) {
        ST_TRY(run_prep(d, G, kappa, emission, nullptr, jprev, p.albedo, p.law, st));
        fresh = true;
        for (int ps = 0; ps < Pi; ++ps) {
          if (ps > 0) ST_TRY(run_pin(d, false, G, xp(it, ps - 1), nullptr, fresh, st));
          else if (it == 0 && warm_saved != nullptr)
            ST_TRY(run_pin(d, false, G, warm_saved, nullptr, fresh, st));
          ST_TRY(run_sweep(d, false, p, G, xp(it, ps), st));
        }
      }
      for (int ps = Pi - 1; ps >= 0; --ps) {
        const bool loss_pass = ps == Pi - 1;
        // pass ps's lambda; through its periodic outflow faces a task takes the later
        // pass's lambda at the partners (the adjoint of the forward pass's periodic
        // inflow, folded into the sources), so the two alternate between two buffers
        float* lam_ps = ((Pi - 1 - ps) & 1) ? d->lam_b.as<float>() : d->lam.as<float>();
        const float* lam_next = loss_pass ? nullptr
                                          : (((Pi - 2 - ps) & 1) ? d->lam_b.as<float>() : d->lam.as<float>());
        // the passes before the last have no source of their own: the denominators
        // of the loss pass stand and only the sources are cleared
        // (once cleared, the sources stay zero but for the periodic tasks', which
        // the fold rewrites from their saved zeros)
        if (loss_pass) {
          ST_TRY(run_prep(d, G, kappa, nullptr, d->gsrc.as<float>(), nullptr, p.albedo, p.law, st));
        } else {
          if (ps == Pi - 2) {
            HIP_TRY(sweep::launch_fill_f32(d->tsrc.as<float>(), d->T * G, 0.0f, st));
            fresh = true;
          }
          ST_TRY(run_pin(d, true, G, lam_next, nullptr, fresh, st));
        }
        ST_TRY(run_sweep(d, true, p, G, lam_ps, st));
        sweep::AdjReduceArgs q{};
        q.D = d->D;
        q.G = G;
        q.C_total = d->C_total;
        q.law = p.law;
        q.n_meshes = d->n_meshes;
        q.mesh_off = d->mesh_off_d.as<int32_t>();
        q.aperp = d->aperp.as<float>();
        q.gsrc = d->gsrc.as<float>();
        q.use_g = loss_pass ? 1 : 0;
        q.accumulate = loss_pass ? 0 : 1;
        q.lam = lam_ps;
        q.phi = xp(it, ps);
        q.kappa = kappa;
        q.vol = d->vol.as<float>();
        q.jsum_prev = jprev;
        q.albedo = p.albedo;
        q.inv_D = 1.0f / (float)d->D;
        q.gsrc_next = d->gsrc.as<float>();
        HIP_TRY(sweep::launch_adj_reduce(q, d->dk64.as<double>(), d->de64.as<double>(), st));
      }
    }
    HIP_TRY(sweep::launch_d2f_pair(d->dk64.as<double>(), d->de64.as<double>(), dL_dkappa,
                                   dL_demission, CG, st));
    return SWEEP_OK;
  };
  // merged order: the passes x^p = M^{-1}(S^p + B x^{p-1}), S^p = L/D + a kappa V
  // jsum^{p-1}/D, are recomputed first (every exit value and direction sum kept);
  // then, p = P-1..0, lambda^p = M^{-T}(r g^p + B^T lambda^{p+1}) with g^{P-1} the
  // loss's and g^{p-1} = a kappa V sum_d lambda^p / D (the adjoint reduction writes
  // it over g^p), each pass adding its own terms to the gradients
  auto xm = [&](int ps) -> float* { return d->xpass.as<float>() + (int64_t)ps * DCG; };
  auto jmp = [&](int ps) -> float* { return d->jpass.as<float>() + (int64_t)ps * CG; };
  auto body_merged = [&](hipStream_t st) -> sweep_status_t {
    bool fresh = false;
    const sweep::ReduceArgs r = reduce_args(d, G, p, kappa, emission, d->jscr.as<float>(),
                                            d->jscr.as<float>() + CG);
    for (int ps = 0; ps < P; ++ps) {
      const float* jprev = ps > 0 ? jmp(ps - 1) : nullptr;
      ST_TRY(run_prep(d, G, kappa, emission, nullptr, jprev, p.albedo, p.law, st));
      fresh = true;
      if (ps > 0) ST_TRY(run_pin(d, false, G, xm(ps - 1), nullptr, fresh, st));
      else if (warm_saved != nullptr) ST_TRY(run_pin(d, false, G, warm_saved, nullptr, fresh, st));
      ST_TRY(run_sweep(d, false, p, G, xm(ps), st));
      sweep::ReduceArgs q = r;
      q.phi = xm(ps);
      q.jsum_prev = jprev;
      q.jsum = jmp(ps);
      HIP_TRY(sweep::launch_reduce(q, d->red_blocks, st));
    }
    HIP_TRY(sweep::launch_adj_init(dL_dJ, dL_dabsorbed, kappa, d->vol.as<float>(), jmp(P - 1),
                                   p.albedo, G, d->C_total, d->gsrc.as<float>(),
                                   d->dk64.as<double>(), d->de64.as<double>(),
                                   d->flag.as<int32_t>(), st));
    for (int ps = P - 1; ps >= 0; --ps) {
      float* lam_ps = ((P - 1 - ps) & 1) ? d->lam_b.as<float>() : d->lam.as<float>();
      const float* lam_next = ps == P - 1 ? nullptr
                                          : (((P - 2 - ps) & 1) ? d->lam_b.as<float>() : d->lam.as<float>());
      ST_TRY(run_prep(d, G, kappa, nullptr, d->gsrc.as<float>(), nullptr, p.albedo, p.law, st));
      fresh = true;
      if (lam_next != nullptr) ST_TRY(run_pin(d, true, G, lam_next, nullptr, fresh, st));
      ST_TRY(run_sweep(d, true, p, G, lam_ps, st));
      sweep::AdjReduceArgs q{};
      q.D = d->D;
      q.G = G;
      q.C_total = d->C_total;
      q.law = p.law;
      q.n_meshes = d->n_meshes;
      q.mesh_off = d->mesh_off_d.as<int32_t>();
      q.aperp = d->aperp.as<float>();
      q.gsrc = d->gsrc.as<float>();
      q.use_g = 1;
      q.accumulate = 0;
      q.lam = lam_ps;
      q.phi = xm(ps);
      q.kappa = kappa;
      q.vol = d->vol.as<float>();
      q.jsum_prev = ps > 0 ? jmp(ps - 1) : nullptr;
      q.albedo = p.albedo;
      q.inv_D = 1.0f / (float)d->D;
      q.gsrc_next = d->gsrc.as<float>();
      HIP_TRY(sweep::launch_adj_reduce(q, d->dk64.as<double>(), d->de64.as<double>(), st));
    }
    HIP_TRY(sweep::launch_d2f_pair(d->dk64.as<double>(), d->de64.as<double>(), dL_dkappa,
                                   dL_demission, CG, st));
    return SWEEP_OK;
  };
  auto body = [&](hipStream_t st) -> sweep_status_t { return merge ? body_merged(st) : body_nested(st); };
  if (!p.use_graph) {
    ST_TRY(body(s));
  } else {
    std::vector<uint64_t> key = {2, (uint64_t)G, pkey(kappa), pkey(emission), pkey(saved),
                                 (uint64_t)saved_bytes, pkey(dL_dJ), pkey(dL_dabsorbed),
                                 pkey(dL_dkappa), pkey(dL_demission)};
    opts_key(key, p);
    for (const Buf* b : {&d->lam, &d->gsrc, &d->dk64, &d->de64, &d->phi_a, &d->xpass, &d->lam_b,
                         &d->pbase, &d->pval, &d->tden, &d->tsrc, &d->crec, &d->out_s, &d->jpass,
                         &d->jscr, &d->partial, &d->mesh_blk_base, &d->blk_mesh, &d->blk_cell0})
      key.push_back(pkey(b->p));
    ST_TRY(run_graph(d, key, s, body));
  }
  return p.check ? take_device_error(d, s) : SWEEP_OK;
}

sweep_status_t sweep_tune(sweep_dag_t d, int32_t G, const float* kappa, const float* emission,
                          const sweep_fwd_opts_t* opts, int32_t reps, sweep_fwd_opts_t* best,
                          double* best_ms, void* stream) {
  g_err.clear();
  ST_TRY(check_common(d, G));
  ST_TRY(check_buffer_range(d, G));
  FwdPlan p;
  ST_TRY(read_opts(opts, &p));
  if (!kappa || !emission || !best || !best_ms) return fail(SWEEP_ERR_INVALID_ARG, "missing argument");
  if (reps < 1) return fail(SWEEP_ERR_INVALID_ARG, "reps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  StreamScope stream_scope(s);
  const int64_t DCG = d->C_total * G * d->D;
  HIP_TRY(d->phi_a.alloc(4 * DCG));
  HIP_TRY(d->tden.alloc(4 * (size_t)d->T * G));
  HIP_TRY(d->tsrc.alloc(4 * (size_t)d->T * G));
  HIP_TRY(d->crec.alloc(8 * (size_t)d->C_total * G));
  HIP_TRY(d->out_s.alloc(4 * (size_t)d->T * G));
  ST_TRY(run_prep(d, G, kappa, emission, nullptr, nullptr, p.albedo, p.law, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(SWEEP_ERR_HIP, "hipEventCreate failed");
  }
  const int gn = group_plan(d, G, false, p.pack)[0].gn;
  double best_t = -1.0;
  FwdPlan bp = p;
  sweep_status_t st = SWEEP_OK;
  for (int block : {256, 512, 1024}) {
    if (block > sweep::kSweepMaxBlock(gn)) continue;
    const int r0 = default_ring(d, gn, block);
    for (int ring : {r0 / 4, r0 / 2, r0}) {
      if (ring < 64) continue;
      FwdPlan q = p;
      q.form = SWEEP_FORM_BATCHED;
      q.block = block;
      q.ring = ring;
      q.use_graph = 0;
      // one untimed sweep, then `reps` timed ones
      st = run_sweep(d, false, q, G, d->phi_a.as<float>(), s);
      if (st != SWEEP_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) { st = fail(SWEEP_ERR_HIP, "hipEventRecord"); break; }
      for (int r = 0; r < reps && st == SWEEP_OK; ++r)
        st = run_sweep(d, false, q, G, d->phi_a.as<float>(), s);
      if (st != SWEEP_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(SWEEP_ERR_HIP, "event timing failed");
        break;
      }
      const double t = ms / reps;
      if (best_t < 0.0 || t < best_t) {
        best_t = t;
        bp = q;
      }
    }
    if (st != SWEEP_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SWEEP_OK) return st;
  ST_TRY(take_device_error(d, s));
  if (best_t < 0.0) return fail(SWEEP_ERR_UNSUPPORTED, "no launch shape fits the LDS");
  if (opts) *best = *opts;
  else std::memset(best, 0, sizeof(*best));
  best->block = bp.block;
  best->ring = bp.ring;
  best->pack = gn;
  *best_ms = best_t;
  return SWEEP_OK;
}

}  // extern "C"

namespace {

// One photoionisation step; `minbuf` (device, 8 bytes) receives the step limit.
sweep_status_t ion_step(sweep_dag_t d, const float* absorbed, const sweep_ion_params_t* p,
                        double t_left, double* neutral, float* kappa, double* dt, hipStream_t s,
                        unsigned long long* minbuf) {
  sweep::IonArgs a{};
  a.n = d->C_total;
  a.vol = d->vol.as<float>();
  a.absorbed = absorbed;
  a.neutral = neutral;
  a.kappa = kappa;
  a.n_H = p->n_H;
  a.sigma_H = p->sigma_H;
  a.alpha_B = p->alpha_B;
  a.photon_rate = p->photon_rate;
  a.length_unit = p->length_unit;
  a.l3 = p->length_unit * p->length_unit * p->length_unit;
  HIP_TRY(sweep::launch_ion_limit(a, minbuf, s));  // writes +inf first, then the minimum
  uint64_t bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, minbuf, 8, hipMemcpyDeviceToHost, s));
  ST_TRY(take_device_error(d, s));
  double lim;
  std::memcpy(&lim, &bits, 8);
  const double step = std::min(std::min(p->dt_max, t_left), p->courant * lim);
  HIP_TRY(sweep::launch_ion_update(a, step, s));
  *dt = step;
  return SWEEP_OK;
}

sweep_status_t check_ion_args(sweep_dag_t d, const float* absorbed, const sweep_ion_params_t* p,
                              double t_left, double* neutral, float* kappa, double* dt) {
  ST_TRY(check_common(d, 1));
  if (!absorbed || !p || !neutral || !kappa || !dt)
    return fail(SWEEP_ERR_INVALID_ARG, "missing argument");
  if (!(p->n_H > 0.0) || !(p->sigma_H > 0.0) || !(p->alpha_B > 0.0) || !(p->photon_rate > 0.0) ||
      !(p->length_unit > 0.0) || !(p->dt_max > 0.0) || !(t_left > 0.0))
    return fail(SWEEP_ERR_INVALID_ARG, "n_H, sigma_H, alpha_B, photon_rate, length_unit, dt_max "
                                       "and t_left must be positive");
  if (!(p->courant > 0.0) || !(p->courant <= 1.0))
    return fail(SWEEP_ERR_INVALID_ARG, "courant must be in (0, 1]");
  return SWEEP_OK;
}

}  // namespace

extern "C" {

sweep_status_t sweep_ion_step(sweep_dag_t d, const float* absorbed, const sweep_ion_params_t* p,
                              double t_left, double* neutral, float* kappa, double* dt,
                              void* stream) {
  g_err.clear();
  ST_TRY(check_ion_args(d, absorbed, p, t_left, neutral, kappa, dt));
  hipStream_t s = (hipStream_t)stream;
  StreamScope stream_scope(s);
  HIP_TRY(d->ion_min.alloc(8));
  return ion_step(d, absorbed, p, t_left, neutral, kappa, dt, s,
                  d->ion_min.as<unsigned long long>());
}

sweep_status_t sweep_ion_step_noalloc(sweep_dag_t d, const float* absorbed,
                                      const sweep_ion_params_t* p, double t_left, double* neutral,
                                      float* kappa, double* dt, void* stream) {
  g_err.clear();
  ST_TRY(check_ion_args(d, absorbed, p, t_left, neutral, kappa, dt));
  hipStream_t s = (hipStream_t)stream;
  StreamScope stream_scope(s);
  unsigned long long* scratch = nullptr;  // the library's static scratch word on this device
  HIP_TRY(sweep::ion_scratch(&scratch));
  return ion_step(d, absorbed, p, t_left, neutral, kappa, dt, s, scratch);
}

sweep_status_t sweep_sync(sweep_dag_t d, void* stream) {
  g_err.clear();
  if (!dag_ok(d)) return fail(SWEEP_ERR_NOT_BUILT, "DAG handle is NULL or was not built");
  return take_device_error(d, (hipStream_t)stream);
}

sweep_status_t sweep_dag_depths(sweep_dag_t d, int32_t* depth) {
  g_err.clear();
  if (!dag_ok(d)) return fail(SWEEP_ERR_NOT_BUILT, "DAG handle is NULL or was not built");
  if (!depth) return fail(SWEEP_ERR_INVALID_ARG, "depth is NULL");
  for (size_t u = 0; u < d->units.size(); ++u) depth[u] = d->units[u].depth;
  return SWEEP_OK;
}

sweep_status_t sweep_dag_level_widths(sweep_dag_t d, int32_t mesh, int64_t* width, int32_t n_levels,
                                      void* stream) {
  g_err.clear();
  if (!dag_ok(d)) return fail(SWEEP_ERR_NOT_BUILT, "DAG handle is NULL or was not built");
  if (!width || n_levels < 0) return fail(SWEEP_ERR_INVALID_ARG, "width is NULL or n_levels < 0");
  if (mesh < -1 || mesh >= d->n_meshes) return fail(SWEEP_ERR_INVALID_ARG, "mesh %d out of range", mesh);
  if (n_levels == 0) return SWEEP_OK;
  hipStream_t s = (hipStream_t)stream;
  StreamScope stream_scope(s);
  Buf w;
  HIP_TRY(w.alloc(8 * (size_t)n_levels));
  HIP_TRY(hipMemsetAsync(w.p, 0, 8 * (size_t)n_levels, s));
  HIP_TRY(sweep::launch_level_widths(d->units_d.as<Unit>(), (int32_t)d->units.size(),
                                     d->lp.as<int32_t>(), mesh, w.as<int64_t>(), n_levels, s));
  HIP_TRY(hipMemcpyAsync(width, w.p, 8 * (size_t)n_levels, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return SWEEP_OK;
}

sweep_status_t sweep_ion_kappa(sweep_dag_t d, const sweep_ion_params_t* p, const double* neutral,
                               float* kappa, void* stream) {
  g_err.clear();
  ST_TRY(check_common(d, 1));
  if (!p || !neutral || !kappa) return fail(SWEEP_ERR_INVALID_ARG, "missing argument");
  if (!(p->n_H > 0.0) || !(p->sigma_H > 0.0) || !(p->length_unit > 0.0))
    return fail(SWEEP_ERR_INVALID_ARG, "n_H, sigma_H and length_unit must be positive");
  sweep::IonArgs a{};
  a.n = d->C_total;
  a.neutral = const_cast<double*>(neutral);
  a.kappa = kappa;
  a.n_H = p->n_H;
  a.sigma_H = p->sigma_H;
  a.length_unit = p->length_unit;
  HIP_TRY(sweep::launch_ion_kappa(a, (hipStream_t)stream));
  return SWEEP_OK;
}

}  // extern "C"
