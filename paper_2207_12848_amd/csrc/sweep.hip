// Forward and adjoint sweep kernels and the per-cell reductions (gfx950).
//
// Schedule: one workgroup owns one (mesh, direction) sweep at a time and walks
// its levels in order (reverse order for the adjoint), one barrier per level.
// The tasks of a level are independent (their upwind tasks sit on earlier
// levels), so the workgroup's threads solve them in parallel; every task pulls
// its inflow from its upwind tasks' results in a fixed row order, so results do
// not depend on which thread runs which task.  Persistent form: a grid sized to
// the resident capacity takes (mesh, direction) units from an atomic counter,
// longest first.
//
// LDS ring: the results of the last `ring` tasks of the schedule are kept in
// LDS, indexed by schedule position modulo `ring`, so most upwind reads are LDS
// reads; an older upwind result is read back from global memory (it was stored
// at least one barrier earlier by the same workgroup).
#include "internal.h"

namespace sweep {

namespace {

constexpr float kInv4Pi = 0.0795774715459476678f;  // 1 / (4 pi)

// Record of one task: cell, row [r0, r1) relative to its level's first entry,
// denominator and source per group.
template <int GN>
struct TaskRec {
  int c;
  int r0, r1;
  float den[GN];
  float src[GN];
};

// Loads prefetched for one level: the thread's share of the level's row block
// and the raw record of the thread's first task of the level (no arithmetic on
// loaded values until they are published, so the loads stay in flight).
// Per-step values, uniform over the workgroup.
struct LevelInfo {
  int l, k0, k1;  // level and its task range
  int nst;        // entries of the level held in LDS staging
  int thr;        // ring-miss threshold for entries served from registers
  int64_t e0;     // first row entry of the level
};

template <int GN, int CH>
struct Pref {
  LevelInfo L;
  int2 st[CH];
  float mv[CH];    // GN == 1: value behind a ring miss or a periodic inflow of st[i]
  uint32_t codes;  // 2 bits per chunk: 1 ring miss, 2 periodic inflow
  int c;
  uint32_t rp0, rp1;  // low words of the row pointers (row offsets are taken mod 2^32)
  float den[GN];
  float src[GN];
};

template <int GN>
__device__ __forceinline__ void load_rec(const SweepArgs& a, int64_t tb, int k, int64_t e0,
                                         TaskRec<GN>& t) {
  t.c = a.sched[tb + k];
  t.r0 = (int)(a.row_ptr[tb + k] - e0);
  t.r1 = (int)(a.row_ptr[tb + k + 1] - e0);
  const int64_t q = (tb + k) * a.G + a.g0;
#pragma unroll
  for (int g = 0; g < GN; ++g) {
    t.den[g] = a.tden[q + g];
    t.src[g] = a.tsrc[q + g];
  }
}

// Unconditional loads (addresses clamped into the arrays) so that every path
// issues the same number of vector-memory operations.
template <int GN, int CH>
__device__ __forceinline__ void issue_pref(const SweepArgs& a, int64_t tb, int tid, int nthr,
                                           int k0, int k1, int64_t e0, int ne, Pref<GN, CH>& P) {
  const int64_t emax = a.n_ent > 0 ? a.n_ent - 1 : 0;
#pragma unroll
  for (int i = 0; i < CH; ++i) {
    int64_t e = e0 + (int64_t)tid + (int64_t)i * nthr;
    e = e < emax ? e : emax;
    P.st[i] = a.ent[e];
  }
  int k = k0 + tid;
  k = k < k1 - 1 ? k : k1 - 1;
  P.c = a.sched[tb + k];
  const uint32_t* rpw = reinterpret_cast<const uint32_t*>(a.row_ptr);
  P.rp0 = rpw[2 * (tb + k)];
  P.rp1 = rpw[2 * (tb + k + 1)];
  const int64_t q = (tb + k) * a.G + a.g0;
#pragma unroll
  for (int g = 0; g < GN; ++g) {
    P.den[g] = a.tden[q + g];
    P.src[g] = a.tsrc[q + g];
  }
}

// Entry codes written into LDS staging for prefetched values (GN == 1): the
// entry's second word then holds w * value.
constexpr int kMissCode = (int)0x80000000;
constexpr int kPerCode = (int)0x80000001;

// Inflow of one task per group (and the periodic part of it).
template <int GN>
struct Inflow {
  float acc[GN];
  float pin[GN];
};

template <int GN, bool REVERSE>
__device__ __forceinline__ void finish_task(const SweepArgs& a, const TaskRec<GN>& t, int k,
                                            const Inflow<GN>& in, float* ring, int64_t obase,
                                            int64_t tb) {
  float* rr = ring + (k & a.ring_mask) * GN;
  float* o = a.out + obase + (int64_t)t.c * a.G;
  float* os = a.out_s + (tb + k) * a.G + a.g0;
#pragma unroll
  for (int g = 0; g < GN; ++g) {
    const float v = __fdiv_rn(__fadd_rn(in.acc[g], t.src[g]), t.den[g]);
    rr[g] = v;
    o[g] = v;
    os[g] = v;
  }
  if (!REVERSE && a.pin != nullptr) {
    float* pp = a.pin + obase + (int64_t)t.c * a.G;
#pragma unroll
    for (int g = 0; g < GN; ++g) pp[g] = in.pin[g];
  }
}

// Inflow of one task.  FAST: the row is in LDS staging, where ring misses and
// periodic inflows prefetched a level ahead appear as coded entries; anything
// else (levels larger than the ring, groups packed by more than one) goes
// through a second pass with global loads, so the main loop issues none.
template <int GN, bool REVERSE, bool FAST>
__device__ __forceinline__ Inflow<GN> gather_task(const SweepArgs& a, const TaskRec<GN>& t,
                                                  int k0, int k1, int64_t e0, const int2* stg,
                                                  const float* ring, int64_t obase, int64_t tb) {
  const int R = a.ring_mask + 1;
  Inflow<GN> in;
  float* acc = in.acc;
  float* pin = in.pin;
#pragma unroll
  for (int g = 0; g < GN; ++g) acc[g] = pin[g] = 0.0f;
  bool miss = false;
  // entries in batches of 8, branch-free: all LDS reads of a batch are issued
  // before any is used and every entry kind is folded in with selects
  for (int rb = t.r0; rb < t.r1; rb += 8) {
    int2 en[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = rb + q < t.r1 ? rb + q : t.r1 - 1;
      en[q] = FAST ? stg[r] : a.ent[e0 + r];
    }
    float rv[8][GN];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int pr = en[q].x >= 0 ? en[q].x : 0;
      const float* rr = ring + (pr & a.ring_mask) * GN;
#pragma unroll
      for (int g = 0; g < GN; ++g) rv[q][g] = rr[g];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool valid = rb + q < t.r1;
      const int p = en[q].x;
      const bool in_ring = p >= 0 && (REVERSE ? (p < k0 + R) : (p >= k1 - R));
      const bool is_miss = GN == 1 && p == kMissCode;
      const bool is_per = GN == 1 && p == kPerCode;
      const float y = __int_as_float(en[q].y);
      // explicit rounding (no contraction): every launch form and group packing
      // computes each task's inflow with the same operations in row order
#pragma unroll
      for (int g = 0; g < GN; ++g) {
        const float c = in_ring ? __fmul_rn(y, rv[q][g]) : ((is_miss || is_per) ? y : 0.0f);
        acc[g] = __fadd_rn(acc[g], valid ? c : 0.0f);
      }
      pin[0] = __fadd_rn(pin[0], (valid && is_per) ? y : 0.0f);
      miss = miss || (valid && !in_ring && !is_miss && !is_per);
    }
  }
  if (miss) {
    for (int r = t.r0; r < t.r1; ++r) {
      const int2 en = FAST ? stg[r] : a.ent[e0 + r];
      const int p = en.x;
      if (p == kMissCode || p == kPerCode) continue;
      const float w = __int_as_float(en.y);
      if (p >= 0) {
        if (REVERSE ? (p < k0 + R) : (p >= k1 - R)) continue;
        const float* q = a.out_s + (tb + p) * a.G + a.g0;
#pragma unroll
        for (int g = 0; g < GN; ++g) acc[g] = __fadd_rn(acc[g], __fmul_rn(w, q[g]));
      } else if (a.phi_prev != nullptr) {
        const float* q = a.phi_prev + obase + (int64_t)(-p - 1) * a.G;
#pragma unroll
        for (int g = 0; g < GN; ++g) {
          const float v = __fmul_rn(w, q[g]);
          acc[g] = __fadd_rn(acc[g], v);
          pin[g] = __fadd_rn(pin[g], v);
        }
      }
    }
  }
  return in;
}

// One workgroup per (mesh, direction) unit at a time, levels in order (reverse
// for the adjoint), one barrier per level.  Each level's rows are one block of
// entries; a level's block and the records of its tasks are loaded three
// levels ahead into registers (three rotating sets) and written to one of two
// LDS staging buffers the level before it is solved.
// LVL_LDS = false (graphs deeper than the LDS level tables hold): the level
// pointers and first entries are read from global memory at every step.
template <int GN, bool REVERSE, int CH, bool LVL_LDS>
__global__ __launch_bounds__(kStageEntries / CH) void k_sweep(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* ring = reinterpret_cast<float*>(smem);
  int2* stage = reinterpret_cast<int2*>(smem + a.stage_off);
  int32_t* lps = reinterpret_cast<int32_t*>(smem + a.lp_off);
  int64_t* levs = reinterpret_cast<int64_t*>(smem + a.lev_off);
  __shared__ int s_unit;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int SE = CH * nthr;
  for (int it = 0;; ++it) {
    int ui;
    if (a.work_counter != nullptr) {
      if (tid == 0) s_unit = atomicAdd(a.work_counter, 1);
      __syncthreads();
      ui = s_unit;
      __syncthreads();
    } else {
      ui = it == 0 ? (int)blockIdx.x : a.n_units;
    }
    if (ui >= a.n_units) break;
    const Unit U = a.units[a.unit_order[ui]];
    const int64_t tb = U.task_base;
    const int depth = U.depth;
    if (depth <= 0) continue;
    // level tables in LDS (the host sizes lp_cap >= depth + 2 for every unit)
    if (LVL_LDS) {
      for (int l = tid; l <= depth + 1; l += nthr) {
        lps[l] = a.lp[U.lp_base + l];
        levs[l] = a.lev[U.lp_base + l];
      }
    }
    __syncthreads();
    const int32_t* lpg = a.lp + U.lp_base;
    const int64_t* levg = a.lev + U.lp_base;
    auto LP = [&](int l) -> int { return LVL_LDS ? lps[l] : lpg[l]; };
    auto LEV = [&](int l) -> int64_t { return LVL_LDS ? levs[l] : levg[l]; };
    auto LVL = [&](int s) -> int {  // level solved at step s (clamped into range)
      s = s < depth - 1 ? s : depth - 1;
      return REVERSE ? depth - 1 - s : s;
    };
    const int64_t obase = ((int64_t)U.dir * a.C_total + U.cell_off) * a.G + a.g0;
    Pref<GN, CH> P0, P1, P2;
    TaskRec<GN> cur;
    const int R = a.ring_mask + 1;
    auto info = [&](int s) -> LevelInfo {
      LevelInfo L;
      L.l = LVL(s);
      L.k0 = LP(L.l);
      L.k1 = LP(L.l + 1);
      L.e0 = LEV(L.l);
      const int ne = (int)(LEV(L.l + 1) - L.e0);
      L.nst = ne < SE ? ne : SE;
      // a ring miss is served from registers when its producer completed before
      // the step two earlier started (its value is then visible to every wave)
      const int ls = LVL(s - 2 < 0 ? 0 : s - 2);
      L.thr = REVERSE ? max(L.k0 + R, LP(ls + 1)) : min(L.k1 - R, LP(ls));
      return L;
    };
    LevelInfo curL;
    auto issue = [&](int s, Pref<GN, CH>& P) {
      P.L = info(s);
      issue_pref<GN, CH>(a, tb, tid, nthr, P.L.k0, P.L.k1, P.L.e0, P.L.nst, P);
    };
    auto missload = [&](Pref<GN, CH>& P) {
      P.codes = 0;
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int p = P.st[i].x;
        uint32_t cd = 0;
        if (GN == 1 && tid + i * nthr < P.L.nst)
          cd = p < 0 ? 2u : ((REVERSE ? p >= P.L.thr : p < P.L.thr) ? 1u : 0u);
        P.codes |= cd << (2 * i);
        const float* q = a.tden;  // any valid address
        if (cd == 1) q = a.out_s + (tb + p) * a.G + a.g0;
        if (cd == 2 && a.phi_prev != nullptr) q = a.phi_prev + obase + (int64_t)(-p - 1) * a.G;
        P.mv[i] = *q;
      }
    };
    auto publish = [&](int s, const Pref<GN, CH>& P) {
      int2* dst = stage + (s & 1) * SE;
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        if (i * nthr >= P.L.nst) break;
        const int idx = tid + i * nthr;
        int2 en = P.st[i];
        const uint32_t cd = (P.codes >> (2 * i)) & 3u;
        if (cd == 1) en = make_int2(kMissCode, __float_as_int(__int_as_float(en.y) * P.mv[i]));
        if (cd == 2)
          en = make_int2(kPerCode, __float_as_int(a.phi_prev != nullptr ? __int_as_float(en.y) * P.mv[i] : 0.0f));
        if (idx < P.L.nst) dst[idx] = en;
      }
      curL = P.L;
      cur.c = P.L.k0 + tid < P.L.k1 ? P.c : -1;
      cur.r0 = (int)(P.rp0 - (uint32_t)P.L.e0);
      cur.r1 = (int)(P.rp1 - (uint32_t)P.L.e0);
#pragma unroll
      for (int g = 0; g < GN; ++g) {
        cur.den[g] = P.den[g];
        cur.src[g] = P.src[g];
      }
    };
    auto solve = [&](int s) {
      const int k0 = curL.k0, k1 = curL.k1;
      const int64_t e0 = curL.e0;
      const int2* stg = stage + (s & 1) * SE;
      if (curL.nst == (int)(LEV(curL.l + 1) - e0)) {
        if (cur.c >= 0) {
          const Inflow<GN> in = gather_task<GN, REVERSE, true>(a, cur, k0, k1, e0, stg, ring, obase, tb);
          finish_task<GN, REVERSE>(a, cur, k0 + tid, in, ring, obase, tb);
        }
        for (int k = k0 + tid + nthr; k < k1; k += nthr) {
          TaskRec<GN> t;
          load_rec<GN>(a, tb, k, e0, t);
          const Inflow<GN> in = gather_task<GN, REVERSE, true>(a, t, k0, k1, e0, stg, ring, obase, tb);
          finish_task<GN, REVERSE>(a, t, k, in, ring, obase, tb);
        }
      } else {
        for (int k = k0 + tid; k < k1; k += nthr) {
          TaskRec<GN> t;
          if (k == k0 + tid) t = cur; else load_rec<GN>(a, tb, k, e0, t);
          const Inflow<GN> in = gather_task<GN, REVERSE, false>(a, t, k0, k1, e0, stg, ring, obase, tb);
          finish_task<GN, REVERSE>(a, t, k, in, ring, obase, tb);
        }
      }
    };
    // prologue: step 0 staged, steps 1 and 2 in flight.  Step s then solves,
    // issues the loads of step s + 3, the prefetches of step s + 2 and
    // publishes step s + 1.
    issue(0, P0);
    issue(1, P1);
    missload(P0);
    publish(0, P0);
    issue(2, P2);
    missload(P1);
    __syncthreads();
    for (int s = 0; s < depth; s += 3) {
      solve(s);
      issue(s + 3, P0);
      missload(P2);
      if (s + 1 < depth) publish(s + 1, P1);
      __syncthreads();
      if (s + 1 >= depth) break;
      solve(s + 1);
      issue(s + 4, P1);
      missload(P0);
      if (s + 2 < depth) publish(s + 2, P2);
      __syncthreads();
      if (s + 2 >= depth) break;
      solve(s + 2);
      issue(s + 5, P2);
      missload(P1);
      if (s + 3 < depth) publish(s + 3, P0);
      __syncthreads();
    }
  }
}

template <int GN, bool REVERSE>
hipError_t launch_sweep_g(const SweepArgs& a, int32_t grid, int32_t block, size_t lds,
                          hipStream_t s) {
  // kStageEntries entries staged per level whatever the block size; level
  // tables outside LDS (lp_cap == 0) only with 512 threads
  if (a.lp_cap == 0) {
    if (block != 512) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_sweep<GN, REVERSE, 8, false>), dim3(grid), dim3(block), lds, s, a);
    return hipGetLastError();
  }
  switch (kStageEntries / block) {
    case 4: hipLaunchKernelGGL((k_sweep<GN, REVERSE, 4, true>), dim3(grid), dim3(block), lds, s, a); break;
    case 8: hipLaunchKernelGGL((k_sweep<GN, REVERSE, 8, true>), dim3(grid), dim3(block), lds, s, a); break;
    case 16: hipLaunchKernelGGL((k_sweep<GN, REVERSE, 16, true>), dim3(grid), dim3(block), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool REVERSE>
hipError_t launch_sweep_t(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                          size_t lds, hipStream_t s) {
  switch (gn) {
    case 1: return launch_sweep_g<1, REVERSE>(a, grid, block, lds, s);
    case 2: return launch_sweep_g<2, REVERSE>(a, grid, block, lds, s);
    case 3: return launch_sweep_g<3, REVERSE>(a, grid, block, lds, s);
    case 4: return launch_sweep_g<4, REVERSE>(a, grid, block, lds, s);
    default: return hipErrorInvalidValue;
  }
}

// Per-task denominators Aperp + kappa V and sources, first in cell order within
// each unit (every access coalesced).
__device__ __forceinline__ int unit_of_block(const int32_t* blk_base, int n_units, int b) {
  int lo = 0, hi = n_units - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk_base[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  const int u = unit_of_block(a.blk_base, a.n_units, blockIdx.x);
  const Unit U = a.units[u];
  const int c = (blockIdx.x - a.blk_base[u]) * 256 + threadIdx.x;
  if (c >= U.n_cells) return;
  const int64_t t = U.task_base + c;  // cell order: every access is coalesced
  const int64_t ci = (int64_t)U.cell_off + c;
  const double V = (double)a.vol[ci];
  const double ap = (double)a.aperp[t];
  for (int g = 0; g < a.G; ++g) {
    const int64_t cg = ci * a.G + g;
    const double kap = (double)a.kappa[cg];
    a.cden[t * a.G + g] = (float)(ap + kap * V);
    double s;
    if (a.emission != nullptr) {
      s = (double)a.emission[cg];
      if (a.jsum_prev != nullptr) s += (double)a.albedo * kap * V * (double)a.jsum_prev[cg];
      s *= (double)a.inv_D;
    } else {
      s = (double)a.gsrc[cg];
    }
    a.csrc[t * a.G + g] = (float)s;
  }
}

// The same values in schedule order (what the sweep streams): a gather of two
// arrays per unit, which the unit-by-unit block order keeps cache resident.
__global__ __launch_bounds__(256) void k_prep_order(PrepArgs a) {
  const int u = unit_of_block(a.blk_base, a.n_units, blockIdx.x);
  const Unit U = a.units[u];
  const int k = (blockIdx.x - a.blk_base[u]) * 256 + threadIdx.x;
  if (k >= U.n_cells) return;
  const int64_t t = U.task_base + k;
  const int64_t tc = U.task_base + a.sched[t];
  for (int g = 0; g < a.G; ++g) {
    a.tden[t * a.G + g] = a.cden[tc * a.G + g];
    a.tsrc[t * a.G + g] = a.csrc[tc * a.G + g];
  }
}

// ----------------------------------------------------------------------- reductions
constexpr int kRedBlock = 256;
constexpr int kNPart = 9;

__global__ __launch_bounds__(kRedBlock) void k_reduce(ReduceArgs a) {
  __shared__ double part[kRedBlock][kNPart];
  const int m = a.blk_mesh[blockIdx.x];
  const int c0 = a.blk_cell0[blockIdx.x];
  const int G = a.G;
  const int i = threadIdx.x;
  const int c = c0 + i / G;
  const int g = i % G;
  const int mend = a.mesh_off[m] + a.mesh_cells[m];
  const bool active = (i < a.cells_per_block * G) && (c < mend);
  double v[kNPart];
#pragma unroll
  for (int k = 0; k < kNPart; ++k) v[k] = 0.0;
  if (active) {
    const int64_t cg = (int64_t)c * G + g;
    const int64_t stride = a.C_total * G;
    const int lc = c - a.mesh_off[m];
    double js = 0.0, pn = 0.0, esc = 0.0, pout = 0.0;
    for (int d = 0; d < a.D; ++d) {
      const double ph = (double)a.phi[d * stride + cg];
      js += ph;
      if (a.pin != nullptr) pn += (double)a.pin[d * stride + cg];
      if (a.last) {
        const float2 b = a.bnd[a.units[m * a.D + d].task_base + lc];
        esc += (double)b.x * ph;
        pout += (double)b.y * ph;
      }
    }
    if (a.pin_sum != nullptr) a.pin_sum[cg] = pn;
    if (a.last) {
      const double V = (double)a.vol[c];
      const double kap = (double)a.kappa[cg];
      const double ka = (1.0 - (double)a.albedo) * kap;
      const double ks = (double)a.albedo * kap;
      const double ab = ka * V * js;
      a.jsum[cg] = (float)js;
      a.J[cg] = (float)(js * (double)kInv4Pi);
      a.absorbed[cg] = (float)ab;
      const double jp = a.jsum_prev != nullptr ? (double)a.jsum_prev[cg] : 0.0;
      v[0] = (double)a.emission[cg];
      v[1] = ab;
      v[2] = esc;
      v[3] = pn;
      v[4] = pout;
      v[5] = ks * V * (jp - js);
      if (a.pin_prev != nullptr) {
        const double po = a.pin_prev[cg];
        const double den = pn + po;
        v[6] = den > 0.0 ? fabs(pn - po) / den : 0.0;
        v[7] = fabs(pn - po);
        v[8] = den;
      }
    }
  }
  if (!a.last) return;
#pragma unroll
  for (int k = 0; k < kNPart; ++k) part[i][k] = v[k];
  __syncthreads();
  if (i < G) {
    double s[kNPart];
#pragma unroll
    for (int k = 0; k < kNPart; ++k) s[k] = 0.0;
    for (int j = i; j < kRedBlock; j += G) {
#pragma unroll
      for (int k = 0; k < kNPart; ++k) {
        if (k == 6) s[k] = fmax(s[k], part[j][k]);
        else s[k] += part[j][k];
      }
    }
#pragma unroll
    for (int k = 0; k < kNPart; ++k) a.partial[((int64_t)blockIdx.x * G + i) * kNPart + k] = s[k];
  }
}

// One workgroup per (mesh, group): strided partial sums then a fixed-order
// tree, so the FP64 totals are reproducible.
__global__ __launch_bounds__(256) void k_totals(const double* partial, const int32_t* mesh_blk_base,
                                                int32_t n_meshes, int32_t G, double* totals) {
  __shared__ double sh[256][kNPart];
  const int t = blockIdx.x;
  const int m = t / G, g = t % G;
  double s[kNPart];
  for (int k = 0; k < kNPart; ++k) s[k] = 0.0;
  for (int b = mesh_blk_base[m] + threadIdx.x; b < mesh_blk_base[m + 1]; b += 256)
    for (int k = 0; k < kNPart; ++k) {
      const double x = partial[((int64_t)b * G + g) * kNPart + k];
      if (k == 6) s[k] = fmax(s[k], x); else s[k] += x;
    }
  for (int k = 0; k < kNPart; ++k) sh[threadIdx.x][k] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < kNPart; ++k) {
        const double x = sh[threadIdx.x + w][k];
        sh[threadIdx.x][k] = k == 6 ? fmax(sh[threadIdx.x][k], x) : sh[threadIdx.x][k] + x;
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = totals + (int64_t)t * 8;
    for (int k = 0; k < 7; ++k) o[k] = sh[0][k];
    o[7] = sh[0][8] > 0.0 ? sh[0][7] / sh[0][8] : 0.0;
  }
}

__global__ void k_adj_init(const float* dJ, const float* dA, const float* kappa, const float* vol,
                           const float* jsum_last, float albedo, int32_t G, int64_t n,
                           float* gsrc, double* dk, double* de) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double V = (double)vol[i / G];
  const double ga = (double)dA[i];
  const double ka = (1.0 - (double)albedo) * (double)kappa[i];
  gsrc[i] = (float)((double)dJ[i] * (double)kInv4Pi + ga * ka * V);
  dk[i] = ga * (1.0 - (double)albedo) * V * (double)jsum_last[i];
  de[i] = 0.0;
}

__global__ void k_adj_reduce(AdjReduceArgs a, double* dk, double* de) {
  const int64_t n = a.C_total * a.G;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ls = 0.0, lph = 0.0;
  for (int d = 0; d < a.D; ++d) {
    const double l = (double)a.lam[d * n + i];
    ls += l;
    lph += l * (double)a.phi[d * n + i];
  }
  const double V = (double)a.vol[i / a.G];
  const double prev = a.jsum_prev != nullptr ? (double)a.jsum_prev[i] : 0.0;
  const double alb = (double)a.albedo;
  const double invD = (double)a.inv_D;
  dk[i] += -V * lph + alb * V * ls * prev * invD;
  de[i] += ls * invD;
  a.gsrc_next[i] = (float)(alb * (double)a.kappa[i] * V * ls * invD);
}

__global__ void k_d2f_pair(const double* a, const double* b, float* oa, float* ob, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    oa[i] = (float)a[i];
    ob[i] = (float)b[i];
  }
}

inline unsigned grid1d(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

LdsLayout sweep_lds_layout(int32_t gn, int32_t ring, int32_t stage, int32_t lp_cap) {
  LdsLayout L;
  size_t off = (size_t)gn * ring * sizeof(float);
  off = (off + 15) & ~(size_t)15;
  L.stage_off = (int32_t)off;
  off += 2 * (size_t)stage * sizeof(int2);
  L.lp_off = (int32_t)off;
  off += (size_t)lp_cap * sizeof(int32_t);
  off = (off + 7) & ~(size_t)7;
  L.lev_off = (int32_t)off;
  off += (size_t)lp_cap * sizeof(int64_t);
  L.bytes = off;
  return L;
}

hipError_t launch_sweep_fwd(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            size_t lds, hipStream_t s) {
  return launch_sweep_t<false>(a, gn, grid, block, lds, s);
}

hipError_t launch_sweep_adj(const SweepArgs& a, int32_t gn, int32_t grid, int32_t block,
                            size_t lds, hipStream_t s) {
  return launch_sweep_t<true>(a, gn, grid, block, lds, s);
}

hipError_t launch_prep(const PrepArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep, dim3(n_blocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_prep_order, dim3(n_blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int GN, bool REVERSE>
hipError_t set_lds_g(int32_t bytes) {
  const void* fns[] = {(const void*)k_sweep<GN, REVERSE, 4, true>,
                       (const void*)k_sweep<GN, REVERSE, 8, true>,
                       (const void*)k_sweep<GN, REVERSE, 16, true>,
                       (const void*)k_sweep<GN, REVERSE, 8, false>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t set_sweep_lds_limit(int32_t bytes) {
  hipError_t e;
  if ((e = set_lds_g<1, false>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_g<2, false>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_g<3, false>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_g<4, false>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_g<1, true>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_g<2, true>(bytes)) != hipSuccess) return e;
  if ((e = set_lds_g<3, true>(bytes)) != hipSuccess) return e;
  return set_lds_g<4, true>(bytes);
}

hipError_t launch_reduce(const ReduceArgs& a, int32_t n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(n_blocks), dim3(kRedBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_totals(const double* partial, const int32_t* mesh_blk_base, int32_t n_meshes,
                         int32_t G, double* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_totals, dim3(n_meshes * G), dim3(256), 0, s, partial, mesh_blk_base,
                     n_meshes, G, totals);
  return hipGetLastError();
}

hipError_t launch_adj_init(const float* dJ, const float* dA, const float* kappa, const float* vol,
                           const float* jsum_last, float albedo, int32_t G, int64_t C,
                           float* gsrc, double* dk, double* de, hipStream_t s) {
  const int64_t n = C * G;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_init, dim3(grid1d(n, 256)), dim3(256), 0, s, dJ, dA, kappa, vol,
                     jsum_last, albedo, G, n, gsrc, dk, de);
  return hipGetLastError();
}

hipError_t launch_adj_reduce(const AdjReduceArgs& a, double* dk, double* de, hipStream_t s) {
  const int64_t n = a.C_total * a.G;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_reduce, dim3(grid1d(n, 256)), dim3(256), 0, s, a, dk, de);
  return hipGetLastError();
}

hipError_t launch_d2f_pair(const double* a, const double* b, float* oa, float* ob, int64_t n,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_d2f_pair, dim3(grid1d(n, 256)), dim3(256), 0, s, a, b, oa, ob, n);
  return hipGetLastError();
}

}  // namespace sweep
